"""Column surrogate driver: training data from the ray tracer, ensemble
training with the library's MFMA kernels, and the coupled surrogate +
fallback step.

Every numerical step runs in the HIP library (features, standardisation,
targets, forward, backward, Adam, gate, drag substitution); this module
only sequences the calls, keeps the normalisation constants, and gathers
minibatch rows (a device index_select).  The normalisation constants are
fitted once on the host from a sample of the training set.

Coupling (one step of the coupled model):
  1. advance the tracer; volumes in the columns trusted at the previous step
     keep their state (rt_step with RT_STEP_SURROGATE);
  2. deposit fluxes and drag of the whole set;
  3. features of the new state -> standardised bfloat16 inputs -> every
     ensemble member's prediction;
  4. gate: a column is trusted if the ensemble spread is at most tau and all
     its raw features lie inside the training range;
  5. the drag of trusted columns is replaced by the ensemble mean; the trust
     mask becomes the frozen-column mask of the next step.
tau = 0 trusts nothing (distinct members never agree exactly), so the coupled
model then reproduces the tracer bit for bit.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Tuple

import numpy as np

from . import _rt, _sg
from . import workloads as W


def log_features(nz: int) -> np.ndarray:
    """Indices of the features that enter the network as log10(x + floor):
    the per-sector sums of W and of |cg_z| k_h W."""
    base = 3 * nz
    return np.array([base + 6 * s + q for s in range(8) for q in (0, 1)])


@dataclass
class Norm:
    x_mean: np.ndarray
    x_std: np.ndarray
    x_floor: np.ndarray
    x_min: np.ndarray
    x_max: np.ndarray
    y_mean: np.ndarray
    y_std: np.ndarray


def fit_norm(nz: int, Xraw: np.ndarray, drag: np.ndarray) -> Norm:
    """Normalisation constants from host samples: Xraw [S][3nz+48] float32,
    drag [S][2nz] (rows = columns)."""
    X = np.asarray(Xraw, np.float64)
    n_in = X.shape[1]
    floor = np.zeros(n_in)
    for f in log_features(nz):
        pos = X[:, f][X[:, f] > 0]
        floor[f] = max(1e-3 * float(np.median(pos)), 1e-30) if pos.size else 1e-30
    T = np.where(floor > 0, np.log10(np.maximum(X + floor, 1e-30)), X)
    mu = T.mean(axis=0)
    sd = T.std(axis=0)
    sd = np.where(sd > 1e-12 * np.maximum(np.abs(mu), 1e-30), sd, 1.0)
    # targets: per-output means removed, one scale per drag component (the
    # root-mean-square over its levels), so the loss weights levels by their
    # physical drag and a level that is almost always zero is not blown up
    Y = np.asarray(drag, np.float64)
    ym = Y.mean(axis=0)
    nz2 = Y.shape[1] // 2
    ys = np.empty(Y.shape[1])
    for comp in range(2):
        blk = Y[:, comp * nz2:(comp + 1) * nz2] - ym[comp * nz2:(comp + 1) * nz2]
        r = float(np.sqrt(np.mean(blk * blk)))
        ys[comp * nz2:(comp + 1) * nz2] = r if r > 0 else 1.0
    f32 = lambda a: np.asarray(a, np.float32)
    return Norm(f32(mu), f32(sd), f32(floor), f32(X.min(axis=0)), f32(X.max(axis=0)), f32(ym), f32(ys))


class ColumnSurrogate:
    def __init__(self, nz: int, n_members: int = 4, n_hidden: int = 512, n_layers: int = 3, max_batch: int = 4096,
                 seed: int = 1, device: str = "cuda:0"):
        self.nz = nz
        self.n_in, self.n_out = 3 * nz + 48, 2 * nz
        self.net = _sg.Surrogate(self.n_in, n_hidden, n_layers, self.n_out, n_members=n_members,
                                 max_batch=max_batch, seed=seed, device=device)
        self.torch = self.net.torch
        self.device = self.net.device
        self.norm: Optional[Norm] = None
        self._dev = {}

    def set_norm(self, norm: Norm):
        self.norm = norm
        t = self.torch
        self._dev = {k: t.from_numpy(np.ascontiguousarray(getattr(norm, k))).to(self.device)
                     for k in ("x_mean", "x_std", "x_floor", "x_min", "x_max", "y_mean", "y_std")}

    def inputs(self, Xraw):
        d = self._dev
        return self.net.standardize(Xraw, d["x_mean"], d["x_std"], d["x_floor"])

    def targets(self, drag):
        d = self._dev
        return self.net.targets(drag.reshape(-1).contiguous(), d["y_mean"], d["y_std"], self.nz)

    def train(self, X, T, epochs: int, batch: int = 4096, lr: float = 1e-3, seed: int = 0,
              members: Optional[List[int]] = None, log=None) -> List[float]:
        """Adam on minibatches of (X bf16 [N][n_in], T float32 [N][n_out]),
        each member with its own shuffling.  Returns each member's last
        minibatch loss."""
        torch = self.torch
        N = X.shape[0]
        batch = min(batch, N, self.net.max_batch)
        loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        out = []
        for m in (members if members is not None else range(self.net.n_members)):
            gen = torch.Generator(device="cpu")
            gen.manual_seed(1000 * seed + m)
            for ep in range(epochs):
                perm = torch.randperm(N, generator=gen).to(self.device)
                for b in range(N // batch):
                    idx = perm[b * batch:(b + 1) * batch]
                    self.net.train_step(m, X.index_select(0, idx), T.index_select(0, idx), lr, loss)
                if log:
                    log(f"member {m} epoch {ep}: minibatch loss {float(loss.item()):.4f}")
            out.append(float(loss.item()))
        return out

    def predict(self, X):
        """Every member's standardised prediction [members][N][n_out]; rows
        in chunks of max_batch."""
        torch = self.torch
        N = X.shape[0]
        if N <= self.net.max_batch:
            return self.net.forward(X, member=-1)
        Y = torch.empty((self.net.n_members, N, self.n_out), dtype=torch.float32, device=self.device)
        for c0 in range(0, N, self.net.max_batch):
            c1 = min(N, c0 + self.net.max_batch)
            Y[:, c0:c1] = self.net.forward(X[c0:c1], member=-1)
        return Y

    def gate(self, Yens, Xraw, tau: float):
        d = self._dev
        return self.net.gate(Yens, Xraw, d["x_min"], d["x_max"], tau)

    def apply(self, Yens, mask, drag):
        d = self._dev
        self.net.apply_drag(Yens, d["y_mean"], d["y_std"], mask, self.nz, drag)

    def close(self):
        self.net.close()


def sample_run(w, steps: int, every: int, spin: int = 0, precision: int = _rt.RT_FP32):
    """Run the tracer on workload w and collect (raw features, drag) device
    tensors every `every` steps after `spin` steps: lists of [ncol][n_in]
    float32 and [2][nz][ncol] float64."""
    tr = _rt.Tracer.for_workload(w, precision)
    tr.init_background_from(w)
    tr.set_rays(w.rays)
    feats, drags = [], []
    for s in range(1, steps + 1):
        tr.step(w.dt)
        if s > spin and (s - spin) % every == 0:
            _, drag = tr.deposit()
            feats.append(tr.features())
            drags.append(drag)
    tr.close()
    return feats, drags


def dataset(sur: ColumnSurrogate, feats, drags, fit: bool, sample_rows: int = 200_000, seed: int = 0):
    """Network inputs and targets [N][...] from sampled runs; fits the
    normalisation on a host sample of rows first if `fit`."""
    torch = sur.torch
    nz = sur.nz
    if fit:
        rng = np.random.default_rng(seed)
        Xs, Ys = [], []
        per = max(1, sample_rows // len(feats))
        for Xr, D in zip(feats, drags):
            ncol = Xr.shape[0]
            rows = rng.choice(ncol, size=min(per, ncol), replace=False)
            idx = torch.from_numpy(rows).to(sur.device)
            Xs.append(Xr.index_select(0, idx).cpu().numpy())
            Ys.append(D.reshape(2 * nz, ncol).index_select(1, idx).t().cpu().numpy())
        sur.set_norm(fit_norm(nz, np.concatenate(Xs), np.concatenate(Ys)))
    X = torch.cat([sur.inputs(Xr) for Xr in feats])
    T = torch.cat([sur.targets(D) for D in drags])
    return X, T


@dataclass
class CoupledResult:
    ms_per_step: float
    trusted_fraction: float
    drag: object


def coupled_run(w, sur: ColumnSurrogate, tau: float, steps: int, precision: int = _rt.RT_FP32,
                mode: str = "surrogate") -> Tuple[CoupledResult, dict]:
    """Run the coupled model for `steps` steps from w's initial state.
    mode "surrogate": trusted columns take the ensemble mean; "persistence":
    trusted columns are frozen but keep the drag deposited from their frozen
    volumes; "zero": trusted columns get zero drag (the last two are the
    no-network baselines at the same routed fraction)."""
    torch = sur.torch
    tr = _rt.Tracer.for_workload(w, precision)
    tr.init_background_from(w)
    tr.set_rays(w.rays)
    ncol, nz = w.nx * w.ny, w.nz
    flux = torch.empty((6, nz + 1, w.ny, w.nx), dtype=torch.float64, device=sur.device)
    drag = torch.empty((2, nz, w.ny, w.nx), dtype=torch.float64, device=sur.device)
    Xraw = torch.empty((ncol, 3 * nz + 48), dtype=torch.float32, device=sur.device)
    mask = None
    trusted = []
    zeros = torch.zeros(2 * nz, dtype=torch.float32, device=sur.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        if mask is not None:
            tr.set_frozen_columns(mask)
            tr.step(w.dt, surrogate=True)
        else:
            tr.step(w.dt)
        tr.deposit(flux, drag)
        tr.features(out=Xraw)
        Yens = sur.predict(sur.inputs(Xraw))
        _, mask = sur.gate(Yens, Xraw, tau)
        if mode == "surrogate":
            sur.apply(Yens, mask, drag)
        elif mode == "zero":
            sur.net.apply_drag(Yens, zeros, zeros, mask, nz, drag)
        trusted.append(mask.sum())
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    frac = float(torch.stack(trusted).double().mean().item()) / ncol
    extra = {"stats": tr.stats()}
    tr.close()
    return CoupledResult(ms, frac, drag), extra


def plain_run(w, steps: int, precision: int):
    """The tracer alone: (ms per step, final drag [2][nz][ny][nx])."""
    import torch
    tr = _rt.Tracer.for_workload(w, precision)
    tr.init_background_from(w)
    tr.set_rays(w.rays)
    flux = torch.empty((6, w.nz + 1, w.ny, w.nx), dtype=torch.float64, device="cuda")
    drag = torch.empty((2, w.nz, w.ny, w.nx), dtype=torch.float64, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        tr.step(w.dt)
        tr.deposit(flux, drag)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    tr.close()
    return ms, drag


def training_runs(n_runs: int, n_rays: int, nx: int, ny: int, steps: int, every: int, spin: int, first: int = 0):
    """Seeded training runs first .. first + n_runs - 1 of the tracer
    (make_c4 backgrounds)."""
    feats, drags = [], []
    for r in range(first, first + n_runs):
        w = W.make_c4(r, n_rays=n_rays, nx=nx, ny=ny, steps=steps)
        f, d = sample_run(w, steps, every, spin)
        feats += f
        drags += d
    return feats, drags
