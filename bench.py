#!/usr/bin/env python3
"""Benchmark of the ray-volume tracer hot path on one MI355X.

A step is one pass of the whole hot path over the ray set: the RK3 step of
every active ray volume (interpolation, dispersion, refraction, face group
velocities, low-storage update, wrap/removal/column keys), the regrouping
sort, the flux deposition and the drag.  Inputs are resident in HBM before
the timed region starts.

Default workload: the global 1x1 degree lat-lon grid, 120 levels to 100 km,
20,000,000 ray volumes (a latitude-dependent background source plus
clustered convective sources with 10x the mean count in 5 % of the columns),
dt = 20 s.  The single-precision path is the headline value; the
double-precision path is timed on the same inputs.  The drag error of both
against the CPU oracle is measured after one step from identical inputs,
and the oracle's own speed on that step is the CPU baseline.

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ray-volume updates/s (RK3+deposit) FP32 vs FP64 at stated drag error"
UNIT = "ray-volume updates/s"

# algorithmic HBM bytes per ray volume and step of the step kernel: the
# state read (x, y, z, k, l, m, Dx, Dy, Dz, Px, Py, Pz, N: 13 values) and the
# 9 evolving values written, at the path's precision -- single precision
# except the vertical wavenumber, which both precisions hold in double
# (FP32: 12 x 4 + 8 read, 8 x 4 + 8 written)
STEP_BYTES = {"fp32": 96, "fp64": 176}
# estimated flops of one RK3 step of one ray volume (three stages of: centre
# interpolation of 12 fields, 6 face interpolations, 7 dispersion
# evaluations, refraction, update), Cartesian count; spherical adds the
# metric terms.  An estimate, reported beside the HBM figure only, against
# the vector rate without packed FP32 (which the build does not use)
STEP_FLOPS = {"cartesian": 2200, "spherical": 2300}
PEAK_HBM_GBS = 8000.0
PEAK_FP32_UNPACKED_TFLOPS = 78.6
PEAK_FP64_TFLOPS = 78.6
# late window: after the timed steps, advance untimed to this step and time
# LATE_STEPS more (the volumes of a column spread over more levels as a run
# goes on; the headline window sees the early part)
LATE_AT, LATE_STEPS = 100, 20
# sources the counted kernels are built from (their HBM traffic in
# profiles/traffic.json is used only while these are unchanged)
KERNEL_SOURCES = {"step": ["paper_2309_11257_amd/csrc/f32.h", "paper_2309_11257_amd/csrc/step32.hip",
                           "paper_2309_11257_amd/csrc/rt_internal.h"],
                  "deposit": ["paper_2309_11257_amd/csrc/deposit_common.h", "paper_2309_11257_amd/csrc/kern32.hip",
                              "paper_2309_11257_amd/csrc/f32.h", "paper_2309_11257_amd/csrc/rt_internal.h"]}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def rel_l2(a, b):
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.sqrt(((a - b) ** 2).sum() / max((b * b).sum(), 1e-300)))


def time_path(w, precision, steps, warmup, late=True):
    import torch

    from paper_2309_11257_amd import _rt
    tr = _rt.Tracer.for_workload(w, precision)
    tr.init_background_from(w)
    # one step from the initial state, for the drag error
    tr.set_rays(w.rays)
    tr.step(w.dt)
    _, drag1 = tr.deposit(host=True)
    ids1 = tr.get_rays()["id"]
    cols1 = tr.get_columns()
    tr.set_rays(w.rays)
    flux = torch.empty((6, w.nz + 1, w.ny, w.nx), dtype=torch.float64, device="cuda")
    drag = torch.empty((2, w.nz, w.ny, w.nx), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        tr.step(w.dt)
        tr.deposit(flux, drag)
    torch.cuda.synchronize()
    n0 = tr.stats()["n_active"]
    tr.profile(True)
    tr.profile_read()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        tr.step(w.dt)
        tr.deposit(flux, drag)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    prof = tr.profile_read()
    tr.profile(False)
    n1 = tr.stats()["n_active"]
    # late window (outside the timed region above): steps LATE_AT + 1 ..
    # LATE_AT + LATE_STEPS of the same run
    do_late, late = late, None
    if do_late and LATE_AT > warmup + steps:
        for _ in range(LATE_AT - warmup - steps):
            tr.step(w.dt)
            tr.deposit(flux, drag)
        torch.cuda.synchronize()
        m0 = tr.stats()["n_active"]
        tr.profile(True)
        tr.profile_read()
        e0.record()
        for _ in range(LATE_STEPS):
            tr.step(w.dt)
            tr.deposit(flux, drag)
        e1.record()
        torch.cuda.synchronize()
        lms = e0.elapsed_time(e1)
        lprof = tr.profile_read()
        tr.profile(False)
        m1 = tr.stats()["n_active"]
        late = dict(steps=f"{LATE_AT + 1}-{LATE_AT + LATE_STEPS}", ms_per_step=round(lms / LATE_STEPS, 4),
                    value=round(0.5 * (m0 + m1) * LATE_STEPS / (lms * 1e-3), 1),
                    kernels_ms_avg={k: round(v[0] / max(v[1], 1), 4) for k, v in lprof.items()})
    tr.close()
    del flux, drag
    torch.cuda.empty_cache()
    ms_per_step = ms / steps
    updates = 0.5 * (n0 + n1) * steps
    return dict(ms_per_step=ms_per_step, wall_s=wall, value=updates / (ms * 1e-3), n_active=(n0, n1),
                kernels={k: {"ms_total": v[0], "launches": v[1], "ms_avg": v[0] / max(v[1], 1)} for k, v in prof.items()},
                drag1=drag1, ids1=ids1, cols1=cols1, late=late)


CPU_STEPS = 6  # oracle steps in the CPU baseline's sample (about 10 s on 16 threads)


def cpu_baseline(w):
    """The oracle as it stands, timed on the host's cores on CPU_STEPS full
    steps of the workload (its own step, deposition and drag each step),
    counting the volumes active at each step.  A separate, untimed oracle
    step from the same inputs is returned for the error measurement."""
    import oracle
    bg = oracle.Background.from_workload(w)
    rs = oracle.RaySet(w.rays)
    oracle.step(bg, rs, w.dt)
    drag = oracle.drag(bg, oracle.deposit(bg, rs))
    rt = oracle.RaySet(w.rays)
    updates = 0
    t0 = time.perf_counter()
    for _ in range(CPU_STEPS):
        updates += int(rt.active().sum())
        oracle.step(bg, rt, w.dt)
        oracle.drag(bg, oracle.deposit(bg, rt))
    t = time.perf_counter() - t0
    del rt
    rec = dict(value=updates / t, unit=UNIT, cores=oracle.num_threads(), kind="oracle",
               sample=f"{CPU_STEPS} full RK3 steps + deposition + drag of the timed workload "
                      f"({w.n_rays} ray volumes at the start, {updates} volume updates, {t:.1f} s)")
    return rec, (oracle, bg, rs, drag)


def drag_errors(orc_state, run):
    """Relative L2 drag error of a GPU path after one step against the oracle:
    raw, and with the oracle taking the kernel's integer decisions (active
    set, parent column) where rounding put a ray on the other side of a cell
    face; plus the number of such flipped decisions."""
    import numpy as np
    orc, bg, rs, drag_ref = orc_state
    raw = rel_l2(run["drag1"], drag_ref)
    ids = rs["id"]
    active = rs.active()
    o = np.argsort(run["ids1"], kind="stable")
    gs, gc = run["ids1"][o], run["cols1"].astype(np.int64)[o]
    p = np.clip(np.searchsorted(gs, ids), 0, max(gs.size - 1, 0))
    found = gs[p] == ids if gs.size else np.zeros(ids.size, bool)
    cols = np.where(found & active, gc[p], -1)
    flips = int(((cols != rs["col"]) & (cols >= 0)).sum())
    nset = int((found != active).sum())
    save = rs.a["state"][: rs.n].copy()
    savec = rs.a["col"][: rs.n].copy()
    rs.a["state"][: rs.n][active & ~found] = orc.INVALID
    flux = orc.deposit(bg, rs, cols=cols)
    aligned = rel_l2(run["drag1"], orc.drag(bg, flux))
    rs.a["state"][: rs.n] = save
    rs.a["col"][: rs.n] = savec
    return {"aligned": aligned, "raw": raw, "column_flips": flips, "active_set_flips": nset}


def surrogate_report(log_rays=50_000_000, steps=100):
    """The learned column surrogate with the tracer as fallback, on the global
    grid with 50 M ray volumes: trained on tracer runs over perturbed global
    backgrounds, then run coupled for `steps` steps at several gate
    thresholds; drag error of every variant against the FP64 tracer after
    the run, and time per step against the plain FP32 tracer."""
    import numpy as np
    import torch

    from paper_2309_11257_amd import _rt
    from paper_2309_11257_amd import surrogate as S
    from paper_2309_11257_amd import workloads as W
    t0 = time.perf_counter()
    feats, drags = S.training_runs(4, 5_000_000, nx=360, ny=180, steps=60, every=20, spin=0)
    hf, hd = S.training_runs(1, 5_000_000, nx=360, ny=180, steps=60, every=20, spin=0, first=4)
    sur = S.ColumnSurrogate(120, n_members=4, max_batch=360 * 180, seed=11)
    X, T = S.dataset(sur, feats, drags, fit=True)
    Xh, Th = S.dataset(sur, hf, hd, fit=False)
    del feats, drags, hf, hd
    t1 = time.perf_counter()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    sur.train(X, T, epochs=2, batch=4096, lr=1e-3)
    ev1.record()
    torch.cuda.synchronize()
    train_ms = ev0.elapsed_time(ev1)
    n_train_steps = 4 * 2 * (X.shape[0] // 4096)
    Y = sur.predict(Xh).mean(dim=0).cpu().numpy().astype(np.float64)
    Tn = Th.cpu().numpy().astype(np.float64)
    zero = -sur.norm.y_mean / sur.norm.y_std
    training = {"samples": int(X.shape[0]), "members": 4, "adam_steps": n_train_steps,
                "train_ms_per_adam_step": round(train_ms / n_train_steps, 4),
                "heldout_mse_network": round(float(np.mean((Y - Tn) ** 2)), 4),
                "heldout_mse_climatology": round(float(np.mean(Tn ** 2)), 4),
                "heldout_mse_zero_drag": round(float(np.mean((zero[None, :] - Tn) ** 2)), 4),
                "data_and_setup_s": round(t1 - t0, 1)}
    del X, T, Xh, Th
    log(f"surrogate training: {training}")

    w = W.make_c5(n_rays=log_rays, steps=steps)
    ms64, ref = S.plain_run(w, steps, _rt.RT_FP64)
    ref = ref.cpu().numpy()
    ms32, d32 = S.plain_run(w, steps, _rt.RT_FP32)
    err32 = rel_l2(d32.cpu().numpy(), ref)
    # gate thresholds from the spread distribution of the initial state
    tr = _rt.Tracer.for_workload(w, _rt.RT_FP32)
    tr.init_background_from(w)
    tr.set_rays(w.rays)
    tr.step(w.dt)
    Xraw = tr.features()
    sp, inside = sur.gate(sur.predict(sur.inputs(Xraw)), Xraw, 1e30)
    tr.close()
    spn = sp.cpu().numpy()[inside.cpu().numpy() > 0]
    taus = [0.0] + ([float(np.quantile(spn, q)) for q in (0.25, 0.5, 0.9)] if spn.size else [])
    rows = []
    for tau in taus:
        row = {"tau": tau}
        for mode in ("surrogate", "persistence", "zero"):
            if tau == 0.0 and mode != "surrogate":
                continue
            res, _ = S.coupled_run(w, sur, tau, steps, mode=mode)
            e = rel_l2(res.drag.cpu().numpy(), ref)
            if mode == "surrogate":
                row.update(trusted_fraction=round(res.trusted_fraction, 4), ms_per_step=round(res.ms_per_step, 4),
                           speedup_vs_plain_fp32=round(ms32 / res.ms_per_step, 3), drag_rel_l2=e)
            else:
                row[f"{mode}_drag_rel_l2"] = e
        rows.append(row)
        log(f"surrogate coupled: {row}")
    sur.close()
    return {"workload": f"global 360x180x120, {w.n_rays} ray volumes, {steps} steps of {w.dt:g} s",
            "reference": "FP64 tracer on the GPU (bitwise the CPU oracle on Cartesian grids, within 1e-13 on the sphere)",
            "training": training, "plain_fp32": {"ms_per_step": round(ms32, 4), "drag_rel_l2": err32},
            "plain_fp64_ms_per_step": round(ms64, 4), "coupled": rows}


def _ev_ms(fn, reps):
    """Mean GPU time of fn() over reps calls (events on the current stream,
    which is the library's stream), after one untimed call."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _row(row, workload, precision, ms, nbytes, oracle_s, cores, sample, note=""):
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"row": row, "workload": workload, "dtype": precision, "gpu_ms": round(ms, 4),
            "algorithmic_bytes": int(nbytes), "achieved_GBs": round(gbs, 1), "bound": "hbm",
            "peak_GBs": PEAK_HBM_GBS, "frac": round(gbs / PEAK_HBM_GBS, 4),
            "oracle_s": round(oracle_s, 3), "oracle_cores": cores, "oracle_sample": sample,
            "gpu_vs_oracle": round(oracle_s / (ms * 1e-3), 1), "note": note}


def rows_report():
    """The rows of the path that the step line does not time: background
    preparation (a0) and surrogate features (a11) on the global 20 M-volume
    workload, vertical splitting with per-cell merging (a9, a10) on the full
    jet box; each with its algorithmic HBM bytes and the oracle timed on the
    same operation.  One JSON line per row."""
    import numpy as np
    import torch

    import oracle
    from paper_2309_11257_amd import _rt
    from paper_2309_11257_amd import workloads as W
    out = []
    cores = oracle.num_threads()
    w3 = W.make_c3()
    cells = w3.nx * w3.ny * w3.nz
    t = time.perf_counter()
    bg3 = oracle.Background.from_workload(w3)
    t_bg = time.perf_counter() - t
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    U, V, N2, f, rho = dev(w3.U), dev(w3.V), dev(w3.N2), dev(w3.f), dev(w3.rho)
    # a0: fields read once (U, V, N2), packed records written once (three
    # records of 4 values per cell)
    for prec, name, rec in ((_rt.RT_FP32, "f32", 4), (_rt.RT_FP64, "f64", 8)):
        tr = _rt.Tracer.for_workload(w3, prec, capacity=1)
        ms = _ev_ms(lambda: tr.init_background(U, V, N2, f, rho), 5)
        out.append(_row("a0", f"global {w3.nx}x{w3.ny}x{w3.nz} background", name, ms, cells * (3 * 8 + 12 * rec),
                        t_bg, cores, f"oracle background preparation of the same grid ({t_bg:.2f} s)",
                        "gradients by centred differences, (f^2)_y, packing into 3 records per cell"))
        tr.close()
    del U, V, N2, f, rho
    # a11: features of the 20 M volumes after one step
    tr = _rt.Tracer.for_workload(w3, _rt.RT_FP32)
    tr.init_background_from(w3)
    tr.set_rays(w3.rays)
    tr.step(w3.dt)
    X = torch.empty((w3.nx * w3.ny, 3 * w3.nz + 48), dtype=torch.float32, device="cuda")
    ms = _ev_ms(lambda: tr.features(X), 5)
    tr.close()
    del X
    rs3 = oracle.RaySet(w3.rays)
    oracle.step(bg3, rs3, w3.dt)
    t = time.perf_counter()
    oracle.features(bg3, rs3)
    t_f = time.perf_counter() - t
    ncol = w3.nx * w3.ny
    # per volume: k, l, m, zeta, xi, eta, lev, col (4 B each) + W (8 B) + the
    # sort permutation (4 B); per column: the background profiles in and the
    # feature row out
    nbytes = w3.n_rays * 48 + ncol * w3.nz * 16 + ncol * (3 * w3.nz + 48) * 4
    out.append(_row("a11", f"global {w3.nx}x{w3.ny}x{w3.nz}, {w3.n_rays} ray volumes", "f32", ms, nbytes, t_f,
                    cores, f"oracle features of the same state ({t_f:.2f} s)", "8 azimuth sectors x 6 moments"))
    # f1, f3: saturation, full fluxes with smoothing and tendencies, budget,
    # each on the state after one step (densities scaled by 1e3 so that part
    # of the cells saturate, as in the parity tests)
    loud = dict(w3.rays)
    loud["n"] = w3.rays["n"] * 1e3
    cells = ncol * w3.nz
    for prec, name in ((_rt.RT_FP32, "f32"), (_rt.RT_FP64, "f64")):
        tr = _rt.Tracer.for_workload(w3, prec)
        tr.init_background_from(w3)
        tr.set_rays(loud)
        tr.step(w3.dt)
        K = torch.empty((w3.nz, w3.ny, w3.nx), dtype=torch.float64, device="cuda")
        ms_sat = _ev_ms(lambda: tr.saturate(w3.dt, kappa=K), 5)
        ms_full = _ev_ms(lambda: tr.full_fluxes(smooth=True), 5)
        ms_bud = _ev_ms(lambda: tr.budget(), 5)
        tr.close()
        del K
        vb = 48 if name == "f32" else 120  # state read per volume and pass (with the permutation)
        t_sat = t_full = t_bud = 0.0
        if name == "f32":
            rs3 = oracle.RaySet(loud)
            oracle.step(bg3, rs3, w3.dt)
            t = time.perf_counter()
            oracle.saturation(bg3, rs3, w3.dt)
            t_sat = time.perf_counter() - t
            t = time.perf_counter()
            oracle.full_tendencies(bg3, oracle.smooth(bg3, oracle.full_fluxes(bg3, rs3)))
            t_full = time.perf_counter() - t
            t = time.perf_counter()
            oracle.budget_terms(bg3, oracle.budget(bg3, rs3))
            t_bud = time.perf_counter() - t
            del rs3
        wl = f"global {w3.nx}x{w3.ny}x{w3.nz}, {w3.n_rays} ray volumes"
        # saturation: two passes over the state (sums, damping with the
        # wave-action write), P, Q and kappa written and read per cell
        out.append(_row("f1", wl, name, ms_sat, w3.n_rays * (2 * vb + 8) + cells * 48, t_sat, cores,
                        f"oracle saturation of the same state ({t_sat:.2f} s)" if t_sat else "",
                        "per-cell P and sum P K^2, kappa, overlap-weighted damping"))
        # full fluxes: one pass over the state; 8 fields written, smoothed
        # (read and written), read by the tendencies, 3 tendencies written
        out.append(_row("f3-fluxes", wl, name, ms_full, w3.n_rays * vb + (ncol * (w3.nz + 1)) * 8 * 8 * 4 + cells * 24,
                        t_full, cores, f"oracle full fluxes, smoothing and tendencies ({t_full:.2f} s)" if t_full else "",
                        "momentum flux tensor, buoyancy flux, 3/2/1 smoothing, elastic term"))
        out.append(_row("f3-budget", wl, name, ms_bud, w3.n_rays * vb + (ncol * (w3.nz + 1)) * 4 * 8 * 2 + cells * 16,
                        t_bud, cores, f"oracle budget fields and terms ({t_bud:.2f} s)" if t_bud else "",
                        "A, cg_h A, cg_z A and the propagation terms"))
    # f2: launch from the ghost layer (latitudinal background source, eight
    # phase speeds, four directions) into the 20 M-volume set after one step:
    # the set is compacted (read and written once), the new volumes written,
    # the whole set regrouped
    lp = dict(lambda_h=300e3, c_min=2.0, c_max=62.0, c_center=25.0, c_width=15.0, n_speeds=8)
    z_launch = 9e3
    for prec, name in ((_rt.RT_FP32, "f32"), (_rt.RT_FP64, "f64")):
        vb = STEP_BYTES["fp32" if name == "f32" else "fp64"]
        tr = _rt.Tracer.for_workload(w3, prec, capacity=w3.n_rays + 8 * 4 * 8 * ncol)
        tr.init_background_from(w3)
        tr.set_rays(w3.rays)
        tr.step(w3.dt)
        n0 = tr.stats()["n_active"]
        ms = _ev_ms(lambda: tr.launch(z_launch, w3.dt, **lp), 5)
        n_new = (tr.stats()["n_active"] - n0) // 6
        tr.close()
        t_l = 0.0
        if name == "f32":
            rs3 = oracle.RaySet(w3.rays, capacity=w3.n_rays + 4 * 8 * ncol)
            t = time.perf_counter()
            oracle.launch(bg3, rs3, oracle.launch_params(z_launch, w3.dt, **lp))
            t_l = time.perf_counter() - t
            del rs3
        out.append(_row("f2", f"global {w3.nx}x{w3.ny}x{w3.nz}, {n0} ray volumes + {n_new} launched", name, ms,
                        n0 * 2 * vb + n_new * vb, t_l, cores,
                        f"oracle launch into the same set ({t_l:.2f} s)" if t_l else "",
                        "candidates flagged, scanned and written after the compacted set, regrouping sort"))
    # f4: a full step (RK3, regrouping, deposition, drag) with the
    # scale-height correction Gamma^2 = 1/(4 H_rho^2) of the reference density
    w3g = W.make_c3()
    w3g.G2 = W.density_gamma2(w3g)
    for prec, name in ((_rt.RT_FP32, "f32"), (_rt.RT_FP64, "f64")):
        r = time_path(w3g, prec, 10, 3, late=False)
        r0 = time_path(w3, prec, 10, 3, late=False)
        vb = STEP_BYTES["fp32" if name == "f32" else "fp64"]
        out.append(_row("f4", f"global {w3.nx}x{w3.ny}x{w3.nz}, {w3.n_rays} ray volumes, Gamma from the density "
                        "scale height", name, r["ms_per_step"], w3.n_rays * vb, 0.0, cores, "",
                        f"whole step with Gamma {r['ms_per_step']:.3f} ms, without {r0['ms_per_step']:.3f} ms; "
                        f"step kernel {r['kernels'].get('step', {}).get('ms_avg', 0):.3f} ms with, "
                        f"{r0['kernels'].get('step', {}).get('ms_avg', 0):.3f} ms without"))
    del bg3
    # a9 + a10: split (alpha = 2) and per-cell merge (64) on the jet box
    w2 = W.make_c2()
    cap = 2 * w2.n_rays
    for prec, name, vb in ((_rt.RT_FP64, "f64", 112), (_rt.RT_FP32, "f32", 72)):
        tr = _rt.Tracer.for_workload(w2, prec, capacity=cap)
        tr.init_background_from(w2)
        tr.set_rays(w2.rays)
        ms_tot, n_tot, nvol = 0.0, 0, 0
        for _ in range(6):
            tr.step(w2.dt)
            tr.profile(True)
            tr.profile_read()
            nvol += tr.stats()["n_active"]
            tr.split_merge(w2.split_alpha, w2.merge_nmax, _rt.RT_MERGE)
            # all timed groups of the call (its regrouping sort times as a sort)
            ms_tot += sum(v[0] for v in tr.profile_read().values())
            tr.profile(False)
            n_tot += 1
        tr.close()
        ms, nv = ms_tot / n_tot, nvol / n_tot
        bg2 = oracle.Background.from_workload(w2)
        rs2 = oracle.RaySet(w2.rays, capacity=cap)
        oracle.step(bg2, rs2, w2.dt)
        t = time.perf_counter()
        oracle.split(bg2, rs2, w2.split_alpha)
        oracle.merge(bg2, rs2, w2.merge_nmax)
        t_sm = time.perf_counter() - t
        # the state is compacted (read and written once) and regrouped
        out.append(_row("a9+a10", f"jet box {w2.nx}x{w2.ny}x{w2.nz}, {int(nv)} ray volumes", name, ms, 2 * vb * nv,
                        t_sm, cores, f"oracle split + merge after one step ({t_sm:.2f} s)",
                        "compaction, split count/scan/write, cell-key sort, per-cell merge, regrouping sort; "
                        "mean over the first 6 steps"))
    for r in out:
        print(json.dumps(r), flush=True)
    return out


def load_traffic(kernel, rays):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))[kernel]
    except (KeyError, ValueError):
        return None
    if d.get("source_sha") != source_sha(KERNEL_SOURCES[kernel]) or d.get("rays") != rays:
        return None
    return float(d["bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rays", type=int, default=20_000_000, help="ray volumes (default: the full workload)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline and the oracle drag error")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-late", action="store_true", help="skip the late window (steps 101-120)")
    ap.add_argument("--surrogate", action="store_true",
                    help="also train the column surrogate and run it coupled with the tracer on 50 M volumes")
    ap.add_argument("--rows", action="store_true",
                    help="only time the rows the step line does not cover (a0, a9+a10, a11), one JSON line each")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding of the "
              "ray set is a design in DESIGN.md, not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 4}))
        return

    if args.rows:
        rows_report()
        return

    from paper_2309_11257_amd import _rt
    from paper_2309_11257_amd import workloads as W

    t = time.perf_counter()
    w = W.make_c3(n_rays=args.rays)
    log(f"workload: {w.n_rays} ray volumes on {w.nx}x{w.ny}x{w.nz} ({time.perf_counter() - t:.1f} s)")

    r32 = time_path(w, _rt.RT_FP32, args.steps, args.warmup, late=not args.no_late)
    log(f"fp32: {r32['ms_per_step']:.3f} ms/step, {r32['value'] / 1e9:.2f} G upd/s, kernels {r32['kernels']}")
    r64 = None
    if not args.no_fp64:
        r64 = time_path(w, _rt.RT_FP64, args.steps, args.warmup, late=not args.no_late)
        log(f"fp64: {r64['ms_per_step']:.3f} ms/step, {r64['value'] / 1e9:.2f} G upd/s, kernels {r64['kernels']}")

    cpu = None
    errs = {}
    if not args.no_cpu:
        cpu, orc_state = cpu_baseline(w)
        log(f"cpu oracle: {cpu['value'] / 1e6:.2f} M upd/s on {cpu['cores']} threads")
        errs["fp32"] = drag_errors(orc_state, r32)
        if r64:
            errs["fp64"] = drag_errors(orc_state, r64)
        log(f"drag rel L2 error vs oracle after one step: {errs}")

    # roofline of the dominant kernel of the FP32 path
    kern = max(r32["kernels"].items(), key=lambda kv: kv[1]["ms_total"])
    name, kd = kern
    nray = 0.5 * (r32["n_active"][0] + r32["n_active"][1])
    avg_s = kd["ms_avg"] * 1e-3
    geom = "spherical" if w.geometry == W.SPHERICAL else "cartesian"
    cells = w.nx * w.ny * w.nz
    if name == "step":
        # HBM roofline on the algorithmic bytes of the step kernel; the flop
        # estimate against the unpacked vector rate is reported beside it
        gbs = STEP_BYTES["fp32"] * nray / avg_s / 1e9
        tflops = STEP_FLOPS[geom] * nray / avg_s / 1e12
        traffic = load_traffic("step", w.n_rays)
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": traffic, "kernel": "k_step32",
                "algorithmic_bytes_per_launch": int(STEP_BYTES["fp32"] * nray),
                "traffic_over_algorithmic": None if traffic is None else round(traffic / (STEP_BYTES["fp32"] * nray), 3),
                "alu_estimate": {"flops_per_volume": STEP_FLOPS[geom], "achieved_TFLOPs": round(tflops, 3),
                                 "peak_unpacked_TFLOPs": PEAK_FP32_UNPACKED_TFLOPS,
                                 "frac": round(tflops / PEAK_FP32_UNPACKED_TFLOPS, 4)}}
    else:
        # deposition / sort / drag are HBM work: algorithmic bytes per ray
        per = {"deposit": 40, "sort": 40, "drag": 0}[name] if name in ("deposit", "sort", "drag") else 0
        gbs = per * nray / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": load_traffic(name, w.n_rays), "kernel": name}
    # the whole step (step, sort, deposition, drag) against the HBM roofline
    # of its algorithmic bytes: the state per volume plus, per cell, the
    # background read (3 fields), the six flux fields (double) and the drag
    # (2 fields, double)
    step_bytes = STEP_BYTES["fp32"] * nray + cells * (3 * 4 + 6 * 8 + 2 * 8)
    roof["whole_step"] = {"algorithmic_bytes": int(step_bytes), "ms": round(r32["ms_per_step"], 4),
                          "frac": round(step_bytes / (r32["ms_per_step"] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    roof["kernel_ms_avg"] = round(kd["ms_avg"], 4)

    out = {
        "metric": METRIC,
        "value": round(r32["value"], 1),
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"global lat-lon 360x180x120 (0-100 km), {w.n_rays} ray volumes "
                               f"(background source + clustered convection), RK3 dt={w.dt:g} s + deposition + drag",
                   "rays": w.n_rays, "grid": [w.nx, w.ny, w.nz], "dt": w.dt, "geometry": "spherical"},
        "drag_rel_l2_vs_oracle_1step": errs or None,
        "fp64": None if r64 is None else {"value": round(r64["value"], 1), "ms_per_step": round(r64["ms_per_step"], 4),
                                          "dtype": "f64"},
        "kernels_ms_avg": {k: round(v["ms_avg"], 4) for k, v in r32["kernels"].items()},
        "kernels_ms_avg_fp64": None if r64 is None else {k: round(v["ms_avg"], 4) for k, v in r64["kernels"].items()},
        "late": r32["late"],
        "late_fp64": None if r64 is None else r64["late"],
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if args.surrogate:
        try:
            out["surrogate"] = surrogate_report()
        except Exception as e:  # report, do not lose the line
            out["surrogate"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
