"""FP64 numpy reference of the column surrogate -- TEST INFRASTRUCTURE.

Only the test-suite, the package smoke check and the benchmark's CPU-baseline
leg may import this module.  It shares no code with the GPU library.

The paper has no learned component; the surrogate is an addition whose
ground truth is the ray tracer.  What is fixed here is plain mathematics:

* a multilayer perceptron n_in -> n_hidden (x n_layers) -> n_out with the
  tanh form of GELU (Hendrycks & Gimpel 2016):
  gelu(z) = z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3)));
* its gradient by the chain rule (reverse mode), for the mean squared error
  L = mean over samples and outputs of (Y - T)^2;
* Adam (Kingma & Ba 2015) with bias-corrected moments;
* bfloat16 emulation: round-to-nearest-even to 8 significant bits, applied
  (when `emulate` is set) exactly where the GPU stores bfloat16 -- the
  inputs, the weights used in products, the hidden activations, the output
  gradient and the pre-activation gradients.  Everything else is float64.

Parameter vector layout (one member): all weight matrices, layer by layer,
each [out][in] row-major, then all bias vectors, layer by layer.

Parity: pinned by finite differences (gradient), closed forms (Adam's first
step, GELU values and slope, the gate's spread of two members) and a brute
force check of the bfloat16 rounding against an independent bit-level
definition.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Tuple

import numpy as np


@dataclass(frozen=True)
class Shape:
    n_in: int
    n_hidden: int
    n_layers: int
    n_out: int

    def layers(self) -> List[Tuple[int, int]]:
        """(fan_in, fan_out) per layer."""
        dims = [self.n_in] + [self.n_hidden] * self.n_layers + [self.n_out]
        return [(dims[i], dims[i + 1]) for i in range(len(dims) - 1)]

    def param_count(self) -> int:
        return sum(i * o + o for i, o in self.layers())


def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 value (8 significant bits, ties to even),
    returned as float64.  Zero, infinities and NaN pass through; values below
    the normal range are not expected here."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)  # x = m 2^e, 0.5 <= |m| < 1
    r = np.rint(m * 256.0) / 256.0  # np.rint rounds half to even
    out = np.ldexp(r, e)
    return np.where(np.isfinite(x), out, x)


def gelu(z):
    c = math.sqrt(2.0 / math.pi)
    return 0.5 * z * (1.0 + np.tanh(c * (z + 0.044715 * z ** 3)))


def dgelu(z):
    c = math.sqrt(2.0 / math.pi)
    t = np.tanh(c * (z + 0.044715 * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * c * (1.0 + 3.0 * 0.044715 * z * z)


def unpack(params: np.ndarray, shape: Shape):
    """List of (W [out][in], b [out]) views of a parameter vector."""
    p = np.asarray(params, dtype=np.float64)
    assert p.shape == (shape.param_count(),)
    Ws, off = [], 0
    for i, o in shape.layers():
        Ws.append(p[off:off + i * o].reshape(o, i))
        off += i * o
    bs = []
    for _, o in shape.layers():
        bs.append(p[off:off + o])
        off += o
    return list(zip(Ws, bs))


def forward(params, shape: Shape, X, emulate: bool = True):
    """Y [B][n_out] and the cache for backward().  X [B][n_in]."""
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    layers = unpack(params, shape)
    h = r(X)
    inputs, zs = [h], []
    for li, (W, b) in enumerate(layers):
        z = h @ r(W).T + b
        if li < len(layers) - 1:
            zs.append(z)
            h = r(gelu(z))
            inputs.append(h)
        else:
            y = z
    return y, (inputs, zs)


def loss_and_grad(params, shape: Shape, X, T, emulate: bool = True):
    """(L, grad) for L = mean (Y - T)^2; grad in the parameter layout."""
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    layers = unpack(params, shape)
    Y, (inputs, zs) = forward(params, shape, X, emulate)
    T = np.asarray(T, dtype=np.float64)
    diff = Y - T
    L = float(np.mean(diff * diff))
    d = r(2.0 * diff / diff.size)  # dL/dY (stored as bfloat16 on the GPU)
    gW = [None] * len(layers)
    gb = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        gW[li] = d.T @ inputs[li]
        gb[li] = d.sum(axis=0)
        if li > 0:
            d = r((d @ r(W)) * dgelu(zs[li - 1]))
    grad = np.concatenate([g.ravel() for g in gW] + list(gb))
    return L, grad


def adam(w, m, v, g, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (Kingma & Ba 2015, Algorithm 1); t counts from 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def gate(Yens, Xraw, fmin, fmax, tau: float):
    """Trust gate.  Yens [members][cols][n_out]; spread per column = root mean
    square over outputs of the members' sample standard deviation (n - 1
    normalisation; 0 for a single member); trusted (1) iff spread <= tau and
    every feature lies in [fmin, fmax]."""
    Y = np.asarray(Yens, dtype=np.float64)
    nm = Y.shape[0]
    var = Y.var(axis=0, ddof=1) if nm > 1 else np.zeros(Y.shape[1:])
    spread = np.sqrt(var.mean(axis=-1))
    X = np.asarray(Xraw, dtype=np.float64)
    inside = np.all((X >= np.asarray(fmin)) & (X <= np.asarray(fmax)), axis=1)
    return spread, (inside & (spread <= tau)).astype(np.uint8)


def standardize(Xraw, mean, std, logfloor):
    """Network input: (T(x) - mean) / std with T(x) = log10(max(x + floor,
    1e-30)) where floor > 0, identity where floor == 0."""
    X = np.asarray(Xraw, dtype=np.float64)
    fl = np.asarray(logfloor, dtype=np.float64)
    T = np.where(fl > 0, np.log10(np.maximum(X + fl, 1e-30)), X)
    return (T - mean) / std


def apply_drag(Yens, mean, std, mask, drag):
    """drag [2*nz][n_cols] with trusted columns replaced by the ensemble mean
    of Y * std + mean (outputs o = comp*nz + k)."""
    Y = np.asarray(Yens, dtype=np.float64) * np.asarray(std, np.float64) + np.asarray(mean, np.float64)
    out = np.array(drag, dtype=np.float64, copy=True)
    sel = np.asarray(mask).astype(bool)
    out[:, sel] = Y.mean(axis=0)[sel].T
    return out
