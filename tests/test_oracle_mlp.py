"""Pins of the surrogate reference (oracle/mlp.py) and of the feature
oracle against mathematics that does not come from the oracle itself."""
import math
import struct

import numpy as np
import pytest

from oracle import mlp

SMALL = mlp.Shape(n_in=7, n_hidden=9, n_layers=2, n_out=5)


def rand_params(shape, seed=0, scale=0.5):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, shape.param_count())


def bf16_bits(x: float) -> float:
    """bfloat16 of a float32 by its bit pattern: add 0x7fff plus the lowest
    kept bit, drop the low half (round to nearest, ties to even)."""
    u = struct.unpack("<I", struct.pack("<f", x))[0]
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return struct.unpack("<f", struct.pack("<I", u))[0]


def test_bf16_rounding_matches_bit_definition():
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.normal(0, 1, 4000), rng.normal(0, 1e4, 2000), rng.normal(0, 1e-4, 2000)])
    xs = xs.astype(np.float32)
    ours = mlp.bf16(xs.astype(np.float64))
    ref = np.array([bf16_bits(float(x)) for x in xs])
    assert np.array_equal(ours, ref)
    # ties to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert mlp.bf16(1.0 + 2.0 ** -8) == 1.0
    assert mlp.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert mlp.bf16(0.0) == 0.0


def test_gelu_closed_forms():
    assert mlp.gelu(0.0) == 0.0
    assert mlp.dgelu(0.0) == pytest.approx(0.5, abs=1e-15)
    # large |z|: identity / zero
    assert mlp.gelu(10.0) == pytest.approx(10.0, rel=1e-15, abs=0)
    assert abs(mlp.gelu(-10.0)) < 1e-15
    # the tanh form approximates z Phi(z) to within 5e-4 absolute
    for z in np.linspace(-5, 5, 101):
        exact = 0.5 * z * (1.0 + math.erf(z / math.sqrt(2.0)))
        assert abs(mlp.gelu(z) - exact) < 5e-4
    # derivative against 50-digit central differences of the formula
    from decimal import Decimal, getcontext
    getcontext().prec = 50

    def g(z):
        c = (Decimal(2) / Decimal(str(math.pi))).sqrt()
        u = c * (z + Decimal("0.044715") * z ** 3)
        e2 = (2 * u).exp()
        return z / 2 * (1 + (e2 - 1) / (e2 + 1))

    h = Decimal("1e-20")
    for z in (-3.1, -0.7, 0.2, 1.3, 2.9):
        zd = Decimal(z)
        fd = float((g(zd + h) - g(zd - h)) / (2 * h))
        assert mlp.dgelu(z) == pytest.approx(fd, rel=1e-12, abs=0)


def test_hand_network():
    """One hidden layer, hand-computed: X = [1, 2], W1 = I, b1 = [0.5, -1],
    W2 = [[1, -2]], b2 = [0.25]."""
    s = mlp.Shape(n_in=2, n_hidden=2, n_layers=1, n_out=1)
    p = np.array([1.0, 0.0, 0.0, 1.0, 1.0, -2.0, 0.5, -1.0, 0.25])
    assert s.param_count() == p.size
    y, _ = mlp.forward(p, s, np.array([[1.0, 2.0]]), emulate=False)

    def g(z):
        return 0.5 * z * (1 + math.tanh(math.sqrt(2 / math.pi) * (z + 0.044715 * z ** 3)))

    assert y[0, 0] == pytest.approx(g(1.5) - 2 * g(1.0) + 0.25, rel=1e-15, abs=0)


def test_gradient_finite_differences():
    """T25: reverse-mode gradient of the float64 network against central
    differences, every parameter, relative error <= 1e-6."""
    p = rand_params(SMALL, seed=3)
    rng = np.random.default_rng(4)
    X = rng.normal(size=(6, SMALL.n_in))
    T = rng.normal(size=(6, SMALL.n_out))
    _, g = mlp.loss_and_grad(p, SMALL, X, T, emulate=False)
    fd = np.zeros_like(p)
    h = 1e-6
    for i in range(p.size):
        q = p.copy()
        q[i] += h
        lp, _ = mlp.loss_and_grad(q, SMALL, X, T, emulate=False)
        q[i] -= 2 * h
        lm, _ = mlp.loss_and_grad(q, SMALL, X, T, emulate=False)
        fd[i] = (lp - lm) / (2 * h)
    assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(fd)
    # every layer's block is non-trivial and checked on its own
    off = 0
    for i, o in SMALL.layers():
        blk = slice(off, off + i * o)
        assert np.linalg.norm(g[blk] - fd[blk]) <= 1e-6 * np.linalg.norm(fd[blk])
        off += i * o


def test_loss_is_mean_square():
    p = rand_params(SMALL, seed=5)
    X = np.ones((3, SMALL.n_in))
    Y, _ = mlp.forward(p, SMALL, X, emulate=False)
    L, _ = mlp.loss_and_grad(p, SMALL, X, Y + 2.0, emulate=False)
    assert L == pytest.approx(4.0, rel=1e-14, abs=0)


def test_adam_first_step_closed_form():
    """T27: with zero moments the first bias-corrected step is
    lr g / (|g| + eps); the second follows the recursion by hand."""
    rng = np.random.default_rng(6)
    w = rng.normal(size=50)
    g = rng.normal(size=50)
    w1, m, v = mlp.adam(w, np.zeros(50), np.zeros(50), g, 1, lr=1e-3)
    assert np.allclose(w1, w - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    g2 = rng.normal(size=50)
    w2, _, _ = mlp.adam(w1, m, v, g2, 2, lr=1e-3)
    m2 = 0.9 * 0.1 * g + 0.1 * g2
    v2 = 0.999 * 0.001 * g * g + 0.001 * g2 * g2
    ref = w1 - 1e-3 * (m2 / (1 - 0.81)) / (np.sqrt(v2 / (1 - 0.999 ** 2)) + 1e-8)
    assert np.allclose(w2, ref, rtol=0, atol=1e-15)


def test_gate_closed_forms():
    """T28: two members a, b give spread |a - b| / sqrt(2) per output; an
    out-of-range feature always routes to the tracer; tau = 0 trusts only
    identical members."""
    a = np.array([[1.0, 2.0], [0.0, 0.0], [3.0, 3.0]])
    b = np.array([[2.0, 4.0], [0.0, 0.0], [3.0, 3.0]])
    X = np.array([[0.5], [0.5], [5.0]])
    sp, mask = mlp.gate(np.stack([a, b]), X, [0.0], [1.0], tau=10.0)
    assert sp[0] == pytest.approx(math.sqrt((0.5 + 2.0) / 2), rel=1e-15, abs=0)
    assert sp[1] == 0.0
    assert list(mask) == [1, 1, 0]
    _, mask0 = mlp.gate(np.stack([a, b]), X, [0.0], [1.0], tau=0.0)
    assert list(mask0) == [0, 1, 0]


def test_standardize():
    Xr = np.array([[1.0, 99.0], [3.0, 999.0]])
    out = mlp.standardize(Xr, np.array([2.0, 2.5]), np.array([1.0, 0.5]), np.array([0.0, 1.0]))
    assert np.allclose(out, [[-1.0, -1.0], [1.0, 1.0]], rtol=0, atol=1e-14)


def test_features_brute_force(orc):
    """Features against a per-ray Python loop that recomputes the sector by
    arctangent and the intrinsic group velocity from the closed form, and
    the height spread by a two-pass variance."""
    from paper_2309_11257_amd import workloads as W
    w = W.make_c1(n_rays=600)
    bg = orc.Background.from_workload(w)
    rs = orc.RaySet(w.rays)
    for _ in range(20):
        orc.step(bg, rs, w.dt)
    X = orc.features(bg, rs)
    nz = w.nz
    assert X.shape == (w.nx * w.ny, 3 * nz + 48)
    # profiles
    c = 37
    i, j = c % w.nx, c // w.nx
    assert np.array_equal(X[c, :nz], w.U[:, j, i])
    assert np.array_equal(X[c, 2 * nz:3 * nz], w.N2[:, j, i])
    sums = np.zeros((w.nx * w.ny, 8, 4))
    members = {}
    snap = rs.snapshot()
    f2 = w.f[0] ** 2
    for q in range(len(snap["id"])):
        k, l, m = snap["k"][q], snap["l"][q], snap["m"][q]
        N2 = bg.interp(snap["x"][q], snap["y"][q], snap["z"][q])[2]
        kh2 = k * k + l * l
        K2 = kh2 + m * m
        om = math.sqrt((N2 * kh2 + f2 * m * m) / K2)
        cgz = -m * kh2 * (N2 - f2) / (om * K2 * K2)
        az = math.degrees(math.atan2(l, k)) % 360.0
        s = int(((az + 22.5) % 360.0) // 45.0)
        Wq = snap["n"][q] * snap["px"][q] * snap["py"][q] * snap["pz"][q]
        col = snap["col"][q]
        kh = math.sqrt(kh2)
        sums[col, s] += [Wq, abs(cgz) * kh * Wq, Wq * math.log10(kh), Wq * math.log10(abs(m))]
        members.setdefault((col, s), []).append((Wq, snap["z"][q]))
    got = X[:, 3 * nz:].reshape(-1, 8, 6)
    ok = sums[:, :, 0] > 0
    den = np.where(ok, sums[:, :, 0], 1)
    assert np.allclose(got[:, :, 0], sums[:, :, 0], rtol=1e-12, atol=0)
    assert np.allclose(got[:, :, 1], sums[:, :, 1], rtol=1e-12, atol=0)
    assert np.allclose(got[:, :, 2], np.where(ok, sums[:, :, 2] / den, 0), rtol=1e-12, atol=0)
    assert np.allclose(got[:, :, 3], np.where(ok, sums[:, :, 3] / den, 0), rtol=1e-12, atol=0)
    nspread = 0
    for (col, s), lst in members.items():
        wv = np.array([a for a, _ in lst])
        zv = np.array([b for _, b in lst])
        zm = (wv * zv).sum() / wv.sum()
        sd = math.sqrt((wv * (zv - zm) ** 2).sum() / wv.sum())
        assert got[col, s, 4] == pytest.approx(zm, rel=1e-12, abs=0)
        assert abs(got[col, s, 5] - sd) <= 1e-6 * zm  # one-pass variance: cancellation floor
        nspread += len(lst) > 1 and sd > 1.0
    assert nspread > 5
    assert np.all(got[~ok] == 0)
    assert got[:, :, 0].sum() == pytest.approx(orc.stats(rs)["sum_W"], rel=1e-12, abs=0)
