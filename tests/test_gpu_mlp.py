"""Surrogate kernels on the GPU against the FP64 reference with bfloat16
emulation (oracle/mlp.py): forward, gradient, Adam, gate, standardisation
and the drag substitution, through the C ABI."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SHAPE = dict(n_in=392, n_hidden=512, n_layers=3, n_out=240)


@pytest.fixture(scope="module")
def sgmod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_11257_amd import _sg
    _sg.lib()
    return _sg


@pytest.fixture(scope="module")
def mlp():
    from oracle import mlp
    return mlp


def he_params(mlp, shape, seed):
    rng = np.random.default_rng(seed)
    parts_w, parts_b = [], []
    for i, o in shape.layers():
        parts_w.append(rng.uniform(-1, 1, i * o) * np.sqrt(6.0 / i))
        parts_b.append(rng.normal(0, 0.1, o))
    return np.concatenate(parts_w + parts_b).astype(np.float32)


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_err_over_rms(a, b):
    """Largest element error over the RMS of the reference block.  The
    kernels sum in single precision in another order than the reference;
    where that moves an activation across a bfloat16 rounding boundary
    (one unit is 2^-8 relative) the layers after it carry the difference,
    so single elements differ by a few thousandths of the block's scale."""
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / np.sqrt(np.mean(b * b)))


def make(sgmod, members=2, max_batch=4096, **kw):
    sh = dict(SHAPE, **kw)
    return sgmod.Surrogate(sh["n_in"], sh["n_hidden"], sh["n_layers"], sh["n_out"], n_members=members,
                           max_batch=max_batch, seed=7)


def test_param_count_and_roundtrip(sgmod, mlp):
    net = make(sgmod)
    shape = mlp.Shape(**SHAPE)
    assert net.P == shape.param_count() == 849648
    p = he_params(mlp, shape, 1)
    net.set_params(1, p)
    assert np.array_equal(net.get_params(1), p)
    # fresh members: He-uniform weights within the bound, zero biases
    p0 = net.get_params(0)
    nw = sum(i * o for i, o in shape.layers())
    assert np.all(p0[nw:] == 0)
    assert np.abs(p0[:392 * 512]).max() <= np.sqrt(6 / 392) and p0[:392 * 512].std() > 0.05
    net.close()


@pytest.mark.parametrize("B", [1, 300, 4096])
def test_forward_matches_reference(sgmod, mlp, B):
    """Several 128-row and 128-column tiles with ragged edges (B = 300,
    n_out = 240), one row, and the full training batch."""
    net = make(sgmod)
    shape = mlp.Shape(**SHAPE)
    p = he_params(mlp, shape, 2)
    net.set_params(0, p)
    net.set_params(1, he_params(mlp, shape, 3))
    rng = np.random.default_rng(B)
    X = mlp.bf16(rng.normal(size=(B, 392)))
    Y = net.forward(X, member=0).cpu().numpy()
    ref, _ = mlp.forward(p.astype(np.float64), shape, X, emulate=True)
    assert rel_l2(Y, ref) <= 2e-2
    assert max_err_over_rms(Y, ref) <= 2e-2  # element by element
    Yall = net.forward(X, member=-1).cpu().numpy()
    assert np.array_equal(Yall[0], Y)
    net.close()


@pytest.mark.parametrize("B", [300, 2500])
def test_gradient_matches_reference(sgmod, mlp, B):
    """B = 2500 takes the split-K weight-gradient path with a ragged last
    chunk; B = 300 the single-pass one.  Every layer's weight and bias block
    within 2e-2 relative L2, and every element within 2e-2 of its block's
    RMS."""
    net = make(sgmod)
    shape = mlp.Shape(**SHAPE)
    p = he_params(mlp, shape, 4)
    net.set_params(0, p)
    rng = np.random.default_rng(5)
    X = mlp.bf16(rng.normal(size=(B, 392)))
    T = rng.normal(size=(B, 240)).astype(np.float32)
    g = net.gradient(0, X, T)
    L, gref = mlp.loss_and_grad(p.astype(np.float64), shape, X, T, emulate=True)
    off = 0
    blocks = [(i * o) for i, o in shape.layers()] + [o for _, o in shape.layers()]
    for n in blocks:
        assert rel_l2(g[off:off + n], gref[off:off + n]) <= 2e-2, (off, n)
        assert max_err_over_rms(g[off:off + n], gref[off:off + n]) <= 2e-2, (off, n)
        off += n
    assert off == g.size
    g2 = net.gradient(0, X, T)
    assert np.array_equal(g, g2), "gradient is not deterministic"
    net.close()


def test_adam_step_and_loss(sgmod, mlp):
    import torch
    net = make(sgmod)
    shape = mlp.Shape(**SHAPE)
    p = he_params(mlp, shape, 6)
    net.set_params(0, p)
    rng = np.random.default_rng(7)
    X = mlp.bf16(rng.normal(size=(512, 392)))
    T = rng.normal(size=(512, 240)).astype(np.float32)
    g = net.gradient(0, X, T).astype(np.float64)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    net.train_step(0, X, T, lr=1e-3, loss=loss)
    p1 = net.get_params(0).astype(np.float64)
    ref, m, v = mlp.adam(p.astype(np.float64), 0.0, 0.0, g, 1, lr=1e-3)
    assert np.abs(p1 - ref).max() <= 1e-6
    L, _ = mlp.loss_and_grad(p.astype(np.float64), shape, X, T, emulate=True)
    assert float(loss.item()) == pytest.approx(L, rel=2e-2, abs=0)
    # second step continues the recursion from the kept moments
    g2 = net.gradient(0, X, T).astype(np.float64)
    net.train_step(0, X, T, lr=1e-3)
    p2 = net.get_params(0).astype(np.float64)
    ref2, _, _ = mlp.adam(p1, m, v, g2, 2, lr=1e-3)
    assert np.abs(p2 - ref2).max() <= 1e-6
    net.close()


def test_training_fits_a_smooth_map(sgmod, mlp):
    """A learnable target (a fixed random two-layer map of the input): 150
    Adam steps cut the loss by more than 5x."""
    import torch
    net = make(sgmod, members=1, n_in=64, n_hidden=128, n_layers=2, n_out=16)
    rng = np.random.default_rng(8)
    A = rng.normal(size=(64, 32)) / 8.0
    Bm = rng.normal(size=(32, 16)) / 6.0
    X = mlp.bf16(rng.normal(size=(1024, 64)))
    T = (np.tanh(X @ A) @ Bm).astype(np.float32)
    T /= T.std()
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    net.train_step(0, X, T, lr=1e-3, loss=loss)
    l0 = float(loss.item())
    for _ in range(150):
        net.train_step(0, X, T, lr=1e-3, loss=loss)
    assert float(loss.item()) < l0 / 5
    net.close()


def test_gate_and_apply_drag(sgmod, mlp):
    import torch
    net = make(sgmod, members=3, n_out=8)
    rng = np.random.default_rng(9)
    nc = 1000
    Y = rng.normal(size=(3, nc, 8)).astype(np.float32)
    Y[:, :100] = Y[0:1, :100]  # identical members: zero spread
    Xr = rng.uniform(0, 1, size=(nc, 392)).astype(np.float32)
    Xr[50, 7] = 2.0  # out of range although the members agree
    fmin = np.zeros(392, np.float32)
    fmax = np.ones(392, np.float32)
    for tau in (0.0, 0.9, 1.1):
        sp, mk = net.gate(Y, Xr, fmin, fmax, tau)
        rsp, rmk = mlp.gate(Y, Xr, fmin, fmax, tau)
        assert np.allclose(sp.cpu().numpy(), rsp, rtol=1e-6, atol=0)
        assert np.array_equal(mk.cpu().numpy(), rmk)
    _, mk0 = net.gate(Y, Xr, fmin, fmax, 0.0)
    mk0 = mk0.cpu().numpy()
    assert mk0[50] == 0 and mk0[:50].all() and not mk0[100:].any()
    mean = rng.normal(size=8).astype(np.float32)
    std = rng.uniform(0.5, 2, 8).astype(np.float32)
    _, mk = net.gate(Y, Xr, fmin, fmax, 1.0)
    drag = torch.from_numpy(rng.normal(size=(8, nc))).cuda()
    ref = mlp.apply_drag(Y, mean, std, mk.cpu().numpy(), drag.cpu().numpy())
    net.apply_drag(Y, mean, std, mk, 4, drag)
    assert np.allclose(drag.cpu().numpy(), ref, rtol=1e-6, atol=1e-7)
    net.close()


def test_standardize(sgmod, mlp):
    net = make(sgmod, members=1)
    rng = np.random.default_rng(10)
    Xr = np.abs(rng.normal(size=(777, 392))).astype(np.float32) * 10
    mean = rng.normal(size=392).astype(np.float32)
    std = rng.uniform(0.5, 3, 392).astype(np.float32)
    fl = np.where(np.arange(392) % 3 == 0, 1e-3, 0).astype(np.float32)
    got = net.standardize(Xr, mean, std, fl).float().cpu().numpy()
    ref = mlp.standardize(Xr, mean, std, fl)
    # bfloat16 of the same value up to one unit in the 8th bit
    assert np.all(np.abs(got - ref) <= np.abs(ref) * 2.0 ** -7 + 1e-30)
    assert np.mean(got == mlp.bf16(ref)) > 0.98
    net.close()
