"""The warm-start network on the GPU against the FP64 reference.

Both sides start from the same parameters and inputs; the reference
rounds the matrix-product operands to BF16 where the kernels do, so the
remaining differences are FP32 accumulation and FP32 transcendental
functions: per tensor relative L2 <= 1e-2 (the bar for BF16 operands).
"""
import numpy as np
import pytest

from oracle import mlp_ref as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_13072_amd import vflb
    vflb.lib()
    return vflb


CFG = dict(in_dim=5, n_freq=32, width=64, hidden=3, out_dim=5)


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-30)


def make(V, seed=11, max_batch=256, cfg=CFG):
    return V.Mlp(**cfg, max_batch=max_batch, sigma=1.0, seed=seed)


def inputs(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, size=(n, 5))
    t = 0.5 * np.sin(3 * x[:, :1] + x[:, 1:2]) + 0.1 * rng.normal(size=(n, 5))
    return x, t


def test_param_count_and_roundtrip(V):
    m = make(V)
    n = 32 * 5 + (64 * 64 + 64) + 2 * (64 * 64 + 64) + (5 * 64 + 5)
    assert m.nparams == n
    p = m.get_params()
    m.set_params(p * 0.5)
    assert np.array_equal(m.get_params(), (p * 0.5).astype(np.float32))


def test_production_shape_param_count(V):
    m = V.Mlp(max_batch=64)
    assert m.nparams == 128 * 5 + 198661  # frequencies + the trained parameters


@pytest.mark.parametrize("n", [64, 100, 256])
def test_forward_matches_reference(V, n):
    m = make(V)
    flat = m.get_params().astype(np.float64)
    x, _ = inputs(n, 1)
    x = x.astype(np.float32).astype(np.float64)
    y_gpu = m.forward(x).cpu().numpy()
    y_ref, _ = M.forward(CFG, flat, x, bf16=True)
    assert rel(y_gpu, y_ref) <= 1e-2
    y64, _ = M.forward(CFG, flat, x, bf16=False)
    assert rel(y_gpu, y64) <= 5e-2  # BF16 operands against exact FP64


def test_forward_chunks_beyond_max_batch(V):
    m = make(V, max_batch=128)
    x, _ = inputs(300, 2)
    y = m.forward(x).cpu().numpy()
    y1 = np.concatenate([m.forward(x[:128]).cpu().numpy(), m.forward(x[128:256]).cpu().numpy(),
                         m.forward(x[256:]).cpu().numpy()])
    assert np.array_equal(y, y1)


@pytest.mark.parametrize("n", [64, 200])
def test_gradients_match_reference(V, n):
    m = make(V)
    flat = m.get_params().astype(np.float64)
    x, t = inputs(n, 3)
    x = x.astype(np.float32).astype(np.float64)
    t = t.astype(np.float32).astype(np.float64)
    loss, g = m.grad(x, t)
    loss_ref, g_ref = M.loss_and_grad(CFG, flat, x, t, bf16=True)
    assert abs(loss - loss_ref) <= 1e-2 * loss_ref
    k = CFG["n_freq"] * CFG["in_dim"]
    assert np.all(g[:k] == 0)
    for l, (out, inp) in enumerate(M.layer_dims(CFG)):
        gw = slice(k, k + out * inp)
        gb = slice(k + out * inp, k + out * inp + out)
        assert rel(g[gw], g_ref[gw]) <= 1e-2, ("W", l, rel(g[gw], g_ref[gw]))
        assert rel(g[gb], g_ref[gb]) <= 1e-2, ("b", l, rel(g[gb], g_ref[gb]))
        k += out * inp + out


def test_adam_step_matches_reference(V):
    import torch
    m = make(V)
    flat = m.get_params().astype(np.float64)
    x, t = inputs(128, 4)
    xd = torch.tensor(x, dtype=torch.float32, device="cuda")
    td = torch.tensor(t, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    lr = 1e-3
    _, g = m.grad(x, t)
    m.train_step(xd, td, lr)
    new = m.get_params().astype(np.float64)
    nfix = CFG["n_freq"] * CFG["in_dim"]
    assert np.array_equal(new[:nfix], flat[:nfix])
    ref, _, _ = M.adam_step(flat, g.astype(np.float64), np.zeros_like(flat), np.zeros_like(flat),
                            1, lr, n_fixed=nfix)
    big = np.abs(g) > 1e-5  # first step moves each parameter by ~lr sign(g)
    d_gpu, d_ref = (new - flat)[big], (ref - flat)[big]
    assert np.all(np.abs(d_gpu - d_ref) <= 1e-3 * lr + 1e-6 * np.abs(flat[big]))


# The shape the warm start trains: 128 frequencies (K = 256 for the first
# product), width 256 (four 64-wide N tiles), 3 hidden layers, on 1024 rows.
PROD = dict(in_dim=5, n_freq=128, width=256, hidden=3, out_dim=5)


@pytest.fixture(scope="module")
def prod_case(V):
    m = make(V, seed=12, max_batch=1024, cfg=PROD)
    flat = m.get_params().astype(np.float64)
    x, t = inputs(1024, 6)
    x = x.astype(np.float32).astype(np.float64)
    t = t.astype(np.float32).astype(np.float64)
    return m, flat, x, t


def test_forward_matches_reference_production_shape(V, prod_case):
    m, flat, x, _ = prod_case
    y_gpu = m.forward(x).cpu().numpy()
    y_ref, _ = M.forward(PROD, flat, x, bf16=True)
    assert rel(y_gpu, y_ref) <= 1e-2, rel(y_gpu, y_ref)


def test_gradients_match_reference_production_shape(V, prod_case):
    m, flat, x, t = prod_case
    loss, g = m.grad(x, t)
    loss_ref, g_ref = M.loss_and_grad(PROD, flat, x, t, bf16=True)
    assert abs(loss - loss_ref) <= 1e-2 * loss_ref
    k = PROD["n_freq"] * PROD["in_dim"]
    assert np.all(g[:k] == 0)
    for l, (out, inp) in enumerate(M.layer_dims(PROD)):
        gw = slice(k, k + out * inp)
        gb = slice(k + out * inp, k + out * inp + out)
        assert rel(g[gw], g_ref[gw]) <= 1e-2, ("W", l, rel(g[gw], g_ref[gw]))
        assert rel(g[gb], g_ref[gb]) <= 1e-2, ("b", l, rel(g[gb], g_ref[gb]))
        k += out * inp + out


def test_adam_step_matches_reference_production_shape(V, prod_case):
    import torch
    m, flat, x, t = prod_case
    m.set_params(flat.astype(np.float32))   # also resets Adam
    xd = torch.tensor(x, dtype=torch.float32, device="cuda")
    td = torch.tensor(t, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    lr = 1e-3
    _, g = m.grad(x, t)
    m.train_step(xd, td, lr)
    new = m.get_params().astype(np.float64)
    nfix = PROD["n_freq"] * PROD["in_dim"]
    assert np.array_equal(new[:nfix], flat[:nfix])
    ref, _, _ = M.adam_step(flat, g.astype(np.float64), np.zeros_like(flat),
                            np.zeros_like(flat), 1, lr, n_fixed=nfix)
    big = np.abs(g) > 1e-5
    d_gpu, d_ref = (new - flat)[big], (ref - flat)[big]
    assert np.all(np.abs(d_gpu - d_ref) <= 1e-3 * lr + 1e-6 * np.abs(flat[big]))
    m.set_params(flat.astype(np.float32))


def test_training_reduces_the_loss(V):
    import torch
    m = make(V, max_batch=512)
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, size=(512, 5))
    t = np.stack([np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1]),
                  -np.cos(2 * np.pi * x[:, 0]) * np.sin(2 * np.pi * x[:, 1]),
                  x[:, 3], x[:, 2] * x[:, 3], 0.5 * np.ones(512)], axis=1)
    xd = torch.tensor(x, dtype=torch.float32, device="cuda")
    td = torch.tensor(t, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    first = m.train_step(xd, td, 3e-3)
    for _ in range(400):
        m.train_step(xd, td, 3e-3, want_loss=False)
    last = m.train_step(xd, td, 3e-3)
    assert np.isfinite(last) and last < 0.05 * first, (first, last)


def test_init_from_mlp_sets_the_predicted_fields(V):
    m = make(V, max_batch=1024)
    nx, ny = 48, 40
    sim = V.Sim(2, nx, ny, 1, "f64", stream=m.stream)
    sim.set_params(1.0, 0.5, 0.5, 0.01, nx / (2 * np.pi))
    extra = (np.log(0.5), 0.5, 0.0)
    sim.init_from_mlp(m, extra, 0.01, 2e-5)
    xs, ys = np.meshgrid(np.arange(nx) / nx, np.arange(ny) / ny)
    X = np.stack([xs.ravel(), ys.ravel(), np.full(nx * ny, extra[0]), np.full(nx * ny, extra[1]),
                  np.full(nx * ny, extra[2])], axis=1)
    y = m.forward(X).cpu().numpy().astype(np.float64)
    mo = sim.moments()
    assert sim.t == 0
    # the forward pass on the same inputs gives the same outputs (FP32
    # scaling); the lattice is periodic on both axes, so the velocity is
    # projected onto the fields without central divergence, mean and
    # staggered modes (numpy's FFT as the reference of the library's DFT)
    y32 = y.astype(np.float32)  # the kernel scales in FP32
    u32 = (np.float32(0.01) * y32[:, :2]).astype(np.float64)
    U = [np.fft.fft2(u32[:, c].reshape(ny, nx)) for c in range(2)]
    KX, KY = np.meshgrid(np.arange(nx), np.arange(ny))
    sx, sy = np.sin(2 * np.pi * KX / nx), np.sin(2 * np.pi * KY / ny)
    blind = ((KX == 0) & (KY == 0)) | (2 * KX == nx) | (2 * KY == ny)
    ss = np.where(blind, 1.0, sx * sx + sy * sy)
    d = (sx * U[0] + sy * U[1]) / ss
    U = [np.where(blind, 0, U[0] - sx * d), np.where(blind, 0, U[1] - sy * d)]
    u0 = np.stack([np.fft.ifft2(U[c]).real.ravel() for c in range(2)], 1)
    assert rel(u32, u0) > 1e-3                     # there was something to remove
    assert rel(mo["u"], u0) <= 1e-5, rel(mo["u"], u0)
    # no central divergence, no mean
    ux, uy = mo["u"][:, 0].reshape(ny, nx), mo["u"][:, 1].reshape(ny, nx)
    div = 0.5 * (np.roll(ux, -1, 1) - np.roll(ux, 1, 1) + np.roll(uy, -1, 0) - np.roll(uy, 1, 0))
    assert np.abs(div).max() <= 1e-5 * np.abs(mo["u"]).max()
    assert np.abs(mo["u"].mean(0)).max() <= 1e-6 * np.abs(mo["u"]).max()
    # tau: the network's, unless the conformation floor moved it (A = I +
    # c tau with c = lambda / eta_p)
    lp = sim.lattice_params()
    c = lp["lam"] / lp["eta_p"]
    t32 = (np.float32(2e-5) * y32[:, 2:]).astype(np.float64)
    axx, axy, ayy = 1 + c * t32[:, 0], c * t32[:, 1], 1 + c * t32[:, 2]
    lmin = 0.5 * (axx + ayy) - np.sqrt(0.25 * (axx - ayy) ** 2 + axy ** 2)
    keep = lmin >= 0.05
    assert rel(mo["tau"][keep], t32[keep]) <= 1e-6
    # the same state as vflb_init_fields of those fields with p = 0 (the
    # read-back pressure carries the tau_f f^B_0 term of the stress)
    ref = V.Sim(2, nx, ny, 1, "f64")
    ref.set_params(1.0, 0.5, 0.5, 0.01, nx / (2 * np.pi))
    ref.init_fields(sim.read(V.FIELD_U), sim.read(V.FIELD_TAU), None)
    mr = ref.moments()
    for k in ("u", "p", "tau"):
        assert rel(mo[k], mr[k]) <= 1e-12, k
    sim.step(20)
    ref.step(20)
    assert rel(sim.read(V.FIELD_U), ref.read(V.FIELD_U)) <= 1e-12
