"""Pins of the FP64 reference network (oracle/mlp_ref.py) against what the
mathematics fixes: a network small enough to evaluate by hand (its outputs
written into the test), central finite differences of the loss, the
feature identity sin^2 + cos^2 = 1, the closed form of a first Adam step,
the loss of an exact fit, and BF16 rounding of known values."""
import numpy as np
import pytest

from oracle import mlp_ref as M

CFG = dict(in_dim=5, n_freq=4, width=8, hidden=2, out_dim=5)


def random_params(cfg, seed):
    rng = np.random.default_rng(seed)
    n = cfg["n_freq"] * cfg["in_dim"] + sum(o * i + o for o, i in M.layer_dims(cfg))
    flat = rng.normal(0.0, 0.5, size=n)
    return flat


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    flat = random_params(CFG, 2)
    x = rng.uniform(-1, 1, size=(7, CFG["in_dim"]))
    t = rng.normal(size=(7, CFG["out_dim"]))
    loss, g = M.loss_and_grad(CFG, flat, x, t)
    nfix = CFG["n_freq"] * CFG["in_dim"]
    assert np.all(g[:nfix] == 0.0)
    h = 1e-6
    fd = np.zeros_like(flat)
    for k in range(nfix, flat.size):
        e = np.zeros_like(flat)
        e[k] = h
        lp, _ = M.loss_and_grad(CFG, flat + e, x, t)
        lm, _ = M.loss_and_grad(CFG, flat - e, x, t)
        fd[k] = (lp - lm) / (2 * h)
    err = np.linalg.norm(g[nfix:] - fd[nfix:]) / np.linalg.norm(fd[nfix:])
    assert err < 1e-6, err
    # every layer's block, separately
    k = nfix
    for out, inp in M.layer_dims(CFG):
        blk = slice(k, k + out * inp + out)
        assert np.linalg.norm(g[blk] - fd[blk]) <= 1e-6 * np.linalg.norm(fd[blk]) + 1e-12
        k += out * inp + out


def test_features_lie_on_the_unit_circle():
    rng = np.random.default_rng(3)
    freq = rng.normal(size=(6, 5))
    freq[0] = 0.0
    phi = M.features(rng.uniform(size=(9, 5)), freq)
    s, c = phi[:, :6], phi[:, 6:]
    assert np.allclose(s * s + c * c, 1.0, atol=1e-15)
    assert np.all(s[:, 0] == 0.0) and np.all(c[:, 0] == 1.0)
    # a frequency of one whole period per unit: phi(x + e_d) = phi(x)
    f1 = np.zeros((1, 5))
    f1[0, 1] = 1.0
    x = rng.uniform(size=(4, 5))
    x2 = x.copy()
    x2[:, 1] += 1.0
    assert np.allclose(M.features(x, f1), M.features(x2, f1), atol=1e-12)


def test_exact_fit_has_zero_loss_and_gradient():
    rng = np.random.default_rng(4)
    flat = random_params(CFG, 5)
    x = rng.uniform(size=(6, 5))
    y, _ = M.forward(CFG, flat, x)
    loss, g = M.loss_and_grad(CFG, flat, x, y)
    assert loss == 0.0 and np.all(g == 0.0)


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(6)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    z = np.zeros(50)
    lr = 1e-3
    p1, m1, v1 = M.adam_step(p, g, z, z, 1, lr, n_fixed=10)
    # bias correction makes the first step lr g / (|g| + eps)
    assert np.array_equal(p1[:10], p[:10])
    assert np.allclose(p1[10:], p[10:] - lr * g[10:] / (np.abs(g[10:]) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m1[10:], 0.1 * g[10:]) and np.allclose(v1[10:], 0.001 * g[10:] ** 2)


@pytest.mark.parametrize("value,expected", [
    (1.0, 1.0),
    (1.0 + 2.0 ** -8, 1.0),                     # tie, to even
    (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),     # tie, to even (upwards)
    (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),
    (-3.140625, -3.140625),                     # exactly representable
    (65504.0, 65536.0),
])
def test_bf16_rounding(value, expected):
    assert M.bf16_round(np.array([value]))[0] == expected


# A network evaluated by hand: two inputs, one frequency B = (1/4, 0), one
# tanh layer of width 2, one linear output.  Flat order: B, W0 [2][2] (its
# columns act on (sin, cos)), b0, W1 [1][2], b1.
HAND_CFG = dict(in_dim=2, n_freq=1, width=2, hidden=1, out_dim=1)
HAND_FLAT = np.array([0.25, 0.0,
                      1.0, 2.0, 0.5, -1.0, 0.0, 0.25,
                      2.0, -1.0, 0.1])
TANH_1 = 0.76159415595576488812
TANH_075 = 0.63514895238728731922
TANH_2 = 0.96402758007581688395


def test_forward_of_a_hand_evaluated_network():
    # x = (1, 0.3): 2 pi B.x = pi/2, phi = (1, 0); hidden pre-activations
    # (1, 0.75); y = 2 tanh(1) - tanh(0.75) + 0.1.
    # x = (0, 0): phi = (0, 1); pre-activations (2, -0.75);
    # y = 2 tanh(2) + tanh(0.75) + 0.1.
    x = np.array([[1.0, 0.3], [0.0, 0.0]])
    y, acts = M.forward(HAND_CFG, HAND_FLAT, x)
    assert y.shape == (2, 1)
    assert y[0, 0] == pytest.approx(0.98803935952424246, rel=0, abs=1e-15)
    assert y[1, 0] == pytest.approx(2.66320411253892109, rel=0, abs=1e-15)
    assert np.allclose(acts[0], [[1.0, 0.0], [0.0, 1.0]], atol=1e-15)
    assert np.allclose(acts[1], [[TANH_1, TANH_075], [TANH_2, -TANH_075]], atol=1e-15)


def test_loss_and_output_gradient_of_the_hand_network():
    x = np.array([[1.0, 0.3], [0.0, 0.0]])
    t = np.array([[1.0], [2.0]])
    d1 = 0.98803935952424246 - 1.0
    d2 = 2.66320411253892109 - 2.0
    loss, g = M.loss_and_grad(HAND_CFG, HAND_FLAT, x, t)
    assert loss == pytest.approx((d1 * d1 + d2 * d2) / 2, rel=1e-14)
    # dL/dy = 2 d / (n out) = d; last layer: dW1 = sum_k d_k h_k, db1 = sum d_k
    assert g[8] == pytest.approx(d1 * TANH_1 + d2 * TANH_2, rel=1e-13)
    assert g[9] == pytest.approx(d1 * TANH_075 - d2 * TANH_075, rel=1e-13)
    assert g[10] == pytest.approx(d1 + d2, rel=1e-13)
    # hidden bias b0[0]: d_k W1[0] (1 - h_k0^2) summed over the points
    want = 2.0 * (d1 * (1 - TANH_1 ** 2) + d2 * (1 - TANH_2 ** 2))
    assert g[6] == pytest.approx(want, rel=1e-13)
    assert g[0] == 0.0 and g[1] == 0.0   # frequencies are fixed
