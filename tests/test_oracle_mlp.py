"""Pins of the FP64 reference network (oracle/mlp_ref.py) against what the
mathematics fixes: central finite differences of the loss, the feature
identity sin^2 + cos^2 = 1, the closed form of a first Adam step, the loss
of an exact fit, and BF16 rounding of known values."""
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
