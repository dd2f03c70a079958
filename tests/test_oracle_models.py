"""Pins of the oracle's Giesekus and Phan-Thien-Tanner source tensors (the
constitutive models the paper names as the next ones for its method).

The source tensor is chi = -R(E)/lambda + A.grad u + grad u^T.A with
E = A - I and R(E) = E + alpha E.E (Giesekus), (1 + eps tr E) E (linear
PTT), exp(eps tr E) E (exponential PTT).  Independent checks:
* the models reduce to Oldroyd-B at alpha = 0 / eps = 0 (whole iteration,
  bitwise);
* the relaxation term is objective (rotations);
* steady simple shear: the Giesekus polymer shear viscosity equals its
  classical closed form (1 - f)^2 / (1 + (1 - 2 alpha) f); the PTT shear
  stress and first normal stress follow from f^3 - f^2 - 2 eps Wi^2 = 0
  (linear) and f = exp(2 eps Wi^2 / f^2) (exponential), with A_yy = 1;
  the oracle's chi vanishes at those states;
* homogeneous relaxation of a uniform conformation at rest through the
  whole lattice iteration follows the ODE dE/dt = -R(E)/lambda, integrated
  in matrix form by a library ODE solver (logistic closed form for the
  diagonal Giesekus case).
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.optimize import brentq, fsolve

from oracle import analytic as AN
from oracle import oracle as O

MODELS = [(O.MODEL_GIESEKUS, 0.3), (O.MODEL_LPTT, 0.25), (O.MODEL_EPTT, 0.25)]


def relax_matrix(model, param, E):
    if model == O.MODEL_GIESEKUS:
        return E + param * E @ E
    tr = np.trace(E)
    if model == O.MODEL_LPTT:
        return (1 + param * tr) * E
    if model == O.MODEL_EPTT:
        return np.exp(param * tr) * E
    return E


def sym_pack(d, M):
    if d == 2:
        return np.array([M[0, 0], M[0, 1], M[1, 1]])
    return np.array([M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2]])


def test_zero_parameter_is_oldroyd_b():
    n = 16
    states = []
    for model in (None, O.MODEL_GIESEKUS, O.MODEL_LPTT, O.MODEL_EPTT):
        s = O.OracleSim(2, n, n)
        s.set_params(0.8, 0.501, 60.0, 0.05)
        if model is not None:
            s.set_model(model, 0.0)
        u0, p0 = AN.tg2d_fields(n, n, 1e-3)
        s.init(u0, None, p0)
        s.step(25)
        states.append(s.get_state())
    for st in states[1:]:
        for key in ("f", "h", "chi_prev"):
            assert np.array_equal(st[key], states[0][key]), key


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("model,param", MODELS)
def test_relaxation_is_objective(d, model, param):
    rng = np.random.default_rng(11)
    B = rng.normal(size=(d, d)) * 0.3
    E = B @ B.T - 0.1 * np.eye(d)          # symmetric, A = I + E positive definite
    Q, _ = np.linalg.qr(rng.normal(size=(d, d)))
    lam = 7.0
    G0 = np.zeros(d * d)
    chi = O.chi_tensor(d, lam, sym_pack(d, E + np.eye(d)), G0, model, param)
    chi_r = O.chi_tensor(d, lam, sym_pack(d, Q @ E @ Q.T + np.eye(d)), G0, model, param)
    C = np.zeros((d, d))
    idx = [(0, 0), (0, 1), (1, 1)] if d == 2 else [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for c, (a, b) in enumerate(idx):
        C[a, b] = C[b, a] = chi[c]
    assert np.allclose(chi_r, sym_pack(d, Q @ C @ Q.T), atol=1e-14)
    assert np.allclose(chi, sym_pack(d, -relax_matrix(model, param, E) / lam), atol=1e-14)


def shear_gradient(d, gd):
    G = np.zeros((d, d))
    G[1, 0] = gd                             # u = (gd y, 0): d_y u_x
    return G


@pytest.mark.parametrize("alpha", [0.1, 0.3, 0.5])
@pytest.mark.parametrize("Wi", [0.5, 1.0, 3.0])
def test_giesekus_steady_shear(alpha, Wi):
    lam = 40.0
    gd = Wi / lam
    G = shear_gradient(2, gd)

    def residual(v):
        E = np.array([[v[0], v[1]], [v[1], v[2]]])
        A = E + np.eye(2)
        chi = -relax_matrix(O.MODEL_GIESEKUS, alpha, E) / lam + A @ G + G.T @ A
        return [chi[0, 0] * lam, chi[0, 1] * lam, chi[1, 1] * lam]

    exx, exy, eyy = fsolve(residual, [2 * Wi ** 2, Wi, 0.0], xtol=1e-13)
    # classical Giesekus shear viscosity (polymer part, relative)
    X = np.sqrt((np.sqrt(1 + 16 * alpha * (1 - alpha) * Wi ** 2) - 1)
                / (8 * alpha * (1 - alpha) * Wi ** 2))
    f = (1 - X) / (1 + (1 - 2 * alpha) * X)
    assert exy / Wi == pytest.approx((1 - f) ** 2 / (1 + (1 - 2 * alpha) * f), rel=1e-10)
    chi = O.chi_tensor(2, lam, [1 + exx, exy, 1 + eyy], G.ravel(), O.MODEL_GIESEKUS, alpha)
    assert np.abs(chi).max() < 1e-12
    assert eyy < 0                            # a negative second normal stress


@pytest.mark.parametrize("model", [O.MODEL_LPTT, O.MODEL_EPTT])
@pytest.mark.parametrize("eps", [0.05, 0.25])
@pytest.mark.parametrize("Wi", [0.5, 2.0])
def test_ptt_steady_shear(model, eps, Wi):
    # A_yy = 1, E_xy = Wi/f, E_xx = 2 Wi^2/f^2, f = f(eps E_xx)
    lam = 40.0
    if model == O.MODEL_LPTT:
        roots = np.roots([1.0, -1.0, 0.0, -2 * eps * Wi ** 2])
        f = max(r.real for r in roots if abs(r.imag) < 1e-12)
    else:
        f = brentq(lambda f: f - np.exp(2 * eps * Wi ** 2 / f ** 2), 1.0, 1e3, xtol=1e-15)
    exy, exx = Wi / f, 2 * Wi ** 2 / f ** 2
    assert f > 1                              # shear thinning
    G = shear_gradient(2, Wi / lam)
    chi = O.chi_tensor(2, lam, [1 + exx, exy, 1.0], G.ravel(), model, eps)
    assert np.abs(chi).max() < 1e-12
    # 3D, the same shear in the x-y plane
    G3 = shear_gradient(3, Wi / lam)
    chi3 = O.chi_tensor(3, lam, [1 + exx, 1.0, 1.0, exy, 0.0, 0.0], G3.ravel(), model, eps)
    assert np.abs(chi3).max() < 1e-12


@pytest.mark.parametrize("model,param", MODELS)
def test_homogeneous_relaxation_follows_the_ode(model, param):
    # a uniform conformation at rest: every node relaxes alike, through the
    # whole iteration (populations, source, its backward difference)
    n, lam, eta_p, steps = 4, 150.0, 0.02, 300
    E0 = np.array([[0.8, 0.3], [0.3, -0.2]])
    s = O.OracleSim(2, n, n)
    s.set_params(0.8, 0.501, lam, eta_p)
    s.set_model(model, param)
    tau0 = np.tile(sym_pack(2, E0) * eta_p / lam, (n * n, 1))
    s.init(None, tau0, None)
    s.step(steps)
    A = s.moments()["A"]
    assert np.ptp(A, axis=0).max() < 1e-13   # still uniform
    sol = solve_ivp(lambda t, y: -relax_matrix(model, param, y.reshape(2, 2)).ravel() / lam,
                    (0, steps), E0.ravel(), rtol=1e-12, atol=1e-14)
    E = sol.y[:, -1].reshape(2, 2)
    got = A[0] - np.array([1.0, 0.0, 1.0])
    assert np.allclose(got, sym_pack(2, E), rtol=0, atol=2e-4 * np.abs(E0).max())


def test_giesekus_diagonal_relaxation_closed_form():
    # E = diag(y, 0): dy/dt = -(y + alpha y^2)/lambda, a logistic decay
    n, lam, alpha, y0, steps = 4, 200.0, 0.4, 1.5, 400
    s = O.OracleSim(2, n, n)
    s.set_params(0.8, 0.501, lam, 0.02)
    s.set_model(O.MODEL_GIESEKUS, alpha)
    s.init(None, np.tile([y0 * 0.02 / lam, 0.0, 0.0], (n * n, 1)), None)
    s.step(steps)
    y = s.moments()["A"][0, 0] - 1
    e = np.exp(-steps / lam)
    want = y0 * e / (1 + alpha * y0 * (1 - e))
    assert y == pytest.approx(want, rel=2e-4)
