"""Pins of the oracle's stress-divergence scheme (the "original" scheme the
paper compares its method against in Sec. 3: the divergence of the polymer
stress as a body force, no fluctuation term).

The paper describes that scheme only in words; the oracle's reading is
second-order central differences of tau_p(t), one-sided second-order
differences normal to a wall, and the force entering the Guo term, the
velocity and the pressure.  The pins: the stencil is exact on quadratic
fields (and on sines up to the closed-form sin(k)/k factor); with no
polymer (beta = 1) the two schemes are the same iteration; the velocity
moment carries half the polymer force; and the whole iteration reproduces
the linear viscoelastic Taylor-Green decay and the steady Oldroyd-B channel
(Sec. 3.2) that the paper's method reproduces.
"""
import numpy as np
import pytest

from oracle import analytic as AN
from oracle import oracle as O

TAU_H = 0.501
D_H = (TAU_H - 0.5) / 3.0


def sim(nx, ny, walls, scheme, tau_f=0.8, lam=50.0, eta_p=0.1):
    s = O.OracleSim(2, nx, ny)
    s.set_params(tau_f, TAU_H, lam, eta_p)
    s.set_walls(walls)
    s.set_scheme(scheme)
    return s


@pytest.mark.parametrize("axis", [0, 1])
def test_divergence_exact_on_quadratics_between_walls(axis):
    n, m = 9, 4
    nx, ny = (n, m) if axis == 0 else (m, n)
    walls = (1, 0, 0) if axis == 0 else (0, 1, 0)
    s = sim(nx, ny, walls, O.SCHEME_STRESS_DIVERGENCE)
    X, Y = np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5)
    r = (X if axis == 0 else Y).ravel()
    txx = 0.01 * r + 0.002 * r * r
    txy = 0.002 + 0.003 * r - 0.0004 * r * r
    tyy = -0.001 * r * r + 0.004
    s.init(None, np.stack([txx, txy, tyy], 1), None)
    div = s.stress_divergence()
    if axis == 0:   # d/dx only: div_x = d_x txx, div_y = d_x txy
        want = np.stack([0.01 + 0.004 * r, 0.003 - 0.0008 * r], 1)
    else:           # d/dy only: div_x = d_y txy, div_y = d_y tyy
        want = np.stack([0.003 - 0.0008 * r, -0.002 * r], 1)
    assert np.abs(div - want).max() < 1e-15


def test_divergence_central_on_a_periodic_mode():
    # central differences of sin(k x) give cos(k x) sin(k): the closed form
    # of the discrete operator, which also fixes the sign and the component
    n = 16
    k = 2 * np.pi / n
    s = sim(n, n, (0, 0, 0), O.SCHEME_STRESS_DIVERGENCE)
    X, Y = np.meshgrid(np.arange(n), np.arange(n))
    x, y = X.ravel(), Y.ravel()
    txx = 1e-3 * np.sin(k * x)
    txy = 2e-3 * np.cos(k * y) + 1e-3 * np.sin(k * x)
    tyy = 3e-3 * np.sin(k * y)
    s.init(None, np.stack([txx, txy, tyy], 1), None)
    div = s.stress_divergence()
    sk = np.sin(k)
    want_x = 1e-3 * np.cos(k * x) * sk - 2e-3 * np.sin(k * y) * sk
    want_y = 1e-3 * np.cos(k * x) * sk + 3e-3 * np.cos(k * y) * sk
    assert np.abs(div[:, 0] - want_x).max() < 1e-17
    assert np.abs(div[:, 1] - want_y).max() < 1e-17


def test_velocity_moment_carries_half_the_polymer_force():
    # at t = 0 with u0 = 0 the populations carry no momentum, so the
    # velocity read back is (F + div tau_p)/2
    n = 12
    s = sim(n, n, (0, 1, 0), O.SCHEME_STRESS_DIVERGENCE)
    s.set_force(O.FORCE_CONST, (1e-6, 0.0, 0.0))
    X, Y = np.meshgrid(np.arange(n), np.arange(n) + 0.5)
    txy = 1e-4 * np.sin(2 * np.pi * X / n).ravel() * (Y.ravel() / n)
    tau = np.stack([0 * txy, txy, 0.5 * txy], 1)
    s.init(None, tau, None)
    div = s.stress_divergence()
    u = s.moments()["u"]
    assert np.abs(u[:, 0] - 0.5 * (1e-6 + div[:, 0])).max() < 1e-18
    assert np.abs(u[:, 1] - 0.5 * div[:, 1]).max() < 1e-18
    # the fluctuating scheme's velocity ignores the stress
    s.set_scheme(O.SCHEME_FLUCTUATING)
    assert np.abs(s.moments()["u"][:, 0] - 0.5e-6).max() < 1e-18


def test_no_polymer_schemes_identical():
    # beta = 1: eta_p = 0, so f^B = 0 and div tau_p = 0: the same iteration
    n = 16
    out = []
    for scheme in (O.SCHEME_FLUCTUATING, O.SCHEME_STRESS_DIVERGENCE):
        s = sim(n, n, (0, 1, 0), scheme, eta_p=0.0)
        s.set_force(O.FORCE_CONST, (2e-6, 0.0, 0.0))
        u0, p0 = AN.tg2d_fields(n, n, 1e-3)
        s.init(u0, None, p0)
        s.step(30)
        out.append(s.get_state())
    for key in ("f", "h", "chi_prev", "u_prev"):
        assert np.array_equal(out[0][key], out[1][key]), key


def test_schemes_differ_with_polymer():
    # the same start with a polymer stress: the schemes are different
    # iterations (a wiring mistake that ignored the scheme would pass above)
    n = 16
    res = []
    for scheme in (O.SCHEME_FLUCTUATING, O.SCHEME_STRESS_DIVERGENCE):
        s = sim(n, n, (0, 0, 0), scheme)
        u0, p0 = AN.tg2d_fields(n, n, 1e-3)
        s.init(u0, None, p0)
        s.step(20)
        res.append(s.moments()["u"])
    d = np.abs(res[0] - res[1]).max()
    assert 1e-12 < d < 1e-4


@pytest.mark.parametrize("beta,lam", [(0.1, 200.0), (0.5, 60.0)])
def test_linear_viscoelastic_taylor_green_2d(beta, lam):
    # the linear mode equations a' = -kappa (nu_s a + s),
    # s' = -(1/lam + kappa D) s + (nu_p/lam) a, with the polymer force of
    # the mode entering through div tau_p instead of f^B.  Central
    # differences scale the force (div tau_p) and the stress source (grad u)
    # by sin(k)/k each; a(t) from a(0) = 1, s(0) = 0 depends on the product
    # of the two couplings only, so nu_p carries the factor (sin k / k)^2.
    n, U0, nu = 32, 1e-4, 0.1
    k = 2 * np.pi / n
    nu_s, nu_p = beta * nu, (1 - beta) * nu
    sinc2 = (np.sin(k) / k) ** 2
    s = O.OracleSim(2, n, n)
    s.set_params(3 * nu_s + 0.5, TAU_H, lam, nu_p)
    s.set_scheme(O.SCHEME_STRESS_DIVERGENCE)
    u0, p0 = AN.tg2d_fields(n, n, U0)
    s.init(u0, None, p0)
    ts = [50, 150, 300, 500]
    a_ref, _ = AN.tg_linear_viscoelastic(ts, 1.0, 0.0, 2 * k * k, nu_s, nu_p * sinc2, lam, D_H)
    for t, ar in zip(ts, a_ref):
        s.step(t - s.t)
        u = s.moments()["u"]
        a = (u * u0 / U0).sum() / ((u0 / U0) ** 2).sum() / U0
        assert abs(a - ar) < 6e-3, (t, a, ar)


def test_steady_poiseuille():
    # steady Oldroyd-B channel (Sec. 3.2), Re = 1, Wi = 1, beta = 0.1, with
    # the conformation scheme's diffusion constant in A_xx
    nu, beta, L = 0.5, 0.1, 32
    U0 = nu / L
    lam = L / U0
    g = 8 * nu * U0 / L ** 2
    s = O.OracleSim(2, 1, L)
    s.set_params(3 * beta * nu + 0.5, TAU_H, lam, (1 - beta) * nu)
    s.set_walls((0, 1, 0))
    s.set_force(O.FORCE_CONST, (g, 0.0, 0.0))
    s.set_scheme(O.SCHEME_STRESS_DIVERGENCE)
    s.init()
    s.step(int(25 * max(L * L / nu, lam)))
    m = s.moments()
    u, A = m["u"], m["A"]
    y = np.arange(L) + 0.5
    ux, Axx, Axy, _ = AN.poiseuille_steady(y, L, g, beta * nu, (1 - beta) * nu, lam, D_H)
    bulk = slice(L // 4, 3 * L // 4)
    assert np.abs(u[:, 1]).max() < 1e-12 * U0
    assert np.abs(A[:, 2] - 1).max() < 1e-9
    assert AN.gre(u[:, 0], ux) < 2e-2
    assert AN.gre(A[:, 1], Axy) < 1e-2
    assert np.allclose(A[bulk, 0], Axx[bulk], rtol=2e-3)


# ------------------------------------------------------------ D3Q19
# The same reading in three dimensions (the Taylor-Green comparison of the
# paper's 3D performance table): six stress components, div tau_p with three
# components, the z axis treated like x and y.

def sim3(n, walls, scheme, tau_f=0.8, lam=50.0, eta_p=0.1):
    s = O.OracleSim(3, *n)
    s.set_params(tau_f, TAU_H, lam, eta_p)
    s.set_walls(walls)
    s.set_scheme(scheme)
    return s


def test_divergence_3d_exact_on_quadratics_between_z_walls():
    nx, ny, nz = 3, 4, 9
    s = sim3((nx, ny, nz), (0, 0, 1), O.SCHEME_STRESS_DIVERGENCE)
    Z = (np.arange(nz) + 0.5)[:, None, None] * np.ones((nz, ny, nx))
    z = Z.ravel()
    # components (xx, yy, zz, xy, xz, yz); only d/dz acts
    tau = np.stack([0.001 * z, 0.002 * z * z, 0.01 * z - 0.0003 * z * z,
                    0.004 + 0.0 * z, 0.003 * z - 0.0004 * z * z, 0.0005 * z * z], 1)
    s.init(None, tau, None)
    div = s.stress_divergence()
    # div_x = d_z tau_xz, div_y = d_z tau_yz, div_z = d_z tau_zz
    want = np.stack([0.003 - 0.0008 * z, 0.001 * z, 0.01 - 0.0006 * z], 1)
    assert np.abs(div - want).max() < 1e-15


def test_divergence_3d_central_on_periodic_modes():
    n = 12
    k = 2 * np.pi / n
    s = sim3((n, n, n), (0, 0, 0), O.SCHEME_STRESS_DIVERGENCE)
    Z, Y, X = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    x, y, z = X.ravel(), Y.ravel(), Z.ravel()
    tau = np.zeros((n ** 3, 6))
    tau[:, 0] = 1e-3 * np.sin(k * x)
    tau[:, 2] = 2e-3 * np.sin(k * z)
    tau[:, 4] = 3e-3 * np.cos(k * z)            # xz
    tau[:, 5] = 4e-3 * np.sin(k * y)            # yz
    s.init(None, tau, None)
    div = s.stress_divergence()
    sk = np.sin(k)
    want = np.stack([1e-3 * np.cos(k * x) * sk - 3e-3 * np.sin(k * z) * sk,
                     0.0 * x,
                     2e-3 * np.cos(k * z) * sk + 3e-3 * 0.0 * x + 4e-3 * np.cos(k * y) * sk], 1)
    # div_x = d_x txx + d_z txz; div_y = d_z tyz (= 0 here); div_z = d_z tzz + d_y tyz
    assert np.abs(div - want).max() < 1e-17


def test_no_polymer_schemes_identical_3d():
    out = []
    for scheme in (O.SCHEME_FLUCTUATING, O.SCHEME_STRESS_DIVERGENCE):
        s = sim3((6, 5, 8), (0, 0, 1), scheme, eta_p=0.0)
        s.set_force(O.FORCE_CONST, (2e-6, -1e-6, 0.0))
        u = 1e-3 * np.random.default_rng(3).normal(size=(240, 3))
        s.init(u, None, None)
        s.step(12)
        out.append(s.get_state())
    for key in ("f", "h", "chi_prev", "u_prev"):
        assert np.array_equal(out[0][key], out[1][key]), key


def test_linear_viscoelastic_taylor_green_3d():
    # The 3D vortex phi = (sin x cos y cos z, -cos x sin y cos z, 0) is one
    # mode of |k|^2 = 3 k^2 (kappa).  With u = U0 a phi and tau = U0 s S,
    # S = grad phi + grad phi^T, central differences give the stress source
    # sinc grad phi and the force sinc div tau (sinc = sin(k)/k):
    #   a' = -kappa (nu_s a + sinc s),  s' = -(1/lam + kappa D) s + (nu_p/lam) sinc a,
    # i.e. the closed form with s~ = sinc s and nu_p sinc^2.  The
    # equilibrium-only start leaves an O(k^2) initial layer, so the closed
    # form starts from the amplitudes measured after it (t0 = 20).
    n, U0, nu, beta, lam = 24, 1e-4, 0.05, 0.2, 80.0
    k = 2 * np.pi / n
    sinc = np.sin(k) / k
    nu_s, nu_p = beta * nu, (1 - beta) * nu
    s = sim3((n, n, n), (0, 0, 0), O.SCHEME_STRESS_DIVERGENCE, tau_f=3 * nu_s + 0.5, lam=lam,
             eta_p=nu_p)
    x = 2 * np.pi * np.arange(n) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    cx, sx, cy, sy, cz, sz = np.cos(X), np.sin(X), np.cos(Y), np.sin(Y), np.cos(Z), np.sin(Z)
    phi = np.stack([sx * cy * cz, -cx * sy * cz, 0 * X], -1).reshape(-1, 3)
    S = np.stack([2 * k * cx * cy * cz, -2 * k * cx * cy * cz, 0 * X, 0 * X,
                  -k * sx * cy * sz, k * cx * sy * sz], -1).reshape(-1, 6)
    wts = np.array([1, 1, 1, 2, 2, 2.0])
    p0 = (U0 ** 2 / 16) * ((np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2)).reshape(-1)
    s.init(U0 * phi, None, p0)
    s.step(20)
    m = s.moments()
    a0 = (m["u"] * phi).sum() / (phi ** 2).sum() / U0
    s0 = (m["tau"] * S * wts).sum() / (S * S * wts).sum() / U0
    assert AN.rel_l2(m["tau"], s0 * U0 * S) < 2e-2   # the stress keeps the strain's shape
    ts = [60, 140, 220]
    a_ref, _ = AN.tg_linear_viscoelastic(np.array(ts) - 20, a0, sinc * s0, 3 * k * k, nu_s,
                                         nu_p * sinc ** 2, lam, D_H)
    for t, ar in zip(ts, a_ref):
        s.step(t - s.t)
        a = (s.moments()["u"] * phi).sum() / (phi ** 2).sum() / U0
        # O(k^2) dispersion of the lattice: 6e-3 at n = 24 (the same closed
        # form without the two sinc factors is 1.4e-2 away at t = 140)
        assert abs(a - ar) < 7e-3, (t, a, ar)
