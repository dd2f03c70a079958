"""Physics pins of the FP64 oracle against closed-form solutions: the
Newtonian limit (Taylor-Green decay), the linear viscoelastic Taylor-Green
mode, steady and start-up Poiseuille flow (Sec. 3.2), Womersley flow
(Sec. 3.3) and the four-roll mill (Sec. 3.1).  These run the whole
iteration, so a dropped term or a wrong sign anywhere in the coupling
f^B <-> h <-> grad u shows up as a wrong decay rate, profile or stress.
"""
import numpy as np
import pytest

from oracle import analytic as AN
from oracle import oracle as O

TAU_H = 0.501
D_H = (TAU_H - 0.5) / 3.0


def tg_mode_amplitude(u, shape_fn):
    phi = shape_fn
    return (u * phi).sum() / (phi * phi).sum()


def test_newtonian_taylor_green_decay():
    # beta = 1: no polymer, Guo incompressible LBGK; the 2D Taylor-Green
    # mode decays as exp(-2 nu k^2 t) at any Re (the advection term is a
    # gradient).  Error budget O(k^2) + O(Ma^2).  The equilibrium-only
    # initial state lacks the non-equilibrium stress, so the first few steps
    # decay faster; the rate is measured after that initial layer.
    n, U0, nu = 32, 0.01, 0.05
    k = 2 * np.pi / n
    s = O.OracleSim(2, n, n)
    s.set_params(3 * nu + 0.5, TAU_H, 10.0, 0.0)
    u0, p0 = AN.tg2d_fields(n, n, U0)
    s.init(u0, None, p0)
    amps = []
    for t in (50, 300):
        s.step(t - s.t)
        u = s.moments()["u"]
        amps.append(tg_mode_amplitude(u, u0 / U0))
        # the field keeps its shape
        assert AN.rel_l2(u, amps[-1] / U0 * u0) < 1e-3
    rate = np.log(amps[0] / amps[1]) / 250.0
    assert rate == pytest.approx(2 * nu * k * k, rel=2e-3)
    assert amps[1] / U0 == pytest.approx(np.exp(-2 * nu * k * k * 300), rel=1.5e-2)


@pytest.mark.parametrize("beta,lam", [(0.1, 200.0), (0.5, 60.0)])
def test_linear_viscoelastic_taylor_green_2d(beta, lam):
    # Small U0: the mode amplitude a(t) and the stress amplitude s(t) follow
    # a' = -kappa (nu_s a + s), s' = -(1/lam + kappa D) s + (nu_p/lam) a,
    # kappa = 2 k^2.  beta = 0.1 with lam = 200 oscillates (elastic recoil).
    n, U0, nu = 32, 1e-4, 0.1
    k = 2 * np.pi / n
    nu_s, nu_p = beta * nu, (1 - beta) * nu
    s = O.OracleSim(2, n, n)
    s.set_params(3 * nu_s + 0.5, TAU_H, lam, nu_p)
    u0, p0 = AN.tg2d_fields(n, n, U0)
    s.init(u0, None, p0)
    ts = [50, 150, 300, 500]
    a_ref, _ = AN.tg_linear_viscoelastic(ts, 1.0, 0.0, 2 * k * k, nu_s, nu_p, lam, D_H)
    for t, ar in zip(ts, a_ref):
        s.step(t - s.t)
        a = tg_mode_amplitude(s.moments()["u"], u0 / U0) / U0
        assert abs(a - ar) < 6e-3, (t, a, ar)


def test_linear_viscoelastic_taylor_green_3d():
    # 3D vortex u = U0 (sin x cos y cos z, -cos x sin y cos z, 0):
    # kappa = 3 k^2.  The equilibrium-only start leaves an O(k^2) initial
    # layer, so the closed form is started from the velocity and stress
    # amplitudes measured after it (t0 = 20) and compared later on.
    n, U0, nu, beta, lam = 16, 1e-4, 0.05, 0.2, 80.0
    k = 2 * np.pi / n
    nu_s, nu_p = beta * nu, (1 - beta) * nu
    s = O.OracleSim(3, n, n, n)
    s.set_params(3 * nu_s + 0.5, TAU_H, lam, nu_p)
    x = 2 * np.pi * np.arange(n) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    cx, sx, cy, sy, cz, sz = np.cos(X), np.sin(X), np.cos(Y), np.sin(Y), np.cos(Z), np.sin(Z)
    u0 = np.stack([sx * cy * cz, -cx * sy * cz, np.zeros_like(X)], -1).reshape(-1, 3)
    # strain rate of the unit-amplitude mode, components (xx, yy, zz, xy, xz, yz)
    S = np.stack([2 * k * cx * cy * cz, -2 * k * cx * cy * cz, 0 * X, 0 * X,
                  -k * sx * cy * sz, k * cx * sy * sz], -1).reshape(-1, 6)
    wts = np.array([1, 1, 1, 2, 2, 2.0])
    # pressure of the theta = 0 vortex: (U0^2/16)(cos 2x + cos 2y)(cos 2z + 2)
    p0 = (U0 ** 2 / 16) * ((np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2)).reshape(-1)
    s.init(U0 * u0, None, p0)
    s.step(20)
    m = s.moments()
    a0 = tg_mode_amplitude(m["u"], u0) / U0
    s0 = (m["tau"] * S * wts).sum() / (S * S * wts).sum() / U0
    # the stress keeps the shape of the strain rate
    assert AN.rel_l2(m["tau"], s0 * U0 * S) < 2e-2
    ts = [60, 140, 220]
    a_ref, _ = AN.tg_linear_viscoelastic(np.array(ts) - 20, a0, s0, 3 * k * k, nu_s, nu_p,
                                         lam, D_H)
    for t, ar in zip(ts, a_ref):
        s.step(t - s.t)
        a = tg_mode_amplitude(s.moments()["u"], u0) / U0
        assert abs(a - ar) < 1e-2, (t, a, ar)   # O(k^2) dispersion at n = 16


def channel(ny, nu_s, nu_p, lam, g, nx=1, tau_h=TAU_H):
    s = O.OracleSim(2, nx, ny)
    s.set_params(3 * nu_s + 0.5, tau_h, lam, nu_p)
    s.set_walls((0, 1, 0))
    s.set_force(O.FORCE_CONST, (g, 0.0, 0.0))
    s.init()
    return s


def channel_profiles(s, ny, nx=1):
    m = s.moments()
    u = m["u"].reshape(ny, nx, 2)[:, 0]
    A = m["A"].reshape(ny, nx, 3)[:, 0]
    return u, A


def test_steady_poiseuille_paper_tau_h():
    # Steady Oldroyd-B channel flow (Sec. 3.2) at Re = 1, Wi = 1,
    # beta = 0.1, tau_h = 0.501.  Away from the walls A_xx carries the
    # diffusion constant 4 D lam^3 (g/nu)^2 of the conformation scheme on
    # top of 1 + 2 (lam du/dy)^2; A_yy = 1 and u_y = 0 exactly at steady
    # state.
    nu, beta, L = 0.5, 0.1, 32
    U0 = nu / L
    lam = L / U0
    g = 8 * nu * U0 / L ** 2
    s = channel(L, beta * nu, (1 - beta) * nu, lam, g)
    s.step(int(25 * max(L * L / nu, lam)))
    u, A = channel_profiles(s, L)
    y = np.arange(L) + 0.5
    ux, Axx, Axy, _ = AN.poiseuille_steady(y, L, g, beta * nu, (1 - beta) * nu, lam, D_H)
    bulk = slice(L // 4, 3 * L // 4)
    assert np.allclose(A[bulk, 0], Axx[bulk], rtol=1e-5)
    # without the diffusion constant the bulk would be off by ~1.5e-3
    _, Axx0, _, _ = AN.poiseuille_steady(y, L, g, beta * nu, (1 - beta) * nu, lam, 0.0)
    assert np.abs(A[bulk, 0] / Axx0[bulk] - 1).max() > 1e-4
    assert np.abs(A[:, 2] - 1).max() < 1e-9
    assert np.abs(u[:, 1]).max() < 1e-12 * U0
    assert AN.gre(u[:, 0], ux) < 1e-2
    assert AN.gre(A[:, 1], Axy) < 5e-3


@pytest.mark.slow
def test_steady_poiseuille_second_order():
    # Grid convergence at fixed Re = 1, Wi = 1, beta = 0.1 against the
    # steady solution of the continuum model with the scheme's conformation
    # diffusion and zero conformation flux at the walls.  tau_h = 0.6
    # resolves the conformation boundary layer (sqrt(lam D) grows with L);
    # the global relative errors (Sec. 3.2) then fall at second order for
    # A_xy and A_xx, and close to it for u (the slope the paper reports).
    nu, beta, th = 0.5, 0.1, 0.6
    D = (th - 0.5) / 3
    errs = []
    for L in (16, 32, 64):
        U0 = nu / L
        lam = L / U0
        g = 8 * nu * U0 / L ** 2
        s = channel(L, beta * nu, (1 - beta) * nu, lam, g, tau_h=th)
        s.step(int(25 * max(L * L / nu, lam)))
        u, A = channel_profiles(s, L)
        y = np.arange(L) + 0.5
        ux, Axx, Axy, _ = AN.poiseuille_steady_zero_flux(
            y, L, g, beta * nu, (1 - beta) * nu, lam, D)
        errs.append((AN.gre(u[:, 0], ux), AN.gre(A[:, 1], Axy), AN.gre(A[:, 0] - 1, Axx - 1)))
        assert np.abs(A[:, 2] - 1).max() < 1e-9
    errs = np.array(errs)
    slopes = np.log2(errs[:-1] / errs[1:])
    assert (slopes[:, 1:] > 1.9).all(), (errs, slopes)
    assert (slopes[:, 0] > 1.5).all(), (errs, slopes)
    assert (errs[-1] < 1e-3).all(), errs


def test_startup_poiseuille_waters_king():
    # Transient centre-line velocity of the start-up problem (Sec. 3.2)
    # at Re = 1, Wi = 1 (El = 1) for beta = 0.1 and 0.5.
    L, nu, Wi, Re = 32, 0.5, 1.0, 1.0
    U0 = Re * nu / L
    lam = Wi * L / U0
    g = 8 * nu * U0 / L ** 2
    for beta in (0.1, 0.5):
        s = channel(L, beta * nu, (1 - beta) * nu, lam, g)
        for ts in (0.05, 0.2, 0.5, 1.0, 2.0):
            s.step(int(round(ts * L * L / nu)) - s.t)
            tstar = s.t * nu / L ** 2
            u, _ = channel_profiles(s, L)
            uc = 0.5 * (u[L // 2 - 1, 0] + u[L // 2, 0]) / U0
            # the nodes next to the centre sit at y = L/2 -+ 1/2
            ref = AN.waters_king(np.array([0.5 - 0.5 / L, 0.5 + 0.5 / L]), tstar, Wi / Re, beta).mean()
            assert abs(uc - ref) < 1.5e-2, (beta, tstar, uc, ref)


def test_womersley_newtonian():
    # Oscillating channel (Sec. 3.3), Newtonian, gamma = 3.070 as in the
    # paper's Re = 30 case; compared over one period after transients.
    L, nu_s, gam = 32, 1.0 / 6.0, 3.070
    omega = nu_s * (2 * gam / L) ** 2
    U = 0.01
    A = 8 * nu_s * U / L ** 2
    s = O.OracleSim(2, 1, L)
    s.set_params(3 * nu_s + 0.5, TAU_H, 1.0, 0.0)
    s.set_walls((0, 1, 0))
    s.set_force(O.FORCE_COS_T, (A, 0.0, 0.0), omega)
    s.init()
    period = 2 * np.pi / omega
    s.step(int(4 * period))
    y = np.arange(L) + 0.5
    for k in range(4):
        s.step(int(period / 4))
        u, _ = channel_profiles(s, L)
        ux, *_ = AN.womersley(y, L, s.t, A, omega, nu_s)
        assert np.abs(u[:, 0] - ux).max() < 1e-2 * np.abs(ux).max() + 2e-3 * U, k


def test_womersley_viscoelastic():
    # Oldroyd-B Womersley flow with the complex viscosity
    # nu* = nu_s + nu_p/(1 + i omega lam) (linear because A_yy = 1).
    L, nu_s, nu_p, lam = 32, 1.0 / 12.0, 1.0 / 12.0, 150.0
    omega = 2 * np.pi / 600.0
    U = 0.01
    A = 8 * (nu_s + nu_p) * U / L ** 2
    s = O.OracleSim(2, 1, L)
    s.set_params(3 * nu_s + 0.5, TAU_H, lam, nu_p)
    s.set_walls((0, 1, 0))
    s.set_force(O.FORCE_COS_T, (A, 0.0, 0.0), omega)
    s.init()
    s.step(6000)
    y = np.arange(L) + 0.5
    for k in range(3):
        s.step(200)
        u, Af = channel_profiles(s, L)
        ux, txy, axx, axy = AN.womersley(y, L, s.t, A, omega, nu_s, nu_p, lam)
        core = slice(3, L - 3)      # conformation boundary layer ~ sqrt(lam D)
        assert np.abs(u[:, 0] - ux).max() < 2e-2 * np.abs(ux).max(), k
        assert np.abs(Af[core, 1] - axy[core]).max() < 3e-2 * np.abs(axy).max(), k


@pytest.mark.slow
def test_four_roll_mill_low_wi():
    # Four-roll mill (Sec. 3.1) at Re = 1: as Wi -> 0 the local elongation
    # rate at the stagnation point tends to beta (the forcing uses nu_s),
    # and the stagnation conformation obeys A_xx = 1/(1 - 2 Wi_eff),
    # A_yy = 1/(1 + 2 Wi_eff), A_xy = 0.
    n, U0, Re, beta = 32, 0.01, 1.0, 0.5
    for Wi in (0.02, 0.2):
        p = O.lattice_params(Re, Wi, beta, U0, n / (2 * np.pi))
        k = 2 * np.pi / n
        s = O.OracleSim(2, n, n)
        s.set_params(p["tau_f"], TAU_H, p["lam"], p["eta_p"])
        amp = 2 * p["nu_s"] * U0 * k * k
        s.set_force(O.FORCE_FOUR_ROLL, (amp, -amp, 0.0))
        s.init()
        s.step(int(12 * max(1 / (2 * (p["nu_s"] + p["nu_p"]) * k * k), p["lam"])))
        m = s.moments()
        u = m["u"].reshape(n, n, 2)
        A = m["A"].reshape(n, n, 3)
        c = n // 2
        dudx = 0.5 * (u[c, c + 1, 0] - u[c, c - 1, 0])
        eps = dudx / (U0 * k)
        Wi_eff = p["lam"] * dudx
        Axx, Ayy, Axy = AN.four_roll_stagnation(Wi_eff)
        if Wi < 0.05:
            assert eps == pytest.approx(beta, rel=1e-2)
        assert A[c, c, 0] - 1 == pytest.approx(Axx - 1, rel=3e-2)
        assert A[c, c, 2] - 1 == pytest.approx(Ayy - 1, rel=3e-2)
        assert abs(A[c, c, 1]) < 1e-10


def test_warm_start_channel_profile_matches_the_analytic_solution():
    # the warm-start module's steady channel state (product side) against
    # the oracle's closed form of Sec. 3.2 (with the conformation scheme's
    # diffusion), written independently
    from paper_2506_13072_amd import warmstart as W
    ny, g, nu_s, nu_p, lam = 64, 3e-7, 0.2, 0.3, 4000.0
    D = (0.501 - 0.5) / 3
    u, tau = W.channel_steady(ny, g, nu_s, nu_p, lam, D)
    y = np.arange(ny) + 0.5
    ux, Axx, Axy, Ayy = AN.poiseuille_steady(y, ny, g, nu_s, nu_p, lam, D)
    k = nu_p / lam
    assert np.allclose(u, ux, rtol=1e-14, atol=0)
    assert np.allclose(tau[:, 0], k * (Axx - 1), rtol=1e-13, atol=0)
    assert np.allclose(tau[:, 1], k * Axy, rtol=1e-13, atol=1e-30)
    assert np.all(tau[:, 2] == 0) and np.all(Ayy == 1)
