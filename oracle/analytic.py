"""Closed-form solutions the oracle is pinned against (FP64, numpy).

TEST INFRASTRUCTURE ONLY.  Every function states the passage of the paper it
comes from or the derivation it rests on.  Lattice units throughout:
dx = dt = 1, rho0 = 1; a node with index j across a channel of width
L = N_y sits at y = j + 1/2, with halfway bounce-back walls at y = 0 and
y = L.
"""
from __future__ import annotations

import numpy as np


# ------------------------------------------------------------- Poiseuille
def poiseuille_steady(y, L, g, nu_s, nu_p, lam, D=0.0):
    """Steady Oldroyd-B channel flow driven by a constant body force g
    (Sec. 3.2).

    u_x = g y (L - y) / (2 nu), nu = nu_s + nu_p;  A_xy = lam du/dy;
    A_yy = 1;  A_xx = 1 + 2 (lam du/dy)^2.  The printed A_xx carries a
    stray factor nu_p that makes it dimensionally inconsistent; the form
    used here is the steady state of the constitutive equation of Sec. 2.1
    for this shear flow.  The advection-diffusion scheme of Sec. 2.3 adds
    the diffusion D = cs^2 (tau_h - 1/2) to the conformation equation; the
    steady state of D A_xx'' + chi_xx = 0 then carries the constant
    4 D lam^3 (g / nu)^2, which is included (set D = 0 to drop it).
    Returns (u_x, A_xx, A_xy, A_yy) on the given y.
    """
    y = np.asarray(y, dtype=np.float64)
    nu = nu_s + nu_p
    ux = g * y * (L - y) / (2.0 * nu)
    gd = g * (L - 2.0 * y) / (2.0 * nu)
    Axy = lam * gd
    Axx = 1.0 + 2.0 * (lam * gd) ** 2 + 4.0 * D * lam ** 3 * (g / nu) ** 2
    Ayy = np.ones_like(y)
    return ux, Axx, Axy, Ayy


def poiseuille_steady_zero_flux(y, L, g, nu_s, nu_p, lam, D, nfine=20001):
    """Steady channel flow of the continuum model that the scheme
    approximates, with the conformation diffusion D of the advection-
    diffusion LB (Sec. 2.3) and zero conformation flux through the walls
    (the reading used for the wall treatment of the conformation
    populations).

    With D > 0 the shear component develops a boundary layer: from the
    integrated momentum balance nu_s u' + (nu_p/lam) A_xy = -g (y - L/2)
    and D A_xy'' - A_xy/lam + u' = 0 with A_xy' = 0 at y = 0, L,
        A_xy = -lam g (y - L/2)/nu + C sinh((y - L/2)/l),
        l = sqrt(D lam nu_s / nu),  C = lam g l / (nu cosh(L/(2 l))),
        u = -g ((y - L/2)^2 - L^2/4)/(2 nu)
            - (nu_p C l / (lam nu_s)) (cosh((y - L/2)/l) - cosh(L/(2 l))).
    A_xx then solves D A_xx'' - (A_xx - 1)/lam + 2 A_xy u' = 0 with zero
    flux at the walls; it is obtained by second-order finite differences on
    a fine grid (nfine points) and interpolated.  A_yy = 1.
    Returns (u_x, A_xx, A_xy, A_yy) on y.
    """
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    nu = nu_s + nu_p
    ell = np.sqrt(D * lam * nu_s / nu)
    Lh = L / 2.0
    C = lam * g * ell / (nu * np.cosh(Lh / ell))

    def fields(yy):
        yc = yy - Lh
        axy = -lam * g * yc / nu + C * np.sinh(yc / ell)
        ux = (-g * (yc ** 2 - Lh ** 2) / (2.0 * nu)
              - nu_p * C * ell / (lam * nu_s) * (np.cosh(yc / ell) - np.cosh(Lh / ell)))
        du = -g * yc / nu - nu_p * C / (lam * nu_s) * np.sinh(yc / ell)
        return ux, axy, du

    # A_xx on a cell-centred fine grid with zero-flux (mirror) ends
    h = L / nfine
    yf = (np.arange(nfine) + 0.5) * h
    _, axy_f, du_f = fields(yf)
    main = np.full(nfine, -2.0 * D / h ** 2 - 1.0 / lam)
    main[0] += D / h ** 2
    main[-1] += D / h ** 2
    off = np.full(nfine - 1, D / h ** 2)
    M = sp.diags([off, main, off], [-1, 0, 1], format="csc")
    rhs = -1.0 / lam - 2.0 * axy_f * du_f
    axx_f = spl.spsolve(M, rhs)
    y = np.asarray(y, dtype=np.float64)
    ux, axy, _ = fields(y)
    axx = np.interp(y, yf, axx_f)
    return ux, axx, axy, np.ones_like(y)


def waters_king(ystar, tstar, El, beta, nterms=200):
    """Start-up of Oldroyd-B channel flow from rest (Sec. 3.2, transient
    series).  ystar = y/L, tstar = t (nu_s + nu_p)/L^2, El = Wi/Re; returns
    u/U0 with U0 the steady centre-line velocity.

    Readings: the second exponential of G_N is taken at t* (the printed t is
    a typo); when beta_N^2 < 0 the oscillating branch uses
    beta_N = sqrt(-beta_N^2).  Both branches satisfy G_N(0) = 1 and
    G_N'(0) = -N^2, which is what the mode equation
    El G'' + alpha_N G' + N^2 G = 0 with zero initial stress requires.
    """
    ystar = np.asarray(ystar, dtype=np.float64)
    u = 4.0 * ystar * (1.0 - ystar)
    for n in range(1, nterms + 1):
        N = (2 * n - 1) * np.pi
        S = 1.0 - (2.0 - beta) * N * N * El
        alpha = 1.0 + beta * El * N * N
        b2 = alpha * alpha - 4.0 * N * N * El
        a_s = alpha / (2.0 * El)
        if b2 >= 0.0:
            bN = np.sqrt(b2)
            b_s = bN / (2.0 * El)
            aN, bbN = 1.0 + S / bN, 1.0 - S / bN
            G = 0.5 * (aN * np.exp((-a_s + b_s) * tstar)
                       + bbN * np.exp((-a_s - b_s) * tstar))
        else:
            bN = np.sqrt(-b2)
            b_s = bN / (2.0 * El)
            G = np.exp(-a_s * tstar) * (np.cos(b_s * tstar)
                                        + S / bN * np.sin(b_s * tstar))
        u = u - 32.0 * np.sin(N * ystar) / N ** 3 * G
    return u


# -------------------------------------------------------------- Womersley
def womersley(y, L, t, A, omega, nu_s, nu_p=0.0, lam=1.0):
    """Periodic state of a channel driven by g_x = A cos(omega t) (Sec. 3.3).

    The printed solution is Newtonian with the Womersley number
    gamma = (L/2) sqrt(omega / nu_s) and y measured from the channel
    centre.  For the Oldroyd-B fluid the shear stress obeys the linear
    equation lam d(tau_xy)/dt + tau_xy = eta_p du/dy (A_yy stays 1), so the
    same formula holds with the complex viscosity
    nu* = nu_s + nu_p / (1 + i omega lam).  Returns
    (u_x, tau_xy, A_xx - 1, A_xy) at time t for y in lattice units from the
    lower wall.  The conformation terms assume nu_p > 0.
    """
    y = np.asarray(y, dtype=np.float64)
    yc = y - L / 2.0
    nus = nu_s + (nu_p / (1.0 + 1j * omega * lam) if nu_p > 0 else 0.0)
    k = np.sqrt(1j * omega / nus)
    U = A / (1j * omega) * (1.0 - np.cosh(k * yc) / np.cosh(k * L / 2.0))
    dU = -A / (1j * omega) * k * np.sinh(k * yc) / np.cosh(k * L / 2.0)
    e = np.exp(1j * omega * t)
    ux = np.real(U * e)
    if nu_p <= 0.0:
        z = np.zeros_like(y)
        return ux, z, z, z
    T = nu_p / (1.0 + 1j * omega * lam) * dU          # tau_xy amplitude
    B = lam / nu_p * T                                  # A_xy amplitude
    # lam dA_xx/dt + (A_xx - 1) = 2 lam (du/dy) A_xy: product of two
    # harmonics = mean + second harmonic.
    mean = 2.0 * lam * 0.5 * np.real(dU * np.conj(B))
    sec = 2.0 * lam * 0.5 * (dU * B) / (1.0 + 2j * omega * lam)
    axx = mean + np.real(sec * e * e)
    return ux, np.real(T * e), axx, np.real(B * e)


# --------------------------------------------------------- Taylor-Green
def tg_linear_viscoelastic(t, a0, s0, kappa, nu_s, nu_p, lam, D):
    """Amplitudes of a single Taylor-Green mode in the linear (small U0)
    regime of the coupled system: the mode amplitude a and the stress
    amplitude s obey
        a' = -kappa (nu_s a + s),
        s' = -(1/lam + kappa D) s + (nu_p / lam) a,
    with kappa = |k|^2 of the mode (2 k^2 in 2D, 3 k^2 for the 3D vortex).
    This follows from the momentum equation of Sec. 2.1 with
    tau_p = s * (strain rate per unit amplitude) and the linearised
    constitutive equation (A close to I) plus the diffusion of the
    conformation scheme.  Returns (a(t), s(t)) by the exact 2x2 matrix
    exponential."""
    M = np.array([[-kappa * nu_s, -kappa],
                  [nu_p / lam, -(1.0 / lam + kappa * D)]], dtype=np.complex128)
    w, V = np.linalg.eig(M)
    c = np.linalg.solve(V, np.array([a0, s0], dtype=np.complex128))
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    out = (V[:, None, :] * (c[None, :] * np.exp(np.outer(t, w)))[None, :, :]).sum(-1)
    return np.real(out[0]), np.real(out[1])


def tg2d_fields(nx, ny, U0):
    """2D Taylor-Green velocity and pressure on an nx*ny periodic grid:
    u = U0 (sin kx cos ky, -cos kx sin ky), p = (U0^2/4)(cos 2kx + cos 2ky)
    (the pressure that balances u.grad u for this field), k = 2 pi / n.  Returns u[N,2], p[N] node-major, x fastest."""
    x = 2.0 * np.pi * np.arange(nx) / nx
    y = 2.0 * np.pi * np.arange(ny) / ny
    X, Y = np.meshgrid(x, y)
    u = np.stack([U0 * np.sin(X) * np.cos(Y), -U0 * np.cos(X) * np.sin(Y)], -1)
    p = (U0 ** 2 / 4.0) * (np.cos(2 * X) + np.cos(2 * Y))
    return u.reshape(-1, 2), p.reshape(-1)


# --------------------------------------------------------- four-roll mill
def four_roll_stagnation(Wi_eff):
    """Steady conformation at the stagnation point of the four-roll mill
    (Sec. 3.1): A_xx = 1/(1 - 2 Wi_eff), A_yy = 1/(1 + 2 Wi_eff), A_xy = 0,
    where Wi_eff = lam * du_x/dx at the stagnation point."""
    return 1.0 / (1.0 - 2.0 * Wi_eff), 1.0 / (1.0 + 2.0 * Wi_eff), 0.0


# ------------------------------------------------------------ error norms
def gre(num, ana):
    """Global relative error of Sec. 3.2: sum |num - ana| / sum |ana|, with
    |.| the Euclidean norm of a vector field (rows) or the absolute value
    of a scalar field."""
    num = np.asarray(num, dtype=np.float64)
    ana = np.asarray(ana, dtype=np.float64)
    if num.ndim == 1:
        return np.abs(num - ana).sum() / np.abs(ana).sum()
    return (np.linalg.norm(num - ana, axis=-1).sum()
            / np.linalg.norm(ana, axis=-1).sum())


def rel_l2(a, b):
    """||a - b||_2 / ||b||_2 over all entries."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
