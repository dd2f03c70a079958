"""Pins of the FP64 oracle's per-node building blocks.

Each test checks the oracle against something other than itself: a
library pseudo-inverse, the moment identities that the paper's
Chapman-Enskog analysis requires (Sec. 2.2) or that the conformation scheme
implies (Sec. 2.3), hand-derived special cases, and hand-computed numbers.
"""
import numpy as np
import pytest

from oracle import oracle as O

C2 = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1],
               [1, 1], [-1, 1], [-1, -1], [1, -1]], dtype=float)
C3 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0],
               [0, 0, 1], [0, 0, -1], [1, 1, 0], [-1, -1, 0], [1, -1, 0],
               [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
               [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=float)
CS2 = 1.0 / 3.0


def vel(d):
    return C2 if d == 2 else C3


def weights(d):
    # recovered from the isotropy conditions, not typed in: the weight of
    # each speed shell solves sum w = 1, sum w c_x^2 = cs2,
    # sum w c_x^2 c_y^2 = cs2^2
    c = vel(d)
    shells = sorted(set((c * c).sum(1).astype(int)))
    rows, rhs = [], [1.0, CS2, CS2 * CS2]
    for f in (lambda v: np.ones(len(v)), lambda v: v[:, 0] ** 2,
              lambda v: v[:, 0] ** 2 * v[:, 1] ** 2):
        rows.append([f(c[(c * c).sum(1) == s]).sum() for s in shells])
    ws = np.linalg.solve(np.array(rows), np.array(rhs))
    return np.array([ws[shells.index(int(s))] for s in (c * c).sum(1)])


def sym_full(d, s):
    T = np.zeros((d, d))
    comps = [(0, 0), (0, 1), (1, 1)] if d == 2 else \
        [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for k, (a, b) in enumerate(comps):
        T[a, b] = T[b, a] = s[k]
    return T


def constraint_matrix(d):
    """Rows of the linear system for f^B in the order of the paper's
    right-hand side (App. A): in 2D the second moments (yx, xx, xy, yy),
    then the zeroth and the first moments; in 3D the second moments
    (xx, yy, zz, xy, xz, yx, yz, zx, zy), then the first moments and last
    the zeroth (the order of the printed 19x13 matrix's columns)."""
    c = vel(d)
    if d == 2:
        pairs = [(1, 0), (0, 0), (0, 1), (1, 1)]
    else:
        pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 0), (1, 2),
                 (2, 0), (2, 1)]
    rows = [c[:, a] * c[:, b] for a, b in pairs]
    if d == 2:
        rows.append(np.ones(len(c)))
        rows += [c[:, a] for a in range(d)]
    else:
        rows += [c[:, a] for a in range(d)]
        rows.append(np.ones(len(c)))
    return np.array(rows)


def test_weights_recovered_match_paper_d2q9():
    assert np.allclose(weights(2), [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, atol=1e-15)


@pytest.mark.parametrize("d", [2, 3])
def test_oracle_weights_are_isotropic(d):
    # h^eq(A = 1, u = 0) = w_i: the oracle's weights equal the isotropic set
    # (for D3Q19 the paper prints no weights)
    assert np.allclose(O.heq(d, 1.0, np.zeros(d)), weights(d), atol=1e-16)


@pytest.mark.parametrize("d", [2, 3])
def test_printed_pseudo_inverse_is_moore_penrose(d):
    C = constraint_matrix(d)
    P = np.linalg.pinv(C)           # SVD-based library routine
    M = O.pinv_matrix(d)
    if d == 2:
        # printed as -1/(72 tau_f) * M applied to the four stress entries:
        # i.e. the first four columns of pinv(C) are M/72.
        assert np.allclose(P[:, :4], M / 72.0, atol=1e-14)
    else:
        assert np.allclose(P, M, atol=1e-14)


@pytest.mark.parametrize("d", [2, 3])
def test_fB_solves_constraints_by_minimum_norm(d):
    rng = np.random.default_rng(11 + d)
    c = vel(d)
    for _ in range(20):
        tau_f = rng.uniform(0.51, 3.0)
        nc = 3 if d == 2 else 6
        tau = rng.normal(size=nc)
        fb = O.fB(d, tau_f, tau)
        T = sym_full(d, tau)
        # the three constraints of the Chapman-Enskog analysis
        assert abs(fb.sum()) < 1e-14
        assert np.allclose(c.T @ fb, 0.0, atol=1e-14)
        assert np.allclose(np.einsum("i,ia,ib->ab", fb, c, c), -T / tau_f, atol=1e-14)
        # minimum-norm solution: orthogonal to the null space of C
        C = constraint_matrix(d)
        b = np.concatenate([
            [-T[a, b] / tau_f for a, b in (
                [(1, 0), (0, 0), (0, 1), (1, 1)] if d == 2 else
                [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)])],
            np.zeros(1 + d)])
        ref, *_ = np.linalg.lstsq(C, b, rcond=None)
        assert np.allclose(fb, ref, atol=1e-13)


@pytest.mark.parametrize("d", [2, 3])
def test_equilibrium_moments(d):
    rng = np.random.default_rng(3 + d)
    c = vel(d)
    for _ in range(20):
        u = rng.normal(scale=0.05, size=d)
        p = rng.normal(scale=0.01)
        fe = O.feq(d, p, u)
        assert abs(fe.sum()) < 1e-15
        assert np.allclose(c.T @ fe, u, atol=1e-15)
        assert np.allclose(np.einsum("i,ia,ib->ab", fe, c, c),
                           np.outer(u, u) + p * np.eye(d), atol=1e-15)
        third = np.einsum("i,ia,ib,ig->abg", fe, c, c, c)
        I = np.eye(d)
        ref = CS2 * (np.einsum("ab,g->abg", I, u) + np.einsum("ag,b->abg", I, u)
                     + np.einsum("bg,a->abg", I, u))
        assert np.allclose(third, ref, atol=1e-15)


@pytest.mark.parametrize("d", [2, 3])
def test_guo_force_moments(d):
    rng = np.random.default_rng(5 + d)
    c = vel(d)
    for _ in range(20):
        tf = rng.uniform(0.51, 2.0)
        u = rng.normal(scale=0.05, size=d)
        F = rng.normal(scale=1e-4, size=d)
        Fi = O.guo(d, tf, F, u)
        k = 1.0 - 0.5 / tf
        assert abs(Fi.sum()) < 1e-18
        assert np.allclose(c.T @ Fi, k * F, atol=1e-18)
        assert np.allclose(np.einsum("i,ia,ib->ab", Fi, c, c),
                           k * (np.outer(F, u) + np.outer(u, F)), atol=1e-18)


@pytest.mark.parametrize("d", [2, 3])
def test_velocity_and_pressure_recover_equilibrium(d):
    rng = np.random.default_rng(7 + d)
    for _ in range(20):
        u = rng.normal(scale=0.05, size=d)
        p = rng.normal(scale=0.01)
        fe = O.feq(d, p, u)
        zero = np.zeros(d)
        assert np.allclose(O.velocity(d, fe, zero), u, atol=1e-16)
        # with no force and no fluctuation the pressure formula inverts f^eq
        assert abs(O.pressure(d, 0.8, fe, u, 0.0, 0.0) - p) < 1e-16
        # the force enters u with weight 1/2
        F = rng.normal(scale=1e-3, size=d)
        assert np.allclose(O.velocity(d, fe, F), u + 0.5 * F, atol=1e-16)


@pytest.mark.parametrize("d", [2, 3])
def test_pressure_prefactor(d):
    # cs2 / (1 - w0): 3/5 for D2Q9, 1/2 for D3Q19
    q = 9 if d == 2 else 19
    f = np.zeros(q)
    f[1] = 1.0
    assert O.pressure(d, 0.7, f, np.zeros(d), 0.0, 0.0) == pytest.approx(
        0.6 if d == 2 else 0.5, abs=1e-15)
    # tau_f F_0 and tau_f f_0^B enter with the same prefactor
    assert O.pressure(d, 0.7, np.zeros(q), np.zeros(d), 1.0, 0.0) == pytest.approx(
        0.7 * (0.6 if d == 2 else 0.5), abs=1e-15)
    assert O.pressure(d, 0.7, np.zeros(q), np.zeros(d), 0.0, 1.0) == pytest.approx(
        0.7 * (0.6 if d == 2 else 0.5), abs=1e-15)


@pytest.mark.parametrize("d", [2, 3])
def test_conformation_equilibrium_and_source_moments(d):
    rng = np.random.default_rng(9 + d)
    c = vel(d)
    for _ in range(20):
        u = rng.normal(scale=0.05, size=d)
        A = rng.uniform(0.5, 2.0)
        th = rng.uniform(0.501, 1.5)
        he = O.heq(d, A, u)
        assert abs(he.sum() - A) < 1e-15
        assert np.allclose(c.T @ he, A * u, atol=1e-15)
        chi = rng.normal()
        ci = O.chi_i(d, th, chi, u)
        assert abs(ci.sum() - chi) < 1e-15
        assert np.allclose(c.T @ ci, (1 - 0.5 / th) * chi * u, atol=1e-15)


def test_chi_simple_shear_2d():
    # u = (g y, 0): d_y u_x = g, all other gradients zero.  The upper-
    # convected source of the Oldroyd-B equation then is
    # chi_xx = 2 g A_xy - (A_xx-1)/lam, chi_xy = g A_yy - A_xy/lam,
    # chi_yy = -(A_yy-1)/lam.
    g, lam = 0.37, 2.5
    A = np.array([1.3, 0.2, 0.9])           # xx, xy, yy
    G = np.array([[0.0, 0.0], [g, 0.0]])     # G[a,b] = d_a u_b
    chi = O.chi_tensor(2, lam, A, G.ravel())
    assert np.allclose(chi, [2 * g * 0.2 - 0.3 / lam, g * 0.9 - 0.2 / lam,
                             0.1 / lam], atol=1e-15)


def test_chi_extension_3d():
    # uniaxial extension u = (2e x, -e y, -e z) with diagonal A
    e, lam = 0.11, 3.0
    A = np.array([1.5, 0.8, 0.7, 0.0, 0.0, 0.0])
    G = np.diag([2 * e, -e, -e])
    chi = O.chi_tensor(3, lam, A, G.ravel())
    ref = [-(0.5) / lam + 2 * 2 * e * 1.5, 0.2 / lam - 2 * e * 0.8,
           0.3 / lam - 2 * e * 0.7, 0.0, 0.0, 0.0]
    assert np.allclose(chi, ref, atol=1e-15)


@pytest.mark.parametrize("d", [2, 3])
def test_chi_rotation_is_objective(d):
    # For A = I and a rigid rotation (antisymmetric gradient) the
    # upper-convected source vanishes.
    rng = np.random.default_rng(21)
    W = rng.normal(size=(d, d))
    W = W - W.T
    I = [1, 0, 1] if d == 2 else [1, 1, 1, 0, 0, 0]
    assert np.allclose(O.chi_tensor(d, 4.0, np.array(I, float), W.ravel()), 0.0,
                       atol=1e-15)


def test_polymer_stress_and_params_c0():
    # 64^2 four-roll mill at Re = 1, Wi = 1, beta = 0.5, U0 = 0.01,
    # L = 64/(2 pi): nu = U0 L / Re = 0.101859..., split evenly.
    p = O.lattice_params(1.0, 1.0, 0.5, 0.01, 64 / (2 * np.pi))
    assert p["nu_s"] == pytest.approx(0.0509295817894065, rel=1e-14)
    assert p["tau_f"] == pytest.approx(3 * 0.0509295817894065 + 0.5, rel=1e-14)
    assert p["lam"] == pytest.approx(1018.5916357881302, rel=1e-14)
    tau = O.polymer_stress(2, 0.05, 100.0, np.array([1.2, 0.1, 0.9]))
    assert np.allclose(tau, [0.05 / 100 * 0.2, 0.05 / 100 * 0.1, -0.05 / 100 * 0.1])
