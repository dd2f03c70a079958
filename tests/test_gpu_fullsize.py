"""Parity at the full benchmark sizes, in the launch configuration the
benchmark times (FP32 storage, the default tile shape, steps replayed from
captured graphs), on sampled outputs: the state of boxes of nodes is read
from the GPU, one oracle step advances each box, and the box interior (at
least 3 nodes from a cut edge; a node's update depends on neighbours at
distance 2) must agree with the GPU's next step.  Channel boxes span the
full height, so both walls are exact; the 3D boxes wrap periodically.
Bar: FP32 storage, relative L2 <= 1e-5 per field; the channel also in place
(one population buffer, the box read at an odd time level), and the 3D
state also with anchored FP16 storage (bar 1e-3)."""
import numpy as np
import pytest

from oracle import analytic as AN
from oracle import oracle as O
from paper_2506_13072_amd import workloads as WL

pytestmark = pytest.mark.gpu

MARGIN = 3


@pytest.fixture(scope="module")
def V():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_13072_amd import vflb
    vflb.lib()
    return vflb


def box_state(V, g, lo, size):
    return dict(f=g.read_box(V.FIELD_F, lo, size), h=g.read_box(V.FIELD_H, lo, size),
                chi_prev=g.read_box(V.FIELD_CHI_PREV, lo, size),
                u_prev=g.read_box(V.FIELD_U_PREV, lo, size))


def interior(a, size, d):
    shape = tuple(size[::-1][-d:]) if d == 3 else (size[1], size[0])
    a = a.reshape(shape + a.shape[1:])
    if d == 2:  # periodic in x only: trim x
        return a[:, MARGIN:-MARGIN].reshape((-1,) + a.shape[2:])
    return a[MARGIN:-MARGIN, MARGIN:-MARGIN, MARGIN:-MARGIN].reshape((-1,) + a.shape[3:])


def compare(V, g, o, lo, size, d, tol=1e-5):
    after = box_state(V, g, lo, size)
    ref = o.get_state()
    out = {}
    for k in ("f", "h", "chi_prev", "u_prev"):
        out[k] = AN.rel_l2(interior(after[k], size, d), interior(ref[k], size, d))
    assert all(v <= tol for v in out.values()), out
    return out


@pytest.mark.parametrize("inplace", [False, True])
def test_channel_8192x1024_sampled_parity(V, inplace):
    w = WL.CHANNEL_8192x1024
    ny, nx = w["shape"]
    g = V.Sim(2, nx, ny, 1, "f32", inplace=inplace)
    g.set_params(w["Re"], w["Wi"], w["beta"], w["U0"], w["L"])
    g.set_boundaries((V.PERIODIC, V.WALLS))
    lp = g.lattice_params()
    force = 8 * (lp["nu_s"] + lp["nu_p"]) * w["U0"] / w["L"] ** 2
    g.set_force(V.FORCE_CONST, (force, 0.0, 0.0))
    u, tau, p = WL.smooth_fields(2, (ny, nx), 11, amp_u=w["U0"], amp_tau=1e-2 * lp["eta_p"],
                                 amp_p=w["U0"] ** 2)
    g.init_fields(u, tau, p)
    g.step(131)  # single launches and two 64-step graphs, tile 64 x 16
    t = g.t
    p_or = O.lattice_params(w["Re"], w["Wi"], w["beta"], w["U0"], w["L"])
    size = (40, ny)
    los = [(x0 - MARGIN, 0) for x0 in (0, 3000, nx - 20)]  # one box across the seam
    befores = [box_state(V, g, lo, size) for lo in los]
    g.step(1)
    for lo, before in zip(los, befores):
        o = O.OracleSim(2, size[0], size[1])
        o.set_params(p_or["tau_f"], 0.501, p_or["lam"], p_or["eta_p"])
        o.set_walls((0, 1, 0))
        o.set_force(O.FORCE_CONST, (force, 0.0, 0.0))
        o.set_state(**before, t=t)
        o.step(1)
        compare(V, g, o, lo, size, 2)


@pytest.mark.parametrize("storage,tol", [("f32", 1e-5), ("f16s", 1e-3)])
def test_tgv_512_sampled_parity(V, storage, tol):
    w = WL.TGV_512
    n = w["shape"][0]
    g = V.Sim(3, n, n, n, storage)
    g.set_params(w["Re"], w["Wi"], w["beta"], w["U0"], w["L"])
    u, p = WL.taylor_green_3d_device(n, w["U0"])
    g.init_fields_device(u, None, p)
    del u, p
    g.step(9)
    t = g.t
    p_or = O.lattice_params(w["Re"], w["Wi"], w["beta"], w["U0"], w["L"])
    boxes = [(200, 17, 300), (n - 8, n - 11, 5)]  # the second wraps on all axes
    size = (22, 22, 22)
    befores = [box_state(V, g, lo, size) for lo in boxes]
    g.step(1)
    for lo, before in zip(boxes, befores):
        o = O.OracleSim(3, *size)
        o.set_params(p_or["tau_f"], 0.501, p_or["lam"], p_or["eta_p"])
        o.set_state(**before, t=t)
        o.step(1)
        compare(V, g, o, lo, size, 3, tol)


def test_channel_8192x1024_holds_the_analytic_poiseuille_state(V):
    # Started from the analytic steady Oldroyd-B channel state (parabolic
    # u, A from the constitutive equation with the conformation scheme's
    # diffusion and zero flux through the walls), the full-size channel in
    # the benchmark's configuration must stay there: after 2000 steps the
    # velocity and conformation keep to the analytic profiles.
    w = WL.CHANNEL_8192x1024
    ny, nx = w["shape"]
    Wi = 0.1
    g = V.Sim(2, nx, ny, 1, "f32")
    g.set_params(w["Re"], Wi, w["beta"], w["U0"], w["L"])
    g.set_boundaries((V.PERIODIC, V.WALLS))
    lp = g.lattice_params()
    nu_s, nu_p, lam = lp["nu_s"], lp["nu_p"], lp["lam"]
    force = 8 * (nu_s + nu_p) * w["U0"] / w["L"] ** 2
    g.set_force(V.FORCE_CONST, (force, 0.0, 0.0))
    y = np.arange(ny) + 0.5
    D = (0.501 - 0.5) / 3.0
    ux, Axx, Axy, _ = AN.poiseuille_steady_zero_flux(y, ny, force, nu_s, nu_p, lam, D)
    k = lp["eta_p"] / lam
    u = np.zeros((ny, nx, 2))
    u[:, :, 0] = ux[:, None]
    tau = np.zeros((ny, nx, 3))
    tau[:, :, 0] = (k * (Axx - 1))[:, None]
    tau[:, :, 1] = (k * Axy)[:, None]
    g.init_fields(u.reshape(-1, 2), tau.reshape(-1, 3), None)
    g.step(2000)
    m = g.moments()
    uu = m["u"].reshape(ny, nx, 2)
    A = m["A"].reshape(ny, nx, 3)
    U0 = w["U0"]
    du = np.abs(uu[:, :, 0] - ux[:, None]).max() / U0
    dv = np.abs(uu[:, :, 1]).max() / U0
    dxx = np.abs(A[:, :, 0] - Axx[:, None]).max() / np.abs(Axx - 1).max()
    dxy = np.abs(A[:, :, 1] - Axy[:, None]).max() / np.abs(Axy).max()
    print("drift after 2000 steps: u %.2e v %.2e A_xx %.2e A_xy %.2e" % (du, dv, dxx, dxy))
    # measured: u 1.3e-4, v 7e-6, A_xx and A_xy 1.7e-4 (the equilibrium-only
    # start lacks the non-equilibrium parts of the populations)
    assert du < 5e-4 and dv < 1e-4 and dxx < 1e-3 and dxy < 1e-3, (du, dv, dxx, dxy)


def test_tgv_64_kinetic_energy_decay_and_conservation(V):
    # The 3D Taylor-Green vortex with the benchmark's parameters on a 64^3
    # copy: the GPU's FP64 reductions of the kinetic energy follow the FP64
    # oracle's as the vortex decays, for FP32 and anchored FP16 storage,
    # and mass and momentum stay at their initial values.
    import math
    w = WL.TGV_512
    n = 64
    L = n / (2 * math.pi)
    p_or = O.lattice_params(w["Re"], w["Wi"], w["beta"], w["U0"], L)
    u = WL.taylor_green_3d_velocity(n, w["U0"])
    x = 2 * np.pi * np.arange(n) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    p = ((w["U0"] ** 2 / 16) * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2)).ravel()
    o = O.OracleSim(3, n, n, n)
    o.set_params(p_or["tau_f"], 0.501, p_or["lam"], p_or["eta_p"])
    o.init(u, None, p)
    sims = {}
    for storage in ("f32", "f16s"):
        g = V.Sim(3, n, n, n, storage)
        g.set_params(w["Re"], w["Wi"], w["beta"], w["U0"], L)
        g.init_fields(u, None, p)
        sims[storage] = g
    C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1],
                  [0, 0, -1], [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1],
                  [-1, 0, -1], [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1],
                  [0, -1, 1]], float)
    ke0 = None
    for k in range(4):
        o.step(10)
        ke_o = 0.5 * float((o.moments()["u"] ** 2).sum()) / n ** 3  # per node, as reported
        f = o.get_state()["f"]
        m_o, p_o = float(f.sum()), f.sum(0) @ C  # totals, as reported
        ke0 = ke0 or ke_o
        for storage, g in sims.items():
            g.step(10)
            r = g.reduce()
            # measured: KE 4.5e-8 (FP32) / 4.2e-7 (FP16) relative; mass and
            # momentum totals over 262 144 nodes within 5e-6 / 6.3e-4
            tol, ctol = (1e-6, 2e-5) if storage == "f32" else (1e-5, 2e-3)
            dm, dp = abs(r["M"] - m_o), np.abs(np.array(r["P"]) - p_o).max()
            print(storage, k, "KE rel %.2e  dM %.2e  dP %.2e" % (r["KE"] / ke_o - 1, dm, dp))
            assert abs(r["KE"] / ke_o - 1) < tol, (storage, k, r["KE"], ke_o)
            assert dm < ctol and dp < ctol, (storage, k, r["M"], m_o, r["P"], p_o)
    assert ke_o < ke0  # the vortex decays


TGV64_STEPS = 40


@pytest.fixture(scope="module")
def tgv_64_copy():
    """The 512^3 Taylor-Green workload's lattice-unit parameters (tau_f,
    lambda, eta_p of Re = 100, Wi = 0.5, beta = 0.9, U0 = 0.02,
    L = 512/(2 pi)) on a 64^3 lattice holding the theta = 0 vortex and its
    pressure; TGV64_STEPS steps of the FP64 oracle."""
    w = WL.TGV_512
    n = 64
    p_or = O.lattice_params(w["Re"], w["Wi"], w["beta"], w["U0"], w["L"])
    u = WL.taylor_green_3d_velocity(n, w["U0"])
    x = 2 * np.pi * np.arange(n) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    p = ((w["U0"] ** 2 / 16) * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2)).ravel()
    o = O.OracleSim(3, n, n, n)
    o.set_params(p_or["tau_f"], 0.501, p_or["lam"], p_or["eta_p"])
    o.init(u, None, p)
    o.step(TGV64_STEPS)
    mo = o.moments()
    mo["Ae"] = mo["A"] - np.array([1, 1, 1, 0, 0, 0], float)
    f = o.get_state()["f"]
    # the pressure is summed from populations of the size of U0, while it is
    # of the size of U0^2: its bar is the storage bar times that ratio
    ratio = max(1.0, np.sqrt((np.abs(f[:, 1:]).sum(1) ** 2).mean()) /
                np.sqrt((mo["p"] ** 2).mean()))
    return dict(u=u, p=p, mo=mo, ratio=ratio, n=n, w=w)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("storage,tol", [("f32", 1e-5), ("f16s", 1e-3)])
def test_tgv_64_copy_per_field_parity(V, tgv_64_copy, storage, tol):
    # per field u, p, tau, A - I against the oracle after TGV64_STEPS steps
    # (relative L2, and the element-wise max over max for u, tau, A - I)
    c = tgv_64_copy
    n, w = c["n"], c["w"]
    g = V.Sim(3, n, n, n, storage)
    g.set_params(w["Re"], w["Wi"], w["beta"], w["U0"], w["L"])
    g.init_fields(c["u"], None, c["p"])
    g.step(TGV64_STEPS)
    mg = g.moments()
    mg["Ae"] = mg["A"] - np.array([1, 1, 1, 0, 0, 0], float)
    out = {}
    for k in ("u", "tau", "Ae", "p"):
        bar = tol * (c["ratio"] if k == "p" else 1.0)
        out[k] = AN.rel_l2(mg[k], c["mo"][k])
        em = np.abs(mg[k] - c["mo"][k]).max() / np.abs(c["mo"][k]).max()
        print(storage, k, "rel L2 %.2e  max %.2e  bar %.1e" % (out[k], em, bar))
        assert out[k] <= bar, (storage, k, out[k], bar)
        if k != "p":
            # a single node may carry a few times the mean rounding error
            assert em <= 10 * bar, (storage, k, em, bar)


def test_channel_8192x1024_follows_the_analytic_womersley_state(V):
    # Oldroyd-B Womersley flow (Sec. 3.3; complex viscosity) at Womersley
    # number 10: started from the analytic periodic state, the full-size
    # channel follows it through one period of the cos(omega t) force.
    import math
    w = WL.CHANNEL_8192x1024
    ny, nx = w["shape"]
    Wi, gam = 0.1, 10.0
    g = V.Sim(2, nx, ny, 1, "f32")
    g.set_params(w["Re"], Wi, w["beta"], w["U0"], w["L"])
    g.set_boundaries((V.PERIODIC, V.WALLS))
    lp = g.lattice_params()
    nu_s, nu_p, lam = lp["nu_s"], lp["nu_p"], lp["lam"]
    omega = nu_s * (2 * gam / ny) ** 2
    amp = 8 * (nu_s + nu_p) * w["U0"] / w["L"] ** 2
    g.set_force(V.FORCE_COS_T, (amp, 0.0, 0.0), omega)
    y = np.arange(ny) + 0.5
    ux, txy, axx, axy = AN.womersley(y, ny, 0.0, amp, omega, nu_s, nu_p, lam)
    k = lp["eta_p"] / lam
    u = np.zeros((ny, nx, 2))
    u[:, :, 0] = ux[:, None]
    tau = np.zeros((ny, nx, 3))
    tau[:, :, 0] = (k * axx)[:, None]
    tau[:, :, 1] = txy[:, None]
    g.init_fields(u.reshape(-1, 2), tau.reshape(-1, 3), None)
    steps = int(round(2 * math.pi / omega))
    g.step(steps)
    ux1, _, _, axy1 = AN.womersley(y, ny, float(g.t), amp, omega, nu_s, nu_p, lam)
    m = g.moments()
    uu = m["u"].reshape(ny, nx, 2)
    A = m["A"].reshape(ny, nx, 3)
    core = slice(8, ny - 8)  # the conformation boundary layer, sqrt(lam D) ~ 2 nodes
    du = np.abs(uu[:, :, 0] - ux1[:, None]).max() / np.abs(ux).max()
    dxy = np.abs(A[core, :, 1] - axy1[core, None]).max() / np.abs(axy).max()
    print("after one period (%d steps): u %.2e  A_xy %.2e" % (steps, du, dxy))
    assert du < 2e-3 and dxy < 3e-3, (du, dxy)  # measured 5.8e-4, 7.5e-4
