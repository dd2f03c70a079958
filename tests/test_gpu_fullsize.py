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
