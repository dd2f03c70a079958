"""Learned warm start for steady four-roll-mill and channel states
(orchestration only).

Every computation runs in libvflb: batches of lattices run to their steady
states (vflb_batch_run_until), the network trains on those states on the
device (vflb_mlp_train: minibatch draws, standardised targets, Adam), and a
new lattice starts from the network's prediction (vflb_init_from_mlp)
instead of from rest.  This module only decides what to call.

Two geometries (one network each): the simplified four-roll mill
(Sec. 3.1; periodic n x n, force of amplitude 2 nu_s U0 k^2) and the planar
Poiseuille channel (Sec. 3.2; walls in y, constant force 8 nu U0 / L^2,
L = ny).  The channel flow does not depend on x, so channels of 4 x ny
nodes hold the state of any longer channel of the same height.

Inputs of the network per node: (x/nx, y/ny, w, b, r) with
w = P (ln Wi - ln 0.1)/ln 50, b = P (beta - 0.1)/0.8, r = P ln Re: the
parameter coordinates span [0, P] with P = 1/4, so that the Gaussian
frequencies vary the features four times more slowly along the parameters
than across the lattice.  Outputs: (u/U0, v/U0, txx/S, txy/S, tyy/S) with
the stress scale S = eta_p U0 k, k = 2 pi / n (viscous stress of the
forcing mode) for the four-roll mill and S = eta_p 4 U0 / L (wall shear
stress) for the channel.

Fallback.  A warm run is judged without running the cold one: the training
runs (from rest) give, for their parameters, the residual after K0 steps
and the steps to the tolerance.  A held-out lattice takes both from its
nearest training runs in (ln Wi, beta).  The warm run is abandoned for a
cold start when its state is non-finite, when its residual after K0 steps
exceeds the predicted cold residual, or when, after a further window of
checks, the decay rate of its residual projects more steps to the
tolerance than the predicted cold run needs.  Its steps so far are then
counted on top of the cold run's.
"""
from __future__ import annotations

import math
import time

import numpy as np

WI_LO, WI_HI = 0.1, 5.0
BETA_LO, BETA_HI = 0.1, 0.9


PARAM_SPAN = 0.25


def norm_inputs(Wi, beta, Re):
    return (PARAM_SPAN * (math.log(Wi) - math.log(WI_LO)) / math.log(WI_HI / WI_LO),
            PARAM_SPAN * (beta - BETA_LO) / (BETA_HI - BETA_LO), PARAM_SPAN * math.log(Re))


CHANNEL_NX = 4


def dims_of(sp):
    """Lattice size of a spec: side x side (four-roll mill) or
    CHANNEL_NX x side (channel)."""
    if sp.get("geometry", "four_roll") == "channel":
        return (CHANNEL_NX, sp["side"])
    return (sp["side"], sp["side"])


def lattice_of(V, sim, sp):
    """Parameters, boundaries and force of one instance; returns the lattice
    parameters and the stress scale."""
    if sp.get("geometry", "four_roll") == "channel":
        L = float(sp["side"])
        sim.set_params(sp["Re"], sp["Wi"], sp["beta"], sp["U0"], L)
        sim.set_boundaries((V.PERIODIC, V.WALLS))
        lp = sim.lattice_params()
        sim.set_force(V.FORCE_CONST, (8 * (lp["nu_s"] + lp["nu_p"]) * sp["U0"] / L ** 2, 0.0, 0.0))
        return lp, lp["eta_p"] * 4 * sp["U0"] / L
    sim.set_params(sp["Re"], sp["Wi"], sp["beta"], sp["U0"], sp["side"] / (2 * math.pi))
    lp = sim.lattice_params()
    k = 2 * math.pi / sp["side"]
    a = 2 * lp["nu_s"] * sp["U0"] * k * k
    sim.set_force(V.FORCE_FOUR_ROLL, (a, -a, 0.0))
    return lp, lp["eta_p"] * sp["U0"] * k


def step_cap(V, sp, cap=2_000_000):
    """min(cap, 50 T) steps, T the slower of the relaxation time lambda and,
    in the channel, the viscous time L^2 / nu."""
    if sp.get("geometry", "four_roll") == "channel":
        L = float(sp["side"])
        nu = sp["U0"] * L / sp["Re"]
        return int(min(cap, 50 * max(sp["Wi"] * L / sp["U0"], L * L / nu)))
    lam = sp["Wi"] * (sp["side"] / (2 * math.pi)) / sp["U0"]
    return int(min(cap, 50 * lam))


def four_roll_batch(V, specs, storage="f32", stream=None):
    """A batch of the instances of specs (either geometry), configured."""
    b = V.Batch([dims_of(sp) for sp in specs], storage, stream=stream)
    scales = [lattice_of(V, b[i], sp)[1] for i, sp in enumerate(specs)]
    return b, scales


batch_of = four_roll_batch


def channel_steady(ny, g, nu_s, nu_p, lam, D):
    """Steady Oldroyd-B channel (Sec. 3.2) on the nodes y = j + 1/2 of a
    channel of height L = ny between halfway walls: u = g y (L - y)/(2 nu),
    A_xy = lam u', A_yy = 1, A_xx = 1 + 2 (lam u')^2 + 4 D lam^3 (g/nu)^2 (the
    last term from the diffusion D of the conformation scheme), and the
    polymer stress tau = (eta_p / lam)(A - I), eta_p = nu_p.  Returns u [ny],
    tau [ny, 3] (xx, xy, yy)."""
    y = np.arange(ny) + 0.5
    nu = nu_s + nu_p
    u = g * y * (ny - y) / (2 * nu)
    du = g * (ny - 2 * y) / (2 * nu)
    axy = lam * du
    axx = 1 + 2 * axy ** 2 + 4 * D * lam ** 3 * (g / nu) ** 2
    k = nu_p / lam
    return u, np.stack([k * (axx - 1), k * axy, 0 * y], 1)


def residual_at(b, t_end, check_every):
    """Step every active instance to time level t_end and return the
    residuals over its last check_every steps."""
    b.step(t_end - check_every - b[0].t)
    b.reduce()
    b.step(check_every)
    return b.reduce()


def cold_runs(V, specs, tol=1e-6, check_every=100, K0=1000, storage="f32", caps=None):
    """Every instance from rest to R < tol (or its cap) in one batch, with its
    residual after K0 steps on the way."""
    b, scales = four_roll_batch(V, specs, storage)
    for i in range(len(specs)):
        b[i].init_fields()
    if caps is None:
        caps = [max(step_cap(V, sp), K0 + check_every) for sp in specs]
    t0 = time.perf_counter()
    red = residual_at(b, K0, check_every)
    steps, res, status = b.run_until(tol, check_every, caps)
    return dict(batch=b, scales=scales, steps=steps, R=res, status=status, R_K0=red[:, 0].copy(),
                seconds=time.perf_counter() - t0)


# the training runs of earlier versions of this module went under this name
steady_states = cold_runs


def training_set(V, run, specs, which):
    """Inputs and normalised targets of the instances `which` (float32)."""
    xs, ts = [], []
    for i in which:
        sp, sim = specs[i], run["batch"][i]
        nx, ny = dims_of(sp)
        u = sim.read(V.FIELD_U)
        tau = sim.read(V.FIELD_TAU)
        gx, gy = np.meshgrid(np.arange(nx) / nx, np.arange(ny) / ny)
        w, bb, r = norm_inputs(sp["Wi"], sp["beta"], sp["Re"])
        m = nx * ny
        x = np.stack([gx.ravel(), gy.ravel(), np.full(m, w), np.full(m, bb),
                      np.full(m, r)], axis=1)
        t = np.concatenate([u / sp["U0"], tau / run["scales"][i]], axis=1)
        xs.append(x)
        ts.append(t)
    return np.concatenate(xs).astype(np.float32), np.concatenate(ts).astype(np.float32)


def train(mlp, X, T, iters, rows, lr, seed=0, log_every=0):
    """vflb_mlp_train on the data set (copied to the device once): random
    minibatches of `rows` points, cosine-decayed rate, targets standardised
    and the standardisation folded into the output layer by the library.
    Returns the loss history (standardised units)."""
    import torch
    Xd = torch.as_tensor(X, device=mlp.device)
    Td = torch.as_tensor(T, device=mlp.device)
    return mlp.train(Xd, Td, rows, iters, lr, seed=seed, log_every=log_every)


class ColdModel:
    """What the training runs (from rest) say about a cold run at new
    parameters: the mean of log R(K0) and of log steps-to-tol over the k
    nearest converged training runs in (ln Wi / ln 50, (beta - 0.1)/0.8)."""

    def __init__(self, specs, run, k=3):
        ok = [i for i in range(len(specs)) if run["status"][i] == 1]
        self.P = np.array([self._coord(specs[i]) for i in ok])
        self.logR = np.log(np.maximum(run["R_K0"][ok], 1e-300))
        self.logS = np.log(run["steps"][ok].astype(np.float64))
        self.k = min(k, len(ok))

    @staticmethod
    def _coord(sp):
        return ((math.log(sp["Wi"]) - math.log(WI_LO)) / math.log(WI_HI / WI_LO),
                (sp["beta"] - BETA_LO) / (BETA_HI - BETA_LO))

    def predict(self, sp):
        d = np.linalg.norm(self.P - np.array(self._coord(sp)), axis=1)
        nn = np.argsort(d)[: self.k]
        return float(np.exp(self.logR[nn].mean())), float(np.exp(self.logS[nn].mean()))


def warm_runs(V, mlp, specs, model, tol=1e-6, check_every=100, K0=1000, window=5,
              storage="f32", settle=0, settle_flags=2, u_scale_factor=1.0):
    """Held-out instances started from the network, judged by the fallback
    rule (module docstring) and run to R < tol.  Returns the batch, the steps
    of each warm run, the step at which a rejected run was abandoned (0
    when kept), and the residual history of the probe."""
    import torch
    n = len(specs)
    caps = np.array([max(step_cap(V, sp), K0 + (window + 1) * check_every) for sp in specs])
    warm, scales = four_roll_batch(V, specs, storage, stream=mlp.stream)
    flags = settle_flags if settle else 0
    t0 = time.perf_counter()
    for i, sp in enumerate(specs):
        warm[i].init_from_mlp(mlp, norm_inputs(sp["Wi"], sp["beta"], sp["Re"]),
                              sp["U0"] * u_scale_factor, scales[i], settle, flags)
    torch.cuda.synchronize()
    t_infer = time.perf_counter() - t0
    pred = [model.predict(sp) for sp in specs]
    red = residual_at(warm, K0, check_every)
    R0 = red[:, 0]
    abandoned = np.zeros(n, dtype=np.int64)
    done = np.zeros(n, dtype=bool)
    steps = np.zeros(n, dtype=np.int64)
    status = np.zeros(n, dtype=np.int32)
    for i in range(n):
        if not np.isfinite(R0[i]) or red[i, 7] > 0 or R0[i] > pred[i][0]:
            abandoned[i] = K0
        elif R0[i] < tol:
            done[i], steps[i], status[i] = True, K0, V.RUN_CONVERGED
        if abandoned[i] or done[i]:
            warm.set_active(i, False)
    # window of checks: decay rate of the residual, projected steps to tol
    hist = [R0.copy()]
    ts = [K0]
    for w in range(window):
        if not any(warm.is_active(i) for i in range(n)):
            break
        warm.step(check_every)
        r = warm.reduce()[:, 0]
        hist.append(r.copy())
        ts.append(K0 + (w + 1) * check_every)
        for i in range(n):
            if warm.is_active(i) and r[i] < tol:
                done[i], steps[i], status[i] = True, ts[-1], V.RUN_CONVERGED
                warm.set_active(i, False)
    H = np.array(hist)
    tt = np.array(ts, dtype=np.float64)
    projected = np.full(n, np.nan)
    for i in range(n):
        if not warm.is_active(i):
            continue
        logR = np.log(np.maximum(H[:, i], 1e-300))
        rate = -np.polyfit(tt, logR, 1)[0]   # per step
        projected[i] = (tt[-1] + math.log(H[-1, i] / tol) / rate) if rate > 0 else math.inf
        if projected[i] > pred[i][1]:
            abandoned[i] = int(tt[-1])
            warm.set_active(i, False)
    t1 = time.perf_counter()
    s_w, R_w, st_w = warm.run_until(tol, check_every, caps)
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t1
    for i in range(n):
        if abandoned[i]:
            status[i] = V.RUN_SKIPPED   # the cold run replaces it
        elif not done[i]:
            steps[i], status[i] = s_w[i], st_w[i]
    return dict(batch=warm, steps=steps, status=status, abandoned=abandoned, R_K0=R0,
                R_hist=H, t_hist=tt, projected=projected,
                pred_R_K0=np.array([p[0] for p in pred]),
                pred_steps=np.array([p[1] for p in pred]),
                seconds_inference=t_infer, seconds_run=t_run)


def analytic_batch(V, specs, storage="f64"):
    """Channels started from the analytic steady state (channel_steady), an
    equilibrium-only start like the network's."""
    b, _ = four_roll_batch(V, specs, storage)
    for i, sp in enumerate(specs):
        lp = b[i].lattice_params()
        nx, ny = dims_of(sp)
        g = 8 * (lp["nu_s"] + lp["nu_p"]) * sp["U0"] / ny ** 2
        u1, tau1 = channel_steady(ny, g, lp["nu_s"], lp["nu_p"], lp["lam"],
                                  (lp["tau_h"] - 0.5) / 3)
        u = np.zeros((ny, nx, 2))
        u[:, :, 0] = u1[:, None]
        tau = np.repeat(tau1[:, None, :], nx, axis=1)
        b[i].init_fields(u.reshape(-1, 2), tau.reshape(-1, 3), None)
    return b


def analytic_runs(V, specs, tol=1e-6, check_every=100, storage="f64"):
    """The analytic start (analytic_batch) run to R < tol: what a perfect
    prediction of the fields buys."""
    b = analytic_batch(V, specs, storage)
    caps = [step_cap(V, sp) for sp in specs]
    steps, res, status = b.run_until(tol, check_every, caps)
    return dict(batch=b, steps=steps, status=status, R=res)


def field_errors(V, sim, ref):
    """Relative L2 distance of u and tau of sim from those of ref."""
    out = []
    for f in (V.FIELD_U, V.FIELD_TAU):
        a, b = sim.read(f), ref.read(f)
        out.append(float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)))
    return out


def steps_to_accuracy(V, b, ref_fields, target, caps, every=500):
    """Step the active instances of b and return, per instance, the first
    time level (checked every `every` steps) at which the larger of its u
    and tau relative L2 distances from ref_fields[i] = (u, tau) is at most
    target[i]; caps[i] when that does not happen by then."""
    n = len(b)
    out = np.array(caps, dtype=np.int64)
    done = np.zeros(n, dtype=bool)

    def check(i):
        u, tau = ref_fields[i]
        e = max(np.linalg.norm(b[i].read(V.FIELD_U) - u) / np.linalg.norm(u),
                np.linalg.norm(b[i].read(V.FIELD_TAU) - tau) / max(np.linalg.norm(tau), 1e-300))
        if e <= target[i]:
            done[i] = True
            out[i] = b[i].t
            b.set_active(i, False)

    for i in range(n):
        if b.is_active(i):
            check(i)
    while any(b.is_active(i) for i in range(n)):
        b.step(every)
        for i in range(n):
            if b.is_active(i):
                if b[i].t >= caps[i]:
                    b.set_active(i, False)
                else:
                    check(i)
    return out


def warm_vs_cold(V, mlp, specs, model, tol=1e-6, check_every=100, K0=1000, window=5,
                 storage="f32", settle=0, settle_flags=2, ref_tol=1e-9, u_scale_factor=1.0):
    """Held-out instances from rest and from the network (with the fallback
    rule), each to R < tol, and an FP64 cold run of each to R < ref_tol as
    the reference the final fields of both are measured against."""
    n = len(specs)
    cold = cold_runs(V, specs, tol, check_every, K0, storage)
    warm = warm_runs(V, mlp, specs, model, tol, check_every, K0, window, storage, settle,
                     settle_flags, u_scale_factor)
    eff = np.where(warm["abandoned"] > 0, warm["abandoned"] + cold["steps"], warm["steps"])
    ref_caps = [3 * max(step_cap(V, sp), K0 + check_every) for sp in specs]
    ref = cold_runs(V, specs, ref_tol, check_every, K0, "f64", caps=ref_caps)
    err_cold = np.array([field_errors(V, cold["batch"][i], ref["batch"][i]) for i in range(n)])
    err_warm = np.array([field_errors(V, (cold if warm["abandoned"][i] else warm)["batch"][i],
                                      ref["batch"][i]) for i in range(n)])
    # the same final accuracy: steps of a fresh warm start until it is as
    # close to the reference as the cold run was when it stopped (a run the
    # fallback rule abandons keeps the cold run's count)
    ref_fields = [(ref["batch"][i].read(V.FIELD_U), ref["batch"][i].read(V.FIELD_TAU))
                  for i in range(n)]
    target = err_cold.max(1)
    again, scales = four_roll_batch(V, specs, storage, stream=mlp.stream)
    for i, sp in enumerate(specs):
        again[i].init_from_mlp(mlp, norm_inputs(sp["Wi"], sp["beta"], sp["Re"]),
                               sp["U0"] * u_scale_factor, scales[i], settle,
                               settle_flags if settle else 0)
        if warm["abandoned"][i]:
            again.set_active(i, False)
    acc = steps_to_accuracy(V, again, ref_fields, target, ref_caps)
    eff_acc = np.where(warm["abandoned"] > 0, warm["abandoned"] + cold["steps"], acc)
    return dict(cold_steps=cold["steps"], cold_status=cold["status"], R_cold_K0=cold["R_K0"],
                warm_steps_same_accuracy=eff_acc,
                warm_steps=warm["steps"], warm_status=warm["status"], R_warm_K0=warm["R_K0"],
                abandoned=warm["abandoned"], effective_warm_steps=eff,
                fallback=warm["abandoned"] > 0, projected=warm["projected"],
                pred_R_K0=warm["pred_R_K0"], pred_steps=warm["pred_steps"],
                err_cold=err_cold, err_warm=err_warm, ref_status=ref["status"],
                ref_R=ref["R"], ref_steps=ref["steps"], ref=ref["batch"],
                seconds_cold=cold["seconds"], seconds_warm=warm["seconds_run"],
                seconds_inference=warm["seconds_inference"], warm=warm["batch"],
                cold=cold["batch"])
