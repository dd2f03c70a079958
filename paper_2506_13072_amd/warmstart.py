"""Learned warm start for steady four-roll-mill states (orchestration only).

Every computation runs in libvflb: batches of lattices run to their steady
states (vflb_batch_run_until), the network trains on those states
(vflb_mlp_train_step), and a new lattice starts from the network's
prediction (vflb_init_from_mlp) instead of from rest.  This module only
decides what to call.

Inputs of the network per node: (x/n, y/n, w, b, r) with
w = P (ln Wi - ln 0.1)/ln 50, b = P (beta - 0.1)/0.8, r = P ln Re: the
parameter coordinates span [0, P] with P = 1/4, so that the Gaussian
frequencies vary the features four times more slowly along the parameters
than across the lattice.  Outputs: (u/U0, v/U0, txx/S, txy/S, tyy/S) with
the stress scale S = eta_p U0 k, k = 2 pi / n (viscous stress of the
forcing mode).  Training standardises each output column; the affine map
back is folded into the output layer afterwards, so the trained network
predicts the normalised fields directly.

Fallback: a warm-started lattice is abandoned for the cold run of the same
lattice when its state is non-finite or its residual after K0 steps
exceeds the cold run's residual after K0 steps.
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


def lattice_of(V, sim, sp):
    """Parameters and four-roll force of one instance; returns the lattice
    parameters and the stress scale."""
    sim.set_params(sp["Re"], sp["Wi"], sp["beta"], sp["U0"], sp["side"] / (2 * math.pi))
    lp = sim.lattice_params()
    k = 2 * math.pi / sp["side"]
    a = 2 * lp["nu_s"] * sp["U0"] * k * k
    sim.set_force(V.FORCE_FOUR_ROLL, (a, -a, 0.0))
    return lp, lp["eta_p"] * sp["U0"] * k


def step_cap(V, sp, cap=2_000_000):
    """min(cap, 50 lambda) steps."""
    lam = sp["Wi"] * (sp["side"] / (2 * math.pi)) / sp["U0"]
    return int(min(cap, 50 * lam))


def four_roll_batch(V, specs, storage="f32", stream=None):
    b = V.Batch([(sp["side"], sp["side"]) for sp in specs], storage, stream=stream)
    scales = [lattice_of(V, b[i], sp)[1] for i, sp in enumerate(specs)]
    return b, scales


def steady_states(V, specs, tol=1e-6, check_every=100, storage="f32"):
    """Run every instance from rest to R < tol (or its cap) in one batch."""
    b, scales = four_roll_batch(V, specs, storage)
    for i in range(len(specs)):
        b[i].init_fields()
    caps = [step_cap(V, sp) for sp in specs]
    t0 = time.perf_counter()
    steps, res, status = b.run_until(tol, check_every, caps)
    return dict(batch=b, scales=scales, steps=steps, R=res, status=status,
                seconds=time.perf_counter() - t0)


def training_set(V, run, specs, which):
    """Inputs and normalised targets of the instances `which` (float32)."""
    xs, ts = [], []
    for i in which:
        sp, sim = specs[i], run["batch"][i]
        n = sp["side"]
        u = sim.read(V.FIELD_U)
        tau = sim.read(V.FIELD_TAU)
        gx, gy = np.meshgrid(np.arange(n) / n, np.arange(n) / n)
        w, bb, r = norm_inputs(sp["Wi"], sp["beta"], sp["Re"])
        x = np.stack([gx.ravel(), gy.ravel(), np.full(n * n, w), np.full(n * n, bb),
                      np.full(n * n, r)], axis=1)
        t = np.concatenate([u / sp["U0"], tau / run["scales"][i]], axis=1)
        xs.append(x)
        ts.append(t)
    return np.concatenate(xs).astype(np.float32), np.concatenate(ts).astype(np.float32)


def fold_output_affine(mlp, mean, std):
    """Make the network predict std * y + mean: scale the rows of the last
    layer and shift its bias (flat order: last layer W, then b, at the end)."""
    p = mlp.get_params().astype(np.float64)
    out = len(mean)
    width = mlp.cfg["width"]
    b0 = p.size - out
    w0 = b0 - out * width
    W = p[w0:b0].reshape(out, width)
    p[w0:b0] = (W * std[:, None]).ravel()
    p[b0:] = p[b0:] * std + mean
    mlp.set_params(p.astype(np.float32))


def train(mlp, X, T, iters, rows, lr, seed=0, log_every=0):
    """Adam on random minibatches of `rows` points with a cosine-decayed
    rate, on standardised targets; the standardisation is folded into the
    output layer at the end.  Returns the loss history (standardised units,
    every log_every iterations)."""
    import torch
    dev = mlp.device
    mean = T.mean(0).astype(np.float64)
    std = T.std(0).astype(np.float64)
    std[std == 0] = 1.0
    Xd = torch.as_tensor(X, device=dev)
    Td = torch.as_tensor(((T - mean) / std).astype(np.float32), device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    xb = torch.empty(rows, X.shape[1], device=dev)
    tb = torch.empty(rows, T.shape[1], device=dev)
    hist = []
    torch.cuda.synchronize(dev)
    with torch.cuda.stream(mlp.stream):
        for it in range(iters):
            idx = torch.randint(0, X.shape[0], (rows,), device=dev, generator=g)
            torch.index_select(Xd, 0, idx, out=xb)
            torch.index_select(Td, 0, idx, out=tb)
            rate = lr * 0.5 * (1 + math.cos(math.pi * it / iters))
            want = log_every and (it % log_every == 0 or it == iters - 1)
            loss = mlp.train_step(xb, tb, max(rate, 1e-3 * lr), want_loss=bool(want))
            if want:
                hist.append((it, loss))
    mlp.stream.synchronize()
    fold_output_affine(mlp, mean, std)
    return hist


def warm_vs_cold(V, mlp, specs, tol=1e-6, check_every=100, K0=1000, storage="f32",
                 u_scale_factor=1.0, settle=0, settle_flags=2):
    """Held-out instances from rest and from the network, with the fallback
    rule at K0.  Returns per-instance step counts and timings."""
    import torch
    n = len(specs)
    caps = np.array([max(step_cap(V, sp), K0 + check_every) for sp in specs])
    cold, scales = four_roll_batch(V, specs, storage)
    warm, _ = four_roll_batch(V, specs, storage, stream=mlp.stream)
    for i in range(n):
        cold[i].init_fields()
    t0 = time.perf_counter()
    for i, sp in enumerate(specs):
        warm[i].init_from_mlp(mlp, norm_inputs(sp["Wi"], sp["beta"], sp["Re"]),
                              sp["U0"] * u_scale_factor, scales[i], settle, settle_flags)
    torch.cuda.synchronize()
    t_infer = time.perf_counter() - t0
    # residual at K0 (change over the last check_every steps) on both sides;
    # settling steps count as steps of the warm run
    out = {}
    for name, b in (("cold", cold), ("warm", warm)):
        b.step(K0 - check_every - (settle if name == "warm" else 0))
        b.reduce()
        b.step(check_every)
        out[name] = b.reduce()
    r_cold, r_warm = out["cold"][:, 0], out["warm"][:, 0]
    bad = ~np.isfinite(r_warm) | (out["warm"][:, 7] > 0) | (r_warm > r_cold)
    for i in range(n):
        if bad[i]:
            warm.set_active(i, False)
    t1 = time.perf_counter()
    s_cold, R_cold, st_cold = cold.run_until(tol, check_every, caps)
    torch.cuda.synchronize()
    t_cold = time.perf_counter() - t1
    t2 = time.perf_counter()
    s_warm, R_warm, st_warm = warm.run_until(tol, check_every, caps)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t2
    eff = np.where(bad, K0 + s_cold, s_warm)
    return dict(cold_steps=s_cold, warm_steps=s_warm, effective_warm_steps=eff, fallback=bad,
                cold_status=st_cold, warm_status=st_warm, R_cold_K0=r_cold, R_warm_K0=r_warm,
                R_cold=R_cold, R_warm=R_warm, seconds_cold_after_K0=t_cold,
                seconds_warm_after_K0=t_warm, seconds_inference=t_infer, cold=cold, warm=warm)
