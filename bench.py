"""Throughput of the fused fluctuating-LB step on one MI355X.

Default workload: the 3D Taylor-Green vortex on a periodic 512^3 D3Q19
lattice (theta = 0 start with its pressure, U0 = 0.02, Re = 100, Wi = 0.5,
beta = 0.9, L = 512/(2 pi); tau = 0 at t = 0), FP32 arithmetic and FP32
population storage; synthetic input generated on the device, no dataset.
One step is one fused stream-and-collide launch over the whole lattice; the
FP64 residual/conservation reduction runs every 100 steps inside the timed
region as in a production run.  `--workload channel` runs the 8192 x 1024
D2Q9 Poiseuille channel instead.

Prints one JSON line: MLUPS (whole job), the roofline of the step kernel
(algorithmic bytes per lattice update / measured kernel time, against the
8 TB/s HBM peak), the CPU oracle timed on a bounded sample of the same
workload (a 64^3 copy with identical lattice-unit parameters), and the time
to a steady state (R < 1e-6) of held-out four-roll lattices started from
rest and from the learned warm start.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
NX, NY = 8192, 1024
RE, WI, BETA, U0, L = 30.72, 1.0, 0.5, 0.01, 1024.0
REDUCE_EVERY = 100


def bytes_per_lup(d, storage):
    """Algorithmic HBM bytes per lattice update: every f and h population
    read once and written once, plus chi(t-1) and u(t-1) read and written;
    16-bit storage also reads and writes each node's FP32 anchor (A - I, p,
    u: 24 bytes in D2Q9, 40 in D3Q19)."""
    q, nc = (9, 3) if d == 2 else (19, 6)
    sb = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}[storage]
    ab = 8 if storage == "f64" else 4
    anchor = 2 * (24 if d == 2 else 40) if sb == 2 else 0
    return 2 * q * (1 + nc) * sb + 2 * (nc + d) * ab + anchor


# stress-divergence scheme: per step one extra pass pulls the 9 (f, h)
# tuples of every node (144 B) and writes tau_p (12 B), one reads tau_p
# (12 B) and writes div tau_p (8 B), and the step reads div tau_p (8 B)
STRESS_DIV_EXTRA_BYTES = 144 + 12 + 12 + 8 + 8


# in-place (AA) streaming: a velocity pass reads the 8 moving f of every
# node (32 B in FP32) and writes u (8 B); the step reads u (8 B)
INPLACE_EXTRA_BYTES = 8 * 4 + 8 + 8


def run_gpu(steps, warmup, storage="f32", tile=0, scheme="fluctuating", inplace=False):
    import torch
    from paper_2506_13072_amd import vflb
    g = vflb.Sim(2, NX, NY, 1, storage, scheme=scheme, inplace=inplace)
    g.set_params(RE, WI, BETA, U0, L)
    g.set_boundaries((vflb.PERIODIC, vflb.WALLS))
    if tile:
        g.set_tile(tile)
    lp = g.lattice_params()
    nu = lp["nu_s"] + lp["nu_p"]
    g.set_force(vflb.FORCE_CONST, (8 * nu * U0 / L ** 2, 0.0, 0.0))
    g.init_fields()
    g.step(1)
    done = 1
    while done < warmup:
        n = min(REDUCE_EVERY, warmup - done)
        g.step(n)
        done += n
    g.reduce()
    g.synchronize()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(g.stream)
    red_ms = 0.0
    left = steps
    r = None
    while left > 0:
        n = min(REDUCE_EVERY, left)
        g.step(n)
        left -= n
        if left > 0 or n == REDUCE_EVERY or r is None:
            r0 = torch.cuda.Event(enable_timing=True)
            r1 = torch.cuda.Event(enable_timing=True)
            r0.record(g.stream)
            r = g.reduce()
            r1.record(g.stream)
            r1.synchronize()
            red_ms += r0.elapsed_time(r1)
    e1.record(g.stream)
    e1.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = e0.elapsed_time(e1)
    step_ms = (total_ms - red_ms) / steps
    return dict(total_ms=total_ms, step_ms=step_ms, red_ms=red_ms, wall=wall,
                R=r["R"], nonfinite=r["nonfinite"],
                buffer_bytes=sum(int(b.numel()) for b in g.buffers))


# stress-divergence scheme in 3D: the tau_p pass pulls the 19 (f, h)
# populations of every node (19 * 7 words) and writes tau_p (6 words), the
# divergence pass reads tau_p (6) and writes div tau_p (3), the step reads
# div tau_p (3): words per update
STRESS_DIV3_EXTRA_WORDS = 19 * 7 + 6 + 6 + 3 + 3


def run_gpu_tgv(n, steps, warmup, storage="f32", tile=0, scheme="fluctuating", inplace=False):
    """3D Taylor-Green vortex, D3Q19, periodic n^3, theta = 0 start,
    U0 = 0.02, Re = 100, Wi = 0.5, beta = 0.9, L = n/(2 pi).  The FP64
    reduction runs every REDUCE_EVERY steps inside the timed region; its
    time is measured on the same stream and left out of the kernel time."""
    import math
    import torch
    from paper_2506_13072_amd import vflb
    from paper_2506_13072_amd.workloads import taylor_green_3d_device
    g = vflb.Sim(3, n, n, n, storage, scheme=scheme, inplace=inplace)
    g.set_params(100.0, 0.5, 0.9, 0.02, n / (2 * math.pi))
    if tile:
        g.set_tile(tile)
    u, p = taylor_green_3d_device(n, 0.02)
    g.init_fields_device(u, None, p)
    del u, p
    g.step(warmup)
    g.reduce()
    g.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(g.stream)
    red_ms = 0.0
    left = steps
    r = None
    while left > 0:
        k = min(REDUCE_EVERY, left)
        g.step(k)
        left -= k
        if k == REDUCE_EVERY or r is None:
            r0 = torch.cuda.Event(enable_timing=True)
            r1 = torch.cuda.Event(enable_timing=True)
            r0.record(g.stream)
            r = g.reduce()
            r1.record(g.stream)
            r1.synchronize()
            red_ms += r0.elapsed_time(r1)
    e1.record(g.stream)
    e1.synchronize()
    wall = time.perf_counter() - t0
    total_ms = e0.elapsed_time(e1)
    step_ms = (total_ms - red_ms) / steps
    out = dict(total_ms=total_ms, step_ms=step_ms, red_ms=red_ms, wall=wall,
               GLUPS=n ** 3 / step_ms / 1e6, KE=r["KE"], R=r["R"], nonfinite=r["nonfinite"],
               buffer_bytes=sum(int(b.numel()) for b in g.buffers))
    del g
    torch.cuda.empty_cache()
    return out


def ensemble_specs(n):
    """The four-roll ensemble: per instance a side in {64..512}, Wi and beta
    from the seeded draws, Re = 1, U0 = 0.01, L = side / (2 pi), the force
    amplitude 2 nu_s U0 k^2 with k = 2 pi / side."""
    import math
    from paper_2506_13072_amd.workloads import ensemble_draws
    return [dict(side=d["side"], Re=d["Re"], Wi=d["Wi"], beta=d["beta"], U0=d["U0"],
                 L=d["side"] / (2 * math.pi)) for d in ensemble_draws(n)]


def setup_instance(V, sim, sp):
    import math
    sim.set_params(sp["Re"], sp["Wi"], sp["beta"], sp["U0"], sp["L"])
    lp = sim.lattice_params()
    k2 = (2 * math.pi / sp["side"]) ** 2
    a = 2 * lp["nu_s"] * sp["U0"] * k2
    sim.set_force(V.FORCE_FOUR_ROLL, (a, -a, 0.0))


def run_gpu_ensemble(n, steps, warmup, storage="f32", compare_unbatched=True):
    """n four-roll instances as one batch: MLUPS of the batched step, and of
    the same instances stepped one lattice at a time (same kernels)."""
    import tempfile
    import torch
    from paper_2506_13072_amd import vflb as V
    specs = ensemble_specs(n)
    b = V.Batch([(sp["side"], sp["side"]) for sp in specs], storage)
    for i, sp in enumerate(specs):
        setup_instance(V, b[i], sp)
    cache = os.path.join(tempfile.gettempdir(), "vflb_autotune.txt")
    tile = b.autotune(cache)
    for i in range(n):
        b[i].init_fields()
    nodes = sum(sp["side"] ** 2 for sp in specs)
    b.step(warmup)
    b.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.step(steps)
    e1.record(b.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    red = b.reduce()
    out = dict(step_ms=ms, MLUPS=nodes / ms / 1e3, nodes=nodes, tile=tile,
               nonfinite=float(red[:, 7].sum()))
    del b
    if compare_unbatched:
        torch.cuda.empty_cache()
        st = torch.cuda.Stream()
        sims = []
        for sp in specs:
            g = V.Sim(2, sp["side"], sp["side"], 1, storage, stream=st)
            setup_instance(V, g, sp)
            g.init_fields()
            sims.append(g)
        for g in sims:
            g.step(warmup)
        st.synchronize()
        e0.record(st)
        for g in sims:
            g.step(steps)
        e1.record(st)
        e1.synchronize()
        ms1 = e0.elapsed_time(e1) / steps
        out.update(unbatched_step_ms=ms1, unbatched_MLUPS=nodes / ms1 / 1e3)
    return out


def run_gpu_ensemble_steady(n, storage="f64", tol=1e-6, every=100, chunk=20000):
    """The four-roll ensemble run to a steady state in one batch: every
    instance from rest until its residual R < tol over `every` steps, capped
    at 40 max(lambda, T_nu) steps (T_nu = 1 / (nu k^2), the viscous time),
    compacted as instances leave.  The run is cut into windows of `chunk`
    steps (each window one vflb_batch_run_until call, instances still short
    of tol resume in the next) only so that progress is printed.  Returns
    per-instance steps and outcomes and the wall time."""
    import math
    import tempfile
    import torch
    from paper_2506_13072_amd import vflb as V
    specs = ensemble_specs(n)
    b = V.Batch([(sp["side"], sp["side"]) for sp in specs], storage)
    for i, sp in enumerate(specs):
        setup_instance(V, b[i], sp)
    tile = b.autotune(os.path.join(tempfile.gettempdir(), "vflb_autotune.txt"))
    for i in range(n):
        b[i].init_fields()
    caps = []
    for sp in specs:
        t_nu = sp["side"] / (2 * math.pi * sp["U0"])   # 1 / (nu k^2) at Re = 1
        lam = sp["Wi"] * t_nu
        caps.append(int(math.ceil(min(2_000_000, 40 * max(lam, t_nu)) / every) * every))
    status = np.zeros(n, dtype=np.int32)
    steps = np.zeros(n, dtype=np.int64)
    resid = np.full(n, np.inf)
    b.synchronize()
    t0 = time.perf_counter()
    level = 0
    while (status == V.RUN_ACTIVE).any():
        run = np.flatnonzero(status == V.RUN_ACTIVE)
        level = min(level + chunk, max(caps[i] for i in run))
        for i in range(n):
            b.set_active(i, int(status[i] == V.RUN_ACTIVE))
        ms = [min(caps[i], level) for i in range(n)]
        st, res, out = b.run_until(tol, every, ms)
        for i in run:
            steps[i], resid[i] = st[i], res[i]
            if not (out[i] == V.RUN_CAPPED and st[i] < caps[i]):
                status[i] = out[i]
        print(f"ensemble to R < {tol:g}: step {level}, {int((status == V.RUN_ACTIVE).sum())} "
              f"running, {int((status == V.RUN_CONVERGED).sum())} converged, "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    nodes = np.array([sp["side"] ** 2 for sp in specs], dtype=np.int64)
    del b
    return dict(specs=specs, steps=steps, resid=resid, status=status, caps=np.array(caps),
                wall_s=wall, lups=float((steps * nodes).sum()), nodes=int(nodes.sum()), tile=tile)


def run_gpu_warmstart(n_train=96, n_test=16, side=64, tol=1e-6, iters=8000, K0=1000,
                      settle=0, window=5, storage="f64", settle_flags=3, geometry="four_roll"):
    """Time to a steady state (R < tol) of held-out four-roll lattices (or
    channels of height `side`), started from rest and from the trained
    network (fallback rule of the warm-start module), and the error of both
    final states against an FP64 cold run of each converged to R < 1e-9; for
    channels also the start from the analytic steady state."""
    import torch
    from paper_2506_13072_amd import vflb as V
    from paper_2506_13072_amd import warmstart as W
    from paper_2506_13072_amd.workloads import ensemble_draws
    draws = ensemble_draws(n_train + n_test, seed=777)
    specs = [dict(side=side, Re=1.0, Wi=d["Wi"], beta=d["beta"], U0=0.01, geometry=geometry)
             for d in draws]
    t0 = time.perf_counter()
    run = W.cold_runs(V, specs[:n_train], tol=tol, K0=K0, storage=storage)
    t_data = time.perf_counter() - t0
    ok = [i for i in range(n_train) if run["status"][i] == V.RUN_CONVERGED]
    X, T = W.training_set(V, run, specs, ok)
    model = W.ColdModel(specs[:n_train], run)
    del run
    mlp = V.Mlp(max_batch=16384, seed=1, sigma=1.5)
    t0 = time.perf_counter()
    hist = W.train(mlp, X, T, iters=iters, rows=16384, lr=2e-3, log_every=iters // 4)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    res = W.warm_vs_cold(V, mlp, specs[n_train:], model, tol=tol, K0=K0, settle=settle,
                         window=window, storage=storage, settle_flags=settle_flags)
    conv = lambda st: int((st == V.RUN_CONVERGED).sum())
    extra = {}
    if geometry == "channel":
        test = specs[n_train:]
        an = W.analytic_runs(V, test, tol=tol, storage=storage)
        ref_fields = [(res["ref"][i].read(V.FIELD_U), res["ref"][i].read(V.FIELD_TAU))
                      for i in range(n_test)]
        an_acc = W.steps_to_accuracy(V, W.analytic_batch(V, test, storage), ref_fields,
                                     res["err_cold"].max(1),
                                     [3 * W.step_cap(V, sp) for sp in test])
        extra = dict(analytic_steps=int(an["steps"].sum()), analytic_converged=conv(an["status"]),
                     analytic_steps_same_accuracy=int(an_acc.sum()),
                     analytic_per_lattice=an["steps"].tolist())
    return dict(n_train=len(ok), t_data=t_data, t_train=t_train, loss=hist[-1][1], **extra,
                cold_steps=int(res["cold_steps"].sum()),
                warm_steps=int(res["effective_warm_steps"].sum()),
                warm_steps_same_accuracy=int(res["warm_steps_same_accuracy"].sum()),
                fallbacks=int(res["fallback"].sum()),
                R_K0_cold_median=float(np.median(res["R_cold_K0"])),
                R_K0_warm_median=float(np.median(res["R_warm_K0"])),
                cold_converged=conv(res["cold_status"]),
                warm_converged=conv(np.where(res["fallback"], res["cold_status"],
                                             res["warm_status"])),
                err_cold=float(np.median(res["err_cold"].max(1))),
                err_warm=float(np.median(res["err_warm"].max(1))),
                ref_converged=conv(res["ref_status"]),
                per_lattice=dict(cold=res["cold_steps"].tolist(),
                                 warm=res["effective_warm_steps"].tolist(),
                                 warm_same_accuracy=res["warm_steps_same_accuracy"].tolist(),
                                 abandoned=res["abandoned"].tolist(),
                                 err_cold=np.round(res["err_cold"].max(1), 9).tolist(),
                                 err_warm=np.round(res["err_warm"].max(1), 9).tolist()),
                t_cold=res["seconds_cold"], t_warm=res["seconds_warm"])


def time_to_steady_state():
    """The metric's second half on bounded samples of both warm-start
    geometries: 16 held-out lattices each, run to R < 1e-6 from rest (the
    plain GPU LB) and from the learned warm start (fallback rule included),
    FP64 storage; steps summed over the lattices, also to the cold runs'
    final accuracy against an FP64 run to R < 1e-9."""
    out = {}
    for geometry, side in (("channel", 128), ("four_roll", 64)):
        r = run_gpu_warmstart(n_train=96, n_test=16, side=side, geometry=geometry)
        keep = ("cold_steps", "warm_steps", "warm_steps_same_accuracy", "fallbacks",
                "cold_converged", "warm_converged", "err_cold", "err_warm", "ref_converged",
                "n_train", "analytic_steps_same_accuracy")
        g = {k: (round(r[k], 6) if isinstance(r[k], float) else r[k]) for k in keep if k in r}
        g["warm_over_cold"] = round(r["warm_steps"] / max(r["cold_steps"], 1), 4)
        g["warm_over_cold_same_accuracy"] = round(r["warm_steps_same_accuracy"] /
                                                  max(r["cold_steps"], 1), 4)
        shape = f"4x{side} channels" if geometry == "channel" else f"{side}x{side} four-roll"
        g["sample"] = (f"16 held-out {shape} (Wi, beta drawn as in the ensemble), network "
                       f"trained on {r['n_train']} steady states; steps summed over the "
                       "lattices; a warm run abandoned by the fallback rule counts its own "
                       "steps plus the cold run's; errors: median over the lattices of the "
                       "larger of the u and tau relative L2 distances from an FP64 run to "
                       "R < 1e-9")
        out[geometry] = g
    return out


# storage modes with committed rocprofv3 records, and the tag in their names
RECORD_TAG = {"f32": "f32", "f16s": "f16"}


def measured_traffic(record, kernel):
    """HBM bytes per launch of the step kernel (FETCH_SIZE + WRITE_SIZE,
    scaled against the streaming-copy kernel) from a committed rocprofv3
    record under profiles/, or None when the record is missing or the kernel
    sources have changed since it was taken."""
    from paper_2506_13072_amd.build import kernel_sources_sha
    try:
        with open(os.path.join(PROFILES, record)) as fh:
            text = fh.read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        key, _, val = line.strip().partition(": ")
        vals[key] = val
    if vals.get("sources_sha256") != kernel_sources_sha(kernel):
        return None
    try:
        return float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_ceiling(nbytes=4 << 30, reps=10, kind=0):
    """Rate of the library's streaming-copy kernel (read + write bytes per
    second), the achievable-bandwidth reference next to the 8 TB/s peak;
    `kind` selects another access kind of the calibration copies."""
    import torch
    from paper_2506_13072_amd import vflb
    st = torch.cuda.Stream()
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    torch.cuda.synchronize()
    vflb.stream_copy(src, dst, st, kind)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        vflb.stream_copy(src, dst, st, kind)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return 2 * nbytes / (ms / 1e3) / 1e9


def host_cpu():
    """CPU model and the number of cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return model, nproc


def run_cpu_baseline_channel(budget_s=15.0):
    """The FP64 oracle, single-threaded, on a 256 x 128 copy of the channel
    (the size of the paper's own timing table) with the same lattice-unit
    parameters except the width; steps until about budget_s of work."""
    from oracle import oracle as O
    nx, ny = 256, 128
    p = O.lattice_params(RE, WI, BETA, U0, L)
    o = O.OracleSim(2, nx, ny)
    o.set_params(p["tau_f"], 0.501, p["lam"], p["eta_p"])
    o.set_walls((0, 1, 0))
    nu = p["nu_s"] + p["nu_p"]
    o.set_force(O.FORCE_CONST, (8 * nu * U0 / L ** 2, 0.0, 0.0))
    o.init()
    o.step(5)
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < budget_s:
        o.step(10)
        n += 10
    dt = time.perf_counter() - t0
    model, nproc = host_cpu()
    return dict(value=nx * ny * n / dt / 1e6, unit="MLUPS", cores=1, kind="oracle",
                cpu_model=model, nproc=nproc,
                sample=f"D2Q9 {nx}x{ny} channel, same lattice parameters, {n} steps, "
                       f"FP64, single thread, {dt:.1f} s")


def run_cpu_baseline_tgv(budget_s=15.0, n=64):
    """The FP64 oracle, single-threaded, on an n^3 copy of the Taylor-Green
    workload with identical lattice-unit parameters (tau_f, lambda, eta_p of
    the 512^3 lattice: L = 512/(2 pi)) and the theta = 0 vortex of the
    smaller lattice; steps until about budget_s of work."""
    import math
    from oracle import oracle as O
    from paper_2506_13072_amd.workloads import taylor_green_3d_velocity
    p = O.lattice_params(100.0, 0.5, 0.9, 0.02, 512 / (2 * math.pi))
    o = O.OracleSim(3, n, n, n)
    o.set_params(p["tau_f"], 0.501, p["lam"], p["eta_p"])
    o.init(taylor_green_3d_velocity(n, 0.02), None, None)
    o.step(1)
    t0 = time.perf_counter()
    k = 0
    while time.perf_counter() - t0 < budget_s:
        o.step(1)
        k += 1
    dt = time.perf_counter() - t0
    model, nproc = host_cpu()
    return dict(value=n ** 3 * k / dt / 1e6, unit="MLUPS", cores=1, kind="oracle",
                cpu_model=model, nproc=nproc,
                sample=f"D3Q19 {n}^3 Taylor-Green copy, lattice parameters of the 512^3 "
                       f"workload, {k} steps, FP64, single thread, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 200 for tgv, 2000 for the D2Q9 workloads)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default: 20 for tgv, 200 otherwise)")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16s", "bf16s", "f64"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tile", type=int, default=0, help="tile height: D2Q9 4, 8, 16; D3Q19 4, 8")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the streaming-copy kernel (counter calibration)")
    ap.add_argument("--copy-kind", type=int, default=0, choices=[0, 1, 2, 3],
                    help="copy probe access kind: 0 non-temporal 16-byte, 1 plain 16-byte, "
                         "2 plain 4-byte, 3 16-byte LDS-DMA loads")
    ap.add_argument("--workload", default="tgv",
                    choices=["channel", "tgv", "ensemble", "ensemble_steady", "warmstart",
                             "schemes", "schemes3d", "inplace", "inplace3d"],
                    help="tgv (default): the 512^3 D3Q19 Taylor-Green vortex; channel: the "
                         "8192x1024 D2Q9 Poiseuille channel; ensemble: 256 four-roll "
                         "lattices of sides 64..512 as one batch")
    ap.add_argument("--no-tts", action="store_true",
                    help="tgv: leave out the time-to-steady-state comparison")
    ap.add_argument("--instances", type=int, default=256)
    ap.add_argument("--ws-side", type=int, default=0,
                    help="warmstart: lattice side (default 64 four-roll, 128 channel height)")
    ap.add_argument("--ws-geometry", default="four_roll", choices=["four_roll", "channel"],
                    help="warmstart: four-roll mill (periodic) or Poiseuille channel (4 x side)")
    ap.add_argument("--ws-train", type=int, default=96, help="warmstart: training lattices")
    ap.add_argument("--ws-test", type=int, default=16, help="warmstart: held-out lattices")
    ap.add_argument("--ws-settle", type=int, default=0,
                    help="warmstart: settling steps after the network's initial state")
    ap.add_argument("--ws-settle-flags", type=int, default=3,
                    help="warmstart: fields prescribed while settling (1 u, 2 A, 3 both)")
    ap.add_argument("--ws-storage", default="f64", choices=["f64", "f32"],
                    help="warmstart and ensemble_steady: storage of the runs to R < 1e-6 (FP32 "
                         "rounding stalls these flows near R = 1e-6)")
    ap.add_argument("--tgv-n", type=int, default=512)
    args = ap.parse_args()
    three_d = args.workload in ("tgv", "schemes3d", "inplace3d")
    if args.steps is None:
        args.steps = 200 if three_d else 2000
    if args.warmup is None:
        args.warmup = 20 if three_d else 200
    if args.copy_probe:
        print(json.dumps({"copy_kind": args.copy_kind,
                          "copy_GBps": round(copy_ceiling(kind=args.copy_kind), 1)}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU slab decomposition is not built)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "warmstart":
        side = args.ws_side or (128 if args.ws_geometry == "channel" else 64)
        r = run_gpu_warmstart(n_train=args.ws_train, n_test=args.ws_test, side=side,
                              settle=args.ws_settle, storage=args.ws_storage,
                              settle_flags=args.ws_settle_flags, geometry=args.ws_geometry)
        shape = f"4x{side} channels" if args.ws_geometry == "channel" else f"four-roll {side}x{side}"
        print(json.dumps({"metric": f"time to steady state (R<1e-6), held-out {shape}, steps "
                                    f"summed over {args.ws_test} lattices",
                          "value": r["warm_steps"], "unit": "steps", "n_gpus": 1,
                          "higher_is_better": False, "vs_baseline": None,
                          "dtype": "f64" if args.ws_storage == "f64" else "f32",
                          "data": "synthetic", "cold_steps": r["cold_steps"],
                          "warm_over_cold": round(r["warm_steps"] / r["cold_steps"], 3),
                          "warm_over_cold_same_accuracy":
                              round(r["warm_steps_same_accuracy"] / r["cold_steps"], 3),
                          "detail": {k: (round(v, 6) if isinstance(v, float) else v)
                                     for k, v in r.items()}}), flush=True)
        return
    if args.workload == "schemes":
        # the paper's comparison (Sec. 3, performance tables): its method
        # against the stress-divergence scheme on the same channel
        nodes = NX * NY
        rows = {}
        for scheme in ("fluctuating", "stress_divergence"):
            r = run_gpu(args.steps, args.warmup, args.storage, args.tile, scheme)
            bpl = bytes_per_lup(2, args.storage) + (
                STRESS_DIV_EXTRA_BYTES * (2 if args.storage == "f64" else 1)
                if scheme == "stress_divergence" else 0)
            rows[scheme] = dict(MLUPS=round(nodes * args.steps / (r["total_ms"] / 1e3) / 1e6, 1),
                                ms_per_step=round(r["total_ms"] / args.steps, 4),
                                bytes_per_lup=bpl,
                                achieved_GBps=round(bpl * nodes / (r["step_ms"] / 1e3) / 1e9, 1),
                                buffer_bytes=r["buffer_bytes"])
        fl, sd = rows["fluctuating"], rows["stress_divergence"]
        ach = sd["achieved_GBps"]
        print(json.dumps({"metric": "MLUPS (stress-divergence scheme, D2Q9 channel)",
                          "value": sd["MLUPS"], "unit": "MLUPS", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": sd["ms_per_step"], "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None,
                          "dtype": "f32" if args.storage != "f64" else "f64", "data": "synthetic",
                          "config": {"workload": "Poiseuille channel D2Q9 8192x1024, both schemes",
                                     "storage": args.storage, "nodes": nodes},
                          "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                                       "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                                       "traffic": None, "bytes_per_lup": sd["bytes_per_lup"]},
                          "schemes": rows,
                          "time_ratio_fluctuating_over_divergence":
                              round(fl["ms_per_step"] / sd["ms_per_step"], 4),
                          "memory_ratio_fluctuating_over_divergence":
                              round(fl["buffer_bytes"] / sd["buffer_bytes"], 4)}), flush=True)
        return
    if args.workload == "schemes3d":
        # the paper's 3D comparison (Taylor-Green performance table): its
        # method against the stress-divergence scheme on the same vortex
        n = args.tgv_n
        nodes = n ** 3
        wb = 8 if args.storage == "f64" else 4
        rows = {}
        for scheme in ("fluctuating", "stress_divergence"):
            r = run_gpu_tgv(n, args.steps, args.warmup, args.storage, args.tile, scheme)
            bpl = bytes_per_lup(3, args.storage) + (
                STRESS_DIV3_EXTRA_WORDS * wb if scheme == "stress_divergence" else 0)
            rows[scheme] = dict(MLUPS=round(nodes * args.steps / (r["total_ms"] / 1e3) / 1e6, 1),
                                ms_per_step=round(r["total_ms"] / args.steps, 4),
                                bytes_per_lup=bpl,
                                achieved_GBps=round(bpl * nodes / (r["step_ms"] / 1e3) / 1e9, 1),
                                buffer_bytes=r["buffer_bytes"])
        fl, sd = rows["fluctuating"], rows["stress_divergence"]
        ach = sd["achieved_GBps"]
        print(json.dumps({"metric": "MLUPS (stress-divergence scheme, D3Q19 Taylor-Green)",
                          "value": sd["MLUPS"], "unit": "MLUPS", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": sd["ms_per_step"], "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None,
                          "dtype": "f32" if args.storage != "f64" else "f64", "data": "synthetic",
                          "config": {"workload": f"3D Taylor-Green vortex D3Q19 {n}^3, both "
                                                 "schemes", "storage": args.storage,
                                     "nodes": nodes},
                          "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                                       "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                                       "traffic": None, "bytes_per_lup": sd["bytes_per_lup"]},
                          "schemes": rows,
                          "time_ratio_fluctuating_over_divergence":
                              round(fl["ms_per_step"] / sd["ms_per_step"], 4),
                          "memory_ratio_fluctuating_over_divergence":
                              round(fl["buffer_bytes"] / sd["buffer_bytes"], 4)}), flush=True)
        return
    if args.workload == "inplace3d":
        # one population buffer (AA streaming, one lane per node) against the
        # two-buffer z-march on the Taylor-Green vortex
        n = args.tgv_n
        nodes = n ** 3
        wb = 8 if args.storage == "f64" else 4
        rows = {}
        for name, inplace in (("two_buffers", False), ("in_place", True)):
            r = run_gpu_tgv(n, args.steps, args.warmup, args.storage, args.tile, inplace=inplace)
            # in place adds a velocity pass: 18 moving f read, u written, u read
            bpl = bytes_per_lup(3, args.storage) + ((18 + 3 + 3) * wb if inplace else 0)
            rows[name] = dict(MLUPS=round(nodes * args.steps / (r["total_ms"] / 1e3) / 1e6, 1),
                              ms_per_step=round(r["total_ms"] / args.steps, 4),
                              bytes_per_lup=bpl,
                              achieved_GBps=round(bpl * nodes / (r["step_ms"] / 1e3) / 1e9, 1),
                              buffer_bytes=r["buffer_bytes"])
        tb, ip = rows["two_buffers"], rows["in_place"]
        ach = ip["achieved_GBps"]
        # one in-place step is two launches (velocity pass, step): their
        # measured bytes together
        traffic = None
        if args.storage == "f32" and n == 512 and not args.tile:
            # FP32 in place: the velocity pass and the z-march with the
            # in-place index maps
            parts = [measured_traffic("aa3_velocity_f32_tgv_512.md", "aa3d"),
                     measured_traffic("step3d_aa_f32_tgv_512.md", "step3d")]
            if None not in parts:
                traffic = sum(parts)
        print(json.dumps({"metric": "MLUPS (in-place AA streaming, D3Q19 Taylor-Green)",
                          "value": ip["MLUPS"], "unit": "MLUPS", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": ip["ms_per_step"], "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None,
                          "dtype": "f32" if args.storage != "f64" else "f64", "data": "synthetic",
                          "config": {"workload": f"3D Taylor-Green vortex D3Q19 {n}^3, one "
                                                 "population buffer vs two",
                                     "storage": args.storage, "nodes": nodes},
                          "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                                       "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                                       "traffic": None if traffic is None else round(traffic / 1e9, 4),
                                       "traffic_unit": "GB per step (both launches)",
                                       "algorithmic_GB_per_step":
                                           round(ip["bytes_per_lup"] * nodes / 1e9, 4),
                                       "bytes_per_lup": ip["bytes_per_lup"]},
                          "layouts": rows,
                          "time_ratio_in_place_over_two_buffers":
                              round(ip["ms_per_step"] / tb["ms_per_step"], 4),
                          "memory_ratio_in_place_over_two_buffers":
                              round(ip["buffer_bytes"] / tb["buffer_bytes"], 4)}), flush=True)
        return
    if args.workload == "inplace":
        # one population buffer (AA streaming) against the two-buffer step
        nodes = NX * NY
        rows = {}
        for name, inplace in (("two_buffers", False), ("in_place", True)):
            r = run_gpu(args.steps, args.warmup, args.storage, args.tile, inplace=inplace)
            bpl = bytes_per_lup(2, args.storage) + (
                INPLACE_EXTRA_BYTES * (2 if args.storage == "f64" else 1) if inplace else 0)
            rows[name] = dict(MLUPS=round(nodes * args.steps / (r["total_ms"] / 1e3) / 1e6, 1),
                              ms_per_step=round(r["total_ms"] / args.steps, 4),
                              bytes_per_lup=bpl,
                              achieved_GBps=round(bpl * nodes / (r["step_ms"] / 1e3) / 1e9, 1),
                              buffer_bytes=r["buffer_bytes"])
        tb, ip = rows["two_buffers"], rows["in_place"]
        ach = ip["achieved_GBps"]
        # one in-place step is two launches (velocity pass, step): their
        # measured bytes together
        traffic = None
        if args.storage == "f32" and not args.tile:
            parts = [measured_traffic(f"aa_{k}_f32_channel_8192x1024.md", "step2d")
                     for k in ("velocity", "step")]
            if None not in parts:
                traffic = sum(parts)
        print(json.dumps({"metric": "MLUPS (in-place AA streaming, D2Q9 channel)",
                          "value": ip["MLUPS"], "unit": "MLUPS", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": ip["ms_per_step"], "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None,
                          "dtype": "f32" if args.storage != "f64" else "f64", "data": "synthetic",
                          "config": {"workload": "Poiseuille channel D2Q9 8192x1024, one "
                                                 "population buffer vs two",
                                     "storage": args.storage, "nodes": nodes},
                          "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                                       "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                                       "traffic": None if traffic is None else round(traffic / 1e9, 4),
                                       "traffic_unit": "GB per step (both launches)",
                                       "algorithmic_GB_per_step":
                                           round(ip["bytes_per_lup"] * nodes / 1e9, 4),
                                       "bytes_per_lup": ip["bytes_per_lup"]},
                          "layouts": rows,
                          "time_ratio_in_place_over_two_buffers":
                              round(ip["ms_per_step"] / tb["ms_per_step"], 4),
                          "memory_ratio_in_place_over_two_buffers":
                              round(ip["buffer_bytes"] / tb["buffer_bytes"], 4)}), flush=True)
        return
    if args.workload == "ensemble_steady":
        r = run_gpu_ensemble_steady(args.instances, args.ws_storage)
        st, sides = r["status"], np.array([sp["side"] for sp in r["specs"]])
        from paper_2506_13072_amd import vflb as V
        by_side = {}
        for side in sorted(set(sides.tolist())):
            m = sides == side
            by_side[str(side)] = dict(instances=int(m.sum()),
                                      converged=int((st[m] == V.RUN_CONVERGED).sum()),
                                      median_steps=int(np.median(r["steps"][m])),
                                      max_steps=int(r["steps"][m].max()))
        print(json.dumps({"metric": "time to steady state (R < 1e-6), batched four-roll ensemble",
                          "value": round(r["wall_s"], 2), "unit": "s", "n_gpus": 1,
                          "steps": int(r["steps"].max()), "warmup": 0,
                          "ms_per_step": None, "higher_is_better": False,
                          "scaling": "weak", "vs_baseline": None,
                          "dtype": args.ws_storage, "data": "synthetic",
                          "config": {"workload": f"four-roll ensemble, {args.instances} D2Q9 "
                                                 "lattices, sides 64..512, seeded Wi and beta, "
                                                 "each from rest to R < 1e-6",
                                     "storage": args.ws_storage, "nodes": r["nodes"],
                                     "tile_y": r["tile"], "check_every": 100,
                                     "cap": "40 max(lambda, 1/(nu k^2)), at most 2e6"},
                          "converged": int((st == V.RUN_CONVERGED).sum()),
                          "capped": int((st == V.RUN_CAPPED).sum()),
                          "unstable": int((st == V.RUN_UNSTABLE).sum()),
                          "steps_total": int(r["steps"].sum()),
                          "lattice_updates": r["lups"],
                          "GLUPS_over_run": round(r["lups"] / r["wall_s"] / 1e9, 2),
                          "by_side": by_side}), flush=True)
        return
    if args.workload == "ensemble":
        r = run_gpu_ensemble(args.instances, args.steps, args.warmup, args.storage)
        bpl = bytes_per_lup(2, args.storage)
        ach = bpl * r["nodes"] / (r["step_ms"] / 1e3) / 1e9
        traffic = None
        if args.storage == "f32" and args.instances == 256:
            traffic = measured_traffic("batch2d_f32_ensemble_256.md", "step2d")
        print(json.dumps({"metric": "MLUPS (batched fused stream-collide, D2Q9 ensemble)",
                          "value": round(r["MLUPS"], 1), "unit": "MLUPS", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": round(r["step_ms"], 4), "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None,
                          "dtype": "f32" if args.storage != "f64" else "f64", "data": "synthetic",
                          "config": {"workload": f"four-roll ensemble, {args.instances} D2Q9 "
                                                 "lattices, sides 64..512, seeded Wi and beta",
                                     "storage": args.storage, "nodes": r["nodes"],
                                     "tile_y": r["tile"]},
                          "roofline": {"bound": "hbm", "achieved": round(ach, 1),
                                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": round(ach / HBM_PEAK_GBS, 4),
                                       "traffic": None if traffic is None else round(traffic / 1e9, 4),
                                       "traffic_unit": "GB per launch",
                                       "algorithmic_GB_per_launch": round(bpl * r["nodes"] / 1e9, 4),
                                       "bytes_per_lup": bpl},
                          "unbatched_MLUPS": round(r.get("unbatched_MLUPS", 0.0), 1),
                          "nonfinite": r["nonfinite"]}), flush=True)
        return
    if args.workload == "tgv":
        r = run_gpu_tgv(args.tgv_n, args.steps, args.warmup, args.storage, args.tile)
        ceiling = copy_ceiling()
        bpl = bytes_per_lup(3, args.storage)
        nodes = args.tgv_n ** 3
        mlups = nodes * args.steps / (r["total_ms"] / 1e3) / 1e6
        ach = bpl * nodes / (r["step_ms"] / 1e3) / 1e9
        traffic = None
        if args.storage in RECORD_TAG and args.tgv_n == 512 and not args.tile:
            traffic = measured_traffic(f"step3d_{RECORD_TAG[args.storage]}_tgv_512.md", "step3d")
        out = {
            "metric": "MLUPS & % HBM peak; time-to-steady-state (1e-6) vs plain GPU LB",
            "value": round(mlups, 1),
            "unit": "MLUPS",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "ms_per_step": round(r["total_ms"] / args.steps, 4),
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f32" if args.storage != "f64" else "f64",
            "data": "synthetic",
            "config": {"workload": f"3D Taylor-Green vortex D3Q19 {args.tgv_n}^3, periodic, "
                                   "theta=0, U0=0.02 Re=100 Wi=0.5 beta=0.9",
                       "storage": args.storage, "nodes": nodes,
                       "reduce_every": REDUCE_EVERY},
            "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                         "traffic": None if traffic is None else round(traffic / 1e9, 4),
                         "traffic_unit": "GB per launch",
                         "algorithmic_GB_per_launch": round(bpl * nodes / 1e9, 4),
                         "bytes_per_lup": bpl,
                         "kernel_ms": round(r["step_ms"], 4),
                         "copy_ceiling_GBps": round(ceiling, 1),
                         "frac_of_copy": round(ach / ceiling, 4)},
            "residual": r["R"],
            "nonfinite": r["nonfinite"],
        }
        if not args.no_tts:
            out["time_to_steady_state"] = time_to_steady_state()
        if not args.no_cpu:
            out["cpu_baseline"] = run_cpu_baseline_tgv()
        print(json.dumps(out), flush=True)
        return
    res = run_gpu(args.steps, args.warmup, args.storage, args.tile)
    ceiling = copy_ceiling()
    nodes = NX * NY
    mlups = nodes * args.steps / (res["total_ms"] / 1e3) / 1e6
    bpl = bytes_per_lup(2, args.storage)
    achieved = bpl * nodes / (res["step_ms"] / 1e3) / 1e9
    traffic = None
    if args.storage in RECORD_TAG and not args.tile:
        traffic = measured_traffic(f"step2d_{RECORD_TAG[args.storage]}_channel_8192x1024.md",
                                   "step2d")
    out = {
        "metric": "MLUPS (fused stream-collide, D2Q9 Oldroyd-B fluctuating LB)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["total_ms"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage != "f64" else "f64",
        "data": "synthetic",
        "config": {"workload": "Poiseuille channel D2Q9 8192x1024, walls in y, "
                               "const force, Re=30.72 Wi=1 beta=0.5",
                   "storage": args.storage, "nodes": nodes,
                   "reduce_every": REDUCE_EVERY},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic / 1e9, 4),
                     "traffic_unit": "GB per launch",
                     "algorithmic_GB_per_launch": round(bpl * nodes / 1e9, 4),
                     "bytes_per_lup": bpl,
                     "kernel_ms": round(res["step_ms"], 5),
                     "copy_ceiling_GBps": round(ceiling, 1),
                     "frac_of_copy": round(achieved / ceiling, 4)},
        "residual": res["R"],
    }
    if not args.no_cpu:
        out["cpu_baseline"] = run_cpu_baseline_channel()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
