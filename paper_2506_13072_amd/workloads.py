"""Seeded synthetic inputs shared by the tests, the benchmark and the workflows.

This module holds no arithmetic of the method: only workload descriptions in
the paper's dimensionless terms (Sec. 3), seeded random draws and smooth
initial fields.  The HIP path and the CPU oracle each map the dimensionless
numbers to lattice units themselves.
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 20250615
MASK64 = (1 << 64) - 1


def splitmix64(state: int):
    """SplitMix64 (Steele, Lea, Flood 2014): returns (next_state, output)."""
    state = (state + 0x9E3779B97F4A7C15) & MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return state, z ^ (z >> 31)


def uniform01(seed: int, k: int) -> float:
    """k-th uniform draw in [0, 1) of the SplitMix64 stream started at seed."""
    s = seed & MASK64
    out = 0
    for _ in range(k + 1):
        s, out = splitmix64(s)
    return (out >> 11) * (1.0 / (1 << 53))


def smooth_fields(d, shape, seed, amp_u=0.02, amp_tau=1e-3, amp_p=1e-3):
    """Seeded smooth periodic fields u [N, d], tau [N, nc], p [N] built from
    three low Fourier modes each; shape is (ny, nx) or (nz, ny, nx)."""
    rng = np.random.default_rng(seed)
    if d == 2:
        grids = np.meshgrid(*[2 * np.pi * np.arange(n) / n for n in shape[::-1]],
                            indexing="xy")
    else:
        grids = np.meshgrid(*[2 * np.pi * np.arange(n) / n for n in shape],
                            indexing="ij")[::-1]
    N = int(np.prod(shape))
    nc = 3 if d == 2 else 6

    def field(scale):
        out = np.zeros(shape)
        for _ in range(3):
            k = rng.integers(0, 2, size=d)
            ph = rng.uniform(0, 2 * np.pi, size=d)
            term = np.ones(shape)
            for a in range(d):
                term = term * np.cos(k[a] * grids[a] + ph[a])
            out += rng.normal() * term
        return scale * out.reshape(N)

    u = np.stack([field(amp_u) for _ in range(d)], -1)
    tau = np.stack([field(amp_tau) for _ in range(nc)], -1)
    p = field(amp_p)
    return u, tau, p


def taylor_green_3d_velocity(n, U0, theta=0.0):
    """Initial velocity of the 3D Taylor-Green vortex (Sec. 3.4) on an n^3
    periodic grid, node-major [N, 3]:
    u = (2 U0/sqrt 3) (sin(theta + 2pi/3) sin x cos y cos z,
                       sin(theta - 2pi/3) cos x sin y cos z,
                       sin(theta) cos x cos y sin z).
    theta = 0 gives U0 (sin x cos y cos z, -cos x sin y cos z, 0)."""
    x = 2 * np.pi * np.arange(n) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    a = 2 * U0 / math.sqrt(3.0)
    u = np.stack([a * math.sin(theta + 2 * math.pi / 3) * np.sin(X) * np.cos(Y) * np.cos(Z),
                  a * math.sin(theta - 2 * math.pi / 3) * np.cos(X) * np.sin(Y) * np.cos(Z),
                  a * math.sin(theta) * np.cos(X) * np.cos(Y) * np.sin(Z)], -1)
    return u.reshape(-1, 3)


def taylor_green_3d_device(n, U0, device="cuda"):
    """The theta = 0 Taylor-Green vortex of taylor_green_3d_velocity plus its
    pressure (U0^2/16)(cos 2x + cos 2y)(cos 2z + 2), generated on the device
    (torch) for large lattices; returns component-major FP64 tensors
    u [3, N] and p [N] in node order (x fastest)."""
    import torch
    x = 2 * math.pi * torch.arange(n, device=device, dtype=torch.float64) / n
    sx, cx = torch.sin(x), torch.cos(x)
    u = torch.empty(3, n, n, n, device=device, dtype=torch.float64)
    # index order [z, y, x]
    u[0] = U0 * sx[None, None, :] * cx[None, :, None] * cx[:, None, None]
    u[1] = -U0 * cx[None, None, :] * sx[None, :, None] * cx[:, None, None]
    u[2] = 0.0
    c2 = torch.cos(2 * x)
    p = (U0 ** 2 / 16) * (c2[None, None, :] + c2[None, :, None]) * (c2[:, None, None] + 2)
    return u.reshape(3, -1), p.reshape(-1)


# ------------------------------------------------------------ workloads
# Dimensionless descriptions of the benchmark flows (Sec. 3).  L is the
# characteristic length in lattice units.
FOUR_ROLL_64 = dict(name="four-roll mill 64x64, D2Q9, periodic", lattice=2,
                    shape=(64, 64), Re=1.0, Wi=1.0, beta=0.5, U0=0.01,
                    L=64 / (2 * math.pi), steps=10000, force="four_roll")

CHANNEL_8192x1024 = dict(name="Poiseuille channel 8192x1024, D2Q9, walls in y",
                         lattice=2, shape=(1024, 8192), Re=30.72, Wi=1.0, beta=0.5,
                         U0=0.01, L=1024.0, force="const")

TGV_512 = dict(name="3D Taylor-Green vortex 512^3, D3Q19, periodic", lattice=3,
               shape=(512, 512, 512), Re=100.0, Wi=0.5, beta=0.9, U0=0.02,
               L=512 / (2 * math.pi), force="none")


def ensemble_draws(n_instances, seed=BASE_SEED):
    """Parameter sweep of the batched four-roll ensemble: per instance a side
    in {64, 128, 256, 512}, ln Wi uniform in [ln 0.1, ln 5], beta uniform in
    [0.1, 0.9] (SplitMix64, one stream per instance)."""
    out = []
    for k in range(n_instances):
        s = seed + k
        side = (64, 128, 256, 512)[min(3, int(uniform01(s, 0) * 4))]
        wi = math.exp(math.log(0.1) + uniform01(s, 1) * (math.log(5.0) - math.log(0.1)))
        beta = 0.1 + 0.8 * uniform01(s, 2)
        out.append(dict(side=side, Wi=wi, beta=beta, Re=1.0, U0=0.01, seed=s))
    return out
