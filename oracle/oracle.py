"""Python access to the FP64 CPU oracle (``vflb_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing here is shared with the HIP
path of the package, and the package never imports this module.

The C library is built by :func:`build` (plain gcc, ``-O2
-ffp-contract=off`` so that no fused multiply-adds change the rounding of
the written-out arithmetic).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vflb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FORCE_NONE, FORCE_CONST, FORCE_FOUR_ROLL, FORCE_COS_T = 0, 1, 2, 3
SCHEME_FLUCTUATING, SCHEME_STRESS_DIVERGENCE = 0, 1
MODEL_OLDROYD_B, MODEL_GIESEKUS, MODEL_LPTT, MODEL_EPTT = 0, 1, 2, 3


def build() -> str:
    """Compile the oracle into ``oracle/liboracle.so`` (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(
        ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99",
         "-Wall", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        D = ctypes.c_double
        I = ctypes.c_int
        LG = ctypes.c_long
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        L.or_create.restype = P
        L.or_create.argtypes = [I, I, I, I]
        L.or_destroy.argtypes = [P]
        L.or_set_params.argtypes = [P, D, D, D, D]
        L.or_set_walls.argtypes = [P, ip]
        L.or_set_force.argtypes = [P, I, dp, D]
        L.or_time.restype = LG
        L.or_time.argtypes = [P]
        L.or_set_time.argtypes = [P, LG]
        L.or_init.argtypes = [P, P, P, P]
        L.or_step.argtypes = [P, LG]
        L.or_moments.argtypes = [P, P, P, P, P]
        L.or_get_state.argtypes = [P, P, P, P, P]
        L.or_set_state.argtypes = [P, P, P, P, P]
        L.or_force_field.argtypes = [P, LG, dp]
        L.or_set_scheme.argtypes = [P, I]
        L.or_stress_divergence.argtypes = [P, dp]
        L.or_pinv_matrix.argtypes = [I, dp]
        L.or_polymer_stress.argtypes = [I, D, D, dp, dp]
        L.or_fB.argtypes = [I, D, dp, dp]
        L.or_feq.argtypes = [I, D, dp, dp]
        L.or_guo.argtypes = [I, D, dp, dp, dp]
        L.or_velocity.argtypes = [I, dp, dp, dp]
        L.or_pressure.restype = D
        L.or_pressure.argtypes = [I, D, dp, dp, D, D]
        L.or_heq.argtypes = [I, D, dp, dp]
        L.or_chi_i.argtypes = [I, D, D, dp, dp]
        L.or_chi_tensor.argtypes = [I, D, dp, dp, dp]
        L.or_chi_tensor_model.argtypes = [I, D, I, D, dp, dp, dp]
        L.or_set_model.argtypes = [P, I, D]
        L.or_lattice_params.argtypes = [D, D, D, D, D, D, dp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


# ---------------------------------------------------------------- per node
def Q(d):
    return 9 if d == 2 else 19


def NC(d):
    return 3 if d == 2 else 6


def pinv_matrix(d):
    out = np.zeros((9, 4) if d == 2 else (19, 13))
    lib().or_pinv_matrix(d, out)
    return out


def fB(d, tau_f, tau):
    out = np.zeros(Q(d))
    lib().or_fB(d, tau_f, _f64(tau), out)
    return out


def feq(d, p, u):
    out = np.zeros(Q(d))
    lib().or_feq(d, p, _f64(u), out)
    return out


def guo(d, tau_f, F, u):
    out = np.zeros(Q(d))
    lib().or_guo(d, tau_f, _f64(F), _f64(u), out)
    return out


def velocity(d, f, F):
    out = np.zeros(d)
    lib().or_velocity(d, _f64(f), _f64(F), out)
    return out


def pressure(d, tau_f, f, u, F0, fB0):
    return lib().or_pressure(d, tau_f, _f64(f), _f64(u), F0, fB0)


def heq(d, A, u):
    out = np.zeros(Q(d))
    lib().or_heq(d, A, _f64(u), out)
    return out


def chi_i(d, tau_h, chi, u):
    out = np.zeros(Q(d))
    lib().or_chi_i(d, tau_h, chi, _f64(u), out)
    return out


def chi_tensor(d, lam, A, G, model=None, param=0.0):
    """Source tensor chi (components as A) for the symmetric A and the full
    gradient G[a*d+b] = d_a u_b; model None is Oldroyd-B, else MODEL_*."""
    out = np.zeros(NC(d))
    if model is None:
        lib().or_chi_tensor(d, lam, _f64(A), _f64(G), out)
    else:
        lib().or_chi_tensor_model(d, lam, int(model), float(param), _f64(A), _f64(G), out)
    return out


def polymer_stress(d, eta_p, lam, A):
    out = np.zeros(NC(d))
    lib().or_polymer_stress(d, eta_p, lam, _f64(A), out)
    return out


def lattice_params(Re, Wi, beta, U0, L, lambda_override=0.0):
    """Return dict nu_s, nu_p, tau_f, lam, eta_p (lattice units)."""
    out = np.zeros(5)
    lib().or_lattice_params(Re, Wi, beta, U0, L, lambda_override, out)
    return dict(nu_s=out[0], nu_p=out[1], tau_f=out[2], lam=out[3],
                eta_p=out[4])


# ---------------------------------------------------------------- lattice
class OracleSim:
    """FP64 single-threaded simulation of the method on an nx*ny(*nz) grid.

    Fields are node-major with x fastest: u[N, d], p[N], A/tau[N, nc] with
    components (xx, xy, yy) in 2D and (xx, yy, zz, xy, xz, yz) in 3D.
    """

    def __init__(self, d, nx, ny, nz=1):
        self.d, self.nx, self.ny = d, nx, ny
        self.nz = nz if d == 3 else 1
        self.N = nx * ny * self.nz
        self.q, self.nc = Q(d), NC(d)
        self._h = lib().or_create(d, nx, ny, self.nz)
        if not self._h:
            raise ValueError("bad oracle lattice")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_destroy(h)
            self._h = None

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx) if self.d == 3 else (self.ny, self.nx)

    def set_params(self, tau_f, tau_h, lam, eta_p):
        self.tau_f, self.tau_h, self.lam, self.eta_p = tau_f, tau_h, lam, eta_p
        lib().or_set_params(self._h, tau_f, tau_h, lam, eta_p)

    def set_walls(self, walls):
        lib().or_set_walls(self._h, np.asarray(list(walls) + [0] * (3 - len(walls)),
                                               dtype=np.int32))

    def set_force(self, kind, amp=(0.0, 0.0, 0.0), omega=0.0):
        a = np.zeros(3)
        a[:len(amp)] = amp
        lib().or_set_force(self._h, kind, a, omega)

    def set_model(self, model, param=0.0):
        """Constitutive model MODEL_* (Oldroyd-B default) with its parameter
        (Giesekus mobility alpha, PTT eps)."""
        lib().or_set_model(self._h, int(model), float(param))

    def set_scheme(self, scheme):
        """SCHEME_FLUCTUATING (the paper's method, default) or
        SCHEME_STRESS_DIVERGENCE (the stress divergence as a body force,
        f^B = 0; the scheme the paper compares against)."""
        self.scheme = int(scheme)
        lib().or_set_scheme(self._h, self.scheme)

    def stress_divergence(self):
        """div tau_p of the current state, [N, d], with the stencil of the
        stress-divergence scheme."""
        div = np.zeros((self.N, self.d))
        lib().or_stress_divergence(self._h, div)
        return div

    def init(self, u=None, tau=None, p=None):
        u = None if u is None else _f64(u, (self.N, self.d))
        tau = None if tau is None else _f64(tau, (self.N, self.nc))
        p = None if p is None else _f64(p, (self.N,))
        lib().or_init(self._h, _ptr(u), _ptr(tau), _ptr(p))

    def step(self, n=1):
        lib().or_step(self._h, int(n))

    @property
    def t(self):
        return lib().or_time(self._h)

    def moments(self):
        u = np.zeros((self.N, self.d))
        p = np.zeros(self.N)
        A = np.zeros((self.N, self.nc))
        tau = np.zeros((self.N, self.nc))
        lib().or_moments(self._h, _ptr(u), _ptr(p), _ptr(A), _ptr(tau))
        return dict(u=u, p=p, A=A, tau=tau)

    def get_state(self):
        f = np.zeros((self.N, self.q))
        h = np.zeros((self.N, self.nc, self.q))
        cp = np.zeros((self.N, self.nc))
        up = np.zeros((self.N, self.d))
        lib().or_get_state(self._h, _ptr(f), _ptr(h), _ptr(cp), _ptr(up))
        return dict(f=f, h=h, chi_prev=cp, u_prev=up, t=self.t)

    def set_state(self, f=None, h=None, chi_prev=None, u_prev=None, t=None):
        f = None if f is None else _f64(f, (self.N, self.q))
        h = None if h is None else _f64(h, (self.N, self.nc, self.q))
        chi_prev = None if chi_prev is None else _f64(chi_prev, (self.N, self.nc))
        u_prev = None if u_prev is None else _f64(u_prev, (self.N, self.d))
        lib().or_set_state(self._h, _ptr(f), _ptr(h), _ptr(chi_prev), _ptr(u_prev))
        if t is not None:
            lib().or_set_time(self._h, int(t))

    def force_field(self, t=None):
        F = np.zeros((self.N, self.d))
        lib().or_force_field(self._h, self.t if t is None else int(t), F)
        return F
