"""Python binding of libvflb (include/vflb.h): argument marshalling only.

Every step of the method runs in the HIP kernels of ``libvflb.so``; PyTorch
supplies device memory (the buffers the library asks for) and the HIP
stream.  Loading fails loudly when the library has not been built: there is
no fallback.

Field arrays returned to Python are node-major, ``[N, ncomp]`` with
x fastest, the same layout as the CPU oracle uses; the library itself works
on component-major ``[ncomp][N]`` arrays.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvflb.so")

D2Q9, D3Q19 = 2, 3
F64, F32, F16S, BF16S = 0, 1, 2, 3
STORAGE = {"f64": F64, "f32": F32, "f16s": F16S, "bf16s": BF16S}
FORCE_NONE, FORCE_CONST, FORCE_FOUR_ROLL, FORCE_COS_T = 0, 1, 2, 3
PERIODIC, WALLS = 0, 1
SCHEME_FLUCTUATING, SCHEME_STRESS_DIVERGENCE = 0, 1
SCHEMES = {"fluctuating": SCHEME_FLUCTUATING, "stress_divergence": SCHEME_STRESS_DIVERGENCE}
MODEL_OLDROYD_B, MODEL_GIESEKUS, MODEL_LPTT, MODEL_EPTT = 0, 1, 2, 3
OPT_INPLACE = 1
(FIELD_U, FIELD_P, FIELD_RHO, FIELD_A, FIELD_TAU, FIELD_F, FIELD_H,
 FIELD_CHI_PREV, FIELD_U_PREV) = range(9)
NBUF = 5
BUF_POP0, BUF_POP1, BUF_AUX, BUF_SNAP, BUF_WORK = range(NBUF)
OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, ESTATE = range(6)
RUN_ACTIVE, RUN_CONVERGED, RUN_CAPPED, RUN_UNSTABLE, RUN_SKIPPED = range(5)
SETTLE_U, SETTLE_A = 1, 2


class VflbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"vflb error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("Re", ctypes.c_double), ("Wi", ctypes.c_double),
                ("beta", ctypes.c_double), ("U0", ctypes.c_double),
                ("L", ctypes.c_double), ("lam", ctypes.c_double),
                ("tau_h", ctypes.c_double)]


class MlpCfg(ctypes.Structure):
    _fields_ = [("in_dim", ctypes.c_int), ("n_freq", ctypes.c_int), ("width", ctypes.c_int),
                ("hidden", ctypes.c_int), ("out_dim", ctypes.c_int), ("max_batch", ctypes.c_int),
                ("sigma", ctypes.c_double)]


class LatticeParams(ctypes.Structure):
    _fields_ = [("nu_s", ctypes.c_double), ("nu_p", ctypes.c_double),
                ("tau_f", ctypes.c_double), ("tau_h", ctypes.c_double),
                ("lam", ctypes.c_double), ("eta_p", ctypes.c_double)]


_lib = None


def lib():
    """The loaded ``libvflb.so`` (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2506_13072_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        I64, SZ = ctypes.c_int64, ctypes.c_size_t
        L.vflb_create.argtypes = [I, I, I, I, I, P, ctypes.POINTER(P)]
        L.vflb_create_scheme.argtypes = [I, I, I, I, I, I, P, ctypes.POINTER(P)]
        L.vflb_create_ex.argtypes = [I, I, I, I, I, I, I, P, ctypes.POINTER(P)]
        L.vflb_set_model.argtypes = [P, I, ctypes.c_double]
        L.vflb_query_buffers.argtypes = [P, ctypes.POINTER(SZ)]
        L.vflb_bind_buffers.argtypes = [P, ctypes.POINTER(P)]
        L.vflb_set_params.argtypes = [P, ctypes.POINTER(Params)]
        L.vflb_get_lattice_params.argtypes = [P, ctypes.POINTER(LatticeParams)]
        L.vflb_set_force.argtypes = [P, I, ctypes.POINTER(D), D]
        L.vflb_set_boundaries.argtypes = [P, ctypes.POINTER(I)]
        L.vflb_set_storage_scale.argtypes = [P, I, I]
        L.vflb_init_fields.argtypes = [P, P, P, P]
        L.vflb_step.argtypes = [P, I64]
        L.vflb_time.argtypes = [P]
        L.vflb_time.restype = I64
        L.vflb_reduce.argtypes = [P, ctypes.POINTER(D)]
        L.vflb_reduce_noalloc.argtypes = [P, ctypes.POINTER(D)]
        L.vflb_read.argtypes = [P, I, P, SZ]
        L.vflb_read_box.argtypes = [P, I, ctypes.POINTER(I), ctypes.POINTER(I), P, SZ]
        L.vflb_read_box.restype = I
        L.vflb_state_size.argtypes = [P, ctypes.POINTER(SZ)]
        L.vflb_save.argtypes = [P, P, SZ]
        L.vflb_load.argtypes = [P, P, SZ]
        L.vflb_set_tile.argtypes = [P, I]
        L.vflb_stream_copy.argtypes = [P, P, SZ, P]
        L.vflb_stream_copy.restype = I
        L.vflb_copy_probe.argtypes = [P, P, SZ, I, P]
        L.vflb_copy_probe.restype = I
        L.vflb_destroy.argtypes = [P]
        L.vflb_destroy.restype = None
        L.vflb_batch_create.argtypes = [I, I, ctypes.POINTER(I), I, P, ctypes.POINTER(P)]
        L.vflb_batch_query_buffers.argtypes = [P, ctypes.POINTER(SZ)]
        L.vflb_batch_bind_buffers.argtypes = [P, ctypes.POINTER(P)]
        L.vflb_batch_instance.argtypes = [P, I]
        L.vflb_batch_instance.restype = P
        L.vflb_batch_size.argtypes = [P]
        L.vflb_batch_size.restype = I
        L.vflb_batch_set_tile.argtypes = [P, I]
        L.vflb_batch_get_tile.argtypes = [P]
        L.vflb_batch_get_tile.restype = I
        L.vflb_batch_set_active.argtypes = [P, I, I]
        L.vflb_batch_is_active.argtypes = [P, I]
        L.vflb_batch_is_active.restype = I
        L.vflb_batch_step.argtypes = [P, I64]
        L.vflb_batch_reduce.argtypes = [P, ctypes.POINTER(D)]
        L.vflb_batch_run_until.argtypes = [P, D, I64, ctypes.POINTER(I64), ctypes.POINTER(I64),
                                           ctypes.POINTER(D), ctypes.POINTER(I)]
        L.vflb_batch_autotune.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(I)]
        L.vflb_mlp_create.argtypes = [ctypes.POINTER(MlpCfg), P, ctypes.POINTER(P)]
        L.vflb_mlp_query_buffers.argtypes = [P, ctypes.POINTER(SZ)]
        L.vflb_mlp_bind_buffers.argtypes = [P, ctypes.POINTER(P)]
        L.vflb_mlp_param_count.argtypes = [P]
        L.vflb_mlp_param_count.restype = SZ
        L.vflb_mlp_init.argtypes = [P, ctypes.c_uint64]
        L.vflb_mlp_set_params.argtypes = [P, P, SZ]
        L.vflb_mlp_get_params.argtypes = [P, P, SZ]
        L.vflb_mlp_forward.argtypes = [P, P, P, I64]
        L.vflb_mlp_grad.argtypes = [P, P, P, I64, P, ctypes.POINTER(D)]
        L.vflb_mlp_train_step.argtypes = [P, P, P, I64, ctypes.c_float, ctypes.POINTER(D)]
        L.vflb_mlp_train.argtypes = [P, P, P, I64, I64, I64, ctypes.c_float, ctypes.c_uint64,
                                     I64, ctypes.POINTER(D)]
        L.vflb_init_from_mlp.argtypes = [P, P, ctypes.POINTER(D), D, D, I64, I]
        L.vflb_settle.argtypes = [P, P, I64, I]
        L.vflb_settle.restype = I
        L.vflb_mlp_destroy.argtypes = [P]
        L.vflb_mlp_destroy.restype = None
        L.vflb_mlp_last_error.argtypes = [P]
        L.vflb_mlp_last_error.restype = ctypes.c_char_p
        for name in ("vflb_mlp_create", "vflb_mlp_query_buffers", "vflb_mlp_bind_buffers",
                     "vflb_mlp_init", "vflb_mlp_set_params", "vflb_mlp_get_params",
                     "vflb_mlp_forward", "vflb_mlp_grad", "vflb_mlp_train_step", "vflb_mlp_train",
                     "vflb_init_from_mlp"):
            getattr(L, name).restype = I
        L.vflb_batch_destroy.argtypes = [P]
        L.vflb_batch_destroy.restype = None
        L.vflb_batch_last_error.argtypes = [P]
        L.vflb_batch_last_error.restype = ctypes.c_char_p
        for name in ("vflb_batch_create", "vflb_batch_query_buffers", "vflb_batch_bind_buffers",
                     "vflb_batch_set_tile", "vflb_batch_set_active", "vflb_batch_step",
                     "vflb_batch_reduce", "vflb_batch_run_until", "vflb_batch_autotune"):
            getattr(L, name).restype = I
        L.vflb_last_error.argtypes = [P]
        L.vflb_last_error.restype = ctypes.c_char_p
        for name in ("vflb_create", "vflb_create_scheme", "vflb_create_ex", "vflb_set_model",
                     "vflb_query_buffers",
                     "vflb_bind_buffers",
                     "vflb_set_params", "vflb_get_lattice_params", "vflb_set_force",
                     "vflb_set_boundaries", "vflb_set_storage_scale", "vflb_init_fields",
                     "vflb_step", "vflb_reduce", "vflb_reduce_noalloc", "vflb_read", "vflb_state_size",
                     "vflb_save", "vflb_load", "vflb_set_tile"):
            getattr(L, name).restype = I
        _lib = L
    return _lib


def _check(handle, code):
    if code != OK:
        msg = lib().vflb_last_error(handle)
        raise VflbError(code, msg.decode() if msg else "")


def _bcheck(handle, code):
    if code != OK:
        msg = lib().vflb_batch_last_error(handle)
        raise VflbError(code, msg.decode() if msg else "")


def _mcheck(handle, code):
    if code != OK:
        msg = lib().vflb_mlp_last_error(handle)
        raise VflbError(code, msg.decode() if msg else "")


def stream_copy(src, dst, stream, kind=0):
    """Device copy of src into dst (torch tensors of equal byte size) on the
    given torch stream, by the library's probe kernels: kind 0 non-temporal
    16-byte accesses, 1 plain 16-byte, 2 plain 4-byte, 3 16-byte LDS-DMA
    loads."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    _check(None, lib().vflb_copy_probe(ctypes.c_void_p(src.data_ptr()),
                                       ctypes.c_void_p(dst.data_ptr()), nbytes, kind,
                                       ctypes.c_void_p(stream.cuda_stream)))


class Sim:
    """One lattice: ``Sim(lattice, nx, ny, nz, storage, scheme=...)``.

    ``stream`` is a ``torch.cuda.Stream`` (a default-priority side stream is
    created when omitted); the library enqueues every kernel on it.
    ``scheme`` is "fluctuating" (the paper's method, default) or
    "stress_divergence" (the comparison scheme, D2Q9 FP32/FP64);
    ``inplace=True`` keeps one population buffer (AA streaming, D2Q9
    FP32/FP64).
    """

    def __init__(self, lattice, nx, ny, nz=1, storage="f32", device="cuda:0",
                 stream=None, _handle=None, scheme="fluctuating", inplace=False):
        import torch
        self.torch = torch
        self.D = 2 if lattice in (2, "d2q9", "D2Q9") else 3
        self.nx, self.ny = int(nx), int(ny)
        self.nz = int(nz) if self.D == 3 else 1
        self.N = self.nx * self.ny * self.nz
        self.Q = 9 if self.D == 2 else 19
        self.NC = 3 if self.D == 2 else 6
        self.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        if _handle is not None:  # an instance of a Batch: the batch owns handle and buffers
            self._h = None
            self._view = ctypes.c_void_p(_handle)
            return
        self.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
        h = ctypes.c_void_p()
        self.inplace = bool(inplace)
        _check(None, lib().vflb_create_ex(self.D, self.nx, self.ny, self.nz, self.storage,
                                          self.scheme, OPT_INPLACE if self.inplace else 0,
                                          ctypes.c_void_p(self.stream.cuda_stream),
                                          ctypes.byref(h)))
        self._h = h
        sizes = (ctypes.c_size_t * NBUF)()
        _check(self._h, lib().vflb_query_buffers(self._h, sizes))
        self.buffers = [torch.empty(int(b), dtype=torch.uint8, device=self.device)
                        for b in sizes]
        ptrs = (ctypes.c_void_p * NBUF)(*[b.data_ptr() for b in self.buffers])
        _check(self._h, lib().vflb_bind_buffers(self._h, ptrs))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.vflb_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h if self._h is not None else self._view

    # ---------------------------------------------------------- set-up
    def set_params(self, Re, Wi, beta, U0, L, lam=0.0, tau_h=0.0):
        p = Params(Re, Wi, beta, U0, L, lam, tau_h)
        _check(self.handle, lib().vflb_set_params(self.handle, ctypes.byref(p)))

    def lattice_params(self):
        lp = LatticeParams()
        _check(self.handle, lib().vflb_get_lattice_params(self.handle, ctypes.byref(lp)))
        return dict(nu_s=lp.nu_s, nu_p=lp.nu_p, tau_f=lp.tau_f, tau_h=lp.tau_h,
                    lam=lp.lam, eta_p=lp.eta_p)

    def set_force(self, kind, amp=(0.0, 0.0, 0.0), omega=0.0):
        a = (ctypes.c_double * 3)(*(list(amp) + [0.0] * (3 - len(amp))))
        _check(self.handle, lib().vflb_set_force(self.handle, int(kind), a, float(omega)))

    def set_boundaries(self, walls):
        w = list(walls) + [0] * (3 - len(walls))
        k = (ctypes.c_int * 3)(*[int(x) for x in w])
        _check(self.handle, lib().vflb_set_boundaries(self.handle, k))

    def set_model(self, model, param=0.0):
        """Constitutive model MODEL_* with its parameter (Giesekus alpha,
        PTT eps); Oldroyd-B by default."""
        _check(self.handle, lib().vflb_set_model(self.handle, int(model), float(param)))

    def set_storage_scale(self, log2_f, log2_h):
        _check(self.handle, lib().vflb_set_storage_scale(self.handle, int(log2_f), int(log2_h)))

    def set_tile(self, tile_y):
        _check(self.handle, lib().vflb_set_tile(self.handle, int(tile_y)))

    def _dev_field(self, a, ncomp):
        """Node-major [N, ncomp] host/torch array -> component-major FP64
        device tensor (or None)."""
        if a is None:
            return None
        t = self.torch.as_tensor(np.asarray(a, dtype=np.float64) if not
                                 isinstance(a, self.torch.Tensor) else a,
                                 dtype=self.torch.float64)
        t = t.reshape(self.N, ncomp).t().contiguous().to(self.device)
        return t

    def init_fields_device(self, u=None, tau=None, p=None):
        """Initial state from component-major FP64 device tensors
        u [D, N], tau [NC, N], p [N] (None = zero)."""
        for t in (u, tau, p):
            assert t is None or (t.is_cuda and t.dtype == self.torch.float64 and t.is_contiguous())
        self.torch.cuda.current_stream(self.device).synchronize()
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        _check(self.handle, lib().vflb_init_fields(self.handle, ptr(u), ptr(tau), ptr(p)))
        self.stream.synchronize()

    def init_fields(self, u=None, tau=None, p=None):
        tu = self._dev_field(u, self.D)
        tt = self._dev_field(tau, self.NC)
        tp = self._dev_field(p, 1)
        self.torch.cuda.current_stream(self.device).synchronize()
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        with self.torch.cuda.stream(self.stream):
            _check(self.handle, lib().vflb_init_fields(self.handle, ptr(tu), ptr(tt), ptr(tp)))
        self.stream.synchronize()
        self._keep = (tu, tt, tp)

    # ------------------------------------------------------------ run
    def step(self, n=1):
        _check(self.handle, lib().vflb_step(self.handle, int(n)))

    @property
    def t(self):
        return lib().vflb_time(self.handle)

    def synchronize(self):
        self.stream.synchronize()

    def reduce(self, allow_unstable=False, noalloc=False):
        """FP64 reductions (vflb_reduce; vflb_reduce_noalloc with
        noalloc=True, which keeps its partial sums in the library's static
        device array instead of the work buffer)."""
        out = (ctypes.c_double * 14)()
        fn = lib().vflb_reduce_noalloc if noalloc else lib().vflb_reduce
        rc = fn(self.handle, out)
        if rc != OK and not (allow_unstable and rc == EUNSTABLE):
            _check(self.handle, rc)
        o = list(out)
        return dict(R=o[0], M=o[1], P=o[2:2 + self.D], KE=o[5], PE=o[6],
                    nonfinite=o[7], A_sum=o[8:8 + self.NC], status=rc)

    def read_device(self, field):
        """Field as a component-major FP64 device tensor [ncomp, N]."""
        ncomp = {FIELD_U: self.D, FIELD_P: 1, FIELD_RHO: 1, FIELD_A: self.NC,
                 FIELD_TAU: self.NC, FIELD_F: self.Q, FIELD_H: self.NC * self.Q,
                 FIELD_CHI_PREV: self.NC, FIELD_U_PREV: self.D}[field]
        out = self.torch.empty(ncomp * self.N, dtype=self.torch.float64,
                               device=self.device)
        _check(self.handle, lib().vflb_read(self.handle, int(field),
                                        ctypes.c_void_p(out.data_ptr()), out.numel()))
        return out.view(ncomp, self.N)

    def read(self, field):
        """Field as a node-major numpy array [N, ncomp] (FP64)."""
        t = self.read_device(field)
        self.stream.synchronize()
        a = t.cpu().numpy().T.copy()
        if field == FIELD_H:
            a = a.reshape(self.N, self.NC, self.Q)
        return a

    def _ncomp(self, field):
        return {FIELD_U: self.D, FIELD_P: 1, FIELD_RHO: 1, FIELD_A: self.NC,
                FIELD_TAU: self.NC, FIELD_F: self.Q, FIELD_H: self.NC * self.Q,
                FIELD_CHI_PREV: self.NC, FIELD_U_PREV: self.D}[field]

    def read_box(self, field, lo, size):
        """Field on a box of nodes (origin lo, extent size; x fastest) as a
        node-major numpy array [box nodes, ncomp] (FP64)."""
        lo3 = (ctypes.c_int * 3)(*(list(lo) + [0] * (3 - len(lo))))
        sz3 = (ctypes.c_int * 3)(*(list(size) + [1] * (3 - len(size))))
        nb = int(np.prod(list(sz3)))
        ncomp = self._ncomp(field)
        out = self.torch.empty(ncomp * nb, dtype=self.torch.float64, device=self.device)
        _check(self.handle, lib().vflb_read_box(self.handle, int(field), lo3, sz3,
                                                ctypes.c_void_p(out.data_ptr()), out.numel()))
        self.stream.synchronize()
        a = out.view(ncomp, nb).cpu().numpy().T.copy()
        if field == FIELD_H:
            a = a.reshape(nb, self.NC, self.Q)
        return a

    def moments(self):
        return dict(u=self.read(FIELD_U), p=self.read(FIELD_P)[:, 0],
                    A=self.read(FIELD_A), tau=self.read(FIELD_TAU))

    def state(self):
        """Pre-collision populations and the auxiliary state, node-major."""
        return dict(f=self.read(FIELD_F), h=self.read(FIELD_H),
                    chi_prev=self.read(FIELD_CHI_PREV), u_prev=self.read(FIELD_U_PREV),
                    t=self.t)

    # ----------------------------------------------------- checkpoint
    def save(self):
        n = ctypes.c_size_t()
        _check(self.handle, lib().vflb_state_size(self.handle, ctypes.byref(n)))
        blob = self.torch.empty(n.value, dtype=self.torch.uint8, device=self.device)
        _check(self.handle, lib().vflb_save(self.handle, ctypes.c_void_p(blob.data_ptr()), n.value))
        return blob

    def init_from_mlp(self, mlp, extra, u_scale, tau_scale, settle_steps=0,
                      settle_flags=SETTLE_A):
        """Start from the network's prediction at every node (inputs
        (x/nx, y/ny, *extra)), then settle_steps settling steps; the network
        must use this simulation's stream."""
        e = (ctypes.c_double * 3)(*[float(v) for v in extra])
        _mcheck(mlp._h, lib().vflb_init_from_mlp(self.handle, mlp._h, e, float(u_scale),
                                                  float(tau_scale), int(settle_steps),
                                                  int(settle_flags)))

    def settle(self, u, tau, nsteps, flags=3):
        """Settling steps towards node-major fields u [N, 2], tau [N, 3]."""
        t = np.concatenate([np.asarray(u, np.float64).T.ravel(),
                            np.asarray(tau, np.float64).T.ravel()]).astype(np.float32)
        dt = self.torch.as_tensor(t, device=self.device)
        self.torch.cuda.current_stream(self.device).synchronize()
        _check(self.handle, lib().vflb_settle(self.handle, ctypes.c_void_p(dt.data_ptr()),
                                              int(nsteps), int(flags)))
        self.stream.synchronize()

    def load(self, blob):
        _check(self.handle, lib().vflb_load(self.handle, ctypes.c_void_p(blob.data_ptr()),
                                        blob.numel()))


class Batch:
    """An ensemble of D2Q9 lattices stepped together:
    ``Batch([(nx, ny), ...], storage)``.  ``batch[i]`` is a :class:`Sim`
    handle of instance i for set-up, initialisation and read-back;
    stepping and reductions go through the batch."""

    def __init__(self, dims, storage="f32", device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.n = len(dims)
        self.dims = [(int(d[0]), int(d[1])) for d in dims]
        self.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        flat = (ctypes.c_int * (3 * self.n))(*[v for d in self.dims for v in (d[0], d[1], 1)])
        h = ctypes.c_void_p()
        _bcheck(None, lib().vflb_batch_create(D2Q9, self.n, flat, self.storage,
                                              ctypes.c_void_p(self.stream.cuda_stream),
                                              ctypes.byref(h)))
        self._h = h
        sizes = (ctypes.c_size_t * NBUF)()
        _bcheck(self._h, lib().vflb_batch_query_buffers(self._h, sizes))
        self.buffers = [torch.empty(int(b), dtype=torch.uint8, device=self.device)
                        for b in sizes]
        ptrs = (ctypes.c_void_p * NBUF)(*[b.data_ptr() for b in self.buffers])
        _bcheck(self._h, lib().vflb_batch_bind_buffers(self._h, ptrs))
        self.instances = []
        for i, (nx, ny) in enumerate(self.dims):
            hv = lib().vflb_batch_instance(self._h, i)
            view = Sim(2, nx, ny, 1, self.storage, device, self.stream, _handle=hv)
            view._batch = self  # the batch owns the handle: keep it alive
            self.instances.append(view)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.vflb_batch_destroy(h)
            self._h = None

    def __len__(self):
        return self.n

    def __getitem__(self, i):
        return self.instances[i]

    def set_tile(self, tile_y):
        _bcheck(self._h, lib().vflb_batch_set_tile(self._h, int(tile_y)))

    @property
    def tile(self):
        return lib().vflb_batch_get_tile(self._h)

    def set_active(self, i, active):
        _bcheck(self._h, lib().vflb_batch_set_active(self._h, int(i), 1 if active else 0))

    def is_active(self, i):
        return bool(lib().vflb_batch_is_active(self._h, int(i)))

    def step(self, n=1):
        _bcheck(self._h, lib().vflb_batch_step(self._h, int(n)))

    def synchronize(self):
        self.stream.synchronize()

    def reduce(self):
        """[n, 14] array, one vflb_reduce row per instance."""
        out = (ctypes.c_double * (14 * self.n))()
        _bcheck(self._h, lib().vflb_batch_reduce(self._h, out))
        return np.array(out[:], dtype=np.float64).reshape(self.n, 14)

    def run_until(self, tol, check_every, max_steps):
        ms = (ctypes.c_int64 * self.n)(*[int(m) for m in np.broadcast_to(max_steps, (self.n,))])
        steps = (ctypes.c_int64 * self.n)()
        res = (ctypes.c_double * self.n)()
        st = (ctypes.c_int * self.n)()
        _bcheck(self._h, lib().vflb_batch_run_until(self._h, float(tol), int(check_every), ms,
                                                     steps, res, st))
        return (np.array(steps[:], dtype=np.int64), np.array(res[:], dtype=np.float64),
                np.array(st[:], dtype=np.int32))

    def autotune(self, cache_path=None):
        ty = ctypes.c_int()
        path = cache_path.encode() if cache_path else None
        _bcheck(self._h, lib().vflb_batch_autotune(self._h, path, ctypes.byref(ty)))
        return ty.value


class Mlp:
    """The warm-start network: ``Mlp(in_dim=5, n_freq=128, width=256,
    hidden=3, out_dim=5, max_batch=16384, sigma=4.0, stream=...)``."""

    def __init__(self, in_dim=5, n_freq=128, width=256, hidden=3, out_dim=5, max_batch=16384,
                 sigma=4.0, device="cuda:0", stream=None, seed=None):
        import torch
        self.torch = torch
        self.cfg = dict(in_dim=in_dim, n_freq=n_freq, width=width, hidden=hidden,
                        out_dim=out_dim, max_batch=max_batch, sigma=sigma)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        c = MlpCfg(in_dim, n_freq, width, hidden, out_dim, max_batch, sigma)
        h = ctypes.c_void_p()
        _mcheck(None, lib().vflb_mlp_create(ctypes.byref(c), ctypes.c_void_p(self.stream.cuda_stream),
                                            ctypes.byref(h)))
        self._h = h
        sizes = (ctypes.c_size_t * 2)()
        _mcheck(self._h, lib().vflb_mlp_query_buffers(self._h, sizes))
        self.buffers = [torch.empty(int(b), dtype=torch.uint8, device=self.device) for b in sizes]
        ptrs = (ctypes.c_void_p * 2)(*[b.data_ptr() for b in self.buffers])
        _mcheck(self._h, lib().vflb_mlp_bind_buffers(self._h, ptrs))
        self.nparams = lib().vflb_mlp_param_count(self._h)
        if seed is not None:
            self.init(seed)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.vflb_mlp_destroy(h)
            self._h = None

    def init(self, seed):
        _mcheck(self._h, lib().vflb_mlp_init(self._h, int(seed)))

    def get_params(self):
        a = np.empty(self.nparams, dtype=np.float32)
        _mcheck(self._h, lib().vflb_mlp_get_params(self._h, a.ctypes.data_as(ctypes.c_void_p),
                                                   self.nparams))
        return a

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        assert a.size == self.nparams
        _mcheck(self._h, lib().vflb_mlp_set_params(self._h, a.ctypes.data_as(ctypes.c_void_p),
                                                   self.nparams))

    def _dev(self, a, width):
        t = self.torch.as_tensor(a, dtype=self.torch.float32, device=self.device)
        return t.reshape(-1, width).contiguous()

    def forward(self, x):
        """Outputs [n, out_dim] (device tensor) for inputs x [n, in_dim]."""
        tx = self._dev(x, self.cfg["in_dim"])
        y = self.torch.empty(tx.shape[0], self.cfg["out_dim"], dtype=self.torch.float32,
                             device=self.device)
        self.torch.cuda.current_stream(self.device).synchronize()
        _mcheck(self._h, lib().vflb_mlp_forward(self._h, ctypes.c_void_p(tx.data_ptr()),
                                                ctypes.c_void_p(y.data_ptr()), tx.shape[0]))
        self.stream.synchronize()
        return y

    def grad(self, x, t):
        tx, tt = self._dev(x, self.cfg["in_dim"]), self._dev(t, self.cfg["out_dim"])
        g = np.empty(self.nparams, dtype=np.float32)
        loss = ctypes.c_double()
        self.torch.cuda.current_stream(self.device).synchronize()
        _mcheck(self._h, lib().vflb_mlp_grad(self._h, ctypes.c_void_p(tx.data_ptr()),
                                             ctypes.c_void_p(tt.data_ptr()), tx.shape[0],
                                             g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss)))
        return loss.value, g

    def train(self, X_dev, T_dev, rows, iters, lr, seed=0, log_every=0):
        """vflb_mlp_train on device tensors X [n, in_dim], T [n, out_dim]
        (random minibatches, cosine rate, target standardisation folded
        into the output layer); returns the logged losses."""
        n_log = (iters - 1) // log_every + 2 if log_every > 0 and iters > 0 else 0
        losses = (ctypes.c_double * max(n_log, 1))()
        self.torch.cuda.current_stream(self.device).synchronize()
        _mcheck(self._h, lib().vflb_mlp_train(self._h, ctypes.c_void_p(X_dev.data_ptr()),
                                              ctypes.c_void_p(T_dev.data_ptr()),
                                              int(X_dev.shape[0]), int(rows), int(iters),
                                              float(lr), int(seed) & ((1 << 64) - 1),
                                              int(log_every), losses))
        if not n_log:
            return []
        steps = list(range(0, iters, log_every))
        if (iters - 1) % log_every:
            steps.append(iters - 1)
        return [(k, losses[j]) for j, k in enumerate(steps)]

    def train_step(self, x_dev, t_dev, lr, want_loss=True):
        """One Adam step on device tensors x [n, in_dim], t [n, out_dim]."""
        loss = ctypes.c_double()
        _mcheck(self._h, lib().vflb_mlp_train_step(self._h, ctypes.c_void_p(x_dev.data_ptr()),
                                                   ctypes.c_void_p(t_dev.data_ptr()),
                                                   x_dev.shape[0], float(lr),
                                                   ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None
