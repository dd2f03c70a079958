// vflb.hip -- host side of libvflb: the C ABI declared in include/vflb.h,
// buffer plans, launches of the fused step, read-back, reductions,
// checkpoints and HIP-graph replay of the step loop.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/vflb.h"
#include "kernels.h"
#include "step2d.h"
#include "step3d.h"

using namespace vflb;

namespace {

constexpr int kRedBlocksMax = 1024;
constexpr int kGraphSteps = 64;  // steps per captured graph (even: ping-pong parity)
constexpr double kPi = 3.14159265358979323846;

thread_local std::string g_create_error;

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

struct vflb_sim {
  int D = 2, Q = 9, NC = 3;
  int nx = 1, ny = 1, nz = 1;
  size_t N = 1;
  int storage = VFLB_F32;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  void* buf[VFLB_NBUF] = {};
  size_t bytes[VFLB_NBUF] = {};
  bool bound = false;
  bool have_params = false;
  vflb_params prm{};
  vflb_lattice_params lp{};
  int fkind = VFLB_FORCE_NONE;
  double famp[3] = {0, 0, 0};
  double omega = 0.0;
  int walls = 0;
  int log2_sf = 0, log2_sh = 0;
  int64_t t = 0;
  int cur = 0;  // buffer index (0/1) holding the current populations
  bool inited = false;
  bool snap_valid = false;
  int tile_y = 0;
  size_t off_tab = 0, off_part = 0, off_res = 0, off_hdr = 0;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  std::string err;

  size_t store_bytes() const {
    return storage == VFLB_F64 ? 8 : (storage == VFLB_F32 ? 4 : 2);
  }
  size_t arith_bytes() const { return storage == VFLB_F64 ? 8 : 4; }
};

namespace {

vflb_status fail(vflb_sim* s, vflb_status code, const char* fmt, ...) {
  char msg[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(msg, sizeof msg, fmt, ap);
  va_end(ap);
  if (s)
    s->err = msg;
  else
    g_create_error = msg;
  return code;
}

#define HIP_TRY(s, call)                                                   \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess)                                                  \
      return fail((s), VFLB_EDEVICE, "%s failed: %s", #call,               \
                  hipGetErrorString(e_));                                  \
  } while (0)

void drop_graphs(vflb_sim* s) {
  for (int k = 0; k < 2; ++k) {
    if (s->gexec[k]) (void)hipGraphExecDestroy(s->gexec[k]);
    s->gexec[k] = nullptr;
  }
}

// D3Q19: 32 x tile_y node columns, tile_y 4 (two workgroups per CU) or 8
int tile_y_3d(const vflb_sim* s) { return s->tile_y == 8 ? 8 : 4; }

int default_tile_y(const vflb_sim* s) {
  if (s->tile_y > 0) return s->tile_y;
  // measured on MI355X (8192 x 1024 channel): 64 x 16 tiles for FP32/FP64,
  // 64 x 8 for 16-bit storage
  return (s->storage == VFLB_F16S || s->storage == VFLB_BF16S) ? 8 : 16;
}

template <class R>
Phys<R> phys_of(const vflb_sim* s) {
  Phys<R> P;
  const vflb_lattice_params& l = s->lp;
  P.tau_f = (R)l.tau_f;
  P.inv_tau_f = (R)(1.0 / l.tau_f);
  P.k_f = (R)(1.0 - 0.5 / l.tau_f);
  P.inv_tau_h = (R)(1.0 / l.tau_h);
  P.k_h3 = (R)(3.0 * (1.0 - 0.5 / l.tau_h));
  P.inv_lam = (R)(1.0 / l.lambda);
  P.eta_over_lam = (R)(l.eta_p / l.lambda);
  return P;
}

template <class R>
ForceArgs<R> force_of(const vflb_sim* s, int64_t t) {
  ForceArgs<R> fa;
  fa.kind = s->fkind;
  fa.F0[0] = fa.F0[1] = fa.F0[2] = 0;
  fa.amp[0] = (R)s->famp[0];
  fa.amp[1] = (R)s->famp[1];
  fa.tab = reinterpret_cast<const R*>(static_cast<char*>(s->buf[VFLB_BUF_WORK]) + s->off_tab);
  if (s->fkind == VFLB_FORCE_CONST) {
    for (int a = 0; a < s->D; ++a) fa.F0[a] = (R)s->famp[a];
  } else if (s->fkind == VFLB_FORCE_COS_T) {
    for (int a = 0; a < s->D; ++a) fa.F0[a] = (R)(s->famp[a] * std::cos(s->omega * (double)t));
  }
  return fa;
}

Geo geo_of(const vflb_sim* s) {
  Geo g;
  g.nx = s->nx;
  g.ny = s->ny;
  g.nz = s->nz;
  g.walls = s->walls;
  g.N = s->N;
  return g;
}

int grid1d(const vflb_sim* s, int block) {
  size_t b = (s->N + block - 1) / block;
  if (b > (size_t)kRedBlocksMax) b = kRedBlocksMax;
  return (int)b;
}

// ----------------------------------------------------------- templated ops
template <int D, class S>
vflb_status launch_step(vflb_sim* s, int64_t t, hipStream_t st, int parity) {
  using R = typename StoreT<S>::R;
  StepArgs<S> a;
  a.pin = static_cast<const S*>(s->buf[VFLB_BUF_POP0 + parity]);
  a.pout = static_cast<S*>(s->buf[VFLB_BUF_POP0 + (parity ^ 1)]);
  a.aux = static_cast<R*>(s->buf[VFLB_BUF_AUX]);
  a.g = geo_of(s);
  a.P = phys_of<R>(s);
  a.F = force_of<R>(s, t);
  a.sf = (R)std::ldexp(1.0, s->log2_sf);
  a.inv_sf = (R)std::ldexp(1.0, -s->log2_sf);
  a.sh = (R)std::ldexp(1.0, s->log2_sh);
  a.inv_sh = (R)std::ldexp(1.0, -s->log2_sh);
  if (s->storage != VFLB_F16S) a.sf = a.inv_sf = a.sh = a.inv_sh = (R)1;
  a.first = (t == 0);
  if constexpr (D == 2) {
    const int ty = default_tile_y(s);
    const int ntx = (s->nx + 63) / 64, nty = (s->ny + ty - 1) / ty;
    const dim3 grid((unsigned)(ntx * nty));
    switch (ty) {
      case 4:
        hipLaunchKernelGGL((step2d_kernel<S, 4>), grid, dim3(64, 4), 0, st, a, ntx, nty);
        break;
      case 16:
        hipLaunchKernelGGL((step2d_kernel<S, 16>), grid, dim3(64, 16), 0, st, a, ntx, nty);
        break;
      default:
        hipLaunchKernelGGL((step2d_kernel<S, 8>), grid, dim3(64, 8), 0, st, a, ntx, nty);
        break;
    }
  } else {
    constexpr int ZC = 32;
    const int ty = tile_y_3d(s);
    const int ntx = (s->nx + 31) / 32, nty = (s->ny + ty - 1) / ty;
    const int nzc = (s->nz + ZC - 1) / ZC;
    const dim3 grid((unsigned)(ntx * nty * nzc));
    if (ty == 8) {
      if (s->walls)
        hipLaunchKernelGGL((step3d_kernel<S, 8, ZC, true>), grid, dim3(64, 8), 0, st, a, ntx, nty);
      else
        hipLaunchKernelGGL((step3d_kernel<S, 8, ZC, false>), grid, dim3(64, 8), 0, st, a, ntx, nty);
    } else {
      if (s->walls)
        hipLaunchKernelGGL((step3d_kernel<S, 4, ZC, true>), grid, dim3(64, 4), 0, st, a, ntx, nty);
      else
        hipLaunchKernelGGL((step3d_kernel<S, 4, ZC, false>), grid, dim3(64, 4), 0, st, a, ntx, nty);
    }
  }
  HIP_TRY(s, hipGetLastError());
  return VFLB_OK;
}

template <int D, class S>
vflb_status launch_init(vflb_sim* s, const double* u, const double* tau,
                        const double* p) {
  using R = typename StoreT<S>::R;
  const double loe = s->lp.eta_p > 0.0 ? s->lp.lambda / s->lp.eta_p : 0.0;
  R sf = (R)1, sh = (R)1;
  if (s->storage == VFLB_F16S) {
    sf = (R)std::ldexp(1.0, s->log2_sf);
    sh = (R)std::ldexp(1.0, s->log2_sh);
  }
  hipLaunchKernelGGL((init_kernel<D, S>), dim3(grid1d(s, 256)), dim3(256), 0,
                     s->stream, static_cast<S*>(s->buf[VFLB_BUF_POP0]),
                     static_cast<R*>(s->buf[VFLB_BUF_AUX]), geo_of(s), u, tau, p,
                     loe, sf, sh);
  HIP_TRY(s, hipGetLastError());
  return VFLB_OK;
}

template <int D, class S>
vflb_status launch_moments(vflb_sim* s, int field, double* out) {
  using R = typename StoreT<S>::R;
  R isf = (R)1, ish = (R)1;
  if (s->storage == VFLB_F16S) {
    isf = (R)std::ldexp(1.0, -s->log2_sf);
    ish = (R)std::ldexp(1.0, -s->log2_sh);
  }
  hipLaunchKernelGGL((moments_kernel<D, S>), dim3(grid1d(s, 256)), dim3(256), 0,
                     s->stream, static_cast<const S*>(s->buf[VFLB_BUF_POP0 + s->cur]),
                     geo_of(s),
                     phys_of<R>(s), force_of<R>(s, s->t), isf, ish, field, out);
  HIP_TRY(s, hipGetLastError());
  return VFLB_OK;
}

template <int D, class S>
vflb_status launch_reduce(vflb_sim* s, double* dev_res) {
  using R = typename StoreT<S>::R;
  R isf = (R)1, ish = (R)1;
  if (s->storage == VFLB_F16S) {
    isf = (R)std::ldexp(1.0, -s->log2_sf);
    ish = (R)std::ldexp(1.0, -s->log2_sh);
  }
  const int nb = grid1d(s, 256);
  double* part = reinterpret_cast<double*>(static_cast<char*>(s->buf[VFLB_BUF_WORK]) + s->off_part);
  hipLaunchKernelGGL((reduce_kernel<D, S>), dim3(nb), dim3(256), 0, s->stream,
                     static_cast<const S*>(s->buf[VFLB_BUF_POP0 + s->cur]),
                     static_cast<R*>(s->buf[VFLB_BUF_SNAP]), s->snap_valid ? 1 : 0,
                     geo_of(s), phys_of<R>(s), force_of<R>(s, s->t), isf, ish, part);
  HIP_TRY(s, hipGetLastError());
  hipLaunchKernelGGL(reduce_finish_kernel, dim3(1), dim3(64), 0, s->stream, part, nb,
                     dev_res);
  HIP_TRY(s, hipGetLastError());
  return VFLB_OK;
}

// dispatch on (lattice, storage)
template <template <int, class> class Op, class... A>
vflb_status dispatch(vflb_sim* s, A... args) {
  if (s->D == 2) {
    switch (s->storage) {
      case VFLB_F64: return Op<2, double>::run(s, args...);
      case VFLB_F32: return Op<2, float>::run(s, args...);
      case VFLB_F16S: return Op<2, _Float16>::run(s, args...);
      default: return Op<2, bf16_t>::run(s, args...);
    }
  }
  switch (s->storage) {
    case VFLB_F64: return Op<3, double>::run(s, args...);
    case VFLB_F32: return Op<3, float>::run(s, args...);
    case VFLB_F16S: return Op<3, _Float16>::run(s, args...);
    default: return Op<3, bf16_t>::run(s, args...);
  }
}

template <int D, class S> struct StepOp {
  static vflb_status run(vflb_sim* s, int64_t t, hipStream_t st, int parity) {
    return launch_step<D, S>(s, t, st, parity);
  }
};
template <int D, class S> struct InitOp {
  static vflb_status run(vflb_sim* s, const double* u, const double* tau, const double* p) {
    return launch_init<D, S>(s, u, tau, p);
  }
};
template <int D, class S> struct MomOp {
  static vflb_status run(vflb_sim* s, int field, double* out) {
    return launch_moments<D, S>(s, field, out);
  }
};
template <int D, class S> struct RedOp {
  static vflb_status run(vflb_sim* s, double* res) { return launch_reduce<D, S>(s, res); }
};

vflb_status need_ready(vflb_sim* s) {
  if (!s) return VFLB_EINVAL;
  if (!s->bound) return fail(s, VFLB_ESTATE, "device buffers are not bound");
  if (!s->have_params) return fail(s, VFLB_ESTATE, "parameters are not set");
  return VFLB_OK;
}

// Capture kGraphSteps steps starting from buffer parity `parity` into an
// executable graph (the steps depend on t only through t == 0 and the
// COS_T force, both excluded by the caller).
vflb_status build_graph(vflb_sim* s, int parity) {
  HIP_TRY(s, hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
  vflb_status rc = VFLB_OK;
  for (int k = 0; k < kGraphSteps && rc == VFLB_OK; ++k)
    rc = dispatch<StepOp>(s, (int64_t)1 + k, s->cap_stream, parity ^ (k & 1));
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(s->cap_stream, &graph);
  if (rc != VFLB_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return fail(s, VFLB_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&s->gexec[parity], graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    s->gexec[parity] = nullptr;
    return fail(s, VFLB_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
  }
  return VFLB_OK;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

vflb_status vflb_create(int lattice, int nx, int ny, int nz, int storage,
                        void* hip_stream, vflb_sim** out) {
  if (!out) return fail(nullptr, VFLB_EINVAL, "out is NULL");
  *out = nullptr;
  if (lattice != VFLB_D2Q9 && lattice != VFLB_D3Q19)
    return fail(nullptr, VFLB_EINVAL, "unknown lattice %d", lattice);
  if (storage < VFLB_F64 || storage > VFLB_BF16S)
    return fail(nullptr, VFLB_EINVAL, "unknown storage %d", storage);
  if (lattice == VFLB_D2Q9) nz = 1;
  if (nx < 1 || ny < 1 || nz < 1)
    return fail(nullptr, VFLB_EINVAL, "bad size %d x %d x %d", nx, ny, nz);
  const size_t N = (size_t)nx * ny * nz;
  if (N > ((size_t)1 << 34)) return fail(nullptr, VFLB_EINVAL, "lattice too large");
  // the D3Q19 step addresses the two planes of an opposite pair (2N tuples) with
  // 32-bit byte offsets, which must stay below 4 GiB
  const int d3_log2_max = storage == VFLB_F64 ? 26 : (storage == VFLB_F32 ? 27 : 28);
  if (lattice == VFLB_D3Q19 && N > ((size_t)1 << d3_log2_max))
    return fail(nullptr, VFLB_EINVAL, "D3Q19 lattice of %zu nodes exceeds 2^%d for this storage",
                N, d3_log2_max);
  vflb_sim* s = new vflb_sim();
  s->D = lattice;
  s->Q = lattice == VFLB_D2Q9 ? 9 : 19;
  s->NC = lattice == VFLB_D2Q9 ? 3 : 6;
  s->nx = nx;
  s->ny = ny;
  s->nz = nz;
  s->N = N;
  s->storage = storage;
  s->stream = static_cast<hipStream_t>(hip_stream);
  const size_t sb = s->store_bytes(), ab = s->arith_bytes();
  const size_t words =
      lattice == VFLB_D2Q9 ? Pops<2, float>::words(N) : Pops<3, float>::words(N);
  s->bytes[VFLB_BUF_POP0] = s->bytes[VFLB_BUF_POP1] = align256(sb * words);
  s->bytes[VFLB_BUF_AUX] = align256(ab * (s->NC + s->D) * N);
  s->bytes[VFLB_BUF_SNAP] = align256(ab * (s->NC + s->D) * N);
  s->off_tab = 0;
  s->off_part = align256(ab * 2 * ((size_t)nx + ny));
  s->off_res = s->off_part + align256(sizeof(double) * NRED * kRedBlocksMax);
  s->off_hdr = s->off_res + align256(sizeof(double) * NRED);
  s->bytes[VFLB_BUF_WORK] = s->off_hdr + 256;
  if (hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    delete s;
    return fail(nullptr, VFLB_EDEVICE, "hipStreamCreate failed");
  }
  *out = s;
  return VFLB_OK;
}

vflb_status vflb_query_buffers(const vflb_sim* s, size_t bytes[VFLB_NBUF]) {
  if (!s || !bytes) return VFLB_EINVAL;
  for (int k = 0; k < VFLB_NBUF; ++k) bytes[k] = s->bytes[k];
  return VFLB_OK;
}

vflb_status vflb_bind_buffers(vflb_sim* s, void* const dev_ptrs[VFLB_NBUF]) {
  if (!s || !dev_ptrs) return VFLB_EINVAL;
  for (int k = 0; k < VFLB_NBUF; ++k)
    if (!dev_ptrs[k]) return fail(s, VFLB_EINVAL, "buffer %d is NULL", k);
  for (int k = 0; k < VFLB_NBUF; ++k) s->buf[k] = dev_ptrs[k];
  s->bound = true;
  s->inited = false;
  drop_graphs(s);
  return VFLB_OK;
}

vflb_status vflb_set_params(vflb_sim* s, const vflb_params* p) {
  if (!s || !p) return VFLB_EINVAL;
  if (!(p->Re > 0) || !(p->U0 > 0) || !(p->L > 0))
    return fail(s, VFLB_EINVAL, "Re, U0 and L must be positive");
  if (!(p->beta > 0) || !(p->beta <= 1))
    return fail(s, VFLB_EINVAL, "beta must lie in (0, 1]");
  vflb_lattice_params l;
  const double nu = p->U0 * p->L / p->Re;
  l.nu_s = p->beta * nu;
  l.nu_p = (1.0 - p->beta) * nu;
  l.tau_f = l.nu_s * 3.0 + 0.5;
  l.tau_h = p->tau_h > 0 ? p->tau_h : 0.501;
  l.lambda = p->lambda > 0 ? p->lambda : p->Wi * p->L / p->U0;
  l.eta_p = l.nu_p;
  if (!(l.tau_f > 0.5)) return fail(s, VFLB_EINVAL, "tau_f = %g must exceed 1/2", l.tau_f);
  if (!(l.tau_h > 0.5)) return fail(s, VFLB_EINVAL, "tau_h = %g must exceed 1/2", l.tau_h);
  if (!(l.lambda > 0) || !std::isfinite(l.lambda))
    return fail(s, VFLB_EINVAL, "lambda = %g must be positive", l.lambda);
  s->prm = *p;
  s->lp = l;
  s->have_params = true;
  // FP16 scales: populations of f are O(U0); shifted h are O(1) at most
  // moderate stretch.  Keep 2^14 * typical magnitude below the FP16 range.
  int ef;
  std::frexp(p->U0, &ef);
  s->log2_sf = 8 - ef;
  if (s->log2_sf < 0) s->log2_sf = 0;
  if (s->log2_sf > 24) s->log2_sf = 24;
  s->log2_sh = 6;
  drop_graphs(s);
  return VFLB_OK;
}

vflb_status vflb_get_lattice_params(const vflb_sim* s, vflb_lattice_params* out) {
  if (!s || !out) return VFLB_EINVAL;
  if (!s->have_params) return VFLB_ESTATE;
  *out = s->lp;
  return VFLB_OK;
}

vflb_status vflb_set_force(vflb_sim* s, int kind, const double amp[3], double omega) {
  if (!s) return VFLB_EINVAL;
  if (kind < VFLB_FORCE_NONE || kind > VFLB_FORCE_COS_T)
    return fail(s, VFLB_EINVAL, "unknown force kind %d", kind);
  if (kind != VFLB_FORCE_NONE && !amp) return fail(s, VFLB_EINVAL, "amp is NULL");
  if (!s->bound) return fail(s, VFLB_ESTATE, "bind buffers before setting the force");
  double a[3] = {0, 0, 0};
  if (amp)
    for (int k = 0; k < 3; ++k) a[k] = amp[k];
  if (kind == VFLB_FORCE_FOUR_ROLL) {
    // tables sin/cos(2 pi i / n) in the arithmetic type, computed in FP64
    const size_t nt = 2 * ((size_t)s->nx + s->ny);
    char* host = static_cast<char*>(malloc(nt * s->arith_bytes()));
    if (!host) return fail(s, VFLB_ENOMEM, "host allocation failed");
    for (size_t k = 0; k < nt; ++k) {
      double v;
      if (k < (size_t)s->nx) v = std::sin(2.0 * kPi * (double)k / s->nx);
      else if (k < 2 * (size_t)s->nx) v = std::cos(2.0 * kPi * (double)(k - s->nx) / s->nx);
      else if (k < 2 * (size_t)s->nx + s->ny) v = std::sin(2.0 * kPi * (double)(k - 2 * s->nx) / s->ny);
      else v = std::cos(2.0 * kPi * (double)(k - 2 * s->nx - s->ny) / s->ny);
      if (s->storage == VFLB_F64) reinterpret_cast<double*>(host)[k] = v;
      else reinterpret_cast<float*>(host)[k] = (float)v;
    }
    hipError_t e = hipMemcpyAsync(static_cast<char*>(s->buf[VFLB_BUF_WORK]) + s->off_tab, host,
                                  nt * s->arith_bytes(), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    free(host);
    if (e != hipSuccess) return fail(s, VFLB_EDEVICE, "table upload failed: %s", hipGetErrorString(e));
  }
  s->fkind = kind;
  for (int k = 0; k < 3; ++k) s->famp[k] = a[k];
  s->omega = omega;
  drop_graphs(s);
  return VFLB_OK;
}

vflb_status vflb_set_boundaries(vflb_sim* s, const int kind_per_axis[3]) {
  if (!s || !kind_per_axis) return VFLB_EINVAL;
  const int n[3] = {s->nx, s->ny, s->nz};
  int w = 0;
  for (int a = 0; a < s->D; ++a) {
    const int k = kind_per_axis[a];
    if (k != VFLB_PERIODIC && k != VFLB_WALLS)
      return fail(s, VFLB_EINVAL, "unknown boundary kind %d on axis %d", k, a);
    if (k == VFLB_WALLS) {
      if (n[a] < 2) return fail(s, VFLB_EINVAL, "a wall axis needs at least 2 nodes");
      w |= 1 << a;
    }
  }
  s->walls = w;
  drop_graphs(s);
  return VFLB_OK;
}

vflb_status vflb_set_storage_scale(vflb_sim* s, int log2_f, int log2_h) {
  if (!s) return VFLB_EINVAL;
  if (log2_f < -40 || log2_f > 40 || log2_h < -40 || log2_h > 40)
    return fail(s, VFLB_EINVAL, "scale exponent out of range");
  s->log2_sf = log2_f;
  s->log2_sh = log2_h;
  drop_graphs(s);
  return VFLB_OK;
}

vflb_status vflb_set_tile(vflb_sim* s, int tile_y) {
  if (!s) return VFLB_EINVAL;
  if (tile_y != 0 && tile_y != 4 && tile_y != 8 && (tile_y != 16 || s->D == 3))
    return fail(s, VFLB_EINVAL, "tile_y must be 0, 4, 8 or 16 (D2Q9), 0, 4 or 8 (D3Q19)");
  s->tile_y = tile_y;
  drop_graphs(s);
  return VFLB_OK;
}

vflb_status vflb_init_fields(vflb_sim* s, const double* u, const double* tau,
                             const double* p) {
  vflb_status rc = need_ready(s);
  if (rc != VFLB_OK) return rc;
  s->cur = 0;
  rc = dispatch<InitOp>(s, u, tau, p);
  if (rc != VFLB_OK) return rc;
  s->t = 0;
  s->inited = true;
  s->snap_valid = false;
  return VFLB_OK;
}

vflb_status vflb_step(vflb_sim* s, int64_t nsteps) {
  vflb_status rc = need_ready(s);
  if (rc != VFLB_OK) return rc;
  if (!s->inited) return fail(s, VFLB_ESTATE, "initialise the fields before stepping");
  if (nsteps < 0) return fail(s, VFLB_EINVAL, "nsteps < 0");
  while (nsteps > 0) {
    const bool graphable = s->t > 0 && s->fkind != VFLB_FORCE_COS_T &&
                           nsteps >= kGraphSteps && s->stream != nullptr;
    if (graphable) {
      if (!s->gexec[s->cur]) {
        rc = build_graph(s, s->cur);
        if (rc != VFLB_OK) return rc;
      }
      HIP_TRY(s, hipGraphLaunch(s->gexec[s->cur], s->stream));
      s->t += kGraphSteps;  // even: parity unchanged
      nsteps -= kGraphSteps;
      continue;
    }
    rc = dispatch<StepOp>(s, s->t, s->stream, s->cur);
    if (rc != VFLB_OK) return rc;
    s->cur ^= 1;
    s->t += 1;
    nsteps -= 1;
  }
  return VFLB_OK;
}

int64_t vflb_time(const vflb_sim* s) { return s ? s->t : -1; }

vflb_status vflb_reduce(vflb_sim* s, double out[14]) {
  vflb_status rc = need_ready(s);
  if (rc != VFLB_OK) return rc;
  if (!out) return fail(s, VFLB_EINVAL, "out is NULL");
  if (!s->inited) return fail(s, VFLB_ESTATE, "initialise the fields first");
  double* dres = reinterpret_cast<double*>(static_cast<char*>(s->buf[VFLB_BUF_WORK]) + s->off_res);
  rc = dispatch<RedOp>(s, dres);
  if (rc != VFLB_OK) return rc;
  double r[NRED];
  HIP_TRY(s, hipMemcpyAsync(r, dres, sizeof r, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  const bool had = s->snap_valid;
  s->snap_valid = true;
  double R = INFINITY;
  if (had) {
    const double ru = r[1] > 0 ? std::sqrt(r[0] / r[1]) : (r[0] > 0 ? INFINITY : 0.0);
    const double rt = r[3] > 0 ? std::sqrt(r[2] / r[3]) : (r[2] > 0 ? INFINITY : 0.0);
    R = ru > rt ? ru : rt;
  }
  out[0] = R;
  out[1] = r[4];
  out[2] = r[5];
  out[3] = r[6];
  out[4] = r[7];
  out[5] = r[8] / (double)s->N;
  out[6] = r[9] / (double)s->N;
  out[7] = r[10];
  for (int c = 0; c < 6; ++c) out[8 + c] = c < s->NC ? r[11 + c] : 0.0;
  if (r[10] > 0) return fail(s, VFLB_EUNSTABLE, "%.0f nodes hold non-finite moments", r[10]);
  return VFLB_OK;
}

vflb_status vflb_read(vflb_sim* s, int field, double* dev_dst, size_t n) {
  vflb_status rc = need_ready(s);
  if (rc != VFLB_OK) return rc;
  if (!s->inited) return fail(s, VFLB_ESTATE, "initialise the fields first");
  if (!dev_dst) return fail(s, VFLB_EINVAL, "destination is NULL");
  size_t need;
  switch (field) {
    case VFLB_FIELD_U: need = (size_t)s->D * s->N; break;
    case VFLB_FIELD_P:
    case VFLB_FIELD_RHO: need = s->N; break;
    case VFLB_FIELD_A:
    case VFLB_FIELD_TAU: need = (size_t)s->NC * s->N; break;
    case VFLB_FIELD_F: need = (size_t)s->Q * s->N; break;
    case VFLB_FIELD_H: need = (size_t)s->NC * s->Q * s->N; break;
    case VFLB_FIELD_CHI_PREV: need = (size_t)s->NC * s->N; break;
    case VFLB_FIELD_U_PREV: need = (size_t)s->D * s->N; break;
    default: return fail(s, VFLB_EINVAL, "unknown field %d", field);
  }
  if (n != need) return fail(s, VFLB_EINVAL, "field %d holds %zu values, not %zu", field, need, n);
  if (field == VFLB_FIELD_CHI_PREV || field == VFLB_FIELD_U_PREV) {
    const int nb = grid1d(s, 256);
    const Geo g = geo_of(s);
    void* aux = s->buf[VFLB_BUF_AUX];
    if (s->D == 2 && s->storage == VFLB_F64)
      hipLaunchKernelGGL((aux_read_kernel<2, double>), dim3(nb), dim3(256), 0, s->stream,
                         static_cast<const double*>(aux), g, field, dev_dst);
    else if (s->D == 2)
      hipLaunchKernelGGL((aux_read_kernel<2, float>), dim3(nb), dim3(256), 0, s->stream,
                         static_cast<const float*>(aux), g, field, dev_dst);
    else if (s->storage == VFLB_F64)
      hipLaunchKernelGGL((aux_read_kernel<3, double>), dim3(nb), dim3(256), 0, s->stream,
                         static_cast<const double*>(aux), g, field, dev_dst);
    else
      hipLaunchKernelGGL((aux_read_kernel<3, float>), dim3(nb), dim3(256), 0, s->stream,
                         static_cast<const float*>(aux), g, field, dev_dst);
    HIP_TRY(s, hipGetLastError());
    return VFLB_OK;
  }
  return dispatch<MomOp>(s, field, dev_dst);
}

// checkpoint blob: 256-byte header, then f, h, aux of the current state
struct CkptHeader {
  uint64_t magic;
  int32_t D, nx, ny, nz, storage, pad;
  int64_t t;
};
static const uint64_t kCkptMagic = 0x76666c62636b7074ull;

vflb_status vflb_state_size(const vflb_sim* s, size_t* bytes) {
  if (!s || !bytes) return VFLB_EINVAL;
  *bytes = 256 + s->bytes[VFLB_BUF_POP0] + s->bytes[VFLB_BUF_AUX];
  return VFLB_OK;
}

vflb_status vflb_save(vflb_sim* s, void* blob, size_t n) {
  vflb_status rc = need_ready(s);
  if (rc != VFLB_OK) return rc;
  if (!s->inited) return fail(s, VFLB_ESTATE, "nothing to save");
  size_t need;
  vflb_state_size(s, &need);
  if (!blob || n < need) return fail(s, VFLB_EINVAL, "blob must hold %zu bytes", need);
  CkptHeader h{};
  h.magic = kCkptMagic;
  h.D = s->D; h.nx = s->nx; h.ny = s->ny; h.nz = s->nz; h.storage = s->storage;
  h.t = s->t;
  char* b = static_cast<char*>(blob);
  HIP_TRY(s, hipMemcpyAsync(b, &h, sizeof h, hipMemcpyHostToDevice, s->stream));
  size_t off = 256;
  HIP_TRY(s, hipMemcpyAsync(b + off, s->buf[VFLB_BUF_POP0 + s->cur], s->bytes[VFLB_BUF_POP0],
                            hipMemcpyDeviceToDevice, s->stream));
  off += s->bytes[VFLB_BUF_POP0];
  HIP_TRY(s, hipMemcpyAsync(b + off, s->buf[VFLB_BUF_AUX], s->bytes[VFLB_BUF_AUX],
                            hipMemcpyDeviceToDevice, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  return VFLB_OK;
}

vflb_status vflb_load(vflb_sim* s, const void* blob, size_t n) {
  vflb_status rc = need_ready(s);
  if (rc != VFLB_OK) return rc;
  size_t need;
  vflb_state_size(s, &need);
  if (!blob || n < need) return fail(s, VFLB_EINVAL, "blob must hold %zu bytes", need);
  CkptHeader h{};
  const char* b = static_cast<const char*>(blob);
  HIP_TRY(s, hipMemcpyAsync(&h, b, sizeof h, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  if (h.magic != kCkptMagic || h.D != s->D || h.nx != s->nx || h.ny != s->ny ||
      h.nz != s->nz || h.storage != s->storage)
    return fail(s, VFLB_EINVAL, "checkpoint does not match this simulation");
  size_t off = 256;
  HIP_TRY(s, hipMemcpyAsync(s->buf[VFLB_BUF_POP0], b + off, s->bytes[VFLB_BUF_POP0],
                            hipMemcpyDeviceToDevice, s->stream));
  off += s->bytes[VFLB_BUF_POP0];
  HIP_TRY(s, hipMemcpyAsync(s->buf[VFLB_BUF_AUX], b + off, s->bytes[VFLB_BUF_AUX],
                            hipMemcpyDeviceToDevice, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  s->cur = 0;
  s->t = h.t;
  s->inited = true;
  s->snap_valid = false;
  return VFLB_OK;
}

vflb_status vflb_stream_copy(const void* src, void* dst, size_t nbytes, void* hip_stream) {
  if (!src || !dst || nbytes % 16 != 0 || ((uintptr_t)src | (uintptr_t)dst) % 16 != 0)
    return fail(nullptr, VFLB_EINVAL, "stream copy needs 16-byte aligned pointers and sizes");
  const size_t n = nbytes / 16;
  if (n == 0) return VFLB_OK;
  const size_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffffu) return fail(nullptr, VFLB_EINVAL, "copy too large");
  hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     static_cast<hipStream_t>(hip_stream), static_cast<const v4u32*>(src),
                     static_cast<v4u32*>(dst), n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(nullptr, VFLB_EDEVICE, "copy launch failed: %s", hipGetErrorString(e));
  return VFLB_OK;
}

void vflb_destroy(vflb_sim* s) {
  if (!s) return;
  drop_graphs(s);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  delete s;
}

const char* vflb_last_error(const vflb_sim* s) {
  if (!s) return g_create_error.c_str();
  return s->err.c_str();
}

}  // extern "C"
