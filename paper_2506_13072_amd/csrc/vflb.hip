// vflb.hip -- host side of libvflb: the C ABI declared in include/vflb.h,
// buffer plans, launches of the fused step, read-back, reductions,
// checkpoints and HIP-graph replay of the step loop.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#include <algorithm>
#include <mutex>

#include "../../include/vflb.h"
#include "kernels.h"
#include "step2d.h"
#include "step3d.h"
#include "aa3d.h"
#include "probe.h"
#include "internal.h"

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
  bool is_view = false;  // an instance of a batch: buffers and stepping belong to the batch
  const float* clamp = nullptr;  // settling targets while vflb::internal::sim_settle runs
  int clamp_flags = 0;
  int scheme = VFLB_SCHEME_FLUCTUATING;
  bool inplace = false;  // one population buffer, AA streaming
  int model = VFLB_MODEL_OLDROYD_B;
  double mparam = 0.0;
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
// (AA: in place, FP32; U the velocity pass's u(t) [3][N])
template <class S, int TY, int ZC, bool WALLS, bool DIV = false, bool AA = false>
void launch_step3d(dim3 grid, hipStream_t st, const StepArgs<S>& a, int ntx, int nty, bool any_full,
                   bool any_ragged, const typename StoreT<S>::R* U = nullptr) {
  if (any_full)
    hipLaunchKernelGGL((step3d_kernel<S, TY, ZC, WALLS, true, DIV, AA>), grid, dim3(64, TY), 0, st,
                       a, ntx, nty, U);
  if (any_ragged)
    hipLaunchKernelGGL((step3d_kernel<S, TY, ZC, WALLS, false, DIV, AA>), grid, dim3(64, TY), 0,
                       st, a, ntx, nty, U);
}

// in-place D3Q19 step: the z-march with the in-place index maps, in 32 x 4
// columns, after the velocity pass has written u(t) to U
template <class S>
vflb_status launch_aa3_march(const vflb_sim* s, hipStream_t st, const StepArgs<S>& a,
                             const typename StoreT<S>::R* U) {
  constexpr int ZC = kStep3dChunk, TY = 4;
  const int ntx = (s->nx + 31) / 32, nty = (s->ny + TY - 1) / TY;
  const int nzc = (s->nz + ZC - 1) / ZC;
  const dim3 grid((unsigned)(ntx * nty * nzc));
  const bool any_full = s->nx >= 32 && s->ny >= TY;
  const bool any_ragged = s->nx % 32 != 0 || s->ny % TY != 0;
  const bool div = s->scheme == VFLB_SCHEME_STRESS_DIVERGENCE;
  if (s->walls) {
    if (div)
      launch_step3d<S, TY, ZC, true, true, true>(grid, st, a, ntx, nty, any_full, any_ragged, U);
    else
      launch_step3d<S, TY, ZC, true, false, true>(grid, st, a, ntx, nty, any_full, any_ragged, U);
  } else {
    if (div)
      launch_step3d<S, TY, ZC, false, true, true>(grid, st, a, ntx, nty, any_full, any_ragged, U);
    else
      launch_step3d<S, TY, ZC, false, false, true>(grid, st, a, ntx, nty, any_full, any_ragged, U);
  }
  return VFLB_OK;
}

// D3Q19 launches for tile height TY: walls or not, the stress-divergence
// scheme or not (FP32 / FP64 storage only)
template <class S, int TY, int ZC>
void launch_step3d_ty(const vflb_sim* s, dim3 grid, hipStream_t st, const StepArgs<S>& a,
                      int ntx, int nty, bool any_full, bool any_ragged) {
  if constexpr (!StoreT<S>::kAnchored) {
    if (s->scheme == VFLB_SCHEME_STRESS_DIVERGENCE) {
      if (s->walls)
        launch_step3d<S, TY, ZC, true, true>(grid, st, a, ntx, nty, any_full, any_ragged);
      else
        launch_step3d<S, TY, ZC, false, true>(grid, st, a, ntx, nty, any_full, any_ragged);
      return;
    }
  }
  if (s->walls)
    launch_step3d<S, TY, ZC, true>(grid, st, a, ntx, nty, any_full, any_ragged);
  else
    launch_step3d<S, TY, ZC, false>(grid, st, a, ntx, nty, any_full, any_ragged);
}

int tile_y_3d(const vflb_sim* s) { return s->tile_y == 8 ? 8 : 4; }

int default_tile_y(const vflb_sim* s) {
  if (s->tile_y > 0) return s->tile_y;
  // measured on MI355X (8192 x 1024 channel): 64 x 16 tiles for FP32 and
  // 64 x 8 for 16-bit storage and for FP64, whose state does not fit the
  // 128 VGPRs a 1024-lane workgroup leaves (1.13 against 2.50 ms per step)
  return s->storage == VFLB_F32 ? 16 : 8;
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
  P.fluct = s->scheme == VFLB_SCHEME_FLUCTUATING ? (R)1 : (R)0;
  P.model = s->model;
  P.mparam = (R)s->mparam;
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
  // stress-divergence scheme: div tau_p [D][N] after chi, u, tau_p in AUX
  fa.div = s->scheme == VFLB_SCHEME_STRESS_DIVERGENCE
               ? static_cast<const R*>(s->buf[VFLB_BUF_AUX]) + (size_t)(2 * s->NC + s->D) * s->N
               : nullptr;
  fa.div_d = fa.div ? s->D : 0;
  if (s->fkind == VFLB_FORCE_CONST) {
    for (int a = 0; a < s->D; ++a) fa.F0[a] = (R)s->famp[a];
  } else if (s->fkind == VFLB_FORCE_COS_T) {
    for (int a = 0; a < s->D; ++a) fa.F0[a] = (R)(s->famp[a] * std::cos(s->omega * (double)t));
  }
  return fa;
}

// geometry of the state at time level t (the in-place layout alternates)
Geo geo_of(const vflb_sim* s, int64_t t) {
  Geo g;
  g.nx = s->nx;
  g.ny = s->ny;
  g.nz = s->nz;
  g.walls = s->walls;
  g.N = s->N;
  g.aa = s->inplace ? ((t & 1) ? 2 : 1) : 0;
  return g;
}

Geo geo_of(const vflb_sim* s) { return geo_of(s, s->t); }

// AUX layout: chi(t-1) [NC][N], u(t-1) [D][N]; stress-divergence scheme:
// tau_p [NC][N], div tau_p [D][N]; in-place streaming: u(t) [D][N]
size_t aux_taup_words(const vflb_sim* s) { return (size_t)(s->NC + s->D) * s->N; }
size_t aux_u_words(const vflb_sim* s) {
  return aux_taup_words(s) +
         (s->scheme == VFLB_SCHEME_STRESS_DIVERGENCE ? (size_t)(s->NC + s->D) * s->N : 0);
}

int grid1d(const vflb_sim* s, int block) {
  size_t b = (s->N + block - 1) / block;
  if (b > (size_t)kRedBlocksMax) b = kRedBlocksMax;
  return (int)b;
}

// ----------------------------------------------------------- templated ops
// arguments of one step from buffer parity `parity` at time level t
template <class S>
StepArgs<S> make_step_args(const vflb_sim* s, int64_t t, int parity) {
  using R = typename StoreT<S>::R;
  StepArgs<S> a;
  if (s->inplace) parity = 0;  // one buffer, read and written in place
  a.pin = static_cast<const S*>(s->buf[VFLB_BUF_POP0 + parity]);
  a.pout = static_cast<S*>(s->buf[VFLB_BUF_POP0 + (s->inplace ? 0 : parity ^ 1)]);
  a.aux = static_cast<R*>(s->buf[VFLB_BUF_AUX]);
  a.g = geo_of(s, t);
  a.P = phys_of<R>(s);
  a.F = force_of<R>(s, t);
  a.sf = (R)std::ldexp(1.0, s->log2_sf);
  a.inv_sf = (R)std::ldexp(1.0, -s->log2_sf);
  a.sh = (R)std::ldexp(1.0, s->log2_sh);
  a.inv_sh = (R)std::ldexp(1.0, -s->log2_sh);
  if (s->storage != VFLB_F16S) a.sf = a.inv_sf = a.sh = a.inv_sh = (R)1;
  a.first = (t == 0);
  a.clamp = nullptr;
  a.clamp_flags = 0;
  return a;
}

// stress-divergence scheme: tau_p and div tau_p of the populations in the
// buffer of parity `parity` (the state the next kernels read)
template <class S>
vflb_status launch_divergence(vflb_sim* s, int64_t t, hipStream_t st, int parity) {
  using R = typename StoreT<S>::R;
  if constexpr (StoreT<S>::kAnchored) {
    return fail(s, VFLB_EINVAL, "the stress-divergence scheme needs FP32 or FP64 storage");
  } else {
    const S* pin = static_cast<const S*>(s->buf[VFLB_BUF_POP0 + (s->inplace ? 0 : parity)]);
    R* taup = static_cast<R*>(s->buf[VFLB_BUF_AUX]) + aux_taup_words(s);
    R* div = taup + (size_t)s->NC * s->N;
    const int g = grid1d(s, 256);
    const R k = (R)(s->lp.eta_p / s->lp.lambda);
    if (s->D == 2) {
      hipLaunchKernelGGL((taup_kernel<2, S>), dim3(g), dim3(256), 0, st, pin, geo_of(s, t), k,
                         taup);
      hipLaunchKernelGGL((stress_div_kernel<2, R>), dim3(g), dim3(256), 0, st, taup,
                         geo_of(s, t), div);
    } else if constexpr (!StoreT<S>::kPlanar) {
      hipLaunchKernelGGL((taup_kernel<3, S>), dim3(g), dim3(256), 0, st, pin, geo_of(s, t), k,
                         taup);
      hipLaunchKernelGGL((stress_div_kernel<3, R>), dim3(g), dim3(256), 0, st, taup,
                         geo_of(s, t), div);
    }
    HIP_TRY(s, hipGetLastError());
    return VFLB_OK;
  }
}

// the two-buffer step: tiled kernels over the whole lattice
template <int D, class S>
vflb_status launch_tiled(vflb_sim* s, hipStream_t st, StepArgs<S> a) {
  if (D == 2) {
    a.clamp = s->clamp;
    a.clamp_flags = s->clamp_flags;
  }
  if constexpr (D == 2) {
    const int ty = default_tile_y(s);
    const int ntx = (s->nx + 63) / 64, nty = (s->ny + ty - 1) / ty;
    const dim3 grid((unsigned)(ntx * nty));
    if (a.clamp) {  // settling steps: one tile height suffices
      hipLaunchKernelGGL((step2d_kernel<S, 8, true>), dim3(ntx * ((s->ny + 7) / 8)), dim3(64, 8),
                         0, st, a, ntx, (s->ny + 7) / 8);
    } else {
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
    }
  } else {
    constexpr int ZC = kStep3dChunk;
    const int ty = tile_y_3d(s);
    const int ntx = (s->nx + 31) / 32, nty = (s->ny + ty - 1) / ty;
    const int nzc = (s->nz + ZC - 1) / ZC;
    const dim3 grid((unsigned)(ntx * nty * nzc));
    // full tiles and ragged tiles run as two launches of one kernel
    const bool any_full = s->nx >= 32 && s->ny >= ty;
    const bool any_ragged = s->nx % 32 != 0 || s->ny % ty != 0;
    bool eight = ty == 8;
    if constexpr (!StoreT<S>::kAnchored) {  // anchored 16-bit: 32 x 4 only (LDS)
      if (eight) launch_step3d_ty<S, 8, ZC>(s, grid, st, a, ntx, nty, any_full, any_ragged);
    } else {
      eight = false;
    }
    if (!eight) launch_step3d_ty<S, 4, ZC>(s, grid, st, a, ntx, nty, any_full, any_ragged);
  }
  HIP_TRY(s, hipGetLastError());
  return VFLB_OK;
}

template <int D, class S>
vflb_status launch_step(vflb_sim* s, int64_t t, hipStream_t st, int parity) {
  if (s->scheme == VFLB_SCHEME_STRESS_DIVERGENCE) {
    vflb_status rc = launch_divergence<S>(s, t, st, parity);
    if (rc != VFLB_OK) return rc;
  }
  StepArgs<S> a = make_step_args<S>(s, t, parity);
  if constexpr (D == 3 && !StoreT<S>::kAnchored) {
    if (s->inplace) {  // in place: same-time velocity, then the step
      using R = typename StoreT<S>::R;
      R* U = static_cast<R*>(s->buf[VFLB_BUF_AUX]) + aux_u_words(s);
      const int nb = (int)std::min<size_t>((s->N + 255) / 256, (size_t)1 << 16);
      hipLaunchKernelGGL((aa3_velocity_kernel<S>), dim3(nb), dim3(256), 0, st, a.pin, a.g, a.F,
                         a.inv_sf, U);
      launch_aa3_march<S>(s, st, a, U);
      HIP_TRY(s, hipGetLastError());
      return VFLB_OK;
    }
  }
  if constexpr (!StoreT<S>::kPlanar) {
    return launch_tiled<D, S>(s, st, a);
  } else {  // in place: same-time velocity, then the step
    using R = typename StoreT<S>::R;
    R* U = static_cast<R*>(s->buf[VFLB_BUF_AUX]) + aux_u_words(s);
    const dim3 grid((s->nx + 255) / 256, s->ny < 65535 ? s->ny : 65535);
    hipLaunchKernelGGL((aa_velocity_kernel<S>), grid, dim3(256), 0, st, a.pin, a.g, a.F, a.inv_sf,
                       U);
    hipLaunchKernelGGL((aa_step_kernel<S>), grid, dim3(256), 0, st, a, (const R*)U);
    HIP_TRY(s, hipGetLastError());
    return VFLB_OK;
  }
}

template <int D, class S, class T>
vflb_status launch_init(vflb_sim* s, const T* u, const T* tau, const T* p) {
  using R = typename StoreT<S>::R;
  const double loe = s->lp.eta_p > 0.0 ? s->lp.lambda / s->lp.eta_p : 0.0;
  R sf = (R)1, sh = (R)1;
  if (s->storage == VFLB_F16S) {
    sf = (R)std::ldexp(1.0, s->log2_sf);
    sh = (R)std::ldexp(1.0, s->log2_sh);
  }
  hipLaunchKernelGGL((init_kernel<D, S, T>), dim3(grid1d(s, 256)), dim3(256), 0,
                     s->stream, static_cast<S*>(s->buf[VFLB_BUF_POP0]),
                     static_cast<R*>(s->buf[VFLB_BUF_AUX]), geo_of(s, 0), u, tau, p,
                     loe, sf, sh);
  HIP_TRY(s, hipGetLastError());
  return VFLB_OK;
}

Box whole_box(const vflb_sim* s) {
  Box b;
  b.lo[0] = b.lo[1] = b.lo[2] = 0;
  b.n[0] = s->nx;
  b.n[1] = s->ny;
  b.n[2] = s->nz;
  b.N = s->N;
  return b;
}

int grid_for(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > (size_t)kRedBlocksMax) b = kRedBlocksMax;
  return (int)(b ? b : 1);
}

template <int D, class S>
vflb_status launch_moments(vflb_sim* s, int field, double* out, const Box& box) {
  using R = typename StoreT<S>::R;
  if (s->scheme == VFLB_SCHEME_STRESS_DIVERGENCE) {  // the force includes div tau_p(t)
    vflb_status rc = launch_divergence<S>(s, s->t, s->stream, s->cur);
    if (rc != VFLB_OK) return rc;
  }
  R isf = (R)1, ish = (R)1;
  if (s->storage == VFLB_F16S) {
    isf = (R)std::ldexp(1.0, -s->log2_sf);
    ish = (R)std::ldexp(1.0, -s->log2_sh);
  }
  hipLaunchKernelGGL((moments_kernel<D, S>), dim3(grid_for(box.N)), dim3(256), 0,
                     s->stream, static_cast<const S*>(s->buf[VFLB_BUF_POP0 + s->cur]),
                     static_cast<const R*>(s->buf[VFLB_BUF_AUX]), geo_of(s), box,
                     phys_of<R>(s), force_of<R>(s, s->t), isf, ish, field, out);
  HIP_TRY(s, hipGetLastError());
  return VFLB_OK;
}

template <int D, class S>
vflb_status launch_reduce(vflb_sim* s, double* part, double* dev_res) {
  using R = typename StoreT<S>::R;
  if (s->scheme == VFLB_SCHEME_STRESS_DIVERGENCE) {
    vflb_status rc = launch_divergence<S>(s, s->t, s->stream, s->cur);
    if (rc != VFLB_OK) return rc;
  }
  R isf = (R)1, ish = (R)1;
  if (s->storage == VFLB_F16S) {
    isf = (R)std::ldexp(1.0, -s->log2_sf);
    ish = (R)std::ldexp(1.0, -s->log2_sh);
  }
  const int nb = grid1d(s, 256);
  hipLaunchKernelGGL((reduce_kernel<D, S>), dim3(nb), dim3(256), 0, s->stream,
                     static_cast<const S*>(s->buf[VFLB_BUF_POP0 + s->cur]),
                     static_cast<const R*>(s->buf[VFLB_BUF_AUX]),
                     static_cast<R*>(s->buf[VFLB_BUF_SNAP]), s->snap_valid ? 1 : 0,
                     geo_of(s), phys_of<R>(s), force_of<R>(s, s->t), isf, ish, part);
  HIP_TRY(s, hipGetLastError());
  hipLaunchKernelGGL(reduce_finish_kernel, dim3(1, NRED), dim3(256), 0, s->stream, part,
                     (const int*)nullptr, nb, dev_res);
  HIP_TRY(s, hipGetLastError());
  return VFLB_OK;
}

// dispatch on (lattice, storage)
template <template <int, class> class Op, class... A>
vflb_status dispatch(vflb_sim* s, A... args) {
  if (s->D == 2) {
    switch (s->storage) {
      case VFLB_F64:
        return s->inplace ? Op<2, Planar<double>>::run(s, args...) : Op<2, double>::run(s, args...);
      case VFLB_F32:
        return s->inplace ? Op<2, Planar<float>>::run(s, args...) : Op<2, float>::run(s, args...);
      case VFLB_F16S: return Op<2, _Float16>::run(s, args...);
      default: return Op<2, bf16_t>::run(s, args...);
    }
  }
  switch (s->storage) {
    case VFLB_F64: return Op<3, double>::run(s, args...);
    case VFLB_F32: return Op<3, float>::run(s, args...);
    case VFLB_F16S: return Op<3, _Float16>::run(s, args...);
    default: return fail(s, VFLB_EINVAL, "no D3Q19 path for storage %d", s->storage);
  }
}

template <int D, class S> struct StepOp {
  static vflb_status run(vflb_sim* s, int64_t t, hipStream_t st, int parity) {
    return launch_step<D, S>(s, t, st, parity);
  }
};
template <int D, class S> struct InitOp {
  template <class T>
  static vflb_status run(vflb_sim* s, const T* u, const T* tau, const T* p) {
    return launch_init<D, S, T>(s, u, tau, p);
  }
};
template <int D, class S> struct MomOp {
  static vflb_status run(vflb_sim* s, int field, double* out, Box box) {
    return launch_moments<D, S>(s, field, out, box);
  }
};
template <int D, class S> struct RedOp {
  static vflb_status run(vflb_sim* s, double* part, double* res) {
    return launch_reduce<D, S>(s, part, res);
  }
};

// The 14 reported values from the NRED sums; marks the snapshot valid.
vflb_status finish_reduce(vflb_sim* s, const double* r, double out[14]) {
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
  // the steps depend on t only through t == 0, the COS_T force (both
  // excluded) and, in place, the parity of t, which `parity` then holds
  const int64_t t0 = s->inplace ? 2 + parity : 1;
  for (int k = 0; k < kGraphSteps && rc == VFLB_OK; ++k)
    rc = dispatch<StepOp>(s, t0 + k, s->cap_stream, parity ^ (k & 1));
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

namespace {

// A lattice and the sizes of its buffers.  A view (an instance of a batch)
// has no capture stream: it is stepped by its batch.
vflb_status sim_new(int lattice, int nx, int ny, int nz, int storage, hipStream_t stream,
                    bool view, vflb_sim** out, int scheme = VFLB_SCHEME_FLUCTUATING,
                    int options = 0) {
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
  // BF16 deviations carry an 8-bit mantissa: on D3Q19 lattices of 16^3
  // they left u and tau 2e-3 .. 7e-3 away from the FP64 iteration, above
  // the 1e-3 accuracy of 16-bit storage that FP16 meets
  if (lattice == VFLB_D3Q19 && storage == VFLB_BF16S)
    return fail(nullptr, VFLB_EINVAL,
                "BF16 storage is not offered on D3Q19 (it misses the 1e-3 accuracy of 16-bit "
                "storage there); use VFLB_F16S");
  if (scheme != VFLB_SCHEME_FLUCTUATING && scheme != VFLB_SCHEME_STRESS_DIVERGENCE)
    return fail(nullptr, VFLB_EINVAL, "unknown scheme %d", scheme);
  if (scheme == VFLB_SCHEME_STRESS_DIVERGENCE && storage != VFLB_F32 && storage != VFLB_F64)
    return fail(nullptr, VFLB_EINVAL,
                "the stress-divergence scheme runs with FP32 or FP64 storage");
  if (options & ~VFLB_OPT_INPLACE) return fail(nullptr, VFLB_EINVAL, "unknown options %#x", options);
  const bool inplace = (options & VFLB_OPT_INPLACE) != 0;
  if (inplace && ((storage != VFLB_F32 && storage != VFLB_F64) || view))
    return fail(nullptr, VFLB_EINVAL,
                "in-place streaming runs on single lattices with FP32 or FP64 storage");
  vflb_sim* s = new vflb_sim();
  s->scheme = scheme;
  s->inplace = inplace;
  s->D = lattice;
  s->Q = lattice == VFLB_D2Q9 ? 9 : 19;
  s->NC = lattice == VFLB_D2Q9 ? 3 : 6;
  s->nx = nx;
  s->ny = ny;
  s->nz = nz;
  s->N = N;
  s->storage = storage;
  s->stream = stream;
  s->is_view = view;
  const size_t sb = s->store_bytes(), ab = s->arith_bytes();
  const size_t words =
      lattice == VFLB_D2Q9 ? Pops<2, float>::words(N) : Pops<3, float>::words(N);
  // anchored 16-bit storage keeps an FP32 anchor per node after the
  // populations of each population buffer (layout.h)
  const bool anchored = storage == VFLB_F16S || storage == VFLB_BF16S;
  s->bytes[VFLB_BUF_POP0] = s->bytes[VFLB_BUF_POP1] = align256(
      anchored ? (lattice == VFLB_D2Q9 ? Anchor2::bytes(N) : Anchor3::bytes(N)) : sb * words);
  if (inplace) s->bytes[VFLB_BUF_POP1] = 256;  // unused
  // AUX: chi(t-1), u(t-1); the stress-divergence scheme adds tau_p [NC][N]
  // and div tau_p [D][N]; in-place streaming u(t) [2][N]
  const size_t u_now = inplace ? (size_t)s->D : 0;
  const size_t div_words = scheme == VFLB_SCHEME_STRESS_DIVERGENCE ? s->NC + s->D : 0;
  s->bytes[VFLB_BUF_AUX] = align256(ab * ((s->NC + s->D) + div_words + u_now) * N);
  s->bytes[VFLB_BUF_SNAP] = align256(ab * (s->NC + s->D) * N);
  s->off_tab = 0;
  s->off_part = align256(ab * 2 * ((size_t)nx + ny));
  s->off_res = s->off_part + align256(sizeof(double) * NRED * kRedBlocksMax);
  s->off_hdr = s->off_res + align256(sizeof(double) * NRED);
  s->bytes[VFLB_BUF_WORK] = s->off_hdr + 256;
  if (!view && hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    delete s;
    return fail(nullptr, VFLB_EDEVICE, "hipStreamCreate failed");
  }
  *out = s;
  return VFLB_OK;
}

}  // namespace

vflb_status vflb_create(int lattice, int nx, int ny, int nz, int storage,
                        void* hip_stream, vflb_sim** out) {
  return sim_new(lattice, nx, ny, nz, storage, static_cast<hipStream_t>(hip_stream), false, out);
}

vflb_status vflb_create_scheme(int lattice, int nx, int ny, int nz, int storage, int scheme,
                               void* hip_stream, vflb_sim** out) {
  return sim_new(lattice, nx, ny, nz, storage, static_cast<hipStream_t>(hip_stream), false, out,
                 scheme);
}

vflb_status vflb_create_ex(int lattice, int nx, int ny, int nz, int storage, int scheme,
                           int options, void* hip_stream, vflb_sim** out) {
  return sim_new(lattice, nx, ny, nz, storage, static_cast<hipStream_t>(hip_stream), false, out,
                 scheme, options);
}

vflb_status vflb_query_buffers(const vflb_sim* s, size_t bytes[VFLB_NBUF]) {
  if (!s || !bytes) return VFLB_EINVAL;
  for (int k = 0; k < VFLB_NBUF; ++k) bytes[k] = s->bytes[k];
  return VFLB_OK;
}

vflb_status vflb_bind_buffers(vflb_sim* s, void* const dev_ptrs[VFLB_NBUF]) {
  if (!s || !dev_ptrs) return VFLB_EINVAL;
  if (s->is_view) return fail(s, VFLB_EINVAL, "a batch instance uses the batch's buffers");
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
  // FP16 scales: anchored storage holds deviations from a reference, the
  // non-equilibrium parts O(U0 k) and below, scaled into FP16's normal range
  int ef;
  std::frexp(p->U0, &ef);
  const int log2_sf = std::min(24, std::max(0, 10 - ef)), log2_sh = 12;
  if (s->storage == VFLB_F16S && s->inited && (log2_sf != s->log2_sf || log2_sh != s->log2_sh))
    return fail(s, VFLB_ESTATE,
                "U0 = %g moves the FP16 storage scale (2^%d -> 2^%d) of initialised fields; "
                "set the parameters before vflb_init_fields",
                p->U0, s->log2_sf, log2_sf);
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
  s->log2_sf = log2_sf;
  s->log2_sh = log2_sh;
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

vflb_status vflb_set_model(vflb_sim* s, int model, double param) {
  if (!s) return VFLB_EINVAL;
  if (model != VFLB_MODEL_OLDROYD_B && model != VFLB_MODEL_GIESEKUS && model != VFLB_MODEL_LPTT &&
      model != VFLB_MODEL_EPTT)
    return fail(s, VFLB_EINVAL, "unknown constitutive model %d", model);
  if (!std::isfinite(param) || param < 0)
    return fail(s, VFLB_EINVAL, "the model parameter must be finite and non-negative");
  if (model == VFLB_MODEL_GIESEKUS && param > 0.5)
    return fail(s, VFLB_EINVAL, "the Giesekus mobility must lie in [0, 1/2]");
  s->model = model;
  s->mparam = model == VFLB_MODEL_OLDROYD_B ? 0.0 : param;
  drop_graphs(s);
  return VFLB_OK;
}

vflb_status vflb_set_storage_scale(vflb_sim* s, int log2_f, int log2_h) {
  if (!s) return VFLB_EINVAL;
  if (log2_f < -40 || log2_f > 40 || log2_h < -40 || log2_h > 40)
    return fail(s, VFLB_EINVAL, "scale exponent out of range");
  // the stored FP16 deviations are in the current scale: changing it under
  // initialised fields would rescale them all by a power of two
  if (s->storage == VFLB_F16S && s->inited && (log2_f != s->log2_sf || log2_h != s->log2_sh))
    return fail(s, VFLB_ESTATE, "the FP16 storage scale is fixed once the fields are initialised");
  s->log2_sf = log2_f;
  s->log2_sh = log2_h;
  drop_graphs(s);
  return VFLB_OK;
}

vflb_status vflb_set_tile(vflb_sim* s, int tile_y) {
  if (!s) return VFLB_EINVAL;
  if (s->is_view) return fail(s, VFLB_EINVAL, "set the tile shape on the batch");
  if (tile_y != 0 && tile_y != 4 && tile_y != 8 && (tile_y != 16 || s->D == 3))
    return fail(s, VFLB_EINVAL, "tile_y must be 0, 4, 8 or 16 (D2Q9), 0, 4 or 8 (D3Q19)");
  if (s->D == 3 && tile_y == 8 && (s->storage == VFLB_F16S || s->storage == VFLB_BF16S))
    return fail(s, VFLB_EINVAL,
                "anchored 16-bit D3Q19 storage runs 32 x 4 tiles (its LDS stages would not fit 8 rows)");
  s->tile_y = tile_y;
  drop_graphs(s);
  return VFLB_OK;
}

vflb_status vflb_init_fields(vflb_sim* s, const double* u, const double* tau,
                             const double* p) {
  vflb_status rc = need_ready(s);
  if (rc != VFLB_OK) return rc;
  s->cur = 0;
  s->t = 0;
  rc = dispatch<InitOp>(s, u, tau, p);
  if (rc != VFLB_OK) return rc;
  s->inited = true;
  s->snap_valid = false;
  return VFLB_OK;
}

vflb_status vflb_step(vflb_sim* s, int64_t nsteps) {
  vflb_status rc = need_ready(s);
  if (rc != VFLB_OK) return rc;
  if (s->is_view) return fail(s, VFLB_ESTATE, "a batch instance is stepped by vflb_batch_step");
  if (!s->inited) return fail(s, VFLB_ESTATE, "initialise the fields before stepping");
  if (nsteps < 0) return fail(s, VFLB_EINVAL, "nsteps < 0");
  while (nsteps > 0) {
    const bool graphable = s->t > 0 && s->fkind != VFLB_FORCE_COS_T &&
                           nsteps >= kGraphSteps && s->stream != nullptr;
    // graphs are kept per parity: of the buffer pair, or in place of t
    const int par = s->inplace ? (int)(s->t & 1) : s->cur;
    if (graphable) {
      if (!s->gexec[par]) {
        rc = build_graph(s, par);
        if (rc != VFLB_OK) return rc;
      }
      HIP_TRY(s, hipGraphLaunch(s->gexec[par], s->stream));
      s->t += kGraphSteps;  // even: parity unchanged
      nsteps -= kGraphSteps;
      continue;
    }
    rc = dispatch<StepOp>(s, s->t, s->stream, s->cur);
    if (rc != VFLB_OK) return rc;
    if (!s->inplace) s->cur ^= 1;
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
  char* work = static_cast<char*>(s->buf[VFLB_BUF_WORK]);
  double* dres = reinterpret_cast<double*>(work + s->off_res);
  rc = dispatch<RedOp>(s, reinterpret_cast<double*>(work + s->off_part), dres);
  if (rc != VFLB_OK) return rc;
  double r[NRED];
  HIP_TRY(s, hipMemcpyAsync(r, dres, sizeof r, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  return finish_reduce(s, r, out);
}

}  // extern "C"

// Reduction scratch of vflb_reduce_noalloc: the per-block partial sums and
// the NRED results, one copy per GPU for the life of the process.  In host
// code `scratch` names a host-side stand-in, never the device memory: the
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kScratchWords = (size_t)NRED * kRedBlocksMax + NRED;
static __device__ __align__(256) double scratch[kScratchWords];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the device of `stream`; looked up once per
// device, with that device current.
vflb_status scratch_address(vflb_sim* s, hipStream_t stream, double** out) {
  int dev = 0;
  if (stream) HIP_TRY(s, hipStreamGetDevice(stream, &dev));
  else HIP_TRY(s, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(s, VFLB_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    int cur = 0;
    HIP_TRY(s, hipGetDevice(&cur));
    if (cur != dev) HIP_TRY(s, hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      return fail(s, VFLB_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return VFLB_OK;
}

}  // namespace

extern "C" {

vflb_status vflb_reduce_noalloc(vflb_sim* s, double out[14]) {
  vflb_status rc = need_ready(s);
  if (rc != VFLB_OK) return rc;
  if (!out) return fail(s, VFLB_EINVAL, "out is NULL");
  if (!s->inited) return fail(s, VFLB_ESTATE, "initialise the fields first");
  const size_t need = (size_t)NRED * grid1d(s, 256) + NRED;
  if (need > kScratchWords)
    return fail(s, VFLB_EINVAL, "reduction needs %zu scratch words, the static buffer holds %zu",
                need, kScratchWords);
  double* sp = nullptr;
  if ((rc = scratch_address(s, s->stream, &sp)) != VFLB_OK) return rc;
  // every partial of [0, grid) is written before the finishing pass reads
  // it, so nothing needs clearing between calls
  double* dres = sp + (size_t)NRED * kRedBlocksMax;
  rc = dispatch<RedOp>(s, sp, dres);
  if (rc != VFLB_OK) return rc;
  double r[NRED];
  HIP_TRY(s, hipMemcpyAsync(r, dres, sizeof r, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  return finish_reduce(s, r, out);
}

namespace {

// values per node of a read-back field (0: unknown field)
size_t field_width(const vflb_sim* s, int field) {
  switch (field) {
    case VFLB_FIELD_U: return (size_t)s->D;
    case VFLB_FIELD_P:
    case VFLB_FIELD_RHO: return 1;
    case VFLB_FIELD_A:
    case VFLB_FIELD_TAU: return (size_t)s->NC;
    case VFLB_FIELD_F: return (size_t)s->Q;
    case VFLB_FIELD_H: return (size_t)s->NC * s->Q;
    case VFLB_FIELD_CHI_PREV: return (size_t)s->NC;
    case VFLB_FIELD_U_PREV: return (size_t)s->D;
    default: return 0;
  }
}

vflb_status read_box(vflb_sim* s, int field, const Box& box, double* dev_dst) {
  if (field == VFLB_FIELD_CHI_PREV || field == VFLB_FIELD_U_PREV) {
    const int nb = grid_for(box.N);
    const Geo g = geo_of(s);
    void* aux = s->buf[VFLB_BUF_AUX];
    if (s->D == 2 && s->storage == VFLB_F64)
      hipLaunchKernelGGL((aux_read_kernel<2, double>), dim3(nb), dim3(256), 0, s->stream,
                         static_cast<const double*>(aux), g, box, field, dev_dst);
    else if (s->D == 2)
      hipLaunchKernelGGL((aux_read_kernel<2, float>), dim3(nb), dim3(256), 0, s->stream,
                         static_cast<const float*>(aux), g, box, field, dev_dst);
    else if (s->storage == VFLB_F64)
      hipLaunchKernelGGL((aux_read_kernel<3, double>), dim3(nb), dim3(256), 0, s->stream,
                         static_cast<const double*>(aux), g, box, field, dev_dst);
    else
      hipLaunchKernelGGL((aux_read_kernel<3, float>), dim3(nb), dim3(256), 0, s->stream,
                         static_cast<const float*>(aux), g, box, field, dev_dst);
    HIP_TRY(s, hipGetLastError());
    return VFLB_OK;
  }
  return dispatch<MomOp>(s, field, dev_dst, box);
}

}  // namespace

vflb_status vflb_read(vflb_sim* s, int field, double* dev_dst, size_t n) {
  vflb_status rc = need_ready(s);
  if (rc != VFLB_OK) return rc;
  if (!s->inited) return fail(s, VFLB_ESTATE, "initialise the fields first");
  if (!dev_dst) return fail(s, VFLB_EINVAL, "destination is NULL");
  const size_t w = field_width(s, field);
  if (!w) return fail(s, VFLB_EINVAL, "unknown field %d", field);
  if (n != w * s->N)
    return fail(s, VFLB_EINVAL, "field %d holds %zu values, not %zu", field, w * s->N, n);
  return read_box(s, field, whole_box(s), dev_dst);
}

vflb_status vflb_read_box(vflb_sim* s, int field, const int lo[3], const int size[3],
                          double* dev_dst, size_t n) {
  vflb_status rc = need_ready(s);
  if (rc != VFLB_OK) return rc;
  if (!s->inited) return fail(s, VFLB_ESTATE, "initialise the fields first");
  if (!dev_dst || !lo || !size) return fail(s, VFLB_EINVAL, "NULL argument");
  const size_t w = field_width(s, field);
  if (!w) return fail(s, VFLB_EINVAL, "unknown field %d", field);
  Box b;
  const int dims[3] = {s->nx, s->ny, s->nz};
  b.N = 1;
  for (int a = 0; a < 3; ++a) {
    const int sz = a < s->D ? size[a] : 1, l = a < s->D ? lo[a] : 0;
    if (sz < 1 || sz > dims[a])
      return fail(s, VFLB_EINVAL, "box extent %d on axis %d outside [1, %d]", sz, a, dims[a]);
    if ((s->walls >> a) & 1) {
      if (l < 0 || l + sz > dims[a])
        return fail(s, VFLB_EINVAL, "box leaves the walls of axis %d", a);
    }
    b.lo[a] = l;
    b.n[a] = sz;
    b.N *= (size_t)sz;
  }
  if (n != w * b.N)
    return fail(s, VFLB_EINVAL, "the box holds %zu values, not %zu", w * b.N, n);
  return read_box(s, field, b, dev_dst);
}

// checkpoint blob: 256-byte header, then f, h, aux of the current state
struct CkptHeader {
  uint64_t magic;
  int32_t D, nx, ny, nz, storage, pad;
  int64_t t;
  int32_t log2_sf, log2_sh;  // FP16 storage scales the populations were written in
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
  h.pad = s->inplace ? 1 : 0;  // in place the layout follows the parity of t
  h.t = s->t;
  h.log2_sf = s->log2_sf;
  h.log2_sh = s->log2_sh;
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
      h.nz != s->nz || h.storage != s->storage || h.pad != (s->inplace ? 1 : 0))
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
  if (s->storage == VFLB_F16S &&
      (h.log2_sf != s->log2_sf || h.log2_sh != s->log2_sh)) {
    // the loaded deviations are in the checkpoint's scale: adopt it
    s->log2_sf = h.log2_sf;
    s->log2_sh = h.log2_sh;
    drop_graphs(s);
  }
  s->inited = true;
  s->snap_valid = false;
  return VFLB_OK;
}

vflb_status vflb_copy_probe(const void* src, void* dst, size_t nbytes, int kind,
                            void* hip_stream) {
  if (kind < 0 || kind > 3) return fail(nullptr, VFLB_EINVAL, "copy kind must be 0..3");
  const size_t unit = kind == 2 ? 4 : 16;
  if (!src || !dst || nbytes % unit != 0 || ((uintptr_t)src | (uintptr_t)dst) % unit != 0)
    return fail(nullptr, VFLB_EINVAL, "copy needs %zu-byte aligned pointers and sizes", unit);
  const size_t n = nbytes / unit;
  if (n == 0) return VFLB_OK;
  const size_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffffu) return fail(nullptr, VFLB_EINVAL, "copy too large");
  const hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const dim3 grid((unsigned)blocks), block(256);
  if (kind == 0)
    hipLaunchKernelGGL(stream_copy_kernel, grid, block, 0, st, static_cast<const v4u32*>(src),
                       static_cast<v4u32*>(dst), n);
  else if (kind == 1)
    hipLaunchKernelGGL(copy_plain16_kernel, grid, block, 0, st, static_cast<const v4u32*>(src),
                       static_cast<v4u32*>(dst), n);
  else if (kind == 2)
    hipLaunchKernelGGL(copy_plain4_kernel, grid, block, 0, st, static_cast<const uint32_t*>(src),
                       static_cast<uint32_t*>(dst), n);
  else
    hipLaunchKernelGGL(copy_lds16_kernel, grid, block, 0, st, static_cast<const v4u32*>(src),
                       static_cast<v4u32*>(dst), n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(nullptr, VFLB_EDEVICE, "copy launch failed: %s", hipGetErrorString(e));
  return VFLB_OK;
}

vflb_status vflb_stream_copy(const void* src, void* dst, size_t nbytes, void* hip_stream) {
  return vflb_copy_probe(src, dst, nbytes, 0, hip_stream);
}

vflb_status vflb_settle(vflb_sim* s, const float* dev_targets, int64_t nsteps, int flags) {
  if (!s) return VFLB_EINVAL;
  if (!dev_targets || nsteps < 0) return fail(s, VFLB_EINVAL, "need targets and nsteps >= 0");
  if (s->is_view && s->t != 0) return fail(s, VFLB_ESTATE, "settle a batch instance right after its initialisation");
  return vflb::internal::sim_settle_f32(s, dev_targets, nsteps, flags);
}

void vflb_destroy(vflb_sim* s) {
  if (!s || s->is_view) return;
  drop_graphs(s);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  delete s;
}

const char* vflb_last_error(const vflb_sim* s) {
  if (!s) return g_create_error.c_str();
  return s->err.c_str();
}


// ================================================================ batches
}  // extern "C"

struct vflb_batch {
  int D = 2, storage = VFLB_F32, n = 0;
  hipStream_t stream = nullptr, cap_stream = nullptr;
  void* buf[VFLB_NBUF] = {};
  size_t bytes[VFLB_NBUF] = {};
  bool bound = false;
  std::vector<vflb_sim*> views;
  std::vector<size_t> off[VFLB_NBUF];  // per-instance byte offsets into the pools
  size_t off_desc = 0, off_tiles = 0, off_part = 0, off_rng = 0, off_res = 0;
  size_t max_tiles = 0;
  std::vector<char> active;
  std::vector<double> last;  // last reduction per instance (14 values)
  int tile_y = 0;            // 0: built-in choice
  // tables of the active set (host copies of what the device holds)
  bool tables_ok = false;
  int tables_ty = 0;
  std::vector<BatchTile> tiles;
  std::vector<int> ranges;  // per active instance: [begin, end) in tiles
  std::vector<int> act;     // active instance ids in table order
  std::vector<char> desc_host, desc_dev;  // descriptor bytes built / last uploaded
  int grid_cap[3] = {0, 0, 0};  // persistent grid per tile height 4, 8, 16
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  std::string err;
};

namespace {

thread_local std::string g_batch_create_error;

vflb_status bfail(vflb_batch* b, vflb_status code, const char* fmt, ...) {
  char msg[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(msg, sizeof msg, fmt, ap);
  va_end(ap);
  if (b)
    b->err = msg;
  else
    g_batch_create_error = msg;
  return code;
}

#define BHIP_TRY(b, call)                                                  \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess)                                                  \
      return bfail((b), VFLB_EDEVICE, "%s failed: %s", #call,              \
                   hipGetErrorString(e_));                                 \
  } while (0)

void bdrop_graphs(vflb_batch* b) {
  for (int k = 0; k < 2; ++k) {
    if (b->gexec[k]) (void)hipGraphExecDestroy(b->gexec[k]);
    b->gexec[k] = nullptr;
  }
}

int batch_ty(const vflb_batch* b) { return b->tile_y ? b->tile_y : 8; }
int ty_slot(int ty) { return ty == 4 ? 0 : (ty == 8 ? 1 : 2); }

size_t desc_size(int storage) {
  switch (storage) {
    case VFLB_F64: return sizeof(BatchInst<double>);
    case VFLB_F32: return sizeof(BatchInst<float>);
    case VFLB_F16S: return sizeof(BatchInst<_Float16>);
    default: return sizeof(BatchInst<bf16_t>);
  }
}

// Tile table of the active instances for tile height ty: per instance its
// 64 x ty tiles in row-major order, instances in index order.
vflb_status build_tables(vflb_batch* b, int ty) {
  b->tiles.clear();
  b->ranges.clear();
  b->act.clear();
  for (int i = 0; i < b->n; ++i) {
    if (!b->active[i]) continue;
    const vflb_sim* v = b->views[i];
    const int ntx = (v->nx + 63) / 64, nty = (v->ny + ty - 1) / ty;
    b->ranges.push_back((int)b->tiles.size());
    for (int yt = 0; yt < nty; ++yt)
      for (int xt = 0; xt < ntx; ++xt) b->tiles.push_back(BatchTile{i, xt * 64, yt * ty, 0});
    b->ranges.push_back((int)b->tiles.size());
    b->act.push_back(i);
  }
  char* w = static_cast<char*>(b->buf[VFLB_BUF_WORK]);
  BHIP_TRY(b, hipStreamSynchronize(b->stream));  // earlier uploads may still read the host copies
  if (!b->tiles.empty())
    BHIP_TRY(b, hipMemcpyAsync(w + b->off_tiles, b->tiles.data(),
                               b->tiles.size() * sizeof(BatchTile), hipMemcpyHostToDevice,
                               b->stream));
  if (!b->ranges.empty())
    BHIP_TRY(b, hipMemcpyAsync(w + b->off_rng, b->ranges.data(), b->ranges.size() * sizeof(int),
                               hipMemcpyHostToDevice, b->stream));
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  b->tables_ok = true;
  b->tables_ty = ty;
  bdrop_graphs(b);
  return VFLB_OK;
}

template <class S>
void fill_desc(vflb_batch* b) {
  using R = typename StoreT<S>::R;
  b->desc_host.assign((size_t)b->n * sizeof(BatchInst<S>), 0);
  BatchInst<S>* d = reinterpret_cast<BatchInst<S>*>(b->desc_host.data());
  for (int i = 0; i < b->n; ++i) {
    const vflb_sim* v = b->views[i];
    d[i].a = make_step_args<S>(v, 1, 0);
    d[i].snap = static_cast<R*>(v->buf[VFLB_BUF_SNAP]);
    d[i].snap_valid = v->snap_valid ? 1 : 0;
  }
}

// (Re)build the per-instance descriptors from the instance views and upload
// them when they changed.
vflb_status sync_desc(vflb_batch* b) {
  switch (b->storage) {
    case VFLB_F64: fill_desc<double>(b); break;
    case VFLB_F32: fill_desc<float>(b); break;
    case VFLB_F16S: fill_desc<_Float16>(b); break;
    default: fill_desc<bf16_t>(b); break;
  }
  if (b->desc_host == b->desc_dev) return VFLB_OK;
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  b->desc_dev = b->desc_host;
  BHIP_TRY(b, hipMemcpyAsync(static_cast<char*>(b->buf[VFLB_BUF_WORK]) + b->off_desc,
                             b->desc_dev.data(), b->desc_dev.size(), hipMemcpyHostToDevice,
                             b->stream));
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  return VFLB_OK;
}

template <class S, int TY>
vflb_status launch_batch_ty(vflb_batch* b, hipStream_t st, int parity, int first) {
  int& cap = b->grid_cap[ty_slot(TY)];
  if (cap == 0) {
    int per_cu = 0, dev = 0, cus = 0;
    BHIP_TRY(b, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch2d_kernel<S, TY>,
                                                             64 * TY, 0));
    BHIP_TRY(b, hipGetDevice(&dev));
    BHIP_TRY(b, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    cap = std::max(1, per_cu) * std::max(1, cus);
  }
  const int ntiles = (int)b->tiles.size();
  const int grid = std::min(ntiles, cap);
  const char* w = static_cast<const char*>(b->buf[VFLB_BUF_WORK]);
  hipLaunchKernelGGL((batch2d_kernel<S, TY>), dim3(grid), dim3(64, TY), 0, st,
                     reinterpret_cast<const BatchInst<S>*>(w + b->off_desc),
                     reinterpret_cast<const BatchTile*>(w + b->off_tiles), ntiles, parity, first);
  BHIP_TRY(b, hipGetLastError());
  return VFLB_OK;
}

template <class S>
vflb_status launch_batch_s(vflb_batch* b, hipStream_t st, int parity, int first) {
  switch (b->tables_ty) {
    case 4: return launch_batch_ty<S, 4>(b, st, parity, first);
    case 16: return launch_batch_ty<S, 16>(b, st, parity, first);
    default: return launch_batch_ty<S, 8>(b, st, parity, first);
  }
}

vflb_status launch_batch(vflb_batch* b, hipStream_t st, int parity, int first) {
  if (b->tiles.empty()) return VFLB_OK;
  switch (b->storage) {
    case VFLB_F64: return launch_batch_s<double>(b, st, parity, first);
    case VFLB_F32: return launch_batch_s<float>(b, st, parity, first);
    case VFLB_F16S: return launch_batch_s<_Float16>(b, st, parity, first);
    default: return launch_batch_s<bf16_t>(b, st, parity, first);
  }
}

vflb_status build_batch_graph(vflb_batch* b, int parity) {
  BHIP_TRY(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  vflb_status rc = VFLB_OK;
  for (int k = 0; k < kGraphSteps && rc == VFLB_OK; ++k)
    rc = launch_batch(b, b->cap_stream, parity ^ (k & 1), 0);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap_stream, &graph);
  if (rc != VFLB_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return bfail(b, VFLB_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&b->gexec[parity], graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    b->gexec[parity] = nullptr;
    return bfail(b, VFLB_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
  }
  return VFLB_OK;
}

// The active instances must share their time level and buffer parity.
vflb_status check_active(vflb_batch* b, int64_t* t, int* cur) {
  if (!b->bound) return bfail(b, VFLB_ESTATE, "device buffers are not bound");
  bool any = false;
  for (int i = 0; i < b->n; ++i) {
    if (!b->active[i]) continue;
    const vflb_sim* v = b->views[i];
    if (!v->have_params) return bfail(b, VFLB_ESTATE, "instance %d has no parameters", i);
    if (!v->inited) return bfail(b, VFLB_ESTATE, "instance %d is not initialised", i);
    if (v->fkind == VFLB_FORCE_COS_T)
      return bfail(b, VFLB_EINVAL, "instance %d: time-periodic forcing is not batched", i);
    if (!any) {
      *t = v->t;
      *cur = v->cur;
      any = true;
    } else if (v->t != *t || v->cur != *cur) {
      return bfail(b, VFLB_ESTATE, "active instances are at different time levels");
    }
  }
  if (!any) {
    *t = 0;
    *cur = 0;
  }
  return VFLB_OK;
}

vflb_status ensure_tables(vflb_batch* b) {
  const int ty = batch_ty(b);
  if (!b->tables_ok || b->tables_ty != ty) return build_tables(b, ty);
  return VFLB_OK;
}

template <class S>
vflb_status launch_batch_reduce_s(vflb_batch* b, int parity) {
  char* w = static_cast<char*>(b->buf[VFLB_BUF_WORK]);
  double* part = reinterpret_cast<double*>(w + b->off_part);
  hipLaunchKernelGGL((batch_reduce_kernel<S>), dim3((unsigned)b->tiles.size()), dim3(256), 0,
                     b->stream, reinterpret_cast<const BatchInst<S>*>(w + b->off_desc),
                     reinterpret_cast<const BatchTile*>(w + b->off_tiles), b->tables_ty, parity,
                     part);
  BHIP_TRY(b, hipGetLastError());
  hipLaunchKernelGGL(reduce_finish_kernel, dim3((unsigned)b->act.size(), NRED), dim3(256), 0,
                     b->stream, part, reinterpret_cast<const int*>(w + b->off_rng), 0,
                     reinterpret_cast<double*>(w + b->off_res));
  BHIP_TRY(b, hipGetLastError());
  return VFLB_OK;
}

}  // namespace

extern "C" {

vflb_status vflb_batch_create(int lattice, int n, const int* dims, int storage,
                              void* hip_stream, vflb_batch** out) {
  if (!out) return bfail(nullptr, VFLB_EINVAL, "out is NULL");
  *out = nullptr;
  if (lattice != VFLB_D2Q9) return bfail(nullptr, VFLB_EINVAL, "batches hold D2Q9 lattices");
  if (n < 1 || !dims) return bfail(nullptr, VFLB_EINVAL, "need n >= 1 and dims");
  if (storage < VFLB_F64 || storage > VFLB_BF16S)
    return bfail(nullptr, VFLB_EINVAL, "unknown storage %d", storage);
  vflb_batch* b = new vflb_batch();
  b->D = lattice;
  b->storage = storage;
  b->n = n;
  b->stream = static_cast<hipStream_t>(hip_stream);
  size_t total[VFLB_NBUF] = {};
  for (int i = 0; i < n; ++i) {
    vflb_sim* v = nullptr;
    if (sim_new(lattice, dims[3 * i], dims[3 * i + 1], 1, storage, b->stream, true, &v) !=
        VFLB_OK) {
      const std::string msg = g_create_error;
      vflb_batch_destroy(b);
      return bfail(nullptr, VFLB_EINVAL, "instance %d: %s", i, msg.c_str());
    }
    b->views.push_back(v);
    for (int k = 0; k < VFLB_NBUF; ++k) {
      b->off[k].push_back(total[k]);
      total[k] += align256(v->bytes[k]);
    }
    b->max_tiles += (size_t)((v->nx + 63) / 64) * ((v->ny + 3) / 4);
  }
  size_t w = total[VFLB_BUF_WORK];
  b->off_desc = w;
  w += align256((size_t)n * desc_size(storage));
  b->off_tiles = w;
  w += align256(b->max_tiles * sizeof(BatchTile));
  b->off_part = w;
  w += align256(b->max_tiles * NRED * sizeof(double));
  b->off_rng = w;
  w += align256((size_t)2 * n * sizeof(int));
  b->off_res = w;
  w += align256((size_t)n * NRED * sizeof(double));
  total[VFLB_BUF_WORK] = w;
  for (int k = 0; k < VFLB_NBUF; ++k) b->bytes[k] = total[k];
  b->active.assign(n, 1);
  b->last.assign((size_t)14 * n, NAN);
  if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    vflb_batch_destroy(b);
    return bfail(nullptr, VFLB_EDEVICE, "hipStreamCreate failed");
  }
  *out = b;
  return VFLB_OK;
}

vflb_status vflb_batch_query_buffers(const vflb_batch* b, size_t bytes[VFLB_NBUF]) {
  if (!b || !bytes) return VFLB_EINVAL;
  for (int k = 0; k < VFLB_NBUF; ++k) bytes[k] = b->bytes[k];
  return VFLB_OK;
}

vflb_status vflb_batch_bind_buffers(vflb_batch* b, void* const dev_ptrs[VFLB_NBUF]) {
  if (!b || !dev_ptrs) return VFLB_EINVAL;
  for (int k = 0; k < VFLB_NBUF; ++k)
    if (!dev_ptrs[k]) return bfail(b, VFLB_EINVAL, "buffer %d is NULL", k);
  for (int k = 0; k < VFLB_NBUF; ++k) b->buf[k] = dev_ptrs[k];
  for (int i = 0; i < b->n; ++i) {
    vflb_sim* v = b->views[i];
    for (int k = 0; k < VFLB_NBUF; ++k) v->buf[k] = static_cast<char*>(dev_ptrs[k]) + b->off[k][i];
    v->bound = true;
    v->inited = false;
  }
  b->bound = true;
  b->tables_ok = false;
  b->desc_dev.clear();
  bdrop_graphs(b);
  return VFLB_OK;
}

vflb_sim* vflb_batch_instance(vflb_batch* b, int i) {
  if (!b || i < 0 || i >= b->n) return nullptr;
  return b->views[i];
}

int vflb_batch_size(const vflb_batch* b) { return b ? b->n : -1; }

vflb_status vflb_batch_set_tile(vflb_batch* b, int tile_y) {
  if (!b) return VFLB_EINVAL;
  if (tile_y != 0 && tile_y != 4 && tile_y != 8 && tile_y != 16)
    return bfail(b, VFLB_EINVAL, "tile_y must be 0, 4, 8 or 16");
  b->tile_y = tile_y;
  bdrop_graphs(b);
  return VFLB_OK;
}

int vflb_batch_get_tile(const vflb_batch* b) { return b ? batch_ty(b) : -1; }

vflb_status vflb_batch_set_active(vflb_batch* b, int i, int active) {
  if (!b || i < 0 || i >= b->n) return VFLB_EINVAL;
  if ((b->active[i] != 0) != (active != 0)) {
    b->active[i] = active ? 1 : 0;
    b->tables_ok = false;
    bdrop_graphs(b);
  }
  return VFLB_OK;
}

int vflb_batch_is_active(const vflb_batch* b, int i) {
  if (!b || i < 0 || i >= b->n) return -1;
  return b->active[i] ? 1 : 0;
}

vflb_status vflb_batch_step(vflb_batch* b, int64_t nsteps) {
  if (!b) return VFLB_EINVAL;
  if (nsteps < 0) return bfail(b, VFLB_EINVAL, "nsteps < 0");
  int64_t t;
  int cur;
  vflb_status rc = check_active(b, &t, &cur);
  if (rc != VFLB_OK) return rc;
  if ((rc = ensure_tables(b)) != VFLB_OK) return rc;
  if (b->act.empty() || nsteps == 0) return VFLB_OK;
  if ((rc = sync_desc(b)) != VFLB_OK) return rc;
  int64_t left = nsteps;
  while (left > 0) {
    if (t > 0 && left >= kGraphSteps && b->stream != nullptr) {
      if (!b->gexec[cur] && (rc = build_batch_graph(b, cur)) != VFLB_OK) return rc;
      BHIP_TRY(b, hipGraphLaunch(b->gexec[cur], b->stream));
      t += kGraphSteps;  // even: parity unchanged
      left -= kGraphSteps;
      continue;
    }
    if ((rc = launch_batch(b, b->stream, cur, t == 0 ? 1 : 0)) != VFLB_OK) return rc;
    cur ^= 1;
    t += 1;
    left -= 1;
  }
  for (int i : b->act) {
    b->views[i]->t = t;
    b->views[i]->cur = cur;
  }
  return VFLB_OK;
}

vflb_status vflb_batch_reduce(vflb_batch* b, double* out) {
  if (!b || !out) return VFLB_EINVAL;
  int64_t t;
  int cur;
  vflb_status rc = check_active(b, &t, &cur);
  if (rc != VFLB_OK) return rc;
  if ((rc = ensure_tables(b)) != VFLB_OK) return rc;
  if (!b->act.empty()) {
    if ((rc = sync_desc(b)) != VFLB_OK) return rc;
    switch (b->storage) {
      case VFLB_F64: rc = launch_batch_reduce_s<double>(b, cur); break;
      case VFLB_F32: rc = launch_batch_reduce_s<float>(b, cur); break;
      case VFLB_F16S: rc = launch_batch_reduce_s<_Float16>(b, cur); break;
      default: rc = launch_batch_reduce_s<bf16_t>(b, cur); break;
    }
    if (rc != VFLB_OK) return rc;
    std::vector<double> r(b->act.size() * NRED);
    BHIP_TRY(b, hipMemcpyAsync(r.data(), static_cast<char*>(b->buf[VFLB_BUF_WORK]) + b->off_res,
                               r.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    for (size_t k = 0; k < b->act.size(); ++k) {
      const int i = b->act[k];
      (void)finish_reduce(b->views[i], &r[k * NRED], &b->last[(size_t)14 * i]);
    }
  }
  std::copy(b->last.begin(), b->last.end(), out);
  return VFLB_OK;
}

vflb_status vflb_batch_run_until(vflb_batch* b, double tol, int64_t check_every,
                                 const int64_t* max_steps, int64_t* steps_out,
                                 double* resid_out, int* status_out) {
  if (!b || !max_steps || !steps_out || !resid_out || !status_out) return VFLB_EINVAL;
  if (!(tol >= 0) || check_every < 1) return bfail(b, VFLB_EINVAL, "need tol >= 0 and check_every >= 1");
  int64_t t;
  int cur;
  vflb_status rc = check_active(b, &t, &cur);
  if (rc != VFLB_OK) return rc;
  std::vector<double> red((size_t)14 * b->n);
  // residual of the last interval of exactly check_every steps per instance
  std::vector<double> full_R((size_t)b->n, INFINITY);
  for (int i = 0; i < b->n; ++i) status_out[i] = b->active[i] ? VFLB_RUN_ACTIVE : VFLB_RUN_SKIPPED;
  // a fresh snapshot, so that every residual below spans a known interval
  if ((rc = vflb_batch_reduce(b, red.data())) != VFLB_OK) return rc;
  for (;;) {
    // the active instances share one time level, so one interval k; it is
    // shortened only to stop an instance exactly at its cap
    int64_t k = check_every;
    for (int i = 0; i < b->n; ++i) {
      if (!b->active[i]) continue;
      const int64_t rem = max_steps[i] - b->views[i]->t;
      if (rem <= 0) {
        status_out[i] = VFLB_RUN_CAPPED;
        vflb_batch_set_active(b, i, 0);
      } else if (rem < k) {
        k = rem;
      }
    }
    bool any = false;
    for (int i = 0; i < b->n; ++i) any = any || b->active[i];
    if (!any) break;
    if ((rc = vflb_batch_step(b, k)) != VFLB_OK) return rc;
    if ((rc = vflb_batch_reduce(b, red.data())) != VFLB_OK) return rc;
    // R is the relative change over the k steps just taken: it is held
    // against tol only when they were a full check_every interval
    const bool full = k == check_every;
    for (int i = 0; i < b->n; ++i) {
      if (!b->active[i]) continue;
      const double R = red[(size_t)14 * i], bad = red[(size_t)14 * i + 7];
      if (full) full_R[i] = R;
      if (bad > 0) status_out[i] = VFLB_RUN_UNSTABLE;
      else if (full && R < tol) status_out[i] = VFLB_RUN_CONVERGED;
      else if (b->views[i]->t >= max_steps[i]) status_out[i] = VFLB_RUN_CAPPED;
      else continue;
      vflb_batch_set_active(b, i, 0);
    }
  }
  for (int i = 0; i < b->n; ++i) {
    steps_out[i] = b->views[i]->t;
    resid_out[i] = status_out[i] == VFLB_RUN_SKIPPED ? b->last[(size_t)14 * i] : full_R[i];
  }
  return VFLB_OK;
}

vflb_status vflb_batch_autotune(vflb_batch* b, const char* cache_path, int* tile_y_out) {
  if (!b) return VFLB_EINVAL;
  if (!b->bound) return bfail(b, VFLB_ESTATE, "device buffers are not bound");
  size_t nodes = 0;
  for (int i = 0; i < b->n; ++i)
    if (b->active[i]) nodes += b->views[i]->N;
  if (nodes == 0) return bfail(b, VFLB_ESTATE, "no active instance");
  int dev = 0;
  hipDeviceProp_t prop;
  BHIP_TRY(b, hipGetDevice(&dev));
  BHIP_TRY(b, hipGetDeviceProperties(&prop, dev));
  char key[256];
  snprintf(key, sizeof key, "d2q9-batch storage=%d log2nodes=%d active=%d arch=%s", b->storage,
           (int)std::lround(std::log2((double)nodes)), (int)std::count(b->active.begin(), b->active.end(), 1),
           prop.gcnArchName);
  std::string path;
  if (cache_path && *cache_path) path = cache_path;
  else if (const char* e = getenv("VFLB_AUTOTUNE_CACHE")) path = e;
  if (!path.empty()) {
    if (FILE* fp = fopen(path.c_str(), "r")) {
      char line[512];
      int found = 0;
      while (fgets(line, sizeof line, fp)) {
        const size_t kl = strlen(key);
        int ty = 0;
        if (strncmp(line, key, kl) == 0 && line[kl] == ' ' && sscanf(line + kl + 1, "%d", &ty) == 1 &&
            (ty == 4 || ty == 8 || ty == 16))
          found = ty;
      }
      fclose(fp);
      if (found) {
        b->tile_y = found;
        bdrop_graphs(b);
        if (tile_y_out) *tile_y_out = found;
        return VFLB_OK;
      }
    }
  }
  // time each tile height on zeroed populations; the state is clobbered
  for (int k = 0; k < 3; ++k)
    if (k != VFLB_BUF_SNAP) BHIP_TRY(b, hipMemsetAsync(b->buf[k], 0, b->bytes[k], b->stream));
  vflb_status rc = sync_desc(b);
  if (rc != VFLB_OK) return rc;
  hipEvent_t e0, e1;
  BHIP_TRY(b, hipEventCreate(&e0));
  BHIP_TRY(b, hipEventCreate(&e1));
  const int cand[3] = {4, 8, 16};
  int best = 8;
  float best_ms = INFINITY;
  for (int c = 0; c < 3 && rc == VFLB_OK; ++c) {
    if ((rc = build_tables(b, cand[c])) != VFLB_OK) break;
    for (int k = 0; k < 3 && rc == VFLB_OK; ++k) rc = launch_batch(b, b->stream, k & 1, 0);
    if (rc != VFLB_OK) break;
    (void)hipEventRecord(e0, b->stream);
    for (int k = 0; k < 10 && rc == VFLB_OK; ++k) rc = launch_batch(b, b->stream, k & 1, 0);
    (void)hipEventRecord(e1, b->stream);
    if (hipEventSynchronize(e1) != hipSuccess) rc = bfail(b, VFLB_EDEVICE, "timing failed");
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (rc == VFLB_OK && ms < best_ms) {
      best_ms = ms;
      best = cand[c];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (vflb_sim* v : b->views) {
    v->inited = false;
    v->snap_valid = false;
  }
  b->tables_ok = false;
  if (rc != VFLB_OK) return rc;
  b->tile_y = best;
  bdrop_graphs(b);
  if (!path.empty()) {
    if (FILE* fp = fopen(path.c_str(), "a")) {
      fprintf(fp, "%s %d\n", key, best);
      fclose(fp);
    }
  }
  if (tile_y_out) *tile_y_out = best;
  return VFLB_OK;
}

void vflb_batch_destroy(vflb_batch* b) {
  if (!b) return;
  bdrop_graphs(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  for (vflb_sim* v : b->views) delete v;
  delete b;
}

const char* vflb_batch_last_error(const vflb_batch* b) {
  if (!b) return g_batch_create_error.c_str();
  return b->err.c_str();
}

}  // extern "C"

// --------------------------------------------- calls from other units
namespace vflb {
namespace internal {

vflb_status sim_scratch(vflb_sim* s, SimScratch* out) {
  vflb_status rc = need_ready(s);
  if (rc != VFLB_OK) return rc;
  out->D = s->D;
  out->nx = s->nx;
  out->ny = s->ny;
  out->walls = s->walls;
  out->stream = s->stream;
  out->lam_over_eta = s->lp.eta_p > 0 ? s->lp.lambda / s->lp.eta_p : 0.0;
  out->scratch = s->buf[VFLB_BUF_SNAP];
  out->bytes = s->bytes[VFLB_BUF_SNAP];
  out->big = s->buf[VFLB_BUF_POP1];
  out->big_bytes = s->bytes[VFLB_BUF_POP1];
  return VFLB_OK;
}

vflb_status sim_init_f32(vflb_sim* s, const float* u, const float* tau) {
  vflb_status rc = need_ready(s);
  if (rc != VFLB_OK) return rc;
  s->cur = 0;
  s->t = 0;
  rc = dispatch<InitOp>(s, u, tau, (const float*)nullptr);
  if (rc != VFLB_OK) return rc;
  s->inited = true;
  s->snap_valid = false;  // the snapshot buffer held the fields
  return VFLB_OK;
}

vflb_status sim_settle_f32(vflb_sim* s, const float* targets, int64_t nsteps, int flags) {
  vflb_status rc = need_ready(s);
  if (rc != VFLB_OK) return rc;
  if (!s->inited) return fail(s, VFLB_ESTATE, "initialise the fields first");
  if (s->D != 2) return fail(s, VFLB_EINVAL, "settling is implemented for D2Q9");
  if (s->inplace) return fail(s, VFLB_EINVAL, "settling needs two population buffers");
  if (flags < 1 || flags > 3) return fail(s, VFLB_EINVAL, "settle flags must be 1, 2 or 3");
  s->clamp = targets;
  s->clamp_flags = flags;
  for (int64_t k = 0; k < nsteps && rc == VFLB_OK; ++k) {
    rc = dispatch<StepOp>(s, s->t, s->stream, s->cur);
    if (rc == VFLB_OK) {
      s->cur ^= 1;
      s->t += 1;
    }
  }
  s->clamp = nullptr;
  s->clamp_flags = 0;
  return rc;
}

}  // namespace internal
}  // namespace vflb
