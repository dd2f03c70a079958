// kernels.h -- HIP kernels of the fused fluctuating-LB step for gfx950.
//
// Populations are post-collision values of the last step (pull scheme:
// streaming happens on the read), h stored minus w_i delta_ab; layout.h
// gives their placement in HBM.  chi(t-1) and u(t-1) for the backward
// difference of the source term are read and written in place by the
// owning node only.
// This file holds what the step kernels (step2d.h, step3d.h) share, and
// the initialisation, moment, reduction and copy kernels.  A step pulls f
// and h, forms the moments, collides f (Sec. 2.2), builds u on a tile plus
// a one-node halo in LDS for the same-time velocity gradient, then forms
// the Oldroyd-B source and collides h (Sec. 2.3); f and h are written to the
// other buffer of a ping-pong pair.
#pragma once

#include "layout.h"

namespace vflb {

enum { FORCE_NONE = 0, FORCE_CONST = 1, FORCE_FOUR_ROLL = 2, FORCE_COS_T = 3 };

struct Geo {
  int nx, ny, nz;
  int walls;  // bit a: halfway bounce-back walls on axis a
  size_t N;
  // how the population buffer holds the state at time t:
  //   0  two buffers: post-collision values of the last step at their
  //      writer's node (the reader pulls them);
  //   1  one buffer, in place (AA), t even: pre-collision values at their
  //      own node and direction;
  //   2  one buffer, in place, t odd: post-collision values at their
  //      writer's node under the opposite direction.
  int aa;
};

template <class R> struct ForceArgs {
  int kind;
  R F0[3];        // uniform force (CONST, COS_T at this time level)
  R amp[2];       // FOUR_ROLL amplitudes
  const R* tab;   // FOUR_ROLL tables: sin(kx x)[nx], cos(kx x)[nx], sin(ky y)[ny], cos(ky y)[ny]
  const R* div;   // stress-divergence scheme: div tau_p [div_d][N] added to F; else null
  int div_d;      // components of div (the lattice dimension)
};

template <class S> struct StepArgs {
  using R = typename StoreT<S>::R;
  const S* pin;   // populations read (pull)
  S* pout;        // populations written
  R* aux;
  Geo g;
  Phys<R> P;
  ForceArgs<R> F;
  R sf, inv_sf, sh, inv_sh;  // storage scales (1 unless FP16)
  int first;                 // t == 0: no previous source term
  // Settling (D2Q9 only; nullptr otherwise): FP32 fields u [2][N] and tau
  // [3][N] that replace the moment u (clamp_flags bit 0) and the moment A
  // (bit 1) of every node in the collision, so that the rest of the state
  // develops consistently with prescribed fields before the run starts.
  const float* clamp;
  int clamp_flags;
};

// Batched ensembles: one entry of the flattened tile table (a 64 x TY tile
// of instance inst at origin (x0, y0)), and the per-instance arguments, with
// pin in the population buffer of parity 0.
struct BatchTile {
  int inst, x0, y0, pad;
};
template <class S> struct BatchInst {
  StepArgs<S> a;
  typename StoreT<S>::R* snap;  // u, tau at the previous reduction
  int snap_valid;
};

__device__ inline size_t node_of(int x, int y, int z, const Geo& g) {
  return ((size_t)z * g.ny + y) * g.nx + x;
}

// Tuple index of population i at node n: plane i, i*N + n.
template <int D>
__host__ __device__ inline size_t tuple_of(int i, size_t n, size_t N) {
  return (size_t)i * N + n;
}

// Index of the post-collision value that streams into direction i of node
// (x, y, z): population i at x - c_i (periodic wrap), or population
// opp(i) at the node itself when x - c_i lies beyond a wall (halfway
// bounce-back).  The returned value is a tuple index (tuple_of).
template <int D>
__device__ inline size_t pull_index(int i, int x, int y, int z, const Geo& g) {
  // index of the value that is f_i (or h_i) of node (x, y, z) at time t
  if (g.aa == 1) return tuple_of<D>(i, node_of(x, y, z, g), g.N);
  int s[3] = {x - cdir<D>(i, 0), y - cdir<D>(i, 1), z - cdir<D>(i, 2)};
  const int n[3] = {g.nx, g.ny, g.nz};
  bool bounce = false;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    if (cdir<D>(i, a) != 0 && (s[a] < 0 || s[a] >= n[a])) {
      if (g.walls & (1 << a))
        bounce = true;
      else
        s[a] = s[a] < 0 ? n[a] - 1 : 0;
    }
  }
  // two buffers: the writer x - c_i keeps it under i, or the node itself
  // under opp(i) behind a wall; in place and t odd the directions swap
  const int j = g.aa == 2 ? Lat<D>::opp(i) : i;
  if (bounce) return tuple_of<D>(Lat<D>::opp(j), node_of(x, y, z, g), g.N);
  return tuple_of<D>(j, node_of(s[0], s[1], s[2], g), g.N);
}

// Body force at node (x, y, z) of the lattice g: the force field of fa
// (four-roll tables depend on x and y only), plus div tau_p of that node in
// the stress-divergence scheme.
template <class R>
__device__ inline void force_at(const ForceArgs<R>& fa, int x, int y, int z, const Geo& g,
                                R* F) {
  const int nx = g.nx, ny = g.ny;
  F[0] = F[1] = F[2] = 0;
  if (fa.kind == FORCE_CONST || fa.kind == FORCE_COS_T) {
    F[0] = fa.F0[0];
    F[1] = fa.F0[1];
    F[2] = fa.F0[2];
  } else if (fa.kind == FORCE_FOUR_ROLL) {
    const R* sx = fa.tab;
    const R* cx = fa.tab + nx;
    const R* sy = fa.tab + 2 * nx;
    const R* cy = fa.tab + 2 * nx + ny;
    F[0] = fa.amp[0] * sx[x] * cy[y];
    F[1] = fa.amp[1] * cx[x] * sy[y];
  }
  if (fa.div) {
    const size_t n = ((size_t)z * ny + y) * nx + x, M = g.N;
    F[0] += fa.div[n];
    F[1] += fa.div[M + n];
    if (fa.div_d == 3) F[2] += fa.div[2 * M + n];
  }
}

// Wrap a coordinate that may lie outside [0, n) by at most one tile: for a
// wall axis the point is outside the fluid (returns false).
__device__ inline bool wrap_coord(int& c, int n, bool wall) {
  if (c >= 0 && c < n) return true;
  if (wall) return false;
  c = ((c % n) + n) % n;
  return true;
}

// --------------------------------------------------------------- step
template <int D, class S>
struct NodeMoments {
  using R = typename StoreT<S>::R;
  R f[Lat<D>::Q];
  R h[Lat<D>::NC][Lat<D>::Q];
  R u[3], e[Lat<D>::NC], tau[Lat<D>::NC], p;
};

template <int D, class S>
__device__ inline void node_moments(const S* pin, const typename StoreT<S>::R* aux, int x, int y,
                                    int z, const Geo& g,
                                    const Phys<typename StoreT<S>::R>& P,
                                    const ForceArgs<typename StoreT<S>::R>& fa,
                                    typename StoreT<S>::R inv_sf,
                                    typename StoreT<S>::R inv_sh,
                                    NodeMoments<D, S>& m) {
  using St = StoreT<S>;
  using R = typename St::R;
  using L = Lat<D>;
  constexpr int Q = L::Q, NC = L::NC;
  constexpr bool ANCHOR = D == 2 && St::kAnchored;
  constexpr bool ANCHOR3 = D == 3 && St::kAnchored;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    R hv[NC];
    const size_t t = pull_index<D>(i, x, y, z, g);
    Pops<D, S>::load(pin, t, g.N, inv_sf, inv_sh, m.f[i], hv);
    if constexpr (ANCHOR3) {  // reference of the writing node + deviation
      const int j = (int)(t / g.N);
      const size_t src = t - (size_t)j * g.N;
      float pa, ua[3], Ea[6];
      Anchor3::load(pin, src, g.N, pa, ua, Ea);
      const R uw[3] = {(R)ua[0], (R)ua[1], (R)ua[2]};
      m.f[i] += fref3<R>(j, (R)pa, uw);
#pragma unroll
      for (int c = 0; c < NC; ++c) hv[c] += href3<R>(j, c, (R)Ea[c], uw);
    }
    if constexpr (ANCHOR) {  // reference of the writing node + deviation
      const int j = (int)(t / g.N);
      const size_t src = t % g.N;
      float4 q;
      float2 v;
      Anchor2::load(pin, src, g.N, q, v);
      const R ux = (R)v.x, uy = (R)v.y;
      m.f[i] += fref2<R>(j, (R)1, (R)q.w, ux, uy);
      hv[0] += href2<R>(j, 0, (R)1, (R)q.x, ux, uy);
      hv[1] += href2<R>(j, 1, (R)1, (R)q.y, ux, uy);
      hv[2] += href2<R>(j, 2, (R)1, (R)q.z, ux, uy);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) m.h[c][i] = hv[c];
  }
  R F[3];
  force_at<R>(fa, x, y, z, g, F);
  m.u[2] = 0;
#pragma unroll
  for (int b = 0; b < D; ++b) {
    R s = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i)
      if (cdir<D>(i, b) != 0) s += (R)cdir<D>(i, b) * m.f[i];
    m.u[b] = s + (R)0.5 * F[b];
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    R s = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) s += m.h[c][i];
    m.e[c] = s;
    m.tau[c] = P.eta_over_lam * s;
  }
  R fB[Q];
  fluct_term<R>(m.tau, P.inv_tau_f * P.fluct, fB, (L*)nullptr);
  R uu = 0, Fu = 0, sum = 0;
#pragma unroll
  for (int b = 0; b < D; ++b) {
    uu += m.u[b] * m.u[b];
    Fu += F[b] * m.u[b];
  }
#pragma unroll
  for (int i = 1; i < Q; ++i) sum += m.f[i];
  constexpr R w0 = (R)L::w(0);
  const R F0 = -3 * w0 * P.k_f * Fu;
  constexpr R pref = (R)((1.0 / 3.0) / (1.0 - L::w(0)));
  m.p = pref * (sum - (R)1.5 * w0 * uu + P.tau_f * F0 + P.tau_f * fB[0]);
}

template <int D>
__device__ inline void node_xyz(size_t n, const Geo& g, int& x, int& y, int& z) {
  x = (int)(n % g.nx);
  y = (int)((n / g.nx) % g.ny);
  z = (int)(n / ((size_t)g.nx * g.ny));
}

// A box of nodes for read-back: origin lo (any integers; coordinates wrap
// periodically) and extent n; box node k (x fastest) maps to a lattice node.
struct Box {
  int lo[3], n[3];
  size_t N;  // n[0] n[1] n[2]
};

__device__ inline void box_node(size_t k, const Box& b, const Geo& g, int& x, int& y, int& z) {
  const int bx = (int)(k % b.n[0]), by = (int)((k / b.n[0]) % b.n[1]),
            bz = (int)(k / ((size_t)b.n[0] * b.n[1]));
  x = ((b.lo[0] + bx) % g.nx + g.nx) % g.nx;
  y = ((b.lo[1] + by) % g.ny + g.ny) % g.ny;
  z = ((b.lo[2] + bz) % g.nz + g.nz) % g.nz;
}

// ------------------------------------------------------------- read-back
enum { FIELD_U = 0, FIELD_P = 1, FIELD_RHO = 2, FIELD_A = 3, FIELD_TAU = 4,
       FIELD_F = 5, FIELD_H = 6, FIELD_CHI_PREV = 7, FIELD_U_PREV = 8 };

// auxiliary state chi(t-1) (field 7) or u(t-1) (field 8), component-major FP64
template <int D, class R>
__global__ void __launch_bounds__(256) aux_read_kernel(const R* aux, Geo g, Box box, int field,
                                                       double* out) {
  constexpr int NC = Lat<D>::NC;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < box.N;
       k += (size_t)gridDim.x * blockDim.x) {
    int x, y, z;
    box_node(k, box, g, x, y, z);
    const size_t n = node_of(x, y, z, g);
    R chi[NC], u[3] = {0, 0, 0};
    Aux<D, R>::load(aux, n, g.N, chi, u);
    if (field == FIELD_CHI_PREV)
      for (int c = 0; c < NC; ++c) out[(size_t)c * box.N + k] = (double)chi[c];
    else
      for (int b = 0; b < D; ++b) out[(size_t)b * box.N + k] = (double)u[b];
  }
}

template <int D, class S>
__global__ void __launch_bounds__(256) moments_kernel(
    const S* pin, const typename StoreT<S>::R* aux, Geo g, Box box, Phys<typename StoreT<S>::R> P,
    ForceArgs<typename StoreT<S>::R> fa, typename StoreT<S>::R inv_sf,
    typename StoreT<S>::R inv_sh, int field, double* out) {
  using L = Lat<D>;
  constexpr int Q = L::Q, NC = L::NC;
  const size_t M = box.N;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < M;
       k += (size_t)gridDim.x * blockDim.x) {
    int x, y, z;
    box_node(k, box, g, x, y, z);
    NodeMoments<D, S> m;
    node_moments<D, S>(pin, aux, x, y, z, g, P, fa, inv_sf, inv_sh, m);
    switch (field) {
      case FIELD_U:
        for (int b = 0; b < D; ++b) out[(size_t)b * M + k] = (double)m.u[b];
        break;
      case FIELD_P:
        out[k] = (double)m.p;
        break;
      case FIELD_RHO:
        out[k] = 1.0 + 3.0 * (double)m.p;
        break;
      case FIELD_A:
        for (int c = 0; c < NC; ++c)
          out[(size_t)c * M + k] = (double)m.e[c] + ((L::ca(c) == L::cb(c)) ? 1.0 : 0.0);
        break;
      case FIELD_TAU:
        for (int c = 0; c < NC; ++c) out[(size_t)c * M + k] = (double)m.tau[c];
        break;
      case FIELD_F:
        for (int i = 0; i < Q; ++i) out[(size_t)i * M + k] = (double)m.f[i];
        break;
      case FIELD_H:
        for (int c = 0; c < NC; ++c)
          for (int i = 0; i < Q; ++i)
            out[((size_t)c * Q + i) * M + k] =
                (double)m.h[c][i] + ((L::ca(c) == L::cb(c)) ? L::w(i) : 0.0);
        break;
    }
  }
}

// ------------------------------------------------------------------ init
// Equilibrium-only state: f = f^eq(p, u), h = h^eq(A, u) (shifted), with
// A = I + lambda tau / eta_p; each value is written where the pull of the
// first step reads it, so that the first step sees exactly this state.
// anchor of node m from the initial fields: (E = lambda tau / eta_p, p)
template <class T>
__device__ inline float4 init_anchor(size_t m, size_t N, const T* tau_in, const T* p_in,
                                     double lam_over_eta) {
  float4 q;
  q.x = tau_in ? (float)(lam_over_eta * tau_in[m]) : 0.0f;
  q.y = tau_in ? (float)(lam_over_eta * tau_in[N + m]) : 0.0f;
  q.z = tau_in ? (float)(lam_over_eta * tau_in[2 * N + m]) : 0.0f;
  q.w = p_in ? (float)p_in[m] : 0.0f;
  return q;
}

template <class T>
__device__ inline float2 init_velocity(size_t m, size_t N, const T* u_in) {
  float2 v;
  v.x = u_in ? (float)u_in[m] : 0.0f;
  v.y = u_in ? (float)u_in[N + m] : 0.0f;
  return v;
}

// D3Q19 anchor of node m from the initial fields
template <class T>
__device__ inline void init_anchor3(size_t m, size_t N, const T* u_in, const T* tau_in,
                                    const T* p_in, double lam_over_eta, float& p, float* u,
                                    float* E) {
  p = p_in ? (float)p_in[m] : 0.0f;
  for (int b = 0; b < 3; ++b) u[b] = u_in ? (float)u_in[(size_t)b * N + m] : 0.0f;
  for (int c = 0; c < 6; ++c) E[c] = tau_in ? (float)(lam_over_eta * tau_in[(size_t)c * N + m]) : 0.0f;
}

template <int D, class S, class T>
__global__ void __launch_bounds__(256) init_kernel(
    S* pbuf, typename StoreT<S>::R* aux, Geo g,
    const T* u_in, const T* tau_in, const T* p_in,
    double lam_over_eta, typename StoreT<S>::R sf, typename StoreT<S>::R sh) {
  using St = StoreT<S>;
  using R = typename St::R;
  using L = Lat<D>;
  constexpr int Q = L::Q, NC = L::NC;
  constexpr bool ANCHOR = D == 2 && St::kAnchored;
  constexpr bool ANCHOR3 = D == 3 && St::kAnchored;
  for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < g.N;
       n += (size_t)gridDim.x * blockDim.x) {
    int x, y, z;
    node_xyz<D>(n, g, x, y, z);
    R u[3] = {0, 0, 0};
    if (u_in)
      for (int b = 0; b < D; ++b) u[b] = (R)u_in[(size_t)b * g.N + n];
    const R p = p_in ? (R)p_in[n] : (R)0;
    R e[NC];
    for (int c = 0; c < NC; ++c)
      e[c] = tau_in ? (R)(lam_over_eta * tau_in[(size_t)c * g.N + n]) : (R)0;
    R uu = 0;
    for (int b = 0; b < D; ++b) uu += u[b] * u[b];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R wi = (R)L::w(i);
      const R lam_i = (R)(i == 0 ? 3.0 * (L::w(0) - 1.0) : 3.0 * L::w(i));
      const R cu = cdot<D, R>(i, u);
      R feq = lam_i * p + wi * (3 * cu + (R)4.5 * cu * cu - (R)1.5 * uu);
      R hv[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const R Ac = e[c] + ((L::ca(c) == L::cb(c)) ? (R)1 : (R)0);
        hv[c] = wi * e[c] + 3 * wi * Ac * cu;
      }
      const size_t t = pull_index<D>(i, x, y, z, g);
      if constexpr (ANCHOR) {
        // deviation from the reference of the node that stores the value
        const int j = (int)(t / g.N);
        const size_t src = t % g.N;
        const float4 q = init_anchor(src, g.N, tau_in, p_in, lam_over_eta);
        const float2 v = init_velocity(src, g.N, u_in);
        const R ux = (R)v.x, uy = (R)v.y;
        feq -= fref2<R>(j, (R)1, (R)q.w, ux, uy);
        hv[0] -= href2<R>(j, 0, (R)1, (R)q.x, ux, uy);
        hv[1] -= href2<R>(j, 1, (R)1, (R)q.y, ux, uy);
        hv[2] -= href2<R>(j, 2, (R)1, (R)q.z, ux, uy);
      }
      if constexpr (ANCHOR3) {
        const int j = (int)(t / g.N);
        const size_t src = t - (size_t)j * g.N;
        float pa, ua[3], Ea[6];
        init_anchor3(src, g.N, u_in, tau_in, p_in, lam_over_eta, pa, ua, Ea);
        const R uw[3] = {(R)ua[0], (R)ua[1], (R)ua[2]};
        feq -= fref3<R>(j, (R)pa, uw);
#pragma unroll
        for (int c = 0; c < NC; ++c) hv[c] -= href3<R>(j, c, (R)Ea[c], uw);
      }
      Pops<D, S>::store(pbuf, t, g.N, sf, sh, feq, hv);
    }
    R zero[NC];
    for (int c = 0; c < NC; ++c) zero[c] = 0;
    Aux<D, R>::store(aux, n, g.N, zero, u);
    if constexpr (ANCHOR)
      Anchor2::store(pbuf, n, g.N, init_anchor(n, g.N, tau_in, p_in, lam_over_eta),
                     init_velocity(n, g.N, u_in));
    if constexpr (ANCHOR3) {
      float pa, ua[3], Ea[6];
      init_anchor3(n, g.N, u_in, tau_in, p_in, lam_over_eta, pa, ua, Ea);
      Anchor3::store(pbuf, n, g.N, pa, ua, Ea);
    }
  }
}

// ------------------------------------------------------------ reductions
constexpr int NRED = 17;  // du2 u2 dt2 t2 | M | Px Py Pz | KE PE | nan | A x6

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Accumulate one node's contribution to the reductions and refresh its
// snapshot of u and tau (the residual compares against the snapshot taken
// at the previous reduction).
template <int D, class S>
__device__ inline void reduce_node(const S* pin, const typename StoreT<S>::R* aux,
                                   typename StoreT<S>::R* snap, int snap_valid,
                                   int x, int y, int z, const Geo& g,
                                   const Phys<typename StoreT<S>::R>& P,
                                   const ForceArgs<typename StoreT<S>::R>& fa,
                                   typename StoreT<S>::R inv_sf, typename StoreT<S>::R inv_sh,
                                   double* acc) {
  using L = Lat<D>;
  constexpr int Q = L::Q, NC = L::NC;
  const size_t n = node_of(x, y, z, g);
  NodeMoments<D, S> m;
  node_moments<D, S>(pin, aux, x, y, z, g, P, fa, inv_sf, inv_sh, m);
  bool finite = true;
#pragma unroll
  for (int b = 0; b < D; ++b) {
    const double ub = (double)m.u[b];
    finite = finite && isfinite(ub);
    if (snap_valid) {
      const double d = ub - (double)snap[(size_t)b * g.N + n];
      acc[0] += d * d;
    }
    acc[1] += ub * ub;
    snap[(size_t)b * g.N + n] = m.u[b];
  }
  double tr = 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double tc = (double)m.tau[c];
    finite = finite && isfinite(tc);
    const double wgt = (L::ca(c) == L::cb(c)) ? 1.0 : 2.0;  // tensor norm
    if (snap_valid) {
      const double d = tc - (double)snap[(size_t)(D + c) * g.N + n];
      acc[2] += wgt * d * d;
    }
    acc[3] += wgt * tc * tc;
    if (L::ca(c) == L::cb(c)) tr += tc;
    acc[11 + c] += (double)m.e[c] + ((L::ca(c) == L::cb(c)) ? 1.0 : 0.0);
    snap[(size_t)(D + c) * g.N + n] = m.tau[c];
  }
  double M = 0.0, Pm[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double fi = (double)m.f[i];
    M += fi;
#pragma unroll
    for (int b = 0; b < D; ++b) Pm[b] += cdir<D>(i, b) * fi;
  }
  finite = finite && isfinite(M) && isfinite((double)m.p);
  acc[4] += M;
  acc[5] += Pm[0];
  acc[6] += Pm[1];
  acc[7] += Pm[2];
  acc[8] += 0.5 * ((double)m.u[0] * m.u[0] + (double)m.u[1] * m.u[1] +
                   (double)m.u[2] * m.u[2]);
  acc[9] += 0.5 * tr;
  acc[10] += finite ? 0.0 : 1.0;
}

// Sum acc over a 256-lane workgroup in a fixed order into out[0..NRED).
__device__ inline void block_partials(const double* acc, double* out) {
  __shared__ double red[4][NRED];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NRED; ++k) {
    const double v = wave_sum(acc[k]);
    if (lane == 0) red[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < NRED) {
    double s = 0.0;
    for (int w = 0; w < 4; ++w) s += red[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

template <int D, class S>
__global__ void __launch_bounds__(256) reduce_kernel(
    const S* pin, const typename StoreT<S>::R* aux, typename StoreT<S>::R* snap, int snap_valid,
    Geo g, Phys<typename StoreT<S>::R> P, ForceArgs<typename StoreT<S>::R> fa,
    typename StoreT<S>::R inv_sf, typename StoreT<S>::R inv_sh,
    double* partials) {
  double acc[NRED];
#pragma unroll
  for (int k = 0; k < NRED; ++k) acc[k] = 0.0;
  for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < g.N;
       n += (size_t)gridDim.x * blockDim.x) {
    int x, y, z;
    node_xyz<D>(n, g, x, y, z);
    reduce_node<D, S>(pin, aux, snap, snap_valid, x, y, z, g, P, fa, inv_sf, inv_sh, acc);
  }
  block_partials(acc, partials + (size_t)blockIdx.x * NRED);
}

// out[r][k] = sum of partials[b][k] over b in [ranges[2r], ranges[2r+1])
// (ranges == nullptr: the single range [0, nb)), for r = blockIdx.x and
// k = blockIdx.y.  Lane j sums b = begin + j, begin + j + 256, ... and the
// lanes combine in a fixed tree, so the result does not depend on timing.
__global__ void __launch_bounds__(256) reduce_finish_kernel(const double* partials,
                                                            const int* ranges, int nb,
                                                            double* out) {
  const int r = blockIdx.x, k = blockIdx.y;
  const int b0 = ranges ? ranges[2 * r] : 0, b1 = ranges ? ranges[2 * r + 1] : nb;
  double s = 0.0;
  for (int b = b0 + (int)threadIdx.x; b < b1; b += 256) s += partials[(size_t)b * NRED + k];
  __shared__ double red[4];
  const double v = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) out[(size_t)r * NRED + k] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Reductions of a batched ensemble: one workgroup per tile-table entry
// (tile_h rows of 64 nodes), partials[k] for entry k.
template <class S>
__global__ void __launch_bounds__(256) batch_reduce_kernel(const BatchInst<S>* __restrict__ desc,
                                                           const BatchTile* __restrict__ tiles,
                                                           int tile_h, int parity,
                                                           double* partials) {
  const BatchTile e = tiles[blockIdx.x];
  const BatchInst<S>& d = desc[e.inst];
  const S* pin = parity ? d.a.pout : d.a.pin;
  double acc[NRED];
#pragma unroll
  for (int k = 0; k < NRED; ++k) acc[k] = 0.0;
  for (int j = threadIdx.x; j < 64 * tile_h; j += blockDim.x) {
    const int x = e.x0 + (j & 63), y = e.y0 + (j >> 6);
    if (x < d.a.g.nx && y < d.a.g.ny)
      reduce_node<2, S>(pin, d.a.aux, d.snap, d.snap_valid, x, y, 0, d.a.g, d.a.P, d.a.F,
                        d.a.inv_sf, d.a.inv_sh, acc);
  }
  block_partials(acc, partials + (size_t)blockIdx.x * NRED);
}

// ------------------------------------------------ stress-divergence scheme
// The scheme the paper compares its method against (Sec. 3, performance
// tables; described in words in the Introduction): the divergence of the
// polymer stress enters the f equation as a body force, F_tot = F +
// div tau_p, and f^B is absent.  Per step: tau_p(t) of every node from its
// pulled h (taup_kernel), then div tau_p by second-order central
// differences, one-sided second order normal to a wall (stress_div_kernel);
// the step kernels add it to F wherever they evaluate the force.  D2Q9 and
// D3Q19.

template <int D, class S>
__global__ void __launch_bounds__(256) taup_kernel(const S* __restrict__ pin, Geo g,
                                                   typename StoreT<S>::R eta_over_lam,
                                                   typename StoreT<S>::R* __restrict__ taup) {
  using R = typename StoreT<S>::R;
  using L = Lat<D>;
  constexpr int Q = L::Q, NC = L::NC;
  const size_t N = g.N;
  for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    int x, y, z;
    node_xyz<D>(n, g, x, y, z);
    R e[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) e[c] = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      R f, hv[NC];
      const size_t t = pull_index<D>(i, x, y, z, g);
      if constexpr (D == 2 && !StoreT<S>::kPlanar)
        Pops<2, S>::template load<true>(pin, t, N, (R)1, (R)1, f, hv);
      else
        Pops<D, S>::load(pin, t, N, (R)1, (R)1, f, hv);
#pragma unroll
      for (int c = 0; c < NC; ++c) e[c] += hv[c];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) taup[(size_t)c * N + n] = eta_over_lam * e[c];
  }
}

// derivative along axis a of the plane t at node (x, y, z): second-order
// central differences, periodic wrap; next to a wall the one-sided second
// order (-3 t0 + 4 t1 - t2)/2 (first order with two nodes across)
template <class R>
__device__ inline R stress_derivative(const R* t, int x, int y, int z, int a, const Geo& g) {
  const int n = a == 0 ? g.nx : (a == 1 ? g.ny : g.nz), c = a == 0 ? x : (a == 1 ? y : z);
  auto at = [&](int k) {
    const int xx = a == 0 ? k : x, yy = a == 1 ? k : y, zz = a == 2 ? k : z;
    return t[((size_t)zz * g.ny + yy) * g.nx + xx];
  };
  if (!(g.walls & (1 << a))) {
    const int cm = c == 0 ? n - 1 : c - 1, cp = c == n - 1 ? 0 : c + 1;
    return (R)0.5 * (at(cp) - at(cm));
  }
  if (c > 0 && c < n - 1) return (R)0.5 * (at(c + 1) - at(c - 1));
  if (n == 1) return (R)0;
  if (n == 2) return at(1) - at(0);
  if (c == 0) return (R)0.5 * ((R)-3 * at(0) + (R)4 * at(1) - at(2));
  return (R)0.5 * ((R)3 * at(n - 1) - (R)4 * at(n - 2) + at(n - 3));
}

// (div tau_p)_b = sum_a d_a tau_ab, tau_p [NC][N] in the component order of
// the lattice (2D: xx, xy, yy; 3D: xx, yy, zz, xy, xz, yz)
template <int D, class R>
__global__ void __launch_bounds__(256) stress_div_kernel(const R* __restrict__ taup, Geo g,
                                                         R* __restrict__ div) {
  using L = Lat<D>;
  const size_t N = g.N;
  for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    int x, y, z;
    node_xyz<D>(n, g, x, y, z);
    R dv[D];
#pragma unroll
    for (int b = 0; b < D; ++b) dv[b] = 0;
#pragma unroll
    for (int c = 0; c < L::NC; ++c) {
      const R* t = taup + (size_t)c * N;
      const int a = L::ca(c), b = L::cb(c);
      dv[b] += stress_derivative(t, x, y, z, a, g);
      if (a != b) dv[a] += stress_derivative(t, x, y, z, b, g);
    }
#pragma unroll
    for (int b = 0; b < D; ++b) div[(size_t)b * N + n] = dv[b];
  }
}


}  // namespace vflb
