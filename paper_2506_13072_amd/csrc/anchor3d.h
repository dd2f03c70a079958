// anchor3d.h -- the D3Q19 step with anchored 16-bit population storage.
//
// Populations are stored as FP16 / BF16 deviations from reference
// populations of the node that wrote them (layout.h: Anchor3, fref3,
// href3), so that the conserved conformation moment and the velocity live
// in FP32 anchors and 16-bit rounding touches only non-equilibrium parts.
// A reader rebuilds each pulled value from the deviation and the writer's
// anchor, which lies in one of the three planes z - 1, z, z + 1.
//
// The step is two launches.  anchor3_velocity_kernel forms the same-time
// velocity u(t) of every node from its pulled f into u [3][N];
// anchor3_step_kernel then rebuilds the pulled f and h, collides (the
// generic per-node collisions of lattice.h), takes the gradient from the
// face neighbours' u, and stores the post-collision deviations from the
// node's new anchor (E = sum of the post-collision h, the pressure and u of
// this step).  One lane owns one node.  In the velocity pass blockIdx.x
// runs over x, blockIdx.y and blockIdx.z (and their strides) over y and z;
// the step runs over 64 x 4 blocks (below).
#pragma once

#include "kernels.h"

namespace vflb {

// Writer of the value that streams into direction i of (x, y, z): its
// stored direction j and node src (as pull_index, without the division).
__device__ inline void pull_src3(int i, int x, int y, int z, const Geo& g, int& j,
                                 size_t& src) {
  int s[3] = {x - Lat<3>::cx(i), y - Lat<3>::cy(i), z - Lat<3>::cz(i)};
  const int n[3] = {g.nx, g.ny, g.nz};
  bool bounce = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (cdir<3>(i, a) != 0 && (s[a] < 0 || s[a] >= n[a])) {
      if (g.walls & (1 << a))
        bounce = true;
      else
        s[a] = s[a] < 0 ? n[a] - 1 : 0;
    }
  }
  if (bounce) {
    j = Lat<3>::opp(i);
    src = node_of(x, y, z, g);
  } else {
    j = i;
    src = node_of(s[0], s[1], s[2], g);
  }
}

template <class S>
__global__ void __launch_bounds__(256) anchor3_velocity_kernel(
    const S* __restrict__ pin, Geo g, ForceArgs<typename StoreT<S>::R> fa,
    typename StoreT<S>::R inv_sf, typename StoreT<S>::R* __restrict__ U) {
  using R = typename StoreT<S>::R;
  using L = Lat<3>;
  const size_t N = g.N;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  for (int z = blockIdx.z; z < g.nz; z += gridDim.z)
    for (int y = blockIdx.y; y < g.ny; y += gridDim.y) {
      R f[L::Q];
      f[0] = 0;
#pragma unroll
      for (int i = 1; i < L::Q; ++i) {
        int j;
        size_t src;
        pull_src3(i, x, y, z, g, j, src);
        float pa, ua[3];
        Anchor3::load_pu(pin, src, N, pa, ua);
        const R uw[3] = {(R)ua[0], (R)ua[1], (R)ua[2]};
        f[i] = Pops<3, S>::load_f(pin, tuple_of<3>(j, src, N), N, inv_sf) + fref3<R>(j, (R)pa, uw);
      }
      R F[3];
      force_at<R>(fa, x, y, g.nx, g.ny, F);
      const size_t n = node_of(x, y, z, g);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        R s = 0;
#pragma unroll
        for (int i = 1; i < L::Q; ++i)
          if (cdir<3>(i, b) != 0) s += (R)cdir<3>(i, b) * f[i];
        U[(size_t)b * N + n] = s + (R)0.5 * F[b];
      }
    }
}

// One lane per node, 256-node runs of x per block (64 x 4 blocks fetched
// 561 instead of 747 B per node but took 53 instead of 50 ms at 512^3: the
// kernel holds the 133 populations of its node and runs one wavefront per
// SIMD, so it is latency-bound); blockIdx.y, blockIdx.z and the strides of
// all three block indices run over the rest of the lattice.
constexpr int A3_TX = 256, A3_TY = 1;

template <class S>
__global__ void __launch_bounds__(256) anchor3_step_kernel(StepArgs<S> a,
                                                           const typename StoreT<S>::R* __restrict__ U) {
  using R = typename StoreT<S>::R;
  using L = Lat<3>;
  constexpr int Q = L::Q, NC = L::NC;
  const Geo g = a.g;
  const size_t N = g.N;
  const int x = blockIdx.x * A3_TX + (int)threadIdx.x;
  if (x >= g.nx) return;
  auto wrapc = [](int c, int n, bool wall) {
    if (c < 0) return wall ? 0 : c + n;
    if (c >= n) return wall ? n - 1 : c - n;
    return c;
  };
  for (int z = blockIdx.z; z < g.nz; z += gridDim.z)
    for (int y = blockIdx.y * A3_TY + (int)threadIdx.y; y < g.ny; y += gridDim.y * A3_TY) {
      const size_t n = node_of(x, y, z, g);
      R f[Q], h[NC][Q];
      static_for<0, Q>([&](auto ic) __attribute__((always_inline)) {
        constexpr int i = decltype(ic)::value;
        int j;
        size_t src;
        pull_src3(i, x, y, z, g, j, src);
        R hv[NC];
        Pops<3, S>::load(a.pin, tuple_of<3>(j, src, N), N, a.inv_sf, a.inv_sh, f[i], hv);
        float pa, ua[3], Ea[6];
        Anchor3::load(a.pin, src, N, pa, ua, Ea);
        const R uw[3] = {(R)ua[0], (R)ua[1], (R)ua[2]};
        f[i] += fref3<R>(j, (R)pa, uw);
  #pragma unroll
        for (int c = 0; c < NC; ++c) h[c][i] = hv[c] + href3<R>(j, c, (R)Ea[c], uw);
        // at most four directions' loads in flight: all 19 at once would
        // need about 500 registers and one wavefront per SIMD
        if constexpr (i % 4 == 3) __builtin_amdgcn_sched_barrier(0);
      });
      R chip[NC] = {0, 0, 0, 0, 0, 0}, up[3] = {0, 0, 0};
      if (!a.first) Aux<3, R>::load(a.aux, n, N, chip, up);
      R F[3];
      force_at<R>(a.F, x, y, g.nx, g.ny, F);
      const R u[3] = {U[n], U[N + n], U[2 * N + n]};
      R e[NC];
  #pragma unroll
      for (int c = 0; c < NC; ++c) {
        R sm = 0;
  #pragma unroll
        for (int i = 0; i < Q; ++i) sm += h[c][i];
        e[c] = sm;
      }
      const R p = collide_f<3, R>(f, e, u, F, a.P);
      // same-time gradient G[a][b] = d_a u_b: central differences, and at a
      // halfway bounce-back wall the one-sided form through the wall value
      R G[3][3];
      const int c3[3] = {x, y, z}, n3[3] = {g.nx, g.ny, g.nz};
  #pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const bool wall = (g.walls >> ax) & 1;
        const int c = c3[ax], nn = n3[ax];
        const bool lo = wall && c == 0, hi = wall && c == nn - 1;
        int qm[3] = {x, y, z}, qp[3] = {x, y, z};
        qm[ax] = wrapc(c - 1, nn, wall);
        qp[ax] = wrapc(c + 1, nn, wall);
        const size_t im = node_of(qm[0], qm[1], qm[2], g), ip = node_of(qp[0], qp[1], qp[2], g);
  #pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
          const R um = U[(size_t)bb * N + im], upl = U[(size_t)bb * N + ip];
          G[ax][bb] = lo ? u[bb] + upl * (R)(1.0 / 3.0)
                    : hi ? -(u[bb] + um * (R)(1.0 / 3.0))
                         : (R)0.5 * (upl - um);
        }
      }
      R chi[NC];
      source_tensor<3, R>(e, G, a.P, chi);
  #pragma unroll
      for (int c = 0; c < NC; ++c) {
        const R Ac = e[c] + (c < 3 ? (R)1 : (R)0);
        collide_h<3, R>(h[c], e[c], Ac, chi[c], chip[c], u, up, a.first != 0, a.P);
      }
      // new anchor: E = sum_i h*_i, the pressure and velocity of this step
      float En[NC], un[3];
  #pragma unroll
      for (int c = 0; c < NC; ++c) {
        R sm = 0;
  #pragma unroll
        for (int i = 0; i < Q; ++i) sm += h[c][i];
        En[c] = (float)sm;
      }
  #pragma unroll
      for (int bb = 0; bb < 3; ++bb) un[bb] = (float)u[bb];
      const float pn = (float)p;
      const R ur[3] = {(R)un[0], (R)un[1], (R)un[2]};
  #pragma unroll
      for (int i = 0; i < Q; ++i) {
        R hv[NC];
  #pragma unroll
        for (int c = 0; c < NC; ++c) hv[c] = h[c][i] - href3<R>(i, c, (R)En[c], ur);
        Pops<3, S>::store(a.pout, tuple_of<3>(i, n, N), N, a.sf, a.sh,
                          f[i] - fref3<R>(i, (R)pn, ur), hv);
      }
      Anchor3::store(a.pout, n, N, pn, un, En);
      Aux<3, R>::store(a.aux, n, N, chi, u);
    }
}

}  // namespace vflb
