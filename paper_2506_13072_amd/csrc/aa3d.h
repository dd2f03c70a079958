// aa3d.h -- in-place (AA) streaming for D3Q19: one population buffer read
// and written in place, its layout alternating with the parity of t, as the
// D2Q9 in-place kernels of step2d.h.  A step at even t reads a node's
// pre-collision populations from its own slots and writes the
// post-collision values back under the opposite directions; a step at odd t
// reads each value where its writer left it (x - c_i, opposite direction;
// Geo::aa and pull_index) and writes into the slots the readers of the next
// step own (x + c_i, same direction; beyond a wall the node itself,
// opposite direction).  Every slot is read and written by one node within a
// step, so no ordering between workgroups is needed.  Neighbours' slots are
// overwritten during the step, so the same-time velocity for the gradient
// comes from a separate pass (aa3_velocity_kernel) into u(t) [3][N].  The
// split D3Q19 layout (layout.h: f planes, then the h tuples) lets that pass
// read the f planes alone.  One lane per node; the per-node arithmetic is
// the generic collision of lattice.h.
#pragma once

#include "kernels.h"

namespace vflb {

// tuple index of the slot that the reader of the next step expects f*_i of
// node (x, y, z) in (g.aa: the layout of the state being read, 1 or 2)
template <int D>
__device__ inline size_t aa_write_index(int i, int x, int y, int z, const Geo& g) {
  const size_t n = node_of(x, y, z, g);
  const int opp = Lat<D>::opp(i);
  if (g.aa == 1) return tuple_of<D>(opp, n, g.N);  // next state swapped: own node
  int t[3] = {x + cdir<D>(i, 0), y + cdir<D>(i, 1), z + cdir<D>(i, 2)};
  const int nn[3] = {g.nx, g.ny, g.nz};
#pragma unroll
  for (int a = 0; a < D; ++a)
    if ((g.walls & (1 << a)) && (t[a] < 0 || t[a] >= nn[a])) return tuple_of<D>(opp, n, g.N);
#pragma unroll
  for (int a = 0; a < D; ++a) t[a] = t[a] < 0 ? nn[a] - 1 : (t[a] >= nn[a] ? 0 : t[a]);
  return tuple_of<D>(i, node_of(t[0], t[1], t[2], g), g.N);
}

// u(t) = sum c f + F/2 of every node into U [3][N]
template <class S>
__global__ void __launch_bounds__(256) aa3_velocity_kernel(const S* __restrict__ pop, Geo g,
                                                           ForceArgs<typename StoreT<S>::R> fa,
                                                           typename StoreT<S>::R inv_sf,
                                                           typename StoreT<S>::R* __restrict__ U) {
  using R = typename StoreT<S>::R;
  using L = Lat<3>;
  const size_t N = g.N;
  for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    int x, y, z;
    node_xyz<3>(n, g, x, y, z);
    R m[3] = {0, 0, 0};
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
      const R fi = Pops<3, S>::load_f(pop, pull_index<3>(i, x, y, z, g), N, inv_sf);
#pragma unroll
      for (int b = 0; b < 3; ++b)
        if (cdir<3>(i, b) != 0) m[b] += (R)cdir<3>(i, b) * fi;
    }
    R F[3];
    force_at<R>(fa, x, y, z, g, F);
#pragma unroll
    for (int b = 0; b < 3; ++b) U[(size_t)b * N + n] = m[b] + (R)0.5 * F[b];
  }
}

// The in-place step: pull, moments, collision of f and h with the gradient
// of u(t) from U (central differences; at a halfway bounce-back wall the
// parabola through the wall value 0 and the first two nodes), write back.
template <class S>
__global__ void __launch_bounds__(256) aa3_step_kernel(StepArgs<S> a,
                                                       const typename StoreT<S>::R* __restrict__ U) {
  using R = typename StoreT<S>::R;
  using L = Lat<3>;
  constexpr int Q = L::Q, NC = L::NC;
  const Geo g = a.g;
  S* __restrict__ pop = a.pout;
  R* __restrict__ aux = a.aux;
  const size_t N = g.N;
  for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    int x, y, z;
    node_xyz<3>(n, g, x, y, z);
    R f[Q], h[NC][Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      R hv[NC];
      Pops<3, S>::load(pop, pull_index<3>(i, x, y, z, g), N, a.inv_sf, a.inv_sh, f[i], hv);
#pragma unroll
      for (int c = 0; c < NC; ++c) h[c][i] = hv[c];
    }
    R chip[NC] = {0, 0, 0, 0, 0, 0}, up[3] = {0, 0, 0};
    if (!a.first) Aux<3, R>::load(aux, n, N, chip, up);
    R F[3];
    force_at<R>(a.F, x, y, z, g, F);
    const R u[3] = {U[n], U[N + n], U[2 * N + n]};
    R e[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      R s = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) s += h[c][i];
      e[c] = s;
    }
    collide_f<3, R>(f, e, u, F, a.P);
    // same-time velocity gradient G[a][b] = d_a u_b
    const int c3[3] = {x, y, z}, n3[3] = {g.nx, g.ny, g.nz};
    const size_t st[3] = {1, (size_t)g.nx, (size_t)g.nx * g.ny};
    R G[3][3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const bool wall = g.walls & (1 << ax);
      const bool lo = wall && c3[ax] == 0, hi = wall && c3[ax] == n3[ax] - 1;
      const size_t nm = c3[ax] == 0 ? n + (size_t)(n3[ax] - 1) * st[ax] : n - st[ax];
      const size_t np = c3[ax] == n3[ax] - 1 ? n - (size_t)(n3[ax] - 1) * st[ax] : n + st[ax];
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const R um = U[(size_t)b * N + nm], upl = U[(size_t)b * N + np];
        G[ax][b] = lo ? u[b] + upl * (R)(1.0 / 3.0)
                 : hi ? -(u[b] + um * (R)(1.0 / 3.0))
                      : (R)0.5 * (upl - um);
      }
    }
    R chi[NC];
    source_tensor<3, R>(e, G, a.P, chi);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const R Ac = e[c] + ((L::ca(c) == L::cb(c)) ? (R)1 : (R)0);
      collide_h<3, R>(h[c], e[c], Ac, chi[c], chip[c], u, up, a.first != 0, a.P);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      R hv[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) hv[c] = h[c][i];
      Pops<3, S>::store(pop, aa_write_index<3>(i, x, y, z, g), N, a.sf, a.sh, f[i], hv);
    }
    Aux<3, R>::store(aux, n, N, chi, u);
  }
}

}  // namespace vflb
