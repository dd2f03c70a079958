// aa3d.h -- the velocity pass of in-place (AA) streaming for D3Q19.  One
// population buffer is read and written in place, its layout alternating
// with the parity of t (Geo::aa, pull_index): a step at even t reads a
// node's pre-collision populations from its own slots and writes the
// post-collision values back under the opposite directions; a step at odd t
// reads each value where its writer left it (x - c_i, opposite direction)
// and writes into the slots the readers of the next step own (x + c_i, same
// direction; beyond a wall the node itself, opposite direction).  Every
// slot is read and written by one node within a step.  Neighbours' slots
// are overwritten during the step, so the same-time velocity for the
// gradient comes from this separate pass into u(t) [3][N]; the step itself
// is the z-march of step3d.h with the same maps in pair form (its AA
// branch, aa_pair_src / aa_pair_dst).  The split D3Q19 layout (layout.h: f
// planes, then the h tuples) lets this pass read the f planes alone.
#pragma once

#include "kernels.h"

namespace vflb {

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

}  // namespace vflb
