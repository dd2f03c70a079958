// internal.h -- calls between the translation units of libvflb (not part of
// the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/vflb.h"

namespace vflb {
namespace internal {

// What a warm start needs to know of a simulation before (re)initialising
// it: shape, wall bits (bit a: walls on axis a), stream, lambda / eta_p
// (0 without polymer), and two device buffers it may use as scratch until
// then: the residual-snapshot buffer (FP32 fields of up to `bytes` bytes)
// and the second population buffer (`big`, `big_bytes`; 256 bytes in
// place).  Needs bound buffers and parameters.
struct SimScratch {
  int D, nx, ny, walls;
  hipStream_t stream;
  double lam_over_eta;
  void* scratch;
  size_t bytes;
  void* big;
  size_t big_bytes;
};
vflb_status sim_scratch(vflb_sim* s, SimScratch* out);

// vflb_init_fields from FP32 component-major device fields u [D][N] and
// tau [NC][N] (pressure 0).
vflb_status sim_init_f32(vflb_sim* s, const float* u, const float* tau);

// Settling: nsteps steps whose collisions use the prescribed FP32 fields
// targets = u [2][N] followed by tau [3][N] in place of the moment u
// (flags bit 0) and the moment A (bit 1) (D2Q9); the time level advances
// by nsteps.
vflb_status sim_settle_f32(vflb_sim* s, const float* targets, int64_t nsteps, int flags);

}  // namespace internal
}  // namespace vflb
