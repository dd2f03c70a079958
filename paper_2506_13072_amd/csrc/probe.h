// probe.h -- copy kernels that move a known number of bytes: the achievable
// HBM copy rate, and the conversion of the hardware byte counters into
// bytes for each kind of access the step kernels make (counters can count
// requests of different widths differently).  Not part of the method.
#pragma once

#include "step3d.h"

namespace vflb {

typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));

// non-temporal 16-byte loads and stores: the streaming copy
__global__ void __launch_bounds__(256) stream_copy_kernel(const v4u32* __restrict__ src,
                                                          v4u32* __restrict__ dst, size_t n) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + k), dst + k);
}
// plain 16-byte loads and stores
__global__ void __launch_bounds__(256) copy_plain16_kernel(const v4u32* __restrict__ src,
                                                           v4u32* __restrict__ dst, size_t n) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = src[k];
}
// plain 4-byte loads and stores
__global__ void __launch_bounds__(256) copy_plain4_kernel(const uint32_t* __restrict__ src,
                                                          uint32_t* __restrict__ dst, size_t n) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = src[k];
}
// 16-byte loads by LDS-DMA (global_load_lds) into the wave's LDS block, each
// lane then stores its own slot with a non-temporal store (the step
// kernels' stage path)
__global__ void __launch_bounds__(256) copy_lds16_kernel(const v4u32* __restrict__ src,
                                                         v4u32* __restrict__ dst, size_t n) {
  __shared__ v4u32 buf[256];
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int wave = threadIdx.x >> 6;
  if (k < n) dma_to_lds<16>(src + k, &buf[wave * 64]);
  __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
  if (k < n) __builtin_nontemporal_store(buf[threadIdx.x], dst + k);
}

}  // namespace vflb
