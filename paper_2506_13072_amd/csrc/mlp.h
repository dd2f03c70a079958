// mlp.h -- device kernels of the warm-start network (gfx950).
//
// A Fourier-feature MLP maps a point and the flow parameters to the steady
// fields: x -> phi(x) = [sin 2 pi B x, cos 2 pi B x] -> tanh layers of width
// W -> a linear output layer.  Every product is one "NT" GEMM on the matrix
// cores, C[m][n] = sum_k A[m][k] B[n][k] with both operands K-contiguous in
// BF16 and FP32 accumulation (v_mfma_f32_16x16x32_bf16), and the epilogue
// of each GEMM writes what the next kernel consumes: activations in FP32
// and BF16, in both orientations (the weight gradients contract over the
// batch, so they read the transposed copies as K-contiguous operands).
// Reductions run in a fixed order: results are independent of timing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vflb {
namespace mlp {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 32, LDS_K = BK + 8;  // +8: spread LDS banks

enum Epi {
  EPI_TANH = 0,     // h = tanh(acc + bias): H32[m][n], H16[m][n], HT16[n][m]
  EPI_LINEAR = 1,   // y = acc + bias: Y32[m][n]
  EPI_DTANH = 2,    // dz = acc * (1 - h^2), h = H32[m][n]: D16[m][n], DT16[n][m]
  EPI_PARTIAL = 3   // P[z][m][n] = acc (split-K partial)
};

struct GemmArgs {
  const bf16* A;  // [M][lda], rows m, K contiguous
  const bf16* B;  // [N][ldb], rows n, K contiguous
  int M, N, K;    // multiples of BM, BN, BK
  int lda, ldb;
  int ksplit;     // K range per blockIdx.z
  const float* bias;  // EPI_TANH, EPI_LINEAR
  const float* H32;   // EPI_DTANH: activations of this layer [M][ldc]
  float* out32;       // EPI_TANH: H32, EPI_LINEAR: Y32, EPI_PARTIAL: P
  bf16* out16;        // EPI_TANH: H16, EPI_DTANH: D16
  bf16* outT16;       // EPI_TANH: HT16, EPI_DTANH: DT16  ([N][ldt])
  int ldc, ldt;
};

// One 64 x 64 output tile per workgroup of four wavefronts; wavefront w
// computes the 32 x 32 quarter (w / 2, w % 2) as 2 x 2 blocks of 16 x 16.
// Operand fragments of v_mfma_f32_16x16x32_bf16: lane l holds row l % 16 of
// its 16-row block and the 8 consecutive k at 8 (l / 16); the result of lane
// l is rows 4 (l / 16) + r, r = 0..3, of column l % 16.
template <int EPI>
__global__ void __launch_bounds__(256) gemm_nt_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) bf16 As[BM][LDS_K];
  __shared__ __attribute__((aligned(16))) bf16 Bs[BN][LDS_K];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int kbeg = blockIdx.z * g.ksplit, kend = min(g.K, kbeg + g.ksplit);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
  // global -> LDS: thread t moves 8 consecutive k of row t / 4
  const int lr = tid >> 2, lk = (tid & 3) * 8;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    *reinterpret_cast<bf16x8*>(&As[lr][lk]) =
        *reinterpret_cast<const bf16x8*>(g.A + (size_t)(m0 + lr) * g.lda + k0 + lk);
    *reinterpret_cast<bf16x8*>(&Bs[lr][lk]) =
        *reinterpret_cast<const bf16x8*>(g.B + (size_t)(n0 + lr) * g.ldb + k0 + lk);
    __syncthreads();
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    bf16x8 af[2], bfr[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) af[i] = *reinterpret_cast<const bf16x8*>(&As[wm + 16 * i + fr][fk]);
#pragma unroll
    for (int j = 0; j < 2; ++j) bfr[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn + 16 * j + fr][fk]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  // epilogue
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn + 16 * j + (lane & 15);
      const int mb = m0 + wm + 16 * i + 4 * (lane >> 4);
      float v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = acc[i][j][r];
      if (EPI == EPI_PARTIAL) {
        float* P = g.out32 + (size_t)blockIdx.z * g.M * g.ldc;
#pragma unroll
        for (int r = 0; r < 4; ++r) P[(size_t)(mb + r) * g.ldc + n] = v[r];
      } else if (EPI == EPI_LINEAR) {
        const float b = g.bias[n];
#pragma unroll
        for (int r = 0; r < 4; ++r) g.out32[(size_t)(mb + r) * g.ldc + n] = v[r] + b;
      } else {
        bf16 t[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float o;
          if (EPI == EPI_TANH) {
            o = tanhf(v[r] + g.bias[n]);
            g.out32[(size_t)(mb + r) * g.ldc + n] = o;
          } else {  // EPI_DTANH
            const float h = g.H32[(size_t)(mb + r) * g.ldc + n];
            o = v[r] * (1.0f - h * h);
          }
          t[r] = (bf16)o;
          g.out16[(size_t)(mb + r) * g.ldc + n] = t[r];
        }
        // transposed copy: the lane's four rows are consecutive in m
        bf16* T = g.outT16 + (size_t)n * g.ldt + mb;
#pragma unroll
        for (int r = 0; r < 4; ++r) T[r] = t[r];
      }
    }
}

// Fourier features of rows [0, n) of x (FP32 [rows][in_dim]); rows up to
// `rows` (the padded batch) are zero.  phi[m][f] = sin(2 pi b_f . x_m),
// phi[m][nf + f] = cos(2 pi b_f . x_m), in BF16 and transposed.
__global__ void __launch_bounds__(256) features_kernel(const float* __restrict__ x, int n,
                                                       int rows, int in_dim,
                                                       const float* __restrict__ freq, int nf,
                                                       bf16* __restrict__ phi,
                                                       bf16* __restrict__ phiT) {
  const int m = blockIdx.x, f = threadIdx.x;
  if (f >= nf) return;
  float sv = 0.0f, cv = 0.0f;
  if (m < n) {
    float z = 0.0f;
    for (int d = 0; d < in_dim; ++d) z += freq[f * in_dim + d] * x[(size_t)m * in_dim + d];
    z *= 6.283185307179586f;
    sv = sinf(z);
    cv = cosf(z);
  }
  const bf16 s16 = (bf16)sv, c16 = (bf16)cv;
  phi[(size_t)m * 2 * nf + f] = s16;
  phi[(size_t)m * 2 * nf + nf + f] = c16;
  phiT[(size_t)f * rows + m] = s16;
  phiT[(size_t)(nf + f) * rows + m] = c16;
}

// Loss 1/(n out) sum (y - t)^2 over the valid rows and outputs, and its
// gradient dY = 2 (y - t)/(n out) (zero in padding), BF16 both ways.
// One workgroup per 256 rows; loss partial per workgroup.
__global__ void __launch_bounds__(256) loss_kernel(const float* __restrict__ Y, int ldy,
                                                   const float* __restrict__ T, int n, int out,
                                                   int rows, bf16* __restrict__ dY,
                                                   bf16* __restrict__ dYT, int ncol,
                                                   double* __restrict__ part) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  double l = 0.0;
  if (m < rows) {
    const float scale = 2.0f / ((float)n * (float)out);
    for (int c = 0; c < ncol; ++c) {
      float g = 0.0f;
      if (m < n && c < out) {
        const float d = Y[(size_t)m * ldy + c] - T[(size_t)m * out + c];
        l += (double)d * d;
        g = scale * d;
      }
      const bf16 g16 = (bf16)g;
      dY[(size_t)m * ncol + c] = g16;
      dYT[(size_t)c * rows + m] = g16;
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[r] = sum over m of src[r][m] (BF16, rows of length `len`), FP32
// accumulation in a fixed order: lane j takes m = j, j + 256, ...
__global__ void __launch_bounds__(256) rowsum_kernel(const bf16* __restrict__ src, int len,
                                                     float* __restrict__ out) {
  const int r = blockIdx.x;
  float s = 0.0f;
  for (int m = threadIdx.x; m < len; m += 256) s += (float)src[(size_t)r * len + m];
  __shared__ float red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = red[0];
}

// G[i] = sum over z of P[z][i], z in order (split-K partials).
__global__ void __launch_bounds__(256) splitk_sum_kernel(const float* __restrict__ P, int nz,
                                                         size_t stride, size_t count,
                                                         float* __restrict__ G) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  float s = 0.0f;
  for (int z = 0; z < nz; ++z) s += P[(size_t)z * stride + i];
  G[i] = s;
}

// Sum of fixed-order partials into one double.
__global__ void sum_kernel(const double* __restrict__ part, int n, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  *out = s;
}

// Adam on one layer: W [out][in] and b [out] in FP32 with their moments,
// gradients G [gld rows][in] (only the first `out` rows used) and gb; writes
// the BF16 copies W16 [out_pad][in] and WT16 [in][out_pad].
struct AdamArgs {
  float* W;
  float* b;
  float *mW, *vW, *mb, *vb;
  const float* G;
  const float* gb;
  bf16* W16;
  bf16* WT16;
  int out, in, out_pad;
  float lr, beta1, beta2, eps, c1, c2;  // c1 = 1 - beta1^t, c2 = 1 - beta2^t
};

__device__ inline float adam_one(float& w, float& m, float& v, float g, const AdamArgs& a) {
  m = a.beta1 * m + (1.0f - a.beta1) * g;
  v = a.beta2 * v + (1.0f - a.beta2) * g * g;
  const float mh = m / a.c1, vh = v / a.c2;
  w -= a.lr * mh / (sqrtf(vh) + a.eps);
  return w;
}

__global__ void __launch_bounds__(256) adam_kernel(AdamArgs a) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int nw = a.out * a.in;
  if (i < nw) {
    const int o = i / a.in, k = i % a.in;
    const float w = adam_one(a.W[i], a.mW[i], a.vW[i], a.G[(size_t)o * a.in + k], a);
    const bf16 w16 = (bf16)w;
    a.W16[(size_t)o * a.in + k] = w16;
    a.WT16[(size_t)k * a.out_pad + o] = w16;
  } else if (i < nw + a.out) {
    const int o = i - nw;
    adam_one(a.b[o], a.mb[o], a.vb[o], a.gb[o], a);
  }
}

// BF16 copies of one layer's weights (after an upload of FP32 values).
__global__ void __launch_bounds__(256) cast_layer_kernel(const float* __restrict__ W, int out,
                                                         int in, int out_pad,
                                                         bf16* __restrict__ W16,
                                                         bf16* __restrict__ WT16) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= out_pad * in) return;
  const int o = i / in, k = i % in;
  const bf16 w16 = (bf16)(o < out ? W[(size_t)o * in + k] : 0.0f);
  W16[(size_t)o * in + k] = w16;
  WT16[(size_t)k * out_pad + o] = w16;
}

// Per-output mean and standard deviation of the targets T [n][out] (FP64,
// two passes, fixed order; one workgroup per output column): stats[c] the
// mean, stats[out + c] the standard deviation (1 where it is 0).
__global__ void __launch_bounds__(256) col_stats_kernel(const float* __restrict__ T, int64_t n,
                                                        int out, double* __restrict__ stats) {
  const int c = blockIdx.x;
  __shared__ double red[256];
  auto block_sum = [&](double v) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
  };
  double s = 0.0;
  for (int64_t m = threadIdx.x; m < n; m += 256) s += (double)T[m * out + c];
  const double mean = block_sum(s) / (double)n;
  double q = 0.0;
  for (int64_t m = threadIdx.x; m < n; m += 256) {
    const double d = (double)T[m * out + c] - mean;
    q += d * d;
  }
  const double var = block_sum(q) / (double)n;
  if (threadIdx.x == 0) {
    stats[c] = mean;
    stats[out + c] = var > 0.0 ? sqrt(var) : 1.0;
  }
}

// A random minibatch of `rows` rows of (X [n][in_dim], T [n][out]): row r
// takes sample floor(z n / 2^64), z the output of position key + r of the
// SplitMix64 stream (Steele, Lea, Flood 2014; counter-based, so every row is
// drawn independently of the launch shape); targets standardised with
// stats (mean, std).
__global__ void __launch_bounds__(256) gather_kernel(const float* __restrict__ X,
                                                     const float* __restrict__ T, int64_t n,
                                                     int in_dim, int out, int rows,
                                                     uint64_t seed, uint64_t key,
                                                     const double* __restrict__ stats,
                                                     float* __restrict__ xb,
                                                     float* __restrict__ tb) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  uint64_t z = seed + (key + (uint64_t)r + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const int64_t m = (int64_t)__umul64hi(z, (uint64_t)n);
  for (int d = 0; d < in_dim; ++d) xb[(size_t)r * in_dim + d] = X[m * in_dim + d];
  for (int c = 0; c < out; ++c)
    tb[(size_t)r * out + c] =
        (float)(((double)T[m * out + c] - stats[c]) / stats[out + c]);
}

// Fold the target standardisation into the output layer (W [out][in],
// b [out], FP32): the network then predicts std * y + mean.
__global__ void __launch_bounds__(256) fold_output_kernel(float* __restrict__ W,
                                                          float* __restrict__ b, int out, int in,
                                                          const double* __restrict__ stats) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < out * in) {
    W[i] = (float)((double)W[i] * stats[out + i / in]);
  } else if (i < out * in + out) {
    const int o = i - out * in;
    b[o] = (float)((double)b[o] * stats[out + o] + stats[o]);
  }
}

// Network inputs of the nodes [n0, n0 + cnt) of an nx x ny lattice:
// (x / nx, y / ny, extra[0], extra[1], extra[2]).
__global__ void __launch_bounds__(256) node_inputs_kernel(int nx, int ny, size_t n0, int cnt,
                                                          float e0, float e1, float e2,
                                                          float* __restrict__ x) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= cnt) return;
  const size_t n = n0 + (size_t)j;
  float* r = x + (size_t)j * 5;
  r[0] = (float)(n % (size_t)nx) / (float)nx;
  r[1] = (float)(n / (size_t)nx) / (float)ny;
  r[2] = e0;
  r[3] = e1;
  r[4] = e2;
}

// Network outputs (u/U, v/U, txx/S, txy/S, tyy/S) of nodes [n0, n0 + cnt)
// into the component-major fields u [2][N], tau [3][N] (FP32).
__global__ void __launch_bounds__(256) node_outputs_kernel(const float* __restrict__ y, int ldy,
                                                           size_t n0, int cnt, size_t N,
                                                           float u_scale, float tau_scale,
                                                           float* __restrict__ u,
                                                           float* __restrict__ tau) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= cnt) return;
  const size_t n = n0 + (size_t)j;
  const float* r = y + (size_t)j * ldy;
  u[n] = u_scale * r[0];
  u[N + n] = u_scale * r[1];
  tau[n] = tau_scale * r[2];
  tau[N + n] = tau_scale * r[3];
  tau[2 * N + n] = tau_scale * r[4];
}

// ---------------------------------------------------------------------
// Projection of a predicted velocity onto the discretely solenoidal fields
// of a periodic nx x ny lattice.  The step's velocity gradient is the
// central difference, whose Fourier symbol is i (sin kx, sin ky); the
// projection removes the part of each mode along that symbol (its central
// divergence), and the four modes where the symbol vanishes: the mean
// (kx, ky) = (0, 0), whose momentum a fully periodic lattice conserves, and
// (pi, 0), (0, pi), (pi, pi), which the gradient cannot see and on which
// streaming flips the sign of the momentum every step (the staggered
// momentum is conserved up to sign), so that a prediction carrying them
// would keep them for good.  Both are absent from a start from rest.
// Naive separable DFTs (n <= 512 per axis): complex FP32 fields, FP64 sums.

// real [ncomp][N] -> complex
__global__ void __launch_bounds__(256) to_complex_kernel(const float* __restrict__ in, size_t cnt,
                                                         float2* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < cnt) out[i] = make_float2(in[i], 0.0f);
}

// One DFT pass of ncomp complex fields [ncomp][ny][nx] along x (axis 0) or
// y (axis 1) with exponent sign sgn: out(k) = sum_j in(j) exp(sgn 2 pi i k j / n).
__global__ void __launch_bounds__(256) dft_pass_kernel(const float2* __restrict__ in,
                                                       float2* __restrict__ out, int nx, int ny,
                                                       int ncomp, int axis, int sgn) {
  const size_t N = (size_t)nx * ny, idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)ncomp * N) return;
  const size_t c = idx / N, r = idx % N;
  const int y = (int)(r / nx), x = (int)(r % nx);
  const int n = axis == 0 ? nx : ny, k = axis == 0 ? x : y;
  const float2* src = in + c * N;
  double re = 0.0, im = 0.0;
  for (int j = 0; j < n; ++j) {
    const float2 v = axis == 0 ? src[(size_t)y * nx + j] : src[(size_t)j * nx + x];
    const long long m = ((long long)k * j) % n;
    double sn, cs;
    sincospi(2.0 * (double)m / (double)n, &sn, &cs);
    sn *= (double)sgn;
    re += (double)v.x * cs - (double)v.y * sn;
    im += (double)v.x * sn + (double)v.y * cs;
  }
  out[idx] = make_float2((float)re, (float)im);
}

// Remove from U [2][ny][nx] (spectrum of u) its part along the central
// difference symbol, the mean, and the Nyquist lines kx = pi and ky = pi
// (a smooth flow has no content there; streaming flips the sign of the
// momentum of the kx = pi line every step, so its sum over the lattice is
// kept up to sign).
__global__ void __launch_bounds__(256) solenoidal_kernel(float2* __restrict__ U, int nx, int ny) {
  const size_t N = (size_t)nx * ny, r = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= N) return;
  const int ky = (int)(r / nx), kx = (int)(r % nx);
  const double sx = sinpi(2.0 * kx / nx), sy = sinpi(2.0 * ky / ny);
  const bool blind = (kx == 0 && ky == 0) || 2 * kx == nx || 2 * ky == ny;
  const float2 a = U[r], b = U[N + r];
  if (blind) {
    U[r] = make_float2(0.0f, 0.0f);
    U[N + r] = make_float2(0.0f, 0.0f);
    return;
  }
  const double ss = sx * sx + sy * sy;
  const double dr = (sx * a.x + sy * b.x) / ss, di = (sx * a.y + sy * b.y) / ss;
  U[r] = make_float2((float)(a.x - sx * dr), (float)(a.y - sx * di));
  U[N + r] = make_float2((float)(b.x - sy * dr), (float)(b.y - sy * di));
}

// On a lattice with walls: remove from u [2][N] the alternating component
// (-1)^c along each periodic axis of even length (axis 0: x, 1: y), line by
// line: its momentum along that axis is kept up to sign by streaming, also
// next to halfway bounce-back walls on the other axis.  One lane per line.
__global__ void __launch_bounds__(256) remove_alternating_kernel(float* __restrict__ u, int nx,
                                                                 int ny, int axis) {
  const int line = blockIdx.x * 256 + threadIdx.x;
  const int nl = axis == 0 ? ny : nx, n = axis == 0 ? nx : ny;
  if (line >= nl) return;
  const size_t N = (size_t)nx * ny;
  for (int c = 0; c < 2; ++c) {
    float* f = u + (size_t)c * N;
    auto at = [&](int j) -> float& {
      return axis == 0 ? f[(size_t)line * nx + j] : f[(size_t)j * nx + line];
    };
    double a = 0.0;
    for (int j = 0; j < n; ++j) a += (j & 1) ? -(double)at(j) : (double)at(j);
    a /= (double)n;
    for (int j = 0; j < n; ++j) at(j) = (float)((double)at(j) - ((j & 1) ? -a : a));
  }
}

// real part / N back into u [2][N]
__global__ void __launch_bounds__(256) from_complex_kernel(const float2* __restrict__ in,
                                                           size_t cnt, double inv_n,
                                                           float* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < cnt) out[i] = (float)((double)in[i].x * inv_n);
}

// Keep the predicted conformation tensor A = I + c tau (c = lambda/eta_p)
// positive definite, as Oldroyd-B keeps it: its eigenvalues are raised to
// at least a_min, eigenvectors kept; tau [3][N] (xx, xy, yy) rewritten.
__global__ void __launch_bounds__(256) conformation_floor_kernel(float* __restrict__ tau, size_t N,
                                                                 double c, double a_min) {
  const size_t n = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  const double axx = 1.0 + c * tau[n], axy = c * tau[N + n], ayy = 1.0 + c * tau[2 * N + n];
  const double m = 0.5 * (axx + ayy), d = 0.5 * (axx - ayy), r = sqrt(d * d + axy * axy);
  const double l1 = m + r, l2 = m - r;
  if (l2 >= a_min) return;
  const double m1 = l1 > a_min ? l1 : a_min, m2 = a_min;
  // A' = m1 e1 e1^T + m2 e2 e2^T, e1 the eigenvector of l1
  double ex = 1.0, ey = 0.0;
  if (r > 0) {
    const double th = 0.5 * atan2(2.0 * axy, axx - ayy);
    ex = cos(th);
    ey = sin(th);
  }
  const double bxx = m1 * ex * ex + m2 * ey * ey, bxy = (m1 - m2) * ex * ey,
               byy = m1 * ey * ey + m2 * ex * ex;
  tau[n] = (float)((bxx - 1.0) / c);
  tau[N + n] = (float)(bxy / c);
  tau[2 * N + n] = (float)((byy - 1.0) / c);
}

}  // namespace mlp
}  // namespace vflb
