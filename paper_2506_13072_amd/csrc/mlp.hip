// mlp.hip -- host side of the warm-start network: the vflb_mlp_* part of
// the C ABI declared in include/vflb.h, and vflb_init_from_mlp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/vflb.h"
#include "internal.h"
#include "mlp.h"

using namespace vflb::mlp;

struct vflb_mlp {
  vflb_mlp_cfg cfg{};
  hipStream_t stream = nullptr;
  void* buf[VFLB_MLP_NBUF] = {};
  size_t bytes[VFLB_MLP_NBUF] = {};
  bool bound = false, have_params = false;
  int nl = 0;                        // layers (hidden + output)
  std::vector<int> lin, lout, lpad;  // fan-in, fan-out, padded fan-out
  size_t nparams = 0;
  // PARAMS buffer (byte offsets)
  size_t off_freq = 0;
  std::vector<size_t> oW, ob, omW, ovW, omb, ovb, oW16, oWT16, oG, ogb;
  // WORK buffer (byte offsets)
  size_t off_x = 0, off_phi = 0, off_phiT = 0, off_Y = 0, off_dY = 0, off_dYT = 0, off_P = 0,
         off_lpart = 0, off_loss = 0, off_tb = 0, off_stats = 0;
  std::vector<size_t> oH32, oH16, oHT16;
  size_t off_dZ[2] = {0, 0}, off_dZT[2] = {0, 0};
  size_t p_floats = 0;  // capacity of the split-K partial buffer
  int64_t adam_t = 0;
  std::string err;

  char* P() const { return static_cast<char*>(buf[VFLB_MLP_BUF_PARAMS]); }
  char* Wk() const { return static_cast<char*>(buf[VFLB_MLP_BUF_WORK]); }
  template <class T> T* p(size_t off) const { return reinterpret_cast<T*>(P() + off); }
  template <class T> T* w(size_t off) const { return reinterpret_cast<T*>(Wk() + off); }
};

namespace {

thread_local std::string g_mlp_create_error;
constexpr int kOutPad = 64;   // padded width of the output layer
constexpr int kMaxSplit = 32; // split-K slices of the weight gradients
// smallest eigenvalue of a predicted conformation tensor (A = I at rest)
constexpr double kConformationFloor = 0.05;

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

vflb_status mfail(vflb_mlp* m, vflb_status code, const char* fmt, ...) {
  char msg[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(msg, sizeof msg, fmt, ap);
  va_end(ap);
  if (m)
    m->err = msg;
  else
    g_mlp_create_error = msg;
  return code;
}

#define MHIP_TRY(m, call)                                                  \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess)                                                  \
      return mfail((m), VFLB_EDEVICE, "%s failed: %s", #call,              \
                   hipGetErrorString(e_));                                 \
  } while (0)

// SplitMix64 (Steele, Lea, Flood 2014) and uniform / normal draws from it
struct SplitMix {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
  double normal() {  // Box-Muller
    double u1 = uniform();
    if (u1 < 1e-300) u1 = 1e-300;
    const double u2 = uniform();
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

int rows_of(int64_t n) { return (int)((n + 63) / 64 * 64); }

vflb_status gemm(vflb_mlp* m, int epi, const GemmArgs& g, int splits) {
  dim3 grid(g.N / BN, g.M / BM, splits);
  switch (epi) {
    case EPI_TANH: hipLaunchKernelGGL(gemm_nt_kernel<EPI_TANH>, grid, dim3(256), 0, m->stream, g); break;
    case EPI_LINEAR: hipLaunchKernelGGL(gemm_nt_kernel<EPI_LINEAR>, grid, dim3(256), 0, m->stream, g); break;
    case EPI_DTANH: hipLaunchKernelGGL(gemm_nt_kernel<EPI_DTANH>, grid, dim3(256), 0, m->stream, g); break;
    default: hipLaunchKernelGGL(gemm_nt_kernel<EPI_PARTIAL>, grid, dim3(256), 0, m->stream, g); break;
  }
  MHIP_TRY(m, hipGetLastError());
  return VFLB_OK;
}

// forward pass over `rows` padded rows of which n are valid; x [n][in_dim]
vflb_status forward(vflb_mlp* m, const float* x, int64_t n, int rows) {
  const int nf = m->cfg.n_freq;
  hipLaunchKernelGGL(features_kernel, dim3(rows), dim3(256), 0, m->stream, x, (int)n, rows,
                     m->cfg.in_dim, m->p<float>(m->off_freq), nf, m->w<bf16>(m->off_phi),
                     m->w<bf16>(m->off_phiT));
  MHIP_TRY(m, hipGetLastError());
  for (int l = 0; l < m->nl; ++l) {
    GemmArgs g{};
    g.A = l == 0 ? m->w<bf16>(m->off_phi) : m->w<bf16>(m->oH16[l - 1]);
    g.lda = m->lin[l];
    g.B = m->p<bf16>(m->oW16[l]);
    g.ldb = m->lin[l];
    g.M = rows;
    g.N = m->lpad[l];
    g.K = m->lin[l];
    g.ksplit = g.K;
    g.bias = m->p<float>(m->ob[l]);
    const bool last = l == m->nl - 1;
    if (last) {
      g.out32 = m->w<float>(m->off_Y);
      g.ldc = kOutPad;
    } else {
      g.out32 = m->w<float>(m->oH32[l]);
      g.out16 = m->w<bf16>(m->oH16[l]);
      g.outT16 = m->w<bf16>(m->oHT16[l]);
      g.ldc = m->lpad[l];
      g.ldt = rows;
    }
    vflb_status rc = gemm(m, last ? EPI_LINEAR : EPI_TANH, g, 1);
    if (rc != VFLB_OK) return rc;
  }
  return VFLB_OK;
}

// weight gradient of layer l: G[out_pad][in] = D^T X over the rows
vflb_status weight_grad(vflb_mlp* m, int l, const bf16* DT, const bf16* XT, int rows) {
  int splits = rows / 512;
  if (splits < 1) splits = 1;
  if (splits > kMaxSplit) splits = kMaxSplit;
  int ks = (rows + splits - 1) / splits;
  ks = (ks + BK - 1) / BK * BK;
  splits = (rows + ks - 1) / ks;
  GemmArgs g{};
  g.A = DT;
  g.lda = rows;
  g.B = XT;
  g.ldb = rows;
  g.M = m->lpad[l];
  g.N = m->lin[l];
  g.K = rows;
  g.ksplit = ks;
  g.out32 = m->w<float>(m->off_P);
  g.ldc = m->lin[l];
  vflb_status rc = gemm(m, EPI_PARTIAL, g, splits);
  if (rc != VFLB_OK) return rc;
  const size_t count = (size_t)g.M * g.N;
  hipLaunchKernelGGL(splitk_sum_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                     m->stream, m->w<float>(m->off_P), splits, count, count,
                     m->p<float>(m->oG[l]));
  MHIP_TRY(m, hipGetLastError());
  return VFLB_OK;
}

// loss and gradients for rows [0, n) (targets t [n][out_dim]); the loss
// (sum of squares / (n out)) lands in WORK at off_loss
vflb_status backward(vflb_mlp* m, const float* t, int64_t n, int rows) {
  const int L = m->nl - 1;
  const int nb = (rows + 255) / 256;
  hipLaunchKernelGGL(loss_kernel, dim3(nb), dim3(256), 0, m->stream, m->w<float>(m->off_Y),
                     kOutPad, t, (int)n, m->cfg.out_dim, rows, m->w<bf16>(m->off_dY),
                     m->w<bf16>(m->off_dYT), kOutPad, m->w<double>(m->off_lpart));
  MHIP_TRY(m, hipGetLastError());
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(64), 0, m->stream, m->w<double>(m->off_lpart), nb,
                     m->w<double>(m->off_loss));
  MHIP_TRY(m, hipGetLastError());
  // output layer
  const bf16* XT = L == 0 ? m->w<bf16>(m->off_phiT) : m->w<bf16>(m->oHT16[L - 1]);
  vflb_status rc = weight_grad(m, L, m->w<bf16>(m->off_dYT), XT, rows);
  if (rc != VFLB_OK) return rc;
  hipLaunchKernelGGL(rowsum_kernel, dim3(kOutPad), dim3(256), 0, m->stream,
                     m->w<bf16>(m->off_dYT), rows, m->p<float>(m->ogb[L]));
  MHIP_TRY(m, hipGetLastError());
  const bf16* Dcur = m->w<bf16>(m->off_dY);  // gradient at the output of layer l + 1
  int cur = 0;
  for (int l = L - 1; l >= 0; --l) {
    // dZ_l = (D_{l+1} W_{l+1}) * (1 - h_l^2)
    GemmArgs g{};
    g.A = Dcur;
    g.lda = m->lpad[l + 1];
    g.B = m->p<bf16>(m->oWT16[l + 1]);
    g.ldb = m->lpad[l + 1];
    g.M = rows;
    g.N = m->lin[l + 1];
    g.K = m->lpad[l + 1];
    g.ksplit = g.K;
    g.H32 = m->w<float>(m->oH32[l]);
    g.out16 = m->w<bf16>(m->off_dZ[cur]);
    g.outT16 = m->w<bf16>(m->off_dZT[cur]);
    g.ldc = m->lin[l + 1];
    g.ldt = rows;
    if ((rc = gemm(m, EPI_DTANH, g, 1)) != VFLB_OK) return rc;
    const bf16* Xl = l == 0 ? m->w<bf16>(m->off_phiT) : m->w<bf16>(m->oHT16[l - 1]);
    if ((rc = weight_grad(m, l, m->w<bf16>(m->off_dZT[cur]), Xl, rows)) != VFLB_OK) return rc;
    hipLaunchKernelGGL(rowsum_kernel, dim3(m->lpad[l]), dim3(256), 0, m->stream,
                       m->w<bf16>(m->off_dZT[cur]), rows, m->p<float>(m->ogb[l]));
    MHIP_TRY(m, hipGetLastError());
    Dcur = m->w<bf16>(m->off_dZ[cur]);
    cur ^= 1;
  }
  return VFLB_OK;
}

vflb_status need_mlp(vflb_mlp* m) {
  if (!m) return VFLB_EINVAL;
  if (!m->bound) return mfail(m, VFLB_ESTATE, "device buffers are not bound");
  if (!m->have_params) return mfail(m, VFLB_ESTATE, "parameters are not initialised");
  return VFLB_OK;
}

vflb_status recast(vflb_mlp* m) {
  for (int l = 0; l < m->nl; ++l) {
    const int cnt = m->lpad[l] * m->lin[l];
    hipLaunchKernelGGL(cast_layer_kernel, dim3((cnt + 255) / 256), dim3(256), 0, m->stream,
                       m->p<float>(m->oW[l]), m->lout[l], m->lin[l], m->lpad[l],
                       m->p<bf16>(m->oW16[l]), m->p<bf16>(m->oWT16[l]));
    MHIP_TRY(m, hipGetLastError());
  }
  return VFLB_OK;
}

// upload flat host parameters (freq, then W, b per layer), zero Adam state
vflb_status upload(vflb_mlp* m, const float* host) {
  const vflb_mlp_cfg& c = m->cfg;
  size_t k = 0;
  MHIP_TRY(m, hipMemcpyAsync(m->p<float>(m->off_freq), host, sizeof(float) * c.n_freq * c.in_dim,
                             hipMemcpyHostToDevice, m->stream));
  k += (size_t)c.n_freq * c.in_dim;
  for (int l = 0; l < m->nl; ++l) {
    const size_t nw = (size_t)m->lout[l] * m->lin[l];
    MHIP_TRY(m, hipMemcpyAsync(m->p<float>(m->oW[l]), host + k, sizeof(float) * nw,
                               hipMemcpyHostToDevice, m->stream));
    k += nw;
    MHIP_TRY(m, hipMemsetAsync(m->p<float>(m->ob[l]), 0, sizeof(float) * m->lpad[l], m->stream));
    MHIP_TRY(m, hipMemcpyAsync(m->p<float>(m->ob[l]), host + k, sizeof(float) * m->lout[l],
                               hipMemcpyHostToDevice, m->stream));
    k += m->lout[l];
    const size_t wbytes = sizeof(float) * nw, bbytes = sizeof(float) * m->lpad[l];
    MHIP_TRY(m, hipMemsetAsync(m->p<float>(m->omW[l]), 0, wbytes, m->stream));
    MHIP_TRY(m, hipMemsetAsync(m->p<float>(m->ovW[l]), 0, wbytes, m->stream));
    MHIP_TRY(m, hipMemsetAsync(m->p<float>(m->omb[l]), 0, bbytes, m->stream));
    MHIP_TRY(m, hipMemsetAsync(m->p<float>(m->ovb[l]), 0, bbytes, m->stream));
  }
  vflb_status rc = recast(m);
  if (rc != VFLB_OK) return rc;
  MHIP_TRY(m, hipStreamSynchronize(m->stream));
  m->adam_t = 0;
  m->have_params = true;
  return VFLB_OK;
}

// one Adam step (learning rate lr) of every layer from the gradients in
// PARAMS; refreshes the BF16 weight copies
vflb_status adam_update(vflb_mlp* m, float lr) {
  m->adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  for (int l = 0; l < m->nl; ++l) {
    AdamArgs a{};
    a.W = m->p<float>(m->oW[l]);
    a.b = m->p<float>(m->ob[l]);
    a.mW = m->p<float>(m->omW[l]);
    a.vW = m->p<float>(m->ovW[l]);
    a.mb = m->p<float>(m->omb[l]);
    a.vb = m->p<float>(m->ovb[l]);
    a.G = m->p<float>(m->oG[l]);
    a.gb = m->p<float>(m->ogb[l]);
    a.W16 = m->p<bf16>(m->oW16[l]);
    a.WT16 = m->p<bf16>(m->oWT16[l]);
    a.out = m->lout[l];
    a.in = m->lin[l];
    a.out_pad = m->lpad[l];
    a.lr = lr;
    a.beta1 = b1;
    a.beta2 = b2;
    a.eps = 1e-8f;
    a.c1 = (float)(1.0 - std::pow((double)b1, (double)m->adam_t));
    a.c2 = (float)(1.0 - std::pow((double)b2, (double)m->adam_t));
    const int cnt = a.out * a.in + a.out;
    hipLaunchKernelGGL(adam_kernel, dim3((cnt + 255) / 256), dim3(256), 0, m->stream, a);
    MHIP_TRY(m, hipGetLastError());
  }
  return VFLB_OK;
}

}  // namespace

extern "C" {

vflb_status vflb_mlp_create(const vflb_mlp_cfg* cfg, void* hip_stream, vflb_mlp** out) {
  if (!out || !cfg) return mfail(nullptr, VFLB_EINVAL, "NULL argument");
  *out = nullptr;
  const vflb_mlp_cfg& c = *cfg;
  if (c.in_dim < 1 || c.in_dim > 8) return mfail(nullptr, VFLB_EINVAL, "in_dim must lie in [1, 8]");
  if (c.n_freq < 32 || (2 * c.n_freq) % 64 != 0 || c.n_freq > 256)
    return mfail(nullptr, VFLB_EINVAL, "n_freq must be a multiple of 32 in [32, 256]");
  if (c.width < 64 || c.width % 64 != 0 || c.width > 1024)
    return mfail(nullptr, VFLB_EINVAL, "width must be a multiple of 64 in [64, 1024]");
  if (c.hidden < 1 || c.hidden > 16) return mfail(nullptr, VFLB_EINVAL, "hidden must lie in [1, 16]");
  if (c.out_dim < 1 || c.out_dim > kOutPad)
    return mfail(nullptr, VFLB_EINVAL, "out_dim must lie in [1, %d]", kOutPad);
  if (c.max_batch < 64 || c.max_batch % 64 != 0 || c.max_batch > (1 << 22))
    return mfail(nullptr, VFLB_EINVAL, "max_batch must be a multiple of 64 in [64, 2^22]");
  if (!(c.sigma > 0)) return mfail(nullptr, VFLB_EINVAL, "sigma must be positive");
  vflb_mlp* m = new vflb_mlp();
  m->cfg = c;
  m->stream = static_cast<hipStream_t>(hip_stream);
  m->nl = c.hidden + 1;
  for (int l = 0; l < m->nl; ++l) {
    m->lin.push_back(l == 0 ? 2 * c.n_freq : c.width);
    const bool last = l == m->nl - 1;
    m->lout.push_back(last ? c.out_dim : c.width);
    m->lpad.push_back(last ? kOutPad : c.width);
  }
  m->nparams = (size_t)c.n_freq * c.in_dim;
  for (int l = 0; l < m->nl; ++l) m->nparams += (size_t)m->lout[l] * m->lin[l] + m->lout[l];
  // PARAMS
  size_t o = 0;
  m->off_freq = o;
  o += a256(sizeof(float) * c.n_freq * c.in_dim);
  size_t maxwg = 0;
  for (int l = 0; l < m->nl; ++l) {
    const size_t nw = (size_t)m->lout[l] * m->lin[l], npw = (size_t)m->lpad[l] * m->lin[l];
    const size_t nb = m->lpad[l];
    m->oW.push_back(o); o += a256(4 * nw);
    m->ob.push_back(o); o += a256(4 * nb);
    m->omW.push_back(o); o += a256(4 * nw);
    m->ovW.push_back(o); o += a256(4 * nw);
    m->omb.push_back(o); o += a256(4 * nb);
    m->ovb.push_back(o); o += a256(4 * nb);
    m->oW16.push_back(o); o += a256(2 * npw);
    m->oWT16.push_back(o); o += a256(2 * npw);
    m->oG.push_back(o); o += a256(4 * npw);
    m->ogb.push_back(o); o += a256(4 * nb);
    if (npw > maxwg) maxwg = npw;
  }
  m->bytes[VFLB_MLP_BUF_PARAMS] = o;
  // WORK, sized for max_batch rows
  const size_t M = c.max_batch, W = c.width, F = 2 * (size_t)c.n_freq;
  o = 0;
  m->off_x = o; o += a256(4 * M * c.in_dim);
  m->off_phi = o; o += a256(2 * M * F);
  m->off_phiT = o; o += a256(2 * M * F);
  for (int l = 0; l < c.hidden; ++l) {
    m->oH32.push_back(o); o += a256(4 * M * W);
    m->oH16.push_back(o); o += a256(2 * M * W);
    m->oHT16.push_back(o); o += a256(2 * M * W);
  }
  m->off_Y = o; o += a256(4 * M * kOutPad);
  m->off_dY = o; o += a256(2 * M * kOutPad);
  m->off_dYT = o; o += a256(2 * M * kOutPad);
  for (int k = 0; k < 2; ++k) {
    m->off_dZ[k] = o; o += a256(2 * M * W);
    m->off_dZT[k] = o; o += a256(2 * M * W);
  }
  m->p_floats = (size_t)kMaxSplit * maxwg;
  m->off_P = o; o += a256(4 * m->p_floats);
  m->off_lpart = o; o += a256(8 * ((M + 255) / 256));
  m->off_loss = o; o += 256;
  m->off_tb = o; o += a256(4 * M * c.out_dim);
  m->off_stats = o; o += a256(8 * 2 * c.out_dim);
  m->bytes[VFLB_MLP_BUF_WORK] = o;
  *out = m;
  return VFLB_OK;
}

vflb_status vflb_mlp_query_buffers(const vflb_mlp* m, size_t bytes[VFLB_MLP_NBUF]) {
  if (!m || !bytes) return VFLB_EINVAL;
  for (int k = 0; k < VFLB_MLP_NBUF; ++k) bytes[k] = m->bytes[k];
  return VFLB_OK;
}

vflb_status vflb_mlp_bind_buffers(vflb_mlp* m, void* const ptrs[VFLB_MLP_NBUF]) {
  if (!m || !ptrs) return VFLB_EINVAL;
  for (int k = 0; k < VFLB_MLP_NBUF; ++k)
    if (!ptrs[k]) return mfail(m, VFLB_EINVAL, "buffer %d is NULL", k);
  for (int k = 0; k < VFLB_MLP_NBUF; ++k) m->buf[k] = ptrs[k];
  m->bound = true;
  m->have_params = false;
  return VFLB_OK;
}

size_t vflb_mlp_param_count(const vflb_mlp* m) { return m ? m->nparams : 0; }

vflb_status vflb_mlp_init(vflb_mlp* m, uint64_t seed) {
  if (!m) return VFLB_EINVAL;
  if (!m->bound) return mfail(m, VFLB_ESTATE, "device buffers are not bound");
  const vflb_mlp_cfg& c = m->cfg;
  std::vector<float> h(m->nparams);
  SplitMix rng{seed};
  size_t k = 0;
  for (int i = 0; i < c.n_freq * c.in_dim; ++i) h[k++] = (float)(c.sigma * rng.normal());
  for (int l = 0; l < m->nl; ++l) {
    const double a = std::sqrt(6.0 / (m->lin[l] + m->lout[l]));  // Glorot uniform
    for (int i = 0; i < m->lout[l] * m->lin[l]; ++i) h[k++] = (float)(a * (2.0 * rng.uniform() - 1.0));
    for (int i = 0; i < m->lout[l]; ++i) h[k++] = 0.0f;
  }
  return upload(m, h.data());
}

vflb_status vflb_mlp_set_params(vflb_mlp* m, const float* host, size_t n) {
  if (!m || !host) return VFLB_EINVAL;
  if (!m->bound) return mfail(m, VFLB_ESTATE, "device buffers are not bound");
  if (n != m->nparams) return mfail(m, VFLB_EINVAL, "expected %zu parameters", m->nparams);
  return upload(m, host);
}

vflb_status vflb_mlp_get_params(vflb_mlp* m, float* host, size_t n) {
  vflb_status rc = need_mlp(m);
  if (rc != VFLB_OK) return rc;
  if (!host || n != m->nparams) return mfail(m, VFLB_EINVAL, "expected %zu parameters", m->nparams);
  const vflb_mlp_cfg& c = m->cfg;
  size_t k = 0;
  MHIP_TRY(m, hipMemcpyAsync(host, m->p<float>(m->off_freq), sizeof(float) * c.n_freq * c.in_dim,
                             hipMemcpyDeviceToHost, m->stream));
  k += (size_t)c.n_freq * c.in_dim;
  for (int l = 0; l < m->nl; ++l) {
    const size_t nw = (size_t)m->lout[l] * m->lin[l];
    MHIP_TRY(m, hipMemcpyAsync(host + k, m->p<float>(m->oW[l]), 4 * nw, hipMemcpyDeviceToHost,
                               m->stream));
    k += nw;
    MHIP_TRY(m, hipMemcpyAsync(host + k, m->p<float>(m->ob[l]), 4 * m->lout[l],
                               hipMemcpyDeviceToHost, m->stream));
    k += m->lout[l];
  }
  MHIP_TRY(m, hipStreamSynchronize(m->stream));
  return VFLB_OK;
}

vflb_status vflb_mlp_forward(vflb_mlp* m, const float* dev_x, float* dev_y, int64_t n) {
  vflb_status rc = need_mlp(m);
  if (rc != VFLB_OK) return rc;
  if (n < 0 || (n > 0 && (!dev_x || !dev_y))) return mfail(m, VFLB_EINVAL, "bad arguments");
  const int out = m->cfg.out_dim, in = m->cfg.in_dim;
  for (int64_t s = 0; s < n; s += m->cfg.max_batch) {
    const int64_t cnt = std::min<int64_t>(m->cfg.max_batch, n - s);
    const int rows = rows_of(cnt);
    if ((rc = forward(m, dev_x + s * in, cnt, rows)) != VFLB_OK) return rc;
    MHIP_TRY(m, hipMemcpy2DAsync(dev_y + s * out, sizeof(float) * out, m->w<float>(m->off_Y),
                                 sizeof(float) * kOutPad, sizeof(float) * out, (size_t)cnt,
                                 hipMemcpyDeviceToDevice, m->stream));
  }
  return VFLB_OK;
}

vflb_status vflb_mlp_grad(vflb_mlp* m, const float* dev_x, const float* dev_t, int64_t n,
                          float* host_grad, double* loss) {
  vflb_status rc = need_mlp(m);
  if (rc != VFLB_OK) return rc;
  if (!dev_x || !dev_t || n < 1 || n > m->cfg.max_batch)
    return mfail(m, VFLB_EINVAL, "need 1 <= n <= max_batch and device inputs");
  const int rows = rows_of(n);
  if ((rc = forward(m, dev_x, n, rows)) != VFLB_OK) return rc;
  if ((rc = backward(m, dev_t, n, rows)) != VFLB_OK) return rc;
  if (host_grad) {
    const vflb_mlp_cfg& c = m->cfg;
    size_t k = (size_t)c.n_freq * c.in_dim;
    std::memset(host_grad, 0, sizeof(float) * k);  // the frequencies are not trained
    for (int l = 0; l < m->nl; ++l) {
      const size_t nw = (size_t)m->lout[l] * m->lin[l];
      MHIP_TRY(m, hipMemcpyAsync(host_grad + k, m->p<float>(m->oG[l]), 4 * nw,
                                 hipMemcpyDeviceToHost, m->stream));
      k += nw;
      MHIP_TRY(m, hipMemcpyAsync(host_grad + k, m->p<float>(m->ogb[l]), 4 * m->lout[l],
                                 hipMemcpyDeviceToHost, m->stream));
      k += m->lout[l];
    }
  }
  if (loss) {
    double s = 0;
    MHIP_TRY(m, hipMemcpyAsync(&s, m->w<double>(m->off_loss), sizeof s, hipMemcpyDeviceToHost,
                               m->stream));
    MHIP_TRY(m, hipStreamSynchronize(m->stream));
    *loss = s / ((double)n * m->cfg.out_dim);
  }
  MHIP_TRY(m, hipStreamSynchronize(m->stream));
  return VFLB_OK;
}

vflb_status vflb_mlp_train_step(vflb_mlp* m, const float* dev_x, const float* dev_t, int64_t n,
                                float lr, double* loss_out) {
  vflb_status rc = need_mlp(m);
  if (rc != VFLB_OK) return rc;
  if (!dev_x || !dev_t || n < 1 || n > m->cfg.max_batch)
    return mfail(m, VFLB_EINVAL, "need 1 <= n <= max_batch and device inputs");
  if (!(lr > 0)) return mfail(m, VFLB_EINVAL, "lr must be positive");
  const int rows = rows_of(n);
  if ((rc = forward(m, dev_x, n, rows)) != VFLB_OK) return rc;
  if ((rc = backward(m, dev_t, n, rows)) != VFLB_OK) return rc;
  if ((rc = adam_update(m, lr)) != VFLB_OK) return rc;
  if (loss_out) {
    double s = 0;
    MHIP_TRY(m, hipMemcpyAsync(&s, m->w<double>(m->off_loss), sizeof s, hipMemcpyDeviceToHost,
                               m->stream));
    MHIP_TRY(m, hipStreamSynchronize(m->stream));
    *loss_out = s / ((double)n * m->cfg.out_dim);
  }
  return VFLB_OK;
}

vflb_status vflb_mlp_train(vflb_mlp* m, const float* dev_X, const float* dev_T, int64_t n,
                           int64_t rows, int64_t iters, float lr, uint64_t seed,
                           int64_t log_every, double* losses) {
  vflb_status rc = need_mlp(m);
  if (rc != VFLB_OK) return rc;
  if (!dev_X || !dev_T || n < 1) return mfail(m, VFLB_EINVAL, "need n >= 1 and device data");
  if (rows < 1 || rows > m->cfg.max_batch)
    return mfail(m, VFLB_EINVAL, "need 1 <= rows <= max_batch");
  if (iters < 0 || !(lr > 0)) return mfail(m, VFLB_EINVAL, "need iters >= 0 and lr > 0");
  if (log_every < 0 || (log_every > 0 && !losses))
    return mfail(m, VFLB_EINVAL, "log_every > 0 needs a losses array");
  const vflb_mlp_cfg& c = m->cfg;
  double* stats = m->w<double>(m->off_stats);
  hipLaunchKernelGGL(col_stats_kernel, dim3(c.out_dim), dim3(256), 0, m->stream, dev_T, n,
                     c.out_dim, stats);
  MHIP_TRY(m, hipGetLastError());
  float* xb = m->w<float>(m->off_x);
  float* tb = m->w<float>(m->off_tb);
  const int prow = rows_of(rows);
  for (int64_t it = 0; it < iters; ++it) {
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0,
                       m->stream, dev_X, dev_T, n, c.in_dim, c.out_dim, (int)rows, seed,
                       (uint64_t)it * (uint64_t)rows, stats, xb, tb);
    MHIP_TRY(m, hipGetLastError());
    const double cosr = 0.5 * (1.0 + std::cos(3.14159265358979323846 * (double)it / (double)iters));
    const float rate = (float)std::max((double)lr * cosr, 1e-3 * (double)lr);
    if ((rc = forward(m, xb, rows, prow)) != VFLB_OK) return rc;
    if ((rc = backward(m, tb, rows, prow)) != VFLB_OK) return rc;
    if ((rc = adam_update(m, rate)) != VFLB_OK) return rc;
    if (log_every > 0 && (it % log_every == 0 || it == iters - 1)) {
      double sq = 0;
      MHIP_TRY(m, hipMemcpyAsync(&sq, m->w<double>(m->off_loss), sizeof sq,
                                 hipMemcpyDeviceToHost, m->stream));
      MHIP_TRY(m, hipStreamSynchronize(m->stream));
      losses[it / log_every + (it % log_every ? 1 : 0)] = sq / ((double)rows * c.out_dim);
    }
  }
  // the network learned standardised targets: fold (mean, std) into its
  // output layer, so that it predicts the targets themselves; the Adam
  // moments no longer match the folded layer and are reset
  const int L = m->nl - 1;
  const int cnt = m->lout[L] * m->lin[L] + m->lout[L];
  hipLaunchKernelGGL(fold_output_kernel, dim3((cnt + 255) / 256), dim3(256), 0, m->stream,
                     m->p<float>(m->oW[L]), m->p<float>(m->ob[L]), m->lout[L], m->lin[L], stats);
  MHIP_TRY(m, hipGetLastError());
  if ((rc = recast(m)) != VFLB_OK) return rc;
  for (int l = 0; l < m->nl; ++l) {
    const size_t wbytes = sizeof(float) * m->lout[l] * m->lin[l], bbytes = sizeof(float) * m->lpad[l];
    MHIP_TRY(m, hipMemsetAsync(m->p<float>(m->omW[l]), 0, wbytes, m->stream));
    MHIP_TRY(m, hipMemsetAsync(m->p<float>(m->ovW[l]), 0, wbytes, m->stream));
    MHIP_TRY(m, hipMemsetAsync(m->p<float>(m->omb[l]), 0, bbytes, m->stream));
    MHIP_TRY(m, hipMemsetAsync(m->p<float>(m->ovb[l]), 0, bbytes, m->stream));
  }
  m->adam_t = 0;
  MHIP_TRY(m, hipStreamSynchronize(m->stream));
  return VFLB_OK;
}

vflb_status vflb_init_from_mlp(vflb_sim* sim, vflb_mlp* m, const double extra[3], double u_scale,
                               double tau_scale, int64_t settle_steps, int settle_flags) {
  vflb_status rc = need_mlp(m);
  if (rc != VFLB_OK) return rc;
  if (!sim || !extra) return mfail(m, VFLB_EINVAL, "NULL argument");
  if (settle_steps < 0) return mfail(m, VFLB_EINVAL, "settle_steps < 0");
  if (m->cfg.in_dim != 5 || m->cfg.out_dim != 5)
    return mfail(m, VFLB_EINVAL, "the network must map 5 inputs to 5 outputs");
  vflb::internal::SimScratch ss{};
  if ((rc = vflb::internal::sim_scratch(sim, &ss)) != VFLB_OK)
    return mfail(m, rc, "simulation: %s", vflb_last_error(sim));
  if (ss.D != 2) return mfail(m, VFLB_EINVAL, "the warm start fills D2Q9 lattices");
  if (ss.stream != m->stream)
    return mfail(m, VFLB_EINVAL, "simulation and network need the same stream");
  const int nx = ss.nx, ny = ss.ny;
  const size_t N = (size_t)nx * ny;
  if (ss.bytes < 5 * N * sizeof(float)) return mfail(m, VFLB_ENOMEM, "scratch too small");
  float* u = static_cast<float*>(ss.scratch);
  float* tau = u + 2 * N;
  float* X = m->w<float>(m->off_x);
  for (size_t s = 0; s < N; s += m->cfg.max_batch) {
    const int cnt = (int)std::min<size_t>(m->cfg.max_batch, N - s);
    hipLaunchKernelGGL(node_inputs_kernel, dim3((cnt + 255) / 256), dim3(256), 0, m->stream, nx,
                       ny, s, cnt, (float)extra[0], (float)extra[1], (float)extra[2], X);
    MHIP_TRY(m, hipGetLastError());
    if ((rc = forward(m, X, cnt, rows_of(cnt))) != VFLB_OK) return rc;
    hipLaunchKernelGGL(node_outputs_kernel, dim3((cnt + 255) / 256), dim3(256), 0, m->stream,
                       m->w<float>(m->off_Y), kOutPad, s, cnt, N, (float)u_scale,
                       (float)tau_scale, u, tau);
    MHIP_TRY(m, hipGetLastError());
  }
  const unsigned g1 = (unsigned)((N + 255) / 256), g2 = (unsigned)((2 * N + 255) / 256);
  if (ss.walls == 0) {
    // periodic on every axis: project u onto the discretely solenoidal
    // fields, without mean and staggered momentum, as a start from rest is
    if (nx > 512 || ny > 512)
      return mfail(m, VFLB_EINVAL, "the velocity projection runs on lattices of side <= 512");
    if (ss.big_bytes < 2 * 2 * N * sizeof(float2))
      return mfail(m, VFLB_EINVAL, "the warm start needs two population buffers");
    float2* A = static_cast<float2*>(ss.big);
    float2* B = A + 2 * N;
    hipLaunchKernelGGL(to_complex_kernel, dim3(g2), dim3(256), 0, m->stream, u, 2 * N, A);
    hipLaunchKernelGGL(dft_pass_kernel, dim3(g2), dim3(256), 0, m->stream, A, B, nx, ny, 2, 0, -1);
    hipLaunchKernelGGL(dft_pass_kernel, dim3(g2), dim3(256), 0, m->stream, B, A, nx, ny, 2, 1, -1);
    hipLaunchKernelGGL(solenoidal_kernel, dim3(g1), dim3(256), 0, m->stream, A, nx, ny);
    hipLaunchKernelGGL(dft_pass_kernel, dim3(g2), dim3(256), 0, m->stream, A, B, nx, ny, 2, 1, 1);
    hipLaunchKernelGGL(dft_pass_kernel, dim3(g2), dim3(256), 0, m->stream, B, A, nx, ny, 2, 0, 1);
    hipLaunchKernelGGL(from_complex_kernel, dim3(g2), dim3(256), 0, m->stream, A, 2 * N,
                       1.0 / (double)N, u);
    MHIP_TRY(m, hipGetLastError());
  } else {
    // walls: remove the alternating component along each periodic axis
    for (int axis = 0; axis < 2; ++axis) {
      const int n = axis == 0 ? nx : ny, lines = axis == 0 ? ny : nx;
      if ((ss.walls >> axis) & 1 || n % 2 != 0) continue;
      hipLaunchKernelGGL(remove_alternating_kernel, dim3((lines + 255) / 256), dim3(256), 0,
                         m->stream, u, nx, ny, axis);
      MHIP_TRY(m, hipGetLastError());
    }
  }
  if (ss.lam_over_eta > 0) {
    hipLaunchKernelGGL(conformation_floor_kernel, dim3(g1), dim3(256), 0, m->stream, tau, N,
                       ss.lam_over_eta, kConformationFloor);
    MHIP_TRY(m, hipGetLastError());
  }
  if ((rc = vflb::internal::sim_init_f32(sim, u, tau)) != VFLB_OK)
    return mfail(m, rc, "simulation: %s", vflb_last_error(sim));
  if (settle_steps > 0 &&
      (rc = vflb::internal::sim_settle_f32(sim, u, settle_steps, settle_flags)) != VFLB_OK)
    return mfail(m, rc, "simulation: %s", vflb_last_error(sim));
  return VFLB_OK;
}

void vflb_mlp_destroy(vflb_mlp* m) { delete m; }

const char* vflb_mlp_last_error(const vflb_mlp* m) {
  if (!m) return g_mlp_create_error.c_str();
  return m->err.c_str();
}

}  // extern "C"
