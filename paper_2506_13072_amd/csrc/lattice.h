// lattice.h -- velocity sets, storage formats and the per-node arithmetic of
// the fluctuating LB step, as device functions for gfx950.
//
// Velocity sets: D2Q9 in the order and with the weights of Sec. 2.2;
// D3Q19 in the order of App. A with the isotropic weights 1/3, 1/18, 1/36
// (the paper prints none).  Everything here is written for the HIP path
// only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace vflb {

// Compile-time loop: fn(std::integral_constant<int, K>()) for K = B .. E-1,
// each body its own instantiation, so the loop is unrolled whatever its size
// and per-direction arrays stay in registers.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& fn) {
  if constexpr (B < E) {
    fn(std::integral_constant<int, B>());
    static_for<B + 1, E>(fn);
  }
}

template <int D> struct Lat;

template <> struct Lat<2> {
  static constexpr int Q = 9;
  static constexpr int NC = 3;  // xx, xy, yy
  __host__ __device__ static constexpr int cx(int i) {
    return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0);
  }
  __host__ __device__ static constexpr int cy(int i) {
    return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0);
  }
  __host__ __device__ static constexpr int cz(int) { return 0; }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
  __host__ __device__ static constexpr int opp(int i) {
    return i == 0 ? 0 : (i < 5 ? ((i + 1) % 4) + 1 : ((i - 5 + 2) % 4) + 5);
  }
  // component c -> tensor indices
  __host__ __device__ static constexpr int ca(int c) { return c == 2 ? 1 : 0; }
  __host__ __device__ static constexpr int cb(int c) { return c == 0 ? 0 : 1; }
};

template <> struct Lat<3> {
  static constexpr int Q = 19;
  static constexpr int NC = 6;  // xx, yy, zz, xy, xz, yz
  __host__ __device__ static constexpr int cx(int i) {
    return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
           : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0;
  }
  __host__ __device__ static constexpr int cy(int i) {
    return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
           : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0;
  }
  __host__ __device__ static constexpr int cz(int i) {
    return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
           : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0;
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  // directions come in opposite pairs (1,2), (3,4), ..., (17,18)
  __host__ __device__ static constexpr int opp(int i) {
    return i == 0 ? 0 : (i % 2 == 1 ? i + 1 : i - 1);
  }
  __host__ __device__ static constexpr int ca(int c) {
    return c < 3 ? c : (c == 5 ? 1 : 0);
  }
  __host__ __device__ static constexpr int cb(int c) {
    return c < 3 ? c : (c == 3 ? 1 : 2);
  }
};

template <int D>
__host__ __device__ constexpr int cdir(int i, int a) {
  return a == 0 ? Lat<D>::cx(i) : (a == 1 ? Lat<D>::cy(i) : Lat<D>::cz(i));
}

// direction index of the unit vector +-e_a
template <int D>
__host__ __device__ constexpr int axis_dir(int a, int sign) {
  return D == 2 ? (a == 0 ? (sign > 0 ? 1 : 3) : (sign > 0 ? 2 : 4))
                : (2 * a + (sign > 0 ? 1 : 2));
}

// ---------------------------------------------------------------- storage
// Populations are stored shifted (h - w delta) and, for FP16, multiplied by
// an exact power of two; the arithmetic type R is double for FP64 storage
// and float otherwise.
struct bf16_t {
  uint16_t bits;
};

// Stores of step outputs are non-temporal: the values are read again only
// by the next step, after the whole lattice has streamed through the caches.
template <class T>
__device__ inline void stream_store(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}

template <class S> struct StoreT;
// kAnchored: D2Q9 populations stored as 16-bit deviations from reference
// populations built from their node's FP32 anchor (see layout.h)
template <> struct StoreT<double> {
  using R = double;
  static constexpr bool kAnchored = false;
  static constexpr bool kPlanar = false;
  __device__ static R ld(const double* p, size_t i, R) { return p[i]; }
  __device__ static void st(double* p, size_t i, R v, R) { stream_store(p + i, v); }
};
template <> struct StoreT<float> {
  using R = float;
  static constexpr bool kAnchored = false;
  static constexpr bool kPlanar = false;
  __device__ static R ld(const float* p, size_t i, R) { return p[i]; }
  __device__ static void st(float* p, size_t i, R v, R) { stream_store(p + i, v); }
};
template <> struct StoreT<_Float16> {
  using R = float;
  static constexpr bool kAnchored = true;
  static constexpr bool kPlanar = false;
  // v = stored * 2^-k ; stored = RNE(v * 2^k)  (the scale is exact)
  __device__ static R ld(const _Float16* p, size_t i, R inv_scale) {
    return (float)p[i] * inv_scale;
  }
  __device__ static void st(_Float16* p, size_t i, R v, R scale) {
    stream_store(p + i, (_Float16)(v * scale));
  }
};
template <> struct StoreT<bf16_t> {
  using R = float;
  static constexpr bool kAnchored = true;
  static constexpr bool kPlanar = false;
  __device__ static R ld(const bf16_t* p, size_t i, R) {
    uint32_t b = (uint32_t)p[i].bits << 16;
    return __uint_as_float(b);
  }
  __device__ static void st(bf16_t* p, size_t i, R v, R) {
    uint32_t b = __float_as_uint(v);
    uint16_t out;
    if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu)) {
      out = (uint16_t)((b >> 16) | 0x0040u);  // keep NaN a NaN
    } else {
      b += 0x7fffu + ((b >> 16) & 1u);          // round to nearest even
      out = (uint16_t)(b >> 16);
    }
    stream_store(reinterpret_cast<uint16_t*>(p) + i, out);
  }
};

// In-place (AA) storage of D2Q9 FP32 and FP64 states: the same numbers as
// float and double, kept in planes (f, then each h component; layout.h)
// rather than in (f, h) tuples, so that a pass which needs f alone reads f
// alone.
template <class T> struct Planar {
  T v;
};
template <class T> struct StoreT<Planar<T>> {
  using R = T;
  static constexpr bool kAnchored = false;
  static constexpr bool kPlanar = true;
  // non-temporal loads: measured on MI355X, the in-place 8192 x 1024 D2Q9
  // FP32 step (velocity pass and step) takes 0.573 instead of 0.634 ms
  __device__ static R ld(const Planar<T>* p, size_t i, R) {
    return __builtin_nontemporal_load(&p[i].v);
  }
  __device__ static void st(Planar<T>* p, size_t i, R v, R) { stream_store(&p[i].v, v); }
};

// ---------------------------------------------------------------- params
template <class R> struct Phys {
  R tau_f, inv_tau_f, k_f;       // k_f = 1 - 1/(2 tau_f)
  R inv_tau_h, k_h3;             // k_h3 = 3 (1 - 1/(2 tau_h))
  R inv_lam, eta_over_lam;
  R fluct;  // 1: the fluctuation term f^B enters the f collision; 0: it does not
            // (the stress-divergence scheme carries the stress as a force)
  int model;  // constitutive model (MODEL_* below) and its parameter
  R mparam;
};

// Constitutive models: the relaxation term R(E) of the conformation
// equation, E = A - I (Oldroyd-B of the paper: R = E; the Giesekus and
// Phan-Thien-Tanner models the paper names as next: R = E + alpha E.E,
// (1 + eps tr E) E, exp(eps tr E) E).
enum { MODEL_OLDROYD_B = 0, MODEL_GIESEKUS = 1, MODEL_LPTT = 2, MODEL_EPTT = 3 };

// ----------------------------------------------------- per-node arithmetic
// Polymer-stress fluctuation term from the pseudo-inverse closed forms
// (the Moore-Penrose solution of the constraints sum f^B = 0,
// sum c f^B = 0, sum c c f^B = -tau_p / tau_f).  tau in component order.
template <class R>
__device__ inline void fluct_term(const R* tau, R inv_tau_f, R* fB, Lat<2>*) {
  const R xx = tau[0], xy = tau[1], yy = tau[2];
  const R T = xx + yy;
  const R k6 = inv_tau_f * (R)(1.0 / 6.0), k12 = inv_tau_f * (R)(1.0 / 12.0);
  fB[0] = T * inv_tau_f * (R)(1.0 / 3.0);
  fB[1] = fB[3] = (2 * yy - xx) * k6;
  fB[2] = fB[4] = (2 * xx - yy) * k6;
  fB[5] = fB[7] = -(3 * xy + 2 * T) * k12;
  fB[6] = fB[8] = (3 * xy - 2 * T) * k12;
}

template <class R>
__device__ inline void fluct_term(const R* tau, R inv_tau_f, R* fB, Lat<3>*) {
  const R xx = tau[0], yy = tau[1], zz = tau[2], xy = tau[3], xz = tau[4],
          yz = tau[5];
  const R k42 = inv_tau_f * (R)(1.0 / 42.0), k84 = inv_tau_f * (R)(1.0 / 84.0);
  fB[0] = (xx + yy + zz) * inv_tau_f * (R)(5.0 / 21.0);
  fB[1] = fB[2] = (6 * (yy + zz) - xx) * k42;
  fB[3] = fB[4] = (6 * (xx + zz) - yy) * k42;
  fB[5] = fB[6] = (6 * (xx + yy) - zz) * k42;
  const R sxy = 10 * (xx + yy) - 4 * zz, sxz = 10 * (xx + zz) - 4 * yy,
          syz = 10 * (yy + zz) - 4 * xx;
  fB[7] = fB[8] = -(sxy + 21 * xy) * k84;
  fB[9] = fB[10] = -(sxy - 21 * xy) * k84;
  fB[11] = fB[12] = -(sxz + 21 * xz) * k84;
  fB[13] = fB[14] = -(sxz - 21 * xz) * k84;
  fB[15] = fB[16] = -(syz + 21 * yz) * k84;
  fB[17] = fB[18] = -(syz - 21 * yz) * k84;
}

// c_i . v
template <int D, class R>
__device__ inline R cdot(int i, const R* v) {
  R s = (R)cdir<D>(i, 0) * v[0] + (R)cdir<D>(i, 1) * v[1];
  if (D == 3) s += (R)cdir<D>(i, 2) * v[2];
  return s;
}

// Collision of the velocity populations at one node (Sec. 2.2):
// f* = f - (f - f^eq)/tau_f + f^B + F_i, with u = sum c f + F/2 already
// formed.  Returns the pressure.  e = A - I (shifted conformation moment).
template <int D, class R>
__device__ inline R collide_f(R* f, const R* e, const R* u, const R* F,
                              const Phys<R>& P) {
  using L = Lat<D>;
  constexpr int Q = L::Q, NC = L::NC;
  R tau[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) tau[c] = P.eta_over_lam * e[c];
  R fB[Q];
  fluct_term<R>(tau, P.inv_tau_f * P.fluct, fB, (L*)nullptr);
  R uu = u[0] * u[0] + u[1] * u[1];
  R Fu = F[0] * u[0] + F[1] * u[1];
  if (D == 3) {
    uu += u[2] * u[2];
    Fu += F[2] * u[2];
  }
  constexpr R w0 = (R)L::w(0);
  // pressure (App. B): cs2/(1-w0) [sum_{i>0} f_i + s_0(u) + tau_f F_0 + tau_f f_0^B]
  R sum = 0;
#pragma unroll
  for (int i = 1; i < Q; ++i) sum += f[i];
  const R F0 = -3 * w0 * P.k_f * Fu;
  constexpr R pref = (R)((1.0 / 3.0) / (1.0 - L::w(0)));
  const R p = pref * (sum - (R)1.5 * w0 * uu + P.tau_f * F0 + P.tau_f * fB[0]);
  // momentum the collision must produce: sum c f* = u + F/2 (exact identity
  // of the BGK + Guo + f^B update).  Rounded weights (sum w c c != cs2 in
  // binary) would bias every step; the residual is put back on the
  // axis-aligned pairs, which leaves mass and second moments unchanged.
  R J[3];
#pragma unroll
  for (int b = 0; b < D; ++b) J[b] = u[b] + (R)0.5 * F[b];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R wi = (R)L::w(i);
    const R lam_i = (R)(i == 0 ? 3.0 * (L::w(0) - 1.0) : 3.0 * L::w(i));
    const R cu = cdot<D, R>(i, u);
    const R cF = cdot<D, R>(i, F);
    const R feq = lam_i * p + wi * (3 * cu + (R)4.5 * cu * cu - (R)1.5 * uu);
    const R Fi = wi * P.k_f * (3 * cF + 9 * cF * cu - 3 * Fu);
    f[i] = f[i] - (f[i] - feq) * P.inv_tau_f + fB[i] + Fi;
  }
#pragma unroll
  for (int b = 0; b < D; ++b) {
    R m = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i)
      if (cdir<D>(i, b) != 0) m += (R)cdir<D>(i, b) * f[i];
    const R half = (R)0.5 * (J[b] - m);
    f[axis_dir<D>(b, +1)] += half;
    f[axis_dir<D>(b, -1)] -= half;
  }
  return p;
}

// Oldroyd-B source tensor chi = -(A - I)/lambda + A.G + G^T.A with
// G[a][b] = d_a u_b (upper-convected form of the constitutive equation).
template <int D, class R>
__device__ inline void source_tensor(const R* e, const R (*G)[3], const Phys<R>& P,
                                     R* chi) {
  using L = Lat<D>;
  R A[3][3];
#pragma unroll
  for (int c = 0; c < L::NC; ++c) {
    const int a = L::ca(c), b = L::cb(c);
    const R v = e[c] + (a == b ? (R)1 : (R)0);
    A[a][b] = v;
    A[b][a] = v;
  }
  // relaxation term R(E) of the constitutive model
  R rel[L::NC];
#pragma unroll
  for (int c = 0; c < L::NC; ++c) rel[c] = e[c];
  if (P.model == MODEL_GIESEKUS) {
#pragma unroll
    for (int c = 0; c < L::NC; ++c) {
      const int a = L::ca(c), b = L::cb(c);
      R ee = 0;
#pragma unroll
      for (int g = 0; g < D; ++g)
        ee += (A[a][g] - (a == g ? (R)1 : (R)0)) * (A[g][b] - (g == b ? (R)1 : (R)0));
      rel[c] = e[c] + P.mparam * ee;
    }
  } else if (P.model == MODEL_LPTT || P.model == MODEL_EPTT) {
    R tr = 0;
#pragma unroll
    for (int c = 0; c < L::NC; ++c)
      if (L::ca(c) == L::cb(c)) tr += e[c];
    const R f = P.model == MODEL_LPTT ? (R)1 + P.mparam * tr : exp(P.mparam * tr);
#pragma unroll
    for (int c = 0; c < L::NC; ++c) rel[c] = f * e[c];
  }
#pragma unroll
  for (int c = 0; c < L::NC; ++c) {
    const int a = L::ca(c), b = L::cb(c);
    R s = -rel[c] * P.inv_lam;
#pragma unroll
    for (int g = 0; g < D; ++g) s += A[a][g] * G[g][b] + G[g][a] * A[g][b];
    chi[c] = s;
  }
}

// Collision of the (shifted) conformation populations of one component
// (Sec. 2.3): h* = h - (h - h^eq)/tau_h + chi_i + (chi_i - chi_i(t-1))/2,
// h^eq - w delta = w e + 3 w A (c.u), chi_i = w chi (1 + 3 k_h c.u).
// The zeroth moment is conserved up to the source: sum_i h*_i =
// A - I + chi + (chi - chi(t-1))/2.  The rest population is set from that
// identity, so that rounded weights (sum w != 1 in binary) cannot make the
// conformation drift over the O(lambda) steps it integrates.
template <int D, class R>
__device__ inline void collide_h(R* ht, R ec, R Ac, R chic, R chip,
                                 const R* u, const R* up, bool first,
                                 const Phys<R>& P) {
  using L = Lat<D>;
  const R target = ec + chic + (first ? (R)0 : (R)0.5 * (chic - chip));
  R rest = target;
#pragma unroll
  for (int i = 1; i < L::Q; ++i) {
    const R wi = (R)L::w(i);
    const R cu = cdot<D, R>(i, u);
    const R heq = wi * ec + 3 * wi * Ac * cu;
    const R chi_i = wi * chic * (1 + P.k_h3 * cu);
    R src = chi_i;
    if (!first) {
      const R chip_i = wi * chip * (1 + P.k_h3 * cdot<D, R>(i, up));
      src += (R)0.5 * (chi_i - chip_i);
    }
    ht[i] = ht[i] - (ht[i] - heq) * P.inv_tau_h + src;
    rest -= ht[i];
  }
  ht[0] = rest;
}

}  // namespace vflb
