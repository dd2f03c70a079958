// layout.h -- where populations and auxiliary fields live in HBM.
//
// One buffer per ping/pong side holds all populations of the lattice.  A
// tuple index t = i*N + n names direction i at node n.
//
//  D2Q9:  tuples [Q][N] of (f_i, h_xx,i, h_xy,i, h_yy,i).  f and the three
//         conformation populations of one direction stream from the same
//         source node, so a pull is one aligned vector load (16 bytes in
//         FP32, 8 in 16-bit storage) and a store one vector store.
//  D3Q19: f [Q N], then (h_xx, h_yy, h_zz, h_xy) tuples [Q N], then
//         (h_xz, h_yz) tuples [Q N], all three indexed by the same tuple
//         index.
//
// Auxiliary state chi(t-1), u(t-1):
//  D2Q9:  chi [N][3] then u [N][2] (one 12-byte and one 8-byte access).
//  D3Q19: chi [NC][N] then u [D][N].
//
// Anchored 16-bit storage (D2Q9 and D3Q19, FP16 and BF16): every node also keeps, in
// FP32 in the population buffer (Anchor2, Anchor3), its anchor (E, p)
// with E = A - I of its post-collision state, p its pressure and u its
// velocity, from which follow reference populations f_ref(p, u) (the
// equilibrium form) and h_ref(E, u) (the shifted equilibrium form).  A stored population is the
// 16-bit deviation of the value from the reference of the node that wrote
// it, and a reader rebuilds the value as reference + deviation.  The
// conserved moment A then lives in FP32: 16-bit rounding touches only the
// small deviations and can no longer random-walk A.
#pragma once

#include "lattice.h"

namespace vflb {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

// 4-wide tuple access in the arithmetic type: component 0 scaled by the f
// scale, components 1..3 by the h scale (scales are 1 except for FP16).
template <class S> struct Tuple4;
template <> struct Tuple4<float> {
  __device__ static void ld(const float* p, size_t t, float, float, float* v) {
    const f32x4 q = reinterpret_cast<const f32x4*>(p)[t];
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
  // non-temporal load: measured on MI355X, the 8192 x 1024 D2Q9 FP32 step
  // takes 0.505 instead of 0.532 ms with it; the batched ensemble of small
  // lattices is 2 % slower with it, and the same hint on the auxiliary
  // loads, on FP64 or 16-bit tuples or on the D3Q19 loads was slower or
  // neutral
  __device__ static void ld_nt(const float* p, size_t t, float, float, float* v) {
    const f32x4 q = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p) + t);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
  __device__ static void st(float* p, size_t t, float, float, const float* v) {
    f32x4 q = {v[0], v[1], v[2], v[3]};
    __builtin_nontemporal_store(q, reinterpret_cast<f32x4*>(p) + t);
  }
};
template <> struct Tuple4<double> {
  __device__ static void ld(const double* p, size_t t, double, double, double* v) {
    const f64x4 q = reinterpret_cast<const f64x4*>(p)[t];
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
  __device__ static void st(double* p, size_t t, double, double, const double* v) {
    f64x4 q = {v[0], v[1], v[2], v[3]};
    __builtin_nontemporal_store(q, reinterpret_cast<f64x4*>(p) + t);
  }
};
template <> struct Tuple4<_Float16> {
  __device__ static void ld(const _Float16* p, size_t t, float isf, float ish, float* v) {
    const f16x4 q = reinterpret_cast<const f16x4*>(p)[t];
    v[0] = (float)q.x * isf; v[1] = (float)q.y * ish;
    v[2] = (float)q.z * ish; v[3] = (float)q.w * ish;
  }
  __device__ static void st(_Float16* p, size_t t, float sf, float sh, const float* v) {
    f16x4 q = {(_Float16)(v[0] * sf), (_Float16)(v[1] * sh), (_Float16)(v[2] * sh),
               (_Float16)(v[3] * sh)};
    __builtin_nontemporal_store(q, reinterpret_cast<f16x4*>(p) + t);
  }
};
__device__ inline float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ inline uint16_t f32_to_bf16(float v) {
  uint32_t b = __float_as_uint(v);
  if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu))
    return (uint16_t)((b >> 16) | 0x0040u);  // keep NaN a NaN
  b += 0x7fffu + ((b >> 16) & 1u);          // round to nearest even
  return (uint16_t)(b >> 16);
}
template <> struct Tuple4<bf16_t> {
  __device__ static void ld(const bf16_t* p, size_t t, float, float, float* v) {
    const u16x4 q = reinterpret_cast<const u16x4*>(p)[t];
    v[0] = bf16_to_f32(q.x); v[1] = bf16_to_f32(q.y);
    v[2] = bf16_to_f32(q.z); v[3] = bf16_to_f32(q.w);
  }
  __device__ static void st(bf16_t* p, size_t t, float, float, const float* v) {
    u16x4 q = {f32_to_bf16(v[0]), f32_to_bf16(v[1]), f32_to_bf16(v[2]), f32_to_bf16(v[3])};
    __builtin_nontemporal_store(q, reinterpret_cast<u16x4*>(p) + t);
  }
};

template <int D, class S> struct Pops;

template <class S> struct Pops<2, S> {
  using St = StoreT<S>;
  using R = typename St::R;
  static constexpr int Q = 9, NC = 3;
  __host__ __device__ static size_t words(size_t N) { return (size_t)4 * Q * N; }
  // NT: a non-temporal load where it measured faster (FP32 tuples)
  template <bool NT = false>
  __device__ static void load(const S* p, size_t t, size_t, R isf, R ish, R& f, R* h) {
    R v[4];
    if constexpr (NT && std::is_same<S, float>::value)
      Tuple4<float>::ld_nt(p, t, isf, ish, v);
    else
      Tuple4<S>::ld(p, t, isf, ish, v);
    f = v[0]; h[0] = v[1]; h[1] = v[2]; h[2] = v[3];
  }
  __device__ static R load_f(const S* p, size_t t, size_t, R isf) {
    return St::ld(p, 4 * t, isf);
  }
  __device__ static void store(S* p, size_t t, size_t, R sf, R sh, R f, const R* h) {
    const R v[4] = {f, h[0], h[1], h[2]};
    Tuple4<S>::st(p, t, sf, sh, v);
  }
};

// D2Q9 in place (Planar storage): f [Q N], then h_xx, h_xy, h_yy, each
// [Q N].  Value t of a plane is direction t / N of node t % N, as in the
// tuple layout; the velocity pass of in-place streaming reads the f plane
// only.
template <class T> struct Pops<2, Planar<T>> {
  using S = Planar<T>;
  using St = StoreT<S>;
  using R = T;
  static constexpr int Q = 9, NC = 3;
  __host__ __device__ static size_t words(size_t N) { return (size_t)4 * Q * N; }
  __device__ static void load(const S* p, size_t t, size_t N, R, R, R& f, R* h) {
    f = St::ld(p, t, (R)1);
#pragma unroll
    for (int c = 0; c < NC; ++c) h[c] = St::ld(p, (size_t)(c + 1) * Q * N + t, (R)1);
  }
  __device__ static R load_f(const S* p, size_t t, size_t, R) { return St::ld(p, t, (R)1); }
  __device__ static void store(S* p, size_t t, size_t N, R, R, R f, const R* h) {
    St::st(p, t, f, (R)1);
#pragma unroll
    for (int c = 0; c < NC; ++c) St::st(p, (size_t)(c + 1) * Q * N + t, h[c], (R)1);
  }
};

// D3Q19: f [Q N], then tuples (h_xx, h_yy, h_zz, h_xy) [Q N], then tuples
// (h_xz, h_yz) [Q N].  f sits alone so that forming u ahead of a plane
// touches only f cache lines; per pulled direction the step issues one
// 4-byte, one 16-byte and one 8-byte access (FP32; twice that in FP64, half
// in 16-bit storage).
template <class S> struct Pops3Split {
  using St = StoreT<S>;
  using R = typename St::R;
  static constexpr int Q = 19, NC = 6;
  __host__ __device__ static size_t words(size_t N) { return (size_t)7 * Q * N; }
  __device__ static size_t h4(size_t N) { return (size_t)Q * N; }
  __device__ static size_t h2(size_t N) { return (size_t)5 * Q * N; }
  __device__ static void load(const S* p, size_t t, size_t N, R isf, R ish, R& f, R* h) {
    f = St::ld(p, t, isf);
#pragma unroll
    for (int c = 0; c < 4; ++c) h[c] = St::ld(p, h4(N) + 4 * t + c, ish);
#pragma unroll
    for (int c = 0; c < 2; ++c) h[4 + c] = St::ld(p, h2(N) + 2 * t + c, ish);
  }
  __device__ static R load_f(const S* p, size_t t, size_t, R isf) { return St::ld(p, t, isf); }
  __device__ static void store(S* p, size_t t, size_t N, R sf, R sh, R f, const R* h) {
    St::st(p, t, f, sf);
#pragma unroll
    for (int c = 0; c < 4; ++c) St::st(p, h4(N) + 4 * t + c, h[c], sh);
#pragma unroll
    for (int c = 0; c < 2; ++c) St::st(p, h2(N) + 2 * t + c, h[4 + c], sh);
  }
};
template <> struct Pops<3, float> : Pops3Split<float> {};
template <> struct Pops<3, double> : Pops3Split<double> {};
template <> struct Pops<3, _Float16> : Pops3Split<_Float16> {};
template <> struct Pops<3, bf16_t> : Pops3Split<bf16_t> {};

// explicit fused multiply-add: the same rounding in every caller, whatever
// contraction the compiler applies around it
template <class R> __device__ inline R fmar(R a, R b, R c);
template <> __device__ inline float fmar<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}
template <> __device__ inline double fmar<double>(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}
template <int C, class R> __device__ inline R csgn(R v) { return C > 0 ? v : -v; }

// reference populations of direction i from an anchor (E = A - I, p, u);
// a bounce-back pull reads the opposite direction: sgn = -1 flips c_i.
// Factored with explicit fused multiply-adds, as the D3Q19 references
// below: fref = fma(w_i, fma(cu, fma(cu, 9/2, 3), -3/2 u.u), lambda_i p),
// href = E (w_i + t) + delta t with t = 3 w_i c.u; c.u sums the nonzero
// components of c_i only (for an unrolled i the selects fold away), so that
// a reader and a writer evaluate the same reference bitwise.
template <class R>
__device__ inline R cdot2(int i, R ux, R uy) {
  const int cx = Lat<2>::cx(i), cy = Lat<2>::cy(i);
  const R tx = cx > 0 ? ux : -ux, ty = cy > 0 ? uy : -uy;
  return cx == 0 ? (cy == 0 ? (R)0 : ty) : (cy == 0 ? tx : tx + ty);
}
template <class R>
__device__ inline R fref2(int i, R sgn, R p, R ux, R uy) {
  const R wi = (R)Lat<2>::w(i);
  const R lam_i = (R)(i == 0 ? 3.0 * (Lat<2>::w(0) - 1.0) : 3.0 * Lat<2>::w(i));
  const R cu = sgn * cdot2<R>(i, ux, uy);
  const R uu = fmar(uy, uy, ux * ux);
  return fmar(wi, fmar(cu, fmar(cu, (R)4.5, (R)3), (R)-1.5 * uu), lam_i * p);
}
template <class R>
__device__ inline R href2(int i, int c, R sgn, R E, R ux, R uy) {
  const R wi = (R)Lat<2>::w(i);
  const R t = (R)(3.0 * Lat<2>::w(i)) * (sgn * cdot2<R>(i, ux, uy));
  return c != 1 ? fmar(E, wi + t, t) : E * (wi + t);
}

// Anchor of node n, kept in the population buffer after the 16-bit tuples
// (so that it ping-pongs with them: a step reads the anchors of the buffer
// it pulls from and writes those of the other): (E_xx, E_xy, E_yy, p) as
// [N] float4 from a 256-byte aligned offset, then u as [N] float2.
struct Anchor2 {
  __host__ __device__ static size_t offset(size_t N) {
    return ((size_t)2 * 4 * 9 * N + 255) & ~(size_t)255;
  }
  __host__ __device__ static size_t bytes(size_t N) { return offset(N) + 24 * N; }
  __device__ static void load(const void* pbuf, size_t n, size_t N, float4& ep, float2& u) {
    const char* b = static_cast<const char*>(pbuf) + offset(N);
    ep = reinterpret_cast<const float4*>(b)[n];
    u = reinterpret_cast<const float2*>(b + 16 * N)[n];
  }
  __device__ static void store(void* pbuf, size_t n, size_t N, float4 ep, float2 u) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    typedef float f2 __attribute__((ext_vector_type(2)));
    char* b = static_cast<char*>(pbuf) + offset(N);
    const f4 q = {ep.x, ep.y, ep.z, ep.w};
    const f2 v = {u.x, u.y};
    __builtin_nontemporal_store(q, reinterpret_cast<f4*>(b) + n);
    __builtin_nontemporal_store(v, reinterpret_cast<f2*>(b + 16 * N) + n);
  }
};

// D3Q19 references of direction i from an anchor (E = A - I, p, u), as
// fref2 / href2; direction i is the stored direction (the writer's), so no
// sign flip is needed for a bounce-back pull.  Written as
//   fref = w_i (3 c.u + 9/2 (c.u)^2 - 3/2 u.u) + lambda_i p
//        = fma(w_i, fma(cu, fma(cu, 9/2, 3), -3/2 uu), lambda_i p),
//   href = w_i E + 3 w_i (E + delta) c.u = E (w_i + t) + delta t,  t = 3 w_i c.u,
// with explicit fused multiply-adds in one fixed order and c.u summed over
// the nonzero components of c only: a reader and a writer evaluate the same
// reference bitwise whatever contraction the compiler applies around them,
// and the rebuilt value is the stored deviation plus exactly the reference
// the writer subtracted.
// c.u for c = (CX, CY, CZ) with components in {-1, 0, 1}
template <int CX, int CY, int CZ, class R>
__device__ inline R cdot3(const R* u) {
  if constexpr (CX != 0) {
    R s = csgn<CX>(u[0]);
    if constexpr (CY != 0) s += csgn<CY>(u[1]);
    if constexpr (CZ != 0) s += csgn<CZ>(u[2]);
    return s;
  } else if constexpr (CY != 0) {
    R s = csgn<CY>(u[1]);
    if constexpr (CZ != 0) s += csgn<CZ>(u[2]);
    return s;
  } else {
    return csgn<CZ>(u[2]);
  }
}
template <class R>
__device__ inline R uu3(const R* u) {
  return fmar(u[2], u[2], fmar(u[1], u[1], u[0] * u[0]));
}

// The member of opposite pair K (K >= 1) with velocity sgn c_{2K-1} (sgn =
// 1: direction 2K - 1, -1: direction 2K).  cu_pair3 is its c.u; the other
// arguments are the writer's anchor.
template <int K, class R>
__device__ inline R cu_pair3(R sgn, const R* u) {
  constexpr int i = 2 * K - 1;
  return sgn * cdot3<Lat<3>::cx(i), Lat<3>::cy(i), Lat<3>::cz(i)>(u);
}
template <int K, class R>
__device__ inline R fref3_cu(R cu, R p, R uu) {
  constexpr R wi = (R)Lat<3>::w(2 * K - 1), lam_i = (R)(3.0 * Lat<3>::w(2 * K - 1));
  return fmar(wi, fmar(cu, fmar(cu, (R)4.5, (R)3), (R)-1.5 * uu), lam_i * p);
}
template <int K, class R>
__device__ inline R href3_cu(R cu, int c, R E) {
  constexpr R wi = (R)Lat<3>::w(2 * K - 1);
  const R t = (R)(3.0 * Lat<3>::w(2 * K - 1)) * cu;
  return c < 3 ? fmar(E, wi + t, t) : E * (wi + t);
}
template <int K, class R>
__device__ inline R fref3_pair(R sgn, R p, const R* u) {
  return fref3_cu<K, R>(cu_pair3<K, R>(sgn, u), p, uu3(u));
}
template <int K, class R>
__device__ inline R href3_pair(R sgn, int c, R E, const R* u) {
  return href3_cu<K, R>(cu_pair3<K, R>(sgn, u), c, E);
}
// the rest direction (c = 0)
template <class R>
__device__ inline R fref3_rest(R p, R uu) {
  constexpr R w0 = (R)Lat<3>::w(0), lam0 = (R)(3.0 * (Lat<3>::w(0) - 1.0));
  return fmar(w0, (R)-1.5 * uu, lam0 * p);
}
template <class R>
__device__ inline R href3_rest(R E) {
  return (R)Lat<3>::w(0) * E;
}
// sc times the references above, exactly, for a power of two sc (scaling by
// sc commutes with every rounding in them, barring overflow and underflow):
// a writer forms its scaled deviation fma(v, sc, -sc ref) in one rounding.
// psc = p sc; for pair K, href = c < 3 ? fma(E, m, t) : E m.
template <int K, class R>
__device__ inline R fref3_cu_scaled(R cu, R psc, R uu, R sc) {
  constexpr R wi = (R)Lat<3>::w(2 * K - 1), lam_i = (R)(3.0 * Lat<3>::w(2 * K - 1));
  return fmar(wi * sc, fmar(cu, fmar(cu, (R)4.5, (R)3), (R)-1.5 * uu), lam_i * psc);
}
template <int K, class R>
__device__ inline void href3_cu_scaled(R cu, R sc, R& m, R& t) {
  constexpr R wi = (R)Lat<3>::w(2 * K - 1);
  const R tt = (R)(3.0 * Lat<3>::w(2 * K - 1)) * cu;
  m = (wi + tt) * sc;
  t = tt * sc;
}
template <class R>
__device__ inline R fref3_rest_scaled(R psc, R uu, R sc) {
  constexpr R w0 = (R)Lat<3>::w(0), lam0 = (R)(3.0 * (Lat<3>::w(0) - 1.0));
  return fmar(w0 * sc, (R)-1.5 * uu, lam0 * psc);
}

// any direction i, by its pair: equal bitwise to the forms above
template <class R>
__device__ inline R fref3(int i, R p, const R* u) {
  if (i == 0) return fref3_rest(p, uu3(u));
  const R sgn = (i & 1) ? (R)1 : (R)-1;
  switch ((i + 1) >> 1) {
    case 1: return fref3_pair<1, R>(sgn, p, u);
    case 2: return fref3_pair<2, R>(sgn, p, u);
    case 3: return fref3_pair<3, R>(sgn, p, u);
    case 4: return fref3_pair<4, R>(sgn, p, u);
    case 5: return fref3_pair<5, R>(sgn, p, u);
    case 6: return fref3_pair<6, R>(sgn, p, u);
    case 7: return fref3_pair<7, R>(sgn, p, u);
    case 8: return fref3_pair<8, R>(sgn, p, u);
    default: return fref3_pair<9, R>(sgn, p, u);
  }
}
template <class R>
__device__ inline R href3(int i, int c, R E, const R* u) {
  if (i == 0) return href3_rest(E);
  const R sgn = (i & 1) ? (R)1 : (R)-1;
  switch ((i + 1) >> 1) {
    case 1: return href3_pair<1, R>(sgn, c, E, u);
    case 2: return href3_pair<2, R>(sgn, c, E, u);
    case 3: return href3_pair<3, R>(sgn, c, E, u);
    case 4: return href3_pair<4, R>(sgn, c, E, u);
    case 5: return href3_pair<5, R>(sgn, c, E, u);
    case 6: return href3_pair<6, R>(sgn, c, E, u);
    case 7: return href3_pair<7, R>(sgn, c, E, u);
    case 8: return href3_pair<8, R>(sgn, c, E, u);
    default: return href3_pair<9, R>(sgn, c, E, u);
  }
}

// D3Q19 anchor of node n, after the 16-bit populations of the buffer (it
// ping-pongs with them): (p, u_x, u_y, u_z) as [N] float4, then (E_xx,
// E_yy, E_zz, E_xy) as [N] float4, then (E_xz, E_yz) as [N] float2, each
// array 256-byte aligned.  A pull that needs only the writer's p and u
// reads the first array alone.
struct Anchor3 {
  __host__ __device__ static size_t offset(size_t N) {
    return ((size_t)2 * 7 * 19 * N + 255) & ~(size_t)255;
  }
  __host__ __device__ static size_t off1(size_t N) { return (16 * N + 255) & ~(size_t)255; }
  __host__ __device__ static size_t off2(size_t N) { return off1(N) + ((16 * N + 255) & ~(size_t)255); }
  __host__ __device__ static size_t bytes(size_t N) { return offset(N) + off2(N) + 8 * N; }
  __device__ static void load_pu(const void* pbuf, size_t n, size_t N, float& p, float* u) {
    const char* b = static_cast<const char*>(pbuf) + offset(N);
    const float4 q = reinterpret_cast<const float4*>(b)[n];
    p = q.x; u[0] = q.y; u[1] = q.z; u[2] = q.w;
  }
  __device__ static void load(const void* pbuf, size_t n, size_t N, float& p, float* u,
                              float* E) {
    load_pu(pbuf, n, N, p, u);
    const char* b = static_cast<const char*>(pbuf) + offset(N);
    const float4 e = reinterpret_cast<const float4*>(b + off1(N))[n];
    const float2 r = reinterpret_cast<const float2*>(b + off2(N))[n];
    E[0] = e.x; E[1] = e.y; E[2] = e.z; E[3] = e.w; E[4] = r.x; E[5] = r.y;
  }
  __device__ static void store(void* pbuf, size_t n, size_t N, float p, const float* u,
                               const float* E) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    typedef float f2 __attribute__((ext_vector_type(2)));
    char* b = static_cast<char*>(pbuf) + offset(N);
    const f4 q = {p, u[0], u[1], u[2]};
    const f4 e = {E[0], E[1], E[2], E[3]};
    const f2 r = {E[4], E[5]};
    __builtin_nontemporal_store(q, reinterpret_cast<f4*>(b) + n);
    __builtin_nontemporal_store(e, reinterpret_cast<f4*>(b + off1(N)) + n);
    __builtin_nontemporal_store(r, reinterpret_cast<f2*>(b + off2(N)) + n);
  }
};

// auxiliary state
template <int D, class R> struct Aux;
template <class R> struct Aux<2, R> {
  static constexpr int NC = 3;
  __host__ __device__ static size_t words(size_t N) { return (size_t)5 * N; }
  __device__ static void load(const R* a, size_t n, size_t N, R* chi, R* u) {
    const R* c = a + 3 * n;
    chi[0] = c[0]; chi[1] = c[1]; chi[2] = c[2];
    const R* w = a + 3 * N + 2 * n;
    u[0] = w[0]; u[1] = w[1];
  }
  __device__ static void store(R* a, size_t n, size_t N, const R* chi, const R* u) {
    R* c = a + 3 * n;
    stream_store(c, chi[0]); stream_store(c + 1, chi[1]); stream_store(c + 2, chi[2]);
    R* w = a + 3 * N + 2 * n;
    stream_store(w, u[0]); stream_store(w + 1, u[1]);
  }
};
template <class R> struct Aux<3, R> {
  static constexpr int NC = 6;
  __host__ __device__ static size_t words(size_t N) { return (size_t)9 * N; }
  __device__ static void load(const R* a, size_t n, size_t N, R* chi, R* u) {
#pragma unroll
    for (int c = 0; c < NC; ++c) chi[c] = a[(size_t)c * N + n];
#pragma unroll
    for (int b = 0; b < 3; ++b) u[b] = a[(size_t)(NC + b) * N + n];
  }
  __device__ static void store(R* a, size_t n, size_t N, const R* chi, const R* u) {
#pragma unroll
    for (int c = 0; c < NC; ++c) stream_store(a + (size_t)c * N + n, chi[c]);
#pragma unroll
    for (int b = 0; b < 3; ++b) stream_store(a + (size_t)(NC + b) * N + n, u[b]);
  }
};

}  // namespace vflb
