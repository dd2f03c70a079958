// step3d.h -- the fused D3Q19 step for gfx950, marching along z.
//
// A workgroup of TY wavefronts owns a 64 x TY column of the lattice and
// walks a chunk of ZC planes in z.  The velocity of three consecutive planes
// (z-1, z, z+1) plus a one-node ring in x and y lives in LDS, so the
// same-time gradient needs no halo in z: per plane the workgroup pulls the
// 18 moving f populations of plane z+1 (own nodes and the x/y ring) to
// form u(z+1), then collides plane z.  Only the first plane of a chunk
// costs an extra u plane.
//
// Register budget: a node's 133 populations are not held at once.  Pass 1
// pulls every direction and keeps the moments; pass 2 pulls each direction
// again (a cache hit), collides and stores it.  Loads address a uniform
// per-direction plane base with a 32-bit node offset.
#pragma once

#include "kernels.h"

namespace vflb {

// 16-bit storage: one 8-wide 16-byte tuple per direction and node
template <class S> struct Plane3x8 {
  using R = float;
  __device__ static float unpack1(uint16_t b);
  __device__ static void unpack8(uint4 q, R* v);
  __device__ static uint4 pack8(const R* v);
  __device__ static void load(const S* p, int i, uint32_t node, size_t N, R isf, R ish, R& f,
                              R* h) {
    const char* A = reinterpret_cast<const char*>(p) + (size_t)i * N * 16;
    R v[8];
    unpack8(*reinterpret_cast<const uint4*>(A + node * 16u), v);
    f = v[0] * isf;
#pragma unroll
    for (int c = 0; c < 6; ++c) h[c] = v[1 + c] * ish;
  }
  __device__ static R load_f(const S* p, int i, uint32_t node, size_t N, R isf) {
    const char* A = reinterpret_cast<const char*>(p) + (size_t)i * N * 16;
    return unpack1(*reinterpret_cast<const uint16_t*>(A + node * 16u)) * isf;
  }
  __device__ static void store(S* p, int i, uint32_t node, size_t N, R sf, R sh, R f,
                               const R* h) {
    char* A = reinterpret_cast<char*>(p) + (size_t)i * N * 16;
    const R v[8] = {f * sf, h[0] * sh, h[1] * sh, h[2] * sh, h[3] * sh, h[4] * sh, h[5] * sh, 0};
    typedef unsigned int u4v __attribute__((ext_vector_type(4)));
    const uint4 q = pack8(v);
    const u4v qv = {q.x, q.y, q.z, q.w};
    __builtin_nontemporal_store(qv, reinterpret_cast<u4v*>(A + node * 16u));
  }
};
template <> __device__ inline float Plane3x8<_Float16>::unpack1(uint16_t b) {
  return (float)__builtin_bit_cast(_Float16, b);
}
template <> __device__ inline float Plane3x8<bf16_t>::unpack1(uint16_t b) { return bf16_to_f32(b); }
template <> __device__ inline void Plane3x8<_Float16>::unpack8(uint4 q, float* v) {
  const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[2 * k] = (float)__builtin_bit_cast(_Float16, (uint16_t)(w[k] & 0xffffu));
    v[2 * k + 1] = (float)__builtin_bit_cast(_Float16, (uint16_t)(w[k] >> 16));
  }
}
template <> __device__ inline void Plane3x8<bf16_t>::unpack8(uint4 q, float* v) {
  const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[2 * k] = __uint_as_float(w[k] << 16);
    v[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
  }
}
template <> __device__ inline uint4 Plane3x8<_Float16>::pack8(const float* v) {
  uint32_t w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    w[k] = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)v[2 * k]) |
           ((uint32_t)__builtin_bit_cast(uint16_t, (_Float16)v[2 * k + 1]) << 16);
  return make_uint4(w[0], w[1], w[2], w[3]);
}
template <> __device__ inline uint4 Plane3x8<bf16_t>::pack8(const float* v) {
  uint32_t w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    w[k] = (uint32_t)f32_to_bf16(v[2 * k]) | ((uint32_t)f32_to_bf16(v[2 * k + 1]) << 16);
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// FP32/FP64 plane access with the same signature as Plane3x8
template <class S> struct Plane3W {
  using R = S;
  __device__ static void load(const S* p, int i, uint32_t node, size_t N, R, R, R& f, R* h) {
    Plane3<S, 19>::load(p, i, node, N, f, h);
  }
  __device__ static R load_f(const S* p, int i, uint32_t node, size_t N, R) {
    return Plane3<S, 19>::load_f(p, i, node, N);
  }
  __device__ static void store(S* p, int i, uint32_t node, size_t N, R, R, R f, const R* h) {
    Plane3<S, 19>::store(p, i, node, N, f, h);
  }
};
template <class S> struct PlaneSel { using T = Plane3W<S>; };
template <> struct PlaneSel<_Float16> { using T = Plane3x8<_Float16>; };
template <> struct PlaneSel<bf16_t> { using T = Plane3x8<bf16_t>; };

// pull offsets of one node: per axis the 32-bit node delta to the source
// for c = +1, 0, -1 (periodic wrap folded in) and the wall flags
struct Pull3 {
  int d[3][3];
  bool lo[3], hi[3];
  uint32_t self;
};

__device__ inline void make_pull3(int x, int y, int z, const Geo& g, Pull3& p) {
  const int c[3] = {x, y, z}, n[3] = {g.nx, g.ny, g.nz};
  const int stride[3] = {1, g.nx, g.nx * g.ny};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const bool wall = g.walls & (1 << a);
    p.lo[a] = wall && c[a] == 0;
    p.hi[a] = wall && c[a] == n[a] - 1;
    p.d[a][0] = (c[a] == 0 ? n[a] - 1 : -1) * stride[a];  // source at x - 1
    p.d[a][1] = 0;
    p.d[a][2] = (c[a] == n[a] - 1 ? 1 - n[a] : 1) * stride[a];  // source at x + 1
  }
  p.self = (uint32_t)(((size_t)z * g.ny + y) * g.nx + x);
}

template <bool WALLS>
__device__ inline bool pull3_bounce(int i, const Pull3& p) {
  if (!WALLS) return false;
  const int cx = Lat<3>::cx(i), cy = Lat<3>::cy(i), cz = Lat<3>::cz(i);
  return (cx > 0 && p.lo[0]) || (cx < 0 && p.hi[0]) || (cy > 0 && p.lo[1]) ||
         (cy < 0 && p.hi[1]) || (cz > 0 && p.lo[2]) || (cz < 0 && p.hi[2]);
}

__device__ inline uint32_t pull3_node(int i, const Pull3& p) {
  const int cx = Lat<3>::cx(i), cy = Lat<3>::cy(i), cz = Lat<3>::cz(i);
  return (uint32_t)((int)p.self + p.d[0][1 - cx] + p.d[1][1 - cy] + p.d[2][1 - cz]);
}

// u = sum c_i f_i + F/2 for D3Q19, in one fixed evaluation order (shared by
// the lanes that own a node and those that fill the ring)
template <class R>
__device__ inline void velocity3(const R* f, const R* F, R* u) {
  u[0] = (((f[1] - f[2]) + (f[7] - f[8])) + ((f[9] - f[10]) + (f[11] - f[12]))) +
         (f[13] - f[14]) + (R)0.5 * F[0];
  u[1] = (((f[3] - f[4]) + (f[7] - f[8])) + ((f[10] - f[9]) + (f[15] - f[16]))) +
         (f[17] - f[18]) + (R)0.5 * F[1];
  u[2] = (((f[5] - f[6]) + (f[11] - f[12])) + ((f[14] - f[13]) + (f[15] - f[16]))) +
         (f[18] - f[17]) + (R)0.5 * F[2];
}

// Direction tables for loops that walk the velocity set with a runtime
// (wavefront-uniform) index: the loop bounds how many populations are in
// flight, and uniform table reads cost scalar loads only.
__constant__ int kC3[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                               {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                               {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                               {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
// f^B_i = sum_c K[i][c] tau_c / tau_f with tau in (xx, yy, zz, xy, xz, yz):
// the pseudo-inverse closed forms written as one row per direction
#define K42(a, b, c) {(a) / 42.0, (b) / 42.0, (c) / 42.0, 0.0, 0.0, 0.0}
__constant__ double kFB3[19][6] = {
    {5.0 / 21, 5.0 / 21, 5.0 / 21, 0, 0, 0},
    K42(-1, 6, 6), K42(-1, 6, 6), K42(6, -1, 6), K42(6, -1, 6), K42(6, 6, -1), K42(6, 6, -1),
    {-10.0 / 84, -10.0 / 84, 4.0 / 84, -21.0 / 84, 0, 0},
    {-10.0 / 84, -10.0 / 84, 4.0 / 84, -21.0 / 84, 0, 0},
    {-10.0 / 84, -10.0 / 84, 4.0 / 84, 21.0 / 84, 0, 0},
    {-10.0 / 84, -10.0 / 84, 4.0 / 84, 21.0 / 84, 0, 0},
    {-10.0 / 84, 4.0 / 84, -10.0 / 84, 0, -21.0 / 84, 0},
    {-10.0 / 84, 4.0 / 84, -10.0 / 84, 0, -21.0 / 84, 0},
    {-10.0 / 84, 4.0 / 84, -10.0 / 84, 0, 21.0 / 84, 0},
    {-10.0 / 84, 4.0 / 84, -10.0 / 84, 0, 21.0 / 84, 0},
    {4.0 / 84, -10.0 / 84, -10.0 / 84, 0, 0, -21.0 / 84},
    {4.0 / 84, -10.0 / 84, -10.0 / 84, 0, 0, -21.0 / 84},
    {4.0 / 84, -10.0 / 84, -10.0 / 84, 0, 0, 21.0 / 84},
    {4.0 / 84, -10.0 / 84, -10.0 / 84, 0, 0, 21.0 / 84}};
#undef K42

// runtime-direction versions of the pull helpers
template <bool WALLS>
__device__ inline bool pull3_bounce_rt(int i, const Pull3& p) {
  if (!WALLS) return false;
  const int cx = kC3[i][0], cy = kC3[i][1], cz = kC3[i][2];
  return (cx > 0 && p.lo[0]) || (cx < 0 && p.hi[0]) || (cy > 0 && p.lo[1]) ||
         (cy < 0 && p.hi[1]) || (cz > 0 && p.lo[2]) || (cz < 0 && p.hi[2]);
}
__device__ inline uint32_t pull3_node_rt(int i, const Pull3& p) {
  int off = (int)p.self;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int c = kC3[i][a];
    off += c > 0 ? p.d[a][0] : (c < 0 ? p.d[a][2] : 0);
  }
  return (uint32_t)off;
}
__device__ inline int opp3_rt(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

template <class S, int TY, int ZC, bool WALLS>
__global__ void __launch_bounds__(64 * TY, 2) step3d_kernel(StepArgs<S> a, int ntx, int nty) {
  using R = typename StoreT<S>::R;
  using PA = typename PlaneSel<S>::T;
  constexpr int Q = 19, NC = 6, TX = 64, SX = TX + 2, SY = TY + 2, NS = SX * SY;
  constexpr int H = 2 * SX + 2 * TY;
  constexpr int GROUP = 5;  // directions pulled together in pass 1 (loads in flight)
  __shared__ R ring[3][3][NS];

  const Geo g = a.g;
  const S* __restrict__ pin = a.pin;
  S* __restrict__ pout = a.pout;
  R* __restrict__ aux = a.aux;
  const size_t N = g.N;

  const int b = blockIdx.x;
  const int tx_tile = b % ntx, rest = b / ntx;
  const int ty_tile = rest % nty, zc = rest / nty;
  const int x0 = tx_tile * TX, y0 = ty_tile * TY;
  const int zs = zc * ZC, ze = min(zs + ZC, g.nz);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  const int x = x0 + tx, y = y0 + ty;
  const bool in_xy = x < g.nx && y < g.ny;
  const int oslot = (ty + 1) * SX + tx + 1;

  int wx = x, wy = y;
  const bool vxy = wrap_coord(wx, g.nx, g.walls & 1) && wrap_coord(wy, g.ny, g.walls & 2);
  bool hxy = false;
  int hx = 0, hy = 0, hslot = 0;
  if (tid < H) {
    int sxl, syl;
    if (tid < SX) { sxl = tid; syl = 0; }
    else if (tid < 2 * SX) { sxl = tid - SX; syl = SY - 1; }
    else if (tid < 2 * SX + TY) { sxl = 0; syl = 1 + tid - 2 * SX; }
    else { sxl = SX - 1; syl = 1 + tid - 2 * SX - TY; }
    hslot = syl * SX + sxl;
    hx = x0 - 1 + sxl;
    hy = y0 - 1 + syl;
    hxy = wrap_coord(hx, g.nx, g.walls & 1) && wrap_coord(hy, g.ny, g.walls & 2);
  }

  // f of direction i streamed into the node described by pl
  auto pull_f = [&](int i, const Pull3& pl) -> R {
    if (pull3_bounce<WALLS>(i, pl)) return PA::load_f(pin, Lat<3>::opp(i), pl.self, N, a.inv_sf);
    return PA::load_f(pin, i, pull3_node(i, pl), N, a.inv_sf);
  };
  auto pull_all = [&](int i, const Pull3& pl, R& f, R* h) {
    if (pull3_bounce_rt<WALLS>(i, pl))
      PA::load(pin, opp3_rt(i), pl.self, N, a.inv_sf, a.inv_sh, f, h);
    else
      PA::load(pin, i, pull3_node_rt(i, pl), N, a.inv_sf, a.inv_sh, f, h);
  };

  // velocity of plane zp (unwrapped index) into its ring slot: each lane
  // handles its own column and, for the first H lanes, one ring node
  auto plane_u = [&](int zp) {
    int zw = zp;
    const bool vz = wrap_coord(zw, g.nz, g.walls & 4);
    const int rs = ((zp % 3) + 3) % 3;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const bool on = vz && (k == 0 ? vxy : hxy);
      if (!on) continue;
      const int px = k == 0 ? wx : hx, py = k == 0 ? wy : hy, ps = k == 0 ? oslot : hslot;
      Pull3 pp;
      make_pull3(px, py, zw, g, pp);
      R f[Q], F[3], u[3];
#pragma unroll
      for (int i = 1; i < Q; ++i) f[i] = pull_f(i, pp);
      force_at<R>(a.F, px, py, g.nx, g.ny, F);
      velocity3(f, F, u);
      ring[rs][0][ps] = u[0];
      ring[rs][1][ps] = u[1];
      ring[rs][2][ps] = u[2];
    }
  };

  auto collide_node = [&](int xn, int yn, int zn) {
    Pull3 pl;
    make_pull3(xn, yn, zn, g, pl);
    const uint32_t n = pl.self;
    const int rc = ((zn % 3) + 3) % 3, rm = (((zn - 1) % 3) + 3) % 3, rp = ((zn + 1) % 3 + 3) % 3;
    // ---- pass 1: moments of the pulled state
    R e[NC] = {0, 0, 0, 0, 0, 0};
    R sum_f = 0;
#pragma unroll 1
    for (int g0 = 0; g0 < Q; g0 += GROUP) {
#pragma unroll
      for (int k = 0; k < GROUP; ++k) {
        const int i = g0 + k;
        if (i < Q) {
          R fi, hv[NC];
          pull_all(i, pl, fi, hv);
          if (i > 0) sum_f += fi;
#pragma unroll
          for (int c = 0; c < NC; ++c) e[c] += hv[c];
        }
      }
    }
    R chip[NC] = {0, 0, 0, 0, 0, 0}, up[3] = {0, 0, 0};
    if (!a.first) Aux<3, R>::load(aux, n, N, chip, up);
    // u(z) of this node is in the ring (same pulled values, same formula)
    const R u[3] = {ring[rc][0][oslot], ring[rc][1][oslot], ring[rc][2][oslot]};
    R F[3];
    force_at<R>(a.F, xn, yn, g.nx, g.ny, F);
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const R Fu = F[0] * u[0] + F[1] * u[1] + F[2] * u[2];
    R tau[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) tau[c] = a.P.eta_over_lam * e[c];
    auto fB_of = [&](int i) -> R {
      R sm = 0;
#pragma unroll
      for (int c = 0; c < NC; ++c) sm += (R)kFB3[i][c] * tau[c];
      return sm * a.P.inv_tau_f;
    };
    constexpr R w0 = (R)(1.0 / 3.0);
    const R F0 = -3 * w0 * a.P.k_f * Fu;
    // pressure (App. B): cs2/(1 - w0) = 1/2 for D3Q19
    const R p = (R)0.5 * (sum_f - (R)1.5 * w0 * uu + a.P.tau_f * F0 + a.P.tau_f * fB_of(0));
    // ---- same-time gradient and source tensor
    const bool lo[3] = {WALLS && (g.walls & 1) && xn == 0, WALLS && (g.walls & 2) && yn == 0,
                        WALLS && (g.walls & 4) && zn == 0};
    const bool hi[3] = {WALLS && (g.walls & 1) && xn == g.nx - 1,
                        WALLS && (g.walls & 2) && yn == g.ny - 1,
                        WALLS && (g.walls & 4) && zn == g.nz - 1};
    R G[3][3];
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) {
      const R* uc = &ring[rc][bb][oslot];
      const R nb[3][2] = {{uc[-1], uc[1]}, {uc[-SX], uc[SX]},
                          {ring[rm][bb][oslot], ring[rp][bb][oslot]}};
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        G[ax][bb] = lo[ax] ? u[bb] + nb[ax][1] * (R)(1.0 / 3.0)
                  : hi[ax] ? -(u[bb] + nb[ax][0] * (R)(1.0 / 3.0))
                           : (R)0.5 * (nb[ax][1] - nb[ax][0]);
      }
    }
    R chi[NC];
    source_tensor<3, R>(e, G, a.P.inv_lam, chi);
    const bool first = a.first != 0;
    R A[NC], target[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      A[c] = e[c] + (c < 3 ? (R)1 : (R)0);
      target[c] = e[c] + chi[c] + (first ? (R)0 : (R)0.5 * (chi[c] - chip[c]));
    }
    // one direction: BGK + Guo + f^B for f (Sec. 2.2), ADE collision for h (Sec. 2.3)
    auto collide_dir = [&](int i, R& fi, R* hv) {
      const int cx = kC3[i][0], cy = kC3[i][1], cz = kC3[i][2];
      const int c2 = cx * cx + cy * cy + cz * cz;
      const R wi = c2 == 0 ? (R)(1.0 / 3.0) : (c2 == 1 ? (R)(1.0 / 18.0) : (R)(1.0 / 36.0));
      const R lam_i = c2 == 0 ? (R)(3.0 * (1.0 / 3.0 - 1.0)) : 3 * wi;
      const R cu = (R)cx * u[0] + (R)cy * u[1] + (R)cz * u[2];
      const R cF = (R)cx * F[0] + (R)cy * F[1] + (R)cz * F[2];
      const R feq = lam_i * p + wi * (3 * cu + (R)4.5 * cu * cu - (R)1.5 * uu);
      const R Fi = wi * a.P.k_f * (3 * cF + 9 * cF * cu - 3 * Fu);
      fi = fi - (fi - feq) * a.P.inv_tau_f + fB_of(i) + Fi;
      const R cup = (R)cx * up[0] + (R)cy * up[1] + (R)cz * up[2];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const R heq = wi * e[c] + 3 * wi * A[c] * cu;
        const R chi_i = wi * chi[c] * (1 + a.P.k_h3 * cu);
        R srcv = chi_i;
        if (!first) srcv += (R)0.5 * (chi_i - wi * chip[c] * (1 + a.P.k_h3 * cup));
        hv[c] = hv[c] - (hv[c] - heq) * a.P.inv_tau_h + srcv;
      }
    };
    // ---- pass 2: moving non-axis directions are collided and stored at once
    R mom[3] = {0, 0, 0}, hsum[NC] = {0, 0, 0, 0, 0, 0};
#pragma unroll 1
    for (int g0 = 7; g0 < Q; g0 += 4) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i = g0 + k;
        R fi, hv[NC];
        pull_all(i, pl, fi, hv);
        collide_dir(i, fi, hv);
        mom[0] += (R)kC3[i][0] * fi;
        mom[1] += (R)kC3[i][1] * fi;
        mom[2] += (R)kC3[i][2] * fi;
#pragma unroll
        for (int c = 0; c < NC; ++c) hsum[c] += hv[c];
        PA::store(pout, i, n, N, a.sf, a.sh, fi, hv);
      }
    }
    // The momentum identity sum c f* = u + F/2 is restored on the axis pairs:
    // their f* is formed once from f alone to finish the momentum sum, then
    // the full populations are collided with the correction applied.  The
    // rest population of h closes sum_i h*_i = A - I + chi + dchi/2.
#pragma unroll
    for (int i = 1; i < 7; ++i) {
      R fi;
      if (pull3_bounce_rt<WALLS>(i, pl)) fi = PA::load_f(pin, opp3_rt(i), pl.self, N, a.inv_sf);
      else fi = PA::load_f(pin, i, pull3_node_rt(i, pl), N, a.inv_sf);
      R hdummy[NC] = {0, 0, 0, 0, 0, 0};
      collide_dir(i, fi, hdummy);
      mom[(i - 1) >> 1] += (i & 1) ? fi : -fi;
    }
    R half[3];
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) half[bb] = (R)0.5 * ((u[bb] + (R)0.5 * F[bb]) - mom[bb]);
#pragma unroll 1
    for (int g0 = 1; g0 < 7; g0 += 3) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int i = g0 + k;
        R fi, hv[NC];
        pull_all(i, pl, fi, hv);
        collide_dir(i, fi, hv);
        const int ax = (i - 1) >> 1;
        const R hb = ax == 0 ? half[0] : (ax == 1 ? half[1] : half[2]);
        fi += (i & 1) ? hb : -hb;
#pragma unroll
        for (int c = 0; c < NC; ++c) hsum[c] += hv[c];
        PA::store(pout, i, n, N, a.sf, a.sh, fi, hv);
      }
    }
    {
      R f0, h0[NC];
      pull_all(0, pl, f0, h0);
      collide_dir(0, f0, h0);
#pragma unroll
      for (int c = 0; c < NC; ++c) h0[c] = target[c] - hsum[c];
      PA::store(pout, 0, n, N, a.sf, a.sh, f0, h0);
    }
    Aux<3, R>::store(aux, n, N, chi, u);
  };

  plane_u(zs - 1);
  plane_u(zs);
#pragma unroll 1
  for (int z = zs; z < ze; ++z) {
    plane_u(z + 1);
    __syncthreads();
    if (in_xy) collide_node(x, y, z);
    __syncthreads();
  }
}

}  // namespace vflb
