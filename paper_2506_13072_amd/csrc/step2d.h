// step2d.h -- the fused D2Q9 step, specialised for gfx950.
//
// Workgroup = TY wavefronts of 64 lanes; each wavefront owns one 64-node
// row segment of a 64 x TY tile.  The 2 (64 + TY) halo nodes of the tile
// are assigned to the first lanes before any load is issued, so the halo
// pulls travel with the tile's own 36 population loads in one round trip.
// Tiles are numbered row-major in launch order (measured faster on MI355X
// than giving each XCD a contiguous band of tiles), and the outputs are
// written with non-temporal stores: they are read back only in the next
// step, long after they would have left the caches.
#pragma once

#include "kernels.h"

namespace vflb {

struct Pull2 {
  // in-plane offsets of the three columns and rows a node pulls from
  size_t col[3], row[3];  // index 0: from c = +1 (x-1), 1: c = 0, 2: c = -1 (x+1)
  bool lo_x, hi_x, lo_y, hi_y;  // node next to a wall on that side
  size_t self;
};

__device__ inline void make_pull2(int x, int y, const Geo& g, Pull2& p) {
  const bool wx = g.walls & 1, wy = g.walls & 2;
  const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
  p.col[0] = (size_t)xm;
  p.col[1] = (size_t)x;
  p.col[2] = (size_t)xp;
  p.row[0] = (size_t)ym * g.nx;
  p.row[1] = (size_t)y * g.nx;
  p.row[2] = (size_t)yp * g.nx;
  p.lo_x = wx && x == 0;
  p.hi_x = wx && x == g.nx - 1;
  p.lo_y = wy && y == 0;
  p.hi_y = wy && y == g.ny - 1;
  p.self = p.row[1] + p.col[1];
}

// index (plane offset included) of the value that streams into direction i
__device__ inline size_t pull2_index(int i, const Pull2& p, size_t N) {
  const int cx = Lat<2>::cx(i), cy = Lat<2>::cy(i);
  const bool bounce = (cx > 0 && p.lo_x) || (cx < 0 && p.hi_x) ||
                      (cy > 0 && p.lo_y) || (cy < 0 && p.hi_y);
  if (bounce) return (size_t)Lat<2>::opp(i) * N + p.self;
  return (size_t)i * N + p.row[1 - cy] + p.col[1 - cx];
}

// u = sum c_i f_i + F/2 (Sec. 2.2).  Evaluated by the owner of a node and
// by the lanes that fill the halo; no contraction into fused multiply-adds,
// so both give the same bits and results do not depend on the tile shape.
template <class R>
__device__ inline void velocity2(const R* f, const R* F, R* u) {
#pragma clang fp contract(off)
  u[0] = (f[1] - f[3] + f[5] - f[6] - f[7] + f[8]) + (R)0.5 * F[0];
  u[1] = (f[2] - f[4] + f[5] + f[6] - f[7] - f[8]) + (R)0.5 * F[1];
}

// LDS of one 64 x TY tile: the velocity on the tile and its one-node halo;
// for anchored storage also the anchors (E, p, u) of the tile and a
// two-node halo (the sources of the halo nodes' pulls)
template <class R, int TY, bool ANCHOR>
struct Tile2Lds {
  R su[2][66 * (TY + 2)];
};
template <class R, int TY>
struct Tile2Lds<R, TY, true> {
  R su[2][66 * (TY + 2)];
  float anc[6][68 * (TY + 4)];
};

// One 64 x TY tile of the step at origin (x0, y0).  The workgroup's lanes
// are (threadIdx.x, threadIdx.y) = (0..63, 0..TY-1); the tile contains one
// barrier, so every lane of the workgroup calls it.
template <class S, int TY>
using Tile2LdsOf = Tile2Lds<typename StoreT<S>::R, TY, StoreT<S>::kAnchored>;

// NT: the tile's own pulls use non-temporal loads (single lattices; the
// batched ensemble measured faster without)
template <class S, int TY, bool CLAMP = false, bool NT = false>
__device__ inline void step2d_tile(const StepArgs<S>& a, int x0, int y0,
                                   Tile2LdsOf<S, TY>& lds) {
  using R = typename StoreT<S>::R;
  constexpr bool ANCHOR = StoreT<S>::kAnchored;
  constexpr int Q = 9, NC = 3, TX = 64, SX = TX + 2, SY = TY + 2;
  // halo nodes of the tile: the rows above and below it and the columns
  // left and right of it, without the four corners (the gradient's stencil
  // reads the axis neighbours only)
  constexpr int H = 2 * TX + 2 * TY;
  constexpr int AX = TX + 4, AY = TY + 4;  // anchor region (two-node halo)
  R (*su)[SX * SY] = lds.su;

  const Geo g = a.g;
  const S* __restrict__ pin = a.pin;
  S* __restrict__ pout = a.pout;
  R* __restrict__ aux = a.aux;
  const size_t N = g.N;
  using P2 = Pops<2, S>;

  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = ty * TX + tx;
  const int x = x0 + tx, y = y0 + ty;
  const bool active = x < g.nx && y < g.ny;

  // ---- halo node of this lane (if any): coordinates, slot, pull offsets
  bool hvalid = false;
  int hslot = 0, hx = 0, hy = 0;
  if (tid < H) {
    int sxl, syl;
    if (tid < TX) { sxl = 1 + tid; syl = 0; }
    else if (tid < 2 * TX) { sxl = 1 + tid - TX; syl = SY - 1; }
    else if (tid < 2 * TX + TY) { sxl = 0; syl = 1 + tid - 2 * TX; }
    else { sxl = SX - 1; syl = 1 + tid - 2 * TX - TY; }
    hslot = syl * SX + sxl;
    hx = x0 - 1 + sxl;
    hy = y0 - 1 + syl;
    hvalid = wrap_coord(hx, g.nx, g.walls & 1) && wrap_coord(hy, g.ny, g.walls & 2);
  }
  // own node, wrapped for lanes past a ragged edge (they supply the slot's
  // velocity for the true last node's gradient)
  int wx = x, wy = y;
  const bool valid = wrap_coord(wx, g.nx, g.walls & 1) && wrap_coord(wy, g.ny, g.walls & 2);

  // ---- issue every load of the step.  With anchored 16-bit storage two
  // workgroups share a CU; raising this wave's priority while it issues
  // lets the other workgroup's collision yield to it (measured on MI355X:
  // the 8192 x 1024 step 0.436 -> 0.408 ms FP16, 0.420 -> 0.409 ms BF16;
  // neutral for FP64, whose tiles also pair up, and for FP32, one per CU)
  if constexpr (ANCHOR) __builtin_amdgcn_s_setprio(2);
  R fh[Q];
  if (hvalid) {
    Pull2 ph;
    make_pull2(hx, hy, g, ph);
#pragma unroll
    for (int i = 1; i < Q; ++i) fh[i] = P2::load_f(pin, pull2_index(i, ph, N), N, a.inv_sf);
  }
  Pull2 p;
  make_pull2(wx, wy, g, p);
  R f[Q];
  R h[NC][Q];
  R chip[NC] = {0, 0, 0}, up[2] = {0, 0};
  const size_t n = p.self;
  if (active) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      R hv[NC];
      P2::template load<NT>(pin, pull2_index(i, p, N), N, a.inv_sf, a.inv_sh, f[i], hv);
#pragma unroll
      for (int c = 0; c < NC; ++c) h[c][i] = hv[c];
    }
    if (!a.first) Aux<2, R>::load(aux, n, N, chip, up);
  } else if (valid) {
#pragma unroll
    for (int i = 1; i < Q; ++i) f[i] = P2::load_f(pin, pull2_index(i, p, N), N, a.inv_sf);
  }

  if constexpr (ANCHOR) {
    __builtin_amdgcn_s_setprio(0);
    // anchors of the tile and a two-node halo into LDS (coordinates wrap
    // like the pulls; slots beyond a wall stay unused)
    for (int k = tid; k < AX * AY; k += TX * TY) {
      int ax = x0 - 2 + k % AX, ay = y0 - 2 + k / AX;
      if (wrap_coord(ax, g.nx, g.walls & 1) && wrap_coord(ay, g.ny, g.walls & 2)) {
        float4 q;
        float2 v;
        Anchor2::load(pin, (size_t)ay * g.nx + ax, N, q, v);
        lds.anc[0][k] = q.x;
        lds.anc[1][k] = q.y;
        lds.anc[2][k] = q.z;
        lds.anc[3][k] = q.w;
        lds.anc[4][k] = v.x;
        lds.anc[5][k] = v.y;
      }
    }
    __syncthreads();
    // value = reference of the writing node + stored deviation; the writer
    // of direction i is x - c_i, or the node itself (direction opp(i))
    // behind a wall
    auto rebuild = [&](int i, int cx0, int cy0, const Pull2& pp, R& fv, R* hv, bool with_h) {
      const int cx = Lat<2>::cx(i), cy = Lat<2>::cy(i);
      const bool bounce = (cx > 0 && pp.lo_x) || (cx < 0 && pp.hi_x) ||
                          (cy > 0 && pp.lo_y) || (cy < 0 && pp.hi_y);
      const int sx = bounce ? cx0 : cx0 - cx, sy = bounce ? cy0 : cy0 - cy;
      const int k = (sy - (y0 - 2)) * AX + (sx - (x0 - 2));
      const R sgn = bounce ? (R)-1 : (R)1;
      const R ux = lds.anc[4][k], uy = lds.anc[5][k];
      fv += fref2<R>(i, sgn, (R)lds.anc[3][k], ux, uy);
      if (with_h) {
#pragma unroll
        for (int c = 0; c < NC; ++c) hv[c] += href2<R>(i, c, sgn, (R)lds.anc[c][k], ux, uy);
      }
    };
    if (hvalid) {
      Pull2 ph;
      make_pull2(hx, hy, g, ph);
      const int ux0 = x0 - 1 + (hslot % SX), uy0 = y0 - 1 + (hslot / SX);
#pragma unroll
      for (int i = 1; i < Q; ++i) rebuild(i, ux0, uy0, ph, fh[i], nullptr, false);
    }
    if (active) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        R hv[NC] = {h[0][i], h[1][i], h[2][i]};
        rebuild(i, x, y, p, f[i], hv, true);
#pragma unroll
        for (int c = 0; c < NC; ++c) h[c][i] = hv[c];
      }
    } else if (valid) {
#pragma unroll
      for (int i = 1; i < Q; ++i) rebuild(i, x, y, p, f[i], nullptr, false);
    }
  }

  // ---- velocities into LDS
  R u[3] = {0, 0, 0}, F[3] = {0, 0, 0};
  if (valid) {
    force_at<R>(a.F, wx, wy, 0, g, F);
    velocity2(f, F, u);
    if (CLAMP && (a.clamp_flags & 1)) {
      u[0] = (R)a.clamp[(size_t)wy * g.nx + wx];
      u[1] = (R)a.clamp[N + (size_t)wy * g.nx + wx];
    }
    const int slot = (ty + 1) * SX + tx + 1;
    su[0][slot] = u[0];
    su[1][slot] = u[1];
  }
  if (hvalid) {
    R Fh[3], uh[3];
    force_at<R>(a.F, hx, hy, 0, g, Fh);
    velocity2(fh, Fh, uh);
    if (CLAMP && (a.clamp_flags & 1)) {
      uh[0] = (R)a.clamp[(size_t)hy * g.nx + hx];
      uh[1] = (R)a.clamp[N + (size_t)hy * g.nx + hx];
    }
    su[0][hslot] = uh[0];
    su[1][hslot] = uh[1];
  }

  // ---- f collision and store (needs A from h, not the gradient)
  R e[NC];
  R pnew = 0;
  if (active) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      R s = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) s += h[c][i];
      e[c] = s;
    }
    if (CLAMP && (a.clamp_flags & 2)) {  // A - I = tau lambda / eta_p
#pragma unroll
      for (int c = 0; c < NC; ++c)
        e[c] = a.P.eta_over_lam > 0 ? (R)a.clamp[(2 + c) * N + n] / a.P.eta_over_lam : (R)0;
    }
    pnew = collide_f<2, R>(f, e, u, F, a.P);
  }
  __syncthreads();
  if (!active) return;

  // ---- same-time velocity gradient G[a][b] = d_a u_b
  R G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  const int slot = (ty + 1) * SX + tx + 1;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const R* ub = &su[b][slot];
    G[0][b] = p.lo_x ? u[b] + ub[1] * (R)(1.0 / 3.0)
            : p.hi_x ? -(u[b] + ub[-1] * (R)(1.0 / 3.0))
                     : (R)0.5 * (ub[1] - ub[-1]);
    G[1][b] = p.lo_y ? u[b] + ub[SX] * (R)(1.0 / 3.0)
            : p.hi_y ? -(u[b] + ub[-SX] * (R)(1.0 / 3.0))
                     : (R)0.5 * (ub[SX] - ub[-SX]);
  }
  R chi[NC];
  source_tensor<2, R>(e, G, a.P, chi);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const R Ac = e[c] + ((c != 1) ? (R)1 : (R)0);
    collide_h<2, R>(h[c], e[c], Ac, chi[c], chip[c], u, up, a.first != 0, a.P);
  }
  if constexpr (ANCHOR) {
    // new anchor: E = sum_i h*_i (the rest population closed that sum), the
    // pressure and the velocity of this step; store the deviations from it
    R En[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      R sm = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) sm += h[c][i];
      En[c] = sm;
    }
    const float4 q = {(float)En[0], (float)En[1], (float)En[2], (float)pnew};
    const float2 v = {(float)u[0], (float)u[1]};
    const R e0 = (R)q.x, e1 = (R)q.y, e2 = (R)q.z, pp = (R)q.w, ux = (R)v.x, uy = (R)v.y;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R fd = f[i] - fref2<R>(i, (R)1, pp, ux, uy);
      const R hv[NC] = {h[0][i] - href2<R>(i, 0, (R)1, e0, ux, uy),
                        h[1][i] - href2<R>(i, 1, (R)1, e1, ux, uy),
                        h[2][i] - href2<R>(i, 2, (R)1, e2, ux, uy)};
      P2::store(pout, (size_t)i * N + n, N, a.sf, a.sh, fd, hv);
    }
    Anchor2::store(pout, n, N, q, v);
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R hv[NC] = {h[0][i], h[1][i], h[2][i]};
      P2::store(pout, (size_t)i * N + n, N, a.sf, a.sh, f[i], hv);
    }
  }
  Aux<2, R>::store(aux, n, N, chi, u);
}

// CLAMP: a settling step (StepArgs::clamp); compiled separately so that the
// production step carries none of it
template <class S, int TY, bool CLAMP = false>
__global__ void __launch_bounds__(64 * TY) step2d_kernel(StepArgs<S> a, int ntx, int nty) {
  __shared__ Tile2LdsOf<S, TY> lds;
  (void)nty;
  step2d_tile<S, TY, CLAMP, true>(a, (blockIdx.x % ntx) * 64, (blockIdx.x / ntx) * TY, lds);
}

// ------------------------------------------- in-place (AA) streaming
// One population buffer instead of two.  A step at even t reads the
// pre-collision values of a node from its own slots and writes the
// post-collision values back into the same node's slots under the opposite
// directions; a step at odd t reads each value from the slot its writer left
// it in (x - c_i, opposite direction) and writes the post-collision values
// into the slots their readers of the next step own (x + c_i, same
// direction; behind a wall the node itself, opposite direction).  Every slot
// is read and written by one node within a step, so the buffer needs no
// copy.  Neighbours' slots are overwritten during the step, so the same-time
// velocity comes from a separate pass (aa_velocity_kernel) into u [2][N].
// The arithmetic is step2d_tile's, operation for operation, so a lattice
// stepped in place takes bitwise the values it takes with two buffers.
// The buffer holds Planar storage (f and each h component in planes), so
// the velocity pass reads the f plane alone.  Both kernels give a lane one
// node: blockIdx.x a run of x, blockIdx.y (and its strides) the rows.

// index of the slot that the reader of the next step expects f*_i of
// node (x, y) in (g.aa: the layout of the state being read, 1 or 2)
__device__ inline size_t aa_write_index(int i, int x, int y, const Geo& g) {
  const size_t n = (size_t)y * g.nx + x;
  const int opp = Lat<2>::opp(i);
  if (g.aa == 1) return (size_t)opp * g.N + n;  // next state swapped: own node
  int tx = x + Lat<2>::cx(i), ty = y + Lat<2>::cy(i);
  if ((g.walls & 1) && (tx < 0 || tx >= g.nx)) return (size_t)opp * g.N + n;
  if ((g.walls & 2) && (ty < 0 || ty >= g.ny)) return (size_t)opp * g.N + n;
  tx = tx < 0 ? g.nx - 1 : (tx >= g.nx ? 0 : tx);
  ty = ty < 0 ? g.ny - 1 : (ty >= g.ny ? 0 : ty);
  return (size_t)i * g.N + (size_t)ty * g.nx + tx;
}

template <class S>
__global__ void __launch_bounds__(256) aa_velocity_kernel(const S* __restrict__ pop, Geo g,
                                                          ForceArgs<typename StoreT<S>::R> fa,
                                                          typename StoreT<S>::R inv_sf,
                                                          typename StoreT<S>::R* __restrict__ U) {
  using R = typename StoreT<S>::R;
  const size_t N = g.N;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  for (int y = blockIdx.y; y < g.ny; y += gridDim.y) {
    const size_t n = (size_t)y * g.nx + x;
    R f[9], F[3], u[3];
    f[0] = 0;
#pragma unroll
    for (int i = 1; i < 9; ++i) f[i] = Pops<2, S>::load_f(pop, pull_index<2>(i, x, y, 0, g), N, inv_sf);
    force_at<R>(fa, x, y, 0, g, F);
    velocity2(f, F, u);
    U[n] = u[0];
    U[N + n] = u[1];
  }
}

template <class S>
__global__ void __launch_bounds__(256) aa_step_kernel(StepArgs<S> a,
                                                      const typename StoreT<S>::R* __restrict__ U) {
  using R = typename StoreT<S>::R;
  constexpr int Q = 9, NC = 3;
  constexpr bool kF64 = std::is_same<R, double>::value;
  using P2 = Pops<2, S>;
  const Geo g = a.g;
  S* __restrict__ pop = a.pout;
  R* __restrict__ aux = a.aux;
  const size_t N = g.N;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  for (int y = blockIdx.y; y < g.ny; y += gridDim.y) {
    const size_t n = (size_t)y * g.nx + x;
    Pull2 p;
    make_pull2(x, y, g, p);
    R f[Q], h[NC][Q];
    R chip[NC] = {0, 0, 0}, up[2] = {0, 0};
    // raised priority while the loads issue (measured on MI355X, 8192 x
    // 1024 FP32: 0.576 -> 0.568 ms per in-place step; FP64 neutral)
    if constexpr (!kF64) __builtin_amdgcn_s_setprio(2);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      R hv[NC];
      P2::load(pop, pull_index<2>(i, x, y, 0, g), N, a.inv_sf, a.inv_sh, f[i], hv);
#pragma unroll
      for (int c = 0; c < NC; ++c) h[c][i] = hv[c];
    }
    if (!a.first) Aux<2, R>::load(aux, n, N, chip, up);
    R F[3] = {0, 0, 0};
    force_at<R>(a.F, x, y, 0, g, F);
    const R u[3] = {U[n], U[N + n], (R)0};
    if constexpr (!kF64) __builtin_amdgcn_s_setprio(0);
    R e[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      R s = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) s += h[c][i];
      e[c] = s;
    }
    collide_f<2, R>(f, e, u, F, a.P);
    // same-time velocity gradient G[a][b] = d_a u_b (as in step2d_tile)
    R G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const R* Ub = U + (size_t)b * N;
      const R uxm = Ub[p.row[1] + p.col[0]], uxp = Ub[p.row[1] + p.col[2]];
      const R uym = Ub[p.row[0] + p.col[1]], uyp = Ub[p.row[2] + p.col[1]];
      G[0][b] = p.lo_x ? u[b] + uxp * (R)(1.0 / 3.0)
              : p.hi_x ? -(u[b] + uxm * (R)(1.0 / 3.0))
                       : (R)0.5 * (uxp - uxm);
      G[1][b] = p.lo_y ? u[b] + uyp * (R)(1.0 / 3.0)
              : p.hi_y ? -(u[b] + uym * (R)(1.0 / 3.0))
                       : (R)0.5 * (uyp - uym);
    }
    R chi[NC];
    source_tensor<2, R>(e, G, a.P, chi);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const R Ac = e[c] + ((c != 1) ? (R)1 : (R)0);
      collide_h<2, R>(h[c], e[c], Ac, chi[c], chip[c], u, up, a.first != 0, a.P);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R hv[NC] = {h[0][i], h[1][i], h[2][i]};
      P2::store(pop, aa_write_index(i, x, y, g), N, a.sf, a.sh, f[i], hv);
    }
    Aux<2, R>::store(aux, n, N, chi, u);
  }
}

// Batched step over many lattices: a persistent launch whose workgroups walk
// a flattened table of (instance, tile) entries.  desc[inst] holds the
// instance's step arguments with pin in the buffer of parity 0; for parity 1
// the two population buffers swap.  Each tile runs the very same tile
// function as the single-lattice kernel, so a lattice advanced inside a
// batch takes bitwise the values it takes alone.
template <class S, int TY>
__global__ void __launch_bounds__(64 * TY) batch2d_kernel(const BatchInst<S>* __restrict__ desc,
                                                         const BatchTile* __restrict__ tiles,
                                                         int ntiles, int parity, int first) {
  __shared__ Tile2LdsOf<S, TY> lds;
  for (int k = blockIdx.x; k < ntiles; k += gridDim.x) {
    const BatchTile e = tiles[k];
    StepArgs<S> a = desc[e.inst].a;
    if (parity) {
      const S* in = a.pout;
      a.pout = const_cast<S*>(a.pin);
      a.pin = in;
    }
    a.first = first;
    step2d_tile<S, TY>(a, e.x0, e.y0, lds);
    __syncthreads();  // the next tile reuses the LDS
  }
}

}  // namespace vflb
