// step3d.h -- the fused D3Q19 step for gfx950, marching along z.
//
// Two lanes own one node.  The even lane holds the rest population and the
// odd member (2k-1) of each opposite pair, the odd lane the even member
// (2k): lane s sees pair k with velocity (1 - 2s) c_{2k-1}.  The pair's
// partial moments meet through one DPP lane swap each, so a lane keeps ten
// populations of f and h (about 70 values) and two workgroups per CU stay
// resident (two wavefronts per SIMD).  Each direction has its own plane in
// HBM (one plane per direction); lane s of a pair addresses the pair's
// plane base with the 32-bit offset s N + source node.
//
// A workgroup of TY wavefronts owns a 32 x TY column of nodes and walks a
// chunk of ZC planes in z.  The velocity of three consecutive planes
// (z-1, z, z+1) plus a one-node ring in x and y lives in LDS, so the
// same-time gradient needs no halo in z.  The walk is software-pipelined:
// while plane z collides, the pulled h tuples, rest f and previous-step
// source state of plane z+1 travel by LDS-DMA (global_load_lds) into an LDS
// stage, and the moving f of plane z+2 (own column and ring, for u(z+2))
// into registers.  A lane keeps the f it pulled for its own node and
// collides it two planes later, so f crosses HBM once and h once.
// Blocks are renumbered so that each XCD walks one contiguous run of tiles.
// 16-bit storage is anchored (layout.h): each pulled value is rebuilt from
// its 16-bit deviation and the reference of its writer's FP32 anchor (read
// from an LDS stage of the anchors around the tile, AnchorStage), and the
// stored values are deviations from the node's new anchor (E = the
// conformation moment the h collision produces, the pressure, u), which the
// even lane stores.  The anchored step has no LDS stage for the tuples (the
// anchor stage takes its place): it loads the raw 16-bit tuples of plane
// z+1 into registers while plane z collides, and runs one wave per SIMD.
// Its per-plane cost is arithmetic more than memory: the references are
// evaluated in a factored form with explicit fused multiply-adds (one
// multiply or fused multiply-add per component), measured on MI355X at
// 512^3: 42.6 ms per step with separate multiplies and adds, 38.0 ms so.
#pragma once

#include "kernels.h"

namespace vflb {

// planes per workgroup chunk of the z march: measured on MI355X (512^3,
// FP32): 8: 29.8 ms, 12: 28.9, 16: 28.7, 24: 30.2, 32: 30.3, 64: 30.0,
// 128: 31.9 ms per step (same box)
constexpr int kStep3dChunk = 16;

// conversion between the storage type and the arithmetic type (scale: the
// exact power of two of FP16 storage; unused otherwise)
template <class S> struct Cvt;
template <> struct Cvt<double> {
  using V = double;
  __device__ static double in(V v, double) { return v; }
  __device__ static V out(double v, double) { return v; }
};
template <> struct Cvt<float> {
  using V = float;
  __device__ static float in(V v, float) { return v; }
  __device__ static V out(float v, float) { return v; }
};
template <> struct Cvt<_Float16> {
  using V = _Float16;
  __device__ static float in(V v, float inv_scale) { return (float)v * inv_scale; }
  __device__ static V out(float v, float scale) { return (_Float16)(v * scale); }
};
template <> struct Cvt<bf16_t> {
  using V = uint16_t;
  __device__ static float in(V v, float) { return bf16_to_f32(v); }
  __device__ static V out(float v, float) { return f32_to_bf16(v); }
};

// Access to the D3Q19 population buffer by pair: k = 0 is the rest plane
// (offset o = node), k = 1..9 the planes of directions 2k-1 and 2k, which
// follow one another (offset o = member N + node).  f, the (xx, yy, zz, xy)
// 4-tuples and the (xz, yz) 2-tuples follow one another, each Q N tuples
// long.
template <class S> struct Pair3 {
  using C = Cvt<S>;
  using V = typename C::V;
  using R = typename StoreT<S>::R;
  typedef V v4 __attribute__((ext_vector_type(4)));
  typedef V v2 __attribute__((ext_vector_type(2)));
  static constexpr int Q = 19;
  __device__ static size_t t0(int k, size_t N) { return k == 0 ? 0 : (size_t)(2 * k - 1) * N; }
  __device__ static const char* fb(const S* p, int k, size_t N) {
    return reinterpret_cast<const char*>(reinterpret_cast<const V*>(p) + t0(k, N));
  }
  __device__ static const char* h4b(const S* p, int k, size_t N) {
    return reinterpret_cast<const char*>(reinterpret_cast<const V*>(p) + (size_t)Q * N +
                                         4 * t0(k, N));
  }
  __device__ static const char* h2b(const S* p, int k, size_t N) {
    return reinterpret_cast<const char*>(reinterpret_cast<const V*>(p) + (size_t)5 * Q * N +
                                         2 * t0(k, N));
  }
  __device__ static R load_f(const S* p, int k, uint32_t o, size_t N, R isf) {
    return C::in(*reinterpret_cast<const V*>(fb(p, k, N) + o * (uint32_t)sizeof(V)), isf);
  }
  // anchored storage: the stored 16-bit values as they are, converted when
  // used (loads issued a plane ahead)
  __device__ static V load_f_raw(const S* p, int k, uint32_t o, size_t N) {
    return *reinterpret_cast<const V*>(fb(p, k, N) + o * (uint32_t)sizeof(V));
  }
  __device__ static void load_h_raw(const S* p, int k, uint32_t o, size_t N, v4& a, v2& b) {
    a = *reinterpret_cast<const v4*>(h4b(p, k, N) + o * (uint32_t)sizeof(v4));
    b = *reinterpret_cast<const v2*>(h2b(p, k, N) + o * (uint32_t)sizeof(v2));
  }
  __device__ static void load_h(const S* p, int k, uint32_t o, size_t N, R ish, R* h) {
    const v4 a = *reinterpret_cast<const v4*>(h4b(p, k, N) + o * (uint32_t)sizeof(v4));
    const v2 b = *reinterpret_cast<const v2*>(h2b(p, k, N) + o * (uint32_t)sizeof(v2));
    h[0] = C::in(a.x, ish); h[1] = C::in(a.y, ish); h[2] = C::in(a.z, ish);
    h[3] = C::in(a.w, ish); h[4] = C::in(b.x, ish); h[5] = C::in(b.y, ish);
  }
  // anchored storage: deviations already scaled, converted as they are
  __device__ static void store_dev(S* p, int k, uint32_t o, size_t N, R f, const R* h) {
    const v4 a = {(V)h[0], (V)h[1], (V)h[2], (V)h[3]};
    const v2 b = {(V)h[4], (V)h[5]};
    __builtin_nontemporal_store(
        (V)f, reinterpret_cast<V*>(const_cast<char*>(fb(p, k, N)) + o * (uint32_t)sizeof(V)));
    __builtin_nontemporal_store(
        a, reinterpret_cast<v4*>(const_cast<char*>(h4b(p, k, N)) + o * (uint32_t)sizeof(v4)));
    __builtin_nontemporal_store(
        b, reinterpret_cast<v2*>(const_cast<char*>(h2b(p, k, N)) + o * (uint32_t)sizeof(v2)));
  }
  __device__ static void store(S* p, int k, uint32_t o, size_t N, R sf, R sh, R f, R hxx, R hyy,
                               R hzz, R hxy, R hxz, R hyz) {
    const v4 a = {C::out(hxx, sh), C::out(hyy, sh), C::out(hzz, sh), C::out(hxy, sh)};
    const v2 b = {C::out(hxz, sh), C::out(hyz, sh)};
    __builtin_nontemporal_store(
        C::out(f, sf),
        reinterpret_cast<V*>(const_cast<char*>(fb(p, k, N)) + o * (uint32_t)sizeof(V)));
    __builtin_nontemporal_store(
        a, reinterpret_cast<v4*>(const_cast<char*>(h4b(p, k, N)) + o * (uint32_t)sizeof(v4)));
    __builtin_nontemporal_store(
        b, reinterpret_cast<v2*>(const_cast<char*>(h2b(p, k, N)) + o * (uint32_t)sizeof(v2)));
  }
};

// value of the partner lane (lanes 2j and 2j + 1): DPP quad permutation
// [1, 0, 3, 2]; both lanes of a pair are always active together
__device__ inline float pair_swap(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ inline double pair_swap(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, 0xB1, 0xF, 0xF,
                                                            false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), 0xB1,
                                                            0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// sum over the pair: the same bits in both lanes (addition commutes)
template <class R>
__device__ inline R pair_sum(R v) {
  return v + pair_swap(v);
}

// Pull geometry of one node as seen by the lane of member s.  A direction
// of this lane with odd-member velocity component c_a = +1 streams from the
// neighbour at node delta dm[a] (wm[a]: a wall lies there, bounce back),
// c_a = -1 from dp[a] (wp[a]); periodic wrap is folded into the deltas.
struct PairPull {
  int dm[3], dp[3];
  bool wm[3], wp[3];
  bool lo[3], hi[3];  // node next to a wall at coordinate 0 / n - 1
  uint32_t self;
};

__device__ inline void make_pair_pull(int x, int y, int z, int s, const Geo& g, PairPull& p) {
  const int c[3] = {x, y, z}, n[3] = {g.nx, g.ny, g.nz};
  const int stride[3] = {1, g.nx, g.nx * g.ny};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const bool wall = g.walls & (1 << a);
    p.lo[a] = wall && c[a] == 0;
    p.hi[a] = wall && c[a] == n[a] - 1;
    const int from_minus = (c[a] == 0 ? n[a] - 1 : -1) * stride[a];     // source at x - 1
    const int from_plus = (c[a] == n[a] - 1 ? 1 - n[a] : 1) * stride[a];  // source at x + 1
    p.dm[a] = s ? from_plus : from_minus;
    p.dp[a] = s ? from_minus : from_plus;
    p.wm[a] = s ? p.hi[a] : p.lo[a];
    p.wp[a] = s ? p.lo[a] : p.hi[a];
  }
  p.self = (uint32_t)(((size_t)z * g.ny + y) * g.nx + x);
}

// offset from pair plane k of the value that streams into this lane's
// member of pair k: the neighbour's member (s N + src) or, beyond a wall,
// the node's own opposite population, the partner's member ((1 - s) N + self)
template <int K, bool WALLS>
__device__ inline uint32_t pair_src(const PairPull& p, int s, uint32_t N) {
  constexpr int i = 2 * K - 1;
  constexpr int cx = Lat<3>::cx(i), cy = Lat<3>::cy(i), cz = Lat<3>::cz(i);
  const int off = (int)p.self + (cx > 0 ? p.dm[0] : (cx < 0 ? p.dp[0] : 0)) +
                  (cy > 0 ? p.dm[1] : (cy < 0 ? p.dp[1] : 0)) +
                  (cz > 0 ? p.dm[2] : (cz < 0 ? p.dp[2] : 0));
  if (WALLS) {
    const bool bounce = (cx > 0 && p.wm[0]) || (cx < 0 && p.wp[0]) || (cy > 0 && p.wm[1]) ||
                        (cy < 0 && p.wp[1]) || (cz > 0 && p.wm[2]) || (cz < 0 && p.wp[2]);
    if (bounce) return (s ? 0u : N) + p.self;
  }
  return (s ? N : 0u) + (uint32_t)off;
}

// In-place (AA) streaming by pairs, the index maps of the in-place D3Q19
// step (aa3d.h) seen from a lane's member: at even t (Geo::aa == 1) a lane
// reads its member from the node's own slots and writes it into the
// partner's member of the same node; at odd t it reads the partner's member
// at x - c (the two-buffer pull with the members swapped; beyond a wall the
// node's own member) and writes its own member at x + c (beyond a wall the
// partner's member of the node itself).
template <int K, bool WALLS>
__device__ inline uint32_t aa_pair_src(const PairPull& p, int s, int aa, uint32_t N) {
  if (aa == 1) return (s ? N : 0u) + p.self;
  const uint32_t o = pair_src<K, WALLS>(p, s, N);
  return o >= N ? o - N : o + N;
}
// p: the pull geometry of the lane (member s); the destination x + c of its
// member is the source of the partner's member
template <int K, bool WALLS>
__device__ inline uint32_t aa_pair_dst(const PairPull& p, int s, int aa, uint32_t N) {
  if (aa == 1) return (s ? 0u : N) + p.self;
  PairPull q = p;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    q.dm[a] = p.dp[a];
    q.dp[a] = p.dm[a];
    q.wm[a] = p.wp[a];
    q.wp[a] = p.wm[a];
  }
  const uint32_t o = pair_src<K, WALLS>(q, 1 - s, N);
  return o >= N ? o - N : o + N;
}

template <int K, class F>
__device__ inline void for_pairs(F&& fn) {
  if constexpr (K <= 9) {
    fn(std::integral_constant<int, K>());
    for_pairs<K + 1>(fn);
  }
}

// Workgroup barrier for the velocity ring in LDS: this wave's LDS accesses
// complete, then all waves meet.  Unlike a fenced barrier it leaves global
// loads, stores and LDS-DMA loads in flight (the LDS-DMA slots are private
// to their lane and waited for explicitly).  The memory clobber keeps the
// compiler from moving memory accesses across it.
__device__ inline void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// s_waitcnt immediates (gfx9 family): vmcnt in bits 3:0 and 15:14, expcnt
// in 6:4, lgkmcnt in 11:8; a field at its maximum does not wait.
constexpr int waitcnt_vm(int n) { return (n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14); }
constexpr int waitcnt_lgkm(int n) { return 15 | (3 << 14) | (7 << 4) | (n << 8); }
static_assert(waitcnt_vm(32) == 0x8F70 && waitcnt_vm(0) == 0x0F70 && waitcnt_lgkm(0) == 0xC07F,
              "s_waitcnt encoding");

// LDS-DMA (global_load_lds): each lane of a wave writes the bytes it loads
// to a lane-contiguous slot of the wave's LDS block, at base + lane * bytes.
template <int BYTES>
__device__ inline void dma_to_lds(const void* src, void* wave_block) {
  static_assert(BYTES == 4 || BYTES == 16, "LDS-DMA of 4 or 16 bytes per lane");
  if constexpr (BYTES == 16)
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)wave_block, 16,
                                     0, 0);
  else
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)wave_block, 4,
                                     0, 0);
}

// One plane of a workgroup's pulled state, staged in LDS by LDS-DMA loads
// issued one plane ahead of their use: per wave and pair the lane slots of
// the h tuples, the rest f and the previous-step source state.  A lane reads
// back only what it loaded itself.
template <class S, int TY> struct Stage3 {};  // FP64, 16-bit: loads straight to registers
template <int TY> struct Stage3<float, TY> {
  float4 h4[TY][10][64];
  float h2[2][TY][10][64];
  float f0[TY][64];
  float aux[5][TY][64];  // previous-step state q = 2 j + s in slot j of lane s
};

template <class S, int TY, bool WALLS, bool AA = false>
__device__ inline void stage_issue(Stage3<S, TY>& st, const S* pin, const typename StoreT<S>::R* aux,
                                   const PairPull& pq, int s, size_t N, bool first, int ty,
                                   int aa = 0) {
  using PA = Pair3<S>;
  const uint32_t N32 = (uint32_t)N, n = pq.self;
  auto issue_h = [&](int k, uint32_t o) {
    const char* a = PA::h4b(pin, k, N) + o * 16u;
    const char* b = PA::h2b(pin, k, N) + o * 8u;
    dma_to_lds<16>(a, &st.h4[ty][k][0]);
    dma_to_lds<4>(b, &st.h2[0][ty][k][0]);
    dma_to_lds<4>(b + 4, &st.h2[1][ty][k][0]);
  };
  issue_h(0, n);  // rest: both lanes, one address
  for_pairs<1>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if constexpr (AA)
      issue_h(k, aa_pair_src<k, WALLS>(pq, s, aa, N32));
    else
      issue_h(k, pair_src<k, WALLS>(pq, s, N32));
  });
  dma_to_lds<4>(pin + n, &st.f0[ty][0]);
  if (!first) {
    // the pair's lanes split the node's 9 words: lane s loads q = 2 j + s
    // (both lanes of a pair are in one wave, whose waits cover both)
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const int q = 2 * j + s;
      if (q < 9) dma_to_lds<4>(aux + (size_t)q * N + n, &st.aux[j][ty][0]);
    }
  }
}

template <class S, int TY, class R>
__device__ inline void stage_read_h(const Stage3<S, TY>& st, int k, int ty, int tx, R, R* h) {
  const float4 a = st.h4[ty][k][tx];
  h[0] = a.x; h[1] = a.y; h[2] = a.z; h[3] = a.w;
  h[4] = st.h2[0][ty][k][tx];
  h[5] = st.h2[1][ty][k][tx];
}

template <class S, int TY, class R>
__device__ inline R stage_read_f0(const Stage3<S, TY>& st, uint32_t, int ty, int tx, R) {
  return st.f0[ty][tx];
}

// Anchored 16-bit storage: the anchors of six consecutive planes of the
// tile and a two-node ring in x and y (planes z - 2 .. z + 3 while plane z
// collides: the h pulls of plane z reach z - 1 .. z + 1, the look-ahead f
// pulls of plane z + 2 reach z + 1 .. z + 3 and, from the ring nodes, two
// nodes beyond the tile), loaded by LDS-DMA one plane ahead.  Every pulled
// value takes its writer's reference from here.
template <bool ANCH, int TY> struct AnchorStage {};
template <int TY> struct AnchorStage<true, TY> {
  static constexpr int AX = 32 + 4, AY = TY + 4, NA = AX * AY;
  float4 pu[6][NA];  // p, u
  float4 e4[6][NA];  // E_xx, E_yy, E_zz, E_xy
  float e5[6][NA];   // E_xz
  float e6[6][NA];   // E_yz
};

// Tiles are walked by full tiles (FULL: every lane owns a lattice node, so
// no load or store is lane-conditional) and ragged tiles (the rest) in two
// launches of the same code; a block whose tile is of the other kind returns.
// FP64 state and the anchored 16-bit step do not fit 256 VGPRs: they run one
// wave per SIMD, which opens the accumulation registers to the allocator
// instead of scratch memory.
// DIV: the stress-divergence scheme (the force of every node includes
// div tau_p of its plane, read from a.F.div; no f^B).
// AA: in-place streaming (FP32, FP64): one population buffer (a.pin == a.pout),
// the pair index maps of aa_pair_src / aa_pair_dst by the parity of t, and
// the same-time velocity of every node from the velocity pass, U [3][N]
// (neighbours' slots are overwritten during the step, so the ring cannot
// pull them); a lane's own f is loaded one plane ahead.
template <class S, int TY, int ZC, bool WALLS, bool FULL, bool DIV = false, bool AA = false>
__global__ void __launch_bounds__(64 * TY, (sizeof(S) == 8 || StoreT<S>::kAnchored) ? 1 : 2)
    step3d_kernel(StepArgs<S> a, int ntx, int nty,
                  const typename StoreT<S>::R* __restrict__ U) {
  using R = typename StoreT<S>::R;
  using PA = Pair3<S>;
  using L = Lat<3>;
  constexpr bool kDma = std::is_same<S, float>::value;
  constexpr bool ANCH = StoreT<S>::kAnchored;
  constexpr bool kF64 = std::is_same<S, double>::value;
  static_assert(!AA || !ANCH, "in-place z-march: FP32 or FP64 storage");
  constexpr int NP = 10, NC = 6, TXN = 32, SX = TXN + 2, SY = TY + 2, NS = SX * SY;
  // ring nodes: the rows above and below the tile and the columns left and
  // right of it, without the four corners (the gradient's stencil reads the
  // axis neighbours only)
  constexpr int H = 2 * TXN + 2 * TY;
  static_assert(2 * H <= 64 * TY, "ring needs more lanes than the workgroup has");
  // velocity planes z - 1 .. z + 1; a fourth slot (when LDS allows: not
  // with the anchor stage) takes plane z + 2 while other waves may still
  // read plane z - 2, so that no barrier has to close a plane
  constexpr int NRS = ANCH ? 3 : 4;
  __shared__ R ring[NRS][3][NS];
  __shared__ Stage3<S, TY> st;
  __shared__ AnchorStage<ANCH, TY> as;

  const Geo g = a.g;
  const S* __restrict__ pin = a.pin;
  S* __restrict__ pout = a.pout;
  R* __restrict__ aux = a.aux;
  const size_t N = g.N;
  const uint32_t N32 = (uint32_t)N;  // N <= 2^27 (2^26 in FP64), checked on the host
  const int aa = g.aa;               // in place: 1 at even t, 2 at odd t

  // Blocks are dealt to the eight XCDs in turn (block b to XCD b mod 8);
  // renumbering gives each XCD one contiguous run of tiles, so tiles that
  // share halo lines run side by side under the same L2.
  int b = blockIdx.x;
  {
    const int G = gridDim.x, q = G >> 3, r = G & 7, xcd = b & 7, j = b >> 3;
    b = (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + j;
  }
  const int tx_tile = b % ntx, rest = b / ntx;
  const int ty_tile = rest % nty, zc = rest / nty;
  const int x0 = tx_tile * TXN, y0 = ty_tile * TY;
  if ((x0 + TXN <= g.nx && y0 + TY <= g.ny) != FULL) return;
  const int zs = zc * ZC, ze = min(zs + ZC, g.nz);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * 64 + tx;
  const int s = tx & 1;
  const R sg = s ? (R)-1 : (R)1;
  const int x = x0 + (tx >> 1), y = y0 + ty;
  const bool in_xy = FULL || (x < g.nx && y < g.ny);
  const int oslot = (ty + 1) * SX + (tx >> 1) + 1;
  auto clampc = [](int c, int n) { return c < 0 ? 0 : (c >= n ? n - 1 : c); };

  // Own column: wrapped for lanes past a ragged edge (they supply the
  // slot's velocity for the true last node's gradient), clamped where the
  // wrap would cross a wall (values unused).  Ring node for the first 2H
  // lanes; other lanes shadow their own column.
  int wx = x, wy = y;
  const bool vxy = wrap_coord(wx, g.nx, g.walls & 1) && wrap_coord(wy, g.ny, g.walls & 2);
  const int ox = clampc(wx, g.nx), oy = clampc(wy, g.ny);
  bool hxy = false;
  int hx = ox, hy = oy, hslot = 0;
  // positions in the anchor stage (two-node ring): own column, ring node
  const int alx = (tx >> 1) + 2, aly = ty + 2;
  int hlx = alx, hly = aly;
  if (tid < 2 * H) {
    const int r = tid >> 1;
    int sxl, syl;
    if (r < TXN) { sxl = 1 + r; syl = 0; }
    else if (r < 2 * TXN) { sxl = 1 + r - TXN; syl = SY - 1; }
    else if (r < 2 * TXN + TY) { sxl = 0; syl = 1 + r - 2 * TXN; }
    else { sxl = SX - 1; syl = 1 + r - 2 * TXN - TY; }
    hslot = syl * SX + sxl;
    hlx = sxl + 1;
    hly = syl + 1;
    hx = x0 - 1 + sxl;
    hy = y0 - 1 + syl;
    hxy = wrap_coord(hx, g.nx, g.walls & 1) && wrap_coord(hy, g.ny, g.walls & 2);
    hx = clampc(hx, g.nx);
    hy = clampc(hy, g.ny);
  }
  // body force of the own column and the ring node, without div tau_p (the
  // force fields are independent of z)
  R Fown[3] = {0, 0, 0}, Fring[3] = {0, 0, 0};
  {
    ForceArgs<R> fb = a.F;
    fb.div = nullptr;
    force_at<R>(fb, ox, oy, 0, g, Fown);
    force_at<R>(fb, hx, hy, 0, g, Fring);
  }

  // plane index for loads: wrapped, clamped beyond a wall (values unused)
  auto load_z = [&](int zp) {
    int zw = zp;
    wrap_coord(zw, g.nz, g.walls & 4);
    return clampc(zw, g.nz);
  };
  auto plane_ok = [&](int zp) {
    int zw = zp;
    return wrap_coord(zw, g.nz, g.walls & 4);
  };
  // the force at column (cx, cy) of plane zp: Fb, plus div tau_p there in
  // the stress-divergence scheme (added as force_at adds it)
  auto force_z = [&](int cx, int cy, int zp, const R* Fb, R* F) {
    F[0] = Fb[0];
    F[1] = Fb[1];
    F[2] = Fb[2];
    if constexpr (DIV) {
      const size_t nd = node_of(cx, cy, load_z(zp), g);
      F[0] += a.F.div[nd];
      F[1] += a.F.div[N + nd];
      F[2] += a.F.div[2 * N + nd];
    }
  };
  // anchored storage: the anchors of plane zp (tile and two-node ring) into
  // its stage slot by LDS-DMA; a lane's slot index follows its lane number,
  // so each wave fills one contiguous run of slots
  auto anc_slot = [](int zp) { return ((zp % 6) + 6) % 6; };
  auto anc_issue = [&](int zp) {
    if constexpr (ANCH) {
      using AS = AnchorStage<true, TY>;
      const int sl = anc_slot(zp), zw = load_z(zp);
      const char* base = reinterpret_cast<const char*>(pin) + Anchor3::offset(N);
#pragma unroll
      for (int r = 0; r * 64 * TY < AS::NA; ++r) {
        const int k0 = r * 64 * TY + ty * 64, k = k0 + tx;
        if (k < AS::NA) {
          int cx = x0 - 2 + k % AS::AX, cy = y0 - 2 + k / AS::AX;
          wrap_coord(cx, g.nx, g.walls & 1);
          wrap_coord(cy, g.ny, g.walls & 2);
          const size_t nd = node_of(clampc(cx, g.nx), clampc(cy, g.ny), zw, g);
          dma_to_lds<16>(base + 16 * nd, &as.pu[sl][k0]);
          dma_to_lds<16>(base + Anchor3::off1(N) + 16 * nd, &as.e4[sl][k0]);
          dma_to_lds<4>(base + Anchor3::off2(N) + 8 * nd, &as.e5[sl][k0]);
          dma_to_lds<4>(base + Anchor3::off2(N) + 8 * nd + 4, &as.e6[sl][k0]);
        }
      }
    }
  };
  // sign of the stored member named by a pulled offset (1: direction
  // 2K - 1, -1: direction 2K); without walls it is the lane's own member
  auto member_sign = [&](uint32_t o) {
    if constexpr (WALLS) return o >= N32 ? (R)-1 : (R)1;
    else return sg;
  };
  // stage index of the writer of this lane's member of pair K, for a node at
  // stage position (lx, ly) in plane zp: the node itself after a bounce-back
  // (the pulled offset names the other member), else the node at -c
  auto anc_at = [&](auto kc, uint32_t o, int lx, int ly, int zp, int& sl) {
    constexpr int K = decltype(kc)::value, i = 2 * K - 1;
    const bool bounce = WALLS && ((o >= N32) != (s != 0));
    const int cx = s ? -L::cx(i) : L::cx(i), cy = s ? -L::cy(i) : L::cy(i),
              cz = s ? -L::cz(i) : L::cz(i);
    sl = anc_slot(bounce ? zp : zp - cz);
    return bounce ? ly * (TXN + 4) + lx : (ly - cy) * (TXN + 4) + lx - cx;
  };
  // moving f of plane zp streamed into the own column (fo) and the ring
  // node (fr), for every lane
  auto pull_plane = [&](int zp, R* fo, R* fr) {
    const int zw = load_z(zp);
    PairPull pp;
    make_pair_pull(ox, oy, zw, s, g, pp);
    for_pairs<1>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const uint32_t o = pair_src<k, WALLS>(pp, s, N32);
      if constexpr (ANCH) {  // deviation + the reference of the writer (member o / N)
        int sl;
        const int ks = anc_at(kc, o, alx, aly, zp, sl);
        const float4 q = as.pu[sl][ks];
        const R uw[3] = {(R)q.y, (R)q.z, (R)q.w};
        fo[k] = fmar((R)PA::load_f_raw(pin, k, o, N), a.inv_sf,
                     fref3_pair<k, R>(member_sign(o), (R)q.x, uw));
      } else {
        fo[k] = PA::load_f(pin, k, o, N, a.inv_sf);
      }
    });
    make_pair_pull(hx, hy, zw, s, g, pp);
    for_pairs<1>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const uint32_t o = pair_src<k, WALLS>(pp, s, N32);
      if constexpr (ANCH) {
        int sl;
        const int ks = anc_at(kc, o, hlx, hly, zp, sl);
        const float4 q = as.pu[sl][ks];
        const R uw[3] = {(R)q.y, (R)q.z, (R)q.w};
        fr[k] = fmar((R)PA::load_f_raw(pin, k, o, N), a.inv_sf,
                     fref3_pair<k, R>(member_sign(o), (R)q.x, uw));
      } else {
        fr[k] = PA::load_f(pin, k, o, N, a.inv_sf);
      }
    });
  };
  // u = sum c f + F/2: each lane sums its members, the pair adds the halves
  auto pair_velocity = [&](const R* f, const R* F, R* u) {
    R m[3] = {0, 0, 0};
    for_pairs<1>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      constexpr int i = 2 * k - 1;
      constexpr int c[3] = {L::cx(i), L::cy(i), L::cz(i)};
#pragma unroll
      for (int bb = 0; bb < 3; ++bb)
        if (c[bb] != 0) m[bb] += (R)c[bb] * f[k];
    });
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) u[bb] = pair_sum(sg * m[bb]) + (R)0.5 * F[bb];
  };
  auto ring_slot = [](int zp) { return ((zp % NRS) + NRS) % NRS; };
  // velocity of plane zp from its pulled f into the ring slots
  // (the sums run for every lane, so that the loaded f are consumed on every
  // path; only the ring writes are conditional)
  auto publish_u = [&](int zp, const R* fo, const R* fr) {
    const bool ok = plane_ok(zp);
    const int rs = ring_slot(zp);
    R u[3], v[3], Fo[3], Fr[3];
    force_z(ox, oy, zp, Fown, Fo);
    force_z(hx, hy, zp, Fring, Fr);
    pair_velocity(fo, Fo, u);
    pair_velocity(fr, Fr, v);
    if (ok && vxy && s == 0) {
      ring[rs][0][oslot] = u[0];
      ring[rs][1][oslot] = u[1];
      ring[rs][2][oslot] = u[2];
    }
    if (ok && hxy && s == 0) {
      ring[rs][0][hslot] = v[0];
      ring[rs][1][hslot] = v[1];
      ring[rs][2][hslot] = v[2];
    }
  };

  // in place: u of plane zp (own column and ring node) from the velocity
  // pass, and the own f of plane zp
  auto publish_aa = [&](int zp) {
    const bool ok = plane_ok(zp);
    const int rs = ring_slot(zp), zw = load_z(zp);
    if (ok && vxy && s == 0) {
      const size_t nd = node_of(ox, oy, zw, g);
#pragma unroll
      for (int bb = 0; bb < 3; ++bb) ring[rs][bb][oslot] = U[(size_t)bb * N + nd];
    }
    if (ok && hxy && s == 0) {
      const size_t nd = node_of(hx, hy, zw, g);
#pragma unroll
      for (int bb = 0; bb < 3; ++bb) ring[rs][bb][hslot] = U[(size_t)bb * N + nd];
    }
  };
  auto pull_aa = [&](int zp, R* fo) {
    PairPull pp;
    make_pair_pull(ox, oy, load_z(zp), s, g, pp);
    for_pairs<1>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      fo[k] = PA::load_f(pin, k, aa_pair_src<k, WALLS>(pp, s, aa, N32), N, a.inv_sf);
    });
  };

  // Software pipeline over the planes of the chunk.  Per plane z: publish
  // u(z + 1) from the f pulled one plane ago; read the staged h, rest f and
  // source state of z (landed during the previous plane); start the LDS-DMA
  // loads of plane z + 1 and the register loads of the moving f of plane
  // z + 2; collide and store z.  The loads are waited for after the
  // collision, before the stores (a whole collision after their issue);
  // nothing waits for the stores inside the loop (the memory counter that
  // covers loads covers stores as well, so a wait placed after them would
  // hold every plane for its write latency).  The own moving f of z and
  // z + 1 ride in registers.  FP64 (no LDS stage: it would not fit)
  // loads plane z straight to registers instead; anchored 16-bit storage
  // loads the raw tuples of plane z + 1 into registers during plane z.
  // (the stage of the first plane is requested before the pulls that start
  // the velocity ring, whose waits then cover it as well)
  if constexpr (kDma) {
    PairPull pq;
    make_pair_pull(ox, oy, zs, s, g, pq);
    stage_issue<S, TY, WALLS, AA>(st, pin, aux, pq, s, N, a.first != 0, ty, aa);
  }
  if constexpr (ANCH) {  // anchors of planes zs - 2 .. zs + 3
    for (int zp = zs - 2; zp <= zs + 3; ++zp) anc_issue(zp);
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
    lds_barrier();
  }
  // Anchored 16-bit storage: the h tuples, rest f and previous-step source
  // state of plane z + 1 are loaded into registers during plane z, as the
  // raw 16-bit values, and rebuilt against their writers' anchors when
  // plane z + 1 collides: their latency hides behind a collision, as the
  // LDS stage hides it for FP32.
  typename PA::v4 rh4[ANCH ? NP : 1];
  typename PA::v2 rh2[ANCH ? NP : 1];
  typename PA::V rf0 = {};
  R raux[ANCH ? 9 : 1];
  auto issue_raw = [&](int zp) {
    if constexpr (ANCH) {
      PairPull pq;
      make_pair_pull(ox, oy, zp, s, g, pq);
      rf0 = PA::load_f_raw(pin, 0, pq.self, N);
      PA::load_h_raw(pin, 0, pq.self, N, rh4[0], rh2[0]);
      for_pairs<1>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        PA::load_h_raw(pin, k, pair_src<k, WALLS>(pq, s, N32), N, rh4[k], rh2[k]);
      });
      if (!a.first) {
#pragma unroll
        for (int q = 0; q < 9; ++q) raux[q] = aux[(size_t)q * N + pq.self];
      }
    }
  };
  if constexpr (ANCH) issue_raw(zs);
  R fz[NP], fn[NP], frn[NP];
  if constexpr (AA) {
    publish_aa(zs - 1);
    publish_aa(zs);
    pull_aa(zs, fz);
  } else {
    {
      R fa[NP];
      pull_plane(zs - 1, fa, frn);
      publish_u(zs - 1, fa, frn);
      pull_plane(zs, fz, frn);
      publish_u(zs, fz, frn);
    }
    pull_plane(zs + 1, fn, frn);
  }
  // the first plane's stage (LDS-DMA loads need not retire in order with
  // other memory operations)
  if constexpr (kDma) __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
  // anchored: the pulls above have read the anchor slot of plane zs - 2
  if constexpr (ANCH) lds_barrier();

#pragma unroll 1
  for (int z = zs; z < ze; ++z) {
    // raised priority while this wave issues the next planes' loads, so that
    // they are not held behind the other resident wave's collision
    // (measured on MI355X, 512^3: FP32 29.60 -> 28.63 ms, FP16 42.93 ->
    // 42.65 ms; FP64, at one wave per SIMD, 7.69 -> 8.01 ms, so not there)
    if constexpr (!kF64) __builtin_amdgcn_s_setprio(2);
    if constexpr (AA)
      publish_aa(z + 1);
    else
      publish_u(z + 1, fn, frn);
    PairPull pl;
    make_pair_pull(ox, oy, z, s, g, pl);
    const uint32_t n = pl.self;
    R f[NP], h[NC][NP];
    R chip[NC] = {0, 0, 0, 0, 0, 0}, up[3] = {0, 0, 0};
    if constexpr (kDma) {
      {
        R h0[NC];
        stage_read_h<S, TY>(st, 0, ty, tx, a.inv_sh, h0);
#pragma unroll
        for (int c = 0; c < NC; ++c) h[c][0] = s ? (R)0 : h0[c];
      }
      for_pairs<1>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        R hv[NC];
        stage_read_h<S, TY>(st, k, ty, tx, a.inv_sh, hv);
#pragma unroll
        for (int c = 0; c < NC; ++c) h[c][k] = hv[c];
      });
      if (!a.first) {
#pragma unroll
        for (int c = 0; c < NC; ++c) chip[c] = st.aux[c >> 1][ty][(tx & ~1) | (c & 1)];
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
          up[bb] = st.aux[(NC + bb) >> 1][ty][(tx & ~1) | ((NC + bb) & 1)];
      }
      f[0] = s ? (R)0 : stage_read_f0<S, TY>(st, n, ty, tx, a.inv_sf);
      // every stage slot of this lane has been read before it is refilled
      __builtin_amdgcn_s_waitcnt(waitcnt_lgkm(0));
      if (z + 1 < ze) {
        PairPull pq;
        make_pair_pull(ox, oy, z + 1, s, g, pq);
        stage_issue<S, TY, WALLS, AA>(st, pin, aux, pq, s, N, a.first != 0, ty, aa);
      }
    } else if constexpr (ANCH) {  // plane z from the registers loaded a plane ago
      {  // the rest population's writer is the node itself
        const int sl = anc_slot(z), ks = aly * (TXN + 4) + alx;
        const float4 q = as.pu[sl][ks], e = as.e4[sl][ks];
        const R uw[3] = {(R)q.y, (R)q.z, (R)q.w};
        const R Ew[6] = {(R)e.x, (R)e.y, (R)e.z, (R)e.w, (R)as.e5[sl][ks], (R)as.e6[sl][ks]};
        const R hr[NC] = {(R)rh4[0].x, (R)rh4[0].y, (R)rh4[0].z,
                          (R)rh4[0].w, (R)rh2[0].x, (R)rh2[0].y};
        const R f0 = fmar((R)rf0, a.inv_sf, fref3_rest<R>((R)q.x, uu3(uw)));
        f[0] = s ? (R)0 : f0;
#pragma unroll
        for (int c = 0; c < NC; ++c)
          h[c][0] = s ? (R)0 : fmar(hr[c], a.inv_sh, href3_rest<R>(Ew[c]));
      }
      for_pairs<1>([&](auto kc) {  // deviation + the reference of the writer (member o / N)
        constexpr int k = decltype(kc)::value;
        const uint32_t o = pair_src<k, WALLS>(pl, s, N32);
        int sl;
        const int ks = anc_at(kc, o, alx, aly, z, sl);
        const float4 q = as.pu[sl][ks], e = as.e4[sl][ks];
        const R uw[3] = {(R)q.y, (R)q.z, (R)q.w};
        const R Ew[6] = {(R)e.x, (R)e.y, (R)e.z, (R)e.w, (R)as.e5[sl][ks], (R)as.e6[sl][ks]};
        const R hr[NC] = {(R)rh4[k].x, (R)rh4[k].y, (R)rh4[k].z,
                          (R)rh4[k].w, (R)rh2[k].x, (R)rh2[k].y};
        const R cw = cu_pair3<k, R>(member_sign(o), uw);
#pragma unroll
        for (int c = 0; c < NC; ++c) h[c][k] = fmar(hr[c], a.inv_sh, href3_cu<k, R>(cw, c, Ew[c]));
      });
      if (!a.first) {
#pragma unroll
        for (int c = 0; c < NC; ++c) chip[c] = raux[c];
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) up[bb] = raux[NC + bb];
      }
      if (z + 1 < ze) issue_raw(z + 1);
    } else {  // FP64: plane z straight to registers
      R h0[NC];
      const R f0 = PA::load_f(pin, 0, n, N, a.inv_sf);
      PA::load_h(pin, 0, n, N, a.inv_sh, h0);
      f[0] = s ? (R)0 : f0;
#pragma unroll
      for (int c = 0; c < NC; ++c) h[c][0] = s ? (R)0 : h0[c];
      for_pairs<1>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        R hv[NC];
        const uint32_t o = AA ? aa_pair_src<k, WALLS>(pl, s, aa, N32) : pair_src<k, WALLS>(pl, s, N32);
        PA::load_h(pin, k, o, N, a.inv_sh, hv);
#pragma unroll
        for (int c = 0; c < NC; ++c) h[c][k] = hv[c];
      });
      if (!a.first) Aux<3, R>::load(aux, n, N, chip, up);
    }
    if constexpr (AA) {
#pragma unroll
      for (int k = 1; k < NP; ++k) f[k] = fz[k];
      if (z + 1 < ze) pull_aa(z + 1, fz);
    } else {
#pragma unroll
      for (int k = 1; k < NP; ++k) {
        f[k] = fz[k];
        fz[k] = fn[k];
      }
      pull_plane(z + 2, fn, frn);
    }
    // anchored: the pulls of this plane have read the anchor stage for the
    // last time (planes z - 1 .. z + 3); the slot of plane z - 2 takes plane
    // z + 4, which lands before this plane's stores and is read after the
    // barrier that closes the plane.  (Issued after the reads, so the
    // compiler need not wait for the transfer before them.)
    if constexpr (ANCH) {
      if (z + 1 < ze) anc_issue(z + 4);
    }
    if constexpr (!kF64) __builtin_amdgcn_s_setprio(0);
    lds_barrier();  // u(z + 1) published

    {
      // the collision may fuse multiply-adds (this node's own arithmetic
      // only; velocities shared through LDS are formed without contraction)
#pragma clang fp contract(fast)
      const int rc = ring_slot(z), rm = ring_slot(z - 1), rp = ring_slot(z + 1);
      const R u[3] = {ring[rc][0][oslot], ring[rc][1][oslot], ring[rc][2][oslot]};
      R F[3];
      force_z(ox, oy, z, Fown, F);
      // moments of the pulled state
      R e[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        R sm = 0;
#pragma unroll
        for (int k = 0; k < NP; ++k) sm += h[c][k];
        e[c] = pair_sum(sm);
      }
      R sum_f = 0;
#pragma unroll
      for (int k = 1; k < NP; ++k) sum_f += f[k];
      sum_f = pair_sum(sum_f);
      R tau[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) tau[c] = a.P.eta_over_lam * e[c];
      R fB[L::Q];
      if constexpr (DIV) {
#pragma unroll
        for (int i = 0; i < L::Q; ++i) fB[i] = 0;
      } else {
        fluct_term<R>(tau, a.P.inv_tau_f, fB, (L*)nullptr);
      }
      const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
      const R Fu = F[0] * u[0] + F[1] * u[1] + F[2] * u[2];
      constexpr R w0 = (R)L::w(0);
      const R F0 = -3 * w0 * a.P.k_f * Fu;
      // pressure (App. B): cs2/(1 - w0) = 1/2 for D3Q19
      const R p = (R)0.5 * (sum_f - (R)1.5 * w0 * uu + a.P.tau_f * F0 + a.P.tau_f * fB[0]);

      // ---- f collision: BGK + Guo forcing + f^B (Sec. 2.2), per direction
      //   f* = (1 - w_f) f + w_f f^eq + f^B_i + F_i, written as
      //   (1 - w_f) f + a0 + f^B_i + a1 cu (3 + 9/2 cu) + a2 cF (1 + 3 cu)
      // with the weight-class constants a0 = w (w_f (3 p - 3/2 u.u) - 3 k_f F.u),
      // a1 = w w_f, a2 = 3 w k_f (w_f = 1/tau_f; the same sum, reordered).
      // Both lanes of the pair carry the rest f and update it alike.
      const R omf = a.P.inv_tau_f, keepf = (R)1 - omf;
      {
        const R feq = (R)(3.0 * (L::w(0) - 1.0)) * p - w0 * (R)1.5 * uu;
        f[0] = f[0] - (f[0] - feq) * omf + fB[0] + F0;
      }
      R a0[2], a1[2], a2[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const R w = q == 0 ? (R)(1.0 / 18.0) : (R)(1.0 / 36.0);
        a0[q] = w * (omf * (3 * p - (R)1.5 * uu) - 3 * a.P.k_f * Fu);
        a1[q] = w * omf;
        a2[q] = 3 * w * a.P.k_f;
      }
      R cu[NP], cup[NP];
      R mp[3] = {0, 0, 0};
      for_pairs<1>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int i = 2 * k - 1;
        constexpr int c[3] = {L::cx(i), L::cy(i), L::cz(i)};
        constexpr int q = k <= 3 ? 0 : 1;
        cu[k] = sg * ((R)c[0] * u[0] + (R)c[1] * u[1] + (R)c[2] * u[2]);
        cup[k] = sg * ((R)c[0] * up[0] + (R)c[1] * up[1] + (R)c[2] * up[2]);
        const R cF = sg * ((R)c[0] * F[0] + (R)c[1] * F[1] + (R)c[2] * F[2]);
        f[k] = keepf * f[k] + a0[q] + fB[i] + a1[q] * cu[k] * (3 + (R)4.5 * cu[k]) +
               a2[q] * cF * (1 + 3 * cu[k]);
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
          if (c[bb] != 0) mp[bb] += (R)c[bb] * f[k];
      });
      // The update's momentum identity sum c f* = u + F/2 is restored on the
      // axis pairs (k = 1, 2, 3): rounded weights would otherwise bias every
      // step; mass and second moments are unchanged by it.
#pragma unroll
      for (int bb = 0; bb < 3; ++bb) {
        const R m = pair_sum(sg * mp[bb]);
        const R half = (R)0.5 * ((u[bb] + (R)0.5 * F[bb]) - m);
        f[1 + bb] += sg * half;
      }

      // ---- same-time gradient G[a][b] = d_a u_b (central; one-sided at walls)
      R G[3][3];
#pragma unroll
      for (int bb = 0; bb < 3; ++bb) {
        const R* uc = &ring[rc][bb][oslot];
        const R nb[3][2] = {{uc[-1], uc[1]}, {uc[-SX], uc[SX]},
                            {ring[rm][bb][oslot], ring[rp][bb][oslot]}};
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          G[ax][bb] = pl.lo[ax] ? u[bb] + nb[ax][1] * (R)(1.0 / 3.0)
                    : pl.hi[ax] ? -(u[bb] + nb[ax][0] * (R)(1.0 / 3.0))
                                : (R)0.5 * (nb[ax][1] - nb[ax][0]);
        }
      }
      R chi[NC];
      source_tensor<3, R>(e, G, a.P, chi);

      // ---- h collision (Sec. 2.3); the rest population closes
      // sum_i h*_i = A - I + chi + (chi - chi(t-1))/2.  Per direction
      //   h* = (1 - w_h) h + w_h h^eq + chi_i + (chi_i - chi_i(t-1))/2
      //      = (1 - w_h) h + k0 + k1 cu - k2 cu(t-1)
      // with per component and weight class k0 = w (w_h e + s chi - r chi_p),
      // k1 = w (3 w_h A + s k chi), k2 = w r k chi_p, k = 3 (1 - 1/(2 tau_h)),
      // s = 3/2, r = 1/2 (s = 1, r = 0 at the first step)
      const bool first = a.first != 0;
      const R omh = a.P.inv_tau_h, keeph = (R)1 - omh;
      const R sc = first ? (R)1 : (R)1.5, rc2 = first ? (R)0 : (R)0.5;
      R En[NC];  // sum_i h*_i: the new anchor of anchored storage
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const R Ac = e[c] + (c < 3 ? (R)1 : (R)0);
        const R target = e[c] + chi[c] + (first ? (R)0 : (R)0.5 * (chi[c] - chip[c]));
        En[c] = target;
        R k0[2], k1[2], k2[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const R w = q == 0 ? (R)(1.0 / 18.0) : (R)(1.0 / 36.0);
          k0[q] = w * (omh * e[c] + sc * chi[c] - rc2 * chip[c]);
          k1[q] = w * (3 * omh * Ac + sc * a.P.k_h3 * chi[c]);
          k2[q] = w * rc2 * a.P.k_h3 * chip[c];
        }
        R hs = 0;
        for_pairs<1>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          constexpr int q = k <= 3 ? 0 : 1;
          h[c][k] = keeph * h[c][k] + k0[q] + k1[q] * cu[k] - k2[q] * cup[k];
          hs += h[c][k];
        });
        h[c][0] = target - pair_sum(hs);
      }

      // ---- stores (the even lane holds the rest populations); chi (6
      // planes) then u (3 planes) split over the pair.  First every load
      // issued during this plane has landed: the next plane reads the LDS
      // stages they fill (a lane its own slots of the pulled state; every
      // wave the anchor stage, after the barrier that closes the plane).
      if constexpr (kDma || ANCH) __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
      if (in_xy) {
        if constexpr (ANCH) {
          // deviations from this node's new anchor (E, p, u)
          float Ef[NC], uf[3];
#pragma unroll
          for (int c = 0; c < NC; ++c) Ef[c] = (float)En[c];
#pragma unroll
          for (int bb = 0; bb < 3; ++bb) uf[bb] = (float)u[bb];
          const float pf = (float)p;
          // scaled deviations (v - ref) sc = fma(v, sc, -(sc ref)), the
          // references scaled exactly (power-of-two scales)
          const R ur[3] = {(R)uf[0], (R)uf[1], (R)uf[2]};
          const R uur = uu3(ur), psc = (R)pf * a.sf;
          if (s == 0) {
            const R w0s = (R)L::w(0) * a.sh;
            R d[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) d[c] = fmar(h[c][0], a.sh, -(w0s * (R)Ef[c]));
            PA::store_dev(pout, 0, n, N, fmar(f[0], a.sf, -fref3_rest_scaled<R>(psc, uur, a.sf)),
                          d);
            Anchor3::store(pout, n, N, pf, uf, Ef);
          }
          for_pairs<1>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const R cr = cu_pair3<k, R>(sg, ur);
            R m, t;
            href3_cu_scaled<k, R>(cr, a.sh, m, t);
            R d[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c)
              d[c] = fmar(h[c][k], a.sh, -(c < 3 ? fmar((R)Ef[c], m, t) : (R)Ef[c] * m));
            PA::store_dev(pout, k, (s ? N32 : 0u) + n, N,
                          fmar(f[k], a.sf, -fref3_cu_scaled<k, R>(cr, psc, uur, a.sf)), d);
          });
        } else {
          if (s == 0)
            PA::store(pout, 0, n, N, a.sf, a.sh, f[0], h[0][0], h[1][0], h[2][0], h[3][0],
                      h[4][0], h[5][0]);
          if constexpr (AA) {
            for_pairs<1>([&](auto kc) {
              constexpr int k = decltype(kc)::value;
              PA::store(pout, k, aa_pair_dst<k, WALLS>(pl, s, aa, N32), N, a.sf, a.sh, f[k],
                        h[0][k], h[1][k], h[2][k], h[3][k], h[4][k], h[5][k]);
            });
          } else {
#pragma unroll
            for (int k = 1; k < NP; ++k)
              PA::store(pout, k, (s ? N32 : 0u) + n, N, a.sf, a.sh, f[k], h[0][k], h[1][k],
                        h[2][k], h[3][k], h[4][k], h[5][k]);
          }
        }
        const R item[9] = {chi[0], chi[1], chi[2], chi[3], chi[4], chi[5], u[0], u[1], u[2]};
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          const int q = 2 * j + s;
          if (q < 9) stream_store(aux + (size_t)q * N + n, item[q]);
        }
      }
    }
    // three ring slots: the slot of z - 1 is free for plane z + 2, and the
    // anchor stage refilled for the next plane is visible to every wave
    // (with four slots the barrier before the next collision suffices: a
    // wave that publishes plane z + 2 has passed it for plane z, which
    // every wave reached only after its collision of z - 1, the last
    // reader of plane z - 2)
    if constexpr (NRS == 3) lds_barrier();
  }
  // no LDS-DMA may land after the workgroup has ended
  __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
}

}  // namespace vflb
