// HIP kernels of one lattice update (gfx950).  Launchers are in lbm2p.hip.
//
// Memory layout: every field is a plane [ny][nx] (x fastest) in the context's
// precision T; populations are 9 such planes per distribution, structure of
// arrays, in the in-place "AA" streaming layout:
//   parity 0 (after an even number of steps): f*_i(x) is stored at A[opp(i)][x];
//   parity 1: f*_i(x) is stored at A[i][x + c_i], or at A[opp(i)][x] when
//             x + c_i lies beyond a wall.
// A step from parity 0 pulls f_i(x) = A[opp(i)][x - c_i] (A[i][x] beyond a
// wall: half-way bounce-back) and pushes f*_i(x) to A[i][x + c_i]; a step from
// parity 1 pulls A[i][x] and writes A[opp(i)][x].  Each thread reads and writes
// the same nine locations of each distribution, so the update is in place.
#pragma once

#include <utility>

#include "lbm2p_math.h"

namespace lbm2p {

// Tile shapes of the forward step's kernels per precision: the stencil passes
// are 64 nodes wide (one wavefront per tile row), TY rows, NT threads per
// workgroup; the collision tile's width is its own (wider tiles cut the partial
// cache lines that the shifted streaming writes leave at tile edges).  Taller
// tiles recompute fewer halo nodes but hold more LDS per workgroup.
// Compile-time tuning parameters, measured on 4096^2.
// The FD stage has a second, smaller shape (FDS) for lattices on which the
// first would give fewer than FD_MIN_TILES workgroups.  On lattices where a
// pass's own shape gives fewer than TINY_TILES workgroups, each pass is one
// workgroup's latency, which shorter tiles cut: the FD stages, the velocity
// sweeps and the filter then take 64 x TINY_TY tiles of TINY_NT threads, the
// collision its COLT shape (128^2 CH-only step 29 -> 20 us FP32; 200^2
// droplet 53 -> 34 us FP32, 77 -> 49 us FP64).
#ifndef LBM2P_F32_TILES
#define LBM2P_F32_TILES 64, 1024, 32, 1024, 32, 512, 16, 512, 128, 32, 512, 8, 512, 64
#endif
#ifndef LBM2P_F64_TILES
#define LBM2P_F64_TILES 16, 512, 8, 512, 16, 512, 16, 256, 64, 16, 512, 4, 256, 64
#endif
constexpr int FD_MIN_TILES = 512, TINY_TILES = 64, TINY_TY = 8, TINY_NT = 512;
// The velocity sweeps' shape on lattices where their own gives fewer than
// VEL_MIN_TILES workgroups (FP32: 64 x 32 tiles of 1024 threads leave CUs idle
// at 256 x 1024, where 64 x 16 tiles of 512 are 9 % faster)
constexpr int VEL_MIN_TILES = 512;
template <typename T>
struct VelSmall {
  static constexpr int TY = 16, NT = 512;
};
template <>
struct VelSmall<double> {
  static constexpr int TY = 8, NT = 512;
};
template <int FD_Y, int FD_T, int VEL_Y, int VEL_T, int FIL_Y, int FIL_T, int COL_Y, int COL_T,
          int COL_X, int FDS_Y, int FDS_T, int COLT_Y, int COLT_T, int COLT_X>
struct StepTiles {
  static constexpr int TX = 64, COL_TX = COL_X;
  static constexpr int FD_TY = FD_Y, FD_NT = FD_T, VEL_TY = VEL_Y, VEL_NT = VEL_T;
  static constexpr int FIL_TY = FIL_Y, FIL_NT = FIL_T, COL_TY = COL_Y, COL_NT = COL_T;
  static constexpr int FDS_TY = FDS_Y, FDS_NT = FDS_T;
  static constexpr int COLT_TY = COLT_Y, COLT_NT = COLT_T, COLT_TX = COLT_X;
};
template <typename T>
struct StepCfg;
template <>
struct StepCfg<float> : StepTiles<LBM2P_F32_TILES> {};
template <>
struct StepCfg<double> : StepTiles<LBM2P_F64_TILES> {};

template <typename T>
struct KParams {
  int nx, ny, wx, wy;
  long long ps;                 // plane stride (elements)
  T c4b, kappa, eta, negM, lam, eps2, W, cJ;
  T rho1, rho2, mu1, mu2, gx, gy, rho_ref;
  T p_ref;                      // g is stored as g_i - 3 w_i p_ref
  T invW;                       // 1 / W rounded once (host)
  T lam12, lamW2, negM12, eps144;  // FP32 FD stage: lambda/12, 2 lambda/W, -M/12, 144 eps^2
  T fa;                         // filter intensity
  T fd[6];                      // filter coefficients d_0..d_N
  int fn;                       // N = half width of the explicit filter
  T s_f[9], s_g[9];
  int opt;                      // LBM2P_OPT_* bits
};

// ---------------------------------------------------------------- boundaries
// Map an extended-lattice index to a node: periodic wrap, or the half-way
// mirror (node -1-i below 0, 2n-1-i above n-1) with a parity flip.  Ghosts feed
// in-domain outputs only within the deepest halo (6 nodes, less than the
// smallest lattice side 16), so one wrap or one reflection suffices; indices
// further out (windows of ragged tiles on small lattices) feed no in-domain
// output and are clamped to stay in bounds.  No integer division: this runs
// once per element of every LDS window.
__device__ __forceinline__ int map_idx(int i, int n, int wall, int& flip) {
  if (!wall) {
    i = i < 0 ? i + n : (i >= n ? i - n : i);
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
  }
  if (i < 0) {
    i = -1 - i;
    flip ^= 1;
  } else if (i >= n) {
    i = 2 * n - 1 - i;
    flip ^= 1;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Tile of this workgroup.  Workgroups are dealt round-robin to the 8 XCDs
// (XCD = blockIdx mod 8), each with its own L2; the remap gives every XCD a
// contiguous band of tiles (row-major), so halo reads and the neighbour
// writes of the in-place streaming mostly stay inside one L2.  A bijection
// of [0, gridDim.x) for any tile count.
__device__ __forceinline__ void tile_of(int tiles_x, int& tx, int& ty) {
  const int nb = (int)gridDim.x, b = (int)blockIdx.x;
  const int q = nb >> 3, r = nb & 7, k = b & 7, j = b >> 3;
  const int t = k * q + (k < r ? k : r) + j;
  ty = t / tiles_x;
  tx = t - ty * tiles_x;
}

// Visit every element (lx, ly), 0 <= lx < W, 0 <= ly < H, of a tile-local
// window: columns in 64-wide chunks with lane = column (wave w of the
// workgroup takes rows w, w + NT/64, ...), the last W % 64 columns spread over
// all threads.  Within a chunk a thread's elements are whole rows apart, so
// every LDS address is one per-thread base plus a compile-time offset and no
// element pays an integer division; a wave reads 64 consecutive elements.
template <int W, int H, int NT, typename F>
__device__ __forceinline__ void for_window(F&& fn) {
  static_assert(NT % 64 == 0, "whole wavefronts");
  constexpr int NW = NT / 64, NC = W / 64, R = W % 64;
  constexpr int KR = (H + NW - 1) / NW;
  const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int r = wv + k * NW;
      if ((k + 1) * NW <= H || r < H) fn(c * 64 + lane, r);
    }
  }
  if constexpr (R > 0) {
    constexpr int KT = (R * H + NT - 1) / NT;
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      const int j = (int)threadIdx.x + k * NT;
      if ((k + 1) * NT <= R * H || j < R * H) fn(NC * 64 + j % R, j / R);
    }
  }
}

// Element k of one field plane (k < 2^31 / 9 nodes, so k * 8 < 2^32): the
// uniform base plus a 32-bit byte offset, so that a load or store takes the
// base from scalar registers and one vector register for the offset (the
// gather's stores; elsewhere measured no faster than 64-bit addresses).
template <typename T>
__device__ __forceinline__ T& fld(T* base, long long k) {
  return *(T*)((char*)base + (unsigned)k * (unsigned)sizeof(T));
}

// Load a (RW x RH) window whose (0,0) sits at node (gx0, gy0) into LDS, in
// for_window's element order.  Each thread first issues all of its global
// loads (independent, so their latencies overlap), then writes them to LDS.
// A thread's slots beyond the window's last row load a node of that row
// instead (no branch around a load: a conditional load would make the
// compiler wait for the loads before it) and are not stored.  A window inside
// the lattice (most tiles) takes plain row addresses; only windows that cross
// an edge map each index through the wrap or mirror.  Node indices fit in 32
// bits (checked at context creation).
// Slots of a thread in a (RW x RH) window, in for_window's element order:
// slot n (compile-time after unrolling) -> element (lx, ly) and whether it is
// one of the window's (a slot beyond the last row names an element of that
// row instead, so that a load through it stays in bounds).
template <int NT, int RW, int RH>
struct WinSlots {
  static constexpr int NW = NT / 64, NC = RW / 64, R = RW % 64, RR = R > 0 ? R : 1;
  static constexpr int KR = (RH + NW - 1) / NW, KT = R > 0 ? (R * RH + NT - 1) / NT : 0;
  static constexpr int NV = NC * KR + KT;
  static_assert(NT % 64 == 0, "whole wavefronts");
  __device__ __forceinline__ static void at(int n, int& lx, int& ly, bool& in) {
    const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
    if (n < NC * KR) {
      lx = (n / KR) * 64 + lane;
      ly = wv + (n % KR) * NW;
      in = ((n % KR) + 1) * NW <= RH || ly < RH;
      ly = in ? ly : RH - 1;
    } else {
      int j = (int)threadIdx.x + (n - NC * KR) * NT;
      in = (n - NC * KR + 1) * NT <= R * RH || j < R * RH;
      j = in ? j : R * RH - 1;
      lx = NC * 64 + j % RR;
      ly = j / RR;
    }
  }
};

template <typename T, typename S, int NT, int RW, int RH>
__device__ __forceinline__ void load_window(T* dst, const S* __restrict__ src, int gx0, int gy0,
                                            const KParams<T>& P, bool odd) {
  using WS = WinSlots<NT, RW, RH>;
  constexpr int NV = WS::NV;
  auto coords = [](int n, int& lx, int& ly, bool& in) { WS::at(n, lx, ly, in); };
  T v[NV];
  if (gx0 >= 0 && gx0 + RW <= P.nx && gy0 >= 0 && gy0 + RH <= P.ny) {
    const S* __restrict__ base = src + (gy0 * P.nx + gx0);
#pragma unroll
    for (int n = 0; n < NV; ++n) {
      int lx, ly;
      bool in;
      coords(n, lx, ly, in);
      v[n] = T(base[ly * P.nx + lx]);
    }
  } else {
#pragma unroll
    for (int n = 0; n < NV; ++n) {
      int lx, ly;
      bool in;
      coords(n, lx, ly, in);
      int flip = 0;
      const int x = map_idx(gx0 + lx, P.nx, P.wx, flip);
      const int y = map_idx(gy0 + ly, P.ny, P.wy, flip);
      const T w = T(src[y * P.nx + x]);
      v[n] = (odd && flip) ? -w : w;
    }
  }
#pragma unroll
  for (int n = 0; n < NV; ++n) {
    int lx, ly;
    bool in;
    coords(n, lx, ly, in);
    if (in) dst[ly * RW + lx] = v[n];
  }
}

// Cache policy of the population loads and stores of the gather and the
// collision when the populations are larger than the last-level cache (the
// launchers pick STREAM = true then): each population is read once and
// written once per kernel, so streaming accesses keep it from displacing the
// fields the next passes read.  One bit per access kind and streaming parity:
// bit PAR for the gather's loads, 2 + PAR for the collision's loads, 4 + PAR
// for its stores.  A set bit makes the gather's loads nontemporal, and the
// collision's accesses where they are aligned (col_load9, col_store9): in
// parity 1 every node reads and writes its own slots (whole cache lines); in
// parity 0 the slots are shifted by c_i, and only the directions with c_x = 0
// (shifted by whole rows) stay aligned.  Measured on
// 4096^2: nontemporal gather loads (both parities), nontemporal collision
// loads and stores in parity 1 and the aligned parity-0 collision loads save
// 5 % of the step; hinting the shifted parity-0 accesses slows the collision
// by 5-9 %.  On lattices whose populations fit in the cache the hints cost
// 2-3 % and are off.
#ifndef LBM2P_POP_NT
#define LBM2P_POP_NT 47
#endif
template <int BIT, bool STREAM, typename T>
__device__ __forceinline__ T pop_ld(const T* p) {
  if constexpr (STREAM && ((LBM2P_POP_NT >> BIT) & 1) != 0) return __builtin_nontemporal_load(p);
  else return *p;
}
template <int BIT, bool STREAM, typename T>
__device__ __forceinline__ void pop_st(T* p, T v) {
  if constexpr (STREAM && ((LBM2P_POP_NT >> BIT) & 1) != 0) __builtin_nontemporal_store(v, p);
  else *p = v;
}
// Slot addresses of the gather: the two slots direction i can use, in planes i
// and opp(i), are addressed from plane lo(i) = min(i, opp(i)) (a uniform base)
// by an element offset rd[i] < 3 planes.  FP32 adds it as a 32-bit byte offset
// (3 planes of < 2^31 / 9 four-byte elements stay below 2^32), so a load takes
// its base from scalar registers and one vector register; FP64 adds elements.
// (The collision keeps 64-bit addresses from the distribution's base: with
// plane bases its FP64 build runs out of scalar registers and its FP32 build,
// though it needs fewer vector registers, measured 2 % slower.)
__host__ __device__ constexpr int lo_of(int i) { return i < opp(i) ? i : opp(i); }
template <int I, typename T>
__device__ __forceinline__ T* slot_ptr(T* A, long long ps, int r) {
  T* plane = A + lo_of(I) * ps;
  if constexpr (sizeof(T) == 4) return (T*)((char*)plane + (unsigned)r * 4u);
  else return plane + r;
}

// The collision's nine loads (v[i] from slot rd[i]) and stores (v[i] to slot
// rd[opp(i)]) of one distribution, each with its direction's alignment known
// at compile time.
template <int PAR, bool STREAM, typename T, int... I>
__device__ __forceinline__ void col_load9(const T* A, const int* rd, T* v,
                                          std::integer_sequence<int, I...>) {
  ((v[I] = pop_ld<2 + PAR, STREAM && (PAR == 1 || cx_of(I) == 0)>(A + rd[I])), ...);
}
template <int PAR, bool STREAM, typename T, int... I>
__device__ __forceinline__ void col_store9(T* A, const int* rd, const T* v,
                                           std::integer_sequence<int, I...>) {
  (pop_st<4 + PAR, STREAM && (PAR == 1 || cx_of(I) == 0)>(A + rd[opp(I)], v[I]), ...);
}
template <int PAR, bool STREAM, typename T, int... I>
__device__ __forceinline__ void gather_load9(const T* A, long long ps, const int* rd, T* v,
                                             std::integer_sequence<int, I...>) {
  ((v[I] = pop_ld<PAR, STREAM>(slot_ptr<I>(A, ps, rd[I]))), ...);
}

// ------------------------------------------------------------- populations
// Element offsets (from a distribution's base, or with REL from plane lo(i)
// of it, for slot_ptr) of the nine slots node (x, y) pulls f_i from.  In both parities the node writes f*_opp(i) back to
// the slot it pulled f_i from (parity 0: the slot of x - c_i, or its own slot
// i beyond a wall; parity 1: its own slot i), so one set of offsets serves the
// pull and the push of f and of g.  32-bit offsets: 9 planes < 2^31 elements
// (checked at context creation).
template <int PAR, bool REL, typename T>
__device__ __forceinline__ void slots(const KParams<T>& P, int x, int y, int rd[9]) {
  const int ps = (int)P.ps;
  const int id = y * P.nx + x;
  if (PAR == 1) {
#pragma unroll
    for (int i = 0; i < 9; ++i) rd[i] = (i - (REL ? lo_of(i) : 0)) * ps + id;
    return;
  }
  const bool lo_x = x == 0, hi_x = x == P.nx - 1, lo_y = y == 0, hi_y = y == P.ny - 1;
  const int xm = lo_x ? P.nx - 1 : x - 1, xp = hi_x ? 0 : x + 1;
  const int rm = (lo_y ? P.ny - 1 : y - 1) * P.nx, r0 = y * P.nx, rp = (hi_y ? 0 : y + 1) * P.nx;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int cx = cx_of(i), cy = cy_of(i);
    // source node x - c_i
    const int sx = cx == 1 ? xm : (cx == -1 ? xp : x);
    const int sr = cy == 1 ? rm : (cy == -1 ? rp : r0);
    const bool out = (P.wx && ((cx == 1 && lo_x) || (cx == -1 && hi_x))) ||
                     (P.wy && ((cy == 1 && lo_y) || (cy == -1 && hi_y)));
    const int b = REL ? lo_of(i) : 0;
    rd[i] = out ? (i - b) * ps + id : (opp(i) - b) * ps + sr + sx;
  }
}

// ------------------------------------------------------------ a1: gather
// phi_bar = sum f_i (eq:compute_phi), p = c_s^2 sum g_i (Eq:p), j = sum g_i c_i;
// with m7, m8 given, also the moments m_7 = g1 - g2 + g3 - g4 and
// m_8 = g5 - g6 + g7 - g8 of eq:D2Q9MRT.  COUPLED = false: phi_bar alone;
// SKIP_F: the moments of g alone (the two halves of a split gather).

// phi_bar = sum f_i of one node's nine pulled populations.  FP32: the eight
// moving populations (|f_i| << 1) summed first, f_0 ~ phi added last, so that
// the sum rounds once at phi's magnitude; FP64 in index order (the oracle's).
template <typename T>
__device__ __forceinline__ T phibar_sum(const T f[9]) {
  if constexpr (std::is_same<T, float>::value) {
    return f[0] + (((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8])));
  } else {
    T s = f[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) s = s + f[i];
    return s;
  }
}

// The gather at node (x, y), element id; SKIP_F: only the moments of g (p, j)
template <typename T, int PAR, bool COUPLED, bool STREAM, bool SKIP_F = false>
__device__ __forceinline__ void gather_node(const KParams<T>& P, const T* __restrict__ Af,
                                            const T* __restrict__ Ag, T* __restrict__ phibar,
                                            T* __restrict__ praw, T* __restrict__ jx,
                                            T* __restrict__ jy, T* __restrict__ m7,
                                            T* __restrict__ m8, T* __restrict__ m1, int x, int y,
                                            long long id) {
  int rd[9];
  slots<PAR, true>(P, x, y, rd);
  if constexpr (!SKIP_F) {
    T f[9];
    gather_load9<PAR, STREAM>(Af, P.ps, rd, f, std::make_integer_sequence<int, 9>{});
    fld(phibar, id) = phibar_sum<T>(f);
  }
  if (!COUPLED) return;
  T g[9];
  gather_load9<PAR, STREAM>(Ag, P.ps, rd, g, std::make_integer_sequence<int, 9>{});
  T sg = g[0];
#pragma unroll
  for (int i = 1; i < 9; ++i) sg = sg + g[i];
  // FP32: the correctly rounded sg / 3 (sg times the rounded 1/3 would scale p
  // by 1 + 3e-8 every step, a drift the collision carries forward)
  if constexpr (std::is_same<T, float>::value) fld(praw, id) = div3_rn(sg) + P.p_ref;
  else fld(praw, id) = divk<3>(sg) + P.p_ref;   // sum_i 3 w_i p_ref / 3 = p_ref
  T ax = g[1];
  ax = ax - g[3];
  ax = ax + g[5];
  ax = ax - g[6];
  ax = ax - g[7];
  ax = ax + g[8];
  T ay = g[2];
  ay = ay - g[4];
  ay = ay + g[5];
  ay = ay + g[6];
  ay = ay - g[7];
  ay = ay - g[8];
  fld(jx, id) = ax;
  fld(jy, id) = ay;
  if (m7) {
    fld(m7, id) = ((g[1] - g[2]) + g[3]) - g[4];
    fld(m8, id) = ((g[5] - g[6]) + g[7]) - g[8];
  }
  if (m1) {
    T a, b, c;
    moments_178<T>(g, a, b, c);
    fld(m1, id) = a;
  }
}

// NTB threads a workgroup, one node each
template <typename T, int PAR, bool COUPLED, bool STREAM, bool SKIP_F = false, int NTB = 256>
__global__ __launch_bounds__(NTB) void k_gather(KParams<T> P, const T* __restrict__ Af,
                                                const T* __restrict__ Ag, T* __restrict__ phibar,
                                                T* __restrict__ praw, T* __restrict__ jx,
                                                T* __restrict__ jy, T* __restrict__ m7,
                                                T* __restrict__ m8, T* __restrict__ m1) {
  const long long n = (long long)P.nx * P.ny;
  const long long id = (long long)blockIdx.x * NTB + threadIdx.x;
  if (id >= n) return;
  const int y = (int)(id / P.nx), x = (int)(id - (long long)y * P.nx);
  gather_node<T, PAR, COUPLED, STREAM, SKIP_F>(P, Af, Ag, phibar, praw, jx, jy, m7, m8, m1, x, y,
                                               id);
}

// ------------------------------------------------- a2: FD sub-step stage
// L(phi*) = div_4 (lambda J_phi + q)  (eq:final_mCHE, eq:fourOrder_FDM) and the
// TVD-RK3 combination of eq:TVD-3order for STAGE 1, 2, 3.
// Outputs of the gather when it is folded into the first FD stage
template <typename T>
struct FoldedGather {
  const T* Af;
  const T* Ag;   // null in CH-only mode
  T *phibar, *praw, *jx, *jy;
};

// GPAR >= 0 (stage 1): the step's gather of phi_bar folded in, phi_bar of
// every window node summed from its populations (parity GPAR; k_gather's
// arithmetic) instead of read from `in` and written for the tile's nodes to
// G.phibar, where the later stages and the state read it; with COUPLED the
// tile's p and j too (small lattices; large ones gather those on a second
// stream).
template <typename T, int STAGE, int TX, int TY, int NT, int GPAR = -1, bool COUPLED = false>
__global__ __launch_bounds__(NT) void k_fd(KParams<T> P, int tiles_x, const T* __restrict__ in,
                                            const T* __restrict__ phibar, T* __restrict__ out,
                                            FoldedGather<T> G = {}) {
  static_assert(GPAR < 0 || STAGE == 1, "the gather folds into the first stage");
  constexpr int W5 = TX + 10, H5 = TY + 10;   // phi*, halo 5
  constexpr int W4 = TX + 8, H4 = TY + 8;     // mu*, halo 4
  constexpr int W2 = TX + 4, H2 = TY + 4;     // J_d, halo 2
  __shared__ T sP[W5 * H5];
  __shared__ T sM[W4 * H4];
  __shared__ T sJx[W2 * H2];
  __shared__ T sJy[W2 * H2];
  int bx, by;
  tile_of(tiles_x, bx, by);
  const int x0 = bx * TX, y0 = by * TY;
  if constexpr (GPAR >= 0) {
    for_window<W5, H5, NT>([&](int ix, int iy) {
      int flip = 0;
      const int x = map_idx(x0 - 5 + ix, P.nx, P.wx, flip);
      const int y = map_idx(y0 - 5 + iy, P.ny, P.wy, flip);
      int rd[9];
      slots<GPAR, true>(P, x, y, rd);
      T f[9];
      gather_load9<GPAR, false>(G.Af, P.ps, rd, f, std::make_integer_sequence<int, 9>{});
      sP[iy * W5 + ix] = phibar_sum<T>(f);
    });
  } else {
    load_window<T, T, NT, W5, H5>(sP, in, x0 - 5, y0 - 5, P, false);
  }
  __syncthreads();
  const Tile<T> tP{sP, W5, 5}, tM{sM, W4, 4}, tJx{sJx, W2, 2}, tJy{sJy, W2, 2};
  if constexpr (GPAR >= 0) {
    // the tile's phi_bar from the window; p and j (COUPLED) from the tile's g
    for_window<TX, TY, NT>([&](int lx, int ly) {
      const int x = x0 + lx, y = y0 + ly;
      if (x < P.nx && y < P.ny) {
        const long long id = (long long)y * P.nx + x;
        fld(G.phibar, id) = tP(lx, ly);
        if constexpr (COUPLED)
          gather_node<T, GPAR, true, false, true>(P, G.Af, G.Ag, G.phibar, G.praw, G.jx, G.jy,
                                                  nullptr, nullptr, nullptr, x, y, id);
      }
    });
  }
  for_window<W4, H4, NT>([&](int ix, int iy) {
    sM[iy * W4 + ix] = chem_pot<T>(tP, ix - 4, iy - 4, P.c4b, P.kappa);
  });
  __syncthreads();
  for_window<W2, H2, NT>([&](int ix, int iy) {
    const int lx = ix - 2, ly = iy - 2, idx = iy * W2 + ix;
    const T ph = tP(lx, ly);
    if constexpr (std::is_same<T, float>::value) {
      // FP32: J_d = lambda J_phi + q = [lambda (|G| - c_W) - M (grad mu . G)/|G|] G/|G|
      // from the unscaled differences G' = 12 G, M' = 12 grad mu:
      // J_d = [lambda/12 |G'|_e - lambda c_W - (M/12) (M'.G') / |G'|_e] G' / |G'|_e with
      // |G'|_e = sqrt(|G'|^2 + 144 eps^2) = 12 |G|_eps, the 1/12 in the constants;
      // one reciprocal and the hardware square root
      const T Gx = d4u<T>(tP(lx - 2, ly), tP(lx - 1, ly), tP(lx + 1, ly), tP(lx + 2, ly));
      const T Gy = d4u<T>(tP(lx, ly - 2), tP(lx, ly - 1), tP(lx, ly + 1), tP(lx, ly + 2));
      const T Mx = d4u<T>(tM(lx - 2, ly), tM(lx - 1, ly), tM(lx + 1, ly), tM(lx + 2, ly));
      const T My = d4u<T>(tM(lx, ly - 2), tM(lx, ly - 1), tM(lx, ly + 1), tM(lx, ly + 2));
      const T mag = __builtin_amdgcn_sqrtf((Gx * Gx + Gy * Gy) + P.eps144);
      const T r = __builtin_amdgcn_rcpf(mag);
      const T a = P.lam12 * mag + (ph * ph - T(1)) * P.lamW2;
      const T coef = (a + P.negM12 * ((Mx * Gx + My * Gy) * r)) * r;
      sJx[idx] = coef * Gx;
      sJy[idx] = coef * Gy;
    } else {
      const T Gx = d4<T>(tP(lx - 2, ly), tP(lx - 1, ly), tP(lx + 1, ly), tP(lx + 2, ly));
      const T Gy = d4<T>(tP(lx, ly - 2), tP(lx, ly - 1), tP(lx, ly + 1), tP(lx, ly + 2));
      const T Mx = d4<T>(tM(lx - 2, ly), tM(lx - 1, ly), tM(lx + 1, ly), tM(lx + 2, ly));
      const T My = d4<T>(tM(lx, ly - 2), tM(lx, ly - 1), tM(lx, ly + 1), tM(lx, ly + 2));
      const T mag = sqrt((Gx * Gx + Gy * Gy) + P.eps2);
      const T nx = qdiv(Gx, mag), ny = qdiv(Gy, mag);
      const T cW = div_by(T(2) * (T(1) - ph * ph), P.W, P.invW);
      const T Jpx = (mag - cW) * nx, Jpy = (mag - cW) * ny;
      const T s = Mx * nx + My * ny;
      const T qx = (P.negM * s) * nx, qy = (P.negM * s) * ny;
      sJx[idx] = P.lam * Jpx + qx;
      sJy[idx] = P.lam * Jpy + qy;
    }
  });
  __syncthreads();
  for_window<TX, TY, NT>([&](int lx, int ly) {
    const int x = x0 + lx, y = y0 + ly;
    if (x >= P.nx || y >= P.ny) return;
    // FP32: the divergence's 1/12 applied once to the sum of the unscaled differences
    const T L =
        std::is_same<T, float>::value
            ? (d4u<T>(tJx(lx - 2, ly), tJx(lx - 1, ly), tJx(lx + 1, ly), tJx(lx + 2, ly)) +
               d4u<T>(tJy(lx, ly - 2), tJy(lx, ly - 1), tJy(lx, ly + 1), tJy(lx, ly + 2))) *
                  T(1.0 / 12.0)
            : d4<T>(tJx(lx - 2, ly), tJx(lx - 1, ly), tJx(lx + 1, ly), tJx(lx + 2, ly)) +
                  d4<T>(tJy(lx, ly - 2), tJy(lx, ly - 1), tJy(lx, ly + 1), tJy(lx, ly + 2));
    const long long id = (long long)y * P.nx + x;
    const T pin = tP(lx, ly);
    T r;
    if (STAGE == 1) {
      r = pin + L;
    } else if constexpr (std::is_same<T, float>::value) {
      // FP32: eq:TVD-3order as increments of phi_bar, phi^(2) = phi_bar +
      // (phi^(1) - phi_bar + L)/4 and phi = phi_bar + 2 (phi^(2) - phi_bar + L)/3,
      // so that the stage rounds once at phi's magnitude (phi_bar / 3 with the
      // rounded 1/3 would also scale phi by 1 + 3e-8 every step)
      const T pb = phibar[id];
      r = STAGE == 2 ? pb + T(0.25) * ((pin - pb) + L) : pb + divk<3>(T(2) * ((pin - pb) + L));
    } else if (STAGE == 2) {
      r = T(0.75) * phibar[id] + T(0.25) * (pin + L);
    } else {
      r = divk<3>(phibar[id]) + divk<3>(T(2) * (pin + L));
    }
    out[id] = r;
  });
}

// ---------------------------------------------------------- forces (a3, a5)
// Derived fields on halo 1 shared by the velocity iteration and the collision:
// grad phi (isotropic), mu_phi (eq:chemical), rho(clamp phi) (eq:rho).
template <typename T, int NT, int W1, int H1>
__device__ __forceinline__ void derived_halo1(const Tile<T>& tP, T* sPx, T* sPy, T* sMu, T* sRho,
                                              const KParams<T>& P) {
  for_window<W1, H1, NT>([&](int ix, int iy) {
    const int lx = ix - 1, ly = iy - 1, idx = iy * W1 + ix;
    T gx, gy;
    iso_grad<T>(tP, lx, ly, gx, gy);
    sPx[idx] = gx;
    sPy[idx] = gy;
    sMu[idx] = chem_pot<T>(tP, lx, ly, P.c4b, P.kappa);
    sRho[idx] = density<T>(tP(lx, ly), P.rho1, P.rho2);
  });
}

// products of grad phi for the stress-form surface force at a neighbour
template <typename T>
struct ProdYY {
  const Tile<T>&py;
  __device__ __forceinline__ T operator()(int x, int y) const { return py(x, y) * py(x, y); }
};
template <typename T>
struct ProdXX {
  const Tile<T>&px;
  __device__ __forceinline__ T operator()(int x, int y) const { return px(x, y) * px(x, y); }
};
template <typename T>
struct ProdXY {
  const Tile<T>&px, &py;
  __device__ __forceinline__ T operator()(int x, int y) const { return px(x, y) * py(x, y); }
};

// F = F_p + F_s + F_nu + F_m + F_g at tile node (x, y)  (Sec. 2.2)
template <typename T>
__device__ __forceinline__ void node_force(const Tile<T>& tP, const Tile<T>& tPx, const Tile<T>& tPy,
                                           const Tile<T>& tMu, const Tile<T>& tRho, const Tile<T>& tUx,
                                           const Tile<T>& tUy, T p, int x, int y, const KParams<T>& P,
                                           T& Fx, T& Fy, T& rho, T& nu, T& duxx, T& duxy, T& duyx,
                                           T& duyy) {
  const T phi = tP(x, y);
  rho = density<T>(phi, P.rho1, P.rho2);
  nu = kin_visc<T>(phi, rho, P.mu1, P.mu2);
  T dmx, dmy;
  iso_grad<T>(tMu, x, y, dmx, dmy);
  const T Jx = P.cJ * dmx, Jy = P.cJ * dmy;
  const T dxyy = iso_grad_x<T>(ProdYY<T>{tPy}, x, y);
  T dxxy, dyxy;
  iso_grad<T>(ProdXY<T>{tPx, tPy}, x, y, dxxy, dyxy);
  const T dyxx = iso_grad_y<T>(ProdXX<T>{tPx}, x, y);
  const T Fsx = P.kappa * (dxyy - dyxy);
  const T Fsy = P.kappa * (dyxx - dxxy);
  T grx, gry;
  iso_grad<T>(tRho, x, y, grx, gry);
  iso_grad<T>(tUx, x, y, duxx, duxy);
  iso_grad<T>(tUy, x, y, duyx, duyy);
  const T Fpx = (-p) * grx, Fpy = (-p) * gry;
  const T Sxx = duxx + duxx, Sxy = duyx + duxy, Syy = duyy + duyy;
  const T Fnx = nu * (Sxx * grx + Sxy * gry);
  const T Fny = nu * (Sxy * grx + Syy * gry);
  const T Fmx = Jx * duxx + Jy * duxy;
  const T Fmy = Jx * duyx + Jy * duyy;
  const T Fgx = (rho - P.rho_ref) * P.gx;
  const T Fgy = (rho - P.rho_ref) * P.gy;
  Fx = (((Fpx + Fsx) + Fnx) + Fmx) + Fgx;
  Fy = (((Fpy + Fsy) + Fny) + Fmy) + Fgy;
}

// F at tile node (x, y) with the strain rate of F_nu from the moments m1, m7,
// m8 of the node's pre-collision g (LBM2P_OPT_STRAIN_MOMENTS): the other force
// parts first, b of the source corrections from them and grad p, then F_nu
// (summed in node_force's order)
template <typename T>
__device__ __forceinline__ void node_force_sm(const Tile<T>& tP, const Tile<T>& tPx,
                                              const Tile<T>& tPy, const Tile<T>& tMu,
                                              const Tile<T>& tRho, const Tile<T>& tUx,
                                              const Tile<T>& tUy, T p, T m1, T m7, T m8, T dpx,
                                              T dpy, int x, int y, const KParams<T>& P, T& Fx,
                                              T& Fy, T& rho, T& nu) {
  const T phi = tP(x, y);
  rho = density<T>(phi, P.rho1, P.rho2);
  nu = kin_visc<T>(phi, rho, P.mu1, P.mu2);
  T dmx, dmy;
  iso_grad<T>(tMu, x, y, dmx, dmy);
  const T Jx = P.cJ * dmx, Jy = P.cJ * dmy;
  const T dxyy = iso_grad_x<T>(ProdYY<T>{tPy}, x, y);
  T dxxy, dyxy;
  iso_grad<T>(ProdXY<T>{tPx, tPy}, x, y, dxxy, dyxy);
  const T dyxx = iso_grad_y<T>(ProdXX<T>{tPx}, x, y);
  const T Fsx = P.kappa * (dxyy - dyxy);
  const T Fsy = P.kappa * (dyxx - dxxy);
  T grx, gry, duxx, duxy, duyx, duyy;
  iso_grad<T>(tRho, x, y, grx, gry);
  iso_grad<T>(tUx, x, y, duxx, duxy);
  iso_grad<T>(tUy, x, y, duyx, duyy);
  const T Fpx = (-p) * grx, Fpy = (-p) * gry;
  const T Fmx = Jx * duxx + Jy * duxy;
  const T Fmy = Jx * duyx + Jy * duyy;
  const T Fgx = (rho - P.rho_ref) * P.gx;
  const T Fgy = (rho - P.rho_ref) * P.gy;
  const T Frx = ((Fpx + Fsx) + Fmx) + Fgx, Fry = ((Fpy + Fsy) + Fmy) + Fgy;
  const T brx = (P.opt & 2) ? qdiv(Frx - dpx, rho) : qdiv(Frx, rho) - dpx;
  const T bry = (P.opt & 2) ? qdiv(Fry - dpy, rho) : qdiv(Fry, rho) - dpy;
  const T s7 = qdiv(T(1), nu * T(3) + T(0.5));
  T Sxx, Sxy, Syy;
  strain_moments<T>(m1, m7, m8, p, tUx(x, y), tUy(x, y), brx, bry, P.s_g[1], s7, P.p_ref, Sxx,
                    Sxy, Syy);
  const T Fnx = nu * (Sxx * grx + Sxy * gry);
  const T Fny = nu * (Sxy * grx + Syy * gry);
  Fx = (((Fpx + Fsx) + Fnx) + Fmx) + Fgx;
  Fy = (((Fpy + Fsy) + Fny) + Fmy) + Fgy;
}

// ------------------------------------------- a3: velocity fixed-point sweeps
// u^{k+1} = j + F(u^k) / (2 rho)   (Eq:u), KS consecutive sweeps in one launch:
// sweep k is evaluated on the tile grown by KS-1-k nodes, so the next sweep
// finds its halo in LDS.  Every sweep computes exactly what a one-sweep launch
// computes at the same node.
template <typename T, int KS, int TX, int TY, int NT, bool SM = false>
__global__ __launch_bounds__(NT) void k_vel(KParams<T> P, int tiles_x, const T* __restrict__ phi,
                                             const T* __restrict__ praw, const T* __restrict__ jx,
                                             const T* __restrict__ jy, const T* __restrict__ uxi,
                                             const T* __restrict__ uyi, T* __restrict__ uxo,
                                             T* __restrict__ uyo, const T* __restrict__ m1 = nullptr,
                                             const T* __restrict__ m7 = nullptr,
                                             const T* __restrict__ m8 = nullptr) {
  constexpr int HP = KS + 1;                      // phi halo
  constexpr int WP = TX + 2 * HP, HPH = TY + 2 * HP;
  constexpr int WD = TX + 2 * KS, HD = TY + 2 * KS;  // derived fields and u^0
  __shared__ T sP[WP * HPH];
  __shared__ T sPx[WD * HD], sPy[WD * HD], sMu[WD * HD], sRho[WD * HD];
  constexpr int NB = KS > 1 ? 2 : 1;               // the last sweep writes to HBM
  __shared__ T sU[NB][2][WD * HD];                // ping-pong velocity iterates
  __shared__ T sPr[SM ? WD * HD : 1];              // p, for grad p (moment strain rate)
  int bx, by;
  tile_of(tiles_x, bx, by);
  const int x0 = bx * TX, y0 = by * TY;
  load_window<T, T, NT, WP, HPH>(sP, phi, x0 - HP, y0 - HP, P, false);
  load_window<T, T, NT, WD, HD>(sU[0][0], uxi, x0 - KS, y0 - KS, P, true);
  load_window<T, T, NT, WD, HD>(sU[0][1], uyi, x0 - KS, y0 - KS, P, true);
  if constexpr (SM) load_window<T, T, NT, WD, HD>(sPr, praw, x0 - KS, y0 - KS, P, false);
  __syncthreads();
  const Tile<T> tP{sP, WP, HP};
  for_window<WD, HD, NT>([&](int ix, int iy) {
    const int lx = ix - KS, ly = iy - KS, idx = iy * WD + ix;
    T gx, gy;
    iso_grad<T>(tP, lx, ly, gx, gy);
    sPx[idx] = gx;
    sPy[idx] = gy;
    sMu[idx] = chem_pot<T>(tP, lx, ly, P.c4b, P.kappa);
    sRho[idx] = density<T>(tP(lx, ly), P.rho1, P.rho2);
  });
  __syncthreads();
  const Tile<T> tPx{sPx, WD, KS}, tPy{sPy, WD, KS}, tMu{sMu, WD, KS}, tRho{sRho, WD, KS};
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const int g = KS - 1 - k;                     // output halo of this sweep
    const int RW = TX + 2 * g, RH = TY + 2 * g;
    const Tile<T> tUx{sU[(k & 1) % NB][0], WD, KS}, tUy{sU[(k & 1) % NB][1], WD, KS};
    T* ox = sU[((k + 1) & 1) % NB][0];
    T* oy = sU[((k + 1) & 1) % NB][1];
    for (int idx = threadIdx.x; idx < RW * RH; idx += NT) {
      const int ly = idx / RW - g, lx = idx % RW - g;
      const int gxn = x0 + lx, gyn = y0 + ly;
      // ghosts beyond a wall are filled below from their mirror node
      if ((P.wx && (gxn < 0 || gxn >= P.nx)) || (P.wy && (gyn < 0 || gyn >= P.ny))) continue;
      if (g == 0 && (gxn >= P.nx || gyn >= P.ny)) continue;
      int flip = 0;
      const int x = map_idx(gxn, P.nx, P.wx, flip);
      const int y = map_idx(gyn, P.ny, P.wy, flip);
      const long long id = (long long)y * P.nx + x;
      T Fx, Fy, rho, nu;
      if constexpr (SM) {
        const Tile<T> tPr{sPr, WD, KS};
        T dpx, dpy;
        iso_grad<T>(tPr, lx, ly, dpx, dpy);
        node_force_sm<T>(tP, tPx, tPy, tMu, tRho, tUx, tUy, praw[id], m1[id], m7[id], m8[id], dpx,
                         dpy, lx, ly, P, Fx, Fy, rho, nu);
      } else {
        T a, b, c, d;
        node_force<T>(tP, tPx, tPy, tMu, tRho, tUx, tUy, praw[id], lx, ly, P, Fx, Fy, rho, nu, a,
                      b, c, d);
      }
      const T vx = jx[id] + qdiv(Fx, T(2) * rho);
      const T vy = jy[id] + qdiv(Fy, T(2) * rho);
      if (g == 0) {
        uxo[id] = vx;
        uyo[id] = vy;
      } else {
        const int o = (ly + KS) * WD + (lx + KS);
        ox[o] = vx;
        oy[o] = vy;
      }
    }
    __syncthreads();
    if (g > 0 && (P.wx || P.wy)) {
      // no-slip ghosts: the mirror node's value with its sign flipped once per
      // mirrored axis (as the oracle's ghost extension does)
      for (int idx = threadIdx.x; idx < RW * RH; idx += NT) {
        const int ly = idx / RW - g, lx = idx % RW - g;
        const int gxn = x0 + lx, gyn = y0 + ly;
        int mx = gxn, my = gyn, flips = 0;
        if (P.wx && gxn < 0) { mx = -1 - gxn; flips ^= 1; }
        if (P.wx && gxn >= P.nx) { mx = 2 * P.nx - 1 - gxn; flips ^= 1; }
        if (P.wy && gyn < 0) { my = -1 - gyn; flips ^= 1; }
        if (P.wy && gyn >= P.ny) { my = 2 * P.ny - 1 - gyn; flips ^= 1; }
        if (mx == gxn && my == gyn) continue;            // not a ghost
        const int lmx = mx - x0, lmy = my - y0;
        const int o = (ly + KS) * WD + (lx + KS);
        if (lmx < -g || lmx >= TX + g || lmy < -g || lmy >= TY + g) {
          ox[o] = T(0);                                  // never read by an in-domain output
          oy[o] = T(0);
          continue;
        }
        const int om = (lmy + KS) * WD + (lmx + KS);
        ox[o] = flips ? -ox[om] : ox[om];
        oy[o] = flips ? -oy[om] : oy[om];
      }
      __syncthreads();
    }
  }
}

// Two velocity sweeps in one launch.  phi and p are fixed during the sweeps,
// so F_p + F_s, J = c_J grad mu, grad rho, nu and rho are the same in both: on
// the tile's own nodes they are evaluated once and kept in registers (each
// thread owns TX*TY/NT nodes in both sweeps), and the second sweep
// re-evaluates only the u-dependent F_nu and F_m.  The first sweep also covers
// the ring of nodes around the tile, which the second sweep's stencils read;
// its results wait in registers until every thread has read u^0, then
// overwrite u^0 in LDS.  grad phi enters only through the products of the
// stress-form surface force, so LDS holds those products (each formed once
// per node, as the force's stencils would form it at every neighbour).
// FP64 sums F in the order (((F_p + F_s) + F_nu) + F_m) + F_g of node_force.
// FP32 without the moment strain rate writes a sweep as the affine map
// u^{k+1} = b + A grad u^k it is (F_nu and F_m are linear in grad u), with b
// and the six entries of A formed once per node.  With u1x, u1y given, the
// first sweep's iterate is written there too (the adjoint keeps every iterate).
template <typename T, int TX, int TY, int NT, bool SM = false>
__global__ __launch_bounds__(NT) void k_vel2(KParams<T> P, int tiles_x, const T* __restrict__ phi,
                                              const T* __restrict__ praw, const T* __restrict__ jx,
                                              const T* __restrict__ jy, const T* __restrict__ uxi,
                                              const T* __restrict__ uyi, T* __restrict__ uxo,
                                              T* __restrict__ uyo, T* __restrict__ u1x,
                                              T* __restrict__ u1y, const T* __restrict__ m1 = nullptr,
                                              const T* __restrict__ m7 = nullptr,
                                              const T* __restrict__ m8 = nullptr) {
  static_assert((TX * TY) % NT == 0, "whole tile rows per thread group");
  constexpr int WP = TX + 6, HPH = TY + 6;   // phi, halo 3
  constexpr int WD = TX + 4, HD = TY + 4;    // derived fields and u^0, then u^1, halo 2
  constexpr int W1 = TX + 2, H1 = TY + 2;    // first sweep, halo 1
  constexpr int NI = TX * TY / NT;           // tile nodes per thread
  constexpr int NRING = 2 * W1 + 2 * TY;     // nodes of the halo-1 ring
  constexpr int KRING = (NRING + NT - 1) / NT;
  constexpr bool LIN = std::is_same<T, float>::value && !SM;
  __shared__ T sP[WP * HPH];
  __shared__ T sQxx[WD * HD], sQyy[WD * HD], sQxy[WD * HD], sMu[WD * HD], sRho[WD * HD];
  __shared__ T sUx[WD * HD], sUy[WD * HD];
  __shared__ T sPr[SM ? WD * HD : 1];        // p, for grad p (moment strain rate)
  int bx, by;
  tile_of(tiles_x, bx, by);
  const int x0 = bx * TX, y0 = by * TY;
  load_window<T, T, NT, WP, HPH>(sP, phi, x0 - 3, y0 - 3, P, false);
  load_window<T, T, NT, WD, HD>(sUx, uxi, x0 - 2, y0 - 2, P, true);
  load_window<T, T, NT, WD, HD>(sUy, uyi, x0 - 2, y0 - 2, P, true);
  if constexpr (SM) load_window<T, T, NT, WD, HD>(sPr, praw, x0 - 2, y0 - 2, P, false);
  __syncthreads();
  const Tile<T> tP{sP, WP, 3};
  for_window<WD, HD, NT>([&](int ix, int iy) {
    const int lx = ix - 2, ly = iy - 2, idx = iy * WD + ix;
    T gx, gy;
    iso_grad<T>(tP, lx, ly, gx, gy);
    sQxx[idx] = gx * gx;
    sQyy[idx] = gy * gy;
    sQxy[idx] = gx * gy;
    sMu[idx] = chem_pot<T>(tP, lx, ly, P.c4b, P.kappa);
    sRho[idx] = density<T>(tP(lx, ly), P.rho1, P.rho2);
  });
  __syncthreads();
  const Tile<T> tQxx{sQxx, WD, 2}, tQyy{sQyy, WD, 2}, tQxy{sQxy, WD, 2}, tMu{sMu, WD, 2},
      tRho{sRho, WD, 2}, tUx{sUx, WD, 2}, tUy{sUy, WD, 2};
  // the tile grown by one lies inside the lattice: plain row addresses
  const bool inner = x0 >= 1 && x0 + W1 - 1 <= P.nx && y0 >= 1 && y0 + H1 - 1 <= P.ny;
  auto node_id = [&](int lx, int ly) {
    const int gxn = x0 + lx, gyn = y0 + ly;
    if (inner) return gyn * P.nx + gxn;
    // wrap or mirror (a ghost beyond a wall reads its mirror node; its u^1 is
    // replaced below)
    int flip = 0;
    const int x = map_idx(gxn, P.nx, P.wx, flip);
    const int y = map_idx(gyn, P.ny, P.wy, flip);
    return y * P.nx + x;
  };
  // the u-independent parts of the surface force and of J at (lx, ly)
  auto surface = [&](int lx, int ly, T& Fsx, T& Fsy, T& Jx, T& Jy, T& gx, T& gy) {
    T dmx, dmy;
    iso_grad<T>(tMu, lx, ly, dmx, dmy);
    const T dxyy = iso_grad_x<T>(tQyy, lx, ly);
    T dxxy, dyxy;
    iso_grad<T>(tQxy, lx, ly, dxxy, dyxy);
    const T dyxx = iso_grad_y<T>(tQxx, lx, ly);
    iso_grad<T>(tRho, lx, ly, gx, gy);
    Fsx = P.kappa * (dxyy - dyxy);
    Fsy = P.kappa * (dyxx - dxxy);
    Jx = P.cJ * dmx;
    Jy = P.cJ * dmy;
  };
  // FP64 / moment strain rate: the force parts, summed in the sweep.
  // FP64: ir2 = 1/(2 rho) rounded once; the four quotients by 2 rho of the two
  // sweeps and nu = mu/rho (2 ir2 = RN(1/rho) exactly) are then FMA-corrected
  // products, bitwise the divisions they replace
  struct Parts {
    T Fx, Fy, Jx, Jy, gx, gy, nu, rho, jx, jy, ir2;
    T p, dpx, dpy, m1, m7, m8, s7;   // moment strain rate only
  };
  // FP32: u^{k+1} = b + A (duxx, duxy, duyx, duyy)
  struct Lin {
    T bx, by, a1, a2, a3, b1, b2, b3;
  };
  using Node = typename std::conditional<LIN, Lin, Parts>::type;
  auto parts = [&](int lx, int ly) {
    const int id = node_id(lx, ly);
    Node q;
    const T p = praw[id];
    const T ph = tP(lx, ly);
    T Fsx, Fsy, Jx, Jy, gx, gy;
    surface(lx, ly, Fsx, Fsy, Jx, Jy, gx, gy);
    if constexpr (LIN) {
      const T rho = density<T>(ph, P.rho1, P.rho2);
      const T ir = __builtin_amdgcn_rcpf(rho);
      const T nu = dyn_visc<T>(ph, P.mu1, P.mu2) * ir;
      const T r2 = T(0.5) * ir;
      const T Fcx = ((-p) * gx + Fsx) + (rho - P.rho_ref) * P.gx;
      const T Fcy = ((-p) * gy + Fsy) + (rho - P.rho_ref) * P.gy;
      const T ngx = nu * gx, ngy = nu * gy;
      q.bx = jx[id] + Fcx * r2;
      q.by = jy[id] + Fcy * r2;
      q.a1 = ((ngx + ngx) + Jx) * r2;
      q.a2 = (ngy + Jy) * r2;
      q.a3 = ngy * r2;
      q.b1 = ngx * r2;
      q.b2 = (ngx + Jx) * r2;
      q.b3 = ((ngy + ngy) + Jy) * r2;
    } else {
      q.jx = jx[id];
      q.jy = jy[id];
      q.rho = density<T>(ph, P.rho1, P.rho2);
      if constexpr (std::is_same<T, float>::value) {
        q.nu = kin_visc<T>(ph, q.rho, P.mu1, P.mu2);
        q.ir2 = T(0);
      } else {
        q.ir2 = T(1) / (T(2) * q.rho);
        q.nu = div_by(dyn_visc<T>(ph, P.mu1, P.mu2), q.rho, T(2) * q.ir2);
      }
      q.gx = gx;
      q.gy = gy;
      q.Fx = (-p) * gx + Fsx;
      q.Fy = (-p) * gy + Fsy;
      q.Jx = Jx;
      q.Jy = Jy;
      if constexpr (SM) {
        const Tile<T> tPr{sPr, WD, 2};
        q.p = p;
        iso_grad<T>(tPr, lx, ly, q.dpx, q.dpy);
        q.m1 = m1[id];
        q.m7 = m7[id];
        q.m8 = m8[id];
        q.s7 = qdiv(T(1), q.nu * T(3) + T(0.5));
      }
    }
    return q;
  };
  auto sweep = [&](const Node& q, int lx, int ly, T& vx, T& vy) {
    T duxx, duxy, duyx, duyy;
    iso_grad<T>(tUx, lx, ly, duxx, duxy);
    iso_grad<T>(tUy, lx, ly, duyx, duyy);
    if constexpr (LIN) {
      vx = ((q.bx + q.a1 * duxx) + q.a2 * duxy) + q.a3 * duyx;
      vy = ((q.by + q.b1 * duxy) + q.b2 * duyx) + q.b3 * duyy;
    } else {
      const T Fmx = q.Jx * duxx + q.Jy * duxy, Fmy = q.Jx * duyx + q.Jy * duyy;
      const T Fgx = (q.rho - P.rho_ref) * P.gx, Fgy = (q.rho - P.rho_ref) * P.gy;
      T Sxx, Sxy, Syy;
      if constexpr (SM) {
        // b of the source corrections from the force parts other than F_nu
        const T Frx = (q.Fx + Fmx) + Fgx, Fry = (q.Fy + Fmy) + Fgy;
        T brx, bry;
        if constexpr (std::is_same<T, float>::value) {
          brx = (P.opt & 2) ? qdiv(Frx - q.dpx, q.rho) : qdiv(Frx, q.rho) - q.dpx;
          bry = (P.opt & 2) ? qdiv(Fry - q.dpy, q.rho) : qdiv(Fry, q.rho) - q.dpy;
        } else {
          brx = (P.opt & 2) ? div_by(Frx - q.dpx, q.rho, T(2) * q.ir2)
                            : div_by(Frx, q.rho, T(2) * q.ir2) - q.dpx;
          bry = (P.opt & 2) ? div_by(Fry - q.dpy, q.rho, T(2) * q.ir2)
                            : div_by(Fry, q.rho, T(2) * q.ir2) - q.dpy;
        }
        strain_moments<T>(q.m1, q.m7, q.m8, q.p, tUx(lx, ly), tUy(lx, ly), brx, bry, P.s_g[1],
                          q.s7, P.p_ref, Sxx, Sxy, Syy);
      } else {
        Sxx = duxx + duxx;
        Sxy = duyx + duxy;
        Syy = duyy + duyy;
      }
      const T Fx = ((q.Fx + q.nu * (Sxx * q.gx + Sxy * q.gy)) + Fmx) + Fgx;
      const T Fy = ((q.Fy + q.nu * (Sxy * q.gx + Syy * q.gy)) + Fmy) + Fgy;
      if constexpr (std::is_same<T, float>::value) {
        vx = q.jx + qdiv(Fx, T(2) * q.rho);
        vy = q.jy + qdiv(Fy, T(2) * q.rho);
      } else {
        vx = q.jx + div_by(Fx, T(2) * q.rho, q.ir2);
        vy = q.jy + div_by(Fy, T(2) * q.rho, q.ir2);
      }
    }
  };
  auto ring_node = [&](int k, int& lx, int& ly) {
    // rows -1 and TY (W1 nodes each), then columns -1 and TX
    if (k < 2 * W1) {
      ly = k < W1 ? -1 : TY;
      lx = (k < W1 ? k : k - W1) - 1;
    } else {
      const int j = k - 2 * W1;
      ly = j >> 1;
      lx = (j & 1) ? TX : -1;
    }
  };
  // first sweep on the tile's nodes and its ring, from u^0
  Node c[NI];
  T v1x[NI], v1y[NI], rvx[KRING], rvy[KRING];
#pragma unroll
  for (int r = 0; r < NI; ++r) {
    const int idx = threadIdx.x + r * NT;
    const int ly = idx / TX, lx = idx - ly * TX;
    c[r] = parts(lx, ly);
    sweep(c[r], lx, ly, v1x[r], v1y[r]);
    if (u1x != nullptr && x0 + lx < P.nx && y0 + ly < P.ny) {
      const int id = (y0 + ly) * P.nx + x0 + lx;
      u1x[id] = v1x[r];
      u1y[id] = v1y[r];
    }
  }
#pragma unroll
  for (int r = 0; r < KRING; ++r) {
    const int k = threadIdx.x + r * NT;
    if (k < NRING) {
      int lx, ly;
      ring_node(k, lx, ly);
      const Node q = parts(lx, ly);
      sweep(q, lx, ly, rvx[r], rvy[r]);
    }
  }
  __syncthreads();   // every read of u^0 done: u^1 replaces it on halo 1
#pragma unroll
  for (int r = 0; r < NI; ++r) {
    const int idx = threadIdx.x + r * NT;
    const int ly = idx / TX, lx = idx - ly * TX;
    tUx.at(lx, ly) = v1x[r];
    tUy.at(lx, ly) = v1y[r];
  }
#pragma unroll
  for (int r = 0; r < KRING; ++r) {
    const int k = threadIdx.x + r * NT;
    if (k < NRING) {
      int lx, ly;
      ring_node(k, lx, ly);
      tUx.at(lx, ly) = rvx[r];
      tUy.at(lx, ly) = rvy[r];
    }
  }
  __syncthreads();
  if (P.wx || P.wy) {
    // no-slip ghosts of u^1: the mirror node's value, sign flipped once per
    // mirrored axis (as the oracle's ghost extension does).  Ghost and mirror
    // sets are disjoint, so reads and writes do not overlap
    for_window<W1, H1, NT>([&](int ix, int iy) {
      const int lx = ix - 1, ly = iy - 1;
      const int gxn = x0 + lx, gyn = y0 + ly;
      int mx = gxn, my = gyn, flips = 0;
      if (P.wx && gxn < 0) { mx = -1 - gxn; flips ^= 1; }
      if (P.wx && gxn >= P.nx) { mx = 2 * P.nx - 1 - gxn; flips ^= 1; }
      if (P.wy && gyn < 0) { my = -1 - gyn; flips ^= 1; }
      if (P.wy && gyn >= P.ny) { my = 2 * P.ny - 1 - gyn; flips ^= 1; }
      if (mx == gxn && my == gyn) return;              // not a ghost
      const int lmx = mx - x0, lmy = my - y0;
      T vx = T(0), vy = T(0);                          // never read by an in-domain output
      if (lmx >= -1 && lmx < TX + 1 && lmy >= -1 && lmy < TY + 1) {
        vx = flips ? -tUx(lmx, lmy) : tUx(lmx, lmy);
        vy = flips ? -tUy(lmx, lmy) : tUy(lmx, lmy);
      }
      tUx.at(lx, ly) = vx;
      tUy.at(lx, ly) = vy;
    });
    __syncthreads();
  }
  // second sweep from u^1 on the tile's own nodes
#pragma unroll
  for (int r = 0; r < NI; ++r) {
    const int idx = threadIdx.x + r * NT;
    const int ly = idx / TX, lx = idx - ly * TX;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= P.nx || y >= P.ny) continue;
    T vx, vy;
    sweep(c[r], lx, ly, vx, vy);
    const int id = y * P.nx + x;
    uxo[id] = vx;
    uyo[id] = vy;
  }
}

// ------------------------------------------------ a4: explicit selective filter
// chi <- chi - a [ sum_j d_|j| chi(x+j, y) + sum_j d_|j| chi(x, y+j) ]  (eq:filter)
template <typename T, int N, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_filter(KParams<T> P, int tiles_x, const T* __restrict__ pin,
                                                const T* __restrict__ uxin,
                                                const T* __restrict__ uyin, T* __restrict__ pout,
                                                T* __restrict__ uxout, T* __restrict__ uyout) {
  static_assert(NT % TX == 0 && (TX * TY) % NT == 0, "whole column strips per thread");
  constexpr int WN = TX + 2 * N, HN = TY + 2 * N, R = TX * TY / NT;
  __shared__ T s0[WN * HN], s1[WN * HN], s2[WN * HN];
  int bx, by;
  tile_of(tiles_x, bx, by);
  const int x0 = bx * TX, y0 = by * TY;
  load_window<T, T, NT, WN, HN>(s0, pin, x0 - N, y0 - N, P, false);
  load_window<T, T, NT, WN, HN>(s1, uxin, x0 - N, y0 - N, P, true);
  load_window<T, T, NT, WN, HN>(s2, uyin, x0 - N, y0 - N, P, true);
  __syncthreads();
  T d[N + 1];
#pragma unroll
  for (int j = 0; j <= N; ++j) d[j] = P.fd[j];
  const T a = P.fa;
  // each thread filters R consecutive rows of one column: the column's
  // 2N + R values of the y-stencil are read from LDS once into registers
  const int lx = threadIdx.x % TX, ly0 = (threadIdx.x / TX) * R;
  const int x = x0 + lx;
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const Tile<T> t{f == 0 ? s0 : f == 1 ? s1 : s2, WN, N};
    T col[R + 2 * N];
#pragma unroll
    for (int k = 0; k < R + 2 * N; ++k) col[k] = t(lx, ly0 - N + k);
    T* out = f == 0 ? pout : f == 1 ? uxout : uyout;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int ly = ly0 + r, y = y0 + ly;
      if (x >= P.nx || y >= P.ny) continue;
      const T* cy = col + r + N;   // cy[j] = chi(x, y + j)
      T sx, sy;
      if constexpr (std::is_same<T, float>::value) {
        // FP32: sum_j d_|j| chi_j = sum_k d_k [(chi_k - chi_0) + (chi_-k - chi_0)]
        // (the d_j sum to zero), so a uniform field passes exactly: the FP32
        // d_j sum to -4.7e-9 for SF-11, a gain of 1 + 4.7e-9 per application
        // in the chained form, and the differences of a smooth field are exact.
        const T c0 = cy[0];
        sx = d[N] * ((t(lx + N, ly) - c0) + (t(lx - N, ly) - c0));
        sy = d[N] * ((cy[N] - c0) + (cy[-N] - c0));
#pragma unroll
        for (int k = N - 1; k >= 1; --k) {
          sx = sx + d[k] * ((t(lx + k, ly) - c0) + (t(lx - k, ly) - c0));
          sy = sy + d[k] * ((cy[k] - c0) + (cy[-k] - c0));
        }
      } else {
        sx = d[N] * t(lx - N, ly);
#pragma unroll
        for (int j = -N + 1; j <= N; ++j) sx = sx + d[j < 0 ? -j : j] * (j == 0 ? cy[0] : t(lx + j, ly));
        sy = d[N] * cy[-N];
#pragma unroll
        for (int j = -N + 1; j <= N; ++j) sy = sy + d[j < 0 ? -j : j] * cy[j];
      }
      out[(long long)y * P.nx + x] = cy[0] - a * (sx + sy);
    }
  }
}

// ------------------------------------------------------ a5: collide + stream
// MRT collision of f (eq:distribution_CH) and g (eq:distribution_NS) at n+1,
// written to the streaming slots of the other parity.
template <typename T, int PAR, bool COUPLED, bool STREAM, int TX, int TY, int NT, bool SM = false>
__global__ __launch_bounds__(NT, (sizeof(T) == 4 && NT == 512) ? 4 : 1) void k_collide(KParams<T> P, int tiles_x, T* __restrict__ Af, T* __restrict__ Ag,
                                                 const T* __restrict__ phi, const T* __restrict__ pt,
                                                 const T* __restrict__ ux, const T* __restrict__ uy,
                                                 const T* __restrict__ uox,
                                                 const T* __restrict__ uoy) {
  constexpr int W2 = TX + 4, H2 = TY + 4, W1 = TX + 2, H1 = TY + 2;
  __shared__ T sP[W2 * H2];
  __shared__ T sPx[COUPLED ? W1 * H1 : 1], sPy[COUPLED ? W1 * H1 : 1], sMu[W1 * H1],
      sRho[COUPLED ? W1 * H1 : 1], sUx[W1 * H1], sUy[W1 * H1], sPt[COUPLED ? W1 * H1 : 1];
  int bx, by;
  tile_of(tiles_x, bx, by);
  const int x0 = bx * TX, y0 = by * TY;
  load_window<T, T, NT, W2, H2>(sP, phi, x0 - 2, y0 - 2, P, false);
  load_window<T, T, NT, W1, H1>(sUx, ux, x0 - 1, y0 - 1, P, true);
  load_window<T, T, NT, W1, H1>(sUy, uy, x0 - 1, y0 - 1, P, true);
  if (COUPLED) load_window<T, T, NT, W1, H1>(sPt, pt, x0 - 1, y0 - 1, P, false);
  __syncthreads();
  const Tile<T> tP{sP, W2, 2};
  if (COUPLED) {
    derived_halo1<T, NT, W1, H1>(tP, sPx, sPy, sMu, sRho, P);
  } else {
    for_window<W1, H1, NT>([&](int ix, int iy) {
      sMu[iy * W1 + ix] = chem_pot<T>(tP, ix - 1, iy - 1, P.c4b, P.kappa);
    });
  }
  __syncthreads();
  const Tile<T> tPx{sPx, W1, 1}, tPy{sPy, W1, 1}, tMu{sMu, W1, 1}, tRho{sRho, W1, 1},
      tUx{sUx, W1, 1}, tUy{sUy, W1, 1}, tPt{sPt, W1, 1};
  for (int idx = threadIdx.x; idx < TX * TY; idx += NT) {
    const int ly = idx / TX, lx = idx % TX;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= P.nx || y >= P.ny) continue;
    const long long id = (long long)y * P.nx + x;
    const T ph = tP(lx, ly), u_x = tUx(lx, ly), u_y = tUy(lx, ly);
    // CH: material acceleration (eq:Fi), chemical potential, equilibrium
    T duxx, duxy, duyx, duyy;
    iso_grad<T>(tUx, lx, ly, duxx, duxy);
    iso_grad<T>(tUy, lx, ly, duyx, duyy);
    const T ax = (u_x - uox[id]) + (u_x * duxx + u_y * duxy);
    const T ay = (u_y - uoy[id]) + (u_x * duyx + u_y * duyy);
    int rd[9];
    slots<PAR, false>(P, x, y, rd);
    T g[9];
    {
      T f[9], feq[9];
      col_load9<PAR, STREAM>(Af, rd, f, std::make_integer_sequence<int, 9>{});
      if constexpr (COUPLED) {   // both distributions' loads in flight together
        col_load9<PAR, STREAM>(Ag, rd, g, std::make_integer_sequence<int, 9>{});
      }
      f_eq<T>(ph, tMu(lx, ly), u_x, u_y, P.eta, feq);
      if constexpr (std::is_same<T, float>::value) {
        // moments of eq:Fi: M F = (0, 0, 0, phi a_x, -phi a_x, phi a_y, -phi a_y, 0, 0)
        const T pax = ph * ax, pay = ph * ay;
        const T mF[9] = {T(0), T(0), T(0), pax, -pax, pay, -pay, T(0), T(0)};
        // FP32: the post-collision mass sum f* = m_0 - s_0 (m_0 - phi) (phi itself for
        // s_0 = 1) is kept exactly up to one rounding: f*_0 is that target minus the
        // eight moving populations (the value M^-1 gives, rounded once at phi's
        // magnitude); f*_0 from M^-1 summed with the moving populations loses
        // ~1e-8 of phi per node and step, a drift of the total mass
        const T m0 = f[0] + (((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8])));
        const T t0 = ph + (T(1) - P.s_f[0]) * (m0 - ph);
        mrt_collide_ms<T>(f, feq, mF, P.s_f);
        f[0] = t0 - (((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8])));
      } else {
        T F[9];
        src_f<T>(ph, ax, ay, F);
        mrt_collide<T>(f, feq, F, P.s_f);
      }
      col_store9<PAR, STREAM>(Af, rd, f, std::make_integer_sequence<int, 9>{});
    }
    if (COUPLED) {
      const T p = tPt(lx, ly);
      T Fx, Fy, rho, nu;
      T dpx, dpy;
      iso_grad<T>(tPt, lx, ly, dpx, dpy);
      if constexpr (SM) {
        T m1, m7, m8;
        moments_178<T>(g, m1, m7, m8);
        node_force_sm<T>(tP, tPx, tPy, tMu, tRho, tUx, tUy, p, m1, m7, m8, dpx, dpy, lx, ly, P, Fx,
                         Fy, rho, nu);
      } else {
        T a, b, c, d;
        node_force<T>(tP, tPx, tPy, tMu, tRho, tUx, tUy, p, lx, ly, P, Fx, Fy, rho, nu, a, b, c,
                      d);
      }
      const T Frx = qdiv(Fx, rho), Fry = qdiv(Fy, rho);
      // R8's b = F/rho - grad p, or eq:Gi as printed, (F - grad p)/rho
      const T bx = (P.opt & 2) ? qdiv(Fx - dpx, rho) : Frx - dpx;
      const T by = (P.opt & 2) ? qdiv(Fy - dpy, rho) : Fry - dpy;
      T s[9];
      const T tau_g = nu * T(3) + T(0.5);
      const T sv = qdiv(T(1), tau_g);
#pragma unroll
      for (int k = 0; k < 9; ++k) s[k] = P.s_g[k];
      s[7] = sv;
      s[8] = sv;
      if constexpr (std::is_same<T, float>::value) {
        // moments of eq:Gi: M G = (0, 6 b.u, -6 b.u, F_x/rho, -F_x/rho, F_y/rho,
        // -F_y/rho, 2 (b_x u_x - b_y u_y), b_x u_y + b_y u_x)
        const T ub6 = T(6) * (u_x * bx + u_y * by);
        const T mG[9] = {T(0), ub6, -ub6, Frx, -Frx, Fry, -Fry,
                         T(2) * (bx * u_x - by * u_y), bx * u_y + by * u_x};
        T meq[9];   // of the stored deviations g^eq - 3 w p_ref
        g_eq_moments<T>(p - P.p_ref, u_x, u_y, meq);
        mrt_collide_meq<T>(g, meq, mG, s);
      } else {
        T geq[9], G[9];
        g_eq<T>(p - P.p_ref, u_x, u_y, geq);   // stored deviations: g^eq - 3 w p_ref
        src_g<T>(Frx, Fry, u_x, u_y, bx, by, G);
        mrt_collide<T>(g, geq, G, s);
      }
      col_store9<PAR, STREAM>(Ag, rd, g, std::make_integer_sequence<int, 9>{});
    }
  }
}

}  // namespace lbm2p
