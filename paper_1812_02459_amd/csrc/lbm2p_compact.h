// Compact (tridiagonal) selective filter -- the variant named in the paper's
// abstract and conclusions (whose explicit filter is eq:filter).  Per line:
//   alpha F_{i-1} + F_i + alpha F_{i+1} = sum_{n=0..N} (a_n / 2)(chi_{i+n} + chi_{i-n})
// and the field update keeps eq:filter's unsplit form and intensity a:
//   chi~ = chi - a [ (chi - F_x chi) + (chi - F_y chi) ].
// The a_n solve T(0) = 1, T(pi) = 0 and the flatness conditions of the transfer
// function T(w) = sum a_n cos(n w) / (1 + 2 alpha cos w) (host side, lbm2p.hip).
//
// The line matrix is factorised once on the host (Thomas: c'_i and 1/pivot_i);
// a periodic line is the cyclic matrix, solved by Sherman-Morrison with a
// precomputed correction vector z.  Beyond a wall the right-hand side uses the
// half-way mirror ghosts (sign kept for p, flipped for u) and the matrix's end
// rows fold the ghost F_{-1} = +-F_0 into the diagonal.
//
// Parallel line solve.  The forward and backward Thomas sweeps are first-order
// linear recurrences,  d_i = (-alpha/piv_i) d_{i-1} + r_i/piv_i  and
// y_i = -c'_i y_{i+1} + d_i.  One wavefront takes one (line, field); each of its
// 64 lanes owns a contiguous chunk of the line, composes its chunk's affine map
// x -> A x + B, and a 6-step shuffle scan over the lanes gives every chunk the
// value entering it; a second pass over the chunk then produces the values.
// x-lines (contiguous rows) are staged in LDS; y-lines are taken 64 columns at
// a time, each column split into chunks over the waves of a workgroup.  The
// periodic lines' Sherman-Morrison correction x_i = y_i - f z_i (f per line)
// is applied where F is consumed.
#pragma once

#include "lbm2p_kernels.h"

namespace lbm2p {

// Table layout per (axis, parity): cp[n] (c'), inv[n] (1/pivot), z[n] (cyclic
// correction, periodic lines only), and the scalars fac = beta/gamma,
// den = 1 + z_0 + fac z_{n-1} of the Sherman-Morrison denominator.
struct CompactLine {
  const double* cp;
  const double* inv;
  const double* z;
  double fac, den;
  int cyclic;
  int K;                   // c'_i, 1/pivot_i equal cp_lim, inv_lim for K <= i <= n - 2
  double cp_lim, inv_lim;
};

// table entries, read only outside their constant run
template <typename T>
__device__ __forceinline__ T cl_inv(const CompactLine& L, int i, int n) {
  return (i < L.K || i == n - 1) ? T(L.inv[i]) : T(L.inv_lim);
}
template <typename T>
__device__ __forceinline__ T cl_cp(const CompactLine& L, int i, int n) {
  return (i < L.K || i == n - 1) ? T(L.cp[i]) : T(L.cp_lim);
}

template <typename T>
struct CompactArgs {
  double a[6];          // a_0 .. a_N
  double alpha;
  CompactLine line[2][2];  // [axis 0 = x, 1 = y][parity 0 = even, 1 = odd]
};

// value of field f (stride s along the line, base offset b) at line index i
template <typename T>
__device__ __forceinline__ T line_val(const T* __restrict__ f, long long b, long long s, int i,
                                      int n, int wall, bool odd) {
  int flip = 0;
  const int k = map_idx(i, n, wall, flip);
  const T v = f[b + s * k];
  return (odd && flip) ? -v : v;
}

// x -> a x + b
template <typename T>
struct Aff {
  T a, b;
};

// l after e
template <typename T>
__device__ __forceinline__ Aff<T> aff_after(const Aff<T>& l, const Aff<T>& e) {
  return Aff<T>{l.a * e.a, l.a * e.b + l.b};
}

// Composite of the maps of lanes 0..k-1 (UP) or k+1..63 (down), applied to 0:
// the value entering lane k's chunk.  Hillis-Steele over the wavefront.
template <typename T, bool UP>
__device__ __forceinline__ T lane_carry(Aff<T> m) {
  const int lane = (int)(threadIdx.x & 63);
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T oa = UP ? __shfl_up(m.a, d, 64) : __shfl_down(m.a, d, 64);
    const T ob = UP ? __shfl_up(m.b, d, 64) : __shfl_down(m.b, d, 64);
    const bool ok = UP ? lane >= d : lane + d < 64;
    if (ok) m = aff_after(m, Aff<T>{oa, ob});
  }
  // exclusive: the neighbour's inclusive composite, applied to 0
  const T b = UP ? __shfl_up(m.b, 1, 64) : __shfl_down(m.b, 1, 64);
  return (UP ? lane == 0 : lane == 63) ? T(0) : b;
}

// The value entering thread t's chunk when NWV waves hold consecutive chunks
// (t = 64 wave + lane): UP composes chunks 0..t-1, down chunks t+1..end, both
// applied to 0.  Intra-wave scans, then the wave totals through LDS.
template <typename T, bool UP, int NWV>
__device__ __forceinline__ T block_carry(Aff<T> m, T* sWa, T* sWb) {
  const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T oa = UP ? __shfl_up(m.a, d, 64) : __shfl_down(m.a, d, 64);
    const T ob = UP ? __shfl_up(m.b, d, 64) : __shfl_down(m.b, d, 64);
    const bool ok = UP ? lane >= d : lane + d < 64;
    if (ok) m = aff_after(m, Aff<T>{oa, ob});
  }
  // this wave's total: the inclusive composite at its last lane in the order
  if (lane == (UP ? 63 : 0)) {
    sWa[wv] = m.a;
    sWb[wv] = m.b;
  }
  // exclusive composite within the wave (identity at the first lane)
  T ea = UP ? __shfl_up(m.a, 1, 64) : __shfl_down(m.a, 1, 64);
  T eb = UP ? __shfl_up(m.b, 1, 64) : __shfl_down(m.b, 1, 64);
  if (lane == (UP ? 0 : 63)) {
    ea = T(1);
    eb = T(0);
  }
  __syncthreads();
  T c = T(0);
  if (UP) {
    for (int k = 0; k < wv; ++k) c = sWa[k] * c + sWb[k];
  } else {
    for (int k = NWV - 1; k > wv; --k) c = sWa[k] * c + sWb[k];
  }
  __syncthreads();
  return ea * c + eb;
}

// Longest line the LDS-staged line solve takes (the FP64 line, padded, in 64 KB).
constexpr int COMPACT_MAX_N = 7680;

// LDS position of line element e: one pad word per chunk of 2^lg elements, so
// that the 64 lanes walking their chunks in step hit distinct banks.
__device__ __forceinline__ int cpad(int e, int lg) { return e + (e >> lg); }

// Solve the line systems of 3 fields of rows of length n (nlines rows per
// field, row stride n): F = A^{-1} r, written to dst.  For periodic lines the
// Sherman-Morrison factor of each line goes to fct (the caller subtracts
// fct z_i).  One workgroup of NWV waves per (line, field); grid = 3 * nlines;
// dynamic LDS of (n + (n >> lg) + 1) elements.  The right-hand side is formed
// and the result written in coalesced passes over the line; the recurrences
// run on LDS in chunks of 2^lg elements per thread.
template <typename T, int N, int NWV>
__global__ __launch_bounds__(64 * NWV) void k_cline(CompactArgs<T> A, CompactLine Le,
                                                    CompactLine Lo, const T* __restrict__ s0,
                                                    const T* __restrict__ s1,
                                                    const T* __restrict__ s2, T* __restrict__ d0,
                                                    T* __restrict__ d1, T* __restrict__ d2,
                                                    double* __restrict__ fct, int n, int nlines,
                                                    int wall, int lg) {
  constexpr int NTH = 64 * NWV;
  extern __shared__ unsigned char smem_raw[];
  T* sd = reinterpret_cast<T*>(smem_raw);
  __shared__ T sWa[NWV], sWb[NWV];
  const int field = (int)blockIdx.x / nlines, line = (int)blockIdx.x - field * nlines;
  const T* src = field == 0 ? s0 : field == 1 ? s1 : s2;
  T* out = field == 0 ? d0 : field == 1 ? d1 : d2;
  const bool odd = field != 0;
  const CompactLine L = odd ? Lo : Le;
  const long long b = (long long)line * n;
  const int t = (int)threadIdx.x;
  const int m = 1 << lg;
  const int i0 = t * m < n ? t * m : n, i1 = (t + 1) * m < n ? (t + 1) * m : n;
  T ah[N + 1];
#pragma unroll
  for (int k = 0; k <= N; ++k) ah[k] = T(A.a[k] / 2.0);
  const T al = T(A.alpha);
  // the raw line into LDS in one coalesced pass; then the right-hand side of
  // each element from LDS, held in registers until every thread has read the
  // raw values it needs, and written over them
  for (int e = t; e < n; e += NTH) sd[cpad(e, lg)] = src[b + e];
  __syncthreads();
  auto raw = [&](int i) {
    int flip = 0;
    const int k = map_idx(i, n, wall, flip);
    const T v = sd[cpad(k, lg)];
    return (odd && flip) ? -v : v;
  };
  constexpr int EPT = (COMPACT_MAX_N + NTH - 1) / NTH;
  T rr[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int e = t + j * NTH;
    if (e < n) {
      T r;
      if (e >= N && e < n - N) {
        r = ah[0] * (sd[cpad(e, lg)] + sd[cpad(e, lg)]);
#pragma unroll
        for (int k = 1; k <= N; ++k) r = r + ah[k] * (sd[cpad(e + k, lg)] + sd[cpad(e - k, lg)]);
      } else {
        r = ah[0] * (raw(e) + raw(e));
#pragma unroll
        for (int k = 1; k <= N; ++k) r = r + ah[k] * (raw(e + k) + raw(e - k));
      }
      rr[j] = r;
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int e = t + j * NTH;
    if (e < n) sd[cpad(e, lg)] = rr[j];
  }
  __syncthreads();
  // forward sweep: compose, scan, replay (d_i in place of r_i); the replay also
  // composes the chunk's backward map, in forward order G <- G o (y -> d_i - c'_i y)
  Aff<T> M{T(1), T(0)};
  for (int i = i0; i < i1; ++i) {
    const T inv = cl_inv<T>(L, i, n);
    M = aff_after(Aff<T>{-(al * inv), sd[cpad(i, lg)] * inv}, M);
  }
  T d = block_carry<T, true, NWV>(M, sWa, sWb);
  Aff<T> Mb{T(1), T(0)};
  for (int i = i0; i < i1; ++i) {
    const int o = cpad(i, lg);
    d = (sd[o] - al * d) * cl_inv<T>(L, i, n);
    sd[o] = d;
    Mb = Aff<T>{-(Mb.a * cl_cp<T>(L, i, n)), Mb.a * d + Mb.b};
  }
  // backward sweep: scan from the last thread, replay
  T y = block_carry<T, false, NWV>(Mb, sWa, sWb);
  for (int i = i1 - 1; i >= i0; --i) {
    const int o = cpad(i, lg);
    y = sd[o] - cl_cp<T>(L, i, n) * y;
    sd[o] = y;
  }
  __syncthreads();
  for (int e = t; e < n; e += NTH) out[b + e] = sd[cpad(e, lg)];
  if (L.cyclic && t == 0) {
    // Sherman-Morrison: x = y - (y_0 + fac y_{n-1}) / den * z, one factor per line
    const T y0 = sd[cpad(0, lg)], yl = sd[cpad(n - 1, lg)];
    fct[(long long)field * nlines + line] = double((y0 + T(L.fac) * yl) / T(L.den));
  }
}

// y-lines and the update.  A workgroup takes CW adjacent columns: lane l of a
// wave works on column l mod CW and chunk slot l / CW, so a wave's loads are
// 64 / CW row segments of CW consecutive values, and the NW waves together
// split each column into NW * 64 / CW chunks.  Three passes per chunk:
//   1. compose the forward map of the chunk (right-hand side from a sliding
//      window of 2N+1 values per column);
//   2. with the carry from the chunks above (through LDS), replay: d to a
//      scratch plane, and compose the chunk's backward map on the way (in
//      forward order, G <- G o (y -> d_i - c'_i y));
//   3. with the carry from the chunks below, replay backward and write
//      chi~ = chi - a [(chi - F_x) + (chi - F_y)] directly, both directions'
//      Sherman-Morrison corrections applied: y_0 and y_{n-1}, which the
//      correction needs, are known once the backward carries are.
// grid = (column blocks, 3).
template <typename T, int N, int NW, int CW>
__global__ __launch_bounds__(64 * NW) void k_cline_y(KParams<T> P, CompactArgs<T> A,
                                                     const T* __restrict__ c0,
                                                     const T* __restrict__ c1,
                                                     const T* __restrict__ c2,
                                                     const T* __restrict__ fx, T* __restrict__ scr,
                                                     const double* __restrict__ fctx,
                                                     T* __restrict__ o0, T* __restrict__ o1,
                                                     T* __restrict__ o2) {
  static_assert(CW == 16 || CW == 32 || CW == 64, "column block of 16, 32 or 64");
  constexpr int S = 64 / CW, NCH = NW * S;
  __shared__ T sA[NCH][CW], sB[NCH][CW];
  __shared__ T sY0[CW], sYl[CW];
  const int f = (int)blockIdx.y;
  const bool odd = f != 0;
  const T* src = f == 0 ? c0 : f == 1 ? c1 : c2;
  T* dst = f == 0 ? o0 : f == 1 ? o1 : o2;
  T* sc = scr + (long long)f * P.ps;
  const T* fxf = fx + (long long)f * P.ps;
  const CompactLine L = odd ? A.line[1][1] : A.line[1][0];
  const CompactLine Lx = odd ? A.line[0][1] : A.line[0][0];
  const int nx = P.nx, n = P.ny;
  const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
  const int col = lane % CW, q = w * S + lane / CW;   // column in the block, chunk
  const int x = (int)blockIdx.x * CW + col;
  const bool live = x < nx;
  // idle lanes (beyond the last column) read a real column and write nothing
  const int xs = live ? x : nx - 1;
  const int m = (n + NCH - 1) / NCH;
  const int i0 = q * m < n ? q * m : n, i1 = (q + 1) * m < n ? (q + 1) * m : n;
  T ah[N + 1];
#pragma unroll
  for (int k = 0; k <= N; ++k) ah[k] = T(A.a[k] / 2.0);
  const T al = T(A.alpha);
  // window[k] = chi(x, i + k - N)
  T win[2 * N + 1];
  auto load_win = [&](int i) {
#pragma unroll
    for (int k = 0; k < 2 * N + 1; ++k) win[k] = line_val<T>(src, xs, nx, i + k - N, n, P.wy, odd);
  };
  auto rhs = [&]() {
    T r = ah[0] * (win[N] + win[N]);
#pragma unroll
    for (int k = 1; k <= N; ++k) r = r + ah[k] * (win[N + k] + win[N - k]);
    return r;
  };
  // The serial passes take the next CB values of each operand in one batch of
  // independent loads, so that their latency is paid once per batch.
  constexpr int CB = 8;
  // 1. forward map of the chunk
  Aff<T> M{T(1), T(0)};
  if (i0 < i1) load_win(i0);
  for (int base = i0; base < i1; base += CB) {
    T nv[CB];
#pragma unroll
    for (int j = 0; j < CB; ++j) nv[j] = line_val<T>(src, xs, nx, base + j + 1 + N, n, P.wy, odd);
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      if (base + j < i1) {
        const T inv = cl_inv<T>(L, base + j, n);
        M = aff_after(Aff<T>{-(al * inv), rhs() * inv}, M);
#pragma unroll
        for (int k = 0; k < 2 * N; ++k) win[k] = win[k + 1];
        win[2 * N] = nv[j];
      }
    }
  }
  sA[q][col] = M.a;
  sB[q][col] = M.b;
  __syncthreads();
  T d = T(0);
  for (int k = 0; k < q; ++k) d = sA[k][col] * d + sB[k][col];
  __syncthreads();
  // 2. forward replay, backward map of the chunk
  Aff<T> G{T(1), T(0)};
  if (i0 < i1) load_win(i0);
  for (int base = i0; base < i1; base += CB) {
    T nv[CB];
#pragma unroll
    for (int j = 0; j < CB; ++j) nv[j] = line_val<T>(src, xs, nx, base + j + 1 + N, n, P.wy, odd);
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      if (base + j < i1) {
        d = (rhs() - al * d) * cl_inv<T>(L, base + j, n);
        if (live) sc[(long long)(base + j) * nx + xs] = d;
        G = Aff<T>{-(G.a * cl_cp<T>(L, base + j, n)), G.a * d + G.b};
#pragma unroll
        for (int k = 0; k < 2 * N; ++k) win[k] = win[k + 1];
        win[2 * N] = nv[j];
      }
    }
  }
  sA[q][col] = G.a;
  sB[q][col] = G.b;
  __syncthreads();
  T y = T(0);
  for (int k = NCH - 1; k > q; --k) y = sA[k][col] * y + sB[k][col];
  // y_{n-1} and y_0 of the column, from the chunks that hold them
  if (i0 < i1 && i1 == n) sYl[col] = d - cl_cp<T>(L, n - 1, n) * y;
  if (i0 == 0 && i1 > 0) sY0[col] = G.a * y + G.b;
  __syncthreads();
  T fct = T(0);
  if (L.cyclic) fct = (sY0[col] + T(L.fac) * sYl[col]) / T(L.den);
  if (!live) return;
  // 3. backward replay and the update
  const T a = P.fa;
  const double* fcx = fctx + (long long)f * n;
  for (int top = i1 - 1; top >= i0; top -= CB) {
    T v[CB], ch[CB], fv[CB];
#pragma unroll
    for (int j = 0; j < CB; ++j)
      if (top - j >= i0) {
        const long long o = (long long)(top - j) * nx + x;
        v[j] = sc[o];
        ch[j] = src[o];
        fv[j] = fxf[o];
      }
#pragma unroll
    for (int j = 0; j < CB; ++j)
      if (top - j >= i0) {
        const int i = top - j;
        y = v[j] - cl_cp<T>(L, i, n) * y;
        T fy = y;
        if (L.cyclic) fy = fy - fct * T(L.z[i]);
        T fxv = fv[j];
        if (Lx.cyclic) fxv = fxv - T(fcx[i]) * T(Lx.z[x]);
        dst[(long long)i * nx + x] = ch[j] - a * ((ch[j] - fxv) + (ch[j] - fy));
      }
  }
}

}  // namespace lbm2p
