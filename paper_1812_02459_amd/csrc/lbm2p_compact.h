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
// y_i = -c'_i y_{i+1} + d_i.  Every thread owns a chunk of consecutive
// elements of a line, held in registers: it forms the chunk's right-hand side,
// composes the chunk's affine maps, and -- once the values entering the chunk
// from its neighbours are known -- replays the chunk.  x-lines: a workgroup
// per line, the carries from a scan over its threads (lane shuffles, then
// LDS across waves).  y-lines: lanes take adjacent columns (coalesced rows),
// and the carries come from a scan over the chunk maps of each column in a
// launch of their own.  The periodic lines' Sherman-Morrison correction
// x_i = y_i - f z_i is applied before F is used.
#pragma once

#include "lbm2p_kernels.h"

namespace lbm2p {

// Tables per (axis, parity), in the kernels' precision (rounded once from the
// host's FP64 factorisation): cp[n] (c'), inv[n] (1/pivot), z[n] (cyclic
// correction, periodic lines only), and the scalars fac = beta/gamma,
// den = 1 + z_0 + fac z_{n-1} of the Sherman-Morrison denominator.  c' and
// 1/pivot are constant (cp_lim, inv_lim) for K <= i <= n - 2; z decays from
// both ends, and |z_i| <= 1e-30 max|z| for Z0 <= i < Z1, where the correction
// f z_i is dropped (a change below 1e-30 of the line's largest value).
template <typename T>
struct CompactLine {
  const T* cp;
  const T* inv;
  const T* z;
  T fac, den;
  int cyclic;
  int K, Z0, Z1;
  T cp_lim, inv_lim;
};

template <typename T>
struct CompactArgs {
  double a[6];          // a_0 .. a_N
  double alpha;
  CompactLine<T> line[2][2];  // [axis 0 = x, 1 = y][parity 0 = even, 1 = odd]
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

// x-lines.  One workgroup of NT threads per (line, field); thread t owns the
// chunk [t M, t M + M) of the line (n <= NT M).  The line, extended by N ghost
// values on each side (wrap or mirror), is staged in LDS in one coalesced pass
// with one pad word per M elements, so that the lanes reading their chunks in
// step hit distinct banks; each thread then holds its chunk and its 2N
// neighbours in registers and forms the right-hand side in place.  Forward
// map, carry (block_carry), replay with d kept in registers while the backward
// map is composed, carry, backward replay; y_0 and y_{n-1} pass through LDS for
// the cyclic correction, and F_x goes back through LDS to a coalesced store
// (each thread storing its own chunk, 32 bytes apart across lanes, measured
// 1.5x slower).
// Chunks inside the tables' constant run take cp_lim, inv_lim; the others
// load their entries in one batch (no load waits inside the recurrences).
template <typename T, int N, int NT, int M>
__global__ __launch_bounds__(NT) void k_cx(CompactArgs<T> A, const T* __restrict__ s0,
                                           const T* __restrict__ s1, const T* __restrict__ s2,
                                           T* __restrict__ d0, T* __restrict__ d1,
                                           T* __restrict__ d2, int n, int nlines, int wall) {
  constexpr int NWV = NT / 64, E = M + 2 * N;
  extern __shared__ unsigned char smem_raw[];
  T* sd = reinterpret_cast<T*>(smem_raw);
  __shared__ T sWa[NWV], sWb[NWV], sY[2];
  const int field = (int)blockIdx.x / nlines, line = (int)blockIdx.x - field * nlines;
  const T* src = field == 0 ? s0 : field == 1 ? s1 : s2;
  T* out = field == 0 ? d0 : field == 1 ? d1 : d2;
  const bool odd = field != 0;
  const CompactLine<T> L = A.line[0][odd ? 1 : 0];
  const long long b = (long long)line * n;
  const int t = (int)threadIdx.x;
  auto pos = [](int e) { return e + e / M; };
  // the extended line: element e holds chi(e - N); every thread's loads are
  // issued before its LDS stores (one load latency, not one per element), the
  // ghost indices mapped without a branch around the load
  constexpr int LPT = (NT * M + 2 * N + NT - 1) / NT;
  T lv[LPT];
#pragma unroll
  for (int q = 0; q < LPT; ++q) {
    const int i = t + q * NT - N;
    int flip = 0;
    const int k = map_idx(i, n, wall, flip);
    const T w = src[b + k];
    lv[q] = (odd && flip) ? -w : w;
  }
#pragma unroll
  for (int q = 0; q < LPT; ++q) {
    const int e = t + q * NT;
    if (e < n + 2 * N) sd[pos(e)] = lv[q];
  }
  const int i0 = t * M;
  const int m = n - i0 <= 0 ? 0 : (n - i0 < M ? n - i0 : M);   // elements of this chunk
  T ti[M], tc[M], tz[M];
  // the cyclic correction's z where it is kept (chunks near the line's ends)
  const bool zk = L.cyclic && m > 0 && (i0 < L.Z0 || i0 + M > L.Z1);
  if (zk) {
#pragma unroll
    for (int k = 0; k < M; ++k) tz[k] = L.z[i0 + k < n ? i0 + k : n - 1];
  }
  if (i0 >= L.K && i0 + M <= n - 1) {
#pragma unroll
    for (int k = 0; k < M; ++k) {
      ti[k] = L.inv_lim;
      tc[k] = L.cp_lim;
    }
  } else {
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const int i = i0 + k < n ? i0 + k : n - 1;
      ti[k] = L.inv[i];
      tc[k] = L.cp[i];
    }
  }
  __syncthreads();
  T v[E];
#pragma unroll
  for (int k = 0; k < E; ++k) v[k] = sd[pos(i0 + k)];
  T ah[N + 1];
#pragma unroll
  for (int k = 0; k <= N; ++k) ah[k] = T(A.a[k] / 2.0);
  const T al = T(A.alpha);
  // right-hand side in place: r_k needs v[k .. k + 2N], and v[k] no later r
#pragma unroll
  for (int k = 0; k < M; ++k) {
    T r = ah[0] * (v[k + N] + v[k + N]);
#pragma unroll
    for (int j = 1; j <= N; ++j) r = r + ah[j] * (v[k + N + j] + v[k + N - j]);
    v[k] = r;
  }
  Aff<T> Mf{T(1), T(0)};
#pragma unroll
  for (int k = 0; k < M; ++k)
    if (k < m) Mf = aff_after(Aff<T>{-(al * ti[k]), v[k] * ti[k]}, Mf);
  T d = block_carry<T, true, NWV>(Mf, sWa, sWb);
  // forward replay (d over r), composing the backward map in forward order,
  // G <- G o (y -> d_i - c'_i y)
  Aff<T> Mb{T(1), T(0)};
#pragma unroll
  for (int k = 0; k < M; ++k)
    if (k < m) {
      d = (v[k] - al * d) * ti[k];
      v[k] = d;
      Mb = Aff<T>{-(Mb.a * tc[k]), Mb.a * d + Mb.b};
    }
  T y = block_carry<T, false, NWV>(Mb, sWa, sWb);
#pragma unroll
  for (int k = M - 1; k >= 0; --k)
    if (k < m) {
      y = v[k] - tc[k] * y;
      v[k] = y;
    }
  if (L.cyclic) {
    // Sherman-Morrison: x = y - (y_0 + fac y_{n-1}) / den * z
#pragma unroll
    for (int k = 0; k < M; ++k) {
      if (k == 0 && i0 == 0) sY[0] = v[k];
      if (k < m && i0 + k == n - 1) sY[1] = v[k];
    }
    __syncthreads();
    const T fc = (sY[0] + L.fac * sY[1]) / L.den;
    if (zk) {
#pragma unroll
      for (int k = 0; k < M; ++k) v[k] = v[k] - fc * tz[k];
    }
  }
  __syncthreads();   // every read of the staged line is done
#pragma unroll
  for (int k = 0; k < M; ++k)
    if (k < m) sd[pos(i0 + k)] = v[k];
  __syncthreads();
  for (int e = t; e < n; e += NT) out[b + e] = sd[pos(e)];
}

// LDS of k_cx: the extended line (NT M + 2N elements) with one pad per M
template <typename T, int N, int NT, int M>
constexpr size_t cx_lds() {
  return ((size_t)(NT * M + 2 * N) + (size_t)(NT * M + 2 * N) / M + 1) * sizeof(T);
}

// y-lines, in three launches over chunks of MY rows of one column: a
// workgroup takes one chunk row range of 256 adjacent columns (lane = column,
// so that every row of a chunk is read and written as coalesced row segments;
// the chunk, and with it the table entries, is the same for the whole
// workgroup and staged once in LDS).
//   k_cy_maps: the chunk's right-hand side (its rows and N ghost rows on each
//     side) and the coefficients of its forward map d_out = Af d_in + Bf and
//     of the solution at its first row, y_top = Sa d_in + Sb + W y_in (y_in:
//     the solution at the row after the chunk): with d_k = a_k d_in + b_k and
//     w_k = prod_{j<k} (-c'_j), W = w_MY, Sa = sum w_k a_k, Sb = sum w_k b_k;
//   k_cy_scan: per column, the carries d_in and y_in of every chunk and the
//     column's cyclic correction factor;
//   k_cy_apply: the chunk replayed with its carries, corrected, and the update
//     chi~ = chi - a [(chi - F_x) + (chi - F_y)] written.
// Scratch per field: 7 planes of nch x nx (Af, Bf, W, Sa, Sb, d_in, y_in), then
// the factors of the three fields (3 nx).
enum { CY_AF, CY_BF, CY_W, CY_SA, CY_SB, CY_DIN, CY_YIN, CY_PLANES };

// a chunk's rows i0 - N .. i0 + MY + N - 1 of column x (ghosts by wrap or
// mirror); with CH, the chunk's own rows also to ch; the right-hand side in
// place in v[0 .. MY)
template <typename T, int N, int MY, bool CH>
__device__ __forceinline__ void cy_load_rhs(const T* __restrict__ src, int xs, int nx, int n,
                                            int i0, int m, int wall, bool odd,
                                            const CompactArgs<T>& A, T* v, T* ch) {
  constexpr int E = MY + 2 * N;
  if (i0 - N >= 0 && i0 + MY + N <= n) {
    const T* __restrict__ col = src + (long long)(i0 - N) * nx + xs;
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = col[(long long)k * nx];
  } else {
#pragma unroll
    for (int k = 0; k < E; ++k)
      v[k] = k < m + 2 * N ? line_val<T>(src, xs, nx, i0 - N + k, n, wall, odd) : T(0);
  }
  if constexpr (CH) {
#pragma unroll
    for (int k = 0; k < MY; ++k) ch[k] = v[k + N];
  }
  T ah[N + 1];
#pragma unroll
  for (int k = 0; k <= N; ++k) ah[k] = T(A.a[k] / 2.0);
#pragma unroll
  for (int k = 0; k < MY; ++k) {
    T r = ah[0] * (v[k + N] + v[k + N]);
#pragma unroll
    for (int j = 1; j <= N; ++j) r = r + ah[j] * (v[k + N + j] + v[k + N - j]);
    v[k] = r;
  }
}

// the chunk's table entries (1/pivot, c', and z where it is kept) into LDS
template <typename T, int MY>
__device__ __forceinline__ void cy_tables(const CompactLine<T>& L, int i0, int n, T* sI, T* sC,
                                          T* sZ) {
  const int k = (int)threadIdx.x;
  if (k < MY) {
    const int i = i0 + k < n ? i0 + k : n - 1;
    const bool flat = i0 >= L.K && i0 + MY <= n - 1;
    sI[k] = flat ? L.inv_lim : L.inv[i];
    sC[k] = flat ? L.cp_lim : L.cp[i];
    if (sZ) sZ[k] = (L.cyclic && (i0 < L.Z0 || i0 + MY > L.Z1)) ? L.z[i] : T(0);
  }
  __syncthreads();
}

template <typename T, int N, int MY>
__global__ __launch_bounds__(256) void k_cy_maps(KParams<T> P, CompactArgs<T> A,
                                                 const T* __restrict__ c0,
                                                 const T* __restrict__ c1,
                                                 const T* __restrict__ c2, T* __restrict__ coef,
                                                 int nch) {
  __shared__ T sI[MY], sC[MY];
  const int f = (int)blockIdx.z;
  const bool odd = f != 0;
  const T* src = f == 0 ? c0 : f == 1 ? c1 : c2;
  const CompactLine<T> L = A.line[1][odd ? 1 : 0];
  const int nx = P.nx, n = P.ny;
  const int x = (int)blockIdx.x * 256 + (int)threadIdx.x, c = (int)blockIdx.y;
  const bool live = x < nx;
  const int xs = live ? x : nx - 1;
  const int i0 = c * MY, m = n - i0 < MY ? n - i0 : MY;
  cy_tables<T, MY>(L, i0, n, sI, sC, nullptr);
  T v[MY + 2 * N];
  cy_load_rhs<T, N, MY, false>(src, xs, nx, n, i0, m, P.wy, odd, A, v, nullptr);
  const T al = T(A.alpha);
  T a = T(1), bb = T(0), wk = T(1), Sa = T(0), Sb = T(0);
#pragma unroll
  for (int k = 0; k < MY; ++k)
    if (k < m) {
      const T g = -(al * sI[k]);
      a = g * a;
      bb = g * bb + v[k] * sI[k];
      Sa = Sa + wk * a;
      Sb = Sb + wk * bb;
      wk = -(sC[k] * wk);
    }
  if (!live) return;
  const long long ps = (long long)nch * nx;
  T* base = coef + (long long)f * CY_PLANES * ps + (long long)c * nx + x;
  base[CY_AF * ps] = a;
  base[CY_BF * ps] = bb;
  base[CY_W * ps] = wk;
  base[CY_SA * ps] = Sa;
  base[CY_SB * ps] = Sb;
}

// Carries of every chunk of a column.  A workgroup takes 64 columns (lane =
// column) and NW waves; wave w owns the consecutive chunks [w G, w G + G) of
// each column (G = ceil(nch / NW)), composes their maps, and the waves'
// composites pass through LDS.  Forward: d_in of each chunk; then, with d_in
// known, the backward values y_top = W y_in + (Sa d_in + Sb) are affine maps of
// y_in, scanned the same way from the last chunk.  y_0 = y_top of chunk 0 and
// y_{n-1} = d_out of the last chunk give the cyclic factor.
template <typename T, int NW>
__global__ __launch_bounds__(64 * NW) void k_cy_scan(KParams<T> P, CompactArgs<T> A,
                                                     T* __restrict__ coef, T* __restrict__ fct,
                                                     int nch) {
  __shared__ T sA[NW][64], sB[NW][64], sY[2][64];
  const int f = (int)blockIdx.y;
  const CompactLine<T> L = A.line[1][f != 0 ? 1 : 0];
  const int nx = P.nx;
  const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
  const int x = (int)blockIdx.x * 64 + lane;
  const bool live = x < nx;
  const int xs = live ? x : nx - 1;
  const int G = (nch + NW - 1) / NW;
  const int c0 = w * G < nch ? w * G : nch, c1 = (w + 1) * G < nch ? (w + 1) * G : nch;
  const long long ps = (long long)nch * nx;
  T* base = coef + (long long)f * CY_PLANES * ps + xs;
  auto at = [&](int plane, int c) -> T& { return base[plane * ps + (long long)c * nx]; };
  // the chunks in batches of CB, every batch's loads issued together (the
  // carries are serial, the coefficients are not)
  constexpr int CB = 8;
  // forward: this wave's composite, the carry from the waves before, replay
  T ca = T(1), cb = T(0);
  for (int c = c0; c < c1; c += CB) {
    T fa[CB], fb[CB];
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int cc = c + j < c1 ? c + j : c1 - 1;
      fa[j] = at(CY_AF, cc);
      fb[j] = at(CY_BF, cc);
    }
#pragma unroll
    for (int j = 0; j < CB; ++j)
      if (c + j < c1) {
        cb = fa[j] * cb + fb[j];
        ca = fa[j] * ca;
      }
  }
  sA[w][lane] = ca;
  sB[w][lane] = cb;
  __syncthreads();
  T d = T(0);
  for (int k = 0; k < w; ++k) d = sA[k][lane] * d + sB[k][lane];
  for (int c = c0; c < c1; c += CB) {
    T fa[CB], fb[CB], sa[CB], sb[CB];
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int cc = c + j < c1 ? c + j : c1 - 1;
      fa[j] = at(CY_AF, cc);
      fb[j] = at(CY_BF, cc);
      sa[j] = at(CY_SA, cc);
      sb[j] = at(CY_SB, cc);
    }
#pragma unroll
    for (int j = 0; j < CB; ++j)
      if (c + j < c1 && live) {
        // d_in, and this chunk's backward map y_top = W y_in + (Sa d_in + Sb):
        // the constant term over Sb (each thread rewrites only its own chunks)
        at(CY_DIN, c + j) = d;
        at(CY_SB, c + j) = sa[j] * d + sb[j];
        d = fa[j] * d + fb[j];
      } else if (c + j < c1) {
        d = fa[j] * d + fb[j];
      }
  }
  if (c0 < c1 && c1 == nch) sY[1][lane] = d;   // y_{n-1} = d_{n-1}
  __syncthreads();
  // backward: composite over this wave's chunks (last to first)
  ca = T(1);
  cb = T(0);
  for (int c = c1 - 1; c >= c0; c -= CB) {
    T ww[CB], sv[CB];
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int cc = c - j >= c0 ? c - j : c0;
      ww[j] = at(CY_W, cc);
      sv[j] = at(CY_SB, cc);
    }
#pragma unroll
    for (int j = 0; j < CB; ++j)
      if (c - j >= c0) {
        cb = ww[j] * cb + sv[j];
        ca = ww[j] * ca;
      }
  }
  sA[w][lane] = ca;
  sB[w][lane] = cb;
  __syncthreads();
  T y = T(0);
  for (int k = NW - 1; k > w; --k) y = sA[k][lane] * y + sB[k][lane];
  for (int c = c1 - 1; c >= c0; c -= CB) {
    T ww[CB], sv[CB];
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      const int cc = c - j >= c0 ? c - j : c0;
      ww[j] = at(CY_W, cc);
      sv[j] = at(CY_SB, cc);
    }
#pragma unroll
    for (int j = 0; j < CB; ++j)
      if (c - j >= c0) {
        if (live) at(CY_YIN, c - j) = y;
        y = ww[j] * y + sv[j];
      }
  }
  if (c0 == 0 && c1 > 0) sY[0][lane] = y;   // y_0
  __syncthreads();
  if (live && w == 0) fct[f * nx + x] = L.cyclic ? (sY[0][lane] + L.fac * sY[1][lane]) / L.den : T(0);
}

template <typename T, int N, int MY>
__global__ __launch_bounds__(256) void k_cy_apply(KParams<T> P, CompactArgs<T> A,
                                                  const T* __restrict__ c0,
                                                  const T* __restrict__ c1,
                                                  const T* __restrict__ c2,
                                                  const T* __restrict__ fx,
                                                  const T* __restrict__ coef,
                                                  const T* __restrict__ fct, T* __restrict__ o0,
                                                  T* __restrict__ o1, T* __restrict__ o2,
                                                  int nch) {
  __shared__ T sI[MY], sC[MY], sZ[MY];
  const int f = (int)blockIdx.z;
  const bool odd = f != 0;
  const T* src = f == 0 ? c0 : f == 1 ? c1 : c2;
  T* dst = f == 0 ? o0 : f == 1 ? o1 : o2;
  const T* fxf = fx + (long long)f * P.ps;
  const CompactLine<T> L = A.line[1][odd ? 1 : 0];
  const int nx = P.nx, n = P.ny;
  const int x = (int)blockIdx.x * 256 + (int)threadIdx.x, c = (int)blockIdx.y;
  const bool live = x < nx;
  const int xs = live ? x : nx - 1;
  const int i0 = c * MY, m = n - i0 < MY ? n - i0 : MY;
  cy_tables<T, MY>(L, i0, n, sI, sC, sZ);
  // F_x of the chunk's rows, loaded ahead of the recurrences
  T fxv[MY];
  {
    const T* __restrict__ fcol = fxf + xs;
#pragma unroll
    for (int k = 0; k < MY; ++k) fxv[k] = fcol[(long long)(i0 + k < n ? i0 + k : n - 1) * nx];
  }
  T v[MY + 2 * N], ch[MY];
  cy_load_rhs<T, N, MY, true>(src, xs, nx, n, i0, m, P.wy, odd, A, v, ch);
  const long long ps = (long long)nch * nx;
  const T* base = coef + (long long)f * CY_PLANES * ps + (long long)c * nx + xs;
  T d = base[CY_DIN * ps];
  T y = base[CY_YIN * ps];
  const T fc = fct[f * nx + xs];
  const T al = T(A.alpha);
#pragma unroll
  for (int k = 0; k < MY; ++k)
    if (k < m) {
      d = (v[k] - al * d) * sI[k];
      v[k] = d;
    }
#pragma unroll
  for (int k = MY - 1; k >= 0; --k)
    if (k < m) {
      y = v[k] - sC[k] * y;
      v[k] = y;
    }
  if (!live) return;
  const T a = P.fa;
  T* __restrict__ dcol = dst + (long long)i0 * nx + x;
#pragma unroll
  for (int k = 0; k < MY; ++k)
    if (k < m) {
      const T fy = v[k] - fc * sZ[k];
      dcol[(long long)k * nx] = ch[k] - a * ((ch[k] - fxv[k]) + (ch[k] - fy));
    }
}

}  // namespace lbm2p
