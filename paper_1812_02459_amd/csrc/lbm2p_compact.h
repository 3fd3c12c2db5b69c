// Compact (tridiagonal) selective filter -- the variant named in the paper's
// abstract and conclusions (whose explicit filter is eq:filter).  Per line:
//   alpha F_{i-1} + F_i + alpha F_{i+1} = sum_{n=0..N} (a_n / 2)(chi_{i+n} + chi_{i-n})
// and the field update keeps eq:filter's unsplit form and intensity a:
//   chi~ = chi - a [ (chi - F_x chi) + (chi - F_y chi) ].
// The a_n solve T(0) = 1, T(pi) = 0 and the flatness conditions of the transfer
// function T(w) = sum a_n cos(n w) / (1 + 2 alpha cos w) (host side, lbm2p.hip).
//
// Lines are solved with the Thomas algorithm on tables precomputed on the host
// for the constant-coefficient matrix (c'_i and 1/pivot_i); a periodic line is
// the cyclic matrix, solved by Sherman-Morrison with a precomputed correction
// vector z.  Beyond a wall the right-hand side uses the half-way mirror ghosts
// (sign kept for p, flipped for u) and the matrix's end rows fold the ghost
// F_{-1} = +-F_0 into the diagonal.  One thread per (line, field); the right-hand
// side comes from a sliding window of 2N+1 values held in registers.
#pragma once

#include "lbm2p_kernels.h"

namespace lbm2p {

// Table layout per (axis, parity): cp[n] (c'), inv[n] (1/pivot), z[n] (cyclic
// correction, periodic lines only), then scalar vz = v.z denominators folded in
// by the host: fac = beta/gamma, den = 1 + z_0 + fac z_{n-1}.
struct CompactLine {
  const double* cp;
  const double* inv;
  const double* z;
  double fac, den;
  int cyclic;
};

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

// One line solve: F = A^{-1} r for the line through base b with stride s.
// Writes F into out (same indexing).  Scratch d holds the forward sweep.
template <typename T, int N>
__device__ __forceinline__ void compact_line(const T* __restrict__ f, T* __restrict__ d,
                                             T* __restrict__ out, long long b, long long s, int n,
                                             int wall, bool odd, const CompactArgs<T>& A,
                                             const CompactLine& L) {
  T w[2 * N + 1];
#pragma unroll
  for (int k = 0; k < 2 * N + 1; ++k) w[k] = line_val<T>(f, b, s, k - N, n, wall, odd);
  T a[N + 1];
#pragma unroll
  for (int k = 0; k <= N; ++k) a[k] = T(A.a[k] / 2.0);
  const T al = T(A.alpha);
  T prev = T(0);
  for (int i = 0; i < n; ++i) {
    // right-hand side at i from the window w[k] = chi_{i + k - N}
    T r = a[0] * (w[N] + w[N]);
#pragma unroll
    for (int k = 1; k <= N; ++k) r = r + a[k] * (w[N + k] + w[N - k]);
    const T di = (i == 0 ? r : r - al * prev) * T(L.inv[i]);
    d[b + s * i] = di;
    prev = di;
#pragma unroll
    for (int k = 0; k < 2 * N; ++k) w[k] = w[k + 1];
    w[2 * N] = line_val<T>(f, b, s, i + N + 1, n, wall, odd);
  }
  // back substitution; y_{n-1} = d_{n-1}
  T y = prev;
  out[b + s * (n - 1)] = y;
  const T ylast = y;
  for (int i = n - 2; i >= 0; --i) {
    y = d[b + s * i] - T(L.cp[i]) * y;
    out[b + s * i] = y;
  }
  if (L.cyclic) {
    // Sherman-Morrison: x = y - (y_0 + fac y_{n-1}) / den * z
    const T fct = (y + T(L.fac) * ylast) / T(L.den);
    for (int i = 0; i < n; ++i) out[b + s * i] = out[b + s * i] - fct * T(L.z[i]);
  }
}

// x-lines of the three fields: Fx of (p, ux, uy) into fx[0..2]
template <typename T, int N>
__global__ __launch_bounds__(64) void k_compact_x(KParams<T> P, CompactArgs<T> A,
                                                  const T* __restrict__ p, const T* __restrict__ ux,
                                                  const T* __restrict__ uy, T* __restrict__ d,
                                                  T* __restrict__ fx) {
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t >= 3 * P.ny) return;
  const int field = t / P.ny, y = t - field * P.ny;
  const T* src = field == 0 ? p : field == 1 ? ux : uy;
  const bool odd = field != 0;
  const long long b = (long long)y * P.nx;
  compact_line<T, N>(src, d + field * P.ps, fx + field * P.ps, b, 1, P.nx, P.wx, odd, A,
                     A.line[0][odd ? 1 : 0]);
}

// y-lines, then the unsplit update chi - a [(chi - Fx) + (chi - Fy)]
template <typename T, int N>
__global__ __launch_bounds__(64) void k_compact_y(KParams<T> P, CompactArgs<T> A,
                                                  const T* __restrict__ p, const T* __restrict__ ux,
                                                  const T* __restrict__ uy, T* __restrict__ d,
                                                  const T* __restrict__ fx, T* __restrict__ fy,
                                                  T* __restrict__ po, T* __restrict__ uxo,
                                                  T* __restrict__ uyo) {
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t >= 3 * P.nx) return;
  const int field = t / P.nx, x = t - field * P.nx;
  const T* src = field == 0 ? p : field == 1 ? ux : uy;
  T* dst = field == 0 ? po : field == 1 ? uxo : uyo;
  const bool odd = field != 0;
  T* fyf = fy + field * P.ps;
  const T* fxf = fx + field * P.ps;
  compact_line<T, N>(src, d + field * P.ps, fyf, x, P.nx, P.ny, P.wy, odd, A,
                     A.line[1][odd ? 1 : 0]);
  const T a = P.fa;
  for (int y = 0; y < P.ny; ++y) {
    const long long id = (long long)y * P.nx + x;
    const T c = src[id];
    dst[id] = c - a * ((c - fxf[id]) + (c - fyf[id]));
  }
}

}  // namespace lbm2p
