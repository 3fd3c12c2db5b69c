// Pointwise and stencil arithmetic of the fractional-step MRT-LBM
// (arXiv:1812.02459), device side.
//
// Every expression is written with a fixed evaluation order and the library is
// compiled with -ffp-contract=off, so the FP64 path rounds exactly as the
// written formula does.  Divisions by c_s^2 = 1/3 are multiplications by 3,
// divisions by c_s^4 multiplications by 9 (exact constants).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace lbm2p {

// Quotients.  FP64 divides (correctly rounded, as the FP64 formulas are
// written).  FP32 multiplies by a reciprocal: a constant divisor's reciprocal
// is rounded once at compile time, a variable one comes from the hardware
// reciprocal (1 ulp), so an FP32 quotient is within about 2 ulp -- no worse
// than the 2.5 ulp division the FP32 build would otherwise emit, at a fifth of
// its instructions.  Divisors here are densities, |grad phi|_eps >= eps, the
// interface width and small integer constants: never zero or subnormal.
template <typename T>
__device__ __forceinline__ T qdiv(T a, T b) {
  if constexpr (std::is_same<T, float>::value) return a * __builtin_amdgcn_rcpf(b);
  else return a / b;
}
// FP64 quotient a / b from y = RN(1/b): q = RN(a y) lies within one ulp of
// a / b, so the remainder a - b q is exact (one FMA) and q + (a - b q) y rounded
// once is the correctly rounded a / b (Markstein's theorem for binary64 with an
// FMA, quotients in the normal range).  Four instructions where the division
// sequence takes eleven, and bitwise the same result.  A zero remainder (q
// exact, including a signed zero) or a non-finite one (infinite or NaN q)
// returns q itself, as a / b would.
__device__ __forceinline__ double div_by(double a, double b, double y) {
  const double q = a * y;
  const double r = fma(-b, q, a);
  return (r != 0.0 && __builtin_isfinite(r)) ? fma(r, y, q) : q;
}
template <int C, typename T>
__device__ __forceinline__ T divk(T a) {
  if constexpr (std::is_same<T, float>::value) return a * float(1.0 / C);
  else return div_by(a, double(C), 1.0 / C);
}

// FP32 a / 3 correctly rounded: q = RN(a RN(1/3)) is within one ulp, the
// remainder a - 3 q is exact (one FMA), q + r RN(1/3) rounds to the nearest
// (the FP32 case of the correction div_by applies in FP64)
__device__ __forceinline__ float div3_rn(float a) {
  const float y = 1.0f / 3.0f;
  const float q = a * y;
  const float r = __builtin_fmaf(-3.0f, q, a);
  return __builtin_fmaf(r, y, q);
}

// eq:D2Q9: c_0 = 0, c_1..4 = axes counter-clockwise from +x, c_5..8 diagonals.
__host__ __device__ constexpr int cx_of(int i) {
  return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0);
}
__host__ __device__ constexpr int cy_of(int i) {
  return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0);
}
// opposite directions, written out: 1<->3, 2<->4, 5<->7, 6<->8
__host__ __device__ constexpr int opp(int i) {
  return i == 1 ? 3 : i == 2 ? 4 : i == 3 ? 1 : i == 4 ? 2 :
         i == 5 ? 7 : i == 6 ? 8 : i == 7 ? 5 : i == 8 ? 6 : 0;
}
// weights: 4/9, 1/9 (axes), 1/36 (diagonals)
__host__ __device__ constexpr double w_of(int i) {
  return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
}
// eq:D2Q9MRT
__host__ __device__ constexpr int mrt(int k, int j) {
  constexpr int Mt[9][9] = {
      {1, 1, 1, 1, 1, 1, 1, 1, 1},
      {-4, -1, -1, -1, -1, 2, 2, 2, 2},
      {4, -2, -2, -2, -2, 1, 1, 1, 1},
      {0, 1, 0, -1, 0, 1, -1, -1, 1},
      {0, -2, 0, 2, 0, 1, -1, -1, 1},
      {0, 0, 1, 0, -1, 1, 1, -1, -1},
      {0, 0, -2, 0, 2, 1, 1, -1, -1},
      {0, 1, -1, 1, -1, 0, 0, 0, 0},
      {0, 0, 0, 0, 0, 1, -1, 1, -1}};
  return Mt[k][j];
}
// 1 / (M M^T)_kk: the rows of M are orthogonal with squared norms 9,36,36,6,12,6,12,4,4
__host__ __device__ constexpr double mm_inv(int k) {
  return k == 0 ? 1.0 / 9.0 : k == 1 || k == 2 ? 1.0 / 36.0 : k == 3 || k == 5 ? 1.0 / 6.0
         : k == 4 || k == 6 ? 1.0 / 12.0 : 1.0 / 4.0;
}

// c_i . a, zero components skipped (c entries are 0 or +-1)
template <typename T>
__device__ __forceinline__ T cdot(int i, T ax, T ay) {
  const int cx = cx_of(i), cy = cy_of(i);
  if (cx == 0 && cy == 0) return T(0);
  if (cy == 0) return cx > 0 ? ax : -ax;
  if (cx == 0) return cy > 0 ? ay : -ay;
  return (cx > 0 ? ax : -ax) + (cy > 0 ? ay : -ay);
}

// m = M v, sums in column order starting from the first non-zero entry
template <typename T>
__device__ __forceinline__ void m_apply(const T v[9], T m[9]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    T acc = T(0);
    bool first = true;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      const int c = mrt(k, j);
      if (c == 0) continue;
      const T t = c == 1 ? v[j] : c == -1 ? -v[j] : T(c) * v[j];
      acc = first ? t : acc + t;
      first = false;
    }
    m[k] = acc;
  }
}

// v = M^{-1} m = M^T diag(1/(M M^T)_kk) m
template <typename T>
__device__ __forceinline__ void minv_apply(const T m[9], T v[9]) {
  T sc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) sc[k] = m[k] * T(mm_inv(k));
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    T acc = T(0);
    bool first = true;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const int c = mrt(k, j);
      if (c == 0) continue;
      const T t = c == 1 ? sc[k] : c == -1 ? -sc[k] : T(c) * sc[k];
      acc = first ? t : acc + t;
      first = false;
    }
    v[j] = acc;
  }
}

// eq:distribution_CH / eq:distribution_NS collision with Lambda = M^-1 S M:
//   f* = f + M^{-1} [ (I - S/2) M F - S M (f - f^eq) ]       (in place on f)
template <typename T>
__device__ __forceinline__ void mrt_collide(T f[9], const T feq[9], const T F[9], const T s[9]) {
  T d[9], md[9], mF[9], r[9], corr[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) d[i] = f[i] - feq[i];
  m_apply(d, md);
  m_apply(F, mF);
#pragma unroll
  for (int k = 0; k < 9; ++k) r[k] = (T(1) - s[k] * T(0.5)) * mF[k] - s[k] * md[k];
  minv_apply(r, corr);
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = f[i] + corr[i];
}

// The same collision with the transforms factorised into sums and differences
// of opposite populations (27 and 30 operations instead of ~55 each) and the
// source given by its moments m_S = M F: f* = f + M^{-1} [ (I - S/2) m_S -
// S M (f - f^eq) ].  Used by the FP32 step, whose rounding order is free; the
// FP64 step keeps mrt_collide's order.
template <typename T>
__device__ __forceinline__ void m_apply_pairs(const T v[9], T m[9]) {
  const T a13 = v[1] + v[3], s13 = v[1] - v[3], a24 = v[2] + v[4], s24 = v[2] - v[4];
  const T a57 = v[5] + v[7], s57 = v[5] - v[7], a68 = v[6] + v[8], s68 = v[6] - v[8];
  const T ax = a13 + a24, dg = a57 + a68, jxd = s57 - s68, jyd = s57 + s68;
  m[0] = (v[0] + ax) + dg;
  m[1] = (T(2) * dg - ax) - T(4) * v[0];
  m[2] = (T(4) * v[0] - T(2) * ax) + dg;
  m[3] = s13 + jxd;
  m[4] = jxd - T(2) * s13;
  m[5] = s24 + jyd;
  m[6] = jyd - T(2) * s24;
  m[7] = a13 - a24;
  m[8] = a57 - a68;
}
template <typename T>
__device__ __forceinline__ void minv_apply_pairs(const T m[9], T v[9]) {
  T c[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) c[k] = m[k] * T(mm_inv(k));
  const T A = (c[0] - c[1]) - T(2) * c[2], D = (c[0] + T(2) * c[1]) + c[2];
  const T X = c[3] - T(2) * c[4], Y = c[5] - T(2) * c[6], Xd = c[3] + c[4], Yd = c[5] + c[6];
  v[0] = (c[0] - T(4) * c[1]) + T(4) * c[2];
  v[1] = (A + X) + c[7];
  v[2] = (A + Y) - c[7];
  v[3] = (A - X) + c[7];
  v[4] = (A - Y) - c[7];
  v[5] = (D + Xd) + (Yd + c[8]);
  v[6] = (D - Xd) + (Yd - c[8]);
  v[7] = (D - Xd) - (Yd - c[8]);
  v[8] = (D + Xd) - (Yd + c[8]);
}
template <typename T>
__device__ __forceinline__ void mrt_collide_ms(T f[9], const T feq[9], const T mS[9], const T s[9]) {
  T d[9], md[9], r[9], corr[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) d[i] = f[i] - feq[i];
  m_apply_pairs(d, md);
#pragma unroll
  for (int k = 0; k < 9; ++k) r[k] = (T(1) - s[k] * T(0.5)) * mS[k] - s[k] * md[k];
  minv_apply_pairs(r, corr);
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = f[i] + corr[i];
}

// The collision of mrt_collide_ms with the equilibrium given by its moments
// m^eq instead of populations: f* = f + M^{-1} [ (I - S/2) m_S - S (M f - m^eq) ].
// M f has integer coefficients, so the conserved moments of f - f^eq carry no
// rounding of the lattice weights (FP32 w_1 = RN(1/9) makes sum_i c_i g_i^eq =
// 9 RN(1/9) u = (1 + 7.5e-9) u, which relaxation at s = 1 turns into a growth
// of the momentum by that factor every step).
template <typename T>
__device__ __forceinline__ void mrt_collide_meq(T f[9], const T meq[9], const T mS[9],
                                                const T s[9]) {
  T mf[9], r[9], corr[9];
  m_apply_pairs(f, mf);
#pragma unroll
  for (int k = 0; k < 9; ++k) r[k] = (T(1) - s[k] * T(0.5)) * mS[k] - s[k] * (mf[k] - meq[k]);
  minv_apply_pairs(r, corr);
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = f[i] + corr[i];
}

// Moments of eq:geq in the basis of m_apply_pairs (rho, e, eps, j_x, q_x, j_y,
// q_y, p_xx, p_xy), from the lattice sums sum w_i = 1, sum w_i c_i c_i = I/3
// and sum w_i (3|c_i|^2 - 4) = -2: (3p, -6p + 3|u|^2, 3p - 3|u|^2, u_x, -u_x,
// u_y, -u_y, u_x^2 - u_y^2, u_x u_y).
template <typename T>
__device__ __forceinline__ void g_eq_moments(T p, T ux, T uy, T meq[9]) {
  const T usq = ux * ux + uy * uy, p3 = T(3) * p;
  meq[0] = p3;
  meq[1] = T(3) * usq - T(2) * p3;
  meq[2] = p3 - T(3) * usq;
  meq[3] = ux;
  meq[4] = -ux;
  meq[5] = uy;
  meq[6] = -uy;
  meq[7] = ux * ux - uy * uy;
  meq[8] = ux * uy;
}

// grad u + grad u^T from the non-equilibrium moments of the pre-collision g
// (eq:Fmu, re-derived from App. A's first-order balances of m_1, m_7, m_8):
// A_k = m_k - m_k^eq + G~_k / 2, div u = -(s_1/2) A_1, d_x u_x - d_y u_y =
// -(3/2) s_7 A_7, d_x u_y + d_y u_x = -3 s_8 A_8 (s_8 = s_7).  m1 is the moment
// of the stored populations (g_i - 3 w_i p_ref), whose m_1 is 6 p_ref larger.
template <typename T>
__device__ __forceinline__ void strain_moments(T m1, T m7, T m8, T p, T ux, T uy, T bx, T by,
                                               T s1, T s7, T p_ref, T& Sxx, T& Sxy, T& Syy) {
  const T A1 = ((m1 - T(6) * p_ref) - (T(-6) * p + T(3) * (ux * ux + uy * uy))) +
               T(3) * (bx * ux + by * uy);
  const T A7 = (m7 - (ux * ux - uy * uy)) + (bx * ux - by * uy);
  const T A8 = (m8 - ux * uy) + T(0.5) * (bx * uy + by * ux);
  const T div = (T(-0.5) * s1) * A1;
  const T D = (T(-1.5) * s7) * A7;
  Sxx = div + D;
  Sxy = (T(-3) * s7) * A8;
  Syy = div - D;
}

// m_1 = sum (3|c|^2 - 4) g, m_7 = g1 - g2 + g3 - g4, m_8 = g5 - g6 + g7 - g8 of
// eq:D2Q9MRT, each accumulated in index order
template <typename T>
__device__ __forceinline__ void moments_178(const T g[9], T& m1, T& m7, T& m8) {
  T a = T(-4) * g[0];
  a = a - g[1];
  a = a - g[2];
  a = a - g[3];
  a = a - g[4];
  a = a + T(2) * g[5];
  a = a + T(2) * g[6];
  a = a + T(2) * g[7];
  a = a + T(2) * g[8];
  m1 = a;
  m7 = ((g[1] - g[2]) + g[3]) - g[4];
  m8 = ((g[5] - g[6]) + g[7]) - g[8];
}

// eq:feq_CH
template <typename T>
__device__ __forceinline__ void f_eq(T phi, T mu, T ux, T uy, T eta, T feq[9]) {
  const T usq = ux * ux + uy * uy;
  feq[0] = (phi + ((T(w_of(0)) - T(1)) * eta) * mu) - ((T(w_of(0)) * phi) * usq) * T(1.5);
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const T cu = cdot(i, ux, uy);
    const T inner = ((cu * T(3)) + ((cu * cu) * T(4.5))) - usq * T(1.5);
    feq[i] = (T(w_of(i)) * eta) * mu + (T(w_of(i)) * phi) * inner;
  }
}

// eq:geq (velocity-based)
template <typename T>
__device__ __forceinline__ void g_eq(T p, T ux, T uy, T geq[9]) {
  const T usq = ux * ux + uy * uy;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const T cu = cdot(i, ux, uy);
    geq[i] = T(w_of(i)) * (((p * T(3) + cu * T(3)) + (cu * cu) * T(4.5)) - usq * T(1.5));
  }
}

// eq:Fi: F_i = w_i phi c_i.a / c_s^2
template <typename T>
__device__ __forceinline__ void src_f(T phi, T ax, T ay, T F[9]) {
  F[0] = T(0);
#pragma unroll
  for (int i = 1; i < 9; ++i) F[i] = ((T(w_of(i)) * phi) * cdot(i, ax, ay)) * T(3);
}

// eq:Gi with b = F/rho - grad p, given (Frx, Fry) = F/rho:
//   G_i = w_i [ c_i.(F/rho) / c_s^2 + ((c_i.u)(c_i.b) - c_s^2 u.b) / c_s^4 ]
template <typename T>
__device__ __forceinline__ void src_g(T Frx, T Fry, T ux, T uy, T bx, T by, T G[9]) {
  const T ub = ux * bx + uy * by;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const T cF = cdot(i, Frx, Fry);
    const T cu = cdot(i, ux, uy);
    const T cb = cdot(i, bx, by);
    G[i] = T(w_of(i)) * ((cF * T(3)) + ((cu * cb) - divk<3>(ub)) * T(9));
  }
}

// ----------------------------------------------------------------- stencils
// A view of an LDS tile: element (x, y) of the tile's node frame sits at
// a[(y + h) * w + (x + h)], h being the tile array's halo.
template <typename T>
struct Tile {
  T* a;
  int w, h;
  __device__ __forceinline__ T operator()(int x, int y) const { return a[(y + h) * w + (x + h)]; }
  __device__ __forceinline__ T& at(int x, int y) const { return a[(y + h) * w + (x + h)]; }
};

// eq:dicretized, first line: sum_{i!=0} w_i c_i P(x + c_i) / c_s^2.  FP32
// groups it by weight, (1/3) on the axis differences and (1/12) on the
// diagonal ones, the diagonal differences shared by both components (10
// operations instead of 14)
template <typename T, typename A>
__device__ __forceinline__ void iso_grad(const A& P, int x, int y, T& gx, T& gy) {
  const T w1 = T(1.0 / 9.0), w2 = T(1.0 / 36.0);
  const T p1 = P(x + 1, y), p2 = P(x, y + 1), p3 = P(x - 1, y), p4 = P(x, y - 1);
  const T p5 = P(x + 1, y + 1), p6 = P(x - 1, y + 1), p7 = P(x - 1, y - 1), p8 = P(x + 1, y - 1);
  if constexpr (std::is_same<T, float>::value) {
    const T s = p5 - p7, t = p8 - p6;
    gx = (p1 - p3) * T(1.0 / 3.0) + (s + t) * T(1.0 / 12.0);
    gy = (p2 - p4) * T(1.0 / 3.0) + (s - t) * T(1.0 / 12.0);
    return;
  }
  T ax = w1 * p1;
  ax = ax - w1 * p3;
  ax = ax + w2 * p5;
  ax = ax - w2 * p6;
  ax = ax - w2 * p7;
  ax = ax + w2 * p8;
  T ay = w1 * p2;
  ay = ay - w1 * p4;
  ay = ay + w2 * p5;
  ay = ay + w2 * p6;
  ay = ay - w2 * p7;
  ay = ay - w2 * p8;
  gx = ax * T(3);
  gy = ay * T(3);
}

template <typename T, typename A>
__device__ __forceinline__ T iso_grad_x(const A& P, int x, int y) {
  if constexpr (std::is_same<T, float>::value) {
    const T s = P(x + 1, y + 1) - P(x - 1, y - 1), t = P(x + 1, y - 1) - P(x - 1, y + 1);
    return (P(x + 1, y) - P(x - 1, y)) * T(1.0 / 3.0) + (s + t) * T(1.0 / 12.0);
  }
  const T w1 = T(1.0 / 9.0), w2 = T(1.0 / 36.0);
  T ax = w1 * P(x + 1, y);
  ax = ax - w1 * P(x - 1, y);
  ax = ax + w2 * P(x + 1, y + 1);
  ax = ax - w2 * P(x - 1, y + 1);
  ax = ax - w2 * P(x - 1, y - 1);
  ax = ax + w2 * P(x + 1, y - 1);
  return ax * T(3);
}

template <typename T, typename A>
__device__ __forceinline__ T iso_grad_y(const A& P, int x, int y) {
  if constexpr (std::is_same<T, float>::value) {
    const T s = P(x + 1, y + 1) - P(x - 1, y - 1), t = P(x + 1, y - 1) - P(x - 1, y + 1);
    return (P(x, y + 1) - P(x, y - 1)) * T(1.0 / 3.0) + (s - t) * T(1.0 / 12.0);
  }
  const T w1 = T(1.0 / 9.0), w2 = T(1.0 / 36.0);
  T ay = w1 * P(x, y + 1);
  ay = ay - w1 * P(x, y - 1);
  ay = ay + w2 * P(x + 1, y + 1);
  ay = ay + w2 * P(x - 1, y + 1);
  ay = ay - w2 * P(x - 1, y - 1);
  ay = ay - w2 * P(x + 1, y - 1);
  return ay * T(3);
}

// eq:dicretized, second line: sum_{i!=0} 2 w_i (P(x + c_i) - P(x)) / c_s^2
template <typename T, typename A>
__device__ __forceinline__ T iso_lap(const A& P, int x, int y) {
  const T a1 = T(2.0 * (1.0 / 9.0)), a2 = T(2.0 * (1.0 / 36.0));
  const T p0 = P(x, y);
  T acc = a1 * (P(x + 1, y) - p0);
  acc = acc + a1 * (P(x, y + 1) - p0);
  acc = acc + a1 * (P(x - 1, y) - p0);
  acc = acc + a1 * (P(x, y - 1) - p0);
  acc = acc + a2 * (P(x + 1, y + 1) - p0);
  acc = acc + a2 * (P(x - 1, y + 1) - p0);
  acc = acc + a2 * (P(x - 1, y - 1) - p0);
  acc = acc + a2 * (P(x + 1, y - 1) - p0);
  return acc * T(3);
}

// eq:chemical: mu = 4 beta (phi^3 - phi) - kappa lap(phi).  FP32 takes the
// Laplacian as (2/3) sum_axes + (1/6) sum_diagonals - (10/3) P(0), the same
// stencil in 9 operations instead of 16 (its bulk cancellation error, ~1e-7 of
// phi, enters mu times kappa)
template <typename T, typename A>
__device__ __forceinline__ T chem_pot(const A& P, int x, int y, T c4b, T kappa) {
  const T p0 = P(x, y);
  if constexpr (std::is_same<T, float>::value) {
    const T sa = (P(x + 1, y) + P(x - 1, y)) + (P(x, y + 1) + P(x, y - 1));
    const T sd = (P(x + 1, y + 1) + P(x - 1, y - 1)) + (P(x - 1, y + 1) + P(x + 1, y - 1));
    const T lap = T(2.0 / 3.0) * sa + (T(1.0 / 6.0) * sd - T(10.0 / 3.0) * p0);
    return c4b * ((p0 * p0) * p0 - p0) - kappa * lap;
  } else {
    return c4b * ((p0 * p0) * p0 - p0) - kappa * iso_lap<T>(P, x, y);
  }
}

// eq:fourOrder_FDM: [P(-2) - 8 P(-1) + 8 P(+1) - P(+2)] / 12
template <typename T>
__device__ __forceinline__ T d4(T m2, T m1, T p1, T p2) {
  return divk<12>(((m2 - T(8) * m1) + T(8) * p1) - p2);
}

// twelve times eq:fourOrder_FDM, [P(-2) - P(+2)] + 8 [P(+1) - P(-1)] (FP32
// folds the 1/12 into the constants it meets)
template <typename T>
__device__ __forceinline__ T d4u(T m2, T m1, T p1, T p2) {
  return (m2 - p2) + T(8) * (p1 - m1);
}

// eq:rho and eq:dynamic_vis on clamp(phi, -1, 1); NaN passes through
template <typename T>
__device__ __forceinline__ T clamp1(T p) {
  return p < T(-1) ? T(-1) : (p > T(1) ? T(1) : p);
}
template <typename T>
__device__ __forceinline__ T density(T phi, T rho1, T rho2) {
  const T c = clamp1(phi);
  return (rho1 * (T(1) + c)) / T(2) + (rho2 * (T(1) - c)) / T(2);
}
template <typename T>
__device__ __forceinline__ T dyn_visc(T phi, T mu1, T mu2) {
  const T c = clamp1(phi);
  return (mu1 * (T(1) + c)) / T(2) + (mu2 * (T(1) - c)) / T(2);
}
template <typename T>
__device__ __forceinline__ T kin_visc(T phi, T rho, T mu1, T mu2) {
  return qdiv(dyn_visc<T>(phi, mu1, mu2), rho);
}

}  // namespace lbm2p
