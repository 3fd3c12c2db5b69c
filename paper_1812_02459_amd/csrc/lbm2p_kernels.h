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

#include "lbm2p_math.h"

namespace lbm2p {

template <typename T>
struct KParams {
  int nx, ny, wx, wy;
  long long ps;                 // plane stride (elements)
  T c4b, kappa, eta, negM, lam, eps2, W, cJ;
  T rho1, rho2, mu1, mu2, gx, gy, rho_ref;
  T fa;                         // filter intensity
  T fd[6];                      // filter coefficients d_0..d_N
  int fn;                       // N = half width of the explicit filter
  T s_f[9], s_g[9];
};

// ---------------------------------------------------------------- boundaries
// Map an extended-lattice index to a node: periodic wrap, or the half-way
// mirror (node -1-i below 0, 2n-1-i above n-1) with a parity flip.  Indices
// further out than the ghost depth never feed an in-domain output; they are
// clamped to stay in bounds.
__device__ __forceinline__ int map_idx(int i, int n, int wall, int& flip) {
  if (!wall) {
    int r = i % n;
    return r < 0 ? r + n : r;
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

// load a (RW x RH) window whose (0,0) sits at node (gx0, gy0) into LDS
template <typename T, typename S, int NT>
__device__ __forceinline__ void load_window(T* dst, int RW, int RH, const S* __restrict__ src,
                                            int gx0, int gy0, const KParams<T>& P, bool odd) {
  for (int idx = threadIdx.x; idx < RW * RH; idx += NT) {
    const int ly = idx / RW, lx = idx - ly * RW;
    int flip = 0;
    const int x = map_idx(gx0 + lx, P.nx, P.wx, flip);
    const int y = map_idx(gy0 + ly, P.ny, P.wy, flip);
    T v = T(src[(long long)y * P.nx + x]);
    dst[idx] = (odd && flip) ? -v : v;
  }
}

// ------------------------------------------------------------- populations
template <typename T, int PAR>
__device__ __forceinline__ T pull(const T* __restrict__ A, const KParams<T>& P, int i, int x, int y) {
  if (PAR == 1) return A[i * P.ps + (long long)y * P.nx + x];
  const int cx = cx_of(i), cy = cy_of(i);
  int sx = x - cx, sy = y - cy;
  const bool outside = (P.wx && (sx < 0 || sx >= P.nx)) || (P.wy && (sy < 0 || sy >= P.ny));
  if (outside) return A[i * P.ps + (long long)y * P.nx + x];
  sx = sx < 0 ? sx + P.nx : (sx >= P.nx ? sx - P.nx : sx);
  sy = sy < 0 ? sy + P.ny : (sy >= P.ny ? sy - P.ny : sy);
  return A[opp(i) * P.ps + (long long)sy * P.nx + sx];
}

template <typename T, int PAR>
__device__ __forceinline__ void push(T* __restrict__ A, const KParams<T>& P, int i, int x, int y, T v) {
  if (PAR == 1) {
    A[opp(i) * P.ps + (long long)y * P.nx + x] = v;
    return;
  }
  const int cx = cx_of(i), cy = cy_of(i);
  int tx = x + cx, ty = y + cy;
  const bool outside = (P.wx && (tx < 0 || tx >= P.nx)) || (P.wy && (ty < 0 || ty >= P.ny));
  if (outside) {
    A[opp(i) * P.ps + (long long)y * P.nx + x] = v;
    return;
  }
  tx = tx < 0 ? tx + P.nx : (tx >= P.nx ? tx - P.nx : tx);
  ty = ty < 0 ? ty + P.ny : (ty >= P.ny ? ty - P.ny : ty);
  A[i * P.ps + (long long)ty * P.nx + tx] = v;
}

// ------------------------------------------------------------ a1: gather
// phi_bar = sum f_i (eq:compute_phi), p = c_s^2 sum g_i (Eq:p), j = sum g_i c_i
template <typename T, int PAR, bool COUPLED>
__global__ __launch_bounds__(256) void k_gather(KParams<T> P, const T* __restrict__ Af,
                                                const T* __restrict__ Ag, T* __restrict__ phibar,
                                                T* __restrict__ praw, T* __restrict__ jx,
                                                T* __restrict__ jy) {
  const long long n = (long long)P.nx * P.ny;
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= n) return;
  const int y = (int)(id / P.nx), x = (int)(id - (long long)y * P.nx);
  T s = pull<T, PAR>(Af, P, 0, x, y);
#pragma unroll
  for (int i = 1; i < 9; ++i) s = s + pull<T, PAR>(Af, P, i, x, y);
  phibar[id] = s;
  if (!COUPLED) return;
  T g[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) g[i] = pull<T, PAR>(Ag, P, i, x, y);
  T sg = g[0];
#pragma unroll
  for (int i = 1; i < 9; ++i) sg = sg + g[i];
  praw[id] = sg / T(3);
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
  jx[id] = ax;
  jy[id] = ay;
}

// ------------------------------------------------- a2: FD sub-step stage
// L(phi*) = div_4 (lambda J_phi + q)  (eq:final_mCHE, eq:fourOrder_FDM) and the
// TVD-RK3 combination of eq:TVD-3order for STAGE 1, 2, 3.
template <typename T, int STAGE, int TX, int TY>
__global__ __launch_bounds__(256) void k_fd(KParams<T> P, const T* __restrict__ in,
                                            const T* __restrict__ phibar, T* __restrict__ out) {
  constexpr int NT = 256;
  constexpr int W5 = TX + 10, H5 = TY + 10;   // phi*, halo 5
  constexpr int W4 = TX + 8, H4 = TY + 8;     // mu*, halo 4
  constexpr int W2 = TX + 4, H2 = TY + 4;     // J_d, halo 2
  __shared__ T sP[W5 * H5];
  __shared__ T sM[W4 * H4];
  __shared__ T sJx[W2 * H2];
  __shared__ T sJy[W2 * H2];
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  load_window<T, T, NT>(sP, W5, H5, in, x0 - 5, y0 - 5, P, false);
  __syncthreads();
  const Tile<T> tP{sP, W5, 5}, tM{sM, W4, 4}, tJx{sJx, W2, 2}, tJy{sJy, W2, 2};
  for (int idx = threadIdx.x; idx < W4 * H4; idx += NT) {
    const int ly = idx / W4 - 4, lx = idx % W4 - 4;
    sM[idx] = chem_pot<T>(tP, lx, ly, P.c4b, P.kappa);
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < W2 * H2; idx += NT) {
    const int ly = idx / W2 - 2, lx = idx % W2 - 2;
    const T Gx = d4<T>(tP(lx - 2, ly), tP(lx - 1, ly), tP(lx + 1, ly), tP(lx + 2, ly));
    const T Gy = d4<T>(tP(lx, ly - 2), tP(lx, ly - 1), tP(lx, ly + 1), tP(lx, ly + 2));
    const T Mx = d4<T>(tM(lx - 2, ly), tM(lx - 1, ly), tM(lx + 1, ly), tM(lx + 2, ly));
    const T My = d4<T>(tM(lx, ly - 2), tM(lx, ly - 1), tM(lx, ly + 1), tM(lx, ly + 2));
    const T ph = tP(lx, ly);
    const T mag = sqrt((Gx * Gx + Gy * Gy) + P.eps2);
    const T nx = Gx / mag, ny = Gy / mag;
    const T cW = (T(2) * (T(1) - ph * ph)) / P.W;
    const T Jpx = (mag - cW) * nx, Jpy = (mag - cW) * ny;
    const T s = Mx * nx + My * ny;
    const T qx = (P.negM * s) * nx, qy = (P.negM * s) * ny;
    sJx[idx] = P.lam * Jpx + qx;
    sJy[idx] = P.lam * Jpy + qy;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < TX * TY; idx += NT) {
    const int ly = idx / TX, lx = idx % TX;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= P.nx || y >= P.ny) continue;
    const T L = d4<T>(tJx(lx - 2, ly), tJx(lx - 1, ly), tJx(lx + 1, ly), tJx(lx + 2, ly)) +
                d4<T>(tJy(lx, ly - 2), tJy(lx, ly - 1), tJy(lx, ly + 1), tJy(lx, ly + 2));
    const long long id = (long long)y * P.nx + x;
    const T pin = tP(lx, ly);
    T r;
    if (STAGE == 1) {
      r = pin + L;
    } else if (STAGE == 2) {
      r = T(0.75) * phibar[id] + T(0.25) * (pin + L);
    } else {
      r = phibar[id] / T(3) + (T(2) * (pin + L)) / T(3);
    }
    out[id] = r;
  }
}

// ---------------------------------------------------------- forces (a3, a5)
// Derived fields on halo 1 shared by the velocity iteration and the collision:
// grad phi (isotropic), mu_phi (eq:chemical), rho(clamp phi) (eq:rho).
template <typename T, int NT>
__device__ __forceinline__ void derived_halo1(const Tile<T>& tP, T* sPx, T* sPy, T* sMu, T* sRho,
                                              int W1, int H1, const KParams<T>& P) {
  for (int idx = threadIdx.x; idx < W1 * H1; idx += NT) {
    const int ly = idx / W1 - 1, lx = idx % W1 - 1;
    T gx, gy;
    iso_grad<T>(tP, lx, ly, gx, gy);
    sPx[idx] = gx;
    sPy[idx] = gy;
    sMu[idx] = chem_pot<T>(tP, lx, ly, P.c4b, P.kappa);
    sRho[idx] = density<T>(tP(lx, ly), P.rho1, P.rho2);
  }
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

// ------------------------------------------- a3: velocity fixed-point sweep
// u^{k+1} = j + F(u^k) / (2 rho)   (Eq:u)
template <typename T, int TX, int TY>
__global__ __launch_bounds__(256) void k_vel(KParams<T> P, const T* __restrict__ phi,
                                             const T* __restrict__ praw, const T* __restrict__ jx,
                                             const T* __restrict__ jy, const T* __restrict__ uxi,
                                             const T* __restrict__ uyi, T* __restrict__ uxo,
                                             T* __restrict__ uyo) {
  constexpr int NT = 256;
  constexpr int W2 = TX + 4, H2 = TY + 4, W1 = TX + 2, H1 = TY + 2;
  __shared__ T sP[W2 * H2];
  __shared__ T sPx[W1 * H1], sPy[W1 * H1], sMu[W1 * H1], sRho[W1 * H1], sUx[W1 * H1],
      sUy[W1 * H1];
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  load_window<T, T, NT>(sP, W2, H2, phi, x0 - 2, y0 - 2, P, false);
  load_window<T, T, NT>(sUx, W1, H1, uxi, x0 - 1, y0 - 1, P, true);
  load_window<T, T, NT>(sUy, W1, H1, uyi, x0 - 1, y0 - 1, P, true);
  __syncthreads();
  const Tile<T> tP{sP, W2, 2};
  derived_halo1<T, NT>(tP, sPx, sPy, sMu, sRho, W1, H1, P);
  __syncthreads();
  const Tile<T> tPx{sPx, W1, 1}, tPy{sPy, W1, 1}, tMu{sMu, W1, 1}, tRho{sRho, W1, 1},
      tUx{sUx, W1, 1}, tUy{sUy, W1, 1};
  for (int idx = threadIdx.x; idx < TX * TY; idx += NT) {
    const int ly = idx / TX, lx = idx % TX;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= P.nx || y >= P.ny) continue;
    const long long id = (long long)y * P.nx + x;
    T Fx, Fy, rho, nu, a, b, c, d;
    node_force<T>(tP, tPx, tPy, tMu, tRho, tUx, tUy, praw[id], lx, ly, P, Fx, Fy, rho, nu, a, b,
                  c, d);
    uxo[id] = jx[id] + Fx / (T(2) * rho);
    uyo[id] = jy[id] + Fy / (T(2) * rho);
  }
}

// ------------------------------------------------ a4: explicit selective filter
// chi <- chi - a [ sum_j d_|j| chi(x+j, y) + sum_j d_|j| chi(x, y+j) ]  (eq:filter)
template <typename T, int TX, int TY>
__global__ __launch_bounds__(256) void k_filter(KParams<T> P, const T* __restrict__ pin,
                                                const T* __restrict__ uxin,
                                                const T* __restrict__ uyin, T* __restrict__ pout,
                                                T* __restrict__ uxout, T* __restrict__ uyout) {
  constexpr int NT = 256;
  constexpr int W5 = TX + 10, H5 = TY + 10;
  __shared__ T s0[W5 * H5], s1[W5 * H5], s2[W5 * H5];
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  load_window<T, T, NT>(s0, W5, H5, pin, x0 - 5, y0 - 5, P, false);
  load_window<T, T, NT>(s1, W5, H5, uxin, x0 - 5, y0 - 5, P, true);
  load_window<T, T, NT>(s2, W5, H5, uyin, x0 - 5, y0 - 5, P, true);
  __syncthreads();
  const int N = P.fn;
  for (int idx = threadIdx.x; idx < TX * TY; idx += NT) {
    const int ly = idx / TX, lx = idx % TX;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= P.nx || y >= P.ny) continue;
    const long long id = (long long)y * P.nx + x;
    const T* src[3] = {s0, s1, s2};
    T* dst[3] = {pout, uxout, uyout};
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const Tile<T> t{const_cast<T*>(src[f]), W5, 5};
      T sx = P.fd[N] * t(lx - N, ly);
      for (int j = -N + 1; j <= N; ++j) sx = sx + P.fd[j < 0 ? -j : j] * t(lx + j, ly);
      T sy = P.fd[N] * t(lx, ly - N);
      for (int j = -N + 1; j <= N; ++j) sy = sy + P.fd[j < 0 ? -j : j] * t(lx, ly + j);
      dst[f][id] = t(lx, ly) - P.fa * (sx + sy);
    }
  }
}

// ------------------------------------------------------ a5: collide + stream
// MRT collision of f (eq:distribution_CH) and g (eq:distribution_NS) at n+1,
// written to the streaming slots of the other parity.
template <typename T, int PAR, bool COUPLED, int TX, int TY>
__global__ __launch_bounds__(256) void k_collide(KParams<T> P, T* __restrict__ Af, T* __restrict__ Ag,
                                                 const T* __restrict__ phi, const T* __restrict__ pt,
                                                 const T* __restrict__ ux, const T* __restrict__ uy,
                                                 const T* __restrict__ uox,
                                                 const T* __restrict__ uoy) {
  constexpr int NT = 256;
  constexpr int W2 = TX + 4, H2 = TY + 4, W1 = TX + 2, H1 = TY + 2;
  __shared__ T sP[W2 * H2];
  __shared__ T sPx[COUPLED ? W1 * H1 : 1], sPy[COUPLED ? W1 * H1 : 1], sMu[W1 * H1],
      sRho[COUPLED ? W1 * H1 : 1], sUx[W1 * H1], sUy[W1 * H1], sPt[COUPLED ? W1 * H1 : 1];
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  load_window<T, T, NT>(sP, W2, H2, phi, x0 - 2, y0 - 2, P, false);
  load_window<T, T, NT>(sUx, W1, H1, ux, x0 - 1, y0 - 1, P, true);
  load_window<T, T, NT>(sUy, W1, H1, uy, x0 - 1, y0 - 1, P, true);
  if (COUPLED) load_window<T, T, NT>(sPt, W1, H1, pt, x0 - 1, y0 - 1, P, false);
  __syncthreads();
  const Tile<T> tP{sP, W2, 2};
  if (COUPLED) {
    derived_halo1<T, NT>(tP, sPx, sPy, sMu, sRho, W1, H1, P);
  } else {
    for (int idx = threadIdx.x; idx < W1 * H1; idx += NT) {
      const int ly = idx / W1 - 1, lx = idx % W1 - 1;
      sMu[idx] = chem_pot<T>(tP, lx, ly, P.c4b, P.kappa);
    }
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
    {
      T f[9], feq[9], F[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = pull<T, PAR>(Af, P, i, x, y);
      f_eq<T>(ph, tMu(lx, ly), u_x, u_y, P.eta, feq);
      src_f<T>(ph, ax, ay, F);
      mrt_collide<T>(f, feq, F, P.s_f);
#pragma unroll
      for (int i = 0; i < 9; ++i) push<T, PAR>(Af, P, i, x, y, f[i]);
    }
    if (COUPLED) {
      const T p = tPt(lx, ly);
      T Fx, Fy, rho, nu, a, b, c, d;
      node_force<T>(tP, tPx, tPy, tMu, tRho, tUx, tUy, p, lx, ly, P, Fx, Fy, rho, nu, a, b, c, d);
      T dpx, dpy;
      iso_grad<T>(tPt, lx, ly, dpx, dpy);
      const T bx = Fx / rho - dpx, by = Fy / rho - dpy;
      T g[9], geq[9], G[9], s[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) g[i] = pull<T, PAR>(Ag, P, i, x, y);
      g_eq<T>(p, u_x, u_y, geq);
      src_g<T>(Fx, Fy, rho, u_x, u_y, bx, by, G);
      const T tau_g = nu * T(3) + T(0.5);
      const T sv = T(1) / tau_g;
#pragma unroll
      for (int k = 0; k < 9; ++k) s[k] = P.s_g[k];
      s[7] = sv;
      s[8] = sv;
      mrt_collide<T>(g, geq, G, s);
#pragma unroll
      for (int i = 0; i < 9; ++i) push<T, PAR>(Ag, P, i, x, y, g[i]);
    }
  }
}

}  // namespace lbm2p
