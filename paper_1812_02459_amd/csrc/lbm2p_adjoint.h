// Reverse-mode (adjoint) kernels of one lattice update (gfx950).
//
// The forward step is a chain of stencils over the ghost extension of a field
// (periodic wrap or half-way mirror, sign kept or flipped per field) and
// pointwise maps, and every intermediate is mirror-equivariant: a value
// computed at a ghost equals the mirror node's value times the field's parity.
// The step is therefore the same function of the real nodes as one that keeps
// every intermediate on the real nodes and extends it where a stencil reads
// it, and its adjoint follows pass by pass:
//   * a pointwise map is reversed at its node with the Jacobian at the
//     recomputed forward values;
//   * a stencil O = S(ext X) is reversed as X_bar = S^T(ext O_bar), the
//     adjoint plane extended with the parity of its primal field O.  (For a
//     node y near a wall, S^T(ext O_bar)(y) collects exactly the terms
//     through which y's mirror ghosts fed the forward outputs: the image
//     term of x under the mirror has the coefficient S(-o) = sym(S) S(o) and
//     the sign of X, and parity(O) = parity(X) sym(S).)
// Every adjoint kernel works on an LDS tile loaded through that extension,
// computes intermediate adjoints on the tile's halo (ghost positions
// included) and writes real nodes only.  No atomics: each output element is
// written by one thread, so the adjoint is deterministic.  Parameter
// derivatives (sigma, M) are accumulated per real node in float64 planes and
// reduced once at the end.
//
// Parities (sign under the x-mirror, the y-mirror), adjoint = primal:
//   phi, mu, rho, p, L, the FD stage adjoint                     (+,+)
//   u_x, u_y, j (no-slip ghosts flip every component)            (-,-)
//   d/dx of an even field (grad_x rho, mu, p; G_x, M_x, J_d,x)   (-,+)
//   d/dy of an even field                                         (+,-)
//   d ux/dx, d uy/dx                                              (+,-)
//   d ux/dy, d uy/dy                                              (-,+)
//   d_x((d_y phi)^2), d_y(d_x phi d_y phi)                        (-,+)
//   d_x(d_x phi d_y phi), d_y((d_x phi)^2)                        (+,-)
#pragma once

#include "lbm2p_kernels.h"


namespace lbm2p {

// The reverse passes may contract a * b + c into fused multiply-adds in FP64
// too: their results are compared within a tolerance, not bit for bit, while
// the FP64 forward kernels of the same unit round exactly as written.  Scoped
// to the function bodies that start with it.
#define LBM2P_ADJ_CONTRACT _Pragma("clang fp contract(fast)")

// derivatives of the derived constants with respect to sigma and M
// (kappa = 3 sigma W / 8, 4 beta = 3 sigma / W, eta = 3 M / (tau_f - 1/2),
// c_J = (rho1 - rho2) M / 2, -M in q)
struct AdjConst {
  double dc4b, dkap, deta, dcJ;  // d/dsigma of 4 beta and kappa; d/dM of eta and c_J
  double c4b, kappa;             // 4 beta and kappa in float64 (initial state)
};

// ------------------------------------------------------------ tile loading
// (RW x RH) window with (0,0) at node (gx0, gy0) of a plane (plus an optional
// second plane of the same parity) extended through the ghosts: periodic
// wrap, or the half-way mirror with the value multiplied by sx for an
// x-mirror and sy for a y-mirror.
template <typename T, int NT, int RW, int RH>
__device__ __forceinline__ void load_par(T* dst, const T* __restrict__ src,
                                         const T* __restrict__ src2, int gx0, int gy0,
                                         const KParams<T>& P, int sx, int sy) {
  using WS = WinSlots<NT, RW, RH>;
  constexpr int NV = WS::NV;
  T v[NV];
  if (gx0 >= 0 && gx0 + RW <= P.nx && gy0 >= 0 && gy0 + RH <= P.ny) {
    // inside the lattice: plain row addresses, no mirror
    const T* __restrict__ base = src + (gy0 * P.nx + gx0);
    const T* __restrict__ base2 = src2 ? src2 + (gy0 * P.nx + gx0) : nullptr;
#pragma unroll
    for (int n = 0; n < NV; ++n) {
      int lx, ly;
      bool in;
      WS::at(n, lx, ly, in);
      const int o = ly * P.nx + lx;
      T w = base[o];
      if (base2) w = w + base2[o];
      v[n] = w;
    }
  } else {
#pragma unroll
    for (int n = 0; n < NV; ++n) {
      int lx, ly;
      bool in;
      WS::at(n, lx, ly, in);
      int fx = 0, fy = 0;
      const int x = map_idx(gx0 + lx, P.nx, P.wx, fx);
      const int y = map_idx(gy0 + ly, P.ny, P.wy, fy);
      const int o = y * P.nx + x;
      T w = src[o];
      if (src2) w = w + src2[o];
      v[n] = ((fx && sx < 0) != (fy && sy < 0)) ? -w : w;
    }
  }
#pragma unroll
  for (int n = 0; n < NV; ++n) {
    int lx, ly;
    bool in;
    WS::at(n, lx, ly, in);
    if (in) dst[ly * RW + lx] = v[n];
  }
}

// forward plane through the ghost extension (mirror with parity, or wrap)
template <typename T>
struct ERead {
  const T* a;
  int nx, ny, wx, wy;
  bool odd;
  __device__ __forceinline__ T operator()(int x, int y) const {
    int flip = 0;
    const int xx = map_idx(x, nx, wx, flip);
    const int yy = map_idx(y, ny, wy, flip);
    const T v = a[(long long)yy * nx + xx];
    return (odd && flip) ? -v : v;
  }
};

template <typename T>
__device__ __forceinline__ ERead<T> eread(const T* a, const KParams<T>& P, bool odd) {
  return ERead<T>{a, P.nx, P.ny, P.wx, P.wy, odd};
}

// ------------------------------------------------------- pointwise adjoints
// (M^T v)_i = sum_k M_ki v_k
template <typename T>
__device__ __forceinline__ void mT_apply(const T v[9], T out[9]) {
  LBM2P_ADJ_CONTRACT
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const int c = mrt(k, i);
      if (c == 0) continue;
      acc = acc + T(c) * v[k];
    }
    out[i] = acc;
  }
}

// Reverse of f* = f + M^-1 [ (I - S/2) M F - S M (f - f^eq) ] given the
// adjoint y of f*:  r = diag(1/(M M^T)_kk) M y,  f_bar = y - M^T (S r),
// feq_bar = M^T (S r),  F_bar = M^T ((I - S/2) r).  r is returned for the
// derivative with respect to a relaxation rate: s_k_bar = r_k (-mF_k/2 - md_k).
template <typename T>
__device__ __forceinline__ void mrt_collide_adj(const T y[9], const T s[9], T fbar[9], T feqb[9],
                                                T Fb[9], T r[9]) {
  LBM2P_ADJ_CONTRACT
  T my[9], sr[9], hr[9];
  m_apply(y, my);
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    r[k] = my[k] * T(mm_inv(k));
    sr[k] = s[k] * r[k];
    hr[k] = (T(1) - s[k] * T(0.5)) * r[k];
  }
  mT_apply(sr, feqb);
  mT_apply(hr, Fb);
#pragma unroll
  for (int i = 0; i < 9; ++i) fbar[i] = y[i] - feqb[i];
}

// reverse of f_eq (eq:feq_CH): adds to phb, mub, ubx, uby, etab
template <typename T>
__device__ __forceinline__ void f_eq_adj(T phi, T mu, T ux, T uy, T eta, const T fb[9], T& phb,
                                         T& mub, T& ubx, T& uby, T& etab) {
  LBM2P_ADJ_CONTRACT
  const T usq = ux * ux + uy * uy;
  const T w0 = T(w_of(0));
  phb = phb + fb[0] * (T(1) - (w0 * usq) * T(1.5));
  mub = mub + fb[0] * ((w0 - T(1)) * eta);
  etab = etab + fb[0] * ((w0 - T(1)) * mu);
  T usqb = -(fb[0] * (w0 * phi)) * T(1.5);
  T cx = T(0), cy = T(0);
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const T w = T(w_of(i));
    const T cu = cdot(i, ux, uy);
    const T inner = ((cu * T(3)) + ((cu * cu) * T(4.5))) - usq * T(1.5);
    const T a = fb[i] * w;
    phb = phb + a * inner;
    mub = mub + a * eta;
    etab = etab + a * mu;
    const T ap = a * phi;
    usqb = usqb - ap * T(1.5);
    const T cub = ap * (T(3) + cu * T(9));
    if (cx_of(i)) cx = cx_of(i) > 0 ? cx + cub : cx - cub;
    if (cy_of(i)) cy = cy_of(i) > 0 ? cy + cub : cy - cub;
  }
  ubx = ubx + (cx + (usqb * T(2)) * ux);
  uby = uby + (cy + (usqb * T(2)) * uy);
}

// reverse of g_eq (eq:geq): adds to pb, ubx, uby
template <typename T>
__device__ __forceinline__ void g_eq_adj(T ux, T uy, const T gb[9], T& pb, T& ubx, T& uby) {
  LBM2P_ADJ_CONTRACT
  T usqb = T(0), cx = T(0), cy = T(0), sp = T(0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const T a = gb[i] * T(w_of(i));
    sp = sp + a;
    usqb = usqb - a * T(1.5);
    const T cu = cdot(i, ux, uy);
    const T cub = a * (T(3) + cu * T(9));
    if (cx_of(i)) cx = cx_of(i) > 0 ? cx + cub : cx - cub;
    if (cy_of(i)) cy = cy_of(i) > 0 ? cy + cub : cy - cub;
  }
  pb = pb + sp * T(3);
  ubx = ubx + (cx + (usqb * T(2)) * ux);
  uby = uby + (cy + (usqb * T(2)) * uy);
}

// reverse of src_f (eq:Fi): adds to phb, abx, aby
template <typename T>
__device__ __forceinline__ void src_f_adj(T phi, T ax, T ay, const T Fb[9], T& phb, T& abx,
                                          T& aby) {
  LBM2P_ADJ_CONTRACT
  T cx = T(0), cy = T(0);
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const T a = (Fb[i] * T(w_of(i))) * T(3);
    phb = phb + a * cdot(i, ax, ay);
    const T ap = a * phi;
    if (cx_of(i)) cx = cx_of(i) > 0 ? cx + ap : cx - ap;
    if (cy_of(i)) cy = cy_of(i) > 0 ? cy + ap : cy - ap;
  }
  abx = abx + cx;
  aby = aby + cy;
}

// reverse of src_g (eq:Gi, b = F/rho - grad p): adds to Frb, ub, bb
template <typename T>
__device__ __forceinline__ void src_g_adj(T ux, T uy, T bx, T by, const T Gb[9], T& Frbx,
                                          T& Frby, T& ubx, T& uby, T& bbx, T& bby) {
  LBM2P_ADJ_CONTRACT
  T ubb = T(0), fx = T(0), fy = T(0), ux_ = T(0), uy_ = T(0), bx_ = T(0), by_ = T(0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const T a = Gb[i] * T(w_of(i));
    ubb = ubb - a * T(3);
    if (i == 0) continue;
    const T cu = cdot(i, ux, uy), cb = cdot(i, bx, by);
    const T cfb = a * T(3), cub = (a * T(9)) * cb, cbb = (a * T(9)) * cu;
    if (cx_of(i)) {
      const bool p = cx_of(i) > 0;
      fx = p ? fx + cfb : fx - cfb;
      ux_ = p ? ux_ + cub : ux_ - cub;
      bx_ = p ? bx_ + cbb : bx_ - cbb;
    }
    if (cy_of(i)) {
      const bool p = cy_of(i) > 0;
      fy = p ? fy + cfb : fy - cfb;
      uy_ = p ? uy_ + cub : uy_ - cub;
      by_ = p ? by_ + cbb : by_ - cbb;
    }
  }
  Frbx = Frbx + fx;
  Frby = Frby + fy;
  ubx = ubx + (ux_ + ubb * bx);
  uby = uby + (uy_ + ubb * by);
  bbx = bbx + (bx_ + ubb * ux);
  bby = bby + (by_ + ubb * uy);
}

// rho, nu from clamp(phi) (eq:rho, eq:dynamic_vis): phi_bar from rho_bar, nu_bar.
// The clamp passes the derivative for -1 <= phi <= 1 (ends included).
template <typename T>
__device__ __forceinline__ T props_adj(T phi, T rho, T nu, T rhob, T nub, const KParams<T>& P) {
  LBM2P_ADJ_CONTRACT
  if (!(phi >= T(-1) && phi <= T(1))) return T(0);
  const T rb = rhob - (nub * nu) / rho;
  const T mb = nub / rho;
  return rb * ((P.rho1 - P.rho2) / T(2)) + mb * ((P.mu1 - P.mu2) / T(2));
}

// forward internals of the force at a tile node (same arithmetic as node_force)
template <typename T>
struct ForceFwd {
  T Fx, Fy, rho, nu;
  T grx, gry;                 // isotropic gradient of rho(clamp phi)
  T du[4];                    // d ux/dx, d ux/dy, d uy/dx, d uy/dy
  T dmx, dmy;                 // isotropic gradient of mu
  T Q[4];                     // d_x(py^2), d_x(px py), d_y(px py), d_y(px^2)
};

template <typename T>
__device__ __forceinline__ void force_fwd(const Tile<T>& tP, const Tile<T>& tPx, const Tile<T>& tPy,
                                          const Tile<T>& tMu, const Tile<T>& tRho,
                                          const Tile<T>& tUx, const Tile<T>& tUy, T p, int x, int y,
                                          const KParams<T>& P, ForceFwd<T>& f) {
  LBM2P_ADJ_CONTRACT
  const T phi = tP(x, y);
  f.rho = density<T>(phi, P.rho1, P.rho2);
  f.nu = kin_visc<T>(phi, f.rho, P.mu1, P.mu2);
  iso_grad<T>(tMu, x, y, f.dmx, f.dmy);
  const T Jx = P.cJ * f.dmx, Jy = P.cJ * f.dmy;
  f.Q[0] = iso_grad_x<T>(ProdYY<T>{tPy}, x, y);
  iso_grad<T>(ProdXY<T>{tPx, tPy}, x, y, f.Q[1], f.Q[2]);
  f.Q[3] = iso_grad_y<T>(ProdXX<T>{tPx}, x, y);
  const T Fsx = P.kappa * (f.Q[0] - f.Q[2]);
  const T Fsy = P.kappa * (f.Q[3] - f.Q[1]);
  iso_grad<T>(tRho, x, y, f.grx, f.gry);
  iso_grad<T>(tUx, x, y, f.du[0], f.du[1]);
  iso_grad<T>(tUy, x, y, f.du[2], f.du[3]);
  const T Fpx = (-p) * f.grx, Fpy = (-p) * f.gry;
  const T Sxx = f.du[0] + f.du[0], Sxy = f.du[2] + f.du[1], Syy = f.du[3] + f.du[3];
  const T Fnx = f.nu * (Sxx * f.grx + Sxy * f.gry);
  const T Fny = f.nu * (Sxy * f.grx + Syy * f.gry);
  const T Fmx = Jx * f.du[0] + Jy * f.du[1];
  const T Fmy = Jx * f.du[2] + Jy * f.du[3];
  const T Fgx = (f.rho - P.rho_ref) * P.gx;
  const T Fgy = (f.rho - P.rho_ref) * P.gy;
  f.Fx = (((Fpx + Fsx) + Fnx) + Fmx) + Fgx;
  f.Fy = (((Fpy + Fsy) + Fny) + Fmy) + Fgy;
}

// adjoint of the force given F_bar; every field is an output (written)
template <typename T>
struct ForceAdj {
  T p, grx, gry, du[4], dmx, dmy, Q[4], rho, nu, kappa, cJ;
};

template <typename T>
__device__ __forceinline__ void force_adj(const ForceFwd<T>& f, T p, T Fbx, T Fby,
                                          const KParams<T>& P, ForceAdj<T>& a) {
  LBM2P_ADJ_CONTRACT
  // F_p = -p grad rho
  a.p = -(Fbx * f.grx + Fby * f.gry);
  T grx = -(p * Fbx), gry = -(p * Fby);
  // F_s = kappa (d_x(py^2) - d_y(px py), d_y(px^2) - d_x(px py))
  a.kappa = Fbx * (f.Q[0] - f.Q[2]) + Fby * (f.Q[3] - f.Q[1]);
  a.Q[0] = P.kappa * Fbx;
  a.Q[2] = -(P.kappa * Fbx);
  a.Q[3] = P.kappa * Fby;
  a.Q[1] = -(P.kappa * Fby);
  // F_nu = nu (grad u + grad u^T) . grad rho
  const T Sxx = f.du[0] + f.du[0], Sxy = f.du[2] + f.du[1], Syy = f.du[3] + f.du[3];
  a.nu = Fbx * (Sxx * f.grx + Sxy * f.gry) + Fby * (Sxy * f.grx + Syy * f.gry);
  grx = grx + f.nu * (Fbx * Sxx + Fby * Sxy);
  gry = gry + f.nu * (Fbx * Sxy + Fby * Syy);
  const T Sbxx = f.nu * (Fbx * f.grx), Sbxy = f.nu * (Fbx * f.gry + Fby * f.grx),
          Sbyy = f.nu * (Fby * f.gry);
  // F_m = (J . grad) u with J = c_J grad mu
  const T Jx = P.cJ * f.dmx, Jy = P.cJ * f.dmy;
  const T Jbx = Fbx * f.du[0] + Fby * f.du[2];
  const T Jby = Fbx * f.du[1] + Fby * f.du[3];
  a.du[0] = (Sbxx + Sbxx) + Jx * Fbx;
  a.du[1] = Sbxy + Jy * Fbx;
  a.du[2] = Sbxy + Jx * Fby;
  a.du[3] = (Sbyy + Sbyy) + Jy * Fby;
  a.dmx = P.cJ * Jbx;
  a.dmy = P.cJ * Jby;
  a.cJ = Jbx * f.dmx + Jby * f.dmy;
  // F_g = (rho - rho_ref) g
  a.rho = Fbx * P.gx + Fby * P.gy;
  a.grx = grx;
  a.gry = gry;
}

// canonical index of the post-collision population that streams into
// f_i(x, y) (x - c_i, or the node itself with opp(i) beyond a wall)
template <typename T>
__device__ __forceinline__ long long src_slot(const KParams<T>& P, int i, int x, int y) {
  const int cx = cx_of(i), cy = cy_of(i);
  int sx = x - cx, sy = y - cy;
  const bool out = (P.wx && (sx < 0 || sx >= P.nx)) || (P.wy && (sy < 0 || sy >= P.ny));
  if (out) return (long long)opp(i) * P.ps + (long long)y * P.nx + x;
  sx = sx < 0 ? sx + P.nx : (sx >= P.nx ? sx - P.nx : sx);
  sy = sy < 0 ? sy + P.ny : (sy >= P.ny ? sy - P.ny : sy);
  return (long long)i * P.ps + (long long)sy * P.nx + sx;
}

// work planes of the reverse step
template <typename T>
struct AdjWork {
  T *lp_p, *lp_ux, *lp_uy, *dp_x, *dp_y;   // collision: local p, u adjoints, grad p adjoint
  T* du[2][4];                             // grad u adjoints (ping-pong)
  T *a_phi, *a_mu, *a_grx, *a_gry, *a_dmx, *a_dmy, *a_Q[4];  // phi-side accumulators
  T *mu_b, *rho_b, *px_b, *py_b;           // transposed phi-side intermediates
  T *pt_b, *utx_b, *uty_b, *ukx_b, *uky_b;  // filtered p, u adjoints; u^K adjoint
  T *praw_b, *jx_b, *jy_b;
  T *phi_b, *phi2_b, *phi1_b, *phib_b;     // adjoints of phi^{n+1}, phi^(2), phi^(1), phi_bar
  T *fd_gx, *fd_gy, *fd_mx, *fd_my, *fd_loc, *fd_mu;
  double *sig, *dM;                        // per-node partials of dL/dsigma, dL/dM
};

template <typename T>
__device__ __forceinline__ T* du_sel(const AdjWork<T>& W, int s, int k) {
  return s ? W.du[1][k] : W.du[0][k];
}

// ------------------------------------------------------- a5^T: collision
// Local adjoint of the collision at every node.  The adjoint of the
// post-collision populations is the reversed step's input plus, when PEND,
// the gather/streaming adjoint of the step reversed before it (phi_bar,
// p and j adjoints of that step's pre-collision populations, which streamed
// from these slots).  Writes the adjoint of this step's pre-collision
// populations to the canonical slot they streamed from (the streaming
// permutation reversed), the local p and u adjoints, the grad u and grad p
// adjoints, and initialises the phi-side accumulators.
template <typename T, bool COUPLED, bool PEND, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_adj_collide(
    KParams<T> P, AdjConst C, int tiles_x, const T* __restrict__ phi, const T* __restrict__ pt,
    const T* __restrict__ ux, const T* __restrict__ uy, const T* __restrict__ uox,
    const T* __restrict__ uoy, const T* __restrict__ m7g, const T* __restrict__ m8g,
    const T* __restrict__ Afi, const T* __restrict__ Agi, const T* __restrict__ pphi,
    const T* __restrict__ pp, const T* __restrict__ pjx, const T* __restrict__ pjy,
    T* __restrict__ Afo, T* __restrict__ Ago, T* __restrict__ Uox, T* __restrict__ Uoy,
    AdjWork<T> Wk) {
  LBM2P_ADJ_CONTRACT
  constexpr int W2 = TX + 4, H2 = TY + 4, W1 = TX + 2, H1 = TY + 2;
  constexpr int NC = COUPLED ? W1 * H1 : 1, NP = PEND ? W1 * H1 : 1,
                NPC = (PEND && COUPLED) ? W1 * H1 : 1;
  __shared__ T sP[W2 * H2];
  __shared__ T sPx[NC], sPy[NC], sMu[W1 * H1], sRho[NC], sUx[W1 * H1], sUy[W1 * H1], sPt[NC];
  __shared__ T sB[NP], sQ[NPC], sJx[NPC], sJy[NPC];
  int bx, by;
  tile_of(tiles_x, bx, by);
  const int x0 = bx * TX, y0 = by * TY;
  load_window<T, T, NT, W2, H2>(sP, phi, x0 - 2, y0 - 2, P, false);
  load_window<T, T, NT, W1, H1>(sUx, ux, x0 - 1, y0 - 1, P, true);
  load_window<T, T, NT, W1, H1>(sUy, uy, x0 - 1, y0 - 1, P, true);
  if (COUPLED) load_window<T, T, NT, W1, H1>(sPt, pt, x0 - 1, y0 - 1, P, false);
  if (PEND) {
    // only real neighbours are read (a population that bounced back streamed
    // from the node itself), so the plain window suffices
    load_window<T, T, NT, W1, H1>(sB, pphi, x0 - 1, y0 - 1, P, false);
    if (COUPLED) {
      load_window<T, T, NT, W1, H1>(sQ, pp, x0 - 1, y0 - 1, P, false);
      load_window<T, T, NT, W1, H1>(sJx, pjx, x0 - 1, y0 - 1, P, false);
      load_window<T, T, NT, W1, H1>(sJy, pjy, x0 - 1, y0 - 1, P, false);
    }
  }
  __syncthreads();
  const Tile<T> tP{sP, W2, 2};
  if (COUPLED) {
    derived_halo1<T, NT, W1, H1>(tP, sPx, sPy, sMu, sRho, P);
  } else {
    for_window<W1, H1, NT>([&](int ix_, int iy_) {
      const int ly = iy_ - 1, lx = ix_ - 1, idx = iy_ * W1 + ix_;
      sMu[idx] = chem_pot<T>(tP, lx, ly, P.c4b, P.kappa);
    });
  }
  __syncthreads();
  const Tile<T> tPx{sPx, W1, 1}, tPy{sPy, W1, 1}, tMu{sMu, W1, 1}, tRho{sRho, W1, 1},
      tUx{sUx, W1, 1}, tUy{sUy, W1, 1}, tPt{sPt, W1, 1}, tB{sB, W1, 1}, tQ{sQ, W1, 1},
      tJx{sJx, W1, 1}, tJy{sJy, W1, 1};
  for (int idx = threadIdx.x; idx < TX * TY; idx += NT) {
    const int ly = idx / TX, lx = idx % TX;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= P.nx || y >= P.ny) continue;
    const long long id = (long long)y * P.nx + x;
    // source node of the population i pulled at this node's slot i: x + c_i,
    // or the node itself where x + c_i lies beyond a wall
    int sxl[9], syl[9];
    bool bb[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int tx = x + cx_of(i), ty = y + cy_of(i);
      bb[i] = (P.wx && (tx < 0 || tx >= P.nx)) || (P.wy && (ty < 0 || ty >= P.ny));
      sxl[i] = bb[i] ? lx : lx + cx_of(i);
      syl[i] = bb[i] ? ly : ly + cy_of(i);
    }
    const T ph = tP(lx, ly), u_x = tUx(lx, ly), u_y = tUy(lx, ly);
    T duxx, duxy, duyx, duyy;
    iso_grad<T>(tUx, lx, ly, duxx, duxy);
    iso_grad<T>(tUy, lx, ly, duyx, duyy);
    const T ax = (u_x - uox[id]) + (u_x * duxx + u_y * duxy);
    const T ay = (u_y - uoy[id]) + (u_x * duyx + u_y * duyy);
    const T mu = tMu(lx, ly);
    T phb = T(0), mub = T(0), ubx = T(0), uby = T(0), etab = T(0), abx = T(0), aby = T(0);
    {
      T yv[9], fb[9], feqb[9], Fb[9], r[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        yv[i] = Afi[i * P.ps + id];
        if (PEND) yv[i] = yv[i] + tB(sxl[i], syl[i]);
      }
      mrt_collide_adj<T>(yv, P.s_f, fb, feqb, Fb, r);
#pragma unroll
      for (int i = 0; i < 9; ++i) Afo[src_slot(P, i, x, y)] = fb[i];
      f_eq_adj<T>(ph, mu, u_x, u_y, P.eta, feqb, phb, mub, ubx, uby, etab);
      src_f_adj<T>(ph, ax, ay, Fb, phb, abx, aby);
    }
    double dM = double(etab) * C.deta;
    if (COUPLED) {
      // accel reversed: a = (u - u_o) + (u . grad) u
      ubx = ubx + (abx + (abx * duxx + aby * duyx));
      uby = uby + (aby + (abx * duxy + aby * duyy));
      Uox[id] = -abx;
      Uoy[id] = -aby;
      T dub[4] = {abx * u_x, abx * u_y, aby * u_x, aby * u_y};
      const T p = tPt(lx, ly);
      ForceFwd<T> ff;
      force_fwd<T>(tP, tPx, tPy, tMu, tRho, tUx, tUy, p, lx, ly, P, ff);
      T dpx, dpy;
      iso_grad<T>(tPt, lx, ly, dpx, dpy);
      const T Frx = ff.Fx / ff.rho, Fry = ff.Fy / ff.rho;
      const T bxv = Frx - dpx, byv = Fry - dpy;
      T geq[9], G[9], s[9], mG[9], mq[9];
      g_eq<T>(p - P.p_ref, u_x, u_y, geq);
      src_g<T>(Frx, Fry, u_x, u_y, bxv, byv, G);
      const T tau_g = ff.nu * T(3) + T(0.5);
      const T sv = T(1) / tau_g;
#pragma unroll
      for (int k = 0; k < 9; ++k) s[k] = P.s_g[k];
      s[7] = sv;
      s[8] = sv;
      m_apply(G, mG);
      m_apply(geq, mq);
      const T md7 = m7g[id] - mq[7], md8 = m8g[id] - mq[8];
      T yv[9], gb[9], geqb[9], Gb[9], r[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        yv[i] = Agi[i * P.ps + id];
        if (PEND) {
          // p = sum g / 3 and j = sum g c of the source node reversed
          const T jc = cdot(i, tJx(sxl[i], syl[i]), tJy(sxl[i], syl[i]));
          yv[i] = yv[i] + (tQ(sxl[i], syl[i]) / T(3) + (bb[i] ? -jc : jc));
        }
      }
      mrt_collide_adj<T>(yv, s, gb, geqb, Gb, r);
#pragma unroll
      for (int i = 0; i < 9; ++i) Ago[src_slot(P, i, x, y)] = gb[i];
      const T svb = r[7] * (-(mG[7] * T(0.5)) - md7) + r[8] * (-(mG[8] * T(0.5)) - md8);
      const T nub = -((svb * T(3)) * (sv * sv));
      T pb = T(0), Frbx = T(0), Frby = T(0), bbx = T(0), bby = T(0);
      g_eq_adj<T>(u_x, u_y, geqb, pb, ubx, uby);
      src_g_adj<T>(u_x, u_y, bxv, byv, Gb, Frbx, Frby, ubx, uby, bbx, bby);
      Frbx = Frbx + bbx;
      Frby = Frby + bby;
      const T Fbx = Frbx / ff.rho, Fby = Frby / ff.rho;
      const T rhob = -((Frbx * Frx + Frby * Fry) / ff.rho);
      ForceAdj<T> fa;
      force_adj<T>(ff, p, Fbx, Fby, P, fa);
      pb = pb + fa.p;
#pragma unroll
      for (int k = 0; k < 4; ++k) dub[k] = dub[k] + fa.du[k];
      phb = phb + props_adj<T>(ph, ff.rho, ff.nu, fa.rho + rhob, fa.nu + nub, P);
      Wk.lp_p[id] = pb;
      Wk.lp_ux[id] = ubx;
      Wk.lp_uy[id] = uby;
      Wk.dp_x[id] = -bbx;
      Wk.dp_y[id] = -bby;
#pragma unroll
      for (int k = 0; k < 4; ++k) Wk.du[0][k][id] = dub[k];
      Wk.a_grx[id] = fa.grx;
      Wk.a_gry[id] = fa.gry;
      Wk.a_dmx[id] = fa.dmx;
      Wk.a_dmy[id] = fa.dmy;
#pragma unroll
      for (int k = 0; k < 4; ++k) Wk.a_Q[k][id] = fa.Q[k];
      Wk.sig[id] = Wk.sig[id] + double(fa.kappa) * C.dkap;
      dM = dM + double(fa.cJ) * C.dcJ;
    }
    Wk.a_phi[id] = phb;
    Wk.a_mu[id] = mub;
    Wk.dM[id] = Wk.dM[id] + dM;
  }
}

// ----------------------------------- a5^T gradients, then a4^T: filter
// Adjoints of the filtered p~, u~ on the tile grown by the filter half width
// N: local parts, the next state's u~ adjoint (u~ is also the next state's
// velocity), and the transposed gradients of the collision's grad u and
// grad p adjoints; then chi_bar = chi~_bar - a F^T chi~_bar (the explicit
// filter's stencil is symmetric; N = 0: no filter, the outputs are the
// adjoints of p~, u~ themselves).  Outputs to (op, oux, ouy); with N = 0 a
// tile reads only its own nodes of lp_*, so the outputs may be lp_*.
template <typename T, int N, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_adj_filter_t(KParams<T> P, int tiles_x,
                                                     const T* __restrict__ Uoix,
                                                     const T* __restrict__ Uoiy, AdjWork<T> Wk,
                                                     T* op, T* oux, T* ouy) {
  LBM2P_ADJ_CONTRACT
  constexpr int WN = TX + 2 * N, HN = TY + 2 * N, WB = WN + 2, HB = HN + 2;
  __shared__ T sB[2][WB * HB];
  __shared__ T sPt[WN * HN], sUx[WN * HN], sUy[WN * HN];
  int bx, by;
  tile_of(tiles_x, bx, by);
  const int x0 = bx * TX, y0 = by * TY;
  load_par<T, NT, WN, HN>(sPt, Wk.lp_p, nullptr, x0 - N, y0 - N, P, 1, 1);
  load_par<T, NT, WN, HN>(sUx, Wk.lp_ux, Uoix, x0 - N, y0 - N, P, -1, -1);
  load_par<T, NT, WN, HN>(sUy, Wk.lp_uy, Uoiy, x0 - N, y0 - N, P, -1, -1);
  const Tile<T> tB0{sB[0], WB, N + 1}, tB1{sB[1], WB, N + 1};
  // pairs (x-derivative plane, y-derivative plane) with their parities and target:
  // (d ux/dx, d ux/dy) -> u_x, (d uy/dx, d uy/dy) -> u_y, grad p -> p
  const T* const src[6] = {Wk.du[0][0], Wk.du[0][1], Wk.du[0][2], Wk.du[0][3], Wk.dp_x, Wk.dp_y};
  const int psx[6] = {1, -1, 1, -1, -1, 1}, psy[6] = {-1, 1, -1, 1, 1, -1};
#pragma unroll 1
  for (int k = 0; k < 3; ++k) {
    __syncthreads();
    load_par<T, NT, WB, HB>(sB[0], src[2 * k], nullptr, x0 - N - 1, y0 - N - 1, P, psx[2 * k],
                    psy[2 * k]);
    load_par<T, NT, WB, HB>(sB[1], src[2 * k + 1], nullptr, x0 - N - 1, y0 - N - 1, P,
                    psx[2 * k + 1], psy[2 * k + 1]);
    __syncthreads();
    T* d = k == 0 ? sUx : (k == 1 ? sUy : sPt);
    for_window<WN, HN, NT>([&](int ix_, int iy_) {
      const int ly = iy_ - N, lx = ix_ - N, idx = iy_ * WN + ix_;
      d[idx] = d[idx] - (iso_grad_x<T>(tB0, lx, ly) + iso_grad_y<T>(tB1, lx, ly));
    });
  }
  __syncthreads();
  T dd[N + 1];
#pragma unroll
  for (int j = 0; j <= N; ++j) dd[j] = P.fd[j];
  const T a = P.fa;
  for (int idx = threadIdx.x; idx < TX * TY; idx += NT) {
    const int ly = idx / TX, lx = idx % TX;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= P.nx || y >= P.ny) continue;
    const long long id = (long long)y * P.nx + x;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const Tile<T> t{f == 0 ? sPt : f == 1 ? sUx : sUy, WN, N};
      T r = t(lx, ly);
      if (N > 0) {
        T sx = dd[N] * t(lx - N, ly);
#pragma unroll
        for (int j = -N + 1; j <= N; ++j) sx = sx + dd[j < 0 ? -j : j] * t(lx + j, ly);
        T sy = dd[N] * t(lx, ly - N);
#pragma unroll
        for (int j = -N + 1; j <= N; ++j) sy = sy + dd[j < 0 ? -j : j] * t(lx, ly + j);
        r = r - a * (sx + sy);
      }
      if (f == 0) op[id] = r;
      else if (f == 1) oux[id] = r;
      else ouy[id] = r;
    }
  }
}

// -------------------------------------------- a3^T: one velocity sweep
// Reverse of u^{k+1} = j + F(u^k)/(2 rho).  The adjoint of u^{k+1} is the
// filter's output for the last sweep (FIRST), else the transposed gradient of
// the previous reverse sweep's grad-u adjoint (du[src]); this sweep writes its
// own grad-u adjoint to du[1 - src].
template <typename T, bool FIRST, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_adj_vel(KParams<T> P, AdjConst C, int tiles_x,
                                                 const T* __restrict__ phi,
                                                 const T* __restrict__ praw,
                                                 const T* __restrict__ ukx,
                                                 const T* __restrict__ uky, int src,
                                                 AdjWork<T> Wk) {
  LBM2P_ADJ_CONTRACT
  constexpr int W2 = TX + 4, H2 = TY + 4, W1 = TX + 2, H1 = TY + 2;
  constexpr int NR = (TX * TY + NT - 1) / NT;
  __shared__ T sP[W2 * H2];
  __shared__ T sPx[W1 * H1], sPy[W1 * H1], sMu[W1 * H1], sRho[W1 * H1], sUx[W1 * H1],
      sUy[W1 * H1], sB[FIRST ? 1 : W1 * H1];
  int bx, by;
  tile_of(tiles_x, bx, by);
  const int x0 = bx * TX, y0 = by * TY;
  T vb[2][NR];
  if (!FIRST) {
    const int psx[4] = {1, -1, 1, -1}, psy[4] = {-1, 1, -1, 1};
    const Tile<T> tB{sB, W1, 1};
#pragma unroll
    for (int r = 0; r < NR; ++r) vb[0][r] = vb[1][r] = T(0);
#pragma unroll 1
    for (int k = 0; k < 4; ++k) {
      if (k) __syncthreads();
      load_par<T, NT, W1, H1>(sB, du_sel(Wk, src, k), nullptr, x0 - 1, y0 - 1, P, psx[k], psy[k]);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int idx = threadIdx.x + r * NT;
        if (idx >= TX * TY) continue;
        const int ly = idx / TX, lx = idx % TX;
        const T g = (k & 1) == 0 ? iso_grad_x<T>(tB, lx, ly) : iso_grad_y<T>(tB, lx, ly);
        vb[k >> 1][r] = vb[k >> 1][r] - g;
      }
    }
  }
  load_window<T, T, NT, W2, H2>(sP, phi, x0 - 2, y0 - 2, P, false);
  load_window<T, T, NT, W1, H1>(sUx, ukx, x0 - 1, y0 - 1, P, true);
  load_window<T, T, NT, W1, H1>(sUy, uky, x0 - 1, y0 - 1, P, true);
  __syncthreads();
  const Tile<T> tP{sP, W2, 2};
  derived_halo1<T, NT, W1, H1>(tP, sPx, sPy, sMu, sRho, P);
  __syncthreads();
  const Tile<T> tPx{sPx, W1, 1}, tPy{sPy, W1, 1}, tMu{sMu, W1, 1}, tRho{sRho, W1, 1},
      tUx{sUx, W1, 1}, tUy{sUy, W1, 1};
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int idx = threadIdx.x + r * NT;
    if (idx >= TX * TY) continue;
    const int ly = idx / TX, lx = idx % TX;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= P.nx || y >= P.ny) continue;
    const long long id = (long long)y * P.nx + x;
    T vbx, vby;
    if (FIRST) {
      vbx = Wk.ukx_b[id];
      vby = Wk.uky_b[id];
      Wk.jx_b[id] = vbx;
      Wk.jy_b[id] = vby;
    } else {
      vbx = vb[0][r];
      vby = vb[1][r];
      Wk.jx_b[id] = Wk.jx_b[id] + vbx;
      Wk.jy_b[id] = Wk.jy_b[id] + vby;
    }
    const T p = praw[id];
    ForceFwd<T> ff;
    force_fwd<T>(tP, tPx, tPy, tMu, tRho, tUx, tUy, p, lx, ly, P, ff);
    const T Fbx = vbx / (T(2) * ff.rho), Fby = vby / (T(2) * ff.rho);
    const T rhob = -((Fbx * ff.Fx + Fby * ff.Fy) / ff.rho);
    ForceAdj<T> fa;
    force_adj<T>(ff, p, Fbx, Fby, P, fa);
    Wk.praw_b[id] = Wk.praw_b[id] + fa.p;
#pragma unroll
    for (int k = 0; k < 4; ++k) du_sel(Wk, 1 - src, k)[id] = fa.du[k];
    Wk.a_phi[id] = Wk.a_phi[id] + props_adj<T>(tP(lx, ly), ff.rho, ff.nu, fa.rho + rhob, fa.nu, P);
    Wk.a_grx[id] = Wk.a_grx[id] + fa.grx;
    Wk.a_gry[id] = Wk.a_gry[id] + fa.gry;
    Wk.a_dmx[id] = Wk.a_dmx[id] + fa.dmx;
    Wk.a_dmy[id] = Wk.a_dmy[id] + fa.dmy;
#pragma unroll
    for (int k = 0; k < 4; ++k) Wk.a_Q[k][id] = Wk.a_Q[k][id] + fa.Q[k];
    Wk.sig[id] = Wk.sig[id] + double(fa.kappa) * C.dkap;
    Wk.dM[id] = Wk.dM[id] + double(fa.cJ) * C.dcJ;
  }
}

// ------------------------------------- phi-side transposes (a3^T and a5^T)
// The adjoint of phi^{n+1}: the pointwise part, mu^T of
// mu_bar = a_mu + grad^T(a_dm), rho' grad^T(a_gr), grad^T of the
// (d_x phi, d_y phi) adjoints obtained from the product-gradient adjoints,
// and the loss seed.  The first sweep's velocity adjoint (grad^T of du[src])
// joins the state's u~ adjoint.
template <typename T, bool COUPLED, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_adj_phi(KParams<T> P, AdjConst C, int tiles_x,
                                                const T* __restrict__ phi, int src,
                                                const double* __restrict__ seed,
                                                T* __restrict__ Uox, T* __restrict__ Uoy,
                                                AdjWork<T> Wk) {
  LBM2P_ADJ_CONTRACT
  constexpr int W2 = TX + 4, H2 = TY + 4, W1 = TX + 2, H1 = TY + 2;
  constexpr int NR = (TX * TY + NT - 1) / NT;
  constexpr int NQ = COUPLED ? W1 * H1 : 1, NB = COUPLED ? W2 * H2 : 1;
  __shared__ T sP[W2 * H2], sB[2][NB], sMu[W1 * H1];
  __shared__ T sQxx[NQ], sQyy[NQ], sQxy[NQ];
  int bx, by;
  tile_of(tiles_x, bx, by);
  const int x0 = bx * TX, y0 = by * TY;
  load_window<T, T, NT, W2, H2>(sP, phi, x0 - 2, y0 - 2, P, false);
  load_par<T, NT, W1, H1>(sMu, Wk.a_mu, nullptr, x0 - 1, y0 - 1, P, 1, 1);
  const Tile<T> tP{sP, W2, 2}, tMu{sMu, W1, 1};
  T rb[NR], ub[2][NR];
  if (COUPLED) {
    // tile-grown (halo 1) accumulations from halo-2 windows, pairs
    // (x-derivative plane, y-derivative plane): grad mu -> mu_bar;
    // (d_y(px^2), d_x(py^2)) -> (Q_xx, Q_yy) adjoints; d(px py) -> Q_xy
    const Tile<T> tA{sB[0], W2, 2}, tC{sB[1], W2, 2};
    const T* const s2[6] = {Wk.a_dmx, Wk.a_dmy, Wk.a_Q[0], Wk.a_Q[3], Wk.a_Q[1], Wk.a_Q[2]};
    const int p2x[6] = {-1, 1, -1, 1, 1, -1}, p2y[6] = {1, -1, 1, -1, -1, 1};
#pragma unroll 1
    for (int k = 0; k < 3; ++k) {
      __syncthreads();
      load_par<T, NT, W2, H2>(sB[0], s2[2 * k], nullptr, x0 - 2, y0 - 2, P, p2x[2 * k], p2y[2 * k]);
      load_par<T, NT, W2, H2>(sB[1], s2[2 * k + 1], nullptr, x0 - 2, y0 - 2, P, p2x[2 * k + 1],
                      p2y[2 * k + 1]);
      __syncthreads();
      for_window<W1, H1, NT>([&](int ix_, int iy_) {
        const int ly = iy_ - 1, lx = ix_ - 1, idx = iy_ * W1 + ix_;
        if (k == 0) {
          sMu[idx] = sMu[idx] - (iso_grad_x<T>(tA, lx, ly) + iso_grad_y<T>(tC, lx, ly));
        } else if (k == 1) {
          sQyy[idx] = -iso_grad_x<T>(tA, lx, ly);
          sQxx[idx] = -iso_grad_y<T>(tC, lx, ly);
        } else {
          sQxy[idx] = -(iso_grad_x<T>(tA, lx, ly) + iso_grad_y<T>(tC, lx, ly));
        }
      });
    }
    __syncthreads();
    // (d_x phi, d_y phi) adjoints on halo 1, in place of the Q_xx, Q_yy adjoints
    for_window<W1, H1, NT>([&](int ix_, int iy_) {
      const int ly = iy_ - 1, lx = ix_ - 1, idx = iy_ * W1 + ix_;
      T px, py;
      iso_grad<T>(tP, lx, ly, px, py);
      const T qxx = sQxx[idx], qyy = sQyy[idx], qxy = sQxy[idx];
      sQxx[idx] = (T(2) * px) * qxx + py * qxy;
      sQyy[idx] = (T(2) * py) * qyy + px * qxy;
    });
    // tile-only accumulations from halo-1 windows: rho_bar, and u^0_bar
    const Tile<T> tA1{sB[0], W1, 1}, tC1{sB[1], W1, 1};
    const T* const s1[6] = {Wk.a_grx, Wk.a_gry, du_sel(Wk, src, 0), du_sel(Wk, src, 1),
                            du_sel(Wk, src, 2), du_sel(Wk, src, 3)};
    const int p1x[6] = {-1, 1, 1, -1, 1, -1}, p1y[6] = {1, -1, -1, 1, -1, 1};
#pragma unroll 1
    for (int k = 0; k < 3; ++k) {
      __syncthreads();
      load_par<T, NT, W1, H1>(sB[0], s1[2 * k], nullptr, x0 - 1, y0 - 1, P, p1x[2 * k], p1y[2 * k]);
      load_par<T, NT, W1, H1>(sB[1], s1[2 * k + 1], nullptr, x0 - 1, y0 - 1, P, p1x[2 * k + 1],
                      p1y[2 * k + 1]);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int idx = threadIdx.x + r * NT;
        if (idx >= TX * TY) continue;
        const int ly = idx / TX, lx = idx % TX;
        const T g = -(iso_grad_x<T>(tA1, lx, ly) + iso_grad_y<T>(tC1, lx, ly));
        if (k == 0) rb[r] = g;
        else ub[k - 1][r] = g;
      }
    }
  }
  __syncthreads();
  const Tile<T> tQx{sQxx, W1, 1}, tQy{sQyy, W1, 1};
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int idx = threadIdx.x + r * NT;
    if (idx >= TX * TY) continue;
    const int ly = idx / TX, lx = idx % TX;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= P.nx || y >= P.ny) continue;
    const long long id = (long long)y * P.nx + x;
    const T p0 = tP(lx, ly);
    const T mub = tMu(lx, ly);
    T v = Wk.a_phi[id] + (P.c4b * ((T(3) * p0) * p0 - T(1))) * mub;
    v = v - P.kappa * iso_lap<T>(tMu, lx, ly);
    if (COUPLED) {
      if (p0 >= T(-1) && p0 <= T(1)) v = v + rb[r] * ((P.rho1 - P.rho2) / T(2));
      v = v - (iso_grad_x<T>(tQx, lx, ly) + iso_grad_y<T>(tQy, lx, ly));
      Uox[id] = Uox[id] + ub[0][r];
      Uoy[id] = Uoy[id] + ub[1][r];
    }
    if (seed) v = v + T(seed[id]);
    Wk.phi_b[id] = v;
    const T dmu_dc4b = (p0 * p0) * p0 - p0;
    const T dmu_dkap = -iso_lap<T>(tP, lx, ly);
    Wk.sig[id] = Wk.sig[id] + double(mub * dmu_dc4b) * C.dc4b + double(mub * dmu_dkap) * C.dkap;
  }
}

// ------------------------------------------------------ a2^T: FD stage
// One TVD-RK3 stage L(phi_s) reversed for the stage adjoint a = coef * src:
// J_d_bar = d4^T a, the pointwise reverse of J_d = lambda J_phi + q on the
// tile grown by 3 (G, grad mu adjoints and the cW term), mu_bar = d4^T of the
// grad-mu adjoints on the tile grown by 1, then DL^T a and the stage's RK3
// combination:
//   STAGE 3: phi2_bar = a + DL^T a,  a = (2/3) phi_bar
//   STAGE 2: phi1_bar = a + DL^T a,  a = phi2_bar / 4
//   STAGE 1: phib_bar = phi_bar/3 + (3/4) phi2_bar + phi1_bar + DL^T phi1_bar
template <typename T, int STAGE, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_adj_fd(KParams<T> P, AdjConst C, int tiles_x,
                                                const T* __restrict__ in,
                                                const T* __restrict__ src, T coef,
                                                AdjWork<T> Wk) {
  LBM2P_ADJ_CONTRACT
  constexpr int W6 = TX + 12, H6 = TY + 12;   // phi_s
  constexpr int W5 = TX + 10, H5 = TY + 10;   // a, mu (then mu_bar on halo 1)
  constexpr int W3 = TX + 6, H3 = TY + 6;     // pointwise adjoints
  constexpr int W1 = TX + 2, H1 = TY + 2;
  __shared__ T sP[W6 * H6], sA[W5 * H5], sM[W5 * H5];
  __shared__ T sGx[W3 * H3], sGy[W3 * H3], sMx[W3 * H3], sMy[W3 * H3], sL[W3 * H3];
  int bx, by;
  tile_of(tiles_x, bx, by);
  const int x0 = bx * TX, y0 = by * TY;
  load_window<T, T, NT, W6, H6>(sP, in, x0 - 6, y0 - 6, P, false);
  load_par<T, NT, W5, H5>(sA, src, nullptr, x0 - 5, y0 - 5, P, 1, 1);
  __syncthreads();
  const Tile<T> tP{sP, W6, 6}, tA{sA, W5, 5}, tM{sM, W5, 5};
  for_window<W5, H5, NT>([&](int ix_, int iy_) {
    const int ly = iy_ - 5, lx = ix_ - 5, idx = iy_ * W5 + ix_;
    sM[idx] = chem_pot<T>(tP, lx, ly, P.c4b, P.kappa);
  });
  __syncthreads();
  for_window<W3, H3, NT>([&](int ix_, int iy_) {
    const int ly = iy_ - 3, lx = ix_ - 3, idx = iy_ * W3 + ix_;
    const T Jbx = coef * (-d4<T>(tA(lx - 2, ly), tA(lx - 1, ly), tA(lx + 1, ly), tA(lx + 2, ly)));
    const T Jby = coef * (-d4<T>(tA(lx, ly - 2), tA(lx, ly - 1), tA(lx, ly + 1), tA(lx, ly + 2)));
    const T Gx = d4<T>(tP(lx - 2, ly), tP(lx - 1, ly), tP(lx + 1, ly), tP(lx + 2, ly));
    const T Gy = d4<T>(tP(lx, ly - 2), tP(lx, ly - 1), tP(lx, ly + 1), tP(lx, ly + 2));
    const T Mx = d4<T>(tM(lx - 2, ly), tM(lx - 1, ly), tM(lx + 1, ly), tM(lx + 2, ly));
    const T My = d4<T>(tM(lx, ly - 2), tM(lx, ly - 1), tM(lx, ly + 1), tM(lx, ly + 2));
    const T ph = tP(lx, ly);
    const T mag = sqrt((Gx * Gx + Gy * Gy) + P.eps2);
    const T nx = Gx / mag, ny = Gy / mag;
    const T cW = (T(2) * (T(1) - ph * ph)) / P.W;
    const T s = Mx * nx + My * ny;
    // J_d = lambda (mag - cW) n + (-M s) n
    const T Jpbx = P.lam * Jbx, Jpby = P.lam * Jby;
    const T qn = Jbx * nx + Jby * ny;          // q_bar . n
    const T sb = P.negM * qn;
    const T mc = mag - cW;
    const T nbx = (P.negM * s) * Jbx + mc * Jpbx + sb * Mx;
    const T nby = (P.negM * s) * Jby + mc * Jpby + sb * My;
    const T t = Jpbx * nx + Jpby * ny;
    const T magb = t - (nbx * nx + nby * ny) / mag;
    sGx[idx] = nbx / mag + magb * nx;
    sGy[idx] = nby / mag + magb * ny;
    sMx[idx] = sb * nx;
    sMy[idx] = sb * ny;
    sL[idx] = (-t) * ((T(-4) * ph) / P.W);
    if (lx >= 0 && lx < TX && ly >= 0 && ly < TY && x0 + lx < P.nx && y0 + ly < P.ny) {
      const long long id = (long long)(y0 + ly) * P.nx + (x0 + lx);
      Wk.dM[id] = Wk.dM[id] - double(s * qn);  // dL/dM = -dL/d(-M); one thread per node
    }
  });
  __syncthreads();
  const Tile<T> tGx{sGx, W3, 3}, tGy{sGy, W3, 3}, tMx{sMx, W3, 3}, tMy{sMy, W3, 3},
      tL{sL, W3, 3};
  // mu_bar on halo 1, over the (now free) mu tile
  T* sMb = sM;
  for_window<W1, H1, NT>([&](int ix_, int iy_) {
    const int ly = iy_ - 1, lx = ix_ - 1, idx = iy_ * W1 + ix_;
    sMb[idx] = -d4<T>(tMx(lx - 2, ly), tMx(lx - 1, ly), tMx(lx + 1, ly), tMx(lx + 2, ly)) -
               d4<T>(tMy(lx, ly - 2), tMy(lx, ly - 1), tMy(lx, ly + 1), tMy(lx, ly + 2));
  });
  __syncthreads();
  const Tile<T> tMb{sMb, W1, 1};
  for (int idx = threadIdx.x; idx < TX * TY; idx += NT) {
    const int ly = idx / TX, lx = idx % TX;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= P.nx || y >= P.ny) continue;
    const long long id = (long long)y * P.nx + x;
    const T p0 = tP(lx, ly);
    const T mub = tMb(lx, ly);
    T dl = tL(lx, ly) - d4<T>(tGx(lx - 2, ly), tGx(lx - 1, ly), tGx(lx + 1, ly), tGx(lx + 2, ly));
    dl = dl - d4<T>(tGy(lx, ly - 2), tGy(lx, ly - 1), tGy(lx, ly + 1), tGy(lx, ly + 2));
    dl = dl + (P.c4b * ((T(3) * p0) * p0 - T(1))) * mub;
    dl = dl - P.kappa * iso_lap<T>(tMb, lx, ly);
    if (STAGE == 3) {
      Wk.phi2_b[id] = (T(2) * Wk.phi_b[id]) / T(3) + dl;
    } else if (STAGE == 2) {
      Wk.phi1_b[id] = Wk.phi2_b[id] * T(0.25) + dl;
    } else {
      Wk.phib_b[id] = ((Wk.phi_b[id] / T(3) + Wk.phi2_b[id] * T(0.75)) + Wk.phi1_b[id]) + dl;
    }
    const T dmu_dc4b = (p0 * p0) * p0 - p0;
    const T dmu_dkap = -iso_lap<T>(tP, lx, ly);
    Wk.sig[id] = Wk.sig[id] + double(mub * dmu_dc4b) * C.dc4b + double(mub * dmu_dkap) * C.dkap;
  }
}

// ------------------------------------------- a1^T: gather and streaming
// phi_bar = sum f_i, p = sum g_i / 3, j = sum g_i c_i reversed, added to the
// canonical slot each pre-collision population streamed from (used once, at
// the end of the reverse sweep; in between, the collision adds these terms).
template <typename T, bool COUPLED>
__global__ __launch_bounds__(256) void k_adj_gather(KParams<T> P, const T* __restrict__ phib_b,
                                                    T* __restrict__ Afo, T* __restrict__ Ago,
                                                    AdjWork<T> Wk) {
  LBM2P_ADJ_CONTRACT
  const long long n = (long long)P.nx * P.ny;
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= n) return;
  const int y = (int)(id / P.nx), x = (int)(id - (long long)y * P.nx);
  const T pb = phib_b[id];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const long long s = src_slot(P, i, x, y);
    Afo[s] = Afo[s] + pb;
  }
  if (!COUPLED) return;
  const T q = Wk.praw_b[id] / T(3), jx = Wk.jx_b[id], jy = Wk.jy_b[id];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const long long s = src_slot(P, i, x, y);
    Ago[s] = Ago[s] + (q + cdot(i, jx, jy));
  }
}

// --------------------------------------------------- initial state^T
// f* = f^eq(phi0, mu(phi0), u0): the pointwise reverse (phi, mu, eta), then
// phi0_bar with the transposed Laplacian of mu_bar.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_init_a(KParams<T> P, AdjConst C,
                                                    const double* __restrict__ phi0,
                                                    const double* __restrict__ ux0,
                                                    const double* __restrict__ uy0,
                                                    const T* __restrict__ Af, AdjWork<T> Wk) {
  LBM2P_ADJ_CONTRACT
  const long long n = (long long)P.nx * P.ny;
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= n) return;
  const int y = (int)(id / P.nx), x = (int)(id - (long long)y * P.nx);
  struct G {
    const double* a;
    const KParams<T>* P;
    __device__ double operator()(int xx, int yy) const {
      int flip = 0;
      const int i = map_idx(xx, P->nx, P->wx, flip);
      const int j = map_idx(yy, P->ny, P->wy, flip);
      return a[(long long)j * P->nx + i];
    }
  } g{phi0, &P};
  const T ph = T(phi0[id]);
  const T mu = T(chem_pot<double>(g, x, y, C.c4b, C.kappa));
  const T u_x = ux0 ? T(ux0[id]) : T(0), u_y = uy0 ? T(uy0[id]) : T(0);
  T fb[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) fb[i] = Af[i * P.ps + id];
  T phb = T(0), mub = T(0), ubx = T(0), uby = T(0), etab = T(0);
  f_eq_adj<T>(ph, mu, u_x, u_y, P.eta, fb, phb, mub, ubx, uby, etab);
  Wk.fd_loc[id] = phb;
  Wk.fd_mu[id] = mub;
  const double p0 = phi0[id];
  const double dmu_dc4b = (p0 * p0) * p0 - p0;
  const double dmu_dkap = -iso_lap<double>(g, x, y);
  Wk.sig[id] = Wk.sig[id] + double(mub) * dmu_dc4b * C.dc4b + double(mub) * dmu_dkap * C.dkap;
  Wk.dM[id] = Wk.dM[id] + double(etab) * C.deta;
}

// (add: dL/dphi of a zero-step run, whose phi is phi0 itself; may be NULL)
template <typename T>
__global__ __launch_bounds__(256) void k_adj_init_b(KParams<T> P, const double* __restrict__ phi0,
                                                    const double* __restrict__ add,
                                                    double* __restrict__ out, AdjWork<T> Wk) {
  const long long n = (long long)P.nx * P.ny;
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= n) return;
  const int y = (int)(id / P.nx), x = (int)(id - (long long)y * P.nx);
  const T p0 = T(phi0[id]);
  T r = Wk.fd_loc[id] + (P.c4b * ((T(3) * p0) * p0 - T(1))) * Wk.fd_mu[id];
  r = r - P.kappa * iso_lap<T>(eread(Wk.fd_mu, P, false), x, y);
  out[id] = add ? double(r) + add[id] : double(r);
}

// deterministic sum of a float64 plane: per-block partials in a fixed tree
// order, then one block over the partials (one copy per translation unit)
namespace {
__global__ __launch_bounds__(256) void k_sum1(const double* __restrict__ a, long long n,
                                              double* __restrict__ part) {
  __shared__ double s[256];
  double acc = 0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)gridDim.x * 256)
    acc += a[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void k_sum2(const double* __restrict__ part, int nb,
                                              double* __restrict__ out) {
  __shared__ double s[256];
  double acc = 0;
  for (int b = threadIdx.x; b < nb; b += 256) acc += part[b];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0];
}
}  // namespace

}  // namespace lbm2p

