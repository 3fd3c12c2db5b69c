// Host orchestration of the adjoint: the recorded forward run with its
// checkpoints (its last segment's steps write their intermediates to the
// per-step slots), and the reverse sweep segment by segment (recompute the
// segment's steps into the slots unless they are still there, then reverse
// them last to first).
// Included once per precision translation unit, after lbm2p_impl.h.
#pragma once

#include "lbm2p_impl.h"

namespace lbm2p {
namespace {

// Tiles (rows of 64 nodes, threads per workgroup) of the tiled reverse kernels,
// per precision.  The adjoint's passes chain several load / sync / compute
// phases, and many waves per tile hide their latency on grids of a few 10^5
// nodes; measured on the 256 x 1024 rising bubble, FP32 gains from 1024-thread
// tiles everywhere, the FP64 reverse collision (252 VGPRs) loses to register
// pressure there.
template <int TY_, int NT_>
struct AdjTile {
  static constexpr int TY = TY_, NT = NT_;
};
template <typename T>
struct AdjCfg {
  using Col = AdjTile<16, 1024>;
  using Vel = AdjTile<16, 1024>;
  using Phi = AdjTile<16, 1024>;
  using Fil = AdjTile<16, 1024>;
  using Fd = AdjTile<16, 512>;
};
template <>
struct AdjCfg<double> {
  using Col = AdjTile<8, 512>;
  using Vel = AdjTile<16, 1024>;
  using Fd = AdjTile<16, 1024>;
  using Phi = AdjTile<16, 1024>;   // 512 or 256 threads measured slower
  using Fil = AdjTile<16, 1024>;
};

// planes of one recorded step
template <typename T>
struct Slot {
  T *phibar, *phi1, *phi2, *phi, *praw, *pt, *utx, *uty, *m7, *m8;
  T* u[8][2];  // u^1 .. u^{K-1}
};

template <typename T>
struct AdjPtrs {
  AdjLayout L;
  char* base;
  T* ckpt(int i) const { return (T*)(base + L.ckpt + (size_t)i * L.cpp * L.plane); }
  T* plane(size_t off, int i) const { return (T*)(base + off + (size_t)i * L.plane); }
  Slot<T> slot(int j, const lbm2p_params& p) const {
    Slot<T> s{};
    T* b = (T*)(base + L.slot + (size_t)j * L.slp * L.plane);
    const long long ps = (long long)(L.plane / sizeof(T));
    int k = 0;
    s.phibar = b + (k++) * ps;
    s.phi1 = b + (k++) * ps;
    s.phi2 = b + (k++) * ps;
    s.phi = b + (k++) * ps;
    if (p.coupled) {
      s.praw = b + (k++) * ps;
      for (int i = 1; i < p.K; ++i) {
        s.u[i][0] = b + (k++) * ps;
        s.u[i][1] = b + (k++) * ps;
      }
      s.pt = b + (k++) * ps;
      s.utx = b + (k++) * ps;
      s.uty = b + (k++) * ps;
      s.m7 = b + (k++) * ps;
      s.m8 = b + (k++) * ps;
    }
    return s;
  }
  // adjoint state copy a: f (9 planes), g (9, coupled), u (2)
  T* astate(int a) const { return (T*)(base + L.astate + (size_t)a * (L.sp + 2) * L.plane); }
  double* dbl() const { return (double*)(base + L.dbl); }
};

template <typename T>
AdjWork<T> adj_work(const AdjPtrs<T>& A) {
  AdjWork<T> w;
  int k = 0;
  auto nx = [&]() { return A.plane(A.L.work, k++); };
  w.lp_p = nx(); w.lp_ux = nx(); w.lp_uy = nx(); w.dp_x = nx(); w.dp_y = nx();
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 4; ++b) w.du[a][b] = nx();
  w.a_phi = nx(); w.a_mu = nx(); w.a_grx = nx(); w.a_gry = nx(); w.a_dmx = nx(); w.a_dmy = nx();
  for (int b = 0; b < 4; ++b) w.a_Q[b] = nx();
  w.mu_b = nx(); w.rho_b = nx(); w.px_b = nx(); w.py_b = nx();
  w.pt_b = nx(); w.utx_b = nx(); w.uty_b = nx(); w.ukx_b = nx(); w.uky_b = nx();
  w.praw_b = nx(); w.jx_b = nx(); w.jy_b = nx();
  w.phi_b = nx(); w.phi2_b = nx(); w.phi1_b = nx(); w.phib_b = nx();
  w.fd_gx = nx(); w.fd_gy = nx(); w.fd_mx = nx(); w.fd_my = nx(); w.fd_loc = nx(); w.fd_mu = nx();
  w.sig = A.dbl();
  w.dM = A.dbl() + (size_t)(A.L.plane / sizeof(T));
  return w;
}

inline AdjConst adj_const(const lbm2p_ctx* c) {
  const lbm2p_params& p = c->p;
  AdjConst C;
  C.dc4b = 3.0 / p.W;
  C.dkap = 3.0 * p.W / 8.0;
  C.deta = 3.0 / (p.tau_f - 0.5);
  C.dcJ = (p.rho1 - p.rho2) / 2.0;
  C.c4b = c->c4b;
  C.kappa = c->kappa;
  return C;
}

// checkpoint i <- current state (populations in the AA layout, u~, phi, p~)
template <typename T>
void save_ckpt(lbm2p_ctx* c, const AdjPtrs<T>& A, int i) {
  const long long ps = c->ps;
  T* d = A.ckpt(i);
  const int nd = c->p.coupled ? 2 : 1;
  k_copy<T><<<blocks1d(9 * ps), 256, 0, c->stream>>>((const T*)c->Af, d, 9 * ps);
  if (nd == 2) k_copy<T><<<blocks1d(9 * ps), 256, 0, c->stream>>>((const T*)c->Ag, d + 9 * ps, 9 * ps);
  T* u = d + 9 * nd * ps;
  const int ui = c->p.coupled ? c->uo : 0;
  k_copy<T><<<blocks1d(ps), 256, 0, c->stream>>>((const T*)c->U[ui][0], u, ps);
  k_copy<T><<<blocks1d(ps), 256, 0, c->stream>>>((const T*)c->U[ui][1], u + ps, ps);
  k_copy<T><<<blocks1d(ps), 256, 0, c->stream>>>((const T*)c->phi, u + 2 * ps, ps);
  if (c->p.coupled) k_copy<T><<<blocks1d(ps), 256, 0, c->stream>>>((const T*)c->pt, u + 3 * ps, ps);
}

// current state <- checkpoint i (u~ into U[0]; the context's own planes)
template <typename T>
void load_ckpt(lbm2p_ctx* c, const AdjPtrs<T>& A, int i, int parity, bool fields) {
  const long long ps = c->ps;
  const T* d = A.ckpt(i);
  const int nd = c->p.coupled ? 2 : 1;
  k_copy<T><<<blocks1d(9 * ps), 256, 0, c->stream>>>(d, (T*)c->Af, 9 * ps);
  if (nd == 2) k_copy<T><<<blocks1d(9 * ps), 256, 0, c->stream>>>(d + 9 * ps, (T*)c->Ag, 9 * ps);
  const T* u = d + 9 * nd * ps;
  if (c->p.coupled) {
    k_copy<T><<<blocks1d(ps), 256, 0, c->stream>>>(u, (T*)c->U[0][0], ps);
    k_copy<T><<<blocks1d(ps), 256, 0, c->stream>>>(u + ps, (T*)c->U[0][1], ps);
  }
  if (fields) {
    k_copy<T><<<blocks1d(ps), 256, 0, c->stream>>>(u + 2 * ps, (T*)c->phi, ps);
    if (c->p.coupled) k_copy<T><<<blocks1d(ps), 256, 0, c->stream>>>(u + 3 * ps, (T*)c->pt, ps);
  }
  c->parity = parity;
  c->uo = 0;
}

// The context's own planes, which a recomputed (or recorded-and-kept) step
// is rebound away from, slot by slot.
struct OwnPlanes {
  void *phibar, *phi1, *phi2, *phi, *praw, *pt;
  void* U[2][2];
};
inline OwnPlanes own_planes(const lbm2p_ctx* c) {
  return OwnPlanes{c->phibar, c->phi1, c->phi2, c->phi, c->praw, c->pt,
                   {{c->U[0][0], c->U[0][1]}, {c->U[1][0], c->U[1][1]}}};
}
inline void restore_planes(lbm2p_ctx* c, const OwnPlanes& o) {
  c->phibar = o.phibar;
  c->phi1 = o.phi1;
  c->phi2 = o.phi2;
  c->phi = o.phi;
  c->praw = o.praw;
  c->pt = o.pt;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) c->U[a][b] = o.U[a][b];
}
// The next step writes its intermediates to slot j: phi_bar, phi^(1), phi^(2),
// phi, p, p~, u~ (as the state's next velocity plane), the iterates and m7, m8.
template <typename T>
void bind_slot(lbm2p_ctx* c, const AdjPtrs<T>& A, int j) {
  const lbm2p_params& p = c->p;
  const Slot<T> sl = A.slot(j, p);
  c->phibar = sl.phibar;
  c->phi1 = sl.phi1;
  c->phi2 = sl.phi2;
  c->phi = sl.phi;
  if (p.coupled) {
    c->praw = sl.praw;
    c->pt = sl.pt;
    c->U[1 - c->uo][0] = sl.utx;
    c->U[1 - c->uo][1] = sl.uty;
    for (int i = 1; i < p.K; ++i) {
      c->rec_uk[i - 1][0] = sl.u[i][0];
      c->rec_uk[i - 1][1] = sl.u[i][1];
    }
    c->rec_uk[p.K - 1][0] = c->uk[0][0];
    c->rec_uk[p.K - 1][1] = c->uk[0][1];
    c->rec_m7 = sl.m7;
    c->rec_m8 = sl.m8;
  }
}

template <typename T>
int record_impl(lbm2p_ctx* c, int nsteps, int k) {
  AdjPtrs<T> A{adj_layout(c->p, c->ps, c->n, c->esz, nsteps, k), c->adj_ws};
  c->adj_ready = 0;
  c->adj_nsteps = nsteps;
  c->adj_k = k;
  c->adj_from_init = c->from_init && c->steps == 0;
  c->adj_parity0 = c->parity;
  c->adj_last_kept = 0;
  save_ckpt<T>(c, A, 0);
  // The last segment is the first one reversed: its steps write their
  // intermediates to the slots now, so the adjoint need not recompute it.
  const int s_last = nsteps > 0 ? (A.L.nseg - 1) * k : 0;
  const OwnPlanes own = own_planes(c);
  for (int s = 0; s < nsteps; ++s) {
    if (s >= s_last) {
      c->rec = 1;
      bind_slot<T>(c, A, s - s_last);
    }
    const int e = step_impl<T>(c, 1);
    if (e) {
      c->rec = 0;
      restore_planes(c, own);
      return e;
    }
    if ((s + 1) % k == 0 && s + 1 < nsteps) save_ckpt<T>(c, A, (s + 1) / k);
  }
  save_ckpt<T>(c, A, A.L.nseg);
  if (nsteps > 0) {
    // back to the context's own planes, holding the final state
    c->rec = 0;
    restore_planes(c, own);
    load_ckpt<T>(c, A, A.L.nseg, c->adj_parity0 ^ (nsteps & 1), true);
    c->adj_last_kept = 1;
  }
  c->adj_steps_end = c->steps;
  c->adj_ready = 1;
  return hipGetLastError() == hipSuccess ? LBM2P_OK : LBM2P_EHIP;
}

// Adjoint planes of the gather of the step reversed last (phi_bar, p, j),
// which the next reversed collision adds to its slots; null before the first.
template <typename T>
struct Pending {
  const T *phi, *p, *jx, *jy;
};

template <typename T, bool COUPLED, bool PEND>
void launch_adj_collide(lbm2p_ctx* c, const KParams<T>& K, const AdjConst& C,
                        const AdjWork<T>& Wk, const Slot<T>& sl, const T* ux, const T* uy,
                        const T* uox, const T* uoy, const T* Afi, const T* Agi,
                        const Pending<T>& pd, T* Afo, T* Ago, T* Uox, T* Uoy) {
  using AdjCol = typename AdjCfg<T>::Col;
  const Tiles<64, AdjCol::TY> tc(c->p);
  k_adj_collide<T, COUPLED, PEND, 64, AdjCol::TY, AdjCol::NT><<<tc.grid(), AdjCol::NT, 0, c->stream>>>(
      K, C, tc.tx, sl.phi, sl.pt, ux, uy, uox, uoy, sl.m7, sl.m8, Afi, Agi, pd.phi, pd.p, pd.jx,
      pd.jy, Afo, Ago, Uox, Uoy, Wk);
}

// one reverse step: adjoint state in (ai) -> out (1 - ai); returns the
// gather adjoints left for the next reversed collision
template <typename T>
Pending<T> adj_step(lbm2p_ctx* c, const AdjPtrs<T>& A, const AdjWork<T>& Wk, const Slot<T>& sl,
                    const T* uox, const T* uoy, const double* seed, int ai, const Pending<T>& pd) {
  const lbm2p_params& p = c->p;
  const KParams<T> K = kparams<T>(c);
  const AdjConst C = adj_const(c);
  hipStream_t st = c->stream;
  const long long ps = c->ps;
  T* Ai = A.astate(ai);
  T* Ao = A.astate(1 - ai);
  const int sp = A.L.sp;
  const T* Afi = Ai;
  const T* Agi = p.coupled ? Ai + 9 * ps : nullptr;
  const T* Uix = Ai + sp * ps;
  const T* Uiy = Uix + ps;
  T* Afo = Ao;
  T* Ago = p.coupled ? Ao + 9 * ps : nullptr;
  T* Uox = Ao + sp * ps;
  T* Uoy = Uox + ps;
  const bool pend = pd.phi != nullptr;
  using AdjPhi = typename AdjCfg<T>::Phi;
  using AdjFil = typename AdjCfg<T>::Fil;
  const Tiles<64, AdjPhi::TY> t16(p);
  if (p.coupled) {
    if (pend)
      launch_adj_collide<T, true, true>(c, K, C, Wk, sl, sl.utx, sl.uty, uox, uoy, Afi, Agi, pd,
                                        Afo, Ago, Uox, Uoy);
    else
      launch_adj_collide<T, true, false>(c, K, C, Wk, sl, sl.utx, sl.uty, uox, uoy, Afi, Agi, pd,
                                         Afo, Ago, Uox, Uoy);
    const Tiles<64, AdjFil::TY> tf(p);
    T* ob[3] = {Wk.praw_b, Wk.ukx_b, Wk.uky_b};
    if (p.compact) {
      // The compact filter per direction, F = A^-1 B, is self-adjoint: the line
      // matrix A and the right-hand-side stencil B are both symmetric stencils
      // on the mirrored (wall) or periodic line, so they commute and
      // (A^-1 B)^T = B A^-1 = A^-1 B.  The reverse of the update is therefore
      // the update itself, applied to the adjoints of p~, u~ (same parities).
      k_adj_filter_t<T, 0, 64, AdjFil::TY, AdjFil::NT><<<tf.grid(), AdjFil::NT, 0, st>>>(
          K, tf.tx, Uix, Uiy, Wk, Wk.lp_p, Wk.lp_ux, Wk.lp_uy);
      switch (p.compact_n) {
        case 1: launch_compact<T, 1>(c, K, Wk.lp_p, Wk.lp_ux, Wk.lp_uy, ob[0], ob[1], ob[2]); break;
        case 2: launch_compact<T, 2>(c, K, Wk.lp_p, Wk.lp_ux, Wk.lp_uy, ob[0], ob[1], ob[2]); break;
        case 3: launch_compact<T, 3>(c, K, Wk.lp_p, Wk.lp_ux, Wk.lp_uy, ob[0], ob[1], ob[2]); break;
        case 4: launch_compact<T, 4>(c, K, Wk.lp_p, Wk.lp_ux, Wk.lp_uy, ob[0], ob[1], ob[2]); break;
        default: launch_compact<T, 5>(c, K, Wk.lp_p, Wk.lp_ux, Wk.lp_uy, ob[0], ob[1], ob[2]); break;
      }
    } else {
      switch (p.filter_n ? c->fn : 0) {
        case 0: k_adj_filter_t<T, 0, 64, AdjFil::TY, AdjFil::NT><<<tf.grid(), AdjFil::NT, 0, st>>>(K, tf.tx, Uix, Uiy, Wk, ob[0], ob[1], ob[2]); break;
        case 2: k_adj_filter_t<T, 2, 64, AdjFil::TY, AdjFil::NT><<<tf.grid(), AdjFil::NT, 0, st>>>(K, tf.tx, Uix, Uiy, Wk, ob[0], ob[1], ob[2]); break;
        case 3: k_adj_filter_t<T, 3, 64, AdjFil::TY, AdjFil::NT><<<tf.grid(), AdjFil::NT, 0, st>>>(K, tf.tx, Uix, Uiy, Wk, ob[0], ob[1], ob[2]); break;
        case 4: k_adj_filter_t<T, 4, 64, AdjFil::TY, AdjFil::NT><<<tf.grid(), AdjFil::NT, 0, st>>>(K, tf.tx, Uix, Uiy, Wk, ob[0], ob[1], ob[2]); break;
        default: k_adj_filter_t<T, 5, 64, AdjFil::TY, AdjFil::NT><<<tf.grid(), AdjFil::NT, 0, st>>>(K, tf.tx, Uix, Uiy, Wk, ob[0], ob[1], ob[2]); break;
      }
    }
    // velocity sweeps last to first; sweep k reads u^k (u^0 = u~^n)
    int cur = 0;
    using AdjVel = typename AdjCfg<T>::Vel;
    const Tiles<64, AdjVel::TY> tv(p);
    for (int k = p.K - 1; k >= 0; --k) {
      const T* ux = k == 0 ? uox : sl.u[k][0];
      const T* uy = k == 0 ? uoy : sl.u[k][1];
      if (k == p.K - 1) {
        k_adj_vel<T, true, 64, AdjVel::TY, AdjVel::NT><<<tv.grid(), AdjVel::NT, 0, st>>>(K, C, tv.tx, sl.phi, sl.praw,
                                                                      ux, uy, 1, Wk);
        cur = 0;
      } else {
        k_adj_vel<T, false, 64, AdjVel::TY, AdjVel::NT><<<tv.grid(), AdjVel::NT, 0, st>>>(K, C, tv.tx, sl.phi,
                                                                       sl.praw, ux, uy, cur, Wk);
        cur = 1 - cur;
      }
    }
    k_adj_phi<T, true, 64, AdjPhi::TY, AdjPhi::NT><<<t16.grid(), AdjPhi::NT, 0, st>>>(K, C, t16.tx, sl.phi, cur, seed,
                                                                 Uox, Uoy, Wk);
  } else {
    const T* ux = (const T*)c->U[0][0];
    const T* uy = (const T*)c->U[0][1];
    if (pend)
      launch_adj_collide<T, false, true>(c, K, C, Wk, sl, ux, uy, ux, uy, Afi, nullptr, pd, Afo,
                                         nullptr, nullptr, nullptr);
    else
      launch_adj_collide<T, false, false>(c, K, C, Wk, sl, ux, uy, ux, uy, Afi, nullptr, pd, Afo,
                                          nullptr, nullptr, nullptr);
    k_adj_phi<T, false, 64, AdjPhi::TY, AdjPhi::NT><<<t16.grid(), AdjPhi::NT, 0, st>>>(K, C, t16.tx, sl.phi, 0, seed,
                                                                  nullptr, nullptr, Wk);
  }
  const T* phib = Wk.phi_b;
  if (!p.original_ch) {
    using AdjFd = typename AdjCfg<T>::Fd;
    constexpr int TY = AdjFd::TY, NTF = AdjFd::NT;
    const Tiles<64, TY> tf(p);
    k_adj_fd<T, 3, 64, TY, NTF><<<tf.grid(), NTF, 0, st>>>(K, C, tf.tx, sl.phi2, Wk.phi_b,
                                                      T(2.0 / 3.0), Wk);
    k_adj_fd<T, 2, 64, TY, NTF><<<tf.grid(), NTF, 0, st>>>(K, C, tf.tx, sl.phi1, Wk.phi2_b, T(0.25),
                                                      Wk);
    k_adj_fd<T, 1, 64, TY, NTF><<<tf.grid(), NTF, 0, st>>>(K, C, tf.tx, sl.phibar, Wk.phi1_b, T(1),
                                                      Wk);
    phib = Wk.phib_b;
  }
  Pending<T> out{phib, nullptr, nullptr, nullptr};
  if (p.coupled) {
    out.p = Wk.praw_b;
    out.jx = Wk.jx_b;
    out.jy = Wk.jy_b;
  }
  (void)Ago;
  return out;
}

template <typename T>
int adjoint_impl(lbm2p_ctx* c, lbm2p_adjoint_io* io) {
  const lbm2p_params& p = c->p;
  const int nsteps = c->adj_nsteps, k = c->adj_k;
  AdjPtrs<T> A{adj_layout(p, c->ps, c->n, c->esz, nsteps, k), c->adj_ws};
  const AdjWork<T> Wk = adj_work<T>(A);
  const long long n = c->n, ps = c->ps;
  hipStream_t st = c->stream;
  const int sp = A.L.sp;
  // seeds into adjoint state 0; zero the parameter partials
  T* A0 = A.astate(0);
  k_fill<T><<<blocks1d((sp + 2) * ps), 256, 0, st>>>(A0, T(0), (sp + 2) * ps);
  k_fill<double><<<blocks1d(2 * ps), 256, 0, st>>>(A.dbl(), 0.0, 2 * ps);
  for (int i = 0; i < 9; ++i) {
    if (io->dL_df)
      k_from_f64<T><<<blocks1d(n), 256, 0, st>>>(io->dL_df + i * n, A0 + i * ps, n);
    if (p.coupled && io->dL_dg)
      k_from_f64<T><<<blocks1d(n), 256, 0, st>>>(io->dL_dg + i * n, A0 + (9 + i) * ps, n);
  }
  if (p.coupled && io->dL_du)
    for (int d = 0; d < 2; ++d)
      k_from_f64<T><<<blocks1d(n), 256, 0, st>>>(io->dL_du + d * n, A0 + (sp + d) * ps, n);
  // the context's own planes, rebound per recomputed step
  const OwnPlanes own = own_planes(c);
  int ai = 0;
  Pending<T> pd{nullptr, nullptr, nullptr, nullptr};
  const int nseg = A.L.nseg;
  // Segment s keeps its step j in slot m(s, j): the last segment in step
  // order, the ones before it alternating.  The recompute of segment s - 1
  // (forward in time) then fills slot m(s - 1, i) = the slot the reverse of
  // segment s (backward in time) releases at its step k - 1 - i, so with a
  // second stream the two run side by side, each recomputed step waiting only
  // for the reverse step that frees its slot.  The recomputes use the
  // context's planes and the reverse sweep does not (coupled step, explicit
  // filter: the compact filter's scratch is shared, so it takes one stream).
  auto slot_of = [&](int s, int j) { return ((nseg - 1 - s) & 1) ? k - 1 - j : j; };
  auto seg_len = [&](int s) { return std::min(k, nsteps - s * k); };
  bool overlap = p.coupled && !p.compact && nseg > 1;
  if (overlap && !c->adj_stream &&
      hipStreamCreateWithFlags(&c->adj_stream, hipStreamNonBlocking) != hipSuccess) {
    c->adj_stream = nullptr;
    overlap = false;
  }
  while (overlap && c->adj_ev.size() < (size_t)k + 2) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      overlap = false;
      break;
    }
    c->adj_ev.push_back(e);
  }
  hipStream_t sb = overlap ? c->adj_stream : st;
  // recompute of segment s on stream sb: its checkpoint, then step by step
  auto recompute_begin = [&](int s) {
    restore_planes(c, own);
    c->stream = sb;
    load_ckpt<T>(c, A, s, c->adj_parity0 ^ ((s * k) & 1), false);
    c->stream = st;
  };
  auto recompute_step = [&](int s, int i) {
    c->stream = sb;
    c->rec = 1;
    bind_slot<T>(c, A, slot_of(s, i));
    const int e = step_impl<T>(c, 1);
    c->rec = 0;
    c->stream = st;
    return e;
  };
  auto fail = [&](int e) {
    c->stream = st;
    c->rec = 0;
    restore_planes(c, own);
    if (overlap) hipStreamSynchronize(sb);
    return e;
  };
  if (nseg > 0) {
    if (c->adj_last_kept) {
      // kept by the record; the recomputes below reuse the slots
      if (nseg > 1) c->adj_last_kept = 0;
    } else {
      hipStream_t keep = sb;
      sb = st;
      recompute_begin(nseg - 1);
      for (int i = 0; i < seg_len(nseg - 1); ++i) {
        const int e = recompute_step(nseg - 1, i);
        if (e) return fail(e);
      }
      sb = keep;
    }
  }
  if (overlap) {
    // the second stream starts after everything issued so far
    if (hipEventRecord(c->adj_ev[k], st) != hipSuccess ||
        hipStreamWaitEvent(sb, c->adj_ev[k], 0) != hipSuccess)
      return fail(LBM2P_EHIP);
  }
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int s0 = seg * k;
    const int len = seg_len(seg);
    const T* cku = A.ckpt(seg) + (size_t)9 * (p.coupled ? 2 : 1) * ps;
    // the recompute of the segment before, alongside (its steps whose slots
    // this segment leaves unused start at once)
    const bool pre = overlap && seg > 0;
    int inext = 0;
    if (pre) {
      recompute_begin(seg - 1);
      for (; inext < seg_len(seg - 1) && k - 1 - inext >= len; ++inext) {
        const int e = recompute_step(seg - 1, inext);
        if (e) return fail(e);
      }
    }
    for (int j = len - 1; j >= 0; --j) {
      const Slot<T> sl = A.slot(slot_of(seg, j), p);
      const T* uox = nullptr;
      const T* uoy = nullptr;
      if (p.coupled) {
        if (j == 0) {
          uox = cku;
          uoy = cku + ps;
        } else {
          const Slot<T> pr = A.slot(slot_of(seg, j - 1), p);
          uox = pr.utx;
          uoy = pr.uty;
        }
      }
      const double* seed = (s0 + j == nsteps - 1) ? io->dL_dphi : nullptr;
      pd = adj_step<T>(c, A, Wk, sl, uox, uoy, seed, ai, pd);
      ai = 1 - ai;
      if (pre && k - 1 - j == inext && inext < seg_len(seg - 1)) {
        // slot m(seg, j) released: the recompute step that fills it
        if (hipEventRecord(c->adj_ev[j], st) != hipSuccess ||
            hipStreamWaitEvent(sb, c->adj_ev[j], 0) != hipSuccess)
          return fail(LBM2P_EHIP);
        const int e = recompute_step(seg - 1, inext++);
        if (e) return fail(e);
      }
    }
    if (pre) {
      // the reverse of the segment before waits for its recompute
      if (hipEventRecord(c->adj_ev[k + 1], sb) != hipSuccess ||
          hipStreamWaitEvent(st, c->adj_ev[k + 1], 0) != hipSuccess)
        return fail(LBM2P_EHIP);
    } else if (seg > 0) {
      recompute_begin(seg - 1);
      for (int i = 0; i < seg_len(seg - 1); ++i) {
        const int e = recompute_step(seg - 1, i);
        if (e) return fail(e);
      }
    }
  }
  // back to the context's own planes and the recorded final state
  restore_planes(c, own);
  load_ckpt<T>(c, A, A.L.nseg, c->adj_parity0 ^ (nsteps & 1), true);
  c->steps = c->adj_steps_end;
  // outputs: the first step's gather adjoint completes the initial state's
  const KParams<T> K = kparams<T>(c);
  T* Af = A.astate(ai);
  if (pd.phi) {
    if (p.coupled)
      k_adj_gather<T, true><<<blocks1d(n), 256, 0, st>>>(K, pd.phi, Af, Af + 9 * ps, Wk);
    else
      k_adj_gather<T, false><<<blocks1d(n), 256, 0, st>>>(K, pd.phi, Af, nullptr, Wk);
  }
  for (int i = 0; i < 9; ++i) {
    if (io->dL_df0) k_to_f64<T><<<blocks1d(n), 256, 0, st>>>(Af + i * ps, io->dL_df0 + i * n, n);
    if (p.coupled && io->dL_dg0)
      k_to_f64<T><<<blocks1d(n), 256, 0, st>>>(Af + (9 + i) * ps, io->dL_dg0 + i * n, n);
  }
  if (io->dL_du0) {
    for (int d = 0; d < 2; ++d) {
      if (p.coupled)
        k_to_f64<T><<<blocks1d(n), 256, 0, st>>>(Af + (sp + d) * ps, io->dL_du0 + d * n, n);
      else
        k_fill<double><<<blocks1d(n), 256, 0, st>>>(io->dL_du0 + d * n, 0.0, n);
    }
  }
  if (io->dL_dphi0) {
    k_adj_init_a<T><<<blocks1d(n), 256, 0, st>>>(K, adj_const(c), io->phi0, io->ux0, io->uy0, Af,
                                                 Wk);
    k_adj_init_b<T><<<blocks1d(n), 256, 0, st>>>(K, io->phi0, nsteps == 0 ? io->dL_dphi : nullptr,
                                                 io->dL_dphi0, Wk);
  }
  double* part = A.dbl() + 2 * ps;
  double* res = part + 1024;
  k_sum1<<<1024, 256, 0, st>>>(Wk.sig, n, part);
  k_sum2<<<1, 256, 0, st>>>(part, 1024, res);
  k_sum1<<<1024, 256, 0, st>>>(Wk.dM, n, part);
  k_sum2<<<1, 256, 0, st>>>(part, 1024, res + 1);
  double h[2];
  if (hipMemcpyAsync(h, res, 2 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess)
    return LBM2P_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return LBM2P_EHIP;
  io->dL_dsigma = h[0];
  io->dL_dM = h[1];
  return hipGetLastError() == hipSuccess ? LBM2P_OK : LBM2P_EHIP;
}

}  // namespace
}  // namespace lbm2p
