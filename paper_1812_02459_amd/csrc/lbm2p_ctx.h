// Context of the C ABI and the precision-specific entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/lbm2p.h"

struct lbm2p_ctx {
  lbm2p_params p;
  int prec;  // 0 fp64, 1 fp32
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  long long n, ps;
  size_t esz;
  // fields (in the context's precision)
  void *Af, *Ag, *phi, *phibar, *phi1, *phi2, *praw, *jx, *jy, *pt;
  void* uk[2][2];  // velocity iterates
  void *sm1, *sm7, *sm8;  // moments m_1, m_7, m_8 of the pre-collision g (moment strain rate)
  void* U[2][2];   // filtered velocity, double buffered (u~^n and u~^{n+1})
  double* red;     // reduction partials (+ 8 results)
  int uo;          // index of u~^n in U
  // CH-only mode: the prescribed velocity is U[0]; after lbm2p_set_velocity
  // (vpend = 1) U[1] holds the velocity the last step used, for d_t u
  int vpend;
  int uk_last;     // index of the last velocity iterate in uk
  // velocity-iteration residual: with track_resid set, a step runs its last
  // sweep alone and leaves its input u^{K-1} and output u^K in these planes
  int track_resid, res_valid;
  void *res_prev[2], *res_last[2];
  int parity;
  int inited;
  long long steps;
  // derived constants (float64, computed exactly as the oracle computes them)
  double kappa, beta, eta, c4b, negM, cJ, eps2;
  double s_f[9], s_g[9];
  double fd[6];
  int fn;
  // compact filter: scratch planes (d, Fx, Fy; 3 fields each), line tables in
  // the workspace (device) and their host image, coefficients a_n
  void* cscratch;
  double* ctab_dev;
  double* cfct;  // room for the FP32 copy of the tables (6 (nx + ny) floats)
  std::vector<double> ctab_host;
  double ca[6];
  double cfac[2][2], cden[2][2];
  int cflat[2][2];        // first index of the tables' constant run (per axis, parity)
  int cz0[2][2], cz1[2][2];  // z_i negligible for cz0 <= i < cz1 (per axis, parity)
  size_t ctab_off[2][2];  // offsets (in doubles) of each (axis, parity) table
  int ctab_n[2];
  int ctab_uploaded;
  // profiling
  int prof_pass;
  std::vector<hipEvent_t> ev0, ev1;
  size_t prof_n;
  // adjoint: record mode of the step (every velocity sweep to its own plane,
  // the stress moments m7, m8 of the pre-collision g) and the recorded run
  int rec;
  void* rec_uk[8][2];
  void *rec_m7, *rec_m8;
  int from_init;          // the state is the one lbm2p_init_fields made
  char* adj_ws;
  size_t adj_bytes;
  int adj_nsteps, adj_k, adj_from_init, adj_parity0, adj_ready;
  int adj_last_kept;            // the slots hold the last recorded segment
  long long adj_steps_end;
  // adjoint: a second stream for the segment recomputes, and events ordering
  // them against the reverse sweep (created at the first adjoint that uses them)
  hipStream_t adj_stream;
  std::vector<hipEvent_t> adj_ev;
  // coupled mode: a second stream on which the gather of p and j runs beside
  // the FD stages (which need only phi_bar), and the events of that fork and
  // join (made by the first lbm2p_init_fields)
  hipStream_t g_stream;
  hipEvent_t g_ev[2];
};

namespace lbm2p {

// Layout of the adjoint workspace (byte offsets, each region 256-aligned):
//   checkpoints: ncp = segments + 1 states (populations, u~, and phi, p~ for
//                the final one), in the context's precision and AA layout;
//   slots:       k per-step records of a segment (phi_bar, phi^(1), phi^(2),
//                phi, then coupled: p, u^1..u^{K-1}, p~, u~, m7, m8);
//   adjoint state: two canonical copies of (f*, g*, u~) adjoints;
//   work:        the reverse step's planes;
//   float64:     per-node dL/dsigma, dL/dM partials and the reduction scratch.
struct AdjLayout {
  int nseg, ncp, sp, cpp, slp, wp;
  size_t plane, ckpt, slot, astate, work, dbl, total;
};

inline AdjLayout adj_layout(const lbm2p_params& p, long long ps, long long n, size_t esz,
                            int nsteps, int k) {
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  AdjLayout L;
  L.nseg = nsteps > 0 ? (nsteps + k - 1) / k : 0;
  L.ncp = L.nseg + 1;
  L.sp = p.coupled ? 18 : 9;
  L.cpp = L.sp + 4;
  L.slp = p.coupled ? 10 + 2 * (p.K - 1) : 4;
  L.wp = 45;
  L.plane = (size_t)ps * esz;
  const int kk = nsteps < k ? (nsteps > 0 ? nsteps : 1) : k;
  L.ckpt = 0;
  L.slot = al(L.ckpt + (size_t)L.ncp * L.cpp * L.plane);
  L.astate = al(L.slot + (size_t)kk * L.slp * L.plane);
  L.work = al(L.astate + (size_t)2 * (L.sp + 2) * L.plane);
  L.dbl = al(L.work + (size_t)L.wp * L.plane);
  L.total = al(L.dbl + ((size_t)2 * ps + 1024 + 64) * sizeof(double));
  return L;
}

}  // namespace lbm2p


namespace lbm2p {

// One set per precision; lbm2p_f64.hip is compiled without floating-point
// contraction (the FP64 path rounds exactly as written), lbm2p_f32.hip with
// contraction and fast single-precision division.
#define LBM2P_DECLARE(SUF)                                                        \
  int init_##SUF(lbm2p_ctx*, const double*, const double*, const double*,       \
                 const double*);                                                  \
  int step_##SUF(lbm2p_ctx*, int);                                                \
  int moments_##SUF(lbm2p_ctx*, double*, double*, double*, double*, double*);    \
  int volume_##SUF(lbm2p_ctx*, double*);                                          \
  int bubble_##SUF(lbm2p_ctx*, double*);                                          \
  int pjump_##SUF(lbm2p_ctx*, double*);                                           \
  int resid_##SUF(lbm2p_ctx*, double*);                                           \
  int state_##SUF(lbm2p_ctx*, double*, double*, double*, int);                    \
  int setvel_##SUF(lbm2p_ctx*, const double*, const double*);                     \
  int to_f64_##SUF(lbm2p_ctx*, const void*, double*);                             \
  int record_##SUF(lbm2p_ctx*, int, int);                                         \
  int adjoint_##SUF(lbm2p_ctx*, lbm2p_adjoint_io*);
LBM2P_DECLARE(f64)
LBM2P_DECLARE(f32)
#undef LBM2P_DECLARE

// the diagnostics of lbm2p_volume on float64 planes, partials in the FP64
// unit's static scratch (lbm2p_volume_noalloc)
int volume_noalloc_f64(const double* phi, const double* p, const double* ux, const double* uy,
                       long long n, double* out, hipStream_t stream);

}  // namespace lbm2p
