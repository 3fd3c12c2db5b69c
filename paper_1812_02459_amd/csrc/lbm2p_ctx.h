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
  void* U[2][2];   // filtered velocity, double buffered (u~^n and u~^{n+1})
  double* red;     // reduction partials (+ 8 results)
  int uo;          // index of u~^n in U
  int uk_last;     // index of the last velocity iterate in uk
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
  std::vector<double> ctab_host;
  double ca[6];
  double cfac[2][2], cden[2][2];
  size_t ctab_off[2][2];  // offsets (in doubles) of each (axis, parity) table
  int ctab_n[2];
  int ctab_uploaded;
  // profiling
  int prof_pass;
  std::vector<hipEvent_t> ev0, ev1;
  size_t prof_n;
};


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
  int state_##SUF(lbm2p_ctx*, double*, double*, double*, int);                    \
  int to_f64_##SUF(lbm2p_ctx*, const void*, double*);
LBM2P_DECLARE(f64)
LBM2P_DECLARE(f32)
#undef LBM2P_DECLARE

}  // namespace lbm2p
