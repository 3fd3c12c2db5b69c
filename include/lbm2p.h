/*
 * lbm2p -- C ABI of the MI355X (gfx950) library for the fractional-step MRT
 * lattice Boltzmann method for two-phase flow with large density ratios
 * (Zhang, Guo & Li, arXiv:1812.02459).
 *
 * One call to lbm2p_step advances the whole D2Q9 lattice by one time step:
 *   1. streaming of the CH populations f and the pressure populations g and
 *      their moments phi_bar = sum f (eq:compute_phi), p = c_s^2 sum g (Eq:p),
 *      j = sum g c (Eq:u);
 *   2. the finite-difference sub-step of the split CH equation (eq:step2) with
 *      the interfacial-profile and flux corrections (eq:final_mCHE), TVD-RK3
 *      in time (eq:TVD-3order) and fourth-order central differences
 *      (eq:fourOrder_FDM);
 *   3. the velocity of Eq:u with the force F = F_p + F_s + F_nu + F_m + F_g
 *      (eq:reformNS, eq:surfaceforce) on the isotropic stencils of
 *      eq:dicretized, solved by K fixed-point iterations;
 *   4. the selective filter of (p, u) (eq:filter, App. B) or the compact
 *      (tridiagonal) variant;
 *   5. the MRT collision of f (eq:distribution_CH, eq:feq_CH, eq:Fi) and g
 *      (eq:distribution_NS, eq:geq, eq:Gi) with Lambda = M^-1 S M
 *      (eq:collison, eq:D2Q9MRT).
 * In CH-only mode (coupled = 0) steps 3-4 are skipped and the velocity is a
 * prescribed field (Sec. 4.1, 4.2).
 *
 * Conventions.
 *  - Every field crossing the ABI is a float64 plane [ny][nx], row-major
 *    (x fastest), in DEVICE memory owned by the caller.  The library keeps
 *    its own state in its precision (FP64 or FP32) inside the workspace.
 *  - The caller owns the workspace (device memory, >= lbm2p_workspace_bytes)
 *    and the HIP stream; the library allocates no device memory.  Pointers
 *    are borrowed for the duration of a call only (the workspace for the
 *    life of the context).
 *  - All calls enqueue work on the context's stream and return without
 *    waiting, except lbm2p_volume and lbm2p_profile_read, which synchronise
 *    the stream.  One context per stream; contexts share no state.
 *  - Every function returns LBM2P_OK (0) or an error code; no exception or
 *    abort crosses the ABI.  lbm2p_strerror names a code.
 */
#ifndef LBM2P_H
#define LBM2P_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBM2P_OK = 0,
  LBM2P_EINVAL = 1,      /* invalid argument or parameter                  */
  LBM2P_ENOSPACE = 2,    /* workspace smaller than lbm2p_workspace_bytes   */
  LBM2P_EHIP = 3,        /* a HIP runtime call failed                      */
  LBM2P_ENONFINITE = 4,  /* a diagnostic found NaN or Inf in the state     */
  LBM2P_ESTATE = 5       /* call out of order (e.g. step before init)      */
};

enum { LBM2P_OPT_STRAIN_MOMENTS = 1, LBM2P_OPT_GI_LITERAL = 2 };

/* Parameters.  Phase phi = +1 has density rho1 and dynamic viscosity mu1,
 * phase phi = -1 has rho2, mu2 (eq:rho, eq:dynamic_vis).  Lattice units,
 * dx = dt = 1 (Sec. 3.1). */
typedef struct lbm2p_params {
  int32_t nx, ny;          /* lattice size, each >= 16                         */
  int32_t wall_x, wall_y;  /* 0 periodic, 1 no-slip walls half-way outside the
                              first/last node (bounce-back, mirror ghosts)     */
  int32_t coupled;         /* 1 NS + CH; 0 CH only with a prescribed velocity  */
  int32_t precision;       /* 0 FP64; 1 FP32 state and arithmetic (FP64
                              diagnostics)                                     */
  double rho1, rho2, mu1, mu2;
  double sigma;            /* surface tension: kappa = 3 sigma W / 8,
                              beta = 3 sigma / (4 W)  (Sec. 2.1)               */
  double W;                /* interface width                                  */
  double M;                /* mobility; eta = M / (c_s^2 (tau_f - 1/2))
                              (eq:mobility)                                    */
  double lam;              /* lambda: J_d = lambda J_phi + q                   */
  double tau_f;            /* CH relaxation time: s_3^f = s_5^f = 1/tau_f      */
  double gx, gy;           /* gravity; F_g = (rho - rho_ref) g                 */
  double rho_ref;
  int32_t filter_n;        /* explicit filter SF-n, n in {5,7,9,11}; 0 = off   */
  int32_t compact;         /* 1 = compact tridiagonal filter instead           */
  int32_t compact_n;       /* compact filter right-hand-side half width, 1..5  */
  int32_t K;               /* fixed-point iterations of Eq:u, 1..8             */
  double filter_a;         /* filter intensity a (eq:filter), 0..1             */
  double compact_alpha;    /* compact filter alpha, (-1/2, 1/2)                */
  double s_f[9];           /* MRT rates of f; entries 3 and 5 are set to 1/tau_f */
  double s_g[9];           /* MRT rates of g; entries 7, 8 are 1/tau_g(x)      */
  double eps;              /* regularisation of |grad phi| in n, >= 0          */
  int32_t original_ch;     /* 1 = no FD sub-step (the original convective CH)  */
  int32_t options;         /* bit flags, 0 = the default readings:
                              LBM2P_OPT_STRAIN_MOMENTS: the strain rate of F_nu
                              from the non-equilibrium moments of g (eq:Fmu,
                              re-derived from App. A) instead of the velocity's
                              isotropic stencil;
                              LBM2P_OPT_GI_LITERAL: eq:Gi as printed,
                              u (F - grad p) / rho, instead of u (F/rho - grad p);
                              neither has an adjoint (lbm2p_record: EINVAL)     */
  double p_ref;            /* reference kinematic pressure of the stored g:
                              the library keeps g_i - 3 w_i p_ref, deviations
                              from the lattice weights (the state I/O converts;
                              0 = plain values).  Finite.                     */
} lbm2p_params;

typedef struct lbm2p_ctx lbm2p_ctx;

/* Device workspace size the context needs for these parameters.
 * Returns EINVAL for invalid parameters (see lbm2p_create). */
int lbm2p_workspace_bytes(const lbm2p_params* p, size_t* bytes);

/* Create a context.  d_workspace: device memory of >= `bytes` bytes, aligned to
 * 256 bytes, owned by the caller and kept alive until lbm2p_destroy.  stream:
 * a hipStream_t (NULL = default stream).  Errors: EINVAL for nx, ny < 16,
 * 9 * nx * ny (rounded up to 64) >= 2^31 (population slots use 32-bit offsets),
 * rho <= 0, mu < 0, W <= 0, M < 0, tau_f <= 1/2, any s outside [0, 2], a filter
 * order not in {0,5,7,9,11}, compact_n outside 1..5, |compact_alpha| >= 1/2,
 * a compact filter on a lattice side above 7680 (its line solve holds a line in LDS),
 * K outside 1..8, filter_a outside [0,1], eps < 0, a wall axis shorter than the
 * ghost depth, unknown option bits (or any option in CH-only mode); ENOSPACE for a
 * small workspace; EHIP if an event cannot be made. */
int lbm2p_create(const lbm2p_params* p, void* d_workspace, size_t bytes,
                 void* stream, lbm2p_ctx** out);

/* Initial state (equilibrium populations, eq:feq_CH / eq:geq with
 * mu = mu_phi(phi0), eq:chemical): f* = f^eq(phi0, mu, u0), g* = g^eq(p0, u0),
 * u~ = u0.  Device float64 planes [ny][nx]; d_ux0/d_uy0/d_p0 may be NULL
 * (zeros).  In CH-only mode (u0x, u0y) is the prescribed velocity of the
 * later steps (until lbm2p_set_velocity).  In coupled mode the first call also
 * makes the context's second stream (non-blocking, default priority) and two
 * events, with which the steps of large lattices (populations above 256 MB)
 * run the gather of p and j beside the FD sub-step (destroyed by
 * lbm2p_destroy); EHIP if they cannot be made. */
int lbm2p_init_fields(lbm2p_ctx* c, const double* d_phi0, const double* d_ux0,
                      const double* d_uy0, const double* d_p0);

/* CH-only mode: the prescribed velocity of every later step, until the next
 * call (Sec. 4.1: the single vortex, whose velocity field is modulated in time
 * by cos(pi t / T); Sec. 4.2: the translating drop).  d_ux, d_uy: device
 * float64 planes [ny][nx], borrowed for the call (converted to the context's
 * precision).  The first step after the call takes d_t u of eq:Fi as the new
 * velocity minus the one the previous step used (the backward difference the
 * coupled mode takes of u~); a velocity held fixed has d_t u = 0.  EINVAL in
 * coupled mode (the velocity there is the solution of Eq:u) or for a NULL
 * pointer; ESTATE before init.  lbm2p_record returns ESTATE between this call
 * and the next step, and a record made before it can no longer be reversed. */
int lbm2p_set_velocity(lbm2p_ctx* c, const double* d_ux, const double* d_uy);

/* Advance n >= 0 time steps (asynchronous on the context's stream; on large
 * coupled lattices part of each step runs on the second stream, forked from
 * and joined back to it by events, so the work stays ordered on the context's
 * stream).  ESTATE before init. */
int lbm2p_step(lbm2p_ctx* c, int32_t n);

/* Copy the current macroscopic fields to device float64 planes: phi^{n}
 * (after the FD sub-step), the filtered velocity u~ and pressure p~ (kinematic,
 * Sec. 2.2) and rho(clamp(phi)) (eq:rho).  Any pointer may be NULL. */
int lbm2p_moments(lbm2p_ctx* c, double* d_phi, double* d_ux, double* d_uy,
                  double* d_p, double* d_rho);

/* Intermediate fields of the last step, one float64 plane:
 *  0 phi_bar  1 p (raw, c_s^2 sum g)  2 j_x  3 j_y  4 u_x after the K
 *  iterations  5 u_y after the K iterations  6 phi^(1)  7 phi^(2). */
int lbm2p_fields(lbm2p_ctx* c, int32_t which, double* d_out);

/* Diagnostics in FP64 (synchronises the stream), host array out[6]:
 *  out[0] #{phi > 0} (volume, Sec. 4.3)  out[1] sum phi  out[2] sum p~
 *  out[3] max |u~|  out[4] min phi  out[5] max phi.
 * Returns ENONFINITE if sum phi or max|u~| is not finite. */
int lbm2p_volume(lbm2p_ctx* c, double out[6]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): the diagnostics
 * of lbm2p_volume on device float64 planes [ny][nx] the caller passes, with no
 * context and no workspace.  d_p may be NULL (out[2] = 0); d_out: device
 * memory for 6 doubles, the values of lbm2p_volume in its order (and bitwise
 * equal to them for the planes lbm2p_moments reports).  Asynchronous on
 * stream (NULL: the null stream); nothing is checked for finiteness (out[1]
 * and out[3] are NaN or Inf for a non-finite state).  The per-workgroup
 * partials live in a static array of the library, 64 KiB on each device that
 * calls it, held until the process ends; it allocates nothing.  Every call on
 * one device shares that array, so calls that overlap on one device (on
 * different streams or threads) race; every partial is written before it is
 * read, so nothing needs clearing between calls.  EINVAL for a NULL plane or
 * output, nx or ny < 1, or more than 2^31 - 1 nodes; EHIP when the device
 * array cannot be located or a launch fails. */
int lbm2p_volume_noalloc(const double* d_phi, const double* d_p, const double* d_ux,
                         const double* d_uy, int32_t nx, int32_t ny, double* d_out,
                         void* stream);

/* Rising-bubble diagnostics of Sec. 4.5 (eq:quantify-yc, eq:quantify-uc) over
 * the nodes with phi < 0 (the light phase): out[0] their number, out[1] their
 * mean row index y_c (the node of row j sits at y = j; a wall in y lies half a
 * node below row 0), out[2] their mean vertical velocity V_c (of u~, as
 * lbm2p_moments reports it), in host memory.  Sums in float64, in a fixed
 * order (deterministic).  y_c and V_c are NaN when no node has phi < 0.
 * Synchronises the stream.  ESTATE before init. */
int lbm2p_bubble(lbm2p_ctx* c, double out[3]);

/* Residual of the velocity iteration, the paper's stopping measure (text
 * after eq:Fmu): zeta = sum |u^K - u^{K-1}| / sum |u^{K-1}| over all nodes and
 * both components, for the K fixed sweeps of a step (u^0 = u~ of the step
 * before).  lbm2p_track_residual(c, 1) makes every later step run its last
 * sweep as a launch of its own, so that u^{K-1} stays in a velocity plane
 * (same results; one more launch per step for even K); 0 restores the
 * two-sweep launches.  It does not apply inside lbm2p_record and
 * lbm2p_adjoint.  EINVAL for on outside {0, 1}.
 * lbm2p_residual: zeta of the last step, in float64 (0 when u^{K-1} = 0), in
 * host memory; synchronises the stream.  ESTATE unless the last step ran with
 * tracking on (and after init or set_state); EINVAL in CH-only mode. */
int lbm2p_track_residual(lbm2p_ctx* c, int32_t on);
int lbm2p_residual(lbm2p_ctx* c, double* out);

/* Pressure jump of the Laplace test (Sec. 4.3): p' = rho p~ (the dynamic
 * pressure from the kinematic p~ of the state, rho of clamp(phi) as eq:rho),
 * averaged over the nodes with phi > 0.99 and over those with phi < -0.99.
 * out[0] the jump <p'>_{phi>0.99} - <p'>_{phi<-0.99}, out[1] and out[2] the two
 * means, out[3] and out[4] the two node counts, in host memory; a mean over no
 * node is NaN.  Float64 sums in a fixed order.  Synchronises the stream.
 * Coupled mode only (EINVAL in CH-only mode); ESTATE before init. */
int lbm2p_pressure_jump(lbm2p_ctx* c, double out[5]);

/* State in canonical order (post-collision f*_i(x), g*_i(x), then u~), as
 * device float64 arrays: d_f [9][ny][nx], d_g [9][ny][nx] (ignored in CH-only
 * mode, may be NULL), d_u [2][ny][nx].  set_state makes a context resume from
 * such a state. */
int lbm2p_get_state(lbm2p_ctx* c, double* d_f, double* d_g, double* d_u);
int lbm2p_set_state(lbm2p_ctx* c, const double* d_f, const double* d_g,
                    const double* d_u);

/* Kernel timing with HIP events on the context's stream.  lbm2p_profile(c, k)
 * starts recording every launch of pass k (0 gather, 1 FD stage, 2 velocity
 * iteration, 3 filter, 4 collide; -1 stops) for up to 65536 launches;
 * lbm2p_profile_read synchronises and returns the summed milliseconds and the
 * number of launches recorded since lbm2p_profile.  While the gather or the
 * FD pass is profiled the steps run them in series (no gather of p and j
 * beside the FD sub-step), so that each is timed on its own. */
int lbm2p_profile(lbm2p_ctx* c, int32_t pass);
int lbm2p_profile_read(lbm2p_ctx* c, double* ms, int64_t* launches);

/* ---------------------------------------------------------------- adjoint
 * Reverse mode of n steps (discrete adjoint of the whole step above, for
 * gradients of a loss of the final phi and state with respect to sigma, M and
 * the initial phi0).  Each step is reversed pass by pass (collision, filter,
 * velocity sweeps, the three FD stages, gather and streaming) with the
 * Jacobians at the forward values, recomputed segment by segment from
 * checkpoints kept every ckpt_every steps (memory O(n/k + k) planes, one extra
 * forward step per step except in the last segment, whose intermediates the
 * record keeps).  Supported for the explicit filter, the compact
 * filter (self-adjoint per direction: its reverse is the same line solves on
 * the adjoint fields) or none, both modes, both precisions (the arithmetic of
 * the adjoint is the context's).
 *
 * lbm2p_adjoint_workspace_bytes: device bytes lbm2p_record needs for these
 * parameters, n >= 0 steps and a checkpoint interval ckpt_every >= 1.
 * EINVAL for invalid values. */
int lbm2p_adjoint_workspace_bytes(const lbm2p_params* p, int32_t nsteps, int32_t ckpt_every,
                                  size_t* bytes);

/* Advance n steps like lbm2p_step and keep the checkpoints of the run, and
 * the per-step intermediates of its last segment, in d_ws (device memory,
 * 256-byte aligned, >= the bytes above, owned by the caller and kept alive
 * until the last lbm2p_adjoint of this record returns or the next record).
 * ESTATE before init or right after lbm2p_set_velocity (see there); EINVAL for
 * invalid values or a context with options set; ENOSPACE for a small d_ws. */
int lbm2p_record(lbm2p_ctx* c, int32_t nsteps, int32_t ckpt_every, void* d_ws, size_t bytes);

/* Inputs (seeds) and outputs of lbm2p_adjoint.  Device float64 arrays in the
 * canonical order of lbm2p_get_state; every pointer may be NULL (a NULL seed
 * is zero, a NULL output is not computed). */
typedef struct lbm2p_adjoint_io {
  const double* dL_dphi;   /* seed: dL/dphi of the last recorded step, [ny][nx]     */
  const double* dL_df;     /* seed: dL/df* of the final state, [9][ny][nx]           */
  const double* dL_dg;     /* seed: dL/dg* (coupled), [9][ny][nx]                    */
  const double* dL_du;     /* seed: dL/du~ (coupled), [2][ny][nx]                    */
  const double* phi0;      /* phi0, ux0, uy0 given to lbm2p_init_fields: needed for  */
  const double* ux0;       /*   dL_dphi0 (ux0, uy0 may be NULL = zeros)              */
  const double* uy0;
  double* dL_dphi0;        /* out: dL/dphi0 [ny][nx]; the recorded run must start at */
                           /*   lbm2p_init_fields (ESTATE otherwise)                 */
  double* dL_df0;          /* out: dL/df* of the state the run started from          */
  double* dL_dg0;          /* out: dL/dg* (coupled)                                  */
  double* dL_du0;          /* out: dL/du~ (coupled)                                  */
  double dL_dsigma;        /* out (host): total derivative with respect to sigma     */
  double dL_dM;            /* out (host): total derivative with respect to M         */
} lbm2p_adjoint_io;

/* Run the adjoint of the last lbm2p_record: seeds at the final step, outputs at
 * the first.  Synchronises the stream (the two scalars are host values).  The
 * context ends in the recorded final state (phi, u~, p~ and the populations;
 * lbm2p_fields reports an earlier step until the next lbm2p_step).  ESTATE
 * without a matching record (or after a step, init or set_state since).
 * With more than one segment (coupled step, explicit filter) the segments'
 * recomputes run on a second stream of the context, ordered against the
 * context's stream by events; the context creates that stream and the events
 * at its first such call and releases them in lbm2p_destroy (no device memory
 * is allocated). */
int lbm2p_adjoint(lbm2p_ctx* c, lbm2p_adjoint_io* io);

/* Copy bytes from d_src to d_dst (device memory, both 16-byte aligned, not
 * overlapping) on stream (NULL: the null stream), asynchronously, with one
 * 16-byte nontemporal load and store per thread: the device's streaming copy
 * rate, the HBM ceiling the step's kernels are measured against.  Needs no
 * context.  bytes = 0 does nothing; EINVAL for NULL, misaligned or
 * overlapping buffers; EHIP for a launch error. */
int lbm2p_stream_copy(const void* d_src, void* d_dst, size_t bytes, void* stream);

/* Release the context (not the workspace or the caller's stream; the adjoint's
 * own stream and events, if created, are released). */
void lbm2p_destroy(lbm2p_ctx* c);

/* Static string naming an error code. */
const char* lbm2p_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* LBM2P_H */
