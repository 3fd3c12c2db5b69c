// C ABI (include/lbm2p.h): parameter checks, context set-up and dispatch to
// the precision-specific implementations.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstdint>
#include <new>
#include <vector>

#include "lbm2p_ctx.h"

using namespace lbm2p;

namespace {

constexpr int RED_BLOCKS = 1024;
constexpr int RED_K = 6;

inline long long align_up(long long v, long long a) { return (v + a - 1) / a * a; }

int validate(const lbm2p_params* p) {
  if (!p) return LBM2P_EINVAL;
  if (p->nx < 16 || p->ny < 16) return LBM2P_EINVAL;
  // population slots are addressed with 32-bit offsets (9 planes per distribution)
  if (9LL * (((long long)p->nx * p->ny + 63) / 64 * 64) >= (1LL << 31)) return LBM2P_EINVAL;
  if (p->precision != 0 && p->precision != 1) return LBM2P_EINVAL;
  if (!(p->rho1 > 0) || !(p->rho2 > 0) || !(p->mu1 >= 0) || !(p->mu2 >= 0)) return LBM2P_EINVAL;
  if (!(p->W > 0) || !(p->M >= 0) || !(p->tau_f > 0.5) || !(p->sigma >= 0)) return LBM2P_EINVAL;
  if (!(p->eps >= 0) || !(p->lam >= 0)) return LBM2P_EINVAL;
  for (int k = 0; k < 9; ++k) {
    if (k != 3 && k != 5 && !(p->s_f[k] >= 0 && p->s_f[k] <= 2)) return LBM2P_EINVAL;
    if (k != 7 && k != 8 && !(p->s_g[k] >= 0 && p->s_g[k] <= 2)) return LBM2P_EINVAL;
  }
  if (1.0 / p->tau_f > 2.0) return LBM2P_EINVAL;
  if (p->filter_n != 0 && p->filter_n != 5 && p->filter_n != 7 && p->filter_n != 9 &&
      p->filter_n != 11)
    return LBM2P_EINVAL;
  if (p->compact != 0 && p->compact != 1) return LBM2P_EINVAL;
  if (p->compact && (p->compact_n < 1 || p->compact_n > 5)) return LBM2P_EINVAL;
  if (p->compact && !(p->compact_alpha > -0.5 && p->compact_alpha < 0.5)) return LBM2P_EINVAL;
  // the compact filter's line solve stages a whole line in LDS
  if (p->compact && (p->nx > 7680 || p->ny > 7680)) return LBM2P_EINVAL;
  if (p->K < 1 || p->K > 8) return LBM2P_EINVAL;
  if (!(p->filter_a >= 0 && p->filter_a <= 1)) return LBM2P_EINVAL;
  if (p->coupled != 0 && p->coupled != 1) return LBM2P_EINVAL;
  if (p->options & ~(LBM2P_OPT_STRAIN_MOMENTS | LBM2P_OPT_GI_LITERAL)) return LBM2P_EINVAL;
  if (p->options && !p->coupled) return LBM2P_EINVAL;
  if (!std::isfinite(p->p_ref)) return LBM2P_EINVAL;
  return LBM2P_OK;
}

long long plane_stride(const lbm2p_params* p) {
  return align_up((long long)p->nx * p->ny, 64);
}

size_t n_planes(const lbm2p_params* p) {
  // f(9) + phi, phibar, phi1, phi2 + U(4)  [+ g(9) + praw, jx, jy, pt + uk(4)]
  // [+ m1, m7, m8 of the pre-collision g for the moment strain rate]
  const size_t sm = (p->options & LBM2P_OPT_STRAIN_MOMENTS) ? 3 : 0;
  return p->coupled ? 9 + 4 + 4 + 9 + 4 + 4 + sm : 9 + 4 + 4;
}

size_t compact_planes(const lbm2p_params* p) { return (p->coupled && p->compact) ? 6 : 0; }

size_t compact_table_doubles(const lbm2p_params* p) {
  if (!(p->coupled && p->compact)) return 0;
  // 2 parities x (cp, inv, z) per axis, then 3 per-line factors per line
  return 2 * 3 * ((size_t)p->nx + (size_t)p->ny) + 3 * ((size_t)p->nx + (size_t)p->ny);
}

size_t ws_size(const lbm2p_params* p) {
  const size_t esz = p->precision ? 4 : 8;
  return (n_planes(p) + compact_planes(p)) * (size_t)plane_stride(p) * esz +
         (RED_BLOCKS + 1) * RED_K * sizeof(double) + compact_table_doubles(p) * sizeof(double) +
         512;
}

// Coefficients a_0..a_N of the compact filter: T(0) = 1, T(pi) = 0 and the
// vanishing w^2 .. w^(2N-2) Taylor terms of T(w) - 1, with
// T(w) = sum a_n cos(n w) / (1 + 2 alpha cos w).  Gaussian elimination with
// partial pivoting on the (N+1) x (N+1) system.
void compact_coeffs(int N, double alpha, double* a) {
  double A[6][7];
  for (int n = 0; n <= N; ++n) A[0][n] = 1.0;
  A[0][N + 1] = 1.0 + 2.0 * alpha;
  for (int k = 1; k < N; ++k) {
    for (int n = 0; n <= N; ++n) A[k][n] = std::pow((double)n, 2.0 * k);
    A[k][N + 1] = 2.0 * alpha;
  }
  for (int n = 0; n <= N; ++n) A[N][n] = (n % 2) ? -1.0 : 1.0;
  A[N][N + 1] = 0.0;
  const int m = N + 1;
  for (int c = 0; c < m; ++c) {
    int piv = c;
    for (int r = c + 1; r < m; ++r)
      if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
    for (int k = 0; k <= m; ++k) std::swap(A[c][k], A[piv][k]);
    for (int r = 0; r < m; ++r) {
      if (r == c) continue;
      const double f = A[r][c] / A[c][c];
      for (int k = c; k <= m; ++k) A[r][k] -= f * A[c][k];
    }
  }
  for (int n = 0; n < 6; ++n) a[n] = n < m ? A[n][m] / A[n][n] : 0.0;
}

// Thomas tables of the line matrix (1 on the diagonal, alpha off it) for n
// nodes: periodic -> cyclic matrix split as B + u v^T (Sherman-Morrison with
// gamma = -1); wall -> end rows 1 + sgn alpha (mirror ghosts).
void compact_table(int n, double alpha, bool cyclic, double sgn, double* cp, double* inv,
                   double* z, double* fac, double* den, int* flat, int* z0, int* z1) {
  std::vector<double> b(n, 1.0);
  double gamma = 0;
  if (cyclic) {
    gamma = -1.0;
    b[0] = 1.0 - gamma;
    b[n - 1] = 1.0 - alpha * alpha / gamma;
  } else {
    b[0] = 1.0 + sgn * alpha;
    b[n - 1] = 1.0 + sgn * alpha;
  }
  double c_prev = 0;
  for (int i = 0; i < n; ++i) {
    const double piv = b[i] - (i ? alpha * c_prev : 0.0);
    inv[i] = 1.0 / piv;
    cp[i] = alpha * inv[i];
    c_prev = cp[i];
  }
  // c'_i and 1/pivot_i depend on rows 0..i only and converge to fixed values;
  // from index *flat up to n - 2 they equal the values at *flat bit for bit
  // (only the last row differs), so the device need not read them there
  int K = n - 1;
  while (K > 0 && cp[K - 1] == cp[n - 2] && inv[K - 1] == inv[n - 2]) --K;
  *flat = n >= 2 ? K : 0;
  if (cyclic) {
    // B z = u with u = (gamma, 0, ..., 0, alpha)
    std::vector<double> d(n);
    for (int i = 0; i < n; ++i) {
      const double r = i == 0 ? gamma : (i == n - 1 ? alpha : 0.0);
      d[i] = (i ? r - alpha * d[i - 1] : r) * inv[i];
    }
    z[n - 1] = d[n - 1];
    for (int i = n - 2; i >= 0; --i) z[i] = d[i] - cp[i] * z[i + 1];
    *fac = alpha / gamma;
    *den = 1.0 + z[0] + (*fac) * z[n - 1];
  } else {
    for (int i = 0; i < n; ++i) z[i] = 0.0;
    *fac = 0;
    *den = 1;
  }
  // z decays from both ends: [z0, z1) holds only |z_i| <= 1e-30 max|z| (the
  // device drops f z_i there); every larger entry of the first half lies below
  // z0, of the second half at or above z1
  double zmax = 0;
  for (int i = 0; i < n; ++i) zmax = std::max(zmax, std::fabs(z[i]));
  const double thr = 1e-30 * zmax;
  *z0 = 0;
  *z1 = n;
  for (int i = 0; i < n / 2; ++i)
    if (std::fabs(z[i]) > thr) *z0 = i + 1;
  for (int i = n - 1; i >= n / 2; --i)
    if (std::fabs(z[i]) > thr) *z1 = i;
  if (!cyclic) {
    *z0 = 0;
    *z1 = n;
  }
}

// filter coefficients d_0..d_N of App. B
void filter_coeffs(int order, double* d, int* N) {
  static const double sf5[] = {6.0 / 16, -4.0 / 16, 1.0 / 16};
  static const double sf7[] = {5.0 / 16, -15.0 / 64, 3.0 / 32, -1.0 / 64};
  static const double sf9[] = {0.243527493120, -0.204788880640, 0.120007591680, -0.045211119360,
                               0.008228661760};
  static const double sf11[] = {0.215044884112, -0.187772883589, 0.123755948787,
                                -0.059227575576, 0.018721609157, -0.002999540835};
  const double* src = order == 5 ? sf5 : order == 7 ? sf7 : order == 9 ? sf9 : sf11;
  *N = (order - 1) / 2;
  for (int k = 0; k < 6; ++k) d[k] = k <= *N ? src[k] : 0.0;
}

// Streaming copy: one 16-byte vector per thread (grid-stride beyond 2^20
// workgroups), nontemporal loads and stores; the last bytes % 16 bytes are
// copied one byte per thread by the first workgroup.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_stream_copy(const u32x4* __restrict__ src,
                                                     u32x4* __restrict__ dst, size_t n16,
                                                     int tail) {
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
  if (blockIdx.x == 0 && (int)threadIdx.x < tail) {
    const unsigned char* s8 = reinterpret_cast<const unsigned char*>(src + n16);
    unsigned char* d8 = reinterpret_cast<unsigned char*>(dst + n16);
    d8[threadIdx.x] = s8[threadIdx.x];
  }
}

}  // namespace

// ======================================================================= ABI
extern "C" {

int lbm2p_stream_copy(const void* d_src, void* d_dst, size_t bytes, void* stream) {
  if (bytes == 0) return LBM2P_OK;
  const uintptr_t s = (uintptr_t)d_src, d = (uintptr_t)d_dst;
  if (!d_src || !d_dst || (s & 15) || (d & 15)) return LBM2P_EINVAL;
  if (s < d + bytes && d < s + bytes) return LBM2P_EINVAL;   // overlapping ranges
  const size_t n16 = bytes / 16;
  const int tail = (int)(bytes % 16);
  const size_t blocks = std::min<size_t>(std::max<size_t>((n16 + 255) / 256, 1), (size_t)1 << 20);
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                     (const u32x4*)d_src, (u32x4*)d_dst, n16, tail);
  return hipGetLastError() == hipSuccess ? LBM2P_OK : LBM2P_EHIP;
}

const char* lbm2p_strerror(int code) {
  switch (code) {
    case LBM2P_OK: return "ok";
    case LBM2P_EINVAL: return "invalid argument";
    case LBM2P_ENOSPACE: return "workspace too small";
    case LBM2P_EHIP: return "HIP runtime error";
    case LBM2P_ENONFINITE: return "non-finite value in the state";
    case LBM2P_ESTATE: return "call out of order";
    default: return "unknown error";
  }
}

int lbm2p_workspace_bytes(const lbm2p_params* p, size_t* bytes) {
  const int e = validate(p);
  if (e) return e;
  if (!bytes) return LBM2P_EINVAL;
  *bytes = ws_size(p);
  return LBM2P_OK;
}

int lbm2p_create(const lbm2p_params* p, void* d_workspace, size_t bytes, void* stream,
                 lbm2p_ctx** out) {
  if (!out) return LBM2P_EINVAL;
  *out = nullptr;
  const int e = validate(p);
  if (e) return e;
  if (!d_workspace || ((uintptr_t)d_workspace & 255)) return LBM2P_EINVAL;
  if (bytes < ws_size(p)) return LBM2P_ENOSPACE;
  lbm2p_ctx* c = new (std::nothrow) lbm2p_ctx();
  if (!c) return LBM2P_EINVAL;
  c->p = *p;
  c->prec = p->precision;
  c->stream = (hipStream_t)stream;
  c->ws = (char*)d_workspace;
  c->ws_bytes = bytes;
  c->n = (long long)p->nx * p->ny;
  c->ps = plane_stride(p);
  c->esz = p->precision ? 4 : 8;
  char* q = c->ws;
  auto take = [&](long long planes) {
    void* r = q;
    q += planes * c->ps * c->esz;
    return r;
  };
  c->Af = take(9);
  c->phi = take(1);
  c->phibar = take(1);
  c->phi1 = take(1);
  c->phi2 = take(1);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) c->U[a][b] = take(1);
  if (p->coupled) {
    c->Ag = take(9);
    c->praw = take(1);
    c->jx = take(1);
    c->jy = take(1);
    c->pt = take(1);
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) c->uk[a][b] = take(1);
    if (p->options & LBM2P_OPT_STRAIN_MOMENTS) {
      c->sm1 = take(1);
      c->sm7 = take(1);
      c->sm8 = take(1);
    } else {
      c->sm1 = c->sm7 = c->sm8 = nullptr;
    }
  } else {
    c->Ag = c->praw = c->jx = c->jy = c->pt = nullptr;
    c->sm1 = c->sm7 = c->sm8 = nullptr;
  }
  c->cscratch = compact_planes(p) ? take((long long)compact_planes(p)) : nullptr;
  c->red = (double*)(((uintptr_t)q + 255) & ~(uintptr_t)255);
  c->ctab_dev = nullptr;
  c->cfct = nullptr;
  c->ctab_uploaded = 0;
  if (compact_table_doubles(p)) {
    c->ctab_dev = c->red + (RED_BLOCKS + 1) * RED_K;
    c->cfct = c->ctab_dev + 2 * 3 * ((size_t)p->nx + (size_t)p->ny);
    c->ctab_host.assign(compact_table_doubles(p), 0.0);
    compact_coeffs(p->compact_n, p->compact_alpha, c->ca);
    size_t off = 0;
    for (int axis = 0; axis < 2; ++axis) {
      const int n = axis == 0 ? p->nx : p->ny;
      const bool cyclic = axis == 0 ? !p->wall_x : !p->wall_y;
      c->ctab_n[axis] = n;
      for (int par = 0; par < 2; ++par) {
        c->ctab_off[axis][par] = off;
        double* base = c->ctab_host.data() + off;
        compact_table(n, p->compact_alpha, cyclic, par ? -1.0 : 1.0, base, base + n, base + 2 * n,
                      &c->cfac[axis][par], &c->cden[axis][par], &c->cflat[axis][par],
                      &c->cz0[axis][par], &c->cz1[axis][par]);
        off += 3 * (size_t)n;
      }
    }
  }
  // derived constants, written as the oracle writes them (Sec. 2.1, eq:mobility)
  c->kappa = 3.0 * p->sigma * p->W / 8.0;
  c->beta = 3.0 * p->sigma / (4.0 * p->W);
  c->eta = (3.0 * p->M) / (p->tau_f - 0.5);
  c->c4b = 4.0 * c->beta;
  c->negM = -p->M;
  c->cJ = (p->rho1 - p->rho2) / 2.0 * p->M;
  c->eps2 = p->eps * p->eps;
  for (int k = 0; k < 9; ++k) {
    c->s_f[k] = p->s_f[k];
    c->s_g[k] = p->s_g[k];
  }
  c->s_f[3] = 1.0 / p->tau_f;
  c->s_f[5] = 1.0 / p->tau_f;
  c->s_g[7] = 0.0;  // per node
  c->s_g[8] = 0.0;
  if (p->filter_n)
    filter_coeffs(p->filter_n, c->fd, &c->fn);
  else {
    for (int k = 0; k < 6; ++k) c->fd[k] = 0;
    c->fn = 0;
  }
  c->prof_pass = -1;
  c->prof_n = 0;
  c->inited = 0;
  c->rec = 0;
  c->from_init = 0;
  c->adj_ready = 0;
  c->adj_ws = nullptr;
  c->track_resid = 0;
  c->res_valid = 0;
  c->vpend = 0;
  c->adj_stream = nullptr;
  c->g_stream = nullptr;
  c->g_ev[0] = c->g_ev[1] = nullptr;
  *out = c;
  return LBM2P_OK;
}

void lbm2p_destroy(lbm2p_ctx* c) {
  if (!c) return;
  for (auto e : c->ev0) hipEventDestroy(e);
  for (auto e : c->ev1) hipEventDestroy(e);
  for (auto e : c->adj_ev) hipEventDestroy(e);
  if (c->adj_stream) hipStreamDestroy(c->adj_stream);
  for (auto e : c->g_ev)
    if (e) hipEventDestroy(e);
  if (c->g_stream) hipStreamDestroy(c->g_stream);
  delete c;
}

int lbm2p_init_fields(lbm2p_ctx* c, const double* phi0, const double* ux0, const double* uy0,
                      const double* p0) {
  if (!c || !phi0) return LBM2P_EINVAL;
  // the coupled step's second stream and its fork/join events, made once here
  // (not in a step, which a caller may be capturing into a graph)
  if (c->p.coupled && !c->g_stream) {
    if (hipStreamCreateWithFlags(&c->g_stream, hipStreamNonBlocking) != hipSuccess) {
      c->g_stream = nullptr;
      return LBM2P_EHIP;
    }
    for (auto& e : c->g_ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        e = nullptr;
        return LBM2P_EHIP;
      }
  }
  return c->prec ? init_f32(c, phi0, ux0, uy0, p0)
                 : init_f64(c, phi0, ux0, uy0, p0);
}

int lbm2p_step(lbm2p_ctx* c, int32_t n) {
  if (!c || n < 0) return LBM2P_EINVAL;
  if (!c->inited) return LBM2P_ESTATE;
  if (n > 0) c->adj_ready = 0;
  return c->prec ? step_f32(c, n) : step_f64(c, n);
}

int lbm2p_set_velocity(lbm2p_ctx* c, const double* ux, const double* uy) {
  if (!c || !ux || !uy || c->p.coupled) return LBM2P_EINVAL;
  if (!c->inited) return LBM2P_ESTATE;
  return c->prec ? setvel_f32(c, ux, uy) : setvel_f64(c, ux, uy);
}

int lbm2p_adjoint_workspace_bytes(const lbm2p_params* p, int32_t nsteps, int32_t ckpt_every,
                                  size_t* bytes) {
  const int e = validate(p);
  if (e) return e;
  if (!bytes || nsteps < 0 || ckpt_every < 1) return LBM2P_EINVAL;
  const AdjLayout L = adj_layout(*p, plane_stride(p), (long long)p->nx * p->ny,
                                 p->precision ? 4 : 8, nsteps, ckpt_every);
  *bytes = L.total;
  return LBM2P_OK;
}

int lbm2p_record(lbm2p_ctx* c, int32_t nsteps, int32_t ckpt_every, void* d_ws, size_t bytes) {
  if (!c || nsteps < 0 || ckpt_every < 1 || !d_ws || ((uintptr_t)d_ws & 255)) return LBM2P_EINVAL;
  if (c->p.options) return LBM2P_EINVAL;   // the reverse step covers the default readings
  // a velocity set since the last step: that step's d_t u is not a constant of
  // the recorded run, which the reverse of the CH-only collision assumes
  if (!c->inited || c->vpend) return LBM2P_ESTATE;
  const AdjLayout L = adj_layout(c->p, c->ps, c->n, c->esz, nsteps, ckpt_every);
  if (bytes < L.total) return LBM2P_ENOSPACE;
  c->adj_ws = (char*)d_ws;
  c->adj_bytes = bytes;
  // the recorded steps and their recomputation run the same launches: no
  // residual tracking inside record and adjoint
  const int track = c->track_resid;
  c->track_resid = 0;
  const int r = c->prec ? record_f32(c, nsteps, ckpt_every) : record_f64(c, nsteps, ckpt_every);
  c->track_resid = track;
  return r;
}

int lbm2p_adjoint(lbm2p_ctx* c, lbm2p_adjoint_io* io) {
  if (!c || !io) return LBM2P_EINVAL;
  if (!c->inited || !c->adj_ready || c->steps != c->adj_steps_end) return LBM2P_ESTATE;
  if (io->dL_dphi0 && !io->phi0) return LBM2P_EINVAL;
  if (io->dL_dphi0 && !c->adj_from_init) return LBM2P_ESTATE;
  const int track = c->track_resid;
  c->track_resid = 0;
  const int r = c->prec ? adjoint_f32(c, io) : adjoint_f64(c, io);
  c->track_resid = track;
  return r;
}

int lbm2p_moments(lbm2p_ctx* c, double* phi, double* ux, double* uy, double* p, double* rho) {
  if (!c) return LBM2P_EINVAL;
  if (!c->inited) return LBM2P_ESTATE;
  return c->prec ? moments_f32(c, phi, ux, uy, p, rho)
                 : moments_f64(c, phi, ux, uy, p, rho);
}

int lbm2p_fields(lbm2p_ctx* c, int32_t which, double* out) {
  if (!c || !out || which < 0 || which > 7) return LBM2P_EINVAL;
  if (!c->inited || c->steps == 0) return LBM2P_ESTATE;
  const int kl = c->uk_last;
  void* src = nullptr;
  switch (which) {
    case 0: src = c->phibar; break;
    case 1: src = c->praw; break;
    case 2: src = c->jx; break;
    case 3: src = c->jy; break;
    case 4: src = c->p.coupled ? c->uk[kl][0] : nullptr; break;
    case 5: src = c->p.coupled ? c->uk[kl][1] : nullptr; break;
    case 6: src = c->phi1; break;
    case 7: src = c->phi2; break;
  }
  if (!src) return LBM2P_EINVAL;
  c->prec ? to_f64_f32(c, src, out) : to_f64_f64(c, src, out);
  return hipGetLastError() == hipSuccess ? LBM2P_OK : LBM2P_EHIP;
}

int lbm2p_volume(lbm2p_ctx* c, double out[6]) {
  if (!c || !out) return LBM2P_EINVAL;
  if (!c->inited) return LBM2P_ESTATE;
  return c->prec ? volume_f32(c, out) : volume_f64(c, out);
}

int lbm2p_volume_noalloc(const double* d_phi, const double* d_p, const double* d_ux,
                         const double* d_uy, int32_t nx, int32_t ny, double* d_out,
                         void* stream) {
  if (!d_phi || !d_ux || !d_uy || !d_out || nx < 1 || ny < 1) return LBM2P_EINVAL;
  if ((long long)nx * ny > (long long)INT32_MAX) return LBM2P_EINVAL;
  return volume_noalloc_f64(d_phi, d_p, d_ux, d_uy, (long long)nx * ny, d_out,
                            (hipStream_t)stream);
}

int lbm2p_bubble(lbm2p_ctx* c, double out[3]) {
  if (!c || !out) return LBM2P_EINVAL;
  if (!c->inited) return LBM2P_ESTATE;
  return c->prec ? bubble_f32(c, out) : bubble_f64(c, out);
}

int lbm2p_track_residual(lbm2p_ctx* c, int32_t on) {
  if (!c || (on != 0 && on != 1)) return LBM2P_EINVAL;
  c->track_resid = on;
  return LBM2P_OK;
}

int lbm2p_residual(lbm2p_ctx* c, double* out) {
  if (!c || !out || !c->p.coupled) return LBM2P_EINVAL;
  if (!c->inited || !c->res_valid) return LBM2P_ESTATE;
  return c->prec ? resid_f32(c, out) : resid_f64(c, out);
}

int lbm2p_pressure_jump(lbm2p_ctx* c, double out[5]) {
  if (!c || !out || !c->p.coupled) return LBM2P_EINVAL;
  if (!c->inited) return LBM2P_ESTATE;
  return c->prec ? pjump_f32(c, out) : pjump_f64(c, out);
}

int lbm2p_get_state(lbm2p_ctx* c, double* f, double* g, double* u) {
  if (!c) return LBM2P_EINVAL;
  if (!c->inited) return LBM2P_ESTATE;
  return c->prec ? state_f32(c, f, g, u, 0) : state_f64(c, f, g, u, 0);
}

int lbm2p_set_state(lbm2p_ctx* c, const double* f, const double* g, const double* u) {
  if (!c || !f || !u || (c->p.coupled && !g)) return LBM2P_EINVAL;
  if (!c->inited) return LBM2P_ESTATE;
  return c->prec ? state_f32(c, (double*)f, (double*)g, (double*)u, 1)
                 : state_f64(c, (double*)f, (double*)g, (double*)u, 1);
}

int lbm2p_profile(lbm2p_ctx* c, int32_t pass) {
  if (!c || pass < -1 || pass > 4) return LBM2P_EINVAL;
  if (pass >= 0 && c->ev0.empty()) {
    const size_t cap = 65536;
    c->ev0.resize(cap);
    c->ev1.resize(cap);
    for (size_t i = 0; i < cap; ++i) {
      if (hipEventCreate(&c->ev0[i]) != hipSuccess || hipEventCreate(&c->ev1[i]) != hipSuccess)
        return LBM2P_EHIP;
    }
  }
  c->prof_pass = pass;
  c->prof_n = 0;
  return LBM2P_OK;
}

int lbm2p_profile_read(lbm2p_ctx* c, double* ms, int64_t* launches) {
  if (!c || !ms || !launches) return LBM2P_EINVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LBM2P_EHIP;
  double tot = 0;
  for (size_t i = 0; i < c->prof_n; ++i) {
    float t = 0;
    if (hipEventElapsedTime(&t, c->ev0[i], c->ev1[i]) != hipSuccess) return LBM2P_EHIP;
    tot += t;
  }
  *ms = tot;
  *launches = (int64_t)c->prof_n;
  return LBM2P_OK;
}

}  // extern "C"
