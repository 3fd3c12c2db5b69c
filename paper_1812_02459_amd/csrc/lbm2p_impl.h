// Host orchestration of one lattice update and its utility kernels, templated
// on the precision.  Included once per precision translation unit.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "lbm2p_ctx.h"
#include "lbm2p_kernels.h"
#include "lbm2p_compact.h"
#include "lbm2p_adjoint.h"

namespace lbm2p {
namespace {

// ------------------------------------------------------------ utility kernels
// Equilibrium initial populations (R15 of the oracle's readings): mu(phi0) with
// the isotropic Laplacian, f* = f^eq(phi0, mu, u0), g* = g^eq(p0, u0), stored in
// the parity-0 layout (f*_i(x) at A[opp(i)][x]).  Evaluated in float64.
template <typename T>
__global__ __launch_bounds__(256) void k_init(KParams<T> P, double c4b, double kappa, double eta,
                                              double p_ref,
                                              const double* __restrict__ phi0,
                                              const double* __restrict__ ux0,
                                              const double* __restrict__ uy0,
                                              const double* __restrict__ p0, T* Af, T* Ag,
                                              T* phi, T* pt, T* ux, T* uy, int coupled) {
  const long long n = (long long)P.nx * P.ny;
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= n) return;
  const int y = (int)(id / P.nx), x = (int)(id - (long long)y * P.nx);
  struct G {
    const double* a;
    const KParams<T>* P;
    int x0, y0;
    __device__ double operator()(int dx, int dy) const {
      int flip = 0;
      const int xx = map_idx(x0 + dx, P->nx, P->wx, flip);
      const int yy = map_idx(y0 + dy, P->ny, P->wy, flip);
      return a[(long long)yy * P->nx + xx];
    }
  } g{phi0, &P, x, y};
  const double ph = phi0[id];
  const double mu = chem_pot<double>(g, 0, 0, c4b, kappa);
  const double u_x = ux0 ? ux0[id] : 0.0, u_y = uy0 ? uy0[id] : 0.0, p = p0 ? p0[id] : 0.0;
  double feq[9];
  f_eq<double>(ph, mu, u_x, u_y, eta, feq);
#pragma unroll
  for (int i = 0; i < 9; ++i) Af[opp(i) * P.ps + id] = T(feq[i]);
  if (coupled) {
    double geq[9];
    g_eq<double>(p - p_ref, u_x, u_y, geq);   // stored as g_i - 3 w_i p_ref
#pragma unroll
    for (int i = 0; i < 9; ++i) Ag[opp(i) * P.ps + id] = T(geq[i]);
  }
  phi[id] = T(ph);
  pt[id] = T(p);
  ux[id] = T(u_x);
  uy[id] = T(u_y);
}

// canonical f*_i(x) <-> in-place layout of the given parity; the canonical
// value is the stored one plus w_i shift (3 p_ref for g, 0 for f)
template <typename T>
__global__ __launch_bounds__(256) void k_state(KParams<T> P, T* A, double* canon, int parity, int set,
                                               double shift) {
  const long long n = (long long)P.nx * P.ny;
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= n) return;
  const int y = (int)(id / P.nx), x = (int)(id - (long long)y * P.nx);
  for (int i = 0; i < 9; ++i) {
    long long loc;
    if (parity == 0) {
      loc = opp(i) * P.ps + id;
    } else {
      int tx = x + cx_of(i), ty = y + cy_of(i);
      const bool outside = (P.wx && (tx < 0 || tx >= P.nx)) || (P.wy && (ty < 0 || ty >= P.ny));
      if (outside) {
        loc = opp(i) * P.ps + id;
      } else {
        tx = tx < 0 ? tx + P.nx : (tx >= P.nx ? tx - P.nx : tx);
        ty = ty < 0 ? ty + P.ny : (ty >= P.ny ? ty - P.ny : ty);
        loc = i * P.ps + (long long)ty * P.nx + tx;
      }
    }
    if (set)
      A[loc] = T(canon[i * n + id] - w_of(i) * shift);
    else
      canon[i * n + id] = double(A[loc]) + w_of(i) * shift;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_to_f64(const T* a, double* o, long long n) {
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id < n) o[id] = double(a[id]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_from_f64(const double* a, T* o, long long n) {
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id < n) o[id] = T(a[id]);
}

// a fill kernel rather than hipMemsetAsync, so that the calls a caller may
// capture into a HIP graph record kernel nodes only
template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* a, T v, long long n) {
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id < n) a[id] = v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy(const T* a, T* o, long long n) {
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id < n) o[id] = a[id];
}

template <typename T>
__global__ __launch_bounds__(256) void k_rho(const T* phi, double* o, long long n, double rho1,
                                             double rho2) {
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id < n) o[id] = density<double>(double(phi[id]), rho1, rho2);
}

// FP64 diagnostics: per-block partials in a fixed tree order, then one block
// reduces the partials in a fixed order (deterministic).
constexpr int RED_NT = 256;
constexpr int RED_K = 6;  // count(phi>0), sum phi, sum p, max|u|, min phi, max phi

template <typename T>
__global__ __launch_bounds__(RED_NT) void k_reduce1(const T* phi, const T* pt, const T* ux,
                                                    const T* uy, long long n, double* part,
                                                    int coupled) {
  __shared__ double s[RED_K][RED_NT];
  double c = 0, sp = 0, spp = 0, um = 0, mn = INFINITY, mx = -INFINITY;
  for (long long id = (long long)blockIdx.x * RED_NT + threadIdx.x; id < n;
       id += (long long)gridDim.x * RED_NT) {
    const double ph = double(phi[id]);
    c += ph > 0.0 ? 1.0 : 0.0;
    sp += ph;
    if (coupled) spp += double(pt[id]);
    const double a = double(ux[id]), b = double(uy[id]);
    const double m = sqrt(a * a + b * b);
    um = (m > um || m != m) ? m : um;
    mn = fmin(mn, ph);
    mx = fmax(mx, ph);
  }
  s[0][threadIdx.x] = c;
  s[1][threadIdx.x] = sp;
  s[2][threadIdx.x] = spp;
  s[3][threadIdx.x] = um;
  s[4][threadIdx.x] = mn;
  s[5][threadIdx.x] = mx;
  __syncthreads();
  for (int w = RED_NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const int o = threadIdx.x + w;
      s[0][threadIdx.x] += s[0][o];
      s[1][threadIdx.x] += s[1][o];
      s[2][threadIdx.x] += s[2][o];
      const double a = s[3][threadIdx.x], b = s[3][o];
      s[3][threadIdx.x] = (b > a || b != b) ? b : a;
      s[4][threadIdx.x] = fmin(s[4][threadIdx.x], s[4][o]);
      s[5][threadIdx.x] = fmax(s[5][threadIdx.x], s[5][o]);
    }
    __syncthreads();
  }
  if (threadIdx.x < RED_K) part[(long long)blockIdx.x * RED_K + threadIdx.x] = s[threadIdx.x][0];
}

__global__ __launch_bounds__(RED_NT) void k_reduce2(const double* part, int nb, double* out) {
  __shared__ double s[RED_K][RED_NT];
  double c = 0, sp = 0, spp = 0, um = 0, mn = INFINITY, mx = -INFINITY;
  for (int b = threadIdx.x; b < nb; b += RED_NT) {
    c += part[b * RED_K + 0];
    sp += part[b * RED_K + 1];
    spp += part[b * RED_K + 2];
    const double m = part[b * RED_K + 3];
    um = (m > um || m != m) ? m : um;
    mn = fmin(mn, part[b * RED_K + 4]);
    mx = fmax(mx, part[b * RED_K + 5]);
  }
  s[0][threadIdx.x] = c;
  s[1][threadIdx.x] = sp;
  s[2][threadIdx.x] = spp;
  s[3][threadIdx.x] = um;
  s[4][threadIdx.x] = mn;
  s[5][threadIdx.x] = mx;
  __syncthreads();
  for (int w = RED_NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const int o = threadIdx.x + w;
      s[0][threadIdx.x] += s[0][o];
      s[1][threadIdx.x] += s[1][o];
      s[2][threadIdx.x] += s[2][o];
      const double a = s[3][threadIdx.x], b = s[3][o];
      s[3][threadIdx.x] = (b > a || b != b) ? b : a;
      s[4][threadIdx.x] = fmin(s[4][threadIdx.x], s[4][o]);
      s[5][threadIdx.x] = fmax(s[5][threadIdx.x], s[5][o]);
    }
    __syncthreads();
  }
  if (threadIdx.x < RED_K) out[threadIdx.x] = s[threadIdx.x][0];
}

// Bubble diagnostics of Sec. 4.5 (eq:quantify-yc, eq:quantify-uc): over the
// nodes with phi < 0, their number, the sum of their row index y and the sum
// of their vertical velocity, in float64 partials per workgroup (fixed tree
// order), then one workgroup sums the partials.
constexpr int BUB_K = 3;
template <typename T>
__global__ __launch_bounds__(RED_NT) void k_bubble1(const T* phi, const T* uy, int nx,
                                                    long long n, double* part) {
  __shared__ double s[BUB_K][RED_NT];
  double c = 0, sy = 0, sv = 0;
  for (long long id = (long long)blockIdx.x * RED_NT + threadIdx.x; id < n;
       id += (long long)gridDim.x * RED_NT) {
    if (double(phi[id]) < 0.0) {
      c += 1.0;
      sy += double(id / nx);
      sv += double(uy[id]);
    }
  }
  s[0][threadIdx.x] = c;
  s[1][threadIdx.x] = sy;
  s[2][threadIdx.x] = sv;
  __syncthreads();
  for (int w = RED_NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < BUB_K; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < BUB_K) part[(long long)blockIdx.x * BUB_K + threadIdx.x] = s[threadIdx.x][0];
}

__global__ __launch_bounds__(RED_NT) void k_bubble2(const double* part, int nb, double* out) {
  __shared__ double s[BUB_K][RED_NT];
  double a[BUB_K] = {0, 0, 0};
  for (int b = threadIdx.x; b < nb; b += RED_NT)
    for (int k = 0; k < BUB_K; ++k) a[k] += part[b * BUB_K + k];
  for (int k = 0; k < BUB_K; ++k) s[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int w = RED_NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < BUB_K; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double cnt = s[0][0];
    out[0] = cnt;
    out[1] = cnt > 0 ? s[1][0] / cnt : NAN;
    out[2] = cnt > 0 ? s[2][0] / cnt : NAN;
  }
}

// Pressure jump of the Laplace test (Sec. 4.3): over the nodes with phi > 0.99
// and with phi < -0.99, the sums of p' = rho(clamp phi) p~ and the node counts,
// in float64 partials per workgroup (fixed tree order).
constexpr int PJ_K = 4;
template <typename T>
__global__ __launch_bounds__(RED_NT) void k_pjump1(const T* phi, const T* pt, long long n,
                                                   double rho1, double rho2, double* part) {
  __shared__ double s[PJ_K][RED_NT];
  double a[PJ_K] = {0, 0, 0, 0};
  for (long long id = (long long)blockIdx.x * RED_NT + threadIdx.x; id < n;
       id += (long long)gridDim.x * RED_NT) {
    const double ph = double(phi[id]);
    const double c = ph < -1.0 ? -1.0 : (ph > 1.0 ? 1.0 : ph);
    const double pp = (rho1 * (1.0 + c) / 2.0 + rho2 * (1.0 - c) / 2.0) * double(pt[id]);
    if (ph > 0.99) {
      a[0] += pp;
      a[1] += 1.0;
    } else if (ph < -0.99) {
      a[2] += pp;
      a[3] += 1.0;
    }
  }
  for (int k = 0; k < PJ_K; ++k) s[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int w = RED_NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < PJ_K; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < PJ_K) part[(long long)blockIdx.x * PJ_K + threadIdx.x] = s[threadIdx.x][0];
}

// Velocity-iteration residual (the paper's stopping measure after eq:Fmu):
// sum over nodes of |u^K - u^{K-1}| (both components) and of |u^{K-1}|.
template <typename T>
__global__ __launch_bounds__(RED_NT) void k_resid1(const T* ax, const T* ay, const T* bx,
                                                   const T* by, long long n, double* part) {
  __shared__ double s[2][RED_NT];
  double num = 0, den = 0;
  for (long long id = (long long)blockIdx.x * RED_NT + threadIdx.x; id < n;
       id += (long long)gridDim.x * RED_NT) {
    const double px = double(bx[id]), py = double(by[id]);
    num += fabs(double(ax[id]) - px) + fabs(double(ay[id]) - py);
    den += fabs(px) + fabs(py);
  }
  s[0][threadIdx.x] = num;
  s[1][threadIdx.x] = den;
  __syncthreads();
  for (int w = RED_NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s[0][threadIdx.x] += s[0][threadIdx.x + w];
      s[1][threadIdx.x] += s[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < 2) part[(long long)blockIdx.x * 2 + threadIdx.x] = s[threadIdx.x][0];
}

// sums of K partials per workgroup over nb workgroups, one workgroup, fixed order
template <int K>
__global__ __launch_bounds__(RED_NT) void k_sum_parts(const double* part, int nb, double* out) {
  __shared__ double s[K][RED_NT];
  double a[K];
  for (int k = 0; k < K; ++k) a[k] = 0;
  for (int b = threadIdx.x; b < nb; b += RED_NT)
    for (int k = 0; k < K; ++k) a[k] += part[b * K + k];
  for (int k = 0; k < K; ++k) s[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int w = RED_NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < K; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < K) out[threadIdx.x] = s[threadIdx.x][0];
}

constexpr int RED_BLOCKS = 1024;

inline long long align_up(long long v, long long a) { return (v + a - 1) / a * a; }

}  // namespace

namespace {

template <typename T>
KParams<T> kparams(const lbm2p_ctx* c) {
  KParams<T> k;
  const lbm2p_params& p = c->p;
  k.nx = p.nx;
  k.ny = p.ny;
  k.wx = p.wall_x;
  k.wy = p.wall_y;
  k.ps = c->ps;
  k.c4b = T(c->c4b);
  k.kappa = T(c->kappa);
  k.eta = T(c->eta);
  k.negM = T(c->negM);
  k.lam = T(p.lam);
  k.eps2 = T(c->eps2);
  k.W = T(p.W);
  k.invW = T(1.0 / p.W);
  k.lam12 = T(p.lam / 12.0);
  k.lamW2 = T(2.0 * p.lam / p.W);
  k.negM12 = T(-p.M / 12.0);
  k.eps144 = T(144.0 * c->eps2);
  k.cJ = T(c->cJ);
  k.rho1 = T(p.rho1);
  k.rho2 = T(p.rho2);
  k.mu1 = T(p.mu1);
  k.mu2 = T(p.mu2);
  k.gx = T(p.gx);
  k.gy = T(p.gy);
  k.rho_ref = T(p.rho_ref);
  k.p_ref = T(p.p_ref);
  k.fa = T(p.filter_a);
  for (int i = 0; i < 6; ++i) k.fd[i] = T(c->fd[i]);
  k.fn = c->fn;
  for (int i = 0; i < 9; ++i) {
    k.s_f[i] = T(c->s_f[i]);
    k.s_g[i] = T(c->s_g[i]);
  }
  k.opt = p.options;
  return k;
}

inline unsigned blocks1d(long long n) { return (unsigned)((n + 255) / 256); }

// 1-D grid of tiles (the kernels remap blockIdx to an XCD-contiguous tile order)
template <int TX, int TY>
struct Tiles {
  int tx, ty;
  explicit Tiles(const lbm2p_params& p) : tx((p.nx + TX - 1) / TX), ty((p.ny + TY - 1) / TY) {}
  dim3 grid() const { return dim3((unsigned)(tx * ty)); }
};

// pass ids for profiling
enum { PASS_GATHER = 0, PASS_FD = 1, PASS_VEL = 2, PASS_FILTER = 3, PASS_COLLIDE = 4 };

struct ProfScope {
  lbm2p_ctx* c;
  bool on;
  ProfScope(lbm2p_ctx* c_, int pass) : c(c_), on(c_->prof_pass == pass && c_->prof_n < c_->ev0.size()) {
    // a failed record leaves the launch untimed (lbm2p_profile_read counts it out)
    if (on) on = hipEventRecord(c->ev0[c->prof_n], c->stream) == hipSuccess;
  }
  ~ProfScope() {
    if (on) {
      if (hipEventRecord(c->ev1[c->prof_n], c->stream) == hipSuccess) c->prof_n++;
    }
  }
};

// the tables in the kernels' precision: FP64 reads the host's tables as
// uploaded, FP32 a copy rounded once (uploaded with them, in the room after)
template <typename T>
CompactArgs<T> compact_args(const lbm2p_ctx* c) {
  CompactArgs<T> A;
  for (int k = 0; k < 6; ++k) A.a[k] = c->ca[k];
  A.alpha = c->p.compact_alpha;
  const T* dev = sizeof(T) == 8 ? (const T*)c->ctab_dev : (const T*)c->cfct;
  for (int axis = 0; axis < 2; ++axis)
    for (int par = 0; par < 2; ++par) {
      const int n = c->ctab_n[axis];
      const T* base = dev + c->ctab_off[axis][par];
      const int K = c->cflat[axis][par];
      const double* h = c->ctab_host.data() + c->ctab_off[axis][par];
      CompactLine<T>& L = A.line[axis][par];
      L.cp = base;
      L.inv = base + n;
      L.z = base + 2 * n;
      L.fac = T(c->cfac[axis][par]);
      L.den = T(c->cden[axis][par]);
      L.cyclic = axis == 0 ? !c->p.wall_x : !c->p.wall_y;
      L.K = K;
      L.Z0 = c->cz0[axis][par];
      L.Z1 = c->cz1[axis][par];
      L.cp_lim = T(n >= 2 ? h[K] : 0.0);
      L.inv_lim = T(n >= 2 ? h[n + K] : 0.0);
    }
  return A;
}

// x-lines of n nodes: one workgroup per (line, field) of NT threads with
// chunks of M nodes, the smallest of the shapes that covers the line
template <typename T, int N, int NT, int M>
void launch_cx(lbm2p_ctx* c, const CompactArgs<T>& A, const T* p, const T* ux, const T* uy,
               T* fx) {
  const int nx = c->p.nx, ny = c->p.ny;
  const long long ps = c->ps;
  k_cx<T, N, NT, M><<<3 * ny, NT, cx_lds<T, N, NT, M>(), c->stream>>>(
      A, p, ux, uy, fx, fx + ps, fx + 2 * ps, nx, ny, c->p.wall_x);
}

template <typename T, int N>
void launch_compact(lbm2p_ctx* c, const KParams<T>& K, const T* p, const T* ux, const T* uy,
                    T* po, T* uxo, T* uyo) {
  const CompactArgs<T> A = compact_args<T>(c);
  const int nx = c->p.nx, ny = c->p.ny;
  T* scr = (T*)c->cscratch;  // chunk coefficients and carries of the y-lines
  T* fx = scr + 3 * c->ps;   // F_x of the three fields
  if (nx <= 64 * 16)
    launch_cx<T, N, 64, 16>(c, A, p, ux, uy, fx);
  else if (nx <= 512 * 8)
    launch_cx<T, N, 512, 8>(c, A, p, ux, uy, fx);
  else
    launch_cx<T, N, 512, 16>(c, A, p, ux, uy, fx);
  // y-lines: chunks of MY = 16 rows (32 rows in FP32 measured slower: their
  // registers halve the waves in flight), one chunk row range of 256 columns
  // per workgroup
  constexpr int MY = 16;
  const int nch = (ny + MY - 1) / MY;
  // after the three fields' planes; 3 (7 nch + 1) nx <= 3 nx ny for ny >= 16
  T* fct = scr + 3 * (long long)CY_PLANES * nch * nx;
  const dim3 grid((nx + 255) / 256, nch, 3);
  k_cy_maps<T, N, MY><<<grid, 256, 0, c->stream>>>(K, A, p, ux, uy, scr, nch);
  k_cy_scan<T, 16><<<dim3((nx + 63) / 64, 3), 1024, 0, c->stream>>>(K, A, scr, fct, nch);
  k_cy_apply<T, N, MY><<<grid, 256, 0, c->stream>>>(K, A, p, ux, uy, fx, scr, fct, po, uxo, uyo,
                                                    nch);
}

// Populations larger than the last-level cache (256 MB): the gather and the
// collision stream them with nontemporal accesses.
template <typename T>
bool stream_populations(const lbm2p_ctx* c) {
  return (double)(c->p.coupled ? 18 : 9) * (double)c->n * sizeof(T) > 256.0 * (1 << 20);
}

template <typename T, bool COUPLED, bool STREAM>
void launch_gather(const KParams<T>& K, int par, long long n, hipStream_t st, T* Af, T* Ag,
                   T* phibar, T* praw, T* jx, T* jy, T* m7, T* m8, T* m1 = nullptr) {
  if (par == 0)
    k_gather<T, 0, COUPLED, STREAM><<<blocks1d(n), 256, 0, st>>>(K, Af, Ag, phibar, praw, jx, jy,
                                                                 m7, m8, m1);
  else
    k_gather<T, 1, COUPLED, STREAM><<<blocks1d(n), 256, 0, st>>>(K, Af, Ag, phibar, praw, jx, jy,
                                                                 m7, m8, m1);
}

// the gather of p and j alone (the coupled step's second stream).  It runs
// beside the FD stages, whose workgroups take 16 (FP32: 1024 threads) or 8
// waves of a CU at once: with the usual 4-wave workgroups the gather refilled
// each CU's wave slots as they freed and the first FD stage waited for it
// (58 -> 162 us at 4096^2 FP32).  Workgroups of 1024 threads free 16 slots at a
// time, which the dispatcher shares with the FD stage's.
template <typename T, bool STREAM>
void launch_gather_g(const KParams<T>& K, int par, long long n, hipStream_t st, const T* Ag,
                     T* praw, T* jx, T* jy) {
  constexpr int NTB = 1024;
  const unsigned grid = (unsigned)((n + NTB - 1) / NTB);
  if (par == 0)
    k_gather<T, 0, true, STREAM, true, NTB><<<grid, NTB, 0, st>>>(K, nullptr, Ag, nullptr, praw,
                                                                  jx, jy, nullptr, nullptr, nullptr);
  else
    k_gather<T, 1, true, STREAM, true, NTB><<<grid, NTB, 0, st>>>(K, nullptr, Ag, nullptr, praw,
                                                                  jx, jy, nullptr, nullptr, nullptr);
}

template <typename T, bool COUPLED, bool STREAM>
void launch_collide(lbm2p_ctx* c, const KParams<T>& K, int par, hipStream_t st, T* Af, T* Ag,
                    const T* phi, const T* pt, const T* ux, const T* uy, const T* uox,
                    const T* uoy) {
  using C = StepCfg<T>;
  const Tiles<C::COL_TX, C::COL_TY> tc(c->p);
  if (COUPLED && (K.opt & LBM2P_OPT_STRAIN_MOMENTS)) {   // the option's own instantiation
    if (par == 0)
      k_collide<T, 0, COUPLED, false, C::COL_TX, C::COL_TY, C::COL_NT, true>
          <<<tc.grid(), C::COL_NT, 0, st>>>(K, tc.tx, Af, Ag, phi, pt, ux, uy, uox, uoy);
    else
      k_collide<T, 1, COUPLED, false, C::COL_TX, C::COL_TY, C::COL_NT, true>
          <<<tc.grid(), C::COL_NT, 0, st>>>(K, tc.tx, Af, Ag, phi, pt, ux, uy, uox, uoy);
    return;
  }
  if constexpr (!STREAM) {   // small lattices (never streamed): the small tiles
    if (tc.tx * (long long)tc.ty < TINY_TILES) {
      const Tiles<C::COLT_TX, C::COLT_TY> tt(c->p);
      if (par == 0)
        k_collide<T, 0, COUPLED, STREAM, C::COLT_TX, C::COLT_TY, C::COLT_NT>
            <<<tt.grid(), C::COLT_NT, 0, st>>>(K, tt.tx, Af, Ag, phi, pt, ux, uy, uox, uoy);
      else
        k_collide<T, 1, COUPLED, STREAM, C::COLT_TX, C::COLT_TY, C::COLT_NT>
            <<<tt.grid(), C::COLT_NT, 0, st>>>(K, tt.tx, Af, Ag, phi, pt, ux, uy, uox, uoy);
      return;
    }
  }
  if (par == 0)
    k_collide<T, 0, COUPLED, STREAM, C::COL_TX, C::COL_TY, C::COL_NT>
        <<<tc.grid(), C::COL_NT, 0, st>>>(K, tc.tx, Af, Ag, phi, pt, ux, uy, uox, uoy);
  else
    k_collide<T, 1, COUPLED, STREAM, C::COL_TX, C::COL_TY, C::COL_NT>
        <<<tc.grid(), C::COL_NT, 0, st>>>(K, tc.tx, Af, Ag, phi, pt, ux, uy, uox, uoy);
}

// the three TVD-RK3 stages with TY x NT tiles
template <typename T, int TY, int NT>
void launch_fd(lbm2p_ctx* c, const KParams<T>& K, hipStream_t st, T* phibar, T* phi1, T* phi2,
               T* phi, int gpar = -1) {
  constexpr int TX = StepCfg<T>::TX;
  const Tiles<TX, TY> tl(c->p);
  {
    ProfScope ps(c, PASS_FD);
    const FoldedGather<T> G{(const T*)c->Af, (const T*)c->Ag, phibar, (T*)c->praw, (T*)c->jx,
                            (T*)c->jy};
    const bool cp = c->p.coupled != 0;
    if (gpar == 0 && cp)
      k_fd<T, 1, TX, TY, NT, 0, true><<<tl.grid(), NT, 0, st>>>(K, tl.tx, nullptr, nullptr, phi1, G);
    else if (gpar == 1 && cp)
      k_fd<T, 1, TX, TY, NT, 1, true><<<tl.grid(), NT, 0, st>>>(K, tl.tx, nullptr, nullptr, phi1, G);
    else if (gpar == 0)
      k_fd<T, 1, TX, TY, NT, 0><<<tl.grid(), NT, 0, st>>>(K, tl.tx, nullptr, nullptr, phi1, G);
    else if (gpar == 1)
      k_fd<T, 1, TX, TY, NT, 1><<<tl.grid(), NT, 0, st>>>(K, tl.tx, nullptr, nullptr, phi1, G);
    else
      k_fd<T, 1, TX, TY, NT><<<tl.grid(), NT, 0, st>>>(K, tl.tx, phibar, phibar, phi1);
  }
  {
    ProfScope ps(c, PASS_FD);
    k_fd<T, 2, TX, TY, NT><<<tl.grid(), NT, 0, st>>>(K, tl.tx, phi1, phibar, phi2);
  }
  {
    ProfScope ps(c, PASS_FD);
    k_fd<T, 3, TX, TY, NT><<<tl.grid(), NT, 0, st>>>(K, tl.tx, phi2, phibar, phi);
  }
}

// one velocity launch (two sweeps, or one) with TY x NT tiles
template <typename T, int TY, int NT>
void launch_vel(const lbm2p_params& p, const KParams<T>& K, hipStream_t st, bool two, const T* phi,
                const T* praw, const T* jx, const T* jy, const T* ux, const T* uy, T* ox, T* oy,
                T* o1x, T* o1y, const T* m1 = nullptr, const T* m7 = nullptr,
                const T* m8 = nullptr) {
  constexpr int TX = StepCfg<T>::TX;
  const Tiles<TX, TY> tv(p);
  if (m1) {   // moment strain rate: its own instantiations
    if (two)
      k_vel2<T, TX, TY, NT, true><<<tv.grid(), NT, 0, st>>>(K, tv.tx, phi, praw, jx, jy, ux, uy,
                                                              ox, oy, o1x, o1y, m1, m7, m8);
    else
      k_vel<T, 1, TX, TY, NT, true><<<tv.grid(), NT, 0, st>>>(K, tv.tx, phi, praw, jx, jy, ux, uy,
                                                                ox, oy, m1, m7, m8);
    return;
  }
  if (two)
    k_vel2<T, TX, TY, NT><<<tv.grid(), NT, 0, st>>>(K, tv.tx, phi, praw, jx, jy, ux, uy, ox, oy,
                                                    o1x, o1y);
  else
    k_vel<T, 1, TX, TY, NT><<<tv.grid(), NT, 0, st>>>(K, tv.tx, phi, praw, jx, jy, ux, uy, ox, oy);
}

// the explicit filter SF-(2N+1) with TY x NT tiles
template <typename T, int TY, int NT>
void launch_filter(const lbm2p_ctx* c, const KParams<T>& K, hipStream_t st, const T* pr,
                   const T* ux, const T* uy, T* po, T* unx, T* uny) {
  constexpr int TX = StepCfg<T>::TX;
  const Tiles<TX, TY> tf(c->p);
  switch (c->fn) {
    case 2: k_filter<T, 2, TX, TY, NT><<<tf.grid(), NT, 0, st>>>(K, tf.tx, pr, ux, uy, po, unx, uny); break;
    case 3: k_filter<T, 3, TX, TY, NT><<<tf.grid(), NT, 0, st>>>(K, tf.tx, pr, ux, uy, po, unx, uny); break;
    case 4: k_filter<T, 4, TX, TY, NT><<<tf.grid(), NT, 0, st>>>(K, tf.tx, pr, ux, uy, po, unx, uny); break;
    default: k_filter<T, 5, TX, TY, NT><<<tf.grid(), NT, 0, st>>>(K, tf.tx, pr, ux, uy, po, unx, uny); break;
  }
}

template <typename T>
int step_impl(lbm2p_ctx* c, int nsteps) {
  const lbm2p_params& p = c->p;
  const KParams<T> K = kparams<T>(c);
  const long long n = c->n;
  hipStream_t st = c->stream;
  T* Af = (T*)c->Af;
  T* Ag = (T*)c->Ag;
  T* phi = (T*)c->phi;
  T* phibar = (T*)c->phibar;
  T* phi1 = (T*)c->phi1;
  T* phi2 = (T*)c->phi2;
  const bool stream = stream_populations<T>(c);
  using Cs = StepCfg<T>;
  const Tiles<Cs::TX, Cs::FDS_TY> tls0(p);
  // On a lattice of few tiles the gather is folded into the first FD stage (one
  // launch less on a step that is a few launches' latency); not while recording
  // for the adjoint or with the moment strain rate (their gather keeps moments
  // of g besides)
  const bool fold_gather = !p.original_ch && tls0.tx * (long long)tls0.ty < TINY_TILES &&
                           !(p.coupled && (c->rec || (p.options & LBM2P_OPT_STRAIN_MOMENTS)));
  for (int s = 0; s < nsteps; ++s) {
    const int par = c->parity;
    // Coupled steps split the gather: p and j on the second stream, beside the
    // FD stages, which need only phi_bar (the FD stages are instruction-bound
    // and leave HBM bandwidth to the gather of g); the velocity sweeps wait for
    // it.  Only on lattices whose populations exceed the last-level cache (on
    // smaller ones the fork and join cost more than the overlap gains: +18 us
    // a step at 256 x 1024); not while recording (that gather keeps m_7, m_8
    // too), with the moment strain rate, or while the gather or FD pass is
    // profiled (lbm2p_profile then times them in the serial order).
    const bool split = p.coupled && stream && c->g_stream && c->g_ev[1] && !c->rec &&
                       !(p.options & LBM2P_OPT_STRAIN_MOMENTS) &&
                       c->prof_pass != PASS_GATHER && c->prof_pass != PASS_FD;
    if (split) {
      // phi_bar first, alone (the FD stages wait for it), then p and j on the
      // second stream while the FD stages run
      if (stream)
        launch_gather<T, false, true>(K, par, n, st, Af, Ag, phibar, nullptr, nullptr, nullptr,
                                      nullptr, nullptr);
      else
        launch_gather<T, false, false>(K, par, n, st, Af, Ag, phibar, nullptr, nullptr, nullptr,
                                       nullptr, nullptr);
      if (hipEventRecord(c->g_ev[0], st) != hipSuccess ||
          hipStreamWaitEvent(c->g_stream, c->g_ev[0], 0) != hipSuccess)
        return LBM2P_EHIP;
      if (stream)
        launch_gather_g<T, true>(K, par, n, c->g_stream, Ag, (T*)c->praw, (T*)c->jx, (T*)c->jy);
      else
        launch_gather_g<T, false>(K, par, n, c->g_stream, Ag, (T*)c->praw, (T*)c->jx, (T*)c->jy);
      if (hipEventRecord(c->g_ev[1], c->g_stream) != hipSuccess) return LBM2P_EHIP;
    } else if (!fold_gather) {
      ProfScope ps(c, PASS_GATHER);
      // while recording for the adjoint, the gather also keeps m_7, m_8 of the
      // pre-collision g (the g-relaxation rate's derivative needs them)
      // (with the moment strain rate it keeps m_1, m_7, m_8 for the velocity sweeps)
      const bool sm = p.coupled && (p.options & LBM2P_OPT_STRAIN_MOMENTS);
      T* m7 = c->rec && p.coupled ? (T*)c->rec_m7 : (sm ? (T*)c->sm7 : nullptr);
      T* m8 = c->rec && p.coupled ? (T*)c->rec_m8 : (sm ? (T*)c->sm8 : nullptr);
      T* m1 = sm ? (T*)c->sm1 : nullptr;
      T* praw = p.coupled ? (T*)c->praw : nullptr;
      T* jx = p.coupled ? (T*)c->jx : nullptr;
      T* jy = p.coupled ? (T*)c->jy : nullptr;
      if (p.coupled) {
        if (stream) launch_gather<T, true, true>(K, par, n, st, Af, Ag, phibar, praw, jx, jy, m7, m8, m1);
        else launch_gather<T, true, false>(K, par, n, st, Af, Ag, phibar, praw, jx, jy, m7, m8, m1);
      } else {
        if (stream) launch_gather<T, false, true>(K, par, n, st, Af, Ag, phibar, praw, jx, jy, m7, m8);
        else launch_gather<T, false, false>(K, par, n, st, Af, Ag, phibar, praw, jx, jy, m7, m8);
      }
    }
    if (p.original_ch) {
      k_copy<T><<<blocks1d(n), 256, 0, st>>>(phibar, phi, n);
    } else {
      using C = StepCfg<T>;
      const Tiles<C::TX, C::FD_TY> tl(p);
      const Tiles<C::TX, C::FDS_TY> tls(p);
      if (tl.tx * (long long)tl.ty >= FD_MIN_TILES)
        launch_fd<T, C::FD_TY, C::FD_NT>(c, K, st, phibar, phi1, phi2, phi);
      else if (tls.tx * (long long)tls.ty >= TINY_TILES)
        launch_fd<T, C::FDS_TY, C::FDS_NT>(c, K, st, phibar, phi1, phi2, phi);
      else
        launch_fd<T, TINY_TY, TINY_NT>(c, K, st, phibar, phi1, phi2, phi, fold_gather ? par : -1);
    }
    if (p.coupled) {
      if (split && hipStreamWaitEvent(st, c->g_ev[1], 0) != hipSuccess) return LBM2P_EHIP;
      T* uox = (T*)c->U[c->uo][0];
      T* uoy = (T*)c->U[c->uo][1];
      T* unx = (T*)c->U[1 - c->uo][0];
      T* uny = (T*)c->U[1 - c->uo][1];
      const T* ux = uox;
      const T* uy = uoy;
      using C = StepCfg<T>;
      const Tiles<C::TX, C::VEL_TY> tv(p);
      int done = 0, launch = 0;
      // residual tracking (outside record mode): the last sweep runs alone, so
      // that its input u^{K-1} stays in a plane (u~^n for K = 1)
      const bool track = c->track_resid && !c->rec;
      while (done < p.K) {
        // two sweeps per launch, one for an odd remainder; when recording for
        // the adjoint, every iterate u^{s+1} goes to its own plane rec_uk[s]
        // (the two-sweep kernel then also writes its first sweep's result)
        const bool two = p.K - done >= (track ? 3 : 2);
        const int last = done + (two ? 1 : 0);
        T* ox = (T*)(c->rec ? c->rec_uk[last][0] : c->uk[launch & 1][0]);
        T* oy = (T*)(c->rec ? c->rec_uk[last][1] : c->uk[launch & 1][1]);
        T* o1x = (T*)(c->rec && two ? c->rec_uk[done][0] : nullptr);
        T* o1y = (T*)(c->rec && two ? c->rec_uk[done][1] : nullptr);
        ProfScope ps(c, PASS_VEL);
        if (p.options & LBM2P_OPT_STRAIN_MOMENTS)
          launch_vel<T, C::VEL_TY, C::VEL_NT>(p, K, st, two, phi, (T*)c->praw, (T*)c->jx,
                                              (T*)c->jy, ux, uy, ox, oy, o1x, o1y,
                                              (const T*)c->sm1, (const T*)c->sm7,
                                              (const T*)c->sm8);
        else if (tv.tx * (long long)tv.ty < TINY_TILES)
          launch_vel<T, TINY_TY, TINY_NT>(
              p, K, st, two, phi, (T*)c->praw, (T*)c->jx, (T*)c->jy, ux, uy, ox, oy, o1x, o1y);
        else if (tv.tx * (long long)tv.ty < VEL_MIN_TILES)
          launch_vel<T, VelSmall<T>::TY, VelSmall<T>::NT>(
              p, K, st, two, phi, (T*)c->praw, (T*)c->jx, (T*)c->jy, ux, uy, ox, oy, o1x, o1y);
        else
          launch_vel<T, C::VEL_TY, C::VEL_NT>(p, K, st, two, phi, (T*)c->praw, (T*)c->jx,
                                              (T*)c->jy, ux, uy, ox, oy, o1x, o1y);
        done += two ? 2 : 1;
        if (done == p.K) {
          c->res_prev[0] = (void*)ux;
          c->res_prev[1] = (void*)uy;
          c->res_last[0] = ox;
          c->res_last[1] = oy;
        }
        ux = ox;
        uy = oy;
        ++launch;
      }
      c->uk_last = (launch - 1) & 1;
      c->res_valid = track ? 1 : 0;
      if (p.compact) {
        ProfScope ps(c, PASS_FILTER);
        const T* pr = (const T*)c->praw;
        switch (p.compact_n) {
          case 1: launch_compact<T, 1>(c, K, pr, ux, uy, (T*)c->pt, unx, uny); break;
          case 2: launch_compact<T, 2>(c, K, pr, ux, uy, (T*)c->pt, unx, uny); break;
          case 3: launch_compact<T, 3>(c, K, pr, ux, uy, (T*)c->pt, unx, uny); break;
          case 4: launch_compact<T, 4>(c, K, pr, ux, uy, (T*)c->pt, unx, uny); break;
          default: launch_compact<T, 5>(c, K, pr, ux, uy, (T*)c->pt, unx, uny); break;
        }
      } else if (p.filter_n == 0) {
        k_copy<T><<<blocks1d(n), 256, 0, st>>>((T*)c->praw, (T*)c->pt, n);
        k_copy<T><<<blocks1d(n), 256, 0, st>>>(ux, unx, n);
        k_copy<T><<<blocks1d(n), 256, 0, st>>>(uy, uny, n);
      } else {
        ProfScope ps(c, PASS_FILTER);
        const Tiles<C::TX, C::FIL_TY> tf(p);
        const T* pr = (const T*)c->praw;
        T* po = (T*)c->pt;
        if (tf.tx * (long long)tf.ty < TINY_TILES)
          launch_filter<T, TINY_TY, TINY_NT>(c, K, st, pr, ux, uy, po, unx, uny);
        else
          launch_filter<T, C::FIL_TY, C::FIL_NT>(c, K, st, pr, ux, uy, po, unx, uny);
      }
      {
        ProfScope ps(c, PASS_COLLIDE);
        if (stream)
          launch_collide<T, true, true>(c, K, par, st, Af, Ag, phi, (T*)c->pt, unx, uny, uox, uoy);
        else
          launch_collide<T, true, false>(c, K, par, st, Af, Ag, phi, (T*)c->pt, unx, uny, uox, uoy);
      }
      c->uo = 1 - c->uo;
    } else {
      // the prescribed velocity; d_t u from the one the last step used when
      // lbm2p_set_velocity replaced it since (R18 of the oracle's readings)
      T* ux = (T*)c->U[0][0];
      T* uy = (T*)c->U[0][1];
      T* uox = (T*)c->U[c->vpend ? 1 : 0][0];
      T* uoy = (T*)c->U[c->vpend ? 1 : 0][1];
      ProfScope ps(c, PASS_COLLIDE);
      if (stream)
        launch_collide<T, false, true>(c, K, par, st, Af, Ag, phi, nullptr, ux, uy, uox, uoy);
      else
        launch_collide<T, false, false>(c, K, par, st, Af, Ag, phi, nullptr, ux, uy, uox, uoy);
      c->vpend = 0;
    }
    c->parity ^= 1;
    c->steps++;
    c->from_init = 0;
  }
  return hipGetLastError() == hipSuccess ? LBM2P_OK : LBM2P_EHIP;
}

template <typename T>
int init_impl(lbm2p_ctx* c, const double* phi0, const double* ux0, const double* uy0,
              const double* p0) {
  if (c->ctab_dev && !c->ctab_uploaded) {
    // the FP64 tables (2 parities x 3 per axis), and in FP32 their rounded copy
    const size_t nt = 2 * 3 * ((size_t)c->p.nx + (size_t)c->p.ny);
    std::vector<float> t32;
    if (hipMemcpyAsync(c->ctab_dev, c->ctab_host.data(), nt * sizeof(double),
                       hipMemcpyHostToDevice, c->stream) != hipSuccess)
      return LBM2P_EHIP;
    if (sizeof(T) == 4) {
      t32.assign(c->ctab_host.begin(), c->ctab_host.begin() + nt);
      if (hipMemcpyAsync(c->cfct, t32.data(), nt * sizeof(float), hipMemcpyHostToDevice,
                         c->stream) != hipSuccess)
        return LBM2P_EHIP;
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) return LBM2P_EHIP;
    c->ctab_uploaded = 1;
  }
  const KParams<T> K = kparams<T>(c);
  T* ux = (T*)c->U[0][0];
  T* uy = (T*)c->U[0][1];
  k_init<T><<<blocks1d(c->n), 256, 0, c->stream>>>(K, c->c4b, c->kappa, c->eta, c->p.p_ref,
                                                   phi0, ux0, uy0, p0,
                                                   (T*)c->Af, (T*)c->Ag, (T*)c->phi,
                                                   c->p.coupled ? (T*)c->pt : (T*)c->phi2, ux, uy,
                                                   c->p.coupled);
  c->uo = 0;
  c->vpend = 0;
  c->parity = 0;
  c->steps = 0;
  c->inited = 1;
  c->from_init = 1;
  c->adj_ready = 0;
  c->res_valid = 0;
  return hipGetLastError() == hipSuccess ? LBM2P_OK : LBM2P_EHIP;
}

template <typename T>
int to_f64(lbm2p_ctx* c, const void* src, double* dst) {
  if (!dst) return LBM2P_OK;
  k_to_f64<T><<<blocks1d(c->n), 256, 0, c->stream>>>((const T*)src, dst, c->n);
  return LBM2P_OK;
}

template <typename T>
int moments_impl(lbm2p_ctx* c, double* phi, double* ux, double* uy, double* p, double* rho) {
  const int u = c->p.coupled ? c->uo : 0;
  to_f64<T>(c, c->phi, phi);
  to_f64<T>(c, c->U[u][0], ux);
  to_f64<T>(c, c->U[u][1], uy);
  if (p) {
    if (c->p.coupled)
      to_f64<T>(c, c->pt, p);
    else
      k_fill<double><<<blocks1d(c->n), 256, 0, c->stream>>>(p, 0.0, c->n);
  }
  if (rho)
    k_rho<T><<<blocks1d(c->n), 256, 0, c->stream>>>((const T*)c->phi, rho, c->n, c->p.rho1,
                                                    c->p.rho2);
  return hipGetLastError() == hipSuccess ? LBM2P_OK : LBM2P_EHIP;
}

template <typename T>
int volume_impl(lbm2p_ctx* c, double out[6]) {
  const int u = c->p.coupled ? c->uo : 0;
  k_reduce1<T><<<RED_BLOCKS, RED_NT, 0, c->stream>>>((const T*)c->phi, (const T*)c->pt,
                                                     (const T*)c->U[u][0], (const T*)c->U[u][1],
                                                     c->n, c->red, c->p.coupled);
  double* res = c->red + RED_BLOCKS * RED_K;
  k_reduce2<<<1, RED_NT, 0, c->stream>>>(c->red, RED_BLOCKS, res);
  if (hipMemcpyAsync(out, res, RED_K * sizeof(double), hipMemcpyDeviceToHost, c->stream) !=
      hipSuccess)
    return LBM2P_EHIP;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LBM2P_EHIP;
  if (!std::isfinite(out[1]) || !std::isfinite(out[3])) return LBM2P_ENONFINITE;
  return LBM2P_OK;
}

template <typename T>
int bubble_impl(lbm2p_ctx* c, double out[3]) {
  const int u = c->p.coupled ? c->uo : 0;
  // the partials fit in the reduction scratch (RED_BLOCKS + 1) * RED_K doubles
  static_assert(BUB_K <= RED_K, "bubble partials in the reduction scratch");
  k_bubble1<T><<<RED_BLOCKS, RED_NT, 0, c->stream>>>((const T*)c->phi, (const T*)c->U[u][1],
                                                     c->p.nx, c->n, c->red);
  double* res = c->red + RED_BLOCKS * BUB_K;
  k_bubble2<<<1, RED_NT, 0, c->stream>>>(c->red, RED_BLOCKS, res);
  if (hipMemcpyAsync(out, res, BUB_K * sizeof(double), hipMemcpyDeviceToHost, c->stream) !=
      hipSuccess)
    return LBM2P_EHIP;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LBM2P_EHIP;
  return LBM2P_OK;
}

template <typename T>
int pjump_impl(lbm2p_ctx* c, double out[5]) {
  static_assert(PJ_K <= RED_K, "pressure-jump partials in the reduction scratch");
  k_pjump1<T><<<RED_BLOCKS, RED_NT, 0, c->stream>>>((const T*)c->phi, (const T*)c->pt, c->n,
                                                    c->p.rho1, c->p.rho2, c->red);
  double* res = c->red + RED_BLOCKS * PJ_K;
  k_sum_parts<PJ_K><<<1, RED_NT, 0, c->stream>>>(c->red, RED_BLOCKS, res);
  double h[PJ_K];
  if (hipMemcpyAsync(h, res, PJ_K * sizeof(double), hipMemcpyDeviceToHost, c->stream) !=
      hipSuccess)
    return LBM2P_EHIP;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LBM2P_EHIP;
  const double in = h[1] > 0 ? h[0] / h[1] : NAN, outm = h[3] > 0 ? h[2] / h[3] : NAN;
  out[0] = in - outm;
  out[1] = in;
  out[2] = outm;
  out[3] = h[1];
  out[4] = h[3];
  return LBM2P_OK;
}

template <typename T>
int resid_impl(lbm2p_ctx* c, double* out) {
  k_resid1<T><<<RED_BLOCKS, RED_NT, 0, c->stream>>>(
      (const T*)c->res_last[0], (const T*)c->res_last[1], (const T*)c->res_prev[0],
      (const T*)c->res_prev[1], c->n, c->red);
  double* res = c->red + RED_BLOCKS * 2;
  k_sum_parts<2><<<1, RED_NT, 0, c->stream>>>(c->red, RED_BLOCKS, res);
  double h[2];
  if (hipMemcpyAsync(h, res, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return LBM2P_EHIP;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LBM2P_EHIP;
  *out = h[1] > 0 ? h[0] / h[1] : 0.0;
  return LBM2P_OK;
}

template <typename T>
int state_impl(lbm2p_ctx* c, double* f, double* g, double* u, int set) {
  const KParams<T> K = kparams<T>(c);
  if (set) {
    c->from_init = 0;
    c->adj_ready = 0;
    c->res_valid = 0;
    c->vpend = 0;
  }
  if (f) k_state<T><<<blocks1d(c->n), 256, 0, c->stream>>>(K, (T*)c->Af, f, c->parity, set, 0.0);
  if (g && c->p.coupled)
    k_state<T><<<blocks1d(c->n), 256, 0, c->stream>>>(K, (T*)c->Ag, g, c->parity, set,
                                                      3.0 * c->p.p_ref);
  if (u) {
    const int ui = c->p.coupled ? c->uo : 0;
    for (int k = 0; k < 2; ++k) {
      if (set)
        k_from_f64<T><<<blocks1d(c->n), 256, 0, c->stream>>>(u + k * c->n, (T*)c->U[ui][k], c->n);
      else
        k_to_f64<T><<<blocks1d(c->n), 256, 0, c->stream>>>((const T*)c->U[ui][k], u + k * c->n,
                                                           c->n);
    }
  }
  return hipGetLastError() == hipSuccess ? LBM2P_OK : LBM2P_EHIP;
}

// CH-only mode: the prescribed velocity of the following steps into U[0];
// the velocity the last step used is kept in U[1] for the next step's d_t u
template <typename T>
int setvel_impl(lbm2p_ctx* c, const double* ux, const double* uy) {
  const long long n = c->n;
  if (!c->vpend) {
    k_copy<T><<<blocks1d(n), 256, 0, c->stream>>>((const T*)c->U[0][0], (T*)c->U[1][0], n);
    k_copy<T><<<blocks1d(n), 256, 0, c->stream>>>((const T*)c->U[0][1], (T*)c->U[1][1], n);
  }
  k_from_f64<T><<<blocks1d(n), 256, 0, c->stream>>>(ux, (T*)c->U[0][0], n);
  k_from_f64<T><<<blocks1d(n), 256, 0, c->stream>>>(uy, (T*)c->U[0][1], n);
  c->vpend = 1;
  c->from_init = 0;
  c->adj_ready = 0;
  return hipGetLastError() == hipSuccess ? LBM2P_OK : LBM2P_EHIP;
}

}  // namespace

}  // namespace lbm2p
