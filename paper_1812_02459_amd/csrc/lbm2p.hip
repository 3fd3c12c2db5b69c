// C ABI (include/lbm2p.h) and host-side orchestration of one lattice update.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/lbm2p.h"
#include "lbm2p_kernels.h"

using namespace lbm2p;

namespace {

// ------------------------------------------------------------ utility kernels
// Equilibrium initial populations (R15 of the oracle's readings): mu(phi0) with
// the isotropic Laplacian, f* = f^eq(phi0, mu, u0), g* = g^eq(p0, u0), stored in
// the parity-0 layout (f*_i(x) at A[opp(i)][x]).  Evaluated in float64.
template <typename T>
__global__ __launch_bounds__(256) void k_init(KParams<T> P, double c4b, double kappa, double eta,
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
    g_eq<double>(p, u_x, u_y, geq);
#pragma unroll
    for (int i = 0; i < 9; ++i) Ag[opp(i) * P.ps + id] = T(geq[i]);
  }
  phi[id] = T(ph);
  pt[id] = T(p);
  ux[id] = T(u_x);
  uy[id] = T(u_y);
}

// canonical f*_i(x) <-> in-place layout of the given parity
template <typename T>
__global__ __launch_bounds__(256) void k_state(KParams<T> P, T* A, double* canon, int parity, int set) {
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
      A[loc] = T(canon[i * n + id]);
    else
      canon[i * n + id] = double(A[loc]);
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

constexpr int RED_BLOCKS = 1024;

// tile shapes (nodes per workgroup of 256 threads)
constexpr int FD_TX = 64, FD_TY = 16;
constexpr int VEL_TX = 64, VEL_TY = 8;
constexpr int FIL_TX = 64, FIL_TY = 16;
constexpr int COL_TX = 64, COL_TY = 4;

inline long long align_up(long long v, long long a) { return (v + a - 1) / a * a; }

}  // namespace

// ----------------------------------------------------------------- context
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
  int parity;
  int inited;
  long long steps;
  // derived constants (float64, computed exactly as the oracle computes them)
  double kappa, beta, eta, c4b, negM, cJ, eps2;
  double s_f[9], s_g[9];
  double fd[6];
  int fn;
  // profiling
  int prof_pass;
  std::vector<hipEvent_t> ev0, ev1;
  size_t prof_n;
};

namespace {

int validate(const lbm2p_params* p) {
  if (!p) return LBM2P_EINVAL;
  if (p->nx < 16 || p->ny < 16) return LBM2P_EINVAL;
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
  if (p->compact) return LBM2P_EINVAL;  // compact variant: not in this library build
  if (p->K < 1 || p->K > 8) return LBM2P_EINVAL;
  if (!(p->filter_a >= 0 && p->filter_a <= 1)) return LBM2P_EINVAL;
  if (p->coupled != 0 && p->coupled != 1) return LBM2P_EINVAL;
  if (p->reserved != 0) return LBM2P_EINVAL;
  return LBM2P_OK;
}

long long plane_stride(const lbm2p_params* p) {
  return align_up((long long)p->nx * p->ny, 64);
}

size_t n_planes(const lbm2p_params* p) {
  // f(9) + phi, phibar, phi1, phi2 + U(4)  [+ g(9) + praw, jx, jy, pt + uk(4)]
  return p->coupled ? 9 + 4 + 4 + 9 + 4 + 4 : 9 + 4 + 4;
}

size_t ws_size(const lbm2p_params* p) {
  const size_t esz = p->precision ? 4 : 8;
  return n_planes(p) * (size_t)plane_stride(p) * esz + (RED_BLOCKS + 1) * RED_K * sizeof(double) +
         256;
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
  k.cJ = T(c->cJ);
  k.rho1 = T(p.rho1);
  k.rho2 = T(p.rho2);
  k.mu1 = T(p.mu1);
  k.mu2 = T(p.mu2);
  k.gx = T(p.gx);
  k.gy = T(p.gy);
  k.rho_ref = T(p.rho_ref);
  k.fa = T(p.filter_a);
  for (int i = 0; i < 6; ++i) k.fd[i] = T(c->fd[i]);
  k.fn = c->fn;
  for (int i = 0; i < 9; ++i) {
    k.s_f[i] = T(c->s_f[i]);
    k.s_g[i] = T(c->s_g[i]);
  }
  return k;
}

inline unsigned blocks1d(long long n) { return (unsigned)((n + 255) / 256); }

template <int TX, int TY>
inline dim3 grid2d(const lbm2p_params& p) {
  return dim3((p.nx + TX - 1) / TX, (p.ny + TY - 1) / TY);
}

// pass ids for profiling
enum { PASS_GATHER = 0, PASS_FD = 1, PASS_VEL = 2, PASS_FILTER = 3, PASS_COLLIDE = 4 };

struct ProfScope {
  lbm2p_ctx* c;
  bool on;
  ProfScope(lbm2p_ctx* c_, int pass) : c(c_), on(c_->prof_pass == pass && c_->prof_n < c_->ev0.size()) {
    if (on) hipEventRecord(c->ev0[c->prof_n], c->stream);
  }
  ~ProfScope() {
    if (on) {
      hipEventRecord(c->ev1[c->prof_n], c->stream);
      c->prof_n++;
    }
  }
};

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
  for (int s = 0; s < nsteps; ++s) {
    const int par = c->parity;
    {
      ProfScope ps(c, PASS_GATHER);
      if (p.coupled) {
        if (par == 0)
          k_gather<T, 0, true><<<blocks1d(n), 256, 0, st>>>(K, Af, Ag, phibar, (T*)c->praw,
                                                             (T*)c->jx, (T*)c->jy);
        else
          k_gather<T, 1, true><<<blocks1d(n), 256, 0, st>>>(K, Af, Ag, phibar, (T*)c->praw,
                                                             (T*)c->jx, (T*)c->jy);
      } else {
        if (par == 0)
          k_gather<T, 0, false><<<blocks1d(n), 256, 0, st>>>(K, Af, Ag, phibar, nullptr, nullptr,
                                                              nullptr);
        else
          k_gather<T, 1, false><<<blocks1d(n), 256, 0, st>>>(K, Af, Ag, phibar, nullptr, nullptr,
                                                              nullptr);
      }
    }
    if (p.original_ch) {
      k_copy<T><<<blocks1d(n), 256, 0, st>>>(phibar, phi, n);
    } else {
      const dim3 g = grid2d<FD_TX, FD_TY>(p);
      {
        ProfScope ps(c, PASS_FD);
        k_fd<T, 1, FD_TX, FD_TY><<<g, 256, 0, st>>>(K, phibar, phibar, phi1);
      }
      {
        ProfScope ps(c, PASS_FD);
        k_fd<T, 2, FD_TX, FD_TY><<<g, 256, 0, st>>>(K, phi1, phibar, phi2);
      }
      {
        ProfScope ps(c, PASS_FD);
        k_fd<T, 3, FD_TX, FD_TY><<<g, 256, 0, st>>>(K, phi2, phibar, phi);
      }
    }
    if (p.coupled) {
      T* uox = (T*)c->U[c->uo][0];
      T* uoy = (T*)c->U[c->uo][1];
      T* unx = (T*)c->U[1 - c->uo][0];
      T* uny = (T*)c->U[1 - c->uo][1];
      const T* ux = uox;
      const T* uy = uoy;
      for (int k = 0; k < p.K; ++k) {
        T* ox = (T*)c->uk[k & 1][0];
        T* oy = (T*)c->uk[k & 1][1];
        ProfScope ps(c, PASS_VEL);
        k_vel<T, VEL_TX, VEL_TY><<<grid2d<VEL_TX, VEL_TY>(p), 256, 0, st>>>(
            K, phi, (T*)c->praw, (T*)c->jx, (T*)c->jy, ux, uy, ox, oy);
        ux = ox;
        uy = oy;
      }
      if (p.filter_n == 0) {
        k_copy<T><<<blocks1d(n), 256, 0, st>>>((T*)c->praw, (T*)c->pt, n);
        k_copy<T><<<blocks1d(n), 256, 0, st>>>(ux, unx, n);
        k_copy<T><<<blocks1d(n), 256, 0, st>>>(uy, uny, n);
      } else {
        ProfScope ps(c, PASS_FILTER);
        k_filter<T, FIL_TX, FIL_TY><<<grid2d<FIL_TX, FIL_TY>(p), 256, 0, st>>>(
            K, (T*)c->praw, ux, uy, (T*)c->pt, unx, uny);
      }
      {
        ProfScope ps(c, PASS_COLLIDE);
        const dim3 g = grid2d<COL_TX, COL_TY>(p);
        if (par == 0)
          k_collide<T, 0, true, COL_TX, COL_TY><<<g, 256, 0, st>>>(K, Af, Ag, phi, (T*)c->pt, unx,
                                                                   uny, uox, uoy);
        else
          k_collide<T, 1, true, COL_TX, COL_TY><<<g, 256, 0, st>>>(K, Af, Ag, phi, (T*)c->pt, unx,
                                                                   uny, uox, uoy);
      }
      c->uo = 1 - c->uo;
    } else {
      T* ux = (T*)c->U[0][0];
      T* uy = (T*)c->U[0][1];
      ProfScope ps(c, PASS_COLLIDE);
      const dim3 g = grid2d<COL_TX, COL_TY>(p);
      if (par == 0)
        k_collide<T, 0, false, COL_TX, COL_TY><<<g, 256, 0, st>>>(K, Af, Ag, phi, nullptr, ux, uy,
                                                                  ux, uy);
      else
        k_collide<T, 1, false, COL_TX, COL_TY><<<g, 256, 0, st>>>(K, Af, Ag, phi, nullptr, ux, uy,
                                                                  ux, uy);
    }
    c->parity ^= 1;
    c->steps++;
  }
  return hipGetLastError() == hipSuccess ? LBM2P_OK : LBM2P_EHIP;
}

template <typename T>
int init_impl(lbm2p_ctx* c, const double* phi0, const double* ux0, const double* uy0,
              const double* p0) {
  const KParams<T> K = kparams<T>(c);
  T* ux = (T*)c->U[0][0];
  T* uy = (T*)c->U[0][1];
  k_init<T><<<blocks1d(c->n), 256, 0, c->stream>>>(K, c->c4b, c->kappa, c->eta, phi0, ux0, uy0, p0,
                                                   (T*)c->Af, (T*)c->Ag, (T*)c->phi,
                                                   c->p.coupled ? (T*)c->pt : (T*)c->phi2, ux, uy,
                                                   c->p.coupled);
  c->uo = 0;
  c->parity = 0;
  c->steps = 0;
  c->inited = 1;
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
      hipMemsetAsync(p, 0, c->n * sizeof(double), c->stream);
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
int state_impl(lbm2p_ctx* c, double* f, double* g, double* u, int set) {
  const KParams<T> K = kparams<T>(c);
  if (f) k_state<T><<<blocks1d(c->n), 256, 0, c->stream>>>(K, (T*)c->Af, f, c->parity, set);
  if (g && c->p.coupled)
    k_state<T><<<blocks1d(c->n), 256, 0, c->stream>>>(K, (T*)c->Ag, g, c->parity, set);
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

}  // namespace

// ======================================================================= ABI
extern "C" {

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
  } else {
    c->Ag = c->praw = c->jx = c->jy = c->pt = nullptr;
  }
  c->red = (double*)(((uintptr_t)q + 255) & ~(uintptr_t)255);
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
  *out = c;
  return LBM2P_OK;
}

void lbm2p_destroy(lbm2p_ctx* c) {
  if (!c) return;
  for (auto e : c->ev0) hipEventDestroy(e);
  for (auto e : c->ev1) hipEventDestroy(e);
  delete c;
}

int lbm2p_init_fields(lbm2p_ctx* c, const double* phi0, const double* ux0, const double* uy0,
                      const double* p0) {
  if (!c || !phi0) return LBM2P_EINVAL;
  return c->prec ? init_impl<float>(c, phi0, ux0, uy0, p0)
                 : init_impl<double>(c, phi0, ux0, uy0, p0);
}

int lbm2p_step(lbm2p_ctx* c, int32_t n) {
  if (!c || n < 0) return LBM2P_EINVAL;
  if (!c->inited) return LBM2P_ESTATE;
  return c->prec ? step_impl<float>(c, n) : step_impl<double>(c, n);
}

int lbm2p_moments(lbm2p_ctx* c, double* phi, double* ux, double* uy, double* p, double* rho) {
  if (!c) return LBM2P_EINVAL;
  if (!c->inited) return LBM2P_ESTATE;
  return c->prec ? moments_impl<float>(c, phi, ux, uy, p, rho)
                 : moments_impl<double>(c, phi, ux, uy, p, rho);
}

int lbm2p_fields(lbm2p_ctx* c, int32_t which, double* out) {
  if (!c || !out || which < 0 || which > 7) return LBM2P_EINVAL;
  if (!c->inited || c->steps == 0) return LBM2P_ESTATE;
  const int kl = (c->p.K - 1) & 1;
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
  c->prec ? to_f64<float>(c, src, out) : to_f64<double>(c, src, out);
  return hipGetLastError() == hipSuccess ? LBM2P_OK : LBM2P_EHIP;
}

int lbm2p_volume(lbm2p_ctx* c, double out[6]) {
  if (!c || !out) return LBM2P_EINVAL;
  if (!c->inited) return LBM2P_ESTATE;
  return c->prec ? volume_impl<float>(c, out) : volume_impl<double>(c, out);
}

int lbm2p_get_state(lbm2p_ctx* c, double* f, double* g, double* u) {
  if (!c) return LBM2P_EINVAL;
  if (!c->inited) return LBM2P_ESTATE;
  return c->prec ? state_impl<float>(c, f, g, u, 0) : state_impl<double>(c, f, g, u, 0);
}

int lbm2p_set_state(lbm2p_ctx* c, const double* f, const double* g, const double* u) {
  if (!c || !f || !u || (c->p.coupled && !g)) return LBM2P_EINVAL;
  if (!c->inited) return LBM2P_ESTATE;
  return c->prec ? state_impl<float>(c, (double*)f, (double*)g, (double*)u, 1)
                 : state_impl<double>(c, (double*)f, (double*)g, (double*)u, 1);
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
