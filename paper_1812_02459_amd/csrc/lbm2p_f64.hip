// double instantiation of the lattice update, compiled without floating-point contraction: every expression rounds
// as written, like the CPU oracle.
#include <mutex>

#include "lbm2p_adjoint_impl.h"

namespace lbm2p {

int init_f64(lbm2p_ctx* c, const double* phi0, const double* ux0, const double* uy0,
              const double* p0) {
  return init_impl<double>(c, phi0, ux0, uy0, p0);
}
int step_f64(lbm2p_ctx* c, int n) { return step_impl<double>(c, n); }
int moments_f64(lbm2p_ctx* c, double* phi, double* ux, double* uy, double* p, double* rho) {
  return moments_impl<double>(c, phi, ux, uy, p, rho);
}
int volume_f64(lbm2p_ctx* c, double* out) { return volume_impl<double>(c, out); }
int bubble_f64(lbm2p_ctx* c, double* out) { return bubble_impl<double>(c, out); }
int pjump_f64(lbm2p_ctx* c, double* out) { return pjump_impl<double>(c, out); }
int resid_f64(lbm2p_ctx* c, double* out) { return resid_impl<double>(c, out); }
int state_f64(lbm2p_ctx* c, double* f, double* g, double* u, int set) {
  return state_impl<double>(c, f, g, u, set);
}
int setvel_f64(lbm2p_ctx* c, const double* ux, const double* uy) {
  return setvel_impl<double>(c, ux, uy);
}
int to_f64_f64(lbm2p_ctx* c, const void* src, double* dst) {
  to_f64<double>(c, src, dst);
  return hipGetLastError() == hipSuccess ? LBM2P_OK : LBM2P_EHIP;
}

int record_f64(lbm2p_ctx* c, int nsteps, int k) { return record_impl<double>(c, nsteps, k); }
int adjoint_f64(lbm2p_ctx* c, lbm2p_adjoint_io* io) { return adjoint_impl<double>(c, io); }

}  // namespace lbm2p

// ------------------------------------------- diagnostics without allocation
// lbm2p_volume_noalloc keeps its per-workgroup partials in this array (one
// copy per device, alive until the process ends) instead of a context's
// workspace.  Host code never passes the array's name to a kernel (on the host
// it is only a stand-in for the symbol): it uses the device address that
// hipGetSymbolAddress gives, looked up once per device.
namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = 65536;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_BYTES / sizeof(double)];
static_assert(((size_t)lbm2p::RED_BLOCKS + 1) * lbm2p::RED_K * sizeof(double) <=
                  NOALLOC_SCRATCH_BYTES,
              "the reduction partials and results fit in the static scratch");

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_ptr[MAX_DEVICES] = {};

// the current device's copy of the scratch array (nullptr on failure)
double* device_scratch() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    scratch_ptr[dev] = (double*)ptr;
  }
  return scratch_ptr[dev];
}

}  // namespace

namespace lbm2p {

int volume_noalloc_f64(const double* phi, const double* p, const double* ux, const double* uy,
                       long long n, double* out, hipStream_t stream) {
  double* part = device_scratch();
  if (!part) return LBM2P_EHIP;
  // the reduction of lbm2p_volume (same grid, same order): every partial is
  // written before it is read, so nothing left by an earlier call matters
  k_reduce1<double><<<RED_BLOCKS, RED_NT, 0, stream>>>(phi, p, ux, uy, n, part, p ? 1 : 0);
  k_reduce2<<<1, RED_NT, 0, stream>>>(part, RED_BLOCKS, out);
  return hipGetLastError() == hipSuccess ? LBM2P_OK : LBM2P_EHIP;
}

}  // namespace lbm2p
