// float instantiation of the lattice update, compiled with contraction into fused multiply-adds and fast
// single-precision division (the FP32 mode is held to error bounds, not to
// bitwise agreement).
#include "lbm2p_adjoint_impl.h"

namespace lbm2p {

int init_f32(lbm2p_ctx* c, const double* phi0, const double* ux0, const double* uy0,
              const double* p0) {
  return init_impl<float>(c, phi0, ux0, uy0, p0);
}
int step_f32(lbm2p_ctx* c, int n) { return step_impl<float>(c, n); }
int moments_f32(lbm2p_ctx* c, double* phi, double* ux, double* uy, double* p, double* rho) {
  return moments_impl<float>(c, phi, ux, uy, p, rho);
}
int volume_f32(lbm2p_ctx* c, double* out) { return volume_impl<float>(c, out); }
int bubble_f32(lbm2p_ctx* c, double* out) { return bubble_impl<float>(c, out); }
int pjump_f32(lbm2p_ctx* c, double* out) { return pjump_impl<float>(c, out); }
int resid_f32(lbm2p_ctx* c, double* out) { return resid_impl<float>(c, out); }
int state_f32(lbm2p_ctx* c, double* f, double* g, double* u, int set) {
  return state_impl<float>(c, f, g, u, set);
}
int setvel_f32(lbm2p_ctx* c, const double* ux, const double* uy) {
  return setvel_impl<float>(c, ux, uy);
}
int to_f64_f32(lbm2p_ctx* c, const void* src, double* dst) {
  to_f64<float>(c, src, dst);
  return hipGetLastError() == hipSuccess ? LBM2P_OK : LBM2P_EHIP;
}

int record_f32(lbm2p_ctx* c, int nsteps, int k) { return record_impl<float>(c, nsteps, k); }
int adjoint_f32(lbm2p_ctx* c, lbm2p_adjoint_io* io) { return adjoint_impl<float>(c, io); }

}  // namespace lbm2p
