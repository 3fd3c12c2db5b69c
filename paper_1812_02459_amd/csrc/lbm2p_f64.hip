// double instantiation of the lattice update, compiled without floating-point contraction: every expression rounds
// as written, like the CPU oracle.
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
