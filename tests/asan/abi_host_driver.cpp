// Host-side driver of the C ABI for the AddressSanitizer build: every check that
// runs without a GPU (parameter validation, workspace sizing, context set-up
// with the compact filter's host tables, call-order and argument errors).
// Exits non-zero on a wrong return code; the sanitizer aborts on a memory error.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "lbm2p.h"

static int fails = 0;
#define EXPECT(expr, code)                                                       \
  do {                                                                           \
    const int r_ = (expr);                                                       \
    if (r_ != (code)) {                                                          \
      std::fprintf(stderr, "%s:%d %s -> %d, expected %d\n", __FILE__, __LINE__,  \
                   #expr, r_, (code));                                           \
      ++fails;                                                                   \
    }                                                                            \
  } while (0)

static lbm2p_params base(int nx, int ny) {
  lbm2p_params p;
  std::memset(&p, 0, sizeof p);
  p.nx = nx;
  p.ny = ny;
  p.coupled = 1;
  p.rho1 = 1.0;
  p.rho2 = 1e-3;
  p.mu1 = 0.01;
  p.mu2 = 1e-4;
  p.sigma = 0.01;
  p.W = 4.0;
  p.M = 0.02;
  p.lam = 0.005;
  p.tau_f = 0.5 + std::sqrt(3.0) / 6.0;
  p.filter_n = 11;
  p.compact_n = 5;
  p.K = 2;
  p.filter_a = 0.5;
  p.compact_alpha = 0.45;
  for (int k = 0; k < 9; ++k) p.s_f[k] = p.s_g[k] = 1.0;
  p.eps = 1e-2;
  return p;
}

// create and destroy a context over a host buffer standing in for the
// workspace (context set-up touches no device memory)
static void create_destroy(const lbm2p_params& p) {
  size_t need = 0;
  EXPECT(lbm2p_workspace_bytes(&p, &need), LBM2P_OK);
  std::vector<unsigned char> buf(need + 512);
  void* ws = (void*)(((uintptr_t)buf.data() + 255) / 256 * 256);
  lbm2p_ctx* c = nullptr;
  EXPECT(lbm2p_create(&p, ws, need - 1, nullptr, &c), LBM2P_ENOSPACE);
  EXPECT(lbm2p_create(&p, (char*)ws + 8, need, nullptr, &c), LBM2P_EINVAL);
  EXPECT(lbm2p_create(&p, ws, need, nullptr, &c), LBM2P_OK);
  EXPECT(lbm2p_step(c, 1), LBM2P_ESTATE);
  EXPECT(lbm2p_step(c, -1), LBM2P_EINVAL);
  double out[6];
  EXPECT(lbm2p_volume(c, out), LBM2P_ESTATE);
  EXPECT(lbm2p_bubble(c, out), LBM2P_ESTATE);
  EXPECT(lbm2p_moments(c, nullptr, nullptr, nullptr, nullptr, nullptr), LBM2P_ESTATE);
  EXPECT(lbm2p_track_residual(c, 2), LBM2P_EINVAL);
  EXPECT(lbm2p_record(c, 4, 0, ws, need), LBM2P_EINVAL);
  lbm2p_adjoint_io io;
  std::memset(&io, 0, sizeof io);
  EXPECT(lbm2p_adjoint(c, &io), LBM2P_ESTATE);
  EXPECT(lbm2p_set_velocity(c, (const double*)ws, (const double*)ws),
         p.coupled ? LBM2P_EINVAL : LBM2P_ESTATE);
  EXPECT(lbm2p_profile(c, 7), LBM2P_EINVAL);
  EXPECT(lbm2p_init_fields(c, nullptr, nullptr, nullptr, nullptr), LBM2P_EINVAL);
  EXPECT(lbm2p_fields(c, 0, out), LBM2P_ESTATE);
  EXPECT(lbm2p_fields(c, 8, out), LBM2P_EINVAL);
  EXPECT(lbm2p_get_state(c, nullptr, nullptr, nullptr), LBM2P_ESTATE);
  EXPECT(lbm2p_set_state(c, out, out, out), LBM2P_ESTATE);
  EXPECT(lbm2p_residual(c, out), p.coupled ? LBM2P_ESTATE : LBM2P_EINVAL);
  EXPECT(lbm2p_pressure_jump(c, out), p.coupled ? LBM2P_ESTATE : LBM2P_EINVAL);
  EXPECT(lbm2p_track_residual(c, 1), LBM2P_OK);
  lbm2p_destroy(c);
}

int main() {
  // valid configurations: periodic, walls, CH-only, FP32, every explicit filter,
  // the compact filter at the smallest and the longest lines, the options
  lbm2p_params p = base(64, 48);
  create_destroy(p);
  p.wall_x = p.wall_y = 1;
  create_destroy(p);
  p = base(64, 48);
  p.coupled = 0;
  create_destroy(p);
  p = base(64, 48);
  p.precision = 1;
  create_destroy(p);
  for (int n : {0, 5, 7, 9}) {
    p = base(40, 32);
    p.filter_n = n;
    create_destroy(p);
  }
  for (int n = 1; n <= 5; ++n)
    for (int wall = 0; wall < 2; ++wall) {
      p = base(16, 16);
      p.compact = 1;
      p.compact_n = n;
      p.wall_x = p.wall_y = wall;
      create_destroy(p);
      p = base(7680, 16);
      p.compact = 1;
      p.compact_n = n;
      p.compact_alpha = -0.3;
      p.wall_y = wall;
      create_destroy(p);
    }
  p = base(64, 48);
  p.options = LBM2P_OPT_STRAIN_MOMENTS | LBM2P_OPT_GI_LITERAL;
  create_destroy(p);
  // invalid parameters
  size_t b = 0;
  EXPECT(lbm2p_workspace_bytes(nullptr, &b), LBM2P_EINVAL);
  p = base(15, 16);
  EXPECT(lbm2p_workspace_bytes(&p, &b), LBM2P_EINVAL);
  p = base(64, 48);
  p.tau_f = 0.5;
  EXPECT(lbm2p_workspace_bytes(&p, &b), LBM2P_EINVAL);
  p = base(64, 48);
  p.options = 4;
  EXPECT(lbm2p_workspace_bytes(&p, &b), LBM2P_EINVAL);
  p = base(64, 48);
  p.compact = 1;
  p.nx = 7681;
  EXPECT(lbm2p_workspace_bytes(&p, &b), LBM2P_EINVAL);
  p = base(64, 48);
  p.p_ref = NAN;
  EXPECT(lbm2p_workspace_bytes(&p, &b), LBM2P_EINVAL);
  p = base(64, 48);
  EXPECT(lbm2p_adjoint_workspace_bytes(&p, -1, 4, &b), LBM2P_EINVAL);
  EXPECT(lbm2p_adjoint_workspace_bytes(&p, 100, 8, &b), LBM2P_OK);
  // context-free entry points: argument checks before any device work
  EXPECT(lbm2p_stream_copy(nullptr, nullptr, 0, nullptr), LBM2P_OK);
  EXPECT(lbm2p_stream_copy(nullptr, (void*)256, 16, nullptr), LBM2P_EINVAL);
  EXPECT(lbm2p_volume_noalloc(nullptr, nullptr, nullptr, nullptr, 4, 4, nullptr, nullptr),
         LBM2P_EINVAL);
  EXPECT(lbm2p_volume_noalloc((const double*)256, nullptr, (const double*)256, (const double*)256,
                              1 << 16, 1 << 16, (double*)256, nullptr),
         LBM2P_EINVAL);
  for (int code = -1; code <= 6; ++code)
    if (!lbm2p_strerror(code) || !*lbm2p_strerror(code)) ++fails;
  lbm2p_destroy(nullptr);
  if (fails) std::fprintf(stderr, "%d failures\n", fails);
  else std::printf("abi host driver: ok\n");
  return fails ? 1 : 0;
}
