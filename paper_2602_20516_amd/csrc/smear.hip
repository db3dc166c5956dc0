// Stout-smeared fermion action: S = S_G(U0) + S_f(U_n), U_n = stout^n(U0).
// Forward: U_n through ping-pong buffers; the solver and the fermion adjoint
// run on U_n.  Backward: for l = n..1, U_{l-1} is recomputed from U0 (no
// level is stored; O(n^2) smearing passes for O(1) extra fields), then one
// level's adjoint maps the gradient from U_l to U_{l-1}.
#include <utility>

#include "lgt_ctx.h"

using namespace lgt;

namespace {
// gauge scratch: 0/1 smearing intermediates, 2 Lambda, 3 partial gradient,
// 4 gradient ping-pong, 5 fermion gradient, 6 thin links (ABI), 7 recomputed
// level, 8 smeared output (ABI)
enum { kPing = 0, kPong = 1, kLam = 2, kGpart = 3, kGtmp = 4, kGf = 5, kRecomp = 7 };
}  // namespace

double2* lgt_ctx::g64(int i) {
  if ((int)gauge64.size() <= i) gauge64.resize(i + 1, nullptr);
  if (!gauge64[i]) LGT_HIP(hipMalloc(&gauge64[i], (size_t)72 * vh * sizeof(double2)));
  return gauge64[i];
}

// dst must not be one of the intermediate buffers 0/1.
void lgt_ctx::smear(const double2* U0, int n, double rho, double2* dst) {
  const int ncx = 72 * vh;
  if (n == 0) {
    LGT_HIP(launch_copy64(ncx, U0, dst, stream));
    return;
  }
  const double2* cur = U0;
  for (int l = 1; l <= n; ++l) {
    double2* out = l == n ? dst : g64(l % 2 ? kPing : kPong);
    LGT_HIP(launch_stout_fwd(g, cur, out, rho, stream));
    cur = out;
  }
}

void lgt_ctx::stout_backprop(const double2* U0, int n, double rho, double2* G) {
  double2* gin = G;
  double2* gout = g64(kGtmp);
  for (int l = n; l >= 1; --l) {
    const double2* ul = U0;
    if (l - 1 > 0) {
      double2* buf = g64(kRecomp);
      smear(U0, l - 1, rho, buf);
      ul = buf;
    }
    LGT_HIP(launch_stout_adjoint(g, ul, gin, rho, g64(kLam), g64(kGpart), gout, stream));
    std::swap(gin, gout);
  }
  if (gin != G) LGT_HIP(launch_copy64(72 * vh, gin, G, stream));
}

SolveStats lgt_ctx::smeared_force(const double2* U0, const double2* phi, double beta, double rho, int n,
                                  const SolverOpts& o, int mode, double dt, void* out, int layout, double* S_F) {
  // operator links: U64 = stout^n(U0) (+ FP32 copy for the mixed solver)
  smear(U0, n, rho, U64);
  if (o.precision != LGT_FP64) {
    ensure_u32();
    LGT_HIP(launch_convert_64_32(72 * vh, U64, U32, stream));
  }
  SolveStats st = solve_ddagd(phi, f64(kX), f64(kY), o);
  if (S_F) *S_F = action_fermion(phi, f64(kX), f64(kY));
  double2* G = g64(kGf);
  LGT_HIP(launch_bilinear_force(g, U64, f64(kY), f64(kX), kappa, -2.0, LGT_OUT_GRAD, 0.0, G, kPacked, stream));
  stout_backprop(U0, n, rho, G);
  // gauge part on the thin links (overwrites out, or subtracts dt F_G in momentum mode)
  LGT_HIP(launch_gauge_force(g, U0, beta, mode, dt, out, layout, stream));
  const int acc = mode == LGT_OUT_FORCE ? 0 : (mode == LGT_OUT_GRAD ? 1 : 2);
  LGT_HIP(launch_grad_to_force(g, U0, G, acc, dt, out, layout, stream));
  return st;
}
