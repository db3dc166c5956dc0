// Stout-smeared fermion action: S = S_G(U0) + S_f(U_n), U_n = stout^n(U0).
// Forward: U_n through ping-pong buffers, keeping the levels the checkpoint
// schedule asks for; the solver and the fermion adjoint run on U_n.
// Backward: the level adjoints for l = n..1, each fed U_{l-1}, which is a
// kept checkpoint, U0, or recomputed from the nearest available level along
// the schedule (stout_schedule.h).  With every level kept nothing is
// recomputed; with none, O(n^2) smearing passes for O(1) extra fields.
#include <utility>

#include "lgt_ctx.h"

using namespace lgt;

namespace {
// gauge scratch: 0/1 smearing intermediates, 2 Lambda, 3 partial gradient,
// 4 gradient ping-pong, 5 fermion gradient, 6 thin links (ABI), 7 recomputed
// level, 8 smeared output (ABI), 9-11 ABI; checkpoint slots from 16
enum { kPing = 0, kPong = 1, kLam = 2, kGpart = 3, kGtmp = 4, kGf = 5, kRecomp = 7, kSlot0 = 16 };
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

// Checkpoint slots for an n-level reverse pass: the caller's cap, or (cap
// < 0) every level that device memory holds beyond a reserve of 1/8 of it.
int lgt_ctx::stout_slots(int n) {
  int want = std::max(0, n - 1);
  if (stout_slot_cap >= 0) return std::min(want, stout_slot_cap);
  int have = 0;
  while (kSlot0 + have < (int)gauge64.size() && gauge64[kSlot0 + have]) ++have;
  if (want <= have) return want;
  size_t fr = 0, tot = 0;
  LGT_HIP(hipMemGetInfo(&fr, &tot));
  const size_t slot = (size_t)72 * vh * sizeof(double2);
  const size_t reserve = tot / 8;
  const int64_t extra = fr > reserve ? (int64_t)((fr - reserve) / slot) : 0;
  return (int)std::min<int64_t>(want, have + extra);
}

const StoutSchedule& lgt_ctx::stout_plan(int n) {
  const int s = stout_slots(n);
  if (!sched || sched->levels() != n || sched->slots() != std::max(0, std::min(s, n - 1)))
    sched.reset(new StoutSchedule(n, s));
  return *sched;
}

// Forward sweep U0 -> U_n (into dst), keeping the schedule's forward
// checkpoints in slots 0, 1, ...; dst must not be a smearing intermediate.
void lgt_ctx::smear_checkpointed(const double2* U0, int n, double rho, double2* dst, const StoutSchedule& plan) {
  if (n == 0) {
    LGT_HIP(launch_copy64(72 * vh, U0, dst, stream));
    return;
  }
  const std::vector<int> cp = plan.forward_checkpoints();
  size_t j = 0;
  const double2* cur = U0;
  for (int l = 1; l <= n; ++l) {
    double2* out;
    if (l == n) out = dst;
    else if (j < cp.size() && cp[j] == l) out = g64(kSlot0 + (int)j++);
    else out = g64(l % 2 ? kPing : kPong);
    LGT_HIP(launch_stout_fwd(g, cur, out, rho, stream));
    cur = out;
  }
}

namespace {
// The reverse pass over one schedule: level adjoints in the order n..1.
struct Reverse {
  lgt_ctx* c;
  const StoutSchedule& plan;
  double rho;
  double2* gin;
  double2* gout;
  int64_t passes = 0;

  void advance(const double2* src, int m, double2* dst) {  // dst = stout^m(src)
    c->smear(src, m, rho, dst);
    passes += m;
  }
  void adjoint(const double2* below) {  // gradient from U_l to U_{l-1}; below = U_{l-1}
    LGT_HIP(launch_stout_adjoint(c->g, below, gin, rho, c->g64(kLam), c->g64(kGpart), gout, c->stream));
    std::swap(gin, gout);
  }
  // segment [a, b]: U_a in ua, `free` slots from slot index `top` on
  void serve(int a, int b, const double2* ua, int free, int top) {
    const int len = b - a;
    if (len == 1) {
      adjoint(ua);
      return;
    }
    if (free == 0) {
      double2* work = c->g64(kRecomp);
      for (int l = b; l >= a + 2; --l) {
        advance(ua, l - 1 - a, work);
        adjoint(work);
      }
      adjoint(ua);
      return;
    }
    const int m = plan.split_F(len, free);
    double2* slot = c->g64(kSlot0 + top);
    advance(ua, m, slot);
    serve(a + m, b, slot, free - 1, top + 1);
    serve(a, a + m, ua, free, top);
  }
};
}  // namespace

// G (packed, in place): gradient at U_n -> gradient at U0.  forward_done:
// the forward checkpoints of plan are already in their slots (the sweep of
// smear_checkpointed); otherwise the sweep up to the last one runs here.
void lgt_ctx::stout_backprop(const double2* U0, int n, double rho, double2* G, const StoutSchedule& plan,
                             bool forward_done) {
  const std::vector<int> cp = plan.forward_checkpoints();
  if (!forward_done && !cp.empty()) {
    const double2* cur = U0;
    for (size_t j = 0; j < cp.size(); ++j) {
      smear(cur, cp[j] - (j ? cp[j - 1] : 0), rho, g64(kSlot0 + (int)j));
      cur = g64(kSlot0 + (int)j);
    }
  }
  Reverse rv{this, plan, rho, G, g64(kGtmp)};
  const int k = (int)cp.size();
  const int s = plan.slots();
  for (int j = k; j >= 0; --j) {
    const int a = j == 0 ? 0 : cp[j - 1];
    const int b = j == k ? n : cp[j];
    const double2* ua = j == 0 ? U0 : g64(kSlot0 + j - 1);
    rv.serve(a, b, ua, s - j, j);
  }
  if (rv.passes != plan.cost())
    throw Error(LGT_ERR_DEVICE, "internal error: stout reverse pass departed from its schedule");
  if (rv.gin != G) LGT_HIP(launch_copy64(72 * vh, rv.gin, G, stream));
  last_stout_slots = s;
  last_stout_passes = rv.passes;
}

SolveStats lgt_ctx::smeared_force(const double2* U0, const double2* phi, double beta, double rho, int n,
                                  const SolverOpts& o, int mode, double dt, void* out, int layout, double* S_F) {
  // operator links: U64 = stout^n(U0) (+ FP32 copy for the mixed solver)
  const StoutSchedule& plan = stout_plan(n);
  smear_checkpointed(U0, n, rho, U64, plan);
  if (o.precision != LGT_FP64) {
    ensure_u32();
    LGT_HIP(launch_convert_64_32(72 * vh, U64, U32, stream));
  }
  SolveStats st = solve_ddagd(phi, f64(kX), f64(kY), o);
  if (S_F) *S_F = action_fermion(phi, f64(kX), f64(kY));
  double2* G = g64(kGf);
  LGT_HIP(launch_bilinear_force(g, U64, f64(kY), f64(kX), kappa, -2.0, LGT_OUT_GRAD, 0.0, G, kPacked, stream));
  stout_backprop(U0, n, rho, G, plan, true);
  // gauge part on the thin links (overwrites out, or subtracts dt F_G in momentum mode)
  LGT_HIP(launch_gauge_force(g, U0, beta, mode, dt, out, layout, stream));
  const int acc = mode == LGT_OUT_FORCE ? 0 : (mode == LGT_OUT_GRAD ? 1 : 2);
  LGT_HIP(launch_grad_to_force(g, U0, G, acc, dt, out, layout, stream));
  return st;
}
