// Solver driver: A X = phi with A = D^dag D (eq. S3.6), X = chi, Y = D X.
//
// Method (the paper names conjugate gradient only as an example; the solve is
// not differentiated): two even/odd Schur-complement solves,
//     D^dag Y = phi,   D X = Y,
// each written as M z = b with M = D or D^dag = 1 - kappa H^(dag):
//     b'_o = b_o + kappa H_oe b_e,     Mhat = 1 - kappa^2 H_oe H_eo  (odd sites),
//     CG on Mhat^dag Mhat z_o = Mhat^dag b'_o   (zero initial guess),
//     z_e = b_e + kappa H_eo z_o,
// then Y is recomputed as D X and the FP64 residual phi - D^dag D X checked;
// FP64 defect-correction passes follow until it meets the tolerance.
//
// The CG iteration is five stream-ordered kernels (four hops and the step
// kernel) whose scalars (alpha, beta, |r|^2, the stop code) stay on the
// device; the host keeps a few iterations queued ahead of the GPU and learns
// of a stop from the mailbox the step kernel posts to (see drive).  Once
// stopped, the iterations still queued return immediately.
//
// Mixed precision: the same CG in FP32 (FP32 links and vectors) with
// reliable updates: whenever the FP32 residual has dropped by reliable_delta
// since the last update (tested on the device every iteration), the FP32
// solution is folded into the FP64 one and the residual recomputed in FP64,
// by kernels the host enqueues without waiting (see cg_normal_mixed).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "lgt_ctx.h"

using namespace lgt;

double2* lgt_ctx::f64(int i) {
  if ((int)full64.size() <= i) full64.resize(i + 1, nullptr);
  if (!full64[i]) {
    LGT_HIP(hipMalloc(&full64[i], full_elems() * sizeof(double2)));
    LGT_HIP(hipMemsetAsync(full64[i], 0, full_elems() * sizeof(double2), stream));
  }
  return full64[i];
}

float2* lgt_ctx::h32(int i) {
  if ((int)half32.size() <= i) half32.resize(i + 1, nullptr);
  if (!half32[i]) {
    LGT_HIP(hipMalloc(&half32[i], half_elems() * sizeof(float2)));
    LGT_HIP(hipMemsetAsync(half32[i], 0, half_elems() * sizeof(float2), stream));
  }
  return half32[i];
}

void lgt_ctx::ensure_u32() {
  if (!U32) LGT_HIP(hipMalloc(&U32, (size_t)72 * vh * sizeof(float2)));
}

void lgt_ctx::compress_links() {
  if (!U32c) LGT_HIP(hipMalloc(&U32c, (size_t)48 * vh * sizeof(float2)));
  LGT_HIP(hipMemsetAsync(flags + 1, 0, sizeof(int), stream));
  LGT_HIP(launch_compress_links(g, U32, U32c, flags + 1, stream));
  LGT_HIP(hipMemcpyAsync(host_flags + 1, flags + 1, sizeof(int), hipMemcpyDeviceToHost, stream));
}

void lgt_ctx::compress_links64() {
  if (!U64c) LGT_HIP(hipMalloc(&U64c, (size_t)48 * vh * sizeof(double2)));
  LGT_HIP(hipMemsetAsync(flags + 2, 0, sizeof(int), stream));
  LGT_HIP(launch_compress_links(g, U64, U64c, flags + 2, stream));
  LGT_HIP(hipMemcpyAsync(host_flags + 2, flags + 2, sizeof(int), hipMemcpyDeviceToHost, stream));
}

void lgt_ctx::ensure_p64() {
  if (!P64) LGT_HIP(hipMalloc(&P64, (size_t)72 * vh * sizeof(double2)));
}

void lgt_ctx::sync() { LGT_HIP(hipStreamSynchronize(stream)); }

void lgt_ctx::read_results(int n) {
  LGT_HIP(hipMemcpyAsync(host_result, result, n * sizeof(double), hipMemcpyDeviceToHost, stream));
  sync();
}


void lgt_ctx::dslash_full(const double2* in, double2* out, double k, bool dag) {
  const size_t h = half_elems();
  HopIn<double> hin{U64, in, in + h};
  if (dag)
    LGT_HIP((launch_hop_axpy<double, true>(g, -1, hin, out, out + h, in, in + h, -k, stream)));
  else
    LGT_HIP((launch_hop_axpy<double, false>(g, -1, hin, out, out + h, in, in + h, -k, stream)));
}

template <typename R, bool DAG>
static void hop(const Geom& g, int p_out, const R2<R>* gauge, const R2<R>* in, R2<R>* out, const R2<R>* self,
                double coef, hipStream_t s, SolverState* guard = nullptr) {
  HopIn<R> hin{gauge, in, in};
  LGT_HIP((launch_hop_axpy<R, DAG>(g, p_out, hin, out, out, self, self, coef, s, guard)));
}

// out_o = Mhat^dag Mhat x_o in FP64 (4 hops), using kW0 even half as scratch.
void lgt_ctx::apply_mhat_dag_mhat64(bool dag, const double2* x, double2* out) {
  const double k2 = -kappa * kappa;
  double2* t = f64(kW0);            // even half
  double2* w = f64(kW4) + half_elems();  // odd half (not used by the mixed CG)
  if (!dag) {
    hop<double, false>(g, 0, U64, x, t, nullptr, 1.0, stream);
    hop<double, false>(g, 1, U64, t, w, x, k2, stream);
    hop<double, true>(g, 0, U64, w, t, nullptr, 1.0, stream);
    hop<double, true>(g, 1, U64, t, out, w, k2, stream);
  } else {
    hop<double, true>(g, 0, U64, x, t, nullptr, 1.0, stream);
    hop<double, true>(g, 1, U64, t, w, x, k2, stream);
    hop<double, false>(g, 0, U64, w, t, nullptr, 1.0, stream);
    hop<double, false>(g, 1, U64, t, out, w, k2, stream);
  }
}

// Largest half volume on which the CG step is folded into the first hop:
// there the iteration is bound by its launches (16^4: 5.96 -> 5.35 ms per
// mixed force call, FP64 8.48 -> 7.95 ms); on larger lattices every block of
// the first hop re-reading all the |r|^2 partials and the extra t, p traffic
// cost more than the launch saved (24^3x48: 71 -> 81 ms).
constexpr int kFuseStepMaxVh = 65536;

// One CG iteration on Mhat^dag Mhat.  t, w, p stored as T; x, r as R2<R>.
// FP64 and FP32 storage on small lattices: four hop launches, the first of
// which also does the previous iteration's step (scalars, stop test,
// p = r + beta p; see EpiStep), except in a fresh iteration (the first of a
// solve and the first after a reliable update, where p has just been set):
// there the first hop is a plain t = H p.  t keeps H p for the next
// iteration's step, so the third hop writes t2.  Otherwise: the four hops
// and a separate step kernel.
template <typename R, typename T, bool DAG>
static void cg_iteration(const Geom& g, const R2<R>* gauge, double kappa, T* t, T* t2, T* w, R2<R>* x, R2<R>* r,
                         T* p, SolverState* st, Reduce red, hipStream_t s, int n, bool fresh, int nk = 9) {
  const double k2 = -kappa * kappa;
  constexpr bool kFused = std::is_same<T, R2<R>>::value;
  const bool fuse = kFused && g.vh <= kFuseStepMaxVh;
  if (fuse && !fresh) {
    if constexpr (kFused) LGT_HIP((launch_hop_step<R, DAG>(g, gauge, nk, t, p, r, st, red, s)));
  } else {
    LGT_HIP((launch_hop_axpy<R, DAG, T>(g, 0, HopIn<R, T>{gauge, p, p, nk}, t, t, nullptr, nullptr, 1.0, s, st)));
  }
  LGT_HIP((launch_hop_schur_norm<R, T, DAG>(g, HopIn<R, T>{gauge, t, t, nk}, w, p, k2, st, red, s)));
  // block 0 also forms alpha from the |w|^2 partials
  LGT_HIP((launch_hop_axpy<R, !DAG, T>(g, 0, HopIn<R, T>{gauge, w, w, nk}, t2, t2, nullptr, nullptr, 1.0, s, st,
                                         red.partials)));
  // x += alpha p: in the fourth hop's epilogue on the fused path, else in the
  // step kernel, which reads p anyway
  LGT_HIP((launch_hop_schur_cg<R, T, !DAG>(g, HopIn<R, T>{gauge, t2, t2, nk}, w, fuse ? x : nullptr, r, p, k2, st,
                                           red, s)));
  if (!fuse) LGT_HIP((launch_cg_step<R, T>(n, r, p, st, red, hop_blocks(g, 1), s, x)));
}

// CG on Mhat^dag Mhat z = rhs (odd half fields), FP64.  Returns the state's done code.
int lgt_ctx::cg_normal64(bool dag, double2* z, const double2* rhs, double tol, int max_iter, SolveStats& stt) {
  const int n = (int)half_elems();
  double2* t = f64(kW0);
  double2* t2 = f64(kW1);  // even half (the odd half holds rhs)
  double2* r = f64(kW2) + half_elems();
  double2* p = f64(kW3) + half_elems();
  double2* w = f64(kW4) + half_elems();
  // the hops read two-row links when the links are SU(3) to FP64 rounding
  // (the third row rebuilt in registers: a quarter less traffic per hop)
  compress_links64();
  sync();
  const bool c12 = host_flags[2] == 0;
  const double2* links = c12 ? U64c : U64;
  const int nk = c12 ? 6 : 9;
  LGT_HIP(launch_cg_init<double>(n, rhs, r, p, z, state, red(), tol, max_iter, stream));
  bool fresh = true;
  for (int iter0 = 0;;) {
    drive(iter0, [&] {
      if (dag) cg_iteration<double, double2, true>(g, links, kappa, t, t2, w, z, r, p, state, red(), stream, n, fresh, nk);
      else cg_iteration<double, double2, false>(g, links, kappa, t, t2, w, z, r, p, state, red(), stream, n, fresh, nk);
      fresh = false;
    });
    LGT_HIP(hipMemcpyAsync(host_state, state, sizeof(SolverState), hipMemcpyDeviceToHost, stream));
    sync();
    const SolverState s = *host_state;
    if (s.done != kDoneRunning) {
      stt.iters += s.iter;
      return s.done;
    }
    iter0 = s.iter;
  }
}

// Mixed-precision CG with reliable updates.  z, rhs: FP64 odd halves.
// The FP32 recursion always works on the current FP64 residual scaled to
// unit norm (sigma = 1/||r||), so its values stay well inside the FP32 range
// whatever the absolute size of the system (defect-correction passes solve
// for residuals many orders below ||phi||).  At every reliable update the
// FP32 solution, in units of 1/sigma, is folded into the FP64 one, the FP64
// residual is recomputed, and the search direction is rescaled to the new
// units.  The recursion stops itself on the device, in the iteration where
// |r|^2 first falls below delta^2 times its largest value since the last
// update (or below the target), and posts the stop to the host (see drive).  Letting it run on until the
// host looks would let a fast-converging recursion go orders of magnitude
// past the accuracy FP32 can hold, after which the kept direction no longer
// matches the true residual and CG diverges.  The stopping iteration skips
// its direction update; the update forms it from the true residual,
// p = r_new + beta p_old (beta of that iteration, p_old rescaled to the new
// units), which keeps the direction consistent even when the recursion's
// own residual has drifted (BF16-stored intermediates drift by ~2^-9 per
// iteration).  After a breakdown the direction is restarted, p = r_new.
// T: storage of the recursion's spinors t, w, p (float2, or Bf16c for the
// BF16-storage variant); x and r stay FP32.
template <typename T>
int lgt_ctx::cg_normal_mixed(bool dag, double2* z, const double2* rhs, double tol, int max_iter, double delta,
                             SolveStats& stt) {
  const int n = (int)half_elems();
  ensure_u32();
  T* ts = reinterpret_cast<T*>(h32(0));  // h32 buffers hold float2; Bf16c uses half of each
  T* ws = reinterpret_cast<T*>(h32(1));
  float2* xs = h32(2);
  float2* rs = h32(3);
  T* ps = reinterpret_cast<T*>(h32(4));
  T* ts2 = std::is_same<T, float2>::value ? reinterpret_cast<T*>(h32(5)) : ts;
  double2* r64 = f64(kW2) + half_elems();
  LGT_HIP(launch_zero64(n, z, stream));
  compress_links();
  LGT_HIP(launch_norm_dot(n, rhs, nullptr, red(), 0, stream));
  read_results(2);
  // the inner hops read two-row links when the links are SU(3) (the third
  // row is rebuilt in registers: a third less link traffic); the FP64
  // residuals of the reliable updates always use the full FP64 links
  const bool c12 = host_flags[1] == 0;
  const float2* links = c12 ? U32c : U32;
  const int nk = c12 ? 6 : 9;
  const double bb = host_result[0];
  if (!std::isfinite(bb)) return kDoneBreakdown;
  if (bb == 0.0) return kDoneConverged;
  const double rr_target = tol * tol * bb;
  double sigma = 1.0 / std::sqrt(bb);
  LGT_HIP(launch_zero32(n, xs, stream));
  LGT_HIP(launch_rescale_residual(n, rhs, sigma, rs, ps, 1, 0.0, stream));
  SolverState s{};
  s.rr = 1.0;
  s.rr0 = 1.0;
  s.rr_max = 1.0;
  s.rr_stop = rr_target * sigma * sigma;
  s.delta2 = delta * delta;
  s.sigma = sigma;
  s.rr_target = rr_target;
  s.max_iter = max_iter;
  s.done = kDoneRunning;
  *host_state = s;
  LGT_HIP(hipMemcpyAsync(state, host_state, sizeof(SolverState), hipMemcpyHostToDevice, stream));
  // The recursion stops itself on the device for each reliable update; the
  // host answers by enqueueing the update (fold, FP64 residual, decision,
  // rescale) without waiting for the device, and the decision kernel either
  // resumes the recursion or ends the solve.
  unsigned min_epoch = 0;
  int iter0 = 0;
  bool fresh = true;  // p has just been set: the next iteration's first hop is a plain t = H p
  for (;;) {
    const unsigned long long v = drive(iter0, [&] {
      if (dag) cg_iteration<float, T, true>(g, links, kappa, ts, ts2, ws, xs, rs, ps, state, red(), stream, n, fresh, nk);
      else cg_iteration<float, T, false>(g, links, kappa, ts, ts2, ws, xs, rs, ps, state, red(), stream, n, fresh, nk);
      fresh = false;
    }, min_epoch, false);
    unsigned act = (unsigned)(v >> 32);
    int dev_iter = (int)(unsigned)v;
    if (!act || (act >> 8) < min_epoch) {  // nothing posted for long: read the state
      LGT_HIP(hipMemcpyAsync(host_state, state, sizeof(SolverState), hipMemcpyDeviceToHost, stream));
      sync();
      s = *host_state;
      dev_iter = s.iter;
      if (s.done == kDoneRunning) {
        iter0 = s.iter;
        continue;
      }
      act = action_word(s.epoch, s.done == kDoneUpdateHeld ? kDoneUpdate : s.done);
    }
    const int code = (int)(act & 0xffu);
    if (code == kDoneUpdate || code == kDoneUpdateHeld || code == kDoneBreakdown) {
      LGT_HIP(launch_mixed_fold(n, xs, z, state, stream));
      apply_mhat_dag_mhat64(dag, z, r64);          // r64 = A z
      LGT_HIP(launch_xmy64(n, rhs, r64, stream));  // r64 = rhs - A z
      LGT_HIP(launch_reliable_decide(n, r64, red(), state, stream));
      LGT_HIP(launch_rescale_residual_dev<T>(n, r64, rs, ps, state, stream));
      min_epoch = (act >> 8) + 1;
      iter0 = dev_iter;
      fresh = true;
      continue;
    }
    if (code == kDoneMaxIter) LGT_HIP(launch_mixed_fold(n, xs, z, state, stream));
    LGT_HIP(hipMemcpyAsync(host_state, state, sizeof(SolverState), hipMemcpyDeviceToHost, stream));
    sync();
    s = *host_state;
    stt.iters += s.iter;
    stt.reliable += s.nupd;
    if (code == kDoneConverged) return kDoneConverged;
    if (code == kDoneMaxIter) return kDoneMaxIter;
    return kDoneBreakdown;
  }
}

void lgt_ctx::solve_M(bool dag, double2* z, const double2* b, double tol, int max_iter, int precision,
                      double delta, SolveStats& stt) {
  const size_t h = half_elems();
  const double2* be = b;
  const double2* bo = b + h;
  double2* bp = f64(kW0) + h;    // b'_o
  double2* te = f64(kW0);        // even scratch
  double2* rhs = f64(kW1) + h;   // Mhat^dag b'_o
  const double k = kappa;
  if (dag) {
    hop<double, true>(g, 1, U64, be, bp, bo, k, stream);
    hop<double, false>(g, 0, U64, bp, te, nullptr, 1.0, stream);
    hop<double, false>(g, 1, U64, te, rhs, bp, -k * k, stream);
  } else {
    hop<double, false>(g, 1, U64, be, bp, bo, k, stream);
    hop<double, true>(g, 0, U64, bp, te, nullptr, 1.0, stream);
    hop<double, true>(g, 1, U64, te, rhs, bp, -k * k, stream);
  }
  double2* zo = z + h;
  const int code = precision == LGT_MIXED_FP32   ? cg_normal_mixed<float2>(dag, zo, rhs, tol, max_iter, delta, stt)
                   : precision == LGT_MIXED_BF16 ? cg_normal_mixed<Bf16c>(dag, zo, rhs, tol, max_iter, delta, stt)
                                                 : cg_normal64(dag, zo, rhs, tol, max_iter, stt);
  if (code == kDoneBreakdown) throw Error(LGT_ERR_NONFINITE, "CG breakdown (non-finite or zero curvature)");
  if (code == kDoneMaxIter) stt.converged = false;
  if (dag) hop<double, true>(g, 0, U64, zo, z, be, k, stream);
  else hop<double, false>(g, 0, U64, zo, z, be, k, stream);
}

SolveStats lgt_ctx::solve_ddagd(const double2* phi, double2* X, double2* Y, const SolverOpts& o) {
  SolveStats st;
  const int nf = (int)full_elems();
  LGT_HIP(launch_norm_dot(nf, phi, nullptr, red(), 0, stream));
  read_results(1);
  const double pp = host_result[0];
  if (!std::isfinite(pp)) throw Error(LGT_ERR_NONFINITE, "phi holds NaN or Inf");
  if (pp == 0.0) {
    LGT_HIP(launch_zero64(nf, X, stream));
    LGT_HIP(launch_zero64(nf, Y, stream));
    st.true_res = 0.0;
    return st;
  }
  // inner tolerance: the two Schur solves and D^dag D compound their
  // residuals, so each aims a little below the requested true residual
  const double tol_in = o.tol * (o.first_pass > 0.0 ? o.first_pass : 0.25);
  solve_M(true, Y, phi, tol_in, o.max_iter, o.precision, o.delta, st);
  solve_M(false, X, Y, tol_in, o.max_iter, o.precision, o.delta, st);
  double2* r = f64(kRes);
  HopIn<double> hin{U64, nullptr, nullptr};
  const size_t h = half_elems();
  double tol_used = tol_in, res_start = 1.0;  // the last pass's CG tolerance and starting residual
  for (int pass = 0;; ++pass) {
    dslash_full(X, Y, kappa, false);
    hin.in_even = Y;
    hin.in_odd = Y + h;
    LGT_HIP(launch_hop_residual<true>(g, hin, Y, phi, r, -kappa, red(), 0, stream));
    read_results(1);
    st.true_res = std::sqrt(host_result[0] / pp);
    if (!std::isfinite(st.true_res)) throw Error(LGT_ERR_NONFINITE, "non-finite residual");
    if (st.true_res <= o.tol || !st.converged || pass >= 4) break;
    // defect correction: D^dag D e = r, X += e.  r only has to shrink by
    // about tol / true_res, not by tol (a pass that missed the target by 2x
    // needs a few iterations, not a full solve that would overshoot to
    // ~tol^2); the CG tolerance of the pass also divides out the
    // magnification the last pass showed (correction_tol)
    const double tol_corr = correction_tol(o.tol, st.true_res, tol_used, res_start);
    tol_used = tol_corr;
    res_start = st.true_res;
    double2* ytmp = f64(kYtmp);
    double2* e = f64(kE);
    solve_M(true, ytmp, r, tol_corr, o.max_iter, o.precision, o.delta, st);
    solve_M(false, e, ytmp, tol_corr, o.max_iter, o.precision, o.delta, st);
    LGT_HIP(launch_axpy64(nf, 1.0, e, X, stream));
    ++st.corrections;
  }
  if (st.true_res > o.tol) st.converged = false;
  return st;
}

double lgt_ctx::action_fermion(const double2* phi, const double2* X, const double2* Y) {
  const int nf = (int)full_elems();
  LGT_HIP(launch_norm_dot(nf, X, phi, red(), 0, stream));
  LGT_HIP(launch_norm_dot(nf, Y, nullptr, red(), 2, stream));
  read_results(4);
  return 2.0 * host_result[1] - host_result[2];
}

// Even/odd-preconditioned action S_eo = phi_o^dag (Mhat^dag Mhat)^-1 phi_o,
// Mhat = 1 - kappa^2 H_oe H_eo (det D = det Mhat): one Schur CGNR solve to
// the FP64 true residual ||phi_o - Mhat^dag Mhat X_o|| <= tol ||phi_o||
// (defect correction), then the fields of its force (the derivative of
// -2 Re[Y_o^dag dMhat X_o] written as a bilinear of the full operator):
//   X = (H_eo X_o on even sites, X_o on odd),  A = (H_oe^dag Y_o, Y_o),
// Y_o = Mhat X_o, so that dS_eo = -2 kappa d Re[A^dag D X].
// phi, X, A: packed full fields; only the odd half of phi is read.
SolveStats lgt_ctx::solve_eo(const double2* phi, double2* X, double2* A, const SolverOpts& o) {
  SolveStats st;
  const size_t h = half_elems();
  const int n = (int)h;
  const double2* phio = phi + h;
  double2* xo = X + h;
  LGT_HIP(launch_norm_dot(n, phio, nullptr, red(), 0, stream));
  read_results(1);
  const double pp = host_result[0];
  if (!std::isfinite(pp)) throw Error(LGT_ERR_NONFINITE, "phi holds NaN or Inf");
  if (pp == 0.0) {
    LGT_HIP(launch_zero64(2 * n, X, stream));
    LGT_HIP(launch_zero64(2 * n, A, stream));
    st.true_res = 0.0;
    return st;
  }
  const double tol_in = o.tol * (o.first_pass > 0.0 ? o.first_pass : 0.5);
  auto schur_solve = [&](double2* z, const double2* rhs, double t) {
    const int code = o.precision == LGT_MIXED_FP32   ? cg_normal_mixed<float2>(false, z, rhs, t, o.max_iter,
                                                                             o.delta, st)
                     : o.precision == LGT_MIXED_BF16 ? cg_normal_mixed<Bf16c>(false, z, rhs, t, o.max_iter,
                                                                            o.delta, st)
                                                     : cg_normal64(false, z, rhs, t, o.max_iter, st);
    if (code == kDoneBreakdown) throw Error(LGT_ERR_NONFINITE, "CG breakdown (non-finite or zero curvature)");
    if (code == kDoneMaxIter) st.converged = false;
  };
  schur_solve(xo, phio, tol_in);
  double2* r = f64(kRes) + h;
  double2* e = f64(kE) + h;
  double tol_used = tol_in, res_start = 1.0;
  for (int pass = 0;; ++pass) {
    apply_mhat_dag_mhat64(false, xo, r);
    LGT_HIP(launch_xmy64(n, phio, r, stream));  // r = phi_o - Mhat^dag Mhat X_o
    LGT_HIP(launch_norm_dot(n, r, nullptr, red(), 0, stream));
    read_results(1);
    st.true_res = std::sqrt(host_result[0] / pp);
    if (!std::isfinite(st.true_res)) throw Error(LGT_ERR_NONFINITE, "non-finite residual");
    if (st.true_res <= o.tol || !st.converged || pass >= 4) break;
    // a correction only has to shrink r by about tol / true_res (as in solve_ddagd)
    const double tol_corr = correction_tol(o.tol, st.true_res, tol_used, res_start);
    tol_used = tol_corr;
    res_start = st.true_res;
    schur_solve(e, r, tol_corr);
    LGT_HIP(launch_axpy64(n, 1.0, e, xo, stream));
    ++st.corrections;
  }
  if (st.true_res > o.tol) st.converged = false;
  const double k2 = -kappa * kappa;
  hop<double, false>(g, 0, U64, xo, X, nullptr, 1.0, stream);     // X_e = H_eo X_o
  hop<double, false>(g, 1, U64, X, A + h, xo, k2, stream);        // Y_o = X_o - kappa^2 H_oe X_e
  hop<double, true>(g, 0, U64, A + h, A, nullptr, 1.0, stream);   // A_e = H_oe^dag Y_o
  return st;
}

// S_eo = 2 Re phi_o^dag X_o - ||Y_o||^2 (equal to phi_o^dag X_o at the
// solution, second order in the solver error); fields as solve_eo.
double lgt_ctx::action_eo(const double2* phi, const double2* X, const double2* A) {
  const size_t h = half_elems();
  const int n = (int)h;
  LGT_HIP(launch_norm_dot(n, X + h, phi + h, red(), 0, stream));
  LGT_HIP(launch_norm_dot(n, A + h, nullptr, red(), 2, stream));
  read_results(4);
  return 2.0 * host_result[1] - host_result[2];
}
