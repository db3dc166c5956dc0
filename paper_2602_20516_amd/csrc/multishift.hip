// Multi-shift CG on the even/odd Schur normal operator A = Mhat^dag Mhat
// (Mhat = 1 - kappa^2 H_oe H_eo, odd sites): X_i = (A + sigma_i)^-1 phi_o for
// several shifts sigma_i >= 0 from one Krylov space, the building block of
// rational (RHMC) pseudofermion actions (Sec. I names RHMC among the targets).
//
// The base CG runs on A itself with the usual four hop launches per
// iteration (the base solution is not tracked).  The shifted residuals stay
// collinear with the base one, r_i = zeta_i r, and the shifted iterates
// follow from scalar recurrences (Jegerlehner's shifted CG):
//   zeta_i' = zeta_i zeta_i^- alpha^- / (alpha beta^- (zeta_i^- - zeta_i)
//                                        + zeta_i^- alpha^- (1 + sigma_i alpha))
//   alpha_i = alpha zeta_i' / zeta_i,  beta_i = beta (zeta_i' / zeta_i)^2
//   x_i += alpha_i p_i;  p_i = zeta_i' r + beta_i p_i
// (^-: previous iteration, ': next).  A one-block finalize forms them and
// the stopping test; one vector kernel then updates every shift's x_i, p_i
// and the base direction in a single pass over memory.  Shift i stops
// updating once |zeta_i|^2 |r|^2 <= tol^2 |phi_o|^2; the solve stops when all
// have.  FP64 throughout.
#include <algorithm>
#include <cmath>

#include "lgt_ctx.h"

using namespace lgt;

namespace {

constexpr int kMaxShift = 32;  // two result slots per shift fill the context's 64

struct ShiftState {
  int ns, pad;
  double alpha_prev, beta_prev;
  double rr_stop;
  double sigma[kMaxShift], zeta[kMaxShift], zeta_prev[kMaxShift], alpha_s[kMaxShift], beta_s[kMaxShift];
  int done[kMaxShift], upd[kMaxShift];
};

// rr = sum of the |r|^2 partials of the last hop; beta; the shift
// recurrences (thread i: shift i) and the stop test.
__global__ __launch_bounds__(256) void k_msfinalize(int nblk, const double* __restrict__ partials, SolverState* st,
                                                    ShiftState* ss, Mailbox* mb) {
  const int i = threadIdx.x;
  const int ns = ss->ns;
  if (st->done != kDoneRunning) {  // the iteration was skipped
    if (i < ns) ss->upd[i] = 0;
    if (i == 0) post_progress(mb, st->iter, 1);
    return;
  }
  __shared__ double s_rr;
  double tot[1];
  sum_partials<256, 1>(partials, nblk, tot);
  if (i == 0) s_rr = tot[0];
  __syncthreads();
  const double rr = s_rr;
  const double a = st->alpha;  // alpha of this iteration (formed by the third hop)
  const double b = rr / st->rr;
  int open = 0;
  if (i < ns) {
    ss->upd[i] = 0;
    if (!ss->done[i]) {
      const double z = ss->zeta[i], zp = ss->zeta_prev[i];
      const double zn = z * zp * ss->alpha_prev /
                        (a * ss->beta_prev * (zp - z) + zp * ss->alpha_prev * (1.0 + ss->sigma[i] * a));
      ss->alpha_s[i] = a * zn / z;
      ss->beta_s[i] = b * (zn / z) * (zn / z);
      ss->zeta_prev[i] = z;
      ss->zeta[i] = zn;
      ss->upd[i] = 1;
      if (zn * zn * rr <= ss->rr_stop) ss->done[i] = 1;
      else open = 1;
    }
  }
  const int all = __syncthreads_and(!open);
  if (i != 0) return;
  ss->alpha_prev = a;
  ss->beta_prev = b;
  st->beta = b;
  st->rr = rr;
  st->iter += 1;
  if (!isfinite(rr)) st->done = kDoneBreakdown;
  else if (all) st->done = kDoneConverged;
  else if (st->iter >= st->max_iter) st->done = kDoneMaxIter;
  post_progress(mb, st->iter, st->done != kDoneRunning);
}

// x_i += alpha_i p_i, p_i = zeta_i r + beta_i p_i for the shifts updated this
// iteration; base p = r + beta p while the solve runs.  Shift fields are
// contiguous: x_i = X + i n, p_i = Pn + i n.
__global__ __launch_bounds__(256) void k_msupdate(int n, int ns, const double2* __restrict__ r, double2* __restrict__ p,
                                                  double2* __restrict__ X, double2* __restrict__ Pn,
                                                  const SolverState* st, const ShiftState* ss) {
  const bool base = st->done == kDoneRunning;
  const double beta = st->beta;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const double2 rv = r[i];
    if (base) {
      double2 pv = p[i];
      pv.x = rv.x + beta * pv.x;
      pv.y = rv.y + beta * pv.y;
      p[i] = pv;
    }
    for (int s = 0; s < ns; ++s) {
      if (!ss->upd[s]) continue;
      const size_t o = (size_t)s * n + i;
      const double2 ps = Pn[o];
      double2 xv = X[o];
      const double as = ss->alpha_s[s], bs = ss->beta_s[s], z = ss->zeta[s];
      xv.x += as * ps.x;
      xv.y += as * ps.y;
      X[o] = xv;
      Pn[o] = make_double2(z * rv.x + bs * ps.x, z * rv.y + bs * ps.y);
    }
  }
}

__global__ __launch_bounds__(256) void k_msinit(int n, int ns, const double2* __restrict__ b, double2* __restrict__ r,
                                                double2* __restrict__ p, double2* __restrict__ X,
                                                double2* __restrict__ Pn) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const double2 v = b[i];
    r[i] = v;
    p[i] = v;
    for (int s = 0; s < ns; ++s) {
      X[(size_t)s * n + i] = make_double2(0.0, 0.0);
      Pn[(size_t)s * n + i] = v;
    }
  }
}

}  // namespace

struct MultiShiftWork {
  int ns = 0;
  double2* X = nullptr;   // ns odd halves
  double2* Pn = nullptr;  // ns odd halves
  double2* r = nullptr;   // base residual, base direction, residual scratch: odd halves
  double2* p = nullptr;
  double2* q = nullptr;
  ShiftState* ss = nullptr;
  ShiftState* hss = nullptr;  // pinned
};

void lgt_ctx_free_multishift(lgt_ctx* c) {
  MultiShiftWork* w = c->mshift;
  if (!w) return;
  (void)hipFree(w->X);
  (void)hipFree(w->Pn);
  (void)hipFree(w->r);
  (void)hipFree(w->p);
  (void)hipFree(w->q);
  (void)hipFree(w->ss);
  if (w->hss) (void)hipHostFree(w->hss);
  delete w;
  c->mshift = nullptr;
}

static MultiShiftWork* mshift_work(lgt_ctx* c, int ns) {
  if (c->mshift && c->mshift->ns >= ns) return c->mshift;
  lgt_ctx_free_multishift(c);
  MultiShiftWork* w = new MultiShiftWork();
  c->mshift = w;
  w->ns = ns;
  const size_t bytes = (size_t)ns * c->half_elems() * sizeof(double2);
  LGT_HIP(hipMalloc(&w->X, bytes));
  LGT_HIP(hipMalloc(&w->Pn, bytes));
  const size_t hb = c->half_elems() * sizeof(double2);
  LGT_HIP(hipMalloc(&w->r, hb));
  LGT_HIP(hipMalloc(&w->p, hb));
  LGT_HIP(hipMalloc(&w->q, hb));
  LGT_HIP(hipMalloc(&w->ss, sizeof(ShiftState)));
  LGT_HIP(hipHostMalloc(&w->hss, sizeof(ShiftState), hipHostMallocDefault));
  return w;
}

int lgt_ctx_max_shifts() { return kMaxShift; }

// phi: packed full field (odd half read).  Xout[i]: the caller's canonical
// full fields, written with X_i on the odd sites and zero on the even ones
// (Xout null: the solutions stay in the workspace, mshift->X + i V/2 * 12).
// The shifted recursions stop at half the tolerance; the returned true_res
// is the largest FP64 true residual ||phi_o - (A + sigma_i) X_i|| / ||phi_o||
// over the shifts, and converged is false if it exceeds the tolerance.
SolveStats lgt_ctx::solve_multishift(const double2* phi, int ns, const double* shifts, void* const* Xout,
                                     const SolverOpts& o) {
  SolveStats st;
  MultiShiftWork* w = mshift_work(this, ns);
  const size_t h = half_elems();
  const int n = (int)h;
  const double2* phio = phi + h;
  double2* stage = f64(kStageB);  // packed full field holding one output at a time
  LGT_HIP(launch_zero64(n, stage, stream));
  auto emit = [&](int i, const double2* xo) {
    if (!Xout) return;
    LGT_HIP(launch_copy64(n, xo, stage + h, stream));
    LGT_HIP(launch_unpack(g, 12, stage, (double2*)Xout[i], stream));
  };
  LGT_HIP(launch_norm_dot(n, phio, nullptr, red(), 0, stream));
  read_results(1);
  const double bb = host_result[0];
  if (!std::isfinite(bb)) throw Error(LGT_ERR_NONFINITE, "phi holds NaN or Inf");
  if (bb == 0.0) {
    LGT_HIP(launch_zero64(n, stage + h, stream));
    LGT_HIP(launch_zero64((int)(ns * h), w->X, stream));
    for (int i = 0; i < ns; ++i)
      if (Xout) LGT_HIP(launch_unpack(g, 12, stage, (double2*)Xout[i], stream));
    st.true_res = 0.0;
    return st;
  }
  double2* r = w->r;
  double2* p = w->p;
  double2* t = f64(kW0);      // even-half scratch, as the FP64 CG's
  double2* wv = f64(kW4) + h;  // odd-half scratch, as the FP64 CG's
  const int nb = std::min((n + 255) / 256, 2048);
  hipLaunchKernelGGL(k_msinit, dim3(nb), dim3(256), 0, stream, n, ns, phio, r, p, w->X, w->Pn);
  LGT_HIP(hipGetLastError());
  ShiftState& s = *w->hss;
  s = ShiftState{};
  s.ns = ns;
  s.alpha_prev = 1.0;
  s.beta_prev = 0.0;
  const double tol_in = 0.5 * o.tol;
  s.rr_stop = tol_in * tol_in * bb;
  for (int i = 0; i < ns; ++i) {
    s.sigma[i] = shifts[i];
    s.zeta[i] = s.zeta_prev[i] = 1.0;
  }
  LGT_HIP(hipMemcpyAsync(w->ss, w->hss, sizeof(ShiftState), hipMemcpyHostToDevice, stream));
  SolverState& b0 = *host_state;
  b0 = SolverState{};
  b0.rr = bb;
  b0.rr0 = bb;
  b0.rr_max = bb;
  b0.rr_stop = 0.0;  // the base recursion never stops on its own: the shifts decide
  b0.max_iter = o.max_iter;
  b0.done = kDoneRunning;
  LGT_HIP(hipMemcpyAsync(state, host_state, sizeof(SolverState), hipMemcpyHostToDevice, stream));
  const double k2 = -kappa * kappa;
  const Reduce rd = red();
  // the recursion's hops read two-row links when the links are SU(3) to FP64
  // rounding, as the single-shift FP64 CG's; the true residuals below use the
  // full links
  compress_links64();
  sync();
  const int nk = host_flags[2] == 0 ? 6 : 9;
  const double2* links = nk == 6 ? U64c : U64;
  auto iteration = [&] {
    LGT_HIP((launch_hop_axpy<double, false>(g, 0, HopIn<double>{links, p, p, nk}, t, t, nullptr, nullptr, 1.0,
                                             stream, state)));
    LGT_HIP((launch_hop_schur_norm<double, double2, false>(g, HopIn<double>{links, t, t, nk}, wv, p, k2, state, rd,
                                                            stream)));
    // block 0 also forms alpha = |r|^2 / |Mhat p|^2 from the partials
    LGT_HIP((launch_hop_axpy<double, true>(g, 0, HopIn<double>{links, wv, wv, nk}, t, t, nullptr, nullptr, 1.0,
                                            stream, state, rd.partials)));
    // r -= alpha A p, |r|^2 partials; the base solution is not formed
    LGT_HIP((launch_hop_schur_cg<double, double2, true>(g, HopIn<double>{links, t, t, nk}, wv, nullptr, r, p, k2,
                                                         state, rd, stream)));
    hipLaunchKernelGGL(k_msfinalize, dim3(1), dim3(256), 0, stream, hop_blocks(g, 1), rd.partials, state, w->ss,
                       rd.mbox);
    LGT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_msupdate, dim3(nb), dim3(256), 0, stream, n, ns, r, p, w->X, w->Pn, state, w->ss);
    LGT_HIP(hipGetLastError());
  };
  for (int iter0 = 0;;) {
    drive(iter0, iteration);
    LGT_HIP(hipMemcpyAsync(host_state, state, sizeof(SolverState), hipMemcpyDeviceToHost, stream));
    sync();
    if (b0.done != kDoneRunning) break;
    iter0 = b0.iter;
  }
  st.iters = b0.iter;
  if (b0.done == kDoneBreakdown) throw Error(LGT_ERR_NONFINITE, "multi-shift CG breakdown");
  if (b0.done == kDoneMaxIter) st.converged = false;
  // true residuals, all norms read back at once (two result slots per shift)
  double2* q = w->q;
  for (int i = 0; i < ns; ++i) {
    double2* xi = w->X + (size_t)i * h;
    apply_mhat_dag_mhat64(false, xi, q);
    LGT_HIP(launch_axpy64(n, shifts[i], xi, q, stream));
    LGT_HIP(launch_xmy64(n, phio, q, stream));  // q = phi_o - (A + sigma_i) X_i
    LGT_HIP(launch_norm_dot(n, q, nullptr, red(), 2 * i, stream));
    emit(i, xi);
  }
  read_results(2 * ns);
  double worst = 0.0;
  for (int i = 0; i < ns; ++i) {
    const double tr = std::sqrt(host_result[2 * i] / bb);
    if (!std::isfinite(tr)) throw Error(LGT_ERR_NONFINITE, "non-finite residual");
    worst = std::max(worst, tr);
  }
  st.true_res = worst;
  if (worst > o.tol) st.converged = false;
  return st;
}

// Rational (RHMC) even/odd pseudofermion action S_R = phi_o^dag R(A) phi_o,
// R(A) = a0 + sum_i a_i (A + sigma_i)^-1, A = Mhat^dag Mhat, and its force.
// With X_i = (A + sigma_i)^-1 phi_o from one multi-shift solve, the term i
// varies as -a_i X_i^dag dA X_i = -2 a_i Re[Y_i^dag dMhat X_i], Y_i = Mhat X_i
// (the shift is constant): the even/odd bilinear of each X_i with the
// coefficient -2 kappa a_i, summed into one gradient.  S_R is evaluated as
// a0 |phi_o|^2 + sum_i a_i (2 Re phi_o^dag X_i - |Y_i|^2 - sigma_i |X_i|^2),
// equal to the action at the solutions and second order in their error.
SolveStats lgt_ctx::rational_force(const double2* phi, int ns, const double* shifts, const double* residues,
                                   double a0, const SolverOpts& o, int mode, double dt, void* out, double* S) {
  SolveStats st = solve_multishift(phi, ns, shifts, nullptr, o);
  MultiShiftWork* w = mshift;
  const size_t h = half_elems();
  const int n = (int)h;
  const int ng = 72 * vh;  // complex elements of a gauge-type field
  const double2* phio = phi + h;
  double2* xf = f64(kStageA);  // (H_eo X_o, X_o)
  double2* af = f64(kE);       // (H_oe^dag Y_o, Y_o)
  double2* gsum = g64(12);
  double2* gtmp = g64(13);
  LGT_HIP(launch_zero64(ng, gsum, stream));
  const double k2 = -kappa * kappa;
  double sr = 0.0;
  if (S) {
    LGT_HIP(launch_norm_dot(n, phio, nullptr, red(), 0, stream));
    read_results(1);
    sr = a0 * host_result[0];
  }
  for (int i = 0; i < ns; ++i) {
    const double2* xo = w->X + (size_t)i * h;
    LGT_HIP(launch_copy64(n, xo, xf + h, stream));
    const HopIn<double> hx{U64, xf + h, xf + h};
    LGT_HIP((launch_hop_axpy<double, false>(g, 0, hx, xf, xf, nullptr, nullptr, 1.0, stream)));  // X_e = H_eo X_o
    const HopIn<double> he{U64, xf, xf};
    LGT_HIP((launch_hop_axpy<double, false>(g, 1, he, af + h, af + h, xf + h, xf + h, k2, stream)));  // Y_o
    const HopIn<double> hy{U64, af + h, af + h};
    LGT_HIP((launch_hop_axpy<double, true>(g, 0, hy, af, af, nullptr, nullptr, 1.0, stream)));  // H_oe^dag Y_o
    LGT_HIP(launch_bilinear_force(g, U64, af, xf, kappa, -2.0 * kappa * residues[i], LGT_OUT_GRAD, 0.0, gtmp,
                                  kPacked, stream));
    LGT_HIP(launch_axpy64(ng, 1.0, gtmp, gsum, stream));
    if (S) {
      LGT_HIP(launch_norm_dot(n, xf + h, phio, red(), 0, stream));  // |X_i|^2, Re <X_i, phi_o>
      LGT_HIP(launch_norm_dot(n, af + h, nullptr, red(), 2, stream));  // |Y_i|^2
      read_results(4);
      sr += residues[i] * (2.0 * host_result[1] - host_result[2] - shifts[i] * host_result[0]);
    }
  }
  if (S) *S = sr;
  // the output: overwritten (force, gradient) or updated in place (momentum)
  if (mode != LGT_OUT_MOMENTUM) LGT_HIP(launch_zero64(ng, (double2*)out, stream));
  const int acc = mode == LGT_OUT_FORCE ? 0 : (mode == LGT_OUT_GRAD ? 1 : 2);
  LGT_HIP(launch_grad_to_force(g, U64, gsum, acc, dt, out, kCanonical, stream));
  return st;
}
