// Batched solver: nr right-hand sides phi_n on one lattice, each with its own
// kappa_n, solved together for X_n = (D_n^dag D_n)^-1 phi_n, Y_n = D_n X_n.
// Same method as the single solve (two even/odd Schur CGNR solves, FP64
// residual, defect correction), with every launch covering all nr fields:
// one link load serves all right-hand sides, and each right-hand side has its
// own CG scalars and stops updating once converged.  Mixed precision: FP32
// recursion per right-hand side on its residual scaled to unit norm; each
// recursion stops itself on the device at its reliable-update threshold
// (as in the single solve), and once half of them have stopped the host
// updates in FP64 every right-hand side not yet verified (a verified
// solution is final and drops out of the batched hops).
#include <algorithm>
#include <cmath>

#include "lgt_ctx.h"
#include "lgt_mrhs.h"

using namespace lgt;

namespace {
enum { bPhi = 0, bX = 1, bY = 2, bRes = 3, bE = 4, bYtmp = 5, bW0 = 6, bW1 = 7, bW2 = 8, bW3 = 9, bW4 = 10,
       bStage = 11 };
}  // namespace

struct BatchWork {
  int nr = 0;
  std::vector<double2*> f;  // multi-RHS FP64 full fields
  std::vector<float2*> h;   // multi-RHS FP32 half fields
  BatchState* st = nullptr;
  BatchState* hst = nullptr;  // pinned
  double* partials = nullptr;
  size_t npart = 0;
  double* dvec = nullptr;   // device per-RHS arrays: 8 x kMaxRhs doubles
  double* hvec = nullptr;   // pinned mirror
  int* dint = nullptr;      // device restart flags
  int* hint = nullptr;
  int G[2] = {0, 0};        // right-hand sides per hop block, tuned per precision (FP32, FP64) for tuned_nr
                            // (FP32: negative = MFMA kernel with groups of -G)
  int tuned_nr = 0;
  int tuned_kind = 0;
};

static void free_batch(BatchWork* w) {
  if (!w) return;
  for (auto* p : w->f) (void)hipFree(p);
  for (auto* p : w->h) (void)hipFree(p);
  (void)hipFree(w->st);
  (void)hipFree(w->partials);
  (void)hipFree(w->dvec);
  (void)hipFree(w->dint);
  if (w->hst) (void)hipHostFree(w->hst);
  if (w->hvec) (void)hipHostFree(w->hvec);
  if (w->hint) (void)hipHostFree(w->hint);
  delete w;
}

void lgt_ctx_free_batch(lgt_ctx* c) {
  free_batch(c->batch);
  c->batch = nullptr;
}

// per-RHS device arrays (slots of kMaxRhs doubles)
enum { vOne = 0, vKap = 1, vMKap = 2, vMK2 = 3, vSigma = 4, vPscale = 5, vScale = 6, vUnverified = 7 };

static BatchWork* batch_work(lgt_ctx* c, int nr) {
  if (c->batch && c->batch->nr >= nr) return c->batch;
  lgt_ctx_free_batch(c);
  BatchWork* w = new BatchWork();
  c->batch = w;
  w->nr = nr;
  const size_t full = (size_t)24 * c->vh * nr, half = (size_t)12 * c->vh * nr;
  w->f.assign(12, nullptr);
  for (auto& p : w->f) {
    LGT_HIP(hipMalloc(&p, full * sizeof(double2)));
    LGT_HIP(hipMemsetAsync(p, 0, full * sizeof(double2), c->stream));
  }
  w->h.assign(5, nullptr);
  for (auto& p : w->h) {
    LGT_HIP(hipMalloc(&p, half * sizeof(float2)));
    LGT_HIP(hipMemsetAsync(p, 0, half * sizeof(float2), c->stream));
  }
  LGT_HIP(hipMalloc(&w->st, sizeof(BatchState)));
  LGT_HIP(hipHostMalloc(&w->hst, sizeof(BatchState), hipHostMallocDefault));
  w->npart = (size_t)std::max(mrhs_hop_blocks(c->g, -1), 1024) * kMaxRhs;
  LGT_HIP(hipMalloc(&w->partials, w->npart * sizeof(double)));
  LGT_HIP(hipMalloc(&w->dvec, 8 * kMaxRhs * sizeof(double)));
  LGT_HIP(hipHostMalloc(&w->hvec, 8 * kMaxRhs * sizeof(double), hipHostMallocDefault));
  LGT_HIP(hipMalloc(&w->dint, kMaxRhs * sizeof(int)));
  LGT_HIP(hipHostMalloc(&w->hint, kMaxRhs * sizeof(int), hipHostMallocDefault));
  return w;
}

// Autotuner of the batched hop: the kernel (VALU, or for FP32 the MFMA form)
// and its group size G (right-hand sides per block): large G loads the
// links fewer times, small G launches more blocks (more waves to hide
// latency on small lattices).  Every VALU G that gives a distinct number of
// groups, and the MFMA groups of 8 and 4 (encoded G = -8, -4), are timed
// once per context, right-hand-side count, precision and kernel choice
// (lgt_set_batch_hop_kernel) with HIP events on the context stream; the
// fastest is kept.
static void tune_group_size(lgt_ctx* c, BatchWork* w, int nr, bool f32) {
  if (w->tuned_nr != nr || w->tuned_kind != c->batch_hop_kind) {
    w->G[0] = w->G[1] = 0;
    w->tuned_nr = nr;
    w->tuned_kind = c->batch_hop_kind;
  }
  int& G = w->G[f32 ? 0 : 1];
  if (G != 0) return;
  if (f32) c->ensure_u32();
  const Reduce red{w->partials, c->result, 0, w->npart, nullptr};
  const double* coef = w->dvec;  // any finite values: only the time is used
  double best = 1e30;
  int prev_groups = 0;
  std::vector<int> cand;
  if (!f32 || c->batch_hop_kind != 2)
    for (int gsz = nr; gsz >= 1; --gsz) {
      const int ngroups = (nr + gsz - 1) / gsz;
      if (ngroups == prev_groups) continue;
      prev_groups = ngroups;
      cand.push_back(gsz);
    }
  if (f32 && c->batch_hop_kind != 1) {
    cand.push_back(-8);
    cand.push_back(-4);
  }
  for (int gsz : cand) {
    auto once = [&] {
      if (f32) {
        HopIn<float> hin{c->U32, w->h[0], w->h[0]};
        LGT_HIP((launch_mhop_axpy<float, false>(c->g, nr, gsz, 0, hin, w->h[1], w->h[1], nullptr, nullptr, coef,
                                                 c->stream, nullptr, nullptr, red)));
      } else {
        HopIn<double> hin{c->U64, w->f[bW0], w->f[bW0]};
        LGT_HIP((launch_mhop_axpy<double, false>(c->g, nr, gsz, 0, hin, w->f[bW1], w->f[bW1], nullptr, nullptr,
                                                  coef, c->stream, nullptr, nullptr, red)));
      }
    };
    once();
    once();
    LGT_HIP(hipEventRecord(c->ev0, c->stream));
    for (int i = 0; i < 8; ++i) once();
    LGT_HIP(hipEventRecord(c->ev1, c->stream));
    LGT_HIP(hipEventSynchronize(c->ev1));
    float ms = 0.f;
    LGT_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    if (ms < best) {
      best = ms;
      G = gsz;
    }
  }
}

namespace {

struct BatchSolver {
  lgt_ctx* c;
  BatchWork* w;
  int nr;
  const SolverOpts& o;
  std::vector<double> kap;
  std::vector<SolveStats> st;  // per right-hand side
  const float2* links32 = nullptr;  // links of the FP32 inner hops (set by the first mixed solve)
  int nk32 = 9;

  Reduce red() const { return Reduce{w->partials, c->result, 0, w->npart, c->mbox_dev}; }
  template <typename R>
  int gsize() const { return w->G[sizeof(R) == 8 ? 1 : 0]; }
  size_t halfn() const { return (size_t)12 * c->vh * nr; }
  double* vec(int slot) const { return w->dvec + slot * kMaxRhs; }
  double2* F(int i) const { return w->f[i]; }

  void upload_vecs() {
    LGT_HIP(hipMemcpyAsync(w->dvec, w->hvec, 8 * kMaxRhs * sizeof(double), hipMemcpyHostToDevice, c->stream));
  }
  void read_results(int n) {
    LGT_HIP(hipMemcpyAsync(c->host_result, c->result, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    c->sync();
  }
  void read_state() {
    LGT_HIP(hipMemcpyAsync(w->hst, w->st, sizeof(BatchState), hipMemcpyDeviceToHost, c->stream));
    c->sync();
  }
  void write_state() {
    LGT_HIP(hipMemcpyAsync(w->st, w->hst, sizeof(BatchState), hipMemcpyHostToDevice, c->stream));
  }

  template <typename R, bool DAG>
  void mhop(int p_out, const R2<R>* gauge, const R2<R>* in, R2<R>* out, const R2<R>* self, const double* coef,
            BatchState* guard = nullptr, const double* pap = nullptr, const double* mask = nullptr, int nk = 9) {
    HopIn<R> hin{gauge, in, in, nk};
    LGT_HIP((launch_mhop_axpy<R, DAG>(c->g, nr, gsize<R>(), p_out, hin, out, out, self, self, coef, c->stream, guard, pap,
                                       red(), mask)));
  }

  // out = Mhat^dag Mhat x (FP64) for the right-hand sides with mask[n] != 0
  // (all if mask is null; the others' out is left as it was), scratch: even
  // half of bW0, odd half of bW4
  void apply_normal64(bool dag, const double2* x, double2* out, const double* mask = nullptr) {
    double2* t = F(bW0);
    double2* wv = F(bW4) + halfn();
    if (!dag) {
      mhop<double, false>(0, c->U64, x, t, nullptr, vec(vOne), nullptr, nullptr, mask);
      mhop<double, false>(1, c->U64, t, wv, x, vec(vMK2), nullptr, nullptr, mask);
      mhop<double, true>(0, c->U64, wv, t, nullptr, vec(vOne), nullptr, nullptr, mask);
      mhop<double, true>(1, c->U64, t, out, wv, vec(vMK2), nullptr, nullptr, mask);
    } else {
      mhop<double, true>(0, c->U64, x, t, nullptr, vec(vOne), nullptr, nullptr, mask);
      mhop<double, true>(1, c->U64, t, wv, x, vec(vMK2), nullptr, nullptr, mask);
      mhop<double, false>(0, c->U64, wv, t, nullptr, vec(vOne), nullptr, nullptr, mask);
      mhop<double, false>(1, c->U64, t, out, wv, vec(vMK2), nullptr, nullptr, mask);
    }
  }

  // gauge: packed links with nk components per link (9, or 6 for the FP32
  // two-row copy of SU(3) links)
  template <typename R, bool DAG>
  void iteration(const R2<R>* gauge, R2<R>* t, R2<R>* wv, R2<R>* x, R2<R>* r, R2<R>* p, int nk = 9) {
    const size_t n = halfn();
    mhop<R, DAG>(0, gauge, p, t, nullptr, vec(vOne), w->st, nullptr, nullptr, nk);
    HopIn<R> h2{gauge, t, t, nk};
    LGT_HIP((launch_mhop_schur_norm<R, DAG>(c->g, nr, gsize<R>(), h2, wv, p, vec(vMK2), w->st, red(), c->stream)));
    mhop<R, !DAG>(0, gauge, wv, t, nullptr, vec(vOne), w->st, w->partials, nullptr, nk);
    HopIn<R> h4{gauge, t, t, nk};
    // x += alpha p moves to the direction update, which reads p anyway
    LGT_HIP((launch_mhop_schur_cg<R, !DAG>(c->g, nr, gsize<R>(), h4, wv, nullptr, r, p, vec(vMK2), w->st, red(),
                                            c->stream)));
    LGT_HIP(launch_mxpay<R>(c->vh, nr, r, p, x, w->st, c->stream));
  }

  void cg64(bool dag, double2* z, const double2* rhs, double tol) {
    const size_t n = halfn();
    double2* t = F(bW0);
    double2* r = F(bW2) + n;
    double2* p = F(bW3) + n;
    double2* wv = F(bW4) + n;
    LGT_HIP(launch_mcg_init64(c->vh, nr, rhs, r, p, z, w->st, red(), tol, o.max_iter, c->stream));
    for (int iter0 = 0;;) {
      c->drive(iter0, [&] {
        if (dag) iteration<double, true>(c->U64, t, wv, z, r, p);
        else iteration<double, false>(c->U64, t, wv, z, r, p);
      });
      read_state();
      if (w->hst->all_done) break;
      iter0 = w->hst->iter;
    }
    for (int k = 0; k < nr; ++k) {
      st[k].iters += w->hst->conv_iter[k];
      if (w->hst->done[k] == kDoneBreakdown) throw Error(LGT_ERR_NONFINITE, "batched CG breakdown");
      if (w->hst->done[k] == kDoneMaxIter) st[k].converged = false;
    }
  }

  void cg_mixed(bool dag, double2* z, const double2* rhs, double tol) {
    const size_t n = halfn();
    c->ensure_u32();
    float2* ts = w->h[0];
    float2* ws = w->h[1];
    float2* xs = w->h[2];
    float2* rs = w->h[3];
    float2* ps = w->h[4];
    double2* r64 = F(bW2) + n;
    // the inner hops read the two-row copy of the links when every link is
    // SU(3) and the VALU batched hop runs (the MFMA form reads full links);
    // the check's flag arrives with the sync below
    const bool first = !links32;
    if (first) c->compress_links();
    LGT_HIP(launch_zero64((int)n, z, c->stream));
    LGT_HIP(launch_zero32((int)n, xs, c->stream));
    LGT_HIP(launch_mnorm<double>(c->vh, 12, nr, rhs, red(), c->stream));
    read_results(nr);
    if (first) {
      const bool two_row = c->host_flags[1] == 0 && gsize<float>() > 0;
      links32 = two_row ? c->U32c : c->U32;
      nk32 = two_row ? 6 : 9;
    }
    std::vector<double> target(nr), sigma(nr);
    std::vector<int> verified(nr, 0);
    for (int k = 0; k < nr; ++k) {
      const double bb = c->host_result[k];
      if (!std::isfinite(bb)) throw Error(LGT_ERR_NONFINITE, "right-hand side holds NaN or Inf");
      target[k] = tol * tol * bb;
      sigma[k] = bb > 0.0 ? 1.0 / std::sqrt(bb) : 1.0;
      verified[k] = bb == 0.0;
    }
    BatchState& s = *w->hst;
    s = BatchState{};
    s.nr = nr;
    s.max_iter = o.max_iter;
    s.delta2 = o.delta * o.delta;
    for (int k = 0; k < nr; ++k) {
      s.rr[k] = s.rr_max[k] = 1.0;
      s.rr_stop[k] = tol * tol;
      s.done[k] = verified[k] ? kDoneConverged : kDoneRunning;
      w->hvec[vSigma * kMaxRhs + k] = sigma[k];
      w->hvec[vPscale * kMaxRhs + k] = 1.0;
      w->hint[k] = 1;
    }
    s.all_done = std::all_of(verified.begin(), verified.end(), [](int v) { return v != 0; });
    upload_vecs();
    LGT_HIP(hipMemcpyAsync(w->dint, w->hint, kMaxRhs * sizeof(int), hipMemcpyHostToDevice, c->stream));
    LGT_HIP(launch_mrescale(c->vh, nr, rhs, vec(vSigma), rs, ps, w->dint, vec(vPscale), c->stream));
    write_state();
    while (!s.all_done) {
      c->drive(s.iter, [&] {
        if (dag) iteration<float, true>(links32, ts, ws, xs, rs, ps, nk32);
        else iteration<float, false>(links32, ts, ws, xs, rs, ps, nk32);
      });
      read_state();
      // the device asks for the update once half of the unverified right-hand
      // sides have stopped (a stopped one idles until then)
      int active = 0, stopped = 0;
      for (int k = 0; k < nr; ++k) {
        if (verified[k]) continue;
        ++active;
        stopped += s.done[k] != kDoneRunning;
      }
      if (!s.all_done && 2 * stopped < active) continue;  // nothing posted for long (see drive)
      // reliable update for every right-hand side not yet verified (a
      // verified one's solution is final: its FP64 residual is not formed,
      // and the batched hops skip it)
      for (int k = 0; k < nr; ++k) {
        w->hvec[vScale * kMaxRhs + k] = 1.0 / sigma[k];
        w->hvec[vUnverified * kMaxRhs + k] = verified[k] ? 0.0 : 1.0;
      }
      upload_vecs();
      LGT_HIP(launch_mmixed_update(c->vh, nr, xs, z, vec(vScale), c->stream));
      apply_normal64(dag, z, r64, vec(vUnverified));
      LGT_HIP(launch_xmy64((int)n, rhs, r64, c->stream));
      LGT_HIP(launch_mnorm<double>(c->vh, 12, nr, r64, red(), c->stream));
      read_results(nr);
      bool all = true;
      for (int k = 0; k < nr; ++k) {
        const double rr64 = c->host_result[k];
        if (!verified[k]) {
          if (!std::isfinite(rr64)) throw Error(LGT_ERR_NONFINITE, "non-finite residual in the batched solve");
          st[k].reliable += 1;
          if (rr64 <= target[k]) verified[k] = 1;
        }
        if (verified[k]) {
          s.done[k] = kDoneConverged;
          w->hint[k] = 0;
          w->hvec[vPscale * kMaxRhs + k] = 1.0;
          w->hvec[vSigma * kMaxRhs + k] = sigma[k];
          continue;
        }
        all = false;
        const double sn = 1.0 / std::sqrt(rr64);
        w->hint[k] = s.done[k] == kDoneBreakdown ? 1 : 0;  // its last direction update did not happen
        w->hvec[vPscale * kMaxRhs + k] = sn / sigma[k];
        w->hvec[vSigma * kMaxRhs + k] = sn;
        sigma[k] = sn;
        s.rr[k] = s.rr_max[k] = 1.0;
        s.rr_stop[k] = target[k] * sn * sn;
        s.done[k] = s.iter >= o.max_iter ? kDoneMaxIter : kDoneRunning;
        if (s.done[k] == kDoneMaxIter) {
          verified[k] = 1;
          st[k].converged = false;
        }
      }
      s.all_done = all || std::all_of(verified.begin(), verified.end(), [](int v) { return v != 0; });
      s.any_update = 0;
      if (s.all_done) break;
      upload_vecs();
      LGT_HIP(hipMemcpyAsync(w->dint, w->hint, kMaxRhs * sizeof(int), hipMemcpyHostToDevice, c->stream));
      LGT_HIP(launch_mrescale(c->vh, nr, r64, vec(vSigma), rs, ps, w->dint, vec(vPscale), c->stream));
      write_state();
    }
    // each right-hand side's count is the iterations its own recursion ran
    // (a stopped one idles until the batch's update without counting)
    for (int k = 0; k < nr; ++k) st[k].iters += s.work[k];
  }

  void solve_M(bool dag, double2* z, const double2* b, double tol) {
    const size_t h = halfn();
    const double2* be = b;
    const double2* bo = b + h;
    double2* bp = F(bW0) + h;
    double2* te = F(bW0);
    double2* rhs = F(bW1) + h;
    if (dag) {
      mhop<double, true>(1, c->U64, be, bp, bo, vec(vKap));
      mhop<double, false>(0, c->U64, bp, te, nullptr, vec(vOne));
      mhop<double, false>(1, c->U64, te, rhs, bp, vec(vMK2));
    } else {
      mhop<double, false>(1, c->U64, be, bp, bo, vec(vKap));
      mhop<double, true>(0, c->U64, bp, te, nullptr, vec(vOne));
      mhop<double, true>(1, c->U64, te, rhs, bp, vec(vMK2));
    }
    double2* zo = z + h;
    if (o.precision == LGT_FP64) cg64(dag, zo, rhs, tol);
    else cg_mixed(dag, zo, rhs, tol);
    if (dag) mhop<double, true>(0, c->U64, zo, z, be, vec(vKap));
    else mhop<double, false>(0, c->U64, zo, z, be, vec(vKap));
  }

  void dslash_full(const double2* in, double2* out, bool dag) {
    const size_t h = halfn();
    HopIn<double> hin{c->U64, in, in + h};
    if (dag)
      LGT_HIP((launch_mhop_axpy<double, true>(c->g, nr, gsize<double>(), -1, hin, out, out + h, in, in + h, vec(vMKap), c->stream,
                                               nullptr, nullptr, red())));
    else
      LGT_HIP((launch_mhop_axpy<double, false>(c->g, nr, gsize<double>(), -1, hin, out, out + h, in, in + h, vec(vMKap), c->stream,
                                                nullptr, nullptr, red())));
  }

  void run() {
    const size_t nfull = 2 * halfn();
    for (int k = 0; k < kMaxRhs; ++k) {
      const double kk = k < nr ? kap[k] : 0.0;
      w->hvec[vOne * kMaxRhs + k] = 1.0;
      w->hvec[vKap * kMaxRhs + k] = kk;
      w->hvec[vMKap * kMaxRhs + k] = -kk;
      w->hvec[vMK2 * kMaxRhs + k] = -kk * kk;
    }
    upload_vecs();
    const double2* phi = F(bPhi);
    LGT_HIP(launch_mnorm<double>(c->vh, 24, nr, phi, red(), c->stream));
    read_results(nr);
    std::vector<double> pp(c->host_result, c->host_result + nr);
    for (double v : pp)
      if (!std::isfinite(v)) throw Error(LGT_ERR_NONFINITE, "phi holds NaN or Inf");
    const double tol_in = o.tol * (o.first_pass > 0.0 ? o.first_pass : 0.25);
    solve_M(true, F(bY), phi, tol_in);
    solve_M(false, F(bX), F(bY), tol_in);
    double tol_used = tol_in;                   // CG tolerance of the last pass
    std::vector<double> res_start(nr, 1.0);     // each residual when that pass started
    for (int pass = 0;; ++pass) {
      dslash_full(F(bX), F(bY), false);
      HopIn<double> hin{c->U64, F(bY), F(bY) + halfn()};
      LGT_HIP(launch_mhop_residual<true>(c->g, nr, gsize<double>(), hin, F(bY), phi, F(bRes), vec(vMKap), red(),
                                         c->stream));
      read_results(nr);
      bool ok = true;
      double tol_corr = 0.5;  // the tightest any right-hand side still above the target needs
      unsigned finished = 0;  // right-hand sides that take no correction
      for (int k = 0; k < nr; ++k) {
        st[k].true_res = pp[k] > 0.0 ? std::sqrt(c->host_result[k] / pp[k]) : 0.0;
        if (!std::isfinite(st[k].true_res)) throw Error(LGT_ERR_NONFINITE, "non-finite residual");
        const bool done_k = st[k].true_res <= o.tol || !st[k].converged;
        ok = ok && done_k;
        if (done_k) finished |= 1u << k;
        else tol_corr = std::min(tol_corr, correction_tol(o.tol, st[k].true_res, tol_used, res_start[k]));
      }
      if (ok || pass >= 4) break;
      // a correction only has to shrink each residual by about tol / true_res
      // (the single solve's rule, correction_tol); the right-hand sides that
      // already meet the target get a zero residual, so their CG stops at
      // once and their solution stays as it is
      LGT_HIP(launch_mzero_rhs(c->vh, 24, nr, F(bRes), finished, c->stream));
      solve_M(true, F(bYtmp), F(bRes), tol_corr);
      solve_M(false, F(bE), F(bYtmp), tol_corr);
      LGT_HIP(launch_axpy64((int)nfull, 1.0, F(bE), F(bX), c->stream));
      tol_used = tol_corr;
      for (int k = 0; k < nr; ++k) {
        res_start[k] = st[k].true_res;
        if (!((finished >> k) & 1u)) ++st[k].corrections;
      }
    }
    for (int k = 0; k < nr; ++k)
      if (st[k].true_res > o.tol) st[k].converged = false;
  }
};

}  // namespace

std::vector<SolveStats> lgt_ctx::solve_batch(int nr, const double* kappas, const void* const* phis,
                                             void* const* Xs, void* const* Ys, const SolverOpts& o) {
  BatchWork* w = batch_work(this, nr);
  tune_group_size(this, w, nr, false);
  if (o.precision != LGT_FP64) tune_group_size(this, w, nr, true);
  BatchSolver b{this, w, nr, o, std::vector<double>(kappas, kappas + nr), std::vector<SolveStats>(nr)};
  for (int k = 0; k < nr; ++k) LGT_HIP(launch_mpack(g, nr, k, (const double2*)phis[k], w->f[bPhi], stream));
  b.run();
  for (int k = 0; k < nr; ++k) {
    LGT_HIP(launch_munpack(g, nr, k, w->f[bX], (double2*)Xs[k], stream));
    if (Ys && Ys[k]) LGT_HIP(launch_munpack(g, nr, k, w->f[bY], (double2*)Ys[k], stream));
  }
  return b.st;
}

// out_n = D_n in_n (or D_n^dag in_n), D_n = 1 - kappa_n H, for nr fields in
// one batched hop launch over both parities: FP64, or (f32) the FP32
// batched hop on FP32 copies of the links and inputs, its output widened
// back to FP64.
void lgt_ctx::dslash_batch(int nr, const double* kappas, const void* const* ins, void* const* outs, bool dag,
                           bool f32) {
  BatchWork* w = batch_work(this, nr);
  tune_group_size(this, w, nr, f32);
  const int G = w->G[f32 ? 0 : 1];
  for (int k = 0; k < kMaxRhs; ++k) {
    w->hvec[vOne * kMaxRhs + k] = 1.0;
    w->hvec[vMKap * kMaxRhs + k] = k < nr ? -kappas[k] : 0.0;
  }
  LGT_HIP(hipMemcpyAsync(w->dvec, w->hvec, 8 * kMaxRhs * sizeof(double), hipMemcpyHostToDevice, stream));
  const double* one = w->dvec + vOne * kMaxRhs;
  const double* mkap = w->dvec + vMKap * kMaxRhs;
  for (int k = 0; k < nr; ++k) LGT_HIP(launch_mpack(g, nr, k, (const double2*)ins[k], w->f[bPhi], stream));
  const size_t h = (size_t)12 * vh * nr;
  const Reduce red{w->partials, result, 0, w->npart, nullptr};
  if (f32) {
    // the half fields h[0], h[1] hold the even and odd FP32 input, h[2], h[3] the output
    LGT_HIP(launch_convert_64_32((int)h, w->f[bPhi], w->h[0], stream));
    LGT_HIP(launch_convert_64_32((int)h, w->f[bPhi] + h, w->h[1], stream));
    HopIn<float> hin{U32, w->h[0], w->h[1]};
    if (dag)
      LGT_HIP((launch_mhop_axpy<float, true>(g, nr, G, -1, hin, w->h[2], w->h[3], w->h[0], w->h[1], mkap, stream,
                                              nullptr, nullptr, red)));
    else
      LGT_HIP((launch_mhop_axpy<float, false>(g, nr, G, -1, hin, w->h[2], w->h[3], w->h[0], w->h[1], mkap, stream,
                                               nullptr, nullptr, red)));
    LGT_HIP(launch_zero64((int)(2 * h), w->f[bX], stream));
    LGT_HIP(launch_mmixed_update(vh, nr, w->h[2], w->f[bX], one, stream));
    LGT_HIP(launch_mmixed_update(vh, nr, w->h[3], w->f[bX] + h, one, stream));
  } else {
    HopIn<double> hin{U64, w->f[bPhi], w->f[bPhi] + h};
    if (dag)
      LGT_HIP((launch_mhop_axpy<double, true>(g, nr, G, -1, hin, w->f[bX], w->f[bX] + h, w->f[bPhi],
                                               w->f[bPhi] + h, mkap, stream, nullptr, nullptr, red)));
    else
      LGT_HIP((launch_mhop_axpy<double, false>(g, nr, G, -1, hin, w->f[bX], w->f[bX] + h, w->f[bPhi],
                                                w->f[bPhi] + h, mkap, stream, nullptr, nullptr, red)));
  }
  for (int k = 0; k < nr; ++k) LGT_HIP(launch_munpack(g, nr, k, w->f[bX], (double2*)outs[k], stream));
}

double lgt_ctx::bench_mhop(int nr, bool f32, const void* psi, int nrep) {
  BatchWork* w = batch_work(this, nr);
  tune_group_size(this, w, nr, f32);
  const int G = w->G[f32 ? 0 : 1];
  for (int k = 0; k < nr; ++k) LGT_HIP(launch_mpack(g, nr, k, (const double2*)psi, w->f[bPhi], stream));
  const size_t h = (size_t)12 * vh * nr;
  for (int k = 0; k < kMaxRhs; ++k) w->hvec[vOne * kMaxRhs + k] = 1.0;
  LGT_HIP(hipMemcpyAsync(w->dvec, w->hvec, 8 * kMaxRhs * sizeof(double), hipMemcpyHostToDevice, stream));
  const double* one = w->dvec + vOne * kMaxRhs;
  // FP32: the links the batched solve's inner hops read (the two-row copy when
  // every link is SU(3) and the VALU kernel runs)
  const float2* links32 = U32;
  int nk32 = 9;
  if (f32) {
    LGT_HIP(launch_convert_64_32((int)h, w->f[bPhi] + h, w->h[0], stream));
    compress_links();
    sync();
    if (host_flags[1] == 0 && G > 0) {
      links32 = U32c;
      nk32 = 6;
    }
  }
  const Reduce red{w->partials, result, 0, w->npart, nullptr};
  auto once = [&] {
    if (f32) {
      HopIn<float> hin{links32, w->h[0], w->h[0], nk32};
      LGT_HIP((launch_mhop_axpy<float, false>(g, nr, G, 0, hin, w->h[1], w->h[1], nullptr, nullptr, one, stream,
                                               nullptr, nullptr, red)));
    } else {
      HopIn<double> hin{U64, w->f[bPhi] + h, w->f[bPhi] + h};
      LGT_HIP((launch_mhop_axpy<double, false>(g, nr, G, 0, hin, w->f[bX], w->f[bX], nullptr, nullptr, one, stream,
                                                nullptr, nullptr, red)));
    }
  };
  once();  // warm-up
  LGT_HIP(hipEventRecord(ev0, stream));
  for (int i = 0; i < nrep; ++i) once();
  LGT_HIP(hipEventRecord(ev1, stream));
  LGT_HIP(hipEventSynchronize(ev1));
  float ms = 0.f;
  LGT_HIP(hipEventElapsedTime(&ms, ev0, ev1));
  return (double)ms / nrep;
}
