// Multi-right-hand-side (batched) solver interface: device state and launchers.
#pragma once

#include "lgt_internal.h"

namespace lgt {

constexpr int kMaxRhs = 16;

// Device-resident state of a batch of CG solves sharing one operator up to
// the per-RHS kappa.  Right-hand side n stops updating once done[n] is set;
// the launches stop when all are done.
// Codes are the kDone* of the single solve; delta2 > 0 turns on the
// device-side stop for reliable updates (kDoneUpdate), any_update says that
// some right-hand side still has its final direction update to do.
struct BatchState {
  int nr, iter, max_iter, all_done, any_update;
  int idle;  // set by an iteration's finalize that found the batch stopped (a queued no-op iteration)
  double delta2;
  int done[kMaxRhs];
  int conv_iter[kMaxRhs];
  int work[kMaxRhs];  // iterations in which the right-hand side's recursion ran (its iteration count)
  double rr[kMaxRhs], pap[kMaxRhs], alpha[kMaxRhs], beta[kMaxRhs], rr_stop[kMaxRhs], rr_max[kMaxRhs];
};

hipError_t launch_mfinalize(int mode, int nblk, int nr, Reduce red, BatchState* st, double tol, int max_iter,
                            hipStream_t s);
// rows of per-RHS partials a reducing batched hop writes (one per site block)
int mrhs_hop_blocks(const Geom& g, int p_out);

// Batched hops over nr fields in the [12][nr][vh] layout; G = right-hand
// sides per block (1..nr; the links are loaded once per group of G) for the
// VALU kernel, or G = -4 / -8 for the MFMA kernel (FP32 only) with groups
// of 4 or 8 right-hand sides.
// out = self + coef_n H in  (coef: device array [nr]); guard/pap_partials as launch_hop_axpy;
// mask (device array [nr], optional): only the right-hand sides with mask[n] != 0 are
// computed, the others' output is left as it was
template <typename R, bool DAG>
hipError_t launch_mhop_axpy(const Geom& g, int nr, int G, int p_out, HopIn<R> hin, R2<R>* out_e, R2<R>* out_o,
                            const R2<R>* self_e, const R2<R>* self_o, const double* coef, hipStream_t s,
                            BatchState* guard, const double* pap_partials, Reduce red,
                            const double* mask = nullptr);
template <typename R, bool DAG>
hipError_t launch_mhop_schur_norm(const Geom& g, int nr, int G, HopIn<R> hin, R2<R>* w, const R2<R>* x,
                                  const double* coef, BatchState* st, Reduce red, hipStream_t s);
template <typename R, bool DAG>
hipError_t launch_mhop_schur_cg(const Geom& g, int nr, int G, HopIn<R> hin, const R2<R>* w, R2<R>* x, R2<R>* r,
                                const R2<R>* p, const double* coef, BatchState* st, Reduce red, hipStream_t s);
// r = phi - (self + coef_n H in) over both parities, result[n] = |r_n|^2
template <bool DAG>
hipError_t launch_mhop_residual(const Geom& g, int nr, int G, HopIn<double> hin, const double2* self_full,
                                const double2* phi_full, double2* r_full, const double* coef, Reduce red,
                                hipStream_t s);

// result[n] = |a_n|^2 over a multi-RHS field of ncomp components (12 half, 24 full)
template <typename R>
hipError_t launch_mnorm(int vh, int ncomp, int nr, const R2<R>* a, Reduce red, hipStream_t s);
// half-field updates, per right-hand side n
template <typename R>
hipError_t launch_mxpay(int vh, int nr, const R2<R>* r, R2<R>* p, R2<R>* x, BatchState* st, hipStream_t s);
hipError_t launch_mmixed_update(int vh, int nr, float2* xs, double2* x, const double* scale, hipStream_t s);
hipError_t launch_mrescale(int vh, int nr, const double2* r64, const double* sigma, float2* r, float2* p,
                           const int* restart, const double* pscale, hipStream_t s);
hipError_t launch_mcg_init64(int vh, int nr, const double2* b, double2* r, double2* p, double2* x,
                             BatchState* st, Reduce red, double tol, int max_iter, hipStream_t s);
// zero right-hand side n of a multi-RHS FP64 field of ncomp components for every bit n of mask
hipError_t launch_mzero_rhs(int vh, int ncomp, int nr, double2* f, unsigned mask, hipStream_t s);
hipError_t launch_mpack(const Geom& g, int nr, int n, const double2* canon, double2* packed, hipStream_t s);
hipError_t launch_munpack(const Geom& g, int nr, int n, const double2* packed, double2* canon, hipStream_t s);

}  // namespace lgt
