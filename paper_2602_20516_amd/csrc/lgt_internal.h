// Internal (non-ABI) interface between the C ABI layer, the solver driver
// and the kernel launchers.  Host and device code both include it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "lgt_device.h"

namespace lgt {

// Device-resident state of one CG solve.  Scalars are produced by the last
// block of the reduction kernels and consumed by the next kernels, so the
// host never has to read them inside the iteration.
struct SolverState {
  double rr;        // |r|^2 of the current iterate
  double pap;       // |M p|^2 = p^dag A p
  double alpha;
  double beta;
  double rr_stop;   // stop when rr <= rr_stop
  double rr0;       // |b|^2
  double rr_max;    // mixed precision: largest |r|^2 since the last FP64 update
  double delta2;    // mixed precision: stop for an FP64 update once rr <= delta2 * rr_max (0: never)
  double rr_prev;   // rr and iter as the third hop of the running iteration found them (the
                    // step kernel's blocks read these copies while its block 0 rewrites rr, iter)
  double sigma;     // mixed precision: units of the FP32 recursion (1 / |FP64 residual| at the last update)
  double rr_target; // mixed precision: FP64 |r|^2 at which the solve has converged
  double bscale;    // mixed precision: factor of the old direction in the first new one
  int iter;
  int max_iter;
  int done;         // a kDone* code
  int iter_prev;
  int epoch;        // reliable updates done; tags the mailbox actions (see action_word)
  int restart;      // mixed precision: the next direction restarts from the residual
  int nupd;         // FP64 residual recomputations
  int pad;
};

// kDoneUpdate: the recursion stopped for an FP64 (reliable) update in this
// iteration; its direction update is skipped (the reliable update forms the
// next direction from the true residual).  The next step kernel turns it
// into kDoneUpdateHeld, which no kernel touches.
enum { kDoneRunning = 0, kDoneConverged = 1, kDoneMaxIter = 2, kDoneBreakdown = 3, kDoneUpdate = 4,
       kDoneUpdateHeld = 5, kDoneFailed = 6 };
// kDoneFailed: the FP64 residual of a reliable update is not finite.

// Output layout of the gauge-type kernels (forces, link update).
enum Layout { kCanonical = 0, kPacked = 1 };

// Arguments of a hop launch.  Half-fields are [12][vh] complex; a "full"
// spinor is even half followed by odd half.  T is the storage type of the
// input spinor (R2<R>, or Bf16c for BF16-stored spinors).
template <typename R, typename T = R2<R>>
struct HopIn {
  const R2<R>* gauge;  // packed links [2][4][nk][vh]
  const T* in_even;
  const T* in_odd;
  int nk = 9;          // 9: full links; 6: the first two rows of SU(3) links (the third
                       // is rebuilt as the conjugate cross product of the two)
};

// Host-visible progress of an iterative solve, in pinned host memory: the
// last kernel of every CG step (step or finalize kernel) posts the device's
// iteration count (low 32 bits) and whether the host has to act (high 32
// bits, nonzero: the recursion stopped, converged, or the batch wants an
// update; for the single-field CG the action word of action_word), so the
// host can keep a few iterations queued ahead of the GPU instead of
// synchronising.  One 64-bit store, so the host never sees a torn pair.
struct Mailbox {
  unsigned long long word;
};

__device__ __forceinline__ void post_progress(Mailbox* mb, int iter, int action) {
  if (!mb) return;
  const unsigned long long v = ((unsigned long long)(unsigned)action << 32) | (unsigned)iter;
  __hip_atomic_store(&mb->word, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Action word of a CG stop: the stop code and the state's epoch, so that the
// host can tell a stop it has already acted on (posted again by iterations
// that were queued behind it) from a new one.
__host__ __device__ inline unsigned action_word(int epoch, int code) {
  return ((unsigned)epoch << 8) | (unsigned)code;
}

// Workspace scalars used by reductions.
struct Reduce {
  double* partials;   // one slot per block (per value) of the reducing launch
  double* result;     // small array of results read by the host
  int capacity;       // largest single-RHS reducing grid (partials hold >= 4 * capacity doubles)
  size_t ndoubles;    // size of partials
  Mailbox* mbox;      // device address of the progress mailbox (CG steps post to it; may be null)
};

// What the one-block finalize kernel does with the summed partials.
enum FinalizeMode {
  kFinResult1 = 0,   // result[slot] = sum (1 value per block)
  kFinResult2 = 1,   // result[slot], result[slot+1] = sums (2 values per block)
  kFinCgInit = 2,    // start a CG: rr = |b|^2, rr_stop = tol^2 |b|^2, ...
  kFinCgStep = 3,    // end of a batched CG iteration (k_mfinalize): rr, beta, iteration count, convergence
};
hipError_t launch_finalize(int mode, int nblk, Reduce red, SolverState* st, int slot, double tol, int max_iter,
                           hipStream_t s);
// number of blocks of a hop launch (p_out >= 0: one parity, -1: both)
int hop_blocks(const Geom& g, int p_out);

// Lattices with at most this many sites per parity run the hop with 32
// sites per block (half-wave hops), larger ones with 64.
constexpr int kHopHalfWaveMaxVh = 8192;
// Above this many sites per parity the 64-site hop takes its blocks
// t-fastest (when a t-slice holds a whole number of blocks).
constexpr int kHopTOrderMinVh = 131072;

// Reduction capacity needed for a lattice with vh sites per parity: the
// largest reducing grid is the both-parity hop (2 * ceil(vh/32) blocks at
// most).
inline int reduce_capacity(int vh) {
  const int nb = 2 * ((vh + 31) / 32);
  return nb < 1024 ? 1024 : nb;
}

// ---- launchers (kernels_*.hip) --------------------------------------------
// All launchers enqueue on `s` and return hipError_t of the launch.

// pack: canonical complex128 [V][nc] -> packed [2][nc][vh] (FP64 and, if
// out32 != nullptr, FP32).  nonfinite: integer flag set to 1 if any input is NaN/Inf.
hipError_t launch_pack(const Geom& g, int nc, const double2* canon, double2* out64, float2* out32,
                       int* nonfinite, hipStream_t s);
hipError_t launch_unpack(const Geom& g, int nc, const double2* packed, double2* canon, hipStream_t s);
// Pi = i sum_a c_a T_a per link from normals [V][4][8] (canonical output)
hipError_t launch_momenta(const Geom& g, const double* normals, double2* P, hipStream_t s);

// Hop variants (kernels_hop.hip).  p_out in {0,1}: one parity; -1: both.
// out = self + coef * H in   (self may be null); T: spinor storage type
// guard: skip once the solve has stopped; pap_partials: block 0 also forms
// pap and alpha from the previous launch's partials (see EpiAxpy::tail)
template <typename T> struct NoDeduce { using type = T; };  // keeps nullptr arguments out of deduction
template <typename R, bool DAG, typename T = R2<R>>
hipError_t launch_hop_axpy(const Geom& g, int p_out, HopIn<R, T> hin, T* out_even, T* out_odd,
                           const typename NoDeduce<T>::type* self_even, const typename NoDeduce<T>::type* self_odd,
                           double coef, hipStream_t s, SolverState* guard = nullptr,
                           const double* pap_partials = nullptr);
// t = H (r + beta p) = H r + beta t and p = r + beta p, after the CG step of
// the previous iteration (every block: beta and the stop test from its |r|^2
// partials; block 0 records the state); a no-op once the solve has stopped.
// For R2<R> storage (FP64, FP32).
template <typename R, bool DAG>
hipError_t launch_hop_step(const Geom& g, const R2<R>* gauge, int nk, R2<R>* t, R2<R>* p, const R2<R>* r,
                           SolverState* st, Reduce red, hipStream_t s);
// One CG iteration on Mhat^dag Mhat (Mhat = 1 - kappa^2 H_oe H_eo, odd sites)
// is four hop launches and the step kernel:
//  (1) t = H p                                      launch_hop_axpy (guard)
//  (2) w = p + coef H t, |w|^2 partials             launch_hop_schur_norm
//  (3) t = H^dag w; block 0: alpha = rr / |w|^2    launch_hop_axpy with pap_partials
//  (4) q = w + coef H^dag t; r -= alpha q; |r|^2 partials
//                                                   launch_hop_schur_cg
//  (5) rr, beta and the stop decision (every block sums the partials),
//      x += alpha p, p = r + beta p unless stopping, block 0 records the
//      state and posts                              launch_cg_step
// (on small lattices (1) also does (5) of the previous iteration, see
// launch_hop_step, and (4) then takes the x update)
// (for the dagger operator the roles of H and H^dag swap).  t, w, p are
// stored as T; x and r as R2<R>.
template <typename R, typename T, bool DAG>
hipError_t launch_hop_schur_norm(const Geom& g, HopIn<R, T> hin, T* w, const T* x, double coef, SolverState* st,
                                 Reduce red, hipStream_t s);
// (x may be null: the multi-shift solver tracks no base solution).  The
// |r|^2 partials are left for the caller's step or finalize kernel.
template <typename R, typename T, bool DAG>
hipError_t launch_hop_schur_cg(const Geom& g, HopIn<R, T> hin, const T* w, R2<R>* x, R2<R>* r, const T* p,
                               double coef, SolverState* st, Reduce red, hipStream_t s);
// Residual of the full operator: r = phi - (self + coef * H in) over both parities,
// result[slot] = |r|^2
template <bool DAG>
hipError_t launch_hop_residual(const Geom& g, HopIn<double> hin, const double2* self_full,
                               const double2* phi_full, double2* r_full, double coef, Reduce red,
                               int slot, hipStream_t s);

// Vector kernels (kernels_field.hip).  n = number of complex elements.
// End of a CG iteration: rr = sum of the nblk |r|^2 partials of (4), beta =
// rr / rr_prev, the stop test (target, reliable-update threshold, iteration
// cap, non-finite), x += alpha p (the iteration's step, whatever the
// decision), p = r + beta p (p stored as T) unless the recursion stops here
// (the reliable update then forms the next direction, see
// launch_rescale_residual); the new state and the mailbox post come from
// block 0.  A skipped iteration only posts (and holds an update).
template <typename R, typename T>
hipError_t launch_cg_step(int n, const R2<R>* r, T* p, SolverState* st, Reduce red, int nblk, hipStream_t s,
                          R2<R>* x);
template <typename R>
hipError_t launch_cg_init(int n, const R2<R>* b, R2<R>* r, R2<R>* p, R2<R>* x, SolverState* st,
                          Reduce red, double tol, int max_iter, hipStream_t s);
// result[slot] = |a|^2 (and result[slot+1] = Re <a,b> if b != null)
hipError_t launch_norm_dot(int n, const double2* a, const double2* b, Reduce red, int slot,
                           hipStream_t s);
hipError_t launch_axpy64(int n, double a, const double2* x, double2* y, hipStream_t s);  // y += a x
hipError_t launch_copy64(int n, const double2* x, double2* y, hipStream_t s);
hipError_t launch_xmy64(int n, const double2* x, double2* y, hipStream_t s);             // y = x - y
hipError_t launch_zero64(int n, double2* y, hipStream_t s);
hipError_t launch_zero32(int n, float2* y, hipStream_t s);
hipError_t launch_convert_64_32(int n, const double2* x, float2* y, hipStream_t s);
// Links in two-row form: Uc[p][mu][6][vh] = rows 0 and 1 of U, and flag set
// to 1 (never cleared here) if for some link the third row stored in U is not
// the conjugate cross product of the first two (FP32 to 1e-5, FP64 to 1e-14),
// i.e. the links are not SU(3) and must not be compressed.
hipError_t launch_compress_links(const Geom& g, const float2* U32, float2* Uc, int* flag, hipStream_t s);
hipError_t launch_compress_links(const Geom& g, const double2* U64, double2* Uc, int* flag, hipStream_t s);
// mixed precision helpers
// Device-side reliable update, enqueued without a host round trip:
//   launch_mixed_fold:       x += xs / st->sigma; xs = 0
//   launch_reliable_decide:  |r64|^2 (deterministic two-launch reduction),
//     then: not finite -> kDoneFailed; <= rr_target -> kDoneConverged; else
//     new units sigma = 1 / |r64|, restart flag (the recursion broke down),
//     bscale = beta sigma_new / sigma_old, the recursion's state reset
//     (rr = rr_max = 1, rr_stop = rr_target sigma^2), kDoneRunning; epoch
//     and nupd counted; a stop is posted to the mailbox
//   launch_rescale_residual_dev: as launch_rescale_residual with sigma,
//     restart and bscale from the state, and only if it is running
hipError_t launch_mixed_fold(int n, float2* xs, double2* x, const SolverState* st, hipStream_t s);
hipError_t launch_reliable_decide(int n, const double2* r64, Reduce red, SolverState* st, hipStream_t s);
template <typename T>
hipError_t launch_rescale_residual_dev(int n, const double2* r64, float2* r, T* p, const SolverState* st,
                                       hipStream_t s);
// reliable update of the FP32 recursion: r = (float)(sigma r64); then the
// next search direction p = r (restart) or p = r + bscale p (bscale = beta
// of the stopping iteration times the change of units), p stored as T
// (float2 or Bf16c)
template <typename T>
hipError_t launch_rescale_residual(int n, const double2* r64, double sigma, float2* r, T* p, int restart,
                                   double bscale, hipStream_t s);

// Forces / gauge kernels (kernels_force.hip).  Gauge-type outputs: layout
// kCanonical -> [V][4][3][3] complex128, kPacked -> [2][4][9][vh].
// mode: 0 force, 1 grad, 2 momentum (P -= dt F).
hipError_t launch_bilinear_force(const Geom& g, const double2* U, const double2* a_full,
                                 const double2* b_full, double kappa, double coeff, int mode, double dt,
                                 void* out, int layout, hipStream_t s);
hipError_t launch_gauge_force(const Geom& g, const double2* U, double beta, int mode, double dt,
                              void* out, int layout, hipStream_t s);
// result[slot] = sum_x sum_{mu<nu} Re tr P_mu,nu(x); with Uold, the sum of
// the per-site differences of that quantity between U and Uold
hipError_t launch_plaquette(const Geom& g, const double2* U, Reduce red, int slot, hipStream_t s,
                            const double2* Uold = nullptr);
// result[slot] = -sum Re tr P^2 over a gauge-type field of either layout;
// with Pold (same layout), the sum of the per-link differences P minus Pold
hipError_t launch_kinetic(const Geom& g, const double2* P, int layout, Reduce red, int slot,
                          hipStream_t s, const double2* Pold = nullptr);
// U <- reunit(exp(dt P) U), both in `layout`; U32 (packed FP32 copy) refreshed if non-null
hipError_t launch_link_update(const Geom& g, double2* U, const double2* P, double dt, int layout,
                              float2* U32, hipStream_t s);

// Stout smearing (kernels_stout.hip), packed FP64 gauge fields.
hipError_t launch_stout_fwd(const Geom& g, const double2* U, double2* Uo, double rho, hipStream_t s);
// Adjoint of one level at input links U: Go = gradient at U given Gp at the output.
hipError_t launch_stout_adjoint(const Geom& g, const double2* U, const double2* Gp, double rho, double2* Lam,
                                double2* Gpart, double2* Go, hipStream_t s);
// mode 0: out += F, 1: out += G, 2: out -= dt F, with F = -1/2 P[U G^dag]
hipError_t launch_grad_to_force(const Geom& g, const double2* U, const double2* G, int mode, double dt, void* out,
                                int layout, hipStream_t s);

}  // namespace lgt
