// Host-side context: geometry, stream, device workspace, and the solver.
#pragma once

#include <algorithm>

#include <hip/hip_runtime.h>

#include <chrono>
#include <memory>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/lgt.h"
#include "lgt_internal.h"
#include "stout_schedule.h"

namespace lgt {

// Error carrying an ABI status across the C++ layers (never across the ABI).
struct Error : std::runtime_error {
  lgt_status status;
  Error(lgt_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define LGT_HIP(call)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      throw ::lgt::Error(e_ == hipErrorOutOfMemory ? LGT_ERR_OUT_OF_MEMORY : LGT_ERR_DEVICE, \
                         std::string(#call) + ": " + hipGetErrorString(e_));                \
  } while (0)

struct SolveStats {
  int iters = 0;
  int reliable = 0;
  int corrections = 0;
  double true_res = 0.0;
  bool converged = true;
};

// slots of the context's full FP64 scratch fields (lgt_ctx::f64)
enum ScratchSlot {
  kPhi = 0, kX = 1, kY = 2, kRes = 3, kE = 4, kYtmp = 5,
  kW0 = 6, kW1 = 7, kW2 = 8, kW3 = 9, kW4 = 10,
  kStageA = 11, kStageB = 12
};

struct SolverOpts {
  int precision = LGT_FP64;
  double tol = 1e-10;
  int max_iter = 20000;
  double delta = 3e-4;
  double first_pass = 0.0;  // first-pass CG tolerance / tol (0: the solver's default)
};

// Tolerance of the next defect-correction pass.  The last pass ran its CG to
// tol_used relative to the residual it started from (res_start, relative to
// ||phi||) and left the FP64 true residual true_res, so the solve chain
// magnified its stopping residual by A = true_res / (tol_used res_start).
// A pass on r with CG tolerance t leaves about A t true_res; t is chosen to
// land at half the target.
inline double correction_tol(double tol, double true_res, double tol_used, double res_start) {
  const double A = true_res / (tol_used * res_start);
  const double t = 0.5 * tol / (A * true_res);
  return std::min(0.5, std::max(t, 1e-15));
}

}  // namespace lgt

struct BatchWork;       // batched-solver workspace (batch.hip)
struct MultiShiftWork;  // multi-shift solver workspace (multishift.hip)
struct lgt_ctx;
void lgt_ctx_free_batch(lgt_ctx* c);
// batch object of lgt_cg_solve_batch: the caller's stream, one stream per
// lattice of a call (created on demand, default priority) and their events
struct lgt_batch {
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> events;
  std::string err;
};
// message lgt_last_error(NULL) returns (calls without a context)
void lgt_set_global_error(const std::string& msg);
void lgt_ctx_free_multishift(lgt_ctx* c);
int lgt_ctx_max_shifts();

struct lgt_ctx {
  lgt::Geom g{};
  int64_t V = 0;
  int vh = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;

  // packed links: FP64 [2][4][9][vh], FP32 copy (mixed precision), and the
  // first two rows [2][4][6][vh] of each for the CG hops
  double2* U64 = nullptr;
  float2* U32 = nullptr;
  float2* U32c = nullptr;
  double2* U64c = nullptr;
  // packed momenta for the MD driver
  double2* P64 = nullptr;

  // spinor workspace: FP64 full fields (24*vh complex each) and FP32 half fields
  std::vector<double2*> full64;
  std::vector<float2*> half32;
  // packed FP64 gauge-type scratch fields (72*vh complex each)
  std::vector<double2*> gauge64;

  // reductions / solver state
  lgt::SolverState* state = nullptr;
  double* partials = nullptr;
  double* result = nullptr;      // device results
  double* host_result = nullptr; // pinned mirror
  int* flags = nullptr;          // device: [0] non-finite input, [1] links not SU(3), [2] the same for FP64
  int* host_flags = nullptr;     // pinned
  lgt::SolverState* host_state = nullptr;  // pinned
  lgt::Mailbox* mbox_host = nullptr;        // pinned, coherent: progress posted by CG steps
  lgt::Mailbox* mbox_dev = nullptr;         // its device address
  hipEvent_t ev0 = nullptr, ev1 = nullptr;

  size_t half_elems() const { return (size_t)12 * vh; }
  size_t full_elems() const { return (size_t)24 * vh; }
  lgt::Reduce red() const {
    return lgt::Reduce{partials, result, lgt::reduce_capacity(vh), (size_t)lgt::reduce_capacity(vh) * 4, mbox_dev};
  }

  double2* f64(int i);   // full FP64 spinor scratch i (allocated on demand)
  double2* g64(int i);   // packed FP64 gauge-type scratch i (allocated on demand)
  float2* h32(int i);    // half FP32 spinor scratch i
  void ensure_u32();
  // Enqueues the two-row copy of U32 and the check that its links are SU(3),
  // whose result (host_flags[1] == 0) is valid after the caller's next sync.
  void compress_links();
  // The same for U64 (host_flags[2] == 0: its links are SU(3) to FP64 rounding).
  void compress_links64();
  void ensure_p64();

  // solver (solver.hip)
  lgt::SolveStats solve_ddagd(const double2* phi, double2* X, double2* Y, const lgt::SolverOpts& o);
  void dslash_full(const double2* in, double2* out, double kappa, bool dag);
  double action_fermion(const double2* phi, const double2* X, const double2* Y);
  // even/odd-preconditioned action (odd half of phi) and its force fields
  lgt::SolveStats solve_eo(const double2* phi, double2* X, double2* A, const lgt::SolverOpts& o);
  double action_eo(const double2* phi, const double2* X, const double2* A);
  void sync();
  void read_results(int n);

  // Enqueues step() -- one CG iteration, ending in a kernel that posts to
  // the mailbox -- until the device posts that the host has to act, keeping
  // kQueueAhead iterations queued beyond the last one the device finished
  // (the surplus ones see the stopped state and return at once).  iter0 is
  // the device's iteration count before the first step; no unfinished CG
  // step may be on the stream.  Actions whose epoch (the high bits of the
  // action, see action_word) is below min_epoch are stale -- posted by
  // iterations queued behind a stop the caller has already acted on -- and
  // ignored.  Returns the mailbox word (action in the high 32 bits; none if
  // nothing was posted for 30 s), after synchronising the stream unless
  // sync_end is false.
  static constexpr int kQueueAhead = 2;
  template <typename Step>
  unsigned long long drive(int iter0, Step&& step, unsigned min_epoch = 0, bool sync_end = true) {
    unsigned long long* w = &mbox_host->word;
    __atomic_store_n(w, (unsigned long long)(unsigned)iter0, __ATOMIC_RELEASE);
    int queued = iter0, seen_prev = iter0;
    unsigned long long v = 0;
    auto t_prev = std::chrono::steady_clock::now();
    for (;;) {
      v = __atomic_load_n(w, __ATOMIC_ACQUIRE);
      const unsigned act = (unsigned)(v >> 32);
      if (act && (act >> 8) >= min_epoch) break;
      const int seen = (int)(unsigned)v;
      if (queued - seen < kQueueAhead) {
        step();
        ++queued;
        continue;
      }
      const auto now = std::chrono::steady_clock::now();
      if (seen != seen_prev) {
        seen_prev = seen;
        t_prev = now;
      } else if (now - t_prev > std::chrono::seconds(30)) {
        v = (unsigned long long)(unsigned)seen;  // nothing posted for long: the caller reads the state
        break;
      }
      __builtin_ia32_pause();
    }
    if (sync_end) sync();
    return v;
  }

  // stout smearing (smear.hip): U0, G packed FP64
  void smear(const double2* U0, int nlevels, double rho, double2* dst);
  // checkpointed reverse pass (stout_schedule.h): slot cap (-1: as many
  // levels as device memory holds), the schedule for n levels, the forward
  // sweep that keeps its checkpoints, and the reverse pass over it
  int stout_slot_cap = -1;
  // kernel of the FP32 batched hop: 0 timed choice, 1 VALU, 2 MFMA (batch.hip)
  int batch_hop_kind = 0;
  int last_stout_slots = 0;
  int64_t last_stout_passes = 0;
  std::unique_ptr<lgt::StoutSchedule> sched;
  int stout_slots(int nlevels);
  const lgt::StoutSchedule& stout_plan(int nlevels);
  void smear_checkpointed(const double2* U0, int nlevels, double rho, double2* dst, const lgt::StoutSchedule& plan);
  void stout_backprop(const double2* U0, int nlevels, double rho, double2* G, const lgt::StoutSchedule& plan,
                      bool forward_done);
  lgt::SolveStats smeared_force(const double2* U0, const double2* phi, double beta, double rho, int nlevels,
                                const lgt::SolverOpts& o, int mode, double dt, void* out, int layout,
                                double* S_F);

  // batched solves (batch.hip): nr right-hand sides with their own kappa
  BatchWork* batch = nullptr;
  double bench_mhop(int nr, bool f32, const void* psi, int nrep);  // ms per multi-RHS hop launch
  void dslash_batch(int nr, const double* kappas, const void* const* ins, void* const* outs, bool dag, bool f32);
  std::vector<lgt::SolveStats> solve_batch(int nr, const double* kappas, const void* const* phis, void* const* Xs,
                                           void* const* Ys, const lgt::SolverOpts& o);

  // multi-shift CG (multishift.hip): X_i = (Mhat^dag Mhat + shifts[i])^-1 phi_o
  MultiShiftWork* mshift = nullptr;
  lgt::SolveStats solve_multishift(const double2* phi, int ns, const double* shifts, void* const* Xout,
                                   const lgt::SolverOpts& o);
  // rational even/odd action and force (multishift.hip); out: canonical gauge field
  lgt::SolveStats rational_force(const double2* phi, int ns, const double* shifts, const double* residues, double a0,
                                 const lgt::SolverOpts& o, int mode, double dt, void* out, double* S);

  double kappa = 0.0;  // hopping parameter of the current solve
 private:
  // precision: an lgt_precision value
  void solve_M(bool dag, double2* z, const double2* b, double tol, int max_iter, int precision,
               double delta, lgt::SolveStats& st);
  int cg_normal64(bool dag, double2* z, const double2* rhs, double tol, int max_iter,
                  lgt::SolveStats& st);
  template <typename T>  // storage of the FP32 recursion's t, w, p: float2 or lgt::Bf16c
  int cg_normal_mixed(bool dag, double2* z, const double2* rhs, double tol, int max_iter, double delta,
                      lgt::SolveStats& st);
  void apply_mhat_dag_mhat64(bool dag, const double2* x, double2* out);
};
