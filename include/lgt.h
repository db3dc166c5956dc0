/*
 * lgt.h -- C ABI of the MI355X (gfx950) Wilson-fermion HMC hot path.
 *
 * The library computes, on one GPU, the pieces of Hybrid Monte Carlo for
 * SU(3) lattice gauge theory with two-flavour Wilson fermions that the paper
 * ("Lattice Gauge Theory via LLVM-Level Automatic Differentiation") obtains
 * by reverse-mode AD of the action code:
 *
 *   - the Wilson-Dirac operator D(U) (used in S_f of eq. S3.1),
 *   - the solve of A chi = phi, A = D^dag D (eq. S3.6; solved by an iterative
 *     method and not differentiated, Supp. S3 remarks on the linear solver),
 *   - the actions S_G (Wilson plaquette) and S_f = phi^dag (D^dag D)^-1 phi,
 *   - the MD forces: the pseudofermion force from
 *     delta S_f = -2 Re[eta^dag (delta D) chi] (eq. S3.12) and the plaquette
 *     (staple) force, projected to su(3) (eq. 7 / S2.9),
 *   - the leapfrog step U -> exp(dt Pi) U, Pi -> Pi - dt F (eqs. S2.1-S2.2).
 *
 * Here the forces are explicit adjoint kernels, not AD output.
 *
 * ---------------------------------------------------------------------------
 * Conventions shared by every call
 * ---------------------------------------------------------------------------
 * Lattice: dims = {Lx, Ly, Lz, Lt}, every extent even and >= 2; lexicographic
 *   site index  s = x + Lx*(y + Ly*(z + Lz*t));  V = Lx*Ly*Lz*Lt.
 *   Directions mu = 0,1,2,3 are x,y,z,t.  Links are periodic; the fermion
 *   field has the temporal boundary sign fermion_t_bc (-1: antiperiodic)
 *   applied to the t-links of the last time slice inside D only.
 *
 * Field buffers (all DEVICE pointers, caller-owned, complex128 = two
 *   little-endian doubles re, im, at least 16-byte aligned):
 *     gauge-type (U, momenta Pi, force F, gradient G): [V][4][3][3],
 *       matrix element (row i, column j) at [s][mu][i][j];
 *     spinor (phi, X, Y, in/out of D): [V][4][3] (spin, colour).
 *   The library never frees a caller buffer nor keeps a pointer to it
 *   past the call.  Input and output buffers of one call must not overlap,
 *   except where a call documents an in-place update.
 *
 * D (the paper leaves it implicit; this is the hopping-parameter form):
 *   (D psi)(x) = psi(x) - kappa * sum_mu [ (1 - gamma_mu) U~_mu(x) psi(x+mu)
 *                                       + (1 + gamma_mu) U~_mu(x-mu)^dag psi(x-mu) ]
 *   chiral basis gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 =
 *   [[0,1],[1,0]], gamma_5 = diag(1,1,-1,-1); U~ = U except on the t-links of
 *   the last time slice, where U~ = fermion_t_bc * U.
 *
 * Gradients and forces (Sec. S2): the gradient of a real action S is
 *   G = dS/dRe U + i dS/dIm U (eq. S2.12), so delta S = Re tr(G^dag delta U);
 *   the force is F = -1/2 P_su3[U G^dag] with
 *   P_su3[A] = (A - A^dag)/2 - tr(A - A^dag)/6 (eq. 7).  The momentum update
 *   Pi <- Pi - dt F equals the paper's Pi <- Pi + (dt/2) P_su3[U G^dag].
 *   Momenta are traceless anti-Hermitian, K = -sum tr Pi^2.
 *
 * Streams: every call enqueues its work on the context's HIP stream
 *   (lgt_create / lgt_set_stream).  Calls that return host values
 *   (actions, solver statistics, Delta H) synchronise that stream before
 *   returning; the others return once the work is enqueued.
 *
 * Errors: every call returns lgt_status; no C++ exception crosses the ABI.
 *   On LGT_ERR_NOT_CONVERGED the outputs hold the last iterate and the
 *   statistics are filled.  On any other error the outputs are unspecified
 *   and lgt_last_error(ctx) describes the failure.
 *
 * Concurrency: one context per stream/thread; contexts are independent.
 *   Calls on one context must not overlap.
 */
#ifndef LGT_H
#define LGT_H

#include <stdint.h>

/* Symbols of the shared library (built with hidden default visibility). */
#define LGT_API __attribute__((visibility("default")))

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lgt_status {
  LGT_OK = 0,
  LGT_ERR_INVALID_ARGUMENT = 1,
  LGT_ERR_NOT_CONVERGED = 2,
  LGT_ERR_NONFINITE = 3,
  LGT_ERR_OUT_OF_MEMORY = 4,
  LGT_ERR_DEVICE = 5,
  LGT_ERR_UNSUPPORTED = 6
} lgt_status;

/* Precision of the solver's inner iterations.  LGT_FP64: every step in
 * FP64.  LGT_MIXED_FP32: inner CG with FP32 links, spinors and hops inside
 * an FP64 reliable-update loop that recomputes the residual in FP64 and
 * accumulates the solution in FP64; the stopping test is on the FP64
 * residual.  LGT_MIXED_BF16: as LGT_MIXED_FP32 with the spinors the inner
 * recursion passes between its hop kernels (search direction and the two
 * Schur intermediates) stored in bfloat16, rounded to nearest even; FP32
 * arithmetic, FP32 solution and residual, FP32 links.  Single-field solves
 * only (lgt_cg_solve_batch returns UNSUPPORTED for it). */
typedef enum lgt_precision {
  LGT_FP64 = 0,
  LGT_MIXED_FP32 = 1,
  LGT_MIXED_BF16 = 2
} lgt_precision;

/* What a force call writes.
 *   LGT_OUT_FORCE:    out = F (traceless anti-Hermitian), overwritten.
 *   LGT_OUT_GRAD:     out = G = dS/dRe U + i dS/dIm U, overwritten.
 *   LGT_OUT_MOMENTUM: out holds the momenta Pi, updated in place:
 *                     Pi <- Pi - dt * F. */
typedef enum lgt_out_mode {
  LGT_OUT_FORCE = 0,
  LGT_OUT_GRAD = 1,
  LGT_OUT_MOMENTUM = 2
} lgt_out_mode;

typedef struct lgt_geom {
  int32_t dims[4];      /* Lx, Ly, Lz, Lt: each even and >= 2 */
  int32_t fermion_t_bc; /* -1 (antiperiodic) or +1 (periodic) */
} lgt_geom;

typedef struct lgt_solver_params {
  int32_t precision;     /* lgt_precision */
  int32_t even_odd;      /* 1: even/odd Schur complement + CGNR (the only form supported) */
  double tol;            /* stop when ||phi - D^dag D X|| / ||phi|| <= tol (FP64, recomputed) */
  int32_t max_iter;      /* cap on inner CG iterations per solve (<= 0: 20000) */
  double reliable_delta; /* mixed precision: FP64 residual update when the inner
                            residual norm drops by this factor (outside (0, 1):
                            3e-4 for LGT_MIXED_FP32, 0.01 for LGT_MIXED_BF16,
                            whose recursion drifts faster; with BF16 storage,
                            values other than the default can cost twice the
                            iterations) */
  double first_pass_factor; /* the first pass of the solve aims its CG at
                            first_pass_factor * tol (<= 0: 0.25 where two Schur
                            solves are chained, 0.5 for one Schur solve), so
                            that the FP64 true residual usually meets tol
                            without a correction pass; a pass that misses is
                            followed by defect-correction passes sized from the
                            measured miss */
} lgt_solver_params;

typedef struct lgt_solver_stats {
  int32_t iters;            /* inner CG iterations, summed over the solves of the call */
  int32_t reliable_updates; /* FP64 residual recomputations (mixed precision) */
  double true_rel_residual; /* ||phi - D^dag D X|| / ||phi|| in FP64 at exit */
  double ms;                /* wall time of the call on the stream, milliseconds */
  int32_t corrections;      /* FP64 defect-correction passes after the first solve */
  int32_t reserved;         /* 0 */
} lgt_solver_stats;

typedef struct lgt_ctx lgt_ctx;

/* Create a context for one lattice geometry on the current HIP device.
 * hip_stream: a hipStream_t (NULL = the default stream).  The context owns
 * its device workspace (packed link copies, solver vectors), allocated here;
 * it grows on first use of the mixed-precision and MD paths.
 * Errors: INVALID_ARGUMENT (odd or < 2 extent, bc not +-1, null out, or a
 * lattice whose FP64 half-lattice spinor reaches 4 GiB: V < 44.7M sites,
 * since kernels address fields with 32-bit offsets), OUT_OF_MEMORY, DEVICE. */
LGT_API lgt_status lgt_create(const lgt_geom* geom, void* hip_stream, lgt_ctx** out);

/* Release the context and its workspace (synchronises its stream). */
LGT_API lgt_status lgt_destroy(lgt_ctx* ctx);

/* Message describing the last failing call on ctx ("" if none).  The
 * pointer stays valid until the next call on ctx.  ctx == NULL gives the
 * message of the last failing call that takes no context (lgt_create,
 * lgt_dslash_noalloc). */
LGT_API const char* lgt_last_error(const lgt_ctx* ctx);

/* Rebind the context to another HIP stream (NULL = default stream). */
LGT_API lgt_status lgt_set_stream(lgt_ctx* ctx, void* hip_stream);

/* Number of lattice sites V of the context. */
LGT_API int64_t lgt_volume(const lgt_ctx* ctx);

/* out = D(U) in (dagger = 0) or D(U)^dag in (dagger = 1), FP64.
 * The operator of the pseudofermion action (eq. S3.1); written out above.
 * U: gauge field; in, out: spinors; kappa: hopping parameter. */
LGT_API lgt_status lgt_dslash(lgt_ctx* ctx, const void* U, const void* in, void* out,
                      double kappa, int32_t dagger);

/* lgt_dslash for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same operator, kernels and results, with no context and no allocation.
 * geom: the lattice (as lgt_create); hip_stream: the stream the work is
 * enqueued on (NULL = default stream); U, in, out, kappa, dagger as
 * lgt_dslash (device pointers, canonical layouts).  Working storage (packed
 * links and spinors, 960 bytes per site) is a device array built into the
 * library, one copy per GPU, held until the process ends; it limits the
 * lattice to V <= 65536 sites (16^4).  Every call on one GPU uses that GPU's
 * copy: calls that overlap in time on one GPU (different streams or threads)
 * race, calls ordered on one stream do not.  Returns once the work is
 * enqueued; no NaN/Inf check of the inputs (non-finite values reach out).
 * Errors: INVALID_ARGUMENT (null pointer, odd or < 2 extent, bc not +-1,
 * non-finite kappa, V > 65536), DEVICE; message via lgt_last_error(NULL). */
LGT_API lgt_status lgt_dslash_noalloc(const lgt_geom* geom, void* hip_stream, const void* U, const void* in,
                                      void* out, double kappa, int32_t dagger);

/* Solve (D^dag D) X = phi (eq. S3.6) and return Y = D X (the paper's
 * eta = D chi below eq. S3.10).  The solve is not differentiated (S3,
 * "Remarks on the role of the linear solver").  Method: two even/odd Schur
 * complement solves, D^dag Y = phi then D X = Y, each by CG on the normal
 * equations from a zero initial guess, followed by FP64 defect correction
 * until ||phi - D^dag D X|| / ||phi|| <= params->tol.  Y_or_null may be NULL.
 * stats may be NULL.  NOT_CONVERGED if max_iter is reached first (X, Y hold
 * the last iterate).  NONFINITE if phi or U holds NaN/Inf. */
LGT_API lgt_status lgt_cg_solve(lgt_ctx* ctx, const void* U, const void* phi, void* X,
                        void* Y_or_null, double kappa, const lgt_solver_params* params,
                        lgt_solver_stats* stats);

/* Actions: *S_G = beta * sum_x sum_{mu<nu} (1 - Re tr P_mu,nu(x) / 3) and
 * *S_F = phi^dag (D^dag D)^-1 phi (eq. S3.1), evaluated in the variational
 * form 2 Re phi^dag X - ||D X||^2, which is exact at the solution and
 * second-order accurate in the solver error.  Either output may be NULL
 * (S_F == NULL skips the solve; phi may then be NULL).  All FP64. */
LGT_API lgt_status lgt_action(lgt_ctx* ctx, const void* U, const void* phi, double beta, double kappa,
                      const lgt_solver_params* params, double* S_G, double* S_F,
                      lgt_solver_stats* stats);

/* Pseudofermion force: solve as in lgt_cg_solve, then the adjoint kernel of
 * delta S_f = -2 Re[Y^dag (delta D) X] (eq. S3.12) for every link, projected
 * by F = -1/2 P_su3[U G^dag].  mode/dt/out as in lgt_out_mode; out is a
 * gauge-type buffer.  The force itself is accumulated in FP64 for every
 * precision. */
LGT_API lgt_status lgt_fermion_force(lgt_ctx* ctx, const void* U, const void* phi, double kappa,
                             const lgt_solver_params* params, int32_t mode, double dt,
                             void* out, lgt_solver_stats* stats);

/* Building block of the fermion force (eq. S3.13): the gradient/force of
 * coeff * Re[a^dag D(U) b] for given spinors a, b (no solve).  The
 * pseudofermion force is coeff = -2, a = Y, b = X.  FP64. */
LGT_API lgt_status lgt_bilinear_force(lgt_ctx* ctx, const void* U, const void* a, const void* b,
                              double kappa, double coeff, int32_t mode, double dt, void* out);

/* Wilson plaquette (staple) force of S_G at coupling beta, the derivative
 * the paper's gauge listing takes by AD of the plaquette action:
 * G = -(beta/3) A^dag with A the staple sum, F = (beta/6) P_su3[U A].  FP64. */
LGT_API lgt_status lgt_gauge_force(lgt_ctx* ctx, const void* U, double beta, int32_t mode, double dt,
                           void* out);

/* U <- reunitarize(exp(dt Pi) U) on every link, in place (eq. 5 / S2.1 in
 * the anti-Hermitian form).  exp by the Cayley-Hamilton closed form;
 * reunitarization by row Gram-Schmidt with row3 = conj(row1 x row2).  FP64. */
LGT_API lgt_status lgt_link_update(lgt_ctx* ctx, void* U, const void* P, double dt);

/* HMC momentum refresh (Sec. III B): P_mu(x) = i sum_a c_a T_a with
 * T_a = lambda_a / 2 (Gell-Mann), from normals: device FP64 [V][4][8],
 * c_a at [s][mu][a-1] (the caller draws them, N(0,1) for the heat bath).
 * P: gauge-type output (canonical).  FP64. */
LGT_API lgt_status lgt_momenta_from_normals(lgt_ctx* ctx, const void* normals, void* P);

/* K = -sum_{x,mu} tr Pi_mu(x)^2 for traceless anti-Hermitian momenta.  FP64. */
LGT_API lgt_status lgt_kinetic(lgt_ctx* ctx, const void* P, double* K);

/* Leapfrog trajectory (Sec. III B; eqs. S2.1-S2.2), nsteps steps of size dt,
 * updating U and P in place:
 *   P <- P - dt/2 F(U); then nsteps times { U <- reunit(exp(dt P) U);
 *   P <- P - dt F(U) } with the last kick dt/2,
 * F = F_G + F_f with phi fixed (phi == NULL or kappa == 0: pure gauge).
 * dH_or_null receives H_end - H_start, H = K + S_G + S_f.  stats sums the
 * solver statistics over all force evaluations. */
LGT_API lgt_status lgt_md_step(lgt_ctx* ctx, void* U, void* P, const void* phi, double beta,
                       double kappa, double dt, int32_t nsteps,
                       const lgt_solver_params* params, double* dH_or_null,
                       lgt_solver_stats* stats);

/* Stout smearing (Morningstar-Peardon, the smearing cited in Sec. I and used
 * in Sec. III B): U_out = stout^nlevels(U_in), each level
 *   C_mu(x) = rho * sum_{nu != mu} [U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag
 *                                   + U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu)],
 *   U' = exp(P_su3[C U^dag]) U,
 * all directions from the previous level, no reunitarization.  FP64;
 * nlevels 0..256; U_in and U_out may not overlap. */
LGT_API lgt_status lgt_stout_smear(lgt_ctx* ctx, const void* U_in, void* U_out, double rho, int32_t nlevels);

/* Reverse mode through the smearing (the adjoint update of eq. 4, written
 * by hand): G_out = gradient at U_in of Re tr(G_top^dag stout^n(U_in)), in the
 * G convention.  The intermediate levels each level's adjoint needs follow
 * the context's checkpoint schedule (lgt_set_stout_checkpoints): the sweep
 * U_in -> the last forward checkpoint runs first, the rest are recomputed as
 * the schedule says.  The result does not depend on the schedule (same bits).
 * FP64.  G_top is a gauge-type buffer at the smeared links.  nlevels 0..256. */
LGT_API lgt_status lgt_stout_backprop(lgt_ctx* ctx, const void* U_in, const void* G_top, double rho,
                                      int32_t nlevels, void* G_out);

/* Checkpointing of deep smearing chains (memory reduction by checkpointing
 * is the first extension the paper's outlook names, Sec. IV).  The reverse
 * pass through n levels needs U_{n-1}, ..., U_0 in that order.  The forward
 * sweep that builds U_n for the solver keeps up to max_stored_levels of them
 * (one gauge field of 72 * V complex doubles each, held by the context);
 * every other level is recomputed from the nearest kept one, along the
 * schedule with the fewest recomputed smearing passes for that many slots
 * (dynamic programming over segment splits, lgt_stout_schedule).  With
 * n - 1 slots nothing is recomputed; with 0 every level is recomputed from
 * the thin links (n(n-1)/2 passes).  max_stored_levels = -1 (the default):
 * as many as the device's free memory holds beyond a reserve of 1/8 of its
 * total.  Applies to lgt_smeared_force, lgt_stout_backprop and the smeared
 * trajectories.  INVALID_ARGUMENT for values below -1. */
LGT_API lgt_status lgt_set_stout_checkpoints(lgt_ctx* ctx, int32_t max_stored_levels);

/* What the last reverse pass through the smearing did: levels kept in
 * checkpoint slots and smearing passes recomputed beyond the forward sweep. */
LGT_API lgt_status lgt_stout_last_schedule(const lgt_ctx* ctx, int32_t* stored_levels, int64_t* recompute_passes);

/* The schedule alone (host computation, no context, no device): the
 * recomputed passes of an nlevels-level reverse pass with stored_levels
 * slots, and the levels the forward sweep keeps (checkpoints_or_null: room
 * for stored_levels entries, increasing; n_checkpoints_or_null: their
 * count).  INVALID_ARGUMENT for nlevels outside 0..256 or stored_levels < 0. */
LGT_API lgt_status lgt_stout_schedule(int32_t nlevels, int32_t stored_levels, int64_t* recompute_passes,
                                      int32_t* checkpoints_or_null, int32_t* n_checkpoints_or_null);

/* Force of the smeared action S = S_G(U) + phi^dag (D^dag D)^-1 phi with D
 * built on stout^n(U) (links enter D only): the pseudofermion force on the
 * smeared links (as lgt_fermion_force), back-propagated through the
 * smearing, plus the staple force of the thin links.  mode/dt/out as
 * lgt_out_mode; S_F_or_null receives S_f. */
LGT_API lgt_status lgt_smeared_force(lgt_ctx* ctx, const void* U, const void* phi, double beta, double kappa,
                                     double rho, int32_t nlevels, const lgt_solver_params* params,
                                     int32_t mode, double dt, void* out, double* S_F_or_null,
                                     lgt_solver_stats* stats);

/* Leapfrog trajectory (as lgt_md_step) for the smeared action:
 * H = K + S_G(U) + S_f(stout^n(U)). */
LGT_API lgt_status lgt_md_step_smeared(lgt_ctx* ctx, void* U, void* P, const void* phi, double beta,
                                       double kappa, double rho, int32_t nlevels, double dt, int32_t nsteps,
                                       const lgt_solver_params* params, double* dH_or_null,
                                       lgt_solver_stats* stats);

/* Sexton-Weingarten multiple time-scale trajectory (the integrator Sec. III B
 * pairs with stout smearing, there with 10 inner steps): nsteps outer steps
 * of size dt, each Pi -= dt/2 F_f; n_inner leapfrog steps of size
 * dt/n_inner on the gauge force alone; Pi -= dt/2 F_f, adjacent outer
 * half-kicks merged.  F_f is the pseudofermion force of the plain action
 * (nlevels = 0) or of the smeared one (nlevels > 0, rho as lgt_stout_smear).
 * n_inner = 1 is the leapfrog of lgt_md_step / lgt_md_step_smeared.  U, P,
 * phi, params, dH_or_null and stats as lgt_md_step. */
LGT_API lgt_status lgt_md_step_sw(lgt_ctx* ctx, void* U, void* P, const void* phi, double beta, double kappa,
                                  double rho, int32_t nlevels, double dt, int32_t nsteps, int32_t n_inner,
                                  const lgt_solver_params* params, double* dH_or_null, lgt_solver_stats* stats);

/* ---- Even/odd-preconditioned pseudofermion action -------------------------
 * With Mhat = 1 - kappa^2 H_oe H_eo on the odd sites (H_eo: odd -> even
 * hops of D = 1 - kappa H), det D = det Mhat, so
 *   S_eo = phi_o^dag (Mhat^dag Mhat)^-1 phi_o
 * carries the determinant weight of the action of eq. S3.1 with one Schur
 * solve per evaluation; its heat bath is phi_o = Mhat^dag eta_o.  Spinors are
 * full canonical fields of which only the odd sites ((x+y+z+t) odd) count. */

/* out = Mhat in (dagger = 0) or Mhat^dag in, on the odd sites; the even
 * sites of out are set to zero and those of in are ignored.  FP64. */
LGT_API lgt_status lgt_schur_dslash(lgt_ctx* ctx, const void* U, const void* in, void* out, double kappa,
                                    int32_t dagger);

/* Force of S_eo (derivative through the Schur solve, projected as in
 * lgt_fermion_force): with X_o = (Mhat^dag Mhat)^-1 phi_o to the FP64 true
 * residual params->tol and Y_o = Mhat X_o, dS_eo = -2 Re[Y_o^dag dMhat X_o],
 * evaluated as the bilinear of the full operator with a = (H_oe^dag Y_o, Y_o),
 * b = (H_eo X_o, X_o) and coefficient -2 kappa.  mode/dt/out as
 * lgt_fermion_force; S_F_or_null receives S_eo. */
LGT_API lgt_status lgt_fermion_force_eo(lgt_ctx* ctx, const void* U, const void* phi, double kappa,
                                        const lgt_solver_params* params, int32_t mode, double dt, void* out,
                                        double* S_F_or_null, lgt_solver_stats* stats);

/* Trajectory (leapfrog for n_inner = 1, Sexton-Weingarten otherwise, as
 * lgt_md_step_sw) for H = K + S_G(U) + S_eo(U; phi_o); thin links. */
LGT_API lgt_status lgt_md_step_eo(lgt_ctx* ctx, void* U, void* P, const void* phi, double beta, double kappa,
                                  double dt, int32_t nsteps, int32_t n_inner, const lgt_solver_params* params,
                                  double* dH_or_null, lgt_solver_stats* stats);

/* ---- Batched solves over several lattices --------------------------------
 * A batch object orders the work of lgt_cg_solve_batch on the caller's
 * stream.  It owns one extra HIP stream per lattice of a call (default
 * priority), on which the lattices' solves run at the same time. */
typedef struct lgt_batch lgt_batch;

/* Create a batch object bound to hip_stream (NULL = the default stream) on
 * the current device.  Errors: INVALID_ARGUMENT (null out), DEVICE. */
LGT_API lgt_status lgt_batch_create(void* hip_stream, lgt_batch** out);
/* Release it (synchronises its streams). */
LGT_API lgt_status lgt_batch_destroy(lgt_batch* b);
/* Message of the last failing call on b ("" if none); valid until the next call. */
LGT_API const char* lgt_batch_last_error(const lgt_batch* b);
/* Rebind the batch object to another HIP stream (NULL = default stream). */
LGT_API lgt_status lgt_batch_set_stream(lgt_batch* b, void* hip_stream);

/* One right-hand side of a batched solve. */
typedef struct lgt_batch_item {
  lgt_ctx* ctx;    /* the lattice of this right-hand side (its context) */
  const void* U;   /* gauge field of that lattice: the same pointer for every item of one context */
  const void* phi; /* spinor (input) */
  void* X;         /* spinor (output): (D^dag D)^-1 phi at this item's kappa */
  void* Y_or_null; /* spinor (output) D X, or NULL */
  double kappa;    /* hopping parameter of this item */
} lgt_batch_item;

/* Batched solve of n pseudofermion fields (the solve of eq. S3.6 for each,
 * as lgt_cg_solve: same method and stopping rule) spread over up to 8
 * lattices of any sizes, each item with its own lattice and kappa: the
 * workload of many pseudofermions, kappa values and lattice sizes in one
 * call.  Items of one context (1..16 of them) are solved together: every
 * launch of that lattice covers all of its right-hand sides, so one link
 * load serves all of them, and each keeps its own CG scalars and stops
 * once converged.  The lattices run at the same time, each on a stream of
 * the batch object that waits for the work already on the caller's stream;
 * the caller's stream waits for all of them before the call returns (the
 * call synchronises).  The contexts' own streams are not used during the
 * call.  stats_per_item (may be NULL) receives n entries in item order; ms
 * is the time of the whole call.  NOT_CONVERGED if any item missed the
 * tolerance (all outputs are written).  INVALID_ARGUMENT: null pointers,
 * n < 1, more than 16 items or two gauge fields for one context, more than
 * 8 contexts, or a batched FP64 field (12 * V/2 * items complex) of 4 GiB
 * or more; UNSUPPORTED for LGT_MIXED_BF16.  The message of a failure inside
 * one lattice's solve names that lattice. */
LGT_API lgt_status lgt_cg_solve_batch(lgt_batch* b, int32_t n, const lgt_batch_item* items,
                                      const lgt_solver_params* params, lgt_solver_stats* stats_per_item);

/* Multi-shift solve, the building block of a rational (RHMC) pseudofermion
 * action (RHMC is one of the method's target algorithms, Sec. I): for each
 * of nshift (1..32) shifts sigma_i >= 0,
 *   X_i = (Mhat^dag Mhat + sigma_i)^-1 phi_o,
 * Mhat = 1 - kappa^2 H_oe H_eo the even/odd Schur operator of
 * lgt_schur_dslash (only the odd sites of phi are read).  All shifts come
 * from one Krylov space: one CG on Mhat^dag Mhat, with each shifted solution
 * formed by scalar recurrences (shifted CG), so the cost is that of one
 * solve plus one vector update per shift and iteration.  X (device, nshift
 * canonical spinor pointers, caller-owned) receive X_i on the odd sites and
 * zero on the even ones.  Each shift stops once its recursive residual is
 * below tol / 2 relative to ||phi_o||; stats->true_rel_residual is the
 * largest FP64 true residual ||phi_o - (Mhat^dag Mhat + sigma_i) X_i|| /
 * ||phi_o|| over the shifts, NOT_CONVERGED if it exceeds tol (or max_iter
 * was reached).  FP64 only: other precisions return UNSUPPORTED.
 * INVALID_ARGUMENT for a null pointer, a negative or non-finite shift, or
 * nshift outside 1..32.  Holds 2 * nshift FP64 half spinors of workspace
 * on the context, kept until it is destroyed or a larger nshift is asked. */
LGT_API lgt_status lgt_cg_solve_multishift(lgt_ctx* ctx, const void* U, const void* phi, double kappa,
                                           int32_t nshift, const double* shifts, void* const* X,
                                           const lgt_solver_params* params, lgt_solver_stats* stats);

/* Rational (RHMC) pseudofermion action on the even/odd operator and its
 * force.  A rational approximation in partial fractions,
 *   R(A) = a0 + sum_{i<nterms} residues[i] (A + shifts[i])^-1,
 * A = Mhat^dag Mhat (the normal Schur operator of lgt_schur_dslash; RHMC
 * is among the algorithms the method targets, Sec. I), defines
 *   S_R = phi_o^dag R(A) phi_o  (odd sites of phi read).
 * One lgt_cg_solve_multishift solve gives X_i = (A + shifts[i])^-1 phi_o;
 * each term varies as -residues[i] X_i^dag dA X_i (the shift is
 * constant), so the force is the sum over terms of the even/odd bilinear
 * force of lgt_fermion_force_eo taken at X_i, weighted by residues[i]; a0
 * adds no force.  mode/dt/out as lgt_fermion_force (out: canonical
 * gauge-type field on U); S_or_null receives S_R, evaluated as
 * a0|phi_o|^2 + sum_i residues[i] (2 Re phi_o^dag X_i - |Mhat X_i|^2 -
 * shifts[i] |X_i|^2), which equals S_R at the solutions and is second order
 * in their error.  nterms 1..32, shifts finite and >= 0, residues and a0
 * finite (else INVALID_ARGUMENT); FP64 only (UNSUPPORTED otherwise);
 * NOT_CONVERGED as lgt_cg_solve_multishift. */
LGT_API lgt_status lgt_rational_force_eo(lgt_ctx* ctx, const void* U, const void* phi, double kappa, int32_t nterms,
                                         const double* shifts, const double* residues, double a0,
                                         const lgt_solver_params* params, int32_t mode, double dt, void* out,
                                         double* S_or_null, lgt_solver_stats* stats);

/* Measurement entry point: times nrep back-to-back launches of the
 * even/odd hop kernel H_eo (the dominant kernel of the CG; FP64 for
 * precision = LGT_FP64, FP32 otherwise) on links U and input spinor psi,
 * with HIP events on the context stream, and returns the mean duration of
 * one launch in *avg_ms.  The algorithmic traffic of one launch is
 * 96 reals per lattice site (all 4V links, the input and output half
 * spinors); 72 in FP32 when the links are SU(3), which the FP32 hop then
 * reads as their first two rows. */
LGT_API lgt_status lgt_hop_benchmark(lgt_ctx* ctx, const void* U, const void* psi, int32_t precision,
                                     int32_t nrep, double* avg_ms);

/* The same for the batched multi-right-hand-side hop of lgt_cg_solve_batch:
 * psi (canonical spinor, device) is copied into all nrhs (1..16) slots of
 * the batched layout, and nrep launches of H_eo over the nrhs fields are
 * timed.  One launch reads all 4V links once for every right-hand side, so
 * its algorithmic traffic is 72 + 24 * nrhs reals per lattice site. */
LGT_API lgt_status lgt_hop_benchmark_mrhs(lgt_ctx* ctx, const void* U, const void* psi, int32_t nrhs,
                                          int32_t precision, int32_t nrep, double* avg_ms);

/* Work shape of the single-field hop kernel (the Wilson hop of eq. S3.1 in
 * every solve, force and dslash call of the context): sites = 64 gives each
 * 256-thread block 64 sites, each wave both hops along one direction;
 * sites = 32 gives a block 32 sites, each half-wave one of the two hops, so
 * a small lattice runs twice as many waves.  0 (the default) takes 32 up to
 * 8192 sites per parity and 64 above.  The two shapes add the eight hop
 * terms of a site in different orders, so results may differ by rounding;
 * each is deterministic.  INVALID_ARGUMENT for any other value, and for 32
 * on a lattice whose FP64 gauge field is 4 GiB or more (V above 7456540). */
LGT_API lgt_status lgt_set_hop_block_sites(lgt_ctx* ctx, int32_t sites);

/* Order in which the 64-site hop kernel takes its blocks (see
 * lgt_set_hop_block_sites): 1 = site order (x fastest); 2 = t-fastest within
 * groups of 8 (else 4 or 2) t-slices, so that a block's t-neighbours are read
 * a few blocks apart instead of a whole slice apart, which keeps them in the
 * L2 of large lattices; 0 (the default) takes 2 above 131072 sites per
 * parity and 1 below.  Order 2 applies only where a t-slice holds a whole
 * number of 64-site blocks (Lx Ly Lz / 128 integer), else site order is
 * used.  Results do not depend on the order except through the summation
 * order of the kernels' reductions.  INVALID_ARGUMENT for other values. */
LGT_API lgt_status lgt_set_hop_block_order(lgt_ctx* ctx, int32_t order);

/* out[k] = D(U) in[k] (dagger = 0) or D(U)^dag in[k] (dagger = 1) with
 * kappa = kappas[k], for n (1..16) spinors on this context's lattice, in one
 * launch of the batched multi-right-hand-side hop (each link load serves
 * all n fields): the operator of eq. S3.1 as lgt_dslash, batched.
 * precision LGT_FP64: FP64 throughout; LGT_MIXED_FP32: the FP32 batched hop
 * of the mixed-precision batched solve (kernel per lgt_set_batch_hop_kernel)
 * on FP32 copies of U and in, its result widened to FP64 (relative error
 * ~1e-7).  in, out: n device pointers (host array) to canonical spinors;
 * kappas: n host values.  INVALID_ARGUMENT: null pointers, n outside 1..16,
 * other precisions, non-finite kappa. */
LGT_API lgt_status lgt_dslash_batch(lgt_ctx* ctx, const void* U, int32_t n, const void* const* in, void* const* out,
                                    const double* kappas, int32_t dagger, int32_t precision);

/* Kernel of the FP32 batched hop in lgt_cg_solve_batch (mixed precision)
 * and lgt_hop_benchmark_mrhs on this context: 1 = the VALU kernel (each
 * lane one site, the link applied to each right-hand side in turn), 2 = the
 * MFMA kernel (the link times the projected half spinors of a group of 4 or
 * 8 right-hand sides as a real 6 x 6 by 6 x 2G product on
 * v_mfma_f32_4x4x1_16b_f32, 16 sites per instruction), 0 (the default) =
 * whichever of them and of their group sizes the first batched call on the
 * context times fastest.  The kernels sum in different orders, so results
 * may differ by rounding.  INVALID_ARGUMENT for other values. */
LGT_API lgt_status lgt_set_batch_hop_kernel(lgt_ctx* ctx, int32_t kind);

#ifdef __cplusplus
}
#endif

#endif /* LGT_H */
