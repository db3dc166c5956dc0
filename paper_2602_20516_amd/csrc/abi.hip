// The C ABI (include/lgt.h): argument checking, layout conversion of the
// caller's canonical buffers, and the drivers that sequence the kernels.
// No C++ exception crosses this boundary.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "lgt_ctx.h"
#include "lgt_mrhs.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <thread>

using namespace lgt;

namespace {

std::string g_create_error;

// the items of one lattice in a batched solve (indices into the caller's array)
struct BatchGroup {
  lgt_ctx* ctx;
  const void* U;
  std::vector<int> idx;
};

// packed gauge scratch used here (see smear.hip): thin links, smeared output, gradient
enum { kThin = 6, kSmeared = 8, kGradIn = 9, kU0 = 10, kP0 = 11 };

template <typename F>
lgt_status guarded(lgt_ctx* ctx, F&& f) {
  try {
    if (ctx) ctx->err.clear();
    f();
    return LGT_OK;
  } catch (const Error& e) {
    if (ctx) ctx->err = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->err = "host allocation failed";
    return LGT_ERR_OUT_OF_MEMORY;
  } catch (const std::exception& e) {
    if (ctx) ctx->err = e.what();
    return LGT_ERR_DEVICE;
  } catch (...) {
    if (ctx) ctx->err = "unknown error";
    return LGT_ERR_DEVICE;
  }
}

void require(bool ok, const char* msg) {
  if (!ok) throw Error(LGT_ERR_INVALID_ARGUMENT, msg);
}

SolverOpts parse(const lgt_solver_params* p) {
  SolverOpts o;
  if (!p) return o;
  require(p->precision >= LGT_FP64 && p->precision <= LGT_MIXED_BF16, "unknown precision");
  require(p->even_odd == 1 || p->even_odd == 0, "even_odd must be 0 or 1");
  if (p->even_odd == 0) throw Error(LGT_ERR_UNSUPPORTED, "only the even/odd solver is implemented");
  require(std::isfinite(p->tol) && p->tol > 0.0, "tol must be positive");
  o.precision = p->precision;
  o.tol = p->tol;
  o.max_iter = p->max_iter > 0 ? p->max_iter : 20000;
  // defaults, from timing the force call over delta at 16^4 and 24^3x48: the
  // FP32 recursion keeps its iteration count down to a residual drop of
  // 1e-4 between updates (3e-4: two updates fewer than 1e-3, same
  // iterations); the BF16-stored one (rounding ~2^-9 per iteration) is
  // sensitive to delta, and 1e-2 was the best setting at both sizes
  const double dflt = p->precision == LGT_MIXED_BF16 ? 0.01 : 3e-4;
  o.delta = p->reliable_delta > 0.0 && p->reliable_delta < 1.0 ? p->reliable_delta : dflt;
  require(std::isfinite(p->first_pass_factor), "first_pass_factor must be finite");
  o.first_pass = p->first_pass_factor > 0.0 ? p->first_pass_factor : 0.0;
  return o;
}

void check_nonfinite(lgt_ctx* c, const char* what) {
  LGT_HIP(hipMemcpyAsync(c->host_flags, c->flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  c->sync();
  if (c->host_flags[0]) {
    LGT_HIP(hipMemsetAsync(c->flags, 0, sizeof(int), c->stream));
    throw Error(LGT_ERR_NONFINITE, std::string(what) + " holds NaN or Inf");
  }
}

void pack_links(lgt_ctx* c, const void* U, bool with32) {
  if (with32) c->ensure_u32();
  LGT_HIP(launch_pack(c->g, 36, (const double2*)U, c->U64, with32 ? c->U32 : nullptr, c->flags, c->stream));
}

void pack_spinor(lgt_ctx* c, const void* in, double2* out) {
  LGT_HIP(launch_pack(c->g, 12, (const double2*)in, out, nullptr, c->flags, c->stream));
}

void fill_stats(lgt_solver_stats* out, const SolveStats& s, double ms) {
  if (!out) return;
  out->iters = s.iters;
  out->reliable_updates = s.reliable;
  out->true_rel_residual = s.true_res;
  out->ms = ms;
  out->corrections = s.corrections;
  out->reserved = 0;
}

struct Timer {
  lgt_ctx* c;
  explicit Timer(lgt_ctx* cc) : c(cc) { LGT_HIP(hipEventRecord(c->ev0, c->stream)); }
  double stop() {
    LGT_HIP(hipEventRecord(c->ev1, c->stream));
    LGT_HIP(hipEventSynchronize(c->ev1));
    float ms = 0.f;
    LGT_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    return ms;
  }
};

double gauge_action(lgt_ctx* c, double beta, const double2* links = nullptr) {
  LGT_HIP(launch_plaquette(c->g, links ? links : c->U64, c->red(), 0, c->stream));
  c->read_results(1);
  return beta * (6.0 * (double)c->V - c->host_result[0] / 3.0);
}

void merge(SolveStats& acc, const SolveStats& s) {
  acc.iters += s.iters;
  acc.reliable += s.reliable;
  acc.corrections += s.corrections;
  acc.true_res = std::max(acc.true_res, s.true_res);
  acc.converged = acc.converged && s.converged;
}

}  // namespace

extern "C" {

lgt_status lgt_create(const lgt_geom* geom, void* hip_stream, lgt_ctx** out) {
  g_create_error.clear();
  if (!geom || !out) {
    g_create_error = "null argument";
    return LGT_ERR_INVALID_ARGUMENT;
  }
  *out = nullptr;
  for (int i = 0; i < 4; ++i) {
    if (geom->dims[i] < 2 || geom->dims[i] % 2 != 0) {
      g_create_error = "every lattice extent must be even and >= 2";
      return LGT_ERR_INVALID_ARGUMENT;
    }
  }
  if (geom->fermion_t_bc != 1 && geom->fermion_t_bc != -1) {
    g_create_error = "fermion_t_bc must be +1 or -1";
    return LGT_ERR_INVALID_ARGUMENT;
  }
  const int64_t V = (int64_t)geom->dims[0] * geom->dims[1] * geom->dims[2] * geom->dims[3];
  // kernels address a field with 32-bit byte offsets: an FP64 half-lattice
  // spinor (12 complex per site) must stay below 4 GiB
  if (V <= 0 || (int64_t)12 * (V / 2) * (int64_t)sizeof(double2) >= ((int64_t)1 << 32)) {
    g_create_error = "lattice too large (a spinor field must stay below 4 GiB: V < 44.7M sites)";
    return LGT_ERR_INVALID_ARGUMENT;
  }
  lgt_ctx* c = new (std::nothrow) lgt_ctx();
  if (!c) {
    g_create_error = "host allocation failed";
    return LGT_ERR_OUT_OF_MEMORY;
  }
  lgt_status st = guarded(c, [&] {
    for (int i = 0; i < 4; ++i) c->g.L[i] = geom->dims[i];
    c->g.hx = geom->dims[0] / 2;
    c->V = V;
    c->vh = (int)(V / 2);
    c->g.vh = c->vh;
    c->g.bc = geom->fermion_t_bc;
    c->g.hop_ns = 0;
    c->g.hop_order = 0;
    c->stream = (hipStream_t)hip_stream;
    LGT_HIP(hipGetDevice(&c->device));
    LGT_HIP(hipMalloc(&c->U64, (size_t)72 * c->vh * sizeof(double2)));
    LGT_HIP(hipMalloc(&c->state, sizeof(SolverState)));
    LGT_HIP(hipMalloc(&c->partials, (size_t)reduce_capacity(c->vh) * 4 * sizeof(double)));
    LGT_HIP(hipMalloc(&c->result, 64 * sizeof(double)));
    LGT_HIP(hipMalloc(&c->flags, 16 * sizeof(int)));
    LGT_HIP(hipHostMalloc(&c->host_result, 64 * sizeof(double), hipHostMallocDefault));
    LGT_HIP(hipHostMalloc(&c->host_flags, 16 * sizeof(int), hipHostMallocDefault));
    LGT_HIP(hipHostMalloc(&c->host_state, sizeof(SolverState), hipHostMallocDefault));
    LGT_HIP(hipHostMalloc(&c->mbox_host, sizeof(Mailbox), hipHostMallocCoherent | hipHostMallocMapped));
    LGT_HIP(hipHostGetDevicePointer((void**)&c->mbox_dev, c->mbox_host, 0));
    c->mbox_host->word = 0;
    LGT_HIP(hipMemsetAsync(c->flags, 0, 16 * sizeof(int), c->stream));
    LGT_HIP(hipMemsetAsync(c->state, 0, sizeof(SolverState), c->stream));
    LGT_HIP(hipEventCreate(&c->ev0));
    LGT_HIP(hipEventCreate(&c->ev1));
    c->sync();
  });
  if (st != LGT_OK) {
    g_create_error = c->err;
    lgt_destroy(c);
    return st;
  }
  *out = c;
  return LGT_OK;
}

lgt_status lgt_destroy(lgt_ctx* c) {
  if (!c) return LGT_OK;
  if (c->stream || c->U64) (void)hipStreamSynchronize(c->stream);
  lgt_ctx_free_batch(c);
  lgt_ctx_free_multishift(c);
  for (auto* p : c->full64) (void)hipFree(p);
  for (auto* p : c->half32) (void)hipFree(p);
  (void)hipFree(c->U64);
  (void)hipFree(c->U32);
  (void)hipFree(c->U32c);
  (void)hipFree(c->U64c);
  (void)hipFree(c->P64);
  (void)hipFree(c->state);
  (void)hipFree(c->partials);
  (void)hipFree(c->result);
  (void)hipFree(c->flags);
  if (c->host_result) (void)hipHostFree(c->host_result);
  if (c->host_flags) (void)hipHostFree(c->host_flags);
  if (c->host_state) (void)hipHostFree(c->host_state);
  if (c->mbox_host) (void)hipHostFree(c->mbox_host);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  delete c;
  return LGT_OK;
}

const char* lgt_last_error(const lgt_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

lgt_status lgt_set_stream(lgt_ctx* c, void* hip_stream) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  c->stream = (hipStream_t)hip_stream;
  return LGT_OK;
}

int64_t lgt_volume(const lgt_ctx* c) { return c ? c->V : 0; }

lgt_status lgt_dslash(lgt_ctx* c, const void* U, const void* in, void* out, double kappa, int32_t dagger) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  return guarded(c, [&] {
    require(U && in && out, "null field pointer");
    require(std::isfinite(kappa), "kappa must be finite");
    pack_links(c, U, false);
    double2* a = c->f64(kStageA);
    double2* b = c->f64(kStageB);
    pack_spinor(c, in, a);
    c->dslash_full(a, b, kappa, dagger != 0);
    LGT_HIP(launch_unpack(c->g, 12, b, (double2*)out, c->stream));
  });
}

lgt_status lgt_cg_solve(lgt_ctx* c, const void* U, const void* phi, void* X, void* Y, double kappa,
                        const lgt_solver_params* params, lgt_solver_stats* stats) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  bool nc = false;
  lgt_status s = guarded(c, [&] {
    require(U && phi && X, "null field pointer");
    require(std::isfinite(kappa), "kappa must be finite");
    const SolverOpts o = parse(params);
    Timer tm(c);
    pack_links(c, U, o.precision != LGT_FP64);
    pack_spinor(c, phi, c->f64(kPhi));
    check_nonfinite(c, "U or phi");
    c->kappa = kappa;
    SolveStats st = c->solve_ddagd(c->f64(kPhi), c->f64(kX), c->f64(kY), o);
    LGT_HIP(launch_unpack(c->g, 12, c->f64(kX), (double2*)X, c->stream));
    if (Y) LGT_HIP(launch_unpack(c->g, 12, c->f64(kY), (double2*)Y, c->stream));
    fill_stats(stats, st, tm.stop());
    nc = !st.converged;
  });
  if (s == LGT_OK && nc) {
    c->err = "solver did not reach the tolerance";
    return LGT_ERR_NOT_CONVERGED;
  }
  return s;
}

lgt_status lgt_action(lgt_ctx* c, const void* U, const void* phi, double beta, double kappa,
                      const lgt_solver_params* params, double* S_G, double* S_F, lgt_solver_stats* stats) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  bool nc = false;
  lgt_status s = guarded(c, [&] {
    require(U != nullptr, "null U");
    require(std::isfinite(kappa), "kappa must be finite");
    require(!S_F || phi, "S_F requested without phi");
    const SolverOpts o = parse(params);
    Timer tm(c);
    pack_links(c, U, o.precision != LGT_FP64 && S_F);
    if (S_F) pack_spinor(c, phi, c->f64(kPhi));
    check_nonfinite(c, "U or phi");
    if (S_G) *S_G = gauge_action(c, beta);
    SolveStats st;
    if (S_F) {
      c->kappa = kappa;
      st = c->solve_ddagd(c->f64(kPhi), c->f64(kX), c->f64(kY), o);
      *S_F = c->action_fermion(c->f64(kPhi), c->f64(kX), c->f64(kY));
    }
    fill_stats(stats, st, tm.stop());
    nc = !st.converged;
  });
  if (s == LGT_OK && nc) {
    c->err = "solver did not reach the tolerance";
    return LGT_ERR_NOT_CONVERGED;
  }
  return s;
}

lgt_status lgt_fermion_force(lgt_ctx* c, const void* U, const void* phi, double kappa,
                             const lgt_solver_params* params, int32_t mode, double dt, void* out,
                             lgt_solver_stats* stats) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  bool nc = false;
  lgt_status s = guarded(c, [&] {
    require(U && phi && out, "null field pointer");
    require(std::isfinite(kappa), "kappa must be finite");
    require(mode >= LGT_OUT_FORCE && mode <= LGT_OUT_MOMENTUM, "unknown output mode");
    const SolverOpts o = parse(params);
    Timer tm(c);
    pack_links(c, U, o.precision != LGT_FP64);
    pack_spinor(c, phi, c->f64(kPhi));
    check_nonfinite(c, "U or phi");
    c->kappa = kappa;
    SolveStats st = c->solve_ddagd(c->f64(kPhi), c->f64(kX), c->f64(kY), o);
    LGT_HIP(launch_bilinear_force(c->g, c->U64, c->f64(kY), c->f64(kX), kappa, -2.0, mode, dt, out, kCanonical,
                                  c->stream));
    fill_stats(stats, st, tm.stop());
    nc = !st.converged;
  });
  if (s == LGT_OK && nc) {
    c->err = "solver did not reach the tolerance";
    return LGT_ERR_NOT_CONVERGED;
  }
  return s;
}

lgt_status lgt_bilinear_force(lgt_ctx* c, const void* U, const void* a, const void* b, double kappa, double coeff,
                              int32_t mode, double dt, void* out) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  return guarded(c, [&] {
    require(U && a && b && out, "null field pointer");
    require(std::isfinite(kappa), "kappa must be finite");
    require(mode >= LGT_OUT_FORCE && mode <= LGT_OUT_MOMENTUM, "unknown output mode");
    pack_links(c, U, false);
    pack_spinor(c, a, c->f64(kStageA));
    pack_spinor(c, b, c->f64(kStageB));
    LGT_HIP(launch_bilinear_force(c->g, c->U64, c->f64(kStageA), c->f64(kStageB), kappa, coeff, mode, dt, out,
                                  kCanonical, c->stream));
  });
}

lgt_status lgt_gauge_force(lgt_ctx* c, const void* U, double beta, int32_t mode, double dt, void* out) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  return guarded(c, [&] {
    require(U && out, "null field pointer");
    require(mode >= LGT_OUT_FORCE && mode <= LGT_OUT_MOMENTUM, "unknown output mode");
    pack_links(c, U, false);
    LGT_HIP(launch_gauge_force(c->g, c->U64, beta, mode, dt, out, kCanonical, c->stream));
  });
}

lgt_status lgt_link_update(lgt_ctx* c, void* U, const void* P, double dt) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  return guarded(c, [&] {
    require(U && P, "null field pointer");
    LGT_HIP(launch_link_update(c->g, (double2*)U, (const double2*)P, dt, kCanonical, nullptr, c->stream));
  });
}

lgt_status lgt_momenta_from_normals(lgt_ctx* c, const void* normals, void* P) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  return guarded(c, [&] {
    require(normals && P, "null pointer");
    LGT_HIP(launch_momenta(c->g, (const double*)normals, (double2*)P, c->stream));
  });
}

lgt_status lgt_kinetic(lgt_ctx* c, const void* P, double* K) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  return guarded(c, [&] {
    require(P && K, "null pointer");
    LGT_HIP(launch_kinetic(c->g, (const double2*)P, kCanonical, c->red(), 0, c->stream));
    c->read_results(1);
    *K = c->host_result[0];
  });
}

// Leapfrog with merged half-kicks (Sec. III B), nlevels = 0: plain action,
// nlevels > 0: stout-smeared fermion action.  n_inner > 1: Sexton-Weingarten
// multiple time-scale integrator (Sec. III B): the fermion force on the outer
// scale dt, the gauge force on n_inner leapfrog sub-steps of dt / n_inner.
static lgt_status md_run(lgt_ctx* c, void* U, void* P, const void* phi, double beta, double kappa, double rho,
                         int32_t nlevels, double dt, int32_t nsteps, int32_t n_inner,
                         const lgt_solver_params* params, double* dH, lgt_solver_stats* stats, bool eo = false) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  bool nc = false;
  lgt_status s = guarded(c, [&] {
    require(U && P, "null field pointer");
    require(nsteps >= 1, "nsteps must be >= 1");
    require(nlevels >= 0 && nlevels <= kMaxStoutLevels, "nlevels must be in 0..256");
    require(n_inner >= 1, "n_inner must be >= 1");
    require(std::isfinite(dt) && std::isfinite(rho) && std::isfinite(kappa) && std::isfinite(beta),
            "dt, rho, kappa and beta must be finite");
    const SolverOpts o = parse(params);
    const bool ferm = phi != nullptr && kappa != 0.0;
    const bool mixed = ferm && o.precision != LGT_FP64;
    const bool smeared = ferm && nlevels > 0;
    require(!(eo && nlevels > 0), "the even/odd-preconditioned action is implemented for thin links only");
    Timer tm(c);
    c->ensure_p64();
    // thin links: U64 for the plain action; a separate field when smearing
    // (U64 then holds the smeared links the solver runs on)
    double2* thin = smeared ? c->g64(kThin) : c->U64;
    if (smeared) LGT_HIP(launch_pack(c->g, 36, (const double2*)U, thin, nullptr, c->flags, c->stream));
    else pack_links(c, U, mixed);
    LGT_HIP(launch_pack(c->g, 36, (const double2*)P, c->P64, nullptr, c->flags, c->stream));
    if (ferm) pack_spinor(c, phi, c->f64(kPhi));
    check_nonfinite(c, "U, P or phi");
    c->kappa = kappa;
    SolveStats all;
    double sf0 = 0.0, sf1 = 0.0;

    // start of the trajectory, kept for the per-site differences of K and S_G
    double2* u0 = dH ? c->g64(kU0) : nullptr;
    double2* p0 = dH ? c->g64(kP0) : nullptr;
    if (dH) {
      LGT_HIP(launch_copy64(72 * c->vh, thin, u0, c->stream));
      LGT_HIP(launch_copy64(72 * c->vh, c->P64, p0, c->stream));
    }

    // plain (or even/odd-preconditioned) pseudofermion force kick at the thin links
    auto fermion_kick = [&](double h, double* sfp) {
      if (eo) {
        merge(all, c->solve_eo(c->f64(kPhi), c->f64(kX), c->f64(kY), o));
        if (sfp) *sfp = c->action_eo(c->f64(kPhi), c->f64(kX), c->f64(kY));
        LGT_HIP(launch_bilinear_force(c->g, thin, c->f64(kY), c->f64(kX), kappa, -2.0 * kappa, LGT_OUT_MOMENTUM, h,
                                      c->P64, kPacked, c->stream));
        return;
      }
      merge(all, c->solve_ddagd(c->f64(kPhi), c->f64(kX), c->f64(kY), o));
      if (sfp) *sfp = c->action_fermion(c->f64(kPhi), c->f64(kX), c->f64(kY));
      LGT_HIP(launch_bilinear_force(c->g, thin, c->f64(kY), c->f64(kX), kappa, -2.0, LGT_OUT_MOMENTUM, h, c->P64,
                                    kPacked, c->stream));
    };
    auto kick = [&](double h, bool first, bool last) {
      double* sfp = first ? &sf0 : (last ? &sf1 : nullptr);
      if (smeared) {
        SolveStats st = c->smeared_force(thin, c->f64(kPhi), beta, rho, nlevels, o, LGT_OUT_MOMENTUM, h, c->P64,
                                         kPacked, sfp);
        merge(all, st);
        return;
      }
      LGT_HIP(launch_gauge_force(c->g, thin, beta, LGT_OUT_MOMENTUM, h, c->P64, kPacked, c->stream));
      if (!ferm) return;
      fermion_kick(h, sfp);
    };
    float2* u32 = (mixed && !smeared) ? c->U32 : nullptr;  // the FP32 copy the inner solver reads
    if (n_inner == 1) {
      kick(0.5 * dt, true, nsteps == 0);
      for (int k = 0; k < nsteps; ++k) {
        LGT_HIP(launch_link_update(c->g, thin, c->P64, dt, kPacked, u32, c->stream));
        const bool last = k == nsteps - 1;
        kick(last ? 0.5 * dt : dt, false, last);
      }
    } else {
      // fermion part alone (beta = 0 removes the gauge term of the smeared force)
      auto kick_fermion = [&](double h, double* sfp) {
        if (!ferm) return;
        if (smeared) {
          merge(all, c->smeared_force(thin, c->f64(kPhi), 0.0, rho, nlevels, o, LGT_OUT_MOMENTUM, h, c->P64,
                                      kPacked, sfp));
          return;
        }
        fermion_kick(h, sfp);
      };
      auto kick_gauge = [&](double h) {
        LGT_HIP(launch_gauge_force(c->g, thin, beta, LGT_OUT_MOMENTUM, h, c->P64, kPacked, c->stream));
      };
      const double hi = dt / n_inner;
      for (int k = 0; k < nsteps; ++k) {
        kick_fermion(k == 0 ? 0.5 * dt : dt, k == 0 ? &sf0 : nullptr);  // adjacent outer half-kicks merged
        kick_gauge(0.5 * hi);
        for (int j = 0; j < n_inner; ++j) {
          LGT_HIP(launch_link_update(c->g, thin, c->P64, hi, kPacked, u32, c->stream));
          kick_gauge(j < n_inner - 1 ? hi : 0.5 * hi);
        }
      }
      kick_fermion(0.5 * dt, &sf1);
    }
    if (dH) {
      // Delta K and Delta S_G as sums of per-link / per-site differences:
      // their rounding error scales with Delta H, not with K or S_G
      LGT_HIP(launch_kinetic(c->g, c->P64, kPacked, c->red(), 0, c->stream, p0));
      LGT_HIP(launch_plaquette(c->g, thin, c->red(), 1, c->stream, u0));
      c->read_results(2);
      const double dk = c->host_result[0];
      const double dsg = -beta / 3.0 * c->host_result[1];
      *dH = dk + dsg + (sf1 - sf0);
    }
    LGT_HIP(launch_unpack(c->g, 36, thin, (double2*)U, c->stream));
    LGT_HIP(launch_unpack(c->g, 36, c->P64, (double2*)P, c->stream));
    fill_stats(stats, all, tm.stop());
    nc = !all.converged;
  });
  if (s == LGT_OK && nc) {
    c->err = "solver did not reach the tolerance";
    return LGT_ERR_NOT_CONVERGED;
  }
  return s;
}

lgt_status lgt_md_step(lgt_ctx* c, void* U, void* P, const void* phi, double beta, double kappa, double dt,
                       int32_t nsteps, const lgt_solver_params* params, double* dH, lgt_solver_stats* stats) {
  return md_run(c, U, P, phi, beta, kappa, 0.0, 0, dt, nsteps, 1, params, dH, stats);
}

lgt_status lgt_md_step_smeared(lgt_ctx* c, void* U, void* P, const void* phi, double beta, double kappa,
                               double rho, int32_t nlevels, double dt, int32_t nsteps,
                               const lgt_solver_params* params, double* dH, lgt_solver_stats* stats) {
  return md_run(c, U, P, phi, beta, kappa, rho, nlevels, dt, nsteps, 1, params, dH, stats);
}

lgt_status lgt_md_step_eo(lgt_ctx* c, void* U, void* P, const void* phi, double beta, double kappa, double dt,
                          int32_t nsteps, int32_t n_inner, const lgt_solver_params* params, double* dH,
                          lgt_solver_stats* stats) {
  return md_run(c, U, P, phi, beta, kappa, 0.0, 0, dt, nsteps, n_inner, params, dH, stats, true);
}

lgt_status lgt_schur_dslash(lgt_ctx* c, const void* U, const void* in, void* out, double kappa, int32_t dagger) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  return guarded(c, [&] {
    require(U && in && out, "null field pointer");
    require(std::isfinite(kappa), "kappa must be finite");
    pack_links(c, U, false);
    double2* a = c->f64(kStageA);
    double2* b = c->f64(kStageB);
    pack_spinor(c, in, a);
    const size_t h = c->half_elems();
    const HopIn<double> ha{c->U64, a, a + h};
    const HopIn<double> hb{c->U64, b, b + h};
    // Mhat: H_eo then H_oe;  Mhat^dag: (H^dag)_eo then (H^dag)_oe
    if (dagger) {
      LGT_HIP((launch_hop_axpy<double, true>(c->g, 0, ha, b, b, nullptr, nullptr, 1.0, c->stream)));
      LGT_HIP((launch_hop_axpy<double, true>(c->g, 1, hb, b, b + h, nullptr, a + h, -kappa * kappa, c->stream)));
    } else {
      LGT_HIP((launch_hop_axpy<double, false>(c->g, 0, ha, b, b, nullptr, nullptr, 1.0, c->stream)));
      LGT_HIP((launch_hop_axpy<double, false>(c->g, 1, hb, b, b + h, nullptr, a + h, -kappa * kappa, c->stream)));
    }
    LGT_HIP(launch_zero64((int)h, b, c->stream));
    LGT_HIP(launch_unpack(c->g, 12, b, (double2*)out, c->stream));
  });
}

lgt_status lgt_fermion_force_eo(lgt_ctx* c, const void* U, const void* phi, double kappa,
                                const lgt_solver_params* params, int32_t mode, double dt, void* out,
                                double* S_F_or_null, lgt_solver_stats* stats) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  bool nc = false;
  lgt_status s = guarded(c, [&] {
    require(U && phi && out, "null field pointer");
    require(std::isfinite(kappa), "kappa must be finite");
    require(mode >= LGT_OUT_FORCE && mode <= LGT_OUT_MOMENTUM, "unknown output mode");
    const SolverOpts o = parse(params);
    Timer tm(c);
    pack_links(c, U, o.precision != LGT_FP64);
    pack_spinor(c, phi, c->f64(kPhi));
    check_nonfinite(c, "U or phi");
    c->kappa = kappa;
    SolveStats st = c->solve_eo(c->f64(kPhi), c->f64(kX), c->f64(kY), o);
    if (S_F_or_null) *S_F_or_null = c->action_eo(c->f64(kPhi), c->f64(kX), c->f64(kY));
    LGT_HIP(launch_bilinear_force(c->g, c->U64, c->f64(kY), c->f64(kX), kappa, -2.0 * kappa, mode, dt, out,
                                  kCanonical, c->stream));
    fill_stats(stats, st, tm.stop());
    nc = !st.converged;
  });
  if (s == LGT_OK && nc) {
    c->err = "solver did not reach the tolerance";
    return LGT_ERR_NOT_CONVERGED;
  }
  return s;
}

lgt_status lgt_md_step_sw(lgt_ctx* c, void* U, void* P, const void* phi, double beta, double kappa, double rho,
                          int32_t nlevels, double dt, int32_t nsteps, int32_t n_inner, const lgt_solver_params* params,
                          double* dH, lgt_solver_stats* stats) {
  return md_run(c, U, P, phi, beta, kappa, rho, nlevels, dt, nsteps, n_inner, params, dH, stats);
}

lgt_status lgt_stout_smear(lgt_ctx* c, const void* U_in, void* U_out, double rho, int32_t nlevels) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  return guarded(c, [&] {
    require(U_in && U_out, "null field pointer");
    require(nlevels >= 0 && nlevels <= kMaxStoutLevels && std::isfinite(rho), "invalid smearing parameters");
    double2* thin = c->g64(kThin);
    double2* out = c->g64(kSmeared);
    LGT_HIP(launch_pack(c->g, 36, (const double2*)U_in, thin, nullptr, c->flags, c->stream));
    c->smear(thin, nlevels, rho, out);
    LGT_HIP(launch_unpack(c->g, 36, out, (double2*)U_out, c->stream));
  });
}

lgt_status lgt_stout_backprop(lgt_ctx* c, const void* U_in, const void* G_top, double rho, int32_t nlevels,
                              void* G_out) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  return guarded(c, [&] {
    require(U_in && G_top && G_out, "null field pointer");
    require(nlevels >= 0 && nlevels <= kMaxStoutLevels && std::isfinite(rho), "invalid smearing parameters");
    double2* thin = c->g64(kThin);
    double2* G = c->g64(kGradIn);
    LGT_HIP(launch_pack(c->g, 36, (const double2*)U_in, thin, nullptr, c->flags, c->stream));
    LGT_HIP(launch_pack(c->g, 36, (const double2*)G_top, G, nullptr, c->flags, c->stream));
    c->stout_backprop(thin, nlevels, rho, G, c->stout_plan(nlevels), false);
    LGT_HIP(launch_unpack(c->g, 36, G, (double2*)G_out, c->stream));
  });
}

lgt_status lgt_smeared_force(lgt_ctx* c, const void* U, const void* phi, double beta, double kappa, double rho,
                             int32_t nlevels, const lgt_solver_params* params, int32_t mode, double dt, void* out,
                             double* S_F, lgt_solver_stats* stats) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  bool nc = false;
  lgt_status s = guarded(c, [&] {
    require(U && phi && out, "null field pointer");
    require(std::isfinite(kappa), "kappa must be finite");
    require(mode >= LGT_OUT_FORCE && mode <= LGT_OUT_MOMENTUM, "unknown output mode");
    require(nlevels >= 0 && nlevels <= kMaxStoutLevels && std::isfinite(rho), "invalid smearing parameters");
    const SolverOpts o = parse(params);
    Timer tm(c);
    double2* thin = c->g64(kThin);
    LGT_HIP(launch_pack(c->g, 36, (const double2*)U, thin, nullptr, c->flags, c->stream));
    pack_spinor(c, phi, c->f64(kPhi));
    check_nonfinite(c, "U or phi");
    c->kappa = kappa;
    SolveStats st = c->smeared_force(thin, c->f64(kPhi), beta, rho, nlevels, o, mode, dt, out, kCanonical, S_F);
    fill_stats(stats, st, tm.stop());
    nc = !st.converged;
  });
  if (s == LGT_OK && nc) {
    c->err = "solver did not reach the tolerance";
    return LGT_ERR_NOT_CONVERGED;
  }
  return s;
}

lgt_status lgt_set_stout_checkpoints(lgt_ctx* c, int32_t max_stored_levels) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  return guarded(c, [&] {
    require(max_stored_levels >= -1, "max_stored_levels must be -1 (automatic) or >= 0");
    c->stout_slot_cap = max_stored_levels;
  });
}

lgt_status lgt_set_hop_block_sites(lgt_ctx* c, int32_t sites) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  return guarded(c, [&] {
    require(sites == 0 || sites == 32 || sites == 64, "hop block sites must be 0 (automatic), 32 or 64");
    // the 32-site kernel addresses both parities' links through one buffer
    // resource with 32-bit offsets
    require(sites != 32 || (size_t)72 * c->vh * sizeof(double2) < ((size_t)1 << 32),
            "32-site hop blocks need a gauge field below 4 GiB (V at most 7456540 sites)");
    c->g.hop_ns = sites;
  });
}

lgt_status lgt_set_hop_block_order(lgt_ctx* c, int32_t order) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  return guarded(c, [&] {
    require(order == 0 || order == 1 || order == 2, "hop block order must be 0 (automatic), 1 or 2");
    c->g.hop_order = order;
  });
}

lgt_status lgt_dslash_batch(lgt_ctx* c, const void* U, int32_t n, const void* const* in, void* const* out,
                            const double* kappas, int32_t dagger, int32_t precision) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  return guarded(c, [&] {
    require(U && in && out && kappas, "null pointer");
    require(n >= 1 && n <= 16, "a batch holds 1 to 16 fields");
    require(precision == LGT_FP64 || precision == LGT_MIXED_FP32, "precision must be LGT_FP64 or LGT_MIXED_FP32");
    require((size_t)12 * c->vh * n * sizeof(double2) < ((size_t)1 << 32),
            "batch too large: the batched spinor field must stay below 4 GiB");
    for (int k = 0; k < n; ++k) {
      require(in[k] && out[k], "null field pointer");
      require(std::isfinite(kappas[k]), "kappa must be finite");
    }
    const bool f32 = precision == LGT_MIXED_FP32;
    pack_links(c, U, f32);
    c->dslash_batch(n, kappas, in, out, dagger != 0, f32);
  });
}

lgt_status lgt_set_batch_hop_kernel(lgt_ctx* c, int32_t kind) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  return guarded(c, [&] {
    require(kind == 0 || kind == 1 || kind == 2, "batched hop kernel must be 0 (timed choice), 1 (VALU) or 2 (MFMA)");
    c->batch_hop_kind = kind;
  });
}

lgt_status lgt_stout_last_schedule(const lgt_ctx* c, int32_t* stored_levels, int64_t* recompute_passes) {
  if (!c || !stored_levels || !recompute_passes) return LGT_ERR_INVALID_ARGUMENT;
  *stored_levels = c->last_stout_slots;
  *recompute_passes = c->last_stout_passes;
  return LGT_OK;
}

lgt_status lgt_stout_schedule(int32_t nlevels, int32_t stored_levels, int64_t* recompute_passes,
                              int32_t* checkpoints_or_null, int32_t* n_checkpoints_or_null) {
  if (!recompute_passes || nlevels < 0 || nlevels > kMaxStoutLevels || stored_levels < 0)
    return LGT_ERR_INVALID_ARGUMENT;
  try {
    const StoutSchedule plan(nlevels, stored_levels);
    *recompute_passes = plan.cost();
    const std::vector<int> cp = plan.forward_checkpoints();
    if (checkpoints_or_null)
      for (size_t i = 0; i < cp.size(); ++i) checkpoints_or_null[i] = cp[i];
    if (n_checkpoints_or_null) *n_checkpoints_or_null = (int32_t)cp.size();
  } catch (...) {
    return LGT_ERR_OUT_OF_MEMORY;
  }
  return LGT_OK;
}

lgt_status lgt_batch_create(void* hip_stream, lgt_batch** out) {
  if (!out) return LGT_ERR_INVALID_ARGUMENT;
  lgt_batch* b = new (std::nothrow) lgt_batch();
  if (!b) return LGT_ERR_OUT_OF_MEMORY;
  b->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return LGT_ERR_DEVICE;
  }
  *out = b;
  return LGT_OK;
}

lgt_status lgt_batch_destroy(lgt_batch* b) {
  if (!b) return LGT_OK;
  for (auto s : b->side) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  for (auto e : b->events) (void)hipEventDestroy(e);
  delete b;
  return LGT_OK;
}

const char* lgt_batch_last_error(const lgt_batch* b) { return b ? b->err.c_str() : ""; }

lgt_status lgt_batch_set_stream(lgt_batch* b, void* hip_stream) {
  if (!b) return LGT_ERR_INVALID_ARGUMENT;
  b->stream = (hipStream_t)hip_stream;
  return LGT_OK;
}

lgt_status lgt_cg_solve_batch(lgt_batch* b, int32_t n, const lgt_batch_item* items,
                              const lgt_solver_params* params, lgt_solver_stats* stats) {
  if (!b) return LGT_ERR_INVALID_ARGUMENT;
  b->err.clear();
  auto fail = [&](lgt_status s, const std::string& m) {
    b->err = m;
    return s;
  };
  if (!items || n < 1) return fail(LGT_ERR_INVALID_ARGUMENT, "null items or n < 1");
  // group the items by lattice (context), in order of first appearance
  std::vector<BatchGroup> groups;
  for (int k = 0; k < n; ++k) {
    const lgt_batch_item& it = items[k];
    if (!it.ctx || !it.U || !it.phi || !it.X) return fail(LGT_ERR_INVALID_ARGUMENT, "null pointer in a batch item");
    if (!std::isfinite(it.kappa)) return fail(LGT_ERR_INVALID_ARGUMENT, "kappa must be finite");
    auto g = std::find_if(groups.begin(), groups.end(), [&](const BatchGroup& x) { return x.ctx == it.ctx; });
    if (g == groups.end()) {
      groups.push_back(BatchGroup{it.ctx, it.U, {}});
      g = groups.end() - 1;
    }
    if (g->U != it.U) return fail(LGT_ERR_INVALID_ARGUMENT, "two gauge fields for one context in a batch");
    g->idx.push_back(k);
  }
  if (groups.size() > 8) return fail(LGT_ERR_INVALID_ARGUMENT, "a batch spans at most 8 lattices (contexts)");
  for (const auto& g : groups) {
    if (g.idx.size() > 16) return fail(LGT_ERR_INVALID_ARGUMENT, "at most 16 right-hand sides per lattice");
    if (g.ctx->device != b->device) return fail(LGT_ERR_INVALID_ARGUMENT, "a context on another device");
  }
  if (params && params->precision == LGT_MIXED_BF16)
    return fail(LGT_ERR_UNSUPPORTED, "the batched solve has no BF16-storage variant (use LGT_MIXED_FP32)");
  try {
    (void)parse(params);
  } catch (const Error& e) {
    return fail(e.status, e.what());
  }
  const size_t ng = groups.size();
  try {
    while (b->side.size() < ng) {
      hipStream_t s = nullptr;
      LGT_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      b->side.push_back(s);
    }
    while (b->events.size() < ng + 1) {
      hipEvent_t e = nullptr;
      LGT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      b->events.push_back(e);
    }
    // the lattices' streams start after the work already on the caller's stream
    LGT_HIP(hipEventRecord(b->events[ng], b->stream));
    for (size_t g = 0; g < ng; ++g) LGT_HIP(hipStreamWaitEvent(b->side[g], b->events[ng], 0));
  } catch (const Error& e) {
    return fail(e.status, e.what());
  }
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<lgt_status> st(ng, LGT_OK);
  std::vector<std::string> msg(ng);
  std::vector<std::vector<SolveStats>> res(ng);
  auto run_group = [&](size_t g) {
    lgt_ctx* c = groups[g].ctx;
    const hipStream_t own = c->stream;
    c->stream = b->side[g];
    st[g] = guarded(c, [&] {
      const int m = (int)groups[g].idx.size();
      require((size_t)12 * c->vh * m * sizeof(double2) < ((size_t)1 << 32),
              "batch too large: the batched spinor field must stay below 4 GiB (use fewer right-hand sides)");
      std::vector<double> kap(m);
      std::vector<const void*> phis(m);
      std::vector<void*> xs(m), ys(m);
      for (int k = 0; k < m; ++k) {
        const lgt_batch_item& it = items[groups[g].idx[k]];
        kap[k] = it.kappa;
        phis[k] = it.phi;
        xs[k] = it.X;
        ys[k] = it.Y_or_null;
      }
      const SolverOpts o = parse(params);
      pack_links(c, groups[g].U, o.precision != LGT_FP64);
      check_nonfinite(c, "U");
      res[g] = c->solve_batch(m, kap.data(), phis.data(), xs.data(), ys.data(), o);
    });
    if (st[g] != LGT_OK) msg[g] = c->err;
    c->stream = own;
  };
  // one host thread per further lattice: each drives its lattice's solve
  // (the CG control loops wait on the device), so the lattices' kernels
  // overlap on the GPU
  std::vector<std::thread> th;
  for (size_t g = 1; g < ng; ++g) th.emplace_back(run_group, g);
  run_group(0);
  for (auto& t : th) t.join();
  lgt_status out = LGT_OK;
  try {
    for (size_t g = 0; g < ng; ++g) {
      LGT_HIP(hipEventRecord(b->events[g], b->side[g]));
      LGT_HIP(hipStreamWaitEvent(b->stream, b->events[g], 0));
    }
    LGT_HIP(hipStreamSynchronize(b->stream));
  } catch (const Error& e) {
    return fail(e.status, e.what());
  }
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  bool nc = false;
  for (size_t g = 0; g < ng; ++g) {
    if (st[g] != LGT_OK) {
      if (out == LGT_OK) {
        out = st[g];
        char head[64];
        std::snprintf(head, sizeof head, "lattice %d (%dx%dx%dx%d): ", (int)g, groups[g].ctx->g.L[0],
                      groups[g].ctx->g.L[1], groups[g].ctx->g.L[2], groups[g].ctx->g.L[3]);
        b->err = head + msg[g];
      }
      continue;
    }
    for (size_t k = 0; k < groups[g].idx.size(); ++k) {
      fill_stats(stats ? stats + groups[g].idx[k] : nullptr, res[g][k], ms);
      nc = nc || !res[g][k].converged;
    }
  }
  if (out == LGT_OK && nc) return fail(LGT_ERR_NOT_CONVERGED, "solver did not reach the tolerance for every right-hand side");
  return out;
}

lgt_status lgt_cg_solve_multishift(lgt_ctx* c, const void* U, const void* phi, double kappa, int32_t nshift,
                                   const double* shifts, void* const* X, const lgt_solver_params* params,
                                   lgt_solver_stats* stats) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  bool nc = false;
  lgt_status s = guarded(c, [&] {
    require(U && phi && shifts && X, "null pointer");
    require(nshift >= 1 && nshift <= lgt_ctx_max_shifts(), "nshift out of range (1 to 32)");
    require(std::isfinite(kappa), "kappa must be finite");
    for (int i = 0; i < nshift; ++i) {
      require(std::isfinite(shifts[i]) && shifts[i] >= 0.0, "shifts must be finite and non-negative");
      require(X[i] != nullptr, "null output field");
    }
    const SolverOpts o = parse(params);
    if (o.precision != LGT_FP64) throw Error(LGT_ERR_UNSUPPORTED, "the multi-shift solve runs in FP64 only");
    Timer tm(c);
    pack_links(c, U, false);
    pack_spinor(c, phi, c->f64(kPhi));
    check_nonfinite(c, "U or phi");
    c->kappa = kappa;
    const SolveStats st = c->solve_multishift(c->f64(kPhi), nshift, shifts, X, o);
    fill_stats(stats, st, tm.stop());
    nc = !st.converged;
  });
  if (s == LGT_OK && nc) {
    c->err = "solver did not reach the tolerance for every shift";
    return LGT_ERR_NOT_CONVERGED;
  }
  return s;
}

lgt_status lgt_rational_force_eo(lgt_ctx* c, const void* U, const void* phi, double kappa, int32_t nterms,
                                 const double* shifts, const double* residues, double a0,
                                 const lgt_solver_params* params, int32_t mode, double dt, void* out,
                                 double* S_or_null, lgt_solver_stats* stats) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  bool nc = false;
  lgt_status s = guarded(c, [&] {
    require(U && phi && shifts && residues && out, "null pointer");
    require(nterms >= 1 && nterms <= lgt_ctx_max_shifts(), "nterms out of range (1 to 32)");
    require(mode >= LGT_OUT_FORCE && mode <= LGT_OUT_MOMENTUM, "unknown output mode");
    require(std::isfinite(kappa) && std::isfinite(a0) && std::isfinite(dt), "kappa, a0 and dt must be finite");
    for (int i = 0; i < nterms; ++i) {
      require(std::isfinite(shifts[i]) && shifts[i] >= 0.0, "shifts must be finite and non-negative");
      require(std::isfinite(residues[i]), "residues must be finite");
    }
    const SolverOpts o = parse(params);
    if (o.precision != LGT_FP64) throw Error(LGT_ERR_UNSUPPORTED, "the rational force runs in FP64 only");
    Timer tm(c);
    pack_links(c, U, false);
    pack_spinor(c, phi, c->f64(kPhi));
    check_nonfinite(c, "U or phi");
    c->kappa = kappa;
    const SolveStats st = c->rational_force(c->f64(kPhi), nterms, shifts, residues, a0, o, mode, dt, out, S_or_null);
    fill_stats(stats, st, tm.stop());
    nc = !st.converged;
  });
  if (s == LGT_OK && nc) {
    c->err = "solver did not reach the tolerance for every shift";
    return LGT_ERR_NOT_CONVERGED;
  }
  return s;
}

lgt_status lgt_hop_benchmark(lgt_ctx* c, const void* U, const void* psi, int32_t precision, int32_t nrep,
                             double* avg_ms) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  return guarded(c, [&] {
    require(U && psi && avg_ms && nrep >= 1, "invalid argument");
    const bool f32 = precision != LGT_FP64;
    pack_links(c, U, f32);
    double2* a = c->f64(kStageA);
    double2* b = c->f64(kStageB);
    pack_spinor(c, psi, a);
    const size_t h = c->half_elems();
    float2* a32 = nullptr;
    float2* b32 = nullptr;
    if (f32) {
      a32 = c->h32(5);
      b32 = c->h32(6);
      LGT_HIP(launch_convert_64_32((int)h, a + h, a32, c->stream));
    }
    // the links in the form the CG hops read them (two rows when they are SU(3))
    int nk = 9;
    if (f32) c->compress_links();
    else c->compress_links64();
    c->sync();
    if (c->host_flags[f32 ? 1 : 2] == 0) nk = 6;
    auto once = [&] {
      if (f32) {
        HopIn<float> hin{nk == 6 ? c->U32c : c->U32, a32, a32, nk};
        LGT_HIP((launch_hop_axpy<float, false>(c->g, 0, hin, b32, b32, nullptr, nullptr, 1.0, c->stream)));
      } else {
        HopIn<double> hin{nk == 6 ? c->U64c : c->U64, a + h, a + h, nk};
        LGT_HIP((launch_hop_axpy<double, false>(c->g, 0, hin, b, b, nullptr, nullptr, 1.0, c->stream)));
      }
    };
    once();  // warm-up
    Timer tm(c);
    for (int i = 0; i < nrep; ++i) once();
    *avg_ms = tm.stop() / nrep;
  });
}

lgt_status lgt_hop_benchmark_mrhs(lgt_ctx* c, const void* U, const void* psi, int32_t nrhs, int32_t precision,
                                  int32_t nrep, double* avg_ms) {
  if (!c) return LGT_ERR_INVALID_ARGUMENT;
  return guarded(c, [&] {
    require(U && psi && avg_ms && nrep >= 1, "invalid argument");
    require(nrhs >= 1 && nrhs <= kMaxRhs, "nrhs must be in [1, 16]");
    require((size_t)12 * c->vh * nrhs * sizeof(double2) < ((size_t)1 << 32), "batched field above 4 GiB");
    const bool f32 = precision != LGT_FP64;
    pack_links(c, U, f32);
    *avg_ms = c->bench_mhop(nrhs, f32, psi, nrep);
  });
}

}  // extern "C"

void lgt_set_global_error(const std::string& msg) { g_create_error = msg; }
