// Multi-right-hand-side kernels: NR spinor fields on one lattice, solved
// together (one pseudofermion per right-hand side, each with its own kappa).
//
// Layout of a multi-RHS half field: [12 components][V/2 sites][NR] complex,
// right-hand side fastest, so the NR threads of one site read one link and
// NR consecutive spinor values: the link traffic is paid once for all NR
// solves (the point of batching; the Schur operator is kappa-independent up
// to the per-RHS factor kappa_n^2 applied in the epilogue).
//
// Work decomposition as in the single-field hop: a 256-thread block owns 64
// consecutive (site, right-hand side) pairs, pair q -> site q / NR, RHS
// q % NR; wave w (= direction mu) computes both hops along mu for the 64
// pairs, the partial spinors meet in LDS and wave w then owns spin w of the
// 64 pairs.  Per-RHS reductions are deterministic: block sums per n in a
// fixed order, one partial per (block, n), summed by a one-block finalize
// launch.
#include "lgt_internal.h"
#include "lgt_hop.h"
#include "lgt_mrhs.h"

namespace lgt {

// ---------------------------------------------------------------------------
// Epilogues (element (k, cb, n) of the hop result).
// ---------------------------------------------------------------------------
template <typename R>
struct MEpiAxpy {  // out = self + coef_n * acc
  static constexpr bool kReduce = false;
  R2<R>* out[2];
  const R2<R>* self[2];
  const double* coef;  // [NR] device array
  const BatchState* guard;
  const double* pap_partials;  // block 0 forms alpha_n (see tail)
  int pap_nblk;
  BatchState* state;
  __device__ bool skip() const { return guard && guard->all_done; }
  __device__ void apply(int p, size_t o, int n, C<R> a, double&) const {
    C<R> v = R(coef[n]) * a;
    if (self[p]) v += ld<R>(self[p] + o);
    st<R>(out[p] + o, v);
  }
  __device__ void tail(int nr) const {
    if (!pap_partials || blockIdx.x != 0) return;
    __shared__ double sh[4];
    for (int n = 0; n < nr; ++n) {
      double s = 0.0;
      for (int i = threadIdx.x; i < pap_nblk; i += 256) s += pap_partials[(size_t)i * kMaxRhs + n];
      const double tot = block_sum<256>(s, sh);
      if (threadIdx.x == 0 && !state->done[n]) {
        state->pap[n] = tot;
        if (!(tot > 0.0) || !isfinite(tot)) {
          state->alpha[n] = 0.0;
          state->done[n] = kDoneBreakdown;
        } else {
          state->alpha[n] = state->rr[n] / tot;
        }
      }
    }
  }
};

template <typename R>
struct MEpiSchurNorm {  // w = x + coef_n acc, per-RHS |w|^2
  static constexpr bool kReduce = true;
  R2<R>* w;
  const R2<R>* x;
  const double* coef;
  const BatchState* state;
  __device__ bool skip() const { return state->all_done; }
  __device__ void apply(int, size_t o, int n, C<R> a, double& red) const {
    const C<R> v = ld<R>(x + o) + R(coef[n]) * a;
    st<R>(w + o, v);
    red += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
  }
  __device__ void tail(int) const {}
};

template <typename R>
struct MEpiSchurCG {  // q = w + coef_n acc; x += alpha_n p; r -= alpha_n q (unless converged)
  static constexpr bool kReduce = true;
  const R2<R>* w;
  R2<R>* x;
  R2<R>* r;
  const R2<R>* p;
  const double* coef;
  const BatchState* state;
  __device__ bool skip() const { return state->all_done; }
  __device__ void apply(int, size_t o, int n, C<R> a, double& red) const {
    C<R> rv = ld<R>(r + o);
    if (!state->done[n]) {
      const R alpha = R(state->alpha[n]);
      const C<R> q = ld<R>(w + o) + R(coef[n]) * a;
      st<R>(x + o, ld<R>(x + o) + alpha * ld<R>(p + o));
      rv = rv - alpha * q;
      st<R>(r + o, rv);
    }
    red += (double)rv.re * (double)rv.re + (double)rv.im * (double)rv.im;
  }
  __device__ void tail(int) const {}
};

struct MEpiResidual {  // r = phi - (self + coef_n acc), per-RHS |r|^2 (both parities, FP64)
  static constexpr bool kReduce = true;
  const double2* self[2];
  const double2* phi[2];
  double2* r[2];
  const double* coef;
  __device__ bool skip() const { return false; }
  __device__ void apply(int p, size_t o, int n, C<double> a, double& red) const {
    const C<double> v = ld<double>(phi[p] + o) - (ld<double>(self[p] + o) + coef[n] * a);
    st<double>(r[p] + o, v);
    red += norm2(v);
  }
  __device__ void tail(int) const {}
};

// Per-RHS block reduction: thread values -> partials[blk * kMaxRhs + n].
// Thread tid carries pair index q0 + (tid % 64) when pairs_per_wave is 64
// (hop kernels, 4 waves on the same 64 pairs) or q0 + tid (vector kernels);
// each n sums its threads in increasing thread order (deterministic).
__device__ __forceinline__ void block_partials_rhs(double v, int nr, long q0, int lane_mask, double* partials,
                                                   int blk) {
  __shared__ double sh[256];
  sh[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x < nr) {
    const int n = threadIdx.x;
    double s = 0.0;
    for (int i = 0; i < 256; ++i)
      if ((int)((q0 + (i & lane_mask)) % nr) == n) s += sh[i];
    partials[(size_t)blk * kMaxRhs + n] = s;
  }
}

template <typename R, bool DAG, typename Epi>
__global__ __launch_bounds__(256) void k_hop_mrhs(Geom g, int nr, int nbp, int p_fixed, HopIn<R> hin, Epi epi,
                                                  double* partials) {
  if (epi.skip()) return;
  __shared__ R2<R> lds[4][12][64];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int p = p_fixed >= 0 ? p_fixed : lb / nbp;
  const int blk = p_fixed >= 0 ? lb : lb % nbp;
  const int lane = threadIdx.x & 63;
  const int mu = threadIdx.x >> 6;
  const long q0 = (long)blk * 64;
  const long q = q0 + lane;
  const int cb = (int)(q / nr), n = (int)(q - (long)cb * nr);
  const bool active = cb < g.vh;
  C<R> acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = czero<R>();
  if (active) {
    int c[4];
    cb_coords(g, p, cb, c);
    const auto in = make_loader<R>(hin, g, p, nr);
    switch (mu) {
      case 0: hop_dir<R, 0, DAG>(g, hin.gauge, in, p, cb, c, acc, n); break;
      case 1: hop_dir<R, 1, DAG>(g, hin.gauge, in, p, cb, c, acc, n); break;
      case 2: hop_dir<R, 2, DAG>(g, hin.gauge, in, p, cb, c, acc, n); break;
      default: hop_dir<R, 3, DAG>(g, hin.gauge, in, p, cb, c, acc, n); break;
    }
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    R2<R> v;
    v.x = acc[k].re;
    v.y = acc[k].im;
    lds[mu][k][lane] = v;
  }
  __syncthreads();
  double red = 0.0;
  if (active) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int k = 3 * mu + i;
      const R2<R> a = lds[0][k][lane], b = lds[1][k][lane], cc = lds[2][k][lane], d = lds[3][k][lane];
      epi.apply(p, ((size_t)k * g.vh + cb) * nr + n, n,
                cmk<R>(((a.x + b.x) + cc.x) + d.x, ((a.y + b.y) + cc.y) + d.y), red);
    }
  }
  if constexpr (Epi::kReduce) block_partials_rhs(red, nr, q0, 63, partials, lb);
  epi.tail(nr);
}

static inline int mrhs_blocks_parity(const Geom& g, int nr) { return (int)(((size_t)g.vh * nr + 63) / 64); }

template <typename R, bool DAG, typename Epi>
static hipError_t mlaunch(const Geom& g, int nr, int p_out, const HopIn<R>& hin, const Epi& epi, Reduce red,
                          hipStream_t s) {
  const int nbp = mrhs_blocks_parity(g, nr);
  const int nb = p_out >= 0 ? nbp : 2 * nbp;
  if (Epi::kReduce && (size_t)nb * kMaxRhs > red.ndoubles) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_hop_mrhs<R, DAG, Epi>), dim3(nb), dim3(256), 0, s, g, nr, nbp, p_out, hin, epi,
                     red.partials);
  return hipGetLastError();
}

int mrhs_hop_blocks(const Geom& g, int nr, int p_out) {
  return p_out >= 0 ? mrhs_blocks_parity(g, nr) : 2 * mrhs_blocks_parity(g, nr);
}

template <typename R, bool DAG>
hipError_t launch_mhop_axpy(const Geom& g, int nr, int p_out, HopIn<R> hin, R2<R>* out_e, R2<R>* out_o,
                            const R2<R>* self_e, const R2<R>* self_o, const double* coef, hipStream_t s,
                            BatchState* guard, const double* pap_partials, Reduce red) {
  MEpiAxpy<R> e;
  e.out[0] = out_e;
  e.out[1] = out_o;
  e.self[0] = self_e;
  e.self[1] = self_o;
  e.coef = coef;
  e.guard = guard;
  e.pap_partials = pap_partials;
  e.pap_nblk = mrhs_blocks_parity(g, nr);
  e.state = guard;
  return mlaunch<R, DAG>(g, nr, p_out, hin, e, red, s);
}

template <typename R, bool DAG>
hipError_t launch_mhop_schur_norm(const Geom& g, int nr, HopIn<R> hin, R2<R>* w, const R2<R>* x,
                                  const double* coef, BatchState* st, Reduce red, hipStream_t s) {
  MEpiSchurNorm<R> e{w, x, coef, st};
  return mlaunch<R, DAG>(g, nr, 1, hin, e, red, s);
}

template <typename R, bool DAG>
hipError_t launch_mhop_schur_cg(const Geom& g, int nr, HopIn<R> hin, const R2<R>* w, R2<R>* x, R2<R>* r,
                                const R2<R>* p, const double* coef, BatchState* st, Reduce red, hipStream_t s) {
  MEpiSchurCG<R> e{w, x, r, p, coef, st};
  hipError_t err = mlaunch<R, DAG>(g, nr, 1, hin, e, red, s);
  if (err != hipSuccess) return err;
  return launch_mfinalize(kFinCgStep, mrhs_blocks_parity(g, nr), nr, red, st, 0.0, 0, s);
}

template <bool DAG>
hipError_t launch_mhop_residual(const Geom& g, int nr, HopIn<double> hin, const double2* self_full,
                                const double2* phi_full, double2* r_full, const double* coef, Reduce red,
                                hipStream_t s) {
  const size_t half = (size_t)12 * g.vh * nr;
  MEpiResidual e;
  e.self[0] = self_full;
  e.self[1] = self_full + half;
  e.phi[0] = phi_full;
  e.phi[1] = phi_full + half;
  e.r[0] = r_full;
  e.r[1] = r_full + half;
  e.coef = coef;
  hipError_t err = mlaunch<double, DAG>(g, nr, -1, hin, e, red, s);
  if (err != hipSuccess) return err;
  return launch_mfinalize(kFinResult1, 2 * mrhs_blocks_parity(g, nr), nr, red, nullptr, 0.0, 0, s);
}

#define LGT_INST_MHOP(R, DAG)                                                                                  \
  template hipError_t launch_mhop_axpy<R, DAG>(const Geom&, int, int, HopIn<R>, R2<R>*, R2<R>*, const R2<R>*, \
                                                const R2<R>*, const double*, hipStream_t, BatchState*,          \
                                                const double*, Reduce);                                        \
  template hipError_t launch_mhop_schur_norm<R, DAG>(const Geom&, int, HopIn<R>, R2<R>*, const R2<R>*,         \
                                                      const double*, BatchState*, Reduce, hipStream_t);       \
  template hipError_t launch_mhop_schur_cg<R, DAG>(const Geom&, int, HopIn<R>, const R2<R>*, R2<R>*, R2<R>*,   \
                                                    const R2<R>*, const double*, BatchState*, Reduce,          \
                                                    hipStream_t);

LGT_INST_MHOP(double, false)
LGT_INST_MHOP(double, true)
LGT_INST_MHOP(float, false)
LGT_INST_MHOP(float, true)
template hipError_t launch_mhop_residual<false>(const Geom&, int, HopIn<double>, const double2*, const double2*,
                                                double2*, const double*, Reduce, hipStream_t);
template hipError_t launch_mhop_residual<true>(const Geom&, int, HopIn<double>, const double2*, const double2*,
                                               double2*, const double*, Reduce, hipStream_t);

// ---------------------------------------------------------------------------
// Vector kernels over multi-RHS fields (n = total complex elements; the
// right-hand side of element i is i % nr).
// ---------------------------------------------------------------------------
static inline int mvec_blocks(size_t n) {
  size_t nb = (n + 255) / 256;
  return (int)(nb < 1024 ? (nb < 1 ? 1 : nb) : 1024);
}

// per-RHS |a|^2 (and Re <a, b>): partials [blk][kMaxRhs] (norm) and, when b
// is given, the dot products in a second finalize slot range
template <typename R>
__global__ __launch_bounds__(256) void k_mnorm(size_t n, int nr, const R2<R>* __restrict__ a, double* partials) {
  // grid-stride with a stride that is a multiple of nr keeps every thread on one RHS
  const size_t stride = (size_t)gridDim.x * 256 / nr * nr;
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  double acc = 0.0;
  if (stride > 0 && t < stride) {
    for (size_t i = t; i < n; i += stride) {
      const R2<R> v = a[i];
      acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
    }
  }
  block_partials_rhs(t < stride ? acc : 0.0, nr, (long)blockIdx.x * 256, 255, partials, blockIdx.x);
}

template <typename R>
hipError_t launch_mnorm(size_t n, int nr, const R2<R>* a, Reduce red, hipStream_t s) {
  const int nb = mvec_blocks(n);
  hipLaunchKernelGGL((k_mnorm<R>), dim3(nb), dim3(256), 0, s, n, nr, a, red.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_mfinalize(kFinResult1, nb, nr, red, nullptr, 0.0, 0, s);
}
template hipError_t launch_mnorm<double>(size_t, int, const double2*, Reduce, hipStream_t);
template hipError_t launch_mnorm<float>(size_t, int, const float2*, Reduce, hipStream_t);

// p = r + beta_n p for right-hand sides still running or stopping for an update
template <typename R>
__global__ __launch_bounds__(256) void k_mxpay(size_t n, int nr, const R2<R>* __restrict__ r, R2<R>* __restrict__ p,
                                               const BatchState* st) {
  if (st->all_done && !st->any_update) return;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const int k = (int)(i % nr);
    if (st->done[k] != kDoneRunning && st->done[k] != kDoneUpdate) continue;
    const R beta = R(st->beta[k]);
    const R2<R> rv = r[i];
    R2<R> pv = p[i];
    pv.x = rv.x + beta * pv.x;
    pv.y = rv.y + beta * pv.y;
    p[i] = pv;
  }
}
template <typename R>
hipError_t launch_mxpay(size_t n, int nr, const R2<R>* r, R2<R>* p, BatchState* st, hipStream_t s) {
  hipLaunchKernelGGL((k_mxpay<R>), dim3((n + 255) / 256), dim3(256), 0, s, n, nr, r, p, st);
  return hipGetLastError();
}
template hipError_t launch_mxpay<double>(size_t, int, const double2*, double2*, BatchState*, hipStream_t);
template hipError_t launch_mxpay<float>(size_t, int, const float2*, float2*, BatchState*, hipStream_t);

// x64 += scale_n * xs; xs = 0
__global__ __launch_bounds__(256) void k_mmixed_update(size_t n, int nr, float2* xs, double2* __restrict__ x,
                                                       const double* __restrict__ scale) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const double sc = scale[i % nr];
    const float2 v = xs[i];
    double2 xv = x[i];
    xv.x += sc * (double)v.x;
    xv.y += sc * (double)v.y;
    x[i] = xv;
    xs[i] = make_float2(0.f, 0.f);
  }
}
hipError_t launch_mmixed_update(size_t n, int nr, float2* xs, double2* x, const double* scale, hipStream_t s) {
  hipLaunchKernelGGL(k_mmixed_update, dim3((n + 255) / 256), dim3(256), 0, s, n, nr, xs, x, scale);
  return hipGetLastError();
}

// r = sigma_n r64; p = r (restart_n) or p *= pscale_n
__global__ __launch_bounds__(256) void k_mrescale(size_t n, int nr, const double2* __restrict__ r64,
                                                  const double* __restrict__ sigma, float2* __restrict__ r,
                                                  float2* __restrict__ p, const int* __restrict__ restart,
                                                  const double* __restrict__ pscale) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const int k = (int)(i % nr);
    const double sg = sigma[k];
    const double2 v = r64[i];
    const float2 w = make_float2((float)(sg * v.x), (float)(sg * v.y));
    r[i] = w;
    if (restart[k]) {
      p[i] = w;
    } else {
      const float2 q = p[i];
      p[i] = make_float2((float)(pscale[k] * (double)q.x), (float)(pscale[k] * (double)q.y));
    }
  }
}
hipError_t launch_mrescale(size_t n, int nr, const double2* r64, const double* sigma, float2* r, float2* p,
                           const int* restart, const double* pscale, hipStream_t s) {
  hipLaunchKernelGGL(k_mrescale, dim3((n + 255) / 256), dim3(256), 0, s, n, nr, r64, sigma, r, p, restart, pscale);
  return hipGetLastError();
}

// r = b, p = b, x = 0 (FP64 multi-RHS CG start); per-RHS |b|^2 to state
__global__ __launch_bounds__(256) void k_mcg_init64(size_t n, int nr, const double2* __restrict__ b,
                                                    double2* __restrict__ r, double2* __restrict__ p,
                                                    double2* __restrict__ x) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const double2 v = b[i];
    r[i] = v;
    p[i] = v;
    x[i] = make_double2(0.0, 0.0);
  }
}
hipError_t launch_mcg_init64(size_t n, int nr, const double2* b, double2* r, double2* p, double2* x,
                             BatchState* st, Reduce red, double tol, int max_iter, hipStream_t s) {
  hipLaunchKernelGGL(k_mcg_init64, dim3((n + 255) / 256), dim3(256), 0, s, n, nr, b, r, p, x);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nb = mvec_blocks(n);
  hipLaunchKernelGGL((k_mnorm<double>), dim3(nb), dim3(256), 0, s, n, nr, b, red.partials);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_mfinalize(kFinCgInit, nb, nr, red, st, tol, max_iter, s);
}

// One block: per-RHS sums of the partials of the previous launch.
// The host has to act once every right-hand side is done or, with reliable
// updates on (delta2 > 0), once half of those not yet verified have stopped
// (a stopped one idles until the update).
__device__ __forceinline__ int batch_action(const BatchState* st, int nr) {
  if (st->all_done) return 1;
  if (!(st->delta2 > 0.0)) return 0;
  int active = 0, stopped = 0;
  for (int n = 0; n < nr; ++n) {
    active += st->done[n] != kDoneConverged;
    stopped += st->done[n] != kDoneConverged && st->done[n] != kDoneRunning;
  }
  return 2 * stopped >= active;
}

__global__ __launch_bounds__(256) void k_mfinalize(int mode, int nblk, int nr, const double* __restrict__ partials,
                                                   BatchState* st, double* result, double tol, int max_iter,
                                                   Mailbox* mb) {
  if (mode == kFinCgStep && st->all_done) {  // the iteration was skipped
    if (threadIdx.x == 0) {
      for (int n = 0; n < nr; ++n)
        if (st->done[n] == kDoneUpdate) st->done[n] = kDoneUpdateHeld;
      st->any_update = 0;
      post_progress(mb, st->iter, 1);
    }
    return;
  }
  __shared__ double sh[4];
  __shared__ double tot[kMaxRhs];
  for (int n = 0; n < nr; ++n) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 256) s += partials[(size_t)i * kMaxRhs + n];
    const double t = block_sum<256>(s, sh);
    if (threadIdx.x == 0) tot[n] = t;
  }
  if (threadIdx.x != 0) return;
  if (mode == kFinResult1) {
    for (int n = 0; n < nr; ++n) result[n] = tot[n];
    return;
  }
  if (mode == kFinCgInit) {
    st->nr = nr;
    st->iter = 0;
    st->max_iter = max_iter;
    st->delta2 = 0.0;
    st->any_update = 0;
    int all = 1;
    for (int n = 0; n < nr; ++n) {
      const double rr = tot[n];
      st->rr[n] = rr;
      st->rr_max[n] = rr;
      st->rr_stop[n] = tol * tol * rr;
      st->alpha[n] = st->beta[n] = st->pap[n] = 0.0;
      st->done[n] = !isfinite(rr) ? kDoneBreakdown : (rr == 0.0 ? kDoneConverged : kDoneRunning);
      st->conv_iter[n] = 0;
      all &= st->done[n] != kDoneRunning;
    }
    st->all_done = all;
    return;
  }
  // kFinCgStep
  st->iter += 1;
  int all = 1, any_update = 0;
  const double d2 = st->delta2;
  for (int n = 0; n < nr; ++n) {
    if (st->done[n] == kDoneUpdate) st->done[n] = kDoneUpdateHeld;
    if (st->done[n] == kDoneRunning) {
      const double rr = tot[n];
      st->beta[n] = rr / st->rr[n];
      st->rr[n] = rr;
      if (rr > st->rr_max[n]) st->rr_max[n] = rr;
      if (!isfinite(rr)) st->done[n] = kDoneBreakdown;
      else if (rr <= st->rr_stop[n]) st->done[n] = d2 > 0.0 ? kDoneUpdate : kDoneConverged;
      else if (rr <= d2 * st->rr_max[n]) st->done[n] = kDoneUpdate;
      else if (st->iter >= st->max_iter) st->done[n] = kDoneMaxIter;
      if (st->done[n] != kDoneRunning) st->conv_iter[n] = st->iter;
    }
    any_update |= st->done[n] == kDoneUpdate;
    all &= st->done[n] != kDoneRunning;
  }
  st->all_done = all;
  st->any_update = any_update;
  post_progress(mb, st->iter, batch_action(st, nr));
}

hipError_t launch_mfinalize(int mode, int nblk, int nr, Reduce red, BatchState* st, double tol, int max_iter,
                            hipStream_t s) {
  if ((size_t)nblk * kMaxRhs > red.ndoubles) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mfinalize, dim3(1), dim3(256), 0, s, mode, nblk, nr, red.partials, st, red.result, tol,
                     max_iter, red.mbox);
  return hipGetLastError();
}

// Multi-RHS pack / unpack of one right-hand side n: canonical [V][12]
// complex128 <-> packed [2][12][vh][nr] (element stride nr).
__global__ __launch_bounds__(256) void k_mpack(Geom g, int nr, int n, const double2* __restrict__ canon,
                                               double2* __restrict__ packed) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= 2 * (size_t)g.vh * 12) return;
  const int s = (int)(t / 12), k = (int)(t % 12);
  int c[4];
  lex_coords(g, s, c);
  packed[(((size_t)parity_of(c) * 12 + k) * g.vh + (s >> 1)) * nr + n] = canon[t];
}
__global__ __launch_bounds__(256) void k_munpack(Geom g, int nr, int n, const double2* __restrict__ packed,
                                                 double2* __restrict__ canon) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= 2 * (size_t)g.vh * 12) return;
  const int s = (int)(t / 12), k = (int)(t % 12);
  int c[4];
  lex_coords(g, s, c);
  canon[t] = packed[(((size_t)parity_of(c) * 12 + k) * g.vh + (s >> 1)) * nr + n];
}
hipError_t launch_mpack(const Geom& g, int nr, int n, const double2* canon, double2* packed, hipStream_t s) {
  const size_t tot = 2 * (size_t)g.vh * 12;
  hipLaunchKernelGGL(k_mpack, dim3((tot + 255) / 256), dim3(256), 0, s, g, nr, n, canon, packed);
  return hipGetLastError();
}
hipError_t launch_munpack(const Geom& g, int nr, int n, const double2* packed, double2* canon, hipStream_t s) {
  const size_t tot = 2 * (size_t)g.vh * 12;
  hipLaunchKernelGGL(k_munpack, dim3((tot + 255) / 256), dim3(256), 0, s, g, nr, n, packed, canon);
  return hipGetLastError();
}

}  // namespace lgt
