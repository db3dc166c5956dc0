// Wilson hop H_{p,1-p} on the even/odd lattice, with the epilogues the
// solver fuses into it.
//
//   (H psi)(x) = sum_mu [ (1 - gamma_mu) U~_mu(x) psi(x+mu) + (1 + gamma_mu) U~_mu(x-mu)^dag psi(x-mu) ]
//   (H^dag: the signs of gamma_mu flip)
//
// so that D = 1 - kappa H (the operator of the pseudofermion action, S3.1).
//
// Work decomposition (gfx950): a 256-thread block owns 64 consecutive
// checkerboard sites of one parity; wave w (= direction mu) computes both
// hops along mu for the 64 sites, using the chiral-basis spin projection
// (1 + s gamma_mu) psi = (h ; s B_mu^dag h), h = psi_up + s B_mu psi_dn, so
// only two colour vectors go through each SU(3) multiply.  The four
// per-direction partial spinors meet in LDS and wave w then owns spin
// component w of the 64 output sites for the epilogue, so every global load
// and store is a unit-stride 64-lane access in the [12][vh] SoA layout.
// Small lattices use 32-site blocks instead, whose half-waves take the
// forward and the backward hop (unit-stride 32-lane halves).
// Blocks are numbered XCD-contiguously (see xcd_block).
#include "lgt_internal.h"
#include "lgt_hop.h"

namespace lgt {

// ---------------------------------------------------------------------------
// Epilogues.  apply() gets the 3 colour components of spin `spin` of the hop
// result at (p, cb); red accumulates this thread's reduction contribution.
// T is the storage type of the spinors t, w, p of the CG (R2<R> or Bf16c);
// x and r are always R2<R>.
// ---------------------------------------------------------------------------
template <typename R, typename T>
struct EpiAxpy {  // out = self + coef * acc
  static constexpr bool kReduce = false;
  static constexpr bool kPrefetch = !std::is_same<T, Bf16c>::value;
  T* out[2];
  const T* self[2];
  R coef;
  int vh;
  SolverState* guard;  // if set, the launch is a no-op once the solve has stopped
  // If set, block 0 also turns the |w|^2 block partials of the previous
  // launch into pap and alpha = rr / pap (the CG step between the two hops
  // of Mhat^dag Mhat, which need no scalar).
  const double* pap_partials;
  int pap_nblk;
  __device__ bool skip() const { return guard && guard->done != kDoneRunning; }
  struct Pre {
    C<R> s[3];
  };
  __device__ Pre pre(int p, int cb, int spin) const {
    Pre q;
#pragma unroll
    for (int i = 0; i < 3; ++i)
      q.s[i] = self[p] ? Store<R, T>::ld(self[p] + (size_t)(3 * spin + i) * vh + cb) : czero<R>();
    return q;
  }
  __device__ void apply(int p, int cb, int spin, const C<R>* acc, double&, const Pre& q) const {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const size_t o = (size_t)(3 * spin + i) * vh + cb;
      Store<R, T>::st(out[p] + o, q.s[i] + coef * acc[i]);
    }
  }
  template <int NT>
  __device__ void tail() const {
    if (!pap_partials || blockIdx.x != 0) return;
    double tot[1];
    sum_partials<NT, 1>(pap_partials, pap_nblk, tot);
    if (threadIdx.x == 0) {
      const double pap = tot[0];
      guard->pap = pap;
      guard->rr_prev = guard->rr;
      guard->iter_prev = guard->iter;
      if (!(pap > 0.0) || !isfinite(pap)) {
        guard->alpha = 0.0;
        guard->done = kDoneBreakdown;
      } else {
        guard->alpha = guard->rr / pap;
      }
    }
  }
};

// First hop of a CG iteration with the previous iteration's step folded in
// (FP64 and FP32-stored recursions).  Every block first sums the |r|^2
// partials the previous iteration's last hop wrote (same partials, same
// order: every block takes the same decision) into rr, beta = rr / rr_prev
// and the stop test; block 0 records the state and posts to the mailbox.
// If the recursion goes on, the hop runs on r instead of p, using
// H p_new = H (r + beta p) = H r + beta H p, with H p the t of the previous
// iteration (kept in t, which the iteration's second use of the even half
// does not overwrite), and each thread updates p = r + beta p at the odd
// sites of its own (site, spin): the hop reads only r, so the update races
// with no reader.  One launch and one pass over r and p fewer per iteration
// than a separate step kernel.  A launch finding the solve stopped returns
// (block 0 turns kDoneUpdate into kDoneUpdateHeld and repeats the action).
template <typename R>
struct EpiStep {
  static constexpr bool kReduce = false;
  static constexpr bool kPrefetch = true;
  R2<R>* t;         // even half: H p, updated in place
  R2<R>* p;         // odd half: search direction
  const R2<R>* r;   // odd half: residual (the hop's input)
  int vh;
  SolverState* state;
  const double* partials;
  int nblk;
  Mailbox* mb;
  __device__ static double& beta_sh() {
    __shared__ double b;
    return b;
  }
  __device__ bool skip() const {  // block-collective: every thread of the block calls it
    __shared__ int s_run;
    SolverState* st = state;
    const int done0 = st->done;
    if (done0 != kDoneRunning) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (done0 == kDoneUpdate) st->done = kDoneUpdateHeld;
        post_progress(mb, st->iter, action_word(st->epoch, done0 == kDoneUpdateHeld ? kDoneUpdate : done0));
      }
      return true;
    }
    double tot[1];
    sum_partials<256, 1>(partials, nblk, tot);
    if (threadIdx.x == 0) {
      const double rr = tot[0];
      const double beta = rr / st->rr_prev;
      const int iter = st->iter_prev + 1;
      const double rr_max = fmax(st->rr_max, rr);
      int code = kDoneRunning;
      if (!isfinite(rr)) code = kDoneBreakdown;
      else if (rr <= st->rr_stop) code = st->delta2 > 0.0 ? kDoneUpdate : kDoneConverged;
      else if (rr <= st->delta2 * rr_max) code = kDoneUpdate;
      else if (iter >= st->max_iter) code = kDoneMaxIter;
      beta_sh() = beta;
      s_run = code == kDoneRunning;
      if (blockIdx.x == 0) {
        st->beta = beta;
        st->rr = rr;
        st->iter = iter;
        st->rr_max = rr_max;
        if (code != kDoneRunning) st->done = code;
        post_progress(mb, iter, code != kDoneRunning ? action_word(st->epoch, code) : 0u);
      }
    }
    __syncthreads();
    return !s_run;
  }
  struct Pre {
    C<R> t[3], r[3], p[3];
  };
  __device__ Pre pre(int, int cb, int spin) const {
    Pre q;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const size_t o = (size_t)(3 * spin + i) * vh + cb;
      q.t[i] = ld<R>(t + o);
      q.r[i] = ld<R>(r + o);
      q.p[i] = ld<R>(p + o);
    }
    return q;
  }
  __device__ void apply(int, int cb, int spin, const C<R>* acc, double&, const Pre& q) const {
    const R b = R(beta_sh());
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const size_t o = (size_t)(3 * spin + i) * vh + cb;
      lgt::st<R>(t + o, acc[i] + b * q.t[i]);
      lgt::st<R>(p + o, q.r[i] + b * q.p[i]);
    }
  }
  template <int NT>
  __device__ void tail() const {}
};

template <typename R, typename T>
struct EpiSchurNorm {  // w = x + coef * acc (odd sites), block partials of |w|^2 (of w as stored)
  static constexpr bool kReduce = true;
  static constexpr bool kPrefetch = !std::is_same<T, Bf16c>::value;
  T* w;
  const T* x;
  R coef;
  int vh;
  SolverState* state;
  __device__ bool skip() const { return state->done != kDoneRunning; }
  struct Pre {
    C<R> x[3];
  };
  __device__ Pre pre(int, int cb, int spin) const {
    Pre q;
#pragma unroll
    for (int i = 0; i < 3; ++i) q.x[i] = Store<R, T>::ld(x + (size_t)(3 * spin + i) * vh + cb);
    return q;
  }
  __device__ void apply(int, int cb, int spin, const C<R>* acc, double& red, const Pre& q) const {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const size_t o = (size_t)(3 * spin + i) * vh + cb;
      const C<R> v = Store<R, T>::round(q.x[i] + coef * acc[i]);
      Store<R, T>::st(w + o, v);
      red += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
    }
  }
  template <int NT>
  __device__ void tail() const {}
};

template <typename R, typename T>
struct EpiSchurCG {  // q = w + coef * acc; x += alpha p (if x); r -= alpha q; block partials of |r|^2
  static constexpr bool kReduce = true;
  static constexpr bool kPrefetch = !std::is_same<T, Bf16c>::value;
  const T* w;
  R2<R>* x;
  R2<R>* r;
  const T* p;
  R coef;
  int vh;
  SolverState* state;
  __device__ bool skip() const { return state->done != kDoneRunning; }
  struct Pre {
    C<R> w[3], x[3], r[3], p[3];
  };
  __device__ Pre pre(int, int cb, int spin) const {
    Pre q;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const size_t o = (size_t)(3 * spin + i) * vh + cb;
      q.w[i] = Store<R, T>::ld(w + o);
      q.r[i] = ld<R>(r + o);
      if (x) {
        q.x[i] = ld<R>(x + o);
        q.p[i] = Store<R, T>::ld(p + o);
      }
    }
    return q;
  }
  __device__ void apply(int, int cb, int spin, const C<R>* acc, double& red, const Pre& pq) const {
    const R alpha = R(state->alpha);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const size_t o = (size_t)(3 * spin + i) * vh + cb;
      const C<R> q = pq.w[i] + coef * acc[i];
      if (x) st<R>(x + o, pq.x[i] + alpha * pq.p[i]);
      C<R> rv = pq.r[i] - alpha * q;
      st<R>(r + o, rv);
      red += (double)rv.re * (double)rv.re + (double)rv.im * (double)rv.im;
    }
  }
  template <int NT>
  __device__ void tail() const {}
};

struct EpiResidual {  // r = phi - (self + coef * acc) over both parities, block partials of |r|^2
  static constexpr bool kReduce = true;
  static constexpr bool kPrefetch = true;
  const double2* self[2];
  const double2* phi[2];
  double2* r[2];
  double coef;
  int vh;
  __device__ bool skip() const { return false; }
  struct Pre {
    C<double> f[3], s[3];
  };
  __device__ Pre pre(int p, int cb, int spin) const {
    Pre q;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const size_t o = (size_t)(3 * spin + i) * vh + cb;
      q.f[i] = ld<double>(phi[p] + o);
      q.s[i] = ld<double>(self[p] + o);
    }
    return q;
  }
  __device__ void apply(int p, int cb, int spin, const C<double>* acc, double& red, const Pre& q) const {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const size_t o = (size_t)(3 * spin + i) * vh + cb;
      C<double> v = q.f[i] - (q.s[i] + coef * acc[i]);
      st<double>(r[p] + o, v);
      red += norm2(v);
    }
  }
  template <int NT>
  __device__ void tail() const {}
};

// ---------------------------------------------------------------------------
// The hop kernel.  Grid: nbp blocks per parity (p_fixed >= 0) or 2*nbp
// (p_fixed < 0, parity = logical block / nbp).  NS = 64: wave mu computes
// both hops along mu for 64 sites.  NS = 32 (small lattices, whose 64-site
// grid would not give every SIMD a wave): wave mu computes the forward hop
// of 32 sites on lanes 0-31 and their backward hop on lanes 32-63, so twice
// as many waves share the latency; waves 0 and 1 then run the epilogue, one
// (site, spin) pair per lane.
//
// Block order (64-site blocks, when a t-slice holds a whole number of
// blocks: bps blocks per slice, tgrp > 0).  Checkerboard sites are x-fastest,
// so in site order a site's t-neighbours are a whole slice away, and on
// large lattices the L2 of an XCD has streamed the slice's links and
// spinors out again before the second read.  The blocks of each group of
// tgrp consecutive slices are therefore taken t-fastest: block j of the
// group covers slice j % tgrp, chunk j / tgrp of that slice, so the t-hops
// of a chunk are a few blocks apart and its z-hops 8 tgrp blocks apart.  A
// bijection of the blocks of a parity: every site is still covered once.
// ---------------------------------------------------------------------------
template <typename R, bool DAG, typename Epi, typename In, int NS>
__global__ __launch_bounds__(256) void k_hop(Geom g, int nbp, int p_fixed, In hin, Epi epi, double* partials,
                                             int bps, int tgrp) {
  static_assert(NS == 64 || NS == 32, "64 or 32 sites per block");
  if (epi.skip()) return;
  __shared__ R2<R> lds[4][12][64];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int p = p_fixed >= 0 ? p_fixed : lb / nbp;
  int blk = p_fixed >= 0 ? lb : lb % nbp;
  if (NS == 64 && tgrp > 0) {
    const int span = tgrp * bps;
    const int grp = blk / span, rem = blk - grp * span;
    const int chunk = rem / tgrp, tl = rem - chunk * tgrp;
    blk = (grp * tgrp + tl) * bps + chunk;
  }
  const int lane = threadIdx.x & 63;
  const int mu = threadIdx.x >> 6;
  const bool bwd = NS == 32 && lane >= 32;
  const int cb = blk * NS + (NS == 64 ? lane : lane & 31);
  const bool active = cb < g.vh;
  // 64-site blocks: the lane's epilogue operands at its own (site, spin =
  // wave) are independent of the hop, so they are loaded before it and
  // arrive while the neighbour loads are in flight (16^4 mixed force call
  // 5.40 -> 5.15 ms, FP64 at 24^3x48 187 -> 183 ms).  Not for BF16-stored
  // vectors, where holding them across the hop cost more than it saved
  // (24^3x48: 65.0 -> 67.5 ms).
  typename Epi::Pre pre{};
  if constexpr (NS == 64 && Epi::kPrefetch) {
    if (active) pre = epi.pre(p, cb, mu);
  }

  C<R> acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = czero<R>();
  if (active) {
    int c[4];
    cb_coords(g, p, cb, c);
    const auto in = make_loader<R>(hin, g, p, 1);
    if constexpr (NS == 64) {
      switch (mu) {
        case 0: hop_dir<R, 0, DAG>(g, hin.gauge, hin.nk, in, p, cb, c, acc, 0); break;
        case 1: hop_dir<R, 1, DAG>(g, hin.gauge, hin.nk, in, p, cb, c, acc, 0); break;
        case 2: hop_dir<R, 2, DAG>(g, hin.gauge, hin.nk, in, p, cb, c, acc, 0); break;
        default: hop_dir<R, 3, DAG>(g, hin.gauge, hin.nk, in, p, cb, c, acc, 0); break;
      }
    } else {
      switch (mu) {
        case 0: hop_one<R, 0, DAG>(g, hin.gauge, hin.nk, in, p, cb, c, acc, bwd); break;
        case 1: hop_one<R, 1, DAG>(g, hin.gauge, hin.nk, in, p, cb, c, acc, bwd); break;
        case 2: hop_one<R, 2, DAG>(g, hin.gauge, hin.nk, in, p, cb, c, acc, bwd); break;
        default: hop_one<R, 3, DAG>(g, hin.gauge, hin.nk, in, p, cb, c, acc, bwd); break;
      }
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
  if constexpr (NS == 64) {
    // wave `mu` now owns spin component `mu` of the 64 sites
    const int spin = mu;
    C<R> out[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int k = 3 * spin + i;
      R2<R> a = lds[0][k][lane], b = lds[1][k][lane], cc = lds[2][k][lane], d = lds[3][k][lane];
      out[i] = cmk<R>(((a.x + b.x) + cc.x) + d.x, ((a.y + b.y) + cc.y) + d.y);
    }
    if constexpr (!Epi::kPrefetch) {
      if (active) pre = epi.pre(p, cb, spin);
    }
    if (active) epi.apply(p, cb, spin, out, red, pre);
  } else if (mu < 2) {
    // lane -> site lane & 31, spin 2 mu + lane / 32; eight partial hops
    const int site = lane & 31;
    const int spin = 2 * mu + (lane >> 5);
    const int cbo = blk * 32 + site;
    C<R> out[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int k = 3 * spin + i;
      R sx = R(0), sy = R(0);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const R2<R> f = lds[m][k][site], b = lds[m][k][32 + site];
        sx += f.x + b.x;
        sy += f.y + b.y;
      }
      out[i] = cmk<R>(sx, sy);
    }
    if (cbo < g.vh) epi.apply(p, cbo, spin, out, red, epi.pre(p, cbo, spin));
  }
  if constexpr (Epi::kReduce) {
    double v[1] = {red};
    block_partials<256, 1>(v, partials, lb);
  }
  epi.template tail<256>();
}

// Sites per hop block: the context's choice, else 32 on small lattices
// (kHopHalfWaveMaxVh sites per parity and below), 64 above.
static inline int hop_sites_per_block(const Geom& g) {
  if (g.hop_ns == 32 || g.hop_ns == 64) return g.hop_ns;
  return g.vh <= kHopHalfWaveMaxVh ? 32 : 64;
}
static inline int nblk_parity(const Geom& g) {
  const int ns = hop_sites_per_block(g);
  return (g.vh + ns - 1) / ns;
}

// t-fastest block groups of the 64-site kernel: (blocks per t-slice, slices
// per group), or tgrp = 0 (site order): by the context's choice, else above
// kHopTOrderMinVh sites per parity (24^3x48: hop 36 -> 32 us, re-read
// traffic 1.29x -> 1.1x; at 16^4, whose fields stay in the caches, site
// order is 3 % faster); never when a slice is not a whole number of blocks.
// Groups of 8 slices where Lt allows, else 4 or 2 (Lt is even).
static inline void hop_block_order(const Geom& g, int& bps, int& tgrp) {
  const int vslice = g.vh / g.L[3];
  bps = vslice / 64;
  tgrp = 0;
  if (vslice % 64 != 0 || bps == 0) return;
  if (g.hop_order == 1 || (g.hop_order == 0 && g.vh <= kHopTOrderMinVh)) return;
  tgrp = g.L[3] % 8 == 0 ? 8 : (g.L[3] % 4 == 0 ? 4 : 2);
}

template <typename R, bool DAG, typename Epi, typename In>
static hipError_t launch(const Geom& g, int p_out, const In& hin, const Epi& epi, double* partials, hipStream_t s,
                         int capacity = 0) {
  const int nbp = nblk_parity(g);
  const int nb = p_out >= 0 ? nbp : 2 * nbp;
  if (Epi::kReduce && nb > capacity) return hipErrorInvalidValue;
  if (hop_sites_per_block(g) == 32) {
    hipLaunchKernelGGL((k_hop<R, DAG, Epi, In, 32>), dim3(nb), dim3(256), 0, s, g, nbp, p_out, hin, epi, partials,
                       0, 0);
  } else {
    int bps, tgrp;
    hop_block_order(g, bps, tgrp);
    hipLaunchKernelGGL((k_hop<R, DAG, Epi, In, 64>), dim3(nb), dim3(256), 0, s, g, nbp, p_out, hin, epi, partials,
                       bps, tgrp);
  }
  return hipGetLastError();
}

int hop_blocks(const Geom& g, int p_out) { return p_out >= 0 ? nblk_parity(g) : 2 * nblk_parity(g); }

template <typename R, bool DAG, typename T>
hipError_t launch_hop_axpy(const Geom& g, int p_out, HopIn<R, T> hin, T* out_even, T* out_odd,
                           const typename NoDeduce<T>::type* self_even, const typename NoDeduce<T>::type* self_odd,
                           double coef, hipStream_t s, SolverState* guard, const double* pap_partials) {
  EpiAxpy<R, T> e;
  e.guard = guard;
  e.pap_partials = pap_partials;
  e.pap_nblk = nblk_parity(g);
  e.out[0] = out_even;
  e.out[1] = out_odd;
  e.self[0] = self_even;
  e.self[1] = self_odd;
  e.coef = R(coef);
  e.vh = g.vh;
  return launch<R, DAG>(g, p_out, hin, e, nullptr, s);
}

template <typename R, typename T, bool DAG>
hipError_t launch_hop_schur_norm(const Geom& g, HopIn<R, T> hin, T* w, const T* x, double coef, SolverState* st,
                                 Reduce red, hipStream_t s) {
  EpiSchurNorm<R, T> e{w, x, R(coef), g.vh, st};
  return launch<R, DAG>(g, 1, hin, e, red.partials, s, red.capacity);
}

template <typename R, typename T, bool DAG>
hipError_t launch_hop_schur_cg(const Geom& g, HopIn<R, T> hin, const T* w, R2<R>* x, R2<R>* r, const T* p,
                               double coef, SolverState* st, Reduce red, hipStream_t s) {
  EpiSchurCG<R, T> e{w, x, r, p, R(coef), g.vh, st};
  return launch<R, DAG>(g, 1, hin, e, red.partials, s, red.capacity);
}

template <bool DAG>
hipError_t launch_hop_residual(const Geom& g, HopIn<double> hin, const double2* self_full,
                               const double2* phi_full, double2* r_full, double coef, Reduce red,
                               int slot, hipStream_t s) {
  const size_t half = (size_t)12 * g.vh;
  EpiResidual e;
  e.self[0] = self_full;
  e.self[1] = self_full + half;
  e.phi[0] = phi_full;
  e.phi[1] = phi_full + half;
  e.r[0] = r_full;
  e.r[1] = r_full + half;
  e.coef = coef;
  e.vh = g.vh;
  hipError_t err = launch<double, DAG>(g, -1, hin, e, red.partials, s, red.capacity);
  if (err != hipSuccess) return err;
  return launch_finalize(kFinResult1, 2 * nblk_parity(g), red, nullptr, slot, 0.0, 0, s);
}

template <typename R, bool DAG>
hipError_t launch_hop_step(const Geom& g, const R2<R>* gauge, int nk, R2<R>* t, R2<R>* p, const R2<R>* r,
                           SolverState* st, Reduce red, hipStream_t s) {
  EpiStep<R> e;
  e.t = t;
  e.p = p;
  e.r = r;
  e.vh = g.vh;
  e.state = st;
  e.partials = red.partials;
  e.nblk = nblk_parity(g);
  e.mb = red.mbox;
  if (e.nblk > red.capacity) return hipErrorInvalidValue;
  const HopIn<R> hin{gauge, r, r, nk};
  return launch<R, DAG>(g, 0, hin, e, nullptr, s);
}
template hipError_t launch_hop_step<double, false>(const Geom&, const double2*, int, double2*, double2*,
                                                   const double2*, SolverState*, Reduce, hipStream_t);
template hipError_t launch_hop_step<double, true>(const Geom&, const double2*, int, double2*, double2*,
                                                  const double2*, SolverState*, Reduce, hipStream_t);
template hipError_t launch_hop_step<float, false>(const Geom&, const float2*, int, float2*, float2*,
                                                  const float2*, SolverState*, Reduce, hipStream_t);
template hipError_t launch_hop_step<float, true>(const Geom&, const float2*, int, float2*, float2*, const float2*,
                                                 SolverState*, Reduce, hipStream_t);

#define LGT_INST_AXPY(R, DAG, T)                                                                          \
  template hipError_t launch_hop_axpy<R, DAG, T>(const Geom&, int, HopIn<R, T>, T*, T*, const T*, const T*, \
                                                  double, hipStream_t, SolverState*, const double*);
#define LGT_INST_CG(R, T, DAG)                                                                            \
  template hipError_t launch_hop_schur_norm<R, T, DAG>(const Geom&, HopIn<R, T>, T*, const T*, double,       \
                                                        SolverState*, Reduce, hipStream_t);                 \
  template hipError_t launch_hop_schur_cg<R, T, DAG>(const Geom&, HopIn<R, T>, const T*, R2<R>*, R2<R>*,     \
                                                      const T*, double, SolverState*, Reduce, hipStream_t);

LGT_INST_AXPY(double, false, double2)
LGT_INST_AXPY(double, true, double2)
LGT_INST_AXPY(float, false, float2)
LGT_INST_AXPY(float, true, float2)
LGT_INST_AXPY(float, false, Bf16c)
LGT_INST_AXPY(float, true, Bf16c)
LGT_INST_CG(double, double2, false)
LGT_INST_CG(double, double2, true)
LGT_INST_CG(float, float2, false)
LGT_INST_CG(float, float2, true)
LGT_INST_CG(float, Bf16c, false)
LGT_INST_CG(float, Bf16c, true)

template hipError_t launch_hop_residual<false>(const Geom&, HopIn<double>, const double2*, const double2*,
                                               double2*, double, Reduce, int, hipStream_t);
template hipError_t launch_hop_residual<true>(const Geom&, HopIn<double>, const double2*, const double2*,
                                              double2*, double, Reduce, int, hipStream_t);

}  // namespace lgt
