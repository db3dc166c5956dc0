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
// Blocks are numbered XCD-contiguously (see xcd_block).
#include <cstdlib>

#include "lgt_internal.h"
#include "lgt_hop.h"

namespace lgt {

// ---------------------------------------------------------------------------
// Epilogues.  apply() gets the 3 colour components of spin `spin` of the hop
// result at (p, cb); red accumulates this thread's reduction contribution.
// ---------------------------------------------------------------------------
template <typename R>
struct EpiAxpy {  // out = self + coef * acc
  static constexpr bool kReduce = false;
  R2<R>* out[2];
  const R2<R>* self[2];
  R coef;
  int vh;
  SolverState* guard;  // if set, the launch is a no-op once the solve has finished
  // If set, block 0 also turns the |w|^2 block partials of the previous
  // launch into pap and alpha = rr / pap (the CG step between the two hops
  // of Mhat^dag Mhat, which need no scalar).
  const double* pap_partials;
  int pap_nblk;
  __device__ bool skip() const { return guard && guard->done != kDoneRunning; }
  __device__ void apply(int p, int cb, int spin, const C<R>* acc, double&) const {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const size_t o = (size_t)(3 * spin + i) * vh + cb;
      C<R> v = coef * acc[i];
      if (self[p]) v += ld<R>(self[p] + o);
      st<R>(out[p] + o, v);
    }
  }
  __device__ void apply1(int p, int cb, int k, C<R> a, double&) const {
    const size_t o = (size_t)k * vh + cb;
    C<R> v = coef * a;
    if (self[p]) v += ld<R>(self[p] + o);
    st<R>(out[p] + o, v);
  }
  template <int NT>
  __device__ void tail() const {
    if (!pap_partials || blockIdx.x != 0) return;
    double tot[1];
    sum_partials<NT, 1>(pap_partials, pap_nblk, tot);
    if (threadIdx.x == 0) {
      const double pap = tot[0];
      guard->pap = pap;
      if (!(pap > 0.0) || !isfinite(pap)) {
        guard->alpha = 0.0;
        guard->done = kDoneBreakdown;
      } else {
        guard->alpha = guard->rr / pap;
      }
    }
  }
};

template <typename R>
struct EpiSchurNorm {  // w = x + coef * acc (odd sites), block partials of |w|^2
  static constexpr bool kReduce = true;
  R2<R>* w;
  const R2<R>* x;
  R coef;
  int vh;
  SolverState* state;
  __device__ bool skip() const { return state->done != kDoneRunning; }
  __device__ void apply(int, int cb, int spin, const C<R>* acc, double& red) const {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const size_t o = (size_t)(3 * spin + i) * vh + cb;
      C<R> v = ld<R>(x + o) + coef * acc[i];
      st<R>(w + o, v);
      red += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
    }
  }
  __device__ void apply1(int, int cb, int k, C<R> a, double& red) const {
    const size_t o = (size_t)k * vh + cb;
    C<R> v = ld<R>(x + o) + coef * a;
    st<R>(w + o, v);
    red += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
  }
  template <int NT>
  __device__ void tail() const {}
};

template <typename R>
struct EpiSchurCG {  // q = w + coef * acc; x += alpha p; r -= alpha q; block partials of |r|^2
  static constexpr bool kReduce = true;
  const R2<R>* w;
  R2<R>* x;
  R2<R>* r;
  const R2<R>* p;
  R coef;
  int vh;
  SolverState* state;
  __device__ bool skip() const { return state->done != kDoneRunning; }
  __device__ void apply(int, int cb, int spin, const C<R>* acc, double& red) const {
    const R alpha = R(state->alpha);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const size_t o = (size_t)(3 * spin + i) * vh + cb;
      const C<R> q = ld<R>(w + o) + coef * acc[i];
      const C<R> pv = ld<R>(p + o);
      C<R> xv = ld<R>(x + o) + alpha * pv;
      C<R> rv = ld<R>(r + o) - alpha * q;
      st<R>(x + o, xv);
      st<R>(r + o, rv);
      red += (double)rv.re * (double)rv.re + (double)rv.im * (double)rv.im;
    }
  }
  __device__ void apply1(int, int cb, int k, C<R> a, double& red) const {
    const R alpha = R(state->alpha);
    const size_t o = (size_t)k * vh + cb;
    const C<R> q = ld<R>(w + o) + coef * a;
    C<R> xv = ld<R>(x + o) + alpha * ld<R>(p + o);
    C<R> rv = ld<R>(r + o) - alpha * q;
    st<R>(x + o, xv);
    st<R>(r + o, rv);
    red += (double)rv.re * (double)rv.re + (double)rv.im * (double)rv.im;
  }
  template <int NT>
  __device__ void tail() const {}
};

struct EpiResidual {  // r = phi - (self + coef * acc) over both parities, block partials of |r|^2
  static constexpr bool kReduce = true;
  const double2* self[2];
  const double2* phi[2];
  double2* r[2];
  double coef;
  int vh;
  __device__ bool skip() const { return false; }
  __device__ void apply(int p, int cb, int spin, const C<double>* acc, double& red) const {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const size_t o = (size_t)(3 * spin + i) * vh + cb;
      C<double> v = ld<double>(phi[p] + o) - (ld<double>(self[p] + o) + coef * acc[i]);
      st<double>(r[p] + o, v);
      red += norm2(v);
    }
  }
  __device__ void apply1(int p, int cb, int k, C<double> a, double& red) const {
    const size_t o = (size_t)k * vh + cb;
    C<double> v = ld<double>(phi[p] + o) - (ld<double>(self[p] + o) + coef * a);
    st<double>(r[p] + o, v);
    red += norm2(v);
  }
  template <int NT>
  __device__ void tail() const {}
};

// ---------------------------------------------------------------------------
// The hop kernel.  Grid: nbp blocks per parity (p_fixed >= 0) or 2*nbp
// (p_fixed < 0, parity = logical block / nbp).
// ---------------------------------------------------------------------------
template <typename R, bool DAG, typename Epi>
__global__ __launch_bounds__(256) void k_hop(Geom g, int nbp, int p_fixed, HopIn<R> hin, Epi epi,
                                             double* partials) {
  if (epi.skip()) return;
  __shared__ R2<R> lds[4][12][64];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int p = p_fixed >= 0 ? p_fixed : lb / nbp;
  const int blk = p_fixed >= 0 ? lb : lb % nbp;
  const int lane = threadIdx.x & 63;
  const int mu = threadIdx.x >> 6;
  const int cb = blk * 64 + lane;
  const bool active = cb < g.vh;

  C<R> acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = czero<R>();
  if (active) {
    int c[4];
    cb_coords(g, p, cb, c);
    const R2<R>* in = p ? hin.in_even : hin.in_odd;
    switch (mu) {
      case 0: hop_dir<R, 0, DAG>(g, hin.gauge, in, p, cb, c, acc, 1, 0); break;
      case 1: hop_dir<R, 1, DAG>(g, hin.gauge, in, p, cb, c, acc, 1, 0); break;
      case 2: hop_dir<R, 2, DAG>(g, hin.gauge, in, p, cb, c, acc, 1, 0); break;
      default: hop_dir<R, 3, DAG>(g, hin.gauge, in, p, cb, c, acc, 1, 0); break;
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
  // wave `mu` now owns spin component `mu` of the 64 sites
  const int spin = mu;
  C<R> out[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int k = 3 * spin + i;
    R2<R> a = lds[0][k][lane], b = lds[1][k][lane], cc = lds[2][k][lane], d = lds[3][k][lane];
    out[i] = cmk<R>(((a.x + b.x) + cc.x) + d.x, ((a.y + b.y) + cc.y) + d.y);
  }
  double red = 0.0;
  if (active) epi.apply(p, cb, spin, out, red);
  if constexpr (Epi::kReduce) {
    double v[1] = {red};
    block_partials<256, 1>(v, partials, lb);
  }
  epi.template tail<256>();
}

// ---------------------------------------------------------------------------
// Eight-wave variant: wave w = (mu = w/2, a = w%2) computes, for 64 sites,
// both hops along mu for projected spin component a only.  In the chiral
// basis B_mu has one non-zero per row, (B_mu d)_a = f_{mu,a} d_{b(a)} with
// b = swap (mu = 0, 1) or identity (mu = 2, 3) and f in {+-1, +-i}, so a
// thread needs half of each neighbour spinor, and its W_a = U h_a feeds
// exactly two output spin components: up_a and dn_{b(a)} (with factor
// S conj(f)).  Twice as many threads per site as k_hop, same LDS footprint.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ C<R> phase_mul(int f, C<R> v) {  // f: 0 -> 1, 1 -> -1, 2 -> i, 3 -> -i
  return f == 0 ? v : (f == 1 ? -v : (f == 2 ? itimes(v) : -itimes(v)));
}
// f_{mu,a} as a phase code and b(a)
__device__ __forceinline__ void bmap(int mu, int a, int& f, int& b) {
  // mu 0: (Bd) = (-i d1, -i d0); mu 1: (-d1, d0); mu 2: (-i d0, i d1); mu 3: (d0, d1)
  const int tab_f[4][2] = {{3, 3}, {1, 0}, {3, 2}, {0, 0}};
  f = tab_f[mu][a];
  b = mu < 2 ? 1 - a : a;
}
__device__ __forceinline__ int conj_phase(int f) { return f < 2 ? f : (f == 2 ? 3 : 2); }

template <typename R, int MU, bool DAG>
__device__ __forceinline__ void hop_dir_half(const Geom& g, const R2<R>* __restrict__ gauge,
                                             const R2<R>* __restrict__ in, int p, int cb, const int c[4], int a,
                                             C<R>* up, C<R>* dn) {
  constexpr int SF = DAG ? +1 : -1;
  const int vh = g.vh;
  int f, b;
  bmap(MU, a, f, b);
  const int fr = conj_phase(f);  // reconstruction factor conj(f)
#pragma unroll
  for (int dir = 0; dir < 2; ++dir) {
    const int S = dir == 0 ? SF : -SF;
    const int n = cb_shift(g, c, MU, dir == 0 ? +1 : -1);
    C<R> h[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const C<R> u = ld<R>(in + (size_t)(3 * a + i) * vh + n);
      const C<R> d = ld<R>(in + (size_t)(6 + 3 * b + i) * vh + n);
      const C<R> bd = phase_mul<R>(f, d);
      h[i] = S > 0 ? u + bd : u - bd;
    }
    const M3<R> U = load_m3<R>(gptr<R>(gauge, g, dir == 0 ? p : 1 - p, MU), vh, dir == 0 ? cb : n);
    C<R> w[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      C<R> sacc;
      if (dir == 0) {
        sacc = U.m[3 * i] * h[0];
        sacc += U.m[3 * i + 1] * h[1];
        sacc += U.m[3 * i + 2] * h[2];
      } else {
        sacc = cjmul(U.m[i], h[0]);
        sacc += cjmul(U.m[3 + i], h[1]);
        sacc += cjmul(U.m[6 + i], h[2]);
      }
      w[i] = sacc;
    }
    const bool edge = MU == 3 && (dir == 0 ? c[3] == g.L[3] - 1 : c[3] == 0);
    const R sg = edge ? R(g.bc) : R(1);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const C<R> wv = sg * w[i];
      up[i] += wv;
      const C<R> t = phase_mul<R>(fr, wv);
      if (S > 0) dn[i] += t;
      else dn[i] -= t;
    }
  }
}

template <typename R, bool DAG, typename Epi>
__global__ __launch_bounds__(512) void k_hop8(Geom g, int nbp, int p_fixed, HopIn<R> hin, Epi epi,
                                              double* partials) {
  if (epi.skip()) return;
  __shared__ R2<R> lds[8][6][64];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int p = p_fixed >= 0 ? p_fixed : lb / nbp;
  const int blk = p_fixed >= 0 ? lb : lb % nbp;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int mu = w >> 1, a = w & 1;
  const int cb = blk * 64 + lane;
  const bool active = cb < g.vh;
  C<R> up[3], dn[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) up[i] = dn[i] = czero<R>();
  if (active) {
    int c[4];
    cb_coords(g, p, cb, c);
    const R2<R>* in = p ? hin.in_even : hin.in_odd;
    switch (mu) {
      case 0: hop_dir_half<R, 0, DAG>(g, hin.gauge, in, p, cb, c, a, up, dn); break;
      case 1: hop_dir_half<R, 1, DAG>(g, hin.gauge, in, p, cb, c, a, up, dn); break;
      case 2: hop_dir_half<R, 2, DAG>(g, hin.gauge, in, p, cb, c, a, up, dn); break;
      default: hop_dir_half<R, 3, DAG>(g, hin.gauge, in, p, cb, c, a, up, dn); break;
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    R2<R> v;
    v.x = up[i].re;
    v.y = up[i].im;
    lds[w][i][lane] = v;
    v.x = dn[i].re;
    v.y = dn[i].im;
    lds[w][3 + i][lane] = v;
  }
  __syncthreads();
  double red = 0.0;
#pragma unroll
  for (int kk = 0; kk < 2; ++kk) {
    const int k = w + 8 * kk;  // output component 3*spin + colour
    if (k >= 12) break;
    const int sp = k / 3, i = k % 3;
    R re = R(0), im = R(0);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      // up spin sp comes from wave (m, a = sp); dn spin c = sp-2 from (m, a = b_m^{-1}(c))
      const int src = sp < 2 ? 2 * m + sp : 2 * m + (m < 2 ? 1 - (sp - 2) : sp - 2);
      const R2<R> v = lds[src][sp < 2 ? i : 3 + i][lane];
      re += v.x;
      im += v.y;
    }
    if (active) epi.apply1(p, cb, k, cmk<R>(re, im), red);
  }
  if constexpr (Epi::kReduce) {
    double v[1] = {red};
    block_partials<512, 1>(v, partials, lb);
  }
  epi.template tail<512>();
}

static inline int nblk_parity(const Geom& g) { return (g.vh + 63) / 64; }

// Hop decomposition: 4 waves (one per direction, the default: faster on
// MI355X at 16^4 and above) or 8 waves (direction x projected spin
// component) per 64-site block; LGT_HOP_WAVES=8 selects the latter.
static int hop_waves() {
  static int w = [] {
    const char* e = getenv("LGT_HOP_WAVES");
    return (e && atoi(e) == 8) ? 8 : 4;
  }();
  return w;
}

template <typename R, bool DAG, typename Epi>
static hipError_t launch(const Geom& g, int p_out, const HopIn<R>& hin, const Epi& epi, double* partials,
                         hipStream_t s, int capacity = 0) {
  const int nbp = nblk_parity(g);
  const int nb = p_out >= 0 ? nbp : 2 * nbp;
  if (Epi::kReduce && nb > capacity) return hipErrorInvalidValue;
  if (hop_waves() == 8)
    hipLaunchKernelGGL((k_hop8<R, DAG, Epi>), dim3(nb), dim3(512), 0, s, g, nbp, p_out, hin, epi, partials);
  else
    hipLaunchKernelGGL((k_hop<R, DAG, Epi>), dim3(nb), dim3(256), 0, s, g, nbp, p_out, hin, epi, partials);
  return hipGetLastError();
}

int hop_blocks(const Geom& g, int p_out) { return p_out >= 0 ? nblk_parity(g) : 2 * nblk_parity(g); }

template <typename R, bool DAG>
hipError_t launch_hop_axpy(const Geom& g, int p_out, HopIn<R> hin, R2<R>* out_even, R2<R>* out_odd,
                           const R2<R>* self_even, const R2<R>* self_odd, double coef, hipStream_t s,
                           SolverState* guard, const double* pap_partials) {
  EpiAxpy<R> e;
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

template <typename R, bool DAG>
hipError_t launch_hop_schur_norm(const Geom& g, HopIn<R> hin, R2<R>* w, const R2<R>* x, double coef,
                                 SolverState* st, Reduce red, hipStream_t s) {
  EpiSchurNorm<R> e{w, x, R(coef), g.vh, st};
  return launch<R, DAG>(g, 1, hin, e, red.partials, s, red.capacity);
}

template <typename R, bool DAG>
hipError_t launch_hop_schur_cg(const Geom& g, HopIn<R> hin, const R2<R>* w, R2<R>* x, R2<R>* r,
                               const R2<R>* p, double coef, SolverState* st, Reduce red,
                               hipStream_t s) {
  EpiSchurCG<R> e{w, x, r, p, R(coef), g.vh, st};
  hipError_t err = launch<R, DAG>(g, 1, hin, e, red.partials, s, red.capacity);
  if (err != hipSuccess) return err;
  return launch_finalize(kFinCgStep, nblk_parity(g), red, st, 0, 0.0, 0, s);
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

#define LGT_INST_HOP(R, DAG)                                                                          \
  template hipError_t launch_hop_axpy<R, DAG>(const Geom&, int, HopIn<R>, R2<R>*, R2<R>*, const R2<R>*, \
                                               const R2<R>*, double, hipStream_t, SolverState*,       \
                                               const double*);                                        \
  template hipError_t launch_hop_schur_norm<R, DAG>(const Geom&, HopIn<R>, R2<R>*, const R2<R>*,      \
                                                     double, SolverState*, Reduce, hipStream_t);     \
  template hipError_t launch_hop_schur_cg<R, DAG>(const Geom&, HopIn<R>, const R2<R>*, R2<R>*,        \
                                                   R2<R>*, const R2<R>*, double, SolverState*, Reduce, \
                                                   hipStream_t);

LGT_INST_HOP(double, false)
LGT_INST_HOP(double, true)
LGT_INST_HOP(float, false)
LGT_INST_HOP(float, true)

template hipError_t launch_hop_residual<false>(const Geom&, HopIn<double>, const double2*, const double2*,
                                               double2*, double, Reduce, int, hipStream_t);
template hipError_t launch_hop_residual<true>(const Geom&, HopIn<double>, const double2*, const double2*,
                                              double2*, double, Reduce, int, hipStream_t);

}  // namespace lgt
