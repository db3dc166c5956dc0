// Multi-right-hand-side kernels: nr spinor fields on one lattice, solved
// together (one pseudofermion per right-hand side, each with its own kappa).
//
// Layout of a multi-RHS half field: [12 components][nr][V/2 sites] complex
// (site fastest), a full field the even half then the odd half.  Every
// per-component access of a wave is unit stride, as in the single field.
//
// Hop decomposition: a 256-thread block owns 64 consecutive sites of one
// parity and a group of G right-hand sides; wave w (= direction mu) loads
// the two links of its direction once, keeps them in registers (FP32; FP64
// reloads them per right-hand side to stay clear of spills) and then, for
// each right-hand side of the group in turn, computes both hops along mu,
// meets the other waves in LDS and runs the epilogue for spin component w.
// The link traffic is paid once per group instead of once per field, and
// the neighbour index arithmetic once per block.  G trades link reuse
// (large G) against parallelism (small G gives more blocks); the host picks
// it by timing (see batch.hip).  Per-RHS reductions are deterministic: a
// fixed-order wave reduction, then the four waves in order, one partial per
// (site block, right-hand side), summed by a one-block finalize launch.
#include <type_traits>

#include "lgt_internal.h"
#include "lgt_hop.h"
#include "lgt_mrhs.h"

namespace lgt {

// ---------------------------------------------------------------------------
// Epilogues (element (k, n, cb) of the hop result, offset o).  rhs_active(n)
// false: nothing of right-hand side n in this launch is used (its CG has
// stopped: converged, or idle until the next reliable update), so the
// kernel skips its hop and writes 0 for its partial.
// ---------------------------------------------------------------------------
template <typename R>
struct MEpiAxpy {  // out = self + coef_n * acc
  static constexpr bool kReduce = false;
  R2<R>* out[2];
  const R2<R>* self[2];
  const double* coef;  // [NR] device array
  const BatchState* guard;
  const double* mask;  // if set: right-hand side n is computed only where mask[n] != 0
  const double* pap_partials;  // block 0 forms alpha_n (see tail)
  int pap_nblk;
  BatchState* state;
  __device__ bool skip() const { return guard && guard->all_done; }
  __device__ bool rhs_active(int n) const {
    return (!mask || mask[n] != 0.0) && (!guard || guard->done[n] == kDoneRunning);
  }
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
  __device__ bool rhs_active(int n) const { return state->done[n] == kDoneRunning; }
  __device__ void apply(int, size_t o, int n, C<R> a, double& red) const {
    const C<R> v = ld<R>(x + o) + R(coef[n]) * a;
    st<R>(w + o, v);
    red += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
  }
  __device__ void tail(int) const {}
};

template <typename R>
struct MEpiSchurCG {  // q = w + coef_n acc; r -= alpha_n q (unless converged); x += alpha_n p if x is set
  static constexpr bool kReduce = true;
  const R2<R>* w;
  R2<R>* x;
  R2<R>* r;
  const R2<R>* p;
  const double* coef;
  const BatchState* state;
  __device__ bool skip() const { return state->all_done; }
  __device__ bool rhs_active(int n) const { return state->done[n] == kDoneRunning; }
  __device__ void apply(int, size_t o, int n, C<R> a, double& red) const {
    C<R> rv = ld<R>(r + o);
    if (!state->done[n]) {
      const R alpha = R(state->alpha[n]);
      const C<R> q = ld<R>(w + o) + R(coef[n]) * a;
      if (x) st<R>(x + o, ld<R>(x + o) + alpha * ld<R>(p + o));
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
  __device__ bool rhs_active(int) const { return true; }
  __device__ void apply(int p, size_t o, int n, C<double> a, double& red) const {
    const C<double> v = ld<double>(phi[p] + o) - (ld<double>(self[p] + o) + coef[n] * a);
    st<double>(r[p] + o, v);
    red += norm2(v);
  }
  __device__ void tail(int) const {}
};


// Loader of one right-hand side of a multi-RHS field: element (k, n, site)
// at (k*nr + n)*vh + site; the per-lane offset carries site and n, the
// component offset is uniform.
template <typename R>
struct MrhsIn {
  BufRsrc rs;
  unsigned ks;  // component stride in bytes (nr * vh elements)
  unsigned ns;  // right-hand-side stride in bytes (vh elements)
  __device__ __forceinline__ unsigned off(int site, int n) const {
    return (unsigned)site * (unsigned)sizeof(R2<R>) + (unsigned)n * ns;
  }
  __device__ __forceinline__ C<R> ld(unsigned o, int k) const { return ld_buf<R>(rs, o, k * ks); }
};

// wave-level sum in a fixed butterfly order (all 64 lanes get the total)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename R, bool DAG, typename Epi>
__global__ __launch_bounds__(256) void k_hop_mrhs(Geom g, int nr, int G, int nbp, int ngrp, int p_fixed,
                                                  HopIn<R> hin, Epi epi, double* partials) {
  if (epi.skip()) return;
  __shared__ R2<R> lds[4][12][64];
  __shared__ double wred[4][kMaxRhs];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int per_par = nbp * ngrp;
  const int p = p_fixed >= 0 ? p_fixed : lb / per_par;
  const int rem = p_fixed >= 0 ? lb : lb % per_par;
  const int blk = rem / ngrp, grp = rem - blk * ngrp;  // neighbouring blocks share a site block
  const int n0 = grp * G, n1 = min(nr, n0 + G);
  const int lane = threadIdx.x & 63;
  const int mu = threadIdx.x >> 6;
  const int cb = blk * 64 + lane;
  const bool active = cb < g.vh;
  // the group's running right-hand sides, read once per block so that every
  // thread skips the same ones (a later write to the state by another block
  // concerns a right-hand side whose results this launch no longer needs)
  __shared__ unsigned s_act;
  if (threadIdx.x == 0) {
    unsigned m = 0;
    for (int n = n0; n < n1; ++n) m |= (epi.rhs_active(n) ? 1u : 0u) << (n - n0);
    s_act = m;
  }
  if (threadIdx.x < 4 * kMaxRhs) wred[threadIdx.x / kMaxRhs][threadIdx.x % kMaxRhs] = 0.0;
  __syncthreads();
  const unsigned act = s_act;
  constexpr unsigned E = sizeof(R2<R>);
  const unsigned gs = (unsigned)g.vh * E;
  const unsigned ns = (unsigned)g.vh * E;
  const MrhsIn<R> in{make_rsrc(p ? hin.in_even : hin.in_odd, (size_t)12 * nr * ns), (unsigned)nr * ns, ns};
  int c[4] = {0, 0, 0, 0};
  int nf = 0, nb = 0;
  if (active) {
    cb_coords(g, p, cb, c);
    nf = cb_shift(g, c, mu, +1);
    nb = cb_shift(g, c, mu, -1);
  }
  // links [2][4][nk][vh]: all nine components, or (FP32) the first two rows
  // of SU(3) links with the third rebuilt in registers (a third less link
  // traffic per group, as in the single-field hop)
  const int nk = hin.nk;
  const BufRsrc ruf = make_rsrc(hin.gauge + (size_t)((p * 4 + mu) * nk) * g.vh, (size_t)nk * gs);
  const BufRsrc rub = make_rsrc(hin.gauge + (size_t)(((1 - p) * 4 + mu) * nk) * g.vh, (size_t)nk * gs);
  constexpr bool kKeepLinks = sizeof(R) == 4;
  M3<R> Uf, Ub;
#pragma unroll
  for (int k = 0; k < 9; ++k) Uf.m[k] = Ub.m[k] = czero<R>();
  if (kKeepLinks && active && act) {
    if (nk == 9) {
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        Uf.m[k] = ld_buf<R>(ruf, (unsigned)cb * E, k * gs);
        Ub.m[k] = ld_buf<R>(rub, (unsigned)nb * E, k * gs);
      }
    } else {
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        Uf.m[k] = ld_buf<R>(ruf, (unsigned)cb * E, k * gs);
        Ub.m[k] = ld_buf<R>(rub, (unsigned)nb * E, k * gs);
      }
      Uf.m[6] = conj(Uf.m[1] * Uf.m[5] - Uf.m[2] * Uf.m[4]);
      Uf.m[7] = conj(Uf.m[2] * Uf.m[3] - Uf.m[0] * Uf.m[5]);
      Uf.m[8] = conj(Uf.m[0] * Uf.m[4] - Uf.m[1] * Uf.m[3]);
      Ub.m[6] = conj(Ub.m[1] * Ub.m[5] - Ub.m[2] * Ub.m[4]);
      Ub.m[7] = conj(Ub.m[2] * Ub.m[3] - Ub.m[0] * Ub.m[5]);
      Ub.m[8] = conj(Ub.m[0] * Ub.m[4] - Ub.m[1] * Ub.m[3]);
    }
  }
  for (int n = n0; n < n1; ++n) {
    if (!((act >> (n - n0)) & 1u)) continue;  // uniform: the block's mask
    C<R> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = czero<R>();
    if (active) {
      if (!kKeepLinks) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          Uf.m[k] = ld_buf<R>(ruf, (unsigned)cb * E, k * gs);
          Ub.m[k] = ld_buf<R>(rub, (unsigned)nb * E, k * gs);
        }
      }
      const unsigned of = in.off(nf, n), ob = in.off(nb, n);
      switch (mu) {
        case 0: hop_dir_u<R, 0, DAG>(g, Uf, Ub, in, of, ob, c, acc); break;
        case 1: hop_dir_u<R, 1, DAG>(g, Uf, Ub, in, of, ob, c, acc); break;
        case 2: hop_dir_u<R, 2, DAG>(g, Uf, Ub, in, of, ob, c, acc); break;
        default: hop_dir_u<R, 3, DAG>(g, Uf, Ub, in, of, ob, c, acc); break;
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
        epi.apply(p, ((size_t)k * nr + n) * g.vh + cb, n,
                  cmk<R>(((a.x + b.x) + cc.x) + d.x, ((a.y + b.y) + cc.y) + d.y), red);
      }
    }
    if constexpr (Epi::kReduce) {
      red = wave_sum(red);
      if (lane == 0) wred[mu][n - n0] = red;
    }
    __syncthreads();
  }
  if constexpr (Epi::kReduce) {
    const int t = threadIdx.x;
    if (t < n1 - n0) {
      const int row = p_fixed >= 0 ? blk : p * nbp + blk;
      partials[(size_t)row * kMaxRhs + n0 + t] = ((wred[0][t] + wred[1][t]) + wred[2][t]) + wred[3][t];
    }
  }
  epi.tail(nr);
}

// ---------------------------------------------------------------------------
// MFMA form of the FP32 batched hop.  Per site x, direction mu and sign, the
// hop applies one link to the projected half spinors of every right-hand
// side of the group: W = U H, a complex 3 x (2 G) product, i.e. the real
// product [[Ur, -Ui], [Ui, Ur]] (6 x 6) times [Hr; Hi] (6 x 2G).  Every
// site has its own U, so the product runs on v_mfma_f32_4x4x1_16b_f32,
// whose 16 independent 4x4 blocks take 16 sites per instruction: block b
// (lanes 4b..4b+3) is site b of the wave's 16; its output rows are the
// real-form rows (Re W_0, Re W_1, Re W_2, Im W_0 | Im W_1, Im W_2, -, -)
// in two row tiles, its columns (spin, right-hand side) in 2G/4 column
// tiles, and the six real input components are six rank-1 steps.  Lane j
// of a block feeds row j of the link operand and column j of the spinor
// operand, and receives column j of every output tile: the whole W of
// right-hand sides j (and j + 4 for G = 8), both spins.  So the lane that
// projects a right-hand side's neighbour spinor is also the lane that
// reconstructs its W, and the link is loaded once per site (each lane one
// or two of its rows).  A 256-thread block takes 16 sites of one parity
// and a group of G right-hand sides; wave w takes direction mu = w (both
// hops); the four directions meet in LDS as in k_hop_mrhs and the same
// epilogues run.  Reductions: per right-hand side, a fixed-order sum over
// the threads that own it, then one partial per (block, right-hand side).
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));

// Rows of the real-form link operand fed by lane j (0..3): tile 0 row j,
// tile 1 row j, as six values over the input components (Re h_c, Im h_c).
// Forward: the link U; backward: U^dag (rows of U^dag = conjugated columns).
template <bool ADJ>
__device__ __forceinline__ void link_rows(const BufRsrc& ru, unsigned o, unsigned gs, int j, float* a0,
                                          float* a1) {
  // element (i, c) of the operator and its real and imaginary parts
  auto el = [&](int i, int c) -> C<float> {
    const C<float> u = ADJ ? ld_buf<float>(ru, o, (3 * c + i) * gs) : ld_buf<float>(ru, o, (3 * i + c) * gs);
    return ADJ ? conj(u) : u;
  };
  if (j < 3) {  // tile 0: Re W_j = sum_c Re u_jc Re h_c - Im u_jc Im h_c
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const C<float> u = el(j, c);
      a0[c] = u.re;
      a0[3 + c] = -u.im;
    }
  } else {      // tile 0 row 3: Im W_0 = sum_c Im u_0c Re h_c + Re u_0c Im h_c
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const C<float> u = el(0, c);
      a0[c] = u.im;
      a0[3 + c] = u.re;
    }
  }
  if (j < 2) {  // tile 1 rows 0, 1: Im W_1, Im W_2
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const C<float> u = el(j + 1, c);
      a1[c] = u.im;
      a1[3 + c] = u.re;
    }
  } else {
#pragma unroll
    for (int c = 0; c < 6; ++c) a1[c] = 0.f;
  }
}

// W (2 spins x 3 colours) of the right-hand side in column tiles (c0, c1)
// (spin 0, spin 1) from the accumulators
__device__ __forceinline__ void tile_w(const v4f (*acc)[4], int c0, int c1, C<float>* w) {
  const int cs[2] = {c0, c1};
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int c = cs[a];
    w[3 * a + 0] = cmk<float>(acc[0][c][0], acc[0][c][3]);
    w[3 * a + 1] = cmk<float>(acc[0][c][1], acc[1][c][0]);
    w[3 * a + 2] = cmk<float>(acc[0][c][2], acc[1][c][1]);
  }
}

// One hop (forward: U_mu(x) psi(x + mu) with projector 1 + S gamma_mu;
// backward: U_mu(x - mu)^dag psi(x - mu) with 1 + S gamma_mu) of the lane's
// right-hand sides, added to out[0..NL-1][12].
template <int MU, int S, bool ADJ, int G>
__device__ __forceinline__ void mfma_hop(const MrhsIn<float>& in, unsigned osite, const BufRsrc& ru, unsigned olink,
                                         unsigned gs, int j, int n0, unsigned live, bool bc, float bcs,
                                         C<float> (*out)[12]) {
  constexpr int NL = G / 4;       // right-hand sides per lane
  constexpr int NCT = 2 * G / 4;  // column tiles
  float a0[6], a1[6];
  link_rows<ADJ>(ru, olink, gs, j, a0, a1);
  C<float> h[NL][6];
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int nl = j + 4 * q;
    if ((live >> nl) & 1u) {
      C<float> psi[12];
      const unsigned o = in.off(0, n0 + nl) + osite;
#pragma unroll
      for (int k = 0; k < 12; ++k) psi[k] = in.ld(o, k);
      project<float, MU, S>(psi, h[q]);
    } else {
#pragma unroll
      for (int k = 0; k < 6; ++k) h[q][k] = czero<float>();
    }
  }
  v4f acc[2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = v4f{0.f, 0.f, 0.f, 0.f};
  // column tile c: spin c / NL, right-hand side (lane's) c % NL
#pragma unroll
  for (int k = 0; k < 6; ++k) {
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      const C<float> hv = h[c % NL][3 * (c / NL) + (k % 3)];
      const float b = k < 3 ? hv.re : hv.im;
      acc[0][c] = __builtin_amdgcn_mfma_f32_4x4x1f32(a0[k], b, acc[0][c], 0, 0, 0);
      acc[1][c] = __builtin_amdgcn_mfma_f32_4x4x1f32(a1[k], b, acc[1][c], 0, 0, 0);
    }
  }
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    C<float> w[6];
    tile_w(acc, q, NL + q, w);
    if (bc) {
#pragma unroll
      for (int k = 0; k < 6; ++k) w[k] = bcs * w[k];
    }
    reconstruct<float, MU, S>(w, out[q]);
  }
}

template <int MU, bool DAG, int G>
__device__ __forceinline__ void mfma_dir(const Geom& g, const MrhsIn<float>& in, const float2* gauge, int p, int cb,
                                         const int c[4], int j, int n0, unsigned live, C<float> (*out)[12]) {
  constexpr int SF = DAG ? +1 : -1;
  constexpr unsigned E = sizeof(float2);
  const unsigned gs = (unsigned)g.vh * E;
  const int nf = cb_shift(g, c, MU, +1), nb = cb_shift(g, c, MU, -1);
  const BufRsrc ruf = make_rsrc(gptr<float>(gauge, g, p, MU), (size_t)9 * gs);
  const BufRsrc rub = make_rsrc(gptr<float>(gauge, g, 1 - p, MU), (size_t)9 * gs);
  const float bcs = (float)g.bc;
  mfma_hop<MU, SF, false, G>(in, (unsigned)nf * E, ruf, (unsigned)cb * E, gs, j, n0, live,
                             MU == 3 && c[3] == g.L[3] - 1, bcs, out);
  mfma_hop<MU, -SF, true, G>(in, (unsigned)nb * E, rub, (unsigned)nb * E, gs, j, n0, live, MU == 3 && c[3] == 0,
                             bcs, out);
}

template <bool DAG, typename Epi, int G>
__global__ __launch_bounds__(256) void k_hop_mrhs_mfma(Geom g, int nr, int nbp, int ngrp, int p_fixed,
                                                       HopIn<float> hin, Epi epi, double* partials) {
  if (epi.skip()) return;
  constexpr int NL = G / 4;
  __shared__ float2 lds[4][G][12][16];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int per_par = nbp * ngrp;
  const int p = p_fixed >= 0 ? p_fixed : lb / per_par;
  const int rem = p_fixed >= 0 ? lb : lb % per_par;
  const int blk = rem / ngrp, grp = rem - blk * ngrp;
  const int n0 = grp * G, ng = min(G, nr - n0);
  const int lane = threadIdx.x & 63;
  const int mu = threadIdx.x >> 6;
  const int j = lane & 3, sb = lane >> 2;
  const int cb = blk * 16 + sb;
  const bool active = cb < g.vh;
  __shared__ unsigned s_act;
  if (threadIdx.x == 0) {
    unsigned m = 0;
    for (int n = 0; n < ng; ++n) m |= (epi.rhs_active(n0 + n) ? 1u : 0u) << n;
    s_act = m;
  }
  __syncthreads();
  const unsigned act = s_act;
  constexpr unsigned E = sizeof(float2);
  const unsigned ns = (unsigned)g.vh * E;
  const MrhsIn<float> in{make_rsrc(p ? hin.in_even : hin.in_odd, (size_t)12 * nr * ns), (unsigned)nr * ns, ns};
  C<float> out[NL][12];
#pragma unroll
  for (int q = 0; q < NL; ++q)
#pragma unroll
    for (int k = 0; k < 12; ++k) out[q][k] = czero<float>();
  // every lane of the wave runs the MFMA (inactive sites read site 0 and
  // are not stored); a block whose group has no running right-hand side
  // skips the work
  if (act) {
    int c[4] = {0, 0, 0, 0};
    cb_coords(g, p, active ? cb : 0, c);
    switch (mu) {
      case 0: mfma_dir<0, DAG, G>(g, in, hin.gauge, p, active ? cb : 0, c, j, n0, act, out); break;
      case 1: mfma_dir<1, DAG, G>(g, in, hin.gauge, p, active ? cb : 0, c, j, n0, act, out); break;
      case 2: mfma_dir<2, DAG, G>(g, in, hin.gauge, p, active ? cb : 0, c, j, n0, act, out); break;
      default: mfma_dir<3, DAG, G>(g, in, hin.gauge, p, active ? cb : 0, c, j, n0, act, out); break;
    }
  }
#pragma unroll
  for (int q = 0; q < NL; ++q)
#pragma unroll
    for (int k = 0; k < 12; ++k) lds[mu][j + 4 * q][k][sb] = make_float2(out[q][k].re, out[q][k].im);
  __syncthreads();
  // epilogue: thread t owns right-hand side nl = t / (256 / G) of the group
  // and components k = kq, kq + KS, ... of site t % 16
  constexpr int TPR = 256 / G;   // threads per right-hand side (32 or 64)
  constexpr int KS = TPR / 16;   // component stride (2 or 4)
  const int nl = threadIdx.x / TPR, q = threadIdx.x % TPR;
  const int site = q & 15, kq = q >> 4;
  const int ocb = blk * 16 + site;
  const bool run = nl < ng && ((act >> nl) & 1u) && ocb < g.vh;
  double red = 0.0;
  if (run) {
    const int n = n0 + nl;
#pragma unroll
    for (int k = kq; k < 12; k += KS) {
      const float2 a = lds[0][nl][k][site], b = lds[1][nl][k][site], cc = lds[2][nl][k][site],
                   d = lds[3][nl][k][site];
      epi.apply(p, ((size_t)k * nr + n) * g.vh + ocb, n, cmk<float>(((a.x + b.x) + cc.x) + d.x,
                                                                     ((a.y + b.y) + cc.y) + d.y), red);
    }
  }
  if constexpr (Epi::kReduce) {
#pragma unroll
    for (int o = TPR / 2; o > 0; o >>= 1) red += __shfl_xor(red, o, 64);
    if (q == 0 && nl < ng) {
      const int row = p_fixed >= 0 ? blk : p * nbp + blk;
      partials[(size_t)row * kMaxRhs + n0 + nl] = red;
    }
  }
  epi.tail(nr);
}

// site blocks per parity of the batched hop: 64 sites (VALU kernel, G > 0)
// or 16 sites (MFMA kernel, G = -4 or -8)
static inline int mrhs_nbp(const Geom& g, int G = 1) { return G < 0 ? (g.vh + 15) / 16 : (g.vh + 63) / 64; }

template <typename R, bool DAG, typename Epi>
static hipError_t mlaunch(const Geom& g, int nr, int G, int p_out, const HopIn<R>& hin, const Epi& epi, Reduce red,
                          hipStream_t s) {
  if (nr < 1 || nr > kMaxRhs) return hipErrorInvalidValue;
  if (hin.nk != 9 && (hin.nk != 6 || sizeof(R) != 4)) return hipErrorInvalidValue;  // two-row links: FP32 only
  const int gs = G < 0 ? -G : G;
  if (gs < 1 || gs > kMaxRhs || (G < 0 && gs != 4 && gs != 8)) return hipErrorInvalidValue;
  const int nbp = mrhs_nbp(g, G);
  const int ngrp = (nr + gs - 1) / gs;
  const int rows = p_out >= 0 ? nbp : 2 * nbp;
  if (Epi::kReduce && (size_t)rows * kMaxRhs > red.ndoubles) return hipErrorInvalidValue;
  if (G < 0) {
    if (hin.nk != 9) return hipErrorInvalidValue;  // the MFMA form reads full links
    if constexpr (std::is_same<R, float>::value) {
      if (gs == 8)
        hipLaunchKernelGGL((k_hop_mrhs_mfma<DAG, Epi, 8>), dim3(rows * ngrp), dim3(256), 0, s, g, nr, nbp, ngrp,
                           p_out, hin, epi, red.partials);
      else
        hipLaunchKernelGGL((k_hop_mrhs_mfma<DAG, Epi, 4>), dim3(rows * ngrp), dim3(256), 0, s, g, nr, nbp, ngrp,
                           p_out, hin, epi, red.partials);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;  // the MFMA form is FP32 only
    }
  }
  hipLaunchKernelGGL((k_hop_mrhs<R, DAG, Epi>), dim3(rows * ngrp), dim3(256), 0, s, g, nr, G, nbp, ngrp, p_out, hin,
                     epi, red.partials);
  return hipGetLastError();
}

// largest number of partial rows a reducing batched hop writes (the 16-site MFMA blocks)
int mrhs_hop_blocks(const Geom& g, int p_out) { return p_out >= 0 ? mrhs_nbp(g, -8) : 2 * mrhs_nbp(g, -8); }

template <typename R, bool DAG>
hipError_t launch_mhop_axpy(const Geom& g, int nr, int G, int p_out, HopIn<R> hin, R2<R>* out_e, R2<R>* out_o,
                            const R2<R>* self_e, const R2<R>* self_o, const double* coef, hipStream_t s,
                            BatchState* guard, const double* pap_partials, Reduce red, const double* mask) {
  MEpiAxpy<R> e;
  e.mask = mask;
  e.out[0] = out_e;
  e.out[1] = out_o;
  e.self[0] = self_e;
  e.self[1] = self_o;
  e.coef = coef;
  e.guard = guard;
  e.pap_partials = pap_partials;
  e.pap_nblk = mrhs_nbp(g, G);
  e.state = guard;
  return mlaunch<R, DAG>(g, nr, G, p_out, hin, e, red, s);
}

template <typename R, bool DAG>
hipError_t launch_mhop_schur_norm(const Geom& g, int nr, int G, HopIn<R> hin, R2<R>* w, const R2<R>* x,
                                  const double* coef, BatchState* st, Reduce red, hipStream_t s) {
  MEpiSchurNorm<R> e{w, x, coef, st};
  return mlaunch<R, DAG>(g, nr, G, 1, hin, e, red, s);
}

template <typename R, bool DAG>
hipError_t launch_mhop_schur_cg(const Geom& g, int nr, int G, HopIn<R> hin, const R2<R>* w, R2<R>* x, R2<R>* r,
                                const R2<R>* p, const double* coef, BatchState* st, Reduce red, hipStream_t s) {
  MEpiSchurCG<R> e{w, x, r, p, coef, st};
  hipError_t err = mlaunch<R, DAG>(g, nr, G, 1, hin, e, red, s);
  if (err != hipSuccess) return err;
  return launch_mfinalize(kFinCgStep, mrhs_nbp(g, G), nr, red, st, 0.0, 0, s);
}

template <bool DAG>
hipError_t launch_mhop_residual(const Geom& g, int nr, int G, HopIn<double> hin, const double2* self_full,
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
  hipError_t err = mlaunch<double, DAG>(g, nr, G, -1, hin, e, red, s);
  if (err != hipSuccess) return err;
  return launch_mfinalize(kFinResult1, 2 * mrhs_nbp(g, G), nr, red, nullptr, 0.0, 0, s);
}

#define LGT_INST_MHOP(R, DAG)                                                                                   \
  template hipError_t launch_mhop_axpy<R, DAG>(const Geom&, int, int, int, HopIn<R>, R2<R>*, R2<R>*,             \
                                                const R2<R>*, const R2<R>*, const double*, hipStream_t,          \
                                                BatchState*, const double*, Reduce, const double*);              \
  template hipError_t launch_mhop_schur_norm<R, DAG>(const Geom&, int, int, HopIn<R>, R2<R>*, const R2<R>*,      \
                                                      const double*, BatchState*, Reduce, hipStream_t);         \
  template hipError_t launch_mhop_schur_cg<R, DAG>(const Geom&, int, int, HopIn<R>, const R2<R>*, R2<R>*, R2<R>*, \
                                                    const R2<R>*, const double*, BatchState*, Reduce, hipStream_t);

LGT_INST_MHOP(double, false)
LGT_INST_MHOP(double, true)
LGT_INST_MHOP(float, false)
LGT_INST_MHOP(float, true)
template hipError_t launch_mhop_residual<false>(const Geom&, int, int, HopIn<double>, const double2*,
                                                const double2*, double2*, const double*, Reduce, hipStream_t);
template hipError_t launch_mhop_residual<true>(const Geom&, int, int, HopIn<double>, const double2*,
                                               const double2*, double2*, const double*, Reduce, hipStream_t);

// ---------------------------------------------------------------------------
// Vector kernels over multi-RHS fields: grid (site blocks, 12 * nr slabs);
// slab s of a half field holds component s / nr of right-hand side s % nr.
// ---------------------------------------------------------------------------
static inline dim3 slab_grid(int vh, int nr) { return dim3((vh + 255) / 256, 12 * nr); }

// per-RHS |a|^2 over ncomp components (12: half field, 24: full field):
// grid (nbx, nr), block (bx, n) sums its sites over all components into
// partials [bx][kMaxRhs]
template <typename R>
__global__ __launch_bounds__(256) void k_mnorm(int vh, int ncomp, int nr, const R2<R>* __restrict__ a,
                                               double* partials) {
  __shared__ double sh[4];
  const int n = blockIdx.y;
  double acc = 0.0;
  for (int s = blockIdx.x * 256 + threadIdx.x; s < vh; s += gridDim.x * 256) {
    for (int k = 0; k < ncomp; ++k) {
      const R2<R> v = a[((size_t)k * nr + n) * vh + s];
      acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
    }
  }
  const double t = block_sum<256>(acc, sh);
  if (threadIdx.x == 0) partials[(size_t)blockIdx.x * kMaxRhs + n] = t;
}

static inline int mnorm_blocks(int vh) {
  const int nb = (vh + 255) / 256;
  return nb > 1024 ? 1024 : nb;
}

template <typename R>
hipError_t launch_mnorm(int vh, int ncomp, int nr, const R2<R>* a, Reduce red, hipStream_t s) {
  const int nb = mnorm_blocks(vh);
  hipLaunchKernelGGL((k_mnorm<R>), dim3(nb, nr), dim3(256), 0, s, vh, ncomp, nr, a, red.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_mfinalize(kFinResult1, nb, nr, red, nullptr, 0.0, 0, s);
}
template hipError_t launch_mnorm<double>(int, int, int, const double2*, Reduce, hipStream_t);
template hipError_t launch_mnorm<float>(int, int, int, const float2*, Reduce, hipStream_t);

// After the finalize of an iteration: x += alpha_n p for every right-hand
// side whose recursion ran it (still running, or stopped by this finalize:
// conv_iter == iter; nothing in an iteration queued after the whole batch
// stopped, whose finalize leaves iter as it was and sets idle), then
// p = r + beta_n p where the recursion goes on or waits for the update.  The x update is here rather than in the Schur-CG
// epilogue because this kernel reads p anyway.
template <typename R>
__global__ __launch_bounds__(256) void k_mxpay(int vh, int nr, const R2<R>* __restrict__ r, R2<R>* __restrict__ p,
                                               R2<R>* __restrict__ x, const BatchState* st) {
  if (st->idle) return;  // a queued iteration after the batch stopped: nothing ran
  const int n = blockIdx.y % nr;
  const int d = st->done[n];
  const bool ran = d == kDoneRunning || st->conv_iter[n] == st->iter;
  const bool upd = d == kDoneRunning || d == kDoneUpdate;
  if (!ran && !upd) return;
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= vh) return;
  const size_t i = (size_t)blockIdx.y * vh + s;
  R2<R> pv = p[i];
  if (ran) {
    const R alpha = R(st->alpha[n]);
    R2<R> xv = x[i];
    xv.x += alpha * pv.x;
    xv.y += alpha * pv.y;
    x[i] = xv;
  }
  if (upd) {
    const R beta = R(st->beta[n]);
    const R2<R> rv = r[i];
    pv.x = rv.x + beta * pv.x;
    pv.y = rv.y + beta * pv.y;
    p[i] = pv;
  }
}
template <typename R>
hipError_t launch_mxpay(int vh, int nr, const R2<R>* r, R2<R>* p, R2<R>* x, BatchState* st, hipStream_t s) {
  hipLaunchKernelGGL((k_mxpay<R>), slab_grid(vh, nr), dim3(256), 0, s, vh, nr, r, p, x, st);
  return hipGetLastError();
}
template hipError_t launch_mxpay<double>(int, int, const double2*, double2*, double2*, BatchState*, hipStream_t);
template hipError_t launch_mxpay<float>(int, int, const float2*, float2*, float2*, BatchState*, hipStream_t);

// x64 += scale_n * xs; xs = 0
__global__ __launch_bounds__(256) void k_mmixed_update(int vh, int nr, float2* xs, double2* __restrict__ x,
                                                       const double* __restrict__ scale) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= vh) return;
  const size_t i = (size_t)blockIdx.y * vh + s;
  const double sc = scale[blockIdx.y % nr];
  const float2 v = xs[i];
  double2 xv = x[i];
  xv.x += sc * (double)v.x;
  xv.y += sc * (double)v.y;
  x[i] = xv;
  xs[i] = make_float2(0.f, 0.f);
}
hipError_t launch_mmixed_update(int vh, int nr, float2* xs, double2* x, const double* scale, hipStream_t s) {
  hipLaunchKernelGGL(k_mmixed_update, slab_grid(vh, nr), dim3(256), 0, s, vh, nr, xs, x, scale);
  return hipGetLastError();
}

// r = sigma_n r64; p = r (restart_n) or p *= pscale_n
__global__ __launch_bounds__(256) void k_mrescale(int vh, int nr, const double2* __restrict__ r64,
                                                  const double* __restrict__ sigma, float2* __restrict__ r,
                                                  float2* __restrict__ p, const int* __restrict__ restart,
                                                  const double* __restrict__ pscale) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= vh) return;
  const int n = blockIdx.y % nr;
  const size_t i = (size_t)blockIdx.y * vh + s;
  const double sg = sigma[n];
  const double2 v = r64[i];
  const float2 w = make_float2((float)(sg * v.x), (float)(sg * v.y));
  r[i] = w;
  if (restart[n]) {
    p[i] = w;
  } else {
    const float2 q = p[i];
    p[i] = make_float2((float)(pscale[n] * (double)q.x), (float)(pscale[n] * (double)q.y));
  }
}
hipError_t launch_mrescale(int vh, int nr, const double2* r64, const double* sigma, float2* r, float2* p,
                           const int* restart, const double* pscale, hipStream_t s) {
  hipLaunchKernelGGL(k_mrescale, slab_grid(vh, nr), dim3(256), 0, s, vh, nr, r64, sigma, r, p, restart, pscale);
  return hipGetLastError();
}

// r = b, p = b, x = 0 (FP64 multi-RHS CG start); per-RHS |b|^2 to state
__global__ __launch_bounds__(256) void k_mcg_init64(size_t n, const double2* __restrict__ b, double2* __restrict__ r,
                                                    double2* __restrict__ p, double2* __restrict__ x) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const double2 v = b[i];
    r[i] = v;
    p[i] = v;
    x[i] = make_double2(0.0, 0.0);
  }
}
hipError_t launch_mcg_init64(int vh, int nr, const double2* b, double2* r, double2* p, double2* x, BatchState* st,
                             Reduce red, double tol, int max_iter, hipStream_t s) {
  const size_t n = (size_t)12 * vh * nr;
  hipLaunchKernelGGL(k_mcg_init64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, b, r, p, x);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nb = mnorm_blocks(vh);
  hipLaunchKernelGGL((k_mnorm<double>), dim3(nb, nr), dim3(256), 0, s, vh, 12, nr, b, red.partials);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_mfinalize(kFinCgInit, nb, nr, red, st, tol, max_iter, s);
}

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

// One block: per-RHS sums of the partials of the previous launch.  Every
// right-hand side is summed in the same pass: each thread adds its rows
// (i = thread, thread + 256, ...) for all of them, then one butterfly per
// right-hand side and the four waves in order -- the order of block_sum, so
// the sums are those of one block_sum per right-hand side, without its 2 nr
// barriers and nr dependent load rounds.
__global__ __launch_bounds__(256) void k_mfinalize(int mode, int nblk, int nr, const double* __restrict__ partials,
                                                   BatchState* st, double* result, double tol, int max_iter,
                                                   Mailbox* mb) {
  if (mode == kFinCgStep && st->all_done) {  // the iteration was skipped
    if (threadIdx.x == 0) {
      for (int n = 0; n < nr; ++n)
        if (st->done[n] == kDoneUpdate) st->done[n] = kDoneUpdateHeld;
      st->any_update = 0;
      st->idle = 1;
      post_progress(mb, st->iter, 1);
    }
    return;
  }
  __shared__ double sh[4][kMaxRhs];
  __shared__ double tot[kMaxRhs];
  double acc[kMaxRhs];
#pragma unroll
  for (int n = 0; n < kMaxRhs; ++n) acc[n] = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) {
    const double* row = partials + (size_t)i * kMaxRhs;
#pragma unroll
    for (int n = 0; n < kMaxRhs; ++n)
      if (n < nr) acc[n] += row[n];
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int n = 0; n < kMaxRhs; ++n) {
    if (n < nr) {
      double v = acc[n];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0) sh[w][n] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int n = 0; n < nr; ++n) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) t += sh[i][n];
    tot[n] = t;
  }
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
    st->idle = 0;
    int all = 1;
    for (int n = 0; n < nr; ++n) {
      const double rr = tot[n];
      st->rr[n] = rr;
      st->rr_max[n] = rr;
      st->rr_stop[n] = tol * tol * rr;
      st->alpha[n] = st->beta[n] = st->pap[n] = 0.0;
      st->done[n] = !isfinite(rr) ? kDoneBreakdown : (rr == 0.0 ? kDoneConverged : kDoneRunning);
      st->conv_iter[n] = 0;
      st->work[n] = 0;
      all &= st->done[n] != kDoneRunning;
    }
    st->all_done = all;
    return;
  }
  // kFinCgStep
  st->idle = 0;
  st->iter += 1;
  int all = 1, any_update = 0;
  const double d2 = st->delta2;
  for (int n = 0; n < nr; ++n) {
    if (st->done[n] == kDoneUpdate) st->done[n] = kDoneUpdateHeld;
    if (st->done[n] == kDoneRunning) {  // the iteration ran for this right-hand side
      st->work[n] += 1;
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

// element (k, n, site) of a multi-RHS field is at (k nr + n) vh + site
__global__ __launch_bounds__(256) void k_mzero_rhs(size_t tot, int vh, int nr, double2* __restrict__ f,
                                                   unsigned mask) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= tot) return;
  const int n = (int)((t / (size_t)vh) % (size_t)nr);
  if ((mask >> n) & 1u) f[t] = make_double2(0.0, 0.0);
}
hipError_t launch_mzero_rhs(int vh, int ncomp, int nr, double2* f, unsigned mask, hipStream_t s) {
  if (!mask) return hipSuccess;
  const size_t tot = (size_t)ncomp * nr * vh;
  hipLaunchKernelGGL(k_mzero_rhs, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, tot, vh, nr, f, mask);
  return hipGetLastError();
}

// canonical spinor [V][4][3] of right-hand side n <-> full multi-RHS field
__global__ __launch_bounds__(256) void k_mpack(Geom g, int nr, int n, const double2* __restrict__ canon,
                                               double2* __restrict__ packed) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= 2 * (size_t)g.vh * 12) return;
  const int s = (int)(t / 12), k = (int)(t % 12);
  int c[4];
  lex_coords(g, s, c);
  packed[(((size_t)parity_of(c) * 12 + k) * nr + n) * g.vh + (s >> 1)] = canon[t];
}
__global__ __launch_bounds__(256) void k_munpack(Geom g, int nr, int n, const double2* __restrict__ packed,
                                                 double2* __restrict__ canon) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= 2 * (size_t)g.vh * 12) return;
  const int s = (int)(t / 12), k = (int)(t % 12);
  int c[4];
  lex_coords(g, s, c);
  canon[t] = packed[(((size_t)parity_of(c) * 12 + k) * nr + n) * g.vh + (s >> 1)];
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
