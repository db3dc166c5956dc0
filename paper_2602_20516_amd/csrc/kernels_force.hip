// Adjoint (force) kernels, gauge action, kinetic energy and the link update.
//
// Conventions (Sec. S2): G = dS/dRe U + i dS/dIm U, delta S = Re tr(G^dag dU),
// F = -1/2 P_su3[U G^dag] with P_su3 the traceless anti-Hermitian projection
// of eq. (7); the momentum update is P <- P - dt F.
//
// Thread mapping of the per-link kernels: thread t handles link (s, mu) with
// s = t/4 the lexicographic site and mu = t%4, so a wavefront covers 16
// consecutive sites and its canonical [V][4][3][3] output is one contiguous
// 9 KB span.
#include "lgt_internal.h"
#include "lgt_su3.h"
#include "lgt_hop.h"

namespace lgt {

// ---------------------------------------------------------------------------
// Adjoint of I(U) = a^dag D(U) b (eq. S3.13): for the link U_mu(x), with s_bc
// its fermion boundary sign,
//   Re I depends on U through -kappa s_bc Re tr(U Z),
//   Z = sum_j h-[b(x+mu)]_j h-[a(x)]_j^dag + sum_j h+[a(x+mu)]_j h+[b(x)]_j^dag,
// where h-/h+ are the projections of (1 - gamma_mu)/(1 + gamma_mu).  For the
// functional coeff * Re I:  G = -coeff kappa s_bc Z^dag and
// F = -1/2 P[U G^dag] = (coeff kappa s_bc / 2) P[U Z].  The pseudofermion
// force of eq. S3.12 is coeff = -2, a = Y = D X, b = X.
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Per-link kernels in site-block form: a 256-thread block owns 64
// consecutive checkerboard sites of one parity and all four directions,
// wave w taking direction mu = w, so every wave's loads of a field
// component (own site, neighbour, link) are 64 consecutive elements.  Blocks
// alternate parity (logical block 2i + p is site block i of parity p), so
// the neighbour spinors a block reads are the own spinors the block next to
// it reads at about the same time, on the same XCD.  Output: the packed
// layout is written directly (coalesced); the canonical [V][4][3][3] layout
// is staged in LDS and written as each site's 576-byte record (all four
// links), by consecutive threads.
// ---------------------------------------------------------------------------
constexpr int kSB = 64;  // sites per block

// non-temporal store of one complex double
typedef double v2d __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_nt2(double2* q, double x, double y) {
  const v2d v = {x, y};
  __builtin_nontemporal_store(v, reinterpret_cast<v2d*>(q));
}

__device__ __forceinline__ int lex_of(const Geom& g, const int c[4]) {
  return c[0] + g.L[0] * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3]));
}

// Stage M (the link's output matrix) and write the block's sites: packed
// layout directly, canonical through LDS.  mode 2 subtracts dt M from the
// momenta in place.
template <int LAYOUT>
__device__ __forceinline__ void emit_block(const Geom& g, double2* out, int p, int blk, int lane, int mu, int mode,
                                           double dt, const M3<double>& M, bool active, int s_lex,
                                           double2 (*sh)[36], int* sh_site) {
  if (LAYOUT == kPacked) {
    if (active) {
      const int cb = blk * kSB + lane;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        double2* q = out + ((size_t)(p * 4 + mu) * 9 + k) * g.vh + cb;
        if (mode == 2) st<double>(q, ld<double>(q) - dt * M.m[k]);
        else st_nt2(q, M.m[k].re, M.m[k].im);
      }
    }
    return;
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) sh[lane][mu * 9 + k] = make_double2(M.m[k].re, M.m[k].im);
  if (mu == 0) sh_site[lane] = active ? s_lex : -1;
  __syncthreads();
  for (int e = threadIdx.x; e < kSB * 36; e += 256) {
    const int site = e / 36, r = e - site * 36;
    const int sl = sh_site[site];
    if (sl < 0) continue;
    double2* q = out + (size_t)sl * 36 + r;
    const double2 v = sh[site][r];
    if (mode == 2) {
      const double2 o = *q;
      *q = make_double2(o.x - dt * v.x, o.y - dt * v.y);
    } else {
      st_nt2(q, v.x, v.y);  // written once: kept out of the caches the inputs use
    }
  }
}

// Z of the bilinear adjoint for direction MU at the block's site `lane`:
// the sum of the outer products of the projected half spinors, one pair of
// spinors at a time; the own-site spinors come from the block's LDS copy
// (sa, sb: [12][64]), the neighbours at x + mu (checkerboard site nf of
// the other parity) from global memory
template <int MU>
__device__ __forceinline__ M3<double> bilinear_z(const double2 (*sa)[kSB], const double2 (*sb)[kSB],
                                                 const SpinorIn<double, double2>& a_nb,
                                                 const SpinorIn<double, double2>& b_nb, int lane, int nf) {
  M3<double> Z;
#pragma unroll
  for (int k = 0; k < 9; ++k) Z.m[k] = czero<double>();
  C<double> psi[12], hx[6], hy[6];
  {  // h-[b(x+mu)] h-[a(x)]^dag
    const unsigned ob = b_nb.off(nf, 0);
#pragma unroll
    for (int k = 0; k < 12; ++k) psi[k] = b_nb.ld(ob, k);
    project<double, MU, -1>(psi, hx);
#pragma unroll
    for (int k = 0; k < 12; ++k) psi[k] = cmk<double>(sa[k][lane].x, sa[k][lane].y);
    project<double, MU, -1>(psi, hy);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Z.m[3 * i + j] += mulcj(hx[i], hy[j]) + mulcj(hx[3 + i], hy[3 + j]);
  }
  {  // h+[a(x+mu)] h+[b(x)]^dag
    const unsigned oa = a_nb.off(nf, 0);
#pragma unroll
    for (int k = 0; k < 12; ++k) psi[k] = a_nb.ld(oa, k);
    project<double, MU, +1>(psi, hx);
#pragma unroll
    for (int k = 0; k < 12; ++k) psi[k] = cmk<double>(sb[k][lane].x, sb[k][lane].y);
    project<double, MU, +1>(psi, hy);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Z.m[3 * i + j] += mulcj(hx[i], hy[j]) + mulcj(hx[3 + i], hy[3 + j]);
  }
  return Z;
}

// The bilinear adjoint (the adjoint of I(U) above) in site-block form.
// Blocks in the t-fastest groups of gauge_site_block (its 4x4 t/z groups
// are not used: a bilinear reads only its +mu neighbours).  Every direction
// needs the own-site a and b of the block's 64 sites, so the block first
// copies them to LDS in one coalesced pass (6 loads per thread) and its four
// waves read them there: 24 of each wave's 57 global loads gone, the rest
// (the +mu neighbours and the link) unchanged (24^3x48: 259 -> 246 us,
// 32^3x64: 776 -> 738 us).  The output staging of the canonical layout
// reuses the same LDS after a barrier.
template <int LAYOUT>
__global__ __launch_bounds__(256) void k_bilinear_sb(Geom g, const double2* __restrict__ U,
                                                     const double2* __restrict__ a, const double2* __restrict__ b,
                                                     double kappa, double coeff, int mode, double dt,
                                                     double2* out, BlockOrder order) {
  // [2][12][64] own-site spinors; for the canonical layout also the [64][36] output staging
  constexpr int kWords = LAYOUT == kCanonical ? kSB * 36 : 2 * 12 * kSB;
  static_assert(kWords >= 2 * 12 * kSB, "the LDS must hold both own-site spinors");
  __shared__ double2 smem[kWords];
  __shared__ int sh_site[kSB];
  double2 (*sa)[kSB] = reinterpret_cast<double2 (*)[kSB]>(smem);
  double2 (*sb)[kSB] = reinterpret_cast<double2 (*)[kSB]>(smem + 12 * kSB);
  double2 (*sh)[36] = reinterpret_cast<double2 (*)[36]>(smem);
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int p = lb & 1, blk = gauge_site_block(lb, order, g.L[2]);
  const int lane = threadIdx.x & 63, mu = threadIdx.x >> 6;
  const int cb = blk * kSB + lane;
  const bool active = cb < g.vh;
  const int vh = g.vh;
  const size_t half = (size_t)12 * vh;
  {  // element e = (field, component, site) of the 2 x 12 x 64 own-site values; sites past vh read zero
    const double2* ap = a + p * half;
    const double2* bp = b + p * half;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const int e = threadIdx.x + 256 * j;
      const int f = e / (12 * kSB), k = (e % (12 * kSB)) / kSB, l = e % kSB;
      const int site = blk * kSB + l;
      double2 v = make_double2(0.0, 0.0);
      if (site < vh) v = (f ? bp : ap)[(size_t)k * vh + site];
      (f ? sb : sa)[k][l] = v;
    }
  }
  int c[4];
  cb_coords(g, p, active ? cb : 0, c);
  const int nf = cb_shift(g, c, mu, +1);
  const unsigned ks = (unsigned)vh * (unsigned)sizeof(double2);
  const SpinorIn<double, double2> a_nb{make_rsrc(a + (1 - p) * half, (size_t)12 * ks), ks, 1u};
  const SpinorIn<double, double2> b_nb{make_rsrc(b + (1 - p) * half, (size_t)12 * ks), ks, 1u};
  __syncthreads();
  M3<double> Z;
  switch (mu) {
    case 0: Z = bilinear_z<0>(sa, sb, a_nb, b_nb, lane, nf); break;
    case 1: Z = bilinear_z<1>(sa, sb, a_nb, b_nb, lane, nf); break;
    case 2: Z = bilinear_z<2>(sa, sb, a_nb, b_nb, lane, nf); break;
    default: Z = bilinear_z<3>(sa, sb, a_nb, b_nb, lane, nf); break;
  }
  const int cbx = active ? cb : 0;
  const double sbc = (mu == 3 && c[3] == g.L[3] - 1) ? double(g.bc) : 1.0;
  M3<double> M;
  if (mode == 1) {
    M = mscale(-coeff * kappa * sbc, mdag(Z));
  } else {
    // each link is read once here: streamed past the caches (non-temporal)
    // so that the neighbour spinors stay in them
    M3<double> Ux;
    const BufRsrc ru = make_rsrc(gptr<double>(U, g, p, mu), (size_t)9 * vh * sizeof(double2));
#pragma unroll
    for (int k = 0; k < 9; ++k)
      Ux.m[k] = ld_buf_nt<double>(ru, (unsigned)cbx * (unsigned)sizeof(double2), (unsigned)(k * vh * sizeof(double2)));
    M = mscale(0.5 * coeff * kappa * sbc, proj_ta(mmul(Ux, Z)));
  }
  if (LAYOUT == kCanonical) __syncthreads();  // every wave is done with sa, sb before sh overwrites them
  emit_block<LAYOUT>(g, out, p, blk, lane, mu, mode, dt, M, active, lex_of(g, c), sh, sh_site);
}

static inline int sb_blocks(const Geom& g) { return 2 * ((g.vh + kSB - 1) / kSB); }

hipError_t launch_bilinear_force(const Geom& g, const double2* U, const double2* a_full, const double2* b_full,
                                 double kappa, double coeff, int mode, double dt, void* out, int layout,
                                 hipStream_t s) {
  const int nb = sb_blocks(g);
  BlockOrder order = gauge_block_order(g);
  order.nyc = 0;
  if (layout == kCanonical)
    hipLaunchKernelGGL((k_bilinear_sb<kCanonical>), dim3(nb), dim3(256), 0, s, g, U, a_full, b_full, kappa, coeff,
                       mode, dt, (double2*)out, order);
  else
    hipLaunchKernelGGL((k_bilinear_sb<kPacked>), dim3(nb), dim3(256), 0, s, g, U, a_full, b_full, kappa, coeff,
                       mode, dt, (double2*)out, order);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Wilson plaquette action: the link U_mu(x) enters S_G through
// -(beta/3) Re tr(U_mu(x) A_mu(x)) with the staple sum
//   A = sum_{nu != mu} [ U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
//                      + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu) ],
// so G = -(beta/3) A^dag and F = (beta/6) P[U A].
// ---------------------------------------------------------------------------
// The staple force in site-block form (see k_bilinear_sb): each thread sums
// the six staples of its link one at a time, each as two 3x3 products, so
// at most the running sum, one partial product and two links are live.
template <int LAYOUT>
__global__ __launch_bounds__(256) void k_gauge_force_sb(Geom g, const double2* __restrict__ U, double beta,
                                                        int mode, double dt, double2* out, BlockOrder order) {
  __shared__ double2 sh[LAYOUT == kCanonical ? kSB : 1][36];
  __shared__ int sh_site[kSB];
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int p = lb & 1, blk = gauge_site_block(lb, order, g.L[2]);
  const int lane = threadIdx.x & 63, mu = threadIdx.x >> 6;
  const int cb = blk * kSB + lane;
  const bool active = cb < g.vh;
  int c[4];
  cb_coords(g, p, active ? cb : 0, c);
  int xpm[4];
  shifted(g, c, mu, +1, xpm);
  M3<double> A;
#pragma unroll
  for (int k = 0; k < 9; ++k) A.m[k] = czero<double>();
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    const int nu = (mu + k) & 3;
    int xpn[4], xmn[4], xpmmn[4];
    shifted(g, c, nu, +1, xpn);
    shifted(g, c, nu, -1, xmn);
    shifted(g, xpm, nu, -1, xpmmn);
    // U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
    M3<double> t = mmul_nd(link_at(U, g, xpm, nu), link_at(U, g, xpn, mu));
    A = mmac_nd(A, t, link_at(U, g, c, nu));
    // U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu) = (U_mu(x-nu) U_nu(x+mu-nu))^dag U_nu(x-nu)
    t = mmul(link_at(U, g, xmn, mu), link_at(U, g, xpmmn, nu));
    A = mmac_dn(A, t, link_at(U, g, xmn, nu));
  }
  M3<double> M;
  if (mode == 1) {
    M = mscale(-beta / 3.0, mdag(A));
  } else {
    const M3<double> Ux = load_m3<double>(gptr<double>(U, g, p, mu), g.vh, active ? cb : 0);
    M = mscale(beta / 6.0, proj_ta(mmul(Ux, A)));
  }
  emit_block<LAYOUT>(g, out, p, blk, lane, mu, mode, dt, M, active, lex_of(g, c), sh, sh_site);
}

hipError_t launch_gauge_force(const Geom& g, const double2* U, double beta, int mode, double dt, void* out,
                              int layout, hipStream_t s) {
  const int nb = sb_blocks(g);
  const BlockOrder order = gauge_block_order(g);
  if (layout == kCanonical)
    hipLaunchKernelGGL((k_gauge_force_sb<kCanonical>), dim3(nb), dim3(256), 0, s, g, U, beta, mode, dt,
                       (double2*)out, order);
  else
    hipLaunchKernelGGL((k_gauge_force_sb<kPacked>), dim3(nb), dim3(256), 0, s, g, U, beta, mode, dt,
                       (double2*)out, order);
  return hipGetLastError();
}

// sum over sites and mu<nu of Re tr P_mu,nu(x)
// sum over plaquettes of Re tr P_mu,nu(x) at the site of this thread
__device__ __forceinline__ double site_plaquettes(const Geom& g, const double2* __restrict__ U, const int c[4]) {
  double acc = 0.0;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    int xpm[4];
    shifted(g, c, mu, +1, xpm);
    const M3<double> a = link_at(U, g, c, mu);
#pragma unroll
    for (int nu = mu + 1; nu < 4; ++nu) {
      int xpn[4];
      shifted(g, c, nu, +1, xpn);
      const M3<double> ab = mmul(a, link_at(U, g, xpm, nu));
      const M3<double> dc = mmul(link_at(U, g, c, nu), link_at(U, g, xpn, mu));
      // Re tr(A B C^dag D^dag) = Re tr((AB)(DC)^dag)
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < 9; ++k) t += ab.m[k].re * dc.m[k].re + ab.m[k].im * dc.m[k].im;
      acc += t;
    }
  }
  return acc;
}

// Sum of Re tr P over all plaquettes of U, or (Uold != null) the sum of the
// per-site differences U minus Uold, which keeps the rounding error of a
// trajectory's Delta S_G proportional to Delta S_G rather than to S_G.
__global__ __launch_bounds__(256) void k_plaquette(Geom g, const double2* __restrict__ U,
                                                   const double2* __restrict__ Uold, double* partials) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int s = lb * 256 + threadIdx.x;
  double acc = 0.0;
  if (s < 2 * g.vh) {
    int c[4];
    lex_coords(g, s, c);
    acc = site_plaquettes(g, U, c);
    if (Uold) acc -= site_plaquettes(g, Uold, c);
  }
  double v[1] = {acc};
  block_partials<256, 1>(v, partials, lb);
}

hipError_t launch_plaquette(const Geom& g, const double2* U, Reduce red, int slot, hipStream_t s,
                            const double2* Uold) {
  const int nb = (2 * g.vh + 255) / 256;
  if (nb > red.capacity) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_plaquette, dim3(nb), dim3(256), 0, s, g, U, Uold, red.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(kFinResult1, nb, red, nullptr, slot, 0.0, 0, s);
}

// Re tr(P P) of link t of a gauge-type field in either layout
__device__ __forceinline__ double link_trsq(const Geom& g, const double2* __restrict__ P, int layout, int t) {
  M3<double> m;
  if (layout == kCanonical) {
#pragma unroll
    for (int k = 0; k < 9; ++k) m.m[k] = ld<double>(P + (size_t)t * 9 + k);
  } else {
    const int cb = t % g.vh, pm = t / g.vh;  // pm = parity*4 + mu
#pragma unroll
    for (int k = 0; k < 9; ++k) m.m[k] = ld<double>(P + ((size_t)pm * 9 + k) * g.vh + cb);
  }
  double tr = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) tr += (m.m[3 * i + j] * m.m[3 * j + i]).re;
  return tr;
}

// -sum Re tr(P P) over all links, or (Pold != null, same layout) the sum of
// the per-link differences P minus Pold
__global__ __launch_bounds__(256) void k_kinetic(Geom g, const double2* __restrict__ P,
                                                 const double2* __restrict__ Pold, int layout, double* partials) {
  const int nlink = 8 * g.vh;
  double acc = 0.0;
  for (int t = blockIdx.x * 256 + threadIdx.x; t < nlink; t += gridDim.x * 256) {
    double d = -link_trsq(g, P, layout, t);
    if (Pold) d += link_trsq(g, Pold, layout, t);
    acc += d;
  }
  double v[1] = {acc};
  block_partials<256, 1>(v, partials, blockIdx.x);
}

hipError_t launch_kinetic(const Geom& g, const double2* P, int layout, Reduce red, int slot, hipStream_t s,
                          const double2* Pold) {
  int nb = (8 * g.vh + 255) / 256;
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(k_kinetic, dim3(nb), dim3(256), 0, s, g, P, Pold, layout, red.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(kFinResult1, nb, red, nullptr, slot, 0.0, 0, s);
}

// U <- reunit(exp(dt P) U).  Canonical: thread = (s, mu) matrix index t.
// Packed: thread = (parity*4+mu, cb), cb fastest.
template <int LAYOUT>
__global__ __launch_bounds__(256) void k_link_update(Geom g, double2* __restrict__ U, const double2* __restrict__ P,
                                                     double dt, float2* __restrict__ U32) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= 8 * g.vh) return;
  size_t base, stride;
  if (LAYOUT == kCanonical) {
    base = (size_t)t * 9;
    stride = 1;
  } else {
    const int cb = t % g.vh, pm = t / g.vh;
    base = (size_t)pm * 9 * g.vh + cb;
    stride = g.vh;
  }
  M3<double> u, x;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    u.m[k] = ld<double>(U + base + k * stride);
    x.m[k] = dt * ld<double>(P + base + k * stride);
  }
  const M3<double> un = reunitarize(mmul(exp_ah(x), u));
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    st<double>(U + base + k * stride, un.m[k]);
    if (LAYOUT == kPacked && U32) U32[base + k * stride] = make_float2((float)un.m[k].re, (float)un.m[k].im);
  }
}

hipError_t launch_link_update(const Geom& g, double2* U, const double2* P, double dt, int layout, float2* U32,
                              hipStream_t s) {
  const int nb = (8 * g.vh + 255) / 256;
  if (layout == kCanonical)
    hipLaunchKernelGGL((k_link_update<kCanonical>), dim3(nb), dim3(256), 0, s, g, U, P, dt, U32);
  else
    hipLaunchKernelGGL((k_link_update<kPacked>), dim3(nb), dim3(256), 0, s, g, U, P, dt, U32);
  return hipGetLastError();
}

}  // namespace lgt
