// Stout smearing (Morningstar-Peardon) and its hand-written adjoint.
//
// Forward, per link:  C = rho A^dag (A = plaquette staple sum of staple_A),
//   Omega = C U^dag,  X = P[Omega] = -rho P[U A]  (= iQ of the MP form),
//   U' = exp(X) U.
//
// Reverse mode of one level, for a cotangent G' at U' (G convention of
// Sec. S2: delta S = Re tr(G^dag delta U)):
//   U' = E U         ->  G_U += E^dag G',  G_E = G' U^dag
//   E = exp(X)       ->  G_X = L(X^dag, G_E), L the Frechet derivative of exp
//                        (the adjoint of L(X, .) under Re tr(A^dag B) is L(X^dag, .))
//   X = P[Omega]     ->  G_Omega = P[G_X]            (P is self-adjoint)
//   Omega = C U^dag  ->  Lambda := G_C = G_Omega U,  G_U += G_Omega^dag C
//   C = rho sum of staples -> every link of every staple receives its share
//   (stage B gathers the 18 terms per link).
// Nothing is stored between levels: the caller recomputes U_{l-1} from U_0.
#include "lgt_internal.h"
#include "lgt_su3.h"

namespace lgt {

// exp(X) = f0 + f1 X + f2 X^2 for a traceless 3x3 X, by Cayley-Hamilton
// (X^3 = c1 X + c0 with c1 = tr(X^2)/2, c0 = det X = tr(X^3)/3), with the
// derivatives df_j/dc0 and df_j/dc1: the Taylor polynomial of order 16 of
// exp(X/2^s), ||X/2^s||_F <= 1/2 (remainder below 1e-19), carried in the
// basis {1, X, X^2} as scalar recurrences -- X^(k+1) = c0 z + (x + c1 z) X
// + y X^2 for X^k = x + y X + z X^2 -- differentiated forward in c0 and c1,
// then squared s times in the same basis.  The truncation is that of the
// matrix series; no 3x3 products are needed.
struct ChCoef {
  C<double> f[3], d0[3], d1[3];
};
__device__ __forceinline__ ChCoef exp_ch(C<double> c0, C<double> c1, double nrm) {
  int s = 0;
  while (nrm > 0.5 && s < 40) {
    nrm *= 0.5;
    ++s;
  }
  const double sc = ldexp(1.0, -s);
  C<double> p[3] = {cmk(1.0, 0.0), czero<double>(), czero<double>()};
  C<double> q0[3] = {czero<double>(), czero<double>(), czero<double>()};
  C<double> q1[3] = {czero<double>(), czero<double>(), czero<double>()};
  ChCoef r;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    r.f[j] = p[j];
    r.d0[j] = czero<double>();
    r.d1[j] = czero<double>();
  }
#pragma unroll
  for (int k = 1; k <= 16; ++k) {
    const double h = sc / double(k);
    const C<double> x = p[0], y = p[1], z = p[2];
    p[0] = h * (c0 * z);
    p[1] = h * (x + c1 * z);
    p[2] = h * y;
    const C<double> x0 = q0[0], y0 = q0[1], z0 = q0[2];
    q0[0] = h * (z + c0 * z0);
    q0[1] = h * (x0 + c1 * z0);
    q0[2] = h * y0;
    const C<double> x1 = q1[0], y1 = q1[1], z1 = q1[2];
    q1[0] = h * (c0 * z1);
    q1[1] = h * (x1 + z + c1 * z1);
    q1[2] = h * y1;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      r.f[j] += p[j];
      r.d0[j] += q0[j];
      r.d1[j] += q1[j];
    }
  }
  // (a0 + a1 X + a2 X^2)^2 = b0 + b1 X + b2 X^2 with X^3 = c1 X + c0, X^4 = c1 X^2 + c0 X
  for (int j = 0; j < s; ++j) {
    const C<double> a0 = r.f[0], a1 = r.f[1], a2 = r.f[2];
    const C<double> a12 = a1 * a2, a22 = a2 * a2;
    const C<double> e0 = r.d0[0], e1 = r.d0[1], e2 = r.d0[2];
    const C<double> g0 = r.d1[0], g1 = r.d1[1], g2 = r.d1[2];
    const C<double> de12 = e1 * a2 + a1 * e2, dg12 = g1 * a2 + a1 * g2;
    const C<double> de22 = 2.0 * (a2 * e2), dg22 = 2.0 * (a2 * g2);
    r.f[0] = a0 * a0 + 2.0 * (a12 * c0);
    r.f[1] = 2.0 * (a0 * a1) + 2.0 * (a12 * c1) + a22 * c0;
    r.f[2] = a1 * a1 + 2.0 * (a0 * a2) + a22 * c1;
    r.d0[0] = 2.0 * (a0 * e0) + 2.0 * (de12 * c0) + 2.0 * a12;
    r.d0[1] = 2.0 * (e0 * a1 + a0 * e1) + 2.0 * (de12 * c1) + de22 * c0 + a22;
    r.d0[2] = 2.0 * (a1 * e1) + 2.0 * (e0 * a2 + a0 * e2) + de22 * c1;
    r.d1[0] = 2.0 * (a0 * g0) + 2.0 * (dg12 * c0);
    r.d1[1] = 2.0 * (g0 * a1 + a0 * g1) + 2.0 * (dg12 * c1) + 2.0 * a12 + dg22 * c0;
    r.d1[2] = 2.0 * (a1 * g1) + 2.0 * (g0 * a2 + a0 * g2) + dg22 * c1 + a22;
  }
  return r;
}

// For anti-Hermitian traceless X and the cotangent GE of E = exp(X):
// Einv = E^dag = exp(-X), and GX, whose traceless anti-Hermitian part is
// that of the adjoint Frechet derivative L(X^dag, GE).  With
// d exp(X)[dX] = sum_j (df_j/dc0 dc0 + df_j/dc1 dc1) X^j + f1 dX + f2 (dX X + X dX)
// and, for traceless dX, dc0 = tr(X^2 dX), dc1 = tr(X dX):
//   GX = conj(k0) X^2 - conj(k1) X + conj(f1) GE - conj(f2) (GE X + X GE),
//   k_i = sum_j tr(GE^dag X^j) df_j/dc_i.
__device__ __forceinline__ void exp_adjoint_ah(const M3<double>& X, const M3<double>& GE, M3<double>& Einv,
                                               M3<double>& GX) {
  const M3<double> X2 = mmul(X, X);
  C<double> c1 = czero<double>(), c0 = czero<double>(), g0 = czero<double>(), g1 = czero<double>(),
            g2 = czero<double>();
  double n2 = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    c1 += X2.m[4 * i];
    g0 += conj(GE.m[4 * i]);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      c0 += X2.m[3 * i + j] * X.m[3 * j + i];
      g1 += cjmul(GE.m[3 * i + j], X.m[3 * i + j]);
      g2 += cjmul(GE.m[3 * i + j], X2.m[3 * i + j]);
      n2 += norm2(X.m[3 * i + j]);
    }
  }
  c1 = 0.5 * c1;
  c0 = (1.0 / 3.0) * c0;
  const ChCoef ch = exp_ch(c0, c1, sqrt(n2));
  const C<double> k0 = g0 * ch.d0[0] + g1 * ch.d0[1] + g2 * ch.d0[2];
  const C<double> k1 = g0 * ch.d1[0] + g1 * ch.d1[1] + g2 * ch.d1[2];
  const C<double> a = conj(k0), b = -conj(k1), f1 = conj(ch.f[1]), f2 = -conj(ch.f[2]);
  const M3<double> GX1 = mmul(GE, X), GX2 = mmul(X, GE);
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    GX.m[k] = a * X2.m[k] + b * X.m[k] + f1 * GE.m[k] + f2 * (GX1.m[k] + GX2.m[k]);
    Einv.m[k] = conj(ch.f[2]) * X2.m[k] - conj(ch.f[1]) * X.m[k];
  }
  const C<double> f0 = conj(ch.f[0]);
#pragma unroll
  for (int i = 0; i < 3; ++i) Einv.m[4 * i] += f0;
}

struct LinkIdx {
  int p, mu, cb;
  int c[4];
};

// Thread -> link: a block owns 64 sites of one parity (a site block, in the
// order of gauge_site_block, parity alternating between blocks), wave w the
// links of direction w there (the four links of a site share most of their
// staple links), and blocks are numbered XCD-contiguously, so that
// neighbouring site blocks -- whose staples read each other's links -- run
// under the same L2.
__device__ __forceinline__ bool link_of_thread(const Geom& g, LinkIdx& li) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  li.p = lb & 1;
  li.cb = gauge_site_block(lb, gauge_block_order(g), g.L[2]) * 64 + (threadIdx.x & 63);
  li.mu = threadIdx.x >> 6;
  if (li.cb >= g.vh) return false;
  cb_coords(g, li.p, li.cb, li.c);
  return true;
}

__global__ __launch_bounds__(256) void k_stout_fwd(Geom g, const double2* __restrict__ U, double2* __restrict__ Uo,
                                                   double rho) {
  LinkIdx li;
  if (!link_of_thread(g, li)) return;
  const M3<double> Ux = load_m3<double>(gptr<double>(U, g, li.p, li.mu), g.vh, li.cb);
  const M3<double> A = staple_A(U, g, li.c, li.mu);
  const M3<double> X = mscale(-rho, proj_ta(mmul(Ux, A)));
  store_m3<double>((double2*)gptr<double>(Uo, g, li.p, li.mu), g.vh, li.cb, mmul(exp_ah(X), Ux));
}

__global__ __launch_bounds__(256) void k_stout_adj_a(Geom g, const double2* __restrict__ U,
                                                     const double2* __restrict__ Gp, double rho,
                                                     double2* __restrict__ Lam, double2* __restrict__ Gpart) {
  LinkIdx li;
  if (!link_of_thread(g, li)) return;
  const int vh = g.vh;
  const M3<double> Ux = load_m3<double>(gptr<double>(U, g, li.p, li.mu), vh, li.cb);
  const M3<double> A = staple_A(U, g, li.c, li.mu);
  const M3<double> X = mscale(-rho, proj_ta(mmul(Ux, A)));
  const M3<double> G1 = load_m3<double>(gptr<double>(Gp, g, li.p, li.mu), vh, li.cb);
  const M3<double> GE = mmul_nd(G1, Ux);  // G' U^dag
  M3<double> Einv, GX;
  exp_adjoint_ah(X, GE, Einv, GX);  // E^dag, and L(X^dag, G_E) up to its non-su(3) part
  const M3<double> GOm = proj_ta(GX);
  const M3<double> C = mscale(rho, mdag(A));
  store_m3<double>((double2*)gptr<double>(Lam, g, li.p, li.mu), vh, li.cb, mmul(GOm, Ux));
  store_m3<double>((double2*)gptr<double>(Gpart, g, li.p, li.mu), vh, li.cb,
                   mmac_dn(mmul(Einv, G1), GOm, C));
}

// Stage B: for the link U_a(y), add rho times the gradient of
// sum_{x,mu} Re tr(Lambda_mu(x)^dag C_mu(x)/rho) with respect to it.  With
// C_mu(x)/rho = sum_nu [U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag
//                       + U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu)], the link is
// a side link of the staples of C_m (m != a) in four ways and the middle
// link of the staples of C_a in two ways (per m != a):
//   L_m(y) U_a(y+m) U_m(y+a)^dag      L_m(y-m)^dag U_a(y-m) U_m(y-m+a)
//   U_m(y) U_a(y+m) L_m(y+a)^dag      U_m(y-m)^dag U_a(y-m) L_m(y-m+a)
//   U_m(y-m)^dag L_a(y-m) U_m(y-m+a)  U_m(y) L_a(y+m) U_m(y+a)^dag
__global__ __launch_bounds__(256) void k_stout_adj_b(Geom g, const double2* __restrict__ U,
                                                     const double2* __restrict__ Lam,
                                                     const double2* __restrict__ Gpart, double rho,
                                                     double2* __restrict__ Go) {
  LinkIdx li;
  if (!link_of_thread(g, li)) return;
  const int a = li.mu;
  const int* y = li.c;
  M3<double> S;
#pragma unroll
  for (int k = 0; k < 9; ++k) S.m[k] = czero<double>();
#pragma unroll 1
  for (int k = 1; k < 4; ++k) {
    const int m = (a + k) & 3;
    int ypm[4], ypa[4], ymm[4], ymmpa[4];
    shifted(g, y, m, +1, ypm);
    shifted(g, y, a, +1, ypa);
    shifted(g, y, m, -1, ymm);
    shifted(g, ymm, a, +1, ymmpa);
    // the first and third terms of each side share their last factor:
    // five 3x3 products per side instead of six
    {  // forward side: sites y, y+m, y+a
      const M3<double> Ua_ypm = link_at(U, g, ypm, a);
      const M3<double> Um_y = link_at(U, g, y, m);
      const M3<double> W = mmac(mmul(link_at(Lam, g, y, m), Ua_ypm), Um_y, link_at(Lam, g, ypm, a));
      S = mmac_nd(S, W, link_at(U, g, ypa, m));
      S = mmac_nd(S, mmul(Um_y, Ua_ypm), link_at(Lam, g, ypa, m));
    }
    {  // backward side: sites y-m, y-m+a
      const M3<double> Ua_ymm = link_at(U, g, ymm, a);
      const M3<double> Um_ymm = link_at(U, g, ymm, m);
      const M3<double> W = mmac_dn(mmul_dn(link_at(Lam, g, ymm, m), Ua_ymm), Um_ymm, link_at(Lam, g, ymm, a));
      S = mmac(S, W, link_at(U, g, ymmpa, m));
      S = mmac(S, mmul_dn(Um_ymm, Ua_ymm), link_at(Lam, g, ymmpa, m));
    }
  }
  const M3<double> Gx = load_m3<double>(gptr<double>(Gpart, g, li.p, a), g.vh, li.cb);
  store_m3<double>((double2*)gptr<double>(Go, g, li.p, a), g.vh, li.cb, madd(Gx, mscale(rho, S)));
}

// out (packed or canonical) accumulates the force of a gradient G at U:
// mode 0: out += F,  mode 1: out += G,  mode 2: out -= dt F,  F = -1/2 P[U G^dag].
template <int LAYOUT>
__global__ __launch_bounds__(256) void k_grad_to_force(Geom g, const double2* __restrict__ U,
                                                       const double2* __restrict__ G, int mode, double dt,
                                                       double2* __restrict__ out) {
  LinkIdx li;
  if (!link_of_thread(g, li)) return;
  const int vh = g.vh;
  const M3<double> Gx = load_m3<double>(gptr<double>(G, g, li.p, li.mu), vh, li.cb);
  M3<double> add;
  if (mode == 1) {
    add = Gx;
  } else {
    const M3<double> Ux = load_m3<double>(gptr<double>(U, g, li.p, li.mu), vh, li.cb);
    add = mscale(mode == 2 ? 0.5 * dt : -0.5, proj_ta(mmul_nd(Ux, Gx)));
  }
  const int s = li.c[0] + g.L[0] * (li.c[1] + g.L[1] * (li.c[2] + g.L[2] * li.c[3]));
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const size_t o = LAYOUT == kCanonical ? ((size_t)s * 4 + li.mu) * 9 + k
                                          : ((size_t)(li.p * 4 + li.mu) * 9 + k) * vh + li.cb;
    st<double>(out + o, ld<double>(out + o) + add.m[k]);
  }
}

static inline int nb_links(const Geom& g) { return 2 * ((g.vh + 63) / 64); }

hipError_t launch_stout_fwd(const Geom& g, const double2* U, double2* Uo, double rho, hipStream_t s) {
  hipLaunchKernelGGL(k_stout_fwd, dim3(nb_links(g)), dim3(256), 0, s, g, U, Uo, rho);
  return hipGetLastError();
}

hipError_t launch_stout_adjoint(const Geom& g, const double2* U, const double2* Gp, double rho, double2* Lam,
                                double2* Gpart, double2* Go, hipStream_t s) {
  hipLaunchKernelGGL(k_stout_adj_a, dim3(nb_links(g)), dim3(256), 0, s, g, U, Gp, rho, Lam, Gpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_stout_adj_b, dim3(nb_links(g)), dim3(256), 0, s, g, U, Lam, Gpart, rho, Go);
  return hipGetLastError();
}

hipError_t launch_grad_to_force(const Geom& g, const double2* U, const double2* G, int mode, double dt, void* out,
                                int layout, hipStream_t s) {
  if (layout == kCanonical)
    hipLaunchKernelGGL((k_grad_to_force<kCanonical>), dim3(nb_links(g)), dim3(256), 0, s, g, U, G, mode, dt,
                       (double2*)out);
  else
    hipLaunchKernelGGL((k_grad_to_force<kPacked>), dim3(nb_links(g)), dim3(256), 0, s, g, U, G, mode, dt,
                       (double2*)out);
  return hipGetLastError();
}

}  // namespace lgt
