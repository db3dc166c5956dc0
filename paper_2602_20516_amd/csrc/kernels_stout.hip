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

// exp(A) and L(A, E) = d/dt exp(A + t E)|_0 for a 3x3 complex A: Taylor
// series of order 16 on A/2^s, E/2^s (||A/2^s||_F <= 1/2, remainder below
// 1e-19), then s doubling steps exp(2A) = exp(A)^2,
// L(2A, 2E) = exp(A) L(A,E) + L(A,E) exp(A).
__device__ __forceinline__ void exp_frechet(const M3<double>& A, const M3<double>& E, M3<double>& F,
                                            M3<double>& L) {
  double n2 = 0.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) n2 += norm2(A.m[k]);
  double nrm = sqrt(n2);
  int s = 0;
  while (nrm > 0.5 && s < 40) {
    nrm *= 0.5;
    ++s;
  }
  const double sc = ldexp(1.0, -s);
  const M3<double> As = mscale(sc, A), Es = mscale(sc, E);
  M3<double> T = mident<double>(), N, Fs = mident<double>(), Ls;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    N.m[k] = czero<double>();
    Ls.m[k] = czero<double>();
  }
  for (int k = 0; k < 16; ++k) {
    const double inv = 1.0 / double(k + 1);
    const M3<double> Nn = mscale(inv, madd(mmul(As, N), mmul(Es, T)));
    T = mscale(inv, mmul(As, T));
    N = Nn;
    Fs = madd(Fs, T);
    Ls = madd(Ls, N);
  }
  for (int j = 0; j < s; ++j) {
    Ls = madd(mmul(Fs, Ls), mmul(Ls, Fs));
    Fs = mmul(Fs, Fs);
  }
  F = Fs;
  L = Ls;
}

struct LinkIdx {
  int p, mu, cb;
  int c[4];
};

// Thread -> link: a block owns 64 consecutive sites of one parity, wave w
// the links of direction w there (the four links of a site share most of
// their staple links), and blocks are numbered XCD-contiguously, so that
// neighbouring site blocks -- whose staples read each other's links -- run
// under the same L2.  (Against one direction per launch segment and
// round-robin XCDs, this raised the L2 hit rate of the forward kernel from
// 11 % to 46 % and cut its time 1.6x at 24^3x48; walking each XCD's slab
// with t fastest gained nothing more.)
__device__ __forceinline__ bool link_of_thread(const Geom& g, LinkIdx& li) {
  const int nbp = (g.vh + 63) / 64;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  li.p = lb / nbp;
  li.cb = (lb - li.p * nbp) * 64 + (threadIdx.x & 63);
  li.mu = threadIdx.x >> 6;
  if (li.p > 1 || li.cb >= g.vh) return false;
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
  exp_frechet(mscale(-1.0, X), GE, Einv, GX);  // exp(X^dag) = E^dag, L(X^dag, G_E)
  const M3<double> GOm = proj_ta(GX);
  const M3<double> C = mscale(rho, mdag(A));
  store_m3<double>((double2*)gptr<double>(Lam, g, li.p, li.mu), vh, li.cb, mmul(GOm, Ux));
  store_m3<double>((double2*)gptr<double>(Gpart, g, li.p, li.mu), vh, li.cb,
                   madd(mmul(Einv, G1), mmul_dn(GOm, C)));
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
    {  // forward side: sites y, y+m, y+a
      const M3<double> Ua_ypm = link_at(U, g, ypm, a);
      const M3<double> Um_ypa = link_at(U, g, ypa, m);
      const M3<double> Um_y = link_at(U, g, y, m);
      S = madd(S, mmul(link_at(Lam, g, y, m), mmul_nd(Ua_ypm, Um_ypa)));
      S = madd(S, mmul_nd(mmul(Um_y, Ua_ypm), link_at(Lam, g, ypa, m)));
      S = madd(S, mmul_nd(mmul(Um_y, link_at(Lam, g, ypm, a)), Um_ypa));
    }
    {  // backward side: sites y-m, y-m+a
      const M3<double> Ua_ymm = link_at(U, g, ymm, a);
      const M3<double> Um_ymmpa = link_at(U, g, ymmpa, m);
      const M3<double> Um_ymm = link_at(U, g, ymm, m);
      S = madd(S, mmul_dn(link_at(Lam, g, ymm, m), mmul(Ua_ymm, Um_ymmpa)));
      S = madd(S, mmul(mmul_dn(Um_ymm, Ua_ymm), link_at(Lam, g, ymmpa, m)));
      S = madd(S, mmul(mmul_dn(Um_ymm, link_at(Lam, g, ymm, a)), Um_ymmpa));
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
