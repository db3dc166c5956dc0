// The spin-projected Wilson hop along one direction, shared by the single-
// and multi-right-hand-side hop kernels.
//
//   (1 + s gamma_mu) psi = (h ; s B_mu^dag h),  h = psi_up + s B_mu psi_dn,
// chiral basis: gamma_mu = [[0, B_mu], [B_mu^dag, 0]], B_0 = -i sigma_1,
// B_1 = -i sigma_2, B_2 = -i sigma_3, B_3 = 1; spinor component = 3*spin + colour.
#pragma once

#include "lgt_internal.h"

namespace lgt {

// h = u + s * B_mu d  for one spinor (comp = 3*spin + colour); s = +-1
// (a per-lane value in the half-wave hop, a constant otherwise).
template <typename R, int MU>
__device__ __forceinline__ void project_s(const C<R>* psi, const R s, C<R>* h) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const C<R> u0 = psi[i], u1 = psi[3 + i], d0 = psi[6 + i], d1 = psi[9 + i];
    if constexpr (MU == 0) {         // B = -i sigma_1: B d = (-i d1, -i d0)
      h[i] = u0 - s * itimes(d1);
      h[3 + i] = u1 - s * itimes(d0);
    } else if constexpr (MU == 1) {  // B = -i sigma_2: B d = (-d1, d0)
      h[i] = u0 - s * d1;
      h[3 + i] = u1 + s * d0;
    } else if constexpr (MU == 2) {  // B = -i sigma_3: B d = (-i d0, i d1)
      h[i] = u0 - s * itimes(d0);
      h[3 + i] = u1 + s * itimes(d1);
    } else {                         // B = 1
      h[i] = u0 + s * d0;
      h[3 + i] = u1 + s * d1;
    }
  }
}
template <typename R, int MU, int S>
__device__ __forceinline__ void project(const C<R>* psi, C<R>* h) {
  project_s<R, MU>(psi, R(S), h);
}

// acc_up += w ; acc_dn += s * B_mu^dag w
template <typename R, int MU>
__device__ __forceinline__ void reconstruct_s(const C<R>* w, const R s, C<R>* acc) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const C<R> w0 = w[i], w1 = w[3 + i];
    acc[i] += w0;
    acc[3 + i] += w1;
    if constexpr (MU == 0) {         // B^dag = i sigma_1: (i w1, i w0)
      acc[6 + i] += s * itimes(w1);
      acc[9 + i] += s * itimes(w0);
    } else if constexpr (MU == 1) {  // B^dag = i sigma_2: (w1, -w0)
      acc[6 + i] += s * w1;
      acc[9 + i] -= s * w0;
    } else if constexpr (MU == 2) {  // B^dag = i sigma_3: (i w0, -i w1)
      acc[6 + i] += s * itimes(w0);
      acc[9 + i] -= s * itimes(w1);
    } else {
      acc[6 + i] += s * w0;
      acc[9 + i] += s * w1;
    }
  }
}
template <typename R, int MU, int S>
__device__ __forceinline__ void reconstruct(const C<R>* w, C<R>* acc) {
  reconstruct_s<R, MU>(w, R(S), acc);
}

// Input loaders: off(site, n) gives the per-lane byte offset of (site, rhs n)
// once per neighbour, ld(off, k) spinor component k there (as C<R>).  All
// loads go through buffer resources with 32-bit offsets, so a field must
// stay below 4 GiB (the host checks 12 * vh * nr * 16 < 2^32).
//
// A plain stored field, element (k, site, n) at (k*vh + site)*nr + n.
template <typename R, typename T>
struct SpinorIn {
  BufRsrc rs;
  unsigned ks;  // component stride in bytes
  unsigned nr;
  __device__ __forceinline__ unsigned off(int site, int n) const {
    return ((unsigned)site * nr + (unsigned)n) * (unsigned)sizeof(T);
  }
  __device__ __forceinline__ C<R> ld(unsigned o, int k) const { return Store<R, T>::ld_buf(rs, o, k * ks); }
};

// loader for the input parity of output parity p
template <typename R, typename T>
__device__ __forceinline__ SpinorIn<R, T> make_loader(const HopIn<R, T>& h, const Geom& g, int p, int nr) {
  const unsigned ks = (unsigned)g.vh * (unsigned)nr * (unsigned)sizeof(T);
  return SpinorIn<R, T>{make_rsrc(p ? h.in_even : h.in_odd, (size_t)12 * ks), ks, (unsigned)nr};
}

// w = U h (forward hop) and w = U^dag h (backward hop) for the two colour
// vectors of a projected half spinor
template <typename R>
__device__ __forceinline__ void umul(const M3<R>& U, const C<R>* h, C<R>* w) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      C<R> s = U.m[3 * i] * h[3 * a];
      s += U.m[3 * i + 1] * h[3 * a + 1];
      s += U.m[3 * i + 2] * h[3 * a + 2];
      w[3 * a + i] = s;
    }
}
template <typename R>
__device__ __forceinline__ void umul_dag(const M3<R>& U, const C<R>* h, C<R>* w) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      C<R> s = cjmul(U.m[i], h[3 * a]);
      s += cjmul(U.m[3 + i], h[3 * a + 1]);
      s += cjmul(U.m[6 + i], h[3 * a + 2]);
      w[3 * a + i] = s;
    }
}
// fermion boundary sign on the temporal links crossing t = Lt-1 -> 0
template <typename R>
__device__ __forceinline__ void apply_bc(const Geom& g, C<R>* w) {
  const R b = R(g.bc);
#pragma unroll
  for (int k = 0; k < 6; ++k) w[k] = b * w[k];
}

// Link fields above this size (bytes, both parities) are streamed past the
// caches by the hop (a quarter below the 256 MB last-level cache, which
// also holds the spinors).
constexpr size_t kLinkStreamBytes = (size_t)192 << 20;

// Link U_mu(x) of parity p at checkerboard site cb from a packed field of
// nk complex components per link: all nine, or the first two rows of an
// SU(3) matrix, whose third row is the conjugate cross product of the two
// (one load per component through a buffer resource; uniform branch).
template <typename R>
__device__ __forceinline__ M3<R> load_link(const R2<R>* __restrict__ gauge, int nk, const Geom& g, int p, int mu,
                                           int cb) {
  constexpr unsigned E = sizeof(R2<R>);
  const unsigned gs = (unsigned)g.vh * E;
  const BufRsrc ru = make_rsrc(gauge + (size_t)((p * 4 + mu) * nk) * g.vh, (size_t)nk * gs);
  // A link field larger than the last-level cache is read with the
  // non-temporal policy: each launch reads every link once, and kept in the
  // caches the links would only push out the spinors the neighbouring sites
  // re-read (FP64 hop at 24^3x48 110 -> 100 us, FP32 two-row at 32^3x64
  // 144 -> 126 us).  A smaller field stays cached, where the next launch of
  // the solve re-reads it (FP32 at 24^3x48: 33 us cached, 44 us streamed).
  const bool stream = (size_t)8 * nk * g.vh * E > kLinkStreamBytes;
  M3<R> U;
  if (nk == 9) {
    if (stream) {
#pragma unroll
      for (int k = 0; k < 9; ++k) U.m[k] = ld_buf_nt<R>(ru, (unsigned)cb * E, k * gs);
    } else {
#pragma unroll
      for (int k = 0; k < 9; ++k) U.m[k] = ld_buf<R>(ru, (unsigned)cb * E, k * gs);
    }
  } else {
    if (stream) {
#pragma unroll
      for (int k = 0; k < 6; ++k) U.m[k] = ld_buf_nt<R>(ru, (unsigned)cb * E, k * gs);
    } else {
#pragma unroll
      for (int k = 0; k < 6; ++k) U.m[k] = ld_buf<R>(ru, (unsigned)cb * E, k * gs);
    }
    U.m[6] = conj(U.m[1] * U.m[5] - U.m[2] * U.m[4]);
    U.m[7] = conj(U.m[2] * U.m[3] - U.m[0] * U.m[5]);
    U.m[8] = conj(U.m[0] * U.m[4] - U.m[1] * U.m[3]);
  }
  return U;
}

// The hop from x + mu (forward) or x - mu (backward) along MU for output
// site (p, cb) with coordinates c, right-hand side n of the loader's field,
// added to acc.
template <typename R, int MU, bool DAG, typename L>
__device__ __forceinline__ void hop_fwd(const Geom& g, const R2<R>* __restrict__ gauge, int nk, const L& in, int p,
                                        int cb, const int c[4], C<R>* acc, int n) {
  constexpr int SF = DAG ? +1 : -1;  // forward projector 1 + SF gamma
  C<R> psi[12], h[6], w[6];
  // (1 + SF gamma) U_mu(x) psi(x + mu)
  const unsigned of = in.off(cb_shift(g, c, MU, +1), n);
#pragma unroll
  for (int k = 0; k < 12; ++k) psi[k] = in.ld(of, k);
  project<R, MU, SF>(psi, h);
  const M3<R> U = load_link<R>(gauge, nk, g, p, MU, cb);
  umul(U, h, w);
  if (MU == 3 && c[3] == g.L[3] - 1) apply_bc(g, w);
  reconstruct<R, MU, SF>(w, acc);
}
template <typename R, int MU, bool DAG, typename L>
__device__ __forceinline__ void hop_bwd(const Geom& g, const R2<R>* __restrict__ gauge, int nk, const L& in, int p,
                                        const int c[4], C<R>* acc, int n) {
  constexpr int SB = DAG ? -1 : +1;  // backward projector 1 + SB gamma
  C<R> psi[12], h[6], w[6];
  // (1 + SB gamma) U_mu(x - mu)^dag psi(x - mu)
  const int nb = cb_shift(g, c, MU, -1);
  const unsigned ob = in.off(nb, n);
#pragma unroll
  for (int k = 0; k < 12; ++k) psi[k] = in.ld(ob, k);
  project<R, MU, SB>(psi, h);
  const M3<R> U = load_link<R>(gauge, nk, g, 1 - p, MU, nb);
  umul_dag(U, h, w);
  if (MU == 3 && c[3] == 0) apply_bc(g, w);
  reconstruct<R, MU, SB>(w, acc);
}

// Both hops along MU (forward first), right-hand side n.
template <typename R, int MU, bool DAG, typename L>
__device__ __forceinline__ void hop_dir(const Geom& g, const R2<R>* __restrict__ gauge, int nk, const L& in, int p,
                                        int cb, const int c[4], C<R>* acc, int n) {
  hop_fwd<R, MU, DAG>(g, gauge, nk, in, p, cb, c, acc, n);
  hop_bwd<R, MU, DAG>(g, gauge, nk, in, p, c, acc, n);
}

// One of the two hops along MU, chosen per lane (bwd): the form of the
// half-wave hop kernel, whose lanes 0-31 take the forward and lanes 32-63 the
// backward hop of the same 32 sites.  Both halves run the same instructions:
// the neighbour, the link's parity and site, the projector sign, the dagger
// and the boundary test are per-lane values, and the link resource spans
// both parities so that its base stays uniform (the host keeps the gauge
// field of a lattice this kernel runs on far below 4 GiB).
template <typename R, int MU, bool DAG, typename L>
__device__ __forceinline__ void hop_one(const Geom& g, const R2<R>* __restrict__ gauge, int nk, const L& in, int p,
                                        int cb, const int c[4], C<R>* acc, bool bwd) {
  constexpr int SF = DAG ? +1 : -1;  // forward projector 1 + SF gamma, backward 1 - SF gamma
  constexpr unsigned E = sizeof(R2<R>);
  const R s = bwd ? R(-SF) : R(SF);
  const int nb = cb_shift(g, c, MU, bwd ? -1 : +1);
  C<R> psi[12], h[6], w[6];
  const unsigned o = in.off(nb, 0);
#pragma unroll
  for (int k = 0; k < 12; ++k) psi[k] = in.ld(o, k);
  project_s<R, MU>(psi, s, h);
  // U_mu(x) of parity p at cb, or U_mu(x - mu) of parity 1 - p at nb
  const unsigned gs = (unsigned)g.vh * E;
  const BufRsrc ru = make_rsrc(gauge, (size_t)8 * nk * gs);
  const unsigned lo = ((unsigned)(((bwd ? 1 - p : p) * 4 + MU) * nk) * (unsigned)g.vh + (unsigned)(bwd ? nb : cb)) * E;
  M3<R> U;
  if (nk == 9) {
#pragma unroll
    for (int k = 0; k < 9; ++k) U.m[k] = ld_buf<R>(ru, lo, k * gs);
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) U.m[k] = ld_buf<R>(ru, lo, k * gs);
    U.m[6] = conj(U.m[1] * U.m[5] - U.m[2] * U.m[4]);
    U.m[7] = conj(U.m[2] * U.m[3] - U.m[0] * U.m[5]);
    U.m[8] = conj(U.m[0] * U.m[4] - U.m[1] * U.m[3]);
  }
  M3<R> A;  // U, or U^dag on the backward lanes
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) A.m[3 * i + j] = bwd ? conj(U.m[3 * j + i]) : U.m[3 * i + j];
  umul(A, h, w);
  if (MU == 3 && c[3] == (bwd ? 0 : g.L[3] - 1)) apply_bc(g, w);
  reconstruct_s<R, MU>(w, s, acc);
}

// The same with the two links already loaded (Uf = U_mu(x), Ub = U_mu(x-mu))
// and the loader offsets of the two neighbours given: the form the batched
// hop uses to apply one pair of links to several right-hand sides.
template <typename R, int MU, bool DAG, typename L>
__device__ __forceinline__ void hop_dir_u(const Geom& g, const M3<R>& Uf, const M3<R>& Ub, const L& in,
                                          unsigned of, unsigned ob, const int c[4], C<R>* acc) {
  constexpr int SF = DAG ? +1 : -1;
  constexpr int SB = -SF;
  C<R> psi[12], h[6], w[6];
#pragma unroll
  for (int k = 0; k < 12; ++k) psi[k] = in.ld(of, k);
  project<R, MU, SF>(psi, h);
  umul(Uf, h, w);
  if (MU == 3 && c[3] == g.L[3] - 1) apply_bc(g, w);
  reconstruct<R, MU, SF>(w, acc);
#pragma unroll
  for (int k = 0; k < 12; ++k) psi[k] = in.ld(ob, k);
  project<R, MU, SB>(psi, h);
  umul_dag(Ub, h, w);
  if (MU == 3 && c[3] == 0) apply_bc(g, w);
  reconstruct<R, MU, SB>(w, acc);
}

}  // namespace lgt
