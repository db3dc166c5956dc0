// SU(3) device functions shared by the force and stout kernels: link access
// by coordinates, the plaquette staple sum, exp of su(3) and reunitarization.
#pragma once

#include "lgt_device.h"

namespace lgt {

// Order of the 64-site blocks of the gauge-link kernels (staple force,
// stout levels; logical block lb, parity lb & 1, so the two parities of a
// site block run side by side).  On lattices above 131072 sites per parity
// whose t-slice holds whole blocks: where the (x, y) plane holds nyc whole
// blocks and Lz, Lt are multiples of 4, t fastest within groups of 4
// t-slices, then z within groups of 4 planes, then the nyc blocks of a
// plane, then the z groups, then the t groups; otherwise t fastest within
// groups of tgrp t-slices of bps blocks.  A block's neighbours in t and z
// were then read a few dozen blocks earlier on the same XCD (32^3x64, staple
// force: 1501 -> 1374 us; stout levels 9.3 -> 8.0 ms).
struct BlockOrder {
  int bps, tgrp, nyc;
};
__host__ __device__ inline BlockOrder gauge_block_order(const Geom& g) {
  BlockOrder o{0, 0, 0};
  const int vslice = g.vh / g.L[3];
  o.bps = vslice / 64;
  if (vslice % 64 != 0 || o.bps == 0 || g.vh <= 131072) return o;
  o.tgrp = g.L[3] % 8 == 0 ? 8 : (g.L[3] % 4 == 0 ? 4 : 2);
  const int plane = g.hx * g.L[1];
  if (plane % 64 == 0 && g.L[2] % 4 == 0 && g.L[3] % 4 == 0) o.nyc = plane / 64;
  return o;
}
__device__ __forceinline__ int gauge_site_block(int lb, const BlockOrder& o, int lz) {
  int r = lb >> 1;
  if (o.nyc > 0) {
    const int t_in = r & 3;
    r >>= 2;
    const int z_in = r & 3;
    r >>= 2;
    const int yc = r % o.nyc;
    r /= o.nyc;
    const int nzg = lz >> 2;
    const int zo = r % nzg, to = r / nzg;
    return ((to * 4 + t_in) * lz + zo * 4 + z_in) * o.nyc + yc;
  }
  if (o.tgrp > 0) {
    const int span = o.tgrp * o.bps;
    const int grp = r / span, rem = r - grp * span;
    const int chunk = rem / o.tgrp, tl = rem - chunk * o.tgrp;
    return (grp * o.tgrp + tl) * o.bps + chunk;
  }
  return r;
}

__device__ __forceinline__ M3<double> link_at(const double2* U, const Geom& g, const int c[4], int mu) {
  return load_m3<double>(gptr<double>(U, g, parity_of(c), mu), g.vh, cb_of(g, c));
}


// Plaquette staple sum of the link U_mu(x):
//   A = sum_{nu != mu} [ U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
//                      + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu) ],
// so that the plaquettes through U_mu(x) sum to Re tr(U_mu(x) A).
__device__ __forceinline__ M3<double> staple_A(const double2* U, const Geom& g, const int c[4], int mu) {
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
    {
      const M3<double> u1 = link_at(U, g, xpm, nu), u2 = link_at(U, g, xpn, mu), u3 = link_at(U, g, c, nu);
      A = mmac_nd(A, mmul_nd(u1, u2), u3);
    }
    {
      const M3<double> v1 = link_at(U, g, xpmmn, nu), v2 = link_at(U, g, xmn, mu), v3 = link_at(U, g, xmn, nu);
      A = mmac_dn(A, mmul(v2, v1), v3);
    }
  }
  return A;
}

// ---------------------------------------------------------------------------
// exp(X) for traceless anti-Hermitian X, by Cayley-Hamilton: with Q = -iX
// (Hermitian, traceless), exp(iQ) = f0 + f1 Q + f2 Q^2 and the f_j of
// Morningstar & Peardon (Phys. Rev. D 69, 054501), using
// c0 = det Q = tr(Q^3)/3, c1 = tr(Q^2)/2 and the symmetry
// f_j(-c0) = (-1)^j conj(f_j(c0)).  Below c1 = 1e-10 a 4th-order series
// through Q^3 = c1 Q + c0 is used instead (error < 1e-25).
// ---------------------------------------------------------------------------
__device__ __forceinline__ M3<double> exp_ah(const M3<double>& X) {
  M3<double> Q;
#pragma unroll
  for (int k = 0; k < 9; ++k) Q.m[k] = cmk<double>(X.m[k].im, -X.m[k].re);  // -i X
  const M3<double> Q2 = mmul(Q, Q);
  const double c1 = 0.5 * (Q2.m[0].re + Q2.m[4].re + Q2.m[8].re);
  double c0 = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) c0 += (Q2.m[3 * i + j] * Q.m[3 * j + i]).re;
  c0 *= (1.0 / 3.0);
  C<double> f0, f1, f2;
  if (c1 < 1e-10) {
    f0 = cmk(1.0, -c0 / 6.0);
    f1 = cmk(c0 / 24.0, 1.0 - c1 / 6.0);
    f2 = cmk(-0.5 + c1 / 24.0, 0.0);
  } else {
    const bool neg = c0 < 0.0;
    const double c0a = fabs(c0);
    const double c0max = 2.0 * c1 / 3.0 * sqrt(c1 / 3.0);
    double ratio = c0a / c0max;
    ratio = ratio > 1.0 ? 1.0 : ratio;
    const double theta = acos(ratio);
    const double u = sqrt(c1 / 3.0) * cos(theta / 3.0);
    const double w = sqrt(c1) * sin(theta / 3.0);
    const double w2 = w * w, u2 = u * u;
    const double xi0 = fabs(w) < 0.05 ? 1.0 - w2 / 6.0 * (1.0 - w2 / 20.0 * (1.0 - w2 / 42.0)) : sin(w) / w;
    const double cw = cos(w);
    const C<double> e2iu = cmk(cos(2.0 * u), sin(2.0 * u));
    const C<double> emiu = cmk(cos(u), -sin(u));
    const C<double> h0 = (u2 - w2) * e2iu + emiu * cmk(8.0 * u2 * cw, 2.0 * u * (3.0 * u2 + w2) * xi0);
    const C<double> h1 = (2.0 * u) * e2iu - emiu * cmk(2.0 * u * cw, -(3.0 * u2 - w2) * xi0);
    const C<double> h2 = e2iu - emiu * cmk(cw, 3.0 * u * xi0);
    const double inv = 1.0 / (9.0 * u2 - w2);
    f0 = inv * h0;
    f1 = inv * h1;
    f2 = inv * h2;
    if (neg) {
      f0 = conj(f0);
      f1 = -conj(f1);
      f2 = conj(f2);
    }
  }
  M3<double> E;
#pragma unroll
  for (int k = 0; k < 9; ++k) E.m[k] = f1 * Q.m[k] + f2 * Q2.m[k];
  E.m[0] += f0;
  E.m[4] += f0;
  E.m[8] += f0;
  return E;
}

// Row Gram-Schmidt on rows 1 and 2, row 3 = conj(row1 x row2).
__device__ __forceinline__ M3<double> reunitarize(const M3<double>& a) {
  C<double> r1[3], r2[3];
  double n1 = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) n1 += norm2(a.m[j]);
  n1 = 1.0 / sqrt(n1);
#pragma unroll
  for (int j = 0; j < 3; ++j) r1[j] = n1 * a.m[j];
  C<double> d = czero<double>();
#pragma unroll
  for (int j = 0; j < 3; ++j) d += cjmul(r1[j], a.m[3 + j]);
#pragma unroll
  for (int j = 0; j < 3; ++j) r2[j] = a.m[3 + j] - d * r1[j];
  double n2 = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) n2 += norm2(r2[j]);
  n2 = 1.0 / sqrt(n2);
#pragma unroll
  for (int j = 0; j < 3; ++j) r2[j] = n2 * r2[j];
  M3<double> o;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    o.m[j] = r1[j];
    o.m[3 + j] = r2[j];
  }
  o.m[6] = conj(r1[1] * r2[2] - r1[2] * r2[1]);
  o.m[7] = conj(r1[2] * r2[0] - r1[0] * r2[2]);
  o.m[8] = conj(r1[0] * r2[1] - r1[1] * r2[0]);
  return o;
}

}  // namespace lgt
