// Layout conversion and vector (BLAS-1) kernels of the solver.
//
// Layout conversion: the ABI's canonical site-major complex128 arrays
// [V][nc] are transposed, through LDS, into the internal even/odd
// structure-of-arrays [parity][nc][V/2], so both the global reads and the
// global writes are unit-stride across a wavefront.
//
// Vector kernels work on flat arrays of n complex numbers (grid-stride,
// unit-stride).  Reductions write block partials; the one-block finalize
// kernel sums them in a fixed order (deterministic, see block_partials).
#include <algorithm>

#include "lgt_internal.h"

namespace lgt {

constexpr int kPackSites = 64;  // lexicographic sites per pack block (32 per parity)

template <int NC, bool W32>
__global__ __launch_bounds__(256) void k_pack(Geom g, const double2* __restrict__ canon,
                                              double2* __restrict__ out64, float2* __restrict__ out32,
                                              int* nonfinite) {
  __shared__ double2 tile[NC][kPackSites];
  __shared__ int par[kPackSites];
  const int V = 2 * g.vh;
  const int s0 = blockIdx.x * kPackSites;
  const int nsite = min(kPackSites, V - s0);
  bool bad = false;
  for (int e = threadIdx.x; e < nsite * NC; e += 256) {
    double2 v = canon[(size_t)s0 * NC + e];
    bad |= !(isfinite(v.x) && isfinite(v.y));
    tile[e % NC][e / NC] = v;
  }
  if (threadIdx.x < nsite) {
    int c[4];
    lex_coords(g, s0 + threadIdx.x, c);
    par[threadIdx.x] = parity_of(c);
  }
  if (bad && nonfinite) atomicOr(nonfinite, 1);
  __syncthreads();
  const int half = kPackSites / 2;
  const int cb0 = s0 / 2;
  for (int e = threadIdx.x; e < 2 * NC * half; e += 256) {
    const int p = e / (NC * half);
    const int k = (e / half) % NC;
    const int j = e % half;
    if (2 * j >= nsite) continue;
    // of the two sites s0+2j, s0+2j+1 (same cb index) pick the one of parity p
    const int site = (par[2 * j] == p) ? 2 * j : 2 * j + 1;
    const double2 v = tile[k][site];
    const size_t o = ((size_t)p * NC + k) * g.vh + cb0 + j;
    out64[o] = v;
    if (W32) out32[o] = make_float2((float)v.x, (float)v.y);
  }
}

template <int NC>
__global__ __launch_bounds__(256) void k_unpack(Geom g, const double2* __restrict__ packed,
                                                double2* __restrict__ canon) {
  __shared__ double2 tile[NC][kPackSites];
  __shared__ int par[kPackSites];
  const int V = 2 * g.vh;
  const int s0 = blockIdx.x * kPackSites;
  const int nsite = min(kPackSites, V - s0);
  if (threadIdx.x < nsite) {
    int c[4];
    lex_coords(g, s0 + threadIdx.x, c);
    par[threadIdx.x] = parity_of(c);
  }
  __syncthreads();
  const int half = kPackSites / 2;
  const int cb0 = s0 / 2;
  for (int e = threadIdx.x; e < 2 * NC * half; e += 256) {
    const int p = e / (NC * half);
    const int k = (e / half) % NC;
    const int j = e % half;
    if (2 * j >= nsite) continue;
    const int site = (par[2 * j] == p) ? 2 * j : 2 * j + 1;
    tile[k][site] = packed[((size_t)p * NC + k) * g.vh + cb0 + j];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nsite * NC; e += 256) canon[(size_t)s0 * NC + e] = tile[e % NC][e / NC];
}

hipError_t launch_pack(const Geom& g, int nc, const double2* canon, double2* out64, float2* out32,
                       int* nonfinite, hipStream_t s) {
  const int V = 2 * g.vh;
  const int nb = (V + kPackSites - 1) / kPackSites;
  if (nc == 12) {
    if (out32) hipLaunchKernelGGL((k_pack<12, true>), dim3(nb), dim3(256), 0, s, g, canon, out64, out32, nonfinite);
    else hipLaunchKernelGGL((k_pack<12, false>), dim3(nb), dim3(256), 0, s, g, canon, out64, out32, nonfinite);
  } else if (nc == 36) {
    if (out32) hipLaunchKernelGGL((k_pack<36, true>), dim3(nb), dim3(256), 0, s, g, canon, out64, out32, nonfinite);
    else hipLaunchKernelGGL((k_pack<36, false>), dim3(nb), dim3(256), 0, s, g, canon, out64, out32, nonfinite);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// HMC momentum refresh (Sec. III B): Pi = i sum_a c_a T_a, T_a = lambda_a / 2
// (Gell-Mann), from eight normals c_a per link, canonical [V][4][3][3].
// Written out per element (traceless anti-Hermitian by construction).
__global__ __launch_bounds__(256) void k_momenta(size_t nlinks, const double* __restrict__ c,
                                                 double2* __restrict__ P) {
  const size_t l = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (l >= nlinks) return;
  const double* a = c + 8 * l;
  const double h = 0.5, r3 = 0.57735026918962576451;  // 1/sqrt(3)
  double2* q = P + 9 * l;
  q[0] = make_double2(0.0, h * (a[2] + r3 * a[7]));
  q[1] = make_double2(h * a[1], h * a[0]);
  q[2] = make_double2(h * a[4], h * a[3]);
  q[3] = make_double2(-h * a[1], h * a[0]);
  q[4] = make_double2(0.0, h * (-a[2] + r3 * a[7]));
  q[5] = make_double2(h * a[6], h * a[5]);
  q[6] = make_double2(-h * a[4], h * a[3]);
  q[7] = make_double2(-h * a[6], h * a[5]);
  q[8] = make_double2(0.0, -2.0 * h * r3 * a[7]);
}
hipError_t launch_momenta(const Geom& g, const double* normals, double2* P, hipStream_t s) {
  const size_t n = (size_t)2 * g.vh * 4;
  hipLaunchKernelGGL(k_momenta, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, normals, P);
  return hipGetLastError();
}

hipError_t launch_unpack(const Geom& g, int nc, const double2* packed, double2* canon, hipStream_t s) {
  const int V = 2 * g.vh;
  const int nb = (V + kPackSites - 1) / kPackSites;
  if (nc == 12) hipLaunchKernelGGL((k_unpack<12>), dim3(nb), dim3(256), 0, s, g, packed, canon);
  else if (nc == 36) hipLaunchKernelGGL((k_unpack<36>), dim3(nb), dim3(256), 0, s, g, packed, canon);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Vector kernels
// ---------------------------------------------------------------------------
static inline int vec_blocks(int n) {
  int nb = (n + 255) / 256;
  return nb < 1024 ? (nb < 1 ? 1 : nb) : 1024;
}

template <typename R>
__global__ __launch_bounds__(256) void k_cg_init(int n, const R2<R>* __restrict__ b, R2<R>* __restrict__ r,
                                                 R2<R>* __restrict__ p, R2<R>* __restrict__ x, double* partials) {
  double acc = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const R2<R> v = b[i];
    r[i] = v;
    p[i] = v;
    R2<R> z;
    z.x = R(0);
    z.y = R(0);
    x[i] = z;
    acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
  }
  double v[1] = {acc};
  block_partials<256, 1>(v, partials, blockIdx.x);
}

template <typename R>
hipError_t launch_cg_init(int n, const R2<R>* b, R2<R>* r, R2<R>* p, R2<R>* x, SolverState* st,
                          Reduce red, double tol, int max_iter, hipStream_t s) {
  const int nb = vec_blocks(n);
  hipLaunchKernelGGL((k_cg_init<R>), dim3(nb), dim3(256), 0, s, n, b, r, p, x, red.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(kFinCgInit, nb, red, st, 0, tol, max_iter, s);
}

// One block: sum the partials of the previous launch and act on the totals.
template <int NV>
__global__ __launch_bounds__(256) void k_finalize(int mode, int nblk, const double* __restrict__ partials,
                                                  SolverState* st, double* result, double tol, int max_iter,
                                                  Mailbox* mb) {
  double tot[NV];
  sum_partials<256, NV>(partials, nblk, tot);
  if (threadIdx.x != 0) return;
  if (mode == kFinResult1 || mode == kFinResult2) {
#pragma unroll
    for (int k = 0; k < NV; ++k) result[k] = tot[k];
  } else if (mode == kFinCgInit) {
    const double rr = tot[0];
    st->rr = rr;
    st->rr0 = rr;
    st->rr_max = rr;
    st->rr_stop = tol * tol * rr;
    st->iter = 0;
    st->max_iter = max_iter;
    st->alpha = 0.0;
    st->beta = 0.0;
    st->pap = 0.0;
    st->delta2 = 0.0;
    st->done = !isfinite(rr) ? kDoneBreakdown : (rr == 0.0 ? kDoneConverged : kDoneRunning);
  }
}

hipError_t launch_finalize(int mode, int nblk, Reduce red, SolverState* st, int slot, double tol, int max_iter,
                           hipStream_t s) {
  if (nblk > red.capacity) return hipErrorInvalidValue;
  if (mode == kFinResult2)
    hipLaunchKernelGGL(k_finalize<2>, dim3(1), dim3(256), 0, s, mode, nblk, red.partials, st, red.result + slot,
                       tol, max_iter, red.mbox);
  else
    hipLaunchKernelGGL(k_finalize<1>, dim3(1), dim3(256), 0, s, mode, nblk, red.partials, st, red.result + slot,
                       tol, max_iter, red.mbox);
  return hipGetLastError();
}

template <typename R, typename T>
__global__ __launch_bounds__(256) void k_cg_step(int n, int nblk, const double* __restrict__ partials,
                                                 const R2<R>* __restrict__ r, T* __restrict__ p, SolverState* st,
                                                 Mailbox* mb, R2<R>* __restrict__ x) {
  const int done0 = st->done;
  if (done0 != kDoneRunning) {  // the iteration was skipped (or block 0 below already stopped it)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (done0 == kDoneUpdate) st->done = kDoneUpdateHeld;
      // the same action as the stop itself, in case the host has not seen it
      post_progress(mb, st->iter, action_word(st->epoch, done0 == kDoneUpdateHeld ? kDoneUpdate : done0));
    }
    return;
  }
  // every block forms the same rr (same partials, same order) and so takes
  // the same decision; the inputs are the copies the third hop made, which
  // block 0's writes below do not touch
  __shared__ double s_rr;
  double tot[1];
  sum_partials<256, 1>(partials, nblk, tot);
  if (threadIdx.x == 0) s_rr = tot[0];
  __syncthreads();
  const double rr = s_rr;
  const double beta = rr / st->rr_prev;
  const int iter = st->iter_prev + 1;
  const double rr_max = fmax(st->rr_max, rr);  // block 0 may have stored this same value already
  int code = kDoneRunning;
  if (!isfinite(rr)) code = kDoneBreakdown;
  else if (rr <= st->rr_stop) code = st->delta2 > 0.0 ? kDoneUpdate : kDoneConverged;
  else if (rr <= st->delta2 * rr_max) code = kDoneUpdate;
  else if (iter >= st->max_iter) code = kDoneMaxIter;
  {
    // x += alpha p (this iteration's step, taken whatever the decision), then
    // p = r + beta p unless the recursion stops; four elements per thread and
    // trip, all loads issued before the stores
    const R b = R(beta), a = R(st->alpha);
    const bool upd = code == kDoneRunning;
    const int stride = gridDim.x * 256;
    int i = blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
      C<R> rv[4], pv[4], xv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        pv[j] = Store<R, T>::ld(p + i + j * stride);
        xv[j] = ld<R>(x + i + j * stride);
        if (upd) rv[j] = ld<R>(r + i + j * stride);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        lgt::st<R>(x + i + j * stride, xv[j] + a * pv[j]);
        if (upd) Store<R, T>::st(p + i + j * stride, C<R>{rv[j].re + b * pv[j].re, rv[j].im + b * pv[j].im});
      }
    }
    for (; i < n; i += stride) {
      const C<R> pv = Store<R, T>::ld(p + i);
      lgt::st<R>(x + i, ld<R>(x + i) + a * pv);
      if (upd) {
        const C<R> rv = ld<R>(r + i);
        Store<R, T>::st(p + i, C<R>{rv.re + b * pv.re, rv.im + b * pv.im});
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->beta = beta;
    st->rr = rr;
    st->iter = iter;
    st->rr_max = rr_max;
    if (code != kDoneRunning) st->done = code;
    post_progress(mb, iter, code != kDoneRunning ? action_word(st->epoch, code) : 0u);
  }
}

template <typename R, typename T>
hipError_t launch_cg_step(int n, const R2<R>* r, T* p, SolverState* st, Reduce red, int nblk, hipStream_t s,
                          R2<R>* x) {
  if (nblk > red.capacity) return hipErrorInvalidValue;
  // each block also sums the nblk partials (a few thousand on large
  // lattices).  With 8-byte elements (FP32, BF16 pairs) a grid of about four
  // elements per thread, at most 1024 blocks, keeps those re-reads small next
  // to the vector work (16^4: 4.6 -> 4.1 us, 24^3x48: 23.2 -> 20.3 us); FP64
  // elements keep enough loads in flight with one per thread (at most 2048
  // blocks), which is faster for them at 16^4 (6.3 against 7.1 us).
  const int nb = sizeof(R) == 4 ? std::max(1, std::min((n + 1023) / 1024, 1024))
                                : std::max(1, std::min((n + 255) / 256, 2048));
  hipLaunchKernelGGL((k_cg_step<R, T>), dim3(nb), dim3(256), 0, s, n, nblk, red.partials, r, p, st, red.mbox, x);
  return hipGetLastError();
}
template hipError_t launch_cg_step<double, double2>(int, const double2*, double2*, SolverState*, Reduce, int,
                                                    hipStream_t, double2*);
template hipError_t launch_cg_step<float, float2>(int, const float2*, float2*, SolverState*, Reduce, int,
                                                  hipStream_t, float2*);
template hipError_t launch_cg_step<float, Bf16c>(int, const float2*, Bf16c*, SolverState*, Reduce, int,
                                                 hipStream_t, float2*);

__global__ __launch_bounds__(256) void k_norm_dot(int n, const double2* __restrict__ a,
                                                  const double2* __restrict__ b, double* partials) {
  double nn = 0.0, dd = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const double2 av = a[i];
    nn += av.x * av.x + av.y * av.y;
    if (b) {
      const double2 bv = b[i];
      dd += av.x * bv.x + av.y * bv.y;
    }
  }
  double v[2] = {nn, dd};
  block_partials<256, 2>(v, partials, blockIdx.x);
}

hipError_t launch_norm_dot(int n, const double2* a, const double2* b, Reduce red, int slot, hipStream_t s) {
  const int nb = vec_blocks(n);
  hipLaunchKernelGGL(k_norm_dot, dim3(nb), dim3(256), 0, s, n, a, b, red.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(kFinResult2, nb, red, nullptr, slot, 0.0, 0, s);
}

__global__ __launch_bounds__(256) void k_axpy64(int n, double a, const double2* __restrict__ x,
                                                double2* __restrict__ y) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const double2 xv = x[i];
    double2 yv = y[i];
    yv.x += a * xv.x;
    yv.y += a * xv.y;
    y[i] = yv;
  }
}
hipError_t launch_axpy64(int n, double a, const double2* x, double2* y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy64, dim3((n + 255) / 256), dim3(256), 0, s, n, a, x, y);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_copy64(int n, const double2* __restrict__ x, double2* __restrict__ y) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) y[i] = x[i];
}
hipError_t launch_copy64(int n, const double2* x, double2* y, hipStream_t s) {
  hipLaunchKernelGGL(k_copy64, dim3((n + 255) / 256), dim3(256), 0, s, n, x, y);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_xmy64(int n, const double2* __restrict__ x, double2* __restrict__ y) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const double2 xv = x[i];
    double2 yv = y[i];
    yv.x = xv.x - yv.x;
    yv.y = xv.y - yv.y;
    y[i] = yv;
  }
}
hipError_t launch_xmy64(int n, const double2* x, double2* y, hipStream_t s) {
  hipLaunchKernelGGL(k_xmy64, dim3((n + 255) / 256), dim3(256), 0, s, n, x, y);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_zero64(int n, double2* __restrict__ y) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) y[i] = make_double2(0.0, 0.0);
}
hipError_t launch_zero64(int n, double2* y, hipStream_t s) {
  hipLaunchKernelGGL(k_zero64, dim3((n + 255) / 256), dim3(256), 0, s, n, y);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_zero32(int n, float2* __restrict__ y) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) y[i] = make_float2(0.f, 0.f);
}
hipError_t launch_zero32(int n, float2* y, hipStream_t s) {
  hipLaunchKernelGGL(k_zero32, dim3((n + 255) / 256), dim3(256), 0, s, n, y);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_convert_64_32(int n, const double2* __restrict__ x, float2* __restrict__ y) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const double2 v = x[i];
    y[i] = make_float2((float)v.x, (float)v.y);
  }
}
hipError_t launch_convert_64_32(int n, const double2* x, float2* y, hipStream_t s) {
  hipLaunchKernelGGL(k_convert_64_32, dim3((n + 255) / 256), dim3(256), 0, s, n, x, y);
  return hipGetLastError();
}

// Two-row copy of a packed link field ([2][4][9][vh] -> [2][4][6][vh]) and
// the check that the links are SU(3): flag is set when a stored third row
// differs from the conjugate cross product of the first two by more than tol
// (per component, |re| + |im|), or is not finite.
// FP64 links whose stored third row is within this of the rebuilt one (a few
// dozen rounding units) are taken as SU(3) by the FP64 solver's hops.
constexpr double kTwoRowTol64 = 1e-14;

template <typename R>
__global__ __launch_bounds__(256) void k_compress_links(int vh, const R2<R>* __restrict__ U, R2<R>* __restrict__ Uc,
                                                        int* flag, R tol) {
  const int t = blockIdx.x * 256 + threadIdx.x;  // link (parity, mu) slowest, site fastest
  if (t >= 8 * vh) return;
  const int pm = t / vh, cb = t - pm * vh;
  const R2<R>* src = U + (size_t)pm * 9 * vh + cb;
  R2<R>* dst = Uc + (size_t)pm * 6 * vh + cb;
  C<R> m[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) m[k] = ld<R>(src + (size_t)k * vh);
#pragma unroll
  for (int k = 0; k < 6; ++k) st<R>(dst + (size_t)k * vh, m[k]);
  const C<R> r6 = conj(m[1] * m[5] - m[2] * m[4]);
  const C<R> r7 = conj(m[2] * m[3] - m[0] * m[5]);
  const C<R> r8 = conj(m[0] * m[4] - m[1] * m[3]);
  const R dev = fmax(fmax(fabs(r6.re - m[6].re) + fabs(r6.im - m[6].im),
                          fabs(r7.re - m[7].re) + fabs(r7.im - m[7].im)),
                     fabs(r8.re - m[8].re) + fabs(r8.im - m[8].im));
  if (!(dev <= tol)) *flag = 1;  // also for NaN
}
hipError_t launch_compress_links(const Geom& g, const float2* U32, float2* Uc, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_compress_links<float>, dim3((8 * g.vh + 255) / 256), dim3(256), 0, s, g.vh, U32, Uc, flag,
                     1e-5f);
  return hipGetLastError();
}
hipError_t launch_compress_links(const Geom& g, const double2* U64, double2* Uc, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_compress_links<double>, dim3((8 * g.vh + 255) / 256), dim3(256), 0, s, g.vh, U64, Uc, flag,
                     kTwoRowTol64);
  return hipGetLastError();
}

// x (FP64) += scale * xs (FP32); xs = 0
__global__ __launch_bounds__(256) void k_mixed_fold(int n, float2* xs, double2* __restrict__ x,
                                                    const SolverState* st) {
  const double scale = 1.0 / st->sigma;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const float2 v = xs[i];
    double2 xv = x[i];
    xv.x += scale * (double)v.x;
    xv.y += scale * (double)v.y;
    x[i] = xv;
    xs[i] = make_float2(0.f, 0.f);
  }
}
hipError_t launch_mixed_fold(int n, float2* xs, double2* x, const SolverState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_mixed_fold, dim3((n + 255) / 256), dim3(256), 0, s, n, xs, x, st);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_reliable_decide(int nblk, const double* __restrict__ partials,
                                                         SolverState* st, Mailbox* mb) {
  double tot[2];
  sum_partials<256, 2>(partials, nblk, tot);
  if (threadIdx.x != 0) return;
  const double rr64 = tot[0];
  const int entry = st->done;
  st->nupd += 1;
  st->epoch += 1;
  int code = kDoneRunning;
  if (!isfinite(rr64)) {
    code = kDoneFailed;
  } else if (rr64 <= st->rr_target) {
    code = kDoneConverged;
  } else {
    const double sn = 1.0 / sqrt(rr64);
    st->restart = entry == kDoneBreakdown;
    st->bscale = st->beta * sn / st->sigma;
    st->sigma = sn;
    st->rr = 1.0;
    st->rr0 = 1.0;
    st->rr_max = 1.0;
    st->rr_stop = st->rr_target * sn * sn;
  }
  st->done = code;
  post_progress(mb, st->iter, code != kDoneRunning ? action_word(st->epoch, code) : 0u);
}
hipError_t launch_reliable_decide(int n, const double2* r64, Reduce red, SolverState* st, hipStream_t s) {
  const int nb = vec_blocks(n);
  if (nb > red.capacity) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_norm_dot, dim3(nb), dim3(256), 0, s, n, r64, (const double2*)nullptr, red.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reliable_decide, dim3(1), dim3(256), 0, s, nb, red.partials, st, red.mbox);
  return hipGetLastError();
}

// Reliable update of the FP32 recursion: r = sigma r64 (FP64 residual scaled
// to unit norm), and the search direction either restarted (p = r) or
// rescaled to the new units (p *= pscale).
template <typename T>
__global__ __launch_bounds__(256) void k_rescale_residual(int n, const double2* __restrict__ r64, double sigma,
                                                          float2* __restrict__ r, T* __restrict__ p, int restart,
                                                          double bscale) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const double2 v = r64[i];
    const double rx = sigma * v.x, ry = sigma * v.y;
    st<float>(r + i, C<float>{(float)rx, (float)ry});
    if (restart) {
      Store<float, T>::st(p + i, C<float>{(float)rx, (float)ry});
    } else {
      const C<float> q = Store<float, T>::ld(p + i);
      Store<float, T>::st(p + i, C<float>{(float)(rx + bscale * (double)q.re), (float)(ry + bscale * (double)q.im)});
    }
  }
}
template <typename T>
hipError_t launch_rescale_residual(int n, const double2* r64, double sigma, float2* r, T* p, int restart,
                                   double bscale, hipStream_t s) {
  hipLaunchKernelGGL((k_rescale_residual<T>), dim3((n + 255) / 256), dim3(256), 0, s, n, r64, sigma, r, p, restart,
                     bscale);
  return hipGetLastError();
}
template <typename T>
__global__ __launch_bounds__(256) void k_rescale_residual_dev(int n, const double2* __restrict__ r64,
                                                              float2* __restrict__ r, T* __restrict__ p,
                                                              const SolverState* state) {
  if (state->done != kDoneRunning) return;
  const double sigma = state->sigma, bscale = state->bscale;
  const int restart = state->restart;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const double2 v = r64[i];
    const double rx = sigma * v.x, ry = sigma * v.y;
    st<float>(r + i, C<float>{(float)rx, (float)ry});
    if (restart) {
      Store<float, T>::st(p + i, C<float>{(float)rx, (float)ry});
    } else {
      const C<float> q = Store<float, T>::ld(p + i);
      Store<float, T>::st(p + i, C<float>{(float)(rx + bscale * (double)q.re), (float)(ry + bscale * (double)q.im)});
    }
  }
}
template <typename T>
hipError_t launch_rescale_residual_dev(int n, const double2* r64, float2* r, T* p, const SolverState* st,
                                       hipStream_t s) {
  hipLaunchKernelGGL((k_rescale_residual_dev<T>), dim3((n + 255) / 256), dim3(256), 0, s, n, r64, r, p, st);
  return hipGetLastError();
}
template hipError_t launch_rescale_residual_dev<float2>(int, const double2*, float2*, float2*, const SolverState*,
                                                        hipStream_t);
template hipError_t launch_rescale_residual_dev<Bf16c>(int, const double2*, float2*, Bf16c*, const SolverState*,
                                                       hipStream_t);

template hipError_t launch_rescale_residual<float2>(int, const double2*, double, float2*, float2*, int, double,
                                                    hipStream_t);
template hipError_t launch_rescale_residual<Bf16c>(int, const double2*, double, float2*, Bf16c*, int, double,
                                                   hipStream_t);

template hipError_t launch_cg_init<double>(int, const double2*, double2*, double2*, double2*, SolverState*,
                                           Reduce, double, int, hipStream_t);
template hipError_t launch_cg_init<float>(int, const float2*, float2*, float2*, float2*, SolverState*, Reduce,
                                          double, int, hipStream_t);


}  // namespace lgt
