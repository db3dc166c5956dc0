// Device-side building blocks for the gfx950 kernels: complex arithmetic,
// SU(3) algebra, lattice geometry in the even/odd (checkerboard) layout,
// XCD-aware block numbering and the deterministic two-level reduction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lgt {

// ---------------------------------------------------------------------------
// Complex numbers.  Storage type R2 (double2 / float2) is what lives in HBM;
// arithmetic type C<R> is a plain struct the compiler keeps in VGPRs.
// ---------------------------------------------------------------------------
template <typename R> struct R2of;
template <> struct R2of<double> { using type = double2; };
template <> struct R2of<float> { using type = float2; };
template <typename R> using R2 = typename R2of<R>::type;

template <typename R> struct C { R re, im; };

template <typename R> __device__ __forceinline__ C<R> cmk(R a, R b) { return C<R>{a, b}; }
template <typename R> __device__ __forceinline__ C<R> czero() { return C<R>{R(0), R(0)}; }
template <typename R> __device__ __forceinline__ C<R> operator+(C<R> a, C<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> __device__ __forceinline__ C<R> operator-(C<R> a, C<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> __device__ __forceinline__ C<R> operator-(C<R> a) { return {-a.re, -a.im}; }
template <typename R> __device__ __forceinline__ C<R> operator*(C<R> a, C<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R> __device__ __forceinline__ C<R> operator*(R s, C<R> a) { return {s * a.re, s * a.im}; }
template <typename R> __device__ __forceinline__ C<R>& operator+=(C<R>& a, C<R> b) { a.re += b.re; a.im += b.im; return a; }
template <typename R> __device__ __forceinline__ C<R>& operator-=(C<R>& a, C<R> b) { a.re -= b.re; a.im -= b.im; return a; }
template <typename R> __device__ __forceinline__ C<R> conj(C<R> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename R> __device__ __forceinline__ C<R> cjmul(C<R> a, C<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// a * conj(b)
template <typename R> __device__ __forceinline__ C<R> mulcj(C<R> a, C<R> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename R> __device__ __forceinline__ C<R> itimes(C<R> a) { return {-a.im, a.re}; }
template <typename R> __device__ __forceinline__ R norm2(C<R> a) { return a.re * a.re + a.im * a.im; }

template <typename R> __device__ __forceinline__ C<R> ld(const R2<R>* p) {
  R2<R> v = *p;
  return {v.x, v.y};
}
template <typename R> __device__ __forceinline__ void st(R2<R>* p, C<R> a) {
  R2<R> v;
  v.x = a.re;
  v.y = a.im;
  *p = v;
}
// Raw buffer resource over [base, base + bytes) (gfx9-family descriptor):
// loads through it take a 32-bit per-lane offset plus a 32-bit uniform
// offset and need no 64-bit address arithmetic; reads past the end return
// zero rather than faulting.
typedef __amdgpu_buffer_rsrc_t BufRsrc;
__device__ __forceinline__ BufRsrc make_rsrc(const void* base, size_t bytes) {
  const unsigned n = bytes < 0xffffffffull ? (unsigned)bytes : 0xffffffffu;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)n, 0x00020000);
}
template <typename R> __device__ __forceinline__ C<R> ld_buf(BufRsrc r, unsigned voff, unsigned soff);
template <> __device__ __forceinline__ C<float> ld_buf<float>(BufRsrc r, unsigned voff, unsigned soff) {
  const float2 v = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  return {v.x, v.y};
}
template <> __device__ __forceinline__ C<double> ld_buf<double>(BufRsrc r, unsigned voff, unsigned soff) {
  const double2 v = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  return {v.x, v.y};
}
// The same with the non-temporal cache policy (cache-policy bit 1, nt): for
// data a kernel reads once (the links of a hop), so that they do not push
// the re-read spinors out of L2.
template <typename R> __device__ __forceinline__ C<R> ld_buf_nt(BufRsrc r, unsigned voff, unsigned soff);
template <> __device__ __forceinline__ C<float> ld_buf_nt<float>(BufRsrc r, unsigned voff, unsigned soff) {
  const float2 v = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 2));
  return {v.x, v.y};
}
template <> __device__ __forceinline__ C<double> ld_buf_nt<double>(BufRsrc r, unsigned voff, unsigned soff) {
  const double2 v = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 2));
  return {v.x, v.y};
}

// ---------------------------------------------------------------------------
// Storage types.  A spinor element lives in HBM as R2<R> (the arithmetic
// precision) or, for the inner solve with BF16-stored spinors, as Bf16c: a
// complex number held as two bfloat16 values (the upper 16 bits of an IEEE
// binary32), computed on in FP32.  Store<R, T> converts between the two.
// ---------------------------------------------------------------------------
struct Bf16c {
  unsigned short re, im;
};

__device__ __forceinline__ float bf16_to_f32(unsigned h) { return __uint_as_float(h << 16); }
// binary32 -> bfloat16 with round-to-nearest-even (NaN stays NaN)
__device__ __forceinline__ unsigned f32_to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

template <typename R, typename T> struct Store;
template <> struct Store<double, double2> {
  static __device__ __forceinline__ C<double> ld(const double2* p) { return lgt::ld<double>(p); }
  static __device__ __forceinline__ void st(double2* p, C<double> v) { lgt::st<double>(p, v); }
  static __device__ __forceinline__ C<double> round(C<double> v) { return v; }
  static __device__ __forceinline__ C<double> ld_buf(BufRsrc r, unsigned vo, unsigned so) {
    return lgt::ld_buf<double>(r, vo, so);
  }
};
template <> struct Store<float, float2> {
  static __device__ __forceinline__ C<float> ld(const float2* p) { return lgt::ld<float>(p); }
  static __device__ __forceinline__ void st(float2* p, C<float> v) { lgt::st<float>(p, v); }
  static __device__ __forceinline__ C<float> round(C<float> v) { return v; }
  static __device__ __forceinline__ C<float> ld_buf(BufRsrc r, unsigned vo, unsigned so) {
    return lgt::ld_buf<float>(r, vo, so);
  }
};
template <> struct Store<float, Bf16c> {
  static __device__ __forceinline__ C<float> unpack(unsigned w) {
    return {bf16_to_f32(w & 0xffffu), bf16_to_f32(w >> 16)};
  }
  static __device__ __forceinline__ C<float> ld(const Bf16c* p) { return unpack(*(const unsigned*)p); }
  static __device__ __forceinline__ void st(Bf16c* p, C<float> v) {
    *(unsigned*)p = f32_to_bf16(v.re) | (f32_to_bf16(v.im) << 16);
  }
  static __device__ __forceinline__ C<float> round(C<float> v) {
    return {bf16_to_f32(f32_to_bf16(v.re)), bf16_to_f32(f32_to_bf16(v.im))};
  }
  static __device__ __forceinline__ C<float> ld_buf(BufRsrc r, unsigned vo, unsigned so) {
    return unpack((unsigned)__builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
  }
};

// Non-temporal store: output streams that are not re-read by this kernel.
template <typename R> __device__ __forceinline__ void st_nt(R2<R>* p, C<R> a) {
  R2<R> v;
  v.x = a.re;
  v.y = a.im;
  __builtin_nontemporal_store(v, p);
}

template <typename R, typename S> __device__ __forceinline__ C<R> cvt(C<S> a) {
  return {R(a.re), R(a.im)};
}

// ---------------------------------------------------------------------------
// 3x3 complex matrices (row-major, m[3*i + j]).
// ---------------------------------------------------------------------------
template <typename R> struct M3 { C<R> m[9]; };

// Products as chains of fused multiply-adds: an element of a product is
// 2 multiplies and 10 FMAs (16 instructions as separate complex multiplies
// and adds); the accumulating forms (acc + a b) fold the sum into the chain.
template <typename R> __device__ __forceinline__ R rfma(R a, R b, R c);
template <> __device__ __forceinline__ double rfma<double>(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}
template <> __device__ __forceinline__ float rfma<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
// s + a b,  s + a conj(b),  s + conj(a) b
template <typename R> __device__ __forceinline__ C<R> cmac(C<R> s, C<R> a, C<R> b) {
  return {rfma(-a.im, b.im, rfma(a.re, b.re, s.re)), rfma(a.im, b.re, rfma(a.re, b.im, s.im))};
}
template <typename R> __device__ __forceinline__ C<R> cmac_cj(C<R> s, C<R> a, C<R> b) {
  return {rfma(a.im, b.im, rfma(a.re, b.re, s.re)), rfma(-a.re, b.im, rfma(a.im, b.re, s.im))};
}
template <typename R> __device__ __forceinline__ C<R> cjmac(C<R> s, C<R> a, C<R> b) {
  return {rfma(a.im, b.im, rfma(a.re, b.re, s.re)), rfma(-a.im, b.re, rfma(a.re, b.im, s.im))};
}
// acc + a b
template <typename R> __device__ __forceinline__ M3<R> mmac(const M3<R>& acc, const M3<R>& a, const M3<R>& b) {
  M3<R> c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      C<R> s = cmac(acc.m[3 * i + j], a.m[3 * i], b.m[j]);
      s = cmac(s, a.m[3 * i + 1], b.m[3 + j]);
      c.m[3 * i + j] = cmac(s, a.m[3 * i + 2], b.m[6 + j]);
    }
  return c;
}
// acc + a b^dag
template <typename R> __device__ __forceinline__ M3<R> mmac_nd(const M3<R>& acc, const M3<R>& a, const M3<R>& b) {
  M3<R> c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      C<R> s = cmac_cj(acc.m[3 * i + j], a.m[3 * i], b.m[3 * j]);
      s = cmac_cj(s, a.m[3 * i + 1], b.m[3 * j + 1]);
      c.m[3 * i + j] = cmac_cj(s, a.m[3 * i + 2], b.m[3 * j + 2]);
    }
  return c;
}
// acc + a^dag b
template <typename R> __device__ __forceinline__ M3<R> mmac_dn(const M3<R>& acc, const M3<R>& a, const M3<R>& b) {
  M3<R> c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      C<R> s = cjmac(acc.m[3 * i + j], a.m[i], b.m[j]);
      s = cjmac(s, a.m[3 + i], b.m[3 + j]);
      c.m[3 * i + j] = cjmac(s, a.m[6 + i], b.m[6 + j]);
    }
  return c;
}
template <typename R> __device__ __forceinline__ M3<R> mmul(const M3<R>& a, const M3<R>& b) {
  M3<R> c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const C<R> x = a.m[3 * i], y = b.m[j];
      C<R> s = {rfma(-x.im, y.im, x.re * y.re), rfma(x.im, y.re, x.re * y.im)};
      s = cmac(s, a.m[3 * i + 1], b.m[3 + j]);
      c.m[3 * i + j] = cmac(s, a.m[3 * i + 2], b.m[6 + j]);
    }
  return c;
}
// a * b^dag
template <typename R> __device__ __forceinline__ M3<R> mmul_nd(const M3<R>& a, const M3<R>& b) {
  M3<R> c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const C<R> x = a.m[3 * i], y = b.m[3 * j];
      C<R> s = {rfma(x.im, y.im, x.re * y.re), rfma(-x.re, y.im, x.im * y.re)};
      s = cmac_cj(s, a.m[3 * i + 1], b.m[3 * j + 1]);
      c.m[3 * i + j] = cmac_cj(s, a.m[3 * i + 2], b.m[3 * j + 2]);
    }
  return c;
}
// a^dag * b
template <typename R> __device__ __forceinline__ M3<R> mmul_dn(const M3<R>& a, const M3<R>& b) {
  M3<R> c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const C<R> x = a.m[i], y = b.m[j];
      C<R> s = {rfma(x.im, y.im, x.re * y.re), rfma(-x.im, y.re, x.re * y.im)};
      s = cjmac(s, a.m[3 + i], b.m[3 + j]);
      c.m[3 * i + j] = cjmac(s, a.m[6 + i], b.m[6 + j]);
    }
  return c;
}
template <typename R> __device__ __forceinline__ M3<R> madd(const M3<R>& a, const M3<R>& b) {
  M3<R> c;
#pragma unroll
  for (int k = 0; k < 9; ++k) c.m[k] = a.m[k] + b.m[k];
  return c;
}
template <typename R> __device__ __forceinline__ M3<R> mscale(R s, const M3<R>& a) {
  M3<R> c;
#pragma unroll
  for (int k = 0; k < 9; ++k) c.m[k] = s * a.m[k];
  return c;
}
template <typename R> __device__ __forceinline__ M3<R> mdag(const M3<R>& a) {
  M3<R> c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) c.m[3 * i + j] = conj(a.m[3 * j + i]);
  return c;
}
template <typename R> __device__ __forceinline__ M3<R> mident() {
  M3<R> c;
#pragma unroll
  for (int k = 0; k < 9; ++k) c.m[k] = czero<R>();
  c.m[0].re = c.m[4].re = c.m[8].re = R(1);
  return c;
}
template <typename R> __device__ __forceinline__ C<R> mtrace(const M3<R>& a) {
  return a.m[0] + a.m[4] + a.m[8];
}
// Traceless anti-Hermitian part: (A - A^dag)/2 - tr(A - A^dag)/6.
template <typename R> __device__ __forceinline__ M3<R> proj_ta(const M3<R>& a) {
  M3<R> c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      C<R> x = a.m[3 * i + j], y = a.m[3 * j + i];
      c.m[3 * i + j] = cmk<R>(R(0.5) * (x.re - y.re), R(0.5) * (x.im + y.im));
    }
  // tr(A - A^dag) = 2i Im tr A; subtract (2i Im tr A)/6 from the diagonal
  R imtr = (a.m[0].im + a.m[4].im + a.m[8].im) * (R(1) / R(3));
  c.m[0].im -= imtr;
  c.m[4].im -= imtr;
  c.m[8].im -= imtr;
  return c;
}

// ---------------------------------------------------------------------------
// Lattice geometry.  Even/odd (checkerboard) index of lexicographic site
// s = x + Lx*(y + Ly*(z + Lz*t)) with parity (x+y+z+t)&1 is cb = s/2
// (Lx even), unique within a parity.
// ---------------------------------------------------------------------------
struct Geom {
  int L[4];   // Lx, Ly, Lz, Lt
  int hx;     // Lx / 2
  int vh;     // V / 2 (sites per parity)
  int bc;     // fermion temporal boundary sign
  int hop_ns; // sites per hop block: 32 or 64, or 0 to choose by volume
  int hop_order;  // order of the 64-site blocks: 1 site order, 2 t-fastest groups, 0 by volume
};

__device__ __forceinline__ void cb_coords(const Geom& g, int p, int cb, int c[4]) {
  int xh = cb % g.hx;
  int r = cb / g.hx;
  c[1] = r % g.L[1];
  r /= g.L[1];
  c[2] = r % g.L[2];
  c[3] = r / g.L[2];
  c[0] = 2 * xh + ((p + c[1] + c[2] + c[3]) & 1);
}
__device__ __forceinline__ void lex_coords(const Geom& g, int s, int c[4]) {
  c[0] = s % g.L[0];
  int r = s / g.L[0];
  c[1] = r % g.L[1];
  r /= g.L[1];
  c[2] = r % g.L[2];
  c[3] = r / g.L[2];
}
__device__ __forceinline__ int cb_of(const Geom& g, const int c[4]) {
  return (c[0] >> 1) + g.hx * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3]));
}
__device__ __forceinline__ int parity_of(const int c[4]) { return (c[0] + c[1] + c[2] + c[3]) & 1; }
// cb index of the site c + d*mu_hat (d = +-1), periodic.
__device__ __forceinline__ int cb_shift(const Geom& g, const int c[4], int mu, int d) {
  int n[4] = {c[0], c[1], c[2], c[3]};
  int v = n[mu] + d;
  n[mu] = v < 0 ? v + g.L[mu] : (v >= g.L[mu] ? v - g.L[mu] : v);
  return cb_of(g, n);
}
__device__ __forceinline__ void shifted(const Geom& g, const int c[4], int mu, int d, int n[4]) {
  n[0] = c[0]; n[1] = c[1]; n[2] = c[2]; n[3] = c[3];
  int v = n[mu] + d;
  n[mu] = v < 0 ? v + g.L[mu] : (v >= g.L[mu] ? v - g.L[mu] : v);
}

// Packed gauge-type field: [parity][mu][9][vh] complex, element (i,j) at k = 3i+j.
template <typename R> __device__ __forceinline__ const R2<R>* gptr(const R2<R>* f, const Geom& g, int p, int mu) {
  return f + (size_t)((p * 4 + mu) * 9) * g.vh;
}
template <typename R> __device__ __forceinline__ M3<R> load_m3(const R2<R>* f, int vh, int cb) {
  M3<R> u;
#pragma unroll
  for (int k = 0; k < 9; ++k) u.m[k] = ld<R>(f + (size_t)k * vh + cb);
  return u;
}
template <typename R> __device__ __forceinline__ void store_m3(R2<R>* f, int vh, int cb, const M3<R>& u) {
#pragma unroll
  for (int k = 0; k < 9; ++k) st<R>(f + (size_t)k * vh + cb, u.m[k]);
}

// ---------------------------------------------------------------------------
// Block numbering.  Workgroups are handed to the 8 XCDs round-robin by
// workgroup id; remapping so that XCD k processes one contiguous range of
// blocks keeps each stencil's neighbours in that XCD's L2.
// ---------------------------------------------------------------------------
constexpr int kXcd = 8;
__device__ __forceinline__ int xcd_block(int b, int nb) {
  int q = nb / kXcd, r = nb % kXcd;
  int x = b % kXcd, slot = b / kXcd;
  return x < r ? x * (q + 1) + slot : r * (q + 1) + (x - r) * q + slot;
}

// ---------------------------------------------------------------------------
// Deterministic reduction in two launches: each block reduces its values
// (wave shuffles, then LDS across the block's waves, fixed order) and writes
// one partial per block with a plain store; a later launch -- a one-block
// finalize kernel, or block 0 of the next kernel -- sums the partials in a
// fixed order.  Kernel boundaries provide the visibility, so no block
// executes an atomic or a device-scope fence, and every run gives the same
// bits.
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) t += sh[i];
  }
  return t;  // valid in thread 0
}

// Write this block's sums of NV values to partials[blk*NV + k].
template <int NT, int NV>
__device__ __forceinline__ void block_partials(const double (&v)[NV], double* partials, int blk) {
  __shared__ double sh[NT / 64];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double t = block_sum<NT>(v[k], sh);
    if (threadIdx.x == 0) partials[(size_t)blk * NV + k] = t;
  }
}

// Sum the partials of nblk blocks (written by an earlier launch) in a fixed
// order; the result is valid in thread 0.  All NT threads must call it.
template <int NT, int NV>
__device__ __forceinline__ void sum_partials(const double* partials, int nblk, double (&out)[NV]) {
  __shared__ double sh[NT / 64];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nblk; i += NT) s += partials[(size_t)i * NV + k];
    out[k] = block_sum<NT>(s, sh);
  }
}

}  // namespace lgt
