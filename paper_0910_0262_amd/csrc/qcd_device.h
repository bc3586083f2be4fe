// Device-side building blocks for the gfx950 Wilson-clover kernels:
// complex arithmetic, spinor / link / clover register types, the
// structure-of-arrays field accessors (FP64, FP32, binary16 + scale), the
// checkerboard geometry, wave64 block reductions and the XCD-aware block
// order.  Everything here is header-only and used by the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qcd {

// ------------------------------------------------------------------ complex
template <typename R>
struct Cx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ Cx<R> cx(R a, R b) { return Cx<R>{a, b}; }
template <typename R>
__device__ __forceinline__ Cx<R> operator+(Cx<R> a, Cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> operator-(Cx<R> a, Cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> operator-(Cx<R> a) { return {-a.re, -a.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> operator*(Cx<R> a, Cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ Cx<R> operator*(R s, Cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> conj(Cx<R> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename R>
__device__ __forceinline__ Cx<R> cmulc(Cx<R> a, Cx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R>
__device__ __forceinline__ Cx<R> ti(Cx<R> a) { return {-a.im, a.re}; }   // i a
template <typename R>
__device__ __forceinline__ Cx<R> tmi(Cx<R> a) { return {a.im, -a.re}; }  // -i a
template <typename R>
__device__ __forceinline__ R norm2(Cx<R> a) { return a.re * a.re + a.im * a.im; }

// Complex multiply-accumulate as four fused multiply-adds, so that the
// product is never rounded on its own and the sum needs no separate add:
// cfma = acc + a b, cfmac = acc + conj(a) b, cfms = acc - a b.
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <typename R>
__device__ __forceinline__ Cx<R> cfma(Cx<R> a, Cx<R> b, Cx<R> acc) {
  acc.re = fmar(a.re, b.re, acc.re);
  acc.re = fmar(-a.im, b.im, acc.re);
  acc.im = fmar(a.re, b.im, acc.im);
  acc.im = fmar(a.im, b.re, acc.im);
  return acc;
}
template <typename R>
__device__ __forceinline__ Cx<R> cfmac(Cx<R> a, Cx<R> b, Cx<R> acc) {
  acc.re = fmar(a.re, b.re, acc.re);
  acc.re = fmar(a.im, b.im, acc.re);
  acc.im = fmar(a.re, b.im, acc.im);
  acc.im = fmar(-a.im, b.re, acc.im);
  return acc;
}
template <typename R>
__device__ __forceinline__ Cx<R> cfms(Cx<R> a, Cx<R> b, Cx<R> acc) {
  acc.re = fmar(-a.re, b.re, acc.re);
  acc.re = fmar(a.im, b.im, acc.re);
  acc.im = fmar(-a.re, b.im, acc.im);
  acc.im = fmar(-a.im, b.re, acc.im);
  return acc;
}
// Leading product of a multiply-add chain.  In FP32 it is an FMA onto +0
// (the product itself, up to the sign of a zero result), so that a binary16
// operand is converted inside a mixed-precision FMA like the rest of the
// chain instead of by an instruction of its own; FP64 keeps the product.
template <typename R>
__device__ __forceinline__ Cx<R> cmul0(Cx<R> a, Cx<R> b) {
  if constexpr (sizeof(R) == 4)
    return cfma(a, b, Cx<R>{R(0), R(0)});
  else
    return a * b;
}
template <typename R>
__device__ __forceinline__ Cx<R> cmulc0(Cx<R> a, Cx<R> b) {
  if constexpr (sizeof(R) == 4)
    return cfmac(a, b, Cx<R>{R(0), R(0)});
  else
    return cmulc(a, b);
}
template <typename R>
__device__ __forceinline__ Cx<R> rmul0(R s, Cx<R> a) {
  if constexpr (sizeof(R) == 4)
    return {fmar(s, a.re, R(0)), fmar(s, a.im, R(0))};
  else
    return s * a;
}

// ------------------------------------------------------------------ register types
template <typename R>
struct Spinor {
  Cx<R> v[4][3];  // [spin][colour]
};
template <typename R>
struct Half {
  Cx<R> h[2][3];
};
template <typename R>
struct Mat {
  Cx<R> m[3][3];  // [row][col]
};

template <typename R>
__device__ __forceinline__ void zero(Spinor<R>& s) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) s.v[a][c] = {R(0), R(0)};
}
template <typename R>
__device__ __forceinline__ void neg_lower(Spinor<R>& s) {
#pragma unroll
  for (int a = 2; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) s.v[a][c] = -s.v[a][c];
}
template <typename R>
__device__ __forceinline__ double site_norm2(const Spinor<R>& s) {
  double n = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) n += double(s.v[a][c].re) * double(s.v[a][c].re) + double(s.v[a][c].im) * double(s.v[a][c].im);
  return n;
}

// U h, colour matrix times the two colour vectors of a half spinor.  FUSED:
// each row as one chain of fused multiply-adds (fewer instructions); the
// unfused form (products, then sums) schedules into fewer registers where a
// kernel is short of them.
template <bool FUSED = true, typename R>
__device__ __forceinline__ void mul_mat(const Mat<R>& u, const Half<R>& in, Half<R>& out) {
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if constexpr (FUSED)
        out.h[k][a] = cfma(u.m[a][2], in.h[k][2], cfma(u.m[a][1], in.h[k][1], cmul0(u.m[a][0], in.h[k][0])));
      else
        out.h[k][a] = u.m[a][0] * in.h[k][0] + u.m[a][1] * in.h[k][1] + u.m[a][2] * in.h[k][2];
    }
}
// U^dag h
template <bool FUSED = true, typename R>
__device__ __forceinline__ void mul_adj(const Mat<R>& u, const Half<R>& in, Half<R>& out) {
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if constexpr (FUSED)
        out.h[k][a] = cfmac(u.m[2][a], in.h[k][2], cfmac(u.m[1][a], in.h[k][1], cmulc0(u.m[0][a], in.h[k][0])));
      else
        out.h[k][a] = cmulc(u.m[0][a], in.h[k][0]) + cmulc(u.m[1][a], in.h[k][1]) + cmulc(u.m[2][a], in.h[k][2]);
    }
}

template <typename R>
__device__ __forceinline__ Mat<R> mm(const Mat<R>& a, const Mat<R>& b) {
  Mat<R> c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) c.m[i][j] = cfma(a.m[i][2], b.m[2][j], cfma(a.m[i][1], b.m[1][j], a.m[i][0] * b.m[0][j]));
  return c;
}
template <typename R>
__device__ __forceinline__ Mat<R> adj(const Mat<R>& a) {
  Mat<R> c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) c.m[i][j] = conj(a.m[j][i]);
  return c;
}
template <typename R>
__device__ __forceinline__ Mat<R> madd(const Mat<R>& a, const Mat<R>& b) {
  Mat<R> c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) c.m[i][j] = a.m[i][j] + b.m[i][j];
  return c;
}
template <typename R>
__device__ __forceinline__ Mat<R> msub(const Mat<R>& a, const Mat<R>& b) {
  Mat<R> c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) c.m[i][j] = a.m[i][j] - b.m[i][j];
  return c;
}
template <typename R>
__device__ __forceinline__ Mat<R> mzero() {
  Mat<R> c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) c.m[i][j] = {R(0), R(0)};
  return c;
}

// ------------------------------------------------------------------ geometry
// Lattice extents and the checkerboard stride of the structure-of-arrays
// fields.  cb = i / 2 for lexicographic site i = x + Lx (y + Ly (z + Lz t)).
struct Geom {
  int X[4];      // Lx, Ly, Lz, Lt
  int Xh;        // Lx / 2
  int V, Vh;
  int stride;    // element stride between components of one field (>= Vh)
  int tb;        // +1 periodic / -1 antiperiodic in time
  double inv_xh, inv_y, inv_z;  // 1 / Xh, 1 / Ly, 1 / Lz (fast division)
};

// n / d and n % d for 0 <= n < 2^31 via the double reciprocal; the quotient
// is off by at most one before the correction step.
__device__ __forceinline__ int fdivmod(int n, int d, double inv, int& r) {
  int q = int(double(n) * inv);
  r = n - q * d;
  if (r < 0) {
    q -= 1;
    r += d;
  } else if (r >= d) {
    q += 1;
    r -= d;
  }
  return q;
}

__device__ __forceinline__ void cb_coords(int cb, int par, const Geom& g, int x[4]) {
  int xh, yy, zz;
  int r = fdivmod(cb, g.Xh, g.inv_xh, xh);
  r = fdivmod(r, g.X[1], g.inv_y, yy);
  x[3] = fdivmod(r, g.X[2], g.inv_z, zz);
  x[1] = yy;
  x[2] = zz;
  x[0] = 2 * xh + ((x[1] + x[2] + x[3] + par) & 1);
}

__device__ __forceinline__ int lex(const int x[4], const Geom& g) {
  return x[0] + g.X[0] * (x[1] + g.X[1] * (x[2] + g.X[2] * x[3]));
}
__device__ __forceinline__ void lex_coords(int i, const Geom& g, int x[4]) {
  x[0] = i % g.X[0];
  int r = i / g.X[0];
  x[1] = r % g.X[1];
  r /= g.X[1];
  x[2] = r % g.X[2];
  x[3] = r / g.X[2];
}
__device__ __forceinline__ int parity_of(const int x[4]) { return (x[0] + x[1] + x[2] + x[3]) & 1; }

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).
// Map hardware block b to a logical block so that XCD k gets one contiguous
// range of logical blocks: neighbouring sites then share an L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, rem = nb & 7;
  const int xcd = b & 7, k = b >> 3;
  return (xcd < rem) ? xcd * (q + 1) + k : rem * (q + 1) + (xcd - rem) * q + k;
}

// ------------------------------------------------------------------ binary16
typedef _Float16 h4_t __attribute__((ext_vector_type(4)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ h8_t as_h8(uint4 w) {
  h8_t h;
  __builtin_memcpy(&h, &w, 16);
  return h;
}
__device__ __forceinline__ uint4 from_h8(h8_t h) {
  uint4 w;
  __builtin_memcpy(&w, &h, 16);
  return w;
}
__device__ __forceinline__ h4_t as_h4(uint2 w) {
  h4_t h;
  __builtin_memcpy(&h, &w, 8);
  return h;
}
__device__ __forceinline__ uint2 from_h4(h4_t h) {
  uint2 w;
  __builtin_memcpy(&w, &h, 8);
  return w;
}
typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ h2_t as_h2(unsigned int w) {
  h2_t h;
  __builtin_memcpy(&h, &w, 4);
  return h;
}
__device__ __forceinline__ unsigned int from_h2(h2_t h) {
  unsigned int w;
  __builtin_memcpy(&w, &h, 4);
  return w;
}

// ------------------------------------------------------------------ field addressing
// Element i of chunk k of a structure-of-arrays field (chunk k starts at
// p + k * stride): the chunk base is the same for the whole grid and i is a
// 32-bit index, so the compiler issues a load with a scalar 64-bit base and a
// 32-bit per-lane byte offset instead of building a 64-bit address per lane
// (fewer vector instructions and registers).  The host keeps every index
// times 16 below 2^32.
template <class T>
__device__ __forceinline__ T* elem(T* p, size_t chunk_off, int i) {
  char* base = (char*)(p + chunk_off);
  return (T*)(base + (unsigned)i * (unsigned)sizeof(T));
}
template <class T>
__device__ __forceinline__ const T* elem(const T* p, size_t chunk_off, int i) {
  const char* base = (const char*)(p + chunk_off);
  return (const T*)(base + (unsigned)i * (unsigned)sizeof(T));
}

// ------------------------------------------------------------------ streaming loads
// Links and clover blocks are read once per kernel: load them nontemporally
// so the caches keep the neighbour spinors, which are read up to 8 times.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef unsigned int nt_u2 __attribute__((ext_vector_type(2)));
typedef unsigned int nt_u4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ double2 ld_stream(const double2* p) {
  const nt_d2 v = __builtin_nontemporal_load((const nt_d2*)p);
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float4 ld_stream(const float4* p) {
  const nt_f4 v = __builtin_nontemporal_load((const nt_f4*)p);
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint2 ld_stream(const uint2* p) {
  const nt_u2 v = __builtin_nontemporal_load((const nt_u2*)p);
  return make_uint2(v.x, v.y);
}
__device__ __forceinline__ uint4 ld_stream(const uint4* p) {
  const nt_u4 v = __builtin_nontemporal_load((const nt_u4*)p);
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ unsigned int ld_stream(const unsigned int* p) { return __builtin_nontemporal_load(p); }

// ------------------------------------------------------------------ spinor fields
// Each field is one checkerboard.  The FP64 and binary16 spinors are stored
// in tiles of 64 elements with the chunks of a tile contiguous: chunk k of
// element i at p[(i / 64 * nchunks + k) * 64 + i % 64] (sp64_at, sph_at), so
// a wavefront's loads of one spinor read one contiguous run (12 KB, 3 KB)
// rather than one run per chunk a field apart; the stride, a multiple of 64,
// only sizes the field.  The FP32 x accumulator is plain structure of
// arrays, chunk k of element i at p[k * stride + i].  The FP64 tile offset
// exceeds 32 bits on large fields, so those accesses take a 64-bit lane
// address.
struct SpF64 {   // 12 chunks of double2 (one complex each), 192 B / site
  double2* p;
  int stride;
};
__device__ __forceinline__ size_t sp64_at(int k, size_t i) { return (((i >> 6) * 12 + k) << 6) + (i & 63); }
// binary16: 16-byte chunk k of element i is element sph_at(i) counted from
// p + 64 k, a 32-bit index (the host keeps 48 i below 2^32); the per-site
// scales are a plain array.
__device__ __forceinline__ int sph_at(int i) { return ((i >> 6) * 3 << 6) + (i & 63); }
struct SpF32 {   // 6 chunks of float4 (two complex each), 96 B / site
  float4* p;
  int stride;
};
struct SpH {     // 3 chunks of 8 x binary16 + one float scale, 52 B / site
  uint4* p;
  float* s;
  int stride;
};

template <typename R>
__device__ __forceinline__ void load(const SpF64& f, int i, Spinor<R>& v) {
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    double2 d = f.p[sp64_at(k, i)];
    v.v[k / 3][k % 3] = {R(d.x), R(d.y)};
  }
}
// Output spinors are written with nontemporal stores: they are not read
// again by the same kernel, and keeping them out of the caches leaves room
// for the neighbour spinors.
template <typename R>
__device__ __forceinline__ void store(const SpF64& f, int i, const Spinor<R>& v) {
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const nt_d2 w = {double(v.v[k / 3][k % 3].re), double(v.v[k / 3][k % 3].im)};
    __builtin_nontemporal_store(w, (nt_d2*)(f.p + sp64_at(k, i)));
  }
}
// Site-local spinor read once per kernel (the k2 site term, the epilogue's y).
template <typename R>
__device__ __forceinline__ void load_once(const SpF64& f, int i, Spinor<R>& v) {
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const double2 d = ld_stream(f.p + sp64_at(k, i));
    v.v[k / 3][k % 3] = {R(d.x), R(d.y)};
  }
}
template <typename R>
__device__ __forceinline__ void load(const SpF32& f, int i, Spinor<R>& v) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    float4 d = *elem(f.p, (size_t)k * f.stride, i);
    v.v[(2 * k) / 3][(2 * k) % 3] = {R(d.x), R(d.y)};
    v.v[(2 * k + 1) / 3][(2 * k + 1) % 3] = {R(d.z), R(d.w)};
  }
}
template <typename R>
__device__ __forceinline__ void store(const SpF32& f, int i, const Spinor<R>& v) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const Cx<R> a = v.v[(2 * k) / 3][(2 * k) % 3], b = v.v[(2 * k + 1) / 3][(2 * k + 1) % 3];
    *elem(f.p, (size_t)k * f.stride, i) = make_float4(float(a.re), float(a.im), float(b.re), float(b.im));
  }
}
// Neighbour loads in the stencil: the components as stored, with the
// per-site scale applied later to the projected half spinor (12 products
// instead of 24).  FP64 fields have no scale.
template <class F>
struct SpinorScale {
  static constexpr bool scaled = false;
};
template <>
struct SpinorScale<SpH> {
  static constexpr bool scaled = true;
};
template <typename R>
__device__ __forceinline__ void load_raw(const SpF64& f, int i, Spinor<R>& v) {
  load(f, i, v);
}
template <typename R>
__device__ __forceinline__ void load_raw(const SpH& f, int i, Spinor<R>& v) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    h8_t h = as_h8(*elem(f.p, (size_t)k * 64, sph_at(i)));
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = 4 * k + j;
      v.v[c / 3][c % 3] = {R(float(h[2 * j])), R(float(h[2 * j + 1]))};
    }
  }
}
__device__ __forceinline__ float scale_of(const SpH& f, int i) { return *elem(f.s, 0, i); }
__device__ __forceinline__ float scale_of(const SpF64&, int) { return 1.0f; }

template <typename R>
__device__ __forceinline__ void load(const SpH& f, int i, Spinor<R>& v) {
  const float s = *elem(f.s, 0, i);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    h8_t h = as_h8(*elem(f.p, (size_t)k * 64, sph_at(i)));
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = 4 * k + j;  // complex component 0..11
      // code * scale as an FMA onto +0: the binary16 code converts inside it
      v.v[c / 3][c % 3] = {R(fmar(float(h[2 * j]), s, 0.f)), R(fmar(float(h[2 * j + 1]), s, 0.f))};
    }
  }
}
// binary16 encoder: scale = max |component| over the 24 reals (float32),
// code = rn_binary16(component * (1 / scale)); an all-zero spinor keeps scale 0.
template <typename R>
__device__ __forceinline__ float encode_site(const Spinor<R>& v, h8_t out[3]) {
  float m = 0.f;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) m = fmaxf(m, fmaxf(fabsf(float(v.v[a][c].re)), fabsf(float(v.v[a][c].im))));
  const float inv = m > 0.f ? 1.0f / m : 0.f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = 4 * k + j;
      out[k][2 * j] = (_Float16)(float(v.v[c / 3][c % 3].re) * inv);
      out[k][2 * j + 1] = (_Float16)(float(v.v[c / 3][c % 3].im) * inv);
    }
  }
  return m;
}
template <typename R>
__device__ __forceinline__ void store(const SpH& f, int i, const Spinor<R>& v) {
  h8_t h[3];
  const float m = encode_site(v, h);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const uint4 w = from_h8(h[k]);
    const nt_u4 q = {w.x, w.y, w.z, w.w};
    __builtin_nontemporal_store(q, (nt_u4*)elem(f.p, (size_t)k * 64, sph_at(i)));
  }
  __builtin_nontemporal_store(m, elem(f.s, 0, i));
}
// binary16 site spinors are small enough to stay cache-resident: plain loads
template <typename R>
__device__ __forceinline__ void load_once(const SpH& f, int i, Spinor<R>& v) {
  load(f, i, v);
}

// ------------------------------------------------------------------ link fields
// Link U_mu(x) for x of parity par and checkerboard index cb.  Chunk k of
// (mu, par) lives at p[((mu * 2 + par) * NC + k) * stride + cb].
template <int NC>  // 9 = full 18-real matrix, 6 = two rows (12 reals), third rebuilt
struct LinkF64 {
  const double2* p;
  int stride;
};
// Two rows as 12 x binary16 (24 B / link): halves 0-7 (row 0, entry 0 of
// row 1) at p[(mu * 2 + par) * stride + cb], halves 8-11 at q[(mu * 2 + par) *
// stride + cb]; q follows the 8 * stride chunks of p in the same allocation.
struct LinkH12 {
  const uint4* p;
  const uint2* q;
  int stride;
};
// All nine entries as 18 x binary16 (36 B / link), for the multi-source
// kernels, whose vector-instruction issue the row rebuild would cost more
// than the 12 extra bytes (shared by all right-hand sides of a site): chunks
// 0 and 1 (8 halves each) at p[((mu * 2 + par) * 2 + k) * stride + cb],
// chunk 2 (the last entry) at q[(mu * 2 + par) * stride + cb]; q follows the
// 16 * stride chunks of p in the same allocation.
struct LinkH18 {
  const uint4* p;
  const unsigned int* q;
  int stride;
};

template <typename R>
__device__ __forceinline__ void reconstruct_row2(Mat<R>& u) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
    u.m[2][j] = conj(cfms(u.m[0][j2], u.m[1][j1], cmul0(u.m[0][j1], u.m[1][j2])));
  }
}
template <typename R, int NC>
__device__ __forceinline__ void load_link(const LinkF64<NC>& f, int mu, int par, int i, Mat<R>& u) {
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    double2 d = ld_stream(elem(f.p, (size_t)((mu * 2 + par) * NC + k) * f.stride, i));
    u.m[k / 3][k % 3] = {R(d.x), R(d.y)};
  }
  if (NC == 6) reconstruct_row2(u);
}
template <typename R>
__device__ __forceinline__ void load_link(const LinkH18& f, int mu, int par, int i, Mat<R>& u) {
  const int d = mu * 2 + par;
  const h8_t a = as_h8(ld_stream(elem(f.p, (size_t)(d * 2) * f.stride, i)));
  const h8_t b = as_h8(ld_stream(elem(f.p, (size_t)(d * 2 + 1) * f.stride, i)));
  const h2_t c = as_h2(ld_stream(elem(f.q, (size_t)d * f.stride, i)));
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    u.m[k / 3][k % 3] = {R(float(a[2 * k])), R(float(a[2 * k + 1]))};
    u.m[(k + 4) / 3][(k + 4) % 3] = {R(float(b[2 * k])), R(float(b[2 * k + 1]))};
  }
  u.m[2][2] = {R(float(c[0])), R(float(c[1]))};
}
template <typename R>
__device__ __forceinline__ void load_link(const LinkH12& f, int mu, int par, int i, Mat<R>& u) {
  const int d = mu * 2 + par;
  const h8_t a = as_h8(ld_stream(elem(f.p, (size_t)d * f.stride, i)));
  const h4_t b = as_h4(ld_stream(elem(f.q, (size_t)d * f.stride, i)));
#pragma unroll
  for (int k = 0; k < 4; ++k) u.m[k / 3][k % 3] = {R(float(a[2 * k])), R(float(a[2 * k + 1]))};
  u.m[1][1] = {R(float(b[0])), R(float(b[1]))};
  u.m[1][2] = {R(float(b[2])), R(float(b[3]))};
  reconstruct_row2(u);
}

// ------------------------------------------------------------------ clover fields
// Two Hermitian 6x6 blocks per site (spins {0,1} and {2,3}, index 3 s + c).
// Packed per block: 6 real diagonal entries then the 15 upper off-diagonal
// entries in row-major order, 36 reals.
struct CloverNone {};
struct CloverF64 {   // 36 chunks of double2 per site: [block][18]
  const double2* p;
  int stride;
};
struct CloverF32 {   // 18 chunks of float4 per site: reals [block * 36 + r]
  const float4* p;
  int stride;
};
struct CloverH {     // 9 chunks of 8 x binary16 + per-block float scale
  const uint4* p;
  const float2* s;
  int stride;
};

__host__ __device__ constexpr int offd(int i, int j) { return i * (11 - i) / 2 + (j - i - 1); }  // i < j

template <typename R>
struct Block {
  R d[6];
  Cx<R> o[15];
};

template <typename R>
__device__ __forceinline__ void load_block(const CloverF64& c, int i, int b, Block<R>& blk) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double2 d = ld_stream(elem(c.p, (size_t)(b * 18 + k) * c.stride, i));
    blk.d[2 * k] = R(d.x);
    blk.d[2 * k + 1] = R(d.y);
  }
#pragma unroll
  for (int k = 0; k < 15; ++k) {
    double2 d = ld_stream(elem(c.p, (size_t)(b * 18 + 3 + k) * c.stride, i));
    blk.o[k] = {R(d.x), R(d.y)};
  }
}
template <typename R>
__device__ __forceinline__ void load_block(const CloverF32& c, int i, int b, Block<R>& blk) {
  float r[36];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    float4 d = ld_stream(elem(c.p, (size_t)(b * 9 + k) * c.stride, i));
    r[4 * k] = d.x;
    r[4 * k + 1] = d.y;
    r[4 * k + 2] = d.z;
    r[4 * k + 3] = d.w;
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) blk.d[k] = R(r[k]);
#pragma unroll
  for (int k = 0; k < 15; ++k) blk.o[k] = {R(r[6 + 2 * k]), R(r[7 + 2 * k])};
}
// binary16 blocks are decoded without their scale; apply_clover multiplies
// the block's product by the scale instead (6 products instead of 36).
template <typename R>
__device__ __forceinline__ void load_block(const CloverH& c, int i, int b, Block<R>& blk) {
  // 72 halves per site = 9 chunks; block b owns halves [36 b, 36 b + 36)
  float r[36];
#pragma unroll
  for (int k = 0; k < 36; ++k) r[k] = 0.f;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int lo = 8 * k, hi = 8 * k + 8;  // half indices of this chunk
    if (hi <= 36 * b || lo >= 36 * b + 36) continue;
    h8_t h = as_h8(ld_stream(elem(c.p, (size_t)k * c.stride, i)));
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int q = lo + j - 36 * b;
      if (q >= 0 && q < 36) r[q] = float(h[j]);
    }
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) blk.d[k] = R(r[k]);
#pragma unroll
  for (int k = 0; k < 15; ++k) blk.o[k] = {R(r[6 + 2 * k]), R(r[7 + 2 * k])};
}
template <class CL>
struct CloverScale {
  static constexpr bool scaled = false;
};
template <>
struct CloverScale<CloverH> {
  static constexpr bool scaled = true;
};
__device__ __forceinline__ float2 block_scales(const CloverH& c, int i) { return *elem(c.s, 0, i); }

// v <- A v for one 6-vector (spins 2b, 2b+1).  FUSED: each row as one chain
// of fused multiply-adds (with binary16 entries the conversion folds into
// them too); the unfused form schedules into fewer registers.
template <bool FUSED = false, typename R>
__device__ __forceinline__ void block_mv(const Block<R>& a, Cx<R> v[6]) {
  Cx<R> out[6];
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    Cx<R> s = FUSED ? rmul0(a.d[r], v[r]) : a.d[r] * v[r];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      if constexpr (FUSED) {
        if (c > r) s = cfma(a.o[offd(r, c)], v[c], s);
        if (c < r) s = cfmac(a.o[offd(c, r)], v[c], s);
      } else {
        if (c > r) s = s + a.o[offd(r, c)] * v[c];
        if (c < r) s = s + cmulc(a.o[offd(c, r)], v[c]);
      }
    }
    out[r] = s;
  }
#pragma unroll
  for (int r = 0; r < 6; ++r) v[r] = out[r];
}

// s <- A s.  FACT: the two chiral halves of the result are multiplied by f0
// (spins 0, 1) and f1 (spins 2, 3), which commutes with the block-diagonal A
// and so costs nothing where the blocks carry a scale of their own.
template <bool FUSED = false, bool FACT = false, typename R, class CL>
__device__ __forceinline__ void apply_clover(const CL& c, int i, Spinor<R>& s, R f0 = R(1), R f1 = R(1)) {
  float2 sc = make_float2(1.f, 1.f);
  if constexpr (CloverScale<CL>::scaled) sc = block_scales(c, i);
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    Block<R> blk;
    load_block(c, i, b, blk);
    Cx<R> v[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = s.v[2 * b + k / 3][k % 3];
    block_mv<FUSED>(blk, v);
    R f = R(b == 0 ? sc.x : sc.y);
    if constexpr (FACT) f = f * (b == 0 ? f0 : f1);
#pragma unroll
    for (int k = 0; k < 6; ++k)
      s.v[2 * b + k / 3][k % 3] = (CloverScale<CL>::scaled || FACT) ? f * v[k] : v[k];
  }
}

// ------------------------------------------------------------------ compact clover blocks
// A chiral block of a clover term built from links has the form
//   1 - [[X3, W], [W^dag, -X3]]     (3x3 blocks over spin 2b, 2b + 1)
// because sigma_mu,nu restricted to a chiral half is traceless in spin and
// F_mu,nu is traceless in colour: X3 is traceless Hermitian and W general.
// Stored per block: 26 reals [d0, d1, x01, x02, x12, W row-major] with
// X3 = [[d0, x01, x02], [x01*, d1, x12], [x02*, x12*, -d0 - d1]], against 36
// for a general Hermitian 6x6 block.
struct CloverF64C {  // 26 chunks of double2 per site: [block * 13 + k]
  const double2* p;
  int stride;
};
struct CloverHC {    // 52 binary16 per site (block b: [26 b, 26 b + 26)): 6 chunks
  const uint4* p;    // of 8 halves, then a chunk of 4 halves at p + 6 stride
  const float2* s;   // per-block scale, max |real|
  int stride;
};
template <typename R>
struct CBlock {
  R d0, d1;
  Cx<R> x01, x02, x12;
  Cx<R> w[3][3];
};
template <typename R>
__device__ __forceinline__ void cblock_from_reals(const R r[26], CBlock<R>& b) {
  b.d0 = r[0];
  b.d1 = r[1];
  b.x01 = {r[2], r[3]};
  b.x02 = {r[4], r[5]};
  b.x12 = {r[6], r[7]};
#pragma unroll
  for (int k = 0; k < 9; ++k) b.w[k / 3][k % 3] = {r[8 + 2 * k], r[9 + 2 * k]};
}
template <typename R>
__device__ __forceinline__ void load_cblock(const CloverF64C& c, int i, int b, CBlock<R>& blk) {
  R r[26];
#pragma unroll
  for (int k = 0; k < 13; ++k) {
    const double2 d = ld_stream(elem(c.p, (size_t)(b * 13 + k) * c.stride, i));
    r[2 * k] = R(d.x);
    r[2 * k + 1] = R(d.y);
  }
  cblock_from_reals(r, blk);
}
// binary16 entries decoded without the block's scale (applied to the vector)
template <typename R>
__device__ __forceinline__ void load_cblock(const CloverHC& c, int i, int b, CBlock<R>& blk) {
  float r[26];
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const int lo = 8 * k, n = k < 6 ? 8 : 4;  // half indices [lo, lo + n) of this chunk
    if (lo + n <= 26 * b || lo >= 26 * b + 26) continue;
    float h[8];
    if (k < 6) {
      const h8_t v = as_h8(ld_stream(elem(c.p, (size_t)k * c.stride, i)));
#pragma unroll
      for (int j = 0; j < 8; ++j) h[j] = float(v[j]);
    } else {
      const h4_t v = as_h4(ld_stream(elem((const uint2*)(c.p + (size_t)6 * c.stride), 0, i)));
#pragma unroll
      for (int j = 0; j < 4; ++j) h[j] = float(v[j]);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int q = lo + j - 26 * b;
      if (j < n && q >= 0 && q < 26) r[q] = h[j];
    }
  }
  R rr[26];
#pragma unroll
  for (int k = 0; k < 26; ++k) rr[k] = R(r[k]);
  cblock_from_reals(rr, blk);
}
template <>
struct CloverScale<CloverHC> {
  static constexpr bool scaled = true;
};
__device__ __forceinline__ float2 block_scales(const CloverHC& c, int i) { return *elem(c.s, 0, i); }

// v <- v - f [[X3, W], [W^dag, -X3]] v for one 6-vector (spins 2b, 2b + 1)
template <typename R>
__device__ __forceinline__ void cblock_mv(const CBlock<R>& a, Cx<R> v[6], R f) {
  Cx<R> u[3], d[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    u[k] = f * v[k];
    d[k] = f * v[3 + k];
  }
  const R d2 = -(a.d0 + a.d1);
  // X3 u + W d and X3 d - W^dag u
  Cx<R> yu[3], yd[3];
  yu[0] = cfma(a.x02, u[2], cfma(a.x01, u[1], a.d0 * u[0]));
  yu[1] = cfma(a.x12, u[2], cfmac(a.x01, u[0], a.d1 * u[1]));
  yu[2] = cfmac(a.x12, u[1], cfmac(a.x02, u[0], d2 * u[2]));
  yd[0] = cfma(a.x02, d[2], cfma(a.x01, d[1], a.d0 * d[0]));
  yd[1] = cfma(a.x12, d[2], cfmac(a.x01, d[0], a.d1 * d[1]));
  yd[2] = cfmac(a.x12, d[1], cfmac(a.x02, d[0], d2 * d[2]));
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      yu[r] = cfma(a.w[r][c], d[c], yu[r]);
      yd[r] = cfms(conj(a.w[c][r]), u[c], yd[r]);
    }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v[k] = v[k] - yu[k];
    v[3 + k] = v[3 + k] + yd[k];
  }
}
template <class CL>
struct CloverCompact {
  static constexpr bool value = false;
};
template <>
struct CloverCompact<CloverF64C> {
  static constexpr bool value = true;
};
template <>
struct CloverCompact<CloverHC> {
  static constexpr bool value = true;
};
// s <- A s with compact blocks (the site term of k2; no FACT form needed)
template <typename R, class CL>
__device__ __forceinline__ void apply_cclover(const CL& c, int i, Spinor<R>& s) {
  float2 sc = make_float2(1.f, 1.f);
  if constexpr (CloverScale<CL>::scaled) sc = block_scales(c, i);
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    CBlock<R> blk;
    load_cblock(c, i, b, blk);
    Cx<R> v[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = s.v[2 * b + k / 3][k % 3];
    cblock_mv(blk, v, R(b == 0 ? sc.x : sc.y));
#pragma unroll
    for (int k = 0; k < 6; ++k) s.v[2 * b + k / 3][k % 3] = v[k];
  }
}

// ------------------------------------------------------------------ spin projection
// Upper two spin components h of (1 + S gamma_mu) psi, S = -1 or +1, in the
// chiral basis; the lower two are a fixed linear map of h (reconstruct()).
template <int MU, int S, typename R>
__device__ __forceinline__ void project(const Spinor<R>& p, Half<R>& h) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const Cx<R> u0 = p.v[0][c], u1 = p.v[1][c], d0 = p.v[2][c], d1 = p.v[3][c];
    if (MU == 0) {
      h.h[0][c] = S < 0 ? u0 + ti(d1) : u0 - ti(d1);
      h.h[1][c] = S < 0 ? u1 + ti(d0) : u1 - ti(d0);
    } else if (MU == 1) {
      h.h[0][c] = S < 0 ? u0 + d1 : u0 - d1;
      h.h[1][c] = S < 0 ? u1 - d0 : u1 + d0;
    } else if (MU == 2) {
      h.h[0][c] = S < 0 ? u0 + ti(d0) : u0 - ti(d0);
      h.h[1][c] = S < 0 ? u1 - ti(d1) : u1 + ti(d1);
    } else {
      h.h[0][c] = S < 0 ? u0 - d0 : u0 + d0;
      h.h[1][c] = S < 0 ? u1 - d1 : u1 + d1;
    }
  }
}
// The same projection with every sum written as a multiply-add onto a unit
// factor `one` that the compiler cannot see is 1 (a literal 1 would be
// simplified back to an add): the two binary16 operands of each sum then
// convert inside one mixed-precision FMA instead of by two conversions and
// an add.  The value is that of the plain sum.
template <typename R, int SG>
__device__ __forceinline__ Cx<R> proj_add(Cx<R> u, Cx<R> d, R one) {  // u + SG d
  const R f = SG > 0 ? one : -one;
  return {fmar(d.re, f, u.re), fmar(d.im, f, u.im)};
}
template <typename R, int SG>
__device__ __forceinline__ Cx<R> proj_addi(Cx<R> u, Cx<R> d, R one) {  // u + SG i d
  const R f = SG > 0 ? one : -one;
  return {fmar(d.im, -f, u.re), fmar(d.re, f, u.im)};
}
template <int MU, int S, typename R>
__device__ __forceinline__ void project(const Spinor<R>& p, Half<R>& h, R one) {
  constexpr int P = S < 0 ? 1 : -1;  // sign of the first lower term
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const Cx<R> u0 = p.v[0][c], u1 = p.v[1][c], d0 = p.v[2][c], d1 = p.v[3][c];
    if (MU == 0) {
      h.h[0][c] = proj_addi<R, P>(u0, d1, one);
      h.h[1][c] = proj_addi<R, P>(u1, d0, one);
    } else if (MU == 1) {
      h.h[0][c] = proj_add<R, P>(u0, d1, one);
      h.h[1][c] = proj_add<R, -P>(u1, d0, one);
    } else if (MU == 2) {
      h.h[0][c] = proj_addi<R, P>(u0, d0, one);
      h.h[1][c] = proj_addi<R, -P>(u1, d1, one);
    } else {
      h.h[0][c] = proj_add<R, -P>(u0, d0, one);
      h.h[1][c] = proj_add<R, -P>(u1, d1, one);
    }
  }
}
// acc += (h, lower(h)) for the projector (1 + S gamma_mu)
template <int MU, int S, typename R>
__device__ __forceinline__ void accumulate(Spinor<R>& a, const Half<R>& h) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const Cx<R> h0 = h.h[0][c], h1 = h.h[1][c];
    a.v[0][c] = a.v[0][c] + h0;
    a.v[1][c] = a.v[1][c] + h1;
    if (MU == 0) {
      a.v[2][c] = a.v[2][c] + (S < 0 ? tmi(h1) : ti(h1));
      a.v[3][c] = a.v[3][c] + (S < 0 ? tmi(h0) : ti(h0));
    } else if (MU == 1) {
      a.v[2][c] = a.v[2][c] + (S < 0 ? -h1 : h1);
      a.v[3][c] = a.v[3][c] + (S < 0 ? h0 : -h0);
    } else if (MU == 2) {
      a.v[2][c] = a.v[2][c] + (S < 0 ? tmi(h0) : ti(h0));
      a.v[3][c] = a.v[3][c] + (S < 0 ? ti(h1) : tmi(h1));
    } else {
      a.v[2][c] = a.v[2][c] + (S < 0 ? -h0 : h0);
      a.v[3][c] = a.v[3][c] + (S < 0 ? -h1 : h1);
    }
  }
}
// a += f * (the same reconstruction of h): the scale of the projected half
// spinor (a binary16 field's site scale, the antiperiodic-time sign) rides on
// the accumulating multiply-adds instead of costing 12 products of its own.
template <typename R>
__device__ __forceinline__ Cx<R> axpy(Cx<R> a, R f, Cx<R> h) {  // a + f h
  return {fmar(f, h.re, a.re), fmar(f, h.im, a.im)};
}
template <typename R>
__device__ __forceinline__ Cx<R> axpy_i(Cx<R> a, R f, Cx<R> h) {  // a + i f h
  return {fmar(-f, h.im, a.re), fmar(f, h.re, a.im)};
}
// fu multiplies the upper two spins of the reconstruction, fl the lower two.
template <int MU, int S, typename R>
__device__ __forceinline__ void accumulate(Spinor<R>& a, const Half<R>& h, R fu, R fl) {
  const R g = S < 0 ? -fl : fl;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const Cx<R> h0 = h.h[0][c], h1 = h.h[1][c];
    a.v[0][c] = axpy(a.v[0][c], fu, h0);
    a.v[1][c] = axpy(a.v[1][c], fu, h1);
    if (MU == 0) {  // S < 0: -i h1, -i h0
      a.v[2][c] = axpy_i(a.v[2][c], g, h1);
      a.v[3][c] = axpy_i(a.v[3][c], g, h0);
    } else if (MU == 1) {  // S < 0: -h1, +h0
      a.v[2][c] = axpy(a.v[2][c], g, h1);
      a.v[3][c] = axpy(a.v[3][c], -g, h0);
    } else if (MU == 2) {  // S < 0: -i h0, +i h1
      a.v[2][c] = axpy_i(a.v[2][c], g, h0);
      a.v[3][c] = axpy_i(a.v[3][c], -g, h1);
    } else {  // S < 0: -h0, -h1
      a.v[2][c] = axpy(a.v[2][c], g, h0);
      a.v[3][c] = axpy(a.v[3][c], g, h1);
    }
  }
}

// ------------------------------------------------------------------ reductions
// Sum of v over the workgroup (wave64 shuffles, then LDS); the result is
// written by thread 0 to partial[slot].  Every thread of the block must call it.
__device__ __forceinline__ void block_sum_store(double v, double* partial, int slot) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __shared__ double red[16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int k = 0; k < nw; ++k) s += red[k];
    partial[slot] = s;
  }
}

// Segmented version for 1 << lg (<= 16) interleaved right-hand sides: thread
// t contributes to right-hand side t & ((1 << lg) - 1); the workgroup's sum
// for right-hand side r goes to partial[r * nblk + slot].  lg = 0 gives the
// same sums, in the same order, as block_sum_store.
__device__ __forceinline__ void block_sum_store_seg(double v, double* partial, int slot, int nblk, int lg) {
  const int nr = 1 << lg;
  for (int off = 32; off >= nr; off >>= 1) v += __shfl_down(v, off, 64);
  __shared__ double red[16][16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane < nr) red[w][lane] = v;
  __syncthreads();
  if ((int)threadIdx.x < nr) {
    double s = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int k = 0; k < nw; ++k) s += red[k][threadIdx.x];
    partial[(size_t)threadIdx.x * nblk + slot] = s;
  }
}

// Fixed-order sum of n partials by one workgroup; the result is returned to
// every thread.  Deterministic for a given n and blockDim.
__device__ __forceinline__ double block_sum_partials(const double* p, int n) {
  double s = 0.0;
  // Each thread adds p[t], p[t + B], p[t + 2B], ... in that order (B =
  // blockDim.x).  Groups of eight are loaded before any of them is added, so
  // eight loads are in flight rather than one; a load past the end reads the
  // last partial instead (it is in bounds) and is not added.
  const int step = blockDim.x;
  for (int k0 = threadIdx.x; k0 < n; k0 += 8 * step) {
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = p[min(k0 + j * step, n - 1)];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (k0 + j * step < n) s += v[j];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  __shared__ double red[16];
  __shared__ double total;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int k = 0; k < nw; ++k) t += red[k];
    total = t;
  }
  __syncthreads();
  return total;
}

}  // namespace qcd
