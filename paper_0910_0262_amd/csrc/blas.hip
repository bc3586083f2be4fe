// Layout conversion, vector updates and reductions for the solver.
//
// Packing kernels move caller arrays (site-major complex128) into the
// per-checkerboard structure-of-arrays fields and back.  The CG kernels keep
// every scalar of the recurrence on the device (CgState): the finalisation
// kernels sum the per-workgroup partials in a fixed order (deterministic) and
// derive alpha, beta and the stopping / reliable-update decisions.
#include <type_traits>

#include "qcd_internal.h"

namespace qcd {

// ------------------------------------------------------------------ spinor packing
__global__ void pack_spinor_full_k(Geom g, const double2* __restrict__ user, SpF64 e, SpF64 o) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  int x[4];
  lex_coords(i, g, x);
  const SpF64 f = parity_of(x) ? o : e;
  const int cb = i >> 1;
  double2 v[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = user[(size_t)i * 12 + k];
#pragma unroll
  for (int k = 0; k < 12; ++k) f.p[sp64_at(k, cb)] = v[k];
}
__global__ void unpack_spinor_full_k(Geom g, SpF64 e, SpF64 o, double2* __restrict__ user) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  int x[4];
  lex_coords(i, g, x);
  const SpF64 f = parity_of(x) ? o : e;
  const int cb = i >> 1;
  double2 v[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = f.p[sp64_at(k, cb)];
#pragma unroll
  for (int k = 0; k < 12; ++k) user[(size_t)i * 12 + k] = v[k];
}
__global__ void pack_spinor_cb_k(int n, const double2* __restrict__ user, SpF64 f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double2 v[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = user[(size_t)i * 12 + k];
#pragma unroll
  for (int k = 0; k < 12; ++k) f.p[sp64_at(k, i)] = v[k];
}
__global__ void unpack_spinor_cb_k(int n, SpF64 f, double2* __restrict__ user) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double2 v[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = f.p[sp64_at(k, i)];
#pragma unroll
  for (int k = 0; k < 12; ++k) user[(size_t)i * 12 + k] = v[k];
}

// n right-hand sides [n][V][12] -> interleaved fields, element (cb << lg) | r;
// one thread per (site, rhs slot), slots r >= n are zero.
__global__ void pack_spinor_multi_k(Geom g, int lg, int n, const double2* __restrict__ user, SpF64 e, SpF64 o) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ((size_t)g.V << lg)) return;
  const int r = (int)(t & ((1u << lg) - 1)), i = (int)(t >> lg);
  int x[4];
  lex_coords(i, g, x);
  const SpF64 f = parity_of(x) ? o : e;
  const size_t v = ((size_t)(i >> 1) << lg) | r;
  double2 w[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) w[k] = r < n ? user[((size_t)r * g.V + i) * 12 + k] : make_double2(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < 12; ++k) f.p[sp64_at(k, v)] = w[k];
}
__global__ void unpack_spinor_multi_k(Geom g, int lg, int n, SpF64 e, SpF64 o, double2* __restrict__ user) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ((size_t)g.V << lg)) return;
  const int r = (int)(t & ((1u << lg) - 1)), i = (int)(t >> lg);
  if (r >= n) return;
  int x[4];
  lex_coords(i, g, x);
  const SpF64 f = parity_of(x) ? o : e;
  const size_t v = ((size_t)(i >> 1) << lg) | r;
  double2 w[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) w[k] = f.p[sp64_at(k, v)];
#pragma unroll
  for (int k = 0; k < 12; ++k) user[((size_t)r * g.V + i) * 12 + k] = w[k];
}
hipError_t launch_pack_spinor_multi(const Geom& g, int lg, int n, const double2* user, SpF64 e, SpF64 o,
                                    hipStream_t s) {
  const size_t nt = (size_t)g.V << lg;
  hipLaunchKernelGGL(pack_spinor_multi_k, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, g, lg, n, user, e, o);
  return hipGetLastError();
}
hipError_t launch_unpack_spinor_multi(const Geom& g, int lg, int n, SpF64 e, SpF64 o, double2* user, hipStream_t s) {
  const size_t nt = (size_t)g.V << lg;
  hipLaunchKernelGGL(unpack_spinor_multi_k, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, g, lg, n, e, o,
                     user);
  return hipGetLastError();
}

hipError_t launch_pack_spinor_full(const Geom& g, const double2* user, SpF64 e, SpF64 o, hipStream_t s) {
  hipLaunchKernelGGL(pack_spinor_full_k, dim3(blocks_for(g.V, 256)), dim3(256), 0, s, g, user, e, o);
  return hipGetLastError();
}
hipError_t launch_unpack_spinor_full(const Geom& g, SpF64 e, SpF64 o, double2* user, hipStream_t s) {
  hipLaunchKernelGGL(unpack_spinor_full_k, dim3(blocks_for(g.V, 256)), dim3(256), 0, s, g, e, o, user);
  return hipGetLastError();
}
hipError_t launch_pack_spinor_cb(const Geom& g, const double2* user, SpF64 f, hipStream_t s) {
  hipLaunchKernelGGL(pack_spinor_cb_k, dim3(blocks_for(g.Vh, 256)), dim3(256), 0, s, g.Vh, user, f);
  return hipGetLastError();
}
hipError_t launch_unpack_spinor_cb(const Geom& g, SpF64 f, double2* user, hipStream_t s) {
  hipLaunchKernelGGL(unpack_spinor_cb_k, dim3(blocks_for(g.Vh, 256)), dim3(256), 0, s, g.Vh, f, user);
  return hipGetLastError();
}

// ------------------------------------------------------------------ gauge packing
// user: complex128 [V][4][3][3]; u18: double2 [(mu*2 + par)*9 + k][stride]
__global__ void pack_gauge_k(Geom g, const double2* __restrict__ user, double2* __restrict__ u18) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * g.V) return;
  const int i = t >> 2, mu = t & 3;
  int x[4];
  lex_coords(i, g, x);
  const int par = parity_of(x), cb = i >> 1;
  double2* dst = u18 + (size_t)((mu * 2 + par) * 9) * g.stride + cb;
#pragma unroll
  for (int k = 0; k < 9; ++k) dst[(size_t)k * g.stride] = user[(size_t)t * 9 + k];
}
__global__ void unpack_gauge_k(Geom g, const double2* __restrict__ u18, double2* __restrict__ user) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * g.V) return;
  const int i = t >> 2, mu = t & 3;
  int x[4];
  lex_coords(i, g, x);
  const int par = parity_of(x), cb = i >> 1;
  const double2* src = u18 + (size_t)((mu * 2 + par) * 9) * g.stride + cb;
#pragma unroll
  for (int k = 0; k < 9; ++k) user[(size_t)t * 9 + k] = src[(size_t)k * g.stride];
}
// FP64 12-real (first two rows) and binary16 12-real copies of the links.
// binary16 entries are rounded float64 -> float32 -> binary16, both to nearest even.
__global__ void derive_links_k(Geom g, const double2* __restrict__ u18, double2* __restrict__ u12,
                               uint2* __restrict__ uh, uint4* __restrict__ uh18) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 8 * g.Vh) return;
  const int q = t / g.Vh, cb = t - q * g.Vh;  // q = mu * 2 + par
  const double2* src = u18 + (size_t)(q * 9) * g.stride + cb;
  double2 r[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) r[k] = src[(size_t)k * g.stride];
#pragma unroll
  for (int k = 0; k < 6; ++k) u12[(size_t)(q * 6 + k) * g.stride + cb] = r[k];
  {  // rows 0, 1: halves 0-7 in a 16-byte chunk, 8-11 in an 8-byte one
    h8_t a;
    h4_t b;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[2 * k] = (_Float16)(float)r[k].x;
      a[2 * k + 1] = (_Float16)(float)r[k].y;
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      b[2 * k] = (_Float16)(float)r[4 + k].x;
      b[2 * k + 1] = (_Float16)(float)r[4 + k].y;
    }
    uint4* p4 = (uint4*)uh;
    p4[(size_t)q * g.stride + cb] = from_h8(a);
    ((uint2*)(p4 + (size_t)8 * g.stride))[(size_t)q * g.stride + cb] = from_h4(b);
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    h8_t h;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      h[2 * j] = (_Float16)(float)r[4 * k + j].x;
      h[2 * j + 1] = (_Float16)(float)r[4 * k + j].y;
    }
    uh18[(size_t)(q * 2 + k) * g.stride + cb] = from_h8(h);
  }
  h2_t h;
  h[0] = (_Float16)(float)r[8].x;
  h[1] = (_Float16)(float)r[8].y;
  ((unsigned int*)(uh18 + (size_t)16 * g.stride))[(size_t)q * g.stride + cb] = from_h2(h);
}

hipError_t launch_pack_gauge(const Geom& g, const double2* user, double2* u18, hipStream_t s) {
  hipLaunchKernelGGL(pack_gauge_k, dim3(blocks_for(4 * g.V, 256)), dim3(256), 0, s, g, user, u18);
  return hipGetLastError();
}
hipError_t launch_unpack_gauge(const Geom& g, const double2* u18, double2* user, hipStream_t s) {
  hipLaunchKernelGGL(unpack_gauge_k, dim3(blocks_for(4 * g.V, 256)), dim3(256), 0, s, g, u18, user);
  return hipGetLastError();
}
hipError_t launch_derive_links(const Geom& g, const double2* u18, double2* u12, uint2* uh, uint4* uh18,
                               hipStream_t s) {
  hipLaunchKernelGGL(derive_links_k, dim3(blocks_for(8 * g.Vh, 256)), dim3(256), 0, s, g, u18, u12, uh, uh18);
  return hipGetLastError();
}

// ------------------------------------------------------------------ clover packing
// user [V][36] double2 (= [V][2][36] doubles) <-> clov [(par*36 + k)][stride]
__global__ void pack_clover_k(Geom g, const double2* __restrict__ user, double2* __restrict__ clov) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  int x[4];
  lex_coords(i, g, x);
  const int par = parity_of(x), cb = i >> 1;
#pragma unroll 4
  for (int k = 0; k < 36; ++k) clov[(size_t)(par * 36 + k) * g.stride + cb] = user[(size_t)i * 36 + k];
}
__global__ void unpack_clover_full_k(Geom g, const double2* __restrict__ clov, double2* __restrict__ user) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  int x[4];
  lex_coords(i, g, x);
  const int par = parity_of(x), cb = i >> 1;
#pragma unroll 4
  for (int k = 0; k < 36; ++k) user[(size_t)i * 36 + k] = clov[(size_t)(par * 36 + k) * g.stride + cb];
}
__global__ void unpack_clover_cb_k(Geom g, const double2* __restrict__ clov, double2* __restrict__ user) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.Vh) return;
#pragma unroll 4
  for (int k = 0; k < 36; ++k) user[(size_t)i * 36 + k] = clov[(size_t)k * g.stride + i];
}
hipError_t launch_pack_clover(const Geom& g, const double2* user, double2* clov, hipStream_t s) {
  hipLaunchKernelGGL(pack_clover_k, dim3(blocks_for(g.V, 256)), dim3(256), 0, s, g, user, clov);
  return hipGetLastError();
}
hipError_t launch_unpack_clover(const Geom& g, const double2* clov, double2* user, int n_par, int par0,
                                hipStream_t s) {
  if (n_par == 2) {
    hipLaunchKernelGGL(unpack_clover_full_k, dim3(blocks_for(g.V, 256)), dim3(256), 0, s, g, clov, user);
  } else {
    hipLaunchKernelGGL(unpack_clover_cb_k, dim3(blocks_for(g.Vh, 256)), dim3(256), 0, s, g,
                       clov + (size_t)par0 * 36 * g.stride, user);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ reductions
// gv: Vh and stride of all interleaved right-hand sides together.
template <class F>
__global__ void __launch_bounds__(256) norm2_k(Geom gv, int lg, F x, double* partial) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int i = blk * blockDim.x + threadIdx.x;
  double n = 0.0;
  if (i < gv.Vh) {
    Spinor<double> v;
    load(x, i, v);
    n = site_norm2(v);
  }
  block_sum_store_seg(n, partial, blk, gridDim.x, lg);
}
__global__ void __launch_bounds__(256) dot_re_k(Geom gv, int lg, SpF64 a, SpF64 b, double* partial) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int i = blk * blockDim.x + threadIdx.x;
  double n = 0.0;
  if (i < gv.Vh) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const double2 u = a.p[sp64_at(k, i)], v = b.p[sp64_at(k, i)];
      n += u.x * v.x + u.y * v.y;
    }
  }
  block_sum_store_seg(n, partial, blk, gridDim.x, lg);
}
hipError_t launch_norm2(const Geom& gv, int lg, SpRef x, double* partial, int block, hipStream_t s) {
  const int nb = blocks_for(gv.Vh, block);
  if (x.kind == SP_F64)
    hipLaunchKernelGGL(norm2_k<SpF64>, dim3(nb), dim3(block), 0, s, gv, lg, SpF64{(double2*)x.p, gv.stride}, partial);
  else if (x.kind == SP_F32)
    hipLaunchKernelGGL(norm2_k<SpF32>, dim3(nb), dim3(block), 0, s, gv, lg, SpF32{(float4*)x.p, gv.stride}, partial);
  else if (x.kind == SP_H)
    hipLaunchKernelGGL(norm2_k<SpH>, dim3(nb), dim3(block), 0, s, gv, lg, SpH{(uint4*)x.p, x.s, gv.stride}, partial);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
hipError_t launch_dot_re(const Geom& gv, int lg, SpF64 a, SpF64 b, double* partial, int block, hipStream_t s) {
  hipLaunchKernelGGL(dot_re_k, dim3(blocks_for(gv.Vh, block)), dim3(block), 0, s, gv, lg, a, b, partial);
  return hipGetLastError();
}

// ------------------------------------------------------------------ CG scalar kernels (one workgroup)
// Each finalisation kernel that ends an iteration posts a copy of the state
// to mailbox[post_seq % ring] (host-mapped memory the host reads once the
// iteration's event has completed) and advances post_seq; the host counts
// the posting launches it issues, so it knows the slot of each without
// passing it as an argument (the same captured graph serves every iteration).
// Workgroup r of a launch handles right-hand side r: its state st[r], its
// partials partial[r * n ...], its mailbox ring mbox[r * ring ...].
__global__ void fin_scalar_k(CgState* st, const double* partial, int n) {
  st += blockIdx.x;
  partial += (size_t)blockIdx.x * n;
  const double s = block_sum_partials(partial, n);
  if (threadIdx.x == 0) st->scalar = s;
}
__global__ void fin_init_k(CgState* st, const double* partial, int n, double tol, double delta, int max_iter,
                           int mixed, CgState* mbox, int ring) {
  st += blockIdx.x;
  partial += (size_t)blockIdx.x * n;
  mbox += (size_t)blockIdx.x * ring;
  const double rr = block_sum_partials(partial, n);
  if (threadIdx.x != 0) return;
  st->rr = rr;
  st->rr_hi = rr;
  st->qq = 0.0;
  st->alpha = 0.0;
  st->beta = 0.0;
  st->stop2 = tol * tol * rr;
  st->maxrr = rr;
  st->delta2 = delta * delta;
  st->scalar = rr;
  st->iter = 0;
  st->max_iter = max_iter;
  st->nan = finite(rr) ? 0 : 1;
  st->done = (st->nan || rr <= st->stop2) ? 1 : 0;
  st->halt = st->done;
  st->need_ru = 0;
  st->do_x = 0;
  st->do_p = 0;
  st->mixed = mixed;
  st->ru_count = 0;
  for (int m = 0; m < 4; ++m) st->ah[m] = 0.0;
  post(st, mbox, ring);
}
__global__ void fin_alpha_k(CgState* st, const double* partial, int n) {
  st += blockIdx.x;
  partial += (size_t)blockIdx.x * n;
  if (st->halt) return;
  const double qq = block_sum_partials(partial, n);
  if (threadIdx.x == 0) state_alpha(st, qq);
}
__global__ void fin_beta_k(CgState* st, const double* partial, int n, CgState* mbox, int ring) {
  st += blockIdx.x;
  partial += (size_t)blockIdx.x * n;
  mbox += (size_t)blockIdx.x * ring;
  if (st->halt) {
    if (threadIdx.x == 0) state_halted(st, mbox, ring);
    return;
  }
  const double rr_new = block_sum_partials(partial, n);
  if (threadIdx.x == 0) state_beta(st, rr_new, mbox, ring);
}
// After an FP64 residual recomputation r = rhs - A x (partials of |r|^2):
//   restart = 0 (reliable update): r replaces the recurrence residual, p is kept;
//   restart = 1 (CG restart): beta = 0, so the following p update sets p = r.
// The newest nclear alphas of the history were already taken into x (the
// reliable update folded the unfinished cycle's directions in): they are
// zeroed, so the end of the cycle does not add those directions again.
__global__ void fin_ru_k(CgState* st, const double* partial, int n, int restart, int nclear, CgState* mbox,
                         int ring) {
  st += blockIdx.x;
  partial += (size_t)blockIdx.x * n;
  mbox += (size_t)blockIdx.x * ring;
  const double rr = block_sum_partials(partial, n);
  if (threadIdx.x != 0) return;
  for (int m = 0; m < nclear && m < 4; ++m) st->ah[m] = 0.0;
  st->rr_hi = rr;
  st->ru_count += 1;
  st->need_ru = 0;
  st->do_x = 0;
  if (!finite(rr)) {
    st->nan = 1;
    st->done = 1;
    st->halt = 1;
    st->do_p = 0;
    post(st, mbox, ring);
    return;
  }
  if (restart) st->beta = 0.0;
  st->rr = rr;
  st->maxrr = rr;
  st->done = (rr <= st->stop2 || st->iter >= st->max_iter) ? 1 : 0;
  st->halt = st->done;
  st->do_p = !st->done;
  post(st, mbox, ring);
}

// Span sums of many partials: workgroup (f, r) sums partial[r * n + f * kFoldSpan ...]
// (at most kFoldSpan of them) in block_sum_partials' fixed order into out[r * nf + f].
__global__ void __launch_bounds__(256) fold_partials_k(const double* partial, int n, double* out, int nf) {
  const int f = blockIdx.x, r = blockIdx.y;
  const int m = min(kFoldSpan, n - f * kFoldSpan);
  const double s = block_sum_partials(partial + (size_t)r * n + (size_t)f * kFoldSpan, m);
  if (threadIdx.x == 0) out[(size_t)r * nf + f] = s;
}

#define FIN_LAUNCH(kernel, ...)                                                                   \
  if (n >= kFoldMin) {                                                                            \
    const int nf = blocks_for(n, kFoldSpan);                                                      \
    hipLaunchKernelGGL(fold_partials_k, dim3(nf, nr), dim3(256), 0, s, partial, n, fold, nf);     \
    const hipError_t e = hipGetLastError();                                                       \
    if (e != hipSuccess) return e;                                                                \
    partial = fold;                                                                               \
    n = nf;                                                                                       \
  }                                                                                               \
  hipLaunchKernelGGL(kernel, dim3(nr), dim3(1024), 0, s, __VA_ARGS__);                             \
  return hipGetLastError();

hipError_t launch_fin_scalar(CgState* st, const double* partial, int n, int nr, double* fold, hipStream_t s) {
  FIN_LAUNCH(fin_scalar_k, st, partial, n)
}
hipError_t launch_fin_init(CgState* st, const double* partial, int n, int nr, double* fold, double tol, double delta,
                           int max_iter, int mixed, CgState* mbox, int ring, hipStream_t s) {
  FIN_LAUNCH(fin_init_k, st, partial, n, tol, delta, max_iter, mixed, mbox, ring)
}
hipError_t launch_fin_alpha(CgState* st, const double* partial, int n, int nr, double* fold, hipStream_t s) {
  FIN_LAUNCH(fin_alpha_k, st, partial, n)
}
hipError_t launch_fin_beta(CgState* st, const double* partial, int n, int nr, double* fold, CgState* mbox, int ring,
                           hipStream_t s) {
  FIN_LAUNCH(fin_beta_k, st, partial, n, mbox, ring)
}
hipError_t launch_fin_ru(CgState* st, const double* partial, int n, int nr, double* fold, int restart, int nclear,
                         CgState* mbox, int ring, hipStream_t s) {
  FIN_LAUNCH(fin_ru_k, st, partial, n, restart, nclear, mbox, ring)
}

// ------------------------------------------------------------------ CG vector updates
// The solution takes each search direction a few iterations late: over a
// cycle of n iterations (n = 1 .. 4) the directions p_0 .. p_{n-1} live in
// buffers of their own, and x += alpha_0 p_0 + ... + alpha_{n-1} p_{n-1} is
// done once, at the end of the cycle, instead of reading and writing x every
// iteration.  Iteration j of the cycle (its direction p_j in `pc`, the older
// ones p_{j-1} .. p_0 in `old`, newest first) sets p_{j+1} = r + beta p_j in
// `pout`; x takes sum_{m <= j} ah[m] p_{j-m} at the end of the cycle (`last`)
// or when the recurrence stops at this iteration (do_p == 0), so every
// direction reaches x once.  ah[] is the state's alpha history, newest first.
// Element i belongs to right-hand side i & ((1 << lg) - 1) and uses its state.
template <class Sp>
struct Older {
  Sp p[3];
};

template <int NOLD>
__global__ void __launch_bounds__(256) xp_update_f64_k(Geom g, int lg, const CgState* st, SpF64 x, SpF64 pc,
                                                       Older<SpF64> old, SpF64 pout, SpF64 r, int last) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  st += i & ((1 << lg) - 1);
  if (!st->do_x) return;
  if (i >= g.Vh) return;
  const double be = st->beta;
  const bool dp = st->do_p;
  const bool dx = last || !dp;
  double a[NOLD + 1];
#pragma unroll
  for (int m = 0; m <= NOLD; ++m) a[m] = st->ah[m];
  // six components at a time, every load of them issued before their stores
  // (the compiler cannot tell the fields apart, so a store would hold back
  // the loads after it: one memory round trip per component instead of two
  // per site, which small lattices cannot hide)
#pragma unroll
  for (int hh = 0; hh < 2; ++hh) {
    double2 pv[6], rv[6], xv[6], acc[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) pv[k] = pc.p[sp64_at(6 * hh + k, i)];
    if (dp) {
#pragma unroll
      for (int k = 0; k < 6; ++k) rv[k] = r.p[sp64_at(6 * hh + k, i)];
    }
    if (dx) {
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        xv[k] = x.p[sp64_at(6 * hh + k, i)];
        acc[k] = make_double2(a[0] * pv[k].x, a[0] * pv[k].y);
      }
#pragma unroll
      for (int m = 1; m <= NOLD; ++m)
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const double2 q = old.p[m - 1].p[sp64_at(6 * hh + k, i)];
          acc[k].x += a[m] * q.x;
          acc[k].y += a[m] * q.y;
        }
#pragma unroll
      for (int k = 0; k < 6; ++k) x.p[sp64_at(6 * hh + k, i)] = make_double2(xv[k].x + acc[k].x, xv[k].y + acc[k].y);
    }
    if (dp) {
#pragma unroll
      for (int k = 0; k < 6; ++k)
        pout.p[sp64_at(6 * hh + k, i)] = make_double2(rv[k].x + be * pv[k].x, rv[k].y + be * pv[k].y);
    }
  }
}
// CG restart (beta is zero after one): p = r where the recurrence continues.
__global__ void __launch_bounds__(256) p_restart_f64_k(Geom g, int lg, const CgState* st, SpF64 p, SpF64 r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  st += i & ((1 << lg) - 1);
  if (!st->do_p) return;
  if (i >= g.Vh) return;
  Spinor<double> v;
  load(r, i, v);
  store(p, i, v);
}
// mixed: the same cycle with x in FP32 and the directions in binary16
// (re-encoded per site when written).
template <int NOLD>
__global__ void __launch_bounds__(256) xp_update_h_k(Geom g, int lg, const CgState* st, SpF32 x, SpH pc,
                                                     Older<SpH> old, SpH pout, SpH r, int last) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  st += i & ((1 << lg) - 1);
  if (!st->do_x) return;
  if (i >= g.Vh) return;
  const float be = float(st->beta);
  const bool dp = st->do_p;
  Spinor<float> pv;
  load(pc, i, pv);
  if (last || !dp) {
    Spinor<float> acc, xv;
    const float a0 = float(st->ah[0]);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc.v[s][c] = a0 * pv.v[s][c];
#pragma unroll
    for (int m = 1; m <= NOLD; ++m) {
      const float am = float(st->ah[m]);
      Spinor<float> q;
      load(old.p[m - 1], i, q);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc.v[s][c] = acc.v[s][c] + am * q.v[s][c];
    }
    load(x, i, xv);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) xv.v[s][c] = xv.v[s][c] + acc.v[s][c];
    store(x, i, xv);
  }
  if (dp) {
    Spinor<float> rv;
    load(r, i, rv);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) rv.v[s][c] = rv.v[s][c] + be * pv.v[s][c];
    store(pout, i, rv);
  }
}
// Reliable update: x_hi += x_lo + the directions of the unfinished cycle
// (pend.p[m] = p_{q-1-m} with weight ah[m], m < NQ, for right-hand sides whose
// last iteration ran); x_lo = 0.  The sum is taken in FP64.
template <int NQ>
__global__ void __launch_bounds__(256) ru_accum_k(Geom g, int lg, const CgState* st, SpF64 xhi, SpF32 xlo,
                                                  Older<SpH> pend) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.Vh) return;
  st += i & ((1 << lg) - 1);
  Spinor<double> a, b;
  load(xhi, i, a);
  load(xlo, i, b);
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) a.v[s][c] = a.v[s][c] + b.v[s][c];
  if (NQ > 0 && st->do_x) {
#pragma unroll
    for (int m = 0; m < NQ; ++m) {
      const double am = st->ah[m];
      Spinor<float> q;
      load(pend.p[m], i, q);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const Cx<float> v = q.v[s][c];
          a.v[s][c] = a.v[s][c] + am * Cx<double>{double(v.re), double(v.im)};
        }
    }
  }
  store(xhi, i, a);
  Spinor<float> z;
  zero(z);
  store(xlo, i, z);
}

namespace {
template <class Sp>
Older<Sp> older_of(const Sp* p, int j) {
  Older<Sp> o{};
  for (int m = 1; m <= j; ++m) o.p[m - 1] = p[j - m];
  return o;
}
}  // namespace

hipError_t launch_xp_update_f64(const Geom& gv, int lg, const CgState* st, SpF64 x, const SpF64* p, int j, int n,
                                SpF64 r, int block, hipStream_t s) {
  if (n < 1 || n > 4 || j < 0 || j >= n) return hipErrorInvalidValue;
  const dim3 grid(blocks_for(gv.Vh, block));
  const Older<SpF64> o = older_of(p, j);
  const SpF64 pout = p[(j + 1) % n];
  const int last = j == n - 1;
  switch (j) {
    case 0: hipLaunchKernelGGL(xp_update_f64_k<0>, grid, dim3(block), 0, s, gv, lg, st, x, p[j], o, pout, r, last); break;
    case 1: hipLaunchKernelGGL(xp_update_f64_k<1>, grid, dim3(block), 0, s, gv, lg, st, x, p[j], o, pout, r, last); break;
    case 2: hipLaunchKernelGGL(xp_update_f64_k<2>, grid, dim3(block), 0, s, gv, lg, st, x, p[j], o, pout, r, last); break;
    default: hipLaunchKernelGGL(xp_update_f64_k<3>, grid, dim3(block), 0, s, gv, lg, st, x, p[j], o, pout, r, last); break;
  }
  return hipGetLastError();
}
hipError_t launch_p_restart_f64(const Geom& gv, int lg, const CgState* st, SpF64 p, SpF64 r, int block,
                                hipStream_t s) {
  hipLaunchKernelGGL(p_restart_f64_k, dim3(blocks_for(gv.Vh, block)), dim3(block), 0, s, gv, lg, st, p, r);
  return hipGetLastError();
}
hipError_t launch_xp_update_h(const Geom& gv, int lg, const CgState* st, SpF32 x, const SpH* p, int j, int n, SpH r,
                              int block, hipStream_t s) {
  if (n < 1 || n > 4 || j < 0 || j >= n) return hipErrorInvalidValue;
  const dim3 grid(blocks_for(gv.Vh, block));
  const Older<SpH> o = older_of(p, j);
  const SpH pout = p[(j + 1) % n];
  const int last = j == n - 1;
  switch (j) {
    case 0: hipLaunchKernelGGL(xp_update_h_k<0>, grid, dim3(block), 0, s, gv, lg, st, x, p[j], o, pout, r, last); break;
    case 1: hipLaunchKernelGGL(xp_update_h_k<1>, grid, dim3(block), 0, s, gv, lg, st, x, p[j], o, pout, r, last); break;
    case 2: hipLaunchKernelGGL(xp_update_h_k<2>, grid, dim3(block), 0, s, gv, lg, st, x, p[j], o, pout, r, last); break;
    default: hipLaunchKernelGGL(xp_update_h_k<3>, grid, dim3(block), 0, s, gv, lg, st, x, p[j], o, pout, r, last); break;
  }
  return hipGetLastError();
}
hipError_t launch_ru_accum(const Geom& gv, int lg, const CgState* st, SpF64 xhi, SpF32 xlo, const SpH* p, int q,
                           int block, hipStream_t s) {
  if (q < 0 || q > 3) return hipErrorInvalidValue;
  const dim3 grid(blocks_for(gv.Vh, block));
  Older<SpH> pend{};
  for (int m = 0; m < q; ++m) pend.p[m] = p[q - 1 - m];
  switch (q) {
    case 0: hipLaunchKernelGGL(ru_accum_k<0>, grid, dim3(block), 0, s, gv, lg, st, xhi, xlo, pend); break;
    case 1: hipLaunchKernelGGL(ru_accum_k<1>, grid, dim3(block), 0, s, gv, lg, st, xhi, xlo, pend); break;
    case 2: hipLaunchKernelGGL(ru_accum_k<2>, grid, dim3(block), 0, s, gv, lg, st, xhi, xlo, pend); break;
    default: hipLaunchKernelGGL(ru_accum_k<3>, grid, dim3(block), 0, s, gv, lg, st, xhi, xlo, pend); break;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ conversions
template <class FS, class FD>
__global__ void __launch_bounds__(256) convert_k(Geom g, FS src, FD dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.Vh) return;
  Spinor<double> vd;
  load(src, i, vd);
  if constexpr (std::is_same_v<FD, SpF64>) {
    store(dst, i, vd);
  } else {
    // round to float32 first: the binary16 and FP32 encoders work on float32 values
    Spinor<float> vf;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) vf.v[s][c] = {float(vd.v[s][c].re), float(vd.v[s][c].im)};
    store(dst, i, vf);
  }
}
template <class FS>
static hipError_t convert_to(const Geom& g, FS src, SpRef dst, int block, hipStream_t s) {
  const int nb = blocks_for(g.Vh, block);
  if (dst.kind == SP_F64)
    hipLaunchKernelGGL((convert_k<FS, SpF64>), dim3(nb), dim3(block), 0, s, g, src, SpF64{(double2*)dst.p, g.stride});
  else if (dst.kind == SP_F32)
    hipLaunchKernelGGL((convert_k<FS, SpF32>), dim3(nb), dim3(block), 0, s, g, src, SpF32{(float4*)dst.p, g.stride});
  else if (dst.kind == SP_H)
    hipLaunchKernelGGL((convert_k<FS, SpH>), dim3(nb), dim3(block), 0, s, g, src, SpH{(uint4*)dst.p, dst.s, g.stride});
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
hipError_t launch_convert(const Geom& g, SpRef src, SpRef dst, int block, hipStream_t s) {
  if (src.kind == SP_F64) return convert_to(g, SpF64{(double2*)src.p, g.stride}, dst, block, s);
  if (src.kind == SP_F32) return convert_to(g, SpF32{(float4*)src.p, g.stride}, dst, block, s);
  if (src.kind == SP_H) return convert_to(g, SpH{(uint4*)src.p, src.s, g.stride}, dst, block, s);
  return hipErrorInvalidValue;
}

template <class F>
__global__ void __launch_bounds__(256) zero_k(Geom g, F x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.Vh) return;
  Spinor<float> z;
  zero(z);
  store(x, i, z);
}
hipError_t launch_zero(const Geom& g, SpRef x, int block, hipStream_t s) {
  const int nb = blocks_for(g.Vh, block);
  if (x.kind == SP_F64)
    hipLaunchKernelGGL(zero_k<SpF64>, dim3(nb), dim3(block), 0, s, g, SpF64{(double2*)x.p, g.stride});
  else if (x.kind == SP_F32)
    hipLaunchKernelGGL(zero_k<SpF32>, dim3(nb), dim3(block), 0, s, g, SpF32{(float4*)x.p, g.stride});
  else if (x.kind == SP_H)
    hipLaunchKernelGGL(zero_k<SpH>, dim3(nb), dim3(block), 0, s, g, SpH{(uint4*)x.p, x.s, g.stride});
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Reference encoder for checking: user complex128 [n][12] -> codes [n][3] x 8 binary16, scale [n]
__global__ void encode_half_k(int n, const double2* __restrict__ user, uint4* __restrict__ codes,
                              float* __restrict__ scale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Spinor<float> v;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const double2 d = user[(size_t)i * 12 + k];
    v.v[k / 3][k % 3] = {float(d.x), float(d.y)};
  }
  h8_t h[3];
  const float m = encode_site(v, h);
#pragma unroll
  for (int k = 0; k < 3; ++k) codes[(size_t)i * 3 + k] = from_h8(h[k]);
  scale[i] = m;
}
hipError_t launch_encode_half(int n, const double2* user, uint4* codes, float* scale, hipStream_t s) {
  hipLaunchKernelGGL(encode_half_k, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, user, codes, scale);
  return hipGetLastError();
}

// ------------------------------------------------------------------ bandwidth calibration
__global__ void __launch_bounds__(256) stream_copy_k(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                     uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}
hipError_t launch_stream_copy(const uint4* src, uint4* dst, uint64_t n16, hipStream_t s) {
  uint64_t nb = (n16 + 255) / 256;
  if (nb > 256 * 64) nb = 256 * 64;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(stream_copy_k, dim3((unsigned)nb), dim3(256), 0, s, src, dst, n16);
  return hipGetLastError();
}

}  // namespace qcd
