// Wilson-clover hopping kernels for gfx950.
//
// One work-item per output site of one checkerboard.  For every direction
// the two neighbour spinors (opposite checkerboard) are spin-projected to
// half spinors, multiplied by the link (or its adjoint), rebuilt and
// accumulated; the 6x6 clover blocks are applied before (site term) or
// after (A^{-1} of the even-odd preconditioner) the hop; an epilogue stores
// the result, or fuses the CG residual update, and leaves per-workgroup
// partial sums of |out|^2 for a deterministic two-pass reduction.
//
// The same template serves every form the solver needs:
//   k1:  t_o = A_oo^{-1} H_oe psi_e                  (site none, post clover)
//   k2:  out_e = A_ee psi_e - kappa^2 H_eo t_o       (site with clover)
//   M:   out_p = A_pp psi_p - kappa H psi_(1-p)      (site with clover)
//   bhat = b_e + kappa H_eo u_o, x_o = A^{-1}(b_o + kappa H_oe x_e)
// Mhat^dag = g5 Mhat g5 uses the g5in / g5out switches.
#include <type_traits>

#include "qcd_internal.h"

namespace qcd {

struct SpNone {};

template <class SIn, class SSite, class SOut, class LK, class CPre, class CPost>
struct DArgs {
  Geom g;
  int par_out;
  SIn in;
  SSite site;
  SOut out;
  SOut y;
  LK U;
  CPre cpre;
  CPost cpost;
  double c;
  int epi;
  double a;
  int a_from_state;
  int g5in, g5out;
  const CgState* st;
  double* partial;
  int lg;  // log2 of the number of interleaved right-hand sides (MULTI kernels)
  // MULTI site order: z-tiles of 1 << tile_lg planes, t inside a tile
  int tile_lg, plane;  // plane = (Lx / 2) Ly checkerboard sites per z-t plane
  double inv_plane, inv_t;
  float one;  // 1, opaque to the compiler (see project())
  CgState* fin_st;  // see DslashOp
  const double* fin_partial;
  int fin_n, fin_nr;
};

// Workgroups r < fin_nr finish alpha for right-hand side r (the sums of the
// previous launch's |Mhat p|^2 partials) with the finalisation kernels' fixed
// summation, run by this kernel's workgroup size, so the result is the same
// on every run; whole workgroups take the same branch.
template <class A>
__device__ __forceinline__ void fused_fin_alpha(const A& a) {
  if ((int)blockIdx.x >= a.fin_nr) return;
  CgState* st = a.fin_st + blockIdx.x;
  if (st->halt) return;
  const double qq = block_sum_partials(a.fin_partial + (size_t)blockIdx.x * a.fin_n, a.fin_n);
  if (threadIdx.x == 0) state_alpha(st, qq);
}

// Site of the multi-source kernel's j-th work position.  The sites are taken
// in xy-planes, then z within a tile of 1 << tile_lg planes, then t, then
// the next z-tile: neighbours in t are two tiles' worth of sites apart in
// this order (in x-fastest order they would be two whole t-slices apart,
// which with 8 interleaved sources no longer fits the L2 of an XCD).
template <class A>
__device__ __forceinline__ int multi_site(const A& a, int j, int x[4]) {
  const Geom& g = a.g;
  int p, t, xh;
  const int q = fdivmod(j, a.plane, a.inv_plane, p);
  const int zi = q & ((1 << a.tile_lg) - 1);
  const int zt = fdivmod(q >> a.tile_lg, g.X[3], a.inv_t, t);
  const int z = (zt << a.tile_lg) + zi;
  const int y = fdivmod(p, g.Xh, g.inv_xh, xh);
  x[1] = y;
  x[2] = z;
  x[3] = t;
  x[0] = 2 * xh + ((y + z + t + a.par_out) & 1);
  return p + a.plane * (z + g.X[2] * t);
}

template <typename R>
__device__ __forceinline__ void scale_half(Half<R>& h, R f) {
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) h.h[k][c] = f * h.h[k][c];
}

// One direction mu: the forward hop (1 - gamma_mu) U_mu(x) psi(x + mu) and
// the backward hop (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu).  gamma5 on
// the input (G5IN) is a compile-time sign that folds into the projection;
// a binary16 field's per-site scale (with the antiperiodic-time sign and
// the factors cu, cl of the upper and lower output spins) enters the
// multiply-adds that accumulate U h; an unscaled field takes the sign on
// the projected half spinor.  No branch may split this block: with a
// branch the FP64 kernel runs out of registers and spills.
// i: checkerboard site (links, clover); r: right-hand side (MULTI: spinor
// element (cb << lg) | r, otherwise cb).
template <int MU, bool G5IN, bool MULTI, bool FUSED, bool SCALED_ACC, typename R, class A>
__device__ __forceinline__ void hop_dir(const A& a, int i, int r, const int x[4], Spinor<R>& acc, R cu, R cl) {
  using SIn = decltype(a.in);
  constexpr bool scaled = SpinorScale<SIn>::scaled;
  const Geom& g = a.g;
  int y[4] = {x[0], x[1], x[2], x[3]};
  y[MU] = (x[MU] + 1 == g.X[MU]) ? 0 : x[MU] + 1;
  const int nf = lex(y, g) >> 1;
  y[MU] = (x[MU] == 0 ? g.X[MU] : x[MU]) - 1;
  const int nb = lex(y, g) >> 1;
  const int ef = MULTI ? ((nf << a.lg) | r) : nf, eb = MULTI ? ((nb << a.lg) | r) : nb;
  Spinor<R> pf, pb;
  Mat<R> uf, ub;
  load_raw(a.in, ef, pf);
  load_link(a.U, MU, a.par_out, i, uf);
  load_raw(a.in, eb, pb);
  load_link(a.U, MU, 1 - a.par_out, nb, ub);
  if constexpr (G5IN) {
    neg_lower(pf);
    neg_lower(pb);
  }
  R sf = R(1), sb = R(1);
  if constexpr (scaled) {
    sf = R(scale_of(a.in, ef));
    sb = R(scale_of(a.in, eb));
  }
  if constexpr (MU == 3) {
    sf = (g.tb < 0 && x[3] == g.X[3] - 1) ? -sf : sf;
    sb = (g.tb < 0 && x[3] == 0) ? -sb : sb;
  }
  Half<R> h, uh;
  if constexpr (scaled)
    project<MU, -1>(pf, h, R(a.one));
  else
    project<MU, -1>(pf, h);
  if constexpr (!SCALED_ACC && MU == 3) scale_half(h, sf);
  mul_mat<FUSED>(uf, h, uh);
  if constexpr (SCALED_ACC)
    accumulate<MU, -1>(acc, uh, sf * cu, sf * cl);
  else
    accumulate<MU, -1>(acc, uh);
  if constexpr (scaled)
    project<MU, +1>(pb, h, R(a.one));
  else
    project<MU, +1>(pb, h);
  if constexpr (!SCALED_ACC && MU == 3) scale_half(h, sb);
  mul_adj<FUSED>(ub, h, uh);
  if constexpr (SCALED_ACC)
    accumulate<MU, +1>(acc, uh, sb * cu, sb * cl);
  else
    accumulate<MU, +1>(acc, uh);
}

// The site term's clover: general Hermitian blocks, or the compact form of
// a clover term built from links.
template <bool FUSED_CL, typename R, class CL>
__device__ __forceinline__ void site_clover(const CL& c, int i, Spinor<R>& s) {
  if constexpr (CloverCompact<CL>::value)
    apply_cclover(c, i, s);
  else
    apply_clover<FUSED_CL>(c, i, s);
}

// MULTI: one work-item per (site, right-hand side) with the right-hand side
// fastest, so the 1 << lg work-items of a site share its link and clover
// loads; halted right-hand sides keep computing with alpha = 0 (the grid
// cannot return early for some of them).
// Wavefronts per SIMD the register allocation must leave room for: FP32
// k1 4 (121 registers), k2 5 (96) except with an FP32 clover (which would
// spill there) and the single-source k2 with the compact clover (5 spills
// 8 bytes per work-item; at 4, 103 registers and 2.6 % faster); FP64
// kernels take what they need (2).
template <typename R, int SITE, class A, bool MULTI>
constexpr int stencil_waves() {
  if (sizeof(R) == 8) return 1;
  if (SITE == 2 && !MULTI && std::is_same<decltype(A::cpre), CloverHC>::value) return 4;
  if (SITE == 2 && !std::is_same<decltype(A::cpre), CloverF32>::value) return 5;
  return 4;
}

template <typename R, int SITE, bool POST, bool G5IN, bool MULTI, class A>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(stencil_waves<R, SITE, A, MULTI>())))
dslash_kernel(A a) {
  // A launch that finishes alpha itself (fin_nr > 0, the dagger k1) may set
  // halt while it runs, so it does not read halt at all: it reads no alpha,
  // and the k2 that consumes its output returns early once halt is set.
  // Otherwise halt was set by an earlier launch and is uniform over the grid.
  if (a.fin_nr > 0)
    fused_fin_alpha(a);
  else if (!MULTI && a.st != nullptr && a.st->halt)
    return;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int w = blk * blockDim.x + threadIdx.x;  // work position
  const int r = MULTI ? (w & ((1 << a.lg) - 1)) : 0;
  double nrm = 0.0;
  if ((MULTI ? (w >> a.lg) : w) < a.g.Vh) {
    int x[4];
    int i;  // checkerboard site
    if constexpr (MULTI) {
      i = multi_site(a, w >> a.lg, x);
    } else {
      i = w;
      cb_coords(i, a.par_out, a.g, x);
    }
    const int e = MULTI ? ((i << a.lg) | r) : i;  // spinor element
    constexpr bool scaled = SpinorScale<decltype(a.in)>::scaled;
    // hop scale, with gamma5 on the output folded into the lower spins
    const R c = R(a.c), cl = a.g5out ? R(-a.c) : R(a.c);
    // binary16 input: the site term comes first (its loads are consumed at
    // once instead of living across the hops) and the hop scale rides on the
    // accumulating multiply-adds; with no site term and a scaled post clover
    // it joins the blocks' scales instead
    constexpr bool SITE_FIRST = SITE != 0;
    constexpr bool HOP_IN_CLOVER = POST && SITE == 0 && scaled && CloverScale<decltype(a.cpost)>::scaled;
    constexpr bool HOP_IN_ACC = SITE_FIRST;
    // fused link matvecs except in the FP32 site-term kernel (k2), which
    // would then spill at four wavefronts per SIMD
    constexpr bool FUSED = SITE == 0 || sizeof(R) == 8;
    // the FP32 clover products as fused chains; FP64 (HBM-bound) keeps the
    // form that needs fewer registers
    constexpr bool FUSED_CL = (FUSED || SITE_FIRST) && sizeof(R) == 4;
    Spinor<R> acc;
    if constexpr (SITE_FIRST) {
      load_once(a.site, e, acc);
      if constexpr (SITE == 2) site_clover<FUSED_CL>(a.cpre, i, acc);
    } else {
      zero(acc);
    }
    const R hu = HOP_IN_ACC ? c : R(1), hl = HOP_IN_ACC ? cl : R(1);
    constexpr bool SCALED_ACC = scaled || HOP_IN_ACC;
    hop_dir<0, G5IN, MULTI, FUSED, SCALED_ACC>(a, i, r, x, acc, hu, hl);
    hop_dir<1, G5IN, MULTI, FUSED, SCALED_ACC>(a, i, r, x, acc, hu, hl);
    hop_dir<2, G5IN, MULTI, FUSED, SCALED_ACC>(a, i, r, x, acc, hu, hl);
    hop_dir<3, G5IN, MULTI, FUSED, SCALED_ACC>(a, i, r, x, acc, hu, hl);
    if constexpr (!HOP_IN_CLOVER && !HOP_IN_ACC) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        acc.v[0][k] = c * acc.v[0][k];
        acc.v[1][k] = c * acc.v[1][k];
        acc.v[2][k] = cl * acc.v[2][k];
        acc.v[3][k] = cl * acc.v[3][k];
      }
    }
    if constexpr (SITE != 0 && !SITE_FIRST) {
      Spinor<R> sv;
      load_once(a.site, e, sv);
      if constexpr (SITE == 2) site_clover<FUSED_CL>(a.cpre, i, sv);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int k = 0; k < 3; ++k) acc.v[s][k] = acc.v[s][k] + sv.v[s][k];
    }
    if constexpr (HOP_IN_CLOVER)
      apply_clover<FUSED_CL, true>(a.cpost, i, acc, c, cl);
    else if constexpr (POST)
      apply_clover<FUSED_CL>(a.cpost, i, acc);
    if (a.epi == 2) {
      Spinor<R> yv;
      load_once(a.y, e, yv);
      R al;
      if constexpr (MULTI)
        al = a.a_from_state ? (a.st[r].halt ? R(0) : R(-a.st[r].alpha)) : R(a.a);
      else
        al = a.a_from_state ? R(-a.st->alpha) : R(a.a);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int k = 0; k < 3; ++k) yv.v[s][k] = yv.v[s][k] + al * acc.v[s][k];
      store(a.out, e, yv);
      nrm = site_norm2(yv);
    } else {
      store(a.out, e, acc);
      if (a.epi == 1) nrm = site_norm2(acc);
    }
  }
  if (a.epi >= 1) {
    if constexpr (MULTI)
      block_sum_store_seg(nrm, a.partial, blk, gridDim.x, a.lg);
    else
      block_sum_store(nrm, a.partial, blk);
  }
}

// ------------------------------------------------------------------ small grids: two wavefronts per 64 sites
// Below one wavefront per SIMD, one work-item per site leaves SIMDs idle and
// each wavefront waits out its own loads.  Here a workgroup of two
// wavefronts takes 64 sites: wavefront 0 the four forward hops, wavefront 1
// the four backward ones.  Each passes the partial sum of the chiral half it
// does not keep to the other through LDS, and wavefront h then finishes
// chiral half h (spins 2h, 2h + 1): the hop factor, its part of the site
// term, its clover block (A is block-diagonal in the chiral halves) and its
// half of the output.  Each branch on h is uniform within a wavefront.

// Half h of a site spinor: complex components 6h .. 6h + 5.
template <int H, typename R>
__device__ __forceinline__ void load_half(const SpF64& f, int i, Cx<R> v[6]) {
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const double2 d = ld_stream(f.p + sp64_at(6 * H + j, i));
    v[j] = {R(d.x), R(d.y)};
  }
}
// binary16 chunk k holds complex components 4k .. 4k + 3: half 0 is chunk 0
// and the first 8 bytes of chunk 1, half 1 the last 8 bytes of chunk 1 and
// chunk 2.
template <int H, typename R>
__device__ __forceinline__ void load_half(const SpH& f, int i, Cx<R> v[6]) {
  const float s = *elem(f.s, 0, i);
  const h4_t m = as_h4(((const uint2*)elem(f.p, (size_t)64, sph_at(i)))[H]);
  const h8_t o = as_h8(*elem(f.p, (size_t)(2 * H) * 64, sph_at(i)));
#pragma unroll
  for (int j = 0; j < 4; ++j) v[H == 0 ? j : j + 2] = {R(float(o[2 * j]) * s), R(float(o[2 * j + 1]) * s)};
#pragma unroll
  for (int j = 0; j < 2; ++j) v[H == 0 ? j + 4 : j] = {R(float(m[2 * j]) * s), R(float(m[2 * j + 1]) * s)};
}
template <typename R>
__device__ __forceinline__ float half_max(const Cx<R> v[6]) {
  float m = 0.f;
#pragma unroll
  for (int j = 0; j < 6; ++j) m = fmaxf(m, fmaxf(fabsf(float(v[j].re)), fabsf(float(v[j].im))));
  return m;
}
template <int H, typename R>
__device__ __forceinline__ void store_half(const SpF64& f, int i, const Cx<R> v[6], float) {
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const nt_d2 w = {double(v[j].re), double(v[j].im)};
    __builtin_nontemporal_store(w, (nt_d2*)(f.p + sp64_at(6 * H + j, i)));
  }
}
// m: the site's max |component| over both halves, as the one-work-item encoder takes it
template <int H, typename R>
__device__ __forceinline__ void store_half(const SpH& f, int i, const Cx<R> v[6], float m) {
  const float inv = m > 0.f ? 1.0f / m : 0.f;
  h8_t o;
  h4_t q;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const Cx<R> z = v[H == 0 ? j : j + 2];
    o[2 * j] = (_Float16)(float(z.re) * inv);
    o[2 * j + 1] = (_Float16)(float(z.im) * inv);
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const Cx<R> z = v[H == 0 ? j + 4 : j];
    q[2 * j] = (_Float16)(float(z.re) * inv);
    q[2 * j + 1] = (_Float16)(float(z.im) * inv);
  }
  const uint4 wo = from_h8(o);
  const uint2 wq = from_h4(q);
  const nt_u4 no = {wo.x, wo.y, wo.z, wo.w};
  const nt_u2 nq = {wq.x, wq.y};
  __builtin_nontemporal_store(no, (nt_u4*)elem(f.p, (size_t)(2 * H) * 64, sph_at(i)));
  __builtin_nontemporal_store(nq, (nt_u2*)elem(f.p, (size_t)64, sph_at(i)) + H);
  if (H == 1) __builtin_nontemporal_store(m, elem(f.s, 0, i));
}

// One hop of direction MU: S = -1 forward, (1 - gamma_mu) U_mu(x) psi(x + mu);
// S = +1 backward, (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu).
template <int MU, int S, bool G5IN, bool FUSED, typename R, class A>
__device__ __forceinline__ void hop_one(const A& a, int i, const int x[4], Spinor<R>& acc) {
  using SIn = decltype(a.in);
  constexpr bool scaled = SpinorScale<SIn>::scaled;
  const Geom& g = a.g;
  int y[4] = {x[0], x[1], x[2], x[3]};
  if (S < 0)
    y[MU] = (x[MU] + 1 == g.X[MU]) ? 0 : x[MU] + 1;
  else
    y[MU] = (x[MU] == 0 ? g.X[MU] : x[MU]) - 1;
  const int n = lex(y, g) >> 1;
  Spinor<R> p;
  Mat<R> u;
  load_raw(a.in, n, p);
  if (S < 0)
    load_link(a.U, MU, a.par_out, i, u);
  else
    load_link(a.U, MU, 1 - a.par_out, n, u);
  if constexpr (G5IN) neg_lower(p);
  R sc = R(1);
  if constexpr (scaled) sc = R(scale_of(a.in, n));
  if constexpr (MU == 3) sc = (g.tb < 0 && x[3] == (S < 0 ? g.X[3] - 1 : 0)) ? -sc : sc;
  Half<R> h, uh;
  if constexpr (scaled)
    project<MU, S>(p, h, R(a.one));
  else
    project<MU, S>(p, h);
  if constexpr (!scaled && MU == 3) scale_half(h, sc);
  if constexpr (S < 0)
    mul_mat<FUSED>(u, h, uh);
  else
    mul_adj<FUSED>(u, h, uh);
  if constexpr (scaled)
    accumulate<MU, S>(acc, uh, sc, sc);
  else
    accumulate<MU, S>(acc, uh);
}

// Clover block H times v, times f (and the block's own scale)
template <int H, bool FUSED, typename R, class CL>
__device__ __forceinline__ void apply_block(const CL& c, int i, Cx<R> v[6], R f) {
  R bs = R(1);
  if constexpr (CloverScale<CL>::scaled) {
    const float2 sc = block_scales(c, i);
    bs = R(H == 0 ? sc.x : sc.y);
  }
  Block<R> blk;
  load_block(c, i, H, blk);
  block_mv<FUSED>(blk, v);
  const R t = bs * f;
#pragma unroll
  for (int j = 0; j < 6; ++j) v[j] = t * v[j];
}

template <typename R>
struct PairLds {
  Cx<R> part[2][6][64];  // [half][component][site]: the other wavefront's partial sums
  float m[2][64];        // per-half max |component| of a binary16 output
};

// Phase 1 of wavefront H: its four hops; hands the other half to LDS and keeps its own.
template <int H, typename R, bool G5IN, class A>
__device__ __forceinline__ void pair_hops(const A& a, int i, int lane, PairLds<R>& L, Cx<R> v[6]) {
  int x[4];
  cb_coords(i, a.par_out, a.g, x);
  Spinor<R> acc;
  zero(acc);
  constexpr int S = H == 0 ? -1 : +1;
  hop_one<0, S, G5IN, true>(a, i, x, acc);
  hop_one<1, S, G5IN, true>(a, i, x, acc);
  hop_one<2, S, G5IN, true>(a, i, x, acc);
  hop_one<3, S, G5IN, true>(a, i, x, acc);
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    L.part[1 - H][j][lane] = acc.v[2 * (1 - H) + j / 3][j % 3];
    v[j] = acc.v[2 * H + j / 3][j % 3];
  }
}

// Chiral half H of a site from the sum v of all its hops: hop factor, site
// term, clover, epilogue value; returns the half's max |component|.
template <int H, typename R, int SITE, bool POST, class A>
__device__ __forceinline__ float finish_half(const A& a, int i, Cx<R> v[6]) {
  const R c = H == 0 ? R(a.c) : (a.g5out ? R(-a.c) : R(a.c));
  constexpr bool FUSED_CL = sizeof(R) == 4;
  if constexpr (POST && SITE == 0) {
    apply_block<H, FUSED_CL>(a.cpost, i, v, c);
  } else {
#pragma unroll
    for (int j = 0; j < 6; ++j) v[j] = c * v[j];
    if constexpr (SITE != 0) {
      Cx<R> sv[6];
      load_half<H>(a.site, i, sv);
      if constexpr (SITE == 2) {
        if constexpr (CloverCompact<decltype(a.cpre)>::value) {
          CBlock<R> blk;
          load_cblock(a.cpre, i, H, blk);
          R f = R(1);
          if constexpr (CloverScale<decltype(a.cpre)>::scaled) {
            const float2 sc = block_scales(a.cpre, i);
            f = R(H == 0 ? sc.x : sc.y);
          }
          cblock_mv(blk, sv, f);
        } else {
          apply_block<H, FUSED_CL>(a.cpre, i, sv, R(1));
        }
      }
#pragma unroll
      for (int j = 0; j < 6; ++j) v[j] = v[j] + sv[j];
    }
    if constexpr (POST) apply_block<H, FUSED_CL>(a.cpost, i, v, R(1));
  }
  if (a.epi == 2) {
    Cx<R> yv[6];
    load_half<H>(a.y, i, yv);
    const R al = a.a_from_state ? R(-a.st->alpha) : R(a.a);
#pragma unroll
    for (int j = 0; j < 6; ++j) v[j] = yv[j] + al * v[j];
  }
  return half_max(v);
}

// Phase 2 of wavefront H: the whole half (its own hops and the other
// wavefront's), then finish_half.
template <int H, typename R, int SITE, bool POST, class A>
__device__ __forceinline__ void pair_finish(const A& a, int i, int lane, PairLds<R>& L, Cx<R> v[6]) {
#pragma unroll
  for (int j = 0; j < 6; ++j) v[j] = v[j] + L.part[H][j][lane];
  L.m[H][lane] = finish_half<H, R, SITE, POST>(a, i, v);
}

template <typename R, int SITE, bool POST, bool G5IN, class A>
__global__ void __launch_bounds__(128) dslash_pair_kernel(A a) {
  // as in dslash_kernel: a launch that finishes alpha never reads halt, so
  // both wavefronts of every workgroup reach the barriers below
  if (a.fin_nr > 0)
    fused_fin_alpha(a);
  else if (a.st != nullptr && a.st->halt)
    return;
  __shared__ PairLds<R> L;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x & 63, h = threadIdx.x >> 6;
  const int i = blk * 64 + lane;
  const bool live = i < a.g.Vh;
  Cx<R> v[6];
  if (live) {
    if (h == 0)
      pair_hops<0, R, G5IN>(a, i, lane, L, v);
    else
      pair_hops<1, R, G5IN>(a, i, lane, L, v);
  }
  __syncthreads();
  if (live) {
    if (h == 0)
      pair_finish<0, R, SITE, POST>(a, i, lane, L, v);
    else
      pair_finish<1, R, SITE, POST>(a, i, lane, L, v);
  }
  __syncthreads();
  double nrm = 0.0;
  if (live) {
    const float m = fmaxf(L.m[0][lane], L.m[1][lane]);
    if (h == 0)
      store_half<0>(a.out, i, v, m);
    else
      store_half<1>(a.out, i, v, m);
    if (a.epi >= 1) {
#pragma unroll
      for (int j = 0; j < 6; ++j) nrm += double(v[j].re) * double(v[j].re) + double(v[j].im) * double(v[j].im);
    }
  }
  if (a.epi >= 1) block_sum_store(nrm, a.partial, blk);
}

// ------------------------------------------------------------------ small grids: four wavefronts per 64 sites
// (small-grid option 2) Wavefront mu of a workgroup of four takes both hops
// of direction mu for the 64 sites; the four partial sums meet in LDS, and
// wavefronts 0 and 1 add them (in the order of the wavefronts) for chiral
// halves 0 and 1 and finish those as in the two-wavefront form.  Each
// wavefront waits out two hops instead of four, and twice as many are in
// flight.
template <typename R>
struct QuadLds {
  Cx<R> part[4][2][6][64];  // [wavefront][half][component][site]
  float m[2][64];           // per-half max |component| of a binary16 output
};

template <int MU, typename R, bool G5IN, class A>
__device__ __forceinline__ void quad_hops(const A& a, int i, Spinor<R>& acc) {
  int x[4];
  cb_coords(i, a.par_out, a.g, x);
  zero(acc);
  hop_one<MU, -1, G5IN, true>(a, i, x, acc);
  hop_one<MU, +1, G5IN, true>(a, i, x, acc);
}

template <typename R, int SITE, bool POST, bool G5IN, class A>
__global__ void __launch_bounds__(256) dslash_quad_kernel(A a) {
  // as in dslash_kernel: a launch that finishes alpha never reads halt, so
  // all four wavefronts of every workgroup reach the barriers below
  if (a.fin_nr > 0)
    fused_fin_alpha(a);
  else if (a.st != nullptr && a.st->halt)
    return;
  __shared__ QuadLds<R> L;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blk * 64 + lane;
  const bool live = i < a.g.Vh;
  if (live) {
    Spinor<R> acc;
    if (w == 0)
      quad_hops<0, R, G5IN>(a, i, acc);
    else if (w == 1)
      quad_hops<1, R, G5IN>(a, i, acc);
    else if (w == 2)
      quad_hops<2, R, G5IN>(a, i, acc);
    else
      quad_hops<3, R, G5IN>(a, i, acc);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int j = 0; j < 6; ++j) L.part[w][h][j][lane] = acc.v[2 * h + j / 3][j % 3];
  }
  __syncthreads();
  Cx<R> v[6];
  if (live && w < 2) {
#pragma unroll
    for (int j = 0; j < 6; ++j)
      v[j] = ((L.part[0][w][j][lane] + L.part[1][w][j][lane]) + L.part[2][w][j][lane]) + L.part[3][w][j][lane];
    if (w == 0)
      L.m[0][lane] = finish_half<0, R, SITE, POST>(a, i, v);
    else
      L.m[1][lane] = finish_half<1, R, SITE, POST>(a, i, v);
  }
  __syncthreads();
  double nrm = 0.0;
  if (live && w < 2) {
    const float m = fmaxf(L.m[0][lane], L.m[1][lane]);
    if (w == 0)
      store_half<0>(a.out, i, v, m);
    else
      store_half<1>(a.out, i, v, m);
    if (a.epi >= 1) {
#pragma unroll
      for (int j = 0; j < 6; ++j) nrm += double(v[j].re) * double(v[j].re) + double(v[j].im) * double(v[j].im);
    }
  }
  if (a.epi >= 1) block_sum_store(nrm, a.partial, blk);
}

// ------------------------------------------------------------------ dispatch
template <class T>
T sp_of(const SpRef& r, int stride);
template <>
SpF64 sp_of<SpF64>(const SpRef& r, int stride) { return SpF64{(double2*)r.p, stride}; }
template <>
SpF32 sp_of<SpF32>(const SpRef& r, int stride) { return SpF32{(float4*)r.p, stride}; }
template <>
SpH sp_of<SpH>(const SpRef& r, int stride) { return SpH{(uint4*)r.p, r.s, stride}; }
template <>
SpNone sp_of<SpNone>(const SpRef&, int) { return SpNone{}; }

template <class T>
T cl_of(const ClovRef& r, int stride);
template <>
CloverF64 cl_of<CloverF64>(const ClovRef& r, int stride) { return CloverF64{(const double2*)r.p, stride}; }
template <>
CloverF32 cl_of<CloverF32>(const ClovRef& r, int stride) { return CloverF32{(const float4*)r.p, stride}; }
template <>
CloverH cl_of<CloverH>(const ClovRef& r, int stride) { return CloverH{(const uint4*)r.p, r.s, stride}; }
template <>
CloverNone cl_of<CloverNone>(const ClovRef&, int) { return CloverNone{}; }
template <>
CloverF64C cl_of<CloverF64C>(const ClovRef& r, int stride) { return CloverF64C{(const double2*)r.p, stride}; }
template <>
CloverHC cl_of<CloverHC>(const ClovRef& r, int stride) { return CloverHC{(const uint4*)r.p, r.s, stride}; }

template <class T>
T lk_of(const void* p, int stride);
template <>
LinkF64<9> lk_of<LinkF64<9>>(const void* p, int stride) { return LinkF64<9>{(const double2*)p, stride}; }
template <>
LinkF64<6> lk_of<LinkF64<6>>(const void* p, int stride) { return LinkF64<6>{(const double2*)p, stride}; }
template <>
LinkH12 lk_of<LinkH12>(const void* p, int stride) {
  const uint4* c = (const uint4*)p;
  return LinkH12{c, (const uint2*)(c + (size_t)8 * stride), stride};
}
template <>
LinkH18 lk_of<LinkH18>(const void* p, int stride) {
  const uint4* c = (const uint4*)p;
  return LinkH18{c, (const unsigned int*)(c + (size_t)16 * stride), stride};
}

// one work-item per site: up to this many sites the grid has less than one
// wavefront per SIMD (256 CUs x 4 SIMDs x 64 lanes), and the single-source
// stencils take two wavefronts per 64 sites instead
constexpr int kSmallVh = 256 * 4 * 64;

template <typename R, class SIn, class SSite, class SOut, class LK, class CPre, class CPost, int SITE, bool POST,
          bool G5IN>
static hipError_t run_g5(const Geom& g, const DslashOp& op, int block, hipStream_t s) {
  DArgs<SIn, SSite, SOut, LK, CPre, CPost> a;
  const int ss = g.stride << op.lg;  // spinor stride: all right-hand sides
  a.g = g;
  a.par_out = op.par_out;
  a.in = sp_of<SIn>(op.in, ss);
  a.site = sp_of<SSite>(op.site, ss);
  a.out = sp_of<SOut>(op.out, ss);
  a.y = op.epi == 2 ? sp_of<SOut>(op.y, ss) : a.out;
  a.U = lk_of<LK>(op.links, g.stride);
  a.cpre = cl_of<CPre>(op.cpre, g.stride);
  a.cpost = cl_of<CPost>(op.cpost, g.stride);
  a.c = op.c;
  a.epi = op.epi;
  a.a = op.a;
  a.a_from_state = op.a_from_state;
  a.g5in = op.g5in;
  a.g5out = op.g5out;
  a.st = op.st;
  a.partial = op.partial;
  a.lg = op.lg;
  a.tile_lg = 0;
  while (a.tile_lg < 2 && g.X[2] % (2 << a.tile_lg) == 0) ++a.tile_lg;
  a.plane = g.Xh * g.X[1];
  a.inv_plane = 1.0 / a.plane;
  a.inv_t = 1.0 / g.X[3];
  a.one = 1.0f;
  a.fin_st = op.fin_st;
  a.fin_partial = op.fin_partial;
  a.fin_n = op.fin_n;
  a.fin_nr = op.fin_nr;
  const int nb = blocks_for(g.Vh << op.lg, block);
  constexpr bool multi_only = std::is_same<LK, LinkH18>::value;  // 18-entry links serve the multi-source kernels
  if (op.lg > 0)
    hipLaunchKernelGGL((dslash_kernel<R, SITE, POST, G5IN, true, decltype(a)>), dim3(nb), dim3(block), 0, s, a);
  else if constexpr (multi_only)
    return hipErrorInvalidValue;
  else if (g.Vh <= kSmallVh && op.small_grid == 1 && block == 64)
    hipLaunchKernelGGL((dslash_pair_kernel<R, SITE, POST, G5IN, decltype(a)>), dim3(nb), dim3(128), 0, s, a);
  else if (g.Vh <= kSmallVh && op.small_grid == 2 && block == 64)
    hipLaunchKernelGGL((dslash_quad_kernel<R, SITE, POST, G5IN, decltype(a)>), dim3(nb), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((dslash_kernel<R, SITE, POST, G5IN, false, decltype(a)>), dim3(nb), dim3(block), 0, s, a);
  return hipGetLastError();
}

template <typename R, class SIn, class SSite, class SOut, class LK, class CPre, class CPost, int SITE, bool POST>
static hipError_t run(const Geom& g, const DslashOp& op, int block, hipStream_t s) {
  if (op.g5in) return run_g5<R, SIn, SSite, SOut, LK, CPre, CPost, SITE, POST, true>(g, op, block, s);
  return run_g5<R, SIn, SSite, SOut, LK, CPre, CPost, SITE, POST, false>(g, op, block, s);
}

template <int NC>
static hipError_t run_f64(const Geom& g, const DslashOp& op, int block, hipStream_t s) {
  using L = LinkF64<NC>;
  if (op.site_mode == 0 && op.post)
    return run<double, SpF64, SpNone, SpF64, L, CloverNone, CloverF64, 0, true>(g, op, block, s);
  if (op.site_mode == 2 && !op.post) {
    if constexpr (NC == 6) {
      if (op.cpre.kind == CL_F64C)
        return run<double, SpF64, SpF64, SpF64, L, CloverF64C, CloverNone, 2, false>(g, op, block, s);
    }
    if (op.cpre.kind != CL_F64) return hipErrorInvalidValue;
    return run<double, SpF64, SpF64, SpF64, L, CloverF64, CloverNone, 2, false>(g, op, block, s);
  }
  if (op.site_mode == 1 && !op.post)
    return run<double, SpF64, SpF64, SpF64, L, CloverNone, CloverNone, 1, false>(g, op, block, s);
  if (op.site_mode == 1 && op.post)
    return run<double, SpF64, SpF64, SpF64, L, CloverNone, CloverF64, 1, true>(g, op, block, s);
  return hipErrorInvalidValue;
}

template <class CL, class LK>
static hipError_t run_mixed(const Geom& g, const DslashOp& op, int block, hipStream_t s) {
  if (op.site_mode == 0 && op.post)
    return run<float, SpH, SpNone, SpH, LK, CloverNone, CL, 0, true>(g, op, block, s);
  if (op.site_mode == 2 && !op.post)
    return run<float, SpH, SpH, SpH, LK, CL, CloverNone, 2, false>(g, op, block, s);
  return hipErrorInvalidValue;
}

hipError_t launch_dslash(const Geom& g, const DslashOp& op, int block, hipStream_t s) {
  if (op.in.kind == SP_F64) {
    if (op.link_kind == LK_F64_12) return run_f64<6>(g, op, block, s);
    if (op.link_kind == LK_F64_18) return run_f64<9>(g, op, block, s);
    return hipErrorInvalidValue;
  }
  if (op.in.kind == SP_H && op.link_kind == LK_H12) {
    const int ck = op.post ? op.cpost.kind : op.cpre.kind;
    if (ck == CL_F32) return run_mixed<CloverF32, LinkH12>(g, op, block, s);
    if (ck == CL_H) return run_mixed<CloverH, LinkH12>(g, op, block, s);
    if (ck == CL_HC && op.site_mode == 2 && !op.post)
      return run<float, SpH, SpH, SpH, LinkH12, CloverHC, CloverNone, 2, false>(g, op, block, s);
  }
  if (op.in.kind == SP_H && op.link_kind == LK_H18 && op.lg > 0) {
    const int ck = op.post ? op.cpost.kind : op.cpre.kind;
    if (ck == CL_F32) return run_mixed<CloverF32, LinkH18>(g, op, block, s);
    if (ck == CL_H) return run_mixed<CloverH, LinkH18>(g, op, block, s);
    if (ck == CL_HC && op.site_mode == 2 && !op.post)
      return run<float, SpH, SpH, SpH, LinkH18, CloverHC, CloverNone, 2, false>(g, op, block, s);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ clover only
// element e = (cb << lg) | r
__global__ void __launch_bounds__(256) clover_apply_kernel(Geom g, int lg, SpF64 in, SpF64 out, CloverF64 c) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (g.Vh << lg)) return;
  Spinor<double> v;
  load(in, e, v);
  apply_clover(c, e >> lg, v);
  store(out, e, v);
}

hipError_t launch_clover_apply(const Geom& g, int lg, SpF64 in, SpF64 out, const double2* clov, hipStream_t s) {
  hipLaunchKernelGGL(clover_apply_kernel, dim3(blocks_for(g.Vh << lg, 256)), dim3(256), 0, s, g, lg, in, out,
                     CloverF64{clov, g.stride});
  return hipGetLastError();
}

}  // namespace qcd
