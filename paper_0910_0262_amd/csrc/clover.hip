// Clover term: field strength from the four-leaf clover and the two 6x6
// Hermitian blocks of A = 1 - kappa c_sw sum_{mu<nu} sigma_mu,nu (x) F_mu,nu,
// then the inverse of the odd-site blocks for the even-odd preconditioner.
//
// In the chiral basis sigma_mu,nu = diag(B_up, B_dn) with 2x2 blocks
//   (0,1): -s3, -s3   (0,2): s2, s2   (0,3): s1, -s1
//   (1,2): -s1, -s1   (1,3): s2, -s2  (2,3): s3, -s3
// so sum sigma (x) F = s1 (x) X + s2 (x) Y + s3 (x) Z per chirality with
//   upper: X = F03 - F12, Y = F02 + F13, Z = F23 - F01
//   lower: X = -F12 - F03, Y = F02 - F13, Z = -F01 - F23,
// and s1 (x) X + s2 (x) Y + s3 (x) Z = [[Z, X - iY], [X + iY, -Z]].
#include "md_order.h"

namespace qcd {

// Each link enters the leaves of many sites: ordinary (cached) loads.
__device__ __forceinline__ Mat<double> link_at(const double2* u18, const Geom& g, int mu, const int x[4]) {
  const double2* base = u18 + (size_t)((mu * 2 + parity_of(x)) * 9) * g.stride + (lex(x, g) >> 1);
  Mat<double> u;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double2 d = base[(size_t)k * g.stride];
    u.m[k / 3][k % 3] = {d.x, d.y};
  }
  return u;
}
__device__ __forceinline__ void shift(const Geom& g, const int x[4], int mu, int n, int y[4]) {
  y[0] = x[0];
  y[1] = x[1];
  y[2] = x[2];
  y[3] = x[3];
  y[mu] = (x[mu] + n + 2 * g.X[mu]) % g.X[mu];
}

// F_mu,nu(x) = traceless part of (Q - Q^dag) / (8i), Q the sum of the four
// counter-clockwise leaves in the mu-nu plane starting at x.
__device__ Mat<double> field_strength(const double2* u18, const Geom& g, const int x[4], int mu, int nu) {
  int xp_mu[4], xp_nu[4], xm_mu[4], xm_nu[4], xm_mu_p_nu[4], xm_mu_m_nu[4], xp_mu_m_nu[4];
  shift(g, x, mu, 1, xp_mu);
  shift(g, x, nu, 1, xp_nu);
  shift(g, x, mu, -1, xm_mu);
  shift(g, x, nu, -1, xm_nu);
  shift(g, xm_mu, nu, 1, xm_mu_p_nu);
  shift(g, xm_mu, nu, -1, xm_mu_m_nu);
  shift(g, xp_mu, nu, -1, xp_mu_m_nu);

  const Mat<double> um_x = link_at(u18, g, mu, x), un_x = link_at(u18, g, nu, x);
  Mat<double> q;
  // U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
  q = mm(mm(um_x, link_at(u18, g, nu, xp_mu)), mm(adj(link_at(u18, g, mu, xp_nu)), adj(un_x)));
  // U_nu(x) U_mu(x-mu+nu)^dag U_nu(x-mu)^dag U_mu(x-mu)
  const Mat<double> um_xm = link_at(u18, g, mu, xm_mu);
  q = madd(q, mm(mm(un_x, adj(link_at(u18, g, mu, xm_mu_p_nu))), mm(adj(link_at(u18, g, nu, xm_mu)), um_xm)));
  // U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_nu(x-nu)
  const Mat<double> un_xm = link_at(u18, g, nu, xm_nu);
  q = madd(q, mm(mm(adj(um_xm), adj(link_at(u18, g, nu, xm_mu_m_nu))), mm(link_at(u18, g, mu, xm_mu_m_nu), un_xm)));
  // U_nu(x-nu)^dag U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^dag
  q = madd(q, mm(mm(adj(un_xm), link_at(u18, g, mu, xm_nu)), mm(link_at(u18, g, nu, xp_mu_m_nu), adj(um_x))));

  Mat<double> f;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const Cx<double> d = q.m[a][b] - conj(q.m[b][a]);
      f.m[a][b] = {d.im / 8.0, -d.re / 8.0};  // d / (8 i)
    }
  const double tr = (f.m[0][0].re + f.m[1][1].re + f.m[2][2].re) / 3.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) f.m[a][a].re -= tr;
  return f;
}

__global__ void __launch_bounds__(64) clover_build_k(Geom g, const double2* __restrict__ u18, double kc,
                                                     double2* __restrict__ clov) {
  const int j = md_position();
  if (j >= g.V) return;
  int x[4];
  const int i = md_site(j, g, x);
  const int par = parity_of(x), cb = i >> 1;
  const Mat<double> f01 = field_strength(u18, g, x, 0, 1);
  const Mat<double> f02 = field_strength(u18, g, x, 0, 2);
  const Mat<double> f03 = field_strength(u18, g, x, 0, 3);
  const Mat<double> f12 = field_strength(u18, g, x, 1, 2);
  const Mat<double> f13 = field_strength(u18, g, x, 1, 3);
  const Mat<double> f23 = field_strength(u18, g, x, 2, 3);
#pragma unroll 1
  for (int b = 0; b < 2; ++b) {
    Mat<double> X, Y, Z;
    if (b == 0) {
      X = msub(f03, f12);
      Y = madd(f02, f13);
      Z = msub(f23, f01);
    } else {
      X = msub(mzero<double>(), madd(f12, f03));
      Y = msub(f02, f13);
      Z = msub(mzero<double>(), madd(f01, f23));
    }
    // 6x6 block entry (r, c): sub-block (r / 3, c / 3), colour (r % 3, c % 3)
    Cx<double> blk[6][6];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const Cx<double> z = Z.m[a][c], xx = X.m[a][c], yy = Y.m[a][c];
        const Cx<double> one = {a == c ? 1.0 : 0.0, 0.0};
        blk[a][c] = one - kc * z;
        blk[3 + a][3 + c] = one + kc * z;
        blk[a][3 + c] = -kc * (xx - ti(yy));
        blk[3 + a][c] = -kc * (xx + ti(yy));
      }
    double2* dst = clov + (size_t)(par * 36 + b * 18) * g.stride + cb;
#pragma unroll
    for (int k = 0; k < 3; ++k) dst[(size_t)k * g.stride] = make_double2(blk[2 * k][2 * k].re, blk[2 * k + 1][2 * k + 1].re);
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int c = r + 1; c < 6; ++c)
        dst[(size_t)(3 + offd(r, c)) * g.stride] = make_double2(blk[r][c].re, blk[r][c].im);
  }
}

hipError_t launch_clover_build(const Geom& g, const double2* u18, double kappa, double csw, double2* clov,
                               hipStream_t s) {
  hipLaunchKernelGGL(clover_build_k, dim3(blocks_for(g.V, 64)), dim3(64), 0, s, g, u18, kappa * csw, clov);
  return hipGetLastError();
}

// ------------------------------------------------------------------ inversion
// Hermitian positive-definite 6x6 inverse by Cholesky A = L L^dag:
// A^{-1} = L^{-dag} L^{-1}, and ln det A = sum_j ln L_jj^2.  Returns false if
// a pivot is not positive.
__device__ __forceinline__ bool invert_block(const Block<double>& a, Block<double>& inv, double& logdet) {
  Cx<double> L[6][6];
  logdet = 0.0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double d = a.d[j];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= norm2(L[j][k]);
    if (!(d > 0.0)) return false;
    logdet += log(d);
    const double ljj = sqrt(d), rinv = 1.0 / ljj;
    L[j][j] = {ljj, 0.0};
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      Cx<double> s = conj(a.o[offd(j, i)]);  // A_ij for i > j
#pragma unroll
      for (int k = 0; k < j; ++k) s = s - L[i][k] * conj(L[j][k]);
      L[i][j] = rinv * s;
    }
  }
  // T = L^{-1}, lower triangular
  Cx<double> T[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    T[i][i] = {1.0 / L[i][i].re, 0.0};
#pragma unroll
    for (int j = 0; j < i; ++j) {
      Cx<double> s = {0.0, 0.0};
#pragma unroll
      for (int k = j; k < i; ++k) s = s + L[i][k] * T[k][j];
      T[i][j] = (-1.0 / L[i][i].re) * s;
    }
  }
  // inv = T^dag T: inv_rc = sum_{k >= max(r,c)} conj(T_kr) T_kc
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    double d = 0.0;
#pragma unroll
    for (int k = r; k < 6; ++k) d += norm2(T[k][r]);
    inv.d[r] = d;
#pragma unroll
    for (int c = r + 1; c < 6; ++c) {
      Cx<double> s = {0.0, 0.0};
#pragma unroll
      for (int k = c; k < 6; ++k) s = s + cmulc(T[k][r], T[k][c]);
      inv.o[offd(r, c)] = s;
    }
  }
  return true;
}

__device__ void store_block_f64(double2* base, int stride, int i, const Block<double>& b) {
#pragma unroll
  for (int k = 0; k < 3; ++k) base[(size_t)k * stride + i] = make_double2(b.d[2 * k], b.d[2 * k + 1]);
#pragma unroll
  for (int k = 0; k < 15; ++k) base[(size_t)(3 + k) * stride + i] = make_double2(b.o[k].re, b.o[k].im);
}
__device__ void block_reals(const Block<double>& b, double r[36]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) r[k] = b.d[k];
#pragma unroll
  for (int k = 0; k < 15; ++k) {
    r[6 + 2 * k] = b.o[k].re;
    r[7 + 2 * k] = b.o[k].im;
  }
}
// The 36 reals of one block in FP32, and their max |real|.
__device__ __forceinline__ float block_reals32(const Block<double>& b, float r[36]) {
  double rr[36];
  block_reals(b, rr);
  float m = 0.f;
#pragma unroll
  for (int k = 0; k < 36; ++k) {
    r[k] = float(rr[k]);
    m = fmaxf(m, fabsf(r[k]));
  }
  return m;
}
// FP32 copy: 18 float4 chunks, reals [b * 36 + r]; binary16 copy: 9 chunks of
// 8 halves with a per-block float32 scale (max |real|).
__device__ __forceinline__ void store_low(const float r[72], const float sc[2], float4* f32, uint4* h16, float2* hs,
                                          int stride, int i) {
#pragma unroll
  for (int k = 0; k < 18; ++k) f32[(size_t)k * stride + i] = make_float4(r[4 * k], r[4 * k + 1], r[4 * k + 2], r[4 * k + 3]);
  const float inv0 = sc[0] > 0.f ? 1.0f / sc[0] : 0.f, inv1 = sc[1] > 0.f ? 1.0f / sc[1] : 0.f;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    h8_t h;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int q = 8 * k + j;
      h[j] = (_Float16)(r[q] * (q < 36 ? inv0 : inv1));
    }
    h16[(size_t)k * stride + i] = from_h8(h);
  }
  hs[i] = make_float2(sc[0], sc[1]);
}

// Odd-site block B: A_oo^{-1} in FP64 (zero if A is not positive definite)
// and its reals in FP32 for the low-precision copies.  The two blocks go
// through this one after the other with compile-time indices: a loop over
// them indexed its arrays at run time, which put both blocks and both
// inverses in scratch memory.
template <int B>
__device__ __forceinline__ bool invert_site_block(const CloverF64& co, int i, double2* clov_inv, int stride,
                                                  float r[36], float& sc, double& ld) {
  Block<double> a, inv;
  load_block(co, i, B, a);
  const bool ok = invert_block(a, inv, ld);
  if (!ok) {
    ld = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) inv.d[k] = 0.0;
#pragma unroll
    for (int k = 0; k < 15; ++k) inv.o[k] = {0.0, 0.0};
  }
  store_block_f64(clov_inv + (size_t)(B * 18) * stride, stride, i, inv);
  sc = block_reals32(inv, r);
  return ok;
}

__global__ void __launch_bounds__(64) clover_invert_k(Geom g, const double2* __restrict__ clov,
                                                      double2* __restrict__ clov_inv, float4* clov32_e,
                                                      float4* clovinv32_o, uint4* clovh_e, float2* clovh_es,
                                                      uint4* clovinvh_o, float2* clovinvh_os,
                                                      double* __restrict__ logdet, int* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.Vh) return;
  const CloverF64 ce{clov, g.stride}, co{clov + (size_t)36 * g.stride, g.stride};
  float r[72], sc[2];
  {
    // even sites: low-precision copies of A_ee
    Block<double> a;
    load_block(ce, i, 0, a);
    sc[0] = block_reals32(a, r);
    load_block(ce, i, 1, a);
    sc[1] = block_reals32(a, r + 36);
    store_low(r, sc, clov32_e, clovh_e, clovh_es, g.stride, i);
  }
  // odd sites: A_oo^{-1}
  double ld0 = 0.0, ld1 = 0.0;
  const bool ok0 = invert_site_block<0>(co, i, clov_inv, g.stride, r, sc[0], ld0);
  const bool ok1 = invert_site_block<1>(co, i, clov_inv, g.stride, r + 36, sc[1], ld1);
  store_low(r, sc, clovinv32_o, clovinvh_o, clovinvh_os, g.stride, i);
  const bool ok = ok0 && ok1;
  logdet[i] = ok ? ld0 + ld1 : 0.0;
  if (!ok) *status = 1;
}

// Compact copies of A_ee (the site term of k2): per chiral block X3 and W of
// 1 - [[X3, W], [W^dag, -X3]] read off the FP64 block, 26 reals, in FP64 and
// in binary16 with a per-block scale.  The form holds for a clover term built
// from links; for any other (a loaded one) status is set and the caller keeps
// the full blocks.
__global__ void __launch_bounds__(64) clover_compact_k(Geom g, const double2* __restrict__ clov, double2* c64,
                                                        uint4* ch, float2* chs, int* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.Vh) return;
  const CloverF64 ce{clov, g.stride};
  float r32[52];
  float sc[2];
  double dev = 0.0;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    Block<double> a;
    load_block(ce, i, b, a);
    double r[26];
    r[0] = 0.5 * (a.d[3] - a.d[0]);
    r[1] = 0.5 * (a.d[4] - a.d[1]);
    const Cx<double> x01 = 0.5 * (a.o[offd(3, 4)] - a.o[offd(0, 1)]);
    const Cx<double> x02 = 0.5 * (a.o[offd(3, 5)] - a.o[offd(0, 2)]);
    const Cx<double> x12 = 0.5 * (a.o[offd(4, 5)] - a.o[offd(1, 2)]);
    r[2] = x01.re;
    r[3] = x01.im;
    r[4] = x02.re;
    r[5] = x02.im;
    r[6] = x12.re;
    r[7] = x12.im;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const Cx<double> w = a.o[offd(k / 3, 3 + k % 3)];
      r[8 + 2 * k] = -w.re;
      r[9 + 2 * k] = -w.im;
    }
    // B00 + B11 = 2 and tr X3 = 0
#pragma unroll
    for (int k = 0; k < 3; ++k) dev = fmax(dev, fabs(a.d[k] + a.d[3 + k] - 2.0));
    const Cx<double> s01 = a.o[offd(0, 1)] + a.o[offd(3, 4)], s02 = a.o[offd(0, 2)] + a.o[offd(3, 5)],
                     s12 = a.o[offd(1, 2)] + a.o[offd(4, 5)];
    dev = fmax(dev, fmax(fmax(fabs(s01.re), fabs(s01.im)), fmax(fabs(s02.re), fabs(s02.im))));
    dev = fmax(dev, fmax(fabs(s12.re), fabs(s12.im)));
    dev = fmax(dev, fabs(a.d[3] + a.d[4] + a.d[5] - a.d[0] - a.d[1] - a.d[2]));
#pragma unroll
    for (int k = 0; k < 13; ++k)
      c64[(size_t)(b * 13 + k) * g.stride + i] = make_double2(r[2 * k], r[2 * k + 1]);
    float m = 0.f;
#pragma unroll
    for (int k = 0; k < 26; ++k) {
      r32[26 * b + k] = float(r[k]);
      m = fmaxf(m, fabsf(r32[26 * b + k]));
    }
    sc[b] = m;
  }
  const float inv0 = sc[0] > 0.f ? 1.0f / sc[0] : 0.f, inv1 = sc[1] > 0.f ? 1.0f / sc[1] : 0.f;
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    h8_t h;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int q = 8 * k + j;
      h[j] = q < 52 ? (_Float16)(r32[q] * (q < 26 ? inv0 : inv1)) : (_Float16)0.f;
    }
    if (k < 6) {
      ch[(size_t)k * g.stride + i] = from_h8(h);
    } else {
      const h4_t t = {h[0], h[1], h[2], h[3]};
      ((uint2*)(ch + (size_t)6 * g.stride))[i] = from_h4(t);
    }
  }
  chs[i] = make_float2(sc[0], sc[1]);
  if (dev > 1e-12) *status = 1;
}

hipError_t launch_clover_compact(const Geom& g, const double2* clov_e, double2* c64, uint4* ch, float2* chs,
                                 int* status, hipStream_t s) {
  hipLaunchKernelGGL(clover_compact_k, dim3(blocks_for(g.Vh, 64)), dim3(64), 0, s, g, clov_e, c64, ch, chs, status);
  return hipGetLastError();
}

hipError_t launch_clover_invert(const Geom& g, const double2* clov, double2* clov_inv, float4* clov32_e,
                                float4* clovinv32_o, uint4* clovh_e, float2* clovh_es, uint4* clovinvh_o,
                                float2* clovinvh_os, double* logdet, int* status, hipStream_t s) {
  hipLaunchKernelGGL(clover_invert_k, dim3(blocks_for(g.Vh, 64)), dim3(64), 0, s, g, clov, clov_inv, clov32_e,
                     clovinv32_o, clovh_e, clovh_es, clovinvh_o, clovinvh_os, logdet, status);
  return hipGetLastError();
}

}  // namespace qcd
