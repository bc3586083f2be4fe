// Fermion force for S = phi^dag (Mhat^dag Mhat)^{-1} phi and the HMD link and
// momentum updates.
//
// With X = (Mhat^dag Mhat)^{-1} phi, Y = Mhat X, Z = A_oo^{-1} H_oe X and
// W = A_oo^{-1} H_eo^dag Y, the first-order change of S is
//   dS = 2 kappa^2 Re[l^dag dH r] + 2 kappa c_sw Re sum_x,mu<nu tr[dF_mu,nu(x) Gamma_mu,nu(x)]
// with full-lattice l = (Y even, W odd), r = (X even, Z odd) and
// Gamma_mu,nu(x)_ba = sum_s,s' (sigma_mu,nu)_ss' Lambda(x)_(s'b),(sa),
// Lambda = X Y^dag on even sites and kappa^2 Z W^dag on odd sites.
// The kernels write G = dS/dRe U + i dS/dIm U per link (dS = Re sum conj(G) dU).
//
// Hopping part, per link U_mu(x) (eta = boundary sign of the hop):
//   G = 2 kappa^2 eta (B^dag + C),
//   B = sum_k h-_k(r(x+mu)) h-_k(l(x))^dag,  C = sum_k h+_k(r(x)) h+_k(l(x+mu))^dag,
// where h-(v), h+(v) are the upper spin pair of (1 -+ gamma_mu) v: the
// projectors are rank two, so the spin trace reduces to two colour outer products.
//
// Clover part: Re tr[dF Gamma] = (1/4) Im tr[dQ Xi] with Xi the Hermitian part
// of the traceless part of Gamma; each link enters the leaves of 6 plaquettes
// at 4 corners each, and a leaf derivative is the product of the other three
// links with Xi inserted at the leaf's corner.
#include "md_order.h"

namespace qcd {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ void shift4(const Geom& g, const int x[4], int mu, int n, int y[4]) {
  y[0] = x[0];
  y[1] = x[1];
  y[2] = x[2];
  y[3] = x[3];
  y[mu] = (x[mu] + n + 2 * g.X[mu]) % g.X[mu];
}
// Links are gathered by many neighbouring threads here, so they are read
// with ordinary (cached) loads, unlike the stencil's streaming loads.
__device__ __forceinline__ Mat<double> u_at(const double2* u18, const Geom& g, int mu, const int x[4]) {
  const double2* base = u18 + (size_t)((mu * 2 + parity_of(x)) * 9) * g.stride + (lex(x, g) >> 1);
  Mat<double> u;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double2 d = base[(size_t)k * g.stride];
    u.m[k / 3][k % 3] = {d.x, d.y};
  }
  return u;
}
__device__ __forceinline__ void spinor_at(SpF64 e, SpF64 o, const Geom& g, const int x[4], Spinor<double>& v) {
  load(parity_of(x) ? o : e, lex(x, g) >> 1, v);
}
// out += sum_k a_k (x) b_k^dag  (colour outer products, out[row][col] = a_row conj(b_col))
__device__ __forceinline__ void outer_acc(Mat<double>& out, const Half<double>& a, const Half<double>& b) {
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) out.m[r][c] = out.m[r][c] + a.h[k][r] * conj(b.h[k][c]);
}
__device__ __forceinline__ void store_mat(double2* base, int stride, int i, const Mat<double>& m) {
#pragma unroll
  for (int k = 0; k < 9; ++k) base[(size_t)k * stride + i] = make_double2(m.m[k / 3][k % 3].re, m.m[k / 3][k % 3].im);
}
__device__ __forceinline__ Mat<double> load_mat(const double2* base, int stride, int i) {
  Mat<double> m;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double2 d = base[(size_t)k * stride + i];
    m.m[k / 3][k % 3] = {d.x, d.y};
  }
  return m;
}

// ------------------------------------------------------------------ hopping force
template <int MU>
__device__ __forceinline__ Mat<double> hop_force_dir(const Geom& g, const int x[4], SpF64 le, SpF64 lo, SpF64 re,
                                                     SpF64 ro) {
  int y[4];
  shift4(g, x, MU, 1, y);
  Spinor<double> l_x, r_x, l_y, r_y;
  spinor_at(le, lo, g, x, l_x);
  spinor_at(re, ro, g, x, r_x);
  spinor_at(le, lo, g, y, l_y);
  spinor_at(re, ro, g, y, r_y);
  Half<double> a, b;
  Mat<double> B = mzero<double>(), C = mzero<double>();
  project<MU, -1>(r_y, a);
  project<MU, -1>(l_x, b);
  outer_acc(B, a, b);
  project<MU, +1>(r_x, a);
  project<MU, +1>(l_y, b);
  outer_acc(C, a, b);
  return madd(adj(B), C);
}

__global__ void __launch_bounds__(128) force_hop_k(Geom g, const double2* __restrict__ u18, SpF64 le, SpF64 lo,
                                                   SpF64 re, SpF64 ro, double coef, double2* __restrict__ gint) {
  const int j = md_position();
  if (j >= g.V) return;
  int x[4];
  const int i = md_site(j, g, x);
  const int par = parity_of(x), cb = i >> 1;
  Mat<double> f[4];
  f[0] = hop_force_dir<0>(g, x, le, lo, re, ro);
  f[1] = hop_force_dir<1>(g, x, le, lo, re, ro);
  f[2] = hop_force_dir<2>(g, x, le, lo, re, ro);
  f[3] = hop_force_dir<3>(g, x, le, lo, re, ro);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const double eta = (mu == 3 && g.tb < 0 && x[3] == g.X[3] - 1) ? -coef : coef;
    Mat<double> m;
#pragma unroll
    for (int k = 0; k < 9; ++k) m.m[k / 3][k % 3] = eta * f[mu].m[k / 3][k % 3];
    store_mat(gint + (size_t)((mu * 2 + par) * 9) * g.stride, g.stride, cb, m);
  }
}

hipError_t launch_force_hop(const Geom& g, const double2* u18, SpF64 ell_e, SpF64 ell_o, SpF64 rho_e, SpF64 rho_o,
                            double coef, double2* gint, hipStream_t s) {
  hipLaunchKernelGGL(force_hop_k, dim3(blocks_for(g.V, 128)), dim3(128), 0, s, g, u18, ell_e, ell_o, rho_e, rho_o,
                     coef, gint);
  return hipGetLastError();
}

// ------------------------------------------------------------------ clover force: Xi per site
// plane p: 0 (0,1), 1 (0,2), 2 (0,3), 3 (1,2), 4 (1,3), 5 (2,3)
// sigma block on a spin pair (a, b): k = 1: (b, a); k = 2: (-i b, i a); k = 3: (a, -b); times sign
__device__ __forceinline__ void pauli(int k, double sgn, const Cx<double> a[3], const Cx<double> b[3],
                                      Cx<double> oa[3], Cx<double> ob[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (k == 1) {
      oa[c] = sgn * b[c];
      ob[c] = sgn * a[c];
    } else if (k == 2) {
      oa[c] = sgn * tmi(b[c]);
      ob[c] = sgn * ti(a[c]);
    } else {
      oa[c] = sgn * a[c];
      ob[c] = -sgn * b[c];
    }
  }
}

// Entry B(r, c) of one packed Hermitian 6x6 block (plain loads: each entry is
// read by several planes).
__device__ __forceinline__ Cx<double> blk_at(const double2* base, int stride, int i, int r, int c) {
  if (r == c) {
    const double2 d = base[(size_t)(r >> 1) * stride + i];
    return {(r & 1) ? d.y : d.x, 0.0};
  }
  const int a = r < c ? r : c, b = r < c ? c : r;
  const double2 o = base[(size_t)(3 + offd(a, b)) * stride + i];
  return r < c ? Cx<double>{o.x, o.y} : Cx<double>{o.x, -o.y};
}
// Gamma(x)_ij += w sum_{s,s'} (sgn s_k)_{s s'} B_{(s' i),(s j)} for one chiral
// block B (local spins 0, 1) whose sigma_mu,nu block is sgn times Pauli s_k.
__device__ __forceinline__ void det_gamma_acc(Mat<double>& G, const double2* base, int stride, int i, int k,
                                              double w) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      Cx<double> v;
      if (k == 1) {
        v = blk_at(base, stride, i, 3 + a, b) + blk_at(base, stride, i, a, 3 + b);
      } else if (k == 2) {
        v = tmi(blk_at(base, stride, i, 3 + a, b)) + ti(blk_at(base, stride, i, a, 3 + b));
      } else {
        v = blk_at(base, stride, i, a, b) - blk_at(base, stride, i, 3 + a, 3 + b);
      }
      G.m[a][b] = G.m[a][b] + w * v;
    }
}

// Xi per site and plane.  FERM: Lambda = r l^dag with weight w_e (even) or w_o
// (odd).  DET: Lambda += w_det A_oo^{-1} on odd sites (the derivative of
// -2 sum_odd ln det A has the same form as the fermion clover term, with
// A_oo^{-1} in place of kappa^2 Z W^dag).
template <bool FERM, bool DET>
__global__ void __launch_bounds__(128) clover_xi_k(Geom g, SpF64 le, SpF64 lo, SpF64 re, SpF64 ro, double w_e,
                                                   double w_o, const double2* __restrict__ cinv, double w_det,
                                                   double2* __restrict__ xi) {
  // work-items 0 .. Vh - 1 take the even sites and Vh .. V - 1 the odd ones
  // (by checkerboard index), so that a wavefront has one parity and the
  // determinant part (odd sites only) runs on whole wavefronts
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.V) return;
  const int par = t >= g.Vh ? 1 : 0, cb = t - par * g.Vh;
  Spinor<double> l, r;
  if constexpr (FERM) {
    load(par ? lo : le, cb, l);
    load(par ? ro : re, cb, r);
  }
  const double w = par ? w_o : w_e;
  // (k_up, sign_up, k_dn, sign_dn) for each plane
  const int ku[6] = {3, 2, 1, 1, 2, 3};
  const double su[6] = {-1, 1, 1, -1, 1, 1};
  const int kd[6] = {3, 2, 1, 1, 2, 3};
  const double sd[6] = {-1, 1, -1, -1, -1, -1};
#pragma unroll 1
  for (int p = 0; p < 6; ++p) {
    Mat<double> G = mzero<double>();
    if constexpr (FERM) {
      Spinor<double> sr;
      pauli(ku[p], su[p], r.v[0], r.v[1], sr.v[0], sr.v[1]);
      pauli(kd[p], sd[p], r.v[2], r.v[3], sr.v[2], sr.v[3]);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) G.m[a][b] = G.m[a][b] + w * (sr.v[s][a] * conj(l.v[s][b]));
    }
    if constexpr (DET) {
      if (par) {
        det_gamma_acc(G, cinv, g.stride, cb, ku[p], w_det * su[p]);
        det_gamma_acc(G, cinv + (size_t)18 * g.stride, g.stride, cb, kd[p], w_det * sd[p]);
      }
    }
    const Cx<double> tr = {(G.m[0][0].re + G.m[1][1].re + G.m[2][2].re) / 3.0,
                           (G.m[0][0].im + G.m[1][1].im + G.m[2][2].im) / 3.0};
#pragma unroll
    for (int a = 0; a < 3; ++a) G.m[a][a] = G.m[a][a] - tr;
    Mat<double> X;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) X.m[a][b] = 0.5 * (G.m[a][b] + conj(G.m[b][a]));
    store_mat(xi + (size_t)((par * 6 + p) * 9) * g.stride, g.stride, cb, X);
  }
}

hipError_t launch_clover_xi(const Geom& g, SpF64 ell_e, SpF64 ell_o, SpF64 rho_e, SpF64 rho_o, double w_e,
                            double w_o, const double2* cinv, double w_det, double2* xi, hipStream_t s) {
  const dim3 grid(blocks_for(g.V, 128)), block(128);
  const bool ferm = ell_e.p != nullptr, det = cinv != nullptr;
  if (ferm && det)
    hipLaunchKernelGGL((clover_xi_k<true, true>), grid, block, 0, s, g, ell_e, ell_o, rho_e, rho_o, w_e, w_o, cinv,
                       w_det, xi);
  else if (ferm)
    hipLaunchKernelGGL((clover_xi_k<true, false>), grid, block, 0, s, g, ell_e, ell_o, rho_e, rho_o, w_e, w_o, cinv,
                       w_det, xi);
  else if (det)
    hipLaunchKernelGGL((clover_xi_k<false, true>), grid, block, 0, s, g, ell_e, ell_o, rho_e, rho_o, w_e, w_o, cinv,
                       w_det, xi);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ------------------------------------------------------------------ clover force: leaf derivatives
__device__ __forceinline__ int plane_index(int a, int b) {  // a < b
  return a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
}
__device__ __forceinline__ Mat<double> xi_at(const double2* xi, const Geom& g, int p, const int x[4]) {
  return load_mat(xi + (size_t)((parity_of(x) * 6 + p) * 9) * g.stride, g.stride, lex(x, g) >> 1);
}
// Derivative matrix of the four leaves of one plaquette with respect to its
// first link: the loop continues with L1 L2 L3, and C0..C3 are Xi at the
// start points of (link, L1, L2, L3).  tr(dQ Xi) summed over the 4 leaves
// equals tr(dU M) with
//   M = L1 L2 L3 C0 + C1 L1 L2 L3 + L1 C2 L2 L3 + L1 L2 C3 L3
//     = L1 T + C1 (L1 A),  A = L2 L3,  T = A C0 + C2 A + L2 (C3 L3).
// The factors are fetched by the callables in the order they are needed,
// which keeps at most four 3x3 matrices live.
template <class F1, class F2, class F3, class G0, class G1, class G2, class G3>
__device__ __forceinline__ Mat<double> insertion(F1 l1, F2 l2, F3 l3, G0 c0, G1 c1, G2 c2, G3 c3,
                                                 Mat<double>* staple = nullptr) {
  Mat<double> A, T;
  {
    const Mat<double> L2 = l2(), L3 = l3();
    A = mm(L2, L3);
    T = mm(L2, mm(c3(), L3));
  }
  T = madd(T, mm(A, c0()));
  T = madd(T, mm(c2(), A));
  const Mat<double> L1 = l1();
  Mat<double> m = mm(L1, T);
  const Mat<double> st = mm(L1, A);  // L1 L2 L3: the plaquette without the link, a staple of the gauge force
  if (staple) *staple = st;
  return madd(m, mm(c1(), st));
}

// GAUGE: the products L1 L2 L3 of the two insertions of a plane are the
// up staple and the adjoint of the down staple of the Wilson gauge force
// (or the reverse), so that force is added here too, with weight coef_g, as
// gauge_force_k would add it.
template <bool GAUGE>
__global__ void __launch_bounds__(64) force_clover_k(Geom g, const double2* __restrict__ u18,
                                                     const double2* __restrict__ xi, double coef, double coef_g,
                                                     double2* __restrict__ gint) {
  int mu, i, y[4];
  if (!md_link(g, mu, i, y)) return;
  const int par = parity_of(y), cb = i >> 1;
  Mat<double> mt = mzero<double>();
  Mat<double> st = mzero<double>();  // staple sum (GAUGE)
  // planes in the order nu = mu ^ s: at each step the four directions of a
  // site pair up on two planes, whose Xi and links the two wavefronts of a
  // pair gather at about the same time
#pragma unroll 1
  for (int s = 1; s < 4; ++s) {
    const int nu = mu ^ s;
    const int p = mu < nu ? plane_index(mu, nu) : plane_index(nu, mu);
    int ypm[4], ypn[4], ymn[4], ypmpn[4], ypmmn[4];
    shift4(g, y, mu, 1, ypm);
    shift4(g, y, nu, 1, ypn);
    shift4(g, y, nu, -1, ymn);
    shift4(g, ypm, nu, 1, ypmpn);
    shift4(g, ypm, nu, -1, ypmmn);
    auto U = [&](int d, const int* c) { return u_at(u18, g, d, c); };
    auto Ud = [&](int d, const int* c) { return adj(u_at(u18, g, d, c)); };
    auto X = [&](const int* c) { return xi_at(xi, g, p, c); };
    Mat<double> mu_, md, s1, s2;
    Mat<double>* const p1 = GAUGE ? &s1 : nullptr;
    Mat<double>* const p2 = GAUGE ? &s2 : nullptr;
    if (mu < nu) {
      // link first in the plaquette at y (mu then nu); s1 = up staple
      mu_ = insertion([&] { return U(nu, ypm); }, [&] { return Ud(mu, ypn); }, [&] { return Ud(nu, y); },
                      [&] { return X(y); }, [&] { return X(ypm); }, [&] { return X(ypmpn); },
                      [&] { return X(ypn); }, p1);
      // link reversed (third) in the plaquette at y - nu; s2 = down staple^dag
      md = insertion([&] { return Ud(nu, ymn); }, [&] { return U(mu, ymn); }, [&] { return U(nu, ypmmn); },
                     [&] { return X(ypm); }, [&] { return X(y); }, [&] { return X(ymn); },
                     [&] { return X(ypmmn); }, p2);
    } else {
      // plane (nu, mu): link second in the plaquette at y - nu; s1 = down staple
      mu_ = insertion([&] { return Ud(nu, ypmmn); }, [&] { return Ud(mu, ymn); }, [&] { return U(nu, ymn); },
                      [&] { return X(y); }, [&] { return X(ypm); }, [&] { return X(ypmmn); },
                      [&] { return X(ymn); }, p1);
      // link reversed (fourth) in the plaquette at y; s2 = up staple^dag
      md = insertion([&] { return U(nu, y); }, [&] { return U(mu, ypn); }, [&] { return Ud(nu, ypm); },
                     [&] { return X(ypm); }, [&] { return X(y); }, [&] { return X(ypn); },
                     [&] { return X(ypmpn); }, p2);
    }
    // reversed occurrences: Im tr(dU^dag M) = -Im tr(dU M^dag)
    mt = madd(mt, msub(mu_, adj(md)));
    if constexpr (GAUGE) st = madd(st, madd(s1, adj(s2)));
  }
  // dS = coef Im tr(dU mt)  =>  G = coef * i * mt^dag
  double2* base = gint + (size_t)((mu * 2 + par) * 9) * g.stride;
  Mat<double> gm = load_mat(base, g.stride, cb);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) gm.m[r][c] = gm.m[r][c] + coef * ti(conj(mt.m[c][r]));
  if constexpr (GAUGE) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) gm.m[r][c] = gm.m[r][c] + coef_g * conj(st.m[c][r]);
  }
  store_mat(base, g.stride, cb, gm);
}

hipError_t launch_force_clover(const Geom& g, const double2* u18, const double2* xi, double coef, double2* gint,
                               hipStream_t s, double coef_g) {
  if (coef_g != 0.0)
    hipLaunchKernelGGL(force_clover_k<true>, dim3(md_link_blocks(g)), dim3(64), 0, s, g, u18, xi, coef, coef_g, gint);
  else
    hipLaunchKernelGGL(force_clover_k<false>, dim3(md_link_blocks(g)), dim3(64), 0, s, g, u18, xi, coef, 0.0, gint);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Wilson gauge action and force
// S_g = beta sum_{x, mu<nu} (1 - Re tr U_mu,nu(x) / 3).  For one link the
// plaquettes through it sum to Re tr(U_mu(x) A_mu(x)) with the staple sum
//   A_mu(x) = sum_{nu != mu} U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
//                          + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu),
// so dS_g = -(beta/3) Re tr(dU A) and G = -(beta/3) A^dag.
__device__ __forceinline__ Mat<double> staple_sum(const double2* u18, const Geom& g, int mu, const int y[4]) {
  Mat<double> a = mzero<double>();
#pragma unroll 1
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    int ypm[4], ypn[4], ymn[4], ypmmn[4];
    shift4(g, y, mu, 1, ypm);
    shift4(g, y, nu, 1, ypn);
    shift4(g, y, nu, -1, ymn);
    shift4(g, ypm, nu, -1, ypmmn);
    const Mat<double> up = mm(mm(u_at(u18, g, nu, ypm), adj(u_at(u18, g, mu, ypn))), adj(u_at(u18, g, nu, y)));
    const Mat<double> dn = mm(adj(mm(u_at(u18, g, mu, ymn), u_at(u18, g, nu, ypmmn))), u_at(u18, g, nu, ymn));
    a = madd(a, madd(up, dn));
  }
  return a;
}

// gint(mu, x) (+)= coef A_mu(x)^dag; one thread per link.
__global__ void __launch_bounds__(64) gauge_force_k(Geom g, const double2* __restrict__ u18, double coef,
                                                    int accumulate, double2* __restrict__ gint) {
  int mu, i, y[4];
  if (!md_link(g, mu, i, y)) return;
  const int par = parity_of(y), cb = i >> 1;
  const Mat<double> a = staple_sum(u18, g, mu, y);
  double2* base = gint + (size_t)((mu * 2 + par) * 9) * g.stride;
  Mat<double> gm = accumulate ? load_mat(base, g.stride, cb) : mzero<double>();
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) gm.m[r][c] = gm.m[r][c] + coef * conj(a.m[c][r]);
  store_mat(base, g.stride, cb, gm);
}

hipError_t launch_gauge_force(const Geom& g, const double2* u18, double coef, int accumulate, double2* gint,
                              hipStream_t s) {
  hipLaunchKernelGGL(gauge_force_k, dim3(md_link_blocks(g)), dim3(64), 0, s, g, u18, coef, accumulate, gint);
  return hipGetLastError();
}

// Per-block partial sums of sum_{mu<nu} (1 - Re tr U_mu,nu(x) / 3); thread t
// covers the two sites 2t and 2t + 1 (one of each parity).
__global__ void __launch_bounds__(256) plaquette_k(Geom g, const double2* __restrict__ u18, double* partial) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (t < g.Vh) {
#pragma unroll 1
    for (int k = 0; k < 2; ++k) {
      int x[4];
      lex_coords(2 * t + k, g, x);
#pragma unroll 1
      for (int mu = 0; mu < 3; ++mu)
#pragma unroll 1
        for (int nu = mu + 1; nu < 4; ++nu) {
          int xpm[4], xpn[4];
          shift4(g, x, mu, 1, xpm);
          shift4(g, x, nu, 1, xpn);
          const Mat<double> a = mm(u_at(u18, g, mu, x), u_at(u18, g, nu, xpm));
          const Mat<double> b = mm(u_at(u18, g, nu, x), u_at(u18, g, mu, xpn));
          // Re tr(a b^dag) = sum_rc Re(a_rc conj(b_rc))
          double re = 0.0;
#pragma unroll
          for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) re += a.m[r][c].re * b.m[r][c].re + a.m[r][c].im * b.m[r][c].im;
          acc += 1.0 - re / 3.0;
        }
    }
  }
  block_sum_store(acc, partial, blockIdx.x);
}

hipError_t launch_plaquette(const Geom& g, const double2* u18, double* partial, int block, hipStream_t s) {
  hipLaunchKernelGGL(plaquette_k, dim3(blocks_for(g.Vh, block)), dim3(block), 0, s, g, u18, partial);
  return hipGetLastError();
}

// Per-block partial sums of a checkerboard array of doubles.
__global__ void __launch_bounds__(256) sum_cb_k(int n, const double* __restrict__ v, double* partial) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  block_sum_store(t < n ? v[t] : 0.0, partial, blockIdx.x);
}

hipError_t launch_sum_cb(const Geom& g, const double* v, double* partial, int block, hipStream_t s) {
  hipLaunchKernelGGL(sum_cb_k, dim3(blocks_for(g.Vh, block)), dim3(block), 0, s, g.Vh, v, partial);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) fill_zero_k(size_t n, double2* __restrict__ p) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = make_double2(0.0, 0.0);
}

hipError_t launch_force_zero(const Geom& g, double2* gint, hipStream_t s) {
  const size_t n = (size_t)8 * 9 * g.stride;
  hipLaunchKernelGGL(fill_zero_k, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, gint);
  return hipGetLastError();
}

// ------------------------------------------------------------------ reunitarisation
// Row 0 normalised, row 1 orthogonalised against it and normalised, row 2 =
// conj(row 0 x row 1): the nearest SU(3) matrix in the Gram-Schmidt sense.
__global__ void __launch_bounds__(128) reunitarize_k(Geom g, double2* __restrict__ u18) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * g.V) return;
  const int mu = t / g.V, i = t - mu * g.V;
  int x[4];
  lex_coords(i, g, x);
  const int par = parity_of(x), cb = i >> 1;
  double2* base = u18 + (size_t)((mu * 2 + par) * 9) * g.stride;
  Mat<double> u = load_mat(base, g.stride, cb);
  double n0 = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) n0 += norm2(u.m[0][c]);
  n0 = 1.0 / sqrt(n0);
#pragma unroll
  for (int c = 0; c < 3; ++c) u.m[0][c] = n0 * u.m[0][c];
  Cx<double> d = {0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 3; ++c) d = d + cmulc(u.m[0][c], u.m[1][c]);  // conj(a) b
  double n1 = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    u.m[1][c] = u.m[1][c] - d * u.m[0][c];
    n1 += norm2(u.m[1][c]);
  }
  n1 = 1.0 / sqrt(n1);
#pragma unroll
  for (int c = 0; c < 3; ++c) u.m[1][c] = n1 * u.m[1][c];
  u.m[2][0] = conj(u.m[0][1] * u.m[1][2] - u.m[0][2] * u.m[1][1]);
  u.m[2][1] = conj(u.m[0][2] * u.m[1][0] - u.m[0][0] * u.m[1][2]);
  u.m[2][2] = conj(u.m[0][0] * u.m[1][1] - u.m[0][1] * u.m[1][0]);
  store_mat(base, g.stride, cb, u);
}

hipError_t launch_reunitarize(const Geom& g, double2* u18, hipStream_t s) {
  hipLaunchKernelGGL(reunitarize_k, dim3(blocks_for(4 * g.V, 128)), dim3(128), 0, s, g, u18);
  return hipGetLastError();
}

// ------------------------------------------------------------------ output: G and the su(3) force
// F^a = Re{ i tr[T^a U G^dag] } = -Im(tr[lambda^a W]) / 2, W = U G^dag
__global__ void __launch_bounds__(128) force_out_k(Geom g, const double2* __restrict__ u18,
                                                   const double2* __restrict__ gint, double2* __restrict__ g_user,
                                                   double* __restrict__ f_user) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * g.V) return;
  const int i = t >> 2, mu = t & 3;
  int x[4];
  lex_coords(i, g, x);
  const int par = parity_of(x), cb = i >> 1;
  const Mat<double> G = load_mat(gint + (size_t)((mu * 2 + par) * 9) * g.stride, g.stride, cb);
  if (g_user != nullptr) {
#pragma unroll
    for (int k = 0; k < 9; ++k) g_user[(size_t)t * 9 + k] = make_double2(G.m[k / 3][k % 3].re, G.m[k / 3][k % 3].im);
  }
  if (f_user == nullptr) return;
  const Mat<double> U = load_mat(u18 + (size_t)((mu * 2 + par) * 9) * g.stride, g.stride, cb);
  const Mat<double> W = mm(U, adj(G));
  const double r3 = 0.57735026918962576451;  // 1 / sqrt(3)
  double tr_im[8];
  tr_im[0] = W.m[0][1].im + W.m[1][0].im;
  tr_im[1] = (W.m[0][1] - W.m[1][0]).re;  // Im(i z) = Re z
  tr_im[2] = W.m[0][0].im - W.m[1][1].im;
  tr_im[3] = W.m[0][2].im + W.m[2][0].im;
  tr_im[4] = (W.m[0][2] - W.m[2][0]).re;
  tr_im[5] = W.m[1][2].im + W.m[2][1].im;
  tr_im[6] = (W.m[1][2] - W.m[2][1]).re;
  tr_im[7] = (W.m[0][0].im + W.m[1][1].im - 2.0 * W.m[2][2].im) * r3;
#pragma unroll
  for (int a = 0; a < 8; ++a) f_user[(size_t)t * 8 + a] = -0.5 * tr_im[a];
}

hipError_t launch_force_out(const Geom& g, const double2* u18, const double2* gint, double2* g_user,
                            double* f_user, hipStream_t s) {
  hipLaunchKernelGGL(force_out_k, dim3(blocks_for(4 * g.V, 128)), dim3(128), 0, s, g, u18, gint, g_user, f_user);
  return hipGetLastError();
}

// ------------------------------------------------------------------ HMD updates
// exp(i Q) for Hermitian traceless Q by the Cayley-Hamilton form of
// Morningstar and Peardon (Phys. Rev. D 69 (2004) 054501):
// exp(iQ) = f0 + f1 Q + f2 Q^2 with f_j from c0 = det Q, c1 = tr(Q^2)/2.
__device__ Mat<double> expi_herm(const Mat<double>& q) {
  const Mat<double> q2 = mm(q, q);
  const double c1 = 0.5 * (q2.m[0][0].re + q2.m[1][1].re + q2.m[2][2].re);
  Mat<double> out;
  if (c1 < 1e-36) {  // exp(iQ) = 1 + iQ - Q^2 / 2 + O(|Q|^3)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        out.m[a][b] = ti(q.m[a][b]) - 0.5 * q2.m[a][b];
        if (a == b) out.m[a][b].re += 1.0;
      }
    return out;
  }
  const Mat<double> q3 = mm(q2, q);
  const double c0 = (q3.m[0][0].re + q3.m[1][1].re + q3.m[2][2].re) / 3.0;
  const bool neg = c0 < 0.0;
  const double c0a = fabs(c0);
  const double c0max = 2.0 * pow(c1 / 3.0, 1.5);
  double ratio = c0a / c0max;
  ratio = ratio > 1.0 ? 1.0 : ratio;
  const double theta = acos(ratio);
  const double u = sqrt(c1 / 3.0) * cos(theta / 3.0);
  const double w = sqrt(c1) * sin(theta / 3.0);
  const double u2 = u * u, w2 = w * w;
  const double xi0 = fabs(w) < 0.05 ? 1.0 - w2 / 6.0 * (1.0 - w2 / 20.0 * (1.0 - w2 / 42.0)) : sin(w) / w;
  const double cw = cos(w);
  const Cx<double> e2iu = {cos(2.0 * u), sin(2.0 * u)}, emiu = {cos(u), -sin(u)};
  Cx<double> h0 = (u2 - w2) * e2iu + emiu * Cx<double>{8.0 * u2 * cw, 2.0 * u * (3.0 * u2 + w2) * xi0};
  Cx<double> h1 = (2.0 * u) * e2iu - emiu * Cx<double>{2.0 * u * cw, -(3.0 * u2 - w2) * xi0};
  Cx<double> h2 = e2iu - emiu * Cx<double>{cw, 3.0 * u * xi0};
  const double den = 1.0 / (9.0 * u2 - w2);
  Cx<double> f0 = den * h0, f1 = den * h1, f2 = den * h2;
  if (neg) {  // f_j(-c0) = (-1)^j conj(f_j(c0))
    f0 = conj(f0);
    f1 = -conj(f1);
    f2 = conj(f2);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      out.m[a][b] = f1 * q.m[a][b] + f2 * q2.m[a][b];
      if (a == b) out.m[a][b] = out.m[a][b] + f0;
    }
  return out;
}

// U_mu(x) <- exp(i c P_mu(x)) U_mu(x), P = sum_a P^a lambda^a / 2
__global__ void __launch_bounds__(128) link_exp_k(Geom g, double2* __restrict__ u18, const double* __restrict__ p_user,
                                                  double c) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * g.V) return;
  const int i = t >> 2, mu = t & 3;
  int x[4];
  lex_coords(i, g, x);
  const int par = parity_of(x), cb = i >> 1;
  double P[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) P[a] = 0.5 * c * p_user[(size_t)t * 8 + a];
  const double r3 = 0.57735026918962576451;
  Mat<double> q;
  q.m[0][0] = {P[2] + P[7] * r3, 0.0};
  q.m[1][1] = {-P[2] + P[7] * r3, 0.0};
  q.m[2][2] = {-2.0 * P[7] * r3, 0.0};
  q.m[0][1] = {P[0], -P[1]};
  q.m[1][0] = {P[0], P[1]};
  q.m[0][2] = {P[3], -P[4]};
  q.m[2][0] = {P[3], P[4]};
  q.m[1][2] = {P[5], -P[6]};
  q.m[2][1] = {P[5], P[6]};
  double2* base = u18 + (size_t)((mu * 2 + par) * 9) * g.stride;
  const Mat<double> U = load_mat(base, g.stride, cb);
  store_mat(base, g.stride, cb, mm(expi_herm(q), U));
}

hipError_t launch_link_exp(const Geom& g, double2* u18, const double* p_user, double c, hipStream_t s) {
  hipLaunchKernelGGL(link_exp_k, dim3(blocks_for(4 * g.V, 128)), dim3(128), 0, s, g, u18, p_user, c);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) mom_update_k(int n, double* __restrict__ p, const double* __restrict__ f,
                                                    double dt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  p[i] -= dt * f[i];
}
hipError_t launch_mom_update(const Geom& g, double* p_user, const double* f_user, double dt, hipStream_t s) {
  const int n = 32 * g.V;
  hipLaunchKernelGGL(mom_update_k, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, p_user, f_user, dt);
  return hipGetLastError();
}

}  // namespace qcd
