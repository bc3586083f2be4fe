// Internal interface between the C-ABI host code (api.hip) and the kernel
// translation units: the on-device solver state, field references and the
// launch functions.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qcd_device.h"

namespace qcd {

// Scalars of the CG recurrence, resident in device memory so that alpha and
// beta never travel to the host.  Kernels of an iteration return at once
// when `halt` is set (converged or non-finite), which lets the host keep a
// few iterations in flight and stop the recurrence without a round trip.
struct CgState {
  double rr;       // |r_k|^2 of the current recurrence residual
  double qq;       // |Mhat p|^2
  double alpha, beta;
  double stop2;    // tol^2 |rhs|^2
  double maxrr;    // max |r|^2 since the last reliable update
  double delta2;   // delta_reliable^2
  double rr_hi;    // last FP64 residual norm^2
  double scalar;   // generic reduction result (dot products, norms)
  double ah[4];    // the last four alphas, newest first (x takes alpha_k p_k a few iterations late)
  int iter, max_iter;
  int halt, done, need_ru, nan, do_x, do_p, mixed, ru_count;
  int post_seq;    // number of states posted so far; the next goes to mailbox[post_seq % ring]
};

// ---- CG state updates, shared by the one-workgroup finalisation kernels and
// the stencil kernels that finish their own reduction (one thread runs them).
__device__ __forceinline__ bool finite(double v) { return v == v && v - v == 0.0; }

// Copy the state to mailbox[post_seq % ring] (host-mapped memory the host
// reads once the iteration's event has completed) and advance post_seq; the
// host counts the posting launches it issues, so it knows each slot.
__device__ __forceinline__ void post(CgState* st, CgState* mbox, int ring) {
  const int slot = st->post_seq % ring;
  st->post_seq = (st->post_seq + 1) % (ring * 1024);
  mbox[slot] = *st;
  __threadfence_system();
}

// alpha = |r|^2 / |Mhat p|^2, also shifted into the alpha history
__device__ __forceinline__ void state_alpha(CgState* st, double qq) {
  st->qq = qq;
  st->ah[3] = st->ah[2];
  st->ah[2] = st->ah[1];
  st->ah[1] = st->ah[0];
  if (!(qq > 0.0) || !finite(qq)) {
    st->nan = 1;
    st->done = 1;
    st->halt = 1;
    st->alpha = 0.0;
    st->ah[0] = 0.0;
    return;
  }
  st->alpha = st->rr / qq;
  st->ah[0] = st->alpha;
}

// End of an iteration: |r_{k+1}|^2, beta, the stopping test (FP64) or the
// reliable-update request (mixed; it does not stop the recurrence).  Posts.
__device__ __forceinline__ void state_beta(CgState* st, double rr_new, CgState* mbox, int ring) {
  st->iter += 1;
  if (!finite(rr_new)) {
    st->nan = 1;
    st->done = 1;
    st->halt = 1;
    st->do_x = 0;
    st->do_p = 0;
    post(st, mbox, ring);
    return;
  }
  st->beta = rr_new / st->rr;
  st->rr = rr_new;
  st->do_x = 1;
  if (!st->mixed) {
    st->done = (rr_new <= st->stop2 || st->iter >= st->max_iter) ? 1 : 0;
    st->halt = st->done;
    st->do_p = !st->done;
  } else {
    if (rr_new > st->maxrr) st->maxrr = rr_new;
    if (rr_new <= st->stop2 || rr_new < st->delta2 * st->maxrr || st->iter >= st->max_iter) st->need_ru = 1;
    st->do_p = 1;
  }
  post(st, mbox, ring);
}

// The iteration was already stopped: nothing to update, but the host still
// expects one posted state per iteration.
__device__ __forceinline__ void state_halted(CgState* st, CgState* mbox, int ring) {
  st->do_x = 0;
  st->do_p = 0;
  post(st, mbox, ring);
}

enum SpKind { SP_NONE = 0, SP_F64 = 1, SP_F32 = 2, SP_H = 3 };
struct SpRef {
  int kind;
  void* p;
  float* s;  // per-site scale (SP_H)
};
enum LinkKind { LK_F64_18 = 0, LK_F64_12 = 1, LK_H12 = 2, LK_H18 = 3 };
enum ClovKind { CL_NONE = 0, CL_F64 = 1, CL_F32 = 2, CL_H = 3, CL_F64C = 4, CL_HC = 5 };  // C: compact A_ee
struct ClovRef {
  int kind;
  const void* p;
  const float2* s;
};

// out(x) = [post ? C(x) : 1] ( [site term] + c * g5^g5out H g5^g5in in )(x)
// on every site x of parity par_out, where the site term is 0, s(x), or A(x) s(x),
// followed by an epilogue: 0 store; 1 store and |out|^2 partials;
// 2 dst = y + a out (a = -alpha from the state if a_from_state), store dst
// into `out`, |dst|^2 partials.
struct DslashOp {
  int par_out;
  SpRef in, site, out, y;
  int link_kind;
  const void* links;
  ClovRef cpre, cpost;
  double c;
  int site_mode;  // 0 none, 1 plain, 2 multiplied by cpre
  int post;
  int epi;
  double a;
  int a_from_state;
  int g5in, g5out;
  const CgState* st;
  double* partial;
  // Several right-hand sides interleaved site by site: spinor element v =
  // (cb << lg) | r holds right-hand side r of checkerboard site cb; links and
  // clover are indexed by cb and shared.  st then points at 1 << lg states
  // and the partial sums of right-hand side r start at partial[r * blocks].
  int lg;
  // single-source kernel on small lattices: 0 one work-item per site, 1 two
  // wavefronts per 64 sites, 2 four
  int small_grid;
  // fin_nr > 0: before its stencil work, workgroup r < fin_nr of the launch
  // finishes alpha for right-hand side r, exactly as the finalisation kernel
  // would (fin_st[r], the fin_n partials at fin_partial + r * fin_n); the
  // launch must not itself read alpha
  CgState* fin_st;
  const double* fin_partial;
  int fin_n, fin_nr;
};

inline int blocks_for(int n, int block) { return (n + block - 1) / block; }

// ---- dslash.hip
hipError_t launch_dslash(const Geom& g, const DslashOp& op, int block, hipStream_t s);
hipError_t launch_clover_apply(const Geom& g, int lg, SpF64 in, SpF64 out, const double2* clov, hipStream_t s);

// ---- blas.hip
hipError_t launch_pack_spinor_full(const Geom& g, const double2* user, SpF64 e, SpF64 o, hipStream_t s);
hipError_t launch_unpack_spinor_full(const Geom& g, SpF64 e, SpF64 o, double2* user, hipStream_t s);
hipError_t launch_pack_spinor_cb(const Geom& g, const double2* user, SpF64 f, hipStream_t s);
hipError_t launch_unpack_spinor_cb(const Geom& g, SpF64 f, double2* user, hipStream_t s);
// n right-hand sides, caller layout [n][V][4][3] complex128, into the
// interleaved even / odd fields (rhs slots n .. (1 << lg) - 1 are zero)
hipError_t launch_pack_spinor_multi(const Geom& g, int lg, int n, const double2* user, SpF64 e, SpF64 o,
                                    hipStream_t s);
hipError_t launch_unpack_spinor_multi(const Geom& g, int lg, int n, SpF64 e, SpF64 o, double2* user, hipStream_t s);
hipError_t launch_pack_gauge(const Geom& g, const double2* user, double2* u18, hipStream_t s);
hipError_t launch_unpack_gauge(const Geom& g, const double2* u18, double2* user, hipStream_t s);
// u12: FP64 rows 0, 1; uh: binary16 rows 0, 1; uh18: all nine binary16 entries
// (16 * stride uint4 chunks followed by 8 * stride 32-bit chunks)
hipError_t launch_derive_links(const Geom& g, const double2* u18, double2* u12, uint2* uh, uint4* uh18,
                               hipStream_t s);
hipError_t launch_pack_clover(const Geom& g, const double2* user, double2* clov, hipStream_t s);
hipError_t launch_unpack_clover(const Geom& g, const double2* clov, double2* user, int n_par, int par0,
                                hipStream_t s);
// Spinor BLAS: gv is the geometry with Vh and stride scaled by the number of
// right-hand sides (1 << lg); per-rhs states and segmented partial sums.
hipError_t launch_norm2(const Geom& gv, int lg, SpRef x, double* partial, int block, hipStream_t s);
hipError_t launch_dot_re(const Geom& gv, int lg, SpF64 a, SpF64 b, double* partial, int block, hipStream_t s);
// Finalisation kernels: one workgroup per right-hand side (nr of them), each
// summing its n partials and updating its own state.  With kFoldMin or more
// partials per right-hand side they are first folded, by one workgroup per
// span of kFoldSpan and right-hand side, into fold[r * nf + f] (nf spans per
// right-hand side; fold holds nr * nf doubles), which the finalisation kernel
// then sums: one workgroup alone cannot keep enough loads in flight.
constexpr int kFoldSpan = 4096;
constexpr int kFoldMin = 32768;
hipError_t launch_fin_scalar(CgState* st, const double* partial, int n, int nr, double* fold, hipStream_t s);
hipError_t launch_fin_init(CgState* st, const double* partial, int n, int nr, double* fold, double tol, double delta,
                           int max_iter, int mixed, CgState* mbox, int ring, hipStream_t s);
hipError_t launch_fin_alpha(CgState* st, const double* partial, int n, int nr, double* fold, hipStream_t s);
hipError_t launch_fin_beta(CgState* st, const double* partial, int n, int nr, double* fold, CgState* mbox, int ring,
                           hipStream_t s);
hipError_t launch_fin_ru(CgState* st, const double* partial, int n, int nr, double* fold, int restart, int nclear,
                         CgState* mbox, int ring, hipStream_t s);
// Iteration j of an n-iteration x cycle; p[0 .. n-1] are the cycle's direction buffers.
hipError_t launch_xp_update_f64(const Geom& gv, int lg, const CgState* st, SpF64 x, const SpF64* p, int j, int n,
                                SpF64 r, int block, hipStream_t s);
hipError_t launch_xp_update_h(const Geom& gv, int lg, const CgState* st, SpF32 x, const SpH* p, int j, int n, SpH r,
                              int block, hipStream_t s);
hipError_t launch_p_restart_f64(const Geom& gv, int lg, const CgState* st, SpF64 p, SpF64 r, int block,
                                hipStream_t s);
// x_hi += x_lo + the first q directions p[0 .. q-1] of the unfinished cycle; x_lo = 0
hipError_t launch_ru_accum(const Geom& gv, int lg, const CgState* st, SpF64 xhi, SpF32 xlo, const SpH* p, int q,
                           int block, hipStream_t s);
hipError_t launch_convert(const Geom& g, SpRef src, SpRef dst, int block, hipStream_t s);
hipError_t launch_zero(const Geom& g, SpRef x, int block, hipStream_t s);
hipError_t launch_encode_half(int n, const double2* user, uint4* codes, float* scale, hipStream_t s);
hipError_t launch_stream_copy(const uint4* src, uint4* dst, uint64_t n16, hipStream_t s);

// ---- clover.hip
hipError_t launch_clover_build(const Geom& g, const double2* u18, double kappa, double csw, double2* clov,
                               hipStream_t s);
hipError_t launch_clover_compact(const Geom& g, const double2* clov_e, double2* c64, uint4* ch, float2* chs,
                                 int* status, hipStream_t s);
hipError_t launch_clover_invert(const Geom& g, const double2* clov, double2* clov_inv, float4* clov32_e,
                                float4* clovinv32_o, uint4* clovh_e, float2* clovh_es, uint4* clovinvh_o,
                                float2* clovinvh_os, double* logdet, int* status, hipStream_t s);

// ---- force.hip
hipError_t launch_force_hop(const Geom& g, const double2* u18, SpF64 ell_e, SpF64 ell_o, SpF64 rho_e,
                            SpF64 rho_o, double coef, double2* gint, hipStream_t s);
// ell_e.p == nullptr drops the fermion term; cinv == nullptr the determinant term
hipError_t launch_clover_xi(const Geom& g, SpF64 ell_e, SpF64 ell_o, SpF64 rho_e, SpF64 rho_o, double w_e,
                            double w_o, const double2* cinv, double w_det, double2* xi, hipStream_t s);
// coef_g != 0 adds the Wilson gauge force (weight coef_g, as launch_gauge_force) in the same pass
hipError_t launch_force_clover(const Geom& g, const double2* u18, const double2* xi, double coef, double2* gint,
                               hipStream_t s, double coef_g = 0.0);
hipError_t launch_force_out(const Geom& g, const double2* u18, const double2* gint, double2* g_user,
                            double* f_user, hipStream_t s);
hipError_t launch_gauge_force(const Geom& g, const double2* u18, double coef, int accumulate, double2* gint,
                              hipStream_t s);
hipError_t launch_plaquette(const Geom& g, const double2* u18, double* partial, int block, hipStream_t s);
hipError_t launch_sum_cb(const Geom& g, const double* v, double* partial, int block, hipStream_t s);
hipError_t launch_force_zero(const Geom& g, double2* gint, hipStream_t s);
hipError_t launch_reunitarize(const Geom& g, double2* u18, hipStream_t s);
hipError_t launch_link_exp(const Geom& g, double2* u18, const double* p_user, double c, hipStream_t s);
hipError_t launch_mom_update(const Geom& g, double* p_user, const double* f_user, double dt, hipStream_t s);

}  // namespace qcd
