/*
 * cloverqcd -- even-odd Wilson-clover solver and fermion force for AMD
 * Instinct MI355X (gfx950).  C ABI.
 *
 * The computation is the hot path of the dynamical-clover-fermion HMD (R
 * algorithm) application that arXiv:0910.0262 ports to the Cell/B.E.
 * (abstract; section 1 names MILC's clover_dynamical / su3_rmd).  The paper
 * describes that application as a set of kernels, each taking site-local
 * fields, contiguous temporaries and neighbour-site fields and writing site
 * fields (section 3), called from the host as "set up, run, wait for
 * completion" (section 3).  The calls below follow that statement: load the
 * gauge field and the clover term, apply M or Mhat^dag Mhat, solve, compute
 * the force, take one molecular-dynamics step.  The paper prints no
 * equation; the definitions used are the textbook ones, stated at each call.
 *
 * Conventions (fixed for every call):
 *   dims = {Lx, Ly, Lz, Lt}, all even and >= 2; V = Lx Ly Lz Lt, Vh = V / 2.
 *   Site index i = x + Lx (y + Ly (z + Lz t)); parity (x + y + z + t) mod 2,
 *   0 = even.  Checkerboard index of site i within its parity is i / 2.
 *   Spinor: 4 spins x 3 colours, complex128, [site][spin][colour].
 *   Link U_mu(x): 3x3 complex128 [row][col], mu = 0..3 for x, y, z, t.
 *   Gamma matrices: chiral Euclidean basis, gamma_k = [[0, -i s_k], [i s_k, 0]],
 *   gamma_4 = [[0, 1], [1, 0]], gamma_5 = diag(1, 1, -1, -1).
 *   Hopping term
 *     (H psi)(x) = sum_mu eta [(1 - g_mu) U_mu(x) psi(x + mu)
 *                              + (1 + g_mu) U_mu(x - mu)^dag psi(x - mu)],
 *   eta = t_boundary on hops across the t boundary, 1 otherwise.
 *   Clover: Q_mu,nu = sum of the four counter-clockwise plaquettes at x,
 *   F = (Q - Q^dag)/(8i) made traceless,
 *   A = 1 - kappa c_sw sum_{mu<nu} sigma_mu,nu (x) F_mu,nu,
 *   sigma_mu,nu = (i/2)[g_mu, g_nu]; A is two Hermitian 6x6 blocks acting on
 *   spins {0,1} and {2,3}, index 3 s + c within a block.
 *   M = A - kappa H.  Even-odd Schur complement on even sites:
 *   Mhat = A_ee - kappa^2 H_eo A_oo^{-1} H_oe,  Mhat^dag = g5 Mhat g5.
 *
 * Memory: every pointer argument named *_dev is device memory on the
 * context's device, allocated and owned by the caller; the library never
 * keeps it past the call.  Host pointers (dims, params, stats, S) are read or
 * written during the call only.  The context owns its internal fields.
 *
 * Streams: all device work is enqueued on the stream given to qcd_create.
 * qcd_apply and the load calls are stream-ordered and return without waiting.
 * qcd_solve, qcd_action_force, qcd_hmd_step and the calls below them wait for their work before
 * returning, because they return host-visible results.
 *
 * Errors: every call returns a qcd_status.  Arguments are validated before
 * any device work is issued.  Nothing aborts or throws across the ABI.
 * qcd_last_error() returns a thread-local message for the last non-OK return.
 */
#ifndef CLOVERQCD_H
#define CLOVERQCD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qcd_ctx qcd_ctx;

typedef enum {
  QCD_OK = 0,
  QCD_EINVAL = -1,  /* invalid argument (shape, null pointer, non-finite parameter)   */
  QCD_ESTATE = -2,  /* call out of order (e.g. apply before a gauge field is loaded)   */
  QCD_ENOMEM = -3,  /* device allocation failed                                        */
  QCD_EHIP = -4,    /* a HIP runtime call failed                                       */
  QCD_ENOCONV = -5, /* solver hit max_iter; the last iterate and the stats are written */
  QCD_ENAN = -6,    /* a non-finite residual or norm appeared                          */
  QCD_ECLOVER = -7  /* a clover block is not positive definite; it cannot be inverted  */
} qcd_status;

typedef enum { QCD_FP64 = 0, QCD_MIXED = 1 } qcd_precision;

typedef enum {
  QCD_OP_M = 0,           /* full lattice: in, out [V][4][3]                        */
  QCD_OP_MDAG = 1,        /* full lattice M^dag = g5 M g5                           */
  QCD_OP_MHAT = 2,        /* even sites: in, out [Vh][4][3], checkerboard order     */
  QCD_OP_MHATDAG = 3,     /* even sites: Mhat^dag                                   */
  QCD_OP_MHATDAGMHAT = 4  /* even sites: Mhat^dag Mhat                              */
} qcd_operator;

typedef enum {
  QCD_OPT_LINK_RECON = 0,   /* FP64 stencil links: 12 (two rows stored, third rebuilt,
                               requires det U = 1; default) or 18 (full matrix)       */
  QCD_OPT_MIXED_CLOVER = 1, /* clover storage in the mixed solver: 16 = binary16 with a
                               per-block FP32 scale (default), 32 = FP32                */
  QCD_OPT_BLOCK = 2,        /* threads per workgroup of the stencil and reduction
                               kernels (64, 128, 192 or 256); 0 (default) = 64 for
                               single-source work, 256 for multi-source solves of 2 or
                               more right-hand sides.  The CG x/p update always runs
                               in 64-thread workgroups.                                 */
  QCD_OPT_GRAPH = 3,        /* 1: each CG iteration is replayed as a captured HIP graph;
                               0 (default): its kernels are launched one by one (graph
                               replay measured no faster on MI355X)                     */
  QCD_OPT_SMALL_GRID = 4,   /* single-source stencils on lattices of at most 2^17 sites
                               (fewer sites per checkerboard than SIMD lanes on the
                               chip), with 64-thread workgroups: 2 (default) = four
                               wavefronts per 64 sites (one direction each, partial
                               sums added in LDS), 1 = two wavefronts per 64 sites
                               (forward and backward hops split), 0 = one work-item per
                               site as on large lattices                                */
  QCD_OPT_MIXED_STALL = 5,  /* mixed CG fallback threshold k in [1, 60], default 1: the
                               FP64 |r|^2 recomputed at a reliable update must fall
                               below 2^-k of the best one so far; after three reliable
                               updates in a row without such a fall the mixed
                               recurrence stops and the solve finishes in FP64 CG from
                               the accumulated solution (stats.restarts counts it).
                               Large k forces the fallback, for testing it.             */
  QCD_OPT_COMPACT_CLOVER = 6, /* A_ee in the k2 stencils (the site term of the even-odd
                               operator, FP64 with 12-real links and binary16): 1
                               (default) = each chiral block as 1 - [[X3, W],
                               [W^dag, -X3]], X3 traceless Hermitian and W a 3x3
                               complex matrix (26 reals instead of 36), the form
                               every clover term built from links has; a loaded
                               clover term without it uses the general blocks.  0 =
                               general Hermitian blocks always                          */
  QCD_OPT_X_CYCLE = 7       /* CG iterations per update of the solution, n in [1, 4],
                               default 4: the search directions of n iterations are
                               kept (n buffers) and x += alpha_0 p_0 + ... +
                               alpha_{n-1} p_{n-1} is done once per n iterations, which
                               saves reading and writing x in the other n - 1; a
                               recurrence that stops or a reliable update inside a
                               cycle takes the directions it has so far.  The same
                               CG iterates up to rounding for every n.                  */
} qcd_option;

/* Library version, (major << 16) | minor. */
int qcd_version(void);

/* Create a context for one lattice on HIP device `device`; all work goes to
 * `hip_stream` (a hipStream_t cast to uintptr_t; 0 = the null stream).
 * dims: {Lx, Ly, Lz, Lt}, each even and >= 2, V / 2 (rounded up to a multiple
 * of 64) x 48 < 2^32, i.e. V up to about 1.79e8 (the kernels address a field
 * element with a 32-bit byte offset).
 * Defaults: kappa = 0.125, c_sw = 1, t_boundary = -1.  Returns QCD_EINVAL on
 * a bad shape, QCD_ENOMEM / QCD_EHIP if the device work buffers cannot be made. */
int qcd_create(const int dims[4], int device, uintptr_t hip_stream, qcd_ctx **out);

/* Free the context and everything it owns.  NULL is accepted. */
int qcd_destroy(qcd_ctx *ctx);

/* kappa > 0 and finite; c_sw finite; t_boundary = +1 (periodic) or -1
 * (antiperiodic) in time.  Space is always periodic.  Invalidates the clover
 * term: call qcd_build_clover (or qcd_load_clover) again before applying. */
int qcd_set_params(qcd_ctx *ctx, double kappa, double csw, int t_boundary);

/* Set a qcd_option (see the enum for the values each accepts). */
int qcd_set_option(qcd_ctx *ctx, int option, int value);

/* Load the gauge field U_dev: complex128 [V][4][3][3] (site, mu, row, col).
 * Packs it into the context's per-parity structure-of-arrays layouts
 * (FP64 18- and 12-real, binary16 12-real).  Invalidates the clover term. */
int qcd_load_gauge(qcd_ctx *ctx, const void *U_dev);

/* Copy the context's gauge field out to U_dev, complex128 [V][4][3][3]. */
int qcd_store_gauge(qcd_ctx *ctx, void *U_dev);

/* Build A on every site from the loaded links (clover leaves, field
 * strength, the two 6x6 blocks) and invert the odd-site blocks.
 * QCD_ECLOVER if an odd-site block is not positive definite. */
int qcd_build_clover(qcd_ctx *ctx);

/* Load A directly instead: A_dev is float64 [V][2][36]; per 6x6 Hermitian
 * block the 6 real diagonal entries, then the 15 upper off-diagonal entries
 * (i < j, row-major: (0,1) ... (0,5), (1,2) ... (4,5)) as (re, im) pairs.
 * The odd-site blocks are inverted on the device. */
int qcd_load_clover(qcd_ctx *ctx, const double *A_dev);

/* Read back A (every site) and A_oo^{-1} (odd sites, checkerboard order) in
 * the packed layout of qcd_load_clover: A_dev [V][2][36], Ainv_dev [Vh][2][36].
 * Either pointer may be NULL. */
int qcd_get_clover(qcd_ctx *ctx, double *A_dev, double *Ainv_dev);

/* out = op(in), op a qcd_operator.  prec = QCD_FP64, or QCD_MIXED for the
 * even-site operators: the input is encoded as binary16 with a per-site
 * scale, the stencil runs in FP32 on binary16 links, and the output is
 * decoded to complex128.  in_dev and out_dev must not overlap. */
int qcd_apply(qcd_ctx *ctx, int op, int prec, const void *in_dev, void *out_dev);

typedef struct {
  int prec;               /* qcd_precision                                            */
  int max_iter;           /* iteration cap (CG iterations, inner ones for QCD_MIXED)  */
  int pipeline_depth;     /* CG iterations kept in flight ahead of the host's check of
                             the oldest one (>= 1; 0 means 1); at most depth - 1
                             iterations are issued past convergence                  */
  double tol;             /* stop when ||r|| <= tol ||Mhat^dag bhat|| (FP64 residual) */
  double delta_reliable;  /* QCD_MIXED: reliable update when ||r|| < delta max||r||   */
} qcd_solver_params;

typedef struct {
  int iters;              /* CG iterations taken                                      */
  int reliable_updates;   /* FP64 residual recomputations (QCD_MIXED)                 */
  int converged;          /* 1 if the FP64 residual met tol                           */
  int restarts;           /* FP64 restarts after a residual check (or mixed fallback) */
  double normal_rel_res;  /* ||Mhat^dag bhat - Mhat^dag Mhat x_e|| / ||Mhat^dag bhat||  */
  double true_rel_res;    /* ||b - M x|| / ||b|| on the full lattice                  */
  double seconds;         /* wall time of the solve on the host clock                 */
  double flops;           /* 2 x 1824 x V per Mhat^dag Mhat, over all applications    */
  double bytes;           /* algorithmic bytes moved by the solve's kernels           */
} qcd_solver_stats;

/* Solve M x = b on the full lattice by even-odd preconditioning:
 * bhat = b_e + kappa H_eo A_oo^{-1} b_o; CG on Mhat^dag Mhat x_e = Mhat^dag bhat
 * from x_e = 0; x_o = A_oo^{-1} (b_o + kappa H_oe x_e).  b_dev, x_dev:
 * complex128 [V][4][3].  stats may be NULL.  QCD_ENOCONV writes the last
 * iterate; QCD_ENAN on a non-finite residual. */
int qcd_solve(qcd_ctx *ctx, const qcd_solver_params *params, const void *b_dev, void *x_dev,
              qcd_solver_stats *stats);

/* Largest number of right-hand sides of one qcd_solve_multi call. */
#define QCD_MAX_RHS 16

/* n_rhs independent solves M x_k = b_k (k < n_rhs <= QCD_MAX_RHS) with the
 * operator loaded in the context, each exactly as qcd_solve (same stopping
 * test, reliable updates and final FP64 residual), run together: the
 * right-hand sides are interleaved site by site in the library's fields, so
 * each link and clover block is read once per site for all of them.  This
 * is the multi-source workload of the paper's application (section 1), whose
 * kernels are bound by memory bandwidth (section 4).  Internally n_rhs is
 * rounded up to a power of two with zero right-hand sides, which converge at
 * once.  b_dev, x_dev: complex128 [n_rhs][V][4][3], not overlapping.  stats:
 * NULL or n_rhs entries; iters and reliable_updates count the joint
 * iterations (the largest over the right-hand sides), seconds the whole call,
 * flops each right-hand side's share, bytes the call's algorithmic bytes over
 * n_rhs.  The first call with a given n_rhs allocates the interleaved work
 * vectors (about 12 x n_rhs' spinor fields, n_rhs' = the rounded count); they
 * are kept for later calls with as many or fewer right-hand sides.
 * QCD_EINVAL if V/2 (rounded up to a multiple of 64) x n_rhs' x 48 reaches
 * 2^32 (the kernels address a field element with a 32-bit byte offset).  QCD_ENOCONV if any right-hand side
 * missed tol (all x are written). */
int qcd_solve_multi(qcd_ctx *ctx, const qcd_solver_params *params, int n_rhs, const void *b_dev, void *x_dev,
                    qcd_solver_stats *stats);

/* Pseudofermion action and its gauge derivative.
 * S = phi^dag (Mhat^dag Mhat)^{-1} phi with phi_dev complex128 [Vh][4][3] on
 * even sites.  Writes *S; G_dev (complex128 [V][4][3][3]) receives
 * dS/dRe(U) + i dS/dIm(U) per element (so dS = Re sum conj(G) dU); F_dev
 * (float64 [V][4][8], may be NULL) receives the su(3) force
 * F^a = dS/dw^a for U -> exp(i w^a T^a) U, T^a = lambda^a / 2 (Gell-Mann);
 * X_dev (complex128 [Vh][4][3], may be NULL) receives the solution
 * X = (Mhat^dag Mhat)^{-1} phi.  The clover determinant is not part of S. */
int qcd_action_force(qcd_ctx *ctx, const qcd_solver_params *params, const void *phi_dev, double *S,
                     void *G_dev, double *F_dev, void *X_dev, qcd_solver_stats *stats);

/* One HMD step of the R algorithm at two flavours, fermion action only.
 * With two flavours per pseudofermion field the R algorithm (Gottlieb, Liu,
 * Toussaint, Renken, Sugar, Phys. Rev. D 35 (1987) 2531) draws the noise at
 * the start of the step, so the step is a heat-bath of phi followed by one
 * leapfrog step at fixed phi:
 *   phi = Mhat^dag(U) xi;  U_1/2 = exp(i dt/2 P) U;
 *   P <- P - dt F(U_1/2, phi);  U <- exp(i dt/2 P) U_1/2.
 * U_dev: complex128 [V][4][3][3], in/out (also reloaded into the context).
 * P_dev: float64 [V][4][8] generator coefficients, in/out.
 * xi_dev: complex128 [Vh][4][3] on even sites.  S (may be NULL) receives the
 * action at U_1/2; stats (may be NULL) the inner solve's stats. */
int qcd_hmd_step(qcd_ctx *ctx, double dt, void *U_dev, double *P_dev, const void *xi_dev,
                 const qcd_solver_params *params, double *S, qcd_solver_stats *stats);

/* Wilson gauge action on the loaded gauge field,
 *   S_g = beta sum_{x, mu<nu} (1 - Re tr U_mu,nu(x) / 3),
 *   U_mu,nu(x) = U_mu(x) U_nu(x + mu) U_mu(x + nu)^dag U_nu(x)^dag,
 * and its derivative in the conventions of qcd_action_force: G_dev
 * (complex128 [V][4][3][3]) and F_dev (float64 [V][4][8]), each may be NULL;
 * S may be NULL.  The R-algorithm application of the paper evolves the gauge
 * field under gauge and fermion forces together (section 1); the paper
 * prints no gauge action, so this is the standard plaquette action.  Waits
 * for its work.  QCD_ESTATE without a gauge field, QCD_EINVAL for a
 * non-finite beta. */
int qcd_gauge_action_force(qcd_ctx *ctx, double beta, double *S, void *G_dev, double *F_dev);

/* Allocation-free variant of qcd_gauge_action_force, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the derivative of the Wilson gauge action
 * on the loaded gauge field, G_dev (complex128 [V][4][3][3]) and F_dev
 * (float64 [V][4][8]) as in qcd_gauge_action_force, each may be NULL but not
 * both; the action itself is not computed (it needs a host synchronisation).
 * It calls no allocator: the force accumulator lives in a fixed 64 MiB
 * device array of the library, one per GPU, so the lattice is limited to
 * V <= 116480 sites (QCD_EINVAL beyond, before any device work; 16^4 and
 * 8x8x16x16 fit, 32^3x64 does not).  Stream-ordered: returns once the two
 * kernels are enqueued on the context's stream, without waiting.  Every call
 * on one GPU uses the same array: calls that overlap on one GPU (contexts on
 * different streams) race; calls on one stream are ordered.  The accumulator
 * is fully overwritten by each call, so no clearing is needed.  QCD_ESTATE
 * without a gauge field, QCD_EINVAL for a non-finite beta. */
int qcd_gauge_force_noalloc(qcd_ctx *ctx, double beta, void *G_dev, double *F_dev);

/* Clover determinant on odd sites, S_det = -2 sum_{x odd} ln det A(x): the
 * factor (det A_oo)^2 of det(M^dag M) = (det A_oo)^2 det(Mhat^dag Mhat) that
 * the even-site pseudofermion does not cover (two flavours).  ln det A comes
 * from the Cholesky pivots of the last qcd_build_clover / qcd_load_clover;
 * the derivative (G_dev, F_dev as in qcd_gauge_action_force, may be NULL)
 * is that of the clover term built from the loaded links (zero for
 * c_sw = 0).  Waits for its work.  QCD_ESTATE without a clover term. */
int qcd_clover_det_action_force(qcd_ctx *ctx, double *S, void *G_dev, double *F_dev);

typedef struct {
  double dt;        /* leapfrog step                                                  */
  double beta;      /* Wilson gauge coupling; 0 drops the gauge action                */
  double n_f;       /* flavours (>= 0): fermion and determinant forces weigh n_f / 2  */
  int n_steps;      /* >= 1; one noise vector per step                                */
  int clover_det;   /* 1: include S_det = -2 sum_odd ln det A; 0: leave it out       */
  int reunitarize;  /* 1: project the links back to SU(3) after every step            */
} qcd_md_params;

/* One trajectory of the R algorithm for n_f flavours (Gottlieb, Liu,
 * Toussaint, Renken, Sugar, Phys. Rev. D 35 (1987) 2531; the update the
 * paper's application runs, section 1): n_steps leapfrog steps, each
 *   U <- exp(i (1 - n_f/2) dt/2 P) U;   phi = Mhat^dag(U) xi_k;
 *   U <- exp(i (n_f/2) dt/2 P) U;
 *   P <- P - dt [(n_f/2) (F_f(U, phi) + F_det(U)) + F_g(U)];
 *   U <- exp(i dt/2 P) U                (then Gram-Schmidt back to SU(3)
 *                                         if reunitarize: row 0 normalised,
 *                                         row 1 orthogonalised and
 *                                         normalised, row 2 = conj(r0 x r1)),
 * with F_f the force of qcd_action_force, F_det that of
 * qcd_clover_det_action_force and F_g that of qcd_gauge_action_force.  The
 * noise is drawn (n_f/2) dt/2 before the force point, which cancels the
 * O(dt) heating of the noisy force; at n_f = 2 that is the start of the step
 * (the step of qcd_hmd_step plus the gauge and determinant forces), for
 * n_f > 2 the links first move back in time; at n_f = 0 the fermion field
 * drops out (params and xi_dev are then not read).
 * U_dev: complex128 [V][4][3][3], in/out.  P_dev: float64 [V][4][8], in/out.
 * xi_dev: complex128 [n_steps][Vh][4][3] on even sites.  actions (host, may
 * be NULL): float64 [n_steps][3] receives (S_f, S_g, S_det) at each step's
 * force evaluation, unweighted.  stats (may be NULL): the sum over the
 * step's solves; seconds of the whole trajectory.  Waits for its work.  On
 * return the context holds the final U (and for n_f > 0 its clover term).
 * QCD_ENOCONV if any solve missed tol (the trajectory still completes). */
int qcd_md_trajectory(qcd_ctx *ctx, const qcd_md_params *md, void *U_dev, double *P_dev, const void *xi_dev,
                      const qcd_solver_params *params, double *actions, qcd_solver_stats *stats);

/* Reference encoder of the mixed solver's spinor storage, for checking:
 * in_dev complex128 [n][4][3] -> codes_dev binary16 [n][24] (re, im
 * interleaved, spin-major), scale_dev float32 [n]; scale = max |component|,
 * code = binary16_rn(float32(component) * (1 / scale)), 0 when scale = 0. */
int qcd_encode_half(qcd_ctx *ctx, int n, const void *in_dev, void *codes_dev, float *scale_dev);

/* Stencil timing on the context's loaded fields and its current work
 * vectors, for prec = QCD_FP64 or QCD_MIXED: n (1..4096) applications of
 * Mhat^dag Mhat (k1, k2, k1^dag, k2^dag, as inside the solver) with a HIP
 * event on the context's stream before and after every launch, then n more
 * launched back to back between two events.  ms[0]: average launch of
 * k1 = A_oo^{-1} H_oe psi_e (the first of the four); ms[1]: of
 * k2 = A_ee psi_e - kappa^2 H_eo t_o (the second); ms[2]: one
 * Mhat^dag Mhat from the back-to-back run.  Milliseconds; waits for the
 * work.  The vectors' contents are whatever the last operator call left
 * (timing does not depend on them). */
int qcd_time_stencil(qcd_ctx *ctx, int prec, int n, double ms[3]);

/* As qcd_time_stencil for n_rhs (1..QCD_MAX_RHS) right-hand sides
 * interleaved as in qcd_solve_multi: each launch processes all of them (one
 * work-item per site and right-hand side, links and clover read once per
 * site).  Uses (and on first use allocates) the multi-source work vectors;
 * their contents are whatever the last multi-source call left, zero before. */
int qcd_time_stencil_multi(qcd_ctx *ctx, int prec, int n_rhs, int n, double ms[3]);

/* Plain device copy of n_bytes (multiple of 16, 16-byte aligned pointers),
 * a bandwidth calibration kernel on the context's stream. */
int qcd_stream_copy(qcd_ctx *ctx, void *dst_dev, const void *src_dev, uint64_t n_bytes);

/* Thread-local message describing the last non-OK return ("" if none). */
const char *qcd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CLOVERQCD_H */
