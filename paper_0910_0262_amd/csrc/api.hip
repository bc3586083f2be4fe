// C-ABI entry points, context management and the solver drivers.
//
// The drivers enqueue kernels on the context's stream and keep every scalar
// of the CG recurrence on the device (CgState).  The host keeps a few
// iterations in flight and reads each iteration's posted state once it has
// completed; kernels of iterations issued past convergence return at once.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "cloverqcd.h"
#include "qcd_internal.h"

// Fixed device scratch of the allocation-free entry point
// (qcd_gauge_force_noalloc): the gauge-force accumulator [mu][parity][9][Vh]
// of a lattice of at most kScratchVh checkerboard sites.  Each GPU the
// library runs on holds its own copy from module load to process end; every
// call on that GPU shares it.  Host code never passes `scratch` itself to a
// kernel (that is a host-side stand-in); it uses the per-device address
// hipGetSymbolAddress returns.
static constexpr size_t kScratchBytes = (size_t)64 << 20;
static constexpr size_t kScratchVh = kScratchBytes / (8 * 9 * sizeof(double2));
static __device__ __align__(256) double2 scratch[kScratchBytes / sizeof(double2)];

using namespace qcd;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) return fail(QCD_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define QCHK(call)         \
  do {                     \
    int s_ = (call);       \
    if (s_ != QCD_OK) return s_; \
  } while (0)

// FP64 work vectors (one checkerboard each)
// (V_P, V_P1, V_P2, V_P3 and H_P .. H_P3: the search directions of one x cycle, see the CG vector updates)
enum Slot { V_IN_E, V_IN_O, V_OUT_E, V_OUT_O, V_T, V_Q, V_X, V_R, V_P, V_RHS, V_B_E, V_B_O, V_AUX, V_Y, V_W, V_Z,
            V_P1, V_P2, V_P3, NSLOT };
// binary16 work vectors
enum HSlot { H_P, H_T, H_Q, H_R, H_IN, H_OUT, H_P1, H_P2, H_P3, NHSLOT };
// ring of mailbox slots / events for the iterations in flight
constexpr int kRing = 64;

}  // namespace

// Solver work set: vectors, partial sums and CG states for nr = 1 << lg
// right-hand sides interleaved site by site (element (cb << lg) | r).  The
// context's single-source set (lg = 0) also serves the operators, the force
// and the trajectory; a second set is allocated for multi-source solves.
struct Work {
  int lg = 0, nr = 1;
  Geom gv;  // Vh and stride of all right-hand sides together (for the BLAS kernels)
  double2* vec[NSLOT] = {};
  uint4* hv[NHSLOT] = {};
  float* hs[NHSLOT] = {};
  float4* x32 = nullptr;
  double* partial = nullptr;
  CgState* st = nullptr;         // nr states
  CgState* st_host = nullptr;    // pinned copy of the last states read (nr)
  CgState* mbox_host = nullptr;  // host-mapped rings of posted states: [nr][kRing]
  CgState* mbox_dev = nullptr;   // device address of mbox_host
  int post_ctr = 0;              // host mirror of CgState::post_seq (equal for all nr states)
};

struct qcd_ctx {
  int dims[4];
  Geom g;
  int device;
  hipStream_t stream;
  double kappa = 0.125, csw = 1.0;
  int tb = -1;
  int link_recon = 12;
  int mixed_clover = 16;
  int use_graph = 0;
  int small_grid = 2;
  int block_opt = 0;
  int stall_log2 = 1;  // mixed CG: a reliable update must take |r|^2 below 2^-stall_log2 of its best
  int x_defer = 4;     // CG: iterations per x update (QCD_OPT_X_CYCLE)
  bool gauge_loaded = false;
  bool clover_ready = false;

  double2* u18 = nullptr;
  double2* u12 = nullptr;
  uint2* uh = nullptr;
  uint4* uh18 = nullptr;        // all nine entries in binary16, for the multi-source kernels
  double2* clov = nullptr;      // A, both parities: [par][36][stride]
  double2* clov_inv = nullptr;  // A_oo^{-1}: [36][stride]
  float4* clov32_e = nullptr;   // A_ee in FP32
  float4* clovinv32_o = nullptr;
  uint4* clovh_e = nullptr;     // A_ee in binary16 + scale
  float2* clovh_es = nullptr;
  uint4* clovinvh_o = nullptr;
  float2* clovinvh_os = nullptr;
  // compact A_ee (1 - [[X3, W], [W^dag, -X3]] per chiral block, 26 reals):
  // valid when the clover term has that form (built from links)
  double2* clovc_e = nullptr;   // FP64: [26][stride] double2
  uint4* clovhc_e = nullptr;    // binary16: 6 chunks of uint4 then one of uint2, [stride] each
  float2* clovhc_es = nullptr;
  bool compact_ok = false;
  int compact_clover = 1;       // QCD_OPT_COMPACT_CLOVER
  Work w1;          // single source (operators, solve, force, trajectory)
  Work wm;          // multi-source solves
  Work* w = &w1;    // the set the solver drivers use
  int wm_lg_alloc = -1;  // right-hand sides (log2) wm was allocated for
  hipEvent_t ev[kRing] = {};
  hipStream_t cap = nullptr;    // private stream used only to capture graphs
  hipGraphExec_t iter_graph[2][4] = {};  // one CG iteration: [FP64, mixed][position in the x cycle]
  int* status = nullptr;
  int* status_host = nullptr;  // pinned
  double2* xi = nullptr;       // clover-force Xi: [par][6][9][stride]
  double2* gint = nullptr;     // force accumulator: [mu][par][9][stride]
  double* fbuf = nullptr;      // su(3) force [V][4][8] for the HMD step
  double* logdet = nullptr;    // ln det A(x) per odd site, from the last clover inversion

  // Workgroup size of the stencils and reductions, measured: 64 threads for
  // single-source work; 256 for the multi-source set, where FP64 solves are
  // about 1 % faster than at 64 and mixed ones equal (the x/p update keeps
  // 64 threads, kXpBlock).
  int block() const { return block_opt ? block_opt : (w->nr > 1 ? 256 : 64); }
  SpF64 f64(int s) const { return SpF64{w->vec[s], w->gv.stride}; }
  SpRef ref64(int s) const { return SpRef{SP_F64, w->vec[s], nullptr}; }
  SpRef refh(int s) const { return SpRef{SP_H, w->hv[s], w->hs[s]}; }
  SpH h(int s) const { return SpH{w->hv[s], w->hs[s], w->gv.stride}; }
  // slot of the j-th search direction of the x cycle
  static int pslot(int j) { return j == 0 ? V_P : V_P1 + j - 1; }
  static int hpslot(int j) { return j == 0 ? H_P : H_P1 + j - 1; }
  SpF32 f32() const { return SpF32{w->x32, w->gv.stride}; }
  const void* links64() const { return link_recon == 12 ? (const void*)u12 : (const void*)u18; }
  int lk64() const { return link_recon == 12 ? LK_F64_12 : LK_F64_18; }
  const double2* clov_par(int par) const { return clov + (size_t)par * 36 * g.stride; }
};

namespace {

template <class T>
int dalloc(T** p, size_t bytes) {
  if (hipMalloc((void**)p, bytes) != hipSuccess) {
    *p = nullptr;
    return fail(QCD_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return QCD_OK;
}

void free_work(Work& w) {
  auto f = [](void* p) {
    if (p) (void)hipFree(p);
  };
  for (auto*& p : w.vec) f(p), p = nullptr;
  for (auto*& p : w.hv) f(p), p = nullptr;
  for (auto*& p : w.hs) f(p), p = nullptr;
  f(w.x32);
  f(w.partial);
  f(w.st);
  if (w.st_host) (void)hipHostFree(w.st_host);
  if (w.mbox_host) (void)hipHostFree(w.mbox_host);
  w = Work();
}

// Allocate a work set for 1 << lg right-hand sides; with all_slots the
// vectors of the operators and the force too, otherwise the solver's only.
int alloc_work(const Geom& g, Work& w, int lg, bool all_slots) {
  w.lg = lg;
  w.nr = 1 << lg;
  w.gv = g;
  w.gv.Vh = g.Vh << lg;
  w.gv.stride = g.stride << lg;
  const size_t S = (size_t)w.gv.stride;
  int rc = QCD_OK;
  auto A = [&](auto** p, size_t bytes) {
    if (rc == QCD_OK) rc = dalloc(p, bytes);
  };
  static const int solver_slots[] = {V_T, V_Q, V_X, V_R, V_P, V_RHS, V_B_E, V_B_O, V_AUX, V_OUT_O, V_P1, V_P2, V_P3};
  static const int solver_hslots[] = {H_P, H_T, H_Q, H_R, H_P1, H_P2, H_P3};
  if (all_slots) {
    for (int k = 0; k < NSLOT; ++k) A(&w.vec[k], 12 * S * sizeof(double2));
    for (int k = 0; k < NHSLOT; ++k) {
      A(&w.hv[k], 3 * S * sizeof(uint4));
      A(&w.hs[k], S * sizeof(float));
    }
  } else {
    for (int k : solver_slots) A(&w.vec[k], 12 * S * sizeof(double2));
    for (int k : solver_hslots) {
      A(&w.hv[k], 3 * S * sizeof(uint4));
      A(&w.hs[k], S * sizeof(float));
    }
  }
  A(&w.x32, 6 * S * sizeof(float4));
  // partial sums: one per workgroup of 64 threads (the smallest block) per
  // right-hand side, then room for their folded span sums
  const size_t nb64 = blocks_for(w.gv.Vh, 64);
  A(&w.partial, (nb64 + 64 + nb64 / kFoldSpan + 1) * w.nr * sizeof(double));
  A(&w.st, w.nr * sizeof(CgState));
  if (rc == QCD_OK && hipHostMalloc((void**)&w.st_host, w.nr * sizeof(CgState), hipHostMallocDefault) != hipSuccess)
    rc = fail(QCD_ENOMEM, "pinned host allocation failed");
  if (rc == QCD_OK && hipHostMalloc((void**)&w.mbox_host, (size_t)w.nr * kRing * sizeof(CgState),
                                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
    rc = fail(QCD_ENOMEM, "pinned host allocation failed");
  if (rc == QCD_OK && hipHostGetDevicePointer((void**)&w.mbox_dev, w.mbox_host, 0) != hipSuccess)
    rc = fail(QCD_EHIP, "hipHostGetDevicePointer failed");
  if (rc == QCD_OK && hipMemset(w.st, 0, w.nr * sizeof(CgState)) != hipSuccess) rc = fail(QCD_EHIP, "hipMemset failed");
  // defined contents for timing calls made before any solve
  for (int k = 0; k < NSLOT && rc == QCD_OK; ++k)
    if (w.vec[k] && hipMemset(w.vec[k], 0, 12 * S * sizeof(double2)) != hipSuccess) rc = fail(QCD_EHIP, "hipMemset failed");
  for (int k = 0; k < NHSLOT && rc == QCD_OK; ++k)
    if (w.hv[k] && (hipMemset(w.hv[k], 0, 3 * S * sizeof(uint4)) != hipSuccess ||
                    hipMemset(w.hs[k], 0, S * sizeof(float)) != hipSuccess))
      rc = fail(QCD_EHIP, "hipMemset failed");
  if (rc != QCD_OK) {
    free_work(w);
    return rc;
  }
  std::memset(w.st_host, 0, w.nr * sizeof(CgState));
  std::memset(w.mbox_host, 0, (size_t)w.nr * kRing * sizeof(CgState));
  w.post_ctr = 0;
  return QCD_OK;
}

void free_ctx(qcd_ctx* c) {
  auto f = [](void* p) {
    if (p) (void)hipFree(p);
  };
  f(c->u18);
  f(c->u12);
  f(c->uh);
  f(c->uh18);
  f(c->clov);
  f(c->clov_inv);
  f(c->clov32_e);
  f(c->clovinv32_o);
  f(c->clovh_e);
  f(c->clovh_es);
  f(c->clovinvh_o);
  f(c->clovinvh_os);
  f(c->clovc_e);
  f(c->clovhc_e);
  f(c->clovhc_es);
  free_work(c->w1);
  free_work(c->wm);
  f(c->status);
  f(c->xi);
  f(c->gint);
  f(c->fbuf);
  f(c->logdet);
  if (c->status_host) (void)hipHostFree(c->status_host);
  for (auto& row : c->iter_graph)
    for (auto& gx : row)
      if (gx) (void)hipGraphExecDestroy(gx);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double2* g_scratch_dev[kMaxDevices] = {};  // device address of `scratch`, per device

// the site term of k2 reads the compact A_ee where the clover term has its form
bool use_compact(const qcd_ctx* c) { return c->compact_clover == 1 && c->compact_ok; }
int check_ctx(qcd_ctx* c) {
  if (!c) return fail(QCD_EINVAL, "null context");
  if (hipSetDevice(c->device) != hipSuccess) return fail(QCD_EHIP, "hipSetDevice failed");
  return QCD_OK;
}
// Resolve the device address of `scratch` on device `dev` (current), once per device.
int resolve_scratch(int dev) {
  if (dev >= kMaxDevices) return fail(QCD_EINVAL, "device index beyond the library's table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev]) return QCD_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr)
    return fail(QCD_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_dev[dev] = static_cast<double2*>(p);
  return QCD_OK;
}
double2* scratch_of(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return dev < kMaxDevices ? g_scratch_dev[dev] : nullptr;
}
int need_gauge(qcd_ctx* c) {
  if (!c->gauge_loaded) return fail(QCD_ESTATE, "no gauge field loaded");
  return QCD_OK;
}
int need_clover(qcd_ctx* c) {
  QCHK(need_gauge(c));
  if (!c->clover_ready) return fail(QCD_ESTATE, "clover term not built (call qcd_build_clover or qcd_load_clover)");
  return QCD_OK;
}

// ------------------------------------------------------------------ operator pieces
DslashOp base_op(const qcd_ctx* c, int par_out) {
  DslashOp op;
  std::memset(&op, 0, sizeof(op));
  op.par_out = par_out;
  op.link_kind = c->lk64();
  op.links = c->links64();
  op.c = 1.0;
  op.partial = c->w->partial;
  op.lg = c->w->lg;
  op.small_grid = c->small_grid;
  return op;
}

// t_o = A_oo^{-1} g5^dag H_oe g5^dag in_e   (dag: g5 on input and output of the hop)
// k1 that also finishes alpha from the work set's partials (in place of a
// finalisation launch): only for the dagger k1 of a CG iteration, which does
// not itself read alpha
void fuse_fin_alpha(const qcd_ctx* c, DslashOp& op) {
  op.fin_st = c->w->st;
  op.fin_partial = c->w->partial;
  op.fin_n = blocks_for(c->w->gv.Vh, c->block());  // the partials of the previous launch
  op.fin_nr = c->w->nr;
}
int k1_f64(qcd_ctx* c, int in, int out, bool dag, const CgState* st, bool fin_alpha = false) {
  DslashOp op = base_op(c, 1);
  op.in = c->ref64(in);
  op.out = c->ref64(out);
  op.site_mode = 0;
  op.post = 1;
  op.cpost = ClovRef{CL_F64, c->clov_inv, nullptr};
  op.g5in = dag;
  op.g5out = 0;
  op.st = st;
  if (fin_alpha) fuse_fin_alpha(c, op);
  HIPCHK(launch_dslash(c->g, op, c->block(), c->stream));
  return QCD_OK;
}
// out_e = A_ee s_e - kappa^2 (g5) H_eo t_o, with epilogue
int k2_f64(qcd_ctx* c, int site, int t, int out, bool dag, int epi, int y, double a, bool a_state,
           const CgState* st) {
  DslashOp op = base_op(c, 0);
  op.in = c->ref64(t);
  op.site = c->ref64(site);
  op.out = c->ref64(out);
  op.site_mode = 2;
  op.cpre = use_compact(c) && c->link_recon == 12 ? ClovRef{CL_F64C, c->clovc_e, nullptr}
                                                    : ClovRef{CL_F64, c->clov_par(0), nullptr};
  op.c = -c->kappa * c->kappa;
  op.g5out = dag;
  op.epi = epi;
  if (epi == 2) op.y = c->ref64(y);
  op.a = a;
  op.a_from_state = a_state;
  op.st = st;
  HIPCHK(launch_dslash(c->g, op, c->block(), c->stream));
  return QCD_OK;
}
// mixed-precision k1 / k2 on binary16 spinors and links, FP32 arithmetic
ClovRef mixed_clov(const qcd_ctx* c, bool inverse_odd) {
  if (c->mixed_clover == 16 && !inverse_odd && use_compact(c)) return ClovRef{CL_HC, c->clovhc_e, c->clovhc_es};
  if (c->mixed_clover == 16)
    return inverse_odd ? ClovRef{CL_H, c->clovinvh_o, c->clovinvh_os} : ClovRef{CL_H, c->clovh_e, c->clovh_es};
  return inverse_odd ? ClovRef{CL_F32, c->clovinv32_o, nullptr} : ClovRef{CL_F32, c->clov32_e, nullptr};
}
// binary16 links for the mixed kernels: rows 0, 1 (row 2 rebuilt) for one
// right-hand side, where bytes decide; all nine entries for several, where
// the rebuild's instructions would be repeated by every right-hand side
void mixed_links(const qcd_ctx* c, DslashOp& op) {
  op.link_kind = c->w->lg > 0 ? LK_H18 : LK_H12;
  op.links = c->w->lg > 0 ? (const void*)c->uh18 : (const void*)c->uh;
}
int k1_h(qcd_ctx* c, int in, int out, bool dag, const CgState* st, bool fin_alpha = false) {
  DslashOp op = base_op(c, 1);
  mixed_links(c, op);
  op.in = c->refh(in);
  op.out = c->refh(out);
  op.post = 1;
  op.cpost = mixed_clov(c, true);
  op.g5in = dag;
  op.st = st;
  if (fin_alpha) fuse_fin_alpha(c, op);
  HIPCHK(launch_dslash(c->g, op, c->block(), c->stream));
  return QCD_OK;
}
int k2_h(qcd_ctx* c, int site, int t, int out, bool dag, int epi, int y, bool a_state, const CgState* st) {
  DslashOp op = base_op(c, 0);
  mixed_links(c, op);
  op.in = c->refh(t);
  op.site = c->refh(site);
  op.out = c->refh(out);
  op.site_mode = 2;
  op.cpre = mixed_clov(c, false);
  op.c = -c->kappa * c->kappa;
  op.g5out = dag;
  op.epi = epi;
  if (epi == 2) op.y = c->refh(y);
  op.a = -1.0;
  op.a_from_state = a_state;
  op.st = st;
  HIPCHK(launch_dslash(c->g, op, c->block(), c->stream));
  return QCD_OK;
}
// full-lattice M (or M^dag) on parity p: out_p = A_pp in_p - kappa g5 H g5 in_(1-p), with epilogue
int m_parity(qcd_ctx* c, int par, int in_site, int in_nbr, int out, bool dag, int epi, int y, double a) {
  DslashOp op = base_op(c, par);
  op.in = c->ref64(in_nbr);
  op.site = c->ref64(in_site);
  op.out = c->ref64(out);
  op.site_mode = 2;
  op.cpre = ClovRef{CL_F64, c->clov_par(par), nullptr};
  op.c = -c->kappa;
  op.g5in = dag;
  op.g5out = dag;
  op.epi = epi;
  if (epi == 2) op.y = c->ref64(y);
  op.a = a;
  HIPCHK(launch_dslash(c->g, op, c->block(), c->stream));
  return QCD_OK;
}

int nblocks(const qcd_ctx* c) { return blocks_for(c->w->gv.Vh, c->block()); }
// Folded partial sums go after the partials of the smallest workgroup size.
double* fold_area(const qcd_ctx* c) {
  return c->w->partial + ((size_t)blocks_for(c->w->gv.Vh, 64) + 64) * c->w->nr;
}

int sync_state(qcd_ctx* c) {
  HIPCHK(hipMemcpyAsync(c->w->st_host, c->w->st, c->w->nr * sizeof(CgState), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return QCD_OK;
}

// |x|^2 of an FP64 vector into st->scalar and returned (synchronises)
int norm2_sync(qcd_ctx* c, int s, double* out) {
  HIPCHK(launch_norm2(c->w->gv, c->w->lg, c->ref64(s), c->w->partial, c->block(), c->stream));
  HIPCHK(launch_fin_scalar(c->w->st, c->w->partial, nblocks(c), c->w->nr, fold_area(c), c->stream));
  QCHK(sync_state(c));
  *out = c->w->st_host->scalar;
  return QCD_OK;
}

// |x|^2 of each right-hand side of an FP64 vector (synchronises)
int norm2_each(qcd_ctx* c, int s, double* out) {
  HIPCHK(launch_norm2(c->w->gv, c->w->lg, c->ref64(s), c->w->partial, c->block(), c->stream));
  HIPCHK(launch_fin_scalar(c->w->st, c->w->partial, nblocks(c), c->w->nr, fold_area(c), c->stream));
  QCHK(sync_state(c));
  for (int r = 0; r < c->w->nr; ++r) out[r] = c->w->st_host[r].scalar;
  return QCD_OK;
}

// algorithmic bytes of one Mhat^dag Mhat per even site (k1 + k2, twice) for
// nr interleaved right-hand sides: spinors nr times, links and clover once
double mdagm_bytes_per_site(const qcd_ctx* c, bool mixed, int nr = 1) {
  // k2's A_ee in the compact form: 26 reals per block instead of 36
  if (!mixed) {
    const double sp = 192.0 * nr, lk = (c->link_recon == 12 ? 96.0 : 144.0), cl = 576.0;
    const double cl_ee = use_compact(c) && c->link_recon == 12 ? 416.0 : cl;
    const double k1 = sp + 8 * lk + cl + sp, k2 = sp + 8 * lk + cl_ee + sp + sp;
    return 2.0 * (k1 + k2);
  }
  // links: two binary16 rows for one right-hand side, all nine entries for several
  const double sp = 52.0 * nr, lk = nr > 1 ? 36.0 : 24.0, cl = (c->mixed_clover == 16 ? 152.0 : 288.0);
  const double cl_ee = c->mixed_clover == 16 && use_compact(c) ? 112.0 : cl;
  const double k1 = sp + 8 * lk + cl + sp, k2 = sp + 8 * lk + cl_ee + sp + sp;
  return 2.0 * (k1 + k2);
}

// ------------------------------------------------------------------ CG drivers
// The host keeps `depth` iterations in flight.  Each iteration ends with a
// finalisation kernel that posts the state to a mailbox slot, followed by an
// event; the host waits on the event of the oldest iteration in flight,
// reads its slot, and enqueues the next iteration, so the GPU never waits for
// the host and at most depth - 1 iterations are issued past convergence
// (their kernels return at once).
struct CgCounters {
  int iters = 0, restarts = 0, ru = 0;
  double mdagm = 0.0;  // FP64 Mhat^dag Mhat applications
  double mdagm_mixed = 0.0;
  double blas_bytes = 0.0;
};

struct Pipe {
  int slot[kRing];
  long long seq = 0, seen = 0;
};

// slot of the next posted state; mirrors post() on the device
int next_slot(qcd_ctx* c) {
  const int s = c->w->post_ctr % kRing;
  c->w->post_ctr = (c->w->post_ctr + 1) % (kRing * 1024);
  return s;
}

// Read the states posted in `slot` once the work before event `slot` has
// completed: into the work set's host copies, and combined into `out`.  With
// several right-hand sides `out` is done / halted when all are, non-finite or
// asking for a reliable update when any is; its rr_hi is the largest
// rr_hi / stop2 over the right-hand sides still running (stop2 = 1).
int wait_slot(qcd_ctx* c, int slot, CgState* out) {
  HIPCHK(hipEventSynchronize(c->ev[slot]));
  Work& w = *c->w;
  for (int r = 0; r < w.nr; ++r)
    std::memcpy(&w.st_host[r], (const void*)&w.mbox_host[(size_t)r * kRing + slot], sizeof(CgState));
  *out = w.st_host[0];
  if (w.nr == 1) return QCD_OK;
  double worst = 0.0;
  for (int r = 0; r < w.nr; ++r) {
    const CgState& q = w.st_host[r];
    if (r > 0) {
      out->done &= q.done;
      out->halt &= q.halt;
      out->nan |= q.nan;
      out->need_ru |= q.need_ru;
      out->iter = std::max(out->iter, q.iter);
      out->ru_count = std::max(out->ru_count, q.ru_count);
    }
    if (!q.done && q.stop2 > 0.0) worst = std::max(worst, q.rr_hi / q.stop2);
  }
  out->rr_hi = worst;
  out->stop2 = 1.0;
  return QCD_OK;
}

int residual_f64(qcd_ctx* c, int x, int out_r, const CgState* st) {
  // out_r = rhs - Mhat^dag Mhat x, |out_r|^2 partials
  QCHK(k1_f64(c, x, V_T, false, st));
  QCHK(k2_f64(c, x, V_T, V_Q, false, 0, 0, 0.0, false, st));
  QCHK(k1_f64(c, V_Q, V_T, true, st));
  QCHK(k2_f64(c, V_Q, V_T, out_r, true, 2, V_RHS, -1.0, false, st));
  return QCD_OK;
}

// r = rhs - A x in FP64, posted as a reliable update (restart = 0) or a restart
// (nclear: the newest alphas whose directions the caller already took into x)
int recompute_residual(qcd_ctx* c, int restart, CgState* posted, int nclear = 0) {
  QCHK(residual_f64(c, V_X, V_R, nullptr));
  const int slot = next_slot(c);
  HIPCHK(launch_fin_ru(c->w->st, c->w->partial, nblocks(c), c->w->nr, fold_area(c), restart, nclear, c->w->mbox_dev,
                       kRing, c->stream));
  HIPCHK(hipEventRecord(c->ev[slot], c->stream));
  if (posted) QCHK(wait_slot(c, slot, posted));
  return QCD_OK;
}

int init_recurrence(qcd_ctx* c, double tol, double delta, int max_iter, int mixed, CgState* posted) {
  HIPCHK(launch_norm2(c->w->gv, c->w->lg, c->ref64(V_RHS), c->w->partial, c->block(), c->stream));
  const int slot = next_slot(c);
  HIPCHK(launch_fin_init(c->w->st, c->w->partial, nblocks(c), c->w->nr, fold_area(c), tol, delta, max_iter, mixed, c->w->mbox_dev, kRing, c->stream));
  HIPCHK(hipEventRecord(c->ev[slot], c->stream));
  return wait_slot(c, slot, posted);
}

// Partials per right-hand side up to which the dagger k1 finishes alpha itself.
constexpr int kFuseFinPartials = 1024;
// Workgroup size of the x/p update, which leaves no partial sums: 64 threads
// streamed faster than 256 for several right-hand sides.
constexpr int kXpBlock = 64;

// The kernels of one CG iteration, the j-th of an x cycle of c->x_defer (they
// read alpha, beta and the halt flag from the device state, so the sequence
// is the same every cycle).
int launch_iter(qcd_ctx* c, bool mixed, int j) {
  const int n = c->x_defer;
  const int nb = nblocks(c);
  // The reductions are finished by one-workgroup kernels, except that on
  // small lattices (launch-bound: a launch costs a few microseconds) the first
  // workgroups of the dagger k1, which does not read alpha, finish it; with
  // many partials per right-hand side those workgroups would outlast the
  // stencil.  (Finishing a reduction inside the stencil that produces it,
  // with a last-workgroup-arrives scheme, needs a device-scope fence per
  // workgroup, which writes back the XCD's L2 on this GPU and made the
  // iteration three times slower.)  Workgroup r of the dagger k1 (a grid of
  // nb workgroups) finishes right-hand side r, so fusing also needs nb >= nr.
  const bool fuse = nb <= kFuseFinPartials && nb >= c->w->nr;
  if (!mixed) {
    const int pj = qcd_ctx::pslot(j);
    QCHK(k1_f64(c, pj, V_T, false, c->w->st));
    QCHK(k2_f64(c, pj, V_T, V_Q, false, 1, 0, 0.0, false, c->w->st));
    if (!fuse) HIPCHK(launch_fin_alpha(c->w->st, c->w->partial, nb, c->w->nr, fold_area(c), c->stream));
    QCHK(k1_f64(c, V_Q, V_T, true, c->w->st, fuse));
    QCHK(k2_f64(c, V_Q, V_T, V_R, true, 2, V_R, 0.0, true, c->w->st));
    HIPCHK(launch_fin_beta(c->w->st, c->w->partial, nb, c->w->nr, fold_area(c), c->w->mbox_dev, kRing, c->stream));
    SpF64 p[4];
    for (int m = 0; m < n; ++m) p[m] = c->f64(qcd_ctx::pslot(m));
    HIPCHK(launch_xp_update_f64(c->w->gv, c->w->lg, c->w->st, c->f64(V_X), p, j, n, c->f64(V_R), kXpBlock, c->stream));
  } else {
    const int pj = qcd_ctx::hpslot(j);
    QCHK(k1_h(c, pj, H_T, false, c->w->st));
    QCHK(k2_h(c, pj, H_T, H_Q, false, 1, 0, false, c->w->st));
    if (!fuse) HIPCHK(launch_fin_alpha(c->w->st, c->w->partial, nb, c->w->nr, fold_area(c), c->stream));
    QCHK(k1_h(c, H_Q, H_T, true, c->w->st, fuse));
    QCHK(k2_h(c, H_Q, H_T, H_R, true, 2, H_R, true, c->w->st));
    HIPCHK(launch_fin_beta(c->w->st, c->w->partial, nb, c->w->nr, fold_area(c), c->w->mbox_dev, kRing, c->stream));
    SpH p[4];
    for (int m = 0; m < n; ++m) p[m] = c->h(qcd_ctx::hpslot(m));
    HIPCHK(launch_xp_update_h(c->w->gv, c->w->lg, c->w->st, c->f32(), p, j, n, c->h(H_R), kXpBlock, c->stream));
  }
  return QCD_OK;
}

void drop_graphs(qcd_ctx* c) {
  for (auto& row : c->iter_graph)
    for (auto& gx : row)
      if (gx) {
        (void)hipGraphExecDestroy(gx);
        gx = nullptr;
      }
}

// Capture one iteration on the private stream into an executable graph.
int capture_iter(qcd_ctx* c, bool mixed, int j) {
  hipGraphExec_t& gx = c->iter_graph[mixed ? 1 : 0][j];
  if (gx) return QCD_OK;
  const hipStream_t saved = c->stream;
  HIPCHK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  c->stream = c->cap;
  const int rc = launch_iter(c, mixed, j);
  c->stream = saved;
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(c->cap, &graph);
  if (rc != QCD_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc != QCD_OK ? rc : fail(QCD_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  }
  const hipError_t ei = hipGraphInstantiate(&gx, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    gx = nullptr;
    return fail(QCD_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
  }
  return QCD_OK;
}

// Iteration pp.seq of the recurrence is the (pp.seq mod x_defer)-th of its x cycle.
int enqueue_iter(qcd_ctx* c, Pipe& pp, bool mixed) {
  const int j = (int)(pp.seq % c->x_defer);
  if (c->use_graph && c->w->lg == 0) {
    QCHK(capture_iter(c, mixed, j));
    HIPCHK(hipGraphLaunch(c->iter_graph[mixed ? 1 : 0][j], c->stream));
  } else {
    QCHK(launch_iter(c, mixed, j));
  }
  const int slot = next_slot(c);
  HIPCHK(hipEventRecord(c->ev[slot], c->stream));
  pp.slot[pp.seq % kRing] = slot;
  ++pp.seq;
  return QCD_OK;
}

int pipeline_depth(const qcd_solver_params* p) { return std::min(std::max(1, p->pipeline_depth), kRing / 4); }

// Bytes per site and iteration of the vector work outside the stencils: the
// residual update in the last stencil's epilogue (read and write r) and the
// x/p update averaged over the x cycle (n - 1 iterations read p and r and
// write p; the last also reads the n directions and reads and writes x).
double xp_bytes_per_iter(const qcd_ctx* c, bool mixed) {
  const double sp = mixed ? 52.0 : 192.0, xb = mixed ? 96.0 : 192.0;
  const int n = c->x_defer;
  return 2 * sp + ((n - 1) * 3 * sp + (n + 2) * sp + 2 * xb) / n;
}

// FP64 CG on Mhat^dag Mhat x = rhs (V_RHS) into V_X, from x = 0 or (use_x0) from V_X.
// Work slots: V_R, V_Q, V_T and the x cycle's directions V_P, V_P1 .. V_P3.
int cg_fp64(qcd_ctx* c, const qcd_solver_params* p, bool use_x0, CgCounters& cnt) {
  const Geom& g = c->g;
  const int B = c->block();
  CgState s;
  QCHK(init_recurrence(c, p->tol, 0.0, p->max_iter, 0, &s));
  if (s.nan) return fail(QCD_ENAN, "non-finite right-hand side");
  if (use_x0) {
    QCHK(recompute_residual(c, 1, &s));
    cnt.mdagm += 1;
    if (s.nan) return fail(QCD_ENAN, "non-finite residual of the starting guess");
    HIPCHK(launch_p_restart_f64(c->w->gv, c->w->lg, c->w->st, c->f64(V_P), c->f64(V_R), B, c->stream));
  } else {
    HIPCHK(launch_zero(c->w->gv, c->ref64(V_X), B, c->stream));
    HIPCHK(launch_convert(c->w->gv, c->ref64(V_RHS), c->ref64(V_R), B, c->stream));
    HIPCHK(launch_convert(c->w->gv, c->ref64(V_RHS), c->ref64(V_P), B, c->stream));
  }
  const int depth = pipeline_depth(p);
  int restarts = 0;
  Pipe pp;
  while (!s.done) {
    while (pp.seq - pp.seen < depth) QCHK(enqueue_iter(c, pp, false));
    QCHK(wait_slot(c, pp.slot[pp.seen % kRing], &s));
    ++pp.seen;
    if (s.nan) return fail(QCD_ENAN, "non-finite residual in FP64 CG");
    if (!s.done) continue;
    // confirm with a recomputed residual (also after max_iter, for the stats);
    // restart the recurrence from it if it drifted above tol
    QCHK(recompute_residual(c, 1, &s));
    cnt.mdagm += 1;
    if (s.nan) return fail(QCD_ENAN, "non-finite residual in FP64 CG");
    if (s.done || restarts >= 8) break;
    ++restarts;
    HIPCHK(launch_p_restart_f64(c->w->gv, c->w->lg, c->w->st, c->f64(V_P), c->f64(V_R), B, c->stream));
    pp = Pipe();
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  cnt.iters += s.iter;
  cnt.mdagm += s.iter;
  cnt.restarts += restarts;
  cnt.blas_bytes += (double)s.iter * xp_bytes_per_iter(c, false) * c->w->gv.Vh;
  return QCD_OK;
}

// x_hi += x_lo + the directions of the x cycle that the iterations enqueued
// so far left pending (the first q = pp.seq mod x_defer of the cycle);
// x_lo = 0.  Returns q (>= 0) or a negative status.
int fold_x(qcd_ctx* c, const Pipe& pp) {
  const int q = (int)(pp.seq % c->x_defer);
  SpH p[4];
  for (int m = 0; m < q; ++m) p[m] = c->h(qcd_ctx::hpslot(m));
  HIPCHK(launch_ru_accum(c->w->gv, c->w->lg, c->w->st, c->f64(V_X), c->f32(), p, q, c->block(), c->stream));
  return q;
}

// Mixed-precision CG with reliable updates.  Inner recurrence on binary16
// spinors (per-site scale) and binary16 links in FP32 arithmetic, dot
// products accumulated in FP64; x accumulates in FP32 and is folded into the
// FP64 solution at every reliable update, where the residual is recomputed
// with the FP64 operator and replaces the recurrence residual (p is kept).
int cg_mixed(qcd_ctx* c, const qcd_solver_params* p, CgCounters& cnt) {
  const Geom& g = c->g;
  const int B = c->block();
  CgState s;
  QCHK(init_recurrence(c, p->tol, p->delta_reliable, p->max_iter, 1, &s));
  if (s.nan) return fail(QCD_ENAN, "non-finite right-hand side");
  HIPCHK(launch_zero(c->w->gv, c->ref64(V_X), B, c->stream));
  HIPCHK(launch_zero(c->w->gv, SpRef{SP_F32, c->w->x32, nullptr}, B, c->stream));
  HIPCHK(launch_convert(c->w->gv, c->ref64(V_RHS), c->refh(H_R), B, c->stream));
  HIPCHK(launch_convert(c->w->gv, c->ref64(V_RHS), c->refh(H_P), B, c->stream));
  const int depth = pipeline_depth(p);
  Pipe pp;
  long long ru_barrier = 0;  // iterations enqueued before the last reliable update
  int ru_seen = 0, stall = 0;
  double best_rr = s.rr_hi;
  while (!s.done) {
    while (pp.seq - pp.seen < depth) QCHK(enqueue_iter(c, pp, true));
    QCHK(wait_slot(c, pp.slot[pp.seen % kRing], &s));
    const long long idx = pp.seen++;
    if (s.nan) return fail(QCD_ENAN, "non-finite residual in mixed CG");
    if (s.done) break;
    if (s.ru_count > ru_seen) {
      ru_seen = s.ru_count;
      // the FP64 residual must keep falling (|r|^2 below 2^-stall_log2 of its
      // best at one reliable update in every three); otherwise finish in FP64
      // from x_hi
      if (s.rr_hi < std::ldexp(best_rr, -c->stall_log2)) {
        best_rr = s.rr_hi;
        stall = 0;
      } else if (++stall >= 3) {
        HIPCHK(hipStreamSynchronize(c->stream));
        if (const int q = fold_x(c, pp); q < 0) return q;
        cnt.iters += s.iter;
        cnt.mdagm_mixed += s.iter;
        cnt.restarts += 1;
        qcd_solver_params q = *p;
        q.max_iter = std::max(1, p->max_iter - s.iter);
        return cg_fp64(c, &q, true, cnt);
      }
    }
    if (s.need_ru && idx >= ru_barrier) {
      // fold x_lo and the unfinished x cycle into x_hi, r = rhs - A x_hi in
      // FP64, re-encode r; p is kept
      const int q = fold_x(c, pp);
      if (q < 0) return q;
      QCHK(recompute_residual(c, 0, nullptr, q));
      HIPCHK(launch_convert(c->w->gv, c->ref64(V_R), c->refh(H_R), B, c->stream));
      cnt.mdagm += 1;
      cnt.ru += 1;
      ru_barrier = pp.seq;
    }
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  cnt.iters += s.iter;
  cnt.mdagm_mixed += s.iter;
  cnt.blas_bytes += (double)s.iter * xp_bytes_per_iter(c, true) * c->w->gv.Vh;
  return QCD_OK;
}

int run_cg(qcd_ctx* c, const qcd_solver_params* p, CgCounters& cnt) {
  if (p->prec == QCD_MIXED) return cg_mixed(c, p, cnt);
  return cg_fp64(c, p, false, cnt);
}

int validate_params(const qcd_solver_params* p) {
  if (!p) return fail(QCD_EINVAL, "null solver params");
  if (p->prec != QCD_FP64 && p->prec != QCD_MIXED) return fail(QCD_EINVAL, "prec must be QCD_FP64 or QCD_MIXED");
  if (p->max_iter < 1) return fail(QCD_EINVAL, "max_iter must be >= 1");
  if (p->pipeline_depth < 0) return fail(QCD_EINVAL, "pipeline_depth must be >= 0");
  if (!(p->tol > 0.0) || !std::isfinite(p->tol)) return fail(QCD_EINVAL, "tol must be finite and > 0");
  if (p->prec == QCD_MIXED && (!(p->delta_reliable > 0.0) || !(p->delta_reliable < 1.0)))
    return fail(QCD_EINVAL, "delta_reliable must lie in (0, 1)");
  return QCD_OK;
}

void fill_stats_from(qcd_ctx* c, const CgState& s, const CgCounters& cnt, const qcd_solver_params* p,
                     double seconds, double true_rel, qcd_solver_stats* out, int n_share = 1) {
  if (!out) return;
  out->iters = cnt.iters;
  out->reliable_updates = cnt.ru;
  out->restarts = cnt.restarts;
  out->converged = s.rr_hi <= s.stop2 ? 1 : 0;
  out->normal_rel_res = s.stop2 > 0 ? std::sqrt(s.rr_hi / (s.stop2 / (p->tol * p->tol))) : 0.0;
  out->true_rel_res = true_rel;
  out->seconds = seconds;
  const double mdagm = cnt.mdagm + cnt.mdagm_mixed;
  const int nr = c->w->nr;
  out->flops = mdagm * 2.0 * 1824.0 * c->g.V;
  out->bytes = ((cnt.mdagm * mdagm_bytes_per_site(c, false, nr) + cnt.mdagm_mixed * mdagm_bytes_per_site(c, true, nr)) *
                    c->g.Vh +
                cnt.blas_bytes) /
               n_share;
}
void fill_stats(qcd_ctx* c, const CgCounters& cnt, const qcd_solver_params* p, double seconds, double true_rel,
                qcd_solver_stats* out) {
  fill_stats_from(c, *c->w->st_host, cnt, p, seconds, true_rel, out);
}

// Solve on even sites for a prepared right-hand side in V_RHS; result in V_X.
int solve_even(qcd_ctx* c, const qcd_solver_params* p, CgCounters& cnt) {
  QCHK(run_cg(c, p, cnt));
  return QCD_OK;
}

int validate_dims(const int dims[4]) {
  if (!dims) return fail(QCD_EINVAL, "null dims");
  long long v = 1;
  for (int k = 0; k < 4; ++k) {
    if (dims[k] < 2 || dims[k] % 2 != 0)
      return fail(QCD_EINVAL, "every lattice extent must be even and >= 2 (got " + std::to_string(dims[k]) + ")");
    v *= dims[k];
  }
  // a binary16 spinor element i is addressed with the 32-bit byte offset 48 i
  // (64-element tiles of three 16-byte chunks): V / 2 * 48 < 2^32
  if (v >= (1LL << 31) / 4 || (((v / 2 + 63) & ~63LL) * 48) >= (1LL << 32))
    return fail(QCD_EINVAL, "lattice volume too large");
  return QCD_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

int qcd_version(void) { return (1 << 16) | 0; }

const char* qcd_last_error(void) { return g_err.c_str(); }

int qcd_create(const int dims[4], int device, uintptr_t hip_stream, qcd_ctx** out) {
  if (!out) return fail(QCD_EINVAL, "null output pointer");
  *out = nullptr;
  QCHK(validate_dims(dims));
  if (device < 0) return fail(QCD_EINVAL, "negative device index");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev)
    return fail(QCD_EINVAL, "device " + std::to_string(device) + " not available");
  HIPCHK(hipSetDevice(device));
  QCHK(resolve_scratch(device));
  qcd_ctx* c = new qcd_ctx();
  for (int k = 0; k < 4; ++k) c->dims[k] = dims[k];
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  Geom& g = c->g;
  for (int k = 0; k < 4; ++k) g.X[k] = dims[k];
  g.Xh = dims[0] / 2;
  g.V = dims[0] * dims[1] * dims[2] * dims[3];
  g.Vh = g.V / 2;
  g.stride = (g.Vh + 63) & ~63;  // FP64 spinor fields are tiled by 64 elements
  g.tb = c->tb;
  g.inv_xh = 1.0 / g.Xh;
  g.inv_y = 1.0 / g.X[1];
  g.inv_z = 1.0 / g.X[2];
  const size_t S = g.stride;
  int rc = QCD_OK;
  auto A = [&](auto** p, size_t bytes) {
    if (rc == QCD_OK) rc = dalloc(p, bytes);
  };
  A(&c->u18, 8 * 9 * S * sizeof(double2));
  A(&c->u12, 8 * 6 * S * sizeof(double2));
  A(&c->uh, 8 * 3 * S * sizeof(uint2));
  A(&c->uh18, 8 * 2 * S * sizeof(uint4) + 8 * S * sizeof(unsigned int));
  A(&c->clov, 2 * 36 * S * sizeof(double2));
  A(&c->clov_inv, 36 * S * sizeof(double2));
  A(&c->clov32_e, 18 * S * sizeof(float4));
  A(&c->clovinv32_o, 18 * S * sizeof(float4));
  A(&c->clovh_e, 9 * S * sizeof(uint4));
  A(&c->clovh_es, S * sizeof(float2));
  A(&c->clovinvh_o, 9 * S * sizeof(uint4));
  A(&c->clovinvh_os, S * sizeof(float2));
  A(&c->logdet, S * sizeof(double));
  A(&c->clovc_e, 26 * S * sizeof(double2));
  A(&c->clovhc_e, 6 * S * sizeof(uint4) + S * sizeof(uint2));
  A(&c->clovhc_es, S * sizeof(float2));
  A(&c->status, 2 * sizeof(int));
  if (rc == QCD_OK) rc = alloc_work(g, c->w1, 0, true);
  if (rc == QCD_OK && hipHostMalloc((void**)&c->status_host, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess)
    rc = fail(QCD_ENOMEM, "pinned host allocation failed");
  for (int k = 0; k < kRing && rc == QCD_OK; ++k)
    if (hipEventCreateWithFlags(&c->ev[k], hipEventDisableTiming) != hipSuccess) rc = fail(QCD_EHIP, "hipEventCreate failed");
  if (rc == QCD_OK && hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess)
    rc = fail(QCD_EHIP, "hipStreamCreate failed");
  if (rc != QCD_OK) {
    free_ctx(c);
    delete c;
    return rc;
  }
  *out = c;
  return QCD_OK;
}

int qcd_destroy(qcd_ctx* c) {
  if (!c) return QCD_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  free_ctx(c);
  delete c;
  return QCD_OK;
}

int qcd_set_params(qcd_ctx* c, double kappa, double csw, int t_boundary) {
  QCHK(check_ctx(c));
  if (!(kappa > 0.0) || !std::isfinite(kappa)) return fail(QCD_EINVAL, "kappa must be finite and > 0");
  if (!std::isfinite(csw)) return fail(QCD_EINVAL, "c_sw must be finite");
  if (t_boundary != 1 && t_boundary != -1) return fail(QCD_EINVAL, "t_boundary must be +1 or -1");
  c->kappa = kappa;
  c->csw = csw;
  c->tb = t_boundary;
  c->g.tb = t_boundary;
  c->clover_ready = false;
  drop_graphs(c);
  return QCD_OK;
}

int qcd_set_option(qcd_ctx* c, int option, int value) {
  QCHK(check_ctx(c));
  drop_graphs(c);
  switch (option) {
    case QCD_OPT_LINK_RECON:
      if (value != 12 && value != 18) return fail(QCD_EINVAL, "link reconstruction must be 12 or 18");
      c->link_recon = value;
      return QCD_OK;
    case QCD_OPT_MIXED_CLOVER:
      if (value != 16 && value != 32) return fail(QCD_EINVAL, "mixed clover storage must be 16 or 32");
      c->mixed_clover = value;
      return QCD_OK;
    case QCD_OPT_BLOCK:
      if (value != 0 && (value < 64 || value > 256 || value % 64 != 0))
        return fail(QCD_EINVAL, "block size must be 0 or a multiple of 64 in [64, 256]");
      c->block_opt = value;
      return QCD_OK;
    case QCD_OPT_GRAPH:
      if (value != 0 && value != 1) return fail(QCD_EINVAL, "graph option must be 0 or 1");
      c->use_graph = value;
      return QCD_OK;
    case QCD_OPT_SMALL_GRID:
      if (value < 0 || value > 2) return fail(QCD_EINVAL, "small-grid option must be 0, 1 or 2");
      c->small_grid = value;
      return QCD_OK;
    case QCD_OPT_COMPACT_CLOVER:
      if (value != 0 && value != 1) return fail(QCD_EINVAL, "compact clover option must be 0 or 1");
      c->compact_clover = value;
      return QCD_OK;
    case QCD_OPT_MIXED_STALL:
      if (value < 1 || value > 60) return fail(QCD_EINVAL, "mixed stall exponent must lie in [1, 60]");
      c->stall_log2 = value;
      return QCD_OK;
    case QCD_OPT_X_CYCLE:
      if (value < 1 || value > 4) return fail(QCD_EINVAL, "x cycle must lie in [1, 4]");
      c->x_defer = value;
      return QCD_OK;
    default:
      return fail(QCD_EINVAL, "unknown option");
  }
}

int qcd_load_gauge(qcd_ctx* c, const void* U_dev) {
  QCHK(check_ctx(c));
  if (!U_dev) return fail(QCD_EINVAL, "null gauge pointer");
  HIPCHK(launch_pack_gauge(c->g, (const double2*)U_dev, c->u18, c->stream));
  HIPCHK(launch_derive_links(c->g, c->u18, c->u12, c->uh, c->uh18, c->stream));
  c->gauge_loaded = true;
  c->clover_ready = false;
  return QCD_OK;
}

int qcd_store_gauge(qcd_ctx* c, void* U_dev) {
  QCHK(check_ctx(c));
  if (!U_dev) return fail(QCD_EINVAL, "null gauge pointer");
  QCHK(need_gauge(c));
  HIPCHK(launch_unpack_gauge(c->g, c->u18, (double2*)U_dev, c->stream));
  return QCD_OK;
}

static int invert_clover(qcd_ctx* c) {
  HIPCHK(hipMemsetAsync(c->status, 0, 2 * sizeof(int), c->stream));
  HIPCHK(launch_clover_invert(c->g, c->clov, c->clov_inv, c->clov32_e, c->clovinv32_o, c->clovh_e, c->clovh_es,
                              c->clovinvh_o, c->clovinvh_os, c->logdet, c->status, c->stream));
  HIPCHK(launch_clover_compact(c->g, c->clov, c->clovc_e, c->clovhc_e, c->clovhc_es, c->status + 1, c->stream));
  HIPCHK(hipMemcpyAsync(c->status_host, c->status, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->compact_ok = c->status_host[1] == 0;
  if (*c->status_host != 0) {
    c->clover_ready = false;
    return fail(QCD_ECLOVER, "an odd-site clover block is not positive definite");
  }
  c->clover_ready = true;
  return QCD_OK;
}

int qcd_build_clover(qcd_ctx* c) {
  QCHK(check_ctx(c));
  QCHK(need_gauge(c));
  HIPCHK(launch_clover_build(c->g, c->u18, c->kappa, c->csw, c->clov, c->stream));
  return invert_clover(c);
}

int qcd_load_clover(qcd_ctx* c, const double* A_dev) {
  QCHK(check_ctx(c));
  if (!A_dev) return fail(QCD_EINVAL, "null clover pointer");
  QCHK(need_gauge(c));
  HIPCHK(launch_pack_clover(c->g, (const double2*)A_dev, c->clov, c->stream));
  return invert_clover(c);
}

int qcd_get_clover(qcd_ctx* c, double* A_dev, double* Ainv_dev) {
  QCHK(check_ctx(c));
  QCHK(need_clover(c));
  if (A_dev) HIPCHK(launch_unpack_clover(c->g, c->clov, (double2*)A_dev, 2, 0, c->stream));
  if (Ainv_dev) HIPCHK(launch_unpack_clover(c->g, c->clov_inv, (double2*)Ainv_dev, 1, 0, c->stream));
  return QCD_OK;
}

int qcd_apply(qcd_ctx* c, int op, int prec, const void* in_dev, void* out_dev) {
  QCHK(check_ctx(c));
  if (!in_dev || !out_dev) return fail(QCD_EINVAL, "null vector pointer");
  if (in_dev == out_dev) return fail(QCD_EINVAL, "in and out must not overlap");
  if (op < QCD_OP_M || op > QCD_OP_MHATDAGMHAT) return fail(QCD_EINVAL, "unknown operator");
  if (prec != QCD_FP64 && prec != QCD_MIXED) return fail(QCD_EINVAL, "unknown precision");
  if (prec == QCD_MIXED && (op == QCD_OP_M || op == QCD_OP_MDAG))
    return fail(QCD_EINVAL, "the full-lattice operators are FP64 only");
  QCHK(need_clover(c));
  const Geom& g = c->g;
  if (op == QCD_OP_M || op == QCD_OP_MDAG) {
    const bool dag = op == QCD_OP_MDAG;
    HIPCHK(launch_pack_spinor_full(g, (const double2*)in_dev, c->f64(V_IN_E), c->f64(V_IN_O), c->stream));
    QCHK(m_parity(c, 0, V_IN_E, V_IN_O, V_OUT_E, dag, 0, 0, 0.0));
    QCHK(m_parity(c, 1, V_IN_O, V_IN_E, V_OUT_O, dag, 0, 0, 0.0));
    HIPCHK(launch_unpack_spinor_full(g, c->f64(V_OUT_E), c->f64(V_OUT_O), (double2*)out_dev, c->stream));
    return QCD_OK;
  }
  HIPCHK(launch_pack_spinor_cb(g, (const double2*)in_dev, c->f64(V_IN_E), c->stream));
  const bool first = op == QCD_OP_MHAT || op == QCD_OP_MHATDAGMHAT;
  const bool second = op == QCD_OP_MHATDAG || op == QCD_OP_MHATDAGMHAT;
  if (prec == QCD_FP64) {
    int cur = V_IN_E;
    if (first) {
      QCHK(k1_f64(c, cur, V_T, false, nullptr));
      QCHK(k2_f64(c, cur, V_T, V_OUT_E, false, 0, 0, 0.0, false, nullptr));
      cur = V_OUT_E;
    }
    if (second) {
      const int dst = cur == V_OUT_E ? V_AUX : V_OUT_E;
      QCHK(k1_f64(c, cur, V_T, true, nullptr));
      QCHK(k2_f64(c, cur, V_T, dst, true, 0, 0, 0.0, false, nullptr));
      cur = dst;
    }
    HIPCHK(launch_unpack_spinor_cb(g, c->f64(cur), (double2*)out_dev, c->stream));
    return QCD_OK;
  }
  HIPCHK(launch_convert(c->w->gv, c->ref64(V_IN_E), c->refh(H_IN), c->block(), c->stream));
  int cur = H_IN;
  if (first) {
    QCHK(k1_h(c, cur, H_T, false, nullptr));
    QCHK(k2_h(c, cur, H_T, H_OUT, false, 0, 0, false, nullptr));
    cur = H_OUT;
  }
  if (second) {
    const int dst = cur == H_OUT ? H_Q : H_OUT;
    QCHK(k1_h(c, cur, H_T, true, nullptr));
    QCHK(k2_h(c, cur, H_T, dst, true, 0, 0, false, nullptr));
    cur = dst;
  }
  HIPCHK(launch_convert(c->w->gv, c->refh(cur), c->ref64(V_OUT_E), c->block(), c->stream));
  HIPCHK(launch_unpack_spinor_cb(g, c->f64(V_OUT_E), (double2*)out_dev, c->stream));
  return QCD_OK;
}

}  // extern "C"

namespace {

// Selects the work set the drivers use for the lifetime of the guard.
struct WorkGuard {
  qcd_ctx* c;
  WorkGuard(qcd_ctx* ctx, Work* w) : c(ctx) { c->w = w; }
  ~WorkGuard() { c->w = &c->w1; }
};

// Make the multi-source work set hold 1 << lg right-hand sides.
int use_multi(qcd_ctx* c, int lg) {
  // the stencils address a chunk element with a 32-bit byte offset (16-byte
  // elements; 48 bytes per element of the tiled binary16 fields)
  if (((long long)c->g.stride << lg) * 48 >= (1LL << 32))
    return fail(QCD_EINVAL, "too many interleaved right-hand sides for this lattice volume");
  if (c->wm.st == nullptr || c->wm_lg_alloc < lg) {
    free_work(c->wm);
    c->wm_lg_alloc = -1;
    QCHK(alloc_work(c->g, c->wm, lg, false));
    c->wm_lg_alloc = lg;
  }
  Work& w = c->wm;
  w.lg = lg;
  w.nr = 1 << lg;
  w.gv = c->g;
  w.gv.Vh = c->g.Vh << lg;
  w.gv.stride = c->g.stride << lg;
  return QCD_OK;
}

// Solve M x = b for the work set's right-hand sides (n of them, packed by the
// caller into V_B_E / V_B_O); writes x into V_X / V_OUT_O and the stats.
int solve_packed(qcd_ctx* c, const qcd_solver_params* p, int n, qcd_solver_stats* stats,
                 std::chrono::steady_clock::time_point t0) {
  const Geom& g = c->g;
  const int B = c->block(), nb = nblocks(c), nr = c->w->nr;
  // bhat = b_e + kappa H_eo A_oo^{-1} b_o; rhs = Mhat^dag bhat
  HIPCHK(launch_clover_apply(g, c->w->lg, c->f64(V_B_O), c->f64(V_T), c->clov_inv, c->stream));
  {
    DslashOp op = base_op(c, 0);
    op.in = c->ref64(V_T);
    op.site = c->ref64(V_B_E);
    op.out = c->ref64(V_AUX);
    op.site_mode = 1;
    op.c = c->kappa;
    HIPCHK(launch_dslash(g, op, B, c->stream));
  }
  QCHK(k1_f64(c, V_AUX, V_T, true, nullptr));
  QCHK(k2_f64(c, V_AUX, V_T, V_RHS, true, 0, 0, 0.0, false, nullptr));
  CgCounters cnt;
  int rc = solve_even(c, p, cnt);
  if (rc != QCD_OK && rc != QCD_ENOCONV) return rc;
  CgState s_end[16];
  std::memcpy(s_end, c->w->st_host, nr * sizeof(CgState));
  // x_o = A_oo^{-1} (b_o + kappa H_oe x_e)
  {
    DslashOp op = base_op(c, 1);
    op.in = c->ref64(V_X);
    op.site = c->ref64(V_B_O);
    op.out = c->ref64(V_OUT_O);
    op.site_mode = 1;
    op.post = 1;
    op.cpost = ClovRef{CL_F64, c->clov_inv, nullptr};
    op.c = c->kappa;
    HIPCHK(launch_dslash(g, op, B, c->stream));
  }
  // true residual ||b - M x|| / ||b|| on the full lattice, per right-hand side
  double rn[16] = {}, bn[16] = {}, t[16];
  QCHK(m_parity(c, 0, V_X, V_OUT_O, V_AUX, false, 2, V_B_E, -1.0));
  HIPCHK(launch_fin_scalar(c->w->st, c->w->partial, nb, nr, fold_area(c), c->stream));
  QCHK(sync_state(c));
  for (int r = 0; r < nr; ++r) rn[r] += c->w->st_host[r].scalar;
  QCHK(m_parity(c, 1, V_OUT_O, V_X, V_AUX, false, 2, V_B_O, -1.0));
  HIPCHK(launch_fin_scalar(c->w->st, c->w->partial, nb, nr, fold_area(c), c->stream));
  QCHK(sync_state(c));
  for (int r = 0; r < nr; ++r) rn[r] += c->w->st_host[r].scalar;
  QCHK(norm2_each(c, V_B_E, t));
  for (int r = 0; r < nr; ++r) bn[r] += t[r];
  QCHK(norm2_each(c, V_B_O, t));
  for (int r = 0; r < nr; ++r) bn[r] += t[r];
  const double seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  std::memcpy(c->w->st_host, s_end, nr * sizeof(CgState));
  bool all_conv = true;
  for (int r = 0; r < n; ++r) {
    if (stats) fill_stats_from(c, s_end[r], cnt, p, seconds, bn[r] > 0 ? std::sqrt(rn[r] / bn[r]) : 0.0, &stats[r], n);
    if (s_end[r].rr_hi > s_end[r].stop2) all_conv = false;
  }
  if (!all_conv) return fail(QCD_ENOCONV, "solver reached max_iter without meeting tol");
  return QCD_OK;
}

}  // namespace

extern "C" {

int qcd_solve(qcd_ctx* c, const qcd_solver_params* p, const void* b_dev, void* x_dev, qcd_solver_stats* stats) {
  QCHK(check_ctx(c));
  QCHK(validate_params(p));
  if (!b_dev || !x_dev) return fail(QCD_EINVAL, "null vector pointer");
  QCHK(need_clover(c));
  const auto t0 = std::chrono::steady_clock::now();
  WorkGuard wg(c, &c->w1);
  HIPCHK(launch_pack_spinor_full(c->g, (const double2*)b_dev, c->f64(V_B_E), c->f64(V_B_O), c->stream));
  const int rc = solve_packed(c, p, 1, stats, t0);
  if (rc != QCD_OK && rc != QCD_ENOCONV) return rc;
  HIPCHK(launch_unpack_spinor_full(c->g, c->f64(V_X), c->f64(V_OUT_O), (double2*)x_dev, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return rc;
}

int qcd_solve_multi(qcd_ctx* c, const qcd_solver_params* p, int n_rhs, const void* b_dev, void* x_dev,
                    qcd_solver_stats* stats) {
  QCHK(check_ctx(c));
  QCHK(validate_params(p));
  if (!b_dev || !x_dev) return fail(QCD_EINVAL, "null vector pointer");
  if (n_rhs < 1 || n_rhs > QCD_MAX_RHS) return fail(QCD_EINVAL, "n_rhs must lie in [1, 16]");
  if (b_dev == x_dev) return fail(QCD_EINVAL, "b and x must not overlap");
  QCHK(need_clover(c));
  const auto t0 = std::chrono::steady_clock::now();
  int lg = 0;
  while ((1 << lg) < n_rhs) ++lg;
  // a set allocated for more right-hand sides serves fewer (its buffers are larger)
  QCHK(use_multi(c, lg));
  Work& w = c->wm;
  // every state posts in step from zero
  HIPCHK(hipMemsetAsync(w.st, 0, ((size_t)1 << c->wm_lg_alloc) * sizeof(CgState), c->stream));
  w.post_ctr = 0;
  WorkGuard wg(c, &w);
  HIPCHK(launch_pack_spinor_multi(c->g, lg, n_rhs, (const double2*)b_dev, c->f64(V_B_E), c->f64(V_B_O), c->stream));
  const int rc = solve_packed(c, p, n_rhs, stats, t0);
  if (rc != QCD_OK && rc != QCD_ENOCONV) return rc;
  HIPCHK(launch_unpack_spinor_multi(c->g, lg, n_rhs, c->f64(V_X), c->f64(V_OUT_O), (double2*)x_dev, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return rc;
}

// Force pipeline on the current context state; phi in V_RHS (even sites).
// The fermion part of the force enters with weight wf; with det the
// derivative of -2 sum_odd ln det A, also weighted wf, joins the clover part.
static int force_core(qcd_ctx* c, const qcd_solver_params* p, double* S, CgCounters& cnt, int* conv_rc,
                      double wf = 1.0, bool det = false, double gauge_coef = 0.0) {
  const Geom& g = c->g;
  const int nb = nblocks(c);
  if (!c->xi) QCHK(dalloc(&c->xi, (size_t)2 * 6 * 9 * g.stride * sizeof(double2)));
  if (!c->gint) QCHK(dalloc(&c->gint, (size_t)8 * 9 * g.stride * sizeof(double2)));
  // keep phi: the solver overwrites work slots but not V_RHS
  int rc = run_cg(c, p, cnt);
  if (rc != QCD_OK) return rc;
  *conv_rc = c->w->st_host->rr_hi <= c->w->st_host->stop2 ? QCD_OK : QCD_ENOCONV;
  CgState s_end = *c->w->st_host;
  // S = Re phi^dag X
  HIPCHK(launch_dot_re(c->w->gv, c->w->lg, c->f64(V_RHS), c->f64(V_X), c->w->partial, c->block(), c->stream));
  HIPCHK(launch_fin_scalar(c->w->st, c->w->partial, nb, c->w->nr, fold_area(c), c->stream));
  QCHK(sync_state(c));
  if (S) *S = c->w->st_host->scalar;
  *c->w->st_host = s_end;
  // Z = A_oo^{-1} H_oe X; Y = Mhat X; W = A_oo^{-1} g5 H_oe g5 Y
  QCHK(k1_f64(c, V_X, V_Z, false, nullptr));
  QCHK(k2_f64(c, V_X, V_Z, V_Y, false, 0, 0, 0.0, false, nullptr));
  {
    DslashOp op = base_op(c, 1);
    op.in = c->ref64(V_Y);
    op.out = c->ref64(V_W);
    op.post = 1;
    op.cpost = ClovRef{CL_F64, c->clov_inv, nullptr};
    op.g5in = 1;
    op.g5out = 1;
    HIPCHK(launch_dslash(g, op, c->block(), c->stream));
  }
  const double k2 = c->kappa * c->kappa;
  HIPCHK(launch_force_hop(g, c->u18, c->f64(V_Y), c->f64(V_W), c->f64(V_X), c->f64(V_Z), 2.0 * k2 * wf, c->gint,
                          c->stream));
  if (c->csw != 0.0) {
    HIPCHK(launch_clover_xi(g, c->f64(V_Y), c->f64(V_W), c->f64(V_X), c->f64(V_Z), wf, wf * k2,
                            det ? c->clov_inv : nullptr, wf, c->xi, c->stream));
    HIPCHK(launch_force_clover(g, c->u18, c->xi, 0.5 * c->kappa * c->csw, c->gint, c->stream, gauge_coef));
  }
  return QCD_OK;
}

int qcd_action_force(qcd_ctx* c, const qcd_solver_params* p, const void* phi_dev, double* S, void* G_dev,
                     double* F_dev, void* X_dev, qcd_solver_stats* stats) {
  QCHK(check_ctx(c));
  QCHK(validate_params(p));
  if (!phi_dev || !G_dev) return fail(QCD_EINVAL, "null pointer (phi and G are required)");
  QCHK(need_clover(c));
  const auto t0 = std::chrono::steady_clock::now();
  HIPCHK(launch_pack_spinor_cb(c->g, (const double2*)phi_dev, c->f64(V_RHS), c->stream));
  CgCounters cnt;
  int conv = QCD_OK;
  QCHK(force_core(c, p, S, cnt, &conv));
  HIPCHK(launch_force_out(c->g, c->u18, c->gint, (double2*)G_dev, F_dev, c->stream));
  if (X_dev) HIPCHK(launch_unpack_spinor_cb(c->g, c->f64(V_X), (double2*)X_dev, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  const double seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  fill_stats(c, cnt, p, seconds, -1.0, stats);
  if (conv != QCD_OK) return fail(QCD_ENOCONV, "force solve reached max_iter without meeting tol");
  return QCD_OK;
}

int qcd_hmd_step(qcd_ctx* c, double dt, void* U_dev, double* P_dev, const void* xi_dev,
                 const qcd_solver_params* p, double* S, qcd_solver_stats* stats) {
  QCHK(check_ctx(c));
  QCHK(validate_params(p));
  if (!U_dev || !P_dev || !xi_dev) return fail(QCD_EINVAL, "null pointer");
  if (!std::isfinite(dt)) return fail(QCD_EINVAL, "dt must be finite");
  const auto t0 = std::chrono::steady_clock::now();
  const Geom& g = c->g;
  if (!c->fbuf) QCHK(dalloc(&c->fbuf, (size_t)32 * g.V * sizeof(double)));
  if (!c->gint) QCHK(dalloc(&c->gint, (size_t)8 * 9 * g.stride * sizeof(double2)));
  // two flavours per pseudofermion at N_f = 2: the R algorithm draws the
  // noise at the start of the step, phi = Mhat^dag(U_0) xi
  HIPCHK(launch_pack_gauge(g, (const double2*)U_dev, c->u18, c->stream));
  HIPCHK(launch_derive_links(g, c->u18, c->u12, c->uh, c->uh18, c->stream));
  c->gauge_loaded = true;
  QCHK(qcd_build_clover(c));
  HIPCHK(launch_pack_spinor_cb(g, (const double2*)xi_dev, c->f64(V_IN_E), c->stream));
  QCHK(k1_f64(c, V_IN_E, V_T, true, nullptr));
  QCHK(k2_f64(c, V_IN_E, V_T, V_RHS, true, 0, 0, 0.0, false, nullptr));
  // U_1/2 = exp(i dt/2 P) U_0, where the force is taken
  HIPCHK(launch_link_exp(g, c->u18, P_dev, 0.5 * dt, c->stream));
  HIPCHK(launch_derive_links(g, c->u18, c->u12, c->uh, c->uh18, c->stream));
  QCHK(qcd_build_clover(c));
  CgCounters cnt;
  int conv = QCD_OK;
  QCHK(force_core(c, p, S, cnt, &conv));
  HIPCHK(launch_force_out(g, c->u18, c->gint, nullptr, c->fbuf, c->stream));
  // P <- P - dt F;  U <- exp(i dt/2 P) U_1/2
  HIPCHK(launch_mom_update(g, P_dev, c->fbuf, dt, c->stream));
  HIPCHK(launch_link_exp(g, c->u18, P_dev, 0.5 * dt, c->stream));
  HIPCHK(launch_derive_links(g, c->u18, c->u12, c->uh, c->uh18, c->stream));
  HIPCHK(launch_unpack_gauge(g, c->u18, (double2*)U_dev, c->stream));
  QCHK(qcd_build_clover(c));
  const double seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  fill_stats(c, cnt, p, seconds, -1.0, stats);
  if (conv != QCD_OK) return fail(QCD_ENOCONV, "force solve reached max_iter without meeting tol");
  return QCD_OK;
}

// beta sum (1 - Re tr P / 3) (synchronises; overwrites the host state mirror)
static int gauge_action_sync(qcd_ctx* c, double beta, double* S) {
  HIPCHK(launch_plaquette(c->g, c->u18, c->w->partial, c->block(), c->stream));
  HIPCHK(launch_fin_scalar(c->w->st, c->w->partial, nblocks(c), c->w->nr, fold_area(c), c->stream));
  QCHK(sync_state(c));
  *S = beta * c->w->st_host->scalar;
  return QCD_OK;
}

// -2 sum_odd ln det A from the last inversion (synchronises)
static int det_action_sync(qcd_ctx* c, double* S) {
  HIPCHK(launch_sum_cb(c->g, c->logdet, c->w->partial, c->block(), c->stream));
  HIPCHK(launch_fin_scalar(c->w->st, c->w->partial, nblocks(c), c->w->nr, fold_area(c), c->stream));
  QCHK(sync_state(c));
  *S = -2.0 * c->w->st_host->scalar;
  return QCD_OK;
}

static int ensure_force_buffers(qcd_ctx* c) {
  const Geom& g = c->g;
  if (!c->xi) QCHK(dalloc(&c->xi, (size_t)2 * 6 * 9 * g.stride * sizeof(double2)));
  if (!c->gint) QCHK(dalloc(&c->gint, (size_t)8 * 9 * g.stride * sizeof(double2)));
  return QCD_OK;
}

int qcd_gauge_action_force(qcd_ctx* c, double beta, double* S, void* G_dev, double* F_dev) {
  QCHK(check_ctx(c));
  if (!std::isfinite(beta)) return fail(QCD_EINVAL, "beta must be finite");
  QCHK(need_gauge(c));
  QCHK(ensure_force_buffers(c));
  if (S) QCHK(gauge_action_sync(c, beta, S));
  if (G_dev || F_dev) {
    HIPCHK(launch_gauge_force(c->g, c->u18, -beta / 3.0, 0, c->gint, c->stream));
    HIPCHK(launch_force_out(c->g, c->u18, c->gint, (double2*)G_dev, F_dev, c->stream));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  return QCD_OK;
}

int qcd_gauge_force_noalloc(qcd_ctx* c, double beta, void* G_dev, double* F_dev) {
  QCHK(check_ctx(c));
  if (!std::isfinite(beta)) return fail(QCD_EINVAL, "beta must be finite");
  if (!G_dev && !F_dev) return fail(QCD_EINVAL, "G_dev and F_dev are both null");
  QCHK(need_gauge(c));
  if ((size_t)c->g.stride > kScratchVh)
    return fail(QCD_EINVAL, "lattice too large for the allocation-free gauge force: " + std::to_string(c->g.V) +
                                " sites need " + std::to_string((size_t)8 * 9 * c->g.stride * sizeof(double2)) +
                                " bytes of scratch, the library holds " + std::to_string(kScratchBytes) +
                                " (at most " + std::to_string(2 * kScratchVh) + " sites)");
  double2* acc = scratch_of(c->device);
  if (!acc) return fail(QCD_ESTATE, "scratch address not resolved on this device");
  // the accumulator is overwritten (not accumulated) for every link: nothing to clear
  HIPCHK(launch_gauge_force(c->g, c->u18, -beta / 3.0, 0, acc, c->stream));
  HIPCHK(launch_force_out(c->g, c->u18, acc, (double2*)G_dev, F_dev, c->stream));
  return QCD_OK;
}

int qcd_clover_det_action_force(qcd_ctx* c, double* S, void* G_dev, double* F_dev) {
  QCHK(check_ctx(c));
  QCHK(need_clover(c));
  QCHK(ensure_force_buffers(c));
  if (S) QCHK(det_action_sync(c, S));
  if (G_dev || F_dev) {
    const Geom& g = c->g;
    HIPCHK(launch_force_zero(g, c->gint, c->stream));
    if (c->csw != 0.0) {
      HIPCHK(launch_clover_xi(g, SpF64{nullptr, g.stride}, SpF64{nullptr, g.stride}, SpF64{nullptr, g.stride},
                              SpF64{nullptr, g.stride}, 0.0, 0.0, c->clov_inv, 1.0, c->xi, c->stream));
      HIPCHK(launch_force_clover(g, c->u18, c->xi, 0.5 * c->kappa * c->csw, c->gint, c->stream));
    }
    HIPCHK(launch_force_out(g, c->u18, c->gint, (double2*)G_dev, F_dev, c->stream));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  return QCD_OK;
}

// U <- exp(i h P) U on the packed links (h = 0 leaves them untouched)
static int move_links(qcd_ctx* c, const double* P_dev, double h, bool reunit) {
  if (h != 0.0) HIPCHK(launch_link_exp(c->g, c->u18, P_dev, h, c->stream));
  if (reunit) HIPCHK(launch_reunitarize(c->g, c->u18, c->stream));
  HIPCHK(launch_derive_links(c->g, c->u18, c->u12, c->uh, c->uh18, c->stream));
  c->gauge_loaded = true;
  c->clover_ready = false;
  return QCD_OK;
}

int qcd_md_trajectory(qcd_ctx* c, const qcd_md_params* md, void* U_dev, double* P_dev, const void* xi_dev,
                      const qcd_solver_params* p, double* actions, qcd_solver_stats* stats) {
  QCHK(check_ctx(c));
  if (!md) return fail(QCD_EINVAL, "null md params");
  if (!U_dev || !P_dev) return fail(QCD_EINVAL, "null pointer");
  if (md->n_steps < 1) return fail(QCD_EINVAL, "n_steps must be >= 1");
  if (!std::isfinite(md->dt) || !std::isfinite(md->beta) || !std::isfinite(md->n_f) || md->n_f < 0.0)
    return fail(QCD_EINVAL, "dt, beta must be finite and n_f finite and >= 0");
  if ((md->clover_det != 0 && md->clover_det != 1) || (md->reunitarize != 0 && md->reunitarize != 1))
    return fail(QCD_EINVAL, "clover_det and reunitarize must be 0 or 1");
  const double wf = 0.5 * md->n_f;
  const bool ferm = wf != 0.0, det = md->clover_det == 1 && wf != 0.0;
  if (ferm) {
    QCHK(validate_params(p));
    if (!xi_dev) return fail(QCD_EINVAL, "null noise pointer");
  }
  const auto t0 = std::chrono::steady_clock::now();
  const Geom& g = c->g;
  const double dt = md->dt;
  QCHK(ensure_force_buffers(c));
  if (!c->fbuf) QCHK(dalloc(&c->fbuf, (size_t)32 * g.V * sizeof(double)));
  HIPCHK(launch_pack_gauge(g, (const double2*)U_dev, c->u18, c->stream));
  QCHK(move_links(c, P_dev, 0.0, false));  // the derived link copies of U_0
  CgCounters cnt;
  int conv_all = QCD_OK;
  for (int k = 0; k < md->n_steps; ++k) {
    double s_f = 0.0, s_g = 0.0, s_d = 0.0;
    if (ferm) {
      // R algorithm (Gottlieb et al. 1987): the noise is drawn (n_f/2) dt/2
      // before the force point, at U(t + (1 - n_f/2) dt/2); at n_f = 2 that
      // is the start of the step, and for n_f > 2 the links first move back
      const double h1 = (1.0 - wf) * 0.5 * dt;
      if (h1 != 0.0) QCHK(move_links(c, P_dev, h1, false));
      QCHK(qcd_build_clover(c));
      const double2* xi_k = (const double2*)xi_dev + (size_t)k * g.Vh * 12;
      HIPCHK(launch_pack_spinor_cb(g, xi_k, c->f64(V_IN_E), c->stream));
      QCHK(k1_f64(c, V_IN_E, V_T, true, nullptr));
      QCHK(k2_f64(c, V_IN_E, V_T, V_RHS, true, 0, 0, 0.0, false, nullptr));
      QCHK(move_links(c, P_dev, wf * 0.5 * dt, false));
      QCHK(qcd_build_clover(c));
    } else {
      QCHK(move_links(c, P_dev, 0.5 * dt, false));
    }
    if (md->beta != 0.0) QCHK(gauge_action_sync(c, md->beta, &s_g));
    if (det) QCHK(det_action_sync(c, &s_d));
    // with a clover force pass the gauge force is added there (its staples
    // are products that pass forms anyway); otherwise it has its own launch
    const bool gauge_fused = ferm && c->csw != 0.0 && md->beta != 0.0;
    if (ferm) {
      int conv = QCD_OK;
      QCHK(force_core(c, p, &s_f, cnt, &conv, wf, det, gauge_fused ? -md->beta / 3.0 : 0.0));
      if (conv != QCD_OK) conv_all = conv;
    } else {
      HIPCHK(launch_force_zero(g, c->gint, c->stream));
    }
    if (md->beta != 0.0 && !gauge_fused)
      HIPCHK(launch_gauge_force(g, c->u18, -md->beta / 3.0, 1, c->gint, c->stream));
    HIPCHK(launch_force_out(g, c->u18, c->gint, nullptr, c->fbuf, c->stream));
    HIPCHK(launch_mom_update(g, P_dev, c->fbuf, dt, c->stream));
    QCHK(move_links(c, P_dev, 0.5 * dt, md->reunitarize == 1));
    if (actions) {
      actions[3 * k] = s_f;
      actions[3 * k + 1] = s_g;
      actions[3 * k + 2] = s_d;
    }
  }
  HIPCHK(launch_unpack_gauge(g, c->u18, (double2*)U_dev, c->stream));
  if (ferm) QCHK(qcd_build_clover(c));
  HIPCHK(hipStreamSynchronize(c->stream));
  const double seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) {
    if (ferm) {
      fill_stats(c, cnt, p, seconds, -1.0, stats);
    } else {
      std::memset(stats, 0, sizeof(*stats));
      stats->converged = 1;
      stats->seconds = seconds;
    }
  }
  if (conv_all != QCD_OK) return fail(QCD_ENOCONV, "a force solve reached max_iter without meeting tol");
  return QCD_OK;
}

}  // extern "C"

namespace {

// Events around each launch of n Mhat^dag Mhat applications on the active
// work set; the vectors are slots a (input) -> b (hop) -> d -> e of the set.
int time_stencil_impl(qcd_ctx* c, int prec, int n, double* ms, const int f[4], const int h[4]) {
  // k1 and k2: an event before and after every launch of n applications of
  // Mhat^dag Mhat; the application itself: n more launched back to back, as
  // inside the solver, between one pair of events
  constexpr int kEv = 5;
  hipEvent_t ev[kEv];
  int made = 0;
  int rc = QCD_OK;
  for (; made < kEv; ++made)
    if (hipEventCreate(&ev[made]) != hipSuccess) {
      rc = fail(QCD_EHIP, "hipEventCreate failed");
      break;
    }
  auto rec = [&](int k) { return hipEventRecord(ev[k], c->stream) == hipSuccess ? QCD_OK : fail(QCD_EHIP, "hipEventRecord failed"); };
  auto launch = [&](int which) {
    if (prec == QCD_FP64) {
      switch (which) {
        case 0: return k1_f64(c, f[0], f[1], false, nullptr);
        case 1: return k2_f64(c, f[0], f[1], f[2], false, 0, 0, 0.0, false, nullptr);
        case 2: return k1_f64(c, f[2], f[1], true, nullptr);
        default: return k2_f64(c, f[2], f[1], f[3], true, 0, 0, 0.0, false, nullptr);
      }
    }
    switch (which) {
      case 0: return k1_h(c, h[0], h[1], false, nullptr);
      case 1: return k2_h(c, h[0], h[1], h[2], false, 0, 0, false, nullptr);
      case 2: return k1_h(c, h[2], h[1], true, nullptr);
      default: return k2_h(c, h[2], h[1], h[3], true, 0, 0, false, nullptr);
    }
  };
  double t_k1 = 0.0, t_k2 = 0.0;
  for (int it = 0; it < n && rc == QCD_OK; ++it) {
    for (int k = 0; k < 4 && rc == QCD_OK; ++k) {
      rc = rec(k);
      if (rc == QCD_OK) rc = launch(k);
    }
    if (rc == QCD_OK) rc = rec(4);
    if (rc == QCD_OK && hipEventSynchronize(ev[4]) != hipSuccess) rc = fail(QCD_EHIP, "hipEventSynchronize failed");
    float d[2] = {0.f, 0.f};
    for (int k = 0; k < 2 && rc == QCD_OK; ++k)
      if (hipEventElapsedTime(&d[k], ev[k], ev[k + 1]) != hipSuccess) rc = fail(QCD_EHIP, "hipEventElapsedTime failed");
    t_k1 += d[0];
    t_k2 += d[1];
  }
  float t_app = 0.f;
  if (rc == QCD_OK) rc = rec(0);
  for (int it = 0; it < n && rc == QCD_OK; ++it)
    for (int k = 0; k < 4 && rc == QCD_OK; ++k) rc = launch(k);
  if (rc == QCD_OK) rc = rec(1);
  if (rc == QCD_OK && hipEventSynchronize(ev[1]) != hipSuccess) rc = fail(QCD_EHIP, "hipEventSynchronize failed");
  if (rc == QCD_OK && hipEventElapsedTime(&t_app, ev[0], ev[1]) != hipSuccess) rc = fail(QCD_EHIP, "hipEventElapsedTime failed");
  for (int k = 0; k < made; ++k) (void)hipEventDestroy(ev[k]);
  if (rc != QCD_OK) return rc;
  ms[0] = t_k1 / n;
  ms[1] = t_k2 / n;
  ms[2] = double(t_app) / n;
  return QCD_OK;
}

int check_time_args(qcd_ctx* c, int prec, int n, double* ms) {
  QCHK(check_ctx(c));
  if (!ms) return fail(QCD_EINVAL, "null output pointer");
  if (n < 1 || n > 4096) return fail(QCD_EINVAL, "n must lie in [1, 4096]");
  if (prec != QCD_FP64 && prec != QCD_MIXED) return fail(QCD_EINVAL, "unknown precision");
  QCHK(need_clover(c));
  return QCD_OK;
}

}  // namespace

extern "C" {

int qcd_time_stencil(qcd_ctx* c, int prec, int n, double* ms) {
  QCHK(check_time_args(c, prec, n, ms));
  WorkGuard wg(c, &c->w1);
  const int f[4] = {V_IN_E, V_T, V_OUT_E, V_AUX}, h[4] = {H_IN, H_T, H_OUT, H_Q};
  return time_stencil_impl(c, prec, n, ms, f, h);
}

int qcd_time_stencil_multi(qcd_ctx* c, int prec, int n_rhs, int n, double* ms) {
  QCHK(check_time_args(c, prec, n, ms));
  if (n_rhs < 1 || n_rhs > QCD_MAX_RHS) return fail(QCD_EINVAL, "n_rhs must lie in [1, 16]");
  int lg = 0;
  while ((1 << lg) < n_rhs) ++lg;
  QCHK(use_multi(c, lg));
  WorkGuard wg(c, &c->wm);
  const int f[4] = {V_P, V_T, V_Q, V_AUX}, h[4] = {H_P, H_T, H_Q, H_R};
  return time_stencil_impl(c, prec, n, ms, f, h);
}

int qcd_encode_half(qcd_ctx* c, int n, const void* in_dev, void* codes_dev, float* scale_dev) {
  QCHK(check_ctx(c));
  if (n < 0) return fail(QCD_EINVAL, "negative count");
  if (n == 0) return QCD_OK;
  if (!in_dev || !codes_dev || !scale_dev) return fail(QCD_EINVAL, "null pointer");
  HIPCHK(launch_encode_half(n, (const double2*)in_dev, (uint4*)codes_dev, scale_dev, c->stream));
  return QCD_OK;
}

int qcd_stream_copy(qcd_ctx* c, void* dst_dev, const void* src_dev, uint64_t n_bytes) {
  QCHK(check_ctx(c));
  if (!dst_dev || !src_dev) return fail(QCD_EINVAL, "null pointer");
  if (n_bytes % 16 != 0 || ((uintptr_t)dst_dev | (uintptr_t)src_dev) % 16 != 0)
    return fail(QCD_EINVAL, "stream copy needs 16-byte multiples and alignment");
  HIPCHK(launch_stream_copy((const uint4*)src_dev, (uint4*)dst_dev, n_bytes / 16, c->stream));
  return QCD_OK;
}

}  // extern "C"
