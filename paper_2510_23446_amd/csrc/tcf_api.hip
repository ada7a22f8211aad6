// libtcf driver: C-ABI entry points, device memory plan, setup and the
// per-step dual-primal PCG.
//
// Per patch s the kept unknowns are ordered [interior i | dual b | primal p].
// Setup (once; W = sigma M + dt nu K is time invariant):
//   partial Cholesky of W over the i then b columns gives L_ii, L_bi, L_pi,
//   S_bb (Schur complement onto b, p held at zero), L_bb, L_pb and the
//   primal Schur complement S_pp;  S_Pi = sum_s N_s^T S_pp N_s;
//   G = [S_bb^-1 | Phi_b] with Phi_b = S_bb^-1 S_bp = L_bb^-T L_pb^T;
//   Q^T = [L_ii^-T | (L_bi L_ii^-1)^T | (L_pi L_ii^-1)^T].
// Per step (Sec. 2.2 implicit Euler; Sec. 3 three-field system reduced by
// two Schur complements):
//   f = M a^(l) + dt g(t_{l+1}) jhat;  [y; g_b; g_p] from Q^T and f;
//   [u; c0] = G^T g_b;  h = sum N^T (g_p - c0);  q0 = S_Pi^-1 h;
//   d = sum Bhat (u - Phi N q0);  PCG on F lambda = d with the unscaled
//   Dirichlet preconditioner sum B S_bb B^T;  recover p, a_b, a_i.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/tcf.h"
#include "tcf_device.h"
#include "tcf_internal.h"
#include "tcf_kernels.h"
#include "tcf_panel_plan.h"

using namespace tcf;

namespace {

thread_local std::string g_create_error;

// Serialises stream capture against device allocation and release in this
// process: hipFree synchronises the device and would invalidate a capture in
// progress on another thread (several handles run concurrently when serving).
std::mutex g_capture_mu;

inline int pad32(int n) { return (n + TCF_NB - 1) / TCF_NB * TCF_NB; }
// Setup factorises the patches in groups whose dense [i|b|p] blocks
// together take at most this many bytes (in FP64).
constexpr int64_t kSetupGroupBytes = (int64_t)16 << 30;
// Below the top separator the coarse nested dissection stops cutting a
// region of at most this many primal unknowns.
constexpr int kCoarseLeafMax = 256;
inline double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}
// A named range of the ROCm marker timeline (rocprofv3 --marker-trace) for
// the lifetime of the object: setup and its phases, each time step, each
// PCG solve and each refinement sweep.  The ranges are host intervals; the
// calls that synchronise (setup, a step) span their device work.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

// Gauss-Legendre rule on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double pp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = 0.0;
      for (int k = 1; k <= n; ++k) {
        const double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
      }
      pp = n * (z * p0 - p1) / (z * z - 1.0);
      const double dz = p0 / pp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = 0.0;
    for (int k = 1; k <= n; ++k) {
      const double p2 = p1;
      p1 = p0;
      p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
    }
    pp = n * (z * p0 - p1) / (z * z - 1.0);
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

template <class T>
std::vector<int> prefix_of(const std::vector<T>& counts) {
  std::vector<int> out(counts.size() + 1, 0);
  for (size_t i = 0; i < counts.size(); ++i) out[i + 1] = out[i] + (int)counts[i];
  return out;
}

}  // namespace

struct tcf_problem {
  // ---- description copy ---------------------------------------------------
  int32_t np[3];
  std::vector<double> breaks[3];
  std::vector<int32_t> nel[3], deg[3];
  std::vector<double> sigma, nu;
  std::vector<uint8_t> src;
  int32_t n_rhs = 1;
  tcf_phi_fn phi = nullptr;
  void* phi_ctx = nullptr;
  tcf_vec_fn jvol = nullptr, ainit = nullptr;
  void* vec_ctx = nullptr;
  double* d_m0 = nullptr;  // initial load int sigma A(x,0) . w (kept local order), per excitation
  std::vector<double> amp;
  double dt = 0.0;
  int32_t n_steps = 0;
  tcf_options opt;
  std::string err;

  // ---- host plan -----------------------------------------------------------
  Grid g;
  Topology topo;
  std::vector<PatchPlan> plans;
  std::vector<DevPatch> hp;  // host copy of the device patch table
  int np_tot = 0;
  int64_t n_rtot = 0, n_itot = 0, n_btot = 0, n_ptot = 0, n_bptot = 0, n_loctot = 0;
  int64_t A_elems = 0, G_elems = 0, S_elems = 0, Q_elems = 0;
  int tab_elems = 0, ptab_elems = 0;
  int n_lambda = 0, n_primal = 0, nPi_pad = 0;
  int max_nb = 0, max_ni = 0, max_np = 0, max_bp = 0, max_nr = 0;
  std::vector<int> cond_list;
  double gx[16 * 17 / 2], gw[16 * 17 / 2];

  // ---- device state ----------------------------------------------------------
  int precision = TCF_FP64;
  double pcg_tol = 1e-10;  // effective PCG tolerance (FP32 path: at least 1e-7, refined after)
  bool trace = false;      // TCF_TRACE=1: refinement sweeps on stderr
  bool fp64_ir = false;    // TCF_FP64_IR=1: refine the FP64 path too (diagnostic)
  bool is_setup = false;
  int device = 0;
  std::vector<DevBuf> bufs;
  size_t dev_bytes = 0, dev_bytes_peak = 0;
  tcf_allocator allocator{nullptr, nullptr, nullptr};  // alloc == NULL: stream-ordered HIP
  hipStream_t mem_stream = nullptr;  // stream of the current (or last) call
  // setup in patch groups: patches [chunk_begin[c], chunk_begin[c + 1]) are
  // assembled and factored together; A_off is relative to the group
  std::vector<int> chunk_begin;
  int64_t A_chunk_max = 0, G_chunk_max = 0, S_chunk_max = 0, Q_chunk_max = 0;
  // coarse factor: nested dissection of the primal unknowns over the patch
  // grid (one node = the dense inverse); the last node is inverted densely
  CoarsePlan cplan;
  std::vector<CoarseNodeDev> cnodes;      // host copy of the node table
  int c_root = -1;                        // node inverted densely (-1: no coarse)
  int c_levels = 0;                       // heights of the other nodes: 0 .. c_levels - 1
  int64_t c_front_elems = 0, c_lop_elems = 0;
  double c_bytes = 0.0;                   // algorithmic bytes of one coarse solve
  int c_launches = 0;                     // tile launches per coarse solve
  std::vector<int> c_fwd_pre, c_bwd_pre;  // per level: job prefix into tj_cfwd / tj_cbwd
  TileJob *tj_cfwd = nullptr, *tj_cbwd = nullptr;
  int* d_cT = nullptr;    // index table of the sweeps: identity over [b | y | x], then the
                          // structure lists as b and as x positions
  double* d_cw1 = nullptr;  // coarse work block, rb columns [b | y | x] (n_Pi each)
  double* d_cL = nullptr;   // per node below the top: [L_JJ^-1 | -L_JJ^-T L_SJ^T]
  // matrix-core path (rb > 4): operators as row panels (symmetric ones whole)
  bool wide = false;
  void *d_pA = nullptr, *d_pB = nullptr;  // apply + Phi panels, preconditioner panels (T)
  double* d_pC = nullptr;                 // coarse panels (FP64)
  PanelTile* d_ptile = nullptr;           // the tiles of every panel
  double* d_xg = nullptr;                 // gathered panel inputs, max(n_b, n_p) x rb
  PanelJob *pj_apply = nullptr, *pj_phi = nullptr, *pj_pre = nullptr, *pj_root = nullptr,
           *pj_cfwd = nullptr, *pj_cbwd = nullptr, *pj_gt = nullptr;
  int n_papply = 0, n_pphi = 0, n_ppre = 0, n_proot = 0, n_pgt = 0;
  // the row panels before they are split into jobs, the tiles they read,
  // and the split length per operator: 0 F apply (and G^T), 1
  // preconditioner, 2 coarse correction, 3 coarse solve
  std::vector<PanelTile> h_ptile;
  std::vector<PanelJob> w_apply, w_gt, w_pre, w_phi, w_root;
  std::vector<std::vector<PanelJob>> w_fwd, w_bwd;
  int p_eb = 8;  // element bytes of the F apply / preconditioner panels
  int chunk[4] = {16, 16, 16, 16};
  int chunk_src = 0;  // 0 default or option, 1 tune table, 2 timed at setup
  // deterministic sums (opt.deterministic): rows that several panels add
  // into are staged and summed in a fixed order, per-job quadratic forms
  // likewise; the F apply's coarse rows (sa_*) and the forward sweep's
  // ancestor rows per height (sf_*) as target -> staged-row lists
  bool determ = false;
  double* d_stage = nullptr;
  int stage_ld = 0;
  double* d_qjob = nullptr;
  int *sa_tgt = nullptr, *sa_ptr = nullptr, *sa_idx = nullptr;
  int n_sa = 0;
  std::vector<int*> sf_tgt, sf_ptr, sf_idx;
  std::vector<int> n_sf;
  double tune_us[4][5] = {};  // per operator and candidate: one launch, timed

  DevPatch* dP = nullptr;
  int *d_rloc = nullptr, *d_loc2r = nullptr, *d_brow = nullptr, *d_prank = nullptr;
  signed char *d_bsgn = nullptr, *d_isint = nullptr;
  // global edge of each local remainder unknown that is its edge's first
  // copy (lowest patch id), -1 for the other copies: the field's readout
  int64_t* d_rgid1 = nullptr;
  int *d_posp_r = nullptr, *d_posm_r = nullptr;  // multiplier -> kept-order position of its copies
  int *d_posp = nullptr, *d_posm = nullptr, *d_cptr = nullptr, *d_cidx_bp = nullptr,
      *d_cidx_r = nullptr, *d_b2bp = nullptr, *d_p2r = nullptr, *d_b2r = nullptr;
  double *d_gx = nullptr, *d_gw = nullptr, *d_tabs = nullptr, *d_ptab = nullptr;
  void *d_G = nullptr, *d_S = nullptr, *d_Q = nullptr;  // T-typed
  double *d_SPinv = nullptr;
  double *d_a = nullptr, *d_fM = nullptr, *d_ygg = nullptr, *d_yggs = nullptr, *d_zr = nullptr;
  double *d_jr = nullptr, *d_floc = nullptr, *d_res = nullptr, *d_delta = nullptr;
  int *d_kptr = nullptr, *d_kidx = nullptr;  // kept global unknown -> its local copies
  int n_kept_i = 0;
  double *d_nrm_part = nullptr, *d_nrm = nullptr, *h_nrm = nullptr;  // norms (pinned host copy)
  int *d_all = nullptr, *d_all_cprefix = nullptr, *d_all_rprefix = nullptr;
  int nt_all_c = 0, nt_all_r = 0;
  double *d_uc = nullptr, *d_vc = nullptr, *d_wb = nullptr, *d_tb = nullptr;
  double *d_h = nullptr, *d_q0 = nullptr;
  double *d_d = nullptr, *d_lam = nullptr, *d_r = nullptr, *d_z = nullptr, *d_p = nullptr,
         *d_Fp = nullptr;
  double *d_part = nullptr;  // 3 partial arrays
  int npart = 0;
  PcgScalars* d_st = nullptr;
  PcgScalars* h_st = nullptr;  // pinned
  int* d_fail = nullptr;
  double* d_field = nullptr;
  // tile storage of the per-iteration operators (lower triangles of the
  // symmetric ones): apply = S_bb^-1 and Phi_b tiles, pre = S_bb tiles (T),
  // coarse = S_Pi^-1 tiles (FP64)
  void *d_tA = nullptr, *d_tB = nullptr;
  double* d_tC = nullptr;
  TileJob *tj_apply = nullptr, *tj_phi = nullptr, *tj_pre = nullptr, *tj_coarse = nullptr;
  int n_tapply = 0, n_tphi = 0, n_tpre = 0, n_tcoarse = 0;
  double* d_acc = nullptr;  // vc | cv | q | tb accumulators of the tile path
  int* d_cmap = nullptr;    // local primal entry -> position of its coarse unknown in d_acc
  int64_t n_acc = 0;
  int *d_posp_bp = nullptr, *d_posm_bp = nullptr;
  int rb = 1;  // excitations per PCG (columns of every PCG vector and accumulator)
  bool bp_gaps = false;  // some patch has primal but no dual unknowns
  // warm starts: lambda of the first solve of the last two steps per
  // excitation ([k][0] latest, [k][1] the one before) and how many are stored
  double* d_lamh = nullptr;
  std::vector<int> lamh_n;
  // projection start (pcg_warm = 3): per excitation a ring of the newest
  // kProjMax solutions H with F H beside them, and the F-orthonormal basis
  // X, F X of their span rebuilt after every solve; work vectors and slots
  static constexpr int kProjMax = 8;
  double *d_ph = nullptr, *d_pfh = nullptr, *d_px = nullptr, *d_pfx = nullptr;
  double *d_pv = nullptr, *d_pfv = nullptr, *d_pc = nullptr;
  std::vector<int> proj_n, proj_head;
  std::vector<double> cond_est;  // per patch, after setup
  bool warm_init = false;  // the next pcg_solve starts from the lambda columns as set
  int graph_iters = 4;     // PCG iterations per replayed graph (even)
  // signed gathers of the tile path: Bhat's +-1 per b entry (F apply) and the
  // preconditioner's (the same, or D Bhat when scaled); weights of the two
  // copies in the preconditioner's jump (null: unscaled)
  double *d_bsgn_d = nullptr, *d_pre_w = nullptr, *d_zwp = nullptr, *d_zwm = nullptr;
  std::vector<int> h_posp, h_posm;  // b-space copies of each multiplier (host)
  hipStream_t cap_stream = nullptr;   // private stream used only to capture graphs
  hipGraphExec_t pcg_graph = nullptr; // graph_iters PCG iterations (parity 0, 1, 0, ...)
  bool graph_failed = false;          // capture refused: stream launches instead
  bool no_graph_call = false;         // this call issues stream launches only

  // job tables
  DotJob *dj_app_g = nullptr, *dj_app_v = nullptr, *dj_pre = nullptr;
  int *dp_app = nullptr, *dp_pre = nullptr;
  int nj_app = 0, nt_app = 0, nj_pre = 0, nt_pre = 0;
  AxpyJob *aj_phi = nullptr, *aj_ab = nullptr, *aj_ai = nullptr;
  int *ap_phi = nullptr, *ap_ai = nullptr, *a_boff_bp = nullptr, *a_boff_b = nullptr;
  int *a_boff_ai = nullptr, *a_boff_ab = nullptr;
  int nj_phi = 0, nt_phi = 0, nj_ai = 0, nt_ai = 0;
  int *d_cond = nullptr, *d_cond_cprefix = nullptr, *d_cond_rprefix = nullptr;
  int nt_cond_c = 0, nt_cond_r = 0;
  // 64-wide blocks of the matrix-core condensation (columns) and recovery
  // (interior rows)
  int *d_cond_wprefix = nullptr, *d_all_wprefix = nullptr, *d_all_iprefix = nullptr;
  int nt_cond_w = 0, nt_all_w = 0, nt_all_i = 0;

  // ---- kernel timing -------------------------------------------------------------
  struct Pend { int g, it; hipEvent_t a, b; };
  bool prof_on = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<Pend> pend;
  double prof_ms[TCF_KG_COUNT] = {0};
  int64_t prof_n[TCF_KG_COUNT] = {0};
  double prof_bytes[TCF_KG_COUNT] = {0};
  double prof_flops[TCF_KG_COUNT] = {0};
  int cur_it = -1;  // PCG iteration of the launches being issued (-1: outside PCG)
  int cur_sweep = 0;  // refinement sweep of the solve being issued (0: first solve)
#define TCF_PRED_KINDS 8
  int pred_iters[TCF_PRED_KINDS] = {0};  // iterations of the last solve of each sweep
  hipEvent_t ev_get() {
    if (ev_pool.empty()) {
      hipEvent_t e;
      (void)hipEventCreate(&e);
      return e;
    }
    hipEvent_t e = ev_pool.back();
    ev_pool.pop_back();
    return e;
  }
  // drop_from: PCG launches with iteration >= drop_from are discarded
  void prof_flush(int drop_from) {
    for (auto& p : pend) {
      if (!(p.it >= 0 && p.it >= drop_from)) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
          prof_ms[p.g] += ms;
          prof_n[p.g]++;
        }
      }
      ev_pool.push_back(p.a);
      ev_pool.push_back(p.b);
    }
    pend.clear();
  }

  // ---- stats -------------------------------------------------------------------
  int steps_done = 0;
  int last_iters = 0, max_iters = 0, nonconv = 0, last_ir = 0, fail_patch = -2;
  int64_t total_iters = 0;
  double last_rel = 0.0, last_ir_res = 0.0, setup_ms = 0.0, step_ms_total = 0.0;
  std::vector<int32_t> log_iters, log_ir;
  std::vector<double> log_ms;

  ~tcf_problem() {
    std::lock_guard<std::mutex> lk(g_capture_mu);
    if (pcg_graph) (void)hipGraphExecDestroy(pcg_graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (auto& p : pend) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    for (auto& b : bufs)
      if (b.p) give_back(b.p);
    if (h_st) (void)hipHostFree(h_st);
    if (h_nrm) (void)hipHostFree(h_nrm);
  }

  // one buffer back to its allocator, on the current call's stream
  void give_back(void* p) {
    if (allocator.alloc) allocator.free(allocator.ctx, p, (void*)mem_stream);
    else (void)hipFreeAsync(p, mem_stream);
  }
  template <class T>
  int alloc(T** out, size_t count) {
    void* p = nullptr;
    // whole multiples of 256 bytes: every buffer starts on a 256-byte boundary
    // whichever allocator serves it
    const size_t bytes = (std::max<size_t>(count, 1) * sizeof(T) + 255) / 256 * 256;
    bool ok;
    {
      std::lock_guard<std::mutex> lk(g_capture_mu);
      if (allocator.alloc) {
        p = allocator.alloc(allocator.ctx, bytes, (void*)mem_stream);
        ok = p != nullptr;
      } else {
        ok = hipMallocAsync(&p, bytes, mem_stream) == hipSuccess;
        if (!ok) (void)hipGetLastError();
      }
    }
    if (!ok) {
      err = "device allocation of " + std::to_string(bytes) + " bytes failed";
      return TCF_ENOMEM;
    }
    // the block may have been given back on this stream by work still in
    // flight, and the handle fills some buffers with blocking copies (the
    // null stream): let that work finish first
    if (hipStreamSynchronize(mem_stream) != hipSuccess) {
      (void)hipGetLastError();
      give_back(p);
      err = "stream synchronisation after a device allocation failed";
      return TCF_EHIP;
    }
    bufs.push_back({p, bytes});
    dev_bytes += bytes;
    dev_bytes_peak = std::max(dev_bytes_peak, dev_bytes);
    *out = (T*)p;
    return TCF_OK;
  }
  void release(void* p) {
    for (auto& b : bufs)
      if (b.p == p) {
        std::lock_guard<std::mutex> lk(g_capture_mu);
        give_back(b.p);
        dev_bytes -= b.bytes;
        b.p = nullptr;
        b.bytes = 0;
      }
  }
  template <class T>
  int upload(T** out, const std::vector<T>& v) {
    int rc = alloc(out, v.size());
    if (rc) return rc;
    hipError_t e = hipSuccess;
    if (!v.empty()) {
      std::lock_guard<std::mutex> lk(g_capture_mu);
      e = hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
      err = "hipMemcpy upload failed";
      return TCF_EHIP;
    }
    return TCF_OK;
  }
  size_t footprint(int prec) const;
};

#define HIPCHK(expr)                                                        \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess) {                                                 \
      h->err = std::string(#expr) + ": " + hipGetErrorString(e_);           \
      return TCF_EHIP;                                                      \
    }                                                                       \
  } while (0)
#define RCCHK(expr)        \
  do {                     \
    int rc_ = (expr);      \
    if (rc_) return rc_;   \
  } while (0)

template <class F>
static inline void timed(tcf_problem* h, int g, hipStream_t st, F&& f) {
  if (!h->prof_on) {
    f();
    return;
  }
  // every timed group is exactly one kernel launch; the events ride on it
  hipEvent_t a = h->ev_get(), b = h->ev_get();
  set_launch_events(a, b);
  f();
  if (launch_events_pending()) {  // nothing was launched
    set_launch_events(nullptr, nullptr);
    h->ev_pool.push_back(a);
    h->ev_pool.push_back(b);
    return;
  }
  h->pend.push_back({g, h->cur_it, a, b});
}

// Algorithmic bytes of one launch of each kernel group (see tcf.h).
static void compute_alg_bytes(tcf_problem* h) {
  const double w = h->precision == TCF_FP64 ? 8.0 : 4.0;  // operator storage
  double app = 0, pre = 0, phi = 0, cond = 0, rec = 0;
  for (int s = 0; s < h->np_tot; ++s) {
    const DevPatch& d = h->hp[s];
    const double nb = d.n_b, np_ = d.n_p, ni = d.n_i;
    if (d.n_b > 0) {
      app += (nb * (nb + 1) / 2 + nb * np_) * w + (2 * nb + np_) * 8;
      pre += nb * (nb + 1) / 2 * w + 2 * nb * 8;
      if (d.n_p > 0) phi += nb * np_ * w + (np_ + 2 * nb) * 8;
    }
    const double qb = (ni * (ni + 1) / 2 + ni * (nb + np_)) * w;
    if (d.cond) cond += qb + (2 * (ni + nb + np_)) * 8;
    rec += qb + (d.n_r + ni) * 8;
  }
  const double nP = h->n_primal;
  // algorithmic flops: 2 per matrix entry and batch column, symmetric
  // matrices whole, triangles as triangles
  double fa = 0, fp = 0, fphi = 0, fc = 0;
  for (int s = 0; s < h->np_tot; ++s) {
    const DevPatch& d = h->hp[s];
    const double nb = d.n_b, np_ = d.n_p;
    fa += 2 * (nb * nb + nb * np_);
    fp += 2 * nb * nb;
    fphi += 2 * nb * np_;
  }
  for (size_t i = 0; i < h->cnodes.size(); ++i) {
    const double nj = h->cnodes[i].nj, ns = h->cnodes[i].ns;
    fc += (int)i == h->c_root ? 2 * nj * nj : 2 * (nj * (nj + 1) + 2 * nj * ns);
  }
  const double R = h->rb;
  h->prof_flops[TCF_KG_APPLY] = R * fa;
  h->prof_flops[TCF_KG_PRECOND] = R * fp;
  h->prof_flops[TCF_KG_PHI] = R * fphi;
  h->prof_flops[TCF_KG_COARSE] = R * fc;
  h->prof_bytes[TCF_KG_APPLY] = app;
  h->prof_bytes[TCF_KG_PRECOND] = pre;
  h->prof_bytes[TCF_KG_PHI] = phi;
  h->prof_bytes[TCF_KG_COARSE] = nP > 0 ? h->c_bytes : 0.0;  // per coarse solve
  h->prof_bytes[TCF_KG_CONDENSE] = cond;
  h->prof_bytes[TCF_KG_RECOVER] = rec;
}

// Device bytes the handle needs at its peak: the resident set (operators in
// their stored precision, their tiles, vectors) plus the largest transient
// of setup (one patch group's dense blocks with the coarse fronts, the
// coarse factor's operators, or the coarse operators while they are tiled).
size_t tcf_problem::footprint(int prec) const {
  const double w = prec == TCF_FP64 ? 8 : 4;          // stored operators
  const double wf = prec == TCF_FP32_FULL_IR ? 4 : 8;  // factorisation
  double ops = (double)(G_elems + S_elems + Q_elems) * w;
  double tiles = 0.0, ctiles = 0.0;
  // narrow batches: lower tiles of the symmetric blocks, each tile of Phi_b
  // once; wide batches (row panels): the symmetric blocks whole, Phi_b and
  // the coarse factor's blocks once per sweep that reads them
  for (const DevPatch& d : hp) {
    const double Tb = (d.n_b + 63) / 64, Tp = (d.n_p + 63) / 64;
    tiles += (wide ? 2 * (Tb * Tb + Tb * Tp) : Tb * (Tb + 1) + Tb * Tp) * 4096.0 * w;
  }
  double root_inv = 0.0;
  for (size_t i = 0; i < cnodes.size(); ++i) {
    const CoarseNodeDev& c = cnodes[i];
    const double Tj = (c.nj + 63) / 64, Ts = (c.ns + 63) / 64;
    if ((int)i == c_root) {
      ctiles += (wide ? Tj * Tj : Tj * (Tj + 1) / 2) * 4096.0 * 8;
      root_inv = (double)c.nj_pad * c.nj_pad * 8;
    } else {
      ctiles += (wide ? 2 : 1) * (Tj * (Tj + 1) / 2 + Tj * Ts) * 4096.0 * 8;
    }
  }
  const double npm = std::max(n_primal, 1);
  double vec = (double)n_rtot * n_rhs * 8 * 6 + (double)n_rtot * rb * 8 * 4;
  vec += ((double)n_bptot * 16 + (double)n_btot * 16 + (double)n_lambda * 8 * 8) * rb;
  vec += (double)rb * (n_bptot + 3 * npm + n_btot + 2 * TCF_QSLOTS) * 8 + npm * 8 * (4 + rb);
  if (wide) vec += (double)std::max(n_btot, n_ptot) * rb * 8;  // gathered panel inputs
  vec += ((double)n_bptot + 3 * npm) * rb * 8;  // per-column v and coarse work block
  vec += (double)(tab_elems + ptab_elems) * 8 + (double)n_rtot * 24 + (double)n_loctot * 4;
  vec += (double)g.n_edges() * 8 + (double)n_rtot * 8;  // field, copy maps
  if (ainit && !cond_list.empty()) vec += (double)n_rtot * n_rhs * 8;  // initial load
  if (opt.pcg_warm == 1 || opt.pcg_warm == 2) vec += (double)n_lambda * 2 * n_rhs * 8;
  if (opt.pcg_warm == 3) vec += (double)tcf_problem::kProjMax * 4 * n_lambda * n_rhs * 8;
  const double fronts = (double)c_front_elems * 8, lops = (double)c_lop_elems * 8;
  // a group's dense blocks, plus the inverted 32 x 32 diagonal blocks of
  // its triangular solves
  double grp = (double)A_chunk_max * wf * (1.0 + 32.0 / 1024) + fronts;
  if (prec == TCF_FP32_IR) grp += (double)(G_chunk_max + S_chunk_max + Q_chunk_max) * 8;
  const double coarse = fronts + lops + root_inv;
  const double pack = tiles + ctiles + lops + root_inv;
  const double peak = ops + vec + std::max(grp, std::max(coarse, pack));
  // the tiles stay resident after setup
  const double resident = ops + vec + tiles + ctiles;
  return (size_t)(std::max(peak, resident) * 1.02) + ((size_t)8 << 20);
}

// ============================================================================
// Plan: sizes, offsets and index tables (host only)
// ============================================================================
// Algorithmic bytes and launches of one coarse solve under a plan: the
// dense top block's lower triangle once (it serves both triangles), every
// other node's L_JJ^-1 triangle and its structure block twice (forward and
// backward sweep), FP64.
static void coarse_cost(const CoarsePlan& cp, double& bytes, int& levels) {
  bytes = 0.0;
  levels = 0;
  const int nn = (int)cp.nodes.size();
  for (int i = 0; i < nn; ++i) {
    const CoarseNode& c = cp.nodes[i];
    const double nj = c.nj, ns = (double)c.S.size();
    if (i == nn - 1) {
      bytes += nj * (nj + 1) / 2 * 8 + 2 * nj * 8;
    } else {
      bytes += 2 * (nj * (nj + 1) / 2 + nj * ns) * 8 + 4 * (nj + ns) * 8;
      levels = std::max(levels, c.height + 1);
    }
  }
}

// Chooses between the dense inverse of S_Pi and the nested-dissection
// factor (coarse_mode 0: whichever a simple model of one solve, streamed
// bytes at 5 TB/s plus 3 us per launch, finds cheaper; the dense inverse
// is also ruled out when its setup would need more than 64 GiB), and lays
// out the fronts, operator blocks and node table.
static void plan_coarse_solver(tcf_problem* h) {
  const int n = h->n_primal;
  h->cnodes.clear();
  h->c_root = -1;
  h->c_levels = 0;
  h->c_front_elems = h->c_lop_elems = 0;
  h->c_bytes = 0.0;
  h->c_launches = 0;
  if (n == 0) return;
  CoarsePlan dense;
  dense.nd.resize(n);
  std::iota(dense.nd.begin(), dense.nd.end(), 0);
  dense.nodes.resize(1);
  dense.nodes[0].nj = n;
  int mode = h->opt.coarse_mode;
  if (mode != 1) {
    CoarsePlan nd = plan_coarse(h->plans, h->np, n, 0, kCoarseLeafMax);
    double bd, bn;
    int ld, ln;
    coarse_cost(dense, bd, ld);
    coarse_cost(nd, bn, ln);
    const double td = bd / 5e12 + 3e-6;
    const double tn = bn / 5e12 + 3e-6 * (2 * ln + 2);
    const double dense_setup = 2.0 * pad32(n) * (double)pad32(n) * 8;
    if (mode == 2 || (nd.nodes.size() > 1 && (tn < td || dense_setup > 64.0 * (1 << 30)))) {
      h->cplan = std::move(nd);
      mode = 2;
    } else {
      mode = 1;
    }
  }
  if (mode == 1) h->cplan = std::move(dense);
  const CoarsePlan& cp = h->cplan;
  const int nn = (int)cp.nodes.size();
  h->cnodes.resize(nn);
  int64_t fo = 0, lo = 0;
  int s_off = 0;
  for (int i = 0; i < nn; ++i) {
    const CoarseNode& c = cp.nodes[i];
    CoarseNodeDev& d = h->cnodes[i];
    d.j0 = c.j0;
    d.nj = c.nj;
    d.nj_pad = pad32(c.nj);
    d.ns = (int)c.S.size();
    d.nf = d.nj_pad + pad32(d.ns);
    d.s_off = s_off;
    s_off += d.ns;
    d.parent = c.parent;
    d.pad = 0;
    d.f_off = fo;
    fo += (int64_t)d.nf * d.nf;
    d.l_off = lo;
    if (i < nn - 1) {
      lo += (int64_t)d.nj_pad * (d.nj + d.ns);
      h->c_levels = std::max(h->c_levels, c.height + 1);
    }
  }
  h->c_root = nn - 1;
  h->c_front_elems = fo;
  h->c_lop_elems = lo;
  int lev;
  coarse_cost(cp, h->c_bytes, lev);
  h->c_launches = nn > 1 ? 2 * h->c_levels + 1 : 1;  // tile launches (timed group)
}

static void build_plan(tcf_problem* h) {
  const int np = h->np_tot;
  h->hp.assign(np, DevPatch());
  int64_t r_off = 0, i_off = 0, b_off = 0, p_off = 0, bp_off = 0, loc_off = 0;
  int64_t A = 0, G = 0, S = 0, Q = 0;
  int tab = 0, ptab = 0;
  h->cond_list.clear();
  for (int s = 0; s < np; ++s) {
    const PatchPlan& pp = h->plans[s];
    DevPatch& d = h->hp[s];
    for (int a = 0; a < 3; ++a) {
      d.m[a] = pp.m[a];
      d.nel[a] = pp.nel[a];
      d.deg[a] = pp.deg[a];
      d.lo[a] = pp.lo[a];
      d.hi[a] = pp.hi[a];
    }
    d.sigma = pp.sigma;
    d.nu = pp.nu;
    d.n_i = pp.n_i; d.n_b = pp.n_b; d.n_p = pp.n_p; d.n_r = pp.n_r(); d.n_loc = pp.n_loc;
    d.ni_pad = pad32(pp.n_i); d.nb_pad = pad32(pp.n_b); d.np_pad = pad32(pp.n_p);
    d.nr_pad = d.ni_pad + d.nb_pad + d.np_pad;
    d.src = pp.src ? 1 : 0;
    d.cond = pp.sigma > 0 ? 1 : 0;
    if (d.cond) h->cond_list.push_back(s);
    d.A_off = A; A += (int64_t)d.nr_pad * d.nr_pad;  // made group-relative below
    d.G_off = G; G += (int64_t)d.nb_pad * (d.n_b + d.n_p);
    d.S_off = S; S += (int64_t)d.nb_pad * d.n_b;
    d.Q_off = Q; Q += (int64_t)d.ni_pad * d.n_r;
    d.r_off = (int)r_off; r_off += d.n_r;
    d.i_off = (int)i_off; i_off += d.n_i;
    d.b_off = (int)b_off; b_off += d.n_b;
    d.p_off = (int)p_off; p_off += d.n_p;
    d.bp_off = (int)bp_off; bp_off += d.n_b + d.n_p;
    d.loc_off = (int)loc_off; loc_off += d.n_loc;
    for (int a = 0; a < 3; ++a) {
      const int m = d.m[a];
      d.tab_off[a] = tab;
      tab += 2 * m * m + (m - 1) * (m - 1) + (m - 1) * m;
      d.nq_load[a] = d.nel[a] * (d.deg[a] + 3);
      d.ptab_off[a] = ptab;
      ptab += d.nq_load[a] * (3 * m + 1);
    }
    h->max_nb = std::max(h->max_nb, d.n_b);
    h->max_ni = std::max(h->max_ni, d.n_i);
    h->max_np = std::max(h->max_np, d.n_p);
    h->max_bp = std::max(h->max_bp, d.n_b + d.n_p);
    h->max_nr = std::max(h->max_nr, d.n_r);
  }
  h->n_rtot = r_off; h->n_itot = i_off; h->n_btot = b_off; h->n_ptot = p_off;
  h->n_bptot = bp_off; h->n_loctot = loc_off;
  h->A_elems = A; h->G_elems = G; h->S_elems = S; h->Q_elems = Q;
  h->tab_elems = tab; h->ptab_elems = ptab;
  h->n_lambda = (int)h->topo.dual.size();
  h->n_primal = (int)h->topo.primal.size();
  h->nPi_pad = pad32(h->n_primal);
  for (int n = 1, o = 0; n <= 16; o += n, ++n) gauss_legendre(n, h->gx + o, h->gw + o);
  // setup groups: consecutive patches whose dense [i|b|p] blocks together
  // stay within the budget (a single larger patch forms its own group)
  const int64_t budget =
      (h->opt.setup_group_mb > 0 ? ((int64_t)h->opt.setup_group_mb << 20) : kSetupGroupBytes) / 8;
  h->chunk_begin.assign(1, 0);
  h->A_chunk_max = h->G_chunk_max = h->S_chunk_max = h->Q_chunk_max = 0;
  auto close = [&](int c0, int c1) {
    const DevPatch &f = h->hp[c0], &l = h->hp[c1 - 1];
    h->A_chunk_max = std::max(h->A_chunk_max, l.A_off + (int64_t)l.nr_pad * l.nr_pad - f.A_off);
    h->G_chunk_max = std::max(h->G_chunk_max, l.G_off + (int64_t)l.nb_pad * (l.n_b + l.n_p) - f.G_off);
    h->S_chunk_max = std::max(h->S_chunk_max, l.S_off + (int64_t)l.nb_pad * l.n_b - f.S_off);
    h->Q_chunk_max = std::max(h->Q_chunk_max, l.Q_off + (int64_t)l.ni_pad * l.n_r - f.Q_off);
    const int64_t base = f.A_off;
    for (int t = c0; t < c1; ++t) h->hp[t].A_off -= base;
    h->chunk_begin.push_back(c1);
  };
  int c0 = 0;
  for (int s = 0; s < np; ++s) {
    const int64_t end = h->hp[s].A_off + (int64_t)h->hp[s].nr_pad * h->hp[s].nr_pad;
    if (s > c0 && end - h->hp[c0].A_off > budget) {
      close(c0, s);
      c0 = s;
    }
  }
  if (np > 0) close(c0, np);
  h->A_elems = h->A_chunk_max;
  plan_coarse_solver(h);
}

// ============================================================================
// C-ABI
// ============================================================================
extern "C" {

void tcf_default_options(tcf_options* o) {
  o->precision = TCF_FP64;
  o->pcg_rtol = 1e-10;
  o->pcg_maxit = 0;
  o->ir_rtol = 1e-8;
  o->ir_maxit = 10;
  o->check_every = 8;
  o->use_graph = 1;
  o->rhs_batch = 0;
  o->pcg_warm = 0;
  o->precond_scaling = 0;
  o->coarse_mode = 0;
  o->setup_group_mb = 0;
  o->panel_chunk = 0;
  o->autotune = 0;
  o->tune_table = nullptr;
  o->deterministic = 0;
}

const char* tcf_last_error(const tcf_problem* h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

int tcf_create(const tcf_problem_desc* desc, const tcf_options* opts,
               const tcf_allocator* allocator, tcf_problem** out) {
  if (!out) { g_create_error = "null output handle"; return TCF_EINVAL; }
  *out = nullptr;
  if (!desc) { g_create_error = "null description"; return TCF_EINVAL; }
  std::string e = validate_desc(*desc);
  if (!e.empty()) { g_create_error = e; return TCF_EINVAL; }
  std::unique_ptr<tcf_problem> h(new (std::nothrow) tcf_problem());
  if (!h) { g_create_error = "out of host memory"; return TCF_ENOMEM; }
  if (opts) h->opt = *opts; else tcf_default_options(&h->opt);
  if (allocator && allocator->alloc) {
    if (!allocator->free) { g_create_error = "allocator without a free function"; return TCF_EINVAL; }
    h->allocator = *allocator;
  }
  if (h->opt.precision != TCF_FP64 && h->opt.precision != TCF_FP32_IR &&
      h->opt.precision != TCF_FP32_FULL_IR) {
    g_create_error = "unknown precision"; return TCF_EINVAL;
  }
  if (!(h->opt.pcg_rtol > 0)) { g_create_error = "pcg_rtol <= 0"; return TCF_EINVAL; }
  if (h->opt.check_every <= 0) h->opt.check_every = 8;
  if (h->opt.ir_maxit <= 0) h->opt.ir_maxit = 10;
  if (h->opt.pcg_warm < 0 || h->opt.pcg_warm > 3) { g_create_error = "pcg_warm not in 0..3"; return TCF_EINVAL; }
  if (h->opt.precond_scaling < 0 || h->opt.precond_scaling > 1) {
    g_create_error = "precond_scaling not in 0..1";
    return TCF_EINVAL;
  }
  if (h->opt.coarse_mode < 0 || h->opt.coarse_mode > 2) {
    g_create_error = "coarse_mode not in 0..2";
    return TCF_EINVAL;
  }
  h->precision = h->opt.precision;
  h->pcg_tol = h->precision == TCF_FP64 ? h->opt.pcg_rtol : std::max(h->opt.pcg_rtol, 1e-7);
  {
    const char* tr = std::getenv("TCF_TRACE");
    h->trace = tr && tr[0] == '1';
    const char* fi = std::getenv("TCF_FP64_IR");
    h->fp64_ir = fi && fi[0] == '1';
    const char* gi = std::getenv("TCF_GRAPH_ITERS");
    if (gi) h->graph_iters = std::max(2, std::min(8, std::atoi(gi) / 2 * 2));
  }
  for (int a = 0; a < 3; ++a) {
    h->np[a] = desc->np[a];
    h->breaks[a].assign(desc->breaks[a], desc->breaks[a] + desc->np[a] + 1);
    h->nel[a].assign(desc->nel[a], desc->nel[a] + desc->np[a]);
    h->deg[a].assign(desc->deg[a], desc->deg[a] + desc->np[a]);
  }
  const int np = desc->np[0] * desc->np[1] * desc->np[2];
  h->np_tot = np;
  h->sigma.assign(desc->sigma, desc->sigma + np);
  h->nu.assign(desc->nu, desc->nu + np);
  h->src.assign(desc->src_mask, desc->src_mask + np);
  h->n_rhs = desc->n_rhs;
  // excitations per batched PCG
  // up to 4 columns on the vector tile kernels; more on the matrix cores,
  // in widths of 8, 16 or 32 (idle columns carry zero right-hand sides)
  {
    const int want = std::min(h->n_rhs, h->opt.rhs_batch > 0 ? std::min(h->opt.rhs_batch, 32) : 32);
    h->rb = want <= 4 ? want : (want <= 8 ? 8 : (want <= 16 ? 16 : 32));
    h->determ = h->opt.deterministic != 0;
    h->wide = h->rb > 4 || h->determ;
  }
  h->phi = desc->phi;
  h->phi_ctx = desc->phi_ctx;
  h->jvol = desc->jvol;
  h->ainit = desc->ainit;
  h->vec_ctx = desc->vec_ctx;
  h->dt = desc->dt;
  h->n_steps = desc->n_steps;
  if (desc->n_steps > 0) h->amp.assign(desc->amp, desc->amp + (size_t)desc->n_rhs * desc->n_steps);
  // a private description pointing at the copies
  tcf_problem_desc d = *desc;
  for (int a = 0; a < 3; ++a) {
    d.breaks[a] = h->breaks[a].data();
    d.nel[a] = h->nel[a].data();
    d.deg[a] = h->deg[a].data();
  }
  d.sigma = h->sigma.data();
  d.nu = h->nu.data();
  d.src_mask = h->src.data();
  try {
    h->g = build_grid(d);
    e = compute_topology(d, h->g, h->topo, h->plans);
    if (e.empty()) build_plan(h.get());
  } catch (const std::bad_alloc&) {
    g_create_error = "out of host memory in topology or device plan";
    return TCF_ENOMEM;
  }
  if (!e.empty()) { g_create_error = e; return TCF_EINVAL; }
  *out = h.release();
  return TCF_OK;
}

int tcf_footprint(const tcf_problem* h, size_t* b64, size_t* b32) {
  if (!h) return TCF_EINVAL;
  if (b64) *b64 = h->footprint(TCF_FP64);
  if (b32) *b32 = h->footprint(TCF_FP32_IR);
  return TCF_OK;
}

int tcf_get_topology(const tcf_problem* h, int32_t kind, int64_t* out, size_t* len) {
  if (!h || !len) return TCF_EINVAL;
  std::vector<int64_t> tmp;
  const std::vector<int64_t>* src = &tmp;
  try {
  switch (kind) {
    case TCF_TOPO_COUNTS:
      tmp = {h->g.n_edges(), h->g.n_nodes(), h->topo.n_vertices_H, h->topo.n_plain,
             h->topo.n_floating, (int64_t)h->topo.dual.size(), (int64_t)h->topo.primal.size(),
             h->topo.n_kept};
      break;
    case TCF_TOPO_DIRICHLET: src = &h->topo.dirichlet; break;
    case TCF_TOPO_TREE_I: src = &h->topo.tree_I; break;
    case TCF_TOPO_TREE_GAMMA: src = &h->topo.tree_gamma; break;
    case TCF_TOPO_PRIMAL: src = &h->topo.primal; break;
    case TCF_TOPO_DUAL: src = &h->topo.dual; break;
    case TCF_TOPO_INTERIOR: src = &h->topo.interior; break;
    case TCF_TOPO_MULT: src = &h->topo.mult; break;
    case TCF_TOPO_N:
      for (int s = 0; s < h->np_tot; ++s) {
        const PatchPlan& pp = h->plans[s];
        for (int j = 0; j < pp.n_p; ++j) {
          tmp.push_back(s);
          tmp.push_back(pp.r_gid[pp.n_i + pp.n_b + j]);
          tmp.push_back(pp.p_rank[j]);
        }
      }
      break;
    case TCF_TOPO_COARSE:
      tmp.assign(h->cplan.nd.begin(), h->cplan.nd.end());
      for (const CoarseNode& c : h->cplan.nodes) {
        tmp.insert(tmp.end(), {c.j0, c.nj, c.parent, c.height, (int64_t)c.S.size()});
        tmp.insert(tmp.end(), c.S.begin(), c.S.end());
      }
      break;
    case TCF_TOPO_LOOP:
    case TCF_TOPO_LOOP_PLAN:
    case TCF_TOPO_LOOP_PSI: {
      // host plans of the loop split: built on demand, so allocation or a
      // lookup can fail here; no exception crosses the C-ABI
      std::string err;
      try {
        if (kind == TCF_TOPO_LOOP) tmp = loop_rows(h->g, h->topo, h->plans);
        else if (kind == TCF_TOPO_LOOP_PLAN) tmp = loop_plan(h->g, h->topo, h->plans);
        else tmp = loop_psi(h->g, h->topo, h->plans, err);
      } catch (const std::bad_alloc&) {
        const_cast<tcf_problem*>(h)->err = "out of host memory in the loop-split plan";
        return TCF_ENOMEM;
      } catch (const std::exception& ex) {
        err = std::string("loop-split plan: ") + ex.what();
      }
      if (!err.empty()) {
        const_cast<tcf_problem*>(h)->err = err;
        return TCF_EINVAL;
      }
      break;
    }
    default:
      return TCF_EINVAL;
  }
  } catch (const std::bad_alloc&) {
    const_cast<tcf_problem*>(h)->err = "out of host memory in the topology query";
    return TCF_ENOMEM;
  }
  if (!out) { *len = src->size(); return TCF_OK; }
  if (*len < src->size()) {
    const_cast<tcf_problem*>(h)->err = "topology buffer too small";
    return TCF_EINVAL;
  }
  std::copy(src->begin(), src->end(), out);
  *len = src->size();
  return TCF_OK;
}

int tcf_get_stats(const tcf_problem* h, tcf_stats* st) {
  if (!h || !st) return TCF_EINVAL;
  std::memset(st, 0, sizeof(*st));
  st->n_patches = h->np_tot;
  st->n_edges = h->g.n_edges();
  st->n_kept = h->topo.n_kept;
  st->n_lambda = h->n_lambda;
  st->n_primal = h->n_primal;
  st->n_tree_I = (int64_t)h->topo.tree_I.size();
  st->steps_done = h->steps_done;
  st->last_pcg_iters = h->last_iters;
  st->total_pcg_iters = h->total_iters;
  st->max_pcg_iters = h->max_iters;
  st->last_ir_sweeps = h->last_ir;
  st->nonconverged_steps = h->nonconv;
  st->fail_patch = h->fail_patch;
  st->last_rel_residual = h->last_rel;
  st->last_ir_residual = h->last_ir_res;
  st->setup_ms = h->setup_ms;
  st->step_ms_total = h->step_ms_total;
  st->device_bytes = h->dev_bytes;
  {
    double f = 0.0;
    for (int s = 0; s < h->np_tot; ++s) {
      const double ni = h->hp[s].n_i, nb = h->hp[s].n_b, np_ = h->hp[s].n_p;
      const double nbp = nb + np_;
      f += ni * ni * ni / 3 + ni * ni * nbp + ni * nbp * nbp;  // interior elimination
      f += nb * nb * nb / 3 + nb * nb * np_ + nb * np_ * np_;  // dual block
      f += nb * nb * nb / 3 + nb * nb * (nb + np_);             // S_bb^-1 and Phi_b
      f += ni * ni * ni / 3 + ni * ni * nbp;                    // Q^T
    }
    // coarse: per node below the top its partial Cholesky, L_JJ^-1 and
    // L_JJ^-T L_SJ^T; the top block's Cholesky and inverse
    for (size_t i = 0; i < h->cnodes.size(); ++i) {
      const double nj = h->cnodes[i].nj, ns = h->cnodes[i].ns;
      if ((int)i == h->c_root) f += 5 * nj * nj * nj / 3;
      else f += 2 * nj * nj * nj / 3 + 2 * nj * nj * ns + nj * ns * ns;
    }
    st->setup_flops = f;
  }
  st->coarse_nodes = (int32_t)h->cnodes.size();
  st->coarse_launches = h->c_launches;
  st->coarse_root = h->c_root >= 0 ? h->cnodes[h->c_root].nj : 0;
  st->setup_chunks = (int32_t)h->chunk_begin.size() - 1;
  st->coarse_bytes = h->c_bytes;
  st->device_bytes_peak = h->dev_bytes_peak;
  st->rhs_batch = h->rb;
  st->panel_jobs = h->n_papply;
  for (int g = 0; g < 4; ++g) st->panel_chunk[g] = h->wide ? h->chunk[g] : 0;
  st->panel_chunk_src = h->chunk_src;
  for (int g = 0; g < 4; ++g)
    for (int c = 0; c < 5; ++c) st->panel_tune_us[g * 5 + c] = h->tune_us[g][c];
  st->cond_est_max = 0.0;
  st->cond_est_patch = -1;
  for (size_t s = 0; s < h->cond_est.size(); ++s)
    if (h->cond_est[s] > st->cond_est_max) {
      st->cond_est_max = h->cond_est[s];
      st->cond_est_patch = (int32_t)s;
    }
  return TCF_OK;
}

int tcf_get_cond_est(const tcf_problem* h, double* out, size_t* len) {
  if (!h || !len) return TCF_EINVAL;
  if (h->cond_est.empty()) return TCF_ESTATE;
  if (!out) {
    *len = h->cond_est.size();
    return TCF_OK;
  }
  if (*len < h->cond_est.size()) return TCF_EINVAL;
  std::copy(h->cond_est.begin(), h->cond_est.end(), out);
  *len = h->cond_est.size();
  return TCF_OK;
}

int tcf_get_step_log(const tcf_problem* h, int32_t n, int32_t* it, int32_t* ir, double* ms) {
  if (!h || n < 0) return TCF_EINVAL;
  n = std::min<int32_t>(n, (int32_t)h->log_iters.size());
  const size_t o = h->log_iters.size() - n;
  for (int k = 0; k < n; ++k) {
    if (it) it[k] = h->log_iters[o + k];
    if (ir) ir[k] = h->log_ir[o + k];
    if (ms) ms[k] = h->log_ms[o + k];
  }
  return TCF_OK;
}

void tcf_destroy(tcf_problem* h) { delete h; }

int tcf_profile_enable(tcf_problem* h, int32_t on) {
  if (!h) return TCF_EINVAL;
  h->prof_flush(INT32_MAX);
  h->prof_on = on != 0;
  for (int g = 0; g < TCF_KG_COUNT; ++g) { h->prof_ms[g] = 0; h->prof_n[g] = 0; }
  compute_alg_bytes(h);
  return TCF_OK;
}

int tcf_copy_probe(size_t bytes, void* stream) {
  const size_t n32 = bytes / 32;
  if (n32 == 0) return TCF_EINVAL;
  void *a = nullptr, *b = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_capture_mu);
    if (hipMalloc(&a, n32 * 32) != hipSuccess) return TCF_ENOMEM;
    if (hipMalloc(&b, n32 * 32) != hipSuccess) {
      (void)hipFree(a);
      return TCF_ENOMEM;
    }
  }
  hipStream_t st = (hipStream_t)stream;
  int rc = TCF_OK;
  if (hipMemsetAsync(a, 0, n32 * 32, st) != hipSuccess) rc = TCF_EHIP;
  if (rc == TCF_OK) launch_copy_probe((int64_t)n32, a, b, st);
  if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) rc = TCF_EHIP;
  std::lock_guard<std::mutex> lk(g_capture_mu);
  (void)hipFree(a);
  (void)hipFree(b);
  return rc;
}

int tcf_bandwidth_probe(size_t bytes, void* stream, double* read_gbs, double* copy_gbs) {
  const size_t n32 = bytes / 32;
  if (n32 == 0 || !read_gbs || !copy_gbs) return TCF_EINVAL;
  void *a = nullptr, *b = nullptr, *o = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_capture_mu);
    if (hipMalloc(&a, n32 * 32) != hipSuccess) return TCF_ENOMEM;
    if (hipMalloc(&b, n32 * 32) != hipSuccess || hipMalloc(&o, 8) != hipSuccess) {
      (void)hipFree(a);
      if (b) (void)hipFree(b);
      return TCF_ENOMEM;
    }
  }
  hipStream_t st = (hipStream_t)stream;
  int rc = TCF_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = TCF_EHIP;
  if (!rc && (hipMemsetAsync(a, 0, n32 * 32, st) != hipSuccess ||
              hipMemsetAsync(b, 0, n32 * 32, st) != hipSuccess))
    rc = TCF_EHIP;
  // best of 3 after one warm launch each, timed by events on the stream
  auto best = [&](auto launch) -> float {
    launch();
    float m = 1e30f;
    for (int r = 0; r < 3 && !rc; ++r) {
      float ms = 0.f;
      if (hipEventRecord(e0, st) != hipSuccess) { rc = TCF_EHIP; break; }
      launch();
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = TCF_EHIP;
        break;
      }
      m = std::min(m, ms);
    }
    return m;
  };
  if (!rc) {
    const float mr = best([&] { launch_read_probe((int64_t)(n32 * 2), a, (double*)o, st); });
    const float mc = best([&] { launch_copy_probe((int64_t)n32, a, b, st); });
    if (!rc) {
      *read_gbs = (double)n32 * 32 / (mr * 1e6);
      *copy_gbs = 2.0 * n32 * 32 / (mc * 1e6);
    }
  }
  if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) rc = TCF_EHIP;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(g_capture_mu);
  (void)hipFree(a);
  (void)hipFree(b);
  (void)hipFree(o);
  return rc;
}

int tcf_profile_get(const tcf_problem* h, int32_t g, double* total_ms, int64_t* launches,
                    double* alg_bytes) {
  if (!h || g < 0 || g >= TCF_KG_COUNT) return TCF_EINVAL;
  if (total_ms) *total_ms = h->prof_ms[g];
  if (launches) *launches = h->prof_n[g];
  if (alg_bytes) *alg_bytes = h->prof_bytes[g];
  return TCF_OK;
}

int tcf_profile_get_flops(const tcf_problem* h, int32_t g, double* alg_flops) {
  if (!h || g < 0 || g >= TCF_KG_COUNT || !alg_flops) return TCF_EINVAL;
  *alg_flops = h->prof_flops[g];
  return TCF_OK;
}

}  // extern "C"

// ============================================================================
// Setup
// ============================================================================
template <class T>
static int run_factor_phase(tcf_problem* h, const std::vector<FactorJob>& jobs, T* A,
                            hipStream_t st) {
  // Blocked right-looking Cholesky of columns [c_begin, c_end) of every job:
  // per panel of TCF_NB columns the diagonal block, the rows below it, and
  // the update of the rest of its super-panel (SP panels); after the last
  // panel of a super-panel one update of the whole trailing matrix with all
  // of the super-panel's columns.
  if (jobs.empty()) return TCF_OK;
  const int nj = (int)jobs.size(), SP = syrk_super_panel();
  int steps = 0;
  for (auto& j : jobs) steps = std::max(steps, (j.c_end - j.c_begin) / TCF_NB);
  std::vector<int> trsm_pre((size_t)steps * (nj + 1)), loc_pre((size_t)steps * (nj + 1)),
      wide_pre((size_t)steps * (nj + 1));
  std::vector<int> trsm_tot(steps), loc_tot(steps), wide_tot(steps);
  for (int k = 0; k < steps; ++k) {
    int* tp = &trsm_pre[(size_t)k * (nj + 1)];
    int* lp = &loc_pre[(size_t)k * (nj + 1)];
    int* wp = &wide_pre[(size_t)k * (nj + 1)];
    tp[0] = lp[0] = wp[0] = 0;
    for (int j = 0; j < nj; ++j) {
      const FactorJob& jb = jobs[j];
      const int col0 = jb.c_begin + TCF_NB * k;
      const int p0 = jb.c_begin + TCF_NB * SP * (k / SP);
      const int p_end = std::min(p0 + TCF_NB * SP, jb.c_end);
      int nt = 0, nl = 0, nw = 0;
      if (col0 < jb.c_end) {
        const int trail0 = col0 + TCF_NB;
        nt = (jb.n - trail0 + 63) / 64;
        if (p_end > trail0) nl = nt * ((p_end - trail0 + 63) / 64);
      }
      // the wide update once the job's super-panel is complete, i.e. after
      // its last panel (the one ending at p_end)
      if (col0 < jb.c_end && col0 + TCF_NB == p_end) {
        const int T_ = (jb.n - p_end + 63) / 64;
        nw = T_ * (T_ + 1) / 2;
      }
      tp[j + 1] = tp[j] + nt;
      lp[j + 1] = lp[j] + nl;
      wp[j + 1] = wp[j] + nw;
    }
    trsm_tot[k] = tp[nj];
    loc_tot[k] = lp[nj];
    wide_tot[k] = wp[nj];
  }
  FactorJob* dj;
  int *dtp, *dlp, *dwp;
  RCCHK(h->upload(&dj, jobs));
  RCCHK(h->upload(&dtp, trsm_pre));
  RCCHK(h->upload(&dlp, loc_pre));
  RCCHK(h->upload(&dwp, wide_pre));
  for (int k = 0; k < steps; ++k) {
    launch_potrf<T>(dj, nj, k, A, h->d_fail, st);
    launch_trsm_panel<T>(dj, dtp + (size_t)k * (nj + 1), nj, trsm_tot[k], k, A, st);
    launch_syrk<T>(dj, dlp + (size_t)k * (nj + 1), nj, loc_tot[k], k, 0, A, st);
    launch_syrk<T>(dj, dwp + (size_t)k * (nj + 1), nj, wide_tot[k], k, 1, A, st);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  h->release(dj);
  h->release(dtp);
  h->release(dlp);
  h->release(dwp);
  return TCF_OK;
}

template <class T>
static int run_trsm(tcf_problem* h, int fwd, const std::vector<TrsmJob>& jobs, const T* L, T* B,
                    hipStream_t st) {
  if (jobs.empty()) return TCF_OK;
  std::vector<int> cnt;
  for (auto& j : jobs) cnt.push_back((j.ncols + 63) / 64);
  std::vector<int> pre = prefix_of(cnt);
  TrsmJob* dj;
  int* dp;
  RCCHK(h->upload(&dj, jobs));
  RCCHK(h->upload(&dp, pre));
  {
    // on the matrix cores: the inverses of the 32 x 32 diagonal blocks
    // first, then the blocked solve
    std::vector<int> dcnt;
    for (auto& j : jobs) dcnt.push_back(j.n / TCF_NB);
    std::vector<int> dpre = prefix_of(dcnt);
    int* ddp;
    T* D;
    RCCHK(h->upload(&ddp, dpre));
    RCCHK(h->alloc(&D, (size_t)dpre.back() * TCF_NB * TCF_NB));
    launch_trsm_dinv(dj, ddp, (int)jobs.size(), dpre.back(), L, D, st);
    // right-looking steps over panels of P row blocks: per step the prefix
    // over jobs of the tiles it updates (row blocks after the panel forward,
    // before it backward)
    const int nj = (int)jobs.size(), P = trsm_rl_panel();
    int steps = 0;
    for (int c : dcnt) steps = std::max(steps, (c + P - 1) / P);
    std::vector<int> tab((size_t)steps * (nj + 1)), tot(steps);
    for (int st_i = 0; st_i < steps; ++st_i) {
      int acc = 0;
      for (int x = 0; x < nj; ++x) {
        tab[(size_t)st_i * (nj + 1) + x] = acc;
        const int nb = dcnt[x];
        const int rows = std::max(0, nb - P * (st_i + 1));  // same count both ways
        acc += rows * cnt[x];
      }
      tab[(size_t)st_i * (nj + 1) + nj] = acc;
      tot[st_i] = acc;
    }
    int* dtab;
    RCCHK(h->upload(&dtab, tab));
    for (int st_i = 0; st_i < steps; ++st_i) {
      launch_trsm_rl_diag(dj, dp, ddp, nj, pre.back(), st_i, fwd, L, D, B, st);
      launch_trsm_rl_update(dj, dtab + (size_t)st_i * (nj + 1), nj, tot[st_i], st_i, fwd, L, B, st);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    h->release(dtab);
    h->release(D);
    h->release(ddp);
  }
  h->release(dj);
  h->release(dp);
  return TCF_OK;
}

static constexpr int kDotCpb = 32;  // columns per block of k_dotcols

static int build_index_tables(tcf_problem* h) {
  const int np = h->np_tot;
  const int rows_per_stripe = 64 * (h->precision == TCF_FP64 ? 2 : 4);
  std::vector<int> rloc, loc2r, brow, prank, posp(h->n_lambda), posm(h->n_lambda), b2bp, p2r, b2r;
  std::vector<int> posp_r(h->n_lambda), posm_r(h->n_lambda);
  std::vector<int> posp_bp(h->n_lambda), posm_bp(h->n_lambda);
  std::vector<signed char> bsgn, isint;
  for (int s = 0; s < np; ++s) {
    const PatchPlan& pp = h->plans[s];
    const DevPatch& d = h->hp[s];
    rloc.insert(rloc.end(), pp.r_loc.begin(), pp.r_loc.end());
    loc2r.insert(loc2r.end(), pp.loc2r.begin(), pp.loc2r.end());
    for (int k = 0; k < pp.n_b; ++k) {
      brow.push_back(pp.b_row[k]);
      bsgn.push_back((signed char)pp.b_sgn[k]);
      b2bp.push_back(d.bp_off + k);
      b2r.push_back(d.r_off + pp.n_i + k);
      if (pp.b_sgn[k] > 0) {
        posp[pp.b_row[k]] = d.b_off + k;
        posp_r[pp.b_row[k]] = d.r_off + pp.n_i + k;
        posp_bp[pp.b_row[k]] = d.bp_off + k;
      } else {
        posm_bp[pp.b_row[k]] = d.bp_off + k;
        posm[pp.b_row[k]] = d.b_off + k;
        posm_r[pp.b_row[k]] = d.r_off + pp.n_i + k;
      }
    }
    // coarse unknowns are numbered in the order of the coarse factor
    for (int j = 0; j < pp.n_p; ++j) {
      prank.push_back(h->cplan.nd[pp.p_rank[j]]);
      p2r.push_back(d.r_off + pp.n_i + pp.n_b + j);
    }
    for (int j = 0; j < pp.n_r(); ++j) isint.push_back(j < pp.n_i ? 1 : 0);
  }
  // coarse owners (deterministic order: by patch id)
  std::vector<std::vector<std::pair<int, int>>> own(h->n_primal);
  for (int s = 0; s < np; ++s) {
    const PatchPlan& pp = h->plans[s];
    const DevPatch& d = h->hp[s];
    for (int j = 0; j < pp.n_p; ++j)
      own[h->cplan.nd[pp.p_rank[j]]].push_back({d.bp_off + pp.n_b + j, d.r_off + pp.n_i + pp.n_b + j});
  }
  std::vector<int> cptr(1, 0), cbp, cr;
  for (int k = 0; k < h->n_primal; ++k) {
    for (auto& x : own[k]) { cbp.push_back(x.first); cr.push_back(x.second); }
    cptr.push_back((int)cbp.size());
  }
  RCCHK(h->upload(&h->d_rloc, rloc));
  RCCHK(h->upload(&h->d_loc2r, loc2r));
  RCCHK(h->upload(&h->d_brow, brow));
  RCCHK(h->upload(&h->d_bsgn, bsgn));
  RCCHK(h->upload(&h->d_isint, isint));
  RCCHK(h->upload(&h->d_prank, prank));
  RCCHK(h->upload(&h->d_posp, posp));
  h->h_posp = posp;
  h->h_posm = posm;
  {
    std::vector<double> sd(bsgn.begin(), bsgn.end());
    RCCHK(h->upload(&h->d_bsgn_d, sd));
    h->d_pre_w = h->d_bsgn_d;
  }
  RCCHK(h->upload(&h->d_posm, posm));
  RCCHK(h->upload(&h->d_posp_r, posp_r));
  RCCHK(h->upload(&h->d_posp_bp, posp_bp));
  RCCHK(h->upload(&h->d_posm_bp, posm_bp));
  RCCHK(h->upload(&h->d_posm_r, posm_r));
  RCCHK(h->upload(&h->d_cptr, cptr));
  RCCHK(h->upload(&h->d_cidx_bp, cbp));
  RCCHK(h->upload(&h->d_cidx_r, cr));
  RCCHK(h->upload(&h->d_b2bp, b2bp));
  RCCHK(h->upload(&h->d_p2r, p2r));
  RCCHK(h->upload(&h->d_b2r, b2r));

  // per-apply job tables
  std::vector<DotJob> app_g, app_v, pre;
  std::vector<int> c_app, c_pre;
  std::vector<AxpyJob> phi, ai;
  std::vector<int> c_phi, c_ai, boff_bp, boff_b, boff_ai;
  for (int s = 0; s < np; ++s) {
    const DevPatch& d = h->hp[s];
    if (d.n_b > 0) {
      app_g.push_back(DotJob{d.G_off, d.nb_pad, d.n_b, d.n_b + d.n_p, d.b_off, d.bp_off});
      app_v.push_back(DotJob{d.G_off, d.nb_pad, d.n_b, d.n_b + d.n_p, d.r_off + d.n_i, d.bp_off});
      c_app.push_back((d.n_b + d.n_p + kDotCpb - 1) / kDotCpb);
      pre.push_back(DotJob{d.S_off, d.nb_pad, d.n_b, d.n_b, d.b_off, d.b_off});
      c_pre.push_back((d.n_b + kDotCpb - 1) / kDotCpb);
      if (d.n_p > 0) {
        phi.push_back(AxpyJob{d.G_off, d.nb_pad, d.n_b, d.n_p, d.n_b, d.p_off, d.b_off});
        c_phi.push_back((d.n_b + rows_per_stripe - 1) / rows_per_stripe);
        boff_bp.push_back(d.bp_off);
        boff_b.push_back(d.b_off);
      }
    }
    if (d.n_i > 0) {
      ai.push_back(AxpyJob{d.Q_off, d.ni_pad, d.n_i, d.n_r, 0, d.r_off, d.r_off});
      c_ai.push_back((d.n_i + rows_per_stripe - 1) / rows_per_stripe);
      boff_ai.push_back(0);
    }
  }
  h->nj_app = (int)app_g.size();
  // a patch with primal but no dual unknowns has no column-dot job, so its
  // entries of the b+p vectors (c = Phi_b^T x = 0) must be cleared first
  h->bp_gaps = false;
  for (int s = 0; s < np; ++s)
    if (h->hp[s].n_b == 0 && h->hp[s].n_p > 0) h->bp_gaps = true;
  h->nj_pre = (int)pre.size();
  h->nj_phi = (int)phi.size();
  h->nj_ai = (int)ai.size();
  auto p_app = prefix_of(c_app), p_pre = prefix_of(c_pre), p_phi = prefix_of(c_phi),
       p_ai = prefix_of(c_ai);
  h->nt_app = p_app.back();
  h->nt_pre = p_pre.back();
  h->nt_phi = p_phi.back();
  h->nt_ai = p_ai.back();
  RCCHK(h->upload(&h->dj_app_g, app_g));
  RCCHK(h->upload(&h->dj_app_v, app_v));
  RCCHK(h->upload(&h->dp_app, p_app));
  RCCHK(h->upload(&h->dj_pre, pre));
  RCCHK(h->upload(&h->dp_pre, p_pre));
  RCCHK(h->upload(&h->aj_phi, phi));
  RCCHK(h->upload(&h->ap_phi, p_phi));
  RCCHK(h->upload(&h->a_boff_bp, boff_bp));
  RCCHK(h->upload(&h->a_boff_b, boff_b));
  RCCHK(h->upload(&h->aj_ai, ai));
  RCCHK(h->upload(&h->ap_ai, p_ai));
  RCCHK(h->upload(&h->a_boff_ai, boff_ai));
  // a_b recovery: same matrices as Phi, output into the state at r_off + n_i
  std::vector<AxpyJob> ab;
  std::vector<int> boff_ab;
  for (int s = 0; s < np; ++s) {
    const DevPatch& d = h->hp[s];
    if (d.n_b > 0 && d.n_p > 0) {
      ab.push_back(AxpyJob{d.G_off, d.nb_pad, d.n_b, d.n_p, d.n_b, d.p_off, d.r_off + d.n_i});
      boff_ab.push_back(d.r_off + d.n_i);
    }
  }
  RCCHK(h->upload(&h->aj_ab, ab));
  RCCHK(h->upload(&h->a_boff_ab, boff_ab));
  // conductor patch lists
  std::vector<int> ccnt, rcnt;
  for (int s : h->cond_list) {
    ccnt.push_back((h->hp[s].n_r + 15) / 16);
    rcnt.push_back(h->hp[s].n_r);
  }
  auto cpre = prefix_of(ccnt), rpre = prefix_of(rcnt);
  h->nt_cond_c = cpre.back();
  h->nt_cond_r = rpre.back();
  RCCHK(h->upload(&h->d_cond, h->cond_list));
  RCCHK(h->upload(&h->d_cond_cprefix, cpre));
  RCCHK(h->upload(&h->d_cond_rprefix, rpre));
  {
    std::vector<int> cw, aw, ai64;
    for (int s : h->cond_list) cw.push_back((h->hp[s].n_r + 63) / 64);
    for (int s = 0; s < np; ++s) {
      aw.push_back((h->hp[s].n_r + 63) / 64);
      ai64.push_back((h->hp[s].n_i + 63) / 64);
    }
    auto pcw = prefix_of(cw), paw = prefix_of(aw), pai = prefix_of(ai64);
    h->nt_cond_w = pcw.back();
    h->nt_all_w = paw.back();
    h->nt_all_i = pai.back();
    RCCHK(h->upload(&h->d_cond_wprefix, pcw));
    RCCHK(h->upload(&h->d_all_wprefix, paw));
    RCCHK(h->upload(&h->d_all_iprefix, pai));
  }
  return TCF_OK;
}

// Coarse factor from its assembled fronts: per height of the elimination
// tree (leaves first) a batched partial Cholesky of the fronts' own columns,
// then each front's update matrix is added into its parent's front; last
// the top block is factored completely.  Then the explicit operators:
// L_JJ^-1 and -L_JJ^-T L_SJ^T per node, and the dense inverse of the top
// block's Schur complement.
static int coarse_factor(tcf_problem* h, double* F, const CoarseNodeDev* dnodes, const int* d_cpos,
                         hipStream_t st) {
  const int nn = (int)h->cnodes.size();
  const int root = h->c_root;
  for (int lv = 0; lv <= h->c_levels; ++lv) {
    std::vector<FactorJob> jobs;
    std::vector<int> done;
    for (int i = 0; i < nn; ++i) {
      const bool here = lv < h->c_levels ? (i != root && h->cplan.nodes[i].height == lv) : i == root;
      if (!here) continue;
      const CoarseNodeDev& c = h->cnodes[i];
      jobs.push_back(FactorJob{c.f_off, c.nf, c.nf, 0, c.nj_pad, -1});
      done.push_back(i);
    }
    RCCHK(run_factor_phase<double>(h, jobs, F, st));
    for (int i : done) {
      const CoarseNodeDev& c = h->cnodes[i];
      if (c.parent >= 0) launch_extend_add(dnodes, i, c.ns, d_cpos, F, st);
    }
    HIPCHK(hipGetLastError());
  }
  // L_JJ^-1 | -L_JJ^-T L_SJ^T of every node below the top block
  if (nn > 1) {
    double* L;
    RCCHK(h->alloc(&L, (size_t)h->c_lop_elems));
    h->d_cL = L;
    std::vector<int> ids, cnt;
    std::vector<TrsmJob> tf, tb;
    for (int i = 0; i < nn; ++i) {
      if (i == root) continue;
      const CoarseNodeDev& c = h->cnodes[i];
      ids.push_back(i);
      cnt.push_back(c.nj + c.ns);
      tf.push_back(TrsmJob{c.f_off, c.nf, 0, c.nj_pad, c.l_off, c.nj_pad, c.nj, c.nj, 0});
      if (c.ns > 0)
        tb.push_back(TrsmJob{c.f_off, c.nf, 0, c.nj_pad, c.l_off + (int64_t)c.nj * c.nj_pad,
                             c.nj_pad, c.ns, 0, 0});
    }
    auto pre = prefix_of(cnt);
    int *dids, *dpre;
    RCCHK(h->upload(&dids, ids));
    RCCHK(h->upload(&dpre, pre));
    launch_front_rhs(dnodes, dids, dpre, (int)ids.size(), pre.back(), F, L, st);
    HIPCHK(hipGetLastError());
    RCCHK(run_trsm<double>(h, 1, tf, F, L, st));
    RCCHK(run_trsm<double>(h, 0, tb, F, L, st));
    h->release(dids);
    h->release(dpre);
  }
  // dense inverse of the top block: L X = I, then L^T Y = X
  {
    const CoarseNodeDev& c = h->cnodes[root];
    const int ld = c.nj_pad;
    double* Sinv;
    RCCHK(h->alloc(&Sinv, (size_t)ld * ld));
    HIPCHK(hipMemsetAsync(Sinv, 0, sizeof(double) * ld * ld, st));
    launch_identity_pad(Sinv, ld, 0, c.nj, st);
    std::vector<TrsmJob> t1{TrsmJob{c.f_off, c.nf, 0, ld, 0, ld, c.nj, c.nj, 0}};
    std::vector<TrsmJob> t0{TrsmJob{c.f_off, c.nf, 0, ld, 0, ld, c.nj, 0, 0}};
    RCCHK(run_trsm<double>(h, 1, t1, F, Sinv, st));
    RCCHK(run_trsm<double>(h, 0, t0, F, Sinv, st));
    h->d_SPinv = Sinv;
  }
  return TCF_OK;
}

// Setup.  T: precision of the factorisation; TO: precision in which the
// explicit operators (G, S, Q^T) are kept.  The patches are factored in
// groups (chunk_begin); within a group the kernels see a copy of the patch
// table whose A, G, S and Q^T offsets are relative to the group, so that
// only one group's dense blocks (and, when TO is narrower than T, its
// operators in T) exist at a time; the group's operators are then written
// to their final storage in TO.
template <class T, class TO>
static int setup_impl(tcf_problem* h, hipStream_t st) {
  const int np = h->np_tot;
  const int nrhs = h->n_rhs;
  const int64_t ldv = h->n_rtot;
  constexpr bool kSame = std::is_same<T, TO>::value;
  RCCHK(h->upload(&h->dP, h->hp));
  RCCHK(build_index_tables(h));
  std::vector<double> gx(h->gx, h->gx + 136), gw(h->gw, h->gw + 136);
  RCCHK(h->upload(&h->d_gx, gx));
  RCCHK(h->upload(&h->d_gw, gw));
  RCCHK(h->alloc(&h->d_tabs, h->tab_elems));
  RCCHK(h->alloc(&h->d_ptab, h->ptab_elems));
  RCCHK(h->alloc(&h->d_fail, 1));
  HIPCHK(hipMemsetAsync(h->d_fail, 0, sizeof(int), st));
  launch_tables(h->dP, np, h->d_gx, h->d_gw, h->d_tabs, h->d_ptab, st);

  // source loads: the curl form (phi) and/or the volume form (jvol) on
  // source patches, and the initial load int sigma A(x,0) . w (ainit) on
  // conductor patches
  double* jr;
  RCCHK(h->alloc(&jr, (size_t)ldv * nrhs));
  HIPCHK(hipMemsetAsync(jr, 0, sizeof(double) * ldv * nrhs, st));
  const bool want_m0 = h->ainit && !h->cond_list.empty();
  if (want_m0) {
    RCCHK(h->alloc(&h->d_m0, (size_t)ldv * nrhs));
    HIPCHK(hipMemsetAsync(h->d_m0, 0, sizeof(double) * ldv * nrhs, st));
  }
  {
    // Three passes (curl-form source, volume source, initial value), each
    // over its patches in chunks: the callbacks fill a host buffer with the
    // values at every patch's load points until the chunk budget is
    // reached, one upload, one launch over every kept edge of the chunk.
    const size_t budget = (size_t)16 << 20;  // doubles per chunk
    double* stage = nullptr;
    size_t stage_cap = 0;
    std::vector<double> hbuf;
    auto points = [&](const DevPatch& d, std::vector<double>* ax) {
      for (int a = 0; a < 3; ++a) {
        const int nq = d.deg[a] + 3;
        const int o = nq * (nq - 1) / 2;
        const double hh = (d.hi[a] - d.lo[a]) / d.nel[a];
        ax[a].clear();
        for (int t = 0; t < d.nel[a]; ++t)
          for (int q = 0; q < nq; ++q) ax[a].push_back((hh * t + d.lo[a]) + 0.5 * hh * (h->gx[o + q] + 1.0));
      }
    };
    for (int kind = 0; kind < 3; ++kind) {
      const int ncomp = kind == 0 ? 1 : 3;
      double* out = kind == 2 ? h->d_m0 : jr;
      std::vector<int> pl;
      for (int s = 0; s < np; ++s) {
        const DevPatch& d = h->hp[s];
        if (d.n_r == 0) continue;
        if (kind == 0 && d.src && h->phi) pl.push_back(s);
        if (kind == 1 && d.src && h->jvol) pl.push_back(s);
        if (kind == 2 && want_m0 && h->sigma[s] > 0) pl.push_back(s);
      }
      size_t next = 0;
      while (next < pl.size()) {
        std::vector<LoadJob> jobs;
        std::vector<int> cnt;
        size_t used = 0;
        while (next < pl.size()) {
          const DevPatch& d = h->hp[pl[next]];
          const size_t npts = (size_t)d.nq_load[0] * d.nq_load[1] * d.nq_load[2];
          const size_t need = npts * ncomp * nrhs;
          if (!jobs.empty() && used + need > budget) break;
          jobs.push_back(LoadJob{(int64_t)used, pl[next], 0, kind == 2 ? h->sigma[pl[next]] : 1.0});
          cnt.push_back((d.n_r + 127) / 128);
          used += need;
          ++next;
        }
        if (hbuf.size() < used) hbuf.resize(used);
        std::vector<double> ax[3];
        for (const LoadJob& jb : jobs) {
          const DevPatch& d = h->hp[jb.s];
          points(d, ax);
          const int nx = (int)ax[0].size(), ny = (int)ax[1].size(), nz = (int)ax[2].size();
          const size_t npts = (size_t)nx * ny * nz;
          for (int k = 0; k < nrhs; ++k) {
            double* o = hbuf.data() + jb.f_off + (size_t)k * ncomp * npts;
            if (kind == 0)
              h->phi(ax[0].data(), nx, ax[1].data(), ny, ax[2].data(), nz, k, o, h->phi_ctx);
            else
              (kind == 1 ? h->jvol : h->ainit)(jb.s, ax[0].data(), nx, ax[1].data(), ny,
                                                ax[2].data(), nz, k, o, h->vec_ctx);
          }
        }
        HIPCHK(hipStreamSynchronize(st));  // the previous chunk's launch has read the stage
        if (stage_cap < used) {
          if (stage) h->release(stage);
          RCCHK(h->alloc(&stage, used));
          stage_cap = used;
        }
        // the copy leaves the pageable host buffer before the next chunk refills it
        HIPCHK(hipMemcpyAsync(stage, hbuf.data(), sizeof(double) * used, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        auto pre = prefix_of(cnt);
        LoadJob* dj;
        int* dp;
        RCCHK(h->upload(&dj, jobs));
        RCCHK(h->upload(&dp, pre));
        launch_load_batch(h->dP, dj, dp, (int)jobs.size(), pre.back(), nrhs, h->d_rloc, h->d_ptab,
                          stage, kind == 0 ? 0 : 1, out, ldv, st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        h->release(dj);
        h->release(dp);
      }
    }
    if (stage) h->release(stage);
  }

  h->d_jr = jr;
  // final operator storage, the condensed source, and per-patch diagnostics
  TO *G, *S, *Q;
  RCCHK(h->alloc(&S, h->S_elems));
  RCCHK(h->alloc(&G, h->G_elems));
  // 64 elements of slack: the matrix-core Q^T products read up to 63 rows
  // past a patch's last column (and discard them)
  RCCHK(h->alloc(&Q, h->Q_elems + 64));
  h->d_G = G;
  h->d_S = S;
  h->d_Q = Q;
  RCCHK(h->alloc(&h->d_yggs, (size_t)ldv * nrhs));
  HIPCHK(hipMemsetAsync(h->d_yggs, 0, sizeof(double) * ldv * nrhs, st));
  const bool scaled = h->opt.precond_scaling == 1 && h->n_lambda > 0;
  double* kd = nullptr;
  if (scaled) RCCHK(h->alloc(&kd, (size_t)std::max<int64_t>(h->n_btot, 1)));
  double* dr;
  RCCHK(h->alloc(&dr, (size_t)2 * np));
  // coarse fronts, assembled patch by patch while the groups are factored
  double* F = nullptr;
  CoarseNodeDev* dnodes = nullptr;
  int *d_nodeof = nullptr, *d_slist = nullptr, *d_cpos = nullptr;
  if (h->c_root >= 0) {
    const int nn = (int)h->cnodes.size();
    std::vector<int> nodeof(h->n_primal), slist, cpos;
    for (int i = 0; i < nn; ++i) {
      const CoarseNode& c = h->cplan.nodes[i];
      for (int g = c.j0; g < c.j0 + c.nj; ++g) nodeof[g] = i;
      slist.insert(slist.end(), c.S.begin(), c.S.end());
    }
    // parent front position of every structure entry
    for (int i = 0; i < nn; ++i) {
      const CoarseNode& c = h->cplan.nodes[i];
      for (int g : c.S) {
        if (c.parent < 0) { cpos.push_back(0); continue; }
        const CoarseNode& p = h->cplan.nodes[c.parent];
        const CoarseNodeDev& pd = h->cnodes[c.parent];
        if (g >= p.j0 && g < p.j0 + p.nj) {
          cpos.push_back(g - p.j0);
        } else {
          const auto it = std::lower_bound(p.S.begin(), p.S.end(), g);
          if (it == p.S.end() || *it != g) {
            h->err = "coarse plan: a structure entry is missing from its parent";
            return TCF_EINVAL;
          }
          cpos.push_back(pd.nj_pad + (int)(it - p.S.begin()));
        }
      }
    }
    slist.push_back(0);
    cpos.push_back(0);
    RCCHK(h->upload(&dnodes, h->cnodes));
    RCCHK(h->upload(&d_nodeof, nodeof));
    RCCHK(h->upload(&d_slist, slist));
    RCCHK(h->upload(&d_cpos, cpos));
    RCCHK(h->alloc(&F, (size_t)h->c_front_elems));
    HIPCHK(hipMemsetAsync(F, 0, sizeof(double) * h->c_front_elems, st));
    launch_front_pad(dnodes, nn, F, st);
  }
  T* A = nullptr;
  RCCHK(h->alloc(&A, h->A_chunk_max));
  T *Gt = nullptr, *St = nullptr, *Qt = nullptr;
  if (!kSame) {
    RCCHK(h->alloc(&Gt, (size_t)std::max<int64_t>(h->G_chunk_max, 1)));
    RCCHK(h->alloc(&St, (size_t)std::max<int64_t>(h->S_chunk_max, 1)));
    RCCHK(h->alloc(&Qt, (size_t)std::max<int64_t>(h->Q_chunk_max, 1) + 64));
  }
  DevPatch* dPc;
  RCCHK(h->alloc(&dPc, (size_t)np));
  const int nchunks = (int)h->chunk_begin.size() - 1;
  for (int ch = 0; ch < nchunks; ++ch) {
    const int s0 = h->chunk_begin[ch], s1 = h->chunk_begin[ch + 1], nc = s1 - s0;
    const int64_t gb = h->hp[s0].G_off, sb = h->hp[s0].S_off, qb = h->hp[s0].Q_off;
    std::vector<DevPatch> tab(h->hp.begin() + s0, h->hp.begin() + s1);
    for (DevPatch& d : tab) {
      d.G_off -= gb;
      d.S_off -= sb;
      d.Q_off -= qb;
    }
    HIPCHK(hipMemcpyAsync(dPc, tab.data(), sizeof(DevPatch) * nc, hipMemcpyHostToDevice, st));
    T* Gw = kSame ? (T*)(G + gb) : Gt;
    T* Sw = kSame ? (T*)(S + sb) : St;
    T* Qw = kSame ? (T*)(Q + qb) : Qt;
    std::vector<int> colcnt(nc), sbc(nc), cg(nc), cq(nc), cc(nc), plist(nc);
    for (int t = 0; t < nc; ++t) {
      const DevPatch& d = tab[t];
      colcnt[t] = d.nr_pad;
      sbc[t] = d.n_b;
      cg[t] = d.n_b > 0 ? d.n_b + d.n_p : 0;
      cq[t] = d.n_i > 0 ? d.n_r : 0;
      // condensation blocks: 16 columns (vector form) or 64 (matrix cores)
      cc[t] = nrhs > 2 ? (d.n_r + 63) / 64 : (d.n_r + 15) / 16;
      plist[t] = t;
    }
    auto colpre = prefix_of(colcnt), sbpre = prefix_of(sbc), pg = prefix_of(cg),
         pq = prefix_of(cq), cpre = prefix_of(cc);
    int *d_colpre, *d_sbpre, *dpg, *dpq, *dcp, *dpl;
    RCCHK(h->upload(&d_colpre, colpre));
    RCCHK(h->upload(&d_sbpre, sbpre));
    RCCHK(h->upload(&dpg, pg));
    RCCHK(h->upload(&dpq, pq));
    RCCHK(h->upload(&dcp, cpre));
    RCCHK(h->upload(&dpl, plist));
    launch_assemble<T>(dPc, d_colpre, nc, colpre.back(), h->d_rloc, h->d_tabs, h->dt, A, st);
    HIPCHK(hipGetLastError());
    // stiffness scaling takes the dual diagonal before factorisation
    if (kd) launch_bdiag<T>(dPc, nc, A, kd, st);
    // factor the interior columns, keep S_bb, factor the dual columns
    std::vector<FactorJob> ja, jbv;
    for (int t = 0; t < nc; ++t) {
      const DevPatch& d = tab[t];
      if (d.ni_pad > 0) ja.push_back(FactorJob{d.A_off, d.nr_pad, d.nr_pad, 0, d.ni_pad, s0 + t});
      if (d.nb_pad > 0)
        jbv.push_back(FactorJob{d.A_off, d.nr_pad, d.nr_pad, d.ni_pad, d.ni_pad + d.nb_pad, s0 + t});
    }
    RCCHK(run_factor_phase<T>(h, ja, A, st));
    launch_copy_sbb<T>(dPc, d_sbpre, nc, sbpre.back(), A, Sw, st);
    RCCHK(run_factor_phase<T>(h, jbv, A, st));
    // per-patch pivot range of the factored [i|b] block
    launch_diag_range<T>(dPc, nc, A, dr + 2 * s0, st);
    // this group's primal Schur complements into the coarse fronts, patch
    // by patch in id order
    if (F)
      for (int t = 0; t < nc; ++t)
        launch_front_add<T>(dPc, t, tab[t].n_p, h->d_prank, A, dnodes, d_nodeof, d_slist, F, st);
    // G = [S_bb^-1 | Phi_b] and Q^T
    launch_fill_G<T>(dPc, dpg, nc, pg.back(), A, Gw, st);
    launch_fill_Q<T>(dPc, dpq, nc, pq.back(), A, Qw, st);
    HIPCHK(hipGetLastError());
    std::vector<TrsmJob> gf, gbk, qbk;
    for (int t = 0; t < nc; ++t) {
      const DevPatch& d = tab[t];
      if (d.n_b > 0) {
        gf.push_back(TrsmJob{d.A_off, d.nr_pad, d.ni_pad, d.nb_pad, d.G_off, d.nb_pad, d.n_b,
                             d.n_b, 0});
        gbk.push_back(TrsmJob{d.A_off, d.nr_pad, d.ni_pad, d.nb_pad, d.G_off, d.nb_pad,
                              d.n_b + d.n_p, 0, 0});
      }
      if (d.n_i > 0)
        qbk.push_back(TrsmJob{d.A_off, d.nr_pad, 0, d.ni_pad, d.Q_off, d.ni_pad, d.n_r, d.n_i, 0});
    }
    RCCHK(run_trsm<T>(h, 1, gf, A, Gw, st));
    RCCHK(run_trsm<T>(h, 0, gbk, A, Gw, st));
    RCCHK(run_trsm<T>(h, 0, qbk, A, Qw, st));
    // the source condenses once (time separable), with the factorisation's
    // own Q^T: yggs = cond(jhat)
    if (nrhs > 2)
      for (int r0 = 0; r0 < nrhs; r0 += 32)
        launch_condense_w<T>(dPc, dpl, dcp, nc, cpre.back(), std::min(32, nrhs - r0), Qw,
                             h->d_jr + (int64_t)r0 * ldv, h->d_yggs + (int64_t)r0 * ldv, ldv, st);
    else
      launch_condense<T>(dPc, dpl, dcp, nc, cpre.back(), nrhs, h->max_ni, Qw, h->d_jr, h->d_yggs,
                         ldv, st);
    HIPCHK(hipGetLastError());
    if (!kSame) {
      const DevPatch& l = h->hp[s1 - 1];
      launch_to_float((l.G_off + (int64_t)l.nb_pad * (l.n_b + l.n_p)) - gb, (const double*)Gt,
                      (float*)(G + gb), st);
      launch_to_float((l.S_off + (int64_t)l.nb_pad * l.n_b) - sb, (const double*)St,
                      (float*)(S + sb), st);
      launch_to_float((l.Q_off + (int64_t)l.ni_pad * l.n_r) - qb, (const double*)Qt,
                      (float*)(Q + qb), st);
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(st));
    for (int* b : {d_colpre, d_sbpre, dpg, dpq, dcp, dpl}) h->release(b);
  }
  h->release(A);
  h->release(dPc);
  if (Gt) h->release(Gt);
  if (St) h->release(St);
  if (Qt) h->release(Qt);
  {
    int fail = 0;
    HIPCHK(hipMemcpyAsync(&fail, h->d_fail, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (fail) {
      h->fail_patch = fail - 2;
      h->err = "non-positive pivot in patch " + std::to_string(fail - 2);
      return TCF_ENOTSPD;
    }
  }
  if (kd) {
    // stiffness scaling: the copy of a dual unknown in patch s is weighted
    // by the other copy's share k_other / (k_s + k_other) of the two local
    // diagonal entries (taken before factorisation)
    std::vector<double> k(h->n_btot);
    HIPCHK(hipMemcpyAsync(k.data(), kd, sizeof(double) * h->n_btot, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    h->release(kd);
    std::vector<double> bw(h->n_btot, 0.0), wp(h->n_lambda), wm(h->n_lambda);
    for (int m = 0; m < h->n_lambda; ++m) {
      const int ep = h->h_posp[m], em = h->h_posm[m];
      const double kp = k[ep], km = k[em];
      if (!(kp > 0 && km > 0)) {
        h->err = "non-positive diagonal entry at a dual unknown";
        return TCF_ENOTSPD;
      }
      wp[m] = km / (kp + km);
      wm[m] = kp / (kp + km);
      bw[ep] = wp[m];    // sign +1
      bw[em] = -wm[m];   // sign -1
    }
    RCCHK(h->upload(&h->d_pre_w, bw));
    RCCHK(h->upload(&h->d_zwp, wp));
    RCCHK(h->upload(&h->d_zwm, wm));
  }
  {
    std::vector<double> r(2 * (size_t)np);
    HIPCHK(hipMemcpyAsync(r.data(), dr, sizeof(double) * 2 * np, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    h->release(dr);
    h->cond_est.assign(np, 1.0);
    for (int s = 0; s < np; ++s)
      if (h->hp[s].n_i + h->hp[s].n_b > 0 && r[2 * s] > 0)
        h->cond_est[s] = (r[2 * s + 1] / r[2 * s]) * (r[2 * s + 1] / r[2 * s]);
  }
  // the coarse factor and its explicit operators (FP64)
  if (F) {
    {
      Range rg("tcf setup: coarse factor");
      RCCHK(coarse_factor(h, F, dnodes, d_cpos, st));
    }
    int fail = 0;
    HIPCHK(hipMemcpyAsync(&fail, h->d_fail, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    h->release(F);
    h->release(dnodes);
    h->release(d_nodeof);
    h->release(d_slist);
    h->release(d_cpos);
    if (fail) {
      h->fail_patch = -1;
      h->err = "non-positive pivot in the coarse matrix";
      return TCF_ENOTSPD;
    }
  }

  // state and work vectors
  RCCHK(h->alloc(&h->d_a, (size_t)ldv * nrhs));
  RCCHK(h->alloc(&h->d_fM, (size_t)ldv * nrhs));
  RCCHK(h->alloc(&h->d_ygg, (size_t)ldv * nrhs));
  RCCHK(h->alloc(&h->d_zr, (size_t)ldv * h->rb));
  HIPCHK(hipMemsetAsync(h->d_a, 0, sizeof(double) * ldv * nrhs, st));
  HIPCHK(hipMemsetAsync(h->d_fM, 0, sizeof(double) * ldv * nrhs, st));
  const int rb = h->rb;
  RCCHK(h->alloc(&h->d_uc, (size_t)h->n_bptot * rb));
  RCCHK(h->alloc(&h->d_vc, (size_t)h->n_bptot * rb));
  RCCHK(h->alloc(&h->d_wb, h->n_btot));
  RCCHK(h->alloc(&h->d_tb, h->n_btot));
  const int nP = std::max(h->n_primal, 1);
  RCCHK(h->alloc(&h->d_h, (size_t)nP * rb));
  RCCHK(h->alloc(&h->d_q0, nP));
  const int nl = std::max(h->n_lambda, 1);
  RCCHK(h->alloc(&h->d_d, (size_t)nl * rb));
  RCCHK(h->alloc(&h->d_lam, (size_t)nl * rb));
  RCCHK(h->alloc(&h->d_r, (size_t)nl * rb));
  RCCHK(h->alloc(&h->d_z, (size_t)nl * rb));
  RCCHK(h->alloc(&h->d_p, (size_t)nl * rb));
  RCCHK(h->alloc(&h->d_Fp, (size_t)nl * rb));
  h->npart = (nl + 255) / 256;
  RCCHK(h->alloc(&h->d_part, (size_t)h->npart * 4 * rb));
  RCCHK(h->alloc(&h->d_st, (size_t)rb + 1));  // per column, plus the all-done flag
  if ((h->opt.pcg_warm == 1 || h->opt.pcg_warm == 2)) {
    RCCHK(h->alloc(&h->d_lamh, (size_t)nl * 2 * h->n_rhs));
    h->lamh_n.assign(h->n_rhs, 0);
  }
  if (h->opt.pcg_warm == 3) {
    const size_t kb = (size_t)tcf_problem::kProjMax * nl * h->n_rhs;
    RCCHK(h->alloc(&h->d_ph, kb));
    RCCHK(h->alloc(&h->d_pfh, kb));
    RCCHK(h->alloc(&h->d_px, kb));
    RCCHK(h->alloc(&h->d_pfx, kb));
    RCCHK(h->alloc(&h->d_pv, (size_t)nl));
    RCCHK(h->alloc(&h->d_pfv, (size_t)nl));
    RCCHK(h->alloc(&h->d_pc, (size_t)tcf_problem::kProjMax + 4));
    h->proj_n.assign(h->n_rhs, 0);
    h->proj_head.assign(h->n_rhs, 0);
  }
  RCCHK(h->alloc(&h->d_field, (size_t)h->g.n_edges()));
  {
    std::lock_guard<std::mutex> lk(g_capture_mu);
    HIPCHK(hipHostMalloc((void**)&h->h_st, sizeof(PcgScalars) * (rb + 1), hipHostMallocDefault));
  }
  HIPCHK(hipMemsetAsync(h->d_lam, 0, sizeof(double) * nl, st));

  // every patch, for the condensation of a general right-hand side
  std::vector<int> all(np), acnt(np);
  for (int s = 0; s < np; ++s) { all[s] = s; acnt[s] = (h->hp[s].n_r + 15) / 16; }
  auto apre = prefix_of(acnt);
  int *d_all, *d_apre;
  RCCHK(h->upload(&d_all, all));
  RCCHK(h->upload(&d_apre, apre));
  h->d_all = d_all;
  h->d_all_cprefix = d_apre;
  h->nt_all_c = apre.back();
  {
    std::vector<int> rc(np);
    for (int s = 0; s < np; ++s) rc[s] = h->hp[s].n_r;
    auto rp = prefix_of(rc);
    h->nt_all_r = rp.back();
    RCCHK(h->upload(&h->d_all_rprefix, rp));
  }
  // refinement work vectors and the kept-unknown -> local-copies map
  RCCHK(h->alloc(&h->d_floc, (size_t)ldv * rb));
  RCCHK(h->alloc(&h->d_res, (size_t)ldv * rb));
  HIPCHK(hipMemsetAsync(h->d_res, 0, sizeof(double) * ldv * rb, st));
  RCCHK(h->alloc(&h->d_delta, (size_t)ldv * rb));
  {
    std::vector<std::vector<int>> copies;
    std::vector<int64_t> kept_ids;
    std::vector<int> where(h->g.n_edges(), -1);
    for (int s = 0; s < np; ++s) {
      const PatchPlan& pp = h->plans[s];
      for (int j = 0; j < pp.n_r(); ++j) {
        const int64_t e = pp.r_gid[j];
        if (where[e] < 0) { where[e] = (int)copies.size(); copies.emplace_back(); }
        copies[where[e]].push_back(h->hp[s].r_off + j);
      }
    }
    std::vector<int> kp(1, 0), ki;
    for (auto& c : copies) { ki.insert(ki.end(), c.begin(), c.end()); kp.push_back((int)ki.size()); }
    h->n_kept_i = (int)copies.size();
    // the field is read out from each edge's first copy: the copies of an
    // interface unknown agree only to the PCG tolerance, and writing all of
    // them would leave whichever copy's store landed last
    {
      std::vector<int64_t> g1((size_t)std::max<int64_t>(ldv, 1), -1);
      for (int s = 0; s < np; ++s) {
        const PatchPlan& pp = h->plans[s];
        for (int j = 0; j < pp.n_r(); ++j) {
          const int64_t e = pp.r_gid[j];
          if (copies[where[e]][0] == h->hp[s].r_off + j) g1[h->hp[s].r_off + j] = e;
        }
      }
      RCCHK(h->upload(&h->d_rgid1, g1));
    }
    RCCHK(h->upload(&h->d_kptr, kp));
    RCCHK(h->upload(&h->d_kidx, ki));
    RCCHK(h->alloc(&h->d_nrm_part, (size_t)(h->n_kept_i + 255) / 256 + 1));
    RCCHK(h->alloc(&h->d_nrm, 4));
    {
      std::lock_guard<std::mutex> lk(g_capture_mu);
      HIPCHK(hipHostMalloc((void**)&h->h_nrm, 4 * sizeof(double), hipHostMallocDefault));
    }
  }
  return TCF_OK;
}

// Tile copies of the per-iteration operators: lower 64x64 tiles of S_bb^-1
// (with the Phi_b tiles), of S_bb and of S_Pi^-1, plus the job lists.
// A tile job and its packing: a block whose last tile row is ragged (nr < nc)
// is stored transposed, so that only the nc <= 64 stored columns of 64 rows
// are read; the roles of rows and columns (N and T parts, their inputs,
// outputs and output maps) swap with it.
static void add_tile(std::vector<PackJob>& pk, std::vector<TileJob>& tj, int64_t& off,
                     int64_t src_off, int ld, int row0, int col0, TileJob jb) {
  const bool trans = jb.nr < jb.nc;
  pk.push_back(PackJob{src_off, off, ld, row0, col0, jb.nr, jb.nc, trans ? 1 : 0});
  if (trans) {
    const int f = jb.flags;
    jb = TileJob{jb.m_off, jb.xc_off, jb.xr_off, jb.yc_off, jb.yr_off, jb.nc, jb.nr,
                 ((f & 1) << 1) | ((f & 2) >> 1) | ((f & 4) << 1) | ((f & 8) >> 1) | (f & ~15),
                 0};
  }
  jb.m_off = off;
  tj.push_back(jb);
  off += 64 * (int64_t)jb.nc;
}

// A tile read by two job lists (Phi: the apply's T part and the coarse
// correction's N part; coarse factor blocks: the forward and the backward
// sweep): one packing, two jobs with the same orientation.
static void add_tile_twice(std::vector<PackJob>& pk, std::vector<TileJob>& ja,
                         std::vector<TileJob>& jphi, int64_t& off, int64_t src_off, int ld,
                         int row0, int col0, TileJob japp, TileJob jphi_) {
  const int64_t off0 = off;
  add_tile(pk, ja, off, src_off, ld, row0, col0, japp);
  const bool trans = jphi_.nr < jphi_.nc;
  if (trans) {
    const int f = jphi_.flags;
    jphi_ = TileJob{0, jphi_.xc_off, jphi_.xr_off, jphi_.yc_off, jphi_.yr_off, jphi_.nc, jphi_.nr,
                    ((f & 1) << 1) | ((f & 2) >> 1) | ((f & 4) << 1) | ((f & 8) >> 1) | (f & ~15),
                    0};
  }
  jphi_.m_off = off0;
  jphi.push_back(jphi_);
}

// One tile of a row panel: the nrB x ncB block at (row0, col0) of a
// column-major source, stored as is (trans 0: the block's ncB columns) or
// transposed (trans 1: its nrB rows become the tile's columns).
static void add_panel_tile(std::vector<PackJob>& pk, std::vector<PanelTile>& tl, int64_t& off,
                           int elem_bytes, int64_t src_off, int ld, int row0, int col0, int nrB,
                           int ncB, int trans, int xc_off) {
  pk.push_back(PackJob{src_off, off, ld, row0, col0, nrB, ncB, trans});
  const int nc = trans ? nrB : ncB;
  tl.push_back(PanelTile{xc_off, nc});
  off += panel_tile_elems(nc, elem_bytes);
}

// Uploads the job lists of operator group g split at the handle's length
// for it (replacing the previous lists).
static int emit_panels(tcf_problem* h, int g) {
  // v: one launch's jobs in dispatch order
  auto up = [&](PanelJob*& dst, int* n, const std::vector<PanelJob>& v) -> int {
    if (dst) h->release(dst);
    dst = nullptr;
    RCCHK(h->upload(&dst, v));
    if (n) *n = (int)v.size();
    return TCF_OK;
  };
  const int c = h->chunk[g];
  const std::vector<PanelTile>& tl = h->h_ptile;
  if (g == 0) {
    RCCHK(up(h->pj_apply, &h->n_papply, split_jobs(h->w_apply, c, tl, h->p_eb)));
    RCCHK(up(h->pj_gt, &h->n_pgt, split_jobs(h->w_gt, c, tl, h->p_eb)));
  } else if (g == 1) {
    RCCHK(up(h->pj_pre, &h->n_ppre, split_jobs(h->w_pre, c, tl, h->p_eb)));
  } else if (g == 2) {
    RCCHK(up(h->pj_phi, &h->n_pphi, split_jobs(h->w_phi, c, tl, h->p_eb)));
  } else {
    RCCHK(up(h->pj_root, &h->n_proot, xcd_order(split_jobs(h->w_root, c, tl, 8))));
    std::vector<PanelJob> f, b;
    h->c_fwd_pre.assign(1, 0);
    h->c_bwd_pre.assign(1, 0);
    for (int lv = 0; lv < h->c_levels; ++lv) {
      // one launch per height: each height's jobs ordered on their own
      const std::vector<PanelJob> fl = xcd_order(split_jobs(h->w_fwd[lv], c, tl, 8));
      const std::vector<PanelJob> bl = xcd_order(split_jobs(h->w_bwd[lv], c, tl, 8));
      f.insert(f.end(), fl.begin(), fl.end());
      b.insert(b.end(), bl.begin(), bl.end());
      h->c_fwd_pre.push_back((int)f.size());
      h->c_bwd_pre.push_back((int)b.size());
    }
    RCCHK(up(h->pj_cfwd, nullptr, f));
    RCCHK(up(h->pj_cbwd, nullptr, b));
  }
  return TCF_OK;
}

// Row panels of the per-iteration operators for the matrix-core path:
// S_bb^-1 and S_bb whole (one panel per 64 dual rows of a patch), Phi_b^T
// (rows: the patch's primal entries) for the F apply and Phi_b for the
// coarse correction; for the coarse solve the top block's inverse whole,
// and per lower node L_JJ^-1 and (L_SJ L_JJ^-1) = -(-L_JJ^-T L_SJ^T)^T for
// the forward sweep, L_JJ^-T together with -L_JJ^-T L_SJ^T for the
// backward sweep.  Shared outputs: the coarse right-hand side (several
// patches hold a primal unknown) and the forward sweep's updates of
// ancestor unknowns (several nodes of one height update one ancestor).
template <class T>
static int build_panels(tcf_problem* h, hipStream_t st) {
  const int npm = std::max(h->n_primal, 1);
  {
    // the panel kernel addresses its column inputs by 32-bit byte offsets
    const int64_t ld = std::max<int64_t>({h->n_bptot + 3 * (int64_t)npm, h->n_btot, h->n_ptot});
    if (ld * h->rb * 8 >= ((int64_t)1 << 32)) {
      h->err = "problem too large for the matrix-core path (inputs beyond 4 GiB)";
      return TCF_EINVAL;
    }
  }
  std::vector<PackJob> pa, pb, pc, pl;
  std::vector<PanelTile> tl;
  std::vector<PanelJob> japp, jphi, jpre, jroot, jgt;
  std::vector<std::vector<PanelJob>> fw(h->c_levels), bw(h->c_levels);
  // deterministic sums: (target, staged row) pairs of the F apply's coarse
  // rows and of each height's ancestor rows, and the staged row counts
  std::vector<std::array<int, 2>> spa;
  std::vector<std::vector<std::array<int, 2>>> spf(h->c_levels);
  int sa = 0;
  std::vector<int> sl(h->c_levels, 0);
  int64_t oa = 0, ob = 0, oc = 0;
  auto begin = [&](int64_t off, int yr_off, int nr, int xr_off, int flags) {
    return PanelJob{off, (int)tl.size(), 0, yr_off, nr, xr_off, flags};
  };
  const int wT = (int)sizeof(T), wD = (int)sizeof(double);
  // a whole panel (split into jobs later, emit_panels)
  auto finish = [&](std::vector<PanelJob>& v, PanelJob j, int) {
    j.nt = (int)tl.size() - j.t0;
    if (j.nt > 0) v.push_back(j);
  };
  for (int s = 0; s < h->np_tot; ++s) {
    const DevPatch& d = h->hp[s];
    if (d.n_b == 0) continue;
    const int Tb = (d.n_b + 63) / 64, Tp = (d.n_p + 63) / 64;
    auto nrb = [&](int I) { return std::min(64, d.n_b - 64 * I); };
    auto nrp = [&](int K) { return std::min(64, d.n_p - 64 * K); };
    for (int I = 0; I < Tb; ++I) {
      // F apply: S_bb^-1 rows (vc, with x^T S_bb^-1 x), Phi_b^T rows (cv)
      PanelJob j = begin(oa, d.bp_off + 64 * I, nrb(I), d.b_off + 64 * I, 4);
      for (int J = 0; J < Tb; ++J)
        add_panel_tile(pa, tl, oa, wT, d.G_off, d.nb_pad, 64 * I, 64 * J, nrb(I), nrb(J), 0,
                       d.b_off + 64 * J);
      const size_t a0 = japp.size();
      finish(japp, j, wT);
      // G^T x unassembled (the dual-primal solve's pre and post phases):
      // the same tiles into the patch's bp block, no quadratic form
      for (size_t q = a0; q < japp.size(); ++q) {
        PanelJob g = japp[q];
        g.flags = 0;
        jgt.push_back(g);
      }
      // preconditioner: S_bb rows (tb, with r.z)
      PanelJob q = begin(ob, d.b_off + 64 * I, nrb(I), d.b_off + 64 * I, 4);
      for (int J = 0; J < Tb; ++J)
        add_panel_tile(pb, tl, ob, wT, d.S_off, d.nb_pad, 64 * I, 64 * J, nrb(I), nrb(J), 0,
                       d.b_off + 64 * J);
      finish(jpre, q, wT);
    }
    for (int K = 0; K < Tp; ++K) {
      PanelJob j = begin(oa, d.p_off + 64 * K, nrp(K), 0, 1 | 2);
      if (h->determ) {
        // staged: rows sa .. sa + nr of the staging block, each summed into
        // its coarse unknown afterwards
        j.yr_off = sa;
        j.flags = 8;
        for (int r = 0; r < nrp(K); ++r)
          spa.push_back({(int)h->n_bptot + h->cplan.nd[h->plans[s].p_rank[64 * K + r]], sa + r});
        sa += nrp(K);
      }
      for (int I = 0; I < Tb; ++I)
        add_panel_tile(pa, tl, oa, wT, d.G_off, d.nb_pad, 64 * I, d.n_b + 64 * K, nrb(I), nrp(K), 1,
                       d.b_off + 64 * I);
      const size_t a0 = japp.size();
      finish(japp, j, wT);
      for (size_t q = a0; q < japp.size(); ++q) {
        PanelJob g = japp[q];
        g.yr_off = d.bp_off + d.n_b + 64 * K;
        g.flags = 0;
        jgt.push_back(g);
      }
    }
    for (int I = 0; I < Tb && Tp > 0; ++I) {
      // coarse correction vc += Phi_b N q (inputs q through the primal ranks)
      PanelJob j = begin(oa, d.bp_off + 64 * I, nrb(I), 0, 0);
      for (int K = 0; K < Tp; ++K)
        add_panel_tile(pa, tl, oa, wT, d.G_off, d.nb_pad, 64 * I, d.n_b + 64 * K, nrb(I), nrp(K), 0,
                       d.p_off + 64 * K);
      finish(jphi, j, wT);
    }
  }
  std::vector<int> ctab(3 * (size_t)npm);
  std::iota(ctab.begin(), ctab.end(), 0);
  if (h->c_root >= 0) {
    const CoarseNodeDev& r = h->cnodes[h->c_root];
    const int Tr = (r.nj + 63) / 64;
    auto nrr = [&](int I) { return std::min(64, r.nj - 64 * I); };
    for (int I = 0; I < Tr; ++I) {
      PanelJob j = begin(oc, r.j0 + 64 * I, nrr(I), r.j0 + 64 * I, 4);
      for (int J = 0; J < Tr; ++J)
        add_panel_tile(pc, tl, oc, wD, 0, r.nj_pad, 64 * I, 64 * J, nrr(I), nrr(J), 0, r.j0 + 64 * J);
      finish(jroot, j, wD);
    }
    int stot = 0;
    for (const CoarseNodeDev& c : h->cnodes) stot += c.ns;
    const int sb0 = 3 * npm, sx0 = 3 * npm + stot;
    ctab.resize((size_t)sx0 + stot);
    for (size_t i = 0; i < h->cnodes.size(); ++i) {
      const CoarseNodeDev& c = h->cnodes[i];
      const std::vector<int>& S = h->cplan.nodes[i].S;
      for (int a = 0; a < c.ns; ++a) {
        ctab[sb0 + c.s_off + a] = S[a];
        ctab[sx0 + c.s_off + a] = 2 * npm + S[a];
      }
      if ((int)i == h->c_root) continue;
      const int lv = h->cplan.nodes[i].height;
      const int Tj = (c.nj + 63) / 64, Ts = (c.ns + 63) / 64;
      auto nrj = [&](int I) { return std::min(64, c.nj - 64 * I); };
      auto nrs = [&](int a) { return std::min(64, c.ns - 64 * a); };
      const int64_t mt = c.l_off + (int64_t)c.nj * c.nj_pad;  // -L_JJ^-T L_SJ^T, ld nj_pad
      for (int I = 0; I < Tj; ++I) {
        // forward: y_J = L_JJ^-1 b_J (into the y part)
        PanelJob j = begin(oc, npm + c.j0 + 64 * I, nrj(I), 0, 0);
        for (int K = 0; K <= I; ++K)
          add_panel_tile(pl, tl, oc, wD, c.l_off, c.nj_pad, 64 * I, 64 * K, nrj(I), nrj(K), 0,
                         c.j0 + 64 * K);
        finish(fw[lv], j, wD);
      }
      for (int a = 0; a < Ts; ++a) {
        // forward: b_S -= L_SJ L_JJ^-1 b_J (shared with the other nodes)
        PanelJob j = begin(oc, sb0 + c.s_off + 64 * a, nrs(a), 0, 1 | 2);
        if (h->determ) {
          j.yr_off = sl[lv];
          j.flags = 8;
          for (int r = 0; r < nrs(a); ++r) spf[lv].push_back({S[64 * a + r], sl[lv] + r});
          sl[lv] += nrs(a);
        }
        for (int K = 0; K < Tj; ++K)
          add_panel_tile(pl, tl, oc, wD, mt, c.nj_pad, 64 * K, 64 * a, nrj(K), nrs(a), 1,
                         c.j0 + 64 * K);
        finish(fw[lv], j, wD);
      }
      for (int K = 0; K < Tj; ++K) {
        // backward: x_J = L_JJ^-T y_J - L_JJ^-T L_SJ^T x_S
        PanelJob j = begin(oc, 2 * npm + c.j0 + 64 * K, nrj(K), 0, 0);
        for (int I = K; I < Tj; ++I)
          add_panel_tile(pl, tl, oc, wD, c.l_off, c.nj_pad, 64 * I, 64 * K, nrj(I), nrj(K), 1,
                         npm + c.j0 + 64 * I);
        for (int a = 0; a < Ts; ++a)
          add_panel_tile(pl, tl, oc, wD, mt, c.nj_pad, 64 * K, 64 * a, nrj(K), nrs(a), 0,
                         sx0 + c.s_off + 64 * a);
        finish(bw[lv], j, wD);
      }
    }
  }
  // the pack jobs of one buffer refer to it from offset 0
  T *pA, *pB;
  RCCHK(h->alloc(&pA, (size_t)std::max<int64_t>(oa, 1)));
  RCCHK(h->alloc(&pB, (size_t)std::max<int64_t>(ob, 1)));
  RCCHK(h->alloc(&h->d_pC, (size_t)std::max<int64_t>(oc, 1)));
  h->d_pA = pA;
  h->d_pB = pB;
  PackJob *dpa, *dpb, *dpc, *dpl;
  RCCHK(h->upload(&dpa, pa));
  RCCHK(h->upload(&dpb, pb));
  RCCHK(h->upload(&dpc, pc));
  RCCHK(h->upload(&dpl, pl));
  launch_pack_panel<T, T>(dpa, (int)pa.size(), (const T*)h->d_G, pA, st);
  launch_pack_panel<T, T>(dpb, (int)pb.size(), (const T*)h->d_S, pB, st);
  if (!pc.empty()) launch_pack_panel<double, double>(dpc, (int)pc.size(), h->d_SPinv, h->d_pC, st);
  if (!pl.empty()) launch_pack_panel<double, double>(dpl, (int)pl.size(), h->d_cL, h->d_pC, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  for (PackJob* b : {dpa, dpb, dpc, dpl}) h->release(b);
  if (h->d_SPinv) h->release(h->d_SPinv);
  if (h->d_cL) h->release(h->d_cL);
  h->d_SPinv = nullptr;
  h->d_cL = nullptr;
  h->h_ptile = tl;
  h->w_apply = std::move(japp);
  h->w_gt = std::move(jgt);
  h->w_pre = std::move(jpre);
  h->w_phi = std::move(jphi);
  h->w_root = std::move(jroot);
  h->w_fwd = std::move(fw);
  h->w_bwd = std::move(bw);
  h->p_eb = wT;
  // deterministic sums need whole panels (a split panel adds its parts)
  const int c0 = h->determ ? (1 << 20) : (h->opt.panel_chunk > 0 ? h->opt.panel_chunk : 16);
  for (int g = 0; g < 4; ++g) {
    h->chunk[g] = c0;
    RCCHK(emit_panels(h, g));
  }
  if (h->determ) {
    auto csr = [&](std::vector<std::array<int, 2>> pr, int*& tgt, int*& ptr, int*& idx,
                   int& n) -> int {
      std::sort(pr.begin(), pr.end());
      std::vector<int> t, pt(1, 0), ix;
      for (size_t i = 0; i < pr.size(); ++i) {
        if (i == 0 || pr[i][0] != pr[i - 1][0]) {
          if (i) pt.push_back((int)ix.size());
          t.push_back(pr[i][0]);
        }
        ix.push_back(pr[i][1]);
      }
      if (!pr.empty()) pt.push_back((int)ix.size());
      n = (int)t.size();
      RCCHK(h->upload(&tgt, t));
      RCCHK(h->upload(&ptr, pt));
      RCCHK(h->upload(&idx, ix));
      return TCF_OK;
    };
    RCCHK(csr(spa, h->sa_tgt, h->sa_ptr, h->sa_idx, h->n_sa));
    const int L = h->c_levels;
    h->sf_tgt.assign(L, nullptr);
    h->sf_ptr.assign(L, nullptr);
    h->sf_idx.assign(L, nullptr);
    h->n_sf.assign(L, 0);
    int rows = std::max(sa, 1);
    for (int lv = 0; lv < L; ++lv) {
      RCCHK(csr(spf[lv], h->sf_tgt[lv], h->sf_ptr[lv], h->sf_idx[lv], h->n_sf[lv]));
      rows = std::max(rows, sl[lv]);
    }
    h->stage_ld = rows;
    RCCHK(h->alloc(&h->d_stage, (size_t)rows * h->rb));
    const int jmax = std::max({h->n_papply, h->n_ppre, h->n_proot, 1});
    RCCHK(h->alloc(&h->d_qjob, (size_t)jmax * h->rb));
  }
  RCCHK(h->upload(&h->d_ptile, tl));
  RCCHK(h->upload(&h->d_cT, ctab));
  RCCHK(h->alloc(&h->d_cw1, (size_t)3 * npm * h->rb));
  RCCHK(h->alloc(&h->d_xg, (size_t)std::max<int64_t>(std::max(h->n_btot, h->n_ptot), 1) * h->rb));
  return TCF_OK;
}

// Tile copies of the per-iteration operators: lower tiles of S_bb^-1 (with
// the Phi_b tiles), of S_bb and of S_Pi^-1, plus the job lists.
template <class T>
static int build_tiles_narrow(tcf_problem* h, hipStream_t st);

template <class T>
static int build_tiles(tcf_problem* h, hipStream_t st) {
  RCCHK(h->wide ? build_panels<T>(h, st) : build_tiles_narrow<T>(h, st));
  const int npm = std::max(h->n_primal, 1);
  // c = Phi_b^T x goes straight into the coarse vector: cv = sum_s N_s^T c_s
  std::vector<int> cmap((size_t)std::max<int64_t>(h->n_ptot, 1), 0);
  for (int s = 0; s < h->np_tot; ++s)
    for (int j = 0; j < h->hp[s].n_p; ++j)
      cmap[h->hp[s].p_off + j] = (int)h->n_bptot + h->cplan.nd[h->plans[s].p_rank[j]];
  RCCHK(h->upload(&h->d_cmap, cmap));
  // per column j of rb: [vc | cv = b | y | x = q] (stride n_bptot + 3 n_Pi),
  // then p.Fp slots, tb, r.z slots, each block rb columns wide
  h->n_acc = (int64_t)h->rb * (h->n_bptot + 3 * npm + 2 * TCF_QSLOTS + h->n_btot);
  RCCHK(h->alloc(&h->d_acc, (size_t)h->n_acc));
  return TCF_OK;
}

template <class T>
static int build_tiles_narrow(tcf_problem* h, hipStream_t st) {
  std::vector<PackJob> pa, pb, pc;
  std::vector<TileJob> ja, jphi, jpre, jc;
  int64_t oa = 0, ob = 0, oc = 0;
  for (int s = 0; s < h->np_tot; ++s) {
    const DevPatch& d = h->hp[s];
    if (d.n_b == 0) continue;
    const int Tb = (d.n_b + 63) / 64, Tp = (d.n_p + 63) / 64;
    for (int J = 0; J < Tb; ++J)
      for (int I = J; I < Tb; ++I) {
        const int nr = std::min(64, d.n_b - 64 * I), nc = std::min(64, d.n_b - 64 * J);
        // N (+T off the diagonal) and the quadratic form x^T A x (bits 4, 5)
        const int fl = 1 | (I != J ? 2 | 32 : 0) | 16;
        add_tile(pa, ja, oa, d.G_off, d.nb_pad, 64 * I, 64 * J,
                 TileJob{0, d.b_off + 64 * I, d.b_off + 64 * J, d.bp_off + 64 * I,
                         d.bp_off + 64 * J, nr, nc, fl, 0});
        add_tile(pb, jpre, ob, d.S_off, d.nb_pad, 64 * I, 64 * J,
                 TileJob{0, d.b_off + 64 * I, d.b_off + 64 * J, d.b_off + 64 * I,
                         d.b_off + 64 * J, nr, nc, fl, 0});
      }
    for (int K = 0; K < Tp; ++K)
      for (int I = 0; I < Tb; ++I) {
        const int nr = std::min(64, d.n_b - 64 * I), nc = std::min(64, d.n_p - 64 * K);
        add_tile_twice(pa, ja, jphi, oa, d.G_off, d.nb_pad, 64 * I, d.n_b + 64 * K,
                     TileJob{0, d.b_off + 64 * I, 0, 0, d.p_off + 64 * K, nr, nc, 2 | 4, 0},
                     TileJob{0, 0, d.p_off + 64 * K, d.bp_off + 64 * I, 0, nr, nc, 1, 0});
      }
  }
  // coarse solve: lower tiles of the top block's dense inverse (both
  // triangles, one launch, inputs and outputs by offset), and per node below
  // it the tiles of L_JJ^-1 and -L_JJ^-T L_SJ^T, each read by a forward job
  // (y_J = L_JJ^-1 b_J, b_S -= L_SJ y_J) and a backward job (x_J = L_JJ^-T
  // y_J - L_JJ^-T L_SJ^T x_S), grouped by the node's height.  Work block per
  // column: b (the right-hand side, updated in place), y, x (the solution),
  // n_Pi entries each; the index table maps tile rows and columns to them.
  const int nP = h->n_primal, npm = std::max(nP, 1);
  std::vector<PackJob> pl;
  std::vector<std::vector<TileJob>> fw(h->c_levels), bw(h->c_levels);
  std::vector<int> ctab(3 * (size_t)npm);
  std::iota(ctab.begin(), ctab.end(), 0);
  if (h->c_root >= 0) {
    const CoarseNodeDev& r = h->cnodes[h->c_root];
    const int Tc = (r.nj + 63) / 64;
    for (int J = 0; J < Tc; ++J)
      for (int I = J; I < Tc; ++I) {
        const int nr = std::min(64, r.nj - 64 * I), nc = std::min(64, r.nj - 64 * J);
        add_tile(pc, jc, oc, 0, r.nj_pad, 64 * I, 64 * J,
                 TileJob{0, r.j0 + 64 * I, r.j0 + 64 * J, r.j0 + 64 * I, r.j0 + 64 * J, nr, nc,
                         1 | (I != J ? 2 | 32 : 0) | 16, 0});
      }
    int stot = 0;
    for (const CoarseNodeDev& c : h->cnodes) stot += c.ns;
    const int sb0 = 3 * npm, sx0 = 3 * npm + stot;
    ctab.resize((size_t)sx0 + stot);
    for (size_t i = 0; i < h->cnodes.size(); ++i) {
      const CoarseNodeDev& c = h->cnodes[i];
      const std::vector<int>& S = h->cplan.nodes[i].S;
      for (int a = 0; a < c.ns; ++a) {
        ctab[sb0 + c.s_off + a] = S[a];
        ctab[sx0 + c.s_off + a] = 2 * npm + S[a];
      }
      if ((int)i == h->c_root) continue;
      const int lv = h->cplan.nodes[i].height;
      const int Tj = (c.nj + 63) / 64, Ts = (c.ns + 63) / 64;
      for (int K = 0; K < Tj; ++K)
        for (int I = K; I < Tj; ++I) {
          const int nr = std::min(64, c.nj - 64 * I), nc = std::min(64, c.nj - 64 * K);
          add_tile_twice(pl, fw[lv], bw[lv], oc, c.l_off, c.nj_pad, 64 * I, 64 * K,
                         TileJob{0, 0, c.j0 + 64 * K, npm + c.j0 + 64 * I, 0, nr, nc, 1 | 8, 0},
                         TileJob{0, npm + c.j0 + 64 * I, 0, 0, 2 * npm + c.j0 + 64 * K, nr, nc,
                                 2 | 4, 0});
        }
      for (int K = 0; K < Tj; ++K)
        for (int a = 0; a < Ts; ++a) {
          const int nr = std::min(64, c.nj - 64 * K), nc = std::min(64, c.ns - 64 * a);
          add_tile_twice(pl, fw[lv], bw[lv], oc, c.l_off + (int64_t)c.nj * c.nj_pad, c.nj_pad,
                         64 * K, 64 * a,
                         TileJob{0, c.j0 + 64 * K, 0, 0, sb0 + c.s_off + 64 * a, nr, nc, 2 | 4, 0},
                         TileJob{0, 0, sx0 + c.s_off + 64 * a, 2 * npm + c.j0 + 64 * K, 0, nr, nc,
                                 1 | 8, 0});
        }
    }
  }
  T *tA, *tB;
  RCCHK(h->alloc(&tA, (size_t)oa));
  RCCHK(h->alloc(&tB, (size_t)ob));
  RCCHK(h->alloc(&h->d_tC, (size_t)oc));
  h->d_tA = tA;
  h->d_tB = tB;
  PackJob *dpa, *dpb, *dpc, *dpl;
  RCCHK(h->upload(&dpa, pa));
  RCCHK(h->upload(&dpb, pb));
  RCCHK(h->upload(&dpc, pc));
  RCCHK(h->upload(&dpl, pl));
  launch_pack_tiles<T, T>(dpa, (int)pa.size(), (const T*)h->d_G, tA, st);
  launch_pack_tiles<T, T>(dpb, (int)pb.size(), (const T*)h->d_S, tB, st);
  if (!pc.empty()) launch_pack_tiles<double, double>(dpc, (int)pc.size(), h->d_SPinv, h->d_tC, st);
  if (!pl.empty()) launch_pack_tiles<double, double>(dpl, (int)pl.size(), h->d_cL, h->d_tC, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  h->release(dpa);
  h->release(dpb);
  h->release(dpc);
  h->release(dpl);
  // the coarse operators live on as tiles only
  if (h->d_SPinv) h->release(h->d_SPinv);
  if (h->d_cL) h->release(h->d_cL);
  h->d_SPinv = nullptr;
  h->d_cL = nullptr;
  {
    std::vector<TileJob> f, b;
    h->c_fwd_pre.assign(1, 0);
    h->c_bwd_pre.assign(1, 0);
    for (int lv = 0; lv < h->c_levels; ++lv) {
      f.insert(f.end(), fw[lv].begin(), fw[lv].end());
      b.insert(b.end(), bw[lv].begin(), bw[lv].end());
      h->c_fwd_pre.push_back((int)f.size());
      h->c_bwd_pre.push_back((int)b.size());
    }
    RCCHK(h->upload(&h->tj_cfwd, f));
    RCCHK(h->upload(&h->tj_cbwd, b));
    RCCHK(h->upload(&h->d_cT, ctab));
    RCCHK(h->alloc(&h->d_cw1, (size_t)3 * npm * h->rb));
  }
  RCCHK(h->upload(&h->tj_apply, ja));
  RCCHK(h->upload(&h->tj_phi, jphi));
  RCCHK(h->upload(&h->tj_pre, jpre));
  RCCHK(h->upload(&h->tj_coarse, jc));
  h->n_tapply = (int)ja.size();
  h->n_tphi = (int)jphi.size();
  h->n_tpre = (int)jpre.size();
  h->n_tcoarse = (int)jc.size();
  return TCF_OK;
}

template <class T>
static int tune_panels(tcf_problem* h, hipStream_t st);

extern "C" int tcf_setup(tcf_problem* h, void* stream) {
  if (!h) return TCF_EINVAL;
  if (h->is_setup) { h->err = "setup already done"; return TCF_ESTATE; }
  hipStream_t st = (hipStream_t)stream;
  h->mem_stream = st;
  HIPCHK(hipGetDevice(&h->device));
  const double t0 = now_ms();
  int rc;
  Range rg("tcf setup");
  try {
    {
      Range r1("tcf setup: assembly, local factors, coarse factor");
      if (h->precision == TCF_FP32_FULL_IR)
        rc = setup_impl<float, float>(h, st);
      else if (h->precision == TCF_FP32_IR)
        rc = setup_impl<double, float>(h, st);
      else
        rc = setup_impl<double, double>(h, st);
    }
    if (!rc) {
      Range r2("tcf setup: operator tiles");
      rc = h->precision == TCF_FP64 ? build_tiles<double>(h, st) : build_tiles<float>(h, st);
    }
    if (!rc && h->wide) {
      Range r3("tcf setup: panel split lengths");
      rc = h->precision == TCF_FP64 ? tune_panels<double>(h, st) : tune_panels<float>(h, st);
    }
  } catch (const std::bad_alloc&) {
    h->err = "out of host memory in setup";
    return TCF_ENOMEM;
  }
  if (rc) return rc;
  h->setup_ms = now_ms() - t0;
  h->is_setup = true;
  return TCF_OK;
}

// ============================================================================
// Per-step dual-primal solve
// ============================================================================
// wb = base_bp[b part] + alpha * Phi_b N_s q  (per patch; Phi_b = columns n_b.. of G)
template <class T>
static void phi_apply(tcf_problem* h, const double* base_bp, double alpha, const double* q,
                      double* wb, const int* done, hipStream_t st) {
  launch_scatter((int)h->n_btot, nullptr, h->d_b2bp, base_bp, 1.0, wb, done, st);
  if (h->n_primal > 0)
    launch_axpyrows<T>(h->aj_phi, h->ap_phi, h->nj_phi, h->nt_phi, h->max_np, (const T*)h->d_G, q,
                       h->d_prank, wb, h->a_boff_b, alpha, wb, 0, done, st);
}

// x = S_Pi^-1 b on R columns of a coarse work block [b | y | x] (n_Pi
// entries each, column stride ld, all cleared beforehand): forward sweep
// over the heights of the factor's elimination tree (b is updated in place,
// y_J = L_JJ^-1 b_J), the top block's dense inverse, backward sweep.  With
// slots, adds b^T S_Pi^-1 b per column: |y|^2 over the lower nodes plus the
// top block's quadratic form.
static void coarse_sweeps(tcf_problem* h, int R, double* base, int ld, double* slots,
                          const int* done, hipStream_t st) {
  if (h->c_root < 0) return;
  const int npm = std::max(h->n_primal, 1);
  // kernel timing covers the PCG's coarse solves (the ones with slots) only
  auto timed = [&](int g, hipStream_t s, auto&& f) {
    if (slots) ::timed(h, g, s, f);
    else f();
  };
  const bool wide = h->wide;
  for (int lv = 0; lv < h->c_levels; ++lv) {
    const int j0 = h->c_fwd_pre[lv], nj = h->c_fwd_pre[lv + 1] - j0;
    timed(TCF_KG_COARSE, st, [&] {
      if (wide)
        launch_panels<double>(4, R, h->pj_cfwd + j0, h->d_ptile, nj, h->d_pC, base, ld, h->d_cT,
                              base, ld, h->d_cT, nullptr, done, st, h->d_stage, h->stage_ld);
      else
        launch_tiles<double>(4, R, h->tj_cfwd + j0, nj, h->d_tC, base, ld, h->d_cT, nullptr, 1.0,
                             base, ld, h->d_cT, nullptr, done, st);
    });
    if (h->determ)
      launch_stage_add(h->n_sf[lv], h->sf_tgt[lv], h->sf_ptr[lv], h->sf_idx[lv], h->d_stage,
                       h->stage_ld, R, base, ld, done, st);
  }
  const CoarseNodeDev& r = h->cnodes[h->c_root];
  if (slots && r.j0 > 0) launch_sumsq_slots(R, r.j0, base + npm, ld, slots, done, st);
  timed(TCF_KG_COARSE, st, [&] {
    if (wide)
      launch_panels<double>(3, R, h->pj_root, h->d_ptile, h->n_proot, h->d_pC, base, ld, nullptr,
                            base + 2 * npm, ld, nullptr, slots, done, st, nullptr, 0,
                            h->determ && slots ? h->d_qjob : nullptr);
    else
      launch_tiles<double>(3, R, h->tj_coarse, h->n_tcoarse, h->d_tC, base, ld, nullptr, nullptr,
                           1.0, base + 2 * npm, ld, nullptr, slots, done, st);
  });
  if (h->determ && slots) launch_qjob_add(R, h->n_proot, h->d_qjob, slots, done, st);
  for (int lv = h->c_levels - 1; lv >= 0; --lv) {
    const int j0 = h->c_bwd_pre[lv], nj = h->c_bwd_pre[lv + 1] - j0;
    timed(TCF_KG_COARSE, st, [&] {
      if (wide)
        launch_panels<double>(4, R, h->pj_cbwd + j0, h->d_ptile, nj, h->d_pC, base, ld, h->d_cT,
                              base, ld, h->d_cT, nullptr, done, st);
      else
        launch_tiles<double>(4, R, h->tj_cbwd + j0, nj, h->d_tC, base, ld, h->d_cT, nullptr, 1.0,
                             base, ld, h->d_cT, nullptr, done, st);
    });
  }
}

// Coarse solves of a batch's columns at once: column j of the coarse work
// block (stride 3 n_Pi) holds its right-hand side in its b part, with y and
// x cleared; the solutions land in the x parts.
static void coarse_solve_cols(tcf_problem* h, int ncols, hipStream_t st) {
  if (h->n_primal == 0 || ncols == 0) return;
  const int npm = std::max(h->n_primal, 1);
  coarse_sweeps(h, ncols, h->d_cw1, 3 * npm, nullptr, nullptr, st);
}

// Views into the tile path's accumulator block (see pcg_iteration).
struct TileAcc {
  double *vc, *q, *pq, *tb, *rz;
  int lf, npm;              // column stride of [vc | b | y | x], and n_Pi (at least 1)
  int64_t n_head, n_tail;   // [vc .. p.Fp slots] and [tb .. r.z slots] lengths
};
static TileAcc tile_acc(tcf_problem* h) {
  TileAcc a;
  const int R = h->rb;
  a.npm = std::max(h->n_primal, 1);
  a.lf = (int)h->n_bptot + 3 * a.npm;
  a.vc = h->d_acc;
  a.q = a.vc + h->n_bptot + 2 * a.npm;
  a.pq = a.vc + (int64_t)a.lf * R;
  a.tb = a.pq + (int64_t)TCF_QSLOTS * R;
  a.rz = a.tb + h->n_btot * R;
  a.n_head = (int64_t)(a.lf + TCF_QSLOTS) * R;
  a.n_tail = (h->n_btot + TCF_QSLOTS) * R;
  return a;
}

// The F apply, the coarse correction (Phi_b N q) and the preconditioner on
// R columns, through the tiles or (wide batches) the row panels, whose
// inputs are gathered first into d_xg.  tm: time the product as its kernel
// group.
template <class F>
static void maybe_timed(tcf_problem* h, bool tm, int g, hipStream_t st, F&& f) {
  if (tm) timed(h, g, st, f);
  else f();
}
template <class T>
static void op_apply(tcf_problem* h, const TileAcc& a, const double* x, const int* done,
                     hipStream_t st, bool tm) {
  const int R = h->rb, nl = h->n_lambda, nb = (int)h->n_btot;
  if (h->wide) {
    launch_gather_cols(R, nb, h->d_brow, h->d_bsgn_d, h->dt, x, nl, h->d_xg, nb, done, st);
    maybe_timed(h, tm, TCF_KG_APPLY, st, [&] {
      launch_panels<T>(0, R, h->pj_apply, h->d_ptile, h->n_papply, (const T*)h->d_pA, h->d_xg,
                       nb, nullptr, a.vc, a.lf, h->d_cmap, a.pq, done, st, h->d_stage,
                       h->stage_ld, h->d_qjob);
    });
    if (h->determ) {
      launch_stage_add(h->n_sa, h->sa_tgt, h->sa_ptr, h->sa_idx, h->d_stage, h->stage_ld, R,
                       a.vc, a.lf, done, st);
      launch_qjob_add(R, h->n_papply, h->d_qjob, a.pq, done, st);
    }
  } else {
    maybe_timed(h, tm, TCF_KG_APPLY, st, [&] {
      launch_tiles<T>(0, R, h->tj_apply, h->n_tapply, (const T*)h->d_tA, x, nl, h->d_brow,
                      h->d_bsgn_d, h->dt, a.vc, a.lf, h->d_cmap, a.pq, done, st);
    });
  }
}
template <class T>
static void op_phi(tcf_problem* h, const TileAcc& a, const int* done, hipStream_t st, bool tm) {
  const int R = h->rb, np = (int)h->n_ptot;
  if (h->wide) {
    launch_gather_cols(R, np, h->d_prank, nullptr, 1.0, a.q, a.lf, h->d_xg, np, done, st);
    maybe_timed(h, tm, TCF_KG_PHI, st, [&] {
      launch_panels<T>(1, R, h->pj_phi, h->d_ptile, h->n_pphi, (const T*)h->d_pA, h->d_xg, np,
                       nullptr, a.vc, a.lf, nullptr, nullptr, done, st);
    });
  } else {
    maybe_timed(h, tm, TCF_KG_PHI, st, [&] {
      launch_tiles<T>(1, R, h->tj_phi, h->n_tphi, (const T*)h->d_tA, a.q, a.lf, h->d_prank,
                      nullptr, 1.0, a.vc, a.lf, nullptr, nullptr, done, st);
    });
  }
}
template <class T>
static void op_precond(tcf_problem* h, const TileAcc& a, const double* r, const int* done,
                       hipStream_t st, bool tm) {
  const int R = h->rb, nl = h->n_lambda, nb = (int)h->n_btot;
  if (h->wide) {
    launch_gather_cols(R, nb, h->d_brow, h->d_pre_w, 1.0, r, nl, h->d_xg, nb, done, st);
    maybe_timed(h, tm, TCF_KG_PRECOND, st, [&] {
      launch_panels<T>(2, R, h->pj_pre, h->d_ptile, h->n_ppre, (const T*)h->d_pB, h->d_xg, nb,
                       nullptr, a.tb, nb, nullptr, a.rz, done, st, nullptr, 0, h->d_qjob);
    });
    if (h->determ) launch_qjob_add(R, h->n_ppre, h->d_qjob, a.rz, done, st);
  } else {
    maybe_timed(h, tm, TCF_KG_PRECOND, st, [&] {
      launch_tiles<T>(2, R, h->tj_pre, h->n_tpre, (const T*)h->d_tB, r, nl, h->d_brow,
                      h->d_pre_w, 1.0, a.tb, nb, nullptr, a.rz, done, st);
    });
  }
}

// Split lengths of the row panels per operator.  A tune table (a text file,
// one line per problem shape: the shape's key, then the four lengths) is
// consulted first; without an entry and with autotune set, each operator
// is timed at setup for every candidate length (one untimed and two timed
// launches on inputs cleared to zero) and the fastest is kept, and written
// to the table when one is named.
static std::string tune_key(const tcf_problem* h) {
  int nb = 0, np = 0;
  for (const DevPatch& d : h->hp) {
    nb = std::max(nb, d.n_b);
    np = std::max(np, d.n_p);
  }
  char buf[256];
  snprintf(buf, sizeof buf, "panels-v1 patches=%d nb_max=%d np_max=%d primal=%d nodes=%d rb=%d prec=%d",
           h->np_tot, nb, np, h->n_primal, (int)h->cnodes.size(), h->rb, h->precision);
  return buf;
}

template <class T>
static int tune_panels(tcf_problem* h, hipStream_t st) {
  const std::string key = tune_key(h);
  if (h->opt.tune_table && !h->determ) {
    FILE* f = fopen(h->opt.tune_table, "r");
    if (f) {
      char line[512];
      while (fgets(line, sizeof line, f)) {
        int c[4];
        const size_t n = key.size();
        if (strncmp(line, key.c_str(), n) == 0 && line[n] == ' ' &&
            sscanf(line + n, " chunks %d %d %d %d", &c[0], &c[1], &c[2], &c[3]) == 4 &&
            c[0] > 0 && c[1] > 0 && c[2] > 0 && c[3] > 0) {
          for (int g = 0; g < 4; ++g) {
            h->chunk[g] = c[g];
            RCCHK(emit_panels(h, g));
          }
          h->chunk_src = 1;
        }
      }
      fclose(f);
      if (h->chunk_src == 1) return TCF_OK;
    }
  }
  if (!h->opt.autotune || h->determ) return TCF_OK;
  const TileAcc a = tile_acc(h);
  launch_zero((int64_t)h->n_lambda * h->rb, h->d_p, st);
  launch_zero((int64_t)h->n_lambda * h->rb, h->d_r, st);
  launch_zero(h->n_acc, h->d_acc, st);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  auto run = [&](int g) {
    if (g == 0) op_apply<T>(h, a, h->d_p, nullptr, st, false);
    else if (g == 1) op_precond<T>(h, a, h->d_r, nullptr, st, false);
    else if (g == 2) op_phi<T>(h, a, nullptr, st, false);
    else coarse_sweeps(h, h->rb, a.vc + h->n_bptot, a.lf, nullptr, nullptr, st);
  };
  int rc = TCF_OK;
  for (int g = 0; g < 4 && !rc; ++g) {
    if ((g == 2 && h->n_pphi == 0) || (g == 3 && h->c_root < 0)) continue;
    const int cands[] = {4, 8, 16, 32, 1 << 20};
    float best = 1e30f;
    int bestc = h->chunk[g];
    for (int ci = 0; ci < 5; ++ci) {
      const int c = cands[ci];
      h->chunk[g] = c;
      if ((rc = emit_panels(h, g))) break;
      run(g);
      if (hipEventRecord(e0, st) != hipSuccess) { rc = TCF_EHIP; break; }
      run(g);
      run(g);
      float ms = 0.f;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = TCF_EHIP;
        break;
      }
      h->tune_us[g][ci] = ms * 500.0;  // two launches, ms -> us per launch
      if (ms < best) {
        best = ms;
        bestc = c;
      }
    }
    h->chunk[g] = bestc;
    if (!rc) rc = emit_panels(h, g);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) {
    if (h->err.empty()) h->err = "panel tuning failed";
    return rc;
  }
  launch_zero(h->n_acc, h->d_acc, st);
  HIPCHK(hipGetLastError());
  h->chunk_src = 2;
  if (h->opt.tune_table) {
    FILE* f = fopen(h->opt.tune_table, "a");
    if (f) {
      fprintf(f, "%s chunks %d %d %d %d\n", key.c_str(), h->chunk[0], h->chunk[1], h->chunk[2],
              h->chunk[3]);
      fclose(f);
    }
  }
  return TCF_OK;
}

// One PCG iteration with the given parity (launch sequence only).
template <class T>
static void pcg_iteration(tcf_problem* h, int par, hipStream_t st) {
  {
    // Tile path, 6 launches, rb columns (excitations) at once.  Accumulators
    // (each block rb columns wide): [vc | cv] per column (vc gets S_bb^-1 x
    // and Phi_b N q, cv = sum_s N_s^T Phi_b^T x_s), q the coarse solution,
    // slots of p.Fp = x^T S_bb^-1 x + cv^T S_Pi^-1 cv, tb = S_bb B^T r, slots
    // of r.z = (B^T r)^T S_bb (B^T r).  The update clears [tb, r.z slots],
    // the search-direction update clears [vc .. p.Fp slots]; all are cleared
    // once before a solve.
    const TileAcc a = tile_acc(h);
    const int R = h->rb, nl = h->n_lambda, npt = h->npart;
    PcgScalars* stv = h->d_st;
    const int* alldone = &h->d_st[R].done;
    double* p_rr = h->d_part;
    const double tol2 = h->pcg_tol * h->pcg_tol;
    op_apply<T>(h, a, h->d_p, alldone, st, true);
    if (h->n_primal > 0) {
      coarse_sweeps(h, R, a.vc + h->n_bptot, a.lf, a.pq, alldone, st);
      op_phi<T>(h, a, alldone, st, true);
    }
    launch_pcg_update_t(R, nl, h->d_posp_bp, h->d_posm_bp, a.vc, a.lf, h->dt, a.pq, stv, par,
                        h->d_lam, h->d_r, h->d_p, p_rr, npt, a.tb, a.n_tail, st);
    op_precond<T>(h, a, h->d_r, alldone, st, true);
    launch_pcg_pupdate_t(R, nl, h->d_posp, h->d_posm, a.tb, (int)h->n_btot, h->d_zwp, h->d_zwm,
                         a.rz, p_rr, npt, stv, par, tol2, h->d_p, a.vc, a.n_head, st);
  }
}

// Captures graph_iters iterations (parity 0, 1, 0, ...) into a graph replayed per chunk.
// If capture or instantiation fails, the handle falls back to stream
// launches (same kernels) instead of failing.
template <class T>
static int build_pcg_graph(tcf_problem* h) {
  if (h->pcg_graph || h->graph_failed) return TCF_OK;
  std::lock_guard<std::mutex> lk(g_capture_mu);
  if (!h->cap_stream && hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    h->graph_failed = true;
    return TCF_OK;
  }
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    h->graph_failed = true;
    (void)hipGetLastError();
    return TCF_OK;
  }
  for (int q = 0; q < h->graph_iters; ++q) pcg_iteration<T>(h, q & 1, h->cap_stream);
  hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  if (e == hipSuccess) e = hipGraphInstantiate(&h->pcg_graph, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    h->pcg_graph = nullptr;
    h->graph_failed = true;
    (void)hipGetLastError();
  }
  return TCF_OK;
}

// PCG on the multipliers for the rb columns of d (columns past the active
// excitations hold zeros and are converged from the start).  Per column:
// iteration count and whether it converged within maxit.
template <class T>
static int pcg_solve(tcf_problem* h, hipStream_t st, int* iters, bool* conv) {
  Range rg("PCG solve");
  const int nl = h->n_lambda, R = h->rb;
  for (int j = 0; j < R; ++j) {
    iters[j] = 0;
    conv[j] = true;
  }
  h->last_rel = 0.0;
  if (nl == 0) return TCF_OK;
  const int npt = h->npart;
  {
    const TileAcc a = tile_acc(h);
    double* p_dd = h->d_part + (int64_t)npt * R;
    launch_zero(h->n_acc, h->d_acc, st);
    if (h->warm_init) {
      // r0 = d - F lambda0: one F apply on the lambda columns as set
      op_apply<T>(h, a, h->d_lam, nullptr, st, false);
      if (h->n_primal > 0) {
        coarse_sweeps(h, R, a.vc + h->n_bptot, a.lf, a.pq, nullptr, st);
        op_phi<T>(h, a, nullptr, st, false);
      }
      launch_pcg_init_w(R, nl, h->d_posp_bp, h->d_posm_bp, a.vc, a.lf, h->dt, h->d_d, h->d_r,
                        p_dd, npt, st);
      launch_zero(a.n_head, a.vc, st);
      h->warm_init = false;
    } else {
      launch_pcg_init_t(R, nl, h->d_d, h->d_lam, h->d_r, p_dd, npt, st);
    }
    op_precond<T>(h, a, h->d_r, nullptr, st, false);
    launch_pcg_init2_t(R, nl, h->d_posp, h->d_posm, a.tb, (int)h->n_btot, h->d_zwp, h->d_zwm,
                       a.rz, p_dd, npt, h->d_st, h->d_p, st);
  }
  // flag the host reads: the all-columns flag on the tile path
  const int fl = R;
  const int maxit = h->opt.pcg_maxit > 0 ? h->opt.pcg_maxit : std::max(1000, nl);
  const bool want_graph = h->opt.use_graph && !h->prof_on && !h->no_graph_call;
  if (want_graph) RCCHK(build_pcg_graph<T>(h));
  const bool graph = want_graph && h->pcg_graph;
  const int chunk = std::max(2, h->opt.check_every / 2 * 2);
  // Host reads of the convergence flag stall the stream.  Solves of the
  // same kind (same refinement sweep) take nearly the same number of
  // iterations from step to step: the first read comes a few iterations
  // before the previous count, later ones every min(chunk, 4) iterations.
  const int kind = std::min(h->cur_sweep, TCF_PRED_KINDS - 1);
  const int pred = h->pred_iters[kind];
  const int gi = h->graph_iters;
  int seg = pred > chunk + 6 ? (pred - 6) / gi * gi : chunk;
  int it = 0;
  bool finished = false;
  auto max_iters = [&] {
    int m = 0;
    for (int j = 0; j < R; ++j) m = std::max(m, h->h_st[j].iters);
    return m;
  };
  while (it < maxit && !finished) {
    const int it1 = std::min(maxit, it + seg);
    seg = std::min(chunk, 4);
    while (it < it1) {
      if (graph && it + h->graph_iters <= it1 && (it & 1) == 0) {
        HIPCHK(hipGraphLaunch(h->pcg_graph, st));
        it += h->graph_iters;
      } else {
        h->cur_it = it;
        pcg_iteration<T>(h, it & 1, st);
        ++it;
      }
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(h->h_st, h->d_st, sizeof(PcgScalars) * (fl + 1), hipMemcpyDeviceToHost,
                          st));
    HIPCHK(hipStreamSynchronize(st));
    finished = h->h_st[fl].done != 0;
    if (h->prof_on) h->prof_flush(finished ? max_iters() : INT32_MAX);
  }
  h->cur_it = -1;
  const int ncol = R;
  double rel = 0.0;
  for (int j = 0; j < ncol; ++j) {
    iters[j] = h->h_st[j].iters;
    conv[j] = h->h_st[j].done != 0;
    if (h->h_st[j].dd > 0) rel = std::max(rel, std::sqrt(h->h_st[j].rr / h->h_st[j].dd));
  }
  if (finished) h->pred_iters[kind] = max_iters();
  h->last_rel = rel;
  return TCF_OK;
}

// Dual-primal solve of W x = f, split around the (batched) PCG.  The
// right-hand side is given per patch (kept order): rhs == nullptr selects
// the time-step form f = M a_k + dt g_k(t_{l+1}) jhat_k of excitation k,
// whose source part was condensed at setup; otherwise f = rhs (all patches
// condensed).  If base != nullptr the solution is a correction to base and
// the interface constraint is Bhat (base + x) = 0, i.e. the dual right-hand
// side becomes d + Bhat base.  Column j of the PCG vectors carries it.
//
// solve_pre: [u; c0] = G^T g_b, h = sum N^T (g_p - c0), q0 = S_Pi^-1 h,
// d = jump(u - Phi N q0) into column j.
// Condensation of the right-hand sides of excitations k0 .. k0 + nc - 1
// into ygg (columns k0 .. of d_ygg).  rhs == nullptr: the time-step form
// f = M a_k + dt g_k(t_{l+1}) jhat_k, whose source part was condensed at
// setup, so only the conductor patches' M a_k is condensed; else rhs
// holds the nc right-hand sides (column j at rhs + j * ldv, all patches).
// Batches wider than two go through the matrix-core form, which reads Q^T
// once for all of them.
template <class T>
static void condense_batch(tcf_problem* h, int k0, int nc, int l, const double* rhs,
                           hipStream_t st) {
  const int64_t ldv = h->n_rtot;
  const T* Q = (const T*)h->d_Q;
  double* ygg = h->d_ygg + (int64_t)k0 * ldv;
  const bool wide = nc > 2;
  if (!rhs) {
    for (int j = 0; j < nc; ++j) {
      const int k = k0 + j;
      const double gk = h->amp[(size_t)k * h->n_steps + l];
      launch_axpby(ldv, h->dt * gk, h->d_yggs + (int64_t)k * ldv, 0.0, ygg + (int64_t)j * ldv, st);
    }
    if (h->cond_list.empty()) return;
    double* a = h->d_a + (int64_t)k0 * ldv;
    double* fM = h->d_fM + (int64_t)k0 * ldv;
    launch_wapply(h->dP, h->d_cond, h->d_cond_rprefix, (int)h->cond_list.size(), h->nt_cond_r, nc,
                  h->d_rloc, h->d_loc2r, h->d_tabs, h->dt, 1, a, fM, ldv, st);
    // the initial value enters the first step as M a^(0) = int sigma A_0 . w
    if (l == 0 && h->d_m0)
      launch_axpby(ldv * nc, 1.0, h->d_m0 + (int64_t)k0 * ldv, 1.0, fM, st);
    timed(h, TCF_KG_CONDENSE, st, [&] {
      if (wide)
        launch_condense_w<T>(h->dP, h->d_cond, h->d_cond_wprefix, (int)h->cond_list.size(),
                             h->nt_cond_w, nc, Q, fM, ygg, ldv, st);
      else
        launch_condense<T>(h->dP, h->d_cond, h->d_cond_cprefix, (int)h->cond_list.size(),
                           h->nt_cond_c, nc, h->max_ni, Q, fM, ygg, ldv, st);
    });
  } else {
    launch_zero(ldv * nc, ygg, st);
    if (wide)
      launch_condense_w<T>(h->dP, h->d_all, h->d_all_wprefix, h->np_tot, h->nt_all_w, nc, Q, rhs,
                           ygg, ldv, st);
    else
      launch_condense<T>(h->dP, h->d_all, h->d_all_cprefix, h->np_tot, h->nt_all_c, nc,
                         h->max_ni, Q, rhs, ygg, ldv, st);
  }
}

// Dual-primal solves of W x = f, split around the batched PCG, for the
// columns cols of a batch whose excitations start at k0 (column j carries
// excitation k0 + j), with f condensed into ygg beforehand (condense_batch).
// With corr the solutions are corrections to the fields a and the interface
// constraint is Bhat (a + x) = 0, i.e. the dual right-hand side becomes
// d + Bhat a.  The coarse solves of all columns run as one batch.
//
// solve_pre: [u; c0] = G^T g_b, h = sum N^T (g_p - c0), q0 = S_Pi^-1 h,
// d = jump(u - Phi N q0) into column j of the PCG's right-hand sides.
template <class T>
static void solve_pre(tcf_problem* h, int k0, const std::vector<int>& cols, bool corr,
                      hipStream_t st) {
  const int64_t ldv = h->n_rtot;
  const int npm = std::max(h->n_primal, 1);
  const T* G = (const T*)h->d_G;
  if (cols.empty()) return;
  const int ncols = cols.back() + 1;
  const int nb = (int)h->n_btot, np = (int)h->n_ptot;
  if (h->n_primal > 0) launch_zero((int64_t)3 * npm * ncols, h->d_cw1, st);
  if (h->wide) {
    // [u; c0] of every column at once through the row panels of G^T
    launch_gather_cols(ncols, nb, h->d_b2r, nullptr, 1.0, h->d_ygg + (int64_t)k0 * ldv, (int)ldv,
                       h->d_xg, nb, nullptr, st);
    launch_zero(h->n_bptot * ncols, h->d_uc, st);
    launch_panels<T>(0, ncols, h->pj_gt, h->d_ptile, h->n_pgt, (const T*)h->d_pA, h->d_xg, nb,
                     nullptr, h->d_uc, (int)h->n_bptot, nullptr, nullptr, nullptr, st);
  }
  for (int j : cols) {
    const double* ygg = h->d_ygg + (int64_t)(k0 + j) * ldv;
    double* uc = h->d_uc + (int64_t)j * h->n_bptot;
    double* hv = h->d_h + (int64_t)j * npm;
    if (!h->wide) {
      if (h->bp_gaps) launch_zero(h->n_bptot, uc, st);
      launch_dotcols<T>(h->dj_app_v, h->dp_app, h->nj_app, h->nt_app, h->max_nb, G, 0, ygg,
                        nullptr, nullptr, 1.0, uc, nullptr, st);
    }
    if (h->n_primal > 0) {
      launch_coarse_gather(h->n_primal, h->d_cptr, h->d_cidx_r, ygg, 1.0, h->d_cidx_bp, uc, -1.0,
                           nullptr, hv, nullptr, st);
      launch_axpby(h->n_primal, 1.0, hv, 0.0, h->d_cw1 + (int64_t)j * 3 * npm, st);
    }
  }
  coarse_solve_cols(h, ncols, st);
  if (h->wide) {
    // v = u - Phi_b N q0 of every column (bp space) through the Phi panels
    launch_axpby(h->n_bptot * ncols, 1.0, h->d_uc, 0.0, h->d_vc, st);
    if (h->n_primal > 0) {
      launch_gather_cols(ncols, np, h->d_prank, nullptr, -1.0, h->d_cw1 + 2 * npm, 3 * npm,
                         h->d_xg, np, nullptr, st);
      launch_panels<T>(1, ncols, h->pj_phi, h->d_ptile, h->n_pphi, (const T*)h->d_pA, h->d_xg, np,
                       nullptr, h->d_vc, (int)h->n_bptot, nullptr, nullptr, nullptr, st);
    }
  }
  for (int j : cols) {
    const double* uc = h->d_uc + (int64_t)j * h->n_bptot;
    const double* q0 = h->n_primal > 0 ? h->d_cw1 + (int64_t)j * 3 * npm + 2 * npm : h->d_q0;
    double* dv = h->d_d + (int64_t)j * h->n_lambda;
    if (h->wide)
      launch_scatter(nb, nullptr, h->d_b2bp, h->d_vc + (int64_t)j * h->n_bptot, 1.0, h->d_wb,
                     nullptr, st);
    else
      phi_apply<T>(h, uc, -1.0, q0, h->d_wb, nullptr, st);
    launch_jump(h->n_lambda, h->d_posp, h->d_posm, h->d_wb, h->dt, dv, nullptr, nullptr, nullptr,
                st);
    if (corr)
      launch_jump_add(h->n_lambda, h->d_posp_r, h->d_posm_r, h->d_a + (int64_t)(k0 + j) * ldv,
                      h->dt, dv, st);
  }
}

// solve_post (lambda of column j from the PCG): p = S_Pi^-1 (h + sum N^T
// Phi^T x) with x = Bhat^T lambda; x_b = (u - v) - Phi N p; x_p = N p; and
// the right-hand side of the interior recovery, z = [y; -x_b; -x_p], into
// column j of d_zr.  The interior unknowns follow for the whole batch in
// recover_batch.  Writes column j's solution (kept order) at
// out + j * n_rtot.
template <class T>
static void solve_post(tcf_problem* h, int k0, const std::vector<int>& cols, double* out,
                       hipStream_t st) {
  const int64_t ldv = h->n_rtot;
  const int npm = std::max(h->n_primal, 1);
  const T* G = (const T*)h->d_G;
  if (cols.empty()) return;
  const int ncols = cols.back() + 1;
  const int nb = (int)h->n_btot, np = (int)h->n_ptot;
  if (h->n_primal > 0) launch_zero((int64_t)3 * npm * ncols, h->d_cw1, st);
  if (h->wide) {
    // G^T x of every column at once, x = dt Bhat^T lambda
    launch_zero(h->n_bptot * ncols, h->d_vc, st);
    if (h->n_lambda > 0) {
      launch_gather_cols(ncols, nb, h->d_brow, h->d_bsgn_d, h->dt, h->d_lam, h->n_lambda,
                         h->d_xg, nb, nullptr, st);
      launch_panels<T>(0, ncols, h->pj_gt, h->d_ptile, h->n_pgt, (const T*)h->d_pA, h->d_xg, nb,
                       nullptr, h->d_vc, (int)h->n_bptot, nullptr, nullptr, nullptr, st);
    }
  }
  for (int j : cols) {
    double* vc = h->d_vc + (int64_t)j * h->n_bptot;
    const double* lam = h->d_lam + (int64_t)j * h->n_lambda;
    if (!h->wide) {
      if (h->n_lambda == 0 || h->bp_gaps) launch_zero(std::max<int64_t>(h->n_bptot, 1), vc, st);
      if (h->n_lambda > 0)
        launch_dotcols<T>(h->dj_app_g, h->dp_app, h->nj_app, h->nt_app, h->max_nb, G, 1, lam,
                          h->d_brow, h->d_bsgn, h->dt, vc, nullptr, st);
    }
    if (h->n_primal > 0)
      launch_coarse_gather(h->n_primal, h->d_cptr, nullptr, nullptr, 0.0, h->d_cidx_bp, vc, 1.0,
                           h->d_h + (int64_t)j * npm, h->d_cw1 + (int64_t)j * 3 * npm, nullptr,
                           st);
  }
  coarse_solve_cols(h, ncols, st);
  if (h->wide) {
    // x_b = (u - v) - Phi_b N p of every column, in bp space
    launch_axpby(h->n_bptot * ncols, 1.0, h->d_uc, -1.0, h->d_vc, st);
    if (h->n_primal > 0) {
      launch_gather_cols(ncols, np, h->d_prank, nullptr, -1.0, h->d_cw1 + 2 * npm, 3 * npm,
                         h->d_xg, np, nullptr, st);
      launch_panels<T>(1, ncols, h->pj_phi, h->d_ptile, h->n_pphi, (const T*)h->d_pA, h->d_xg, np,
                       nullptr, h->d_vc, (int)h->n_bptot, nullptr, nullptr, nullptr, st);
    }
  }
  for (int j : cols) {
    const double* ygg = h->d_ygg + (int64_t)(k0 + j) * ldv;
    const double* uc = h->d_uc + (int64_t)j * h->n_bptot;
    const double* vc = h->d_vc + (int64_t)j * h->n_bptot;
    const double* q = h->d_cw1 + (int64_t)j * 3 * npm + 2 * npm;
    double* x_out = out + (int64_t)j * ldv;
    if (h->wide) {
      launch_scatter(nb, h->d_b2r, h->d_b2bp, vc, 1.0, x_out, nullptr, st);
    } else {
      launch_sub_gather(nb, h->d_b2bp, uc, h->d_b2bp, vc, h->d_tb, st);
      launch_scatter(nb, h->d_b2r, nullptr, h->d_tb, 1.0, x_out, nullptr, st);
      if (h->n_primal > 0 && h->nj_phi > 0)
        launch_axpyrows<T>(h->aj_ab, h->ap_phi, h->nj_phi, h->nt_phi, h->max_np, G, q,
                           h->d_prank, x_out, h->a_boff_ab, -1.0, x_out, 0, nullptr, st);
    }
    if (h->n_primal > 0)
      launch_scatter(np, h->d_p2r, h->d_prank, q, 1.0, x_out, nullptr, st);
    launch_build_z(ldv, h->d_isint, ygg, x_out, h->d_zr + (int64_t)j * ldv, st);
  }
}

// Interior recovery x_i = Q^T z of the nc columns of a batch (column j of
// z at d_zr + j ldv, of x at x_out + j ldv): the matrix-core form reads Q^T
// once for the batch; up to two columns use the row-stripe product.
template <class T>
static void recover_batch(tcf_problem* h, int nc, double* x_out, hipStream_t st) {
  const int64_t ldv = h->n_rtot;
  const T* Q = (const T*)h->d_Q;
  if (nc > 2) {
    timed(h, TCF_KG_RECOVER, st, [&] {
      launch_qapply_w<T>(h->dP, h->d_all, h->d_all_iprefix, h->np_tot, h->nt_all_i, nc, Q,
                         h->d_zr, x_out, ldv, st);
    });
    return;
  }
  for (int j = 0; j < nc; ++j)
    timed(h, TCF_KG_RECOVER, st, [&] {
      launch_axpyrows<T>(h->aj_ai, h->ap_ai, h->nj_ai, h->nt_ai, h->max_nr, Q,
                         h->d_zr + (int64_t)j * ldv, nullptr, nullptr, h->a_boff_ai, 1.0,
                         x_out + (int64_t)j * ldv, 1, nullptr, st);
    });
}

// Relative interface jump ||Bhat x|| (diagnostics with TCF_TRACE=1; syncs).
static double jump_norm(tcf_problem* h, const double* x, hipStream_t st) {
  if (h->n_lambda == 0) return 0.0;
  std::vector<double> jv(h->n_lambda);
  launch_zero(h->n_lambda, h->d_Fp, st);
  launch_jump_add(h->n_lambda, h->d_posp_r, h->d_posm_r, x, 1.0, h->d_Fp, st);
  (void)hipMemcpyAsync(jv.data(), h->d_Fp, sizeof(double) * h->n_lambda, hipMemcpyDeviceToHost,
                       st);
  (void)hipStreamSynchronize(st);
  double s2 = 0.0;
  for (double v : jv) s2 += v * v;
  return std::sqrt(s2);
}

// Squared global norm of a kept-ordered vector into h_nrm[slot] (syncs):
// assembled (sum of local copies) for residuals, first copy for fields.
static int asm_norm2(tcf_problem* h, const double* x, int first_copy, int slot, hipStream_t st) {
  launch_asm_norm2(h->n_kept_i, h->d_kptr, h->d_kidx, x, first_copy, h->d_nrm_part,
                   h->d_nrm + slot, st);
  HIPCHK(hipMemcpyAsync(h->h_nrm + slot, h->d_nrm + slot, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return TCF_OK;
}

// One implicit Euler step for excitations k0 .. k0 + nc - 1 (nc <= rb), one
// PCG column each.  FP64: one dual-primal solve.  FP32 operators:
// refinement a <- a + solve(f - W a) with the residual of the FP64 operator
// (matrix-free per patch, double-double row sums), assembled and split
// evenly over interface copies, the correction also closing the interface
// jump left in a.  At least one correction; an excitation stops when its
// estimated remaining error (last correction times the observed
// contraction, relative to the field) is <= ir_rtol, and then sits out
// (zero right-hand side) while the others continue.  The final assembled
// residual ||f - W a|| / ||f|| is reported in the stats (largest over the
// batch).  Per excitation: PCG iterations summed over its solves, sweeps.
// Projection start (Fischer's method for successive right-hand sides, over
// a sliding window): the newest kProjMax solutions of excitation k span X
// (F-orthonormal, F X kept beside), and the first solve of a step starts
// from the F-orthogonal projection of its solution onto that span,
// lambda0 = X X^T d (X^T F X = I and F lambda = d).
static void proj_start(tcf_problem* h, int k, int j, hipStream_t st) {
  const int nl = h->n_lambda, nb = h->proj_n[k];
  double* lam = h->d_lam + (int64_t)j * nl;
  launch_zero(nl, lam, st);
  if (nb == 0) return;
  const double* X = h->d_px + (int64_t)k * tcf_problem::kProjMax * nl;
  launch_rowdot(nl, nb, X, nl, h->d_d + (int64_t)j * nl, h->d_pc, nullptr, nullptr, 0, st);
  launch_multiaxpy(nl, nb, h->d_pc, 1.0, X, nullptr, nl, lam, nullptr, st);
}

// After the solve: lambda (column j) and F lambda = d - r (the PCG's own
// residual) enter the ring in place of the oldest pair, and the basis of the
// window is rebuilt newest first: each raw pair gets two classical
// Gram-Schmidt passes in the F inner product and is normalised; one that
// lies in the span of the newer ones to the solver's accuracy is stored as
// zero.  All on the stream, no host reads.
static void proj_update(tcf_problem* h, int k, int j, hipStream_t st) {
  const int nl = h->n_lambda, K = tcf_problem::kProjMax;
  const int64_t off = (int64_t)k * K * nl;
  double *H = h->d_ph + off, *FH = h->d_pfh + off, *X = h->d_px + off, *FX = h->d_pfx + off;
  double *v = h->d_pv, *Fv = h->d_pfv, *c = h->d_pc;
  const int slot = h->proj_head[k];
  launch_copy_sub(nl, h->d_lam + (int64_t)j * nl, h->d_d + (int64_t)j * nl,
                  h->d_r + (int64_t)j * nl, H + (int64_t)slot * nl, FH + (int64_t)slot * nl, st);
  h->proj_head[k] = (slot + 1) % K;
  const int cnt = std::min(h->proj_n[k] + 1, K);
  for (int i = 0; i < cnt; ++i) {
    const int src = ((slot - i) % K + K) % K;  // newest first
    launch_copy_sub(nl, H + (int64_t)src * nl, FH + (int64_t)src * nl, nullptr, v, Fv, st);
    // pass 1 (and lambda^T F lambda into c[K]), pass 2, then nu^2 into c[K+1]
    launch_rowdot(nl, i, FX, nl, v, c, v, Fv, K, st);
    launch_multiaxpy(nl, i, c, -1.0, X, FX, nl, v, Fv, st);
    if (i > 0) {
      launch_rowdot(nl, i, FX, nl, v, c, nullptr, nullptr, 0, st);
      launch_multiaxpy(nl, i, c, -1.0, X, FX, nl, v, Fv, st);
    }
    launch_rowdot(nl, 0, nullptr, 0, nullptr, c, v, Fv, K + 1, st);
    launch_store_dir(nl, c + K + 1, c + K, 1e-18, v, Fv, X + (int64_t)i * nl, FX + (int64_t)i * nl,
                     st);
  }
  h->proj_n[k] = cnt;
}

template <class T>
static int step_batch(tcf_problem* h, int k0, int nc, int l, hipStream_t st, int* iters,
                      int* sweeps, bool* conv) {
  const int64_t ldv = h->n_rtot;
  const int R = h->rb, nl = h->n_lambda;
  std::vector<int> it(R);
  std::vector<char> cv(R);
  std::vector<int> itv(R);
  std::unique_ptr<bool[]> cvb(new bool[R]);
  for (int j = 0; j < nc; ++j) {
    iters[j] = 0;
    sweeps[j] = 0;
    conv[j] = true;
  }
  auto zero_idle = [&](const std::vector<char>& active) {
    for (int j = 0; j < R; ++j)
      if (j >= nc || !active[j]) launch_zero(nl, h->d_d + (int64_t)j * nl, st);
  };
  auto collect = [&](const std::vector<char>& active) {
    for (int j = 0; j < nc; ++j)
      if (active[j]) {
        iters[j] += it[j];
        conv[j] = conv[j] && cv[j];
      }
  };
  auto run_pcg = [&]() -> int {
    RCCHK(pcg_solve<T>(h, st, itv.data(), cvb.get()));
    for (int j = 0; j < R; ++j) {
      it[j] = itv[j];
      cv[j] = cvb[j];
    }
    return TCF_OK;
  };
  std::vector<char> all(R, 0);
  for (int j = 0; j < nc; ++j) all[j] = 1;
  // first solve: the time-step right-hand side of every excitation
  h->cur_sweep = 0;
  condense_batch<T>(h, k0, nc, l, nullptr, st);
  std::vector<int> cols_all(nc);
  std::iota(cols_all.begin(), cols_all.end(), 0);
  solve_pre<T>(h, k0, cols_all, false, st);
  zero_idle(all);
  if (h->d_px) {
    for (int j = 0; j < R; ++j) {
      if (j < nc)
        proj_start(h, k0 + j, j, st);
      else
        launch_zero(nl, h->d_lam + (int64_t)j * nl, st);
    }
    h->warm_init = true;
  }
  if (h->d_lamh) {
    // lambda0 per column from the excitation's history (zero without one)
    for (int j = 0; j < R; ++j) {
      double* lam = h->d_lam + (int64_t)j * nl;
      const int k = k0 + j;
      const int nh = j < nc ? h->lamh_n[k] : 0;
      const double* h1 = h->d_lamh + ((int64_t)k * 2 + 0) * nl;
      const double* h2 = h->d_lamh + ((int64_t)k * 2 + 1) * nl;
      if (nh == 0)
        launch_zero(nl, lam, st);
      else if (nh == 1 || h->opt.pcg_warm == 1)
        launch_axpby(nl, 1.0, h1, 0.0, lam, st);
      else {
        launch_axpby(nl, 1.0, h2, 0.0, lam, st);
        launch_axpby(nl, 2.0, h1, -1.0, lam, st);  // 2 h1 - h2
      }
    }
    h->warm_init = true;
  }
  RCCHK(run_pcg());
  if (h->d_lamh) {
    for (int j = 0; j < nc; ++j) {
      const int k = k0 + j;
      double* h1 = h->d_lamh + ((int64_t)k * 2 + 0) * nl;
      double* h2 = h->d_lamh + ((int64_t)k * 2 + 1) * nl;
      HIPCHK(hipMemcpyAsync(h2, h1, sizeof(double) * nl, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(h1, h->d_lam + (int64_t)j * nl, sizeof(double) * nl,
                            hipMemcpyDeviceToDevice, st));
      h->lamh_n[k] = std::min(h->lamh_n[k] + 1, 2);
    }
  }
  if (h->d_px)
    for (int j = 0; j < nc; ++j) proj_update(h, k0 + j, j, st);
  solve_post<T>(h, k0, cols_all, h->d_a + (int64_t)k0 * ldv, st);
  recover_batch<T>(h, nc, h->d_a + (int64_t)k0 * ldv, st);
  collect(all);
  for (int j = 0; j < nc; ++j) sweeps[j] = 1;
  if (h->precision == TCF_FP64 && !h->fp64_ir) return TCF_OK;

  // refinement: f = M a^(l) + dt g jhat per excitation (local, FP64)
  std::vector<double> fn(nc), rel_prev(nc, 0.0), est(nc, 1.0), rn(nc, 0.0);
  for (int j = 0; j < nc; ++j) {
    const int k = k0 + j;
    double* a = h->d_a + (int64_t)k * ldv;
    double* fM = h->d_fM + (int64_t)k * ldv;
    double* floc = h->d_floc + (int64_t)j * ldv;
    const double gk = h->amp[(size_t)k * h->n_steps + l];
    // fM still holds M a^(l) from the first solve's condensation (conductor
    // patches) and zeros elsewhere
    (void)a;
    HIPCHK(hipMemcpyAsync(floc, fM, sizeof(double) * ldv, hipMemcpyDeviceToDevice, st));
    launch_axpby(ldv, h->dt * gk, h->d_jr + (int64_t)k * ldv, 1.0, floc, st);
    RCCHK(asm_norm2(h, floc, 0, 0, st));
    fn[j] = std::sqrt(h->h_nrm[0]);
  }
  std::vector<char> active(R, 0), settled(nc, 0);
  for (int sweep = 1;; ++sweep) {
    Range rg("refinement sweep");
    int n_active = 0;
    for (int j = 0; j < nc; ++j) {
      active[j] = 0;
      if (settled[j]) continue;
      const int k = k0 + j;
      double* a = h->d_a + (int64_t)k * ldv;
      double* res = h->d_res + (int64_t)j * ldv;
      launch_residual(h->dP, h->d_all, h->d_all_rprefix, h->np_tot, h->nt_all_r, h->d_rloc,
                      h->d_loc2r, h->d_tabs, h->dt, h->d_floc + (int64_t)j * ldv, a, res, st);
      RCCHK(asm_norm2(h, res, 0, 1, st));
      rn[j] = std::sqrt(h->h_nrm[1]);
      bool act = !(fn[j] == 0.0 || rn[j] == 0.0) && !(sweeps[j] >= 2 && est[j] <= h->opt.ir_rtol);
      if (act && sweeps[j] >= h->opt.ir_maxit) {
        conv[j] = false;
        act = false;
      }
      active[j] = act ? 1 : 0;
      settled[j] = act ? 0 : 1;
      n_active += act ? 1 : 0;
    }
    if (n_active == 0) break;
    // the correction sees the assembled residual split evenly over copies, so
    // its dual right-hand side is as small as the true residual and the PCG
    // tolerance also resolves the interface jump carried over from a
    h->cur_sweep = sweep;
    for (int j = 0; j < nc; ++j)
      if (active[j])
        launch_assemble_split(h->n_kept_i, h->d_kptr, h->d_kidx, h->d_res + (int64_t)j * ldv, st);
    // (columns of settled excitations are condensed too and left unused)
    condense_batch<T>(h, k0, nc, l, h->d_res, st);
    std::vector<int> cols_act;
    for (int j = 0; j < nc; ++j)
      if (active[j]) cols_act.push_back(j);
    solve_pre<T>(h, k0, cols_act, true, st);
    zero_idle(active);
    RCCHK(run_pcg());
    solve_post<T>(h, k0, cols_act, h->d_delta, st);
    recover_batch<T>(h, nc, h->d_delta, st);
    for (int j = 0; j < nc; ++j) {
      if (!active[j]) continue;
      const int k = k0 + j;
      double* a = h->d_a + (int64_t)k * ldv;
      double* delta = h->d_delta + (int64_t)j * ldv;
      launch_axpby(ldv, 1.0, delta, 1.0, a, st);
      RCCHK(asm_norm2(h, delta, 1, 2, st));
      RCCHK(asm_norm2(h, a, 1, 3, st));
      const double dn = std::sqrt(h->h_nrm[2]), an = std::sqrt(h->h_nrm[3]);
      // error left after this correction ~ its size times the contraction
      // of one inexact solve: the first correction's relative size
      // estimates that contraction, later ones use the observed ratio
      const double rel = an > 0 ? dn / an : 0.0;
      const double ratio = rel_prev[j] > 0 ? rel / rel_prev[j] : rel;
      est[j] = rel * std::min(1.0, ratio);
      rel_prev[j] = rel;
      ++sweeps[j];
      if (h->trace)
        std::fprintf(stderr,
                     "[tcf] step %d rhs %d sweep %d: |r|/|f| %.3e  |da|/|a| %.3e  |Ba|/|a| %.3e  "
                     "pcg %d%s\n",
                     l, k, sweeps[j] - 1, rn[j] / fn[j], dn / std::max(an, 1e-300),
                     jump_norm(h, a, st) / std::max(an, 1e-300), it[j],
                     cv[j] ? "" : " (not converged)");
    }
    collect(active);
  }
  double worst = 0.0;
  for (int j = 0; j < nc; ++j) worst = std::max(worst, fn[j] > 0 ? rn[j] / fn[j] : 0.0);
  h->last_ir_res = worst;
  return TCF_OK;
}

template <class T>
static int step_impl(tcf_problem* h, int nsteps, hipStream_t st) {
  int status = TCF_OK;
  std::vector<int> iters(h->rb), sweeps(h->rb);
  std::unique_ptr<bool[]> conv(new bool[h->rb]);
  for (int s = 0; s < nsteps; ++s) {
    Range rg("tcf step: one time step");
    const int l = h->steps_done;
    const double t0 = now_ms();
    int it_sum = 0, ir_sum = 0;
    bool all_conv = true;
    for (int k0 = 0; k0 < h->n_rhs; k0 += h->rb) {
      const int nc = std::min(h->rb, h->n_rhs - k0);
      RCCHK(step_batch<T>(h, k0, nc, l, st, iters.data(), sweeps.data(), conv.get()));
      for (int j = 0; j < nc; ++j) {
        it_sum += iters[j];
        ir_sum += sweeps[j];
        all_conv &= conv[j];
        h->last_iters = iters[j];
        h->last_ir = sweeps[j];
        h->max_iters = std::max(h->max_iters, iters[j]);
        h->total_iters += iters[j];
      }
    }
    HIPCHK(hipStreamSynchronize(st));
    if (h->prof_on) h->prof_flush(INT32_MAX);
    const double ms = now_ms() - t0;
    if (!all_conv) {
      ++h->nonconv;
      status = TCF_ENOCONV;
      h->err = "PCG or refinement reached its iteration limit at step " + std::to_string(l);
    }
    h->log_iters.push_back(it_sum);
    h->log_ir.push_back(ir_sum);
    h->log_ms.push_back(ms);
    h->step_ms_total += ms;
    h->steps_done++;
  }
  return status;
}

extern "C" {

int tcf_step(tcf_problem* h, int32_t nsteps, void* stream) {
  if (!h) return TCF_EINVAL;
  if (!h->is_setup) { h->err = "tcf_step before tcf_setup"; return TCF_ESTATE; }
  if (nsteps < 0) { h->err = "nsteps < 0"; return TCF_EINVAL; }
  nsteps = std::min(nsteps, h->n_steps - h->steps_done);
  if (nsteps <= 0) return TCF_OK;
  hipStream_t st = (hipStream_t)stream;
  h->mem_stream = st;
  try {
    return h->precision == TCF_FP64 ? step_impl<double>(h, nsteps, st)
                                    : step_impl<float>(h, nsteps, st);  // FP32 operators
  } catch (const std::bad_alloc&) {
    h->err = "out of host memory in step";
    return TCF_ENOMEM;
  }
}

int tcf_sync(tcf_problem* h, void* stream) {
  if (!h) return TCF_EINVAL;
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  HIPCHK(hipGetLastError());
  return TCF_OK;
}

int tcf_get_field(tcf_problem* h, int32_t k, double* out, size_t len, int32_t on_device,
                  void* stream) {
  if (!h || !out) return TCF_EINVAL;
  if (!h->is_setup) { h->err = "tcf_get_field before tcf_setup"; return TCF_ESTATE; }
  if (k < 0 || k >= h->n_rhs) { h->err = "excitation index out of range"; return TCF_EINVAL; }
  const int64_t nE = h->g.n_edges();
  if (len < (size_t)nE) { h->err = "field buffer too small"; return TCF_EINVAL; }
  hipStream_t st = (hipStream_t)stream;
  double* dst = on_device ? out : h->d_field;
  HIPCHK(hipMemsetAsync(dst, 0, sizeof(double) * nE, st));
  launch_to_global(h->n_rtot, h->d_rgid1, h->d_a + (int64_t)k * h->n_rtot, dst, st);
  HIPCHK(hipGetLastError());
  if (!on_device)
    HIPCHK(hipMemcpyAsync(out, h->d_field, sizeof(double) * nE, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return TCF_OK;
}

int tcf_get_state(tcf_problem* h, void* buf, size_t* bytes, void* stream) {
  if (!h || !bytes) return TCF_EINVAL;
  if (!h->is_setup) { h->err = "tcf_get_state before tcf_setup"; return TCF_ESTATE; }
  const size_t need = 16 + sizeof(double) * (size_t)h->n_rtot * h->n_rhs;
  if (!buf) { *bytes = need; return TCF_OK; }
  if (*bytes < need) { h->err = "state buffer too small"; return TCF_EINVAL; }
  int64_t hdr[2] = {h->steps_done, h->n_rtot * h->n_rhs};
  std::memcpy(buf, hdr, 16);
  HIPCHK(hipMemcpyAsync((char*)buf + 16, h->d_a, need - 16, hipMemcpyDeviceToHost,
                        (hipStream_t)stream));
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  *bytes = need;
  return TCF_OK;
}

int tcf_set_state(tcf_problem* h, const void* buf, size_t bytes, void* stream) {
  if (!h || !buf) return TCF_EINVAL;
  if (!h->is_setup) { h->err = "tcf_set_state before tcf_setup"; return TCF_ESTATE; }
  const size_t need = 16 + sizeof(double) * (size_t)h->n_rtot * h->n_rhs;
  int64_t hdr[2];
  if (bytes < need) { h->err = "state buffer too small"; return TCF_EINVAL; }
  std::memcpy(hdr, buf, 16);
  if (hdr[1] != h->n_rtot * h->n_rhs || hdr[0] < 0 || hdr[0] > h->n_steps) {
    h->err = "state does not match this problem";
    return TCF_EINVAL;
  }
  HIPCHK(hipMemcpyAsync(h->d_a, (const char*)buf + 16, need - 16, hipMemcpyHostToDevice,
                        (hipStream_t)stream));
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  h->steps_done = (int)hdr[0];
  std::fill(h->lamh_n.begin(), h->lamh_n.end(), 0);  // warm-start history no longer applies
  std::fill(h->proj_n.begin(), h->proj_n.end(), 0);
  std::fill(h->proj_head.begin(), h->proj_head.end(), 0);
  return TCF_OK;
}

}  // extern "C"

// ============================================================================
// Allocation-free stepping
// ============================================================================
// The PCG's per-solve scratch (tile accumulators and quadratic-form slots,
// reduction partials, per-column scalars and flags) can come from one
// file-scope device array instead of the handle's buffers.  Every solve
// initialises all of it before reading it (the accumulators are cleared by
// a fill kernel, the scalars by the first PCG kernel), so the contents left
// by an earlier call do not matter.  Each device holds its own copy of the
// array; its address is looked up once per device.
namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }
}  // namespace

extern "C" int tcf_step_noalloc(tcf_problem* h, int32_t nsteps, void* stream) {
  if (!h) return TCF_EINVAL;
  if (!h->is_setup) { h->err = "tcf_step_noalloc before tcf_setup"; return TCF_ESTATE; }
  if (nsteps < 0) { h->err = "nsteps < 0"; return TCF_EINVAL; }
  const size_t acc_b = align256(sizeof(double) * (size_t)h->n_acc);
  const size_t part_b = align256(sizeof(double) * (size_t)h->npart * 4 * h->rb);
  const size_t st_b = align256(sizeof(PcgScalars) * (size_t)(h->rb + 1));
  const size_t need = acc_b + part_b + st_b;
  if (need > kScratchBytes) {
    h->err = "tcf_step_noalloc: this problem needs " + std::to_string(need) +
             " bytes of PCG scratch, more than the " + std::to_string(kScratchBytes) +
             " the allocation-free step holds";
    return TCF_EINVAL;
  }
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) { h->err = "device index out of range"; return TCF_EINVAL; }
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        h->err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return TCF_EHIP;
      }
      g_scratch_ptr[dev] = p;
    }
    base = g_scratch_ptr[dev];
  }
  // the handle's scratch pointers point into the device array for this call
  // (graphs captured by tcf_step hold the handle's own buffers, so this call
  // issues stream launches only)
  double* acc0 = h->d_acc;
  double* part0 = h->d_part;
  PcgScalars* st0 = h->d_st;
  h->d_acc = (double*)base;
  h->d_part = (double*)((char*)base + acc_b);
  h->d_st = (PcgScalars*)((char*)base + acc_b + part_b);
  h->no_graph_call = true;
  const int rc = tcf_step(h, nsteps, stream);
  h->no_graph_call = false;
  h->d_acc = acc0;
  h->d_part = part0;
  h->d_st = st0;
  return rc;
}
