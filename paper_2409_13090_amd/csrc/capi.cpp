// C-ABI of the rlb library: symbolic handles (host), numeric handles (device
// plan + factor in caller storage), batched factorization, solves and FP64
// iterative refinement. Every step of the numeric path runs in the kernels of
// kernels.hip; this file only plans, uploads and enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <string>
#include <vector>

#include "../../include/rlb.h"
#include "device.h"
#include "symbolic.h"

using namespace rlb;

namespace {

thread_local std::string g_err;

// the merge key of a launch's variant: update variants that differ only in
// how K is staged are one class (a panel launch's variant is its width class)
int32_t merge_class(const Launch& l) {
  return l.kind == LAUNCH_UPDATE && (l.variant == UPD_TILE_WIN || l.variant == UPD_TILE_PACK)
             ? UPD_TILE
             : l.variant;
}

rlb_status fail(rlb_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_OK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(RLB_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

template <typename T>
rlb_status upload(T** dptr, const std::vector<T>& v) {
  *dptr = nullptr;
  if (v.empty()) return RLB_OK;
  HIP_OK(hipMalloc((void**)dptr, v.size() * sizeof(T)));
  HIP_OK(hipMemcpy(*dptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return RLB_OK;
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

// device copy of everything the factor and the solves need for one matrix
struct DevPlan {
  PanelTile* panels = nullptr;
  UpdTile* updates = nullptr;
  UpdSeg* segs = nullptr;
  DiagTile* dtiles = nullptr;
  DiagTile* ptiles = nullptr;
  int64_t* amap = nullptr;
  SolveTile* stiles = nullptr;
  int32_t* gl = nullptr;
  int64_t* perm = nullptr;
  int64_t* a_rowptr = nullptr;
  int32_t* a_col = nullptr;
  int64_t* a_src = nullptr;
  AsmCol* asmcols = nullptr;    // RL assembly
  int32_t* asm_rows = nullptr;
  PartReduce* reduces = nullptr;  // the parts of split target tiles
  // chained solve launches: signals each step counter waits for, and the
  // counters (step counters, one ticket counter per chained launch, the
  // timeout word), cleared at the start of every solve
  int32_t* sneed = nullptr;
  int32_t* chain = nullptr;
  int64_t nslots = 0, nchains = 0;
  ChainArgs chain_args(int32_t c) const {
    if (c < 0 || !chain) return ChainArgs{nullptr, nullptr, nullptr, nullptr};
    return ChainArgs{chain + nslots + c, chain, sneed, chain + nslots + nchains};
  }
  void release() {
    dfree(panels);
    dfree(updates);
    dfree(segs);
    dfree(dtiles);
    dfree(ptiles);
    dfree(amap);
    dfree(stiles);
    dfree(gl);
    dfree(perm);
    dfree(a_rowptr);
    dfree(a_col);
    dfree(a_src);
    dfree(asmcols);
    dfree(asm_rows);
    dfree(reduces);
    dfree(sneed);
    dfree(chain);
  }
};

// solve/refine data (no factor tiles)
rlb_status upload_solve(const Symbolic& s, int64_t base, DevPlan& d) {
  rlb_status st;
  std::vector<SolveTile> tiles = s.plan.stiles;
  for (SolveTile& t : tiles) t.off += base;
  if ((st = upload(&d.stiles, tiles))) return st;
  if ((st = upload(&d.gl, s.gl))) return st;
  if ((st = upload(&d.perm, s.perm))) return st;
  if ((st = upload(&d.a_rowptr, s.plan.a_rowptr))) return st;
  if ((st = upload(&d.a_col, s.plan.a_col))) return st;
  if ((st = upload(&d.a_src, s.plan.a_src))) return st;
  d.nslots = (int64_t)s.plan.sneed.size();
  d.nchains = s.plan.nchains;
  if (d.nchains > 0) {
    if ((st = upload(&d.sneed, s.plan.sneed))) return st;
    HIP_OK(hipMalloc((void**)&d.chain, (d.nslots + d.nchains + 1) * sizeof(int32_t)));
    // cleared once here as well: the timeout word is read by calls that
    // synchronize, also on a handle that has not solved yet
    HIP_OK(hipMemset(d.chain, 0, (d.nslots + d.nchains + 1) * sizeof(int32_t)));
  }
  return RLB_OK;
}

// scratch for the solves and the refinement of one matrix
struct SolveScratch {
  double* y = nullptr;  // n x SOLVE_MAXRHS: right-hand side in the factored order
  double* z = nullptr;  // forward solution
  double* x = nullptr;  // backward solution
  double* r = nullptr;   // residual B - A X (original order)
  double* d = nullptr;   // correction M^-1 r
  double* p = nullptr;   // PCG search direction
  double* rr = nullptr;  // PCG residual by recurrence
  double* q = nullptr;   // -A p
  double* dots = nullptr;  // SOLVE_MAXRHS column dot products
  unsigned long long* norms = nullptr;  // 3*SOLVE_MAXRHS + 1
  int64_t n = 0;
  rlb_status ensure(int64_t n_) {
    if (y && n >= n_) return RLB_OK;  // buffers sized for the largest n seen
    release();
    n = n_;
    size_t bytes = (size_t)std::max<int64_t>(n, 1) * SOLVE_MAXRHS * sizeof(double);
    HIP_OK(hipMalloc((void**)&y, bytes));
    HIP_OK(hipMalloc((void**)&z, bytes));
    HIP_OK(hipMalloc((void**)&x, bytes));
    HIP_OK(hipMalloc((void**)&r, bytes));
    HIP_OK(hipMalloc((void**)&d, bytes));
    HIP_OK(hipMalloc((void**)&p, bytes));
    HIP_OK(hipMalloc((void**)&rr, bytes));
    HIP_OK(hipMalloc((void**)&q, bytes));
    HIP_OK(hipMalloc((void**)&dots, SOLVE_MAXRHS * sizeof(double)));
    HIP_OK(hipMalloc((void**)&norms, (3 * SOLVE_MAXRHS + 1) * sizeof(unsigned long long)));
    return RLB_OK;
  }
  void release() {
    dfree(y);
    dfree(z);
    dfree(x);
    dfree(r);
    dfree(d);
    dfree(p);
    dfree(rr);
    dfree(q);
    dfree(dots);
    dfree(norms);
  }
};

// forward then backward supernodal solve of nrhs (<= SOLVE_MAXRHS) columns
// already gathered into sc.y (factored order, ld = n); the solution ends in sc.x
void enqueue_solve_levels(const Symbolic& s, const DevPlan& d, const double* L, SolveScratch& sc,
                          int nrhs, hipStream_t st) {
  // counters of the chained launches start at zero (a fill kernel, which a
  // captured graph replays correctly)
  if (d.chain) launch_zero_i32(d.chain, d.nslots + d.nchains + 1, st);
  for (const SolveLaunch& l : s.plan.slaunches) {
    const SolveTile* t = d.stiles + l.start;
    if (l.kind == SOLVE_FWD)
      launch_fwd_step(t, l.count, d.gl, L, sc.y, sc.z, nrhs, s.n, st, d.chain_args(l.chain));
    else if (l.kind == SOLVE_BELOW)
      launch_bwd_below(t, l.count, d.gl, L, sc.x, sc.z, nrhs, s.n, st);
    else
      launch_bwd_step(t, l.count, L, sc.z, sc.x, nrhs, s.n, st, d.chain_args(l.chain));
  }
}

// after a synchronization: a chained solve launch whose wait timed out (a
// plan error) makes the solution invalid
rlb_status chain_status(const DevPlan& d) {
  if (!d.chain) return RLB_OK;
  int32_t err = 0;
  HIP_OK(hipMemcpy(&err, d.chain + d.nslots + d.nchains, sizeof(err), hipMemcpyDeviceToHost));
  return err ? fail(RLB_ERR_HIP, "a chained solve launch timed out waiting for its inputs")
             : RLB_OK;
}

rlb_status solve_into(const Symbolic& s, const DevPlan& d, SolveScratch& sc, const double* L,
                      int64_t nrhs, const double* B, int64_t ldb, double* X, int64_t ldx,
                      hipStream_t st) {
  rlb_status e = sc.ensure(s.n);
  if (e) return e;
  for (int64_t c0 = 0; c0 < nrhs; c0 += SOLVE_MAXRHS) {
    int nr = (int)std::min<int64_t>(SOLVE_MAXRHS, nrhs - c0);
    launch_perm_in(d.perm, B + c0 * ldb, ldb, sc.y, s.n, s.n, nr, st);
    enqueue_solve_levels(s, d, L, sc, nr, st);
    launch_perm_out(d.perm, sc.x, s.n, X + c0 * ldx, ldx, s.n, nr, st);
  }
  HIP_OK(hipGetLastError());
  return RLB_OK;
}

// backward errors of nrhs (<= SOLVE_MAXRHS) columns; synchronizes
rlb_status backward_errors(const Symbolic& s, const DevPlan& d, SolveScratch& sc,
                           const double* values, int nrhs, const double* B, const double* X,
                           int64_t ld, hipStream_t st, double* out, double* anorm_cache) {
  rlb_status e = sc.ensure(s.n);
  if (e) return e;
  launch_zero_u64(sc.norms, 3 * SOLVE_MAXRHS + 1, st);
  launch_residual(s.n, d.a_rowptr, d.a_col, d.a_src, values, X, ld, B, ld, sc.r, s.n, nrhs, st);
  launch_absmax(sc.r, s.n, s.n, nrhs, sc.norms, st);
  launch_absmax(X, s.n, ld, nrhs, sc.norms + SOLVE_MAXRHS, st);
  bool need_a = !anorm_cache || *anorm_cache < 0;
  if (need_a) launch_anorm(s.n, d.a_rowptr, d.a_src, values, sc.norms + 3 * SOLVE_MAXRHS, st);
  unsigned long long h[3 * SOLVE_MAXRHS + 1];
  HIP_OK(hipMemcpyAsync(h, sc.norms, sizeof(h), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  if (rlb_status ce = chain_status(d)) return ce;
  double an;
  if (need_a) {
    std::memcpy(&an, &h[3 * SOLVE_MAXRHS], sizeof(double));
    if (anorm_cache) *anorm_cache = an;
  } else {
    an = *anorm_cache;
  }
  for (int k = 0; k < nrhs; ++k) {
    double rn, xn;
    std::memcpy(&rn, &h[k], sizeof(double));
    std::memcpy(&xn, &h[SOLVE_MAXRHS + k], sizeof(double));
    out[k] = (an > 0 && xn > 0) ? rn / (an * xn) : (rn == 0 ? 0.0 : INFINITY);
  }
  return RLB_OK;
}

}  // namespace

// ===========================================================================
struct rlb_symbolic_s {
  Symbolic s;
};

struct rlb_numeric_s {
  rlb_symbolic_s* sym = nullptr;
  int precision = 0;
  int device = 0;
  DevPlan d;
  int* status = nullptr;
  int* counters = nullptr;  // panel group counters (zero between launches), then the
  int ncounters = 0;         // count of patched pivots
  // reduced-precision forms: pivot thresholds, largest diagonal entry, panel maxima
  double* thr = nullptr;
  int64_t* dsrc = nullptr;
  unsigned long long* amax = nullptr;
  unsigned long long* smax = nullptr;
  float* Ls = nullptr;  // FP32-update form: FP32 copy of the finished factor entries
  double* L = nullptr;
  bool factored = false;        // a factorization was enqueued into L
  bool status_checked = false;  // its pivot status has been read since
  hipStream_t stream = nullptr;
  SolveScratch sc;
  // graph replay
  bool graph_mode = false;
  hipGraphExec_t gexec = nullptr;
  const void* g_vals = nullptr;
  void* g_L = nullptr;
  hipStream_t g_stream = nullptr;
  // per-launch timing
  bool profiling = false;
  std::vector<hipEvent_t> ev;
  double prof_update_ms = 0, prof_panel_ms = 0;
  int64_t prof_nupd = 0, prof_npan = 0;
  std::vector<double> prof_launch_ms;  // every launch of the plan, in order
  ~rlb_numeric_s() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    for (auto e : ev) (void)hipEventDestroy(e);
    d.release();
    sc.release();
    dfree(status);
    dfree(counters);
    dfree(thr);
    dfree(dsrc);
    dfree(amax);
    dfree(smax);
    dfree(Ls);
  }
};

struct rlb_batch_s {
  std::vector<rlb_symbolic_s*> syms;
  int precision = 0;
  std::vector<int64_t> base;     // factor storage offset of every matrix
  std::vector<int64_t> nnz_ptr;  // concatenated entry space
  int64_t l_elems = 0;
  std::vector<Launch> launches;
  std::vector<PanelTile> panels;
  std::vector<UpdTile> updates;
  std::vector<UpdSeg> segs;
  std::vector<PartReduce> reduces;  // the parts of split target tiles
  PartReduce* d_reduces = nullptr;
  std::vector<DiagTile> dtiles;  // by width class, as in a plan
  int64_t dt_ptr[4] = {0, 0, 0, 0};
  DiagTile* d_dtiles = nullptr;
  std::vector<DiagTile> ptiles;
  DiagTile* d_ptiles = nullptr;
  PanelTile* d_panels = nullptr;
  UpdTile* d_updates = nullptr;
  UpdSeg* d_segs = nullptr;
  int64_t* d_amap = nullptr;
  int64_t* d_nnz_ptr = nullptr;
  const double** d_vals = nullptr;
  int* status = nullptr;
  int* counters = nullptr;
  int ncounters = 0;
  std::vector<DevPlan> per;  // solve data of every matrix
  std::vector<int64_t> segbase;  // first contribution of every matrix
  int32_t schedule = -1;         // RLB_BATCH_SCHED_*
  // a merged launch with at least this many narrow work items (update tiles
  // of <= 16 columns, panel members of <= 16 columns) runs them one per
  // wavefront
  int64_t narrow_min = WAVE_SPLIT_MIN;
  SolveScratch sc;
  double* L = nullptr;
  bool factored = false;         // a factorization was enqueued into L
  std::vector<int64_t> h_info;   // per-matrix status, once read since that factorization
  hipStream_t stream = nullptr;
  bool graph_mode = false;
  hipGraphExec_t gexec = nullptr;
  std::vector<const double*> g_vals;
  void* g_L = nullptr;
  hipStream_t g_stream = nullptr;
  ~rlb_batch_s() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    dfree(d_panels);
    dfree(d_updates);
    dfree(d_reduces);
    dfree(d_segs);
    dfree(d_dtiles);
    dfree(d_ptiles);
    dfree(d_amap);
    dfree(d_nnz_ptr);
    if (d_vals) (void)hipFree((void*)d_vals);
    dfree(status);
    dfree(counters);
    for (auto& p : per) p.release();
    sc.release();
  }
};

extern "C" {

const char* rlb_last_error(void) { return g_err.c_str(); }

const char* rlb_status_string(rlb_status s) {
  switch (s) {
    case RLB_OK: return "ok";
    case RLB_ERR_ARG: return "bad argument";
    case RLB_ERR_PATTERN: return "malformed lower-triangle CSC pattern";
    case RLB_ERR_ALLOC: return "allocation failed";
    case RLB_ERR_WORKSPACE: return "workspace too small";
    case RLB_ERR_HIP: return "HIP runtime error";
    case RLB_ERR_STATE: return "handle not ready (no successful factorization)";
    case RLB_ERR_NOT_CONVERGED: return "refinement did not converge";
    case RLB_ERR_UNSUPPORTED: return "unsupported option";
    default: return s > 0 ? "matrix not positive definite" : "unknown status";
  }
}

rlb_status rlb_default_options(rlb_options* o) {
  if (!o) return fail(RLB_ERR_ARG, "null options");
  std::memset(o, 0, sizeof(*o));
  o->struct_size = (int32_t)sizeof(rlb_options);
  o->ordering = RLB_ORDER_GRID_ND;
  o->grid[3] = 1;
  o->merge_cap = 0.125;
  o->deterministic = 1;
  o->reorder = 1;
  o->maximal_blocks = 1;
  o->precision = RLB_PREC_FP64;
  return RLB_OK;
}

rlb_status rlb_analyze(int64_t n, const int64_t* colptr, const int64_t* rowidx,
                       const rlb_options* opt, rlb_symbolic* out) {
  if (!out) return fail(RLB_ERR_ARG, "null output handle");
  *out = nullptr;
  AnalyzeOptions ao;
  if (opt) {
    if (opt->struct_size != (int32_t)sizeof(rlb_options))
      return fail(RLB_ERR_ARG, "rlb_options.struct_size mismatch");
    if (opt->ordering < 0 || opt->ordering > 3) return fail(RLB_ERR_ARG, "bad ordering");
    if (!(opt->merge_cap >= 0) || opt->merge_cap > 10) return fail(RLB_ERR_ARG, "bad merge_cap");
    if (opt->precision < RLB_PREC_FP64 || opt->precision > RLB_PREC_FP16_UPDATES)
      return fail(RLB_ERR_ARG, "bad precision");
    ao.ordering = opt->ordering;
    ao.user_perm = opt->user_perm;
    for (int k = 0; k < 4; ++k) ao.grid[k] = opt->grid[k];
    ao.merge_cap = opt->merge_cap;
    ao.reorder = opt->reorder;
    ao.maximal_blocks = opt->maximal_blocks;
    ao.precision = opt->precision;
    if (opt->panel_spread < 0) return fail(RLB_ERR_ARG, "bad panel_spread");
    ao.panel_spread = opt->panel_spread ? opt->panel_spread : 512;
    if (opt->deterministic < 0 || opt->deterministic > 1)
      return fail(RLB_ERR_ARG, "bad deterministic (0 or 1)");
    ao.deterministic = opt->deterministic;
    if (opt->outer_block < 0 || opt->outer_block % 64)
      return fail(RLB_ERR_ARG, "bad outer_block (a multiple of 64)");
    ao.outer_block = opt->outer_block ? opt->outer_block : 256;
    ao.big_tile_min = opt->big_tile_min;
    if (opt->method < 0 || opt->method > 2) return fail(RLB_ERR_ARG, "bad method");
    ao.method = opt->method;
    if (opt->tile_order < 0 || opt->tile_order > 1) return fail(RLB_ERR_ARG, "bad tile_order");
    ao.tile_order = opt->tile_order;
    ao.tall_tile_min = opt->tall_tile_min;
    ao.split_chunks = opt->split_chunks;
    if (!(opt->hybrid_step_us == opt->hybrid_step_us)) return fail(RLB_ERR_ARG, "bad hybrid_step_us");
    ao.hybrid_step_us = opt->hybrid_step_us == 0 ? 30.0 : std::max(0.0, opt->hybrid_step_us);
  } else {
    ao.ordering = 0;
  }
  std::unique_ptr<rlb_symbolic_s> h;
  try {
    h.reset(new rlb_symbolic_s());
    std::string err;
    int st = analyze(n, colptr, rowidx, ao, h->s, err);
    if (st) return fail(st, err);
    st = build_plan(h->s, err);
    if (st) return fail(RLB_ERR_ARG, err);
  } catch (const std::bad_alloc&) {
    return fail(RLB_ERR_ALLOC, "host allocation failed in analyze");
  }
  *out = h.release();
  return RLB_OK;
}

rlb_status rlb_symbolic_info(rlb_symbolic sym, rlb_info* o) {
  if (!sym || !o) return fail(RLB_ERR_ARG, "null argument");
  const Symbolic& s = sym->s;
  std::memset(o, 0, sizeof(*o));
  o->n = s.n;
  o->nnz_a = s.nnz_a;
  o->n_supernodes = (int64_t)s.sn_ptr.size() - 1;
  o->n_fundamental = (int64_t)s.fund_ptr.size() - 1;
  o->n_levels = s.plan.nlevels;
  o->nnz_exact = s.nnz_exact;
  o->nnz_stored = s.nnz_stored;
  o->flops_exact = s.flops_exact;
  o->flops_padded = s.flops_padded;
  o->n_blocks = s.n_blocks;
  o->n_pairs = s.n_pairs;
  o->n_calls = s.n_calls;
  o->merge_added = s.merge_added;
  o->merge_base = s.merge_base;
  o->factor_bytes = s.plan.ws_elems * (int64_t)sizeof(double);
  o->u_bytes = s.plan.u_elems * (int64_t)sizeof(double);
  o->n_panel_tiles = (int64_t)s.plan.panels.size();
  o->n_update_tiles = (int64_t)s.plan.updates.size();
  o->n_merged_tiles = s.plan.n_merged_tiles;
  o->n_split_tiles = s.plan.n_split_tiles;
  o->n_launches = (int64_t)s.plan.launches.size();
  o->flops_tiles = s.plan.flops_tiles;
  o->flops_upd_alg = s.plan.flops_upd_alg;
  o->flops_panel = s.plan.flops_panel;
  o->flops_upd_launch = s.plan.flops_upd_launch;
  return RLB_OK;
}

rlb_status rlb_symbolic_array(rlb_symbolic sym, const char* which, int64_t* out, int64_t* len) {
  if (!sym || !which || !len) return fail(RLB_ERR_ARG, "null argument");
  const Symbolic& s = sym->s;
  std::vector<int64_t> tmp;
  auto put64 = [&](const std::vector<int64_t>& v) { tmp = v; };
  auto put32 = [&](const std::vector<int32_t>& v) { tmp.assign(v.begin(), v.end()); };
  std::string w(which);
  if (w == "perm") put64(s.perm);
  else if (w == "perm_nd") put64(s.perm_nd);
  else if (w == "perm_post") put64(s.perm_post);
  else if (w == "etree_post") put64(s.etree_post);
  else if (w == "etree") put64(s.etree);
  else if (w == "fund_ptr") put64(s.fund_ptr);
  else if (w == "sn_ptr") put64(s.sn_ptr);
  else if (w == "sn_parent") put64(s.sn_parent);
  else if (w == "gl_ptr") put64(s.gl_ptr);
  else if (w == "gl") put32(s.gl);
  else if (w == "rel_ptr") put64(s.rel_ptr);
  else if (w == "rel") put32(s.rel);
  else if (w == "blk_ptr") put64(s.blk_ptr);
  else if (w == "blk") put32(s.blk);
  else if (w == "rbp_ptr") put64(s.rbp_ptr);
  else if (w == "rbp_anc") put32(s.rbp_anc);
  else if (w == "rbv_ptr") put64(s.rbv_ptr);
  else if (w == "rbv") put32(s.rbv);
  else if (w == "colcount") put64(s.colcount);
  else if (w == "level") put32(s.plan.level);
  else if (w == "off") put64(s.plan.off);
  else if (w == "amap") put64(s.plan.amap);
  else if (w == "asm_rows") put32(s.plan.asm_rows);
  else if (w == "asm_cols") {  // src, dst, rp, len per update-matrix column (RL)
    for (const AsmCol& c : s.plan.asmcols) {
      int64_t v[4] = {c.src, c.dst, c.rp, c.len};
      tmp.insert(tmp.end(), v, v + 4);
    }
  }
  else if (w == "update_tiles") {  // c, ldc, m, n, flags, seg0, nseg per tile
    for (const UpdTile& t : s.plan.updates) {
      int64_t v[7] = {t.c, t.ldc, t.m, t.n, t.flags, t.seg0, t.nseg};
      tmp.insert(tmp.end(), v, v + 7);
    }
  } else if (w == "diag_tiles") {  // diag, ld, nb per diagonal tile
    for (const DiagTile& t : s.plan.dtiles) {
      int64_t v[3] = {t.diag, t.ld, t.nb};
      tmp.insert(tmp.end(), v, v + 3);
    }
  } else if (w == "solve_tiles") {  // off, ld, f, w, gl, c0, nb, r0, r1, flags, cslot per tile
    for (const SolveTile& t : s.plan.stiles) {
      int64_t v[11] = {t.off, t.ld, t.f, t.w, t.gl, t.c0, t.nb, t.r0, t.r1, t.flags, t.cslot};
      tmp.insert(tmp.end(), v, v + 11);
    }
  } else if (w == "solve_launches") {  // kind, level, first tile, tile count, chain per launch
    for (const SolveLaunch& l : s.plan.slaunches) {
      int64_t v[5] = {l.kind, l.level, l.start, l.count, l.chain};
      tmp.insert(tmp.end(), v, v + 5);
    }
  } else if (w == "solve_need") {  // signals each step counter of the chained launches waits for
    for (int32_t v : s.plan.sneed) tmp.push_back(v);
  } else if (w == "update_segs") {  // x, y, lds, k, ra, rb, ca, cb, src per contribution
    for (const UpdSeg& g : s.plan.segs) {
      int64_t v[9] = {g.x, g.y, g.lds, g.k, g.ra, g.rb, g.ca, g.cb, g.src};
      tmp.insert(tmp.end(), v, v + 9);
    }
  } else if (w == "part_reduces") {  // c, pbase, ldc, m, n, flags, nparts per split tile
    for (const PartReduce& r : s.plan.reduces) {
      int64_t v[7] = {r.c, r.pbase, r.ldc, r.m, r.n, r.flags, r.nparts};
      tmp.insert(tmp.end(), v, v + 7);
    }
  } else if (w == "panel_tiles") {  // diag, ld, nb, nrows, row0, col, slot, grp, gcnt, rw, nrt
    for (const PanelTile& t : s.plan.panels) {
      int64_t v[11] = {t.diag, t.ld, t.nb, t.nrows, t.row0, t.col, t.slot, t.grp, t.gcnt, t.rw,
                       t.nrt};
      tmp.insert(tmp.end(), v, v + 11);
    }
  } else if (w == "launches") {
    // kind, level, step, start, count, variant, pre, ustart, ucount, ncount,
    // alt_start, alt_count
    for (const Launch& l : s.plan.launches) {
      int64_t v[12] = {l.kind,    l.level,  l.step,   l.start,     l.count,     l.variant,
                       l.pre,     l.ustart, l.ucount, l.ncount, l.alt_start, l.alt_count};
      tmp.insert(tmp.end(), v, v + 12);
    }
  }
  else return fail(RLB_ERR_ARG, "unknown array " + w);
  *len = (int64_t)tmp.size();
  if (out && !tmp.empty()) std::memcpy(out, tmp.data(), tmp.size() * sizeof(int64_t));
  return RLB_OK;
}

void rlb_symbolic_free(rlb_symbolic sym) { delete sym; }

// unit roundoff of the update operands of each form: the pivot threshold factor
static double update_unit_roundoff(int precision) {
  switch (precision) {
    case RLB_PREC_FP32_UPDATES: return std::ldexp(1.0, -24);
    case RLB_PREC_BF16_UPDATES: return std::ldexp(1.0, -8);
    case RLB_PREC_FP16_UPDATES: return std::ldexp(1.0, -11);
    default: return 0.0;
  }
}

rlb_status rlb_numeric_create(rlb_symbolic sym, int32_t precision, rlb_numeric* out) {
  if (!sym || !out) return fail(RLB_ERR_ARG, "null argument");
  if (precision < RLB_PREC_FP64 || precision > RLB_PREC_FP16_UPDATES)
    return fail(RLB_ERR_ARG, "bad precision");
  if (sym->s.opt.method != 0 && precision != RLB_PREC_FP64)
    return fail(RLB_ERR_UNSUPPORTED, "the RL method is FP64 only");
  *out = nullptr;
  std::unique_ptr<rlb_numeric_s> h(new rlb_numeric_s());
  h->sym = sym;
  h->precision = precision;
  HIP_OK(hipGetDevice(&h->device));
  const Symbolic& s = sym->s;
  rlb_status st;
  if ((st = upload(&h->d.panels, s.plan.panels))) return st;
  if ((st = upload(&h->d.updates, s.plan.updates))) return st;
  if ((st = upload(&h->d.segs, s.plan.segs))) return st;
  if ((st = upload(&h->d.dtiles, s.plan.dtiles))) return st;
  if ((st = upload(&h->d.ptiles, s.plan.ptiles))) return st;
  if ((st = upload(&h->d.amap, s.plan.amap))) return st;
  if ((st = upload(&h->d.asmcols, s.plan.asmcols))) return st;
  if ((st = upload(&h->d.asm_rows, s.plan.asm_rows))) return st;
  if ((st = upload(&h->d.reduces, s.plan.reduces))) return st;
  if ((st = upload_solve(s, 0, h->d))) return st;
  HIP_OK(hipMalloc((void**)&h->status, sizeof(int)));
  h->ncounters = std::max<int32_t>(1, s.plan.max_groups);
  HIP_OK(hipMalloc((void**)&h->counters, sizeof(int) * (h->ncounters + 1)));
  HIP_OK(hipMemset(h->counters, 0, sizeof(int) * (h->ncounters + 1)));
  if (precision != RLB_PREC_FP64) {
    if ((st = upload(&h->dsrc, s.plan.diag_src))) return st;
    HIP_OK(hipMalloc((void**)&h->thr, sizeof(double) * std::max<int64_t>(1, s.n)));
    HIP_OK(hipMalloc((void**)&h->amax, sizeof(unsigned long long)));
    HIP_OK(hipMalloc((void**)&h->smax,
                     sizeof(unsigned long long) * std::max<int32_t>(1, s.plan.n_scale_slots)));
  }
  if (precision == RLB_PREC_FP32_UPDATES)
    HIP_OK(hipMalloc((void**)&h->Ls, sizeof(float) * std::max<int64_t>(1, s.plan.l_elems)));
  *out = h.release();
  return RLB_OK;
}

static void enqueue_factor(rlb_numeric_s* h, const double* values, double* L, hipStream_t st,
                           bool timed) {
  const Symbolic& s = h->sym->s;
  const Plan& p = s.plan;
  launch_init_status(h->status, 1, h->counters, h->ncounters + 1, st);
  launch_fill(L, p.l_elems, 0.0, st);
  launch_scatter_a(values, h->d.amap, s.nnz_a, L, st);
  const double u = update_unit_roundoff(h->precision);
  unsigned int* nfixed = reinterpret_cast<unsigned int*>(h->counters + h->ncounters);
  if (h->precision != RLB_PREC_FP64) {
    launch_zero_u64(h->amax, 1, st);
    if (h->precision >= RLB_PREC_BF16_UPDATES) launch_zero_u64(h->smax, p.n_scale_slots, st);
    launch_pivthr(values, h->dsrc, s.n, u, h->thr, h->amax, st);
  }
  const int pmode = h->precision == RLB_PREC_FP64 ? 0 : (h->precision == RLB_PREC_FP32_UPDATES ? 1 : 2);
  size_t ei = 0;
  for (const Launch& l : p.launches) {
    if (timed) (void)hipEventRecord(h->ev[ei++], st);
    hipStream_t ls = st;
    if (l.kind == LAUNCH_ASSEMBLE) {
      launch_assemble(h->d.asmcols + l.start, l.count, h->d.asm_rows, L, ls);
    } else if (l.kind == LAUNCH_REDUCE) {
      launch_part_reduce(h->d.reduces + l.start, l.count, L, ls);
    } else if (l.kind == LAUNCH_UPDATE) {
      if ((l.variant == UPD_BIG && h->precision >= RLB_PREC_BF16_UPDATES) ||
          (l.variant == UPD_TALL && h->precision != RLB_PREC_FP64))
        launch_update(h->d.updates + l.alt_start, h->d.segs, l.alt_count, L, h->precision,
                      h->smax, UPD_TILE, ls, 0, h->Ls);
      else
        launch_update(h->d.updates + l.start, h->d.segs, l.count, L, h->precision, h->smax,
                      l.variant, ls, l.nwave, h->Ls);
    } else {
      launch_panel(h->d.panels + l.start, l.count, L, h->status, h->counters, pmode, l.variant,
                   l.pre != 0, h->thr, h->amax, u, h->smax, nfixed, h->d.updates + l.ustart,
                   h->d.segs, l.ucount, ls, h->Ls);
      // the 16-bit forms run the fused update tiles as a launch of their own
      if (pmode == 2 && l.ucount)
        launch_update(h->d.updates + l.ustart, h->d.segs, l.ucount, L, h->precision, h->smax,
                      UPD_TILE, ls);
    }
    if (timed) (void)hipEventRecord(h->ev[ei++], st);
  }
  const int cls_nbb[3] = {1, 2, 4};
  for (int ci = 0; ci < 3; ++ci)
    launch_tile_inverse(h->d.dtiles + p.dt_ptr[ci], p.dt_ptr[ci + 1] - p.dt_ptr[ci], cls_nbb[ci],
                        L, st);
  launch_pair_inverse(h->d.ptiles, (int64_t)p.ptiles.size(), L, st);
}

rlb_status rlb_factor(rlb_numeric h, const double* values, void* workspace, size_t ws_bytes,
                      void* stream) {
  if (!h || (!values && h->sym->s.nnz_a) || (!workspace && h->sym->s.plan.ws_elems))
    return fail(RLB_ERR_ARG, "null argument");
  const Symbolic& s = h->sym->s;
  if (ws_bytes < (size_t)s.plan.ws_elems * sizeof(double))
    return fail(RLB_ERR_WORKSPACE, "workspace smaller than factor_bytes");
  if (((uintptr_t)workspace & 7) != 0) return fail(RLB_ERR_ARG, "workspace not 8-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  h->L = (double*)workspace;
  h->stream = st;
  h->factored = false;
  h->status_checked = false;
  if (h->profiling) {
    size_t need = 2 * s.plan.launches.size();
    while (h->ev.size() < need) {
      hipEvent_t e;
      HIP_OK(hipEventCreate(&e));
      h->ev.push_back(e);
    }
    enqueue_factor(h, values, h->L, st, true);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(st));
    h->prof_update_ms = h->prof_panel_ms = 0;
    h->prof_nupd = h->prof_npan = 0;
    h->prof_launch_ms.clear();
    size_t ei = 0;
    for (const Launch& l : s.plan.launches) {
      float ms = 0;
      HIP_OK(hipEventElapsedTime(&ms, h->ev[ei], h->ev[ei + 1]));
      h->prof_launch_ms.push_back(ms);
      ei += 2;
      if (l.kind != LAUNCH_PANEL) {  // update and (RL) assembly launches
        h->prof_update_ms += ms;
        h->prof_nupd++;
      } else {
        h->prof_panel_ms += ms;
        h->prof_npan++;
      }
    }
  } else if (h->graph_mode) {
    if (!h->gexec || h->g_vals != values || h->g_L != workspace || h->g_stream != st) {
      if (h->gexec) {
        (void)hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
      }
      hipStream_t cs;
      HIP_OK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      hipGraph_t g;
      HIP_OK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      enqueue_factor(h, values, h->L, cs, false);
      hipError_t ce = hipStreamEndCapture(cs, &g);
      (void)hipStreamDestroy(cs);
      if (ce != hipSuccess) return fail(RLB_ERR_HIP, "graph capture failed");
      hipError_t ie = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) return fail(RLB_ERR_HIP, "graph instantiate failed");
      h->g_vals = values;
      h->g_L = workspace;
      h->g_stream = st;
    }
    HIP_OK(hipGraphLaunch(h->gexec, st));
  } else {
    enqueue_factor(h, values, h->L, st, false);
  }
  HIP_OK(hipGetLastError());
  h->factored = true;
  return RLB_OK;
}

rlb_status rlb_factor_status(rlb_numeric h, int64_t* info) {
  if (!h || !info) return fail(RLB_ERR_ARG, "null argument");
  if (!h->L) return fail(RLB_ERR_STATE, "no factorization enqueued");
  int v = 0;
  HIP_OK(hipMemcpyAsync(&v, h->status, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIP_OK(hipStreamSynchronize(h->stream));
  *info = (v == 0x7fffffff) ? 0 : v;
  h->status_checked = true;
  if (*info) h->factored = false;
  return (rlb_status)*info;
}

// rlb_solve and rlb_refine need a successful factor: read the pivot status of
// the last factorization once (synchronizing its stream) if the caller has
// not done so through rlb_factor_status
static rlb_status require_factor(rlb_numeric h) {
  if (!h->factored) return fail(RLB_ERR_STATE, "no successful factorization");
  if (!h->status_checked) {
    int64_t info = 0;
    rlb_status st = rlb_factor_status(h, &info);
    if (st < 0) return st;
    if (info) return fail(RLB_ERR_STATE, "the last factorization failed (matrix not positive definite)");
  }
  return RLB_OK;
}

rlb_status rlb_factor_pivots_patched(rlb_numeric h, int64_t* count) {
  if (!h || !count) return fail(RLB_ERR_ARG, "null argument");
  if (!h->L) return fail(RLB_ERR_STATE, "no factorization enqueued");
  unsigned int v = 0;
  HIP_OK(hipMemcpyAsync(&v, h->counters + h->ncounters, sizeof(v), hipMemcpyDeviceToHost,
                        h->stream));
  HIP_OK(hipStreamSynchronize(h->stream));
  *count = v;
  return RLB_OK;
}

rlb_status rlb_solve(rlb_numeric h, int64_t nrhs, double* B, int64_t ldb, void* stream) {
  if (!h || nrhs < 0) return fail(RLB_ERR_ARG, "bad argument");
  const Symbolic& s = h->sym->s;
  if (nrhs > 0 && s.n > 0 && !B) return fail(RLB_ERR_ARG, "null B");
  if (ldb < s.n) return fail(RLB_ERR_ARG, "ldb < n");
  rlb_status e = require_factor(h);
  if (e) return e;
  if (nrhs == 0 || s.n == 0) return RLB_OK;
  return solve_into(s, h->d, h->sc, h->L, nrhs, B, ldb, B, ldb, (hipStream_t)stream);
}

rlb_status rlb_solve_noalloc(rlb_numeric h, int64_t nrhs, double* B, int64_t ldb, void* stream) {
  if (!h || nrhs < 0 || nrhs > SOLVE_MAXRHS)
    return fail(RLB_ERR_ARG, "bad argument (0 <= nrhs <= 16)");
  const Symbolic& s = h->sym->s;
  if (nrhs > 0 && s.n > 0 && !B) return fail(RLB_ERR_ARG, "null B");
  if (ldb < s.n) return fail(RLB_ERR_ARG, "ldb < n");
  if (s.n * nrhs > NOALLOC_SOLVE_ELEMS)
    return fail(RLB_ERR_ARG, "n * nrhs exceeds the allocation-free solve's capacity (2^21)");
  rlb_status e = require_factor(h);
  if (e) return e;
  if (nrhs == 0 || s.n == 0) return RLB_OK;
  int dev = -1;
  HIP_OK(hipGetDevice(&dev));
  if (dev != h->device) return fail(RLB_ERR_ARG, "the handle's device is not the current device");
  double* base = nullptr;
  HIP_OK(noalloc_solve_scratch(&base));
  // the three work vectors, ld = n, views into the device's scratch (not owned)
  SolveScratch v;
  v.y = base;
  v.z = base + NOALLOC_SOLVE_ELEMS;
  v.x = base + 2 * NOALLOC_SOLVE_ELEMS;
  hipStream_t st = (hipStream_t)stream;
  const int nr = (int)nrhs;
  launch_perm_in(h->d.perm, B, ldb, v.y, s.n, s.n, nr, st);
  enqueue_solve_levels(s, h->d, h->L, v, nr, st);
  launch_perm_out(h->d.perm, v.x, s.n, B, ldb, s.n, nr, st);
  HIP_OK(hipGetLastError());
  return RLB_OK;
}

rlb_status rlb_backward_error(rlb_numeric h, const double* values, int64_t nrhs, const double* B,
                              const double* X, int64_t ld, void* stream, double* out) {
  if (!h || nrhs < 0 || (nrhs > 0 && !out)) return fail(RLB_ERR_ARG, "bad argument");
  const Symbolic& s = h->sym->s;
  // (null buffers are accepted where they would hold no element)
  if ((s.nnz_a > 0 && !values) || (nrhs > 0 && s.n > 0 && (!B || !X)))
    return fail(RLB_ERR_ARG, "null values, B or X");
  if (ld < s.n) return fail(RLB_ERR_ARG, "ld < n");
  // ||A||_inf is recomputed from `values` on every call (the caller may have
  // changed them in place since the last one)
  double anorm = -1.0;
  for (int64_t c0 = 0; c0 < nrhs; c0 += SOLVE_MAXRHS) {
    int nr = (int)std::min<int64_t>(SOLVE_MAXRHS, nrhs - c0);
    rlb_status e = backward_errors(s, h->d, h->sc, values, nr, B + c0 * ld, X + c0 * ld, ld,
                                   (hipStream_t)stream, out + c0, &anorm);
    if (e) return e;
  }
  return RLB_OK;
}

rlb_status rlb_refine(rlb_numeric h, const double* values, int64_t nrhs, const double* B,
                      double* X, int64_t ld, double tol, int32_t max_iter, void* stream,
                      rlb_refine_report* rep) {
  if (!h || nrhs < 1 || nrhs > SOLVE_MAXRHS || max_iter < 0)
    return fail(RLB_ERR_ARG, "bad argument (1 <= nrhs <= 16)");
  const Symbolic& s = h->sym->s;
  if ((s.nnz_a > 0 && !values) || (s.n > 0 && (!B || !X)))
    return fail(RLB_ERR_ARG, "null values, B or X");
  if (ld < s.n) return fail(RLB_ERR_ARG, "ld < n");
  rlb_status e = require_factor(h);
  if (e) return e;
  hipStream_t st = (hipStream_t)stream;
  const int nr = (int)nrhs;
  const int64_t n = s.n;
  SolveScratch& sc = h->sc;
  rlb_refine_report r;
  std::memset(&r, 0, sizeof(r));
  r.pcg_from = -1;
  e = solve_into(s, h->d, sc, h->L, nrhs, B, ld, X, ld, st);
  if (e) return e;
  double anorm = -1.0;  // ||A||_inf of `values`, formed once per call
  // column scalars: r.z, p.(-Ap) and |d| of the last correction
  auto dots = [&](const double* x, const double* y, double* out) -> rlb_status {
    launch_zero_u64(reinterpret_cast<unsigned long long*>(sc.dots), SOLVE_MAXRHS, st);
    launch_dot_cols(x, n, y, n, n, nr, sc.dots, st);
    HIP_OK(hipMemcpyAsync(out, sc.dots, sizeof(double) * nr, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    return RLB_OK;
  };
  auto solve_r = [&](const double* rv) {  // d = M^-1 rv with M = L L^T
    launch_perm_in(h->d.perm, rv, n, sc.y, n, n, nr, st);
    enqueue_solve_levels(s, h->d, h->L, sc, nr, st);
    launch_perm_out(h->d.perm, sc.x, n, sc.d, n, n, nr, st);
  };
  double be[SOLVE_MAXRHS], rz[SOLVE_MAXRHS] = {0}, dd[SOLVE_MAXRHS], prev_dn = -1.0;
  int strikes = 0, it = 0, since_best = 0;
  double best_pcg = INFINITY;
  bool pcg = false;
  ColCoef one, zero;
  for (int k = 0; k < SOLVE_MAXRHS; ++k) {
    one.v[k] = 1.0;
    zero.v[k] = 0.0;
  }
  for (;;) {
    e = backward_errors(s, h->d, sc, values, nr, B, X, ld, st, be, &anorm);
    if (e) return e;
    double worst = 0;
    for (int k = 0; k < nr; ++k) worst = std::max(worst, be[k]);
    if (it < 64) r.history[it] = worst;
    if (worst <= tol || it >= max_iter) {
      r.converged = worst <= tol;
      break;
    }
    if (pcg) {
      if (worst <= 0.5 * best_pcg) {
        best_pcg = worst;
        since_best = 0;
      } else {
        ++since_best;
      }
    }
    if (!pcg) {
      solve_r(sc.r);  // sc.d = M^-1 (B - A X)
      // classic refinement: X += d; switch to PCG after the correction fails
      // to halve twice
      if ((e = dots(sc.d, sc.d, dd))) return e;
      double dn = 0;
      for (int k = 0; k < nr; ++k) dn = std::max(dn, std::sqrt(dd[k]));
      if (prev_dn >= 0 && dn > 0.5 * prev_dn) ++strikes;
      prev_dn = dn;
      if (strikes < 2) {
        launch_axpy(X, ld, sc.d, n, n, nr, st);
        HIP_OK(hipGetLastError());
        ++it;
        continue;
      }
      // PCG from the current iterate: rr = B - A X, z = M^-1 rr, p = z
      pcg = true;
      r.pcg_from = it;
      launch_axpby_cols(sc.rr, n, sc.r, n, n, nr, one, zero, st);
      if ((e = dots(sc.rr, sc.d, rz))) return e;
      launch_axpby_cols(sc.p, n, sc.d, n, n, nr, one, zero, st);
    } else if (since_best >= 8) {
      // restart from the true residual when the backward error has not halved
      // in 8 steps (the recurrence residual drifts from B - A X)
      since_best = 0;
      best_pcg = worst;
      launch_axpby_cols(sc.rr, n, sc.r, n, n, nr, one, zero, st);
      solve_r(sc.rr);
      if ((e = dots(sc.rr, sc.d, rz))) return e;
      launch_axpby_cols(sc.p, n, sc.d, n, n, nr, one, zero, st);
    } else {
      // z = M^-1 rr; beta = (rr.z) / (rr.z)_old; p = z + beta p
      solve_r(sc.rr);
      double rzn[SOLVE_MAXRHS];
      if ((e = dots(sc.rr, sc.d, rzn))) return e;
      ColCoef beta;
      for (int k = 0; k < SOLVE_MAXRHS; ++k) {
        beta.v[k] = (k < nr && rz[k] != 0.0) ? rzn[k] / rz[k] : 0.0;
        if (k < nr) rz[k] = rzn[k];
      }
      launch_axpby_cols(sc.p, n, sc.d, n, n, nr, one, beta, st);
    }
    // q = -A p; alpha = (rr.z) / (p.A p); X += alpha p; rr -= alpha A p
    launch_residual(n, h->d.a_rowptr, h->d.a_col, h->d.a_src, values, sc.p, n, nullptr, 0, sc.q,
                    n, nr, st);
    double pq[SOLVE_MAXRHS];
    if ((e = dots(sc.p, sc.q, pq))) return e;
    ColCoef alpha;
    for (int k = 0; k < SOLVE_MAXRHS; ++k)
      alpha.v[k] = (k < nr && pq[k] != 0.0) ? rz[k] / -pq[k] : 0.0;
    launch_axpby_cols(X, ld, sc.p, n, n, nr, alpha, one, st);
    launch_axpby_cols(sc.rr, n, sc.q, n, n, nr, alpha, one, st);
    HIP_OK(hipGetLastError());
    ++it;
  }
  r.iterations = it;
  for (int k = 0; k < nr; ++k) r.backward_error[k] = be[k];
  if (rep) *rep = r;
  return r.converged ? RLB_OK : fail(RLB_ERR_NOT_CONVERGED, "refinement did not reach tol");
}

rlb_status rlb_factor_export(rlb_numeric h, int64_t* colptr, int64_t* rowidx, double* vals) {
  if (!h || !colptr || !rowidx || !vals) return fail(RLB_ERR_ARG, "null argument");
  if (!h->L) return fail(RLB_ERR_STATE, "no factorization");
  const Symbolic& s = h->sym->s;
  std::vector<double> hl(s.plan.l_elems);
  HIP_OK(hipStreamSynchronize(h->stream));
  if (!hl.empty())
    HIP_OK(hipMemcpy(hl.data(), h->L, hl.size() * sizeof(double), hipMemcpyDeviceToHost));
  int64_t S = (int64_t)s.sn_ptr.size() - 1, q = 0;
  colptr[0] = 0;
  for (int64_t J = 0; J < S; ++J) {
    int64_t f = s.sn_ptr[J], w = s.sn_ptr[J + 1] - f, m = s.gl_ptr[J + 1] - s.gl_ptr[J];
    const int32_t* g = s.gl.data() + s.gl_ptr[J];
    for (int64_t c = 0; c < w; ++c) {
      for (int64_t r = c; r < m; ++r) {
        rowidx[q] = g[r];
        vals[q] = hl[s.plan.off[J] + c * m + r];
        ++q;
      }
      colptr[f + c + 1] = q;
    }
  }
  return RLB_OK;
}

rlb_status rlb_last_profile_launches(rlb_numeric h, double* ms, int64_t* count) {
  if (!h || !count) return fail(RLB_ERR_ARG, "null argument");
  const int64_t n = (int64_t)h->prof_launch_ms.size();
  if (ms)
    for (int64_t i = 0; i < std::min(n, *count); ++i) ms[i] = h->prof_launch_ms[i];
  *count = n;
  return RLB_OK;
}

void rlb_numeric_free(rlb_numeric h) { delete h; }

rlb_status rlb_set_graph_mode(rlb_numeric h, int32_t on) {
  if (!h) return fail(RLB_ERR_ARG, "null handle");
  h->graph_mode = on != 0;
  return RLB_OK;
}

rlb_status rlb_set_profiling(rlb_numeric h, int32_t on) {
  if (!h) return fail(RLB_ERR_ARG, "null handle");
  h->profiling = on != 0;
  return RLB_OK;
}

rlb_status rlb_last_profile(rlb_numeric h, double* update_ms, double* panel_ms, int64_t* n_update,
                            int64_t* n_panel) {
  if (!h) return fail(RLB_ERR_ARG, "null handle");
  if (update_ms) *update_ms = h->prof_update_ms;
  if (panel_ms) *panel_ms = h->prof_panel_ms;
  if (n_update) *n_update = h->prof_nupd;
  if (n_panel) *n_panel = h->prof_npan;
  return RLB_OK;
}

// ---------------------------------------------------------------------------
// batched form

// Merged launch lists of a batch: for each (shifted level, step, kind) the
// tiles of every matrix, in matrix order. The level of matrix i is shifted
// by 0 (leaves aligned), by (max levels - its levels) (roots aligned) or by
// half of that (centered); each matrix keeps its own launch order, and
// matrices are independent, so every schedule computes the same factors.
static rlb_status batch_schedule(rlb_batch_s* b, int32_t schedule) {
  const int32_t count = (int32_t)b->syms.size();
  const auto& syms = b->syms;
  int32_t maxlev = 0;
  for (int32_t i = 0; i < count; ++i) maxlev = std::max(maxlev, syms[i]->s.plan.nlevels);
  std::vector<int32_t> shift(count, 0);
  for (int32_t i = 0; i < count; ++i) {
    int32_t gap = maxlev - syms[i]->s.plan.nlevels;
    shift[i] = schedule == RLB_BATCH_SCHED_ROOTS ? gap
               : schedule == RLB_BATCH_SCHED_CENTERED ? gap / 2 : 0;
  }
  const std::vector<int64_t>& segbase = b->segbase;
  // every matrix's launches in the unfused form: a panel launch that applies
  // the previous block's update itself (and runs the rest of that step's
  // update beside its workgroups) becomes that step's update launch followed
  // by a plain panel launch -- one merged launch then holds the work of many
  // matrices, more than one fused launch runs beside its panels. When every
  // matrix was analysed deterministic the fused launches are kept, so that
  // each matrix's tiles run the very arithmetic of its own factorization.
  bool keep_fused = true;
  for (int32_t i = 0; i < count; ++i) keep_fused = keep_fused && syms[i]->s.opt.deterministic;
  std::vector<std::vector<Launch>> lists(count);
  for (int32_t i = 0; i < count; ++i) {
    const std::vector<Launch>& L = syms[i]->s.plan.launches;
    for (size_t j = 0; j < L.size(); ++j) {
      Launch l = L[j];
      if (l.kind == LAUNCH_PANEL && l.pre && !keep_fused) {
        const bool first = j == 0 || L[j - 1].kind != LAUNCH_PANEL || L[j - 1].level != l.level ||
                           L[j - 1].step != l.step;
        for (size_t q = j; first && q < L.size() && L[q].kind == LAUNCH_PANEL &&
                           L[q].level == l.level && L[q].step == l.step;
             ++q)
          if (L[q].ucount + L[q].ncount > 0)
            lists[i].push_back(Launch{LAUNCH_UPDATE, l.level, l.step - 1, UPD_SHORT, L[q].ustart,
                                      L[q].ucount + L[q].ncount, 0, 0, 0, 0, 0});
        l.pre = 0;
        l.ustart = l.ucount = l.ncount = 0;
      }
      lists[i].push_back(l);
    }
  }
  b->launches.clear();
  b->panels.clear();
  b->updates.clear();
  b->reduces.clear();
  b->ncounters = 0;
  // merge: for each (level, step, kind) the tiles of every matrix, in matrix order
  std::vector<size_t> cur(count, 0);
  for (;;) {
    // the smallest (level, step, kind) among the matrices' next launches
    bool any = false;
    int32_t bl = 0, bs = 0, bk = 0, bv = 0, bp = 0;
    for (int32_t i = 0; i < count; ++i) {
      const auto& L = lists[i];
      if (cur[i] >= L.size()) continue;
      const Launch& l = L[cur[i]];
      const int32_t lv = l.level + shift[i];
      // the dense, windowed and packed staging of one step are one class,
      // the variant of the merged launch is chosen from its merged tiles
      // (deterministic: each matrix's tiles keep the kernel of its own plan)
      const int32_t vv = keep_fused ? l.variant : merge_class(l);
      const int32_t pp = l.kind == LAUNCH_PANEL ? l.pre : 0;
      if (!any ||
          std::make_tuple(lv, l.step, l.kind, vv, pp) < std::make_tuple(bl, bs, bk, bv, bp)) {
        bl = lv;
        bs = l.step;
        bk = l.kind;
        bv = vv;
        bp = pp;
        any = true;
      }
    }
    if (!any) break;
    Launch m{bk, bl, bs, bv, 0, 0, bp, 0, 0, 0, 0};
    int32_t gbase = 0;  // group counters are numbered across the merged matrices
    std::vector<UpdTile> narrow;  // update launch: the narrow tiles, placed last
    m.start = bk == LAUNCH_REDUCE   ? (int64_t)b->reduces.size()
              : bk != LAUNCH_UPDATE ? (int64_t)b->panels.size()
                                    : (int64_t)b->updates.size();
    m.ustart = (int64_t)b->updates.size();
    for (int32_t i = 0; i < count; ++i) {
      const Plan& p = syms[i]->s.plan;
      if (cur[i] >= lists[i].size()) continue;
      const Launch& l = lists[i][cur[i]];
      if (l.level + shift[i] != bl || l.step != bs || l.kind != bk ||
          (keep_fused ? l.variant : merge_class(l)) != bv)
        continue;
      if (bk == LAUNCH_PANEL && l.pre != bp) continue;
      if (bk == LAUNCH_REDUCE) {
        for (int64_t t = 0; t < l.count; ++t) {
          PartReduce r = p.reduces[l.start + t];
          r.c += b->base[i];
          r.pbase += b->base[i];
          b->reduces.push_back(r);
        }
      } else if (bk != LAUNCH_UPDATE) {
        int32_t g_hi = 0;
        for (int64_t t = 0; t < l.count; ++t) {
          PanelTile pt = p.panels[l.start + t];
          pt.diag += b->base[i];
          pt.slot = i;
          g_hi = std::max(g_hi, pt.grp + 1);
          pt.grp += gbase;
          b->panels.push_back(pt);
        }
        gbase += g_hi;
        // the fused update tiles of the previous step ride along
        for (int64_t t = 0; t < l.ucount; ++t) {
          UpdTile ut = p.updates[l.ustart + t];
          ut.c += b->base[i];
          ut.seg0 += (int32_t)segbase[i];
          b->updates.push_back(ut);
        }
        m.ucount += l.ucount;
      } else {
        // the regular tiles now, the narrow ones after every matrix's
        for (int64_t t = 0; t < l.count; ++t) {
          UpdTile ut = p.updates[l.start + t];
          ut.c += b->base[i];
          ut.seg0 += (int32_t)segbase[i];
          if (ut.n <= NARROW_COLS && bv != UPD_BIG && bv != UPD_TALL)
            narrow.push_back(ut);
          else
            b->updates.push_back(ut);
        }
      }
      cur[i]++;
    }
    if (bk == LAUNCH_UPDATE) {
      if (bv == UPD_TILE && !keep_fused)
        m.variant = tile_variant(b->updates.data() + m.start,
                                 (int64_t)b->updates.size() - m.start, b->segs.data());
      b->updates.insert(b->updates.end(), narrow.begin(), narrow.end());
      m.nwave = (int32_t)narrow.size();
    }
    m.count = (bk == LAUNCH_REDUCE   ? (int64_t)b->reduces.size()
               : bk != LAUNCH_UPDATE ? (int64_t)b->panels.size()
                                     : (int64_t)b->updates.size()) -
              m.start;
    b->launches.push_back(m);
    b->ncounters = std::max(b->ncounters, (int)gbase);
  }
  dfree(b->d_panels);
  dfree(b->d_updates);
  dfree(b->d_reduces);
  dfree(b->counters);
  rlb_status st;
  if ((st = upload(&b->d_panels, b->panels))) return st;
  if ((st = upload(&b->d_updates, b->updates))) return st;
  if ((st = upload(&b->d_reduces, b->reduces))) return st;
  b->ncounters = std::max(1, b->ncounters);
  HIP_OK(hipMalloc((void**)&b->counters, sizeof(int) * b->ncounters));
  HIP_OK(hipMemset(b->counters, 0, sizeof(int) * b->ncounters));
  if (b->gexec) {
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
  }
  b->schedule = schedule;
  return RLB_OK;
}

rlb_status rlb_batch_create(int32_t count, const rlb_symbolic* syms, int32_t precision,
                            rlb_batch* out, int64_t* ws_bytes) {
  if (count < 1 || !syms || !out) return fail(RLB_ERR_ARG, "bad argument");
  if (precision < RLB_PREC_FP64 || precision > RLB_PREC_FP16_UPDATES)
    return fail(RLB_ERR_ARG, "bad precision");
  if (precision != RLB_PREC_FP64)
    return fail(RLB_ERR_UNSUPPORTED, "the batched form is FP64 (reduced forms are single-matrix)");
  *out = nullptr;
  std::unique_ptr<rlb_batch_s> b(new rlb_batch_s());
  b->precision = precision;
  b->syms.assign(syms, syms + count);
  b->base.resize(count);
  b->nnz_ptr.assign(count + 1, 0);
  int64_t run = 0;
  int32_t maxlev = 0;
  for (int32_t i = 0; i < count; ++i) {
    if (!syms[i]) return fail(RLB_ERR_ARG, "null symbolic handle");
    if (syms[i]->s.opt.method != 0)
      return fail(RLB_ERR_UNSUPPORTED, "the batched form runs RLB plans only");
    b->base[i] = run;
    // the matrix's factor storage and the part blocks of its split tiles
    run += syms[i]->s.plan.ws_elems;
    b->nnz_ptr[i + 1] = b->nnz_ptr[i] + syms[i]->s.nnz_a;
    maxlev = std::max(maxlev, syms[i]->s.plan.nlevels);
  }
  b->l_elems = run;
  // contributions of every matrix, concatenated
  std::vector<int64_t> segbase(count, 0);
  for (int32_t i = 0; i < count; ++i) {
    segbase[i] = (int64_t)b->segs.size();
    for (UpdSeg g : syms[i]->s.plan.segs) {
      g.x += b->base[i];
      g.y += b->base[i];
      b->segs.push_back(g);
    }
  }
  if (b->segs.size() > (size_t)INT32_MAX) return fail(RLB_ERR_ARG, "batch too large");
  b->segbase = segbase;
  rlb_status st;
  if ((st = batch_schedule(b.get(), RLB_BATCH_SCHED_LEAVES))) return st;
  (void)maxlev;
  std::vector<int64_t> amap;
  amap.reserve(b->nnz_ptr[count]);
  for (int32_t i = 0; i < count; ++i)
    for (int64_t a : syms[i]->s.plan.amap) amap.push_back(a + b->base[i]);
  if ((st = upload(&b->d_segs, b->segs))) return st;
  for (int ci = 0; ci < 3; ++ci) {
    b->dt_ptr[ci] = (int64_t)b->dtiles.size();
    for (int32_t i = 0; i < count; ++i) {
      const Plan& p = syms[i]->s.plan;
      for (int64_t q = p.dt_ptr[ci]; q < p.dt_ptr[ci + 1]; ++q) {
        DiagTile d = p.dtiles[q];
        d.diag += b->base[i];
        b->dtiles.push_back(d);
      }
    }
  }
  b->dt_ptr[3] = (int64_t)b->dtiles.size();
  if ((st = upload(&b->d_dtiles, b->dtiles))) return st;
  for (int32_t i = 0; i < count; ++i)
    for (DiagTile d : syms[i]->s.plan.ptiles) {
      d.diag += b->base[i];
      b->ptiles.push_back(d);
    }
  if ((st = upload(&b->d_ptiles, b->ptiles))) return st;
  if ((st = upload(&b->d_amap, amap))) return st;
  if ((st = upload(&b->d_nnz_ptr, b->nnz_ptr))) return st;
  HIP_OK(hipMalloc((void**)&b->d_vals, sizeof(double*) * count));
  HIP_OK(hipMalloc((void**)&b->status, sizeof(int) * count));
  b->per.resize(count);
  for (int32_t i = 0; i < count; ++i)
    if ((st = upload_solve(syms[i]->s, b->base[i], b->per[i]))) return st;
  if (ws_bytes) *ws_bytes = b->l_elems * (int64_t)sizeof(double);
  *out = b.release();
  return RLB_OK;
}

static void enqueue_batch(rlb_batch_s* b, double* L, hipStream_t st) {
  int32_t count = (int32_t)b->syms.size();
  launch_init_status(b->status, count, b->counters, b->ncounters, st);
  launch_fill(L, b->l_elems, 0.0, st);
  launch_scatter_batch(b->d_vals, b->d_nnz_ptr, count, b->nnz_ptr[count], b->d_amap, L, st);
  for (const Launch& l : b->launches) {
    if (l.kind == LAUNCH_UPDATE)
      launch_update(b->d_updates + l.start, b->d_segs, l.count, L, b->precision, nullptr,
                    l.variant, st, l.nwave, nullptr, b->narrow_min);
    else if (l.kind == LAUNCH_REDUCE)
      launch_part_reduce(b->d_reduces + l.start, l.count, L, st);
    else {
      // the batch factors with the FP64 panel kernel; its fused update tiles
      // run inside it in the FP64 form and as a short launch of their own in
      // the FP32 form
      const bool inside = b->precision == RLB_PREC_FP64;
      launch_panel(b->d_panels + l.start, l.count, L, b->status, b->counters, 0, l.variant,
                   l.pre != 0, nullptr, nullptr, 0.0, nullptr, nullptr,
                   b->d_updates + l.ustart, b->d_segs, inside ? l.ucount : 0, st, nullptr,
                   b->narrow_min);
      if (!inside && l.ucount)
        launch_update(b->d_updates + l.ustart, b->d_segs, l.ucount, L, b->precision, nullptr,
                      UPD_SHORT, st);
    }
  }
  const int cls_nbb[3] = {1, 2, 4};
  for (int ci = 0; ci < 3; ++ci)
    launch_tile_inverse(b->d_dtiles + b->dt_ptr[ci], b->dt_ptr[ci + 1] - b->dt_ptr[ci],
                        cls_nbb[ci], L, st);
  launch_pair_inverse(b->d_ptiles, (int64_t)b->ptiles.size(), L, st);
}

rlb_status rlb_batch_factor(rlb_batch b, const double* const* values, void* workspace,
                            size_t ws_bytes, void* stream) {
  if (!b || !values || !workspace) return fail(RLB_ERR_ARG, "null argument");
  if (ws_bytes < (size_t)b->l_elems * sizeof(double))
    return fail(RLB_ERR_WORKSPACE, "workspace smaller than the batch needs");
  hipStream_t st = (hipStream_t)stream;
  int32_t count = (int32_t)b->syms.size();
  std::vector<const double*> vals(values, values + count);
  b->L = (double*)workspace;
  b->stream = st;
  bool same = b->gexec && b->g_vals == vals && b->g_L == workspace && b->g_stream == st;
  if (!same) {
    // pointer table: a pageable copy enqueued on the stream before the factor
    HIP_OK(hipMemcpyAsync((void*)b->d_vals, vals.data(), sizeof(double*) * count,
                          hipMemcpyHostToDevice, st));
    HIP_OK(hipStreamSynchronize(st));
  }
  if (b->graph_mode) {
    if (!same) {
      if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
      }
      hipStream_t cs;
      HIP_OK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      hipGraph_t g;
      HIP_OK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      enqueue_batch(b, b->L, cs);
      hipError_t ce = hipStreamEndCapture(cs, &g);
      (void)hipStreamDestroy(cs);
      if (ce != hipSuccess) return fail(RLB_ERR_HIP, "graph capture failed");
      hipError_t ie = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) return fail(RLB_ERR_HIP, "graph instantiate failed");
      b->g_vals = vals;
      b->g_L = workspace;
      b->g_stream = st;
    }
    HIP_OK(hipGraphLaunch(b->gexec, st));
  } else {
    enqueue_batch(b, b->L, st);
    b->g_vals = vals;  // pointer table on the device matches these values
    b->g_L = nullptr;
  }
  HIP_OK(hipGetLastError());
  b->factored = true;
  b->h_info.clear();
  return RLB_OK;
}

rlb_status rlb_batch_status(rlb_batch b, int64_t* info) {
  if (!b || !info) return fail(RLB_ERR_ARG, "null argument");
  if (!b->L) return fail(RLB_ERR_STATE, "no factorization enqueued");
  int32_t count = (int32_t)b->syms.size();
  std::vector<int> v(count);
  HIP_OK(hipMemcpyAsync(v.data(), b->status, sizeof(int) * count, hipMemcpyDeviceToHost,
                        b->stream));
  HIP_OK(hipStreamSynchronize(b->stream));
  rlb_status worst = RLB_OK;
  b->h_info.assign(count, 0);
  for (int32_t i = 0; i < count; ++i) {
    info[i] = v[i] == 0x7fffffff ? 0 : v[i];
    b->h_info[i] = info[i];
    if (info[i] && !worst) worst = (rlb_status)info[i];
  }
  return worst;
}

rlb_status rlb_batch_solve(rlb_batch b, int32_t i, int64_t nrhs, double* B, int64_t ldb,
                           void* stream) {
  if (!b || i < 0 || i >= (int32_t)b->syms.size() || nrhs < 0)
    return fail(RLB_ERR_ARG, "bad argument");
  if (nrhs > 0 && b->syms[i]->s.n > 0 && !B) return fail(RLB_ERR_ARG, "null B");
  if (!b->factored) return fail(RLB_ERR_STATE, "no factorization");
  if (b->h_info.empty()) {  // the statuses of the last factorization, read once
    std::vector<int64_t> info(b->syms.size());
    rlb_status e = rlb_batch_status(b, info.data());
    if (e < 0) return e;
  }
  if (b->h_info[i]) return fail(RLB_ERR_STATE, "this matrix's factorization failed");
  const Symbolic& s = b->syms[i]->s;
  if (ldb < s.n) return fail(RLB_ERR_ARG, "ldb < n");
  if (nrhs == 0 || s.n == 0) return RLB_OK;
  return solve_into(s, b->per[i], b->sc, b->L, nrhs, B, ldb, B, ldb, (hipStream_t)stream);
}

rlb_status rlb_batch_set_schedule(rlb_batch b, int32_t schedule) {
  if (!b || schedule < RLB_BATCH_SCHED_LEAVES || schedule > RLB_BATCH_SCHED_CENTERED)
    return fail(RLB_ERR_ARG, "bad schedule");
  if (schedule == b->schedule) return RLB_OK;
  HIP_OK(hipDeviceSynchronize());
  // the factor storage of every matrix does not depend on the schedule, so a
  // factorization already in the workspace stays valid for the solves
  return batch_schedule(b, schedule);
}

rlb_status rlb_batch_set_narrow_min(rlb_batch b, int64_t min_items) {
  if (!b) return fail(RLB_ERR_ARG, "null handle");
  const int64_t v = min_items > 0 ? min_items : std::numeric_limits<int64_t>::max();
  if (v == b->narrow_min) return RLB_OK;
  HIP_OK(hipDeviceSynchronize());
  b->narrow_min = v;
  if (b->gexec) {  // the launch sequence changed: record the graph again
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
  }
  return RLB_OK;
}

rlb_status rlb_batch_get_tuning(rlb_batch b, int32_t* schedule, int64_t* narrow_min) {
  if (!b) return fail(RLB_ERR_ARG, "null handle");
  if (schedule) *schedule = b->schedule;
  if (narrow_min)
    *narrow_min = b->narrow_min == std::numeric_limits<int64_t>::max() ? 0 : b->narrow_min;
  return RLB_OK;
}

rlb_status rlb_batch_autotune(rlb_batch b, const double* const* values, void* workspace,
                              size_t ws_bytes, void* stream, int32_t reps, int32_t* chosen,
                              double* ms) {
  if (!b || !values || !workspace || reps < 1) return fail(RLB_ERR_ARG, "bad argument");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  // the level schedule, and for each the narrow-item threshold of the
  // one-per-wavefront kernels (0: never)
  static const int64_t kNarrow[] = {256, 1024, 4096, 0};
  double best = 0;
  int32_t best_s = RLB_BATCH_SCHED_LEAVES;
  int64_t best_n = WAVE_SPLIT_MIN;
  bool have = false;
  rlb_status r = RLB_OK;
  for (int32_t sch = RLB_BATCH_SCHED_LEAVES; sch <= RLB_BATCH_SCHED_CENTERED && !r; ++sch) {
    if ((r = rlb_batch_set_schedule(b, sch))) break;
    double best_here = 0;
    for (int q = 0; q < 4 && !r; ++q) {
      if ((r = rlb_batch_set_narrow_min(b, kNarrow[q]))) break;
      // one untimed factorization (graph capture when enabled), then reps timed
      if ((r = rlb_batch_factor(b, values, workspace, ws_bytes, stream))) break;
      float total = 0;
      for (int32_t k = 0; k < reps && !r; ++k) {
        (void)hipEventRecord(e0, st);
        r = rlb_batch_factor(b, values, workspace, ws_bytes, stream);
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) r = fail(RLB_ERR_HIP, "event");
        float t = 0;
        (void)hipEventElapsedTime(&t, e0, e1);
        total += t;
      }
      const double avg = total / reps;
      if (q == 0 || avg < best_here) best_here = avg;
      if (!have || avg < best) {
        best = avg;
        best_s = sch;
        best_n = kNarrow[q];
        have = true;
      }
    }
    if (ms) ms[sch] = best_here;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (r) return r;
  if (chosen) *chosen = best_s;
  if ((r = rlb_batch_set_narrow_min(b, best_n))) return r;
  return rlb_batch_set_schedule(b, best_s);
}

rlb_status rlb_batch_set_graph_mode(rlb_batch b, int32_t on) {
  if (!b) return fail(RLB_ERR_ARG, "null handle");
  b->graph_mode = on != 0;
  return RLB_OK;
}

void rlb_batch_free(rlb_batch b) { delete b; }

}  // extern "C"
