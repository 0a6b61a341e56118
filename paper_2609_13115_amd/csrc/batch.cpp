// Batch engine: many uneven subdomains advanced together (the paper runs the
// subsystems of a process one after another with threads inside each,
// Sec. V-B; here one GPU holds them all).
//
// One batch iteration =
//   m_max grouped filter steps on the batch stream: every step is one
//   persistent forward-projection launch and one persistent stencil launch
//   per tile shape, covering all subdomains whose degree exceeds the step;
//   then, per subdomain on a pool of streams: H Psi_f, the two projection
//   GEMMs, the dense FP64 eigensolve (no host synchronisation), the
//   rotation, the FP64 residual and the next filter coefficients (computed on
//   the device from the new Ritz values).
// The iteration's launches are captured into a hipGraph per (active set,
// buffer parity, degrees) and replayed; only the convergence test reads
// results back to the host between iterations.  The autotuner times the fused filter
// kernel's tile shapes per subdomain shape and keeps the winners in a small
// JSON cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "xls_handle.h"

using namespace xls;

namespace {

constexpr int kMaxDegree = 256;
// Streams carrying the per-subdomain tails (H Psi_f, GEMMs, dense solve,
// rotation, residual) of one batch iteration: the dense solve is latency
// bound, so several run side by side.  XLS_BATCH_STREAMS overrides (1..32).
int pool_streams() {
  const char* e = std::getenv("XLS_BATCH_STREAMS");
  const int v = e ? std::atoi(e) : 0;
  return v >= 1 && v <= 32 ? v : 4;
}
constexpr int kGraphCache = 8;

struct GroupHolder {
  FilterGroup<float>* g32 = nullptr;
  FilterGroup<double>* g64 = nullptr;
  ~GroupHolder() {
    if (g32) filter_group_free(g32);
    if (g64) filter_group_free(g64);
  }
};

struct GraphEntry {
  std::string key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  GroupHolder* group = nullptr;
  int seen = 0;
  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    delete group;
    exec = nullptr;
    graph = nullptr;
    group = nullptr;
  }
};

struct SubState {
  double lmax = 0.0;
  int degree = 0, max_iter = 0, gate = 0, gprec = XLS_PREC_FP64;
  int pprec = XLS_PREC_FP64;  // projection and rotation precision this iteration (polish_prec)
  double resid_tol = 0.0;
  int iters = 0;        // iterations of the current run (bounded by max_iter)
  int total_iters = 0;  // including a fallback run
  int status = XLS_OK;
  bool active = false;
  // learned bounds with the Lanczos fallback
  double fb_tol = 0.0;  // > 0: fallback on
  int fb_degree = 0;
  int lanczos_k = 0;
  int cur0 = 0;         // block parity at the start (the backup's contents)
  bool fell_back = false;
  bool started = false;  // begun in the current xls_batch_chefsi call
};

// Core rows of a subdomain kept after its working set is released (slot
// residency): the density and the interior weights read only core points.
struct CoreStore {
  void* blk = nullptr;         // ncore x ns, leading dimension ld, storage precision
  int64_t ncore = 0, ld = 0;
  int32_t* rows = nullptr;     // device: local grid index of each core row (ascending)
  int64_t* gidx = nullptr;     // device: global index of each core row
  std::vector<int32_t> hrows;  // host copy of rows
  void release_blk() {
    dfree(blk);
    blk = nullptr;
  }
  ~CoreStore() {
    dfree(blk);
    dfree(rows);
    dfree(gidx);
  }
};

}  // namespace

struct xls_batch_s {
  int n = 0;
  int prec = XLS_PREC_FP64;
  std::vector<xls_subdomain_s*> subs;
  hipStream_t main = nullptr;
  std::vector<hipStream_t> pool;
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  std::vector<double*> coef;
  int32_t* flags = nullptr;  // [n] bad-bounds flags from the coefficient kernel
  std::vector<GraphEntry> graphs;
  std::vector<SubState> st;
  // statistics
  int64_t iterations = 0, captures = 0, replays = 0;
  double iter_ms = 0.0, last_iter_ms = 0.0;
  // occupation of the whole batch (xls_batch_fermi / xls_batch_assemble)
  double* lam_all = nullptr;  // [sum ns] Ritz values, subdomain order
  double* c_all = nullptr;    // [sum ns] interior weights
  double* fout = nullptr;     // [8] solver outputs
  int64_t nstates = 0;
  bool have_fermi = false;
  double mu = 0.0, sigma = 0.0;
  std::vector<int64_t*> gidx;  // per subdomain: device copy of the local->global map
  std::vector<int8_t> gidx_ok;  // per subdomain: 1 = core points map to distinct global points, -1 = not
  double* rho_global = nullptr;
  int64_t rho_global_n = 0;
  double* dos_buf = nullptr;  // [2 * nbins + 1]: edges, then bins
  int dos_cap = 0;
  // slot residency (xls_batch_create_slots): working sets allocated on
  // admission and released when a subdomain finishes, within a byte budget
  bool slots = false;
  int64_t budget = 0;
  int64_t resident_bytes = 0, peak_bytes = 0;  // working sets and core stores held
  int max_active = 0;
  std::vector<double*> pool_gwork;  // split-K workspace per pool stream (shared by its handles)
  size_t pool_gwork_elems = 0;
  std::vector<CoreStore> core;      // per subdomain (slot mode)
  uint8_t* ones = nullptr;          // all-ones mask over the largest core
  int64_t ones_n = 0;

  ~xls_batch_s() {
    if (main) (void)hipStreamSynchronize(main);
    for (auto* s : subs)
      if (s) xls_subdomain_destroy(s);
    for (auto& g : graphs) g.release();
    for (auto* c : coef) dfree(c);
    dfree(flags);
    dfree(lam_all);
    dfree(c_all);
    dfree(fout);
    for (auto* g : gidx) dfree(g);
    dfree(rho_global);
    dfree(dos_buf);
    core.clear();
    dfree(ones);
    for (auto* g : pool_gwork) dfree(g);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    for (auto e : ev_join) (void)hipEventDestroy(e);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    for (auto p : pool) (void)hipStreamDestroy(p);
    if (main) (void)hipStreamDestroy(main);
  }
};

namespace {

// Rotation and FP64 residual with explicit buffers (the handle's parity is
// advanced by the caller once per iteration, outside any capture).
template <typename TS>
void tail_stages(xls_subdomain_s* s, const SubState& ss, int cur_f, double* coef, int32_t* bad) {
  const int ns = s->ns;
  TS* Bc = B<TS>(s, cur_f);
  TS* W = B<TS>(s, 1 - cur_f);
  apply_H<TS>(s, Bc, W, ns, static_cast<TS*>(s->alpha));
  gemm_tn<TS>(ss.pprec, Bc, s->ld, Bc, s->ld, ns, ns, s->nd, s->Mdev, ns, 1, 0, s->gwork, s->gwork_elems, s->st, s->gplan);
  gemm_tn<TS>(ss.pprec, Bc, s->ld, W, s->ld, ns, ns, s->nd, s->Hsdev, ns, 1, 1, s->gwork, s->gwork_elems, s->st, s->gplan);
  (void)dense_geneig(s->dw, s->Hsdev, s->Mdev, s->Ydev, s->st, /*check_spd=*/false);
  XLS_HIP(hipMemcpyAsync(s->lam_dev, s->dw.lam(), ns * 8, hipMemcpyDeviceToDevice, s->st));
  // Psi <- Psi_f Y into the other buffer
  gemm_nn<TS>(ss.pprec, Bc, s->ld, s->Ydev, ns, static_cast<int>(s->nd), ns, ns, W, s->ld, s->bwork, s->st, s->gplan);
  launch_proj_forward<TS, double>(s->op64, W, s->ld, ns, s->alpha64, s->st);
  launch_stencil<TS, double>(kResid, s->op64, W, s->ld, ns, s->alpha64, nullptr, nullptr, 1.0, 0.0, 0.0,
                             s->lam_dev, s->partial, s->resid_dev, s->st, s->cfg64, s->rq_dev);
  launch_filter_coef(s->lam_dev, ns, 0.0, 0.0, ss.lmax, ss.degree, coef, bad, s->st);
}

template <typename TS>
FilterGroup<TS>* build_group(xls_batch_s* b, const std::vector<int>& act) {
  std::vector<FilterGroupOp<TS>> ops;
  for (int i : act) {
    xls_subdomain_s* s = b->subs[i];
    FilterGroupOp<TS> o{};
    o.op = &op_of<TS>(s);
    o.buf[0] = B<TS>(s, 0);
    o.buf[1] = B<TS>(s, 1);
    o.cur0 = s->cur;
    o.ld = s->ld;
    o.ncols = s->ns;
    o.alpha = static_cast<TS*>(s->alpha);
    o.coef = b->coef[i];
    o.degree = b->st[i].degree;
    o.cfg = cfg_of<TS>(s);
    ops.push_back(o);
  }
  return filter_group_build<TS>(ops);
}

// Records one batch iteration over the active subdomains (eager, or inside a
// stream capture of b->main).
template <typename TS>
void record_iteration(xls_batch_s* b, FilterGroup<TS>* g, const std::vector<int>& act) {
  // the filter runs on main, after the previous iteration's tails (joined
  // into main at the end of every iteration)
  for (int k = 0; k < filter_group_steps(g); ++k) filter_group_step<TS>(g, k, b->main);
  XLS_HIP(hipEventRecord(b->ev_fork, b->main));
  for (auto p : b->pool) XLS_HIP(hipStreamWaitEvent(p, b->ev_fork, 0));
  for (int i : act) {
    xls_subdomain_s* s = b->subs[i];
    const int cur_f = (s->cur + b->st[i].degree) & 1;
    tail_stages<TS>(s, b->st[i], cur_f, b->coef[i], b->flags + i);
  }
  for (size_t p = 0; p < b->pool.size(); ++p) {
    XLS_HIP(hipEventRecord(b->ev_join[p], b->pool[p]));
    XLS_HIP(hipStreamWaitEvent(b->main, b->ev_join[p], 0));
  }
}

// Everything a captured iteration bakes in: the active set, each block's
// parity, degree, GEMM precision, lam_max (a kernel argument of the
// coefficient update) and stencil launch shape.
std::string graph_key(xls_batch_s* b, const std::vector<int>& act) {
  std::ostringstream k;
  k << std::hexfloat;
  for (int i : act) {
    const xls_subdomain_s* s = b->subs[i];
    // the launch shape too: a handle re-tuned through xls_subdomain_tune
    // must not replay a graph of its old tiles
    const StencilLaunch& c = s->prec == XLS_PREC_FP32 ? s->cfg32 : s->cfg64;
    k << i << (s->cur ? 'b' : 'a') << b->st[i].degree << 'p' << b->st[i].gprec << 'q' << b->st[i].pprec << 'l'
      << b->st[i].lmax << 's' << c.block << '.' << c.ty << '.' << c.tz << '.' << c.nv << 'g'
      << s->gplan.split_scale << '.' << s->gplan.tile_tn << '.' << s->gplan.tile_nn << ',';
  }
  return k.str();
}

// The first time an (active set, parity, degrees) key is seen the iteration
// runs eagerly, so that every one-time kernel configuration happens outside a
// capture; from the second time on it is captured once and replayed.
template <typename TS>
void run_iteration(xls_batch_s* b, const std::vector<int>& act, bool use_graph) {
  const std::string key = graph_key(b, act);
  GraphEntry* ge = nullptr;
  for (auto& g : b->graphs)
    if (g.key == key) ge = &g;
  if (!ge) {
    if (static_cast<int>(b->graphs.size()) >= kGraphCache) {
      XLS_HIP(hipStreamSynchronize(b->main));
      b->graphs.front().release();
      b->graphs.erase(b->graphs.begin());
    }
    b->graphs.push_back(GraphEntry{});
    ge = &b->graphs.back();
    ge->key = key;
    ge->group = new GroupHolder();
    FilterGroup<TS>* g = build_group<TS>(b, act);
    if (std::is_same<TS, float>::value)
      ge->group->g32 = reinterpret_cast<FilterGroup<float>*>(g);
    else
      ge->group->g64 = reinterpret_cast<FilterGroup<double>*>(g);
  }
  FilterGroup<TS>* g = std::is_same<TS, float>::value ? reinterpret_cast<FilterGroup<TS>*>(ge->group->g32)
                                                      : reinterpret_cast<FilterGroup<TS>*>(ge->group->g64);
  if (use_graph && !ge->exec && ge->seen > 0) {
    XLS_HIP(hipStreamBeginCapture(b->main, hipStreamCaptureModeThreadLocal));
    try {
      record_iteration<TS>(b, g, act);
    } catch (...) {
      hipGraph_t dead = nullptr;
      (void)hipStreamEndCapture(b->main, &dead);
      if (dead) (void)hipGraphDestroy(dead);
      throw;
    }
    XLS_HIP(hipStreamEndCapture(b->main, &ge->graph));
    XLS_HIP(hipGraphInstantiate(&ge->exec, ge->graph, nullptr, nullptr, 0));
    ++b->captures;
  }
  ++ge->seen;
  XLS_HIP(hipEventRecord(b->t0, b->main));
  if (use_graph && ge->exec) {
    XLS_HIP(hipGraphLaunch(ge->exec, b->main));
    ++b->replays;
  } else {
    record_iteration<TS>(b, g, act);
  }
  XLS_HIP(hipEventRecord(b->t1, b->main));
}

// First-iteration Lanczos bounds of a subdomain (cached per handle and k).
template <typename TS>
void lanczos_bounds_of(xls_subdomain_s* s, int k_req, double& a0, double& lc, double& lmax) {
  const int k = lanczos_steps(s, k_req);
  if (!s->have_lanczos || s->lz_k != k) lanczos_run<TS>(s, k);
  a0 = s->lz_lo;
  lmax = s->lz_up;
  lc = a0 + 0.1 * (lmax - a0);
}

void check_params(const xls_chefsi_params_t& p, bool fp64) {
  if (p.degree < 1 || p.degree > kMaxDegree || p.max_iter < 1)
    fail(XLS_ERR_INVALID_ARG, "degree must be in [1, 256] and max_iter >= 1");
  if (p.lanczos_k > kMaxLanczos) fail(XLS_ERR_INVALID_ARG, "lanczos_k must be <= 60");
  if (p.gemm_prec < XLS_PREC_FP64 || p.gemm_prec > XLS_PREC_BF16X3) fail(XLS_ERR_INVALID_ARG, "bad gemm_prec");
  if (fp64 && p.gemm_prec != XLS_PREC_FP64) fail(XLS_ERR_INVALID_ARG, "FP64 batches run FP64 GEMMs");
  if (p.bounds_mode < XLS_BOUNDS_GIVEN || p.bounds_mode > XLS_BOUNDS_LEARNED)
    fail(XLS_ERR_INVALID_ARG, "unknown bounds_mode");
  if (p.bounds_mode == XLS_BOUNDS_LEARNED && !(p.fallback_tol >= 0))
    fail(XLS_ERR_INVALID_ARG, "fallback_tol must be >= 0");
  if (p.bounds_mode == XLS_BOUNDS_LEARNED && p.fallback_tol > 0 && p.fallback_degree > kMaxDegree)
    fail(XLS_ERR_INVALID_ARG, "fallback_degree must be <= 256");
  if (p.bounds_mode != XLS_BOUNDS_LANCZOS &&
      (!std::isfinite(p.lam_max) || !std::isfinite(p.lam_cut) ||
       (p.bounds_mode == XLS_BOUNDS_GIVEN && !std::isfinite(p.lam_lo))))
    fail(XLS_ERR_INVALID_ARG, "bounds must be finite");
}

// Starts subdomain i's run from its current block: first bounds, state,
// the backup of the start block (fallback, resident mode) and the filter
// coefficients (on the handle's stream).
template <typename TS>
void begin_run(xls_batch_s* b, int i, const xls_chefsi_params_t& p) {
  xls_subdomain_s* s = b->subs[i];
  SubState& ss = b->st[i];
  double a0, lc, lmax;
  if (p.bounds_mode == XLS_BOUNDS_GIVEN) {
    a0 = p.lam_lo;
    lc = p.lam_cut;
    lmax = p.lam_max;
  } else if (p.bounds_mode == XLS_BOUNDS_LANCZOS) {
    lanczos_bounds_of<TS>(s, p.lanczos_k, a0, lc, lmax);
  } else {
    lmax = p.lam_max;
    lc = p.lam_cut;
    a0 = std::min(s->a0_bound, lc - 1e-3 * std::fabs(lmax - lc));
  }
  if (!(a0 < lc && lc < lmax) || !std::isfinite(a0) || !std::isfinite(lmax))
    fail(XLS_ERR_INVALID_ARG, "subdomain " + std::to_string(i) + ": bounds must satisfy a0 < lam_cut < lam_max");
  ss.lmax = lmax;
  ss.degree = p.degree;
  ss.max_iter = p.max_iter;
  ss.gprec = p.gemm_prec;
  ss.pprec = polish_prec(p.gemm_prec, HUGE_VAL);
  ss.resid_tol = p.resid_tol;
  ss.gate = p.n_gate > 0 ? std::min(p.n_gate, s->ns) : std::max(1, static_cast<int>(std::floor(s->ns / 1.1 + 1e-9)));
  ss.iters = 0;
  ss.total_iters = 0;
  ss.status = XLS_OK;
  ss.fb_tol = p.bounds_mode == XLS_BOUNDS_LEARNED ? p.fallback_tol : 0.0;
  ss.fb_degree = p.fallback_degree > 0 ? p.fallback_degree : p.degree;
  ss.lanczos_k = p.lanczos_k;
  ss.cur0 = s->cur;
  ss.fell_back = false;
  ss.started = true;
  s->happly = 0;
  s->last_fallback = 0;
  s->last_iters = 0;
  ss.active = true;
  if (ss.fb_tol > 0 && !b->slots) {  // the start block, for a restart with Lanczos bounds
    if (!s->backup) s->backup = dalloc<TS>(static_cast<size_t>(s->ld) * s->ns);
    XLS_HIP(hipMemcpyAsync(s->backup, B<TS>(s, s->cur), static_cast<size_t>(s->ld) * s->ns * sizeof(TS),
                           hipMemcpyDeviceToDevice, s->st));
  }
  launch_filter_coef(nullptr, s->ns, a0, lc, lmax, p.degree, b->coef[i], b->flags + i, s->st);
}

// Learned bounds that missed (M_s not positive definite, or the gated
// residual above fallback_tol or NaN) restart from the start block with
// Lanczos bounds and the fallback degree.
bool needs_fallback(const SubState& ss, const std::vector<double>& hr) {
  if (!(ss.fb_tol > 0) || ss.fell_back) return false;
  return ss.status != XLS_OK || !(gated_max(hr.data(), ss.gate) <= ss.fb_tol);
}

template <typename TS>
void begin_fallback(xls_batch_s* b, int i) {
  xls_subdomain_s* s = b->subs[i];
  SubState& ss = b->st[i];
  if (b->slots) {
    load_start_block<TS>(s, nullptr);  // the start block is X0: drawn or uploaded again
  } else {
    XLS_HIP(hipMemcpyAsync(B<TS>(s, ss.cur0), s->backup, static_cast<size_t>(s->ld) * s->ns * sizeof(TS),
                           hipMemcpyDeviceToDevice, s->st));
    s->cur = ss.cur0;
  }
  double a0, lc, lmax;
  lanczos_bounds_of<TS>(s, ss.lanczos_k, a0, lc, lmax);
  ss.lmax = lmax;
  ss.degree = ss.fb_degree;
  ss.pprec = polish_prec(ss.gprec, HUGE_VAL);
  ss.iters = 0;
  ss.status = XLS_OK;
  ss.active = true;
  ss.fell_back = true;
  s->last_fallback = 1;
  launch_filter_coef(nullptr, s->ns, a0, lc, lmax, ss.degree, b->coef[i], b->flags + i, s->st);
}

// One batch iteration over the active subdomains; updates their states and
// returns those that became inactive.
template <typename TS>
std::vector<int> iterate_once(xls_batch_s* b, bool use_graph, std::vector<std::vector<double>>& hl,
                              std::vector<std::vector<double>>& hr) {
  std::vector<int> act, ended;
  for (int i = 0; i < b->n; ++i)
    if (b->st[i].active) act.push_back(i);
  if (act.empty()) return ended;
  b->max_active = std::max(b->max_active, static_cast<int>(act.size()));
  std::vector<int32_t> hflag(b->n), hspd(b->n);
  std::vector<std::vector<double>> hq(b->n);
  // reported Ritz values as in a single run: FP64 Rayleigh quotients unless
  // the block and the projection are FP64
  auto use_rq = [&](int i) { return !std::is_same<TS, double>::value || b->st[i].gprec != XLS_PREC_FP64; };
  run_iteration<TS>(b, act, use_graph);
  for (int i : act) {
    xls_subdomain_s* s = b->subs[i];
    XLS_HIP(hipMemcpyAsync(hl[i].data(), s->lam_dev, s->ns * 8, hipMemcpyDeviceToHost, b->main));
    if (use_rq(i)) {
      hq[i].resize(s->ns);
      XLS_HIP(hipMemcpyAsync(hq[i].data(), s->rq_dev, s->ns * 8, hipMemcpyDeviceToHost, b->main));
    }
    XLS_HIP(hipMemcpyAsync(hr[i].data(), s->resid_dev, s->ns * 8, hipMemcpyDeviceToHost, b->main));
    XLS_HIP(hipMemcpyAsync(&hspd[i], s->dw.flag, 4, hipMemcpyDeviceToHost, b->main));
    XLS_HIP(hipMemcpyAsync(&hflag[i], b->flags + i, 4, hipMemcpyDeviceToHost, b->main));
  }
  XLS_HIP(hipStreamSynchronize(b->main));
  float ms = 0.0f;
  XLS_HIP(hipEventElapsedTime(&ms, b->t0, b->t1));
  b->last_iter_ms = ms;
  b->iter_ms += ms;
  ++b->iterations;
  for (int i : act) {
    xls_subdomain_s* s = b->subs[i];
    SubState& ss = b->st[i];
    s->cur = (s->cur + ss.degree + 1) & 1;
    ++ss.iters;
    ++ss.total_iters;
    s->last_iters = ss.total_iters;
    s->happly += static_cast<int64_t>(ss.degree + 1) * s->ns;  // filter + residual (H Psi_f counted by apply_H)
    s->ritz = use_rq(i) ? hq[i] : hl[i];
    s->have_ritz = true;
    if (hspd[i]) {
      ss.status = XLS_ERR_NOT_SPD;
      ss.active = false;
    } else if (hflag[i]) {  // degenerate bounds for the next filter: stop with what we have
      ss.active = false;
    } else {
      const double mx = gated_max(hr[i].data(), ss.gate);
      ss.pprec = polish_prec(ss.gprec, mx);
      if (ss.resid_tol > 0 && mx <= ss.resid_tol) ss.active = false;
      if (ss.iters >= ss.max_iter) ss.active = false;
    }
    if (!ss.active) ended.push_back(i);
  }
  return ended;
}

// Slot residency: the subdomain's core rows move to its core store and its
// working set is released.
template <typename TS>
void finalize_slot(xls_batch_s* b, int i) {
  xls_subdomain_s* s = b->subs[i];
  CoreStore& cs = b->core[i];
  if (cs.ncore > 0) {
    cs.release_blk();
    cs.blk = dalloc<TS>(static_cast<size_t>(cs.ld) * s->ns);
    b->resident_bytes += cs.ld * s->ns * static_cast<int64_t>(sizeof(TS));
    launch_gather_rows<TS>(B<TS>(s, s->cur), s->ld, cs.rows, cs.ncore, s->ns, static_cast<TS*>(cs.blk), cs.ld,
                           s->st);
  }
  XLS_HIP(hipStreamSynchronize(s->st));
  b->resident_bytes -= static_cast<int64_t>(subdomain_ws_bytes(s, true));
  b->peak_bytes = std::max(b->peak_bytes, b->resident_bytes);
  subdomain_ws_free(s);
}

// Working set of subdomain i from the batch's budget, start block loaded.
template <typename TS>
void admit_slot(xls_batch_s* b, int i) {
  xls_subdomain_s* s = b->subs[i];
  const int p = static_cast<int>(std::find(b->pool.begin(), b->pool.end(), s->st) - b->pool.begin());
  subdomain_ws_alloc(s, b->pool_gwork[p], b->pool_gwork_elems);
  b->resident_bytes += static_cast<int64_t>(subdomain_ws_bytes(s, true));
  b->peak_bytes = std::max(b->peak_bytes, b->resident_bytes);
  load_start_block<TS>(s, nullptr);
}

// Device bytes a subdomain's run takes while resident (its working set plus
// the Lanczos vectors when its bounds come from Lanczos).
int64_t run_bytes(const xls_subdomain_s* s, const xls_chefsi_params_t& p) {
  int64_t bytes = static_cast<int64_t>(subdomain_ws_bytes(s, true));
  const bool lanczos = p.bounds_mode == XLS_BOUNDS_LANCZOS ||
                       (p.bounds_mode == XLS_BOUNDS_LEARNED && p.fallback_tol > 0);
  if (lanczos) bytes += static_cast<int64_t>(s->ld) * (lanczos_steps(s, p.lanczos_k) + 2) * s->esize();
  return bytes;
}

template <typename TS>
void batch_chefsi(xls_batch_s* b, const xls_chefsi_params_t* P, int use_graph) {
  b->have_fermi = false;  // new blocks: a stored Fermi level no longer applies
  const int n = b->n;
  for (int i = 0; i < n; ++i) check_params(P[i], std::is_same<TS, double>::value);
  std::vector<std::vector<double>> hl(n), hr(n);
  for (int i = 0; i < n; ++i) {
    hl[i].assign(b->subs[i]->ns, 0.0);
    hr[i].assign(b->subs[i]->ns, 0.0);
    b->st[i].started = false;
    b->st[i].active = false;
  }
  b->iterations = 0;
  b->iter_ms = 0.0;
  b->max_active = 0;
  // every pending subdomain, largest work first (the tail holds the small ones)
  std::vector<int> pending;
  if (b->slots) {
    for (int i = 0; i < n; ++i) {
      b->core[i].release_blk();
      if (b->subs[i]->resident) subdomain_ws_free(b->subs[i]);  // left by an interrupted call
      b->subs[i]->have_ritz = false;
      pending.push_back(i);
    }
    b->resident_bytes = 0;  // no working set or core store is held between calls
    b->peak_bytes = 0;
    std::stable_sort(pending.begin(), pending.end(), [&](int x, int y) {
      const double cx = static_cast<double>(b->subs[x]->nd) * b->subs[x]->ns * P[x].degree;
      const double cy = static_cast<double>(b->subs[y]->nd) * b->subs[y]->ns * P[y].degree;
      return cx > cy;
    });
  } else {
    for (int i = 0; i < n; ++i) begin_run<TS>(b, i, P[i]);
    for (auto* s : b->subs) XLS_HIP(hipStreamSynchronize(s->st));
  }
  size_t next = 0;
  // optional progress lines on stderr (XLS_BATCH_PROGRESS=seconds between lines)
  const char* prog_env = std::getenv("XLS_BATCH_PROGRESS");
  const double prog_every = prog_env ? std::atof(prog_env) : 0.0;
  auto t_start = std::chrono::steady_clock::now();
  auto t_last = t_start;
  for (;;) {
    if (prog_every > 0) {
      const auto now = std::chrono::steady_clock::now();
      if (std::chrono::duration<double>(now - t_last).count() >= prog_every) {
        t_last = now;
        int act = 0, done = 0;
        for (int i = 0; i < n; ++i) {
          act += b->st[i].active;
          done += b->st[i].started && !b->st[i].active;
        }
        std::fprintf(stderr, "[xls batch] %.1f s: iteration %lld, %d active, %d done of %d, resident %.1f GB\n",
                     std::chrono::duration<double>(now - t_start).count(), static_cast<long long>(b->iterations),
                     act, done, n, b->resident_bytes / 1e9);
        std::fflush(stderr);
      }
    }
    if (b->slots) {  // admit while the budget allows (always at least one)
      bool any_active = false;
      for (int i = 0; i < n; ++i) any_active = any_active || b->st[i].active;
      std::vector<int> adm;
      while (next < pending.size()) {
        const int i = pending[next];
        const int64_t need = run_bytes(b->subs[i], P[i]);
        if ((any_active || !adm.empty()) && b->resident_bytes + need > b->budget) break;
        admit_slot<TS>(b, i);
        begin_run<TS>(b, i, P[i]);
        if (b->subs[i]->lz && P[i].bounds_mode == XLS_BOUNDS_LANCZOS) {  // bounds cached: vectors not needed
          XLS_HIP(hipStreamSynchronize(b->subs[i]->st));
          dfree(b->subs[i]->lz);
          b->subs[i]->lz = nullptr;
          b->subs[i]->lz_cols = 0;
        }
        adm.push_back(i);
        ++next;
      }
      for (int i : adm) XLS_HIP(hipStreamSynchronize(b->subs[i]->st));
    }
    const std::vector<int> ended = iterate_once<TS>(b, use_graph != 0, hl, hr);
    if (ended.empty()) {
      bool any = false;
      for (int i = 0; i < n; ++i) any = any || b->st[i].active;
      if (!any && (!b->slots || next >= pending.size())) break;
      continue;
    }
    for (int i : ended) {
      if (needs_fallback(b->st[i], hr[i])) {
        begin_fallback<TS>(b, i);
        XLS_HIP(hipStreamSynchronize(b->subs[i]->st));
      } else if (b->slots) {
        finalize_slot<TS>(b, i);
      }
    }
  }
}

// --- autotuner -------------------------------------------------------------

// Shape classes: the filter kernel's tile depends on the exact row length
// (n_x: halo budget, points per lane) and the boundary; n_y, n_z and the
// atom count (LDS for the projection coefficients) only through their size,
// so they are bucketed (8 planes, 64 atoms) and one timing serves a class.
std::string shape_key(xls_subdomain_s* s) {
  std::ostringstream o;
  o << (s->prec == XLS_PREC_FP32 ? "f32" : "f64") << "_nx" << s->n[0] << "_ny" << (s->n[1] + 7) / 8 * 8 << "_nz"
    << (s->n[2] + 7) / 8 * 8 << (s->bc == XLS_BC_PERIODIC ? "_p" : "_d") << "_na" << (s->n_atoms + 63) / 64 * 64;
  return o.str();
}

// tile shape of a class: block threads, rows per tile, vectors per tile
using Shape = std::array<int, 3>;

std::map<std::string, Shape> read_cache(const char* path) {
  std::map<std::string, Shape> m;
  if (!path) return m;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    // lines of the form  "key": [block, ty, nv],
    const size_t q0 = line.find('"'), q1 = line.find('"', q0 + 1), lb = line.find('['),
                 rb = line.find(']', lb);
    if (q0 == std::string::npos || q1 == std::string::npos || lb == std::string::npos || rb == std::string::npos)
      continue;
    std::istringstream in(line.substr(lb + 1, rb - lb - 1));
    Shape v{0, 0, 0};
    char sep = 0;
    if (in >> v[0] >> sep >> v[1] >> sep >> v[2]) m[line.substr(q0 + 1, q1 - q0 - 1)] = v;
  }
  return m;
}

void write_cache(const char* path, const std::map<std::string, Shape>& m) {
  if (!path) return;
  std::ofstream f(path);
  if (!f) fail(XLS_ERR_INVALID_ARG, std::string("cannot write tuning cache ") + path);
  f << "{\n";
  size_t k = 0;
  for (const auto& e : m)
    f << "  \"" << e.first << "\": [" << e.second[0] << ", " << e.second[1] << ", " << e.second[2] << "]"
      << (++k < m.size() ? ",\n" : "\n");
  f << "}\n";
}

// Average fused-filter kernel time (ms) of subdomain s under launch shape cfg;
// reads the current block and overwrites the spare one.
template <typename TS>
double time_filter(xls_subdomain_s* s, const StencilLaunch& cfg, hipEvent_t e0, hipEvent_t e1) {
  const auto& op = op_of<TS>(s);
  TS* y = B<TS>(s, s->cur);
  TS* o = B<TS>(s, 1 - s->cur);
  TS* al = static_cast<TS*>(s->alpha);
  auto once = [&]() {
    launch_stencil<TS, TS>(kFilter, op, y, s->ld, s->ns, al, o, o, 0.1, 0.0, 0.01, nullptr, nullptr, nullptr,
                           s->st, cfg);
  };
  once();
  XLS_HIP(hipEventRecord(e0, s->st));
  constexpr int reps = 3;
  for (int r = 0; r < reps; ++r) once();
  XLS_HIP(hipEventRecord(e1, s->st));
  XLS_HIP(hipEventSynchronize(e1));
  float ms = 0.0f;
  XLS_HIP(hipEventElapsedTime(&ms, e0, e1));
  return ms / reps;
}

// GEMM classes: N_d bucketed to 32768 rows (the split-K count follows it),
// ns to 32 columns (the tile grid follows it).
std::string gemm_key(xls_subdomain_s* s) {
  std::ostringstream o;
  o << "gemm_" << (s->prec == XLS_PREC_FP32 ? "f32" : "f64") << "_nd" << (s->nd + 32767) / 32768 * 32768 << "_ns"
    << (s->ns + 31) / 32 * 32;
  return o.str();
}

// Average device ms of the projection Psi^T (H Psi) (upper triangle) and the
// rotation Psi Q under plan g, on the current block and the spare one.
template <typename TS>
std::array<double, 2> time_gemm_plan(xls_subdomain_s* s, const GemmPlan& g, hipEvent_t e0, hipEvent_t e1) {
  const int gprec = std::is_same<TS, float>::value ? XLS_PREC_FP32 : XLS_PREC_FP64;
  TS* Bc = B<TS>(s, s->cur);
  TS* W = B<TS>(s, 1 - s->cur);
  std::array<double, 2> out{};
  for (int which = 0; which < 2; ++which) {
    auto once = [&]() {
      if (which == 0)
        gemm_tn<TS>(gprec, Bc, s->ld, Bc, s->ld, s->ns, s->ns, s->nd, s->Hsdev, s->ns, 1, 1, s->gwork,
                    s->gwork_elems, s->st, g);
      else
        gemm_nn<TS>(gprec, Bc, s->ld, s->Ydev, s->ns, static_cast<int>(s->nd), s->ns, s->ns, W, s->ld, s->bwork,
                    s->st, g);
    };
    once();
    XLS_HIP(hipEventRecord(e0, s->st));
    constexpr int reps = 3;
    for (int r = 0; r < reps; ++r) once();
    XLS_HIP(hipEventRecord(e1, s->st));
    XLS_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    XLS_HIP(hipEventElapsedTime(&ms, e0, e1));
    out[which] = ms / reps;
  }
  return out;
}

// Chooses each class's GEMM plan (split scale and tile kind of the
// projection, tile kind of the rotation) by timing, or from the cache, and
// applies it to every handle of the class.  Returns the classes timed.
template <typename TS>
int tune_gemms(xls_batch_s* b, std::map<std::string, Shape>& cache, std::map<std::string, Shape>& chosen) {
  hipEvent_t e0, e1;
  XLS_HIP(hipEventCreate(&e0));
  XLS_HIP(hipEventCreate(&e1));
  int tuned = 0;
  try {
    for (auto* s : b->subs) {
      const std::string key = gemm_key(s);
      if (chosen.count(key)) continue;
      auto hit = cache.find(key);
      if (hit != cache.end()) {
        chosen[key] = hit->second;
        continue;
      }
      const bool temp = !s->resident;
      if (temp) {
        const int p = static_cast<int>(std::find(b->pool.begin(), b->pool.end(), s->st) - b->pool.begin());
        subdomain_ws_alloc(s, b->pool_gwork[p], b->pool_gwork_elems);
        load_start_block<TS>(s, nullptr);
      }
      // the rotation operand: a well-scaled fixed matrix (scheduling only)
      std::vector<double> q(static_cast<size_t>(s->ns) * s->ns, 0.0);
      for (int i = 0; i < s->ns; ++i) q[static_cast<size_t>(i) * s->ns + i] = 1.0;
      XLS_HIP(hipMemcpyAsync(s->Ydev, q.data(), q.size() * 8, hipMemcpyHostToDevice, s->st));
      double best_tn = 1e30, best_nn = 1e30;
      Shape arg{0, 0, 0};
      for (int tile : {0, 1})
        for (int scale : {0, 1, 4, 8}) {
          GemmPlan g;
          g.split_scale = scale;
          g.tile_tn = tile;
          g.tile_nn = tile;
          const auto t = time_gemm_plan<TS>(s, g, e0, e1);
          if (t[0] < best_tn) {
            best_tn = t[0];
            arg[0] = scale;
            arg[1] = tile;
          }
          if (scale == 0 && t[1] < best_nn) {
            best_nn = t[1];
            arg[2] = tile;
          }
        }
      if (temp) subdomain_ws_free(s);
      chosen[key] = arg;
      ++tuned;
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (auto* s : b->subs) {
    const Shape& c = chosen[gemm_key(s)];
    s->gplan.split_scale = c[0];
    s->gplan.tile_tn = c[1];
    s->gplan.tile_nn = c[2];
  }
  return tuned;
}

template <typename TS>
int tune_batch(xls_batch_s* b, const char* cache_path, double* best_ms_out) {
  auto cache = read_cache(cache_path);
  std::map<std::string, Shape> chosen;
  std::map<std::string, double> best_ms;
  hipEvent_t e0, e1;
  XLS_HIP(hipEventCreate(&e0));
  XLS_HIP(hipEventCreate(&e1));
  int tuned = 0;
  try {
    for (auto* s : b->subs) {
      const std::string key = shape_key(s);
      if (chosen.count(key)) continue;
      auto hit = cache.find(key);
      if (hit != cache.end()) {
        chosen[key] = hit->second;
        continue;
      }
      // slot residency: a temporary working set with the start block
      const bool temp = !s->resident;
      if (temp) {
        const int p = static_cast<int>(std::find(b->pool.begin(), b->pool.end(), s->st) - b->pool.begin());
        subdomain_ws_alloc(s, b->pool_gwork[p], b->pool_gwork_elems);
        load_start_block<TS>(s, nullptr);
      }
      double best = 1e30;
      Shape arg{256, 0, 1};
      for (int nv : {1, 2})
      for (int block : {256, 512})
        for (int ty : {0, 1, 2, 4, 8, 16}) {
          StencilLaunch cfg = cfg_of<TS>(s);
          cfg.block = block;
          cfg.ty = ty;
          cfg.nv = nv;
          try {
            stencil_validate(s->n[0], s->n[1], s->n[2], s->bc == XLS_BC_PERIODIC, sizeof(TS), s->nproj(), cfg);
          } catch (const Error&) {
            continue;
          }
          const double ms = time_filter<TS>(s, cfg, e0, e1);
          if (ms < best) {
            best = ms;
            arg = {block, ty, nv};
          }
        }
      if (temp) subdomain_ws_free(s);
      chosen[key] = arg;
      best_ms[key] = best;
      ++tuned;
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (auto* s : b->subs) {  // a member whose extents do not admit its class's shape keeps its own
    const auto& c = chosen[shape_key(s)];
    (void)xls_subdomain_tune(s, s->prec, c[0], c[1], 0, c[2]);
  }
  // projection / rotation GEMM plans per (precision, N_d, ns) class
  tuned += tune_gemms<TS>(b, cache, chosen);
  for (auto& e : chosen) cache[e.first] = e.second;
  if (tuned > 0) write_cache(cache_path, cache);
  if (best_ms_out) {
    double t = 0;
    for (auto& e : best_ms) t += e.second;
    *best_ms_out = t;
  }
  for (auto& g : b->graphs) g.release();  // tile shapes changed: recapture
  b->graphs.clear();
  return tuned;
}

}  // namespace

namespace {

// The rows the occupation calls read: the whole block with the core mask
// (resident batches), or the core store with an all-ones mask (slot
// residency).  STATE when a subdomain has no block.
struct BlockView {
  const void* psi;
  int64_t nd, ld;
  const uint8_t* mask;
};

BlockView view_of(xls_batch_s* b, int i) {
  xls_subdomain_s* s = b->subs[i];
  if (!s->have_ritz) fail(XLS_ERR_STATE, "needs a completed xls_batch_chefsi");
  if (!b->slots) return BlockView{s->blk[s->cur], s->nd, s->ld, s->mask};
  const CoreStore& cs = b->core[i];
  if (cs.ncore > 0 && !cs.blk) fail(XLS_ERR_STATE, "subdomain has no stored core block");
  return BlockView{cs.blk, cs.ncore, cs.ld, b->ones};
}

// rho (2/h^3) sum_n g_n psi_n^2 over the view's rows, c_n into resid_dev
// (the handle's scratch for per-state values); returns the device rho.
double* density_rows(xls_batch_s* b, int i, const BlockView& v, double mu, double sigma, hipStream_t st) {
  xls_subdomain_s* s = b->subs[i];
  if (b->slots) {
    dfree(s->rho_dev);
    s->rho_dev = nullptr;
    s->rho_dev = dalloc<double>(static_cast<size_t>(std::max<int64_t>(1, v.nd)));
  } else if (!s->rho_dev) {
    s->rho_dev = dalloc<double>(s->nd);
  }
  XLS_HIP(hipMemcpyAsync(s->lam_dev, s->ritz.data(), s->ns * 8, hipMemcpyHostToDevice, st));
  launch_density(s->lam_dev, mu, sigma, v.mask, s->h, v.psi, s->prec == XLS_PREC_FP32, v.nd, v.ld, s->ns,
                 s->rho_dev, s->cpart, 64, s->resid_dev, s->gocc, st);
  return s->rho_dev;
}

// Shared part of both create calls; slot_budget < 0: everything resident.
xls_batch_s* batch_new(int32_t n, const xls_subdomain_desc_t* descs, int64_t slot_budget) {
  if (!descs || n < 1) fail(XLS_ERR_INVALID_ARG, "bad argument");
  for (int i = 1; i < n; ++i)
    if (descs[i].filter_prec != descs[0].filter_prec)
      fail(XLS_ERR_INVALID_ARG, "all subdomains of a batch share one filter precision");
  auto* b = new xls_batch_s();
  try {
    b->n = n;
    b->prec = descs[0].filter_prec;
    b->slots = slot_budget >= 0;
    XLS_HIP(hipStreamCreateWithFlags(&b->main, hipStreamNonBlocking));
    const int np = std::min(n, pool_streams());
    for (int p = 0; p < np; ++p) {
      hipStream_t st;
      XLS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      b->pool.push_back(st);
      hipEvent_t e;
      XLS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      b->ev_join.push_back(e);
    }
    XLS_HIP(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    XLS_HIP(hipEventCreate(&b->t0));
    XLS_HIP(hipEventCreate(&b->t1));
    b->flags = dalloc<int32_t>(n);
    b->subs.assign(n, nullptr);
    b->st.assign(n, SubState{});
    for (int i = 0; i < n; ++i) {
      xls_subdomain_desc_t d = descs[i];
      d.stream = b->pool[i % np];
      if (!b->slots) {
        const int rc = xls_subdomain_create(&d, &b->subs[i]);
        if (rc != XLS_OK) fail(rc, "subdomain " + std::to_string(i) + ": " + xls_last_error());
      } else {
        b->subs[i] = subdomain_create_tables(&d);
      }
      b->coef.push_back(dalloc<double>(3 * kMaxDegree));
    }
    if (b->slots) {
      // split-K workspace per pool stream: the largest any of its handles needs
      size_t need = 64 * 1024;
      int64_t max_core = 1;
      for (auto* s : b->subs) {
        need = std::max(need, gemm_tn_work_elems(s->ns, s->ns, s->nd));
        need = std::max(need, gemm_tn_work_elems(s->ns, s->ns, s->ns));
      }
      b->pool_gwork_elems = need;
      for (size_t p = 0; p < b->pool.size(); ++p) b->pool_gwork.push_back(dalloc<double>(need));
      b->core.resize(n);
      for (int i = 0; i < n; ++i) {
        xls_subdomain_s* s = b->subs[i];
        CoreStore& cs = b->core[i];
        for (int64_t g = 0; g < s->nd; ++g)
          if (s->tab.core_mask[g]) cs.hrows.push_back(static_cast<int32_t>(g));
        cs.ncore = static_cast<int64_t>(cs.hrows.size());
        cs.ld = (cs.ncore + 63) / 64 * 64;
        max_core = std::max(max_core, cs.ncore);
        cs.rows = dalloc<int32_t>(std::max<int64_t>(1, cs.ncore));
        if (cs.ncore > 0)
          XLS_HIP(hipMemcpy(cs.rows, cs.hrows.data(), cs.ncore * 4, hipMemcpyHostToDevice));
      }
      b->ones = dalloc<uint8_t>(max_core);
      b->ones_n = max_core;
      XLS_HIP(hipMemset(b->ones, 1, max_core));
      size_t free_b = 0, total_b = 0;
      XLS_HIP(hipMemGetInfo(&free_b, &total_b));
      b->budget = slot_budget > 0 ? slot_budget : static_cast<int64_t>(0.85 * static_cast<double>(free_b));
    }
  } catch (...) {
    delete b;
    throw;
  }
  return b;
}

}  // namespace

extern "C" {

int xls_batch_create_slots(int32_t n, const xls_subdomain_desc_t* descs, int64_t max_resident_bytes,
                           xls_batch_t* out) {
  return guarded([&]() -> int {
    if (!out || max_resident_bytes < 0) fail(XLS_ERR_INVALID_ARG, "bad argument");
    *out = batch_new(n, descs, max_resident_bytes);
    return XLS_OK;
  });
}

int xls_batch_create(int32_t n, const xls_subdomain_desc_t* descs, xls_batch_t* out) {
  return guarded([&]() -> int {
    if (!out) fail(XLS_ERR_INVALID_ARG, "bad argument");
    *out = batch_new(n, descs, -1);
    return XLS_OK;
  });
}

void xls_batch_destroy(xls_batch_t b) { delete b; }

int xls_batch_chefsi(xls_batch_t b, const xls_chefsi_params_t* per_sub, double* ritz_concat,
                     double* resid_concat, int32_t* iters, int32_t* status, int32_t use_graph) {
  return guarded([&]() -> int {
    if (!b || !per_sub || !ritz_concat || !resid_concat) fail(XLS_ERR_INVALID_ARG, "bad argument");
    if (b->prec == XLS_PREC_FP32)
      batch_chefsi<float>(b, per_sub, use_graph);
    else
      batch_chefsi<double>(b, per_sub, use_graph);
    int64_t off = 0;
    int worst = XLS_OK;
    for (int i = 0; i < b->n; ++i) {
      xls_subdomain_s* s = b->subs[i];
      std::memcpy(ritz_concat + off, s->ritz.data(), s->ns * 8);
      XLS_HIP(hipMemcpy(resid_concat + off, s->resid_dev, s->ns * 8, hipMemcpyDeviceToHost));
      off += s->ns;
      if (iters) iters[i] = b->st[i].total_iters;
      if (status) status[i] = b->st[i].status;
      if (b->st[i].status != XLS_OK) worst = b->st[i].status;
    }
    if (worst != XLS_OK && !status) fail(worst, "a subdomain of the batch failed (M_s not positive definite)");
    return XLS_OK;
  });
}

int xls_batch_density(xls_batch_t b, double mu, double sigma, double* rho_concat, double* c_concat) {
  return guarded([&]() -> int {
    if (!b || !rho_concat || !c_concat) fail(XLS_ERR_INVALID_ARG, "bad argument");
    if (!(sigma > 0) || !std::isfinite(sigma) || !std::isfinite(mu)) fail(XLS_ERR_INVALID_ARG, "bad mu/sigma");
    int64_t off_r = 0, off_c = 0;
    for (int i = 0; i < b->n; ++i) {
      xls_subdomain_s* s = b->subs[i];
      if (!b->slots) {
        const int rc = xls_subdomain_density(s, mu, sigma, rho_concat + off_r, c_concat + off_c);
        if (rc != XLS_OK) fail(rc, xls_last_error());
      } else {  // core rows only: rho is zero elsewhere
        const BlockView v = view_of(b, i);
        double* rho = density_rows(b, i, v, mu, sigma, s->st);
        std::vector<double> hr(static_cast<size_t>(std::max<int64_t>(1, v.nd)));
        XLS_HIP(hipMemcpyAsync(hr.data(), rho, v.nd * 8, hipMemcpyDeviceToHost, s->st));
        XLS_HIP(hipMemcpyAsync(c_concat + off_c, s->resid_dev, s->ns * 8, hipMemcpyDeviceToHost, s->st));
        XLS_HIP(hipStreamSynchronize(s->st));
        std::fill(rho_concat + off_r, rho_concat + off_r + s->nd, 0.0);
        for (int64_t r = 0; r < v.nd; ++r) rho_concat[off_r + b->core[i].hrows[r]] = hr[r];
      }
      off_r += s->nd;
      off_c += s->ns;
    }
    return XLS_OK;
  });
}

int xls_batch_fermi(xls_batch_t b, double sigma, double n_electrons, double* out, int32_t cap) {
  return guarded([&]() -> int {
    if (!b || !out || cap < 1) fail(XLS_ERR_INVALID_ARG, "bad argument");
    if (!(sigma > 0) || !std::isfinite(sigma) || !(n_electrons > 0) || !std::isfinite(n_electrons))
      fail(XLS_ERR_INVALID_ARG, "sigma and n_electrons must be positive and finite");
    int64_t total = 0;
    for (auto* s : b->subs) {
      if (!s->have_ritz) fail(XLS_ERR_STATE, "xls_batch_fermi needs a completed xls_batch_chefsi");
      total += s->ns;
    }
    XLS_HIP(hipStreamSynchronize(b->main));
    for (auto* s : b->subs) XLS_HIP(hipStreamSynchronize(s->st));
    if (total != b->nstates) {
      dfree(b->lam_all);
      dfree(b->c_all);
      b->lam_all = nullptr;
      b->c_all = nullptr;
      b->lam_all = dalloc<double>(total);
      b->c_all = dalloc<double>(total);
      b->nstates = total;
    }
    if (!b->fout) b->fout = dalloc<double>(8);
    b->have_fermi = false;
    int64_t off = 0;
    for (int i = 0; i < b->n; ++i) {
      xls_subdomain_s* s = b->subs[i];
      const BlockView v = view_of(b, i);
      XLS_HIP(hipMemcpyAsync(b->lam_all + off, s->ritz.data(), s->ns * 8, hipMemcpyHostToDevice, b->main));
      launch_core_weights(v.mask, v.psi, s->prec == XLS_PREC_FP32, v.nd, v.ld, s->ns, s->cpart, 64, b->c_all + off,
                          b->main);
      off += s->ns;
    }
    launch_fermi_level(b->lam_all, b->c_all, total, sigma, n_electrons, 200, b->fout, b->main);
    double h[8] = {0};
    XLS_HIP(hipMemcpyAsync(h, b->fout, 6 * 8, hipMemcpyDeviceToHost, b->main));
    XLS_HIP(hipStreamSynchronize(b->main));
    if (h[5] != 0.0) fail(XLS_ERR_INVALID_ARG, "n_electrons is outside the range the batch's states can hold");
    b->mu = h[0];
    b->sigma = sigma;
    b->have_fermi = true;
    const int k = std::min<int>(cap, 5);
    for (int i = 0; i < k; ++i) out[i] = h[i];
    return k;
  });
}

int xls_batch_assemble(xls_batch_t b, int64_t n_global, double* rho_global, int32_t nbins, const double* edges,
                       double* dos) {
  return guarded([&]() -> int {
    if (!b) fail(XLS_ERR_INVALID_ARG, "NULL batch");
    if (!b->have_fermi) fail(XLS_ERR_STATE, "xls_batch_assemble needs a completed xls_batch_fermi");
    if (nbins < 0 || (nbins > 0 && (!edges || !dos))) fail(XLS_ERR_INVALID_ARG, "bad DOS arguments");
    for (int i = 0; i < nbins; ++i)
      if (!(edges[i] < edges[i + 1])) fail(XLS_ERR_INVALID_ARG, "DOS edges must increase");
    if (rho_global) {
      if (n_global < 1) fail(XLS_ERR_INVALID_ARG, "n_global must be >= 1");
      if (b->gidx.size() != b->subs.size()) {
        b->gidx.assign(b->subs.size(), nullptr);
        b->gidx_ok.assign(b->subs.size(), 0);
      }
      for (int i = 0; i < b->n; ++i) (void)view_of(b, i);  // STATE unless every block is available
      // every core point inside the global grid, and distinct within a subdomain
      for (size_t i = 0; i < b->subs.size(); ++i) {
        auto* s = b->subs[i];
        std::vector<int64_t> core;
        core.reserve(static_cast<size_t>(s->nd));
        for (int64_t g = 0; g < s->nd; ++g)
          if (s->tab.core_mask[g]) core.push_back(s->tab.global_index[g]);
        for (int64_t v : core)
          if (v < 0 || v >= n_global) fail(XLS_ERR_INVALID_ARG, "a core point maps outside the global grid");
        if (b->gidx_ok[i] == 0) {
          std::sort(core.begin(), core.end());
          b->gidx_ok[i] = std::adjacent_find(core.begin(), core.end()) == core.end() ? 1 : -1;
        }
        if (b->gidx_ok[i] < 0) fail(XLS_ERR_INVALID_ARG, "two core points of one subdomain share a global point");
      }
      XLS_HIP(hipStreamSynchronize(b->main));
      for (auto* s : b->subs) XLS_HIP(hipStreamSynchronize(s->st));
      if (n_global != b->rho_global_n) {
        dfree(b->rho_global);
        b->rho_global = nullptr;
        b->rho_global = dalloc<double>(n_global);
        b->rho_global_n = n_global;
      }
      XLS_HIP(hipMemsetAsync(b->rho_global, 0, n_global * 8, b->main));
      for (size_t i = 0; i < b->subs.size(); ++i) {
        auto* s = b->subs[i];
        const BlockView v = view_of(b, static_cast<int>(i));
        if (!b->gidx[i]) {  // global index of every row of the view
          std::vector<int64_t> gi(static_cast<size_t>(std::max<int64_t>(1, v.nd)));
          for (int64_t r = 0; r < v.nd; ++r)
            gi[r] = s->tab.global_index[b->slots ? b->core[i].hrows[r] : r];
          b->gidx[i] = dalloc<int64_t>(gi.size());
          XLS_HIP(hipMemcpyAsync(b->gidx[i], gi.data(), v.nd * 8, hipMemcpyHostToDevice, b->main));
          XLS_HIP(hipStreamSynchronize(b->main));
        }
        double* rho = density_rows(b, static_cast<int>(i), v, b->mu, b->sigma, b->main);
        launch_scatter_core(rho, v.mask, b->gidx[i], v.nd, b->rho_global, b->main);
      }
      XLS_HIP(hipMemcpyAsync(rho_global, b->rho_global, n_global * 8, hipMemcpyDeviceToHost, b->main));
    }
    if (nbins > 0) {
      if (nbins > b->dos_cap) {
        dfree(b->dos_buf);
        b->dos_buf = nullptr;
        b->dos_buf = dalloc<double>(2 * static_cast<size_t>(nbins) + 1);
        b->dos_cap = nbins;
      }
      XLS_HIP(hipMemcpyAsync(b->dos_buf, edges, (nbins + 1) * 8, hipMemcpyHostToDevice, b->main));
      launch_dos(b->lam_all, b->c_all, b->nstates, b->dos_buf, nbins, b->dos_buf + nbins + 1, b->main);
      XLS_HIP(hipMemcpyAsync(dos, b->dos_buf + nbins + 1, nbins * 8, hipMemcpyDeviceToHost, b->main));
    }
    XLS_HIP(hipStreamSynchronize(b->main));
    return XLS_OK;
  });
}

int xls_batch_subdomain(xls_batch_t b, int32_t i, xls_subdomain_t* out) {
  return guarded([&]() -> int {
    if (!b || !out || i < 0 || i >= b->n) fail(XLS_ERR_INVALID_ARG, "bad argument");
    XLS_HIP(hipStreamSynchronize(b->main));
    *out = b->subs[i];
    return XLS_OK;
  });
}

int xls_batch_tune(xls_batch_t b, const char* cache_path, int32_t* tuned, double* best_ms) {
  return guarded([&]() -> int {
    if (!b) fail(XLS_ERR_INVALID_ARG, "bad argument");
    XLS_HIP(hipStreamSynchronize(b->main));
    const int t = b->prec == XLS_PREC_FP32 ? tune_batch<float>(b, cache_path, best_ms)
                                           : tune_batch<double>(b, cache_path, best_ms);
    if (tuned) *tuned = t;
    return XLS_OK;
  });
}

int xls_batch_stats(xls_batch_t b, double* out, int32_t cap) {
  return guarded([&]() -> int {
    if (!b || !out || cap < 1) fail(XLS_ERR_INVALID_ARG, "bad argument");
    const double v[7] = {static_cast<double>(b->iterations), static_cast<double>(b->captures),
                         static_cast<double>(b->replays), b->iter_ms, b->last_iter_ms,
                         static_cast<double>(b->peak_bytes), static_cast<double>(b->max_active)};
    const int k = std::min(cap, 7);
    for (int i = 0; i < k; ++i) out[i] = v[i];
    return k;
  });
}

}  // extern "C"
