// C ABI of the subdomain CheFSI engine: handle lifetime, argument checks,
// error mapping, and the orchestration of one CheFSI iteration (Sec. V-A.3)
// from the stage kernels.  Every numerical step runs in the HIP kernels; the
// host only computes the scalar filter coefficients and makes the
// convergence decisions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "xls_handle.h"

namespace xls {

namespace {
thread_local std::string g_last_error;
bool g_profiling = false;
bool g_graphs = true;
}  // namespace

void fail(int code, const std::string& msg) { throw Error{code, msg}; }

void check_hip(hipError_t e, const char* what, const char* file, int line) {
  if (e == hipSuccess) return;
  const int code = (e == hipErrorOutOfMemory) ? XLS_ERR_OUT_OF_MEMORY : XLS_ERR_DEVICE;
  fail(code, std::string(what) + ": " + hipGetErrorString(e) + " (" + file + ":" + std::to_string(line) + ")");
}

namespace {

template <typename T>
T* dupload(const std::vector<T>& h, hipStream_t st) {
  T* d = dalloc<T>(h.size());
  if (!h.empty()) XLS_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return d;
}


struct StageTimer {
  bool on;
  hipStream_t st;
  std::vector<hipEvent_t> ev;
  explicit StageTimer(bool enabled, hipStream_t s) : on(enabled), st(s) {}
  void mark() {
    if (!on) return;
    hipEvent_t e;
    XLS_HIP(hipEventCreate(&e));
    XLS_HIP(hipEventRecord(e, st));
    ev.push_back(e);
  }
  ~StageTimer() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
  double ms(size_t a, size_t b) const {
    float t = 0;
    if (!on || b >= ev.size()) return 0.0;
    (void)hipEventElapsedTime(&t, ev[a], ev[b]);
    return t;
  }
};

}  // namespace
}  // namespace xls

namespace xls {

void set_last_error(const std::string& m) { g_last_error = m; }
bool profiling_on() { return g_profiling; }
bool graphs_on() { return g_graphs; }

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

void require_resident(const xls_subdomain_s* s) {
  if (!s->resident)
    fail(XLS_ERR_STATE, "the subdomain has no working set (a slot-residency batch releases it between runs)");
}

void materialize_half(xls_subdomain_s* s) {
  if (!s->half_src) return;
  const uint16_t* h = s->half_src;
  s->half_src = nullptr;
  if (s->prec == XLS_PREC_FP32)
    launch_block_half<float>(B<float>(s, s->cur), s->ld, s->nd, s->ns, const_cast<uint16_t*>(h), 0, s->st);
  else
    launch_block_half<double>(B<double>(s, s->cur), s->ld, s->nd, s->ns, const_cast<uint16_t*>(h), 0, s->st);
}

bool finite_all(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// out = H y in the storage precision.
template <typename TS>
void apply_H(xls_subdomain_s* s, const TS* y, TS* out, int ncols, TS* alpha) {
  s->happly += ncols;
  const auto& op = op_of<TS>(s);
  launch_proj_forward<TS, TS>(op, y, s->ld, ncols, alpha, s->st);
  launch_stencil<TS, TS>(kApply, op, y, s->ld, ncols, alpha, out, nullptr, 1.0, 0.0, 0.0, nullptr, nullptr,
                         nullptr, s->st, cfg_of<TS>(s));
}

// Block <- p_m(H) block by the scaled three-term recurrence (the oracle's
// filter_coefficients, same scalar sequence).  With profiling on, HIP events
// bracket every fused-filter stencil launch on the handle's stream.
template <typename TS>
void filter_block(xls_subdomain_s* s, int m, double a0, double lc, double lmax) {
  const double e = (lmax - lc) / 2.0;
  const double c = (lmax + lc) / 2.0;
  const double sigma1 = e / (a0 - c);
  const double tau = 2.0 / sigma1;
  const auto& op = op_of<TS>(s);
  const auto& cfg = cfg_of<TS>(s);
  TS* alpha = static_cast<TS*>(s->alpha);
  const bool prof = profiling_on();
  s->happly += static_cast<int64_t>(m) * s->ns;
  if (prof && static_cast<int>(s->fev.size()) < 2 * m) {
    for (auto ev : s->fev) (void)hipEventDestroy(ev);
    s->fev.assign(2 * m, nullptr);
    for (auto& ev : s->fev) XLS_HIP(hipEventCreate(&ev));
  }
  int y0 = s->cur, y1 = 1 - s->cur;
  // a binary16 warm start is read as Y_0 by step 0 and as Y_{-1} by step 1
  const uint16_t* h16 = s->half_src;
  s->half_src = nullptr;
  // Y1 = (sigma1/e)(H X - c X)
  if (h16) {
    launch_proj_forward<_Float16, TS>(op, reinterpret_cast<const _Float16*>(h16), s->nd, s->ns, alpha, s->st);
    if (prof) XLS_HIP(hipEventRecord(s->fev[0], s->st));
    launch_filter_half<TS, TS>(op, nullptr, h16, s->ld, s->nd, s->ns, alpha, B<TS>(s, y1), nullptr, sigma1 / e, c,
                               0.0, s->st, cfg);
  } else {
    launch_proj_forward<TS, TS>(op, B<TS>(s, y0), s->ld, s->ns, alpha, s->st);
    if (prof) XLS_HIP(hipEventRecord(s->fev[0], s->st));
    launch_stencil<TS, TS>(kFilter, op, B<TS>(s, y0), s->ld, s->ns, alpha, B<TS>(s, y1), nullptr, sigma1 / e,
                           c, 0.0, nullptr, nullptr, nullptr, s->st, cfg);
  }
  if (prof) XLS_HIP(hipEventRecord(s->fev[1], s->st));
  s->filter_launches++;
  double sig = sigma1;
  for (int k = 1; k < m; ++k) {
    const double signew = 1.0 / (tau - sig);
    // Y_{k+1} overwrites Y_{k-1} in place (step 1 of a binary16 warm start
    // reads Y_0 from the half buffer and writes the other block)
    launch_proj_forward<TS, TS>(op, B<TS>(s, y1), s->ld, s->ns, alpha, s->st);
    if (prof) XLS_HIP(hipEventRecord(s->fev[2 * k], s->st));
    if (k == 1 && h16)
      launch_filter_half<TS, TS>(op, B<TS>(s, y1), nullptr, s->ld, s->nd, s->ns, alpha, B<TS>(s, y0), h16,
                                 2.0 * signew / e, c, sig * signew, s->st, cfg);
    else
      launch_stencil<TS, TS>(kFilter, op, B<TS>(s, y1), s->ld, s->ns, alpha, B<TS>(s, y0), B<TS>(s, y0),
                             2.0 * signew / e, c, sig * signew, nullptr, nullptr, nullptr, s->st, cfg);
    if (prof) XLS_HIP(hipEventRecord(s->fev[2 * k + 1], s->st));
    s->filter_launches++;
    sig = signew;
    std::swap(y0, y1);
  }
  s->cur = y1;
  if (prof) {
    XLS_HIP(hipEventSynchronize(s->fev[2 * m - 1]));
    for (int k = 0; k < m; ++k) {
      float t = 0;
      XLS_HIP(hipEventElapsedTime(&t, s->fev[2 * k], s->fev[2 * k + 1]));
      s->filter_kernel_ms += t;
    }
  }
}

// M = B^T B and Hs = B^T H B (upper block triangles, Hs exactly symmetric) of
// the current block (W = H B in the other buffer).
template <typename TS>
void project_block(xls_subdomain_s* s, int gprec) {
  TS* Bc = B<TS>(s, s->cur);
  TS* W = B<TS>(s, 1 - s->cur);
  apply_H<TS>(s, Bc, W, s->ns, static_cast<TS*>(s->alpha));
  gemm_tn<TS>(gprec, Bc, s->ld, Bc, s->ld, s->ns, s->ns, s->nd, s->Mdev, s->ns, 1, 0, s->gwork,
              s->gwork_elems, s->st, s->gplan);
  gemm_tn<TS>(gprec, Bc, s->ld, W, s->ld, s->ns, s->ns, s->nd, s->Hsdev, s->ns, 1, 1, s->gwork,
              s->gwork_elems, s->st, s->gplan);
}

template <typename TS>
void rotate_block(xls_subdomain_s* s, int gprec, const double* Ydev) {
  TS* Bc = B<TS>(s, s->cur);
  TS* O = B<TS>(s, 1 - s->cur);
  gemm_nn<TS>(gprec, Bc, s->ld, Ydev, s->ns, static_cast<int>(s->nd), s->ns, s->ns, O, s->ld, s->bwork, s->st, s->gplan);
  s->cur = 1 - s->cur;
}

// FP64 residual norms of the current block against lam (device), and the
// columns' FP64 Rayleigh quotients when rq_dev is not null.
template <typename TS>
void residual_block(xls_subdomain_s* s, const double* lam_dev, double* resid_dev, double* rq_dev) {
  s->happly += s->ns;
  TS* Bc = B<TS>(s, s->cur);
  launch_proj_forward<TS, double>(s->op64, Bc, s->ld, s->ns, s->alpha64, s->st);
  StencilLaunch cfg = s->cfg64;
  launch_stencil<TS, double>(kResid, s->op64, Bc, s->ld, s->ns, s->alpha64, nullptr, nullptr, 1.0, 0.0, 0.0,
                             lam_dev, s->partial, resid_dev, s->st, cfg, rq_dev);
}

int lanczos_steps(const xls_subdomain_s* s, int k) {
  k = k > 0 ? std::min(k, kMaxLanczos) : 20;
  return static_cast<int>(std::min<int64_t>(k, s->nd));
}

double gated_max(const double* r, int gate) {
  double mx = 0.0;
  for (int k = 0; k < gate; ++k) {
    if (std::isnan(r[k])) return r[k];
    mx = std::max(mx, r[k]);
  }
  return mx;
}

template <typename TS>
void lanczos_run(xls_subdomain_s* s, int k) {
  k = lanczos_steps(s, k);
  if (!s->lz || s->lz_cols < k + 2) {
    dfree(s->lz);
    s->lz = nullptr;
    s->lz = dalloc<TS>(static_cast<size_t>(s->ld) * (k + 2));
    s->lz_cols = k + 2;
  }
  const int64_t ld = s->ld;
  TS* V = static_cast<TS*>(s->lz);
  TS* w = V + ld * (k + 1);
  double* al = s->vsmall;         // [k]
  double* be = s->vsmall + 64;    // [k]
  double* coef = s->vsmall + 128; // [k]
  double* nrm = s->vsmall + 192;
  double* part = s->vsmall + 256;  // [256]
  const int nblocks = 256;
  // v_1 = v0 / ||v0||
  if (s->lanczos_v0.empty()) {  // column 0 of the generated start block
    launch_philox_block<TS>(w, ld, s->nd, 1, s->x0_seed, s->st);
  } else {
    std::vector<TS> hv(s->nd);
    for (int64_t i = 0; i < s->nd; ++i) hv[i] = static_cast<TS>(s->lanczos_v0[i]);
    XLS_HIP(hipMemcpyAsync(w, hv.data(), s->nd * sizeof(TS), hipMemcpyHostToDevice, s->st));
    XLS_HIP(hipStreamSynchronize(s->st));  // hv is released at scope exit
  }
  launch_dot<TS>(w, w, s->nd, part, nblocks, nrm, 1, s->st);
  launch_scale_to<TS>(V, w, nrm, s->nd, s->st);
  TS* alph = static_cast<TS*>(s->alpha);
  std::vector<double> ha, hb;
  int keff = k;
  for (int j = 0; j < k; ++j) {
    TS* vj = V + j * ld;
    apply_H<TS>(s, vj, w, 1, alph);
    launch_dot<TS>(vj, w, s->nd, part, nblocks, al + j, 0, s->st);
    launch_lanczos_update<TS>(w, vj, j > 0 ? vj - ld : nullptr, al + j, j > 0 ? be + j - 1 : nullptr, s->nd,
                              s->st);
    // coef = V_{0..j}^T w (full reorthogonalisation): a skinny product
    const int rb = static_cast<int>(std::max<size_t>(1, std::min<size_t>(256, s->gwork_elems / (j + 1))));
    launch_multi_dot<TS>(V, ld, j + 1, w, s->nd, s->gwork, rb, coef, s->st);
    launch_reorth<TS>(w, V, ld, coef, j + 1, s->nd, s->st);
    launch_dot<TS>(w, w, s->nd, part, nblocks, be + j, 1, s->st);
    double ab[2];
    XLS_HIP(hipMemcpyAsync(&ab[0], al + j, 8, hipMemcpyDeviceToHost, s->st));
    XLS_HIP(hipMemcpyAsync(&ab[1], be + j, 8, hipMemcpyDeviceToHost, s->st));
    XLS_HIP(hipStreamSynchronize(s->st));
    ha.push_back(ab[0]);
    hb.push_back(ab[1]);
    double scale = 0;
    for (double x : ha) scale = std::max(scale, std::fabs(x));
    for (double x : hb) scale = std::max(scale, x);
    if (ab[1] <= 1e-12 * scale) {  // invariant Krylov space
      keff = j + 1;
      break;
    }
    launch_scale_to<TS>(V + (j + 1) * ld, w, be + j, s->nd, s->st);
  }
  launch_tridiag_extremes(al, be, keff, nrm, s->st);
  double ext[2];
  XLS_HIP(hipMemcpyAsync(ext, nrm, 16, hipMemcpyDeviceToHost, s->st));
  XLS_HIP(hipStreamSynchronize(s->st));
  s->lz_lo = ext[0];
  s->lz_up = ext[1] + std::fabs(hb[keff - 1]);
  s->lz_k = k;
  s->have_lanczos = true;
}


#define XLS_INST_STAGES(TS)                                                          \
  template void apply_H<TS>(xls_subdomain_s*, const TS*, TS*, int, TS*);             \
  template void rotate_block<TS>(xls_subdomain_s*, int, const double*);              \
  template void residual_block<TS>(xls_subdomain_s*, const double*, double*, double*);        \
  template void lanczos_run<TS>(xls_subdomain_s*, int);                              \
  template void filter_block<TS>(xls_subdomain_s*, int, double, double, double);
XLS_INST_STAGES(float)
XLS_INST_STAGES(double)

}  // namespace xls

using namespace xls;

namespace {

void validate_desc(const xls_subdomain_desc_t* d) {
  if (!d) fail(XLS_ERR_INVALID_ARG, "desc is NULL");
  for (int a = 0; a < 3; ++a)
    if (d->n[a] < 1) fail(XLS_ERR_INVALID_ARG, "grid size must be >= 1");
  const int64_t nd = static_cast<int64_t>(d->n[0]) * d->n[1] * d->n[2];
  if (nd >= (int64_t(1) << 31)) fail(XLS_ERR_INVALID_ARG, "N_d must be < 2^31");
  if (!(d->h > 0) || !std::isfinite(d->h)) fail(XLS_ERR_INVALID_ARG, "h must be finite and > 0");
  if (d->bc != XLS_BC_PERIODIC && d->bc != XLS_BC_DIRICHLET0) fail(XLS_ERR_INVALID_ARG, "unknown bc");
  if (d->fd_n0 != kRadius) fail(XLS_ERR_INVALID_ARG, "fd_n0 must be 6");
  if (d->n[0] > 1024) fail(XLS_ERR_INVALID_ARG, "n[0] must be <= 1024");
  if (!d->v_eff || !finite_all(d->v_eff, nd)) fail(XLS_ERR_INVALID_ARG, "v_eff NULL or not finite");
  if (!finite_all(d->origin, 3)) fail(XLS_ERR_INVALID_ARG, "origin not finite");
  if (d->n_atoms < 0) fail(XLS_ERR_INVALID_ARG, "n_atoms < 0");
  if (d->n_atoms > 0 && (!d->atom_xyz || !d->proj)) fail(XLS_ERR_INVALID_ARG, "atoms NULL");
  if (d->n_atoms > 0 && !finite_all(d->atom_xyz, 3 * static_cast<int64_t>(d->n_atoms)))
    fail(XLS_ERR_INVALID_ARG, "atom positions not finite");
  for (int a = 0; a < d->n_atoms; ++a) {
    const xls_projset_t& p = d->proj[a];
    if (!(p.rc > 0) || !(p.gauss_width > 0) || !std::isfinite(p.rc) || !std::isfinite(p.gauss_width) ||
        !finite_all(p.gamma, 4))
      fail(XLS_ERR_INVALID_ARG, "bad projector set");
  }
  for (int a = 0; a < 3; ++a) {
    if (d->core_lo[a] < 0 || d->core_hi[a] > d->n[a] || d->core_lo[a] > d->core_hi[a])
      fail(XLS_ERR_INVALID_ARG, "core box outside the grid");
    if (d->global_n[a] < 1) fail(XLS_ERR_INVALID_ARG, "global_n must be >= 1");
  }
  if (d->ns < 1 || d->ns > nd) fail(XLS_ERR_INVALID_ARG, "ns must be in [1, N_d]");
  if (d->x0 && !finite_all(d->x0, nd * d->ns)) fail(XLS_ERR_INVALID_ARG, "x0 not finite");
  if (d->lanczos_v0 && !finite_all(d->lanczos_v0, nd)) fail(XLS_ERR_INVALID_ARG, "lanczos_v0 not finite");
  if (d->filter_prec != XLS_PREC_FP64 && d->filter_prec != XLS_PREC_FP32)
    fail(XLS_ERR_INVALID_ARG, "filter_prec must be FP64 or FP32");
}

// Dense stage of one CheFSI iteration without host synchronisation (the
// caller checks the positive-definiteness flag after its own sync).  The
// first call runs eagerly, the second is captured into a hipGraph, and later
// calls replay it: every buffer and the launch sequence are fixed per handle.
void dense_stage(xls_subdomain_s* s) {
  if (graphs_on() && !s->dexec && s->dwarm) {
    XLS_HIP(hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal));
    try {
      (void)dense_geneig(s->dw, s->Hsdev, s->Mdev, s->Ydev, s->st, false);
    } catch (...) {
      hipGraph_t dead = nullptr;
      (void)hipStreamEndCapture(s->st, &dead);
      if (dead) (void)hipGraphDestroy(dead);
      throw;
    }
    XLS_HIP(hipStreamEndCapture(s->st, &s->dgraph));
    XLS_HIP(hipGraphInstantiate(&s->dexec, s->dgraph, nullptr, nullptr, 0));
  }
  if (graphs_on() && s->dexec) {
    XLS_HIP(hipGraphLaunch(s->dexec, s->st));
  } else {
    (void)dense_geneig(s->dw, s->Hsdev, s->Mdev, s->Ydev, s->st, false);
    s->dwarm = true;
  }
}

// Up to max_iter CheFSI iterations from the handle's current block with
// first-iteration bounds (a0, lc, lmax); total is advanced by the iterations
// run (also when an iteration throws NOT_SPD).
template <typename TS>
void chefsi_loop(xls_subdomain_s* s, const xls_chefsi_params_t* p, int gprec, int gate, int degree, double a0,
                 double lc, double lmax, std::vector<double>& hl, std::vector<double>& hr, int& total) {
  const int ns = s->ns;
  double prev_resid = HUGE_VAL;
  // Reported Ritz values: the projected eigenvalues when the block and the
  // projection are FP64; otherwise the FP64 Rayleigh quotients of the rotated
  // columns from the residual sweep (second order in the vectors' error, so
  // free of the GEMMs' rounding).  The next filter's bounds always come from
  // the projected eigenvalues.
  const bool use_rq = !std::is_same<TS, double>::value || gprec != XLS_PREC_FP64;
  std::vector<double> hq(ns);
  for (int it = 0; it < p->max_iter;) {
    StageTimer tm(profiling_on(), s->st);
    tm.mark();
    filter_block<TS>(s, degree, a0, lc, lmax);
    tm.mark();
    const int pprec = polish_prec(gprec, prev_resid);
    {
      TS* Bc = B<TS>(s, s->cur);
      TS* W = B<TS>(s, 1 - s->cur);
      apply_H<TS>(s, Bc, W, s->ns, static_cast<TS*>(s->alpha));
      tm.mark();
      gemm_tn<TS>(pprec, Bc, s->ld, Bc, s->ld, ns, ns, s->nd, s->Mdev, ns, 1, 0, s->gwork, s->gwork_elems,
                  s->st, s->gplan);
      gemm_tn<TS>(pprec, Bc, s->ld, W, s->ld, ns, ns, s->nd, s->Hsdev, ns, 1, 1, s->gwork, s->gwork_elems,
                  s->st, s->gplan);
    }
    tm.mark();
    dense_stage(s);
    XLS_HIP(hipMemcpyAsync(s->lam_dev, s->dw.lam(), ns * 8, hipMemcpyDeviceToDevice, s->st));
    tm.mark();
    rotate_block<TS>(s, pprec, s->Ydev);
    tm.mark();
    residual_block<TS>(s, s->lam_dev, s->resid_dev, use_rq ? s->rq_dev : nullptr);
    tm.mark();
    int32_t spd_flag = 0;
    XLS_HIP(hipMemcpyAsync(hl.data(), s->lam_dev, ns * 8, hipMemcpyDeviceToHost, s->st));
    if (use_rq) XLS_HIP(hipMemcpyAsync(hq.data(), s->rq_dev, ns * 8, hipMemcpyDeviceToHost, s->st));
    XLS_HIP(hipMemcpyAsync(hr.data(), s->resid_dev, ns * 8, hipMemcpyDeviceToHost, s->st));
    XLS_HIP(hipMemcpyAsync(&spd_flag, s->dw.flag, 4, hipMemcpyDeviceToHost, s->st));
    XLS_HIP(hipStreamSynchronize(s->st));
    if (spd_flag) {
      ++total;
      fail(XLS_ERR_NOT_SPD, "overlap matrix M_s is not positive definite");
    }
    if (profiling_on()) {
      for (int k = 0; k < 6; ++k) s->stage_ms[k] += tm.ms(k, k + 1);
      s->stage_ms[6] += tm.ms(0, 6);
    }
    ++it;
    ++total;
    s->ritz = use_rq ? hq : hl;
    s->have_ritz = true;
    a0 = hl[0];
    lc = hl[ns - 1];
    const double mx = gated_max(hr.data(), gate);
    prev_resid = mx;
    if (!(a0 < lc && lc < lmax)) break;  // degenerate bounds: stop with what we have
    if (p->resid_tol > 0 && mx <= p->resid_tol) break;
  }
}

template <typename TS>
void lanczos_first_bounds(xls_subdomain_s* s, const xls_chefsi_params_t* p, double& a0, double& lc,
                          double& lmax) {
  const int k = lanczos_steps(s, p->lanczos_k);
  if (!s->have_lanczos || s->lz_k != k) lanczos_run<TS>(s, k);
  a0 = s->lz_lo;
  lmax = s->lz_up;
  lc = a0 + 0.1 * (lmax - a0);
}

template <typename TS>
int chefsi_impl(xls_subdomain_s* s, const xls_chefsi_params_t* p, double* ritz, double* resid,
                int32_t* iters_done) {
  if (p->degree < 1 || p->max_iter < 1) fail(XLS_ERR_INVALID_ARG, "degree and max_iter must be >= 1");
  if (p->lanczos_k > kMaxLanczos) fail(XLS_ERR_INVALID_ARG, "lanczos_k must be <= 60");
  if (p->bounds_mode == XLS_BOUNDS_LEARNED && (!(p->fallback_tol >= 0) || p->fallback_degree > 4096))
    fail(XLS_ERR_INVALID_ARG, "fallback_tol must be >= 0");
  const int gprec = p->gemm_prec;
  if (gprec < XLS_PREC_FP64 || gprec > XLS_PREC_BF16X3) fail(XLS_ERR_INVALID_ARG, "bad gemm_prec");
  if (std::is_same<TS, double>::value && gprec != XLS_PREC_FP64)
    fail(XLS_ERR_INVALID_ARG, "FP64 handles run FP64 GEMMs");
  const int ns = s->ns;
  const int gate = p->n_gate > 0 ? std::min(p->n_gate, ns) : std::max(1, static_cast<int>(std::floor(ns / 1.1 + 1e-9)));
  s->happly = 0;
  s->last_fallback = 0;
  s->last_iters = 0;
  double a0, lc, lmax;
  const bool learned = p->bounds_mode == XLS_BOUNDS_LEARNED;
  if (p->bounds_mode == XLS_BOUNDS_GIVEN) {
    a0 = p->lam_lo;
    lc = p->lam_cut;
    lmax = p->lam_max;
  } else if (p->bounds_mode == XLS_BOUNDS_LANCZOS) {
    lanczos_first_bounds<TS>(s, p, a0, lc, lmax);
  } else if (learned) {
    a0 = std::min(s->a0_bound, p->lam_cut - 1e-3 * std::fabs(p->lam_max - p->lam_cut));
    lmax = p->lam_max;
    lc = p->lam_cut;
  } else {
    fail(XLS_ERR_INVALID_ARG, "unknown bounds_mode");
  }
  if (!(a0 < lc && lc < lmax) || !std::isfinite(a0) || !std::isfinite(lmax))
    fail(XLS_ERR_INVALID_ARG, "bounds must satisfy a0 < lam_cut < lam_max");
  const bool fallback = learned && p->fallback_tol > 0;
  if (fallback) materialize_half(s);  // the backup holds the widened start block
  const int cur0 = s->cur;
  const size_t bbytes = static_cast<size_t>(s->ld) * ns * sizeof(TS);
  if (fallback) {
    if (!s->backup) s->backup = dalloc<TS>(static_cast<size_t>(s->ld) * ns);
    XLS_HIP(hipMemcpyAsync(s->backup, B<TS>(s, cur0), bbytes, hipMemcpyDeviceToDevice, s->st));
  }
  std::vector<double> hl(ns), hr(ns);
  s->stage_ms.assign(8, 0.0);
  s->filter_launches = 0;
  s->filter_kernel_ms = 0.0;
  int it = 0;
  bool miss = false;
  try {
    chefsi_loop<TS>(s, p, gprec, gate, p->degree, a0, lc, lmax, hl, hr, it);
  } catch (const Error& e) {
    // predicted bounds that miss the top of the spectrum amplify it until
    // M_s is numerically singular: that is a miss of the learned bounds,
    // not a failure of the call, when the fallback is on
    if (!fallback || e.code != XLS_ERR_NOT_SPD) throw;
    miss = true;
  }
  if (fallback && (miss || !(gated_max(hr.data(), gate) <= p->fallback_tol))) {
    XLS_HIP(hipMemcpyAsync(B<TS>(s, cur0), s->backup, bbytes, hipMemcpyDeviceToDevice, s->st));
    s->cur = cur0;
    lanczos_first_bounds<TS>(s, p, a0, lc, lmax);
    const int deg = p->fallback_degree > 0 ? p->fallback_degree : p->degree;
    chefsi_loop<TS>(s, p, gprec, gate, deg, a0, lc, lmax, hl, hr, it);
    s->last_fallback = 1;
  }
  s->last_iters = it;
  std::memcpy(ritz, s->ritz.data(), ns * 8);
  std::memcpy(resid, hr.data(), ns * 8);
  if (iters_done) *iters_done = it;
  return XLS_OK;
}

// Host column-major N_d x ncols (FP64) <-> device block with leading dimension ld.
template <typename TS>
void upload_block(xls_subdomain_s* s, const double* X, void* dst, int ncols) {
  const int64_t n = s->nd * ncols;
  const size_t es = sizeof(TS);
  if (std::is_same<TS, double>::value) {
    XLS_HIP(hipMemcpy2DAsync(dst, s->ld * es, X, s->nd * es, s->nd * es, ncols, hipMemcpyHostToDevice, s->st));
    XLS_HIP(hipStreamSynchronize(s->st));
  } else {
    std::vector<float> tmp(n);
    for (int64_t i = 0; i < n; ++i) tmp[i] = static_cast<float>(X[i]);
    XLS_HIP(hipMemcpy2DAsync(dst, s->ld * es, tmp.data(), s->nd * es, s->nd * es, ncols, hipMemcpyHostToDevice,
                             s->st));
    XLS_HIP(hipStreamSynchronize(s->st));
  }
}

template <typename TS>
void download_block(xls_subdomain_s* s, const void* src, double* X, int ncols) {
  const int64_t n = s->nd * ncols;
  const size_t es = sizeof(TS);
  if (std::is_same<TS, double>::value) {
    XLS_HIP(hipMemcpy2DAsync(X, s->nd * es, src, s->ld * es, s->nd * es, ncols, hipMemcpyDeviceToHost, s->st));
    XLS_HIP(hipStreamSynchronize(s->st));
  } else {
    std::vector<float> tmp(n);
    XLS_HIP(hipMemcpy2DAsync(tmp.data(), s->nd * es, src, s->ld * es, s->nd * es, ncols, hipMemcpyDeviceToHost,
                             s->st));
    XLS_HIP(hipStreamSynchronize(s->st));
    for (int64_t i = 0; i < n; ++i) X[i] = tmp[i];
  }
}

template <typename F>
auto by_prec(xls_subdomain_s* s, F&& f) {
  if (s->prec == XLS_PREC_FP32) return f(float{});
  return f(double{});
}

}  // namespace

namespace xls {
// Throws INVALID_ARG unless [p, p + bytes) lies inside one device allocation.
void check_device_range(const void* p, size_t bytes) {
  hipPointerAttribute_t at{};
  const hipError_t e = hipPointerGetAttributes(&at, p);
  (void)hipGetLastError();  // a host pointer leaves an error that later launch checks must not see
  if (e != hipSuccess || at.type != hipMemoryTypeDevice) fail(XLS_ERR_INVALID_ARG, "pointer is not device memory");
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  const hipError_t e2 = hipMemGetAddressRange(&base, &size, const_cast<void*>(p));
  (void)hipGetLastError();
  if (e2 != hipSuccess) fail(XLS_ERR_INVALID_ARG, "device allocation not found");
  const char* b = static_cast<const char*>(base);
  const char* q = static_cast<const char*>(p);
  if (q < b || q + bytes > b + size) fail(XLS_ERR_INVALID_ARG, "device buffer too small");
}
}  // namespace xls

namespace xls {

void subdomain_tables(xls_subdomain_s* s, const xls_subdomain_desc_t* d, bool keep_x0) {
  for (int a = 0; a < 3; ++a) {
    s->n[a] = d->n[a];
    s->core_lo[a] = d->core_lo[a];
    s->core_hi[a] = d->core_hi[a];
  }
  s->h = d->h;
  s->bc = d->bc;
  s->prec = d->filter_prec;
  s->ns = d->ns;
  s->nd = static_cast<int64_t>(d->n[0]) * d->n[1] * d->n[2];
  s->ld = (s->nd + 63) / 64 * 64;  // 256-byte aligned columns (vector loads, GEMM tiles)
  if (d->stream) {
    s->st = static_cast<hipStream_t>(d->stream);
  } else {
    XLS_HIP(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking));
    s->own_stream = true;
  }
  build_setup(*d, s->tab);
  {  // lambda_1 >= min V + sum of negative projector coefficients (-1/2 Lap >= 0)
    double vmin = d->v_eff[0];
    for (int64_t i = 1; i < s->nd; ++i) vmin = std::min(vmin, d->v_eff[i]);
    double neg = 0.0;
    for (int a = 0; a < d->n_atoms; ++a)
      for (int l = 0; l < 4; ++l) neg += std::min(0.0, d->proj[a].gamma[l]);
    s->a0_bound = vmin + neg;
  }
  s->n_atoms = d->n_atoms;
  const int64_t nd = s->nd;
  // operator tables
  std::vector<double> v(d->v_eff, d->v_eff + nd);
  s->v64 = dupload(v, s->st);
  std::vector<float> v32(v.begin(), v.end());
  s->v32 = dupload(v32, s->st);
  s->val64 = dupload(s->tab.sup_val, s->st);
  std::vector<float> val32(s->tab.sup_val.begin(), s->tab.sup_val.end());
  s->val32 = dupload(val32, s->st);
  s->rev_pk = dupload(s->tab.rev_pk, s->st);
  s->rev_aoff = dupload(s->tab.rev_aoff, s->st);
  s->rev_val64 = dupload(s->tab.rev_val, s->st);
  std::vector<float> rv32(s->tab.rev_val.begin(), s->tab.rev_val.end());
  s->rev_val32 = dupload(rv32, s->st);
  s->sup_off = dupload(s->tab.sup_off, s->st);
  s->sup_idx = dupload(s->tab.sup_idx, s->st);
  s->gamma = dupload(s->tab.gamma, s->st);
  s->mask = dupload(s->tab.core_mask, s->st);
  auto fill_op = [&](auto& op, auto* vv, auto* val, auto* rval) {
    op.v = vv;
    op.slot_val = val;
    op.rev_pk = s->rev_pk;
    op.rev_val = rval;
    op.rev_aoff = s->rev_aoff;
    op.nent = static_cast<int64_t>(s->tab.rev_slot.size());
    op.sup_off = s->sup_off;
    op.sup_idx = s->sup_idx;
    op.gamma = s->gamma;
    op.n_atoms = s->n_atoms;
    op.nx = s->n[0];
    op.ny = s->n[1];
    op.nz = s->n[2];
    op.periodic = s->bc == XLS_BC_PERIODIC;
    op.h = s->h;
  };
  fill_op(s->op64, s->v64, s->val64, s->rev_val64);
  fill_op(s->op32, s->v32, s->val32, s->rev_val32);
  s->cfg64.block = 0;  // 256 threads unless the tile's halo needs 512
  s->cfg32.block = 0;
  stencil_validate(s->n[0], s->n[1], s->n[2], s->bc == XLS_BC_PERIODIC, 8, s->nproj(), s->cfg64);
  stencil_validate(s->n[0], s->n[1], s->n[2], s->bc == XLS_BC_PERIODIC, 4, s->nproj(), s->cfg32);
  for (int a = 0; a < 3; ++a) {
    s->origin[a] = d->origin[a];
    s->global_offset[a] = d->global_offset[a];
    s->global_n[a] = d->global_n[a];
  }
  if (d->n_atoms > 0) {
    s->atom_xyz.assign(d->atom_xyz, d->atom_xyz + 3 * static_cast<size_t>(d->n_atoms));
    s->proj.assign(d->proj, d->proj + d->n_atoms);
  }
  s->atom_core.assign(d->n_atoms, 0);
  for (int a = 0; a < d->n_atoms; ++a) {  // core_lo h <= X - origin < core_hi h on every axis
    bool in = true;
    for (int k = 0; k < 3; ++k) {
      const double x = d->atom_xyz[3 * a + k] - d->origin[k];
      in = in && d->core_lo[k] * d->h <= x && x < d->core_hi[k] * d->h;
    }
    s->atom_core[a] = in ? 1 : 0;
  }
  // small per-state buffers (kept for the handle's lifetime)
  s->lam_dev = dalloc<double>(s->ns);
  s->resid_dev = dalloc<double>(s->ns);
  s->rq_dev = dalloc<double>(s->ns);
  s->vsmall = dalloc<double>(1024);
  s->cpart = dalloc<double>(static_cast<size_t>(s->ns) * 64);
  s->gocc = dalloc<double>(s->ns);
  // start block source and Lanczos vector
  s->x0_seed = d->x0_seed;
  s->x0_gen = d->x0 == nullptr;
  if (keep_x0 && d->x0) s->x0_host.assign(d->x0, d->x0 + nd * s->ns);
  if (d->lanczos_v0)
    s->lanczos_v0.assign(d->lanczos_v0, d->lanczos_v0 + nd);
  else if (d->x0)
    s->lanczos_v0.assign(d->x0, d->x0 + nd);
  else
    s->lanczos_v0.clear();  // column 0 of the generated start block
}

xls_subdomain_s* subdomain_create_tables(const xls_subdomain_desc_t* d) {
  validate_desc(d);
  auto* s = new xls_subdomain_s();
  try {
    subdomain_tables(s, d, true);
    XLS_HIP(hipStreamSynchronize(s->st));
  } catch (...) {
    delete s;
    throw;
  }
  return s;
}

size_t subdomain_ws_bytes(const xls_subdomain_s* s, bool shared_gemm_work) {
  const size_t es = s->esize();
  const size_t bl = static_cast<size_t>(s->ld) * s->ns;
  const size_t na = static_cast<size_t>(std::max(1, s->nproj())) * std::max(s->ns, 1);
  const size_t nn = static_cast<size_t>(s->ns) * s->ns;
  size_t b = 2 * bl * es + na * (es + 8);
  b += std::max(stencil_partial_elems(s->op64, s->ns, s->cfg64), static_cast<size_t>(s->ns) * 64) * 8;
  b += 3 * nn * 8 + 2 * nn_work_doubles(s->ns, s->ns) * 4;
  b += dense_bytes(s->ns, !shared_gemm_work);
  if (!shared_gemm_work) b += std::max(gemm_tn_work_elems(s->ns, s->ns, s->nd), static_cast<size_t>(64) * 1024) * 8;
  return b;
}

void subdomain_ws_alloc(xls_subdomain_s* s, double* shared_gwork, size_t shared_elems) {
  const size_t es = s->esize();
  const size_t bl = static_cast<size_t>(s->ld) * s->ns;
  s->blk[0] = es == 4 ? static_cast<void*>(dalloc<float>(bl)) : static_cast<void*>(dalloc<double>(bl));
  s->blk[1] = es == 4 ? static_cast<void*>(dalloc<float>(bl)) : static_cast<void*>(dalloc<double>(bl));
  const size_t na = static_cast<size_t>(std::max(1, s->nproj())) * std::max(s->ns, 1);
  s->alpha = es == 4 ? static_cast<void*>(dalloc<float>(na)) : static_cast<void*>(dalloc<double>(na));
  s->alpha64 = dalloc<double>(na);
  s->partial_elems = std::max(stencil_partial_elems(s->op64, s->ns, s->cfg64), static_cast<size_t>(s->ns) * 64);
  s->partial = dalloc<double>(s->partial_elems);
  const size_t nn = static_cast<size_t>(s->ns) * s->ns;
  s->Mdev = dalloc<double>(nn);
  s->Hsdev = dalloc<double>(nn);
  s->Ydev = dalloc<double>(nn);
  s->bwork = dalloc<float>(2 * nn_work_doubles(s->ns, s->ns));
  if (shared_gwork) {
    s->gwork = shared_gwork;
    s->gwork_elems = shared_elems;
    s->own_gwork = false;
  } else {
    s->gwork_elems = std::max(gemm_tn_work_elems(s->ns, s->ns, s->nd), static_cast<size_t>(64) * 1024);
    s->gwork = dalloc<double>(s->gwork_elems);
    s->own_gwork = true;
  }
  dense_alloc(s->dw, s->ns, shared_gwork, shared_elems);
  s->resident = true;
}

void subdomain_ws_free(xls_subdomain_s* s) {
  (void)hipStreamSynchronize(s->st);
  if (s->dexec) (void)hipGraphExecDestroy(s->dexec);
  if (s->dgraph) (void)hipGraphDestroy(s->dgraph);
  s->dexec = nullptr;
  s->dgraph = nullptr;
  s->dwarm = false;
  void* ps[] = {s->blk[0], s->blk[1], s->alpha, s->alpha64, s->partial, s->Mdev, s->Hsdev, s->Ydev,
                s->bwork, s->lz, s->backup, s->rho_dev};
  for (void* p : ps) dfree(p);
  if (s->own_gwork) dfree(s->gwork);
  s->blk[0] = s->blk[1] = nullptr;
  s->alpha = s->backup = s->lz = nullptr;
  s->alpha64 = s->partial = s->Mdev = s->Hsdev = s->Ydev = s->gwork = s->rho_dev = nullptr;
  s->bwork = nullptr;
  s->lz_cols = 0;
  dense_free(s->dw);
  s->resident = false;
}

template <typename TS>
void load_start_block(xls_subdomain_s* s, const double* x0) {
  if (x0)
    upload_block<TS>(s, x0, s->blk[0], s->ns);
  else if (!s->x0_host.empty())
    upload_block<TS>(s, s->x0_host.data(), s->blk[0], s->ns);
  else
    launch_philox_block<TS>(B<TS>(s, 0), s->ld, s->nd, s->ns, s->x0_seed, s->st);
  s->cur = 0;
  s->have_ritz = false;
}
template void load_start_block<float>(xls_subdomain_s*, const double*);
template void load_start_block<double>(xls_subdomain_s*, const double*);

}  // namespace xls

extern "C" {

const char* xls_last_error(void) { return g_last_error.c_str(); }

int xls_set_graphs(int32_t on) {
  g_graphs = on != 0;
  return XLS_OK;
}

int xls_set_profiling(int32_t on) {
  g_profiling = on != 0;
  return XLS_OK;
}

int xls_subdomain_create(const xls_subdomain_desc_t* d, xls_subdomain_t* out) {
  return guarded([&]() -> int {
    if (!out) fail(XLS_ERR_INVALID_ARG, "out is NULL");
    validate_desc(d);
    auto* s = new xls_subdomain_s();
    try {
      subdomain_tables(s, d, false);
      subdomain_ws_alloc(s, nullptr, 0);
      by_prec(s, [&](auto tag) {
        load_start_block<decltype(tag)>(s, d->x0);
        return 0;
      });
      XLS_HIP(hipStreamSynchronize(s->st));
    } catch (...) {
      delete s;
      throw;
    }
    *out = s;
    return XLS_OK;
  });
}

void xls_subdomain_destroy(xls_subdomain_t s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->st);
  delete s;
}

int xls_chefsi_step(xls_subdomain_t s, const xls_chefsi_params_t* p, double* ritz, double* resid,
                    int32_t* iters_done) {
  return guarded([&]() -> int {
    if (!s || !p || !ritz || !resid) fail(XLS_ERR_INVALID_ARG, "NULL argument");
    require_resident(s);
    return by_prec(s, [&](auto tag) { return chefsi_impl<decltype(tag)>(s, p, ritz, resid, iters_done); });
  });
}

int xls_subdomain_counters(xls_subdomain_t s, int64_t* out, int32_t cap) {
  return guarded([&]() -> int {
    if (!s || !out || cap < 1) fail(XLS_ERR_INVALID_ARG, "bad argument");
    const int64_t v[3] = {s->happly, s->last_fallback, s->last_iters};
    const int k = std::min(cap, 3);
    for (int i = 0; i < k; ++i) out[i] = v[i];
    return k;
  });
}

int xls_subdomain_density(xls_subdomain_t s, double mu, double sigma, double* rho, double* c) {
  return guarded([&]() -> int {
    if (!s || !rho || !c) fail(XLS_ERR_INVALID_ARG, "NULL argument");
    if (!s->have_ritz) fail(XLS_ERR_STATE, "density needs a completed xls_chefsi_step");
    require_resident(s);
    if (!(sigma > 0) || !std::isfinite(sigma) || !std::isfinite(mu)) fail(XLS_ERR_INVALID_ARG, "bad mu/sigma");
    if (!s->rho_dev) s->rho_dev = dalloc<double>(s->nd);
    XLS_HIP(hipMemcpyAsync(s->lam_dev, s->ritz.data(), s->ns * 8, hipMemcpyHostToDevice, s->st));
    const int nchunk = 64;
    launch_density(s->lam_dev, mu, sigma, s->mask, s->h, s->blk[s->cur], s->prec == XLS_PREC_FP32, s->nd,
                   s->ld, s->ns, s->rho_dev, s->cpart, nchunk, s->resid_dev, s->gocc, s->st);
    XLS_HIP(hipMemcpyAsync(rho, s->rho_dev, s->nd * 8, hipMemcpyDeviceToHost, s->st));
    XLS_HIP(hipMemcpyAsync(c, s->resid_dev, s->ns * 8, hipMemcpyDeviceToHost, s->st));
    XLS_HIP(hipStreamSynchronize(s->st));
    return XLS_OK;
  });
}

int xls_hamiltonian_apply(xls_subdomain_t s, const double* X, double* HX, int32_t ncols) {
  return guarded([&]() -> int {
    if (!s || !X || !HX || ncols < 1) fail(XLS_ERR_INVALID_ARG, "bad argument");
    return by_prec(s, [&](auto tag) -> int {
      using TS = decltype(tag);
      const size_t n = static_cast<size_t>(s->ld) * ncols;
      TS* x = dalloc<TS>(n);
      TS* y = nullptr;
      TS* al = nullptr;
      try {
        y = dalloc<TS>(n);
        al = dalloc<TS>(static_cast<size_t>(std::max(1, s->nproj())) * ncols);
        upload_block<TS>(s, X, x, ncols);
        apply_H<TS>(s, x, y, ncols, al);
        download_block<TS>(s, y, HX, ncols);
      } catch (...) {
        dfree(x);
        dfree(y);
        dfree(al);
        throw;
      }
      dfree(x);
      dfree(y);
      dfree(al);
      return XLS_OK;
    });
  });
}

int xls_subdomain_filter(xls_subdomain_t s, int32_t degree, double a0, double lam_cut, double lam_max) {
  return guarded([&]() -> int {
    if (!s || degree < 1) fail(XLS_ERR_INVALID_ARG, "bad argument");
    if (!(a0 < lam_cut && lam_cut < lam_max)) fail(XLS_ERR_INVALID_ARG, "need a0 < lam_cut < lam_max");
    require_resident(s);
    s->filter_launches = 0;
    s->filter_kernel_ms = 0.0;
    s->stage_ms.assign(8, 0.0);
    by_prec(s, [&](auto tag) {
      filter_block<decltype(tag)>(s, degree, a0, lam_cut, lam_max);
      return 0;
    });
    XLS_HIP(hipStreamSynchronize(s->st));
    return XLS_OK;
  });
}

int xls_subdomain_project(xls_subdomain_t s, int32_t gemm_prec, double* M, double* Hs) {
  return guarded([&]() -> int {
    if (!s || !M || !Hs) fail(XLS_ERR_INVALID_ARG, "NULL argument");
    if (s->prec == XLS_PREC_FP64 && gemm_prec != XLS_PREC_FP64)
      fail(XLS_ERR_INVALID_ARG, "FP64 handles run FP64 GEMMs");
    if (gemm_prec < 0 || gemm_prec > 2) fail(XLS_ERR_INVALID_ARG, "bad gemm_prec");
    require_resident(s);
    materialize_half(s);
    by_prec(s, [&](auto tag) {
      project_block<decltype(tag)>(s, gemm_prec);
      return 0;
    });
    const size_t nn = static_cast<size_t>(s->ns) * s->ns;
    XLS_HIP(hipMemcpyAsync(M, s->Mdev, nn * 8, hipMemcpyDeviceToHost, s->st));
    XLS_HIP(hipMemcpyAsync(Hs, s->Hsdev, nn * 8, hipMemcpyDeviceToHost, s->st));
    XLS_HIP(hipStreamSynchronize(s->st));
    return XLS_OK;
  });
}

int xls_subdomain_rotate(xls_subdomain_t s, int32_t gemm_prec, const double* Q) {
  return guarded([&]() -> int {
    if (!s || !Q) fail(XLS_ERR_INVALID_ARG, "NULL argument");
    if (s->prec == XLS_PREC_FP64 && gemm_prec != XLS_PREC_FP64)
      fail(XLS_ERR_INVALID_ARG, "FP64 handles run FP64 GEMMs");
    if (gemm_prec < 0 || gemm_prec > 2) fail(XLS_ERR_INVALID_ARG, "bad gemm_prec");
    if (!finite_all(Q, static_cast<int64_t>(s->ns) * s->ns)) fail(XLS_ERR_INVALID_ARG, "Q not finite");
    require_resident(s);
    materialize_half(s);
    XLS_HIP(hipMemcpyAsync(s->Ydev, Q, static_cast<size_t>(s->ns) * s->ns * 8, hipMemcpyHostToDevice, s->st));
    by_prec(s, [&](auto tag) {
      rotate_block<decltype(tag)>(s, gemm_prec, s->Ydev);
      return 0;
    });
    XLS_HIP(hipStreamSynchronize(s->st));
    return XLS_OK;
  });
}

int xls_subdomain_residual(xls_subdomain_t s, const double* lam, double* resid) {
  return guarded([&]() -> int {
    if (!s || !lam || !resid) fail(XLS_ERR_INVALID_ARG, "NULL argument");
    require_resident(s);
    materialize_half(s);
    XLS_HIP(hipMemcpyAsync(s->lam_dev, lam, s->ns * 8, hipMemcpyHostToDevice, s->st));
    by_prec(s, [&](auto tag) {
      residual_block<decltype(tag)>(s, s->lam_dev, s->resid_dev);
      return 0;
    });
    XLS_HIP(hipMemcpyAsync(resid, s->resid_dev, s->ns * 8, hipMemcpyDeviceToHost, s->st));
    XLS_HIP(hipStreamSynchronize(s->st));
    return XLS_OK;
  });
}

int xls_lanczos_bounds(xls_subdomain_t s, int32_t k, double* theta_min, double* upper) {
  return guarded([&]() -> int {
    if (!s || !theta_min || !upper || k < 1 || k > 60) fail(XLS_ERR_INVALID_ARG, "bad argument (1 <= k <= 60)");
    require_resident(s);
    by_prec(s, [&](auto tag) {
      lanczos_run<decltype(tag)>(s, k);
      return 0;
    });
    *theta_min = s->lz_lo;
    *upper = s->lz_up;
    return XLS_OK;
  });
}

int xls_dense_geneig(int32_t n, const double* Hs, const double* M, double* lam, double* Y) {
  return guarded([&]() -> int {
    if (n < 1 || !Hs || !M || !lam || !Y) fail(XLS_ERR_INVALID_ARG, "bad argument");
    const int64_t nn = static_cast<int64_t>(n) * n;
    if (!finite_all(Hs, nn) || !finite_all(M, nn)) fail(XLS_ERR_INVALID_ARG, "input not finite");
    hipStream_t st;
    XLS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    DenseWork w;
    double *dH = nullptr, *dM = nullptr, *dY = nullptr;
    int rc = XLS_OK;
    try {
      dense_alloc(w, n);
      dH = dalloc<double>(nn);
      dM = dalloc<double>(nn);
      dY = dalloc<double>(nn);
      XLS_HIP(hipMemcpyAsync(dH, Hs, nn * 8, hipMemcpyHostToDevice, st));
      XLS_HIP(hipMemcpyAsync(dM, M, nn * 8, hipMemcpyHostToDevice, st));
      rc = dense_geneig(w, dH, dM, dY, st);
      if (rc == XLS_OK) {
        XLS_HIP(hipMemcpyAsync(lam, w.lam(), n * 8, hipMemcpyDeviceToHost, st));
        XLS_HIP(hipMemcpyAsync(Y, dY, nn * 8, hipMemcpyDeviceToHost, st));
      }
      XLS_HIP(hipStreamSynchronize(st));
    } catch (...) {
      (void)hipStreamSynchronize(st);
      dfree(dH);
      dfree(dM);
      dfree(dY);
      dense_free(w);
      (void)hipStreamDestroy(st);
      throw;
    }
    dfree(dH);
    dfree(dM);
    dfree(dY);
    dense_free(w);
    (void)hipStreamDestroy(st);
    if (rc != XLS_OK) g_last_error = rc == XLS_ERR_NOT_SPD ? "M is not positive definite" : "no convergence";
    return rc;
  });
}

int xls_subdomain_get_block(xls_subdomain_t s, double* X) {
  return guarded([&]() -> int {
    if (!s || !X) fail(XLS_ERR_INVALID_ARG, "NULL argument");
    require_resident(s);
    materialize_half(s);
    by_prec(s, [&](auto tag) {
      download_block<decltype(tag)>(s, s->blk[s->cur], X, s->ns);
      return 0;
    });
    return XLS_OK;
  });
}

int xls_subdomain_set_block(xls_subdomain_t s, const double* X) {
  return guarded([&]() -> int {
    if (!s || !X) fail(XLS_ERR_INVALID_ARG, "NULL argument");
    if (!finite_all(X, s->nd * s->ns)) fail(XLS_ERR_INVALID_ARG, "block not finite");
    require_resident(s);
    s->half_src = nullptr;
    by_prec(s, [&](auto tag) {
      upload_block<decltype(tag)>(s, X, s->blk[s->cur], s->ns);
      return 0;
    });
    XLS_HIP(hipStreamSynchronize(s->st));
    s->have_ritz = false;
    return XLS_OK;
  });
}


int xls_subdomain_store_half(xls_subdomain_t s, uint16_t* dst) {
  return guarded([&]() -> int {
    if (!s || !dst) fail(XLS_ERR_INVALID_ARG, "NULL argument");
    require_resident(s);
    materialize_half(s);
    check_device_range(dst, static_cast<size_t>(s->nd) * s->ns * 2);
    by_prec(s, [&](auto tag) {
      using TS = decltype(tag);
      launch_block_half<TS>(B<TS>(s, s->cur), s->ld, s->nd, s->ns, dst, 1, s->st);
      return 0;
    });
    XLS_HIP(hipStreamSynchronize(s->st));
    return XLS_OK;
  });
}

int xls_subdomain_load_half(xls_subdomain_t s, const uint16_t* src) {
  return guarded([&]() -> int {
    if (!s || !src) fail(XLS_ERR_INVALID_ARG, "NULL argument");
    require_resident(s);
    s->half_src = nullptr;
    check_device_range(src, static_cast<size_t>(s->nd) * s->ns * 2);
    by_prec(s, [&](auto tag) {
      using TS = decltype(tag);
      launch_block_half<TS>(B<TS>(s, s->cur), s->ld, s->nd, s->ns, const_cast<uint16_t*>(src), 0, s->st);
      return 0;
    });
    XLS_HIP(hipStreamSynchronize(s->st));
    s->have_ritz = false;
    return XLS_OK;
  });
}

int xls_subdomain_use_half(xls_subdomain_t s, const uint16_t* src) {
  return guarded([&]() -> int {
    if (!s || !src) fail(XLS_ERR_INVALID_ARG, "NULL argument");
    require_resident(s);
    check_device_range(src, static_cast<size_t>(s->nd) * s->ns * 2);
    s->half_src = src;
    s->have_ritz = false;
    return XLS_OK;
  });
}

int xls_subdomain_pdos(xls_subdomain_t s, double orb_width, double orb_rc, double* weights, int32_t nbins,
                       const double* edges, double* pdos, uint8_t* in_core) {
  return guarded([&]() -> int {
    if (!s || !weights) fail(XLS_ERR_INVALID_ARG, "NULL argument");
    if (!(orb_width > 0) || !(orb_rc > 0) || !std::isfinite(orb_width) || !std::isfinite(orb_rc))
      fail(XLS_ERR_INVALID_ARG, "orbital width and cutoff must be finite and > 0");
    if (nbins < 0 || (nbins > 0 && (!edges || !pdos))) fail(XLS_ERR_INVALID_ARG, "bad PDOS bins");
    for (int b = 0; b < nbins; ++b)
      if (!(edges[b] < edges[b + 1])) fail(XLS_ERR_INVALID_ARG, "PDOS edges must increase");
    if (nbins > 0 && !s->have_ritz) fail(XLS_ERR_STATE, "PDOS bins need the Ritz values of a completed xls_chefsi_step");
    require_resident(s);
    materialize_half(s);
    const int na = s->n_atoms, norb = 4 * na, ns = s->ns;
    if (na == 0) return XLS_OK;  // no atomic orbitals: every output is empty
    if (!s->orb_val || s->orb_width != orb_width || s->orb_rc != orb_rc) {
      // atomic orbitals: the projector support rule and shape with the
      // orbitals' width and cutoff, unit coefficients
      xls_subdomain_desc_t d{};
      for (int a = 0; a < 3; ++a) {
        d.n[a] = s->n[a];
        d.origin[a] = s->origin[a];
        d.core_lo[a] = s->core_lo[a];
        d.core_hi[a] = s->core_hi[a];
        d.global_offset[a] = s->global_offset[a];
        d.global_n[a] = s->global_n[a];
      }
      d.h = s->h;
      d.bc = s->bc;
      d.fd_n0 = kRadius;
      d.n_atoms = na;
      d.atom_xyz = s->atom_xyz.data();
      std::vector<xls_projset_t> orb(na);
      for (int a = 0; a < na; ++a) {
        orb[a].rc = orb_rc;
        orb[a].gauss_width = orb_width;
        for (int l = 0; l < 4; ++l) orb[a].gamma[l] = 1.0;
      }
      d.proj = orb.data();
      SetupTables t;
      build_setup(d, t);
      void* ps[] = {s->orb_off, s->orb_idx, s->orb_val, s->orb_gamma, s->orb_alpha, s->orb_P, s->orb_core};
      XLS_HIP(hipStreamSynchronize(s->st));
      for (void* p : ps) dfree(p);
      s->orb_off = s->orb_idx = nullptr;
      s->orb_val = s->orb_gamma = s->orb_alpha = s->orb_P = nullptr;
      s->orb_core = nullptr;
      s->orb_off = dupload(t.sup_off, s->st);
      s->orb_idx = dupload(t.sup_idx, s->st);
      s->orb_val = dupload(t.sup_val, s->st);
      s->orb_gamma = dupload(t.gamma, s->st);
      s->orb_core = dupload(s->atom_core, s->st);
      s->orb_alpha = dalloc<double>(static_cast<size_t>(ns) * norb);
      s->orb_P = dalloc<double>(static_cast<size_t>(ns) * norb);
      s->orb_width = orb_width;
      s->orb_rc = orb_rc;
    }
    OpTables<double> op = s->op64;
    op.sup_off = s->orb_off;
    op.sup_idx = s->orb_idx;
    op.slot_val = s->orb_val;
    op.gamma = s->orb_gamma;
    if (nbins > static_cast<int>(s->orb_dcap)) {
      XLS_HIP(hipStreamSynchronize(s->st));
      dfree(s->orb_D);
      dfree(s->orb_edges);
      s->orb_D = nullptr;
      s->orb_edges = nullptr;
      s->orb_D = dalloc<double>(static_cast<size_t>(norb) * nbins);
      s->orb_edges = dalloc<double>(static_cast<size_t>(nbins) + 1);
      s->orb_dcap = nbins;
    }
    by_prec(s, [&](auto tag) {
      using TS = decltype(tag);
      launch_proj_forward<TS, double>(op, B<TS>(s, s->cur), s->ld, ns, s->orb_alpha, s->st);
      return 0;
    });
    if (nbins > 0) {
      XLS_HIP(hipMemcpyAsync(s->lam_dev, s->ritz.data(), ns * 8, hipMemcpyHostToDevice, s->st));
      XLS_HIP(hipMemcpyAsync(s->orb_edges, edges, (static_cast<size_t>(nbins) + 1) * 8, hipMemcpyHostToDevice,
                             s->st));
    }
    launch_pdos(s->orb_alpha, ns, norb, s->h, s->lam_dev, s->orb_edges, nbins, s->orb_core, s->orb_P, s->orb_D,
                s->st);
    XLS_HIP(hipMemcpyAsync(weights, s->orb_P, static_cast<size_t>(ns) * norb * 8, hipMemcpyDeviceToHost, s->st));
    if (nbins > 0)
      XLS_HIP(hipMemcpyAsync(pdos, s->orb_D, static_cast<size_t>(norb) * nbins * 8, hipMemcpyDeviceToHost, s->st));
    XLS_HIP(hipStreamSynchronize(s->st));
    if (in_core) std::memcpy(in_core, s->atom_core.data(), na);
    return XLS_OK;
  });
}

int xls_subdomain_get_maps(xls_subdomain_t s, uint8_t* core_mask, int64_t* global_index) {
  return guarded([&]() -> int {
    if (!s || !core_mask || !global_index) fail(XLS_ERR_INVALID_ARG, "NULL argument");
    std::memcpy(core_mask, s->tab.core_mask.data(), s->nd);
    std::memcpy(global_index, s->tab.global_index.data(), s->nd * 8);
    return XLS_OK;
  });
}

int xls_subdomain_get_projectors(xls_subdomain_t s, int64_t* sizes, int32_t* offsets, int32_t* idx,
                                 double* val, int32_t* rev_offsets, int32_t* rev_slot) {
  return guarded([&]() -> int {
    if (!s || !sizes) fail(XLS_ERR_INVALID_ARG, "NULL argument");
    const size_t total = s->tab.sup_idx.size();
    sizes[0] = static_cast<int64_t>(total);
    sizes[1] = s->n_atoms;
    if (offsets) std::memcpy(offsets, s->tab.sup_off.data(), (s->n_atoms + 1) * 4);
    if (idx) std::memcpy(idx, s->tab.sup_idx.data(), total * 4);
    if (val) std::memcpy(val, s->tab.sup_val.data(), total * 4 * 8);
    if (rev_offsets) std::memcpy(rev_offsets, s->tab.rev_off.data(), (s->nd + 1) * 4);
    if (rev_slot) std::memcpy(rev_slot, s->tab.rev_slot.data(), total * 4);
    return XLS_OK;
  });
}

int xls_split_bf16(const float* a, uint16_t* hi, uint16_t* lo, int64_t n) {
  return guarded([&]() -> int {
    if (n < 0 || (n > 0 && (!a || !hi || !lo))) fail(XLS_ERR_INVALID_ARG, "bad argument");
    if (n == 0) return XLS_OK;
    float* da = dalloc<float>(n);
    uint16_t *dh = nullptr, *dl = nullptr;
    try {
      dh = dalloc<uint16_t>(n);
      dl = dalloc<uint16_t>(n);
      XLS_HIP(hipMemcpy(da, a, n * 4, hipMemcpyHostToDevice));
      split_bf16_device(da, dh, dl, n, nullptr);
      XLS_HIP(hipMemcpy(hi, dh, n * 2, hipMemcpyDeviceToHost));
      XLS_HIP(hipMemcpy(lo, dl, n * 2, hipMemcpyDeviceToHost));
    } catch (...) {
      dfree(da);
      dfree(dh);
      dfree(dl);
      throw;
    }
    dfree(da);
    dfree(dh);
    dfree(dl);
    return XLS_OK;
  });
}

int xls_subdomain_tune(xls_subdomain_t s, int32_t prec, int32_t block, int32_t ty, int32_t tz, int32_t nv) {
  return guarded([&]() -> int {
    if (!s) fail(XLS_ERR_INVALID_ARG, "NULL handle");
    if (prec != XLS_PREC_FP64 && prec != XLS_PREC_FP32) fail(XLS_ERR_INVALID_ARG, "prec must be FP64 or FP32");
    StencilLaunch c;
    c.block = block;
    c.ty = ty;
    c.tz = tz;
    c.nv = nv;
    stencil_validate(s->n[0], s->n[1], s->n[2], s->bc == XLS_BC_PERIODIC, prec == XLS_PREC_FP64 ? 8 : 4,
                     s->nproj(), c);
    if (prec == XLS_PREC_FP64) {
      // the residual sweep uses the FP64 shape: grow its partial buffer if needed
      const size_t need = std::max(stencil_partial_elems(s->op64, s->ns, c), static_cast<size_t>(s->ns) * 64);
      if (s->resident && need > s->partial_elems) {
        XLS_HIP(hipStreamSynchronize(s->st));
        double* np = dalloc<double>(need);
        dfree(s->partial);
        s->partial = np;
        s->partial_elems = need;
      }
      s->cfg64 = c;
    } else {
      s->cfg32 = c;
    }
    return XLS_OK;
  });
}

int xls_subdomain_tune_gemm(xls_subdomain_t s, int32_t split_scale, int32_t tile_tn, int32_t tile_nn) {
  return guarded([&]() -> int {
    if (!s) fail(XLS_ERR_INVALID_ARG, "NULL handle");
    if (split_scale < 0 || split_scale > 64 || tile_tn < 0 || tile_tn > 3 || tile_nn < 0 || tile_nn > 3)
      fail(XLS_ERR_INVALID_ARG, "split_scale must be in [0, 64], tile_tn and tile_nn in [0, 3]");
    s->gplan.split_scale = split_scale;
    s->gplan.tile_tn = tile_tn;
    s->gplan.tile_nn = tile_nn;
    return XLS_OK;
  });
}

int xls_subdomain_time_gemms(xls_subdomain_t s, int32_t gemm_prec, int32_t reps, double* ms) {
  return guarded([&]() -> int {
    if (!s || !ms || reps < 1) fail(XLS_ERR_INVALID_ARG, "bad argument");
    if (s->prec == XLS_PREC_FP64 && gemm_prec != XLS_PREC_FP64)
      fail(XLS_ERR_INVALID_ARG, "FP64 handles run FP64 GEMMs");
    if (gemm_prec < 0 || gemm_prec > 2) fail(XLS_ERR_INVALID_ARG, "bad gemm_prec");
    require_resident(s);
    materialize_half(s);
    by_prec(s, [&](auto tag) {
      using TS = decltype(tag);
      TS* Bc = B<TS>(s, s->cur);
      TS* W = B<TS>(s, 1 - s->cur);
      apply_H<TS>(s, Bc, W, s->ns, static_cast<TS*>(s->alpha));
      // rotation operand: a fixed well-scaled matrix (scheduling only)
      std::vector<double> q(static_cast<size_t>(s->ns) * s->ns, 0.0);
      for (int i = 0; i < s->ns; ++i) q[static_cast<size_t>(i) * s->ns + i] = 1.0;
      XLS_HIP(hipMemcpyAsync(s->Ydev, q.data(), q.size() * 8, hipMemcpyHostToDevice, s->st));
      auto run = [&](int which) {
        if (which == 0)
          gemm_tn<TS>(gemm_prec, Bc, s->ld, Bc, s->ld, s->ns, s->ns, s->nd, s->Mdev, s->ns, 1, 0, s->gwork,
                      s->gwork_elems, s->st, s->gplan);
        else if (which == 1)
          gemm_tn<TS>(gemm_prec, Bc, s->ld, W, s->ld, s->ns, s->ns, s->nd, s->Hsdev, s->ns, 1, 1, s->gwork,
                      s->gwork_elems, s->st, s->gplan);
        else  // into the spare block: the current block is left as it was
          gemm_nn<TS>(gemm_prec, Bc, s->ld, s->Ydev, s->ns, static_cast<int>(s->nd), s->ns, s->ns, W, s->ld,
                      s->bwork, s->st, s->gplan);
      };
      hipEvent_t e0, e1;
      XLS_HIP(hipEventCreate(&e0));
      XLS_HIP(hipEventCreate(&e1));
      try {
        for (int which = 0; which < 3; ++which) {
          run(which);  // warm-up
          XLS_HIP(hipEventRecord(e0, s->st));
          for (int r = 0; r < reps; ++r) run(which);
          XLS_HIP(hipEventRecord(e1, s->st));
          XLS_HIP(hipEventSynchronize(e1));
          float t = 0.0f;
          XLS_HIP(hipEventElapsedTime(&t, e0, e1));
          ms[which] = static_cast<double>(t) / reps;
        }
      } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return 0;
    });
    return 3;
  });
}

int xls_get_stage_times(xls_subdomain_t s, double* ms, int64_t* counts, int32_t cap) {
  return guarded([&]() -> int {
    if (!s || !ms || cap < 1) fail(XLS_ERR_INVALID_ARG, "bad argument");
    if (s->stage_ms.size() < 8) s->stage_ms.resize(8, 0.0);
    s->stage_ms[7] = s->filter_kernel_ms;
    const int n = std::min<int>(cap, static_cast<int>(s->stage_ms.size()));
    for (int i = 0; i < n; ++i) ms[i] = s->stage_ms[i];
    if (counts) counts[0] = s->filter_launches;
    return n;
  });
}

}  // extern "C"
