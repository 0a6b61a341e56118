// Subdomain handle and the per-subdomain stage helpers shared by the C ABI
// (api.cpp) and the batch engine (batch.cpp).  Internal to libxls.
#pragma once
#include <hip/hip_runtime.h>

#include <new>
#include <string>
#include <vector>

#include "xls_internal.h"

namespace xls {
void dfree(void* p);
}  // namespace xls

using xls::DenseWork;
using xls::OpTables;
using xls::SetupTables;
using xls::StencilLaunch;

struct xls_subdomain_s {
  int n[3] = {0, 0, 0};
  int core_lo[3] = {0, 0, 0}, core_hi[3] = {0, 0, 0};
  double a0_bound = 0.0;  // rigorous lower bound of lambda_1 (learned bounds)
  double h = 0;
  int bc = 0;
  int prec = XLS_PREC_FP64;
  int ns = 0;
  int64_t nd = 0, ld = 0;
  hipStream_t st = nullptr;
  bool own_stream = false;
  SetupTables tab;
  int n_atoms = 0;
  // device: operator tables in both precisions
  double* v64 = nullptr;
  float* v32 = nullptr;
  double* val64 = nullptr;
  float* val32 = nullptr;
  int32_t *rev_pk = nullptr, *rev_aoff = nullptr, *sup_off = nullptr, *sup_idx = nullptr;
  double* rev_val64 = nullptr;
  float* rev_val32 = nullptr;
  double* gamma = nullptr;
  uint8_t* mask = nullptr;
  OpTables<double> op64;
  OpTables<float> op32;
  StencilLaunch cfg64, cfg32;
  xls::GemmPlan gplan;  // projection and rotation GEMM launch plan
  // blocks
  void* blk[2] = {nullptr, nullptr};
  int cur = 0;
  void* alpha = nullptr;      // [ns][nproj] in storage type
  double* alpha64 = nullptr;  // [ns][nproj] FP64 (residuals of FP32 blocks)
  double* partial = nullptr;
  size_t partial_elems = 0;
  double* lam_dev = nullptr;
  double* resid_dev = nullptr;
  double* rq_dev = nullptr;  // FP64 Rayleigh quotients of the block's columns (residual sweep)
  double* Mdev = nullptr;
  double* Hsdev = nullptr;
  double* Ydev = nullptr;
  float* bwork = nullptr;
  double* gwork = nullptr;
  size_t gwork_elems = 0;
  bool own_gwork = true;  // false: a batch's per-stream split-K workspace
  DenseWork dw;
  double* vsmall = nullptr;  // density / Lanczos scalars
  double* rho_dev = nullptr;
  double* cpart = nullptr;
  double* gocc = nullptr;
  // start block: the caller's (uploaded at create, or kept here for a batch
  // that allocates working sets on demand), else drawn on the device from
  // x0_seed (counter-based, Philox4x32-10 + Box-Muller)
  std::vector<double> x0_host;
  uint64_t x0_seed = 0;
  bool x0_gen = false;
  // working set (blocks, projections, GEMM and dense workspaces) allocated
  bool resident = false;
  // geometry kept for tables built later (atomic orbitals of the PDOS)
  double origin[3] = {0, 0, 0};
  int64_t global_offset[3] = {0, 0, 0}, global_n[3] = {1, 1, 1};
  std::vector<double> atom_xyz;
  std::vector<xls_projset_t> proj;
  // PDOS orbital tables, built for (orb_width, orb_rc) on first use
  double orb_width = 0.0, orb_rc = 0.0;
  int32_t *orb_off = nullptr, *orb_idx = nullptr;
  double *orb_val = nullptr, *orb_gamma = nullptr, *orb_alpha = nullptr, *orb_P = nullptr, *orb_D = nullptr,
         *orb_edges = nullptr;
  uint8_t* orb_core = nullptr;
  std::vector<uint8_t> atom_core;  // atoms whose position lies in the core box
  int orb_dcap = 0;
  // binary16 warm start not yet widened (xls_subdomain_use_half): the
  // caller's device buffer, N_d x ns with leading dimension N_d
  const uint16_t* half_src = nullptr;
  // Lanczos
  std::vector<double> lanczos_v0;
  void* lz = nullptr;  // [nd * (kmax + 2)]
  int lz_cols = 0;
  bool have_lanczos = false;
  double lz_lo = 0, lz_up = 0;
  int lz_k = 0;
  // state
  std::vector<double> ritz;
  bool have_ritz = false;
  std::vector<double> stage_ms;
  int64_t filter_launches = 0;
  double filter_kernel_ms = 0.0;  // sum over fused-filter stencil launches (profiling on)
  std::vector<hipEvent_t> fev;
  // work counters of the last chefsi step
  int64_t happly = 0;
  int last_fallback = 0;
  int last_iters = 0;
  void* backup = nullptr;  // start block kept for a learned-bounds fallback
  // dense stage replayed from a hipGraph (its launch sequence depends on ns only)
  hipGraph_t dgraph = nullptr;
  hipGraphExec_t dexec = nullptr;
  bool dwarm = false;

  ~xls_subdomain_s() {
    void* ps[] = {v64, v32, val64, val32, rev_pk, rev_aoff, rev_val64, rev_val32, sup_off, sup_idx, gamma, mask,
                  blk[0], blk[1], alpha, alpha64, partial, lam_dev, resid_dev, rq_dev, Mdev, Hsdev, Ydev, bwork,
                  vsmall, rho_dev, cpart, gocc, lz, backup, orb_off, orb_idx, orb_val, orb_gamma, orb_alpha,
                  orb_P, orb_D, orb_edges, orb_core};
    for (void* p : ps) xls::dfree(p);
    if (own_gwork) xls::dfree(gwork);
    for (auto e : fev) (void)hipEventDestroy(e);
    if (dexec) (void)hipGraphExecDestroy(dexec);
    if (dgraph) (void)hipGraphDestroy(dgraph);
    xls::dense_free(dw);
    if (own_stream && st) (void)hipStreamDestroy(st);
  }
  size_t esize() const { return prec == XLS_PREC_FP32 ? 4 : 8; }
  int nproj() const { return 4 * n_atoms; }
};

namespace xls {

void set_last_error(const std::string& m);
bool profiling_on();
bool graphs_on();
void dfree(void* p);
bool finite_all(const double* p, int64_t n);
// STATE unless the handle's working set is allocated.
void require_resident(const xls_subdomain_s* s);
// Widens a pending binary16 warm start into the current block.
void materialize_half(xls_subdomain_s* s);

template <typename T>
T* dalloc(size_t n) {
  void* p = nullptr;
  if (n == 0) n = 1;
  const hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(XLS_ERR_OUT_OF_MEMORY, "device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed");
  }
  return static_cast<T*>(p);
}

// Runs f, mapping exceptions to status codes (no exception crosses the ABI).
template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return XLS_ERR_OUT_OF_MEMORY;
  } catch (...) {
    set_last_error("unexpected internal error");
    return XLS_ERR_DEVICE;
  }
}

template <typename TS>
TS* B(xls_subdomain_s* s, int i) {
  return static_cast<TS*>(s->blk[i]);
}
inline const OpTables<double>& op_of(xls_subdomain_s* s, double) { return s->op64; }
inline const OpTables<float>& op_of(xls_subdomain_s* s, float) { return s->op32; }
template <typename TS>
const OpTables<TS>& op_of(xls_subdomain_s* s) {
  return op_of(s, TS{});
}
template <typename TS>
const StencilLaunch& cfg_of(xls_subdomain_s* s) {
  return std::is_same<TS, float>::value ? s->cfg32 : s->cfg64;
}

// Precision schedule of the projection and rotation GEMMs: split-BF16 keeps
// about 16 mantissa bits per operand.  In the projection that bounds Ritz
// values near 1e-5 relative; in the rotation it adds white noise of about
// 1e-5 relative to every vector, which the residual check sees amplified by
// up to lambda_max (no filter step damps it first).  So once the previous
// iteration's largest gated residual is at most kPolishResid, both run in
// FP32.
constexpr double kPolishResid = 1e-2;
inline int polish_prec(int gprec, double prev_gated_resid) {
  return (gprec == XLS_PREC_BF16X3 && prev_gated_resid <= kPolishResid) ? XLS_PREC_FP32 : gprec;
}

// Lanczos steps a run takes for a requested k (<= 0: 20), at most
// kMaxLanczos and N_d; the cached bounds of a handle are keyed by it.
constexpr int kMaxLanczos = 60;
int lanczos_steps(const xls_subdomain_s* s, int k);
// Largest of r[0..gate); NaN when any of them is NaN (a NaN residual is a
// miss of every gate).
double gated_max(const double* r, int gate);

// Handle construction in parts (api.cpp).  subdomain_tables: geometry,
// operator tables and small per-state buffers (always resident); keep_x0
// keeps a copy of the caller's start block for later loads.
// subdomain_ws_alloc / _free: the working set (both blocks, projection
// coefficients, GEMM and dense workspaces); shared_gwork (may be null) is a
// split-K workspace the caller owns and shares between handles that issue
// on one stream.  subdomain_ws_bytes: device bytes of the working set.
// load_start_block: the start block into block 0 (x0, else the kept copy,
// else drawn on the device from x0_seed).
void subdomain_tables(xls_subdomain_s* s, const xls_subdomain_desc_t* d, bool keep_x0);
// A validated handle with its tables only (no working set), keeping the caller's x0.
xls_subdomain_s* subdomain_create_tables(const xls_subdomain_desc_t* d);
size_t subdomain_ws_bytes(const xls_subdomain_s* s, bool shared_gemm_work);
void subdomain_ws_alloc(xls_subdomain_s* s, double* shared_gwork, size_t shared_elems);
void subdomain_ws_free(xls_subdomain_s* s);
template <typename TS>
void load_start_block(xls_subdomain_s* s, const double* x0);

// Stage helpers on the handle's stream (api.cpp).
template <typename TS>
void apply_H(xls_subdomain_s* s, const TS* y, TS* out, int ncols, TS* alpha);
template <typename TS>
void filter_block(xls_subdomain_s* s, int m, double a0, double lc, double lmax);
template <typename TS>
void rotate_block(xls_subdomain_s* s, int gprec, const double* Ydev);
template <typename TS>
void residual_block(xls_subdomain_s* s, const double* lam_dev, double* resid_dev, double* rq_dev = nullptr);
template <typename TS>
void lanczos_run(xls_subdomain_s* s, int k);

}  // namespace xls
