// Internal declarations shared by the engine's host code and HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/xls.h"

namespace xls {

constexpr int kRadius = 6;  // FD half-width n0 (12th-order Laplacian)

// ---------------------------------------------------------------------------
// error plumbing: every internal failure throws Error; the ABI layer turns it
// into a status code and a thread-local message.
// ---------------------------------------------------------------------------
struct Error {
  int code;
  std::string msg;
};
[[noreturn]] void fail(int code, const std::string& msg);
void check_hip(hipError_t e, const char* what, const char* file, int line);
#define XLS_HIP(call) ::xls::check_hip((call), #call, __FILE__, __LINE__)
#define XLS_LAUNCH_CHECK(name) ::xls::check_hip(hipGetLastError(), name, __FILE__, __LINE__)

// ---------------------------------------------------------------------------
// host-side setup tables (setup.cpp)
// ---------------------------------------------------------------------------
struct SetupTables {
  std::vector<uint8_t> core_mask;     // [nd]
  std::vector<int64_t> global_index;  // [nd]
  std::vector<int32_t> sup_off;       // [n_atoms + 1]
  std::vector<int32_t> sup_idx;       // [total]
  std::vector<double> sup_val;        // [4 * total]  slot-major
  std::vector<int32_t> slot_atom;     // [total]
  std::vector<int32_t> rev_off;       // [nd + 1]
  std::vector<int32_t> rev_slot;      // [total]
  std::vector<double> gamma;          // [4 * n_atoms]
  // kernel form of the reverse CSR: per point (first entry | count << 27),
  // per entry the four projector values and 4*atom (offset into alpha)
  std::vector<int32_t> rev_pk;        // [nd]
  std::vector<double> rev_val;        // [4 * (total + 1)] reverse-CSR order, then a zero sentinel
  std::vector<int32_t> rev_aoff;      // [total + 1]
};
void build_setup(const xls_subdomain_desc_t& d, SetupTables& t);

// ---------------------------------------------------------------------------
// kernel launchers
// ---------------------------------------------------------------------------
enum StencilMode { kApply = 0, kFilter = 1, kResid = 2 };

// Geometry + operator tables on the device for one subdomain, in compute type TC.
template <typename TC>
struct OpTables {
  const TC* v = nullptr;         // [nd]
  const TC* slot_val = nullptr;  // [4 * total] support order
  const int32_t* rev_pk = nullptr;
  const TC* rev_val = nullptr;   // [4 * (nent + 1)] reverse-CSR order, then a zero sentinel
  const int32_t* rev_aoff = nullptr;
  int64_t nent = 0;              // reverse-CSR entries (= support slots)
  const int32_t* sup_off = nullptr;
  const int32_t* sup_idx = nullptr;
  const double* gamma = nullptr;  // [4 * n_atoms]
  int32_t n_atoms = 0;
  int32_t nx = 0, ny = 0, nz = 0;
  int32_t periodic = 0;
  double h = 0;
};

struct StencilLaunch {
  int block = 0;    // threads: 256 or 512 (0 = 256 when its halo budget suffices, else 512)
  int ty = 0;       // rows per tile (0 = choose)
  int tz = 0;       // z-chunk (0 = whole nz)
  int nv = 0;       // vectors per tile: 1 or 2 (0 = choose; residual sweeps take 1)
};

// HY / filter step / residual over ncols columns of y (ld elements apart).
//   kApply : out = H y
//   kFilter: out = a (H y - c y) - b yprev   (yprev may alias out; b = 0 ignores yprev)
//   kResid : resid2[col] = sqrt(sum_g (H y - lam[col] y)^2)   (needs partial scratch,
//            stencil_partial_elems doubles); when rq is not null also
//            rq[col] = (y^T H y) / (y^T y), the column's Rayleigh quotient, in FP64
// alpha: [ncols][4*n_atoms] gamma-scaled projections of y (proj_forward).
template <typename TS, typename TC>
void launch_stencil(StencilMode mode, const OpTables<TC>& op, const TS* y, int64_t ld, int ncols,
                    const TC* alpha, TS* out, const TS* yprev, double a, double c, double b,
                    const double* lam, double* partial, double* resid2, hipStream_t st,
                    const StencilLaunch& cfg, double* rq = nullptr);
// Filter step (kFilter, TS == TC) with one binary16 input stream of leading
// dimension ld16: y16 as Y_k (then yprev16 is null and Y_{k-1} absent), or
// yprev16 as Y_{k-1} (y is then the TS block); out is a TS block.
template <typename TS, typename TC>
void launch_filter_half(const OpTables<TC>& op, const TS* y, const uint16_t* y16, int64_t ld, int64_t ld16,
                        int ncols, const TC* alpha, TS* out, const uint16_t* yprev16, double a, double c, double b,
                        hipStream_t st, const StencilLaunch& cfg);
// alpha[col][4a+l] = gamma_{a,l} h^3 sum_{s in S_a} chi_{a,l}(s) y(idx(s), col)
template <typename TS, typename TC>
void launch_proj_forward(const OpTables<TC>& op, const TS* y, int64_t ld, int ncols, TC* alpha,
                         hipStream_t st);
// Raises a kernel's dynamic-LDS limit to at least `bytes` (no-op at or below
// 64 KiB; each kernel is configured once per size, so launches inside a
// graph capture make no runtime-configuration calls after warm-up).
void ensure_dyn_smem(const void* fn, size_t bytes);

// Grouped filter steps over many operators of one precision (batch engine).
// Operator i filters its block in place between buf[0] and buf[1]: step k
// reads buf[(cur0 + k) & 1] and writes buf[(cur0 + k + 1) & 1], with the
// recurrence coefficients coef[3k .. 3k+2] read from device memory; operators
// take part in steps k < degree.  Build and free synchronise; steps only
// launch kernels (graph-capturable).
template <typename TS>
struct FilterGroupOp {
  const OpTables<TS>* op;
  TS* buf[2];
  int cur0;
  int64_t ld;
  int ncols;
  TS* alpha;           // [ncols][4 n_atoms]
  const double* coef;  // device, 3 * degree doubles
  int degree;
  StencilLaunch cfg;
};
template <typename TS>
struct FilterGroup;
template <typename TS>
FilterGroup<TS>* filter_group_build(const std::vector<FilterGroupOp<TS>>& ops);
template <typename TS>
void filter_group_step(FilterGroup<TS>* g, int k, hipStream_t st);
template <typename TS>
int filter_group_steps(const FilterGroup<TS>* g);
template <typename TS>
void filter_group_free(FilterGroup<TS>* g);
// coef[3k..3k+2] = (a_k, c, b_k) of the scaled recurrence for degree m:
// from (a0, lam_cut, lam_max), or with lam != NULL from a0 = lam[0] and
// lam_cut = lam[ns-1]; bad = 1 when a0 < lam_cut < lam_max fails.
void launch_filter_coef(const double* lam, int ns, double a0, double lc, double lmax, int m, double* coef,
                        int32_t* bad, hipStream_t st);

// Throws INVALID_ARG when the launch shape cannot run on this grid.
void stencil_validate(int nx, int ny, int nz, int periodic, int elem_bytes, int nproj,
                      const StencilLaunch& cfg);
size_t stencil_partial_elems(const OpTables<float>& op, int ncols, const StencilLaunch& cfg);
size_t stencil_partial_elems(const OpTables<double>& op, int ncols, const StencilLaunch& cfg);

// GEMMs.  Matrices column-major.
//   gemm_tn: C[M x N] = A^T B, A is K x M (lda), B is K x N (ldb); FP64 result.
//            sym = 1: only C's upper tiles are formed, then mirrored.
//            symmetrize = 1: C = (S + S^T)/2 (M == N); with sym = 1 too,
//            the entries of diagonal tiles are averaged with their
//            transposes and the rest mirrored from the upper tiles (the
//            projected Hamiltonian, of which the eigensolver reads one
//            triangle).
//   gemm_nn: C[M x N] = A[M x K] B[K x N]; B given in FP64 and converted
//            (or padded) into bwork, nn_work_doubles(K, N) doubles, 16-byte
//            aligned; bwork may be null only for FP64 calls (the small-tile
//            path is taken when B would need padding).
// Launch plan of the projection and rotation GEMMs (the autotuner's choice
// per shape class): split_scale 0 keeps the default split-K count (about as
// many workgroups as are resident at once, at least 16 k-slabs per split;
// the rotation's tiles do not split), k > 0 scales it
// by k/2; tile_tn 0 takes the large-tile projection kernel when shapes
// allow (edge 96 or 128, whichever issues less padded work by 10 %), 1 the
// 64 x 64 tiles, 2 and 3 force the 128 and 96 edges; tile_nn 0 takes the
// large rotation kernel with 64 x 128 tiles when shapes allow (3 too), 1
// the 64 x 64 tiles, 2 the large kernel with 64 x 256 tiles.
// A plan changes the order of the split sums, never a product.
struct GemmPlan {
  int split_scale = 0;
  int tile_tn = 0;
  int tile_nn = 0;
};
template <typename TS>
void gemm_tn(int prec, const TS* A, int64_t lda, const TS* B, int64_t ldb, int M, int N, int64_t K,
             double* C, int64_t ldc, int sym, int symmetrize, double* work, size_t work_elems,
             hipStream_t st, const GemmPlan& plan = GemmPlan{});
size_t gemm_tn_work_elems(int M, int N, int64_t K);
// doubles of the rotation work buffer (B copied with rows padded to 8)
size_t nn_work_doubles(int K, int N);
template <typename TS>
void gemm_nn(int prec, const TS* A, int64_t lda, const double* B, int64_t ldb, int M, int N, int K,
             TS* C, int64_t ldc, void* bwork, hipStream_t st, const GemmPlan& plan = GemmPlan{});
void split_bf16_device(const float* a, uint16_t* hi, uint16_t* lo, int64_t n, hipStream_t st);

// Learned filter bounds: the margins a run applies to a prediction (the
// cutoff is raised by kLearnedCutSigmas times the model's RMS error on its
// training rows, lambda_max by kLearnedLmaxMargin of its distance above the
// cutoff) and the range the predicted degree is rounded and clamped into.
constexpr double kLearnedCutSigmas = 3.0;
constexpr double kLearnedLmaxMargin = 1.03;
constexpr int kLearnedDegMin = 16;
constexpr int kLearnedDegMax = 32;

// Dense FP64 generalized eigensolver: Hs y = lambda M y (n x n, 1 <= n <= kDenseMaxN).
constexpr int kDenseMaxN = 2800;  // bounded by the inverse-iteration LDS (7n doubles + n bytes)
struct DenseWork {
  static constexpr int kVecs = 11;   // lam, raw, d, e, ez, e2, tau, vbuf[2], pbuf[2]
  static constexpr int kIvecs = 4;   // perm, block start, block end, cluster start
  int n = 0;
  double *R = nullptr, *Rinv = nullptr, *C0 = nullptr, *C1 = nullptr, *T = nullptr;
  double* Vh = nullptr;        // Householder vectors, column k = v_k
  double* Z = nullptr;         // eigenvectors of the tridiagonal matrix
  double* vec = nullptr;       // kVecs * n doubles; the first n are the sorted eigenvalues
  double* scal = nullptr;      // |T|_1, pivot floor, then diag(M) at offset 16
  int32_t* flag = nullptr;     // device status flag (nonzero: M not positive definite)
  int32_t* ivec = nullptr;     // kIvecs * n ints + cluster count
  double* gemm_work = nullptr;
  size_t gemm_work_elems = 0;
  bool own_gemm_work = true;
  bool borrowed = false;  // every buffer carved from caller-owned memory (dense_free leaves them)
  const double* lam() const { return vec; }
};
// ext_work (may be null): a split-K workspace of ext_elems doubles owned by
// the caller (at least n*n), used instead of an own one.
void dense_alloc(DenseWork& w, int n, double* ext_work = nullptr, size_t ext_elems = 0);
void dense_free(DenseWork& w);
// device bytes dense_alloc takes for n (with or without its own split-K workspace)
size_t dense_bytes(int n, bool own_gemm_work);
// On XLS_OK, w.lam() (device, ascending) and Y (device, n x n, M-orthonormal
// columns) hold the result; XLS_ERR_NOT_SPD when M is not positive definite.
// Synchronises st once (after the Cholesky factorisation) when check_spd.
// With check_spd false nothing synchronises: the caller reads w.flag later
// (nonzero: not positive definite; the later stages then skip their work).
int dense_geneig(DenseWork& w, const double* Hs, const double* M, double* Y, hipStream_t st,
                 bool check_spd = true);

// Throws INVALID_ARG unless [p, p + bytes) lies inside one device allocation
// (host memory, pinned or not, is refused).
void check_device_range(const void* p, size_t bytes);

// vector helpers (vecops.hip)
template <typename TS>
void launch_convert_block(const double* src, int64_t lds_, TS* dst, int64_t ldd, int64_t rows,
                          int cols, hipStream_t st);
template <typename TS>
void launch_block_to_double(const TS* src, int64_t lds_, double* dst, int64_t ldd, int64_t rows,
                            int cols, hipStream_t st);
// out[c] = (sum_i num[c nper + i]) / (sum_i den[c nper + i]), both sums in
// the fixed order of launch_reduce_cols
void launch_reduce_rq(const double* num, const double* den, int nper, int ncols, double* out, hipStream_t st);
void launch_reduce_cols(const double* partial, int nper, int ncols, double* out, int take_sqrt,
                        hipStream_t st);
void launch_density(const double* lam, double mu, double sigma, const uint8_t* mask, double h,
                    const void* psi, int is_float, int64_t nd, int64_t ld, int ns, double* rho,
                    double* cpart, int nchunk, double* c, double* gocc, hipStream_t st);
// Start blocks drawn on the device: blk[g + j ld] for g < nd, j < ncols is the
// standard normal of counter (g, j, 0, 0) under key (seed mod 2^32,
// seed >> 32): Philox4x32-10 (Salmon et al., SC 2011) words (o0, o1, o2,
// o3), u1 = 1 - (2^26 (o0 >> 5) + (o1 >> 6)) 2^-53, u2 likewise from
// (o2, o3), x = sqrt(-2 ln u1) cos(2 pi u2) (Box-Muller), rounded to TS.
template <typename TS>
void launch_philox_block(TS* blk, int64_t ld, int64_t nd, int ncols, uint64_t seed, hipStream_t st);
// PDOS: P = alpha^2 / h^3 (ns x norb, row n), then D (norb x nbins) = sum of
// P[n][j] over lam_n in bin b for orbitals of atoms with in_core set.
void launch_pdos(const double* alpha, int ns, int norb, double h, const double* lam, const double* edges, int nbins,
                 const uint8_t* in_core, double* P, double* D, hipStream_t st);
// out[r + c ldo] = blk[rows[r] + c ld] for r < nrows, c < ncols
template <typename TS>
void launch_gather_rows(const TS* blk, int64_t ld, const int32_t* rows, int64_t nrows, int ncols, TS* out,
                        int64_t ldo, hipStream_t st);
// to_half: half[r + c nd] = binary16(blk[r + c ld]) (round to nearest even);
// otherwise blk[r + c ld] = half[r + c nd] widened (blk is written)
template <typename TS>
void launch_block_half(const TS* blk, int64_t ld, int64_t nd, int ncols, uint16_t* half, int to_half,
                       hipStream_t st);
// c[n] = sum over core points of psi_{g,n}^2 (no density)
void launch_core_weights(const uint8_t* mask, const void* psi, int is_float, int64_t nd, int64_t ld, int ns,
                         double* cpart, int nchunk, double* c, hipStream_t st);
// Fermi level of n states (device lam, c) for sigma and an electron count;
// out[0..5] = mu, N_e(mu), E_band, E_entropy, evaluations, status (1: count
// out of reach)
void launch_fermi_level(const double* lam, const double* c, int64_t n, double sigma, double target, int max_eval,
                        double* out, hipStream_t st);
// rho_global[gidx[g]] += rho[g] on core points
void launch_scatter_core(const double* rho, const uint8_t* mask, const int64_t* gidx, int64_t nd,
                         double* rho_global, hipStream_t st);
// dos[b] = 2 sum c over lam in bin b of edges[0..nbins]
void launch_dos(const double* lam, const double* c, int64_t n, const double* edges, int nbins, double* dos,
                hipStream_t st);
// Lanczos helpers
template <typename TS>
void launch_dot(const TS* x, const TS* y, int64_t n, double* partial, int nblocks, double* out,
                int take_sqrt, hipStream_t st);
// out[i] = sum_g V[i ldv + g] y[g] for i < m: nblocks partial sums per i
// (partial holds m * nblocks doubles), then a fixed-order reduction
template <typename TS>
void launch_multi_dot(const TS* V, int64_t ldv, int m, const TS* y, int64_t n, double* partial, int nblocks,
                      double* out, hipStream_t st);
template <typename TS>
void launch_lanczos_update(TS* w, const TS* v, const TS* vprev, const double* alpha_j,
                           const double* beta_prev, int64_t n, hipStream_t st);
template <typename TS>
void launch_reorth(TS* w, const TS* V, int64_t ldv, const double* coef, int k, int64_t n,
                   hipStream_t st);
template <typename TS>
void launch_scale_to(TS* dst, const TS* src, const double* norm, int64_t n, hipStream_t st);
void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);
void launch_tridiag_extremes(const double* alpha, const double* beta, int k, double* out,
                             hipStream_t st);

}  // namespace xls
