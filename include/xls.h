/*
 * xls.h — C ABI of the MI355X subdomain CheFSI engine.
 *
 * The engine solves the Kohn-Sham problem of one buffered divide-and-conquer
 * subdomain (Sec. V-A.2: the global effective potential restricted to the
 * subdomain box, the atoms whose nonlocal projectors reach it, a core box that
 * defines the binary partition of unity) by Chebyshev-filtered subspace
 * iteration (Sec. V-A.3), and assembles the subdomain's core density and
 * interior weights (Sec. V-A.4).
 *
 * Conventions for every call
 *  - Every entry point returns XLS_OK (0) or a negative status; no C++
 *    exception crosses the ABI.  xls_last_error() returns a thread-local
 *    message for the last failure on the calling thread.
 *  - Output arrays are written only when the call returns XLS_OK.
 *  - All pointers in this header are HOST pointers unless the name says
 *    "device".  Input arrays are read during the call and may be freed by the
 *    caller afterwards; the library owns every device allocation it makes.
 *  - Hartree atomic units: lengths in bohr, energies in Ha.
 *  - Grid node (i, j, k) sits at origin + h*(i, j, k); its linear index is
 *    g = i + n[0]*(j + n[1]*k) (x fastest).  A block of vectors is stored
 *    column-major N_d x ncols (column c starts at c*N_d).
 *  - A handle is used by one host thread at a time.  Different handles may
 *    run concurrently on different streams.  Results are bitwise
 *    reproducible for the same inputs on the same device (fixed reduction
 *    orders, no floating-point atomics).
 *  - Work is issued on the handle's stream (the one given at create, else a
 *    stream the library creates with default priority).  Calls that return
 *    host results synchronise that stream before returning.
 */
#ifndef XLS_H
#define XLS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define XLS_OK 0
#define XLS_ERR_INVALID_ARG (-1)  /* bad size, NULL, NaN/Inf input, unsupported option  */
#define XLS_ERR_OUT_OF_MEMORY (-2) /* a device allocation failed                        */
#define XLS_ERR_DEVICE (-3)       /* a HIP runtime call failed                           */
#define XLS_ERR_NOT_SPD (-4)      /* Cholesky of the overlap matrix M_s failed           */
#define XLS_ERR_EIG_NOCONV (-5)   /* the dense eigensolver did not converge              */
#define XLS_ERR_STATE (-6)        /* call not valid in the handle's current state        */

/* ---- enums ---------------------------------------------------------------- */
enum { XLS_BC_PERIODIC = 0, XLS_BC_DIRICHLET0 = 1 };
/* Storage / arithmetic precision.  XLS_PREC_BF16X3: FP32 operands split into
 * (hi, lo) bfloat16 pairs, products hi*hi + hi*lo + lo*hi on MFMA with FP32
 * accumulation (only meaningful for GEMMs). */
enum { XLS_PREC_FP64 = 0, XLS_PREC_FP32 = 1, XLS_PREC_BF16X3 = 2 };
enum { XLS_BOUNDS_GIVEN = 0, XLS_BOUNDS_LANCZOS = 1, XLS_BOUNDS_LEARNED = 2 };

/* ---- subdomain description ---------------------------------------------- */

/* Per-atom Kleinman-Bylander projector set (Sec. V-B.2, "Nonlocal
 * pseudopotential": projectors grouped by atom, gamma scaling).  Four
 * projectors s, px, py, pz with radial part exp(-r^2/(2 w^2)) (times x-X etc.
 * for p), support r^2 < rc^2, each normalised to h^3 sum chi^2 = 1 on the box;
 * V_nl psi = sum_j gamma_j chi_j (h^3 chi_j^T psi). */
typedef struct {
  double rc;          /* cutoff radius (bohr), > 0                      */
  double gauss_width; /* w (bohr), > 0                                   */
  double gamma[4];    /* Ha: s, px, py, pz                               */
} xls_projset_t;

typedef struct {
  int32_t n[3];            /* grid points per axis, each >= 1                              */
  double h;                /* grid spacing (bohr), > 0                                     */
  int32_t bc;              /* XLS_BC_PERIODIC (box = whole periodic cell) or XLS_BC_DIRICHLET0 */
  int32_t fd_n0;           /* half-width of the FD stencil; must be 6 (12th order, Sec. VI-A) */
  double origin[3];        /* coordinate of node (0,0,0)                                   */
  const double* v_eff;     /* [N_d] V_eff restricted to the box (Ha), finite              */
  int32_t n_atoms;         /* >= 0                                                          */
  const double* atom_xyz;  /* [3*n_atoms] positions; periodic: one copy per atom            */
  const xls_projset_t* proj; /* [n_atoms]                                                  */
  int32_t core_lo[3];      /* core = half-open index box [core_lo, core_hi) (Sec. V-A.2)   */
  int32_t core_hi[3];
  int64_t global_offset[3]; /* global index of local node (0,0,0) (may be negative)        */
  int64_t global_n[3];      /* global grid size, for the periodic local->global map       */
  int32_t ns;              /* number of vectors N_s, 1 <= ns <= N_d                         */
  const double* x0;        /* [N_d*ns] column-major start block (caller-seeded), or NULL:
                              drawn on the device from x0_seed (below)                      */
  const double* lanczos_v0; /* [N_d] Lanczos start vector, or NULL for column 0 of x0       */
  int32_t filter_prec;     /* storage and filter precision: XLS_PREC_FP64 or XLS_PREC_FP32  */
  void* stream;            /* hipStream_t to issue work on, or NULL                         */
  uint64_t x0_seed;        /* with x0 NULL: element (g, j) of the start block is the standard
                              normal of counter (g, j, 0, 0) under key (x0_seed mod 2^32,
                              x0_seed >> 32) of Philox4x32-10 (Salmon et al., SC 2011):
                              words o0..o3, u1 = 1 - (2^26 (o0>>5) + (o1>>6)) 2^-53, u2 from
                              (o2, o3) alike, x = sqrt(-2 ln u1) cos(2 pi u2) (Box-Muller),
                              rounded to the storage precision                            */
} xls_subdomain_desc_t;

typedef struct xls_subdomain_s* xls_subdomain_t;

/* Parameters of a CheFSI run (Sec. V-A.3).
 * First iteration bounds: XLS_BOUNDS_GIVEN takes (lam_lo, lam_cut, lam_max);
 * XLS_BOUNDS_LANCZOS runs lanczos_k Lanczos steps once per handle and takes
 * a0 = theta_min, lam_max = theta_max + |beta_k|, lam_cut = a0 + 0.1(lam_max - a0);
 * XLS_BOUNDS_LEARNED takes lam_max and lam_cut from the caller (the learned
 * model's prediction, xls_mlp_predict) and for a0 the rigorous lower bound
 * min V + sum of the negative projector coefficients (-1/2 Lap is positive
 * semi-definite), so no Lanczos run is needed; with fallback_tol > 0, if the
 * largest gated residual after the run exceeds fallback_tol (a NaN residual
 * counts as exceeding it) or an iteration finds M_s not positive definite,
 * the call restarts from the same start block with Lanczos bounds and
 * fallback_degree (<= 0: degree).  lanczos_k > 60 is INVALID_ARG.  Later iterations of the same call use
 * a0 = lambda_1 and lam_cut = lambda_ns of the previous iteration, lam_max
 * unchanged. */
typedef struct {
  int32_t bounds_mode;
  double lam_lo, lam_cut, lam_max;
  int32_t degree;          /* filter degree m >= 1                                 */
  int32_t max_iter;        /* >= 1                                                   */
  double resid_tol;        /* stop when max residual over the gated states <= this (0: never) */
  int32_t n_gate;          /* gated states (lowest n_gate); <= 0: floor(ns/1.1)     */
  int32_t lanczos_k;       /* Lanczos steps (<= 0: 20)                              */
  int32_t gemm_prec;       /* XLS_PREC_*: projection and rotation GEMMs; with BF16X3
                              both switch to FP32 once the previous iteration's
                              largest gated residual is <= 1e-2                  */
  double fallback_tol;     /* XLS_BOUNDS_LEARNED only: Lanczos restart above this (0: none) */
  int32_t fallback_degree; /* degree of the Lanczos restart (<= 0: degree)          */
} xls_chefsi_params_t;

/* ---- core calls ---------------------------------------------------------- */

/* Build a subdomain (Sec. V-A.2, V-B.2): copies V_eff and x0 to the device,
 * builds the core mask, the local->global map, the per-atom projector support
 * lists (sorted by grid index), projector values and the reverse CSR over grid
 * points.  Support rule, evaluated in FP64 without fused multiply-add:
 * dx = (origin_x + i*h) - X', r2 = (dx*dx + dy*dy) + dz*dz, member iff
 * r2 < rc*rc; periodic boxes sum the images X' = X + s*n*h, s in {-1,0,1}^3.
 * Errors: INVALID_ARG (sizes, NULL, non-finite input), OUT_OF_MEMORY, DEVICE. */
int xls_subdomain_create(const xls_subdomain_desc_t* desc, xls_subdomain_t* out);

/* Run up to p->max_iter CheFSI iterations on the handle's block (Sec. V-A.3):
 * filter Psi_f = p_m(H) Psi (scaled three-term recurrence, p(a0) = 1);
 * M_s = Psi_f^T Psi_f and H_s = Psi_f^T H Psi_f (upper block triangles;
 * H_s's diagonal tiles averaged with their transposes); Cholesky
 * M_s = R^T R; C = R^-T H_s R^-1; C = Z Lambda Z^T; Psi = Psi_f R^-1 Z;
 * residuals r_n = ||H psi_n - lambda_n psi_n||_2 in FP64 arithmetic.
 * Outputs: ritz[ns], resid[ns], *iters_done.  With an FP64 block and FP64
 * GEMMs ritz holds the eigenvalues lambda_n (ascending).  Otherwise (FP32
 * block, or FP32 / split-BF16 GEMMs) it holds the FP64 Rayleigh quotients
 * psi_n^T H psi_n / psi_n^T psi_n of the returned columns, taken in the same
 * FP64 sweep as the residuals.  They are second-order accurate in the
 * vectors' error and carry no GEMM rounding, and they are given in the order
 * of the lambda_n (a near-degenerate pair may differ from ascending in the
 * last bits).  resid is measured against lambda_n, and the next iteration's
 * bounds come from the lambda_n.  The handle keeps the rotated block and these
 * Ritz values for the next call and for density.
 * Errors: INVALID_ARG, NOT_SPD (the block is left as it was before the
 * failing iteration's rotation), EIG_NOCONV, DEVICE. */
int xls_chefsi_step(xls_subdomain_t s, const xls_chefsi_params_t* p,
                    double* ritz, double* resid, int32_t* iters_done);

/* Core density and interior weights of the current Ritz pairs (Sec. V-A.4):
 * g_n = 1/(1 + exp((lambda_n - mu)/sigma)); rho[g] = (2/h^3) sum_n g_n psi_{g,n}^2
 * on core points and 0 elsewhere; c[n] = sum over core points of psi_{g,n}^2.
 * Requires a completed xls_chefsi_step (else STATE); sigma > 0. */
int xls_subdomain_density(xls_subdomain_t s, double mu, double sigma, double* rho, double* c);

void xls_subdomain_destroy(xls_subdomain_t s);
const char* xls_last_error(void);

/* ---- stage calls (each one row of the hot path, for tests and benchmarks) */

/* HX = H X for a host block X [N_d*ncols] (Sec. V, eq. (ks) operator form):
 * -1/2 (12th-order FD Laplacian) + V_eff + V_nl, in the handle's filter
 * precision (FP32 handles round X to FP32).  ncols >= 1. */
int xls_hamiltonian_apply(xls_subdomain_t s, const double* X, double* HX, int32_t ncols);

/* Replace the handle's block by p_m(H) block (step (1) of Sec. V-A.3), scaled
 * so that p(a0) = 1: e = (lam_max - lam_cut)/2, c = (lam_max + lam_cut)/2.
 * Requires a0 < lam_cut < lam_max and degree >= 1. */
int xls_subdomain_filter(xls_subdomain_t s, int32_t degree, double a0, double lam_cut,
                         double lam_max);

/* Projection of the handle's block (step (2)): M = B^T B, Hs = B^T H B,
 * both ns x ns column-major FP64, GEMMs in gemm_prec.  Both products form
 * only their upper block triangle (tiles of 96 or 128): Hs is exactly
 * symmetric, with the entries of its diagonal tiles averaged with their
 * transposes and the rest mirrored from the upper triangle (the generalized
 * eigensolver of Sec. V-B.3 reads one triangle). */
int xls_subdomain_project(xls_subdomain_t s, int32_t gemm_prec, double* M, double* Hs);

/* Rotation (step (4)): block <- block * Q, Q ns x ns column-major FP64,
 * GEMM in gemm_prec. */
int xls_subdomain_rotate(xls_subdomain_t s, int32_t gemm_prec, const double* Q);

/* FP64 residuals of the handle's block against given values lam[ns]. */
int xls_subdomain_residual(xls_subdomain_t s, const double* lam, double* resid);

/* Lanczos bounds (k steps, full reorthogonalisation, from the handle's
 * Lanczos start vector): theta_min and theta_max + |beta_k|. */
int xls_lanczos_bounds(xls_subdomain_t s, int32_t k, double* theta_min, double* upper);

/* Dense generalized symmetric eigenproblem on the GPU (step (3); the
 * paper's DSYGVD stage, Sec. V-B.3), FP64: Hs y = lambda M y, n x n column-major
 * inputs; lam[n] ascending, Y[n*n] with Y^T M Y = I.  Cholesky, Householder
 * tridiagonalisation, bisection + inverse iteration, back-transformation;
 * 1 <= n <= 2800.  Errors: INVALID_ARG, NOT_SPD. */
int xls_dense_geneig(int32_t n, const double* Hs, const double* M, double* lam, double* Y);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as xls_dense_geneig, with Hs, M (n x n column-major), lam[n] and
 * Y[n*n] all DEVICE pointers owned by the caller, issued on stream (a
 * hipStream_t, NULL for the default stream) and synchronised before
 * returning.  Its workspace lives in a static device array of the library
 * (24 MiB per GPU, held until the process ends), so 1 <= n <= 512;
 * larger n, NULL or non-device pointers are INVALID_ARG; NOT_SPD as for
 * xls_dense_geneig.  The call makes no device allocation.  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (other
 * threads or streams) race, and must be serialised by the caller.  Results
 * are bit-identical to xls_dense_geneig's. */
int xls_dense_geneig_noalloc(int32_t n, const double* Hs, const double* M, double* lam, double* Y, void* stream);

int xls_subdomain_get_block(xls_subdomain_t s, double* X);       /* [N_d*ns] */
int xls_subdomain_set_block(xls_subdomain_t s, const double* X); /* [N_d*ns] */

/* FP16 orbital warm-start storage (Sec. V-B.2: orbital guesses are kept in
 * half precision between SCF iterations; all arithmetic stays in the
 * handle's precision).  Both buffers are DEVICE memory holding N_d*ns
 * IEEE binary16 values, column-major with leading dimension N_d, owned by
 * the caller (half the size of an FP32 block, a quarter of FP64).
 * xls_subdomain_store_half: dst receives the current block rounded to
 *   nearest even (|x| > 65504 becomes +-inf); the handle is unchanged.
 * xls_subdomain_load_half: the block is replaced by src widened exactly to
 *   the storage precision, as xls_subdomain_set_block would (Ritz values are
 *   dropped); the next xls_chefsi_step starts from it.
 * Both run on the handle's stream and return when it is done.  INVALID_ARG
 * for NULL, for a pointer that is not device memory (pageable or pinned
 * host memory included), or when the device allocation holding the pointer
 * ends before N_d*ns values (a buffer carved from a larger pooled
 * allocation is checked against that allocation only). */
int xls_subdomain_store_half(xls_subdomain_t s, uint16_t* dst);
int xls_subdomain_load_half(xls_subdomain_t s, const uint16_t* src);
/* The same warm start read in half precision by the filter itself (Sec.
 * V-B.2): src (as for xls_subdomain_load_half) becomes the handle's block
 * without a widening pass; the first filter step of the next
 * xls_chefsi_step or xls_subdomain_filter reads it as Y_0 and the second as
 * Y_{-1}, in binary16 (half the bytes of an FP32 block), with the
 * arithmetic in the handle's precision.  Results are those of
 * xls_subdomain_load_half followed by the same call (binary16 widens
 * exactly).  src must stay valid and unchanged until that call returns.
 * Calls that read the block before then (get_block, store_half, project,
 * rotate, residual, time_gemms, a learned run with the fallback) widen src
 * into the block first; set_block, load_half or another use_half replace
 * it.  Ritz values are dropped.  Errors as for xls_subdomain_load_half. */
int xls_subdomain_use_half(xls_subdomain_t s, const uint16_t* src);
/* Projected density of states (Sec. V-A.4, the PDOS equations): overlaps of
 * the handle's current block with atom-centred atomic orbitals and the
 * orbital-resolved PDOS.  The paper's atomic orbitals come with its
 * pseudopotentials; here each atom carries s, px, py, pz orbitals of the
 * projector shape (exp(-r^2/(2 w^2)), times x - X etc.; support r^2 <
 * rc^2 by the rule of xls_subdomain_create, periodic images summed) with
 * w = orb_width and rc = orb_rc, normalised so h^3 sum phi^2 = 1.  With the
 * block's columns psi_n (unit 2-norm, the continuum orbital being psi_n /
 * h^(3/2)): weights[n * 4 n_atoms + 4 I + l] = h^3 (sum_g phi_{I,l}(g)
 * psi_n(g))^2 (the squared overlap |<phi|psi_n>|^2), for every atom.  With
 * nbins > 0 (needs a completed xls_chefsi_step: STATE otherwise) and
 * increasing edges[nbins + 1]: pdos[(4 I + l) * nbins + b] = sum of the
 * weights of orbital (I, l) over the states with Ritz value in [edges[b],
 * edges[b+1]) (the last bin closed), for atoms in the core and 0 for the
 * others; an atom is in the core iff core_lo h <= X - origin < core_hi h on
 * every axis (in_core[n_atoms], may be NULL, receives those flags).  Atom-
 * and species-resolved PDOS are sums of these rows.  Host outputs; runs on
 * the handle's stream and synchronises it.  INVALID_ARG for non-positive or
 * non-finite w, rc, or non-increasing edges. */
int xls_subdomain_pdos(xls_subdomain_t s, double orb_width, double orb_rc, double* weights, int32_t nbins,
                       const double* edges, double* pdos, uint8_t* in_core);
/* Integer maps: core_mask u8[N_d], global_index i64[N_d]. */
int xls_subdomain_get_maps(xls_subdomain_t s, uint8_t* core_mask, int64_t* global_index);
/* sizes[0] = total support slots, sizes[1] = n_atoms.  With NULL arrays only
 * sizes is written.  offsets i32[n_atoms+1], idx i32[total] (grid index per slot),
 * val f64[4*total] (slot-major: s, px, py, pz), rev_offsets i32[N_d+1],
 * rev_slot i32[total] (slots covering each grid point, ascending). */
int xls_subdomain_get_projectors(xls_subdomain_t s, int64_t* sizes, int32_t* offsets,
                                 int32_t* idx, double* val, int32_t* rev_offsets,
                                 int32_t* rev_slot);

/* Split FP32 values into round-to-nearest-even bfloat16 (hi, lo) bit patterns
 * on the device: hi = bf16(a), lo = bf16(a - hi).  n >= 0. */
int xls_split_bf16(const float* a, uint16_t* hi, uint16_t* lo, int64_t n);

/* Launch shape of the handle's stencil sweeps in storage precision prec
 * (XLS_PREC_FP64 or XLS_PREC_FP32): block threads (256 or 512; 0: 256
 * when its per-thread halo budget covers the tile, else 512), ty rows
 * per tile (0: about 2 points per thread), tz planes per
 * z-chunk (0: the whole box), nv vectors per tile (1 or 2; 0: choose).  A
 * tile of 2 vectors reads the operator tables (V, projector entries) once
 * for both; residual sweeps always take 1.  The shape changes scheduling
 * only, never the arithmetic of a grid point.  Errors: INVALID_ARG when the
 * tile does not fit (LDS, registers, halo budget) or nv is not 0, 1 or 2. */
int xls_subdomain_tune(xls_subdomain_t s, int32_t prec, int32_t block, int32_t ty, int32_t tz, int32_t nv);

/* Launch plan of the handle's projection and rotation GEMMs (Sec. V-B.3:
 * split-K over the long N_d dimension).  split_scale 0 keeps the default
 * split count (about as many workgroups as are resident at once: two per
 * CU with 128 x 128 tiles, three with 96 x 96; at least 16 k-slabs per
 * split); k in [1, 64] scales it by k/2 (still bounded by K and the
 * workspace).  tile_tn (projection): 0 takes the large-tile MFMA kernel
 * when the shapes allow, with 96 x 96 tiles where they issue at least 10 %
 * less padded and redundant work than 128 x 128 (an order of 480, say) and
 * 128 x 128 otherwise; 1 the 64 x 64 tiles; 2 and 3 force the 128 and 96
 * edges of the large kernel (FP64 products of FP32 blocks always take
 * 128).  tile_nn (rotation): 0 and 3 take the large-tile kernel with
 * 64 x 128 tiles when the shapes allow, 1 the 64 x 64 tiles, 2 the large
 * kernel with 64 x 256 tiles.  A plan changes the
 * order of the split-K partial sums (results stay deterministic per plan),
 * never a product.  INVALID_ARG outside those ranges. */
int xls_subdomain_tune_gemm(xls_subdomain_t s, int32_t split_scale, int32_t tile_tn, int32_t tile_nn);

/* Profiling switch (process-wide, default off): with 1, xls_chefsi_step
 * records HIP events around its stages and every fused-filter launch. */
int xls_set_profiling(int32_t on);

/* Graph replay of fixed launch sequences (default on): after one eager call
 * with the same buffers, the dense FP64 stage of xls_chefsi_step is captured
 * into a hipGraph and replayed.  Results are identical either way; 0 launches
 * everything eagerly (tests compare the two). */
int xls_set_graphs(int32_t on);

/* Per-stage device time of the handle's last xls_chefsi_step, from HIP events
 * on the handle's stream when profiling is on (xls_set_profiling(1)).
 * ms[0] filter (all m sweeps), ms[1] H*Psi_f, ms[2] projection GEMMs,
 * ms[3] dense FP64, ms[4] rotation, ms[5] residual, ms[6] total, ms[7] sum of
 * the fused-filter stencil kernels alone (events around each launch);
 * counts[0] filter launches.  Returns the number of values written. */
int xls_get_stage_times(xls_subdomain_t s, double* ms, int64_t* counts, int32_t cap);

/* Device time of the projection and rotation GEMMs (steps (2) and (4) of
 * Sec. V-A.3: M_s = Psi^T Psi, H_s = Psi^T (H Psi), Psi Q) on the handle's
 * current block in precision gemm_prec (XLS_PREC_*; FP64 handles take FP64), from
 * HIP events around reps back-to-back launches after one warm-up:
 * ms[0] Psi^T Psi, ms[1] Psi^T (H Psi) (both on their upper block
 * triangle), ms[2]
 * Psi Q into the spare block (Q = I).  H Psi is computed first (untimed);
 * the current block is not changed.  ms holds 3 doubles; returns 3.
 * Errors: INVALID_ARG (NULL, reps < 1, precision). */
int xls_subdomain_time_gemms(xls_subdomain_t s, int32_t gemm_prec, int32_t reps, double* ms);

/* Work counters of the handle's last xls_chefsi_step: out[0] H applications
 * (one per vector: Lanczos steps, m*ns per filter, ns for H Psi_f and for the
 * residual), out[1] 1 if the learned-bounds run fell back to Lanczos,
 * out[2] CheFSI iterations including a fallback run.  Returns values written. */
int xls_subdomain_counters(xls_subdomain_t s, int64_t* out, int32_t cap);

/* ---- Learned filter bounds: a small MLP on the GPU ---------------------------
 * The paper leaves the source of the filter bounds open (Sec. V-A.3 defines the
 * filter by its centre and half-width only).  The model maps 64 features of a
 * subdomain (xls_subdomain_features) to (lam_max, lam_cut, degree); it is trained
 * by FP32 forward, backward and Adam kernels on labels the method itself
 * produces, and evaluated with bfloat16 weights and activations.
 * sizes[nsizes]: layer widths, sizes[0] <= 64 inputs, last <= 8 outputs, each
 * <= 256, at most 4 layers; ReLU between layers; parameters per layer: W
 * (fan_in x fan_out, row-major) then b.  params (NULL: zeros) has
 * xls_mlp_get_params(m, NULL, 0) floats.
 * xls_mlp_forward / xls_mlp_gradient: FP32, raw inputs and targets, B rows
 *   (row-major B x in, B x out); gradient of the mean squared error over all
 *   B*out entries, loss optional.
 * xls_mlp_train: Adam (lr, beta 0.9/0.999, eps 1e-8) over minibatches
 *   idx[offsets[s] .. offsets[s+1]) of the n training rows, s < nsteps; the
 *   Adam state persists across calls (reset by xls_mlp_set_params); losses[s]
 *   (may be NULL) receives each minibatch's loss before its update.
 * xls_mlp_set_norm: input standardisation (x - in_mean)/in_std and output
 *   de-standardisation y * out_std + out_mean used by xls_mlp_predict.
 * xls_mlp_predict: bfloat16 inference on B feature rows (f64[B x in]) ->
 *   out f64[B x outputs].
 * xls_mlp_fit: the whole training step of the learned bounds on raw data:
 *   F f64[n x in] and T f64[n x outputs] (row-major, finite) are standardised
 *   on the device (per column: mean and population standard deviation, 1 for
 *   a constant column), the model is trained as by xls_mlp_train on the
 *   standardised rows, keeps that standardisation for xls_mlp_predict, and
 *   records its RMS error per output on the n training rows with bfloat16
 *   inference (xls_mlp_train_rms).  minibatches as for xls_mlp_train:
 *   offsets[0] must be 0 and offsets must increase strictly; INVALID_ARG
 *   otherwise.
 * xls_mlp_train_rms: the per-output RMS error of the last fit (cap values at
 *   most); STATE before a fit.  Returns the number written.
 * xls_mlp_bounds: the bounds a learned CheFSI run takes for B subdomains'
 *   features (3-output models only, after a fit; STATE otherwise).  With the
 *   prediction (p_max, p_cut, p_deg): degree = round-half-even(p_deg)
 *   clamped to [16, 32]; p_cut is replaced by p_max/2 unless p_cut < p_max;
 *   lam_cut = p_cut + 3 rms_cut (a cutoff below the true lambda_ns damps
 *   wanted states, and the plain method's later cutoffs, Ritz values, are
 *   upper bounds for that reason); lam_max = lam_cut + 1.03 (p_max - lam_cut)
 *   (an estimate below the top of the spectrum lets the Chebyshev polynomial
 *   grow there), or lam_cut + 0.03|lam_cut| + 1e-3 Ha when that is not above
 *   lam_cut.  Outputs are host arrays of B values.
 * xls_learned_safe_bounds: the same margins for given (lam_max, lam_cut)
 *   pairs with cut margin cut_margin >= 0 (the labels' bounds use 0). */
typedef struct xls_mlp_s* xls_mlp_t;
int xls_mlp_create(int32_t nsizes, const int32_t* sizes, const float* params, xls_mlp_t* out);
void xls_mlp_destroy(xls_mlp_t m);
int xls_mlp_get_params(xls_mlp_t m, float* params, int64_t n);
int xls_mlp_set_params(xls_mlp_t m, const float* params, int64_t n);
int xls_mlp_set_norm(xls_mlp_t m, const float* in_mean, const float* in_std, const double* out_mean,
                     const double* out_std);
int xls_mlp_forward(xls_mlp_t m, const float* X, int32_t B, float* Y);
int xls_mlp_gradient(xls_mlp_t m, const float* X, const float* T, int32_t B, float* grads, float* loss);
int xls_mlp_train(xls_mlp_t m, const float* X, const float* T, int32_t n, const int32_t* idx,
                  const int32_t* offsets, int32_t nsteps, float lr, float* losses);
int xls_mlp_predict(xls_mlp_t m, const double* features, int32_t B, double* out);
int xls_mlp_fit(xls_mlp_t m, const double* F, const double* T, int32_t n, const int32_t* idx,
                const int32_t* offsets, int32_t nsteps, float lr, float* losses);
int xls_mlp_train_rms(xls_mlp_t m, double* rms, int32_t cap);
int xls_mlp_bounds(xls_mlp_t m, const double* features, int32_t B, double* lam_max, double* lam_cut,
                   int32_t* degree);
int xls_learned_safe_bounds(int32_t B, const double* lam_max, const double* lam_cut, double cut_margin,
                            double* lm_out, double* lc_out);
/* Features of a subdomain (f64[64], zero-padded): [0,32) histogram of V over
 * [min V, max V] (fractions, numpy.histogram bin rule), then atom count, n[0],
 * n[1], n[2], h, buffer width min(core_lo)*h, min V, max V, mean V, std V, ns,
 * projector count, sum |gamma|, core fraction, largest eigenvalue of -1/2 Lap
 * (periodic closed form).  V statistics are computed on the device. */
int xls_subdomain_features(xls_subdomain_t s, double* f);

/* ---- Batch engine: many uneven subdomains on one GPU -----------------------
 * The paper advances the subsystems assigned to a process independently
 * (Sec. V-B); a batch holds n of them on one device and advances them
 * together: every Chebyshev filter step of the whole batch is one persistent
 * launch per tile shape (work items = subdomain x tile), the rest of each
 * CheFSI iteration runs per subdomain on a small stream pool, and an
 * iteration's launches are captured into a hipGraph and replayed while the
 * set of unconverged subdomains is unchanged.  Results are bit-identical to
 * running xls_chefsi_step on each subdomain alone with the same parameters.
 *
 * xls_batch_create: descs[n] as for xls_subdomain_create (all with the same
 *   filter_prec; their stream fields are ignored).  Host arrays are copied.
 * xls_batch_chefsi: per_sub[n] parameters (degree <= 256, lanczos_k <= 60);
 *   runs each subdomain until its gated residual is <= resid_tol, its
 *   max_iter is reached or its bounds degenerate.  LEARNED subdomains with
 *   fallback_tol > 0 whose run ends with the gated residual above
 *   fallback_tol (NaN included) or with M_s not positive definite are then
 *   restarted from their start blocks with Lanczos bounds and
 *   fallback_degree in a second batched pass (xls_subdomain_counters of the
 *   subdomain's handle reports the fallback; iters counts both runs).  Outputs are
 *   concatenated in subdomain order: ritz_concat and resid_concat hold
 *   sum(ns_i) values, the Ritz values as xls_chefsi_step reports them (FP64
 *   Rayleigh quotients unless block and GEMMs are FP64); iters[n] and
 *   status[n] may be NULL.  status[i] is
 *   XLS_OK or XLS_ERR_NOT_SPD (that subdomain's block is then undefined); with
 *   status NULL such a failure is returned as the call's status.  use_graph:
 *   1 replays captured iterations, 0 launches eagerly (same results).
 * xls_batch_density: xls_subdomain_density of every subdomain, rho and c
 *   concatenated (sum N_d_i and sum ns_i values).
 * xls_batch_fermi: the Fermi level of the whole batch (Sec. V-A.5): with
 *   every subdomain's Ritz values lambda_n and interior weights c_n
 *   (Sec. V-A.4, computed here from the current blocks), the mu at which
 *   N_e(mu) = 2 sum_i sum_n g(lambda_n; mu, sigma) c_n equals n_electrons,
 *   by Newton steps kept inside a shrinking bracket (first bracket: the
 *   extreme Ritz values -/+ 40 sigma), on the device.  out (cap >= 1
 *   values): mu, N_e(mu), E_band = 2 sum g c lambda, E_entropy =
 *   -2 sigma sum c [g ln g + (1 - g) ln(1 - g)], count evaluations.  Needs a
 *   completed xls_batch_chefsi (else XLS_ERR_STATE); INVALID_ARG for sigma or
 *   n_electrons <= 0 or an n_electrons outside (N_e(lo), N_e(hi)).  Returns
 *   the number of values written.
 * xls_batch_assemble: at the mu and sigma of the last xls_batch_fermi, the
 *   global density (Sec. V-A.4) and the density of states.  rho_global (host,
 *   n_global doubles, or NULL to skip): the sum over subdomains of rho~ on
 *   their core points, placed by their local->global maps (subdomains are
 *   added in order, so the result is deterministic; cores are meant to
 *   partition the global grid).  INVALID_ARG when a core point maps outside
 *   [0, n_global) or two core points of one subdomain map to one global
 *   point.  dos (host, nbins doubles; edges holds nbins + 1 increasing
 *   values): 2 sum c_n over the states with lambda_n in [edges[b],
 *   edges[b+1]), the last bin closed on the right.  nbins = 0 skips it.
 * xls_batch_subdomain: borrowed handle of subdomain i (for the per-handle
 *   hooks); owned by the batch, never destroyed by the caller.
 * xls_batch_tune: times the fused filter kernel of one subdomain per shape
 *   class (precision, n[0], n[1] and n[2] rounded up to 8, boundary, atom
 *   count rounded up to 64; a member whose extents do not admit its class's
 *   shape keeps its own) over block {256, 512} x
 *   rows-per-tile {auto, 1, 2, 4, 8, 16} x vectors per tile {1, 2}, and the
 *   projection and rotation GEMMs of one subdomain per (precision, N_d
 *   rounded up to 32768, ns rounded up to 32) class over split scale {default, 1/2, 2, 4} x tile kind (FP32 GEMMs for
 *   FP32 batches), and applies the fastest to each class
 *   (xls_subdomain_tune, xls_subdomain_tune_gemm).  cache_path (may be
 *   NULL): JSON object "shape key": [block, ty, nv] and "gemm_... key":
 *   [split_scale, tile_tn, tile_nn]; known keys are taken from it without
 *   timing, new results are written back.
 *   tuned (may be NULL) = classes timed; best_ms (may be NULL) = sum over timed
 *   classes of the winning per-launch time.
 * xls_batch_stats: out[0] iterations of the last xls_batch_chefsi, out[1]
 *   graphs captured, out[2] graph replays, out[3] device time of those
 *   iterations (ms, events on the batch stream), out[4] the last one's,
 *   out[5] the largest device bytes of working sets resident at once (slot
 *   residency; 0 otherwise), out[6] the most subdomains active in one
 *   iteration.  Returns the number written (cap at most 7).
 *
 * Slot residency (xls_batch_create_slots): for batches whose blocks do not
 * all fit at once (a 256-subdomain draw holds ~170 GB per FP32 block set).
 * Creation builds every subdomain's operator tables only (and keeps a host
 * copy of a given x0; descs with x0 NULL draw their start blocks on the
 * device from x0_seed, which needs no host copy).  xls_batch_chefsi then
 * admits subdomains, largest N_d*ns*degree first, while the bytes of the
 * resident working sets (both blocks, projection, GEMM and dense
 * workspaces) stay within max_resident_bytes (0: 85 % of the free device
 * memory at creation; one subdomain is always admitted), loads each start
 * block (every call starts from X0), runs the same iterations as a resident
 * batch (bit-identical results), and when a subdomain finishes keeps only
 * its core rows (all the occupation calls read) and releases the rest, so
 * the next one can be admitted.  A learned-bounds fallback restarts from
 * X0.  xls_batch_density, _fermi and _assemble work as for resident
 * batches (rho is zero off the core in either case); per-handle calls that
 * need a block (xls_chefsi_step, get/set_block, filter, project, rotate,
 * residual, Lanczos bounds, half storage, GEMM timing, density) return
 * XLS_ERR_STATE on a handle of such a batch.  xls_batch_tune times each
 * shape class with a temporary working set. */
typedef struct xls_batch_s* xls_batch_t;
int xls_batch_create(int32_t n, const xls_subdomain_desc_t* descs, xls_batch_t* out);
int xls_batch_create_slots(int32_t n, const xls_subdomain_desc_t* descs, int64_t max_resident_bytes,
                           xls_batch_t* out);
int xls_batch_chefsi(xls_batch_t b, const xls_chefsi_params_t* per_sub, double* ritz_concat,
                     double* resid_concat, int32_t* iters, int32_t* status, int32_t use_graph);
int xls_batch_density(xls_batch_t b, double mu, double sigma, double* rho_concat, double* c_concat);
int xls_batch_fermi(xls_batch_t b, double sigma, double n_electrons, double* out, int32_t cap);
int xls_batch_assemble(xls_batch_t b, int64_t n_global, double* rho_global, int32_t nbins, const double* edges,
                       double* dos);
int xls_batch_subdomain(xls_batch_t b, int32_t i, xls_subdomain_t* out);
int xls_batch_tune(xls_batch_t b, const char* cache_path, int32_t* tuned, double* best_ms);
int xls_batch_stats(xls_batch_t b, double* out, int32_t cap);
void xls_batch_destroy(xls_batch_t b);

/* ---- Electrostatic Poisson solve (Sec. IV Poisson equation; Sec. V-B.1) ----
 * phi with -(1/(4 pi)) Lap phi = f on an n[0] x n[1] x n[2] grid (spacing h,
 * index g = i + n[0] (j + n[1] k)), Lap the 12th-order FD Laplacian of the
 * Hamiltonian with zero Dirichlet or periodic boundaries: A phi = 4 pi f
 * with A = -Lap, by CG in FP64 from phi = 0, stopped when ||r|| <= tol ||4 pi
 * f||.  Periodic: f is taken with its mean removed and phi is returned with
 * zero mean (the constants are A's null space).  Preconditioner (precond
 * 1): one FP32 multigrid V-cycle, finest level the 7-point Laplacian
 * (6 u - sum of the 6 neighbours)/h^2 applied matrix-free, coarse levels the
 * Galerkin operators P^T A P of trilinear prolongation (coarse point I on
 * fine point 2I + 1 for zero Dirichlet, n -> (n - 1)/2 with n odd; on 2I for
 * periodic, n -> n/2 with n even; levels are added while every axis
 * coarsens exactly to at least 3 (Dirichlet) or 4 (periodic) points, at
 * most max_levels (0: 8)); damped Jacobi (omega = 2/3) smoothing, 2 sweeps
 * before and after each coarse correction, 10 from zero on the coarsest
 * level; the zero start makes it symmetric.
 * xls_poisson_create: INVALID_ARG for sizes < 1, non-positive h, unknown bc.
 * xls_poisson_solve: f and phi host arrays of N values; info (may be NULL)
 *   receives [iterations, final relative residual, levels, wall ms].
 *   Returns XLS_OK also when max_iter is reached (info[1] tells).
 * xls_poisson_solve_device: the same solve with f and phi device arrays of N
 *   doubles (each inside one device allocation, else INVALID_ARG); f is not
 *   checked for finiteness (a NaN shows as info[1]).  Wall ms covers the
 *   device solve only.
 * xls_poisson_vcycle: z = the preconditioner applied to r (host arrays of
 *   N values), for tests. */
typedef struct xls_poisson_s* xls_poisson_t;
int xls_poisson_create(const int32_t* n, double h, int32_t bc, int32_t max_levels, xls_poisson_t* out);
int xls_poisson_solve(xls_poisson_t p, const double* f, double* phi, double tol, int32_t max_iter,
                      int32_t precond, double* info);
int xls_poisson_solve_device(xls_poisson_t p, const double* f, double* phi, double tol, int32_t max_iter,
                             int32_t precond, double* info);
int xls_poisson_vcycle(xls_poisson_t p, const double* r, double* z);
void xls_poisson_destroy(xls_poisson_t p);

#ifdef __cplusplus
}
#endif
#endif /* XLS_H */
