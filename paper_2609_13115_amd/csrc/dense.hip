// Dense FP64 generalized symmetric eigensolver for the subspace problem
// H_s y = lambda M_s y (Sec. V-A.3 step (3); the paper's DSYGVD stage of
// Sec. V-B.3: Cholesky of M_s, reduction to a standard problem, symmetric
// eigensolve, back-transformation).
//
//   M = R^T R        right-looking Cholesky, one launch per column; a pivot at
//                    or below n*eps*M_kk reports NOT_SPD
//   Rinv = R^-1      one workgroup per column, back-substitution in LDS
//   C = Rinv^T H Rinv, symmetrised (MFMA GEMMs)
//   C = Z L Z^T      two-sided block Jacobi: 32-index blocks paired round-robin,
//                    each pair's subproblem diagonalised in LDS by one
//                    workgroup, rotations applied to C and V; converged when
//                    off(C) <= 1e-14 |C|_F
//   Y = Rinv Z       with Z's columns ordered by ascending eigenvalue
// The paper reduces to tridiagonal form and runs implicit QL; Jacobi is used
// here because every step is a wide, regular, launch-parallel update and it
// converges in two or three sweeps once CheFSI's subspace is nearly settled.
#include <algorithm>
#include <cmath>

#include "xls_internal.h"

namespace xls {
namespace {

__global__ void copy_diag_kernel(const double* __restrict__ A, int n, double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = A[i + static_cast<int64_t>(i) * n];
}

// Schur-complement update of the trailing lower triangle by column k.
__global__ void chol_step_kernel(double* __restrict__ A, int n, int k, const double* __restrict__ diag0,
                                 int32_t* __restrict__ flag) {
  if (*flag) return;
  const double d = A[k + static_cast<int64_t>(k) * n];
  const double thr = static_cast<double>(n) * 2.220446049250313e-16 * diag0[k];
  if (!(d > thr)) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && threadIdx.y == 0) *flag = 1;
    return;
  }
  const int i = k + 1 + blockIdx.x * 16 + threadIdx.x;
  const int j = k + 1 + blockIdx.y * 16 + threadIdx.y;
  if (i >= n || j >= n || j > i) return;
  const double aik = A[i + static_cast<int64_t>(k) * n];
  const double ajk = A[j + static_cast<int64_t>(k) * n];
  A[i + static_cast<int64_t>(j) * n] -= aik * ajk / d;
}

// R (upper, column-major) from the factored lower triangle: R[j][i] = A[i][j]/sqrt(A[j][j]).
__global__ void chol_finish_kernel(const double* __restrict__ A, int n, double* __restrict__ R) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(n) * n) return;
  const int r = static_cast<int>(e % n), c = static_cast<int>(e / n);  // R[r][c]
  double v = 0.0;
  if (r <= c) v = A[c + static_cast<int64_t>(r) * n] / sqrt(A[r + static_cast<int64_t>(r) * n]);
  R[r + static_cast<int64_t>(c) * n] = v;
}

// Column j of R^-1 by back-substitution R x = e_j.
__global__ __launch_bounds__(256) void trinv_kernel(const double* __restrict__ R, int n,
                                                    double* __restrict__ Rinv) {
  extern __shared__ double b[];
  __shared__ double xi_s;
  const int j = blockIdx.x;
  for (int t = threadIdx.x; t < n; t += blockDim.x) b[t] = (t == j) ? 1.0 : 0.0;
  __syncthreads();
  for (int i = j; i >= 0; --i) {
    if (threadIdx.x == 0) xi_s = b[i] / R[i + static_cast<int64_t>(i) * n];
    __syncthreads();
    const double xi = xi_s;
    const double* Rc = R + static_cast<int64_t>(i) * n;
    for (int t = threadIdx.x; t < i; t += blockDim.x) b[t] -= Rc[t] * xi;
    if (threadIdx.x == 0) b[i] = xi;
    __syncthreads();
  }
  double* out = Rinv + static_cast<int64_t>(j) * n;
  for (int t = threadIdx.x; t < n; t += blockDim.x) out[t] = (t <= j) ? b[t] : 0.0;
}

__global__ void symmetrize_kernel(const double* __restrict__ A, int n, double* __restrict__ B) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(n) * n) return;
  const int r = static_cast<int>(e % n), c = static_cast<int>(e / n);
  B[e] = 0.5 * (A[e] + A[c + static_cast<int64_t>(r) * n]);
}

__global__ void identity_kernel(double* __restrict__ V, int n) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(n) * n) return;
  V[e] = (e % n == e / n) ? 1.0 : 0.0;
}

// Round-robin (circle method) pairing: at step s, position 0 is fixed and the
// other np-1 players rotate; pair k meets positions k and np-1-k.
__device__ __forceinline__ int rr_player(int pos, int s, int np) {
  return pos == 0 ? 0 : ((pos - 1 + s) % (np - 1)) + 1;
}

// off = sum_{i != j} C_ij^2, tot = sum C_ij^2, single workgroup, fixed order.
__global__ __launch_bounds__(256) void offnorm_kernel(const double* __restrict__ C, int n,
                                                      double* __restrict__ out) {
  __shared__ double so[256], st[256];
  double off = 0.0, tot = 0.0;
  const int64_t nn = static_cast<int64_t>(n) * n;
  for (int64_t e = threadIdx.x; e < nn; e += 256) {
    const double v = C[e];
    tot += v * v;
    if (e % n != e / n) off += v * v;
  }
  so[threadIdx.x] = off;
  st[threadIdx.x] = tot;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      so[threadIdx.x] += so[threadIdx.x + w];
      st[threadIdx.x] += st[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = so[0];
    out[1] = st[0];
  }
}

// Ascending order of the diagonal (ties by index): lam[rank] = d_i, perm[rank] = i.
__global__ void sort_diag_kernel(const double* __restrict__ C, int n, double* __restrict__ lam,
                                 int32_t* __restrict__ perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double di = C[i + static_cast<int64_t>(i) * n];
  int rank = 0;
  for (int j = 0; j < n; ++j) {
    const double dj = C[j + static_cast<int64_t>(j) * n];
    rank += (dj < di || (dj == di && j < i)) ? 1 : 0;
  }
  lam[rank] = di;
  perm[rank] = i;
}

__global__ void permute_cols_kernel(const double* __restrict__ V, const int32_t* __restrict__ perm, int n,
                                    double* __restrict__ T) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(n) * n) return;
  const int r = static_cast<int>(e % n), c = static_cast<int>(e / n);
  T[e] = V[r + static_cast<int64_t>(perm[c]) * n];
}

// ---------------------------------------------------------------------------
// Two-sided block Jacobi.  C is cut into blocks of BJ_NB indices; at each
// round-robin step the blocks are paired, every pair's (<= 2 BJ_NB)^2
// subproblem is diagonalised in LDS by one workgroup (cyclic Jacobi), and the
// pair rotations U_k are applied to C (C <- J^T C J, J = diag(U_k) after the
// pairing permutation) and to V (V <- V J) with register-tiled products.
// ---------------------------------------------------------------------------
constexpr int BJ_NB = 32;
constexpr int BJ_M = 2 * BJ_NB;  // largest subproblem
constexpr int BJ_LD = BJ_M + 1;   // padded LDS row

struct BlockPair {
  int a, b;          // block ids (b may be the empty padding block)
  int a0, am, b0, bm;
};

__device__ __forceinline__ BlockPair pair_of(int k, int s, int nblk, int nreal, int n) {
  BlockPair bp;
  const int x = rr_player(k, s, nblk), y = rr_player(nblk - 1 - k, s, nblk);
  bp.a = min(x, y);
  bp.b = max(x, y);
  bp.a0 = bp.a * BJ_NB;
  bp.am = bp.a < nreal ? min(n, bp.a0 + BJ_NB) - bp.a0 : 0;
  bp.b0 = bp.b * BJ_NB;
  bp.bm = bp.b < nreal ? min(n, bp.b0 + BJ_NB) - bp.b0 : 0;
  return bp;
}
__device__ __forceinline__ int pair_index(const BlockPair& bp, int i) {
  return i < bp.am ? bp.a0 + i : bp.b0 + (i - bp.am);
}

// One workgroup per block pair: diagonalise S = C[P,P] (m x m, m <= 64),
// writing the rotation U (column-major, leading dimension BJ_M) and diag.
__global__ __launch_bounds__(256) void bj_solve_kernel(const double* __restrict__ C, int n, int nblk, int nreal,
                                                       int s, int max_sweeps, double* __restrict__ Uo,
                                                       double* __restrict__ Do) {
  __shared__ double S[BJ_M * BJ_LD];
  __shared__ double U[BJ_M * BJ_LD];
  __shared__ double rc[BJ_M / 2], rs[BJ_M / 2], rt[BJ_M / 2];
  __shared__ int rp[BJ_M / 2], rq[BJ_M / 2], rid[BJ_M / 2];
  __shared__ double red[2][256];
  const int k = blockIdx.x, tid = threadIdx.x;
  const BlockPair bp = pair_of(k, s, nblk, nreal, n);
  const int m = bp.am + bp.bm;
  double* Uk = Uo + static_cast<int64_t>(k) * BJ_M * BJ_M;
  double* Dk = Do + static_cast<int64_t>(k) * BJ_M;
  if (m == 0) return;
  for (int e = tid; e < m * m; e += 256) {
    const int i = e % m, j = e / m;
    S[i + j * BJ_LD] = C[pair_index(bp, i) + static_cast<int64_t>(pair_index(bp, j)) * n];
    U[i + j * BJ_LD] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int M = m + (m & 1);
  const int half = M / 2;
  for (int sw = 0; sw < max_sweeps && m > 1; ++sw) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < m * m; e += 256) {
      const int i = e % m, j = e / m;
      const double v = S[i + j * BJ_LD];
      tot += v * v;
      if (i != j) off += v * v;
    }
    red[0][tid] = off;
    red[1][tid] = tot;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) {
        red[0][tid] += red[0][tid + w];
        red[1][tid] += red[1][tid + w];
      }
      __syncthreads();
    }
    const bool done = red[0][0] <= 1e-30 * red[1][0];
    __syncthreads();
    if (done) break;
    for (int st = 0; st < M - 1; ++st) {
      if (tid < half) {
        const int x = rr_player(tid, st, M), y = rr_player(M - 1 - tid, st, M);
        const int p = min(x, y), q = max(x, y);
        double c = 1.0, sn = 0.0, t = 0.0;
        int id = 1;
        if (q < m) {
          const double app = S[p + p * BJ_LD], aqq = S[q + q * BJ_LD], apq = S[p + q * BJ_LD];
          const double aapq = fabs(apq);
          if (!(aapq <= 1e-300 || (aapq < 1e-17 * fabs(app) && aapq < 1e-17 * fabs(aqq)))) {
            const double tau = (aqq - app) / (2.0 * apq);
            t = fabs(tau) > 1e150 ? 0.5 / tau : (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = t * c;
            id = 0;
          }
        }
        rc[tid] = c;
        rs[tid] = sn;
        rt[tid] = t;
        rp[tid] = p;
        rq[tid] = q;
        rid[tid] = id;
      }
      __syncthreads();
      // S <- J^T S J over disjoint 2x2 blocks (in place)
      for (int e = tid; e < half * half; e += 256) {
        const int bi = e % half, bj = e / half;
        const int P0 = rp[bi], P1 = rq[bi], Q0 = rp[bj], Q1 = rq[bj];
        const int P[2] = {P0, P1}, Qc[2] = {Q0, Q1};
        double a[2][2];
        for (int x = 0; x < 2; ++x)
          for (int y = 0; y < 2; ++y) a[x][y] = (P[x] < m && Qc[y] < m) ? S[P[x] + Qc[y] * BJ_LD] : 0.0;
        double o[2][2];
        if (bi == bj && !rid[bi]) {
          const double apq = a[0][1];
          o[0][0] = a[0][0] - rt[bi] * apq;
          o[1][1] = a[1][1] + rt[bi] * apq;
          o[0][1] = 0.0;
          o[1][0] = 0.0;
        } else {
          double b2[2][2];
          for (int x = 0; x < 2; ++x) {
            b2[x][0] = rc[bj] * a[x][0] - rs[bj] * a[x][1];
            b2[x][1] = rs[bj] * a[x][0] + rc[bj] * a[x][1];
          }
          for (int y = 0; y < 2; ++y) {
            o[0][y] = rc[bi] * b2[0][y] - rs[bi] * b2[1][y];
            o[1][y] = rs[bi] * b2[0][y] + rc[bi] * b2[1][y];
          }
        }
        for (int x = 0; x < 2; ++x)
          for (int y = 0; y < 2; ++y)
            if (P[x] < m && Qc[y] < m) S[P[x] + Qc[y] * BJ_LD] = o[x][y];
      }
      // U <- U J
      for (int e = tid; e < m * half; e += 256) {
        const int r = e % m, kk = e / m;
        if (rid[kk]) continue;
        const int p = rp[kk], q = rq[kk];
        const double x = U[r + p * BJ_LD], y = U[r + q * BJ_LD];
        U[r + p * BJ_LD] = rc[kk] * x - rs[kk] * y;
        U[r + q * BJ_LD] = rs[kk] * x + rc[kk] * y;
      }
      __syncthreads();
    }
  }
  for (int e = tid; e < m * m; e += 256) {
    const int i = e % m, j = e / m;
    Uk[i + j * BJ_M] = U[i + j * BJ_LD];
  }
  for (int i = tid; i < m; i += 256) Dk[i] = S[i + i * BJ_LD];
}

// 64 x 64 x 64 product R = op(A) B in LDS, 4 x 4 outputs per thread.
// TA: use A^T.  Matrices column-major with leading dimension BJ_LD.
template <bool TA>
__device__ __forceinline__ void bj_mm(const double* A, const double* B, double* R, int mi, int mk, int mj) {
  const int tid = threadIdx.x;
  const int ti = (tid % 16) * 4, tj = (tid / 16) * 4;
  double acc[4][4] = {};
  for (int l = 0; l < mk; ++l) {
    double av[4], bv[4];
    for (int x = 0; x < 4; ++x) av[x] = TA ? A[l + (ti + x) * BJ_LD] : A[(ti + x) + l * BJ_LD];
    for (int y = 0; y < 4; ++y) bv[y] = B[l + (tj + y) * BJ_LD];
    for (int x = 0; x < 4; ++x)
      for (int y = 0; y < 4; ++y) acc[x][y] += av[x] * bv[y];
  }
  for (int x = 0; x < 4; ++x)
    for (int y = 0; y < 4; ++y)
      if (ti + x < mi && tj + y < mj) R[(ti + x) + (tj + y) * BJ_LD] = acc[x][y];
}

// Apply the step's pair rotations.  Workgroups [0, npair^2): C blocks
// Cout[P_a, P_b] = U_a^T Cin[P_a, P_b] U_b (diagonal pairs get their
// eigenvalues, exact zeros elsewhere).  Workgroups beyond: V[rows, P_k] U_k.
__global__ __launch_bounds__(256) void bj_update_kernel(const double* __restrict__ Cin, double* __restrict__ Cout,
                                                        double* __restrict__ V, int n, int nblk, int nreal, int s,
                                                        const double* __restrict__ Uo,
                                                        const double* __restrict__ Do) {
  extern __shared__ double sm[];
  double* A = sm;
  double* Ua = sm + BJ_M * BJ_LD;
  double* Ub = sm + 2 * BJ_M * BJ_LD;
  double* T = sm + 3 * BJ_M * BJ_LD;
  const int npair = nblk / 2;
  const int tid = threadIdx.x;
  const int wg = blockIdx.x;
  if (wg < npair * npair) {
    const int ka = wg % npair, kb = wg / npair;
    const BlockPair pa = pair_of(ka, s, nblk, nreal, n), pb = pair_of(kb, s, nblk, nreal, n);
    const int ma = pa.am + pa.bm, mb = pb.am + pb.bm;
    if (ma == 0 || mb == 0) return;
    if (ka == kb) {
      for (int e = tid; e < ma * ma; e += 256) {
        const int i = e % ma, j = e / ma;
        Cout[pair_index(pa, i) + static_cast<int64_t>(pair_index(pa, j)) * n] =
            (i == j) ? Do[static_cast<int64_t>(ka) * BJ_M + i] : 0.0;
      }
      return;
    }
    const double* U1 = Uo + static_cast<int64_t>(ka) * BJ_M * BJ_M;
    const double* U2 = Uo + static_cast<int64_t>(kb) * BJ_M * BJ_M;
    for (int e = tid; e < BJ_M * BJ_M; e += 256) {
      const int i = e % BJ_M, j = e / BJ_M;
      A[i + j * BJ_LD] = (i < ma && j < mb) ? Cin[pair_index(pa, i) + static_cast<int64_t>(pair_index(pb, j)) * n] : 0.0;
      Ua[i + j * BJ_LD] = (i < ma && j < ma) ? U1[i + j * BJ_M] : 0.0;
      Ub[i + j * BJ_LD] = (i < mb && j < mb) ? U2[i + j * BJ_M] : 0.0;
    }
    __syncthreads();
    bj_mm<true>(Ua, A, T, BJ_M, BJ_M, BJ_M);  // T = Ua^T A
    __syncthreads();
    bj_mm<false>(T, Ub, A, BJ_M, BJ_M, BJ_M);  // A = T Ub
    __syncthreads();
    for (int e = tid; e < ma * mb; e += 256) {
      const int i = e % ma, j = e / ma;
      Cout[pair_index(pa, i) + static_cast<int64_t>(pair_index(pb, j)) * n] = A[i + j * BJ_LD];
    }
    return;
  }
  // V update: row block rb (64 rows), pair k
  const int v = wg - npair * npair;
  const int k = v % npair, rb = v / npair;
  const BlockPair pk = pair_of(k, s, nblk, nreal, n);
  const int mk = pk.am + pk.bm;
  if (mk == 0) return;
  const int r0 = rb * BJ_M, rm = min(n - r0, BJ_M);
  const double* Uk = Uo + static_cast<int64_t>(k) * BJ_M * BJ_M;
  for (int e = tid; e < BJ_M * BJ_M; e += 256) {
    const int i = e % BJ_M, j = e / BJ_M;
    A[i + j * BJ_LD] = (i < rm && j < mk) ? V[(r0 + i) + static_cast<int64_t>(pair_index(pk, j)) * n] : 0.0;
    Ua[i + j * BJ_LD] = (i < mk && j < mk) ? Uk[i + j * BJ_M] : 0.0;
  }
  __syncthreads();
  bj_mm<false>(A, Ua, T, BJ_M, BJ_M, BJ_M);
  __syncthreads();
  for (int e = tid; e < rm * mk; e += 256) {
    const int i = e % rm, j = e / rm;
    V[(r0 + i) + static_cast<int64_t>(pair_index(pk, j)) * n] = T[i + j * BJ_LD];
  }
}

inline unsigned nblk(int64_t n, int b) { return static_cast<unsigned>((n + b - 1) / b); }

}  // namespace

void dense_alloc(DenseWork& w, int n) {
  dense_free(w);
  w.n = n;
  const size_t nn = static_cast<size_t>(n) * n;
  auto al = [&](void** p, size_t bytes) {
    if (hipMalloc(p, std::max<size_t>(bytes, 256)) != hipSuccess)
      fail(XLS_ERR_OUT_OF_MEMORY, "dense workspace allocation failed");
  };
  al(reinterpret_cast<void**>(&w.R), nn * 8);
  al(reinterpret_cast<void**>(&w.Rinv), nn * 8);
  al(reinterpret_cast<void**>(&w.C0), nn * 8);
  al(reinterpret_cast<void**>(&w.C1), nn * 8);
  al(reinterpret_cast<void**>(&w.V), nn * 8);
  al(reinterpret_cast<void**>(&w.T), nn * 8);
  al(reinterpret_cast<void**>(&w.lam), static_cast<size_t>(n) * 8);
  al(reinterpret_cast<void**>(&w.scal), (static_cast<size_t>(n) + 16) * 8);
  al(reinterpret_cast<void**>(&w.flag), 64);
  al(reinterpret_cast<void**>(&w.perm), static_cast<size_t>(n) * 4);
  const size_t npair = ((n + 31) / 32 + 1) / 2 + 1;
  al(reinterpret_cast<void**>(&w.U), npair * 64 * 64 * 8);
  al(reinterpret_cast<void**>(&w.D), npair * 64 * 8);
  w.gemm_work_elems = gemm_tn_work_elems(n, n, n);
  al(reinterpret_cast<void**>(&w.gemm_work), w.gemm_work_elems * 8);
}

void dense_free(DenseWork& w) {
  double** ds[] = {&w.R, &w.Rinv, &w.C0, &w.C1, &w.V, &w.T, &w.lam, &w.scal, &w.gemm_work, &w.U, &w.D};
  for (double** p : ds)
    if (*p) {
      (void)hipFree(*p);
      *p = nullptr;
    }
  if (w.flag) (void)hipFree(w.flag);
  if (w.perm) (void)hipFree(w.perm);
  w.flag = nullptr;
  w.perm = nullptr;
  w.n = 0;
}

int dense_geneig(DenseWork& w, const double* Hs, const double* M, double* Y, hipStream_t st,
                 int* sweeps_out) {
  const int n = w.n;
  const int64_t nn = static_cast<int64_t>(n) * n;
  // --- Cholesky M = R^T R (factor a copy in C0) ---
  XLS_HIP(hipMemcpyAsync(w.C0, M, nn * 8, hipMemcpyDeviceToDevice, st));
  launch_fill_i32(w.flag, 0, 16, st);
  double* diag0 = w.scal + 16;
  hipLaunchKernelGGL(copy_diag_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, w.C0, n, diag0);
  for (int k = 0; k < n; ++k) {
    const int m = n - k - 1;
    const dim3 grid(std::max(1u, nblk(m, 16)), std::max(1u, nblk(m, 16)));
    hipLaunchKernelGGL(chol_step_kernel, grid, dim3(16, 16), 0, st, w.C0, n, k, diag0, w.flag);
  }
  XLS_LAUNCH_CHECK("chol_step_kernel");
  int32_t hflag = 0;
  XLS_HIP(hipMemcpyAsync(&hflag, w.flag, 4, hipMemcpyDeviceToHost, st));
  XLS_HIP(hipStreamSynchronize(st));
  if (hflag) return XLS_ERR_NOT_SPD;
  hipLaunchKernelGGL(chol_finish_kernel, dim3(nblk(nn, 256)), dim3(256), 0, st, w.C0, n, w.R);
  // --- Rinv ---
  const size_t trinv_smem = static_cast<size_t>(n) * sizeof(double);
  if (trinv_smem > 64 * 1024) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(trinv_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            static_cast<int>(trinv_smem)) != hipSuccess)
      fail(XLS_ERR_INVALID_ARG, "dense eigensolver: n too large for the triangular inverse");
  }
  hipLaunchKernelGGL(trinv_kernel, dim3(n), dim3(256), trinv_smem, st, w.R, n, w.Rinv);
  XLS_LAUNCH_CHECK("trinv_kernel");
  // --- C = Rinv^T Hs Rinv, symmetrised ---
  gemm_tn<double>(XLS_PREC_FP64, w.Rinv, n, Hs, n, n, n, n, w.T, n, 0, 0, w.gemm_work,
                  w.gemm_work_elems, st);
  gemm_nn<double>(XLS_PREC_FP64, w.T, n, w.Rinv, n, n, n, n, w.C1, n, nullptr, st);
  hipLaunchKernelGGL(symmetrize_kernel, dim3(nblk(nn, 256)), dim3(256), 0, st, w.C1, n, w.C0);
  hipLaunchKernelGGL(identity_kernel, dim3(nblk(nn, 256)), dim3(256), 0, st, w.V, n);
  // --- block Jacobi sweeps ---
  const int nreal = (n + BJ_NB - 1) / BJ_NB;
  const int nbk = nreal + (nreal & 1);
  const int npair = nbk / 2;
  const size_t upd_smem = 4 * static_cast<size_t>(BJ_M) * BJ_LD * sizeof(double);
  static bool smem_set = false;
  if (!smem_set) {
    XLS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(bj_update_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(upd_smem)));
    smem_set = true;
  }
  const int nrb = (n + BJ_M - 1) / BJ_M;
  double* cin = w.C0;
  double* cout = w.C1;
  int sweeps = 0;
  bool conv = (n == 1);
  double hs[2] = {0.0, 1.0};
  for (int sw = 0; sw < 40 && !conv; ++sw) {
    for (int s2 = 0; s2 < nbk - 1; ++s2) {
      hipLaunchKernelGGL(bj_solve_kernel, dim3(npair), dim3(256), 0, st, cin, n, nbk, nreal, s2, 12, w.U, w.D);
      hipLaunchKernelGGL(bj_update_kernel, dim3(npair * npair + npair * nrb), dim3(256), upd_smem, st, cin, cout,
                         w.V, n, nbk, nreal, s2, w.U, w.D);
      std::swap(cin, cout);
    }
    XLS_LAUNCH_CHECK("block Jacobi");
    ++sweeps;
    hipLaunchKernelGGL(offnorm_kernel, dim3(1), dim3(256), 0, st, cin, n, w.scal);
    XLS_HIP(hipMemcpyAsync(hs, w.scal, 16, hipMemcpyDeviceToHost, st));
    XLS_HIP(hipStreamSynchronize(st));
    if (!(hs[0] == hs[0]) || !(hs[1] == hs[1])) return XLS_ERR_EIG_NOCONV;
    conv = hs[0] <= 1e-28 * hs[1];
  }
  if (!conv && n > 1) {
    if (!(hs[0] <= 1e-20 * hs[1])) return XLS_ERR_EIG_NOCONV;
  }
  if (sweeps_out) *sweeps_out = sweeps;
  // --- ascending order, Y = Rinv Z ---
  hipLaunchKernelGGL(sort_diag_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, cin, n, w.lam, w.perm);
  hipLaunchKernelGGL(permute_cols_kernel, dim3(nblk(nn, 256)), dim3(256), 0, st, w.V, w.perm, n, w.T);
  gemm_nn<double>(XLS_PREC_FP64, w.Rinv, n, w.T, n, n, n, n, Y, n, nullptr, st);
  XLS_LAUNCH_CHECK("dense back-transform");
  return XLS_OK;
}

}  // namespace xls
