// Dense FP64 generalized symmetric eigensolver for the subspace problem
// H_s y = lambda M_s y (Sec. V-A.3 step (3); the paper's DSYGVD stage of
// Sec. V-B.3: Cholesky of M_s, reduction to a standard problem, symmetric
// eigensolve, back-transformation).
//
//   M = R^T R        right-looking Cholesky, one launch per column; a pivot at
//                    or below n*eps*M_kk reports NOT_SPD
//   Rinv = R^-1      one workgroup per column, back-substitution in LDS
//   C = Rinv^T H Rinv, symmetrised (MFMA GEMMs)
//   C = Z L Z^T      parallel cyclic Jacobi: each round-robin step rotates n/2
//                    disjoint (p, q) pairs at once, one launch per step; a
//                    sweep is n-1 steps; converged when off(C) <= 1e-14 |C|_F
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

struct Rot {
  int p, q;
  double c, s, t;
  bool id;
};

__device__ __forceinline__ Rot make_rot(const double* __restrict__ C, int n, int np, int s, int k) {
  Rot r;
  int a = rr_player(k, s, np), b = rr_player(np - 1 - k, s, np);
  r.p = min(a, b);
  r.q = max(a, b);
  r.c = 1.0;
  r.s = 0.0;
  r.t = 0.0;
  r.id = true;
  if (r.q >= n) return r;  // paired with the padding index
  const double app = C[r.p + static_cast<int64_t>(r.p) * n];
  const double aqq = C[r.q + static_cast<int64_t>(r.q) * n];
  const double apq = C[r.p + static_cast<int64_t>(r.q) * n];
  const double aapq = fabs(apq);
  if (aapq <= 1e-300 || (aapq < 1e-17 * fabs(app) && aapq < 1e-17 * fabs(aqq))) return r;
  const double tau = (aqq - app) / (2.0 * apq);
  double t;
  if (fabs(tau) > 1e150) {
    t = 0.5 / tau;
  } else {
    t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  }
  r.c = 1.0 / sqrt(1.0 + t * t);
  r.s = t * r.c;
  r.t = t;
  r.id = false;
  return r;
}

// One Jacobi step: Cout = J^T Cin J and V <- V J for the step's n/2 rotations.
// Threads [0, nb*nb) update 2x2 blocks of C; the rest update V (row, pair).
__global__ void jacobi_step_kernel(const double* __restrict__ Cin, double* __restrict__ Cout,
                                   double* __restrict__ V, int n, int np, int s) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int nb = np / 2;
  const int64_t ncb = static_cast<int64_t>(nb) * nb;
  if (e < ncb) {
    const int bi = static_cast<int>(e % nb), bj = static_cast<int>(e / nb);
    const Rot ri = make_rot(Cin, n, np, s, bi);
    const Rot rj = make_rot(Cin, n, np, s, bj);
    const int P[2] = {ri.p, ri.q}, Qc[2] = {rj.p, rj.q};
    double a[2][2];
    for (int x = 0; x < 2; ++x)
      for (int y = 0; y < 2; ++y)
        a[x][y] = (P[x] < n && Qc[y] < n) ? Cin[P[x] + static_cast<int64_t>(Qc[y]) * n] : 0.0;
    double out[2][2];
    if (bi == bj && !ri.id) {
      const double apq = a[0][1];
      out[0][0] = a[0][0] - ri.t * apq;
      out[1][1] = a[1][1] + ri.t * apq;
      out[0][1] = 0.0;
      out[1][0] = 0.0;
    } else {
      double b[2][2];  // columns: A J_j
      for (int x = 0; x < 2; ++x) {
        b[x][0] = rj.c * a[x][0] - rj.s * a[x][1];
        b[x][1] = rj.s * a[x][0] + rj.c * a[x][1];
      }
      for (int y = 0; y < 2; ++y) {  // rows: J_i^T (A J_j)
        out[0][y] = ri.c * b[0][y] - ri.s * b[1][y];
        out[1][y] = ri.s * b[0][y] + ri.c * b[1][y];
      }
    }
    for (int x = 0; x < 2; ++x)
      for (int y = 0; y < 2; ++y)
        if (P[x] < n && Qc[y] < n) Cout[P[x] + static_cast<int64_t>(Qc[y]) * n] = out[x][y];
    return;
  }
  const int64_t ev = e - ncb;
  if (ev >= static_cast<int64_t>(n) * nb) return;
  const int row = static_cast<int>(ev % n), k = static_cast<int>(ev / n);
  const Rot r = make_rot(Cin, n, np, s, k);
  if (r.id) return;
  double* vp = V + row + static_cast<int64_t>(r.p) * n;
  double* vq = V + row + static_cast<int64_t>(r.q) * n;
  const double x = *vp, y = *vq;
  *vp = r.c * x - r.s * y;
  *vq = r.s * x + r.c * y;
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
  w.gemm_work_elems = gemm_tn_work_elems(n, n, n);
  al(reinterpret_cast<void**>(&w.gemm_work), w.gemm_work_elems * 8);
}

void dense_free(DenseWork& w) {
  double** ds[] = {&w.R, &w.Rinv, &w.C0, &w.C1, &w.V, &w.T, &w.lam, &w.scal, &w.gemm_work};
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
  // --- Jacobi sweeps ---
  const int np = n + (n & 1);
  double* cin = w.C0;
  double* cout = w.C1;
  const int64_t work = static_cast<int64_t>(np / 2) * (np / 2) + static_cast<int64_t>(n) * (np / 2);
  int sweeps = 0;
  bool conv = (n == 1);
  double hs[2];
  for (int sw = 0; sw < 40 && !conv && np > 1; ++sw) {
    for (int s = 0; s < np - 1; ++s) {
      // every element of Cout is written by the step, so ping-pong needs no copy
      hipLaunchKernelGGL(jacobi_step_kernel, dim3(nblk(work, 256)), dim3(256), 0, st, cin, cout, w.V, n,
                         np, s);
      std::swap(cin, cout);
    }
    XLS_LAUNCH_CHECK("jacobi_step_kernel");
    ++sweeps;
    hipLaunchKernelGGL(offnorm_kernel, dim3(1), dim3(256), 0, st, cin, n, w.scal);
    XLS_HIP(hipMemcpyAsync(hs, w.scal, 16, hipMemcpyDeviceToHost, st));
    XLS_HIP(hipStreamSynchronize(st));
    if (!(hs[0] == hs[0]) || !(hs[1] == hs[1])) return XLS_ERR_EIG_NOCONV;
    conv = hs[0] <= 1e-28 * hs[1];
  }
  if (!conv && np > 1) {
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
