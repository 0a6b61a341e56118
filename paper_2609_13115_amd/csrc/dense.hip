// Dense FP64 generalized symmetric eigensolver for the subspace problem
// H_s y = lambda M_s y (Sec. V-A.3 step (3); the DSYGVD decomposition of
// Sec. V-B.3: Cholesky of M_s, reduction to a standard problem, reduction to
// tridiagonal form, tridiagonal eigensolve, back-transformation).
//
//   M = R^T R          blocked right-looking Cholesky, 32-column panels; a
//                      pivot at or below n*eps*M_kk reports NOT_SPD
//   Rinv = R^-1        one workgroup per column, back-substitution in LDS
//   C = Rinv^T H Rinv  MFMA GEMMs, symmetrised
//   C = Q T Q^T        Householder tridiagonalisation, one launch per column:
//                      every workgroup rebuilds the next Householder vector
//                      from the previous step's product (deferred rank-2
//                      update), then owns four trailing columns, applies the
//                      pending update to them and forms their part of C v
//   T = S L S^T        split at negligible off-diagonals; eigenvalues by
//                      Sturm-count multisection (one wavefront per eigenvalue);
//                      eigenvectors by inverse iteration with partial
//                      pivoting (one workgroup per cluster of close
//                      eigenvalues, modified Gram-Schmidt inside a cluster)
//   Y = Rinv Q S       reflectors applied in reverse order (LDS-resident
//                      column blocks), then an MFMA GEMM
// Every launch count depends on n only, never on the data.
// The paper's tridiagonal stage is implicit QL with the rotation sequence
// computed serially and applied across eigenvector rows in parallel; on a GPU
// that serial chain of square roots and divisions is latency bound, so the
// tridiagonal problem is solved with bisection and inverse iteration instead,
// which are parallel over eigenvalues.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "xls_handle.h"

namespace xls {
namespace {

constexpr double kEps = 2.220446049250313e-16;
constexpr double kSafeMin = 2.2250738585072014e-308;
constexpr int kPanel = 32;       // Cholesky panel width
constexpr int kInvIters = 3;     // inverse-iteration solves per vector in a cluster (2 when alone)
constexpr int kInvChunk = 16;    // steps of a sequential sweep whose inputs load together
constexpr double kOrtol = 1e-3;  // cluster gap, relative to |T|_1
constexpr int kSturmChunk = 16;  // rows of a Sturm-count recurrence read per LDS batch
constexpr int kTrdPre = 8;       // column values per lane loaded ahead in a tridiagonalisation step
constexpr int kTrdTail = 128;    // trailing steps done in one workgroup, block in LDS (m (m + 2) + 2m doubles);
                                 // the tail kernel's update gives each lane two rows, so at most 128

inline unsigned nblk(int64_t n, int b) { return static_cast<unsigned>((n + b - 1) / b); }

// 1/q from the hardware estimate and two Newton-Raphson steps (each squares
// the relative error), a few instructions shorter on the dependent chain
// than a correctly rounded division
__device__ __forceinline__ double rcp_nr(double q) {
  double r = __builtin_amdgcn_rcp(q);
  double e = fma(-q, r, 1.0);
  r = fma(r, e, r);
  e = fma(-q, r, 1.0);
  return fma(r, e, r);
}

// Cross-lane moves for wave reductions (full wave active at every call).
// Within each row of 16 lanes: rotate by 8, 4, 2, 1 (DPP row_ror), so every
// lane of a row ends with the row's result, in the same operand order; the
// four rows are then read out and combined in a fixed order.  Every lane
// returns the same bits.
template <int CTRL>
__device__ __forceinline__ double row_ror(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_value(double x, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                          __builtin_amdgcn_readlane(__double2loint(x), l));
}
// sum over each row of 16 lanes, in every lane of the row
__device__ __forceinline__ double row_sum(double v) {
  v += row_ror<0x128>(v);
  v += row_ror<0x124>(v);
  v += row_ror<0x122>(v);
  v += row_ror<0x121>(v);
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
  v = row_sum(v);
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, row_ror<0x128>(v));
  v = fmax(v, row_ror<0x124>(v));
  v = fmax(v, row_ror<0x122>(v));
  v = fmax(v, row_ror<0x121>(v));
  return fmax(fmax(lane_value(v, 0), lane_value(v, 16)), fmax(lane_value(v, 32), lane_value(v, 48)));
}
// Sum over a 256-thread workgroup in a fixed order; every thread gets the
// result and red[] is free again on return.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double s = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return s;
}
__device__ __forceinline__ double block_max(double v, double* red) {
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double s = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  return s;
}

// SplitMix64 finaliser (Steele, Lea and Flood 2014) mapped to [-1, 1): the
// start vector of inverse iteration for eigenvalue slot s.
__device__ __forceinline__ double start_value(uint32_t s, uint32_t j) {
  uint64_t z = ((static_cast<uint64_t>(s) << 32) | j) + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return static_cast<double>(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void copy_diag_kernel(const double* __restrict__ A, int n, double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = A[i + static_cast<int64_t>(i) * n];
}

// ---------------------------------------------------------------------------
// Cholesky.  Panel j0: every workgroup factors the nb x nb diagonal block of
// the (updated) upper triangle in LDS; workgroup 0 stores R11, the others
// solve R11^T R12 = A12 for 256 columns each (one column per thread).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void chol_panel_kernel(const double* __restrict__ A, int n, int j0, int nb,
                                                         const double* __restrict__ diag0,
                                                         int32_t* __restrict__ flag, double* __restrict__ R) {
  __shared__ double S[kPanel * (kPanel + 1)];
  if (*flag) return;
  const int tid = threadIdx.x;
  constexpr int LD = kPanel + 1;
  for (int e = tid; e < kPanel * kPanel; e += 256) {
    const int i = e % kPanel, j = e / kPanel;
    S[i + j * LD] = (i < nb && j < nb && i <= j) ? A[(j0 + i) + static_cast<int64_t>(j0 + j) * n] : 0.0;
  }
  __syncthreads();
  for (int kk = 0; kk < nb; ++kk) {
    const double piv = S[kk + kk * LD];
    if (!(piv > static_cast<double>(n) * kEps * diag0[j0 + kk])) {  // uniform across the workgroup
      if (blockIdx.x == 0 && tid == 0) *flag = 1;
      return;
    }
    const double r = sqrt(piv);
    __syncthreads();
    if (tid < nb) {
      if (tid > kk) S[kk + tid * LD] /= r;
      if (tid == kk) S[kk + kk * LD] = r;
    }
    __syncthreads();
    for (int e = tid; e < kPanel * kPanel; e += 256) {
      const int i = e % kPanel, j = e / kPanel;
      if (i > kk && i <= j && j < nb) S[i + j * LD] -= S[kk + i * LD] * S[kk + j * LD];
    }
    __syncthreads();
  }
  if (blockIdx.x == 0) {
    for (int e = tid; e < nb * nb; e += 256) {
      const int i = e % nb, j = e / nb;
      R[(j0 + i) + static_cast<int64_t>(j0 + j) * n] = (i <= j) ? S[i + j * LD] : 0.0;
    }
    return;
  }
  const int c = j0 + nb + (blockIdx.x - 1) * 256 + tid;
  if (c >= n) return;
  const double* a = A + static_cast<int64_t>(c) * n + j0;
  double x[kPanel];
#pragma unroll
  for (int i = 0; i < kPanel; ++i) {
    if (i < nb) {
      double s = a[i];
#pragma unroll
      for (int l = 0; l < i; ++l) s -= S[l + i * LD] * x[l];
      x[i] = s / S[i + i * LD];
    } else {
      x[i] = 0.0;
    }
  }
  double* out = R + static_cast<int64_t>(c) * n + j0;
#pragma unroll
  for (int i = 0; i < kPanel; ++i)
    if (i < nb) out[i] = x[i];
}

// Trailing update of the upper triangle: A22 -= R12^T R12 on 64 x 64 tiles
// (I <= J), 4 x 4 outputs per thread.
__global__ __launch_bounds__(256) void chol_update_kernel(double* __restrict__ A, const double* __restrict__ R,
                                                          int n, int j0, int nb, const int32_t* __restrict__ flag) {
  __shared__ double Ri[kPanel][64], Rj[kPanel][64];
  if (*flag) return;
  const int j1 = j0 + nb;
  // tile (I, J) from the upper-triangle enumeration idx = J (J + 1) / 2 + I
  const int idx = blockIdx.x;
  int J = static_cast<int>((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
  while ((J + 1) * (J + 2) / 2 <= idx) ++J;
  while (J * (J + 1) / 2 > idx) --J;
  const int I = idx - J * (J + 1) / 2;
  const int r0 = j1 + I * 64, c0 = j1 + J * 64;
  const int tid = threadIdx.x;
  for (int e = tid; e < kPanel * 64; e += 256) {
    const int l = e / 64, q = e % 64;
    Ri[l][q] = (l < nb && r0 + q < n) ? R[(j0 + l) + static_cast<int64_t>(r0 + q) * n] : 0.0;
    Rj[l][q] = (l < nb && c0 + q < n) ? R[(j0 + l) + static_cast<int64_t>(c0 + q) * n] : 0.0;
  }
  __syncthreads();
  const int ti = (tid % 16) * 4, tj = (tid / 16) * 4;
  double acc[4][4] = {};
  for (int l = 0; l < nb; ++l) {
    double av[4], bv[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) av[x] = Ri[l][ti + x];
#pragma unroll
    for (int y = 0; y < 4; ++y) bv[y] = Rj[l][tj + y];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] += av[x] * bv[y];
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int r = r0 + ti + x, c = c0 + tj + y;
      if (r < n && c < n) A[r + static_cast<int64_t>(c) * n] -= acc[x][y];
    }
}

// Column j of R^-1 by back-substitution R x = e_j.
__global__ __launch_bounds__(256) void trinv_kernel(const double* __restrict__ R, int n,
                                                    double* __restrict__ Rinv, const int32_t* __restrict__ flag) {
  extern __shared__ double b[];
  __shared__ double xi_s;
  if (*flag) return;
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

// ---------------------------------------------------------------------------
// Householder tridiagonalisation, step k (lower form: H_k = I - tau v v^T with
// v_{k+1} = 1, zero above).  On entry A holds the reduction with updates
// 0..k-2 applied to the columns that are still live; vbuf/pbuf slot (k+1)&1
// hold v_{k-1} and p_{k-1} = tau_{k-1} A v_{k-1}.  Every workgroup forms
// w_{k-1} = p - (tau/2)(p^T v) v and the updated column k, and from it the
// reflector (v_k, tau_k) and T's entries d_k, e_k; workgroup 0 stores them.
// Wave q of workgroup g then owns column i = k+1+4g+q: it applies the
// deferred update A -= v w^T + w v^T to rows >= k+1 and forms p_k[i].
// LDS: w, c/v and v_{k-1}, n doubles each.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void trd_step_kernel(double* __restrict__ A, int n, int k,
                                                       double* __restrict__ Vh, double* __restrict__ tau,
                                                       double* __restrict__ d, double* __restrict__ e,
                                                       double* __restrict__ vbuf, double* __restrict__ pbuf,
                                                       const int32_t* __restrict__ flag) {
  extern __shared__ double sm[];
  __shared__ double red[4];
  // the failure flag, the stored column k, this wave's trailing column and
  // the previous step's reflector, p and tau do not depend on this launch's
  // vector work: all of them are loaded before the flag is tested (every
  // address is in range either way), so their latencies overlap
  const int32_t failed = *flag;
  double* w = sm;
  double* cv = sm + n;
  double* vp = sm + 2 * n;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double* colk = A + static_cast<int64_t>(k) * n;
  double ck[kTrdPre];
#pragma unroll
  for (int r = 0; r < kTrdPre; ++r) {
    const int j = k + tid + 256 * r;
    ck[r] = (j < n) ? colk[j] : 0.0;
  }
  const int iown = k + 1 + blockIdx.x * 4 + wv;
  double* colown = A + static_cast<int64_t>(min(iown, n - 1)) * n;
  double co[kTrdPre];
#pragma unroll
  for (int r = 0; r < kTrdPre; ++r) {
    const int j = k + 1 + lane + 64 * r;
    co[r] = (iown < n && j < n) ? colown[j] : 0.0;
  }
  // the previous step's reflector, p and tau are loaded in the same batch
  const double* vprev = vbuf + ((k + 1) & 1) * static_cast<int64_t>(n);
  const double* pprev = pbuf + ((k + 1) & 1) * static_cast<int64_t>(n);
  double* vcur = vbuf + (k & 1) * static_cast<int64_t>(n);
  double* pcur = pbuf + (k & 1) * static_cast<int64_t>(n);
  double vr[kTrdPre], pr[kTrdPre];
  double tprev = 0.0;
  if (k > 0) {
    tprev = tau[k - 1];
#pragma unroll
    for (int r = 0; r < kTrdPre; ++r) {
      const int j = k + tid + 256 * r;
      vr[r] = (j < n) ? vprev[j] : 0.0;
      pr[r] = (j < n) ? pprev[j] : 0.0;
    }
  }
  if (failed) return;
  if (k > 0) {
    double part = 0.0;
#pragma unroll
    for (int r = 0; r < kTrdPre; ++r) {
      const int j = k + tid + 256 * r;
      if (j < n) {
        vp[j] = vr[r];
        part += pr[r] * vr[r];
      }
    }
    for (int j = k + tid + 256 * kTrdPre; j < n; j += 256) {
      const double vj = vprev[j];
      vp[j] = vj;
      part += pprev[j] * vj;
    }
    const double K = 0.5 * tprev * block_sum(part, red);
#pragma unroll
    for (int r = 0; r < kTrdPre; ++r) {
      const int j = k + tid + 256 * r;
      if (j < n) w[j] = pr[r] - K * vr[r];
    }
    for (int j = k + tid + 256 * kTrdPre; j < n; j += 256) w[j] = pprev[j] - K * vp[j];
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < kTrdPre; ++r) {
    const int j = k + tid + 256 * r;
    if (j < n) {
      double c = ck[r];
      if (k > 0) c -= vp[j] * w[k] + w[j] * vp[k];
      cv[j] = c;
    }
  }
  for (int j = k + tid + 256 * kTrdPre; j < n; j += 256) {
    double c = colk[j];
    if (k > 0) c -= vp[j] * w[k] + w[j] * vp[k];
    cv[j] = c;
  }
  __syncthreads();
  const double dk = cv[k], alpha = cv[k + 1];
  double part = 0.0;
  for (int j = k + 2 + tid; j < n; j += 256) part += cv[j] * cv[j];
  const double sig = block_sum(part, red);
  double t = 0.0, beta = alpha, sc = 0.0;
  if (sig > 0.0) {
    beta = -copysign(sqrt(alpha * alpha + sig), alpha);
    t = (beta - alpha) / beta;
    sc = 1.0 / (alpha - beta);
  }
  for (int j = k + 1 + tid; j < n; j += 256) cv[j] = (j == k + 1) ? 1.0 : (sig > 0.0 ? cv[j] * sc : 0.0);
  __syncthreads();
  if (blockIdx.x == 0) {
    if (tid == 0) {
      tau[k] = t;
      d[k] = dk;
      e[k] = beta;
    }
    for (int j = k + 1 + tid; j < n; j += 256) {
      Vh[j + static_cast<int64_t>(k) * n] = cv[j];
      vcur[j] = cv[j];
    }
  }
  const int i = iown;
  if (i >= n) return;
  const double wi = (k > 0) ? w[i] : 0.0, vpi = (k > 0) ? vp[i] : 0.0;
  double* col = colown;
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < kTrdPre; ++r) {
    const int j = k + 1 + lane + 64 * r;
    if (j < n) {
      double a = co[r];
      if (k > 0) a -= vp[j] * wi + w[j] * vpi;
      col[j] = a;
      acc += a * cv[j];
    }
  }
  for (int j = k + 1 + lane + 64 * kTrdPre; j < n; j += 64) {
    double a = col[j];
    if (k > 0) a -= vp[j] * wi + w[j] * vpi;
    col[j] = a;
    acc += a * cv[j];
  }
  acc = wave_sum(acc);
  if (lane == 0) pcur[i] = t * acc;
}

// The same step for trailing sizes n - k <= 64 kTrdPre.  Every wavefront
// forms the step's reflector itself, in registers: lane l holds entries
// j = k + l + 64 r of column k, of v_{k-1}, p_{k-1}, w_{k-1} and of its own
// trailing column, and every sum is a butterfly over the wave (each lane ends
// with the same bits), so there is no LDS traffic and no workgroup barrier.
// Every wave computes the same reflector bit for bit; workgroup 0's first
// wave stores it.
__global__ __launch_bounds__(256) void trd_step_wave_kernel(double* __restrict__ A, int n, int k,
                                                            double* __restrict__ Vh, double* __restrict__ tau,
                                                            double* __restrict__ d, double* __restrict__ e,
                                                            double* __restrict__ vbuf, double* __restrict__ pbuf,
                                                            const int32_t* __restrict__ flag) {
  constexpr int R = kTrdPre;
  const int32_t failed = *flag;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int iown = k + 1 + blockIdx.x * 4 + wv;
  const double* colk = A + static_cast<int64_t>(k) * n;
  double* colown = A + static_cast<int64_t>(min(iown, n - 1)) * n;
  const double* vprev = vbuf + ((k + 1) & 1) * static_cast<int64_t>(n);
  const double* pprev = pbuf + ((k + 1) & 1) * static_cast<int64_t>(n);
  double* vcur = vbuf + (k & 1) * static_cast<int64_t>(n);
  double* pcur = pbuf + (k & 1) * static_cast<int64_t>(n);
  // every load is issued before the failure flag is tested (all in range)
  double c[R], a[R], vp[R], w[R];
  const double tprev = (k > 0) ? tau[k - 1] : 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = k + lane + 64 * r;
    const bool in = j < n;
    c[r] = in ? colk[j] : 0.0;
    a[r] = (in && iown < n) ? colown[j] : 0.0;
    vp[r] = (in && k > 0) ? vprev[j] : 0.0;
    w[r] = (in && k > 0) ? pprev[j] : 0.0;  // p_{k-1} until w is formed
  }
  if (failed) return;
  if (k > 0) {
    double part = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) part += w[r] * vp[r];
    const double K = 0.5 * tprev * wave_sum(part);
#pragma unroll
    for (int r = 0; r < R; ++r) w[r] -= K * vp[r];
    const double wk = lane_value(w[0], 0), vpk = lane_value(vp[0], 0);
#pragma unroll
    for (int r = 0; r < R; ++r) c[r] -= vp[r] * wk + w[r] * vpk;
  }
  const double dk = lane_value(c[0], 0), alpha = lane_value(c[0], 1);
  double part = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = k + lane + 64 * r;
    if (j >= k + 2 && j < n) part += c[r] * c[r];
  }
  const double sig = wave_sum(part);
  double t = 0.0, beta = alpha, sc = 0.0;
  if (sig > 0.0) {
    beta = -copysign(sqrt(alpha * alpha + sig), alpha);
    t = (beta - alpha) / beta;
    sc = 1.0 / (alpha - beta);
  }
  double v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = k + lane + 64 * r;
    v[r] = (j == k + 1) ? 1.0 : ((j >= k + 2 && j < n && sig > 0.0) ? c[r] * sc : 0.0);
  }
  if (blockIdx.x == 0 && wv == 0) {
    if (lane == 0) {
      tau[k] = t;
      d[k] = dk;
      e[k] = beta;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = k + lane + 64 * r;
      if (j >= k + 1 && j < n) {
        Vh[j + static_cast<int64_t>(k) * n] = v[r];
        vcur[j] = v[r];
      }
    }
  }
  if (iown >= n) return;
  // w_{k-1} and v_{k-1} at row iown, from the lane and slot that hold them
  const int idx = iown - k, rsel = idx >> 6;
  double wsel = 0.0, vsel = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (r == rsel) {
      wsel = w[r];
      vsel = vp[r];
    }
  const double wi = lane_value(wsel, idx & 63), vpi = lane_value(vsel, idx & 63);
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = k + lane + 64 * r;
    if (j >= k + 1 && j < n) {
      const double x = (k > 0) ? a[r] - (vp[r] * wi + w[r] * vpi) : a[r];
      colown[j] = x;
      acc += x * v[r];
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) pcur[iown] = t * acc;
}

// The last m = n - k0 <= kTrdTail steps of the tridiagonalisation in one
// workgroup: the trailing m x m block (with step k0-1's deferred update
// applied on load) lives in LDS, column stride m + 2, and each step forms its
// reflector, p = tau A v, w = p - (tau/2)(p^T v) v and the rank-2 update
// there, with workgroup barriers in place of kernel boundaries.  Writes the
// same tau, d, e and Householder columns as the per-step kernels, and the
// final block back to A (its last diagonal entry is T's).
constexpr int kTailThreads = 1024;  // 16 waves: short dependent chains per lane, latency hidden across waves
__global__ __launch_bounds__(kTailThreads) void trd_tail_kernel(double* __restrict__ A, int n, int k0,
                                                                double* __restrict__ Vh, double* __restrict__ tau,
                                                                double* __restrict__ d, double* __restrict__ e,
                                                                const double* __restrict__ vbuf,
                                                                const double* __restrict__ pbuf,
                                                                const int32_t* __restrict__ flag) {
  constexpr int NT = kTailThreads, NW = NT / 64;
  extern __shared__ double sm[];
  __shared__ double red[2 * NW];  // two halves, used in turn: one barrier per sum
  if (*flag) return;
  const int m = n - k0, ld = m + 2, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double* As = sm;  // m columns of ld
  double* vs = sm + static_cast<int64_t>(m) * ld;
  double* ps = vs + m;  // p, then w
  int phase = 0;
  // fixed-order workgroup sum with one barrier; red's halves alternate
  auto bsum = [&](double v) {
    v = wave_sum(v);
    double* rr = red + NW * (phase & 1);
    ++phase;
    if (lane == 0) rr[wv] = v;
    __syncthreads();
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int q = 0; q < NW; q += 2) {
      s0 += rr[q];
      s1 += rr[q + 1];
    }
    return s0 + s1;
  };
  if (k0 > 0) {
    const double* vprev = vbuf + ((k0 - 1) & 1) * static_cast<int64_t>(n);
    const double* pprev = pbuf + ((k0 - 1) & 1) * static_cast<int64_t>(n);
    double part = 0.0;
    for (int r = tid; r < m; r += NT) {
      const double vv = vprev[k0 + r], pp = pprev[k0 + r];
      vs[r] = vv;
      ps[r] = pp;
      part += pp * vv;
    }
    const double K = 0.5 * tau[k0 - 1] * bsum(part);
    for (int r = tid; r < m; r += NT) ps[r] -= K * vs[r];
    __syncthreads();
  }
  for (int c = wv; c < m; c += NW) {
    const double* src = A + k0 + static_cast<int64_t>(k0 + c) * n;
    const double pc = (k0 > 0) ? ps[c] : 0.0, vc = (k0 > 0) ? vs[c] : 0.0;
    for (int r = lane; r < m; r += 64) {
      double x = src[r];
      if (k0 > 0) x -= vs[r] * pc + ps[r] * vc;
      As[r + c * ld] = x;
    }
  }
  __syncthreads();
  for (int k = 0; k + 1 < m; ++k) {
    const double* colk = As + k * ld;
    const double dk = colk[k], alpha = colk[k + 1];
    const int rk = k + 2 + tid;
    const double ck = (rk < m) ? colk[rk] : 0.0;
    const double sig = bsum(ck * ck);
    double t = 0.0, beta = alpha, sc = 0.0;
    if (sig > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + sig), alpha);
      t = (beta - alpha) / beta;
      sc = 1.0 / (alpha - beta);
    }
    {
      const int r = k + 1 + tid;
      if (r < m) {
        const double v = (r == k + 1) ? 1.0 : (sig > 0.0 ? colk[r] * sc : 0.0);
        vs[r] = v;
        Vh[(k0 + r) + static_cast<int64_t>(k0 + k) * n] = v;
      }
    }
    if (tid == 0) {
      tau[k0 + k] = t;
      d[k0 + k] = dk;
      e[k0 + k] = beta;
    }
    __syncthreads();
    // p_i = t sum_{j > k} A_ji v_j (a row of 16 lanes per column i > k) and
    // K = (t/2) p^T v
    double kpart = 0.0;
    for (int i0 = k + 1; i0 < m; i0 += NT / 16) {
      const int i = i0 + (tid >> 4), h = tid & 15;
      double acc = 0.0;
      if (i < m) {
        const double* col = As + i * ld;
        for (int r = k + 1 + h; r < m; r += 16) acc += col[r] * vs[r];
      }
      acc = row_sum(acc);
      if (i < m && h == 0) {
        const double pi = t * acc;
        ps[i] = pi;
        kpart += pi * vs[i];
      }
    }
    const double K = 0.5 * t * bsum(kpart);
    // A -= v w^T + w v^T with w = p - K v; lane rows r0, r0 + 64, wave columns
    const int r0 = k + 1 + lane, r1 = r0 + 64;
    const double v0 = (r0 < m) ? vs[r0] : 0.0, w0 = (r0 < m) ? ps[r0] - K * v0 : 0.0;
    const double v1 = (r1 < m) ? vs[r1] : 0.0, w1 = (r1 < m) ? ps[r1] - K * v1 : 0.0;
    for (int c = k + 1 + wv; c < m; c += NW) {
      const double vc = vs[c], wc = ps[c] - K * vc;
      double* col = As + c * ld;
      if (r0 < m) col[r0] -= v0 * wc + w0 * vc;
      if (r1 < m) col[r1] -= v1 * wc + w1 * vc;
    }
    __syncthreads();
  }
  for (int c = wv; c < m; c += NW) {
    double* dst = A + k0 + static_cast<int64_t>(k0 + c) * n;
    for (int r = lane; r < m; r += 64) dst[r] = As[r + c * ld];
  }
}

// T's last diagonal entry, |T|_1, negligible off-diagonals set to zero
// (|e_i| <= eps |T|_1), and for every row the [start, end) of its unreduced
// block.  scal[0] = |T|_1, scal[1] = pivot floor of the Sturm recurrence.
__global__ __launch_bounds__(256) void tri_prepare_kernel(const double* __restrict__ A, int n,
                                                          double* __restrict__ d, const double* __restrict__ e,
                                                          double* __restrict__ ez, double* __restrict__ e2,
                                                          int32_t* __restrict__ bs, int32_t* __restrict__ be,
                                                          double* __restrict__ scal,
                                                          const int32_t* __restrict__ flag) {
  __shared__ double red[4];
  __shared__ int last_start[256], first_start[256];
  if (*flag) return;
  const int tid = threadIdx.x;
  const double dlast = A[(n - 1) + static_cast<int64_t>(n - 1) * n];
  if (tid == 0) d[n - 1] = dlast;
  double rmax = 0.0;
  for (int i = tid; i < n; i += 256) {
    const double di = (i == n - 1) ? dlast : d[i];
    const double r = fabs(di) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
    rmax = fmax(rmax, r);
  }
  const double tn = block_max(rmax, red);
  double emax = 0.0;
  for (int i = tid; i + 1 < n; i += 256) {
    const double v = (fabs(e[i]) <= kEps * tn) ? 0.0 : e[i];
    ez[i] = v;
    e2[i] = v * v;
    emax = fmax(emax, v * v);
  }
  const double e2max = block_max(emax, red);
  if (tid == 0) {
    scal[0] = tn;
    scal[1] = kSafeMin * fmax(1.0, e2max);
  }
  // row j starts a block when j == 0 or e_{j-1} is negligible; contiguous
  // chunks per thread, prefix max / suffix min over the chunk summaries.
  auto starts = [&](int j) { return j == 0 || fabs(e[j - 1]) <= kEps * tn; };
  const int C = (n + 255) / 256;
  const int j0 = min(n, tid * C), j1 = min(n, j0 + C);
  int ls = -1, fs = n;
  for (int j = j0; j < j1; ++j)
    if (starts(j)) {
      ls = j;
      if (fs == n) fs = j;
    }
  last_start[tid] = ls;
  first_start[tid] = fs;
  __syncthreads();
  int cur = -1;
  for (int u = 0; u < tid; ++u) cur = max(cur, last_start[u]);
  for (int j = j0; j < j1; ++j) {
    if (starts(j)) cur = j;
    bs[j] = cur;
  }
  int nxt = n;
  for (int u = 255; u > tid; --u) nxt = min(nxt, first_start[u]);
  for (int j = j1 - 1; j >= j0; --j) {
    be[j] = nxt;
    if (starts(j)) nxt = j;
  }
}

// Eigenvalue slot s (one wavefront): the (s - start)-th smallest eigenvalue of
// the block that contains row s, by 65-section on Sturm counts (LDL^T pivots
// of T - x I): each lane counts at one of 64 interior points, and the first
// lane whose count exceeds the index bounds the new interval, which shrinks
// 65-fold per pass (about 9 passes to full precision instead of 54 halvings).
__global__ __launch_bounds__(64) void tri_multisect_kernel(const double* __restrict__ d,
                                                           const double* __restrict__ ez,
                                                           const double* __restrict__ e2,
                                                           const int32_t* __restrict__ bs,
                                                           const int32_t* __restrict__ be,
                                                           const double* __restrict__ scal, int n,
                                                           double* __restrict__ lam,
                                                           const int32_t* __restrict__ flag) {
  extern __shared__ double sh[];
  if (*flag) return;
  const int s = blockIdx.x, lane = threadIdx.x;
  const int s0 = bs[s], s1 = be[s], l = s - s0, m = s1 - s0;
  double* dd = sh;
  double* ee = sh + n;
  const double tn = scal[0], pivmin = scal[1];
  double gl = HUGE_VAL, gu = -HUGE_VAL;
  for (int j = lane; j < m; j += 64) {
    const int i = s0 + j;
    dd[j] = d[i];
    ee[j] = (j + 1 < m) ? e2[i] : 0.0;
    const double r = (j > 0 ? fabs(ez[i - 1]) : 0.0) + (j + 1 < m ? fabs(ez[i]) : 0.0);
    gl = fmin(gl, d[i] - r);
    gu = fmax(gu, d[i] + r);
  }
  for (int o = 32; o > 0; o >>= 1) {
    gl = fmin(gl, __shfl_xor(gl, o, 64));
    gu = fmax(gu, __shfl_xor(gu, o, 64));
  }
  __syncthreads();
  const double atol = 0.5 * kEps * tn;
  double lo = gl - 2.0 * kEps * tn - pivmin, hi = gu + 2.0 * kEps * tn + pivmin;
  for (int pass = 0; pass < 40; ++pass) {
    if (hi - lo <= fmax(2.0 * kEps * fmax(fabs(lo), fabs(hi)), atol)) break;
    const double x = lo + (hi - lo) * (static_cast<double>(lane + 1) / 65.0);
    int cnt = 0;
    double q = dd[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
    // The recurrence in chunks of kSturmChunk rows whose d and e^2 are read
    // from LDS up front (clamped, in range): the chain then waits on its
    // own arithmetic only, not on an LDS read per row.  Same operations in
    // the same order as a row-by-row loop.
    for (int j0 = 1; j0 < m; j0 += kSturmChunk) {
      double dv[kSturmChunk], ev[kSturmChunk];
#pragma unroll
      for (int t = 0; t < kSturmChunk; ++t) {
        const int j = min(j0 + t, m - 1);
        dv[t] = dd[j];
        ev[t] = ee[j - 1];
      }
#pragma unroll
      for (int t = 0; t < kSturmChunk; ++t) {
        if (j0 + t < m) {
          q = (dv[t] - x) - ev[t] * rcp_nr(q);
          if (fabs(q) < pivmin) q = -pivmin;
          cnt += q < 0.0;
        }
      }
    }
    const uint64_t above = __ballot(cnt > l);
    const double xprev = __shfl_up(x, 1, 64);
    if (above == 0) {
      lo = __shfl(x, 63, 64);
    } else {
      const int j = __ffsll(static_cast<unsigned long long>(above)) - 1;  // first lane counting past l
      const double nlo = (j == 0) ? lo : __shfl(xprev, j, 64);
      hi = __shfl(x, j, 64);
      lo = nlo;
    }
    if (!(lo < hi)) break;
  }
  if (lane == 0) lam[s] = 0.5 * (lo + hi);
}

// Clusters: a new cluster starts at every block start and wherever the gap to
// the previous eigenvalue of the block exceeds kOrtol |T|_1.  cstart lists the
// first slot of each cluster, ncl their number.
__global__ __launch_bounds__(256) void tri_cluster_kernel(const double* __restrict__ lam,
                                                          const int32_t* __restrict__ bs,
                                                          const double* __restrict__ scal, int n,
                                                          int32_t* __restrict__ cstart, int32_t* __restrict__ ncl,
                                                          const int32_t* __restrict__ flag) {
  __shared__ int cnt[256];
  if (*flag) return;
  const double ortol = kOrtol * scal[0];
  const int tid = threadIdx.x, C = (n + 255) / 256;
  const int j0 = min(n, tid * C), j1 = min(n, j0 + C);
  auto first = [&](int s) { return s == bs[s] || lam[s] - lam[s - 1] > ortol; };
  int c = 0;
  for (int s = j0; s < j1; ++s) c += first(s) ? 1 : 0;
  cnt[tid] = c;
  __syncthreads();
  int off = 0;
  for (int u = 0; u < tid; ++u) off += cnt[u];
  if (tid == 255) *ncl = off + c;
  for (int s = j0; s < j1; ++s)
    if (first(s)) cstart[off++] = s;
}

// One workgroup per cluster: for each slot s of the cluster, in order, inverse
// iteration on the cluster's block with shift lam_s (raised to at least the
// previous shift + 10 eps |T|_1 so that equal eigenvalues get distinct
// vectors): LU of T - x I with partial pivoting (thread 0), kInvIters solves,
// each followed by modified Gram-Schmidt against the cluster's earlier vectors
// and normalisation.  Column s of Z receives the vector (zero off the block).
// LDS: d, e, u0^-1, u1, u2, multipliers, x (m doubles each) and pivots.
__global__ __launch_bounds__(256) void tri_inviter_kernel(const double* __restrict__ d,
                                                          const double* __restrict__ ez,
                                                          const int32_t* __restrict__ bs,
                                                          const int32_t* __restrict__ be,
                                                          const double* __restrict__ lam,
                                                          const int32_t* __restrict__ cstart,
                                                          const int32_t* __restrict__ ncl,
                                                          const double* __restrict__ scal, int n,
                                                          double* __restrict__ Z, const int32_t* __restrict__ flag) {
  extern __shared__ double sm[];
  __shared__ double red[4];
  if (*flag) return;
  const int c = blockIdx.x, nc = *ncl;
  if (c >= nc) return;
  const int tid = threadIdx.x;
  const int sb = cstart[c], se = (c + 1 < nc) ? cstart[c + 1] : n;
  const int s0 = bs[sb], s1 = be[sb], m = s1 - s0;
  double* dd = sm;
  double* ee = sm + n;
  double* r0 = sm + 2 * n;
  double* u1 = sm + 3 * n;
  double* u2 = sm + 4 * n;
  double* ll = sm + 5 * n;
  double* x = sm + 6 * n;
  uint8_t* piv = reinterpret_cast<uint8_t*>(sm + 7 * n);
  for (int j = tid; j < m; j += 256) {
    dd[j] = d[s0 + j];
    ee[j] = (j + 1 < m) ? ez[s0 + j] : 0.0;
  }
  __syncthreads();
  const double tn = scal[0];
  const double pertol = 10.0 * kEps * tn;
  const double pmin = fmax(1e-3 * kEps * tn, 1e-150);  // pivot floor; growth stays far from overflow
  double xprev = 0.0;
  for (int s = sb; s < se; ++s) {
    double xs = lam[s];
    if (s > sb && xs - xprev < pertol) xs = xprev + pertol;
    xprev = xs;
    // The three sequential sweeps below (LU, forward, backward) run on one
    // thread.  Each loads kInvChunk steps' inputs into registers before it
    // runs them, so the dependent chain waits on LDS once per chunk instead
    // of once per step (the arrays share one LDS block, so the compiler
    // cannot move a load above an earlier store by itself).
    if (tid == 0) {
      double bb = dd[0] - xs, cc = ee[0];
      for (int i0 = 0; i0 + 1 < m; i0 += kInvChunk) {
        const int nstep = min(kInvChunk, m - 1 - i0);
        double ea[kInvChunk + 1], db[kInvChunk];
#pragma unroll
        for (int t = 0; t <= kInvChunk; ++t) ea[t] = ee[min(i0 + t, m - 1)];
#pragma unroll
        for (int t = 0; t < kInvChunk; ++t) db[t] = dd[min(i0 + 1 + t, m - 1)];
#pragma unroll
        for (int t = 0; t < kInvChunk; ++t) {
          if (t < nstep) {
            const int i = i0 + t;
            const double a = ea[t], b = db[t] - xs, cn = ea[t + 1];
            const double ra = rcp_nr(a);  // depends on the inputs only: off the recurrence's chain
            if (fabs(a) > fabs(bb)) {
              piv[i] = 1;
              r0[i] = ra;
              u1[i] = b;
              u2[i] = cn;
              const double mult = bb * ra;
              ll[i] = mult;
              bb = cc - mult * b;
              cc = -mult * cn;
            } else {
              piv[i] = 0;
              const double p = (fabs(bb) < pmin) ? copysign(pmin, bb) : bb;
              const double rp = rcp_nr(p);
              r0[i] = rp;
              u1[i] = cc;
              u2[i] = 0.0;
              const double mult = a * rp;
              ll[i] = mult;
              bb = b - mult * cc;
              cc = cn;
            }
          }
        }
      }
      r0[m - 1] = rcp_nr((fabs(bb) < pmin) ? copysign(pmin, bb) : bb);
    }
    double part = 0.0;
    for (int j = tid; j < m; j += 256) {
      const double b = start_value(static_cast<uint32_t>(s), static_cast<uint32_t>(j));
      x[j] = b;
      part += b * b;
    }
    const double scale0 = 1.0 / sqrt(block_sum(part, red));
    for (int j = tid; j < m; j += 256) x[j] *= scale0;
    __syncthreads();
    const int iters = (se - sb == 1) ? kInvIters - 1 : kInvIters;  // clusters get one more solve
    for (int it = 0; it < iters; ++it) {
      if (tid == 0) {
        double cur = x[0];
        for (int i0 = 0; i0 + 1 < m; i0 += kInvChunk) {
          const int nstep = min(kInvChunk, m - 1 - i0);
          double xn[kInvChunk], lc[kInvChunk];
          uint8_t pc[kInvChunk];
#pragma unroll
          for (int t = 0; t < kInvChunk; ++t) {
            const int i = min(i0 + t, m - 2);
            xn[t] = x[i + 1];  // read before this chunk writes x[i0 + t]
            lc[t] = ll[i];
            pc[t] = piv[i];
          }
#pragma unroll
          for (int t = 0; t < kInvChunk; ++t) {
            if (t < nstep) {
              const double nx = xn[t];
              if (pc[t]) {
                x[i0 + t] = nx;
                cur = cur - lc[t] * nx;
              } else {
                x[i0 + t] = cur;
                cur = nx - lc[t] * cur;
              }
            }
          }
        }
        double x1 = cur * r0[m - 1], x2 = 0.0;
        x[m - 1] = x1;
        for (int i1 = m - 2; i1 >= 0; i1 -= kInvChunk) {
          const int nstep = min(kInvChunk, i1 + 1);
          double xc[kInvChunk], a1[kInvChunk], a2[kInvChunk], rc[kInvChunk];
#pragma unroll
          for (int t = 0; t < kInvChunk; ++t) {
            const int i = max(i1 - t, 0);
            xc[t] = x[i];
            a1[t] = u1[i];
            a2[t] = u2[i];
            rc[t] = r0[i];
          }
#pragma unroll
          for (int t = 0; t < kInvChunk; ++t) {
            if (t < nstep) {
              const double xi = (xc[t] - a1[t] * x1 - a2[t] * x2) * rc[t];
              x[i1 - t] = xi;
              x2 = x1;
              x1 = xi;
            }
          }
        }
      }
      __syncthreads();
      for (int t = sb; t < s; ++t) {
        const double* zt = Z + static_cast<int64_t>(t) * n + s0;
        double p = 0.0;
        for (int j = tid; j < m; j += 256) p += zt[j] * x[j];
        const double dot = block_sum(p, red);
        for (int j = tid; j < m; j += 256) x[j] -= dot * zt[j];
      }
      double mx = 0.0;
      for (int j = tid; j < m; j += 256) mx = fmax(mx, fabs(x[j]));
      const double rmx = 1.0 / block_max(mx, red);
      double q = 0.0;
      for (int j = tid; j < m; j += 256) {
        const double y = x[j] * rmx;
        q += y * y;
      }
      const double rs = rmx / sqrt(block_sum(q, red));
      for (int j = tid; j < m; j += 256) x[j] *= rs;
      __syncthreads();
    }
    double* zs = Z + static_cast<int64_t>(s) * n;
    for (int r = tid; r < n; r += 256) zs[r] = (r >= s0 && r < s1) ? x[r - s0] : 0.0;
    __syncthreads();
  }
}

// The same inverse iteration for n <= kPipeMaxN with the next slot's LU
// overlapped: while wave 0 runs slot s's solves, Gram-Schmidt and
// normalisation (wave reductions only, no workgroup barrier inside a slot),
// the first lane of wave 1 factors T - x_{s+1} I into the other set of
// factor arrays; one barrier per slot.  Same steps and shifts as
// tri_inviter_kernel; its sums run over one wave instead of the workgroup.
// LDS: d, e, x (n each), two sets of u0^-1, u1, u2 and multipliers (4n each)
// and two pivot arrays (n bytes each).
constexpr int kPipeMaxN = 1800;
__global__ __launch_bounds__(256) void tri_inviter_pipe_kernel(const double* __restrict__ d,
                                                               const double* __restrict__ ez,
                                                               const int32_t* __restrict__ bs,
                                                               const int32_t* __restrict__ be,
                                                               const double* __restrict__ lam,
                                                               const int32_t* __restrict__ cstart,
                                                               const int32_t* __restrict__ ncl,
                                                               const double* __restrict__ scal, int n,
                                                               double* __restrict__ Z,
                                                               const int32_t* __restrict__ flag) {
  extern __shared__ double sm[];
  if (*flag) return;
  const int c = blockIdx.x, nc = *ncl;
  if (c >= nc) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int sb = cstart[c], se = (c + 1 < nc) ? cstart[c + 1] : n;
  const int s0 = bs[sb], s1 = be[sb], m = s1 - s0;
  double* dd = sm;
  double* ee = sm + n;
  double* x = sm + 2 * n;
  double* fac = sm + 3 * n;  // set b: r0, u1, u2, ll at fac + (4 b + k) n
  uint8_t* pvs = reinterpret_cast<uint8_t*>(sm + 11 * n);  // set b at pvs + b n
  for (int j = tid; j < m; j += 256) {
    dd[j] = d[s0 + j];
    ee[j] = (j + 1 < m) ? ez[s0 + j] : 0.0;
  }
  __syncthreads();
  const double tn = scal[0];
  const double pertol = 10.0 * kEps * tn;
  const double pmin = fmax(1e-3 * kEps * tn, 1e-150);
  // LU with partial pivoting of T - xs I into factor set b (one thread)
  auto lu = [&](double xs, int b) {
    double* r0 = fac + (4 * b + 0) * static_cast<int64_t>(n);
    double* u1 = fac + (4 * b + 1) * static_cast<int64_t>(n);
    double* u2 = fac + (4 * b + 2) * static_cast<int64_t>(n);
    double* ll = fac + (4 * b + 3) * static_cast<int64_t>(n);
    uint8_t* piv = pvs + b * static_cast<int64_t>(n);
    double bb = dd[0] - xs, cc = ee[0];
    for (int i0 = 0; i0 + 1 < m; i0 += kInvChunk) {
      const int nstep = min(kInvChunk, m - 1 - i0);
      double ea[kInvChunk + 1], db[kInvChunk];
#pragma unroll
      for (int t = 0; t <= kInvChunk; ++t) ea[t] = ee[min(i0 + t, m - 1)];
#pragma unroll
      for (int t = 0; t < kInvChunk; ++t) db[t] = dd[min(i0 + 1 + t, m - 1)];
#pragma unroll
      for (int t = 0; t < kInvChunk; ++t) {
        if (t < nstep) {
          const int i = i0 + t;
          const double a = ea[t], bv = db[t] - xs, cn = ea[t + 1];
          const double ra = rcp_nr(a);
          if (fabs(a) > fabs(bb)) {
            piv[i] = 1;
            r0[i] = ra;
            u1[i] = bv;
            u2[i] = cn;
            const double mult = bb * ra;
            ll[i] = mult;
            bb = cc - mult * bv;
            cc = -mult * cn;
          } else {
            piv[i] = 0;
            const double p = (fabs(bb) < pmin) ? copysign(pmin, bb) : bb;
            const double rp = rcp_nr(p);
            r0[i] = rp;
            u1[i] = cc;
            u2[i] = 0.0;
            const double mult = a * rp;
            ll[i] = mult;
            bb = bv - mult * cc;
            cc = cn;
          }
        }
      }
    }
    r0[m - 1] = rcp_nr((fabs(bb) < pmin) ? copysign(pmin, bb) : bb);
  };
  double xcur = lam[sb];
  if (tid == 0) lu(xcur, 0);
  __syncthreads();
  const int iters = (se - sb == 1) ? kInvIters - 1 : kInvIters;  // clusters get one more solve
  for (int s = sb; s < se; ++s) {
    const int b = (s - sb) & 1;
    double xnext = 0.0;
    if (s + 1 < se) {
      xnext = lam[s + 1];
      if (xnext - xcur < pertol) xnext = xcur + pertol;
    }
    if (wv == 0) {
      const double* r0 = fac + (4 * b + 0) * static_cast<int64_t>(n);
      const double* u1 = fac + (4 * b + 1) * static_cast<int64_t>(n);
      const double* u2 = fac + (4 * b + 2) * static_cast<int64_t>(n);
      const double* ll = fac + (4 * b + 3) * static_cast<int64_t>(n);
      const uint8_t* piv = pvs + b * static_cast<int64_t>(n);
      double part = 0.0;
      for (int j = lane; j < m; j += 64) {
        const double v = start_value(static_cast<uint32_t>(s), static_cast<uint32_t>(j));
        x[j] = v;
        part += v * v;
      }
      const double scale0 = 1.0 / sqrt(wave_sum(part));
      for (int j = lane; j < m; j += 64) x[j] *= scale0;
      asm volatile("" ::: "memory");
      for (int it = 0; it < iters; ++it) {
        if (lane == 0) {
          double cur = x[0];
          for (int i0 = 0; i0 + 1 < m; i0 += kInvChunk) {
            const int nstep = min(kInvChunk, m - 1 - i0);
            double xn[kInvChunk], lc[kInvChunk];
            uint8_t pc[kInvChunk];
#pragma unroll
            for (int t = 0; t < kInvChunk; ++t) {
              const int i = min(i0 + t, m - 2);
              xn[t] = x[i + 1];
              lc[t] = ll[i];
              pc[t] = piv[i];
            }
#pragma unroll
            for (int t = 0; t < kInvChunk; ++t) {
              if (t < nstep) {
                const double nx = xn[t];
                if (pc[t]) {
                  x[i0 + t] = nx;
                  cur = cur - lc[t] * nx;
                } else {
                  x[i0 + t] = cur;
                  cur = nx - lc[t] * cur;
                }
              }
            }
          }
          double x1 = cur * r0[m - 1], x2 = 0.0;
          x[m - 1] = x1;
          for (int i1 = m - 2; i1 >= 0; i1 -= kInvChunk) {
            const int nstep = min(kInvChunk, i1 + 1);
            double xc[kInvChunk], a1[kInvChunk], a2[kInvChunk], rc[kInvChunk];
#pragma unroll
            for (int t = 0; t < kInvChunk; ++t) {
              const int i = max(i1 - t, 0);
              xc[t] = x[i];
              a1[t] = u1[i];
              a2[t] = u2[i];
              rc[t] = r0[i];
            }
#pragma unroll
            for (int t = 0; t < kInvChunk; ++t) {
              if (t < nstep) {
                const double xi = (xc[t] - a1[t] * x1 - a2[t] * x2) * rc[t];
                x[i1 - t] = xi;
                x2 = x1;
                x1 = xi;
              }
            }
          }
        }
        asm volatile("" ::: "memory");  // the wave reads x after lane 0's writes (LDS is in order per wave)
        for (int t = sb; t < s; ++t) {
          const double* zt = Z + static_cast<int64_t>(t) * n + s0;
          double p = 0.0;
          for (int j = lane; j < m; j += 64) p += zt[j] * x[j];
          const double dot = wave_sum(p);
          for (int j = lane; j < m; j += 64) x[j] -= dot * zt[j];
          asm volatile("" ::: "memory");
        }
        double mx = 0.0;
        for (int j = lane; j < m; j += 64) mx = fmax(mx, fabs(x[j]));
        const double rmx = 1.0 / wave_max(mx);
        double q = 0.0;
        for (int j = lane; j < m; j += 64) {
          const double y = x[j] * rmx;
          q += y * y;
        }
        const double rs = rmx / sqrt(wave_sum(q));
        for (int j = lane; j < m; j += 64) x[j] *= rs;
        asm volatile("" ::: "memory");
      }
      double* zs = Z + static_cast<int64_t>(s) * n;
      for (int r = lane; r < n; r += 64) zs[r] = (r >= s0 && r < s1) ? x[r - s0] : 0.0;
    } else if (wv == 1 && lane == 0 && s + 1 < se) {
      lu(xnext, b ^ 1);
    }
    __syncthreads();
    xcur = xnext;
  }
}

// Ascending order of all eigenvalues (ties by slot): lam[rank] = raw[s],
// perm[rank] = s.
__global__ __launch_bounds__(256) void tri_rank_kernel(const double* __restrict__ raw, int n,
                                                       double* __restrict__ lam, int32_t* __restrict__ perm,
                                                       const int32_t* __restrict__ flag) {
  extern __shared__ double L[];
  if (*flag) return;
  for (int t = threadIdx.x; t < n; t += 256) L[t] = raw[t];
  __syncthreads();
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= n) return;
  const double ls = L[s];
  int rank = 0;
  for (int t = 0; t < n; ++t) rank += (L[t] < ls || (L[t] == ls && t < s)) ? 1 : 0;
  lam[rank] = ls;
  perm[rank] = s;
}

// Compact WY form of the back-transform for moderate n: blocks of kWyNB
// consecutive reflectors, H_kb ... H_{kb+nb-1} = I - V T V^T with V the
// block's reflectors (column j holds v_{kb+j}) and T upper triangular
// (T_jj = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] V[:, 0:j]^T v_j).
constexpr int kWyNB = 16;
constexpr int kWyMaxN = 900;  // LDS: 4 columns + the block's 16 reflectors + T, (20 n + 256) doubles
// T of block b (reflectors 16 b ...) into Tbuf + 256 b, column-major 16 x 16
// (zero beyond the block's nb reflectors).  The block's reflectors are
// staged in LDS (kWyNB n doubles); each wave forms a share of the Gram
// entries with lanes over the rows and a wave sum.
__global__ __launch_bounds__(256) void bt_tfactor_kernel(const double* __restrict__ Vh,
                                                         const double* __restrict__ tau, int n,
                                                         double* __restrict__ Tbuf,
                                                         const int32_t* __restrict__ flag) {
  extern __shared__ double vsh[];  // kWyNB * n
  __shared__ double G[kWyNB * kWyNB];
  __shared__ double Ts[kWyNB * kWyNB];
  if (*flag) return;
  const int b = blockIdx.x, kb = b * kWyNB, nb = min(kWyNB, n - 1 - kb), tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  for (int q = 0; q < kWyNB; ++q) {
    const double* v = Vh + static_cast<int64_t>(min(kb + q, n - 1)) * n;
    for (int r = tid; r < n; r += 256) vsh[q * n + r] = (q < nb && r > kb + q) ? v[r] : 0.0;
  }
  G[tid] = 0.0;
  Ts[tid] = 0.0;
  __syncthreads();
  // G[i + 16 j] = v_{kb+i} . v_{kb+j} for i < j (v_{kb+j} is zero in rows <= kb + j):
  // pair p = (i, j) goes to wave p mod 4
  for (int pr = wv; pr < kWyNB * kWyNB; pr += 4) {
    const int i = pr % kWyNB, j = pr / kWyNB;
    if (!(i < j && j < nb)) continue;  // uniform across the wave
    double g = 0.0;
    for (int r = kb + j + 1 + lane; r < n; r += 64) g += vsh[i * n + r] * vsh[j * n + r];
    g = wave_sum(g);
    if (lane == 0) G[pr] = g;
  }
  __syncthreads();
  for (int i = 0; i < nb; ++i) {
    const double ti = tau[kb + i];
    if (tid < i) {
      double acc = 0.0;
      for (int c = tid; c < i; ++c) acc += Ts[tid + c * kWyNB] * G[c + i * kWyNB];
      Ts[tid + i * kWyNB] = -ti * acc;
    }
    if (tid == i) Ts[i + i * kWyNB] = ti;
    __syncthreads();
  }
  Tbuf[static_cast<int64_t>(b) * kWyNB * kWyNB + tid] = Ts[tid];
}

// out[:, c] = H_0 ... H_{n-2} Z[:, perm[c]], blocks applied from the last to
// the first as z -= V (T (V^T z)).  Four columns per workgroup (one per
// wave) in LDS; each block's reflectors and T are staged in LDS; a wave forms
// its 16 dot products in one pass over the rows, then 16 wave sums, T, and
// one update pass.
__global__ __launch_bounds__(256) void bt_wy_kernel(const double* __restrict__ Z, const int32_t* __restrict__ perm,
                                                    const double* __restrict__ Vh,
                                                    const double* __restrict__ Tbuf, int n,
                                                    double* __restrict__ out, const int32_t* __restrict__ flag) {
  extern __shared__ double sm[];
  if (*flag) return;
  constexpr int NB = kWyNB;
  double* zs = sm;               // 4 n
  double* vs = sm + 4 * n;       // NB n: vs[q n + r] = v_{kb+q}[r]
  double* ts = vs + NB * n;      // NB * NB
  const int c0 = blockIdx.x * 4, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int cc = 0; cc < 4; ++cc) {
    const int c = c0 + cc;
    int pc = (c < n) ? perm[c] : 0;
    pc = (pc >= 0 && pc < n) ? pc : c;  // a rank is always in range; never index out of bounds
    const double* src = (c < n) ? Z + static_cast<int64_t>(pc) * n : nullptr;
    for (int j = tid; j < n; j += 256) zs[cc * n + j] = src ? src[j] : 0.0;
  }
  double* zw = zs + wv * n;
  const int nblocks = (n - 1 + NB - 1) / NB;
  // the next block's reflectors and T are loaded into registers while the
  // current block computes (rows tid + 256 p, n <= 256 PF)
  constexpr int PF = (kWyMaxN + 255) / 256;
  double pre[NB][PF], tpre;
  auto fetch = [&](int b) {
    const int kb = b * NB, nb = min(NB, n - 1 - kb);
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const double* v = Vh + static_cast<int64_t>(min(kb + q, n - 1)) * n;
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        const int r = tid + 256 * p;
        pre[q][p] = (q < nb && r < n && r > kb + q) ? v[r] : 0.0;
      }
    }
    tpre = Tbuf[static_cast<int64_t>(b) * NB * NB + tid];
  };
  fetch(nblocks - 1);
  for (int b = nblocks - 1; b >= 0; --b) {
    const int kb = b * NB;
    __syncthreads();  // the previous block's readers of vs and ts are done (and zs is loaded)
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        const int r = tid + 256 * p;
        if (r < n) vs[q * n + r] = pre[q][p];
      }
    ts[tid] = tpre;
    __syncthreads();
    if (b > 0) fetch(b - 1);
    const int r0 = kb + 1;  // every reflector of the block is zero above this row
    double acc[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) acc[q] = 0.0;
    for (int r = r0 + lane; r < n; r += 64) {
      const double zr = zw[r];
#pragma unroll
      for (int q = 0; q < NB; ++q) acc[q] += vs[q * n + r] * zr;
    }
    double w[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) w[q] = wave_sum(acc[q]);
    double u[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      double t = 0.0;
#pragma unroll
      for (int j = i; j < NB; ++j) t += ts[i + j * NB] * w[j];
      u[i] = t;
    }
    for (int r = r0 + lane; r < n; r += 64) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < NB; ++q) t += vs[q * n + r] * u[q];
      zw[r] -= t;
    }
  }
  __syncthreads();
  for (int cc = 0; cc < 4; ++cc) {
    const int c = c0 + cc;
    if (c >= n) break;
    for (int j = tid; j < n; j += 256) out[j + static_cast<int64_t>(c) * n] = zs[cc * n + j];
  }
}

// out[:, c] = H_0 H_1 ... H_{n-2} Z[:, perm[c]]: four columns per workgroup,
// one per wavefront, held in LDS.  Each wavefront steps through the
// reflectors on its own (dot product by shuffles, no workgroup barrier);
// reflectors are staged into LDS ch at a time, so the only barriers are at
// chunk boundaries.
constexpr int kBtCols = 4;
__global__ __launch_bounds__(256) void bt_kernel(const double* __restrict__ Z, const int32_t* __restrict__ perm,
                                                 const double* __restrict__ Vh, const double* __restrict__ tau,
                                                 int n, int ch, double* __restrict__ out,
                                                 const int32_t* __restrict__ flag) {
  extern __shared__ double sm[];
  if (*flag) return;
  double* zs = sm;                        // kBtCols * n
  double* vch = sm + kBtCols * n;         // ch * n
  double* tch = vch + static_cast<int64_t>(ch) * n;  // ch
  const int c0 = blockIdx.x * kBtCols, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int cc = 0; cc < kBtCols; ++cc) {
    const int c = c0 + cc;
    int pc = (c < n) ? perm[c] : 0;
    pc = (pc >= 0 && pc < n) ? pc : c;  // a rank is always in range; never index out of bounds
    const double* src = (c < n) ? Z + static_cast<int64_t>(pc) * n : nullptr;
    for (int j = tid; j < n; j += 256) zs[cc * n + j] = src ? src[j] : 0.0;
  }
  double* zw = zs + wv * n;
  for (int kc = n - 2; kc >= 0; kc -= ch) {
    const int qn = min(ch, kc + 1);
    __syncthreads();
    for (int e = tid; e < qn * n; e += 256) {
      const int q = e / n, j = e % n, k = kc - q;
      vch[e] = (j > k) ? Vh[j + static_cast<int64_t>(k) * n] : 0.0;
    }
    if (tid < qn) tch[tid] = tau[kc - tid];
    __syncthreads();
    for (int q = 0; q < qn; ++q) {
      const double t = tch[q];
      if (t == 0.0) continue;
      const int k = kc - q;
      const double* v = vch + q * n;
      double acc = 0.0;
      for (int j = k + 1 + lane; j < n; j += 64) acc += v[j] * zw[j];
      const double d = t * wave_sum(acc);
      for (int j = k + 1 + lane; j < n; j += 64) zw[j] -= d * v[j];
      asm volatile("" ::: "memory");  // keep the next step's reads after these writes (LDS is in order per wave)
    }
  }
  __syncthreads();
  for (int cc = 0; cc < kBtCols; ++cc) {
    const int c = c0 + cc;
    if (c >= n) break;
    for (int j = tid; j < n; j += 256) out[j + static_cast<int64_t>(c) * n] = zs[cc * n + j];
  }
}

void set_smem(const void* fn, size_t bytes) { ensure_dyn_smem(fn, bytes); }

}  // namespace

size_t dense_bytes(int n, bool own_gemm_work) {
  const size_t nn = static_cast<size_t>(n) * n;
  size_t b = 7 * nn * 8 + static_cast<size_t>(n) * 8 * DenseWork::kVecs + (static_cast<size_t>(n) + 16) * 8 + 64 +
             static_cast<size_t>(n) * 4 * DenseWork::kIvecs + 64;
  if (own_gemm_work) b += gemm_tn_work_elems(n, n, n) * 8;
  return b;
}

void dense_alloc(DenseWork& w, int n, double* ext_work, size_t ext_elems) {
  dense_free(w);
  if (n < 1 || n > kDenseMaxN) fail(XLS_ERR_INVALID_ARG, "dense eigensolver supports 1 <= n <= 2800");
  w.n = n;
  const size_t nn = static_cast<size_t>(n) * n;
  auto al = [&](void** p, size_t bytes) {
    if (hipMalloc(p, std::max<size_t>(bytes, 256)) != hipSuccess)
      fail(XLS_ERR_OUT_OF_MEMORY, "dense workspace allocation failed");
  };
  double** mats[] = {&w.R, &w.Rinv, &w.C0, &w.C1, &w.T, &w.Vh, &w.Z};
  for (double** p : mats) al(reinterpret_cast<void**>(p), nn * 8);
  al(reinterpret_cast<void**>(&w.vec), static_cast<size_t>(n) * 8 * DenseWork::kVecs);
  al(reinterpret_cast<void**>(&w.scal), (static_cast<size_t>(n) + 16) * 8);
  al(reinterpret_cast<void**>(&w.flag), 64);
  al(reinterpret_cast<void**>(&w.ivec), static_cast<size_t>(n) * 4 * DenseWork::kIvecs + 64);
  if (ext_work) {
    if (ext_elems < nn) fail(XLS_ERR_INVALID_ARG, "shared dense GEMM workspace too small");
    w.gemm_work = ext_work;
    w.gemm_work_elems = ext_elems;
    w.own_gemm_work = false;
  } else {
    w.gemm_work_elems = gemm_tn_work_elems(n, n, n);
    al(reinterpret_cast<void**>(&w.gemm_work), w.gemm_work_elems * 8);
    w.own_gemm_work = true;
  }
}

void dense_free(DenseWork& w) {
  if (w.borrowed) {
    w = DenseWork{};
    return;
  }
  if (!w.own_gemm_work) w.gemm_work = nullptr;  // borrowed: the owner frees it
  w.own_gemm_work = true;
  double** ds[] = {&w.R, &w.Rinv, &w.C0, &w.C1, &w.T, &w.Vh, &w.Z, &w.vec, &w.scal, &w.gemm_work};
  for (double** p : ds)
    if (*p) {
      (void)hipFree(*p);
      *p = nullptr;
    }
  if (w.flag) (void)hipFree(w.flag);
  if (w.ivec) (void)hipFree(w.ivec);
  w.flag = nullptr;
  w.ivec = nullptr;
  w.n = 0;
}

int dense_geneig(DenseWork& w, const double* Hs, const double* M, double* Y, hipStream_t st, bool check_spd) {
  const int n = w.n;
  const int64_t nn = static_cast<int64_t>(n) * n;
  double* vec = w.vec;
  double* lam = vec;  // sorted eigenvalues (w.lam)
  double* raw = vec + n;
  double* d = vec + 2 * static_cast<int64_t>(n);
  double* e = vec + 3 * static_cast<int64_t>(n);
  double* ez = vec + 4 * static_cast<int64_t>(n);
  double* e2 = vec + 5 * static_cast<int64_t>(n);
  double* tau = vec + 6 * static_cast<int64_t>(n);
  double* vbuf = vec + 7 * static_cast<int64_t>(n);   // 2n
  double* pbuf = vec + 9 * static_cast<int64_t>(n);   // 2n
  int32_t* perm = w.ivec;
  int32_t* bs = w.ivec + n;
  int32_t* be = w.ivec + 2 * n;
  int32_t* cstart = w.ivec + 3 * n;
  int32_t* ncl = w.ivec + 4 * n;
  double* diag0 = w.scal + 16;
  // --- Cholesky M = R^T R (factor a copy in C0) ---
  XLS_HIP(hipMemcpyAsync(w.C0, M, nn * 8, hipMemcpyDeviceToDevice, st));
  launch_fill_i32(w.flag, 0, 16, st);
  launch_fill_i32(reinterpret_cast<int32_t*>(w.R), 0, 2 * nn, st);
  hipLaunchKernelGGL(copy_diag_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, w.C0, n, diag0);
  for (int j0 = 0; j0 < n; j0 += kPanel) {
    const int nb = std::min(kPanel, n - j0), rest = n - j0 - nb;
    hipLaunchKernelGGL(chol_panel_kernel, dim3(1 + nblk(rest, 256)), dim3(256), 0, st, w.C0, n, j0, nb, diag0,
                       w.flag, w.R);
    if (rest > 0) {
      const unsigned T = nblk(rest, 64);
      hipLaunchKernelGGL(chol_update_kernel, dim3(T * (T + 1) / 2), dim3(256), 0, st, w.C0, w.R, n, j0, nb,
                         w.flag);
    }
  }
  XLS_LAUNCH_CHECK("cholesky");
  if (check_spd) {
    int32_t hflag = 0;
    XLS_HIP(hipMemcpyAsync(&hflag, w.flag, 4, hipMemcpyDeviceToHost, st));
    XLS_HIP(hipStreamSynchronize(st));
    if (hflag) return XLS_ERR_NOT_SPD;
  }
  // --- Rinv ---
  const size_t trinv_smem = static_cast<size_t>(n) * sizeof(double);
  set_smem(reinterpret_cast<const void*>(trinv_kernel), trinv_smem);
  hipLaunchKernelGGL(trinv_kernel, dim3(n), dim3(256), trinv_smem, st, w.R, n, w.Rinv, w.flag);
  XLS_LAUNCH_CHECK("trinv_kernel");
  // --- C = Rinv^T Hs Rinv, symmetrised ---
  gemm_tn<double>(XLS_PREC_FP64, w.Rinv, n, Hs, n, n, n, n, w.T, n, 0, 0, w.gemm_work,
                  w.gemm_work_elems, st);
  gemm_nn<double>(XLS_PREC_FP64, w.T, n, w.Rinv, n, n, n, n, w.C1, n, nullptr, st);
  hipLaunchKernelGGL(symmetrize_kernel, dim3(nblk(nn, 256)), dim3(256), 0, st, w.C1, n, w.C0);
  // --- tridiagonalisation ---
  const size_t trd_smem = 3 * static_cast<size_t>(n) * sizeof(double);
  set_smem(reinterpret_cast<const void*>(trd_step_kernel), trd_smem);
  const int k0 = std::max(0, n - kTrdTail);
  for (int k = 0; k < k0; ++k) {
    const dim3 grid(std::max(1u, nblk(n - k - 1, 4)));
    if (n - k <= 64 * kTrdPre)
      hipLaunchKernelGGL(trd_step_wave_kernel, grid, dim3(256), 0, st, w.C0, n, k, w.Vh, tau, d, e, vbuf, pbuf,
                         w.flag);
    else
      hipLaunchKernelGGL(trd_step_kernel, grid, dim3(256), trd_smem, st, w.C0, n, k, w.Vh, tau, d, e, vbuf, pbuf,
                         w.flag);
  }
  if (n > 1) {
    const int m = n - k0;
    const size_t tail_smem = (static_cast<size_t>(m) * (m + 2) + 2 * static_cast<size_t>(m)) * sizeof(double);
    set_smem(reinterpret_cast<const void*>(trd_tail_kernel), tail_smem);
    hipLaunchKernelGGL(trd_tail_kernel, dim3(1), dim3(kTailThreads), tail_smem, st, w.C0, n, k0, w.Vh, tau, d, e, vbuf, pbuf,
                       w.flag);
  }
  XLS_LAUNCH_CHECK("trd_step_kernel");
  // --- tridiagonal eigenproblem ---
  hipLaunchKernelGGL(tri_prepare_kernel, dim3(1), dim3(256), 0, st, w.C0, n, d, e, ez, e2, bs, be, w.scal,
                     w.flag);
  hipLaunchKernelGGL(tri_multisect_kernel, dim3(n), dim3(64), 2 * static_cast<size_t>(n) * sizeof(double), st, d,
                     ez, e2, bs, be, w.scal, n, raw, w.flag);
  hipLaunchKernelGGL(tri_cluster_kernel, dim3(1), dim3(256), 0, st, raw, bs, w.scal, n, cstart, ncl, w.flag);
  if (n <= kPipeMaxN) {
    const size_t pipe_smem =
        11 * static_cast<size_t>(n) * sizeof(double) + ((2 * static_cast<size_t>(n) + 7) & ~size_t{7});
    set_smem(reinterpret_cast<const void*>(tri_inviter_pipe_kernel), pipe_smem);
    hipLaunchKernelGGL(tri_inviter_pipe_kernel, dim3(n), dim3(256), pipe_smem, st, d, ez, bs, be, raw, cstart, ncl,
                       w.scal, n, w.Z, w.flag);
  } else {
    const size_t inv_smem = 7 * static_cast<size_t>(n) * sizeof(double) + ((static_cast<size_t>(n) + 7) & ~size_t{7});
    set_smem(reinterpret_cast<const void*>(tri_inviter_kernel), inv_smem);
    hipLaunchKernelGGL(tri_inviter_kernel, dim3(n), dim3(256), inv_smem, st, d, ez, bs, be, raw, cstart, ncl,
                       w.scal, n, w.Z, w.flag);
  }
  hipLaunchKernelGGL(tri_rank_kernel, dim3(nblk(n, 256)), dim3(256), static_cast<size_t>(n) * sizeof(double), st,
                     raw, n, lam, perm, w.flag);
  XLS_LAUNCH_CHECK("tridiagonal eigensolver");
  // --- back-transformation, Y = Rinv Q Z ---
  if (n >= 2 * kWyNB && n <= kWyMaxN) {
    // T of every block into C1 (free after C was formed): 256 (n / 16 + 1) <= n^2 doubles here
    const int nblocks = (n - 1 + kWyNB - 1) / kWyNB;
    const size_t tf_sm = static_cast<size_t>(kWyNB) * n * sizeof(double);
    set_smem(reinterpret_cast<const void*>(bt_tfactor_kernel), tf_sm);
    hipLaunchKernelGGL(bt_tfactor_kernel, dim3(nblocks), dim3(256), tf_sm, st, w.Vh, tau, n, w.C1, w.flag);
    const size_t sm = (static_cast<size_t>(4 + kWyNB) * n + kWyNB * kWyNB) * sizeof(double);
    set_smem(reinterpret_cast<const void*>(bt_wy_kernel), sm);
    hipLaunchKernelGGL(bt_wy_kernel, dim3(nblk(n, 4)), dim3(256), sm, st, w.Z, perm, w.Vh, w.C1, n, w.T, w.flag);
  } else {
    const size_t zbytes = kBtCols * static_cast<size_t>(n) * sizeof(double);
    const size_t budget = 150 * 1024;
    const int ch = static_cast<int>(std::max<size_t>(1, std::min<size_t>(32, (budget - zbytes) / ((n + 1) * sizeof(double)))));
    const size_t sm = zbytes + (static_cast<size_t>(ch) * n + ch) * sizeof(double);
    set_smem(reinterpret_cast<const void*>(bt_kernel), sm);
    hipLaunchKernelGGL(bt_kernel, dim3(nblk(n, kBtCols)), dim3(256), sm, st, w.Z, perm, w.Vh, tau, n, ch, w.T,
                       w.flag);
  }
  gemm_nn<double>(XLS_PREC_FP64, w.Rinv, n, w.T, n, n, n, n, Y, n, nullptr, st);
  XLS_LAUNCH_CHECK("dense back-transform");
  return XLS_OK;
}

}  // namespace xls

// ---------------------------------------------------------------------------
// Allocation-free dense solve: the workspace is carved from a file-scope
// device array instead of hipMalloc.  Host code never passes the array's
// name to a kernel (that is a host-side stand-in); it takes the device
// address from hipGetSymbolAddress once per device and uses that.
// ---------------------------------------------------------------------------
namespace xls {
namespace {

constexpr int kNoAllocMaxN = 512;
constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
// bytes the carve below takes for n: seven n x n matrices, the vectors, the
// pivot scalars, the flag, the integer vectors and the split-K workspace
// (the same size dense_alloc gives it, so the split counts are the same)
size_t noalloc_bytes(int n) {
  const size_t nn = static_cast<size_t>(n) * n;
  return 7 * align256(nn * 8) + align256(static_cast<size_t>(n) * 8 * DenseWork::kVecs) +
         align256((static_cast<size_t>(n) + 16) * 8) + align256(64) +
         align256(static_cast<size_t>(n) * 4 * DenseWork::kIvecs + 64) + align256(gemm_tn_work_elems(n, n, n) * 8);
}
// 7 * 512^2 doubles (14 MiB) + a 4-split workspace (8 MiB) + vectors
constexpr size_t kScratchBytes = 24u << 20;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

// Device address of this device's copy of scratch (looked up once per device).
void* scratch_address() {
  int dev = 0;
  XLS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) fail(XLS_ERR_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      fail(XLS_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// DenseWork for n with every buffer inside [base, base + bytes).
void dense_carve(DenseWork& w, int n, unsigned char* base, size_t bytes) {
  if (noalloc_bytes(n) > bytes) fail(XLS_ERR_INVALID_ARG, "dense scratch too small");
  const size_t nn = static_cast<size_t>(n) * n;
  size_t off = 0;
  auto take = [&](size_t b) {
    unsigned char* p = base + off;
    off += align256(b);
    return p;
  };
  w = DenseWork{};
  w.n = n;
  w.borrowed = true;
  double** mats[] = {&w.R, &w.Rinv, &w.C0, &w.C1, &w.T, &w.Vh, &w.Z};
  for (double** p : mats) *p = reinterpret_cast<double*>(take(nn * 8));
  w.vec = reinterpret_cast<double*>(take(static_cast<size_t>(n) * 8 * DenseWork::kVecs));
  w.scal = reinterpret_cast<double*>(take((static_cast<size_t>(n) + 16) * 8));
  w.flag = reinterpret_cast<int32_t*>(take(64));
  w.ivec = reinterpret_cast<int32_t*>(take(static_cast<size_t>(n) * 4 * DenseWork::kIvecs + 64));
  w.gemm_work_elems = gemm_tn_work_elems(n, n, n);
  w.gemm_work = reinterpret_cast<double*>(take(w.gemm_work_elems * 8));
  w.own_gemm_work = false;
}

static_assert(kNoAllocMaxN * kNoAllocMaxN * 8 * 7 < kScratchBytes, "scratch holds the largest solve");

}  // namespace
}  // namespace xls

extern "C" int xls_dense_geneig_noalloc(int32_t n, const double* Hs, const double* M, double* lam, double* Y,
                                        void* stream) {
  using namespace xls;
  return guarded([&]() -> int {
    if (n < 1 || n > kNoAllocMaxN) fail(XLS_ERR_INVALID_ARG, "xls_dense_geneig_noalloc supports 1 <= n <= 512");
    if (!Hs || !M || !lam || !Y) fail(XLS_ERR_INVALID_ARG, "NULL argument");
    const size_t nn8 = static_cast<size_t>(n) * n * 8;
    check_device_range(Hs, nn8);
    check_device_range(M, nn8);
    check_device_range(Y, nn8);
    check_device_range(lam, static_cast<size_t>(n) * 8);
    hipStream_t st = static_cast<hipStream_t>(stream);
    DenseWork w;
    dense_carve(w, n, static_cast<unsigned char*>(scratch_address()), kScratchBytes);
    const int rc = dense_geneig(w, Hs, M, Y, st, true);
    if (rc != XLS_OK) {
      set_last_error("M is not positive definite");
      return rc;
    }
    XLS_HIP(hipMemcpyAsync(lam, w.lam(), static_cast<size_t>(n) * 8, hipMemcpyDeviceToDevice, st));
    XLS_HIP(hipStreamSynchronize(st));
    return XLS_OK;
  });
}
