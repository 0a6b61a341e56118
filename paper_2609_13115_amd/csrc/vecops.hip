// Vector-level kernels: deterministic column reductions, the subdomain core
// density and interior weights (Sec. V-A.4), Lanczos building blocks for the
// filter bounds, block conversions and fills.  Every reduction runs in a
// fixed order (no floating-point atomics), so results are bitwise repeatable.
#include <cmath>

#include <map>
#include <mutex>

#include "xls_internal.h"

namespace xls {
namespace {

inline unsigned nblk(int64_t n, int b) { return static_cast<unsigned>((n + b - 1) / b); }

// One wave per column: lane l adds entries l, l + 64, ... in order, then a
// fixed xor-shuffle tree (the order never depends on scheduling).
__global__ __launch_bounds__(256) void reduce_cols_kernel(const double* __restrict__ partial, int nper, int ncols,
                                                          double* __restrict__ out, int take_sqrt) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (c >= ncols) return;
  double s = 0.0;
  const double* p = partial + static_cast<int64_t>(c) * nper;
  for (int i = lane; i < nper; i += 64) s += p[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) out[c] = take_sqrt ? sqrt(s) : s;
}

// g_n = 1/(1 + exp((lam_n - mu)/sigma)), overflow-free form.
__global__ void fermi_kernel(const double* __restrict__ lam, int n, double mu, double sigma,
                             double* __restrict__ g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double t = (lam[i] - mu) / sigma;
  if (t > 0) {
    const double e = exp(-t);
    g[i] = e / (1.0 + e);
  } else {
    g[i] = 1.0 / (1.0 + exp(t));
  }
}

// rho[g] = (2/h^3) sum_n g_n psi_{g,n}^2 on core points, 0 elsewhere.
template <typename TS>
__global__ __launch_bounds__(256) void rho_kernel(const TS* __restrict__ psi, int64_t nd, int64_t ld,
                                                  int ns, const uint8_t* __restrict__ mask,
                                                  const double* __restrict__ gocc, double scale,
                                                  double* __restrict__ rho) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= nd) return;
  double s = 0.0;
  if (mask[g]) {
    for (int n = 0; n < ns; ++n) {
      const double v = static_cast<double>(psi[g + n * ld]);
      s += gocc[n] * v * v;
    }
    s *= scale;
  }
  rho[g] = s;
}

// Partial core sums of psi^2 per column: partial[col * nchunk + chunk].
template <typename TS>
__global__ __launch_bounds__(256) void core_weight_kernel(const TS* __restrict__ psi, int64_t nd,
                                                          int64_t ld, const uint8_t* __restrict__ mask,
                                                          int nchunk, double* __restrict__ partial) {
  __shared__ double red[4];
  const int col = blockIdx.y, chunk = blockIdx.x;
  const int64_t per = (nd + nchunk - 1) / nchunk;
  const int64_t g0 = chunk * per, g1 = min(nd, g0 + per);
  const TS* __restrict__ c = psi + col * ld;
  double s = 0.0;
  for (int64_t g = g0 + threadIdx.x; g < g1; g += 256) {
    if (mask[g]) {
      const double v = static_cast<double>(c[g]);
      s += v * v;
    }
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[static_cast<int64_t>(col) * nchunk + chunk] = (red[0] + red[1]) + (red[2] + red[3]);
}

template <typename TS>
__global__ __launch_bounds__(256) void dot_partial_kernel(const TS* __restrict__ x, const TS* __restrict__ y,
                                                          int64_t n, int nblocks, double* __restrict__ partial) {
  __shared__ double red[4];
  const int64_t per = (n + nblocks - 1) / nblocks;
  const int64_t i0 = blockIdx.x * per, i1 = min(n, i0 + per);
  double s = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256)
    s += static_cast<double>(x[i]) * static_cast<double>(y[i]);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// partial[i nblocks + b] = block b's share of sum_g V[i ldv + g] y[g]; grid
// (nblocks, m), the layout of dot_partial_kernel per row i
template <typename TS>
__global__ __launch_bounds__(256) void multi_dot_partial_kernel(const TS* __restrict__ V, int64_t ldv,
                                                                const TS* __restrict__ y, int64_t n, int nblocks,
                                                                double* __restrict__ partial) {
  __shared__ double red[4];
  const TS* __restrict__ x = V + static_cast<int64_t>(blockIdx.y) * ldv;
  const int64_t per = (n + nblocks - 1) / nblocks;
  const int64_t i0 = blockIdx.x * per, i1 = min(n, i0 + per);
  double s = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256)
    s += static_cast<double>(x[i]) * static_cast<double>(y[i]);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[static_cast<int64_t>(blockIdx.y) * nblocks + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// w <- w - alpha_j v - beta_{j-1} v_prev  (beta_prev may be null)
template <typename TS>
__global__ void lanczos_update_kernel(TS* __restrict__ w, const TS* __restrict__ v, const TS* __restrict__ vp,
                                      const double* __restrict__ alpha, const double* __restrict__ beta,
                                      int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double r = static_cast<double>(w[i]) - (*alpha) * static_cast<double>(v[i]);
  if (vp) r -= (*beta) * static_cast<double>(vp[i]);
  w[i] = static_cast<TS>(r);
}

// w <- w - V coef  (classical Gram-Schmidt against k columns of V)
template <typename TS>
__global__ void reorth_kernel(TS* __restrict__ w, const TS* __restrict__ V, int64_t ldv,
                              const double* __restrict__ coef, int k, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < k; ++j) s += static_cast<double>(V[i + j * ldv]) * coef[j];
  w[i] = static_cast<TS>(static_cast<double>(w[i]) - s);
}

template <typename TS>
__global__ void scale_to_kernel(TS* __restrict__ dst, const TS* __restrict__ src, const double* __restrict__ nrm,
                                int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  dst[i] = static_cast<TS>(static_cast<double>(src[i]) / (*nrm));
}

__global__ void fill_i32_kernel(int32_t* __restrict__ p, int32_t v, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Smallest and largest eigenvalue of the k x k symmetric tridiagonal T
// (diagonal alpha, off-diagonal beta[0..k-2]) by Sturm-count bisection; one
// thread per end, 200 halvings of the Gershgorin interval (exact to the last
// bits in FP64).
__global__ void tridiag_extremes_kernel(const double* __restrict__ alpha, const double* __restrict__ beta,
                                        int k, double* __restrict__ out) {
  const int which = threadIdx.x;  // 0: min, 1: max
  if (which > 1) return;
  double lo = alpha[0], hi = alpha[0];
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? fabs(beta[i - 1]) : 0.0) + (i < k - 1 ? fabs(beta[i]) : 0.0);
    lo = fmin(lo, alpha[i] - r);
    hi = fmax(hi, alpha[i] + r);
  }
  const double target = which == 0 ? 1.0 : static_cast<double>(k);  // count of eigenvalues <= x
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    // number of eigenvalues < mid
    int cnt = 0;
    double q = alpha[0] - mid;
    if (q < 0) ++cnt;
    for (int i = 1; i < k; ++i) {
      const double qq = (q != 0.0) ? q : 1e-300;
      q = alpha[i] - mid - beta[i - 1] * beta[i - 1] / qq;
      if (q < 0) ++cnt;
    }
    if (cnt >= target) hi = mid; else lo = mid;
  }
  out[which] = 0.5 * (lo + hi);
}

template <typename TS>
__global__ void convert_block_kernel(const double* __restrict__ src, int64_t lds_, TS* __restrict__ dst,
                                     int64_t ldd, int64_t rows, int cols) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t r = e % rows, c = e / rows;
  dst[r + c * ldd] = static_cast<TS>(src[r + c * lds_]);
}

template <typename TS>
__global__ void block_to_double_kernel(const TS* __restrict__ src, int64_t lds_, double* __restrict__ dst,
                                       int64_t ldd, int64_t rows, int cols) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t r = e % rows, c = e / rows;
  dst[r + c * ldd] = static_cast<double>(src[r + c * lds_]);
}

}  // namespace

void launch_reduce_cols(const double* partial, int nper, int ncols, double* out, int take_sqrt,
                        hipStream_t st) {
  hipLaunchKernelGGL(reduce_cols_kernel, dim3(nblk(ncols, 4)), dim3(256), 0, st, partial, nper, ncols, out,
                     take_sqrt);
  XLS_LAUNCH_CHECK("reduce_cols_kernel");
}

void launch_density(const double* lam, double mu, double sigma, const uint8_t* mask, double h,
                    const void* psi, int is_float, int64_t nd, int64_t ld, int ns, double* rho,
                    double* cpart, int nchunk, double* c, double* gocc, hipStream_t st) {
  hipLaunchKernelGGL(fermi_kernel, dim3(nblk(ns, 256)), dim3(256), 0, st, lam, ns, mu, sigma, gocc);
  const double scale = 2.0 / (h * h * h);
  if (is_float) {
    hipLaunchKernelGGL(rho_kernel<float>, dim3(nblk(nd, 256)), dim3(256), 0, st,
                       static_cast<const float*>(psi), nd, ld, ns, mask, gocc, scale, rho);
    hipLaunchKernelGGL(core_weight_kernel<float>, dim3(nchunk, ns), dim3(256), 0, st,
                       static_cast<const float*>(psi), nd, ld, mask, nchunk, cpart);
  } else {
    hipLaunchKernelGGL(rho_kernel<double>, dim3(nblk(nd, 256)), dim3(256), 0, st,
                       static_cast<const double*>(psi), nd, ld, ns, mask, gocc, scale, rho);
    hipLaunchKernelGGL(core_weight_kernel<double>, dim3(nchunk, ns), dim3(256), 0, st,
                       static_cast<const double*>(psi), nd, ld, mask, nchunk, cpart);
  }
  XLS_LAUNCH_CHECK("density kernels");
  launch_reduce_cols(cpart, nchunk, ns, c, 0, st);
}

template <typename TS>
void launch_dot(const TS* x, const TS* y, int64_t n, double* partial, int nblocks, double* out,
                int take_sqrt, hipStream_t st) {
  hipLaunchKernelGGL(dot_partial_kernel<TS>, dim3(nblocks), dim3(256), 0, st, x, y, n, nblocks, partial);
  launch_reduce_cols(partial, nblocks, 1, out, take_sqrt, st);
}

template <typename TS>
void launch_multi_dot(const TS* V, int64_t ldv, int m, const TS* y, int64_t n, double* partial, int nblocks,
                      double* out, hipStream_t st) {
  if (m <= 0) return;
  hipLaunchKernelGGL(multi_dot_partial_kernel<TS>, dim3(nblocks, m), dim3(256), 0, st, V, ldv, y, n, nblocks,
                     partial);
  XLS_LAUNCH_CHECK("multi_dot_partial_kernel");
  launch_reduce_cols(partial, nblocks, m, out, 0, st);
}

void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(fill_i32_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, p, v, n);
  XLS_LAUNCH_CHECK("fill_i32_kernel");
}

template <typename TS>
void launch_lanczos_update(TS* w, const TS* v, const TS* vprev, const double* alpha_j,
                           const double* beta_prev, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(lanczos_update_kernel<TS>, dim3(nblk(n, 256)), dim3(256), 0, st, w, v, vprev, alpha_j,
                     beta_prev, n);
  XLS_LAUNCH_CHECK("lanczos_update_kernel");
}

template <typename TS>
void launch_reorth(TS* w, const TS* V, int64_t ldv, const double* coef, int k, int64_t n,
                   hipStream_t st) {
  hipLaunchKernelGGL(reorth_kernel<TS>, dim3(nblk(n, 256)), dim3(256), 0, st, w, V, ldv, coef, k, n);
  XLS_LAUNCH_CHECK("reorth_kernel");
}

template <typename TS>
void launch_scale_to(TS* dst, const TS* src, const double* norm2, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(scale_to_kernel<TS>, dim3(nblk(n, 256)), dim3(256), 0, st, dst, src, norm2, n);
  XLS_LAUNCH_CHECK("scale_to_kernel");
}

void launch_tridiag_extremes(const double* alpha, const double* beta, int k, double* out,
                             hipStream_t st) {
  hipLaunchKernelGGL(tridiag_extremes_kernel, dim3(1), dim3(64), 0, st, alpha, beta, k, out);
  XLS_LAUNCH_CHECK("tridiag_extremes_kernel");
}

template <typename TS>
void launch_convert_block(const double* src, int64_t lds_, TS* dst, int64_t ldd, int64_t rows,
                          int cols, hipStream_t st) {
  const int64_t tot = rows * cols;
  if (tot <= 0) return;
  hipLaunchKernelGGL(convert_block_kernel<TS>, dim3(nblk(tot, 256)), dim3(256), 0, st, src, lds_, dst, ldd,
                     rows, cols);
  XLS_LAUNCH_CHECK("convert_block_kernel");
}

template <typename TS>
void launch_block_to_double(const TS* src, int64_t lds_, double* dst, int64_t ldd, int64_t rows,
                            int cols, hipStream_t st) {
  const int64_t tot = rows * cols;
  if (tot <= 0) return;
  hipLaunchKernelGGL(block_to_double_kernel<TS>, dim3(nblk(tot, 256)), dim3(256), 0, st, src, lds_, dst, ldd,
                     rows, cols);
  XLS_LAUNCH_CHECK("block_to_double_kernel");
}

#define XLS_INST_VEC(TS)                                                                            \
  template void launch_dot<TS>(const TS*, const TS*, int64_t, double*, int, double*, int, hipStream_t); \
  template void launch_multi_dot<TS>(const TS*, int64_t, int, const TS*, int64_t, double*, int, double*,  \
                                     hipStream_t);                                                       \
  template void launch_lanczos_update<TS>(TS*, const TS*, const TS*, const double*, const double*,  \
                                          int64_t, hipStream_t);                                    \
  template void launch_reorth<TS>(TS*, const TS*, int64_t, const double*, int, int64_t, hipStream_t); \
  template void launch_scale_to<TS>(TS*, const TS*, const double*, int64_t, hipStream_t);           \
  template void launch_convert_block<TS>(const double*, int64_t, TS*, int64_t, int64_t, int,        \
                                         hipStream_t);                                              \
  template void launch_block_to_double<TS>(const TS*, int64_t, double*, int64_t, int64_t, int,      \
                                           hipStream_t);
XLS_INST_VEC(double)
XLS_INST_VEC(float)

void ensure_dyn_smem(const void* fn, size_t bytes) {
  if (bytes <= 64 * 1024) return;
  static std::mutex mu;
  static std::map<const void*, size_t> done;
  std::lock_guard<std::mutex> lock(mu);
  size_t& cur = done[fn];
  if (bytes <= cur) return;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes)) != hipSuccess) {
    (void)hipGetLastError();
    fail(XLS_ERR_INVALID_ARG, "kernel needs more LDS than the device allows");
  }
  cur = bytes;
}

namespace {
// Coefficients of the scaled Chebyshev recurrence (the same scalar sequence
// as the host path): e = (lmax - lc)/2, c = (lmax + lc)/2, sigma_1 =
// e/(a0 - c), tau = 2/sigma_1, sigma_{k+1} = 1/(tau - sigma_k);
// step 0: (sigma_1/e, c, 0); step k: (2 sigma_{k+1}/e, c, sigma_k sigma_{k+1}).
__global__ void filter_coef_kernel(const double* __restrict__ lam, int ns, double a0, double lc, double lmax,
                                   int m, double* __restrict__ coef, int32_t* __restrict__ bad) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  if (lam) {
    a0 = lam[0];
    lc = lam[ns - 1];
  }
  const bool ok = (a0 < lc) && (lc < lmax);
  if (bad) *bad = ok ? 0 : 1;
  if (!ok) return;
  const double e = (lmax - lc) / 2.0;
  const double c = (lmax + lc) / 2.0;
  const double sigma1 = e / (a0 - c);
  const double tau = 2.0 / sigma1;
  coef[0] = sigma1 / e;
  coef[1] = c;
  coef[2] = 0.0;
  double sig = sigma1;
  for (int k = 1; k < m; ++k) {
    const double signew = 1.0 / (tau - sig);
    coef[3 * k] = 2.0 * signew / e;
    coef[3 * k + 1] = c;
    coef[3 * k + 2] = sig * signew;
    sig = signew;
  }
}
}  // namespace

void launch_filter_coef(const double* lam, int ns, double a0, double lc, double lmax, int m, double* coef,
                        int32_t* bad, hipStream_t st) {
  hipLaunchKernelGGL(filter_coef_kernel, dim3(1), dim3(64), 0, st, lam, ns, a0, lc, lmax, m, coef, bad);
  XLS_LAUNCH_CHECK("filter_coef_kernel");
}

}  // namespace xls
