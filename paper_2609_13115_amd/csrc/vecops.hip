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

// Rayleigh quotients from the residual sweep's partial sums: the same lane
// order and shuffle tree as reduce_cols_kernel for numerator and denominator.
__global__ __launch_bounds__(256) void reduce_rq_kernel(const double* __restrict__ num,
                                                        const double* __restrict__ den, int nper, int ncols,
                                                        double* __restrict__ out) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (c >= ncols) return;
  double a = 0.0, b = 0.0;
  const double* pn = num + static_cast<int64_t>(c) * nper;
  const double* pd = den + static_cast<int64_t>(c) * nper;
  for (int i = lane; i < nper; i += 64) {
    a += pn[i];
    b += pd[i];
  }
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  if (lane == 0) out[c] = a / b;  // a zero column gives NaN, as its residual would be meaningless
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

__device__ __forceinline__ double occupation(double lam, double mu, double sigma) {
  const double t = (lam - mu) / sigma;
  if (t > 0) {
    const double e = exp(-t);
    return e / (1.0 + e);
  }
  return 1.0 / (1.0 + exp(t));
}

// Fermi level of n states (lam_i, c_i): the root of
// N_e(mu) = 2 sum_i g(lam_i; mu, sigma) c_i - target, continuous and
// increasing in mu.  Newton steps with dN_e/dmu = (2/sigma) sum c g (1 - g),
// kept inside a bracket that every evaluation shrinks (a step that would leave
// it is replaced by the midpoint); the bracket starts at the extreme
// eigenvalues -/+ 40 sigma.  Stops when the step or the bracket falls to
// rounding level.  One workgroup; every sum is per thread over a fixed
// stride, then over the workgroup in a fixed order.
// out: mu, N_e(mu), E_band, E_entropy, evaluations, status (0 ok, 1 count
// out of reach).
constexpr int kFermiThreads = 1024;
__global__ __launch_bounds__(kFermiThreads) void fermi_level_kernel(const double* __restrict__ lam,
                                                                    const double* __restrict__ c, int64_t n,
                                                                    double sigma, double target, int max_eval,
                                                                    double* __restrict__ out) {
  constexpr int NW = kFermiThreads / 64;
  __shared__ double red[2][4][NW];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int phase = 0;
  // fixed-order workgroup sums of K values (one barrier; buffers alternate)
  auto bsum = [&](double (&v)[4], int K) {
    double(*rr)[NW] = red[phase & 1];
    ++phase;
    for (int q = 0; q < K; ++q) {
      double x = v[q];
      for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
      if (lane == 0) rr[q][wv] = x;
    }
    __syncthreads();
    for (int q = 0; q < K; ++q) {
      double a = 0.0, b = 0.0;
      for (int w = 0; w < NW; w += 2) {
        a += rr[q][w];
        b += rr[q][w + 1];
      }
      v[q] = a + b;
    }
  };
  double v[4] = {HUGE_VAL, HUGE_VAL, 0.0, 0.0};
  for (int64_t i = tid; i < n; i += kFermiThreads) {
    v[0] = fmin(v[0], lam[i]);
    v[1] = fmin(v[1], -lam[i]);
  }
  {  // min and -max over the workgroup (exact in any order)
    double(*rr)[NW] = red[phase & 1];
    ++phase;
    for (int q = 0; q < 2; ++q) {
      double x = v[q];
      for (int o = 32; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o, 64));
      if (lane == 0) rr[q][wv] = x;
    }
    __syncthreads();
    for (int q = 0; q < 2; ++q) {
      double a = HUGE_VAL;
      for (int w = 0; w < NW; ++w) a = fmin(a, rr[q][w]);
      v[q] = a;
    }
  }
  double lo = v[0] - 40.0 * sigma, hi = -v[1] + 40.0 * sigma;
  // N_e - target and its derivative at x
  auto count = [&](double x, double& F, double& dF) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = tid; i < n; i += kFermiThreads) {
      const double g = occupation(lam[i], x, sigma);
      a[0] += g * c[i];
      a[1] += c[i] * g * (1.0 - g);
    }
    bsum(a, 2);
    F = 2.0 * a[0] - target;
    dF = 2.0 * a[1] / sigma;
  };
  double F, dF;
  int evals = 0, status = 0;
  count(lo, F, dF);
  const bool lo_ok = F < 0.0;
  count(hi, F, dF);
  const bool hi_ok = F > 0.0;
  evals = 2;
  double mu = 0.5 * (lo + hi);
  if (!(lo_ok && hi_ok)) {
    status = 1;
  } else {
    while (evals < max_eval) {
      count(mu, F, dF);
      ++evals;
      if (F == 0.0) break;
      if (F < 0.0)
        lo = mu;
      else
        hi = mu;
      double nxt = (dF > 0.0) ? mu - F / dF : 0.5 * (lo + hi);
      if (!(nxt > lo && nxt < hi)) nxt = 0.5 * (lo + hi);
      const double tolx = 4.0 * 2.220446049250313e-16 * fmax(fabs(mu), sigma);
      if (fabs(nxt - mu) <= tolx || !(hi - lo > tolx)) {
        mu = nxt;
        break;
      }
      mu = nxt;
    }
  }
  // final count and energies at mu
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = tid; i < n; i += kFermiThreads) {
    const double g = occupation(lam[i], mu, sigma);
    a[0] += g * c[i];
    a[1] += g * c[i] * lam[i];
    double sg = 0.0;
    if (g > 0.0) sg += g * log(g);
    if (g < 1.0) sg += (1.0 - g) * log1p(-g);
    a[2] += c[i] * sg;
  }
  bsum(a, 3);
  if (tid == 0) {
    out[0] = mu;
    out[1] = 2.0 * a[0];
    out[2] = 2.0 * a[1];
    out[3] = -2.0 * sigma * a[2];
    out[4] = static_cast<double>(evals + 1);
    out[5] = static_cast<double>(status);
  }
}

// rho_global[gidx[g]] += rho[g] on core points (distinct global points within
// one call; calls for different subsystems are ordered on the stream).
__global__ void scatter_core_kernel(const double* __restrict__ rho, const uint8_t* __restrict__ mask,
                                    const int64_t* __restrict__ gidx, int64_t nd,
                                    double* __restrict__ rho_global) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= nd || !mask[g]) return;
  rho_global[gidx[g]] += rho[g];
}

// dos[b] = 2 sum of c_i over lam_i in [edges[b], edges[b+1]) (the last bin
// also takes its right edge); one thread per bin, states in order.
__global__ void dos_kernel(const double* __restrict__ lam, const double* __restrict__ c, int64_t n,
                           const double* __restrict__ edges, int nbins, double* __restrict__ dos) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  const double e0 = edges[b], e1 = edges[b + 1];
  const bool last = b == nbins - 1;
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double x = lam[i];
    if (x >= e0 && (x < e1 || (last && x == e1))) s += c[i];
  }
  dos[b] = 2.0 * s;
}

// PDOS weights P[n][j] = alpha[n][j]^2 / h^3 from the overlaps alpha = h^3
// sum phi_j psi_n, and the orbital-resolved PDOS D[j][b] = sum of P[n][j]
// over the states n with lambda_n in [edges[b], edges[b+1]) (the last bin
// also takes its right edge), zero for orbitals of atoms outside the core;
// one thread per (orbital, bin), states in order.
__global__ void pdos_weight_kernel(const double* __restrict__ alpha, int64_t n, double inv_h3,
                                   double* __restrict__ P) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < n) P[e] = alpha[e] * alpha[e] * inv_h3;
}
__global__ void pdos_hist_kernel(const double* __restrict__ P, const double* __restrict__ lam, int ns, int norb,
                                 const double* __restrict__ edges, int nbins, const uint8_t* __restrict__ in_core,
                                 double* __restrict__ D) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<int64_t>(norb) * nbins) return;
  const int j = static_cast<int>(t / nbins), b = static_cast<int>(t % nbins);
  double s = 0.0;
  if (in_core[j / 4]) {
    const double e0 = edges[b], e1 = edges[b + 1];
    const bool last = b == nbins - 1;
    for (int n = 0; n < ns; ++n) {
      const double x = lam[n];
      if (x >= e0 && (x < e1 || (last && x == e1))) s += P[static_cast<int64_t>(n) * norb + j];
    }
  }
  D[t] = s;
}

// Column c of a block (leading dimension ld) to and from IEEE binary16
// storage with leading dimension nd: rounding to nearest even on the way
// down, exact widening on the way up.  One thread per element, grid.y =
// column.
template <typename TS>
__global__ void block_to_half_kernel(const TS* __restrict__ src, int64_t ld, int64_t nd,
                                     uint16_t* __restrict__ dst) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= nd) return;
  const _Float16 h = static_cast<_Float16>(src[r + c * ld]);
  dst[r + c * nd] = __builtin_bit_cast(uint16_t, h);
}
template <typename TS>
__global__ void half_to_block_kernel(const uint16_t* __restrict__ src, int64_t ld, int64_t nd,
                                     TS* __restrict__ dst) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= nd) return;
  dst[r + c * ld] = static_cast<TS>(__builtin_bit_cast(_Float16, src[r + c * nd]));
}

// Counter-based start block: Philox4x32-10 (multipliers 0xD2511F53 and
// 0xCD9E8D57, Weyl key increments 0x9E3779B9 and 0xBB67AE85, 10 rounds) on
// counter (g, j, 0, 0), then Box-Muller on two 53-bit uniforms in (0, 1].
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

template <typename TS>
__global__ void philox_block_kernel(TS* __restrict__ blk, int64_t ld, int64_t nd, uint32_t k0, uint32_t k1) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const uint32_t j = blockIdx.y;
  if (g >= nd) return;
  uint32_t c[4] = {static_cast<uint32_t>(g), j, 0u, 0u};
  philox4x32_10(c, k0, k1);
  const uint64_t a = (static_cast<uint64_t>(c[0] >> 5) << 26) + (c[1] >> 6);
  const uint64_t b = (static_cast<uint64_t>(c[2] >> 5) << 26) + (c[3] >> 6);
  const double twom53 = 1.1102230246251565e-16;  // 2^-53
  const double u1 = 1.0 - static_cast<double>(a) * twom53;
  const double u2 = 1.0 - static_cast<double>(b) * twom53;
  const double two_pi = 6.283185307179586;  // 2 * fl(pi), exact
  blk[g + static_cast<int64_t>(j) * ld] = static_cast<TS>(sqrt(-2.0 * log(u1)) * cos(two_pi * u2));
}

template <typename TS>
__global__ void gather_rows_kernel(const TS* __restrict__ blk, int64_t ld, const int32_t* __restrict__ rows,
                                   int64_t nrows, TS* __restrict__ out, int64_t ldo) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= nrows) return;
  out[r + c * ldo] = blk[rows[r] + c * ld];
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

void launch_reduce_rq(const double* num, const double* den, int nper, int ncols, double* out, hipStream_t st) {
  hipLaunchKernelGGL(reduce_rq_kernel, dim3(nblk(ncols, 4)), dim3(256), 0, st, num, den, nper, ncols, out);
  XLS_LAUNCH_CHECK("reduce_rq_kernel");
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
void launch_block_half(const TS* blk, int64_t ld, int64_t nd, int ncols, uint16_t* half, int to_half,
                       hipStream_t st) {
  if (nd <= 0 || ncols <= 0) return;
  const dim3 grid(nblk(nd, 256), static_cast<unsigned>(ncols));
  if (to_half)
    hipLaunchKernelGGL(block_to_half_kernel<TS>, grid, dim3(256), 0, st, blk, ld, nd, half);
  else
    hipLaunchKernelGGL(half_to_block_kernel<TS>, grid, dim3(256), 0, st, half, ld, nd, const_cast<TS*>(blk));
  XLS_LAUNCH_CHECK("block_half");
}
template void launch_block_half<float>(const float*, int64_t, int64_t, int, uint16_t*, int, hipStream_t);
template void launch_block_half<double>(const double*, int64_t, int64_t, int, uint16_t*, int, hipStream_t);

void launch_pdos(const double* alpha, int ns, int norb, double h, const double* lam, const double* edges, int nbins,
                 const uint8_t* in_core, double* P, double* D, hipStream_t st) {
  const int64_t ne = static_cast<int64_t>(ns) * norb;
  if (ne > 0) {
    hipLaunchKernelGGL(pdos_weight_kernel, dim3(nblk(ne, 256)), dim3(256), 0, st, alpha, ne, 1.0 / (h * h * h), P);
    XLS_LAUNCH_CHECK("pdos_weight_kernel");
  }
  const int64_t nt = static_cast<int64_t>(norb) * nbins;
  if (nt > 0) {
    hipLaunchKernelGGL(pdos_hist_kernel, dim3(nblk(nt, 256)), dim3(256), 0, st, P, lam, ns, norb, edges, nbins,
                       in_core, D);
    XLS_LAUNCH_CHECK("pdos_hist_kernel");
  }
}

template <typename TS>
void launch_philox_block(TS* blk, int64_t ld, int64_t nd, int ncols, uint64_t seed, hipStream_t st) {
  if (nd <= 0 || ncols <= 0) return;
  hipLaunchKernelGGL(philox_block_kernel<TS>, dim3(nblk(nd, 256), static_cast<unsigned>(ncols)), dim3(256), 0, st,
                     blk, ld, nd, static_cast<uint32_t>(seed & 0xFFFFFFFFu), static_cast<uint32_t>(seed >> 32));
  XLS_LAUNCH_CHECK("philox_block_kernel");
}
template void launch_philox_block<float>(float*, int64_t, int64_t, int, uint64_t, hipStream_t);
template void launch_philox_block<double>(double*, int64_t, int64_t, int, uint64_t, hipStream_t);

template <typename TS>
void launch_gather_rows(const TS* blk, int64_t ld, const int32_t* rows, int64_t nrows, int ncols, TS* out,
                        int64_t ldo, hipStream_t st) {
  if (nrows <= 0 || ncols <= 0) return;
  hipLaunchKernelGGL(gather_rows_kernel<TS>, dim3(nblk(nrows, 256), static_cast<unsigned>(ncols)), dim3(256), 0,
                     st, blk, ld, rows, nrows, out, ldo);
  XLS_LAUNCH_CHECK("gather_rows_kernel");
}
template void launch_gather_rows<float>(const float*, int64_t, const int32_t*, int64_t, int, float*, int64_t,
                                        hipStream_t);
template void launch_gather_rows<double>(const double*, int64_t, const int32_t*, int64_t, int, double*, int64_t,
                                         hipStream_t);

void launch_core_weights(const uint8_t* mask, const void* psi, int is_float, int64_t nd, int64_t ld, int ns,
                         double* cpart, int nchunk, double* c, hipStream_t st) {
  if (is_float)
    hipLaunchKernelGGL(core_weight_kernel<float>, dim3(nchunk, ns), dim3(256), 0, st,
                       static_cast<const float*>(psi), nd, ld, mask, nchunk, cpart);
  else
    hipLaunchKernelGGL(core_weight_kernel<double>, dim3(nchunk, ns), dim3(256), 0, st,
                       static_cast<const double*>(psi), nd, ld, mask, nchunk, cpart);
  XLS_LAUNCH_CHECK("core_weight_kernel");
  launch_reduce_cols(cpart, nchunk, ns, c, 0, st);
}

void launch_fermi_level(const double* lam, const double* c, int64_t n, double sigma, double target, int max_eval,
                        double* out, hipStream_t st) {
  hipLaunchKernelGGL(fermi_level_kernel, dim3(1), dim3(kFermiThreads), 0, st, lam, c, n, sigma, target, max_eval,
                     out);
  XLS_LAUNCH_CHECK("fermi_level_kernel");
}

void launch_scatter_core(const double* rho, const uint8_t* mask, const int64_t* gidx, int64_t nd,
                         double* rho_global, hipStream_t st) {
  if (nd <= 0) return;
  hipLaunchKernelGGL(scatter_core_kernel, dim3(nblk(nd, 256)), dim3(256), 0, st, rho, mask, gidx, nd, rho_global);
  XLS_LAUNCH_CHECK("scatter_core_kernel");
}

void launch_dos(const double* lam, const double* c, int64_t n, const double* edges, int nbins, double* dos,
                hipStream_t st) {
  if (nbins <= 0) return;
  hipLaunchKernelGGL(dos_kernel, dim3(nblk(nbins, 64)), dim3(64), 0, st, lam, c, n, edges, nbins, dos);
  XLS_LAUNCH_CHECK("dos_kernel");
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
