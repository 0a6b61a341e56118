// Learned filter bounds: a small MLP trained and evaluated on the GPU.
//
// The paper defines the filter only through its centre c and half-width e
// (Sec. V-A.3) and leaves the source of the bounds open; the engine predicts a
// subdomain's (lambda_max, lambda_cut, degree) from cheap features of its
// local potential and geometry.  Layers y = x W + b with W (fan_in x fan_out,
// row-major), ReLU between layers, MSE loss, Adam.  Training runs in FP32 with
// fixed-order reductions (no atomics: bit-reproducible); inference rounds
// weights and activations to bfloat16 and accumulates in FP32.
//
// Parameter vector: for each layer l, W_l then b_l.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "xls_handle.h"

using namespace xls;

namespace {

constexpr int kMaxLayers = 4;
constexpr int kMaxWidth = 256;

struct Dims {
  int nl = 0;                    // layers
  int size[kMaxLayers + 1] = {};  // widths, size[0] = inputs
  int64_t woff[kMaxLayers] = {}, boff[kMaxLayers] = {};
  int64_t nparam = 0;
};

__device__ __forceinline__ uint16_t bf16_rne(float a) {
  uint32_t u = __float_as_uint(a);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf16_f(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }

__global__ void gather_rows_kernel(const float* __restrict__ X, int F, const int32_t* __restrict__ idx, int B,
                                   float* __restrict__ out) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(B) * F) return;
  const int b = static_cast<int>(e / F), f = static_cast<int>(e % F);
  out[e] = X[static_cast<int64_t>(idx[b]) * F + f];
}

// Z[b, o] = bias[o] + sum_i X[b, i] W[i, o] (i ascending); H = relu(Z) or Z.
__global__ void linear_fwd_kernel(const float* __restrict__ X, const float* __restrict__ W,
                                  const float* __restrict__ bias, int B, int fi, int fo, int relu,
                                  float* __restrict__ Z, float* __restrict__ H) {
  const int o = blockIdx.x * 64 + (threadIdx.x & 63);
  const int b = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (o >= fo || b >= B) return;
  const float* x = X + static_cast<int64_t>(b) * fi;
  float z = bias[o];
  for (int i = 0; i < fi; ++i) z = fmaf(x[i], W[static_cast<int64_t>(i) * fo + o], z);
  Z[static_cast<int64_t>(b) * fo + o] = z;
  H[static_cast<int64_t>(b) * fo + o] = relu ? fmaxf(z, 0.0f) : z;
}

// dY = 2 (Y - T) / (B fo); loss = mean (Y - T)^2 (one workgroup, fixed order).
__global__ __launch_bounds__(256) void mse_grad_kernel(const float* __restrict__ Y, const float* __restrict__ T,
                                                       int n, float* __restrict__ dY, float* __restrict__ loss) {
  __shared__ float red[256];
  float acc = 0.0f;
  const float scale = 2.0f / static_cast<float>(n);
  for (int e = threadIdx.x; e < n; e += 256) {
    const float d = Y[e] - T[e];
    dY[e] = scale * d;
    acc = fmaf(d, d, acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = red[0] / static_cast<float>(n);
}

// dW[i, o] = sum_b X[b, i] dZ[b, o]; row i == fi holds db[o] = sum_b dZ[b, o].
__global__ void linear_bwd_w_kernel(const float* __restrict__ X, const float* __restrict__ dZ, int B, int fi,
                                    int fo, float* __restrict__ dW, float* __restrict__ db) {
  const int o = blockIdx.x * 64 + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (o >= fo || i > fi) return;
  float acc = 0.0f;
  if (i < fi) {
    for (int b = 0; b < B; ++b) acc = fmaf(X[static_cast<int64_t>(b) * fi + i], dZ[static_cast<int64_t>(b) * fo + o], acc);
    dW[static_cast<int64_t>(i) * fo + o] = acc;
  } else {
    for (int b = 0; b < B; ++b) acc += dZ[static_cast<int64_t>(b) * fo + o];
    db[o] = acc;
  }
}

// dZprev[b, i] = [Zprev[b, i] > 0] * sum_o dZ[b, o] W[i, o].
__global__ void linear_bwd_x_kernel(const float* __restrict__ dZ, const float* __restrict__ W,
                                    const float* __restrict__ Zprev, int B, int fi, int fo,
                                    float* __restrict__ dZprev) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int b = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= fi || b >= B) return;
  const float* d = dZ + static_cast<int64_t>(b) * fo;
  const float* w = W + static_cast<int64_t>(i) * fo;
  float acc = 0.0f;
  for (int o = 0; o < fo; ++o) acc = fmaf(d[o], w[o], acc);
  dZprev[static_cast<int64_t>(b) * fi + i] = Zprev[static_cast<int64_t>(b) * fi + i] > 0.0f ? acc : 0.0f;
}

// Adam (Kingma and Ba 2015) with bias corrections bc1 = 1 - b1^t, bc2 = 1 - b2^t.
__global__ void adam_kernel(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ M,
                            float* __restrict__ V, int64_t n, float lr, float b1, float b2, float eps, float bc1,
                            float bc2) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = G[i];
  const float m = b1 * M[i] + (1.0f - b1) * g;
  const float v = b2 * V[i] + (1.0f - b2) * g * g;
  M[i] = m;
  V[i] = v;
  P[i] -= lr * (m / bc1) / (sqrtf(v / bc2) + eps);
}

__global__ void to_bf16_kernel(const float* __restrict__ a, uint16_t* __restrict__ o, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) o[i] = bf16_rne(a[i]);
}

struct InferArgs {
  int nl;
  int size[kMaxLayers + 1];
  int64_t woff[kMaxLayers], boff[kMaxLayers];
  float in_mean[64], in_scale[64];  // x' = (x - mean) * scale
  double out_mean[8], out_std[8];
};

// One workgroup per sample: bf16 weights and activations, FP32 accumulation
// in ascending input order, outputs de-standardised in FP64.
__global__ __launch_bounds__(256) void infer_bf16_kernel(const double* __restrict__ F, int B,
                                                         const uint16_t* __restrict__ Wb,
                                                         const float* __restrict__ P, InferArgs a,
                                                         double* __restrict__ out) {
  __shared__ float act[2][kMaxWidth];
  const int b = blockIdx.x, t = threadIdx.x;
  if (b >= B) return;
  const int f0 = a.size[0];
  if (t < f0) {
    const float x = (static_cast<float>(F[static_cast<int64_t>(b) * f0 + t]) - a.in_mean[t]) * a.in_scale[t];
    act[0][t] = bf16_f(bf16_rne(x));
  }
  __syncthreads();
  int cur = 0;
  for (int l = 0; l < a.nl; ++l) {
    const int fi = a.size[l], fo = a.size[l + 1];
    const uint16_t* W = Wb + a.woff[l];
    if (t < fo) {
      float z = P[a.boff[l] + t];
      for (int i = 0; i < fi; ++i) z = fmaf(act[cur][i], bf16_f(W[static_cast<int64_t>(i) * fo + t]), z);
      const bool last = l + 1 == a.nl;
      act[cur ^ 1][t] = last ? z : bf16_f(bf16_rne(fmaxf(z, 0.0f)));
    }
    __syncthreads();
    cur ^= 1;
  }
  const int fo = a.size[a.nl];
  if (t < fo) out[static_cast<int64_t>(b) * fo + t] = static_cast<double>(act[cur][t]) * a.out_std[t] + a.out_mean[t];
}

// ---- features of a subdomain's potential ----------------------------------
// Pass 1: min, max, sum (FP64, fixed order: per-thread strided partials then
// a fixed tree).  Pass 2: sum of squared deviations from the mean and the
// 32-bin histogram over [min, max] with the bin rule of numpy.histogram
// (index = floor((v - lo) * 32 / (hi - lo)), corrected against the edges
// lo + k (hi - lo)/32; the last bin is closed).
__global__ __launch_bounds__(1024) void vstats_kernel(const double* __restrict__ v, int64_t n,
                                                      double* __restrict__ out /*lo, hi, sum, ssd, 32 counts*/) {
  __shared__ double r0[1024], r1[1024], r2[1024];
  __shared__ uint32_t hist[32];
  const int t = threadIdx.x;
  double lo = HUGE_VAL, hi = -HUGE_VAL, s = 0.0;
  for (int64_t i = t; i < n; i += 1024) {
    const double x = v[i];
    lo = fmin(lo, x);
    hi = fmax(hi, x);
    s += x;
  }
  r0[t] = lo;
  r1[t] = hi;
  r2[t] = s;
  if (t < 32) hist[t] = 0;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) {
      r0[t] = fmin(r0[t], r0[t + w]);
      r1[t] = fmax(r1[t], r1[t + w]);
      r2[t] += r2[t + w];
    }
    __syncthreads();
  }
  lo = r0[0];
  hi = r1[0];
  const double mean = r2[0] / static_cast<double>(n);
  __syncthreads();
  const double delta = hi - lo;
  const double norm = 32.0 / delta;
  const double step = delta / 32.0;
  double ssd = 0.0;
  for (int64_t i = t; i < n; i += 1024) {
    const double x = v[i];
    const double d = x - mean;
    ssd = fma(d, d, ssd);
    if (delta > 0.0) {
      int k = static_cast<int>(__dmul_rn(__dsub_rn(x, lo), norm));
      if (k >= 32) k = 31;
      if (x < __dadd_rn(__dmul_rn(static_cast<double>(k), step), lo)) --k;
      const double upper = (k + 1 == 32) ? hi : __dadd_rn(__dmul_rn(static_cast<double>(k + 1), step), lo);
      if (x >= upper && k != 31) ++k;
      atomicAdd(&hist[k], 1u);  // LDS integer counts: order-independent
    }
  }
  r2[t] = ssd;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) r2[t] += r2[t + w];
    __syncthreads();
  }
  if (t == 0) {
    out[0] = lo;
    out[1] = hi;
    out[2] = mean;
    out[3] = r2[0];
  }
  if (t < 32) out[4 + t] = (delta > 0.0) ? static_cast<double>(hist[t]) : (t == 0 ? static_cast<double>(n) : 0.0);
}

// Column statistics of a row-major n x c FP64 matrix, one workgroup per
// column: mean and population standard deviation (two passes; per-thread
// strided partial sums, then a fixed tree).  A column with zero spread gets
// scale 1, so standardising it yields zeros.
__global__ __launch_bounds__(256) void col_stats_kernel(const double* __restrict__ X, int n, int c,
                                                        double* __restrict__ mean, double* __restrict__ scale) {
  __shared__ double red[256];
  const int col = blockIdx.x, t = threadIdx.x;
  double acc = 0.0;
  for (int i = t; i < n; i += 256) acc += X[static_cast<int64_t>(i) * c + col];
  red[t] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  const double mu = red[0] / static_cast<double>(n);
  __syncthreads();
  acc = 0.0;
  for (int i = t; i < n; i += 256) {
    const double d = X[static_cast<int64_t>(i) * c + col] - mu;
    acc = fma(d, d, acc);
  }
  red[t] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) {
    const double sd = sqrt(red[0] / static_cast<double>(n));
    mean[col] = mu;
    scale[col] = sd > 0.0 ? sd : 1.0;
  }
}

// Xs[i, j] = FP32((X[i, j] - mean[j]) / scale[j]).
__global__ void standardise_kernel(const double* __restrict__ X, int64_t n, int c, const double* __restrict__ mean,
                                   const double* __restrict__ scale, float* __restrict__ Xs) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n * c) return;
  const int j = static_cast<int>(e % c);
  Xs[e] = static_cast<float>((X[e] - mean[j]) / scale[j]);
}

// rms[j] = sqrt(mean over rows (P[i, j] - T[i, j])^2), one workgroup per column.
__global__ __launch_bounds__(256) void rms_err_kernel(const double* __restrict__ P, const double* __restrict__ T,
                                                      int n, int c, double* __restrict__ rms) {
  __shared__ double red[256];
  const int col = blockIdx.x, t = threadIdx.x;
  double acc = 0.0;
  for (int i = t; i < n; i += 256) {
    const int64_t e = static_cast<int64_t>(i) * c + col;
    const double d = P[e] - T[e];
    acc = fma(d, d, acc);
  }
  red[t] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) rms[col] = sqrt(red[0] / static_cast<double>(n));
}

// The learned-bounds policy applied to raw predictions P[b] = (lambda_max,
// lambda_cut, degree) (learned_policy on the host states the same rule).
__device__ __host__ inline void learned_policy(double pm, double pc, double pd, double cut_margin, double* lm,
                                               double* lc, int32_t* m) {
  double d = rint(pd);
  d = d < kLearnedDegMin ? kLearnedDegMin : (d > kLearnedDegMax ? kLearnedDegMax : d);
  if (!(pc < pm)) pc = 0.5 * pm;
  const double c = pc + cut_margin;
  double x = c + kLearnedLmaxMargin * (pm - c);
  if (!(c < x)) x = c + (kLearnedLmaxMargin - 1.0) * fabs(c) + 1e-3;
  *lm = x;
  *lc = c;
  *m = static_cast<int32_t>(d);
}

__global__ void policy_kernel(const double* __restrict__ P, int B, int fo, double cut_margin,
                              double* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const double* p = P + static_cast<int64_t>(b) * fo;
  double lm, lc;
  int32_t m;
  learned_policy(p[0], p[1], p[2], cut_margin, &lm, &lc, &m);
  out[3 * b] = lm;
  out[3 * b + 1] = lc;
  out[3 * b + 2] = static_cast<double>(m);
}

void launch_check(const char* what) { XLS_LAUNCH_CHECK(what); }

}  // namespace

struct xls_mlp_s {
  Dims d;
  float* P = nullptr;   // parameters
  float* G = nullptr;   // gradients
  float* M = nullptr;   // Adam first moment
  float* V = nullptr;   // Adam second moment
  uint16_t* Wb = nullptr;  // bf16 copy of P for inference
  int64_t t = 0;        // Adam step count
  bool bf16_stale = true;
  // activations for up to cap rows: Z_l, H_l per layer (+ input), dZ
  int cap = 0;
  std::vector<float*> Z, H;
  float *Xb = nullptr, *Tb = nullptr, *dA = nullptr, *dB = nullptr, *loss = nullptr;
  int32_t* idx = nullptr;
  double* dF = nullptr;
  double* dOut = nullptr;
  int fcap = 0;
  std::vector<float> in_mean, in_std;
  std::vector<double> out_mean, out_std;
  std::vector<double> train_rms;  // per output, on the training rows (xls_mlp_fit)
  hipStream_t st = nullptr;

  ~xls_mlp_s() {
    if (st) (void)hipStreamSynchronize(st);
    release_rows();
    void* ps[] = {P, G, M, V, Wb, loss, dF, dOut};
    for (void* p : ps) dfree(p);
    if (st) (void)hipStreamDestroy(st);
  }
  void release_rows() {
    for (auto* p : Z) dfree(p);
    for (auto* p : H) dfree(p);
    Z.clear();
    H.clear();
    dfree(Xb);
    dfree(Tb);
    dfree(dA);
    dfree(dB);
    dfree(idx);
    Xb = Tb = dA = dB = nullptr;
    idx = nullptr;
    cap = 0;
  }
  void ensure_rows(int B) {
    if (B <= cap) return;
    release_rows();
    int maxw = 0;
    for (int l = 0; l <= d.nl; ++l) maxw = std::max(maxw, d.size[l]);
    for (int l = 0; l < d.nl; ++l) {
      Z.push_back(dalloc<float>(static_cast<size_t>(B) * d.size[l + 1]));
      H.push_back(dalloc<float>(static_cast<size_t>(B) * d.size[l + 1]));
    }
    Xb = dalloc<float>(static_cast<size_t>(B) * d.size[0]);
    Tb = dalloc<float>(static_cast<size_t>(B) * d.size[d.nl]);
    dA = dalloc<float>(static_cast<size_t>(B) * maxw);
    dB = dalloc<float>(static_cast<size_t>(B) * maxw);
    idx = dalloc<int32_t>(B);
    cap = B;
  }
  void ensure_pred(int B) {
    if (B <= fcap) return;
    dfree(dF);
    dfree(dOut);
    dF = nullptr;
    dOut = nullptr;
    dF = dalloc<double>(static_cast<size_t>(B) * d.size[0]);
    dOut = dalloc<double>(static_cast<size_t>(B) * d.size[d.nl]);
    fcap = B;
  }
};

namespace {

void forward(xls_mlp_s* m, const float* X, int B) {
  const Dims& d = m->d;
  const float* in = X;
  for (int l = 0; l < d.nl; ++l) {
    const int fi = d.size[l], fo = d.size[l + 1];
    const dim3 grid((fo + 63) / 64, (B + 3) / 4);
    hipLaunchKernelGGL(linear_fwd_kernel, grid, dim3(256), 0, m->st, in, m->P + d.woff[l], m->P + d.boff[l], B, fi,
                       fo, l + 1 < d.nl ? 1 : 0, m->Z[l], m->H[l]);
    in = m->H[l];
  }
  launch_check("linear_fwd_kernel");
}

// Gradients of the MSE into m->G for the rows in Xb/Tb (forward already run).
void backward(xls_mlp_s* m, const float* X, const float* T, int B) {
  const Dims& d = m->d;
  const int L = d.nl;
  const int fo_last = d.size[L];
  hipLaunchKernelGGL(mse_grad_kernel, dim3(1), dim3(256), 0, m->st, m->H[L - 1], T, B * fo_last, m->dA, m->loss);
  float* dz = m->dA;
  float* other = m->dB;
  for (int l = L - 1; l >= 0; --l) {
    const int fi = d.size[l], fo = d.size[l + 1];
    const float* in = l == 0 ? X : m->H[l - 1];
    hipLaunchKernelGGL(linear_bwd_w_kernel, dim3((fo + 63) / 64, (fi + 1 + 3) / 4), dim3(256), 0, m->st, in, dz, B,
                       fi, fo, m->G + d.woff[l], m->G + d.boff[l]);
    if (l > 0) {
      hipLaunchKernelGGL(linear_bwd_x_kernel, dim3((fi + 63) / 64, (B + 3) / 4), dim3(256), 0, m->st, dz,
                         m->P + d.woff[l], m->Z[l - 1], B, fi, fo, other);
      std::swap(dz, other);
    }
  }
  launch_check("mlp backward");
}

void adam(xls_mlp_s* m, float lr) {
  ++m->t;
  const double b1 = 0.9, b2 = 0.999;
  const float bc1 = static_cast<float>(1.0 - std::pow(b1, static_cast<double>(m->t)));
  const float bc2 = static_cast<float>(1.0 - std::pow(b2, static_cast<double>(m->t)));
  const int64_t n = m->d.nparam;
  hipLaunchKernelGGL(adam_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, m->st, m->P, m->G,
                     m->M, m->V, n, lr, 0.9f, 0.999f, 1e-8f, bc1, bc2);
  launch_check("adam_kernel");
  m->bf16_stale = true;
}

void upload_f(float* dst, const float* src, int64_t n, hipStream_t st) {
  XLS_HIP(hipMemcpyAsync(dst, src, n * sizeof(float), hipMemcpyHostToDevice, st));
}

// Device buffer freed on scope exit (after the owner synchronised its stream).
template <typename T>
struct DevBuf {
  T* p = nullptr;
  explicit DevBuf(size_t n) : p(dalloc<T>(n)) {}
  ~DevBuf() { dfree(p); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

// Validates minibatches idx[offsets[s] .. offsets[s+1]) of n rows: offsets
// start at 0 and increase strictly, every index is a row.  Returns the
// largest minibatch.
int check_minibatches(int n, const int32_t* idx, const int32_t* offsets, int nsteps) {
  if (offsets[0] != 0) fail(XLS_ERR_INVALID_ARG, "offsets[0] must be 0");
  int maxb = 1;
  for (int s = 0; s < nsteps; ++s) {
    const int b = offsets[s + 1] - offsets[s];
    if (b < 1) fail(XLS_ERR_INVALID_ARG, "empty minibatch (offsets must increase)");
    maxb = std::max(maxb, b);
  }
  for (int64_t k = 0; k < offsets[nsteps]; ++k)
    if (idx[k] < 0 || idx[k] >= n) fail(XLS_ERR_INVALID_ARG, "minibatch index out of range");
  return maxb;
}

// Adam over the minibatches of device rows X (n x in, FP32) and T; losses
// (host, may be NULL) receives each minibatch's loss before its update.
// Synchronises the model's stream before returning.
void train_steps(xls_mlp_s* m, const float* dX, const float* dT, int maxb, const int32_t* idx,
                 const int32_t* offsets, int nsteps, float lr, float* losses) {
  const int F = m->d.size[0], O = m->d.size[m->d.nl];
  DevBuf<int32_t> dI(std::max<int64_t>(1, offsets[nsteps]));
  DevBuf<float> dL(std::max(1, nsteps));
  try {
    m->ensure_rows(maxb);
    XLS_HIP(hipMemcpyAsync(dI.p, idx, offsets[nsteps] * sizeof(int32_t), hipMemcpyHostToDevice, m->st));
    for (int s = 0; s < nsteps; ++s) {
      const int B = offsets[s + 1] - offsets[s];
      const int32_t* ib = dI.p + offsets[s];
      hipLaunchKernelGGL(gather_rows_kernel, dim3((B * F + 255) / 256), dim3(256), 0, m->st, dX, F, ib, B, m->Xb);
      hipLaunchKernelGGL(gather_rows_kernel, dim3((B * O + 255) / 256), dim3(256), 0, m->st, dT, O, ib, B, m->Tb);
      forward(m, m->Xb, B);
      backward(m, m->Xb, m->Tb, B);
      XLS_HIP(hipMemcpyAsync(dL.p + s, m->loss, sizeof(float), hipMemcpyDeviceToDevice, m->st));
      adam(m, lr);
    }
    if (losses && nsteps > 0)
      XLS_HIP(hipMemcpyAsync(losses, dL.p, nsteps * sizeof(float), hipMemcpyDeviceToHost, m->st));
    XLS_HIP(hipStreamSynchronize(m->st));
  } catch (...) {
    (void)hipStreamSynchronize(m->st);
    throw;
  }
}

// bfloat16 inference of B device feature rows into device out (B x outputs),
// with the model's standardisation.
void infer(xls_mlp_s* m, const double* dF, int B, double* dOut) {
  const Dims& d = m->d;
  if (m->bf16_stale) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(static_cast<unsigned>((d.nparam + 255) / 256)), dim3(256), 0, m->st,
                       m->P, m->Wb, d.nparam);
    launch_check("to_bf16_kernel");
    m->bf16_stale = false;
  }
  InferArgs a{};
  a.nl = d.nl;
  for (int l = 0; l <= d.nl; ++l) a.size[l] = d.size[l];
  for (int l = 0; l < d.nl; ++l) {
    a.woff[l] = d.woff[l];
    a.boff[l] = d.boff[l];
  }
  for (int i = 0; i < d.size[0]; ++i) {
    a.in_mean[i] = m->in_mean[i];
    a.in_scale[i] = 1.0f / m->in_std[i];
  }
  for (int i = 0; i < d.size[d.nl]; ++i) {
    a.out_mean[i] = m->out_mean[i];
    a.out_std[i] = m->out_std[i];
  }
  hipLaunchKernelGGL(infer_bf16_kernel, dim3(B), dim3(256), 0, m->st, dF, B, m->Wb, m->P, a, dOut);
  launch_check("infer_bf16_kernel");
}

}  // namespace

extern "C" {

int xls_mlp_create(int32_t nsizes, const int32_t* sizes, const float* params, xls_mlp_t* out) {
  return guarded([&]() -> int {
    if (!out || !sizes || nsizes < 2 || nsizes > kMaxLayers + 1) fail(XLS_ERR_INVALID_ARG, "bad MLP sizes");
    auto* m = new xls_mlp_s();
    try {
      Dims& d = m->d;
      d.nl = nsizes - 1;
      int64_t off = 0;
      for (int l = 0; l < nsizes; ++l) {
        if (sizes[l] < 1 || sizes[l] > kMaxWidth) fail(XLS_ERR_INVALID_ARG, "layer widths must be in [1, 256]");
        d.size[l] = sizes[l];
      }
      if (d.size[0] > 64 || d.size[d.nl] > 8) fail(XLS_ERR_INVALID_ARG, "at most 64 inputs and 8 outputs");
      for (int l = 0; l < d.nl; ++l) {
        d.woff[l] = off;
        off += static_cast<int64_t>(d.size[l]) * d.size[l + 1];
        d.boff[l] = off;
        off += d.size[l + 1];
      }
      d.nparam = off;
      XLS_HIP(hipStreamCreateWithFlags(&m->st, hipStreamNonBlocking));
      m->P = dalloc<float>(off);
      m->G = dalloc<float>(off);
      m->M = dalloc<float>(off);
      m->V = dalloc<float>(off);
      m->Wb = dalloc<uint16_t>(off);
      m->loss = dalloc<float>(1);
      std::vector<float> z(off, 0.0f);
      upload_f(m->P, params ? params : z.data(), off, m->st);
      upload_f(m->M, z.data(), off, m->st);
      upload_f(m->V, z.data(), off, m->st);
      m->in_mean.assign(d.size[0], 0.0f);
      m->in_std.assign(d.size[0], 1.0f);
      m->out_mean.assign(d.size[d.nl], 0.0);
      m->out_std.assign(d.size[d.nl], 1.0);
      XLS_HIP(hipStreamSynchronize(m->st));
    } catch (...) {
      delete m;
      throw;
    }
    *out = m;
    return XLS_OK;
  });
}

void xls_mlp_destroy(xls_mlp_t m) { delete m; }

int xls_mlp_get_params(xls_mlp_t m, float* params, int64_t n) {
  return guarded([&]() -> int {
    if (!m || (params && n < m->d.nparam)) fail(XLS_ERR_INVALID_ARG, "bad argument");
    if (params) {
      XLS_HIP(hipMemcpyAsync(params, m->P, m->d.nparam * sizeof(float), hipMemcpyDeviceToHost, m->st));
      XLS_HIP(hipStreamSynchronize(m->st));
    }
    return static_cast<int>(m->d.nparam);
  });
}

int xls_mlp_set_params(xls_mlp_t m, const float* params, int64_t n) {
  return guarded([&]() -> int {
    if (!m || !params || n != m->d.nparam) fail(XLS_ERR_INVALID_ARG, "bad argument");
    std::vector<float> z(n, 0.0f);
    upload_f(m->P, params, n, m->st);
    upload_f(m->M, z.data(), n, m->st);
    upload_f(m->V, z.data(), n, m->st);
    XLS_HIP(hipStreamSynchronize(m->st));
    m->t = 0;
    m->bf16_stale = true;
    return XLS_OK;
  });
}

int xls_mlp_set_norm(xls_mlp_t m, const float* in_mean, const float* in_std, const double* out_mean,
                     const double* out_std) {
  return guarded([&]() -> int {
    if (!m || !in_mean || !in_std || !out_mean || !out_std) fail(XLS_ERR_INVALID_ARG, "bad argument");
    const int fi = m->d.size[0], fo = m->d.size[m->d.nl];
    for (int i = 0; i < fi; ++i)
      if (!(in_std[i] > 0.0f) || !std::isfinite(in_mean[i])) fail(XLS_ERR_INVALID_ARG, "input scale must be > 0");
    for (int i = 0; i < fo; ++i)
      if (!(out_std[i] > 0.0) || !std::isfinite(out_mean[i])) fail(XLS_ERR_INVALID_ARG, "output scale must be > 0");
    m->in_mean.assign(in_mean, in_mean + fi);
    m->in_std.assign(in_std, in_std + fi);
    m->out_mean.assign(out_mean, out_mean + fo);
    m->out_std.assign(out_std, out_std + fo);
    return XLS_OK;
  });
}

int xls_mlp_forward(xls_mlp_t m, const float* X, int32_t B, float* Y) {
  return guarded([&]() -> int {
    if (!m || !X || !Y || B < 1) fail(XLS_ERR_INVALID_ARG, "bad argument");
    m->ensure_rows(B);
    upload_f(m->Xb, X, static_cast<int64_t>(B) * m->d.size[0], m->st);
    forward(m, m->Xb, B);
    const int fo = m->d.size[m->d.nl];
    XLS_HIP(hipMemcpyAsync(Y, m->H[m->d.nl - 1], static_cast<size_t>(B) * fo * sizeof(float), hipMemcpyDeviceToHost,
                           m->st));
    XLS_HIP(hipStreamSynchronize(m->st));
    return XLS_OK;
  });
}

int xls_mlp_gradient(xls_mlp_t m, const float* X, const float* T, int32_t B, float* grads, float* loss) {
  return guarded([&]() -> int {
    if (!m || !X || !T || !grads || B < 1) fail(XLS_ERR_INVALID_ARG, "bad argument");
    m->ensure_rows(B);
    upload_f(m->Xb, X, static_cast<int64_t>(B) * m->d.size[0], m->st);
    upload_f(m->Tb, T, static_cast<int64_t>(B) * m->d.size[m->d.nl], m->st);
    forward(m, m->Xb, B);
    backward(m, m->Xb, m->Tb, B);
    XLS_HIP(hipMemcpyAsync(grads, m->G, m->d.nparam * sizeof(float), hipMemcpyDeviceToHost, m->st));
    if (loss) XLS_HIP(hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->st));
    XLS_HIP(hipStreamSynchronize(m->st));
    return XLS_OK;
  });
}

int xls_mlp_train(xls_mlp_t m, const float* X, const float* T, int32_t n, const int32_t* idx,
                  const int32_t* offsets, int32_t nsteps, float lr, float* losses) {
  return guarded([&]() -> int {
    if (!m || !X || !T || !idx || !offsets || n < 1 || nsteps < 0 || !(lr > 0.0f))
      fail(XLS_ERR_INVALID_ARG, "bad argument");
    const int maxb = check_minibatches(n, idx, offsets, nsteps);
    const int F = m->d.size[0], O = m->d.size[m->d.nl];
    DevBuf<float> dX(static_cast<size_t>(n) * F), dT(static_cast<size_t>(n) * O);
    upload_f(dX.p, X, static_cast<int64_t>(n) * F, m->st);
    upload_f(dT.p, T, static_cast<int64_t>(n) * O, m->st);
    train_steps(m, dX.p, dT.p, maxb, idx, offsets, nsteps, lr, losses);
    return XLS_OK;
  });
}

int xls_mlp_fit(xls_mlp_t m, const double* F, const double* T, int32_t n, const int32_t* idx,
                const int32_t* offsets, int32_t nsteps, float lr, float* losses) {
  return guarded([&]() -> int {
    if (!m || !F || !T || !idx || !offsets || n < 1 || nsteps < 0 || !(lr > 0.0f))
      fail(XLS_ERR_INVALID_ARG, "bad argument");
    const int fi = m->d.size[0], fo = m->d.size[m->d.nl];
    if (!finite_all(F, static_cast<int64_t>(n) * fi) || !finite_all(T, static_cast<int64_t>(n) * fo))
      fail(XLS_ERR_INVALID_ARG, "features and targets must be finite");
    const int maxb = check_minibatches(n, idx, offsets, nsteps);
    DevBuf<double> dF(static_cast<size_t>(n) * fi), dT(static_cast<size_t>(n) * fo), stats(2 * (fi + fo));
    DevBuf<double> pred(static_cast<size_t>(n) * fo), rms(fo);
    DevBuf<float> sF(static_cast<size_t>(n) * fi), sT(static_cast<size_t>(n) * fo);
    XLS_HIP(hipMemcpyAsync(dF.p, F, static_cast<size_t>(n) * fi * 8, hipMemcpyHostToDevice, m->st));
    XLS_HIP(hipMemcpyAsync(dT.p, T, static_cast<size_t>(n) * fo * 8, hipMemcpyHostToDevice, m->st));
    double* fmean = stats.p;
    double* fscale = stats.p + fi;
    double* tmean = stats.p + 2 * fi;
    double* tscale = stats.p + 2 * fi + fo;
    hipLaunchKernelGGL(col_stats_kernel, dim3(fi), dim3(256), 0, m->st, dF.p, n, fi, fmean, fscale);
    hipLaunchKernelGGL(col_stats_kernel, dim3(fo), dim3(256), 0, m->st, dT.p, n, fo, tmean, tscale);
    const int64_t ef = static_cast<int64_t>(n) * fi, eo = static_cast<int64_t>(n) * fo;
    hipLaunchKernelGGL(standardise_kernel, dim3(static_cast<unsigned>((ef + 255) / 256)), dim3(256), 0, m->st,
                       dF.p, static_cast<int64_t>(n), fi, fmean, fscale, sF.p);
    hipLaunchKernelGGL(standardise_kernel, dim3(static_cast<unsigned>((eo + 255) / 256)), dim3(256), 0, m->st,
                       dT.p, static_cast<int64_t>(n), fo, tmean, tscale, sT.p);
    launch_check("standardise_kernel");
    train_steps(m, sF.p, sT.p, maxb, idx, offsets, nsteps, lr, losses);
    std::vector<double> h(2 * (fi + fo));
    XLS_HIP(hipMemcpyAsync(h.data(), stats.p, h.size() * 8, hipMemcpyDeviceToHost, m->st));
    XLS_HIP(hipStreamSynchronize(m->st));
    for (int i = 0; i < fi; ++i) {
      m->in_mean[i] = static_cast<float>(h[i]);
      m->in_std[i] = static_cast<float>(h[fi + i]);
      if (!(m->in_std[i] > 0.0f)) m->in_std[i] = 1.0f;  // a spread below FP32's range
    }
    for (int i = 0; i < fo; ++i) {
      m->out_mean[i] = h[2 * fi + i];
      m->out_std[i] = h[2 * fi + fo + i];
    }
    // the model's error on its training rows, with the inference it will run
    infer(m, dF.p, n, pred.p);
    hipLaunchKernelGGL(rms_err_kernel, dim3(fo), dim3(256), 0, m->st, pred.p, dT.p, n, fo, rms.p);
    launch_check("rms_err_kernel");
    m->train_rms.assign(fo, 0.0);
    XLS_HIP(hipMemcpyAsync(m->train_rms.data(), rms.p, fo * 8, hipMemcpyDeviceToHost, m->st));
    XLS_HIP(hipStreamSynchronize(m->st));
    return XLS_OK;
  });
}

int xls_mlp_train_rms(xls_mlp_t m, double* rms, int32_t cap) {
  return guarded([&]() -> int {
    if (!m || !rms || cap < 1) fail(XLS_ERR_INVALID_ARG, "bad argument");
    if (m->train_rms.empty()) fail(XLS_ERR_STATE, "the model has not been fitted (xls_mlp_fit)");
    const int k = std::min<int>(cap, static_cast<int>(m->train_rms.size()));
    for (int i = 0; i < k; ++i) rms[i] = m->train_rms[i];
    return k;
  });
}

int xls_mlp_bounds(xls_mlp_t m, const double* features, int32_t B, double* lam_max, double* lam_cut,
                   int32_t* degree) {
  return guarded([&]() -> int {
    if (!m || !features || !lam_max || !lam_cut || !degree || B < 1) fail(XLS_ERR_INVALID_ARG, "bad argument");
    const int fi = m->d.size[0], fo = m->d.size[m->d.nl];
    if (fo < 3) fail(XLS_ERR_INVALID_ARG, "the model needs 3 outputs (lambda_max, lambda_cut, degree)");
    if (m->train_rms.size() < 2) fail(XLS_ERR_STATE, "the model has not been fitted (xls_mlp_fit)");
    if (!finite_all(features, static_cast<int64_t>(B) * fi)) fail(XLS_ERR_INVALID_ARG, "features not finite");
    m->ensure_pred(B);
    XLS_HIP(hipMemcpyAsync(m->dF, features, static_cast<size_t>(B) * fi * 8, hipMemcpyHostToDevice, m->st));
    infer(m, m->dF, B, m->dOut);
    DevBuf<double> pol(3 * static_cast<size_t>(B));
    hipLaunchKernelGGL(policy_kernel, dim3((B + 63) / 64), dim3(64), 0, m->st, m->dOut, B, fo,
                       kLearnedCutSigmas * m->train_rms[1], pol.p);
    launch_check("policy_kernel");
    std::vector<double> h(3 * static_cast<size_t>(B));
    XLS_HIP(hipMemcpyAsync(h.data(), pol.p, h.size() * 8, hipMemcpyDeviceToHost, m->st));
    XLS_HIP(hipStreamSynchronize(m->st));
    for (int b = 0; b < B; ++b) {
      lam_max[b] = h[3 * b];
      lam_cut[b] = h[3 * b + 1];
      degree[b] = static_cast<int32_t>(h[3 * b + 2]);
    }
    return XLS_OK;
  });
}

int xls_learned_safe_bounds(int32_t B, const double* lam_max, const double* lam_cut, double cut_margin,
                            double* lm_out, double* lc_out) {
  return guarded([&]() -> int {
    if (B < 0 || (B > 0 && (!lam_max || !lam_cut || !lm_out || !lc_out)) || !(cut_margin >= 0))
      fail(XLS_ERR_INVALID_ARG, "bad argument");
    for (int b = 0; b < B; ++b) {
      int32_t m;
      learned_policy(lam_max[b], lam_cut[b], kLearnedDegMin, cut_margin, &lm_out[b], &lc_out[b], &m);
    }
    return XLS_OK;
  });
}

int xls_mlp_predict(xls_mlp_t m, const double* features, int32_t B, double* out) {
  return guarded([&]() -> int {
    if (!m || !features || !out || B < 1) fail(XLS_ERR_INVALID_ARG, "bad argument");
    const Dims& d = m->d;
    const int fi = d.size[0], fo = d.size[d.nl];
    m->ensure_pred(B);
    XLS_HIP(hipMemcpyAsync(m->dF, features, static_cast<size_t>(B) * fi * 8, hipMemcpyHostToDevice, m->st));
    infer(m, m->dF, B, m->dOut);
    XLS_HIP(hipMemcpyAsync(out, m->dOut, static_cast<size_t>(B) * fo * 8, hipMemcpyDeviceToHost, m->st));
    XLS_HIP(hipStreamSynchronize(m->st));
    return XLS_OK;
  });
}

int xls_subdomain_features(xls_subdomain_t s, double* f) {
  return guarded([&]() -> int {
    if (!s || !f) fail(XLS_ERR_INVALID_ARG, "bad argument");
    double* dst = dalloc<double>(36);
    double h[36];
    try {
      hipLaunchKernelGGL(vstats_kernel, dim3(1), dim3(1024), 0, s->st, s->v64, s->nd, dst);
      launch_check("vstats_kernel");
      XLS_HIP(hipMemcpyAsync(h, dst, sizeof(h), hipMemcpyDeviceToHost, s->st));
      XLS_HIP(hipStreamSynchronize(s->st));
    } catch (...) {
      dfree(dst);
      throw;
    }
    dfree(dst);
    const double nd = static_cast<double>(s->nd);
    std::fill(f, f + 64, 0.0);
    for (int k = 0; k < 32; ++k) f[k] = h[4 + k] / nd;
    int cmin = s->n[0];
    int64_t ncore = 1;
    for (int a = 0; a < 3; ++a) {
      cmin = std::min(cmin, s->core_lo[a]);
      ncore *= s->core_hi[a] - s->core_lo[a];
    }
    double gsum = 0.0;
    for (double g : s->tab.gamma) gsum += std::fabs(g);
    // largest eigenvalue of -1/2 Lap per axis: (1/(2h^2)) sum_p |w| terms at k = pi
    double w[kRadius + 1];
    {
      double fct[2 * kRadius + 1];
      fct[0] = 1.0;
      for (int i = 1; i <= 2 * kRadius; ++i) fct[i] = fct[i - 1] * i;
      double sw = 0.0;
      for (int p = 1; p <= kRadius; ++p) {
        w[p] = 2.0 * ((p % 2 == 1) ? 1.0 : -1.0) * fct[kRadius] * fct[kRadius] /
               (static_cast<double>(p) * p * fct[kRadius - p] * fct[kRadius + p]);
        sw += w[p];
      }
      w[0] = -2.0 * sw;
    }
    double s_pi = -w[0];
    for (int p = 1; p <= kRadius; ++p) s_pi -= 2.0 * w[p] * ((p % 2 == 1) ? -1.0 : 1.0);
    const double vals[15] = {static_cast<double>(s->n_atoms),
                             static_cast<double>(s->n[0]),
                             static_cast<double>(s->n[1]),
                             static_cast<double>(s->n[2]),
                             s->h,
                             cmin * s->h,
                             h[0],
                             h[1],
                             h[2],
                             std::sqrt(h[3] / nd),
                             static_cast<double>(s->ns),
                             4.0 * s->n_atoms,
                             gsum,
                             static_cast<double>(ncore) / nd,
                             1.5 * s_pi / (s->h * s->h)};
    for (int k = 0; k < 15; ++k) f[32 + k] = vals[k];
    return XLS_OK;
  });
}

}  // extern "C"
