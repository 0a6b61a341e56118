// Projection and rotation GEMMs on the matrix cores (Sec. V-B.3: the
// Rayleigh-Ritz projection H_s = Psi_f^T (H Psi_f), M_s = Psi_f^T Psi_f and the
// subspace rotation Psi = Psi_f Y are dense products).
//
//   gemm_tn : C = A^T B with a long inner dimension K = N_d, split along K
//             (each split's partial tile is written in FP64 and the splits are
//             summed in a fixed order: deterministic, no atomics).
//   gemm_nn : C = A B with A the tall N_d x N_s block and B the N_s x N_s
//             rotation.
// Arithmetic forms (all accumulate in the MFMA accumulator type):
//   FP64  v_mfma_f64_16x16x4f64 (FP32 inputs are widened exactly),
//   FP32  v_mfma_f32_16x16x4f32,
//   BF16X3 each FP32 operand a = a_hi + a_lo with a_hi = bf16(a),
//          a_lo = bf16(a - a_hi) (round to nearest even), three products
//          hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16.
// Tiles: TILE x TILE per workgroup of 4 wavefronts (2 x 2), each wavefront a
// (TILE/2)^2 block of 16 x 16 MFMA tiles; operands staged through LDS with k
// contiguous.
#include <algorithm>
#include <atomic>

#include "xls_internal.h"

namespace xls {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

constexpr int MF_F64 = XLS_PREC_FP64;
constexpr int MF_F32 = XLS_PREC_FP32;
constexpr int MF_BF = XLS_PREC_BF16X3;

__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nb) {
  const uint32_t xcd = bid & 7u, idx = bid >> 3;
  const uint32_t q = nb >> 3, r = nb & 7u;
  return xcd * q + min(xcd, r) + idx;
}

__device__ __forceinline__ uint16_t bf16_rne_bits(float a) {
  uint32_t u = __float_as_uint(a);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) {
  return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

typedef __bf16 bf2_t __attribute__((ext_vector_type(2)));
typedef float f2_t __attribute__((ext_vector_type(2)));
// Split of two FP32 values with the hardware's packed round-to-nearest-even
// conversion: hi = bf16(a), lo = bf16(a - hi); each word holds element 0 in
// its low half (the LDS order of two consecutive bf16 values).  For finite
// values the bits equal bf16_rne_bits'.
__device__ __forceinline__ void split_pair(float a0, float a1, uint32_t& hi, uint32_t& lo) {
  const f2_t a = {a0, a1};
  hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(a, bf2_t));
  const f2_t h = {__uint_as_float(hi << 16), __uint_as_float(hi & 0xFFFF0000u)};
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(a - h, bf2_t));
}

// ---- per-form traits: LDS element, k per MFMA, operand loads, MFMA --------
template <int MF>
struct Form;

template <>
struct Form<MF_F64> {
  using acc_t = d4_t;
  static constexpr int BK = 16;
  static constexpr int KS = 4;
  static constexpr int PAD = 1;
  using lds_t = double;
  template <typename T>
  __device__ static void put(lds_t* hi, lds_t*, int off, T v) {
    hi[off] = static_cast<double>(v);
  }
  __device__ static void step(acc_t& acc, const lds_t* xh, const lds_t*, const lds_t* yh,
                              const lds_t*, int xrow, int yrow, int stride, int k, int lane) {
    const double a = xh[xrow * stride + k + (lane >> 4)];
    const double b = yh[yrow * stride + k + (lane >> 4)];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  __device__ static double get(const acc_t& a, int r) { return a[r]; }
  // accumulator element r of a lane holds row (lane/16) + 4r of the 16x16 tile
  __device__ static int orow(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <>
struct Form<MF_F32> {
  using acc_t = f4_t;
  static constexpr int BK = 16;
  static constexpr int KS = 4;
  static constexpr int PAD = 1;
  using lds_t = float;
  template <typename T>
  __device__ static void put(lds_t* hi, lds_t*, int off, T v) {
    hi[off] = static_cast<float>(v);
  }
  __device__ static void step(acc_t& acc, const lds_t* xh, const lds_t*, const lds_t* yh,
                              const lds_t*, int xrow, int yrow, int stride, int k, int lane) {
    const float a = xh[xrow * stride + k + (lane >> 4)];
    const float b = yh[yrow * stride + k + (lane >> 4)];
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
  __device__ static double get(const acc_t& a, int r) { return a[r]; }
  // accumulator element r of a lane holds row 4(lane/16) + r of the 16x16 tile
  __device__ static int orow(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <>
struct Form<MF_BF> {
  using acc_t = f4_t;
  static constexpr int BK = 32;
  static constexpr int KS = 32;
  static constexpr int PAD = 8;
  using lds_t = uint16_t;
  template <typename T>
  __device__ static void put(lds_t* hi, lds_t* lo, int off, T v) {
    const float a = static_cast<float>(v);
    const uint16_t h = bf16_rne_bits(a);
    hi[off] = h;
    lo[off] = bf16_rne_bits(a - bf16_bits_to_f32(h));
  }
  __device__ static void step(acc_t& acc, const lds_t* xh, const lds_t* xl, const lds_t* yh,
                              const lds_t* yl, int xrow, int yrow, int stride, int k, int lane) {
    const int ko = k + 8 * (lane >> 4);
    const bf8_t ah = *reinterpret_cast<const bf8_t*>(xh + xrow * stride + ko);
    const bf8_t al = *reinterpret_cast<const bf8_t*>(xl + xrow * stride + ko);
    const bf8_t bh = *reinterpret_cast<const bf8_t*>(yh + yrow * stride + ko);
    const bf8_t bl = *reinterpret_cast<const bf8_t*>(yl + yrow * stride + ko);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
  }
  __device__ static double get(const acc_t& a, int r) { return a[r]; }
  __device__ static int orow(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <int MF, int TILE>
struct Smem {
  using F = Form<MF>;
  static constexpr int stride = F::BK + F::PAD;
  static constexpr int elems = TILE * stride;                 // one operand, one part
  static constexpr int parts = (MF == MF_BF) ? 2 : 1;
  static constexpr size_t bytes = 2 * parts * elems * sizeof(typename F::lds_t);
};

// C = A^T B partial over one K split.  A: K x M (lda), B: K x N (ldb).
template <typename TIN, int MF, int TILE>
__global__ __launch_bounds__(256) void gemm_tn_kernel(const TIN* __restrict__ A, int64_t lda,
                                                      const TIN* __restrict__ B, int64_t ldb, int M,
                                                      int N, int64_t K, int64_t kchunk, int tm,
                                                      int tn, int sym, double* __restrict__ P) {
  using F = Form<MF>;
  using L = typename F::lds_t;
  constexpr int BK = F::BK, ST = Smem<MF, TILE>::stride, E = Smem<MF, TILE>::elems;
  constexpr int WB = TILE / 32;
  __shared__ __align__(16) L sm[Smem<MF, TILE>::bytes / sizeof(L)];
  L* xh = sm;
  L* yh = sm + E;
  L* xl = (MF == MF_BF) ? sm + 2 * E : nullptr;
  L* yl = (MF == MF_BF) ? sm + 3 * E : nullptr;

  const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
  const int ntile = sym ? tm * (tm + 1) / 2 : tm * tn;
  const int split = static_cast<int>(lb / ntile);
  int tt = static_cast<int>(lb % ntile);
  int bm, bn;
  if (sym) {  // enumerate upper tiles bm <= bn column by column
    bn = 0;
    while (tt > bn) {
      tt -= bn + 1;
      ++bn;
    }
    bm = tt;
  } else {
    bm = tt % tm;
    bn = tt / tm;
  }
  const int m0 = bm * TILE, n0 = bn * TILE;
  const int64_t kb0 = static_cast<int64_t>(split) * kchunk;
  const int64_t kend = min(K, kb0 + kchunk);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  typename F::acc_t acc[WB][WB];
#pragma unroll
  for (int i = 0; i < WB; ++i)
#pragma unroll
    for (int j = 0; j < WB; ++j) acc[i][j] = typename F::acc_t{};

  for (int64_t kb = kb0; kb < kend; kb += BK) {
#pragma unroll
    for (int it = 0; it < (TILE * BK) / 256; ++it) {
      const int l = tid + it * 256;
      const int k = l % BK, r = l / BK;
      const int64_t kk = kb + k;
      const bool kin = kk < kend;
      const TIN av = (kin && m0 + r < M) ? A[kk + static_cast<int64_t>(m0 + r) * lda] : TIN(0);
      const TIN bv = (kin && n0 + r < N) ? B[kk + static_cast<int64_t>(n0 + r) * ldb] : TIN(0);
      F::put(xh, xl, r * ST + k, av);
      F::put(yh, yl, r * ST + k, bv);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < BK; k += F::KS)
#pragma unroll
      for (int bi = 0; bi < WB; ++bi)
#pragma unroll
        for (int bj = 0; bj < WB; ++bj)
          F::step(acc[bi][bj], xh, xl, yh, yl, wr * (TILE / 2) + bi * 16 + (lane & 15),
                  wc * (TILE / 2) + bj * 16 + (lane & 15), ST, k, lane);
    __syncthreads();
  }
  double* Ps = P + static_cast<int64_t>(split) * M * N;
#pragma unroll
  for (int bi = 0; bi < WB; ++bi)
#pragma unroll
    for (int bj = 0; bj < WB; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr * (TILE / 2) + bi * 16 + F::orow(lane, r);
        const int cl = n0 + wc * (TILE / 2) + bj * 16 + (lane & 15);
        if (row < M && cl < N) Ps[row + static_cast<int64_t>(cl) * M] = F::get(acc[bi][bj], r);
      }
}

__global__ void tn_reduce_kernel(const double* __restrict__ P, int splits, int M, int N, int tile,
                                 int sym, int symmetrize, double* __restrict__ C, int64_t ldc) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(M) * N) return;
  const int i = static_cast<int>(e % M), j = static_cast<int>(e / M);
  const int64_t MN = static_cast<int64_t>(M) * N;
  auto get = [&](int a, int b) {
    if (sym && (a / tile) > (b / tile)) {
      const int t = a;
      a = b;
      b = t;
    }
    double s = 0.0;
    for (int sp = 0; sp < splits; ++sp) s += P[sp * MN + a + static_cast<int64_t>(b) * M];
    return s;
  };
  double v = get(i, j);
  if (symmetrize) v = 0.5 * (v + get(j, i));
  C[i + static_cast<int64_t>(j) * ldc] = v;
}

// The same reduction for square products that are symmetric (only tiles on
// or above the block diagonal computed) or symmetrized: one block per pair of
// 16 x 16 output tiles (I, J), I <= J, sums the partials of both tiles in
// split order into LDS with coalesced reads, then writes both tiles
// coalesced.  Per element the arithmetic is that of tn_reduce_kernel.
constexpr int kRedT = 16;
__global__ __launch_bounds__(256) void tn_reduce_pairs_kernel(const double* __restrict__ P, int splits, int M,
                                                              int tile, int sym, int symmetrize,
                                                              double* __restrict__ C, int64_t ldc, int nt) {
  __shared__ double a[kRedT][kRedT + 1], b[kRedT][kRedT + 1];
  int p = static_cast<int>(blockIdx.x), I = 0;
  while (p >= nt - I) {
    p -= nt - I;
    ++I;
  }
  const int J = I + p;
  const int r = threadIdx.x % kRedT, c = threadIdx.x / kRedT;
  const int64_t MN = static_cast<int64_t>(M) * M;
  const int ai = I * kRedT + r, aj = J * kRedT + c;  // a[r][c] = P(ai, aj)
  const int bi = J * kRedT + r, bj = I * kRedT + c;  // b[r][c] = P(bi, bj)
  const bool va = ai < M && aj < M, vb = bi < M && bj < M;
  const double* pa = P + ai + static_cast<int64_t>(aj) * M;
  const double* pb = P + bi + static_cast<int64_t>(bj) * M;
  double sa = 0.0, sb = 0.0;
  for (int sp = 0; sp < splits; ++sp) {
    if (va) sa += pa[sp * MN];
    if (vb) sb += pb[sp * MN];
  }
  a[r][c] = sa;
  b[r][c] = sb;
  __syncthreads();
  // element (x, y) of the product: P(x, y), or P(y, x) where a symmetric
  // product kept only the upper block triangle
  {
    const int i = ai, j = aj;  // output (i, j): row in tile I, column in tile J
    const double vij = (sym && i / tile > j / tile) ? b[c][r] : a[r][c];
    const double vji = (sym && j / tile > i / tile) ? a[r][c] : b[c][r];
    if (va) C[i + static_cast<int64_t>(j) * ldc] = symmetrize ? 0.5 * (vij + vji) : vij;
  }
  if (I != J) {
    const int i = bi, j = bj;  // output (i, j): row in tile J, column in tile I
    const double vij = (sym && i / tile > j / tile) ? a[c][r] : b[r][c];
    const double vji = (sym && j / tile > i / tile) ? b[r][c] : a[c][r];
    if (vb) C[i + static_cast<int64_t>(j) * ldc] = symmetrize ? 0.5 * (vij + vji) : vij;
  }
}

void launch_tn_reduce(const double* work, int splits, int M, int N, int tile, int sym, int symmetrize, double* C,
                      int64_t ldc, hipStream_t st) {
  if ((sym || symmetrize) && M == N) {
    const int nt = (M + kRedT - 1) / kRedT;
    const int64_t pairs = static_cast<int64_t>(nt) * (nt + 1) / 2;
    hipLaunchKernelGGL(tn_reduce_pairs_kernel, dim3(static_cast<unsigned>(pairs)), dim3(256), 0, st, work, splits,
                       M, tile, sym, symmetrize, C, ldc, nt);
    XLS_LAUNCH_CHECK("tn_reduce_pairs_kernel");
    return;
  }
  const int64_t tot = static_cast<int64_t>(M) * N;
  hipLaunchKernelGGL(tn_reduce_kernel, dim3(static_cast<unsigned>((tot + 255) / 256)), dim3(256), 0, st, work,
                     splits, M, N, tile, sym, symmetrize, C, ldc);
  XLS_LAUNCH_CHECK("tn_reduce_kernel");
}

// C[M x N] = A[M x K] B[K x N]; the MFMA computes the transposed tile so that
// each lane's results run down a column of C (coalesced stores).
template <typename TIN, typename TB, typename TOUT, int MF, int TILE>
__global__ __launch_bounds__(256) void gemm_nn_kernel(const TIN* __restrict__ A, int64_t lda,
                                                      const TB* __restrict__ B, int64_t ldb, int M,
                                                      int N, int K, int tmM, int tnN,
                                                      TOUT* __restrict__ C, int64_t ldc) {
  using F = Form<MF>;
  using L = typename F::lds_t;
  constexpr int BK = F::BK, ST = Smem<MF, TILE>::stride, E = Smem<MF, TILE>::elems;
  constexpr int WB = TILE / 32;
  __shared__ __align__(16) L sm[Smem<MF, TILE>::bytes / sizeof(L)];
  L* ah = sm;  // A tile rows = m
  L* bh = sm + E;  // B tile rows = n
  L* al = (MF == MF_BF) ? sm + 2 * E : nullptr;
  L* bl = (MF == MF_BF) ? sm + 3 * E : nullptr;

  const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
  const int bn = static_cast<int>(lb % tnN), bm = static_cast<int>(lb / tnN);
  const int m0 = bm * TILE, n0 = bn * TILE;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;  // wr: n direction, wc: m direction
  typename F::acc_t acc[WB][WB];
#pragma unroll
  for (int i = 0; i < WB; ++i)
#pragma unroll
    for (int j = 0; j < WB; ++j) acc[i][j] = typename F::acc_t{};

  for (int kb = 0; kb < K; kb += BK) {
#pragma unroll
    for (int it = 0; it < (TILE * BK) / 256; ++it) {
      const int l = tid + it * 256;
      {  // A: coalesced along m
        const int m = l % TILE, k = l / TILE;
        const bool ok = (m0 + m < M) && (kb + k < K);
        const TIN v = ok ? A[(m0 + m) + static_cast<int64_t>(kb + k) * lda] : TIN(0);
        F::put(ah, al, m * ST + k, v);
      }
      {  // B: coalesced along k
        const int k = l % BK, n = l / BK;
        const bool ok = (n0 + n < N) && (kb + k < K);
        const TB v = ok ? B[(kb + k) + static_cast<int64_t>(n0 + n) * ldb] : TB(0);
        F::put(bh, bl, n * ST + k, v);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < BK; k += F::KS)
#pragma unroll
      for (int bi = 0; bi < WB; ++bi)
#pragma unroll
        for (int bj = 0; bj < WB; ++bj)
          F::step(acc[bi][bj], bh, bl, ah, al, wr * (TILE / 2) + bi * 16 + (lane & 15),
                  wc * (TILE / 2) + bj * 16 + (lane & 15), ST, k, lane);
    __syncthreads();
  }
#pragma unroll
  for (int bi = 0; bi < WB; ++bi)
#pragma unroll
    for (int bj = 0; bj < WB; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = n0 + wr * (TILE / 2) + bi * 16 + F::orow(lane, r);
        const int m = m0 + wc * (TILE / 2) + bj * 16 + (lane & 15);
        if (m < M && n < N) C[m + static_cast<int64_t>(n) * ldc] = static_cast<TOUT>(F::get(acc[bi][bj], r));
      }
}

__global__ void split_bf16_kernel(const float* __restrict__ a, uint16_t* __restrict__ hi,
                                  uint16_t* __restrict__ lo, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint16_t h = bf16_rne_bits(a[i]);
  hi[i] = h;
  lo[i] = bf16_rne_bits(a[i] - bf16_bits_to_f32(h));
}

__global__ void d2f_kernel(const double* __restrict__ s, float* __restrict__ d, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) d[i] = static_cast<float>(s[i]);
}


// ---------------------------------------------------------------------------
// Large-tile kernels for the long-K projection and the tall rotation.  Each
// wavefront holds a 4 x 4 block of 16 x 16 MFMA tiles and reuses its operand
// fragments across that block; operands arrive through 16-byte global loads
// staged in registers (the next K slab loads while the current one computes).
// Used when leading dimensions are multiples of the vector width.
// ---------------------------------------------------------------------------
template <int MF>
struct Frag;
template <>
struct Frag<MF_F64> {
  using t = double;
  static constexpr int KS = 4;
  __device__ static t load(const double* h, const double*, int row, int stride, int k, int lane) {
    return h[row * stride + k + (lane >> 4)];
  }
  __device__ static void mma(d4_t& acc, const t& a, const t& b) {
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
};
template <>
struct Frag<MF_F32> {
  using t = float;
  static constexpr int KS = 4;
  __device__ static t load(const float* h, const float*, int row, int stride, int k, int lane) {
    return h[row * stride + k + (lane >> 4)];
  }
  __device__ static void mma(f4_t& acc, const t& a, const t& b) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
};
// LDS layout of the large-tile BF operands: rows of 32 bf16 (four 16-byte
// chunks) without padding; chunk c of row r sits at position
// c ^ (((r >> 2) ^ (r >> 4)) & 3).  Sixteen consecutive rows then cover all
// 64 banks once for a 16-byte fragment read, eight rows of 64 bytes are
// written in the minimum two passes, and the transposed 32-bit stores of
// the NN kernel (rows 4 j + e) spread over every bank.
__device__ __forceinline__ int bf_off(int r, int k) {
  return r * 32 + (((k >> 3) ^ (((r >> 2) ^ (r >> 4)) & 3)) << 3) + (k & 7);
}

template <>
struct Frag<MF_BF> {
  struct t {
    bf8_t h, l;
  };
  static constexpr int KS = 32;
  // stride is fixed at 32 for this form (bf_off)
  __device__ static t load(const uint16_t* h, const uint16_t* l, int row, int, int k, int lane) {
    const int o = bf_off(row, k + 8 * (lane >> 4));
    return t{*reinterpret_cast<const bf8_t*>(h + o), *reinterpret_cast<const bf8_t*>(l + o)};
  }
  __device__ static void mma(f4_t& acc, const t& a, const t& b) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l, b.h, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.l, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.h, acc, 0, 0, 0);
  }
};

template <int MF>
struct BigLds {
  using L = typename Form<MF>::lds_t;
  static constexpr int BK = (MF == MF_F64) ? 16 : 32;
  // padded rows (16-byte aligned) for FP64/FP32; the BF form swizzles instead (bf_off)
  static constexpr int STRIDE = BK + (MF == MF_BF ? 0 : (MF == MF_F64 ? 2 : 4));
  static constexpr int PARTS = (MF == MF_BF) ? 2 : 1;
};

// Writes VEC consecutive-k values of row r into the LDS operand (split into
// bf16 hi/lo for the BF form); values past kend are zero.
template <int MF, typename TIN, int VEC>
__device__ __forceinline__ void big_put_row(typename Form<MF>::lds_t* h, typename Form<MF>::lds_t* l, int off,
                                            const TIN (&v)[VEC]) {
  if constexpr (MF == MF_BF) {
    static_assert(VEC == 2 || VEC == 4, "pairs of k values");
    uint32_t hp[VEC / 2], lp[VEC / 2];
#pragma unroll
    for (int e = 0; e < VEC / 2; ++e)
      split_pair(static_cast<float>(v[2 * e]), static_cast<float>(v[2 * e + 1]), hp[e], lp[e]);
    if constexpr (VEC == 4) {
      *reinterpret_cast<uint2*>(h + off) = make_uint2(hp[0], hp[1]);
      *reinterpret_cast<uint2*>(l + off) = make_uint2(lp[0], lp[1]);
    } else {
      *reinterpret_cast<uint32_t*>(h + off) = hp[0];
      *reinterpret_cast<uint32_t*>(l + off) = lp[0];
    }
  } else {
    using L = typename Form<MF>::lds_t;
#pragma unroll
    for (int e = 0; e < VEC; ++e) h[off + e] = static_cast<L>(v[e]);
  }
}

// Partial C = A^T B over one K split, T x T output tile per workgroup (T =
// 128 or 96): four waves in a 2 x 2 grid, each owning a (T/2) x (T/2)
// sub-tile of NI x NI MFMA blocks of 16 x 16.  The 96 tile covers an order
// of 480 (or any multiple of 96) without padding, and the triangle of a
// symmetric product with less redundant work on its diagonal tiles.
template <typename TIN, int MF, int T>
__global__ __launch_bounds__(256, 2) void gemm_tn_big_kernel(const TIN* __restrict__ A, int64_t lda,
                                                          const TIN* __restrict__ B, int64_t ldb, int M,
                                                          int N, int64_t K, int64_t kchunk, int tm, int tn,
                                                          int sym, double* __restrict__ P) {
  using Lc = BigLds<MF>;
  using L = typename Lc::L;
  using FR = Frag<MF>;
  static_assert(T == 128 || T == 96, "large TN tiles are 128 or 96");
  constexpr int BK = Lc::BK, ST = Lc::STRIDE;
  constexpr int WT = T / 2, NI = WT / 16;
  constexpr int VEC = 16 / sizeof(TIN);
  constexpr int PERCOL = BK / VEC;
  static_assert((T * PERCOL) % 256 == 0, "whole loads per thread");
  constexpr int LOADS = T * PERCOL / 256;
  __shared__ __align__(16) L sm[2 * Lc::PARTS * T * ST];
  L* xh = sm;
  L* yh = sm + T * ST;
  L* xl = (MF == MF_BF) ? sm + 2 * T * ST : nullptr;
  L* yl = (MF == MF_BF) ? sm + 3 * T * ST : nullptr;

  const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
  const int ntile = sym ? tm * (tm + 1) / 2 : tm * tn;
  const int split = static_cast<int>(lb / ntile);
  int tt = static_cast<int>(lb % ntile);
  int bm, bn;
  if (sym) {
    bn = 0;
    while (tt > bn) {
      tt -= bn + 1;
      ++bn;
    }
    bm = tt;
  } else {
    bm = tt % tm;
    bn = tt / tm;
  }
  const int m0 = bm * T, n0 = bn * T;
  const int64_t kb0 = static_cast<int64_t>(split) * kchunk;
  const int64_t kend = min(K, kb0 + kchunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;

  TIN ra[LOADS][VEC], rb[LOADS][VEC];
  auto load = [&](int64_t kb) {
#pragma unroll
    for (int i = 0; i < LOADS; ++i) {
      const int l = tid + i * 256;
      const int c = l / PERCOL, kv = l % PERCOL;
      const int64_t k = kb + kv * VEC;
      const bool kin = k < kend;
      const bool ina = kin && m0 + c < M, inb = kin && n0 + c < N;
      using V = __attribute__((ext_vector_type(VEC))) TIN;
      V va{}, vb{};
      if (ina) va = *reinterpret_cast<const V*>(A + k + static_cast<int64_t>(m0 + c) * lda);
      if (inb) vb = *reinterpret_cast<const V*>(B + k + static_cast<int64_t>(n0 + c) * ldb);
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const bool ke = k + e < kend;
        ra[i][e] = (ina && ke) ? va[e] : TIN(0);
        rb[i][e] = (inb && ke) ? vb[e] : TIN(0);
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < LOADS; ++i) {
      const int l = tid + i * 256;
      const int c = l / PERCOL, kv = l % PERCOL;
      const int off = (MF == MF_BF) ? bf_off(c, kv * VEC) : c * ST + kv * VEC;
      big_put_row<MF, TIN, VEC>(xh, xl, off, ra[i]);
      big_put_row<MF, TIN, VEC>(yh, yl, off, rb[i]);
    }
  };

  typename Form<MF>::acc_t acc[NI][NI];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = typename Form<MF>::acc_t{};
  // The FP32 form (the polish projection) moves its MFMA sums into a
  // second FP32 accumulator every kFlushSteps k-blocks (128 k), so rounding
  // grows over 32 MFMA steps and then over the few hundred flushes of a K
  // split, instead of over thousands of steps in one accumulator.  (FP64
  // registers measured no more accurate at the Ritz level and cost
  // occupancy.)
  constexpr bool FLUSH = (MF == MF_F32);
  constexpr int kFlushSteps = 4;
  float accd[FLUSH ? NI : 1][FLUSH ? NI : 1][4] = {};
  int since_flush = 0;
  auto flush = [&]() {
    if constexpr (FLUSH) {
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) accd[i][j][r] += acc[i][j][r];
          acc[i][j] = typename Form<MF>::acc_t{};
        }
    }
  };
  (void)since_flush;

  load(kb0);
  for (int64_t kb = kb0; kb < kend; kb += BK) {
    __syncthreads();
    store();
    __syncthreads();
    if (kb + BK < kend) load(kb + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += FR::KS) {
      typename FR::t fa[NI], fb[NI];
#pragma unroll
      for (int i = 0; i < NI; ++i) fa[i] = FR::load(xh, xl, wr * WT + i * 16 + (lane & 15), ST, ks, lane);
#pragma unroll
      for (int j = 0; j < NI; ++j) fb[j] = FR::load(yh, yl, wc * WT + j * 16 + (lane & 15), ST, ks, lane);
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j) FR::mma(acc[i][j], fa[i], fb[j]);
    }
    if constexpr (FLUSH) {
      if (++since_flush == kFlushSteps) {
        flush();
        since_flush = 0;
      }
    }
  }
  if constexpr (FLUSH) flush();
  double* Ps = P + static_cast<int64_t>(split) * M * N;
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr * WT + i * 16 + Form<MF>::orow(lane, r);
        const int cl = n0 + wc * WT + j * 16 + (lane & 15);
        const double v = FLUSH ? static_cast<double>(accd[i][j][r]) : Form<MF>::get(acc[i][j], r);
        if (row < M && cl < N) Ps[row + static_cast<int64_t>(cl) * M] = v;
      }
}

// C[M x N] = A[M x K] B[K x N]: 64 rows x TN columns per workgroup (TN =
// 256 or 128), wave w owns columns (TN/4) w .. (TN/4)(w + 1) - 1.  The MFMA x
// operand is B (rows of the accumulator = columns of C), so each lane's
// results for one column are rows m .. m + 15 across lanes (coalesced
// stores).  TB is the B operand as stored: double (FP64), float (FP32) or
// bf16 hi/lo pairs (BF; Bh/Bl).  The 128-column tile pads an order such as
// 300 to 384 instead of 512 and is the default width.
template <typename TIN, typename TB, typename TOUT, int MF, int TN>
__global__ __launch_bounds__(256, 2) void gemm_nn_big_kernel(const TIN* __restrict__ A, int64_t lda,
                                                          const TB* __restrict__ Bh, const TB* __restrict__ Bl,
                                                          int64_t ldb, int M, int N, int K, int tnN,
                                                          TOUT* __restrict__ C, int64_t ldc) {
  using Lc = BigLds<MF>;
  using L = typename Lc::L;
  using FR = Frag<MF>;
  static_assert(TN == 256 || TN == 128, "large NN tiles are 256 or 128 columns");
  constexpr int TM = 64, BK = Lc::BK, ST = Lc::STRIDE;
  constexpr int WN = TN / 4, NJ = WN / 16;                // columns and 16-column blocks per wave
  constexpr int VA = 16 / sizeof(TIN);                    // A loads along m
  constexpr int ALOADS = TM * BK / VA / 256;
  constexpr int VB = 16 / sizeof(TB);                     // B loads along k
  static_assert((TN * BK / VB) % 256 == 0, "whole B loads per thread");
  constexpr int BLOADS = TN * BK / VB / 256;
  __shared__ __align__(16) L sm[Lc::PARTS * (TM + TN) * ST];
  L* ah = sm;
  L* bh = sm + TM * ST;
  L* al = (MF == MF_BF) ? sm + (TM + TN) * ST : nullptr;
  L* bl = (MF == MF_BF) ? sm + (TM + TN) * ST + TM * ST : nullptr;

  const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
  const int bn = static_cast<int>(lb % tnN), bm = static_cast<int>(lb / tnN);
  const int m0 = bm * TM, n0 = bn * TN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  using VAt = __attribute__((ext_vector_type(VA))) TIN;
  using VBt = __attribute__((ext_vector_type(VB))) TB;
  // The BF form gives each thread the same VA rows at two consecutive k, so
  // that its split stores (hi, lo) pairs of k values as 32-bit words.
  constexpr bool PAIRK = (MF == MF_BF) && ALOADS == 2;
  auto a_k = [&](int i) { return PAIRK ? 2 * (tid / (TM / VA)) + i : (tid + i * 256) / (TM / VA); };
  auto a_m = [&](int i) { return PAIRK ? (tid % (TM / VA)) * VA : ((tid + i * 256) % (TM / VA)) * VA; };
  VAt ra[ALOADS];
  VBt rbh[BLOADS], rbl[BLOADS];
  auto load = [&](int kb) {
#pragma unroll
    for (int i = 0; i < ALOADS; ++i) {
      const int k = a_k(i), mv = a_m(i);
      const bool ok = (kb + k < K) && (m0 + mv < M);
      ra[i] = ok ? *reinterpret_cast<const VAt*>(A + (m0 + mv) + static_cast<int64_t>(kb + k) * lda) : VAt{};
    }
#pragma unroll
    for (int i = 0; i < BLOADS; ++i) {
      const int l = tid + i * 256;
      const int n = l / (BK / VB), kv = (l % (BK / VB)) * VB;
      const bool ok = (n0 + n < N) && (kb + kv < K);
      const int64_t o = (kb + kv) + static_cast<int64_t>(n0 + n) * ldb;
      rbh[i] = ok ? *reinterpret_cast<const VBt*>(Bh + o) : VBt{};
      if constexpr (MF == MF_BF) rbl[i] = ok ? *reinterpret_cast<const VBt*>(Bl + o) : VBt{};
    }
  };
  auto store = [&](int kb) {
    if constexpr (PAIRK) {  // transpose: LDS rows are m, k contiguous
      const int k = a_k(0), mv = a_m(0);
      const int rot = (mv / VA) & (VA - 1);  // lanes write different rows mod 4 per store (bf_off)
#pragma unroll
      for (int e0 = 0; e0 < VA; ++e0) {
        const int e = (e0 + rot) & (VA - 1);
        float x0 = static_cast<float>(ra[0][0]), x1 = static_cast<float>(ra[1][0]);
#pragma unroll
        for (int q = 1; q < VA; ++q)
          if (e == q) {
            x0 = static_cast<float>(ra[0][q]);
            x1 = static_cast<float>(ra[1][q]);
          }
        const bool mi = m0 + mv + e < M;
        uint32_t hp, lp;
        split_pair(mi ? x0 : 0.0f, mi ? x1 : 0.0f, hp, lp);
        const int off = bf_off(mv + e, k);
        *reinterpret_cast<uint32_t*>(ah + off) = hp;
        *reinterpret_cast<uint32_t*>(al + off) = lp;
      }
    }
#pragma unroll
    for (int i = 0; i < (PAIRK ? 0 : ALOADS); ++i) {  // transpose: LDS rows are m, k contiguous
      const int k = a_k(i), mv = a_m(i);
#pragma unroll
      for (int e = 0; e < VA; ++e) {
        const TIN v = (m0 + mv + e < M) ? ra[i][e] : TIN(0);
        if constexpr (MF == MF_BF) {
          const float a = static_cast<float>(v);
          const uint16_t hb = bf16_rne_bits(a);
          ah[(mv + e) * ST + k] = hb;
          al[(mv + e) * ST + k] = bf16_rne_bits(a - bf16_bits_to_f32(hb));
        } else {
          ah[(mv + e) * ST + k] = static_cast<L>(v);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < BLOADS; ++i) {  // LDS rows are n, k contiguous
      const int l = tid + i * 256;
      const int n = l / (BK / VB), kv = (l % (BK / VB)) * VB;
      if constexpr (MF == MF_BF) {  // one 16-byte chunk per part
        VBt vh = rbh[i], vl = rbl[i];
#pragma unroll
        for (int e = 0; e < VB; ++e)
          if (kb + kv + e >= K) {
            vh[e] = 0;
            vl[e] = 0;
          }
        const int off = bf_off(n, kv);
        *reinterpret_cast<VBt*>(bh + off) = vh;
        *reinterpret_cast<VBt*>(bl + off) = vl;
      } else {
#pragma unroll
        for (int e = 0; e < VB; ++e) {
          const bool ke = kb + kv + e < K;
          bh[n * ST + kv + e] = ke ? static_cast<L>(rbh[i][e]) : L(0);
        }
      }
    }
  };

  typename Form<MF>::acc_t acc[NJ][4];
#pragma unroll
  for (int i = 0; i < NJ; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = typename Form<MF>::acc_t{};

  load(0);
  for (int kb = 0; kb < K; kb += BK) {
    __syncthreads();
    store(kb);
    __syncthreads();
    if (kb + BK < K) load(kb + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += FR::KS) {
      typename FR::t fb[NJ], fa[4];
#pragma unroll
      for (int i = 0; i < NJ; ++i) fb[i] = FR::load(bh, bl, wave * WN + i * 16 + (lane & 15), ST, ks, lane);
#pragma unroll
      for (int j = 0; j < 4; ++j) fa[j] = FR::load(ah, al, j * 16 + (lane & 15), ST, ks, lane);
#pragma unroll
      for (int i = 0; i < NJ; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) FR::mma(acc[i][j], fb[i], fa[j]);
    }
  }
#pragma unroll
  for (int i = 0; i < NJ; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = n0 + wave * WN + i * 16 + Form<MF>::orow(lane, r);
        const int m = m0 + j * 16 + (lane & 15);
        if (m < M && n < N) C[m + static_cast<int64_t>(n) * ldc] = static_cast<TOUT>(Form<MF>::get(acc[i][j], r));
      }
}

// The rotation matrix B (rows x cols, leading dimension lds) copied with a
// leading dimension ldd >= rows padded to the kernels' 16-byte k loads; the
// padding rows are zero.  FP64 copy, FP32 rounding, or bf16 hi/lo split.
__global__ void pad_f64_kernel(const double* __restrict__ s, int64_t lds, double* __restrict__ d, int64_t ldd,
                               int64_t rows, int64_t cols) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= ldd * cols) return;
  const int64_t r = i % ldd, c = i / ldd;
  d[i] = r < rows ? s[r + c * lds] : 0.0;
}
__global__ void pad_f32_kernel(const double* __restrict__ s, int64_t lds, float* __restrict__ d, int64_t ldd,
                               int64_t rows, int64_t cols) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= ldd * cols) return;
  const int64_t r = i % ldd, c = i / ldd;
  d[i] = r < rows ? static_cast<float>(s[r + c * lds]) : 0.0f;
}
__global__ void split_bf16_from_f64_kernel(const double* __restrict__ s, int64_t lds, uint16_t* __restrict__ hi,
                                           uint16_t* __restrict__ lo, int64_t ldd, int64_t rows, int64_t cols) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= ldd * cols) return;
  const int64_t r = i % ldd, c = i / ldd;
  const float a = r < rows ? static_cast<float>(s[r + c * lds]) : 0.0f;
  const uint16_t h = bf16_rne_bits(a);
  hi[i] = h;
  lo[i] = bf16_rne_bits(a - bf16_bits_to_f32(h));
}

constexpr int kTile = 64;

// compute units of the current device (cached per device)
int device_cus() {
  static std::atomic<int> cached[64];
  int dev = 0;
  XLS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) dev = 0;
  int c = cached[dev].load(std::memory_order_relaxed);
  if (c == 0) {
    XLS_HIP(hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev));
    c = std::max(1, c);
    cached[dev].store(c, std::memory_order_relaxed);
  }
  return c;
}

int planned_splits(int def, const GemmPlan& plan);

int choose_splits(int tiles, int64_t K, int bk, int M, int N, size_t work_elems, const GemmPlan& plan) {
  // aim for ~2048 workgroups; each split must keep >= 8 k-blocks
  int s = planned_splits(std::max(1, 2048 / std::max(1, tiles)), plan);
  const int64_t kblocks = (K + bk - 1) / bk;
  s = static_cast<int>(std::min<int64_t>(s, std::max<int64_t>(1, kblocks / 8)));
  const size_t per = static_cast<size_t>(M) * N;
  if (per > 0) s = static_cast<int>(std::min<size_t>(s, std::max<size_t>(1, work_elems / per)));
  return std::max(1, s);
}

template <typename T>
bool aligned16(const T* p) {
  return (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
}

// Split count of a plan: the default rule's count scaled by split_scale / 2.
int planned_splits(int def, const GemmPlan& plan) {
  return plan.split_scale > 0 ? std::max(1, def * plan.split_scale / 2) : def;
}

// Issued output area of the large TN kernel with tile edge T: every tile
// (on or above the block diagonal of a symmetric product) is computed whole.
int64_t tn_issued_area(int M, int N, int sym, int T) {
  const int64_t tm = (M + T - 1) / T, tn = (N + T - 1) / T;
  return (sym ? tm * (tm + 1) / 2 : tm * tn) * T * T;
}

// Large-tile edge: 96 where it issues at least 10 % less padded and
// redundant work than 128 (a forced edge through the plan otherwise).
int tn_tile_edge(int M, int N, int sym, const GemmPlan& plan) {
  if (plan.tile_tn == 2) return 128;
  if (plan.tile_tn == 3) return 96;
  return 10 * tn_issued_area(M, N, sym, 96) < 9 * tn_issued_area(M, N, sym, 128) ? 96 : 128;
}

template <typename TIN, int MF, int T>
void tn_big_launch(const TIN* A, int64_t lda, const TIN* B, int64_t ldb, int M, int N, int64_t K, double* C,
                   int64_t ldc, int sym, int symmetrize, double* work, size_t work_elems, hipStream_t st,
                   const GemmPlan& plan) {
  const int tm = (M + T - 1) / T, tn = (N + T - 1) / T;
  const int ntile = sym ? tm * (tm + 1) / 2 : tm * tn;
  const int bk = BigLds<MF>::BK;
  // about as many workgroups as are resident at once (2 per CU at edge 128,
  // 3 at edge 96: its smaller accumulator tile leaves room for a third; 1.5x
  // the splits measured 3-22 % faster there), so that symmetric products
  // (fewer tiles) get more splits; >= 16 K slabs each
  constexpr int kResident = (T == 96) ? 3 : 2;
  int splits = planned_splits(std::max(1, kResident * device_cus() / ntile), plan);
  splits = static_cast<int>(std::min<int64_t>(splits, std::max<int64_t>(1, K / (16 * bk))));
  const size_t per = static_cast<size_t>(M) * N;
  splits = static_cast<int>(std::min<size_t>(splits, std::max<size_t>(1, work_elems / per)));
  int64_t kchunk = (K + splits - 1) / splits;
  kchunk = ((kchunk + bk - 1) / bk) * bk;
  const int real_splits = static_cast<int>((K + kchunk - 1) / kchunk);
  const int64_t nb = static_cast<int64_t>(ntile) * real_splits;
  if (nb > 0x7fffffff) fail(XLS_ERR_INVALID_ARG, "gemm_tn grid too large");
  hipLaunchKernelGGL((gemm_tn_big_kernel<TIN, MF, T>), dim3(static_cast<unsigned>(nb)), dim3(256), 0, st, A,
                     lda, B, ldb, M, N, K, kchunk, tm, tn, sym, work);
  XLS_LAUNCH_CHECK("gemm_tn_big_kernel");
  launch_tn_reduce(work, real_splits, M, N, T, sym, symmetrize, C, ldc, st);
}

template <typename TIN, int MF>
void tn_dispatch(const TIN* A, int64_t lda, const TIN* B, int64_t ldb, int M, int N, int64_t K,
                 double* C, int64_t ldc, int sym, int symmetrize, double* work, size_t work_elems,
                 hipStream_t st, const GemmPlan& plan) {
  constexpr int VEC = 16 / sizeof(TIN);
  if (plan.tile_tn != 1 && M >= 64 && N >= 64 && lda % VEC == 0 && ldb % VEC == 0 && K <= lda && K <= ldb &&
      aligned16(A) && aligned16(B)) {
    // the 96 edge needs whole 16-byte loads per thread (not the FP64
    // products of FP32 blocks: 4 loads per 16-wide k slab and row)
    constexpr bool k96 = (96 * (BigLds<MF>::BK / VEC)) % 256 == 0;
    if constexpr (k96) {
      if (tn_tile_edge(M, N, sym, plan) == 96) {
        tn_big_launch<TIN, MF, 96>(A, lda, B, ldb, M, N, K, C, ldc, sym, symmetrize, work, work_elems, st, plan);
        return;
      }
    }
    tn_big_launch<TIN, MF, 128>(A, lda, B, ldb, M, N, K, C, ldc, sym, symmetrize, work, work_elems, st, plan);
    return;
  }
  const int tm = (M + kTile - 1) / kTile, tn = (N + kTile - 1) / kTile;
  const int ntile = sym ? tm * (tm + 1) / 2 : tm * tn;
  const int bk = Form<MF>::BK;
  const int splits = choose_splits(ntile, K, bk, M, N, work_elems, plan);
  int64_t kchunk = (K + splits - 1) / splits;
  kchunk = ((kchunk + bk - 1) / bk) * bk;
  const int real_splits = static_cast<int>((K + kchunk - 1) / kchunk);
  const int64_t nb = static_cast<int64_t>(ntile) * real_splits;
  if (nb > 0x7fffffff) fail(XLS_ERR_INVALID_ARG, "gemm_tn grid too large");
  hipLaunchKernelGGL((gemm_tn_kernel<TIN, MF, kTile>), dim3(static_cast<unsigned>(nb)), dim3(256), 0,
                     st, A, lda, B, ldb, M, N, K, kchunk, tm, tn, sym, work);
  XLS_LAUNCH_CHECK("gemm_tn_kernel");
  launch_tn_reduce(work, real_splits, M, N, kTile, sym, symmetrize, C, ldc, st);
}

}  // namespace

size_t nn_work_doubles(int K, int N) {
  return static_cast<size_t>((static_cast<int64_t>(K) + 7) / 8 * 8) * static_cast<size_t>(N);
}

size_t gemm_tn_work_elems(int M, int N, int64_t K) {
  // room for every split either kernel takes (each split keeps >= 8 k-blocks
  // of >= 16, so at most K/128 of them; at most 64), capped at 32 Mi doubles
  // (256 MB)
  const size_t per = static_cast<size_t>(M) * N;
  const size_t splits = static_cast<size_t>(std::min<int64_t>(64, std::max<int64_t>(1, K / 128)));
  return std::max<size_t>(per, std::min<size_t>(splits * per, static_cast<size_t>(32) << 20));
}

template <typename TS>
void gemm_tn(int prec, const TS* A, int64_t lda, const TS* B, int64_t ldb, int M, int N, int64_t K,
             double* C, int64_t ldc, int sym, int symmetrize, double* work, size_t work_elems,
             hipStream_t st, const GemmPlan& plan) {
  if (M <= 0 || N <= 0) return;
  if (work_elems < static_cast<size_t>(M) * N) fail(XLS_ERR_INVALID_ARG, "gemm_tn workspace too small");
  if constexpr (std::is_same<TS, double>::value) {
    if (prec != MF_F64) fail(XLS_ERR_INVALID_ARG, "FP64 blocks use FP64 GEMMs");
    tn_dispatch<double, MF_F64>(A, lda, B, ldb, M, N, K, C, ldc, sym, symmetrize, work, work_elems, st, plan);
  } else {
    if (prec == MF_F64)
      tn_dispatch<float, MF_F64>(A, lda, B, ldb, M, N, K, C, ldc, sym, symmetrize, work, work_elems, st, plan);
    else if (prec == MF_F32)
      tn_dispatch<float, MF_F32>(A, lda, B, ldb, M, N, K, C, ldc, sym, symmetrize, work, work_elems, st, plan);
    else if (prec == MF_BF)
      tn_dispatch<float, MF_BF>(A, lda, B, ldb, M, N, K, C, ldc, sym, symmetrize, work, work_elems, st, plan);
    else
      fail(XLS_ERR_INVALID_ARG, "unknown GEMM precision");
  }
}

// Column width of the large rotation tile: 128 unless the plan forces 256.
// The 128 tile pads N no more than 256 does, and where both pad alike
// (N = 480) it still measured 2-5 % faster in every precision: half the
// accumulators per wave leave room for more resident waves.
int nn_tile_cols(const GemmPlan& plan) { return plan.tile_nn == 2 ? 256 : 128; }

// Large-tile rotation with TN-column tiles; false when the shapes or
// alignment do not allow it.
template <typename TS, int TN>
bool nn_big_t(int prec, const TS* A, int64_t lda, const double* B, int64_t ldb, int M, int N, int K, TS* C,
              int64_t ldc, void* bwork, hipStream_t st) {
  constexpr int VA = 16 / sizeof(TS);
  if (M < 64 || N < 64 || lda % VA != 0 || !aligned16(A) || M > lda || K > ldb) return false;
  const bool have_work = bwork != nullptr && aligned16(bwork);
  const int tnN = (N + TN - 1) / TN;
  const int64_t nb = static_cast<int64_t>((M + 63) / 64) * tnN;
  if (nb > 0x7fffffff) return false;
  const dim3 grid(static_cast<unsigned>(nb));
  // B goes through bwork with its leading dimension padded to 8 rows
  // (bwork holds nn_work_elems(K, N) doubles)
  const int64_t ldp = (static_cast<int64_t>(K) + 7) / 8 * 8;
  const int64_t nbv = ldp * static_cast<int64_t>(N);
  const unsigned pgrid = static_cast<unsigned>((nbv + 255) / 256);
  if (prec == MF_F64) {
    const double* Bd = B;
    int64_t ldbd = ldb;
    if (ldb % 2 != 0 || !aligned16(B)) {
      if (!have_work) return false;
      double* Bp = static_cast<double*>(bwork);
      hipLaunchKernelGGL(pad_f64_kernel, dim3(pgrid), dim3(256), 0, st, B, ldb, Bp, ldp, K, N);
      Bd = Bp;
      ldbd = ldp;
    }
    hipLaunchKernelGGL((gemm_nn_big_kernel<TS, double, TS, MF_F64, TN>), grid, dim3(256), 0, st, A, lda, Bd,
                       static_cast<const double*>(nullptr), ldbd, M, N, K, tnN, C, ldc);
  } else if constexpr (std::is_same<TS, float>::value) {
    if (!have_work) return false;
    if (prec == MF_F32) {
      float* Bf = static_cast<float*>(bwork);
      hipLaunchKernelGGL(pad_f32_kernel, dim3(pgrid), dim3(256), 0, st, B, ldb, Bf, ldp, K, N);
      hipLaunchKernelGGL((gemm_nn_big_kernel<float, float, float, MF_F32, TN>), grid, dim3(256), 0, st, A, lda, Bf,
                         static_cast<const float*>(nullptr), ldp, M, N, K, tnN, C, ldc);
    } else if (prec == MF_BF) {
      // the rotation matrix is split into bf16 hi/lo once (same bytes as its FP32 copy)
      uint16_t* bh = static_cast<uint16_t*>(bwork);
      uint16_t* bl = bh + nbv;
      hipLaunchKernelGGL(split_bf16_from_f64_kernel, dim3(pgrid), dim3(256), 0, st, B, ldb, bh, bl, ldp, K, N);
      hipLaunchKernelGGL((gemm_nn_big_kernel<float, uint16_t, float, MF_BF, TN>), grid, dim3(256), 0, st, A, lda, bh, bl,
                         ldp, M, N, K, tnN, C, ldc);
    } else {
      return false;
    }
  } else {
    return false;
  }
  XLS_LAUNCH_CHECK("gemm_nn_big_kernel");
  return true;
}

template <typename TS>
bool nn_big(int prec, const TS* A, int64_t lda, const double* B, int64_t ldb, int M, int N, int K, TS* C,
            int64_t ldc, void* bwork, hipStream_t st, const GemmPlan& plan) {
  if (nn_tile_cols(plan) == 128)
    return nn_big_t<TS, 128>(prec, A, lda, B, ldb, M, N, K, C, ldc, bwork, st);
  return nn_big_t<TS, 256>(prec, A, lda, B, ldb, M, N, K, C, ldc, bwork, st);
}

template <typename TS>
void gemm_nn(int prec, const TS* A, int64_t lda, const double* B, int64_t ldb, int M, int N, int K,
             TS* C, int64_t ldc, void* bwork, hipStream_t st, const GemmPlan& plan) {
  if (M <= 0 || N <= 0) return;
  if (plan.tile_nn != 1 && nn_big<TS>(prec, A, lda, B, ldb, M, N, K, C, ldc, bwork, st, plan)) return;
  const int tmM = (M + kTile - 1) / kTile, tnN = (N + kTile - 1) / kTile;
  const int64_t nb = static_cast<int64_t>(tmM) * tnN;
  if (nb > 0x7fffffff) fail(XLS_ERR_INVALID_ARG, "gemm_nn grid too large");
  const dim3 grid(static_cast<unsigned>(nb));
  if constexpr (std::is_same<TS, double>::value) {
    if (prec != MF_F64) fail(XLS_ERR_INVALID_ARG, "FP64 blocks use FP64 GEMMs");
    hipLaunchKernelGGL((gemm_nn_kernel<double, double, double, MF_F64, kTile>), grid, dim3(256), 0, st,
                       A, lda, B, ldb, M, N, K, tmM, tnN, C, ldc);
  } else {
    if (prec == MF_F64) {
      hipLaunchKernelGGL((gemm_nn_kernel<float, double, float, MF_F64, kTile>), grid, dim3(256), 0, st,
                         A, lda, B, ldb, M, N, K, tmM, tnN, C, ldc);
    } else {
      // the rotation matrix is rounded to FP32 once, then fed like the block
      float* Bf = static_cast<float*>(bwork);
      const int64_t nbv = ldb * static_cast<int64_t>(N);
      hipLaunchKernelGGL(d2f_kernel, dim3(static_cast<unsigned>((nbv + 255) / 256)), dim3(256), 0, st, B, Bf,
                         nbv);
      if (prec == MF_F32)
        hipLaunchKernelGGL((gemm_nn_kernel<float, float, float, MF_F32, kTile>), grid, dim3(256), 0, st,
                           A, lda, Bf, ldb, M, N, K, tmM, tnN, C, ldc);
      else if (prec == MF_BF)
        hipLaunchKernelGGL((gemm_nn_kernel<float, float, float, MF_BF, kTile>), grid, dim3(256), 0, st,
                           A, lda, Bf, ldb, M, N, K, tmM, tnN, C, ldc);
      else
        fail(XLS_ERR_INVALID_ARG, "unknown GEMM precision");
    }
  }
  XLS_LAUNCH_CHECK("gemm_nn_kernel");
}

void split_bf16_device(const float* a, uint16_t* hi, uint16_t* lo, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(split_bf16_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st,
                     a, hi, lo, n);
  XLS_LAUNCH_CHECK("split_bf16_kernel");
}

template void gemm_tn<double>(int, const double*, int64_t, const double*, int64_t, int, int, int64_t,
                              double*, int64_t, int, int, double*, size_t, hipStream_t, const GemmPlan&);
template void gemm_tn<float>(int, const float*, int64_t, const float*, int64_t, int, int, int64_t,
                             double*, int64_t, int, int, double*, size_t, hipStream_t, const GemmPlan&);
template void gemm_nn<double>(int, const double*, int64_t, const double*, int64_t, int, int, int,
                              double*, int64_t, void*, hipStream_t, const GemmPlan&);
template void gemm_nn<float>(int, const float*, int64_t, const double*, int64_t, int, int, int, float*,
                             int64_t, void*, hipStream_t, const GemmPlan&);

}  // namespace xls
