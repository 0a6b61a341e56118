// Electrostatic Poisson solve (Sec. IV Poisson equation; Sec. V-B.1
// structured-multigrid-preconditioned CG): A phi = 4 pi f with A = -L the
// 12th-order FD Laplacian (zero Dirichlet or periodic), CG in FP64,
// preconditioned by one FP32 V-cycle whose finest level is the 7-point
// Laplacian applied matrix-free and whose coarse levels are the Galerkin
// operators P^T A P of trilinear prolongation.  On a uniform grid with exact
// coarsening those are one 27-point stencil per level, computed once on the
// host from the fine stencil; every level is applied matrix-free.
//
// Coarsening: zero Dirichlet n -> (n - 1)/2 (coarse point I on fine 2I + 1),
// periodic n -> n/2 (coarse I on fine 2I), while every axis coarsens exactly
// to at least 3 (4) points.  Smoothing: damped Jacobi (omega = 2/3), nu
// sweeps before and after the coarse correction, nu_c sweeps from zero on the
// coarsest level; zero start makes the V-cycle symmetric.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "xls_handle.h"

using namespace xls;

namespace {

constexpr int R12 = 6;  // half-width of the 12th-order Laplacian
constexpr float kOmega = 2.0f / 3.0f;
constexpr int kNu = 2, kNuCoarse = 10;

inline unsigned nblk(int64_t n, int b) { return static_cast<unsigned>((n + b - 1) / b); }

struct Grid {
  int nx, ny, nz;
  int periodic;
};

__device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// out = A u = -L u, L the 12th-order Laplacian (weights w[0..6] already
// scaled by 1/h^2), FP64; one thread per point.
struct W12 {
  double w[R12 + 1];
};
__global__ void lap12_kernel(const double* __restrict__ u, double* __restrict__ out, Grid g, W12 w) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nd = static_cast<int64_t>(g.nx) * g.ny * g.nz;
  if (p >= nd) return;
  const int i = static_cast<int>(p % g.nx), j = static_cast<int>((p / g.nx) % g.ny),
            k = static_cast<int>(p / (static_cast<int64_t>(g.nx) * g.ny));
  auto at = [&](int a, int b, int c) -> double {
    if (g.periodic) {
      a = wrap(a, g.nx);
      b = wrap(b, g.ny);
      c = wrap(c, g.nz);
    } else if (a < 0 || a >= g.nx || b < 0 || b >= g.ny || c < 0 || c >= g.nz) {
      return 0.0;
    }
    return u[a + static_cast<int64_t>(g.nx) * (b + static_cast<int64_t>(g.ny) * c)];
  };
  double s = 3.0 * w.w[0] * u[p];
  for (int q = 1; q <= R12; ++q)
    s += w.w[q] * ((at(i + q, j, k) + at(i - q, j, k)) + (at(i, j + q, k) + at(i, j - q, k)) +
                   (at(i, j, k + q) + at(i, j, k - q)));
  out[p] = -s;
}

// Constant 27-point stencil c[(dz+1)*9 + (dy+1)*3 + (dx+1)] (the 7-point
// finest operator is the same form with zeros), FP32.
struct S27 {
  float c[27];
};

__device__ __forceinline__ float apply27(const float* __restrict__ x, const Grid& g, int i, int j, int k,
                                         const S27& s, bool seven) {
  float acc = 0.0f;
  auto at = [&](int a, int b, int c) -> float {
    if (g.periodic) {
      a = wrap(a, g.nx);
      b = wrap(b, g.ny);
      c = wrap(c, g.nz);
    } else if (a < 0 || a >= g.nx || b < 0 || b >= g.ny || c < 0 || c >= g.nz) {
      return 0.0f;
    }
    return x[a + static_cast<int64_t>(g.nx) * (b + static_cast<int64_t>(g.ny) * c)];
  };
  if (seven) {
    acc = s.c[13] * at(i, j, k);
    acc += s.c[12] * at(i - 1, j, k) + s.c[14] * at(i + 1, j, k);
    acc += s.c[10] * at(i, j - 1, k) + s.c[16] * at(i, j + 1, k);
    acc += s.c[4] * at(i, j, k - 1) + s.c[22] * at(i, j, k + 1);
    return acc;
  }
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) acc += s.c[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] * at(i + dx, j + dy, k + dz);
  return acc;
}

// Damped Jacobi sweep xo = x + omega (r - A x) / c_0 (x may be null: zero start).
__global__ void jacobi_kernel(const float* __restrict__ x, const float* __restrict__ r, float* __restrict__ xo,
                              Grid g, S27 s, int seven) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nd = static_cast<int64_t>(g.nx) * g.ny * g.nz;
  if (p >= nd) return;
  const float ax = x ? apply27(x, g, static_cast<int>(p % g.nx), static_cast<int>((p / g.nx) % g.ny),
                               static_cast<int>(p / (static_cast<int64_t>(g.nx) * g.ny)), s, seven != 0)
                     : 0.0f;
  const float xv = x ? x[p] : 0.0f;
  xo[p] = xv + kOmega * (r[p] - ax) / s.c[13];
}

// t = r - A x
__global__ void resid_kernel(const float* __restrict__ x, const float* __restrict__ r, float* __restrict__ t,
                             Grid g, S27 s, int seven) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nd = static_cast<int64_t>(g.nx) * g.ny * g.nz;
  if (p >= nd) return;
  t[p] = r[p] - apply27(x, g, static_cast<int>(p % g.nx), static_cast<int>((p / g.nx) % g.ny),
                        static_cast<int>(p / (static_cast<int64_t>(g.nx) * g.ny)), s, seven != 0);
}

// Fine index of coarse index I along an axis, and the 1-D trilinear weight of
// fine offset d in {-1, 0, 1}.
__device__ __forceinline__ int fine_of(int I, int periodic) { return periodic ? 2 * I : 2 * I + 1; }
__device__ __forceinline__ float pw(int d) { return d == 0 ? 1.0f : 0.5f; }

// rc[I] = sum over the 27 fine neighbours f of fine(I) of P(f, I) t[f]
// (restriction P^T), in a fixed order.
__global__ void restrict_kernel(const float* __restrict__ t, Grid gf, float* __restrict__ rc, Grid gc) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nc = static_cast<int64_t>(gc.nx) * gc.ny * gc.nz;
  if (p >= nc) return;
  const int I = static_cast<int>(p % gc.nx), J = static_cast<int>((p / gc.nx) % gc.ny),
            K = static_cast<int>(p / (static_cast<int64_t>(gc.nx) * gc.ny));
  const int fi = fine_of(I, gf.periodic), fj = fine_of(J, gf.periodic), fk = fine_of(K, gf.periodic);
  float acc = 0.0f;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int a = fi + dx, b = fj + dy, c = fk + dz;
        if (gf.periodic) {
          a = wrap(a, gf.nx);
          b = wrap(b, gf.ny);
          c = wrap(c, gf.nz);
        } else if (a < 0 || a >= gf.nx || b < 0 || b >= gf.ny || c < 0 || c >= gf.nz) {
          continue;
        }
        acc += pw(dx) * pw(dy) * pw(dz) * t[a + static_cast<int64_t>(gf.nx) * (b + static_cast<int64_t>(gf.ny) * c)];
      }
  rc[p] = acc;
}

// 1-D coarse neighbours of fine index i: up to two (index, weight) pairs.
__device__ __forceinline__ int coarse_of(int i, int m, int periodic, int* idx, float* w) {
  if (periodic) {
    if ((i & 1) == 0) {
      idx[0] = i / 2;
      w[0] = 1.0f;
      return 1;
    }
    idx[0] = (i - 1) / 2;
    idx[1] = wrap((i + 1) / 2, m);
    w[0] = w[1] = 0.5f;
    return 2;
  }
  if (i & 1) {
    idx[0] = (i - 1) / 2;
    w[0] = 1.0f;
    return 1;
  }
  int k = 0;
  if (i / 2 - 1 >= 0) {
    idx[k] = i / 2 - 1;
    w[k++] = 0.5f;
  }
  if (i / 2 < m) {
    idx[k] = i / 2;
    w[k++] = 0.5f;
  }
  return k;
}

// xf[f] += sum_I P(f, I) xc[I] (prolongation), fixed order.
__global__ void prolong_kernel(const float* __restrict__ xc, Grid gc, float* __restrict__ xf, Grid gf) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nf = static_cast<int64_t>(gf.nx) * gf.ny * gf.nz;
  if (p >= nf) return;
  const int i = static_cast<int>(p % gf.nx), j = static_cast<int>((p / gf.nx) % gf.ny),
            k = static_cast<int>(p / (static_cast<int64_t>(gf.nx) * gf.ny));
  int ia[2], ja[2], ka[2];
  float wi[2], wj[2], wk[2];
  const int ni = coarse_of(i, gc.nx, gf.periodic, ia, wi), nj = coarse_of(j, gc.ny, gf.periodic, ja, wj),
            nk = coarse_of(k, gc.nz, gf.periodic, ka, wk);
  float acc = 0.0f;
  for (int c = 0; c < nk; ++c)
    for (int b = 0; b < nj; ++b)
      for (int a = 0; a < ni; ++a)
        acc += wi[a] * wj[b] * wk[c] *
               xc[ia[a] + static_cast<int64_t>(gc.nx) * (ja[b] + static_cast<int64_t>(gc.ny) * ka[c])];
  xf[p] += acc;
}

__global__ void to_f32_kernel(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < n) b[p] = static_cast<float>(a[p]);
}
__global__ void to_f64_kernel(const float* __restrict__ a, double* __restrict__ b, int64_t n) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < n) b[p] = static_cast<double>(a[p]);
}

// Partial sums of x.y per block (256 threads, strided loop, fixed tree).
constexpr int kDotBlocks = 512;
__global__ __launch_bounds__(256) void dot_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                                  int64_t n, double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; p < n; p += 256 * kDotBlocks)
    s += (y ? x[p] * y[p] : x[p]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ __launch_bounds__(256) void sum_parts_kernel(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < kDotBlocks; b += 256) s += part[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// y = a x + b y (a, b from device scalars: a = num[0]/den[0] * sa)
__global__ void axpby_kernel(const double* __restrict__ x, double* __restrict__ y, int64_t n, double a, double b) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < n) y[p] = a * x[p] + b * y[p];
}
__global__ void add_const_kernel(double* __restrict__ y, int64_t n, const double* __restrict__ sum, double scale) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < n) y[p] -= (*sum) * scale;
}

void check(const char* what) { XLS_LAUNCH_CHECK(what); }

int coarse_size(int m, bool periodic) {
  if (periodic) return (m % 2 == 0 && m / 2 >= 4) ? m / 2 : -1;
  return (m % 2 == 1 && (m - 1) / 2 >= 3) ? (m - 1) / 2 : -1;
}

// Galerkin stencil P^T A P of a constant 27-point stencil a with trilinear P:
// c(J) = sum_{u, v} p(u) a(v) p(u + v - 2 J), offsets in {-1, 0, 1}^3.
std::array<double, 27> galerkin(const std::array<double, 27>& a) {
  auto p1 = [](int d) { return d == 0 ? 1.0 : (d == -1 || d == 1 ? 0.5 : 0.0); };
  std::array<double, 27> c{};
  for (int J = 0; J < 27; ++J) {
    const int jx = J % 3 - 1, jy = (J / 3) % 3 - 1, jz = J / 9 - 1;
    double s = 0.0;
    for (int U = 0; U < 27; ++U) {
      const int ux = U % 3 - 1, uy = (U / 3) % 3 - 1, uz = U / 9 - 1;
      for (int V = 0; V < 27; ++V) {
        if (a[V] == 0.0) continue;
        const int vx = V % 3 - 1, vy = (V / 3) % 3 - 1, vz = V / 9 - 1;
        const int wx = ux + vx - 2 * jx, wy = uy + vy - 2 * jy, wz = uz + vz - 2 * jz;
        const double pu = p1(ux) * p1(uy) * p1(uz), pwv = p1(wx) * p1(wy) * p1(wz);
        s += pu * a[V] * pwv;
      }
    }
    c[J] = s;
  }
  return c;
}

}  // namespace

struct xls_poisson_s {
  Grid g{};
  double h = 0.0;
  int64_t nd = 0;
  std::vector<Grid> lev;
  std::vector<S27> st;
  std::vector<float*> xl, rl, tl;  // per level: solution, right-hand side, work
  double *b = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *Ap = nullptr, *part = nullptr,
         *sc = nullptr;
  hipStream_t s = nullptr;
  W12 w12{};
  ~xls_poisson_s() {
    if (s) (void)hipStreamSynchronize(s);
    for (auto* q : xl) dfree(q);
    for (auto* q : rl) dfree(q);
    for (auto* q : tl) dfree(q);
    void* ps[] = {b, x, r, z, p, Ap, part, sc};
    for (void* q : ps) dfree(q);
    if (s) (void)hipStreamDestroy(s);
  }
  int64_t size(int l) const { return static_cast<int64_t>(lev[l].nx) * lev[l].ny * lev[l].nz; }
};

namespace {

double dot(xls_poisson_s* P, const double* a, const double* b_) {
  hipLaunchKernelGGL(dot_kernel, dim3(kDotBlocks), dim3(256), 0, P->s, a, b_, P->nd, P->part);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(256), 0, P->s, P->part, P->sc);
  check("dot");
  double h = 0.0;
  XLS_HIP(hipMemcpyAsync(&h, P->sc, 8, hipMemcpyDeviceToHost, P->s));
  XLS_HIP(hipStreamSynchronize(P->s));
  return h;
}

// y -= mean(y) (periodic null space), on the device
void remove_mean(xls_poisson_s* P, double* y) {
  hipLaunchKernelGGL(dot_kernel, dim3(kDotBlocks), dim3(256), 0, P->s, y, nullptr, P->nd, P->part);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(256), 0, P->s, P->part, P->sc);
  hipLaunchKernelGGL(add_const_kernel, dim3(nblk(P->nd, 256)), dim3(256), 0, P->s, y, P->nd, P->sc,
                     1.0 / static_cast<double>(P->nd));
  check("remove_mean");
}

void vcycle(xls_poisson_s* P, int l) {
  const int L = static_cast<int>(P->lev.size());
  const Grid& g = P->lev[l];
  const S27& s = P->st[l];
  const int seven = l == 0 ? 1 : 0;
  const int64_t n = P->size(l);
  const dim3 gr(nblk(n, 256)), bl(256);
  float *x = P->xl[l], *r = P->rl[l], *t = P->tl[l];
  const int nu = l == L - 1 ? kNuCoarse : kNu;
  // pre-smoothing from zero (ping-pong between x and t)
  hipLaunchKernelGGL(jacobi_kernel, gr, bl, 0, P->s, static_cast<const float*>(nullptr), r, x, g, s, seven);
  for (int k = 1; k < nu; ++k) {
    hipLaunchKernelGGL(jacobi_kernel, gr, bl, 0, P->s, x, r, t, g, s, seven);
    std::swap(x, t);
  }
  if (l < L - 1) {
    hipLaunchKernelGGL(resid_kernel, gr, bl, 0, P->s, x, r, t, g, s, seven);
    hipLaunchKernelGGL(restrict_kernel, dim3(nblk(P->size(l + 1), 256)), bl, 0, P->s, t, g, P->rl[l + 1],
                       P->lev[l + 1]);
    vcycle(P, l + 1);
    hipLaunchKernelGGL(prolong_kernel, gr, bl, 0, P->s, P->xl[l + 1], P->lev[l + 1], x, g);
    for (int k = 0; k < kNu; ++k) {
      hipLaunchKernelGGL(jacobi_kernel, gr, bl, 0, P->s, x, r, t, g, s, seven);
      std::swap(x, t);
    }
  }
  if (x != P->xl[l]) XLS_HIP(hipMemcpyAsync(P->xl[l], x, n * 4, hipMemcpyDeviceToDevice, P->s));
  check("vcycle");
}

// z = B r: FP32 V-cycle of the FP64 vector r (mean removed when periodic)
void precondition(xls_poisson_s* P, const double* r, double* z) {
  hipLaunchKernelGGL(to_f32_kernel, dim3(nblk(P->nd, 256)), dim3(256), 0, P->s, r, P->rl[0], P->nd);
  vcycle(P, 0);
  hipLaunchKernelGGL(to_f64_kernel, dim3(nblk(P->nd, 256)), dim3(256), 0, P->s, P->xl[0], z, P->nd);
  check("precondition");
  if (P->g.periodic) remove_mean(P, z);
}

void apply_A(xls_poisson_s* P, const double* u, double* out) {
  hipLaunchKernelGGL(lap12_kernel, dim3(nblk(P->nd, 256)), dim3(256), 0, P->s, u, out, P->g, P->w12);
  check("lap12_kernel");
}

void axpby(xls_poisson_s* P, const double* x, double* y, double a, double b) {
  hipLaunchKernelGGL(axpby_kernel, dim3(nblk(P->nd, 256)), dim3(256), 0, P->s, x, y, P->nd, a, b);
  check("axpby_kernel");
}

}  // namespace

extern "C" {

int xls_poisson_create(const int32_t* n, double h, int32_t bc, int32_t max_levels, xls_poisson_t* out) {
  return guarded([&]() -> int {
    if (!out || !n) fail(XLS_ERR_INVALID_ARG, "NULL argument");
    for (int a = 0; a < 3; ++a)
      if (n[a] < 1) fail(XLS_ERR_INVALID_ARG, "grid size must be >= 1");
    if (!(h > 0) || !std::isfinite(h)) fail(XLS_ERR_INVALID_ARG, "h must be finite and > 0");
    if (bc != XLS_BC_PERIODIC && bc != XLS_BC_DIRICHLET0) fail(XLS_ERR_INVALID_ARG, "unknown bc");
    if (max_levels < 0 || max_levels > 16) fail(XLS_ERR_INVALID_ARG, "max_levels must be in [0, 16]");
    const int64_t nd = static_cast<int64_t>(n[0]) * n[1] * n[2];
    if (nd >= (int64_t(1) << 31)) fail(XLS_ERR_INVALID_ARG, "grid too large");
    auto* P = new xls_poisson_s();
    try {
      P->g = Grid{n[0], n[1], n[2], bc == XLS_BC_PERIODIC ? 1 : 0};
      P->h = h;
      P->nd = nd;
      XLS_HIP(hipStreamCreateWithFlags(&P->s, hipStreamNonBlocking));
      // 12th-order weights scaled by 1/h^2
      double f[2 * R12 + 1];
      f[0] = 1.0;
      for (int i = 1; i <= 2 * R12; ++i) f[i] = f[i - 1] * i;
      double sw = 0.0;
      for (int q = 1; q <= R12; ++q) {
        P->w12.w[q] = 2.0 * ((q % 2 == 1) ? 1.0 : -1.0) * f[R12] * f[R12] /
                      (static_cast<double>(q) * q * f[R12 - q] * f[R12 + q]) / (h * h);
        sw += P->w12.w[q];
      }
      P->w12.w[0] = -2.0 * sw;
      // levels and their constant stencils
      std::array<double, 27> a{};
      a[13] = 6.0 / (h * h);
      a[12] = a[14] = a[10] = a[16] = a[4] = a[22] = -1.0 / (h * h);
      const int maxl = max_levels > 0 ? max_levels : 8;
      P->lev.push_back(P->g);
      for (;;) {
        S27 s;
        for (int k = 0; k < 27; ++k) s.c[k] = static_cast<float>(a[k]);
        P->st.push_back(s);
        if (static_cast<int>(P->lev.size()) >= maxl) break;
        const Grid& g = P->lev.back();
        const int cx = coarse_size(g.nx, g.periodic), cy = coarse_size(g.ny, g.periodic),
                  cz = coarse_size(g.nz, g.periodic);
        if (cx < 0 || cy < 0 || cz < 0) break;
        P->lev.push_back(Grid{cx, cy, cz, g.periodic});
        a = galerkin(a);
      }
      for (size_t l = 0; l < P->lev.size(); ++l) {
        const size_t m = static_cast<size_t>(P->size(static_cast<int>(l)));
        P->xl.push_back(dalloc<float>(m));
        P->rl.push_back(dalloc<float>(m));
        P->tl.push_back(dalloc<float>(m));
      }
      double** vs[] = {&P->b, &P->x, &P->r, &P->z, &P->p, &P->Ap};
      for (double** v : vs) *v = dalloc<double>(nd);
      P->part = dalloc<double>(kDotBlocks);
      P->sc = dalloc<double>(8);
    } catch (...) {
      delete P;
      throw;
    }
    *out = P;
    return XLS_OK;
  });
}

void xls_poisson_destroy(xls_poisson_t P) { delete P; }

int xls_poisson_vcycle(xls_poisson_t P, const double* r, double* z) {
  return guarded([&]() -> int {
    if (!P || !r || !z) fail(XLS_ERR_INVALID_ARG, "NULL argument");
    if (!finite_all(r, P->nd)) fail(XLS_ERR_INVALID_ARG, "r not finite");
    XLS_HIP(hipMemcpyAsync(P->r, r, P->nd * 8, hipMemcpyHostToDevice, P->s));
    hipLaunchKernelGGL(to_f32_kernel, dim3(nblk(P->nd, 256)), dim3(256), 0, P->s, P->r, P->rl[0], P->nd);
    vcycle(P, 0);
    hipLaunchKernelGGL(to_f64_kernel, dim3(nblk(P->nd, 256)), dim3(256), 0, P->s, P->xl[0], P->z, P->nd);
    check("xls_poisson_vcycle");
    XLS_HIP(hipMemcpyAsync(z, P->z, P->nd * 8, hipMemcpyDeviceToHost, P->s));
    XLS_HIP(hipStreamSynchronize(P->s));
    return XLS_OK;
  });
}

}  // extern "C"

namespace {

// CG on the handle's device vectors: P->b holds f on entry; the solution is
// left in P->x.  info as xls_poisson_solve (wall ms from t0).
void solve_on_device(xls_poisson_t P, double tol, int32_t max_iter, int32_t precond, double* info,
                     std::chrono::steady_clock::time_point t0) {
    const int64_t nd = P->nd;
    axpby(P, P->b, P->b, 0.0, 4.0 * M_PI);  // b = 4 pi f
    if (P->g.periodic) remove_mean(P, P->b);
    XLS_HIP(hipMemsetAsync(P->x, 0, nd * 8, P->s));
    XLS_HIP(hipMemcpyAsync(P->r, P->b, nd * 8, hipMemcpyDeviceToDevice, P->s));
    const double nb = std::sqrt(dot(P, P->b, P->b));
    int it = 0;
    double rel = 0.0;
    if (nb > 0.0) {
      if (precond)
        precondition(P, P->r, P->z);
      else
        XLS_HIP(hipMemcpyAsync(P->z, P->r, nd * 8, hipMemcpyDeviceToDevice, P->s));
      XLS_HIP(hipMemcpyAsync(P->p, P->z, nd * 8, hipMemcpyDeviceToDevice, P->s));
      double rz = dot(P, P->r, P->z);
      rel = 1.0;
      for (it = 1; it <= max_iter; ++it) {
        apply_A(P, P->p, P->Ap);
        const double alpha = rz / dot(P, P->p, P->Ap);
        axpby(P, P->p, P->x, alpha, 1.0);
        axpby(P, P->Ap, P->r, -alpha, 1.0);
        rel = std::sqrt(dot(P, P->r, P->r)) / nb;
        if (!(rel > tol)) break;  // NaN ends the loop too
        if (precond)
          precondition(P, P->r, P->z);
        else
          XLS_HIP(hipMemcpyAsync(P->z, P->r, nd * 8, hipMemcpyDeviceToDevice, P->s));
        const double rz_new = dot(P, P->r, P->z);
        axpby(P, P->z, P->p, 1.0, rz_new / rz);
        rz = rz_new;
      }
      if (it > max_iter) it = max_iter;
      if (P->g.periodic) remove_mean(P, P->x);
    }
    XLS_HIP(hipStreamSynchronize(P->s));
    if (info) {
      info[0] = it;
      info[1] = rel;
      info[2] = static_cast<double>(P->lev.size());
      info[3] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
}

void check_solve_args(xls_poisson_t P, const void* f, const void* phi, double tol, int32_t max_iter) {
  if (!P || !f || !phi) fail(XLS_ERR_INVALID_ARG, "NULL argument");
  if (!(tol > 0) || max_iter < 1) fail(XLS_ERR_INVALID_ARG, "tol must be > 0 and max_iter >= 1");
}

}  // namespace

extern "C" {

int xls_poisson_solve(xls_poisson_t P, const double* f, double* phi, double tol, int32_t max_iter,
                      int32_t precond, double* info) {
  return guarded([&]() -> int {
    check_solve_args(P, f, phi, tol, max_iter);
    if (!finite_all(f, P->nd)) fail(XLS_ERR_INVALID_ARG, "f not finite");
    const auto t0 = std::chrono::steady_clock::now();
    XLS_HIP(hipMemcpyAsync(P->b, f, P->nd * 8, hipMemcpyHostToDevice, P->s));
    solve_on_device(P, tol, max_iter, precond, info, t0);
    XLS_HIP(hipMemcpyAsync(phi, P->x, P->nd * 8, hipMemcpyDeviceToHost, P->s));
    XLS_HIP(hipStreamSynchronize(P->s));
    if (info) info[3] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return XLS_OK;
  });
}

int xls_poisson_solve_device(xls_poisson_t P, const double* f, double* phi, double tol, int32_t max_iter,
                             int32_t precond, double* info) {
  return guarded([&]() -> int {
    check_solve_args(P, f, phi, tol, max_iter);
    check_device_range(f, P->nd * 8);
    check_device_range(phi, P->nd * 8);
    const auto t0 = std::chrono::steady_clock::now();
    XLS_HIP(hipMemcpyAsync(P->b, f, P->nd * 8, hipMemcpyDeviceToDevice, P->s));
    solve_on_device(P, tol, max_iter, precond, info, t0);
    XLS_HIP(hipMemcpyAsync(phi, P->x, P->nd * 8, hipMemcpyDeviceToDevice, P->s));
    XLS_HIP(hipStreamSynchronize(P->s));
    if (info) info[3] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return XLS_OK;
  });
}

}  // extern "C"
