// Hamiltonian application and the fused Chebyshev filter step (Sec. V-B.2).
// Kernel templates; instantiated by stencil_f64.hip, stencil_f32.hip and
// stencil_mix.hip (compiled in parallel).
//
// H y = -1/2 Lap y + V y + V_nl y with the 12th-order (n0 = 6) FD Laplacian:
// 36 neighbour terms (+-1..6 along x, y, z) plus the centre.  One workgroup
// owns NV columns (vectors; two by default), a band of ty full-width x-rows
// and a z-chunk.  It streams along z: the 13 values of its points' z-column
// live in a register queue, the current xy plane (with a 6-point halo) is
// staged in a double-buffered LDS tile, so each input plane is read from HBM
// once per workgroup.  The nonlocal term is a gather over the reverse CSR of the point
// (no atomics); the projection coefficients alpha of the same input come from
// proj_forward.  The Chebyshev recurrence AXPY is fused into the store
// (Y_{k+1} = a (H Y_k - c Y_k) - b Y_{k-1}, in place over Y_{k-1}), and the
// residual mode accumulates ||H y - lam y||^2 instead of storing.
#pragma once
#include <algorithm>
#include <type_traits>

#include "xls_internal.h"

namespace xls {
namespace stencil_detail {

constexpr int R = kRadius;
constexpr int Q = 2 * R + 1;  // register-queue depth
constexpr int HMAX = 4;       // halo cells per thread per plane (host checks)
constexpr int EMAX = 1;       // reverse-CSR entries per point prefetched (more: slow path)
constexpr int EMASK = (1 << 27) - 1;
constexpr int kResidSums = 3;  // residual sweep partial planes: ||H y - lam y||^2, y^T H y, y^T y

template <typename TS, typename TC>
struct HArgs {
  const TS* y;
  const TS* yprev;
  TS* out;
  const TC* v;
  const TC* alpha;
  const int32_t* rev_pk;
  const TC* rev_val;
  const int32_t* rev_aoff;
  int64_t nent;  // reverse-CSR entries
  int32_t nproj;
  int32_t ncols;
  int32_t nx, ny, nz;
  int64_t ld;
  int64_t ld16;  // leading dimension (elements) of a binary16 y / yprev stream (half-input steps)
  int32_t periodic;
  int32_t ty, tz, nyt, nzt;
  TC wc;     // -1/2 * 3 w0 / h^2
  TC w[R];   // -1/2 * w_p / h^2
  TC a, c, b;
  const double* coef;  // grouped launches: per-step (a, c, b) triples in device memory
  int32_t has_prev;
  const double* lam;
  double* partial;
};

__device__ __forceinline__ int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Block id -> logical id such that consecutive logical ids (tiles of the same
// column) land on the same XCD: the hardware deals workgroups round-robin to
// the 8 XCDs, and neighbouring tiles share halo rows in that XCD's L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nb) {
  const uint32_t xcd = bid & 7u, idx = bid >> 3;
  const uint32_t q = nb >> 3, r = nb & 7u;
  return xcd * q + min(xcd, r) + idx;
}

// Workgroup barrier that waits only for this wave's LDS traffic
// (lgkmcnt = 0) and leaves global loads in flight: the next plane's
// prefetches keep streaming across the barrier.  s_waitcnt immediate on
// gfx9: vmcnt[3:0] | expcnt[6:4] | lgkmcnt[11:8] | vmcnt_hi[15:14];
// 0xC07F = vmcnt 63 (no wait), expcnt 7 (no wait), lgkmcnt 0.
__device__ __forceinline__ void lds_barrier() {
  __asm__ __volatile__("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
  __asm__ __volatile__("" ::: "memory");
}

template <typename TS, typename TC>
__device__ __forceinline__ TC load_bc(const TS* __restrict__ col, int x, int y, int z, int nx,
                                      int ny, int nz, int periodic) {
  if (periodic) {
    x = wrapi(x, nx);
    y = wrapi(y, ny);
    z = wrapi(z, nz);
  } else if (x < 0 || x >= nx || y < 0 || y >= ny || z < 0 || z >= nz) {
    return TC(0);
  }
  return static_cast<TC>(col[x + nx * (y + ny * z)]);
}

// ---- buffer-resource loads and stores -------------------------------------
// Each stream is addressed through a buffer resource: the plane offset lives
// in a scalar register and each lane keeps a fixed 32-bit byte offset, so a
// load costs no vector ALU.  A lane offset at or beyond the resource size
// (kOOB) reads 0 and drops stores: zero halo cells, absent projector entries
// and inactive lanes need no branches.
constexpr int kOOB = 0x7FFF0000;
constexpr int kBufWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int64_t bytes) {
  const int n = bytes >= kOOB ? kOOB : static_cast<int>(bytes);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), static_cast<short>(0), n, kBufWord3);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ int bload<int>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return static_cast<int>(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, 0);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff, 0);
}
// cache policy word of a buffer access (bit 1: non-temporal)
template <int AUX>
__device__ __forceinline__ float bload_p(__amdgpu_buffer_rsrc_t r, int voff, int soff, float*) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
}
template <int AUX>
__device__ __forceinline__ double bload_p(__amdgpu_buffer_rsrc_t r, int voff, int soff, double*) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
}
template <int AUX>
__device__ __forceinline__ void bstore_p(float v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, AUX);
}
template <int AUX>
__device__ __forceinline__ void bstore_p(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff, AUX);
}
// binary16 stream element (a warm start kept in half precision), widened
template <typename TC, int AUX>
__device__ __forceinline__ TC bload_h(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  const unsigned short u = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, AUX);
  return static_cast<TC>(__builtin_bit_cast(_Float16, u));
}
// Y_{k-1} is read once and Y_{k+1} written once per launch: both go
// non-temporal, which leaves more of the L2 to the reused data (Y_k's halo
// rows, V, the projector words); -1 % (FP32) and -2 % (FP64) launch time
constexpr int kPrevAux = 2;
constexpr int kOutAux = 2;
// four projector values of one reverse-CSR entry
template <typename TC>
struct Ent4 {
  TC v[4];
};
__device__ __forceinline__ Ent4<float> bload_ent(__amdgpu_buffer_rsrc_t r, int voff) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  typedef float f4 __attribute__((ext_vector_type(4)));
  // cast the whole vector: bit-casting a single vector element reads element 0
  const f4 f = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0));
  Ent4<float> e;
  for (int l = 0; l < 4; ++l) e.v[l] = f[l];
  return e;
}
__device__ __forceinline__ Ent4<double> bload_ent_d(__amdgpu_buffer_rsrc_t r, int voff) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  const u4 a = __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0);
  const u4 b = __builtin_amdgcn_raw_buffer_load_b128(r, voff + 16, 0, 0);
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  Ent4<double> e;
  e.v[0] = __builtin_bit_cast(double, u2{a[0], a[1]});
  e.v[1] = __builtin_bit_cast(double, u2{a[2], a[3]});
  e.v[2] = __builtin_bit_cast(double, u2{b[0], b[1]});
  e.v[3] = __builtin_bit_cast(double, u2{b[2], b[3]});
  return e;
}
template <typename TC>
__device__ __forceinline__ Ent4<TC> load_ent(__amdgpu_buffer_rsrc_t r, int voff);
template <>
__device__ __forceinline__ Ent4<float> load_ent<float>(__amdgpu_buffer_rsrc_t r, int voff) {
  return bload_ent(r, voff);
}
template <>
__device__ __forceinline__ Ent4<double> load_ent<double>(__amdgpu_buffer_rsrc_t r, int voff) {
  return bload_ent_d(r, voff);
}

// WS: LDS row stride in elements (compile time, so every neighbour read uses
// an immediate offset); rows hold nx + 2R entries, nx + 2R <= WS.
// One tile (NV consecutive columns, y band, z chunk) given by its logical
// index; coefficients ca, cc, cb of the fused recurrence.  The NV columns of
// a tile share the grid geometry, V, the reverse-CSR words and the projector
// entries, so those tables are read once per NV columns; each column has its
// own LDS plane buffers, register queue and projection coefficients.  A
// column index at or beyond ncols gets empty buffer resources (loads read
// zero, stores drop).  Shared by the single-operator launch and the grouped
// persistent launch.
// HF (half-input filter steps of a warm start): bit 0, y (Y_k) is binary16
// with leading dimension ld16; bit 1, yprev (Y_{k-1}) is.  The output and
// the arithmetic keep TS / TC.
template <typename TS, typename TC, int MODE, int P, int NT, int WS, int NV, int HF = 0>
__device__ __forceinline__ void stencil_tile(const HArgs<TS, TC>& A, uint32_t logical, TC ca, TC cc, TC cb,
                                             unsigned char* smem_raw) {
  static_assert(NV == 1 || MODE != kResid, "residual sweeps take one column per tile");
  static_assert(HF == 0 || MODE == kFilter, "binary16 inputs only in filter steps");
  TC* lds = reinterpret_cast<TC*>(smem_raw);
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  constexpr int W = WS;
  const int dumpi = W * (A.ty + 2 * R);  // spare slot at the end of each plane buffer
  const int plane = dumpi + 1;
  TC* alds = lds + 2 * NV * plane;     // the columns' projection coefficients

  // Logical order: z chunk, then column group, then y band.  The xcd remap
  // hands each XCD a contiguous run of logical tiles, so when the grid is cut
  // into z chunks (a tuning option; one chunk by default) an XCD sweeps one
  // chunk of many columns and its L2 holds only that chunk's V, reverse-CSR
  // words and projector payload; the bands of one column stay neighbours, so
  // their shared y-halo rows meet in the same L2.
  const int tiles = A.nyt * A.nzt;
  const uint32_t ncg = static_cast<uint32_t>((A.ncols + NV - 1) / NV);
  const uint32_t per_chunk = ncg * static_cast<uint32_t>(A.nyt);
  const int zt = static_cast<int>(logical / per_chunk);
  const uint32_t rem = logical % per_chunk;
  const int col0 = static_cast<int>(rem / static_cast<uint32_t>(A.nyt)) * NV;
  const int yt = static_cast<int>(rem % static_cast<uint32_t>(A.nyt));
  const int t = yt + A.nyt * zt;  // tile index within a column (residual partials)
  const int y0 = yt * A.ty;
  const int tyv = min(A.ty, ny - y0);
  const int z0 = zt * A.tz;
  const int z1 = min(z0 + A.tz, nz);
  const int npts = nx * tyv;
  const int tid = threadIdx.x;
  const int pp = nx * ny;  // points per plane
  constexpr int ES = sizeof(TS), EC = sizeof(TC);
  constexpr int ESY = (HF & 1) ? 2 : ES;  // element bytes of the y stream
  constexpr int ESP = (HF & 2) ? 2 : ES;  // of the yprev stream

  const int64_t colpts = static_cast<int64_t>(nx) * ny * nz;
  __amdgpu_buffer_rsrc_t ry[NV], rp[NV], ro[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const bool live = col0 + v < A.ncols;
    const int64_t c = live ? col0 + v : col0;
    const int64_t pts = live ? colpts : 0;
    const void* yb = (HF & 1) ? static_cast<const void*>(reinterpret_cast<const uint16_t*>(A.y) + c * A.ld16)
                              : static_cast<const void*>(A.y + c * A.ld);
    ry[v] = make_rsrc(yb, pts * ESY);
    // without Y_{k-1} the stream is empty and reads zero
    const bool prev = MODE == kFilter && A.has_prev;
    const void* pb = !prev ? static_cast<const void*>(A.y)
                     : (HF & 2) ? static_cast<const void*>(reinterpret_cast<const uint16_t*>(A.yprev) + c * A.ld16)
                                : static_cast<const void*>(A.yprev + c * A.ld);
    rp[v] = make_rsrc(pb, prev ? pts * ESP : 0);
    ro[v] = make_rsrc(MODE == kResid ? A.y : A.out + c * A.ld, pts * ES);
  }
  const __amdgpu_buffer_rsrc_t rv = make_rsrc(A.v, static_cast<int64_t>(nx) * ny * nz * EC);
  const __amdgpu_buffer_rsrc_t rk = make_rsrc(A.rev_pk, static_cast<int64_t>(nx) * ny * nz * 4);
  const __amdgpu_buffer_rsrc_t re = make_rsrc(A.rev_val, static_cast<int64_t>(A.nent + 1) * 4 * EC);
  const __amdgpu_buffer_rsrc_t ra = make_rsrc(A.rev_aoff, static_cast<int64_t>(A.nent + 1) * 4);

  // points owned by this lane: in-plane byte offsets per stream element size
  // (kOOB when inactive), LDS index written and LDS index read (inactive
  // slots write the spare cell and read the star of the first point)
  int vo[P], os[P], oy[P], opv[P], oc[P], o4[P], li[P], lr[P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int lin = tid + i * NT;
    const bool act = lin < npts;
    const int x = act ? lin % nx : 0, yy = act ? y0 + lin / nx : y0;
    vo[i] = act ? (x + nx * yy) : -1;
    os[i] = act ? vo[i] * ES : kOOB;
    oy[i] = act ? vo[i] * ESY : kOOB;
    opv[i] = act ? vo[i] * ESP : kOOB;
    oc[i] = act ? vo[i] * EC : kOOB;
    o4[i] = act ? vo[i] * 4 : kOOB;
    li[i] = act ? (R + yy - y0) * W + R + x : dumpi;
    lr[i] = (R + yy - y0) * W + R + x;
  }

  // halo cells of a plane (y-halo rows, then periodic x-halo columns): LDS
  // target (dump when unused) and source byte offset (kOOB reads zero)
  const int nhy = 2 * R * nx;
  const int nh = nhy + (A.periodic ? 2 * R * tyv : 0);
  int hl[HMAX], hoff[HMAX];
#pragma unroll
  for (int j = 0; j < HMAX; ++j) {
    const int e = tid + j * NT;
    hl[j] = dumpi;
    hoff[j] = kOOB;
    if (e < nh) {
      int x, yy;
      if (e < nhy) {
        const int r = e / nx;
        x = e % nx;
        yy = r < R ? y0 - R + r : y0 + tyv + (r - R);
        hl[j] = (r < R ? r : R + tyv + (r - R)) * W + R + x;
      } else {
        const int e2 = e - nhy;
        const int row = e2 / (2 * R), c2 = e2 % (2 * R);
        x = c2 < R ? c2 - R : nx + (c2 - R);
        yy = y0 + row;
        hl[j] = (R + row) * W + (c2 < R ? c2 : nx + c2);
      }
      if (A.periodic)
        hoff[j] = (wrapi(x, nx) + nx * wrapi(yy, ny)) * ESY;
      else if (x >= 0 && x < nx && yy >= 0 && yy < ny)
        hoff[j] = (x + nx * yy) * ESY;
    }
  }

  // Dirichlet: x-halo columns are zero for every plane; clear every buffer once
  if (!A.periodic) {
    const int nxh = 2 * R * (A.ty + 2 * R);
    for (int e = tid; e < 2 * NV * nxh; e += NT) {
      const int b = e / nxh, r = e % nxh;
      const int row = r / (2 * R), c2 = r % (2 * R);
      lds[b * plane + row * W + (c2 < R ? c2 : nx + c2)] = TC(0);
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const bool live = col0 + v < A.ncols;
    const TC* __restrict__ ac = A.alpha + static_cast<int64_t>(live ? col0 + v : col0) * A.nproj;
    for (int e = tid; e < A.nproj; e += NT) alds[v * A.nproj + e] = live ? ac[e] : TC(0);
  }

  // plane index of plane zz for the queue (wrapped when periodic), or -1
  // for a zero plane beyond a Dirichlet face; uniform across the workgroup
  auto qplane = [&](int zz) -> int {
    if (zz >= 0 && zz < nz) return zz;
    if (!A.periodic) return -1;
    return wrapi(zz, nz);
  };
  // Every prefetch is issued unconditionally: a plane past the chunk is
  // clamped into the grid (valid memory, value never used) and a zero plane
  // is read through an out-of-range lane offset.  A load under a branch ends
  // in a register merge whose copy waits for the load at once, which drains
  // every prefetch in flight.
  auto clampz = [&](int zz) { return min(zz, nz - 1); };
  // one element of the y stream (plane offset in elements), and of yprev
  auto ldy = [&](int v, int voff, int splane) -> TC {
    if constexpr ((HF & 1) != 0)
      return bload_h<TC, 0>(ry[v], voff, splane * 2);
    else
      return static_cast<TC>(bload<TS>(ry[v], voff, splane * ES));
  };
  auto ldp = [&](int i, int v, int splane) -> TC {
    if constexpr ((HF & 2) != 0)
      return bload_h<TC, kPrevAux>(rp[v], opv[i], splane * 2);
    else
      return static_cast<TC>(bload_p<kPrevAux>(rp[v], opv[i], splane * ES, (TS*)nullptr));
  };
  auto ldq = [&](int i, int v, int zq) -> TC { return ldy(v, zq < 0 ? kOOB : oy[i], max(zq, 0) * pp); };

  // register queue: q[i][v][slot] holds plane z - R + ((slot - ph) mod Q)
  // while plane z is computed at phase ph = (z - z0) mod Q, so the queue
  // advances by renaming (the z-loop is unrolled Q times) instead of moving
  // registers
  TC q[P][NV][Q];
#pragma unroll
  for (int s = 0; s < Q - 1; ++s) {
    const int zq = qplane(z0 - R + s);
#pragma unroll
    for (int i = 0; i < P; ++i)
#pragma unroll
      for (int v = 0; v < NV; ++v) q[i][v][s] = ldq(i, v, zq);
  }

  // prefetch registers.  Two planes ahead: the queue front fr (plane z+1+R
  // while computing z) and Y_{k-1} yp2; the reverse-CSR word rp2.  One plane
  // ahead: q's newest slot, V, Y_{k-1}, the entry payload, the halo cells.
  TC fr[P][NV], yp1[P][NV], yp2[P][NV], vn[P];
  int rp1[P], rp2[P], ea[P];
  Ent4<TC> ev[P];
  TC hv[NV][HMAX];
  auto load_rest = [&](int z) {  // V, entry payload, rev word (z+1) of plane z
    const int so = z * pp;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      vn[i] = bload<TC>(rv, oc[i], so * EC);
      rp1[i] = rp2[i];
      const int e0 = rp1[i] & EMASK;  // points without projectors name the zero sentinel
      ev[i] = load_ent<TC>(re, e0 * 4 * EC);
      ea[i] = bload<int>(ra, e0 * 4, 0);
      rp2[i] = bload<int>(rk, o4[i], clampz(z + 1) * pp * 4);  // unused past the chunk
    }
  };
  {
    const int zq0 = qplane(z0 + R), zq1 = qplane(z0 + 1 + R);
#pragma unroll
    for (int i = 0; i < P; ++i) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        q[i][v][Q - 1] = ldq(i, v, zq0);
        fr[i][v] = ldq(i, v, zq1);
        if (MODE == kFilter) {
          yp1[i][v] = ldp(i, v, z0 * pp);
          yp2[i][v] = ldp(i, v, clampz(z0 + 1) * pp);
        }
      }
      rp2[i] = bload<int>(rk, o4[i], z0 * pp * 4);
    }
  }
  load_rest(z0);
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int j = 0; j < HMAX; ++j) hv[v][j] = ldy(v, hoff[j], z0 * pp);

  // residual sweep: ||H y - lam y||^2, y^T H y and y^T y of the column (the
  // last two give its FP64 Rayleigh quotient)
  double racc = 0.0, hacc = 0.0, nacc = 0.0;
  const double lamc = (MODE == kResid) ? A.lam[col0] : 0.0;

  // one plane at compile-time phase PH
  auto step = [&](auto phc, int z) {
    constexpr int PH = decltype(phc)::value;
    auto QS = [](int s2) { return (s2 + PH) % Q; };  // physical slot of logical s2
    TC* buf = lds + (z & 1) * plane;  // column v's buffer: buf + 2 v plane
    // (a) centre plane and its halo into LDS
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
      for (int i = 0; i < P; ++i) buf[2 * v * plane + li[i]] = q[i][v][QS(R)];
#pragma unroll
      for (int j = 0; j < HMAX; ++j) buf[2 * v * plane + hl[j]] = hv[v][j];
    }
    // (b) next plane's halo
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int j = 0; j < HMAX; ++j) hv[v][j] = ldy(v, hoff[j], clampz(z + 1) * pp);
    lds_barrier();
    // (c) plane z
    const int so = z * pp * ES;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      // two bases behind opaque registers, the row and the column of the
      // star: every LDS offset is then a small non-negative immediate (the
      // row's pair up in ds_read2; with W a multiple of 64 the column's pair
      // up in ds_read2st64), so no per-read address arithmetic remains
      int bxi = lr[i] - R, byi = lr[i] - R * W;
      asm("" : "+v"(bxi));
      asm("" : "+v"(byi));
      TC hy[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const TC* bx = buf + 2 * v * plane + bxi;
        const TC* by = buf + 2 * v * plane + byi;
        const TC ctr = q[i][v][QS(R)];
        TC lap = A.wc * ctr;
#pragma unroll
        for (int p = 1; p <= R; ++p) {
          const TC sm = (bx[R + p] + bx[R - p]) + (by[(R + p) * W] + by[(R - p) * W]) +
                        (q[i][v][QS(R + p)] + q[i][v][QS(R - p)]);
          lap += A.w[p - 1] * sm;
        }
        hy[v] = lap + vn[i] * ctr;
        // one projector set per point is prefetched (absent: zero payload)
        const TC* al = alds + v * A.nproj + ea[i];
        hy[v] += ev[i].v[0] * al[0] + ev[i].v[1] * al[1] + ev[i].v[2] * al[2] + ev[i].v[3] * al[3];
      }
      const int ne = static_cast<int>(static_cast<uint32_t>(rp1[i]) >> 27);
      if (ne > 1) {  // rare: overlapping projector sets
        const int e0 = rp1[i] & EMASK;
        for (int e = e0 + 1; e < e0 + ne; ++e) {
          const TC* sv = A.rev_val + 4 * static_cast<int64_t>(e);
          const int ao = A.rev_aoff[e];
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const TC* a2 = alds + v * A.nproj + ao;
            hy[v] += sv[0] * a2[0] + sv[1] * a2[1] + sv[2] * a2[2] + sv[3] * a2[3];
          }
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (MODE == kApply) {
          bstore(static_cast<TS>(hy[v]), ro[v], os[i], so);
        } else if (MODE == kFilter) {
          const TC r = ca * (hy[v] - cc * q[i][v][QS(R)]) - cb * yp1[i][v];
          bstore_p<kOutAux>(static_cast<TS>(r), ro[v], os[i], so);
        } else if (vo[i] >= 0) {
          const double hv = static_cast<double>(hy[v]), yv = static_cast<double>(q[i][v][QS(R)]);
          const double d = hv - lamc * yv;
          racc += d * d;
          hacc += yv * hv;
          nacc += yv * yv;
        }
      }
    }
    // (d) advance: the oldest slot takes the next front; refill the
    // registers just consumed
#pragma unroll
    for (int i = 0; i < P; ++i)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        q[i][v][QS(0)] = fr[i][v];
        if (MODE == kFilter) yp1[i][v] = yp2[i][v];
      }
    {
      const int zq = qplane(z + 2 + R);
#pragma unroll
      for (int i = 0; i < P; ++i)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          fr[i][v] = ldq(i, v, zq);
          if (MODE == kFilter) yp2[i][v] = ldp(i, v, clampz(z + 2) * pp);
        }
      load_rest(clampz(z + 1));
    }
  };

  using std::integral_constant;
  for (int z = z0; z < z1; z += Q) {
    step(integral_constant<int, 0>{}, z);
    if (z + 1 < z1) step(integral_constant<int, 1>{}, z + 1); else break;
    if (z + 2 < z1) step(integral_constant<int, 2>{}, z + 2); else break;
    if (z + 3 < z1) step(integral_constant<int, 3>{}, z + 3); else break;
    if (z + 4 < z1) step(integral_constant<int, 4>{}, z + 4); else break;
    if (z + 5 < z1) step(integral_constant<int, 5>{}, z + 5); else break;
    if (z + 6 < z1) step(integral_constant<int, 6>{}, z + 6); else break;
    if (z + 7 < z1) step(integral_constant<int, 7>{}, z + 7); else break;
    if (z + 8 < z1) step(integral_constant<int, 8>{}, z + 8); else break;
    if (z + 9 < z1) step(integral_constant<int, 9>{}, z + 9); else break;
    if (z + 10 < z1) step(integral_constant<int, 10>{}, z + 10); else break;
    if (z + 11 < z1) step(integral_constant<int, 11>{}, z + 11); else break;
    if (z + 12 < z1) step(integral_constant<int, 12>{}, z + 12); else break;
  }
  if (MODE == kResid) {
    // deterministic block reduction of the three sums: fixed shuffle tree,
    // then fixed LDS order; sum q of the tile goes to partial plane q
    __syncthreads();
    double* red = reinterpret_cast<double*>(smem_raw);
    double acc3[kResidSums] = {racc, hacc, nacc};
    const int wid = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int qq = 0; qq < kResidSums; ++qq) {
      for (int o2 = 32; o2 > 0; o2 >>= 1) acc3[qq] += __shfl_xor(acc3[qq], o2, 64);
      if (lane == 0) red[qq * (NT / 64) + wid] = acc3[qq];
    }
    __syncthreads();
    if (tid < kResidSums) {
      double sacc = 0.0;
      for (int w = 0; w < NT / 64; ++w) sacc += red[tid * (NT / 64) + w];
      const int64_t plane_elems = static_cast<int64_t>(A.ncols) * tiles;
      A.partial[tid * plane_elems + static_cast<int64_t>(col0) * tiles + t] = sacc;
    }
  }
}

template <typename TS, typename TC, int MODE, int P, int NT, int WS, int NV, int HF = 0>
__global__ __launch_bounds__(NT) void hstencil_kernel(HArgs<TS, TC> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  stencil_tile<TS, TC, MODE, P, NT, WS, NV, HF>(A, xcd_remap(blockIdx.x, gridDim.x), A.a, A.c, A.b, smem_raw);
}

// Grouped persistent filter step over many operators: item = (operator,
// logical tile).  Workgroups walk the item list with a grid stride; the
// xcd remap gives the workgroups of one XCD consecutive items, so the tiles
// that share halo rows meet in the same L2.  Step k reads its recurrence
// coefficients from the operator's device table.
template <typename TS, typename TC, int P, int NT, int WS, int NV>
__global__ __launch_bounds__(NT) void hstencil_group_kernel(const HArgs<TS, TC>* __restrict__ tab,
                                                            const uint2* __restrict__ items, int nitems,
                                                            int k) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const uint32_t G = gridDim.x;
  for (uint32_t it = xcd_remap(blockIdx.x, G); it < static_cast<uint32_t>(nitems); it += G) {
    const uint2 w = items[it];
    const HArgs<TS, TC> A = tab[w.x];
    const double* cf = A.coef + 3 * k;
    stencil_tile<TS, TC, kFilter, P, NT, WS, NV>(A, w.y, static_cast<TC>(cf[0]), static_cast<TC>(cf[1]),
                                             static_cast<TC>(cf[2]), smem_raw);
    __syncthreads();
  }
}

// alpha[col][4a+l] = gamma_{a,l} h^3 sum_s chi_{a,l}(s) y(idx(s), col).  One
// wavefront per (atom, kProjCols columns): lanes stride over the atom's
// support and load each point's index and projector values once for all its
// columns; per column, FP64 partial sums per lane then a fixed xor-shuffle
// reduction (deterministic).  Four columns per wave: eight were measured no
// faster (the gathered column values, not the index and payload reads, set
// its time).
constexpr int kProjCols = 4;
constexpr int kProjSums = 4 * kProjCols;  // one sum per (column, projector)
static_assert(kProjSums == 16, "the reduction below halves 16 sums over 4 lane bits");
template <typename TS, typename TC>
__device__ __forceinline__ void proj_forward_wave(const TS* __restrict__ y, int64_t ld, int ncols, int cbase,
                                                  const int32_t* __restrict__ sup_off,
                                                  const int32_t* __restrict__ sup_idx, const TC* __restrict__ val,
                                                  const double* __restrict__ gamma, double h3,
                                                  TC* __restrict__ alpha, int nproj, int a, int lane) {
  const int s0 = sup_off[a], s1 = sup_off[a + 1];
  const int nc = min(kProjCols, ncols - cbase);
  double acc[kProjCols][4];
#pragma unroll
  for (int c = 0; c < kProjCols; ++c)
#pragma unroll
    for (int l = 0; l < 4; ++l) acc[c][l] = 0.0;
  // Two support points per lane and iteration (s and s + 64, added in that
  // order, so each lane's order is that of a one-point loop): their column
  // loads are in flight together.  The next pair's indices and values load
  // one iteration ahead.  Every load is unconditional from a clamped,
  // in-range entry (a guarded load becomes a branch that waits for it);
  // products of entries past the support are skipped.
  struct Ent {
    int g;
    TC v[4];
  };
  auto fetch = [&](int s) {
    Ent e;
    const int sc = min(s, s1 - 1);
    e.g = sup_idx[sc];
    const TC* v4 = val + 4 * static_cast<int64_t>(sc);
#pragma unroll
    for (int l = 0; l < 4; ++l) e.v[l] = v4[l];
    return e;
  };
  const TS* yc[kProjCols];
#pragma unroll
  for (int c = 0; c < kProjCols; ++c) yc[c] = y + static_cast<int64_t>(cbase + min(c, nc - 1)) * ld;
  if (s0 + lane < s1) {
    Ent na = fetch(s0 + lane), nb = fetch(s0 + lane + 64);
    for (int s = s0 + lane; s < s1; s += 128) {
      const Ent ea = na, eb = nb;
      na = fetch(s + 128);
      nb = fetch(s + 192);
      TS ya[kProjCols], yb[kProjCols];
#pragma unroll
      for (int c = 0; c < kProjCols; ++c) {
        ya[c] = yc[c][ea.g];
        yb[c] = yc[c][eb.g];
      }
#pragma unroll
      for (int c = 0; c < kProjCols; ++c)
#pragma unroll
        for (int l = 0; l < 4; ++l) acc[c][l] += static_cast<double>(ea.v[l]) * static_cast<double>(ya[c]);
      if (s + 64 < s1) {
#pragma unroll
        for (int c = 0; c < kProjCols; ++c)
#pragma unroll
          for (int l = 0; l < 4; ++l) acc[c][l] += static_cast<double>(eb.v[l]) * static_cast<double>(yb[c]);
      }
    }
  }
  // Reduction of the 16 sums by recursive halving: at offsets 32, 16, 8, 4 a
  // lane keeps half of its values, each added to its partner's copy (the
  // pairs and operand order of a full xor-shuffle tree, so every sum is
  // bit-identical to it, in 32 shuffles instead of 96); offsets 2 and 1
  // finish, and lane 4 v holds sum v = 4 c + l.  Both halves are shuffled
  // and the kept sum selected, so no register array is indexed at run time.
  double r[kProjSums];
#pragma unroll
  for (int c = 0; c < kProjCols; ++c)
#pragma unroll
    for (int l = 0; l < 4; ++l) r[4 * c + l] = acc[c][l];
#pragma unroll
  for (int lev = 0; lev < 4; ++lev) {
    const int off = 32 >> lev, half = (kProjSums / 2) >> lev;
    const bool up = (lane & off) != 0;
#pragma unroll
    for (int j = 0; j < half; ++j) {
      const double lo = r[j] + __shfl_xor(r[j], off, 64);
      const double hi = r[j + half] + __shfl_xor(r[j + half], off, 64);
      r[j] = up ? hi : lo;
    }
  }
  double t = r[0];
  t += __shfl_xor(t, 2, 64);
  t += __shfl_xor(t, 1, 64);
  const int vi = lane >> 2, c = vi >> 2, l = vi & 3;
  if ((lane & 3) == 0 && c < nc)
    alpha[static_cast<int64_t>(cbase + c) * nproj + 4 * a + l] = static_cast<TC>(gamma[4 * a + l] * h3 * t);
}

template <typename TS, typename TC>
__global__ __launch_bounds__(256) void proj_forward_kernel(const TS* __restrict__ y, int64_t ld,
                                                           int ncols, const int32_t* __restrict__ sup_off,
                                                           const int32_t* __restrict__ sup_idx,
                                                           const TC* __restrict__ val,
                                                           const double* __restrict__ gamma,
                                                           double h3, TC* __restrict__ alpha,
                                                           int nproj, int n_atoms) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // logical block = atom + n_atoms * column group, remapped so that the
  // atoms of one column group share an XCD: neighbouring atoms' supports
  // gather from the same cache lines, which then meet in that XCD's L2
  const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
  const int a = static_cast<int>(lb % static_cast<uint32_t>(n_atoms));
  const int cbase = (static_cast<int>(lb / static_cast<uint32_t>(n_atoms)) * 4 + wave) * kProjCols;
  if (cbase >= ncols) return;
  proj_forward_wave<TS, TC>(y, ld, ncols, cbase, sup_off, sup_idx, val, gamma, h3, alpha, nproj, a, lane);
}

// Grouped forward projection: item = (operator, atom + n_atoms * column group).
template <typename TS, typename TC>
struct PArgs {
  const TS* y;
  int64_t ld;
  const int32_t* sup_off;
  const int32_t* sup_idx;
  const TC* val;
  const double* gamma;
  double h3;
  TC* alpha;
  int32_t nproj, ncols, n_atoms;
};

template <typename TS, typename TC>
__global__ __launch_bounds__(256) void proj_forward_group_kernel(const PArgs<TS, TC>* __restrict__ tab,
                                                                 const uint2* __restrict__ items, int nitems) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // consecutive items (atoms of one operator and column group) share an XCD
  const uint32_t G = gridDim.x;
  for (uint32_t it = xcd_remap(blockIdx.x, G); it < static_cast<uint32_t>(nitems); it += G) {
    const uint2 w = items[it];
    const PArgs<TS, TC> A = tab[w.x];
    const int a = static_cast<int>(w.y % static_cast<uint32_t>(A.n_atoms));
    const int cbase = (static_cast<int>(w.y / static_cast<uint32_t>(A.n_atoms)) * 4 + wave) * kProjCols;
    if (cbase >= A.ncols) continue;
    proj_forward_wave<TS, TC>(A.y, A.ld, A.ncols, cbase, A.sup_off, A.sup_idx, A.val, A.gamma, A.h3, A.alpha,
                              A.nproj, a, lane);
  }
}

struct TileChoice {
  int block, ty, nyt, tz, nzt, P, ws, nv;
  size_t smem;
};

// Launch plan: one grid point per lane-slot, at most 2 slots per lane.
inline int default_ty(int nx, int ny, int elem, int block, const StencilLaunch& cfg) {
  // default tile: ~2 points per lane (measured best on the 64^3 box in both
  // precisions, and for the FP64 residual sweep of FP32 blocks: -16 %)
  const int target = 2 * block;
  (void)elem;
  const int ty = cfg.ty > 0 ? cfg.ty : std::max(1, target / nx);
  return std::max(1, std::min(ty, ny));
}

inline TileChoice choose_tiles(int nx, int ny, int nz, int elem, int nproj, int64_t ld, int periodic,
                               const StencilLaunch& cfg) {
  TileChoice tc{};
  if (cfg.block == 0) {  // 256 threads when their halo budget covers the tile's halo, else 512
    const int ty = default_ty(nx, ny, elem, 256, cfg);
    tc.block = (2 * R * nx + (periodic ? 2 * R * ty : 0) <= HMAX * 256) ? 256 : 512;
  } else {
    tc.block = cfg.block == 256 ? 256 : 512;
  }
  (void)ld;
  const int ty = default_ty(nx, ny, elem, tc.block, cfg);
  tc.ty = ty;
  tc.nyt = (ny + ty - 1) / ty;
  tc.tz = cfg.tz > 0 ? std::min(cfg.tz, nz) : nz;
  tc.nzt = (nz + tc.tz - 1) / tc.tz;
  tc.P = (nx * ty + tc.block - 1) / tc.block;
  tc.ws = (nx + 2 * R <= 80) ? 80 : 128;
  auto smem_of = [&](int nv) {
    return static_cast<size_t>(elem) * nv * (2 * (static_cast<size_t>(tc.ws) * (ty + 2 * R) + 1) + nproj);
  };
  // Default: two vectors per tile, so V, the reverse-CSR words and the
  // projector payload are read once for both (these tables outweigh a
  // column's own traffic; -10 % launch time on the 64^3 box in both
  // precisions); one when two would not fit the LDS.
  tc.nv = cfg.nv > 0 ? cfg.nv : (smem_of(2) <= 160 * 1024 ? 2 : 1);
  tc.smem = smem_of(tc.nv);
  return tc;
}

inline void check_tiles(const TileChoice& tc, int nx, int periodic, int elem) {
  {
    if (nx + 2 * R > 128) fail(XLS_ERR_INVALID_ARG, "grid x extent must be <= 116");
    if (tc.P > 2) fail(XLS_ERR_INVALID_ARG, "stencil tile needs more than 2 points per thread");
    if (tc.nv != 1 && tc.nv != 2) fail(XLS_ERR_INVALID_ARG, "stencil vectors per tile must be 1 or 2");
    const int halo = 2 * R * nx + (periodic ? 2 * R * tc.ty : 0);
    if (halo > HMAX * tc.block) fail(XLS_ERR_INVALID_ARG, "stencil halo exceeds the per-thread budget");
  }
  if (tc.smem > 160 * 1024) fail(XLS_ERR_INVALID_ARG, "stencil tile exceeds LDS");
}

template <typename K>
void allow_smem(K kern, size_t smem) {
  ensure_dyn_smem(reinterpret_cast<const void*>(kern), smem);
}

template <typename TS, typename TC, int MODE, int P, int WS, int NV, int HF>
void launch_mode(const HArgs<TS, TC>& args, dim3 grid, int block, size_t smem, hipStream_t st) {
  if (block == 256) {
    allow_smem(hstencil_kernel<TS, TC, MODE, P, 256, WS, NV, HF>, smem);
    hipLaunchKernelGGL((hstencil_kernel<TS, TC, MODE, P, 256, WS, NV, HF>), grid, dim3(256), smem, st, args);
  } else {
    allow_smem(hstencil_kernel<TS, TC, MODE, P, 512, WS, NV, HF>, smem);
    hipLaunchKernelGGL((hstencil_kernel<TS, TC, MODE, P, 512, WS, NV, HF>), grid, dim3(512), smem, st, args);
  }
}

template <typename TS, typename TC, int MODE, int WS, int NV, int HF>
void launch_pnv(const TileChoice& tc, const HArgs<TS, TC>& args, dim3 grid, size_t smem, hipStream_t st) {
  switch (tc.P) {
    case 1: launch_mode<TS, TC, MODE, 1, WS, NV, HF>(args, grid, tc.block, smem, st); break;
    case 2: launch_mode<TS, TC, MODE, 2, WS, NV, HF>(args, grid, tc.block, smem, st); break;
    default: fail(XLS_ERR_INVALID_ARG, "stencil tile needs more than 2 points per thread");
  }
}

template <typename TS, typename TC, int MODE, int WS, int HF>
void launch_ws(const TileChoice& tc, const HArgs<TS, TC>& args, dim3 grid, size_t smem, hipStream_t st) {
  if (tc.nv == 1) {
    launch_pnv<TS, TC, MODE, WS, 1, HF>(tc, args, grid, smem, st);
  } else if constexpr (MODE != kResid) {
    launch_pnv<TS, TC, MODE, WS, 2, HF>(tc, args, grid, smem, st);
  } else {
    fail(XLS_ERR_INVALID_ARG, "residual sweeps take one vector per tile");
  }
}

template <typename TS, typename TC, int MODE, int HF = 0>
void launch_any(const TileChoice& tc, const HArgs<TS, TC>& args, dim3 grid, size_t smem, hipStream_t st) {
  if (tc.ws == 80)
    launch_ws<TS, TC, MODE, 80, HF>(tc, args, grid, smem, st);
  else
    launch_ws<TS, TC, MODE, 128, HF>(tc, args, grid, smem, st);
}

// FD weights of d^2/dx^2 at 12th order (n0 = 6), from the closed form
// w_p = 2 (-1)^(p+1) (n0!)^2 / (p^2 (n0-p)! (n0+p)!), w_0 = -2 sum_p w_p.
inline void fd_weights6(double w[R + 1]) {
  double f[2 * R + 1];
  f[0] = 1.0;
  for (int i = 1; i <= 2 * R; ++i) f[i] = f[i - 1] * i;
  double s = 0.0;
  for (int p = 1; p <= R; ++p) {
    const double sign = (p % 2 == 1) ? 1.0 : -1.0;
    w[p] = 2.0 * sign * f[R] * f[R] / (static_cast<double>(p) * p * f[R - p] * f[R + p]);
    s += w[p];
  }
  w[0] = -2.0 * s;
}

}  // namespace stencil_detail

using namespace stencil_detail;

template <typename TC>
static TileChoice tiles_for(const OpTables<TC>& op, int64_t ld, const StencilLaunch& cfg) {
  return choose_tiles(op.nx, op.ny, op.nz, sizeof(TC), 4 * op.n_atoms, ld, op.periodic, cfg);
}

#ifdef XLS_STENCIL_DEFINE_HOST
void stencil_validate(int nx, int ny, int nz, int periodic, int elem_bytes, int nproj,
                      const StencilLaunch& cfg) {
  if (cfg.block != 0 && cfg.block != 256 && cfg.block != 512)
    fail(XLS_ERR_INVALID_ARG, "stencil block must be 0 (choose), 256 or 512");
  if (cfg.ty < 0 || cfg.tz < 0) fail(XLS_ERR_INVALID_ARG, "stencil tile sizes must be >= 0");
  if (cfg.nv < 0 || cfg.nv > 2) fail(XLS_ERR_INVALID_ARG, "stencil vectors per tile must be 0, 1 or 2");
  // both variants a launch may take (vector runs need an aligned column stride)
  check_tiles(choose_tiles(nx, ny, nz, elem_bytes, nproj, 64, periodic, cfg), nx, periodic, elem_bytes);
  check_tiles(choose_tiles(nx, ny, nz, elem_bytes, nproj, 1, periodic, cfg), nx, periodic, elem_bytes);
}

size_t stencil_partial_elems(const OpTables<float>& op, int ncols, const StencilLaunch& cfg) {
  const TileChoice a = tiles_for(op, 64, cfg), b = tiles_for(op, 1, cfg);
  return static_cast<size_t>(kResidSums) * ncols * std::max(a.nyt * a.nzt, b.nyt * b.nzt);
}
size_t stencil_partial_elems(const OpTables<double>& op, int ncols, const StencilLaunch& cfg) {
  const TileChoice a = tiles_for(op, 64, cfg), b = tiles_for(op, 1, cfg);
  return static_cast<size_t>(kResidSums) * ncols * std::max(a.nyt * a.nzt, b.nyt * b.nzt);
}

#endif  // XLS_STENCIL_DEFINE_HOST

// Operator tables, geometry and FD weights of one launch (coefficients,
// residual outputs and has_prev are set by the caller).
template <typename TS, typename TC>
static HArgs<TS, TC> make_hargs(const OpTables<TC>& op, const TileChoice& tc, const TS* y, int64_t ld,
                                int ncols, const TC* alpha, TS* out, const TS* yprev) {
  HArgs<TS, TC> A{};
  A.y = y;
  A.yprev = yprev;
  A.out = out;
  A.v = op.v;
  A.alpha = alpha;
  A.rev_pk = op.rev_pk;
  A.rev_val = op.rev_val;
  A.rev_aoff = op.rev_aoff;
  A.nent = op.nent;
  A.nproj = 4 * op.n_atoms;
  A.ncols = ncols;
  A.nx = op.nx;
  A.ny = op.ny;
  A.nz = op.nz;
  A.ld = ld;
  A.periodic = op.periodic;
  A.ty = tc.ty;
  A.tz = tc.tz;
  A.nyt = tc.nyt;
  A.nzt = tc.nzt;
  double w[R + 1];
  fd_weights6(w);
  const double s = -0.5 / (op.h * op.h);
  A.wc = static_cast<TC>(3.0 * w[0] * s);
  for (int p = 1; p <= R; ++p) A.w[p - 1] = static_cast<TC>(w[p] * s);
  return A;
}

template <typename TS, typename TC>
void launch_stencil(StencilMode mode, const OpTables<TC>& op, const TS* y, int64_t ld, int ncols,
                    const TC* alpha, TS* out, const TS* yprev, double a, double c, double b,
                    const double* lam, double* partial, double* resid2, hipStream_t st,
                    const StencilLaunch& cfg, double* rq) {
  if (ncols <= 0) return;
  StencilLaunch cfg1 = cfg;
  if (mode == kResid) cfg1.nv = 1;  // per-column partial sums
  const TileChoice tc = tiles_for(op, ld, cfg1);
  check_tiles(tc, op.nx, op.periodic, sizeof(TC));
  HArgs<TS, TC> A = make_hargs<TS, TC>(op, tc, y, ld, ncols, alpha, out, yprev);
  A.a = static_cast<TC>(a);
  A.c = static_cast<TC>(c);
  A.b = static_cast<TC>(b);
  A.has_prev = (yprev != nullptr && b != 0.0) ? 1 : 0;
  A.lam = lam;
  A.partial = partial;
  const int64_t nblocks = static_cast<int64_t>((ncols + tc.nv - 1) / tc.nv) * tc.nyt * tc.nzt;
  if (nblocks > 0x7fffffff) fail(XLS_ERR_INVALID_ARG, "too many stencil tiles");
  size_t smem = tc.smem;
  if (mode == kResid) smem = std::max(smem, static_cast<size_t>(kResidSums * (tc.block / 64) * sizeof(double)));
  const dim3 grid(static_cast<unsigned>(nblocks));
  // FP32-arithmetic sweeps never accumulate residuals, and FP64 sweeps of
  // FP32 blocks never run the filter recurrence: those pairs are not built
  constexpr bool kHasFilter = std::is_same<TS, TC>::value;
  constexpr bool kHasResid = std::is_same<TC, double>::value;
  switch (mode) {
    case kApply: launch_any<TS, TC, kApply>(tc, A, grid, smem, st); break;
    case kFilter:
      if constexpr (kHasFilter) launch_any<TS, TC, kFilter>(tc, A, grid, smem, st);
      else fail(XLS_ERR_INVALID_ARG, "filter sweep not available for this precision pair");
      break;
    case kResid:
      if constexpr (kHasResid) {
        launch_any<TS, TC, kResid>(tc, A, grid, smem, st);
        XLS_LAUNCH_CHECK("hstencil_kernel");
        const int tiles = tc.nyt * tc.nzt;
        const int64_t plane_elems = static_cast<int64_t>(ncols) * tiles;
        launch_reduce_cols(partial, tiles, ncols, resid2, 1, st);
        if (rq) launch_reduce_rq(partial + plane_elems, partial + 2 * plane_elems, tiles, ncols, rq, st);
        return;
      } else {
        fail(XLS_ERR_INVALID_ARG, "residual sweep needs FP64 arithmetic");
      }
  }
  XLS_LAUNCH_CHECK("hstencil_kernel");
}

// Filter step whose Y_k (y16) or Y_{k-1} (yprev16) is a binary16 block with
// leading dimension ld16 (the first two steps from a half-precision warm
// start); the other operands, the output and the arithmetic are TS.
template <typename TS, typename TC>
void launch_filter_half(const OpTables<TC>& op, const TS* y, const uint16_t* y16, int64_t ld, int64_t ld16,
                        int ncols, const TC* alpha, TS* out, const uint16_t* yprev16, double a, double c, double b,
                        hipStream_t st, const StencilLaunch& cfg) {
  static_assert(std::is_same<TS, TC>::value, "filter steps run in the storage precision");
  if (ncols <= 0) return;
  if ((y16 == nullptr) == (yprev16 == nullptr)) fail(XLS_ERR_INVALID_ARG, "one binary16 stream per half step");
  const TileChoice tc = tiles_for(op, ld, cfg);
  check_tiles(tc, op.nx, op.periodic, sizeof(TC));
  HArgs<TS, TC> A = make_hargs<TS, TC>(op, tc, y16 ? reinterpret_cast<const TS*>(y16) : y, ld, ncols, alpha, out,
                                       reinterpret_cast<const TS*>(yprev16));
  A.ld16 = ld16;
  A.a = static_cast<TC>(a);
  A.c = static_cast<TC>(c);
  A.b = static_cast<TC>(b);
  A.has_prev = (yprev16 != nullptr && b != 0.0) ? 1 : 0;
  const int64_t nblocks = static_cast<int64_t>((ncols + tc.nv - 1) / tc.nv) * tc.nyt * tc.nzt;
  if (nblocks > 0x7fffffff) fail(XLS_ERR_INVALID_ARG, "too many stencil tiles");
  const dim3 grid(static_cast<unsigned>(nblocks));
  if (y16)
    launch_any<TS, TC, kFilter, 1>(tc, A, grid, tc.smem, st);
  else
    launch_any<TS, TC, kFilter, 2>(tc, A, grid, tc.smem, st);
  XLS_LAUNCH_CHECK("hstencil_kernel (binary16 input)");
}

template <typename TS, typename TC>
void launch_proj_forward(const OpTables<TC>& op, const TS* y, int64_t ld, int ncols, TC* alpha,
                         hipStream_t st) {
  if (op.n_atoms == 0 || ncols <= 0) return;
  const int64_t nb = static_cast<int64_t>(op.n_atoms) * ((ncols + 4 * kProjCols - 1) / (4 * kProjCols));
  if (nb > 0x7fffffff) fail(XLS_ERR_INVALID_ARG, "too many projection blocks");
  const double h3 = op.h * op.h * op.h;
  hipLaunchKernelGGL((proj_forward_kernel<TS, TC>), dim3(static_cast<unsigned>(nb)), dim3(256), 0, st, y, ld, ncols,
                     op.sup_off, op.sup_idx, op.slot_val, op.gamma, h3, alpha, 4 * op.n_atoms, op.n_atoms);
  XLS_LAUNCH_CHECK("proj_forward_kernel");
}

// ---------------------------------------------------------------------------
// Grouped filter steps (batch engine)
// ---------------------------------------------------------------------------
template <typename T>
T* group_alloc(size_t n) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess)
    fail(XLS_ERR_OUT_OF_MEMORY, "grouped filter: device allocation failed");
  return static_cast<T*>(p);
}
inline void group_release(void* p) {
  if (p) (void)hipFree(p);
}

template <typename TS>
struct FilterGroup {
  struct Bucket {
    int P = 1, block = 256, ws = 80, nv = 1;
    size_t smem = 0;
    uint2* items = nullptr;
    std::vector<int> count;  // items taking part in step k
    int grid_cap = 0;
  };
  std::vector<Bucket> buckets;
  HArgs<TS, TS>* tab[3] = {nullptr, nullptr, nullptr};  // step 0, odd steps, even steps >= 2
  PArgs<TS, TS>* ptab[2] = {nullptr, nullptr};          // steps with k even / odd
  uint2* pitems = nullptr;
  std::vector<int> pcount;
  int pgrid = 0;
  int steps = 0;
};

template <typename TS, int P, int NT, int WS, int NV>
int group_occupancy(size_t smem) {
  allow_smem(hstencil_group_kernel<TS, TS, P, NT, WS, NV>, smem);
  int nb = 0;
  XLS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &nb, reinterpret_cast<const void*>(hstencil_group_kernel<TS, TS, P, NT, WS, NV>), NT, smem));
  return std::max(1, nb);
}

// one grouped launch shape: calls f with compile-time (P, WS, NV) of bucket b
template <typename F>
void group_dispatch(int P, int ws, int nv, F&& f) {
  using std::integral_constant;
  auto by_nv = [&](auto pc, auto wc) {
    if (nv == 1) f(pc, wc, integral_constant<int, 1>{});
    else f(pc, wc, integral_constant<int, 2>{});
  };
  auto by_ws = [&](auto pc) {
    if (ws == 80) by_nv(pc, integral_constant<int, 80>{});
    else by_nv(pc, integral_constant<int, 128>{});
  };
  if (P == 1) by_ws(integral_constant<int, 1>{});
  else if (P == 2) by_ws(integral_constant<int, 2>{});
  else fail(XLS_ERR_INVALID_ARG, "grouped stencil launches take at most 2 points per thread");
}

template <typename TS>
int group_occ(int P, int block, int ws, int nv, size_t smem) {
  int nb = 1;
  group_dispatch(P, ws, nv, [&](auto pc, auto wc, auto vc) {
    constexpr int PP = decltype(pc)::value, WW = decltype(wc)::value, VV = decltype(vc)::value;
    nb = block == 256 ? group_occupancy<TS, PP, 256, WW, VV>(smem) : group_occupancy<TS, PP, 512, WW, VV>(smem);
  });
  return nb;
}

template <typename TS>
void group_launch(const typename FilterGroup<TS>::Bucket& b, const HArgs<TS, TS>* tab, int n, int k,
                  hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(std::min(n, b.grid_cap)));
  group_dispatch(b.P, b.ws, b.nv, [&](auto pc, auto wc, auto vc) {
    constexpr int PP = decltype(pc)::value, WW = decltype(wc)::value, VV = decltype(vc)::value;
    if (b.block == 256)
      hipLaunchKernelGGL((hstencil_group_kernel<TS, TS, PP, 256, WW, VV>), grid, dim3(256), b.smem, st, tab,
                         b.items, n, k);
    else
      hipLaunchKernelGGL((hstencil_group_kernel<TS, TS, PP, 512, WW, VV>), grid, dim3(512), b.smem, st, tab,
                         b.items, n, k);
  });
}

template <typename TS>
void filter_group_free(FilterGroup<TS>* g) {
  if (!g) return;
  for (auto& b : g->buckets) group_release(b.items);
  for (auto* t : g->tab) group_release(t);
  for (auto* t : g->ptab) group_release(t);
  group_release(g->pitems);
  delete g;
}

template <typename TS>
FilterGroup<TS>* filter_group_build(const std::vector<FilterGroupOp<TS>>& ops) {
  auto* g = new FilterGroup<TS>();
  try {
    const int n = static_cast<int>(ops.size());
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ops[a].degree > ops[b].degree; });
    for (const auto& o : ops) g->steps = std::max(g->steps, o.degree);
    std::vector<TileChoice> tcs(n);
    std::vector<int> bucket_of(n);
    for (int i = 0; i < n; ++i) {
      const auto& o = ops[i];
      if (o.degree < 1 || o.ncols < 1) fail(XLS_ERR_INVALID_ARG, "grouped filter: degree and ncols must be >= 1");
      tcs[i] = tiles_for(*o.op, o.ld, o.cfg);
      check_tiles(tcs[i], o.op->nx, o.op->periodic, sizeof(TS));
      int bi = -1;
      for (size_t j = 0; j < g->buckets.size(); ++j) {
        const auto& b = g->buckets[j];
        if (b.P == tcs[i].P && b.block == tcs[i].block && b.ws == tcs[i].ws && b.nv == tcs[i].nv)
          bi = static_cast<int>(j);
      }
      if (bi < 0) {
        typename FilterGroup<TS>::Bucket b;
        b.P = tcs[i].P;
        b.block = tcs[i].block;
        b.ws = tcs[i].ws;
        b.nv = tcs[i].nv;
        g->buckets.push_back(b);
        bi = static_cast<int>(g->buckets.size()) - 1;
      }
      g->buckets[bi].smem = std::max(g->buckets[bi].smem, tcs[i].smem);
      bucket_of[i] = bi;
    }
    // operator tables for the three step kinds and two input parities
    for (int v = 0; v < 3; ++v) {
      const int k = v;  // representative step: 0, 1 (odd), 2 (even >= 2)
      std::vector<HArgs<TS, TS>> h(n);
      for (int i = 0; i < n; ++i) {
        const auto& o = ops[i];
        TS* in = o.buf[(o.cur0 + k) & 1];
        TS* out = o.buf[(o.cur0 + k + 1) & 1];
        h[i] = make_hargs<TS, TS>(*o.op, tcs[i], in, o.ld, o.ncols, o.alpha, out, k >= 1 ? out : nullptr);
        h[i].coef = o.coef;
        h[i].has_prev = k >= 1 ? 1 : 0;
      }
      g->tab[v] = group_alloc<HArgs<TS, TS>>(n);
      XLS_HIP(hipMemcpy(g->tab[v], h.data(), n * sizeof(h[0]), hipMemcpyHostToDevice));
    }
    for (int v = 0; v < 2; ++v) {
      std::vector<PArgs<TS, TS>> h(n);
      for (int i = 0; i < n; ++i) {
        const auto& o = ops[i];
        PArgs<TS, TS> a{};
        a.y = o.buf[(o.cur0 + v) & 1];
        a.ld = o.ld;
        a.sup_off = o.op->sup_off;
        a.sup_idx = o.op->sup_idx;
        a.val = o.op->slot_val;
        a.gamma = o.op->gamma;
        a.h3 = o.op->h * o.op->h * o.op->h;
        a.alpha = o.alpha;
        a.nproj = 4 * o.op->n_atoms;
        a.ncols = o.ncols;
        a.n_atoms = o.op->n_atoms;
        h[i] = a;
      }
      g->ptab[v] = group_alloc<PArgs<TS, TS>>(n);
      XLS_HIP(hipMemcpy(g->ptab[v], h.data(), n * sizeof(h[0]), hipMemcpyHostToDevice));
    }
    int cus = 0;
    XLS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
    // work items; operators in descending degree, so step k uses a prefix
    auto build_items = [&](auto count_of, std::vector<int>& count, uint2*& dst, auto member) {
      std::vector<uint2> items;
      std::vector<int64_t> end_of;
      std::vector<int> degs;
      for (int i : order) {
        if (!member(i)) continue;
        const int64_t nt = count_of(i);
        if (static_cast<int64_t>(items.size()) + nt > 0x7fffffff) fail(XLS_ERR_INVALID_ARG, "too many work items");
        for (int64_t l = 0; l < nt; ++l)
          items.push_back(make_uint2(static_cast<unsigned>(i), static_cast<unsigned>(l)));
        end_of.push_back(static_cast<int64_t>(items.size()));
        degs.push_back(ops[i].degree);
      }
      count.assign(g->steps, 0);
      for (int k = 0; k < g->steps; ++k)
        for (size_t j = 0; j < degs.size(); ++j)
          if (degs[j] > k) count[k] = static_cast<int>(end_of[j]);
      dst = group_alloc<uint2>(items.size());
      if (!items.empty())
        XLS_HIP(hipMemcpy(dst, items.data(), items.size() * sizeof(uint2), hipMemcpyHostToDevice));
    };
    for (size_t bi = 0; bi < g->buckets.size(); ++bi) {
      auto& b = g->buckets[bi];
      build_items(
          [&](int i) {
            return static_cast<int64_t>((ops[i].ncols + tcs[i].nv - 1) / tcs[i].nv) * tcs[i].nyt * tcs[i].nzt;
          },
          b.count, b.items, [&](int i) { return bucket_of[i] == static_cast<int>(bi); });
      b.grid_cap = group_occ<TS>(b.P, b.block, b.ws, b.nv, b.smem) * cus;
    }
    build_items([&](int i) {
      return static_cast<int64_t>(ops[i].op->n_atoms) * ((ops[i].ncols + 4 * kProjCols - 1) / (4 * kProjCols));
    },
                g->pcount, g->pitems, [](int) { return true; });
    g->pgrid = 16 * cus;
  } catch (...) {
    filter_group_free(g);
    throw;
  }
  return g;
}

template <typename TS>
void filter_group_step(FilterGroup<TS>* g, int k, hipStream_t st) {
  if (k < 0 || k >= g->steps) fail(XLS_ERR_INVALID_ARG, "grouped filter: step out of range");
  if (g->pcount[k] > 0) {
    const dim3 grid(static_cast<unsigned>(std::min(g->pcount[k], g->pgrid)));
    hipLaunchKernelGGL((proj_forward_group_kernel<TS, TS>), grid, dim3(256), 0, st, g->ptab[k & 1], g->pitems,
                       g->pcount[k]);
    XLS_LAUNCH_CHECK("proj_forward_group_kernel");
  }
  const HArgs<TS, TS>* tab = g->tab[k == 0 ? 0 : ((k & 1) ? 1 : 2)];
  for (const auto& b : g->buckets) {
    const int n = b.count[k];
    if (n <= 0) continue;
    group_launch<TS>(b, tab, n, k, st);
    XLS_LAUNCH_CHECK("hstencil_group_kernel");
  }
}

template <typename TS>
int filter_group_steps(const FilterGroup<TS>* g) {
  return g->steps;
}

}  // namespace xls
