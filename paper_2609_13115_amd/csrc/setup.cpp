// Subdomain setup on the host: core mask (binary partition of unity,
// Sec. V-A.2), local->global grid map, per-atom projector support lists and
// values, and the reverse CSR over grid points used by the gather-only
// backprojection (Sec. V-B.2, "Nonlocal pseudopotential").
//
// Integer contract (bit-exact): x_i = origin_x + i*h, dx = x_i - X',
// r2 = (dx*dx + dy*dy) + dz*dz, all in FP64 with no contraction (this file
// is compiled with -ffp-contract=off); a point is in the support iff
// r2 < rc*rc.  Periodic boxes take every image X' = X + s*(n*h),
// s in {-1, 0, 1} per axis, and sum the values of images that land on the
// same point.  Support lists ascend in grid index; the reverse CSR of a point
// lists the covering slots in ascending slot order.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>

#include "xls_internal.h"

namespace xls {

namespace {
inline int64_t wrap64(int64_t a, int64_t n) {
  int64_t r = a % n;
  return r < 0 ? r + n : r;
}
}  // namespace

void build_setup(const xls_subdomain_desc_t& d, SetupTables& t) {
  const int64_t nx = d.n[0], ny = d.n[1], nz = d.n[2];
  const int64_t nd = nx * ny * nz;
  const bool periodic = d.bc == XLS_BC_PERIODIC;

  // core mask and local->global map
  t.core_mask.assign(nd, 0);
  t.global_index.assign(nd, 0);
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) {
        const int64_t g = i + nx * (j + ny * k);
        const bool in = i >= d.core_lo[0] && i < d.core_hi[0] && j >= d.core_lo[1] &&
                        j < d.core_hi[1] && k >= d.core_lo[2] && k < d.core_hi[2];
        t.core_mask[g] = in ? 1 : 0;
        const int64_t gi = wrap64(d.global_offset[0] + i, d.global_n[0]);
        const int64_t gj = wrap64(d.global_offset[1] + j, d.global_n[1]);
        const int64_t gk = wrap64(d.global_offset[2] + k, d.global_n[2]);
        t.global_index[g] = gi + d.global_n[0] * (gj + d.global_n[1] * gk);
      }

  // node coordinates, rounded exactly as origin + i*h
  std::vector<double> xs[3];
  for (int a = 0; a < 3; ++a) {
    xs[a].resize(d.n[a]);
    for (int i = 0; i < d.n[a]; ++i) {
      const double ih = static_cast<double>(i) * d.h;
      xs[a][i] = d.origin[a] + ih;
    }
  }
  const double L[3] = {static_cast<double>(d.n[0]) * d.h, static_cast<double>(d.n[1]) * d.h,
                       static_cast<double>(d.n[2]) * d.h};
  const int smin = periodic ? -1 : 0, smax = periodic ? 1 : 0;
  const double h3 = d.h * d.h * d.h;

  t.sup_off.assign(1, 0);
  t.sup_idx.clear();
  t.sup_val.clear();
  t.slot_atom.clear();
  t.gamma.assign(4 * static_cast<size_t>(d.n_atoms), 0.0);
  for (int a = 0; a < d.n_atoms; ++a) {
    const double X[3] = {d.atom_xyz[3 * a], d.atom_xyz[3 * a + 1], d.atom_xyz[3 * a + 2]};
    const double rc = d.proj[a].rc, w = d.proj[a].gauss_width;
    const double rc2 = rc * rc;
    const double inv2w2 = 2.0 * w * w;
    for (int l = 0; l < 4; ++l) t.gamma[4 * a + l] = d.proj[a].gamma[l];
    std::map<int64_t, std::array<double, 4>> acc;
    for (int sz = smin; sz <= smax; ++sz)
      for (int sy = smin; sy <= smax; ++sy)
        for (int sx = smin; sx <= smax; ++sx) {
          const double Xp[3] = {X[0] + static_cast<double>(sx) * L[0],
                                X[1] + static_cast<double>(sy) * L[1],
                                X[2] + static_cast<double>(sz) * L[2]};
          for (int64_t k = 0; k < nz; ++k) {
            const double dz = xs[2][k] - Xp[2];
            const double dz2 = dz * dz;
            if (!(dz2 < rc2)) continue;  // r2 >= dz2 for every point of this plane
            for (int64_t j = 0; j < ny; ++j) {
              const double dy = xs[1][j] - Xp[1];
              const double dy2 = dy * dy;
              for (int64_t i = 0; i < nx; ++i) {
                const double dx = xs[0][i] - Xp[0];
                const double dx2 = dx * dx;
                const double sxy = dx2 + dy2;
                const double r2 = sxy + dz2;
                if (!(r2 < rc2)) continue;
                const double f = std::exp(-r2 / inv2w2);
                const int64_t g = i + nx * (j + ny * k);
                auto it = acc.find(g);
                const std::array<double, 4> v = {f, dx * f, dy * f, dz * f};
                if (it == acc.end()) {
                  acc.emplace(g, v);
                } else {
                  for (int l = 0; l < 4; ++l) it->second[l] += v[l];
                }
              }
            }
          }
        }
    // discrete normalisation h^3 sum chi^2 = 1 (identically-zero projectors stay zero)
    double nrm[4] = {0, 0, 0, 0};
    for (auto& kv : acc)
      for (int l = 0; l < 4; ++l) nrm[l] += kv.second[l] * kv.second[l];
    double scale[4];
    for (int l = 0; l < 4; ++l) {
      const double n2 = h3 * nrm[l];
      scale[l] = n2 > 0 ? 1.0 / std::sqrt(n2) : 0.0;
    }
    for (auto& kv : acc) {
      t.sup_idx.push_back(static_cast<int32_t>(kv.first));
      for (int l = 0; l < 4; ++l) t.sup_val.push_back(kv.second[l] * scale[l]);
      t.slot_atom.push_back(a);
    }
    t.sup_off.push_back(static_cast<int32_t>(t.sup_idx.size()));
  }

  // reverse CSR: counting sort of slots by grid index (stable => ascending slot)
  const size_t total = t.sup_idx.size();
  t.rev_off.assign(nd + 1, 0);
  for (size_t s = 0; s < total; ++s) t.rev_off[t.sup_idx[s] + 1]++;
  for (int64_t g = 0; g < nd; ++g) t.rev_off[g + 1] += t.rev_off[g];
  t.rev_slot.assign(total, 0);
  std::vector<int32_t> fill(t.rev_off.begin(), t.rev_off.end() - 1);
  for (size_t s = 0; s < total; ++s) t.rev_slot[fill[t.sup_idx[s]]++] = static_cast<int32_t>(s);

  // kernel form: packed per-point (first entry, count) and per-entry payload
  if (total >= (size_t(1) << 27)) fail(XLS_ERR_INVALID_ARG, "too many projector support points");
  // a point without projectors points at a zero-payload sentinel entry
  // (index total), so the kernel's prefetch needs no select
  t.rev_pk.assign(nd, 0);
  for (int64_t g = 0; g < nd; ++g) {
    const int32_t cnt = t.rev_off[g + 1] - t.rev_off[g];
    if (cnt > 31) fail(XLS_ERR_INVALID_ARG, "more than 31 projector sets overlap one grid point");
    const int32_t first = cnt > 0 ? t.rev_off[g] : static_cast<int32_t>(total);
    t.rev_pk[g] = first | (cnt << 27);
  }
  t.rev_val.assign(4 * (total + 1), 0.0);
  t.rev_aoff.assign(total + 1, 0);
  for (size_t e = 0; e < total; ++e) {
    const int32_t sl = t.rev_slot[e];
    for (int l = 0; l < 4; ++l) t.rev_val[4 * e + l] = t.sup_val[4 * static_cast<size_t>(sl) + l];
    t.rev_aoff[e] = 4 * t.slot_atom[sl];
  }
}

}  // namespace xls
