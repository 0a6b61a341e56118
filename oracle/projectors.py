"""Kleinman-Bylander nonlocal projectors (oracle, test infrastructure only).

The paper's V_nl groups projectors by atom; the forward projection and
gamma scaling act per atom and the backprojection gathers, for every grid
point, the projector values that cover it through a reverse CSR over grid
points (Sec. V-B.2, "Nonlocal pseudopotential").  The paper's ONCV
projectors are not available, so each atom carries four synthetic
projectors (s, px, py, pz):

  f(r) = exp(-r^2 / (2 w^2)),  chi_s = f,  chi_px = (x - X) f, ...

truncated at r < r_c and normalised so that h^3 sum chi^2 = 1 (a projector
that is identically zero on the box is left at zero).
V_nl psi = sum_j gamma_j chi_j (h^3 chi_j^T psi).

Integer contract (must be reproduced bit for bit by any implementation):
  x_i = origin_x + i*h, dx = x_i - X' (X' = X + s*L for periodic image
  shift s in {-1,0,1} with L = n*h; only s = 0 for a Dirichlet box),
  r2 = (dx*dx + dy*dy) + dz*dz, every operation rounded in FP64 with no
  fused multiply-add; a point belongs to the support iff r2 < rc*rc.
  Values from several images landing on the same point are summed.
  Support lists are sorted by ascending g; the reverse CSR of a point lists
  support slots in ascending slot order (= ascending atom order).
Pins: lattice-point counts in a ball, normalisation, s/p orthogonality at a
node-centred atom, the radial shape at listed lattice points (width
convention), the explicit sum over periodic images in a box smaller than
2 r_c, dense assembly symmetry (tests/test_oracle_projectors.py).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Sequence

import numpy as np


@dataclass
class ProjectorTables:
    offsets: np.ndarray   # i32[n_atoms + 1]
    idx: np.ndarray       # i32[total]   grid index of each support slot
    val: np.ndarray       # f64[total, 4] chi_s, chi_px, chi_py, chi_pz
    gamma: np.ndarray     # f64[n_atoms, 4]
    rev_offsets: np.ndarray  # i32[N_d + 1]
    rev_slot: np.ndarray     # i32[total]


def build(n: Sequence[int], h: float, origin: Sequence[float], periodic: bool,
          atoms: np.ndarray, proj: np.ndarray) -> ProjectorTables:
    """proj rows: (rc, width, gamma_s, gamma_px, gamma_py, gamma_pz)."""
    n = [int(x) for x in n]
    nd = n[0] * n[1] * n[2]
    xs = [np.float64(origin[a]) + np.arange(n[a], dtype=np.float64) * np.float64(h) for a in range(3)]
    L = [np.float64(n[a]) * np.float64(h) for a in range(3)]
    shifts = (-1, 0, 1) if periodic else (0,)
    offsets = [0]
    idx_all, val_all = [], []
    for a_i in range(len(atoms)):
        X = atoms[a_i]
        rc = np.float64(proj[a_i, 0])
        wd = np.float64(proj[a_i, 1])
        rc2 = rc * rc
        acc = {}
        for sz in shifts:
            for sy in shifts:
                for sx in shifts:
                    Xp = [X[0] + np.float64(sx) * L[0], X[1] + np.float64(sy) * L[1],
                          X[2] + np.float64(sz) * L[2]]
                    dx = xs[0] - Xp[0]
                    dy = xs[1] - Xp[1]
                    dz = xs[2] - Xp[2]
                    dx2 = dx * dx
                    dy2 = dy * dy
                    dz2 = dz * dz
                    r2 = (dx2[None, None, :] + dy2[None, :, None]) + dz2[:, None, None]
                    kk, jj, ii = np.nonzero(r2 < rc2)
                    if len(ii) == 0:
                        continue
                    rr = r2[kk, jj, ii]
                    f = np.exp(-rr / (2.0 * wd * wd))
                    vals = np.stack([f, dx[ii] * f, dy[jj] * f, dz[kk] * f], axis=1)
                    g = ii + n[0] * (jj + n[1] * kk)
                    for t in range(len(g)):
                        key = int(g[t])
                        if key in acc:
                            acc[key] = acc[key] + vals[t]
                        else:
                            acc[key] = vals[t].copy()
        gs = np.array(sorted(acc.keys()), dtype=np.int64)
        V = np.array([acc[int(g)] for g in gs]).reshape(-1, 4)
        for l in range(4):
            nrm2 = h ** 3 * np.sum(V[:, l] ** 2)
            if nrm2 > 0:
                V[:, l] = V[:, l] / np.sqrt(nrm2)
        idx_all.append(gs)
        val_all.append(V)
        offsets.append(offsets[-1] + len(gs))
    idx = np.concatenate(idx_all) if idx_all else np.zeros(0, dtype=np.int64)
    val = np.concatenate(val_all) if val_all else np.zeros((0, 4))
    total = len(idx)
    # reverse CSR over grid points: slots that cover each point, ascending slot
    counts = np.bincount(idx, minlength=nd) if total else np.zeros(nd, dtype=np.int64)
    rev_offsets = np.zeros(nd + 1, dtype=np.int64)
    rev_offsets[1:] = np.cumsum(counts)
    order = np.argsort(idx, kind="stable")   # stable: ascending slot within each point
    rev_slot = order
    return ProjectorTables(
        offsets=np.asarray(offsets, dtype=np.int32), idx=idx.astype(np.int32), val=val,
        gamma=np.asarray(proj[:, 2:6], dtype=np.float64).reshape(-1, 4),
        rev_offsets=rev_offsets.astype(np.int32), rev_slot=rev_slot.astype(np.int32))


def apply_vnl(t: ProjectorTables, psi: np.ndarray, h: float) -> np.ndarray:
    """V_nl psi = sum_j gamma_j chi_j (h^3 chi_j^T psi), psi (N_d, ncols)."""
    out = np.zeros_like(psi)
    h3 = h ** 3
    for a in range(len(t.offsets) - 1):
        s0, s1 = t.offsets[a], t.offsets[a + 1]
        if s1 == s0:
            continue
        S = t.idx[s0:s1]
        C = t.val[s0:s1]                       # (|S|, 4)
        alpha = h3 * (C.T @ psi[S, :])         # forward projection (4, ncols)
        alpha = t.gamma[a][:, None] * alpha    # gamma scaling
        out[S, :] += C @ alpha                 # backprojection
    return out


def dense_vnl(t: ProjectorTables, nd: int, h: float) -> np.ndarray:
    """Dense N_d x N_d matrix sum_j gamma_j h^3 chi_j chi_j^T (small grids only)."""
    M = np.zeros((nd, nd))
    for a in range(len(t.offsets) - 1):
        s0, s1 = t.offsets[a], t.offsets[a + 1]
        S = t.idx[s0:s1]
        for l in range(4):
            chi = np.zeros(nd)
            chi[S] = t.val[s0:s1, l]
            M += t.gamma[a, l] * h ** 3 * np.outer(chi, chi)
    return M
