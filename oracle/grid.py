"""Grid-level pieces of the oracle (test infrastructure only).

* FD weights of the central 2*n0-order second derivative (Sec. V-B.2:
  the stencil uses fixed coefficients w_0..w_n0 with n0 = 6).
* The 3-D Laplacian as the sum of 1-D stencils along x, y, z (Sec. V-B.2,
  36 neighbour terms plus the centre), periodic or zero-Dirichlet.
* The binary partition of unity p^alpha as a core mask and the
  local->global grid map of a buffered subdomain (Sec. V-A.2).

Conventions: Hartree units, isotropic spacing h, node (i, j, k) sits at
origin + h*(i, j, k), linear index g = i + n0*(j + n1*k).
Pins: exact rationals, polynomial exactness, plane-wave closed form,
Kronecker-sum assembly, tiling of a periodic grid (tests/test_oracle_grid.py).
"""
from __future__ import annotations

from fractions import Fraction
from math import factorial
from typing import Sequence, Tuple

import numpy as np


def fd_weights_exact(n0: int) -> list:
    """Central 2*n0-order weights of d^2/dx^2 as exact rationals [w_0, ..., w_n0].

    w_p = 2 (-1)^(p+1) (n0!)^2 / (p^2 (n0-p)! (n0+p)!) for p >= 1 and
    w_0 = -2 sum_p w_p (the stencil annihilates constants)."""
    if n0 < 1:
        raise ValueError("n0 must be >= 1")
    w = [Fraction(0)]
    for p in range(1, n0 + 1):
        w.append(Fraction(2 * (-1) ** (p + 1) * factorial(n0) ** 2,
                          p * p * factorial(n0 - p) * factorial(n0 + p)))
    w[0] = -2 * sum(w[1:])
    return w


def fd_weights(n0: int) -> np.ndarray:
    return np.array([float(x) for x in fd_weights_exact(n0)])


def _shift(a: np.ndarray, p: int, axis: int, periodic: bool) -> np.ndarray:
    """b[..., i, ...] = a[..., i + p, ...]; zero outside the box when not periodic."""
    n = a.shape[axis]
    if periodic:
        idx = np.mod(np.arange(n) + p, n)
        return np.take(a, idx, axis=axis)
    b = np.zeros_like(a)
    src = [slice(None)] * a.ndim
    dst = [slice(None)] * a.ndim
    if p >= n or -p >= n:
        return b
    if p >= 0:
        src[axis] = slice(p, n)
        dst[axis] = slice(0, n - p)
    else:
        src[axis] = slice(0, n + p)
        dst[axis] = slice(-p, n)
    b[tuple(dst)] = a[tuple(src)]
    return b


def laplacian(psi: np.ndarray, n: Sequence[int], h: float, periodic: bool, n0: int = 6) -> np.ndarray:
    """(L psi)_g = h^-2 [3 w_0 psi_g + sum_p w_p sum_axes (psi_{g+p e_a} + psi_{g-p e_a})].

    psi: (N_d,) or (N_d, ncols) with g = i + n0*(j + n1*k)."""
    w = fd_weights(n0)
    squeeze = psi.ndim == 1
    X = psi.reshape(-1, 1) if squeeze else psi
    ncols = X.shape[1]
    A = X.reshape((n[0], n[1], n[2], ncols), order="F")
    out = 3.0 * w[0] * A
    for axis in range(3):
        for p in range(1, n0 + 1):
            out = out + w[p] * (_shift(A, p, axis, periodic) + _shift(A, -p, axis, periodic))
    out = out / (h * h)
    out = out.reshape((-1, ncols), order="F")
    return out[:, 0] if squeeze else out


def core_mask(n: Sequence[int], core_lo: Sequence[int], core_hi: Sequence[int]) -> np.ndarray:
    """p^alpha as u8[N_d]: 1 on the half-open index box [core_lo, core_hi)."""
    i = np.arange(n[0])
    j = np.arange(n[1])
    k = np.arange(n[2])
    mi = (i >= core_lo[0]) & (i < core_hi[0])
    mj = (j >= core_lo[1]) & (j < core_hi[1])
    mk = (k >= core_lo[2]) & (k < core_hi[2])
    m = mk[:, None, None] & mj[None, :, None] & mi[None, None, :]
    return m.reshape(-1).astype(np.uint8)


def global_index(n: Sequence[int], global_offset: Sequence[int], global_n: Sequence[int]) -> np.ndarray:
    """i64[N_d]: global linear index of each local node, periodic wrap of the global grid."""
    gi = np.mod(global_offset[0] + np.arange(n[0], dtype=np.int64), global_n[0])
    gj = np.mod(global_offset[1] + np.arange(n[1], dtype=np.int64), global_n[1])
    gk = np.mod(global_offset[2] + np.arange(n[2], dtype=np.int64), global_n[2])
    G = gi[None, None, :] + global_n[0] * (gj[None, :, None] + global_n[1] * gk[:, None, None])
    return G.reshape(-1).astype(np.int64)


def laplacian_symbol(theta: np.ndarray, n0: int = 6) -> np.ndarray:
    """s(theta) = -w_0 - 2 sum_p w_p cos(p theta): eigenvalue of -h^2 d^2/dx^2 on a plane wave."""
    w = fd_weights(n0)
    s = -w[0] * np.ones_like(theta)
    for p in range(1, n0 + 1):
        s = s - 2.0 * w[p] * np.cos(p * theta)
    return s


def grid_shape(sd) -> Tuple[int, int, int]:
    return tuple(int(x) for x in sd.n)
