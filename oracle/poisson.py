"""Electrostatic Poisson solve by multigrid-preconditioned CG (oracle, test
infrastructure only).

The paper obtains the electrostatic potential from -(1/(4 pi)) Lap phi =
rho + b (the Poisson equation of Sec. IV, pseudocharges b), discretised with
the same 2 n0-order FD Laplacian as the Hamiltonian, zero-Dirichlet or
periodic, and solved by CG preconditioned with a structured algebraic
multigrid V-cycle whose finest level replaces the wide operator by the
7-point (3D7) Laplacian, applied matrix-free; the V-cycle runs in FP32 and
the CG in FP64 (Sec. V-B.1).

Discrete problem: A phi = 4 pi f with A = -L (L the 12th-order Laplacian of
grid.laplacian), so A is symmetric positive definite (Dirichlet) or positive
semi-definite with the constants as null space (periodic: f and phi are
taken with zero mean).

Preconditioner, one V-cycle (this oracle runs it in FP64):
* level 0: A_0 = the 7-point operator (6 u_g - sum of the 6 neighbours)/h^2;
* coarsening by 2 per axis: zero-Dirichlet sizes n -> (n - 1)/2 (n odd;
  coarse point I sits on fine point 2I + 1), periodic n -> n/2 (n even;
  coarse I on fine 2I); levels are added while every axis coarsens exactly
  to at least 3 (Dirichlet) or 4 (periodic) points, up to max_levels;
* P: trilinear prolongation (weight 1 on the coincident fine point, 1/2 on
  its axis neighbours, products across axes; zero beyond a Dirichlet face,
  wrapped when periodic), restriction P^T, coarse operators Galerkin
  A_{l+1} = P^T A_l P (sparse matrix products here);
* smoothing: nu sweeps of damped Jacobi x <- x + omega D^-1 (r - A x),
  omega = 2/3, before and after the coarse correction; on the coarsest level
  nu_c sweeps from zero stand in for the solve.  Zero start and equal pre-
  and post-smoothing make the V-cycle a symmetric operator.
CG: x_0 = 0, stop when ||r|| <= tol ||4 pi f|| (2-norms).
Pins (tests/test_oracle_poisson.py): the periodic solution against the FFT
closed form of the 12th-order symbol, the Dirichlet solution against a
sparse direct solve, the 7-point and Galerkin operators against their
closed-form stencils, the V-cycle's symmetry and positivity on a small grid.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np
import scipy.sparse as sp

from . import grid

OMEGA = 2.0 / 3.0


def apply_A(u: np.ndarray, n: Sequence[int], h: float, periodic: bool) -> np.ndarray:
    """A u = -L u with the 12th-order Laplacian."""
    return -grid.laplacian(u, n, h, periodic)


def _lap7_1d(m: int, periodic: bool) -> sp.csr_matrix:
    """1-D second difference -d^2 (unscaled): 2 on the diagonal, -1 off it."""
    T = sp.diags([-np.ones(m - 1), 2.0 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1], format="lil")
    if periodic and m > 2:
        T[0, m - 1] = -1.0
        T[m - 1, 0] = -1.0
    return T.tocsr()


def lap7_matrix(n: Sequence[int], h: float, periodic: bool) -> sp.csr_matrix:
    """A_0 = (T_x (+) T_y (+) T_z) / h^2 with g = i + n0 (j + n1 k) (x fastest)."""
    Tx, Ty, Tz = (_lap7_1d(int(m), periodic) for m in n)
    Ix, Iy, Iz = (sp.identity(int(m), format="csr") for m in n)
    A = sp.kron(Iz, sp.kron(Iy, Tx)) + sp.kron(Iz, sp.kron(Ty, Ix)) + sp.kron(Tz, sp.kron(Iy, Ix))
    return (A / (h * h)).tocsr()


def coarse_size(m: int, periodic: bool):
    """Size of the next level along an axis, or None if it does not coarsen exactly."""
    if periodic:
        return m // 2 if m % 2 == 0 and m // 2 >= 4 else None
    return (m - 1) // 2 if m % 2 == 1 and (m - 1) // 2 >= 3 else None


def _prolong_1d(mf: int, mc: int, periodic: bool) -> sp.csr_matrix:
    P = sp.lil_matrix((mf, mc))
    for I in range(mc):
        c = 2 * I if periodic else 2 * I + 1
        P[c, I] = 1.0
        for d in (-1, 1):
            f = c + d
            if periodic:
                P[f % mf, I] += 0.5
            elif 0 <= f < mf:
                P[f, I] += 0.5
    return P.tocsr()


def prolongation(nf: Sequence[int], nc: Sequence[int], periodic: bool) -> sp.csr_matrix:
    Px, Py, Pz = (_prolong_1d(int(a), int(b), periodic) for a, b in zip(nf, nc))
    return sp.kron(Pz, sp.kron(Py, Px)).tocsr()


@dataclass
class Hierarchy:
    sizes: List[tuple]
    A: List[sp.csr_matrix]
    P: List[sp.csr_matrix]          # P[l]: level l+1 -> level l
    Dinv: List[np.ndarray] = field(default_factory=list)


def hierarchy(n: Sequence[int], h: float, periodic: bool, max_levels: int = 8) -> Hierarchy:
    sizes = [tuple(int(m) for m in n)]
    A = [lap7_matrix(n, h, periodic)]
    P = []
    while len(sizes) < max_levels:
        nc = [coarse_size(m, periodic) for m in sizes[-1]]
        if any(c is None for c in nc):
            break
        Pl = prolongation(sizes[-1], nc, periodic)
        P.append(Pl)
        A.append((Pl.T @ A[-1] @ Pl).tocsr())
        sizes.append(tuple(nc))
    H = Hierarchy(sizes, A, P)
    H.Dinv = [1.0 / Al.diagonal() for Al in A]
    return H


def vcycle(H: Hierarchy, r: np.ndarray, nu: int = 2, nu_coarse: int = 10, level: int = 0) -> np.ndarray:
    A, Dinv = H.A[level], H.Dinv[level]
    x = np.zeros_like(r)
    if level == len(H.A) - 1:
        for _ in range(nu_coarse):
            x = x + OMEGA * Dinv * (r - A @ x)
        return x
    for _ in range(nu):
        x = x + OMEGA * Dinv * (r - A @ x)
    rc = H.P[level].T @ (r - A @ x)
    x = x + H.P[level] @ vcycle(H, rc, nu, nu_coarse, level + 1)
    for _ in range(nu):
        x = x + OMEGA * Dinv * (r - A @ x)
    return x


@dataclass
class PoissonResult:
    phi: np.ndarray
    iters: int
    rel_resid: float
    history: List[float]


def solve(f: np.ndarray, n: Sequence[int], h: float, periodic: bool, tol: float = 1e-10,
          max_iter: int = 2000, precondition: bool = True, max_levels: int = 8, nu: int = 2,
          nu_coarse: int = 10) -> PoissonResult:
    """phi with -(1/(4 pi)) L phi = f by (preconditioned) CG from zero."""
    b = 4.0 * np.pi * np.asarray(f, dtype=np.float64)
    if periodic:
        b = b - b.mean()
    H = hierarchy(n, h, periodic, max_levels) if precondition else None

    def prec(r):
        if H is None:
            return r.copy()
        z = vcycle(H, r, nu, nu_coarse)
        return z - z.mean() if periodic else z

    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    hist = [1.0]
    if nb == 0.0:
        return PoissonResult(x, 0, 0.0, hist)
    z = prec(r)
    p = z.copy()
    rz = r @ z
    it = 0
    for it in range(1, max_iter + 1):
        Ap = apply_A(p, n, h, periodic)
        alpha = rz / (p @ Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        hist.append(float(np.linalg.norm(r) / nb))
        if hist[-1] <= tol:
            break
        z = prec(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    if periodic:
        x = x - x.mean()
    return PoissonResult(x, it, hist[-1], hist)
