"""Chebyshev-filtered subspace iteration, FP64 (oracle, test infrastructure only).

One CheFSI iteration on a subdomain (Sec. V-A.3, after Zhou et al. 2006):
  (1) filter     Psi_f = p_m(H) Psi, p_m(t) = C_m((t - c)/e), three-term recurrence;
  (2) projection H_s = Psi_f^T H Psi_f, M_s = Psi_f^T Psi_f;
  (3) dense      H_s y = lambda M_s y, solved as the paper's generalized
                 symmetric solver does (Sec. V-B.3): Cholesky M_s = R^T R,
                 C = R^-T H_s R^-1, C = Z Lambda Z^T, Y = R^-1 Z;
  (4) rotation   Psi = Psi_f Y.
The residual r_n = ||H psi_n - lambda_n psi_n||_2 gates convergence.

Readings where the paper is silent (each listed in the design notes):
* the filter is the scaled recurrence normalised so that p(a_0) = 1: the
  same polynomial as C_m((t-c)/e) up to a positive scalar, which keeps FP32
  from overflowing;  e = (lam_max - lam_c)/2, c = (lam_max + lam_c)/2;
* bounds: k-step Lanczos with full reorthogonalisation gives theta_min and
  the upper bound theta_max + |beta_k|; first iteration a_0 = theta_min,
  lam_c = a_0 + 0.1 (lam_max - a_0); later iterations a_0 = lambda_1 and
  lam_c = lambda_Ns of the previous iteration, lam_max kept;
* H_s is symmetrised as (H_s + H_s^T)/2, and so is C;
* Ritz values ascending; eigenvectors are never compared one by one.
Pins: Chebyshev closed form on a diagonal operator, Lanczos bound above
lambda_max, Rayleigh-Ritz invariants, brute-force eigh on 8^3 grids
(tests/test_oracle_chefsi.py).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla


class NotSPD(Exception):
    """The overlap matrix M_s = Psi_f^T Psi_f is not positive definite."""


# ---------------------------------------------------------------------------
# bounds
# ---------------------------------------------------------------------------

LANCZOS_BREAKDOWN = 1e-12   # beta_j below this fraction of max|T| ends the run


def lanczos(apply_H: Callable[[np.ndarray], np.ndarray], v0: np.ndarray, k: int = 20):
    """k steps of Lanczos with full reorthogonalisation from v0.

    Returns (alpha[k], beta[k], theta ascending) where beta[j] is the norm of
    the residual after step j; theta are the eigenvalues of T_k.  The run
    ends early when beta_j <= 1e-12 max(|alpha_i|, beta_i) (breakdown:
    the Krylov space is invariant); then the bound's |beta_k| term is that
    tiny last beta."""
    nd = v0.shape[0]
    k = int(min(k, nd))
    V = np.zeros((nd, k + 1))
    alpha = np.zeros(k)
    beta = np.zeros(k)
    V[:, 0] = v0 / np.linalg.norm(v0)
    for j in range(k):
        w = apply_H(V[:, j])
        alpha[j] = V[:, j] @ w
        w = w - alpha[j] * V[:, j]
        if j > 0:
            w = w - beta[j - 1] * V[:, j - 1]
        # full reorthogonalisation against every Lanczos vector so far
        w = w - V[:, :j + 1] @ (V[:, :j + 1].T @ w)
        beta[j] = np.linalg.norm(w)
        scale = max(np.max(np.abs(alpha[:j + 1])), np.max(beta[:j + 1]))
        if beta[j] <= LANCZOS_BREAKDOWN * scale:
            # invariant subspace found: T_j holds exact eigenvalues of H
            alpha = alpha[:j + 1]
            beta = beta[:j + 1]
            break
        V[:, j + 1] = w / beta[j]
    kk = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:kk - 1], 1) + np.diag(beta[:kk - 1], -1)
    theta = np.linalg.eigvalsh(T)
    return alpha, beta, theta


def lanczos_bounds(apply_H, v0: np.ndarray, k: int = 20):
    """(theta_min, upper bound theta_max + |beta_k|) of the spectrum of H."""
    _, beta, theta = lanczos(apply_H, v0, k)
    return float(theta[0]), float(theta[-1] + abs(beta[-1]))


def first_cutoff(a0: float, lam_max: float) -> float:
    return a0 + 0.1 * (lam_max - a0)


# ---------------------------------------------------------------------------
# filter
# ---------------------------------------------------------------------------

def filter_coefficients(m: int, a0: float, lam_c: float, lam_max: float):
    """Scalars of the scaled recurrence: (c, e, [sigma_1..sigma_m])."""
    e = (lam_max - lam_c) / 2.0
    c = (lam_max + lam_c) / 2.0
    sigma1 = e / (a0 - c)
    tau = 2.0 / sigma1
    sig = [sigma1]
    for _ in range(1, m):
        sig.append(1.0 / (tau - sig[-1]))
    return c, e, sig


def chebyshev_filter(apply_H, X: np.ndarray, m: int, a0: float, lam_c: float,
                     lam_max: float) -> np.ndarray:
    """Y_m = C_m((H - c)/e) X / C_m((a0 - c)/e) by the scaled three-term recurrence.

    Y_0 = X, Y_1 = (sigma_1/e)(H X - c X),
    Y_{k+1} = (2 sigma_{k+1}/e)(H Y_k - c Y_k) - sigma_k sigma_{k+1} Y_{k-1}."""
    if m < 1:
        raise ValueError("degree must be >= 1")
    c, e, sig = filter_coefficients(m, a0, lam_c, lam_max)
    Y0 = X
    Y1 = (sig[0] / e) * (apply_H(X) - c * X)
    for k in range(1, m):
        Y2 = (2.0 * sig[k] / e) * (apply_H(Y1) - c * Y1) - (sig[k - 1] * sig[k]) * Y0
        Y0, Y1 = Y1, Y2
    return Y1


def chebyshev_value(m: int, t: np.ndarray) -> np.ndarray:
    """C_m(t) by its closed form (cos / cosh), for pins."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    a = np.abs(t) <= 1
    out[a] = np.cos(m * np.arccos(t[a]))
    b = t > 1
    out[b] = np.cosh(m * np.arccosh(t[b]))
    c = t < -1
    out[c] = (-1.0) ** m * np.cosh(m * np.arccosh(-t[c]))
    return out


# ---------------------------------------------------------------------------
# Rayleigh-Ritz
# ---------------------------------------------------------------------------

def rayleigh_ritz(apply_H, Psi_f: np.ndarray):
    """Steps (2)-(4): returns (ritz ascending, Psi rotated, Y, M_s, H_s)."""
    W = apply_H(Psi_f)
    M = Psi_f.T @ Psi_f
    Hs = Psi_f.T @ W
    Hs = 0.5 * (Hs + Hs.T)
    lam, Y = generalized_eigh(Hs, M)
    Psi = Psi_f @ Y
    return lam, Psi, Y, M, Hs


def generalized_eigh(Hs: np.ndarray, M: np.ndarray):
    """H_s y = lambda M y via Cholesky M = R^T R, C = R^-T H_s R^-1, eigh, Y = R^-1 Z.

    Raises NotSPD when a Cholesky pivot is <= n * eps * M_kk (not positive
    definite, or numerically singular, e.g. duplicated columns)."""
    try:
        R = sla.cholesky(M, lower=False)
    except np.linalg.LinAlgError as exc:
        raise NotSPD(str(exc)) from exc
    # a pivot R_kk^2 at or below n*eps*M_kk is numerically zero: M is singular
    n = M.shape[0]
    piv = np.diag(R) ** 2
    if np.any(piv <= n * np.finfo(np.float64).eps * np.diag(M)):
        raise NotSPD("numerically singular overlap matrix")
    A = sla.solve_triangular(R, Hs, trans="T", lower=False)        # R^-T H_s
    C = sla.solve_triangular(R, A.T, trans="T", lower=False).T     # (R^-T H_s) R^-1
    C = 0.5 * (C + C.T)
    lam, Z = np.linalg.eigh(C)
    Y = sla.solve_triangular(R, Z, lower=False)                    # R^-1 Z
    return lam, Y


def residuals(apply_H, Psi: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """r_n = ||H psi_n - lambda_n psi_n||_2."""
    R = apply_H(Psi) - Psi * lam[None, :]
    return np.sqrt(np.sum(R * R, axis=0))


# ---------------------------------------------------------------------------
# the iteration
# ---------------------------------------------------------------------------

@dataclass
class ChefsiResult:
    ritz: np.ndarray
    resid: np.ndarray
    psi: np.ndarray
    iters: int
    history: List[np.ndarray] = field(default_factory=list)
    bounds: List[tuple] = field(default_factory=list)


def n_gate(ns: int) -> int:
    """Number of states the convergence gate covers: floor(ns / 1.1), at least 1."""
    return max(1, int(np.floor(ns / 1.1 + 1e-9)))


def chefsi(apply_H, X0: np.ndarray, degree: int, max_iter: int, lam_lo: float,
           lam_cut: float, lam_max: float, resid_tol: float = 0.0,
           gate: Optional[int] = None) -> ChefsiResult:
    """Run up to max_iter CheFSI iterations from X0 with first-iteration bounds
    (lam_lo, lam_cut, lam_max); later iterations use a_0 = lambda_1 and
    lam_c = lambda_Ns of the previous iteration.  Stops early when the
    largest residual over the lowest `gate` states is <= resid_tol."""
    ns = X0.shape[1]
    gate = n_gate(ns) if gate is None else gate
    Psi = np.array(X0, dtype=np.float64, order="F")
    a0, lc = float(lam_lo), float(lam_cut)
    res = ChefsiResult(np.zeros(ns), np.zeros(ns), Psi, 0)
    for it in range(max_iter):
        res.bounds.append((a0, lc, float(lam_max)))
        Pf = chebyshev_filter(apply_H, Psi, degree, a0, lc, lam_max)
        lam, Psi, _, _, _ = rayleigh_ritz(apply_H, Pf)
        r = residuals(apply_H, Psi, lam)
        res.history.append(lam.copy())
        res.ritz, res.resid, res.psi, res.iters = lam, r, Psi, it + 1
        a0, lc = float(lam[0]), float(lam[-1])
        if resid_tol > 0 and np.max(r[:gate]) <= resid_tol:
            break
    return res


def subspace_sin_theta(Qa: np.ndarray, Qb: np.ndarray) -> float:
    """sin of the largest principal angle between span(Qa) and span(Qb).

    Both are orthonormalised first; returns ||Qa - Qb (Qb^T Qa)||_2."""
    A, _ = np.linalg.qr(Qa)
    B, _ = np.linalg.qr(Qb)
    D = A - B @ (B.T @ A)
    return float(np.linalg.norm(D, 2)) if D.size else 0.0
