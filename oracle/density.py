"""Subdomain observables (oracle, test infrastructure only).

* g(lambda; mu, sigma) = 1 / (1 + exp((lambda - mu)/sigma)), the
  Fermi-Dirac occupation (Sec. V-A.1, eq. (dm)); evaluated as
  exp(-t)/(1 + exp(-t)) for t > 0 so that it never overflows.
* rho~(x) = 2 sum_n g_n |psi_n(x)|^2 restricted to the core by p^alpha
  (Sec. V-A.4, eq. (density)); with unit 2-norm columns the continuum
  |psi|^2 is psi_g^2 / h^3, so rho~_g = (2/h^3) sum_n g_n psi_{g,n}^2.
* interior weights c_n = int_core |psi_n|^2 = sum_{g in core} psi_{g,n}^2
  (Sec. V-A.4).
* E_band = 2 sum g c lambda, E_entropy = -2 sigma sum c s(lambda) with
  s = g log g + (1 - g) log(1 - g), DOS D(E) = 2 sum c delta(E - lambda)
  (Sec. V-A.4), and the electron count N_e(mu) = 2 sum g c (Sec. V-A.5).
* the Fermi level mu of a set of subsystems: the root of
  N_e(mu) = n_electrons over all their states (Sec. V-A.5); N_e is continuous
  and strictly increasing in mu, so plain bisection finds it.
* the global density: every subsystem's core density placed at its global
  grid points and summed (Sec. V-A.4; the cores partition the global grid).
Pins: charge identity h^3 sum rho~ = 2 sum g c, c = 1 for a whole-box
core, the sigma -> 0 limit, the Fermi level of a spectrum symmetric about
mu0 at half filling (exactly mu0), assembly against a point-by-point loop
(tests/test_oracle_density.py).
"""
from __future__ import annotations

import numpy as np


def fermi(lam: np.ndarray, mu: float, sigma: float) -> np.ndarray:
    t = (np.asarray(lam, dtype=np.float64) - mu) / sigma
    out = np.empty_like(t)
    pos = t > 0
    ep = np.exp(-t[pos])
    out[pos] = ep / (1.0 + ep)
    out[~pos] = 1.0 / (1.0 + np.exp(t[~pos]))
    return out


def core_density(psi: np.ndarray, lam: np.ndarray, mu: float, sigma: float, mask: np.ndarray,
                 h: float):
    """(rho~ on core points, zero elsewhere; c_n)."""
    g = fermi(lam, mu, sigma)
    sq = psi * psi
    core = mask.astype(bool)
    rho = np.zeros(psi.shape[0])
    rho[core] = (2.0 / h ** 3) * (sq[core, :] @ g)
    c = np.sum(sq[core, :], axis=0)
    return rho, c


def band_energy(lam, c, mu, sigma) -> float:
    g = fermi(lam, mu, sigma)
    return float(2.0 * np.sum(g * c * lam))


def entropy_energy(lam, c, mu, sigma) -> float:
    g = fermi(lam, mu, sigma)
    with np.errstate(divide="ignore", invalid="ignore"):
        s = np.where(g > 0, g * np.log(g), 0.0) + np.where(g < 1, (1 - g) * np.log1p(-g), 0.0)
    return float(-2.0 * sigma * np.sum(c * s))


def electron_count(lam, c, mu, sigma) -> float:
    return float(2.0 * np.sum(fermi(lam, mu, sigma) * c))


def dos_histogram(lam, c, edges) -> np.ndarray:
    """D(E) binned: 2 sum_n c_n over eigenvalues falling in each bin."""
    hist, _ = np.histogram(np.asarray(lam), bins=np.asarray(edges), weights=2.0 * np.asarray(c))
    return hist


def fermi_level(lam, c, sigma: float, n_electrons: float) -> float:
    """mu with electron_count(lam, c, mu, sigma) = n_electrons, by bisection on
    [min lam - 40 sigma, max lam + 40 sigma] until the midpoint no longer
    splits the bracket.  ValueError when the count is out of reach."""
    lam = np.asarray(lam, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    lo = float(lam.min()) - 40.0 * sigma
    hi = float(lam.max()) + 40.0 * sigma
    if not (electron_count(lam, c, lo, sigma) < n_electrons < electron_count(lam, c, hi, sigma)):
        raise ValueError("electron count outside (N_e(lo), N_e(hi))")
    while True:
        mid = 0.5 * (lo + hi)
        if not (lo < mid < hi):
            return mid
        if electron_count(lam, c, mid, sigma) < n_electrons:
            lo = mid
        else:
            hi = mid


def assemble_density(parts, n_global: int) -> np.ndarray:
    """sum over subsystems of rho~ on their core points, placed by their
    local->global maps: parts is a sequence of (rho_local, core_mask,
    global_index)."""
    rho = np.zeros(int(n_global))
    for r, mask, gidx in parts:
        core = np.asarray(mask).astype(bool)
        np.add.at(rho, np.asarray(gidx)[core], np.asarray(r)[core])
    return rho
