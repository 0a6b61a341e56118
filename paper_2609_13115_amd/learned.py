"""Learned filter bounds: labels from the method, GPU training, prediction.

The paper leaves the source of the Chebyshev filter bounds open (it defines
the filter by its centre c and half-width e, Sec. V-A.3).  This module trains
the library's MLP (xls_mlp_*; FP32 forward/backward/Adam kernels, bfloat16
inference) to predict a subdomain's (lambda_max, lambda_cut, degree) from the
64 features of xls_subdomain_features, with labels the method itself
produces:

* lambda_max: the k = 20 Lanczos upper bound theta_max + |beta_k|;
* lambda_cut: lambda_ns of a converged CheFSI run with Lanczos bounds and
  degree 24 (the last iteration's if it did not converge);
* degree: among the m in DEGREES whose run with the bounds a learned run
  would take from exact labels (lambda_max padded, lambda_cut as above)
  reaches the residual gate within max_iter iterations, the one with the least
  filter work m * iterations (ties: smaller m).

A learned run takes the bounds xls_mlp_bounds returns: the predicted
lambda_max raised by a margin (an estimate below the true top of the
spectrum makes the Chebyshev polynomial grow there), the predicted
lambda_cut raised by three times the model's RMS error on its training rows
(a cutoff below the true lambda_ns damps the highest wanted states; the
plain method's later cutoffs, Ritz values, are upper bounds for the same
reason) and the predicted degree rounded into [16, 32]; a0 is the library's
rigorous lower bound, and the run falls back to Lanczos bounds (same start
block) when its gated residual misses the gate.  Standardisation, training,
the RMS error, the margins and the degree rule all live in the library
(xls_mlp_fit, xls_mlp_bounds, xls_learned_safe_bounds); this module only
orchestrates calls and picks the degree labels.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

from . import xls

DEGREES = (16, 20, 24, 28, 32)
SIZES = (64, 128, 128, 3)


@dataclasses.dataclass
class Labels:
    features: np.ndarray      # (n, 64)
    targets: np.ndarray       # (n, 3): lambda_max, lambda_cut, degree
    converged: np.ndarray     # (n,) bool: some degree reached the gate
    work: np.ndarray          # (n, len(DEGREES)): H applications per degree trial (0: not run)


def batch_features(b: "xls.Batch") -> np.ndarray:
    return np.stack([b.xls_batch_subdomain(i).xls_subdomain_features() for i in range(b.n)])


def label_subdomains(sds: Sequence, filter_prec: int = xls.XLS_PREC_FP32,
                     gemm_prec: int = xls.XLS_PREC_FP32, tol: float = 1e-4, max_iter: int = 12,
                     degrees: Sequence[int] = DEGREES, lanczos_k: int = 20) -> Labels:
    """Labels of the training boxes, computed with the batch engine (start
    blocks drawn on the device for boxes without a host x0)."""
    from . import workloads

    n = len(sds)
    seeds = None if all(sd.x0 is not None for sd in sds) else [workloads.x0_seed(sd.seed_key) for sd in sds]

    def batch():
        return xls.Batch(list(sds), filter_prec=filter_prec, x0_seeds=seeds)

    with batch() as b:
        F = batch_features(b)
        lmax = np.array([b.xls_batch_subdomain(i).xls_lanczos_bounds(lanczos_k)[1] for i in range(n)])
    params = [xls.chefsi_params(24, max_iter, xls.XLS_BOUNDS_LANCZOS, resid_tol=tol, lanczos_k=lanczos_k,
                                gemm_prec=gemm_prec) for _ in range(n)]
    with batch() as b:
        ritz, _, _, _ = b.xls_batch_chefsi(params)
    cut = np.array([r[-1] for r in ritz])
    ok_all = np.zeros((n, len(degrees)), dtype=bool)
    work = np.zeros((n, len(degrees)))
    lm_safe, lc_safe = xls.xls_learned_safe_bounds(lmax, cut)
    for j, m in enumerate(degrees):
        params = [xls.chefsi_params(m, max_iter, xls.XLS_BOUNDS_LEARNED, lam_cut=float(lc_safe[i]),
                                    lam_max=float(lm_safe[i]), resid_tol=tol, gemm_prec=gemm_prec)
                  for i in range(n)]
        with batch() as b:
            _, resid, iters, status = b.xls_batch_chefsi(params)
        for i, sd in enumerate(sds):
            gate = max(1, int(np.floor(sd.ns / 1.1 + 1e-9)))
            ok_all[i, j] = status[i] == xls.XLS_OK and float(np.max(resid[i][:gate])) <= tol
            work[i, j] = m * iters[i]
    conv = ok_all.any(axis=1)
    best_m = np.full(n, float(degrees[-1]))
    for i in range(n):
        if conv[i]:
            j = min(range(len(degrees)), key=lambda j: (not ok_all[i, j], work[i, j], degrees[j]))
            best_m[i] = degrees[j]
    T = np.stack([lmax, cut, best_m], axis=1)
    return Labels(F, T, conv, work)


def train_model(F: np.ndarray, T: np.ndarray, epochs: int = 400, batch: int = 16, lr: float = 1e-3,
                seed: int = 0, model: Optional["xls.Mlp"] = None):
    """Fits the library MLP (xls_mlp_fit: the library standardises features
    and targets and keeps its training RMS error); returns (model, per-step
    losses).  Minibatch order and initial weights come from the seeded
    workload generators."""
    from . import workloads

    if model is None:
        model = xls.Mlp(SIZES, workloads.mlp_init(SIZES, seed))
    order = workloads.minibatch_order(len(F), batch, epochs, seed)
    losses = model.fit(F, T, order, lr)
    return model, losses


def learned_params(lmax: float, lcut: float, degree: int, max_iter: int = 12, tol: float = 1e-4,
                   fallback_degree: int = 24, gemm_prec: int = xls.XLS_PREC_FP32):
    return xls.chefsi_params(int(degree), max_iter, xls.XLS_BOUNDS_LEARNED, lam_cut=float(lcut),
                             lam_max=float(lmax), resid_tol=tol, gemm_prec=gemm_prec, fallback_tol=tol,
                             fallback_degree=fallback_degree)


def batch_learned_params(model: "xls.Mlp", F: np.ndarray, max_iter: int = 30, tol: float = 1e-4,
                         gemm_prec: int = xls.XLS_PREC_BF16X3, fallback: bool = True,
                         fallback_degree: int = 24) -> list:
    """Per-subdomain learned parameters for a batch: xls_mlp_bounds, with the
    Lanczos fallback at the gate tolerance."""
    lmax, lcut, deg = model.bounds(F)
    return [xls.chefsi_params(int(m), max_iter, xls.XLS_BOUNDS_LEARNED, lam_cut=float(lc), lam_max=float(lm),
                              resid_tol=tol, gemm_prec=gemm_prec, fallback_tol=tol if fallback else 0.0,
                              fallback_degree=fallback_degree)
            for lm, lc, m in zip(lmax, lcut, deg)]


@dataclasses.dataclass
class RunStats:
    h_applies: int
    iterations: int
    fallbacks: int
    gated_max_resid: List[float]
    seconds: float


def run_learned(sds: Sequence, model: "xls.Mlp", filter_prec: int = xls.XLS_PREC_FP32,
                gemm_prec: int = xls.XLS_PREC_FP32, tol: float = 1e-4, max_iter: int = 12,
                fallback_degree: int = 24) -> RunStats:
    """Learned bounds on each subdomain (features -> bf16 MLP -> CheFSI with
    Lanczos fallback)."""
    import time

    hs, its, fbs, res = 0, 0, 0, []
    t = 0.0
    for sd in sds:
        with xls.Subdomain(sd, filter_prec=filter_prec) as s:
            t0 = time.perf_counter()
            lmax, lcut, deg = model.bounds(s.xls_subdomain_features())
            p = learned_params(lmax[0], lcut[0], int(deg[0]), max_iter, tol, fallback_degree, gemm_prec)
            ritz, resid, it = s.xls_chefsi_step(p.degree, p.max_iter, p.bounds_mode, p.lam_lo, p.lam_cut,
                                                p.lam_max, p.resid_tol, 0, 20, p.gemm_prec, p.fallback_tol,
                                                p.fallback_degree)
            t += time.perf_counter() - t0
            c = s.xls_subdomain_counters()
            gate = max(1, int(np.floor(sd.ns / 1.1 + 1e-9)))
            hs += c["h_applies"]
            its += c["iterations"]
            fbs += int(c["fallback"])
            res.append(float(np.max(resid[:gate])))
    return RunStats(hs, its, fbs, res, t)


def run_lanczos(sds: Sequence, degree: int = 24, filter_prec: int = xls.XLS_PREC_FP32,
                gemm_prec: int = xls.XLS_PREC_FP32, tol: float = 1e-4, max_iter: int = 12) -> RunStats:
    """The plain method: Lanczos bounds and a fixed degree."""
    import time

    hs, its, res = 0, 0, []
    t = 0.0
    for sd in sds:
        with xls.Subdomain(sd, filter_prec=filter_prec) as s:
            t0 = time.perf_counter()
            ritz, resid, it = s.xls_chefsi_step(degree, max_iter, xls.XLS_BOUNDS_LANCZOS, resid_tol=tol,
                                                gemm_prec=gemm_prec)
            t += time.perf_counter() - t0
            c = s.xls_subdomain_counters()
            gate = max(1, int(np.floor(sd.ns / 1.1 + 1e-9)))
            hs += c["h_applies"]
            its += c["iterations"]
            res.append(float(np.max(resid[:gate])))
    return RunStats(hs, its, 0, res, t)
