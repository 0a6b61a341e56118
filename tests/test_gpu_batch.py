"""Batch engine on the GPU, through the C ABI.

The batch path (grouped persistent filter launches, per-subdomain tails on a
stream pool, hipGraph capture and replay, device-side filter coefficients)
must give bit-identical results to running each subdomain alone through
xls_chefsi_step, which the parity suite checks against the oracle; one FP64
batch is also checked against the oracle directly.
"""
import json
import os

import numpy as np
import pytest

from oracle import chefsi, hamiltonian
from paper_2609_13115_amd import workloads, xls

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[case] {msg}", flush=True)


def uneven_boxes():
    """Three uneven subdomains: two ragged zero-Dirichlet boxes and a periodic cell."""
    return [
        workloads.small_dirichlet(ns=10, index=1, shape=(13, 9, 20), h=0.6),
        workloads.small_dirichlet(ns=6, index=2, shape=(16, 16, 12), h=0.6),
        workloads.small_periodic(n=12, ns=8, index=3),
    ]


def single_runs(sds, prec, params):
    out = []
    for sd, p in zip(sds, params):
        with xls.Subdomain(sd, filter_prec=prec) as s:
            r = s.xls_chefsi_step(p.degree, p.max_iter, p.bounds_mode, p.lam_lo, p.lam_cut, p.lam_max,
                                  p.resid_tol, p.n_gate, p.lanczos_k, p.gemm_prec)
            out.append(r + (s.xls_subdomain_get_block(),))
    return out


def batch_run(sds, prec, params, use_graph=True):
    with xls.Batch(sds, filter_prec=prec) as b:
        ritz, resid, iters, status = b.xls_batch_chefsi(params, use_graph=use_graph)
        blocks = [b.xls_batch_subdomain(i).xls_subdomain_get_block() for i in range(len(sds))]
        stats = b.xls_batch_stats()
    return ritz, resid, iters, status, blocks, stats


def assert_same(single, batch):
    ritz, resid, iters, status, blocks, _ = batch
    for i, (r, e, it, blk) in enumerate(single):
        assert status[i] == xls.XLS_OK
        assert iters[i] == it, (i, iters[i], it)
        assert np.array_equal(ritz[i], r), (i, np.max(np.abs(ritz[i] - r)))
        assert np.array_equal(resid[i], e), (i, np.max(np.abs(resid[i] - e)))
        assert np.array_equal(blocks[i], blk), i


@pytest.mark.parametrize("prec,gprec", [(xls.XLS_PREC_FP64, xls.XLS_PREC_FP64),
                                        (xls.XLS_PREC_FP32, xls.XLS_PREC_FP32),
                                        (xls.XLS_PREC_FP32, xls.XLS_PREC_BF16X3)])
def test_batch_bitexact_vs_single(prec, gprec):
    case(f"batch vs single prec={prec} gemm={gprec}")
    sds = uneven_boxes()
    params = [xls.chefsi_params(d, 4, xls.XLS_BOUNDS_LANCZOS, gemm_prec=gprec) for d in (7, 10, 12)]
    single = single_runs(sds, prec, params)
    eager = batch_run(sds, prec, params, use_graph=False)
    assert_same(single, eager)
    graph = batch_run(sds, prec, params, use_graph=True)
    assert_same(single, graph)
    st = graph[5]
    assert st["iterations"] == 4 and st["captures"] >= 1 and st["replays"] >= 1, st


def test_batch_early_stop_changes_active_set():
    """Different convergence per subdomain: the active set shrinks and the
    captured graph is rebuilt; results still match the single path."""
    case("batch early stop")
    sds = uneven_boxes()
    params = [xls.chefsi_params(d, 9, xls.XLS_BOUNDS_LANCZOS, resid_tol=tol)
              for d, tol in ((12, 1e-3), (8, 1e-6), (10, 3e-2))]
    single = single_runs(sds, xls.XLS_PREC_FP64, params)
    assert len({it for _, _, it, _ in single}) > 1, [it for _, _, it, _ in single]
    assert_same(single, batch_run(sds, xls.XLS_PREC_FP64, params))


def test_batch_fp64_vs_oracle():
    case("batch fp64 vs oracle")
    sds = [workloads.small_dirichlet(ns=8, index=5), workloads.small_periodic(n=8, ns=6, index=6)]
    degs = (9, 12)
    params = [xls.chefsi_params(d, 5, xls.XLS_BOUNDS_LANCZOS) for d in degs]
    ritz, resid, iters, status, _, _ = batch_run(sds, xls.XLS_PREC_FP64, params)
    for i, (sd, m) in enumerate(zip(sds, degs)):
        op = hamiltonian.from_subdomain(sd)
        lo, up = chefsi.lanczos_bounds(op.apply, sd.lanczos_v0, 20)
        ref = chefsi.chefsi(op.apply, sd.x0, m, 5, lo, chefsi.first_cutoff(lo, up), up)
        assert iters[i] == 5
        assert np.max(np.abs(ritz[i] - ref.ritz) / np.maximum(np.abs(ref.ritz), 1e-2)) <= 1e-10
        assert np.max(np.abs(resid[i] - ref.resid)) <= 1e-9 * np.max(np.abs(ref.ritz)) + 1e-6 * np.max(ref.resid)


def test_batch_of_generated_subdomains():
    """Uneven boxes cut from one crystal (the batch workload's recipe at
    reduced size), mixed degrees, FP32 filter + split-BF16 GEMMs."""
    case("batch generated subdomains")
    _, sds, degs = workloads.batch_subdomains(count=5, ncells=4, nmin=16, nmax=26, with_x0=True)
    params = [xls.chefsi_params(min(d, 20), 3, xls.XLS_BOUNDS_LANCZOS, gemm_prec=xls.XLS_PREC_BF16X3)
              for d in degs]
    single = single_runs(sds, xls.XLS_PREC_FP32, params)
    assert_same(single, batch_run(sds, xls.XLS_PREC_FP32, params))


def test_batch_tuner_cache_and_invariance(tmp_path):
    """The tuner picks a filter tile shape and a GEMM plan per class and
    reuses its cache.  A tile shape changes scheduling only; a GEMM plan
    changes the order of the split-K sums only: the tuned batch equals single
    runs under the same choices bit for bit, and the untuned batch to
    rounding."""
    case("batch tuner")
    sds = uneven_boxes()
    params = [xls.chefsi_params(d, 3, xls.XLS_BOUNDS_LANCZOS, gemm_prec=xls.XLS_PREC_FP32) for d in (7, 10, 12)]
    ref = batch_run(sds, xls.XLS_PREC_FP32, params)
    path = str(tmp_path / "tune.json")
    with xls.Batch(sds, filter_prec=xls.XLS_PREC_FP32) as b:
        tuned, best = b.xls_batch_tune(path)
        keys = {k for sd in sds for k in xls.tune_keys(sd, xls.XLS_PREC_FP32)}
        assert tuned == len(keys) and best > 0
        cache = json.load(open(path))
        assert set(cache) == keys
        for k, v in cache.items():
            if k.startswith("gemm_"):
                assert v[0] in (0, 1, 4, 8) and v[1] in (0, 1) and v[2] in (0, 1)
            else:
                assert v[0] in (256, 512) and v[1] in (0, 1, 2, 4, 8, 16) and v[2] in (1, 2)
        again, _ = b.xls_batch_tune(path)
        assert again == 0
        ritz, resid, iters, status = b.xls_batch_chefsi(params)
        blocks = [b.xls_batch_subdomain(i).xls_subdomain_get_block() for i in range(3)]
    single = []
    for sd, p in zip(sds, params):
        with xls.Subdomain(sd, filter_prec=xls.XLS_PREC_FP32) as s:
            skey, gkey = xls.tune_keys(sd, xls.XLS_PREC_FP32)
            blk, ty, nv = cache[skey]
            s.xls_subdomain_tune(xls.XLS_PREC_FP32, blk, ty, 0, nv)
            s.xls_subdomain_tune_gemm(*cache[gkey])
            r = s.xls_chefsi_step(p.degree, p.max_iter, p.bounds_mode, lanczos_k=p.lanczos_k, gemm_prec=p.gemm_prec)
            single.append(r + (s.xls_subdomain_get_block(),))
    assert_same(single, (ritz, resid, iters, status, blocks, None))
    for a, b2 in zip(ritz, ref[0]):
        assert np.max(np.abs(a - b2) / np.maximum(np.abs(b2), 1.0)) <= 1e-5


@pytest.mark.parametrize("prec", [xls.XLS_PREC_FP64, xls.XLS_PREC_FP32])
def test_batch_two_vectors_per_tile_bit_identical(prec):
    """Grouped launches over tiles of 2 vectors (odd Ns leaves an empty
    second vector) give the same bits as 1-vector tiles."""
    case(f"batch nv=2 prec={prec}")
    sds = uneven_boxes()
    sds[0] = workloads.small_dirichlet(ns=9, index=1, shape=(13, 9, 20), h=0.6)
    params = [xls.chefsi_params(d, 3, xls.XLS_BOUNDS_LANCZOS) for d in (7, 10, 12)]
    ref = batch_run(sds, prec, params)
    with xls.Batch(sds, filter_prec=prec) as b:
        for i in range(len(sds)):
            b.xls_batch_subdomain(i).xls_subdomain_tune(prec, 256, 0, 0, 2)
        ritz, resid, iters, status = b.xls_batch_chefsi(params)
        blocks = [b.xls_batch_subdomain(i).xls_subdomain_get_block() for i in range(len(sds))]
    assert_same([(r, e, it, blk) for r, e, it, blk in zip(ref[0], ref[1], ref[2], ref[4])],
                (ritz, resid, iters, status, blocks, None))


def test_batch_density_matches_single():
    case("batch density")
    sds = uneven_boxes()
    params = [xls.chefsi_params(d, 2, xls.XLS_BOUNDS_LANCZOS) for d in (7, 10, 12)]
    with xls.Batch(sds, filter_prec=xls.XLS_PREC_FP64) as b:
        ritz, _, _, _ = b.xls_batch_chefsi(params)
        mu = float(np.median(np.concatenate(ritz)))
        rho_b, c_b = b.xls_batch_density(mu, 0.01)
    for i, (sd, p) in enumerate(zip(sds, params)):
        with xls.Subdomain(sd, filter_prec=xls.XLS_PREC_FP64) as s:
            s.xls_chefsi_step(p.degree, p.max_iter, p.bounds_mode)
            rho, c = s.xls_subdomain_density(mu, 0.01)
        assert np.array_equal(rho, rho_b[i]) and np.array_equal(c, c_b[i])


def test_batch_argument_errors():
    case("batch errors")
    sds = uneven_boxes()[:2]
    with xls.Batch(sds, filter_prec=xls.XLS_PREC_FP64) as b:
        bad = [xls.chefsi_params(300, 2), xls.chefsi_params(8, 2)]
        with pytest.raises(xls.XlsError) as ei:
            b.xls_batch_chefsi(bad)
        assert ei.value.code == xls.XLS_ERR_INVALID_ARG
        mixed = [xls.chefsi_params(8, 2, gemm_prec=xls.XLS_PREC_BF16X3), xls.chefsi_params(8, 2)]
        with pytest.raises(xls.XlsError):
            b.xls_batch_chefsi(mixed)
        learned = [xls.chefsi_params(8, 2, xls.XLS_BOUNDS_LEARNED), xls.chefsi_params(8, 2)]
        with pytest.raises(xls.XlsError):
            b.xls_batch_chefsi(learned)
