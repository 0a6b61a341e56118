"""Slot residency of the batch engine and device-drawn start blocks, through
the C ABI.

* A start block drawn on the device from x0_seed equals the counter-based
  generator written out in numpy (Philox4x32-10 + Box-Muller; the integer
  stream is pinned by its published known answers in the CPU tests): FP64
  to a few ulps of the transcendental functions, FP32 to one FP32 rounding.
* A slot-residency batch whose budget admits one or two subdomains at a time
  gives bit-identical Ritz values, residuals, iteration counts, densities,
  interior weights and Fermi level to a resident batch, with host and with
  device start blocks, and with a learned-bounds fallback restarted from X0.
* Per-handle calls that need a block return STATE on its handles."""
import numpy as np
import pytest

from oracle import chefsi as ochefsi
from oracle import hamiltonian
from paper_2609_13115_amd import workloads, xls

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[case] {msg}", flush=True)


@pytest.mark.parametrize("prec", [xls.XLS_PREC_FP64, xls.XLS_PREC_FP32])
def test_device_start_block_matches_numpy_generator(prec):
    case(f"philox start block prec {prec}")
    sd = workloads.small_dirichlet(ns=7, index=2, shape=(13, 11, 17), with_x0=False)
    seed = workloads.x0_seed(sd.seed_key)
    ref = workloads.philox_normal_block(sd.nd, sd.ns, seed)
    with xls.Subdomain(sd, filter_prec=prec, x0_seed=seed) as s:
        X = s.xls_subdomain_get_block()
    if prec == xls.XLS_PREC_FP64:
        assert np.max(np.abs(X - ref) / np.maximum(np.abs(ref), 1.0)) <= 1e-14
    else:
        r32 = ref.astype(np.float32).astype(np.float64)
        assert np.all(np.abs(X - r32) <= np.spacing(np.abs(r32).astype(np.float32)).astype(np.float64))
    assert abs(ref.mean()) < 0.1 and abs(ref.std() - 1.0) < 0.1


def boxes():
    return [workloads.small_dirichlet(ns=10, index=3, shape=(14, 12, 16), h=0.7),
            workloads.small_dirichlet(ns=8, index=4, shape=(12, 12, 12), h=0.7),
            workloads.small_dirichlet(ns=12, index=6, shape=(16, 14, 15), h=0.7),
            workloads.small_dirichlet(ns=9, index=5, shape=(13, 11, 15), h=0.7)]


def run(sds, slots, prec, params, seeds=None):
    with xls.Batch(sds, filter_prec=prec, x0_seeds=seeds, slots=slots) as b:
        ritz, resid, iters, status = b.xls_batch_chefsi(params)
        fb = [b.xls_batch_subdomain(i).xls_subdomain_counters()["fallback"] for i in range(len(sds))]
        rho, c = b.xls_batch_density(-0.2, 0.01)
        ne = 2.0 * sum(int(np.floor(sd.ns / 1.1)) for sd in sds) * 0.5
        fermi = b.xls_batch_fermi(0.01, ne)
        stats = b.xls_batch_stats()
        if slots is not None:
            with pytest.raises(xls.XlsError) as e:
                b.xls_batch_subdomain(0).xls_subdomain_get_block()
            assert e.value.code == xls.XLS_ERR_STATE
    return ritz, resid, iters, status, fb, rho, c, fermi, stats


def assert_same(a, b):
    """Eigenpairs, iterations and densities bit for bit; interior weights and
    the Fermi level to rounding (the core store sums c_n over its compact
    rows, a different order than the masked sum over the whole box)."""
    for x, y in zip(a[:3], b[:3]):
        for u, v in zip(x, y):
            assert np.array_equal(u, v)
    assert list(a[3]) == list(b[3]) and a[4] == b[4]
    for u, v in zip(a[5], b[5]):
        assert np.array_equal(u, v)
    for u, v in zip(a[6], b[6]):
        assert np.allclose(u, v, rtol=1e-13, atol=1e-15)
    assert np.allclose(a[7][:4], b[7][:4], rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("prec,seeded", [(xls.XLS_PREC_FP64, False), (xls.XLS_PREC_FP32, True)])
def test_slot_batch_is_bit_identical_to_resident(prec, seeded):
    case(f"slot vs resident batch prec {prec} seeded {seeded}")
    sds = boxes()
    gp = xls.XLS_PREC_FP64 if prec == xls.XLS_PREC_FP64 else xls.XLS_PREC_BF16X3
    params = [xls.chefsi_params(12 + 2 * i, 30, xls.XLS_BOUNDS_LANCZOS, resid_tol=3e-4, gemm_prec=gp)
              for i in range(len(sds))]
    seeds = [workloads.x0_seed(sd.seed_key) for sd in sds] if seeded else None
    ref = run(sds, None, prec, params, seeds)
    # a budget that admits at most two of them at once
    got = run(sds, 1, prec, params, seeds)
    assert got[8]["max_active"] == 1 and got[8]["peak_bytes"] > 0
    assert_same(got, ref)
    with xls.Batch(sds, filter_prec=prec, x0_seeds=seeds, slots=0) as b:  # default budget: all at once
        r2 = b.xls_batch_chefsi(params)
        assert b.xls_batch_stats()["max_active"] == len(sds)
    for u, v in zip(r2[0], ref[0]):
        assert np.array_equal(u, v)


def test_slot_batch_learned_fallback_restarts_from_x0():
    case("slot batch learned fallback")
    sds = boxes()[:3]
    op = hamiltonian.from_subdomain(sds[1])
    lo, up = ochefsi.lanczos_bounds(op.apply, sds[1].lanczos_v0, 20)
    lc = lo + 0.3 * (up - lo)
    bad = xls.chefsi_params(16, 25, xls.XLS_BOUNDS_LEARNED, lam_cut=lc, lam_max=lc + 0.02 * (up - lo),
                            resid_tol=1e-4, fallback_tol=1e-4, fallback_degree=20)
    params = [xls.chefsi_params(20, 25, xls.XLS_BOUNDS_LANCZOS, resid_tol=1e-4), bad,
              xls.chefsi_params(18, 25, xls.XLS_BOUNDS_LANCZOS, resid_tol=1e-4)]
    ref = run(sds, None, xls.XLS_PREC_FP64, params)
    got = run(sds, 1, xls.XLS_PREC_FP64, params)
    assert got[4] == [False, True, False]
    assert_same(got, ref)
