"""Learned filter bounds through the C ABI: the library's fit (standardisation
and training RMS), its bounds policy (margins, degree rule), and the Lanczos
fallback a learned run takes when its bounds miss, for one subdomain
(xls_chefsi_step) and inside a batch (xls_batch_chefsi).

The fallback tests plant the miss on purpose from the host: lam_max is set
just above lam_cut, far below the top of the spectrum, so the filter
amplifies the unwanted end and the run cannot meet the gate.  Every kernel
still runs to completion; only the host-side decision is exercised."""
import numpy as np
import pytest

from oracle import bf16 as obf
from oracle import chefsi as ochefsi
from oracle import hamiltonian
from paper_2609_13115_amd import workloads, xls

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[case] {msg}", flush=True)


def bf16_round(a):
    return obf.bf16_to_f32(obf.bf16_rne_bits(np.asarray(a, np.float32))).astype(np.float64)


def emulate_predict(P, F, fmu, fsd, tmu, tsd):
    """bf16 inference as the library defines it (inputs, weights and hidden
    activations rounded to bf16, FP32 sums in ascending input order)."""
    x = (F.astype(np.float32) - fmu) * (np.float32(1.0) / fsd)
    h = bf16_round(x).astype(np.float32)
    nl = len(P) // 2
    for l in range(nl):
        W = bf16_round(P[2 * l].astype(np.float32)).astype(np.float32)
        z = np.broadcast_to(P[2 * l + 1].astype(np.float32), (h.shape[0], W.shape[1])).copy()
        for i in range(W.shape[0]):
            z = (z + h[:, i:i + 1] * W[i:i + 1, :]).astype(np.float32)
        h = bf16_round(np.maximum(z, 0)).astype(np.float32) if l < nl - 1 else z
    return h.astype(np.float64) * tsd + tmu


def policy(p, rms_cut):
    """The bounds rule of xls_mlp_bounds, restated from its declaration."""
    out = []
    for pm, pc, pd in p:
        d = int(min(max(np.rint(pd), 16), 32))
        if not pc < pm:
            pc = 0.5 * pm
        c = pc + 3.0 * rms_cut
        x = c + 1.03 * (pm - c)
        if not c < x:
            x = c + 0.03 * abs(c) + 1e-3
        out.append((x, c, d))
    return np.array(out)


def test_fit_standardises_and_applies_the_bounds_policy():
    case("mlp fit + bounds policy")
    sizes = (64, 128, 128, 3)
    rng = np.random.default_rng(11)
    n = 40
    F = rng.standard_normal((n, 64)) * rng.uniform(0.5, 20, 64) + rng.uniform(-5, 5, 64)
    F[:, 50:] = 0.0                      # zero padding: constant columns
    F[:, 47] = 3.25                      # a constant nonzero column
    T = np.stack([rng.uniform(30, 60, n), rng.uniform(-1, 1, n), rng.uniform(14, 34, n)], axis=1)
    P = workloads.mlp_init(sizes, 7)
    for p in P[1::2]:
        p[:] = rng.standard_normal(p.shape) * 0.1
    with xls.Mlp(sizes, P) as m:
        m.fit(F, T, [], lr=1e-3)         # no steps: the parameters stay as given
        pred = m.predict(F)
        rms = m.train_rms()
        lm, lc, deg = m.bounds(F)
    fsd = F.std(0)
    fsd = np.where(fsd > 0, fsd, 1.0)
    tsd = T.std(0)
    ref = emulate_predict(P, F, F.mean(0).astype(np.float32), fsd.astype(np.float32), T.mean(0), tsd)
    # the library's fixed-order mean/std may differ from numpy's in the last
    # bit, which can move an FP32-rounded input scale by one ulp
    assert np.max(np.abs(pred - ref) / (np.abs(ref) + 1.0)) <= 1e-5
    rms_ref = np.sqrt(np.mean((pred - T) ** 2, axis=0))
    assert np.allclose(rms, rms_ref, rtol=1e-12, atol=0)
    pol = policy(pred, rms[1])
    assert np.allclose(lm, pol[:, 0], rtol=1e-13, atol=1e-13)
    assert np.allclose(lc, pol[:, 1], rtol=1e-13, atol=1e-13)
    assert np.array_equal(deg, pol[:, 2].astype(np.int32))
    assert np.all(lc < lm) and np.all((deg >= 16) & (deg <= 32))


def test_fit_rejects_bad_minibatches():
    case("mlp fit argument errors")
    with xls.Mlp((4, 3, 3)) as m:
        F = np.zeros((5, 4))
        T = np.zeros((5, 3))
        for batches in ([np.array([0, 9])], [np.array([-1])]):
            with pytest.raises(xls.XlsError):
                m.fit(F, T, batches)
        with pytest.raises(xls.XlsError) as e:
            m.bounds(F)                    # three outputs, but never fitted
        assert e.value.code == xls.XLS_ERR_STATE


def forced_miss_bounds(sd):
    """(lam_max, lam_cut) whose lam_max lies far below the top of the spectrum."""
    op = hamiltonian.from_subdomain(sd)
    lo, up = ochefsi.lanczos_bounds(op.apply, sd.lanczos_v0, 20)
    lc = lo + 0.3 * (up - lo)
    return lc + 0.02 * (up - lo), lc


@pytest.mark.parametrize("prec", [xls.XLS_PREC_FP64, xls.XLS_PREC_FP32])
def test_learned_fallback_fires_and_meets_the_gate(prec):
    case(f"forced learned fallback, single subdomain, prec {prec}")
    sd = workloads.small_dirichlet(ns=10, index=3, shape=(14, 12, 16), h=0.7)
    lm, lc = forced_miss_bounds(sd)
    tol = 1e-4 if prec == xls.XLS_PREC_FP64 else 5e-4
    gp = xls.XLS_PREC_FP64 if prec == xls.XLS_PREC_FP64 else xls.XLS_PREC_FP32
    with xls.Subdomain(sd, filter_prec=prec) as s:
        ritz, resid, it = s.xls_chefsi_step(16, 25, xls.XLS_BOUNDS_LEARNED, lam_cut=lc, lam_max=lm,
                                            resid_tol=tol, gemm_prec=gp, fallback_tol=tol,
                                            fallback_degree=20)
        c = s.xls_subdomain_counters()
    gate = int(np.floor(sd.ns / 1.1 + 1e-9))
    print(f"[fallback] iterations {c['iterations']} fallback {c['fallback']} "
          f"gated resid {np.max(resid[:gate]):.2e}", flush=True)
    assert c["fallback"] and np.max(resid[:gate]) <= tol
    # the restart is a plain Lanczos run from the same start block
    with xls.Subdomain(sd, filter_prec=prec) as s2:
        r2, res2, it2 = s2.xls_chefsi_step(20, 25, xls.XLS_BOUNDS_LANCZOS, resid_tol=tol, gemm_prec=gp)
    assert np.array_equal(ritz, r2)
    assert it == c["iterations"] and it > it2


def test_learned_fallback_inside_a_batch():
    case("forced learned fallback inside a batch")
    sds = [workloads.small_dirichlet(ns=10, index=3, shape=(14, 12, 16), h=0.7),
           workloads.small_dirichlet(ns=8, index=4, shape=(12, 12, 12), h=0.7),
           workloads.small_dirichlet(ns=9, index=5, shape=(13, 11, 15), h=0.7)]
    lm, lc = forced_miss_bounds(sds[0])
    tol = 1e-4
    bad = xls.chefsi_params(16, 25, xls.XLS_BOUNDS_LEARNED, lam_cut=lc, lam_max=lm, resid_tol=tol,
                            fallback_tol=tol, fallback_degree=20)
    good = [xls.chefsi_params(20, 25, xls.XLS_BOUNDS_LANCZOS, resid_tol=tol) for _ in sds[1:]]
    with xls.Batch(sds, filter_prec=xls.XLS_PREC_FP64) as b:
        ritz, resid, iters, status = b.xls_batch_chefsi([bad] + good)
        fb = [b.xls_batch_subdomain(i).xls_subdomain_counters()["fallback"] for i in range(3)]
    assert list(status) == [0, 0, 0]
    assert fb == [True, False, False]
    for sd, r in zip(sds, resid):
        gate = int(np.floor(sd.ns / 1.1 + 1e-9))
        assert np.max(r[:gate]) <= tol
    # bit-identical to the same learned run on the subdomain alone
    with xls.Subdomain(sds[0], filter_prec=xls.XLS_PREC_FP64) as s:
        r1, _, it1 = s.xls_chefsi_step(16, 25, xls.XLS_BOUNDS_LEARNED, lam_cut=lc, lam_max=lm, resid_tol=tol,
                                       fallback_tol=tol, fallback_degree=20)
    assert np.array_equal(ritz[0], r1) and iters[0] == it1
