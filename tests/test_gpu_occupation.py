"""Fermi level, global density and density of states of a batch on the GPU
(Sec. V-A.4, V-A.5), through the C ABI, against the oracle."""
import numpy as np
import pytest

from oracle import density, grid
from paper_2609_13115_amd import workloads, xls

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[case] {msg}", flush=True)


def tiled_pair(ns=8):
    """Two zero-Dirichlet boxes cut from one displaced crystal whose cores
    split the 16^3 global grid in half along x (buffers of 3 points in x and
    2 in y, z; the boxes wrap the periodic global cell in y and z)."""
    key = (workloads.SEED_BASE + 93000, 0)
    gs = workloads.diamond_si_system(2, 16, 0.1, key)
    out = []
    for i, x0 in enumerate((0, 8)):
        out.append(gs.subdomain((x0, 0, 0), (8, 16, 16), (3, 2, 2), (14, 20, 20), ns,
                                workloads.BC_DIRICHLET0, key + (i,), True, name=f"half {i}"))
    return gs, out


def params_for(sds, degree=10, iters=6, gemm_prec=xls.XLS_PREC_FP64):
    return [xls.chefsi_params(degree, iters, xls.XLS_BOUNDS_LANCZOS, gemm_prec=gemm_prec) for _ in sds]


def oracle_weights(blocks, sds, ritz, mu, sigma):
    rhos, cs = [], []
    for psi, sd, lam in zip(blocks, sds, ritz):
        mask = grid.core_mask(sd.n, sd.core_lo, sd.core_hi)
        r, c = density.core_density(psi, lam, mu, sigma, mask, sd.h)
        rhos.append(r)
        cs.append(c)
    return rhos, cs


@pytest.mark.parametrize("prec", [xls.XLS_PREC_FP64, xls.XLS_PREC_FP32])
def test_batch_fermi_level_and_energies_match_oracle(prec):
    """The solve's inputs are the batch's own Ritz values and blocks (FP32
    blocks widened exactly); the oracle redoes the weights and the level."""
    case(f"batch fermi prec={prec}")
    gs, sds = tiled_pair()
    sigma = 0.02
    with xls.Batch(sds, filter_prec=prec) as b:
        with pytest.raises(xls.XlsError) as ei:
            b.xls_batch_fermi(sigma, 4.0)
        assert ei.value.code == xls.XLS_ERR_STATE
        ritz, resid, iters, status = b.xls_batch_chefsi(params_for(sds, gemm_prec=prec))
        blocks = [b.xls_batch_subdomain(i).xls_subdomain_get_block() for i in range(len(sds))]
        lam = np.concatenate(ritz)
        _, cs = oracle_weights(blocks, sds, ritz, 0.0, sigma)
        c = np.concatenate(cs)
        ne = 0.5 * float(np.sum(2.0 * c))  # half of what the states can hold
        mu, n_at, e_band, e_ent, evals = b.xls_batch_fermi(sigma, ne)
        mu_ref = density.fermi_level(lam, c, sigma, ne)
        scale = max(1.0, float(np.max(np.abs(lam))))
        assert abs(mu - mu_ref) <= 1e-10 * scale, (mu, mu_ref)
        assert abs(n_at - ne) <= 1e-10 * ne
        assert abs(density.electron_count(lam, c, mu, sigma) - ne) <= 1e-10 * ne
        assert abs(e_band - density.band_energy(lam, c, mu, sigma)) <= 1e-11 * max(1.0, abs(e_band))
        assert abs(e_ent - density.entropy_energy(lam, c, mu, sigma)) <= 1e-11 * max(1.0, abs(e_ent))
        assert 3 <= evals <= 200
        # a count the states cannot hold, and bad arguments
        for bad in ((sigma, 2.0 * float(np.sum(c)) + 1.0), (0.0, ne), (sigma, -1.0)):
            with pytest.raises(xls.XlsError) as ei:
                b.xls_batch_fermi(*bad)
            assert ei.value.code == xls.XLS_ERR_INVALID_ARG


def test_batch_global_density_and_dos_match_oracle():
    case("batch assemble fp64")
    gs, sds = tiled_pair()
    sigma = 0.03
    n_global = int(np.prod(gs.global_n))
    with xls.Batch(sds, filter_prec=xls.XLS_PREC_FP64) as b:
        ritz, resid, iters, status = b.xls_batch_chefsi(params_for(sds))
        with pytest.raises(xls.XlsError) as ei:
            b.xls_batch_assemble(n_global)
        assert ei.value.code == xls.XLS_ERR_STATE
        blocks = [b.xls_batch_subdomain(i).xls_subdomain_get_block() for i in range(len(sds))]
        lam = np.concatenate(ritz)
        _, cs = oracle_weights(blocks, sds, ritz, 0.0, sigma)
        ne = 0.6 * float(np.sum(2.0 * np.concatenate(cs)))
        mu = b.xls_batch_fermi(sigma, ne)[0]
        edges = np.sort(np.random.default_rng(3).uniform(lam.min() - 0.1, lam.max() + 0.1, 17))
        rho, dos = b.xls_batch_assemble(n_global, edges)
        # a global grid too small for the maps
        with pytest.raises(xls.XlsError) as ei:
            b.xls_batch_assemble(n_global - 1)
        assert ei.value.code == xls.XLS_ERR_INVALID_ARG
    rhos, cs = oracle_weights(blocks, sds, ritz, mu, sigma)
    parts = [(r, grid.core_mask(sd.n, sd.core_lo, sd.core_hi), grid.global_index(sd.n, sd.global_offset, sd.global_n))
             for r, sd in zip(rhos, sds)]
    ref = density.assemble_density(parts, n_global)
    assert np.max(np.abs(rho - ref)) <= 1e-12 * np.max(np.abs(ref))
    # the cores tile the global grid: its charge is the electron count
    assert abs(gs.h ** 3 * rho.sum() - ne) <= 1e-10 * ne
    c = np.concatenate(cs)
    dref = density.dos_histogram(lam, c, edges)
    assert np.max(np.abs(dos - dref)) <= 1e-12 * max(1.0, np.max(np.abs(dref)))
