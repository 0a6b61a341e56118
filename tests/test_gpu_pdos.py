"""Projected density of states (Sec. V-A.4) through the C ABI, against the
oracle.

* The weights are a plain function of the block: on a seeded block set into
  the handle they match the oracle's squared overlaps (FP64 to 1e-12; the
  FP32 block against the oracle on the same FP32-rounded block), and the
  atoms-in-core flags match bit for bit.
* After converged runs from the same inputs (the GPU's FP64 path, the
  oracle's CheFSI), the orbital-resolved PDOS in bins whose edges sit in
  spectral gaps (so degenerate clusters, whose single vectors are not
  unique, fall inside one bin) agree to 1e-7."""
import numpy as np
import pytest

from oracle import chefsi, hamiltonian
from oracle import pdos as opdos
from paper_2609_13115_amd import workloads, xls

pytestmark = pytest.mark.gpu

W, RC = 0.8, 2.5


def case(msg):
    print(f"[case] {msg}", flush=True)


@pytest.mark.parametrize("prec", [xls.XLS_PREC_FP64, xls.XLS_PREC_FP32])
def test_pdos_weights_of_a_given_block(prec):
    case(f"pdos weights prec {prec}")
    sd = workloads.small_dirichlet(ns=9, index=11, shape=(15, 13, 14), h=0.6)
    X = sd.x0 if prec == xls.XLS_PREC_FP64 else sd.x0.astype(np.float32).astype(np.float64)
    t = opdos.orbital_tables(sd, W, RC)
    ref = opdos.weights(t, X, sd.h)
    with xls.Subdomain(sd, filter_prec=prec) as s:
        s.xls_subdomain_set_block(X)
        w, d, inc = s.xls_subdomain_pdos(W, RC)
    assert d is None
    assert np.array_equal(inc, opdos.atoms_in_core(sd))
    assert 0 < inc.sum() < len(inc)
    assert np.allclose(w, ref, rtol=1e-12, atol=1e-14 * np.max(ref))


def gap_edges(lam, upto, gap=2e-3):
    """Bin edges at the midpoints of the spectral gaps between consecutive
    Ritz values up to the last gap at or below index upto, plus a lower edge."""
    cuts = [k for k in range(1, min(upto, len(lam) - 1) + 1) if lam[k] - lam[k - 1] >= gap]
    return np.array([lam[0] - 1.0] + [0.5 * (lam[k] + lam[k - 1]) for k in cuts])


def test_pdos_after_converged_runs_matches_oracle():
    case("pdos full pipeline")
    sd = workloads.small_dirichlet(ns=16, index=12, shape=(16, 15, 14), h=0.6)
    op = hamiltonian.from_subdomain(sd)
    lo, up = chefsi.lanczos_bounds(op.apply, sd.lanczos_v0, 20)
    lc = chefsi.first_cutoff(lo, up)
    ref = chefsi.chefsi(op.apply, sd.x0, 16, 40, lo, lc, up, resid_tol=1e-10)
    gate = chefsi.n_gate(sd.ns)
    assert np.max(ref.resid[:gate]) <= 1e-10
    edges = gap_edges(ref.ritz, gate)
    assert len(edges) >= 4
    t = opdos.orbital_tables(sd, W, RC)
    D_ref = opdos.pdos(opdos.weights(t, ref.psi, sd.h), ref.ritz, edges, opdos.atoms_in_core(sd))
    with xls.Subdomain(sd, filter_prec=xls.XLS_PREC_FP64) as s:
        ritz, resid, it = s.xls_chefsi_step(16, 40, xls.XLS_BOUNDS_GIVEN, lo, lc, up, resid_tol=1e-10)
        w, D, inc = s.xls_subdomain_pdos(W, RC, edges)
    assert np.max(np.abs(ritz[:gate] - ref.ritz[:gate])) <= 1e-9
    assert np.max(np.abs(D - D_ref)) <= 1e-7
    assert D.sum() > 0.1 * D_ref.size ** 0 and np.all(D[np.repeat(~inc, 4)] == 0.0)
