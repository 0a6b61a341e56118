"""Pins of the oracle's density, interior weights and derived energies."""
import numpy as np
import pytest

from oracle import density, grid
from paper_2609_13115_amd import workloads


def _orthonormal(nd, ns, seed=0):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((nd, ns)))
    return q


def test_fermi_limits_and_symmetry():
    mu, s = 0.3, 0.01
    x = np.linspace(-2, 2, 101)
    g = density.fermi(mu + x, mu, s)
    gm = density.fermi(mu - x, mu, s)
    assert np.allclose(g + gm, 1.0, atol=1e-15)
    assert density.fermi(np.array([mu]), mu, s)[0] == 0.5
    # no overflow far from mu
    big = density.fermi(np.array([1e6, -1e6]), 0.0, 1e-3)
    assert big[0] == 0.0 and big[1] == 1.0


def test_charge_identity():
    """h^3 sum_g rho~_g = 2 sum_n g_n c_n exactly in exact arithmetic."""
    sd = workloads.small_dirichlet(8, 6)
    psi = _orthonormal(sd.nd, 6)
    lam = np.linspace(-1, 1, 6)
    mask = grid.core_mask(sd.n, sd.core_lo, sd.core_hi)
    rho, c = density.core_density(psi, lam, 0.1, 0.0037, mask, sd.h)
    g = density.fermi(lam, 0.1, 0.0037)
    assert abs(sd.h ** 3 * rho.sum() - 2 * np.sum(g * c)) < 1e-12
    assert np.all(rho[mask == 0] == 0.0)
    assert np.all((c >= 0) & (c <= 1 + 1e-14))


def test_whole_box_core_gives_unit_weights():
    n = (6, 5, 4)
    psi = _orthonormal(120, 5, 1)
    mask = grid.core_mask(n, (0, 0, 0), n)
    _, c = density.core_density(psi, np.zeros(5), 0.0, 0.01, mask, 0.5)
    assert np.allclose(c, 1.0, atol=1e-13)


def test_zero_temperature_limit():
    """sigma -> 0 with mu in a gap: rho~ = (2/h^3) sum_occ psi^2."""
    n = (4, 4, 4)
    psi = _orthonormal(64, 6, 2)
    lam = np.array([-2.0, -1.5, -1.0, 1.0, 1.5, 2.0])
    mask = grid.core_mask(n, (0, 0, 0), n)
    h = 0.5
    rho, _ = density.core_density(psi, lam, 0.0, 1e-6, mask, h)
    ref = (2 / h ** 3) * np.sum(psi[:, :3] ** 2, axis=1)
    assert np.allclose(rho, ref, atol=1e-12)


def test_energies_and_count():
    lam = np.array([-1.0, -0.5, 0.2, 0.9])
    c = np.array([0.9, 0.8, 0.7, 0.4])
    sigma = 0.05
    # sigma -> 0: E_entropy -> 0, E_band -> 2 sum_occ c lambda
    assert abs(density.entropy_energy(lam, c, 0.0, 1e-6)) < 1e-12
    assert abs(density.band_energy(lam, c, 0.0, 1e-6) - 2 * (-0.9 - 0.4)) < 1e-12
    # N_e monotone in mu
    ne = [density.electron_count(lam, c, mu, sigma) for mu in np.linspace(-2, 2, 50)]
    assert np.all(np.diff(ne) >= 0)
    # entropy term has the closed form at g = 1/2: s = log(1/2)
    e = density.entropy_energy(np.array([0.0]), np.array([1.0]), 0.0, sigma)
    assert abs(e - (-2 * sigma * np.log(0.5))) < 1e-15
    # DOS integrates to 2 sum c
    hist = density.dos_histogram(lam, c, np.linspace(-2, 2, 9))
    assert abs(hist.sum() - 2 * c.sum()) < 1e-14


def test_fermi_level_symmetric_spectrum_is_the_centre():
    """A spectrum symmetric about mu0 with mirrored weights holds exactly half
    its states' weight at mu0 (g(mu0 - d) + g(mu0 + d) = 1), so the Fermi
    level at that electron count is mu0."""
    mu0, sigma = -0.137, 0.02
    d = np.array([0.003, 0.05, 0.2, 0.71, 1.3])
    cw = np.array([0.9, 0.4, 1.0, 0.25, 0.6])
    lam = np.concatenate([mu0 - d, mu0 + d])
    c = np.concatenate([cw, cw])
    mu = density.fermi_level(lam, c, sigma, float(np.sum(c)))
    assert abs(mu - mu0) <= 1e-13


def test_fermi_level_small_sigma_falls_in_the_gap():
    """sigma -> 0: with unit weights and 2 k electrons the level sits between
    the k-th and (k+1)-th eigenvalue and the count is met."""
    lam = np.array([-1.0, -0.4, 0.25, 0.3, 1.9, 2.0])
    c = np.ones_like(lam)
    for k in (1, 3, 5):
        mu = density.fermi_level(lam, c, 1e-3, 2.0 * k)
        assert lam[k - 1] < mu < lam[k]
        assert abs(density.electron_count(lam, c, mu, 1e-3) - 2.0 * k) <= 1e-9
    with pytest.raises(ValueError):
        density.fermi_level(lam, c, 1e-3, 2.0 * len(lam) + 1.0)


def test_assemble_density_places_each_core_by_its_map():
    """Two subsystems whose cores tile a global box: the assembled density
    equals every core value at its global point (loop over points), and its
    integral is the sum of the subsystems' charges."""
    gn = (6, 4, 3)
    n_global = gn[0] * gn[1] * gn[2]
    rng = np.random.default_rng(7)
    parts, charge = [], 0.0
    h = 0.5
    for off, lo, hi in (((-2, 0, 0), (2, 0, 0), (5, 4, 3)), ((1, 0, 0), (2, 0, 0), (5, 4, 3))):
        n = (7, 4, 3)
        mask = grid.core_mask(n, lo, hi)
        gidx = grid.global_index(n, off, gn)
        r = rng.random(n[0] * n[1] * n[2])
        parts.append((r, mask, gidx))
        charge += h ** 3 * float(np.sum(r[mask == 1]))
    rho = density.assemble_density(parts, n_global)
    ref = np.zeros(n_global)
    seen = np.zeros(n_global, dtype=int)
    for r, mask, gidx in parts:
        for g in range(len(r)):
            if mask[g]:
                ref[gidx[g]] += r[g]
                seen[gidx[g]] += 1
    assert np.all(seen == 1)  # the two cores partition the global box
    assert np.array_equal(rho, ref)
    assert abs(h ** 3 * rho.sum() - charge) <= 1e-12
