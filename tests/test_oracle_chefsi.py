"""Pins of the oracle's CheFSI: closed forms, invariants, brute force."""
import numpy as np
import pytest

from oracle import chefsi, hamiltonian
from paper_2609_13115_amd import workloads


def _diag_op(d):
    return lambda X: d[:, None] * X if X.ndim == 2 else d * X


@pytest.mark.parametrize("m", [1, 2, 7, 20, 24])
def test_filter_closed_form_on_diagonal_operator(m):
    """On H = diag(d): Y_m / X = C_m((d - c)/e) / C_m((a0 - c)/e) row by row."""
    d = workloads.diagonal_spectrum(200)
    X = workloads.random_block(200, 5, (7, 7))
    a0, lc, lmax = d[0], d[40], d[-1] + 0.3
    Y = chefsi.chebyshev_filter(_diag_op(d), X, m, a0, lc, lmax)
    e = (lmax - lc) / 2
    c = (lmax + lc) / 2
    ratio = chefsi.chebyshev_value(m, (d - c) / e) / chefsi.chebyshev_value(m, np.array([(a0 - c) / e]))[0]
    assert np.allclose(Y, ratio[:, None] * X, rtol=1e-11, atol=1e-13)
    # normalisation p(a0) = 1
    assert abs(ratio[0] - 1.0) < 1e-12


def test_chebyshev_closed_form_matches_recurrence_definition():
    """C_m via cos/cosh equals the textbook recurrence C_{k+1} = 2t C_k - C_{k-1}."""
    t = np.linspace(-3, 3, 61)
    C0, C1 = np.ones_like(t), t.copy()
    for m in range(2, 15):
        C0, C1 = C1, 2 * t * C1 - C0
        assert np.allclose(chefsi.chebyshev_value(m, t), C1, rtol=1e-10, atol=1e-10)


def test_lanczos_bound_on_diagonal_operator():
    d = workloads.diagonal_spectrum(300)
    v0 = workloads.random_block(300, 1, (9, 9))[:, 0]
    lo, up = chefsi.lanczos_bounds(_diag_op(d), v0, 20)
    assert up >= d[-1]
    assert lo >= d[0] - 1e-12
    assert up - d[-1] < 0.5 * (d[-1] - d[0])


def test_lanczos_bound_free_periodic_24_grid():
    """V = 0, no projectors, 24^3, h = 0.4275: spectrum [0, 58.0522] (closed form)."""
    op = hamiltonian.free_operator((24, 24, 24), 0.4275, True)
    v0 = workloads.random_block(op.nd, 1, (3, 3))[:, 0]
    lo, up = chefsi.lanczos_bounds(op.apply, v0, 20)
    assert up >= 58.0522 - 1e-4
    assert lo >= -1e-10


def test_lanczos_exact_on_small_krylov_space():
    """An operator with 3 distinct eigenvalues: Lanczos terminates with the exact spectrum."""
    d = np.repeat([1.0, 2.5, 4.0], 30)
    v0 = np.ones(90)
    _, beta, theta = chefsi.lanczos(_diag_op(d), v0, 10)
    assert len(theta) == 3
    assert np.allclose(theta, [1.0, 2.5, 4.0], atol=1e-12)


def _brute(sd):
    op = hamiltonian.from_subdomain(sd)
    ev = np.linalg.eigvalsh(op.dense())
    return op, ev


@pytest.fixture(scope="module", params=["periodic", "dirichlet"])
def small_system(request):
    if request.param == "periodic":
        sd = workloads.small_periodic(8, 12)
    else:
        sd = workloads.small_dirichlet(8, 12)
    op, ev = _brute(sd)
    return sd, op, ev


def test_rayleigh_ritz_invariants(small_system):
    sd, op, ev = small_system
    lo, up = chefsi.lanczos_bounds(op.apply, sd.lanczos_v0, 20)
    Pf = chefsi.chebyshev_filter(op.apply, sd.x0, 10, lo, chefsi.first_cutoff(lo, up), up)
    lam, Psi, Y, M, Hs = chefsi.rayleigh_ritz(op.apply, Pf)
    ns = sd.ns
    # orthonormal columns
    assert np.allclose(Psi.T @ Psi, np.eye(ns), atol=1e-12)
    # Cauchy interlacing: Ritz values bound the exact eigenvalues from above
    assert np.all(lam >= ev[:ns] - 1e-10)
    # residual bound: an exact eigenvalue lies within r_n of every Ritz value
    r = chefsi.residuals(op.apply, Psi, lam)
    for l, rr in zip(lam, r):
        assert np.min(np.abs(ev - l)) <= rr + 1e-10
    # invariance under X -> X G for invertible G
    G = np.random.default_rng(4).standard_normal((ns, ns)) + 3 * np.eye(ns)
    lam2, _, _, _, _ = chefsi.rayleigh_ritz(op.apply, Pf @ G)
    assert np.allclose(lam, lam2, rtol=1e-9, atol=1e-9)


def test_chefsi_converges_to_brute_force(small_system):
    """Converged Ritz values equal the lowest eigenvalues of the dense H."""
    sd, op, ev = small_system
    lo, up = chefsi.lanczos_bounds(op.apply, sd.lanczos_v0, 20)
    res = chefsi.chefsi(op.apply, sd.x0, 16, 60, lo, chefsi.first_cutoff(lo, up), up,
                        resid_tol=1e-11)
    g = chefsi.n_gate(sd.ns)
    assert np.max(res.resid[:g]) <= 1e-9
    rel = np.abs(res.ritz[:g] - ev[:g]) / np.maximum(np.abs(ev[:g]), 1e-3)
    assert np.max(rel) <= 1e-10


def test_not_spd_raised_for_duplicated_columns():
    sd = workloads.small_dirichlet(8, 4)
    op = hamiltonian.from_subdomain(sd)
    X = sd.x0.copy()
    X[:, 2] = X[:, 1]
    with pytest.raises(chefsi.NotSPD):
        chefsi.rayleigh_ritz(op.apply, X)


def test_generalized_eigh_matches_scipy_eigh():
    """Special case that reduces to a library routine: the Cholesky-based
    solve of H y = lambda M y agrees with scipy's generalized eigh."""
    import scipy.linalg as sla
    rng = np.random.default_rng(8)
    A = rng.standard_normal((30, 30))
    M = A @ A.T + 30 * np.eye(30)
    B = rng.standard_normal((30, 30))
    H = B + B.T
    lam, Y = chefsi.generalized_eigh(H, M)
    ref = sla.eigh(H, M, eigvals_only=True)
    assert np.allclose(lam, ref, rtol=1e-12, atol=1e-12)
    assert np.allclose(Y.T @ M @ Y, np.eye(30), atol=1e-12)


def test_n_gate():
    assert chefsi.n_gate(20) == 18
    assert chefsi.n_gate(480) == 436
    assert chefsi.n_gate(1) == 1
    assert chefsi.n_gate(11) == 10


def test_subspace_angle_of_rotated_basis_is_zero():
    rng = np.random.default_rng(2)
    Q = rng.standard_normal((50, 6))
    G = rng.standard_normal((6, 6)) + 4 * np.eye(6)
    assert chefsi.subspace_sin_theta(Q, Q @ G) < 1e-12
    Q2 = Q.copy()
    Q2[:, 0] = rng.standard_normal(50)
    assert chefsi.subspace_sin_theta(Q, Q2) > 1e-3


def test_subspace_sin_theta_is_the_largest_principal_angle():
    """Two columns rotated by known angles a and b into orthogonal planes: the
    principal angles are a and b, and the value is sin(max(a, b)) (a norm
    other than the spectral one would mix the two)."""
    from oracle import chefsi as oc
    n = 7
    e = np.eye(n)
    for a, b in [(0.3, 0.1), (0.05, 0.9), (0.4, 0.4)]:
        Qo = np.stack([e[0], e[2]], axis=1)
        Qg = np.stack([np.cos(a) * e[0] + np.sin(a) * e[1], np.cos(b) * e[2] + np.sin(b) * e[3]], axis=1)
        assert oc.subspace_sin_theta(Qg, Qo) == pytest.approx(np.sin(max(a, b)), rel=1e-13)
        assert oc.subspace_sin_theta(Qo, Qg) == pytest.approx(np.sin(max(a, b)), rel=1e-13)
    # invariant to the basis chosen inside each span
    G = np.array([[2.0, 1.0], [0.5, 3.0]])
    assert oc.subspace_sin_theta(Qg @ G, Qo) == pytest.approx(np.sin(max(a, b)), rel=1e-12)
