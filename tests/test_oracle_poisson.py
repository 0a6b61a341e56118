"""Pins of the oracle's multigrid-preconditioned Poisson solve (Sec. V-B.1)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import grid, poisson


def rhs(n, seed, periodic):
    f = np.random.default_rng(seed).standard_normal(int(np.prod(n)))
    return f - f.mean() if periodic else f


def test_periodic_solution_against_fft_closed_form():
    """On a periodic grid -L is diagonal in plane waves with eigenvalues
    sum_a s(theta_a)/h^2 (s the 12th-order symbol): phi_hat = 4 pi f_hat /
    eigenvalue, zero mean."""
    n, h = (16, 12, 8), 0.45
    f = rhs(n, 1, True)
    res = poisson.solve(f, n, h, True, tol=1e-13)
    F = np.fft.fftn(f.reshape(n[::-1]))  # axes (k, j, i)
    th = [2 * np.pi * np.fft.fftfreq(m) for m in n[::-1]]
    ev = sum(np.meshgrid(*[grid.laplacian_symbol(t) for t in th], indexing="ij")) / h ** 2
    ev.flat[0] = 1.0
    Phi = 4 * np.pi * F / ev
    Phi.flat[0] = 0.0
    ref = np.real(np.fft.ifftn(Phi)).reshape(-1)
    assert res.rel_resid <= 1e-13
    assert np.max(np.abs(res.phi - ref)) <= 1e-10 * np.max(np.abs(ref))


def toeplitz12(m):
    w = grid.fd_weights(6)
    diags = [w[0] * np.ones(m)]
    offs = [0]
    for p in range(1, 7):
        if p < m:
            diags += [w[p] * np.ones(m - p)] * 2
            offs += [p, -p]
    return sp.diags(diags, offs, format="csr")


def test_dirichlet_solution_against_direct_solve():
    """Zero Dirichlet: -L as a Kronecker sum of 1-D 12th-order Toeplitz
    matrices (zero padding), solved directly."""
    n, h = (11, 9, 13), 0.5
    f = rhs(n, 2, False)
    Tx, Ty, Tz = (toeplitz12(m) for m in n)
    Ix, Iy, Iz = (sp.identity(m) for m in n)
    L = (sp.kron(Iz, sp.kron(Iy, Tx)) + sp.kron(Iz, sp.kron(Ty, Ix)) + sp.kron(Tz, sp.kron(Iy, Ix))) / h ** 2
    ref = spla.spsolve((-L).tocsc(), 4 * np.pi * f)
    res = poisson.solve(f, n, h, False, tol=1e-13)
    assert np.max(np.abs(res.phi - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_seven_point_and_galerkin_operators_closed_forms():
    """A_0 applied to a quadratic equals -Lap exactly away from the faces;
    the Galerkin operator of one coarsening is (1/h^2) sum over axes of
    (T_c / 2) along that axis (x) M on the other two, M = tridiag(1/4, 3/2, 1/4)
    (Dirichlet, linear interpolation)."""
    n, h = (15, 7, 7), 0.3
    H = poisson.hierarchy(n, h, False, max_levels=2)
    assert H.sizes == [(15, 7, 7), (7, 3, 3)]
    x = np.arange(n[0]) * h
    u = np.tile(x * x, n[1] * n[2])                      # u = x^2: -Lap u = -2
    Au = (H.A[0] @ u).reshape(n[::-1])
    assert np.allclose(Au[1:-1, 1:-1, 1:-1], -2.0, atol=1e-11)

    def T(m):
        return sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])

    def M(m):
        return sp.diags([0.25 * np.ones(m - 1), 1.5 * np.ones(m), 0.25 * np.ones(m - 1)], [-1, 0, 1])

    cx, cy, cz = H.sizes[1]
    Ac = (sp.kron(M(cz), sp.kron(M(cy), T(cx) / 2)) + sp.kron(M(cz), sp.kron(T(cy) / 2, M(cx))) +
          sp.kron(T(cz) / 2, sp.kron(M(cy), M(cx)))) / h ** 2
    assert abs(H.A[1] - Ac).max() <= 1e-10 / h ** 2


@pytest.mark.parametrize("periodic", [False, True])
def test_vcycle_is_symmetric_and_positive(periodic):
    n = (8, 8, 8) if periodic else (7, 7, 15)
    H = poisson.hierarchy(n, 0.4, periodic)
    assert len(H.sizes) >= 2
    N = int(np.prod(n))
    B = np.stack([poisson.vcycle(H, e) for e in np.eye(N)], axis=1)
    assert np.max(np.abs(B - B.T)) <= 1e-12 * np.max(np.abs(B))
    ev = np.linalg.eigvalsh(0.5 * (B + B.T))
    assert ev.min() > 0


@pytest.mark.parametrize("periodic", [False, True])
def test_preconditioning_cuts_iterations(periodic):
    n = (32, 32, 32) if periodic else (31, 31, 31)
    f = rhs(n, 3, periodic)
    plain = poisson.solve(f, n, 0.4, periodic, tol=1e-8, precondition=False)
    pcg = poisson.solve(f, n, 0.4, periodic, tol=1e-8)
    assert pcg.rel_resid <= 1e-8 and plain.rel_resid <= 1e-8
    assert pcg.iters * 3 <= plain.iters, (pcg.iters, plain.iters)
    assert np.max(np.abs(pcg.phi - plain.phi)) <= 1e-6 * np.max(np.abs(plain.phi))
