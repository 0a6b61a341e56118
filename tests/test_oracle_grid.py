"""Pins of the oracle's grid pieces: FD weights, Laplacian, maps.

Every check compares the oracle with something other than itself: printed
rationals, exact polynomial arithmetic, the plane-wave closed form, a
Kronecker-sum assembly, and an integer tiling argument."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import grid
from oracle import hamiltonian

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_fd():
    vals = []
    with open(os.path.join(GOLDEN, "fd_weights_n6.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                vals.append(Fraction(line))
    return vals


def test_fd_weights_match_printed_table():
    assert grid.fd_weights_exact(6) == _golden_fd()


@pytest.mark.parametrize("n0", range(1, 9))
def test_fd_w0_equals_minus_two_sum_inverse_squares(n0):
    w = grid.fd_weights_exact(n0)
    assert w[0] == -2 * sum(Fraction(1, p * p) for p in range(1, n0 + 1))


@pytest.mark.parametrize("n0", [1, 3, 6])
def test_fd_polynomial_exactness(n0):
    """Exact rational arithmetic: the 2*n0-order stencil differentiates x^q
    exactly for q <= 2*n0 + 1 and not for q = 2*n0 + 2."""
    w = grid.fd_weights_exact(n0)
    x = Fraction(3, 7)
    for q in range(0, 2 * n0 + 3):
        approx = w[0] * x ** q + sum(w[p] * ((x + p) ** q + (x - p) ** q) for p in range(1, n0 + 1))
        exact = q * (q - 1) * x ** (q - 2) if q >= 2 else Fraction(0)
        if q <= 2 * n0 + 1:
            assert approx == exact, (n0, q)
        else:
            assert approx != exact


def _symbol(theta, n0=6):
    w = [float(v) for v in _golden_fd()] if n0 == 6 else None
    return -w[0] - 2 * sum(w[p] * np.cos(p * theta) for p in range(1, 7))


@pytest.mark.parametrize("n,h", [((8, 8, 8), 1.2825), ((24, 24, 24), 0.4275), ((6, 10, 7), 0.5)])
def test_periodic_plane_wave_eigenvalues(n, h):
    """-1/2 L on a periodic grid has plane waves as eigenvectors with
    eigenvalue (1/(2h^2)) sum_a s(theta_a), s(theta) = -w_0 - 2 sum w_p cos(p theta)."""
    rng = np.random.default_rng(5)
    op = hamiltonian.free_operator(n, h, True)
    i, j, k = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    for _ in range(4):
        m = [int(rng.integers(0, n[a])) for a in range(3)]
        th = [2 * np.pi * m[a] / n[a] for a in range(3)]
        phase = th[0] * i + th[1] * j + th[2] * k
        psi = np.cos(phase).reshape(-1, order="F")
        lam = sum(_symbol(t) for t in th) / (2 * h * h)
        out = op.apply(psi)
        assert np.allclose(out, lam * psi, atol=1e-10 * max(1, abs(lam)))


def test_periodic_lambda_max_si_cell_24():
    """Checkerboard mode (-1)^(i+j+k) on the 24^3, h = 0.4275 grid:
    lambda_max = 1.5 s(pi) / h^2 = 58.0522 Ha."""
    n, h = (24, 24, 24), 0.4275
    op = hamiltonian.free_operator(n, h, True)
    i, j, k = np.meshgrid(np.arange(24), np.arange(24), np.arange(24), indexing="ij")
    psi = ((-1.0) ** (i + j + k)).reshape(-1, order="F")
    out = op.apply(psi)
    lam = out @ psi / (psi @ psi)
    assert abs(lam - 58.0522) < 5e-4
    assert np.allclose(out, lam * psi, atol=1e-10)


def _toeplitz_1d(n, periodic, n0=6):
    w = [float(v) for v in grid.fd_weights_exact(n0)]
    T = np.zeros((n, n))
    for i in range(n):
        T[i, i] += w[0]
        for p in range(1, n0 + 1):
            for jj in (i + p, i - p):
                if periodic:
                    T[i, jj % n] += w[p]
                elif 0 <= jj < n:
                    T[i, jj] += w[p]
    return T


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("n", [(8, 8, 8), (5, 7, 4), (3, 9, 2)])
def test_laplacian_kronecker_sum(periodic, n):
    """Dense L from the oracle equals the Kronecker sum of 1-D stencil matrices
    (x fastest: L = I_z (x) I_y (x) T_x + I_z (x) T_y (x) I_x + T_z (x) I_y (x) I_x)."""
    h = 0.7
    op = hamiltonian.free_operator(n, h, periodic)
    Hd = op.dense()
    Tx, Ty, Tz = (_toeplitz_1d(n[a], periodic) for a in range(3))
    Ix, Iy, Iz = (np.eye(n[a]) for a in range(3))
    L = (np.kron(Iz, np.kron(Iy, Tx)) + np.kron(Iz, np.kron(Ty, Ix)) + np.kron(Tz, np.kron(Iy, Ix))) / h ** 2
    assert np.allclose(Hd, -0.5 * L, atol=1e-13 * np.abs(L).max())
    assert np.allclose(Hd, Hd.T, atol=1e-13 * np.abs(L).max())


def test_symbol_is_twelfth_order():
    """s(theta) = theta^2 + O(theta^14): at theta = 0.1 the difference is < 1e-13."""
    for th in (0.1, 0.05):
        assert abs(_symbol(th) - th * th) < 1e-13


def test_core_masks_tile_a_periodic_grid():
    """Disjoint cores tile the global grid; local->global is injective on cores."""
    gn = (10, 9, 8)
    cuts = [(0, 4, 10), (0, 3, 5, 9), (0, 8)]
    buf = (2, 3, 1)
    seen = np.zeros(np.prod(gn), dtype=np.int64)
    for a0, a1 in zip(cuts[0][:-1], cuts[0][1:]):
        for b0, b1 in zip(cuts[1][:-1], cuts[1][1:]):
            for c0, c1 in zip(cuts[2][:-1], cuts[2][1:]):
                core_n = np.array([a1 - a0, b1 - b0, c1 - c0])
                n = core_n + 2 * np.array(buf)
                goff = np.array([a0, b0, c0]) - np.array(buf)
                mask = grid.core_mask(n, buf, np.array(buf) + core_n)
                G = grid.global_index(n, goff, gn)
                assert G.min() >= 0 and G.max() < np.prod(gn)
                core_G = G[mask.astype(bool)]
                assert len(np.unique(core_G)) == len(core_G) == int(np.prod(core_n))
                seen[core_G] += 1
    assert np.all(seen == 1)


def test_global_index_wraps_negative_offsets():
    G = grid.global_index((3, 1, 1), (-1, 0, 0), (5, 1, 1))
    assert list(G) == [4, 0, 1]


def test_philox_known_answers():
    """The counter-based start-block generator reproduces the published
    Philox4x32-10 known-answer vectors (tests/golden/philox4x32_10_kat.txt)."""
    import os
    from paper_2609_13115_amd import workloads
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = workloads.philox4x32_10(*v[0:4], v[4], v[5])
        assert [int(x) for x in out] == v[6:10]
