"""Multigrid-preconditioned Poisson CG (Sec. V-B.1) through the C ABI,
against the oracle.

* One V-cycle (FP32 on the GPU) against the oracle's FP64 V-cycle on the
  same vector: 1e-5 relative (FP32 arithmetic over a few dozen operations
  per point and level).
* Solves (tol 1e-10) on zero-Dirichlet (31^3, 63^3, ragged 15 x 31 x 7) and
  periodic (32^3, 16 x 32 x 8) grids: the solution within 1e-8 relative of
  the oracle's, the iteration count within 2 of the oracle's (the FP32
  V-cycle perturbs the Krylov recurrence slightly), and unpreconditioned
  CG reaching the same solution in many more iterations.
* At 127^3 (Dirichlet) and 128^3 (periodic): the residual of the GPU
  solution recomputed with the oracle's operator, and for the periodic grid
  the FFT closed form of the 12th-order symbol.
"""
import numpy as np
import pytest

from oracle import grid, poisson
from paper_2609_13115_amd import xls

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[case] {msg}", flush=True)


def rhs(n, seed, periodic):
    f = np.random.default_rng(seed).standard_normal(int(np.prod(n)))
    return f - f.mean() if periodic else f


CASES = [((31, 31, 31), False), ((63, 63, 63), False), ((15, 31, 7), False), ((32, 32, 32), True),
         ((16, 32, 8), True)]


@pytest.mark.parametrize("n,periodic", CASES)
def test_vcycle_matches_oracle(n, periodic):
    case(f"poisson vcycle {n} periodic={periodic}")
    h = 0.45
    r = rhs(n, 5, periodic)
    H = poisson.hierarchy(n, h, periodic)
    ref = poisson.vcycle(H, r)
    with xls.Poisson(n, h, 0 if periodic else 1) as p:
        z = p.vcycle(r)
    assert np.linalg.norm(z - ref) <= 1e-5 * np.linalg.norm(ref)


@pytest.mark.parametrize("n,periodic", CASES)
def test_solve_matches_oracle(n, periodic):
    case(f"poisson solve {n} periodic={periodic}")
    h = 0.45
    f = rhs(n, 6, periodic)
    ref = poisson.solve(f, n, h, periodic, tol=1e-10)
    with xls.Poisson(n, h, 0 if periodic else 1) as p:
        phi, info = p.solve(f, tol=1e-10)
        phi0, info0 = p.solve(f, tol=1e-10, max_iter=3000, precondition=False)
    print(f"[poisson] {n} periodic={periodic}: pcg {info[0]} it (oracle {ref.iters}), cg {info0[0]} it, "
          f"levels {info[2]}, {info[3]:.1f} ms", flush=True)
    assert info[1] <= 1e-10 and abs(info[0] - ref.iters) <= 2
    assert np.linalg.norm(phi - ref.phi) <= 1e-8 * np.linalg.norm(ref.phi)
    assert info0[1] <= 1e-10 and info0[0] > 3 * info[0]
    assert np.linalg.norm(phi0 - ref.phi) <= 1e-8 * np.linalg.norm(ref.phi)


@pytest.mark.parametrize("n,periodic", [((127, 127, 127), False), ((128, 128, 128), True)])
def test_large_grid_residual_and_closed_form(n, periodic):
    case(f"poisson large {n} periodic={periodic}")
    h = 0.4
    f = rhs(n, 7, periodic)
    with xls.Poisson(n, h, 0 if periodic else 1) as p:
        phi, info = p.solve(f, tol=1e-10)
    b = 4 * np.pi * f
    r = b - poisson.apply_A(phi, n, h, periodic)
    print(f"[poisson] {n}: {info[0]} it, levels {info[2]}, {info[3]:.1f} ms", flush=True)
    assert info[1] <= 1e-10 and np.linalg.norm(r) <= 1.5e-10 * np.linalg.norm(b)
    assert info[0] <= 20
    if periodic:
        F = np.fft.fftn(f.reshape(n[::-1]))
        th = [2 * np.pi * np.fft.fftfreq(m) for m in n[::-1]]
        ev = sum(np.meshgrid(*[grid.laplacian_symbol(t) for t in th], indexing="ij")) / h ** 2
        ev.flat[0] = 1.0
        Phi = 4 * np.pi * F / ev
        Phi.flat[0] = 0.0
        ref = np.real(np.fft.ifftn(Phi)).reshape(-1)
        assert np.linalg.norm(phi - ref) <= 1e-8 * np.linalg.norm(ref)


def test_solve_device_matches_host_solve():
    """xls_poisson_solve_device runs the same solve on device arrays: the
    same iterations and bit-identical phi; host memory is refused."""
    import torch

    case("poisson device-array solve")
    n = (31, 15, 23)
    f = rhs(n, 3, False)
    fd = torch.tensor(f, dtype=torch.float64, device="cuda")
    pd = torch.zeros_like(fd)
    with xls.Poisson(n, 0.4, 1) as p:
        phi, info = p.solve(f, tol=1e-10)
        info_d = p.solve_device(fd, pd, tol=1e-10)
        with pytest.raises(ValueError):
            p.solve_device(fd.cpu(), pd, tol=1e-10)
    assert info_d[0] == info[0] and info_d[1] == info[1]
    assert np.array_equal(pd.cpu().numpy(), phi)
