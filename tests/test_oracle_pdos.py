"""Pins of the oracle's projected density of states (Sec. V-A.4)."""
from types import SimpleNamespace

import numpy as np
import pytest

from oracle import pdos


def box(n=6, h=0.7, atoms=((2.1, 2.1, 2.1), (0.7, 1.4, 2.8)), periodic=False):
    return SimpleNamespace(n=(n, n, n), h=h, origin=(0.0, 0.0, 0.0), bc=0 if periodic else 1,
                           atoms=np.array(atoms), core_lo=(1, 1, 1), core_hi=(5, 5, 5))


@pytest.mark.parametrize("periodic", [False, True])
def test_weights_over_a_complete_basis_sum_to_one(periodic):
    """Parseval: over any orthonormal basis of the grid functions, the weights
    of one atomic orbital sum to h^3 sum phi^2 = 1."""
    sd = box(periodic=periodic)
    t = pdos.orbital_tables(sd, 0.6, 1.5)
    Q, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((216, 216)))
    P = pdos.weights(t, Q, sd.h)
    assert np.allclose(P.sum(axis=0), 1.0, atol=1e-12)


def test_a_state_equal_to_an_orbital():
    """psi = h^(3/2) phi_s of a node-centred atom: weight 1 on that s orbital,
    0 on its p orbitals (odd along their axis), and the state's weights on
    the other atom are its squared overlaps."""
    sd = box(n=9, atoms=((2.8, 2.8, 2.8),))
    t = pdos.orbital_tables(sd, 0.6, 1.8)
    psi = np.zeros((729, 1))
    psi[t.idx, 0] = t.val[:, 0] * sd.h ** 1.5
    assert np.linalg.norm(psi) == pytest.approx(1.0, rel=1e-14)
    P = pdos.weights(t, psi, sd.h)
    assert P[0, 0] == pytest.approx(1.0, rel=1e-13)
    assert np.all(np.abs(P[0, 1:4]) < 1e-28)


def test_bins_and_core_membership():
    sd = box(atoms=((2.1, 2.1, 2.1), (0.7, 1.4, 2.8), (3.4, 3.4, 3.4)))
    inc = pdos.atoms_in_core(sd)
    # core = [0.7, 3.5) per axis: the first and third atoms are in, the second
    # is in (0.7 <= 0.7); move it out along y to check the strict upper edge
    assert list(inc) == [True, True, True]
    sd2 = box(atoms=((2.1, 3.5, 2.1), (0.69, 1.4, 2.8)))
    assert list(pdos.atoms_in_core(sd2)) == [False, False]
    P = np.arange(16, dtype=float).reshape(4, 4)   # 4 states, the 4 orbitals of one atom
    lam = np.array([-1.0, 0.5, 0.5, 2.0])
    D = pdos.pdos(P, lam, np.array([0.0, 1.0, 2.0]), np.array([True]))
    assert np.array_equal(D[:, 0], P[1] + P[2]) and np.array_equal(D[:, 1], P[3])
    assert np.all(pdos.pdos(P, lam, np.array([0.0, 1.0, 2.0]), np.array([False])) == 0.0)
