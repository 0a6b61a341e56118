"""Projected density of states of a subdomain (oracle, test infrastructure only).

The paper evaluates the PDOS by projecting the local Kohn-Sham orbitals
onto atom-centred atomic orbitals phi_{I,lm} of the atoms whose positions
lie in the core region: the weight of orbital n is the squared overlap
|int phi* psi_n|^2, the orbital-resolved PDOS puts that weight at the
orbital's eigenvalue, and atom- and species-resolved PDOS sum over the
atom's orbitals and over a species' atoms (Sec. V-A.4, the PDOS
equations).

Discrete form used here.  psi_n are unit 2-norm columns (the continuum
orbital is psi_n / h^(3/2)); the atomic orbitals are synthetic s and p
Gaussians of the projector shape (the paper's atomic orbitals come with its
pseudopotentials, which are not available), built by projectors.build with
unit coefficients and normalised so that h^3 sum phi^2 = 1.  Then
  P[n, 4I + l] = h^3 (sum_g phi_{I,l}(g) psi_n(g))^2,
and the PDOS of a set of bins with increasing edges is
  D[4I + l, b] = sum over n with lambda_n in [e_b, e_{b+1}) of P[n, 4I + l]
(the last bin closed), for atoms in the core and 0 for the others.  An atom
is in the core iff core_lo[a] h <= X_a - origin_a < core_hi[a] h on every
axis.
Pins (tests/test_oracle_pdos.py): over a complete orthonormal basis the
weights of each orbital sum to 1 (Parseval); a state equal to an orbital
has weight 1 on it and 0 on the orbitals orthogonal to it; the bins sum to
the weights of the states inside the edges.
"""
from __future__ import annotations

import numpy as np

from . import projectors


def orbital_tables(sd, width: float, rc: float):
    """Support lists and values of the atomic orbitals (s, px, py, pz per atom)."""
    atoms = np.asarray(sd.atoms, dtype=np.float64).reshape(-1, 3)
    proj = np.zeros((len(atoms), 6))
    proj[:, 0] = rc
    proj[:, 1] = width
    proj[:, 2:] = 1.0
    return projectors.build(sd.n, sd.h, sd.origin, int(sd.bc) == 0, atoms, proj)


def atoms_in_core(sd) -> np.ndarray:
    atoms = np.asarray(sd.atoms, dtype=np.float64).reshape(-1, 3)
    out = np.ones(len(atoms), dtype=bool)
    for a in range(3):
        x = atoms[:, a] - sd.origin[a]
        out &= (sd.core_lo[a] * sd.h <= x) & (x < sd.core_hi[a] * sd.h)
    return out


def weights(t: projectors.ProjectorTables, psi: np.ndarray, h: float) -> np.ndarray:
    """P[n, 4 I + l] = h^3 (sum_{g in S_I} phi_{I,l}(g) psi_n(g))^2."""
    na = len(t.offsets) - 1
    P = np.zeros((psi.shape[1], 4 * na))
    for a in range(na):
        s0, s1 = t.offsets[a], t.offsets[a + 1]
        S = t.idx[s0:s1]
        ov = t.val[s0:s1].T @ psi[S, :]          # (4, ns) overlaps sum phi psi
        P[:, 4 * a:4 * a + 4] = h ** 3 * (ov * ov).T
    return P


def pdos(P: np.ndarray, lam: np.ndarray, edges: np.ndarray, in_core: np.ndarray) -> np.ndarray:
    """D[j, b]: the weights of orbital j over the states in bin b; orbitals of
    atoms outside the core get 0."""
    nb = len(edges) - 1
    D = np.zeros((P.shape[1], nb))
    for n, e in enumerate(lam):
        if e < edges[0] or e > edges[-1]:
            continue
        b = int(np.searchsorted(edges, e, side="right")) - 1
        b = min(b, nb - 1)
        D[:, b] += P[n]
    D[np.repeat(~np.asarray(in_core, dtype=bool), 4)] = 0.0
    return D
