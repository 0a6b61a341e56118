"""The subdomain Hamiltonian H^alpha (oracle, test infrastructure only).

H = -1/2 Lap + V_eff + V_nl (Sec. V, eq. (ks)), with V_eff the global
effective potential restricted to the subdomain (Sec. V-A.2) and the
Laplacian and projector parts from grid.py / projectors.py.
Pins: Kronecker-sum dense assembly, symmetry, plane-wave spectrum
(tests/test_oracle_grid.py, tests/test_oracle_projectors.py).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import grid, projectors


@dataclass
class Operator:
    n: tuple
    h: float
    periodic: bool
    v: np.ndarray
    proj: Optional[projectors.ProjectorTables]
    n0: int = 6

    @property
    def nd(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    def apply(self, psi: np.ndarray) -> np.ndarray:
        squeeze = psi.ndim == 1
        X = psi.reshape(-1, 1) if squeeze else psi
        out = -0.5 * grid.laplacian(X, self.n, self.h, self.periodic, self.n0) + self.v[:, None] * X
        if self.proj is not None:
            out = out + projectors.apply_vnl(self.proj, X, self.h)
        return out[:, 0] if squeeze else out

    def dense(self) -> np.ndarray:
        """Dense H by applying H to the unit vectors (small grids only)."""
        return self.apply(np.eye(self.nd))


def from_subdomain(sd, with_nonlocal: bool = True) -> Operator:
    periodic = sd.bc == 0
    tables = None
    if with_nonlocal and len(sd.atoms):
        tables = projectors.build(sd.n, sd.h, sd.origin, periodic, sd.atoms, sd.proj)
    return Operator(tuple(int(x) for x in sd.n), float(sd.h), periodic,
                    np.asarray(sd.v, dtype=np.float64), tables, int(sd.fd_n0))


def free_operator(n: Sequence[int], h: float, periodic: bool, v: Optional[np.ndarray] = None,
                  n0: int = 6) -> Operator:
    nd = int(n[0] * n[1] * n[2])
    vv = np.zeros(nd) if v is None else np.asarray(v, dtype=np.float64)
    return Operator(tuple(int(x) for x in n), float(h), periodic, vv, None, n0)
