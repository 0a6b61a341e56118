"""Seeded synthetic workloads for the subdomain CheFSI engine.

This module only *builds inputs*: atom positions, the local potential
V_eff restricted to a box, per-atom projector parameters, core boxes, the
random start block X0 and the Lanczos start vector.  It holds none of the
method's arithmetic (no stencil, no projector support or values, no
filter, no Rayleigh-Ritz).  Both the FP64 CPU oracle and the HIP library
receive exactly the arrays built here.

Stand-ins for the paper's workloads (Sec. VI-A: diamond Si at h ~ 0.4-0.5
bohr with 12th-order FD; a Li / solid-electrolyte interface):

* a diamond-cubic Si lattice (a = 10.26 bohr), optionally displaced;
* V_eff = sum of Gaussians at atom sites (width 0.8 bohr, depth -3 Ha
  +/- 5 %, truncated at 6.4 bohr, periodic images of the global cell);
* four Gaussian Kleinman-Bylander projectors per atom (s, px, py, pz),
  width 0.5 bohr, cut at r_c = 2 bohr, gamma_s ~ U[0.5, 1.5] Ha and
  gamma_p ~ U[0.2, 0.8] Ha (one gamma_p per atom for all three p);
* a bcc Li-like lattice (a = 6.6 bohr, depth -1 Ha) for the two-phase
  system.

Random numbers come from NumPy PCG64 streams keyed by
SeedSequence([260913115 + 1000 * cfg, index, ...]); every column of X0 has
its own stream so that any column can be regenerated on its own.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 260913115
BC_PERIODIC = 0
BC_DIRICHLET0 = 1

SI_A = 10.26          # diamond Si cubic lattice constant, bohr
LI_A = 6.6            # bcc Li-like lattice constant, bohr
VLOC_SIGMA = 0.8      # Gaussian width of the local potential, bohr
VLOC_CUT = 6.4        # truncation radius of each Gaussian (8 sigma), bohr
PROJ_RC = 2.0         # projector cutoff radius, bohr
PROJ_WIDTH = 0.5      # projector Gaussian width, bohr

DIAMOND_BASIS = np.array([
    [0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0],
    [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75], [0.75, 0.75, 0.25],
])
BCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(k) for k in key])))


# ---------------------------------------------------------------------------
# Counter-based start blocks.  Large batches draw their start blocks on the
# device; both sides implement the same published generator: Philox4x32-10
# (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
# SC 2011) and the Box-Muller transform.  Element (g, j) of a block with
# seed s uses counter (g, j, 0, 0) and key (s mod 2^32, s >> 32):
#   u1 = 1 - (2^26 (o0 >> 5) + (o1 >> 6)) / 2^53,  u2 likewise from (o2, o3),
#   x  = sqrt(-2 ln u1) cos(2 pi u2).
# ---------------------------------------------------------------------------
_PHILOX_M0 = np.uint64(0xD2511F53)
_PHILOX_M1 = np.uint64(0xCD9E8D57)
_PHILOX_W0 = 0x9E3779B9
_PHILOX_W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Philox4x32 with 10 rounds on uint32 counter arrays; returns four uint32 arrays."""
    c = [np.asarray(x, dtype=np.uint64) & _MASK32 for x in (c0, c1, c2, c3)]
    c = np.broadcast_arrays(*c)
    c = [x.copy() for x in c]
    k0, k1 = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    for _ in range(10):
        p0 = _PHILOX_M0 * c[0]
        p1 = _PHILOX_M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
        k0 = (k0 + _PHILOX_W0) & 0xFFFFFFFF
        k1 = (k1 + _PHILOX_W1) & 0xFFFFFFFF
    return [x.astype(np.uint32) for x in c]


def philox_normal_block(nd: int, ncols: int, seed: int, col0: int = 0) -> np.ndarray:
    """f64[nd, ncols] (Fortran order) of standard normals, column j drawn with
    counter column index col0 + j."""
    out = np.empty((nd, ncols), order="F")
    g = np.arange(nd, dtype=np.uint64)
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    for j in range(ncols):
        o0, o1, o2, o3 = philox4x32_10(g, col0 + j, 0, 0, k0, k1)
        a = (o0.astype(np.uint64) >> np.uint64(5)) * np.uint64(67108864) + (o1.astype(np.uint64) >> np.uint64(6))
        b = (o2.astype(np.uint64) >> np.uint64(5)) * np.uint64(67108864) + (o3.astype(np.uint64) >> np.uint64(6))
        u1 = 1.0 - a.astype(np.float64) / 9007199254740992.0
        u2 = 1.0 - b.astype(np.float64) / 9007199254740992.0
        out[:, j] = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return out


def x0_seed(key: Tuple[int, ...]) -> int:
    """64-bit seed of a subdomain's counter-based start block, from its key."""
    return int(np.random.SeedSequence([int(k) for k in key] + [0x5830]).generate_state(1, np.uint64)[0])


@dataclasses.dataclass
class Subdomain:
    """Everything the subdomain problem is defined by (Sec. V-A.2/V-A.3).

    Arrays follow the library's conventions: grid index g = i + n0*(j + n1*k)
    (x fastest), X0 column-major N_d x ns.
    """
    n: Tuple[int, int, int]
    h: float
    bc: int
    origin: Tuple[float, float, float]
    v: np.ndarray                 # f64[N_d]
    atoms: np.ndarray             # f64[n_atoms, 3]
    proj: np.ndarray              # f64[n_atoms, 6] = rc, width, gamma_s, gamma_px, gamma_py, gamma_pz
    core_lo: Tuple[int, int, int]
    core_hi: Tuple[int, int, int]
    global_offset: Tuple[int, int, int]
    global_n: Tuple[int, int, int]
    ns: int
    x0: Optional[np.ndarray] = None      # f64[N_d, ns] Fortran order
    lanczos_v0: Optional[np.ndarray] = None  # f64[N_d]
    fd_n0: int = 6
    n_valence: float = 0.0               # electrons attributed to atoms in the box
    seed_key: Tuple[int, ...] = ()
    name: str = ""

    @property
    def nd(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    def make_x0(self, ns: Optional[int] = None) -> np.ndarray:
        ns = self.ns if ns is None else ns
        x = np.empty((self.nd, ns), order="F")
        for c in range(ns):
            x[:, c] = _rng(*self.seed_key, 7, c).standard_normal(self.nd)
        return x

    def x0_column(self, c: int) -> np.ndarray:
        return _rng(*self.seed_key, 7, c).standard_normal(self.nd)

    def make_lanczos_v0(self) -> np.ndarray:
        return _rng(*self.seed_key, 11).standard_normal(self.nd)


class GlobalSystem:
    """A periodic global cell holding atoms and its global grid.

    The paper restricts a global V_eff to each buffered subdomain
    (Sec. V-A.2, V-A.5); here the global V_eff is the Gaussian sum
    evaluated once on the global grid and each subdomain is a slice of it.
    """

    def __init__(self, cell: np.ndarray, global_n: Sequence[int], atoms: np.ndarray,
                 depth: np.ndarray, gamma: np.ndarray, zval: np.ndarray, key: Tuple[int, ...]):
        self.cell = np.asarray(cell, dtype=np.float64)          # box lengths (3,)
        self.global_n = tuple(int(v) for v in global_n)
        self.h = float(self.cell[0] / self.global_n[0])
        self.atoms = np.asarray(atoms, dtype=np.float64)
        self.depth = np.asarray(depth, dtype=np.float64)
        self.gamma = np.asarray(gamma, dtype=np.float64)        # (N, 4)
        self.zval = np.asarray(zval, dtype=np.float64)
        self.key = key
        self._v = None

    # -- global potential -------------------------------------------------
    def potential(self) -> np.ndarray:
        """V_eff on the global grid, shape (n2, n1, n0) [k, j, i]."""
        if self._v is not None:
            return self._v
        n0, n1, n2 = self.global_n
        h = self.h
        v = np.zeros((n2, n1, n0))
        r = int(math.ceil(VLOC_CUT / h)) + 1
        off = np.arange(-r, r + 1)
        for X, d in zip(self.atoms, self.depth):
            c = np.floor(X / h).astype(np.int64)
            ii = c[0] + off
            jj = c[1] + off
            kk = c[2] + off
            dx = ii * h - X[0]
            dy = jj * h - X[1]
            dz = kk * h - X[2]
            r2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
            val = np.where(r2 < VLOC_CUT ** 2, d * np.exp(-r2 / (2 * VLOC_SIGMA ** 2)), 0.0)
            np.add.at(v, (np.mod(kk, n2)[:, None, None], np.mod(jj, n1)[None, :, None],
                          np.mod(ii, n0)[None, None, :]), val)
        self._v = v
        return v

    # -- subdomain extraction ---------------------------------------------
    def subdomain(self, core_lo_g: Sequence[int], core_n: Sequence[int], buf_lo: Sequence[int],
                  n: Sequence[int], ns: int, bc: int, key: Tuple[int, ...],
                  with_x0: bool = True, name: str = "") -> Subdomain:
        """Box of n points per axis whose core is the global index box
        [core_lo_g, core_lo_g + core_n), placed buf_lo points in from the low face."""
        core_lo_g = np.asarray(core_lo_g, dtype=np.int64)
        core_n = np.asarray(core_n, dtype=np.int64)
        buf_lo = np.asarray(buf_lo, dtype=np.int64)
        n = np.asarray(n, dtype=np.int64)
        if np.any(buf_lo + core_n > n) or np.any(buf_lo < 0):
            raise ValueError("core does not fit in the box")
        goff = core_lo_g - buf_lo
        h = self.h
        origin = goff * h
        vg = self.potential()
        gn = np.asarray(self.global_n)
        kk = np.mod(goff[2] + np.arange(n[2]), gn[2])
        jj = np.mod(goff[1] + np.arange(n[1]), gn[1])
        ii = np.mod(goff[0] + np.arange(n[0]), gn[0])
        v = vg[np.ix_(kk, jj, ii)].reshape(-1).copy()
        # atoms (any periodic image of the global cell) whose projector
        # support can meet the box
        top = origin + (n - 1) * h
        lo = origin - PROJ_RC
        hi = top + PROJ_RC
        L = self.cell
        if bc == BC_PERIODIC:
            # a periodic box is the whole global cell: every atom once, the
            # library sums the periodic images of its projectors itself
            if np.any(n != gn) or np.any(goff != 0):
                raise ValueError("a periodic subdomain must be the whole global cell")
            pos = self.atoms.copy()
            idx = np.arange(len(pos))
        else:
            pos, idx = [], []
            reps = [int(math.ceil((n[a] * h + 2 * PROJ_RC) / L[a])) + 1 for a in range(3)]
            for sx in range(-reps[0], reps[0] + 1):
                for sy in range(-reps[1], reps[1] + 1):
                    for sz in range(-reps[2], reps[2] + 1):
                        P = self.atoms + np.array([sx, sy, sz]) * L
                        m = np.all((P > lo) & (P < hi), axis=1)
                        pos.append(P[m])
                        idx.append(np.nonzero(m)[0])
            pos = np.concatenate(pos)
            idx = np.concatenate(idx)
        order = np.lexsort((pos[:, 0], pos[:, 1], pos[:, 2]))
        pos, idx = pos[order], idx[order]
        proj = np.zeros((len(pos), 6))
        proj[:, 0] = PROJ_RC
        proj[:, 1] = PROJ_WIDTH
        proj[:, 2:] = self.gamma[idx]
        inbox = np.all((pos >= origin) & (pos <= top), axis=1)
        sd = Subdomain(
            n=tuple(int(x) for x in n), h=h, bc=bc, origin=tuple(float(x) for x in origin),
            v=v, atoms=pos, proj=proj,
            core_lo=tuple(int(x) for x in buf_lo), core_hi=tuple(int(x) for x in buf_lo + core_n),
            global_offset=tuple(int(x) for x in goff), global_n=tuple(int(x) for x in gn),
            ns=int(ns), seed_key=tuple(key), name=name,
            n_valence=float(self.zval[idx[inbox]].sum()))
        if with_x0:
            sd.x0 = sd.make_x0()
            sd.lanczos_v0 = sd.make_lanczos_v0()
        return sd


def diamond_si_system(ncells: int, global_n: int, displacement: float, key: Tuple[int, ...],
                      depth: float = -3.0) -> GlobalSystem:
    rng = _rng(*key, 1)
    cells = np.array([[i, j, k] for k in range(ncells) for j in range(ncells) for i in range(ncells)])
    frac = (cells[:, None, :] + DIAMOND_BASIS[None, :, :]).reshape(-1, 3)
    atoms = frac * SI_A
    if displacement > 0:
        atoms = atoms + rng.uniform(-displacement, displacement, size=atoms.shape)
    n = len(atoms)
    d = depth * (1.0 + 0.05 * rng.uniform(-1.0, 1.0, size=n))
    gamma = np.empty((n, 4))
    gamma[:, 0] = rng.uniform(0.5, 1.5, size=n)
    gp = rng.uniform(0.2, 0.8, size=n)
    gamma[:, 1:] = gp[:, None]
    L = ncells * SI_A
    return GlobalSystem(np.array([L, L, L]), (global_n,) * 3, atoms, d, gamma,
                        np.full(n, 4.0), key)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def workload_key(tag: int, index: int = 0) -> Tuple[int, int]:
    return (SEED_BASE + 1000 * tag, index)


def periodic_si_cell(n: int = 24, ns: int = 20, key: Tuple[int, ...] = workload_key(1),
                     with_x0: bool = True) -> Subdomain:
    """One periodic 8-atom diamond cell on an n^3 grid (h = a/n)."""
    gs = diamond_si_system(1, n, 0.0, key)
    return gs.subdomain((0, 0, 0), (n, n, n), (0, 0, 0), (n, n, n), ns, BC_PERIODIC, key,
                        with_x0, name=f"periodic Si cell {n}^3 ns={ns}")


def si_cell_24(with_x0: bool = True) -> Subdomain:
    """Periodic 8-atom diamond cell, 24^3 grid (h = 0.4275), ns = 20."""
    return periodic_si_cell(24, 20, workload_key(1), with_x0)


def dirichlet_si_box(n: int, ns: int, key: Tuple[int, ...], ncells: int = 4,
                     core_cells: int = 2, h_target: float = 0.43, displacement: float = 0.1,
                     with_x0: bool = True) -> Subdomain:
    """A zero-Dirichlet n^3 box centred on a core of core_cells^3 diamond cells.

    The core is the index box of grid points whose coordinate lies in
    [a, a + core_cells * a) (first index ceil(x/h)); the rest of the box is buffer."""
    gn = int(round(ncells * SI_A / h_target))
    gs = diamond_si_system(ncells, gn, displacement, key)
    h = gs.h
    lo = int(math.ceil(SI_A / h - 1e-12))
    hi = int(math.ceil((SI_A + core_cells * SI_A) / h - 1e-12))
    core_n = hi - lo
    if n < core_n:
        raise ValueError("box smaller than core")
    b0 = (n - core_n) // 2
    return gs.subdomain((lo,) * 3, (core_n,) * 3, (b0,) * 3, (n,) * 3, ns, BC_DIRICHLET0, key,
                        with_x0, name=f"Dirichlet Si box {n}^3 ns={ns}")


def si_box_64(with_x0: bool = True, ns: int = 480) -> Subdomain:
    """64-atom displaced diamond core in a zero-Dirichlet 64^3 box, h ~ 0.43, ns = 480."""
    return dirichlet_si_box(64, ns, workload_key(2), with_x0=with_x0)


def si_box_96(with_x0: bool = False, ns: int = 2400) -> Subdomain:
    """96^3 zero-Dirichlet Si box (3x3x3-cell core), ns = 2400."""
    return dirichlet_si_box(96, ns, workload_key(4), ncells=5, core_cells=3, with_x0=with_x0)


def small_periodic(n: int = 8, ns: int = 8, index: int = 0, with_x0: bool = True) -> Subdomain:
    """Periodic diamond cell on a coarse n^3 grid (h = 10.26/n) for brute-force checks."""
    return periodic_si_cell(n, ns, (SEED_BASE + 90000, index), with_x0)


def small_dirichlet(n: int = 8, ns: int = 8, index: int = 0, with_x0: bool = True,
                    h: float = 0.9, shape: Optional[Sequence[int]] = None) -> Subdomain:
    """A small zero-Dirichlet box cut from a displaced diamond crystal (brute-force size).

    shape overrides the cubic n (for ragged boxes)."""
    key = (SEED_BASE + 91000, index)
    gn = int(round(2 * SI_A / h))
    gs = diamond_si_system(2, gn, 0.1, key)
    shp = np.asarray(shape if shape is not None else (n, n, n), dtype=np.int64)
    core = np.maximum(shp - 2, 1)
    buf = np.minimum(np.ones(3, dtype=np.int64), shp - core)
    return gs.subdomain((3, 4, 5), core, buf, shp, ns, BC_DIRICHLET0, key, with_x0,
                        name=f"small Dirichlet {tuple(int(x) for x in shp)}")


def batch_subdomains(count: int = 256, key_cfg: int = 3, with_x0: bool = False,
                     ncells: int = 10, h_target: float = 0.43,
                     nmin: int = 40, nmax: int = 80, core_atoms: Tuple[int, int] = (27, 125),
                     ) -> Tuple[GlobalSystem, List[Subdomain], List[int]]:
    """Uneven buffered subdomains of one large displaced diamond crystal.

    Core atom count n_c ~ U{27..125}, buffer R ~ U[3, 6] bohr, core side
    s = (n_c a^3 / 8)^(1/3), n = clamp(round((s + 2R)/h), nmin, nmax),
    ns = clamp(ceil(2.2 * atoms in box), 60, 900), degree m ~ U{16..32}.
    Returns (global system, subdomains, degrees).  core_atoms widens or
    narrows the n_c range (smaller boxes of the same recipe, e.g. to train
    learned bounds on).
    """
    key = (SEED_BASE + 1000 * key_cfg, 0)
    gn = int(round(ncells * SI_A / h_target))
    gs = diamond_si_system(ncells, gn, 0.1, key)
    h = gs.h
    rng = _rng(*key, 3)
    subs, degs = [], []
    for b in range(count):
        nc = int(rng.integers(core_atoms[0], core_atoms[1] + 1))
        R = float(rng.uniform(3.0, 6.0))
        s = (nc * SI_A ** 3 / 8.0) ** (1.0 / 3.0)
        n = int(min(max(round((s + 2 * R) / h), nmin), nmax))
        core_n = int(min(max(round(s / h), 1), n - 2))
        b0 = (n - core_n) // 2
        start = rng.integers(0, gn, size=3)
        m = int(rng.integers(16, 33))
        sd = gs.subdomain(tuple(int(x) for x in start), (core_n,) * 3, (b0,) * 3, (n,) * 3, 60,
                          BC_DIRICHLET0, key + (b,), with_x0=False)
        org = np.asarray(sd.origin)
        natoms_box = int(np.sum(np.all((sd.atoms >= org) & (sd.atoms <= org + (n - 1) * h), axis=1)))
        sd.ns = int(min(max(math.ceil(2.2 * natoms_box), 60), 900))
        sd.name = f"batch[{b}] n={n} ns={sd.ns} m={m}"
        if with_x0:
            sd.x0 = sd.make_x0()
            sd.lanczos_v0 = sd.make_lanczos_v0()
        subs.append(sd)
        degs.append(m)
    return gs, subs, degs


def two_phase_system(key: Tuple[int, ...] = (SEED_BASE + 5000 * 1, 0), n_xy: int = 34,
                     interface: float = 5.0, min_dist: float = 3.0) -> GlobalSystem:
    """Diamond Si (z < Lz/2) joined to a bcc Li-like phase (z >= Lz/2) in a
    periodic 2x2x4 Si-cell box; atoms within `interface` bohr of either
    interface plane are kept with probability 1/2 and displaced by U[-1, 1]
    bohr per axis, all others by U[-0.1, 0.1]; sites closer than `min_dist`
    to an already kept site are dropped.  The bcc constant is Lx/3 = 6.84
    bohr (6.6 stretched so that the lattice tiles the periodic cell).
    Depths: Si -3 Ha, Li -1 Ha (both +/- 5 %); gamma_s/gamma_p ~ U[0.5, 1.5]/
    U[0.2, 0.8] Ha for Si and U[0.2, 0.6]/U[0.1, 0.3] Ha for Li."""
    rng = _rng(*key, 1)
    Lx = 2 * SI_A
    Lz = 4 * SI_A
    a_li = Lx / 3.0
    si = np.array([[i, j, k] for k in range(2) for j in range(2) for i in range(2)])
    si = ((si[:, None, :] + DIAMOND_BASIS[None]).reshape(-1, 3)) * SI_A
    li = np.array([[i, j, k] for k in range(3) for j in range(3) for i in range(3)])
    li = ((li[:, None, :] + BCC_BASIS[None]).reshape(-1, 3)) * a_li
    li[:, 2] += Lz / 2
    sites = np.concatenate([si, li])
    kind = np.concatenate([np.zeros(len(si), dtype=np.int64), np.ones(len(li), dtype=np.int64)])
    z = sites[:, 2]
    near = (np.abs(z - Lz / 2) < interface) | (z < interface) | (z > Lz - interface)
    keep = ~near | (rng.uniform(size=len(sites)) < 0.5)
    disp = np.where(near[:, None], 1.0, 0.1)
    sites = sites + rng.uniform(-1.0, 1.0, size=sites.shape) * disp
    cell = np.array([Lx, Lx, Lz])
    order = rng.permutation(len(sites))
    kept = []
    for i in order:
        if not keep[i]:
            continue
        ok = True
        for j in kept:
            d = sites[i] - sites[j]
            d -= cell * np.round(d / cell)
            if np.dot(d, d) < min_dist ** 2:
                ok = False
                break
        if ok:
            kept.append(i)
    kept = np.sort(np.asarray(kept))
    atoms = np.mod(sites[kept], cell)
    kind = kind[kept]
    n = len(atoms)
    depth = np.where(kind == 0, -3.0, -1.0) * (1.0 + 0.05 * rng.uniform(-1.0, 1.0, size=n))
    gamma = np.empty((n, 4))
    gs = np.where(kind == 0, rng.uniform(0.5, 1.5, size=n), rng.uniform(0.2, 0.6, size=n))
    gp = np.where(kind == 0, rng.uniform(0.2, 0.8, size=n), rng.uniform(0.1, 0.3, size=n))
    gamma[:, 0] = gs
    gamma[:, 1:] = gp[:, None]
    zval = np.where(kind == 0, 4.0, 1.0)
    return GlobalSystem(cell, (n_xy, n_xy, 2 * n_xy), atoms, depth, gamma, zval, key)


def learned_bounds_subdomains(count: int, index0: int = 0, gs: Optional[GlobalSystem] = None,
                              nmin: int = 14, nmax: int = 22) -> Tuple[GlobalSystem, List[Subdomain]]:
    """Small zero-Dirichlet training boxes at random places of the two-phase
    system (Si, Li and the interfaces): n ~ U{nmin..nmax} per axis, buffer
    b ~ U{2..4} points, ns = clamp(ceil(1.1 * electrons in the box / 2), 8, 48)."""
    gs = two_phase_system() if gs is None else gs
    subs = []
    for b in range(index0, index0 + count):
        rng = _rng(*gs.key, 2, b)
        n = rng.integers(nmin, nmax + 1, size=3)
        buf = rng.integers(2, 5, size=3)
        core = n - 2 * buf
        start = rng.integers(0, np.asarray(gs.global_n), size=3)
        sd = gs.subdomain(tuple(int(x) for x in start), core, buf, n, 8, BC_DIRICHLET0, gs.key + (b,),
                          with_x0=False)
        sd.ns = int(min(max(math.ceil(1.1 * sd.n_valence / 2.0), 8), 48))
        sd.name = f"two-phase[{b}] n={tuple(int(x) for x in n)} ns={sd.ns}"
        sd.x0 = sd.make_x0()
        sd.lanczos_v0 = sd.make_lanczos_v0()
        subs.append(sd)
    return gs, subs


def diagonal_spectrum(n: int, key: Tuple[int, ...] = (SEED_BASE + 95000, 0),
                      lo: float = -1.0, hi: float = 10.0) -> np.ndarray:
    """Sorted random diagonal entries for operator-level closed-form checks."""
    return np.sort(_rng(*key).uniform(lo, hi, size=n))


def random_block(nd: int, ns: int, key: Tuple[int, ...]) -> np.ndarray:
    x = np.empty((nd, ns), order="F")
    for c in range(ns):
        x[:, c] = _rng(*key, 7, c).standard_normal(nd)
    return x


def mlp_init(sizes: Sequence[int] = (64, 128, 128, 3), seed: int = 0) -> List[np.ndarray]:
    """He-normal initial weights and zero biases of an MLP with the given layer
    widths, as [W1, b1, W2, b2, ...] with W_l of shape (fan_in, fan_out)."""
    rng = _rng(SEED_BASE + 5000, seed)
    out = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        out.append(rng.standard_normal((a, b)) * np.sqrt(2.0 / a))
        out.append(np.zeros(b))
    return out


def minibatch_order(n: int, batch: int, epochs: int, seed: int = 0) -> List[np.ndarray]:
    """Index lists of the minibatches of `epochs` shuffled passes over n samples."""
    rng = _rng(SEED_BASE + 6000, seed)
    out = []
    for _ in range(epochs):
        perm = rng.permutation(n)
        for s in range(0, n, batch):
            out.append(perm[s:s + batch])
    return out
