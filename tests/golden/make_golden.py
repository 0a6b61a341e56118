"""Writes the stored expected values under tests/golden/ from the FP64 oracle.

    python tests/golden/make_golden.py box64

Only oracle/ and the seeded input builders (workloads) are called; nothing
here touches the HIP library.  Each output file records the recipe it was
made from.

box64: the 64^3 zero-Dirichlet Si box of the bench (64-atom displaced
diamond core, h = 0.432, degree 24) with the start block cut to its first
NS columns.  The oracle takes Lanczos bounds (k = 20, its own start vector)
for the first iteration and runs CheFSI (Sec. V-A.3) until the largest
residual over the gated states is <= 1e-4; the file holds those bounds, the
iteration count, and the Ritz values and residuals after the last
iteration.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import chefsi, hamiltonian  # noqa: E402
from paper_2609_13115_amd import workloads  # noqa: E402

BOX64_NS = 40
BOX64_DEGREE = 24


def box64_path() -> str:
    return os.path.join(HERE, f"box64_ns{BOX64_NS}_m{BOX64_DEGREE}.txt")


def make_box64() -> str:
    sd = workloads.si_box_64(with_x0=True, ns=BOX64_NS)
    op = hamiltonian.from_subdomain(sd)
    t0 = time.time()
    lo, up = chefsi.lanczos_bounds(op.apply, sd.lanczos_v0, 20)
    lc = chefsi.first_cutoff(lo, up)
    res = chefsi.chefsi(op.apply, sd.x0, BOX64_DEGREE, 60, lo, lc, up, resid_tol=1e-4)
    gate = chefsi.n_gate(sd.ns)
    path = box64_path()
    with open(path, "w") as f:
        f.write("# FP64 oracle CheFSI on the 64^3 zero-Dirichlet Si box (workloads.si_box_64,\n")
        f.write(f"# first {BOX64_NS} start columns), degree {BOX64_DEGREE}, first-iteration bounds from\n")
        f.write("# 20 Lanczos steps, run until the gated residual is <= 1e-4 (Sec. V-A.3).\n")
        f.write("# Written by tests/golden/make_golden.py box64 (oracle only).\n")
        f.write(f"# oracle wall time {time.time() - t0:.0f} s\n")
        f.write(f"bounds {float(lo)!r} {float(lc)!r} {float(up)!r}\n")
        f.write(f"degree {BOX64_DEGREE}\n")
        f.write(f"iterations {res.iters}\n")
        f.write(f"gate {gate}\n")
        f.write(f"gated_max_resid {float(np.max(res.resid[:gate]))!r}\n")
        for lam, r in zip(res.ritz, res.resid):
            f.write(f"{float(lam)!r} {float(r)!r}\n")
    return path


def read_box64(path: str = None):
    """(bounds, degree, iterations, gate, ritz, resid) from the box64 file."""
    path = path or box64_path()
    vals, kv = [], {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] in ("bounds", "degree", "iterations", "gate", "gated_max_resid"):
                kv[parts[0]] = [float(x) for x in parts[1:]]
            else:
                vals.append([float(x) for x in parts])
    v = np.array(vals)
    return (tuple(kv["bounds"]), int(kv["degree"][0]), int(kv["iterations"][0]), int(kv["gate"][0]),
            v[:, 0], v[:, 1])


if __name__ == "__main__":
    what = sys.argv[1:] or ["box64"]
    for w in what:
        if w == "box64":
            print(make_box64())
        else:
            raise SystemExit(f"unknown golden set {w}")
