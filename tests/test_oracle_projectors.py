"""Pins of the oracle's Kleinman-Bylander projector tables and V_nl."""
import os

import numpy as np
import pytest

from oracle import projectors, hamiltonian
from paper_2609_13115_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _r3():
    out = []
    with open(os.path.join(GOLDEN, "r3_sum_of_three_squares.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                out.append(int(line))
    return out


def _one_atom(rc, n=13, h=1.0, periodic=False, pos=None, gam=(1.0, 0.5, 0.5, 0.5)):
    c = (n - 1) // 2
    atom = np.array([[c * h, c * h, c * h]]) if pos is None else np.asarray(pos, dtype=float)
    proj = np.array([[rc, 0.7, *gam]])
    return projectors.build((n, n, n), h, (0.0, 0.0, 0.0), periodic, atom, proj)


@pytest.mark.parametrize("rc2", [1, 2, 4, 5, 9, 11, 12])
def test_support_count_equals_lattice_points_in_ball(rc2):
    """Node-centred atom, h = 1: |support| = sum_{k < rc^2} r_3(k) (OEIS A005875)."""
    r3 = _r3()
    t = _one_atom(np.sqrt(rc2))
    expect = sum(r3[k] for k in range(rc2)) if rc2 <= len(r3) else None
    # rc = sqrt(k) may round either way; the oracle compares r2 < fl(rc*rc)
    rcf = np.sqrt(float(rc2))
    thresh = rcf * rcf
    if thresh > rc2:
        expect += r3[rc2]
    assert t.offsets[1] == expect


def test_projectors_normalised_and_orthogonal_at_node():
    h = 0.5
    t = _one_atom(2.0, n=17, h=h)
    V = t.val
    G = h ** 3 * V.T @ V
    assert np.allclose(np.diag(G), 1.0, atol=1e-14)
    # s is even, p_x / p_y / p_z are odd along their own axis: mutually orthogonal
    assert np.allclose(G - np.diag(np.diag(G)), 0.0, atol=1e-14)


def test_dense_vnl_spectrum_single_atom():
    """With orthonormal (h^3-weighted) projectors V_nl has eigenvalues
    gamma_s, gamma_px, gamma_py, gamma_pz and zeros."""
    gam = (1.3, 0.6, 0.45, 0.7)
    t = _one_atom(2.0, n=11, h=0.6, gam=gam)
    nd = 11 ** 3
    M = projectors.dense_vnl(t, nd, 0.6)
    ev = np.sort(np.linalg.eigvalsh(M))
    assert np.allclose(ev[-4:], np.sort(gam), atol=1e-13)
    assert np.allclose(ev[:-4], 0.0, atol=1e-13)


def test_periodic_translation_permutes_values():
    """Shifting the atom by one grid spacing in a periodic box cyclically
    shifts its support and values (h = 1 keeps every coordinate exact);
    the box is smaller than 2 r_c so several images overlap."""
    n = 5
    t0 = _one_atom(3.0, n=n, periodic=True, pos=[[1.0, 2.0, 0.0]])
    t1 = _one_atom(3.0, n=n, periodic=True, pos=[[2.0, 2.0, 0.0]])
    A0 = np.zeros((n ** 3, 4))
    A1 = np.zeros((n ** 3, 4))
    A0[t0.idx] = t0.val
    A1[t1.idx] = t1.val
    A0 = A0.reshape(n, n, n, 4)  # [k, j, i]
    A1 = A1.reshape(n, n, n, 4)
    assert np.allclose(np.roll(A0, 1, axis=2), A1, atol=1e-15)
    assert t0.offsets[1] == t1.offsets[1]


def test_reverse_csr_is_inverse_of_support():
    sd = workloads.small_dirichlet(8, 4)
    t = projectors.build(sd.n, sd.h, sd.origin, False, sd.atoms, sd.proj)
    nd = sd.nd
    pairs_fwd = sorted((int(t.idx[s]), s) for s in range(len(t.idx)))
    pairs_rev = []
    for g in range(nd):
        for e in range(t.rev_offsets[g], t.rev_offsets[g + 1]):
            pairs_rev.append((g, int(t.rev_slot[e])))
    assert pairs_fwd == pairs_rev
    for a in range(len(t.offsets) - 1):
        seg = t.idx[t.offsets[a]:t.offsets[a + 1]]
        assert np.all(np.diff(seg) > 0)


def test_apply_vnl_equals_dense_and_is_symmetric_psd():
    sd = workloads.small_periodic(8, 4)
    op = hamiltonian.from_subdomain(sd)
    t = op.proj
    M = projectors.dense_vnl(t, sd.nd, sd.h)
    X = np.random.default_rng(1).standard_normal((sd.nd, 3))
    assert np.allclose(projectors.apply_vnl(t, X, sd.h), M @ X, atol=1e-12)
    assert np.allclose(M, M.T, atol=1e-14)
    assert np.linalg.eigvalsh(M).min() > -1e-12


def test_full_hamiltonian_symmetric():
    for sd in (workloads.small_periodic(8, 4), workloads.small_dirichlet(8, 4)):
        op = hamiltonian.from_subdomain(sd)
        rng = np.random.default_rng(3)
        x = rng.standard_normal(sd.nd)
        y = rng.standard_normal(sd.nd)
        assert abs(x @ op.apply(y) - y @ op.apply(x)) < 1e-10 * abs(x @ op.apply(y)) + 1e-10


def test_radial_shape_at_listed_lattice_points():
    """Before normalisation chi_s = exp(-r^2 / (2 w^2)) and chi_px = (x - X) chi_s:
    ratios of values at hand-listed lattice points of a node-centred atom
    cancel the normalisation and fix the width convention."""
    h, w, n = 0.5, 0.7, 17
    c = (n - 1) // 2
    proj_w = np.array([[2.0, w, 1.0, 0.5, 0.5, 0.5]])
    t = projectors.build((n, n, n), h, (0.0, 0.0, 0.0), False, np.array([[c * h] * 3]), proj_w)
    where = {int(g): s for s, g in enumerate(t.idx)}

    def val(i, j, k, l):
        return t.val[where[(c + i) + n * ((c + j) + n * (c + k))], l]

    centre = val(0, 0, 0, 0)
    for (i, j, k) in [(1, 0, 0), (0, 2, 0), (1, 1, 1), (2, 1, 0), (3, 0, 1), (2, 2, 1)]:
        r2 = h * h * (i * i + j * j + k * k)
        assert val(i, j, k, 0) / centre == pytest.approx(np.exp(-r2 / (2 * w * w)), rel=1e-13)
    # p_x: odd in x, and px(1,0,0)/px(2,1,0) = (h e^{-h^2/2w^2}) / (2h e^{-5h^2/2w^2})
    assert val(1, 0, 0, 1) == pytest.approx(-val(-1, 0, 0, 1), rel=1e-14)
    want = (1 * h * np.exp(-h * h / (2 * w * w))) / (2 * h * np.exp(-5 * h * h / (2 * w * w)))
    assert val(1, 0, 0, 1) / val(2, 1, 0, 1) == pytest.approx(want, rel=1e-13)
    assert val(0, 2, 1, 2) / val(1, 1, 0, 2) == pytest.approx(
        (2 * np.exp(-5 * h * h / (2 * w * w))) / (1 * np.exp(-2 * h * h / (2 * w * w))), rel=1e-13)


def test_periodic_images_are_summed_in_a_small_box():
    """A periodic box smaller than 2 r_c: every point's unnormalised value is
    the sum over the 27 images X + s L (s in {-1,0,1}^3) that lie within r_c,
    written out here point by point; the oracle's values are that sum
    normalised (h^3 sum chi^2 = 1)."""
    n, h, rc, w = 4, 0.6, 2.0, 0.5
    L = n * h
    X = np.array([0.7, 1.3, 2.9])
    t = projectors.build((n, n, n), h, (0.0, 0.0, 0.0), True, X[None, :], np.array([[rc, w, 1, 1, 1, 1]]))
    S = np.zeros((n ** 3, 4))
    multi = 0
    for k in range(n):
        for j in range(n):
            for i in range(n):
                g = i + n * (j + n * k)
                hits = 0
                for sz in (-1, 0, 1):
                    for sy in (-1, 0, 1):
                        for sx in (-1, 0, 1):
                            d = np.array([i * h, j * h, k * h]) - (X + np.array([sx, sy, sz]) * L)
                            r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
                            if r2 < rc * rc:
                                e = np.exp(-r2 / (2 * w * w))
                                S[g] += [e, d[0] * e, d[1] * e, d[2] * e]
                                hits += 1
                multi += hits > 1
    assert multi > 0                       # the pin needs overlapping images
    got = np.zeros((n ** 3, 4))
    got[t.idx] = t.val
    for l in range(4):
        ref = S[:, l] / np.sqrt(h ** 3 * np.sum(S[:, l] ** 2))
        assert np.allclose(got[:, l], ref, rtol=1e-12, atol=1e-14), l
