"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Tolerances: integer work bit-exact; FP64 results <= 1e-10 relative (to the
largest entry of the compared quantity for elementwise fields, since single
entries can sit near zero); mixed-precision results against the FP64 oracle
at the bars stated in each test."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import chefsi, density, grid, hamiltonian, projectors
from oracle import bf16 as obf16
from paper_2609_13115_amd import workloads
from paper_2609_13115_amd import xls

pytestmark = pytest.mark.gpu


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def case(name):
    print(f"[case] {name}", flush=True)


# ---------------------------------------------------------------------------
# fixtures
# ---------------------------------------------------------------------------

SYSTEMS = {
    "periodic8": lambda: workloads.small_periodic(8, 6),
    "dirichlet_ragged": lambda: workloads.small_dirichlet(ns=5, shape=(13, 9, 20)),
    "si_cell_24": lambda: workloads.si_cell_24(),
}


@pytest.fixture(scope="module", params=sorted(SYSTEMS))
def system(request):
    sd = SYSTEMS[request.param]()
    op = hamiltonian.from_subdomain(sd)
    return request.param, sd, op


# ---------------------------------------------------------------------------
# a1: setup maps and projector tables (integer work bit-exact)
# ---------------------------------------------------------------------------

def test_maps_and_projector_tables_bit_exact(system):
    name, sd, op = system
    case(f"maps {name}")
    with xls.Subdomain(sd) as s:
        m, g = s.xls_subdomain_get_maps()
        off, idx, val, roff, rslot = s.xls_subdomain_get_projectors()
    assert np.array_equal(m, grid.core_mask(sd.n, sd.core_lo, sd.core_hi))
    assert np.array_equal(g, grid.global_index(sd.n, sd.global_offset, sd.global_n))
    t = op.proj
    assert np.array_equal(off, t.offsets)
    assert np.array_equal(idx, t.idx)
    assert np.array_equal(roff, t.rev_offsets)
    assert np.array_equal(rslot, t.rev_slot)
    assert rel_err(val, t.val) <= 1e-13


def test_maps_si_box_64_bit_exact():
    case("maps 64^3 box")
    sd = workloads.si_box_64(with_x0=False, ns=4)
    sd.x0 = sd.make_x0(4)
    t = projectors.build(sd.n, sd.h, sd.origin, False, sd.atoms, sd.proj)
    with xls.Subdomain(sd) as s:
        m, g = s.xls_subdomain_get_maps()
        off, idx, val, roff, rslot = s.xls_subdomain_get_projectors()
    assert np.array_equal(m, grid.core_mask(sd.n, sd.core_lo, sd.core_hi))
    assert np.array_equal(g, grid.global_index(sd.n, sd.global_offset, sd.global_n))
    assert np.array_equal(off, t.offsets) and np.array_equal(idx, t.idx)
    assert np.array_equal(roff, t.rev_offsets) and np.array_equal(rslot, t.rev_slot)
    assert rel_err(val, t.val) <= 1e-13


# ---------------------------------------------------------------------------
# a3: H apply and filter
# ---------------------------------------------------------------------------

# (block, rows per tile, z-chunk, vectors per tile); 3 columns leave the
# second vector of the last 2-vector tile empty
TILES = [(512, 0, 0, 1), (512, 3, 7, 2), (256, 5, 0, 2), (256, 1, 1, 1)]


@pytest.mark.parametrize("tile", TILES)
def test_hamiltonian_apply_fp64(system, tile):
    name, sd, op = system
    case(f"H apply fp64 {name} tile={tile}")
    X = sd.x0[:, :3]
    ref = op.apply(X)
    with xls.Subdomain(sd) as s:
        s.xls_subdomain_tune(xls.XLS_PREC_FP64, *tile)
        out = s.xls_hamiltonian_apply(X)
    assert rel_err(out, ref) <= 1e-12


def test_hamiltonian_apply_fp32(system):
    name, sd, op = system
    case(f"H apply fp32 {name}")
    X = sd.x0[:, :2].astype(np.float32).astype(np.float64)
    ref = op.apply(X)
    with xls.Subdomain(sd, filter_prec=xls.XLS_PREC_FP32) as s:
        out = s.xls_hamiltonian_apply(X)
    assert rel_err(out, ref) <= 2e-6


def test_hamiltonian_apply_si_box_64_fp64():
    case("H apply 64^3 box fp64")
    sd = workloads.si_box_64(with_x0=False, ns=3)
    sd.x0 = sd.make_x0(3)
    op = hamiltonian.from_subdomain(sd)
    ref = op.apply(sd.x0)
    with xls.Subdomain(sd) as s:
        out = s.xls_hamiltonian_apply(sd.x0)
    assert rel_err(out, ref) <= 1e-12


@pytest.mark.parametrize("m", [1, 2, 7])
def test_filter_fp64(system, m):
    name, sd, op = system
    case(f"filter fp64 {name} m={m}")
    lo, up = chefsi.lanczos_bounds(op.apply, sd.lanczos_v0, 20)
    lc = chefsi.first_cutoff(lo, up)
    ref = chefsi.chebyshev_filter(op.apply, sd.x0, m, lo, lc, up)
    with xls.Subdomain(sd) as s:
        s.xls_subdomain_filter(m, lo, lc, up)
        out = s.xls_subdomain_get_block()
    assert rel_err(out, ref) <= 1e-11


@pytest.mark.parametrize("prec", [xls.XLS_PREC_FP64, xls.XLS_PREC_FP32])
def test_filter_two_vectors_per_tile_bit_identical(system, prec):
    """Tiles of 2 vectors share the operator tables but not the arithmetic of
    a point: the filtered block is bit-identical to 1-vector tiles (odd
    column counts leave the second vector of the last tile empty)."""
    name, sd, op = system
    case(f"filter nv=2 {name} prec={prec}")
    lo, up = chefsi.lanczos_bounds(op.apply, sd.lanczos_v0, 20)
    lc = chefsi.first_cutoff(lo, up)
    outs = []
    for nv, ty in ((1, 0), (2, 0), (2, 3)):
        with xls.Subdomain(sd, filter_prec=prec) as s:
            s.xls_subdomain_tune(prec, 256, ty, 0, nv)
            s.xls_subdomain_filter(5, lo, lc, up)
            outs.append(s.xls_subdomain_get_block())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    ref = chefsi.chebyshev_filter(op.apply, sd.x0, 5, lo, lc, up)
    assert rel_err(outs[2], ref) <= (1e-11 if prec == xls.XLS_PREC_FP64 else 1e-4)


def test_filter_si_cell_24_degree20_fp64_and_fp32():
    case("filter 24^3 cell m=20")
    sd = workloads.si_cell_24()
    op = hamiltonian.from_subdomain(sd)
    lo, up = chefsi.lanczos_bounds(op.apply, sd.lanczos_v0, 20)
    lc = chefsi.first_cutoff(lo, up)
    ref = chefsi.chebyshev_filter(op.apply, sd.x0, 20, lo, lc, up)
    with xls.Subdomain(sd) as s:
        s.xls_subdomain_filter(20, lo, lc, up)
        out = s.xls_subdomain_get_block()
    assert rel_err(out, ref) <= 1e-11
    with xls.Subdomain(sd, filter_prec=xls.XLS_PREC_FP32) as s:
        s.xls_subdomain_filter(20, lo, lc, up)
        out32 = s.xls_subdomain_get_block()
    assert rel_err(out32, ref) <= 1e-4


# ---------------------------------------------------------------------------
# a2: Lanczos bounds
# ---------------------------------------------------------------------------

def test_lanczos_bounds_fp64(system):
    name, sd, op = system
    case(f"lanczos {name}")
    lo, up = chefsi.lanczos_bounds(op.apply, sd.lanczos_v0, 20)
    with xls.Subdomain(sd) as s:
        glo, gup = s.xls_lanczos_bounds(20)
    assert abs(glo - lo) <= 1e-10 * max(1.0, abs(lo))
    assert abs(gup - up) <= 1e-10 * max(1.0, abs(up))


# ---------------------------------------------------------------------------
# a4/a5: projection; a7: rotation; a8: residual
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ns", [5, 37, 100])
def test_projection_fp64(ns):
    case(f"projection fp64 ns={ns}")
    sd = workloads.small_dirichlet(ns=ns, shape=(12, 14, 16))
    op = hamiltonian.from_subdomain(sd)
    X = sd.x0
    with xls.Subdomain(sd) as s:
        M, Hs = s.xls_subdomain_project(xls.XLS_PREC_FP64)
    Mr = X.T @ X
    Hr = X.T @ op.apply(X)
    Hr = 0.5 * (Hr + Hr.T)
    assert rel_err(M, Mr) <= 1e-12
    assert rel_err(Hs, Hr) <= 1e-12


# split-BF16 keeps 16 mantissa bits per operand and drops lo*lo: sums of
# squares are biased low by ~2^-16/3 relative, so its bar is 1e-5
@pytest.mark.parametrize("prec,tol", [(xls.XLS_PREC_FP64, 1e-12), (xls.XLS_PREC_FP32, 2e-6),
                                      (xls.XLS_PREC_BF16X3, 1e-5)])
def test_projection_fp32_block(prec, tol):
    case(f"projection fp32 block gemm={prec}")
    sd = workloads.small_dirichlet(ns=70, shape=(16, 16, 16))
    op = hamiltonian.from_subdomain(sd)
    X = sd.x0.astype(np.float32).astype(np.float64)
    with xls.Subdomain(sd, filter_prec=xls.XLS_PREC_FP32) as s:
        M, Hs = s.xls_subdomain_project(prec)
    Mr = X.T @ X
    W = op.apply(X).astype(np.float32).astype(np.float64)
    Hr = X.T @ W
    Hr = 0.5 * (Hr + Hr.T)
    assert rel_err(M, Mr) <= tol
    assert rel_err(Hs, Hr) <= max(tol, 2e-6)


@pytest.mark.parametrize("ns", [6, 65])
def test_rotation_fp64(ns):
    case(f"rotation ns={ns}")
    sd = workloads.small_dirichlet(ns=ns, shape=(10, 11, 12))
    Q = np.random.default_rng(3).standard_normal((ns, ns))
    with xls.Subdomain(sd) as s:
        s.xls_subdomain_rotate(Q, xls.XLS_PREC_FP64)
        out = s.xls_subdomain_get_block()
    assert rel_err(out, sd.x0 @ Q) <= 1e-13


@pytest.mark.parametrize("prec,tol", [(xls.XLS_PREC_FP32, 2e-6), (xls.XLS_PREC_BF16X3, 2e-5)])
def test_rotation_fp32(prec, tol):
    case(f"rotation fp32 gemm={prec}")
    sd = workloads.small_dirichlet(ns=40, shape=(10, 11, 12))
    Q = np.random.default_rng(3).standard_normal((40, 40))
    X = sd.x0.astype(np.float32).astype(np.float64)
    with xls.Subdomain(sd, filter_prec=xls.XLS_PREC_FP32) as s:
        s.xls_subdomain_rotate(Q, prec)
        out = s.xls_subdomain_get_block()
    assert rel_err(out, X @ Q) <= tol


# ns = 304 spans three 128-wide output tiles of the projection (ragged last)
# and two 256-wide column tiles of the rotation; ns = 300 exercises the
# fallback kernels where the bf16 path needs 8-aligned leading dimensions.
@pytest.mark.parametrize("ns", [300, 304])
@pytest.mark.parametrize("prec,tol", [(xls.XLS_PREC_FP64, 1e-12), (xls.XLS_PREC_FP32, 2e-6),
                                      (xls.XLS_PREC_BF16X3, 1e-5)])
def test_projection_and_rotation_large(prec, tol, ns):
    case(f"projection/rotation large ns={ns} gemm={prec}")
    sd = workloads.small_dirichlet(ns=ns, shape=(20, 19, 21))
    op = hamiltonian.from_subdomain(sd)
    X = sd.x0.astype(np.float32).astype(np.float64)
    Q = np.random.default_rng(5).standard_normal((ns, ns)) / np.sqrt(ns)
    with xls.Subdomain(sd, filter_prec=xls.XLS_PREC_FP32) as s:
        M, Hs = s.xls_subdomain_project(prec)
        s.xls_subdomain_rotate(Q, prec)
        out = s.xls_subdomain_get_block()
    Mr = X.T @ X
    W = op.apply(X).astype(np.float32).astype(np.float64)
    Hr = X.T @ W
    Hr = 0.5 * (Hr + Hr.T)
    assert rel_err(M, Mr) <= tol
    assert rel_err(Hs, Hr) <= max(tol, 2e-6)
    rtol = {xls.XLS_PREC_FP64: 2e-7, xls.XLS_PREC_FP32: 2e-6, xls.XLS_PREC_BF16X3: 2e-5}[prec]
    assert rel_err(out, X @ Q) <= rtol  # the FP32 block stores the result in FP32


# Both edges of the large projection kernel, forced through the GEMM plan
# (tile_tn 2 = 128, 3 = 96), on orders that leave a ragged last tile at
# either edge (200: 96 + 96 + 8; 304: 3 x 96 + 16), and the automatic choice
# at ns = 480 (five whole 96 tiles, where it takes 96).
@pytest.mark.parametrize("ns,tile", [(200, 2), (200, 3), (304, 3), (480, 0)])
@pytest.mark.parametrize("prec,tol", [(xls.XLS_PREC_FP64, 1e-12), (xls.XLS_PREC_FP32, 2e-6),
                                      (xls.XLS_PREC_BF16X3, 1e-5)])
def test_projection_tile_edges(prec, tol, ns, tile):
    case(f"projection tile edge ns={ns} tile_tn={tile} gemm={prec}")
    sd = workloads.small_dirichlet(ns=ns, shape=(20, 19, 21))
    op = hamiltonian.from_subdomain(sd)
    X = sd.x0.astype(np.float32).astype(np.float64)
    with xls.Subdomain(sd, filter_prec=xls.XLS_PREC_FP32) as s:
        s.xls_subdomain_tune_gemm(0, tile, 0)
        M, Hs = s.xls_subdomain_project(prec)
    Mr = X.T @ X
    W = op.apply(X).astype(np.float32).astype(np.float64)
    Hr = X.T @ W
    Hr = 0.5 * (Hr + Hr.T)
    assert rel_err(M, Mr) <= tol
    assert rel_err(Hs, Hr) <= max(tol, 2e-6)


@pytest.mark.parametrize("ns,tile", [(200, 3), (480, 0)])
def test_projection_tile_edges_fp64_block(ns, tile):
    case(f"projection tile edge fp64 block ns={ns} tile_tn={tile}")
    sd = workloads.small_dirichlet(ns=ns, shape=(18, 20, 19))
    op = hamiltonian.from_subdomain(sd)
    X = sd.x0
    with xls.Subdomain(sd) as s:
        s.xls_subdomain_tune_gemm(0, tile, 0)
        M, Hs = s.xls_subdomain_project(xls.XLS_PREC_FP64)
    Hr = X.T @ op.apply(X)
    assert rel_err(M, X.T @ X) <= 1e-12
    assert rel_err(Hs, 0.5 * (Hr + Hr.T)) <= 1e-12


# Both column widths of the large rotation kernel (tile_nn 2 = 256, 0 and 3 =
# 128): ns = 200 is ragged at either width, 300 pads to 384 at 128, 480 is
# four 128-column tiles with the last ragged.
@pytest.mark.parametrize("ns,tile", [(200, 2), (200, 3), (300, 0), (480, 3)])
@pytest.mark.parametrize("prec,tol", [(xls.XLS_PREC_FP64, 2e-7), (xls.XLS_PREC_FP32, 2e-6),
                                      (xls.XLS_PREC_BF16X3, 2e-5)])
def test_rotation_tile_widths(prec, tol, ns, tile):
    case(f"rotation tile width ns={ns} tile_nn={tile} gemm={prec}")
    sd = workloads.small_dirichlet(ns=ns, shape=(20, 19, 21))
    X = sd.x0.astype(np.float32).astype(np.float64)
    Q = np.random.default_rng(7).standard_normal((ns, ns)) / np.sqrt(ns)
    with xls.Subdomain(sd, filter_prec=xls.XLS_PREC_FP32) as s:
        s.xls_subdomain_tune_gemm(0, 0, tile)
        s.xls_subdomain_rotate(Q, prec)
        out = s.xls_subdomain_get_block()
    assert rel_err(out, X @ Q) <= tol  # the FP32 block stores the result in FP32


@pytest.mark.parametrize("ns,tile", [(200, 3), (300, 0)])
def test_rotation_tile_widths_fp64_block(ns, tile):
    case(f"rotation tile width fp64 block ns={ns} tile_nn={tile}")
    sd = workloads.small_dirichlet(ns=ns, shape=(18, 20, 19))
    Q = np.random.default_rng(8).standard_normal((ns, ns)) / np.sqrt(ns)
    with xls.Subdomain(sd) as s:
        s.xls_subdomain_tune_gemm(0, 0, tile)
        s.xls_subdomain_rotate(Q, xls.XLS_PREC_FP64)
        out = s.xls_subdomain_get_block()
    assert rel_err(out, sd.x0 @ Q) <= 1e-13


def test_gemm_plan_rejects_unknown_tile():
    case("gemm plan range")
    sd = workloads.small_dirichlet(ns=8, shape=(8, 8, 8))
    with xls.Subdomain(sd) as s:
        with pytest.raises(xls.XlsError):
            s.xls_subdomain_tune_gemm(0, 4, 0)
        with pytest.raises(xls.XlsError):
            s.xls_subdomain_tune_gemm(0, 0, 4)
        with pytest.raises(xls.XlsError):
            s.xls_subdomain_tune_gemm(65, 0, 0)


@pytest.mark.parametrize("ns", [128, 304])
def test_projection_rotation_large_fp64_block(ns):
    case(f"projection/rotation large fp64 block ns={ns}")
    sd = workloads.small_dirichlet(ns=ns, shape=(18, 20, 19))
    op = hamiltonian.from_subdomain(sd)
    X = sd.x0
    Q = np.random.default_rng(6).standard_normal((ns, ns)) / np.sqrt(ns)
    with xls.Subdomain(sd) as s:
        M, Hs = s.xls_subdomain_project(xls.XLS_PREC_FP64)
        s.xls_subdomain_rotate(Q, xls.XLS_PREC_FP64)
        out = s.xls_subdomain_get_block()
    Hr = X.T @ op.apply(X)
    assert rel_err(M, X.T @ X) <= 1e-12
    assert rel_err(Hs, 0.5 * (Hr + Hr.T)) <= 1e-12
    assert rel_err(out, X @ Q) <= 1e-13


def test_residual_fp64(system):
    name, sd, op = system
    case(f"residual {name}")
    lam = np.linspace(-1.0, 2.0, sd.ns)
    ref = chefsi.residuals(op.apply, sd.x0, lam)
    with xls.Subdomain(sd) as s:
        r = s.xls_subdomain_residual(lam)
    assert np.max(np.abs(r - ref) / ref) <= 1e-11


# ---------------------------------------------------------------------------
# a6: dense FP64 generalized eigensolver
# ---------------------------------------------------------------------------

# 128, 129: the one-workgroup tail alone, then one step before it; 480: the
# register-only steps and the tail; 700: all three step kernels; 31/32 and
# 900/901: either side of the compact-WY back-transform's range; 1900: the
# inverse iteration without the overlapped factorisation (n > 1800)
@pytest.mark.parametrize("n", [1, 2, 7, 20, 31, 32, 37, 100, 128, 129, 161, 480, 700, 900, 901, 1500, 1900,
                               2400, 2800])
def test_dense_geneig(n):
    case(f"dense n={n}")
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    M = A @ A.T + n * np.eye(n)
    B = rng.standard_normal((n, n))
    H = 0.5 * (B + B.T)
    lam, Y = xls.xls_dense_geneig(H, M)
    ref = sla.eigh(H, M, eigvals_only=True)
    assert np.max(np.abs(lam - ref)) <= 1e-10 * max(1.0, np.max(np.abs(ref)))
    assert np.allclose(Y.T @ M @ Y, np.eye(n), atol=1e-11)
    assert np.allclose(H @ Y, M @ Y * lam[None, :], atol=1e-9 * max(1, np.abs(ref).max()))
    lo, Yo = chefsi.generalized_eigh(H, M)
    assert np.max(np.abs(lam - lo)) <= 1e-10 * max(1.0, np.max(np.abs(lo)))


def test_dense_geneig_degenerate_spectrum():
    """Exactly repeated eigenvalues (the free periodic Laplacian has them)."""
    case("dense degenerate")
    n = 24
    Q, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((n, n)))
    d = np.repeat([1.0, 2.0, 3.0, 5.0], 6)
    H = Q @ np.diag(d) @ Q.T
    H = 0.5 * (H + H.T)
    M = np.eye(n)
    lam, Y = xls.xls_dense_geneig(H, M)
    assert np.max(np.abs(lam - d)) <= 1e-12
    assert np.allclose(Y.T @ Y, np.eye(n), atol=1e-12)


def test_dense_not_spd():
    case("dense not spd")
    n = 10
    A = np.random.default_rng(0).standard_normal((n, n))
    M = A @ A.T
    M[:, 3] = M[:, 2]
    M[3, :] = M[2, :]
    with pytest.raises(xls.XlsError) as ei:
        xls.xls_dense_geneig(np.eye(n), M)
    assert ei.value.code == xls.XLS_ERR_NOT_SPD


# ---------------------------------------------------------------------------
# full CheFSI step (FP64) and brute force
# ---------------------------------------------------------------------------

def test_chefsi_si_cell_24_fp64_parity():
    """Periodic 24^3 Si cell: 10 iterations, degree 20, Lanczos bounds; Ritz values <= 1e-10 relative."""
    case("chefsi 24^3 cell fp64")
    sd = workloads.si_cell_24()
    op = hamiltonian.from_subdomain(sd)
    lo, up = chefsi.lanczos_bounds(op.apply, sd.lanczos_v0, 20)
    ref = chefsi.chefsi(op.apply, sd.x0, 20, 10, lo, chefsi.first_cutoff(lo, up), up)
    with xls.Subdomain(sd) as s:
        ritz, resid, it = s.xls_chefsi_step(20, 10, xls.XLS_BOUNDS_LANCZOS)
        psi = s.xls_subdomain_get_block()
    assert it == 10
    assert np.max(np.abs(ritz - ref.ritz) / np.maximum(np.abs(ref.ritz), 1e-2)) <= 1e-10
    assert np.max(np.abs(resid - ref.resid)) <= 1e-9 * np.max(np.abs(ref.ritz)) + 1e-6 * np.max(ref.resid)
    assert np.allclose(psi.T @ psi, np.eye(sd.ns), atol=1e-12)
    g = chefsi.n_gate(sd.ns)
    # the well-converged states span the same subspace
    conv = int(np.sum(ref.resid[:g] < 1e-6))
    if conv:
        assert chefsi.subspace_sin_theta(psi[:, :conv], ref.psi[:, :conv]) <= 1e-8


@pytest.mark.parametrize("kind", ["periodic", "dirichlet"])
def test_chefsi_brute_force_8cubed(kind):
    case(f"chefsi brute force {kind}")
    sd = workloads.small_periodic(8, 12) if kind == "periodic" else workloads.small_dirichlet(8, 12)
    op = hamiltonian.from_subdomain(sd)
    ev = np.linalg.eigvalsh(op.dense())
    with xls.Subdomain(sd) as s:
        ritz, resid, it = s.xls_chefsi_step(16, 60, xls.XLS_BOUNDS_LANCZOS, resid_tol=1e-11)
    g = chefsi.n_gate(sd.ns)
    assert np.max(resid[:g]) <= 1e-9
    assert np.max(np.abs(ritz[:g] - ev[:g]) / np.maximum(np.abs(ev[:g]), 1e-3)) <= 1e-10


def test_chefsi_given_bounds_matches_oracle_dirichlet_ragged():
    case("chefsi given bounds ragged")
    sd = workloads.small_dirichlet(ns=5, shape=(13, 9, 20))
    op = hamiltonian.from_subdomain(sd)
    lo, up = chefsi.lanczos_bounds(op.apply, sd.lanczos_v0, 20)
    lc = chefsi.first_cutoff(lo, up)
    ref = chefsi.chefsi(op.apply, sd.x0, 9, 4, lo, lc, up)
    with xls.Subdomain(sd) as s:
        s.xls_subdomain_tune(xls.XLS_PREC_FP64, 512, 4, 6)
        ritz, resid, it = s.xls_chefsi_step(9, 4, xls.XLS_BOUNDS_GIVEN, lo, lc, up)
    assert np.max(np.abs(ritz - ref.ritz) / np.maximum(np.abs(ref.ritz), 1e-2)) <= 1e-10


# ---------------------------------------------------------------------------
# a9: density and interior weights
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", [xls.XLS_PREC_FP64, xls.XLS_PREC_FP32])
def test_density_parity(prec):
    case(f"density prec={prec}")
    sd = workloads.small_dirichlet(ns=8, shape=(12, 10, 14))
    op = hamiltonian.from_subdomain(sd)
    mask = grid.core_mask(sd.n, sd.core_lo, sd.core_hi)
    with xls.Subdomain(sd, filter_prec=prec) as s:
        with pytest.raises(xls.XlsError) as ei:
            s.xls_subdomain_density(0.0, 0.01)
        assert ei.value.code == xls.XLS_ERR_STATE
        ritz, resid, it = s.xls_chefsi_step(10, 3, xls.XLS_BOUNDS_LANCZOS,
                                            gemm_prec=prec)
        psi = s.xls_subdomain_get_block()
        mu = 0.5 * (ritz[3] + ritz[4])
        rho, c = s.xls_subdomain_density(mu, 0.0037)
    rr, cr = density.core_density(psi, ritz, mu, 0.0037, mask, sd.h)
    tol = 1e-12 if prec == xls.XLS_PREC_FP64 else 1e-12
    assert rel_err(rho, rr) <= tol
    assert np.max(np.abs(c - cr)) <= tol
    assert abs(sd.h ** 3 * rho.sum() - 2 * np.sum(density.fermi(ritz, mu, 0.0037) * c)) <= 1e-10


# ---------------------------------------------------------------------------
# bf16 split, determinism, failure paths
# ---------------------------------------------------------------------------

def test_split_bf16_bit_exact():
    case("bf16 split")
    rng = np.random.default_rng(11)
    a = np.concatenate([rng.standard_normal(100000).astype(np.float32),
                        (rng.standard_normal(1000) * 1e-30).astype(np.float32),
                        np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 0.0, -0.0], dtype=np.float32)])
    hi, lo = xls.xls_split_bf16(a)
    rh, rl = obf16.split(a)
    assert np.array_equal(hi, rh)
    assert np.array_equal(lo, rl)


def test_bitwise_determinism():
    case("determinism")
    sd = workloads.si_cell_24()
    outs = []
    for _ in range(2):
        with xls.Subdomain(sd) as s:
            ritz, resid, it = s.xls_chefsi_step(20, 3, xls.XLS_BOUNDS_LANCZOS)
            outs.append((ritz, resid, s.xls_subdomain_get_block()))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_wide_box_takes_512_thread_tiles():
    """A 96-point row: its y-halo exceeds what 256 threads stage, so the
    default launch shape takes 512-thread tiles; H apply and a filter pass
    still match the oracle."""
    case("wide box 96 x 10 x 12")
    sd = workloads.small_dirichlet(ns=3, shape=(96, 10, 12), h=0.2, index=4)
    op = hamiltonian.from_subdomain(sd)
    with xls.Subdomain(sd) as s:
        assert rel_err(s.xls_hamiltonian_apply(sd.x0), op.apply(sd.x0)) <= 1e-12
        lo, up = chefsi.lanczos_bounds(op.apply, sd.lanczos_v0, 20)
        lc = chefsi.first_cutoff(lo, up)
        s.xls_subdomain_filter(3, lo, lc, up)
        assert rel_err(s.xls_subdomain_get_block(), chefsi.chebyshev_filter(op.apply, sd.x0, 3, lo, lc, up)) <= 1e-11
        with pytest.raises(xls.XlsError) as ei:
            s.xls_subdomain_tune(xls.XLS_PREC_FP64, 256, 0, 0)  # 256 threads cannot stage this halo
        assert ei.value.code == xls.XLS_ERR_INVALID_ARG


def test_time_gemms_leaves_block_and_checks_precision():
    case("time gemms")
    sd = workloads.small_dirichlet(ns=70, shape=(13, 9, 20), index=2)
    with xls.Subdomain(sd, filter_prec=xls.XLS_PREC_FP32) as s:
        before = s.xls_subdomain_get_block()
        for p in (xls.XLS_PREC_FP32, xls.XLS_PREC_BF16X3):
            ms = s.xls_subdomain_time_gemms(p, 2)
            assert ms.shape == (3,) and np.all(ms > 0)
        assert np.array_equal(before, s.xls_subdomain_get_block())
    with xls.Subdomain(sd) as s:
        assert np.all(s.xls_subdomain_time_gemms(xls.XLS_PREC_FP64, 1) > 0)
        with pytest.raises(xls.XlsError) as ei:
            s.xls_subdomain_time_gemms(xls.XLS_PREC_BF16X3, 1)
        assert ei.value.code == xls.XLS_ERR_INVALID_ARG


def test_failure_paths():
    case("failure paths")
    sd = workloads.small_dirichlet(ns=4)
    bad = workloads.small_dirichlet(ns=4)
    bad.v = bad.v.copy()
    bad.v[5] = np.nan
    with pytest.raises(xls.XlsError) as ei:
        xls.Subdomain(bad)
    assert ei.value.code == xls.XLS_ERR_INVALID_ARG
    X = sd.x0.copy()
    X[:, 2] = X[:, 1]
    with xls.Subdomain(sd, x0=X) as s:
        with pytest.raises(xls.XlsError) as ei:
            s.xls_chefsi_step(6, 1, xls.XLS_BOUNDS_LANCZOS)
        assert ei.value.code == xls.XLS_ERR_NOT_SPD
    with xls.Subdomain(sd) as s:
        with pytest.raises(xls.XlsError) as ei:
            s.xls_chefsi_step(6, 1, xls.XLS_BOUNDS_GIVEN, 1.0, 0.5, 2.0)
        assert ei.value.code == xls.XLS_ERR_INVALID_ARG
        with pytest.raises(xls.XlsError) as ei:
            s.xls_subdomain_tune(xls.XLS_PREC_FP64, 128, 0, 0)
        assert ei.value.code == xls.XLS_ERR_INVALID_ARG
        with pytest.raises(xls.XlsError) as ei:
            s.xls_subdomain_tune(xls.XLS_PREC_FP32, 256, 0, 0, 3)
        assert ei.value.code == xls.XLS_ERR_INVALID_ARG


def test_dense_graph_replay_matches_eager():
    """The dense stage is replayed from a hipGraph from the third iteration on;
    every replay (with eager filter work and host syncs in between) must give
    the same bits as eager launches."""
    case("dense graph replay vs eager")
    sd = workloads.small_dirichlet(ns=12, index=4, shape=(14, 12, 16), h=0.6)
    outs = []
    for on in (True, False):
        xls.xls_set_graphs(on)
        try:
            with xls.Subdomain(sd) as s:
                ritz, resid, it = s.xls_chefsi_step(11, 7, xls.XLS_BOUNDS_LANCZOS)
                outs.append((ritz, resid, it, s.xls_subdomain_get_block()))
        finally:
            xls.xls_set_graphs(True)
    (r1, e1, i1, b1), (r2, e2, i2, b2) = outs
    assert i1 == i2 == 7
    assert np.array_equal(r1, r2) and np.array_equal(e1, e2) and np.array_equal(b1, b2)


def gap_edge(ritz, gate, gap=1e-3):
    """Largest k <= gate with ritz[k] - ritz[k-1] >= gap (0 if none)."""
    for k in range(gate, 0, -1):
        if k < len(ritz) and ritz[k] - ritz[k - 1] >= gap:
            return k
    return 0


@pytest.mark.parametrize("gprec", [xls.XLS_PREC_FP32, xls.XLS_PREC_BF16X3])
def test_mixed_precision_ritz_gate_si_cell_24(gprec):
    """The mixed forms (FP32 filter sweeps; FP32 or split-BF16 GEMMs; FP64
    Cholesky, eigensolve and residual) against the FP64 oracle on the periodic 24^3 cell:
    every gated Ritz value within 1e-6 Ha, and the gated subspace within
    1e-5 (largest principal-angle sine, clusters closed)."""
    case(f"mixed gate 24^3 cell gemm={gprec}")
    sd = workloads.si_cell_24()
    op = hamiltonian.from_subdomain(sd)
    lo, up = chefsi.lanczos_bounds(op.apply, sd.lanczos_v0, 20)
    ref = chefsi.chefsi(op.apply, sd.x0, 20, 14, lo, chefsi.first_cutoff(lo, up), up)
    with xls.Subdomain(sd, filter_prec=xls.XLS_PREC_FP32) as s:
        ritz, resid, it = s.xls_chefsi_step(20, 14, xls.XLS_BOUNDS_LANCZOS, gemm_prec=gprec)
        psi = s.xls_subdomain_get_block()
    gate = int(np.floor(sd.ns / 1.1 + 1e-9))
    assert np.max(np.abs(ritz[:gate] - ref.ritz[:gate])) <= 1e-6
    # subspace of the gated states up to the last spectral gap at or below
    # the gate edge (a degenerate cluster is never cut)
    k = gap_edge(ref.ritz, gate)
    assert k >= gate // 2
    assert chefsi.subspace_sin_theta(ref.psi[:, :k], psi[:, :k]) <= 1e-5


def test_mixed_precision_ritz_gate_dirichlet():
    case("mixed gate dirichlet box")
    sd = workloads.small_dirichlet(ns=24, index=9, shape=(18, 16, 20), h=0.6)
    op = hamiltonian.from_subdomain(sd)
    lo, up = chefsi.lanczos_bounds(op.apply, sd.lanczos_v0, 20)
    ref = chefsi.chefsi(op.apply, sd.x0, 16, 16, lo, chefsi.first_cutoff(lo, up), up)
    with xls.Subdomain(sd, filter_prec=xls.XLS_PREC_FP32) as s:
        ritz, resid, it = s.xls_chefsi_step(16, 16, xls.XLS_BOUNDS_LANCZOS, gemm_prec=xls.XLS_PREC_BF16X3)
        psi = s.xls_subdomain_get_block()
    gate = int(np.floor(sd.ns / 1.1 + 1e-9))
    assert np.max(np.abs(ritz[:gate] - ref.ritz[:gate])) <= 1e-6
    k = gap_edge(ref.ritz, gate)
    assert k >= gate // 2
    assert chefsi.subspace_sin_theta(ref.psi[:, :k], psi[:, :k]) <= 1e-5


@pytest.mark.parametrize("fprec,gprec", [(xls.XLS_PREC_FP32, xls.XLS_PREC_BF16X3),
                                         (xls.XLS_PREC_FP32, xls.XLS_PREC_FP32),
                                         (xls.XLS_PREC_FP64, xls.XLS_PREC_FP64)])
def test_reported_ritz_values_are_rayleigh_quotients(fprec, gprec):
    """The returned Ritz values against the Rayleigh quotients
    psi^T H psi / psi^T psi of the returned columns, with H applied by the
    oracle in FP64.  For a Rayleigh-Ritz vector psi = Psi_f y the quotient
    equals the projected eigenvalue exactly (y^T H_s y / y^T M_s y), so the
    FP64 form (projected eigenvalues, ascending) must agree to rounding; the
    mixed forms report the quotients themselves (FP64 sweep of the FP32
    block), which must agree to the FP64 summation order."""
    case(f"reported Ritz values filter={fprec} gemm={gprec}")
    sd = workloads.small_dirichlet(ns=24, index=9, shape=(18, 16, 20), h=0.6)
    op = hamiltonian.from_subdomain(sd)
    with xls.Subdomain(sd, filter_prec=fprec) as s:
        ritz, resid, it = s.xls_chefsi_step(16, 6, xls.XLS_BOUNDS_LANCZOS, gemm_prec=gprec)
        psi = s.xls_subdomain_get_block()
    hp = op.apply(psi)
    rq = np.sum(psi * hp, axis=0) / np.sum(psi * psi, axis=0)
    err = float(np.max(np.abs(ritz - rq) / np.maximum(np.abs(rq), 1.0)))
    print(f"[ritz] filter={fprec} gemm={gprec}: max rel |ritz - rq| {err:.2e}", flush=True)
    if fprec == xls.XLS_PREC_FP64:
        assert np.all(np.diff(ritz) >= 0)
        assert err <= 1e-10
    else:
        assert err <= 1e-12
