"""The allocation-free dense eigensolver entry point (xls_dense_geneig_noalloc)
through the C ABI: device inputs and outputs, workspace in the library's
static scratch.  Two calls in a row, the second smaller, each checked against
xls_dense_geneig (the allocating entry point, same kernels: bit for bit) and
against scipy's generalized eigenvalues (1e-10); sizes beyond the scratch's
limit and a non-positive-definite M are refused."""
import ctypes as C

import numpy as np
import pytest
import scipy.linalg as sla
import torch

from paper_2609_13115_amd import xls

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[case] {msg}", flush=True)


def pencil(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    M = A @ A.T + n * np.eye(n)
    B = rng.standard_normal((n, n))
    return 0.5 * (B + B.T), M


def noalloc(H, M):
    n = H.shape[0]
    dH = torch.from_numpy(np.asfortranarray(H).ravel(order="F").copy()).cuda()
    dM = torch.from_numpy(np.asfortranarray(M).ravel(order="F").copy()).cuda()
    dlam = torch.zeros(n, dtype=torch.float64, device="cuda")
    dY = torch.zeros(n * n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    rc = xls.lib().xls_dense_geneig_noalloc(C.c_int32(n), C.c_void_p(dH.data_ptr()), C.c_void_p(dM.data_ptr()),
                                            C.c_void_p(dlam.data_ptr()), C.c_void_p(dY.data_ptr()), None)
    if rc != 0:
        raise xls.XlsError(rc, xls.lib().xls_last_error().decode())
    return dlam.cpu().numpy(), dY.cpu().numpy().reshape(n, n, order="F")


@pytest.mark.parametrize("sizes", [(480, 97), (512, 1)])
def test_noalloc_matches_allocating_entry_point(sizes):
    for k, n in enumerate(sizes):
        case(f"dense noalloc n={n} (call {k + 1})")
        H, M = pencil(n, 100 + n)
        lam, Y = noalloc(H, M)
        lam_ref, Y_ref = xls.xls_dense_geneig(H, M)
        assert np.array_equal(lam, lam_ref) and np.array_equal(Y, Y_ref)
        ref = sla.eigh(H, M, eigvals_only=True)
        assert np.max(np.abs(lam - ref)) <= 1e-10 * max(1.0, np.max(np.abs(ref)))


def test_noalloc_refuses_what_it_cannot_hold():
    case("dense noalloc errors")
    H, M = pencil(513, 1)
    with pytest.raises(xls.XlsError) as e:
        noalloc(H, M)
    assert e.value.code == xls.XLS_ERR_INVALID_ARG
    n = 12
    A = np.random.default_rng(0).standard_normal((n, n))
    M = A @ A.T
    M[:, 3] = M[:, 2]
    M[3, :] = M[2, :]
    with pytest.raises(xls.XlsError) as e:
        noalloc(np.eye(n), M)
    assert e.value.code == xls.XLS_ERR_NOT_SPD
    # the scratch is reused correctly after the refused calls
    H, M = pencil(64, 3)
    lam, _ = noalloc(H, M)
    assert np.array_equal(lam, xls.xls_dense_geneig(H, M)[0])
    # host memory is refused
    rc = xls.lib().xls_dense_geneig_noalloc(C.c_int32(4), C.c_void_p(np.zeros(16).ctypes.data),
                                            C.c_void_p(np.zeros(16).ctypes.data), C.c_void_p(np.zeros(4).ctypes.data),
                                            C.c_void_p(np.zeros(16).ctypes.data), None)
    assert rc == xls.XLS_ERR_INVALID_ARG
