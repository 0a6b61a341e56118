"""Thin Python binding of the C ABI in include/xls.h (argument marshalling only).

Every numerical step runs in libxls.so's HIP kernels.  Loading fails loudly
when the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxls.so")

XLS_OK = 0
XLS_ERR_INVALID_ARG = -1
XLS_ERR_OUT_OF_MEMORY = -2
XLS_ERR_DEVICE = -3
XLS_ERR_NOT_SPD = -4
XLS_ERR_EIG_NOCONV = -5
XLS_ERR_STATE = -6

XLS_BC_PERIODIC = 0
XLS_BC_DIRICHLET0 = 1
XLS_PREC_FP64 = 0
XLS_PREC_FP32 = 1
XLS_PREC_BF16X3 = 2
XLS_BOUNDS_GIVEN = 0
XLS_BOUNDS_LANCZOS = 1
XLS_BOUNDS_LEARNED = 2

EXPORTED = [
    "xls_subdomain_create", "xls_chefsi_step", "xls_subdomain_density", "xls_subdomain_destroy",
    "xls_last_error", "xls_hamiltonian_apply", "xls_subdomain_filter", "xls_subdomain_project",
    "xls_subdomain_rotate", "xls_subdomain_residual", "xls_lanczos_bounds", "xls_dense_geneig",
    "xls_subdomain_get_block", "xls_subdomain_set_block", "xls_subdomain_get_maps",
    "xls_subdomain_get_projectors", "xls_split_bf16", "xls_set_profiling", "xls_get_stage_times",
    "xls_subdomain_tune", "xls_subdomain_store_half", "xls_subdomain_load_half",
    "xls_batch_create", "xls_batch_chefsi", "xls_batch_density", "xls_batch_fermi", "xls_batch_assemble",
    "xls_batch_subdomain", "xls_batch_tune",
    "xls_batch_stats", "xls_batch_destroy",
    "xls_subdomain_counters", "xls_subdomain_features", "xls_mlp_create", "xls_mlp_destroy",
    "xls_mlp_get_params", "xls_mlp_set_params", "xls_mlp_set_norm", "xls_mlp_forward", "xls_mlp_gradient",
    "xls_mlp_train", "xls_mlp_predict", "xls_set_graphs", "xls_subdomain_time_gemms",
    "xls_mlp_fit", "xls_mlp_train_rms", "xls_mlp_bounds", "xls_learned_safe_bounds",
    "xls_batch_create_slots", "xls_subdomain_tune_gemm", "xls_subdomain_use_half",
    "xls_dense_geneig_noalloc", "xls_subdomain_pdos",
    "xls_poisson_create", "xls_poisson_solve", "xls_poisson_solve_device", "xls_poisson_vcycle",
    "xls_poisson_destroy",
]


class XlsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"xls error {code}: {msg}")
        self.code = code


class xls_projset_t(C.Structure):
    _fields_ = [("rc", C.c_double), ("gauss_width", C.c_double), ("gamma", C.c_double * 4)]


class xls_subdomain_desc_t(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3), ("h", C.c_double), ("bc", C.c_int32), ("fd_n0", C.c_int32),
        ("origin", C.c_double * 3), ("v_eff", C.POINTER(C.c_double)),
        ("n_atoms", C.c_int32), ("atom_xyz", C.POINTER(C.c_double)),
        ("proj", C.POINTER(xls_projset_t)),
        ("core_lo", C.c_int32 * 3), ("core_hi", C.c_int32 * 3),
        ("global_offset", C.c_int64 * 3), ("global_n", C.c_int64 * 3),
        ("ns", C.c_int32), ("x0", C.POINTER(C.c_double)), ("lanczos_v0", C.POINTER(C.c_double)),
        ("filter_prec", C.c_int32), ("stream", C.c_void_p), ("x0_seed", C.c_uint64),
    ]


class xls_chefsi_params_t(C.Structure):
    _fields_ = [
        ("bounds_mode", C.c_int32), ("lam_lo", C.c_double), ("lam_cut", C.c_double),
        ("lam_max", C.c_double), ("degree", C.c_int32), ("max_iter", C.c_int32),
        ("resid_tol", C.c_double), ("n_gate", C.c_int32), ("lanczos_k", C.c_int32),
        ("gemm_prec", C.c_int32), ("fallback_tol", C.c_double), ("fallback_degree", C.c_int32),
    ]


_lib = None


def lib() -> C.CDLL:
    """The loaded libxls.so (raises if it was never built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2609_13115_amd.build")
        L = C.CDLL(LIB_PATH)
        L.xls_last_error.restype = C.c_char_p
        L.xls_subdomain_destroy.restype = None
        L.xls_batch_destroy.restype = None
        L.xls_mlp_destroy.restype = None
        L.xls_poisson_destroy.restype = None
        _lib = L
    return _lib


def _check(rc: int):
    if rc < 0:
        raise XlsError(rc, lib().xls_last_error().decode(errors="replace"))
    return rc


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None, order="F") -> np.ndarray:
    out = np.ascontiguousarray(a, dtype=np.float64) if order == "C" else np.asfortranarray(a, dtype=np.float64)
    if shape is not None and out.size != int(np.prod(shape)):
        raise ValueError(f"expected {shape} elements, got {out.shape}")
    return out


def xls_set_profiling(on: bool) -> None:
    _check(lib().xls_set_profiling(C.c_int32(1 if on else 0)))


def xls_set_graphs(on: bool) -> None:
    _check(lib().xls_set_graphs(C.c_int32(1 if on else 0)))


def xls_dense_geneig(Hs: np.ndarray, M: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    n = Hs.shape[0]
    H = _f64(Hs)
    Mm = _f64(M)
    lam = np.zeros(n)
    Y = np.zeros((n, n), order="F")
    _check(lib().xls_dense_geneig(C.c_int32(n), _dp(H), _dp(Mm), _dp(lam), _dp(Y)))
    return lam, Y


def xls_split_bf16(a: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    a = np.ascontiguousarray(a, dtype=np.float32)
    hi = np.zeros(a.size, dtype=np.uint16)
    lo = np.zeros(a.size, dtype=np.uint16)
    _check(lib().xls_split_bf16(a.ctypes.data_as(C.POINTER(C.c_float)),
                                hi.ctypes.data_as(C.POINTER(C.c_uint16)),
                                lo.ctypes.data_as(C.POINTER(C.c_uint16)), C.c_int64(a.size)))
    return hi, lo


def make_desc(sd, filter_prec: int = XLS_PREC_FP64, x0: Optional[np.ndarray] = None,
              stream: Optional[int] = None, lanczos_v0: Optional[np.ndarray] = None,
              x0_seed: Optional[int] = None):
    """xls_subdomain_desc_t for a workload subdomain, plus the arrays it points
    into (keep them alive until the create call returns).  With x0_seed the
    start block is drawn on the device (x0 NULL) and the Lanczos vector is its
    column 0 unless given."""
    x0 = sd.x0 if (x0 is None and x0_seed is None) else x0
    if x0 is None and x0_seed is None:
        raise ValueError("start block x0 (or x0_seed) is required")
    d = xls_subdomain_desc_t()
    d.n = (C.c_int32 * 3)(*[int(v) for v in sd.n])
    d.h = float(sd.h)
    d.bc = int(sd.bc)
    d.fd_n0 = int(getattr(sd, "fd_n0", 6))
    d.origin = (C.c_double * 3)(*[float(v) for v in sd.origin])
    v = _f64(sd.v, order="C")
    d.v_eff = _dp(v)
    atoms = np.ascontiguousarray(sd.atoms, dtype=np.float64).reshape(-1, 3)
    d.n_atoms = atoms.shape[0]
    d.atom_xyz = _dp(atoms)
    ps = (xls_projset_t * max(1, atoms.shape[0]))()
    for i in range(atoms.shape[0]):
        ps[i].rc = float(sd.proj[i, 0])
        ps[i].gauss_width = float(sd.proj[i, 1])
        for l in range(4):
            ps[i].gamma[l] = float(sd.proj[i, 2 + l])
    d.proj = C.cast(ps, C.POINTER(xls_projset_t))
    d.core_lo = (C.c_int32 * 3)(*sd.core_lo)
    d.core_hi = (C.c_int32 * 3)(*sd.core_hi)
    d.global_offset = (C.c_int64 * 3)(*sd.global_offset)
    d.global_n = (C.c_int64 * 3)(*sd.global_n)
    if x0 is not None:
        d.ns = int(x0.shape[1])
        X = _f64(x0)
        d.x0 = _dp(X)
        lv = lanczos_v0 if lanczos_v0 is not None else getattr(sd, "lanczos_v0", None)
    else:
        d.ns = int(sd.ns)
        X = None
        d.x0_seed = int(x0_seed)
        lv = lanczos_v0
    if lv is not None:
        lv = _f64(lv, order="C")
        d.lanczos_v0 = _dp(lv)
    d.filter_prec = int(filter_prec)
    d.stream = C.c_void_p(stream) if stream else None
    return d, [v, atoms, ps, X, lv]


def tune_keys(sd, prec: int):
    """(filter shape class, GEMM class) keys of xls_batch_tune's cache for a subdomain."""
    n = [int(v) for v in sd.n]
    pr = "f32" if prec == XLS_PREC_FP32 else "f64"
    up = lambda v, q: (v + q - 1) // q * q  # noqa: E731
    shape = (f"{pr}_nx{n[0]}_ny{up(n[1], 8)}_nz{up(n[2], 8)}_{'p' if int(sd.bc) == XLS_BC_PERIODIC else 'd'}"
             f"_na{up(len(sd.atoms), 64)}")
    nd = n[0] * n[1] * n[2]
    return shape, f"gemm_{pr}_nd{up(nd, 32768)}_ns{up(int(sd.ns), 32)}"


def chefsi_params(degree: int, max_iter: int, bounds_mode: int = XLS_BOUNDS_LANCZOS, lam_lo: float = 0.0,
                  lam_cut: float = 0.0, lam_max: float = 0.0, resid_tol: float = 0.0, n_gate: int = 0,
                  lanczos_k: int = 20, gemm_prec: int = XLS_PREC_FP64, fallback_tol: float = 0.0,
                  fallback_degree: int = 0) -> "xls_chefsi_params_t":
    return xls_chefsi_params_t(bounds_mode, lam_lo, lam_cut, lam_max, degree, max_iter, resid_tol, n_gate,
                               lanczos_k, gemm_prec, fallback_tol, fallback_degree)


class Subdomain:
    """Owner of one xls_subdomain_t handle (xls_subdomain_create / _destroy)."""

    def __init__(self, sd, filter_prec: int = XLS_PREC_FP64, x0: Optional[np.ndarray] = None,
                 stream: Optional[int] = None, lanczos_v0: Optional[np.ndarray] = None,
                 x0_seed: Optional[int] = None):
        d, keep = make_desc(sd, filter_prec, x0, stream, lanczos_v0, x0_seed)
        h = C.c_void_p()
        _check(lib().xls_subdomain_create(C.byref(d), C.byref(h)))
        del keep
        self._h = h
        self._borrowed = False
        self._set_shape(sd.n, d.ns, filter_prec)

    def _set_shape(self, n, ns, prec):
        self.n = tuple(int(v) for v in n)
        self.nd = int(np.prod(self.n))
        self.ns = int(ns)
        self.prec = int(prec)

    @classmethod
    def _borrow(cls, handle: C.c_void_p, n, ns, prec) -> "Subdomain":
        self = cls.__new__(cls)
        self._h = handle
        self._borrowed = True
        self._set_shape(n, ns, prec)
        return self

    # lifetime
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value and not getattr(self, "_borrowed", False):
            lib().xls_subdomain_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # calls
    def xls_chefsi_step(self, degree: int, max_iter: int, bounds_mode: int = XLS_BOUNDS_LANCZOS,
                        lam_lo: float = 0.0, lam_cut: float = 0.0, lam_max: float = 0.0,
                        resid_tol: float = 0.0, n_gate: int = 0, lanczos_k: int = 20,
                        gemm_prec: int = XLS_PREC_FP64, fallback_tol: float = 0.0, fallback_degree: int = 0):
        p = chefsi_params(degree, max_iter, bounds_mode, lam_lo, lam_cut, lam_max, resid_tol, n_gate,
                          lanczos_k, gemm_prec, fallback_tol, fallback_degree)
        ritz = np.zeros(self.ns)
        resid = np.zeros(self.ns)
        it = C.c_int32(0)
        _check(lib().xls_chefsi_step(self._h, C.byref(p), _dp(ritz), _dp(resid), C.byref(it)))
        return ritz, resid, int(it.value)

    def xls_subdomain_density(self, mu: float, sigma: float):
        rho = np.zeros(self.nd)
        c = np.zeros(self.ns)
        _check(lib().xls_subdomain_density(self._h, C.c_double(mu), C.c_double(sigma), _dp(rho), _dp(c)))
        return rho, c

    def xls_hamiltonian_apply(self, X: np.ndarray) -> np.ndarray:
        X = _f64(X.reshape(self.nd, -1))
        out = np.zeros_like(X, order="F")
        _check(lib().xls_hamiltonian_apply(self._h, _dp(X), _dp(out), C.c_int32(X.shape[1])))
        return out

    def xls_subdomain_filter(self, degree: int, a0: float, lam_cut: float, lam_max: float):
        _check(lib().xls_subdomain_filter(self._h, C.c_int32(degree), C.c_double(a0), C.c_double(lam_cut),
                                          C.c_double(lam_max)))

    def xls_subdomain_project(self, gemm_prec: int = XLS_PREC_FP64):
        M = np.zeros((self.ns, self.ns), order="F")
        Hs = np.zeros((self.ns, self.ns), order="F")
        _check(lib().xls_subdomain_project(self._h, C.c_int32(gemm_prec), _dp(M), _dp(Hs)))
        return M, Hs

    def xls_subdomain_rotate(self, Q: np.ndarray, gemm_prec: int = XLS_PREC_FP64):
        Qf = _f64(Q)
        _check(lib().xls_subdomain_rotate(self._h, C.c_int32(gemm_prec), _dp(Qf)))

    def xls_subdomain_residual(self, lam: np.ndarray) -> np.ndarray:
        lam = _f64(lam, order="C")
        r = np.zeros(self.ns)
        _check(lib().xls_subdomain_residual(self._h, _dp(lam), _dp(r)))
        return r

    def xls_lanczos_bounds(self, k: int = 20):
        lo = C.c_double()
        up = C.c_double()
        _check(lib().xls_lanczos_bounds(self._h, C.c_int32(k), C.byref(lo), C.byref(up)))
        return lo.value, up.value

    def xls_subdomain_get_block(self) -> np.ndarray:
        X = np.zeros((self.nd, self.ns), order="F")
        _check(lib().xls_subdomain_get_block(self._h, _dp(X)))
        return X

    def xls_subdomain_set_block(self, X: np.ndarray):
        Xf = _f64(X)
        _check(lib().xls_subdomain_set_block(self._h, _dp(Xf)))

    def xls_subdomain_get_maps(self):
        m = np.zeros(self.nd, dtype=np.uint8)
        g = np.zeros(self.nd, dtype=np.int64)
        _check(lib().xls_subdomain_get_maps(self._h, m.ctypes.data_as(C.POINTER(C.c_uint8)),
                                            g.ctypes.data_as(C.POINTER(C.c_int64))))
        return m, g

    def xls_subdomain_get_projectors(self):
        sizes = np.zeros(2, dtype=np.int64)
        P64 = C.POINTER(C.c_int64)
        _check(lib().xls_subdomain_get_projectors(self._h, sizes.ctypes.data_as(P64), None, None, None,
                                                  None, None))
        total, na = int(sizes[0]), int(sizes[1])
        off = np.zeros(na + 1, dtype=np.int32)
        idx = np.zeros(total, dtype=np.int32)
        val = np.zeros((total, 4))
        roff = np.zeros(self.nd + 1, dtype=np.int32)
        rslot = np.zeros(total, dtype=np.int32)
        P32 = C.POINTER(C.c_int32)
        _check(lib().xls_subdomain_get_projectors(
            self._h, sizes.ctypes.data_as(P64), off.ctypes.data_as(P32), idx.ctypes.data_as(P32),
            _dp(val), roff.ctypes.data_as(P32), rslot.ctypes.data_as(P32)))
        return off, idx, val, roff, rslot

    def xls_subdomain_store_half(self, buf):
        """Current block -> buf, a contiguous device torch.float16 tensor of at
        least N_d*ns elements (column-major, leading dimension N_d)."""
        _check(lib().xls_subdomain_store_half(self._h, C.c_void_p(int(buf.data_ptr()))))
        return buf

    def xls_subdomain_load_half(self, buf):
        """Block <- buf (device torch.float16, as written by xls_subdomain_store_half)."""
        _check(lib().xls_subdomain_load_half(self._h, C.c_void_p(int(buf.data_ptr()))))

    def xls_subdomain_pdos(self, orb_width: float, orb_rc: float, edges=None, n_atoms: Optional[int] = None):
        """(weights [ns, 4 n_atoms], pdos [4 n_atoms, nbins] or None, in_core [n_atoms])."""
        if n_atoms is None:
            sizes = np.zeros(2, dtype=np.int64)
            _check(lib().xls_subdomain_get_projectors(self._h, sizes.ctypes.data_as(C.POINTER(C.c_int64)), None,
                                                      None, None, None, None))
            n_atoms = int(sizes[1])
        w = np.zeros((self.ns, 4 * n_atoms))
        e = None if edges is None else np.ascontiguousarray(edges, dtype=np.float64)
        nb = 0 if e is None else len(e) - 1
        d = np.zeros((4 * n_atoms, max(nb, 1)))
        inc = np.zeros(max(n_atoms, 1), dtype=np.uint8)
        _check(lib().xls_subdomain_pdos(self._h, C.c_double(orb_width), C.c_double(orb_rc), _dp(w), C.c_int32(nb),
                                        _dp(e) if e is not None else None, _dp(d) if nb > 0 else None,
                                        inc.ctypes.data_as(C.POINTER(C.c_uint8))))
        return w, (d[:, :nb] if nb > 0 else None), inc[:n_atoms].astype(bool)

    def xls_subdomain_use_half(self, buf):
        """Next filter reads its start block from buf (device torch.float16) directly."""
        _check(lib().xls_subdomain_use_half(self._h, C.c_void_p(int(buf.data_ptr()))))

    def xls_subdomain_tune(self, prec: int, block: int = 512, ty: int = 0, tz: int = 0, nv: int = 0):
        _check(lib().xls_subdomain_tune(self._h, C.c_int32(prec), C.c_int32(block), C.c_int32(ty),
                                        C.c_int32(tz), C.c_int32(nv)))

    def xls_subdomain_tune_gemm(self, split_scale: int = 0, tile_tn: int = 0, tile_nn: int = 0):
        _check(lib().xls_subdomain_tune_gemm(self._h, C.c_int32(split_scale), C.c_int32(tile_tn),
                                             C.c_int32(tile_nn)))

    def xls_subdomain_time_gemms(self, gemm_prec: int, reps: int = 5) -> np.ndarray:
        """Average device ms of (Psi^T Psi, Psi^T H Psi, Psi Q) at gemm_prec."""
        ms = np.zeros(3)
        rc = lib().xls_subdomain_time_gemms(self._h, C.c_int32(gemm_prec), C.c_int32(reps), _dp(ms))
        if rc < 0:
            _check(rc)
        return ms

    def xls_subdomain_features(self) -> np.ndarray:
        f = np.zeros(64)
        _check(lib().xls_subdomain_features(self._h, _dp(f)))
        return f

    def xls_subdomain_counters(self):
        out = np.zeros(3, dtype=np.int64)
        _check(lib().xls_subdomain_counters(self._h, out.ctypes.data_as(C.POINTER(C.c_int64)), C.c_int32(3)))
        return {"h_applies": int(out[0]), "fallback": bool(out[1]), "iterations": int(out[2])}

    def xls_get_stage_times(self):
        ms = np.zeros(8)
        cnt = np.zeros(1, dtype=np.int64)
        n = _check(lib().xls_get_stage_times(self._h, _dp(ms), cnt.ctypes.data_as(C.POINTER(C.c_int64)),
                                             C.c_int32(8)))
        return ms[:n], int(cnt[0])


class Batch:
    """Owner of one xls_batch_t (xls_batch_create / _destroy): many subdomains
    advanced together."""

    def __init__(self, sds, filter_prec: int = XLS_PREC_FP32, x0s=None, x0_seeds=None,
                 slots: Optional[int] = None):
        """x0_seeds: per subdomain, draw the start block on the device;
        slots: None for a resident batch (xls_batch_create), else the byte
        budget of xls_batch_create_slots (0: 85 % of free device memory)."""
        x0s = [None] * len(sds) if x0s is None else x0s
        seeds = [None] * len(sds) if x0_seeds is None else x0_seeds
        descs = (xls_subdomain_desc_t * len(sds))()
        keep = []
        for i, (sd, x0, sdseed) in enumerate(zip(sds, x0s, seeds)):
            d, k = make_desc(sd, filter_prec, x0, x0_seed=sdseed)
            descs[i] = d
            keep.append(k)
        h = C.c_void_p()
        if slots is None:
            _check(lib().xls_batch_create(C.c_int32(len(sds)), descs, C.byref(h)))
        else:
            _check(lib().xls_batch_create_slots(C.c_int32(len(sds)), descs, C.c_int64(int(slots)), C.byref(h)))
        del keep
        self._h = h
        self.prec = int(filter_prec)
        self.shapes = [(tuple(int(v) for v in sd.n), int(descs[i].ns)) for i, sd in enumerate(sds)]
        self.n = len(sds)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().xls_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def xls_batch_chefsi(self, params, use_graph: bool = True):
        """params: list of xls_chefsi_params_t (chefsi_params(...)), one per subdomain.
        Returns (ritz list, resid list, iters, status)."""
        P = (xls_chefsi_params_t * self.n)(*params)
        tot = sum(ns for _, ns in self.shapes)
        ritz = np.zeros(tot)
        resid = np.zeros(tot)
        iters = np.zeros(self.n, dtype=np.int32)
        status = np.zeros(self.n, dtype=np.int32)
        _check(lib().xls_batch_chefsi(self._h, P, _dp(ritz), _dp(resid),
                                      iters.ctypes.data_as(C.POINTER(C.c_int32)),
                                      status.ctypes.data_as(C.POINTER(C.c_int32)), C.c_int32(1 if use_graph else 0)))
        off = np.cumsum([0] + [ns for _, ns in self.shapes])
        return ([ritz[off[i]:off[i + 1]] for i in range(self.n)], [resid[off[i]:off[i + 1]] for i in range(self.n)],
                iters, status)

    def xls_batch_density(self, mu: float, sigma: float):
        nds = [int(np.prod(n)) for n, _ in self.shapes]
        rho = np.zeros(sum(nds))
        c = np.zeros(sum(ns for _, ns in self.shapes))
        _check(lib().xls_batch_density(self._h, C.c_double(mu), C.c_double(sigma), _dp(rho), _dp(c)))
        ro = np.cumsum([0] + nds)
        co = np.cumsum([0] + [ns for _, ns in self.shapes])
        return [rho[ro[i]:ro[i + 1]] for i in range(self.n)], [c[co[i]:co[i + 1]] for i in range(self.n)]

    def xls_batch_fermi(self, sigma: float, n_electrons: float):
        """(mu, N_e(mu), E_band, E_entropy, evaluations) of the whole batch."""
        out = np.zeros(5)
        n = _check(lib().xls_batch_fermi(self._h, C.c_double(sigma), C.c_double(n_electrons), _dp(out),
                                         C.c_int32(5)))
        return tuple(float(v) for v in out[:n])

    def xls_batch_assemble(self, n_global: int = 0, edges=None):
        """(global density or None, DOS or None) at the last xls_batch_fermi's mu."""
        rho = np.zeros(int(n_global)) if n_global > 0 else None
        e = None if edges is None else np.ascontiguousarray(edges, dtype=np.float64)
        nb = 0 if e is None else len(e) - 1
        dos = np.zeros(max(nb, 0))
        _check(lib().xls_batch_assemble(self._h, C.c_int64(int(n_global)), _dp(rho) if rho is not None else None,
                                        C.c_int32(nb), _dp(e) if e is not None else None,
                                        _dp(dos) if nb > 0 else None))
        return rho, (dos if nb > 0 else None)

    def xls_batch_subdomain(self, i: int) -> Subdomain:
        h = C.c_void_p()
        _check(lib().xls_batch_subdomain(self._h, C.c_int32(i), C.byref(h)))
        n, ns = self.shapes[i]
        return Subdomain._borrow(h, n, ns, self.prec)

    def xls_batch_tune(self, cache_path: Optional[str] = None):
        tuned = C.c_int32(0)
        best = C.c_double(0.0)
        path = cache_path.encode() if cache_path else None
        _check(lib().xls_batch_tune(self._h, C.c_char_p(path), C.byref(tuned), C.byref(best)))
        return int(tuned.value), float(best.value)

    def xls_batch_stats(self):
        out = np.zeros(7)
        _check(lib().xls_batch_stats(self._h, _dp(out), C.c_int32(7)))
        return {"iterations": int(out[0]), "captures": int(out[1]), "replays": int(out[2]),
                "iter_ms": float(out[3]), "last_iter_ms": float(out[4]), "peak_bytes": int(out[5]),
                "max_active": int(out[6])}


def _fp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Mlp:
    """Owner of one xls_mlp_t.  Parameters are exchanged as the oracle's list
    [W1, b1, W2, b2, ...] with W_l of shape (fan_in, fan_out)."""

    def __init__(self, sizes=(64, 128, 128, 3), params=None):
        self.sizes = tuple(int(v) for v in sizes)
        sz = (C.c_int32 * len(self.sizes))(*self.sizes)
        flat = None if params is None else self._flatten(params)
        h = C.c_void_p()
        _check(lib().xls_mlp_create(C.c_int32(len(self.sizes)), sz, None if flat is None else _fp(flat),
                                    C.byref(h)))
        self._h = h
        self.nparam = _check(lib().xls_mlp_get_params(self._h, None, C.c_int64(0)))

    def _flatten(self, params) -> np.ndarray:
        return np.concatenate([np.ascontiguousarray(p, dtype=np.float32).ravel() for p in params])

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().xls_mlp_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def get_params(self):
        flat = np.zeros(self.nparam, dtype=np.float32)
        _check(lib().xls_mlp_get_params(self._h, _fp(flat), C.c_int64(flat.size)))
        out, off = [], 0
        for a, b in zip(self.sizes[:-1], self.sizes[1:]):
            out.append(flat[off:off + a * b].reshape(a, b))
            off += a * b
            out.append(flat[off:off + b].copy())
            off += b
        return out

    def set_params(self, params):
        flat = self._flatten(params)
        _check(lib().xls_mlp_set_params(self._h, _fp(flat), C.c_int64(flat.size)))

    def set_norm(self, in_mean, in_std, out_mean, out_std):
        im = np.ascontiguousarray(in_mean, dtype=np.float32)
        isd = np.ascontiguousarray(in_std, dtype=np.float32)
        om = np.ascontiguousarray(out_mean, dtype=np.float64)
        osd = np.ascontiguousarray(out_std, dtype=np.float64)
        _check(lib().xls_mlp_set_norm(self._h, _fp(im), _fp(isd), _dp(om), _dp(osd)))

    def forward(self, X: np.ndarray) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.zeros((X.shape[0], self.sizes[-1]), dtype=np.float32)
        _check(lib().xls_mlp_forward(self._h, _fp(X), C.c_int32(X.shape[0]), _fp(Y)))
        return Y

    def gradient(self, X: np.ndarray, T: np.ndarray):
        X = np.ascontiguousarray(X, dtype=np.float32)
        T = np.ascontiguousarray(T, dtype=np.float32)
        g = np.zeros(self.nparam, dtype=np.float32)
        loss = C.c_float(0.0)
        _check(lib().xls_mlp_gradient(self._h, _fp(X), _fp(T), C.c_int32(X.shape[0]), _fp(g), C.byref(loss)))
        out, off = [], 0
        for a, b in zip(self.sizes[:-1], self.sizes[1:]):
            out.append(g[off:off + a * b].reshape(a, b))
            off += a * b
            out.append(g[off:off + b].copy())
            off += b
        return out, float(loss.value)

    def train(self, X: np.ndarray, T: np.ndarray, batches, lr: float = 1e-3) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float32)
        T = np.ascontiguousarray(T, dtype=np.float32)
        idx = np.ascontiguousarray(np.concatenate([np.asarray(b) for b in batches]) if batches else np.zeros(0),
                                   dtype=np.int32)
        off = np.ascontiguousarray(np.cumsum([0] + [len(b) for b in batches]), dtype=np.int32)
        losses = np.zeros(max(1, len(batches)), dtype=np.float32)
        _check(lib().xls_mlp_train(self._h, _fp(X), _fp(T), C.c_int32(X.shape[0]),
                                   idx.ctypes.data_as(C.POINTER(C.c_int32)),
                                   off.ctypes.data_as(C.POINTER(C.c_int32)), C.c_int32(len(batches)),
                                   C.c_float(lr), _fp(losses)))
        return losses[:len(batches)]

    def predict(self, F: np.ndarray) -> np.ndarray:
        F = np.ascontiguousarray(F, dtype=np.float64)
        out = np.zeros((F.shape[0], self.sizes[-1]))
        _check(lib().xls_mlp_predict(self._h, _dp(F), C.c_int32(F.shape[0]), _dp(out)))
        return out

    def fit(self, F: np.ndarray, T: np.ndarray, batches, lr: float = 1e-3) -> np.ndarray:
        """xls_mlp_fit: standardise raw features and targets, train, keep the
        standardisation and the training RMS error in the model."""
        F = np.ascontiguousarray(F, dtype=np.float64)
        T = np.ascontiguousarray(T, dtype=np.float64)
        idx = np.ascontiguousarray(np.concatenate([np.asarray(b) for b in batches]) if batches else np.zeros(0),
                                   dtype=np.int32)
        off = np.ascontiguousarray(np.cumsum([0] + [len(b) for b in batches]), dtype=np.int32)
        losses = np.zeros(max(1, len(batches)), dtype=np.float32)
        _check(lib().xls_mlp_fit(self._h, _dp(F), _dp(T), C.c_int32(F.shape[0]),
                                 idx.ctypes.data_as(C.POINTER(C.c_int32)),
                                 off.ctypes.data_as(C.POINTER(C.c_int32)), C.c_int32(len(batches)),
                                 C.c_float(lr), _fp(losses)))
        return losses[:len(batches)]

    def train_rms(self) -> np.ndarray:
        out = np.zeros(8)
        n = _check(lib().xls_mlp_train_rms(self._h, _dp(out), C.c_int32(8)))
        return out[:n]

    def bounds(self, F: np.ndarray):
        """xls_mlp_bounds: (lambda_max, lambda_cut, degree) a learned run takes."""
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(-1, self.sizes[0])
        B = F.shape[0]
        lm, lc = np.zeros(B), np.zeros(B)
        deg = np.zeros(B, dtype=np.int32)
        _check(lib().xls_mlp_bounds(self._h, _dp(F), C.c_int32(B), _dp(lm), _dp(lc),
                                    deg.ctypes.data_as(C.POINTER(C.c_int32))))
        return lm, lc, deg


def xls_learned_safe_bounds(lam_max, lam_cut, cut_margin: float = 0.0):
    """Bounds a learned run takes from given (lambda_max, lambda_cut)."""
    lmx = np.ascontiguousarray(np.atleast_1d(lam_max), dtype=np.float64)
    lct = np.ascontiguousarray(np.atleast_1d(lam_cut), dtype=np.float64)
    lm, lc = np.zeros(lmx.size), np.zeros(lmx.size)
    _check(lib().xls_learned_safe_bounds(C.c_int32(lmx.size), _dp(lmx), _dp(lct), C.c_double(cut_margin),
                                         _dp(lm), _dp(lc)))
    return lm, lc


class Poisson:
    """Owner of one xls_poisson_t: -(1/(4 pi)) Lap phi = f by multigrid-preconditioned CG."""

    def __init__(self, n, h: float, bc: int, max_levels: int = 0):
        self.n = tuple(int(v) for v in n)
        self.nd = int(np.prod(self.n))
        nn = (C.c_int32 * 3)(*self.n)
        hh = C.c_void_p()
        _check(lib().xls_poisson_create(nn, C.c_double(h), C.c_int32(bc), C.c_int32(max_levels), C.byref(hh)))
        self._h = hh

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().xls_poisson_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def solve(self, f, tol: float = 1e-10, max_iter: int = 500, precondition: bool = True):
        """(phi, info) with info = (iterations, relative residual, levels, ms)."""
        ff = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        phi = np.zeros(self.nd)
        info = np.zeros(4)
        _check(lib().xls_poisson_solve(self._h, _dp(ff), _dp(phi), C.c_double(tol), C.c_int32(max_iter),
                                       C.c_int32(1 if precondition else 0), _dp(info)))
        return phi, (int(info[0]), float(info[1]), int(info[2]), float(info[3]))

    def solve_device(self, f, phi, tol: float = 1e-10, max_iter: int = 500, precondition: bool = True):
        """Solve with f and phi device tensors of nd float64 values (device
        pointers only; no transfer).  Returns info = (iterations, relative
        residual, levels, ms)."""
        for t, name in ((f, "f"), (phi, "phi")):
            if not (t.is_cuda and t.dtype.itemsize == 8 and t.is_contiguous() and t.numel() == self.nd):
                raise ValueError(f"{name} must be a contiguous float64 device tensor of {self.nd} values")
        info = np.zeros(4)
        _check(lib().xls_poisson_solve_device(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(phi.data_ptr()),
                                              C.c_double(tol), C.c_int32(max_iter),
                                              C.c_int32(1 if precondition else 0), _dp(info)))
        return int(info[0]), float(info[1]), int(info[2]), float(info[3])

    def vcycle(self, r):
        rr = np.ascontiguousarray(r, dtype=np.float64).reshape(-1)
        z = np.zeros(self.nd)
        _check(lib().xls_poisson_vcycle(self._h, _dp(rr), _dp(z)))
        return z
