"""Benchmark: subdomain CheFSI on one MI355X.

Headline (value, dtype f64): a 64^3 zero-Dirichlet box (h = 0.432 bohr)
around a 64-atom displaced diamond-Si core, 279 atoms with Kleinman-Bylander
projectors, ns = 480 vectors, filter degree m = 24 (synthetic stand-in for
the paper's Si subsystems).  A step is one FP64 CheFSI iteration: m fused
filter sweeps, H*Psi_f, the two projection GEMMs, the FP64 dense eigensolve,
the rotation and the FP64 residual check; value = N_d * ns * m / step time.
The mixed form (FP32 filter + split-BF16 GEMMs + FP64 dense) is reported
beside it.  roofline prices the FP64 fused filter kernel (3 words per
grid-pt*vec*deg) against 8 TB/s from HIP events around every filter launch,
and against a device-to-device copy measured in the same run.

batch: the 256-subdomain uneven draw at full size, solved to a gated
residual of 1e-4 (at most 45 iterations, so the plain method converges at
the low degrees of the draw) with slot residency, once in FP64 with Lanczos
bounds and the draw's degrees, and once mixed with learned bounds and
degrees (model trained first on method-made labels of smaller boxes of the
same recipe); subdomains/s, converged counts, and the |Ritz difference| over
the gated states of subdomains both forms converged (largest, 99th
percentile, count above 1e-6 Ha).  The mixed form reports the FP64 Rayleigh
quotients of its vectors, so what separates the two forms is the
convergence error of each (about r^2 / gap).  learned_gain: the first 32 subdomains, mixed with Lanczos
bounds against mixed with learned bounds (one precision).  gemm_large: the
96^3, Ns = 2,400 GEMM rates and their errors against FP64.  cpu_baseline
times the FP64 oracle's filter on a column sample on the host.  widened:
the binary16 warm-start filter steps, the PDOS of the 64^3 block and a
255^3 multigrid-preconditioned Poisson solve.  The optional learned_gain
leg is skipped, and the line says so, when the run
has used more than --budget-s seconds before it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch 256] [--gain 32]
                    [--no-gemm-large] [--headline-only] [--no-cpu] [--budget-s 720]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"bf16x3": 2500.0, "fp32": 157.3, "fp64": 78.6}  # dense, per MFMA dtype
METRIC = "filtered grid-pt\u00b7vec\u00b7deg/s + subdomains/s: FP64 vs mixed+learned, dE<=1e-6 Ha"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "filter_traffic.json")
STENCIL_SOURCES = ["stencil_impl.h", "stencil_f32.hip", "stencil_f64.hip", "stencil_mix.hip"]
BATCH_TOL = 1e-4        # gated residual of the batch legs
BATCH_MAX_ITER = 45


def stencil_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in STENCIL_SOURCES:
        with open(os.path.join(ROOT, "paper_2609_13115_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(form: str):
    """HBM bytes per filter launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes (scaled by the copy-kernel calibration), or None when
    the filter kernel's sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != stencil_source_hash() or form not in t.get("forms", {}):
        return None
    f = t["forms"][form]
    return f["fetch_bytes"] + f["write_bytes"]


def _pmc_values(path: str, counter: str, form: str):
    """Per-dispatch values of one counter from a rocprofv3 counter CSV:
    (the form's fused-filter launches, device-to-device copy launches).  A
    --headline-only process runs both forms; the block type tells them apart
    (double: fp64, float: mixed)."""
    import csv

    want = "double" if form == "fp64" else "float"
    filt, copy = [], []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            name, v = r["Kernel_Name"], float(r["Counter_Value"])
            if "hstencil_kernel<" in name:
                args = [a.strip() for a in name[name.index("<") + 1:name.index(">")].split(",")]
                if args[0] == want and args[2] == "1":  # MODE 1: fused filter step
                    filt.append(v)
            elif "copyBuffer" in name:
                copy.append(v)
    return filt, copy


def write_traffic(form: str, fetch_csv: str, write_csv: str):
    """profiles/filter_traffic.json entry of one form from a FETCH_SIZE and a
    WRITE_SIZE rocprofv3 pass of `bench.py --calib-mib 1024`: the median per
    filter launch (KiB), scaled by what the same counter reads for the
    largest (1 GiB) device-to-device copies, which move exactly 1 GiB each
    way.  Stamped with the stencil sources' hash."""
    out = {}
    for key, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        filt, copy = _pmc_values(path, counter, form)
        if not filt or not copy:
            raise SystemExit(f"{path}: no filter or copy dispatches for {counter}")
        big = [c for c in copy if c >= 0.9 * max(copy)]
        cal = float(np.median(big))
        scale = float(1 << 20) / cal  # 1 GiB in KiB over the counter's reading
        med = float(np.median(filt))
        out[f"{key}_bytes"] = med * 1024 * scale
        out[f"{key}_kib_raw_median"] = med
        out[f"{key}_scale"] = scale
        out[f"copy_1GiB_{key}_kib"] = cal
        out["launches"] = len(filt)
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        t = {}
    h = stencil_source_hash()
    if t.get("source_sha256") != h:
        t = {"source_sha256": h, "kiB": 1024, "forms": {}}
    t["forms"][form] = out
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(t, fh, indent=1)
    print(json.dumps({form: out}))


def run_form(sd, x0, form: str, steps: int, warmup: int, degree: int):
    import torch
    from paper_2609_13115_amd import xls

    prec = xls.XLS_PREC_FP64 if form == "fp64" else xls.XLS_PREC_FP32
    gprec = xls.XLS_PREC_FP64 if form == "fp64" else xls.XLS_PREC_BF16X3
    wbytes = 8 if form == "fp64" else 4
    with xls.Subdomain(sd, filter_prec=prec, x0=x0) as s:
        lo, up = s.xls_lanczos_bounds(20)
        ritz, resid, _ = s.xls_chefsi_step(degree, max(1, warmup), xls.XLS_BOUNDS_LANCZOS, gemm_prec=gprec)
        xls.xls_set_profiling(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ritz, resid, it = s.xls_chefsi_step(degree, steps, xls.XLS_BOUNDS_GIVEN, ritz[0], ritz[-1], up,
                                            gemm_prec=gprec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        xls.xls_set_profiling(False)
        ms, nlaunch = s.xls_get_stage_times()
        gemm = time_gemms(s, sd.nd, x0.shape[1], form)
        half = half_storage_timing(s, sd.nd, x0.shape[1], wbytes)
    step_ms = (t1 - t0) * 1e3 / it
    nd, ns = sd.nd, x0.shape[1]
    units = nd * ns * degree
    filt_avg_ms = ms[7] / max(1, nlaunch)
    bytes_per_launch = 3.0 * nd * ns * wbytes
    achieved = bytes_per_launch / (filt_avg_ms * 1e-3) / 1e9
    return {
        "value": units / (step_ms * 1e-3),
        "ms_per_step": step_ms,
        "iters": it,
        "filter_rate": nd * ns * nlaunch / (ms[7] * 1e-3) if ms[7] > 0 else None,
        "filter_kernel_avg_ms": filt_avg_ms,
        "filter_launches": nlaunch,
        "stage_ms_per_step": {k: v / it for k, v in zip(
            ["filter", "h_psi", "projection", "dense", "rotation", "residual", "total"], ms[:7])},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(form),
                     "algorithmic_bytes": bytes_per_launch},
        "max_resid": float(np.max(resid)),
        "ritz_lo": float(ritz[0]),
        "gemm": gemm,
        "half_storage": half,
    }


def half_storage_timing(s, nd: int, ns: int, wbytes: int, reps: int = 5):
    """FP16 warm-start storage of the block (xls_subdomain_store_half / _load_half):
    best wall time of reps calls each, priced at the bytes they must move
    (read w + write 2 bytes per value, and back)."""
    import torch

    buf = torch.empty(nd * ns, dtype=torch.float16, device="cuda")
    s.xls_subdomain_store_half(buf)
    ts, tl = 1e9, 1e9
    for _ in range(reps):
        t0 = time.perf_counter()
        s.xls_subdomain_store_half(buf)
        ts = min(ts, time.perf_counter() - t0)
    for _ in range(reps):
        t0 = time.perf_counter()
        s.xls_subdomain_load_half(buf)
        tl = min(tl, time.perf_counter() - t0)
    nbytes = float(nd) * ns * (wbytes + 2)
    return {"store_ms": ts * 1e3, "load_ms": tl * 1e3, "bytes_each": nbytes,
            "store_gbs": nbytes / ts / 1e9, "load_gbs": nbytes / tl / 1e9, "half_bytes": float(nd) * ns * 2}


def widened_rows(sd, reps: int = 3):
    """The rows beyond the CheFSI step, measured beside it.
    warm_start: the first two filter steps on the 64^3 box (FP32 form, degree
    24 bounds) reading a binary16 warm start directly (xls_subdomain_use_half)
    against the same two steps from an FP32 block holding the same values
    (xls_subdomain_load_half): fused-kernel time from HIP events, best of
    reps; bytes per point*vector 6 + 10 (half input) against 8 + 12.
    pdos: xls_subdomain_pdos of the box's block after two mixed CheFSI
    iterations (s and p orbitals on all 279 atoms, width 0.5 bohr, rc 2 bohr,
    200 bins over the Ritz range), best wall time of reps calls including the
    host copy of the weights (ns x 4 atoms doubles).
    poisson: -(1/(4 pi)) Lap phi = f on a 255^3 zero-Dirichlet grid at
    h = 0.4 bohr (16.6 M points), f random-normal (seeded), tol 1e-10, device
    arrays (xls_poisson_solve_device): wall time, iterations, multigrid
    levels, and unpreconditioned CG's iteration count beside it."""
    import torch
    from paper_2609_13115_amd import xls

    out = {}
    nd, ns = sd.nd, sd.x0.shape[1]
    buf = torch.empty(nd * ns, dtype=torch.float16, device="cuda")
    with xls.Subdomain(sd, filter_prec=xls.XLS_PREC_FP32) as s:
        lo, up = s.xls_lanczos_bounds(20)
        lc = lo + 0.1 * (up - lo)
        s.xls_subdomain_store_half(buf)
        xls.xls_set_profiling(True)
        best = {"half": 1e9, "fp32": 1e9}
        for _ in range(reps):
            for form in ("half", "fp32"):
                if form == "half":
                    s.xls_subdomain_use_half(buf)
                else:
                    s.xls_subdomain_load_half(buf)
                s.xls_subdomain_filter(2, lo, lc, up)
                ms, n = s.xls_get_stage_times()
                best[form] = min(best[form], float(ms[7]))
        xls.xls_set_profiling(False)
        out["warm_start"] = {"two_steps_half_input_ms": best["half"], "two_steps_fp32_ms": best["fp32"],
                             "ratio": best["half"] / best["fp32"], "bytes_ratio": 16.0 / 20.0,
                             "half_input_gbs": 16.0 * nd * ns / (best["half"] * 1e-3) / 1e9,
                             "fp32_gbs": 20.0 * nd * ns / (best["fp32"] * 1e-3) / 1e9}
        s.xls_subdomain_load_half(buf)
        ritz, _, _ = s.xls_chefsi_step(24, 2, xls.XLS_BOUNDS_LANCZOS, gemm_prec=xls.XLS_PREC_BF16X3)
        edges = np.linspace(float(ritz.min()) - 1e-9, float(ritz.max()) + 1e-9, 201)
        t = 1e9
        for _ in range(reps):
            t0 = time.perf_counter()
            w, d, inc = s.xls_subdomain_pdos(0.5, 2.0, edges)
            t = min(t, time.perf_counter() - t0)
        out["pdos"] = {"ms": t * 1e3, "states": int(w.shape[0]), "orbitals": int(w.shape[1]), "bins": 200,
                       "core_atoms": int(np.sum(inc)), "weight_sum": float(np.sum(d))}
    del buf
    torch.cuda.empty_cache()
    n = (255, 255, 255)
    f = torch.tensor(np.random.default_rng(20260913).standard_normal(int(np.prod(n))), dtype=torch.float64,
                     device="cuda")
    phi = torch.zeros_like(f)
    with xls.Poisson(n, 0.4, 1) as p:
        p.solve_device(f, phi, tol=1e-10)  # warm-up
        it, rel, lev, ms = p.solve_device(f, phi, tol=1e-10)
        it0, rel0, _, ms0 = p.solve_device(f, phi, tol=1e-10, max_iter=20000, precondition=False)
    npts = float(np.prod(n))
    out["poisson"] = {"grid": "255^3 zero Dirichlet, h 0.4 bohr", "points": npts, "tol": 1e-10,
                      "iterations": it, "rel_resid": rel, "levels": lev, "ms": ms, "ms_per_iteration": ms / it,
                      "unpreconditioned_iterations": it0, "unpreconditioned_ms": ms0}
    del f, phi
    torch.cuda.empty_cache()
    print(f"[bench] widened rows: {json.dumps(out)}", file=sys.stderr, flush=True)
    return out


def time_gemms(s, nd: int, ns: int, form: str, reps: int = 5):
    """TFLOP/s of the three GEMMs at each precision of the form: algorithmic
    flops (N_d N_s^2 for the two projections, which form one triangle each,
    2 N_d N_s^2 for the rotation) and issued MFMA flops (x3 for the
    split-BF16 form) against the dtype's dense peak."""
    from paper_2609_13115_amd import xls

    precs = [("fp64", xls.XLS_PREC_FP64)] if form == "fp64" else [("bf16x3", xls.XLS_PREC_BF16X3),
                                                                   ("fp32", xls.XLS_PREC_FP32)]
    flops = {"xtx": nd * ns * ns, "xthx": nd * ns * ns, "rotation": 2.0 * nd * ns * ns}
    out = {}
    for name, p in precs:
        ms = s.xls_subdomain_time_gemms(p, reps)
        issue = 3.0 if name == "bf16x3" else 1.0
        o = {}
        for (k, f), t in zip(flops.items(), ms):
            tf = f / (t * 1e-3) / 1e12
            o[k] = {"ms": t, "tflops": tf, "issued_tflops": issue * tf,
                    "frac": issue * tf / MFMA_PEAK_TFLOPS[name]}
        out[name] = o
    return out


def gemm_large(reps: int = 3):
    """The large-subdomain GEMM shape (96^3 box, N_d = 884,736, Ns = 2,400):
    X random-normal (drawn on the device), filtered twice at degree 24 by the
    FP64 path with Lanczos bounds.  On that X: M = X^T X and H_s = X^T H X in
    FP64 (FP64 block), and in FP32 and split-BF16 on the FP32 rounding of X
    (FP32 block, FP32 H); rates of the three GEMMs (HIP events) in every
    precision; errors against the FP64 products: relative Frobenius error of
    M and H_s, the largest |Ritz value difference| of the pencils (H_s, M)
    over the lowest N_occ = floor(Ns / 1.1), and sin theta between their
    lowest N_occ eigenvector spaces (in the metric of the FP64 M, so equal to
    the angle between the rotated blocks up to the FP32 rounding of X)."""
    import scipy.linalg as sla
    from paper_2609_13115_amd import workloads, xls

    sd = workloads.si_box_96(with_x0=False)
    nd, ns = sd.nd, sd.ns
    seed = workloads.x0_seed(sd.seed_key)
    nocc = int(np.floor(ns / 1.1 + 1e-9))
    out = {"workload": f"96^3 zero-Dirichlet Si box, N_d = {nd}, Ns = {ns}; X random-normal filtered twice "
                       f"(degree 24, FP64)"}
    t0 = time.perf_counter()
    with xls.Subdomain(sd, filter_prec=xls.XLS_PREC_FP64, x0_seed=seed) as s:
        lo, up = s.xls_lanczos_bounds(20)
        lc = lo + 0.1 * (up - lo)
        s.xls_subdomain_filter(24, lo, lc, up)
        s.xls_subdomain_filter(24, lo, lc, up)
        M64, H64 = s.xls_subdomain_project(xls.XLS_PREC_FP64)
        out.update(time_gemms(s, nd, ns, "fp64", reps))
        X = s.xls_subdomain_get_block()
    print(f"[bench] gemm_large fp64 done ({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    lam64, Y64 = xls.xls_dense_geneig(H64, M64)
    R = sla.cholesky(M64, lower=False)
    B64 = R @ Y64[:, :nocc]  # orthonormal: Y^T M Y = I
    errs = {}
    with xls.Subdomain(sd, filter_prec=xls.XLS_PREC_FP32, x0_seed=seed) as s:
        s.xls_subdomain_set_block(X)
        del X
        out.update(time_gemms(s, nd, ns, "mixed", reps))
        for name, prec in (("fp32", xls.XLS_PREC_FP32), ("bf16x3", xls.XLS_PREC_BF16X3)):
            M, H = s.xls_subdomain_project(prec)
            lam, Y = xls.xls_dense_geneig(H, M)
            Bp, _ = np.linalg.qr(R @ Y[:, :nocc])
            D = Bp - B64 @ (B64.T @ Bp)
            errs[name] = {"M_rel_fro": float(np.linalg.norm(M - M64) / np.linalg.norm(M64)),
                          "Hs_rel_fro": float(np.linalg.norm(H - H64) / np.linalg.norm(H64)),
                          "max_ritz_diff": float(np.max(np.abs(lam[:nocc] - lam64[:nocc]))),
                          "max_ritz_diff_rel": float(np.max(np.abs(lam[:nocc] - lam64[:nocc]) /
                                                            np.maximum(np.abs(lam64[:nocc]), 1e-3))),
                          "sin_theta": float(np.linalg.norm(D, 2))}
    out["errors_vs_fp64"] = errs
    out["n_occ"] = nocc
    print(f"[bench] gemm_large: {json.dumps(errs)} ({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    return out


def train_learned(n_train: int = 64, max_iter: int = 16, tol: float = BATCH_TOL):
    """The learned-bounds model for the batch workload: labels from the method
    (batch engine, FP32 filter and GEMMs) on n_train smaller boxes of the same
    recipe (core 8-40 atoms, a different draw of the crystal), then training
    with the library's kernels (xls_mlp_fit)."""
    from paper_2609_13115_amd import learned, workloads

    t0 = time.perf_counter()
    _, train, _ = workloads.batch_subdomains(count=n_train, key_cfg=6, nmin=20, nmax=60, core_atoms=(8, 40))
    lab = learned.label_subdomains(train, max_iter=max_iter, tol=tol)
    t1 = time.perf_counter()
    model, losses = learned.train_model(lab.features, lab.targets, epochs=300)
    t2 = time.perf_counter()
    info = {"training_boxes": n_train, "grids": f"{min(sd.n[0] for sd in train)}^3-{max(sd.n[0] for sd in train)}^3",
            "labels_s": t1 - t0, "train_s": t2 - t1, "labels_converged": float(lab.converged.mean()),
            "loss_first": float(np.mean(losses[:20])), "loss_last": float(np.mean(losses[-20:])),
            "train_rms": [float(v) for v in model.train_rms()]}
    print(f"[bench] learned model: {json.dumps(info)}", file=sys.stderr, flush=True)
    return model, info


def copy_rate(mib: int = 1024, reps: int = 5):
    """Device-to-device copy GB/s (read + write bytes) from torch events: the
    practical HBM rate of a plain streaming kernel on this GPU."""
    import torch

    src = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    dst.copy_(src)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    del src, dst
    t = float(np.median(times))
    return 2.0 * (mib << 20) / (t * 1e-3) / 1e9


def run_cfg3(count: int, forms, max_iter: int = BATCH_MAX_ITER, tol: float = BATCH_TOL, model=None,
             budget: int = 0, tune_cache: str = None, occupation: bool = False):
    """The uneven batch workload at full size: `count` subdomains of the
    256-subdomain draw (start blocks drawn on the device), run with slot
    residency (working sets admitted largest-first within the device memory
    budget, released when a subdomain finishes), until each subdomain's gated
    residual is <= tol or max_iter iterations.  Forms: "fp64" (FP64 filter
    and GEMMs, Lanczos bounds), "mixed" (FP32 filter, split-BF16 GEMMs with
    the FP32 polish, Lanczos bounds) and "mixed_learned" (the same with the
    model's bounds and degree, Lanczos fallback).  subdomains/s counts every
    subdomain; converged ones are reported beside."""
    import torch
    from paper_2609_13115_amd import learned, workloads, xls

    t0 = time.perf_counter()
    _, subs, degs = workloads.batch_subdomains(count=count)
    seeds = [workloads.x0_seed(sd.seed_key) for sd in subs]
    gates = [max(1, int(np.floor(sd.ns / 1.1 + 1e-9))) for sd in subs]
    work = sum(sd.nd * sd.ns * m for sd, m in zip(subs, degs))
    out = {"workload": f"{count} subdomains of the uneven batch draw: grids {min(sd.n[0] for sd in subs)}^3-"
                       f"{max(sd.n[0] for sd in subs)}^3, ns {min(sd.ns for sd in subs)}-"
                       f"{max(sd.ns for sd in subs)}, degree {min(degs)}-{max(degs)}; {work:.3e} pt*vec*deg per "
                       f"iteration over all; FP32 blocks of all of them {2 * 4 * sum(sd.nd * sd.ns for sd in subs) / 1e9:.0f} GB "
                       f"(two per subdomain)",
           "subdomains": count, "setup_s": time.perf_counter() - t0, "gate": tol, "max_iter": max_iter}
    print(f"[bench] cfg3 draw built in {out['setup_s']:.1f} s", file=sys.stderr, flush=True)
    ritz_of = {}
    os.environ.setdefault("XLS_BATCH_PROGRESS", "20")
    for form in forms:
        prec = xls.XLS_PREC_FP64 if form == "fp64" else xls.XLS_PREC_FP32
        gprec = xls.XLS_PREC_FP64 if form == "fp64" else xls.XLS_PREC_BF16X3
        with xls.Batch(subs, filter_prec=prec, x0_seeds=seeds, slots=budget) as b:
            tt = time.perf_counter()
            b.xls_batch_tune(tune_cache)
            t_tune = time.perf_counter() - tt
            torch.cuda.synchronize()
            t = time.perf_counter()
            if form == "mixed_learned":
                F = learned.batch_features(b)
                params = learned.batch_learned_params(model, F, max_iter, tol, gprec)
            else:
                params = [xls.chefsi_params(m, max_iter, xls.XLS_BOUNDS_LANCZOS, resid_tol=tol, gemm_prec=gprec)
                          for m in degs]
            ritz, resid, iters, status = b.xls_batch_chefsi(params)
            torch.cuda.synchronize()
            t = time.perf_counter() - t
            st = b.xls_batch_stats()
            fb = sum(int(b.xls_batch_subdomain(i).xls_subdomain_counters()["fallback"]) for i in range(count))
            happ = sum(b.xls_batch_subdomain(i).xls_subdomain_counters()["h_applies"] for i in range(count))
            occ = occupation_timing(b, subs, prec) if occupation else None
        conv = [int(s_ == xls.XLS_OK and float(np.max(r[:g])) <= tol) for s_, r, g in zip(status, resid, gates)]
        ritz_of[form] = (ritz, conv)
        out[form] = {"seconds": t, "subdomains_per_s": count / t, "converged": int(sum(conv)),
                     "unconverged": count - int(sum(conv)), "converged_per_s": sum(conv) / t,
                     "iterations_total": int(sum(iters)), "iterations_max": int(max(iters)),
                     "h_applies": int(happ), "fallbacks": int(fb), "tune_s": t_tune,
                     "batch_iterations": st["iterations"], "peak_resident_gb": st["peak_bytes"] / 1e9,
                     "max_active": st["max_active"], "device_ms": st["iter_ms"]}
        if occ is not None:
            out[form]["occupation"] = occ
        print(f"[bench] cfg3 {form}: {json.dumps(out[form])}", file=sys.stderr, flush=True)
    ref = ritz_of.get("fp64")
    if ref is not None:
        for form in forms:
            if form == "fp64":
                continue
            rm, cm = ritz_of[form]
            rf, cf = ref
            d = [float(np.max(np.abs(a[:g] - b_[:g]))) for a, b_, g, u, v in zip(rm, rf, gates, cm, cf) if u and v]
            out[form]["max_ritz_diff_ha_both_converged"] = max(d) if d else None
            out[form]["p99_ritz_diff_ha"] = float(np.percentile(d, 99)) if d else None
            out[form]["subdomains_ritz_diff_over_1e-6"] = int(sum(v > 1e-6 for v in d))
            out[form]["both_converged"] = len(d)
            out[form]["speedup_vs_fp64"] = out["fp64"]["seconds"] / out[form]["seconds"]
            out[form]["gate_met"] = bool(d) and max(d) <= 1e-6 and out[form]["converged"] >= out["fp64"]["converged"]
    return out


def occupation_timing(b, subs, prec, sigma: float = 0.01, reps: int = 3):
    """Fermi level of the whole batch at half filling (core-weight pass over
    every block, then the device solve) and a 200-bin density of states:
    best wall time of reps calls each, with the core-weight pass priced at
    its algorithmic bytes (one read of every block)."""
    _, cs = b.xls_batch_density(0.0, sigma)
    ne = float(sum(np.sum(c) for c in cs))  # half of 2 sum c
    best = 1e9
    for _ in range(reps):
        t0 = time.perf_counter()
        mu, n_at, e_band, e_ent, evals = b.xls_batch_fermi(sigma, ne)
        best = min(best, time.perf_counter() - t0)
    lam_lo, lam_hi = mu - 2.0, mu + 2.0
    edges = np.linspace(lam_lo, lam_hi, 201)
    bd = 1e9
    for _ in range(reps):
        t0 = time.perf_counter()
        b.xls_batch_assemble(0, edges)
        bd = min(bd, time.perf_counter() - t0)
    w = 4 if prec == 1 else 8
    nbytes = float(sum(sd.nd * sd.ns * w for sd in subs))
    return {"fermi_ms": best * 1e3, "dos_ms": bd * 1e3, "mu": mu, "n_electrons": ne, "count_at_mu": n_at,
            "evaluations": int(evals), "e_band": e_band, "e_entropy": e_ent,
            "core_weight_bytes": nbytes, "core_weight_gbs_lower_bound": nbytes / best / 1e9}


def cpu_baseline(sd, degree: int, ncols: int):
    from oracle import chefsi, hamiltonian

    op = hamiltonian.from_subdomain(sd)
    X = sd.x0[:, :ncols] if sd.x0 is not None else np.stack([sd.x0_column(c) for c in range(ncols)], 1)
    lo, up = -3.5, 60.0
    t0 = time.perf_counter()
    chefsi.chebyshev_filter(op.apply, X, degree, lo, lo + 0.1 * (up - lo), up)
    t = time.perf_counter() - t0
    return {"value": sd.nd * ncols * degree / t, "unit": "grid-pt*vec*deg/s", "cores": 1,
            "kind": "oracle",
            "sample": f"FP64 oracle Chebyshev filter, degree {degree}, {ncols} of {sd.ns} columns of the "
                      f"same 64^3 box ({t:.1f} s; NumPy elementwise, one thread; host affinity "
                      f"{len(os.sched_getaffinity(0))} cores)"}


T_START = time.perf_counter()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--ns", type=int, default=480)
    ap.add_argument("--degree", type=int, default=24)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-cols", type=int, default=64)
    ap.add_argument("--calib-mib", type=int, default=0,
                    help="first run a device-to-device copy of this many MiB (counter calibration)")
    ap.add_argument("--batch", type=int, default=256,
                    help="subdomains of the uneven batch draw to solve, FP64 and mixed + learned (0: skip)")
    ap.add_argument("--gain", type=int, default=32,
                    help="subdomains for the learned gain at one precision, mixed + Lanczos vs mixed + learned")
    ap.add_argument("--no-gemm-large", action="store_true", help="skip the 96^3, Ns = 2400 GEMM table")
    ap.add_argument("--headline-only", action="store_true", help="only the 64^3 steps (profiling runs)")
    ap.add_argument("--widened-only", action="store_true",
                    help="only the widened rows (warm-start steps, PDOS, Poisson; profiling runs)")
    ap.add_argument("--batch-only", type=int, default=0, metavar="N",
                    help="only the first N subdomains of the uneven batch draw in the mixed form with Lanczos "
                         "bounds (profiling runs)")
    ap.add_argument("--budget-s", type=float, default=720.0,
                    help="skip the optional learned_gain leg once this many seconds have passed")
    ap.add_argument("--write-traffic", nargs=3, metavar=("FORM", "FETCH_CSV", "WRITE_CSV"),
                    help="record filter HBM traffic from two rocprofv3 --pmc passes and exit (no GPU)")
    a = ap.parse_args()
    if a.write_traffic:
        write_traffic(*a.write_traffic)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this engine runs on one GPU; multi-GPU sharding is a design note only "
                                   "(subdomains are independent: one batch per GPU)"}))
        sys.exit(2)
    import torch
    from paper_2609_13115_amd import workloads

    torch.cuda.set_device(0)
    torch.cuda.synchronize()
    if a.batch_only > 0:
        print(json.dumps({"batch": run_cfg3(a.batch_only, ["mixed"]), "wall_s": time.perf_counter() - T_START}),
              flush=True)
        return
    sd = workloads.si_box_64(with_x0=False, ns=a.ns)
    x0 = sd.make_x0(a.ns)
    sd.x0 = x0
    if a.widened_only:
        print(json.dumps({"widened": widened_rows(sd), "wall_s": time.perf_counter() - T_START}), flush=True)
        return
    if a.calib_mib > 0:
        src = torch.empty(a.calib_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {a.calib_mib} MiB", file=sys.stderr, flush=True)
        del src, dst
    copy_gbs = copy_rate()
    torch.cuda.empty_cache()
    print(f"[bench] device copy: {copy_gbs:.1f} GB/s", file=sys.stderr, flush=True)
    res = {}
    for f in ("fp64", "mixed"):
        res[f] = run_form(sd, x0, f, a.steps, a.warmup, a.degree)
        print(f"[bench] {f}: {json.dumps(res[f])}", file=sys.stderr, flush=True)
    r = res["fp64"]
    m = res["mixed"]
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "grid-pt*vec*deg/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"64^3 zero-Dirichlet Si subdomain (64-atom core, 279 projector atoms), "
                               f"ns={a.ns}, degree={a.degree}, one FP64 CheFSI iteration per step "
                               f"(FP64 filter, GEMMs, dense and residual)",
                   "parallelism": "single GPU"},
        "roofline": dict(r["roofline"], copy_gbs=copy_gbs, frac_of_copy=r["roofline"]["achieved"] / copy_gbs),
        "filter_rate": r["filter_rate"],
        "stage_ms_per_step": r["stage_ms_per_step"],
        "gemm": r["gemm"],
        "mixed": {"form": "FP32 filter + split-BF16 GEMMs (FP32 polish) + FP64 dense and residual",
                  "value": m["value"], "ms_per_step": m["ms_per_step"], "filter_rate": m["filter_rate"],
                  "roofline": dict(m["roofline"], frac_of_copy=m["roofline"]["achieved"] / copy_gbs),
                  "stage_ms_per_step": m["stage_ms_per_step"], "gemm": m["gemm"],
                  "half_storage": m["half_storage"]},
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(sd, a.degree, a.cpu_cols)
    if not a.headline_only:
        skipped = []

        def over_budget(leg):
            if time.perf_counter() - T_START > a.budget_s:
                skipped.append(leg)
                print(f"[bench] {leg} skipped: {time.perf_counter() - T_START:.0f} s used of the "
                      f"{a.budget_s:.0f} s budget", file=sys.stderr, flush=True)
                return True
            return False

        out["widened"] = widened_rows(sd)
        if not a.no_gemm_large:
            out["gemm_large"] = gemm_large()
        tune = os.path.join("/tmp", f"xls_tune_{os.getpid()}.json")
        model, info = train_learned()
        if a.batch > 0:
            out["batch"] = run_cfg3(a.batch, ["fp64", "mixed_learned"], model=model, tune_cache=tune,
                                    occupation=True)
            out["batch"]["learned_model"] = info
            b = out["batch"]
            out["subdomains_per_s"] = {"fp64": b["fp64"]["subdomains_per_s"],
                                       "mixed_learned": b["mixed_learned"]["subdomains_per_s"]}
            out["max_ritz_diff_ha"] = b["mixed_learned"].get("max_ritz_diff_ha_both_converged")
            out["gate_met"] = b["mixed_learned"].get("gate_met")
        if a.gain > 0 and not over_budget("learned_gain"):
            out["learned_gain"] = run_cfg3(a.gain, ["mixed", "mixed_learned"], model=model, tune_cache=tune)
        model.close()
        if skipped:
            out["skipped_legs"] = skipped
    out["wall_s"] = time.perf_counter() - T_START
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
