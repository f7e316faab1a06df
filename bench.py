#!/usr/bin/env python3
"""Benchmark of the IPT hot path on one MI355X.

A step is one full-spectrum IPT solve (setup, product-free first sweep, the
Delta x Z sweeps with their fused epilogues, finalize, copy-out) of the dense
n = 4096 problem D = diag(1..n), Delta = eps (R + R^T)/2, R iid N(0, 1/n), seed 0,
with inputs already resident in HBM.  The headline value is eigenpairs/s at
per-column relative step 1e-10 with the BF16 -> FP32 -> FP64 precision ladder
(only FP64 sweeps certify); plain FP64 IPT on the same matrix, and eps = 0.05,
are reported alongside.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "eigenpairs/s at rel. residual 1e-10: mixed-prec/warm-start vs plain FP64"
PEAK = {"fp64": 78.6, "fp32": 157.3, "low": 2500.0}  # TFLOP/s, MI355X dense MFMA
HBM_PEAK = 8000.0  # GB/s
PROFILE = os.path.join(ROOT, "profiles", "gemm_f64_dense_n4096_traffic.txt")
GEMM_SRC = os.path.join(ROOT, "paper_2012_14702_amd", "csrc", "ipt_gemm.hip")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def source_sha():
    return hashlib.sha256(open(GEMM_SRC, "rb").read()).hexdigest()[:16]


def read_traffic():
    """HBM bytes per FP64 sweep-GEMM launch (average over the launches of one plain FP64
    solve) from the committed rocprofv3 --pmc summary, or None when the kernel source
    changed since the counters were taken."""
    if not os.path.exists(PROFILE):
        return None
    vals = {}
    for line in open(PROFILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha") != source_sha():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def solve_many(ipt, handle, theta, delta, zbuf, opts, steps):
    import torch
    infos = []
    if steps <= 0:
        return 0.0, infos, None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = ipt.ipt_solve_dense(theta, delta, opts=opts, handle=handle, colinfo=False, z_out=zbuf)
        infos.append(r.info)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, infos, r


def gemm_stats(infos, n, prec):
    """Algorithmic flops 2 n^2 k_active per product launch of the given precision,
    and the summed device time of those launches (HIP events on the solve stream)."""
    flops, ms, launches = 0.0, 0.0, 0
    for inf in infos:
        for p, act in zip(inf["sweep_prec"], inf["sweep_active"]):
            if p == prec:
                flops += 2.0 * n * n * act
                launches += 1
        ms += inf["prec_ms"][prec]
    return flops, ms, launches


def cpu_baseline(theta, delta, seconds):
    import numpy as np
    import oracle
    threads = oracle.max_threads()
    n = theta.shape[0]
    probe = min(n, 2 * threads)
    t0 = time.perf_counter()
    oracle.ipt_dense(theta, delta, idx=np.arange(probe, dtype=np.int32), tol=1e-10, resid=False)
    per_col = (time.perf_counter() - t0) / probe
    cols = int(max(probe, min(n, seconds / max(per_col, 1e-9))))
    cols = max(threads, cols // threads * threads)
    idx = np.arange(cols, dtype=np.int32)
    t0 = time.perf_counter()
    r = oracle.ipt_dense(theta, delta, idx=idx, tol=1e-10, resid=False)
    dt = time.perf_counter() - t0
    conv = int((r.status == 0).sum())
    return {"value": conv / dt, "unit": "eigenpairs/s", "cores": threads, "kind": "oracle",
            "sample": "columns 0..%d of the same n=%d matrix (independent per-column solves, tol 1e-10, "
                      "plain C FP64, OpenMP over columns); %.1f s" % (cols - 1, n, dt)}


def _timeboxed(unit_fn, budget):
    """Runs unit_fn() (which returns the eigenpairs it converged) until budget seconds
    have passed (at least once); returns (eigenpairs, seconds, units)."""
    done, units = 0, 0
    t0 = time.perf_counter()
    while True:
        done += unit_fn(units)
        units += 1
        dt = time.perf_counter() - t0
        if dt >= budget:
            return done, dt, units


def cpu_baselines(host_dense, seconds):
    """The oracle (plain C FP64 IPT, OpenMP over columns) timed on this host for every
    configuration, on all cores and on one core, each on a bounded sample of the
    configuration's work (eigenpairs/s of the sample; the columns and problems are
    independent, so the rate scales)."""
    import numpy as np
    import oracle
    import workloads
    threads = oracle.max_threads()
    out = {"cores_all": threads, "host_cpus": os.cpu_count()}
    th1, de1 = workloads.dense_sym_gaussian(256, 0.01, 0)
    ths, rps, cols, vals = workloads.sparse_sym_uniform(200000, seed=0)
    idx16 = workloads.lowest_indices(ths, 16)
    ns = workloads.batched_sizes(4096, 32, 512, 0)
    order = np.random.default_rng(7).permutation(4096)
    thf, basef = workloads.family_base(1024, 0)
    idx32 = workloads.lowest_indices(thf, 32)
    eps_te = workloads.family_eps(128, 0.0, 0.08, seed=2)
    budget = max(0.5, seconds / 12.0)

    def dense_cols(th, de, per):
        n = th.shape[0]
        def unit(u):
            lo = (u * per) % n
            ids = np.arange(lo, min(n, lo + per), dtype=np.int32)
            r = oracle.ipt_dense(th, de, idx=ids, tol=1e-10, resid=False)
            return int((r.status == 0).sum())
        return unit

    def c1(u):
        r = oracle.ipt_dense(th1, de1, tol=1e-12, resid=False)
        return int((r.status == 0).sum())

    def c3(u):
        r = oracle.ipt_csr(ths, rps, cols, vals, idx16, tol=1e-10, resid=False)
        return int((r.status == 0).sum())

    def c4(u):
        b = int(order[u % 4096])
        th, de = workloads.batched_problem(b, int(ns[b]), 0.02, 0)
        r = oracle.ipt_dense(th, de, tol=1e-10, max_iter=64, resid=False)
        return int((r.status == 0).sum())

    def c5(u):
        e = float(eps_te[u % 128])
        r = oracle.ipt_dense(thf, e * basef, idx=idx32, tol=1e-10, resid=False)
        return int((r.status == 0).sum())

    th2a, de2a = host_dense[0.01]
    th2b, de2b = host_dense[0.05]
    cases = [("dense n=256 eps=0.01 full spectrum, tol 1e-12", c1, "whole solves"),
             ("dense n=4096 eps=0.01, tol 1e-10", None, "columns in blocks of 2 x cores"),
             ("dense n=4096 eps=0.05, tol 1e-10", None, "columns in blocks of 2 x cores"),
             ("sparse n=200000 k=16 lowest, tol 1e-10", c3, "whole solves"),
             ("batched n~U{32..512}, tol 1e-10, 64 sweeps", c4, "whole problems in a fixed random order"),
             ("learned family n=1024 k=32 cold start, tol 1e-10", c5, "test members in order")]
    res = {}
    for label, fn, sample in cases:
        res[label] = {}
        for cores in (threads, 1):
            oracle.set_threads(cores)
            f = fn
            if f is None:
                th, de = (th2a, de2a) if "0.01" in label else (th2b, de2b)
                f = dense_cols(th, de, 2 * cores)
            got, dt, units = _timeboxed(f, budget if cores > 1 else 2 * budget)
            res[label]["all_cores" if cores > 1 else "one_core"] = {
                "value": round(got / dt, 2), "unit": "eigenpairs/s", "cores": cores,
                "sample": "%d units (%s), %d eigenpairs, %.2f s" % (units, sample, got, dt)}
        log("cpu baseline %s: %s" % (label, {k: v["value"] for k, v in res[label].items()}))
    oracle.set_threads(threads)
    out["configs"] = res
    return out


def dtype_of(sweep_prec, mode):
    """The arithmetic of the headline solve's sweeps, in the order they ran (the
    ladder's rungs follow the steps, so this is read from the solve, not the mode)."""
    names = {"exact-first": "f64 (first sweep, no product)", "low": "bf16",
             "fp32": "f32" if mode == "ladder_fp32_mma" else "fp32-class (3 x fp16 split products)", "fp64": "f64"}
    seq = []
    for p in sweep_prec:
        if not seq or seq[-1] != names[p]:
            seq.append(names[p])
    return " -> ".join(seq) + (" (f64 certifies)" if len(seq) > 1 else "")


def _time(fn, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, r


def bench_sparse(ipt, handle, args):
    """Sparse extremal workload: n = 200000, theta_i = i, about 12 symmetric
    off-diagonal entries per row with values U(-0.05, 0.05), the 16 lowest eigenpairs,
    tol 1e-10; FP64 SpMM sweeps and the FP32-SpMM + FP64-finish ladder.  |M|_1 only
    scales the reported eigen-residual (the stopping test is the relative step), so
    these solves skip it (IPT_FLAG_NO_NORM); "fp64_norm" times the FP64 solve with it."""
    import torch
    import workloads
    n, k = 200000, 16
    th, rp, col, val = workloads.sparse_sym_uniform(n, seed=0)
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(a).to(dev)
    thd, rpd, cold, vald = T(th), T(rp), T(col), T(val)
    idx = T(workloads.lowest_indices(th, k))
    nnz = int(val.shape[0])
    res = {}
    for name, prec, fl in (("fp64", ipt.PREC_FP64, ipt.FLAG_NO_NORM), ("ladder", ipt.PREC_LADDER, ipt.FLAG_NO_NORM),
                           ("fp64_norm", ipt.PREC_FP64, 0)):
        if args.sparse_modes and name not in args.sparse_modes.split(","):
            continue
        o = ipt.default_opts(tol=1e-10, precision=prec, flags=fl)
        run = lambda: ipt.ipt_solve_csr(thd, rpd, cold, vald, idx, opts=o, handle=handle, colinfo=False)
        _time(run, 3)
        sec, r = _time(run, max(5, args.steps))
        # the per-precision kernel times come from one more solve with events around the
        # products (they cost launch gaps, so the timed solves above go without)
        ot = ipt.default_opts(tol=1e-10, precision=prec, flags=ipt.FLAG_TIME_KERNELS | fl)
        inf = ipt.ipt_solve_csr(thd, rpd, cold, vald, idx, opts=ot, handle=handle, colinfo=False).info
        # algorithmic bytes of one FP64 SpMM sweep: the CSR arrays (12 B per entry), the
        # row pointers, one read of Z and one write of W (the gathered rows of Z are
        # meant to be served by the caches); only the product sweeps count (the first
        # sweep of a cold start has no product)
        per = 12.0 * nnz + 4.0 * (n + 1) + 2 * 8.0 * n * k
        ms = inf["prec_ms"].get("fp64", 0.0)
        nl = inf["prec_sweeps"].get("fp64", 0)
        res[name] = {"eigenpairs_per_s": round(int(inf["converged"]) / sec, 1), "ms_per_solve": round(sec * 1e3, 4),
                     "converged": inf["converged"], "sweeps": inf["sweeps"], "sweep_prec": inf["sweep_prec"],
                     "max_resid": inf["max_resid"], "prec_ms": inf["prec_ms"], "prec_sweeps": inf["prec_sweeps"],
                     "spmm_fp64_bytes_per_sweep": per,
                     "spmm_fp64_avg_launch_ms": round(ms / max(nl, 1), 5),
                     "spmm_fp64_GBps": round(per / (ms / max(nl, 1) * 1e-3) / 1e9, 1) if nl else None,
                     "spmm_fp64_frac_of_hbm": round(per / (ms / max(nl, 1) * 1e-3) / 1e9 / HBM_PEAK, 4) if nl else None}
        log("sparse %s: %.3f ms/solve, sweeps %s" % (name, sec * 1e3, inf["sweep_prec"]))
    # the same matrix over C^n: imaginary parts sign(l - j) val / 2 on the off-diagonal
    # entries (a Hermitian perturbation), the complex CSR solve (FP64 sweeps)
    if not args.sparse_modes or "complex" in args.sparse_modes.split(","):
        import numpy as np
        rows = np.repeat(np.arange(n), np.diff(rp))
        valz = val + 0.5j * np.sign(col - rows) * val
        thz, valzd = T(th.astype(np.complex128)), T(valz.astype(np.complex128))
        o = ipt.default_opts(tol=1e-10, precision=ipt.PREC_FP64, flags=ipt.FLAG_NO_NORM)
        run = lambda: ipt.ipt_solve_csr_z(thz, rpd, cold, valzd, idx, opts=o, handle=handle, colinfo=False)
        _time(run, 3)
        sec, r = _time(run, max(5, args.steps))
        inf = r.info
        res["complex_fp64"] = {"eigenpairs_per_s": round(int(inf["converged"]) / sec, 1),
                               "ms_per_solve": round(sec * 1e3, 4), "converged": inf["converged"],
                               "sweeps": inf["sweeps"], "sweep_prec": inf["sweep_prec"]}
        log("sparse complex_fp64: %.3f ms/solve, %d converged, sweeps %s" % (sec * 1e3, int(inf["converged"]),
                                                                             inf["sweep_prec"]))
    return {"workload": "sparse n=200000, ~12 sym off-diagonals/row U(-0.05,0.05), k=16 lowest, tol 1e-10; "
                        "complex_fp64: the same pattern with imaginary parts sign(l - j) val / 2 (Hermitian)",
            "nnz": nnz, "modes": res}


def bench_batched(ipt, handle, args):
    """Batched workload: problems with n ~ U{32..512}, theta sorted U(0, n),
    Delta = 0.02 (R + R^T)/2, R iid N(0, 1/n), full spectra, tol 1e-10, max 64 sweeps;
    FP32 split-form sweeps + FP64 finish vs plain FP64."""
    import numpy as np
    import torch
    import workloads
    B = args.batch
    t0 = time.perf_counter()
    ns, th, de, th_off, de_off = workloads.batched_sym_gaussian(B, 32, 512, 0.02, seed=0)
    log("batched inputs generated in %.1f s (%d problems, %.2f GB)" % (time.perf_counter() - t0, B, de.nbytes / 1e9))
    dev = torch.device("cuda:0")
    thd = torch.from_numpy(th).to(dev)
    ded = torch.from_numpy(de).to(dev)
    del de
    t0 = time.perf_counter()
    tiles = ipt.ipt_batched_tune(ns, thd, ded, th_off, de_off, handle=handle)
    t_tune = time.perf_counter() - t0
    buckets = sorted(set(int(x) for x in (ns - 1) // 64))
    log("batched tile table (tuned in %.2f s): %s" % (t_tune, {64 * (q + 1): tiles[q] for q in buckets}))
    z_out = torch.empty_like(ded)
    lam_out = torch.empty_like(thd)
    st_out = torch.empty(thd.shape[0], dtype=torch.int32, device=dev)
    res = {}
    modes = (("ladder", ipt.PREC_LADDER, 0), ("ladder_no_graph", ipt.PREC_LADDER, ipt.FLAG_NO_GRAPH),
             ("fp64", ipt.PREC_FP64, 0), ("acx", ipt.PREC_FP64, ipt.FLAG_ACX),
             ("ladder_choose_d", ipt.PREC_LADDER, ipt.FLAG_CHOOSE_D),
             ("acx_choose_d", ipt.PREC_FP64, ipt.FLAG_ACX | ipt.FLAG_CHOOSE_D))
    for name, prec, flags in modes:
        if args.batched_modes and name not in args.batched_modes.split(","):
            continue
        o = ipt.default_opts(tol=1e-10, precision=prec, max_iter=64, flags=flags)
        run = lambda: ipt.ipt_solve_batched(ns, thd, ded, th_off, de_off, opts=o, handle=handle, z_out=z_out,
                                            lam_out=lam_out, status_out=st_out)
        _time(run, 1)
        sec, r = _time(run, 3)
        inf = r.info
        res[name] = {"eigenpairs_per_s": round(int(inf["converged"]) / sec, 1), "ms_per_solve": round(sec * 1e3, 3),
                     "device_ms": round(inf["time_ms"], 3),
                     "converged": inf["converged"], "not_converged": inf["not_converged"],
                     "diverged": inf["diverged"], "sweeps": inf["sweeps"],
                     "sweep_equivalents": round(inf["matvecs"] / float(ns.sum()), 3),
                     "converged_fraction": round(inf["converged"] / float(ns.sum()), 5)}
        log("batched %s: %.2f ms/solve, %d/%d converged, %d sweeps, %.2f sweep-equivalents" % (
            name, sec * 1e3, inf["converged"], int(ns.sum()), inf["sweeps"], inf["matvecs"] / float(ns.sum())))
        del r
    # Roofline of the batched GEMM on a full sweep: sweep 2 (every column still active
    # after the product-free first sweep) timed on its own (host-launched sweeps with
    # events around the GEMM launches); algorithmic flops sum_b 2 n_b^3, algorithmic
    # bytes per entry of Delta_b: the Delta shadow and the Z operand (4 + 4 B for FP32
    # tiles, 8 + 8 for FP64), the epilogue's read of Z and write of W (8 + 8 B) and, for
    # FP32 tiles, the FP32 shadow of W - E (4 B).
    n3 = float((ns.astype(np.float64) ** 3).sum())
    n2 = float((ns.astype(np.float64) ** 2).sum())
    roof = {}
    for name, prec, peak, bpe in (("ladder", ipt.PREC_LADDER, PEAK["fp32"], 28.0),
                                  ("fp64", ipt.PREC_FP64, PEAK["fp64"], 32.0)):
        if args.batched_modes and name not in args.batched_modes.split(","):
            continue
        o = ipt.default_opts(tol=1e-10, precision=prec, max_iter=64, flags=ipt.FLAG_TIME_KERNELS)
        run = lambda: ipt.ipt_solve_batched(ns, thd, ded, th_off, de_off, opts=o, handle=handle, z_out=z_out,
                                            lam_out=lam_out, status_out=st_out)
        _time(run, 1)
        _, r = _time(run, 1)
        inf = r.info
        t2 = inf["sweep_ms"][1]
        frac_active = inf["sweep_active"][1] / float(ns.sum())
        gemm_ms = sum(inf["sweep_ms"][1:])
        # the columns the first sweep certified (few) are taken as spread like the rest
        tf = 2.0 * n3 * frac_active / (t2 * 1e-3) / 1e12
        roof[name] = {"bound": "mfma", "unit": "TFLOP/s", "peak": peak, "sweep2_ms": round(t2, 4),
                      "sweep2_active_fraction": round(frac_active, 6), "achieved": round(tf, 2),
                      "frac": round(tf / peak, 4),
                      "flops_per_full_sweep": 2.0 * n3,
                      "bytes_per_full_sweep": bpe * n2,
                      "GBps": round(bpe * n2 * frac_active / (t2 * 1e-3) / 1e9, 1),
                      "frac_of_hbm": round(bpe * n2 * frac_active / (t2 * 1e-3) / 1e9 / HBM_PEAK, 4),
                      "sweep_ms": [round(x, 4) for x in inf["sweep_ms"]],
                      "sweep_active": inf["sweep_active"],
                      "gemm_ms_all_sweeps": round(gemm_ms, 3), "solve_ms_timed_kernels": round(inf["time_ms"], 3),
                      "sweeps": inf["sweeps"]}
        log("batched roofline %s: sweep 2 %.3f ms, %.1f TFLOP/s (%.1f%% of peak), %.0f GB/s" % (
            name, t2, tf, 100 * tf / peak, bpe * n2 / (t2 * 1e-3) / 1e9))
        del r
    tiles_used = {"bucket_upper_n": [64 * (q + 1) for q in buckets], "tile": [tiles[q] for q in buckets],
                  "tune_s": round(t_tune, 3)}
    return {"workload": "batched %d problems n~U{32..512}, theta=sort(U(0,n)), Delta=0.02*sym N(0,1/n), "
                        "full spectra, tol 1e-10, max 64 sweeps" % B, "eigenpairs": int(ns.sum()), "modes": res,
            "roofline": roof, "tiles": tiles_used}


def bench_morgan(ipt, handle, args):
    """Morgan's tridiagonal matrix (n = 5000, theta_i = i, off-diagonals 0.5; Sec. 6.1),
    the k lowest eigenpairs for k = 1 and 50, tol 1e-12: plain IPT vs IPT-ACX on the
    sparse path (FP64 SpMM sweeps)."""
    import numpy as np
    import torch
    import workloads
    dev = torch.device("cuda:0")
    th, rp, col, val = workloads.morgan_tridiagonal(5000, 0.5)
    tt = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    thd, rpd, cold, vald = tt(th), tt(rp), tt(col), tt(val)
    res = {}
    for k in (1, 50):
        idx = tt(np.arange(k, dtype=np.int32))
        for name, flags in (("plain", 0), ("acx", ipt.FLAG_ACX)):
            o = ipt.default_opts(tol=1e-12, precision=ipt.PREC_FP64, max_iter=2000, flags=flags)
            run = lambda: ipt.ipt_solve_csr(thd, rpd, cold, vald, idx, opts=o, handle=handle)
            _time(run, 1)
            sec, r = _time(run, 5)
            inf = r.info
            res["k%d_%s" % (k, name)] = {"ms_per_solve": round(sec * 1e3, 3), "converged": inf["converged"],
                                         "sweeps": inf["sweeps"], "matvecs": inf["matvecs"],
                                         "eigenpairs_per_s": round(inf["converged"] / sec, 1)}
            log("morgan k=%d %s: %.3f ms/solve, %d/%d converged, %d sweeps, %d matvecs" % (
                k, name, sec * 1e3, inf["converged"], k, inf["sweeps"], inf["matvecs"]))
    return {"workload": "Morgan tridiagonal n=5000, off-diagonal 0.5, k lowest, tol 1e-12", "modes": res}


def bench_nonsym(ipt, handle, args):
    """The paper's dense test family (Sec. 6.2): D = diag(1..n), Delta = eps R with R iid
    U[0,1] (non-centred, non-symmetric), eps = 0.01, full spectrum, tol 1e-10; plain FP64
    and the ladder (the epilogue's next d reads Delta_ij itself, the matrix not being
    symmetric)."""
    import numpy as np
    import torch
    import workloads
    dev = torch.device("cuda:0")
    n = args.nonsym_n
    t0 = time.perf_counter()
    th, de = workloads.dense_uniform_nonsym(n, 0.01, 0)
    thd, ded = torch.from_numpy(th).to(dev), torch.from_numpy(de).to(dev)
    del de
    log("nonsym n=%d inputs in %.1f s" % (n, time.perf_counter() - t0))
    zbuf = torch.empty((n, n), dtype=torch.float64, device=dev)
    res = {}
    for name, prec in (("fp64", ipt.PREC_FP64), ("ladder", ipt.PREC_LADDER)):
        o = ipt.default_opts(tol=1e-10, precision=prec, flags=ipt.FLAG_TIME_KERNELS)
        sec, infos, r = solve_many(ipt, handle, thd, ded, zbuf, o, 1)
        sec, infos, r = solve_many(ipt, handle, thd, ded, zbuf, o, 2)
        inf = infos[-1]
        fl, ms, la = gemm_stats(infos, n, "fp64")
        res[name] = {"ms_per_solve": round(sec * 1e3, 3), "eigenpairs_per_s": round(inf["converged"] / sec, 1),
                     "converged": inf["converged"], "sweeps": inf["sweeps"], "sweep_prec": inf["sweep_prec"],
                     "sweep_active": inf["sweep_active"], "max_resid": inf["max_resid"],
                     "fp64_gemm_tflops": round(fl / (ms * 1e-3) / 1e12, 2) if ms > 0 else None,
                     "fp64_gemm_frac_of_peak": round(fl / (ms * 1e-3) / 1e12 / PEAK["fp64"], 4) if ms > 0 else None}
        log("nonsym n=%d %s: %.2f ms/solve, %d converged, sweeps %s" % (n, name, sec * 1e3, inf["converged"],
                                                                        inf["sweep_prec"]))
        del r
    res["ladder_speedup_vs_fp64"] = round(res["fp64"]["ms_per_solve"] / res["ladder"]["ms_per_solve"], 3)
    return {"workload": "paper's dense family diag(1..n) + 0.01 U[0,1] (non-symmetric), n=%d, full spectrum, "
                        "tol 1e-10" % n, "modes": res}


def bench_morgan_sweep(ipt, handle, args):
    """Morgan's tridiagonal matrix (n = 5000, theta_i = i) with off-diagonal eps over a
    grid (the failure study of Sec. 6.1): status, sweeps and matvecs of the ground state
    (k = 1) and of the 50 lowest eigenpairs, plain IPT against IPT-ACX, tol 1e-12,
    at most 2000 applications of F."""
    import numpy as np
    import torch
    import workloads
    dev = torch.device("cuda:0")
    tt = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    grid = [0.1, 0.3, 0.5, 0.6, 0.7, 0.75, 1.0, 1.5, 2.0]
    res = {}
    for off in grid:
        th, rp, col, val = workloads.morgan_tridiagonal(5000, off)
        thd, rpd, cold, vald = tt(th), tt(rp), tt(col), tt(val)
        row = {}
        for k in (1, 50):
            idx = tt(np.arange(k, dtype=np.int32))
            for name, flags in (("plain", 0), ("acx", ipt.FLAG_ACX)):
                o = ipt.default_opts(tol=1e-12, precision=ipt.PREC_FP64, max_iter=2000, flags=flags | ipt.FLAG_NO_NORM)
                t0 = time.perf_counter()
                r = ipt.ipt_solve_csr(thd, rpd, cold, vald, idx, opts=o, handle=handle, colinfo=False)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                inf = r.info
                row["k%d_%s" % (k, name)] = {"converged": inf["converged"], "diverged": inf["diverged"],
                                              "not_converged": inf["not_converged"], "sweeps": inf["sweeps"],
                                              "matvecs": inf["matvecs"], "ms": round(dt * 1e3, 3)}
        res["%g" % off] = row
        log("morgan off-diagonal %g: k=1 plain %s/%d sweeps, acx %s/%d; k=50 plain %d conv, acx %d conv" % (
            off, row["k1_plain"]["converged"], row["k1_plain"]["sweeps"], row["k1_acx"]["converged"],
            row["k1_acx"]["sweeps"], row["k50_plain"]["converged"], row["k50_acx"]["converged"]))
    return {"workload": "Morgan tridiagonal n=5000, theta_i=i, off-diagonal eps, k=1 and 50 lowest, tol 1e-12, "
                        "at most 2000 applications of F", "by_offdiagonal": res}


def bench_continuation(ipt, handle, args):
    """Non-autonomous continuation (opts.cont_alpha; the concluding discussion of the
    3 x 3 example) and the homotopy restart (opts.homotopy_q, concluding section): the
    paper's 3 x 3 matrix D = diag(0, 1, 3) + eps P over a grid of real eps, columns
    converged by plain IPT, by the continuation (alpha = 1/2) and by a 2-stage restart
    (tol 1e-12); and their cost on the dense n = 4096 workload against plain FP64."""
    import numpy as np
    import torch
    import workloads
    dev = torch.device("cuda:0")
    tt = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    step = args.cont_grid_step
    grid = [] if step <= 0 else [e for e in np.round(np.arange(-0.6, 0.6 + step / 2, step), 6) if e != 0.0]
    conv = {"plain": [0, 0, 0], "continuation": [0, 0, 0], "homotopy_q2": [0, 0, 0]}
    rescued, rescued_h = [], []
    t0 = time.perf_counter()
    for eps in grid:
        th, de = workloads.three_by_three(float(eps))
        st = {}
        for name, alpha, q in (("plain", 0.0, 0), ("continuation", 0.5, 0), ("homotopy_q2", 0.0, 2)):
            r = ipt.ipt_solve_dense(tt(th), tt(de), handle=handle, tol=1e-12, max_iter=1000, cont_alpha=alpha,
                                    homotopy_q=q)
            st[name] = r.status.cpu().numpy()
            for c in range(3):
                conv[name][c] += int(st[name][c] == ipt.CONVERGED)
        rescued += ["eps=%g col %d" % (eps, c + 1) for c in range(3)
                    if st["continuation"][c] == ipt.CONVERGED and st["plain"][c] != ipt.CONVERGED]
        rescued_h += ["eps=%g col %d" % (eps, c + 1) for c in range(3)
                      if st["homotopy_q2"][c] == ipt.CONVERGED and st["plain"][c] != ipt.CONVERGED]
    t_grid = time.perf_counter() - t0
    log("continuation 3x3 grid (%d eps): converged plain %s, continuation %s, homotopy (2 stages) %s; "
        "rescued by the continuation: %s; by the homotopy: %s" % (
            len(grid), conv["plain"], conv["continuation"], conv["homotopy_q2"], rescued, rescued_h))
    th, de = workloads.dense_sym_gaussian(args.n, args.eps, 0)
    thd, ded = tt(th), tt(de)
    dense = {}
    for name, alpha, q in (("fp64", 0.0, 0), ("continuation", 0.5, 0), ("homotopy_q2", 0.0, 2)):
        o = ipt.default_opts(tol=1e-10, precision=ipt.PREC_FP64, max_iter=200, cont_alpha=alpha, homotopy_q=q)
        run = lambda: ipt.ipt_solve_dense(thd, ded, opts=o, handle=handle, colinfo=False)
        _time(run, 1)
        sec, r = _time(run, 2)
        inf = r.info
        dense[name] = {"ms_per_solve": round(sec * 1e3, 3), "sweeps": inf["sweeps"], "converged": inf["converged"],
                       "eigenpairs_per_s": round(inf["converged"] / sec, 1)}
        log("continuation dense n=%d eps=%g %s: %.2f ms/solve, %d sweeps, %d converged" % (
            args.n, args.eps, name, sec * 1e3, inf["sweeps"], inf["converged"]))
        del r
    return {"workload": "3x3 D=diag(0,1,3)+eps*[[0,1,2],[1,0,3],[2,3,0]], %d real eps in [-0.6, 0.6] (step %g), "
                        "tol 1e-12, max 1000 sweeps, alpha=0.5; dense n=%d eps=%g full spectrum, tol 1e-10" % (
                            len(grid), step, args.n, args.eps),
            "grid_converged_per_column": conv, "rescued": rescued, "rescued_homotopy_q2": rescued_h,
            "grid_seconds": round(t_grid, 3),
            "dense": dense}


def bench_complex(ipt, handle, args):
    """Dense IPT over C^n (ipt_solve_dense_z): M = diag(1..n) + Delta, Delta = eps (A + A^H)/2
    with A iid complex Gaussian (variance 1/n), full spectrum, tol 1e-10, FP64 sweeps
    (four real matrix-core products per complex product)."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    n = args.complex_n
    rng = np.random.default_rng(0)
    a = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    de = torch.from_numpy(args.eps * (a + a.conj().T) / 2).to(dev)
    del a
    th = torch.from_numpy(np.arange(1, n + 1).astype(np.complex128)).to(dev)
    o = ipt.default_opts(tol=1e-10, precision=ipt.PREC_FP64, flags=ipt.FLAG_TIME_KERNELS)
    run = lambda: ipt.ipt_solve_dense_z(th, de, opts=o, handle=handle, colinfo=False)
    _time(run, 1)
    sec, r = _time(run, 3)
    inf = r.info
    ms = inf["prec_ms"]["fp64"]
    act = inf["sweep_active"]
    # four real products of 2 n^2 per active column, in the product sweeps (the first
    # sweep of the cold start has none)
    flops = sum(8.0 * n * n * a_ for a_, p_ in zip(act, inf["sweep_prec"]) if p_ == "fp64")
    tf = flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    log("complex n=%d: %.2f ms/solve, %d sweeps, %d converged, product %.1f TFLOP/s" % (
        n, sec * 1e3, inf["sweeps"], inf["converged"], tf))
    return {"workload": "complex Hermitian n=%d, theta=1..n, Delta=eps*(A+A^H)/2, A iid CN(0,1/n) seed 0, eps=%g, "
                        "full spectrum, tol 1e-10, FP64 sweeps" % (n, args.eps),
            "ms_per_solve": round(sec * 1e3, 3), "eigenpairs_per_s": round(inf["converged"] / sec, 1),
            "converged": inf["converged"], "sweeps": inf["sweeps"], "sweep_active": act,
            "product_ms": round(ms, 3), "product_tflops": round(tf, 2),
            "product_frac_of_fp64_peak": round(tf / PEAK["fp64"], 4)}


def bench_learned(ipt, handle, args):
    """Learned warm start: M(eps) = diag(1..1024) + eps R, R = (R'+R'^T)/2, R' iid N(0,1/n)
    seed 0, k = 32 lowest; the network is trained on 512 eps ~ U[0, 0.08] (seed 1) and
    tested on 128 new eps (seed 2).  Starts compared (FP64 sweeps, tol 1e-10; the cost
    of a start is included in its eigenpairs/s): cold (Z0 = I, whose first sweep is the
    free first-order start F(I)); the family's Rayleigh-Schroedinger partial sums of
    orders 2, 3 and 4 (terms computed once per family); the MLP on top of the series of
    the configured order; linear interpolation between the two neighbouring training
    solutions.  Every warm answer is compared with the cold one."""
    import numpy as np
    import torch
    import workloads
    from paper_2012_14702_amd import warmstart
    n, k = 1024, 32
    th, base = workloads.family_base(n, 0)
    dev = torch.device("cuda:0")
    thd, based = torch.from_numpy(th).to(dev), torch.from_numpy(base).to(dev)
    idx = torch.from_numpy(workloads.lowest_indices(th, k)).to(dev)
    eps_tr = workloads.family_eps(512, 0.0, 0.08, seed=1)
    eps_te = workloads.family_eps(128, 0.0, 0.08, seed=2)
    ztr, _, _, _, t_train_solves = warmstart.solve_family(thd, based, eps_tr, idx, handle=handle, tol=1e-12)
    ws = warmstart.WarmStarter(n, k, hidden=256, depth=2, seed=0, handle=handle, order=args.learned_order)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    terms4 = ipt.ipt_rs_terms(thd, based, idx, 4, handle=handle)
    torch.cuda.synchronize()
    t_terms = time.perf_counter() - t0
    ws.terms = terms4[:args.learned_order].contiguous() if args.learned_order > 0 else None
    loss, t_fit = ws.fit(ztr, eps_tr, idx, steps=args.train_steps, lr=1e-3)
    log("learned: trained %d steps in %.3f s (%.1f us/step), loss %.3g" % (
        args.train_steps, t_fit, t_fit / max(args.train_steps, 1) * 1e6, loss))
    res = {}
    zc, lc, sc, swc, t_cold = warmstart.solve_family(thd, based, eps_te, idx, handle=handle, tol=1e-10)
    res["cold"] = (sc, swc, t_cold, 0.0)
    for p_ in (2, 3, 4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        z0 = warmstart.series_start(terms4[:p_].contiguous(), eps_te, idx, handle=handle)
        torch.cuda.synchronize()
        t_start = time.perf_counter() - t0
        _, _, ss, sws, t_s = warmstart.solve_family(thd, based, eps_te, idx, z0=z0, handle=handle, tol=1e-10)
        res["series%d" % p_] = (ss, sws, t_s, t_start)
    # learned: inference for all 128 eps (features and parameters already on the
    # device), then the warm-started solves
    xin, ein = ws.inputs(eps_te)
    z0 = ws.predict_from(xin, ein, idx)  # warm-up of the inference path
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ws.predict_from(xin, ein, idx, z0=z0)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    # device span: a spin kernel queued first keeps the stream busy while the host
    # marshals the call and launches its kernels, so the start event falls just before
    # the first of them; the end event follows the call's own synchronisation
    spans = []
    for _ in range(10):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda._sleep(200000)
        ev0.record()
        ws.predict_from(xin, ein, idx, z0=z0)
        ev1.record()
        torch.cuda.synchronize()
        spans.append(ev0.elapsed_time(ev1) * 1e-3)
    t_inf_dev = float(np.median(spans))
    zw, lw, sw, sww, t_warm = warmstart.solve_family(thd, based, eps_te, idx, z0=z0, handle=handle, tol=1e-10)
    res["mlp"] = (sw, sww, t_warm, t_inf)
    # control: linear interpolation between neighbouring training solutions
    order = np.argsort(eps_tr)
    es = eps_tr[order]
    zs = ztr[torch.from_numpy(order).to(dev)]
    zi = torch.empty_like(z0)
    for p_, e in enumerate(eps_te):
        q = int(np.clip(np.searchsorted(es, e), 1, len(es) - 1))
        w = (e - es[q - 1]) / (es[q] - es[q - 1])
        zi[p_] = (1 - w) * zs[q - 1] + w * zs[q]
    _, _, si, swi, t_interp = warmstart.solve_family(thd, based, eps_te, idx, z0=zi, handle=handle, tol=1e-10)
    res["interp_control"] = (si, swi, t_interp, 0.0)
    za, zb = zw.cpu().numpy(), zc.cpu().numpy()
    an = za / np.linalg.norm(za, axis=1, keepdims=True)
    bn = zb / np.linalg.norm(zb, axis=1, keepdims=True)
    max_angle = float(np.max(2 * np.arcsin(np.minimum(1.0, np.linalg.norm(an - bn, axis=1) / 2))))
    max_dlam = float((lw - lc).abs().max())
    # MLP kernels: training-step flops (forward, input and weight gradients of every
    # layer) and the inference flops, against the BF16 dense peak
    h = 256
    mac = 2 * h + h * h + h * n * k
    step_flops = 3 * 2.0 * 512 * mac - 2.0 * 512 * 2 * h  # the first layer has no input gradient
    step_s = t_fit / max(args.train_steps, 1)
    inf_flops = 2.0 * 128 * mac
    roof = {"bound": "mfma", "unit": "TFLOP/s", "peak": PEAK["low"],
            "train_step_us": round(step_s * 1e6, 2), "train_step_flops": step_flops,
            "train_achieved": round(step_flops / step_s / 1e12, 2),
            "train_frac": round(step_flops / step_s / 1e12 / PEAK["low"], 4),
            "inference_us_for_128": round(t_inf * 1e6, 2), "inference_device_us_for_128": round(t_inf_dev * 1e6, 2),
            "inference_flops": inf_flops, "inference_achieved": round(inf_flops / t_inf_dev / 1e12, 2),
            "note": "a training step is one graph replay, host-clocked over the run; inference: median over 10 calls "
                    "of the stream's events, from just before the first kernel (a spin kernel queued first hides the "
                    "call's launches) to the end of its synchronisation; the host-clocked figure is one whole call"}
    log("learned: mean sweeps " + ", ".join("%s %.3f" % (nm, v[1].mean()) for nm, v in res.items()))
    total = 128 * k
    return {"workload": "family diag(1..1024)+eps*R, k=32 lowest, train 512 eps~U[0,0.08], test 128 new eps, "
                        "FP64 sweeps, tol 1e-10",
            "network": "2 -> 256 -> 256 -> 32768 tanh MLP on the remainder after the order-%d series, BF16 GEMM "
                       "operands / FP32 accumulation, Adam, %d steps" % (args.learned_order, args.train_steps),
            "train_loss": loss, "train_seconds": round(t_fit, 4), "train_solves_seconds": round(t_train_solves, 3),
            "series_terms_seconds": round(t_terms, 4),
            "mean_sweeps": {nm: float(v[1].mean()) for nm, v in res.items()},
            "eigenpairs_per_s": {nm: round(int((v[0] == 0).sum()) / (v[2] + v[3]), 1) for nm, v in res.items()},
            "converged": {nm: int((v[0] == 0).sum()) for nm, v in res.items()}, "of": total,
            "start_seconds": {nm: round(v[3], 6) for nm, v in res.items()},
            "mlp_inference_ms_for_128": round(t_inf * 1e3, 4),
            "roofline": roof,
            "warm_vs_cold": {"max_angle": max_angle, "max_abs_dlambda": max_dlam}}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--eps", type=float, default=0.01)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["all", "ladder", "ladder_fp32_mma", "fp64"], default="all",
                    help="restrict the dense workload to one mode (for profiler runs)")
    ap.add_argument("--extra", default="sparse,morgan,batched,learned,nonsym,morgan_sweep,continuation,complex",
                    help="comma list of secondary workloads to time: sparse, morgan, batched, learned, nonsym, "
                         "morgan_sweep, continuation, complex ('' for none)")
    ap.add_argument("--nonsym-n", type=int, default=16384, help="size of the paper's non-symmetric dense family")
    ap.add_argument("--complex-n", type=int, default=4096, help="size of the complex workload")
    ap.add_argument("--train-steps", type=int, default=3000, help="Adam steps of the warm-start network")
    ap.add_argument("--learned-order", type=int, default=2,
                    help="order of the series partial sum the warm-start network corrects")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense workload (profiling of the others)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (to scale HBM counters) and exit")
    ap.add_argument("--batch", type=int, default=4096, help="problems in the batched workload")
    ap.add_argument("--batched-modes", default="", help="comma list of batched modes to time (default: all)")
    ap.add_argument("--sparse-modes", default="", help="comma list of sparse modes to time: fp64, ladder (default: all)")
    ap.add_argument("--cont-grid-step", type=float, default=0.0025,
                    help="eps step of the 3x3 continuation grid (0: skip the grid)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the IPT solve here runs on a single MI355X and no multi-GPU "
              "path is built (requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_2012_14702_amd import ipt

    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8}))
        return

    ipt.load_library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.n
    handle = ipt.Handle()
    if args.no_dense:
        extras = [e for e in args.extra.split(",") if e]
        out = {}
        for name, fn in (("sparse", bench_sparse), ("morgan", bench_morgan), ("batched", bench_batched),
                         ("learned", bench_learned), ("nonsym", bench_nonsym), ("morgan_sweep", bench_morgan_sweep),
                         ("continuation", bench_continuation), ("complex", bench_complex)):
            if name in extras:
                out[name] = fn(ipt, handle, args)
        print(json.dumps(out), flush=True)
        return

    def prep(eps):
        th, de = workloads.dense_sym_gaussian(n, eps, 0)
        return th, de, torch.from_numpy(th).to(dev), torch.from_numpy(de).to(dev)

    zbuf = torch.empty((n, n), dtype=torch.float64, device=dev)
    # "ladder": BF16 -> FP32-class rung as three FP16 products (the default) -> FP64;
    # "ladder_fp32_mma": the same ladder with the FP32 rung on FP32 matrix cores
    modes = {"ladder": dict(precision=ipt.PREC_LADDER, low_type=ipt.LOW_BF16),
             "ladder_fp32_mma": dict(precision=ipt.PREC_LADDER, low_type=ipt.LOW_BF16, flags=ipt.FLAG_MID_FP32),
             "fp64": dict(precision=ipt.PREC_FP64)}
    if args.only != "all":
        modes = {args.only: modes[args.only]}
    results = {}
    host = {}
    for eps in ([args.eps, 0.05] if args.only == "all" and args.eps != 0.05 else [args.eps]):
        th, de, thd, ded = prep(eps)
        host[eps] = (th, de)
        for name, kw in modes.items():
            kw2 = dict(kw)
            fl = kw2.pop("flags", 0)
            o = ipt.default_opts(tol=1e-10, flags=fl, **kw2)
            log("eps=%g mode=%s warmup %d" % (eps, name, args.warmup))
            solve_many(ipt, handle, thd, ded, zbuf, o, args.warmup)
            steps = args.steps if eps == args.eps else max(3, args.steps // 4)
            log("eps=%g mode=%s timing %d steps" % (eps, name, steps))
            sec, infos_t, last = solve_many(ipt, handle, thd, ded, zbuf, o, steps)
            # per-kernel times: the same solves again with HIP events around each sweep's
            # product (the events cost launch gaps, so the solves timed above go without)
            ot = ipt.default_opts(tol=1e-10, flags=ipt.FLAG_TIME_KERNELS | fl, **kw2)
            sec_ev, infos, _ = solve_many(ipt, handle, thd, ded, zbuf, ot, steps)
            conv = int(last.info["converged"])
            results[(eps, name)] = {"sec": sec, "sec_events": sec_ev, "infos": infos, "conv": conv,
                                    "eigenpairs_per_s": conv / sec,
                                    "device_ms": float(np.mean([i["time_ms"] for i in infos_t])),
                                    "sweeps": infos[-1]["sweeps"], "sweep_prec": infos[-1]["sweep_prec"],
                                    "sweep_active": infos[-1]["sweep_active"],
                                    "sweep_max_step": [float("%.3g" % s) for s in infos[-1]["sweep_max_step"]],
                                    "max_resid": max(float(i["max_resid"]) for i in infos)}
            log("eps=%g mode=%s: %.3f ms/solve, %d converged, sweeps %s" % (
                eps, name, sec * 1e3, conv, infos[-1]["sweep_prec"]))
        del thd, ded

    head_mode = "ladder" if "ladder" in modes else ("ladder_fp32_mma" if "ladder_fp32_mma" in modes else "fp64")
    head = results[(args.eps, head_mode)]
    # Roofline of the dominant kernel, the sweep GEMM in its FP64 body.  One kernel
    # (k_sweep_gemm) serves every precision, so it is measured in the plain FP64 run,
    # where every dispatch of it is an FP64 sweep (the profiler's average over that
    # run's dispatches is then the same quantity).
    roof_src = results[(args.eps, "fp64")] if "fp64" in modes else head
    f64_flops, f64_ms, f64_launches = gemm_stats(roof_src["infos"], n, "fp64")
    achieved = f64_flops / (f64_ms * 1e-3) / 1e12 if f64_ms > 0 else 0.0
    traffic = read_traffic()
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK["fp64"], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK["fp64"], 4), "traffic": traffic,
                "kernel": "k_sweep_gemm, FP64 body (v_mfma_f64_16x16x4f64 + fused IPT epilogue)",
                "measured_in": "plain FP64 solves, eps=%g" % args.eps if "fp64" in modes else "ladder solves",
                "launches": f64_launches, "avg_launch_ms": round(f64_ms / max(f64_launches, 1), 4),
                "flops_per_launch": f64_flops / max(f64_launches, 1),
                "flops_per_unit": "2 n^2 per active column (n = 4096)"}
    per_prec = {}
    for prec in ("low", "fp32", "fp64", "exact-first"):
        fl, ms, la = gemm_stats(head["infos"], n, prec)
        if la:
            entry = {"launches": la, "avg_launch_ms": round(ms / la, 4)}
            if prec in PEAK:
                entry["tflops"] = round(fl / (ms * 1e-3) / 1e12, 2)
                entry["frac_of_peak"] = round(fl / (ms * 1e-3) / 1e12 / PEAK[prec], 4)
            if prec == "fp32" and head_mode == "ladder":
                # the dense FP32-class rung runs three FP16 matrix-core products per product:
                # priced against the FP16 peak at three products' flops
                entry["arithmetic"] = "3 x FP16 (hi/lo split), FP32 accumulation"
                entry["frac_of_peak"] = round(3 * fl / (ms * 1e-3) / 1e12 / PEAK["low"], 4)
                entry["peak_basis"] = "FP16 dense MFMA 2500 TFLOP/s, 3 products"
            per_prec[prec] = entry

    out = {
        "metric": METRIC,
        "value": round(head["eigenpairs_per_s"], 1),
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["sec"] * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_of(head["sweep_prec"], head_mode),
        "data": "synthetic",
        "config": {"workload": "dense full spectrum n=%d, D=diag(1..n), Delta=eps*(R+R^T)/2, R iid N(0,1/n) "
                               "seed 0, eps=%g, k=n, tol 1e-10 (per-column relative step)" % (n, args.eps),
                   "mode": head_mode, "global_batch": 1, "parallelism": "none (1 GPU)"},
        "roofline": roofline,
        "kernels": per_prec,
        "solve": {"%s eps=%g" % (m, e): {"eigenpairs_per_s": round(v["eigenpairs_per_s"], 1),
                                         "ms_per_solve": round(v["sec"] * 1e3, 4), "device_ms": round(v["device_ms"], 4),
                                         "ms_per_solve_with_kernel_events": round(v["sec_events"] * 1e3, 4),
                                         "converged": v["conv"], "sweeps": v["sweeps"], "sweep_prec": v["sweep_prec"],
                                         "sweep_active": v["sweep_active"],
                                         "sweep_max_step": v["sweep_max_step"],
                                         "max_resid": v["max_resid"],
                                         "max_resid_within_1e-10": v["max_resid"] <= 1e-10}
                  for (e, m), v in results.items()},
    }
    if ("fp64" in modes) and ("ladder" in modes):
        out["ladder_speedup_vs_fp64"] = round(results[(args.eps, "fp64")]["sec"] / results[(args.eps, "ladder")]["sec"], 3)
    if ("fp64" in modes) and ("ladder_fp32_mma" in modes):
        out["ladder_fp32_mma_speedup_vs_fp64"] = round(
            results[(args.eps, "fp64")]["sec"] / results[(args.eps, "ladder_fp32_mma")]["sec"], 3)
    extras = [e for e in args.extra.split(",") if e]
    if "sparse" in extras:
        out["sparse"] = bench_sparse(ipt, handle, args)
    if "morgan" in extras:
        out["morgan"] = bench_morgan(ipt, handle, args)
    if "batched" in extras:
        out["batched"] = bench_batched(ipt, handle, args)
    if "learned" in extras:
        out["learned"] = bench_learned(ipt, handle, args)
    if "nonsym" in extras:
        out["nonsym"] = bench_nonsym(ipt, handle, args)
    if "morgan_sweep" in extras:
        out["morgan_sweep"] = bench_morgan_sweep(ipt, handle, args)
    if "continuation" in extras:
        out["continuation"] = bench_continuation(ipt, handle, args)
    if "complex" in extras:
        out["complex"] = bench_complex(ipt, handle, args)
    if not args.no_cpu_baseline and int(os.environ.get("RANK", "0")) == 0:
        log("cpu baseline (oracle) ~%.0f s" % args.cpu_seconds)
        th, de = host[args.eps]
        out["cpu_baseline"] = cpu_baseline(th, de, args.cpu_seconds)
        if 0.01 in host and 0.05 in host:
            out["cpu_baseline"]["all_configs"] = cpu_baselines(host, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
