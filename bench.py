"""Benchmark: DAFMM matvec/s and GMRES time-to-1e-8 at N = 512^2, mixed vs FP64.

Workload (one step = the whole hot path once): the constant-contrast disc (R = 0.6, q = 1)
on a 512 x 512 cell-centred grid of [-1, 1]^2, kappa = 80, NCA tolerance 1e-10, HODLR
preconditioner of rank 256 (capped at child size / 4 on the deepest levels), plane wave at
angle 0; one step is one mixed-precision flexible GMRES solve from zero to a true relative
residual of 1e-8: complex128 DAFMM products until every residual estimate is below tol / delta
(delta = 1e-4), complex64 products after that, complex-bfloat16 HODLR off-diagonal factors,
complex128 Krylov basis, refinement residual and leaf/core solves.  `value` = solves/s over the
timed steps; the setup (tree, NCA, HODLR factorisation) is reported separately and with the
solve as the paper's totals, and the same solve with a rank-128 preconditioner beside it
(`rank_tradeoff`: shorter setup, more iterations).

Also reported (outside the timed region): the same solve in FP64 (warmed up and timed over the
same number of steps), DAFMM matvec/s for the FP64 and FP32 operators (median of 30 applies)
with their roofline (one column, and a block of 64 columns against the matrix-core peak), the
error of the mixed solution against the FP64 one, a block of 64 plane waves on Gaussian bumps
solved as one right-hand-side block (right-hand-side columns/s), the high-order panel operator
(p = 4) on a uniform tree (table setup, the dense product against the FP64 matrix-core peak, a
plane-wave solve without and with its HODLR preconditioner), the
roofline of the dominant kernel class (timed with HIP events on the launch stream during the
timed region), and the CPU oracle on the host cores: its FFT product of A timed, its GMRES run
for a bounded time, and the residual of the GPU solutions under the oracle operator.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DAFMM matvec/s and GMRES time-to-1e-8 at N=512^2, mixed vs FP64"
HBM_PEAK_GBS = 8000.0
# Dense matrix-core peaks of the MI355X (published): FP64 78.6, FP32 157.3 TFLOP/s.
MFMA_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(n, kappa, q, psis, seconds=20.0):
    """The oracle (numpy/scipy, FP64) on the host cores, on the same problem:
    * the FFT product of A (median of 3): the CPU counterpart of the DAFMM matvec;
    * its plain MGS GMRES(200) without preconditioner, run for a bounded number of iterations
      sized to about `seconds` from a short probe; the residual it reaches is reported as it is
      (no extrapolation);
    * the true relative residual ||A psi - f|| / ||f|| of each GPU solution in `psis` under the
      oracle operator (the paper's stopping criterion, evaluated independently of the library)."""
    import numpy as np

    from oracle import gmres as og
    from oracle import lsop
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = min(cores, 16)
    Vop = lsop.FFTApplyV(n, 1.0, kappa, workers=cores)
    f = lsop.rhs_planewave(n, 1.0, kappa, q, 0.0)
    A = lambda v: lsop.apply_A(Vop, v, q, kappa)
    oracle_relres = {k: float(np.linalg.norm(A(v) - f) / np.linalg.norm(f)) for k, v in psis.items()}
    x = np.random.default_rng(3).standard_normal(n * n) + 0j
    A(x)
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        A(x)
        ts.append(time.perf_counter() - t0)
    t_mv = float(np.median(ts))
    # GMRES: a probe of n1 iterations, then as many iterations as fit the budget under the MGS
    # cost model t(k) ~ k^2 (at most one restart cycle of 200)
    n1 = 20
    t0 = time.perf_counter()
    og.gmres(A, f, 1e-8, restart=200, maxit=n1)
    t1 = time.perf_counter() - t0
    nit = int(max(n1, min(200, n1 * math.sqrt(max(seconds, t1) / t1))))
    t1 = time.perf_counter()
    _, its, hist = og.gmres(A, f, 1e-8, restart=200, maxit=nit)
    t_run = time.perf_counter() - t1
    r_end = hist[-1]
    small = cpu_small_configs(cores)
    return {
        "small_configs": small,
        "value": round(1.0 / t_mv, 3),
        "unit": "matvec/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"oracle FFT product of A (complex128, zero-padded 2-D FFT over {cores} threads) on the same "
                   f"N={n*n} problem, median of 3: {t_mv * 1e3:.1f} ms per product; oracle GMRES(200) without "
                   f"preconditioner with that product: {its} iterations in {t_run:.1f} s reach relres {r_end:.2e} "
                   f"(not 1e-8)"),
        "matvec_ms": round(t_mv * 1e3, 2),
        "gmres": {"iters": its, "seconds": round(t_run, 2), "relres_reached": r_end,
                  "converged_to_1e-8": bool(r_end <= 1e-8)},
        "oracle_relres": oracle_relres,
    }


def cpu_small_configs(cores, seconds=10.0):
    """The oracle on the two smaller configurations: the 32^2 Gaussian problem (kappa 10: the
    dense 1024 x 1024 product, the FFT product, unpreconditioned GMRES(200) to 1e-10) and the
    256^2 problem with 8 Gaussian bumps (seed 0, kappa 40: the FFT product, unpreconditioned
    GMRES(200) towards 1e-8 for a bounded number of iterations sized to about `seconds`)."""
    import numpy as np

    from oracle import gmres as og
    from oracle import lsop
    from paper_2204_00326_amd import inputs

    def med(fn, reps):
        fn()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    out = {}
    pb = inputs.problem_gaussian_small()
    Ad = lsop.dense_A(pb.n, pb.L, pb.kappa, pb.q)
    Vop = lsop.FFTApplyV(pb.n, pb.L, pb.kappa, workers=cores)
    x = np.random.default_rng(4).standard_normal(pb.n ** 2) + 0j
    f = lsop.rhs_planewave(pb.n, pb.L, pb.kappa, pb.q, 0.0)
    t0 = time.perf_counter()
    _, its, hist = og.gmres(lambda v: Ad @ v, f, 1e-10, restart=200)
    out[pb.name] = {"dense_matvec_ms": round(1e3 * med(lambda: Ad @ x, 20), 4),
                    "fft_matvec_ms": round(1e3 * med(lambda: lsop.apply_A(Vop, x, pb.q, pb.kappa), 20), 4),
                    "gmres_to_1e-10": {"iters": its, "seconds": round(time.perf_counter() - t0, 3),
                                       "relres": hist[-1]}}
    pb = inputs.problem_bumps(256, 40.0, 0, count=8)
    Vop = lsop.FFTApplyV(pb.n, pb.L, pb.kappa, workers=cores)
    A = lambda v: lsop.apply_A(Vop, v, pb.q, pb.kappa)
    x = np.random.default_rng(5).standard_normal(pb.n ** 2) + 0j
    f = lsop.rhs_planewave(pb.n, pb.L, pb.kappa, pb.q, 0.0)
    t_mv = med(lambda: A(x), 5)
    n1 = 20
    t0 = time.perf_counter()
    og.gmres(A, f, 1e-8, restart=200, maxit=n1)
    t1 = time.perf_counter() - t0
    nit = int(max(n1, min(2000, n1 * math.sqrt(max(seconds, t1) / t1))))
    t0 = time.perf_counter()
    _, its, hist = og.gmres(A, f, 1e-8, restart=200, maxit=nit)
    out[pb.name] = {"fft_matvec_ms": round(1e3 * t_mv, 3),
                    "gmres_to_1e-8": {"iters": its, "seconds": round(time.perf_counter() - t0, 2),
                                      "relres_reached": hist[-1], "converged": bool(hist[-1] <= 1e-8)}}
    return out


COPY_BYTES = 256 << 20   # calibration copy: bytes read and bytes written
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_disc512_k80.txt")  # JSON text
KERNELS_SRC = os.path.join(ROOT, "paper_2204_00326_amd", "csrc", "kernels.hip")
# kernel names (before the argument list) of the classes the roofline may report
# (the HBM-bound ones; the matrix-core stencil kernel serves every DAFMM pass under one name)
COUNTED = {"hodlr_dot": ("lsk::k_hodlr_dot_seg<lsk::bf16, 4, 8>",),
           "hodlr_update": ("lsk::k_hodlr_update_wide<lsk::bf16>", "lsk::k_hodlr_update_list<lsk::bf16>"),
           "hodlr_upd_dot": ("lsk::k_hodlr_upd_dot<",),
           "hodlr_subtree": ("lsk::k_hodlr_subtree<lsk::bf16, 512>", "lsk::k_hodlr_subtree<lsk::bf16, 256>")}


def hodlr_launch_bytes(N, levels, rank, rank_div, max_rows, fsz, fused_ok, act=1.0, listed=False, dot_rows=None,
                       core_nodes=None, per_level=False, sub_level=-1, dense_leaves=0, leaf_rows=64):
    """Algorithmic HBM bytes per launch of the HODLR level kernels of one apply (one right-hand
    side), averaged over the launches of each class: a level's factor (N x r_l entries of fsz
    bytes) plus z (complex128) read, and z written by an update.  Mirrors the library's level
    plan: rank min(rank, child size / rank_div), chunks of at most max_rows rows, and an update
    fused with the next level's dot where that level's chunks are 1024 rows.  act: the fraction
    of rows in 256-row blocks with contrast; an update reads Y and writes z only there (the
    other rows of Y are zero).  listed: the library runs the updates over the listed blocks only
    (z read there too) and fuses none, the last one included (the z~ copy for flexible GMRES is
    a launch of its own); unlisted, the last update also stores z~, reading all of z and writing
    the copy.  dot_rows / core_nodes (per level, from the library's
    statistics): the rows whose W^T z an unfused dot forms and the nodes whose K^-1 block is read
    (the others meet a zero Y: a child without contrast).  per_level: ({class: {level: GB}},
    ranks) instead of the averages.  sub_level >= 0: the leaf solves and the levels sub_level..levels-1
    run in one launch per apply (class hodlr_subtree: b read, z written, the complex128 inverses
    of the dense_leaves leaves with contrast, W and Y on the dot_rows rows of each such level,
    the core inverses of its core_nodes); the level launches start one level above."""
    ranks = [max(1, min(rank, (N >> (l + 1)) // rank_div)) if rank_div > 0 else rank for l in range(levels)]
    def chunk(l):
        ch = N >> (l + 1)
        while ch > max_rows and ch % 2 == 0:
            ch //= 2
        return ch
    # per class: {level: bytes}, keyed like the library's launch tags (the level whose factors
    # a launch reads; an update fused with the next level's dot is tagged with that level)
    cls = {"hodlr_dot": {}, "hodlr_update": {}, "hodlr_upd_dot": {}}
    upd = (lambda ra: act * N * ra * fsz + 2 * act * N * 16) if listed else \
          (lambda ra: act * N * ra * fsz + (1 + act) * N * 16)
    top = levels if sub_level < 0 else sub_level
    if sub_level >= 0:
        b = 2 * N * 16 + dense_leaves * leaf_rows * leaf_rows * 16
        for l in range(sub_level, levels):
            rows = dot_rows[l] if dot_rows else N
            b += 2 * rows * ranks[l] * fsz
            b += (core_nodes[l] if core_nodes else 1 << l) * ((2 * ranks[l] + 15) // 16 * 16) * 2 * ranks[l] * 16
        cls["hodlr_subtree"] = {sub_level: b}
    pend = -1
    for l in range(top - 1, -1, -1):
        if pend >= 0 and fused_ok and not listed and N % 1024 == 0 and (N >> pend) % 128 == 0 and chunk(l) == 1024:
            cls["hodlr_upd_dot"][l] = N * (act * ranks[pend] + ranks[l]) * fsz + (1 + act) * N * 16
        else:
            if pend >= 0:
                cls["hodlr_update"][pend] = upd(ranks[pend])
            rows = dot_rows[l] if dot_rows else N
            cls["hodlr_dot"][l] = rows * ranks[l] * fsz + rows * 16
        pend = l
    # the last update: listed like the others (the z~ copy is a launch of its own), else it
    # also reads all of z and writes the copy
    cls["hodlr_update"][pend] = upd(ranks[pend]) if listed else act * N * ranks[pend] * fsz + (2 + act) * N * 16
    # SMW core products: the complex128 core inverses (2^l nodes of (2 r_l)^2), the chunk
    # partials of W^T z read once, s written
    cls["hodlr_core"] = {l: (core_nodes[l] if core_nodes else 1 << l) * (2 * ranks[l]) ** 2 * 16
                         + (N // chunk(l)) * ranks[l] * 16
                         + (1 << l) * 2 * ranks[l] * 16 for l in range(top)}
    if per_level:
        return {c: {l: b / 1e9 for l, b in v.items()} for c, v in cls.items()}, ranks
    return {c: sum(v.values()) / len(v) / 1e9 for c, v in cls.items() if v}


def _sha256(path):
    import hashlib
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def _read_counters(path, counter):
    """per-dispatch values of one counter from a rocprofv3 counter_collection.csv: {name: [KiB, ...]}"""
    import csv
    per = {}
    with open(path) as fh:
        for row in csv.DictReader(fh):
            if row.get("Counter_Name") != counter:
                continue
            key = (row["Kernel_Name"], int(row["Dispatch_Id"]))
            per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
    out = {}
    for (name, did), v in sorted(per.items(), key=lambda kv: kv[0][1]):
        out.setdefault(name, []).append(v)
    return out


def pmc_summary(fetch_csv, write_csv, cmd_fetch, cmd_write, workload):
    """Turn two rocprofv3 --pmc runs of this bench (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch)
    into HBM bytes per launch of the roofline kernels, each counter scaled by what it reads for
    the calibration copy of COPY_BYTES (the largest copyBuffer dispatch)."""
    fetch, write = _read_counters(fetch_csv, "FETCH_SIZE"), _read_counters(write_csv, "WRITE_SIZE")
    def copy_val(d):
        vals = [v for name, vs in d.items() if "copyBuffer" in name for v in vs]
        return max(vals)
    f_fetch = COPY_BYTES / 1024.0 / copy_val(fetch)
    f_write = COPY_BYTES / 1024.0 / copy_val(write)
    res = {"source_sha256": _sha256(KERNELS_SRC), "workload": workload, "copy_bytes": COPY_BYTES,
           "scale": {"FETCH_SIZE": f_fetch, "WRITE_SIZE": f_write}, "commands": [cmd_fetch, cmd_write], "kernels": {}}
    for cls, prefixes in COUNTED.items():
        hit = lambda name: any((p in name) if p.endswith("<") else (p + "(" in name) for p in prefixes)
        # per kernel, the last 80 % of its dispatches: the timed solves, past the autotuner's trials
        fv = [v for name, vs in fetch.items() if hit(name) for v in vs[len(vs) // 5:]]
        wv = [v for name, vs in write.items() if hit(name) for v in vs[len(vs) // 5:]]
        if not fv or not wv:
            continue
        fk, wk = sum(fv) / len(fv), sum(wv) / len(wv)
        res["kernels"][cls] = {"kernel": " + ".join(prefixes), "dispatches": len(fv), "fetch_kib": fk,
                               "write_kib": wk, "hbm_bytes_per_launch": (fk * f_fetch + wk * f_write) * 1024.0}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(res, fh, indent=1)
    md = TRAFFIC_FILE[:-4] + ".md"
    with open(md, "w") as fh:
        fh.write("# HBM traffic per launch (rocprofv3 counters), disc 512x512, kappa 80, mixed bench\n\n")
        fh.write("Commands (repository root, one MI355X):\n\n```\n" + cmd_fetch + "\n" + cmd_write + "\n```\n\n")
        fh.write(f"Calibration: a device copy of {COPY_BYTES >> 20} MiB reads FETCH_SIZE x {f_fetch:.4f} and "
                 f"WRITE_SIZE x {f_write:.4f} of its true bytes; both factors are applied below.\n\n")
        fh.write("| class | kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM MB per launch |\n|---|---|---:|---:|---:|---:|\n")
        for cls, v in res["kernels"].items():
            fh.write(f"| {cls} | `{v['kernel']}` | {v['dispatches']} | {v['fetch_kib']:.0f} | {v['write_kib']:.0f} | "
                     f"{v['hbm_bytes_per_launch'] / 1e6:.2f} |\n")
        fh.write(f"\nWorkload {workload}; kernels.hip sha256 {res['source_sha256']} (bench.py reports traffic only for "
                 "this source and workload).\n")
    print(json.dumps(res, indent=1))


def measured_traffic(cls, workload):
    """HBM bytes per launch of a class from the committed counter summary, or None when absent or
    taken on a different kernel source or workload"""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
        if t["source_sha256"] != _sha256(KERNELS_SRC) or t.get("workload") != workload or cls not in t["kernels"]:
            return None
        return t["kernels"][cls]["hbm_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def panels_bench(args, torch, np, ls):
    """High-order panels (p = 4 Chebyshev nodes per box side) on a uniform tree of args.panels^2
    boxes of [-1, 1]^2, kappa / 2, the disc contrast at the nodes: table setup time and the dense
    product A x (event-timed median of 20; FP64 matrix cores), against the FP64 MFMA peak (8
    flops per complex multiply-add of the nb^2 p^4 operator entries); then a plane-wave solve to
    1e-8 without and with the panel system's HODLR preconditioner (rank args.panels_rank)."""
    nside, p, kappa = args.panels, 4, args.kappa / 2
    beta = 1.0 / nside
    c = -1.0 + (2 * np.arange(nside) + 1) * beta
    xi = np.sort(np.cos((2 * np.arange(p) + 1) * np.pi / (2 * p)))
    X = np.array([(cx + beta * u, cy + beta * v) for cx in c for cy in c for u in xi for v in xi])
    q = (np.hypot(X[:, 0], X[:, 1]) < 0.6).astype(float)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Pp = ls.Panels(nside, 1.0, p, kappa, q)
    t_setup = time.perf_counter() - t0
    x = torch.from_numpy(np.random.default_rng(1).standard_normal(Pp.N) + 0j).cuda()
    y = torch.empty_like(x)
    s = torch.cuda.current_stream()
    for _ in range(3):
        Pp.apply(x, y)
    ts = []
    for _ in range(20):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        Pp.apply(x, y)
        e1.record(s)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    us = 1e3 * float(np.median(ts))
    flops = 8.0 * (nside * nside) ** 2 * (p * p) ** 2
    out = {"workload": f"uniform {nside}x{nside} boxes, p={p} ({Pp.N} unknowns), kappa={kappa}, disc R=0.6",
           "setup_s": round(t_setup, 3), "apply_us": round(us, 1), "far_rule_points": Pp.nfar,
           "roofline": {"bound": "mfma", "achieved": round(flops / (us * 1e-6) / 1e12, 3), "peak": 78.6,
                        "unit": "TFLOP/s", "frac": round(flops / (us * 1e-6) / 1e12 / 78.6, 4)}}
    # plane-wave solve to 1e-8 (theta = 0): unpreconditioned GMRES, then right-preconditioned by
    # the panel system's HODLR approximation (fixed rank)
    u = np.exp(1j * kappa * X[:, 0])
    f = torch.from_numpy(kappa ** 2 * q * u).cuda()
    solves = {}
    if args.panels_rank > 0:
        for name in ("none", "hodlr"):
            if name == "hodlr":
                pinfo = Pp.precondition(args.panels_rank)
            Pp.solve(f, tol=1e-8, restart=100, maxit=3000)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, info = Pp.solve(f, tol=1e-8, restart=100, maxit=3000)
            torch.cuda.synchronize()
            solves[name] = {"ms": round(1e3 * (time.perf_counter() - t1), 2), "iters": info["iters"],
                            "relres": info["relres"], "status": info["status"]}
        solves["hodlr_factors"] = {k: (round(v, 2) if isinstance(v, float) else v) for k, v in pinfo.items()}
        out["solve_1e-8"] = solves
    log("panels", out)
    Pp.close()
    return out


def rhs_block(args, torch, np, inputs, ls):
    """Many incidence angles as one right-hand-side block: Gaussian bumps (8, seed 1) on the same
    grid and wavenumber, theta_j = 2 pi j / nrhs, one mixed solve of the block after a warmup
    solve; right-hand-side columns per second and per-column iterations."""
    n, kappa, nrhs = args.n, args.kappa, args.block_rhs
    pb = inputs.problem_bumps(n, kappa, seed=1, count=8)
    t0 = time.perf_counter()
    P = ls.Problem(pb.points(), pb.q, kappa, 1e-10,
                   ls.Options(hodlr_rank=args.rank, hodlr_rank_div=args.rank_div, prec=ls.LS_MIXED, eps_inner=1e-7,
                              inner_tol=args.delta32, restart=60, maxit=2000, pc_bf16=args.pc_bf16))
    t_setup = time.perf_counter() - t0
    F = P.rhs_planewave([2.0 * math.pi * j / nrhs for j in range(nrhs)])
    P.solve(F, tol=1e-8, prec=ls.LS_MIXED)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    X, infos = P.solve(F, tol=1e-8, prec=ls.LS_MIXED)
    torch.cuda.synchronize()
    t_blk = time.perf_counter() - t1
    # one column alone, for the per-column cost of the block against a single solve
    f1 = P.rhs_planewave([0.0])
    P.solve(f1, tol=1e-8, prec=ls.LS_MIXED)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, i1 = P.solve(f1, tol=1e-8, prec=ls.LS_MIXED)
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t1
    its = [i["iters"] for i in infos]
    out = {"workload": f"bumps8_seed1_{n}_k{kappa:g}_{nrhs}angles", "nrhs": nrhs, "setup_s": round(t_setup, 3),
           "block_solve_s": round(t_blk, 4), "rhs_columns_per_s": round(nrhs / t_blk, 2),
           "ms_per_column": round(1e3 * t_blk / nrhs, 3), "single_column_ms": round(1e3 * t_one, 3),
           "iters_min_max": [min(its), max(its)], "relres_max": max(i["relres"] for i in infos),
           "all_converged": all(i["status"] in ("CONVERGED", "REFINE_STAGNATED") and i["relres"] <= 1e-8
                                for i in infos), "hodlr_rank": args.rank, "gmres_restart": 60}
    log("rhs block", out)
    P.close()
    del X, F
    torch.cuda.synchronize()
    return out


def matvec_block(P, st, n, torch, np, ls, nrhs):
    """The product on a block of nrhs columns (the batched form: one launch per pass for every
    column): median of 10 event-timed block products per precision, per-column time and the
    matrix-core roof of the whole block."""
    stream = torch.cuda.current_stream()
    x = torch.randn(nrhs, n * n, dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    out = {}
    for name, prec, dt, far in (("fp64", ls.LS_FP64, "f64", "entries_far64"), ("fp32", ls.LS_FP32, "f32", "entries_far32")):
        for _ in range(3):
            P.matvec(x, y, prec=prec)
        ts = []
        for _ in range(10):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            P.matvec(x, y, prec=prec)
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        flops = 8.0 * (st["entries_near"] + st[far]) * nrhs
        ach = flops / (ms * 1e-3) / 1e12
        out[name] = {"bound": "mfma", "achieved": round(ach, 3), "peak": MFMA_PEAK_TFLOPS[dt], "unit": "TFLOP/s",
                     "frac": round(ach / MFMA_PEAK_TFLOPS[dt], 4), "nrhs": nrhs, "us_per_block": round(1e3 * ms, 1),
                     "us_per_column": round(1e3 * ms / nrhs, 2), "columns_per_s": round(nrhs / (ms * 1e-3), 1)}
    del x, y
    log(f"matvec block of {nrhs}", out)
    return out


def matvec_rates(P, st, n, torch, np, ls):
    """Median time of the FP64 and FP32 products (30 event-timed products each after 3 warm-up
    ones), their per-pass split and the whole product against the matrix-core roof."""
    stream = torch.cuda.current_stream()
    x = torch.randn(n * n, dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    rates = {}
    for name, prec in (("fp64", ls.LS_FP64), ("fp32", ls.LS_FP32)):
        for _ in range(3):
            P.matvec(x, y, prec=prec)
        ts = []
        for _ in range(30):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            P.matvec(x, y, prec=prec)
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        rates[name] = 1e3 / float(np.median(ts))
    log("matvec/s", rates)
    # per-pass split of the product: each pass group timed between two events on the stream
    # (launch gaps and split-K reductions included) over 30 products of each precision, in
    # microseconds per product; outside the median-timed loop above, so its timers do not
    # touch the rates
    passes = {}
    for name, prec, b in (("fp64", ls.LS_FP64, "64"), ("fp32", ls.LS_FP32, "32")):
        keys = [k for k in ls.PROFILE_SPANS if k.startswith(f"mv{b}_")]
        for k in keys:
            P.profile_enable(k, 1)
        for _ in range(30):
            P.matvec(x, y, prec=prec)
        torch.cuda.synchronize()
        sp = {}
        for k in keys:
            ms, timed, _ = P.profile_read(k)
            P.profile_enable(k, 0)
            sp[k.split("_", 1)[1]] = round(1e3 * ms / timed, 2) if timed else 0.0
        sp["sum"] = round(sum(sp.values()), 2)
        passes[name] = sp
    log("matvec passes (us)", passes)
    # the whole DAFMM product against the matrix-core roof: 8 real flops per complex entry of
    # every pass (near field, P2M, M2M, M2L, L2L, L2P) over the median product time
    mv_flops = {"fp64": 8.0 * (st["entries_near"] + st["entries_far64"]),
                "fp32": 8.0 * (st["entries_near"] + st["entries_far32"])}
    roof_mv = {}
    for name, dt in (("fp64", "f64"), ("fp32", "f32")):
        ach = mv_flops[name] * rates[name] / 1e12
        roof_mv[name] = {"bound": "mfma", "achieved": round(ach, 3), "peak": MFMA_PEAK_TFLOPS[dt],
                         "unit": "TFLOP/s", "frac": round(ach / MFMA_PEAK_TFLOPS[dt], 4),
                         "flops_per_matvec": mv_flops[name], "us_per_matvec": round(1e6 / rates[name], 2),
                         "passes_us": passes[name]}
    return rates, passes, roof_mv


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--kappa", type=float, default=80.0)
    ap.add_argument("--rank", type=int, default=256, help="HODLR rank (levels capped at child size / rank-div)")
    ap.add_argument("--restart", type=int, default=500)
    ap.add_argument("--rank-div", type=int, default=4)
    ap.add_argument("--delta32", type=float, default=1e-4)
    ap.add_argument("--graph-iters", type=int, default=1, help="Arnoldi steps per captured graph (0: host-driven)")
    ap.add_argument("--dcgs2", type=int, default=0,
                    help="device-driven steps: 1 delayed CGS2 (one basis pass, stop test one step late), 0 CGS2")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false")
    ap.add_argument("--sample-every", type=int, default=7, help="time every k-th launch of a kernel class")
    ap.add_argument("--pc-bf16", type=int, default=1, help="bfloat16 HODLR factors in mixed solves (0: complex64)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tradeoff-rank", type=int, default=128,
                    help="also time the mixed solve with this HODLR rank (setup against solve time); 0: skip")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--panels", type=int, default=32,
                    help="also time the high-order panel operator on this many boxes per side (0: skip)")
    ap.add_argument("--panels-rank", type=int, default=64,
                    help="rank of the panel system's HODLR preconditioner for the panel solves (0: no solves)")
    ap.add_argument("--block-rhs", type=int, default=64,
                    help="also solve this many plane waves on Gaussian bumps as one block (0: skip)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "CMD_FETCH", "CMD_WRITE"),
                    help="summarise two rocprofv3 --pmc runs of this bench into the traffic file and exit")
    ap.add_argument("--mv-block", type=int, default=64,
                    help="columns of the block product measured beside the single-column one (0: none)")
    ap.add_argument("--matvec-only", action="store_true",
                    help="time only the DAFMM products (no preconditioner, no solve) and print their line")
    args = ap.parse_args()
    workload = f"disc{args.n}_k{args.kappa:g}_mixed_hodlr{args.rank}"
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, workload)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only (the batch axes, right-hand sides and queued problems, "
              "shard across GPUs without exchange); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2204_00326_amd import inputs, ls

    torch.cuda.set_device(0)
    n, kappa = args.n, args.kappa
    pb = inputs.problem_disc(n, kappa)
    if args.matvec_only:
        P = ls.Problem(pb.points(), pb.q, kappa, 1e-10, ls.Options(hodlr_rank=0, eps_inner=1e-7))
        st = P.stats()
        rates, _, roof_mv = matvec_rates(P, st, n, torch, np, ls)
        blk = matvec_block(P, st, n, torch, np, ls, args.mv_block) if args.mv_block > 0 else None
        print(json.dumps({"metric": "DAFMM matvec/s", "value": round(rates["fp64"], 1), "unit": "matvec/s",
                          "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
                          "config": {"workload": f"disc{n}_k{kappa:g}_matvec", "n": n, "kappa": kappa,
                                     "eps_nca": 1e-10, "eps_inner": 1e-7},
                          "matvec_per_s": {k: round(v, 1) for k, v in rates.items()},
                          "roofline_matvec": roof_mv, "roofline_matvec_block": blk}), flush=True)
        P.close()
        return
    t0 = time.perf_counter()
    P = ls.Problem(pb.points(), pb.q, kappa, 1e-10,
                   ls.Options(hodlr_rank=args.rank, hodlr_rank_div=args.rank_div, prec=ls.LS_MIXED,
                              eps_inner=1e-7, inner_tol=args.delta32, restart=args.restart, maxit=2000,
                              graph_iters=args.graph_iters, pc_bf16=args.pc_bf16, dcgs2=args.dcgs2))
    tune = P.autotune() if args.autotune else None
    pc_fmt = "bf16" if args.pc_bf16 else "c64"
    t_setup = time.perf_counter() - t0
    log("autotune", tune)
    st = P.stats()
    log(f"setup {t_setup:.2f} s", st)
    f = P.rhs_planewave([0.0])
    stream = torch.cuda.current_stream()

    def solve(prec):
        psi, info = P.solve(f, tol=1e-8, prec=prec)
        return psi, info[0]

    for _ in range(args.warmup):
        solve(ls.LS_MIXED)
        log("warmup done")
    torch.cuda.synchronize()
    # every 7th launch of each class is timed (7 is coprime with the HODLR level count, so
    # every level is sampled alike; timed dispatches run one at a time)
    for c in ls.PROFILE_CLASSES:
        P.profile_enable(c, args.sample_every)
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        psi_m, info = solve(ls.LS_MIXED)
        infos.append(info)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    prof = {c: P.profile_read(c) for c in ls.PROFILE_CLASSES}
    for c in ls.PROFILE_CLASSES:
        P.profile_enable(c, 0)
    log("timed steps", infos)
    ms_step = 1e3 * t_total / args.steps

    # the same mixed solve replayed from captured graphs (kernel timers off), outside the
    # timed region: what a caller without timers gets
    ms_graph = None
    if args.graph_iters > 0:
        solve(ls.LS_MIXED)   # capture
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            solve(ls.LS_MIXED)
        torch.cuda.synchronize()
        ms_graph = 1e3 * (time.perf_counter() - t1) / args.steps
        log(f"graph-replayed mixed solve {ms_graph:.1f} ms")

    # FP64 comparison (outside the timed region), timed like the mixed solve: warmup solves
    # (which also capture its graphs), then the same number of timed solves
    for _ in range(max(1, args.warmup)):
        solve(ls.LS_FP64)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        psi_d, info_d = solve(ls.LS_FP64)
    torch.cuda.synchronize()
    t_fp64 = (time.perf_counter() - t1) / args.steps
    err_mixed = float(torch.linalg.vector_norm(psi_m - psi_d) / torch.linalg.vector_norm(psi_d))
    log("fp64 solve", info_d, f"{t_fp64*1e3:.1f} ms per solve over {args.steps}; mixed vs fp64 rel diff {err_mixed:.2e}")

    # the error function E(x) of the mixed solution at random points of the domain (off the
    # grid), Eq. (eq:error): the paper's accuracy measure; direct summation over the cells
    rng = np.random.default_rng(7)
    M = 256
    pts = rng.uniform(-1.0, 1.0, (M, 2))
    qx = (np.hypot(pts[:, 0], pts[:, 1]) < 0.6).astype(np.float64)
    tg = torch.from_numpy(pts).cuda()
    qd = torch.from_numpy(qx).cuda()
    P.error_eval(tg, qd, 0.0, psi_m)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    E = P.error_eval(tg, qd, 0.0, psi_m)
    torch.cuda.synchronize()
    t_err = time.perf_counter() - t1
    E = E.cpu().numpy()
    inside = qx > 0
    psi_scale = float(torch.linalg.vector_norm(psi_m, ord=float("inf"))) / kappa ** 2
    err_fn = {"targets": M, "ms": round(1e3 * t_err, 3), "cells_per_target": n * n,
              "cell_integrals_per_s": round(M * n * n / t_err, 1),
              "E_median_in_disc": float(np.median(E[inside])) / psi_scale,
              "E_max_in_disc": float(E[inside].max()) / psi_scale,
              "E_median_outside": float(np.median(E[~inside])) / psi_scale,
              "scale": "E / (max|psi| / kappa^2)",
              "note": "per target all n^2 cells are visited; cells with zero density are skipped"}
    log("error function", err_fn)

    rates, passes, roof_mv = matvec_rates(P, st, n, torch, np, ls)
    # the batched form: one block of right-hand sides per product (operator tiles reused across
    # the columns, the passes' latency shared by all of them)
    roof_blk = matvec_block(P, st, n, torch, np, ls, args.mv_block) if args.mv_block > 0 else None

    # calibration copy of COPY_BYTES for the HBM counters (read and written once)
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    # roofline of the dominant kernel class over the timed region: achieved = algorithmic
    # bytes (or flops) per launch / average duration of the timed launches of the class
    N = n * n
    r = args.rank
    lb = st["hodlr_levels"]
    fsz = {"bf16": 4, "c64": 8}[pc_fmt]   # bytes per stored HODLR factor entry in mixed solves
    act = st["hodlr_rows_active"] / N
    listed = N % 256 == 0 and st["hodlr_rows_active"] * 4 < 3 * N   # the library's rule
    sub = dict(sub_level=st["hodlr_subtree_level"], dense_leaves=st["hodlr_dense_leaves"],
               leaf_rows=st["leaf_side"] ** 2)
    hb = hodlr_launch_bytes(N, lb, args.rank, args.rank_div, tune["hodlr_rows"] if tune else 1024, fsz,
                            pc_fmt == "bf16", act, listed, st["hodlr_dot_rows"][:lb], st["hodlr_core_nodes"][:lb],
                            **sub)
    per_launch = {
        # flops of the product's middle launch (8 real flops per complex multiply-add), matrix
        # cores: the top-level M2L and the near-field classes not packed into the upward pass
        "near_m2l64": ("mfma", "f64", 8.0 * st["entries_mid64"] / 1e12),
        "near_m2l32": ("mfma", "f32", 8.0 * st["entries_mid32"] / 1e12),
        # HODLR level launches (unfused dot, unfused update, update fused with the next dot)
        **{c: ("hbm", None, v) for c, v in hb.items()},
        # leaf solves: the complex128 inverses of the leaves with contrast (leaf_side^2 points
        # each), b read and z written
        "leaf_solve": ("hbm", None, (st["hodlr_dense_leaves"] * (st["leaf_side"] ** 2) ** 2 * 16 + 2 * N * 16) / 1e9),
    }
    cand = {c: prof[c] for c in per_launch if prof[c][1] > 0}

    def roof_of(c):
        tot_ms, timed, _ = cand[c]
        bound, dt, amount = per_launch[c]
        achieved = amount / (tot_ms / timed / 1e3)
        if bound == "hbm":
            tb = measured_traffic(c, workload) if pc_fmt == "bf16" else None
            return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    # measured HBM bytes per launch (counters, copy-calibrated) vs the algorithmic bytes
                    "traffic": None if tb is None else round(tb / 1e9, 6),
                    "traffic_unit": "GB per launch", "algorithmic_per_launch": round(amount, 6)}
        peak = MFMA_PEAK_TFLOPS[dt]
        return {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": None}

    # dominant: largest estimated total time (average timed duration x all launches)
    dom = max(cand, key=lambda c: cand[c][0] / cand[c][1] * cand[c][2])
    roof = roof_of(dom)
    tot_ms, launches, all_launches = cand[dom]
    roof["kernel"] = {"near_m2l64": "k_stencil_mfma<double> (middle launch of the product)",
                      "near_m2l32": "k_stencil_mfma<float> (middle launch of the product)",
                      "hodlr_update": f"k_hodlr_update_list / k_hodlr_update_wide<{'bf16' if args.pc_bf16 else 'float'}> "
                                      "(HODLR z -= Y s)",
                      "hodlr_dot": f"k_hodlr_dot_seg<{'bf16, 4' if args.pc_bf16 else 'float, 2'}> (HODLR W^T z)",
                      "hodlr_upd_dot": "k_hodlr_upd_dot<1024> (HODLR z -= Y s fused with the next level's W^T z)",
                      "hodlr_core": "k_hodlr_core_rows (HODLR SMW core products s = K^-1 t)",
                      "leaf_solve": "k_leaf_apply<double> (HODLR leaf inverses)",
                      "hodlr_subtree": "k_hodlr_subtree (HODLR leaf solves and deepest levels, one launch)"}[dom]
    roof["avg_launch_us"] = round(tot_ms / launches * 1e3, 2)
    roof["launches_timed"] = launches
    roof["launches"] = all_launches
    # every measured class against its own roof (the dominant one is reported above)
    roof["classes"] = {c: dict(roof_of(c), avg_launch_us=round(cand[c][0] / cand[c][1] * 1e3, 2),
                               launches_timed=cand[c][1], launches=cand[c][2],
                               est_total_ms=round(cand[c][0] / cand[c][1] * cand[c][2], 3)) for c in cand}
    # per binary level: every HODLR launch of one more mixed solve timed (outside the timed
    # region), averaged per (class, level), against the level's algorithmic bytes
    lvl_bytes, lvl_ranks = hodlr_launch_bytes(N, lb, args.rank, args.rank_div, tune["hodlr_rows"] if tune else 1024,
                                              fsz, pc_fmt == "bf16", act, listed, st["hodlr_dot_rows"][:lb],
                                              st["hodlr_core_nodes"][:lb], per_level=True, **sub)
    hcls = ("hodlr_dot", "hodlr_update", "hodlr_upd_dot", "hodlr_core")
    for c in hcls:
        P.profile_enable(c, 1)
    solve(ls.LS_MIXED)
    each = {c: P.profile_read_each(c) for c in hcls}
    for c in hcls:
        P.profile_enable(c, 0)
    levels_tab = []
    for l in range(lb):
        row = {"level": l, "rank": lvl_ranks[l], "dot_rows": st["hodlr_dot_rows"][l],
               "core_nodes": st["hodlr_core_nodes"][l]}
        for c in hcls:
            t = [ms for ms, tag in each[c] if tag == l]
            if t and l in lvl_bytes[c]:
                us = 1e3 * sum(t) / len(t)
                gbs = lvl_bytes[c][l] / (us / 1e6)
                row[c] = {"us": round(us, 2), "launches": len(t), "GB": round(lvl_bytes[c][l], 5),
                          "GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
        levels_tab.append(row)
    log("hodlr levels", levels_tab)


    line = {
        "metric": METRIC,
        "value": round(args.steps / t_total, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128 operator (c64 once the residual is below tol / 1e-4) + bf16/c64 HODLR factors + c128 "
                 "Krylov/refinement/leaf/core solves (mixed)",
        # near-field + M2L launches (one per operator application) of each precision per timed solve
        "operator_applies_per_solve": {"c128": round(prof["near_m2l64"][2] / args.steps, 2),
                                       "c64": round(prof["near_m2l32"][2] / args.steps, 2)},
        "data": "synthetic",
        "config": {"workload": workload, "n": n, "N": N, "kappa": kappa,
                   "contrast": "disc R=0.6 q=1", "eps_nca": 1e-10, "eps_inner": 1e-7, "hodlr_rank": r,
                   "tol": 1e-8, "nrhs": 1, "gmres_restart": args.restart, "hodlr_rank_div": args.rank_div,
                   "fp32_relax_delta": args.delta32, "hodlr_factors_mixed": pc_fmt,
                   "hodlr_update_rows_active": round(act, 4),
                   # W^T z rows and K^-1 blocks the applies form (the rest meet a zero Y)
                   "hodlr_dot_rows_frac": round(sum(st["hodlr_dot_rows"][:lb]) / (lb * N), 4),
                   "hodlr_core_nodes_frac": round(sum(st["hodlr_core_nodes"][:lb]) / ((1 << lb) - 1), 4),
                   "gmres_driver": (f"device-driven {'delayed CGS2' if args.dcgs2 else 'CGS2'}, "
                                    f"{args.graph_iters} step(s) per graph") if args.graph_iters
                   else "host-driven CGS2"},
        "time_to_1e8_ms": {"mixed": round(ms_step, 3), "fp64": round(t_fp64 * 1e3, 3),
                           "mixed_graph_replay": None if ms_graph is None else round(ms_graph, 3)},
        "mixed_speedup_vs_fp64": round(t_fp64 * 1e3 / ms_step, 3),
        # the paper's notation (Section 6.2): T_Pf = HODLR factorisation, T_Ps = preconditioned
        # solve, T_Hybrid = T_Pf + T_Ps; the DAFMM precompute (tree, NCA) and the whole setup too
        "paper_times_s": {"T_Pf": round(st["t_hodlr_ms"] / 1e3, 4), "T_Ps": round(ms_step / 1e3, 5),
                          "T_Hybrid": round(st["t_hodlr_ms"] / 1e3 + ms_step / 1e3, 4),
                          "dafmm_precompute": round((st["t_plan_ms"] + st["t_nca_ms"]) / 1e3, 4),
                          "setup_plus_solve": round(t_setup + ms_step / 1e3, 4),
                          "T_Ps_fp64": round(t_fp64, 5), "setup_plus_solve_fp64": round(t_setup + t_fp64, 4)},
        "iters": {"mixed": infos[-1]["iters"], "fp64": info_d["iters"], "n_refine": infos[-1]["n_refine"]},
        "relres": {"mixed": infos[-1]["relres"], "fp64": info_d["relres"]},
        "mixed_vs_fp64_rel_diff": err_mixed,
        "matvec_per_s": {k: round(v, 1) for k, v in rates.items()},
        # the spec roof of the matvec: the whole ls_matvec (all passes) against the MFMA peak
        "roofline_matvec": roof_mv,
        "roofline_matvec_block": roof_blk,
        "setup_s": round(t_setup, 3),
        "setup_ms": {k: round(st[f"t_{k}_ms"], 1) for k in ("plan", "nca", "hodlr", "hodlr_aca", "hodlr_apply",
                                                             "hodlr_cores")},
        "ranks": {"fp64": st["rank_max64"], "fp32": st["rank_max32"]},
        "roofline": roof,
        "hodlr_levels": levels_tab,
        "error_function": err_fn,
    }
    if args.tradeoff_rank > 0:
        # the same problem with another preconditioner rank (setup against iterations);
        # reported beside the headline, not in it
        P.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P2 = ls.Problem(pb.points(), pb.q, kappa, 1e-10,
                        ls.Options(hodlr_rank=args.tradeoff_rank, hodlr_rank_div=args.rank_div, prec=ls.LS_MIXED,
                                   eps_inner=1e-7, inner_tol=args.delta32, restart=args.restart, maxit=2000,
                                   graph_iters=args.graph_iters, pc_bf16=args.pc_bf16, dcgs2=args.dcgs2))
        if args.autotune:
            P2.autotune()
        t_setup2 = time.perf_counter() - t0
        f2 = P2.rhs_planewave([0.0])
        P2.solve(f2, tol=1e-8, prec=ls.LS_MIXED)
        torch.cuda.synchronize()
        ts2 = []
        for _ in range(max(2, min(args.steps, 5))):
            t1 = time.perf_counter()
            psi2, i2 = P2.solve(f2, tol=1e-8, prec=ls.LS_MIXED)
            torch.cuda.synchronize()
            ts2.append(time.perf_counter() - t1)
        d2 = float(torch.linalg.vector_norm(psi2 - psi_d) / torch.linalg.vector_norm(psi_d))
        line["rank_tradeoff"] = {"hodlr_rank": args.tradeoff_rank, "setup_s": round(t_setup2, 3),
                                 "time_to_1e8_ms": round(1e3 * float(np.median(ts2)), 3), "iters": i2[0]["iters"],
                                 "relres": i2[0]["relres"], "vs_fp64_rel_diff": d2,
                                 "headline_setup_s": round(t_setup, 3), "headline_ms": round(ms_step, 3)}
        log("rank tradeoff", line["rank_tradeoff"])
        P2.close()
    if args.panels > 0:
        line["panels"] = panels_bench(args, torch, np, ls)
    if args.block_rhs > 0:
        P.close()
        line["rhs_block"] = rhs_block(args, torch, np, inputs, ls)
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        psis = {"mixed": psi_m.cpu().numpy(), "fp64": psi_d.cpu().numpy()}
        cb = cpu_baseline(n, kappa, pb.q, psis, args.cpu_seconds)
        line["oracle_relres"] = cb.pop("oracle_relres")
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
