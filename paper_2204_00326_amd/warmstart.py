"""Learned GMRES warm start: dataset generation with the solver, training with the
ls_nop_* kernels, and held-out evaluation (iterations and time to tol, zero vs learned start).

Every arithmetic step of the network runs in the library's kernels; this module only
orchestrates (batching, shuffling, learning-rate schedule) and stores tensors.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import inputs, ls


@dataclass
class Dataset:
    X: "torch.Tensor"       # [S, 6, n, n] float32
    w: "torch.Tensor"       # [S, n, n] complex64  b / kappa^2, b = f exp(i phi) the WKB start
    t: "torch.Tensor"       # [S, n, n] complex64  (psi - b) / kappa^2
    snorm2: "torch.Tensor"  # [S] float32          |psi / kappa^2|^2
    solve_ms: float
    setup_ms: float


def solver_options(**kw) -> ls.Options:
    o = dict(hodlr_rank=15, restart=300, maxit=1000, build_fp32=0)
    o.update(kw)
    return ls.Options(**o)


def generate(seeds, n: int, angles_per_contrast: int = 1, tol: float = 1e-8, log=None) -> Dataset:
    """Solve one problem per seed (inputs.problem_learned) and collect network inputs and targets."""
    import torch
    Xs, ws, ts, ss = [], [], [], []
    t_solve = t_setup = 0.0
    for k, seed in enumerate(seeds):
        pb = inputs.problem_learned(seed, n, angles_per_contrast)
        t0 = time.perf_counter()
        P = ls.Problem(pb.points(), pb.q, pb.kappa, 1e-10, solver_options())
        t1 = time.perf_counter()
        F = P.rhs_planewave(pb.thetas)
        psi, info = P.solve(F, tol=tol)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t_setup += t1 - t0
        t_solve += t2 - t1
        qd = torch.from_numpy(pb.q).cuda()
        F2 = F.reshape(-1, n * n)
        psi2 = psi.reshape(-1, n * n)
        for a, th in enumerate(pb.thetas):
            Xs.append(ls.nop_features(n, pb.L, qd, pb.kappa, float(th)))
            base = ls.nop_warmstart(n, pb.L, qd, pb.kappa, float(th), None, F2[a].contiguous())
            ws.append((base / pb.kappa ** 2).reshape(n, n).to(torch.complex64))
            ts.append(((psi2[a] - base) / pb.kappa ** 2).reshape(n, n).to(torch.complex64))
            ss.append(float((psi2[a].abs() ** 2).sum()) / pb.kappa ** 4)
        P.close()
        if log and (k + 1) % 50 == 0:
            log(f"generated {k + 1}/{len(seeds)} contrasts, solve {t_solve:.1f}s setup {t_setup:.1f}s")
    return Dataset(torch.stack(Xs), torch.stack(ws), torch.stack(ts),
                   torch.tensor(ss, dtype=torch.float32, device="cuda"), 1e3 * t_solve, 1e3 * t_setup)


def validate(net: "ls.NeuralOperator", data: Dataset, batch: int) -> float:
    """Mean loss of the network over a dataset (forward and loss kernels only)."""
    S = data.X.shape[0]
    tot = 0.0
    for b0 in range(0, S, batch):
        b1 = min(S, b0 + batch)
        O = net.forward(data.X[b0:b1].contiguous())
        lb, _ = net.loss(O, data.w[b0:b1].contiguous(), data.t[b0:b1].contiguous(), data.snorm2[b0:b1].contiguous())
        tot += float(lb.sum())                  # per-sample losses
    return tot / S


def train(net: "ls.NeuralOperator", data: Dataset, epochs: int, batch: int, lr: float = 2e-3, seed: int = 0,
          log=None, val: Dataset | None = None):
    """Adam with a cosine learning-rate schedule; returns the per-epoch mean training loss.

    With a validation set the parameters of the epoch with the lowest validation loss are kept
    (early stopping) and the per-epoch validation losses are returned as a second list."""
    import torch
    S = data.X.shape[0]
    rng = np.random.default_rng(seed)
    steps = epochs * (S // batch)
    hist, vhist = [], []
    best, best_params = float("inf"), None
    step = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(S)).cuda()
        tot = 0.0
        nb = 0
        for b0 in range(0, S - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            X = data.X[idx].contiguous()
            O = net.forward(X)
            lb, dO = net.loss(O, data.w[idx].contiguous(), data.t[idx].contiguous(), data.snorm2[idx].contiguous())
            net.backward(dO)
            cur = lr * 0.5 * (1 + math.cos(math.pi * step / max(steps, 1)))
            net.adam_step(max(cur, 1e-6))
            tot += float(lb.mean())
            nb += 1
            step += 1
        hist.append(tot / max(nb, 1))
        msg = f"epoch {ep}: loss {hist[-1]:.4f}"
        if val is not None:
            vhist.append(validate(net, val, batch))
            msg += f" val {vhist[-1]:.4f}"
            if vhist[-1] < best:
                best, best_params = vhist[-1], net.get_params()
        if log and (ep % max(1, epochs // 10) == 0 or ep == epochs - 1):
            log(msg)
    if best_params is not None:
        net.set_params(best_params)
    return (hist, vhist) if val is not None else hist


def evaluate(net: "ls.NeuralOperator", seeds, n: int, tol: float = 1e-8, prec: int = ls.LS_FP64,
             hodlr_rank: int = 15):
    """Per held-out seed: GMRES iterations and time from zero and from the learned start."""
    import torch
    rows = []
    for seed in seeds:
        pb = inputs.problem_learned(seed, n, 1)
        P = ls.Problem(pb.points(), pb.q, pb.kappa, 1e-10, solver_options(hodlr_rank=hodlr_rank))
        f = P.rhs_planewave([float(pb.thetas[0])])
        qd = torch.from_numpy(pb.q).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        psi_ref, i0 = P.solve(f, tol=tol, prec=prec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        th = float(pb.thetas[0])
        X = ls.nop_features(n, pb.L, qd, pb.kappa, th)[None]
        O = net.forward(X)
        psi0 = ls.nop_warmstart(n, pb.L, qd, pb.kappa, th, O[0], f)
        psi, i1 = P.solve(f, psi=psi0.clone(), x0=True, tol=tol, prec=prec)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        # the WKB start alone (no network), to separate the two contributions
        b0 = ls.nop_warmstart(n, pb.L, qd, pb.kappa, th, None, f)
        _, i2 = P.solve(f, psi=b0.clone(), x0=True, tol=tol, prec=prec)
        fn = torch.linalg.vector_norm(f)
        raw0 = float(torch.linalg.vector_norm(P.matvec(psi0) - f) / fn)
        pn = torch.linalg.vector_norm(psi_ref)
        err0 = float(torch.linalg.vector_norm(psi0 - psi_ref) / pn)
        errb = float(torch.linalg.vector_norm(b0 - psi_ref) / pn)
        rows.append({"seed": seed, "kappa": pb.kappa, "its_zero": i0[0]["iters"], "its_warm": i1[0]["iters"],
                     "its_wkb": i2[0]["iters"], "ms_zero": 1e3 * (t1 - t0), "ms_warm": 1e3 * (t2 - t1),
                     "warm_err": err0, "wkb_err": errb, "warm_relres0_raw": raw0, "warm_relres0": i1[0]["relres0"],
                     "wkb_relres0": i2[0]["relres0"], "status_warm": i1[0]["status"],
                     "relres_warm": i1[0]["relres"], "relres_zero": i0[0]["relres"]})
        P.close()
    return rows


def summarize(rows, tol: float = 1e-8) -> dict:
    z = np.array([r["its_zero"] for r in rows], dtype=float)
    w = np.array([r["its_warm"] for r in rows], dtype=float)
    tz = np.array([r["ms_zero"] for r in rows])
    tw = np.array([r["ms_warm"] for r in rows])
    med = lambda k: float(np.median([r[k] for r in rows]))
    ok = all(r["relres_warm"] <= 1.01 * tol for r in rows)
    wk = np.array([r["its_wkb"] for r in rows], dtype=float)
    return {"samples": len(rows), "its_zero_mean": float(z.mean()), "its_warm_mean": float(w.mean()),
            "its_wkb_mean": float(wk.mean()), "its_saved_frac_wkb_only": float(1 - wk.sum() / z.sum()),
            "its_saved_frac": float(1 - w.sum() / z.sum()), "ms_zero_mean": float(tz.mean()),
            "ms_warm_mean": float(tw.mean()), "time_saved_frac": float(1 - tw.sum() / tz.sum()),
            "fewer_its": int((w < z).sum()), "more_its": int((w > z).sum()),
            "warm_err_median": med("warm_err"), "wkb_err_median": med("wkb_err"),
            "wkb_relres0_median": med("wkb_relres0"), "warm_relres0_raw_median": med("warm_relres0_raw"),
            "warm_relres0_median": med("warm_relres0"),
            "rejected": sum(r["status_warm"] == "WARMSTART_REJECTED" for r in rows), "all_reach_tol": ok}


def main():
    import argparse
    import json
    import sys
    import torch

    ap = argparse.ArgumentParser(description="train and evaluate the learned GMRES warm start")
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--train", type=int, default=2000, help="training solutions")
    ap.add_argument("--angles", type=int, default=1, help="incidence angles per training contrast")
    ap.add_argument("--val", type=int, default=200, help="validation contrasts (early stopping)")
    ap.add_argument("--test", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--width", type=int, default=32)
    ap.add_argument("--modes", type=int, default=12)
    ap.add_argument("--layers", type=int, default=4)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--bf16", type=int, default=1, help="channel mixing on BF16 matrix cores (0: FP32)")
    args = ap.parse_args()
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    data = generate(range(0, args.train // args.angles), args.n, args.angles, log=log)
    t_gen = time.perf_counter() - t0
    log(f"dataset {data.X.shape[0]} samples in {t_gen:.1f}s")
    val = generate(range(50000, 50000 + args.val), args.n, 1) if args.val > 0 else None
    net = ls.NeuralOperator(args.n, args.width, args.modes, args.layers, batch_max=args.batch, seed=0,
                            bf16=bool(args.bf16))
    t0 = time.perf_counter()
    out = train(net, data, args.epochs, args.batch, args.lr, log=log, val=val)
    hist, vhist = out if val is not None else (out, [])
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    seeds = range(100000, 100000 + args.test)
    res = {"n": args.n, "train_solutions": int(data.X.shape[0]), "epochs": args.epochs,
           "net": {"width": args.width, "modes": args.modes, "layers": args.layers, "params": net.nparams,
                   "bf16_channel_mixing": bool(args.bf16)},
           "t_generate_s": t_gen, "t_train_s": t_train, "loss_first": hist[0], "loss_last": hist[-1],
           "val_loss_best": min(vhist) if vhist else None,
           "val_epoch_best": int(np.argmin(vhist)) if vhist else None}
    for rank in (15, 0):
        rows = evaluate(net, seeds, args.n, hodlr_rank=rank)
        res[f"heldout_hodlr{rank}"] = summarize(rows)
        log(f"hodlr {rank}:", res[f"heldout_hodlr{rank}"])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
