"""Train the warm-start network on GPU-solved instances and measure what it saves.

    python -m paper_2001_01978_amd.train_warm --omega 24 --n 12 --train 4096 \\
        --out paper_2001_01978_amd/weights/warm_o24_n12.npz --report report.json

Large training sets can be labelled over several runs (--labels-only with
--train-seed0 and --labels-cache), then joined with --labels-from.

Training instances: the random family at fixed (omega, n) with seeds
[seed0, seed0 + train); held-out instances: seeds [10^6, 10^6 + heldout).  Labels are the
half occupations from the batched GPU solver (tol 1e-8).  The report holds
the training curve and, per held-out instance, the Lanczos products from the
warm start (with its RANDOM fallback) and from the RANDOM start, both run to
the same residual.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def log(msg):
    print(f"[train_warm] {msg}", flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--omega", type=int, default=24)
    ap.add_argument("--n", type=int, default=12)
    ap.add_argument("--train", type=int, default=4096)
    ap.add_argument("--heldout", type=int, default=200)
    ap.add_argument("--chunk", type=int, default=1024)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--hidden", type=int, default=256)
    ap.add_argument("--label-tol", type=float, default=1e-8)
    ap.add_argument("--krylov", type=int, default=20)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--out", required=True)
    ap.add_argument("--report", required=True)
    ap.add_argument("--labels-cache", default=None, help="npz of (X, T) to reuse instead of solving")
    ap.add_argument("--family", default="family3", choices=["family3", "large"],
                    help="family3: G0 ~ U[0.1,0.6); large: G0 = 0.3 (the Omega=32/34 workload family)")
    ap.add_argument("--train-seed0", type=int, default=0, help="first training seed (training seeds: seed0 .. seed0+train)")
    ap.add_argument("--single", action="store_true",
                    help="label with the single-instance mixed-precision solver (spaces beyond the batched kernel)")
    ap.add_argument("--labels-only", action="store_true",
                    help="stop after writing --labels-cache (labels of large training sets over several runs)")
    ap.add_argument("--labels-from", nargs="*", default=None,
                    help="npz files of (X, T) to concatenate as the training set instead of solving")
    args = ap.parse_args(argv)

    import torch
    from . import inputs, pairdiag, warm

    om, n = args.omega, args.n

    def instance(seed):
        if args.family == "large":
            return inputs.c5_instance(om, n, seed=seed)
        return inputs.family3_instance(seed, omega=om, n=n)

    t0 = time.perf_counter()
    if args.labels_from:
        parts = [np.load(f, allow_pickle=False) for f in args.labels_from]
        X = np.concatenate([d["X"] for d in parts])
        T = np.concatenate([d["T"] for d in parts])
        log(f"labels from {len(parts)} files: {X.shape}")
        label_seconds = 0.0
    elif args.labels_cache and os.path.exists(args.labels_cache):
        d = np.load(args.labels_cache, allow_pickle=False)
        X, T = d["X"], d["T"]
        log(f"labels from {args.labels_cache}: {X.shape}")
        label_seconds = 0.0
    else:
        Xs, Ts = [], []
        for c0 in range(0, args.train, args.chunk):
            insts = [instance(args.train_seed0 + s) for s in range(c0, min(args.train, c0 + args.chunk))]
            if args.single:
                X, T = warm.labels_single(insts, tol=args.label_tol, krylov=args.krylov, log=log)
            else:
                X, T, r = warm.labels(insts, tol=args.label_tol, krylov=args.krylov)
                log(f"labels {c0 + len(insts)}/{args.train}: batched kernel {r.info['kernel_seconds']:.1f} s, "
                    f"{r.converged.sum()}/{len(insts)} converged")
            Xs.append(X)
            Ts.append(T)
            if args.labels_cache:
                np.savez(args.labels_cache, X=np.concatenate(Xs), T=np.concatenate(Ts))
        X, T = np.concatenate(Xs), np.concatenate(Ts)
        label_seconds = time.perf_counter() - t0
        if args.labels_only:
            log(f"labels for seeds {args.train_seed0}..{args.train_seed0 + args.train - 1} written to "
                f"{args.labels_cache} in {label_seconds:.0f} s")
            return 0

    t1 = time.perf_counter()
    net = warm.WarmNet(om, hidden=args.hidden, seed=0)
    hist = net.train(torch.tensor(X, device="cuda"), torch.tensor(T, device="cuda"), epochs=args.epochs,
                     batch=args.batch, lr=args.lr, log=log)
    train_seconds = time.perf_counter() - t1
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    net.save(args.out)
    log(f"saved {args.out} (loss {hist[0]:.3e} -> {hist[-1]:.3e}, {train_seconds:.1f} s)")

    basis = pairdiag.Basis(om, n, store_states=False)
    rows = []
    for s in range(10 ** 6, 10 ** 6 + args.heldout):
        _, _, eps, V = instance(s)
        prec = "f32" if args.single else "f64"
        rw = warm.solve(basis, eps, V, net, krylov=args.krylov, tol=args.tol, want_psi=False, precision=prec)
        rr = warm.solve(basis, eps, V, None, krylov=args.krylov, tol=args.tol, want_psi=False, seed=s,
                        precision=prec)
        rows.append(dict(seed=s, warm_products=rw.iterations, random_products=rr.iterations,
                         warm_seconds=rw.seconds, random_seconds=rr.seconds, fallback=rw.fallback_used,
                         dE=abs(rw.E0 - rr.E0) / abs(rr.E0), converged=bool(rw.converged and rr.converged)))
        if len(rows) % 20 == 0 or args.single:
            w = np.mean([r["warm_products"] for r in rows])
            rnd = np.mean([r["random_products"] for r in rows])
            log(f"held-out {len(rows)}: mean products warm {w:.1f} vs random {rnd:.1f}")
    if not rows:
        with open(args.report, "w") as f:
            json.dump(dict(omega=om, n=n, train_instances=int(X.shape[0]), epochs=args.epochs, loss_first=hist[0],
                           loss_last=hist[-1], label_seconds=label_seconds, train_seconds=train_seconds), f, indent=1)
        return 0
    w = np.array([r["warm_products"] for r in rows])
    rnd = np.array([r["random_products"] for r in rows])
    report = dict(omega=om, n=n, train_instances=int(X.shape[0]), heldout=len(rows), epochs=args.epochs,
                  loss_first=hist[0], loss_last=hist[-1], loss_history=hist[:: max(1, len(hist) // 50)],
                  label_seconds=label_seconds, train_seconds=train_seconds,
                  mean_products_warm=float(w.mean()), mean_products_random=float(rnd.mean()),
                  median_products_warm=float(np.median(w)), median_products_random=float(np.median(rnd)),
                  fallbacks=int(sum(r["fallback"] for r in rows)),
                  max_rel_dE=float(max(r["dE"] for r in rows)), all_converged=all(r["converged"] for r in rows),
                  rows=rows)
    with open(args.report, "w") as f:
        json.dump(report, f, indent=1)
    log(f"held-out: warm {w.mean():.1f} vs random {rnd.mean():.1f} products "
        f"({100 * (1 - w.mean() / rnd.mean()):.0f}% fewer); max |dE|/E {report['max_rel_dE']:.1e}")


if __name__ == "__main__":
    sys.exit(main())
