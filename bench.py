#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X: prints one JSON line.

Workload: the large random family at Omega=32, n=16 (601,080,390 states,
256 pair hops per row), eps ~ U[0, 32), G_ij = 0.3(1 + 0.2u), seed 0.  One
step is one ground-state solve (pd_lanczos_ground: basis by unranking, sigma,
recurrence, full reorthogonalisation, tridiagonal solve, restarts, FP64
acceptance, occupations) in mixed precision (FP32 products, FP64 everything
else) to an FP64-checked residual of 1e-10, from a seeded random start.

value = sigma non-zeros generated per second of the timed solves (whole job).
Also reported: time-to-E0 for plain FP64, mixed precision and the learned
warm start (mixed precision from the network's product-state start), per-
product sigma rates, the roofline of the dominant kernel (the FP32 sigma:
VALU-issue bound; its gather-model and measured HBM rates alongside) from
its HIP-event durations inside the timed region, the batched solver on
4096 instances of the uneven random family, and the oracle's CPU rate on a
bounded sample of rows of the same instance.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# 32-bit VALU lane operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (one wave64 instruction per SIMD every 4 cycles; FP32 FMA counted as one op).
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic VALU work per non-zero of the prefix-delta sigma: target rank =
# rank + A + B (2 adds), up/down choice (compare + select), gather address,
# coefficient address, FMA.
OPS_PER_NONZERO = 7


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--omega", type=int, default=32)
    ap.add_argument("--n", type=int, default=16)
    ap.add_argument("--krylov", type=int, default=20)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-FP64 time-to-E0 solve")
    ap.add_argument("--no-warm", action="store_true", help="skip the learned-warm-start time-to-E0 solve")
    ap.add_argument("--no-batched", action="store_true", help="skip the 4096-instance batched solve")
    ap.add_argument("--no-odd", action="store_true", help="skip the odd-system (all blocks) solve")
    ap.add_argument("--no-trunc", action="store_true", help="skip the truncated-space leg")
    ap.add_argument("--no-eigs", action="store_true", help="skip the lowest-eigenpairs (thick restart) leg")
    ap.add_argument("--no-scf", action="store_true", help="skip the self-consistent loop leg")
    ap.add_argument("--no-f64cols", action="store_true",
                    help="skip the mixed solve with every Krylov column in FP64")
    ap.add_argument("--no-starts", action="store_true", help="skip the E1 and HF start solves (context)")
    ap.add_argument("--no-prev", action="store_true",
                    help="skip the previous-solution start (couplings x1.01 from the converged state)")
    ap.add_argument("--batched-count", type=int, default=4096)
    ap.add_argument("--cpu-rows", type=int, default=0, help="oracle sample size in rows (0: auto)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--sigma-reps", type=int, default=5)
    ap.add_argument("--verbose", action="store_true", help="per-cycle progress of the solves on stderr")
    ap.add_argument("--kernel-only", action="store_true",
                    help="for counter runs: one 1 GiB device copy (the known-size reference), then "
                         "--sigma-reps FP32 and FP64 products of the workload, and exit")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


KERNEL_SOURCES = ["paper_2001_01978_amd/csrc/sigma_impl.h"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(name):
    """Per-launch HBM bytes of the dominant kernel from the committed rocprofv3
    counter summary profiles/<name>.txt ('key: value' lines), or None when the
    summary is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", name + ".txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(om, n, eps, V, rows_req):
    import numpy as np
    import oracle
    oracle.build(force=False)
    d = math.comb(om, n)
    K = n * (om - n)
    x = np.ones(d)              # values do not change the work; the full vector is needed for the gathers
    r0 = d // 3
    rows = rows_req or 200000
    t = time.perf_counter()
    oracle.sigma_block(om, n, eps, V, x, r0, r0 + 2000)      # warm caches / threads
    t = time.perf_counter()
    oracle.sigma_block(om, n, eps, V, x, r0, r0 + rows)
    dt = time.perf_counter() - t
    if not rows_req and dt < 10.0:
        rows = int(rows * min(20.0 / max(dt, 1e-3), 200.0))
        rows = min(rows, d - r0)
        t = time.perf_counter()
        oracle.sigma_block(om, n, eps, V, x, r0, r0 + rows)
        dt = time.perf_counter() - t
    return dict(value=rows * K / dt, unit="nnz/s", cores=oracle.num_threads(), kind="oracle",
                sample=f"hash-search oracle sigma (states by '01' inversion, targets by the hash) over "
                       f"{rows} consecutive rows from rank {r0} of the same Omega={om}, n={n} instance "
                       f"({rows * K:.3e} non-zeros, {dt:.1f} s)")


def stream_probe(torch, gib=8, reps=5):
    """Achievable HBM bandwidth on this machine, event-timed over `gib` GiB buffers:
    a read-only stream (a sum), 16 columns read together (a matrix-vector
    product, the access pattern of a Gram-Schmidt pass), a device-to-device
    copy (read + write bytes) and a fill (write only).  Returns (best,
    {probe: GB/s})."""
    n = gib * (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    cols = a.view(16, n // 16)          # 16 columns streamed together, as in a Gram-Schmidt pass
    v = torch.ones(n // 16, dtype=torch.float32, device="cuda")
    probes = {"read (sum)": (lambda: a.sum(), n * 4),
              "read 16 columns (gemv)": (lambda: torch.mv(cols, v), n * 4 + (n // 16) * 4),
              "copy": (lambda: b.copy_(a), 2 * n * 4),
              "write (fill)": (lambda: b.fill_(2.0), n * 4)}
    out = {}
    for name, (fn, nbytes) in probes.items():
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = nbytes / (e0.elapsed_time(e1) / reps / 1e3) / 1e9
    del a, b, cols, v
    torch.cuda.empty_cache()
    return max(out.values()), out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path (the product "
              "would shard by row ranges with an all-gather of x per step); use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2001_01978_amd import inputs, pairdiag

    torch.cuda.set_device(0)
    om, n = args.omega, args.n
    _, _, eps, V = inputs.c5_instance(om, n, seed=0)
    K = n * (om - n)
    tb = time.perf_counter()
    basis = pairdiag.Basis(om, n, store_states=False)
    torch.cuda.synchronize()
    basis_seconds = time.perf_counter() - tb
    D = basis.dim
    log(f"workload omega={om} n={n} dim={D} hops/row={K}")

    if args.kernel_only:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").uniform_(-1, 1)
        dst = torch.empty_like(src)
        dst.copy_(src)                       # reads and writes exactly 1 GiB each
        torch.cuda.synchronize()
        del src, dst
        for dt in (torch.float32, torch.float64):
            x = torch.empty(D, dtype=dt, device="cuda").uniform_(-1, 1)
            y = torch.empty_like(x)
            for _ in range(args.sigma_reps):
                basis.sigma(eps, V, x, y)
            torch.cuda.synchronize()
            del x, y
        log(f"kernel-only run done (kernel source {kernel_source_hash()})")
        return

    # ---- per-product sigma rates (separate buffers, same stream)
    sig = {}
    for name, dt in (("f32", torch.float32), ("f64", torch.float64)):
        x = torch.empty(D, dtype=dt, device="cuda").uniform_(-1, 1)
        y = torch.empty_like(x)
        basis.sigma(eps, V, x, y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.sigma_reps):
            basis.sigma(eps, V, x, y)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3 / args.sigma_reps
        es = 4 if name == "f32" else 8
        balg = D * (K * es + 2 * es)
        sig[name] = dict(ms=t * 1e3, nnz_per_s=D * K / t, alg_GBps=balg / t / 1e9, alg_bytes=balg)
        log(f"sigma {name}: {t*1e3:.2f} ms  {D*K/t:.3e} nnz/s  {balg/t/1e9:.0f} GB/s algorithmic")
        del x, y
    torch.cuda.empty_cache()

    common = dict(krylov=args.krylov, tol=args.tol, start="random", seed=1, want_psi=False, verbose=args.verbose)
    nb_mixed = pairdiag.workspace_bytes(basis, krylov=args.krylov, precision="f32")
    nb_f64 = 0 if args.no_plain else pairdiag.workspace_bytes(basis, krylov=args.krylov, precision="f64")
    nb_f64c = 0 if args.no_f64cols else pairdiag.workspace_bytes(basis, krylov=args.krylov, precision="f32_f64cols")
    ws = pairdiag.device_buffer(max(nb_mixed, nb_f64, nb_f64c))

    def solve(precision, want_psi=False):
        kw = dict(common, want_psi=want_psi)
        return pairdiag.lanczos_ground(basis, eps, V, precision=precision, workspace=ws, **kw)

    for w in range(args.warmup):
        r = solve("f32")
        log(f"warmup {w}: E0={r.E0:.12f} products={r.iterations} ({r.iterations_f32} f32) {r.seconds:.1f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for k in range(args.steps):
        r = solve("f32", want_psi=(k == args.steps - 1 and not args.no_prev))
        results.append(r)
        log(f"step {k}: E0={r.E0:.12f} rho={r.residual:.2e} products={r.iterations} ({r.iterations_f32} f32) "
            f"{r.seconds:.2f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    nnz = sum(r.iterations for r in results) * D * K
    value = nnz / elapsed
    mixed = results[-1]
    n32 = sum(r.iterations_f32 for r in results)
    s32 = sum(r.sigma_seconds_f32 for r in results)
    avg32 = s32 / max(n32, 1)
    balg32 = D * (K * 4 + 8)
    ops32 = D * K * OPS_PER_NONZERO
    achieved = ops32 / avg32 / 1e12 if n32 else None

    plain = None
    if not args.no_plain:
        r64 = solve("f64")
        plain = r64
        log(f"plain f64: E0={r64.E0:.12f} products={r64.iterations} {r64.seconds:.2f} s")

    # Mixed precision with every Krylov column in FP64 (FP32 copies for the
    # products), beside the default FP32 storage of q_2..q_m.
    f64cols = None
    if not args.no_f64cols:
        rc = solve("f32_f64cols")
        f64cols = dict(seconds=rc.seconds, products=rc.iterations, products_f32=rc.iterations_f32,
                       E0_rel_diff_vs_mixed=abs(rc.E0 - mixed.E0) / abs(mixed.E0))
        log(f"mixed, FP64 columns: {rc.iterations} products {rc.seconds:.2f} s")

    # Previous-solution start: the next problem of a self-consistent sweep,
    # here the same instance with the couplings scaled by 1.01, started from
    # the converged state of the timed solve, against a random start.
    prev = None
    if not args.no_prev and mixed.psi is not None:
        VB = np.asarray(V) * 1.01
        kw = dict(krylov=args.krylov, tol=args.tol, want_psi=False, precision="f32", workspace=ws,
                  verbose=args.verbose)
        rp = pairdiag.lanczos_ground(basis, eps, VB, x0=mixed.psi, **kw)
        rr = pairdiag.lanczos_ground(basis, eps, VB, start="random", seed=1, **kw)
        prev = dict(change="couplings x1.01", seconds_previous_start=rp.seconds, products_previous_start=rp.iterations,
                    seconds_random_start=rr.seconds, products_random_start=rr.iterations,
                    E0_rel_diff=abs(rp.E0 - rr.E0) / abs(rr.E0))
        log(f"previous-solution start: {rp.iterations} products {rp.seconds:.2f} s vs random {rr.iterations} "
            f"products {rr.seconds:.2f} s")
        mixed.psi = None
        torch.cuda.empty_cache()

    # The deterministic starts of the paper (E1) and of the Hartree-Fock state, for context.
    starts = None
    if not args.no_starts:
        starts = {}
        for st in ("e1", "hf"):
            kw = dict(common, start=st)
            r_s = pairdiag.lanczos_ground(basis, eps, V, precision="f32", workspace=ws, **kw)
            starts[st] = dict(seconds=r_s.seconds, products=r_s.iterations, converged=r_s.converged,
                              E0_rel_diff_vs_random=abs(r_s.E0 - mixed.E0) / abs(mixed.E0))
            log(f"start {st}: {r_s.iterations} products {r_s.seconds:.2f} s")

    warm_r, warm_info = None, None
    wpath = os.path.join(ROOT, "paper_2001_01978_amd", "weights", f"warm_o{om}_n{n}.npz")
    if not args.no_warm and os.path.exists(wpath):
        from paper_2001_01978_amd import warm
        t = time.perf_counter()
        net = warm.WarmNet.load(wpath)
        lo = net.logits(om, eps, V)
        x0 = basis.warm_start(torch.tensor(lo, dtype=torch.float32))
        warm_r = pairdiag.lanczos_ground(basis, eps, V, x0=x0, fallback=True, precision="f32", workspace=ws,
                                         krylov=args.krylov, tol=args.tol, want_psi=False, verbose=args.verbose)
        torch.cuda.synchronize()
        warm_total = time.perf_counter() - t
        warm_info = dict(weights=os.path.relpath(wpath, ROOT), seconds_including_network=warm_total,
                         fallback_used=warm_r.fallback_used)
        log(f"warm (mixed): E0={warm_r.E0:.12f} products={warm_r.iterations} {warm_total:.2f} s incl. network")

    del ws
    torch.cuda.empty_cache()

    batched = None
    if not args.no_batched:
        insts = [inputs.family3_instance(s) for s in range(args.batched_count)]
        dims = np.array([math.comb(i[0], i[1]) for i in insts])
        Ks = np.array([i[1] * (i[0] - i[1]) for i in insts])
        rb = pairdiag.lanczos_ground_batched(insts, krylov=20, tol=args.tol)   # includes the autotuner
        rb = pairdiag.lanczos_ground_batched(insts, krylov=20, tol=args.tol)   # tuned
        bnnz = float((rb.iterations * dims * Ks).sum())
        batched = dict(workload=f"{args.batched_count} instances, omega ~ U{{10..24}}, n ~ U{{ceil(omega/4)..omega/2}}, "
                                f"eps ~ U[0,omega), G_ij = G0(1+0.2u), G0 ~ U[0.1,0.6), seeds 0..{args.batched_count-1}",
                       sum_dim=int(dims.sum()), max_dim=int(dims.max()), converged=int(rb.converged.sum()),
                       seconds=rb.info["kernel_seconds"], call_seconds=rb.info["seconds"],
                       instances_per_s=args.batched_count / rb.info["kernel_seconds"],
                       products=int(rb.iterations.sum()), nnz_per_s=bnnz / rb.info["kernel_seconds"],
                       block=rb.info["block"], teams=rb.info["teams"], team_size=rb.info["team_size"],
                       team_instances=rb.info["large"], status=pairdiag._STATUS.get(rb.status))
        log(f"batched: {batched['converged']}/{args.batched_count} converged in {batched['seconds']:.2f} s, "
            f"{batched['nnz_per_s']:.3e} nnz/s")

    # The first few states (thick-restart Lanczos, FP64): the four lowest of the
    # same instance, and the ground state alone against the paper's restart.
    eigs = None
    if not args.no_eigs:
        kw_e = dict(krylov=args.krylov, tol=args.tol, seed=1, want_psi=False)
        re4 = pairdiag.lanczos_eigs(basis, eps, V, 4, **kw_e)
        re1 = pairdiag.lanczos_eigs(basis, eps, V, 1, **kw_e)
        eigs = dict(nev4=dict(E=[float(e) for e in re4.E], products=re4.iterations, cycles=re4.restarts,
                              seconds=re4.seconds, max_residual=float(re4.residuals.max()), converged=re4.converged),
                    nev1=dict(E=float(re1.E[0]), products=re1.iterations, seconds=re1.seconds,
                              E0_rel_diff_vs_f64=(abs(re1.E[0] - plain.E0) / abs(plain.E0)) if plain else None,
                              single_vector_restart_f64_products=plain.iterations if plain else None,
                              single_vector_restart_f64_seconds=plain.seconds if plain else None))
        log(f"eigs: nev=4 {re4.iterations} products {re4.seconds:.2f} s; nev=1 thick {re1.iterations} products "
            f"{re1.seconds:.2f} s")

    # Truncated space (Sec. 3.5): the same Omega=32 instance cut to 1e8 states
    # with the paper's 1e8 histogram bins; products with both rank-to-row maps.
    trunc = None
    if not args.no_trunc:
        tl, tb = 100_000_000, 10**8
        pairdiag.trunc_select(om, n, eps, V, tl, tb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tinfo = pairdiag.trunc_select(om, n, eps, V, tl, tb)
        t1 = time.perf_counter()
        tbas = pairdiag.Basis.truncated(om, n, eps, V, tl, tb, info=tinfo)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        tms = {}
        for index in ("bitmap", "bsearch"):
            tb_i = tbas if index == "bitmap" else pairdiag.Basis.truncated(om, n, eps, V, tl, tb, index=index,
                                                                          info=tinfo)
            for dt in (torch.float32, torch.float64):
                xt = torch.ones(tb_i.dim, dtype=dt, device="cuda")
                yt = tb_i.sigma(eps, V, xt)
                reps = 5 if index == "bitmap" else 2
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    tb_i.sigma(eps, V, xt, yt)
                e1.record()
                torch.cuda.synchronize()
                tms[f"{index}_{'f32' if dt == torch.float32 else 'f64'}_ms"] = e0.elapsed_time(e1) / reps
                del xt, yt
            del tb_i
        tg = pairdiag.lanczos_ground(tbas, eps, V, krylov=args.krylov, tol=args.tol, start="random", seed=1,
                                     precision="f32", want_psi=False)
        trunc = dict(workload=f"Omega={om}, n={n} truncated to <= {tl} states, {tb} bins", kept=int(tinfo.kept),
                     cut_bin=int(tinfo.cut_bin), cutoff=tinfo.cutoff, select_seconds=t1 - t0,
                     build_seconds=t2 - t1, sigma=tms, solve_seconds=tg.seconds, products=tg.iterations,
                     E0=tg.E0, E0_minus_full=tg.E0 - mixed.E0, converged=tg.converged)
        log(f"truncated: kept {tinfo.kept}, select {t1 - t0:.3f} s, build {t2 - t1:.3f} s, sigma {tms}, "
            f"solve {tg.iterations} products {tg.seconds:.2f} s")
        del tbas
        torch.cuda.empty_cache()

    # Self-consistent loop (synthetic mean field eps0 + W <N>/2) on an Omega=24,
    # 12-pair instance, with and without the previous-solution start.
    scf = None
    if not args.no_scf:
        so, sn = 24, 12
        _, _, seps, sV = inputs.c5_instance(so, sn, seed=0)
        u = inputs.uniform01(5, 0, so * so).reshape(so, so)
        sW = 0.3 * 0.5 * (u + u.T)
        sb = pairdiag.Basis(so, sn, store_states=False)
        scf = dict(workload=f"Omega={so}, n={sn}, W = 0.3 (U + U^T)/2, mixing 0.6, field tol 1e-8, "
                            f"solve tol 1e-11, krylov 20")
        for reuse in (True, False):
            rs = pairdiag.scf_ground(sb, seps, sW, sV, mixing=0.6, tol=1e-8, krylov=20, start="random",
                                     reuse_psi=reuse, lanczos_tol=1e-11)
            scf["previous_solution_start" if reuse else "random_start_each"] = dict(
                iterations=rs.info["iterations"], products=rs.info["products"], seconds=rs.info["seconds"],
                converged=bool(rs.info["converged"]), E0=rs.E0)
        log(f"scf: {scf['previous_solution_start']['products']} products {scf['previous_solution_start']['seconds']:.2f} s "
            f"vs {scf['random_start_each']['products']} / {scf['random_start_each']['seconds']:.2f} s")
        del sb

    # Odd particle number (blocking): every block of an omega = 25, 12-pair
    # instance (2n + 1 = 25 particles), each block 12 pairs on 24 orbits.
    odd = None
    if not args.no_odd:
        oo, on = 25, 12
        _, _, oeps, oV = inputs.c5_instance(oo, on, seed=0)
        okw = dict(krylov=20, tol=args.tol, start="random", seed=1)
        pairdiag.lanczos_ground_odd(oo, on, oeps, oV, **okw)
        ro = pairdiag.lanczos_ground_odd(oo, on, oeps, oV, **okw)
        odim = math.comb(oo - 1, on)
        odd = dict(workload=f"odd system omega={oo}, {2 * on + 1} particles, all {oo} blocks of {on} pairs on "
                            f"{oo - 1} orbits (dim {odim} each), FP64, krylov 20",
                   seconds=ro.seconds, products=ro.iterations, converged=ro.converged, E=ro.E, block=ro.block,
                   nnz_per_s=ro.iterations * odim * on * (oo - 1 - on) / ro.seconds,
                   status=pairdiag._STATUS.get(ro.status))
        log(f"odd: E={ro.E:.12f} block {ro.block}, {ro.iterations} products in {ro.seconds:.2f} s")

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(om, n, eps, V, args.cpu_rows)
        log(f"cpu baseline: {cpu['value']:.3e} nnz/s on {cpu['cores']} threads")

    traffic = traffic_from_profiles(f"sigma_f32_omega{om}_n{n}_counters")
    achievable, probes = stream_probe(torch)
    log("stream probes (8 GiB): " + ", ".join(f"{k} {v:.0f} GB/s" for k, v in probes.items()))
    out = {
        "metric": "sigma nonzeros/s + HBM GB/s; time-to-E0 at Omega=32,n=16, plain vs mixed vs warm",
        "value": value,
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (seeded SplitMix64 instance, eps~U[0,32), G_ij=0.3(1+0.2u))",
        "config": {"workload": f"ground state, Omega={om}, n={n}, dim={D}, mixed precision, "
                               f"krylov={args.krylov}, tol={args.tol:g}",
                   "omega": om, "n": n, "dim": D, "hops_per_row": K, "krylov": args.krylov},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TOPS, "unit": "Top/s",
                     "frac": (achieved / PEAK_VALU_TOPS) if achieved else None,
                     "traffic": traffic,
                     "kernel": "sigma_kernel<uint32,float,16>",
                     "ops_per_nonzero": OPS_PER_NONZERO,
                     "algorithmic_ops_per_launch": ops32,
                     "avg_launch_ms": avg32 * 1e3,
                     "hbm": {"gather_model_bytes_per_launch": balg32,
                             "gather_model_GBps": balg32 / avg32 / 1e9 if n32 else None,
                             "measured_GBps": traffic / avg32 / 1e9 if (traffic and n32) else None,
                             "measured_frac_of_peak": traffic / avg32 / 1e9 / PEAK_HBM_GBS
                             if (traffic and n32) else None,
                             "achievable_GBps": achievable,
                             "achievable_probes_GBps": probes,
                             "measured_frac_of_achievable": traffic / avg32 / 1e9 / achievable
                             if (traffic and n32) else None,
                             "measured_frac_of_16_column_stream": traffic / avg32 / 1e9
                             / probes["read 16 columns (gemv)"] if (traffic and n32) else None,
                             "peak_GBps": PEAK_HBM_GBS}},
        "cpu_baseline": cpu,
        "time_to_E0_s": {"f64": plain.seconds if plain else None, "mixed": mixed.seconds,
                         "warm": warm_info["seconds_including_network"] if warm_info else None},
        "E0": {"f64": plain.E0 if plain else None, "mixed": mixed.E0, "warm": warm_r.E0 if warm_r else None,
               "mixed_rel_diff_vs_f64": abs(mixed.E0 - plain.E0) / abs(plain.E0) if plain else None,
               "warm_rel_diff_vs_f64": abs(warm_r.E0 - plain.E0) / abs(plain.E0) if (plain and warm_r) else None},
        "products": {"f64": plain.iterations if plain else None, "mixed": mixed.iterations,
                     "mixed_f32": mixed.iterations_f32, "warm": warm_r.iterations if warm_r else None},
        "reorth_second_passes": {"f64": plain.reorth_second_passes if plain else None,
                                 "mixed": mixed.reorth_second_passes,
                                 "warm": warm_r.reorth_second_passes if warm_r else None},
        "warm": warm_info,
        "mixed_f64_columns": f64cols,
        "previous_solution_start": prev,
        "mixed_other_starts": starts,
        "basis_create_seconds": basis_seconds,
        "batched": batched,
        "odd": odd,
        "truncated": trunc,
        "eigenpairs": eigs,
        "scf": scf,
        "sigma": sig,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
