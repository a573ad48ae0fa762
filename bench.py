#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X: prints one JSON line.

Workload: the large random family at Omega=32, n=16 (601,080,390 states,
256 pair hops per row), eps ~ U[0, 32), G_ij = 0.3(1 + 0.2u), seed 0.

One step is one FP64 product y = Hx over the whole space (pd_sigma: unranking,
diagonal, every pair hop located by its rank, Sec. 3.3), the operation a
Lanczos iteration spends its time in (Sec. 5.3); FP64 is the paper's
arithmetic.  x is a seeded random vector already resident in HBM.  W untimed
products, then K timed products bracketed by device synchronisations, each
also timed by HIP events on the stream it runs on.

value = sigma non-zeros per second of the timed products (D * n(Omega-n) per
product).  Then, once each whatever --steps says, the three time-to-E0 solves
(pd_lanczos_ground to an FP64-checked residual of 1e-10 from a seeded random
start): plain FP64, mixed precision (FP32 products, FP64 everything else) and
the learned warm start (mixed precision from the network's product-state
start).  The roofline is that of the timed kernel (the FP64 product): HBM
bytes per launch from the committed rocprofv3 counter summary over its mean
HIP-event duration, against the 8 TB/s peak and the library's own streaming
kernels (achievable bandwidth).  The oracle's CPU rate on a bounded sample of
rows of the same instance is the CPU baseline.  Context legs (batched solver,
odd systems, self-consistent loop, truncated space, several eigenpairs, other
starts) follow under a wall-clock budget: a leg that would not fit is
recorded as skipped, a leg that fails as its error, and the JSON line is
printed in every case.
"""
import argparse
import json
import math
import os
import signal
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# 32-bit VALU lane operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (one wave64 instruction per SIMD every 4 cycles; an FMA counted as one op).
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic VALU work per non-zero of the prefix-delta product: target rank =
# rank + A + B (2 adds), up/down choice (compare + select), gather address,
# coefficient address, FMA.
OPS_PER_NONZERO = 7
METRIC = "sigma nonzeros/s + HBM GB/s; time-to-E0 at Omega=32,n=16, plain vs mixed vs warm"

T_START = time.perf_counter()
OUT = {}
_printed = False


def log(msg):
    print(f"[bench {time.perf_counter() - T_START:6.1f}s] {msg}", file=sys.stderr, flush=True)


def emit():
    global _printed
    if not _printed:
        _printed = True
        print(json.dumps(OUT), flush=True)


def _on_term(signum, frame):
    OUT.setdefault("error", f"terminated by signal {signum} before every leg ran")
    emit()
    sys.exit(1)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed FP64 products")
    ap.add_argument("--warmup", type=int, default=5, help="untimed FP64 products before them")
    ap.add_argument("--omega", type=int, default=32)
    ap.add_argument("--n", type=int, default=16)
    ap.add_argument("--krylov", type=int, default=20)
    ap.add_argument("--krylov-f64", type=int, default=0, help="Krylov size of the plain FP64 solve (0: --krylov)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--budget", type=float, default=420.0,
                    help="wall seconds after which no further context leg starts")
    ap.add_argument("--legs", default="all",
                    help="comma list of context legs to run (all, none, or names: " + ",".join(LEG_NAMES) + ")")
    ap.add_argument("--batched-count", type=int, default=4096)
    ap.add_argument("--cpu-rows", type=int, default=0, help="oracle sample size in rows (0: about 20 s of work)")
    ap.add_argument("--verbose", action="store_true", help="per-cycle progress of the solves on stderr")
    ap.add_argument("--kernel-only", action="store_true",
                    help="for counter runs: the library's 1 GiB copy kernel (the known-size reference), then "
                         "--sigma-reps FP32 and FP64 products of the workload, and exit")
    ap.add_argument("--trunc", action="store_true",
                    help="with --kernel-only: the truncated-space products (the space cut to 1e8 states, 1e8 "
                         "histogram bins, bitmap map) instead of the full ones")
    ap.add_argument("--sigma-reps", type=int, default=2)
    return ap.parse_args()


KERNEL_SOURCES = ["paper_2001_01978_amd/csrc/sigma_impl.h"]
COUNTERS = "sigma_omega{om}_n{n}_counters"
PIPELINE = "sigma_omega{om}_n{n}_pipeline_counters"
CLOCK_HZ, N_CU, N_SIMD = 2.4e9, 256, 1024


def code_tokens(text):
    """C++ source without its comments and with every run of whitespace
    collapsed to one space (string and character literals kept whole), so
    that an edit of comments or layout leaves the hash of the code alone."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash():
    """First 16 hex digits of the SHA-256 of the product kernel's code
    (comments and layout excluded): the counter summaries carry the hash of
    the source they were taken on."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(code_tokens(f.read()).encode())
    return h.hexdigest()[:16]


def counters_from_profiles(name):
    """'key: value' lines of the committed counter summary profiles/<name>.txt,
    or None when it is missing or was taken on a different kernel source."""
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
    return vals


def timed_products(torch, basis, eps, V, dt, reps, warmup, seed):
    """warmup + reps products y = Hx on the current stream: wall seconds of
    the reps (synchronised on both sides) and the HIP-event duration of
    each launch (events recorded between launches on that stream)."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    x = (torch.rand(basis.dim, dtype=torch.float64, device="cuda", generator=g) * 2 - 1).to(dt)
    y = torch.empty_like(x)
    for _ in range(warmup):
        basis.sigma(eps, V, x, y)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(reps):
        basis.sigma(eps, V, x, y)
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches = [ev[k].elapsed_time(ev[k + 1]) / 1e3 for k in range(reps)]
    del x, y
    torch.cuda.empty_cache()
    return wall, launches


def stream_probe(torch, pairdiag, gib=4, reps=5):
    """Achievable HBM bandwidth from the library's own streaming kernels
    (pd_stream_probe), event-timed over gib-GiB float buffers."""
    n = gib * (1 << 30) // 4
    a = torch.full((n,), 1.0, dtype=torch.float32, device="cuda")
    b = torch.full((n,), 2.0, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    out = {}
    for kind in ("read", "copy", "triad", "write"):
        for nt in (False, True):
            args = (a if kind != "write" else None, b if kind == "triad" else None, c)
            nbytes = pairdiag.stream_probe(kind, *args, nontemporal=nt)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                pairdiag.stream_probe(kind, *args, nontemporal=nt)
            e1.record()
            torch.cuda.synchronize()
            out[kind + ("_nontemporal" if nt else "")] = nbytes / (e0.elapsed_time(e1) / reps / 1e3) / 1e9
    del a, b, c
    torch.cuda.empty_cache()
    return out


def cpu_baseline(om, n, eps, V, rows_req):
    import numpy as np
    import oracle
    oracle.build(force=False)
    d = math.comb(om, n)
    K = n * (om - n)
    x = np.ones(d)              # values do not change the work; the full vector is needed for the gathers
    r0 = d // 3
    rows = rows_req or 200000
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
    rate = rows * K / dt
    return dict(value=rate, unit="nnz/s", cores=oracle.num_threads(), kind="oracle",
                sample=f"hash-search oracle sigma (states by '01' inversion, targets by the hash, FP64) over "
                       f"{rows} consecutive rows from rank {r0} of the same Omega={om}, n={n} instance "
                       f"({rows * K:.3e} non-zeros, {dt:.1f} s)",
                seconds_per_product_extrapolated=d * K / rate)


# ------------------------------------------------------------------ context legs

def leg_batched(ctx):
    import numpy as np
    from paper_2001_01978_amd import inputs, pairdiag
    cnt, tol = ctx["args"].batched_count, ctx["args"].tol
    insts = [inputs.family3_instance(s) for s in range(cnt)]
    dims = np.array([math.comb(i[0], i[1]) for i in insts])
    Ks = np.array([i[1] * (i[0] - i[1]) for i in insts])
    rb = pairdiag.lanczos_ground_batched(insts, krylov=20, tol=tol)   # includes the autotuner
    rb = pairdiag.lanczos_ground_batched(insts, krylov=20, tol=tol)   # tuned
    bnnz = float((rb.iterations * dims * Ks).sum())
    log(f"batched: {int(rb.converged.sum())}/{cnt} converged in {rb.info['kernel_seconds']:.2f} s")
    return dict(workload=f"{cnt} instances, omega ~ U{{10..24}}, n ~ U{{ceil(omega/4)..omega/2}}, "
                         f"eps ~ U[0,omega), G_ij = G0(1+0.2u), G0 ~ U[0.1,0.6), seeds 0..{cnt - 1}, FP64",
                sum_dim=int(dims.sum()), max_dim=int(dims.max()), converged=int(rb.converged.sum()),
                seconds=rb.info["kernel_seconds"], call_seconds=rb.info["seconds"],
                instances_per_s=cnt / rb.info["kernel_seconds"], products=int(rb.iterations.sum()),
                nnz_per_s=bnnz / rb.info["kernel_seconds"], block=rb.info["block"], teams=rb.info["teams"],
                team_size=rb.info["team_size"], team_instances=rb.info["large"],
                status=pairdiag._STATUS.get(rb.status))


def leg_odd(ctx):
    from paper_2001_01978_amd import inputs, pairdiag
    oo, on = 25, 12
    _, _, oeps, oV = inputs.c5_instance(oo, on, seed=0)
    okw = dict(krylov=20, tol=ctx["args"].tol, start="random", seed=1)
    pairdiag.lanczos_ground_odd(oo, on, oeps, oV, **okw)
    ro = pairdiag.lanczos_ground_odd(oo, on, oeps, oV, **okw)
    odim = math.comb(oo - 1, on)
    log(f"odd: E={ro.E:.12f} block {ro.block}, {ro.iterations} products in {ro.seconds:.2f} s")
    return dict(workload=f"odd system omega={oo}, {2 * on + 1} particles, all {oo} blocks of {on} pairs on "
                         f"{oo - 1} orbits (dim {odim} each), FP64, krylov 20",
                seconds=ro.seconds, products=ro.iterations, converged=ro.converged, E=ro.E, block=ro.block,
                nnz_per_s=ro.iterations * odim * on * (oo - 1 - on) / ro.seconds,
                status=pairdiag._STATUS.get(ro.status))


def leg_scf(ctx):
    from paper_2001_01978_amd import inputs, pairdiag
    so, sn = 24, 12
    _, _, seps, sV = inputs.c5_instance(so, sn, seed=0)
    u = inputs.uniform01(5, 0, so * so).reshape(so, so)
    sW = 0.3 * 0.5 * (u + u.T)
    sb = pairdiag.Basis(so, sn, store_states=False)
    res = dict(workload=f"Omega={so}, n={sn}, W = 0.3 (U + U^T)/2, mixing 0.6, field tol 1e-8, "
                        f"solve tol 1e-11, krylov 20")
    for reuse in (True, False):
        rs = pairdiag.scf_ground(sb, seps, sW, sV, mixing=0.6, tol=1e-8, krylov=20, start="random",
                                 reuse_psi=reuse, lanczos_tol=1e-11)
        res["previous_solution_start" if reuse else "random_start_each"] = dict(
            iterations=rs.info["iterations"], products=rs.info["products"], seconds=rs.info["seconds"],
            converged=bool(rs.info["converged"]), E0=rs.E0)
    log(f"scf: {res['previous_solution_start']['seconds']:.2f} s vs {res['random_start_each']['seconds']:.2f} s")
    return res


def leg_truncated(ctx):
    import torch
    from paper_2001_01978_amd import pairdiag
    om, n, eps, V, args = ctx["om"], ctx["n"], ctx["eps"], ctx["V"], ctx["args"]
    tl, tb = 100_000_000, 10**8
    if math.comb(om, n) <= tl:
        return dict(skipped=f"the space has at most {tl} states")
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
    del tbas
    torch.cuda.empty_cache()
    full = ctx.get("E0_mixed")
    log(f"truncated: kept {tinfo.kept}, sigma {tms}, solve {tg.iterations} products {tg.seconds:.2f} s")
    return dict(workload=f"Omega={om}, n={n} truncated to <= {tl} states, {tb} bins", kept=int(tinfo.kept),
                cut_bin=int(tinfo.cut_bin), cutoff=tinfo.cutoff, select_seconds=t1 - t0, build_seconds=t2 - t1,
                sigma=tms, solve_seconds=tg.seconds, products=tg.iterations, E0=tg.E0,
                E0_minus_full=(tg.E0 - full) if full is not None else None, converged=tg.converged)


def leg_eigenpairs(ctx):
    from paper_2001_01978_amd import pairdiag
    basis, eps, V, args = ctx["basis"], ctx["eps"], ctx["V"], ctx["args"]
    kw_e = dict(krylov=args.krylov, tol=args.tol, seed=1, want_psi=False)
    re4 = pairdiag.lanczos_eigs(basis, eps, V, 4, **kw_e)
    re1 = pairdiag.lanczos_eigs(basis, eps, V, 1, **kw_e)
    plain = ctx.get("plain")
    log(f"eigs: nev=4 {re4.iterations} products {re4.seconds:.2f} s; nev=1 {re1.iterations} products")
    return dict(nev4=dict(E=[float(e) for e in re4.E], products=re4.iterations, cycles=re4.restarts,
                          seconds=re4.seconds, max_residual=float(re4.residuals.max()), converged=re4.converged),
                nev1=dict(E=float(re1.E[0]), products=re1.iterations, seconds=re1.seconds,
                          E0_rel_diff_vs_f64=(abs(re1.E[0] - plain.E0) / abs(plain.E0)) if plain else None,
                          single_vector_restart_f64_products=plain.iterations if plain else None,
                          single_vector_restart_f64_seconds=plain.seconds if plain else None))


def leg_mixed_f64_columns(ctx):
    rc = ctx["solve"]("f32_f64cols")
    mixed = ctx["mixed"]
    log(f"mixed, FP64 columns: {rc.iterations} products {rc.seconds:.2f} s")
    return dict(seconds=rc.seconds, products=rc.iterations, products_f32=rc.iterations_f32,
                E0_rel_diff_vs_mixed=abs(rc.E0 - mixed.E0) / abs(mixed.E0))


def leg_other_starts(ctx):
    from paper_2001_01978_amd import pairdiag
    basis, eps, V, args, mixed = ctx["basis"], ctx["eps"], ctx["V"], ctx["args"], ctx["mixed"]
    res = {}
    for st in ("e1", "hf"):
        r_s = pairdiag.lanczos_ground(basis, eps, V, precision="f32", workspace=ctx["ws"], krylov=args.krylov,
                                      tol=args.tol, start=st, want_psi=False)
        res[st] = dict(seconds=r_s.seconds, products=r_s.iterations, converged=r_s.converged,
                       E0_rel_diff_vs_random=abs(r_s.E0 - mixed.E0) / abs(mixed.E0))
        log(f"start {st}: {r_s.iterations} products {r_s.seconds:.2f} s")
    return res


def leg_previous_solution(ctx):
    """The next problem of a self-consistent sweep: couplings x1.01, started
    from the converged state of the mixed solve, against a random start."""
    import numpy as np
    from paper_2001_01978_amd import pairdiag
    basis, eps, V, args, mixed = ctx["basis"], ctx["eps"], ctx["V"], ctx["args"], ctx["mixed"]
    if mixed.psi is None:
        return dict(skipped="no converged state kept")
    VB = np.asarray(V) * 1.01
    kw = dict(krylov=args.krylov, tol=args.tol, want_psi=False, precision="f32", workspace=ctx["ws"])
    rp = pairdiag.lanczos_ground(basis, eps, VB, x0=mixed.psi, **kw)
    rr = pairdiag.lanczos_ground(basis, eps, VB, start="random", seed=1, **kw)
    log(f"previous-solution start: {rp.iterations} products vs random {rr.iterations}")
    return dict(change="couplings x1.01", seconds_previous_start=rp.seconds, products_previous_start=rp.iterations,
                seconds_random_start=rr.seconds, products_random_start=rr.iterations,
                E0_rel_diff=abs(rp.E0 - rr.E0) / abs(rr.E0))


# (name, function, estimated seconds at Omega=32 n=16, scales with the product
# size).  The legs that use the solve workspace come before "eigenpairs",
# which needs a workspace of its own; the solve workspace is released first.
LEGS = [
    ("batched", leg_batched, 45, False),
    ("odd", leg_odd, 8, False),
    ("scf", leg_scf, 8, False),
    ("truncated", leg_truncated, 25, True),
    ("mixed_f64_columns", leg_mixed_f64_columns, 25, True),
    ("mixed_other_starts", leg_other_starts, 35, True),
    ("previous_solution_start", leg_previous_solution, 30, True),
    ("eigenpairs", leg_eigenpairs, 70, True),
]
LEG_NAMES = [l[0] for l in LEGS]


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the product would shard by row "
              "ranges with an all-gather of x per step); run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2001_01978_amd import inputs, pairdiag

    torch.cuda.set_device(0)
    om, n = args.omega, args.n
    _, _, eps, V = inputs.c5_instance(om, n, seed=0)
    K = n * (om - n)
    D = math.comb(om, n)

    if args.kernel_only:
        # The known-size reference for the counters: one copy of 1 GiB (read 1 GiB, write 1 GiB).
        src = torch.full((1 << 28,), 1.0, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        pairdiag.stream_probe("copy", src, None, dst)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
        if args.trunc:
            basis = pairdiag.Basis.truncated(om, n, eps, V, 100_000_000, 10**8)
            log(f"truncated space: {basis.dim} kept states")
        else:
            basis = pairdiag.Basis(om, n, store_states=False)
        for dt in (torch.float32, torch.float64):
            _, launches = timed_products(torch, basis, eps, V, dt, args.sigma_reps, 0, 7)
            log(f"{dt}: mean launch {1e3 * sum(launches) / len(launches):.3f} ms over {len(launches)}")
        log(f"kernel-only run done (kernel source {kernel_source_hash()})")
        return

    signal.signal(signal.SIGTERM, _on_term)
    OUT.update({
        "metric": METRIC, "value": None, "unit": "nnz/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64",
        "data": f"synthetic (seeded SplitMix64 instance, eps~U[0,{om}), G_ij=0.3(1+0.2u), V=-G; seeded random x)",
        "config": {"workload": f"sigma y=Hx in FP64 over the full Omega={om}, n={n} pairing space "
                               f"(dim {D}, {K} hops per row); one step = one product",
                   "omega": om, "n": n, "dim": D, "hops_per_row": K, "krylov": args.krylov, "tol": args.tol},
    })
    try:
        run(args, torch, np, inputs, pairdiag, om, n, eps, V, K, D)
    except Exception as e:          # the line is printed whatever failed
        import traceback
        traceback.print_exc()
        OUT["error"] = f"{type(e).__name__}: {e}"
    if OUT.get("value"):
        # Context only (another machine, another workload): the paper's CPU rate, 6.469e-8 CPU-seconds
        # per off-diagonal non-zero on an i7-7700K (Sec. 5.3), about 1.2e8 non-zeros/s of wall time on
        # its 8 threads.
        OUT["paper_context"] = {"nnz_per_s_wall_8_threads": 1.2e8, "nnz_per_cpu_second": 1.0 / 6.469e-8,
                                "hardware": "Intel i7-7700K, 8 threads, FP64",
                                "value_over_paper_wall_rate": OUT["value"] / 1.2e8}
    OUT["bench_seconds"] = time.perf_counter() - T_START
    emit()


def run(args, torch, np, inputs, pairdiag, om, n, eps, V, K, D):
    tb = time.perf_counter()
    basis = pairdiag.Basis(om, n, store_states=False)
    torch.cuda.synchronize()
    OUT["basis_create_seconds"] = time.perf_counter() - tb
    log(f"workload omega={om} n={n} dim={D} hops/row={K}")

    # ---- the timed steps: FP64 products
    wall, launches = timed_products(torch, basis, eps, V, torch.float64, args.steps, args.warmup, 11)
    avg64 = sum(launches) / len(launches)
    OUT["ms_per_step"] = wall / args.steps * 1e3
    OUT["value"] = D * K * args.steps / wall
    log(f"FP64 product: {OUT['ms_per_step']:.2f} ms/step (events {avg64 * 1e3:.2f} ms), {OUT['value']:.3e} nnz/s")
    # FP32 products (the mixed solve's kernel), same measure
    wall32, launches32 = timed_products(torch, basis, eps, V, torch.float32, args.steps, 2, 12)
    avg32 = sum(launches32) / len(launches32)
    log(f"FP32 product: {avg32 * 1e3:.2f} ms")

    # ---- achievable bandwidth (the library's streaming kernels)
    probes = stream_probe(torch, pairdiag)
    achievable = max(probes.values())
    log("stream probes: " + ", ".join(f"{k} {v:.0f}" for k, v in probes.items()) + " GB/s")

    pipe = counters_from_profiles(PIPELINE.format(om=om, n=n))

    def pipeline(avg, tag):
        # Busy fractions of the units that bound the product, from the per-launch SQ/TA/L1 counter totals
        # of the committed pipeline profile over this run's launch time (2.4 GHz; 256 texture addressers;
        # 1024 SIMDs, 4 cycles per wave64 VALU instruction).
        if not pipe or f"ta_busy_cycles_per_launch_{tag}" not in pipe:
            return None
        cyc = avg * CLOCK_HZ
        ta = float(pipe[f"ta_busy_cycles_per_launch_{tag}"])
        valu = float(pipe[f"valu_instructions_per_launch_{tag}"])
        vmem = float(pipe[f"vmem_read_instructions_per_launch_{tag}"])
        l1 = float(pipe[f"l1_accesses_per_launch_{tag}"])
        return {"ta_busy": ta / (N_CU * cyc), "valu_busy": valu * 4 / (N_SIMD * cyc),
                "ta_cycles_per_gather": ta / vmem, "l1_accesses_per_gather": l1 / vmem,
                "source": "profiles/" + PIPELINE.format(om=om, n=n) + ".txt"}

    def roof(avg, es, key_bytes, kernel):
        cnt = counters_from_profiles(COUNTERS.format(om=om, n=n))
        dram = float(cnt[key_bytes]) if cnt and key_bytes in cnt else None
        balg = D * (K * es + 2 * es)
        bmin = D * 2 * es
        ach = dram / avg / 1e9 if dram else None
        return {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": ach / PEAK_HBM_GBS if ach else None, "traffic": dram,
                "kernel": kernel, "avg_launch_ms": avg * 1e3, "launches_timed": args.steps,
                "achieved_is": "HBM bytes per launch (rocprofv3 FETCH_SIZE x copy-calibrated read scale + "
                               "WRITE_SIZE, profiles/" + COUNTERS.format(om=om, n=n) + ".txt) / mean HIP-event "
                               "launch time in this run; FETCH_SIZE counts every byte the L2s fetch from below "
                               "them, hits in the 256 MB Infinity Cache included, so it bounds true HBM traffic "
                               "from above",
                "achievable_GBps": achievable, "frac_of_achievable": ach / achievable if ach else None,
                "probes_GBps": probes,
                "algorithmic": {"gather_model_bytes": balg, "gather_model_GBps": balg / avg / 1e9,
                                "compulsory_bytes": bmin, "compulsory_GBps": bmin / avg / 1e9,
                                "hbm_over_compulsory": dram / bmin if dram else None,
                                "hbm_over_gather_model": dram / balg if dram else None},
                "valu": {"kind": "algorithmic: the lane operations per non-zero the method needs (hand count); "
                                 "pipeline.valu_busy is the measured issue",
                         "ops_per_nonzero": OPS_PER_NONZERO, "achieved_Tops": D * K * OPS_PER_NONZERO / avg / 1e12,
                         "peak_Tops": PEAK_VALU_TOPS,
                         "frac": D * K * OPS_PER_NONZERO / avg / 1e12 / PEAK_VALU_TOPS},
                "nnz_per_s": D * K / avg}

    OUT["roofline"] = roof(avg64, 8, "hbm_bytes_per_launch_f64", "sigma_kernel<uint32,double,16> (FP64 product)")
    OUT["roofline"]["pipeline"] = pipeline(avg64, "f64")
    OUT["roofline_f32"] = roof(avg32, 4, "hbm_bytes_per_launch_f32", "sigma_kernel<uint32,float,16> (FP32 product)")
    OUT["roofline_f32"]["pipeline"] = pipeline(avg32, "f32")

    # ---- time-to-E0: plain FP64, mixed, warm (once each)
    kf64 = args.krylov_f64 or args.krylov
    nb_mixed = pairdiag.workspace_bytes(basis, krylov=args.krylov, precision="f32")
    nb_f64 = pairdiag.workspace_bytes(basis, krylov=kf64, precision="f64")
    nb_f64c = pairdiag.workspace_bytes(basis, krylov=args.krylov, precision="f32_f64cols")
    free = torch.cuda.mem_get_info()[0]
    need = max(nb_mixed, nb_f64, nb_f64c if nb_f64c < free * 0.9 else 0)
    ws = pairdiag.device_buffer(need)

    def solve(precision, want_psi=False, krylov=None):
        return pairdiag.lanczos_ground(basis, eps, V, precision=precision, workspace=ws,
                                       krylov=krylov or args.krylov, tol=args.tol, start="random", seed=1,
                                       want_psi=want_psi, verbose=args.verbose)

    plain = solve("f64", krylov=kf64)
    log(f"plain FP64: E0={plain.E0:.12f} products={plain.iterations} {plain.seconds:.2f} s")
    mixed = solve("f32", want_psi=True)
    log(f"mixed: E0={mixed.E0:.12f} products={mixed.iterations} ({mixed.iterations_f32} f32) {mixed.seconds:.2f} s")
    warm_r, warm_info = None, None
    wpath = os.path.join(ROOT, "paper_2001_01978_amd", "weights", f"warm_o{om}_n{n}.npz")
    if os.path.exists(wpath):
        from paper_2001_01978_amd import warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        net = warm.WarmNet.load(wpath)
        lo = net.logits(om, eps, V)
        x0 = basis.warm_start(torch.tensor(lo, dtype=torch.float32))
        warm_r = pairdiag.lanczos_ground(basis, eps, V, x0=x0, fallback=True, precision="f32", workspace=ws,
                                         krylov=args.krylov, tol=args.tol, want_psi=False, verbose=args.verbose)
        torch.cuda.synchronize()
        warm_info = dict(weights=os.path.relpath(wpath, ROOT), seconds_including_network=time.perf_counter() - t,
                         fallback_used=warm_r.fallback_used)
        del x0
        log(f"warm: E0={warm_r.E0:.12f} products={warm_r.iterations} {warm_info['seconds_including_network']:.2f} s")
    OUT["time_to_E0_s"] = {"f64": plain.seconds, "mixed": mixed.seconds,
                           "warm": warm_info["seconds_including_network"] if warm_info else None}
    OUT["time_to_E0_workload"] = (f"pd_lanczos_ground, Omega={om}, n={n}, krylov {args.krylov} (FP64: {kf64}), "
                                  f"tol {args.tol:g} (FP64-checked residual), random start seed 1")
    OUT["E0"] = {"f64": plain.E0, "mixed": mixed.E0, "warm": warm_r.E0 if warm_r else None,
                 "mixed_rel_diff_vs_f64": abs(mixed.E0 - plain.E0) / abs(plain.E0),
                 "warm_rel_diff_vs_f64": abs(warm_r.E0 - plain.E0) / abs(plain.E0) if warm_r else None}
    OUT["residual"] = {"f64": plain.residual, "mixed": mixed.residual, "warm": warm_r.residual if warm_r else None}
    OUT["products"] = {"f64": plain.iterations, "mixed": mixed.iterations, "mixed_f32": mixed.iterations_f32,
                       "warm": warm_r.iterations if warm_r else None}
    OUT["solve_product_seconds"] = {"f64": plain.sigma_seconds_f64,
                                    "mixed_f64": mixed.sigma_seconds_f64, "mixed_f32": mixed.sigma_seconds_f32}
    OUT["reorth_second_passes"] = {"f64": plain.reorth_second_passes, "mixed": mixed.reorth_second_passes,
                                   "warm": warm_r.reorth_second_passes if warm_r else None}
    OUT["warm"] = warm_info
    OUT["solve_nnz_per_s"] = {"f64": plain.iterations * D * K / plain.seconds,
                              "mixed": mixed.iterations * D * K / mixed.seconds}

    # ---- the oracle on the host cores
    log("cpu baseline (oracle) ...")
    try:
        cpu = cpu_baseline(om, n, eps, V, args.cpu_rows)
        cpu["time_to_E0_f64_s_extrapolated"] = cpu["seconds_per_product_extrapolated"] * plain.iterations
        cpu["extrapolation"] = ("per-product seconds from the sampled rate x the products of the GPU plain-FP64 "
                                "solve (extrapolated, not run)")
        OUT["cpu_baseline"] = cpu
        log(f"cpu baseline: {cpu['value']:.3e} nnz/s on {cpu['cores']} threads")
    except Exception as e:
        OUT["cpu_baseline"] = {"error": f"{type(e).__name__}: {e}"}

    # ---- context legs under the budget
    want = set(LEG_NAMES) if args.legs == "all" else (set() if args.legs == "none" else set(args.legs.split(",")))
    ctx = dict(args=args, om=om, n=n, eps=eps, V=V, basis=basis, ws=ws, solve=solve, plain=plain, mixed=mixed,
               E0_mixed=mixed.E0)
    scale = D * K / (601080390 * 256)
    for name, fn, est, scales in LEGS:
        if name == "eigenpairs":
            mixed.psi = None
            ctx["ws"] = ws = None
            torch.cuda.empty_cache()
        if name not in want:
            OUT[name] = {"skipped": "not requested"}
            continue
        est_s = est * max(scale, 1.0) if scales else est
        left = args.budget - (time.perf_counter() - T_START)
        if est_s > left:
            OUT[name] = {"skipped": f"time budget: {left:.0f} s left, the leg takes about {est_s:.0f} s"}
            log(f"{name}: skipped ({left:.0f} s left)")
            continue
        try:
            OUT[name] = fn(ctx)
        except Exception as e:
            OUT[name] = {"error": f"{type(e).__name__}: {e}"}
            log(f"{name}: {type(e).__name__}: {e}")
            torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
