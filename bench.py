"""Benchmark: one step = one whole pass of the path (occupancy scan, block Grams reduced into G,
FP64 eigensolve, rank-safe threshold, back-projection of V) through ranky_svd on one synthetic
power-law matrix resident in HBM.  Prints ONE JSON line.

Default workload: 1024 x 2^20, ~1.01M nnz, Zipf(1.1) row degrees, N(0,1) FP64 values,
64 column blocks (8 with 30% of rows emptied inside the block), top k = 128, FP64 path.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", choices=["fp64", "fp32", "bf16x3"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 256-matrix leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-seconds", type=float, default=4.0)
    ap.add_argument("--no-other", action="store_true", help="skip the other-precision leg of the headline matrix")
    ap.add_argument("--powerlaw-200m", action="store_true",
                    help="also time config 5 (4096 x 2^24, ~200M nnz, mixed path; generation takes ~25-60 s)")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="only run a device-to-device copy of this many GiB (counter calibration) and exit")
    return ap.parse_args()


# HBM bytes per working launch of k_jround on the 1M power-law FP64 leg, from two rocprofv3 counter
# runs (FETCH_SIZE and WRITE_SIZE, KiB per dispatch, averaged over the launches that did work),
# each scaled by what the same counter reads back for a plain device copy of 1 GiB (x2.0 for
# FETCH_SIZE, x1.0 for WRITE_SIZE).  Valid only for the kernel source it was taken on.
JROUND_TRAFFIC = {"bytes": (6778.62 * 2.0 + 15473.13) * 1024, "source": "k_jacobi.hip",
                  "source_sha256": "fc714e93f5894848e58f024434390430ad3155f9b849fb6a2a593d53dc8f4f0d"}
# The same for k_backproject on that leg (FP64 V, 32 workgroups per CU): the CSC, U and V.
BACKPROJECT_TRAFFIC = {"bytes": (13605.64 * 2.0 + 1048841.05) * 1024, "source": "k_select.hip",
                       "source_sha256": "10ec62b8b56e6f7f358da962eb913eaae2dca55ea1235111e7c3b02a437fe775"}


def counted_traffic(entry):
    """The counted bytes per launch, or None once the kernel's source differs from the one counted."""
    import hashlib

    src = os.path.join(ROOT, "paper_2009_09767_amd", "csrc", entry["source"])
    with open(src, "rb") as f:
        ok = hashlib.sha256(f.read()).hexdigest() == entry["source_sha256"]
    return entry["bytes"] if ok else None


def jround_flops(n):
    """Algorithmic FP64 flops of the Jacobi round launches of one sweep on an n x n Gram, per
    launch.  npad = 32 ceil(n / 32), P = npad / 32 subproblems per round, nb = 2P launches.
    Update (rounds 1..nb-1): the P(P-1)/2 off-diagonal 32 x 32 tiles of G take two 32^3
    products (J_a^T G_ab J_b, the mirror tile is a copy), the npad/32 x P tiles of W one
    (W J): 2 * 32^3 flops per product.  Solve (rounds 0..nb-2), per subproblem: the build
    (32 x 32 x 16 and 16 x 32 x 16 products) and the steps of the subproblem sweep, 31 in
    the full rounds (every max(1, (nb-1) // 4)-th round from round 0) and 16 (cross pairs
    only) in the others; a step is 120 off-diagonal 2 x 2 two-sided rotations (24 flops),
    16 diagonal ones (12), 16 x 32 J-row rotations (6) and 16 rotation angles (about 20)."""
    npad = 32 * ((n + 31) // 32)
    P = npad // 32
    nb = 2 * P
    gemm = 2 * 32 ** 3
    upd = (P * (P - 1) // 2) * 2 * gemm + (npad // 32) * P * gemm
    build = 2 * 32 * 32 * 16 + 2 * 16 * 32 * 16
    step = 120 * 24 + 16 * 12 + 16 * 32 * 6 + 16 * 20
    period = max(1, (nb - 1) // 4)
    solve = sum(P * (build + (31 if r % period == 0 else 16) * step) for r in range(nb - 1))
    return ((nb - 1) * upd + solve) / nb


def copy_calibration(gib):
    """A plain device copy of known size, run under the same counters as the kernels."""
    import torch

    n = int(gib * 2**30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": 8 * n, "launches": 3}), flush=True)


def spmm_bytes(nnz, N, k, M, val_bytes, out_bytes):
    """Algorithmic HBM bytes of the back-projection: CSC read once (rowidx + values + colptr),
    U read once, V written once."""
    return nnz * (4 + val_bytes) + 4 * (N + 1) + N * k * out_bytes + M * k * 8


def time_path(ranky, torch, np, dA, A, k, D, prec, steps, warmup):
    """Wall time per ranky_svd call (host clock around synchronised calls) and the
    per-phase times from the library's HIP events on the same stream."""
    vdt = torch.float64 if prec == "fp64" else torch.float32
    kw = dict(n_blocks=D, gram_prec=prec, v_dtype=vdt)
    opts = ranky.make_opts(**kw)
    ws = torch.empty(ranky.workspace_bytes(A.M, A.N, A.nnz, k, opts), dtype=torch.uint8, device="cuda:0")
    out = ranky.SVDResult(torch.empty(k, dtype=torch.float64, device="cuda:0"),
                          torch.empty((A.M, k), dtype=torch.float64, device="cuda:0"),
                          torch.empty((A.N, k), dtype=vdt, device="cuda:0"), {})
    ctx = ranky.context(0)
    # a stream of our own, so the Jacobi sweep can be replayed as a captured HIP graph
    stream = torch.cuda.Stream()
    kw["graph"] = True
    with torch.cuda.stream(stream):
        # launch shapes picked by measurement on this matrix, before (and outside) the timed region
        tune = ranky.autotune(dA, k, ctx=ctx, out=out, workspace=ws, stream=stream, **kw)
        for _ in range(warmup):
            ranky.svd(dA, k, 0.0, ctx=ctx, out=out, workspace=ws, stream=stream, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ranky.svd(dA, k, 0.0, ctx=ctx, out=out, workspace=ws, stream=stream, **kw)
        torch.cuda.synchronize()
        ms_step = 1e3 * (time.perf_counter() - t0) / steps
        phases = np.zeros(8)
        round_ms, round_launches = 0.0, 0
        for _ in range(steps):
            r = ranky.svd(dA, k, 0.0, ctx=ctx, out=out, workspace=ws, stream=stream, timing=True, **kw)
            phases += np.array(r.info["ms"])
            round_ms += r.info["round_ms"]
            round_launches += r.info["round_launches"]
    phases /= steps
    names = ["occupancy", "transpose", "gram", "eigensolve", "select", "refine", "backproject", "total"]
    info = dict(r.info)
    info["autotune"] = tune
    info["round_us_avg"] = 1e3 * round_ms / max(round_launches, 1)
    info["round_launches_per_call"] = round_launches / steps
    return ms_step, dict(zip(names, phases.tolist())), info, out.sigma.cpu().numpy(), vdt


def time_batch(ranky, torch, gen, steps, warmup):
    """Batched leg: 256 independent matrices (M ~ U{32..512}, N ~ U{1e4..1e5}, density 0.5%,
    FP32 values, 20% with half their rows zeroed), full spectrum each, through ranky_batch
    with the Jacobi sweep replayed as a captured graph.  FP64 Gram and FP32 Gram."""
    mats = gen.batch_mixed()
    dms = [ranky.to_device(A, "cuda:0") for A in mats]
    ks = [A.M for A in mats]
    Ds = [int(A.meta["D"]) for A in mats]
    nnz = sum(A.nnz for A in mats)
    stream = torch.cuda.Stream()
    out = {"workload": "batch of 256 matrices, M~U{32..512}, N~U{1e4..1e5}, density 0.5%, 20% half-rank, full spectrum",
           "matrices": len(mats), "nnz": nnz}
    for prec, vdt in (("fp64", torch.float64), ("fp32", torch.float32)):
        outs = [ranky.SVDResult(torch.empty(k, dtype=torch.float64, device="cuda:0"),
                                torch.empty((A.M, k), dtype=torch.float64, device="cuda:0"),
                                torch.empty((A.N, k), dtype=vdt, device="cuda:0"), {}) for A, k in zip(mats, ks)]
        ws = torch.empty(ranky.batch_workspace_bytes(dms, ks, gram_prec=prec, v_dtype=vdt, n_blocks=Ds),
                         dtype=torch.uint8, device="cuda:0")
        with torch.cuda.stream(stream):
            for _ in range(warmup):
                ranky.batch(dms, ks, 0.0, n_blocks=Ds, outs=outs, workspace=ws, gram_prec=prec, v_dtype=vdt, graph=True)
            stream.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                ranky.batch(dms, ks, 0.0, n_blocks=Ds, outs=outs, workspace=ws, gram_prec=prec, v_dtype=vdt, graph=True)
            stream.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        out[prec + "_gram"] = {"ms_per_batch": ms, "value": nnz / (ms * 1e-3), "unit": "nnz/s",
                               "max_sweeps": max(o.info["sweeps"] for o in outs),
                               "ranks_ok": all(o.info["status"] == 0 for o in outs)}
        del outs, ws
        torch.cuda.empty_cache()
    return out


def time_powerlaw_200m(ranky, torch, np, gen, steps, warmup):
    """Config 5: one large matrix (4096 x 2^24, Zipf(1.2) rows capped at N, ~200M nnz, FP32
    values, 256 column blocks, k = 100) through the mixed path (FP32 Gram, FP64 eigensolve and
    Rayleigh-Ritz, FP32 V), inputs resident in HBM."""
    A = gen.powerlaw_200m(progress=lambda m: print(m, file=sys.stderr, flush=True))
    dA = ranky.to_device(A, "cuda:0")
    k, D = A.meta["k"], A.meta["D"]
    kw = dict(n_blocks=D, gram_prec="fp32", refine=1, v_dtype=torch.float32)
    out = ranky.SVDResult(torch.empty(k, dtype=torch.float64, device="cuda:0"),
                          torch.empty((A.M, k), dtype=torch.float64, device="cuda:0"),
                          torch.empty((A.N, k), dtype=torch.float32, device="cuda:0"), {})
    ctx = ranky.context(0)
    ws = torch.empty(ranky.workspace_bytes(A.M, A.N, A.nnz, k, ranky.make_opts(**kw)), dtype=torch.uint8,
                     device="cuda:0")
    for _ in range(warmup):
        ranky.svd(dA, k, 0.0, ctx=ctx, out=out, workspace=ws, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ranky.svd(dA, k, 0.0, ctx=ctx, out=out, workspace=ws, **kw)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    r = ranky.svd(dA, k, 0.0, ctx=ctx, out=out, workspace=ws, timing=True, **kw)
    names = ["occupancy", "transpose", "gram", "eigensolve", "select", "refine", "backproject", "total"]
    res = {"workload": f"power-law CSC M={A.M} N={A.N} nnz={A.nnz} Zipf(1.2) D={D} k={k} mixed (fp32 gram, fp64 eig+RR, fp32 V)",
           "value": A.nnz / (ms * 1e-3), "unit": "nnz/s", "ms_per_step": ms, "steps": steps,
           "phase_ms": dict(zip(names, [round(x, 4) for x in r.info["ms"]])), "rank": r.info["rank"],
           "sweeps": r.info["sweeps"]}
    del out, ws, dA
    torch.cuda.empty_cache()
    return res


def time_serving(ranky, torch, gen, seconds, pool_size=48, slots=8):
    """Serving leg: the open-loop Poisson arrivals (200 req/s) replayed for `seconds`, each
    arrival drawing the next matrix of a seeded pool of serving requests (M in {128..1024},
    N = 2^U{14..20}, LogUniform nnz up to 20M, Zipf(1.1) rows, FP32 values, k = min(M, 64)).
    Latency = completion - submit through ranky_serve_*.  Requests that share a pool entry
    share its output buffers (identical results)."""
    reqs = gen.serving_requests()
    pool = [gen.serving_matrix(r) for r in reqs[:pool_size]]
    dpool = [ranky.to_device(A, "cuda:0") for A in pool]
    arrivals = [r.arrival_s for r in reqs if r.arrival_s < seconds]
    res = {"workload": f"serving: Poisson 200 req/s for {seconds:g} s over a pool of {pool_size} requests",
           "requests": len(arrivals), "slots": slots}
    for prec in ("fp64", "fp32"):
        vdt = torch.float64 if prec == "fp64" else torch.float32
        outs = [ranky.SVDResult(torch.empty(min(A.M, 64), dtype=torch.float64, device="cuda:0"),
                                torch.empty((A.M, min(A.M, 64)), dtype=torch.float64, device="cuda:0"),
                                torch.empty((A.N, min(A.M, 64)), dtype=vdt, device="cuda:0"), {}) for A in pool]
        srv = ranky.Server(arena_bytes=16 << 30, max_slots=slots, max_queue=4096, gram_prec=prec, v_dtype=vdt,
                           refine=0 if prec == "fp64" else 1)
        # warm every pool entry once (kernel loading, allocator)
        for i in range(0, pool_size, 8):
            ts = [srv.submit(dpool[j], min(pool[j].M, 64), outs[j])[1] for j in range(i, min(i + 8, pool_size))]
            for t in ts:
                srv.wait(t)
        srv.close()
        srv = ranky.Server(arena_bytes=16 << 30, max_slots=slots, max_queue=4096, gram_prec=prec, v_dtype=vdt,
                           refine=0 if prec == "fp64" else 1)
        t0 = time.perf_counter()
        tickets, busy = [], 0
        for i, ta in enumerate(arrivals):
            now = time.perf_counter() - t0
            if ta > now:
                time.sleep(ta - now)
            j = i % pool_size
            st, t = srv.submit(dpool[j], min(pool[j].M, 64), outs[j])
            if st == ranky.OK:
                tickets.append(t)
            else:
                busy += 1
        bad = sum(1 for t in tickets if srv.wait(t)[0] != ranky.OK)
        st = srv.stats()
        srv.close()
        res[prec + "_gram"] = {"p50_ms": st["p50_us"] / 1e3, "p99_ms": st["p99_us"] / 1e3,
                               "mean_ms": st["mean_us"] / 1e3, "req_per_s": st["req_per_s"],
                               "nnz_per_s": st["nnz_per_s"], "completed": st["completed"], "failed": bad,
                               "rejected": busy, "peak_running": st["peak_running"],
                               "arena_peak_gb": st["arena_peak_bytes"] / 2**30}
        del outs
        torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the path runs on one GPU (no collectives); --gpus above 1 is not supported"}))
        sys.exit(2)
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return
    import numpy as np
    import torch

    from paper_2009_09767_amd import gen, ranky

    A = gen.powerlaw_1m(seed=args.seed)
    k, D = 128, 64
    dA = ranky.to_device(A, "cuda:0")
    ms_step, phases, info, sig64, vdt = time_path(ranky, torch, np, dA, A, k, D, args.prec, args.steps, args.warmup)
    # the other precisions of the same workload (FP32 Gram and split-bf16 dense tiles, both
    # with the FP64 Rayleigh-Ritz step), reported beside the headline
    others = [p for p in ("fp64", "fp32", "bf16x3") if p != args.prec]
    other_res = {}
    if not args.no_other:
        for p in others:
            other_res[p] = time_path(ranky, torch, np, dA, A, k, D, p, args.steps, args.warmup)

    val_bytes = 8 if A.values.dtype == np.float64 else 4
    out_bytes = 8 if vdt == torch.float64 else 4
    sb = spmm_bytes(A.nnz, A.N, k, A.M, val_bytes, out_bytes)
    spmm_ms = float(phases["backproject"])
    achieved = sb / (spmm_ms * 1e-3) / 1e9
    # the dominant kernel: the Jacobi round (FP64 matrix cores for the update, FP64 ALU for the solve)
    jf = jround_flops(info["n_nonempty"])
    jr_tfs = jf / (info["round_us_avg"] * 1e-6) / 1e12

    line = {
        "metric": "nnz/s, full sparse SVD at stated sigma error vs FP64 path",
        "value": A.nnz / (ms_step * 1e-3),
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32-gram/f64-eig", "bf16x3": "bf16x3-gram/f64-eig"}[args.prec],
        "data": "synthetic",
        "config": {"workload": f"power-law CSC M={A.M} N={A.N} nnz={A.nnz} Zipf(1.1) D={D} k={k} "
                               f"gram={args.prec}", "M": A.M, "N": A.N, "nnz": A.nnz, "n_blocks": D, "k": k},
        "rank": info["rank"],
        "sweeps": info["sweeps"],
        "autotune": info["autotune"],
        "phase_ms": phases,
        "roofline": {"kernel": "k_jround (Jacobi round: subproblem sweep + FP64 MFMA tile update)",
                     "bound": "mfma", "achieved": jr_tfs, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": jr_tfs / FP64_PEAK_TFS, "traffic": counted_traffic(JROUND_TRAFFIC), "flops_per_launch": jf,
                     "avg_launch_us": info["round_us_avg"], "launches_per_step": info["round_launches_per_call"],
                     "dtype": "fp64"},
        "roofline_spmm": {"kernel": "k_backproject (V = A^T U Sigma^-1)", "bound": "hbm", "achieved": achieved,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                          "traffic": counted_traffic(BACKPROJECT_TRAFFIC),
                          "bytes_per_launch": sb},
    }
    for p, (ms2, phases2, info2, sig2, vdt2) in other_res.items():
        line[p + "_path"] = {"value": A.nnz / (ms2 * 1e-3), "ms_per_step": ms2, "phase_ms": phases2,
                             "rank": info2["rank"], "sweeps": info2["sweeps"]}

    if not args.no_batch:
        line["batch"] = time_batch(ranky, torch, gen, max(2, args.steps // 3), 1)
    if not args.no_serve:
        line["serving"] = time_serving(ranky, torch, gen, args.serve_seconds)
    if args.powerlaw_200m:
        line["powerlaw_200m"] = time_powerlaw_200m(ranky, torch, np, gen, max(2, args.steps // 3), 1)

    if not args.no_cpu_baseline:
        import oracle

        # the oracle's OpenMP loops run OMP_NUM_THREADS threads (all cores of the affinity mask if unset)
        cores = len(os.sched_getaffinity(0))
        if os.environ.get("OMP_NUM_THREADS", "").isdigit():
            cores = min(cores, max(1, int(os.environ["OMP_NUM_THREADS"])))
        # the whole workload, repeated until at least 10 s of CPU work (at most 30 passes)
        reps, t_cpu = 0, 0.0
        while reps < 30 and (reps == 0 or t_cpu < 10.0):
            t0 = time.perf_counter()
            ref = oracle.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=k, method="gram", want_v=True)
            t_cpu += time.perf_counter() - t0
            reps += 1
        r = ref.rank
        line["cpu_baseline"] = {"value": reps * A.nnz / t_cpu, "unit": "nnz/s", "cores": cores, "kind": "oracle",
                                "sample": "the whole workload, %d passes: FP64 sparse Gram + cyclic Jacobi + V "
                                          "(Gram route)" % reps,
                                "seconds": t_cpu}
        line["sigma_rel_err_vs_oracle"] = float(np.max(np.abs(sig64[:r] - ref.sigma[:r]) / ref.sigma[:r]))
        for p, res in other_res.items():
            sig2 = res[3]
            line[p + "_path"]["sigma_rel_err_vs_oracle"] = float(np.max(np.abs(sig2[:r] - ref.sigma[:r]) / ref.sigma[:r]))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
