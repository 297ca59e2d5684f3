"""Benchmark: effective GF(2) bit-ops/s of the 65536 x 65536 decomposition on one MI355X.

One step = one call of gf2_decompose on a device-resident 65536 x 65536
Bernoulli(1/2) matrix (512 MB bit-packed), writing L, E, the permutation, the
pivot columns and the rank.  Effective bit-ops = 2 * sum_t (n-1-t)(m-1-p_t)
(one AND and one XOR per multiply-add of textbook elimination, from the pivot
columns p_t the run returns); value = effective bit-ops / seconds per step.

The timed steps run with the library's profiling off (events between steps
give min / median); a separate instrumented pass of --profile-steps steps then
measures the dominant kernel (the trailing-update Four-Russians product): each
of its launches records its own start and end (HIP events on the launch
stream) and its lookup count; its algorithmic work is one 8-byte LDS table
read and one 64-bit XOR per table lookup (one lookup per output word per 8
inner bits); the bound is the on-chip table-read rate: LDS reads of 256 B/clk
per CU (gfx950) x 256 CUs x 2.4 GHz = 157.3 TB/s.

cpu_baseline: the CPU oracle (plain elimination, OpenMP) timed on a bounded
sample of the same workload (dense matrices of the same distribution, the
largest size that fits the time budget, repeated to about ten seconds),
expressed in the same unit.

batched: the 4096-matrix workload (sides uniform in [64, 2048], density 1/2 or
1/10, half with a planted rank, one random right-hand side each) factored by
gf2_decompose_batched and solved by gf2_solve_batched, timed with HIP events
over `--batch-steps` passes with the inputs resident; reported as matrices/s,
solves/s (decomposition + solve per system) and effective bit-ops/s, beside one
gf2_decompose call per matrix on the same GPU (same outputs, checked equal).

serving: a stream of rank / solve / decompose requests (square sides
log-uniform in [128, 16384] or 1:4 rectangles, Bernoulli(1/2), data in pinned
host memory until admitted) through the continuous-batching loop of
paper_1209_5198_amd/serve.py under a 64 GB admission cap: first all requests at
once (saturated throughput), then Poisson arrivals at 50/80/95% of that rate,
each reported with p50/p99 latency, requests/s and solves/s.

configs: the other single-matrix configurations on the same GPU (one 2048^2
decomposition, the 16384^3 product, the 16384^2 decomposition and the planted
rank-20000 32768 x 65536 decomposition), HIP-event timed, inputs resident.

HBM traffic of that kernel is read from rocprofv3 counters (FETCH_SIZE and
WRITE_SIZE, separate runs); --copy-calibration runs only a plain 1 GiB device
copy, whose counter readings give the scale factor between counter units and
bytes.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n N] [--copy-calibration]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

# Hardware queues per process for the HIP runtime (read when it starts): the
# serving sessions run up to 4 large requests concurrently, each with its own
# pipeline stream pair, plus the batch and copy streams; with the default 4
# queues, waits of unrelated streams that share a queue serialise them.  Set
# outright: an inherited default of 4 would otherwise win.
os.environ["GPU_MAX_HW_QUEUES"] = "16"

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "effective GF(2) bit-ops/s for 65536² decompose; batched solves/s + p99 latency"
PAPER_BITOPS_PER_S = 1.876e14 / 86.156   # paper's best 65536^2 time (Table 4, b = 128, recursive), context
LDS_PEAK_TBS = 256 * 256 * 2.4e9 / 1e12   # 157.3 TB/s: 256 CUs x 256 B/clk x 2.4 GHz
# HBM bytes per product launch in this decomposition, from rocprofv3 counters:
# FETCH_SIZE (KiB per dispatch, x2: a plain 1 GiB copy reads 524305 KiB) and
# WRITE_SIZE (KiB, x1: the copy writes 1048576 KiB), averaged over the 253
# product launches of one 65536^2 decomposition (four decompositions counted).
# Valid only for the product kernel source they were measured on.
TRAFFIC = {"kernel_source_sha256": "33e40c7051b76f206a87d0ce4e69bc76b0ed3b66db79e5eb967367a223cd5711",
           "fetch_bytes": 62864.12 * 2 * 1024, "write_bytes": 93206.40 * 1024}
SEED = 65536
# The oracle on the bench's own 65536^2 input (seed 65536), run once on the
# whole matrix (about 7e11 word operations, minutes of CPU time, so this script
# does not repeat it): 43.2 s with 16 threads on a GPU host; 186.4 s with the
# 8 threads of the build host when tests/golden/make_fullsize_hashes.py wrote
# the digests (its record holds the time and thread count).
ORACLE_65536_ONCE = [{"s": 43.2, "cores": 16, "host": "GPU host (MI355X box)"},
                     {"s": 186.4, "cores": 8, "host": "build host (tests/golden/fullsize_hashes.json)"}]


def eff_bitops(n: int, m: int, pivcols: np.ndarray) -> float:
    p = pivcols[pivcols >= 0].astype(np.float64)
    t = np.arange(p.size, dtype=np.float64)
    return float(2.0 * np.sum((n - 1 - t) * (m - 1 - p)))


def cpu_baseline(budget_s: float = 24.0, min_s: float = 10.0):
    """Time the oracle on a bounded dense sample: sizes double from 2048 while the
    next one is predicted (16x the time) to fit budget_s, then the largest size is
    repeated on fresh matrices until min_s seconds of oracle time are reached."""
    import oracle
    from paper_1209_5198_amd import synth

    oracle.build()
    n = 2048
    stream = 7
    while True:
        A = synth.dense(SEED, stream, n, n)
        t0 = time.perf_counter()
        res = oracle.ple(A, n, n, want_le=False)
        dt = time.perf_counter() - t0
        if dt * 16 > budget_s or n >= 65536:
            break
        n *= 2
    total_t, total_ops, runs, ranks = dt, eff_bitops(n, n, res["pivcols"]), 1, [res["rank"]]
    while total_t < min_s:
        stream += 1
        A = synth.dense(SEED, stream, n, n)
        t0 = time.perf_counter()
        res = oracle.ple(A, n, n, want_le=False)
        total_t += time.perf_counter() - t0
        total_ops += eff_bitops(n, n, res["pivcols"])
        runs += 1
        ranks.append(res["rank"])
    return {"value": total_ops / total_t, "unit": "bit-ops/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"oracle PLE (plain elimination) of {runs} Bernoulli(1/2) {n}x{n} matrices "
                      f"(seed {SEED}, streams {stream - runs + 1}..{stream}), {total_t:.2f} s, ranks {ranks}"}


BATCH_SEED, BATCH_COUNT = 4096, 4096


def batched_section(gf2, synth, steps: int, per_matrix: bool = True):
    """The batched workload: device-resident batch, decomposition + solve per pass."""
    import concurrent.futures

    import torch

    wpr = synth.wpr
    t0 = time.perf_counter()
    specs = synth.batch_specs(BATCH_SEED, BATCH_COUNT)
    with concurrent.futures.ThreadPoolExecutor(16) as ex:
        kinds = list(ex.map(lambda s: synth.batch_matrix(BATCH_SEED, s), specs))
    shapes = [(s["n"], s["m"]) for s in specs]
    b = gf2.Batch(shapes)
    b.set_matrices([k[1] if k[0] == "iid" else np.zeros((s["n"], wpr(s["m"])), np.uint64)
                    for k, s in zip(kinds, specs)])
    for k, s in zip(kinds, specs):  # planted products X*Y formed on the GPU
        if k[0] == "planted":
            n, m, r = s["n"], s["m"], s["r"]
            gf2.gf2_matmul(b.mat_view(s["i"]), gf2.Mat.from_rowmajor(k[1], n, r), gf2.Mat.from_rowmajor(k[2], r, m))
    b.set_rhs([synth.batch_rhs(BATCH_SEED, s) for s in specs])
    del kinds
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_dec = timed(lambda: b.decompose(stream=stream), steps)
    ms_solve = timed(lambda: b.solve(stream=stream), steps)
    ms_rank = timed(lambda: b.decompose(want_le=False, stream=stream), steps)
    b.decompose(stream=stream)
    b.solve(stream=stream)
    torch.cuda.synchronize()
    h = b.fetch()
    ops = 0.0
    for i, (n, m) in enumerate(shapes):
        o = b.off[i]["c"]
        ops += eff_bitops(n, m, h["pivcols"][o:o + min(n, m)])
    out = {"workload": f"{BATCH_COUNT} matrices, n and m uniform in [64, 2048], Bernoulli(1/2 or 1/10), "
                       "half planted rank, one rhs each; seed %d" % BATCH_SEED,
           "steps": steps, "ms_decompose": ms_dec, "ms_solve": ms_solve, "ms_rank_only": ms_rank,
           "matrices_per_s": BATCH_COUNT / (ms_dec / 1e3),
           "solves_per_s": BATCH_COUNT / ((ms_dec + ms_solve) / 1e3),
           "eff_bitops_per_s": ops / (ms_dec / 1e3), "eff_bitops_per_pass": ops,
           "consistent_systems": int(h["consistent"][:BATCH_COUNT].sum()), "setup_s": round(setup_s, 1)}
    if per_matrix:
        keep = {k: h[k].copy() for k in ("L", "E", "perm", "pivcols", "rank")}

        def one_by_one():
            for i, (n, m) in enumerate(shapes):
                k = min(n, m)
                o = b.off[i]
                L = gf2.Mat(b.L[o["l"]:o["l"] + max(n * wpr(k), 1)], n, k, max(wpr(k), 1), max(n, 1))
                E = gf2.Mat(b.E[o["e"]:o["e"] + max(k * wpr(m), 1)], k, m, max(wpr(m), 1), max(k, 1))
                gf2.gf2_decompose(b.mat_view(i), L, E, b.perm[o["p"]:], b.pivcols[o["c"]:], b.rank[i:i + 1],
                                  stream)

        one_by_one()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        one_by_one()
        torch.cuda.synchronize()
        ms_pm = (time.perf_counter() - t1) * 1e3
        h2 = b.fetch()
        out["one_launch_per_matrix"] = {"ms_decompose": ms_pm, "matrices_per_s": BATCH_COUNT / (ms_pm / 1e3),
                                        "batched_speedup": ms_pm / ms_dec,
                                        "outputs_identical": all(np.array_equal(keep[k], h2[k]) for k in keep)}
    return out


def other_configs(gf2, synth, reps: int = 5):
    """The remaining single-matrix configurations, device-resident, HIP-event timed."""
    import torch

    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {}
    for n, seed in ((2048, 2048), (16384, 16384)):
        A = gf2.Mat.from_rowmajor(synth.dense(seed, 1, n, n), n, n)
        res = gf2.decompose(A, stream=stream)
        ms = timed(lambda: gf2.decompose(A, stream=stream, L=res["L"], E=res["E"]))
        ops = eff_bitops(n, n, res["pivcols"].cpu().numpy())
        out[f"decompose_{n}"] = {"ms": ms, "eff_bitops_per_s": ops / (ms / 1e3), "rank": int(res["rank"].item())}
        del A, res
    n = 16384
    A = gf2.Mat.from_rowmajor(synth.dense(16384, 2, n, n), n, n)
    B = gf2.Mat.from_rowmajor(synth.dense(16384, 3, n, n), n, n)
    C = gf2.Mat.zeros(n, n)
    ms = timed(lambda: gf2.gf2_matmul(C, A, B, False, stream))
    out["matmul_16384"] = {"ms": ms, "bitops_per_s": 2.0 * n ** 3 / (ms / 1e3)}
    del A, B, C
    # products whose output is too small for the table kernels to fill the chip:
    # the automatic choice is the fp4 matrix-core product; beside it the
    # Four-Russians kernel the automatic rule would otherwise take (256-row tiles)
    for (n, k, m) in ((8192, 8192, 8192), (4096, 16384, 4096)):
        A = gf2.Mat.from_rowmajor(synth.dense(8192, 4, n, k), n, k)
        B = gf2.Mat.from_rowmajor(synth.dense(8192, 5, k, m), k, m)
        C = gf2.Mat.zeros(n, m)
        ms = timed(lambda: gf2.gf2_matmul(C, A, B, False, stream))
        ref = C.t.clone()
        gf2.gf2_set_param("gemm_variant", 3)
        try:
            ms_fr = timed(lambda: gf2.gf2_matmul(C, A, B, False, stream))
        finally:
            gf2.gf2_set_param("gemm_variant", -1)
        same = bool(torch.equal(ref, C.t))
        out[f"matmul_{n}x{k}x{m}"] = {"ms": ms, "bitops_per_s": 2.0 * n * k * m / (ms / 1e3), "kernel": "fp4 MFMA",
                                      "ms_four_russians": ms_fr, "identical": same}
        del A, B, C, ref
    nr, r, m = 32768, 20000, 65536
    X, Y = synth.planted(20000, 9, nr, m, r)
    A = gf2.matmul(gf2.Mat.from_rowmajor(X, nr, r), gf2.Mat.from_rowmajor(Y, r, m), stream=stream)
    del X, Y
    res = gf2.decompose(A, stream=stream)
    ms = timed(lambda: gf2.decompose(A, stream=stream, L=res["L"], E=res["E"]))
    ops = eff_bitops(nr, m, res["pivcols"].cpu().numpy())
    out["decompose_planted_32768x65536_r20000"] = {"ms": ms, "eff_bitops_per_s": ops / (ms / 1e3),
                                                   "rank": int(res["rank"].item())}
    del A, res
    torch.cuda.empty_cache()
    return out


SERVE_SEED, SERVE_COUNT = 5, 1500


def serving_section(synth, count: int):
    from paper_1209_5198_amd import serve

    t0 = time.perf_counter()
    specs = synth.serving_specs(SERVE_SEED, count)
    data = serve.make_request_data(SERVE_SEED, specs)
    gen_s = time.perf_counter() - t0

    def session(arrivals):
        srv = serve.Server(cap_bytes=64 << 30, big_streams=4)
        return srv.run(serve.make_requests(specs, data, arrivals))

    session(np.zeros(count))  # warm-up: library workspaces, kernels
    sat = session(np.zeros(count))
    out = {"workload": f"{count} requests, kind uniform over rank/solve/decompose, square sides log-uniform "
                       "in [128, 16384] or 1:4 with the long side log-uniform in [512, 16384]; "
                       f"seed {SERVE_SEED}; 64 GB admission cap; sides <= 2048 batched",
           "data_gen_s": round(gen_s, 1), "saturated": sat, "poisson": {}}
    rate = sat["requests_per_s"]
    for frac in (0.5, 0.8, 0.95):
        arr = synth.poisson_arrivals(SERVE_SEED, count, frac * rate)
        st = session(arr)
        st["offered_rate"] = frac * rate
        out["poisson"][f"{int(frac * 100)}%"] = st
    return out


# Nominal MI355X figures beside which the microbenchmarks are reported (256 CUs,
# 2.4 GHz): HBM3E 8 TB/s; 32-bit VALU 128 lanes/clk/CU = 78.6 Tops/s (the lane
# rate behind the 157.3 TFLOP/s fp32 vector figure); LDS 64 banks x 4 B =
# 256 B/clk/CU = 157.3 TB/s; dense matrix cores int8 5.0 POPS, fp4 10.1 PFLOP/s
# (two operations per multiply-accumulate).
PEAKS = (  # name, kind argument, unit, nominal, scale of the measured rate into the unit
    ("hbm_read", dict(nbytes=2 << 30), "TB/s", 8.0, 1e-12),
    ("hbm_copy", dict(nbytes=2 << 30), "TB/s", 8.0, 1e-12),
    ("valu_xor32", dict(iters=2048), "Tops/s", 78.6, 1e-12),
    ("lds_read", dict(iters=2048), "TB/s", 157.3, 1e-12),
    ("mfma_int8", dict(iters=8192), "TOPS", 5000.0, 2e-12),
    ("mfma_fp4", dict(iters=8192), "TFLOP/s", 10100.0, 2e-12),
)


def peaks_section(gf2):
    """Measured ceilings of the units the kernels use, beside the nominal figures."""
    out = {}
    for name, kw, unit, nominal, scale in PEAKS:
        rate, ms = gf2.gf2_microbench(name, **kw)
        v = rate * scale
        out[name] = {"measured": v, "nominal": nominal, "unit": unit, "frac": v / nominal, "ms": ms}
    return out


def headline_section(args, gf2, synth):
    """The 65536^2 decomposition: timed steps, roofline of the product kernel."""
    import torch

    n = m = args.n
    print(f"# generating {n}x{m} Bernoulli(1/2) input (seed {SEED})", file=sys.stderr, flush=True)
    words = synth.dense(SEED, 1, n, m)
    A = gf2.Mat.from_rowmajor(words, n, m)
    del words
    kmin = min(n, m)
    L = gf2.Mat.zeros(n, kmin)
    E = gf2.Mat.zeros(kmin, m)
    perm = torch.empty(n, dtype=torch.int64, device="cuda")
    piv = torch.empty(kmin, dtype=torch.int64, device="cuda")
    rank = torch.empty(1, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        gf2.gf2_decompose(A, L, E, perm, piv, rank, stream)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"# warmup {i} done", file=sys.stderr, flush=True)
    # timed steps, library profiling off; an event between consecutive steps
    # gives each step's own duration (min / median)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(args.steps):
        step()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    print(f"# timed {args.steps} steps: wall {wall*1e3:.1f} ms, events {step_ms.sum():.1f} ms", file=sys.stderr,
          flush=True)
    # a separate instrumented pass: every product launch records its own start
    # and end (HIP events on its launch stream) and its lookup count
    gf2.gf2_profile(True)
    for _ in range(args.profile_steps):
        step()
    torch.cuda.synchronize()
    kms, klaunch, lookups = gf2.gf2_profile_read()
    gf2.gf2_profile(False)

    r = int(rank.item())
    pc = piv.cpu().numpy()
    ops = eff_bitops(n, m, pc)
    ms_per_step = wall * 1e3 / args.steps
    value = ops / (ms_per_step / 1e3)

    per_launch_ms = kms / max(klaunch, 1)
    lookups_per_launch = lookups / max(klaunch, 1)
    achieved_tbs = (8.0 * lookups_per_launch) / (per_launch_ms / 1e3) / 1e12 if per_launch_ms > 0 else 0.0
    traffic = None
    src = os.path.join(ROOT, "paper_1209_5198_amd", "csrc", "k_gemm.hip")
    if n == 65536 and os.path.exists(src):
        with open(src, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() == TRAFFIC["kernel_source_sha256"]:
                traffic = TRAFFIC["fetch_bytes"] + TRAFFIC["write_bytes"]
    roof = {"bound": "lds", "achieved": achieved_tbs, "peak": LDS_PEAK_TBS, "unit": "TB/s",
            "frac": achieved_tbs / LDS_PEAK_TBS, "traffic": traffic,
            "kernel": "k_gemm_wide / k_gemm_narrow (trailing-update Four-Russians product)",
            "work_per_launch": {"lookups": lookups_per_launch, "lds_bytes": 8.0 * lookups_per_launch},
            "avg_launch_ms": per_launch_ms, "launches": klaunch, "profiled_steps": args.profile_steps,
            "kernel_share_of_step": (kms / args.profile_steps) / ms_per_step if ms_per_step > 0 else None}

    out = {"metric": METRIC, "value": value, "unit": "bit-ops/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": value / PAPER_BITOPS_PER_S if n == 65536 else None,
           "dtype": "u64", "data": "synthetic",
           "config": {"workload": f"gf2_decompose {n}x{m} Bernoulli(1/2), P*A=L*E with L, E, perm, pivcols, rank",
                      "n": n, "m": m, "seed": SEED, "rank": r, "eff_bitops_per_step": ops,
                      "panel_words": 8},
           "step_ms": {"min": float(step_ms.min()), "median": float(np.median(step_ms)),
                       "max": float(step_ms.max())},
           "roofline": roof}
    del A, L, E
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--profile-steps", type=int, default=3,
                    help="steps of the separate instrumented pass that measures the product launches")
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--no-cpu", action="store_true", help="skip the cpu_baseline leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched workload")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving sessions")
    ap.add_argument("--no-configs", action="store_true", help="skip the other single-matrix configurations")
    ap.add_argument("--no-headline", action="store_true", help="skip the 65536^2 decomposition (profiling runs)")
    ap.add_argument("--no-peaks", action="store_true", help="skip the microbenchmarks of HBM, VALU, LDS, MFMA")
    ap.add_argument("--no-per-matrix", action="store_true",
                    help="skip the one-call-per-matrix comparison of the batched workload")
    ap.add_argument("--serve-count", type=int, default=SERVE_COUNT)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}), flush=True)
        sys.exit(2)

    import torch

    from paper_1209_5198_amd import gf2, synth

    torch.cuda.set_device(0)
    if args.copy_calibration:
        nbytes = 1 << 30
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read": nbytes, "bytes_written": nbytes, "copies": 3}}),
              flush=True)
        return
    if args.no_headline:
        out = {"metric": METRIC, "note": "headline skipped (--no-headline)"}
    else:
        out = headline_section(args, gf2, synth)
    if not args.no_peaks:
        print("# unit microbenchmarks", file=sys.stderr, flush=True)
        out["peaks"] = peaks_section(gf2)
    if not args.no_configs:
        print("# other configurations", file=sys.stderr, flush=True)
        out["configs"] = other_configs(gf2, synth)
    if not args.no_batched:
        print("# batched workload", file=sys.stderr, flush=True)
        out["batched"] = batched_section(gf2, synth, args.batch_steps, per_matrix=not args.no_per_matrix)
    if not args.no_serving:
        print("# serving sessions", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        out["serving"] = serving_section(synth, args.serve_count)
    if not args.no_cpu:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
        ops65536 = out.get("config", {}).get("eff_bitops_per_step") if args.n == 65536 else None
        out["cpu_baseline"]["full_size_once"] = [
            dict(r, input="65536x65536 Bernoulli(1/2), seed 65536 (the headline matrix), run once, cached",
                 eff_bitops_per_s=(ops65536 / r["s"]) if ops65536 else None) for r in ORACLE_65536_ONCE]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
