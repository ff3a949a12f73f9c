"""Benchmark: block-layer QGT SR steps/s on one MI355X.

One step = form + solve of the whole hot path (centred energy, column means,
force and block traces, centre-and-pack, block Grams, FP64 Cholesky of the
shifted blocks, preconditioned FP64 CG on the exact operator with its
triangular solves, back-projection and scatter) on inputs resident in HBM.
The step is captured once in a HIP graph and the replays are timed
(--no-graph: eager launches).

Default workload: the 2-layer complex FFNN 100-400-400 on the 10x10 lattice,
n_s = 8192 zero-magnetisation samples, layer blocks [40400, 160400] (both in
the sample-space form), complex64 Jacobian, lambda = 1e-4, automatic Gram
precision (BF16 on both blocks), FP64 factors, at most six CG iterations with
the per-block convergence test at 1e-5.

Prints one JSON line.  Also reported: delta against the FP64 oracle on a
bounded sample of the workload (the GPU path in the same settings, on the
sample the CPU oracle is timed on), the same step with FP32 factors of the
BF16 blocks, the full-QGT FP64 solve on the same GPU, the Gram kernels' MFMA
roofline fractions from HIP events recorded on the launch stream during eager
steps, the device formation of O, and the FP64 CPU oracle timed on that
sample.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "block-QGT SR steps/s (form+solve) vs full-QGT FP64, at rel err ≤1e-5 on δ"
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2516.0}  # TFLOP/s, dense MFMA
# the Gram launches timed per precision; a BF16 block runs the kernel of its
# tile kind (1: 128x128 tiles, 2: 256x128 wide tiles, 3: 128x128 tiles with
# two workgroups per CU), and the BF16 time covers the kinds the plan uses
GRAM_KERNELS = {"fp64": "k_gram<0>", "fp32": "k_gram<1>"}
BF16_TILE_KERNELS = {1: "k_gram<2>", 2: "k_gram_wide", 3: "k_gram_duo"}


def gram_kernel(prec: str, sr) -> str:
    """The Gram kernels timed for precision `prec` in plan `sr`, '+'-joined."""
    if prec != "bf16":
        return GRAM_KERNELS[prec]
    tiles = {sr.block_tuning(g)["gram_tile"] for g in range(sr.num_blocks)
             if sr.block_info(g)["precision"] == "bf16"}
    return "+".join(BF16_TILE_KERNELS[t] for t in sorted(tiles))
HBM_PEAK = 8000.0  # GB/s
DEFAULT_CONFIG = "2b"
# tuning cache written by the library's autotuner on an MI355X (bench.py --tune)
TUNE_CACHE = os.path.join(ROOT, "paper_2510_08430_amd", "tuning", "gfx950.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(cfg: str):
    """(workloads, description, Gram precision, bound on the CG iterations,
    oracle sample).  Every workload runs the per-block convergence test at
    1e-5: a block stops as soon as its last correction is below it, so the
    bound is an upper bound.  The oracle sample is the bounded part of the
    workload the CPU oracle solves (problem, block, rows; None = all).  The
    CNN and the uneven blocks take BF16 Grams for every block: the CG
    iterations they add (two or three more, each two passes over O) cost far
    less than the FP32 Grams the default policy gives their parameter-space
    blocks, and every block still meets 1e-5; the 32-instance stream keeps
    the default policy (some of its blocks do not converge within four
    iterations from a BF16 Gram)."""
    from gen import workloads
    if cfg == "1":
        w = workloads.config1(o_dtype=np.complex64)
        desc = ("FFNN 64-128-128-64 logcosh + dense readout, 64-spin chain, n_s=4096 zero-magnetisation "
                "samples, blocks [8320,16512,8256,65], complex64 O, E_loc re N(-7,1) im N(0,0.1^2), lambda=1e-3")
        return [w], desc, "auto", 4, dict(problem=0, block=2, rows=2048)
    if cfg == "0":
        w = workloads.config0(o_dtype=np.complex128)
        return ([w], "complex RBM N=16 M=32, n_s=1024, blocks [512,32,16], complex128 O, lambda=1e-4", "fp64", 0,
                dict(problem=0, block=None, rows=None))
    if cfg == "2a":
        w = workloads.config2_cnn()
        return [w], ("4-layer complex CNN 3x3 16 channels on 10x10 PBC, n_s=8192, blocks [160,2320,2320,2320], "
                     "complex64 O, lambda=1e-4"), "bf16", 6, dict(problem=0, block=1, rows=None)
    if cfg == "2b":
        w = workloads.config2_ffnn()
        return [w], ("2-layer complex FFNN 100-400-400 on 10x10, n_s=8192 zero-magnetisation samples, blocks "
                     "[40400,160400] (sample form), complex64 O, E_loc re N(-50,3^2) im N(0,0.5^2), lambda=1e-4"), \
            "auto", 6, dict(problem=0, block=0, rows=2048)
    if cfg == "3":
        w = workloads.config3()
        pick = min(range(len(w.block_sizes)), key=lambda b: abs(w.block_sizes[b] - 2048))
        return [w], (f"64 blocks log-uniform in [64,8192] (n_p={w.n_p}), n_s=8192, complex normal O with "
                     "per-block geometric column decay, lambda=1e-5"), "bf16", 6, dict(problem=0, block=pick,
                                                                                       rows=None)
    if cfg == "4":
        ws = [workloads.config4_instance(i) for i in range(32)]
        return ws, ("32 independent chain FFNN N-2N-N instances, N in {16,24,32,48,64}, n_s in {1024,2048,4096}, "
                    "lambda=1e-4, one plan"), "auto", 4, dict(problem=0, block=None, rows=None)
    raise SystemExit(f"unknown config {cfg}")


def measured_traffic(kernel: str, config: str):
    """HBM bytes per launch of `kernel` on workload `config`, from the counter
    summaries under profiles/ (FETCH_SIZE and WRITE_SIZE, each scaled by the
    same counter's reading for a plain copy of known size).  None when no
    summary covers it or when a source file the launch depends on (the
    kernel's, and the planner's, which orders its work items) has changed
    since the counters were taken (their SHA-256 are recorded in the
    summary, comma-separated in the order of the sources)."""
    import glob
    import hashlib
    import re
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.md"))):
        text = open(path).read()
        fields = dict(re.findall(r"^- (\w+): (\S+)\s*$", text, flags=re.M))
        if fields.get("kernel") != kernel or fields.get("workload") != config:
            continue
        srcs = [os.path.join(ROOT, f) for f in fields.get("source", "").split(",") if f]
        shas = fields.get("source_sha256", "").split(",")
        if not srcs or len(srcs) != len(shas) or not all(os.path.isfile(f) for f in srcs):
            return None
        if any(hashlib.sha256(open(f, "rb").read()).hexdigest() != h for f, h in zip(srcs, shas)):
            return None
        return int(fields["traffic_bytes_per_launch"])
    return None


def sample_problem(wls, sample):
    """(O, e_loc, block sizes, lambda) of the oracle sample: the chosen block's
    columns (or all) of the chosen problem, its first `rows` samples (or
    all)."""
    from oracle import block_sr as orc
    w = wls[sample["problem"]]
    rows = w.n_s if sample["rows"] is None else min(sample["rows"], w.n_s)
    if sample["block"] is None:
        sizes = list(w.block_sizes)
        O = w.O[:rows]
    else:
        offs = orc.block_offsets(w.block_sizes)
        b = sample["block"]
        sizes = [w.block_sizes[b]]
        O = w.O[:rows, offs[b]:offs[b + 1]]
    return np.ascontiguousarray(O), np.ascontiguousarray(w.e_loc[:rows]), sizes, w.lam


def host_info():
    """Host CPU model, logical CPUs usable by this process and the BLAS threads."""
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except Exception:
        nproc = os.cpu_count() or 1
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = nproc
    return model, nproc, threads


def cpu_baseline(wls, sample, reps=3):
    """Time the FP64 oracle, as it stands, on a bounded sample of the workload
    (one warm-up, then the median of `reps` runs): block_sr on the sample, and
    the Gram step alone so that the sample splits into Gram time and the rest
    (mostly the eigensolver).  The whole step is scaled from the sample block
    by block: Gram time by Gram flops, the rest by m^3 (m the matrix order,
    n_b or n_s).  The same sample solved by the oracle's Cholesky form is the
    fair CPU comparator of the GPU path's method.  Returns the record and the
    oracle's delta of the sample."""
    from oracle import block_sr as orc
    O, e, sizes, lam = sample_problem(wls, sample)
    n_s = O.shape[0]
    model, nproc, threads = host_info()

    def m_of(nb, ns):
        return min(nb, ns)

    def gram_flops(nb, ns):
        return 4.0 * ns * nb * m_of(nb, ns)

    def timed(fn):
        fn()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            out = fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), ts, out

    def gram_only():
        offs = orc.block_offsets(sizes)
        for b, nb in enumerate(sizes):
            dO = orc.centred_block(O, offs[b], offs[b + 1])
            (orc.sample_space_matrix if n_s < nb else orc.qgt_block)(dO)

    t_all, all_runs, ref = timed(lambda: orc.block_sr(O, e, sizes, lam))
    t_gram, _, _ = timed(gram_only)
    t_rest = max(t_all - t_gram, 0.0)
    t_ch, _, _ = timed(lambda: orc.block_sr_cholesky(O, e, sizes, lam))
    t_ch_rest = max(t_ch - t_gram, 0.0)
    fl_s = sum(gram_flops(nb, n_s) for nb in sizes)
    m3_s = sum(m_of(nb, n_s) ** 3 for nb in sizes)
    fl = sum(gram_flops(nb, w.n_s) for w in wls for nb in w.block_sizes)
    m3 = sum(m_of(nb, w.n_s) ** 3 for w in wls for nb in w.block_sizes)
    t_step = t_gram * fl / fl_s + t_rest * m3 / m3_s
    t_ch_step = t_gram * fl / fl_s + t_ch_rest * m3 / m3_s
    n_inst = len(wls)
    what = ("the whole workload" if sample["block"] is None and sample["rows"] is None and n_inst == 1 else
            f"problem {sample['problem']}, " + ("all blocks" if sample["block"] is None else
                                                  f"block {sample['block']} ({sizes[0]} columns, "
                                                  f"{'sample' if n_s < sizes[0] else 'parameter'} form)")
            + f", first {n_s} samples")
    rec = {"value": n_inst / t_step, "unit": "steps/s", "cores": int(threads), "kind": "oracle",
           "host_cpu": model, "host_nproc": int(nproc),
           "cholesky_comparator_steps_per_s": n_inst / t_ch_step,
           "sample_s_median": t_all, "sample_s_runs": all_runs,
           "sample": (f"FP64 oracle (numpy/scipy, eigh with spectral cutoff) on {what}: median of {reps} runs after "
                      f"a warm-up {t_all:.2f} s, of which Gram {t_gram:.2f} s; scaled to the whole step block by "
                      f"block (Gram by flops, the rest by m^3): {t_step:.1f} s per step")}
    return rec, ref.delta, (O, e, sizes, lam)


def oracle_check(qgt, dt, gram, refine, rtol, factor, sample_data, ref_delta, cholesky="auto"):
    """The GPU path, in the benchmark's settings, on the oracle's sample:
    per-block relative error of delta against the oracle's delta."""
    import torch
    from oracle import block_sr as orc
    O, e, sizes, lam = sample_data
    sr = qgt.BlockSR([(O.shape[0], sizes, lam)], dt, gram, refine, rtol=rtol, factor=factor, cholesky=cholesky)
    d = sr([torch.from_numpy(O).cuda()], [torch.from_numpy(e).cuda()])[0].cpu().numpy()
    st = sr.status()
    errs = orc.block_relative_errors(d, ref_delta, sizes)
    sr.close()
    return max(errs), errs, st


def time_graph(qgt, probs, dt, gram, refine, rtol, factor, Os, Es, deltas, steps, warmup, cholesky="auto"):
    """Capture one step (form + solve) in a HIP graph and time its replays.
    Returns (ms per step, plan, graph) so the caller can read the plan's
    status after the replays."""
    import torch
    plan = qgt.BlockSR(probs, dt, gram, refine, rtol=rtol, factor=factor, cholesky=cholesky)
    plan.form(Os, Es)
    plan.solve(deltas)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        with torch.cuda.graph(graph, stream=cap):
            plan.form(Os, Es)
            plan.solve(deltas)
    torch.cuda.current_stream().wait_stream(cap)
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / steps, plan, graph


def dtype_label(sr):
    """Arithmetic of the path: Gram precision and factor precision per block,
    then the FP64 iteration."""
    kinds = sorted({f"{i['precision']}-gram/{'f32' if i['factor'] == 'fp32' else 'f64'}-factor"
                    for i in (sr.block_info(g) for g in range(sr.num_blocks))})
    return "+".join(kinds) + ",f64-cg"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default=DEFAULT_CONFIG)
    ap.add_argument("--gram", default=None, help="fp64 | fp32 | bf16 (default per workload)")
    ap.add_argument("--refine", type=int, default=None, help="bound on the CG iterations after the first solve")
    ap.add_argument("--rtol", type=float, default=1e-5,
                    help="per-block convergence test of the CG iteration (0: a fixed number of iterations)")
    ap.add_argument("--factor", default="fp64", help="fp64 (default) | fp32: factor precision of BF16-Gram blocks")
    ap.add_argument("--cholesky", default="auto", help="auto (the tuning cache's choice for the workload, else "
                    "persistent) | persistent (one launch over the tile tasks of every block) | host-steps (one "
                    "launch per tile step of all blocks)")
    ap.add_argument("--tune", action="store_true",
                    help="first run the autotuner for this workload's block shapes and merge the result into the "
                         "tuning cache")
    ap.add_argument("--tune-reps", type=int, default=3, help="timed runs per autotuner candidate (the fastest counts)")
    ap.add_argument("--tune-cache", default=None,
                    help="tuning cache to plan with (default: $QGT_TUNE_CACHE, else the committed cache)")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches instead of a HIP-graph replay")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (a known-size reference for HBM counters)")
    ap.add_argument("--no-full", action="store_true", help="skip the full-QGT FP64 comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and the oracle check")
    ap.add_argument("--no-variant", action="store_true", help="skip timing the FP32-factor variant")
    ap.add_argument("--vendor", action="store_true", help="also time a torch.linalg FP64 full solve")
    ap.add_argument("--vendor-gemm", action="store_true",
                    help="also time the vendor BF16 GEMM (torch.matmul) on the largest BF16 block's real shape, "
                         "as a practical ceiling for the matrix cores")
    ap.add_argument("--no-jacobian", action="store_true", help="skip timing the device formation of O")
    ap.add_argument("--vmc-iters", type=int, default=20,
                    help="RBM workload: iterations of the device VMC loop to time (0 skips it)")
    ap.add_argument("--vmc-converge", type=int, default=0,
                    help="RBM workload: also run the device VMC loop this many iterations with block SR and with "
                         "full-QGT SR (same seeds and moves) and report both energy curves")
    ap.add_argument("--vmc-eta", default="0.05",
                    help="learning rates of the --vmc-converge runs, comma-separated (each runs block and full)")
    ap.add_argument("--vmc-lam", type=float, default=1e-4, help="diagonal shift of the --vmc-converge runs")
    args = ap.parse_args()
    if args.gpus != 1:
        raise SystemExit("bench.py runs on one GPU only: the library has no multi-GPU path (use --gpus 1)")

    import torch
    import paper_2510_08430_amd as qgt

    qgt.load()
    torch.cuda.set_device(0)
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: 3 copies of {args.copy_probe_mib} MiB")
        del src, dst
    t0 = time.perf_counter()
    wls, desc, gram, refine, sample = make_workload(args.config)
    gram = args.gram or gram
    refine = args.refine if args.refine is not None else refine
    log(f"[bench] workload {args.config}: generated in {time.perf_counter() - t0:.1f} s; gram={gram} "
        f"refine<={refine} rtol={args.rtol} factor={args.factor}")

    dt = "c64" if wls[0].O.dtype == np.complex64 else "c128"
    probs = [(w.n_s, w.block_sizes, w.lam) for w in wls]
    cache = args.tune_cache or os.environ.get("QGT_TUNE_CACHE") or TUNE_CACHE
    if args.tune:
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        t0 = time.perf_counter()
        os.environ.setdefault("QGT_TUNE_LOG", "1")  # one line per tuning decision on stderr
        n = qgt.autotune(probs, dt, gram, cache, reps=args.tune_reps)
        log(f"[bench] autotuned {n} block classes into {cache} in {time.perf_counter() - t0:.1f} s")
    os.environ["QGT_TUNE_CACHE"] = cache
    Os = [torch.from_numpy(w.O).cuda() for w in wls]
    Es = [torch.from_numpy(w.e_loc).cuda() for w in wls]
    deltas = [torch.empty(w.n_p, dtype=torch.complex128, device="cuda") for w in wls]
    sr = qgt.BlockSR(probs, dt, gram, refine, timing=True, rtol=args.rtol, factor=args.factor, cholesky=args.cholesky)
    precs = sr.precisions()
    label = dtype_label(sr)
    tuning = [{"block": g, **sr.block_tuning(g)} for g in range(sr.num_blocks)]
    chol = sr.cholesky_mode()
    log(f"[bench] plan: {sr.num_blocks} blocks, {label}, workspace {sr.workspace_bytes / 2**30:.2f} GiB, "
        f"Cholesky {chol['mode']} ({chol['source']})")

    def step(plan):
        plan.form(Os, Es)
        plan.solve(deltas)

    # eager steps: per-kernel HIP-event timing of the Gram launches (roofline)
    for _ in range(args.warmup):
        step(sr)
    torch.cuda.synchronize()
    for pr in precs:
        sr.gram_timing(pr, reset=True)
    log("[bench] warmup done; timing eager steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(sr)
    torch.cuda.synchronize()
    eager_ms = 1e3 * (time.perf_counter() - t0) / args.steps
    status = sr.status()
    floors = sr.pivot_floors()
    its = [sr.cg_iterations(g) for g in range(sr.num_blocks)]
    gtime = {pr: sr.gram_timing(pr, reset=True) for pr in precs}
    log(f"[bench] eager {eager_ms:.3f} ms/step; Gram ms/launch "
        + ", ".join(f"{pr}: {ms / max(n, 1):.3f}" for pr, (ms, n, _) in gtime.items()))

    # the same step captured once in a HIP graph and replayed
    ms_per_step = eager_ms
    mode = "eager"
    if not args.no_graph:
        log("[bench] timing graph replays")
        ms_per_step, gsr, graph = time_graph(qgt, probs, dt, gram, refine, args.rtol, args.factor, Os, Es, deltas,
                                             args.steps, args.warmup, args.cholesky)
        mode = "hip-graph"
        status = [max(a, b) for a, b in zip(status, gsr.status())]
        floors = [max(a, b) for a, b in zip(floors, gsr.pivot_floors())]
        del graph, gsr
        log(f"[bench] graph {ms_per_step:.3f} ms/step")
    inst_per_step = len(wls)
    value = inst_per_step * 1e3 / ms_per_step

    bad = {g: v for g, v in enumerate(status) if v != 0}
    its_hist = {str(k): its.count(k) for k in sorted(set(its))}
    log(f"[bench] CG iterations run per block (iterations: blocks) {its_hist}; pivots raised to lambda "
        f"{sum(floors)}")
    result = {
        "metric": METRIC, "value": value, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": label, "data": "synthetic",
        "config": {"workload": desc, "instances_per_step": inst_per_step, "gram": gram,
                   "gram_precisions": precs, "factor": args.factor,
                   "cholesky": chol["mode"], "cholesky_source": chol["source"],
                   "cg_iterations_max": refine,
                   "refine_rtol": args.rtol, "o_dtype": dt, "timing": mode},
        "eager_ms_per_step": eager_ms, "status_ok": not bad, "bad_block_status": bad,
        "cg_iterations_run": its_hist, "pivots_raised_to_lambda": int(sum(floors)),
        "tuning": tuning if len(tuning) <= 8 else {"blocks": len(tuning), "sources": sorted({t["source"] for t in tuning}),
                                                   "chol_chunks": sorted({t["chol_chunk"] for t in tuning})},
        "tuning_cache": os.path.relpath(cache, ROOT) if os.path.isfile(cache) else None,
    }

    # the same step with the BF16-Gram blocks stored in complex64 and factored in FP32
    if not args.no_variant and args.factor == "fp64" and "bf16" in precs:
        log("[bench] timing the FP32-factor variant")
        ms_v, vsr, graph = time_graph(qgt, probs, dt, gram, refine, args.rtol, "fp32", Os, Es, deltas, args.steps,
                                      args.warmup, args.cholesky)
        vst = vsr.status()
        result["fp32_factor_variant"] = {"ms_per_step": ms_v, "steps_per_s": inst_per_step * 1e3 / ms_v,
                                         "dtype": dtype_label(vsr), "status_ok": not any(vst),
                                         "pivots_raised_to_lambda": int(sum(vsr.pivot_floors()))}
        del graph, vsr
        log(f"[bench] FP32-factor variant {ms_v:.3f} ms/step")

    kernels = {}
    for pr, (ms, n, fl) in gtime.items():
        if n > 0:
            ach = fl / (ms / n * 1e-3) / 1e12
            kernels[pr] = {"kernel": gram_kernel(pr, sr), "ms_per_launch": ms / n, "flops_per_launch": fl,
                           "achieved_tflops": ach, "peak_tflops": PEAK[pr], "frac": ach / PEAK[pr]}
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["ms_per_launch"])
        kd = kernels[dom]
        result["roofline"] = {"bound": "mfma", "achieved": kd["achieved_tflops"], "peak": kd["peak_tflops"],
                              "unit": "TFLOP/s", "frac": kd["frac"],
                              "traffic": measured_traffic(kd["kernel"], args.config), "kernel": kd["kernel"],
                              "ms_per_launch": kd["ms_per_launch"], "flops_per_launch": kd["flops_per_launch"]}
        result["gram_kernels"] = kernels

    if not args.no_full and len(wls) == 1:
        w = wls[0]
        full = qgt.BlockSR([(w.n_s, [w.n_p], w.lam)], dt, "fp64", 0)
        fd = torch.empty_like(deltas[0])
        for _ in range(2):
            full.form(Os, Es)
            full.solve([fd])
        torch.cuda.synchronize()
        nfull = max(2, args.steps // 4)
        t0 = time.perf_counter()
        for _ in range(nfull):
            full.form(Os, Es)
            full.solve([fd])
        torch.cuda.synchronize()
        tf = (time.perf_counter() - t0) / nfull
        result["full_fp64"] = {"steps_per_s": 1.0 / tf, "ms_per_step": 1e3 * tf,
                               "form": "sample" if w.n_s < w.n_p else "parameter",
                               "speedup_block_vs_full": value * tf}
        log(f"[bench] full FP64: {1e3 * tf:.2f} ms/step")
        del full
        if args.vendor:
            result["vendor_full_fp64"] = vendor_full(Os[0], Es[0], w.lam)

    if args.vendor_gemm:
        vg = vendor_bf16_gemm(sr, probs)
        if vg is not None:
            result["vendor_bf16_gemm"] = vg
            log(f"[bench] vendor BF16 GEMM {vg['shape']}: {vg['tflops']:.0f} TFLOP/s; this Gram: "
                f"{kernels['bf16']['achieved_tflops'] if 'bf16' in kernels else float('nan'):.0f} TFLOP/s")

    if not args.no_jacobian:
        jf = jacobian_formation(args.config, Os, max(5, args.steps // 2))
        if jf is not None:
            result["jacobian_formation"] = jf
            log(f"[bench] device formation of O: {jf['ms']:.3f} ms, {jf['achieved_gbs']:.0f} GB/s, "
                f"{jf['achieved_fp64_tflops']:.1f} FP64 TFLOP/s ({100 * jf['frac']:.1f}% of the {jf['bound']} peak), "
                f"max rel diff vs host O {jf['max_rel_diff_vs_host_O']:.2e}")

    if args.config == "0" and args.vmc_iters > 0:
        vl = vmc_loop(args.vmc_iters)
        result["vmc_loop"] = vl
        log(f"[bench] VMC loop: {vl['ms_per_iteration']:.3f} ms/iteration, energy {vl['energy_first']:.4f} -> "
            f"{vl['energy_last']:.4f} (exact {vl['exact_e0']:.4f})")
    if args.config == "0" and args.vmc_converge > 0:
        result["vmc_block_vs_full"] = []
        for eta in [float(v) for v in args.vmc_eta.split(",") if v]:
            for full_qgt in (False, True):
                vc = vmc_convergence(args.vmc_converge, full_qgt, eta=eta, lam=args.vmc_lam)
                result["vmc_block_vs_full"].append(vc)
                log(f"[bench] VMC {vc['qgt']} QGT, eta={eta}, lambda={args.vmc_lam}, {vc['iterations']} iterations "
                    f"({vc['wall_s']:.1f} s): mean energy of the last 100 {vc['energy_last100_mean']:.5f}, "
                    f"rel err {vc['rel_err_last100']:.2e}")

    if not args.no_cpu:
        del Os, Es
        torch.cuda.empty_cache()
        log("[bench] timing the CPU oracle on a bounded sample")
        rec, ref_delta, sample_data = cpu_baseline(wls, sample)
        result["cpu_baseline"] = rec
        err, errs, st = oracle_check(qgt, dt, gram, refine, args.rtol, args.factor, sample_data, ref_delta,
                                     args.cholesky)
        result["max_block_rel_err_vs_oracle"] = err
        result["oracle_check"] = {"sample": rec["sample"].split(":")[0].replace("FP64 oracle (numpy/scipy, eigh "
                                                                                "with spectral cutoff) on ", ""),
                                  "per_block_rel_err": errs, "status_ok": not any(st)}
        log(f"[bench] CPU oracle {rec['sample']}; delta vs oracle on the sample: max block rel err {err:.3e}")
    print(json.dumps(result), flush=True)


def jacobian_networks(cfg: str):
    """The networks and samples behind the workload's O (the same seeded
    generators as make_workload), for the device formation of O; None where O
    is drawn directly."""
    from gen import workloads as W
    def smp(c, N, n_s, inst=0):
        return W.zero_magnetisation_samples(W.rng(c, W.P_SAMPLES, inst), n_s, N)
    if cfg == "1":
        net = W.ffnn_network([64, 128, 128, 64], config=1, readout=True, dtype=np.complex64)
        return [("ffnn", net.flat(), [64, 128, 128, 64], True, smp(1, 64, 4096), "c64")]
    if cfg == "0":
        net = W.rbm_network(N=16, M=32, config=0)
        return [("rbm", net.flat(), [16, 32], False, smp(0, 16, 1024), "c128")]
    if cfg == "2a":
        net = W.cnn_network(L=10, config=2, dtype=np.complex64)
        return [("cnn", net.flat(), [10, 16, 4], False, smp(2, 100, 8192), "c64")]
    if cfg == "2b":
        net = W.ffnn_network([100, 400, 400], config=2, instance=1, dtype=np.complex64)
        return [("ffnn", net.flat(), [100, 400, 400], False, smp(2, 100, 8192, 1), "c64")]
    if cfg == "4":
        out = []
        for i in range(32):
            g = W.rng(4, W.P_BLOCKS, i)
            N = int(g.choice(W.CONFIG4_CHAINS))
            n_s = int(g.choice(W.CONFIG4_NS))
            net = W.ffnn_network([N, 2 * N, N], config=4, instance=i, dtype=np.complex64)
            out.append(("ffnn", net.flat(), [N, 2 * N, N], False, smp(4, N, n_s, i), "c64"))
        return out
    return None


def jacobian_formation(cfg: str, host_O, reps: int):
    """Times the device formation of O (include/qgt_jacobian.h) for the
    workload's networks: the whole call (dense layers forward and backward,
    then the row writer), captured in a HIP graph, with HIP events around the
    replays on the launch stream.  Algorithmic
    bytes: O written once, plus the spins, theta and the per-sample
    derivative and activation rows read once."""
    import torch
    import paper_2510_08430_amd as qgt
    nets = jacobian_networks(cfg)
    if nets is None:
        return None
    calls, nbytes, outs, flops = [], 0, [], 0
    for kind, theta, widths, readout, x, dt in nets:
        th = torch.from_numpy(np.ascontiguousarray(theta)).cuda()
        xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.int8)).cuda()
        n_s = x.shape[0]
        eo = 8 if dt == "c64" else 16
        if kind == "rbm":
            N, M = widths
            n_p = M * N + M + N
            O = torch.empty((n_s, n_p), dtype=torch.complex64 if dt == "c64" else torch.complex128, device="cuda")
            wsb = qgt.rbm_jacobian_workspace_bytes(N, M, n_s)
            ws = torch.empty(max(wsb, 256), dtype=torch.uint8, device="cuda")
            calls.append(lambda th=th, xd=xd, M=M, O=O, ws=ws: qgt.rbm_jacobian(th, xd, M, O=O, workspace=ws))
            rows = n_s * (M + N) * 16
        elif kind == "cnn":
            side, C, L = widths
            n_p = qgt.cnn_n_params(side, C, L)
            O = torch.empty((n_s, n_p), dtype=torch.complex64 if dt == "c64" else torch.complex128, device="cuda")
            wsb = qgt.cnn_jacobian_workspace_bytes(side, C, L, n_s)
            ws = torch.empty(max(wsb, 256), dtype=torch.uint8, device="cuda")
            calls.append(lambda th=th, xd=xd, side=side, C=C, L=L, O=O, ws=ws:
                         qgt.cnn_jacobian(th, xd, side, C, L, O=O, workspace=ws))
            S = side * side
            # activations and derivatives of every layer written and read once
            rows = n_s * S * C * 16 * (2 * L - 1) * 2
            flops += n_s * S * 8 * 9 * (2 * C + 2 * C * C * (L - 1) + C * C * (L - 1))
        else:
            n_p = qgt.ffnn_n_params(widths, readout)
            O = torch.empty((n_s, n_p), dtype=torch.complex64 if dt == "c64" else torch.complex128, device="cuda")
            wsb = qgt.ffnn_jacobian_workspace_bytes(widths, readout, n_s)
            ws = torch.empty(max(wsb, 256), dtype=torch.uint8, device="cuda")
            calls.append(lambda th=th, xd=xd, w=widths, r=readout, O=O, ws=ws:
                         qgt.ffnn_jacobian(th, xd, w, r, O=O, workspace=ws))
            rows = n_s * sum(widths[l] + widths[l + 1] for l in range(len(widths) - 1)) * 16
            flops += n_s * 8 * sum(widths[l] * widths[l + 1] for l in range(len(widths) - 1)) * 2
        nbytes += n_s * n_p * eo + n_s * widths[0] + n_p * 16 + rows
        outs.append(O)
    for c in calls:
        c()
    torch.cuda.synchronize()
    # the device-formed O against the host-formed input of the step (same
    # networks and samples; both round FP64 values once to the output type)
    diff = 0.0
    for O, H in zip(outs, host_O):
        d = (O - H).abs().max().item()
        diff = max(diff, d / max(H.abs().max().item(), 1e-300))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        for c in calls:
            c()
    e1.record()
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1) / reps
    # the calls allocate nothing and never synchronise: capture them once in a
    # HIP graph and time the replays (the host-side cost of many small calls
    # drops out, as in the timed step)
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        with torch.cuda.graph(graph, stream=cap):
            for c in calls:
                c()
    torch.cuda.current_stream().wait_stream(cap)
    graph.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = nbytes / (ms * 1e-3) / 1e9
    # a plain device fill of the same output buffers: the write rate HBM gives
    # a store-only stream, for context
    e0.record()
    for _ in range(reps):
        for O in outs:
            O.zero_()
    e1.record()
    torch.cuda.synchronize()
    ms_fill = e0.elapsed_time(e1) / reps
    obytes = sum(O.numel() * O.element_size() for O in outs)
    del outs
    torch.cuda.empty_cache()
    del graph
    entry = {"rbm": "qgt_rbm_jacobian", "ffnn": "qgt_ffnn_jacobian", "cnn": "qgt_cnn_jacobian"}[nets[0][0]]
    tf = flops / (ms * 1e-3) / 1e12
    # the dense networks are bound by writing O, the CNN by its FP64 products
    bound = {"bound": "fp64-mfma", "peak_tflops": PEAK["fp64"], "frac": tf / PEAK["fp64"]} if nets[0][0] == "cnn" \
        else {"bound": "hbm", "peak_gbs": HBM_PEAK, "frac": gbs / HBM_PEAK}
    return {"entry": entry, "calls_per_step": len(calls), "fp64_flops": flops, "achieved_fp64_tflops": tf,
            "timing": "hip-graph", "ms": ms, "eager_ms": eager_ms, "bytes": nbytes, "achieved_gbs": gbs, **bound,
            "plain_fill_gbs": obytes / (ms_fill * 1e-3) / 1e9, "max_rel_diff_vs_host_O": diff}


# exact ground-state energy of the 16-site periodic Heisenberg ring in S.S
# units (Lanczos on the zero-magnetisation sector); in Pauli units 4 E0 =
# -28.5692, the scale of the energies of Sec. 3, Tab. 2
HEISENBERG_L16_E0 = -7.142296360616785


def vmc_loop(iters: int, sweeps: int = 10, eta: float = 0.05, lam: float = 1e-4):
    """A VMC loop on the device for the complex RBM N=16 M=32 on the periodic
    Heisenberg chain of 16 sites, n_s = 1024 chains: per iteration sweeps x 16
    Metropolis exchange steps per chain, local energies, O formed on the
    device, block SR (three blocks W, b, a; FP64) and theta <- theta - eta
    delta.  The random inputs of all iterations are generated and uploaded
    before the timed region; one iteration is captured in a HIP graph and
    replayed, with the next iteration's moves copied into its input buffers
    before each replay (the copies are inside the timed region)."""
    import torch
    import paper_2510_08430_amd as qgt
    from gen import workloads as W
    N, M, n_s = 16, 32, 1024
    theta = torch.from_numpy(W.rbm_network(N=N, M=M, config=0).flat()).cuda()
    x = torch.from_numpy(W.zero_magnetisation_samples(W.rng(0, W.P_SAMPLES), n_s, N)).cuda()
    moves = [W.mcmc_moves(0, it, sweeps * N, n_s, N) for it in range(iters + 2)]
    moves = [(torch.from_numpy(p).cuda(), torch.from_numpy(u).cuda()) for p, u in moves]
    n_p = M * N + M + N
    O = torch.empty((n_s, n_p), dtype=torch.complex128, device="cuda")
    ws = torch.empty(qgt.rbm_jacobian_workspace_bytes(N, M, n_s), dtype=torch.uint8, device="cuda")
    delta = torch.empty(n_p, dtype=torch.complex128, device="cuda")
    e = torch.empty(n_s, dtype=torch.complex128, device="cuda")
    acc = torch.zeros(n_s, dtype=torch.int32, device="cuda")
    sr = qgt.BlockSR([(n_s, [M * N, M, N], lam)], "c128", "fp64", 0)
    energies, accept = [], 0

    def iteration(p, u):
        qgt.rbm_metropolis(theta, x, M, p, u, acc)
        qgt.rbm_heisenberg_eloc(theta, x, M, e_loc=e)
        qgt.rbm_jacobian(theta, x, M, O=O, workspace=ws)
        sr.form([O], [e])
        sr.solve([delta])
        qgt.sr_update(theta, delta, eta)

    for p, u in moves[:2]:
        iteration(p, u)
        energies.append(e.mean().real.item())
    torch.cuda.synchronize()
    # one iteration captured in a HIP graph that reads its moves from fixed
    # buffers; before each replay the next iteration's moves are copied in
    pbuf, ubuf = moves[0][0].clone(), moves[0][1].clone()
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        with torch.cuda.graph(graph, stream=cap):
            iteration(pbuf, ubuf)
    torch.cuda.current_stream().wait_stream(cap)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for p, u in moves[2:]:
        pbuf.copy_(p)
        ubuf.copy_(u)
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    energies.append(e.mean().real.item())
    del graph
    accept = int(acc.sum().item())
    bad = any(sr.status())
    del sr
    return {"workload": "complex RBM N=16 M=32 on the 16-site periodic Heisenberg chain, n_s=1024 chains, "
                        f"{sweeps * N} exchange steps per chain per iteration, lambda={lam}, eta={eta}",
            "ms_per_iteration": ms, "iterations_per_s": 1e3 / ms, "iterations_timed": iters,
            "energy_first": energies[0], "energy_last": energies[-1], "exact_e0": HEISENBERG_L16_E0,
            "acceptance_last": accept / (n_s * sweeps * N), "status_ok": not bad}


def vmc_convergence(iters: int, full_qgt: bool, sweeps: int = 10, eta: float = 0.05, lam: float = 1e-4,
                    every: int = 25):
    """The device VMC loop of vmc_loop run for `iters` iterations, with block
    SR over the layer blocks W, b, a or with full-QGT SR (one block of all 560
    parameters, the same entry points); the same initial parameters, chains
    and Metropolis moves for both.  Untimed; the moves of each iteration are
    drawn and uploaded when it starts.  Returns the energy curve (mean local
    energy every `every` iterations) and the mean over the last 100
    iterations, with its relative error against the exact ground-state
    energy."""
    import torch
    import paper_2510_08430_amd as qgt
    from gen import workloads as W
    N, M, n_s = 16, 32, 1024
    n_p = M * N + M + N
    theta = torch.from_numpy(W.rbm_network(N=N, M=M, config=0).flat()).cuda()
    x = torch.from_numpy(W.zero_magnetisation_samples(W.rng(0, W.P_SAMPLES), n_s, N)).cuda()
    O = torch.empty((n_s, n_p), dtype=torch.complex128, device="cuda")
    ws = torch.empty(qgt.rbm_jacobian_workspace_bytes(N, M, n_s), dtype=torch.uint8, device="cuda")
    delta = torch.empty(n_p, dtype=torch.complex128, device="cuda")
    e = torch.empty(n_s, dtype=torch.complex128, device="cuda")
    sr = qgt.BlockSR([(n_s, [n_p] if full_qgt else [M * N, M, N], lam)], "c128", "fp64", 0)
    energies = []
    t0 = time.perf_counter()
    for it in range(iters):
        p, u = W.mcmc_moves(0, it, sweeps * N, n_s, N)
        qgt.rbm_metropolis(theta, x, M, torch.from_numpy(p).cuda(), torch.from_numpy(u).cuda())
        qgt.rbm_heisenberg_eloc(theta, x, M, e_loc=e)
        qgt.rbm_jacobian(theta, x, M, O=O, workspace=ws)
        sr.form([O], [e])
        sr.solve([delta])
        qgt.sr_update(theta, delta, eta)
        energies.append(e.mean().real)
    energies = torch.stack(energies).cpu().numpy()
    wall = time.perf_counter() - t0
    bad = any(sr.status())
    del sr
    tail = float(energies[-100:].mean())
    return {"qgt": "full" if full_qgt else "block (W, b, a)", "eta": eta, "lambda": lam, "iterations": iters,
            "wall_s": wall,
            "energy_curve": [[i, float(energies[i])] for i in range(0, iters, every)] + [[iters - 1,
                                                                                         float(energies[-1])]],
            "energy_last100_mean": tail, "exact_e0": HEISENBERG_L16_E0,
            "rel_err_last100": abs(tail - HEISENBERG_L16_E0) / abs(HEISENBERG_L16_E0), "status_ok": not bad}


def vendor_bf16_gemm(sr, probs, reps=10):
    """torch.matmul in BF16 (hipBLASLt) on the real GEMM one BF16 Gram block
    amounts to: m x m output, contraction 2 x the block's contraction length
    (the real and imaginary planes), both operands contiguous along the
    contraction as in the Gram.  A practical ceiling for the matrix cores on
    this chip under the same kind of load; flops counted as 2 m^2 k."""
    import torch
    best = None
    for g in range(sr.num_blocks):
        b = sr.block_info(g)
        if b["precision"] != "bf16":
            continue
        n_s, n_b = int(probs[b["problem"]][0]), int(b["size"])
        m, k = (n_s, 2 * n_b) if b["form"] == "S" else (n_b, 2 * n_s)
        if best is None or m * m * k > best[0] * best[0] * best[1]:
            best = (m, k)
    if best is None:
        return None
    m, k = best
    a = torch.randn(m, k, dtype=torch.bfloat16, device="cuda")
    bt = torch.randn(m, k, dtype=torch.bfloat16, device="cuda")
    for _ in range(3):
        a @ bt.t()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        a @ bt.t()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, bt
    torch.cuda.empty_cache()
    return {"shape": f"{m}x{m}x{k}", "ms": ms, "tflops": 2.0 * m * m * k / (ms * 1e-3) / 1e12,
            "peak_tflops": PEAK["bf16"]}


def vendor_full(O, e, lam, reps=3):
    """torch.linalg FP64 full-QGT solve (rocBLAS/rocSOLVER) as a cross-check."""
    import torch
    n_s, n_p = O.shape

    def once():
        Od = O.to(torch.complex128)
        dO = Od - Od.mean(0, keepdim=True)
        dE = e - e.mean()
        if n_s < n_p:
            T = (dO @ dO.conj().T) / n_s
            T.diagonal().add_(lam)
            L = torch.linalg.cholesky(T)
            z = torch.cholesky_solve(dE[:, None], L)[:, 0]
            return dO.conj().T @ z / n_s
        S = (dO.conj().T @ dO) / n_s
        S.diagonal().add_(lam)
        L = torch.linalg.cholesky(S)
        return torch.cholesky_solve((dO.conj().T @ dE / n_s)[:, None], L)[:, 0]

    once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        once()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    return {"steps_per_s": 1.0 / t, "ms_per_step": 1e3 * t}


if __name__ == "__main__":
    main()
