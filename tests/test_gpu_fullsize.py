"""GPU parity at the full sizes of the larger workloads, in the plans the
benchmark times and with the default precision per block (at most six CG
iterations with the convergence test at 1e-5), against the FP64 oracle.

* CNN 10x10, n_s = 8192 (blocks 160, 2320, 2320, 2320): every block against
  the Cholesky form of the oracle, with the default precisions and with BF16
  Grams for every block (the benchmark's plan).
* 64 uneven blocks with column decay, n_s = 8192, lambda = 1e-5: every block
  against the oracle (GPU solves with the default precisions under each way
  of launching the Cholesky, and with BF16 Grams for every block, the
  benchmark's plan; the oracle's blocks split over six tests),
  and the largest block (n_b = 8156) also against the eigendecomposition form;
  every block must report convergence.
* FFNN 100-400-400, n_s = 8192: both sample-form blocks (40400 and 160400
  columns, BF16 Grams) against the oracle, with the FP64 factor (default) and
  the FP32 factor.

The oracle is the Cholesky form of the block oracle (pinned against the
eigendecomposition form on the CPU); the error is the per-block relative
2-norm error of delta.
"""
import sys
import time

import numpy as np
import pytest

from gen import workloads
from oracle import block_sr as orc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_solve(qgt, w, refine=6, factor="fp64", cholesky="auto", gram="auto"):
    O = torch.from_numpy(np.ascontiguousarray(w.O)).cuda()
    e = torch.from_numpy(w.e_loc).cuda()
    sr = qgt.BlockSR([(w.n_s, w.block_sizes, w.lam)], "c64", gram, refine, rtol=1e-5, factor=factor,
                     cholesky=cholesky)
    d = sr([O], [e])[0].cpu().numpy()
    st = sr.status()
    info = [sr.block_info(g)["precision"] for g in range(len(w.block_sizes))]
    its = [sr.cg_iterations(g) for g in range(len(w.block_sizes))]
    sr.close()
    del O, e
    torch.cuda.empty_cache()
    return d, st, info, its


def test_cnn_full_size(gpu_lib):
    say("case: CNN 10x10, n_s=8192 full size, default precision and BF16 Grams, CG <= 6 at 1e-5")
    t0 = time.perf_counter()
    w = workloads.config2_cnn()
    say(f"  generated in {time.perf_counter() - t0:.1f} s")
    runs = {}
    for gram in ("auto", "bf16"):
        d, st, prec, its = gpu_solve(gpu_lib, w, cholesky="host-steps", gram=gram)
        say(f"  {gram}: precisions {prec}, CG iterations {its}, status {st}")
        assert all(v == 0 for v in st)
        runs[gram] = d
    t0 = time.perf_counter()
    ref = orc.block_sr_cholesky(w.O, w.e_loc, w.block_sizes, w.lam)
    say(f"  oracle {time.perf_counter() - t0:.1f} s")
    for gram, d in runs.items():
        e = orc.block_relative_errors(d, ref, w.block_sizes)
        say(f"  {gram}: per-block rel err {['%.2e' % v for v in e]}")
        assert max(e) <= 1e-5


@pytest.fixture(scope="module")
def uneven(gpu_lib):
    """The 64 uneven decayed blocks at full size, solved once on the GPU in the
    benchmark's plan."""
    say("case: 64 uneven decayed blocks, n_s=8192 full size, default precision, CG <= 6 at 1e-5")
    t0 = time.perf_counter()
    w = workloads.config3()
    say(f"  generated in {time.perf_counter() - t0:.1f} s (n_p = {w.n_p})")
    d, st, prec, its = gpu_solve(gpu_lib, w)
    bad = {g: v for g, v in enumerate(st) if v != 0}
    say(f"  precisions {sorted(set(prec))}, CG iterations {sorted(set(its))}, non-zero status {bad}")
    dp, stp, _, itp = gpu_solve(gpu_lib, w, cholesky="persistent")
    say(f"  persistent Cholesky: CG iterations {sorted(set(itp))}, non-zero status "
        f"{ {g: v for g, v in enumerate(stp) if v != 0} }")
    db, stb, _, itb = gpu_solve(gpu_lib, w, gram="bf16")
    say(f"  BF16 Grams: CG iterations {sorted(set(itb))}, non-zero status "
        f"{ {g: v for g, v in enumerate(stb) if v != 0} }")
    return (w, {"host-steps": d, "persistent": dp, "bf16": db}, [max(a, b, c) for a, b, c in zip(st, stp, stb)],
            prec)


def _uneven_groups(sizes, n_groups=6):
    """The blocks split into groups of about equal oracle cost (Gram flops
    n_s n_b^2 plus the factorisation n_b^3), largest blocks first."""
    order = sorted(range(len(sizes)), key=lambda b: -sizes[b])
    cost = [8192.0 * sizes[b] ** 2 + sizes[b] ** 3 / 3.0 for b in range(len(sizes))]
    groups, acc = [[] for _ in range(n_groups)], [0.0] * n_groups
    for b in order:
        i = min(range(n_groups), key=lambda j: acc[j])
        groups[i].append(b)
        acc[i] += cost[b]
    return [sorted(g) for g in groups]


@pytest.mark.parametrize("group", range(6))
def test_uneven_blocks_full_size(uneven, group):
    """Every one of the 64 blocks (FP64 and FP32 Grams by default, BF16 Grams in
    the benchmark's plan; FP64 factors up to order 8192, condition numbers up
    to ~1e8 from the column decay) against the Cholesky form of the oracle, a
    sixth of them per test."""
    w, runs, st, prec = uneven
    assert all(v == 0 for v in st)
    offs = orc.block_offsets(w.block_sizes)
    blocks = _uneven_groups(w.block_sizes)[group]
    say(f"case: uneven blocks, group {group}: blocks {blocks}")
    for b in blocks:
        lo, hi = offs[b], offs[b + 1]
        t0 = time.perf_counter()
        ref = orc.block_sr_cholesky(w.O[:, lo:hi], w.e_loc, [hi - lo], w.lam)
        errs = {k: orc.relative_error(d[lo:hi], ref) for k, d in runs.items()}
        say(f"  block {b} (n_b={hi - lo}, {prec[b]} Gram): oracle {time.perf_counter() - t0:.1f} s, rel err "
            + ", ".join(f"{k} {e:.2e}" for k, e in errs.items()))
        assert max(errs.values()) <= 1e-5


def test_uneven_largest_block_eigh(uneven):
    """The largest block (n_b = 8156) against the oracle's definition itself
    (eigendecomposition with the spectral cutoff, nothing cut)."""
    w, runs, st, prec = uneven
    b = max(range(len(w.block_sizes)), key=lambda i: w.block_sizes[i])
    offs = orc.block_offsets(w.block_sizes)
    lo, hi = offs[b], offs[b + 1]
    say(f"case: uneven blocks, largest block {b} (n_b={hi - lo}) vs the eigendecomposition oracle")
    t0 = time.perf_counter()
    ref = orc.block_sr(w.O[:, lo:hi], w.e_loc, [hi - lo], w.lam)
    errs = {k: orc.relative_error(d[lo:hi], ref.delta) for k, d in runs.items()}
    say(f"  oracle {time.perf_counter() - t0:.1f} s, kappa {ref.kappa[0]:.2e}, cut {ref.n_cut[0]}, rel err "
        + ", ".join(f"{k} {e:.2e}" for k, e in errs.items()))
    assert ref.n_cut[0] == 0
    assert max(errs.values()) <= 1e-5


def test_wide_ffnn_full_size(gpu_lib):
    say("case: FFNN 100-400-400, n_s=8192 full size, default precision; both blocks vs oracle, FP64 and FP32 factor")
    t0 = time.perf_counter()
    w = workloads.config2_ffnn()
    say(f"  generated in {time.perf_counter() - t0:.1f} s")
    runs = {}
    for factor in ("fp64", "fp32"):
        d, st, prec, its = gpu_solve(gpu_lib, w, factor=factor)
        say(f"  factor {factor}: precisions {prec}, CG iterations {its}, status {st}")
        assert all(v == 0 for v in st)
        runs[factor] = d
    offs = orc.block_offsets(w.block_sizes)
    for b in range(len(w.block_sizes)):
        lo, hi = offs[b], offs[b + 1]
        t0 = time.perf_counter()
        ref = orc.block_sr_cholesky(w.O[:, lo:hi], w.e_loc, [hi - lo], w.lam)
        errs = {f: orc.relative_error(d[lo:hi], ref) for f, d in runs.items()}
        say(f"  block {b} ({hi - lo} columns): oracle {time.perf_counter() - t0:.1f} s, rel err "
            + ", ".join(f"{f} factor {e:.2e}" for f, e in errs.items()))
        del ref
        assert max(errs.values()) <= 1e-5
