"""GPU parity at the full sizes of the larger workloads, in the plans the
benchmark times (default precision per block, at most six CG iterations with
the convergence test at 1e-5), against the FP64 oracle.

* CNN 10x10, n_s = 8192 (blocks 160, 2320, 2320, 2320): every block against
  the Cholesky form of the oracle.
* 64 uneven blocks with column decay, n_s = 8192, lambda = 1e-5: the blocks
  are independent, so a sample of them (every block with n_b <= 2600: FP64
  Grams and the smaller FP32 ones) is solved by the oracle and compared; every
  block must report convergence.
* FFNN 100-400-400, n_s = 8192: both sample-form blocks (40400 and 160400
  columns, BF16 Grams, FP32 factors) against the oracle.

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


def gpu_solve(qgt, w, refine=6):
    O = torch.from_numpy(np.ascontiguousarray(w.O)).cuda()
    e = torch.from_numpy(w.e_loc).cuda()
    sr = qgt.BlockSR([(w.n_s, w.block_sizes, w.lam)], "c64", "auto", refine, rtol=1e-5)
    d = sr([O], [e])[0].cpu().numpy()
    st = sr.status()
    info = [sr.block_info(g)["precision"] for g in range(len(w.block_sizes))]
    its = [sr.cg_iterations(g) for g in range(len(w.block_sizes))]
    sr.close()
    del O, e
    torch.cuda.empty_cache()
    return d, st, info, its


def test_cnn_full_size(gpu_lib):
    say("case: CNN 10x10, n_s=8192 full size, default precision, CG <= 6 at 1e-5")
    t0 = time.perf_counter()
    w = workloads.config2_cnn()
    say(f"  generated in {time.perf_counter() - t0:.1f} s")
    d, st, prec, its = gpu_solve(gpu_lib, w)
    say(f"  precisions {prec}, CG iterations {its}, status {st}")
    assert all(v == 0 for v in st)
    t0 = time.perf_counter()
    ref = orc.block_sr_cholesky(w.O, w.e_loc, w.block_sizes, w.lam)
    say(f"  oracle {time.perf_counter() - t0:.1f} s")
    e = orc.block_relative_errors(d, ref, w.block_sizes)
    say(f"  per-block rel err {['%.2e' % v for v in e]}")
    assert max(e) <= 1e-5


def test_uneven_blocks_full_size_sampled(gpu_lib):
    say("case: 64 uneven decayed blocks, n_s=8192 full size, default precision; blocks n_b <= 2600 vs oracle")
    t0 = time.perf_counter()
    w = workloads.config3()
    say(f"  generated in {time.perf_counter() - t0:.1f} s (n_p = {w.n_p})")
    d, st, prec, its = gpu_solve(gpu_lib, w)
    bad = {g: v for g, v in enumerate(st) if v != 0}
    say(f"  precisions {sorted(set(prec))}, CG iterations {sorted(set(its))}, non-zero status {bad}")
    assert not bad
    offs = orc.block_offsets(w.block_sizes)
    sample = [b for b, nb in enumerate(w.block_sizes) if nb <= 2600]
    t0 = time.perf_counter()
    worst = {}
    for b in sample:
        lo, hi = offs[b], offs[b + 1]
        ref = orc.block_sr_cholesky(w.O[:, lo:hi], w.e_loc, [hi - lo], w.lam)
        worst[prec[b]] = max(worst.get(prec[b], 0.0), orc.relative_error(d[lo:hi], ref))
    say(f"  {len(sample)} sampled blocks, oracle {time.perf_counter() - t0:.1f} s, "
        f"max rel err per Gram precision {({k: '%.2e' % v for k, v in worst.items()})}")
    assert set(worst) == {"fp32", "fp64"}
    assert max(worst.values()) <= 1e-5


def test_wide_ffnn_full_size(gpu_lib):
    say("case: FFNN 100-400-400, n_s=8192 full size, default precision; both blocks vs oracle")
    t0 = time.perf_counter()
    w = workloads.config2_ffnn()
    say(f"  generated in {time.perf_counter() - t0:.1f} s")
    d, st, prec, its = gpu_solve(gpu_lib, w)
    say(f"  precisions {prec}, CG iterations {its}, status {st}")
    assert all(v == 0 for v in st)
    offs = orc.block_offsets(w.block_sizes)
    for b in range(len(w.block_sizes)):
        lo, hi = offs[b], offs[b + 1]
        t0 = time.perf_counter()
        ref = orc.block_sr_cholesky(w.O[:, lo:hi], w.e_loc, [hi - lo], w.lam)
        err = orc.relative_error(d[lo:hi], ref)
        say(f"  block {b} ({hi - lo} columns): oracle {time.perf_counter() - t0:.1f} s, rel err {err:.2e}")
        del ref
        assert err <= 1e-5
