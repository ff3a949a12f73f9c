"""GPU parity on the benchmark workloads, against the FP64 oracle.

* Chain FFNN 64-128-128-64 + readout, n_s = 4096 (the benchmark workload, full
  size, in the plans the benchmark times): FP32, BF16 and default-precision
  Grams with one or two FP64 CG iterations, the FP64 Gram, and the one-block
  full-QGT FP64 solve.
* RBM N=16 M=32, n_s = 1024, FP64 (full size).
* CNN 10x10, 4 conv layers, n_s = 4096 (all blocks in parameter form, as at
  the full n_s = 8192), BF16 and FP32 Grams + CG.
* FFNN 100-400-400 (blocks 40400 and 160400), n_s = 1024 (sample form, as at
  full size), BF16 Gram + CG.
* Uneven blocks with column decay (16 blocks log-uniform in [64, 2048],
  n_s = 2048, lambda = 1e-5), FP32 and BF16 Grams + CG.
* 32 independent chain instances in one plan (n_s = 1024 each), default
  precision + CG, per-instance error.

The oracle here is the Cholesky form of the block oracle (pinned against the
eigendecomposition form on the CPU) where the blocks are large; the error
measure is the per-block relative 2-norm error of delta.
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


def solve(qgt, ws, gram, refine, forms=None):
    """One plan over all workloads ws; returns delta per workload (numpy)."""
    dt = "c64" if ws[0].O.dtype == np.complex64 else "c128"
    say(f"  gpu: {len(ws)} problem(s), gram={gram} refine={refine} dtype={dt}")
    Os = [torch.from_numpy(np.ascontiguousarray(w.O)).cuda() for w in ws]
    Es = [torch.from_numpy(w.e_loc.astype(np.complex128)).cuda() for w in ws]
    sr = qgt.BlockSR([(w.n_s, w.block_sizes, w.lam) for w in ws], dt, gram, refine, forms=forms)
    out = [d.cpu().numpy() for d in sr(Os, Es)]
    st = sr.status()
    bad = {g: v for g, v in enumerate(st) if v != 0}
    if bad:
        say(f"  non-zero block status {bad}")
    assert not bad, bad
    sr.close()
    del Os, Es
    torch.cuda.empty_cache()
    return out


def oracle(w, key, cache):
    if key not in cache:
        t0 = time.perf_counter()
        cache[key] = orc.block_sr_cholesky(w.O, w.e_loc, w.block_sizes, w.lam)
        say(f"  oracle {key}: {time.perf_counter() - t0:.1f} s")
    return cache[key]


def errs(d, ref, sizes):
    return orc.block_relative_errors(d, ref, sizes)


@pytest.fixture(scope="module")
def cache():
    return {}


@pytest.fixture(scope="module")
def chain64():
    say("generating the chain FFNN workload (n_s=4096, blocks 8320/16512/8256/65)")
    return workloads.config1(o_dtype=np.complex64)


@pytest.mark.parametrize("gram,refine,tol", [("bf16", 2, 1e-5), ("fp32", 2, 1e-5), ("auto", 1, 1e-5),
                                             ("auto", 2, 1e-5), ("fp64", 0, 1e-10)])
def test_chain_ffnn_full_size(gpu_lib, chain64, cache, gram, refine, tol):
    say(f"case: chain FFNN n_s=4096 full size, {gram} Gram, {refine} CG iterations")
    w = chain64
    ref = oracle(w, "chain64", cache)
    d = solve(gpu_lib, [w], gram, refine)[0]
    e = errs(d, ref, w.block_sizes)
    say(f"  per-block rel err {['%.2e' % v for v in e]}")
    assert max(e) <= tol


def test_chain_ffnn_full_qgt_fp64(gpu_lib, chain64, cache):
    say("case: chain FFNN n_s=4096, one-block full-QGT FP64 solve (sample form 4096)")
    w = chain64
    if "chain64_full" not in cache:
        t0 = time.perf_counter()
        cache["chain64_full"] = orc.block_sr_cholesky(w.O, w.e_loc, [w.n_p], w.lam)
        say(f"  oracle full: {time.perf_counter() - t0:.1f} s")
    O = torch.from_numpy(w.O).cuda()
    e = torch.from_numpy(w.e_loc).cuda()
    d = gpu_lib.full_solve(O, e, w.lam).cpu().numpy()
    err = orc.relative_error(d, cache["chain64_full"])
    say(f"  rel err {err:.2e}")
    assert err <= 1e-10


def test_rbm_full_size_fp64(gpu_lib, cache):
    say("case: RBM N=16 M=32 n_s=1024 full size, FP64")
    w = workloads.config0()
    ref = orc.block_sr(w.O, w.e_loc, w.block_sizes, w.lam).delta
    for refine in (0, 1):
        d = solve(gpu_lib, [w], "fp64", refine)[0]
        e = errs(d, ref, w.block_sizes)
        say(f"  refine={refine}: per-block rel err {['%.2e' % v for v in e]}")
        assert max(e) <= 1e-10


def test_cnn_bf16_refined(gpu_lib, cache):
    """All four CNN blocks are parameter-space blocks with heavy-tailed columns
    (tanh near its poles) and lambda = 1e-4: the BF16 Gram alone is ~3e-2 off on
    the 2320-blocks, above the 1e-2 stated for BF16 before refinement, and the
    CG iteration needs five steps to reach 1e-5.  The FP32 Gram needs two."""
    say("case: CNN 10x10, n_s=4096 (all parameter form), BF16 Gram + CG, FP32 Gram + CG")
    w = workloads.config2_cnn(n_s=4096)
    ref = oracle(w, "cnn", cache)
    d0 = solve(gpu_lib, [w], "bf16", 0)[0]
    d5 = solve(gpu_lib, [w], "bf16", 5)[0]
    d2 = solve(gpu_lib, [w], "fp32", 2)[0]
    e0, e5, e2 = (max(errs(d, ref, w.block_sizes)) for d in (d0, d5, d2))
    say(f"  BF16: before CG {e0:.2e}, after 5 steps {e5:.2e}; FP32 after 2 steps {e2:.2e}")
    assert e0 <= 5e-2
    assert e5 <= 1e-5
    assert e2 <= 1e-5


def test_wide_ffnn_sample_form_bf16(gpu_lib, cache):
    say("case: FFNN 100-400-400, n_s=1024 (blocks 40400 and 160400, sample form), BF16 + CG")
    w = workloads.config2_ffnn(n_s=1024)
    ref = oracle(w, "wide", cache)
    d0 = solve(gpu_lib, [w], "bf16", 0)[0]
    d3 = solve(gpu_lib, [w], "bf16", 4)[0]
    e0, e3 = max(errs(d0, ref, w.block_sizes)), max(errs(d3, ref, w.block_sizes))
    say(f"  before CG {e0:.2e}, after 4 steps {e3:.2e}")
    assert e0 <= 1e-2
    assert e3 <= 1e-5


@pytest.mark.parametrize("gram,refine", [("fp32", 2), ("bf16", 5)])
def test_uneven_decay_blocks(gpu_lib, cache, gram, refine):
    say(f"case: 16 uneven blocks with column decay, n_s=2048, lambda=1e-5, {gram} + {refine} CG iterations")
    w = workloads.config3(n_s=2048, n_blocks=16, lo=64, hi=2048)
    ref = oracle(w, "uneven", cache)
    d = solve(gpu_lib, [w], gram, refine)[0]
    e = errs(d, ref, w.block_sizes)
    say(f"  max per-block rel err {max(e):.2e} (blocks {w.block_sizes})")
    assert max(e) <= 1e-5


def test_many_instances_batched(gpu_lib, cache):
    """32 instances in one plan.  The first-layer blocks of the N=16 chains are
    parameter-space blocks with 32 exact null directions (zero magnetisation):
    kappa(S~) ~ 2e6 at lambda = 1e-4, beyond what a BF16 Gram resolves, and an
    FP32 Gram can even lose positive definiteness there (the pivot floor keeps
    the factor usable).  The default precision (FP32 on parameter-space, BF16
    on sample-space blocks) with four CG iterations meets 1e-5 per instance."""
    say("case: 32 chain instances in one plan (n_s=1024 each), auto precision + 4 CG iterations")
    ws = [workloads.config4_instance(i, n_s_override=1024) for i in range(32)]
    ds = solve(gpu_lib, ws, "auto", 4)
    worst = 0.0
    for i, (w, d) in enumerate(zip(ws, ds)):
        ref = orc.block_sr_cholesky(w.O, w.e_loc, w.block_sizes, w.lam)
        e = max(errs(d, ref, w.block_sizes))
        say(f"  instance {i} ({w.name}, blocks {w.block_sizes}): {e:.2e}")
        worst = max(worst, e)
    say(f"  worst instance error {worst:.2e}")
    assert worst <= 1e-5


def test_many_instances_full_size_sampled(gpu_lib, cache):
    """The 32-instance stream at its full sizes (n_s in {1024, 2048, 4096}), in
    the plan the benchmark times (default precision, four CG iterations,
    convergence test at 1e-5): every block reports convergence, and six sampled
    instances covering every form and precision are checked against the
    oracle."""
    say("case: 32 chain instances, full sizes, one plan; sampled instances vs oracle")
    ws = [workloads.config4_instance(i) for i in range(32)]
    Os = [torch.from_numpy(np.ascontiguousarray(w.O)).cuda() for w in ws]
    Es = [torch.from_numpy(w.e_loc).cuda() for w in ws]
    sr = gpu_lib.BlockSR([(w.n_s, w.block_sizes, w.lam) for w in ws], "c64", "auto", 4, rtol=1e-5)
    ds = [d.cpu().numpy() for d in sr(Os, Es)]
    st = sr.status()
    bad = {g: v for g, v in enumerate(st) if v != 0}
    say(f"  precisions {sr.precisions()}, non-zero status {bad}")
    assert not bad
    for i in (1, 6, 10, 4, 11, 14):
        w = ws[i]
        ref = orc.block_sr_cholesky(w.O, w.e_loc, w.block_sizes, w.lam)
        info = [sr.block_info(2 * i + b) for b in range(2)]
        e = max(errs(ds[i], ref, w.block_sizes))
        say(f"  instance {i} ({w.name}, n_s={w.n_s}, {[x['form'] + x['precision'] for x in info]}): {e:.2e}")
        assert e <= 1e-5
    sr.close()
