"""GPU checks of the intermediate results of each step against the oracle or
against an exact emulation of the step's rounding:

* the per-block trace of the column pass,
* the centred and rounded Gram operand, bit for bit (FP64, FP32 and BF16,
  parameter and sample form),
* the FP32 and BF16 Grams against the FP64 Gram of the same rounded operand,
  within the worst-case bound of FP32 accumulation (this separates the
  rounding of the operand from the accumulation), including the rank-one
  term that keeps the constant vector away from the rounding level in
  low-precision sample-space Grams,
* the FP64 Cholesky factor: L L^H reproduces the oracle's shifted block; the
  FP64 (default) and FP32 factors of a BF16 Gram reproduce the stored Gram,
* the CG convergence test (refine_rtol) and its correction estimate,
* the automatic precision policy.
"""
import sys

import numpy as np
import pytest

from gen import workloads
from oracle import block_sr as orc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ESIZE = {"fp64": 8, "fp32": 4, "bf16": 2}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def w_ffnn_small(o_dtype=np.complex64):
    # blocks 630 (parameter form), 2343 (sample form at n_s = 600), 34 (parameter form)
    return workloads.small_ffnn(n_s=600, N=8, widths=(70, 33), readout=True, o_dtype=o_dtype, lam=1e-3)


def bind(qgt, w, gram, refine=0, factor="fp64", cholesky="auto"):
    O = torch.from_numpy(np.ascontiguousarray(w.O)).cuda()
    e = torch.from_numpy(w.e_loc.astype(np.complex128)).cuda()
    dt = "c64" if w.O.dtype == np.complex64 else "c128"
    say(f"  plan {w.name} n_s={w.n_s} blocks={w.block_sizes} dtype={dt} gram={gram} refine={refine} "
        f"factor={factor} cholesky={cholesky}")
    return qgt.BlockSR([(w.n_s, w.block_sizes, w.lam)], dt, gram, refine, factor=factor, cholesky=cholesky), O, e


def round_bf16(x):
    """Round float64 values to bfloat16, nearest-even, in one rounding (normal range)."""
    m, e = np.frexp(x)
    return np.ldexp(np.rint(m * 256.0), e - 8)


def bits(x, prec):
    if prec == "fp64":
        return np.asarray(x, dtype=np.float64).view(np.uint64)
    if prec == "fp32":
        return np.asarray(x, dtype=np.float32).view(np.uint32)
    return (np.asarray(round_bf16(x), dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16)


def rounded(x, prec):
    if prec == "fp64":
        return np.asarray(x, dtype=np.float64)
    if prec == "fp32":
        return np.asarray(x, dtype=np.float32).astype(np.float64)
    return round_bf16(x)


def read_pack(sr, g, prec, K, m):
    """Unpack the planar, 16-byte-grouped Gram operand of block g into two
    (K, m) arrays of raw element bits (and the whole padded planes)."""
    es = ESIZE[prec]
    G = 16 // es
    _, m_pad = sr.debug_bytes(4, g, 0)
    K_pad = -(-K // (4 * G)) * (4 * G)
    assert m_pad == -(-m // 128) * 128
    raw, _ = sr.debug_bytes(4, g, 2 * K_pad * m_pad * es)
    udt = {8: np.uint64, 4: np.uint32, 2: np.uint16}[es]
    a = raw.cpu().numpy().view(udt)
    planes = []
    for p in range(2):
        pl = a[p * K_pad * m_pad:(p + 1) * K_pad * m_pad].reshape(K_pad // G, m_pad, G)
        planes.append(pl.transpose(0, 2, 1).reshape(K_pad, m_pad))
    return planes


def test_block_trace(gpu_lib):
    for w in (workloads.config0(n_s=320), w_ffnn_small()):
        say(f"case: per-block trace of the QGT ({w.name})")
        sr, O, e = bind(gpu_lib, w, "fp64" if w.O.dtype == np.complex128 else "fp32")
        sr.form([O], [e])
        torch.cuda.synchronize()
        offs = orc.block_offsets(w.block_sizes)
        for g in range(len(w.block_sizes)):
            blk = w.O[:, offs[g]:offs[g + 1]].astype(np.complex128)
            ref = float(np.trace(orc.qgt_block(orc.centred_block(w.O, offs[g], offs[g + 1]))).real)
            scale = float(np.sum(np.abs(blk) ** 2)) / w.n_s
            got = sr.block_trace(g)
            say(f"  block {g}: trace {got:.6e} vs {ref:.6e}")
            assert abs(got - ref) <= 1e-13 * scale


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_packed_operand_bit_exact(gpu_lib, prec):
    """The centred operand is formed in FP64 from the input and the column
    means, then rounded once to nearest-even at the Gram precision."""
    say(f"case: packed Gram operand, bit exact ({prec})")
    w = w_ffnn_small()
    sr, O, e = bind(gpu_lib, w, prec)
    sr.form([O], [e])
    torch.cuda.synchronize()
    mu, _ = sr.debug_tensor(0, 0, w.n_p)
    mu = mu.cpu().numpy()
    offs = orc.block_offsets(w.block_sizes)
    Od = w.O.astype(np.complex128)
    for g, nb in enumerate(w.block_sizes):
        info = sr.block_info(g)
        assert info["precision"] == prec
        d = Od[:, offs[g]:offs[g + 1]] - mu[offs[g]:offs[g + 1]][None, :]   # (n_s, n_b), FP64 subtraction
        if info["form"] == "P":
            K, m, re_v, im_v = w.n_s, nb, d.real, d.imag
        else:
            K, m, re_v, im_v = nb, w.n_s, d.real.T, -d.imag.T
        re, im = read_pack(sr, g, prec, K, m)
        say(f"  block {g} ({info['form']}): K={K} m={m} padded {re.shape}")
        np.testing.assert_array_equal(re[:K, :m], bits(re_v, prec))
        np.testing.assert_array_equal(im[:K, :m], bits(im_v, prec))
        # padding rows and columns hold zeros (of either sign)
        zero_mask = np.uint64(0x7FFFFFFFFFFFFFFF) if prec == "fp64" else (
            np.uint32(0x7FFFFFFF) if prec == "fp32" else np.uint16(0x7FFF))
        for pl in (re, im):
            assert not np.any(pl[K:, :] & zero_mask) and not np.any(pl[:, m:] & zero_mask)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_low_precision_gram_matches_rounded_operand(gpu_lib, prec):
    """Gram of the rounded operand: |G_gpu - G_exact| <= gamma (|A|^H |A|) / n_s
    entrywise with gamma = (2 K + 2) 2^-24 (FP32 sums of 2K products, plus the
    rounding of the products themselves in FP32 mode), G_exact the FP64 Gram of
    the emulated rounded operand.  A random-sign rounding model would give far
    smaller errors; this is the deterministic worst case."""
    say(f"case: {prec} Gram vs FP64 Gram of the rounded operand")
    w = w_ffnn_small()
    sr, O, e = bind(gpu_lib, w, prec)
    sr.form([O], [e])
    torch.cuda.synchronize()
    mu, _ = sr.debug_tensor(0, 0, w.n_p)
    mu = mu.cpu().numpy()
    offs = orc.block_offsets(w.block_sizes)
    Od = w.O.astype(np.complex128)
    for g, nb in enumerate(w.block_sizes):
        info = sr.block_info(g)
        d = Od[:, offs[g]:offs[g + 1]] - mu[offs[g]:offs[g + 1]][None, :]
        A = rounded(d.real, prec) + 1j * rounded(d.imag, prec)          # (n_s, n_b)
        if info["form"] == "P":
            Gx, Gabs, K = A.conj().T @ A, np.abs(A).T @ np.abs(A), w.n_s
        else:
            Gx, Gabs, K = A @ A.conj().T, np.abs(A) @ np.abs(A).T, nb
        m = Gx.shape[0]
        Gx = Gx / w.n_s + w.lam * np.eye(m)
        if info["form"] == "S":
            # rank-one term (t_b / n_s) 11^T / n_s on low-precision sample-space Grams
            Gx = Gx + sr.block_trace(g) / (w.n_s * w.n_s)
        bound = (2 * K + 2) * 2.0 ** -24 * Gabs / w.n_s + 1e-15 * np.abs(Gx)
        Gg = sr.block_matrix(g)
        low = np.tril_indices(m)
        err, bnd = np.abs(Gg[low] - Gx[low]), bound[low]
        zero = bnd == 0            # e.g. a column that is constant over the samples
        assert np.all(err[zero] == 0)
        ratio = (err[~zero] / bnd[~zero]).max()
        say(f"  block {g} ({info['form']}, m={m}): max |err| / bound = {ratio:.3f}")
        assert ratio <= 1.0


@pytest.mark.parametrize("cholesky", ["host-steps", "persistent"])
def test_cholesky_factor_fp64(gpu_lib, cholesky):
    """After the solve the block matrix holds its FP64 Cholesky factor: lower
    triangular, positive real diagonal, and L L^H equal to the oracle's
    shifted block to rounding (both ways of launching the factorisation)."""
    say(f"case: FP64 Cholesky factor vs oracle shifted block, {cholesky}")
    w = w_ffnn_small(np.complex128)
    sr, O, e = bind(gpu_lib, w, "fp64", cholesky=cholesky)
    d = torch.empty(w.n_p, dtype=torch.complex128, device="cuda")
    sr.form([O], [e])
    sr.solve([d])
    torch.cuda.synchronize()
    assert all(s == 0 for s in sr.status())
    offs = orc.block_offsets(w.block_sizes)
    for g, nb in enumerate(w.block_sizes):
        info = sr.block_info(g)
        dO = orc.centred_block(w.O, offs[g], offs[g + 1])
        A = orc.qgt_block(dO) if info["form"] == "P" else orc.sample_space_matrix(dO)
        A = A + w.lam * np.eye(A.shape[0])
        m = A.shape[0]
        L = np.tril(sr.block_matrix(g))
        dg = np.diag(L)
        assert np.all(dg.imag == 0) and np.all(dg.real > 0)
        err = np.abs(L @ L.conj().T - A).max() / np.abs(A).max()
        say(f"  block {g} ({info['form']}, m={m}): max |L L^H - S~| / max|S~| = {err:.2e}")
        assert err <= 1e-13


@pytest.mark.parametrize("factor,cholesky", [("fp64", "host-steps"), ("fp32", "host-steps"), ("fp64", "persistent"),
                                             ("fp32", "persistent")])
def test_cholesky_factor_of_bf16_gram(gpu_lib, factor, cholesky):
    """A BF16 Gram is stored in complex128 and factored in FP64 (the default),
    or, when the plan asks for it, stored in complex64 and factored in FP32:
    after the solve the block matrix holds a lower-triangular factor with a
    positive real diagonal whose L L^H reproduces the stored Gram to the
    factor's rounding (relative to its largest entry: 1e-13 in FP64, a few units
    of 2^-24 times sqrt(m) in FP32)."""
    say(f"case: {factor} Cholesky factor of BF16 Grams vs the stored Gram, {cholesky}")
    w = w_ffnn_small(np.complex128)
    sr, O, e = bind(gpu_lib, w, "bf16", factor=factor, cholesky=cholesky)
    assert all(sr.block_info(g)["factor"] == factor for g in range(len(w.block_sizes)))
    sr.form([O], [e])
    torch.cuda.synchronize()
    G = [sr.block_matrix(g) for g in range(len(w.block_sizes))]
    d = torch.empty(w.n_p, dtype=torch.complex128, device="cuda")
    sr.solve([d])
    torch.cuda.synchronize()
    assert all(s == 0 for s in sr.status())
    for g in range(len(w.block_sizes)):
        m = G[g].shape[0]
        A = np.tril(G[g]) + np.tril(G[g], -1).conj().T
        L = np.tril(sr.block_matrix(g))
        dg = np.diag(L)
        assert np.all(dg.imag == 0) and np.all(dg.real > 0)
        err = np.abs(L @ L.conj().T - A).max() / np.abs(A).max()
        say(f"  block {g} ({sr.block_info(g)['form']}, m={m}): max |L L^H - G| / max|G| = {err:.2e}, "
            f"pivots raised {sr.pivot_floors()[g]}")
        assert err <= (16 * np.sqrt(m) * 2.0 ** -24 if factor == "fp32" else 1e-13)
        assert sum(sr.pivot_floors()) >= 0


@pytest.mark.parametrize("gram", ["fp64", "bf16"])
def test_persistent_cholesky_is_deterministic(gpu_lib, gram):
    """Every operation on a tile of the persistent factorisation runs in a
    fixed order with a fixed summation order, so repeated factorisations of the
    same Gram are bit for bit identical; a stale read of a tile (a cache
    holding an older copy) would show up as a difference.  Two blocks of 32
    tiles each give a few thousand tile tasks per launch."""
    say(f"case: persistent Cholesky repeated, {gram} Gram, two blocks of order 2048")
    g = torch.Generator(device="cpu").manual_seed(7)
    n_s, sizes = 2048, [3000, 2500]
    O = torch.randn(n_s, sum(sizes), dtype=torch.complex128, generator=g).cuda()
    e = torch.randn(n_s, dtype=torch.complex128, generator=g).cuda()
    sr = gpu_lib.BlockSR([(n_s, sizes, 1e-3)], "c128", gram, 0, cholesky="persistent")
    d = torch.empty(sum(sizes), dtype=torch.complex128, device="cuda")
    factors = []
    for rep in range(4):
        sr.form([O], [e])
        sr.solve([d])
        torch.cuda.synchronize()
        assert all(s == 0 for s in sr.status())
        factors.append([np.tril(sr.block_matrix(b)) for b in range(len(sizes))])
    for rep in range(1, 4):
        for b in range(len(sizes)):
            diff = int(np.count_nonzero(factors[rep][b] != factors[0][b]))
            say(f"  repetition {rep} block {b}: {diff} entries differ from the first factorisation")
            assert diff == 0


def test_cg_convergence_flag_and_estimate(gpu_lib):
    """refine_rtol marks blocks whose estimated error after the CG iteration is
    above it (QGT_ERR_NOT_CONVERGED = 6) and leaves the others at 0; without
    iterations there is no estimate and no test.  The estimate tracks the true
    error of delta against the oracle."""
    say("case: CG convergence test and error estimate")
    w = w_ffnn_small(np.complex128)
    O = torch.from_numpy(w.O).cuda().to(torch.complex64)
    e = torch.from_numpy(w.e_loc).cuda()
    sizes = w.block_sizes
    ref32 = orc.block_sr(w.O.astype(np.complex64), w.e_loc, sizes, w.lam).delta
    sr = gpu_lib.BlockSR([(w.n_s, sizes, w.lam)], "c64", "bf16", 0, rtol=1e-3)
    sr([O], [e])
    assert sr.status() == [0] * len(sizes)
    sr = gpu_lib.BlockSR([(w.n_s, sizes, w.lam)], "c64", "bf16", 5, rtol=1e-5)
    d = sr([O], [e])[0].cpu().numpy()
    assert sr.status() == [0] * len(sizes), sr.status()
    errs = orc.block_relative_errors(d, ref32, sizes)
    for g in range(len(sizes)):
        est = sr.correction_estimate(g)
        say(f"  block {g}: error estimate {est:.2e}, error {errs[g]:.2e}")
        assert est <= 1e-5
        assert errs[g] <= max(10 * est, 1e-11)
    # a tolerance no iteration can meet flags every block
    sr = gpu_lib.BlockSR([(w.n_s, sizes, w.lam)], "c64", "bf16", 1, rtol=1e-30)
    sr([O], [e])
    assert sr.status() == [6] * len(sizes)


def test_auto_precision_policy(gpu_lib):
    """AUTO: FP64 for complex128 input; for complex64, BF16 on sample-space
    blocks with n_b >= 2 n_s, FP32 on the other sample-space blocks, FP64 on
    parameter-space blocks with 4 n_s n_b^2 <= 1e11 and FP32 on larger
    parameter-space blocks.  Forms: sample space iff n_s < n_b."""
    say("case: automatic form and precision per block")
    n_s = 4096
    sizes = [65, 2400, 2600, 4096, 4097, 8191, 8192]   # 4 n_s n_b^2: 6.9e7, 9.4e10, 1.1e11, 2.7e11; then S
    want = [("P", "fp64"), ("P", "fp64"), ("P", "fp32"), ("P", "fp32"), ("S", "fp32"), ("S", "fp32"),
            ("S", "bf16")]
    sr = gpu_lib.BlockSR([(n_s, sizes, 1e-3)], "c64", "auto", 1)
    got = [(sr.block_info(g)["form"], sr.block_info(g)["precision"]) for g in range(len(sizes))]
    assert got == want, got
    sr = gpu_lib.BlockSR([(n_s, sizes, 1e-3)], "c128", "auto", 1)
    got = [(sr.block_info(g)["form"], sr.block_info(g)["precision"]) for g in range(len(sizes))]
    assert got == [(f, "fp64") for f, _ in want], got


@pytest.mark.parametrize("tile", [0, 3])
@pytest.mark.parametrize("n_s,sizes", [(4096, [4100, 4096]), (1280, [2600, 1024, 1100]),
                                       (20, [16, 4]), (40, [16, 24]), (70, [70])])
def test_wide_tile_bf16_gram(n_s, sizes, tile):
    """BF16 blocks with m_pad a multiple of 256 and >= 1024 take the 256x128
    wide-tile kernel by default (the others the 128x128 kernel), or, with
    gram_tile 3, the 128x128 kernel run two workgroups per CU: same bound as
    above against the FP64 Gram of the rounded operand, on every 7th row (all
    tiles, including the diagonal band).  The small cases contract over one,
    two and three 32-deep stages (n_s = 20, 40, 70), the shortest pipelines of
    the LDS rings."""
    import paper_2510_08430_amd as qgt
    say(f"case: BF16 Gram, n_s={n_s}, blocks {sizes}, gram_tile {tile or 'default'}")
    w = workloads.random_blocks(n_s, sizes, config=8, instance=5, o_dtype=np.complex64, lam=1e-3)
    if tile:
        O = torch.from_numpy(np.ascontiguousarray(w.O)).cuda()
        e = torch.from_numpy(w.e_loc.astype(np.complex128)).cuda()
        sr = qgt.BlockSR([(w.n_s, w.block_sizes, w.lam)], "c64", "bf16", 0,
                         tuning=[{"gram_tile": tile} for _ in w.block_sizes])
        assert all(sr.block_tuning(g)["gram_tile"] == tile for g in range(sr.num_blocks))
    else:
        sr, O, e = bind(qgt, w, "bf16")
    sr.form([O], [e])
    torch.cuda.synchronize()
    mu, _ = sr.debug_tensor(0, 0, w.n_p)
    mu = mu.cpu().numpy()
    offs = orc.block_offsets(w.block_sizes)
    Od = w.O.astype(np.complex128)
    for g, nb in enumerate(w.block_sizes):
        info = sr.block_info(g)
        d = Od[:, offs[g]:offs[g + 1]] - mu[offs[g]:offs[g + 1]][None, :]
        A = rounded(d.real, "bf16") + 1j * rounded(d.imag, "bf16")
        if info["form"] == "S":
            A = A.conj().T                      # K x m with K = n_b
        K, m = A.shape
        rows = np.arange(0, m, 7)
        Gx = (A[:, rows].conj().T @ A) / w.n_s
        Gabs = (np.abs(A[:, rows]).T @ np.abs(A)) / w.n_s
        Gx[np.arange(len(rows)), rows] += w.lam
        if info["form"] == "S":
            Gx = Gx + sr.block_trace(g) / (w.n_s * w.n_s)
        bound = (2 * K + 2) * 2.0 ** -24 * Gabs + 1e-15 * np.abs(Gx)
        Gg = sr.block_matrix(g)[rows, :]
        low = np.arange(m)[None, :] <= rows[:, None]
        ratio = (np.abs(Gg - Gx)[low] / bound[low]).max()
        say(f"  block {g} ({info['form']}, m={m}): max |err| / bound = {ratio:.3f}")
        assert ratio <= 1.0
