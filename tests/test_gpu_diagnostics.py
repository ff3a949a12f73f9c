"""Eq. 4 (a) and (b) on the device (qgt_block_inverse_diagnostics, from the
Cholesky factors of a solve) against the diagnostics oracle: the inverse of
the shifted block-layer QGT of a sampled RBM against the inverse of the shifted
exact QGT over the whole Hilbert space."""
import sys

import numpy as np
import pytest

from gen import networks, workloads
from oracle import diagnostics as dg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def all_configs(N):
    idx = np.arange(2 ** N)[:, None]
    return (1 - 2 * ((idx >> np.arange(N)) & 1)).astype(np.int8)


@pytest.mark.parametrize("n_s,lam", [(1024, 1e-3), (300, 1e-2)])
def test_inverse_diagnostics_match_the_oracle(gpu_lib, n_s, lam):
    N, M = 8, 16
    net = workloads.rbm_network(N=N, M=M, config=13, sd=0.25)
    X = all_configs(N)
    logp = 2 * net.log_psi(X).real
    p = np.exp(logp - logp.max())
    p /= p.sum()
    g = workloads.rng(13, workloads.P_SAMPLES)
    x = X[g.choice(len(X), size=n_s, p=p)]          # exact samples of |psi|^2
    O = net.jacobian(x)
    O_all = net.jacobian(X)
    sizes = net.block_sizes
    B = dg.shifted_inverse(dg.qgt(O_all, weights=p), lam)
    A = dg.block_layer_inverse(dg.qgt(O), sizes, lam)
    ref = dg.diagnostics(A, B)
    say(f"case: RBM N={N} M={M}, n_s={n_s}, lambda={lam}: oracle F={ref['frobenius_overlap']:.6f} "
        f"eps_F={ref['frobenius_relative_error']:.6f}")
    sr = gpu_lib.BlockSR([(n_s, sizes, lam)], "c128", "fp64", 0)
    d = sr([torch.from_numpy(O).cuda()], [torch.zeros(n_s, dtype=torch.complex128, device="cuda")])
    got = sr.inverse_diagnostics(torch.from_numpy(B).cuda())
    say(f"  gpu F={got['frobenius_overlap']:.6f} eps_F={got['frobenius_relative_error']:.6f}")
    assert got["frobenius_overlap"] == pytest.approx(ref["frobenius_overlap"], rel=1e-9)
    assert got["frobenius_relative_error"] == pytest.approx(ref["frobenius_relative_error"], rel=1e-9)
    # the device sums themselves: ||A||_F^2 and ||B||_F^2
    assert got["sums"][1] == pytest.approx(np.linalg.norm(A) ** 2, rel=1e-9)
    assert got["sums"][2] == pytest.approx(np.linalg.norm(B) ** 2, rel=1e-12)


def test_inverse_diagnostics_refuse_sample_space_blocks(gpu_lib):
    w = workloads.small_ffnn(n_s=200, N=8, widths=(40, 12), readout=True, o_dtype=np.complex128, lam=1e-3)
    sr = gpu_lib.BlockSR([(w.n_s, w.block_sizes, w.lam)], "c128", "fp64", 0)
    sr([torch.from_numpy(w.O).cuda()], [torch.from_numpy(w.e_loc).cuda()])
    B = torch.zeros((w.n_p, w.n_p), dtype=torch.complex128, device="cuda")
    with pytest.raises(gpu_lib.QgtError):
        sr.inverse_diagnostics(B)
