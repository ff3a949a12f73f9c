"""GPU parity of the device formation of O (include/qgt_jacobian.h) against
the FP64 Jacobian oracle (oracle/jacobian.py), all through the C ABI.

O_k(x) = d log psi(x) / d theta_k (paper, Sec. 2, the definition after Eq. 2).
Both sides compute every entry in FP64; the library rounds once to the output
type.  Bars:
  * complex128 output: |O_gpu - O_oracle| <= 1e-10 |O_oracle| + 1e-12 max|O|
    (FP64 rounding of the dense products, of tanh and of logcosh, which the
    two sides evaluate by different formulas);
  * complex64 output: each component equals the oracle's value rounded to
    FP32 except where the two FP64 values straddle a rounding boundary (at
    most one entry in 10^5); there it is within one FP32 rounding
    (2^-24 relative to the component) of the oracle value plus the FP64 bound
    above (which is relative to |O|, so a component much smaller than |O| may
    move by more than one of its own units in the last place).

Cases: reduced shapes that span several 64 x 32 product tiles with ragged
edges, one sample, one layer, eight layers, widths of 1; the RBM of the FP64
workload (N=16, M=32, n_s=1024, full size); the chain FFNN 64-128-128-64 with
readout at n_s=4096 (full size, every entry); the FFNN 100-400-400 at
n_s=8192 (full size, 64 sampled rows); instances of the 32-instance stream;
strided samples and a strided O with untouched padding; and O formed on the
device feeding the block solve.
"""
import sys

import numpy as np
import pytest

from gen import workloads
from oracle import jacobian as jac

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def check(O_gpu, O_or, dt):
    O_gpu = np.asarray(O_gpu)
    if dt == "c128":
        err = np.abs(O_gpu - O_or)
        bound = 1e-10 * np.abs(O_or) + 1e-12 * np.abs(O_or).max()
        worst = float((err / np.maximum(bound, 1e-300)).max())
        assert np.all(err <= bound), f"worst error / bound = {worst:.3g}"
        return
    ref = O_or.astype(np.complex64)
    fp64_bound = 1e-10 * np.abs(O_or) + 1e-12 * np.abs(O_or).max()
    n_bad = 0
    for part in ("real", "imag"):
        a = np.ascontiguousarray(getattr(O_gpu, part)).view(np.int32).astype(np.int64)
        b = np.ascontiguousarray(getattr(ref, part)).view(np.int32).astype(np.int64)
        off = a != b
        n_bad += int(np.count_nonzero(off))
        if off.any():
            g = getattr(O_gpu, part)[off].astype(np.float64)
            o = getattr(O_or, part)[off]
            assert np.all(np.abs(g - o) <= 2.0 ** -24 * np.abs(o) + fp64_bound[off]), part
    assert n_bad <= max(2, O_or.size // 100000), n_bad


def samples(config, N, n_s, instance=0):
    return workloads.zero_magnetisation_samples(workloads.rng(config, workloads.P_SAMPLES, instance), n_s, N)


def ffnn_gpu(qgt, theta, x, widths, readout, dt):
    say(f"  gpu: ffnn_jacobian widths={widths} readout={readout} n_s={x.shape[0]} {dt}")
    th = torch.from_numpy(np.ascontiguousarray(theta, dtype=np.complex128)).cuda()
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.int8)).cuda()
    O = qgt.ffnn_jacobian(th, xd, widths, readout, dt)
    torch.cuda.synchronize()
    return O


@pytest.mark.parametrize("widths,readout,n_s,dt", [
    ([8, 10, 6], True, 77, "c128"),
    ([8, 10, 6], False, 77, "c64"),
    ([16, 40, 33, 20], True, 130, "c128"),
    ([16, 40, 33, 20], False, 130, "c64"),
    ([5, 3], False, 1, "c128"),
    ([12] * 9, True, 65, "c128"),
    ([2, 1, 1], True, 3, "c128"),
    ([24, 48, 24], False, 200, "c64"),
])
def test_ffnn_reduced_shapes(gpu_lib, widths, readout, n_s, dt):
    net = workloads.ffnn_network(widths, config=9, readout=readout)
    x = samples(9, widths[0], n_s)
    O = ffnn_gpu(gpu_lib, net.flat(), x, widths, readout, dt).cpu().numpy()
    check(O, jac.ffnn_jacobian(net.flat(), widths, readout, x), dt)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_rbm_fp64_workload_full_size(gpu_lib, dt):
    N, M, n_s = 16, 32, 1024
    net = workloads.rbm_network(N=N, M=M, config=0)
    x = samples(0, N, n_s)
    say(f"  gpu: rbm_jacobian N={N} M={M} n_s={n_s} {dt}")
    th = torch.from_numpy(net.flat()).cuda()
    O = gpu_lib.rbm_jacobian(th, torch.from_numpy(x).cuda(), M, dt).cpu().numpy()
    check(O, jac.rbm_jacobian(net.flat(), N, M, x), dt)
    # the visible-bias columns are the spins, exactly
    assert np.array_equal(O[:, M * N + M:], x.astype(O.dtype))


def test_ffnn_chain_n64_full_size_every_entry(gpu_lib):
    widths, n_s = [64, 128, 128, 64], 4096
    net = workloads.ffnn_network(widths, config=1, readout=True, dtype=np.complex64)
    x = samples(1, 64, n_s)
    O = ffnn_gpu(gpu_lib, net.flat(), x, widths, True, "c64").cpu().numpy()
    assert O.shape == (n_s, 33153)
    check(O, jac.ffnn_jacobian(net.flat(), widths, True, x), "c64")


def test_ffnn_100_400_400_full_size_sampled_rows(gpu_lib):
    widths, n_s = [100, 400, 400], 8192
    net = workloads.ffnn_network(widths, config=2, instance=1, dtype=np.complex64)
    x = samples(2, 100, n_s, instance=1)
    O = ffnn_gpu(gpu_lib, net.flat(), x, widths, False, "c64")
    rows = np.unique(np.concatenate([[0, 1, n_s - 1], np.random.default_rng(0).choice(n_s, 61, replace=False)]))
    sub = O[torch.from_numpy(rows).cuda()].cpu().numpy()
    del O
    torch.cuda.empty_cache()
    check(sub, jac.ffnn_jacobian(net.flat(), widths, False, x[rows]), "c64")


@pytest.mark.parametrize("instance", [0, 5, 17, 31])
def test_stream_instances(gpu_lib, instance):
    g = workloads.rng(4, workloads.P_BLOCKS, instance)
    N = int(g.choice(workloads.CONFIG4_CHAINS))
    n_s = int(g.choice(workloads.CONFIG4_NS))
    widths = [N, 2 * N, N]
    net = workloads.ffnn_network(widths, config=4, instance=instance, dtype=np.complex64)
    x = samples(4, N, n_s, instance)
    O = ffnn_gpu(gpu_lib, net.flat(), x, widths, False, "c64").cpu().numpy()
    check(O, jac.ffnn_jacobian(net.flat(), widths, False, x), "c64")


def test_strided_samples_and_output_padding(gpu_lib):
    widths, n_s, pad_x, pad_o = [10, 14, 9], 70, 3, 5
    net = workloads.ffnn_network(widths, config=9, instance=3, readout=True)
    x = samples(9, 10, n_s, 3)
    n_p = gpu_lib.ffnn_n_params(widths, True)
    xb = np.zeros((n_s, 10 + pad_x), np.int8)
    xb[:, :10] = x
    xb[:, 10:] = 77                                   # must never be read as a spin
    xd = torch.from_numpy(xb).cuda()[:, :10]
    Ob = torch.full((n_s, n_p + pad_o), complex(-3.5, 2.25), dtype=torch.complex128, device="cuda")
    say(f"  gpu: ffnn_jacobian strided ldx={xd.stride(0)} ldo={Ob.stride(0)}")
    gpu_lib.ffnn_jacobian(torch.from_numpy(net.flat()).cuda(), xd, widths, True, O=Ob[:, :n_p])
    Oh = Ob.cpu().numpy()
    check(Oh[:, :n_p], jac.ffnn_jacobian(net.flat(), widths, True, x), "c128")
    assert np.all(Oh[:, n_p:] == complex(-3.5, 2.25))


def test_device_formed_O_feeds_the_block_solve(gpu_lib):
    """O formed on the device and O built on the host (the vectorised input
    generator, rounded to complex64) give the same block-SR update."""
    qgt = gpu_lib
    wl = workloads.small_ffnn(n_s=512, N=16, widths=(24, 20), readout=True, o_dtype=np.complex64, lam=1e-3)
    net = workloads.ffnn_network([16, 24, 20], config=9, readout=True, dtype=np.complex64)
    x = samples(9, 16, 512)
    O_dev = ffnn_gpu(qgt, net.flat(), x, [16, 24, 20], True, "c64")
    O_host = torch.from_numpy(np.ascontiguousarray(wl.O)).cuda()
    E = torch.from_numpy(wl.e_loc).cuda()
    say("  gpu: block solve on device-formed and host-formed O")
    sr = qgt.BlockSR([(512, wl.block_sizes, wl.lam)], "c64", "fp64", 2)
    d_dev = sr([O_dev], [E])[0].cpu().numpy()
    d_host = sr([O_host], [E])[0].cpu().numpy()
    assert np.abs(O_dev.cpu().numpy() - wl.O).max() <= 2.0 ** -23 * np.abs(wl.O).max()
    assert np.linalg.norm(d_dev - d_host) <= 1e-5 * np.linalg.norm(d_host)


def test_graph_capture_replays_match_eager(gpu_lib):
    """The entry points allocate nothing and never synchronise: captured in a
    HIP graph, every replay (with eager work and synchronisation between
    replays) writes exactly the eager result."""
    qgt = gpu_lib
    widths = [24, 40, 24]
    net = workloads.ffnn_network(widths, config=9, instance=4, readout=True, dtype=np.complex64)
    x = samples(9, 24, 300, 4)
    th = torch.from_numpy(net.flat()).cuda()
    xd = torch.from_numpy(x).cuda()
    n_p = qgt.ffnn_n_params(widths, True)
    O = torch.empty((300, n_p), dtype=torch.complex64, device="cuda")
    ws = torch.empty(qgt.ffnn_jacobian_workspace_bytes(widths, True, 300), dtype=torch.uint8, device="cuda")
    say("  gpu: eager ffnn_jacobian, then capture")
    qgt.ffnn_jacobian(th, xd, widths, True, O=O, workspace=ws)
    torch.cuda.synchronize()
    eager = O.clone()
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        with torch.cuda.graph(graph, stream=cap):
            qgt.ffnn_jacobian(th, xd, widths, True, O=O, workspace=ws)
    torch.cuda.current_stream().wait_stream(cap)
    torch.cuda.synchronize()
    for rep in range(3):
        O.zero_()
        ws.fill_(0xFF)
        torch.cuda.synchronize()
        say(f"  gpu: replay {rep}")
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(O.view(torch.float32), eager.view(torch.float32)), rep
    check(eager.cpu().numpy(), jac.ffnn_jacobian(net.flat(), widths, True, x), "c64")


def cnn_gpu(qgt, theta, x, side, C, L, dt):
    say(f"  gpu: cnn_jacobian side={side} channels={C} layers={L} n_s={x.shape[0]} {dt}")
    th = torch.from_numpy(np.ascontiguousarray(theta, dtype=np.complex128)).cuda()
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.int8)).cuda()
    O = qgt.cnn_jacobian(th, xd, side, C, L, dt)
    torch.cuda.synchronize()
    return O


@pytest.mark.parametrize("side,C,L,n_s,dt", [
    (4, 3, 3, 37, "c128"),
    (5, 2, 1, 9, "c64"),
    (6, 4, 2, 70, "c64"),
    (2, 1, 2, 5, "c128"),
    (7, 16, 3, 11, "c128"),
])
def test_cnn_reduced_shapes(gpu_lib, side, C, L, n_s, dt):
    net = workloads.cnn_network(L=side, channels=C, layers=L, config=9)
    x = samples(9, side * side, n_s)
    O = cnn_gpu(gpu_lib, net.flat(), x, side, C, L, dt).cpu().numpy()
    check(O, jac.cnn_jacobian(net.flat(), side, C, L, x), dt)


def test_cnn_10x10_full_size_sampled_rows(gpu_lib):
    n_s = 8192
    net = workloads.cnn_network(L=10, config=2, dtype=np.complex64)
    x = samples(2, 100, n_s)
    O = cnn_gpu(gpu_lib, net.flat(), x, 10, 16, 4, "c64")
    assert O.shape == (n_s, 7120)
    rows = np.unique(np.concatenate([[0, n_s - 1], np.random.default_rng(1).choice(n_s, 46, replace=False)]))
    sub = O[torch.from_numpy(rows).cuda()].cpu().numpy()
    check(sub, jac.cnn_jacobian(net.flat(), 10, 16, 4, x[rows]), "c64")
