"""Host-only checks that the binding rejects malformed arguments of the
device-pointer entry points before any launch (the C ABI receives bare
pointers and cannot check lengths, types or layouts).  CPU tensors are used:
the shape and type checks come before the device check, so each case below
must fail on the argument it names."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def qgt():
    import paper_2510_08430_amd as q
    try:
        q.load()
    except RuntimeError as e:  # library not built
        pytest.skip(str(e))
    return q


def spins(n, N):
    x = np.ones((n, N), np.int8)
    x[:, N // 2:] = -1
    return torch.from_numpy(x)


def theta_rbm(N, M, dtype=torch.complex128, extra=0):
    return torch.zeros(M * N + M + N + extra, dtype=dtype)


def raises(fn, word):
    with pytest.raises(ValueError) as e:
        fn()
    assert word in str(e.value), str(e.value)


def test_metropolis_rejections(qgt):
    N, M, C, S = 8, 4, 5, 3
    x = spins(C, N)
    th = theta_rbm(N, M)
    pairs = torch.zeros((S, C, 2), dtype=torch.int32)
    u = torch.zeros((S, C), dtype=torch.float64)
    acc = torch.zeros(C, dtype=torch.int32)
    raises(lambda: qgt.rbm_metropolis(theta_rbm(N, M, torch.complex64), x, M, pairs, u, acc), "theta")
    raises(lambda: qgt.rbm_metropolis(theta_rbm(N, M, extra=-1), x, M, pairs, u, acc), "theta")
    raises(lambda: qgt.rbm_metropolis(th, x.to(torch.int32), M, pairs, u, acc), "x")
    raises(lambda: qgt.rbm_metropolis(th, x.t(), M, pairs, u, acc), "x")
    raises(lambda: qgt.rbm_metropolis(th, x, M, pairs[:, :, :1].contiguous(), u, acc), "pairs")
    raises(lambda: qgt.rbm_metropolis(th, x, M, pairs.to(torch.int64), u, acc), "pairs")
    raises(lambda: qgt.rbm_metropolis(th, x, M, pairs, u[:, :2].contiguous(), acc), "u")
    raises(lambda: qgt.rbm_metropolis(th, x, M, pairs, u.to(torch.float32), acc), "u")
    raises(lambda: qgt.rbm_metropolis(th, x, M, pairs, u, acc[:2]), "accepted")
    raises(lambda: qgt.rbm_metropolis(th, x, M, pairs, u, acc), "CUDA")  # all well formed, but on the host


def test_eloc_and_update_rejections(qgt):
    N, M, n = 8, 4, 6
    x = spins(n, N)
    th = theta_rbm(N, M)
    raises(lambda: qgt.rbm_heisenberg_eloc(theta_rbm(N, M, extra=3), x, M), "theta")
    raises(lambda: qgt.rbm_heisenberg_eloc(th, x, M, e_loc=torch.zeros(n - 1, dtype=torch.complex128)), "e_loc")
    raises(lambda: qgt.rbm_heisenberg_eloc(th, x, M, e_loc=torch.zeros(n, dtype=torch.complex64)), "e_loc")
    raises(lambda: qgt.rbm_heisenberg_eloc(th, x, M), "CUDA")
    d = torch.zeros_like(th)
    raises(lambda: qgt.sr_update(th, d[:-1], 0.1), "delta")
    raises(lambda: qgt.sr_update(th.to(torch.complex64), d.to(torch.complex64), 0.1), "theta")
    raises(lambda: qgt.sr_update(th, d, 0.1), "CUDA")


def test_jacobian_rejections(qgt):
    N, M, n = 8, 4, 6
    x = spins(n, N)
    th = theta_rbm(N, M)
    n_p = M * N + M + N
    raises(lambda: qgt.rbm_jacobian(theta_rbm(N, M, extra=1), x, M), "theta")
    raises(lambda: qgt.rbm_jacobian(th, x, M, O=torch.zeros((n - 1, n_p), dtype=torch.complex128)), "O")
    raises(lambda: qgt.rbm_jacobian(th, x, M, O=torch.zeros((n, n_p), dtype=torch.complex128).t().contiguous().t()),
           "O")
    raises(lambda: qgt.rbm_jacobian(th, x, M, O=torch.zeros((n, n_p), dtype=torch.float64)), "O")
    widths = [N, 5, 3]
    n_pf = qgt.ffnn_n_params(widths, False)
    raises(lambda: qgt.ffnn_jacobian(torch.zeros(n_pf + 1, dtype=torch.complex128), x, widths), "theta")
    raises(lambda: qgt.ffnn_jacobian(torch.zeros(n_pf, dtype=torch.complex128), spins(n, N + 2), widths), "x")
    raises(lambda: qgt.ffnn_jacobian(torch.zeros(n_pf, dtype=torch.complex128), x, widths,
                                     workspace=torch.zeros(64, dtype=torch.float32)), "CUDA")
    n_pc = qgt.cnn_n_params(3, 2, 1)
    raises(lambda: qgt.cnn_jacobian(torch.zeros(n_pc, dtype=torch.complex128), spins(n, 8), 3, 2, 1), "x")
    raises(lambda: qgt.cnn_jacobian(torch.zeros(n_pc - 1, dtype=torch.complex128), spins(n, 9), 3, 2, 1), "theta")


def test_block_sr_rejects_unknown_settings(qgt):
    with pytest.raises(ValueError):
        qgt.workspace_query([(64, [10, 20], 1e-3)], factor="fp16")
    assert qgt.workspace_query([(64, [10, 200], 1e-3)], "c64", "bf16", factor="fp32") < \
        qgt.workspace_query([(64, [10, 200], 1e-3)], "c64", "bf16", factor="fp64")
