"""Pins of the FP64 Jacobian oracle (oracle/jacobian.py), which checks the
device formation of O (O_k(x) = d log psi(x) / d theta_k, paper Sec. 2, the
definition after Eq. 2):

  * central finite differences of the oracle's own log-amplitudes, in the real
    and in the imaginary direction of each checked parameter (a holomorphic
    function has the same derivative along both);
  * exact structure that the definition fixes: the RBM visible-bias columns
    are the spins themselves, the first-layer weight columns are the bias
    columns times the spins (x_i = +-1 makes the product exact);
  * agreement with the independent vectorised construction of the input
    generators (a second implementation, not a retyped formula);
  * planted mistakes (a dropped activation derivative, a conjugated
    back-propagated derivative, a transposed outer product, the backward
    shift of a convolution taken the wrong way) are caught.
Everything runs on the CPU.
"""
import numpy as np
import pytest

from gen import workloads
from oracle import jacobian as jac


def _samples(n_s, N, seed):
    return workloads.zero_magnetisation_samples(np.random.default_rng(seed), n_s, N)


def _fd(log_psi, theta, x, O, n_checked=40, seed=0, h=1e-6):
    """Central differences of log psi along theta_k, real and imaginary steps;
    the log of a ratio (differences reduced modulo 2 pi i) avoids branch jumps."""
    g = np.random.default_rng(seed)
    ks = g.choice(theta.size, size=min(n_checked, theta.size), replace=False)
    base = log_psi(theta, x)
    for k in ks:
        for step in (h, 1j * h):
            tp = theta.copy(); tp[k] += step
            tm = theta.copy(); tm[k] -= step
            lp = log_psi(tp, x) - base
            lm = log_psi(tm, x) - base
            lp = lp - 2j * np.pi * np.round(lp.imag / (2 * np.pi))
            lm = lm - 2j * np.pi * np.round(lm.imag / (2 * np.pi))
            fd = (lp - lm) / (2 * step)
            np.testing.assert_allclose(fd, O[:, k], rtol=2e-6, atol=2e-7 * (1 + np.abs(O[:, k]).max()))


def _ffnn_case(widths=(8, 10, 6), readout=True, n_s=12, seed=5):
    net = workloads.ffnn_network(list(widths), config=7, readout=readout)
    return net.flat(), list(widths), readout, _samples(n_s, widths[0], seed)


def test_logcosh_branch():
    g = np.random.default_rng(0)
    z = g.normal(0, 3, 300) + 1j * g.normal(0, 3, 300)
    np.testing.assert_allclose(np.exp(jac.logcosh(z)), np.cosh(z), rtol=1e-12)


def test_rbm_finite_differences_and_closed_columns():
    N, M = 8, 12
    net = workloads.rbm_network(N=N, M=M, config=7, sd=0.3)
    theta, x = net.flat(), _samples(16, N, 1)
    O = jac.rbm_jacobian(theta, N, M, x)
    _fd(lambda t, xx: jac.rbm_log_psi(t, N, M, xx), theta, x, O)
    # d/da_i = x_i exactly; d/dW_ji = (d/db_j) x_i exactly
    assert np.array_equal(O[:, M * N + M:], x.astype(np.complex128))
    dW = O[:, : M * N].reshape(-1, M, N)
    assert np.array_equal(dW, O[:, M * N: M * N + M][:, :, None] * x[:, None, :])


@pytest.mark.parametrize("readout", [False, True])
def test_ffnn_finite_differences(readout):
    theta, widths, ro, x = _ffnn_case(readout=readout)
    O = jac.ffnn_jacobian(theta, widths, ro, x)
    _fd(lambda t, xx: jac.ffnn_log_psi(t, widths, ro, xx), theta, x, O, n_checked=48)


def test_ffnn_first_layer_structure_and_readout_columns():
    theta, widths, ro, x = _ffnn_case(widths=(8, 10, 6, 4), readout=True)
    O = jac.ffnn_jacobian(theta, widths, ro, x)
    N, w1 = widths[0], widths[1]
    dW1 = O[:, : w1 * N].reshape(-1, w1, N)
    db1 = O[:, w1 * N: w1 * N + w1]
    assert np.array_equal(dW1, db1[:, :, None] * x[:, None, :])
    # readout block: d/dc = 1 exactly
    assert np.all(O[:, -1] == 1.0)


def test_cnn_finite_differences():
    L, C, nl = 4, 3, 3
    net = workloads.cnn_network(L=L, channels=C, layers=nl, config=7)
    theta, x = net.flat(), _samples(6, L * L, 3)
    O = jac.cnn_jacobian(theta, L, C, nl, x)
    _fd(lambda t, xx: jac.cnn_log_psi(t, L, C, nl, xx), theta, x, O, n_checked=40)
    assert jac.cnn_block_sizes(C, nl) == net.block_sizes


@pytest.mark.parametrize("family", ["rbm", "ffnn", "ffnn_sum", "cnn"])
def test_matches_independent_vectorised_generator(family):
    if family == "rbm":
        N, M = 16, 32
        net = workloads.rbm_network(N=N, M=M, config=7, sd=0.2)
        x = _samples(40, N, 4)
        O = jac.rbm_jacobian(net.flat(), N, M, x)
    elif family.startswith("ffnn"):
        widths = [16, 24, 20, 8]
        net = workloads.ffnn_network(widths, config=7, readout=(family == "ffnn"))
        x = _samples(40, widths[0], 4)
        O = jac.ffnn_jacobian(net.flat(), widths, family == "ffnn", x)
    else:
        net = workloads.cnn_network(L=6, channels=4, layers=3, config=7)
        x = _samples(10, 36, 4)
        O = jac.cnn_jacobian(net.flat(), 6, 4, 3, x)
    ref = net.jacobian(x)
    np.testing.assert_allclose(O, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


# ---------------------------------------------------------------------------
# planted mistakes in the oracle must fail a pin
# ---------------------------------------------------------------------------
def _mutant_ffnn(kind):
    def f(theta, widths, readout, x):
        Ws, bs, ro = jac.ffnn_split(theta, widths, readout)
        sizes = jac.ffnn_block_sizes(widths, readout)
        offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        L = len(Ws)
        xs_all = np.asarray(x, dtype=np.float64)
        O = np.empty((xs_all.shape[0], int(offs[-1])), dtype=np.complex128)
        for r, xs in enumerate(xs_all):
            hs, zs = [xs.astype(np.complex128)], []
            for W, b in zip(Ws, bs):
                zs.append(W @ hs[-1] + b)
                hs.append(jac.logcosh(zs[-1]))
            if readout:
                o = offs[L]
                O[r, o: o + widths[-1]] = hs[L]
                O[r, o + widths[-1]] = 1.0
                dh = ro[0].copy()
            else:
                dh = np.ones(widths[-1], dtype=np.complex128)
            for l in range(L - 1, -1, -1):
                g = (dh if kind == "no_tanh" else np.tanh(zs[l]) * dh)
                if kind == "conj_backprop":
                    g = np.tanh(zs[l]) * dh.conj()
                nout, nin = Ws[l].shape
                o = offs[l]
                if kind == "transposed_outer" and nout == nin:
                    O[r, o: o + nout * nin] = np.outer(hs[l], g).reshape(-1)
                else:
                    O[r, o: o + nout * nin] = np.outer(g, hs[l]).reshape(-1)
                O[r, o + nout * nin: o + nout * nin + nout] = g
                dh = Ws[l].T @ g
        return O
    return f


@pytest.mark.parametrize("kind", ["no_tanh", "conj_backprop", "transposed_outer"])
def test_planted_ffnn_mistakes_are_caught(kind, monkeypatch):
    monkeypatch.setattr(jac, "ffnn_jacobian", _mutant_ffnn(kind))
    widths = (8, 10, 10, 6)
    with pytest.raises(AssertionError):
        theta, w, ro, x = _ffnn_case(widths=widths, readout=True)
        O = jac.ffnn_jacobian(theta, w, ro, x)
        _fd(lambda t, xx: jac.ffnn_log_psi(t, w, ro, xx), theta, x, O, n_checked=60)


def _cnn_backward_shift_reversed(theta, L, channels, n_layers, x):
    """The CNN chain rule with the backward shift of g taken the wrong way."""
    Ks, bs = jac.cnn_split(theta, channels, n_layers)
    offs = np.concatenate([[0], np.cumsum(jac.cnn_block_sizes(channels, n_layers))]).astype(np.int64)
    xs_all = np.asarray(x, dtype=np.float64)
    O = np.empty((xs_all.shape[0], int(offs[-1])), dtype=np.complex128)
    for r, xs in enumerate(xs_all):
        hs, zs = [xs.reshape(1, L, L).astype(np.complex128)], []
        for K, b in zip(Ks, bs):
            zs.append(jac._correlate(K, b, hs[-1]))
            hs.append(jac.logcosh(zs[-1]))
        dh = np.ones_like(hs[-1])
        for l in range(n_layers - 1, -1, -1):
            g = np.tanh(zs[l]) * dh
            K = Ks[l]
            dK = np.empty(K.shape, dtype=np.complex128)
            dprev = np.zeros((K.shape[1], L, L), dtype=np.complex128)
            for dy in range(3):
                for dx in range(3):
                    dK[:, :, dy, dx] = np.tensordot(g, jac._shifted(hs[l], dy - 1, dx - 1), axes=((1, 2), (1, 2)))
                    dprev += np.tensordot(K[:, :, dy, dx], jac._shifted(g, dy - 1, dx - 1), axes=(0, 0))
            O[r, offs[l]: offs[l] + K.size] = dK.reshape(-1)
            O[r, offs[l] + K.size: offs[l + 1]] = g.sum(axis=(1, 2))
            dh = dprev
    return O


def test_planted_cnn_reversed_backward_shift_is_caught():
    L, C, nl = 4, 2, 3
    net = workloads.cnn_network(L=L, channels=C, layers=nl, config=7)
    theta, x = net.flat(), _samples(4, L * L, 3)
    O_bad = _cnn_backward_shift_reversed(theta, L, C, nl, x)
    with pytest.raises(AssertionError):
        _fd(lambda t, xx: jac.cnn_log_psi(t, L, C, nl, xx), theta, x, O_bad, n_checked=60)
