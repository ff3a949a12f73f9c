"""FP64 CPU oracle for forming the log-derivative matrix O on the device.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow reference that the
GPU Jacobian kernels are checked against.  Only the tests, the smoke check and
the benchmark's CPU-baseline leg may import it; the product path never does.
It shares no code with the HIP library (nor with the input generators, which
build the same matrix by a vectorised route of their own).

What it computes (paper: Sec. 2, the definition that follows Eq. 2): the
per-sample log-derivatives O_k(x) = d log psi_theta(x) / d theta_k, one row per
sample, one column per parameter, parameters in the flat order of the layer
blocks of Eq. 3.  The networks are holomorphic in their complex parameters, so
O is the plain complex derivative and the chain rule uses plain (unconjugated)
transposes.  Each function takes the parameter vector theta (complex128, flat)
and the samples x (n_s x N, entries +-1) and works one sample at a time.

Network definitions (stand-ins for the paper's Vision Transformer, which is
out of scope):
  * logcosh(z) = s z + log1p(exp(-2 s z)) - log 2, s = +1 if Re z >= 0 else -1:
    one fixed branch of log cosh; its derivative is tanh(z) on either branch.
  * RBM, N visible and M hidden units:
        log psi(x) = sum_i a_i x_i + sum_j logcosh(b_j + sum_i W_ji x_i),
    parameters [W (M x N, row-major) | b (M) | a (N)].
  * FFNN with widths [N, w_1, ..., w_L]:
        h^0 = x,  z^l = W^l h^{l-1} + b^l,  h^l = logcosh(z^l),
        log psi = sum_k h^L_k, or v . h^L + c with a dense readout,
    parameters [W^1 (row-major, out x in) | b^1 | ... | W^L | b^L (| v | c)].
  * CNN on a periodic L x L lattice, 3 x 3 cross-correlations:
        z^l[c, y, x] = b^l[c] + sum_{c', dy, dx} K^l[c, c', dy, dx]
                       h^{l-1}[c', (y + dy - 1) mod L, (x + dx - 1) mod L],
        h^l = logcosh(z^l),  log psi = sum_{c, y, x} h^last[c, y, x],
    h^0 the one-channel spin lattice (sites row-major), parameters
    [K^1 (c_out, c_in, dy, dx) | b^1 | ... ].

Pins (in the tests): central finite differences of the log-amplitudes defined
here, in the real and the imaginary direction (holomorphy); the closed-form
columns of the RBM (O_a = x, O_b = tanh of the hidden field); agreement with the
independent vectorised construction of the input generators.
"""
from __future__ import annotations

import numpy as np

LOG2 = np.log(2.0)


def logcosh(z):
    """log cosh on the fixed branch s z + log1p(exp(-2 s z)) - log 2."""
    z = np.asarray(z, dtype=np.complex128)
    s = np.where(z.real >= 0, 1.0, -1.0)
    return s * z + np.log1p(np.exp(-2.0 * s * z)) - LOG2


def _x(x):
    return np.asarray(x, dtype=np.float64)


# ---------------------------------------------------------------------------
# RBM
# ---------------------------------------------------------------------------
def rbm_split(theta, N, M):
    theta = np.asarray(theta, dtype=np.complex128)
    assert theta.size == M * N + M + N
    W = theta[: M * N].reshape(M, N)
    b = theta[M * N: M * N + M]
    a = theta[M * N + M:]
    return W, b, a


def rbm_log_psi(theta, N, M, x):
    W, b, a = rbm_split(theta, N, M)
    out = []
    for xs in _x(x):
        out.append(a @ xs + logcosh(W @ xs + b).sum())
    return np.array(out, dtype=np.complex128)


def rbm_jacobian(theta, N, M, x):
    """Rows [d/dW_ji = tanh(theta_j) x_i | d/db_j = tanh(theta_j) | d/da_i = x_i]."""
    W, b, a = rbm_split(theta, N, M)
    xs_all = _x(x)
    O = np.empty((xs_all.shape[0], M * N + M + N), dtype=np.complex128)
    for r, xs in enumerate(xs_all):
        t = np.tanh(W @ xs + b)
        O[r, : M * N] = np.outer(t, xs).reshape(-1)
        O[r, M * N: M * N + M] = t
        O[r, M * N + M:] = xs
    return O


# ---------------------------------------------------------------------------
# FFNN
# ---------------------------------------------------------------------------
def ffnn_block_sizes(widths, readout):
    sizes = [widths[l + 1] * widths[l] + widths[l + 1] for l in range(len(widths) - 1)]
    if readout:
        sizes.append(widths[-1] + 1)
    return sizes


def ffnn_split(theta, widths, readout):
    theta = np.asarray(theta, dtype=np.complex128)
    assert theta.size == sum(ffnn_block_sizes(widths, readout))
    Ws, bs, p = [], [], 0
    for l in range(len(widths) - 1):
        nin, nout = widths[l], widths[l + 1]
        Ws.append(theta[p: p + nout * nin].reshape(nout, nin)); p += nout * nin
        bs.append(theta[p: p + nout]); p += nout
    ro = (theta[p: p + widths[-1]], theta[p + widths[-1]]) if readout else None
    return Ws, bs, ro


def ffnn_log_psi(theta, widths, readout, x):
    Ws, bs, ro = ffnn_split(theta, widths, readout)
    out = []
    for xs in _x(x):
        h = xs.astype(np.complex128)
        for W, b in zip(Ws, bs):
            h = logcosh(W @ h + b)
        out.append(ro[0] @ h + ro[1] if readout else h.sum())
    return np.array(out, dtype=np.complex128)


def ffnn_jacobian(theta, widths, readout, x):
    """Chain rule, output to input: with dh = d log psi / d h^L (v, or ones),
    g^l = tanh(z^l) * dh is d log psi / d z^l; the layer's derivatives are
    g^l (h^{l-1})^T for W^l and g^l for b^l; then dh = (W^l)^T g^l."""
    Ws, bs, ro = ffnn_split(theta, widths, readout)
    sizes = ffnn_block_sizes(widths, readout)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    L = len(Ws)
    xs_all = _x(x)
    O = np.empty((xs_all.shape[0], int(offs[-1])), dtype=np.complex128)
    for r, xs in enumerate(xs_all):
        hs, zs = [xs.astype(np.complex128)], []
        for W, b in zip(Ws, bs):
            zs.append(W @ hs[-1] + b)
            hs.append(logcosh(zs[-1]))
        if readout:
            o = offs[L]
            O[r, o: o + widths[-1]] = hs[L]
            O[r, o + widths[-1]] = 1.0
            dh = ro[0].copy()
        else:
            dh = np.ones(widths[-1], dtype=np.complex128)
        for l in range(L - 1, -1, -1):
            g = np.tanh(zs[l]) * dh
            nout, nin = Ws[l].shape
            o = offs[l]
            O[r, o: o + nout * nin] = np.outer(g, hs[l]).reshape(-1)
            O[r, o + nout * nin: o + nout * nin + nout] = g
            dh = Ws[l].T @ g
    return O


# ---------------------------------------------------------------------------
# CNN
# ---------------------------------------------------------------------------
def cnn_block_sizes(channels, n_layers):
    sizes, cin = [], 1
    for _ in range(n_layers):
        sizes.append(channels * cin * 9 + channels)
        cin = channels
    return sizes


def cnn_split(theta, channels, n_layers):
    theta = np.asarray(theta, dtype=np.complex128)
    assert theta.size == sum(cnn_block_sizes(channels, n_layers))
    Ks, bs, p, cin = [], [], 0, 1
    for _ in range(n_layers):
        n = channels * cin * 9
        Ks.append(theta[p: p + n].reshape(channels, cin, 3, 3)); p += n
        bs.append(theta[p: p + channels]); p += channels
        cin = channels
    return Ks, bs


def _shifted(h, dy, dx):
    """h'[c, y, x] = h[c, (y + dy) mod L, (x + dx) mod L]."""
    return np.roll(h, shift=(-dy, -dx), axis=(1, 2))


def _correlate(K, b, h):
    cout = K.shape[0]
    L = h.shape[1]
    z = np.empty((cout, L, L), dtype=np.complex128)
    z[:] = b[:, None, None]
    for dy in range(3):
        for dx in range(3):
            hs = _shifted(h, dy - 1, dx - 1)
            z += np.tensordot(K[:, :, dy, dx], hs, axes=(1, 0))
    return z


def cnn_log_psi(theta, L, channels, n_layers, x):
    Ks, bs = cnn_split(theta, channels, n_layers)
    out = []
    for xs in _x(x):
        h = xs.reshape(1, L, L).astype(np.complex128)
        for K, b in zip(Ks, bs):
            h = logcosh(_correlate(K, b, h))
        out.append(h.sum())
    return np.array(out, dtype=np.complex128)


def cnn_jacobian(theta, L, channels, n_layers, x):
    """With g^l = d log psi / d z^l (tanh(z^l) times the derivative reaching
    h^l): d/dK^l[c, c', dy, dx] = sum_sites g^l[c, y, x] h^{l-1}[c', y+dy-1,
    x+dx-1], d/db^l[c] = sum_sites g^l[c], and the derivative reaching h^{l-1}
    is sum_{c, dy, dx} K^l[c, c', dy, dx] g^l[c, y-dy+1, x-dx+1]."""
    Ks, bs = cnn_split(theta, channels, n_layers)
    sizes = cnn_block_sizes(channels, n_layers)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    xs_all = _x(x)
    O = np.empty((xs_all.shape[0], int(offs[-1])), dtype=np.complex128)
    for r, xs in enumerate(xs_all):
        hs, zs = [xs.reshape(1, L, L).astype(np.complex128)], []
        for K, b in zip(Ks, bs):
            zs.append(_correlate(K, b, hs[-1]))
            hs.append(logcosh(zs[-1]))
        dh = np.ones_like(hs[-1])
        for l in range(n_layers - 1, -1, -1):
            g = np.tanh(zs[l]) * dh
            K = Ks[l]
            cout, cin = K.shape[:2]
            dK = np.empty(K.shape, dtype=np.complex128)
            dprev = np.zeros((cin, L, L), dtype=np.complex128)
            for dy in range(3):
                for dx in range(3):
                    hs_l = _shifted(hs[l], dy - 1, dx - 1)
                    dK[:, :, dy, dx] = np.tensordot(g, hs_l, axes=((1, 2), (1, 2)))
                    # h^{l-1} at site s' feeds z^l at s' - d: shift g the other way
                    dprev += np.tensordot(K[:, :, dy, dx], _shifted(g, 1 - dy, 1 - dx), axes=(0, 0))
            o = offs[l]
            O[r, o: o + K.size] = dK.reshape(-1)
            O[r, o + K.size: o + K.size + cout] = g.sum(axis=(1, 2))
            dh = dprev
    return O
