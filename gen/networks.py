"""Neural quantum states and their per-sample log-derivative Jacobians.

This module produces the *input* of the block stochastic-reconfiguration path:
the matrix O with O[x, i] = d log psi_theta(x) / d theta_i (paper, Sec. 2, the
definition that follows Eq. 2, and Eq. 3 for the layer blocks).  It contains no
part of the SR arithmetic itself (no centring, Gram, force or solve).

All networks are holomorphic in their complex parameters, so O is the plain
(unconjugated) complex derivative and back-propagation uses the plain transpose.

Conventions fixed here (the paper is silent on them):
  * logcosh branch: logcosh(z) = s*z + log1p(exp(-2 s z)) - log 2 with s = +1 if
    Re z >= 0 else -1.  Its derivative tanh(z) does not depend on the branch.
  * Parameter vector order per layer: [W row-major (out, in) | b].  RBM order is
    [W (hidden j, visible i) row-major | b | a], i.e. blocks (M*N, M, N).
  * CNN: periodic 3x3 cross-correlation on an L x L lattice, kernel index order
    (c_out, c_in, dy, dx) with offsets dy-1, dx-1, sites row-major, channel-major
    activations.
"""
from __future__ import annotations

import numpy as np

LOG2 = np.log(2.0)


def logcosh(z):
    """Branch-fixed complex log cosh (see module docstring)."""
    z = np.asarray(z)
    s = np.where(z.real >= 0, 1.0, -1.0)
    return s * z + np.log1p(np.exp(-2.0 * s * z)) - LOG2


# ----------------------------------------------------------------------------
# RBM: log psi(x) = sum_i a_i x_i + sum_j logcosh(b_j + W_j . x)
# ----------------------------------------------------------------------------
class RBM:
    def __init__(self, a, b, W):
        self.a = np.asarray(a, dtype=np.complex128)
        self.b = np.asarray(b, dtype=np.complex128)
        self.W = np.asarray(W, dtype=np.complex128)  # (M, N)

    @property
    def block_sizes(self):
        M, N = self.W.shape
        return [M * N, M, N]

    @property
    def n_params(self):
        return sum(self.block_sizes)

    def flat(self):
        return np.concatenate([self.W.reshape(-1), self.b, self.a])

    @classmethod
    def from_flat(cls, theta, N, M):
        theta = np.asarray(theta, dtype=np.complex128)
        W = theta[: M * N].reshape(M, N)
        b = theta[M * N: M * N + M]
        a = theta[M * N + M:]
        return cls(a, b, W)

    def log_psi(self, x):
        x = np.asarray(x, dtype=np.float64)
        theta = x @ self.W.T + self.b
        return x @ self.a + logcosh(theta).sum(axis=-1)

    def jacobian(self, x, out_dtype=np.complex128):
        x = np.asarray(x, dtype=np.float64)
        ns, N = x.shape
        M = self.W.shape[0]
        t = np.tanh(x @ self.W.T + self.b)  # (ns, M)
        O = np.empty((ns, self.n_params), dtype=out_dtype)
        O[:, : M * N] = (t[:, :, None] * x[:, None, :]).reshape(ns, M * N)
        O[:, M * N: M * N + M] = t
        O[:, M * N + M:] = x
        return O


# ----------------------------------------------------------------------------
# FFNN: h0 = x, z^l = W^l h^{l-1} + b^l, h^l = logcosh(z^l);
#       log psi = sum_k h^L_k  (sum pool), or v . h^L + c with a dense readout.
# ----------------------------------------------------------------------------
class FFNN:
    def __init__(self, Ws, bs, readout=None):
        self.Ws = [np.asarray(W, dtype=np.complex128) for W in Ws]
        self.bs = [np.asarray(b, dtype=np.complex128) for b in bs]
        self.readout = None
        if readout is not None:
            v, c = readout
            self.readout = (np.asarray(v, dtype=np.complex128), np.complex128(c))

    @property
    def block_sizes(self):
        sizes = [W.size + b.size for W, b in zip(self.Ws, self.bs)]
        if self.readout is not None:
            sizes.append(self.readout[0].size + 1)
        return sizes

    @property
    def n_params(self):
        return sum(self.block_sizes)

    def flat(self):
        parts = []
        for W, b in zip(self.Ws, self.bs):
            parts += [W.reshape(-1), b]
        if self.readout is not None:
            parts += [self.readout[0], np.array([self.readout[1]])]
        return np.concatenate(parts)

    def with_flat(self, theta):
        theta = np.asarray(theta, dtype=np.complex128)
        Ws, bs, p = [], [], 0
        for W, b in zip(self.Ws, self.bs):
            Ws.append(theta[p: p + W.size].reshape(W.shape)); p += W.size
            bs.append(theta[p: p + b.size]); p += b.size
        ro = None
        if self.readout is not None:
            nv = self.readout[0].size
            ro = (theta[p: p + nv], theta[p + nv])
        return FFNN(Ws, bs, ro)

    def _forward(self, x):
        h = [np.asarray(x, dtype=np.complex128)]
        zs = []
        for W, b in zip(self.Ws, self.bs):
            z = h[-1] @ W.T + b
            zs.append(z)
            h.append(logcosh(z))
        return h, zs

    def log_psi(self, x):
        h, _ = self._forward(x)
        if self.readout is not None:
            v, c = self.readout
            return h[-1] @ v + c
        return h[-1].sum(axis=-1)

    def jacobian(self, x, out_dtype=np.complex128):
        h, zs = self._forward(x)
        ns = h[0].shape[0]
        O = np.empty((ns, self.n_params), dtype=out_dtype)
        L = len(self.Ws)
        # offsets of each layer block
        offs = np.concatenate([[0], np.cumsum(self.block_sizes)]).astype(np.int64)
        if self.readout is not None:
            v, _ = self.readout
            o = offs[L]
            O[:, o: o + v.size] = h[L]
            O[:, o + v.size] = 1.0
            g = np.tanh(zs[L - 1]) * v
        else:
            g = np.tanh(zs[L - 1])
        for l in range(L - 1, -1, -1):
            W = self.Ws[l]
            nout, nin = W.shape
            o = offs[l]
            O[:, o: o + nout * nin] = (g[:, :, None] * h[l][:, None, :]).reshape(ns, nout * nin)
            O[:, o + nout * nin: o + nout * nin + nout] = g
            if l > 0:
                g = np.tanh(zs[l - 1]) * (g @ W)
        return O


# ----------------------------------------------------------------------------
# CNN: periodic 3x3 cross-correlation layers on an L x L lattice, logcosh
# activations, sum pooling of the last layer.
# ----------------------------------------------------------------------------
_OFFSETS = [(dy - 1, dx - 1) for dy in range(3) for dx in range(3)]


def _neighbours(L, dy, dx):
    """Site index of (y+dy mod L, x+dx mod L) for every site s = y*L + x."""
    y, x = np.divmod(np.arange(L * L), L)
    return ((y + dy) % L) * L + (x + dx) % L


def _shift(h, L, dy, dx):
    """h: (ns, C, L*L) -> h'[..., s] = h[..., (y+dy mod L, x+dx mod L)]."""
    return h[..., _neighbours(L, dy, dx)]


def _im2col(h, L):
    """(ns, C, L*L) -> (ns, L*L, C*9): the 3x3 patch of every site, index c*9 + t."""
    idx = np.stack([_neighbours(L, dy, dx) for dy, dx in _OFFSETS])  # (9, L*L)
    cols = h[:, :, idx]                                              # (ns, C, 9, L*L)
    return np.ascontiguousarray(cols.transpose(0, 3, 1, 2)).reshape(h.shape[0], L * L, -1)


class CNN:
    def __init__(self, Ks, bs, L):
        self.Ks = [np.asarray(K, dtype=np.complex128) for K in Ks]  # (cout, cin, 3, 3)
        self.bs = [np.asarray(b, dtype=np.complex128) for b in bs]
        self.L = L

    @property
    def block_sizes(self):
        return [K.size + b.size for K, b in zip(self.Ks, self.bs)]

    @property
    def n_params(self):
        return sum(self.block_sizes)

    def flat(self):
        parts = []
        for K, b in zip(self.Ks, self.bs):
            parts += [K.reshape(-1), b]
        return np.concatenate(parts)

    def with_flat(self, theta):
        theta = np.asarray(theta, dtype=np.complex128)
        Ks, bs, p = [], [], 0
        for K, b in zip(self.Ks, self.bs):
            Ks.append(theta[p: p + K.size].reshape(K.shape)); p += K.size
            bs.append(theta[p: p + b.size]); p += b.size
        return CNN(Ks, bs, self.L)

    def _conv(self, K, b, h):
        # z[n, o, s] = b[o] + sum_{c, t} K[o, c, t] h[n, c, s + d_t]: one GEMM over all sites
        ns, L = h.shape[0], self.L
        cols = _im2col(h, L).reshape(ns * L * L, -1)                 # (ns*s, C*9)
        z = (cols @ K.reshape(K.shape[0], -1).T).reshape(ns, L * L, -1)
        return np.ascontiguousarray(z.transpose(0, 2, 1)) + b[None, :, None]

    def _forward(self, x):
        x = np.asarray(x, dtype=np.complex128)
        h = [x.reshape(x.shape[0], 1, self.L * self.L)]
        zs = []
        for K, b in zip(self.Ks, self.bs):
            z = self._conv(K, b, h[-1])
            zs.append(z)
            h.append(logcosh(z))
        return h, zs

    def log_psi(self, x):
        h, _ = self._forward(x)
        return h[-1].sum(axis=(1, 2))

    def jacobian(self, x, out_dtype=np.complex128):
        L = self.L
        h, zs = self._forward(x)
        ns = h[0].shape[0]
        O = np.empty((ns, self.n_params), dtype=out_dtype)
        offs = np.concatenate([[0], np.cumsum(self.block_sizes)]).astype(np.int64)
        g = np.tanh(zs[-1])
        for l in range(len(self.Ks) - 1, -1, -1):
            K = self.Ks[l]
            cout, cin = K.shape[:2]
            # O_K[n, o, c, t] = sum_s g[n, o, s] h^{l-1}[n, c, s + d_t]  (a per-sample product)
            dK = np.matmul(np.ascontiguousarray(g), _im2col(h[l], L))  # (ns, cout, cin*9)
            o = offs[l]
            O[:, o: o + K.size] = dK.reshape(ns, -1)
            O[:, o + K.size: o + K.size + cout] = g.sum(axis=2)
            if l > 0:
                # d log psi / d h^{l-1}[c', s'] = sum_{c, t} K[c, c', t] g[c, s' - d_t]
                P = (K.reshape(cout, cin * 9).T @ g.transpose(1, 0, 2).reshape(cout, -1)).reshape(cin, 9, ns, L * L)
                back = np.zeros((ns, cin, L * L), dtype=np.complex128)
                for t, (dy, dx) in enumerate(_OFFSETS):
                    back += P[:, t][..., _neighbours(L, -dy, -dx)].transpose(1, 0, 2)
                g = np.tanh(zs[l - 1]) * back
        return O
