"""FP64 CPU oracle for a variational Monte Carlo loop around block SR.

TEST INFRASTRUCTURE ONLY.  The plain, slow reference that the device sampler,
local energies and loop are checked against.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg may import it; the product path never
does.  It shares no code with the HIP library.

What it computes (paper, Sec. 2 and Sec. 3):
  * The spin-1/2 Heisenberg chain H = J sum_i S_i . S_{i+1}, S = sigma / 2
    (Sec. 3, Heisenberg paragraph), periodic or open.  In the sigma^z basis
    S_i . S_j = sigma^z_i sigma^z_j / 4 + (sigma^+_i sigma^-_j + h.c.) / 2, so
    the local energy (Eq. 1 estimated over samples) is
        E_loc(x) = sum_x' H[x, x'] psi(x') / psi(x)
                 = J sum_bonds [ x_i x_j / 4 + [x_i != x_j] psi(x^{ij}) / (2 psi(x)) ],
    x^{ij} the configuration with spins i and j exchanged.
  * Samples from |psi|^2 by a Metropolis chain of exchange moves (the
    magnetisation is conserved): the move exchanges spins i and j (a no-op
    when they are equal) and is accepted when u < |psi(x') / psi(x)|^2.  The
    pairs (i, j) and the uniforms u are inputs, drawn by the input generators.
  * The exact ground-state energy by Lanczos (scipy's eigsh) on the sparse H
    restricted to the zero-magnetisation sector.
  * One VMC iteration: sample, local energies, O (oracle.jacobian), the block
    SR update delta (oracle.block_sr), theta <- theta - eta delta.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import block_sr as orc
from . import jacobian as jac


def bonds(N, pbc=True):
    """Nearest-neighbour bonds (i, i + 1) of a chain, with (N - 1, 0) when periodic."""
    out = [(i, i + 1) for i in range(N - 1)]
    if pbc and N > 2:
        out.append((N - 1, 0))
    return out


def heisenberg_eloc(log_psi, x, J=1.0, pbc=True):
    """Local energies of the samples x (n_s x N, +-1) for a log-amplitude
    function log_psi(configs) -> complex array."""
    x = np.asarray(x, dtype=np.int8)
    n_s, N = x.shape
    lp = log_psi(x)
    e = np.zeros(n_s, dtype=np.complex128)
    for i, j in bonds(N, pbc):
        e += J * 0.25 * x[:, i].astype(np.float64) * x[:, j]
        flip = x[:, i] != x[:, j]
        if flip.any():
            xs = x[flip].copy()
            xs[:, [i, j]] = xs[:, [j, i]]
            e[flip] += J * 0.5 * np.exp(log_psi(xs) - lp[flip])
    return e


def metropolis_exchange(log_psi, x0, pairs, u):
    """Chains started at x0 (n_chains x N); step s of chain c exchanges spins
    pairs[s, c] and is accepted when u[s, c] < |psi(x') / psi(x)|^2.
    Returns the final configurations and the number of accepted moves."""
    x = np.array(x0, dtype=np.int8, copy=True)
    n_steps, n_chains = u.shape
    accepted = 0
    for s in range(n_steps):
        for c in range(n_chains):
            i, j = pairs[s, c]
            if x[c, i] == x[c, j]:
                continue
            xp = x[c].copy()
            xp[i], xp[j] = xp[j], xp[i]
            d = log_psi(xp[None, :])[0] - log_psi(x[c][None, :])[0]
            if u[s, c] < np.exp(2.0 * d.real):
                x[c] = xp
                accepted += 1
    return x, accepted


def heisenberg_matrix_sz0(N, J=1.0, pbc=True):
    """Sparse H on the zero-magnetisation sector; returns (H, basis), basis the
    configurations (+-1) in lexicographic order of their up positions."""
    ups = list(itertools.combinations(range(N), N // 2))
    basis = -np.ones((len(ups), N), dtype=np.int8)
    for r, u in enumerate(ups):
        basis[r, list(u)] = 1
    index = {b.tobytes(): r for r, b in enumerate(basis)}
    rows, cols, vals = [], [], []
    for r, b in enumerate(basis):
        diag = 0.0
        for i, j in bonds(N, pbc):
            diag += 0.25 * J * b[i] * b[j]
            if b[i] != b[j]:
                bb = b.copy()
                bb[i], bb[j] = bb[j], bb[i]
                rows.append(r); cols.append(index[bb.tobytes()]); vals.append(0.5 * J)
        rows.append(r); cols.append(r); vals.append(diag)
    H = sp.csr_matrix((vals, (rows, cols)), shape=(len(basis), len(basis)))
    return H, basis


def ground_state(N, J=1.0, pbc=True):
    """(E0, psi0, basis) of the chain in the zero-magnetisation sector (Lanczos)."""
    H, basis = heisenberg_matrix_sz0(N, J, pbc)
    w, v = spla.eigsh(H, k=1, which="SA", tol=1e-12)
    return float(w[0]), v[:, 0], basis


def rbm_vmc_iteration(theta, N, M, x0, pairs, u, lam, eta, J=1.0, pbc=True, full_qgt=False):
    """One VMC iteration with the RBM: Metropolis sampling, local energies, O,
    the SR update and the parameter step.  The update is block SR over the
    layer blocks W, b, a (Sec. 2, Eq. 3), or with full_qgt the SR of the whole
    QGT (Eq. 2: one block of all parameters).  Returns (new theta, final
    samples, mean local energy, delta)."""
    log_psi = lambda xx: jac.rbm_log_psi(theta, N, M, xx)
    x, _ = metropolis_exchange(log_psi, x0, pairs, u)
    e = heisenberg_eloc(log_psi, x, J, pbc)
    O = jac.rbm_jacobian(theta, N, M, x)
    res = orc.block_sr(O, e, [M * N + M + N] if full_qgt else [M * N, M, N], lam)
    return np.asarray(theta) - eta * res.delta, x, complex(e.mean()), res.delta
