"""FP64 CPU oracle for block-layer stochastic reconfiguration.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference that the
GPU library is checked against.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.  It
shares no code with the HIP library.

What it computes (paper: Sec. 2):
  * O_i(x) = d log psi(x) / d theta_i is the input (the definition after Eq. 2).
  * Delta O_i(x) = O_i(x) - <O_i>, sample means with population weights 1/n_s
    (the expectation in Eq. 2 estimated over the samples).
  * The QGT S_ij = E[conj(Delta O_i) Delta O_j] (Eq. 2, covariance form); the
    block-layer QGT keeps only the diagonal blocks S_l of the layer partition
    (Eq. 3).
  * The force F_i = E[conj(Delta O_i) Delta E], Delta E = E_loc - <E_loc>: the
    holomorphic gradient of the variational energy of Eq. 1 with respect to
    conj(theta_i), estimated from the same samples as S (Sec. 2, the NGD
    paragraph).
  * Each block is shifted, S~_l = S_l + lambda I, and solved independently:
    delta_l = S~_l^{-1} F_l (Sec. 2, block-layer QGT paragraph).  The inverse is
    taken by full diagonalisation with a spectral cutoff, the pseudo-inverse the
    paper describes for the full QGT (Sec. 1 and Sec. 2).  The learning rate and
    the minus sign of the update are left to the caller.
  * delta = (delta_1, ..., delta_L) concatenated in parameter order.
  * Sample-space form: where n_s < n_l the same solve is taken through the
    n_s x n_s matrix T_l = Delta O_l Delta O_l^H / n_s (the NTK-like
    reformulation mentioned in Sec. 1), (T_l + lambda I) z = Delta E,
    delta_l = Delta O_l^H z / n_s.  By the push-through (Woodbury) identity this
    equals (S_l + lambda I)^{-1} F_l exactly.

Readings of points the paper leaves open are listed in the design notes:
population normalisation 1/n_s; the conjugate sits on the first index; the
library returns S~^{-1} F without -eta; the energy is centred before use;
a cutoff rcond = 1e-14 relative to the largest shifted eigenvalue.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

DEFAULT_RCOND = 1e-14


def block_offsets(block_sizes):
    """Start offset of each block (prefix sums of the layer sizes)."""
    offs = [0]
    for n in block_sizes:
        offs.append(offs[-1] + int(n))
    return offs


def centred_energy(e_loc, weights=None):
    """Delta E = E_loc - <E_loc> (Eq. 1 estimated over the samples)."""
    e = np.asarray(e_loc, dtype=np.complex128)
    if weights is None:
        return e - e.mean()
    w = np.asarray(weights, dtype=np.float64)
    return e - np.sum(w * e)


def centred_block(O, lo, hi, weights=None):
    """Delta O for the columns [lo, hi) of O, in complex128 (Eq. 2)."""
    blk = np.asarray(O[:, lo:hi], dtype=np.complex128)
    if weights is None:
        mu = blk.mean(axis=0)
    else:
        mu = np.asarray(weights, dtype=np.float64) @ blk
    return blk - mu


def qgt_block(dO, weights=None):
    """S_l = E[conj(dO_i) dO_j] for one block (Eq. 2 covariance form, Eq. 3)."""
    if weights is None:
        return dO.conj().T @ dO / dO.shape[0]
    w = np.asarray(weights, dtype=np.float64)
    return dO.conj().T @ (w[:, None] * dO)


def force_block(dO, dE, weights=None):
    """F_l = E[conj(dO_i) dE] for one block."""
    if weights is None:
        return dO.conj().T @ dE / dO.shape[0]
    w = np.asarray(weights, dtype=np.float64)
    return dO.conj().T @ (w * dE)


def sample_space_matrix(dO):
    """T_l = dO dO^H / n_s, the n_s x n_s sample-space matrix of one block."""
    return dO @ dO.conj().T / dO.shape[0]


def shifted_pinv_apply(A, rhs, lam, rcond=DEFAULT_RCOND):
    """x = (A + lam I)^+ rhs by full diagonalisation with a spectral cutoff.

    Returns (x, info) with info = dict(kappa, n_cut, eig_min, eig_max) of A + lam I.
    """
    w, V = np.linalg.eigh(A)
    d = w + lam
    dmax = d.max()
    keep = d > rcond * dmax
    Vk = V[:, keep]
    x = Vk @ ((Vk.conj().T @ rhs) / d[keep])
    info = dict(kappa=float(dmax / d[keep].min()), n_cut=int((~keep).sum()),
                eig_min=float(d.min()), eig_max=float(dmax))
    return x, info


@dataclass
class BlockResult:
    delta: np.ndarray
    forms: list = field(default_factory=list)      # 'P' or 'S' per block
    kappa: list = field(default_factory=list)      # condition number of the shifted block
    n_cut: list = field(default_factory=list)      # eigenvalues removed by the cutoff
    force: np.ndarray | None = None
    mu: np.ndarray | None = None


def choose_form(n_b, n_s):
    """Sample-space form iff n_s < n_b; at equality the parameter form is used."""
    return "S" if n_s < n_b else "P"


def block_sr(O, e_loc, block_sizes, lam, rcond=DEFAULT_RCOND, forms=None, weights=None,
             keep_force=True):
    """Block-layer SR step: delta = (S~_l^{-1} F_l)_l (Sec. 2, Eq. 3).

    O: (n_s, n_p) complex (any precision, promoted to complex128).
    forms: optional list of 'P'/'S' overriding the automatic choice.
    weights: optional per-sample probabilities replacing 1/n_s (the exact
      expectation of Eq. 2 over an enumerated Hilbert space); only the
      parameter form is defined for them.
    """
    n_s, n_p = O.shape
    offs = block_offsets(block_sizes)
    if offs[-1] != n_p:
        raise ValueError("block sizes do not sum to the number of columns")
    if not (lam > 0):
        raise ValueError("lambda must be positive")
    dE = centred_energy(e_loc, weights)
    delta = np.zeros(n_p, dtype=np.complex128)
    F = np.zeros(n_p, dtype=np.complex128) if keep_force else None
    mu = np.zeros(n_p, dtype=np.complex128) if keep_force else None
    res = BlockResult(delta=delta, force=F, mu=mu)
    for b, n_b in enumerate(block_sizes):
        lo, hi = offs[b], offs[b + 1]
        dO = centred_block(O, lo, hi, weights)
        if keep_force:
            blk = np.asarray(O[:, lo:hi], dtype=np.complex128)
            mu[lo:hi] = blk.mean(axis=0) if weights is None else np.asarray(weights) @ blk
        form = forms[b] if forms is not None else choose_form(n_b, n_s)
        Fb = force_block(dO, dE, weights)
        if keep_force:
            F[lo:hi] = Fb
        if form == "P":
            Sb = qgt_block(dO, weights)
            db, info = shifted_pinv_apply(Sb, Fb, lam, rcond)
        else:
            if weights is not None:
                raise ValueError("the sample-space form is defined for equal weights only")
            Tb = sample_space_matrix(dO)
            z, info = shifted_pinv_apply(Tb, dE, lam, rcond)
            db = dO.conj().T @ z / n_s
        delta[lo:hi] = db
        res.forms.append(form)
        res.kappa.append(info["kappa"])
        res.n_cut.append(info["n_cut"])
    return res


def full_sr(O, e_loc, lam, rcond=DEFAULT_RCOND, form=None, weights=None):
    """Full-QGT SR: the block method with a single block spanning all parameters."""
    n_p = O.shape[1]
    return block_sr(O, e_loc, [n_p], lam, rcond, None if form is None else [form], weights)


def sample_space_z(O, e_loc, lo, hi, lam, rcond=DEFAULT_RCOND):
    """The sample-space solution z of (T_l + lam I) z = Delta E for one block."""
    dE = centred_energy(e_loc)
    dO = centred_block(O, lo, hi)
    z, _ = shifted_pinv_apply(sample_space_matrix(dO), dE, lam, rcond)
    return z


def block_residual_norms(O, e_loc, block_sizes, lam, delta):
    """Matrix-free FP64 residual r_l = F_l - S_l delta_l - lam delta_l per block.

    Returns a list of (||r_l||, ||delta_l||).  Since S_l + lam I >= lam I, the
    error of delta_l is bounded by ||r_l|| / lam: an a-posteriori check usable
    at any size.
    """
    n_s = O.shape[0]
    dE = centred_energy(e_loc)
    out = []
    offs = block_offsets(block_sizes)
    for b in range(len(block_sizes)):
        lo, hi = offs[b], offs[b + 1]
        dO = centred_block(O, lo, hi)
        d = np.asarray(delta[lo:hi], dtype=np.complex128)
        Fb = dO.conj().T @ dE / n_s
        r = Fb - dO.conj().T @ (dO @ d) / n_s - lam * d
        out.append((float(np.linalg.norm(r)), float(np.linalg.norm(d))))
    return out


def block_sr_cholesky(O, e_loc, block_sizes, lam):
    """CPU block SR by Cholesky factorisation (scipy), the CPU speed comparator.

    Same definition as block_sr; only the inversion method differs (Cholesky of
    the shifted Hermitian positive-definite block instead of diagonalisation).
    """
    n_s, n_p = O.shape
    offs = block_offsets(block_sizes)
    dE = centred_energy(e_loc)
    delta = np.zeros(n_p, dtype=np.complex128)
    for b, n_b in enumerate(block_sizes):
        lo, hi = offs[b], offs[b + 1]
        dO = centred_block(O, lo, hi)
        if choose_form(n_b, n_s) == "P":
            A = qgt_block(dO)
            A[np.diag_indices_from(A)] += lam
            delta[lo:hi] = sla.cho_solve(sla.cho_factor(A, lower=True), force_block(dO, dE))
        else:
            A = sample_space_matrix(dO)
            A[np.diag_indices_from(A)] += lam
            z = sla.cho_solve(sla.cho_factor(A, lower=True), dE)
            delta[lo:hi] = dO.conj().T @ z / n_s
    return delta


def relative_error(a, b):
    """||a - b|| / ||b|| (b the reference)."""
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0))


def block_relative_errors(delta, ref, block_sizes):
    offs = block_offsets(block_sizes)
    return [relative_error(delta[offs[b]:offs[b + 1]], ref[offs[b]:offs[b + 1]])
            for b in range(len(block_sizes))]
