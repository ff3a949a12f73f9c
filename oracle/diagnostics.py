"""FP64 CPU oracle of the paper's diagnostics of the inverse QGT (Sec. 3, Eq. 4).

TEST INFRASTRUCTURE ONLY, like the rest of oracle/: the tests, the smoke check
and the benchmark's CPU leg may import it; the product path never does.

Let A be an approximate inverse metric (the inverse of the shifted block-layer
QGT, or of the shifted full sampled QGT) and B the reference (the inverse of
the shifted QGT computed exactly over the Hilbert space).  Eq. 4 defines

  (a) the Frobenius overlap      F(A, B)    = Tr[A^dagger B] / (||A||_F ||B||_F)
  (b) the Frobenius rel. error   eps_F(A,B) = ||A - B||_F / ||B||_F
  (c) the condition number       kappa(A)   = lambda_max(A) / lambda_min(A)
  (d) the spectral correlation   r(A, B)    = corr of the eigenvalues of A and
                                              of B, each sorted in descending
                                              order

Readings (the paper leaves these open):
  * corr in (d) is Pearson's correlation coefficient of the two sorted
    eigenvalue lists.
  * The matrices are Hermitian, so Tr[A^dagger B] is real up to rounding; (a)
    returns its real part.
  * The inverses are those of the shifted matrices S + lambda I (the shift the
    method uses, Sec. 2), for the block-layer approximation the block-diagonal
    matrix of the inverses of the shifted blocks.
  * The exact QGT is the covariance form of Eq. 2 with the expectation taken
    over the normalised Born distribution |psi(x)|^2 / sum |psi|^2 on an
    enumerated set of configurations (the whole Hilbert space, or a symmetry
    sector of it).
"""
from __future__ import annotations

import numpy as np

from . import block_sr as orc


def frobenius_overlap(A, B):
    """Eq. 4 (a): Re Tr[A^dagger B] / (||A||_F ||B||_F)."""
    A = np.asarray(A)
    B = np.asarray(B)
    return float(np.real(np.sum(np.conj(A) * B)) / (np.linalg.norm(A) * np.linalg.norm(B)))


def frobenius_relative_error(A, B):
    """Eq. 4 (b): ||A - B||_F / ||B||_F."""
    return float(np.linalg.norm(np.asarray(A) - np.asarray(B)) / np.linalg.norm(B))


def condition_number(A):
    """Eq. 4 (c): largest over smallest eigenvalue of the Hermitian matrix A."""
    w = np.linalg.eigvalsh(A)
    return float(w[-1] / w[0])


def spectral_correlation(A, B):
    """Eq. 4 (d): Pearson correlation of the eigenvalues of A and of B, each
    list sorted in descending order."""
    a = np.sort(np.linalg.eigvalsh(A))[::-1]
    b = np.sort(np.linalg.eigvalsh(B))[::-1]
    a = a - a.mean()
    b = b - b.mean()
    return float(np.dot(a, b) / np.sqrt(np.dot(a, a) * np.dot(b, b)))


def shifted_inverse(S, lam):
    """(S + lambda I)^{-1} of a Hermitian positive semi-definite S, by
    diagonalisation."""
    w, V = np.linalg.eigh(S)
    return (V / (w + lam)) @ V.conj().T


def qgt(O, weights=None):
    """The QGT of all parameters (Eq. 2, covariance form): sample means, or
    expectations under the normalised weights."""
    dO = orc.centred_block(O, 0, O.shape[1], weights=weights)
    return orc.qgt_block(dO, weights=weights)


def block_layer_inverse(S, block_sizes, lam):
    """The inverse of the shifted block-layer QGT (Eq. 3 and the shift after
    it): the block-diagonal matrix of the inverses of the shifted diagonal
    blocks of S."""
    n = S.shape[0]
    A = np.zeros((n, n), dtype=np.complex128)
    offs = orc.block_offsets(block_sizes)
    for b in range(len(block_sizes)):
        lo, hi = offs[b], offs[b + 1]
        A[lo:hi, lo:hi] = shifted_inverse(S[lo:hi, lo:hi], lam)
    return A


def diagnostics(A, B):
    """All four quantities of Eq. 4 for an approximate inverse A against B."""
    return {"frobenius_overlap": frobenius_overlap(A, B),
            "frobenius_relative_error": frobenius_relative_error(A, B),
            "condition_number": condition_number(A),
            "spectral_correlation": spectral_correlation(A, B)}


def compare_block_full_exact(O_samples, O_all, p_all, block_sizes, lam):
    """The comparison of the paper's table of diagnostics: the inverse of the
    shifted block-layer QGT and of the shifted full QGT, both estimated from
    the samples (rows of O_samples), against the inverse of the shifted exact
    QGT (rows of O_all over the enumerated configurations, Born weights
    p_all).  Returns {"block": {...}, "full": {...}, "exact_condition_number": ...}."""
    S_samp = qgt(O_samples)
    p = np.asarray(p_all, dtype=np.float64)
    S_exact = qgt(O_all, weights=p / p.sum())
    B = shifted_inverse(S_exact, lam)
    A_block = block_layer_inverse(S_samp, block_sizes, lam)
    A_full = shifted_inverse(S_samp, lam)
    return {"block": diagnostics(A_block, B), "full": diagnostics(A_full, B),
            "exact_condition_number": condition_number(B)}
