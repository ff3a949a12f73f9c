"""Pins of the Eq. 4 diagnostics oracle (oracle/diagnostics.py) against closed
forms, invariants and special cases fixed by the definitions, plus planted
mistakes that they catch."""
import numpy as np
import pytest

from gen import workloads
from oracle import block_sr as orc
from oracle import diagnostics as dg


def random_hpd(n, seed, spread=1e3):
    """Hermitian positive definite matrix with eigenvalues spanning `spread`."""
    g = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(g.normal(size=(n, n)) + 1j * g.normal(size=(n, n)))
    w = np.geomspace(1.0, spread, n)
    return (Q * w) @ Q.conj().T, w, Q


def test_overlap_and_error_identities():
    A, _, _ = random_hpd(12, 1)
    B, _, _ = random_hpd(12, 2)
    assert dg.frobenius_overlap(A, A) == pytest.approx(1.0, abs=1e-14)
    assert dg.frobenius_relative_error(A, A) == 0.0
    assert dg.frobenius_overlap(A, 3.5 * A) == pytest.approx(1.0, abs=1e-14)   # scale invariant
    assert dg.frobenius_overlap(A, -A) == pytest.approx(-1.0, abs=1e-14)
    assert dg.frobenius_overlap(A, B) == pytest.approx(dg.frobenius_overlap(B, A), abs=1e-14)
    assert dg.frobenius_relative_error(0.75 * B, B) == pytest.approx(0.25, abs=1e-14)
    assert -1.0 <= dg.frobenius_overlap(A, B) <= 1.0


def test_diagonal_closed_forms():
    a = np.array([4.0, 1.0, 0.5, 2.0])
    b = np.array([3.0, 2.0, 0.25, 1.0])
    A, B = np.diag(a), np.diag(b)
    assert dg.frobenius_overlap(A, B) == pytest.approx((12 + 2 + 0.125 + 2) / np.sqrt(21.25 * 14.0625), rel=1e-14)
    assert dg.frobenius_relative_error(A, B) == pytest.approx(np.sqrt(1 + 1 + 0.0625 + 1) / np.sqrt(14.0625),
                                                              rel=1e-14)
    assert dg.condition_number(A) == 8.0
    # eigenvalues sorted descending: (4, 2, 1, 0.5) and (3, 2, 1, 0.25)
    x, y = np.array([4, 2, 1, 0.5]), np.array([3, 2, 1, 0.25])
    x, y = x - x.mean(), y - y.mean()
    assert dg.spectral_correlation(A, B) == pytest.approx(x @ y / np.sqrt((x @ x) * (y @ y)), rel=1e-13)


def test_condition_number_and_spectrum_are_basis_free():
    A, w, Q = random_hpd(10, 3, spread=1e6)
    assert dg.condition_number(A) == pytest.approx(1e6, rel=1e-8)
    # the same spectrum in another basis: perfectly correlated spectra,
    # although the matrices differ (a list sorted one way against the other
    # way would give -1)
    B, _, _ = random_hpd(10, 4, spread=1e6)
    assert dg.spectral_correlation(A, B) == pytest.approx(1.0, abs=1e-12)
    assert dg.frobenius_overlap(A, B) < 0.9
    # Pearson: invariant under positive scaling and shifts of one spectrum
    C, _, _ = random_hpd(10, 5, spread=50.0)
    r = dg.spectral_correlation(A, C)
    assert dg.spectral_correlation(7.0 * A, C) == pytest.approx(r, abs=1e-12)
    assert dg.spectral_correlation(A + 2.0 * np.eye(10), C) == pytest.approx(r, abs=1e-12)


def test_two_by_two_block_versus_full_closed_form():
    """S = [[s1, c], [conj(c), s2]] with one parameter per block: the block
    inverse is diag(1/(s1+l), 1/(s2+l)), the full inverse
    [[s2+l, -c], [-conj(c), s1+l]] / det."""
    s1, s2, c, lam = 2.0, 0.5, 0.6 - 0.3j, 0.1
    S = np.array([[s1, c], [np.conj(c), s2]])
    A_blk = dg.block_layer_inverse(S, [1, 1], lam)
    A_full = dg.shifted_inverse(S, lam)
    p, q = s1 + lam, s2 + lam
    det = p * q - abs(c) ** 2
    np.testing.assert_allclose(A_blk, np.diag([1 / p, 1 / q]), rtol=1e-14)
    np.testing.assert_allclose(A_full, np.array([[q, -c], [-np.conj(c), p]]) / det, rtol=1e-13)
    tr = q / (det * p) + p / (det * q)
    na = np.sqrt(1 / p ** 2 + 1 / q ** 2)
    nb = np.sqrt(p ** 2 + q ** 2 + 2 * abs(c) ** 2) / det
    assert dg.frobenius_overlap(A_blk, A_full) == pytest.approx(tr / (na * nb), rel=1e-13)


def test_block_diagonal_qgt_gives_identical_inverses():
    """Hadamard columns (exactly orthogonal over the samples) make the QGT
    exactly block-diagonal: block-layer and full inverses coincide."""
    n_s = 32
    H = np.array([[1.0]])
    while H.shape[0] < n_s:
        H = np.block([[H, H], [H, -H]])
    O = (H[:, 1:6] * np.array([1.0, 2.0, 0.5, 1j, 3.0])).astype(np.complex128)
    S = dg.qgt(O)
    assert np.abs(S - np.diag(np.diag(S))).max() == 0.0
    A_blk = dg.block_layer_inverse(S, [2, 3], 1e-2)
    A_full = dg.shifted_inverse(S, 1e-2)
    d = dg.diagnostics(A_blk, A_full)
    assert d["frobenius_overlap"] == pytest.approx(1.0, abs=1e-13)
    assert d["frobenius_relative_error"] <= 1e-13
    assert d["spectral_correlation"] == pytest.approx(1.0, abs=1e-13)


def test_full_qgt_of_the_enumerated_set_is_exact():
    """Samples that are the enumerated configurations with uniform Born weights
    make the sampled full QGT the exact one: the full inverse against the exact
    inverse gives F = 1, eps_F = 0, r = 1; the block-layer inverse differs by
    the dropped cross-layer blocks."""
    w = workloads.config0(n_s=256)
    res = dg.compare_block_full_exact(w.O, w.O, np.ones(w.n_s), w.block_sizes, w.lam)
    assert res["full"]["frobenius_overlap"] == pytest.approx(1.0, abs=1e-12)
    assert res["full"]["frobenius_relative_error"] <= 1e-10
    assert res["full"]["spectral_correlation"] == pytest.approx(1.0, abs=1e-12)
    assert res["block"]["frobenius_overlap"] < 1.0
    assert res["block"]["frobenius_relative_error"] > 1e-6


def test_planted_mistakes_are_caught():
    A, _, _ = random_hpd(8, 6, spread=1e4)
    B, _, _ = random_hpd(8, 7, spread=1e2)
    # spectra sorted in opposite orders
    a = np.sort(np.linalg.eigvalsh(A))[::-1]
    b = np.sort(np.linalg.eigvalsh(B))
    assert np.corrcoef(a, b)[0, 1] < 0 < dg.spectral_correlation(A, B)
    # the overlap without the normalisation, or the error relative to A
    assert abs(np.real(np.trace(A.conj().T @ B)) - dg.frobenius_overlap(A, B)) > 1e-3
    assert abs(np.linalg.norm(A - B) / np.linalg.norm(A) - dg.frobenius_relative_error(A, B)) > 1e-3
    # the inverse of the unshifted block is not the inverse of the shifted one
    S, _, _ = random_hpd(6, 8, spread=10.0)
    assert np.abs(np.linalg.inv(S) - dg.shifted_inverse(S, 0.5)).max() > 1e-3
    np.testing.assert_allclose(dg.shifted_inverse(S, 0.5) @ (S + 0.5 * np.eye(6)), np.eye(6), atol=1e-12)
