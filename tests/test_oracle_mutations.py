"""Planted mistakes in the oracle must be caught by its pins.

Each case replaces one oracle function with a plausibly wrong version (a
dropped term, a wrong conjugation, a wrong normalisation, a wrong sign) and
checks that at least one pin of tests/test_oracle_pins.py fails.  Everything
runs on the CPU.
"""
import numpy as np
import pytest

import tests.test_oracle_pins as pins
from oracle import block_sr as orc

PIN_TESTS = [
    lambda: pins.test_sample_space_with_large_energy_offset(),
    lambda: pins.test_exact_qgt_state_vector_form("rbm"),
    lambda: pins.test_force_is_gradient_of_exact_energy(),
    lambda: pins.test_hadamard_closed_form_pform(),
    lambda: pins.test_hadamard_closed_form_sform(),
    lambda: pins.test_golden_fixtures("tiny_pform.json"),
    lambda: pins.test_golden_fixtures("tiny_sform.json"),
    lambda: pins.test_woodbury_parameter_vs_sample_space(
        pins.workloads.small_ffnn(n_s=96, N=8, widths=(12, 6), readout=True, lam=1e-3)),
]


def _qgt_transposed(dO, weights=None):
    n = dO.shape[0]
    if weights is None:
        return dO.T @ dO.conj() / n
    return dO.T @ (np.asarray(weights)[:, None] * dO.conj())


def _centred_not(O, lo, hi, weights=None):
    return np.asarray(O[:, lo:hi], dtype=np.complex128)


def _force_no_conj(dO, dE, weights=None):
    if weights is None:
        return dO.T @ dE / dO.shape[0]
    return dO.T @ (np.asarray(weights) * dE)


def _qgt_unbiased(dO, weights=None):
    if weights is None:
        return dO.conj().T @ dO / (dO.shape[0] - 1)
    return dO.conj().T @ (np.asarray(weights)[:, None] * dO) * 1.01


def _energy_not_centred(e_loc, weights=None):
    return np.asarray(e_loc, dtype=np.complex128)


def _sample_matrix_unscaled(dO):
    return dO @ dO.conj().T


def _pinv_wrong_shift_sign(A, rhs, lam, rcond=orc.DEFAULT_RCOND):
    w, V = np.linalg.eigh(A)
    d = w + lam
    d = np.where(d > 0.5 * d.max(), d, d - 2 * lam)  # drop the shift on the small modes
    d[np.abs(d) < 1e-300] = 1.0
    x = V @ ((V.conj().T @ rhs) / d)
    return x, dict(kappa=1.0, n_cut=0, eig_min=float(d.min()), eig_max=float(d.max()))


def _pinv_transposed_eigvec(A, rhs, lam, rcond=orc.DEFAULT_RCOND):
    w, V = np.linalg.eigh(A)
    d = w + lam
    x = V.conj() @ ((V.T @ rhs) / d)
    return x, dict(kappa=1.0, n_cut=0, eig_min=float(d.min()), eig_max=float(d.max()))


MUTATIONS = {
    "qgt_conjugate_on_second_index": ("qgt_block", _qgt_transposed),
    "no_centring_of_O": ("centred_block", _centred_not),
    "force_without_conjugate": ("force_block", _force_no_conj),
    "wrong_normalisation": ("qgt_block", _qgt_unbiased),
    "energy_not_centred": ("centred_energy", _energy_not_centred),
    "sample_space_missing_1_over_ns": ("sample_space_matrix", _sample_matrix_unscaled),
    "shift_dropped_on_small_modes": ("shifted_pinv_apply", _pinv_wrong_shift_sign),
    "eigenvectors_transposed": ("shifted_pinv_apply", _pinv_transposed_eigvec),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, bad = MUTATIONS[name]
    monkeypatch.setattr(orc, attr, bad)
    caught = 0
    for t in PIN_TESTS:
        try:
            t()
        except (AssertionError, ValueError, np.linalg.LinAlgError):
            caught += 1
    assert caught >= 1, f"no pin catches the planted mistake {name}"
