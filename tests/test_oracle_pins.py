"""Pins of the FP64 oracle (and of the input Jacobians) against facts fixed by
the paper and by mathematics, independent of the oracle's own formulas:

  C1  explicit Jacobians vs central finite differences of log psi
  C2  the covariance form of the QGT vs the state-vector form of Eq. 2 over an
      enumerated Hilbert space (derivatives of psi by finite differences), and
      the force vs the finite-difference gradient of the exact energy (Eq. 1)
      of a Heisenberg chain
  C3  parameter-space vs sample-space solve (Woodbury)
  C4  one block spanning all parameters reproduces full SR; exactly
      block-diagonal QGT gives block SR == full SR
  I*  invariants (Hermiticity, shift invariances, scaling, gradient limit,
      zero-magnetisation null directions, permutation of samples)
  H*  Hadamard closed forms, including the conjugation convention and exact
      centring
  golden  hand-derived tiny cases under tests/golden/
"""
import json
import os

import numpy as np
import pytest

from gen import networks, workloads
from oracle import block_sr as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# helpers local to the tests (not shared with the oracle)
# ---------------------------------------------------------------------------
def all_configs(N):
    idx = np.arange(2 ** N)[:, None]
    bits = (idx >> np.arange(N)[None, :]) & 1
    return (2 * bits - 1).astype(np.int8)


def hadamard(n):
    H = np.array([[1.0]])
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    return H


def heisenberg_matrix(N):
    """H = sum_i S_i . S_{i+1} with periodic boundaries, S = sigma/2 (Sec. 3)."""
    X = all_configs(N)
    dim = X.shape[0]
    H = np.zeros((dim, dim))
    for i in range(N):
        j = (i + 1) % N
        zz = X[:, i].astype(float) * X[:, j]
        H[np.arange(dim), np.arange(dim)] += zz / 4.0
        anti = zz < 0
        flipped = np.arange(dim) ^ ((1 << i) | (1 << j))
        H[np.arange(dim)[anti], flipped[anti]] += 0.5
    return X, H


# ---------------------------------------------------------------------------
# logcosh branch convention
# ---------------------------------------------------------------------------
def test_logcosh_is_a_log_of_cosh():
    g = np.random.default_rng(0)
    z = g.normal(0, 3, 200) + 1j * g.normal(0, 3, 200)
    lc = networks.logcosh(z)
    np.testing.assert_allclose(np.exp(lc), np.cosh(z), rtol=1e-12)
    # even function, up to the 2 pi i of the branch
    d = (networks.logcosh(-z) - lc) / (2j * np.pi)
    np.testing.assert_allclose(d, np.round(d.real), atol=1e-12)


# ---------------------------------------------------------------------------
# C1: explicit Jacobians vs central finite differences of log psi
# ---------------------------------------------------------------------------
def _fd_check(net_from_flat, theta, x, O, n_params_checked=48, seed=0, h=1e-6):
    g = np.random.default_rng(seed)
    ks = g.choice(theta.size, size=min(n_params_checked, theta.size), replace=False)
    base = net_from_flat(theta).log_psi(x)
    for k in ks:
        for step in (h, 1j * h):  # holomorphy: real and imaginary steps agree
            tp = theta.copy(); tp[k] += step
            tm = theta.copy(); tm[k] -= step
            # log of a ratio to stay away from 2 pi i jumps
            lp = net_from_flat(tp).log_psi(x) - base
            lm = net_from_flat(tm).log_psi(x) - base
            lp = lp - 2j * np.pi * np.round(lp.imag / (2 * np.pi))
            lm = lm - 2j * np.pi * np.round(lm.imag / (2 * np.pi))
            fd = (lp - lm) / (2 * step)
            np.testing.assert_allclose(fd, O[:, k], rtol=2e-6, atol=2e-7 * (1 + np.abs(O[:, k]).max()))


def test_jacobian_rbm_finite_differences():
    net = workloads.rbm_network(N=8, M=12, config=7, sd=0.3)
    x = workloads.zero_magnetisation_samples(np.random.default_rng(1), 16, 8)
    O = net.jacobian(x)
    _fd_check(lambda t: networks.RBM.from_flat(t, 8, 12), net.flat(), x, O)
    assert net.block_sizes == [96, 12, 8]


def test_jacobian_ffnn_finite_differences():
    for readout in (False, True):
        net = workloads.ffnn_network([8, 10, 6], config=7, readout=readout)
        x = workloads.zero_magnetisation_samples(np.random.default_rng(2), 16, 8)
        O = net.jacobian(x)
        _fd_check(net.with_flat, net.flat(), x, O)


def test_jacobian_cnn_finite_differences():
    net = workloads.cnn_network(L=4, channels=3, layers=3, config=7)
    x = workloads.zero_magnetisation_samples(np.random.default_rng(3), 8, 16)
    O = net.jacobian(x)
    _fd_check(net.with_flat, net.flat(), x, O, n_params_checked=40)
    assert net.block_sizes == [3 * 9 + 3, 3 * 3 * 9 + 3, 3 * 3 * 9 + 3]


def test_config_block_sizes():
    assert workloads.rbm_network().block_sizes == [512, 32, 16]
    assert workloads.ffnn_network([64, 128, 128, 64], config=1, readout=True).block_sizes == [8320, 16512, 8256, 65]
    assert workloads.cnn_network(L=10).block_sizes == [160, 2320, 2320, 2320]
    assert workloads.ffnn_network([100, 400, 400], config=2).block_sizes == [40400, 160400]
    for N in workloads.CONFIG4_CHAINS:
        assert workloads.ffnn_network([N, 2 * N, N], config=4).block_sizes == [2 * N * N + 2 * N, 2 * N * N + N]


def test_zero_magnetisation_samples():
    x = workloads.zero_magnetisation_samples(np.random.default_rng(0), 500, 16)
    assert x.dtype == np.int8 and set(np.unique(x)) == {-1, 1}
    assert np.all(x.sum(axis=1) == 0)


# ---------------------------------------------------------------------------
# C2: covariance form vs the state-vector form of Eq. 2 on the whole Hilbert
# space; force vs the gradient of the exact energy of Eq. 1.
# ---------------------------------------------------------------------------
def _state_vector_qgt(psi_of_theta, theta, h=1e-6):
    psi = psi_of_theta(theta)
    dpsi = np.empty((psi.size, theta.size), dtype=np.complex128)
    for k in range(theta.size):
        tp = theta.copy(); tp[k] += h
        tm = theta.copy(); tm[k] -= h
        dpsi[:, k] = (psi_of_theta(tp) - psi_of_theta(tm)) / (2 * h)
    nrm = np.vdot(psi, psi).real
    a = dpsi.conj().T @ dpsi / nrm
    b = dpsi.conj().T @ psi / nrm
    return a - np.outer(b, b.conj()), psi


@pytest.mark.parametrize("family", ["rbm", "ffnn"])
def test_exact_qgt_state_vector_form(family):
    N = 8
    X = all_configs(N)
    if family == "rbm":
        net = workloads.rbm_network(N=N, M=16, config=7, sd=0.25)
        make = lambda t: networks.RBM.from_flat(t, N, 16)
    else:
        net = workloads.ffnn_network([N, 16, 8], config=7)
        make = net.with_flat
    theta = net.flat()
    S_exact, psi = _state_vector_qgt(lambda t: np.exp(make(t).log_psi(X)), theta)
    p = np.abs(psi) ** 2
    p /= p.sum()
    O = net.jacobian(X)
    dO = orc.centred_block(O, 0, O.shape[1], weights=p)
    S_orc = orc.qgt_block(dO, weights=p)
    scale = np.abs(S_exact).max()
    assert np.abs(S_orc - S_exact).max() <= 1e-8 * scale
    # each layer block of the full QGT is the block QGT of that layer (Eq. 3)
    offs = orc.block_offsets(net.block_sizes)
    for b in range(len(net.block_sizes)):
        lo, hi = offs[b], offs[b + 1]
        Sb = orc.qgt_block(orc.centred_block(O, lo, hi, weights=p), weights=p)
        assert np.abs(Sb - S_exact[lo:hi, lo:hi]).max() <= 1e-8 * scale


def test_force_is_gradient_of_exact_energy():
    """F_k = dE/d conj(theta_k) = (dE/dRe theta_k + i dE/dIm theta_k) / 2 for the
    Heisenberg chain energy of Eq. 1 (exact expectation over all 2^N states)."""
    N = 8
    X, H = heisenberg_matrix(N)
    net = workloads.rbm_network(N=N, M=8, config=7, sd=0.3)
    theta = net.flat()

    def energy(t):
        psi = np.exp(networks.RBM.from_flat(t, N, 8).log_psi(X))
        return (np.vdot(psi, H @ psi) / np.vdot(psi, psi)).real

    psi = np.exp(net.log_psi(X))
    p = np.abs(psi) ** 2
    p /= p.sum()
    e_loc = (H @ psi) / psi
    O = net.jacobian(X)
    dO = orc.centred_block(O, 0, O.shape[1], weights=p)
    F = orc.force_block(dO, orc.centred_energy(e_loc, weights=p), weights=p)
    h = 1e-6
    for k in np.random.default_rng(0).choice(theta.size, 30, replace=False):
        grad = []
        for step in (h, 1j * h):
            tp = theta.copy(); tp[k] += step
            tm = theta.copy(); tm[k] -= step
            grad.append((energy(tp) - energy(tm)) / (2 * h))
        fd = 0.5 * (grad[0] + 1j * grad[1])
        assert abs(F[k] - fd) <= 1e-7 * (1 + abs(fd)), (k, F[k], fd)


# ---------------------------------------------------------------------------
# C3 / C4: Woodbury and single-block identities
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small_ffnn():
    return workloads.small_ffnn(n_s=96, N=8, widths=(12, 6), readout=True, lam=1e-3)


def test_woodbury_parameter_vs_sample_space(small_ffnn):
    w = small_ffnn
    sizes = w.block_sizes
    rp = orc.block_sr(w.O, w.e_loc, sizes, w.lam, forms=["P"] * len(sizes))
    rs = orc.block_sr(w.O, w.e_loc, sizes, w.lam, forms=["S"] * len(sizes))
    assert orc.relative_error(rs.delta, rp.delta) <= 1e-10
    for e in orc.block_relative_errors(rs.delta, rp.delta, sizes):
        assert e <= 1e-10


def test_single_block_is_full_sr(small_ffnn):
    w = small_ffnn
    full = orc.full_sr(w.O, w.e_loc, w.lam)
    one = orc.block_sr(w.O, w.e_loc, [w.n_p], w.lam)
    np.testing.assert_array_equal(full.delta, one.delta)
    # directly: (S + lam I) delta = F with S the full covariance
    dO = w.O - w.O.mean(0)
    dE = w.e_loc - w.e_loc.mean()
    S = dO.conj().T @ dO / w.n_s
    F = dO.conj().T @ dE / w.n_s
    r = F - S @ full.delta - w.lam * full.delta
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(F)


def test_block_sr_equals_full_sr_when_qgt_is_block_diagonal():
    n_s = 64
    Hm = hadamard(n_s)
    g = np.random.default_rng(5)
    cols = g.permutation(np.arange(1, n_s))[:30]  # distinct, non-constant columns
    sizes = [7, 11, 12]
    c = (g.integers(-3, 4, 30) + 1j * g.integers(-3, 4, 30)) * 2.0 ** g.integers(-2, 3, 30)
    c[c == 0] = 1.0
    O = Hm[:, cols] * c + (g.normal(size=30) + 1j * g.normal(size=30))
    E = g.normal(size=n_s) + 1j * g.normal(size=n_s)
    blk = orc.block_sr(O, E, sizes, 1e-3)
    full = orc.full_sr(O, E, 1e-3)
    assert orc.relative_error(blk.delta, full.delta) <= 1e-12


# ---------------------------------------------------------------------------
# Invariants
# ---------------------------------------------------------------------------
def test_qgt_hermitian_psd(small_ffnn):
    w = small_ffnn
    offs = orc.block_offsets(w.block_sizes)
    for b in range(len(w.block_sizes)):
        S = orc.qgt_block(orc.centred_block(w.O, offs[b], offs[b + 1]))
        np.testing.assert_allclose(S, S.conj().T, atol=1e-14 * np.abs(S).max())
        assert np.all(np.diag(S).imag == 0) or np.abs(np.diag(S).imag).max() < 1e-15 * np.abs(S).max()
        assert np.linalg.eigvalsh(S).min() >= -1e-12 * np.abs(S).max()


def test_row_constant_shift_of_O_is_invisible(small_ffnn):
    w = small_ffnn
    g = np.random.default_rng(1)
    cvec = g.normal(size=w.n_p) + 1j * g.normal(size=w.n_p)
    a = orc.block_sr(w.O, w.e_loc, w.block_sizes, w.lam)
    b = orc.block_sr(w.O + cvec[None, :], w.e_loc, w.block_sizes, w.lam)
    assert orc.relative_error(b.delta, a.delta) <= 1e-9


def test_energy_shift_and_scale(small_ffnn):
    w = small_ffnn
    a = orc.block_sr(w.O, w.e_loc, w.block_sizes, w.lam)
    b = orc.block_sr(w.O, w.e_loc + (123.0 - 4.0j), w.block_sizes, w.lam)
    assert orc.relative_error(b.delta, a.delta) <= 1e-10
    c = orc.block_sr(w.O, (2.5 - 1.0j) * w.e_loc, w.block_sizes, w.lam)
    assert orc.relative_error(c.delta, (2.5 - 1.0j) * a.delta) <= 1e-10


def test_large_shift_gives_gradient_descent(small_ffnn):
    w = small_ffnn
    lam = 1e9
    r = orc.block_sr(w.O, w.e_loc, w.block_sizes, lam)
    assert orc.relative_error(lam * r.delta, r.force) <= 1e-6


def test_zero_magnetisation_null_directions():
    """With sum_i x_i = 0 for every sample, the RBM visible-bias Jacobian x has
    sum_i O_a[i] = 0 and each W row has sum_i O_W[j,i] = tanh(theta_j) sum_i x_i = 0;
    these are exact null directions of S, so delta has zero component on them."""
    w = workloads.config0(n_s=256)
    r = orc.block_sr(w.O, w.e_loc, w.block_sizes, w.lam)
    dW = r.delta[:512].reshape(32, 16)
    da = r.delta[544:]
    scale = np.abs(r.delta).max()
    assert np.abs(da.sum()) <= 1e-10 * scale * 16
    assert np.abs(dW.sum(axis=1)).max() <= 1e-10 * scale * 16


def test_sample_space_z_sums_to_zero(small_ffnn):
    w = small_ffnn
    offs = orc.block_offsets(w.block_sizes)
    b = int(np.argmax(w.block_sizes))
    z = orc.sample_space_z(w.O, w.e_loc, offs[b], offs[b + 1], w.lam)
    assert abs(z.sum()) <= 1e-10 * np.abs(z).sum()


def test_sample_permutation_invariance(small_ffnn):
    w = small_ffnn
    perm = np.random.default_rng(3).permutation(w.n_s)
    a = orc.block_sr(w.O, w.e_loc, w.block_sizes, w.lam)
    b = orc.block_sr(w.O[perm], w.e_loc[perm], w.block_sizes, w.lam)
    assert orc.relative_error(b.delta, a.delta) <= 1e-10


def test_residual_bound_small(small_ffnn):
    w = small_ffnn
    r = orc.block_sr(w.O, w.e_loc, w.block_sizes, w.lam)
    for rn, dn in orc.block_residual_norms(w.O, w.e_loc, w.block_sizes, w.lam, r.delta):
        assert rn <= 1e-12 * max(dn, 1e-300) * 1e3


def test_cholesky_comparator_matches(small_ffnn):
    w = small_ffnn
    a = orc.block_sr(w.O, w.e_loc, w.block_sizes, w.lam)
    b = orc.block_sr_cholesky(w.O, w.e_loc, w.block_sizes, w.lam)
    assert orc.relative_error(b, a.delta) <= 1e-10


@pytest.mark.parametrize("n_s,sizes,decades,lam", [
    (512, [64, 300, 512], 4.0, 1e-5),      # parameter form, column decay (condition numbers up to ~1e9)
    (256, [700, 40], 0.0, 1e-4),           # a sample-form block next to a parameter-form one
    (128, [1000], 2.0, 1e-4),              # sample form, n_b ~ 8 n_s (like the wide FFNN's blocks)
])
def test_cholesky_comparator_matches_definition(n_s, sizes, decades, lam):
    """The Cholesky form of the oracle (used at full size, where diagonalising
    is too slow) against its eigendecomposition form, block by block, within
    the difference two backward-stable FP64 solvers may show: a small multiple
    of kappa * 2^-52 per block."""
    w = workloads.random_blocks(n_s, sizes, config=21, instance=len(sizes), decades=decades, lam=lam,
                                o_dtype=np.complex64)
    a = orc.block_sr(w.O, w.e_loc, w.block_sizes, w.lam)
    b = orc.block_sr_cholesky(w.O, w.e_loc, w.block_sizes, w.lam)
    offs = orc.block_offsets(w.block_sizes)
    for k in range(len(sizes)):
        err = orc.relative_error(b[offs[k]:offs[k + 1]], a.delta[offs[k]:offs[k + 1]])
        assert a.n_cut[k] == 0
        assert err <= max(1e-13, 64 * a.kappa[k] * 2.0 ** -52), (k, err, a.kappa[k])


# ---------------------------------------------------------------------------
# H1/H2: Hadamard closed forms
# ---------------------------------------------------------------------------
def hadamard_pform_case(n_s=64, sizes=(5, 3, 8), lam=0.25, seed=0):
    """Delta O columns are power-of-two complex multiples of distinct non-constant
    Hadamard columns; the last column of each block is i times its first column.
    Returns O (with exact power-of-two offsets), E and the closed-form delta."""
    g = np.random.default_rng(seed)
    Hm = hadamard(n_s)
    n_p = sum(sizes)
    picks = g.permutation(np.arange(1, n_s))
    O = np.zeros((n_s, n_p), complex)
    E = 2.0 ** g.integers(-2, 3, n_s) * g.choice([-1, 1], n_s) + 1j * g.choice([-0.5, 0.5], n_s)
    dE = E - E.mean()
    delta = np.zeros(n_p, complex)
    col, p = 0, 0
    for nb in sizes:
        for k in range(nb):
            if k == nb - 1 and nb > 1:
                # paired column: i * (first column of this block)
                c = 1j * c0
                h = h0
            else:
                h = Hm[:, picks[p]]; p += 1
                c = (2.0 ** g.integers(-2, 2)) * g.choice([1, -1]) + 1j * (2.0 ** g.integers(-2, 2)) * g.choice([1, -1])
                if k == 0:
                    c0, h0 = c, h
            O[:, col + k] = c * h + (2.0 ** g.integers(-1, 3) - 1j * 2.0 ** g.integers(-1, 3))
        # closed form per block: unpaired columns are decoupled; the pair (0, nb-1)
        for k in range(nb):
            hk = O[:, col + k] - O[:, col + k].mean()
            e = hk.conj() @ dE / n_s  # = conj(c) (h . dE)/n_s
            a = np.vdot(hk, hk).real / n_s
            if nb > 1 and k in (0, nb - 1):
                delta[col + k] = e / (2 * a + lam)  # pair: F/(2a + lam) on each member
            else:
                delta[col + k] = e / (a + lam)
        col += nb
    return O, E, list(sizes), lam, delta


def test_hadamard_closed_form_pform():
    O, E, sizes, lam, expect = hadamard_pform_case()
    r = orc.block_sr(O, E, sizes, lam)
    assert orc.relative_error(r.delta, expect) <= 1e-14
    # the QGT of a paired block has the exact off-diagonal +i |c|^2 (conjugate on the first index)
    dO = orc.centred_block(O, 0, sizes[0])
    S = orc.qgt_block(dO)
    a = S[0, 0].real
    assert S[0, sizes[0] - 1] == 1j * a and S[sizes[0] - 1, 0] == -1j * a


def test_hadamard_centring_is_exact():
    O, E, sizes, lam, _ = hadamard_pform_case(seed=3)
    dO = orc.centred_block(O, 0, sum(sizes))
    # centred columns are +-c: every entry has the same modulus within a column
    assert np.all(np.abs(np.abs(dO) - np.abs(dO[0:1])) == 0)
    assert np.all(dO.sum(axis=0) == 0)


def test_hadamard_closed_form_sform():
    n_s, nb, lam = 16, 40, 0.5
    g = np.random.default_rng(11)
    Hm = hadamard(n_s)
    idx = g.integers(1, n_s, nb)  # repeated non-constant columns
    c = 2.0 ** g.integers(-2, 2, nb) * g.choice([1, -1], nb) + 1j * 2.0 ** g.integers(-2, 2, nb)
    O = Hm[:, idx] * c + 3.0
    E = g.normal(size=n_s) + 1j * g.normal(size=n_s)
    dE = E - E.mean()
    sig2 = np.zeros(n_s)
    np.add.at(sig2, idx, np.abs(c) ** 2)
    e = Hm.T @ dE / n_s
    expect = c.conj() * e[idx] / (sig2[idx] + lam)
    r = orc.block_sr(O, E, [nb], lam)
    assert r.forms == ["S"]
    assert orc.relative_error(r.delta, expect) <= 1e-13
    rp = orc.block_sr(O, E, [nb], lam, forms=["P"])
    assert orc.relative_error(rp.delta, expect) <= 1e-12


# ---------------------------------------------------------------------------
# Hand-derived golden fixtures
# ---------------------------------------------------------------------------
def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        d = json.load(f)
    O = np.array(d["O_re"], float) + 1j * np.array(d["O_im"], float)
    E = np.array(d["E_re"], float) + 1j * np.array(d["E_im"], float)
    delta = np.array(d["delta_re"]) + 1j * np.array(d["delta_im"])
    return O, E, d["block_sizes"], d["lambda"], delta


@pytest.mark.parametrize("name", ["tiny_pform.json", "tiny_sform.json"])
def test_golden_fixtures(name):
    O, E, sizes, lam, expect = load_golden(name)
    r = orc.block_sr(O, E, sizes, lam)
    np.testing.assert_allclose(r.delta, expect, rtol=1e-14, atol=1e-15)
    full = orc.full_sr(O, E, lam)
    np.testing.assert_allclose(full.delta, expect, rtol=1e-14, atol=1e-15)


def test_sample_space_with_large_energy_offset():
    """Shifting E by a constant leaves delta unchanged; in the sample-space form
    the uncentred mean would sit on the null vector 1 of T with weight E/lambda
    and cancel only to rounding, so the energy must be centred first."""
    w = workloads.random_blocks(48, [80], config=8, instance=2, lam=1e-3, e_mean=-1e7)
    rp = orc.block_sr(w.O, w.e_loc, w.block_sizes, w.lam, forms=["P"])
    rs = orc.block_sr(w.O, w.e_loc, w.block_sizes, w.lam, forms=["S"])
    assert orc.relative_error(rs.delta, rp.delta) <= 1e-9
