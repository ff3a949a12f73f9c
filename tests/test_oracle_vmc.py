"""Pins of the VMC oracle (oracle/vmc.py): the Heisenberg local energy, the
Metropolis exchange sampler and the exact ground-state energy, against facts
fixed by the paper and by mathematics:

  * exact ground-state energies: the two-site singlet (-3/4), the four-site
    ring (-2), and the sixteen-site ring of the paper's benchmark, whose
    energy in Pauli units (4 E0) the paper tabulates as -28.57 (Sec. 3,
    Tab. 2);
  * zero variance: the local energy of the exact ground state equals E0 on
    every configuration;
  * the mean local energy under the exact |psi|^2 of an RBM equals
    <psi|H|psi> / <psi|psi> from the sparse Hamiltonian;
  * the sampler's empirical distribution matches |psi|^2 (chi-square);
  * the oracle's whole VMC loop brings the energy of the 8-site ring to
    within 2% of the exact value;
  * planted mistakes (a missing factor 1/2 on the exchange term, acceptance
    by |ratio| instead of |ratio|^2, the parameter step taken with the wrong
    sign) are caught.
"""
import numpy as np
import pytest

from gen import workloads
from oracle import jacobian as jac
from oracle import vmc


def _table_log_psi(basis, psi):
    """log psi on the basis configurations, from a state vector."""
    idx = {b.tobytes(): r for r, b in enumerate(basis)}
    lp = np.log(psi.astype(np.complex128))

    def f(x):
        return np.array([lp[idx[np.asarray(r, dtype=np.int8).tobytes()]] for r in x])
    return f


def test_exact_energies():
    assert abs(vmc.ground_state(2, pbc=False)[0] + 0.75) < 1e-12
    assert abs(vmc.ground_state(4)[0] + 2.0) < 1e-12
    e16 = vmc.ground_state(16)[0]
    assert abs(4 * e16 - (-28.57)) < 0.005


def test_zero_variance_of_the_ground_state():
    E0, psi0, basis = vmc.ground_state(8)
    e = vmc.heisenberg_eloc(_table_log_psi(basis, psi0), basis)
    np.testing.assert_allclose(e, E0, atol=1e-9)


def _rbm_state(N, M, sd=0.3, seed=11):
    net = workloads.rbm_network(N=N, M=M, config=7, instance=seed, sd=sd)
    return net.flat()


def test_mean_local_energy_is_the_variational_energy():
    N, M = 8, 6
    theta = _rbm_state(N, M)
    H, basis = vmc.heisenberg_matrix_sz0(N)
    lp = jac.rbm_log_psi(theta, N, M, basis)
    psi = np.exp(lp)
    p = np.abs(psi) ** 2
    p /= p.sum()
    e = vmc.heisenberg_eloc(lambda x: jac.rbm_log_psi(theta, N, M, x), basis)
    exact = np.vdot(psi, H @ psi) / np.vdot(psi, psi)
    assert abs(np.sum(p * e) - exact) < 1e-12 * abs(exact)


def _chi_square(theta, N, M, n_chains=1500, sweeps=8, seed=3, accept_power=2.0):
    x0 = workloads.zero_magnetisation_samples(np.random.default_rng(seed), n_chains, N)
    pairs, u = workloads.mcmc_moves(7, seed, sweeps * N, n_chains, N)
    log_psi = lambda xx: jac.rbm_log_psi(theta, N, M, xx)
    if accept_power == 2.0:
        x, _ = vmc.metropolis_exchange(log_psi, x0, pairs, u)
    else:  # a planted mistake: acceptance by |ratio|
        x = x0.copy()
        for s in range(u.shape[0]):
            for c in range(n_chains):
                i, j = pairs[s, c]
                if x[c, i] == x[c, j]:
                    continue
                xp = x[c].copy(); xp[i], xp[j] = xp[j], xp[i]
                d = log_psi(xp[None])[0] - log_psi(x[c][None])[0]
                if u[s, c] < np.exp(accept_power * d.real):
                    x[c] = xp
    _, basis = vmc.heisenberg_matrix_sz0(N)
    p = np.abs(np.exp(jac.rbm_log_psi(theta, N, M, basis))) ** 2
    p /= p.sum()
    idx = {b.tobytes(): r for r, b in enumerate(basis)}
    counts = np.zeros(len(basis))
    for r in x:
        counts[idx[r.tobytes()]] += 1
    expected = p * n_chains
    return float(np.sum((counts - expected) ** 2 / expected)), len(basis) - 1


def test_sampler_distribution():
    theta = _rbm_state(6, 4, sd=0.2, seed=5)
    chi2, dof = _chi_square(theta, 6, 4)
    # mean dof, sd sqrt(2 dof): a bound five sd above the mean
    assert chi2 < dof + 5 * np.sqrt(2 * dof), (chi2, dof)


def test_planted_acceptance_by_modulus_is_caught():
    theta = _rbm_state(6, 4, sd=0.2, seed=5)
    chi2, dof = _chi_square(theta, 6, 4, accept_power=1.0)
    assert chi2 > dof + 5 * np.sqrt(2 * dof), (chi2, dof)


def test_planted_missing_half_is_caught(monkeypatch):
    E0, psi0, basis = vmc.ground_state(6)
    orig = vmc.heisenberg_eloc

    def wrong(log_psi, x, J=1.0, pbc=True):
        x = np.asarray(x, dtype=np.int8)
        lp = log_psi(x)
        e = np.zeros(len(x), dtype=np.complex128)
        for i, j in vmc.bonds(x.shape[1], pbc):
            e += J * 0.25 * x[:, i].astype(float) * x[:, j]
            flip = x[:, i] != x[:, j]
            xs = x[flip].copy(); xs[:, [i, j]] = xs[:, [j, i]]
            e[flip] += J * np.exp(log_psi(xs) - lp[flip])
        return e
    e = wrong(_table_log_psi(basis, psi0), basis)
    assert np.abs(e - E0).max() > 1e-3
    e = orig(_table_log_psi(basis, psi0), basis)
    assert np.abs(e - E0).max() < 1e-9


@pytest.mark.parametrize("full_qgt", [False, True])
def test_oracle_vmc_loop_reaches_the_ground_state_energy(full_qgt):
    """Thirty iterations of the oracle's VMC loop (RBM N=8 M=8, 256 chains,
    eta = 0.05) bring the mean local energy of the 8-site ring to within 2% of
    the exact ground-state energy from above; a wrong sign anywhere in the SR
    update or the force would drive the energy up instead."""
    N, M, n_s, sweeps = 8, 8, 256, 8
    E0 = vmc.ground_state(N)[0]
    theta = workloads.rbm_network(N=N, M=M, config=10, sd=0.05).flat()
    x = workloads.zero_magnetisation_samples(workloads.rng(10, workloads.P_SAMPLES), n_s, N)
    energies = []
    for it in range(30):
        pairs, u = workloads.mcmc_moves(10, it, sweeps * N, n_s, N)
        theta, x, e, _ = vmc.rbm_vmc_iteration(theta, N, M, x, pairs, u, lam=1e-3, eta=0.05,
                                                  full_qgt=full_qgt)
        energies.append(e.real)
    assert energies[0] > 0 > energies[-1]
    # variational bound (within the sampling noise) for both; in these thirty
    # iterations block SR gets within 2% of E0, full-QGT SR only to about 60%
    assert E0 - 0.05 < energies[-1], (energies[-5:], E0)
    if not full_qgt:
        assert energies[-1] < E0 * 0.98, (energies[-5:], E0)


def test_planted_update_sign_is_caught():
    """theta <- theta + eta delta (the wrong sign) raises the energy."""
    N, M, n_s, sweeps = 8, 8, 256, 8
    theta = workloads.rbm_network(N=N, M=M, config=10, sd=0.05).flat()
    x = workloads.zero_magnetisation_samples(workloads.rng(10, workloads.P_SAMPLES), n_s, N)
    energies = []
    for it in range(10):
        pairs, u = workloads.mcmc_moves(10, it, sweeps * N, n_s, N)
        new_theta, x, e, delta = vmc.rbm_vmc_iteration(theta, N, M, x, pairs, u, lam=1e-3, eta=0.05)
        theta = new_theta + 2 * 0.05 * delta   # undo the step and take it the other way
        energies.append(e.real)
    assert energies[-1] > energies[0]
