"""GPU parity of the VMC pieces (include/qgt_vmc.h) against the FP64 VMC
oracle (oracle/vmc.py), through the C ABI:

  * the Metropolis exchange sampler: with the same starting configurations,
    spin pairs and uniforms, every chain ends in the oracle's configuration
    with the oracle's number of accepted moves (the decisions are taken in
    FP64 on both sides; a tie within rounding would show as a mismatch);
  * the Heisenberg local energies of an RBM (periodic and open chains)
    within 1e-12 relative;
  * a whole VMC loop on the device (sampler, local energies, O on the
    device, block SR, parameter step) follows the oracle's loop: same
    samples and energies to 1e-9 over eight iterations, and the energy falls
    towards the exact ground-state energy.
"""
import sys

import numpy as np
import pytest

from gen import workloads
from oracle import jacobian as jac
from oracle import vmc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# M <= 256 takes the sampler's cached hidden fields, M = 300 the uncached
# ratio of every proposal
@pytest.mark.parametrize("N,M,n_chains,sweeps,sd", [(8, 8, 300, 6, 0.2), (16, 32, 257, 4, 0.05), (6, 70, 64, 5, 0.3),
                                                    (8, 300, 200, 3, 0.1)])
def test_metropolis_matches_oracle_chains(gpu_lib, N, M, n_chains, sweeps, sd):
    theta = workloads.rbm_network(N=N, M=M, config=11, sd=sd).flat()
    x0 = workloads.zero_magnetisation_samples(workloads.rng(11, workloads.P_SAMPLES), n_chains, N)
    pairs, u = workloads.mcmc_moves(11, 0, sweeps * N, n_chains, N)
    say(f"  gpu: rbm_metropolis N={N} M={M} chains={n_chains} steps={sweeps * N}")
    xd = dev(x0)
    acc = torch.zeros(n_chains, dtype=torch.int32, device="cuda")
    gpu_lib.rbm_metropolis(dev(theta), xd, M, dev(pairs), dev(u), acc)
    torch.cuda.synchronize()
    x_or, acc_or = vmc.metropolis_exchange(lambda xx: jac.rbm_log_psi(theta, N, M, xx), x0, pairs, u)
    assert np.array_equal(xd.cpu().numpy(), x_or)
    assert int(acc.sum().item()) == acc_or
    # exchange moves keep the magnetisation
    assert np.all(xd.cpu().numpy().sum(axis=1) == x0.sum(axis=1))


@pytest.mark.parametrize("N,M,periodic", [(16, 32, True), (8, 5, False), (64, 3, True), (3, 4, True)])
def test_local_energies_match_oracle(gpu_lib, N, M, periodic):
    theta = workloads.rbm_network(N=N, M=M, config=12, sd=0.3).flat()
    x = workloads.zero_magnetisation_samples(workloads.rng(12, workloads.P_SAMPLES), 333, N)
    say(f"  gpu: rbm_heisenberg_eloc N={N} M={M} periodic={periodic}")
    e = gpu_lib.rbm_heisenberg_eloc(dev(theta), dev(x), M, 1.0, periodic).cpu().numpy()
    ref = vmc.heisenberg_eloc(lambda xx: jac.rbm_log_psi(theta, N, M, xx), x, 1.0, periodic)
    np.testing.assert_allclose(e, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("full_qgt", [False, True])
def test_vmc_loop_follows_the_oracle(gpu_lib, full_qgt):
    """Block SR over the layer blocks W, b, a, and full-QGT SR (one block of
    all parameters, the same entry points with a one-block plan)."""
    qgt = gpu_lib
    N, M, n_s, sweeps, lam, eta, iters = 8, 8, 256, 8, 1e-3, 0.05, 8
    theta0 = workloads.rbm_network(N=N, M=M, config=10, sd=0.05).flat()
    x0 = workloads.zero_magnetisation_samples(workloads.rng(10, workloads.P_SAMPLES), n_s, N)
    th, xd = dev(theta0), dev(x0)
    n_p = M * N + M + N
    O = torch.empty((n_s, n_p), dtype=torch.complex128, device="cuda")
    delta = torch.empty(n_p, dtype=torch.complex128, device="cuda")
    sr = qgt.BlockSR([(n_s, [n_p] if full_qgt else [M * N, M, N], lam)], "c128", "fp64", 0)
    theta_or, x_or = theta0.copy(), x0.copy()
    energies = []
    for it in range(iters):
        pairs, u = workloads.mcmc_moves(10, it, sweeps * N, n_s, N)
        say(f"  gpu: vmc iteration {it} ({'full QGT' if full_qgt else 'block SR'})")
        qgt.rbm_metropolis(th, xd, M, dev(pairs), dev(u))
        e = qgt.rbm_heisenberg_eloc(th, xd, M)
        qgt.rbm_jacobian(th, xd, M, O=O)
        sr.form([O], [e])
        sr.solve([delta])
        qgt.sr_update(th, delta, eta)
        torch.cuda.synchronize()
        theta_or, x_or, e_or, _ = vmc.rbm_vmc_iteration(theta_or, N, M, x_or, pairs, u, lam, eta, full_qgt=full_qgt)
        assert np.array_equal(xd.cpu().numpy(), x_or), it
        e_gpu = complex(e.mean().item())
        assert abs(e_gpu - e_or) <= 1e-9 * abs(e_or), (it, e_gpu, e_or)
        np.testing.assert_allclose(th.cpu().numpy(), theta_or, rtol=1e-8, atol=1e-10)
        energies.append(e_gpu.real)
    assert not any(sr.status())
    E0 = vmc.ground_state(N)[0]
    # the energy falls (in these eight iterations by about 0.4 with block SR,
    # 0.08 with full-QGT SR, as the oracle's loop does) and stays variational
    assert energies[-1] < energies[0] - (0.05 if full_qgt else 0.2) and energies[-1] > E0 - 0.05, (energies, E0)
