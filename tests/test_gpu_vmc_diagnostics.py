"""Block-layer against full-QGT SR on states the device VMC loop reaches
(paper, Sec. 3, Heisenberg chain paragraph, Tab. 1 and Tab. 2), for the
complex RBM N=16 M=32 on the 16-site periodic Heisenberg ring.

The device loop (Metropolis exchange moves, local energies, O and SR, all HIP)
runs block SR over the layer blocks (W, b, a) and full-QGT SR from the same
parameters, chains and moves.  At each final state the oracle computes what
Tab. 1 and Tab. 2 report: the Eq. 4 diagnostics of the inverse of the shifted
block-layer QGT and of the shifted full sampled QGT against the inverse of the
shifted exact QGT (over the zero-magnetisation sector, Born weights), the
energy, the variance of the local energy and the infidelity to the exact
ground state.  The device's Eq. 4 (a) and (b) (from its Cholesky factors) must
match the oracle's for both the block plan and the one-block (full) plan.

The table is printed; the readings behind it (shift on both inverses, Pearson
correlation of the sorted spectra) are those of oracle/diagnostics.py."""
import sys

import numpy as np
import pytest

from gen import workloads as W
from oracle import diagnostics as dg
from oracle import jacobian as jac
from oracle import vmc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N, M, N_S, SWEEPS = 16, 32, 1024, 10
ITERS, ETA, LAM = 600, 0.02, 1e-4


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def device_vmc(qgt, full_qgt):
    """ITERS device VMC iterations; returns (theta, chains resampled once more
    under the final theta, per-iteration mean energies, final local energies)."""
    n_p = M * N + M + N
    theta = torch.from_numpy(W.rbm_network(N=N, M=M, config=0).flat()).cuda()
    x = torch.from_numpy(W.zero_magnetisation_samples(W.rng(0, W.P_SAMPLES), N_S, N)).cuda()
    O = torch.empty((N_S, n_p), dtype=torch.complex128, device="cuda")
    ws = torch.empty(qgt.rbm_jacobian_workspace_bytes(N, M, N_S), dtype=torch.uint8, device="cuda")
    delta = torch.empty(n_p, dtype=torch.complex128, device="cuda")
    e = torch.empty(N_S, dtype=torch.complex128, device="cuda")
    sr = qgt.BlockSR([(N_S, [n_p] if full_qgt else [M * N, M, N], LAM)], "c128", "fp64", 0)
    energies = []
    for it in range(ITERS + 1):
        p, u = W.mcmc_moves(0, it, SWEEPS * N, N_S, N)
        qgt.rbm_metropolis(theta, x, M, torch.from_numpy(p).cuda(), torch.from_numpy(u).cuda())
        qgt.rbm_heisenberg_eloc(theta, x, M, e_loc=e)
        if it == ITERS:
            break
        qgt.rbm_jacobian(theta, x, M, O=O, workspace=ws)
        sr.form([O], [e])
        sr.solve([delta])
        qgt.sr_update(theta, delta, ETA)
        energies.append(e.mean().real)
    assert not any(sr.status())
    return (theta.cpu().numpy(), x.cpu().numpy(), torch.stack(energies).cpu().numpy(), e.cpu().numpy())


def device_diagnostics(qgt, O, sizes, B):
    """Eq. 4 (a), (b) of the plan's inverse from its Cholesky factors on the device."""
    sr = qgt.BlockSR([(O.shape[0], sizes, LAM)], "c128", "fp64", 0)
    sr([torch.from_numpy(O).cuda()], [torch.zeros(O.shape[0], dtype=torch.complex128, device="cuda")])
    out = sr.inverse_diagnostics(torch.from_numpy(B).cuda())
    sr.close()
    return out


@pytest.fixture(scope="module")
def ground():
    return vmc.ground_state(N)


@pytest.mark.parametrize("trained_with", ["block", "full"])
def test_eq4_and_tab2_on_vmc_states(gpu_lib, ground, trained_with):
    E0, psi0, basis = ground
    say(f"case: RBM N={N} M={M} Heisenberg ring, {ITERS} device VMC iterations with {trained_with} SR, "
        f"eta={ETA}, lambda={LAM}, n_s={N_S}")
    theta, x, energies, e_last = device_vmc(gpu_lib, trained_with == "full")
    assert np.all(np.isfinite(energies))
    # the state: amplitudes on the sector, Born weights, infidelity to psi0
    lp = jac.rbm_log_psi(theta, N, M, basis)
    amp = np.exp(lp - lp.real.max())
    p = np.abs(amp) ** 2
    p /= p.sum()
    infid = 1.0 - abs(np.vdot(psi0, amp)) ** 2 / (np.vdot(amp, amp).real * np.vdot(psi0, psi0).real)
    e_mean = float(energies[-50:].mean())
    var = float(np.mean(np.abs(e_last - e_last.mean()) ** 2))
    # Eq. 4 of the sampled block and full inverses against the exact inverse
    O_s = jac.rbm_jacobian(theta, N, M, x)
    O_all = jac.rbm_jacobian(theta, N, M, basis)
    sizes = [M * N, M, N]
    res = dg.compare_block_full_exact(O_s, O_all, p, sizes, LAM)
    say(f"  energy (mean of the last 50) {e_mean:.5f} vs exact {E0:.5f} (rel err {abs(e_mean - E0) / abs(E0):.2e}), "
        f"variance {var:.4f}, infidelity {infid:.3e}")
    say(f"  {'Eq. 4 metric':32s} {'block vs exact':>16s} {'full vs exact':>16s}")
    for k, name in [("frobenius_overlap", "(a) Frobenius overlap"),
                    ("frobenius_relative_error", "(b) Frobenius relative error"),
                    ("condition_number", "(c) condition number"),
                    ("spectral_correlation", "(d) spectral correlation")]:
        say(f"  {name:32s} {res['block'][k]:16.6g} {res['full'][k]:16.6g}")
    say(f"  condition number of the exact inverse {res['exact_condition_number']:.6g}")
    for which in ("block", "full"):
        d = res[which]
        assert 0.0 < d["frobenius_overlap"] <= 1.0 + 1e-12
        assert d["frobenius_relative_error"] >= 0.0
        assert d["condition_number"] >= 1.0
        assert -1.0 <= d["spectral_correlation"] <= 1.0 + 1e-12
    assert 0.0 <= infid <= 1.0
    # the device's Eq. 4 (a), (b) for both plans, from their Cholesky factors
    B = dg.shifted_inverse(dg.qgt(O_all, weights=p), LAM)
    for which, plan_sizes in (("block", sizes), ("full", [sum(sizes)])):
        got = device_diagnostics(gpu_lib, O_s, plan_sizes, B)
        say(f"  device {which}: F={got['frobenius_overlap']:.9f} eps_F={got['frobenius_relative_error']:.9f}")
        assert got["frobenius_overlap"] == pytest.approx(res[which]["frobenius_overlap"], rel=1e-8)
        assert got["frobenius_relative_error"] == pytest.approx(res[which]["frobenius_relative_error"], rel=1e-8)
