"""Seeded synthetic workloads for the block-SR hot path.

The paper's experiments (Sec. 3: L=16 Heisenberg chain, J1-J2 square lattices)
need a trained Vision Transformer, a Monte Carlo sampler and a Hamiltonian, none
of which is part of the SR hot path.  The inputs here stand in for them: the
shapes (n_s samples x n_p parameters split into layer blocks), value
distributions (configurations in {-1,+1}^N with zero magnetisation, local
energies around the paper's energy scales) and network families match the
workloads described in the build's configuration list.

Every random number is drawn from numpy's PCG64 via
    numpy.random.default_rng([config, purpose, instance])
with purpose 0 params, 1 samples, 2 local energies, 3 block sizes, 4 O entries,
5 decay permutation, 6 Markov-chain moves.  Nothing here performs SR arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .networks import CNN, FFNN, RBM

P_PARAMS, P_SAMPLES, P_ELOC, P_BLOCKS, P_OENTRIES, P_DECAY, P_MCMC = range(7)


def rng(config: int, purpose: int, instance: int = 0) -> np.random.Generator:
    return np.random.default_rng([config, purpose, instance])


def zero_magnetisation_samples(g: np.random.Generator, n_s: int, N: int) -> np.ndarray:
    """n_s i.i.d. uniform configurations with N/2 up and N/2 down spins (int8)."""
    base = np.concatenate([np.ones(N // 2, np.int8), -np.ones(N - N // 2, np.int8)])
    keys = g.random((n_s, N))
    return base[np.argsort(keys, axis=1)]


def local_energies(g: np.random.Generator, n_s: int, mean_re: float, sd_re: float, sd_im: float) -> np.ndarray:
    re = g.normal(mean_re, sd_re, n_s)
    im = g.normal(0.0, sd_im, n_s)
    return (re + 1j * im).astype(np.complex128)


def complex_normal(g: np.random.Generator, shape, var_total: float) -> np.ndarray:
    """Complex normal with E|z|^2 = var_total (each part variance var_total / 2)."""
    sd = np.sqrt(var_total / 2.0)
    return g.normal(0.0, sd, shape) + 1j * g.normal(0.0, sd, shape)


def _round_params(arr, dtype):
    return np.asarray(arr).astype(dtype).astype(np.complex128)


@dataclass
class Workload:
    """One SR-step problem: O (n_s x n_p), E_loc (n_s), block sizes, lambda."""
    name: str
    O: np.ndarray
    e_loc: np.ndarray
    block_sizes: list
    lam: float
    meta: dict = field(default_factory=dict)

    @property
    def n_s(self):
        return self.O.shape[0]

    @property
    def n_p(self):
        return self.O.shape[1]


# ---------------------------------------------------------------------------
# Networks with the initialisations of each configuration
# ---------------------------------------------------------------------------
def rbm_network(N=16, M=32, config=0, instance=0, sd=0.01, dtype=np.complex128):
    g = rng(config, P_PARAMS, instance)
    a = g.normal(0, sd, N) + 1j * g.normal(0, sd, N)
    b = g.normal(0, sd, M) + 1j * g.normal(0, sd, M)
    W = g.normal(0, sd, (M, N)) + 1j * g.normal(0, sd, (M, N))
    return RBM(_round_params(a, dtype), _round_params(b, dtype), _round_params(W, dtype))


def ffnn_network(widths, config, instance=0, readout=False, dtype=np.complex128):
    """widths = [N_in, w1, ..., wL]; params N(0, 1/fan_in) complex."""
    g = rng(config, P_PARAMS, instance)
    Ws, bs = [], []
    for fan_in, fan_out in zip(widths[:-1], widths[1:]):
        Ws.append(_round_params(complex_normal(g, (fan_out, fan_in), 1.0 / fan_in), dtype))
        bs.append(_round_params(complex_normal(g, fan_out, 1.0 / fan_in), dtype))
    ro = None
    if readout:
        fan_in = widths[-1]
        v = _round_params(complex_normal(g, fan_in, 1.0 / fan_in), dtype)
        c = _round_params(complex_normal(g, 1, 1.0 / fan_in), dtype)[0]
        ro = (v, c)
    return FFNN(Ws, bs, ro)


def cnn_network(L=10, channels=16, layers=4, config=2, instance=0, dtype=np.complex128):
    g = rng(config, P_PARAMS, instance)
    Ks, bs = [], []
    cin = 1
    for _ in range(layers):
        fan_in = cin * 9
        Ks.append(_round_params(complex_normal(g, (channels, cin, 3, 3), 1.0 / fan_in), dtype))
        bs.append(_round_params(complex_normal(g, channels, 1.0 / fan_in), dtype))
        cin = channels
    return CNN(Ks, bs, L)


def _jacobian_workload(name, net, x, e_loc, lam, o_dtype, config, extra=None):
    # every entry is formed in complex128 and rounded once on assignment into
    # the output type (the same values as forming in complex128 and casting)
    O = net.jacobian(x, out_dtype=o_dtype)
    meta = dict(config=config, n_spins=x.shape[1])
    if extra:
        meta.update(extra)
    return Workload(name, O, e_loc, list(net.block_sizes), lam, meta)


# ---------------------------------------------------------------------------
# The five workloads and reduced-size variants of them
# ---------------------------------------------------------------------------
def config0(n_s=1024, N=16, M=32, o_dtype=np.complex128):
    """Complex RBM, N=16 spins, M=32 hidden units; blocks W 512, b 32, a 16."""
    net = rbm_network(N, M, config=0)
    x = zero_magnetisation_samples(rng(0, P_SAMPLES), n_s, N)
    e = local_energies(rng(0, P_ELOC), n_s, -7.0, 1.0, 0.1)
    w = _jacobian_workload("rbm_n16_m32", net, x, e, 1e-4, o_dtype, 0)
    w.meta["net"] = net
    w.meta["x"] = x
    return w


def config1(n_s=4096, N=64, widths=(128, 128, 64), o_dtype=np.complex64):
    """FFNN 64-128-128-64 with logcosh and a dense 64->1 readout (4 blocks)."""
    dt = np.complex64 if o_dtype == np.complex64 else np.complex128
    net = ffnn_network([N, *widths], config=1, readout=True, dtype=dt)
    x = zero_magnetisation_samples(rng(1, P_SAMPLES), n_s, N)
    e = local_energies(rng(1, P_ELOC), n_s, -7.0, 1.0, 0.1)
    return _jacobian_workload("ffnn_chain_n64", net, x, e, 1e-3, o_dtype, 1)


def config2_cnn(n_s=8192, L=10, o_dtype=np.complex64):
    net = cnn_network(L=L, config=2, dtype=np.complex64)
    x = zero_magnetisation_samples(rng(2, P_SAMPLES), n_s, L * L)
    e = local_energies(rng(2, P_ELOC), n_s, -50.0, 3.0, 0.5)
    return _jacobian_workload("cnn_10x10", net, x, e, 1e-4, o_dtype, 2)


def config2_ffnn(n_s=8192, N=100, width=400, o_dtype=np.complex64):
    net = ffnn_network([N, width, width], config=2, instance=1, dtype=np.complex64)
    x = zero_magnetisation_samples(rng(2, P_SAMPLES, 1), n_s, N)
    e = local_energies(rng(2, P_ELOC, 1), n_s, -50.0, 3.0, 0.5)
    return _jacobian_workload("ffnn_10x10_w400", net, x, e, 1e-4, o_dtype, 2)


def config3_block_sizes(n_blocks=64, lo=64, hi=8192, seed_instance=0):
    g = rng(3, P_BLOCKS, seed_instance)
    return [int(v) for v in np.rint(np.exp(g.uniform(np.log(lo), np.log(hi), n_blocks)))]


def config3(n_s=8192, n_blocks=64, lo=64, hi=8192, decades=4.0, seed_instance=0, o_dtype=np.complex64):
    """O drawn directly: complex standard normal entries; the columns of each block
    get a seeded geometric decay r^k (r = 10^(-decades/(n_b-1))) in a seeded order,
    so that the block condition numbers reach ~10^(2*decades)."""
    sizes = config3_block_sizes(n_blocks, lo, hi, seed_instance)
    n_p = sum(sizes)
    O = np.empty((n_s, n_p), dtype=o_dtype)
    gO = rng(3, P_OENTRIES, seed_instance)
    gD = rng(3, P_DECAY, seed_instance)
    off = 0
    for nb in sizes:
        blk = complex_normal(gO, (n_s, nb), 1.0)
        r = 10.0 ** (-decades / max(nb - 1, 1))
        scale = np.empty(nb)
        scale[gD.permutation(nb)] = r ** np.arange(nb)
        O[:, off: off + nb] = (blk * scale).astype(o_dtype)
        off += nb
    e = local_energies(rng(3, P_ELOC, seed_instance), n_s, -7.0, 1.0, 0.1)
    return Workload("random_decay_blocks", O, e, sizes, 1e-5, dict(config=3))


CONFIG4_CHAINS = (16, 24, 32, 48, 64)
CONFIG4_NS = (1024, 2048, 4096)


def config4_instance(i, o_dtype=np.complex64, n_s_override=None):
    """Instance i of the 32-instance stream: FFNN N -> 2N -> N with sum pooling."""
    g = rng(4, P_BLOCKS, i)
    N = int(g.choice(CONFIG4_CHAINS))
    n_s = int(g.choice(CONFIG4_NS)) if n_s_override is None else n_s_override
    net = ffnn_network([N, 2 * N, N], config=4, instance=i, dtype=np.complex64)
    x = zero_magnetisation_samples(rng(4, P_SAMPLES, i), n_s, N)
    e = local_energies(rng(4, P_ELOC, i), n_s, -7.0, 1.0, 0.1)
    return _jacobian_workload(f"ffnn_chain_n{N}", net, x, e, 1e-4, o_dtype, 4, dict(instance=i))


def small_ffnn(n_s, N, widths, config=9, instance=0, readout=False, o_dtype=np.complex128, lam=1e-3):
    """Reduced-size FFNN workload for parity tests (several tiles, ragged tails)."""
    net = ffnn_network([N, *widths], config=config, instance=instance, readout=readout,
                       dtype=np.complex128 if o_dtype == np.complex128 else np.complex64)
    x = zero_magnetisation_samples(rng(config, P_SAMPLES, instance), n_s, N)
    e = local_energies(rng(config, P_ELOC, instance), n_s, -7.0, 1.0, 0.1)
    return _jacobian_workload(f"ffnn_small_n{N}", net, x, e, lam, o_dtype, config)


def random_blocks(n_s, block_sizes, config=8, instance=0, decades=0.0, o_dtype=np.complex128, lam=1e-4,
                  e_mean=-7.0):
    """Directly drawn O with optional per-block column decay (reduced config 3)."""
    n_p = sum(block_sizes)
    gO = rng(config, P_OENTRIES, instance)
    gD = rng(config, P_DECAY, instance)
    O = np.empty((n_s, n_p), dtype=o_dtype)
    off = 0
    for nb in block_sizes:
        blk = complex_normal(gO, (n_s, nb), 1.0)
        if decades > 0:
            r = 10.0 ** (-decades / max(nb - 1, 1))
            scale = np.empty(nb)
            scale[gD.permutation(nb)] = r ** np.arange(nb)
            blk = blk * scale
        O[:, off: off + nb] = blk.astype(o_dtype)
        off += nb
    e = local_energies(rng(config, P_ELOC, instance), n_s, e_mean, 1.0, 0.1)
    return Workload("random_blocks", O, e, list(block_sizes), lam, dict(config=config))


def mcmc_moves(config: int, iteration: int, n_steps: int, n_chains: int, N: int):
    """Random inputs of n_steps Metropolis exchange moves of n_chains chains:
    the spin pairs (n_steps x n_chains x 2, int32, each index uniform in
    [0, N)) and the acceptance uniforms (n_steps x n_chains, float64 in
    [0, 1))."""
    g = rng(config, P_MCMC, iteration)
    pairs = g.integers(0, N, size=(n_steps, n_chains, 2), dtype=np.int32)
    u = g.random((n_steps, n_chains))
    return pairs, u
