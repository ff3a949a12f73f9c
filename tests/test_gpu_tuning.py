"""GPU checks of the tuning: the autotuner writes a cache the planner then
uses, and every tuning choice (Gram tile shape, split, patch order, Cholesky
chunk, either way of launching the Cholesky) keeps block indexing bit-exact
and delta within tolerance."""
import json
import sys

import numpy as np
import pytest

from gen import workloads
from oracle import block_sr as orc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_autotune_writes_a_cache_the_planner_uses(gpu_lib, tmp_path, monkeypatch):
    w = workloads.small_ffnn(n_s=600, N=8, widths=(70, 33), readout=True, o_dtype=np.complex64, lam=1e-3)
    probs = [(w.n_s, w.block_sizes, w.lam)]
    path = tmp_path / "tune.json"
    say(f"case: autotune {w.block_sizes} at n_s={w.n_s}")
    n = gpu_lib.autotune(probs, "c64", "bf16", str(path), reps=1)
    text = path.read_text()
    say(text)
    data = json.loads(text)
    plans = {k: t for k, t in data["entries"].items() if "cholesky" in t}
    # one entry for the set's Cholesky launch mode
    assert len(plans) == 1
    (pkey, pt), = plans.items()
    assert pkey.startswith("gfx950/plan/") and pt["cholesky"] in (1, 2)
    assert pt["persistent_ms"] > 0 and pt["host_steps_ms"] > 0
    # host steps only where measured faster (by more than the 1% margin)
    assert (pt["cholesky"] == 1) == (pt["host_steps_ms"] < 0.99 * pt["persistent_ms"])
    # one entry per block shape class, and the same choice again inside the
    # set's class
    classes = {k: t for k, t in data["entries"].items() if "gram_tile" in t and not k.startswith("gfx950/plan/")}
    inside = {k: t for k, t in data["entries"].items() if "gram_tile" in t and k.startswith(pkey + "/")}
    assert n == len(classes) == len(inside) >= 2
    fields = ("gram_tile", "gram_items", "chol_chunk", "gram_patch")
    for key, t in classes.items():
        assert key.startswith("gfx950/bf16/")
        assert t["gram_tile"] in (1, 2, 3) and 1 <= t["chol_chunk"] <= 16 and t["form_ms"] > 0 and t["step_ms"] > 0
        u = inside[pkey + "/" + key[len("gfx950/"):]]
        assert all(u[f] == t[f] for f in fields)
    # a second run merges (same classes: the same number of entries)
    assert gpu_lib.autotune(probs, "c64", "bf16", str(path), reps=1) == n
    assert len(json.loads(path.read_text())["entries"]) == 2 * n + 1
    monkeypatch.setenv("QGT_TUNE_CACHE", str(path))
    sr = gpu_lib.BlockSR(probs, "c64", "bf16", 4, rtol=1e-7)
    src = [sr.block_tuning(g)["source"] for g in range(sr.num_blocks)]
    assert src.count("plan-cache") >= 2, src
    mode = sr.cholesky_mode()
    say(f"  Cholesky launch from the cache: {mode}")
    assert mode["source"] == "cache" and mode["mode"] in ("persistent", "host-steps")
    O = torch.from_numpy(w.O).cuda()
    e = torch.from_numpy(w.e_loc).cuda()
    d = sr([O], [e])[0].cpu().numpy()
    assert not any(sr.status())
    ref = orc.block_sr(w.O, w.e_loc, w.block_sizes, w.lam).delta
    err = max(orc.block_relative_errors(d, ref, w.block_sizes))
    say(f"  tuned plan: max block rel err {err:.2e}")
    assert err <= 1e-5


TUNINGS = [{"gram_tile": 1}, {"gram_tile": 2}, {"gram_tile": 3}, {"gram_tile": 3, "gram_patch": 16},
           {"gram_tile": 1, "gram_items": 1024, "gram_patch": 2},
           {"gram_patch": 8, "chol_chunk": 1}, {"chol_chunk": 3}, {"chol_chunk": 8}, {"chol_chunk": 16}]


@pytest.mark.parametrize("cholesky", ["host-steps", "persistent"])
@pytest.mark.parametrize("tuning", TUNINGS)
def test_every_tuning_keeps_block_indexing_exact(gpu_lib, tuning, cholesky):
    """Power-of-two multiples of Hadamard columns: every Gram entry is exact in
    BF16, so under any tuning the shifted Gram equals the closed form bit for
    bit (block offsets, tiles, splits and patch orders all exercised; the
    900-column block takes the 256x128 tiles when asked), and delta meets the
    closed form."""
    from tests.test_oracle_pins import hadamard_pform_case
    O, E, sizes, lam, expect = hadamard_pform_case(n_s=1024, sizes=(900, 70, 9))
    w = workloads.Workload("hadamard", O, E, list(sizes), lam)
    offs = orc.block_offsets(w.block_sizes)
    tun = [dict(tuning) for _ in sizes]
    for g, nb in enumerate(sizes):   # the wide tiles only where the block can take them
        if tun[g].get("gram_tile") == 2 and nb < 897:
            tun[g]["gram_tile"] = 1
    say(f"case: Hadamard exact Gram under tuning {tuning}, {cholesky}")
    Od = torch.from_numpy(O.astype(np.complex64)).cuda()
    e = torch.from_numpy(E).cuda()
    sr = gpu_lib.BlockSR([(w.n_s, w.block_sizes, w.lam)], "c64", "bf16", 2, tuning=tun, cholesky=cholesky)
    assert [sr.block_tuning(g)["source"] for g in range(3)] == ["caller"] * 3
    delta = sr([Od], [e])[0].cpu().numpy()
    assert not any(sr.status())
    sr.form([Od], [e])
    torch.cuda.synchronize()
    for g in range(len(sizes)):
        dO = orc.centred_block(O, offs[g], offs[g + 1])
        A = orc.qgt_block(dO) + lam * np.eye(sizes[g])
        G = sr.block_matrix(g)
        low = np.tril_indices(sizes[g])
        np.testing.assert_array_equal(G[low], A[low])
    assert orc.relative_error(delta, expect) <= 1e-12
