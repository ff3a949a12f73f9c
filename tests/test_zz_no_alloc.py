"""qgt_block_form_static: the form step in the library's static per-device
workspace, for callers that cannot allocate device memory.  Two plans run one
after the other through it (the second smaller, so it finds the first one's
data in the shared array) and must give, bit for bit, the delta of the same
plan run through qgt_block_form with a caller workspace, and meet the oracle.
A plan whose workspace exceeds the static array is refused before any launch."""
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


def run(qgt, w, dt, gram, refine, static):
    O = torch.from_numpy(np.ascontiguousarray(w.O)).cuda()
    e = torch.from_numpy(w.e_loc).cuda()
    sr = qgt.BlockSR([(w.n_s, w.block_sizes, w.lam)], dt, gram, refine, rtol=0.0)
    d = torch.empty(w.n_p, dtype=torch.complex128, device="cuda")
    if static:
        sr.form_static([O], [e])
    else:
        sr.form([O], [e])
    sr.solve([d])
    torch.cuda.synchronize()
    st = sr.status()
    sr.close()
    return d.cpu().numpy(), st


def test_static_workspace_matches_caller_workspace(gpu_lib):
    big = workloads.small_ffnn(n_s=600, N=8, widths=(70, 33), readout=True, o_dtype=np.complex64, lam=1e-3)
    small = workloads.config0(n_s=256)
    cases = [(big, "c64", "auto", 3, 1e-5), (small, "c128", "fp64", 0, 1e-10)]
    for w, dt, gram, refine, tol in cases:
        need = gpu_lib.workspace_query([(w.n_s, w.block_sizes, w.lam)], dt, gram, refine)
        say(f"case: {w.name} n_s={w.n_s} blocks={w.block_sizes} {dt} {gram} refine={refine}: workspace {need} B")
        assert need <= 64 << 20
        ds, sts = run(gpu_lib, w, dt, gram, refine, static=True)
        dr, str_ = run(gpu_lib, w, dt, gram, refine, static=False)
        assert all(v == 0 for v in sts) and all(v == 0 for v in str_)
        assert np.array_equal(ds.view(np.uint64), dr.view(np.uint64))
        ref = orc.block_sr(w.O, w.e_loc, w.block_sizes, w.lam).delta
        err = max(orc.block_relative_errors(ds, ref, w.block_sizes))
        say(f"  static == caller workspace bit for bit; max block rel err vs oracle {err:.2e}")
        assert err <= tol


def test_static_workspace_refuses_large_plans(gpu_lib):
    sizes = [8192]
    sr = gpu_lib.BlockSR([(4096, sizes, 1e-3)], "c64", "fp32", 0)
    assert sr.workspace_bytes > 64 << 20
    O = torch.zeros((4096, 8192), dtype=torch.complex64, device="cuda")
    e = torch.zeros(4096, dtype=torch.complex128, device="cuda")
    with pytest.raises(gpu_lib.QgtError) as exc:
        sr.form_static([O], [e])
    assert exc.value.status == 3 and "static workspace" in str(exc.value)
    sr.close()
