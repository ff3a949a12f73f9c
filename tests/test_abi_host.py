"""Host-only checks of the C ABI: the library loads, exports every function the
header declares, validates arguments synchronously and sizes the workspace.
No GPU call is made."""
import ctypes

import numpy as np

import pytest

import paper_2510_08430_amd as qgt


@pytest.fixture(scope="module")
def lib():
    return qgt.load()


def test_exports_every_header_function(lib):
    names = qgt.header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    for s in range(9):
        assert lib.qgt_status_string(s)
    assert lib.qgt_status_string(99) == b"unknown status"


@pytest.mark.parametrize("problems,err", [
    ([(1, [4], 1e-3)], qgt.STATUS_NAMES[1]),            # n_s < 2
    ([(16, [4, 0], 1e-3)], qgt.STATUS_NAMES[1]),        # empty block
    ([(16, [4, -3], 1e-3)], qgt.STATUS_NAMES[1]),       # negative block
    ([(16, [4], 0.0)], qgt.STATUS_NAMES[1]),            # lambda = 0
    ([(16, [4], -1e-3)], qgt.STATUS_NAMES[1]),          # lambda < 0
    ([(16, [4], float("nan"))], qgt.STATUS_NAMES[1]),   # lambda NaN
    ([(16, [4], float("inf"))], qgt.STATUS_NAMES[1]),   # lambda inf
    ([(16, [], 1e-3)], qgt.STATUS_NAMES[1]),            # no blocks
])
def test_invalid_arguments(problems, err):
    with pytest.raises(qgt.QgtError) as ei:
        qgt.workspace_query(problems)
    assert err in str(ei.value)


def test_invalid_refine_and_counts():
    with pytest.raises(qgt.QgtError):
        qgt.workspace_query([(16, [4], 1e-3)], max_refine=17)
    with pytest.raises(qgt.QgtError):
        qgt.workspace_query([(16, [4], 1e-3)] * 65)
    with pytest.raises(qgt.QgtError):
        qgt.workspace_query([(16, [4, 5], 1e-3)], forms=["P", 7])


def test_null_problem_pointer(lib):
    ws = ctypes.c_size_t(0)
    assert lib.qgt_block_workspace_query(None, 1, 0, 0, 0, None, ctypes.byref(ws)) == 1
    assert b"null" in lib.qgt_last_error()


def test_workspace_grows_with_problem():
    a = qgt.workspace_query([(1024, [512, 32, 16], 1e-4)], "c128", "fp64")
    b = qgt.workspace_query([(2048, [512, 32, 16], 1e-4)], "c128", "fp64")
    c = qgt.workspace_query([(1024, [512, 32, 16, 100], 1e-4)], "c128", "fp64")
    assert 0 < a < b and a < c
    # two instances need more than one
    d = qgt.workspace_query([(1024, [512, 32, 16], 1e-4)] * 2, "c128", "fp64")
    assert d > a
    # BF16 packs the operand in fewer bytes than FP32, FP32 fewer than FP64
    w64 = qgt.workspace_query([(4096, [3000], 1e-3)], "c64", "fp64")
    w32 = qgt.workspace_query([(4096, [3000], 1e-3)], "c64", "fp32")
    w16 = qgt.workspace_query([(4096, [3000], 1e-3)], "c64", "bf16")
    assert w16 < w32 < w64


def test_sample_form_workspace_is_sample_sized():
    # n_b = 20000 > n_s = 1024: the sample form needs an n_s x n_s matrix, far
    # smaller than the n_b x n_b parameter-form matrix
    s = qgt.workspace_query([(1024, [20000], 1e-3)], "c64", "fp32")
    p = qgt.workspace_query([(1024, [20000], 1e-3)], "c64", "fp32", forms=["P"])
    assert s < p / 10
    assert s < 20000 * 20000 * 16


def test_full_workspace_matches_single_block(lib):
    arr, keep = qgt._problems([(256, [100, 60], 1e-3)])
    full = lib.qgt_full_workspace_bytes(arr, 1)
    assert full == qgt.workspace_query([(256, [160], 1e-3)], "c128", "fp64", max_refine=0)


def test_planner_task_orders_are_topological():
    """The planner checks on the host that the tickets of the persistent
    Cholesky (tile tasks of all blocks) and of the triangular solves are in
    dependency order, by executing them one at a time in ticket order (the
    property that makes the device-side waits end), and that every tile ends
    factored; it fails with QGT_ERR_INTERNAL otherwise."""
    import random
    rng = random.Random(7)
    cases = [[(4096, [8320, 16512, 8256, 65], 1e-3)], [(1024, [512, 32, 16], 1e-4)],
             [(8192, [160, 2320, 2320, 2320], 1e-4)]]
    for _ in range(40):
        cases.append([(rng.choice([64, 2048, 8192]), [rng.randint(64, 8192) for _ in range(rng.randint(1, 8))], 1e-5)])
        cases.append([(rng.choice([2, 64, 100, 777, 1024, 2000]),
                       [rng.randint(1, 3000) for _ in range(rng.randint(1, 6))], 1e-3)
                      for _ in range(rng.randint(1, 4))])
    for c in cases:
        assert qgt.workspace_query(c, "c64", "fp32") > 0


# ---------------------------------------------------------------------------
# device formation of O: host-side validation and sizes (no GPU call is made:
# every call below is rejected before any launch)
# ---------------------------------------------------------------------------
def test_ffnn_parameter_count_and_workspace():
    assert qgt.ffnn_n_params([64, 128, 128, 64], readout=True) == 33153
    assert qgt.ffnn_n_params([100, 400, 400]) == 200800
    assert qgt.ffnn_n_params([16, 32, 16]) == 2 * 16 * 16 * 2 + 32 + 16
    # two complex128 arrays per layer (tanh/derivative and activation), no
    # activation array for the last layer without a readout
    a = qgt.ffnn_jacobian_workspace_bytes([8, 10, 6], False, 100)
    b = qgt.ffnn_jacobian_workspace_bytes([8, 10, 6], True, 100)
    assert a >= 100 * (10 + 10 + 6) * 16 and b >= a + 100 * 6 * 16
    assert qgt.rbm_jacobian_workspace_bytes(16, 32, 1024) >= 1024 * 32 * 16
    with pytest.raises(qgt.QgtError):
        qgt.ffnn_n_params([8])                    # no layer
    with pytest.raises(qgt.QgtError):
        qgt.ffnn_n_params([8, 0, 4])              # empty layer
    with pytest.raises(qgt.QgtError):
        qgt.ffnn_n_params([8, 70000])             # width beyond 2^16
    with pytest.raises(qgt.QgtError):
        qgt.ffnn_n_params([8] * 10)               # more than 8 layers
    assert qgt.ffnn_jacobian_workspace_bytes([8, 4], False, 0) == 0


def _gpu_reachable():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


# The calls below pass placeholder device addresses with exactly one invalid
# argument each, so the library must reject them before any launch; they are
# kept off machines with a GPU, where a validation bug would launch kernels on
# those addresses.
no_gpu_only = pytest.mark.skipif(_gpu_reachable(), reason="placeholder device pointers: host-only machines")


def _ffnn_call(lib, widths, readout=0, theta=0x1000, x=0x2000, ldx=None, n_s=16, dt=0, O=0x3000, ldo=None,
               ws=0x4000, wsb=1 << 30):
    w = (ctypes.c_int32 * len(widths))(*widths)
    d = qgt._Ffnn(len(widths) - 1, ctypes.cast(w, qgt._c_i32p), readout)
    n_p = qgt.ffnn_n_params(widths, readout == 1)
    return lib.qgt_ffnn_jacobian(ctypes.byref(d), theta, x, widths[0] if ldx is None else ldx, n_s, dt, O,
                                 n_p if ldo is None else ldo, ws, wsb, None)


@pytest.mark.parametrize("kw,err", [
    (dict(theta=None), 1), (dict(x=None), 1), (dict(O=None), 1), (dict(ws=None), 1),
    (dict(dt=7), 1), (dict(ldx=4), 1), (dict(ldo=5), 1), (dict(wsb=16), 3),
    (dict(ws=0x4010), 1), (dict(n_s=0), 2), (dict(n_s=(1 << 24) + 1), 2), (dict(readout=2), 1),
])
@no_gpu_only
def test_ffnn_jacobian_rejects_bad_arguments(lib, kw, err):
    assert _ffnn_call(lib, [8, 10, 6], **kw) == err
    assert lib.qgt_last_error()


@no_gpu_only
def test_rbm_jacobian_rejects_bad_arguments(lib):
    f = lib.qgt_rbm_jacobian
    ok = dict(N=16, M=32, theta=0x1000, x=0x2000, ldx=16, n_s=8, dt=1, O=0x3000, ldo=560, ws=0x4000, wsb=1 << 20)

    def call(**kw):
        a = {**ok, **kw}
        return f(a["N"], a["M"], a["theta"], a["x"], a["ldx"], a["n_s"], a["dt"], a["O"], a["ldo"], a["ws"],
                 a["wsb"], None)
    assert call(N=0) == 2 and call(M=70000) == 2
    assert call(theta=None) == 1 and call(ldx=15) == 1 and call(ldo=559) == 1
    assert call(wsb=100) == 3 and call(n_s=0) == 2


def test_cnn_parameter_count_and_limits():
    assert qgt.cnn_n_params(10, 16, 4) == 7120
    assert qgt.cnn_n_params(4, 3, 3) == 3 * 9 + 3 + 2 * (3 * 3 * 9 + 3)
    assert qgt.cnn_jacobian_workspace_bytes(10, 16, 4, 8192) >= 7 * 8192 * 16 * 100 * 16
    assert qgt.cnn_n_params(11, 16, 2) > 0
    for bad in [(1, 4, 2), (10, 17, 2), (10, 16, 9), (12, 16, 2), (10, 0, 2)]:
        with pytest.raises(qgt.QgtError):
            qgt.cnn_n_params(*bad)


@no_gpu_only
def test_vmc_entry_points_reject_bad_arguments(lib):
    P = 0x1000
    f = lib.qgt_rbm_metropolis
    assert f(1, 4, P, P, 16, 8, 4, P, P, None, None) == 2          # N < 2
    assert f(65, 4, P, P, 65, 8, 4, P, P, None, None) == 2         # N > 64
    assert f(16, 0, P, P, 16, 8, 4, P, P, None, None) == 2         # M < 1
    assert f(16, 4, None, P, 16, 8, 4, P, P, None, None) == 1      # theta null
    assert f(16, 4, P, P, 15, 8, 4, P, P, None, None) == 1         # ldx < N
    assert f(16, 4, P, P, 16, 8, -1, P, P, None, None) == 1        # n_steps < 0
    assert f(16, 4, P, P, 16, 8, 4, None, P, None, None) == 1      # pairs null
    assert f(16, 4, P, P, 16, 0, 4, P, P, None, None) == 2         # no chains
    g = lib.qgt_rbm_heisenberg_eloc
    assert g(16, 4, P, P, 16, 8, 1.0, 1, None, None) == 1          # e_loc null
    assert g(16, 4, P, None, 16, 8, 1.0, 1, P, None) == 1          # x null
    h = lib.qgt_sr_update
    assert h(None, P, 10, 0.1, None) == 1 and h(P, P, 0, 0.1, None) == 2


@no_gpu_only
def test_cnn_jacobian_rejects_bad_arguments(lib):
    P = 0x1000
    n_p = qgt.cnn_n_params(6, 4, 2)

    def call(side=6, C=4, L=2, theta=P, x=P, ldx=36, n_s=8, dt=0, O=P, ldo=None, ws=P, wsb=1 << 30):
        d = qgt._Cnn(side, C, L)
        return lib.qgt_cnn_jacobian(ctypes.byref(d), theta, x, ldx, n_s, dt, O, n_p if ldo is None else ldo, ws,
                                    wsb, None)
    assert call(side=1) == 2 and call(C=17) == 2 and call(L=0) == 2 and call(n_s=0) == 2
    assert call(theta=None) == 1 and call(x=None) == 1 and call(O=None) == 1
    assert call(ldx=35) == 1 and call(ldo=n_p - 1) == 1 and call(dt=5) == 1
    assert call(wsb=1000) == 3 and call(ws=0x1010) == 1
