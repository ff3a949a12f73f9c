"""Host-only checks of the C ABI: the library loads, exports every function the
header declares, validates arguments synchronously and sizes the workspace.
No GPU call is made."""
import ctypes

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
    """The planner checks on the host that the Cholesky task tickets and the
    triangular-solve tickets are in dependency order (the property that makes
    the device-side waits end); it fails with QGT_ERR_INTERNAL otherwise."""
    import random
    rng = random.Random(7)
    cases = [[(4096, [8320, 16512, 8256, 65], 1e-3)], [(1024, [512, 32, 16], 1e-4)],
             [(8192, [160, 2320, 2320, 2320], 1e-4)]]
    for _ in range(40):
        cases.append([(rng.choice([2, 64, 100, 777, 1024, 2000]),
                       [rng.randint(1, 3000) for _ in range(rng.randint(1, 6))], 1e-3)
                      for _ in range(rng.randint(1, 4))])
    for c in cases:
        assert qgt.workspace_query(c, "c64", "fp32") > 0
