"""Python binding of libqgtblock.so, the MI355X (gfx950) block-layer QGT
stochastic-reconfiguration library.

Argument marshalling only: every step of the SR path runs in the library's HIP
kernels.  PyTorch supplies device memory (O, E_loc, delta, the workspace) and
streams.  The entry points mirror the C ABI in include/qgt_block.h:

    BlockSR(problems, o_dtype, gram, max_refine)   -> qgt_block_plan
    BlockSR.form(O, e_loc)                         -> qgt_block_form
    BlockSR.solve(delta)                           -> qgt_block_solve
    full_solve(O, e_loc, lam)                      -> qgt_full_solve

If the shared library has not been built, loading fails with an error; there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqgtblock.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
HEADER = os.path.join(INCLUDE, "qgt_block.h")
HEADERS = [os.path.join(INCLUDE, "qgt_block.h"), os.path.join(INCLUDE, "qgt_jacobian.h"),
           os.path.join(INCLUDE, "qgt_vmc.h")]

QGT_OK = 0
STATUS_NAMES = {0: "QGT_OK", 1: "QGT_ERR_INVALID_ARGUMENT", 2: "QGT_ERR_UNSUPPORTED", 3: "QGT_ERR_WORKSPACE_TOO_SMALL",
                4: "QGT_ERR_HIP", 5: "QGT_ERR_NOT_POSITIVE_DEFINITE", 6: "QGT_ERR_NOT_CONVERGED",
                7: "QGT_ERR_NON_FINITE", 8: "QGT_ERR_INTERNAL"}
DTYPES = {"c64": 0, "c128": 1}
GRAMS = {"fp64": 0, "fp32": 1, "bf16": 2, "auto": 3}
FORMS = {"auto": 0, "P": 1, "S": 2}
FORM_NAMES = {1: "P", 2: "S"}
FACTORS = {"fp64": 0, "fp32": 1}  # fp32: complex64 storage and an FP32 factorisation of BF16-Gram blocks
PREC_NAMES = {0: "fp64", 1: "fp32", 2: "bf16"}

_c_i64p = ctypes.POINTER(ctypes.c_int64)
_c_i32p = ctypes.POINTER(ctypes.c_int32)


class QgtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _Problem(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int64), ("n_blocks", ctypes.c_int32),
                ("block_sizes", _c_i64p), ("lambda_", ctypes.c_double)]


class _Ffnn(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("widths", ctypes.POINTER(ctypes.c_int32)),
                ("readout", ctypes.c_int32)]


class _Cnn(ctypes.Structure):
    _fields_ = [("side", ctypes.c_int32), ("channels", ctypes.c_int32), ("n_layers", ctypes.c_int32)]


class _Tuning(ctypes.Structure):
    _fields_ = [("gram_tile", ctypes.c_int32), ("gram_items", ctypes.c_int32), ("chol_chunk", ctypes.c_int32),
                ("gram_patch", ctypes.c_int32)]


class _Options(ctypes.Structure):
    _fields_ = [("forms", _c_i32p), ("timing", ctypes.c_int32), ("factor", ctypes.c_int32),
                ("tuning", ctypes.POINTER(_Tuning)), ("cholesky", ctypes.c_int32), ("pad", ctypes.c_int32)]


CHOLESKY = {"auto": 0, "host-steps": 1, "persistent": 2}
CHOLESKY_NAMES = {v: k for k, v in CHOLESKY.items()}


TUNING_FIELDS = ("gram_tile", "gram_items", "chol_chunk", "gram_patch")
TUNING_SOURCES = {0: "default", 1: "caller", 2: "cache", 3: "plan-cache"}


_lib = None


def header_functions() -> list[str]:
    """Names of the functions declared in the public headers under include/."""
    names = set()
    for path in HEADERS:
        with open(path) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(qgt_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the built library (build it with `python -m paper_2510_08430_amd.build`)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2510_08430_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    sig = {
        "qgt_block_plan": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.c_int32, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int32, ctypes.c_double, ctypes.POINTER(vp),
                                          ctypes.POINTER(sz)]),
        "qgt_block_plan_ex": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.c_int32, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int32, ctypes.c_double, ctypes.POINTER(_Options),
                                             ctypes.POINTER(vp), ctypes.POINTER(sz)]),
        "qgt_block_workspace_query": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.c_int32, ctypes.c_int,
                                                     ctypes.c_int, ctypes.c_int32, ctypes.POINTER(_Options),
                                                     ctypes.POINTER(sz)]),
        "qgt_block_form": (ctypes.c_int, [vp, ctypes.POINTER(vp), _c_i64p, ctypes.POINTER(vp), vp, sz, vp]),
        "qgt_block_solve": (ctypes.c_int, [vp, ctypes.POINTER(vp), vp]),
        "qgt_block_form_static": (ctypes.c_int, [vp, ctypes.POINTER(vp), _c_i64p, ctypes.POINTER(vp), vp]),
        "qgt_full_workspace_bytes": (sz, [ctypes.POINTER(_Problem), ctypes.c_int]),
        "qgt_full_release": (None, []),
        "qgt_block_inverse_scratch_bytes": (sz, [vp, ctypes.c_int32]),
        "qgt_block_inverse_diagnostics": (ctypes.c_int, [vp, ctypes.c_int32, vp, ctypes.c_int64, vp, sz, vp, vp]),
        "qgt_full_solve": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.c_int, vp, ctypes.c_int64, vp, vp, vp,
                                          sz, vp]),
        "qgt_plan_status": (ctypes.c_int, [vp, _c_i32p]),
        "qgt_plan_num_blocks": (ctypes.c_int32, [vp]),
        "qgt_plan_block_info": (ctypes.c_int, [vp, ctypes.c_int32, _c_i32p, _c_i64p, _c_i64p, _c_i32p, _c_i32p]),
        "qgt_plan_block_factor": (ctypes.c_int, [vp, ctypes.c_int32, _c_i32p]),
        "qgt_plan_block_tuning": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.POINTER(_Tuning), _c_i32p]),
        "qgt_plan_cholesky": (ctypes.c_int, [vp, _c_i32p, _c_i32p]),
        "qgt_cholesky_query": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.c_int32, ctypes.c_int, ctypes.c_int,
                                              ctypes.POINTER(_Options), _c_i32p, _c_i32p]),
        "qgt_block_tuning_query": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.c_int32, ctypes.c_int, ctypes.c_int,
                                                  ctypes.POINTER(_Options), ctypes.c_int32, ctypes.POINTER(_Tuning),
                                                  _c_i32p]),
        "qgt_autotune": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.c_int32, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_char_p, ctypes.c_int32, _c_i32p]),
        "qgt_plan_pivot_floors": (ctypes.c_int, [vp, _c_i32p]),
        "qgt_plan_debug_ptr": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(vp), _c_i64p]),
        "qgt_plan_gram_timing": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), _c_i64p,
                                                ctypes.POINTER(ctypes.c_double), ctypes.c_int32]),
        "qgt_plan_destroy": (None, [vp]),
        "qgt_rbm_jacobian_workspace_bytes": (sz, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64]),
        "qgt_rbm_jacobian": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, vp, vp, ctypes.c_int64, ctypes.c_int64,
                                            ctypes.c_int, vp, ctypes.c_int64, vp, sz, vp]),
        "qgt_ffnn_n_params": (ctypes.c_int64, [ctypes.POINTER(_Ffnn)]),
        "qgt_cnn_n_params": (ctypes.c_int64, [ctypes.POINTER(_Cnn)]),
        "qgt_rbm_metropolis": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, vp, vp, ctypes.c_int64, ctypes.c_int64,
                                              ctypes.c_int32, vp, vp, vp, vp]),
        "qgt_rbm_heisenberg_eloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, vp, vp, ctypes.c_int64,
                                                   ctypes.c_int64, ctypes.c_double, ctypes.c_int32, vp, vp]),
        "qgt_sr_update": (ctypes.c_int, [vp, vp, ctypes.c_int64, ctypes.c_double, vp]),
        "qgt_cnn_jacobian_workspace_bytes": (sz, [ctypes.POINTER(_Cnn), ctypes.c_int64]),
        "qgt_cnn_jacobian": (ctypes.c_int, [ctypes.POINTER(_Cnn), vp, vp, ctypes.c_int64, ctypes.c_int64,
                                            ctypes.c_int, vp, ctypes.c_int64, vp, sz, vp]),
        "qgt_ffnn_jacobian_workspace_bytes": (sz, [ctypes.POINTER(_Ffnn), ctypes.c_int64]),
        "qgt_ffnn_jacobian": (ctypes.c_int, [ctypes.POINTER(_Ffnn), vp, vp, ctypes.c_int64, ctypes.c_int64,
                                             ctypes.c_int, vp, ctypes.c_int64, vp, sz, vp]),
        "qgt_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "qgt_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != QGT_OK:
        raise QgtError(status, _lib.qgt_last_error().decode())


def _problems(problems):
    """problems: sequence of (n_samples, block_sizes, lambda)."""
    arr = (_Problem * len(problems))()
    keep = []
    for i, (ns, sizes, lam) in enumerate(problems):
        bs = (ctypes.c_int64 * len(sizes))(*[int(s) for s in sizes])
        keep.append(bs)
        arr[i] = _Problem(int(ns), len(sizes), ctypes.cast(bs, _c_i64p), float(lam))
    return arr, keep


def _options(forms, timing, factor="fp64", tuning=None, cholesky="auto"):
    """The qgt_plan_options struct (and the arrays it points to, which the
    caller keeps alive).  tuning: None, or one dict per block over all
    problems with any of TUNING_FIELDS (missing or 0: the planner's default)."""
    if factor not in FACTORS:
        raise ValueError(f"factor must be one of {sorted(FACTORS)}")
    if cholesky not in CHOLESKY:
        raise ValueError(f"cholesky must be one of {sorted(CHOLESKY)}")
    if forms is None and not timing and factor == "fp64" and tuning is None and cholesky == "auto":
        return None, None
    fa = ta = None
    if forms is not None:
        fa = (ctypes.c_int32 * len(forms))(*[FORMS[f] if isinstance(f, str) else int(f) for f in forms])
    if tuning is not None:
        for t in tuning:
            bad = set(t) - set(TUNING_FIELDS)
            if bad:
                raise ValueError(f"unknown tuning fields {sorted(bad)}")
        ta = (_Tuning * len(tuning))(*[_Tuning(*[int(t.get(k, 0)) for k in TUNING_FIELDS]) for t in tuning])
    opt = _Options(ctypes.cast(fa, _c_i32p) if fa is not None else None, 1 if timing else 0, FACTORS[factor],
                   ctypes.cast(ta, ctypes.POINTER(_Tuning)) if ta is not None else None, CHOLESKY[cholesky], 0)
    return opt, (fa, ta)


def workspace_query(problems, o_dtype="c64", gram="auto", max_refine=1, forms=None, factor="fp64") -> int:
    """Host-only planning: the workspace size in bytes (no HIP call)."""
    lib = load()
    arr, keep = _problems(problems)
    opt, fa = _options(forms, False, factor)
    ws = ctypes.c_size_t(0)
    _check(lib.qgt_block_workspace_query(arr, len(problems), DTYPES[o_dtype], GRAMS[gram], int(max_refine),
                                         ctypes.byref(opt) if opt is not None else None, ctypes.byref(ws)))
    return ws.value


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class BlockSR:
    """One plan for a batch of independent block-SR problems.

    problems: sequence of (n_samples, block_sizes, lambda).
    factor: "fp64" (every block factored in FP64, the default) or "fp32"
    (blocks with a BF16 Gram stored in complex64 and factored in FP32).
    tuning: None, or one dict per block of tile shapes and schedules
    (TUNING_FIELDS).  cholesky: "persistent" (one launch over the tile tasks
    of every block), "host-steps" (one launch per tile step of all blocks) or
    "auto" (the mode the tuning cache records for this set of blocks, else
    persistent).
    """

    def __init__(self, problems, o_dtype="c64", gram="auto", max_refine=1, forms=None, timing=False, device=None,
                 rtol=0.0, factor="fp64", tuning=None, cholesky="auto"):
        import torch
        lib = load()
        self.problems = [(int(ns), [int(s) for s in sizes], float(lam)) for ns, sizes, lam in problems]
        self.o_dtype = o_dtype
        if o_dtype not in DTYPES or gram not in GRAMS:
            raise ValueError(f"o_dtype must be one of {sorted(DTYPES)} and gram one of {sorted(GRAMS)}")
        arr, keep = _problems(self.problems)
        opt, fa = _options(forms, timing, factor, tuning, cholesky)
        plan = ctypes.c_void_p()
        ws = ctypes.c_size_t(0)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        with torch.cuda.device(self.device):
            _check(lib.qgt_block_plan_ex(arr, len(self.problems), DTYPES[o_dtype], GRAMS[gram], int(max_refine),
                                         float(rtol),
                                         ctypes.byref(opt) if opt is not None else None, ctypes.byref(plan),
                                         ctypes.byref(ws)))
        self._plan = plan
        self.workspace_bytes = ws.value
        self.workspace = torch.empty(max(ws.value, 256), dtype=torch.uint8, device=self.device)
        self._refs = []

    # -- plan introspection ------------------------------------------------
    @property
    def num_blocks(self) -> int:
        return load().qgt_plan_num_blocks(self._plan)

    def block_info(self, g: int) -> dict:
        p, f, pr = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        off, size = ctypes.c_int64(), ctypes.c_int64()
        _check(load().qgt_plan_block_info(self._plan, g, ctypes.byref(p), ctypes.byref(off), ctypes.byref(size),
                                          ctypes.byref(f), ctypes.byref(pr)))
        fp32 = ctypes.c_int32()
        _check(load().qgt_plan_block_factor(self._plan, g, ctypes.byref(fp32)))
        return dict(problem=p.value, offset=off.value, size=size.value, form=FORM_NAMES[f.value],
                    precision=PREC_NAMES[pr.value], factor="fp32" if fp32.value else "fp64")

    # -- the two steps ------------------------------------------------------
    def _bind_inputs(self, O, e_loc):
        import torch
        n = len(self.problems)
        if len(O) != n or len(e_loc) != n:
            raise ValueError("one O and one e_loc per problem")
        want = torch.complex64 if self.o_dtype == "c64" else torch.complex128
        for p, (o, e) in enumerate(zip(O, e_loc)):
            if o.dtype != want or o.dim() != 2 or o.stride(1) != 1 or not o.is_cuda:
                raise ValueError(f"O[{p}] must be a row-major {want} CUDA matrix")
            if o.shape[0] != self.problems[p][0] or o.shape[1] != sum(self.problems[p][1]):
                raise ValueError(f"O[{p}] has shape {tuple(o.shape)}, expected "
                                 f"({self.problems[p][0]}, {sum(self.problems[p][1])})")
            if e.dtype != torch.complex128 or not e.is_contiguous() or e.numel() != self.problems[p][0]:
                raise ValueError(f"e_loc[{p}] must be a contiguous complex128 vector of n_samples")
        optrs = (ctypes.c_void_p * n)(*[o.data_ptr() for o in O])
        lds = (ctypes.c_int64 * n)(*[o.stride(0) for o in O])
        eptrs = (ctypes.c_void_p * n)(*[e.data_ptr() for e in e_loc])
        self._refs = [list(O), list(e_loc)]  # O and E are read again by solve
        return optrs, lds, eptrs

    def form(self, O: Sequence, e_loc: Sequence, stream=None):
        optrs, lds, eptrs = self._bind_inputs(O, e_loc)
        _check(load().qgt_block_form(self._plan, optrs, lds, eptrs, ctypes.c_void_p(self.workspace.data_ptr()),
                                     self.workspace_bytes, _stream_handle(stream)))

    def form_static(self, O: Sequence, e_loc: Sequence, stream=None):
        """qgt_block_form_static: the form step in the library's static
        per-device workspace (for callers that cannot allocate); the plan's
        own workspace tensor is left untouched, and the debug views of this
        class do not apply until the next form()."""
        optrs, lds, eptrs = self._bind_inputs(O, e_loc)
        _check(load().qgt_block_form_static(self._plan, optrs, lds, eptrs, _stream_handle(stream)))

    def solve(self, delta: Sequence, stream=None):
        import torch
        n = len(self.problems)
        if len(delta) != n:
            raise ValueError("one delta per problem")
        for p, d in enumerate(delta):
            if d.dtype != torch.complex128 or not d.is_contiguous() or d.numel() != sum(self.problems[p][1]):
                raise ValueError(f"delta[{p}] must be a contiguous complex128 vector of n_p")
        dptrs = (ctypes.c_void_p * n)(*[d.data_ptr() for d in delta])
        _check(load().qgt_block_solve(self._plan, dptrs, _stream_handle(stream)))

    def __call__(self, O, e_loc, stream=None):
        import torch
        delta = [torch.empty(sum(sizes), dtype=torch.complex128, device=self.device) for _, sizes, _ in self.problems]
        self.form(O, e_loc, stream)
        self.solve(delta, stream)
        return delta

    # -- diagnostics --------------------------------------------------------
    def status(self):
        """Per-block numerical status (synchronises the device first)."""
        import torch
        torch.cuda.synchronize(self.device)
        nb = self.num_blocks
        arr = (ctypes.c_int32 * nb)()
        st = load().qgt_plan_status(self._plan, arr)
        # the call returns the worst block status, or an error of its own
        # (no workspace bound, a failed copy) when it could not read them
        if st not in [int(v) for v in arr] + [QGT_OK]:
            _check(st)
        return [int(v) for v in arr]

    def pivot_floors(self):
        """Per-block count of Cholesky pivots raised to lambda in the last solve
        (synchronises the device first)."""
        import torch
        torch.cuda.synchronize(self.device)
        nb = self.num_blocks
        arr = (ctypes.c_int32 * nb)()
        _check(load().qgt_plan_pivot_floors(self._plan, arr))
        return [int(v) for v in arr]

    def debug_tensor(self, which: int, index: int, count: int):
        """View of an intermediate buffer of the bound workspace (see qgt_plan_debug_ptr)."""
        import torch
        ptr = ctypes.c_void_p()
        ld = ctypes.c_int64()
        _check(load().qgt_plan_debug_ptr(self._plan, which, index, ctypes.byref(ptr), ctypes.byref(ld)))
        off = ptr.value - self.workspace.data_ptr()
        return self.workspace[off: off + 16 * count].view(torch.complex128), ld.value

    def block_matrix(self, g: int):
        """Stored matrix of global block g as an (m, m) complex128 numpy array,
        m = n_b (parameter form) or n_s (sample form): the shifted Gram after
        form(), its Cholesky factor after solve(); the lower triangle is
        returned (the rest is zero).  Blocks factored in FP32 store it in
        complex64."""
        import numpy as np
        import torch
        info = self.block_info(g)
        m = info["size"] if info["form"] == "P" else self.problems[info["problem"]][0]
        _, ld = self.debug_bytes(3, g, 0)
        c64 = info["factor"] == "fp32"
        raw, _ = self.debug_bytes(3, g, ld * ld * (8 if c64 else 16))
        a = raw.view(torch.complex64 if c64 else torch.complex128).cpu().numpy().reshape(ld, ld)
        return np.tril(a[:m, :m]).astype(np.complex128)

    def debug_bytes(self, which: int, index: int, nbytes: int):
        """Raw bytes of an intermediate buffer (uint8 view) and its leading dimension."""
        ptr = ctypes.c_void_p()
        ld = ctypes.c_int64()
        _check(load().qgt_plan_debug_ptr(self._plan, which, index, ctypes.byref(ptr), ctypes.byref(ld)))
        off = ptr.value - self.workspace.data_ptr()
        return self.workspace[off: off + nbytes], ld.value

    def block_trace(self, g: int) -> float:
        """Trace of the QGT of global block g, as computed by the column pass."""
        import torch
        raw, _ = self.debug_bytes(5, g, 8)
        return float(raw.view(torch.float64).cpu()[0])

    def correction_estimate(self, g: int) -> float:
        """Relative size of the last CG correction of global block g (after a solve)."""
        import torch
        raw, _ = self.debug_bytes(6, g, 8)
        return float(raw.view(torch.float64).cpu()[0])

    def cg_iterations(self, g: int) -> int:
        """CG iterations global block g ran in the last solve (at most max_refine;
        fewer when it met refine_rtol early)."""
        import torch
        raw, _ = self.debug_bytes(7, g, 4)
        return int(raw.view(torch.int32).cpu()[0])

    def gram_timing(self, precision="fp32", reset=False):
        """(total ms, launches, flops per launch) of the Gram kernel of one precision."""
        ms, n, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        _check(load().qgt_plan_gram_timing(self._plan, GRAMS[precision], ctypes.byref(ms), ctypes.byref(n),
                                           ctypes.byref(fl), 1 if reset else 0))
        return ms.value, n.value, fl.value

    def inverse_diagnostics(self, B, problem: int = 0, stream=None) -> dict:
        """Eq. 4 (a) and (b) of the inverse of the shifted block-layer QGT of
        `problem` (from the Cholesky factors of the last solve) against the
        reference B (n_p x n_p complex128 device matrix with contiguous rows):
        qgt_block_inverse_diagnostics, then F and eps_F from its five sums."""
        import torch
        n_p = sum(self.problems[problem][1])
        if B.dtype != torch.complex128 or B.dim() != 2 or tuple(B.shape) != (n_p, n_p) or B.stride(1) != 1:
            raise ValueError(f"B must be a ({n_p}, {n_p}) complex128 matrix with contiguous rows")
        if not B.is_cuda:
            raise ValueError("B must be a CUDA (HIP device) tensor")
        lib = load()
        nb = lib.qgt_block_inverse_scratch_bytes(self._plan, int(problem))
        if nb == 0:
            raise QgtError(2, lib.qgt_last_error().decode())
        scratch = torch.empty(nb, dtype=torch.uint8, device=self.device)
        sums = torch.empty(5, dtype=torch.float64, device=self.device)
        _check(lib.qgt_block_inverse_diagnostics(self._plan, int(problem), ctypes.c_void_p(B.data_ptr()), B.stride(0),
                                                 ctypes.c_void_p(scratch.data_ptr()), nb,
                                                 ctypes.c_void_p(sums.data_ptr()), _stream_handle(stream)))
        v = sums.cpu().tolist()
        return {"frobenius_overlap": v[0] / (v[1] * v[2]) ** 0.5,
                "frobenius_relative_error": (max(v[3] + v[2] - v[4], 0.0) / v[2]) ** 0.5, "sums": v}

    def cholesky_mode(self) -> dict:
        """How this plan's factorisations launch ("persistent" or "host-steps")
        and where that came from ("default", "caller" or "cache")."""
        mode, src = ctypes.c_int32(), ctypes.c_int32()
        _check(load().qgt_plan_cholesky(self._plan, ctypes.byref(mode), ctypes.byref(src)))
        return {"mode": CHOLESKY_NAMES[mode.value], "source": TUNING_SOURCES[src.value]}

    def block_tuning(self, g: int) -> dict:
        """Tile shapes and schedules block g runs with, and their source
        ("default", "caller", "cache": the entry of the block's shape class,
        or "plan-cache": the entry of that class tuned inside this set of
        blocks)."""
        t, src = _Tuning(), ctypes.c_int32()
        _check(load().qgt_plan_block_tuning(self._plan, g, ctypes.byref(t), ctypes.byref(src)))
        return {**{k: getattr(t, k) for k in TUNING_FIELDS}, "source": TUNING_SOURCES[src.value]}

    def precisions(self):
        """Gram precisions used by the blocks of this plan."""
        return sorted({self.block_info(g)["precision"] for g in range(self.num_blocks)})

    def close(self):
        if getattr(self, "_plan", None):
            load().qgt_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def full_workspace_bytes(n_samples, n_params, lam, o_dtype="c64") -> int:
    arr, keep = _problems([(n_samples, [n_params], lam)])
    return load().qgt_full_workspace_bytes(arr, DTYPES[o_dtype])


def full_solve(O, e_loc, lam, stream=None, workspace=None):
    """Full-QGT SR in FP64 through qgt_full_solve (one block of all parameters)."""
    import torch
    lib = load()
    o_dtype = "c64" if O.dtype == torch.complex64 else "c128"
    n_s, n_p = O.shape
    arr, keep = _problems([(n_s, [n_p], lam)])
    wsb = lib.qgt_full_workspace_bytes(arr, DTYPES[o_dtype])
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(max(wsb, 256), dtype=torch.uint8, device=O.device)
    delta = torch.empty(n_p, dtype=torch.complex128, device=O.device)
    _check(lib.qgt_full_solve(arr, DTYPES[o_dtype], ctypes.c_void_p(O.data_ptr()), O.stride(0),
                              ctypes.c_void_p(e_loc.data_ptr()), ctypes.c_void_p(delta.data_ptr()),
                              ctypes.c_void_p(workspace.data_ptr()), wsb, _stream_handle(stream)))
    return delta


def tuning_query(problems, o_dtype="c64", gram="auto", g=0, forms=None, factor="fp64", tuning=None) -> dict:
    """Host only: the tuning block g of a plan of these problems would get
    (reads QGT_TUNE_CACHE like the planner)."""
    lib = load()
    arr, keep = _problems(problems)
    opt, fa = _options(forms, False, factor, tuning)
    t, src = _Tuning(), ctypes.c_int32()
    _check(lib.qgt_block_tuning_query(arr, len(problems), DTYPES[o_dtype], GRAMS[gram],
                                      ctypes.byref(opt) if opt is not None else None, int(g), ctypes.byref(t),
                                      ctypes.byref(src)))
    return {**{k: getattr(t, k) for k in TUNING_FIELDS}, "source": TUNING_SOURCES[src.value]}


def cholesky_query(problems, o_dtype="c64", gram="auto", forms=None, factor="fp64", cholesky="auto") -> dict:
    """Host only: the Cholesky launch mode (and its source) a plan of these
    problems would get (reads QGT_TUNE_CACHE like the planner)."""
    lib = load()
    arr, keep = _problems(problems)
    opt, fa = _options(forms, False, factor, None, cholesky)
    mode, src = ctypes.c_int32(), ctypes.c_int32()
    _check(lib.qgt_cholesky_query(arr, len(problems), DTYPES[o_dtype], GRAMS[gram],
                                  ctypes.byref(opt) if opt is not None else None, ctypes.byref(mode),
                                  ctypes.byref(src)))
    return {"mode": CHOLESKY_NAMES[mode.value], "source": TUNING_SOURCES[src.value]}


def autotune(problems, o_dtype="c64", gram="auto", cache_path=None, reps=3) -> int:
    """qgt_autotune: time candidate tile shapes and schedules for every shape
    class of the blocks of these problems on the current device and merge the
    fastest into the JSON cache at cache_path.  Returns the classes tuned."""
    if not cache_path:
        raise ValueError("cache_path is required")
    lib = load()
    arr, keep = _problems(problems)
    n = ctypes.c_int32()
    _check(lib.qgt_autotune(arr, len(problems), DTYPES[o_dtype], GRAMS[gram], os.fsencode(cache_path), int(reps),
                            ctypes.byref(n)))
    return n.value


def full_release():
    """Free the plans qgt_full_solve caches per shape (synchronises the device)."""
    load().qgt_full_release()


# ---------------------------------------------------------------------------
# Argument checks of the device-pointer entry points below: the C ABI receives
# bare pointers and sizes, so every length, type and layout it relies on is
# checked here before any launch (device last, so that these checks also run
# on the host).
# ---------------------------------------------------------------------------
def _dt(t):
    return str(t.dtype).replace("torch.", "")


def _need(cond, msg):
    if not cond:
        raise ValueError(msg)


def _check_vec(name, t, dtype, numel):
    _need(t is not None, f"{name} is missing")
    _need(_dt(t) == dtype, f"{name} must be {dtype}, got {_dt(t)}")
    _need(t.is_contiguous(), f"{name} must be contiguous")
    _need(t.numel() == numel, f"{name} must have {numel} elements, got {t.numel()}")


def _check_rows(name, t, dtype, cols, rows=None):
    """A 2-D matrix of the given element type whose rows are contiguous."""
    _need(t is not None, f"{name} is missing")
    _need(_dt(t) == dtype, f"{name} must be {dtype}, got {_dt(t)}")
    _need(t.dim() == 2, f"{name} must be a 2-D matrix")
    _need(t.shape[1] == cols, f"{name} must have {cols} columns, got {t.shape[1]}")
    _need(rows is None or t.shape[0] == rows, f"{name} must have {rows} rows, got {t.shape[0]}")
    _need(t.stride(1) == 1 and t.stride(0) >= max(cols, 1), f"{name} must have contiguous rows")


def _check_device(*named):
    ts = [(n, t) for n, t in named if t is not None]
    for n, t in ts:
        _need(t.is_cuda, f"{n} must be a CUDA (HIP device) tensor")
    devs = {t.device for _, t in ts}
    _need(len(devs) == 1, "all tensors must be on one device")


def _check_o_out(O, n_s, n_p):
    _need(_dt(O) in ("complex64", "complex128"), "O must be complex64 or complex128")
    _check_rows("O", O, _dt(O), n_p, n_s)


def _check_spins(x, n_spins):
    _check_rows("x", x, "int8", n_spins)


# ---------------------------------------------------------------------------
# Device formation of O (include/qgt_jacobian.h)
# ---------------------------------------------------------------------------
def _ffnn_desc(widths, readout):
    w = (ctypes.c_int32 * len(widths))(*[int(v) for v in widths])
    return _Ffnn(len(widths) - 1, ctypes.cast(w, _c_i32p), 1 if readout else 0), w


def ffnn_n_params(widths, readout=False) -> int:
    lib = load()
    d, keep = _ffnn_desc(widths, readout)
    n = lib.qgt_ffnn_n_params(ctypes.byref(d))
    if n < 0:
        raise QgtError(1, lib.qgt_last_error().decode())
    return n


def ffnn_jacobian_workspace_bytes(widths, readout, n_s) -> int:
    lib = load()
    d, keep = _ffnn_desc(widths, readout)
    return lib.qgt_ffnn_jacobian_workspace_bytes(ctypes.byref(d), int(n_s))


def rbm_jacobian_workspace_bytes(n_visible, n_hidden, n_s) -> int:
    return load().qgt_rbm_jacobian_workspace_bytes(int(n_visible), int(n_hidden), int(n_s))


def _o_dtype_of(O, o_dtype):
    if O is None:
        return o_dtype
    return "c64" if str(O.dtype) == "torch.complex64" else "c128"


def _jacobian_out(O, n_s, n_p, o_dtype, device):
    import torch
    if O is None:
        O = torch.empty((n_s, n_p), dtype=torch.complex64 if o_dtype == "c64" else torch.complex128, device=device)
    return O


def _workspace(workspace, nbytes, device):
    import torch
    if workspace is not None:
        _need(_dt(workspace) == "uint8" and workspace.is_contiguous(), "workspace must be a contiguous uint8 tensor")
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
    return workspace


def ffnn_jacobian(theta, x, widths, readout=False, o_dtype="c64", O=None, workspace=None, stream=None):
    """O (n_s x n_p) of a dense logcosh network through qgt_ffnn_jacobian.

    theta: complex128 device tensor (flat parameters); x: int8 device tensor
    (n_s x N, row stride >= N); O: optional output (complex64 or complex128,
    row stride >= n_p)."""
    lib = load()
    d, keep = _ffnn_desc(widths, readout)
    n_p = ffnn_n_params(widths, readout)
    _check_spins(x, int(widths[0]))
    _check_vec("theta", theta, "complex128", n_p)
    n_s = x.shape[0]
    o_dtype = _o_dtype_of(O, o_dtype)
    if O is not None:
        _check_o_out(O, n_s, n_p)
    _check_device(("theta", theta), ("x", x), ("O", O), ("workspace", workspace))
    O = _jacobian_out(O, n_s, n_p, o_dtype, x.device)
    workspace = _workspace(workspace, lib.qgt_ffnn_jacobian_workspace_bytes(ctypes.byref(d), n_s), x.device)
    _check(lib.qgt_ffnn_jacobian(ctypes.byref(d), ctypes.c_void_p(theta.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                 x.stride(0), n_s, DTYPES[o_dtype], ctypes.c_void_p(O.data_ptr()), O.stride(0),
                                 ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream_handle(stream)))
    return O


def rbm_jacobian(theta, x, n_hidden, o_dtype="c128", O=None, workspace=None, stream=None):
    """O (n_s x (M N + M + N)) of an RBM through qgt_rbm_jacobian."""
    lib = load()
    _need(x is not None and x.dim() == 2, "x must be a 2-D int8 matrix")
    n_s, N = x.shape
    M = int(n_hidden)
    _check_spins(x, N)
    _check_vec("theta", theta, "complex128", M * N + M + N)
    o_dtype = _o_dtype_of(O, o_dtype)
    if O is not None:
        _check_o_out(O, n_s, M * N + M + N)
    _check_device(("theta", theta), ("x", x), ("O", O), ("workspace", workspace))
    O = _jacobian_out(O, n_s, M * N + M + N, o_dtype, x.device)
    workspace = _workspace(workspace, lib.qgt_rbm_jacobian_workspace_bytes(N, M, n_s), x.device)
    _check(lib.qgt_rbm_jacobian(N, M, ctypes.c_void_p(theta.data_ptr()), ctypes.c_void_p(x.data_ptr()), x.stride(0),
                                n_s, DTYPES[o_dtype], ctypes.c_void_p(O.data_ptr()), O.stride(0),
                                ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream_handle(stream)))
    return O


def cnn_n_params(side, channels, n_layers) -> int:
    lib = load()
    n = lib.qgt_cnn_n_params(ctypes.byref(_Cnn(int(side), int(channels), int(n_layers))))
    if n < 0:
        raise QgtError(1, lib.qgt_last_error().decode())
    return n


def cnn_jacobian_workspace_bytes(side, channels, n_layers, n_s) -> int:
    return load().qgt_cnn_jacobian_workspace_bytes(ctypes.byref(_Cnn(int(side), int(channels), int(n_layers))),
                                                  int(n_s))


def cnn_jacobian(theta, x, side, channels, n_layers, o_dtype="c64", O=None, workspace=None, stream=None):
    """O (n_s x n_p) of a periodic 3x3 convolutional network through qgt_cnn_jacobian;
    x: int8 device tensor (n_s x side^2, row stride >= side^2)."""
    lib = load()
    d = _Cnn(int(side), int(channels), int(n_layers))
    n_p = cnn_n_params(side, channels, n_layers)
    _check_spins(x, int(side) * int(side))
    _check_vec("theta", theta, "complex128", n_p)
    n_s = x.shape[0]
    o_dtype = _o_dtype_of(O, o_dtype)
    if O is not None:
        _check_o_out(O, n_s, n_p)
    _check_device(("theta", theta), ("x", x), ("O", O), ("workspace", workspace))
    O = _jacobian_out(O, n_s, n_p, o_dtype, x.device)
    workspace = _workspace(workspace, lib.qgt_cnn_jacobian_workspace_bytes(ctypes.byref(d), n_s), x.device)
    _check(lib.qgt_cnn_jacobian(ctypes.byref(d), ctypes.c_void_p(theta.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                x.stride(0), n_s, DTYPES[o_dtype], ctypes.c_void_p(O.data_ptr()), O.stride(0),
                                ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream_handle(stream)))
    return O


# ---------------------------------------------------------------------------
# Variational Monte Carlo (include/qgt_vmc.h)
# ---------------------------------------------------------------------------
def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def rbm_metropolis(theta, x, n_hidden, pairs, u, accepted=None, stream=None):
    """Metropolis exchange moves on the chains x (int8, n_chains x N, updated in
    place): pairs int32 (n_steps x n_chains x 2), u float64 (n_steps x n_chains)."""
    _need(x is not None and x.dim() == 2, "x must be a 2-D int8 matrix")
    n_chains, N = x.shape
    M = int(n_hidden)
    _check_spins(x, N)
    _check_vec("theta", theta, "complex128", M * N + M + N)
    _need(u is not None and u.dim() == 2 and u.shape[1] == n_chains, "u must be (n_steps, n_chains)")
    n_steps = u.shape[0]
    _check_vec("u", u, "float64", n_steps * n_chains)
    _need(pairs is not None and tuple(pairs.shape) == (n_steps, n_chains, 2),
          "pairs must be (n_steps, n_chains, 2)")
    _check_vec("pairs", pairs, "int32", n_steps * n_chains * 2)
    if accepted is not None:
        _check_vec("accepted", accepted, "int32", n_chains)
    _check_device(("theta", theta), ("x", x), ("pairs", pairs), ("u", u), ("accepted", accepted))
    _check(load().qgt_rbm_metropolis(N, int(n_hidden), _ptr(theta), _ptr(x), x.stride(0), n_chains, n_steps,
                                     _ptr(pairs), _ptr(u), _ptr(accepted), _stream_handle(stream)))
    return x


def rbm_heisenberg_eloc(theta, x, n_hidden, J=1.0, periodic=True, e_loc=None, stream=None):
    """Local energies (complex128, n_s) of the samples x for the Heisenberg chain."""
    import torch
    _need(x is not None and x.dim() == 2, "x must be a 2-D int8 matrix")
    n_s, N = x.shape
    M = int(n_hidden)
    _check_spins(x, N)
    _check_vec("theta", theta, "complex128", M * N + M + N)
    if e_loc is not None:
        _check_vec("e_loc", e_loc, "complex128", n_s)
    _check_device(("theta", theta), ("x", x), ("e_loc", e_loc))
    if e_loc is None:
        e_loc = torch.empty(n_s, dtype=torch.complex128, device=x.device)
    _check(load().qgt_rbm_heisenberg_eloc(N, int(n_hidden), _ptr(theta), _ptr(x), x.stride(0), n_s, float(J),
                                          1 if periodic else 0, _ptr(e_loc), _stream_handle(stream)))
    return e_loc


def sr_update(theta, delta, eta, stream=None):
    """theta <- theta - eta delta (complex128 device tensors)."""
    _need(theta is not None, "theta is missing")
    _check_vec("theta", theta, "complex128", theta.numel())
    _check_vec("delta", delta, "complex128", theta.numel())
    _check_device(("theta", theta), ("delta", delta))
    _check(load().qgt_sr_update(_ptr(theta), _ptr(delta), theta.numel(), float(eta), _stream_handle(stream)))
    return theta
