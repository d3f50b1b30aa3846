"""Thin ctypes binding of libpaco.so, with the C ABI's names (include/paco.h).

Argument marshalling only: every step of the transform runs in the HIP
kernels of the library.  There is no fallback -- if the library is missing
the import fails loudly.  Device pointers and streams are plain integers
(e.g. ``tensor.data_ptr()`` and ``torch.cuda.current_stream().cuda_stream``).
"""
from __future__ import annotations

import ctypes
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpaco.so")

PACO_OK = 0
PACO_ERR_INVALID_ARG = 1
PACO_ERR_NOT_POWER_OF_B = 2
PACO_ERR_DIVISIBILITY = 3
PACO_ERR_UNSUPPORTED = 4
PACO_ERR_WORKSPACE = 5
PACO_ERR_ALLOC = 6
PACO_ERR_HIP = 7

PACO_C64 = 0
PACO_C64_MFMA_FP16X3 = 1
PACO_C64_MFMA_BF16X3 = 2
PACO_C64_MFMA_BF16X6 = 3

PACO_NO_TWIDDLE = 1
PACO_PACKED = 2
PACO_TWO_PASS = 4
PACO_SPLIT = 8

# paco_plan_options.flags
PACO_PLAN_MIXED = 1
PACO_PLAN_PAPER_LAYOUT = 2
PACO_PLAN_NO_SPLIT = 4
PACO_PLAN_GENERIC = 8
PACO_PLAN_NO_SYM = 16

# paco_batch_options.flags
PACO_BATCH_NO_TUNE = 1
PACO_BATCH_ONE_QUEUE = 2
PACO_BATCH_SET_GAP = 4

PACO_NOALLOC_MAX_ITEMS = 1 << 22


class PlanOptions(ctypes.Structure):
    """paco_plan_options (include/paco.h): every field 0 = the default."""
    _fields_ = [("flags", ctypes.c_uint32), ("groups1", ctypes.c_int32), ("groups3", ctypes.c_int32),
                ("cols_long", ctypes.c_int32)]


class BatchOptions(ctypes.Structure):
    """paco_batch_options (include/paco.h): every field 0 = the default."""
    _fields_ = [("flags", ctypes.c_uint32), ("spin_limit", ctypes.c_uint32), ("gap", ctypes.c_int64)]

# every symbol include/paco.h declares
EXPORTED = (
    "paco_plan_validate", "paco_plan_create", "paco_plan_validate_mixed", "paco_plan_create_mixed",
    "paco_plan_create_ex", "paco_plan_workspace_size", "paco_execute", "paco_execute_noalloc",
    "paco_execute_stage", "paco_execute_inverse", "paco_execute_two_pass", "paco_plan_has_two_pass", "paco_plan_has_split", "paco_plan_describe",
    "paco_plan_destroy", "paco_status_string",
    "paco_last_error", "paco_batch_plan_create", "paco_batch_plan_create_ex", "paco_batch_workspace_size",
    "paco_execute_batched",
    "paco_batch_plan_describe", "paco_batch_errors", "paco_batch_plan_destroy",
)


class PacoError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


def _load() -> ctypes.CDLL:
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is not built; run `python -m paper_2609_06449_amd.build`")
    # PyTorch-ROCm ships its own libamdhip64 (same soname).  Loading torch first
    # makes the dynamic linker resolve libpaco.so's HIP runtime to that copy, so
    # the process holds one HIP runtime and torch tensors/streams are valid in
    # the library.  Without torch the system ROCm runtime is used.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(_LIB_PATH)
    i64, i32, P, sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t
    st = ctypes.c_int
    sig = {
        "paco_plan_validate": (st, [i64, i64, i64, i32, st]),
        "paco_plan_create": (st, [ctypes.POINTER(P), i64, i64, i64, i32, st]),
        "paco_plan_validate_mixed": (st, [i64, i64, i64, i32, st]),
        "paco_plan_create_mixed": (st, [ctypes.POINTER(P), i64, i64, i64, i32, st]),
        "paco_plan_create_ex": (st, [ctypes.POINTER(P), i64, i64, i64, i32, st, ctypes.POINTER(PlanOptions)]),
        "paco_execute_noalloc": (st, [P, P, P, P]),
        "paco_plan_workspace_size": (st, [P, ctypes.POINTER(sz)]),
        "paco_execute": (st, [P, P, P, P, sz, P]),
        "paco_execute_stage": (st, [P, st, st, P, P, P]),
        "paco_execute_two_pass": (st, [P, P, P, P, sz, P]),
        "paco_execute_inverse": (st, [P, P, P, P, sz, P]),
        "paco_plan_has_two_pass": (st, [P, ctypes.POINTER(i32)]),
        "paco_plan_has_split": (st, [P, ctypes.POINTER(i32)]),
        "paco_plan_describe": (st, [P, ctypes.POINTER(i32), ctypes.c_char_p, sz]),
        "paco_plan_destroy": (st, [P]),
        "paco_status_string": (ctypes.c_char_p, [st]),
        "paco_last_error": (ctypes.c_char_p, []),
        "paco_batch_plan_create": (st, [ctypes.POINTER(P), i32, ctypes.POINTER(i64), st, ctypes.c_char_p]),
        "paco_batch_plan_create_ex": (st, [ctypes.POINTER(P), i32, ctypes.POINTER(i64), st, ctypes.c_char_p,
                                           ctypes.POINTER(BatchOptions)]),
        "paco_batch_workspace_size": (st, [P, ctypes.POINTER(sz)]),
        "paco_execute_batched": (st, [P, P, P, P, sz, P]),
        "paco_batch_plan_describe": (st, [P, i32, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                          ctypes.POINTER(i32), ctypes.c_char_p, sz]),
        "paco_batch_errors": (st, [P, ctypes.POINTER(ctypes.c_uint32)]),
        "paco_batch_plan_destroy": (st, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def lib() -> ctypes.CDLL:
    return _lib


def paco_status_string(status: int) -> str:
    return _lib.paco_status_string(status).decode()


def paco_last_error() -> str:
    return _lib.paco_last_error().decode()


def _check(status: int, where: str):
    if status != PACO_OK:
        raise PacoError(status, where, f"{paco_status_string(status)}: {paco_last_error()}")


def paco_plan_validate(N1: int, N2: int, p: int, b: int, dt: int = PACO_C64) -> int:
    """Returns the status code (no exception): pure host check, no GPU needed."""
    return int(_lib.paco_plan_validate(N1, N2, p, b, dt))


def paco_plan_create(N1: int, N2: int, p: int, b: int, dt: int = PACO_C64) -> int:
    h = ctypes.c_void_p()
    _check(_lib.paco_plan_create(ctypes.byref(h), N1, N2, p, b, dt), "paco_plan_create")
    return h.value


def paco_plan_validate_mixed(N1: int, N2: int, p: int, b: int, dt: int = PACO_C64) -> int:
    return int(_lib.paco_plan_validate_mixed(N1, N2, p, b, dt))


def paco_plan_create_mixed(N1: int, N2: int, p: int, b: int, dt: int = PACO_C64) -> int:
    h = ctypes.c_void_p()
    _check(_lib.paco_plan_create_mixed(ctypes.byref(h), N1, N2, p, b, dt), "paco_plan_create_mixed")
    return h.value


def paco_plan_create_ex(N1: int, N2: int, p: int, b: int, dt: int = PACO_C64, flags: int = 0, groups1: int = 0,
                        groups3: int = 0, cols_long: int = 0) -> int:
    opt = PlanOptions(flags, groups1, groups3, cols_long)
    h = ctypes.c_void_p()
    _check(_lib.paco_plan_create_ex(ctypes.byref(h), N1, N2, p, b, dt, ctypes.byref(opt)), "paco_plan_create_ex")
    return h.value


def paco_plan_create_ex_status(N1: int, N2: int, p: int, b: int, dt: int = PACO_C64, **fields) -> int:
    """Status code only (no exception); destroys the plan when one was made."""
    opt = PlanOptions(**fields)
    h = ctypes.c_void_p()
    st = int(_lib.paco_plan_create_ex(ctypes.byref(h), N1, N2, p, b, dt, ctypes.byref(opt)))
    if h.value:
        _lib.paco_plan_destroy(h)
    return st


def paco_plan_workspace_size(plan: int) -> int:
    n = ctypes.c_size_t()
    _check(_lib.paco_plan_workspace_size(plan, ctypes.byref(n)), "paco_plan_workspace_size")
    return n.value


def paco_execute(plan: int, src: int, dst: int, workspace: int, workspace_bytes: int, stream: int = 0):
    _check(_lib.paco_execute(plan, src, dst, workspace, workspace_bytes, stream), "paco_execute")


def paco_execute_noalloc(plan: int, src: int, dst: int, stream: int = 0):
    _check(_lib.paco_execute_noalloc(plan, src, dst, stream), "paco_execute_noalloc")


def paco_execute_stage(plan: int, stage: int, flags: int, src: int, dst: int, stream: int = 0):
    _check(_lib.paco_execute_stage(plan, stage, flags, src, dst, stream), "paco_execute_stage")


def paco_execute_inverse(plan: int, src: int, dst: int, workspace: int, workspace_bytes: int, stream: int = 0):
    _check(_lib.paco_execute_inverse(plan, src, dst, workspace, workspace_bytes, stream), "paco_execute_inverse")


def paco_execute_two_pass(plan: int, src: int, dst: int, workspace: int, workspace_bytes: int, stream: int = 0):
    _check(_lib.paco_execute_two_pass(plan, src, dst, workspace, workspace_bytes, stream), "paco_execute_two_pass")


def paco_plan_has_two_pass(plan: int) -> bool:
    yes = ctypes.c_int32()
    _check(_lib.paco_plan_has_two_pass(plan, ctypes.byref(yes)), "paco_plan_has_two_pass")
    return bool(yes.value)


def paco_plan_has_split(plan: int) -> int:
    """0: no split form, 1: the split form of Phase I, 2: the symmetric split form."""
    yes = ctypes.c_int32()
    _check(_lib.paco_plan_has_split(plan, ctypes.byref(yes)), "paco_plan_has_split")
    return int(yes.value)


def paco_plan_describe(plan: int):
    n = ctypes.c_int32()
    buf = ctypes.create_string_buffer(1024)
    _check(_lib.paco_plan_describe(plan, ctypes.byref(n), buf, 1024), "paco_plan_describe")
    return n.value, buf.value.decode()


def paco_plan_destroy(plan: int):
    _check(_lib.paco_plan_destroy(plan), "paco_plan_destroy")


class Plan:
    """Owns one paco_plan handle (created on the current HIP device)."""

    def __init__(self, N1: int, N2: int, p: int, b: int, dt: int = PACO_C64, mixed: bool = False, flags: int = 0,
                 groups1: int = 0, groups3: int = 0, cols_long: int = 0):
        """flags, groups1, groups3, cols_long: paco_plan_options (mixed adds
        PACO_PLAN_MIXED); all defaults: paco_plan_create."""
        self.N1, self.N2, self.p, self.b, self.dt = N1, N2, p, b, dt
        flags |= PACO_PLAN_MIXED if mixed else 0
        if flags or groups1 or groups3 or cols_long:
            self.handle = paco_plan_create_ex(N1, N2, p, b, dt, flags, groups1, groups3, cols_long)
        else:
            self.handle = paco_plan_create(N1, N2, p, b, dt)
        self.workspace_bytes = paco_plan_workspace_size(self.handle)
        self.launches, self.description = paco_plan_describe(self.handle)
        self.has_two_pass = paco_plan_has_two_pass(self.handle)
        self.has_split = paco_plan_has_split(self.handle)

    def execute(self, src: int, dst: int, workspace: int, stream: int = 0):
        paco_execute(self.handle, src, dst, workspace, self.workspace_bytes, stream)

    def execute_noalloc(self, src: int, dst: int, stream: int = 0):
        paco_execute_noalloc(self.handle, src, dst, stream)

    def execute_inverse(self, src: int, dst: int, workspace: int, stream: int = 0):
        paco_execute_inverse(self.handle, src, dst, workspace, self.workspace_bytes, stream)

    def execute_two_pass(self, src: int, dst: int, workspace: int, stream: int = 0):
        paco_execute_two_pass(self.handle, src, dst, workspace, self.workspace_bytes, stream)

    def execute_stage(self, stage: int, src: int, dst: int, stream: int = 0, flags: int = 0):
        paco_execute_stage(self.handle, stage, flags, src, dst, stream)

    def close(self):
        if self.handle:
            paco_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- batched form ----------------------------------------------------------


def paco_batch_plan_create(sizes, dt: int = PACO_C64, tune_cache_path=None) -> int:
    arr = (ctypes.c_int64 * len(sizes))(*[int(n) for n in sizes])
    h = ctypes.c_void_p()
    path = tune_cache_path.encode() if tune_cache_path is not None else None
    _check(_lib.paco_batch_plan_create(ctypes.byref(h), len(sizes), arr, dt, path), "paco_batch_plan_create")
    return h.value


def paco_batch_plan_create_ex(sizes, dt: int = PACO_C64, tune_cache_path=None, flags: int = 0,
                              spin_limit: int = 0, gap: int = 0) -> int:
    arr = (ctypes.c_int64 * len(sizes))(*[int(n) for n in sizes])
    h = ctypes.c_void_p()
    path = tune_cache_path.encode() if tune_cache_path is not None else None
    opt = BatchOptions(flags, spin_limit, gap)
    _check(_lib.paco_batch_plan_create_ex(ctypes.byref(h), len(sizes), arr, dt, path, ctypes.byref(opt)),
           "paco_batch_plan_create_ex")
    return h.value


def paco_batch_plan_create_status(sizes, dt: int = PACO_C64, tune_cache_path=None) -> int:
    """Status code only (no exception); destroys the plan when one was made."""
    arr = (ctypes.c_int64 * max(len(sizes), 1))(*[int(n) for n in sizes])
    h = ctypes.c_void_p()
    path = tune_cache_path.encode() if tune_cache_path is not None else None
    st = int(_lib.paco_batch_plan_create(ctypes.byref(h), len(sizes), arr, dt, path))
    if h.value:
        _lib.paco_batch_plan_destroy(h)
    return st


def paco_batch_workspace_size(bp: int) -> int:
    n = ctypes.c_size_t()
    _check(_lib.paco_batch_workspace_size(bp, ctypes.byref(n)), "paco_batch_workspace_size")
    return n.value


def paco_execute_batched(bp: int, src: int, dst: int, workspace: int, workspace_bytes: int, stream: int = 0):
    _check(_lib.paco_execute_batched(bp, src, dst, workspace, workspace_bytes, stream), "paco_execute_batched")


def paco_batch_plan_describe(bp: int, index: int = -1):
    n1, n2, p, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    buf = ctypes.create_string_buffer(4096)
    _check(_lib.paco_batch_plan_describe(bp, index, ctypes.byref(n1), ctypes.byref(n2), ctypes.byref(p),
                                         ctypes.byref(b), buf, 4096), "paco_batch_plan_describe")
    return (n1.value, n2.value, p.value, b.value), buf.value.decode()


def paco_batch_errors(bp: int) -> int:
    n = ctypes.c_uint32()
    _check(_lib.paco_batch_errors(bp, ctypes.byref(n)), "paco_batch_errors")
    return n.value


def paco_batch_plan_destroy(bp: int):
    _check(_lib.paco_batch_plan_destroy(bp), "paco_batch_plan_destroy")


class BatchPlan:
    """Owns one paco_batch_plan handle: transform i has sizes[i] items, packed
    back to back (offsets = running sums)."""

    def __init__(self, sizes, dt: int = PACO_C64, tune_cache_path=None, flags: int = 0, spin_limit: int = 0,
                 gap: int = 0):
        """flags, spin_limit, gap: paco_batch_options; all defaults:
        paco_batch_plan_create."""
        self.sizes = [int(n) for n in sizes]
        self.offsets = [0]
        for n in self.sizes:
            self.offsets.append(self.offsets[-1] + n)
        self.total = self.offsets[-1]
        if flags or spin_limit or gap:
            self.handle = paco_batch_plan_create_ex(self.sizes, dt, tune_cache_path, flags, spin_limit, gap)
        else:
            self.handle = paco_batch_plan_create(self.sizes, dt, tune_cache_path)
        self.workspace_bytes = paco_batch_workspace_size(self.handle)
        _, self.description = paco_batch_plan_describe(self.handle, -1)

    def transform_plan(self, i: int):
        """(N1, N2, p, b) chosen for transform i."""
        return paco_batch_plan_describe(self.handle, i)[0]

    def execute(self, src: int, dst: int, workspace: int, stream: int = 0):
        paco_execute_batched(self.handle, src, dst, workspace, self.workspace_bytes, stream)

    def errors(self) -> int:
        return paco_batch_errors(self.handle)

    def close(self):
        if self.handle:
            paco_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
