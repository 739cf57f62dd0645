"""ctypes binding of libbds (include/bds.h): argument marshalling only.

Every step of the solver runs in the HIP library; this module loads
``_lib/libbds.so`` and declares the C signatures.  It raises if the library
has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libbds.so")

BDS_OK, BDS_EINVAL, BDS_ENOTSPD, BDS_ENOCONV, BDS_EWORKSPACE, BDS_EHIP = range(6)
STATUS_NAMES = {0: "BDS_OK", 1: "BDS_EINVAL", 2: "BDS_ENOTSPD", 3: "BDS_ENOCONV", 4: "BDS_EWORKSPACE",
                5: "BDS_EHIP"}
BDS_F64, BDS_F32, BDS_BF16 = 0, 1, 2

# Every function declared in include/bds.h.
EXPORTS = ("bds_workspace_size", "bds_factor", "bds_solve", "bds_backward", "bds_batched_workspace_size",
           "bds_factor_batched", "bds_solve_batched", "bds_tune_workspace_size", "bds_tune", "bds_tune_batched",
           "bds_trace_enable", "bds_trace_read", "bds_version")

# Tile shape codes of bds_desc.tiles (BDS_TILE_*) and the field packing of BDS_TILES.
BDS_TILE_RULE, BDS_TILE_W16, BDS_TILE_W32, BDS_TILE_G64, BDS_TILE_G128 = range(5)
TILE_NAMES = {0: "rule", 1: "w16", 2: "w32", 3: "g64", 4: "g128"}


def tiles(couple: int = 0, schur: int = 0, solve: int = 0) -> int:
    """BDS_TILES(couple, schur, solve)."""
    return int(couple) | (int(schur) << 4) | (int(solve) << 8)


def tiles_fields(t: int) -> dict:
    """{"couple": name, "schur": name, "solve": name} of a bds_desc.tiles value."""
    return {k: TILE_NAMES.get((int(t) >> (4 * i)) & 15, "?") for i, k in enumerate(("couple", "schur", "solve"))}


class BdsDesc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("n", ctypes.c_int64), ("d", ctypes.c_int64),
                ("prec", ctypes.c_int32), ("nstar", ctypes.c_int32), ("max_refine", ctypes.c_int32),
                ("tiles", ctypes.c_int32), ("refine_tol", ctypes.c_double)]


class BdsInfo(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in ("status", "level", "position", "orig_block", "column", "iters",
                                              "converged", "reserved")]


_lib = None


def load():
    """Load libbds.so; raises RuntimeError if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2509_03015_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, S, I64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64
    D = ctypes.POINTER(BdsDesc)
    PS = ctypes.POINTER(ctypes.c_size_t)
    lib.bds_workspace_size.argtypes = [D, PS, PS]
    lib.bds_factor.argtypes = [D, P, P, P, S, P, P]
    lib.bds_solve.argtypes = [D, P, S, P, P, P, P, P, S, P, P]
    lib.bds_backward.argtypes = [D, P, S, P, P, P, P, P, P, P, P, S, P, P]
    lib.bds_factor_batched.argtypes = [I64, P, P, P, P, S, P, P]
    lib.bds_solve_batched.argtypes = [I64, P, P, S, P, P, P, P, P, S, P, P]
    lib.bds_batched_workspace_size.argtypes = [I64, P, PS, PS]
    lib.bds_tune_workspace_size.argtypes = [D, PS, PS]
    lib.bds_tune.argtypes = [D, P, P, P, P, P, S, P, S, P, ctypes.c_int, P, D]
    lib.bds_tune_batched.argtypes = [I64, P, P, P, P, P, P, S, P, S, P, ctypes.c_int, P, P]
    lib.bds_trace_enable.argtypes = [I64]
    lib.bds_trace_read.argtypes = [I64, P, P, P, P, P]
    for f in EXPORTS[:-1]:
        getattr(lib, f).restype = ctypes.c_int
    lib.bds_version.argtypes = []
    lib.bds_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def trace_enable(max_launches: int):
    rc = load().bds_trace_enable(int(max_launches))
    if rc != BDS_OK:
        raise RuntimeError(f"bds_trace_enable: {STATUS_NAMES.get(rc, rc)}")


def trace_read(max_kernels: int = 64):
    """Per-kernel (launches, total_ms) of the timed launches since the last read, and the dropped count."""
    names = ctypes.create_string_buffer(64 * max_kernels)
    launches = (ctypes.c_int64 * max_kernels)()
    total = (ctypes.c_double * max_kernels)()
    nk = ctypes.c_int64(0)
    dropped = ctypes.c_int64(0)
    rc = load().bds_trace_read(max_kernels, names, launches, total, ctypes.byref(nk), ctypes.byref(dropped))
    if rc != BDS_OK:
        raise RuntimeError(f"bds_trace_read: {STATUS_NAMES.get(rc, rc)}")
    out = {}
    for k in range(min(nk.value, max_kernels)):
        name = names.raw[64 * k: 64 * (k + 1)].split(b"\0", 1)[0].decode()
        out[name] = (int(launches[k]), float(total[k]))
    return out, int(dropped.value)


def workspace_size(desc: BdsDesc):
    f = ctypes.c_size_t(0)
    s = ctypes.c_size_t(0)
    rc = load().bds_workspace_size(ctypes.byref(desc), ctypes.byref(f), ctypes.byref(s))
    return rc, f.value, s.value


def tune_workspace_size(desc: BdsDesc):
    f = ctypes.c_size_t(0)
    s = ctypes.c_size_t(0)
    rc = load().bds_tune_workspace_size(ctypes.byref(desc), ctypes.byref(f), ctypes.byref(s))
    return rc, f.value, s.value
