"""ctypes binding of libfwapsp.so: the C ABI of include/fw_apsp.h, same names.

Argument marshalling only.  Every step of the computation runs in the HIP
library; if the library is missing this module raises instead of falling back.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfwapsp.so")

FW_F32, FW_F64, FW_F16 = 0, 1, 2
FW_OK, FW_EINVAL, FW_ENOMEM, FW_EHIP, FW_EUNSUPPORTED, FW_EINPUT = 0, -1, -2, -3, -4, -5
FW_P4_PANELS, FW_P4_WAVEROWS = 1, 2
FW_SCHED_SERIAL, FW_SCHED_LOOKAHEAD, FW_SCHED_PAIRS, FW_SCHED_PAIRS_LOOKAHEAD = 1, 2, 3, 4

EXPORTS = ("fw_apsp", "fw_apsp_config", "fw_query_config", "fw_list_configs", "fw_apsp_ooc", "fw_ooc_superblock",
           "fw_apsp_batched", "fw_apsp_batched_config", "fw_apsp_batched_device", "fw_apsp_batched_device_noalloc",
           "fw_apsp_backward",
           "fw_status_string", "fw_last_error", "fw_version", "fw_prof_enable", "fw_prof_read",
           "fw_debug_fail_next", "fw_validate_input")


class FwConfig(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("tile_m", ctypes.c_int32),
                ("tile_n", ctypes.c_int32), ("variant", ctypes.c_int32), ("schedule", ctypes.c_int32)]


class FwBatchedConfig(ctypes.Structure):
    _fields_ = [("small_max_n", ctypes.c_int32), ("route", ctypes.c_int32),
                ("reserved1", ctypes.c_int32), ("reserved2", ctypes.c_int32)]


class FwError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where} failed with status {status}: {detail}")
        self.status = status


_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    L.fw_apsp.argtypes = [ctypes.c_int, i64, vp, vp, vp]
    L.fw_apsp_config.argtypes = [ctypes.c_int, i64, vp, vp, ctypes.POINTER(FwConfig), vp]
    L.fw_query_config.argtypes = [ctypes.c_int, i64, i32, ctypes.POINTER(FwConfig)]
    L.fw_query_config.restype = ctypes.c_int
    L.fw_apsp_ooc.argtypes = [ctypes.c_int, i64, vp, vp, ctypes.c_size_t, vp]
    L.fw_apsp_ooc.restype = ctypes.c_int
    L.fw_ooc_superblock.argtypes = [ctypes.c_int, i64, i32, ctypes.c_size_t]
    L.fw_ooc_superblock.restype = i64
    L.fw_list_configs.argtypes = [ctypes.c_int, ctypes.POINTER(FwConfig), i32]
    L.fw_list_configs.restype = ctypes.c_int32
    L.fw_apsp_batched.argtypes = [ctypes.c_int, i32, vp, vp, vp, vp, vp]
    L.fw_apsp_batched_config.argtypes = [ctypes.c_int, i32, vp, vp, vp, vp, ctypes.POINTER(FwBatchedConfig), vp]
    L.fw_apsp_backward.argtypes = [ctypes.c_int, i64, i32, vp, vp, vp, vp, vp]
    L.fw_apsp_batched_device.argtypes = [ctypes.c_int, i32, vp, vp, vp, vp, vp]
    L.fw_apsp_batched_device_noalloc.argtypes = [ctypes.c_int, i32, vp, vp, vp, vp, vp]
    for f in ("fw_apsp", "fw_apsp_config", "fw_apsp_batched", "fw_apsp_batched_config", "fw_apsp_backward",
              "fw_apsp_batched_device", "fw_apsp_batched_device_noalloc"):
        getattr(L, f).restype = ctypes.c_int
    L.fw_status_string.argtypes = [ctypes.c_int]
    L.fw_status_string.restype = ctypes.c_char_p
    L.fw_last_error.restype = ctypes.c_char_p
    L.fw_version.restype = ctypes.c_char_p
    L.fw_prof_enable.argtypes = [ctypes.c_int]
    L.fw_prof_read.argtypes = [ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), ctypes.c_int]
    L.fw_prof_read.restype = ctypes.c_int
    L.fw_validate_input.argtypes = [ctypes.c_int, i64, vp, vp]
    L.fw_validate_input.restype = ctypes.c_int
    L.fw_debug_fail_next.argtypes = [ctypes.c_int]
    L.fw_debug_fail_next.restype = None
    _lib = L
    return L


def _check(st: int, where: str):
    if st != FW_OK:
        L = lib()
        raise FwError(st, where, f"{L.fw_status_string(st).decode()}: {L.fw_last_error().decode()}")


def fw_apsp(dt: int, n: int, dist: int, path: int | None, stream: int | None = None):
    _check(lib().fw_apsp(dt, n, dist, path, stream), "fw_apsp")


def fw_apsp_config(dt, n, dist, path, block=0, tile_m=0, tile_n=0, variant=0, schedule=0, stream=None):
    cfg = FwConfig(block, tile_m, tile_n, variant, schedule)
    _check(lib().fw_apsp_config(dt, n, dist, path, ctypes.byref(cfg), stream), "fw_apsp_config")


def fw_query_config(dt: int, n: int, path: bool):
    """(block, tile_m, tile_n, variant, schedule) that fw_apsp uses for this case (the tuned table)."""
    cfg = FwConfig(0, 0, 0, 0, 0)
    _check(lib().fw_query_config(dt, n, 1 if path else 0, ctypes.byref(cfg)), "fw_query_config")
    return int(cfg.block), int(cfg.tile_m), int(cfg.tile_n), int(cfg.variant), int(cfg.schedule)


def fw_list_configs(dt: int):
    """Every compiled (block, tile_m, tile_n, variant) for dtype code dt (any schedule applies)."""
    L = lib()
    count = L.fw_list_configs(dt, None, 0)
    if count < 0:
        _check(count, "fw_list_configs")
    arr = (FwConfig * count)()
    L.fw_list_configs(dt, arr, count)
    return [(int(c.block), int(c.tile_m), int(c.tile_n), int(c.variant)) for c in arr]


def fw_apsp_ooc(dt, n, dist_host, path_host=None, device_bytes=0, stream=None):
    """dist_host, path_host: host pointers (n*n elements; path_host may be None);
    blocks until the results are there."""
    _check(lib().fw_apsp_ooc(dt, n, dist_host, path_host, device_bytes, stream), "fw_apsp_ooc")


def fw_ooc_superblock(dt, n, path=False, device_bytes=0) -> int:
    s = lib().fw_ooc_superblock(dt, n, 1 if path else 0, device_bytes)
    if s < 0:
        _check(int(s), "fw_ooc_superblock")
    return int(s)


def fw_apsp_batched(dt, batch, n_host, off_host, dist, path, stream=None):
    """n_host / off_host: host pointers (e.g. numpy .ctypes.data)."""
    _check(lib().fw_apsp_batched(dt, batch, n_host, off_host, dist, path, stream), "fw_apsp_batched")


def fw_apsp_batched_config(dt, batch, n_host, off_host, dist, path, small_max_n=-1, stream=None, route=0):
    cfg = FwBatchedConfig(small_max_n, route, 0, 0)
    _check(lib().fw_apsp_batched_config(dt, batch, n_host, off_host, dist, path, ctypes.byref(cfg), stream),
           "fw_apsp_batched_config")


def fw_apsp_batched_device(dt, batch, n_dev, off_dev, dist, path, stream=None):
    """n_dev / off_dev: device pointers (int32 counts, int64 offsets)."""
    _check(lib().fw_apsp_batched_device(dt, batch, n_dev, off_dev, dist, path, stream), "fw_apsp_batched_device")


def fw_apsp_batched_device_noalloc(dt, batch, n_dev, off_dev, dist, path, stream=None):
    """As fw_apsp_batched_device, with the library's static job table (no allocation)."""
    _check(lib().fw_apsp_batched_device_noalloc(dt, batch, n_dev, off_dev, dist, path, stream),
           "fw_apsp_batched_device_noalloc")


def fw_apsp_backward(dt, n, batch, dist, path, grad_dist, grad_w, stream=None):
    _check(lib().fw_apsp_backward(dt, n, batch, dist, path, grad_dist, grad_w, stream), "fw_apsp_backward")


def fw_validate_input(dt, n, dist, stream=None):
    """Raises FwError (status FW_EINPUT) when the matrix breaks the input contract."""
    _check(lib().fw_validate_input(dt, n, dist, stream), "fw_validate_input")


def fw_status_string(st: int) -> str:
    return lib().fw_status_string(st).decode()


def fw_last_error() -> str:
    return lib().fw_last_error().decode()


def fw_version() -> str:
    return lib().fw_version().decode()


def fw_prof_enable(on: bool):
    lib().fw_prof_enable(1 if on else 0)


def fw_prof_read(reset: bool = True):
    """(count, total_ms, updates) of bracketed last-phase launches since the last reset."""
    c = ctypes.c_int64(0)
    t = ctypes.c_double(0.0)
    u = ctypes.c_int64(0)
    _check(lib().fw_prof_read(ctypes.byref(c), ctypes.byref(t), ctypes.byref(u), 1 if reset else 0),
           "fw_prof_read")
    return int(c.value), float(t.value), int(u.value)


def lookahead_applies(block: int, tile_m: int, tile_n: int, n: int) -> bool:
    """Whether FW_SCHED_LOOKAHEAD changes anything for this configuration (else it runs serially):
    tiles one block wide and at most one block tall, and at least 3 rounds after padding."""
    unit = max(block, tile_m, tile_n)
    npad = -(-n // unit) * unit
    return tile_n == block and block % tile_m == 0 and npad // block >= 3


def pairs_applies(block: int, tile_m: int, tile_n: int, variant: int, n: int) -> bool:
    """Whether FW_SCHED_PAIRS changes anything for this configuration (else it runs serially):
    LDS-panel tiles exactly one block square and at least 2 rounds after padding."""
    unit = max(block, tile_m, tile_n)
    npad = -(-n // unit) * unit
    return variant == FW_P4_PANELS and tile_m == block and tile_n == block and npad // block >= 2


def pairs_lookahead_applies(block: int, tile_m: int, tile_n: int, variant: int, n: int) -> bool:
    """Whether FW_SCHED_PAIRS_LOOKAHEAD changes anything (else it runs serially): the
    pairs tiles and at least 3 rounds after padding."""
    unit = max(block, tile_m, tile_n)
    npad = -(-n // unit) * unit
    return pairs_applies(block, tile_m, tile_n, variant, n) and npad // block >= 3
