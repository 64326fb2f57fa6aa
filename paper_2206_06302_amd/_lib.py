"""ctypes declarations for libtstream (include/tstream.h).  Marshalling only."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtstream.so")

TS_OK = 0
STATUS_NAMES = {
    0: "TS_OK", -1: "TS_E_INVALID", -2: "TS_E_SHAPE", -3: "TS_E_DTYPE", -4: "TS_E_PLACEMENT",
    -5: "TS_E_ALIAS", -6: "TS_E_DEVICE", -7: "TS_E_OOM", -8: "TS_E_UNSUPPORTED",
}


class KernelCfg(ctypes.Structure):
    _fields_ = [
        ("block", ctypes.c_int32),
        ("unroll", ctypes.c_int32),
        ("vec_bytes", ctypes.c_int32),
        ("nt_load", ctypes.c_int32),
        ("nt_store", ctypes.c_int32),
        ("grid_per_cu", ctypes.c_int32),
        ("tile_elems", ctypes.c_int64),
        ("tiles_per_wg", ctypes.c_int32),
        ("record_ahead", ctypes.c_int32),
        ("wgs_per_tile", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}

    @classmethod
    def from_dict(cls, d: dict) -> "KernelCfg":
        c = cls()
        c.block = int(d.get("block", 256))
        c.unroll = int(d.get("unroll", 4))
        c.vec_bytes = int(d.get("vec_bytes", 16))
        c.nt_load = int(d.get("nt_load", 0))
        c.nt_store = int(d.get("nt_store", 1))
        c.grid_per_cu = int(d.get("grid_per_cu", 0))
        c.tile_elems = int(d.get("tile_elems", 0))
        c.tiles_per_wg = int(d.get("tiles_per_wg", 0))
        c.record_ahead = int(d.get("record_ahead", 0))
        c.wgs_per_tile = int(d.get("wgs_per_tile", 0))
        return c


class ProbeCfg(ctypes.Structure):
    _fields_ = [
        ("reads", ctypes.c_int32),
        ("writes", ctypes.c_int32),
        ("block", ctypes.c_int32),
        ("unroll", ctypes.c_int32),
        ("nt_load", ctypes.c_int32),
        ("nt_store", ctypes.c_int32),
        ("wave_contiguous", ctypes.c_int32),
        ("lds_bytes", ctypes.c_int32),
        ("vec_bytes", ctypes.c_int32),
    ]

    @classmethod
    def from_dict(cls, d: dict) -> "ProbeCfg":
        c = cls()
        for f, _ in cls._fields_:
            setattr(c, f, int(d.get(f, 0)))
        return c


class DeviceInfo(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int),
        ("compute_units", ctypes.c_int),
        ("wavefront_size", ctypes.c_int),
        ("max_threads_per_block", ctypes.c_int),
        ("clock_khz", ctypes.c_int),
        ("memory_clock_khz", ctypes.c_int),
        ("memory_bus_width_bits", ctypes.c_int),
        ("hbm_bytes", ctypes.c_uint64),
        ("l2_bytes", ctypes.c_uint64),
        ("peak_bytes_per_s", ctypes.c_double),
        ("arch", ctypes.c_char * 64),
        ("name", ctypes.c_char * 128),
    ]


class ChecksumOut(ctypes.Structure):
    _fields_ = [
        ("sum", ctypes.c_double),
        ("abs_dev_sum", ctypes.c_double),
        ("max_abs_dev", ctypes.c_double),
        ("mismatches", ctypes.c_uint64),
    ]


class BatchDescC(ctypes.Structure):
    _fields_ = [
        ("a", ctypes.c_void_p),
        ("b", ctypes.c_void_p),
        ("c", ctypes.c_void_p),
        ("len", ctypes.c_uint64),
        ("q", ctypes.c_double),
    ]


H = ctypes.c_void_p  # every handle is an opaque pointer
P = ctypes.c_void_p
I = ctypes.c_int
SZ = ctypes.c_size_t
U64 = ctypes.c_uint64
I64 = ctypes.c_int64
D = ctypes.c_double
F = ctypes.c_float
CALLBACK = ctypes.CFUNCTYPE(None, ctypes.c_void_p)

# name -> argument types (every function returns int unless listed in RESTYPES)
PROTOTYPES = {
    "ts_last_error": [],
    "ts_version": [ctypes.POINTER(I), ctypes.POINTER(I)],
    "ts_target_create": [I, P, ctypes.POINTER(H)],
    "ts_target_create_owned": [I, ctypes.POINTER(H)],
    "ts_target_create_host": [ctypes.POINTER(I), I, ctypes.POINTER(H)],
    "ts_host_numa_domains": [ctypes.POINTER(I)],
    "ts_host_domain_cpus": [I, ctypes.POINTER(I), I, ctypes.POINTER(I)],
    "ts_target_destroy": [H],
    "ts_target_synchronize": [H],
    "ts_target_info": [H, ctypes.POINTER(DeviceInfo)],
    "ts_target_stream": [H, ctypes.POINTER(P)],
    "ts_target_then": [H, CALLBACK, P],
    "ts_array_alloc": [H, I, SZ, SZ, ctypes.POINTER(H)],
    "ts_array_wrap": [H, I, P, SZ, ctypes.POINTER(H)],
    "ts_array_free": [H],
    "ts_array_info": [H, ctypes.POINTER(P), ctypes.POINTER(SZ), ctypes.POINTER(I)],
    "ts_fill": [H, D],
    "ts_fill_uniform": [H, U64, U64, U64],
    "ts_fill_uniform_range": [H, U64, U64, U64, D, D],
    "ts_copy_from_host": [H, P, SZ],
    "ts_copy_to_host": [P, H, SZ],
    "ts_copy": [H, H, H],
    "ts_scale": [H, H, H, D],
    "ts_add": [H, H, H, H],
    "ts_triad": [H, H, H, H, D],
    "ts_stream_iteration": [H, H, H, H, D],
    "ts_checksum": [H, H, D, ctypes.POINTER(ChecksumOut)],
    "ts_checksum_noalloc": [H, H, D, ctypes.c_void_p],
    "ts_mismatch_count": [H, H, H, ctypes.POINTER(U64)],
    "ts_get_kernel_cfg": [I, I, SZ, I, I, ctypes.POINTER(KernelCfg)],
    "ts_set_kernel_cfg": [I, I, I, ctypes.POINTER(KernelCfg)],
    "ts_autotune_candidates": [I, ctypes.POINTER(KernelCfg), SZ, ctypes.POINTER(SZ)],
    "ts_autotune": [H, I, I, SZ, SZ, I, ctypes.POINTER(KernelCfg), ctypes.POINTER(D)],
    "ts_autotune_batch": [H, H, I, I, ctypes.POINTER(KernelCfg), ctypes.POINTER(D)],
    "ts_tune_cache_load": [ctypes.c_char_p],
    "ts_tune_cache_save": [ctypes.c_char_p],
    "ts_tune_cache_clear": [],
    "ts_time_op": [H, I, H, H, H, D, I, ctypes.POINTER(F)],
    "ts_probe_bandwidth": [H, ctypes.POINTER(ProbeCfg), H, H, H, SZ, ctypes.c_uint32],
    "ts_batch_create": [H, I, ctypes.POINTER(BatchDescC), SZ, ctypes.POINTER(H)],
    "ts_batch_destroy": [H],
    "ts_batch_info": [H, ctypes.POINTER(SZ), ctypes.POINTER(U64), ctypes.POINTER(U64), ctypes.POINTER(I64)],
    "ts_batch_set_tile": [H, I64],
    "ts_batch_op": [H, H, I],
    "ts_batch_op_plain": [H, H, I],
    "ts_batch_fill": [H, H, I, D],
    "ts_batch_fill_uniform": [H, H, I, U64],
    "ts_batch_mismatch_count": [H, H, I, P, P],
    "ts_graph_capture_stream_iteration": [H, H, ctypes.POINTER(H)],
    "ts_graph_capture_batch_op": [H, H, I, ctypes.POINTER(H)],
    "ts_graph_capture_arrays_iteration": [H, H, H, H, D, ctypes.POINTER(H)],
    "ts_graph_capture_arrays_iterations": [H, H, H, H, D, I, ctypes.POINTER(H)],
    "ts_graph_capture_stream_iterations": [H, H, I, ctypes.POINTER(H)],
    "ts_graph_launch": [H, H, I],
    "ts_graph_destroy": [H],
    "ts_event_create": [ctypes.POINTER(H)],
    "ts_event_create_timing": [ctypes.POINTER(H)],
    "ts_event_destroy": [H],
    "ts_event_record": [H, H],
    "ts_event_synchronize": [H],
    "ts_event_query": [H],
    "ts_event_elapsed_ms": [H, H, ctypes.POINTER(F)],
    "ts_target_async": [H, ctypes.POINTER(H)],
    "ts_future_wait": [H],
    "ts_future_ready": [H],
    "ts_future_destroy": [H],
    "ts_transform_create": [H, ctypes.c_char_p, I, I, ctypes.POINTER(H)],
    "ts_transform_apply": [H, H, H, H, H, D],
    "ts_transform_log": [H, ctypes.POINTER(ctypes.c_char_p)],
    "ts_transform_destroy": [H],
}
RESTYPES = {"ts_last_error": ctypes.c_char_p}


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(
            f"libtstream.so not found at {path}; build it with "
            "`python paper_2206_06302_amd/build.py` (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    for name, args in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = RESTYPES.get(name, ctypes.c_int)
    return lib


def hip_runtimes_loaded() -> list[str]:
    """Distinct libamdhip64 files mapped into this process."""
    found = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                parts = line.split()
                if len(parts) >= 6 and "libamdhip64" in parts[-1]:
                    found.add(os.path.realpath(parts[-1]))
    except OSError:
        pass
    return sorted(found)
