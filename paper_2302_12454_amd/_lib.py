"""ctypes declarations of the C ABI in include/ssqa.h (libssqa.so, built in-tree)."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libssqa.so")

c_int32_p = ctypes.POINTER(ctypes.c_int32)
c_int64_p = ctypes.POINTER(ctypes.c_int64)
c_uint32_p = ctypes.POINTER(ctypes.c_uint32)
c_uint8_p = ctypes.POINTER(ctypes.c_uint8)


class AnnealState(ctypes.Structure):
    _fields_ = [
        ("counters", ctypes.c_void_p),
        ("history", ctypes.c_void_p),
    ]


class AnnealParams(ctypes.Structure):
    _fields_ = [
        ("replicas", ctypes.c_int32),
        ("trials", ctypes.c_int32),
        ("cycles", ctypes.c_int32),
        ("delay", ctypes.c_int32),
        ("alpha", ctypes.c_int32),
        ("noise_amp", ctypes.c_int32),
        ("coupling_mode", ctypes.c_int32),
        ("cycles_per_launch", ctypes.c_int32),
        ("jperp", c_int32_p),
        ("i0", c_int32_p),
        ("seed", ctypes.c_uint64),
        ("target_energy", ctypes.c_int64),
        ("block_columns", ctypes.c_int32),
        ("operand_format", ctypes.c_int32),
        ("start_cycle", ctypes.c_int32),
        ("stop_cycle", ctypes.c_int32),
        ("resume", ctypes.POINTER(AnnealState)),
        ("split_rows", ctypes.c_int32),
    ]


class AnnealOutputs(ctypes.Structure):
    _fields_ = [
        ("best_energy", ctypes.c_void_p),
        ("first_hit", ctypes.c_void_p),
        ("energy_trace", ctypes.c_void_p),
        ("final_is", ctypes.c_void_p),
        ("checkpoint", ctypes.POINTER(AnnealState)),
    ]


class SAParams(ctypes.Structure):
    _fields_ = [
        ("trials", ctypes.c_int32),
        ("cycles", ctypes.c_int32),
        ("beta", ctypes.POINTER(ctypes.c_double)),
        ("seed", ctypes.c_uint64),
        ("target_energy", ctypes.c_int64),
    ]


class SAOutputs(ctypes.Structure):
    _fields_ = [
        ("best_energy", ctypes.c_void_p),
        ("first_hit", ctypes.c_void_p),
        ("final_energy", ctypes.c_void_p),
        ("final_spins", ctypes.c_void_p),
        ("energy_trace", ctypes.c_void_p),
    ]


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int32),
        ("cycles_per_step", ctypes.c_int32),
        ("max_active", ctypes.c_int32),
        ("memory_budget", ctypes.c_int64),
        ("split_rows", ctypes.c_int32),
    ]


class Request(ctypes.Structure):
    _fields_ = [
        ("n_spins", ctypes.c_int32),
        ("h", c_int32_p),
        ("J", c_int32_p),
        ("params", AnnealParams),
        ("early_exit", ctypes.c_int32),
    ]


class RequestInfo(ctypes.Structure):
    _fields_ = [
        ("state", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("cycles_done", ctypes.c_int32),
        ("trials", ctypes.c_int32),
        ("submit_s", ctypes.c_double),
        ("admit_s", ctypes.c_double),
        ("done_s", ctypes.c_double),
        ("memory_bytes", ctypes.c_int64),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("queued", ctypes.c_int32),
        ("active", ctypes.c_int32),
        ("memory_in_use", ctypes.c_int64),
        ("spin_updates", ctypes.c_double),
        ("elapsed_s", ctypes.c_double),
    ]


class Tile(ctypes.Structure):
    _fields_ = [
        ("block_columns", ctypes.c_int32),
        ("trials_per_block", ctypes.c_int32),
        ("operand_format", ctypes.c_int32),
        ("blocks", ctypes.c_int32),
        ("ms_per_cycle", ctypes.c_double),
    ]


# Every symbol include/ssqa.h declares, with (restype, argtypes).
SIGNATURES = {
    "ssqa_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ssqa_last_error": (ctypes.c_char_p, []),
    "ssqa_create_problem": (ctypes.c_int, [ctypes.c_int32, c_int32_p, c_int32_p, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_void_p)]),
    "ssqa_destroy_problem": (None, [ctypes.c_void_p]),
    "ssqa_problem_spins": (ctypes.c_int32, [ctypes.c_void_p]),
    "ssqa_problem_planes": (ctypes.c_int32, [ctypes.c_void_p]),
    "ssqa_problem_padded": (ctypes.c_int32, [ctypes.c_void_p]),
    "ssqa_problem_fp4_exact": (ctypes.c_int32, [ctypes.c_void_p]),
    "ssqa_anneal": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(AnnealParams),
                                   ctypes.POINTER(AnnealOutputs), ctypes.c_void_p]),
    "ssqa_anneal_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(AnnealParams),
                                           ctypes.POINTER(AnnealOutputs), ctypes.c_void_p]),
    "ssqa_tune_anneal": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(AnnealParams), ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.POINTER(Tile), ctypes.c_int32, c_int32_p, ctypes.POINTER(Tile)]),
    "ssqa_tune_batch": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(AnnealParams),
                                       ctypes.c_int32, ctypes.c_void_p, c_int32_p, ctypes.POINTER(ctypes.c_double)]),
    "ssqa_tune_lookup": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(AnnealParams), ctypes.POINTER(Tile),
                                        c_int32_p]),
    "ssqa_tune_set": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(AnnealParams), ctypes.POINTER(Tile)]),
    "ssqa_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "ssqa_tune_load": (ctypes.c_int, [ctypes.c_char_p, c_int32_p]),
    "ssqa_tune_entries": (ctypes.c_int32, []),
    "ssqa_tune_clear": (None, []),
    "ssqa_energy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_void_p]),
    "ssqa_qmc_energy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "ssqa_jperp_schedule": (ctypes.c_int, [ctypes.c_int32] * 7 + [c_int32_p]),
    "ssqa_ssa_i0_schedule": (ctypes.c_int, [ctypes.c_int32] * 6 + [c_int32_p]),
    "ssqa_gi_to_ising": (ctypes.c_int, [ctypes.c_int32, c_uint8_p, c_uint8_p, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, c_int32_p, c_int32_p, c_int64_p]),
    "ssqa_philox4x32_10": (None, [c_uint32_p, c_uint32_p, c_uint32_p]),
    "ssqa_sa_anneal": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SAParams), ctypes.POINTER(SAOutputs),
                                      ctypes.c_void_p]),
    "ssqa_sa_schedule": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_double)]),
    "ssqa_sa_accept_threshold": (ctypes.c_double, [ctypes.c_int64, ctypes.c_double]),
    "ssqa_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(AnnealParams),
                                         ctypes.POINTER(AnnealOutputs), ctypes.POINTER(ctypes.c_void_p)]),
    "ssqa_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "ssqa_batch_blocks": (ctypes.c_int32, [ctypes.c_void_p]),
    "ssqa_batch_destroy": (None, [ctypes.c_void_p]),
    "ssqa_server_create": (ctypes.c_int, [ctypes.POINTER(ServerConfig), ctypes.POINTER(ctypes.c_void_p)]),
    "ssqa_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Request), c_int64_p]),
    "ssqa_server_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, c_int32_p]),
    "ssqa_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(RequestInfo), c_int64_p,
                                        c_int32_p]),
    "ssqa_server_cancel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "ssqa_server_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerStats)]),
    "ssqa_server_destroy": (None, [ctypes.c_void_p]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libssqa.so; raises ImportError when it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
