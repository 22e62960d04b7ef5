"""ctypes declarations of the C ABI in include/alto.h (argument marshalling only)."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libalto_mi355x.so")

MAX_MODES = 8
MAX_RANK = 128

OK = 0
ERR_ARG = 1
ERR_COORD_RANGE = 2
ERR_INDEX_BITS = 3
ERR_OOM = 4
ERR_HIP = 5
ERR_NOT_SPD = 6
ERR_STATE = 7
ERR_BUDGET = 8

STATUS_NAMES = {
    0: "ALTO_OK", 1: "ALTO_ERR_ARG", 2: "ALTO_ERR_COORD_RANGE", 3: "ALTO_ERR_INDEX_BITS", 4: "ALTO_ERR_OOM",
    5: "ALTO_ERR_HIP", 6: "ALTO_ERR_NOT_SPD", 7: "ALTO_ERR_STATE", 8: "ALTO_ERR_BUDGET",
}

F32 = 0
BF16 = 1

CR_AUTO = 0
CR_TILE = 1
CR_RUN = 2
CR_DIRECT = 3
CR_HOT = 4

ACC_DEFAULT = 0
ACC_F64 = 1
ACC_F32 = 2
ACC_XCD_F32 = 3
ACC_XCD_F64 = 4

ORDER_DEFAULT = 0
ORDER_CONTIGUOUS = 1
ORDER_INTERLEAVED = 2


class MttkrpPlan(ctypes.Structure):
    _fields_ = [
        ("conflict", ctypes.c_int),
        ("tile_nnz", ctypes.c_int),
        ("block_threads", ctypes.c_int),
        ("table_slots", ctypes.c_int),
        ("accumulate", ctypes.c_int),
        ("rank_tile", ctypes.c_int),
        ("tile_order", ctypes.c_int),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class CpaprParams(ctypes.Structure):
    _fields_ = [
        ("k_max", ctypes.c_int),
        ("l_max", ctypes.c_int),
        ("tau", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("kappa_tol", ctypes.c_double),
        ("eps", ctypes.c_float),
        ("pi_form", ctypes.c_int),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("nmodes", ctypes.c_int),
        ("index_bits", ctypes.c_int),
        ("index_words", ctypes.c_int),
        ("nbits", ctypes.c_int * MAX_MODES),
        ("dims", ctypes.c_uint64 * MAX_MODES),
        ("mask_lo", ctypes.c_uint64 * MAX_MODES),
        ("mask_hi", ctypes.c_uint64 * MAX_MODES),
        ("nnz", ctypes.c_uint64),
        ("device_bytes", ctypes.c_uint64),
    ]

    def as_dict(self):
        n = self.nmodes
        return dict(
            nmodes=n,
            index_bits=self.index_bits,
            index_words=self.index_words,
            nbits=list(self.nbits[:n]),
            dims=list(self.dims[:n]),
            masks=[int(self.mask_lo[k]) | (int(self.mask_hi[k]) << 64) for k in range(n)],
            nnz=int(self.nnz),
            device_bytes=int(self.device_bytes),
        )


class ServeJob(ctypes.Structure):
    _fields_ = [
        ("nmodes", ctypes.c_int),
        ("rank", ctypes.c_int),
        ("sweeps", ctypes.c_int),
        ("fdt", ctypes.c_int),
        ("dims", ctypes.c_uint64 * MAX_MODES),
        ("nnz", ctypes.c_uint64),
        ("coords", ctypes.c_void_p * MAX_MODES),
        ("vals", ctypes.c_void_p),
        ("factors", ctypes.c_void_p * MAX_MODES),
        ("lambda_out", ctypes.c_void_p),
        ("user_tag", ctypes.c_uint64),
    ]


class ServeStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "submitted", "admitted", "completed", "rejected", "active", "queued", "bytes_in_use", "bytes_peak",
        "sweeps_done", "nnz_modes_done", "rounds")]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class ServeDone(ctypes.Structure):
    _fields_ = [
        ("user_tag", ctypes.c_uint64),
        ("status", ctypes.c_int),
        ("sweeps", ctypes.c_int),
        ("submit_s", ctypes.c_double),
        ("admit_s", ctypes.c_double),
        ("done_s", ctypes.c_double),
        ("sweep_ms_sum", ctypes.c_double),
        ("sweep_ms_max", ctypes.c_double),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


P = ctypes.c_void_p
I32 = ctypes.c_int
U64 = ctypes.c_uint64
I64 = ctypes.c_int64

# name -> (restype, argtypes); every symbol include/alto.h declares
SIGNATURES = {
    "alto_plan_dims": (I32, [I32, P, ctypes.POINTER(Info)]),
    "alto_plan_decode_host": (I32, [ctypes.POINTER(Info), U64, P, P]),
    "alto_build": (I32, [I32, P, U64, P, P, P, ctypes.POINTER(P)]),
    "alto_info": (I32, [P, ctypes.POINTER(Info)]),
    "alto_export": (I32, [P, P, P, P]),
    "alto_decode": (I32, [P, U64, P, P, P]),
    "alto_partition": (I32, [P, I64, P, P, P]),
    "alto_free": (I32, [P]),
    "alto_mttkrp": (I32, [P, I32, I32, I32, P, P, P]),
    "alto_mttkrp_ex": (I32, [P, I32, I32, I32, P, P, ctypes.POINTER(MttkrpPlan), P]),
    "alto_mttkrp_get_plan": (I32, [P, I32, I32, I32, ctypes.POINTER(MttkrpPlan)]),
    "alto_mttkrp_noalloc": (I32, [P, I32, I32, I32, P, P, ctypes.POINTER(MttkrpPlan), P]),
    "alto_autotune": (I32, [P, I32, I32, I32, P, P, P, ctypes.POINTER(MttkrpPlan)]),
    "alto_mttkrp_batched": (I32, [I32, P, P, P, P, P, P, P]),
    "cpd_als_sweep": (I32, [P, I32, P, P, P]),
    "cpd_als_sweep_ex": (I32, [P, I32, I32, P, P, P]),
    "alto_sweep_flags": (I32, [P, P, ctypes.POINTER(ctypes.c_uint32)]),
    "alto_tensor_norm2": (I32, [P, ctypes.POINTER(ctypes.c_double), P]),
    "alto_cpapr_phi": (I32, [P, I32, I32, P, P, ctypes.c_float, P, P, ctypes.POINTER(MttkrpPlan), P]),
    "alto_cpapr_pi": (I32, [P, I32, I32, P, P, P]),
    "alto_cpapr_prefer_pre": (I32, [P, I32, I32, ctypes.POINTER(I32)]),
    "alto_cp_fit": (I32, [P, I32, I32, P, P, ctypes.POINTER(ctypes.c_double), P]),
    "cpd_als": (I32, [P, I32, I32, P, P, I32, ctypes.c_double, P, ctypes.POINTER(I32), P]),
    "cpd_als_sweep_batched": (I32, [I32, P, P, P, P, P, P]),
    "alto_sweep_batch_create": (I32, [I32, P, P, P, P, P, P, ctypes.POINTER(P)]),
    "alto_cpapr_mu": (I32, [P, I32, P, P, ctypes.POINTER(CpaprParams), ctypes.POINTER(I32), P,
                            ctypes.POINTER(I32), P]),
    "alto_sweep_batch_run": (I32, [P, P]),
    "alto_sweep_batch_destroy": (I32, [P]),
    "alto_server_create": (I32, [U64, I32, ctypes.POINTER(P)]),
    "alto_server_submit": (I32, [P, ctypes.POINTER(ServeJob)]),
    "alto_server_poll": (I32, [P, P, I32, ctypes.POINTER(I32)]),
    "alto_server_stats": (I32, [P, ctypes.POINTER(ServeStats)]),
    "alto_server_drain": (I32, [P]),
    "alto_server_sweep_latencies": (I32, [P, P, U64, ctypes.POINTER(U64)]),
    "alto_server_destroy": (I32, [P]),
    "alto_serve_footprint": (I32, [ctypes.POINTER(ServeJob), ctypes.POINTER(U64)]),
    "alto_timing_enable": (I32, [I32]),
    "alto_timing_read": (I32, [ctypes.POINTER(U64), ctypes.POINTER(ctypes.c_double)]),
    "alto_release_cached_memory": (I32, []),
    "alto_last_error": (ctypes.c_char_p, []),
    "alto_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load the in-tree HIP library; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
            )
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_symbols(path: str | None = None):
    """Function names declared in include/alto.h."""
    import re

    path = path or os.path.join(os.path.dirname(HERE), "include", "alto.h")
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(alto_\w+|cpd_\w+)\s*\(", text)))
