"""ctypes declarations of the C ABI in include/symphase.h (argument
marshalling only).  Loading fails loudly when the library is not built."""

from __future__ import annotations

import ctypes
import os

# torch first: it loads the HIP runtime that this library then shares
# (same soname), so streams and device pointers from torch are valid here.
import torch  # noqa: F401

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsymphase_hip.so")

SP_OK = 0
SP_E_INVALID, SP_E_PARSE, SP_E_UNSUPPORTED, SP_E_NOMEM, SP_E_DEVICE, SP_E_LIMIT = -1, -2, -3, -4, -5, -6
SP_E_BUDGET, SP_E_TIMEOUT = -7, -8
SP_REQ_QUEUED, SP_REQ_ACTIVE, SP_REQ_DONE, SP_REQ_FAILED = 0, 1, 2, 3
SP_PATH_AUTO, SP_PATH_SPARSE, SP_PATH_DENSE = 0, 1, 2
SP_SCHED_PERSISTENT, SP_SCHED_FLAT = 0, 1
SP_OUT_MEASUREMENTS, SP_OUT_DETECTORS = 0, 1
SP_INIT_AUTO, SP_INIT_ONE_PASS, SP_INIT_TWO_PASS = 0, 1, 2

#: every function the header declares (checked by the tests)
EXPORTS = (
    "sp_circuit_parse", "sp_circuit_free", "sp_circuit_add_noise", "sp_circuit_counts", "sp_symbolize", "sp_symbolize_outputs",
    "sp_symbolize_device_work_bytes", "sp_symbolize_device", "sp_symbolize_device_work_bytes_mode",
    "sp_symbolize_device_mode", "sp_model_free", "sp_model_dims",
    "sp_model_expected_work",
    "sp_model_export_dense", "sp_model_export_csc", "sp_model_export_vars", "sp_model_device_bytes",
    "sp_model_upload", "sp_model_device_bytes_tiled", "sp_model_upload_tiled", "sp_dmodel_free", "sp_dmodel_dims",
    "sp_dmodel_tiles", "sp_dmodel_get_launch", "sp_dmodel_set_launch",
    "sp_sample", "sp_sample_host", "sp_batch_work_bytes", "sp_batch_create", "sp_batch_info", "sp_batch_launch", "sp_batch_free",
    "sp_sample_batch_static",
    "sp_graph_capture_batch", "sp_graph_capture_plain", "sp_graph_launch", "sp_graph_free",
    "sp_server_work_bytes", "sp_server_create", "sp_server_submit", "sp_server_status", "sp_server_wait",
    "sp_server_release", "sp_server_stats", "sp_server_destroy", "sp_last_error",
)


class sp_noise(ctypes.Structure):
    _fields_ = [("p_1q", ctypes.c_char_p), ("p_2q", ctypes.c_char_p), ("p_meas", ctypes.c_char_p),
                ("p_reset", ctypes.c_char_p), ("p_idle", ctypes.c_char_p)]


class sp_dims(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_uint32), ("n_meas", ctypes.c_uint32), ("n_locs", ctypes.c_uint32),
                ("n_vars", ctypes.c_uint32), ("n_random_meas", ctypes.c_uint32), ("n_drawn", ctypes.c_uint32),
                ("n_draw_blocks", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("nnz", ctypes.c_uint64)]


class sp_launch(ctypes.Structure):
    _fields_ = [("waves_per_group", ctypes.c_uint32), ("words_per_group", ctypes.c_uint32)]


class sp_batch_item(ctypes.Structure):
    _fields_ = [("model", ctypes.c_void_p), ("seed", ctypes.c_uint64), ("first_shot", ctypes.c_uint64),
                ("shots", ctypes.c_uint64), ("d_out", ctypes.c_void_p), ("ld_words", ctypes.c_size_t)]


class sp_server_config(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_uint32), ("max_queued", ctypes.c_uint32), ("tick_cost", ctypes.c_uint64),
                ("launch", sp_launch)]


class sp_request_status(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("n_meas", ctypes.c_uint32), ("d_out", ctypes.c_void_p),
                ("ld_words", ctypes.c_uint64), ("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64)]


class sp_server_counters(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_uint32), ("active", ctypes.c_uint32), ("arena_in_use", ctypes.c_uint64),
                ("arena_capacity", ctypes.c_uint64), ("ticks", ctypes.c_uint64), ("groups_launched", ctypes.c_uint64),
                ("words_launched", ctypes.c_uint64)]


class SymphaseError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2311_03906_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, u32, u64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_uint64
    P = ctypes.POINTER
    sig = {
        "sp_circuit_parse": ([ctypes.c_char_p, sz, P(vp)], ctypes.c_int),
        "sp_circuit_free": ([vp], None),
        "sp_circuit_add_noise": ([vp, P(sp_noise), P(vp)], ctypes.c_int),
        "sp_symbolize": ([vp, P(vp)], ctypes.c_int),
        "sp_symbolize_outputs": ([vp, ctypes.c_int, P(vp)], ctypes.c_int),
        "sp_symbolize_device_work_bytes": ([vp, P(sz)], ctypes.c_int),
        "sp_symbolize_device": ([vp, ctypes.c_int, vp, sz, vp, P(vp)], ctypes.c_int),
        "sp_symbolize_device_work_bytes_mode": ([vp, ctypes.c_int, P(sz)], ctypes.c_int),
        "sp_symbolize_device_mode": ([vp, ctypes.c_int, ctypes.c_int, vp, sz, vp, P(vp), P(sz)], ctypes.c_int),
        "sp_circuit_counts": ([vp, P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)],
                              ctypes.c_int),
        "sp_model_free": ([vp], None),
        "sp_model_dims": ([vp, P(sp_dims)], ctypes.c_int),
        "sp_model_expected_work": ([vp, P(ctypes.c_double), P(ctypes.c_double)], ctypes.c_int),
        "sp_model_export_dense": ([vp, vp, sz, vp], ctypes.c_int),
        "sp_model_export_csc": ([vp, vp, vp], ctypes.c_int),
        "sp_model_export_vars": ([vp, vp, vp], ctypes.c_int),
        "sp_model_device_bytes": ([vp, ctypes.c_int, P(sz)], ctypes.c_int),
        "sp_model_upload": ([vp, ctypes.c_int, vp, sz, vp, P(vp)], ctypes.c_int),
        "sp_model_device_bytes_tiled": ([vp, ctypes.c_int, u32, P(sz)], ctypes.c_int),
        "sp_model_upload_tiled": ([vp, ctypes.c_int, u32, vp, sz, vp, P(vp)], ctypes.c_int),
        "sp_dmodel_tiles": ([vp, P(u32), P(u32)], ctypes.c_int),
        "sp_dmodel_free": ([vp], None),
        "sp_dmodel_dims": ([vp, P(sp_dims)], ctypes.c_int),
        "sp_dmodel_get_launch": ([vp, P(sp_launch)], ctypes.c_int),
        "sp_dmodel_set_launch": ([vp, P(sp_launch)], ctypes.c_int),
        "sp_sample": ([vp, u64, u64, u64, vp, sz, vp], ctypes.c_int),
        "sp_sample_host": ([vp, u64, u64, u64, vp, sz, ctypes.c_int], ctypes.c_int),
        "sp_batch_work_bytes": ([vp, sz, vp, ctypes.c_int, P(sz)], ctypes.c_int),
        "sp_batch_create": ([vp, sz, vp, ctypes.c_int, vp, sz, vp, P(vp)], ctypes.c_int),
        "sp_batch_info": ([vp, P(u32), P(u32), P(u32), P(sp_launch)], ctypes.c_int),
        "sp_batch_launch": ([vp, vp], ctypes.c_int),
        "sp_batch_free": ([vp], None),
        "sp_sample_batch_static": ([vp, sz, vp, ctypes.c_int, vp], ctypes.c_int),
        "sp_graph_capture_batch": ([vp, P(vp)], ctypes.c_int),
        "sp_graph_capture_plain": ([vp, sz, P(vp)], ctypes.c_int),
        "sp_graph_launch": ([vp, vp], ctypes.c_int),
        "sp_graph_free": ([vp], None),
        "sp_server_work_bytes": ([P(sp_server_config), P(sz)], ctypes.c_int),
        "sp_server_create": ([P(sp_server_config), vp, sz, vp, sz, P(vp)], ctypes.c_int),
        "sp_server_submit": ([vp, vp, u64, u64, u64, P(u64)], ctypes.c_int),
        "sp_server_status": ([vp, u64, P(sp_request_status)], ctypes.c_int),
        "sp_server_wait": ([vp, u64, ctypes.c_int64, P(sp_request_status)], ctypes.c_int),
        "sp_server_release": ([vp, u64], ctypes.c_int),
        "sp_server_stats": ([vp, P(sp_server_counters)], ctypes.c_int),
        "sp_server_destroy": ([vp], None),
        "sp_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def check(rc: int):
    if rc != SP_OK:
        raise SymphaseError(rc, lib().sp_last_error().decode(errors="replace"))
