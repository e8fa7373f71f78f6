"""ctypes binding of libqforte_mi355x.so (argument marshalling only).

Every function here forwards to the C ABI declared in
include/qforte_mi355x.h; device buffers are torch tensors (complex128 on a
ROCm device), host tables are numpy arrays.  Nothing is computed in Python.
If the shared library is missing this module raises at import time: there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqforte_mi355x.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2108_04413_amd/build.py`")

# torch's ROCm build loads its own libamdhip64 (DT_NEEDED "libamdhip64.so",
# SONAME "libamdhip64.so.7").  Loading torch first lets this library's
# "libamdhip64.so.7" dependency bind to that same runtime; in the other order
# the process would hold two HIP runtimes that do not share devices.
import torch  # noqa: E402,F401

TERM_DTYPE = np.dtype([("x", "<u8"), ("z", "<u8"), ("c", "<f8")])

QF_OK = 0
STATUS = {0: "QF_OK", -1: "QF_E_ARG", -2: "QF_E_RANGE", -3: "QF_E_NOMEM", -4: "QF_E_HIP",
          -5: "QF_E_SIZE", -6: "QF_E_NOTHERM"}
QF_HAMILTONIAN, QF_UCCSD, QF_UCCD, QF_UCCD_TOP, QF_PUCCD, QF_GSD_POOL = 0, 1, 2, 3, 4, 5

EXPORTS = ("qf_build_paulis", "qf_ansatz_angles", "qf_grad_t", "qf_prepare_state", "qf_apply_pauli_exp",
           "qf_energy", "qf_energy_grad", "qf_plan_create", "qf_plan_destroy", "qf_plan_apply",
           "qf_plan_energy", "qf_plan_energy_grad", "qf_plan_sigma", "qf_last_error", "qf_version",
           "qf_batch_create", "qf_batch_run", "qf_batch_info", "qf_batch_set_spin_limit", "qf_batch_destroy",
           "qf_batch_create_arena", "qf_batch_launch", "qf_batch_poll", "qf_batch_collect",
           "qf_mailbox_alloc", "qf_mailbox_free", "qf_batch_mailbox_bytes", "qf_batch_launch_mailbox",
           "qf_plan_set_energy_tile", "qf_plan_info", "qf_plan_set_block_bits", "qf_plan_apply_info",
           "qf_plan_create_arena", "qf_energy_static", "qf_batch_status", "qf_batch_teams",
           "qf_batch_resident_grid", "qf_pool_grad", "qf_plan_create_pool", "qf_plan_pool_grad",
           "qf_excited_determinants", "qf_mp_denominators", "qf_pqe_residuals", "qf_plan_pqe_residuals",
           "qf_plan_pqe_solve", "qf_plan_trotter", "qf_plan_qk_matrices",
           "qf_plan_grad_info", "qf_excitations", "qf_sector_create", "qf_sector_info", "qf_sector_prepare",
           "qf_sector_apply", "qf_sector_energy", "qf_sector_destroy", "qf_sector_energy_grad")


class QFError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_u64 = ctypes.c_uint64
_int = ctypes.c_int

lib = ctypes.CDLL(LIB_PATH)
_sig = {
    "qf_build_paulis": [_int, _int, _int, _vp, _vp, _dbl, _vp, _i64, _vp, _i64, _vp, _vp, _i64, _vp, _vp],
    "qf_ansatz_angles": [_vp, _vp, _i64, _vp, _vp],
    "qf_grad_t": [_vp, _vp, _i64, _vp, _vp],
    "qf_prepare_state": [_vp, _int, _u64, _vp],
    "qf_apply_pauli_exp": [_vp, _int, _vp, _vp, _i64, _int, _vp],
    "qf_energy": [_vp, _int, _vp, _vp, _i64, _vp, _vp],
    "qf_energy_grad": [_int, _u64, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _vp],
    "qf_plan_create": [_int, _vp, _i64, _vp, _vp, _i64, _vp],
    "qf_plan_create_arena": [_int, _vp, _i64, _vp, _vp, _i64, _int, _int, _vp, _i64, _vp, _vp, _vp],
    "qf_energy_static": [_vp, _int, _vp, _vp, _i64, _vp, _vp],
    "qf_plan_destroy": [_vp],
    "qf_plan_apply": [_vp, _vp, _vp, _int, _vp],
    "qf_plan_energy": [_vp, _vp, _vp, _vp],
    "qf_plan_energy_grad": [_vp, _u64, _vp, _vp, _vp, _vp, _vp],
    "qf_plan_sigma": [_vp, _vp, _vp, _vp, _vp],
    "qf_batch_create": [_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "qf_batch_run": [_vp, _vp, _vp, _vp, _int, _vp],
    "qf_batch_info": [_vp, _vp, _vp, _vp],
    "qf_batch_set_spin_limit": [_vp, ctypes.c_uint32],
    "qf_batch_destroy": [_vp],
    "qf_batch_create_arena": [_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _int, _vp, _i64, _vp, _vp, _vp],
    "qf_batch_status": [_vp, _vp],
    "qf_pool_grad": [_int, _u64, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _vp],
    "qf_plan_create_pool": [_int, _vp, _vp, _i64, _vp],
    "qf_plan_trotter": [_vp, _vp, _dbl, _int, _vp],
    "qf_plan_grad_info": [_vp, _vp, _vp],
    "qf_excitations": [_int, _int, _int, _vp, _i64, _vp, _i64, _vp],
    "qf_sector_create": [_int, _int, _int, _vp, _i64, _vp, _vp, _i64, _vp],
    "qf_sector_info": [_vp, _vp, _vp, _vp, _vp],
    "qf_sector_prepare": [_vp, _vp, _u64, _vp],
    "qf_sector_apply": [_vp, _vp, _vp, _int, _vp],
    "qf_sector_energy": [_vp, _vp, _vp, _vp],
    "qf_sector_energy_grad": [_vp, _u64, _vp, _vp, _vp, _vp, _vp],
    "qf_sector_destroy": [_vp],
    "qf_plan_qk_matrices": [_vp, _u64, _dbl, _int, _int, _vp, _vp, _vp, _vp],
    "qf_excited_determinants": [_int, _int, _int, _vp, _i64, _vp, _vp, _i64, _vp],
    "qf_mp_denominators": [_int, _int, _int, _vp, _vp, _vp, _i64, _vp, _i64, _vp],
    "qf_pqe_residuals": [_int, _u64, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _vp],
    "qf_plan_pqe_residuals": [_vp, _u64, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp],
    "qf_plan_pqe_solve": [_vp, _u64, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _int, _dbl, _vp, _vp, _vp, _vp, _vp],
    "qf_plan_pool_grad": [_vp, _vp, _u64, _vp, _vp, _vp, _vp, _vp],
    "qf_batch_resident_grid": [_vp],
    "qf_batch_teams": [_int, _vp, _vp, _vp, _vp, _int, _int, _vp],
    "qf_batch_launch": [_vp, _vp, _vp],
    "qf_batch_poll": [_vp],
    "qf_batch_collect": [_vp, _vp, _vp],
    "qf_mailbox_alloc": [_i64, _vp],
    "qf_mailbox_free": [_vp],
    "qf_batch_mailbox_bytes": [_vp, _vp],
    "qf_batch_launch_mailbox": [_vp, _vp, _vp, _i64, _vp],
    "qf_plan_set_energy_tile": [_vp, _int, _int],
    "qf_plan_info": [_vp, _vp, _vp, _vp],
    "qf_plan_set_block_bits": [_vp, _int],
    "qf_plan_apply_info": [_vp, _vp, _vp, _vp],
}
for _name, _args in _sig.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
lib.qf_last_error.restype = ctypes.c_char_p
lib.qf_version.restype = ctypes.c_char_p


def check(status: int, where: str) -> None:
    if status != QF_OK:
        raise QFError(status, where, lib.qf_last_error().decode())


def ptr(a) -> int | None:
    """Address of a numpy array, a torch tensor or None."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def stream_handle(stream=None):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream) if hasattr(stream, "cuda_stream") else ctypes.c_void_p(stream)


def terms_array(x, z, c) -> np.ndarray:
    t = np.empty(len(x), dtype=TERM_DTYPE)
    t["x"] = np.asarray(x, dtype=np.uint64)
    t["z"] = np.asarray(z, dtype=np.uint64)
    t["c"] = np.asarray(c, dtype=np.float64)
    return t
