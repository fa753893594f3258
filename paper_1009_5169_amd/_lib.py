"""ctypes binding of libmfq.so: argument marshalling only.

Every operation runs in the HIP library; this module passes device pointers
of torch tensors and the current HIP stream.  If the library is not built or
cannot be loaded, every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch  # loaded first, so libmfq binds to the HIP runtime torch already mapped

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfq.so")

BC = {"sf": 0, "periodic": 1, "antiperiodic": 2}
PREC = {"fp64": 0, "fp32": 1, "fp16": 2}
OPS = {"hop_eo": 0, "hop_oe": 1, "D": 2, "Ddag": 3, "DdagD": 4, "hop": 5, "hop_dag": 6,
       "schur": 7, "schur_dag": 8, "schur_normal": 9}
ROUTE = {"full": 0, "schur": 1}
PRECOND = {"none": 0, "ptc": 1, "identity": 2, "blockcg": 3, "bicgstab": 4, "gl_bicgstab": 5,
           "bl_bicgstab": 6}

MFQ_OK, MFQ_NOT_CONVERGED, MFQ_FELL_BACK = 0, 1, 2


class MfqError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mfq error {code}: {msg}")
        self.code = code


class _Lattice(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("bc", ctypes.c_int), ("kappa", ctypes.c_double)]


class SolveParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("prec", ctypes.c_int),
                ("reliable_delta", ctypes.c_double), ("precond", ctypes.c_int),
                ("restart", ctypes.c_int), ("check_every", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("route", ctypes.c_int), ("inner_tol", ctypes.c_double), ("inner_max_iter", ctypes.c_int)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("reliable_updates", ctypes.c_int),
                ("true_rel_resid", ctypes.c_double), ("seconds", ctypes.c_double),
                ("status", ctypes.c_int), ("inner_iters", ctypes.c_int), ("inner_calls", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class HmcParams(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("n_steps", ctypes.c_int), ("rand_uniform", ctypes.c_double)]


class HmcResult(ctypes.Structure):
    _fields_ = [("delta_h", ctypes.c_double), ("kinetic_old", ctypes.c_double), ("kinetic_new", ctypes.c_double),
                ("action_old", ctypes.c_double), ("action_new", ctypes.c_double), ("accepted", ctypes.c_int),
                ("force_evals", ctypes.c_int), ("solver_iters", ctypes.c_int), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lock = threading.Lock()
_lib = None

_P = ctypes.c_void_p
_SIGNATURES = {
    "mfq_create": ([ctypes.POINTER(_Lattice), _P, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "mfq_update_links": ([_P, _P, _P], ctypes.c_int),
    "mfq_dslash": ([_P, ctypes.c_int, _P, _P, ctypes.c_int, _P], ctypes.c_int),
    "mfq_dslash_noalloc": ([_P, ctypes.c_int, _P, _P, ctypes.c_int, _P], ctypes.c_int),
    "mfq_dslash_prec": ([_P, ctypes.c_int, ctypes.c_int, _P, _P, ctypes.c_int, _P], ctypes.c_int),
    "mfq_solve_multi_rhs": ([_P, _P, _P, ctypes.c_int, ctypes.POINTER(SolveParams),
                             ctypes.POINTER(SolveStats), _P], ctypes.c_int),
    "mfq_solve_dirac": ([_P, ctypes.c_int, _P, _P, ctypes.c_int, ctypes.POINTER(SolveParams),
                         ctypes.POINTER(SolveStats), _P], ctypes.c_int),
    "mfq_fermion_force": ([_P, _P, ctypes.c_int, ctypes.POINTER(SolveParams), _P,
                           ctypes.POINTER(ctypes.c_double), _P, _P, ctypes.POINTER(SolveStats), _P],
                          ctypes.c_int),
    "mfq_fermion_force_eo": ([_P, _P, ctypes.c_int, ctypes.POINTER(SolveParams), _P,
                              ctypes.POINTER(ctypes.c_double), _P, _P, ctypes.POINTER(SolveStats), _P],
                             ctypes.c_int),
    "mfq_kinetic_energy": ([_P, _P, ctypes.POINTER(ctypes.c_double), _P], ctypes.c_int),
    "mfq_md_momenta": ([_P, _P, _P, ctypes.c_double, _P], ctypes.c_int),
    "mfq_md_links": ([_P, _P, _P, ctypes.c_double, _P], ctypes.c_int),
    "mfq_hmc_trajectory": ([_P, _P, _P, _P, ctypes.c_int, ctypes.POINTER(HmcParams), ctypes.POINTER(SolveParams),
                            ctypes.POINTER(HmcResult), _P], ctypes.c_int),
    "mfq_time_hop": ([_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P,
                      ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "mfq_set_autotune": ([_P, ctypes.c_int], ctypes.c_int),
    "mfq_hop_shape": ([_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "mfq_batch_create": ([ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int, _P,
                          ctypes.POINTER(_P)], ctypes.c_int),
    "mfq_batch_solve": ([_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(SolveParams),
                         ctypes.POINTER(SolveStats), _P], ctypes.c_int),
    "mfq_solve_batch": ([ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(_P),
                         ctypes.POINTER(ctypes.c_int), ctypes.POINTER(SolveParams), ctypes.POINTER(SolveStats),
                         _P], ctypes.c_int),
    "mfq_batch_grid": ([_P], ctypes.c_int),
    "mfq_batch_split": ([_P], ctypes.c_int),
    "mfq_batch_set_shape": ([_P, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "mfq_batch_destroy": ([_P], None),
    "mfq_precond_init": ([_P, ctypes.c_ulonglong, ctypes.c_double], ctypes.c_int),
    "mfq_precond_set_weights": ([_P, _P], ctypes.c_int),
    "mfq_precond_get_weights": ([_P, ctypes.c_int, _P], ctypes.c_int),
    "mfq_precond_apply": ([_P, _P, _P, ctypes.c_int, _P], ctypes.c_int),
    "mfq_precond_loss_grad": ([_P, _P, _P, ctypes.c_int, ctypes.POINTER(ctypes.c_double), _P, _P], ctypes.c_int),
    "mfq_precond_train": ([_P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_double, _P, _P], ctypes.c_int),
    "mfq_precond_pairs": ([_P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P, _P], ctypes.c_int),
    "mfq_precond_save": ([_P, ctypes.c_char_p], ctypes.c_int),
    "mfq_precond_load": ([_P, ctypes.c_char_p], ctypes.c_int),
    "mfq_last_error": ([], ctypes.c_char_p),
    "mfq_destroy": ([_P], None),
}


def exported_symbols() -> list[str]:
    return list(_SIGNATURES)


def _hip_runtimes_mapped() -> set[str]:
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64.so" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return paths


def lib():
    """Load libmfq.so once (raises if it is missing)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1009_5169_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(handle, name)
            fn.argtypes = args
            fn.restype = res
        runtimes = _hip_runtimes_mapped()
        if len(runtimes) > 1:
            raise RuntimeError(f"more than one HIP runtime mapped: {sorted(runtimes)}")
        _lib = handle
        return _lib


def check(code: int, allow=(MFQ_OK,)) -> int:
    if code in allow:
        return code
    if code > 0:  # a status, not an error: the last error message is unrelated
        raise MfqError(code, "unexpected status")
    msg = lib().mfq_last_error()
    raise MfqError(code, msg.decode() if msg else "")


def stream_ptr(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def dptr(t: torch.Tensor) -> ctypes.c_void_p:
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if t.dtype not in (torch.complex128, torch.float64):
        raise ValueError("expected complex128 (or float64 re/im) data")
    return ctypes.c_void_p(t.data_ptr())


def make_params(tol=1e-10, max_iter=20000, prec="fp32", reliable_delta=0.1, precond="none",
                restart=16, check_every=0, use_graph=True, route="full", inner_tol=0.0,
                inner_max_iter=0) -> SolveParams:
    return SolveParams(float(tol), int(max_iter), PREC[prec], float(reliable_delta), PRECOND[precond],
                       int(restart), int(check_every), int(bool(use_graph)), ROUTE[route], float(inner_tol),
                       int(inner_max_iter))
