"""ctypes loader and prototypes for libfracctl.so (see include/fracctl.h)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfracctl.so")

STATUS = {
    0: "FC_OK", 1: "FC_ERR_INVALID_ARG", 2: "FC_ERR_OUT_OF_MEMORY", 3: "FC_ERR_NOT_CONVERGED",
    4: "FC_ERR_RANK_OVERFLOW", 5: "FC_ERR_NUMERIC", 6: "FC_ERR_HIP", 7: "FC_ERR_INTERNAL",
}


class LibraryMissing(RuntimeError):
    pass


class FcError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {detail}")
        self.status = status
        self.detail = detail


class SetupParams(C.Structure):
    _fields_ = [
        ("n", C.c_int),
        ("a", C.POINTER(C.c_double) * 3),
        ("alpha", C.c_double),
        ("beta", C.c_double),
        ("gamma", C.c_double),
        ("eps", C.c_double),
        ("tol", C.c_double),
        ("op_accuracy", C.c_double),
        ("max_iter", C.c_int),
        ("max_rank", C.c_int),
        ("precond_rank", C.c_int),
        ("precision", C.c_int),
        ("precond", C.c_int),
        ("precond_b0", C.c_double * 3),
        ("dims", C.c_int),
    ]


class Info(C.Structure):
    _fields_ = [
        ("iterations", C.c_int),
        ("refinements", C.c_int),
        ("rank_u", C.c_int),
        ("tucker_rank", C.c_int * 3),
        ("max_tucker_rank", C.c_int),
        ("op_rank", C.c_int),
        ("precond_rank", C.c_int),
        ("rel_residual", C.c_double),
        ("op_max_rel_err", C.c_double),
        ("precond_max_rel_err", C.c_double),
        ("state_rank", C.c_int),
        ("state_max_rel_err", C.c_double),
        ("subspace_miss", C.c_double),
    ]

    def as_dict(self):
        return {
            "iterations": self.iterations, "refinements": self.refinements,
            "rank_u": self.rank_u,
            "tucker_rank": list(self.tucker_rank), "max_tucker_rank": self.max_tucker_rank,
            "op_rank": self.op_rank, "precond_rank": self.precond_rank,
            "rel_residual": self.rel_residual, "op_max_rel_err": self.op_max_rel_err,
            "precond_max_rel_err": self.precond_max_rel_err,
            "state_rank": self.state_rank, "state_max_rel_err": self.state_max_rel_err,
            "subspace_miss": self.subspace_miss,
        }


# every symbol the header declares, with (restype, argtypes)
_D = C.c_double
_PD = C.POINTER(C.c_double)
_VP = C.c_void_p
_I = C.c_int
_PI = C.POINTER(C.c_int)
PROTOTYPES = {
    "fc_setup": (_I, [_I, _PD, _PD, _PD, _D, _D, _D, C.POINTER(_VP)]),
    "fc_setup_ex": (_I, [C.POINTER(SetupParams), _VP, C.POINTER(_VP)]),
    "fc_solve": (_I, [_VP, _I, _VP, _VP, _VP, _VP, _I, _PI, _VP, _VP, _VP, _VP,
                      C.POINTER(Info), _VP]),
    "fc_solve2d": (_I, [_VP, _I, _VP, _VP, _VP, _I, _PI, _VP, _VP, _VP, C.POINTER(Info), _VP]),
    "fc_solve_state": (_I, [_VP, _I, _VP, _VP, _VP, _VP, _I, _PI, _VP, _VP, _VP, _VP,
                            _I, _PI, _VP, _VP, _VP, _VP, _PD, C.POINTER(Info), _VP]),
    "fc_solve_batched": (_I, [_I, C.POINTER(_VP), _PI, C.POINTER(_VP), C.POINTER(_VP),
                              C.POINTER(_VP), C.POINTER(_VP), _PI, _PI, C.POINTER(_VP),
                              C.POINTER(_VP), C.POINTER(_VP), C.POINTER(_VP), _PI,
                              C.POINTER(Info), _VP]),
    "fc_destroy": (None, [_VP]),
    "fc_plan_spectrum": (_I, [_VP, _PD, _PD]),
    "fc_plan_separable": (_I, [_VP, _I, _I, _PI, _PD, _PD]),
    "fc_plan_tuning": (_I, [_VP, _PI, _PD]),
    "fc_mode_transform": (_I, [_VP, _I, _I, _I, _VP, _VP, _VP]),
    "fc_cp_inner": (_I, [_VP, _I, _VP, _VP, _VP, _VP, _I, _VP, _VP, _VP, _VP, _PD, _VP]),
    "fc_cp_inner_noalloc": (_I, [_I, _I, _VP, _VP, _VP, _VP, _I, _VP, _VP, _VP, _VP, _VP, _VP]),
    "fc_cp_truncate": (_I, [_VP, _I, _VP, _VP, _VP, _VP, _D, _I, _PI, _VP, _VP, _VP, _VP, _VP]),
    "fc_apply_separable": (_I, [_VP, _I, _I, _VP, _VP, _VP, _VP, _D, _I, _PI, _VP, _VP, _VP,
                                _VP, _VP]),
    "fc_host_fd_eigen": (_I, [_I, _PD, _PD, _PD]),
    "fc_host_expsum": (_I, [_I, _D, _D, _D, _D, _D, _I, _PD, _PD, _PD]),
    "fc_host_separable": (_I, [C.POINTER(SetupParams), _I, _I, _PI, _PD, _PD, _PD]),
    "fc_selftest_mfma": (_I, [_PD]),
    "fc_selftest_eig": (_I, [_I, _PD, _PD, _PD]),
    "fc_profile_gemm": (_I, [_I]),
    "fc_profile_kernel_read": (_I, [_I, C.POINTER(C.c_long), _PD, _PD, _PD]),
    "fc_profile_gemm_read": (_I, [C.POINTER(C.c_long), _PD, _PD, _PD]),
    "fc_status_string": (C.c_char_p, [_I]),
    "fc_last_error": (C.c_char_p, []),
}

_LIB = None


def lib() -> C.CDLL:
    """Load libfracctl.so (built in-tree by build.py).  Raises LibraryMissing
    if it has not been built: there is no fallback path."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(
                f"{LIB_PATH} not found; build it with `python -m paper_2006_09314_amd.build`")
        # torch first: its HIP runtime (the one that owns the device buffers
        # this binding passes) is then the one the library binds to by soname;
        # loading the library first would bring in a second runtime that
        # torch's own initialisation cannot share.
        import torch  # noqa: F401
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _LIB = h
    return _LIB


def check(status: int, where: str) -> None:
    if status != 0:
        raise FcError(status, where, lib().fc_last_error().decode(errors="replace"))
