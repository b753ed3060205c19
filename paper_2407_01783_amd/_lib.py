"""ctypes binding of libstokes.so (argument marshalling only).

Every name mirrors an entry point of ``include/stokes.h``; the structures
mirror the C structs field by field.  Loading fails loudly when the library
has not been built: there is no fallback implementation.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstokes.so")

STOKES_OK = 0
STOKES_NOT_CONVERGED = 1
ERRORS = {
    -1: "STOKES_ERR_ARG", -2: "STOKES_ERR_ALLOC", -3: "STOKES_ERR_HIP", -4: "STOKES_ERR_NONFINITE",
    -5: "STOKES_ERR_BREAKDOWN", -6: "STOKES_ERR_STATE", -7: "STOKES_ERR_UNSUPPORTED",
}
FP64, MIXED = 0, 1
INNER_TOL, INNER_FIXED = 0, 1
CC_LAPLACE, CC_LUMPED, CC_MASS = 0, 1, 2
PC_FULL, PC_UPPER, PC_LOWER = 0, 1, 2
FLAG_STRAIN = 1
FLAG_P3 = 2
VEL_CHEB, VEL_MG = 0, 1
ARNOLDI_FP32, ARNOLDI_FP64, ARNOLDI_FP64_K = 0, 1, 2


class StokesError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{ERRORS.get(status, status)}: {message}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32), ("mesh_seed", ctypes.c_uint64),
                ("jitter", ctypes.c_double), ("mu", ctypes.c_double), ("alpha", ctypes.c_double),
                ("gamma", ctypes.c_double), ("flags", ctypes.c_int32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("rtol", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("restart", ctypes.c_int32), ("max_inner", ctypes.c_int32), ("inner_mode", ctypes.c_int32),
                ("cheb_degree", ctypes.c_int32), ("inner_rtol_u", ctypes.c_double),
                ("inner_rtol_p", ctypes.c_double), ("schur_pc", ctypes.c_int32), ("coupled_pc", ctypes.c_int32),
                ("max_refine", ctypes.c_int32), ("profile", ctypes.c_int32), ("inner_its_u", ctypes.c_int32),
                ("inner_its_p", ctypes.c_int32), ("vel_pc", ctypes.c_int32), ("arnoldi_fp64", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int32), ("outer_iters", ctypes.c_int32), ("inner_iters_u", ctypes.c_int32),
                ("inner_iters_p", ctypes.c_int32), ("refinements", ctypes.c_int32),
                ("spmv_launches", ctypes.c_int32), ("rel_res", ctypes.c_double),
                ("seconds_total", ctypes.c_double), ("spmv_seconds", ctypes.c_double),
                ("spmv_bytes", ctypes.c_double), ("seconds_inner_u", ctypes.c_double),
                ("seconds_inner_p", ctypes.c_double), ("seconds_orth", ctypes.c_double),
                ("res_hist", ctypes.POINTER(ctypes.c_double)), ("res_hist_cap", ctypes.c_int32),
                ("res_hist_len", ctypes.c_int32), ("bytes_alg", ctypes.c_double)]

    def attach_history(self, cap):
        """Give the call a caller-owned history buffer of ``cap`` entries."""
        self._hist = (ctypes.c_double * max(1, int(cap)))()
        self.res_hist = ctypes.cast(self._hist, ctypes.POINTER(ctypes.c_double))
        self.res_hist_cap = int(cap)

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("res_hist", "res_hist_cap")}
        if getattr(self, "_hist", None) is not None:
            d["res_hist"] = list(self._hist[: self.res_hist_len])
        return d


EXPORTS = [
    "stokes_default_opts", "stokes_problem_sizes", "stokes_build_mesh_host", "stokes_host_pattern",
    "stokes_assemble", "stokes_solve_schur", "stokes_solve_coupled", "stokes_solve_adjoint", "stokes_apply",
    "stokes_residual", "stokes_query", "stokes_set_mu", "stokes_set_stream", "stokes_export_mesh",
    "stokes_export_csr", "stokes_bounds", "stokes_destroy", "stokes_last_error", "stokes_projection_step",
    "stokes_residual_noalloc", "stokes_bandwidth_probe",
]

_lib = None

_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)


def load():
    """Load libstokes.so (once) and declare every signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libstokes.so is not built ({LIB_PATH}); run paper_2407_01783_amd/build.py "
                          "or __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int32
    pp = ctypes.POINTER(Problem)
    po = ctypes.POINTER(SolveOpts)
    pi = ctypes.POINTER(SolveInfo)
    sig = {
        "stokes_default_opts": (None, [po]),
        "stokes_problem_sizes": (st, [pp, _I64]),
        "stokes_build_mesh_host": (st, [pp, _P, _P, _P, _P]),
        "stokes_host_pattern": (st, [pp, ctypes.c_int32, _I64, _I64, _P, _P]),
        "stokes_assemble": (st, [pp, _P, ctypes.POINTER(_P)]),
        "stokes_solve_schur": (st, [_P, ctypes.c_int32, _P, _P, _P, _P, _P, _P, po, pi]),
        "stokes_solve_coupled": (st, [_P, ctypes.c_int32, _P, _P, _P, _P, _P, _P, po, pi]),
        "stokes_solve_adjoint": (st, [_P, ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P, po, pi]),
        "stokes_projection_step": (st, [_P, ctypes.c_int32, _P, _P, _P, _P, _P, po, pi]),
        "stokes_apply": (st, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P]),
        "stokes_residual": (st, [_P, ctypes.c_int32, _P, _P, _P, _P, _D]),
        "stokes_residual_noalloc": (st, [_P, ctypes.c_int32, _P, _P, _P, _P, _D]),
        "stokes_bandwidth_probe": (st, [_P, ctypes.c_int64, ctypes.c_int32, _D]),
        "stokes_query": (st, [_P, _I64]),
        "stokes_set_mu": (st, [_P, ctypes.c_double]),
        "stokes_set_stream": (st, [_P, _P]),
        "stokes_export_mesh": (st, [_P, _P, _P]),
        "stokes_export_csr": (st, [_P, ctypes.c_int32, _P, _P, _P]),
        "stokes_bounds": (st, [_P, _D]),
        "stokes_destroy": (None, [_P]),
        "stokes_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status, what=""):
    """Raise StokesError for a negative status; return the status otherwise."""
    if status < 0:
        msg = load().stokes_last_error().decode(errors="replace")
        raise StokesError(status, f"{what}: {msg}" if what else msg)
    return status


def default_opts(**kw):
    o = SolveOpts()
    load().stokes_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def make_problem(dim, n, mesh_seed=0, jitter=0.0, mu=1.0, alpha=1.0, gamma=0.0, flags=0):
    return Problem(dim=int(dim), n=int(n), mesh_seed=int(mesh_seed), jitter=float(jitter), mu=float(mu),
                   alpha=float(alpha), gamma=float(gamma), flags=int(flags))


def ptr(x):
    """Device or host address of a torch tensor / numpy array (None -> NULL)."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return ctypes.c_void_p(x.data_ptr())
    return ctypes.c_void_p(x.ctypes.data)
