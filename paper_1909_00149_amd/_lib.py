"""ctypes view of the C ABI in include/uot.h (structures and signatures only)."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libuot.so")
# digest of the sources libuot.so was built from, written by build.py beside it
DIGEST_PATH = LIB_PATH + ".sources"


def sources_digest():
    """SHA-256 over the library's sources (csrc/, include/) and build script,
    in a fixed file order."""
    import hashlib
    root = os.path.dirname(_PKG)
    files = []
    for d, exts in ((os.path.join(_PKG, "csrc"), (".hip", ".hpp", ".cpp", ".h")),
                    (os.path.join(root, "include"), (".h",))):
        files += sorted(os.path.join(d, f) for f in os.listdir(d) if f.endswith(exts))
    files.append(os.path.join(_PKG, "build.py"))
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.relpath(f, root).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()

UOT_OK, UOT_ERR_ARG, UOT_ERR_SHAPE, UOT_ERR_STEP, UOT_ERR_NONFINITE = 0, 1, 2, 3, 4
UOT_ERR_NEGATIVE, UOT_ERR_DEVICE, UOT_ERR_OOM, UOT_ERR_MASS, UOT_ERR_TOO_LARGE = 5, 6, 7, 8, 9
UOT_NOALLOC_SCRATCH_BYTES, UOT_NOALLOC_MAX_PIXELS, UOT_NOALLOC_MAX_TILES = 32 << 20, 1 << 20, 1 << 14
STATUS_NAMES = {0: "CONVERGED", 1: "MAX_ITER", 2: "DIVERGED"}

UOT_WARM_START = 0x1
UOT_ALLOW_SIGNED = 0x4
UOT_UNSAFE_STEPS = 0x8
UOT_NO_GRAPH = 0x10
UOT_AUTOTUNE = 0x20
UOT_ADAPTIVE_STEPS = 0x40
UOT_RECORD_HISTORY = 0x80
UOT_WARM_FALLBACK = 0x100


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("balanced", ctypes.c_int32),
                ("residual_p", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("mu", ctypes.c_double), ("rho", ctypes.c_double),
                ("tau1", ctypes.c_double), ("tau2", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("tol", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("tile_rows", ctypes.c_int32), ("pitch", ctypes.c_int32),
                ("norm", ctypes.c_int32), ("max_groups", ctypes.c_int32)]


class State(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("Mx", "My", "r", "a", "x0", "x1")]


class DrReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("fixed_point_res", ctypes.c_double), ("objective", ctypes.c_double),
                ("infeasibility", ctypes.c_double), ("seconds", ctypes.c_double),
                ("ms_per_iter", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["status_name"] = STATUS_NAMES.get(self.status, str(self.status))
        return d


class Report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("rel_res", ctypes.c_double), ("rel_gap", ctypes.c_double),
                ("primal", ctypes.c_double), ("dual", ctypes.c_double),
                ("feas", ctypes.c_double), ("objective", ctypes.c_double),
                ("seconds", ctypes.c_double), ("tau1", ctypes.c_double),
                ("tau2", ctypes.c_double), ("tile_rows", ctypes.c_int32),
                ("cold_start", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["status_name"] = STATUS_NAMES.get(self.status, str(self.status))
        return d


class DfParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("balanced", ctypes.c_int32), ("residual_p", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("kappa", ctypes.c_double), ("mu", ctypes.c_double), ("lam", ctypes.c_double),
                ("rho", ctypes.c_double), ("prox_iters", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("eps", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("prox_tau_ratio", ctypes.c_double)]


class DfReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("r_primal", ctypes.c_double), ("r_dual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("ms_per_iter", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RpParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("frames", ctypes.c_int32),
                ("balanced", ctypes.c_int32), ("residual_p", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("lam", ctypes.c_double), ("gam", ctypes.c_double), ("kappa", ctypes.c_double),
                ("mu", ctypes.c_double), ("rho", ctypes.c_double), ("prox_iters", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32), ("eps", ctypes.c_double),
                ("flags", ctypes.c_uint32), ("prox_tau_ratio", ctypes.c_double),
                ("signed_sparse", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class RpReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("r_primal", ctypes.c_double), ("r_dual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("ms_per_iter", ctypes.c_double),
                ("jacobi_sweeps", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_lib = None

SIGNATURES = {
    "uot_check_params": (ctypes.c_int, [ctypes.POINTER(Params)]),
    "uot_knorm2": (ctypes.c_double, [ctypes.c_int32] * 5),
    "uot_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "uot_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.POINTER(State), ctypes.POINTER(Report)]),
    "uot_solve_batched": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.POINTER(State), ctypes.POINTER(Report)]),
    "uot_solve_batched_pitched": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                                 ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                                 ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                                 ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.POINTER(State), ctypes.POINTER(Report)]),
    "uot_objective": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.POINTER(State), ctypes.POINTER(State), ctypes.POINTER(Report)]),
    "uot_time_iterations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.POINTER(State), ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]),
    "uot_time_iterations_batched": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                                   ctypes.POINTER(ctypes.c_int64),
                                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(State),
                                                   ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                                   ctypes.POINTER(ctypes.c_int32)]),
    "uot_history": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "uot_dr_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_double, ctypes.c_void_p]),
    "uot_poisson": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                   ctypes.c_void_p, ctypes.c_void_p]),
    "uot_init_poisson": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.POINTER(State)]),
    "uot_init_poisson_pitched": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                                ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                                ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(State)]),
    "uot_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(State),
                                ctypes.POINTER(State), ctypes.c_int32]),
    "uot_solve_noalloc": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.POINTER(State), ctypes.POINTER(Report)]),
    "uot_destroy": (None, [ctypes.c_void_p]),
    "uotdf_check_params": (ctypes.c_int, [ctypes.POINTER(DfParams)]),
    "uotdf_create": (ctypes.c_int, [ctypes.POINTER(DfParams), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "uotdf_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.POINTER(DfReport)]),
    "uotdf_copy_planes": (ctypes.c_int, [ctypes.c_void_p] * 5),
    "uotdf_destroy": (None, [ctypes.c_void_p]),
    "rpca_check_params": (ctypes.c_int, [ctypes.POINTER(RpParams)]),
    "rpca_create": (ctypes.c_int, [ctypes.POINTER(RpParams), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "rpca_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.POINTER(RpReport)]),
    "rpca_copy_planes": (ctypes.c_int, [ctypes.c_void_p] * 9),
    "rpca_copy_sparse": (ctypes.c_int, [ctypes.c_void_p] * 3),
    "rpca_destroy": (None, [ctypes.c_void_p]),
    "uot_status_string": (ctypes.c_char_p, [ctypes.c_int]),
}


def load():
    """Loads libuot.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1909_00149_amd.build`")
    # the library must have been built from the sources in this tree
    try:
        with open(DIGEST_PATH) as f:
            built = f.read().strip()
    except OSError:
        built = None
    if built != sources_digest():
        raise RuntimeError(f"{LIB_PATH} was not built from the current sources "
                           f"({'no ' + DIGEST_PATH if built is None else 'source digest differs'}): "
                           "rebuild it with `python -m paper_1909_00149_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
