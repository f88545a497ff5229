"""ctypes view of libeslb.so (argument marshalling only; every step runs in HIP)."""
import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("ESLB_LIBRARY") or os.path.join(HERE, "libeslb.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "eslb.h")

c_int32, c_int64, c_double, c_void_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
P = ctypes.POINTER

D1Q2, D2Q4 = 1, 2
ADVECTION, BURGERS, SHALLOW_WATER, EULER = 0, 1, 2, 3
OMEGA_FIXED, OMEGA_ENTROPIC = 0, 1
FUSE_OFF, FUSE_AUTO, FUSE_ALWAYS = 0, 1, 2
OK = 0
ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_HIP, ERR_NOMEM, ERR_INADMISSIBLE, ERR_NAN = -1, -2, -3, -4, -6, -7
WARN_OMEGA_FALLBACK, WARN_T_NOT_MULTIPLE, WARN_SUBCHARACTERISTIC = 1, 2, 3


class Problem(ctypes.Structure):
    _fields_ = [("lattice", c_int32), ("system", c_int32), ("nx", c_int32), ("ny", c_int32),
                ("kappa", c_int32), ("relax", c_int32), ("scheme", c_int32), ("reserved", c_int32),
                ("V", c_double), ("dx", c_double), ("omega", c_double), ("param", c_double * 4)]


class Diag(ctypes.Structure):
    _fields_ = [("mass", c_double * 4), ("micro_entropy", c_double), ("macro_entropy", c_double),
                ("omega_min", c_double), ("omega_max", c_double), ("n_fallback", c_int64),
                ("n_outside", c_int64), ("n_inadmissible", c_int64), ("n_nan", c_int64)]


_SIGNATURES = {
    "eslb_create": (c_int32, [P(Problem), c_void_p, P(c_void_p)]),
    "eslb_destroy": (None, [c_void_p]),
    "eslb_state_bytes": (c_int32, [c_void_p, P(ctypes.c_size_t)]),
    "eslb_dims": (c_int32, [c_void_p, P(c_int32), P(c_int32)]),
    "eslb_dt": (c_int32, [c_void_p, P(c_double)]),
    "eslb_steps_for_time": (c_int32, [c_void_p, c_double, P(c_int64)]),
    "eslb_init_equilibrium": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "eslb_step": (c_int32, [c_void_p, c_void_p, c_int64]),
    "eslb_transport": (c_int32, [c_void_p, c_int32]),
    "eslb_relax": (c_int32, [c_void_p, c_void_p]),
    "eslb_project": (c_int32, [c_void_p, c_void_p]),
    "eslb_moments": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "eslb_gather": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "eslb_get_offsets": (c_int32, [c_void_p, P(c_int64)]),
    "eslb_set_offsets": (c_int32, [c_void_p, P(c_int64)]),
    "eslb_diagnostics": (c_int32, [c_void_p, c_void_p, P(Diag)]),
    "eslb_diagnostics_noalloc": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "eslb_set_stats": (c_int32, [c_void_p, c_int32]),
    "eslb_reset_counters": (c_int32, [c_void_p]),
    "eslb_sync_status": (c_int32, [c_void_p]),
    "eslb_relax_adjoint": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "eslb_moments_adjoint": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "eslb_init_adjoint": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "eslb_adjoint_workspace_bytes": (c_int32, [c_void_p, c_int64, c_int64, P(ctypes.c_size_t)]),
    "eslb_adjoint_tape_bytes": (c_int32, [c_void_p, c_int64, c_int64, P(ctypes.c_size_t)]),
    "eslb_set_step_workspace": (c_int32, [c_void_p, c_void_p, ctypes.c_size_t]),
    "eslb_fused_step_available": (c_int32, [c_void_p, P(c_int32)]),
    "eslb_set_fusion": (c_int32, [c_void_p, c_int32]),
    "eslb_checkpoint_bytes": (c_int32, [c_void_p, c_int64, c_int64, P(ctypes.c_size_t)]),
    "eslb_step_checkpointed": (c_int32, [c_void_p, c_void_p, c_int64, c_int64, c_void_p]),
    "eslb_adjoint_checkpointed": (c_int32, [c_void_p, c_void_p, c_int64, c_int64, c_void_p, c_void_p,
                                            ctypes.c_size_t]),
    "eslb_adjoint": (c_int32, [c_void_p, c_void_p, c_int64, c_int64, c_void_p, c_void_p, ctypes.c_size_t]),
    "eslb_batch_create": (c_int32, [P(Problem), c_int32, c_void_p, P(c_void_p)]),
    "eslb_batch_destroy": (None, [c_void_p]),
    "eslb_batch_run": (c_int32, [c_void_p, P(c_void_p), P(c_int64)]),
    "eslb_batch_get_offsets": (c_int32, [c_void_p, c_int32, P(c_int64)]),
    "eslb_batch_set_offsets": (c_int32, [c_void_p, c_int32, P(c_int64)]),
    "eslb_batch_sync_status": (c_int32, [c_void_p]),
    "eslb_batch_set_config": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_int32]),
    "eslb_batch_get_config": (c_int32, [c_void_p, P(c_int32)]),
    "eslb_batch_autotune": (c_int32, [c_void_p, P(c_void_p), c_int32, P(c_double)]),
    "eslb_batch_last_error": (ctypes.c_char_p, [c_void_p]),
    "eslb_status_string": (ctypes.c_char_p, [c_int32]),
    "eslb_last_error": (ctypes.c_char_p, [c_void_p]),
}

_lib = None


def declared_functions(header=HEADER):
    """Names of every function the public header declares."""
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eslb_[a-z_0-9]+)\s*\(", text)))


def load():
    """Load libeslb.so once; raise if it is missing (there is no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libeslb.so is not built (%s); run paper_2403_13406_amd.build or "
                           "__graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
