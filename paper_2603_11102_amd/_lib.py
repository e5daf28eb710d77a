"""ctypes binding of libgks.so (the C ABI of include/gks.h). Argument marshalling only: every step of
the method runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GKS_LIBRARY") or os.path.join(HERE, "libgks.so")

GKS_OK = 0
GKS_E_INVALID_ARG = 1
GKS_E_STATE = 2
GKS_E_HIP = 3
GKS_E_NONFINITE = 4
GKS_E_UNSTABLE = 5
GKS_E_UNSUPPORTED = 6
GKS_E_BODY_LEFT = 7
GKS_WARN_EPS_SMALL = 1
GKS_WARN_MACH = 2
GKS_ADJ_EXACT_WENO = 1

BC = {"periodic": 0, "noslip": 1, "slip": 2, "inflow": 3, "outflow": 4}
GKS_FP32 = 0
GKS_FP64 = 1
GKS_STATIC_SCRATCH_BYTES = 64 << 20


class gks_config(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("precision", C.c_int32),
        ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
        ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
        ("ma", C.c_double), ("u_ref", C.c_double), ("rho_ref", C.c_double), ("mu", C.c_double),
        ("cfl", C.c_double), ("dt_fixed", C.c_double),
        ("bc", C.c_int32 * 6),
        ("u_in", C.c_double * 3), ("body_force", C.c_double * 3),
        ("weno_eps", C.c_double),
        ("ibm_iters", C.c_int32), ("max_act", C.c_int32), ("max_ibm", C.c_int64),
        ("order", C.c_int32),
        ("faces", C.POINTER(C.c_double) * 3),
    ]


class gks_field(C.Structure):
    _fields_ = [("rho", C.c_void_p), ("mx", C.c_void_p), ("my", C.c_void_p), ("mz", C.c_void_p)]


class gks_rotor(C.Structure):
    _fields_ = [
        ("n_blades", C.c_int32), ("n_per_blade", C.c_int32),
        ("hub", C.c_double * 3),
        ("omega", C.c_double), ("theta0", C.c_double), ("radius", C.c_double), ("u_inf", C.c_double),
        ("r", C.POINTER(C.c_double)), ("chord", C.POINTER(C.c_double)),
        ("twist", C.POINTER(C.c_double)), ("width", C.POINTER(C.c_double)),
        ("eps", C.c_double), ("cl_slope", C.c_double), ("alpha_clip", C.c_double),
        ("cd0", C.c_double), ("cd2", C.c_double),
        ("u_inf_correction", C.c_int32), ("tip_correction", C.c_int32),
        ("scale", C.c_void_p),
        ("line_points", C.c_int32), ("line_half_length", C.c_double),
    ]


class gks_motion(C.Structure):
    _fields_ = [("center", C.c_double * 3), ("velocity", C.c_double * 3), ("omega", C.c_double * 3),
                ("t0", C.c_double)]


class gks_forces_out(C.Structure):
    _fields_ = [
        ("t", C.c_double), ("dt", C.c_double), ("step", C.c_int64),
        ("thrust", C.c_double), ("torque", C.c_double), ("power", C.c_double),
        ("cp", C.c_double), ("ct", C.c_double),
        ("ibm_force", C.c_double * 3), ("ibm_residual", C.c_double),
        ("ibm_iters_used", C.c_int32), ("flags", C.c_int32),
        ("mass", C.c_double), ("mom", C.c_double * 3), ("umax", C.c_double),
        ("window_power", C.c_double), ("window_thrust", C.c_double), ("window_steps", C.c_int64),
        ("alpha", C.POINTER(C.c_double)), ("fx", C.POINTER(C.c_double)),
        ("ftheta", C.POINTER(C.c_double)), ("urel", C.POINTER(C.c_double)),
    ]


EXPORTS = (
    "gks_workspace_bytes", "gks_init", "gks_set_actuators", "gks_set_ibm_points", "gks_set_ibm_motion", "gks_step",
    "gks_forces", "gks_reset_window", "gks_field_changed", "gks_checkpoint_slot_bytes", "gks_set_checkpoints",
    "gks_adjoint_workspace_bytes", "gks_adjoint", "gks_set_timing", "gks_read_timing", "gks_destroy",
    "gks_last_error", "gks_statistics_bytes", "gks_set_statistics", "gks_read_statistics", "gks_set_history",
    "gks_history_count", "gks_init_static",
)
TIMERS = ("ghost", "dt", "s1x", "s1y", "s1z", "s2x", "s2y", "s2z", "alm", "ibm", "other")

_lib = None


def load(path: str = LIB_PATH):
    """Load libgks.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2603_11102_amd.build`")
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.gks_workspace_bytes.argtypes = [C.POINTER(gks_config)]
    lib.gks_workspace_bytes.restype = C.c_size_t
    lib.gks_init.argtypes = [C.POINTER(gks_config), gks_field, gks_field, gks_field, P, C.c_size_t, P, C.POINTER(P)]
    lib.gks_init.restype = C.c_int
    lib.gks_init_static.argtypes = [C.POINTER(gks_config), gks_field, gks_field, gks_field, P, C.POINTER(P)]
    lib.gks_init_static.restype = C.c_int
    lib.gks_set_actuators.argtypes = [P, C.POINTER(gks_rotor)]
    lib.gks_set_actuators.restype = C.c_int
    lib.gks_set_ibm_points.argtypes = [P, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double), P]
    lib.gks_set_ibm_points.restype = C.c_int
    lib.gks_set_ibm_motion.argtypes = [P, C.POINTER(gks_motion)]
    lib.gks_set_ibm_motion.restype = C.c_int
    lib.gks_step.argtypes = [P, C.c_int32]
    lib.gks_step.restype = C.c_int
    lib.gks_forces.argtypes = [P, C.POINTER(gks_forces_out)]
    lib.gks_forces.restype = C.c_int
    lib.gks_reset_window.argtypes = [P]
    lib.gks_reset_window.restype = C.c_int
    lib.gks_field_changed.argtypes = [P]
    lib.gks_field_changed.restype = C.c_int
    lib.gks_checkpoint_slot_bytes.argtypes = [C.POINTER(gks_config)]
    lib.gks_checkpoint_slot_bytes.restype = C.c_size_t
    lib.gks_set_checkpoints.argtypes = [P, P, C.c_int32]
    lib.gks_set_checkpoints.restype = C.c_int
    lib.gks_adjoint_workspace_bytes.argtypes = [C.POINTER(gks_config), C.c_int32]
    lib.gks_adjoint_workspace_bytes.restype = C.c_size_t
    lib.gks_adjoint.argtypes = [P, C.c_int32, C.POINTER(C.c_double), P, P, P, C.c_size_t, C.c_int32]
    lib.gks_adjoint.restype = C.c_int
    lib.gks_set_timing.argtypes = [P, C.c_int32]
    lib.gks_set_timing.restype = C.c_int
    lib.gks_read_timing.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]
    lib.gks_read_timing.restype = C.c_int
    lib.gks_statistics_bytes.argtypes = [C.POINTER(gks_config)]
    lib.gks_statistics_bytes.restype = C.c_size_t
    lib.gks_set_statistics.argtypes = [P, P, C.c_int32]
    lib.gks_set_statistics.restype = C.c_int
    lib.gks_read_statistics.argtypes = [P, C.c_double, P, P, P, P, C.POINTER(C.c_int64)]
    lib.gks_read_statistics.restype = C.c_int
    lib.gks_set_history.argtypes = [P, P, C.c_int32]
    lib.gks_set_history.restype = C.c_int
    lib.gks_history_count.argtypes = [P, C.POINTER(C.c_int64)]
    lib.gks_history_count.restype = C.c_int
    lib.gks_destroy.argtypes = [P]
    lib.gks_destroy.restype = None
    lib.gks_last_error.argtypes = [P]
    lib.gks_last_error.restype = C.c_char_p
    _lib = lib
    return lib


class GksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gks error {code}: {msg}")
        self.code = code


def last_error(lib, ctx) -> str:
    msg = lib.gks_last_error(ctx)
    return msg.decode() if msg else ""


def check(lib, ctx, rc):
    if rc != GKS_OK:
        msg = lib.gks_last_error(ctx)
        raise GksError(rc, msg.decode() if msg else "")
    return rc
