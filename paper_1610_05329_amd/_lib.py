"""ctypes declarations of libdgpe's C ABI (include/dgpe.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation of any step of the method.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgpe.so")

c_int32 = ctypes.c_int32
c_uint32 = ctypes.c_uint32
c_double = ctypes.c_double
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p
c_char_p = ctypes.c_char_p
P_int32 = ctypes.POINTER(c_int32)
P_double = ctypes.POINTER(c_double)

DGPE_OK = 0
STATUS_NAMES = {
    0: "DGPE_OK", 1: "DGPE_EINVAL", 2: "DGPE_EUNSUPPORTED_SIZE", 3: "DGPE_EWORKSPACE",
    4: "DGPE_EHIP", 5: "DGPE_ENONFINITE", 6: "DGPE_ESTATE",
}
DGPE_IMAG, DGPE_REAL, DGPE_F64, DGPE_F32 = 0, 1, 0, 2
Q2D = {None: 0, "perp": 4, "inplane": 8}  # DGPE_Q2D_PERP, DGPE_Q2D_INPLANE
PARAM = {"g": 0, "gd": 1, "nu": 2, "lambda": 3, "gamma": 4, "dt": 5, "real_time": 6, "fast_fft": 7,
         "fused_y": 8, "scheme": 9}
SCHEME = {"lie": 0, "strang": 1}
OBJECTIVE = {"energy": 0, "overlap": 1}
NPASS = 8
NOALLOC_MAX_BYTES = 64 << 20  # DGPE_NOALLOC_MAX_BYTES
PASS_NAMES = ["r2c_z", "fft_y", "fft_x_mul", "ifft_y", "c2r_z_nonlinear_cn_z", "cn_y", "cn_x", "norm_reduce"]


class DgpeObs(ctypes.Structure):
    _fields_ = [
        ("norm", c_double), ("mu", c_double), ("energy", c_double), ("e_kin", c_double),
        ("e_trap", c_double), ("e_contact", c_double), ("e_dd", c_double), ("rms", c_double * 4),
    ]


# name -> (restype, argtypes); the exported symbols of include/dgpe.h
SIGNATURES = {
    "dgpe_workspace_bytes": (c_size_t, [P_int32, c_uint32]),
    "dgpe_plan_create": (c_int32, [ctypes.POINTER(c_void_p), P_int32, P_double, c_double, P_double,
                                   c_double, c_double, c_double, c_uint32, c_void_p, c_size_t,
                                   c_void_p]),
    "dgpe_plan_create_noalloc": (c_int32, [ctypes.POINTER(c_void_p), P_int32, P_double, c_double,
                                           P_double, c_double, c_double, c_double, c_uint32,
                                           c_void_p]),
    "dgpe_plan_set": (c_int32, [c_void_p, c_int32, c_double]),
    "dgpe_plan_set_stream": (c_int32, [c_void_p, c_void_p]),
    "dgpe_plan_fused_y": (c_int32, [c_void_p]),
    "dgpe_step": (c_int32, [c_void_p, c_void_p, c_int32, P_double]),
    "dgpe_ground_state": (c_int32, [c_void_p, c_void_p, c_double, c_int32, c_int32, P_int32,
                                    P_double, ctypes.POINTER(DgpeObs)]),
    "dgpe_potential": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "dgpe_density": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "dgpe_write_density": (c_int32, [c_void_p, c_void_p, c_char_p]),
    "dgpe_energy_mu_rms": (c_int32, [c_void_p, c_void_p, c_double, ctypes.POINTER(DgpeObs)]),
    "dgpe_adjoint_workspace_bytes": (c_size_t, [c_void_p, c_int32, c_int32]),
    "dgpe_step_adjoint": (c_int32, [c_void_p, c_void_p, c_int32, P_double, c_int32, c_int32,
                                    c_void_p, c_void_p, c_size_t, c_void_p, P_double, P_double,
                                    P_double, c_void_p]),
    "dgpe_pass_bytes": (c_int32, [c_void_p, P_double]),
    "dgpe_step_profiled": (c_int32, [c_void_p, c_void_p, c_int32, P_double, P_double, P_double]),
    "dgpe_plan_destroy": (None, [c_void_p]),
    "dgpe_status_string": (c_char_p, [c_int32]),
    "dgpe_last_error": (c_char_p, []),
}

_lib = None


def load(path=LIB_PATH):
    """Load libdgpe.so and declare its signatures (cached)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is not built; run `python -m paper_1610_05329_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path == LIB_PATH:
        _lib = lib
    return lib


class DgpeError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")


def check(status):
    if status != DGPE_OK:
        raise DgpeError(status, load().dgpe_last_error().decode())
