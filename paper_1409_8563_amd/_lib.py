"""ctypes binding of libpr.so (include/pr.h).  Argument marshalling only:
every step of the computation runs in the library's HIP kernels.  torch is
used for device memory (tensors) and streams."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpr.so")

PR_OK, PR_EINVAL, PR_EUNSTABLE, PR_ENOMEM, PR_EDEVICE, PR_EUNSUPPORTED, PR_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
PR_FP32, PR_FP64 = 1, 2
PR_MODE_FP64, PR_MODE_MIXED, PR_MODE_PER_SLICE, PR_MODE_GRAPH, PR_MODE_TIMED = 0, 1, 16, 32, 64
PR_MODE_PIPELINED = 128


def PR_MODE_PIPELINE_GROUPS(g):
    """slice groups of PR_MODE_PIPELINED, OR-ed into a plan mode (1..255)"""
    return int(g) << 16

PR_DEFECT_STATIC_MAX_BATCH = 64
PR_NU_FROZEN, PR_ALLOW_UNSTABLE, PR_EARLY_STOP, PR_SKIP_CONVERGED, PR_COARSEN_G, PR_CUBIC_INTERP = 1, 2, 4, 8, 16, 32

STATUS_NAMES = {0: "PR_OK", -1: "PR_EINVAL", -2: "PR_EUNSTABLE", -3: "PR_ENOMEM", -4: "PR_EDEVICE",
                -5: "PR_EUNSUPPORTED", -6: "PR_ENONFINITE"}

# every symbol declared in include/pr.h
EXPORTS = ["pr_last_error", "pr_version", "pr_check_stability", "pr_fine_sweep", "pr_coarse_sweep",
           "pr_sweep_workspace_bytes", "pr_parareal_update", "pr_defect_norm", "pr_defect_workspace_bytes",
           "pr_plan_workspace_bytes", "pr_plan_create", "pr_plan_destroy", "pr_parareal_solve",
           "pr_plan_iterations", "pr_plan_kernel_variants", "pr_plan_fine_groups", "pr_plan_timings", "pr_plan_slice_state", "pr_set_kernel_variant",
           "pr_kernel_variant_count", "pr_kernel_variant_name", "pr_kernel_variant_info",
           "pr_autotune_workspace_bytes", "pr_autotune", "pr_plan_autotune", "pr_transfer_workspace_bytes",
           "pr_restrict", "pr_prolong", "pr_sweep_kernel_variant", "pr_defect_norm_static",
           "pr_defect_static_scratch_bytes", "pr_copy_probe", "pr_autotune_save", "pr_autotune_load",
           "pr_autotune_clear"]


class PrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, str(code)), msg))
        self.code = code


class PrProblem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("a", ctypes.c_double * 3), ("nu0", ctypes.c_double),
                ("nu_amp", ctypes.c_double), ("nu_omega", ctypes.c_double), ("T", ctypes.c_double),
                ("P", ctypes.c_int32), ("nt_fine", ctypes.c_int32), ("nt_coarse", ctypes.c_int32),
                ("K", ctypes.c_int32), ("fine_order", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("tol", ctypes.c_double)]


_lib = None
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load libpr.so from the package directory; raise if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libpr.so not found at %s: build it with `python -m paper_1409_8563_amd.build`"
                          % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    pp = ctypes.POINTER(PrProblem)
    L.pr_last_error.restype = ctypes.c_char_p
    L.pr_version.restype = ctypes.c_char_p
    L.pr_check_stability.argtypes = [pp, _dp, _dp]
    sweep = [pp, _i32, _i32, _vp, _vp, ctypes.POINTER(_i64), _i32, _vp, _sz, _vp]
    L.pr_fine_sweep.argtypes = sweep
    L.pr_coarse_sweep.argtypes = sweep
    L.pr_sweep_workspace_bytes.argtypes = [pp, _i32, _i32]
    L.pr_sweep_workspace_bytes.restype = _sz
    L.pr_parareal_update.argtypes = [_i64, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp]
    L.pr_defect_norm.argtypes = [_i64, _i32, _i32, _vp, _i32, _vp, _vp, _vp, _sz, _vp]
    L.pr_defect_workspace_bytes.argtypes = [_i32]
    L.pr_defect_workspace_bytes.restype = _sz
    L.pr_defect_norm_static.argtypes = [_i64, _i32, _i32, _vp, _i32, _vp, _vp, _vp]
    L.pr_defect_static_scratch_bytes.argtypes = []
    L.pr_defect_static_scratch_bytes.restype = _sz
    L.pr_copy_probe.argtypes = [_vp, _vp, _sz, _i32, _i32, _vp]
    L.pr_autotune_save.argtypes = [ctypes.c_char_p]
    L.pr_autotune_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(_i32)]
    L.pr_autotune_clear.argtypes = []
    L.pr_plan_workspace_bytes.argtypes = [pp, _i32, _i32]
    L.pr_plan_workspace_bytes.restype = _sz
    L.pr_plan_create.argtypes = [pp, _i32, _i32, _vp, _sz, ctypes.POINTER(_vp)]
    L.pr_plan_destroy.argtypes = [_vp]
    L.pr_plan_destroy.restype = None
    L.pr_parareal_solve.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _dp, _vp]
    L.pr_plan_iterations.argtypes = [_vp]
    L.pr_plan_kernel_variants.argtypes = [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]
    L.pr_plan_fine_groups.argtypes = [_vp, _i32] + [ctypes.POINTER(_i32)] * 4
    L.pr_plan_timings.argtypes = [_vp, _dp]
    L.pr_plan_slice_state.argtypes = [_vp, _i32, _i32, ctypes.POINTER(_vp)]
    L.pr_set_kernel_variant.argtypes = [_i32, _i32]
    L.pr_kernel_variant_count.argtypes = [_i32]
    L.pr_kernel_variant_name.argtypes = [_i32, _i32]
    L.pr_kernel_variant_name.restype = ctypes.c_char_p
    ip = ctypes.POINTER(_i32)
    L.pr_kernel_variant_info.argtypes = [_i32, _i32, ip, ip, ip, ip, ip, ip, ip]
    L.pr_autotune_workspace_bytes.argtypes = [pp, _i32, _i32]
    L.pr_autotune_workspace_bytes.restype = _sz
    L.pr_autotune.argtypes = [pp, _i32, _i32, _i32, _vp, _sz, _vp, ip]
    L.pr_plan_autotune.argtypes = [_vp, _vp, ip, ip, ip, ip]
    L.pr_sweep_kernel_variant.argtypes = [pp, _i32, _i32, _i32, ip]
    L.pr_transfer_workspace_bytes.argtypes = [_i32]
    L.pr_transfer_workspace_bytes.restype = _sz
    L.pr_restrict.argtypes = [pp, _i32, _i32, _vp, _vp, _vp, _sz, _vp]
    L.pr_prolong.argtypes = [pp, _i32, _i32, _i32, _vp, _vp, _vp, _sz, _vp]
    _lib = L
    return L


def check(rc):
    if rc != PR_OK:
        raise PrError(rc, lib().pr_last_error().decode())
    return rc


def last_error() -> str:
    return lib().pr_last_error().decode()


def to_struct(p) -> PrProblem:
    """Build the C struct from a workloads.Problem (or any object with the same fields)."""
    s = PrProblem()
    for d in range(3):
        s.n[d] = int(p.n[d])
        s.a[d] = float(p.a[d])
    s.nu0 = float(p.nu0)
    s.nu_amp = float(p.nu_amp)
    s.nu_omega = float(p.nu_omega)
    s.T = float(p.T)
    s.P = int(p.P)
    s.nt_fine = int(p.nt_fine)
    s.nt_coarse = int(p.nt_coarse)
    s.K = int(p.K)
    s.fine_order = int(p.fine_order)
    s.flags = int(getattr(p, "flags", 0))
    s.tol = float(getattr(p, "tol", 0.0))
    return s
