"""CPU oracle for Parareal over 3D advection-diffusion stencils.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
calls it and it never calls the GPU library; the two share nothing but the
seeded input generators of ``workloads``.

``oracle.c`` is the plain serial FP64 grid implementation (compiled with gcc,
``-O2 -ffp-contract=off``, optional OpenMP over z with thread-count
independent results).  ``spectral.py`` is an independent per-Fourier-mode
reference of the same discrete scheme.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, FP64, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c11", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class OrProb(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("order", ctypes.c_int32),
                ("ax", ctypes.c_double), ("ay", ctypes.c_double), ("az", ctypes.c_double),
                ("nu0", ctypes.c_double), ("nu_amp", ctypes.c_double), ("nu_omega", ctypes.c_double),
                ("T", ctypes.c_double),
                ("P", ctypes.c_int32), ("nt_fine", ctypes.c_int32), ("nt_coarse", ctypes.c_int32),
                ("nu_frozen", ctypes.c_int32), ("coarsen", ctypes.c_int32), ("interp_order", ctypes.c_int32)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        pp = ctypes.POINTER(OrProb)
        L.or_nu.argtypes = [pp, ctypes.c_double]
        L.or_nu.restype = ctypes.c_double
        L.or_fine_rhs.argtypes = [pp, ctypes.c_double, _dp, _dp]
        L.or_coarse_rhs.argtypes = [pp, ctypes.c_double, _dp, _dp]
        L.or_rk4_step_alloc.argtypes = [pp, ctypes.c_long, _dp, _dp]
        L.or_euler_step_alloc.argtypes = [pp, ctypes.c_long, _dp, _dp]
        L.or_fine_steps.argtypes = [pp, ctypes.c_long, ctypes.c_int, _dp, _dp]
        L.or_coarse_steps.argtypes = [pp, ctypes.c_long, ctypes.c_int, _dp, _dp]
        L.or_serial_fine.argtypes = [pp, _dp, _dp, _dp]
        L.or_serial_coarse.argtypes = [pp, _dp, _dp, _dp]
        L.or_parareal.argtypes = [pp, ctypes.c_int, _dp, _dp, _dp, _dp]
        L.or_norms.argtypes = [ctypes.c_long, _dp, _dp, _dp]
        L.or_restrict.argtypes = [pp, _dp, _dp]
        L.or_restrict.restype = None
        L.or_prolong.argtypes = [pp, ctypes.c_int, _dp, _dp]
        L.or_prolong.restype = None
        L.or_threads.restype = ctypes.c_int
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_set_threads.restype = None
        for f in ("or_rk4_step_alloc", "or_euler_step_alloc", "or_fine_steps", "or_coarse_steps",
                  "or_serial_fine", "or_serial_coarse", "or_parareal"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _prob(p) -> OrProb:
    """Convert a workloads.Problem into the oracle's struct."""
    flags = int(getattr(p, "flags", 0))
    nu_frozen = 1 if flags & 1 else 0
    coarsen = 1 if flags & 16 else 0
    order = 3 if flags & 32 else 1
    return OrProb(int(p.n[0]), int(p.n[1]), int(p.n[2]), int(p.fine_order),
                  float(p.a[0]), float(p.a[1]), float(p.a[2]),
                  float(p.nu0), float(p.nu_amp), float(p.nu_omega), float(p.T),
                  int(p.P), int(p.nt_fine), int(p.nt_coarse), nu_frozen, coarsen, order)


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _field(p, u) -> np.ndarray:
    nx, ny, nz = (int(v) for v in p.n)
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert u.size == nx * ny * nz
    return u.reshape(nz, ny, nx)


def restrict(p, u) -> np.ndarray:
    """Injection onto the grid coarsened by 2 per direction ([nz/2, ny/2, nx/2])."""
    s = _prob(p)
    u = _field(p, u)
    nx, ny, nz = (int(v) for v in p.n)
    out = np.empty((nz // 2, ny // 2, nx // 2))
    lib().or_restrict(ctypes.byref(s), _ptr(u), _ptr(out))
    return out


def prolong(p, uc, order: int = 1) -> np.ndarray:
    """Interpolation (order 1 or 3) from the coarsened grid to the grid of p."""
    s = _prob(p)
    nx, ny, nz = (int(v) for v in p.n)
    uc = np.ascontiguousarray(uc, dtype=np.float64).reshape(nz // 2, ny // 2, nx // 2)
    out = np.empty((nz, ny, nx))
    lib().or_prolong(ctypes.byref(s), int(order), _ptr(uc), _ptr(out))
    return out


def threads() -> int:
    """OpenMP threads used by the oracle's z loops."""
    return int(lib().or_threads())


def set_threads(n: int) -> None:
    """Run the oracle's z loops on n threads from now on (same results)."""
    lib().or_set_threads(int(n))


def nu(p, t: float) -> float:
    s = _prob(p)
    return lib().or_nu(ctypes.byref(s), float(t))


def fine_rhs(p, nu_val: float, u) -> np.ndarray:
    s = _prob(p)
    u = _field(p, u)
    out = np.empty_like(u)
    lib().or_fine_rhs(ctypes.byref(s), float(nu_val), _ptr(u), _ptr(out))
    return out


def coarse_rhs(p, nu_val: float, u) -> np.ndarray:
    s = _prob(p)
    u = _field(p, u)
    out = np.empty_like(u)
    lib().or_coarse_rhs(ctypes.byref(s), float(nu_val), _ptr(u), _ptr(out))
    return out


def rk4_step(p, j: int, u) -> np.ndarray:
    s = _prob(p)
    u = _field(p, u)
    out = np.empty_like(u)
    assert lib().or_rk4_step_alloc(ctypes.byref(s), int(j), _ptr(u), _ptr(out)) == 0
    return out


def euler_step(p, j: int, u) -> np.ndarray:
    s = _prob(p)
    u = _field(p, u)
    out = np.empty_like(u)
    assert lib().or_euler_step_alloc(ctypes.byref(s), int(j), _ptr(u), _ptr(out)) == 0
    return out


def fine_steps(p, j0: int, nsteps: int, u) -> np.ndarray:
    s = _prob(p)
    u = _field(p, u)
    out = np.empty_like(u)
    assert lib().or_fine_steps(ctypes.byref(s), int(j0), int(nsteps), _ptr(u), _ptr(out)) == 0
    return out


def coarse_steps(p, j0: int, nsteps: int, u) -> np.ndarray:
    s = _prob(p)
    u = _field(p, u)
    out = np.empty_like(u)
    assert lib().or_coarse_steps(ctypes.byref(s), int(j0), int(nsteps), _ptr(u), _ptr(out)) == 0
    return out


def fine_prop(p, slice_index: int, u) -> np.ndarray:
    return fine_steps(p, slice_index * p.nf, p.nf, u)


def coarse_prop(p, slice_index: int, u) -> np.ndarray:
    return coarse_steps(p, slice_index * p.nc, p.nc, u)


def serial_fine(p, u0, trajectory: bool = False):
    s = _prob(p)
    u0 = _field(p, u0)
    out = np.empty_like(u0)
    traj = np.empty((p.P + 1,) + u0.shape) if trajectory else None
    assert lib().or_serial_fine(ctypes.byref(s), _ptr(u0), _ptr(out),
                                _ptr(traj) if trajectory else None) == 0
    return (out, traj) if trajectory else out


def serial_coarse(p, u0, trajectory: bool = False):
    s = _prob(p)
    u0 = _field(p, u0)
    out = np.empty_like(u0)
    traj = np.empty((p.P + 1,) + u0.shape) if trajectory else None
    assert lib().or_serial_coarse(ctypes.byref(s), _ptr(u0), _ptr(out),
                                  _ptr(traj) if trajectory else None) == 0
    return (out, traj) if trajectory else out


def parareal(p, u0, K: int = None, history: bool = False):
    """Run K Parareal iterations.  Returns (U, log) or (U, log, hist):
    U[s] = U^K_s for s = 0..P, log[k] the 8 inter-iterate norms of iteration k,
    hist[k, s] = U^k_s."""
    K = p.K if K is None else int(K)
    s = _prob(p)
    u0 = _field(p, u0)
    U = np.empty((p.P + 1,) + u0.shape)
    log = np.zeros((max(K, 1), 8))
    hist = np.empty((K + 1, p.P + 1) + u0.shape) if history else None
    rc = lib().or_parareal(ctypes.byref(s), K, _ptr(u0), _ptr(U),
                           _ptr(hist) if history else None, _ptr(log))
    assert rc == 0
    log = log[:K]
    return (U, log, hist) if history else (U, log)


def norms(x, ref) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    ref = np.ascontiguousarray(ref, dtype=np.float64).ravel()
    assert x.size == ref.size
    out = np.zeros(4)
    lib().or_norms(x.size, _ptr(x), _ptr(ref), _ptr(out))
    return out


def rel_l2(x, ref) -> float:
    n = norms(x, ref)
    return float(np.sqrt(n[2] / n[3])) if n[3] > 0 else float(np.sqrt(n[2]))


def rel_inf(x, ref) -> float:
    """d = ||x - ref||_inf / ||ref||_inf  (eq. defect)."""
    n = norms(x, ref)
    return float(n[0] / n[1]) if n[1] > 0 else float(n[0])
