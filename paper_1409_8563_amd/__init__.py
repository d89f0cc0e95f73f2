"""Parareal over 3D advection-diffusion stencils on MI355X (gfx950).

Python face of libpr.so (include/pr.h): the fine propagator F (RK4), the
coarse propagator G (Euler, upwind), the Parareal correction, the defect
norms and the batched Parareal solve.  All computation happens in the HIP
library; this module passes torch tensors' device pointers and streams.
The functions raise ImportError if the library was not built and
``PrError`` for any non-OK status.
"""
from __future__ import annotations

import ctypes
import os

from . import _lib as L
from ._lib import (PR_ALLOW_UNSTABLE, PR_COARSEN_G, PR_CUBIC_INTERP, PR_EARLY_STOP, PR_FP32,  # noqa: F401
                   PR_FP64, PR_MODE_FP64, PR_MODE_GRAPH, PR_MODE_MIXED, PR_MODE_PER_SLICE,
                   PR_MODE_PIPELINE_GROUPS, PR_MODE_PIPELINED, PR_MODE_TIMED,
                   PR_NU_FROZEN, PR_SKIP_CONVERGED, PrError, check, lib, to_struct)

__all__ = ["fine_sweep", "coarse_sweep", "parareal_update", "defect_norm", "restrict", "prolong",
           "Plan",
           "check_stability", "set_kernel_variant", "variants", "sweep_kernel_variant", "autotune", "PrError",
           "lib"]


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return PR_FP64
    if t.dtype == torch.float32:
        return PR_FP32
    raise TypeError("fields must be float32 or float64, got %s" % t.dtype)


def _shape(t, name, numel=None, dtype=None):
    """Check a tensor handed to the library: a torch tensor of the expected
    dtype and element count, contiguous.  The library receives bare device
    pointers and cannot check sizes itself, so a short buffer would be read
    or written out of bounds on the device.  Runs before any device check, so
    every rejection here is exercised without a GPU."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must hold %d values, got %d" % (name, numel, t.numel()))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def _ptr(t, name, like=None):
    """Device pointer of a checked tensor; it must live on the GPU, on the
    device of `like` when given."""
    if not t.is_cuda:
        raise ValueError("%s must live on the GPU" % name)
    if like is not None and t.device != like.device:
        raise ValueError("%s is on %s, expected %s" % (name, t.device, like.device))
    return ctypes.c_void_p(t.data_ptr())


def _dev(t):
    return _ptr(_shape(t, "tensor"), "tensor")


def _workspace(nbytes, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _keep_alive(stream, *tensors):
    """Tensors allocated here but used by kernels queued on a stream other
    than the current one: tell the caching allocator, so their memory is not
    handed to the current stream while those kernels still run."""
    torch = _torch()
    if stream is None or stream == torch.cuda.current_stream():
        return
    for t in tensors:
        if t is not None:
            t.record_stream(stream)


def _sweep(fn, prob, u_in, step0, nsteps, u_out, stream):
    torch = _torch()
    s = to_struct(prob)
    nx, ny, nz = (int(v) for v in prob.n)
    npts = nx * ny * nz
    dt = _code(u_in)
    _shape(u_in, "u_in")
    if npts <= 0 or u_in.numel() == 0 or u_in.numel() % npts:
        raise ValueError("u_in size is not a positive multiple of the grid size")
    batch = u_in.numel() // npts
    if u_out is not None:
        _shape(u_out, "u_out", numel=u_in.numel(), dtype=u_in.dtype)
    s0 = [int(step0)] * batch if isinstance(step0, int) else [int(v) for v in step0]
    if len(s0) != batch:
        raise ValueError("step0 needs one entry per field (%d), got %d" % (batch, len(s0)))
    pin = _ptr(u_in, "u_in")
    made = u_out is None
    if made:
        u_out = torch.empty_like(u_in)
    pout = _ptr(u_out, "u_out", like=u_in)
    steps = (ctypes.c_int64 * batch)(*s0)
    ws = _workspace(lib().pr_sweep_workspace_bytes(ctypes.byref(s), dt, batch), u_in.device)
    check(fn(ctypes.byref(s), dt, batch, pin, pout, steps, int(nsteps),
             ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)))
    _keep_alive(stream, ws, u_out if made else None)
    return u_out


def fine_sweep(prob, u_in, step0, nsteps, u_out=None, stream=None):
    """nsteps RK4 steps of F on every field of u_in (shape [..., nz, ny, nx]);
    step0 is the global fine step index of the first step (int or one per field)."""
    return _sweep(lib().pr_fine_sweep, prob, u_in, step0, nsteps, u_out, stream)


def coarse_sweep(prob, u_in, step0, nsteps, u_out=None, stream=None):
    """nsteps forward Euler / upwind steps of G (Algorithm 2)."""
    return _sweep(lib().pr_coarse_sweep, prob, u_in, step0, nsteps, u_out, stream)


def _transfer(prob, u_in, order, prolong, stream):
    torch = _torch()
    s = to_struct(prob)
    nx, ny, nz = (int(v) for v in prob.n)
    fine, coarse = nx * ny * nz, (nx // 2) * (ny // 2) * (nz // 2)
    n_in = coarse if prolong else fine
    dt = _code(u_in)
    _shape(u_in, "u_in")
    if n_in <= 0 or u_in.numel() == 0 or u_in.numel() % n_in:
        raise ValueError("input size is not a positive multiple of the %s grid size"
                         % ("coarse" if prolong else "fine"))
    batch = u_in.numel() // n_in
    pin = _ptr(u_in, "u_in")
    shape = (batch, nz, ny, nx) if prolong else (batch, nz // 2, ny // 2, nx // 2)
    out = torch.empty(shape, dtype=u_in.dtype, device=u_in.device)
    ws = _workspace(lib().pr_transfer_workspace_bytes(batch), u_in.device)
    if prolong:
        check(lib().pr_prolong(ctypes.byref(s), dt, int(order), batch, pin, _ptr(out, "out"),
                               ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)))
    else:
        check(lib().pr_restrict(ctypes.byref(s), dt, batch, pin, _ptr(out, "out"), ctypes.c_void_p(ws.data_ptr()),
                                ws.numel(), _stream_ptr(stream)))
    _keep_alive(stream, ws, out)
    return out


def restrict(prob, u_fine, stream=None):
    """Injection of fine fields (grid of prob) onto the grid coarsened by 2: [batch, nz/2, ny/2, nx/2]."""
    return _transfer(prob, u_fine, 1, False, stream)


def prolong(prob, u_coarse, order=1, stream=None):
    """Interpolation (order 1 or 3) of coarse fields to the grid of prob: [batch, nz, ny, nx]."""
    return _transfer(prob, u_coarse, order, True, stream)


def parareal_update(f_new, g_new, g_old, u_out=None, u_out_lo=None, stream=None):
    """u_out = f_new + (g_new - g_old) in FP64; optional rounded copy u_out_lo.
    g_new, g_old and u_out_lo have f_new's dtype and size; u_out is FP64."""
    torch = _torch()
    dt = _code(f_new)
    n = _shape(f_new, "f_new").numel()
    _shape(g_new, "g_new", numel=n, dtype=f_new.dtype)
    _shape(g_old, "g_old", numel=n, dtype=f_new.dtype)
    if u_out is not None:
        _shape(u_out, "u_out", numel=n, dtype=torch.float64)
    if u_out_lo is not None:
        _shape(u_out_lo, "u_out_lo", numel=n, dtype=f_new.dtype)
    pf = _ptr(f_new, "f_new")
    pgn = _ptr(g_new, "g_new", like=f_new)
    pgo = _ptr(g_old, "g_old", like=f_new)
    made = u_out is None
    if made:
        u_out = torch.empty(f_new.shape, dtype=torch.float64, device=f_new.device)
    pu = _ptr(u_out, "u_out", like=f_new)
    plo = _ptr(u_out_lo, "u_out_lo", like=f_new) if u_out_lo is not None else None
    check(lib().pr_parareal_update(n, 1, dt, pf, pgn, pgo, pu, plo, _stream_ptr(stream)))
    _keep_alive(stream, u_out if made else None)
    return u_out


def defect_norm(x, ref, batch=1, stream=None):
    """Device tensor [batch, 4]: max|x-r|, max|r|, sum (x-r)^2, sum r^2.
    x and ref hold the same number of values (FP32 or FP64 each)."""
    torch = _torch()
    xd, rd = _code(x), _code(ref)
    batch = int(batch)
    _shape(x, "x")
    if batch < 1 or x.numel() == 0 or x.numel() % batch:
        raise ValueError("x must hold a positive multiple of batch values")
    _shape(ref, "ref", numel=x.numel())
    n = x.numel() // batch
    px = _ptr(x, "x")
    pref = _ptr(ref, "ref", like=x)
    out = torch.empty((batch, 4), dtype=torch.float64, device=x.device)
    ws = _workspace(lib().pr_defect_workspace_bytes(batch), x.device)
    check(lib().pr_defect_norm(n, batch, xd, px, rd, pref, _ptr(out, "out"),
                               ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)))
    _keep_alive(stream, ws, out)
    return out


def defect_norm_static(x, ref, batch=1, out=None, stream=None):
    """defect_norm through the allocation-free entry point: the library's own
    per-GPU scratch array replaces the workspace; `out` ([batch, 4] FP64) may
    be supplied so that the call allocates nothing at all."""
    torch = _torch()
    xd, rd = _code(x), _code(ref)
    batch = int(batch)
    _shape(x, "x")
    if batch < 1 or x.numel() == 0 or x.numel() % batch:
        raise ValueError("x must hold a positive multiple of batch values")
    _shape(ref, "ref", numel=x.numel())
    n = x.numel() // batch
    px = _ptr(x, "x")
    pref = _ptr(ref, "ref", like=x)
    made = out is None
    if made:
        out = torch.empty((batch, 4), dtype=torch.float64, device=x.device)
    _shape(out, "out", numel=4 * batch, dtype=torch.float64)
    check(lib().pr_defect_norm_static(n, batch, xd, px, rd, pref, _ptr(out, "out", like=x), _stream_ptr(stream)))
    _keep_alive(stream, out if made else None)
    return out


def copy_probe(src, dst, variant=0, blocks_per_cu=0, stream=None):
    """Copy src into dst (same byte count, multiple of 16) with the library's
    bandwidth-probe kernel."""
    _shape(src, "src")
    _shape(dst, "dst")
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("src and dst must hold the same number of bytes")
    check(lib().pr_copy_probe(_ptr(src, "src"), _ptr(dst, "dst", like=src), nb, int(variant), int(blocks_per_cu),
                              _stream_ptr(stream)))
    return dst


def autotune_save(path):
    """Write the library's tuned-kernel table as JSON to `path`."""
    check(lib().pr_autotune_save(os.fsencode(path)))


def autotune_load(path):
    """Merge a saved tuned-kernel table; returns the number of entries merged."""
    n = ctypes.c_int32(0)
    check(lib().pr_autotune_load(os.fsencode(path), ctypes.byref(n)))
    return n.value


def autotune_clear():
    check(lib().pr_autotune_clear())


def check_stability(prob):
    """(status, fine_margin, coarse_margin); margins <= 1 are stable."""
    s = to_struct(prob)
    fm, cm = ctypes.c_double(0), ctypes.c_double(0)
    rc = lib().pr_check_stability(ctypes.byref(s), ctypes.byref(fm), ctypes.byref(cm))
    return rc, fm.value, cm.value


def set_kernel_variant(fine=0, coarse=0):
    check(lib().pr_set_kernel_variant(int(fine), int(coarse)))


def variants(which):
    """List of dicts describing the fused variants of F (which=0) or G (which=1)."""
    out = []
    for v in range(2, lib().pr_kernel_variant_count(which)):
        vals = [ctypes.c_int32() for _ in range(7)]
        check(lib().pr_kernel_variant_info(which, v, *[ctypes.byref(x) for x in vals]))
        out.append(dict(index=v, name=lib().pr_kernel_variant_name(which, v).decode(), dtype=vals[0].value,
                        order=vals[1].value, tile=(vals[2].value, vals[3].value), nxp=vals[4].value,
                        steps=vals[5].value, nx_exact=vals[6].value))
    return out


def sweep_kernel_variant(prob, dtype, batch, which):
    """Name of the fused variant a sweep would launch (which: 0 = F, 1 = G)."""
    s = to_struct(prob)
    v = ctypes.c_int32()
    check(lib().pr_sweep_kernel_variant(ctypes.byref(s), int(dtype), int(batch), int(which), ctypes.byref(v)))
    return lib().pr_kernel_variant_name(int(which), v.value).decode()


def autotune(prob, dtype, batch, which, stream=None):
    torch = _torch()
    s = to_struct(prob)
    nb = lib().pr_autotune_workspace_bytes(ctypes.byref(s), dtype, batch)
    ws = _workspace(nb, torch.device("cuda"))
    best = ctypes.c_int32(0)
    check(lib().pr_autotune(ctypes.byref(s), dtype, batch, which, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                            _stream_ptr(stream), ctypes.byref(best)))
    return best.value


class Plan:
    """A validated batched Parareal solve over one or more problem instances."""

    def __init__(self, probs, mode=PR_MODE_FP64, device=None):
        torch = _torch()
        if not isinstance(probs, (list, tuple)):
            probs = [probs]
        self.probs = list(probs)
        self.mode = int(mode)
        self._arr = (L.PrProblem * len(probs))(*[to_struct(p) for p in probs])
        nb = lib().pr_plan_workspace_bytes(self._arr, len(probs), self.mode)
        if nb == 0:
            # reproduce the validation error
            h = ctypes.c_void_p()
            check(lib().pr_plan_create(self._arr, len(probs), self.mode, None, 0, ctypes.byref(h)))
        self.ws = _workspace(nb, device or torch.device("cuda"))
        self._h = ctypes.c_void_p()
        check(lib().pr_plan_create(self._arr, len(probs), self.mode, ctypes.c_void_p(self.ws.data_ptr()),
                                   self.ws.numel(), ctypes.byref(self._h)))

    def solve(self, u0, uT=None, ref=None, want_log=True, stream=None):
        """u0: list of FP64 device tensors (one per instance).  Returns (uT list,
        log numpy [ninst, K, 12] or None).  Blocking."""
        import numpy as np
        torch = _torch()
        n = len(self.probs)
        if len(u0) != n or (uT is not None and len(uT) != n) or (ref is not None and len(ref) != n):
            raise ValueError("u0, uT and ref need one tensor per instance (%d)" % n)
        npts = [int(p.n[0]) * int(p.n[1]) * int(p.n[2]) for p in self.probs]
        groups = [("u0", u0)] + ([("uT", uT)] if uT is not None else []) + ([("ref", ref)] if ref is not None else [])
        for name, ts in groups:
            for i, x in enumerate(ts):
                _shape(x, "%s[%d]" % (name, i), numel=npts[i], dtype=torch.float64)
        for name, ts in groups:
            for i, x in enumerate(ts):
                _ptr(x, "%s[%d]" % (name, i), like=self.ws)
        if uT is None:
            uT = [torch.empty_like(x) for x in u0]
        pu0 = (ctypes.c_void_p * n)(*[x.data_ptr() for x in u0])
        puT = (ctypes.c_void_p * n)(*[x.data_ptr() for x in uT])
        pref = (ctypes.c_void_p * n)(*[x.data_ptr() for x in ref]) if ref is not None else None
        K = int(self.probs[0].K)
        log = np.zeros((n, max(K, 1), 12)) if want_log else None
        lp = log.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if want_log else None
        rc = lib().pr_parareal_solve(self._h, pu0, puT, pref, lp, _stream_ptr(stream))
        check(rc)
        if want_log:
            log = log[:, :K]
        return uT, log

    def autotune(self, stream=None):
        """Tune the plan's F and G launches (variant, blocks per CU); returns
        {"fine": (name, bpc), "coarse": (name, bpc)}.  Blocking."""
        vals = [ctypes.c_int32() for _ in range(4)]
        check(lib().pr_plan_autotune(self._h, _stream_ptr(stream), *[ctypes.byref(v) for v in vals]))
        return {"fine": (lib().pr_kernel_variant_name(0, vals[0].value).decode(), vals[1].value),
                "coarse": (lib().pr_kernel_variant_name(1, vals[2].value).decode(), vals[3].value)}

    def iterations(self):
        return lib().pr_plan_iterations(self._h)

    def kernel_variants(self):
        """(fine, coarse) kernel variant names launched by this plan."""
        f, c = ctypes.c_int32(), ctypes.c_int32()
        check(lib().pr_plan_kernel_variants(self._h, ctypes.byref(f), ctypes.byref(c)))
        return (lib().pr_kernel_variant_name(0, f.value).decode(), lib().pr_kernel_variant_name(1, c.value).decode())

    def fine_groups(self):
        """F launch groups: list of (variant name, blocks per CU, instances)."""
        cnt = ctypes.c_int32()
        check(lib().pr_plan_fine_groups(self._h, 0, ctypes.byref(cnt), None, None, None))
        n = cnt.value
        v, b, i = (ctypes.c_int32 * n)(), (ctypes.c_int32 * n)(), (ctypes.c_int32 * n)()
        check(lib().pr_plan_fine_groups(self._h, n, ctypes.byref(cnt), v, b, i))
        return [(lib().pr_kernel_variant_name(0, v[g]).decode(), b[g], i[g]) for g in range(n)]

    def timings(self):
        out = (ctypes.c_double * 6)()
        check(lib().pr_plan_timings(self._h, out))
        return dict(fine_ms=out[0], coarse_chain_ms=out[1], init_ms=out[2], fine_launches=out[3],
                    coarse_launches=out[4], total_ms=out[5])

    def slice_state(self, inst, n):
        """FP64 tensor view (no copy) of the current U_n of instance `inst`."""
        torch = _torch()
        p = ctypes.c_void_p()
        check(lib().pr_plan_slice_state(self._h, int(inst), int(n), ctypes.byref(p)))
        nx, ny, nz = (int(v) for v in self.probs[inst].n)
        off = p.value - self.ws.data_ptr()
        return self.ws[off:off + nx * ny * nz * 8].view(torch.float64).view(nz, ny, nx)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().pr_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
