"""The C-ABI library loads, exports every declared symbol, and validates its
arguments without a GPU (device work fails with PR_EDEVICE).  CPU only."""
import ctypes
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1409_8563_amd import _lib as L
    return L


def header_functions():
    txt = open(os.path.join(ROOT, "include", "pr.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pr_[a-z0-9_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    L = _lib()
    assert header_functions() == sorted(L.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = _lib()
    so = ctypes.CDLL(L.LIB_PATH)
    for name in header_functions():
        assert hasattr(so, name), name


def test_version_and_error_string():
    L = _lib()
    assert L.lib().pr_version().startswith(b"pr ")
    assert isinstance(L.last_error(), str)


def _status(fn, *args):
    return fn(*args)


@pytest.mark.parametrize("name", ["c2_128_fp64", "c3_256_mixed", "c5_512_mixed"])
def test_literal_coarse_counts_rejected_stabilised_accepted(name):
    """Forward Euler/upwind with the literal coarse step counts violates
    Dt (sum|a|/h + 2 nu_max sum 1/h^2) <= 1; the raised counts satisfy it."""
    import paper_1409_8563_amd as pr
    p, _ = W.config(name)
    rc, fm, cm = pr.check_stability(p)
    assert rc == 0 and cm <= 0.9 + 1e-12 and fm <= 1.0 + 1e-12
    p.nt_coarse = W.LITERAL_COARSE[name]
    rc, fm, cm = pr.check_stability(p)
    assert rc == _lib().PR_EUNSTABLE and cm > 1.5
    L = _lib()
    arr = (L.PrProblem * 1)(L.to_struct(p))
    assert L.lib().pr_plan_workspace_bytes(arr, 1, 0) == 0
    h = ctypes.c_void_p()
    assert L.lib().pr_plan_create(arr, 1, 0, None, 0, ctypes.byref(h)) == L.PR_EUNSTABLE
    p.flags |= W.ALLOW_UNSTABLE
    arr = (L.PrProblem * 1)(L.to_struct(p))
    assert L.lib().pr_plan_workspace_bytes(arr, 1, 0) > 0


def test_coarse_margin_formula():
    import paper_1409_8563_amd as pr
    p, _ = W.config("c1_32_fp64")
    _, _, cm = pr.check_stability(p)
    expect = (p.T / p.nt_coarse) * W.coarse_bound(p.n, p.a, p.nu0 * 1.5)
    assert abs(cm - expect) <= 1e-12 * expect


def test_fine_margin_detects_unstable_rk4():
    import paper_1409_8563_amd as pr
    p = W.small_problem(n=(32, 32, 32), nu0=0.5, nf=1, nc=200, P=1, T=0.05)
    rc, fm, _ = pr.check_stability(p)
    assert fm > 1.0 and rc == _lib().PR_EUNSTABLE


def test_batched_instances_all_stable():
    import paper_1409_8563_amd as pr
    for p, _ in W.batched_config(64):
        rc, fm, cm = pr.check_stability(p)
        assert rc == 0, (p.n, cm)


def _sweep_rc(p, **kw):
    L = _lib()
    s = L.to_struct(p)
    args = dict(dtype=2, batch=1, u_in=1 << 20, u_out=1 << 40, step0=(ctypes.c_int64 * 1)(0), nsteps=1,
                ws=1 << 42, ws_bytes=1 << 40)
    args.update(kw)
    return L.lib().pr_fine_sweep(ctypes.byref(s), args["dtype"], args["batch"], ctypes.c_void_p(args["u_in"]),
                                 ctypes.c_void_p(args["u_out"]), args["step0"], args["nsteps"],
                                 ctypes.c_void_p(args["ws"]), args["ws_bytes"], None)


def test_sweep_validation_without_device():
    L = _lib()
    p = W.small_problem(n=(16, 16, 16))
    assert _sweep_rc(p) == L.PR_EDEVICE                      # valid request, no GPU here
    assert _sweep_rc(p, dtype=3) == L.PR_EINVAL
    assert _sweep_rc(p, batch=0) == L.PR_EINVAL
    assert _sweep_rc(p, nsteps=-1) == L.PR_EINVAL
    assert _sweep_rc(p, u_out=(1 << 20) + 16) == L.PR_EINVAL  # overlapping fields
    assert _sweep_rc(p, u_out=(1 << 30) + 8) == L.PR_EINVAL   # misaligned
    assert _sweep_rc(p, ws_bytes=16) == L.PR_ENOMEM
    assert _sweep_rc(p, step0=(ctypes.c_int64 * 1)(-1)) == L.PR_EINVAL
    bad = W.small_problem(n=(2, 16, 16))
    assert _sweep_rc(bad) == L.PR_EINVAL
    bad = W.small_problem(n=(16, 16, 16))
    bad.nu0 = 0.0
    assert _sweep_rc(bad) == L.PR_EINVAL
    bad = W.small_problem(n=(16, 16, 16))
    bad.nu_amp = 1.0
    assert _sweep_rc(bad) == L.PR_EINVAL
    bad = W.small_problem(n=(4, 16, 16), order=4)
    assert _sweep_rc(bad) == L.PR_EINVAL
    assert "n[0]" in L.last_error()
    # the largest field a kernel can index with 32-bit point offsets: 2^31 - 1 points
    bad = W.small_problem(n=(1291, 1291, 1291))
    assert _sweep_rc(bad) == L.PR_EINVAL and "2^31" in L.last_error()
    ok = W.small_problem(n=(1024, 1024, 1024))
    ok.flags |= W.ALLOW_UNSTABLE
    assert _sweep_rc(ok) in (L.PR_EDEVICE, L.PR_ENOMEM)


def test_plan_validation():
    L = _lib()
    good = W.small_problem(n=(16, 16, 16), P=4, K=2)

    def rc_for(*probs, mode=0):
        arr = (L.PrProblem * len(probs))(*[L.to_struct(q) for q in probs])
        h = ctypes.c_void_p()
        return L.lib().pr_plan_create(arr, len(probs), mode, ctypes.c_void_p(1 << 40), 1 << 50, ctypes.byref(h))

    assert rc_for(good) == L.PR_EDEVICE
    bad = W.small_problem(n=(16, 16, 16), P=4, K=5)
    assert rc_for(bad) == L.PR_EINVAL
    bad = W.small_problem(n=(16, 16, 16), P=4, K=2)
    bad.nt_fine = 10
    assert rc_for(bad) == L.PR_EINVAL
    other = W.small_problem(n=(16, 16, 16), P=4, K=1)
    assert rc_for(good, other) == L.PR_EINVAL               # K differs
    assert rc_for(good, mode=1 << 10) == L.PR_EINVAL
    arr = (L.PrProblem * 1)(L.to_struct(good))
    h = ctypes.c_void_p()
    assert L.lib().pr_plan_create(arr, 1, 0, ctypes.c_void_p(1 << 40), 100, ctypes.byref(h)) == L.PR_ENOMEM


def test_pipelined_mode_validation():
    """The pipelined schedule is a plan mode: it takes a slice-group count,
    refuses the per-slice F and early stop, and keeps a second set of F
    tables in the workspace."""
    L = _lib()
    good = W.small_problem(n=(16, 16, 16), P=4, K=2)

    def rc_for(q, mode):
        arr = (L.PrProblem * 1)(L.to_struct(q))
        h = ctypes.c_void_p()
        rc = L.lib().pr_plan_create(arr, 1, mode, ctypes.c_void_p(1 << 40), 1 << 50, ctypes.byref(h))
        return rc, L.last_error()

    pipe = L.PR_MODE_PIPELINED
    assert rc_for(good, pipe)[0] == L.PR_EDEVICE            # valid: fails only for want of a device
    assert rc_for(good, pipe | L.PR_MODE_PIPELINE_GROUPS(3) | L.PR_MODE_GRAPH)[0] == L.PR_EDEVICE
    rc, msg = rc_for(good, L.PR_MODE_PIPELINE_GROUPS(2))
    assert rc == L.PR_EINVAL and "PR_MODE_PIPELINED" in msg
    rc, msg = rc_for(good, pipe | L.PR_MODE_PER_SLICE)
    assert rc == L.PR_EINVAL and "PER_SLICE" in msg
    early = W.small_problem(n=(16, 16, 16), P=4, K=2)
    early.flags |= L.PR_EARLY_STOP
    rc, msg = rc_for(early, pipe)
    assert rc == L.PR_EINVAL and "EARLY_STOP" in msg
    arr = (L.PrProblem * 1)(L.to_struct(good))
    plain = L.lib().pr_plan_workspace_bytes(arr, 1, 0)
    piped = L.lib().pr_plan_workspace_bytes(arr, 1, pipe)
    assert piped > plain


def test_workspace_sizes():
    """The largest single-instance workload fits in 288 GB of HBM."""
    L = _lib()
    for name, mode in (("c2_128_fp64", 0), ("c3_256_mixed", 1), ("c5_512_mixed", 1)):
        p, _ = W.config(name)
        arr = (L.PrProblem * 1)(L.to_struct(p))
        nb = L.lib().pr_plan_workspace_bytes(arr, 1, mode)
        n = p.npts
        es = 4 if mode else 8
        assert nb >= (p.P + 1) * n * 8 + 4 * p.P * n * es
        assert nb < 288e9
    insts = [q for q, _ in W.batched_config(64)]
    arr = (L.PrProblem * len(insts))(*[L.to_struct(q) for q in insts])
    assert 0 < L.lib().pr_plan_workspace_bytes(arr, len(insts), 1) < 64e9


def test_defect_and_update_validation():
    L = _lib()
    assert L.lib().pr_parareal_update(10, 1, 3, 1, 1, 1, 1, None, None) == L.PR_EINVAL
    assert L.lib().pr_parareal_update(10, 1, 2, None, 1, 1, 1, None, None) == L.PR_EINVAL
    assert L.lib().pr_defect_norm(10, 1, 2, 1, 2, 1, 1, 1, 0, None) == L.PR_ENOMEM
    assert L.lib().pr_defect_norm(0, 1, 2, 1, 2, 1, 1, 1, 1 << 20, None) == L.PR_EINVAL
    assert L.lib().pr_defect_workspace_bytes(3) > 0


def test_variant_registry():
    import paper_1409_8563_amd as pr
    L = _lib()
    fine = pr.variants(0)
    coarse = pr.variants(1)
    assert len(fine) >= 4 and len(coarse) >= 4
    for v in fine:
        assert v["dtype"] in (1, 2) and v["order"] in (2, 4) and v["steps"] == 1
        assert v["tile"][0] > 0 and v["tile"][1] > 0
        if v["nx_exact"]:
            # whole-row kernels: a grid row spans a 64-lane wavefront or a
            # 16-lane DPP row, each lane holding nxp consecutive x
            assert v["nx_exact"] == v["tile"][0] and v["nx_exact"] in (16 * v["nxp"], 64 * v["nxp"])
    assert any(v["nx_exact"] for v in fine)
    for v in coarse:
        assert v["order"] == 0 and v["steps"] >= 1
    assert L.lib().pr_kernel_variant_name(0, 1) == b"rk4_unfused_reference"
    assert L.lib().pr_set_kernel_variant(10 ** 6, 0) == L.PR_EINVAL
    assert L.lib().pr_set_kernel_variant(0, 0) == 0


@pytest.mark.parametrize("n3,dtype,batch,name", [
    ((128, 128, 128), 2, 16, "rk4w_f64_x128_y8_p2x1_w16"),
    ((64, 64, 64), 2, 8, "rk4w_f64_x64_y16_p1x2_w12"),
    ((64, 64, 64), 2, 1, "rk4w_f64_x64_y8_p1x2_w8"),
    ((40, 36, 20), 2, 4, "rk4x_f64_t56x8_p1x2_w8"),
    ((160, 160, 160), 2, 8, "rk4x_f64_t56x16_p1x3_w8"),
    ((256, 256, 256), 1, 32, "rk4w_f32_x256_y8_p4x2_w8"),
    ((128, 128, 128), 1, 136, "rk4w_f32_x128_y16_p2x2_w12"),
    ((128, 128, 128), 1, 1, "rk4w_f32_x128_y8_p2x2_w8"),
    ((96, 96, 96), 1, 88, "rk4s_f32_x96_y24_p6x1_w8"),
    ((64, 64, 64), 1, 152, "rk4s_f32_x64_y24_p4x1_w8"),
    ((64, 64, 64), 1, 16, "rk4s_f32_x64_y40_p4x1_w12"),
    ((48, 48, 48), 1, 136, "rk4s_f32_x48_y24_p3x1_w8"),
    ((48, 48, 48), 2, 8, "rk4s_f64_x48_y24_p3x1_w8"),
    ((32, 32, 32), 2, 4, "rk4s_f64_x32_y32_p2x1_w10"),
    ((32, 32, 32), 1, 16, "rk4s_f32_x32_y32_p2x1_w10"),
    ((80, 60, 40), 1, 16, "rk4x_f32_t56x40_p1x3_w16"),
    ((192, 60, 40), 1, 16, "rk4b_f32_t64x32_p2x2_d2"),
    ((512, 512, 512), 1, 32, "rk4b_f32_t64x32_p2x2_d2"),
    ((37, 29, 23), 1, 2, "rk4x_f32_t56x40_p1x3_w16"),
])
def test_builtin_fine_kernel_choice(n3, dtype, batch, name):
    """Host logic, no device: the built-in F kernel for a grid (whole rows for
    n_x = 64/128/256, 16-lane rows for n_x = 32/48/96, as measured; other
    widths: x-tiled rows, except FP32 rows whose n_x is a multiple of 64,
    which take the 2-D tile that computes the fewest points per output
    point)."""
    import paper_1409_8563_amd as pr
    p = W.small_problem(n=n3, P=2, nf=4)
    p.flags |= W.ALLOW_UNSTABLE
    assert pr.sweep_kernel_variant(p, dtype, batch, 0) == name


@pytest.mark.parametrize("n3,dtype,name", [
    ((128, 128, 128), 2, "euler4w_f64_x128_y8_p2x1_w16"),
    ((64, 64, 64), 2, "euler4w_f64_x64_y8_p1x1_w16"),
    ((256, 256, 256), 2, "euler4x_f64_t56x24_p1x2_w16"),
    ((37, 29, 23), 2, "euler4x_f64_t56x24_p1x2_w16"),
    ((32, 32, 32), 2, "euler4b_f64_t32x32_p2x2_d2"),
    ((256, 256, 256), 1, "euler4w_f32_x256_y8_p4x1_w16"),
    ((128, 128, 128), 1, "euler4w_f32_x128_y8_p2x1_w16"),
    ((96, 96, 96), 1, "euler4b_f32_t32x32_p2x2_d2"),
    ((512, 512, 512), 1, "euler4x_f32_t56x40_p1x3_w16"),
    ((48, 48, 48), 1, "euler4x_f32_t56x24_p1x2_w16"),
])
def test_builtin_coarse_kernel_choice(n3, dtype, name):
    """Host logic, no device: the built-in G kernel for a grid (whole rows
    where a kernel exists; FP32 2-D tiles where 32-wide tiles cover the row
    up to 128; FP64 2-D tiles on rows too narrow for 64-column x tiles;
    x-tiled rows otherwise)."""
    import paper_1409_8563_amd as pr
    p = W.small_problem(n=n3, P=2, nf=4)
    p.flags |= W.ALLOW_UNSTABLE
    assert pr.sweep_kernel_variant(p, dtype, 1, 1) == name


def test_fp32_tile_choice_minimises_computed_points():
    """FP32 grids without a whole-row kernel: where n_x is a multiple of 64
    the chosen 2-D tile has the fewest computed points per output point (a
    4-point halo per side) among the four two-point tiles; every other width
    takes the x-tiled rows."""
    import paper_1409_8563_amd as pr
    cands = {v["name"]: v for v in pr.variants(0)
             if v["name"] in ("rk4b_f32_t64x32_p2x2_d2", "rk4b_f32_t64x24_p2x2_d2",
                              "rk4b_f32_t48x32_p2x2_d2", "rk4b_f32_t48x24_p2x2_d2")}
    assert len(cands) == 4

    def waste(v, nx, ny):
        tx, ty = v["tile"]
        return (-(-nx // tx) * (tx + 8) / nx) * (-(-ny // ty) * (ty + 8) / ny)

    for nx in (192, 320, 384, 448, 512, 576, 640):
        for ny in (10, 24, 48, 72, 100, 200):
            p = W.small_problem(n=(nx, ny, 12), P=2, nf=4)
            p.flags |= W.ALLOW_UNSTABLE
            got = pr.sweep_kernel_variant(p, 1, 4, 0)
            assert got in cands, (nx, ny, got)
            assert waste(cands[got], nx, ny) <= min(waste(v, nx, ny) for v in cands.values()) * (1 + 1e-12)
    for nx in range(8, 260, 6):
        if nx in (32, 48, 64, 96, 128, 256) or nx % 64 == 0:
            continue
        p = W.small_problem(n=(nx, 40, 12), P=2, nf=4)
        p.flags |= W.ALLOW_UNSTABLE
        assert pr.sweep_kernel_variant(p, 1, 4, 0) == "rk4x_f32_t56x40_p1x3_w16", nx


def test_whole_row_variant_rejects_other_nx():
    """A forced whole-row variant on a grid whose n_x it does not cover is
    refused before any launch."""
    import ctypes
    import paper_1409_8563_amd as pr
    import workloads as W
    L = _lib()
    row = [v for v in pr.variants(0) if v["nx_exact"] == 128 and v["dtype"] == 2][0]
    p = W.small_problem(n=(64, 40, 20), P=2, nf=4)
    p.flags |= W.ALLOW_UNSTABLE
    s = L.to_struct(p)
    steps = (ctypes.c_int64 * 1)(0)
    try:
        assert L.lib().pr_set_kernel_variant(row["index"], 0) == 0
        rc = L.lib().pr_fine_sweep(ctypes.byref(s), 2, 1, 16, 16 + (1 << 30), steps, 1, 16, 1 << 40, None)
    finally:
        L.lib().pr_set_kernel_variant(0, 0)
    assert rc == L.PR_EUNSUPPORTED


def test_coarsened_g_validation_and_margin():
    """PR_COARSEN_G needs even n >= 6 per direction and takes the coarse
    stability margin on the coarsened grid (h = 2/n): the 128^3 workload's G
    with 128 coarse steps is unstable on the fine grid and stable when
    coarsened.  PR_CUBIC_INTERP alone is rejected."""
    import paper_1409_8563_amd as pr
    L = _lib()
    p, _ = W.config("c2_128_fp64")
    p.nt_coarse = 128
    rc, fm, cm_fine = pr.check_stability(p)
    assert rc == L.PR_EUNSTABLE and cm_fine > 1.0
    p.flags = W.COARSEN_G
    rc, fm, cm = pr.check_stability(p)
    assert rc == 0 and cm < 1.0
    # the coarsened margin is the same bound evaluated with n/2
    nm = p.nu0 * (1 + abs(p.nu_amp))
    ref = (p.T / p.nt_coarse) * sum(abs(p.a[d]) * 64 + 2 * nm * 64 * 64 for d in range(3))
    assert abs(cm - ref) <= 1e-12 * ref
    arr = (L.PrProblem * 1)(L.to_struct(p))
    assert L.lib().pr_plan_workspace_bytes(arr, 1, 0) > 0
    q = W.small_problem(n=(10, 7, 8), P=2, nf=8, nc=8, flags=W.COARSEN_G)
    arr = (L.PrProblem * 1)(L.to_struct(q))
    assert L.lib().pr_plan_workspace_bytes(arr, 1, 0) == 0 and "even" in L.last_error()
    q = W.small_problem(n=(10, 8, 8), P=2, nf=8, nc=8, flags=W.CUBIC_INTERP)
    arr = (L.PrProblem * 1)(L.to_struct(q))
    assert L.lib().pr_plan_workspace_bytes(arr, 1, 0) == 0 and "PR_COARSEN_G" in L.last_error()


def test_grid_transfer_validation_without_device():
    L = _lib()
    p = W.small_problem(n=(12, 10, 8), P=2)
    s = L.to_struct(p)
    big = 1 << 30
    assert L.lib().pr_transfer_workspace_bytes(3) >= 3 * 8
    assert L.lib().pr_prolong(ctypes.byref(s), 2, 2, 1, 16, 16 + big, 16, 1 << 20, None) == L.PR_EINVAL
    assert L.lib().pr_restrict(ctypes.byref(s), 2, 1, 16, 16 + big, 16, 0, None) == L.PR_ENOMEM
    assert L.lib().pr_restrict(ctypes.byref(s), 2, 1, 16, 16 + 8, 16, 1 << 20, None) == L.PR_EINVAL  # overlap
    q = W.small_problem(n=(12, 9, 8), P=2)
    s = L.to_struct(q)
    assert L.lib().pr_restrict(ctypes.byref(s), 2, 1, 16, 16 + big, 16, 1 << 20, None) == L.PR_EINVAL


def test_plan_autotune_validation():
    L = _lib()
    cnt = ctypes.c_int32()
    assert L.lib().pr_plan_fine_groups(None, 0, ctypes.byref(cnt), None, None, None) == L.PR_EINVAL
    v = (ctypes.c_int32 * 4)()
    assert L.lib().pr_plan_autotune(None, None, None, None, None, None) == L.PR_EINVAL


def test_binding_rejects_mismatched_buffers_before_any_device_work():
    """The C ABI receives bare device pointers and cannot see buffer sizes,
    so the binding checks dtype, element count and contiguity of every
    tensor (before the device check, so this runs on the CPU)."""
    import torch

    import paper_1409_8563_amd as pr
    p = W.small_problem(n=(8, 6, 5))
    npts = 8 * 6 * 5
    f64 = lambda k: torch.zeros(k, dtype=torch.float64)   # noqa: E731
    f32 = lambda k: torch.zeros(k, dtype=torch.float32)   # noqa: E731
    # sweeps: u_out of the wrong size or dtype, step0 of the wrong length
    with pytest.raises(ValueError, match="u_out"):
        pr.fine_sweep(p, f64(2 * npts), 0, 1, u_out=f64(npts))
    with pytest.raises(TypeError, match="u_out"):
        pr.coarse_sweep(p, f64(npts), 0, 1, u_out=f32(npts))
    with pytest.raises(ValueError, match="step0"):
        pr.fine_sweep(p, f64(2 * npts), [0, 1, 2], 1)
    with pytest.raises(ValueError, match="multiple"):
        pr.fine_sweep(p, f64(npts + 1), 0, 1)
    with pytest.raises(ValueError, match="contiguous"):
        pr.fine_sweep(p, f64(2 * npts).view(2, npts).t(), 0, 1)
    # correction: operands and outputs must match f_new
    with pytest.raises(ValueError, match="g_new"):
        pr.parareal_update(f32(10), f32(9), f32(10))
    with pytest.raises(TypeError, match="g_old"):
        pr.parareal_update(f32(10), f32(10), f64(10))
    with pytest.raises(TypeError, match="u_out"):
        pr.parareal_update(f32(10), f32(10), f32(10), u_out=f32(10))
    with pytest.raises(ValueError, match="u_out_lo"):
        pr.parareal_update(f32(10), f32(10), f32(10), u_out=f64(10), u_out_lo=f32(5))
    # norms: ref must match x; batch must divide x
    with pytest.raises(ValueError, match="ref"):
        pr.defect_norm(f64(12), f64(11))
    with pytest.raises(ValueError, match="batch"):
        pr.defect_norm(f64(12), f64(12), batch=5)
    # every check passed: only then the device check
    with pytest.raises(ValueError, match="GPU"):
        pr.parareal_update(f32(10), f32(10), f32(10))




def test_copy_probe_validation_without_device():
    L = _lib()
    lib = L.lib()
    assert lib.pr_copy_probe(None, 16, 16, 0, 0, None) == L.PR_EINVAL
    assert lib.pr_copy_probe(16, 4096, 24, 0, 0, None) == L.PR_EINVAL      # not a multiple of 16
    assert lib.pr_copy_probe(16, 32, 64, 0, 0, None) == L.PR_EINVAL        # overlap
    assert lib.pr_copy_probe(8, 4096, 16, 0, 0, None) == L.PR_EINVAL       # misaligned
    assert lib.pr_copy_probe(16, 4096, 16, 4, 0, None) == L.PR_EINVAL      # unknown variant
    assert lib.pr_copy_probe(16, 4096, 16, 0, 65, None) == L.PR_EINVAL     # grid size

def test_static_defect_norm_validation_without_device():
    """The allocation-free norm entry point rejects a batch beyond its static
    scratch (and bad arguments) before any device work."""
    L = _lib()
    lib = L.lib()
    assert lib.pr_defect_static_scratch_bytes() >= L.PR_DEFECT_STATIC_MAX_BATCH * 512 * 4 * 8
    assert lib.pr_defect_norm_static(10, L.PR_DEFECT_STATIC_MAX_BATCH + 1, 2, 1, 2, 1, 1, None) == L.PR_EINVAL
    assert "exceeds" in L.last_error()
    assert lib.pr_defect_norm_static(0, 1, 2, 1, 2, 1, 1, None) == L.PR_EINVAL
    assert lib.pr_defect_norm_static(10, 1, 3, 1, 2, 1, 1, None) == L.PR_EINVAL
    assert lib.pr_defect_norm_static(10, 1, 2, None, 2, 1, 1, None) == L.PR_EINVAL


def test_autotune_cache_round_trip(tmp_path):
    """The tuned-kernel table is saved as JSON and loaded back; lookups use
    entries of the current architecture ("none" without a device); entries
    naming an unknown variant are skipped; PR_AUTOTUNE_CACHE loads a file
    before the first lookup in a fresh process.  Host logic only."""
    import json
    import subprocess
    import sys
    import paper_1409_8563_amd as pr
    p = W.small_problem(n=(40, 36, 20), P=2, nf=4)
    p.flags |= W.ALLOW_UNSTABLE
    default = pr.sweep_kernel_variant(p, 1, 4, 0)
    tuned = "rk4b_f32_t48x24_p2x2_d2"
    assert default != tuned
    src = tmp_path / "tune.json"
    src.write_text(json.dumps({"format": "pr-autotune-1", "entries": [
        {"arch": "none", "which": 0, "n": [40, 36, 20], "dtype": 1, "order": 2, "batch": 4,
         "variant": tuned, "blocks_per_cu": 2},
        {"arch": "gfx942", "which": 0, "n": [40, 36, 20], "dtype": 1, "order": 2, "batch": 4,
         "variant": "rk4b_f32_t64x32_p2x2_d2", "blocks_per_cu": 0},
        {"arch": "none", "which": 0, "n": [64, 64, 64], "dtype": 1, "order": 2, "batch": 4,
         "variant": "no_such_kernel", "blocks_per_cu": 0}]}))
    try:
        pr.autotune_clear()
        assert pr.autotune_load(str(src)) == 2
        assert pr.sweep_kernel_variant(p, 1, 4, 0) == tuned
        assert pr.sweep_kernel_variant(p, 1, 7, 0) == tuned        # any tuned batch of the shape
        out = tmp_path / "saved.json"
        pr.autotune_save(str(out))
        saved = json.loads(out.read_text())
        key = lambda e: json.dumps(e, sort_keys=True)
        assert sorted(map(key, saved["entries"])) == sorted(map(key, json.loads(src.read_text())["entries"][:2]))
        pr.autotune_clear()
        assert pr.sweep_kernel_variant(p, 1, 4, 0) == default
        assert pr.autotune_load(str(out)) == 2
        assert pr.sweep_kernel_variant(p, 1, 4, 0) == tuned
    finally:
        pr.autotune_clear()
    with pytest.raises(Exception):
        pr.autotune_load(str(tmp_path / "missing.json"))
    code = ("import sys; sys.path.insert(0, %r); import workloads as W, paper_1409_8563_amd as pr\n"
            "p = W.small_problem(n=(40, 36, 20), P=2, nf=4); p.flags |= W.ALLOW_UNSTABLE\n"
            "print(pr.sweep_kernel_variant(p, 1, 4, 0))" % ROOT)
    env = dict(os.environ, PR_AUTOTUNE_CACHE=str(out))
    got = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert got.stdout.strip().splitlines()[-1] == tuned, got.stderr
