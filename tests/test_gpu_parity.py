"""GPU parity of the HIP path (through the C ABI) against the FP64 CPU oracle
and the per-mode reference.  Bars: FP64 relative L2 <= 1e-12, FP32 relative
L2 <= 1e-5 (against FP64), bitwise equality where the arithmetic is the same
(kernel variants, tile shapes, batching, graph replay, slice skipping)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


@pytest.fixture(scope="module")
def pr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1409_8563_amd as prm
    prm.lib()
    prm.set_kernel_variant(0, 0)
    yield prm
    prm.set_kernel_variant(0, 0)


def cuda(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().double().numpy()


def rel_l2(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def say(*a):
    print(*a, flush=True)


# ---------------------------------------------------------------------------
# sweeps
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n3", [(40, 36, 20), (37, 29, 23), (64, 33, 70)])
@pytest.mark.parametrize("order", [2, 4])
def test_fine_step_fp64(pr, orc, n3, order):
    import torch
    say("fine step fp64", n3, order)
    p = W.small_problem(n=n3, a=(0.9, -0.6, 0.35), nu0=0.003, order=order, nf=8, P=4)
    u = W.random_field(n3, 101)
    ref = orc.rk4_step(p, 5, u)
    got = host(pr.fine_sweep(p, cuda(u), 5, 1))
    assert rel_l2(got, ref) <= FP64_TOL
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_fine_sweep_batch_of_slices_fp64(pr, orc):
    say("fine sweep batch fp64")
    p = W.small_problem(n=(34, 30, 26), P=3, nf=5, nc=2)
    u = np.stack([W.random_field(p.n, 110 + s) for s in range(p.P)])
    got = host(pr.fine_sweep(p, cuda(u), [s * p.nf for s in range(p.P)], p.nf))
    for s in range(p.P):
        ref = orc.fine_steps(p, s * p.nf, p.nf, u[s])
        assert rel_l2(got[s], ref) <= FP64_TOL, s


@pytest.mark.parametrize("nsteps", [0, 1, 3, 7, 8])
@pytest.mark.parametrize("a", [(0.9, -0.6, 0.0), (-0.3, 0.7, 1.1)])
def test_coarse_sweep_fp64(pr, orc, nsteps, a):
    say("coarse sweep fp64", nsteps, a)
    p = W.small_problem(n=(36, 34, 22), a=a, nu0=0.004, P=2, nc=8)
    u = W.random_field(p.n, 120)
    got = host(pr.coarse_sweep(p, cuda(u), 3, nsteps))
    ref = orc.coarse_steps(p, 3, nsteps, u)
    if nsteps == 0:
        assert np.array_equal(got, u)
    else:
        assert rel_l2(got, ref) <= FP64_TOL


@pytest.mark.parametrize("order", [2, 4])
def test_fp32_sweeps_against_fp64_oracle(pr, orc, order):
    import torch
    say("fp32 sweeps", order)
    p = W.small_problem(n=(48, 40, 36), a=(1.0, 0.5, 0.25), nu0=0.004, P=2, nf=16, nc=16, order=order)
    modes = W.draw_modes(np.random.default_rng(130), 6, 4)
    u = W.synth_u0(p.n, modes)
    gf = host(pr.fine_sweep(p, cuda(u, torch.float32), 0, 16))
    gc = host(pr.coarse_sweep(p, cuda(u, torch.float32), 0, 4))
    assert rel_l2(gf, orc.fine_steps(p, 0, 16, u)) <= FP32_TOL
    assert rel_l2(gc, orc.coarse_steps(p, 0, 4, u)) <= FP32_TOL


def _applicable(pr, which, dtype, order, nx):
    out = [1]
    for v in pr.variants(which):
        if v["dtype"] == dtype and (which == 1 or v["order"] == order) and nx % v["nxp"] == 0 \
                and v.get("nx_exact", 0) in (0, nx):
            out.append(v["index"])
    return out


@pytest.mark.parametrize("dtype", [1, 2])
@pytest.mark.parametrize("order", [2, 4])
def test_fine_variants_bitwise_identical(pr, dtype, order):
    """Every tile configuration and the unfused reference give the same bits:
    the per-point arithmetic does not depend on tiling or schedule."""
    import torch
    tdt = torch.float64 if dtype == 2 else torch.float32
    p = W.small_problem(n=(72, 52, 41), a=(0.7, -0.45, 0.3), nu0=0.002, order=order, P=2, nf=4)
    u = cuda(W.random_field(p.n, 140), tdt)
    outs = {}
    try:
        for v in _applicable(pr, 0, dtype, order, p.n[0]):
            say("fine variant", v, dtype, order)
            pr.set_kernel_variant(v, 0)
            outs[v] = pr.fine_sweep(p, u, 3, 3)
    finally:
        pr.set_kernel_variant(0, 0)
    base = outs[1]
    assert len(outs) >= 2
    for v, o in outs.items():
        assert torch.equal(o, base), v


@pytest.mark.parametrize("dtype", [2])
@pytest.mark.parametrize("n3", [(131, 45, 17), (7, 9, 11), (200, 20, 9), (57, 100, 6)])
def test_fine_x_tiled_fourth_order_bitwise_and_oracle(pr, orc, dtype, n3):
    """The FP64 fourth-order F over x tiles (two launches of two fused
    radius-2 stages, 4-column x halo, rows of any length) gives the bits of
    the unfused reference and follows the oracle."""
    import torch
    tdt = torch.float64 if dtype == 2 else torch.float32
    p = W.small_problem(n=n3, a=(0.7, -0.45, 0.3), nu0=0.0005, P=2, nf=64, order=4)
    u = cuda(W.random_field(p.n, 152), tdt)
    xt = [v["index"] for v in pr.variants(0) if v["name"].startswith("rk4hx_") and v["dtype"] == dtype]
    assert xt
    outs = {}
    try:
        for v in [1] + xt:
            say("x-tiled order-4 variant", v, dtype, n3)
            pr.set_kernel_variant(v, 0)
            outs[v] = pr.fine_sweep(p, u, 3, 3)
    finally:
        pr.set_kernel_variant(0, 0)
    for v, o in outs.items():
        assert torch.equal(o, outs[1]), v
    ref = orc.fine_steps(p, 3, 3, host(u).reshape(p.n[2], p.n[1], p.n[0]))
    got = host(outs[xt[0]]).reshape(ref.shape)
    assert rel_l2(got, ref) <= (FP64_TOL if dtype == 2 else FP32_TOL)


@pytest.mark.parametrize("dtype", [1, 2])
@pytest.mark.parametrize("n3", [(131, 45, 17), (7, 9, 11), (200, 8, 5), (57, 100, 6)])
def test_coarse_x_tiled_rows_bitwise_and_oracle(pr, orc, dtype, n3):
    """The x-tiled Euler kernels (4 steps per launch, x tiles with a
    4-column halo wrapped onto rows of any length) give the bits of the
    unfused reference, including a partial last chunk, and follow the
    oracle."""
    import torch
    tdt = torch.float64 if dtype == 2 else torch.float32
    p = W.small_problem(n=n3, a=(0.3, -0.2, 0.0), nu0=0.0005, P=1, nc=64)
    u0 = W.random_field(p.n, 151)
    u = cuda(u0, tdt)
    xt = [v["index"] for v in pr.variants(1) if v["name"].startswith("euler4x_") and v["dtype"] == dtype]
    assert xt
    outs = {}
    try:
        for v in [1] + xt:
            say("x-tiled coarse variant", v, dtype, n3)
            pr.set_kernel_variant(0, v)
            outs[v] = pr.coarse_sweep(p, u, 2, 11)
    finally:
        pr.set_kernel_variant(0, 0)
    for v, o in outs.items():
        assert torch.equal(o, outs[1]), v
    ref = orc.coarse_steps(p, 2, 11, host(u).reshape(p.n[2], p.n[1], p.n[0]))
    got = host(outs[xt[0]]).reshape(ref.shape)
    assert rel_l2(got, ref) <= (FP64_TOL if dtype == 2 else FP32_TOL)


@pytest.mark.parametrize("dtype", [1, 2])
@pytest.mark.parametrize("n3", [(131, 45, 17), (7, 9, 11), (200, 8, 5), (57, 100, 6), (112, 41, 3)])
def test_fine_x_tiled_rows_bitwise_and_oracle(pr, orc, dtype, n3):
    """The x-tiled row kernels (x tiles of 64 columns with a 4-column halo,
    wrapped onto rows of any length) give the bits of the unfused reference
    on ragged widths, on rows shorter than one tile (columns held twice),
    on fewer rows than a tile and on z shorter than the pipeline; and they
    follow the oracle."""
    import torch
    tdt = torch.float64 if dtype == 2 else torch.float32
    p = W.small_problem(n=n3, a=(0.7, -0.45, 0.3), nu0=0.002, P=2, nf=64)
    u0 = W.random_field(p.n, 150)
    u = cuda(u0, tdt)
    xt = [v["index"] for v in pr.variants(0) if v["name"].startswith("rk4x_") and v["dtype"] == dtype]
    assert xt
    outs = {}
    try:
        for v in [1] + xt:
            say("x-tiled variant", v, dtype, n3)
            pr.set_kernel_variant(v, 0)
            outs[v] = pr.fine_sweep(p, u, 3, 3)
    finally:
        pr.set_kernel_variant(0, 0)
    for v, o in outs.items():
        assert torch.equal(o, outs[1]), v
    ref = orc.fine_steps(p, 3, 3, host(u).reshape(p.n[2], p.n[1], p.n[0]))
    got = host(outs[xt[0]]).reshape(ref.shape)
    assert rel_l2(got, ref) <= (FP64_TOL if dtype == 2 else FP32_TOL)


@pytest.mark.parametrize("dtype", [1, 2])
@pytest.mark.parametrize("n3,order", [((128, 52, 21), 2), ((64, 37, 19), 2), ((256, 20, 9), 2), ((128, 8, 5), 2),
                                      ((96, 52, 21), 2), ((48, 37, 19), 2), ((48, 8, 5), 2), ((96, 100, 6), 2),
                                      ((32, 29, 13), 2), ((32, 8, 5), 2), ((64, 70, 9), 2),
                                      ((128, 52, 21), 4), ((128, 8, 5), 4), ((128, 19, 40), 4)])
def test_fine_whole_row_variants_bitwise_identical(pr, dtype, n3, order):
    """The whole-row kernels (x neighbours across the wavefront; for order 4
    two launches of two stages each) agree bit for bit with the unfused
    reference and the tiled kernels, on grids with a ragged last y tile,
    fewer rows than one tile and z shorter than the pipeline."""
    import torch
    tdt = torch.float64 if dtype == 2 else torch.float32
    p = W.small_problem(n=n3, a=(0.7, -0.45, 0.3), nu0=0.002, P=2, nf=64, order=order)
    u = cuda(W.random_field(p.n, 141), tdt)
    vs = _applicable(pr, 0, dtype, order, p.n[0])
    rows = [v["index"] for v in pr.variants(0)
            if v["nx_exact"] == p.n[0] and v["dtype"] == dtype and v["order"] == order]
    if not rows:
        pytest.skip("no whole-row variant for n_x=%d" % p.n[0])
    outs = {}
    try:
        for v in vs:
            say("fine variant", v, dtype, n3)
            pr.set_kernel_variant(v, 0)
            outs[v] = pr.fine_sweep(p, u, 3, 3)
    finally:
        pr.set_kernel_variant(0, 0)
    assert set(rows) <= set(outs)
    for v, o in outs.items():
        assert torch.equal(o, outs[1]), v


@pytest.mark.parametrize("dtype", [1, 2])
def test_coarse_variants_bitwise_identical(pr, dtype):
    import torch
    tdt = torch.float64 if dtype == 2 else torch.float32
    p = W.small_problem(n=(66, 40, 37), a=(0.7, -0.45, 0.0), nu0=0.002, P=1, nc=13)
    u = cuda(W.random_field(p.n, 150), tdt)
    outs = {}
    try:
        for v in _applicable(pr, 1, dtype, 0, p.n[0]):
            say("coarse variant", v, dtype)
            pr.set_kernel_variant(0, v)
            outs[v] = pr.coarse_sweep(p, u, 2, 13)
    finally:
        pr.set_kernel_variant(0, 0)
    assert len(outs) >= 3
    for v, o in outs.items():
        assert torch.equal(o, outs[1]), v


@pytest.mark.parametrize("dtype", [1, 2])
@pytest.mark.parametrize("n3", [(128, 44, 19), (64, 21, 11), (256, 12, 7)])
def test_coarse_whole_row_variants_bitwise_identical(pr, dtype, n3):
    """Whole-row Euler chunks agree bit for bit with the reference and the
    tiled chunks, including a step count that leaves a partial chunk."""
    import torch
    tdt = torch.float64 if dtype == 2 else torch.float32
    p = W.small_problem(n=n3, a=(0.7, -0.45, 0.0), nu0=0.002, P=1, nc=13)
    p.flags |= W.ALLOW_UNSTABLE    # 13 steps of a random field: only the bits are compared
    u = cuda(W.random_field(p.n, 151), tdt)
    rows = [v["index"] for v in pr.variants(1) if v["nx_exact"] == p.n[0] and v["dtype"] == dtype]
    if not rows:
        pytest.skip("no whole-row variant for n_x=%d" % p.n[0])
    outs = {}
    try:
        for v in _applicable(pr, 1, dtype, 0, p.n[0]):
            say("coarse variant", v, dtype, n3)
            pr.set_kernel_variant(0, v)
            outs[v] = pr.coarse_sweep(p, u, 2, 13)
    finally:
        pr.set_kernel_variant(0, 0)
    assert set(rows) <= set(outs)
    for v, o in outs.items():
        assert torch.equal(o, outs[1]), v


@pytest.mark.parametrize("dtype", [1, 2])
def test_translation_equivariance_bitwise(pr, dtype):
    import torch
    say("translation", dtype)
    tdt = torch.float64 if dtype == 2 else torch.float32
    p = W.small_problem(n=(64, 48, 40), a=(0.8, -0.3, 0.5), nu0=0.002, P=2, nf=8, nc=8)
    u = cuda(W.random_field(p.n, 160), tdt)
    sh = (7, -5, 11)
    a1 = pr.fine_sweep(p, torch.roll(u, sh, (0, 1, 2)).contiguous(), 1, 3)
    a2 = torch.roll(pr.fine_sweep(p, u, 1, 3), sh, (0, 1, 2))
    assert torch.equal(a1, a2)
    b1 = pr.coarse_sweep(p, torch.roll(u, sh, (0, 1, 2)).contiguous(), 1, 5)
    b2 = torch.roll(pr.coarse_sweep(p, u, 1, 5), sh, (0, 1, 2))
    assert torch.equal(b1, b2)


def test_update_and_defect_norm(pr, orc):
    import torch
    say("update/defect")
    n3 = (30, 20, 17)
    f, g, h = (W.random_field(n3, s) for s in (170, 171, 172))
    for tdt in (torch.float64, torch.float32):
        F, G, H = cuda(f, tdt), cuda(g, tdt), cuda(h, tdt)
        lo = torch.empty_like(F)
        u = host(pr.parareal_update(F, G, G, u_out_lo=lo))
        assert np.array_equal(u, host(F))                    # G_new == G_old gives F exactly
        assert torch.equal(lo, F)
        u = host(pr.parareal_update(F, G, H))
        Fd, Gd, Hd = host(F), host(G), host(H)
        assert np.array_equal(u, Fd + (Gd - Hd))
    x, r = W.random_field(n3, 173), W.random_field(n3, 174)
    got = host(pr.defect_norm(cuda(np.stack([x, r])), cuda(np.stack([r, x])), batch=2))
    for b, (xx, rr) in enumerate(((x, r), (r, x))):
        ref = orc.norms(xx, rr)
        assert got[b, 0] == ref[0] and got[b, 1] == ref[1]
        assert abs(got[b, 2] - ref[2]) <= 1e-13 * ref[2] and abs(got[b, 3] - ref[3]) <= 1e-13 * ref[3]


# ---------------------------------------------------------------------------
# Parareal solves
# ---------------------------------------------------------------------------

def _solve(pr, probs, u0s, mode, ref=None):
    plan = pr.Plan(probs, mode)
    uT, log = plan.solve([cuda(u) for u in u0s], ref=ref)
    states = [[host(plan.slice_state(i, n)) for n in range(probs[i].P + 1)] for i in range(len(probs))]
    out = [host(x) for x in uT], log, states, plan
    return out


def test_parareal_c1_fp64_against_oracle(pr, orc):
    say("parareal c1 fp64")
    p, modes = W.config("c1_32_fp64")
    u0 = W.synth_u0(p.n, modes)
    _, olog, hist = orc.parareal(p, u0, K=p.K, history=True)
    uT, log, states, plan = _solve(pr, [p], [u0], pr.PR_MODE_FP64)
    for n in range(p.P + 1):
        assert rel_l2(states[0][n], hist[p.K, n]) <= FP64_TOL, n
    assert rel_l2(uT[0], hist[p.K, p.P]) <= FP64_TOL
    # inter-iterate monitors agree with the oracle's
    assert np.allclose(log[0][:, :8], olog, rtol=1e-9, atol=1e-14)
    # K = P: the result is the GPU serial fine solution, bitwise
    ser = host(pr.fine_sweep(p, cuda(u0), 0, p.nt_fine))
    assert np.array_equal(uT[0], ser)


def test_parareal_every_iterate_against_oracle(pr, orc):
    """K = 0..P on a problem with odd n_x (one-point-per-thread kernels)."""
    p = W.small_problem(n=(21, 18, 15), a=(0.6, 0.9, -0.4), nu0=0.01, P=3, nf=6, nc=3)
    u0 = W.random_field(p.n, 180)
    _, _, hist = orc.parareal(p, u0, K=p.P, history=True)
    for K in range(p.P + 1):
        say("parareal K", K)
        p.K = K
        uT, _, states, _ = _solve(pr, [p], [u0], pr.PR_MODE_FP64)
        for n in range(p.P + 1):
            assert rel_l2(states[0][n], hist[K, n]) <= FP64_TOL, (K, n)


@pytest.mark.parametrize("n3", [(128, 12, 10), (26, 18, 15)])
def test_parareal_fourth_order_every_iterate_against_oracle(pr, orc, n3):
    """The paper's fourth-order F inside Parareal, K = 0..P, every slice state
    element by element against the oracle: on a 128-wide grid (whole-row
    kernels, two launches per RK4 step) and on an odd grid (the same pair
    over x tiles)."""
    p = W.small_problem(n=n3, a=(0.6, 0.9, -0.4), nu0=0.0005, P=3, nf=12, nc=6, order=4)
    u0 = W.random_field(p.n, 181)
    _, _, hist = orc.parareal(p, u0, K=p.P, history=True)
    for K in range(p.P + 1):
        say("parareal order 4", n3, "K", K)
        p.K = K
        uT, _, states, _ = _solve(pr, [p], [u0], pr.PR_MODE_FP64)
        for n in range(p.P + 1):
            assert rel_l2(states[0][n], hist[K, n]) <= FP64_TOL, (K, n)
    plan = pr.Plan([p], pr.PR_MODE_FP64)
    fv = plan.kernel_variants()[0]
    assert fv.startswith("rk4h_f64_o4") if n3[0] == 128 else fv.startswith("rk4hx_f64_o4"), fv


def test_parareal_modes_bitwise_identical(pr):
    """Batched vs per-slice F, skipping converged slices, and HIP-graph replay
    (several replays, with eager work in between) give identical bits."""
    import torch
    p = W.small_problem(n=(40, 24, 28), P=5, nf=4, nc=6, K=3)
    u0 = W.random_field(p.n, 190)
    say("modes: eager")
    base, blog, bstates, _ = _solve(pr, [p], [u0], pr.PR_MODE_FP64)
    say("modes: per-slice")
    ps, plog, _, _ = _solve(pr, [p], [u0], pr.PR_MODE_FP64 | pr.PR_MODE_PER_SLICE)
    assert np.array_equal(ps[0], base[0]) and np.array_equal(plog, blog)
    q = W.small_problem(n=(40, 24, 28), P=5, nf=4, nc=6, K=3, flags=W.SKIP_CONVERGED)
    say("modes: skip")
    sk, slog, sstates, _ = _solve(pr, [q], [u0], pr.PR_MODE_FP64)
    assert np.array_equal(sk[0], base[0])
    for n in range(p.P + 1):
        assert np.array_equal(sstates[0][n], bstates[0][n]), n
    assert np.allclose(slog, blog, rtol=0, atol=0)
    say("modes: graph")
    plan = pr.Plan([p], pr.PR_MODE_FP64 | pr.PR_MODE_GRAPH)
    x = cuda(u0)
    for rep in range(3):
        uT, glog = plan.solve([x])
        scratch = torch.randn(1000, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(host(uT[0]), base[0]), rep
        assert np.array_equal(glog, blog), rep
        del scratch


@pytest.mark.parametrize("groups", [1, 2, 3, 7])
def test_pipelined_schedule_bitwise_identical(pr, groups):
    """The pipelined schedule (F of a slice group starts as soon as the
    previous iteration's chain has corrected it, while the chain goes on)
    reads and writes every buffer in the phase-by-phase order: every slice
    state, the result and the logs are the same bits, in FP64 and mixed
    precision, with and without skipping converged slices, with the
    reference defect, timed, and replayed from a recorded graph."""
    import torch
    ref_u = None
    for mode in (pr.PR_MODE_FP64, pr.PR_MODE_MIXED):
        for flags in (0, W.SKIP_CONVERGED):
            p = W.small_problem(n=(40, 24, 28), P=7, nf=4, nc=6, K=4, flags=flags)
            u0 = W.random_field(p.n, 195)
            if ref_u is None:
                ref_u = cuda(W.random_field(p.n, 196))
            say("pipelined: groups", groups, "mode", mode, "flags", flags)
            base, blog, bstates, _ = _solve(pr, [p], [u0], mode, ref=[ref_u])
            pm = mode | pr.PR_MODE_PIPELINED | pr.PR_MODE_PIPELINE_GROUPS(groups)
            for extra in (0, pr.PR_MODE_TIMED):
                uT, log, states, plan = _solve(pr, [p], [u0], pm | extra, ref=[ref_u])
                assert np.array_equal(uT[0], base[0]), extra
                assert np.array_equal(log, blog), extra
                for n in range(p.P + 1):
                    assert np.array_equal(states[0][n], bstates[0][n]), (extra, n)
                if extra:
                    tm = plan.timings()
                    assert tm["fine_ms"] > 0 and tm["coarse_chain_ms"] > 0 and tm["total_ms"] > 0, tm
                    assert tm["fine_launches"] >= p.K * (p.nt_fine // p.P), tm
            plan = pr.Plan([p], pm | pr.PR_MODE_GRAPH)
            x = cuda(u0)
            for rep in range(3):
                uT, glog = plan.solve([x], ref=[ref_u])
                scratch = torch.randn(1000, device="cuda").sum()   # eager work between replays
                torch.cuda.synchronize()
                assert np.array_equal(host(uT[0]), base[0]), rep
                assert np.array_equal(glog, blog), rep
                del scratch


def test_pipelined_schedule_other_paths_bitwise(pr):
    """Pipelined solves of the fourth-order F (two launches per step through
    scratch fields) and of the coarsened G match their phase-by-phase solves."""
    cases = [("order 4", W.small_problem(n=(128, 20, 18), P=5, nf=6, nc=4, K=3, order=4, nu0=0.0005)),
             ("coarsened G", W.small_problem(n=(32, 24, 20), P=6, nf=8, nc=4, K=3, flags=W.COARSEN_G))]
    for name, p in cases:
        u0 = W.random_field(p.n, 197)
        say("pipelined:", name)
        base, blog, bstates, _ = _solve(pr, [p], [u0], pr.PR_MODE_FP64)
        uT, log, states, _ = _solve(pr, [p], [u0], pr.PR_MODE_FP64 | pr.PR_MODE_PIPELINED)
        assert np.array_equal(uT[0], base[0]) and np.array_equal(log, blog), name
        for n in range(p.P + 1):
            assert np.array_equal(states[0][n], bstates[0][n]), (name, n)


def test_parareal_mixed_against_oracle(pr, orc):
    say("parareal mixed")
    modes = W.draw_modes(np.random.default_rng(200), 8, 4)
    p = W.small_problem(n=(48, 40, 32), a=(1.0, 0.5, 0.25), nu0=0.005, P=4, nf=16, nc=4, K=2)
    u0 = W.synth_u0(p.n, modes)
    U, olog = orc.parareal(p, u0, K=p.K)
    uT, log, states, _ = _solve(pr, [p], [u0], pr.PR_MODE_MIXED)
    assert rel_l2(uT[0], U[-1]) <= FP32_TOL
    for n in range(p.P + 1):
        assert rel_l2(states[0][n], U[n]) <= FP32_TOL, n


@pytest.mark.parametrize("dtype", [1, 2])
@pytest.mark.parametrize("order", [1, 3])
def test_grid_transfers_against_oracle(pr, orc, dtype, order):
    """Restriction (injection) and interpolation of the coarsened G, batch of
    two fields, against the oracle: bitwise in FP64 (same terms in the same
    order), within FP32 rounding otherwise."""
    import torch
    tdt = torch.float64 if dtype == 2 else torch.float32
    p = W.small_problem(n=(36, 20, 14))
    u = np.stack([W.random_field(p.n, 230 + b) for b in range(2)])
    say("grid transfers", dtype, order)
    uc = np.stack([orc.restrict(p, u[b]) for b in range(2)])
    f = np.stack([orc.prolong(p, uc[b], order) for b in range(2)])
    gr = host(pr.restrict(p, cuda(u, tdt)))
    gf = host(pr.prolong(p, cuda(uc, tdt), order))
    if dtype == 2:
        assert np.array_equal(gr, uc) and np.array_equal(gf, f)
    else:
        assert np.array_equal(gr, uc.astype(np.float32).astype(np.float64))
        assert rel_l2(gf, f) <= 1e-6


@pytest.mark.parametrize("flags", [W.COARSEN_G, W.COARSEN_G | W.CUBIC_INTERP])
def test_parareal_coarsened_g_against_oracle(pr, orc, flags):
    """Parareal with G on the grid coarsened by 2 (linear or cubic transfer):
    every slice state for K = 0, 2, P against the oracle, mixed precision
    within the FP32 bar, and eager / per-slice / skip / graph replay bitwise
    identical."""
    import torch
    p = W.small_problem(n=(32, 24, 20), a=(0.8, -0.5, 0.3), nu0=0.004, P=4, nf=8, nc=4, K=4, flags=flags)
    modes = W.draw_modes(np.random.default_rng(240), 6, 3)
    u0 = W.synth_u0(p.n, modes)
    _, _, hist = orc.parareal(p, u0, K=p.P, history=True)
    for K in (0, 2, p.P):
        say("coarsened G", flags, "K", K)
        p.K = K
        _, _, states, _ = _solve(pr, [p], [u0], pr.PR_MODE_FP64)
        for n in range(p.P + 1):
            assert rel_l2(states[0][n], hist[K, n]) <= FP64_TOL, (K, n)
    p.K = 2
    say("coarsened G mixed")
    _, _, states, _ = _solve(pr, [p], [u0], pr.PR_MODE_MIXED)
    for n in range(p.P + 1):
        assert rel_l2(states[0][n], hist[2, n]) <= FP32_TOL, n
    say("coarsened G modes")
    base, blog, _, _ = _solve(pr, [p], [u0], pr.PR_MODE_FP64)
    ps, plog, _, _ = _solve(pr, [p], [u0], pr.PR_MODE_FP64 | pr.PR_MODE_PER_SLICE)
    assert np.array_equal(ps[0], base[0]) and np.array_equal(plog, blog)
    q = W.small_problem(n=(32, 24, 20), a=(0.8, -0.5, 0.3), nu0=0.004, P=4, nf=8, nc=4, K=2,
                        flags=flags | W.SKIP_CONVERGED)
    sk, _, _, _ = _solve(pr, [q], [u0], pr.PR_MODE_FP64)
    assert np.array_equal(sk[0], base[0])
    plan = pr.Plan([p], pr.PR_MODE_FP64 | pr.PR_MODE_GRAPH)
    x = cuda(u0)
    for rep in range(3):
        uT, glog = plan.solve([x])
        scratch = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        assert np.array_equal(host(uT[0]), base[0]), rep
        assert np.array_equal(glog, blog), rep
        del scratch


def test_multi_instance_uneven(pr, orc):
    """Instances of different sizes, coefficients and step counts in one plan:
    each equals its own single-instance solve bitwise and the oracle to 1e-12."""
    probs, u0s = [], []
    for i, (n, nu0, a, nf, nc) in enumerate([(16, 0.01, (0.5, 0.3, -0.2), 4, 2), (24, 0.004, (-0.9, 0.2, 0.6), 6, 3),
                                             (20, 0.006, (0.3, -0.8, 0.1), 5, 2)]):
        p = W.small_problem(n=(n, n, n), a=a, nu0=nu0, P=4, nf=nf, nc=nc, K=2)
        probs.append(p)
        u0s.append(W.random_field(p.n, 210 + i))
    for mode in (pr.PR_MODE_FP64, pr.PR_MODE_MIXED):
        say("multi-instance mode", mode)
        uT, log, _, _ = _solve(pr, probs, u0s, mode)
        for i, p in enumerate(probs):
            one, one_log, _, _ = _solve(pr, [p], [u0s[i]], mode)
            assert np.array_equal(uT[i], one[0]), i
            assert np.array_equal(log[i], one_log[0]), i
            if mode == pr.PR_MODE_FP64:
                U, _ = orc.parareal(p, u0s[i], K=p.K)
                assert rel_l2(uT[i], U[-1]) <= FP64_TOL


def test_multi_instance_whole_row_kernels(pr, orc):
    """Instances that share n_x = 128 (whole-row F and G kernels) but differ in
    n_y, n_z, a, nu and step counts, in one FP64 plan: each instance matches
    the oracle and its own single-instance solve bitwise."""
    probs, u0s = [], []
    for i, (ny, nz, a, nu0, nf, nc) in enumerate([(24, 16, (0.7, -0.4, 0.2), 0.002, 8, 8),
                                                  (40, 12, (-0.5, 0.9, 0.3), 0.001, 10, 10)]):
        p = W.small_problem(n=(128, ny, nz), a=a, nu0=nu0, P=3, nf=nf, nc=nc, K=2)
        probs.append(p)
        u0s.append(W.random_field(p.n, 260 + i))
    plan = pr.Plan(probs, pr.PR_MODE_FP64)
    assert plan.kernel_variants()[0].startswith("rk4w_") and plan.kernel_variants()[1].startswith("euler4w_")
    uT, _ = plan.solve([cuda(u) for u in u0s])
    for i, p in enumerate(probs):
        say("whole-row multi-instance", i)
        U, _ = orc.parareal(p, u0s[i], K=p.K)
        got = host(uT[i])
        assert rel_l2(got, U[-1]) <= FP64_TOL, i
        one, _, _, _ = _solve(pr, [p], [u0s[i]], pr.PR_MODE_FP64)
        assert np.array_equal(one[0], got), i


@pytest.mark.parametrize("mode", [0, 1])
def test_multi_instance_x_tiled_rows(pr, orc, mode):
    """Instances of different widths (40, 100, 131) in one plan whose F and G
    run over x tiles: each launch covers items of different n_x (tiles per
    row from each item); every instance equals its own single-instance solve
    bitwise and, in FP64, the oracle."""
    probs, u0s = [], []
    for i, (n3, a, nu0, nf, nc) in enumerate([((40, 36, 20), (0.6, -0.4, 0.2), 0.002, 8, 8),
                                              ((100, 30, 24), (-0.5, 0.7, 0.3), 0.001, 10, 16),
                                              ((131, 20, 16), (0.4, 0.5, -0.6), 0.001, 12, 16)]):
        p = W.small_problem(n=n3, a=a, nu0=nu0, P=3, nf=nf, nc=nc, K=2)
        probs.append(p)
        u0s.append(W.random_field(p.n, 290 + i))
    dt = 2 if mode == pr.PR_MODE_FP64 else 1
    xf = "rk4x_f64_t56x8_p1x2_w8" if dt == 2 else "rk4x_f32_t56x40_p1x3_w16"
    xg = "euler4x_f64_t56x24_p1x2_w16" if dt == 2 else "euler4x_f32_t56x40_p1x3_w16"
    fi = {v["name"]: v["index"] for v in pr.variants(0)}[xf]
    gi = {v["name"]: v["index"] for v in pr.variants(1)}[xg]
    singles = []
    try:
        pr.set_kernel_variant(fi, gi)
        for i, p in enumerate(probs):
            singles.append(_solve(pr, [p], [u0s[i]], mode)[0][0])
        plan = pr.Plan(probs, mode)
        assert plan.kernel_variants() == (xf, xg)
        assert len(plan.fine_groups()) == 1
        uT, _ = plan.solve([cuda(u) for u in u0s])
    finally:
        pr.set_kernel_variant(0, 0)
    for i, p in enumerate(probs):
        say("x-tiled multi-instance", mode, i)
        got = host(uT[i])
        assert np.array_equal(got, singles[i]), i
        if mode == pr.PR_MODE_FP64:
            U, _ = orc.parareal(p, u0s[i], K=p.K)
            assert rel_l2(got, U[-1]) <= FP64_TOL, i


def test_multi_instance_launch_groups(pr, orc):
    """Instances whose grids call for different F kernels (whole rows of a
    wavefront at n_x = 128, of 16 lanes at n_x = 48) run as separate launch
    groups of one plan:
    every instance matches the oracle, and the batched, per-slice and
    graph-replayed solves, before and after tuning, agree bit for bit with
    the single-instance solves."""
    probs, u0s = [], []
    for i, (n3, a, nu0, nf, nc) in enumerate([((128, 24, 16), (0.7, -0.4, 0.2), 0.002, 8, 8),
                                              ((48, 36, 20), (-0.6, 0.5, 0.4), 0.004, 6, 4),
                                              ((128, 40, 12), (-0.5, 0.9, 0.3), 0.001, 10, 10)]):
        p = W.small_problem(n=n3, a=a, nu0=nu0, P=3, nf=nf, nc=nc, K=2)
        probs.append(p)
        u0s.append(W.random_field(p.n, 270 + i))
    for mode in (pr.PR_MODE_FP64, pr.PR_MODE_MIXED):
        say("launch groups mode", mode)
        singles = [_solve(pr, [p], [u0s[i]], mode)[0][0] for i, p in enumerate(probs)]
        if mode == pr.PR_MODE_FP64:
            for i, p in enumerate(probs):
                U, _ = orc.parareal(p, u0s[i], K=p.K)
                assert rel_l2(singles[i], U[-1]) <= FP64_TOL, i
        # skipping converged slices and early stopping at tol = 0 change no bit
        skip_early = [W.Problem(**{**p.__dict__, "flags": p.flags | W.SKIP_CONVERGED | W.EARLY_STOP})
                      for p in probs]
        skip_only = [W.Problem(**{**p.__dict__, "flags": p.flags | W.SKIP_CONVERGED}) for p in probs]
        pipe = pr.PR_MODE_PIPELINED
        for extra, ps in ((0, probs), (pr.PR_MODE_PER_SLICE, probs), (pr.PR_MODE_GRAPH, probs),
                          (pr.PR_MODE_TIMED, probs), (0, skip_early), (pipe, probs),
                          (pipe | pr.PR_MODE_GRAPH, skip_only), (pipe | pr.PR_MODE_PIPELINE_GROUPS(3), probs)):
            say("launch groups", mode, extra, ps[0].flags)
            # built-in kernel choices: a tuned table (from the previous round of
            # this loop) may pick one kernel that serves every grid, which
            # merges the groups
            pr.autotune_clear()
            plan = pr.Plan(ps, mode | extra)
            groups = plan.fine_groups()
            assert len(groups) == 2 and sorted(g[2] for g in groups) == [1, 2], groups
            assert any(g[0].startswith("rk4w_") for g in groups), groups
            for rep in range(2):
                if rep == 1:
                    plan.autotune()
                uT, _ = plan.solve([cuda(u) for u in u0s])
                for i in range(len(ps)):
                    assert np.array_equal(host(uT[i]), singles[i]), (mode, extra, rep, i)


def test_reference_defect_and_early_stop(pr, orc):
    import torch
    p = W.small_problem(n=(24, 24, 24), P=4, nf=6, nc=5, K=4)
    u0 = W.random_field(p.n, 220)
    ufine = orc.serial_fine(p, u0)
    say("ref defect")
    uT, log, _, _ = _solve(pr, [p], [u0], pr.PR_MODE_FP64, ref=[cuda(ufine)])
    _, _, hist = orc.parareal(p, u0, K=p.K, history=True)
    for k in range(p.K):
        nr = orc.norms(hist[k + 1, p.P], ufine)
        assert abs(log[0, k, 8] - nr[0]) <= 1e-12 * nr[1] + 1e-300
        assert abs(log[0, k, 9] - nr[1]) <= 1e-12 * nr[1]
    assert log[0, p.K - 1, 8] <= 1e-13 * log[0, p.K - 1, 9]   # K = P: exact
    say("early stop")
    q = W.small_problem(n=(24, 24, 24), P=4, nf=6, nc=5, K=4, flags=W.EARLY_STOP)
    q.tol = 1e30
    plan = pr.Plan([q], pr.PR_MODE_FP64)
    plan.solve([cuda(u0)])
    assert plan.iterations() == 1
    q.tol = 0.0
    plan = pr.Plan([q], pr.PR_MODE_FP64)
    plan.solve([cuda(u0)])
    assert plan.iterations() == 4


def test_nonfinite_input_is_reported(pr):
    say("nonfinite")
    p = W.small_problem(n=(16, 16, 16), P=2, nf=2, nc=5, K=1)
    u0 = W.random_field(p.n, 230)
    u0[3, 4, 5] = np.nan
    plan = pr.Plan([p], pr.PR_MODE_FP64)
    with pytest.raises(pr.PrError) as e:
        plan.solve([cuda(u0)])
    assert e.value.code == -6


def test_nan_propagates_through_norms_and_blocks_early_stop(pr):
    """A single NaN makes every maximum of the norms NaN (a max that dropped
    it would report a finite defect), and the early-stop test on a NaN
    defect never fires: the solve runs all K iterations and reports
    PR_ENONFINITE."""
    import torch
    say("nan norms")
    n3 = (24, 20, 18)
    x, r = W.random_field(n3, 231), W.random_field(n3, 232)
    x[5, 6, 7] = np.nan
    got = host(pr.defect_norm(cuda(x), cuda(r)))
    assert np.isnan(got[0, 0]) and np.isfinite(got[0, 1]) and np.isnan(got[0, 2])
    got = host(pr.defect_norm(cuda(r), cuda(x)))
    assert np.isnan(got[0, 0]) and np.isnan(got[0, 1])
    say("nan early stop")
    q = W.small_problem(n=(16, 16, 16), P=4, nf=4, nc=5, K=3, flags=W.EARLY_STOP)
    q.tol = 1e30
    u0 = W.random_field(q.n, 233)
    u0[2, 3, 4] = np.nan
    plan = pr.Plan([q], pr.PR_MODE_FP64)
    with pytest.raises(pr.PrError) as e:
        plan.solve([cuda(u0)])
    assert e.value.code == -6
    assert plan.iterations() == q.K


def test_plan_solve_rejects_mismatched_buffers(pr):
    import torch
    p = W.small_problem(n=(16, 12, 10), P=2, nf=2, nc=4, K=1)
    plan = pr.Plan([p], pr.PR_MODE_FP64)
    u0 = cuda(W.random_field(p.n, 234))
    with pytest.raises(ValueError, match="u0"):
        plan.solve([u0[:-1]])
    with pytest.raises(TypeError, match="u0"):
        plan.solve([u0.float()])
    with pytest.raises(ValueError, match="uT"):
        plan.solve([u0], uT=[torch.empty(p.npts + 8, dtype=torch.float64, device="cuda")])
    with pytest.raises(ValueError, match="ref"):
        plan.solve([u0], ref=[u0.reshape(-1)[:100]])
    with pytest.raises(ValueError, match="one tensor per instance"):
        plan.solve([u0, u0])
    uT, _ = plan.solve([u0])
    assert uT[0].shape == u0.shape


def test_plan_autotune_keeps_results(pr):
    """Tuning a plan's launches (variant and z-chunk depth) changes no bit of
    the result, eager or replayed from a graph recorded before the tuning."""
    probs, u0s = [], []
    for i, (n, nu0) in enumerate([(32, 0.004), (48, 0.006), (40, 0.005)]):
        p = W.small_problem(n=(n, n, n), nu0=nu0, P=4, nf=8, nc=8, K=2)
        probs.append(p)
        u0s.append(cuda(W.random_field(p.n, 250 + i)))
    for mode in (pr.PR_MODE_MIXED, pr.PR_MODE_FP64 | pr.PR_MODE_GRAPH):
        say("plan autotune mode", mode)
        plan = pr.Plan(probs, mode)
        before, blog = plan.solve(u0s)
        before = [host(x) for x in before]
        choice = plan.autotune()
        assert choice["fine"][1] in (0, 1, 2, 4) and choice["coarse"][1] in (0, 1, 2, 4)
        for rep in range(2):
            after, alog = plan.solve(u0s)
            for i in range(len(probs)):
                assert np.array_equal(host(after[i]), before[i]), (mode, rep, i)
            assert np.array_equal(alog, blog)


def test_autotune_keeps_results(pr):
    import torch
    p = W.small_problem(n=(64, 64, 64), nu0=0.002, P=2, nf=50, nc=50)
    u = cuda(W.random_field(p.n, 240))
    say("autotune")
    before = pr.fine_sweep(p, u, 0, 2)
    best = pr.autotune(p, 2, 1, 0)
    assert best >= 2
    after = pr.fine_sweep(p, u, 0, 2)
    assert torch.equal(before, after)
    bestc = pr.autotune(p, 2, 1, 1)
    assert bestc >= 2


# ---------------------------------------------------------------------------
# full-size workloads, sampled against the per-mode reference
# ---------------------------------------------------------------------------

def _samples(p, count=4096, seed=7):
    return np.random.default_rng(seed).integers(0, p.npts, size=count)


def _at(t, idx):
    """Values of a device field at flat indices, gathered on the device."""
    import torch
    return host(t.reshape(-1)[torch.from_numpy(idx).cuda()])


def test_full_size_c2_fp64(pr):
    """128^3, P = 16, K = 6, FP64 (the benchmark configuration): every slice
    state over the whole field against the exact discrete solution (the
    oracle's per-mode model, synthesised on the grid)."""
    from oracle import spectral as S
    say("c2 full size")
    p, modes = W.config("c2_128_fp64")
    u0 = W.synth_u0(p.n, modes)
    ms = S.ModalSolution(p, modes)
    plan = pr.Plan([p], pr.PR_MODE_FP64)
    uT, log = plan.solve([cuda(u0)])
    for n in range(p.P + 1):
        got = host(plan.slice_state(0, n)).reshape(p.n[2], p.n[1], p.n[0])
        ref = ms.iterate_fft(p.K, n)
        assert rel_l2(got, ref) <= FP64_TOL, n
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref)), n
    assert rel_l2(host(uT[0]).reshape(p.n[2], p.n[1], p.n[0]), ms.iterate_fft(p.K, p.P)) <= FP64_TOL


@pytest.mark.parametrize("cubic", [False, True])
def test_full_size_c2_coarsened_g(pr, cubic):
    """The 128^3 FP64 workload with G on the 64^3 grid (128 coarse steps, the
    smallest power of two the coarsened grid keeps stable), every slice state
    at sampled points against the alias-group modal solution."""
    from oracle import spectral as S
    say("c2 coarsened", cubic)
    p, modes = W.config("c2_128_fp64")
    p.nt_coarse = 128
    p.flags = W.COARSEN_G | (W.CUBIC_INTERP if cubic else 0)
    u0 = W.synth_u0(p.n, modes)
    ms = S.CoarsenedModalSolution(p, modes, order=3 if cubic else 1)
    plan = pr.Plan([p], pr.PR_MODE_FP64)
    plan.solve([cuda(u0)])
    idx = _samples(p)
    for n in range(p.P + 1):
        got = _at(plan.slice_state(0, n), idx)
        assert rel_l2(got, ms.iterate_points(p.K, n, idx)) <= FP64_TOL, n


def test_full_size_c3_mixed(pr):
    """256^3, P = 32, K = 6, FP32 sweeps with FP64 correction: every slice
    state within 1e-5 relative L2 of the FP64 discrete solution at samples,
    every eighth slice state and the result over the whole field."""
    from oracle import spectral as S
    say("c3 full size")
    p, modes = W.config("c3_256_mixed")
    u0 = W.synth_u0(p.n, modes)
    ms = S.ModalSolution(p, modes)
    plan = pr.Plan([p], pr.PR_MODE_MIXED)
    uT, log = plan.solve([cuda(u0)])
    idx = _samples(p)
    for n in range(p.P + 1):
        got = _at(plan.slice_state(0, n), idx)
        ref = ms.iterate_points(p.K, n, idx)
        assert rel_l2(got, ref) <= FP32_TOL, n
    # every eighth slice state and the result over the whole field
    shape = (p.n[2], p.n[1], p.n[0])
    for n in range(0, p.P + 1, 8):
        got = host(plan.slice_state(0, n)).reshape(shape)
        assert rel_l2(got, ms.iterate_fft(p.K, n)) <= FP32_TOL, n
    assert rel_l2(host(uT[0]).reshape(shape), ms.iterate_fft(p.K, p.P)) <= FP32_TOL


def test_paper_setup_fourth_order(pr):
    """The paper's benchmark (Section 3.1): 128^3, c = (1,1,1), nu0 = 0.1,
    omega = 100, T = 0.1, fourth-order F with dt = T/2^15 (nu frozen per
    step), G with Dt = T/2^11, P = 8, K = 3.  The GPU serial fine error
    against the continuous solution is the printed 4.8e-6, and the defects
    d^k of the GPU Parareal iterates match the exact discrete ones."""
    from oracle import spectral as S
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    say("paper setup")
    p = W.paper_setup(100.0, P=8, K=3)
    p.flags = W.NU_FROZEN
    m = W.single_mode((1, 1, 1))
    u0 = W.synth_u0(p.n, m)
    x = cuda(u0)
    uf = pr.fine_sweep(p, x, 0, p.nt_fine)
    ufh = host(uf)
    ex = S.analytic(p, m, p.T)
    eps = np.max(np.abs(ufh - ex)) / np.max(np.abs(ex))
    assert abs(eps - gold["eps_fine"]["omega_100"]) <= 0.05 * gold["eps_fine"]["omega_100"], eps
    plan = pr.Plan([p], pr.PR_MODE_FP64)
    uT, log = plan.solve([x], ref=[uf])
    ms = S.ModalSolution(p, m)
    fine = ms.serial_fine()
    assert rel_l2(ufh, fine) <= FP64_TOL
    for k in range(p.K):
        d_gpu = log[0, k, 8] / log[0, k, 9]
        it = ms.iterate(k + 1, p.P)
        d_ref = np.max(np.abs(it - fine)) / np.max(np.abs(fine))
        assert abs(d_gpu - d_ref) <= 1e-3 * d_ref, (k, d_gpu, d_ref)
    assert log[0, 2, 8] / log[0, 2, 9] < 0.1 * gold["eps_fine"]["omega_100"]


@pytest.mark.parametrize("omega,P", [(0.0, 8), (0.0, 32), (100.0, 32)])
def test_paper_setup_defects_after_three_iterations(pr, omega, P):
    """Section 3.3.1 on the GPU: the paper's setup (fourth-order F, nu frozen
    per step) with N_p slices.  The serial fine error is the printed eps_fine
    of this omega; d^k of the GPU iterates equals the exact discrete value;
    after three iterations d^3 is far below eps_fine for omega = 100 and of
    its order for omega = 0, and smaller than d^2."""
    from oracle import spectral as S
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    eps = gold["eps_fine"]["omega_0" if omega == 0.0 else "omega_100"]
    say("paper setup omega", omega, "P", P)
    p = W.paper_setup(omega, P=P, K=3)
    p.flags = W.NU_FROZEN
    m = W.single_mode((1, 1, 1))
    x = cuda(W.synth_u0(p.n, m))
    uf = pr.fine_sweep(p, x, 0, p.nt_fine)
    ufh = host(uf)
    ex = S.analytic(p, m, p.T)
    e_fine = np.max(np.abs(ufh - ex)) / np.max(np.abs(ex))
    assert abs(e_fine - eps) <= 0.05 * eps, e_fine
    plan = pr.Plan([p], pr.PR_MODE_FP64)
    _, log = plan.solve([x], ref=[uf])
    ms = S.ModalSolution(p, m)
    fine = ms.serial_fine()
    d = [log[0, k, 8] / log[0, k, 9] for k in range(p.K)]
    for k in range(p.K):
        it = ms.iterate(k + 1, p.P)
        d_ref = np.max(np.abs(it - fine)) / np.max(np.abs(fine))
        assert abs(d[k] - d_ref) <= 1e-3 * d_ref, (k, d[k], d_ref)
    if omega == 0.0:
        assert 0.1 * eps < d[2] < 10 * eps, d[2]
    else:
        assert d[2] < 0.1 * eps, d[2]
    assert d[2] < d[1]


def test_full_size_c4_batched(pr):
    """64 uneven instances (48^3..128^3, own a and nu0, P = 8, K = 3) in one
    mixed-precision plan: every instance's final state within 1e-5 of its
    exact discrete solution over the whole field; one instance bitwise equal
    to its own single-instance solve."""
    import torch
    from oracle import spectral as S
    insts = W.batched_config(64)
    probs = [p for p, _ in insts]
    say("c4 batched: %d instances" % len(probs))
    u0s = [cuda(W.synth_u0(p.n, m)) for p, m in insts]
    # per fine step one launch per kernel group over all slices of its
    # instances (groups concurrent), tuned tiles and z chunks, the whole
    # solve replayed from a recorded graph
    plan = pr.Plan(probs, pr.PR_MODE_MIXED | pr.PR_MODE_GRAPH)
    say("c4 tuned", plan.autotune())
    uT, log = plan.solve(u0s)
    for i, (p, m) in enumerate(insts):
        ms = S.ModalSolution(p, m)
        got = host(uT[i]).reshape(p.n[2], p.n[1], p.n[0])
        assert rel_l2(got, ms.iterate_fft(p.K, p.P)) <= FP32_TOL, (i, p.n)   # whole field
    del plan
    torch.cuda.empty_cache()
    j = next(i for i, p in enumerate(probs) if p.n[0] == 96)
    one = pr.Plan([probs[j]], pr.PR_MODE_MIXED)
    uj, _ = one.solve([u0s[j]])
    assert torch.equal(uj[0], uT[j])


def test_full_size_c5_mixed(pr):
    """The largest workload: 512^3, P = 32, K = 5, FP32 sweeps (all slice
    states resident, ~110 GB): every fourth slice state within 1e-5 relative
    L2 of the FP64 discrete solution at sampled points, the result over the
    whole field."""
    import torch
    from oracle import spectral as S
    say("c5 full size")
    p, modes = W.config("c5_512_mixed")
    u0 = cuda(W.synth_u0(p.n, modes))
    plan = pr.Plan([p], pr.PR_MODE_MIXED)
    uT, log = plan.solve([u0])
    ms = S.ModalSolution(p, modes)
    idx = _samples(p, count=2048)
    for n in range(0, p.P + 1, 4):
        got = _at(plan.slice_state(0, n), idx)
        assert rel_l2(got, ms.iterate_points(p.K, n, idx)) <= FP32_TOL, n
    assert rel_l2(_at(uT[0], idx), ms.iterate_points(p.K, p.P, idx)) <= FP32_TOL
    del plan
    torch.cuda.empty_cache()
    # the result over the whole field (one inverse FFT of 512^3 on the host)
    say("c5 whole-field result")
    got = host(uT[0]).reshape(p.n[2], p.n[1], p.n[0])
    assert rel_l2(got, ms.iterate_fft(p.K, p.P)) <= FP32_TOL
    torch.cuda.empty_cache()
