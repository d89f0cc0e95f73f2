"""The allocation-free norm entry point (pr_defect_norm_static) against the
workspace entry point (pr_defect_norm) through the C ABI: bitwise the same
out4 on two calls in a row, the second with a smaller input, on a GPU."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _call_ws(L, torch, x, r, batch, xd, rd):
    n = x.numel() // batch
    out = torch.full((batch, 4), -1.0, dtype=torch.float64, device="cuda")
    ws = torch.empty(L.lib().pr_defect_workspace_bytes(batch), dtype=torch.uint8, device="cuda")
    L.check(L.lib().pr_defect_norm(n, batch, xd, ctypes.c_void_p(x.data_ptr()), rd, ctypes.c_void_p(r.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _call_static(L, torch, x, r, batch, xd, rd):
    n = x.numel() // batch
    out = torch.full((batch, 4), -1.0, dtype=torch.float64, device="cuda")
    L.check(L.lib().pr_defect_norm_static(n, batch, xd, ctypes.c_void_p(x.data_ptr()), rd,
                                          ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_static_defect_norm_matches_workspace_entry_point():
    import torch
    from paper_1409_8563_amd import _lib as L
    torch.cuda.set_device(0)
    g = torch.Generator(device="cpu").manual_seed(1409)
    cases = [  # (batch, points per field, x dtype, ref dtype): the second call is smaller
        (L.PR_DEFECT_STATIC_MAX_BATCH, 40 * 36 * 20 + 7, torch.float64, torch.float64),
        (3, 1000, torch.float32, torch.float64),
    ]
    codes = {torch.float32: L.PR_FP32, torch.float64: L.PR_FP64}
    for batch, n, xdt, rdt in cases:
        print("case batch=%d n=%d x=%s ref=%s" % (batch, n, xdt, rdt), flush=True)
        r = torch.randn(batch * n, generator=g, dtype=torch.float64).to(rdt).cuda()
        x = (r.double() + 1e-3 * torch.randn(batch * n, generator=g, dtype=torch.float64).cuda()).to(xdt)
        want = _call_ws(L, torch, x, r, batch, codes[xdt], codes[rdt])
        got = _call_static(L, torch, x, r, batch, codes[xdt], codes[rdt])
        assert np.array_equal(got, want), (batch, n, got, want)
        # the reduction itself, in FP64 on the host
        xh = x.double().cpu().numpy().reshape(batch, n)
        rh = r.double().cpu().numpy().reshape(batch, n)
        d = xh - rh
        assert np.array_equal(got[:, 0], np.abs(d).max(axis=1))
        assert np.array_equal(got[:, 1], np.abs(rh).max(axis=1))
        np.testing.assert_allclose(got[:, 2], (d * d).sum(axis=1), rtol=1e-12)
        np.testing.assert_allclose(got[:, 3], (rh * rh).sum(axis=1), rtol=1e-12)
