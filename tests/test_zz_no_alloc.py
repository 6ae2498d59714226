"""lbfv_totals_device, the allocation-free form of lbfv_totals, through the C ABI.

It enqueues the same totals reduction as lbfv_totals, with its per-block partial sums
in the library's fixed scratch array instead of a buffer it allocates, and writes the
three totals and the non-finite count to caller-owned device memory.  Compared with
lbfv_totals on two calls in a row, the second on a smaller mesh (and another storage
form): the same bits.
"""
import ctypes as C

import numpy as np
import pytest

from paper_1511_00242_amd import inputs as I
from paper_1511_00242_amd import lbfv as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    yield


def _totals_device(ctx, out):
    return L.lib().lbfv_totals_device(ctx.h, C.c_void_p(out.data_ptr()))


def test_totals_device_equals_totals_on_two_calls():
    import torch
    stream = torch.cuda.current_stream()
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    runs = [(I.taylor_green(700), L.LBFV_FP64, L.LBFV_STORE_NATIVE, L.LBFV_DUGKS, 6),
            (I.cavity(64, stretched=True), L.LBFV_FP32, L.LBFV_STORE_DEV_FP32, L.LBFV_BKG, 9)]
    for w, compute, storage, scheme, n in runs:
        with L.Context(w.xf, w.yf, w.tau, w.dt, rt=w.rt, bcs=w.bcs, compute=compute, storage=storage,
                       stream=stream.cuda_stream) as ctx:
            ctx.init_equilibrium(w.rho, w.ux, w.uy)
            # before the mesh metrics are on the device the call refuses (their upload allocates)
            assert _totals_device(ctx, out) == L.LBFV_ESTATE
            assert "metrics" in L.lib().lbfv_last_error(ctx.h).decode()
            ctx.step(scheme, n)
            assert _totals_device(ctx, out) == L.LBFV_OK
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            ref = ctx.totals()
            print(f"{w.name} {w.nx}x{w.ny} compute={compute}: totals_device {got[:3]} count {got[3]}; "
                  f"totals {ref}", flush=True)
            assert np.array_equal(got[:3], ref)
            assert got[3] == 0.0
            assert L.lib().lbfv_totals_device(ctx.h, None) == L.LBFV_EINVAL


def test_totals_device_counts_non_finite_cells():
    import torch
    stream = torch.cuda.current_stream()
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    w = I.taylor_green(48)
    with L.Context(w.xf, w.yf, w.tau, w.dt, rt=w.rt, bcs=w.bcs, stream=stream.cuda_stream) as ctx:
        ctx.init_equilibrium(w.rho, w.ux, w.uy)
        ctx.dugks_step(1)
        f = ctx.get_f()
        f[3, 7, 11] = np.nan
        f[0, 40, 2] = np.inf
        ctx.set_f(f)
        assert _totals_device(ctx, out) == L.LBFV_OK
        torch.cuda.synchronize()
        assert out.cpu().numpy()[3] == 2.0
