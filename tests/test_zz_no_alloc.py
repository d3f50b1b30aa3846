"""paco_execute_noalloc: the transform of paco_execute with the workspace in
the library's own per-GPU device array, for callers that cannot allocate.

Checked through the C ABI against paco_execute (the same kernels, so the
same bits) on two calls in a row, the second with a smaller transform, in
place as well, and its refusal of a transform above the array's size."""
import ctypes

import numpy as np
import pytest

from paper_2609_06449_amd import inputs, paco

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _reference(plan, xd):
    out = torch.empty_like(xd)
    ws = torch.empty_like(xd)
    plan.execute(xd.data_ptr(), out.data_ptr(), ws.data_ptr(), _stream())
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _noalloc(plan, xd, out=None):
    if out is None:
        out = torch.empty_like(xd)
    st = paco.lib().paco_execute_noalloc(ctypes.c_void_p(plan.handle), ctypes.c_void_p(xd.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(_stream()))
    assert st == paco.PACO_OK, paco.paco_last_error()
    torch.cuda.synchronize()
    return out


def test_noalloc_matches_execute_on_two_calls():
    # the largest transform the array holds (2^22 items, the split form's
    # 4096 x 1024 plan), then a smaller one (64 x 64): the second call finds
    # the first one's contents in the array and must not depend on them
    cases = [(4096, 1024, 64, 4), (64, 64, 4, 4)]
    for N1, N2, p, b in cases:
        N = N1 * N2
        assert N <= paco.PACO_NOALLOC_MAX_ITEMS
        plan = paco.Plan(N1, N2, p, b)
        xd = torch.from_numpy(inputs.normal(N, seed=N1 + N2)).to("cuda")
        want = _reference(plan, xd)
        free0 = torch.cuda.mem_get_info()[0]
        got = _noalloc(plan, xd).cpu().numpy()
        print(f"{N1}x{N2}: {plan.description}", flush=True)
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
        # in place (in == out)
        buf = xd.clone()
        _noalloc(plan, buf, out=buf)
        assert np.array_equal(buf.cpu().numpy().view(np.uint64), want.view(np.uint64))
        assert torch.cuda.mem_get_info()[0] >= free0  # nothing new held on the device
        plan.close()


def test_noalloc_refuses_a_transform_above_the_array():
    plan = paco.Plan(4096, 2048, 64, 2)  # 2^23 items
    x = torch.empty(plan.N1 * plan.N2, dtype=torch.complex64, device="cuda")
    st = paco.lib().paco_execute_noalloc(ctypes.c_void_p(plan.handle), ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(_stream()))
    assert st == paco.PACO_ERR_WORKSPACE
    assert "PACO_NOALLOC_MAX_ITEMS" in paco.paco_last_error()
    assert paco.lib().paco_execute_noalloc(None, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                           None) == paco.PACO_ERR_INVALID_ARG
