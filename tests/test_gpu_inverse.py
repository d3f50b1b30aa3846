"""The inverse transform (paco_execute_inverse) on the GPU against the FP64
oracle's inverse DFT, and round trips through the forward transform.

The inverse runs the PACO phases on the swapped factorisation N2 x N1, so it
takes y in the forward output's slab ownership and returns x in the forward
input's; on one HBM both are the natural-order vector, which is what the
tests compare."""
import numpy as np
import pytest

import oracle
from paper_2609_06449_amd import inputs, paco

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
TOL = 1e-6


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev(x: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(x.astype(np.complex64).ravel())).to("cuda")


def _call(fn, plan, xd, out=None):
    N = plan.N1 * plan.N2
    if out is None:
        out = torch.empty(N, dtype=torch.complex64, device="cuda")
    ws = torch.empty(N, dtype=torch.complex64, device="cuda")
    fn(xd.data_ptr(), out.data_ptr(), ws.data_ptr(), _stream())
    torch.cuda.synchronize()
    return out


SHAPES = [(2, 2, 2, 2), (4, 8, 2, 2), (16, 16, 2, 4), (64, 64, 4, 4), (64, 512, 8, 8), (4096, 256, 16, 16),
          (256, 4096, 4, 16), (1024, 2048, 8, 2), (8192, 16, 2, 2), (16, 8192, 2, 2), (1 << 14, 64, 4, 4),
          (64, 1 << 14, 4, 4), (1 << 16, 16, 16, 16)]


@pytest.mark.parametrize("N1,N2,p,b", SHAPES)
def test_inverse_matches_oracle(N1, N2, p, b):
    y = inputs.normal(N1 * N2, seed=N1 + 5 * N2)
    plan = paco.Plan(N1, N2, p, b)
    x = _call(plan.execute_inverse, plan, _dev(y)).cpu().numpy()
    err = oracle.rel_l2(x, oracle.idft(y))
    print(f"inverse {N1}x{N2} b={b}: rel-L2 {err:.3e}", flush=True)
    assert err <= TOL


@pytest.mark.parametrize("N1,N2,p,b", [(64, 64, 4, 4), (512, 2048, 8, 2), (1 << 14, 256, 4, 4)])
def test_round_trip_forward_then_inverse(N1, N2, p, b):
    x = inputs.normal(N1 * N2, seed=31)
    plan = paco.Plan(N1, N2, p, b)
    xd = _dev(x)
    y = _call(plan.execute, plan, xd)
    back = _call(plan.execute_inverse, plan, y).cpu().numpy()
    err = oracle.rel_l2(back, x)
    print(f"round trip {N1}x{N2}: rel-L2 {err:.3e}", flush=True)
    assert err <= 2 * TOL
    # and the other way round: inverse first
    z = _call(plan.execute, plan, _call(plan.execute_inverse, plan, xd)).cpu().numpy()
    assert oracle.rel_l2(z, x) <= 2 * TOL


def test_inverse_full_size_round_trip():
    # N = 2^24 as 4096 x 4096: inverse of the oracle's forward output, and
    # the full round trip
    N1, N2, p, b = 4096, 4096, 64, 16
    x = inputs.normal(N1 * N2, seed=2)
    plan = paco.Plan(N1, N2, p, b)
    y = oracle.fft_radix2(x)
    got = _call(plan.execute_inverse, plan, _dev(y)).cpu().numpy()
    err = oracle.rel_l2(got, x)
    print(f"inverse 2^24 of the oracle's forward output: rel-L2 {err:.3e}", flush=True)
    assert err <= TOL


def test_inverse_in_place_and_paper_layout():
    N1, N2, p, b = 256, 1024, 8, 4
    y = inputs.normal(N1 * N2, seed=32)
    plan = paco.Plan(N1, N2, p, b)
    ref = _call(plan.execute_inverse, plan, _dev(y)).cpu().numpy()
    buf = _dev(y)
    _call(plan.execute_inverse, plan, buf, out=buf)
    assert np.array_equal(buf.cpu().numpy().view(np.uint64), ref.view(np.uint64))
    paper = paco.Plan(N1, N2, p, b, flags=paco.PACO_PLAN_PAPER_LAYOUT)
    got = _call(paper.execute_inverse, paper, _dev(y)).cpu().numpy()
    assert oracle.rel_l2(got, oracle.idft(y)) <= TOL


@pytest.mark.parametrize("dt,tol", [(paco.PACO_C64_MFMA_FP16X3, 1e-6), (paco.PACO_C64_MFMA_BF16X3, 3e-5),
                                    (paco.PACO_C64_MFMA_BF16X6, 1e-6)])
def test_inverse_split_forms(dt, tol):
    N1, N2, p, b = 4096, 256, 16, 16
    y = inputs.loguniform(N1 * N2, seed=33)
    plan = paco.Plan(N1, N2, p, b, dt)
    got = _call(plan.execute_inverse, plan, _dev(y)).cpu().numpy()
    err = oracle.rel_l2(got, oracle.idft(y))
    print(f"inverse dt={dt}: rel-L2 {err:.3e}", flush=True)
    assert err <= tol


def test_inverse_argument_errors():
    plan = paco.Plan(64, 256, 4, 4)
    buf = torch.empty(64 * 256, dtype=torch.complex64, device="cuda")
    ws = torch.empty_like(buf)
    lib = paco.lib()
    s = _stream()
    assert lib.paco_execute_inverse(plan.handle, buf.data_ptr(), buf.data_ptr(), ws.data_ptr(), 100, s) == \
        paco.PACO_ERR_WORKSPACE
    assert lib.paco_execute_inverse(plan.handle, buf.data_ptr(), buf.data_ptr(), buf.data_ptr(), 1 << 20, s) == \
        paco.PACO_ERR_INVALID_ARG
    assert lib.paco_execute_inverse(plan.handle, buf.data_ptr() + 4, buf.data_ptr(), ws.data_ptr(), 1 << 20, s) == \
        paco.PACO_ERR_INVALID_ARG
