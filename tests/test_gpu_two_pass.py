"""The two-pass form (paco_execute_two_pass) on the GPU: Phase I into the
packed buffer, then Phase III straight from it with the top-level twiddle
formed on load (the fused global permutation of section 4.2 with pi_{m2}
cancelled against Phase III's input-layout read, pi_{m2} being an
involution).  The output is the same DFT as paco_execute's, held to the
same FP32 target against the FP64 oracle; it is not bit-equal to the
three-pass output (the twiddle is formed from two other table factors)."""
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


def _two_pass(plan, xd, out=None):
    N = plan.N1 * plan.N2
    if out is None:
        out = torch.empty(N, dtype=torch.complex64, device="cuda")
    ws = torch.empty(N, dtype=torch.complex64, device="cuda")
    plan.execute_two_pass(xd.data_ptr(), out.data_ptr(), ws.data_ptr(), _stream())
    torch.cuda.synchronize()
    return out.cpu().numpy()


SHAPES = [(64, 64, 4, 4), (128, 64, 4, 2), (64, 512, 8, 8), (512, 512, 8, 8), (4096, 256, 16, 16),
          (256, 4096, 4, 16), (1024, 2048, 8, 2), (2048, 1024, 16, 2), (4096, 64, 4, 4), (64, 4096, 64, 4)]


@pytest.mark.parametrize("N1,N2,p,b", SHAPES)
def test_two_pass_matches_oracle(N1, N2, p, b):
    x = inputs.normal(N1 * N2, seed=N1 * 3 + N2)
    plan = paco.Plan(N1, N2, p, b)
    assert plan.has_two_pass, plan.description
    assert "two_pass" in plan.description
    y = _two_pass(plan, _dev(x))
    err = oracle.rel_l2(y, oracle.dft(x))
    print(f"two-pass {N1}x{N2} b={b}: rel-L2 {err:.3e}", flush=True)
    assert err <= TOL


def test_two_pass_full_size_against_oracle():
    # N = 2^24 as 4096 x 4096, p = 64, b = 16, N(0,1) inputs, seed 2
    N1, N2, p, b = 4096, 4096, 64, 16
    N = N1 * N2
    x = inputs.normal(N, seed=2)
    plan = paco.Plan(N1, N2, p, b)
    y = _two_pass(plan, _dev(x))
    ref = oracle.fft_radix2(x)
    err = oracle.rel_l2(y, ref)
    print(f"two-pass 2^24 rel-L2 {err:.3e}", flush=True)
    assert err <= TOL
    ks = np.array([0, 1, 4095, 4096, N // 2, N - 1, 12345678, 9876543])
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    assert np.max(np.abs(y[ks] - oracle.dft_at(x, ks))) < 1e-5 * rms


def test_two_pass_in_place_and_deterministic():
    N1, N2, p, b = 1024, 512, 8, 2
    x = inputs.normal(N1 * N2, seed=21)
    plan = paco.Plan(N1, N2, p, b)
    buf = _dev(x)
    a = _two_pass(plan, _dev(x))
    c = _two_pass(plan, buf, out=buf)  # in == out
    assert np.array_equal(a.view(np.uint64), c.view(np.uint64))
    assert oracle.rel_l2(a, oracle.dft(x)) <= TOL


@pytest.mark.parametrize("N1,N2,p,b,dt,layout", [
    (64, 64, 4, 4, paco.PACO_C64, "paper"),                 # not fused
    (64, 64, 4, 4, paco.PACO_C64_MFMA_BF16X3, None),       # split MFMA form
    (64, 8192, 4, 2, paco.PACO_C64, None),                 # Phase III in two on-chip passes
    (8192, 64, 4, 2, paco.PACO_C64, None),                 # Phase I in two passes: not fused
    (16, 16, 2, 4, paco.PACO_C64, None),                   # slabs below one 64-item tile: not fused
])
def test_two_pass_unsupported_plans(N1, N2, p, b, dt, layout):
    plan = paco.Plan(N1, N2, p, b, dt, flags=paco.PACO_PLAN_PAPER_LAYOUT if layout == "paper" else 0)
    assert not plan.has_two_pass
    buf = torch.empty(N1 * N2, dtype=torch.complex64, device="cuda")
    ws = torch.empty_like(buf)
    st = paco.lib().paco_execute_two_pass(plan.handle, buf.data_ptr(), buf.data_ptr(), ws.data_ptr(),
                                          plan.workspace_bytes, _stream())
    assert st == paco.PACO_ERR_UNSUPPORTED


def test_two_pass_argument_errors():
    plan = paco.Plan(64, 64, 4, 4)
    buf = torch.empty(4096, dtype=torch.complex64, device="cuda")
    ws = torch.empty(4096, dtype=torch.complex64, device="cuda")
    lib = paco.lib()
    s = _stream()
    assert lib.paco_execute_two_pass(plan.handle, buf.data_ptr(), buf.data_ptr(), ws.data_ptr(), 100, s) == \
        paco.PACO_ERR_WORKSPACE
    assert lib.paco_execute_two_pass(plan.handle, buf.data_ptr() + 8, buf.data_ptr(), ws.data_ptr(), 1 << 20, s) == \
        paco.PACO_ERR_INVALID_ARG
    assert lib.paco_execute_two_pass(plan.handle, buf.data_ptr(), buf.data_ptr(), buf.data_ptr(), 1 << 20, s) == \
        paco.PACO_ERR_INVALID_ARG


@pytest.mark.parametrize("N1,N2,p,b", [(64, 64, 4, 4), (4096, 512, 8, 2), (256, 4096, 4, 16)])
def test_two_pass_phase3_stage(N1, N2, p, b):
    # stage 3 with PACO_PACKED is the two-pass Phase III: on a seeded packed
    # buffer W[c, v] = A[v, c] it equals the oracle's twiddled middle stage
    # followed by its Phase III, and stage 1 + stage 3 (both packed) is
    # paco_execute_two_pass bit for bit
    plan = paco.Plan(N1, N2, p, b)
    s = _stream()
    W = inputs.normal(N1 * N2, seed=22).reshape(N2, N1)
    t = b.bit_length() - 1
    m1 = round(np.log2(N1)) // t
    pi1 = np.array([oracle.digit_reverse(a, b, m1) for a in range(N1)])
    Atilde = W.T[pi1, :]                      # paper-layout Phase-I buffer holding the same A
    want = oracle.phase3(oracle.phase2(Atilde, N1, N2, b, twiddle=True), N1, N2, b)
    wd = _dev(W)
    got = torch.empty_like(wd)
    plan.execute_stage(3, wd.data_ptr(), got.data_ptr(), s, paco.PACO_PACKED)
    torch.cuda.synchronize()
    assert oracle.rel_l2(got.cpu().numpy().reshape(N2, N1), want) <= TOL
    plan.execute_stage(3, wd.data_ptr(), wd.data_ptr(), s, paco.PACO_PACKED)  # in place
    torch.cuda.synchronize()
    assert np.array_equal(wd.cpu().numpy().view(np.uint64), got.cpu().numpy().view(np.uint64))
    x = _dev(inputs.normal(N1 * N2, seed=23))
    ws = torch.empty_like(x)
    y = torch.empty_like(x)
    plan.execute_stage(1, x.data_ptr(), ws.data_ptr(), s, paco.PACO_PACKED | paco.PACO_TWO_PASS)
    plan.execute_stage(3, ws.data_ptr(), y.data_ptr(), s, paco.PACO_PACKED)
    ref = _two_pass(plan, x)
    assert np.array_equal(y.cpu().numpy().view(np.uint64), ref.view(np.uint64))
    # the two-pass Phase I writes the same packed buffer as the three-pass one
    ws3 = torch.empty_like(x)
    plan.execute_stage(1, x.data_ptr(), ws3.data_ptr(), s, paco.PACO_PACKED)
    torch.cuda.synchronize()
    assert np.array_equal(ws.cpu().numpy().view(np.uint64), ws3.cpu().numpy().view(np.uint64))


def test_packed_stage3_flag_errors():
    lib = paco.lib()
    s = _stream()
    buf = torch.empty(4096, dtype=torch.complex64, device="cuda")
    out = torch.empty_like(buf)
    paper = paco.Plan(64, 64, 4, 4, flags=paco.PACO_PLAN_PAPER_LAYOUT)
    assert lib.paco_execute_stage(paper.handle, 3, paco.PACO_PACKED, buf.data_ptr(), out.data_ptr(), s) == \
        paco.PACO_ERR_UNSUPPORTED
    fused = paco.Plan(64, 64, 4, 4)
    for stage in (1, 3):
        assert lib.paco_execute_stage(fused.handle, stage, paco.PACO_NO_TWIDDLE, buf.data_ptr(), out.data_ptr(), s) == \
            paco.PACO_ERR_INVALID_ARG
    for stage, fl in ((1, paco.PACO_TWO_PASS), (3, paco.PACO_TWO_PASS | paco.PACO_PACKED), (2, paco.PACO_TWO_PASS | paco.PACO_PACKED)):
        assert lib.paco_execute_stage(fused.handle, stage, fl, buf.data_ptr(), out.data_ptr(), s) == \
            paco.PACO_ERR_INVALID_ARG
    assert lib.paco_execute_stage(paper.handle, 1, paco.PACO_PACKED | paco.PACO_TWO_PASS, buf.data_ptr(),
                                  out.data_ptr(), s) == paco.PACO_ERR_UNSUPPORTED
