"""The split form of the fused pipeline on the GPU (FP32, N1 = 4096):
Phase I's column transforms split once more by Lemma 1 as 16 x 256, pass 1
taking the first radix-16 stage with its twiddle (read in whole 128-byte
row runs of x), pass 2 the 256-point tails together with Phase II's
redistribution and top-level twiddle.  Checked against the FP64 oracle: the
whole transform, each pass on its own (pass 1 against the oracle's 16-point
DFTs, pass 2 against the oracle's Phase II output), the stage hooks
composing to paco_execute bit for bit, and the entry-point checks."""

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


def _execute(plan, xd, out=None):
    N = plan.N1 * plan.N2
    if out is None:
        out = torch.empty(N, dtype=torch.complex64, device="cuda")
    ws = torch.empty(N, dtype=torch.complex64, device="cuda")
    plan.execute(xd.data_ptr(), out.data_ptr(), ws.data_ptr(), _stream())
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _stage(plan, stage, src, flags):
    dst = torch.empty(plan.N1 * plan.N2, dtype=torch.complex64, device="cuda")
    plan.execute_stage(stage, src.data_ptr(), dst.data_ptr(), _stream(), flags)
    torch.cuda.synchronize()
    return dst


def _packed_plan(N1, N2, p, b):
    return paco.Plan(N1, N2, p, b, flags=paco.PACO_PLAN_NO_SPLIT)


def _split_buffer(x, N1, N2):
    """T[c][j][k0] = w_4096^{-j k0} * DFT_16(X[j + 256 r, c] over r)[k0],
    laid out as the pass-1 buffer [c*N1 + 16 j + k0]; the 16-point DFTs are
    the oracle's, the twiddle is evaluated in FP64 from the exact product."""
    X = x.astype(np.complex128).reshape(16, N1 // 16, N2)  # [r, j, c]
    T = np.empty((N2, N1 // 16, 16), dtype=np.complex128)
    for c in range(N2):
        for j in range(N1 // 16):
            T[c, j] = oracle.dft(X[:, j, c])
    jk = np.outer(np.arange(N1 // 16), np.arange(16)) % N1
    T *= np.exp(-2j * np.pi * jk / N1)[None, :, :]
    return T.ravel()


SHAPES = [(4096, 64, 4, 4), (4096, 256, 16, 16), (4096, 512, 8, 2), (4096, 1024, 16, 4), (4096, 128, 64, 2),
          (4096, 16384, 64, 4), (4096, 512, 8, 8)]  # b = 8: the general digit reversal in pass 2


@pytest.mark.parametrize("N1,N2,p,b", SHAPES)
def test_split_matches_oracle(N1, N2, p, b):
    x = inputs.normal(N1 * N2, seed=N2 + 7)
    # (4096 x 16384 runs the symmetric split form by default: the option
    # keeps this form, which the other shapes take anyway)
    plan = paco.Plan(N1, N2, p, b, flags=paco.PACO_PLAN_NO_SYM)
    assert plan.has_split, plan.description
    assert plan.description.startswith("fused[") and "split[" in plan.description
    y = _execute(plan, _dev(x))
    err = oracle.rel_l2(y, oracle.dft(x))
    print(f"split {N1}x{N2} p={p} b={b}: rel-L2 {err:.3e}", flush=True)
    assert err <= TOL


# N1 = 2^13, 2^14: pass 2 runs 512- / 1024-point tails in three stages and
# replaces Phase I's two on-chip passes and Phase II
LONG_SHAPES = [(8192, 64, 4, 2), (16384, 64, 4, 4), (16384, 256, 16, 4), (8192, 128, 8, 2), (16384, 128, 64, 2)]


@pytest.mark.parametrize("N1,N2,p,b", LONG_SHAPES)
def test_split_long_columns_match_oracle(N1, N2, p, b):
    x = inputs.normal(N1 * N2, seed=N1 // 64 + N2)
    plan = paco.Plan(N1, N2, p, b)
    assert plan.has_split and f"pass2: {N1 // 16}-point tails" in plan.description, plan.description
    y = _execute(plan, _dev(x))
    err = oracle.rel_l2(y, oracle.dft(x))
    print(f"split {N1}x{N2} p={p} b={b}: rel-L2 {err:.3e}", flush=True)
    assert err <= TOL


@pytest.mark.parametrize("N1,N2,p,b", [(16384, 256, 16, 16), (8192, 512, 8, 8)])
def test_split_long_columns_mixed_radix(N1, N2, p, b):
    # 2^14 = 16^3 * 4 and 2^13 = 8^4 * 2: mixed-radix plans (b = 8: the general digit reversal)
    x = inputs.normal(N1 * N2, seed=N1 // 128 + N2)
    plan = paco.Plan(N1, N2, p, b, mixed=True)
    assert plan.has_split, plan.description
    err = oracle.rel_l2(_execute(plan, _dev(x)), oracle.dft(x))
    print(f"split mixed {N1}x{N2} b={b}: rel-L2 {err:.3e}", flush=True)
    assert err <= TOL


def test_split_long_stage_hooks_compose_to_execute():
    N1, N2, p, b = 16384, 64, 4, 4
    x = _dev(inputs.normal(N1 * N2, seed=78))
    plan = paco.Plan(N1, N2, p, b)
    t = _stage(plan, 1, x, paco.PACO_SPLIT)
    z = _stage(plan, 2, t, paco.PACO_SPLIT)
    want = oracle.phase2(oracle.phase1(x.cpu().numpy(), N1, N2, b), N1, N2, b).ravel()
    assert oracle.rel_l2(z.cpu().numpy(), want) <= TOL  # pass 2's output is Phase II's
    plan.execute_stage(3, z.data_ptr(), z.data_ptr(), _stream(), 0)
    torch.cuda.synchronize()
    assert np.array_equal(z.cpu().numpy().view(np.uint64), _execute(plan, x).view(np.uint64))


def test_split_mixed_radix_matches_oracle():
    # N2 = 2048 = 16^2 * 2^3 with b = 16: the redistribution's digit map has a short digit
    N1, N2, p, b = 4096, 2048, 16, 16
    x = inputs.normal(N1 * N2, seed=71)
    plan = paco.Plan(N1, N2, p, b, mixed=True)
    assert plan.has_split, plan.description
    err = oracle.rel_l2(_execute(plan, _dev(x)), oracle.dft(x))
    print(f"split mixed {N1}x{N2} b={b}: rel-L2 {err:.3e}", flush=True)
    assert err <= TOL


def test_split_full_size_sampled():
    # N = 2^24 as 4096 x 4096, p = 64, b = 16, N(0,1) inputs, seed 2, in the
    # split form of Phase I alone; outputs sampled one by one
    N1, N2, p, b = 4096, 4096, 64, 16
    N = N1 * N2
    x = inputs.normal(N, seed=2)
    plan = paco.Plan(N1, N2, p, b, flags=paco.PACO_PLAN_NO_SYM)  # the symmetric form has its own tests
    assert plan.has_split == 1
    y = _execute(plan, _dev(x))
    ks = np.array([0, 1, 15, 16, 255, 256, 4095, 4096, 65537, N // 2, N - 1, 12345678, 9876543])
    ref = oracle.dft_at(x, ks)
    rms = np.sqrt(np.sum(np.abs(x.astype(np.complex128)) ** 2))  # |y| rms by Parseval
    assert np.max(np.abs(y[ks] - ref)) < 1e-5 * rms


def test_pass1_against_oracle_sub_dfts():
    N1, N2, p, b = 4096, 64, 4, 4
    x = inputs.normal(N1 * N2, seed=72)
    plan = paco.Plan(N1, N2, p, b)
    got = _stage(plan, 1, _dev(x), paco.PACO_SPLIT).cpu().numpy()
    want = _split_buffer(x, N1, N2)
    err = oracle.rel_l2(got, want)
    print(f"split pass 1 against the oracle's 16-point DFTs: rel-L2 {err:.3e}", flush=True)
    assert err <= TOL


def test_pass2_against_oracle_phase2():
    # pass 2 on the oracle's split buffer gives Phase II's output Zhat
    N1, N2, p, b = 4096, 64, 4, 4
    x = inputs.normal(N1 * N2, seed=73)
    plan = paco.Plan(N1, N2, p, b)
    got = _stage(plan, 2, _dev(_split_buffer(x, N1, N2)), paco.PACO_SPLIT).cpu().numpy()
    want = oracle.phase2(oracle.phase1(x, N1, N2, b), N1, N2, b).ravel()
    err = oracle.rel_l2(got, want)
    print(f"split pass 2 against the oracle's Phase II: rel-L2 {err:.3e}", flush=True)
    assert err <= TOL


def test_stage_hooks_compose_to_execute():
    N1, N2, p, b = 4096, 256, 16, 16
    x = _dev(inputs.normal(N1 * N2, seed=74))
    plan = paco.Plan(N1, N2, p, b)
    t = _stage(plan, 1, x, paco.PACO_SPLIT)
    z = _stage(plan, 2, t, paco.PACO_SPLIT)
    plan.execute_stage(3, z.data_ptr(), z.data_ptr(), _stream(), 0)
    torch.cuda.synchronize()
    y = _execute(plan, x)
    assert np.array_equal(z.cpu().numpy().view(np.uint64), y.view(np.uint64))


def test_split_in_place_and_deterministic():
    N1, N2, p, b = 4096, 512, 8, 2
    x = inputs.normal(N1 * N2, seed=75)
    plan = paco.Plan(N1, N2, p, b)
    a = _execute(plan, _dev(x))
    buf = _dev(x)
    c = _execute(plan, buf, out=buf)  # in == out
    assert np.array_equal(a.view(np.uint64), c.view(np.uint64))
    assert np.array_equal(a.view(np.uint64), _execute(plan, _dev(x)).view(np.uint64))


def test_knob_keeps_the_packed_form():
    N1, N2, p, b = 4096, 256, 16, 16
    x = inputs.normal(N1 * N2, seed=76)
    packed = _packed_plan(N1, N2, p, b)
    assert not packed.has_split and "split[" not in packed.description
    split = paco.Plan(N1, N2, p, b)
    ref = oracle.dft(x)
    a, c = _execute(packed, _dev(x)), _execute(split, _dev(x))
    assert oracle.rel_l2(a, ref) <= TOL and oracle.rel_l2(c, ref) <= TOL


def test_square_inverse_through_the_split_passes():
    # a square plan's inverse runs on its own passes: pass 1 conjugates on load
    N1 = N2 = 4096
    x = inputs.normal(N1 * N2, seed=77)
    plan = paco.Plan(N1, N2, 64, 16, flags=paco.PACO_PLAN_NO_SYM)
    assert plan.has_split == 1
    yd = _dev(x)
    out = torch.empty_like(yd)
    ws = torch.empty_like(yd)
    plan.execute(yd.data_ptr(), out.data_ptr(), ws.data_ptr(), _stream())
    back = torch.empty_like(yd)
    plan.execute_inverse(out.data_ptr(), back.data_ptr(), ws.data_ptr(), _stream())
    torch.cuda.synchronize()
    err = oracle.rel_l2(back.cpu().numpy(), x)
    print(f"split 2^24 round trip: rel-L2 {err:.3e}", flush=True)
    assert err <= 2 * TOL


def test_which_plans_split():
    assert paco.Plan(4096, 64, 4, 4).has_split == 1
    assert paco.Plan(4096, 4096, 64, 16).has_split == 2                       # the symmetric split form
    assert paco.Plan(4096, 4096, 64, 16, flags=paco.PACO_PLAN_NO_SYM).has_split == 1
    assert not paco.Plan(256, 4096, 4, 16).has_split          # N1 != 4096
    assert not paco.Plan(1024, 4096, 4, 4).has_split
    assert paco.Plan(4096, 8192, 64, 2).has_split == 2                         # non-square symmetric form
    assert paco.Plan(4096, 16384, 64, 4).has_split == 2
    assert paco.Plan(4096, 16384, 64, 4, flags=paco.PACO_PLAN_NO_SYM).has_split == 1
    assert paco.Plan(4096, 16384, 64, 4, paco.PACO_C64_MFMA_FP16X3).has_split != 2  # FP32 only there
    assert paco.Plan(4096, 32768, 64, 2).has_split == 2                        # the wide symmetric form
    # N2 above 2^14 outside the symmetric forms: not measured, the packed form
    assert not paco.Plan(4096, 32768, 64, 2, flags=paco.PACO_PLAN_NO_SYM).has_split
    assert paco.Plan(16384, 64, 4, 4).has_split and paco.Plan(8192, 64, 4, 2).has_split
    # launches paco_execute makes: pass 1, pass 2 and Phase III's passes
    assert paco.Plan(4096, 4096, 64, 16).launches == 3
    assert paco.Plan(16384, 64, 4, 4).launches == 3
    assert paco.Plan(16384, 16384, 256, 4).launches == 3                     # the symmetric split form
    assert paco.Plan(16384, 16384, 256, 4, flags=paco.PACO_PLAN_NO_SYM).launches == 4
    assert paco.Plan(8192, 32768, 128, 2).launches == 3                      # the wide symmetric form
    assert paco.Plan(8192, 32768, 128, 2, flags=paco.PACO_PLAN_NO_SYM).launches == 4  # long-column split
    assert not paco.Plan(16384, 32, 2, 2).has_split           # N2 below 64
    assert not paco.Plan(16384, 64, 4, 4, paco.PACO_C64_MFMA_FP16X3).has_split
    assert not paco.Plan(4096, 256, 16, 16, paco.PACO_C64_MFMA_BF16X3).has_split  # FP32 only
    paper = paco.PACO_PLAN_PAPER_LAYOUT
    assert not paco.Plan(4096, 256, 16, 16, flags=paper).has_split   # the paper's layouts: no fused pipeline
    assert not paco.Plan(16384, 64, 4, 4, flags=paper).has_split      # nor the long-column split form
    assert not paco.Plan(8192, 1 << 11, 8, 2, flags=paper).has_split
    assert not paco.Plan(4096, 4096, 64, 16, flags=paco.PACO_PLAN_GENERIC).has_split


def test_split_flag_errors():
    lib = paco.lib()
    plan = paco.Plan(4096, 64, 4, 4)
    a = torch.empty(4096 * 64, dtype=torch.complex64, device="cuda")
    c = torch.empty_like(a)
    s = _stream()
    for stage, flags in [(3, paco.PACO_SPLIT), (1, paco.PACO_SPLIT | paco.PACO_PACKED),
                         (2, paco.PACO_SPLIT | paco.PACO_NO_TWIDDLE)]:
        assert lib.paco_execute_stage(plan.handle, stage, flags, a.data_ptr(), c.data_ptr(), s) == \
            paco.PACO_ERR_INVALID_ARG
    assert lib.paco_execute_stage(plan.handle, 1, paco.PACO_SPLIT, a.data_ptr(), a.data_ptr(), s) == \
        paco.PACO_ERR_INVALID_ARG                                # out of place only
    other = paco.Plan(256, 4096, 4, 16)
    assert lib.paco_execute_stage(other.handle, 1, paco.PACO_SPLIT, a.data_ptr(), c.data_ptr(), s) == \
        paco.PACO_ERR_UNSUPPORTED
