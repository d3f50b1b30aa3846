"""The split-precision MFMA forms (dtype PACO_C64_MFMA_*) on the GPU.

The paper's DFT is exact in exact arithmetic and says nothing of 16-bit
matrix arithmetic, so these forms have no bound of their own ("parity
unpinned beyond the FP64 oracle"): each is compared with the FP64 oracle and
held to a bound derived from its operand precision.  An FP32 value split into
16-bit parts keeps about 22 (FP16x3), 16 (BF16x3) or 24 (BF16x6) significant
bits; every radix-16 butterfly then carries a relative error of order 2^-bits
and a transform of 3 to 7 radix-16 stages a few times that in rel-L2:
FP16x3 and BF16x6 are held to the FP32 target 1e-6, BF16x3 to 3e-5.

Inputs follow the precision workload: |x| = 10^U[-4, 4], arg x ~ U[0, 2 pi).
"""
import numpy as np
import pytest

import oracle
from paper_2609_06449_amd import inputs, paco

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

FORMS = {
    "fp16x3": (paco.PACO_C64_MFMA_FP16X3, 1e-6),
    "bf16x3": (paco.PACO_C64_MFMA_BF16X3, 3e-5),
    "bf16x6": (paco.PACO_C64_MFMA_BF16X6, 1e-6),
}


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _run(plan, xd):
    N = plan.N1 * plan.N2
    out = torch.empty(N, dtype=torch.complex64, device="cuda")
    ws = torch.empty(N, dtype=torch.complex64, device="cuda")
    plan.execute(xd.data_ptr(), out.data_ptr(), ws.data_ptr(), _stream())
    torch.cuda.synchronize()
    return out.cpu().numpy()


SHAPES = [(64, 64, 4, 4), (16, 4096, 4, 16), (256, 4096, 16, 16), (512, 1024, 8, 2), (1 << 14, 256, 4, 4),
          (64, 1 << 14, 4, 4)]


@pytest.mark.parametrize("form", sorted(FORMS))
@pytest.mark.parametrize("N1,N2,p,b", SHAPES)
def test_mfma_forms_match_oracle(form, N1, N2, p, b):
    dt, tol = FORMS[form]
    x = inputs.loguniform(N1 * N2, seed=5)
    plan = paco.Plan(N1, N2, p, b, dt)
    assert f"prec={form}" in plan.description, plan.description
    y = _run(plan, torch.from_numpy(x).to("cuda"))
    err = oracle.rel_l2(y, oracle.dft(x.astype(np.complex128)))
    print(f"{form} {N1}x{N2} b={b}: rel-L2 {err:.3e}", flush=True)
    assert err <= tol, err


@pytest.mark.parametrize("form", sorted(FORMS))
@pytest.mark.parametrize("N1,N2,p,b", [(4096, 4096, 64, 16), (4096, 1 << 14, 64, 4)])
def test_mfma_forms_precision_configs(form, N1, N2, p, b):
    """N = 2^24 and 2^26 (4096 x 16384, b = 4: one two-pass local phase)
    against the full FP64 oracle: rel-L2 within the form's bound, and the
    worst single output, normalised by max |y|, within ten times it (the
    split forms' errors are not spread evenly over frequency: the lowest
    frequencies carry more, see the accumulation note in stages.h)."""
    dt, tol = FORMS[form]
    N = N1 * N2
    x = inputs.loguniform(N, seed=5)
    plan = paco.Plan(N1, N2, p, b, dt)
    y = _run(plan, torch.from_numpy(x).to("cuda"))
    ref = oracle.dft(x.astype(np.complex128))
    err = oracle.rel_l2(y, ref)
    worst = float(np.max(np.abs(y - ref)) / np.max(np.abs(ref)))
    print(f"{form} N=2^{int(np.log2(N))}: rel-L2 {err:.3e}, max|err|/max|y| {worst:.3e}", flush=True)
    assert err <= tol, err
    assert worst <= 10 * tol, worst


@pytest.mark.parametrize("form", sorted(FORMS))
@pytest.mark.parametrize("N1,N2,p,b", [(4096, 4096, 64, 16), (256, 1024, 4, 4)])
def test_mfma_fast_and_generic_kernels_agree(form, N1, N2, p, b):
    # the same split arithmetic in the fast and the descriptor-driven kernels
    dt, _ = FORMS[form]
    x = torch.from_numpy(inputs.loguniform(N1 * N2, seed=9)).to("cuda")
    fast = paco.Plan(N1, N2, p, b, dt, flags=paco.PACO_PLAN_PAPER_LAYOUT)
    generic = paco.Plan(N1, N2, p, b, dt, flags=paco.PACO_PLAN_PAPER_LAYOUT | paco.PACO_PLAN_GENERIC)
    assert "(fast)" in fast.description and "(fast)" not in generic.description
    a, g = _run(fast, x), _run(generic, x)
    assert np.array_equal(a.view(np.uint64), g.view(np.uint64))


@pytest.mark.parametrize("N1,N2,p,b", [(8, 8, 2, 2), (4, 8, 2, 2), (2, 2, 2, 2)])
def test_mfma_forms_without_radix16_stage_equal_fp32(N1, N2, p, b):
    # lengths below 16 have no radix-16 butterfly: the FP32 kernels run
    x = torch.from_numpy(inputs.loguniform(N1 * N2, seed=4)).to("cuda")
    ref = _run(paco.Plan(N1, N2, p, b), x)
    for dt, _ in FORMS.values():
        got = _run(paco.Plan(N1, N2, p, b, dt), x)
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


def test_batched_rejects_mfma_forms():
    for dt, _ in FORMS.values():
        assert paco.paco_batch_plan_create_status([256, 4096], dt=dt) == paco.PACO_ERR_UNSUPPORTED
