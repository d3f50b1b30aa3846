"""The symmetric split form on non-square shapes (FP32): N1 = 16 L1 and
N2 = 16 L2 with L1 != L2 in {256, 512, 1024}.  Pass 1 runs the L1-point
children of Phase I over the N2 columns, pass 2 both 16-point children with
the top-level twiddle (w_N^{-v c} split as w_N^{-k c} w_{16 N2}^{-s jc}
w_256^{-s rr}, which holds for any L1, L2 because N / L1 = 16 N2 and
16 N2 / L2 = 256), pass 3 the L2-point children of Phase III over the N1
columns.  The wide form N2 = 2^15 = 32 L2 (L2 = 1024; N1 = 2^12 here, 2^13
in the full-size tests) gives pass 2 a 32-point Phase III child instead
(w_N^{-v c} = w_N^{-k c} w_{16 N2}^{-s jc} w_512^{-s rr}, rr < 32) and
pass 3 the rows 32 t + q0.  Every output against the FP64 oracle, for both
orientations of each pair of sides up to 2^27 items; the inverse (whose
passes are the N2 x N1 plan's); the stage hooks composing to paco_execute
bit for bit; and the plan choice (the split MFMA forms keep their own plan
on these shapes)."""

import numpy as np
import pytest

import oracle
from paper_2609_06449_amd import inputs, paco

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
TOL = 1e-6

# (N1, N2, p, b): b = 2 or 4 so that both sides are powers of it
SHAPES = [(4096, 8192, 64, 2), (8192, 4096, 64, 2), (4096, 16384, 64, 4), (16384, 4096, 64, 4),
          (8192, 16384, 128, 2), (16384, 8192, 128, 2), (4096, 32768, 64, 8)]


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev(x: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(x.astype(np.complex64).ravel())).to("cuda")


def _execute(plan, xd, out=None, fn=None):
    n = xd.numel()
    if out is None:
        out = torch.empty(n, dtype=torch.complex64, device="cuda")
    ws = torch.empty(n, dtype=torch.complex64, device="cuda")
    (fn or plan.execute)(xd.data_ptr(), out.data_ptr(), ws.data_ptr(), _stream())
    torch.cuda.synchronize()
    return out


def _stage(plan, stage, src, dst=None):
    if dst is None:
        dst = torch.empty(src.numel(), dtype=torch.complex64, device="cuda")
    plan.execute_stage(stage, src.data_ptr(), dst.data_ptr(), _stream(), paco.PACO_SPLIT)
    torch.cuda.synchronize()
    return dst


_REF = {}


def _x_and_reference(n: int):
    if n not in _REF:
        _REF.clear()
        x = inputs.normal(n, seed=11)
        print(f"oracle: N = 2^{n.bit_length() - 1} on {oracle.cpu_threads()} host threads", flush=True)
        _REF[n] = (x, oracle.fft_radix2(x, threads=oracle.cpu_threads()))
    return _REF[n]


@pytest.mark.parametrize("N1,N2,p,b", SHAPES)
def test_plan_takes_the_symmetric_form(N1, N2, p, b):
    plan = paco.Plan(N1, N2, p, b)
    r2 = 32 if N2 == 32768 else 16  # the radix of pass 2's Phase III child
    assert plan.description.startswith(f"sym[pass1: phase1 {N1 // 16}-point children"), plan.description
    assert f"phase3 radix-{r2}; pass3: phase3 {N2 // r2}-point children" in plan.description
    assert plan.launches == 3 and plan.has_split == 2
    plan.close()
    for dt in (paco.PACO_C64_MFMA_FP16X3, paco.PACO_C64_MFMA_BF16X6):  # FP32 only on these shapes
        mf = paco.Plan(N1, N2, p, b, dt)
        assert not mf.description.startswith("sym["), mf.description
        mf.close()


@pytest.mark.parametrize("N1,N2,p,b", SHAPES)
def test_every_output_against_oracle(N1, N2, p, b):
    # the oracle of each size is computed once (the shapes come in pairs of
    # the same N)
    x, ref = _x_and_reference(N1 * N2)
    plan = paco.Plan(N1, N2, p, b)
    y = _execute(plan, _dev(x)).cpu().numpy()
    err = oracle.rel_l2(y, ref)
    print(f"symmetric split {N1} x {N2}: rel-L2 vs FP64 oracle over all outputs {err:.3e}", flush=True)
    assert err <= TOL
    plan.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("N1,N2,p,b", [(4096, 8192, 64, 2), (16384, 4096, 64, 4)])
def test_inverse_of_the_oracle_output(N1, N2, p, b):
    x, ref = _x_and_reference(N1 * N2)
    plan = paco.Plan(N1, N2, p, b)
    back = _execute(plan, _dev(ref), fn=plan.execute_inverse).cpu().numpy()
    err = oracle.rel_l2(back, x)
    print(f"symmetric split {N1} x {N2} inverse of the oracle's output: rel-L2 vs x {err:.3e}", flush=True)
    assert err <= TOL
    plan.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("N1,N2,p,b", [(8192, 4096, 64, 2), (4096, 16384, 64, 4), (4096, 32768, 64, 8)])
def test_stage_hooks_compose_to_execute_and_in_place(N1, N2, p, b):
    x = inputs.normal(N1 * N2, seed=12)
    xd = _dev(x)
    plan = paco.Plan(N1, N2, p, b)
    u = _stage(plan, 1, xd)
    w = _stage(plan, 2, u)
    _stage(plan, 3, w, dst=w)
    y = _execute(plan, xd).cpu().numpy()
    assert np.array_equal(w.cpu().numpy().view(np.uint64), y.view(np.uint64))
    buf = xd.clone()
    _execute(plan, buf, out=buf)
    assert np.array_equal(buf.cpu().numpy().view(np.uint64), y.view(np.uint64))
    plan.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("p,b,mixed", [(2, 2, False), (512, 8, False), (32, 16, True)])
def test_wide_output_independent_of_b_and_p(p, b, mixed):
    # the digit reversals of the layouts cancel in the symmetric form, so
    # neither b nor p reaches an address: every (b, p) runs the same passes
    N1, N2 = 4096, 32768
    x = inputs.normal(N1 * N2, seed=13)
    xd = _dev(x)
    base = paco.Plan(N1, N2, 64, 8)
    want = _execute(base, xd).cpu().numpy()
    base.close()
    plan = paco.Plan(N1, N2, p, b, mixed=mixed)
    assert plan.has_split == 2 and plan.launches == 3, plan.description
    got = _execute(plan, xd).cpu().numpy()
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    plan.close()
    torch.cuda.empty_cache()
