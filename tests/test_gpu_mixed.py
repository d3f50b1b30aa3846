"""Mixed-radix plans (paco_plan_create_mixed) on the GPU: N1, N2 powers of two
that are not powers of b, outside the paper's preconditions (section 5,
Limitations).  The digit reversal reads (b, ..., b, r) and is checked
against the oracle's, whose mixed-radix reading is pinned in test_perm.py:
end to end against the FP64 DFT, stage by stage against the oracle's stage
references (the bare permutation bit for bit), in both layouts, and the
inverse.  The 2^28 shapes with their literal bases b = 16 and b = 8 are
compared output by output in test_gpu_full_size.py."""

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


def _plan(N1, N2, p, b, layout=None, dt=paco.PACO_C64):
    flags = paco.PACO_PLAN_PAPER_LAYOUT if layout == "paper" else 0
    return paco.Plan(N1, N2, p, b, dt, mixed=True, flags=flags)


SHAPES = [(32, 64, 4, 16), (64, 32, 4, 16), (128, 512, 8, 8), (8, 8, 2, 4), (2, 16, 2, 4), (4096, 2048, 16, 16),
          (1 << 13, 16, 16, 8), (16, 1 << 13, 16, 8), (1 << 14, 64, 4, 16), (64, 1 << 14, 4, 16),
          (1 << 13, 1 << 11, 8, 8), (1 << 15, 8, 8, 16)]


@pytest.mark.parametrize("layout", [None, "paper"])
@pytest.mark.parametrize("N1,N2,p,b", SHAPES)
def test_mixed_end_to_end(N1, N2, p, b, layout):
    x = inputs.normal(N1 * N2, seed=N1 + 11 * N2)
    plan = _plan(N1, N2, p, b, layout)
    y = _call(plan.execute, plan, _dev(x)).cpu().numpy()
    err = oracle.rel_l2(y, oracle.dft(x))
    print(f"mixed {N1}x{N2} b={b} {layout or 'default'}: rel-L2 {err:.3e} | {plan.description}", flush=True)
    assert err <= TOL


@pytest.mark.parametrize("N1,N2,p,b", [(32, 64, 4, 16), (128, 512, 8, 8), (1 << 13, 16, 16, 8), (64, 1 << 14, 4, 16)])
def test_mixed_stages_against_oracle(N1, N2, p, b):
    x = inputs.normal(N1 * N2, seed=41)
    plan = _plan(N1, N2, p, b)
    xd = _dev(x)
    s = _stream()
    N = N1 * N2
    s1 = torch.empty(N, dtype=torch.complex64, device="cuda")
    plan.execute_stage(1, xd.data_ptr(), s1.data_ptr(), s)
    torch.cuda.synchronize()
    assert oracle.rel_l2(s1.cpu().numpy().reshape(N1, N2), oracle.phase1(x, N1, N2, b)) <= TOL
    # the bare permutation of a seeded Phase-I buffer, bit for bit
    W = inputs.normal(N, seed=42)
    wd = _dev(W)
    z = torch.empty_like(wd)
    plan.execute_stage(2, wd.data_ptr(), z.data_ptr(), s, paco.PACO_NO_TWIDDLE)
    torch.cuda.synchronize()
    want = oracle.phase2(W, N1, N2, b, twiddle=False).astype(np.complex64).ravel()
    assert np.array_equal(z.cpu().numpy().view(np.uint64), want.view(np.uint64))
    # Phase III on a seeded Zhat
    plan.execute_stage(3, wd.data_ptr(), z.data_ptr(), s)
    torch.cuda.synchronize()
    assert oracle.rel_l2(z.cpu().numpy().reshape(N2, N1), oracle.phase3(W, N1, N2, b)) <= TOL


@pytest.mark.parametrize("N1,N2,p,b", [(32, 64, 4, 16), (1 << 13, 16, 16, 8), (2048, 4096, 16, 16)])
def test_mixed_inverse(N1, N2, p, b):
    y = inputs.normal(N1 * N2, seed=43)
    plan = _plan(N1, N2, p, b)
    x = _call(plan.execute_inverse, plan, _dev(y)).cpu().numpy()
    assert oracle.rel_l2(x, oracle.idft(y)) <= TOL


def test_mixed_two_pass_form():
    N1, N2, p, b = 2048, 1024, 16, 16            # 16^2 * 8, 16^2 * 4
    x = inputs.normal(N1 * N2, seed=44)
    plan = _plan(N1, N2, p, b)
    assert plan.has_two_pass
    y = _call(plan.execute_two_pass, plan, _dev(x)).cpu().numpy()
    assert oracle.rel_l2(y, oracle.dft(x)) <= TOL


def test_mixed_plans_need_the_mixed_entry_point():
    with pytest.raises(paco.PacoError) as e:
        paco.Plan(1 << 14, 1 << 14, 256, 16)
    assert e.value.status == paco.PACO_ERR_NOT_POWER_OF_B
    # with powers of b the two entry points build the same plan: same output bits
    x = _dev(inputs.normal(4096 * 256, seed=45))
    strict = paco.Plan(4096, 256, 16, 16)
    mixed = _plan(4096, 256, 16, 16)
    assert strict.description == mixed.description
    a = _call(strict.execute, strict, x).cpu().numpy()
    c = _call(mixed.execute, mixed, x).cpu().numpy()
    assert np.array_equal(a.view(np.uint64), c.view(np.uint64))


@pytest.mark.parametrize("dt,tol", [(paco.PACO_C64_MFMA_FP16X3, 1e-6), (paco.PACO_C64_MFMA_BF16X3, 3e-5),
                                    (paco.PACO_C64_MFMA_BF16X6, 1e-6)])
@pytest.mark.parametrize("N1,N2,p,b", [(32, 64, 4, 16), (4096, 2048, 16, 16), (1 << 13, 16, 16, 8)])
def test_mixed_split_forms(N1, N2, p, b, dt, tol):
    # the split MFMA butterflies with mixed-radix row maps (generic passes)
    x = inputs.loguniform(N1 * N2, seed=46)
    plan = _plan(N1, N2, p, b, dt=dt)
    y = _call(plan.execute, plan, _dev(x)).cpu().numpy()
    err = oracle.rel_l2(y, oracle.dft(x))
    print(f"mixed {N1}x{N2} b={b} dt={dt}: rel-L2 {err:.3e}", flush=True)
    assert err <= tol
    back = _call(plan.execute_inverse, plan, _dev(y)).cpu().numpy()
    assert oracle.rel_l2(back, x) <= 2 * tol
