"""The symmetric split form on the GPU (FP32, N1 = N2 = 4096): Phase I and
Phase III each split once more by Lemma 1 with a 16-point child, both
children in the redistribution pass (see paco.h, paco_execute).

Checked against the FP64 oracle: every output of the 2^24 transform the
bench times, each pass on its own against expected values built from the
oracle's DFTs (pass 1 on sampled columns, pass 2 on sampled workgroup
blocks of seeded input, pass 3 on sampled columns of seeded input), the
stage hooks composing to paco_execute bit for bit, in place, the inverse,
and independence of b and p (the form's addresses contain neither)."""

import numpy as np
import pytest

import oracle
from paper_2609_06449_amd import inputs, paco

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
TOL = 1e-6
N1 = N2 = 4096
N = N1 * N2


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev(x: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(x.astype(np.complex64).ravel())).to("cuda")


def _execute(plan, xd, out=None, fn=None):
    if out is None:
        out = torch.empty(N, dtype=torch.complex64, device="cuda")
    ws = torch.empty(N, dtype=torch.complex64, device="cuda")
    (fn or plan.execute)(xd.data_ptr(), out.data_ptr(), ws.data_ptr(), _stream())
    torch.cuda.synchronize()
    return out


def _stage(plan, stage, src, dst=None):
    if dst is None:
        dst = torch.empty(N, dtype=torch.complex64, device="cuda")
    plan.execute_stage(stage, src.data_ptr(), dst.data_ptr(), _stream(), paco.PACO_SPLIT)
    torch.cuda.synchronize()
    return dst


# the split MFMA forms and their bounds (see test_gpu_mfma.py)
MFMA_FORMS = {
    "fp16x3": (paco.PACO_C64_MFMA_FP16X3, 1e-6),
    "bf16x3": (paco.PACO_C64_MFMA_BF16X3, 3e-5),
    "bf16x6": (paco.PACO_C64_MFMA_BF16X6, 1e-6),
}


def _w(n, e):
    """w_n^{-e} in FP64 from the exact integer exponent."""
    return np.exp(-2j * np.pi * (np.asarray(e, dtype=np.int64) % n) / n)


_X2 = {}


def _x_and_reference():
    if not _X2:
        x = inputs.normal(N, seed=2)
        _X2["x"], _X2["y"] = x, oracle.fft_radix2(x, threads=oracle.cpu_threads())
    return _X2["x"], _X2["y"]


def test_plan_takes_the_symmetric_form():
    plan = paco.Plan(N1, N2, 64, 16)
    assert plan.has_split == 2 and plan.description.startswith("sym["), plan.description
    assert plan.launches == 3
    for dt in MFMA_FORMS.values():                                 # every dtype
        mp = paco.Plan(N1, N2, 64, 16, dt[0])
        assert mp.has_split == 2 and mp.launches == 3, mp.description
    assert paco.Plan(N1, 2048, 64, 16, mixed=True).has_split != 2  # N1 = N2 = 4096 only
    for fl in (paco.PACO_PLAN_NO_SYM, paco.PACO_PLAN_NO_SPLIT, paco.PACO_PLAN_PAPER_LAYOUT, paco.PACO_PLAN_GENERIC):
        assert paco.Plan(N1, N2, 64, 16, flags=fl).has_split != 2


def test_full_2p24_output_against_oracle():
    # the bench's workload: N = 2^24, p = 64, b = 16, N(0,1) inputs, seed 2
    x, ref = _x_and_reference()
    plan = paco.Plan(N1, N2, 64, 16)
    y = _execute(plan, _dev(x)).cpu().numpy()
    err = oracle.rel_l2(y, ref)
    print(f"symmetric split 2^24: rel-L2 vs FP64 oracle over all outputs {err:.3e}", flush=True)
    assert err <= TOL


@pytest.mark.parametrize("p,b,mixed", [(2, 2, False), (8, 8, False), (64, 64, False), (256, 4, False),
                                       (16, 32, True)])
def test_output_independent_of_b_and_p(p, b, mixed):
    x, _ = _x_and_reference()
    xd = _dev(x)
    base = _execute(paco.Plan(N1, N2, 64, 16), xd).cpu().numpy()
    plan = paco.Plan(N1, N2, p, b, mixed=mixed)
    assert plan.has_split == 2
    got = _execute(plan, xd).cpu().numpy()
    assert np.array_equal(got.view(np.uint64), base.view(np.uint64))


def _u_from_workspace(ws):
    """U[c][r][k] from the workspace layout ((k >> 4) N2 + c) 256 + 16 r + (k & 15)."""
    return ws.reshape(16, N2, 16, 16).transpose(1, 2, 0, 3).reshape(N2, 16, 256)


def _u_to_workspace(U):
    return np.ascontiguousarray(U.reshape(N2, 16, 16, 16).transpose(2, 0, 1, 3)).ravel()


def test_workspace_layout_helpers_are_inverse():
    U = np.arange(N, dtype=np.float64).reshape(N2, 16, 256)
    ws = _u_to_workspace(U)
    assert ws[((3 >> 4) * N2 + 5) * 256 + 16 * 7 + (3 & 15)] == U[5, 7, 3]
    assert ws[((200 >> 4) * N2 + 4095) * 256 + 16 * 15 + (200 & 15)] == U[4095, 15, 200]
    assert np.array_equal(_u_from_workspace(ws), U)


def test_pass1_against_oracle_sub_dfts():
    # U[c][r][k] = w_4096^{-k r} DFT_256(X[16 j + r, c] over j)[k] at
    # ws[((k >> 4) N2 + c) 256 + 16 r + (k & 15)]
    x = inputs.normal(N, seed=81)
    plan = paco.Plan(N1, N2, 64, 16)
    got = _u_from_workspace(_stage(plan, 1, _dev(x)).cpu().numpy())
    X = x.astype(np.complex128).reshape(N1, N2)
    k = np.arange(256)
    for c in (0, 1, 15, 16, 255, 1000, 4095):
        want = np.empty((16, 256), dtype=np.complex128)
        for r in range(16):
            want[r] = oracle.dft(X[r::16, c]) * _w(N1, k * r)
        assert oracle.rel_l2(got[c], want) <= TOL, c


def test_pass2_against_definition_on_seeded_input():
    # on a seeded U: A[k + 256 s, c] = sum_r w_16^{-s r} U[c][r][k],
    # Z[v, c] = A[v, c] w_N^{-v c}, W[v][jc][q0] = w_N2^{-q0 jc} sum_rr
    # Z[v, jc + 256 rr] w_16^{-q0 rr} at out[(16 jc + q0) N1 + v]
    U = inputs.normal(N, seed=82)
    plan = paco.Plan(N1, N2, 64, 16)
    got = _stage(plan, 2, _dev(_u_to_workspace(U))).cpu().numpy().reshape(N2, N1)
    U3 = U.astype(np.complex128).reshape(N2, 16, 256)  # [c, r, k]
    v = np.arange(N1)
    for jc in (0, 1, 100, 255):
        cs = jc + 256 * np.arange(16)
        A = np.empty((16, N1), dtype=np.complex128)   # [rr, v]
        for i, c in enumerate(cs):
            for kk in range(256):
                A[i, kk + 256 * np.arange(16)] = oracle.dft(U3[c, :, kk])
            A[i] *= _w(N, v * c)
        W = np.empty((16, N1), dtype=np.complex128)   # [q0, v]
        for vv in range(N1):
            W[:, vv] = oracle.dft(A[:, vv])
        W *= _w(N2, np.arange(16) * jc)[:, None]
        assert oracle.rel_l2(got[16 * jc:16 * jc + 16], W) <= TOL, jc


def test_pass3_against_oracle_on_seeded_input():
    # Y[q0 + 16 q, v] = DFT_256(rows 16 jc + q0 of column v over jc)[q]
    Wb = inputs.normal(N, seed=83)
    plan = paco.Plan(N1, N2, 64, 16)
    got = _stage(plan, 3, _dev(Wb)).cpu().numpy().reshape(N2, N1)
    W2 = Wb.astype(np.complex128).reshape(N2, N1)
    for v in (0, 1, 17, 2048, 4095):
        for q0 in range(16):
            want = oracle.dft(W2[q0::16, v])
            assert oracle.rel_l2(got[q0::16, v], want) <= TOL, (v, q0)


def test_stage_hooks_compose_to_execute_and_in_place():
    x = _dev(inputs.normal(N, seed=84))
    plan = paco.Plan(N1, N2, 64, 16)
    u = _stage(plan, 1, x)
    w = _stage(plan, 2, u)
    _stage(plan, 3, w, dst=w)                       # pass 3 in place
    y = _execute(plan, x).cpu().numpy()
    assert np.array_equal(w.cpu().numpy().view(np.uint64), y.view(np.uint64))
    buf = x.clone()
    _execute(plan, buf, out=buf)                    # in == out
    assert np.array_equal(buf.cpu().numpy().view(np.uint64), y.view(np.uint64))
    again = _execute(plan, x).cpu().numpy()         # deterministic
    assert np.array_equal(again.view(np.uint64), y.view(np.uint64))


def test_inverse_of_the_oracle_output():
    # the square plan's inverse runs on the same passes (conjugating loads in
    # pass 1, conjugating 1/N stores in pass 3)
    x, ref = _x_and_reference()
    plan = paco.Plan(N1, N2, 64, 16)
    back = _execute(plan, _dev(ref), fn=plan.execute_inverse).cpu().numpy()
    err = oracle.rel_l2(back, x)
    print(f"symmetric split inverse: rel-L2 vs x {err:.3e}", flush=True)
    assert err <= TOL


def test_stage_flag_errors():
    lib = paco.lib()
    plan = paco.Plan(N1, N2, 64, 16)
    buf = torch.empty(N, dtype=torch.complex64, device="cuda")
    s = _stream()
    for stage in (1, 2):  # out of place only
        assert lib.paco_execute_stage(plan.handle, stage, paco.PACO_SPLIT, buf.data_ptr(), buf.data_ptr(), s) == \
            paco.PACO_ERR_INVALID_ARG
    assert lib.paco_execute_stage(plan.handle, 4, paco.PACO_SPLIT, buf.data_ptr(), buf.data_ptr(), s) == \
        paco.PACO_ERR_INVALID_ARG
    old = paco.Plan(N1, N2, 64, 16, flags=paco.PACO_PLAN_NO_SYM)
    out = torch.empty_like(buf)
    assert lib.paco_execute_stage(old.handle, 3, paco.PACO_SPLIT, buf.data_ptr(), out.data_ptr(), s) == \
        paco.PACO_ERR_INVALID_ARG


@pytest.mark.parametrize("form", sorted(MFMA_FORMS))
def test_mfma_passes_against_the_fp32_passes(form):
    # each pass of an MFMA form on the same seeded input as the FP32 pass
    # (whose passes are checked against the oracle above), within the
    # form's bound; log-uniform magnitudes stress the split
    dt, tol = MFMA_FORMS[form]
    fp32 = paco.Plan(N1, N2, 64, 16)
    mf = paco.Plan(N1, N2, 64, 16, dt)
    for stage, seed in ((1, 85), (2, 86), (3, 87)):
        src = _dev(inputs.loguniform(N, seed=seed))
        a = _stage(fp32, stage, src).cpu().numpy()
        b = _stage(mf, stage, src).cpu().numpy()
        err = oracle.rel_l2(b, a)
        print(f"{form} pass {stage}: rel-L2 against the FP32 pass {err:.3e}", flush=True)
        assert err <= tol, (stage, err)


@pytest.mark.parametrize("form", sorted(MFMA_FORMS))
def test_mfma_stage_hooks_compose_in_place_and_inverse(form):
    dt, tol = MFMA_FORMS[form]
    x = inputs.loguniform(N, seed=88)
    xd = _dev(x)
    plan = paco.Plan(N1, N2, 64, 16, dt)
    u = _stage(plan, 1, xd)
    w = _stage(plan, 2, u)
    _stage(plan, 3, w, dst=w)
    y = _execute(plan, xd).cpu().numpy()
    assert np.array_equal(w.cpu().numpy().view(np.uint64), y.view(np.uint64))
    buf = xd.clone()
    _execute(plan, buf, out=buf)
    assert np.array_equal(buf.cpu().numpy().view(np.uint64), y.view(np.uint64))
    ref = oracle.fft_radix2(x, threads=oracle.cpu_threads())
    assert oracle.rel_l2(y, ref) <= tol
    back = _execute(plan, _dev(ref), fn=plan.execute_inverse).cpu().numpy()
    err = oracle.rel_l2(back, x)
    print(f"{form} inverse of the oracle's output: rel-L2 vs x {err:.3e}", flush=True)
    assert err <= 2 * tol


@pytest.mark.parametrize("form", sorted(MFMA_FORMS) + ["fp32"])
def test_power_of_two_input_scale_passes_through_exactly(form):
    # The FP16x3 form scales each tile (passes 1, 3) or wave (pass 2) by a
    # power of two taken from its largest operand; the BF16 forms and FP32
    # need none.  Scaling the input by 2^s must then scale every output by
    # exactly 2^s, bit for bit, as long as nothing leaves FP32's normal range:
    # s = 60 puts |x| near 10^22 (far outside FP16), s = -80 near 10^-28.
    dt = paco.PACO_C64 if form == "fp32" else MFMA_FORMS[form][0]
    plan = paco.Plan(N1, N2, 64, 16, dt)
    x = inputs.loguniform(N, seed=89)
    y = _execute(plan, _dev(x)).cpu().numpy()
    for s in (60, -80):
        xs = np.ldexp(x.view(np.float32), s).view(np.complex64)  # componentwise, exact
        ys = _execute(plan, _dev(xs)).cpu().numpy()
        scaled = np.ldexp(y.view(np.float32), s).view(np.complex64)
        assert np.array_equal(ys.view(np.uint64), scaled.view(np.uint64)), (form, s)
    zero = _execute(plan, _dev(np.zeros(N, np.complex64))).cpu().numpy()
    assert not np.any(zero), form


def test_fp16x3_scale_sees_every_lane():
    # Small noise (|x| ~ 1e-3) with 10^6 spikes at 4096 random positions:
    # a scale that missed the lane of a spike would leave it near 5e8 in
    # FP16 units (FP16 overflows at 65504) and poison the pass with inf.
    # Each pass alone on that input, against the FP32 pass.
    dt, tol = MFMA_FORMS["fp16x3"]
    fp32 = paco.Plan(N1, N2, 64, 16)
    mf = paco.Plan(N1, N2, 64, 16, dt)
    rng = np.random.default_rng(90)
    x = (1e-3 * inputs.normal(N, seed=90)).astype(np.complex64)
    pos = rng.choice(N, size=4096, replace=False)
    x[pos] = (1e6 * np.exp(2j * np.pi * rng.random(4096))).astype(np.complex64)
    src = _dev(x)
    for stage in (1, 2, 3):
        a = _stage(fp32, stage, src).cpu().numpy()
        b = _stage(mf, stage, src).cpu().numpy()
        assert np.all(np.isfinite(b.view(np.float32))), stage
        err = oracle.rel_l2(b, a)
        print(f"fp16x3 pass {stage} on spikes: rel-L2 against the FP32 pass {err:.3e}", flush=True)
        assert err <= tol, (stage, err)
