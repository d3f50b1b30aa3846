"""The symmetric split form at N1 = N2 = 8192 (L = 512: 512-point children
in passes 1 and 3, each split as radix 16, an LDS exchange, radix 16 and a
radix-2 step across lanes 16 apart) on the GPU, FP32, against the FP64
oracle: every output of the 2^26 transform, each pass on its own against
expected values built from the oracle's DFTs (sampled columns or blocks of
seeded input), the stage hooks composing to paco_execute bit for bit, in
place, the inverse, and independence of b and p.  The split MFMA forms at
the same size (their 32-point stage as two MFMA groups of one wave joined by
a radix-2 step in registers): each pass against the FP32 pass, every output
against the oracle, stage hooks, in place, inverse, exact power-of-two scale
invariance and spikes in every lane (FP16x3).  N1 = N2 = 16384 (L = 1024,
radix 4 across lanes; FP32 only) has every 2^28 output compared with the
oracle in test_gpu_full_size.py."""

import numpy as np
import pytest

import oracle
from paper_2609_06449_amd import inputs, paco

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
TOL = 1e-6
N1 = N2 = 8192
L = N1 // 16
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


def _w(n, e):
    """w_n^{-e} in FP64 from the exact integer exponent."""
    return np.exp(-2j * np.pi * (np.asarray(e, dtype=np.int64) % n) / n)


# the split MFMA forms and their bounds (see test_gpu_mfma.py)
MFMA_FORMS = {
    "fp16x3": (paco.PACO_C64_MFMA_FP16X3, 1e-6),
    "bf16x3": (paco.PACO_C64_MFMA_BF16X3, 3e-5),
    "bf16x6": (paco.PACO_C64_MFMA_BF16X6, 1e-6),
}

_X = {}


def _x_and_reference():
    if not _X:
        x = inputs.normal(N, seed=7)
        print(f"oracle: N = 2^26 on {oracle.cpu_threads()} host threads", flush=True)
        _X["x"], _X["y"] = x, oracle.fft_radix2(x, threads=oracle.cpu_threads())
    return _X["x"], _X["y"]


def test_plan_takes_the_symmetric_form():
    plan = paco.Plan(N1, N2, 64, 2)
    assert plan.has_split == 2 and plan.launches == 3, plan.description
    assert plan.description.startswith("sym[pass1: phase1 512-point"), plan.description
    sq = paco.Plan(1 << 14, 1 << 14, 256, 4)
    assert sq.has_split == 2 and sq.launches == 3 and "1024-point" in sq.description, sq.description
    # the split MFMA forms run it at 8192 x 8192 too, not at 16384 x 16384
    for dt, _ in MFMA_FORMS.values():
        mp = paco.Plan(N1, N2, 64, 2, dt)
        assert mp.has_split == 2 and mp.launches == 3, mp.description
        assert paco.Plan(1 << 14, 1 << 14, 256, 4, dt).has_split != 2
    assert paco.Plan(N1, N2, 64, 2, flags=paco.PACO_PLAN_NO_SYM).has_split != 2


def test_full_2p26_output_against_oracle():
    x, ref = _x_and_reference()
    plan = paco.Plan(N1, N2, 64, 2)
    y = _execute(plan, _dev(x)).cpu().numpy()
    err = oracle.rel_l2(y, ref)
    print(f"symmetric split 8192 x 8192: rel-L2 vs FP64 oracle over all 2^26 outputs {err:.3e}", flush=True)
    assert err <= TOL


@pytest.mark.parametrize("p,b,mixed", [(2, 2, False), (128, 8, True), (32, 16, True)])
def test_output_independent_of_b_and_p(p, b, mixed):
    x, _ = _x_and_reference()
    xd = _dev(x)
    base = _execute(paco.Plan(N1, N2, 64, 2), xd).cpu().numpy()
    plan = paco.Plan(N1, N2, p, b, mixed=mixed)
    assert plan.has_split == 2
    got = _execute(plan, xd).cpu().numpy()
    assert np.array_equal(got.view(np.uint64), base.view(np.uint64))


def _u_from_workspace(ws):
    """U[c][r][k], k < L, from the layout ((k >> 4) N2 + c) 256 + 16 r + (k & 15)."""
    return ws.reshape(L // 16, N2, 16, 16).transpose(1, 2, 0, 3).reshape(N2, 16, L)


def _u_to_workspace(U):
    return np.ascontiguousarray(U.reshape(N2, 16, L // 16, 16).transpose(2, 0, 1, 3)).ravel()


def test_workspace_layout_helpers_are_inverse():
    U = np.arange(N, dtype=np.float64).reshape(N2, 16, L)
    ws = _u_to_workspace(U)
    for c, r, k in ((5, 7, 3), (8191, 15, 511), (100, 0, 300)):
        assert ws[((k >> 4) * N2 + c) * 256 + 16 * r + (k & 15)] == U[c, r, k]
    assert np.array_equal(_u_from_workspace(ws), U)


def test_pass1_against_oracle_sub_dfts():
    # U[c][r][k] = w_8192^{-k r} DFT_512(X[16 j + r, c] over j)[k]
    x = inputs.normal(N, seed=71)
    plan = paco.Plan(N1, N2, 64, 2)
    got = _u_from_workspace(_stage(plan, 1, _dev(x)).cpu().numpy())
    X = x.astype(np.complex128).reshape(N1, N2)
    k = np.arange(L)
    for c in (0, 1, 15, 16, 511, 4000, 8191):
        want = np.empty((16, L), dtype=np.complex128)
        for r in range(16):
            want[r] = oracle.dft(X[r::16, c]) * _w(N1, k * r)
        assert oracle.rel_l2(got[c], want) <= TOL, c


def test_pass2_against_definition_on_seeded_input():
    # A[k + L s, c] = sum_r w_16^{-s r} U[c][r][k], Z[v, c] = A[v, c] w_N^{-v c},
    # W[v][jc][q0] = w_N2^{-q0 jc} sum_rr Z[v, jc + L rr] w_16^{-q0 rr} at out[(16 jc + q0) N1 + v]
    U = inputs.normal(N, seed=72)
    plan = paco.Plan(N1, N2, 64, 2)
    got = _stage(plan, 2, _dev(_u_to_workspace(U))).cpu().numpy().reshape(N2, N1)
    U3 = U.astype(np.complex128).reshape(N2, 16, L)  # [c, r, k]
    v = np.arange(N1)
    F16 = np.array([oracle.dft(e) for e in np.eye(16, dtype=np.complex128)]).T  # the oracle's 16-point DFT matrix
    for jc in (0, 1, 300, 511):
        cs = jc + L * np.arange(16)
        A = np.empty((16, N1), dtype=np.complex128)   # [rr, v], v = k + L s
        for i, c in enumerate(cs):
            A[i] = (F16 @ U3[c]).ravel()                  # [s, k] -> v = k + L s
            A[i] *= _w(N, v * c)
        W = F16 @ A                                        # [q0, v]
        W *= _w(N2, np.arange(16) * jc)[:, None]
        assert oracle.rel_l2(got[16 * jc:16 * jc + 16], W) <= TOL, jc


def test_pass3_against_oracle_on_seeded_input():
    # Y[q0 + 16 q, v] = DFT_512(rows 16 jc + q0 of column v over jc)[q]
    Wb = inputs.normal(N, seed=73)
    plan = paco.Plan(N1, N2, 64, 2)
    got = _stage(plan, 3, _dev(Wb)).cpu().numpy().reshape(N2, N1)
    W2 = Wb.astype(np.complex128).reshape(N2, N1)
    for v in (0, 1, 17, 4096, 8191):
        for q0 in range(16):
            assert oracle.rel_l2(got[q0::16, v], oracle.dft(W2[q0::16, v])) <= TOL, (v, q0)


def test_stage_hooks_compose_to_execute_in_place_and_inverse():
    x, ref = _x_and_reference()
    xd = _dev(x)
    plan = paco.Plan(N1, N2, 64, 2)
    u = _stage(plan, 1, xd)
    w = _stage(plan, 2, u)
    del u
    _stage(plan, 3, w, dst=w)
    y = _execute(plan, xd).cpu().numpy()
    assert np.array_equal(w.cpu().numpy().view(np.uint64), y.view(np.uint64))
    del w
    buf = xd.clone()
    _execute(plan, buf, out=buf)
    assert np.array_equal(buf.cpu().numpy().view(np.uint64), y.view(np.uint64))
    del buf
    back = _execute(plan, _dev(ref), fn=plan.execute_inverse).cpu().numpy()
    err = oracle.rel_l2(back, x)
    print(f"symmetric split 8192 x 8192 inverse: rel-L2 vs x {err:.3e}", flush=True)
    assert err <= TOL


@pytest.mark.parametrize("form", sorted(MFMA_FORMS))
def test_mfma_passes_against_the_fp32_passes(form):
    dt, tol = MFMA_FORMS[form]
    fp32 = paco.Plan(N1, N2, 64, 2)
    mf = paco.Plan(N1, N2, 64, 2, dt)
    for stage, seed in ((1, 75), (2, 76), (3, 77)):
        src = _dev(inputs.loguniform(N, seed=seed))
        a = _stage(fp32, stage, src).cpu().numpy()
        b = _stage(mf, stage, src).cpu().numpy()
        err = oracle.rel_l2(b, a)
        print(f"{form} 8192 x 8192 pass {stage}: rel-L2 against the FP32 pass {err:.3e}", flush=True)
        assert err <= tol, (stage, err)


@pytest.mark.parametrize("form", sorted(MFMA_FORMS))
def test_mfma_full_output_stage_hooks_and_inverse(form):
    dt, tol = MFMA_FORMS[form]
    x = inputs.loguniform(N, seed=78)
    xd = _dev(x)
    plan = paco.Plan(N1, N2, 64, 2, dt)
    y = _execute(plan, xd).cpu().numpy()
    ref = oracle.fft_radix2(x, threads=oracle.cpu_threads())
    err = oracle.rel_l2(y, ref)
    print(f"{form} 8192 x 8192: rel-L2 vs FP64 oracle over all 2^26 outputs {err:.3e}", flush=True)
    assert err <= tol
    u = _stage(plan, 1, xd)
    w = _stage(plan, 2, u)
    del u
    _stage(plan, 3, w, dst=w)
    assert np.array_equal(w.cpu().numpy().view(np.uint64), y.view(np.uint64))
    del w
    buf = xd.clone()
    _execute(plan, buf, out=buf)
    assert np.array_equal(buf.cpu().numpy().view(np.uint64), y.view(np.uint64))
    del buf
    back = _execute(plan, _dev(ref), fn=plan.execute_inverse).cpu().numpy()
    assert oracle.rel_l2(back, x) <= 2 * tol


@pytest.mark.parametrize("form", sorted(MFMA_FORMS))
def test_mfma_power_of_two_input_scale_passes_through_exactly(form):
    plan = paco.Plan(N1, N2, 64, 2, MFMA_FORMS[form][0])
    x = inputs.loguniform(N, seed=79)
    y = _execute(plan, _dev(x)).cpu().numpy()
    for s in (60, -80):
        ys = _execute(plan, _dev(np.ldexp(x.view(np.float32), s).view(np.complex64))).cpu().numpy()
        assert np.array_equal(ys.view(np.uint64), np.ldexp(y.view(np.float32), s).view(np.uint64)), (form, s)


def test_fp16x3_scale_sees_every_lane():
    # 10^6 spikes over 1e-3 noise: a scale that missed a spike's lane would
    # overflow FP16 (see test_gpu_sym.py)
    dt, tol = MFMA_FORMS["fp16x3"]
    fp32 = paco.Plan(N1, N2, 64, 2)
    mf = paco.Plan(N1, N2, 64, 2, dt)
    rng = np.random.default_rng(80)
    x = (1e-3 * inputs.normal(N, seed=80)).astype(np.complex64)
    pos = rng.choice(N, size=16384, replace=False)
    x[pos] = (1e6 * np.exp(2j * np.pi * rng.random(16384))).astype(np.complex64)
    src = _dev(x)
    for stage in (1, 2, 3):
        a = _stage(fp32, stage, src).cpu().numpy()
        b = _stage(mf, stage, src).cpu().numpy()
        assert np.all(np.isfinite(b.view(np.float32))), stage
        assert oracle.rel_l2(b, a) <= tol, stage
