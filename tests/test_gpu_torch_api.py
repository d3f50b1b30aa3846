"""The torch-tensor convenience layer (allocation and stream plumbing over
the C ABI) against the FP64 oracle: forward, inverse, two-pass, mixed radix,
a split form, one stage and a batch plan."""
import numpy as np
import pytest

import oracle
from paper_2609_06449_amd import inputs, paco

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x.astype(np.complex64))).to("cuda")


def test_fft_ifft_two_pass_mixed_and_split():
    from paper_2609_06449_amd import torch_api as ta
    x = inputs.normal(256 * 1024, seed=61)
    xd = _dev(x)
    ref = oracle.dft(x)
    y = ta.fft(xd, 256, 1024, 8, 4)
    assert oracle.rel_l2(y.cpu().numpy(), ref) <= 1e-6
    assert oracle.rel_l2(ta.fft(xd, 256, 1024, 8, 4, two_pass=True).cpu().numpy(), ref) <= 1e-6
    assert oracle.rel_l2(ta.fft(xd, 256, 1024, 8, 16, mixed=True).cpu().numpy(), ref) <= 1e-6  # 1024 = 16^2 * 4
    assert oracle.rel_l2(ta.fft(xd, 256, 1024, 8, 4, dt=paco.PACO_C64_MFMA_BF16X6).cpu().numpy(), ref) <= 1e-6
    back = ta.ifft(y, 256, 1024, 8, 4)
    assert oracle.rel_l2(back.cpu().numpy(), x) <= 2e-6
    assert ta.get_plan(256, 1024, 8, 4) is ta.get_plan(256, 1024, 8, 4)   # cached
    with pytest.raises(ValueError):
        ta.fft(xd[:-1], 256, 1024, 8, 4)


def test_stage_and_batched():
    from paper_2609_06449_amd import torch_api as ta
    N1, N2, b = 64, 64, 4
    x = inputs.normal(N1 * N2, seed=62)
    s1 = ta.stage(_dev(x), N1, N2, 4, b, 1).cpu().numpy().reshape(N1, N2)
    assert oracle.rel_l2(s1, oracle.phase1(x, N1, N2, b)) <= 1e-6
    sizes = [256, 4096, 1 << 14]
    plan = paco.BatchPlan(sizes)
    xb = inputs.batch_inputs(sizes, seed=63)
    yb = ta.fft_batched(_dev(xb), plan).cpu().numpy()
    for i in range(len(sizes)):
        a, c = plan.offsets[i], plan.offsets[i + 1]
        assert oracle.rel_l2(yb[a:c], oracle.dft(xb[a:c])) <= 1e-6
