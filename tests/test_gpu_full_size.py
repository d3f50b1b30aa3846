"""Complete outputs at full size, compared with the FP64 oracle.

* N = 2^28 (2 GiB per complex64 buffer) in all four shapes the benchmark
  times: 16384 x 16384 with b = 4 and with its literal base b = 16 (mixed
  radix), 8192 x 32768 with b = 2 and with its literal base b = 8 (mixed
  radix); the last also in the long-column split form (PACO_PLAN_NO_SYM).  Every one of the 2^28 outputs is compared with the oracle's
  recursive radix-2 FFT (run on all host cores, bit-identical to its one-thread
  form) at the same rel-L2 bound as up to 2^24 (1e-6: an FP32 FFT's error grows
  like sqrt(log N), sqrt(28/24) ~ 1.08).  The inverse of each shape is then
  run on the oracle's own output (rounded to complex64) and compared with x.
* Phase III over N2 = 2^15 rows (the last local phase of the 8192 x 32768
  shapes) at small N1, forward and inverse, against the full oracle: the
  32768-row pass descriptors pinned at CPU-cheap sizes.

The theorem that PACO computes the DFT (section 3.4) holds for every
admissible shape, so the bound is the same everywhere.
"""
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
    return torch.from_numpy(np.ascontiguousarray(x.astype(np.complex64, copy=False).ravel())).to("cuda")


def _call(fn, plan, xd):
    N = plan.N1 * plan.N2
    out = torch.empty(N, dtype=torch.complex64, device="cuda")
    ws = torch.empty(N, dtype=torch.complex64, device="cuda")
    fn(xd.data_ptr(), out.data_ptr(), ws.data_ptr(), _stream())
    torch.cuda.synchronize()
    del ws
    return out


# one seed's input and oracle output at a time (x 2 GiB + y 4 GiB of host memory)
_CACHE = {}


def _reference(cfg):
    key = (cfg["gen"], cfg["seed"], cfg["N1"] * cfg["N2"])
    if key not in _CACHE:
        _CACHE.clear()
        N = key[2]
        x = inputs.make(cfg["gen"], N, cfg["seed"])
        print(f"oracle: N = 2^{N.bit_length() - 1} on {oracle.cpu_threads()} host threads", flush=True)
        _CACHE[key] = (x, oracle.fft_radix2(x, threads=oracle.cpu_threads()))
    return _CACHE[key]


# (the default plans run the symmetric split form, 8192 x 32768 its wide form;
# the last case keeps the long-column split form, which the other dtypes and
# PACO_PLAN_NO_SYM take, checked at full size)
@pytest.mark.parametrize("name,flags", [("n2p28_16384x16384_b4", 0), ("n2p28_16384x16384_b16", 0),
                                        ("n2p28_8192x32768_b2", 0), ("n2p28_8192x32768_b8", 0),
                                        ("n2p28_8192x32768_b8", paco.PACO_PLAN_NO_SYM)])
def test_2p28_complete_output_against_oracle(name, flags):
    cfg = inputs.CONFIGS[name]
    N1, N2, p, b = cfg["N1"], cfg["N2"], cfg["p"], cfg["b"]
    mixed = paco.paco_plan_validate(N1, N2, p, b) != paco.PACO_OK
    x, ref = _reference(cfg)
    plan = paco.Plan(N1, N2, p, b, mixed=mixed, flags=flags)
    print(f"{name}: {plan.description}", flush=True)
    yd = _call(plan.execute, plan, _dev(x))
    y = yd.cpu().numpy()
    del yd
    err = oracle.rel_l2(y, ref)
    print(f"{name} forward: rel-L2 vs FP64 oracle over all 2^28 outputs = {err:.3e}", flush=True)
    assert err <= TOL
    del y
    back = _call(plan.execute_inverse, plan, _dev(ref)).cpu().numpy()
    err_inv = oracle.rel_l2(back, x)
    print(f"{name} inverse of the oracle's output: rel-L2 vs x = {err_inv:.3e}", flush=True)
    assert err_inv <= TOL
    plan.close()
    torch.cuda.empty_cache()


# (N1, N2, p, b, mixed): Phase III over 2^15 rows split as two on-chip passes
# (b = 2: 2^8 x 2^7; b = 8: 8^3 x 8^2; b = 16 and b = 4: mixed radix with the
# short digit in the first pass)
LONG_N2 = [(16, 1 << 15, 16, 2, False), (64, 1 << 15, 8, 8, False), (32, 1 << 15, 16, 16, True),
           (256, 1 << 15, 16, 4, True), (512, 1 << 15, 64, 8, False)]


@pytest.mark.parametrize("N1,N2,p,b,mixed", LONG_N2)
def test_phase3_over_2p15_rows_forward_and_inverse(N1, N2, p, b, mixed):
    N = N1 * N2
    x = inputs.normal(N, seed=N1 + 15)
    plan = paco.Plan(N1, N2, p, b, mixed=mixed)
    print(f"{N1}x{N2} b={b}: {plan.description}", flush=True)
    y = _call(plan.execute, plan, _dev(x)).cpu().numpy()
    ref = oracle.dft(x)
    err = oracle.rel_l2(y, ref)
    print(f"{N1}x{N2} b={b} forward rel-L2 {err:.3e}", flush=True)
    assert err <= TOL
    back = _call(plan.execute_inverse, plan, _dev(y)).cpu().numpy()
    assert oracle.rel_l2(back, oracle.idft(y)) <= TOL


@pytest.mark.parametrize("N1,N2,p,b,mixed", [(1 << 15, 16, 16, 2, False), (1 << 15, 64, 8, 8, False),
                                              (1 << 15, 32, 16, 16, True)])
def test_inverse_whose_phase3_has_2p15_rows(N1, N2, p, b, mixed):
    # the inverse runs the phases on the swapped factorisation N2 x N1, so
    # its Phase III transforms the 2^15-row columns (with the conjugating,
    # scaling store)
    N = N1 * N2
    y = inputs.normal(N, seed=N2 + 16)
    plan = paco.Plan(N1, N2, p, b, mixed=mixed)
    got = _call(plan.execute_inverse, plan, _dev(y)).cpu().numpy()
    err = oracle.rel_l2(got, oracle.idft(y))
    print(f"inverse {N1}x{N2} b={b}: rel-L2 {err:.3e}", flush=True)
    assert err <= TOL
