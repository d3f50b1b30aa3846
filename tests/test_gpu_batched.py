"""The batched form on the GPU, through the C ABI: many transforms of uneven
power-of-two sizes in one persistent launch.

Every transform is checked against the FP64 oracle (rel-L2 <= 1e-6, the same
bound as the single-transform path); transforms of at least 2^13 items are
also compared bit for bit with paco_execute on a single plan with the same
(N1, N2, p, b), since both run the same stage arithmetic and tables.  The full
4096-transform workload (k ~ U{8..20}, seed 6) is checked transform by
transform against the oracle, on every host core.
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
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _run(plan, xd, out=None, ws=None):
    if out is None:
        out = torch.empty(plan.total, dtype=torch.complex64, device="cuda")
    if ws is None:
        ws = torch.empty(plan.total, dtype=torch.complex64, device="cuda")
    plan.execute(xd.data_ptr(), out.data_ptr(), ws.data_ptr(), _stream())
    return out


def _host(t) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _mixed_sizes(seed=11):
    ks = list(range(2, 21)) + [8, 13, 16, 20, 3, 12, 14, 19, 9]
    rng = np.random.default_rng(seed)
    rng.shuffle(ks)
    return [1 << k for k in ks]


def _check_against_oracle(plan, x, y, idx=None, tol=TOL):
    worst = 0.0
    for i in (range(len(plan.sizes)) if idx is None else idx):
        a, b = plan.offsets[i], plan.offsets[i + 1]
        ref = oracle.dft(x[a:b].astype(np.complex128))
        err = oracle.rel_l2(y[a:b], ref)
        assert err <= tol, (i, b - a, plan.transform_plan(i), err)
        worst = max(worst, err)
    return worst


NO_TUNE = paco.PACO_BATCH_NO_TUNE  # default per-size plans, no timing


def test_batched_matches_oracle_default_plans():
    sizes = _mixed_sizes()
    plan = paco.BatchPlan(sizes, flags=NO_TUNE)
    print(plan.description, flush=True)
    x = inputs.batch_inputs(sizes, seed=12)
    y = _host(_run(plan, _dev(x)))
    _check_against_oracle(plan, x, y)
    assert plan.errors() == 0


def test_batched_tuned_cache_roundtrip(tmp_path):
    sizes = [1 << k for k in (5, 12, 13, 17, 20)]
    cache = str(tmp_path / "tune.txt")
    plan = paco.BatchPlan(sizes, tune_cache_path=cache)
    text = open(cache).read().splitlines()
    keys = [ln for ln in text if ln.startswith("key ")]
    assert len(keys) == 1 and "gfx950" in keys[0], keys      # measured on this device
    lines = [ln for ln in text if ln and not ln.startswith("#") and not ln.startswith("key ")]
    assert sorted(int(ln.split()[0]) for ln in lines) == [5, 12, 13, 17, 20]
    choices = [plan.transform_plan(i) for i in range(len(sizes))]
    for (n1, n2, p, b), n in zip(choices, sizes):
        assert n1 * n2 == n and n1 % p == 0 and n2 % p == 0 and p >= 2
        assert b in (2, 4, 16) and round(np.log(n1) / np.log(b)) == np.log(n1) / np.log(b)
    again = paco.BatchPlan(sizes, tune_cache_path=cache)  # every size cached: no tuning
    assert [again.transform_plan(i) for i in range(len(sizes))] == choices
    x = inputs.batch_inputs(sizes, seed=13)
    y = _host(_run(again, _dev(x)))
    _check_against_oracle(again, x, y)
    # a cache measured elsewhere is not trusted: retuned and rewritten with this device's key
    with open(cache, "w") as f:
        f.write("key some-other-device cus=1 format=1\n" + "\n".join(lines) + "\n")
    paco.BatchPlan(sizes[:2], tune_cache_path=cache)
    assert [ln for ln in open(cache).read().splitlines() if ln.startswith("key ")] == keys


def test_batched_bit_identical_to_single_plans():
    sizes = [1 << k for k in (13, 14, 15, 16, 17, 18, 19, 20, 9)]
    plan = paco.BatchPlan(sizes, flags=NO_TUNE)
    x = inputs.batch_inputs(sizes, seed=14)
    xd = _dev(x)
    y = _host(_run(plan, xd))
    for i, n in enumerate(sizes):
        if n < 1 << 13:
            continue
        N1, N2, p, b = plan.transform_plan(i)
        single = paco.Plan(N1, N2, p, b)
        a, c = plan.offsets[i], plan.offsets[i + 1]
        out = torch.empty(n, dtype=torch.complex64, device="cuda")
        ws = torch.empty(n, dtype=torch.complex64, device="cuda")
        single.execute(xd[a:c].data_ptr(), out.data_ptr(), ws.data_ptr(), _stream())
        ys = _host(out)
        assert np.array_equal(ys.view(np.uint64), y[a:c].view(np.uint64)), (n, N1, N2, b)
        single.close()


def test_batched_repeat_inplace_and_rearm():
    sizes = _mixed_sizes(seed=21)
    plan = paco.BatchPlan(sizes, flags=NO_TUNE)
    x = inputs.batch_inputs(sizes, seed=15)
    xd = _dev(x)
    ws = torch.empty(plan.total, dtype=torch.complex64, device="cuda")
    y1 = _host(_run(plan, xd, ws=ws))
    y2 = _host(_run(plan, xd, ws=ws))  # the counters were rearmed by the first launch
    assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64))
    buf = xd.clone()
    plan.execute(buf.data_ptr(), buf.data_ptr(), ws.data_ptr(), _stream())  # in place
    assert np.array_equal(_host(buf).view(np.uint64), y1.view(np.uint64))
    assert plan.errors() == 0


def test_batched_graph_replay():
    sizes = _mixed_sizes(seed=31)
    plan = paco.BatchPlan(sizes, flags=NO_TUNE)
    x = inputs.batch_inputs(sizes, seed=16)
    xd = _dev(x)
    out = torch.empty(plan.total, dtype=torch.complex64, device="cuda")
    ws = torch.empty(plan.total, dtype=torch.complex64, device="cuda")
    eager = _host(_run(plan, xd, out=out, ws=ws)).copy()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.execute(xd.data_ptr(), out.data_ptr(), ws.data_ptr(), s.cuda_stream)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        out.zero_()
        ws.fill_(float(rep + 1))
        torch.cuda.synchronize()
        g.replay()
        got = _host(out)
        assert np.array_equal(got.view(np.uint64), eager.view(np.uint64)), rep
    _check_against_oracle(plan, x, eager)
    assert plan.errors() == 0


def test_batched_argument_errors():
    sizes = [256, 4096, 1 << 14]
    plan = paco.BatchPlan(sizes, flags=NO_TUNE)
    n = plan.total
    a = torch.empty(n + 8, dtype=torch.complex64, device="cuda")
    b = torch.empty(n + 8, dtype=torch.complex64, device="cuda")
    w = torch.empty(n + 8, dtype=torch.complex64, device="cuda")
    h, S = plan.handle, _stream()
    err = paco.PacoError
    with pytest.raises(err) as e:
        paco.paco_execute_batched(h, a.data_ptr(), b.data_ptr(), w.data_ptr(), n * 8 - 8, S)
    assert e.value.status == paco.PACO_ERR_WORKSPACE
    with pytest.raises(err) as e:
        paco.paco_execute_batched(h, a.data_ptr() + 8, b.data_ptr(), w.data_ptr(), n * 8, S)
    assert e.value.status == paco.PACO_ERR_INVALID_ARG
    with pytest.raises(err) as e:
        paco.paco_execute_batched(h, a.data_ptr(), b.data_ptr(), a.data_ptr(), n * 8, S)
    assert e.value.status == paco.PACO_ERR_INVALID_ARG
    with pytest.raises(err) as e:
        paco.paco_execute_batched(h, a.data_ptr(), a.data_ptr() + 16, w.data_ptr(), n * 8, S)
    assert e.value.status == paco.PACO_ERR_INVALID_ARG
    with pytest.raises(err) as e:
        paco.paco_execute_batched(h, 0, b.data_ptr(), w.data_ptr(), n * 8, S)
    assert e.value.status == paco.PACO_ERR_INVALID_ARG
    torch.cuda.synchronize()


def _check_all_threaded(plan, x, y, tol=TOL):
    """Every transform against the FP64 oracle, on the host's cores (the
    oracle's C calls release the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    def one(i):
        a, b = plan.offsets[i], plan.offsets[i + 1]
        return oracle.rel_l2(y[a:b], oracle.dft(x[a:b].astype(np.complex128)))

    with ThreadPoolExecutor(oracle.cpu_threads()) as ex:
        errs = np.array(list(ex.map(one, range(len(plan.sizes)))))
    return errs


def test_batched_full_workload(tmp_path):
    """4096 transforms, k ~ U{8..20} (seed 6): every transform against the
    FP64 oracle."""
    sizes = inputs.batch_sizes(4096, seed=6)
    print(f"total items {int(sizes.sum())}", flush=True)
    plan = paco.BatchPlan(sizes.tolist(), tune_cache_path=str(tmp_path / "tune.txt"))
    print(plan.description, flush=True)
    x = inputs.batch_inputs(sizes, seed=6)
    xd = _dev(x)
    y = _host(_run(plan, xd))
    assert plan.errors() == 0
    del xd
    errs = _check_all_threaded(plan, x, y)
    i = int(errs.argmax())
    print(f"all {len(sizes)} transforms: worst rel-L2 {errs[i]:.3e} (transform {i}, N = {sizes[i]}), "
          f"median {np.median(errs):.3e}", flush=True)
    assert errs.max() <= TOL, (i, float(errs[i]))


def test_batched_fewer_transforms_than_queues():
    # one to three transforms on a device with eight work queues: every
    # queue with work must have a server, and none may be skipped silently
    for sizes in ([1 << 8, 1 << 12, 1 << 16], [1 << 20], [4, 1 << 13]):
        plan = paco.BatchPlan(sizes, flags=NO_TUNE)
        x = inputs.batch_inputs(sizes, seed=29)
        y = _host(_run(plan, _dev(x)))
        assert plan.errors() == 0, plan.description
        _check_against_oracle(plan, x, y)


def test_batched_shared_queue_mode():
    """One work queue served by every XCD (device-coherent stores between
    tasks) gives the same bits as the per-XCD queues."""
    sizes = _mixed_sizes(seed=41)
    x = inputs.batch_inputs(sizes, seed=17)
    xd = _dev(x)
    per_xcd = paco.BatchPlan(sizes, flags=NO_TUNE)
    y1 = _host(_run(per_xcd, xd))
    shared = paco.BatchPlan(sizes, flags=NO_TUNE | paco.PACO_BATCH_ONE_QUEUE)
    assert "shared queue" in shared.description or "1 queues" in shared.description, shared.description
    y2 = _host(_run(shared, xd))
    assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64))
    _check_against_oracle(shared, x, y2)
    assert shared.errors() == 0 and per_xcd.errors() == 0


def test_batched_wait_limit_forced_from_the_host():
    """A poll limit of one makes completion waits give up while their
    producers are still running: the launch must still finish (every wave
    exits), the give-ups must be counted, and a plan with the default limit
    on the same buffers must be correct again afterwards."""
    sizes = [1 << 20] * 4 + [1 << 16] * 16
    x = inputs.batch_inputs(sizes, seed=23)
    xd = _dev(x)
    hasty = paco.BatchPlan(sizes, flags=NO_TUNE, spin_limit=1)
    out = torch.empty(hasty.total, dtype=torch.complex64, device="cuda")
    ws = torch.empty(hasty.total, dtype=torch.complex64, device="cuda")
    for _ in range(3):                         # the count is cumulative; stop once it moved
        _run(hasty, xd, out, ws)
        torch.cuda.synchronize()              # the launch finished
        if hasty.errors():
            break
    gave_up = hasty.errors()
    print(f"waits that gave up at a limit of one poll: {gave_up}", flush=True)
    assert gave_up > 0
    patient = paco.BatchPlan(sizes, flags=NO_TUNE)
    y = _host(_run(patient, xd, out, ws))
    assert patient.errors() == 0
    _check_against_oracle(patient, x, y, idx=[0, 4, 19])
