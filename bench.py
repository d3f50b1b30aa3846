"""Benchmark of the PACO hot path on one MI355X.

One step = one complete transform (Phase I LocalFFT -> Phase II fused
permutation -> Phase III LocalFFT) of the N = 2^24 complex64 workload
(N1 = N2 = 4096, p = 64 slabs, b = 16, N(0,1) inputs, seed 2) through the C
ABI, in the plan's default (symmetric split) form: three HBM passes, the
16-point children of both local phases in the middle one.  Inputs are
resident in HBM before the timed region.  Prints one JSON line: GFLOP/s =
5 N log2 N / t, plus the dominant kernel's roofline (HIP events on the stream
the kernels run on; phase_us times passes 1, 2 and 3 one launch each) and the
CPU oracle baseline (one thread and all host cores, with the core count and
CPU model).  Cold figures: the same transform with the 256 MB MALL flushed
before each one, by reading a 1 GiB buffer (cold_*), and by writing it
(cold_dirty_*: the transform also pays for writing back 256 MB of the
flush's dirty lines).

Further fields of the same line (each leg can be skipped by a flag):
  two_pass   the two-HBM-pass form of the same transform (an ablation,
             reported beside the three-pass value, never as it)
  batched    4096 transforms, N_i = 2^k, k ~ U{8..20}, in one persistent
             launch replayed from a graph, against a loop of single calls
  large      N = 2^28 in two shapes, with their literal (mixed-radix) bases
             and with the largest bases of which both sizes are powers; each
             complete output's rel-L2 against the FP64 oracle
  precision  FP32 and the split MFMA forms at 2^24 and 2^26 on log-uniform
             inputs, with their rel-L2 and worst-output errors vs FP64; the
             forms take turns in 5 rounds of timed launches, median round
--calibrate-copy adds the device copy that scales rocprofv3's FETCH_SIZE /
WRITE_SIZE counters; --traffic-from turns two such counter files into
profiles/traffic_2p24_4096x4096.json (the roofline's traffic field).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "FFT GFLOP/s (5N·log2N/t) + % HBM roofline, N=2^24 c64; MFMA-split vs FP32"
WORKLOAD = dict(name="2^24 as 4096 x 4096", N1=4096, N2=4096, p=64, b=16, gen="normal", seed=2)
KERNEL_SOURCES = ["paper_2609_06449_amd/csrc/" + f for f in ("local_fft.hip", "middle.hip", "stages.h", "middle_dev.h",
                                                                  "paco_internal.h", "split.hip", "sym.hip", "addr.h")]


class HipEvents:
    """Timing events of the HIP runtime the library runs on, recorded on the
    stream the kernels are launched on.  Created with hipEventDisableSystemFence:
    a default event's system-scope release writes back and invalidates the
    caches at every record, which lengthened each phase that followed one
    by several microseconds against the kernel trace (HIP accepts one
    release-scope flag per event)."""

    FLAGS = 0x20000000  # hipEventDisableSystemFence

    def __init__(self):
        import ctypes

        path = None
        with open("/proc/self/maps") as f:  # the copy torch loaded (one HIP runtime per process)
            for line in f:
                if "libamdhip64" in line:
                    path = line.split()[-1]
                    break
        self.ct = ctypes
        self.hip = ctypes.CDLL(path or "libamdhip64.so")
        self.hip.hipEventCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
        self.hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.events = []

    def new(self):
        e = self.ct.c_void_p()
        rc = self.hip.hipEventCreateWithFlags(self.ct.byref(e), self.FLAGS)
        if rc != 0:
            raise RuntimeError(f"hipEventCreateWithFlags failed ({rc})")
        self.events.append(e)
        return e

    def record(self, e, stream: int):
        rc = self.hip.hipEventRecord(e, self.ct.c_void_p(stream))
        if rc != 0:
            raise RuntimeError(f"hipEventRecord failed ({rc})")

    def ms(self, a, b) -> float:
        t = self.ct.c_float()
        rc = self.hip.hipEventElapsedTime(self.ct.byref(t), a, b)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return t.value

    def close(self):
        for e in self.events:
            self.hip.hipEventDestroy(e)
        self.events = []


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


TRAFFIC_PATH = os.path.join(ROOT, "profiles", "traffic_2p24_4096x4096.json")
# the passes of the default plan of the 2^24 workload, as rocprofv3 names their kernels
SYM_KERNELS = ["pass1 sym_first_kernel<true>", "pass2 sym_middle_kernel<8,8>", "pass3 sym_last_kernel"]
COPY_BYTES = 1 << 28  # the --calibrate-copy device-to-device copy


def short_kernel_name(name: str) -> str:
    """'void paco::(anonymous namespace)::k<12, 1>(paco::P)' -> 'k<12,1>'."""
    name = name.split("(paco::")[0].replace("(anonymous namespace)::", "")
    name = name.replace("void ", "").replace("paco::", "").replace(" ", "")
    return name


def load_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources."""
    try:
        with open(TRAFFIC_PATH) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


def traffic_from(fetch_csv: str, write_csv: str):
    """Turns two `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of
    `bench.py --calibrate-copy` (csv output) into HBM bytes per launch.  Each
    counter (KiB per dispatch) is scaled by what it reads for the 256 MiB
    device-to-device copy: the largest-grid copyBuffer dispatch."""
    import csv

    def per_kernel(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"]]
        gmax = max(int(r["Grid_Size"]) for r in copies)
        cal = [float(r["Counter_Value"]) * 1024 for r in copies if int(r["Grid_Size"]) == gmax]
        scale = COPY_BYTES / (sum(cal) / len(cal))
        acc = {}
        for r in rows:
            if "paco::" in r["Kernel_Name"]:
                acc.setdefault(short_kernel_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]) * 1024)
        return scale, {k: sum(v) / len(v) for k, v in acc.items()}

    fs, fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    ws, write = per_kernel(write_csv, "WRITE_SIZE")
    kernels = {}
    for k in sorted(set(fetch) & set(write)):
        kernels[k] = dict(fetch_bytes=round(fetch[k] * fs), write_bytes=round(write[k] * ws),
                          hbm_bytes_per_launch=round(fetch[k] * fs + write[k] * ws))
    rec = dict(kernel_hash=kernel_hash(), workload=WORKLOAD, fetch_scale=round(fs, 4), write_scale=round(ws, 4),
               copy_bytes=COPY_BYTES, kernels=kernels)
    with open(TRAFFIC_PATH, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec, indent=1))


def cpu_baseline(x, N: int, budget_s: float):
    """The FP64 oracle (recursive radix-2) on whole N-point transforms of the
    same input, on one host thread and on all of the host's cores (the same
    recursion with its top levels spread over threads: bit-identical output),
    each repeated (at least 3 times) until about budget_s / 2 of wall time;
    medians reported.  `value` is the all-cores figure."""
    import numpy as np
    import oracle

    xs = x.astype(np.complex128)
    gflop = 5.0 * N * math.log2(N) / 1e9
    threads = oracle.cpu_threads()

    def timed(nthreads):
        times, ref = [], None
        t_all = time.perf_counter()
        while True:
            t0 = time.perf_counter()
            ref = oracle.fft_radix2(xs, threads=nthreads)
            times.append(time.perf_counter() - t0)
            if len(times) >= 3 and (time.perf_counter() - t_all > budget_s / 2 or len(times) >= 20):
                break
        t = sorted(times)[len(times) // 2]
        return ref, dict(value=round(gflop / t, 3), unit="GFLOP/s", threads=nthreads, median_s=round(t, 4),
                         runs=len(times))

    ref, one = timed(1)
    ref_all, many = timed(threads)
    assert np.array_equal(ref.view(np.uint64), ref_all.view(np.uint64)), "threaded oracle differs"
    return ref, dict(value=many["value"], unit="GFLOP/s", cores=threads, kind="oracle",
                     sample=f"full N=2^{int(math.log2(N))} transforms of the bench input, FP64 recursive radix-2: "
                            f"{one['runs']} on one thread (median {one['median_s']:.3f} s), {many['runs']} on "
                            f"{threads} threads (median {many['median_s']:.3f} s); value = all cores",
                     threads_1=one, threads_all=many, nproc=os.cpu_count(), cpu_model=oracle.cpu_model())


def bench_batched(steps: int, warmup: int):
    """The batched form: 4096 transforms, N_i = 2^k_i with k_i ~ U{8..20}
    (seed 6), N(0,1) entries, packed back to back; one persistent launch per
    step, replayed from a captured graph, against a loop of single-transform
    calls with the same per-size plans (eager, and captured in a graph)."""
    import numpy as np
    import torch

    from paper_2609_06449_amd import inputs, paco

    sizes = inputs.batch_sizes(4096, seed=6)
    t0 = time.perf_counter()
    plan = paco.BatchPlan(sizes.tolist())
    tune_s = time.perf_counter() - t0
    x = torch.from_numpy(inputs.batch_inputs(sizes, seed=6)).to("cuda")
    out = torch.empty_like(x)
    ws = torch.empty_like(x)
    flops = float(np.sum(5.0 * sizes * np.log2(sizes)))
    E = int(sizes.sum())

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):
            plan.execute(x.data_ptr(), out.data_ptr(), ws.data_ptr(), s.cuda_stream)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            plan.execute(x.data_ptr(), out.data_ptr(), ws.data_ptr(), s.cuda_stream)
    torch.cuda.synchronize()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    errors = plan.errors()

    # loop of single calls, same per-size plans
    singles = {}
    for i, n in enumerate(sizes.tolist()):
        if n not in singles:
            singles[n] = paco.Plan(*plan.transform_plan(i))
    offs = plan.offsets
    calls = [(singles[n], x.data_ptr() + 8 * offs[i], out.data_ptr() + 8 * offs[i], ws.data_ptr() + 8 * offs[i])
             for i, n in enumerate(sizes.tolist())]

    def loop(stream_handle):
        for pl, a, b, w in calls:
            pl.execute(a, b, w, stream_handle)

    sh = torch.cuda.current_stream().cuda_stream
    loop(sh)
    torch.cuda.synchronize()
    reps = max(1, min(steps, 5))
    t0 = time.perf_counter()
    for _ in range(reps):
        loop(sh)
    torch.cuda.synchronize()
    loop_ms = (time.perf_counter() - t0) * 1e3 / reps
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g2, stream=s):
            loop(s.cuda_stream)
    torch.cuda.synchronize()
    g2.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g2.replay()
    torch.cuda.synchronize()
    loop_graph_ms = (time.perf_counter() - t0) * 1e3 / reps
    rec = dict(workload="4096 complex64 transforms, N_i = 2^k, k ~ U{8..20} (seed 6), N(0,1) entries, "
                        f"{E} items in total, one persistent launch replayed from a graph",
               gflops=round(flops / (ms * 1e-3) / 1e9, 1), ms_per_step=round(ms, 4),
               hbm_frac_3pass=round(48.0 * E / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               loop_single_calls_ms=round(loop_ms, 3), loop_single_calls_graph_ms=round(loop_graph_ms, 3),
               speedup_vs_loop=round(loop_ms / ms, 2), speedup_vs_loop_graph=round(loop_graph_ms / ms, 2),
               plan_create_s=round(tune_s, 2), wait_timeouts=errors, plan=plan.description)
    if errors:  # a wait gave up: the launch completed with unspecified results
        rec.update(valid=False, gflops=None, hbm_frac_3pass=None,
                   note=f"{errors} completion waits hit their poll limit: results unspecified, not a measurement")
    del g, g2, x, out, ws
    for pl in singles.values():
        pl.close()
    plan.close()
    torch.cuda.empty_cache()
    return rec


PRECISION_WORKLOADS = [  # N = 2^24 and 2^26, |x| = 10^U[-4,4], arg x ~ U[0, 2 pi), seed 5
    dict(name="2^24", N1=4096, N2=4096, p=64, b=16),
    dict(name="2^26", N1=1 << 13, N2=1 << 13, p=64, b=2),  # the square shape: the symmetric form, 3 passes
]
FORMS = [(0, "fp32"), (1, "fp16x3"), (2, "bf16x3"), (3, "bf16x6")]


PRECISION_REPEATS = 5


def bench_precision(steps: int, warmup: int):
    """Every arithmetic form on the precision workloads: milliseconds per
    transform (back-to-back launches on one stream, inputs resident).
    Returns the timing record and the outputs (their error against the FP64
    oracle is taken in the CPU-baseline leg)."""
    import numpy as np
    import torch

    from paper_2609_06449_amd import inputs, paco

    rec, outs = {}, {}
    sh = torch.cuda.current_stream().cuda_stream
    for w in PRECISION_WORKLOADS:
        N = w["N1"] * w["N2"]
        x = inputs.loguniform(N, seed=5)
        xd = torch.from_numpy(x).to("cuda")
        out = torch.empty_like(xd)
        ws = torch.empty_like(xd)
        plans = {name: paco.Plan(w["N1"], w["N2"], w["p"], w["b"], dt) for dt, name in FORMS}
        for plan in plans.values():
            for _ in range(warmup):
                plan.execute(xd.data_ptr(), out.data_ptr(), ws.data_ptr(), sh)
        torch.cuda.synchronize()
        # the forms take turns, PRECISION_REPEATS rounds of `steps` launches
        # each, so that a drift of the clock or of the caches hits every form
        # alike; the median round is reported
        runs = {name: [] for name in plans}
        for _ in range(PRECISION_REPEATS):
            for name, plan in plans.items():
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    plan.execute(xd.data_ptr(), out.data_ptr(), ws.data_ptr(), sh)
                torch.cuda.synchronize()
                runs[name].append((time.perf_counter() - t0) * 1e3 / steps)
        for name, plan in plans.items():
            ms = sorted(runs[name])[len(runs[name]) // 2]
            rec.setdefault(name, {})[w["name"]] = dict(
                ms=round(ms, 4), ms_min=round(min(runs[name]), 4),
                gflops=round(5.0 * N * math.log2(N) / (ms * 1e-3) / 1e9, 1),
                hbm_frac_passes=round(16.0 * N * plan.launches / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                launches=plan.launches)
            plan.execute(xd.data_ptr(), out.data_ptr(), ws.data_ptr(), sh)
            torch.cuda.synchronize()
            outs[(name, w["name"])] = out.cpu().numpy()
            plan.close()
        outs[("x", w["name"])] = x
        del xd, out, ws
        torch.cuda.empty_cache()
    return rec, outs


LARGE_WORKLOADS = [  # the full-HBM-scale shapes: N = 2^28 (2 GiB per buffer), N(0,1) inputs
    # literal bases (mixed radix: 2^14 = 16^3 * 4, 2^13 = 8^4 * 2) ...
    dict(name="2^28 square b=16", N1=1 << 14, N2=1 << 14, p=256, b=16, seed=3, mixed=True),
    dict(name="2^28 non-square b=8", N1=1 << 13, N2=1 << 15, p=128, b=8, seed=4, mixed=True),
    # ... and the largest bases of which both sizes are powers
    dict(name="2^28 square b=4", N1=1 << 14, N2=1 << 14, p=256, b=4, seed=3),
    dict(name="2^28 non-square b=2", N1=1 << 13, N2=1 << 15, p=128, b=2, seed=4),
]


def bench_large(steps: int, warmup: int, keep_outputs: bool = True):
    """The N = 2^28 shapes: milliseconds per transform and the fraction of the
    roofline of the HBM passes the plan makes (`launches`: pass 1, pass 2 and
    Phase III's two on-chip passes, 4 per transform) and of the 3-pass one.
    Inputs are the seeded N(0,1) recipes of the tests (seed 3 for the square
    shapes, 4 for the non-square ones).  With keep_outputs, each shape's
    complete output is copied to the host after its timed launches (the
    CPU-baseline leg compares them with the FP64 oracle)."""
    import torch

    from paper_2609_06449_amd import inputs, paco

    rec, outs = {}, {}
    sh = torch.cuda.current_stream().cuda_stream
    xs = {}
    for w in LARGE_WORKLOADS:
        N = w["N1"] * w["N2"]
        if w["seed"] not in xs:
            xs[w["seed"]] = inputs.normal(N, w["seed"])
        xd = torch.from_numpy(xs[w["seed"]]).to("cuda")
        out = torch.empty_like(xd)
        ws = torch.empty_like(xd)
        plan = paco.Plan(w["N1"], w["N2"], w["p"], w["b"], mixed=w.get("mixed", False))
        for _ in range(warmup):
            plan.execute(xd.data_ptr(), out.data_ptr(), ws.data_ptr(), sh)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.execute(xd.data_ptr(), out.data_ptr(), ws.data_ptr(), sh)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        rec[w["name"]] = dict(N1=w["N1"], N2=w["N2"], p=w["p"], b=w["b"], mixed=w.get("mixed", False),
                              ms=round(ms, 4),
                              gflops=round(5.0 * N * math.log2(N) / (ms * 1e-3) / 1e9, 1),
                              hbm_frac_passes=round(16.0 * N * plan.launches / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                              hbm_frac_3pass=round(48.0 * N / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                              launches=plan.launches)
        if keep_outputs:
            outs[w["name"]] = out.cpu().numpy()
        plan.close()
        del xd, out, ws
        torch.cuda.empty_cache()
    return rec, outs, xs


def large_errors(outs, xs):
    """rel-L2 of every 2^28 output against the FP64 oracle (all host cores,
    one oracle run per input)."""
    import oracle

    errs = {}
    for seed, x in xs.items():
        ref = oracle.fft_radix2(x, threads=oracle.cpu_threads())
        for w in LARGE_WORKLOADS:
            if w["seed"] == seed and w["name"] in outs:
                errs[w["name"]] = float(f"{oracle.rel_l2(outs[w['name']], ref):.4e}")
        del ref
    return errs


def precision_errors(outs):
    """rel-L2 and max|err|/max|y| of every form against the FP64 oracle."""
    import numpy as np
    import oracle

    errs = {}
    for w in PRECISION_WORKLOADS:
        ref = oracle.dft(outs[("x", w["name"])].astype(np.complex128))
        for _, name in FORMS:
            y = outs[(name, w["name"])]
            errs.setdefault(name, {})[w["name"]] = dict(
                rel_l2=float(f"{oracle.rel_l2(y, ref):.4e}"),
                max_err_over_max_y=float(f"{np.max(np.abs(y - ref)) / np.max(np.abs(ref)):.4e}"))
    return errs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--skip-cpu-baseline", action="store_true")
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--skip-precision", action="store_true")
    ap.add_argument("--skip-large", action="store_true")
    ap.add_argument("--skip-cold", action="store_true",
                    help="no MALL-flushed launches (profiling runs: every traced launch is then a warm one)")
    ap.add_argument("--skip-two-pass", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run plain 256 MiB device copies (traffic-counter calibration)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM-traffic summary from two rocprofv3 --pmc csv files and exit")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_from(*args.traffic_from)
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of the path is described, not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2609_06449_amd import inputs, paco

    torch.cuda.init()
    dev = torch.device("cuda:0")
    N1, N2, p, b = WORKLOAD["N1"], WORKLOAD["N2"], WORKLOAD["p"], WORKLOAD["b"]
    N = N1 * N2
    x = inputs.make(WORKLOAD["gen"], N, WORKLOAD["seed"])
    xd = torch.from_numpy(x).to(dev)
    out = torch.empty(N, dtype=torch.complex64, device=dev)
    ws = torch.empty(N, dtype=torch.complex64, device=dev)
    plan = paco.Plan(N1, N2, p, b)
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream

    def step():
        plan.execute(xd.data_ptr(), out.data_ptr(), ws.data_ptr(), sh)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # ---- headline: K back-to-back transforms -------------------------------
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    gflops = 5.0 * N * math.log2(N) / (ms_per_step * 1e-3) / 1e9

    # ---- per-phase durations with HIP events on the same stream ------------
    # the same launches paco_execute makes, one phase per call (split form:
    # its pass 1 and pass 2 in place of Phases I and II; symmetric split
    # form: its three passes)
    fused = plan.description.startswith("fused")
    fl = paco.PACO_SPLIT if plan.has_split else (paco.PACO_PACKED if fused else 0)
    fl3 = paco.PACO_SPLIT if plan.has_split == 2 else 0
    hev = HipEvents()
    ev = [[hev.new() for _ in range(4)] for _ in range(args.steps)]
    for i in range(args.steps):
        e = ev[i]
        hev.record(e[0], sh)
        plan.execute_stage(1, xd.data_ptr(), ws.data_ptr(), sh, fl)
        hev.record(e[1], sh)
        plan.execute_stage(2, ws.data_ptr(), out.data_ptr(), sh, fl)
        hev.record(e[2], sh)
        plan.execute_stage(3, out.data_ptr(), out.data_ptr(), sh, fl3)
        hev.record(e[3], sh)
    torch.cuda.synchronize()
    ph = np.array([[hev.ms(ev[i][k], ev[i][k + 1]) for k in range(3)] for i in range(args.steps)])
    ph_us = ph.mean(axis=0) * 1e3

    # ---- cold: the 256 MB MALL flushed before each transform.  The flush
    # reads a 1 GiB scratch buffer, which leaves the MALL holding clean lines
    # of that buffer only: the transform then reads its input from HBM.
    # Writing the buffer instead (the dirty variant, also reported) leaves
    # 256 MB of dirty lines there, whose write-back the transform's first
    # pass then pays for (measured: pass 1 61 -> 87 us at 2^24).
    flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    flush.fill_(1.0)
    sink = torch.empty(1, dtype=torch.float32, device=dev)

    def cold_run(dirty):
        ms = []
        for i in range(0 if args.skip_cold else min(args.steps, 50)):
            if dirty:
                flush.fill_(float(i))
            else:
                sink.copy_(flush.sum().view(1))
            a = torch.cuda.Event(enable_timing=True)
            z = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            step()
            z.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(z))
        return float(np.median(ms)) if ms else None

    cold_ms = cold_run(False)
    cold_dirty_ms = cold_run(True)
    del flush, sink

    y = out.cpu().numpy()  # the three-pass output (out is reused below)

    # ---- two-pass form (Phase III reads the packed buffer, twiddle on load)
    two, y2 = None, None
    if plan.has_two_pass and not args.skip_two_pass:
        def step2():
            plan.execute_two_pass(xd.data_ptr(), out.data_ptr(), ws.data_ptr(), sh)

        for _ in range(args.warmup):
            step2()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step2()
        torch.cuda.synchronize()
        ms2 = (time.perf_counter() - t0) * 1e3 / args.steps
        y2 = out.cpu().numpy()
        ev2 = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
        for i in range(args.steps):
            e = ev2[i]
            e[0].record(stream)
            plan.execute_stage(1, xd.data_ptr(), ws.data_ptr(), sh, paco.PACO_PACKED | paco.PACO_TWO_PASS)
            e[1].record(stream)
            plan.execute_stage(3, ws.data_ptr(), out.data_ptr(), sh, paco.PACO_PACKED)
            e[2].record(stream)
        torch.cuda.synchronize()
        ph2 = np.array([[ev2[i][k].elapsed_time(ev2[i][k + 1]) for k in range(2)] for i in range(args.steps)])
        ph2_us = ph2.mean(axis=0) * 1e3
        p3_gbs = 16.0 * N / (ph2_us[1] * 1e-6) / 1e9
        two = dict(ms_per_step=round(ms2, 5), value=round(5.0 * N * math.log2(N) / (ms2 * 1e-3) / 1e9, 1),
                   unit="GFLOP/s", speedup_vs_3pass=round(ms_per_step / ms2, 3),
                   hbm_frac_2pass=round(32.0 * N / (ms2 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   phase_us=[round(float(v), 2) for v in ph2_us],
                   phase3_roofline=dict(bound="hbm", achieved=round(p3_gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                                        frac=round(p3_gbs / HBM_PEAK_GBS, 4),
                                        traffic=load_traffic("local_fft_fast_kernel<12,3,1,2,32,0>"),
                                        kernel="phase3 local_fft_fast_kernel<12,3,1,2,32,0>",
                                        alg_bytes_per_launch=int(16.0 * N)),
                   note="ablation: two HBM passes (32 B per item) instead of the paper's three; "
                        "not the headline metric")

    if args.calibrate_copy:
        src = torch.empty(1 << 25, dtype=torch.complex64, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1.0)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # the dominant kernel: the slowest of the three phases (each one launch)
    if plan.has_split == 2:  # the kernels of the default plan for this workload
        names = SYM_KERNELS
    elif plan.has_split:
        names = ["pass1 split_first_kernel", "pass2 split_middle_kernel<false>",
                 "phase3 local_fft_fast_kernel<12,1,4,2,32,0>"]
    elif fl:  # the packed form (plan option PACO_PLAN_NO_SPLIT)
        names = ["phase1 local_fft_fast_kernel<12,2,1,2,16,0>", "phase2 middle_packed2_kernel<false,true>",
                 "phase3 local_fft_fast_kernel<12,1,4,2,32,0>"]
    else:
        names = ["phase1 local_fft_fast_kernel<12,0,4,2,16,0>", "phase2 middle_kernel<false,true,true>",
                 "phase3 local_fft_fast_kernel<12,1,4,2,32,0>"]
    dom = int(np.argmax(ph_us))
    alg_bytes = 16.0 * N  # each phase reads and writes N complex64 items once
    achieved = alg_bytes / (ph_us[dom] * 1e-6) / 1e9
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=load_traffic(names[dom].split()[1]),
                    kernel=names[dom], alg_bytes_per_launch=int(alg_bytes))
    # the same figures for every launch of the step
    phase_roofline = []
    for k in range(3):
        gbs = alg_bytes / (ph_us[k] * 1e-6) / 1e9
        phase_roofline.append(dict(kernel=names[k], us=round(float(ph_us[k]), 2), achieved_gbs=round(gbs, 1),
                                   frac=round(gbs / HBM_PEAK_GBS, 4), traffic=load_traffic(names[k].split()[1])))

    rec = dict(metric=METRIC, value=round(gflops, 1), unit="GFLOP/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(ms_per_step, 5), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload="single 1D complex64 DFT, N=2^24 as N1=N2=4096, p=64 slabs, b=16, "
                                    "N(0,1) inputs (seed 2), plain FP32 path",
                           N=N, N1=N1, N2=N2, p=p, b=b, precision="fp32", parallelism="1 GPU, 64 HBM slabs"),
               roofline=roofline,
               hbm_frac_3pass=round(48.0 * N / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               phase_us=[round(float(v), 2) for v in ph_us],
               phase_roofline=phase_roofline,
               cold_ms_per_step=round(cold_ms, 5) if cold_ms else None,
               cold_hbm_frac_3pass=round(48.0 * N / (cold_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if cold_ms else None,
               cold_dirty_ms_per_step=round(cold_dirty_ms, 5) if cold_dirty_ms else None,
               cold_dirty_hbm_frac_3pass=(round(48.0 * N / (cold_dirty_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                          if cold_dirty_ms else None),
               plan=plan.description)
    if two is not None:
        rec["two_pass"] = two

    if not args.skip_batched:
        del xd, out, ws
        torch.cuda.empty_cache()
        rec["batched"] = bench_batched(max(10, args.steps // 10), 3)

    if not args.skip_large:
        if "xd" in locals():
            del xd, out, ws
        torch.cuda.empty_cache()
        rec["large"], large_outs, large_xs = bench_large(max(5, args.steps // 20), 2,
                                                         keep_outputs=not args.skip_cpu_baseline)

    prec_outs = None
    if args.skip_large:
        large_outs, large_xs = {}, {}
    if not args.skip_precision:
        if "xd" in locals():
            del xd, out, ws
        torch.cuda.empty_cache()
        rec["precision"], prec_outs = bench_precision(max(20, args.steps), 3)
        rec["precision"]["workload"] = ("log-uniform |x| = 10^U[-4,4], uniform phase (seed 5); N = 2^24 as 4096 x 4096 "
                                       "(b = 16) and N = 2^26 as 8192 x 8192 (b = 2), both in the symmetric split "
                                       "form; split forms run every radix-16 butterfly on MFMA")

    if not args.skip_cpu_baseline:
        import oracle

        ref, cb = cpu_baseline(x, N, args.cpu_budget)
        rec["cpu_baseline"] = cb
        rec["rel_l2_vs_oracle"] = float(oracle.rel_l2(y, ref))
        if y2 is not None:
            rec["two_pass"]["rel_l2_vs_oracle"] = float(oracle.rel_l2(y2, ref))
        if prec_outs is not None:
            for name, by_w in precision_errors(prec_outs).items():
                for wname, e in by_w.items():
                    rec["precision"][name][wname].update(e)
        for name, e in large_errors(large_outs, large_xs).items():
            rec["large"][name]["rel_l2_vs_oracle"] = e
    else:
        rec["cpu_baseline"] = None
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
