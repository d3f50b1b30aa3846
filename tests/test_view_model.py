"""The literal view model of the local FFT scheduler (oracle/view_model.py,
appendix A.3-A.8 and appendix B) against Lemma 1, the first oracle's stage
references, the appendix's worked example and its stated bounds."""
import math
import random

import numpy as np
import pytest

import oracle
from oracle import view_model as vm


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


SIZES = [(2, 3, 2), (2, 5, 0), (4, 2, 1), (4, 3, 2), (8, 2, 1), (3, 3, 1), (16, 2, 0), (2, 1, 3), (4, 1, 1)]


@pytest.mark.parametrize("b,mr,mc", SIZES)
def test_output_layout_is_lemma_1(b, mr, mc):
    # theorem app-output-layout: physical row r holds frequency pi(r)
    x = _rand((b ** mr, b ** mc), seed=b + mr)
    got, _ = vm.local_phase(x, b, mr, mc, vm.OUT)
    perm = [oracle.digit_reverse(r, b, mr) for r in range(b ** mr)]
    want = np.fft.fft(x, axis=0)[perm, :]
    assert np.max(np.abs(got - want)) < 1e-9
    if b ** mc > 1 and b & (b - 1) == 0:        # the same buffer as the stage reference
        assert np.max(np.abs(got - oracle.phase1(x.ravel(), b ** mr, b ** mc, b))) < 1e-9


@pytest.mark.parametrize("b,mr,mc", SIZES)
def test_input_layout_gives_natural_order(b, mr, mc):
    # theorem app-input-layout: physical row u holds logical pi(u), output natural
    logical = _rand((b ** mr, b ** mc), seed=3 * b + mr)
    perm = [oracle.digit_reverse(u, b, mr) for u in range(b ** mr)]
    got, _ = vm.local_phase(logical[perm, :], b, mr, mc, vm.IN)
    assert np.max(np.abs(got - np.fft.fft(logical, axis=0))) < 1e-9


@pytest.mark.parametrize("N1,N2,b", [(16, 8, 2), (64, 16, 4), (16, 64, 4), (64, 64, 8)])
def test_model_local_phases_compose_with_the_middle_stage_to_the_dft(N1, N2, b):
    # Phase I and Phase III by the view model, Phase II by the stage reference
    m1, m2 = round(math.log(N1, b)), round(math.log(N2, b))
    x = _rand(N1 * N2, seed=7)
    ws, _ = vm.local_phase(x.reshape(N1, N2), b, m1, m2, vm.OUT)
    z = oracle.phase2(ws.ravel(), N1, N2, b)
    Y, _ = vm.local_phase(z, b, m2, m1, vm.IN)
    assert oracle.rel_l2(Y.ravel(), oracle.dft(x)) < 1e-12


@pytest.mark.parametrize("b", [2, 3, 4])
def test_appendix_example_a1_a0_c1_c0(b):
    # physical digit order [a1][a0][c1][c0]; T = [a1, a0], C = [c1, c0]
    root = vm.View(b=b, T=("a1", "a0"), O=(), C=("c1", "c0"), F=(),
                   P=(("a1", 3), ("a0", 2), ("c1", 1), ("c0", 0)))
    st = vm.co_batched_fft(root, _rand(b ** 4, seed=b).astype(complex), 4)
    seen = {(v.T, v.O, v.C, tuple(sorted(v.F, key=str))) for v in st.views}
    for d in range(b):
        # the contiguous-field split fixes c1 = d first (s = b^2 >= n = b^2, O empty)
        assert (("a1", "a0"), (), ("c0",), (("c1", d),)) in seen
        # the transform split [a1] (+) [a0]: the first child's outer field is [a0]
        assert (("a1",), ("a0",), ("c0",), (("c1", d),)) in seen
        # the second child: transform field [a0], outer field [A1] in a1's slot
        assert (("a0",), (("A", "a1"),), ("c0",), (("c1", d),)) in seen
        for e in range(b):
            # the batch split fixes A1 = e: T = [a0], O = {}, C = [c0], F = {c1: d, A1: e}
            key = (("a0",), (), ("c0",), tuple(sorted(((("A", "a1"), e), ("c1", d)), key=str)))
            assert key in seen
    # at that view, varying c0 traverses a contiguous run although the
    # fixed slots (c1 and the former a1) are not adjacent
    v = next(v for v in st.views if v.T == ("a0",) and not v.O and len(v.F) == 2)
    A = v.addr()
    assert np.array_equal(A[:, :, :] - A[:, :, :1], np.broadcast_to(np.arange(b), A.shape))
    assert dict(v.P)[("A", "a1")] == 3


def _random_ops(V, D, rng, depth):
    # any interleaving of legal operations keeps views admissible (theorem app-view-closure)
    vm.check_admissible(V, D)
    if depth == 0:
        return
    ops = []
    if V.O:
        ops.append("outer")
    if not V.O and V.C:
        ops.append("contig")
    if len(V.T) >= 2:
        ops.append("transform")
    if not ops:
        return
    op = rng.choice(ops)
    parent = np.sort(V.addr().ravel())
    if op == "outer":
        d = rng.choice(V.O)
        kids = [vm.outer_batch_child(V, d, r) for r in range(V.b)]
    elif op == "contig":
        kids = [vm.contiguous_child(V, r) for r in range(V.b)]
    else:
        cut = rng.randrange(1, len(V.T))            # any split point, not only the balanced one
        T1, T2 = V.T[:cut], V.T[cut:]
        VI = vm.first_transform_child(V, T1, T2)
        A, Vr = vm.relabel_output(V, T1)
        VII = vm.second_transform_child(Vr, T2, A)
        for k in (VI, VII):                           # each group reindexes the whole working set
            assert k.mass == V.mass and np.array_equal(np.sort(k.addr().ravel()), parent)
        # the relabelled output field keeps T1's slots
        assert [dict(Vr.P)[a] for a in A] == [dict(V.P)[t] for t in T1]
        kids = [VI, VII]
        for k in kids:
            _random_ops(k, D, rng, depth - 1)
        return
    got = np.sort(np.concatenate([k.addr().ravel() for k in kids]))
    assert np.array_equal(got, parent)                # batch children partition the parent
    for k in kids:
        assert k.mass * V.b == V.mass
        _random_ops(k, D, rng, depth - 1)


@pytest.mark.parametrize("seed", range(6))
def test_closure_under_random_interleavings(seed):
    rng = random.Random(seed)
    b = rng.choice([2, 3, 4])
    mr, mc = rng.randint(1, 4), rng.randint(0, 3)
    _random_ops(vm.matrix_view(b, mr, mc, vm.OUT), mr + mc, rng, depth=6)


@pytest.mark.parametrize("b,mr,mc", [(2, 6, 0), (2, 8, 2), (4, 4, 0), (2, 5, 5), (3, 4, 2), (2, 9, 1)])
def test_split_counts_and_work(b, mr, mc):
    x = _rand((b ** mr, b ** mc), seed=1)
    _, st = vm.local_phase(x, b, mr, mc, vm.OUT, check=False)
    n, s = b ** mr, b ** mc
    # lemma B-depth: O(1 + log log_b n) transform splits (balanced halving
    # of the mr digits: at most ceil(log2 mr)) and at most log_b(ns) batch splits
    assert st.max_tsplits <= max(0, math.ceil(math.log2(mr)))
    assert st.max_bsplits <= mr + mc
    # proposition B-work: every item is loaded by exactly one leaf per radix-b
    # level, mr levels in all, always in place
    counts = np.bincount(np.concatenate(st.written), minlength=n * s)
    assert np.all(counts == mr)


def test_views_are_runs_of_the_contiguous_field():
    # lemma app-active-runs: a view of s transforms of length n is ns/c runs of length c
    _, st = vm.local_phase(_rand((16, 8), seed=2), 2, 4, 3, vm.OUT)
    for v in st.views:
        A = v.addr().reshape(-1, v.c)
        assert A.shape[0] == v.mass // v.c
        assert np.array_equal(A - A[:, :1], np.broadcast_to(np.arange(v.c), A.shape))
