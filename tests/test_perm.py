"""Pins of the oracle's digit reversal, the middle permutation and the staged
pipeline against the paper's worked example, identities and counts.

* Base-b digit reversal pi_ell (appendix A.1): against an independent bit-group
  formula for b = 2^t, bit reversal for b = 2, the involution property and the
  composition identity of the output-layout proof (appendix A.8).
* The middle permutation (section 3.3): the literal per-processor procedure of
  appendix C.5 reproduces Fig. 1 cell for cell and equals the definition-based
  stage reference, with and without the top-level twiddle; every
  source/destination slab pair moves exactly N/p^2 items (section 4.2).
* Theorem 3: the three stage references composed equal the plain DFT.
"""
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig1_para_co_drp.txt")


def _bitgroup_reverse(i, t, ell):
    # b = 2^t: the ell groups of t bits, read in the opposite order
    out = 0
    for g in range(ell):
        out |= ((i >> (t * g)) & ((1 << t) - 1)) << (t * (ell - 1 - g))
    return out


@pytest.mark.parametrize("b,ell", [(2, 1), (2, 6), (4, 3), (8, 4), (16, 3), (2, 12), (4, 7)])
def test_digit_reverse_bitgroup_formula(b, ell):
    t = b.bit_length() - 1
    n = b ** ell
    idx = range(n) if n <= 4096 else np.random.default_rng(0).integers(0, n, 4096).tolist()
    for i in idx:
        r = oracle.digit_reverse(i, b, ell)
        assert r == _bitgroup_reverse(i, t, ell)
        assert r == oracle.digit_reverse_py(i, b, ell)


def test_digit_reverse_binary_is_bit_reversal():
    for ell in range(1, 11):
        for i in range(2 ** ell):
            assert oracle.digit_reverse(i, 2, ell) == int(format(i, f"0{ell}b")[::-1], 2)


@pytest.mark.parametrize("b,ell", [(3, 4), (5, 3), (10, 3), (16, 2), (4, 5)])
def test_digit_reverse_involution_any_base(b, ell):
    for i in range(b ** ell):
        assert oracle.digit_reverse(oracle.digit_reverse(i, b, ell), b, ell) == i


def test_digit_reverse_decimal_example():
    # a base-10 reading is the easiest to check by eye: 123 -> 321, 120 -> 021
    assert oracle.digit_reverse(123, 10, 3) == 321
    assert oracle.digit_reverse(120, 10, 3) == 21
    assert oracle.digit_reverse(7, 10, 3) == 700


@pytest.mark.parametrize("b,l1,l2", [(2, 3, 4), (4, 2, 3), (16, 1, 2), (8, 2, 2)])
def test_composition_identity(b, l1, l2):
    # pi_ell(a*n2 + c) = pi_l1(a) + pi_l2(c)*n1  (appendix A.8)
    n1, n2 = b ** l1, b ** l2
    for a in range(n1):
        for c in range(n2):
            lhs = oracle.digit_reverse(a * n2 + c, b, l1 + l2)
            rhs = oracle.digit_reverse(a, b, l1) + oracle.digit_reverse(c, b, l2) * n1
            assert lhs == rhs


def test_digit_reverse_rejects_out_of_range():
    with pytest.raises(ValueError):
        oracle.digit_reverse(16, 2, 4)
    with pytest.raises(ValueError):
        oracle.digit_reverse(0, 1, 4)


# ---------------------------------------------------------------------------
# Fig. 1
# ---------------------------------------------------------------------------

def _read_golden():
    stages, cur = {}, None
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                cur = line[1:-1]
                stages[cur] = []
                continue
            row = []
            for cell in line.split():
                ac, owner = cell.split("/")
                a, c = ac.split(",")
                row.append(((int(a, 2), int(c, 2)), int(owner[1:])))
            stages[cur].append(row)
    return stages


def test_fig1_trace_cell_for_cell():
    N1 = N2 = 4
    p, b = 2, 2
    gold = _read_golden()
    labels = [[(a, c) for c in range(N2)] for a in range(N1)]
    trace = {}
    slabs = oracle.slabs_from_matrix(labels, p)
    oracle.para_co_drp(slabs, N1, N2, p, b, twiddle=False, trace=trace)
    trace["initial"] = labels

    def owner(stage, r, col):
        if stage == "received":            # row slabs of N1/p rows
            return r // (N1 // p)
        ncol = len(trace[stage][0])        # column slabs
        return col // (ncol // p)

    for stage in ("initial", "packed", "received", "transposed", "output"):
        got = trace[stage]
        want = gold[stage]
        assert len(got) == len(want)
        for r, (grow, wrow) in enumerate(zip(got, want)):
            for col, (item, (wlabel, wowner)) in enumerate(zip(grow, wrow)):
                assert item == wlabel, (stage, r, col)
                assert owner(stage, r, col) == wowner, (stage, r, col)
    # the figure's highlighted item (01,00) starts on P0 and ends on P1
    out = gold["output"]
    pos = [(u, v) for u in range(N2) for v in range(N1) if out[u][v][0] == (1, 0)]
    assert pos == [(0, 2)] and out[0][2][1] == 1


# ---------------------------------------------------------------------------
# the middle permutation: literal procedure vs definition, balance counts
# ---------------------------------------------------------------------------

SMALL = [(4, 4, 2, 2), (8, 8, 2, 2), (16, 16, 4, 4), (16, 64, 4, 4), (64, 16, 8, 4),
         (64, 64, 4, 4), (16, 256, 16, 16), (27, 9, 3, 3)]


@pytest.mark.parametrize("N1,N2,p,b", SMALL)
def test_procedure_equals_definition(N1, N2, p, b):
    rng = np.random.default_rng(N1 * 1000 + N2)
    ws = rng.standard_normal((N1, N2)) + 1j * rng.standard_normal((N1, N2))
    Y = oracle.para_co_drp(oracle.slabs_from_matrix(ws.tolist(), p), N1, N2, p, b)
    got = np.array(oracle.matrix_from_target_slabs(Y))
    want = oracle.phase2(ws, N1, N2, b, twiddle=True)
    assert got.shape == (N2, N1)
    assert np.max(np.abs(got - want)) < 1e-13
    # bare permutation, exactly
    Yb = oracle.para_co_drp(oracle.slabs_from_matrix(ws.tolist(), p), N1, N2, p, b, twiddle=False)
    assert np.array_equal(np.array(oracle.matrix_from_target_slabs(Yb)),
                          oracle.phase2(ws, N1, N2, b, twiddle=False))


@pytest.mark.parametrize("N1,N2,b", [(16, 16, 4), (64, 64, 4)])
def test_procedure_independent_of_p(N1, N2, b):
    rng = np.random.default_rng(7)
    ws = (rng.standard_normal((N1, N2)) + 1j * rng.standard_normal((N1, N2))).tolist()
    outs = []
    for p in (2, 4, 8, 16):
        if N1 % p or N2 % p:
            continue
        Y = oracle.para_co_drp(oracle.slabs_from_matrix(ws, p), N1, N2, p, b)
        outs.append(np.array(oracle.matrix_from_target_slabs(Y)))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def _balance(N1, N2, p, b):
    """counts[q, q'] = items moving from source slab q to target slab q'.

    Up to 2^24 items the oracle's bare permutation is run on index labels
    (re = a, im = c) and each landed item is attributed from where it landed:
    owner_1 from its output column v, owner_0 from its label's column c.
    Above that, the count is taken over a and c separately (the source owner
    depends on c only, the destination owner on v = pi_{m1}(a) only)."""
    if N1 * N2 <= (1 << 24):
        a = np.arange(N1, dtype=np.float64)[:, None]
        c = np.arange(N2, dtype=np.float64)[None, :]
        z = oracle.phase2(a + 1j * c, N1, N2, b, twiddle=False)      # N2 x N1
        src = (z.imag.astype(np.int64) // (N2 // p)).ravel()
        dst = np.broadcast_to(np.arange(N1) // (N1 // p), (N2, N1)).ravel()
        counts = np.zeros((p, p), dtype=np.int64)
        np.add.at(counts, (src, dst), 1)
        return counts
    m1 = round(np.log(N1) / np.log(b))
    v = np.array([oracle.digit_reverse(a, b, m1) for a in range(N1)])
    src_hist = np.bincount(np.arange(N2) // (N2 // p), minlength=p)
    dst_hist = np.bincount(v // (N1 // p), minlength=p)
    return np.outer(src_hist, dst_hist)


@pytest.mark.parametrize("N1,N2,p,b", [(4, 4, 2, 2), (64, 64, 4, 4), (4096, 4096, 64, 16),
                                       (1 << 14, 1 << 14, 256, 4), (1 << 13, 1 << 15, 128, 2)])
def test_exchange_balance(N1, N2, p, b):
    # section 4.2: every (q,q') pair moves N/p^2 items, N/p stay home,
    # h = N/p (1 - 1/p) per processor, mu = N (1 - 1/p) in total
    N = N1 * N2
    counts = _balance(N1, N2, p, b)
    assert np.all(counts == N // (p * p))
    assert int(np.trace(counts)) == N // p
    h = counts.sum(axis=1) - np.diag(counts)
    assert np.all(h == N // p - N // (p * p))
    assert int(counts.sum() - np.trace(counts)) == N - N // p


def test_fig1_counts():
    counts = _balance(4, 4, 2, 2)
    assert np.all(counts == 4)                                   # N/p^2 = 4 items per pair
    assert int(counts.sum() - np.trace(counts)) == 8             # mu = 8
    assert np.all(counts.sum(axis=1) - np.diag(counts) == 4)     # h = 4


# ---------------------------------------------------------------------------
# Lemma 1 and Theorem 3 on the stage references
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N1,N2,b", [(4, 4, 2), (16, 8, 2), (64, 64, 4), (16, 256, 16),
                                     (256, 16, 16), (64, 512, 8), (27, 9, 3), (4096, 16, 16)])
def test_three_stages_compose_to_dft(N1, N2, b):
    rng = np.random.default_rng(N1 + 7 * N2)
    x = rng.standard_normal(N1 * N2) + 1j * rng.standard_normal(N1 * N2)
    Y = oracle.paco_reference(x, N1, N2, b)
    # factor-swapped output view: Y[k2,k1] = y[k1 + k2*N1], i.e. Y row-major = y
    assert Y.shape == (N2, N1)
    assert oracle.rel_l2(Y.ravel(), oracle.dft(x)) < 1e-12
    assert oracle.rel_l2(Y.ravel(), np.fft.fft(x)) < 1e-12


@pytest.mark.parametrize("N1,N2,b", [(64, 32, 4), (16, 16, 2), (256, 8, 16)])
def test_phase1_output_layout(N1, N2, b):
    # Lemma 1: the Phase-I buffer is P_pi Omega applied per column; checked
    # with numpy's FFT and the independent bit-group reversal
    rng = np.random.default_rng(3)
    x = rng.standard_normal(N1 * N2) + 1j * rng.standard_normal(N1 * N2)
    t = b.bit_length() - 1
    m1 = round(np.log(N1) / np.log(b))
    A = np.fft.fft(x.reshape(N1, N2), axis=0)
    perm = [_bitgroup_reverse(a, t, m1) for a in range(N1)]
    assert np.max(np.abs(oracle.phase1(x, N1, N2, b) - A[perm, :])) < 1e-10
    cols = [0, N2 - 1, 3]
    assert np.max(np.abs(oracle.phase1(x, N1, N2, b, cols=cols) - A[perm][:, cols])) < 1e-10


@pytest.mark.parametrize("N1,N2,b", [(32, 64, 2), (16, 64, 4)])
def test_phase3_input_layout(N1, N2, b):
    # Lemma 1, input layout: reading row u as logical j2 = pi(u) and
    # transforming gives the natural-order DFT of the logical column
    rng = np.random.default_rng(4)
    logical = rng.standard_normal((N2, N1)) + 1j * rng.standard_normal((N2, N1))
    t = b.bit_length() - 1
    m2 = round(np.log(N2) / np.log(b))
    perm = [_bitgroup_reverse(u, t, m2) for u in range(N2)]
    phys = logical[perm, :]                      # physical row u holds logical pi(u)
    want = np.fft.fft(logical, axis=0)
    assert np.max(np.abs(oracle.phase3(phys, N1, N2, b) - want)) < 1e-10


# ---------------------------------------------------------------------------
# Mixed-radix reading: sizes n = b^m * r (1 < r < b) lie outside the paper's
# preconditions (section 5, Limitations); digits (b, ..., b, r) least
# significant first, reversed with the radices reversed
# ---------------------------------------------------------------------------

def test_mixed_digit_reverse_hand_values():
    # n = 8, b = 4: radices (4, 2); i = d0 + 4 d1 maps to d1 + 2 d0
    assert [oracle.digit_reverse_n(i, 4, 8) for i in range(8)] == [0, 2, 4, 6, 1, 3, 5, 7]
    # n = 32, b = 16: radices (16, 2); i = d0 + 16 d1 maps to d1 + 2 d0
    assert [oracle.digit_reverse_n(i, 16, 32) for i in (1, 15, 16, 17, 31)] == [2, 30, 1, 3, 31]
    # n = 30, b = 10 (not a power of two): radices (10, 3); 27 = 7 + 10*2 maps to 2 + 3*7
    assert oracle.digit_reverse_n(27, 10, 30) == 23
    # n = 2^14, b = 16: radices (16, 16, 16, 4); i = 1 maps to 4 * 16^2 = 1024
    assert oracle.digit_reverse_n(1, 16, 1 << 14) == 1024
    assert oracle.digit_reverse_n(1 << 12, 16, 1 << 14) == 1    # the top (radix-4) digit comes first


@pytest.mark.parametrize("b,n", [(4, 8), (16, 32), (16, 64), (16, 1 << 10), (8, 1 << 7), (8, 1 << 13),
                                 (16, 1 << 14), (4, 2), (10, 30), (3, 18)])
def test_mixed_matches_python_digit_lists(b, n):
    rad = oracle.radices(b, n)
    assert int(np.prod(rad)) == n and all(R == b for R in rad[:-1]) and rad[-1] <= b
    got = [oracle.digit_reverse_n(i, b, n) for i in range(n)]
    assert got == [oracle.reverse_with_radices(i, rad) for i in range(n)]
    assert sorted(got) == list(range(n))                       # a permutation
    inv = [oracle.reverse_with_radices(v, rad[::-1]) for v in got]
    assert inv == list(range(n))                               # inverse: the reversed radices


@pytest.mark.parametrize("b,m", [(2, 5), (4, 3), (8, 2), (16, 2), (3, 3)])
def test_mixed_reduces_to_pi_m(b, m):
    n = b ** m
    assert [oracle.digit_reverse_n(i, b, n) for i in range(n)] == [oracle.digit_reverse(i, b, m) for i in range(n)]


def test_mixed_is_not_an_involution():
    # with a short digit the map and its inverse differ: the pipeline must
    # use each where the layouts ask for it (pinned by the composition below)
    n, b = 32, 16
    fwd = [oracle.digit_reverse_n(i, b, n) for i in range(n)]
    assert any(fwd[fwd[i]] != i for i in range(n))


@pytest.mark.parametrize("N1,N2,b", [(8, 32, 16), (32, 8, 4), (128, 64, 8), (2, 8, 4)])
def test_mixed_composition_identity(N1, N2, b):
    # the global index a (+) c = a*N2 + c has the radices of c then those of a;
    # reversing the whole string equals pi_{N2}(c) (+) pi_{N1}(a)
    R = oracle.radices(b, N2) + oracle.radices(b, N1)
    for a in range(N1):
        for c in range(N2):
            want = oracle.digit_reverse_n(c, b, N2) * N1 + oracle.digit_reverse_n(a, b, N1)
            assert oracle.reverse_with_radices(a * N2 + c, R) == want


@pytest.mark.parametrize("N1,N2,b", [(32, 64, 16), (64, 32, 16), (8, 8, 4), (128, 512, 8), (2, 16, 4),
                                     (1024, 32, 16), (30, 9, 10)])
def test_mixed_three_stages_compose_to_dft(N1, N2, b):
    rng = np.random.default_rng(N1 + 3 * N2)
    x = rng.standard_normal(N1 * N2) + 1j * rng.standard_normal(N1 * N2)
    Y = oracle.paco_reference(x, N1, N2, b)
    assert oracle.rel_l2(Y.ravel(), oracle.dft(x)) < 1e-12
    assert oracle.rel_l2(Y.ravel(), np.fft.fft(x)) < 1e-12


@pytest.mark.parametrize("N1,N2,b", [(32, 64, 16), (128, 16, 8)])
def test_mixed_stage_layouts(N1, N2, b):
    rng = np.random.default_rng(5)
    x = rng.standard_normal(N1 * N2) + 1j * rng.standard_normal(N1 * N2)
    p1 = [oracle.reverse_with_radices(a, oracle.radices(b, N1)) for a in range(N1)]
    p2 = [oracle.reverse_with_radices(c, oracle.radices(b, N2)) for c in range(N2)]
    # Phase I: row a holds frequency pi1(a) of each column's DFT
    A = np.fft.fft(x.reshape(N1, N2), axis=0)
    At = oracle.phase1(x, N1, N2, b)
    assert np.max(np.abs(At - A[p1, :])) < 1e-9
    # Phase II without the twiddle: item (a, c) lands at (pi2(c), pi1(a))
    ws = rng.standard_normal((N1, N2)) + 1j * rng.standard_normal((N1, N2))
    Z = oracle.phase2(ws, N1, N2, b, twiddle=False)
    want = np.empty((N2, N1), complex)
    for a in range(N1):
        want[p2, p1[a]] = ws[a, :]
    assert np.array_equal(Z, want)
    # Phase III: physical row pi2(j) holds logical j
    logical = rng.standard_normal((N2, N1)) + 1j * rng.standard_normal((N2, N1))
    phys = np.empty_like(logical)
    phys[p2, :] = logical
    assert np.max(np.abs(oracle.phase3(phys, N1, N2, b) - np.fft.fft(logical, axis=0))) < 1e-9


# ---------------------------------------------------------------------------
# Operator identities of the proof of Theorem 3 (section 3.4), as matrices
# ---------------------------------------------------------------------------

def _perm_matrix(perm):
    # layout operator P_pi: (P z)[i] = z[pi(i)]
    n = len(perm)
    P = np.zeros((n, n))
    P[np.arange(n), perm] = 1.0
    return P


def _omega_exact(n):
    k = np.arange(n)
    return np.exp(-2j * np.pi * ((np.outer(k, k)) % n) / n)


def _swap(n1, n2):
    # Pi_swap: C^{n1} (x) C^{n2} -> C^{n2} (x) C^{n1}, (Pi z)[u, v] = z[v, u]
    S = np.zeros((n1 * n2, n1 * n2))
    for u in range(n2):
        for v in range(n1):
            S[u * n1 + v, v * n2 + u] = 1.0
    return S


@pytest.mark.parametrize("N1,N2,b", [(4, 8, 2), (16, 4, 4), (8, 8, 8), (16, 16, 4), (9, 27, 3)])
def test_middle_permutation_factorisation(N1, N2, b):
    # P_{pi_m} = (P_{pi_m2} (x) I_N1) Pi_swap (P_{pi_m1} (x) I_N2)
    m1, m2 = round(math.log(N1, b)), round(math.log(N2, b))
    N = N1 * N2
    pim = _perm_matrix([oracle.digit_reverse_py(i, b, m1 + m2) for i in range(N)])
    p1 = _perm_matrix([oracle.digit_reverse_py(a, b, m1) for a in range(N1)])
    p2 = _perm_matrix([oracle.digit_reverse_py(c, b, m2) for c in range(N2)])
    rhs = np.kron(p2, np.eye(N1)) @ _swap(N1, N2) @ np.kron(p1, np.eye(N2))
    assert np.array_equal(pim, rhs)


@pytest.mark.parametrize("N1,N2,b", [(4, 8, 2), (16, 4, 4), (8, 8, 8), (9, 27, 3)])
def test_twiddle_conjugation_and_four_step(N1, N2, b):
    m1 = round(math.log(N1, b))
    N = N1 * N2
    P1 = np.kron(_perm_matrix([oracle.digit_reverse_py(a, b, m1) for a in range(N1)]), np.eye(N2))
    k1 = np.repeat(np.arange(N1), N2)
    j2 = np.tile(np.arange(N2), N1)
    Dt = np.diag(np.exp(-2j * np.pi * ((k1 * j2) % N) / N))              # D~_{(k1, j2)} = w_N^{-k1 j2}
    pk = np.repeat([oracle.digit_reverse_py(a, b, m1) for a in range(N1)], N2)
    Dtw = np.diag(np.exp(-2j * np.pi * ((pk * j2) % N) / N))             # w_N^{-pi(a) c} at (a, c)
    assert np.max(np.abs(Dtw - P1 @ Dt @ P1)) < 1e-12
    # the four-step operator (Omega_N2 (x) I) Pi_swap D~ (Omega_N1 (x) I) is the DFT
    # with output (k2, k1) = y[k1 + k2 N1], i.e. Omega_N itself on the flat vectors
    F = np.kron(_omega_exact(N2), np.eye(N1)) @ _swap(N1, N2) @ Dt @ np.kron(_omega_exact(N1), np.eye(N2))
    assert np.max(np.abs(F - _omega_exact(N))) < 1e-9
    # and PACO's composite (B (x) I) P_{pi_m} D_tw (A (x) I), A = P_pi Omega, B = Omega P_pi
    m2 = round(math.log(N2, b))
    pi1 = _perm_matrix([oracle.digit_reverse_py(a, b, m1) for a in range(N1)])
    pi2 = _perm_matrix([oracle.digit_reverse_py(c, b, m2) for c in range(N2)])
    pim = _perm_matrix([oracle.digit_reverse_py(i, b, m1 + m2) for i in range(N)])
    A = np.kron(pi1 @ _omega_exact(N1), np.eye(N2))
    B = np.kron(_omega_exact(N2) @ pi2, np.eye(N1))
    assert np.max(np.abs(B @ pim @ Dtw @ A - _omega_exact(N))) < 1e-9
