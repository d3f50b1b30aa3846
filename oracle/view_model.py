"""Literal CPU model of the view-based cache-oblivious batched local FFT
(paper, appendix A.3-A.8 and appendix B).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the tests use it as a
second, structurally faithful reference for the layout algebra.  It shares
nothing with the GPU library.

What it models:

* ``View``: the tuple (T, O, C, F, P, mode) of appendix A.3.
  - T is the active transform field, O the outer-batch field and C the
    distinguished contiguous field, each an ordered tuple of digit labels,
    most significant first.
  - F holds the fixed labels and their values.
  - P maps each label to its physical base-b digit slot (slot 0 least
    significant).
  - ``addr`` is the address map, eq. app-address-map.
* The three legal view operations of appendix A.4: the outer-batch split,
  the contiguous-field split and the transform split.  The transform split
  renames the first child's field T1 as the output field A afterwards,
  without moving any item.
* ``co_batched_fft``: the scheduler of appendix B (figure cofft).
  - A leaf (n <= b and s <= b) runs natural-order DFTs of length n.
  - s >= n: batch split (an outer-batch digit when one is active, else the
    most significant contiguous digit).
  - Otherwise: a balanced digit-aligned transform split.
  The layout-aware twiddle of eq. app-layout-aware-twiddle,
  w_n^{-pi_{l1}(a) j2}, is not a separate pass: it rides on the second child
  group as a pending factor that the first leaf to load an item applies.
  Input layout (theorem app-input-layout) is the output-layout traversal
  under digit-reversed entrance and exit interpretations: the transform
  field's digit order is reversed in the view, and no data moves.

Instrumentation:
* ``check_admissible``: checks definition app-admissible-view after every
  operation.  Run on every view, it checks theorem app-view-closure
  (closure of admissible views).
* A trace of the views the scheduler visits.
* Counts of transform and batch splits along every root-to-leaf path, for
  lemma B-depth.
* The set of addresses each leaf writes, for theorem app-no-local-transpose.
"""
from __future__ import annotations

import cmath
from dataclasses import dataclass, field, replace

import numpy as np

OUT, IN = "OutputLayout", "InputLayout"


@dataclass(frozen=True)
class View:
    b: int
    T: tuple          # active transform field, most significant label first
    O: tuple          # active outer-batch field (flattened eta), most significant first
    C: tuple          # distinguished contiguous batch field, most significant first
    F: tuple          # fixed labels: ((label, value), ...)
    P: tuple          # ((label, physical slot), ...) for every current label
    mode: str = OUT
    # twiddles still to be applied on first access: (n, A labels, T2 labels)
    pending: tuple = field(default=())

    # ---- parameters (eq. app-view-parameters, eq. B-params) --------------
    @property
    def n(self) -> int:
        return self.b ** len(self.T)

    @property
    def o(self) -> int:
        return self.b ** len(self.O)

    @property
    def c(self) -> int:
        return self.b ** len(self.C)

    @property
    def s(self) -> int:
        return self.o * self.c

    @property
    def mass(self) -> int:
        return self.n * self.s

    def slot(self, label) -> int:
        return dict(self.P)[label]

    def fixed(self) -> dict:
        return dict(self.F)

    # ---- address map (eq. app-address-map) -------------------------------
    def label_values(self):
        """For every label, its digit value on the (tau, eta, chi) grid of
        shape (n, o, c), as an int64 array broadcastable to that grid."""
        b = self.b
        n, o, c = self.n, self.o, self.c
        tau = np.arange(n).reshape(n, 1, 1)
        eta = np.arange(o).reshape(1, o, 1)
        chi = np.arange(c).reshape(1, 1, c)
        vals = {}
        for field_, coord in ((self.T, tau), (self.O, eta), (self.C, chi)):
            L = len(field_)
            for i, lab in enumerate(field_):           # i = 0 is the most significant
                vals[lab] = (coord // b ** (L - 1 - i)) % b
        for lab, v in self.F:
            vals[lab] = np.full((1, 1, 1), v, dtype=np.int64)
        return vals

    def addr(self) -> np.ndarray:
        """Physical address of every view coordinate, shape (n, o, c):
        base_0 (= 0) + sum over fixed, transform and outer labels of
        digit * b^slot, + chi (the contiguous field sits in slots 0..|C|-1)."""
        b = self.b
        vals = self.label_values()
        out = np.zeros((self.n, self.o, self.c), dtype=np.int64)
        for lab in list(self.T) + list(self.O) + [lab for lab, _ in self.F]:
            out = out + vals[lab] * b ** self.slot(lab)
        out = out + np.arange(self.c).reshape(1, 1, self.c)
        return out


# ---------------------------------------------------------------------------
# admissibility (definition app-admissible-view)
# ---------------------------------------------------------------------------

def check_admissible(V: View, D: int) -> None:
    """Raises AssertionError unless V is admissible over D root digit slots."""
    active = list(V.T) + list(V.O) + list(V.C)
    fixed = [lab for lab, _ in V.F]
    labels = active + fixed
    # 1. active and fixed labels partition the root's digit slots
    assert len(set(labels)) == len(labels), "a label appears twice"
    Pm = dict(V.P)
    assert set(labels) == set(Pm), "P must cover exactly the current labels"
    slots = [Pm[lab] for lab in labels]
    # 2. P assigns every label a unique physical slot
    assert sorted(slots) == list(range(D)), "labels must cover each slot once"
    # fixed values are digits
    assert all(0 <= v < V.b for _, v in V.F)
    # 3. the active C digits are the least significant slots 0..|C|-1, in order
    assert [Pm[lab] for lab in V.C] == list(range(len(V.C) - 1, -1, -1)), "C not least-significant contiguous"
    # 4./5. the address map is injective over the view's coordinates
    A = V.addr().ravel()
    assert A.size == V.mass and np.unique(A).size == A.size, "address map not injective"
    assert A.min() >= 0 and A.max() < V.b ** D


# ---------------------------------------------------------------------------
# legal view operations (appendix A.4)
# ---------------------------------------------------------------------------

def outer_batch_child(V: View, d, r: int) -> View:
    assert d in V.O
    return replace(V, O=tuple(x for x in V.O if x != d), F=V.F + ((d, r),))


def contiguous_child(V: View, r: int) -> View:
    assert not V.O and V.C, "contiguous-field split needs O empty"
    d = V.C[0]                       # the most significant active digit of C
    return replace(V, C=V.C[1:], F=V.F + ((d, r),))


def transform_split_fields(T: tuple):
    """Balanced digit-aligned split T = T1 (+) T2, | |T1| - |T2| | <= 1; the
    first factor takes the extra digit."""
    l1 = (len(T) + 1) // 2
    return T[:l1], T[l1:]


def first_transform_child(V: View, T1: tuple, T2: tuple) -> View:
    """eq. app-first-child-view: T_I = T1, O_I = T2 (+) O, C_I = C."""
    assert V.T == T1 + T2
    return replace(V, T=T1, O=T2 + V.O)


def relabel_output(V: View, T1: tuple):
    """After the first child group: the physical T1 slots hold first-stage
    frequencies; rename each label (field A) keeping its slot (eq.
    app-output-field-relabeling)."""
    A = tuple(("A", lab) for lab in T1)
    ren = dict(zip(T1, A))
    P = tuple((ren.get(lab, lab), s) for lab, s in V.P)
    return A, replace(V, P=P)


def second_transform_child(V: View, T2: tuple, A: tuple) -> View:
    """eq. app-second-child-view: T_II = T2, O_II = A (+) O, C_II = C, with
    the layout-aware twiddle pending on first access."""
    return replace(V, T=T2, O=A + V.O, pending=(V.n, A, T2))


# ---------------------------------------------------------------------------
# the scheduler (appendix B, figure cofft)
# ---------------------------------------------------------------------------

def _digit_reverse(a: int, b: int, ell: int) -> int:
    out = 0
    for _ in range(ell):
        out = out * b + a % b
        a //= b
    return out


def _dft_matrix(n: int) -> np.ndarray:
    k = np.arange(n)
    return np.array([[cmath.exp(-2j * cmath.pi * ((kk * jj) % n) / n) for jj in k] for kk in k])


@dataclass
class Stats:
    max_tsplits: int = 0
    max_bsplits: int = 0
    leaves: int = 0
    views: list = field(default_factory=list)
    written: list = field(default_factory=list)   # address set of every leaf


def co_batched_fft(V: View, data: np.ndarray, D: int, stats: Stats | None = None, check: bool = True,
                   _depth=(0, 0), _pend=()) -> Stats:
    """Runs the scheduler on view V over the physical array ``data`` (b^D
    complex items, modified in place).  Returns the instrumentation."""
    if stats is None:
        stats = Stats()
    if V.mode == IN:
        # digit-reversed entrance and exit interpretations: reverse the
        # transform field's digit order in the view (no item moves)
        V = replace(V, T=V.T[::-1], mode=OUT)
    if check:
        check_admissible(V, D)
    stats.views.append(V)
    pend = _pend + ((V.pending,) if V.pending else ())
    V = replace(V, pending=())
    b, n, s = V.b, V.n, V.s
    ts, bs = _depth

    if n <= b and s <= b:                               # leaf: constant-size DFTs
        stats.leaves += 1
        stats.max_tsplits = max(stats.max_tsplits, ts)
        stats.max_bsplits = max(stats.max_bsplits, bs)
        A = V.addr()                                     # (n, o, c)
        X = data[A]
        if pend:                                         # first access: layout-aware twiddles
            vals = V.label_values()
            for (nn, Alab, T2lab) in pend:
                l1 = len(Alab)
                a = np.zeros_like(A)
                for lab in Alab:                         # physical first-stage coordinate
                    a = a * b + vals[lab]
                j2 = np.zeros_like(A)
                for lab in T2lab:                        # logical second-stage input
                    j2 = j2 * b + vals[lab]
                k1 = np.vectorize(lambda q: _digit_reverse(int(q), b, l1))(a)
                X = X * np.exp(-2j * np.pi * ((k1 * j2) % nn) / nn)
        Y = np.tensordot(_dft_matrix(n), X, axes=(1, 0)) if n > 1 else X
        data[A] = Y                                      # in place: the leaf's own addresses
        stats.written.append(np.sort(A.ravel()))
        return stats

    if s >= n:                                           # batch split
        if V.O:
            d = V.O[0]
            kids = [outer_batch_child(V, d, r) for r in range(b)]
        else:
            kids = [contiguous_child(V, r) for r in range(b)]
        if check:                                        # data-disjoint children covering the parent
            parent = np.sort(V.addr().ravel())
            got = np.sort(np.concatenate([k.addr().ravel() for k in kids]))
            assert np.array_equal(parent, got)
        for k in kids:
            co_batched_fft(k, data, D, stats, check, (ts, bs + 1), pend)
        return stats

    # transform split: two sequential child groups over the same working set
    T1, T2 = transform_split_fields(V.T)
    VI = first_transform_child(V, T1, T2)
    if check:
        assert VI.mass == V.mass and np.array_equal(np.sort(VI.addr().ravel()), np.sort(V.addr().ravel()))
    co_batched_fft(VI, data, D, stats, check, (ts + 1, bs), pend)
    A, Vr = relabel_output(V, T1)
    VII = second_transform_child(Vr, T2, A)
    if check:
        assert VII.mass == V.mass and np.array_equal(np.sort(VII.addr().ravel()), np.sort(V.addr().ravel()))
    co_batched_fft(VII, data, D, stats, check, (ts + 1, bs), ())
    return stats


# ---------------------------------------------------------------------------
# root views of PACO's local phases
# ---------------------------------------------------------------------------

def matrix_view(b: int, m_rows: int, m_cols: int, mode: str) -> View:
    """Root view of a b^m_rows x b^m_cols row-major matrix: the row digits
    are the transform field, the column digits the contiguous field."""
    T = tuple(("r", i) for i in range(m_rows - 1, -1, -1))
    C = tuple(("c", i) for i in range(m_cols - 1, -1, -1))
    P = tuple((("r", i), m_cols + i) for i in range(m_rows)) + tuple((("c", i), i) for i in range(m_cols))
    return View(b=b, T=T, O=(), C=C, F=(), P=P, mode=mode)


def local_phase(x, b: int, m_rows: int, m_cols: int, mode: str, check: bool = True):
    """Runs the scheduler on a b^m_rows x b^m_cols row-major matrix: output
    layout gives Lemma 1's A (x) I (rows digit-reversed), input layout
    B (x) I.  Returns (result matrix, Stats)."""
    R, Cn = b ** m_rows, b ** m_cols
    data = np.array(x, dtype=np.complex128).reshape(R * Cn).copy()
    st = co_batched_fft(matrix_view(b, m_rows, m_cols, mode), data, m_rows + m_cols, check=check)
    return data.reshape(R, Cn), st
