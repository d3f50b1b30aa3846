"""Plain FP64 CPU oracle for the PACO transform.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The GPU
library and its Python binding never import it, and this package never
imports them: the two sides share no code, tables or constants.  Inputs for
both sides come from the seeded generators, which hold none of the method's
arithmetic.

Contents
--------
* ``liboracle.so`` (``oracle.c``): the DFT by its definition (section 2), a
  textbook recursive radix-2 FFT, the inverse DFT, brute-force base-b digit
  reversal (appendix A.1) and its mixed-radix reading for sizes b^m * r, and
  the three stage-wise references (Phase I output layout, the fused middle
  permutation with the top-level twiddle, Phase III input layout; sections
  3.1-3.4 and 4.2).  All in FP64.
* ``view_model``: a literal model of the view-based local scheduler
  (appendix A.3-A.8, appendix B), a second reference for the layout algebra.
* ``para_co_drp``: a literal, per-processor model of the redistribution
  procedure of appendix C.5 (pack by fused macro-element digit reversal, one
  block exchange, block transposes, unpack by macro-element digit reversal),
  in pure Python on small cases.  It exists to pin the definition-based
  permutation to the paper's own procedure and to Fig. 1.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

__all__ = [
    "build", "digit_reverse", "digit_reverse_py", "dft", "dft_naive", "fft_radix2",
    "dft_at", "idft", "digit_reverse_n", "radices", "reverse_with_radices", "phase1", "phase2", "phase3",
    "paco_reference",
    "para_co_drp", "fused_macro_digit_reversal", "macro_digit_reversal",
    "rel_l2",
]


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (plain C, -O2)."""
    import subprocess

    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.oracle_digit_reverse.restype = i64
    lib.oracle_digit_reverse.argtypes = [i64, i64, ctypes.c_int32]
    lib.oracle_digit_reverse_n.restype = i64
    lib.oracle_digit_reverse_n.argtypes = [i64, i64, i64]
    for name in ("oracle_dft_naive", "oracle_fft_radix2", "oracle_dft", "oracle_idft"):
        getattr(lib, name).restype = ctypes.c_int
        getattr(lib, name).argtypes = [P, P, i64]
    lib.oracle_fft_radix2_mt.restype = ctypes.c_int
    lib.oracle_fft_radix2_mt.argtypes = [P, P, i64, ctypes.c_int32]
    lib.oracle_dft_at.restype = ctypes.c_int
    lib.oracle_dft_at.argtypes = [P, i64, P, i64, P]
    lib.oracle_phase1.restype = ctypes.c_int
    lib.oracle_phase1.argtypes = [P, i64, i64, i64, P, i64, P]
    lib.oracle_phase2.restype = ctypes.c_int
    lib.oracle_phase2.argtypes = [P, P, i64, i64, i64, ctypes.c_int]
    lib.oracle_phase3.restype = ctypes.c_int
    lib.oracle_phase3.argtypes = [P, i64, i64, i64, P, i64, P]
    _lib = lib
    return lib


def _c128(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x).astype(np.complex128, copy=False))


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


# ---------------------------------------------------------------------------
# digit reversal (appendix A.1)
# ---------------------------------------------------------------------------

def digit_reverse(i: int, b: int, ell: int) -> int:
    """pi_ell(i) in base b, by the C brute force on the digit list."""
    r = _load().oracle_digit_reverse(int(i), int(b), int(ell))
    if r < 0:
        raise ValueError(f"bad digit reversal arguments i={i} b={b} ell={ell}")
    return int(r)


def digit_reverse_py(i: int, b: int, ell: int) -> int:
    """pi_ell(i) in pure Python: list the ell base-b digits most significant
    first, reverse the list, read it back."""
    msb_first = []
    v = i
    for _ in range(ell):
        msb_first.insert(0, v % b)
        v //= b
    if v:
        raise ValueError("i >= b**ell")
    out = 0
    for d in msb_first[::-1]:         # the reversed string d_0 .. d_{ell-1}
        out = out * b + d
    return out


def digit_reverse_n(i: int, b: int, n: int) -> int:
    """pi(i) over [0, n), n = b^m * r (1 <= r < b): digit radices (b, ..., b, r)
    least significant first, reversed and read back with the radices
    reversed; for n = b^m the paper's pi_m (appendix A.1).  Sizes other than
    powers of b lie outside the paper's preconditions (section 5,
    Limitations): this is the mixed-radix reading."""
    r = _load().oracle_digit_reverse_n(int(i), int(b), int(n))
    if r < 0:
        raise ValueError(f"bad digit reversal arguments i={i} b={b} n={n}")
    return int(r)


def radices(b: int, n: int) -> list:
    """The digit radices of [0, n) in the mixed-radix reading, least
    significant first: (b, ..., b, r)."""
    out = []
    while n > 1:
        R = b if n % b == 0 else n
        if R > b:
            raise ValueError("n is not b^m * r with r < b")
        out.append(R)
        n //= R
    return out


def reverse_with_radices(i: int, rad) -> int:
    """Digit reversal for an explicit radix list (least significant first),
    in pure Python: split i into digits, reverse the list, read it back with
    the reversed radix list."""
    digits = []
    for R in rad:
        digits.append(i % R)
        i //= R
    if i:
        raise ValueError("i out of range")
    out, w = 0, 1
    for d, R in zip(digits[::-1], rad[::-1]):
        out += d * w
        w *= R
    return out


def digit_reverse_table(b: int, ell: int) -> np.ndarray:
    return np.array([digit_reverse(i, b, ell) for i in range(b ** ell)], dtype=np.int64)


# ---------------------------------------------------------------------------
# the DFT (section 2) and the stage-wise references
# ---------------------------------------------------------------------------

def dft_naive(x) -> np.ndarray:
    x = _c128(x)
    y = np.empty_like(x)
    _check(_load().oracle_dft_naive(_ptr(x), _ptr(y), x.size), "dft_naive")
    return y


def fft_radix2(x, threads: int = 1) -> np.ndarray:
    """The recursive radix-2 FFT; threads > 1 runs the same recursion with
    its top levels spread over that many threads (bit-identical output)."""
    x = _c128(x)
    y = np.empty_like(x)
    if threads > 1:
        _check(_load().oracle_fft_radix2_mt(_ptr(x), _ptr(y), x.size, int(threads)), "fft_radix2_mt")
    else:
        _check(_load().oracle_fft_radix2(_ptr(x), _ptr(y), x.size), "fft_radix2")
    return y


def cpu_threads() -> int:
    """Host threads the all-cores oracle uses: the CPUs this process may run
    on, at most 16 (the host share that goes with one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model() -> str:
    """The host CPU's model string (from /proc/cpuinfo, as lscpu prints it)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def dft(x) -> np.ndarray:
    """y = Omega_N x (naive definition for small N, radix-2 above)."""
    x = _c128(x)
    y = np.empty_like(x)
    _check(_load().oracle_dft(_ptr(x), _ptr(y), x.size), "dft")
    return y


def idft(y) -> np.ndarray:
    """x = Omega_N^{-1} y = (1/N) sum_k y[k] w_N^{+jk}: the inverse the paper
    names (sections 1 and 5) for the forward convention of section 2."""
    y = _c128(y)
    x = np.empty_like(y)
    _check(_load().oracle_idft(_ptr(y), _ptr(x), y.size), "idft")
    return x


def dft_at(x, ks) -> np.ndarray:
    """Selected outputs y[k] of the length-len(x) DFT, each O(N)."""
    x = _c128(x).ravel()
    ks = np.ascontiguousarray(np.asarray(ks, dtype=np.int64))
    y = np.empty(ks.size, dtype=np.complex128)
    _check(_load().oracle_dft_at(_ptr(x), x.size, _ptr(ks), ks.size, _ptr(y)), "dft_at")
    return y


def phase1(x, N1: int, N2: int, b: int, cols=None) -> np.ndarray:
    """Phase-I buffer Atilde[a,c] = A[pi_{m1}(a), c] (output layout, Lemma 1).
    With ``cols``, only those columns (an N1 x len(cols) array)."""
    x = _c128(x).reshape(N1 * N2)
    if cols is None:
        out = np.empty((N1, N2), dtype=np.complex128)
        _check(_load().oracle_phase1(_ptr(x), N1, N2, b, None, 0, _ptr(out)), "phase1")
        return out
    cols = np.ascontiguousarray(np.asarray(cols, dtype=np.int64))
    out = np.empty((N1, cols.size), dtype=np.complex128)
    _check(_load().oracle_phase1(_ptr(x), N1, N2, b, _ptr(cols), cols.size, _ptr(out)), "phase1")
    return out


def phase2(ws, N1: int, N2: int, b: int, twiddle: bool = True) -> np.ndarray:
    """Middle stage: out[pi_{m2}(c), pi_{m1}(a)] = ws[a,c] * w_N^{-pi_{m1}(a) c}
    (section 3.3 / 4.2).  ``twiddle=False``: the bare permutation."""
    ws = _c128(ws).reshape(N1 * N2)
    z = np.empty((N2, N1), dtype=np.complex128)
    _check(_load().oracle_phase2(_ptr(ws), _ptr(z), N1, N2, b, 1 if twiddle else 0), "phase2")
    return z


def phase3(z, N1: int, N2: int, b: int, cols=None) -> np.ndarray:
    """Phase III: Y[k2,v] = sum_j2 Zhat[pi_{m2}(j2), v] w_{N2}^{-k2 j2}."""
    z = _c128(z).reshape(N2 * N1)
    if cols is None:
        out = np.empty((N2, N1), dtype=np.complex128)
        _check(_load().oracle_phase3(_ptr(z), N1, N2, b, None, 0, _ptr(out)), "phase3")
        return out
    cols = np.ascontiguousarray(np.asarray(cols, dtype=np.int64))
    out = np.empty((N2, cols.size), dtype=np.complex128)
    _check(_load().oracle_phase3(_ptr(z), N1, N2, b, _ptr(cols), cols.size, _ptr(out)), "phase3")
    return out


def paco_reference(x, N1: int, N2: int, b: int) -> np.ndarray:
    """The three stage references composed (section 3.4, eq. paco-composite-op):
    returns the N2 x N1 output Y, which Theorem 3 says equals y = Omega_N x
    under Y[k2,k1] = y[k1 + k2 N1]."""
    return phase3(phase2(phase1(x, N1, N2, b), N1, N2, b), N1, N2, b)


def rel_l2(got, ref) -> float:
    got = np.asarray(got, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (den if den > 0 else 1.0))


# ---------------------------------------------------------------------------
# literal model of the redistribution procedure (appendix C)
# ---------------------------------------------------------------------------

def macro_digit_reversal(X, n: int, b: int):
    """Macro-element digit reversal (appendix C.1) in place: X is a list of n
    macro-elements (lists); swap each two-cycle {i, pi(i)} once (i < pi(i))."""
    ell = round(math.log(n, b))
    assert b ** ell == n
    for i in range(n):
        k = digit_reverse_py(i, b, ell)
        if i < k:
            for j in range(len(X[i])):
                X[i][j], X[k][j] = X[k][j], X[i][j]


def fused_macro_digit_reversal(X, n: int, b: int, g, mul):
    """Appendix C.2: X'[i][j] = g(i,j) * X[pi(i)][j], in place by two-cycles;
    ``mul(w, x)`` applies the coefficient."""
    ell = round(math.log(n, b))
    assert b ** ell == n
    for i in range(n):
        k = digit_reverse_py(i, b, ell)
        if i < k:
            for j in range(len(X[i])):
                x, y = X[i][j], X[k][j]
                X[i][j] = mul(g(i, j), y)
                X[k][j] = mul(g(k, j), x)
        elif i == k:
            for j in range(len(X[i])):
                X[i][j] = mul(g(i, j), X[i][j])


def _omega_neg(r: int, N: int) -> complex:
    a = 2.0 * math.pi * ((r % N) / N)
    return complex(math.cos(a), -math.sin(a))


def para_co_drp(slabs, N1: int, N2: int, p: int, b: int, twiddle: bool = True, trace=None):
    """Per-processor redistribution of appendix C.5, run for all p processors.

    ``slabs[q]`` is processor q's Phase-I slab: N1 rows (lists) of N2/p items,
    global column c = q*N2/p + c_loc.  Items are complex numbers, or any
    labels when ``twiddle`` is False.  Returns the p target slabs, each N2
    rows of N1/p items.  ``trace`` (a dict) receives, when given, the global
    views after pack / exchange / transpose / unpack, each a list of rows.
    """
    N = N1 * N2
    s2, s1 = N2 // p, N1 // p
    assert s2 * p == N2 and s1 * p == N1
    X = [[list(row) for row in slabs[q]] for q in range(p)]

    # local pack: N1-field reversal with the top-level twiddle g(v,c)
    for q in range(p):
        def g(v, c_loc, q=q):
            return _omega_neg(v * (q * s2 + c_loc), N) if twiddle else None
        mul = (lambda w, x: w * x) if twiddle else (lambda w, x: x)
        fused_macro_digit_reversal(X[q], N1, b, g, mul)
    if trace is not None:
        trace["packed"] = [sum((X[q][r] for q in range(p)), []) for r in range(N1)]

    # one exchange: block S_{q,q'} (rows q'*s1 .. +s1 of the packed slab) goes
    # to raw region R_{q',q} on processor q'; raw regions ordered by source
    R = [[None] * p for _ in range(p)]
    for q in range(p):
        for qd in range(p):
            R[qd][q] = [list(X[q][qd * s1 + vl]) for vl in range(s1)]
    if trace is not None:
        # received view: processor q' holds rows v = q'*s1 + v_loc, all c
        trace["received"] = [sum((R[qd][q][vl] for q in range(p)), [])
                             for qd in range(p) for vl in range(s1)]

    # local transpose of each received block into the target slab rows
    Y = []
    for qd in range(p):
        Yq = [[None] * s1 for _ in range(N2)]
        for r in range(p):
            T = [[R[qd][r][vl][cl] for vl in range(s1)] for cl in range(s2)]  # CO-Transpose
            for cl in range(s2):
                Yq[r * s2 + cl] = list(T[cl])                               # copy T -> Y_{q,r}
        Y.append(Yq)
    if trace is not None:
        trace["transposed"] = [sum((Y[qd][c] for qd in range(p)), []) for c in range(N2)]

    # local unpack: N2-field reversal of row macro-elements of length N1/p
    for qd in range(p):
        macro_digit_reversal(Y[qd], N2, b)
    if trace is not None:
        trace["output"] = [sum((Y[qd][u] for qd in range(p)), []) for u in range(N2)]
    return Y


def slabs_from_matrix(A, p: int):
    """Split an N1 x N2 matrix (list of rows) into p column slabs."""
    N2 = len(A[0])
    s2 = N2 // p
    return [[list(row[q * s2:(q + 1) * s2]) for row in A] for q in range(p)]


def matrix_from_target_slabs(Y):
    """Join p target slabs (N2 rows of N1/p) into the N2 x N1 matrix."""
    p = len(Y)
    return [sum((Y[q][u] for q in range(p)), []) for u in range(len(Y[0]))]
