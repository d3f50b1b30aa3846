"""The factorisation the symmetric split form's kernels implement, on the CPU
at small sizes, against numpy's FFT (no GPU, no oracle code).

N = N1 N2 with x viewed as N1 x N2 row-major (section 2).  Both local phases
are split once more by Cooley-Tukey (Lemma 1):

  Phase I,   N1 = 16 L1:  j1 = 16 j + r,  k1 = k + L1 s     (r, s < 16);
  Phase III, N2 = R L2:   j2 = jc + L2 rr, k2 = q0 + R q    (rr, q0 < R),

with R = 16 (the symmetric form) or R = 32 (its wide variant, N2 = 2^15 on
the GPU).  Pass 1 computes U[c][r][k] = w_N1^{-k r} sum_j X[16 j + r, c]
w_L1^{-k j} into the workspace layout ((k >> 4) N2 + c) 256 + 16 r + (k & 15);
pass 2 transforms over r, applies the top-level factor of section 3.3 split
as w_N^{-v c} = w_N^{-k c} w_{16 N2}^{-s jc} w_{16 R}^{-s rr}, transforms over
rr, applies w_N2^{-q0 jc} and stores row R jc + q0; pass 3 transforms the
rows R t + q0 (t < L2) and stores row q0 + R q.  The model follows those
steps with numpy's FFT for each child; the output must be the DFT of x
(Theorem 3's claim for the whole method), and the workspace and output maps
must be bijections.  A wrong index, a dropped factor or a wrong radix in
the factor split fails this at 1e-12."""
import numpy as np
import pytest


def _w(n, e):
    return np.exp(-2j * np.pi * (np.asarray(e) % n) / n)


def sym_model(x, N1, N2, R, rr_radix=None):
    # rr_radix: the root the factor's s rr part uses (16 R; another value
    # models a wrong split)
    L1, L2, N = N1 // 16, N2 // R, N1 * N2
    rr_radix = rr_radix or 16 * R
    X = x.reshape(N1, N2)
    k = np.arange(L1)[:, None, None]
    r = np.arange(16)[None, :, None]
    c = np.arange(N2)[None, None, :]
    # pass 1: L1-point transforms over the rows 16 j + r of each column c
    U = np.fft.fft(X.reshape(L1, 16, N2), axis=0) * _w(N1, k * r)  # [k, r, c]
    ws_idx = ((k >> 4) * N2 + c) * 256 + 16 * r + (k & 15)
    assert np.unique(ws_idx).size == N
    ws = np.empty(N, complex)
    ws[ws_idx] = U
    # pass 2: over r (-> s), the top-level factor, over rr (-> q0)
    A = np.fft.fft(ws[ws_idx], axis=1)  # [k, s, c]
    s = np.arange(16)[None, :, None]
    jc, rr = c % L2, c // L2
    Z = A * _w(N, k * c) * _w(16 * N2, s * jc) * _w(rr_radix, s * rr)
    W = np.fft.fft(Z.reshape(L1, 16, R, L2), axis=2)  # [k, s, q0, jc]
    q0 = np.arange(R)[None, None, :, None]
    jcv = np.arange(L2)[None, None, None, :]
    W = W * _w(N2, q0 * jcv)
    v = np.arange(L1)[:, None, None, None] + L1 * np.arange(16)[None, :, None, None]
    out_idx = (R * jcv + q0) * N1 + v
    assert np.unique(out_idx).size == N
    out = np.empty(N, complex)
    out[out_idx] = W
    # pass 3: L2-point transforms over the rows R t + q0, to row q0 + R q
    Y = np.fft.fft(out.reshape(L2, R, N1), axis=0)  # [q, q0, column]
    return Y.reshape(N)


@pytest.mark.parametrize("N1,N2,R", [(256, 256, 16), (512, 256, 16), (256, 1024, 16), (256, 512, 32),
                                     (512, 512, 32), (1024, 1024, 32)])
def test_symmetric_factorisation_is_the_dft(N1, N2, R):
    rng = np.random.default_rng(N1 + N2 + R)
    x = rng.standard_normal(N1 * N2) + 1j * rng.standard_normal(N1 * N2)
    y = sym_model(x, N1, N2, R)
    ref = np.fft.fft(x)
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-12


def test_a_wrong_factor_radix_is_caught():
    # the wide variant with the radix-16 split of the factor (w_256 in place
    # of w_512) is not the DFT: the test above would fail on it
    rng = np.random.default_rng(5)
    N1, N2, R = 256, 512, 32
    x = rng.standard_normal(N1 * N2) + 1j * rng.standard_normal(N1 * N2)
    ref = np.fft.fft(x)
    bad = sym_model(x, N1, N2, R, rr_radix=256)
    assert np.linalg.norm(bad - ref) / np.linalg.norm(ref) > 1e-3
