"""Pins of the FP64 oracle's DFT against facts fixed by the mathematics.

The oracle computes y = Omega_N x with (Omega_N)_{k,j} = w_N^{-kj},
w_N = exp(2*pi*i/N) (paper, section 2).  Each check below would fail for a
plausible slip in the oracle: a flipped exponent sign (delta, tone, numpy),
a dropped or doubled term (Parseval, tone), a wrong twiddle index (naive vs
radix-2 vs numpy), a missing normalisation convention (round trip).
"""
import numpy as np
import pytest

import oracle

RNG = np.random.default_rng(1234)


def _rand(n):
    return RNG.standard_normal(n) + 1j * RNG.standard_normal(n)


@pytest.mark.parametrize("fn", [oracle.dft_naive, oracle.fft_radix2, oracle.dft])
@pytest.mark.parametrize("N", [1, 2, 8, 64, 1024, 4096])
def test_delta_gives_exponential(fn, N):
    # x = delta_{j0}  =>  y[k] = exp(-2 pi i k j0 / N); j0 = 0 gives all ones
    for j0 in {j for j in (0, 1, N // 3, N - 1) if j < N}:
        x = np.zeros(N, complex)
        x[j0] = 1.0
        k = np.arange(N)
        want = np.exp(-2j * np.pi * ((k * j0) % N) / N)
        assert np.max(np.abs(fn(x) - want)) < 1e-12


@pytest.mark.parametrize("fn", [oracle.dft_naive, oracle.fft_radix2, oracle.dft])
@pytest.mark.parametrize("N", [2, 16, 256, 2048])
def test_single_tone_gives_scaled_delta(fn, N):
    # x[j] = exp(+2 pi i k0 j / N)  =>  y = N * delta_{k0}
    for k0 in {0, 1, N // 2 - 1, N - 1}:
        j = np.arange(N)
        x = np.exp(2j * np.pi * ((k0 * j) % N) / N)
        want = np.zeros(N, complex)
        want[k0] = N
        assert np.max(np.abs(fn(x) - want)) < 1e-9 * N


@pytest.mark.parametrize("N", [4, 128, 4096, 1 << 16])
def test_parseval(N):
    x = _rand(N)
    y = oracle.dft(x)
    assert abs(np.vdot(y, y).real - N * np.vdot(x, x).real) < 1e-11 * N * np.vdot(x, x).real


@pytest.mark.parametrize("N", [8, 512, 8192])
def test_linearity(N):
    x, z = _rand(N), _rand(N)
    a, b = 0.3 - 1.7j, -2.25 + 0.5j
    lhs = oracle.dft(a * x + b * z)
    rhs = a * oracle.dft(x) + b * oracle.dft(z)
    assert oracle.rel_l2(lhs, rhs) < 1e-13


@pytest.mark.parametrize("N", [16, 1024, 1 << 15])
def test_round_trip(N):
    # the inverse by the conjugation identity: x = conj(F(conj(F x))) / N
    x = _rand(N)
    back = np.conj(oracle.dft(np.conj(oracle.dft(x)))) / N
    assert oracle.rel_l2(back, x) < 1e-13


@pytest.mark.parametrize("N", [1 << k for k in range(1, 13)])
def test_naive_and_radix2_agree(N):
    x = _rand(N)
    assert oracle.rel_l2(oracle.fft_radix2(x), oracle.dft_naive(x)) < 1e-12


@pytest.mark.parametrize("N", [1, 3, 5, 12, 64, 100, 4096, 1 << 18])
def test_matches_numpy_fft(N):
    # library routine (pocketfft, FP64) with the same sign convention
    x = _rand(N)
    assert oracle.rel_l2(oracle.dft(x), np.fft.fft(x)) < 1e-12


@pytest.mark.parametrize("N", [16, 4096, 1 << 14])
def test_real_input_conjugate_symmetry(N):
    x = RNG.standard_normal(N).astype(complex)
    y = oracle.dft(x)
    k = np.arange(1, N)
    assert np.max(np.abs(y[N - k] - np.conj(y[k]))) < 1e-11 * np.sqrt(N)


def test_dft_at_matches_full_transform():
    N = 4096
    x = _rand(N)
    ks = np.array([0, 1, 7, 2048, 4095, 1234])
    assert oracle.rel_l2(oracle.dft_at(x, ks), oracle.dft(x)[ks]) < 1e-13


def test_two_level_root_table_large_n():
    # above 2^22 the oracle's roots are a product of two libm values; a
    # single tone pins both the sampled and the radix-2 paths there
    N = 1 << 23
    k0 = 3_000_017
    j = np.arange(N, dtype=np.int64)
    x = np.exp(2j * np.pi * ((k0 * j) % N) / N)
    ys = oracle.dft_at(x, [k0, 0, k0 + 1, N - 1])
    assert abs(ys[0] - N) < 1e-6 * N
    assert np.max(np.abs(ys[1:])) < 1e-6 * N
    y = oracle.fft_radix2(x)
    y[k0] -= N
    assert np.max(np.abs(y)) < 1e-6 * N


# ---- the inverse (oracle.idft): pinned by closed forms, numpy and round trips

@pytest.mark.parametrize("N", [1, 2, 8, 64, 1024, 2048, 1 << 14])
def test_idft_delta_gives_positive_exponential(N):
    # y = delta_{k0}  =>  x[j] = exp(+2 pi i j k0 / N) / N  (small N: naive sum, large: radix-2)
    for k0 in {k for k in (0, 1, N // 3, N - 1) if k < N}:
        y = np.zeros(N, complex)
        y[k0] = 1.0
        j = np.arange(N)
        want = np.exp(2j * np.pi * ((j * k0) % N) / N) / N
        assert np.max(np.abs(oracle.idft(y) - want)) < 1e-12 / N


@pytest.mark.parametrize("N", [1, 3, 12, 64, 1000, 2048, 1 << 16])
def test_idft_matches_numpy_ifft(N):
    y = _rand(N)
    assert oracle.rel_l2(oracle.idft(y), np.fft.ifft(y)) < 1e-12


@pytest.mark.parametrize("N", [16, 1024, 4096, 1 << 15])
def test_idft_inverts_dft_both_ways(N):
    x = _rand(N)
    assert oracle.rel_l2(oracle.idft(oracle.dft(x)), x) < 1e-13
    assert oracle.rel_l2(oracle.dft(oracle.idft(x)), x) < 1e-13


def test_idft_is_not_the_forward_transform():
    # a sign slip would make idft(y) = dft(y)/N; these differ for N >= 3
    y = _rand(64)
    assert oracle.rel_l2(oracle.idft(y), oracle.dft(y) / 64) > 0.5


@pytest.mark.parametrize("N,threads", [(1 << 11, 2), (1 << 16, 4), (1 << 20, 8), (1 << 23, 16), (1 << 12, 3)])
def test_threaded_radix2_is_bit_identical(N, threads):
    # the all-cores form (CPU baseline) runs the same recursion over threads:
    # every output is the same FP64 value as the one-thread oracle's; 2^23
    # takes the two-level root table
    x = np.random.default_rng(N).standard_normal((N, 2)).view(np.complex128).ravel()
    one = oracle.fft_radix2(x)
    many = oracle.fft_radix2(x, threads=threads)
    assert np.array_equal(one.view(np.uint64), many.view(np.uint64))


def test_cpu_threads_and_model():
    assert 1 <= oracle.cpu_threads() <= 16
    assert isinstance(oracle.cpu_model(), str) and oracle.cpu_model()
