"""The C oracle built with the host address and undefined-behaviour
sanitizers (gcc) and driven through every entry point, including the
two-level root table above 2^22 points and the threaded form of the radix-2
recursion: any out-of-bounds access, leak or undefined operation aborts the
driver."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_C = os.path.join(os.path.dirname(HERE), "oracle", "oracle.c")

DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
int64_t oracle_digit_reverse(int64_t i, int64_t b, int32_t ell);
int64_t oracle_digit_reverse_n(int64_t i, int64_t b, int64_t n);
int oracle_dft_naive(const double *x, double *y, int64_t N);
int oracle_dft_at(const double *x, int64_t N, const int64_t *ks, int64_t nk, double *y);
int oracle_fft_radix2(const double *x, double *y, int64_t N);
int oracle_fft_radix2_mt(const double *x, double *y, int64_t N, int32_t threads);
int oracle_dft(const double *x, double *y, int64_t N);
int oracle_idft(const double *y, double *x, int64_t N);
int oracle_phase1(const double *x, int64_t N1, int64_t N2, int64_t b, const int64_t *cols, int64_t ncols, double *out);
int oracle_phase2(const double *ws, double *z, int64_t N1, int64_t N2, int64_t b, int twiddle);
int oracle_phase3(const double *z, int64_t N1, int64_t N2, int64_t b, const int64_t *cols, int64_t ncols, double *out);

static double *vec(int64_t n) {
    double *v = malloc(sizeof(double) * 2 * (size_t)n);
    for (int64_t i = 0; i < 2 * n; ++i) v[i] = sin(0.37 * (double)i) + 0.1 * (double)(i % 7);
    return v;
}

int main(void) {
    int rc = 0;
    for (int64_t n = 1; n <= 64; n *= 2)
        for (int64_t i = 0; i < n; ++i) rc |= oracle_digit_reverse_n(i, 16, n) < 0;
    rc |= oracle_digit_reverse(5, 4, 2) != 5;
    rc |= oracle_digit_reverse(16, 4, 2) != -1;          /* out of range is reported */
    rc |= oracle_digit_reverse_n(24, 4, 24) != -1;       /* 24 = 4 * 6, 6 >= 4: rejected */
    const int64_t sizes[] = {1, 3, 12, 64, 1024, 2048, 4096};
    for (int s = 0; s < 7; ++s) {
        int64_t N = sizes[s];
        double *x = vec(N), *y = vec(N), *z = vec(N);
        rc |= oracle_dft(x, y, N);
        rc |= oracle_idft(y, z, N);
        if ((N & (N - 1)) == 0) rc |= oracle_fft_radix2(x, y, N);
        if (N <= 64) rc |= oracle_dft_naive(x, y, N);
        free(x); free(y); free(z);
    }
    {   /* the all-cores form: threads over the top levels, bit-identical */
        const int64_t ns[] = {2048, 1 << 15};
        const int32_t th[] = {2, 4, 8, 3};
        for (int s = 0; s < 2; ++s)
            for (int k = 0; k < 4; ++k) {
                double *x = vec(ns[s]), *y = vec(ns[s]), *z = vec(ns[s]);
                rc |= oracle_fft_radix2(x, y, ns[s]);
                rc |= oracle_fft_radix2_mt(x, z, ns[s], th[k]);
                rc |= memcmp(y, z, sizeof(double) * 2 * (size_t)ns[s]) != 0;
                free(x); free(y); free(z);
            }
        rc |= oracle_fft_radix2_mt(NULL, NULL, 12, 4) != -1;  /* not a power of two */
    }
    {   /* the two-level root table: N above 2^22 */
        int64_t N = (int64_t)1 << 23, ks[3] = {0, 1, N - 1};
        double *x = vec(N), y[6];
        rc |= oracle_dft_at(x, N, ks, 3, y);
        free(x);
    }
    const int64_t shapes[][3] = {{4, 4, 2}, {16, 8, 2}, {32, 64, 16}, {8, 8, 4}, {27, 9, 3}};
    for (int s = 0; s < 5; ++s) {
        int64_t N1 = shapes[s][0], N2 = shapes[s][1], b = shapes[s][2], N = N1 * N2;
        int64_t cols[2] = {0, N2 - 1}, cols3[2] = {0, N1 - 1};
        double *x = vec(N), *a = vec(N), *z = vec(N), *y = vec(N), *c1 = vec(2 * N1), *c3 = vec(2 * N2);
        rc |= oracle_phase1(x, N1, N2, b, NULL, 0, a);
        rc |= oracle_phase1(x, N1, N2, b, cols, 2, c1);
        rc |= oracle_phase2(a, z, N1, N2, b, 1);
        rc |= oracle_phase2(a, z, N1, N2, b, 0);
        rc |= oracle_phase3(z, N1, N2, b, NULL, 0, y);
        rc |= oracle_phase3(z, N1, N2, b, cols3, 2, c3);
        rc |= oracle_phase3(z, N1, N2, b, cols, 2, c3) != (N2 - 1 < N1 ? 0 : -1);  /* bad column reported */
        free(x); free(a); free(z); free(y); free(c1); free(c3);
    }
    printf("oracle driver rc=%d\n", rc);
    return rc;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "oracle_asan"
    cc = ["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-pthread", str(drv), ORACLE_C, "-lm", "-o", str(exe)]
    r = subprocess.run(cc, capture_output=True, text=True)
    if r.returncode != 0 and "sanitizer" in r.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "oracle driver rc=0" in run.stdout
