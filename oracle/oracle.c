/*
 * oracle.c -- plain FP64 CPU reference for the PACO transform.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU library
 * never includes, links or calls anything here, and nothing here includes or
 * calls the GPU library: the two share no code, tables or constants.
 *
 * Every routine is the plain definition of what the paper computes, written
 * for a reader to check by eye: no blocking, no fusion, no reordering beyond
 * what the cited definition states.  Complex values are interleaved
 * (re, im) pairs of double.  All index arithmetic is exact int64.
 *
 * Sign and scale (paper, section 2 "Model and Main Result"): the forward DFT
 *   y = Omega_N x,  (Omega_N)_{k,j} = w_N^{-kj},  w_N = exp(2*pi*i/N),
 * negative exponent, no normalisation.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------ */
/* roots of unity                                                       */
/* ------------------------------------------------------------------ */

/* w_N^{-r} = exp(-2*pi*i*r/N) for an exactly reduced integer r in [0,N).
 * One libm cos/sin call per value, no recurrence. */
static void root_neg(int64_t r, int64_t N, double *re, double *im)
{
    double a = 2.0 * M_PI * ((double)r / (double)N);
    *re = cos(a);
    *im = -sin(a);
}

/* Exact power table for w_N^{-r}, r in [0,N).  Up to 2^22 entries every
 * value is one direct libm call; above that a two-level split
 * r = hi*L + lo is used, w^{-r} = w^{-hi*L} * w^{-lo}, both factors direct
 * libm values, product in FP64 (about 1 ulp of FP64). */
typedef struct {
    int64_t N, L;      /* L == 0: direct table of N entries */
    double *hi, *lo;   /* hi: N/L entries (or N if direct), lo: L entries */
} roots_t;

static int roots_init(roots_t *t, int64_t N)
{
    memset(t, 0, sizeof(*t));
    t->N = N;
    if (N <= ((int64_t)1 << 22)) {
        t->hi = (double *)malloc(sizeof(double) * 2 * (size_t)N);
        if (!t->hi) return -1;
        for (int64_t r = 0; r < N; ++r) root_neg(r, N, &t->hi[2 * r], &t->hi[2 * r + 1]);
        return 0;
    }
    int64_t L = 1;
    while (L * L < N) L <<= 1;            /* N is a power of two here */
    t->L = L;
    int64_t H = N / L;
    t->hi = (double *)malloc(sizeof(double) * 2 * (size_t)H);
    t->lo = (double *)malloc(sizeof(double) * 2 * (size_t)L);
    if (!t->hi || !t->lo) { free(t->hi); free(t->lo); return -1; }
    for (int64_t h = 0; h < H; ++h) root_neg(h * L, N, &t->hi[2 * h], &t->hi[2 * h + 1]);
    for (int64_t l = 0; l < L; ++l) root_neg(l, N, &t->lo[2 * l], &t->lo[2 * l + 1]);
    return 0;
}

static void roots_free(roots_t *t) { free(t->hi); free(t->lo); memset(t, 0, sizeof(*t)); }

/* w_N^{-r} for r in [0,N). */
static inline void roots_get(const roots_t *t, int64_t r, double *re, double *im)
{
    if (t->L == 0) { *re = t->hi[2 * r]; *im = t->hi[2 * r + 1]; return; }
    int64_t h = r / t->L, l = r % t->L;
    double ar = t->hi[2 * h], ai = t->hi[2 * h + 1];
    double br = t->lo[2 * l], bi = t->lo[2 * l + 1];
    *re = ar * br - ai * bi;
    *im = ar * bi + ai * br;
}

/* ------------------------------------------------------------------ */
/* base-b digit reversal (appendix A.1)                                 */
/* ------------------------------------------------------------------ */

/* pi_ell(i): write i as ell base-b digits d_{ell-1} .. d_0 (most significant
 * first), reverse the digit string, read it back.  Brute force on the digit
 * list, for any b >= 2 (not only powers of two).  Returns -1 on bad input. */
int64_t oracle_digit_reverse(int64_t i, int64_t b, int32_t ell)
{
    if (b < 2 || ell < 0 || ell > 62 || i < 0) return -1;
    int64_t digits[64];
    int64_t v = i;
    for (int32_t r = 0; r < ell; ++r) { digits[r] = v % b; v /= b; } /* digits[r] = d_r */
    if (v != 0) return -1;                                           /* i >= b^ell */
    int64_t out = 0;
    /* reversed string d_0 .. d_{ell-1}, d_0 most significant */
    for (int32_t r = 0; r < ell; ++r) out = out * b + digits[r];
    return out;
}

/* Mixed-radix digit reversal of i in [0, n), for n = b^m * r with
 * 1 <= r < b: the paper's preconditions (section 2) ask for n = b^m; the
 * Limitations of section 5 name other sizes as outside its scope.  The
 * reading used here: i has the digit radices (b, ..., b, r), least
 * significant first (m digits of radix b, then one of radix r when r > 1);
 * pi reverses the digit string and reads it back with the radices reversed,
 * (r, b, ..., b).  For r = 1 this is pi_m of appendix A.1.  Brute force on
 * the digit list; returns -1 on bad input. */
int64_t oracle_digit_reverse_n(int64_t i, int64_t b, int64_t n)
{
    if (b < 2 || n < 1 || i < 0 || i >= n) return -1;
    int64_t radix[64], digit[64];
    int L = 0;
    int64_t rest = n, v = i;
    while (rest > 1) {                       /* radices, least significant first */
        int64_t R = (rest % b == 0) ? b : rest;
        if (R > b) return -1;                /* n is not b^m * r with r < b */
        radix[L] = R;
        digit[L] = v % R;
        v /= R;
        rest /= R;
        ++L;
    }
    /* reversed string: digit[L-1] least significant (radix[L-1]), then
     * digit[L-2] (radix[L-2]), ..., digit[0] most significant */
    int64_t out = 0, w = 1;
    for (int k = L - 1; k >= 0; --k) {
        out += digit[k] * w;
        w *= radix[k];
    }
    return out;
}

/* ------------------------------------------------------------------ */
/* the DFT itself (section 2)                                           */
/* ------------------------------------------------------------------ */

/* y[k] = sum_j x[j] w_N^{-(k*j mod N)}, O(N^2).  Intended for small N. */
int oracle_dft_naive(const double *x, double *y, int64_t N)
{
    if (N < 1) return -1;
    roots_t t;
    if (roots_init(&t, N)) return -2;
    for (int64_t k = 0; k < N; ++k) {
        double sr = 0.0, si = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            int64_t r = (k * j) % N;
            double wr, wi;
            roots_get(&t, r, &wr, &wi);
            double xr = x[2 * j], xi = x[2 * j + 1];
            sr += xr * wr - xi * wi;
            si += xr * wi + xi * wr;
        }
        y[2 * k] = sr;
        y[2 * k + 1] = si;
    }
    roots_free(&t);
    return 0;
}

/* Selected outputs of the same definition: y[ks[i]] for i < nk, O(N) each.
 * Used to check single outputs of transforms too large for a full run. */
int oracle_dft_at(const double *x, int64_t N, const int64_t *ks, int64_t nk, double *y)
{
    if (N < 1) return -1;
    roots_t t;
    if (roots_init(&t, N)) return -2;
    for (int64_t i = 0; i < nk; ++i) {
        int64_t k = ks[i] % N;
        double sr = 0.0, si = 0.0;
        int64_t r = 0;                          /* r = (k*j) mod N, kept exact */
        for (int64_t j = 0; j < N; ++j, r = (r + k >= N) ? r + k - N : r + k) {
            double wr, wi;
            roots_get(&t, r, &wr, &wi);
            double xr = x[2 * j], xi = x[2 * j + 1];
            sr += xr * wr - xi * wi;
            si += xr * wi + xi * wr;
        }
        y[2 * i] = sr;
        y[2 * i + 1] = si;
    }
    roots_free(&t);
    return 0;
}

/* The butterflies of one level of the radix-2 recursion for k in [k0, k1):
 * y[k] and y[k + h] (h = n/2) hold the transforms of the even and the odd
 * samples; they become y[k] +- w_n^{-k} y[k + h], w_n^{-k} = w_N^{-k*(N/n)}. */
static void fft_r2_combine(double *y, int64_t n, int64_t N, const roots_t *t, int pos, int64_t k0, int64_t k1)
{
    int64_t h = n / 2;
    for (int64_t k = k0; k < k1; ++k) {
        double wr, wi;
        roots_get(t, k * (N / n), &wr, &wi);
        if (pos) wi = -wi;                           /* w_n^{+k}: the inverse's roots */
        double er = y[2 * k], ei = y[2 * k + 1];
        double orr = y[2 * (k + h)], oi = y[2 * (k + h) + 1];
        double tr = orr * wr - oi * wi, ti = orr * wi + oi * wr;
        y[2 * k] = er + tr;
        y[2 * k + 1] = ei + ti;
        y[2 * (k + h)] = er - tr;
        y[2 * (k + h) + 1] = ei - ti;
    }
}

/* Textbook recursive radix-2 decimation-in-time FFT (N a power of two):
 * the even- and odd-indexed halves are transformed, then combined with
 * w_n^{-k} = w_N^{-k*(N/n)}.  x is read with stride `xs` (in complex items),
 * y is written contiguously. */
static void fft_r2_rec(const double *x, int64_t xs, double *y, int64_t n, int64_t N, const roots_t *t, int pos)
{
    if (n == 1) { y[0] = x[0]; y[1] = x[1]; return; }
    int64_t h = n / 2;
    fft_r2_rec(x, 2 * xs, y, h, N, t, pos);             /* even samples -> y[0..h)   */
    fft_r2_rec(x + 2 * xs, 2 * xs, y + 2 * h, h, N, t, pos); /* odd samples -> y[h..n) */
    fft_r2_combine(y, n, N, t, pos, 0, h);
}

int oracle_fft_radix2(const double *x, double *y, int64_t N)
{
    if (N < 1 || (N & (N - 1))) return -1;
    roots_t t;
    if (roots_init(&t, N)) return -2;
    fft_r2_rec(x, 1, y, N, N, &t, 0);
    roots_free(&t);
    return 0;
}

/* ------------------------------------------------------------------ */
/* all-cores form of the same recursion (CPU baseline timing only)      */
/* ------------------------------------------------------------------ */

/* The recursion above with its top `depth` levels spread over threads: the
 * two half transforms of such a level run concurrently and its butterfly
 * loop is cut into 2^depth independent k ranges.  Every output is formed
 * by exactly the operations of fft_r2_rec, in the same order, so the result
 * is bit-identical to oracle_fft_radix2; only the wall time differs. */
typedef struct {
    const double *x;
    int64_t xs;
    double *y;
    int64_t n, N;
    const roots_t *t;
    int pos, depth;
    int64_t k0, k1;     /* combine jobs: the k range */
} r2_job;

static void fft_r2_rec_mt(const double *x, int64_t xs, double *y, int64_t n, int64_t N, const roots_t *t, int pos,
                          int depth);

static void *r2_half_entry(void *a)
{
    r2_job *j = (r2_job *)a;
    fft_r2_rec_mt(j->x, j->xs, j->y, j->n, j->N, j->t, j->pos, j->depth);
    return NULL;
}

static void *r2_combine_entry(void *a)
{
    r2_job *j = (r2_job *)a;
    fft_r2_combine(j->y, j->n, j->N, j->t, j->pos, j->k0, j->k1);
    return NULL;
}

static void fft_r2_rec_mt(const double *x, int64_t xs, double *y, int64_t n, int64_t N, const roots_t *t, int pos,
                          int depth)
{
    if (depth <= 0 || n < 2048) { fft_r2_rec(x, xs, y, n, N, t, pos); return; }
    int64_t h = n / 2;
    r2_job even = {x, 2 * xs, y, h, N, t, pos, depth - 1, 0, 0};
    pthread_t th;
    int spawned = pthread_create(&th, NULL, r2_half_entry, &even) == 0;
    if (!spawned) r2_half_entry(&even);
    fft_r2_rec_mt(x + 2 * xs, 2 * xs, y + 2 * h, h, N, t, pos, depth - 1);
    if (spawned) pthread_join(th, NULL);
    /* the butterfly loop of this level in 2^depth k ranges */
    enum { kMaxParts = 64 };
    int parts = 1 << (depth < 6 ? depth : 6);
    r2_job cj[kMaxParts];
    pthread_t ct[kMaxParts];
    int ok[kMaxParts];
    for (int i = 0; i < parts; ++i) {
        r2_job j = {x, xs, y, n, N, t, pos, 0, h * i / parts, h * (i + 1) / parts};
        cj[i] = j;
        ok[i] = i > 0 && pthread_create(&ct[i], NULL, r2_combine_entry, &cj[i]) == 0;
    }
    r2_combine_entry(&cj[0]);
    for (int i = 1; i < parts; ++i) {
        if (ok[i]) pthread_join(ct[i], NULL);
        else r2_combine_entry(&cj[i]);
    }
}

typedef struct {
    roots_t *t;
    int64_t r0, r1;
} roots_job;

static void *roots_fill_entry(void *a)
{
    roots_job *j = (roots_job *)a;
    for (int64_t r = j->r0; r < j->r1; ++r) root_neg(r, j->t->N, &j->t->hi[2 * r], &j->t->hi[2 * r + 1]);
    return NULL;
}

/* oracle_fft_radix2 on up to `threads` threads (rounded down to a power of
 * two, at most 64): the same root table (direct entries filled in
 * independent ranges) and the recursion above.  Bit-identical output. */
int oracle_fft_radix2_mt(const double *x, double *y, int64_t N, int32_t threads)
{
    if (N < 1 || (N & (N - 1)) || threads < 1) return -1;
    int depth = 0;
    while (depth < 6 && (2 << depth) <= threads) ++depth;
    roots_t t;
    if (N <= ((int64_t)1 << 22) && depth > 0) {
        memset(&t, 0, sizeof(t));
        t.N = N;
        t.hi = (double *)malloc(sizeof(double) * 2 * (size_t)N);
        if (!t.hi) return -2;
        int parts = 1 << depth;
        roots_job rj[64];
        pthread_t rt[64];
        int ok[64];
        for (int i = 0; i < parts; ++i) {
            roots_job j = {&t, N * i / parts, N * (i + 1) / parts};
            rj[i] = j;
            ok[i] = i > 0 && pthread_create(&rt[i], NULL, roots_fill_entry, &rj[i]) == 0;
        }
        roots_fill_entry(&rj[0]);
        for (int i = 1; i < parts; ++i) {
            if (ok[i]) pthread_join(rt[i], NULL);
            else roots_fill_entry(&rj[i]);
        }
    } else if (roots_init(&t, N)) {
        return -2;
    }
    fft_r2_rec_mt(x, 1, y, N, N, &t, 0, depth);
    roots_free(&t);
    return 0;
}

/* y = Omega_N x: the naive definition for small N, the radix-2 FFT above. */
int oracle_dft(const double *x, double *y, int64_t N)
{
    if (N <= 1024 || (N & (N - 1))) return oracle_dft_naive(x, y, N);
    return oracle_fft_radix2(x, y, N);
}

/* The inverse DFT x = Omega_N^{-1} y, (Omega_N^{-1})_{j,k} = w_N^{+jk} / N.
 * The paper names the inverse transform without specifying it (sections 1
 * and 5, Limitations); this is the textbook definition for its forward
 * convention of section 2: the naive sum for small N, the same radix-2
 * recursion with w_n^{+k} above, then the 1/N scale. */
int oracle_idft(const double *y, double *x, int64_t N)
{
    if (N < 1) return -1;
    roots_t t;
    if (roots_init(&t, N)) return -2;
    if (N <= 1024 || (N & (N - 1))) {
        for (int64_t j = 0; j < N; ++j) {
            double sr = 0.0, si = 0.0;
            for (int64_t k = 0; k < N; ++k) {
                double wr, wi;
                roots_get(&t, (j * k) % N, &wr, &wi);
                wi = -wi;                       /* w_N^{+jk} */
                double yr = y[2 * k], yi = y[2 * k + 1];
                sr += yr * wr - yi * wi;
                si += yr * wi + yi * wr;
            }
            x[2 * j] = sr;
            x[2 * j + 1] = si;
        }
    } else {
        fft_r2_rec(y, 1, x, N, N, &t, 1);
    }
    for (int64_t j = 0; j < 2 * N; ++j) x[j] /= (double)N;
    roots_free(&t);
    return 0;
}

/* ------------------------------------------------------------------ */
/* stage-wise references (sections 3.1-3.4, 4.2)                       */
/* ------------------------------------------------------------------ */

/* In all three, pi_{m1} and pi_{m2} are oracle_digit_reverse_n over [0, N1)
 * and [0, N2): the paper's base-b reversals when N1, N2 are powers of b, the
 * mixed-radix reading above otherwise. */

/* n = b^m * r with 1 <= r < b (r = 1: the paper's n = b^m). */
static int digit_shape_ok(int64_t n, int64_t b)
{
    if (b < 2 || n < 1) return 0;
    while (n % b == 0) n /= b;
    return n < b;
}

/* Phase I, output layout A_{m1} (x) I_{N2} (Lemma 1; section 3.4):
 *   A[k1,c] = sum_{j1} X[j1,c] w_{N1}^{-k1*j1}  (inner sum of the
 *   two-factor Cooley-Tukey identity, section 3.1), and the buffer holds
 *   Atilde[a,c] = A[pi_{m1}(a), c]  (digit-reversed rows).
 * x: N1 x N2 row-major.  Only the ncols columns listed in cols are formed
 * (cols == NULL: all N2 columns, ncols ignored); out is N1 x ncols
 * row-major, out[a*ncols + i] = Atilde[a, cols[i]]. */
int oracle_phase1(const double *x, int64_t N1, int64_t N2, int64_t b,
                  const int64_t *cols, int64_t ncols, double *out)
{
    if (!digit_shape_ok(N1, b) || N2 < 1) return -1;
    if (!cols) ncols = N2;
    double *col = (double *)malloc(sizeof(double) * 2 * (size_t)N1);
    double *dft = (double *)malloc(sizeof(double) * 2 * (size_t)N1);
    if (!col || !dft) { free(col); free(dft); return -2; }
    int rc = 0;
    for (int64_t i = 0; i < ncols && rc == 0; ++i) {
        int64_t c = cols ? cols[i] : i;
        if (c < 0 || c >= N2) { rc = -1; break; }
        for (int64_t j1 = 0; j1 < N1; ++j1) {
            col[2 * j1] = x[2 * (j1 * N2 + c)];
            col[2 * j1 + 1] = x[2 * (j1 * N2 + c) + 1];
        }
        rc = oracle_dft(col, dft, N1);
        for (int64_t a = 0; a < N1; ++a) {
            int64_t k1 = oracle_digit_reverse_n(a, b, N1);
            out[2 * (a * ncols + i)] = dft[2 * k1];
            out[2 * (a * ncols + i) + 1] = dft[2 * k1 + 1];
        }
    }
    free(col);
    free(dft);
    return rc;
}

/* Phase II, the fused middle permutation with the top-level twiddle
 * (section 3.3, eq. full-middle-digit-reversal; section 4.2, eq.
 * unpacked-phase-three-layout; appendix C.2 destination-indexed twiddle):
 * the item at Phase-I physical (a,c) represents k1 = pi_{m1}(a), is scaled
 * by w_N^{-k1*c} (c the global column) and lands at
 *   (u,v) = (pi_{m2}(c), pi_{m1}(a))  of the N2 x N1 output.
 * twiddle == 0 gives the bare permutation (values moved, not scaled). */
int oracle_phase2(const double *ws, double *z, int64_t N1, int64_t N2, int64_t b, int twiddle)
{
    if (!digit_shape_ok(N1, b) || !digit_shape_ok(N2, b)) return -1;
    int64_t N = N1 * N2;
    roots_t t;
    if (twiddle && roots_init(&t, N)) return -2;
    for (int64_t a = 0; a < N1; ++a) {
        int64_t v = oracle_digit_reverse_n(a, b, N1);
        for (int64_t c = 0; c < N2; ++c) {
            int64_t u = oracle_digit_reverse_n(c, b, N2);
            double xr = ws[2 * (a * N2 + c)], xi = ws[2 * (a * N2 + c) + 1];
            double outr = xr, outi = xi;
            if (twiddle) {
                double wr, wi;
                roots_get(&t, (v * c) % N, &wr, &wi);
                outr = xr * wr - xi * wi;
                outi = xr * wi + xi * wr;
            }
            z[2 * (u * N1 + v)] = outr;
            z[2 * (u * N1 + v) + 1] = outi;
        }
    }
    if (twiddle) roots_free(&t);
    return 0;
}

/* Phase III, input layout B_{m2} (x) I_{N1} (Lemma 1; appendix A.8):
 * physical row u of column v holds logical input j2 = pi_{m2}(u);
 *   Y[k2,v] = sum_{j2} Zhat[pi_{m2}(j2), v] w_{N2}^{-k2*j2},
 * natural-order output.  z: N2 x N1 row-major.  Only the ncols columns v
 * listed in cols are formed (cols == NULL: all N1); out is N2 x ncols
 * row-major, out[k2*ncols + i] = Y[k2, cols[i]]. */
int oracle_phase3(const double *z, int64_t N1, int64_t N2, int64_t b,
                  const int64_t *cols, int64_t ncols, double *out)
{
    if (!digit_shape_ok(N2, b) || N1 < 1) return -1;
    if (!cols) ncols = N1;
    double *col = (double *)malloc(sizeof(double) * 2 * (size_t)N2);
    double *dft = (double *)malloc(sizeof(double) * 2 * (size_t)N2);
    if (!col || !dft) { free(col); free(dft); return -2; }
    int rc = 0;
    for (int64_t i = 0; i < ncols && rc == 0; ++i) {
        int64_t v = cols ? cols[i] : i;
        if (v < 0 || v >= N1) { rc = -1; break; }
        for (int64_t j2 = 0; j2 < N2; ++j2) {
            int64_t u = oracle_digit_reverse_n(j2, b, N2);
            col[2 * j2] = z[2 * (u * N1 + v)];
            col[2 * j2 + 1] = z[2 * (u * N1 + v) + 1];
        }
        rc = oracle_dft(col, dft, N2);
        for (int64_t k2 = 0; k2 < N2; ++k2) {
            out[2 * (k2 * ncols + i)] = dft[2 * k2];
            out[2 * (k2 * ncols + i) + 1] = dft[2 * k2 + 1];
        }
    }
    free(col);
    free(dft);
    return rc;
}
