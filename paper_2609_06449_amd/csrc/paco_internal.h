// Internal declarations shared by the PACO HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "addr.h"

namespace paco {

// Complex product with an explicit fused multiply-add in each component:
// with a plain a*b - c*d the compiler may fuse either product, and its choice
// depends on the surrounding code, so two kernels doing the same arithmetic
// could round differently.  Every kernel multiplies through this function.
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}

// Largest transform length one local pass keeps on chip (LDS + registers).
constexpr int kMaxOnChipLog2 = 12;

// ---------------------------------------------------------------------------
// Stage plan of an on-chip transform of length n = 2^l: radix-16 Stockham
// stages, then one radix-2^(l mod 4) stage when l is not a multiple of 4.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int stage_count(int l) { return l / 4 + (l % 4 ? 1 : 0); }
__host__ __device__ constexpr int stage_log2radix(int l, int s) { return s < l / 4 ? 4 : l % 4; }
__host__ __device__ constexpr int stage_log2ns(int l, int s)
{
    int a = 0;
    for (int i = 0; i < s; ++i) a += stage_log2radix(l, i);
    return a;
}

// Stage twiddles w_M^{-k r} (M = Ns*R, k < Ns, 1 <= r < R) are stored as two
// factor tables per stage S >= 1, indexed (r-1, .):
//   lo[r-1][kl] = w_M^{-kl*r},       kl < min(Ns, 16)
//   hi[r-1][kh] = w_M^{-16*kh*r},    kh < Ns/16        (only when Ns > 16)
// with k = 16*kh + kl, so w_M^{-k r} = hi * lo.  Lanes of a wave hold
// consecutive k, so every table read is a broadcast or a contiguous run.
__host__ __device__ constexpr int stage_lo_width(int l, int s)
{
    return (1 << stage_log2ns(l, s)) < 16 ? (1 << stage_log2ns(l, s)) : 16;
}
__host__ __device__ constexpr int stage_hi_width(int l, int s)
{
    return (1 << stage_log2ns(l, s)) > 16 ? (1 << stage_log2ns(l, s)) / 16 : 0;
}
__host__ __device__ constexpr int stage_tw_size(int l, int s)
{
    return s == 0 ? 0 : ((1 << stage_log2radix(l, s)) - 1) * (stage_lo_width(l, s) + stage_hi_width(l, s));
}
__host__ __device__ constexpr int stage_tw_offset(int l, int s)
{
    int a = 0;
    for (int i = 1; i < s; ++i) a += stage_tw_size(l, i);
    return a;
}
__host__ __device__ constexpr int stage_tw_total(int l) { return stage_tw_offset(l, stage_count(l)); }

// Tile width of the fast kernels: 4096 items per workgroup for short
// transforms, 4 columns (32-byte row runs) for long ones.
__host__ __device__ constexpr int fast_log2T(int l) { return l >= 10 ? 2 : 12 - l; }

// Columns (log2) of the split forms' operand-layout tile (mode 2: the
// transposed store of Phase I): a 4096-point Phase I takes 2 columns (512
// threads, half the LDS, so two workgroups per CU overlap each other;
// measured 18-20% faster than one 4-column workgroup per CU); every other
// tile keeps fast_log2T columns (a 2-column row store, 16-byte runs, is
// slower).
__host__ __device__ constexpr int mf_log2T(int l, int mode) { return (mode == 2 && l == 12) ? 1 : fast_log2T(l); }

// Largest workgroup of the generic local-FFT kernel for butterfly
// arithmetic prec (0: FP32 VALU; the split MFMA forms get 512 threads and
// with them 256 VGPRs per lane).
__host__ __device__ constexpr int generic_max_threads(int prec) { return prec == 0 ? 1024 : 512; }

// One HBM pass of a batched local FFT: the GPU form of a digit-field view
// (paper, appendix A.3-A.4).  The pass has n_outer * (ncols / T) independent
// tiles; tile (o, c) transforms the T contiguous columns [c*T, c*T + T) of
// the rows
//     input  row of logical j : o*o_in  + pi_in(j)  * j_in
//     output row of logical k : o*o_out + pi_out(k) * k_out
// where pi_in / pi_out are base-2^t digit reversals over ell digits
// (ell = 0: identity), with an extra short digit of s bits on top in the
// mixed-radix case (digmap: pi_in forward, pi_out inverse).  A row is ld complex64 items long; the column field C
// of the paper's view is the run of T items every access reads or writes
// whole.  With pre_tw set, input j of tile o is first scaled by the
// Cooley-Tukey twiddle w_M^{-f(o)*j}, f(o) = pi_tw(o) (the layout-aware
// twiddle of appendix A.2).
struct LocalPass {
    const float2 *src;
    float2 *dst;
    int64_t ld;            // row length (items)
    int64_t ncols;         // columns transformed: [0, ncols)
    int32_t log2n;         // transform length n = 2^log2n (<= 2^kMaxOnChipLog2)
    int32_t log2T;         // columns per workgroup
    int64_t n_outer;       // outer batch count
    int64_t o_in, j_in;    // input row strides
    int64_t o_out, k_out;  // output row strides
    int32_t in_t, in_ell, in_s;     // pi_in = digmap(., in_t, in_ell, in_s, forward)
    int32_t out_t, out_ell, out_s;  // pi_out = digmap(., out_t, out_ell, out_s, inverse)
    const float2 *stw;     // stage twiddle tables of length n (stage_tw_total entries)
    const float2 *tw;      // w_L^{-r}, r < L = 2^log2L (pre-twiddle)
    int32_t log2L;
    int32_t pre_tw;        // 0: none; 1: w_M^{-f(o) j} before the DFT
    int32_t log2M;         // M of the pre-twiddle (M <= L)
    int32_t tw_t, tw_ell, tw_s;  // f(o) = digmap(o, tw_t, tw_ell, tw_s, forward)
    int32_t no_fast;       // 1: always use the generic kernel (testing)
    int32_t out_tr;        // 1: write the output transposed (row = column, n items; fast kernel only)
    int32_t src_last;      // with out_tr: the source is read for the last time (non-temporal loads)
    int32_t groups;        // fast kernel: 1, or 2 column groups taking turns in LDS
    int32_t prec;          // radix-16 butterflies: 0 FP32 VALU, 1 FP16x3, 2 BF16x3, 3 BF16x6 (MFMA)
    // top-level twiddle on load (the two-pass form of Phase III): input item
    // (row j, column v) is scaled by w_N^{-(v j mod N)}, N = 2^top_log2N,
    // from the two-level tables top_hi / top_lo (split at 2^top_log2Lo) and
    // top_cw[k] = w_{16 ncols}^{-k}, k < 16 ncols (see TopTw)
    int32_t top_tw;
    int32_t top_log2N, top_log2Lo;
    const float2 *top_hi, *top_lo, *top_cw;
    // the inverse transform as conj(Omega conj(y)) / N: conj_in negates the
    // imaginary part of every item the pass loads; out_scale != 0 stores
    // conj(item) * out_scale
    int32_t conj_in;
    float out_scale;
};

// Phase II: out[pi2(c)*N1 + v] = ws[pi1(v)*N2 + c] * w_N^{-(v*c mod N)}, the
// fused middle permutation (section 3.3) indexed by v = pi_{m1}(a).  With
// v = v0 + vi and c = c0 + ci inside a TV x TC tile,
//   w_N^{-v c} = w_N^{-v0 c} * w_N^{-vi c0} * w_N^{-vi ci}
// the first factor per thread (tw_hi/tw_lo two-level table), the second per
// tile row, the third from a fixed 128 x 128 table (tw_tile, symmetric,
// [i*128 + j] = w_N^{-(i*j mod N)}).
struct MiddlePass {
    const float2 *ws;
    float2 *out;
    int64_t N1, N2;
    int32_t t, m1, m2;        // b = 2^t, N1 = b^m1 2^s1, N2 = b^m2 2^s2
    int32_t s1, s2;           // short top digit (mixed-radix sizes; 0: N_i = b^m_i)
    const float2 *tw_hi;      // w_N^{-h*Lo}, h < N/Lo
    const float2 *tw_lo;      // w_N^{-l}, l < Lo
    const float2 *tw_tile;    // [i*128 + j] = w_N^{-(i*j mod N)}, i, j < 128
    int32_t log2N, log2Lo;
    int32_t twiddle;          // 0: bare permutation
    int32_t packed;           // 1: ws is the transposed natural buffer ws[c*N1 + v] = A[v, c]
};

constexpr int kMidTile = 64;

// The split form (split.hip), FP32, N1 = 16 M (M = 2^8, 2^9, 2^10): pass 1
// runs the first radix-16 stage of every Phase I column transform (with its
// twiddle) over whole 128-byte row runs of x and stores ws[c*N1 + 16 j + k0];
// pass 2 finishes each column's 16 transforms of length M and applies the
// redistribution of Phase II (row c -> row pi_{m2}(c) of out, times
// w_N^{-k1 c}) in the same pass.
constexpr int kSplitLog2N1 = 12;
struct SplitPass {
    const float2 *src;
    float2 *dst;
    int64_t N1, N2;
    const float2 *tw;             // w_L^{-r}, r < L = N1 << tw_shift: w_{N1}^{-m} = tw[m << tw_shift]
    int32_t tw_shift;
    const float2 *tw_hi, *tw_lo;  // w_N^{-e} = tw_hi[e >> log2Lo] * tw_lo[e mod 2^log2Lo]
    int32_t log2N, log2Lo;
    int32_t t, m2, s2;            // pi_{m2}(c) = digmap(c, t, m2, s2, forward)
    int32_t conj_in;              // pass 1: conjugate x on load (the inverse transform's input map)
};
constexpr int kTwTile = 128;  // tile-twiddle table side: [i*128 + j] = w_N^{-(i*j mod N)}

// The symmetric split form (sym.hip), N1 = N2 = 16 L, L = 256, 512, 1024
// (the split MFMA forms: L = 256): Lemma 1 once more on both local phases,
// with the 16-point children next to the redistribution.
//   Phase I:   j1 = 16 j + r,  k1 = k + L s;
//   Phase III: j2 = jc + L rr, k2 = q0 + 16 q.
//   pass 1: U[c][r][k] = w_N1^{-k r} sum_j X[16 j + r, c] w_L^{-k j}
//           -> ws[((k >> 4) N2 + c) 256 + 16 r + (k & 15)]
//   pass 2: A[k + L s, c] = sum_r w_16^{-s r} U[c][r][k];
//           Z[v, c] = A[v, c] w_N^{-v c};
//           W[v][jc][q0] = w_N2^{-q0 jc} sum_rr Z[v, jc + L rr] w_16^{-q0 rr}
//           -> out[(16 jc + q0) N1 + v]
//   pass 3: Y[q0 + 16 q, v] = sum_jc w_L^{-q jc} W[v][jc][q0]
//           -> out[(q0 + 16 q) N1 + v], in place (a tile reads and writes the
//           same rows {q0 + 16 t})
constexpr int kSymLog2N = 12;  // the smallest side of the symmetric split form (L = 256)
struct SymPass {
    const float2 *src;
    float2 *dst;
    int64_t N1, N2;
    const float2 *tw;             // w_L^{-r}, r < L = 2^log2L (L >= N1, N2)
    int32_t log2L;
    const float2 *tw_hi, *tw_lo;  // w_N^{-e} = tw_hi[e >> log2Lo] * tw_lo[e mod 2^log2Lo]
    int32_t log2N, log2Lo;
    const float2 *tw_sj;          // [s N2/16 + j] = w_{16 N2}^{-s j}, s < 16, j < N2 / 16
    const float *w16;             // split MFMA forms: 64 lanes x 16 DFT-matrix operands (w16_operands)
    int32_t conj_in;              // pass 1: conjugate x on load (the inverse's input map)
    float out_scale;              // pass 3: nonzero stores conj(y) * out_scale (the inverse's output map)
    uint32_t resident1, resident3;  // passes 1 and 3 at L >= 512: workgroups of their persistent launches
                                    // (sym_resident_groups; 0: one per tile)
    uint32_t resident2;             // pass 2 of the wide form (N2 = 2^15), likewise
};

// Workgroup geometry a local pass is launched with.
struct LocalLaunch {
    int threads;       // per workgroup
    size_t lds_bytes;  // dynamic LDS per workgroup
    int64_t tiles;     // column tiles in the pass
};

// Thread-local detail string returned by paco_last_error (plan.hip).
void set_last_error(const std::string &msg);

// ---- host tables (tables.hip) -------------------------------------------
// w_M^{-r} = exp(-2 pi i r / M) from the exact integer r, in FP64, rounded
// once to FP32.
float2 root_neg(int64_t r, int64_t M);
// Stage twiddle factor tables of every on-chip length 2^1 .. 2^12,
// concatenated; off[l] is the first entry of length 2^l.
bool stage_tables(std::vector<float2> &stw, int64_t off[kMaxOnChipLog2 + 1]);
// Phase-II tables of N = 2^lN: w_N^{-h*Lo} (hi), w_N^{-l} (lo) with
// Lo = 2^middle_log2lo(lN), and the 128 x 128 tile table.
constexpr int middle_log2lo(int lN) { return (lN + 1) / 2; }
void middle_tables(int lN, std::vector<float2> &hi, std::vector<float2> &lo, std::vector<float2> &tile);

// Kernel tables of the split MFMA forms (local_fft_fp16x3.hip,
// local_fft_bf16x3.hip, local_fft_bf16x6.hip); nullptr where no kernel exists.
const void *fast_kernel_fp16x3(int log2n, int mode, int tb, int groups);
const void *fast_kernel_bf16x3(int log2n, int mode, int tb, int groups);
const void *fast_kernel_bf16x6(int log2n, int mode, int tb, int groups);
const void *generic_kernel_fp16x3(int log2n, bool pre, bool gen);
const void *generic_kernel_bf16x3(int log2n, bool pre, bool gen);
const void *generic_kernel_bf16x6(int log2n, bool pre, bool gen);

LocalLaunch local_fft_geometry(const LocalPass &p);
hipError_t local_fft_prepare();  // raises the dynamic-LDS limit of every kernel once
hipError_t launch_local_fft(const LocalPass &p, hipStream_t s);
hipError_t launch_middle(const MiddlePass &p, hipStream_t s);
// Pass 1 and pass 2 of the split form; hipErrorInvalidValue unless N1 is
// 2^12, 2^13 or 2^14 and N2 is a multiple of 16.
hipError_t launch_split_first(const SplitPass &p, hipStream_t s);
hipError_t launch_split_middle(const SplitPass &p, hipStream_t s);
hipError_t split_prepare();  // raises the dynamic-LDS limit of the three-stage pass 2 once
// The three passes of the symmetric split form; hipErrorInvalidValue unless
// sym_log2_child(p) is nonzero.
// The child sizes of a shape the symmetric form runs, or false: L1 = N1/16
// and L2 = N2/R as log2 ll1, ll2 (8, 9 or 10 each), and lr2 = log2 R, the
// radix of pass 2's Phase III child: 4 for N1, N2 in {2^12, 2^13, 2^14}, 5
// (the wide form) for N2 = 2^15 with N1 = 2^12 or 2^13.
bool sym_children(const SymPass &p, int &ll1, int &ll2, int &lr2);
// log2 L of a square shape the symmetric form runs (N1 = N2 = 16 L; the
// split MFMA forms run L = 256 and 512), else 0
int sym_log2_child(const SymPass &p);
// Workgroups the current device holds at once of the persistent pass-1 or
// pass-3 kernel of p's shape (L >= 512) or of the wide form's pass 2, 0 for
// the other passes or if the runtime does not say; the MFMA forms' kernels:
// sym_mf_resident_groups.
uint32_t sym_resident_groups(int pass, const SymPass &p);
uint32_t sym_mf_resident_groups(int prec, int pass, const SymPass &p);
hipError_t launch_sym_first(const SymPass &p, hipStream_t s);
hipError_t launch_sym_middle(const SymPass &p, hipStream_t s);
hipError_t launch_sym_last(const SymPass &p, hipStream_t s);
// Pass 1, 2 or 3 of the symmetric split form with the radix-16 butterflies
// on MFMA in split form prec (kPrecFP16x3, kPrecBF16x3, kPrecBF16x6; sym_mf.hip).
hipError_t launch_sym_mf(int prec, int pass, const SymPass &p, hipStream_t s);
// The radix-16 DFT-matrix operands of every MFMA lane (64 x 16 floats).
void w16_operands(float *table);

// Columns per workgroup for an on-chip pass of length 2^log2n over ncols.
int32_t choose_log2T(int32_t log2n, int64_t ncols);
// Fast-kernel mode of a pass: 0 (Phase I rows), 1 (Phase III rows), 2
// (transposed natural output) or -1 when the pass needs the generic kernel.
int32_t local_fft_fast_mode(const LocalPass &p);

}  // namespace paco
