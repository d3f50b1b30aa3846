// LocalFFT kernels (generic descriptor-driven pass and fast single-pass
// tiles) and their dispatch tables, templated on the butterfly arithmetic
// PREC.  Each arithmetic form is instantiated in its own translation unit
// (local_fft.hip: FP32; local_fft_fp16x3.hip, local_fft_bf16x3.hip,
// local_fft_bf16x6.hip: the split MFMA forms) so they compile in parallel.
#pragma once

#include "stages.h"

namespace paco {
namespace {

// Generic pass: any descriptor, runtime tile width (at most
// generic_max_threads(PREC) threads: the split MFMA forms' butterflies need
// more registers, so their tiles are kept to 512 threads).
template <int LOG2N, bool PRE, bool GEN, int PREC>
__global__ __launch_bounds__(generic_max_threads(PREC)) void local_fft_kernel(LocalPass P)
{
    constexpr int EG = LOG2N < 4 ? (1 << LOG2N) : 16;
    constexpr int LR0 = stage_log2radix(LOG2N, 0);
    constexpr int R0 = 1 << LR0;
    constexpr int NB0 = EG / R0;
    constexpr int LNR0 = LOG2N - LR0;
    constexpr int TWN = stage_tw_total(LOG2N);
    extern __shared__ float2 smem[];
    const int log2T = P.log2T;
    const int Tm = (1 << log2T) - 1;
    const int tid = threadIdx.x, nt = blockDim.x;
    float2 *twl = smem;
    float2 *lds = smem + ((TWN + 63) & ~63);

    const int64_t ntc = P.ncols >> log2T;
    const int64_t tile = tile_order(blockIdx.x, gridDim.x);
    const int64_t o = tile / ntc;
    const int64_t col0 = (tile - o * ntc) << log2T;
    const char *src = reinterpret_cast<const char *>(P.src + col0);
    const uint32_t orow = uint32_t(o * P.o_in), ld8 = uint32_t(P.ld) * 8u, j_in = uint32_t(P.j_in);

    float2 v[EG];
#pragma unroll
    for (int q = 0; q < NB0; ++q) {
        const int g = tid + q * nt;
        const int t = g & Tm, j = g >> log2T;
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const uint32_t jj = j + (r << LNR0);
            const uint32_t m = uint32_t(digmap<GEN>(jj, P.in_t, P.in_ell, P.in_s, false));
            v[q * R0 + r] = *reinterpret_cast<const float2 *>(src + ((orow + m * j_in) * ld8 + uint32_t(t) * 8u));
        }
    }
    if (P.conj_in) {  // the inverse transform's input map
#pragma unroll
        for (int k = 0; k < EG; ++k) v[k].y = -v[k].y;
    }
    // the stage twiddle table is copied after the data loads are issued, so
    // waiting for it does not delay them
    copy_twiddles(twl, P.stw, TWN, tid, nt);
    if constexpr (PRE) {
        const int64_t f = digmap<GEN>(o, P.tw_t, P.tw_ell, P.tw_s, false);
        const int64_t Mm = (int64_t(1) << P.log2M) - 1;
        const int shM = P.log2L - P.log2M;
#pragma unroll
        for (int q = 0; q < NB0; ++q) {
            const int j = (tid + q * nt) >> log2T;
#pragma unroll
            for (int r = 0; r < R0; ++r)
                v[q * R0 + r] = cmul(v[q * R0 + r], P.tw[((f * (j + (r << LNR0))) & Mm) << shM]);
        }
    }
    Ctx c;
    c.lds = lds;
    c.twl = twl;
    c.tid = tid;
    c.nt = nt;
    c.log2T = log2T;
    c.dst = reinterpret_cast<char *>(P.dst + col0);
    c.ld8 = ld8;
    c.orow_out = uint32_t(o * P.o_out);
    c.k_out = uint32_t(P.k_out);
    c.out_t = P.out_t;
    c.out_ell = P.out_ell;
    c.out_s = P.out_s;
    c.act = true;
    c.oscale = P.out_scale;
    run_stage<LOG2N, 0, EG, -1, -1, 1, GEN, 1, false, PREC>(v, c);
}

template <int LOG2N, int MODE, int TB, int H, int EG, int PREC>
__global__ __launch_bounds__(fast_threads(LOG2N, H, EG)) void local_fft_fast_kernel(LocalPass P)
{
    constexpr int LT = fast_tile_log2T(LOG2N, H, EG);
    extern __shared__ float2 smem[];
    const int64_t col0 = tile_order(blockIdx.x, gridDim.x) << LT;
    TopTw top;
    if constexpr (MODE == 3) {
        top.hi = P.top_hi;
        top.lo = P.top_lo;
        top.cw = P.top_cw;
        top.cmask = uint32_t(16 * P.ncols - 1);
        top.nmask = uint32_t((uint64_t(1) << P.top_log2N) - 1);
        top.lomask = (1u << P.top_log2Lo) - 1;
        top.lshift = P.top_log2Lo;
    }
    // MODE 2 streams the packed buffer out (Phase II reads it back in 1 KB
    // runs); the two-pass form's MODE 4 keeps plain stores, its Phase III
    // reads that buffer in column tiles and finds it in the MALL
    // (streaming there measured 160 -> 180 us per 2^24 transform, against
    // 194 -> 177 us for the packed three-pass form)
    fast_tile<LOG2N, MODE, TB, H, EG, LT, false, PREC>(P.src, P.dst, uint32_t(P.ld), col0, P.stw, smem, threadIdx.x,
                                                       &top, P.conj_in != 0, P.out_scale, MODE == 2);
}

// Single-pass tile of a 16^s-point transform with every butterfly on MFMA in
// the operand layout (the split forms' fast kernel for those lengths).
template <int LOG2N, int MODE, int TB, int PREC>
__global__ __launch_bounds__((1 << (LOG2N + mf_log2T(LOG2N, MODE))) / 16) void local_fft_mf_kernel(LocalPass P)
{
    constexpr int LT = mf_log2T(LOG2N, MODE);
    extern __shared__ float2 smem[];
    const int64_t col0 = tile_order(blockIdx.x, gridDim.x) << LT;
    mf_tile<LOG2N, MODE, TB, PREC, LT>(P.src, P.dst, uint32_t(P.ld), col0, P.stw, smem, threadIdx.x, P.conj_in != 0,
                                       P.out_scale);
}

template <int L, bool PRE, bool GEN, int PREC>
const void *kptr()
{
    return reinterpret_cast<const void *>(&local_fft_kernel<L, PRE, GEN, PREC>);
}

template <bool PRE, bool GEN, int PREC>
const void *kernel_for_pre(int log2n)
{
    switch (log2n) {
    case 1: return kptr<1, PRE, GEN, PREC>();
    case 2: return kptr<2, PRE, GEN, PREC>();
    case 3: return kptr<3, PRE, GEN, PREC>();
    case 4: return kptr<4, PRE, GEN, PREC>();
    case 5: return kptr<5, PRE, GEN, PREC>();
    case 6: return kptr<6, PRE, GEN, PREC>();
    case 7: return kptr<7, PRE, GEN, PREC>();
    case 8: return kptr<8, PRE, GEN, PREC>();
    case 9: return kptr<9, PRE, GEN, PREC>();
    case 10: return kptr<10, PRE, GEN, PREC>();
    case 11: return kptr<11, PRE, GEN, PREC>();
    case 12: return kptr<12, PRE, GEN, PREC>();
    default: return nullptr;
    }
}

template <int L, int TB, int H, int EG, int PREC>
const void *fast_for_tb(int mode)
{
    // (the split MFMA forms have no 32-item tile: their scratch and operands
    // would not fit the registers)
    if constexpr (L % TB != 0 || (H == 2 && L < 10) || (L < 4 && EG != (1 << L)) || (L >= 4 && EG < 16) ||
                  (EG == 32 && H != 2) || (EG == 32 && PREC != kPrecFP32)) {
        return nullptr;
    } else if constexpr (PREC != kPrecFP32 && L % 4 == 0 && H == 1 && EG == 16) {
        if (mode == 3 || mode == 4) return nullptr;
        if (mode == 2) return TB == 1 ? reinterpret_cast<const void *>(&local_fft_mf_kernel<L, 2, 1, PREC>) : nullptr;
        return mode == 0 ? reinterpret_cast<const void *>(&local_fft_mf_kernel<L, 0, TB, PREC>)
                         : reinterpret_cast<const void *>(&local_fft_mf_kernel<L, 1, TB, PREC>);

    } else {
        if (mode == 3 || mode == 4) {  // the two-pass form's Phase III and Phase I: FP32 only
            if constexpr (TB == 1 && PREC == kPrecFP32)
                return mode == 3 ? reinterpret_cast<const void *>(&local_fft_fast_kernel<L, 3, 1, H, EG, PREC>)
                                 : reinterpret_cast<const void *>(&local_fft_fast_kernel<L, 4, 1, H, EG, PREC>);
            return nullptr;
        }
        if (mode == 2) return TB == 1 ? reinterpret_cast<const void *>(&local_fft_fast_kernel<L, 2, 1, H, EG, PREC>) : nullptr;
        return mode == 0 ? reinterpret_cast<const void *>(&local_fft_fast_kernel<L, 0, TB, H, EG, PREC>)
                         : reinterpret_cast<const void *>(&local_fft_fast_kernel<L, 1, TB, H, EG, PREC>);
    }
}

template <int L, int H, int EG, int PREC>
const void *fast_for_len(int mode, int tb)
{
    switch (tb) {
    case 1: return fast_for_tb<L, 1, H, EG, PREC>(mode);
    case 2: return fast_for_tb<L, 2, H, EG, PREC>(mode);
    case 4: return fast_for_tb<L, 4, H, EG, PREC>(mode);
    default: return nullptr;
    }
}

template <int H, int EGW, int PREC>
const void *fast_kernel_h(int log2n, int mode, int tb)
{
    // EGW: 0 = the natural per-thread width min(16, n), 32 = wide
    switch (log2n) {
    case 4: return fast_for_len<4, H, EGW ? EGW : 16, PREC>(mode, tb);
    case 5: return fast_for_len<5, H, EGW ? EGW : 16, PREC>(mode, tb);
    case 6: return fast_for_len<6, H, EGW ? EGW : 16, PREC>(mode, tb);
    case 7: return fast_for_len<7, H, EGW ? EGW : 16, PREC>(mode, tb);
    case 8: return fast_for_len<8, H, EGW ? EGW : 16, PREC>(mode, tb);
    case 9: return fast_for_len<9, H, EGW ? EGW : 16, PREC>(mode, tb);
    case 10: return fast_for_len<10, H, EGW ? EGW : 16, PREC>(mode, tb);
    case 11: return fast_for_len<11, H, EGW ? EGW : 16, PREC>(mode, tb);
    case 12: return fast_for_len<12, H, EGW ? EGW : 16, PREC>(mode, tb);
    default: return nullptr;
    }
}

// groups: 1, 2 (two 16-item groups) or 3 (two 32-item groups: tile twice as wide)
template <int PREC>
const void *fast_kernel_t(int log2n, int mode, int tb, int groups)
{
    if (groups == 3) return fast_kernel_h<2, 32, PREC>(log2n, mode, tb);
    return groups == 2 ? fast_kernel_h<2, 0, PREC>(log2n, mode, tb) : fast_kernel_h<1, 0, PREC>(log2n, mode, tb);
}

template <int PREC>
const void *generic_kernel_t(int log2n, bool pre, bool gen)
{
    if (gen) return pre ? kernel_for_pre<true, true, PREC>(log2n) : kernel_for_pre<false, true, PREC>(log2n);
    return pre ? kernel_for_pre<true, false, PREC>(log2n) : kernel_for_pre<false, false, PREC>(log2n);
}

}  // namespace
}  // namespace paco
