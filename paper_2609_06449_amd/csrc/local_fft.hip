// LocalFFT passes (paper, section 4.1 and appendix A) for gfx950.
//
// A workgroup transforms T contiguous columns of an n-row tile (n <= 4096)
// entirely on chip.  The transform is a radix-16 Stockham sequence (one
// radix-2/4/8 stage when log2 n is not a multiple of 4): every thread holds
// E = min(16, n) items in registers; the first stage reads its operands
// straight from HBM rows, the last stage writes its results straight to HBM
// rows, and only the exchanges between stages go through LDS.
//
// The arithmetic order inside a workgroup is free (Lemma 1 of the paper holds
// for any digit-aligned split); what the paper fixes is the layout at the HBM
// boundary, which the pass descriptor states: Phase I writes the item of
// logical frequency k to row pi(k) (output layout P_pi Omega), Phase III reads
// logical input j from row pi(j) (input layout Omega P_pi).  Rows are
// contiguous runs of T items, so a digit-reversed row order costs nothing.
//
// One tile per workgroup of up to 1024 threads.  Stage twiddles come from
// small factor tables copied to LDS by each workgroup (broadcast or
// contiguous reads).  Two kernel families share the stage code:
//  * fast: one HBM pass of a single-pass Phase I or Phase III with b in
//    {2, 4, 16}; the tile width is a compile-time constant (LDS addresses fold
//    to immediates) and the digit reversal of the 16 rows a thread touches
//    costs one reversal per thread, by the composition identity
//    pi(r*2^L + j) = pi(j)*2^LR + pi(r) (appendix A.8) with pi(r) a constant;
//  * generic: any pass descriptor (two-pass steps, pre-twiddles, any b).
#include "local_fft_kernels.h"

namespace paco {
namespace {

bool pass_needs_gen(const LocalPass &p)
{
    return (p.in_ell && !digrev_fast(p.in_t)) || (p.out_ell && !digrev_fast(p.out_t)) ||
           (p.tw_ell && !digrev_fast(p.tw_t));
}

}  // namespace

int32_t choose_log2T(int32_t log2n, int64_t ncols)
{
    // 4096 items per workgroup for short transforms, at least 4 columns
    // (32-byte row runs) for long ones; never more columns than exist.
    int32_t lt = 12 - log2n;
    if (lt < 2) lt = 2;
    int32_t lc = 0;
    while ((int64_t(1) << (lc + 1)) <= ncols) ++lc;
    return lt < lc ? lt : lc;
}

const void *fast_kernel_fp32(int log2n, int mode, int tb, int groups)
{
    return fast_kernel_t<kPrecFP32>(log2n, mode, tb, groups);
}
const void *generic_kernel_fp32(int log2n, bool pre, bool gen) { return generic_kernel_t<kPrecFP32>(log2n, pre, gen); }

// The butterfly stages of the split forms differ only for lengths with a
// radix-16 stage (n >= 16); shorter transforms use the FP32 kernels.
const void *fast_kernel(int prec, int log2n, int mode, int tb, int groups)
{
    if (log2n >= 4) {
        if (prec == kPrecFP16x3) return fast_kernel_fp16x3(log2n, mode, tb, groups);
        if (prec == kPrecBF16x3) return fast_kernel_bf16x3(log2n, mode, tb, groups);
        if (prec == kPrecBF16x6) return fast_kernel_bf16x6(log2n, mode, tb, groups);
    }
    return fast_kernel_fp32(log2n, mode, tb, groups);
}

const void *kernel_for(int prec, int log2n, bool pre, bool gen)
{
    if (log2n >= 4) {
        if (prec == kPrecFP16x3) return generic_kernel_fp16x3(log2n, pre, gen);
        if (prec == kPrecBF16x3) return generic_kernel_bf16x3(log2n, pre, gen);
        if (prec == kPrecBF16x6) return generic_kernel_bf16x6(log2n, pre, gen);
    }
    return generic_kernel_fp32(log2n, pre, gen);
}

int32_t local_fft_fast_mode(const LocalPass &p)
{
    // single-pass Phase I (pi on output rows) or Phase III (pi on input rows)
    if (p.pre_tw || p.n_outer != 1 || p.o_in || p.o_out || p.j_in != 1 || p.k_out != 1) return -1;
    if (p.in_s || p.out_s) return -1;  // mixed-radix row maps: generic kernel
    // tile width: the split forms' operand-layout tile (16^s points, one
    // group) has its own (mf_log2T); every other fast tile fast_tile_log2T
    const bool mf = p.prec != 0 && p.log2n >= 4 && p.log2n % 4 == 0 && p.groups < 2;
    const int want = mf ? mf_log2T(p.log2n, p.out_tr ? 2 : 0)
                        : fast_tile_log2T(p.log2n, p.groups >= 2 ? 2 : 1, p.groups == 3 ? 32 : 16);
    if (p.log2T != want) return -1;
    int mode = -1, tb = 0;
    if (p.top_tw) {
        if (p.in_ell || p.out_ell || p.out_tr) return -1;
        mode = 3;
        tb = 1;
    } else if (p.out_tr) {
        if (p.in_ell || p.out_ell) return -1;
        mode = p.src_last ? 4 : 2;
        tb = 1;
    } else {
        if (p.out_ell && !p.in_ell) { mode = 0; tb = p.out_t; }
        if (p.in_ell && !p.out_ell) { mode = 1; tb = p.in_t; }
    }
    if (mode < 0 || !fast_kernel(p.prec, p.log2n, mode, tb, p.groups)) return -1;
    return mode;
}

LocalLaunch local_fft_geometry(const LocalPass &p)
{
    const bool fast = !p.no_fast && local_fft_fast_mode(p) >= 0;
    const bool grouped = fast && p.groups >= 2;
    const int EG = (fast && p.groups == 3) ? 32 : (p.log2n < 4 ? (1 << p.log2n) : 16);
    const int64_t items = int64_t(1) << (p.log2n + p.log2T - (grouped ? 1 : 0));  // one LDS group
    const int64_t twn = (stage_tw_total(p.log2n) + 63) & ~63;
    LocalLaunch g;
    g.threads = int(items / EG);
    g.lds_bytes = size_t(twn + items + ((items >> 6) << 2) + 4) * sizeof(float2);
    g.tiles = p.n_outer * (p.ncols >> p.log2T);
    return g;
}

hipError_t local_fft_prepare()
{
    for (int prec = 0; prec < 4; ++prec)
    for (int l = 1; l <= kMaxOnChipLog2; ++l) {
        for (int v = 0; v < 4; ++v) {
            hipError_t e = hipFuncSetAttribute(kernel_for(prec, l, v & 1, v & 2),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e != hipSuccess) return e;
        }
        for (int mode = 0; mode < 5; ++mode)
            for (int tb : {1, 2, 4})
                for (int grp : {1, 2, 3}) {
                const void *k = fast_kernel(prec, l, mode, tb, grp);
                if (!k) continue;
                hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
                if (e != hipSuccess) return e;
            }
    }
    return hipSuccess;
}

hipError_t launch_local_fft(const LocalPass &p, hipStream_t s)
{
    const int mode = p.no_fast ? -1 : local_fft_fast_mode(p);
    const void *k = mode >= 0 ? fast_kernel(p.prec, p.log2n, mode, mode >= 2 ? 1 : (mode == 0 ? p.out_t : p.in_t), p.groups)
                              : kernel_for(p.prec, p.log2n, p.pre_tw != 0, pass_needs_gen(p));
    if (!k) return hipErrorInvalidValue;
    const LocalLaunch g = local_fft_geometry(p);
    if (g.tiles < 1 || g.tiles > 0x7fffffff) return hipErrorInvalidValue;
    if (mode < 0 && g.threads > generic_max_threads(p.prec)) return hipErrorInvalidValue;
    void *args[] = {const_cast<LocalPass *>(&p)};
    return hipLaunchKernel(k, dim3(unsigned(g.tiles)), dim3(unsigned(g.threads)), args, g.lds_bytes, s);
}

}  // namespace paco
