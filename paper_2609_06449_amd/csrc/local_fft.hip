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
#include "stages.h"

namespace paco {
namespace {

// Generic pass: any descriptor, runtime tile width.
template <int LOG2N, bool PRE, bool GEN>
__global__ __launch_bounds__(1024) void local_fft_kernel(LocalPass P)
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
            const uint32_t m = uint32_t(digrev<GEN>(jj, P.in_t, P.in_ell));
            v[q * R0 + r] = *reinterpret_cast<const float2 *>(src + ((orow + m * j_in) * ld8 + uint32_t(t) * 8u));
        }
    }
    // the stage twiddle table is copied after the data loads are issued, so
    // waiting for it does not delay them
    copy_twiddles(twl, P.stw, TWN, tid, nt);
    if constexpr (PRE) {
        const int64_t f = digrev<GEN>(o, P.tw_t, P.tw_ell);
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
    c.act = true;
    run_stage<LOG2N, 0, EG, -1, -1, 1, GEN, 1>(v, c);
}

template <int LOG2N, int MODE, int TB, int H, int EG>
__global__ __launch_bounds__(fast_threads(LOG2N, H, EG)) void local_fft_fast_kernel(LocalPass P)
{
    constexpr int LT = fast_tile_log2T(LOG2N, H, EG);
    extern __shared__ float2 smem[];
    const int64_t col0 = tile_order(blockIdx.x, gridDim.x) << LT;
    fast_tile<LOG2N, MODE, TB, H, EG, LT>(P.src, P.dst, uint32_t(P.ld), col0, P.stw, smem, threadIdx.x);
}

template <int L, bool PRE, bool GEN>
const void *kptr()
{
    return reinterpret_cast<const void *>(&local_fft_kernel<L, PRE, GEN>);
}

template <bool PRE, bool GEN>
const void *kernel_for_pre(int log2n)
{
    switch (log2n) {
    case 1: return kptr<1, PRE, GEN>();
    case 2: return kptr<2, PRE, GEN>();
    case 3: return kptr<3, PRE, GEN>();
    case 4: return kptr<4, PRE, GEN>();
    case 5: return kptr<5, PRE, GEN>();
    case 6: return kptr<6, PRE, GEN>();
    case 7: return kptr<7, PRE, GEN>();
    case 8: return kptr<8, PRE, GEN>();
    case 9: return kptr<9, PRE, GEN>();
    case 10: return kptr<10, PRE, GEN>();
    case 11: return kptr<11, PRE, GEN>();
    case 12: return kptr<12, PRE, GEN>();
    default: return nullptr;
    }
}

template <int L, int TB, int H, int EG>
const void *fast_for_tb(int mode)
{
    if constexpr (L % TB != 0 || (H == 2 && L < 10) || (L < 4 && EG != (1 << L)) || (L >= 4 && EG < 16) ||
                  (EG == 32 && H != 2)) {
        return nullptr;
    } else {
        if (mode == 2) return TB == 1 ? reinterpret_cast<const void *>(&local_fft_fast_kernel<L, 2, 1, H, EG>) : nullptr;
        return mode == 0 ? reinterpret_cast<const void *>(&local_fft_fast_kernel<L, 0, TB, H, EG>)
                         : reinterpret_cast<const void *>(&local_fft_fast_kernel<L, 1, TB, H, EG>);
    }
}

template <int L, int H, int EG>
const void *fast_for_len(int mode, int tb)
{
    switch (tb) {
    case 1: return fast_for_tb<L, 1, H, EG>(mode);
    case 2: return fast_for_tb<L, 2, H, EG>(mode);
    case 4: return fast_for_tb<L, 4, H, EG>(mode);
    default: return nullptr;
    }
}

template <int H, int EGW>
const void *fast_kernel_h(int log2n, int mode, int tb)
{
    // EGW: 0 = the natural per-thread width min(16, n), 32 = wide
    switch (log2n) {
    case 4: return fast_for_len<4, H, EGW ? EGW : 16>(mode, tb);
    case 5: return fast_for_len<5, H, EGW ? EGW : 16>(mode, tb);
    case 6: return fast_for_len<6, H, EGW ? EGW : 16>(mode, tb);
    case 7: return fast_for_len<7, H, EGW ? EGW : 16>(mode, tb);
    case 8: return fast_for_len<8, H, EGW ? EGW : 16>(mode, tb);
    case 9: return fast_for_len<9, H, EGW ? EGW : 16>(mode, tb);
    case 10: return fast_for_len<10, H, EGW ? EGW : 16>(mode, tb);
    case 11: return fast_for_len<11, H, EGW ? EGW : 16>(mode, tb);
    case 12: return fast_for_len<12, H, EGW ? EGW : 16>(mode, tb);
    default: return nullptr;
    }
}

// groups: 1, 2 (two 16-item groups) or 3 (two 32-item groups: tile twice as wide)
const void *fast_kernel(int log2n, int mode, int tb, int groups)
{
    if (groups == 3) return fast_kernel_h<2, 32>(log2n, mode, tb);
    return groups == 2 ? fast_kernel_h<2, 0>(log2n, mode, tb) : fast_kernel_h<1, 0>(log2n, mode, tb);
}

const void *kernel_for(int log2n, bool pre, bool gen)
{
    if (gen) return pre ? kernel_for_pre<true, true>(log2n) : kernel_for_pre<false, true>(log2n);
    return pre ? kernel_for_pre<true, false>(log2n) : kernel_for_pre<false, false>(log2n);
}

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

int32_t local_fft_fast_mode(const LocalPass &p)
{
    // single-pass Phase I (pi on output rows) or Phase III (pi on input rows)
    if (p.pre_tw || p.n_outer != 1 || p.o_in || p.o_out || p.j_in != 1 || p.k_out != 1) return -1;
    if (p.log2T != fast_tile_log2T(p.log2n, p.groups >= 2 ? 2 : 1, p.groups == 3 ? 32 : 16)) return -1;
    int mode = -1, tb = 0;
    if (p.out_tr) {
        if (p.in_ell || p.out_ell) return -1;
        mode = 2;
        tb = 1;
    } else {
        if (p.out_ell && !p.in_ell) { mode = 0; tb = p.out_t; }
        if (p.in_ell && !p.out_ell) { mode = 1; tb = p.in_t; }
    }
    if (mode < 0 || !fast_kernel(p.log2n, mode, tb, p.groups)) return -1;
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
    for (int l = 1; l <= kMaxOnChipLog2; ++l) {
        for (int v = 0; v < 4; ++v) {
            hipError_t e = hipFuncSetAttribute(kernel_for(l, v & 1, v & 2), hipFuncAttributeMaxDynamicSharedMemorySize,
                                               160 * 1024);
            if (e != hipSuccess) return e;
        }
        for (int mode = 0; mode < 3; ++mode)
            for (int tb : {1, 2, 4})
                for (int grp : {1, 2, 3}) {
                const void *k = fast_kernel(l, mode, tb, grp);
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
    const void *k = mode >= 0 ? fast_kernel(p.log2n, mode, mode == 2 ? 1 : (mode == 0 ? p.out_t : p.in_t), p.groups)
                              : kernel_for(p.log2n, p.pre_tw != 0, pass_needs_gen(p));
    if (!k) return hipErrorInvalidValue;
    const LocalLaunch g = local_fft_geometry(p);
    if (g.tiles < 1 || g.tiles > 0x7fffffff) return hipErrorInvalidValue;
    void *args[] = {const_cast<LocalPass *>(&p)};
    return hipLaunchKernel(k, dim3(unsigned(g.tiles)), dim3(unsigned(g.threads)), args, g.lds_bytes, s);
}

}  // namespace paco
