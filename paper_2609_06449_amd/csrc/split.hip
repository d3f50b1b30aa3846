// The split form (FP32) for N1 = 16 M, M = 2^8, 2^9, 2^10 (N1 = 2^12 .. 2^14).
//
// Phase I transforms every column c of X (N1 x N2, row-major) over its N1
// rows.  Split once more by Cooley-Tukey (Lemma 1 with a first child of
// length 16): with row j1 = j + M r and frequency k1 = k0 + 16 k,
//
//   A[k1, c] = sum_j w_M^{-j k} T[c][j][k0],
//   T[c][j][k0] = w_N1^{-j k0} sum_r X[j + M r, c] w_16^{-r k0}.
//
// The bracket needs only 16 rows of a column at a time, so pass 1 can read
// x in whole 128-byte row runs (16 columns per workgroup), where a tile that
// holds entire 4096-point columns on chip reads 32-byte runs; its HBM
// pattern measured ~30% faster.  The rest of the column transform (16
// transforms of length M per column) needs each column's T contiguous,
// which is exactly what the redistribution of Phase II reads, so pass 2
// finishes them there: it reads column c's block once (N1 items), runs the
// M-point transforms (two radix-16 stages for M = 256, three stages for 512
// and 1024), multiplies by the top-level twiddle w_N^{-k1 c} (Phase II,
// Sec. 4) and writes row pi_{m2}(c) of out in natural k1 order, as the
// packed Phase II does.  Phase III is unchanged.  For N1 = 2^12 the pipeline
// stays at three HBM passes; for 2^13 and 2^14, whose Phase I otherwise
// takes two on-chip passes, the split form saves one.

#include "stages.h"

namespace paco {
namespace {

constexpr int kSplitThreads = 256;
constexpr int kFirstPad = 257;  // LDS row of pass 1: 256 items + 1

// Pass 1.  Workgroup (cg, jg) owns columns c = 16 cg + cl and indices
// j = 16 jg + jl (cl, jl < 16), i.e. rows j + M r (M = N1 / 16) of 16
// adjacent columns: every load instruction reads four full 128-byte row
// runs.  Its 16 x 256 results are ws[c*N1 + 256 jg + (16 jl + k0)]: 2 KiB
// contiguous per column, stored through LDS so that every store instruction
// writes 512 bytes, with streaming stores.  Pass 2 reads ws once, in whole
// column blocks that HBM serves at copy speed; left out of the 256 MiB
// MALL, ws no longer pushes x
// (read again by the next transform) and out (Phase III's input) out of
// it: 2^24 back to back, pass 1 59 -> 47 us, pass 2 56 -> 53 us, Phase III
// 67 -> 65 us, the transform 175 -> 157 us.
__global__ __launch_bounds__(kSplitThreads) void split_first_kernel(SplitPass P)
{
    __shared__ float2 lds[16 * kFirstPad];
    const int tid = threadIdx.x;
    const int64_t jg = int64_t(blockIdx.x) / (P.N2 >> 4);
    const int cl = tid & 15, jl = tid >> 4;
    const int j = int(jg << 4) + jl;
    const uint32_t N1 = uint32_t(P.N1), N2 = uint32_t(P.N2);
    const float2 *src = P.src + addr::split1_load_base(N2, blockIdx.x, tid);
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = src[addr::split1_load_off(N1, N2, r)];  // rows j + (N1/16) r
    if (P.conj_in) {
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r].y = -v[r].y;
    }
    dft_regs<4>(v);
#pragma unroll
    for (int k0 = 1; k0 < 16; ++k0) v[k0] = cmul(v[k0], P.tw[(j * k0) << P.tw_shift]);
#pragma unroll
    for (int k0 = 0; k0 < 16; ++k0) lds[cl * kFirstPad + jl * 16 + k0] = v[k0];
    __syncthreads();
    float2 *dst = P.dst + addr::split1_store_base(N1, N2, blockIdx.x, tid);
#pragma unroll
    for (int q = 0; q < 16; ++q) st2_stream(dst + addr::split1_store_off(N1, q), lds[q * kFirstPad + tid]);
}

// Pass 2.  Workgroup c: y_k0[j] = T[c][j][k0] (j = jl + 16 jh) is
// transformed over j by two radix-16 stages,
//   DFT_256(y)[kl + 16 kh] = sum_jl w_16^{-jl kh} w_256^{-jl kl} sum_jh y[jl + 16 jh] w_16^{-jh kl},
// thread (k0, jl) taking the inner sums and thread (k0, kl) the outer ones.
// Output k1 = k0 + 16 kl + 256 kh goes to out[pi_{m2}(c)*N1 + k1] times
//   w_N^{-k1 c} = w_N^{-k0 c} * w_N^{-16 kl c} * w_N^{-256 kh c},
// factors with 16, 4 and 1 distinct table entries per wave (the last is the
// same for the whole workgroup).  Every twiddle load is issued right behind
// the data loads so that its latency overlaps theirs: 69 -> 61 us per
// 2^24 launch against loading each factor where it is used.  The exchange
// buffer is unpadded (32 KiB: five workgroups fit a CU) with an XOR swizzle of
// the 16-item rows: row k of the buffer holds item (jl, k0) at
// 16 (jl ^ (k & 3)) + k0, so the writes of a wave cover 64 distinct banks
// and its reads of four rows k fall into two bank halves.  A 96-VGPR budget
// (five waves per SIMD, which that buffer allows) took the launch from 60
// to 55 us (no spills).
template <bool GEN>
__global__ __launch_bounds__(kSplitThreads) __attribute__((amdgpu_waves_per_eu(5))) void split_middle_kernel(
    SplitPass P)
{
    __shared__ float2 lds[16 * 256];
    const int tid = threadIdx.x;
    const int64_t c = blockIdx.x;
    const int lo = tid & 15, hi = tid >> 4;  // k0, and jl (inner sums) or kl (outer sums)
    const uint32_t N1 = uint32_t(P.N1);
    float2 v[16];
    const float2 *src = P.src + addr::split2_load_base(N1, uint32_t(c), tid);
#pragma unroll
    for (int jh = 0; jh < 16; ++jh) v[jh] = ld2_last(src + addr::split2_load_off(jh));  // last use
    float2 t256[16];
#pragma unroll
    for (int k = 1; k < 16; ++k) t256[k] = P.tw[(16 * hi * k) << P.tw_shift];  // w_256^{-jl kl}
    const uint32_t nmask = uint32_t((uint64_t(1) << P.log2N) - 1), lomask = (1u << P.log2Lo) - 1;
    const uint32_t e0 = (uint32_t(lo) * uint32_t(c)) & nmask, e1 = (uint32_t(16 * hi) * uint32_t(c)) & nmask;
    const float2 a0 = P.tw_hi[e0 >> P.log2Lo], a1 = P.tw_lo[e0 & lomask];
    const float2 a2 = P.tw_hi[e1 >> P.log2Lo], a3 = P.tw_lo[e1 & lomask];
    float2 bh[16], bl[16];
#pragma unroll
    for (int kh = 0; kh < 16; ++kh) {
        const uint32_t e2 = (uint32_t(256 * kh) * uint32_t(c)) & nmask;
        bh[kh] = P.tw_hi[e2 >> P.log2Lo];
        bl[kh] = P.tw_lo[e2 & lomask];
    }
    const int64_t u = digmap<GEN>(c, P.t, P.m2, P.s2, false);

    dft_regs<4>(v);
#pragma unroll
    for (int k = 1; k < 16; ++k) v[k] = cmul(v[k], t256[k]);
#pragma unroll
    for (int k = 0; k < 16; ++k) lds[k * 256 + (((hi ^ (k & 3)) << 4) | lo)] = v[k];
    __syncthreads();
#pragma unroll
    for (int jl = 0; jl < 16; ++jl) v[jl] = lds[hi * 256 + (((jl ^ (hi & 3)) << 4) | lo)];
    dft_regs<4>(v);

    const float2 a = cmul(cmul(a0, a1), cmul(a2, a3));  // w_N^{-(k0 + 16 kl) c}
    float2 *dst = P.dst + addr::split2_store_base(N1, uint32_t(u), tid);
#pragma unroll
    for (int kh = 0; kh < 16; ++kh) dst[addr::split2_store_off(kh)] = cmul(v[kh], cmul(a, cmul(bh[kh], bl[kh])));
}

// Pass 2 for N1 = 16 M with M = 256 R (R = 2^LR = 2 or 4: N1 = 2^13, 2^14).
// Workgroup c, M threads, 16 items each; the M-point transforms over
// j = jl + (M/16) jh (jl < M/16) run as three stages:
//   A  thread (k0, jl): radix 16 over jh -> ka, times w_M^{-jl ka};
//   B  thread (k0, ka, jlo) (jl = jlo + R jhi): radix 16 over jhi -> kb,
//      times w_{16R}^{-jlo kb};
//   C  thread (k0, q), pairs (ka, kb) = q + (M/16) i (i < 16/R): radix R
//      over jlo -> kc,
// so k1 = k0 + 16 ka + 256 kb + 4096 kc = k0 + 16 (ka + 16 kb) + 4096 kc.
// Both exchanges go through the same 32R KiB of dynamic LDS, in 16-item
// rows whose index is XOR-swizzled by ka & 3 (a wave's four ka values then
// fall into two bank halves).  The top-level twiddle is
//   w_N^{-k1 c} = w_N^{-k0 c} * w_N^{-16 (ka + 16 kb) c} * w_N^{-4096 kc c}.
// A 128-VGPR budget (no spills) lets two 512-thread workgroups share a CU
// for N1 = 2^13 (64 KiB of LDS each): 8192 x 32768 took 3.63 against
// 3.94 ms per transform with 142 VGPRs.
template <bool GEN, int LR>
__global__ __launch_bounds__(256 << LR) __attribute__((amdgpu_waves_per_eu(4))) void split_middle3_kernel(
    SplitPass P)
{
    extern __shared__ float2 xbuf[];
    constexpr int R = 1 << LR, JL = (256 << LR) / 16, NPAIR = 16 / R;
    const int tid = threadIdx.x;
    const int64_t c = blockIdx.x;
    const int k0 = tid & 15;
    const uint32_t N1 = uint32_t(P.N1);
    const float2 *src = P.src + addr::split3_load_base(N1, uint32_t(c), tid);
    const uint32_t nmask = uint32_t((uint64_t(1) << P.log2N) - 1), lomask = (1u << P.log2Lo) - 1;

    // stage A operands, then every twiddle, issued before the first butterfly
    const int jl = tid >> 4;
    float2 v[16];
#pragma unroll
    for (int jh = 0; jh < 16; ++jh) v[jh] = ld2_last(src + addr::split3_load_off(N1, jh));  // last use
    // stage B: (k0, ka, jlo); jlo is the same for a whole wave (its twiddles
    // are scalar loads)
    const int kab = (tid >> 4) & 15, jlo = __builtin_amdgcn_readfirstlane(tid >> 8);
    const int q = tid >> 4;                           // stage C: (k0, q)
    float2 tA[16], tB[16];
#pragma unroll
    for (int k = 1; k < 16; ++k) {
        tA[k] = P.tw[(16 * jl * k) << P.tw_shift];    // w_M^{-jl ka}
        tB[k] = P.tw[(256 * jlo * k) << P.tw_shift];  // w_{16R}^{-jlo kb}
    }
    float2 h0, l0, hp[NPAIR], lp[NPAIR], hc[R], lc[R];
    {
        const uint32_t e = (uint32_t(k0) * uint32_t(c)) & nmask;
        h0 = P.tw_hi[e >> P.log2Lo];
        l0 = P.tw_lo[e & lomask];
    }
#pragma unroll
    for (int i = 0; i < NPAIR; ++i) {
        const uint32_t e = (uint32_t(16 * (q + JL * i)) * uint32_t(c)) & nmask;
        hp[i] = P.tw_hi[e >> P.log2Lo];
        lp[i] = P.tw_lo[e & lomask];
    }
#pragma unroll
    for (int kc = 0; kc < R; ++kc) {
        const uint32_t e = (uint32_t(4096 * kc) * uint32_t(c)) & nmask;
        hc[kc] = P.tw_hi[e >> P.log2Lo];
        lc[kc] = P.tw_lo[e & lomask];
    }
    const int64_t u = digmap<GEN>(c, P.t, P.m2, P.s2, false);

    // A: Y[ka][jl][k0] in row ka JL + (jl ^ (ka & 3))
    dft_regs<4>(v);
#pragma unroll
    for (int k = 1; k < 16; ++k) v[k] = cmul(v[k], tA[k]);
#pragma unroll
    for (int ka = 0; ka < 16; ++ka) xbuf[((ka * JL + (jl ^ (ka & 3))) << 4) | k0] = v[ka];
    __syncthreads();
    // B: items jhi of (ka, jlo), jl = jlo + R jhi
#pragma unroll
    for (int jhi = 0; jhi < 16; ++jhi) v[jhi] = xbuf[((kab * JL + ((jlo + R * jhi) ^ (kab & 3))) << 4) | k0];
    dft_regs<4>(v);
#pragma unroll
    for (int k = 1; k < 16; ++k) v[k] = cmul(v[k], tB[k]);
    __syncthreads();  // every wave has read its stage-B operands
    // Z[pr = ka + 16 kb][jlo][k0] in row ((pr R + jlo) ^ (ka & 3))
#pragma unroll
    for (int kb = 0; kb < 16; ++kb) xbuf[(((((kb << 4) + kab) << LR) + jlo) ^ (kab & 3)) << 4 | k0] = v[kb];
    __syncthreads();
    // C: NPAIR radix-R butterflies per thread, stored straight to row pi_{m2}(c)
    const float2 a0 = cmul(h0, l0);
    float2 *dst = P.dst + addr::split3_store_base(N1, uint32_t(u), tid);
#pragma unroll
    for (int i = 0; i < NPAIR; ++i) {
        const int pr = q + JL * i, ka = pr & 15;
        float2 z[R];
#pragma unroll
        for (int j2 = 0; j2 < R; ++j2) z[j2] = xbuf[((((pr << LR) + j2) ^ (ka & 3)) << 4) | k0];
        dft_regs<LR>(z);
        const float2 a = cmul(a0, cmul(hp[i], lp[i]));
#pragma unroll
        for (int kc = 0; kc < R; ++kc)
            dst[addr::split3_store_off(N1, i, kc)] = cmul(z[kc], cmul(a, cmul(hc[kc], lc[kc])));
    }
}

bool split_shape_ok(const SplitPass &p)
{
    return (p.N1 == 4096 || p.N1 == 8192 || p.N1 == 16384) && p.N2 >= 16 && p.N2 % 16 == 0 && p.log2N <= 32 &&
           p.src && p.dst && p.tw && p.tw_hi && p.tw_lo;
}

}  // namespace

hipError_t split_prepare()
{
    for (const void *k : {reinterpret_cast<const void *>(&split_middle3_kernel<false, 1>),
                          reinterpret_cast<const void *>(&split_middle3_kernel<true, 1>),
                          reinterpret_cast<const void *>(&split_middle3_kernel<false, 2>),
                          reinterpret_cast<const void *>(&split_middle3_kernel<true, 2>)}) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_split_first(const SplitPass &p, hipStream_t s)
{
    if (!split_shape_ok(p)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(split_first_kernel, dim3(addr::split1_groups(uint32_t(p.N1), uint32_t(p.N2))),
                       dim3(kSplitThreads), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_split_middle(const SplitPass &p, hipStream_t s)
{
    if (!split_shape_ok(p)) return hipErrorInvalidValue;
    const bool f = digrev_fast(p.t);
    if (p.N1 != 4096) {  // three stages: 512 or 1024 threads, 64 or 128 KiB of LDS
        void (*k3)(SplitPass) = p.N1 == 8192 ? (f ? split_middle3_kernel<false, 1> : split_middle3_kernel<true, 1>)
                                             : (f ? split_middle3_kernel<false, 2> : split_middle3_kernel<true, 2>);
        hipLaunchKernelGGL(k3, dim3(unsigned(p.N2)), dim3(unsigned(p.N1 / 16)), size_t(p.N1) * 8u, s, p);
        return hipGetLastError();
    }
    void (*k)(SplitPass) = f ? split_middle_kernel<false> : split_middle_kernel<true>;
    hipLaunchKernelGGL(k, dim3(unsigned(p.N2)), dim3(kSplitThreads), 0, s, p);
    return hipGetLastError();
}

}  // namespace paco
