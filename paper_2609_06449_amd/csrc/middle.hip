// Phase II: the single fused redistribution (paper, sections 3.3 and 4.2,
// appendix C) as one HBM pass on gfx950.
//
// The paper's per-processor procedure packs (row macro-element digit
// reversal a -> v = pi_{m1}(a) fused with the twiddle w_N^{-v c}), exchanges
// balanced (N1/p) x (N2/p) blocks, transposes each block and unpacks (row
// macro-element digit reversal c -> u = pi_{m2}(c)).  The composite is the
// coordinate map (a, c) -> (pi_{m2}(c), pi_{m1}(a)) with the twiddle, and on
// one device every step is an address: a workgroup owns a TV x TC tile of
// logical (v, c) coordinates, reads rows a = pi_{m1}(v) (contiguous runs of
// TC items), scales each item by its destination-indexed twiddle, transposes
// the tile in LDS and writes rows u = pi_{m2}(c) (contiguous runs of TV
// items).  When TV | N1/p and TC | N2/p every tile lies inside one
// source/destination slab pair (q, q'), so the launch is the paper's block
// exchange cut into equal tiles.
//
// The twiddle of item (v0 + vi, c0 + ci) is assembled from three factors,
//   w_N^{-v c} = w_N^{-v0 c} * w_N^{-vi c0} * w_N^{-vi ci},
// a per-thread value, a per-row value shared through LDS and a fixed
// TV x TC table read with the same coalesced pattern as the data, so no
// lane-divergent table gather sits on the per-item path.
#include "middle_dev.h"

namespace paco {
namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = kMidTile * kMidTile / kThreads;  // 16


// FULL: N1, N2 >= 64, every tile is 64 x 64 (no guards).  TW: apply the
// twiddle (else the bare permutation).
template <bool GEN, bool FULL, bool TW>
__global__ __launch_bounds__(kThreads) void middle_kernel(MiddlePass P)
{
    __shared__ float2 tile[kMidTile * (kMidTile + 1)];
    __shared__ float2 rowtw[kMidTile];
    const int lTV = FULL ? 6 : (P.N1 < kMidTile ? __builtin_ctzll(P.N1) : 6);
    const int lTC = FULL ? 6 : (P.N2 < kMidTile ? __builtin_ctzll(P.N2) : 6);
    const int TV = 1 << lTV, TC = 1 << lTC;
    const int64_t nct = P.N2 >> lTC;
    const int64_t vt = blockIdx.x / nct;
    const int64_t ct = blockIdx.x - vt * nct;
    const int64_t v0 = vt << lTV, c0 = ct << lTC;
    const int64_t Nm = (int64_t(1) << P.log2N) - 1;
    const int64_t Lm = (int64_t(1) << P.log2Lo) - 1;
    const int tid = threadIdx.x;

    // read side: thread owns column ci and rows rg + q*rstep
    const int ci = tid & (TC - 1);
    const int rg = tid >> lTC;
    const int rstep = kThreads >> lTC;
    const int64_t c = c0 + ci;
    float2 x[kPerThread], t4[kPerThread];
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
        const int vi = rg + q * rstep;
        if (FULL || vi < TV) {
            const int64_t a = digmap<GEN>(v0 + vi, P.t, P.m1, P.s1, true);
            x[q] = ld2_last(P.ws + a * P.N2 + c);
            if (TW) t4[q] = P.tw_tile[vi * kTwTile + ci];
        }
    }
    float2 wc = make_float2(1.f, 0.f);
    if (TW) {
        const int64_t r = (v0 * c) & Nm;
        wc = cmul(P.tw_hi[r >> P.log2Lo], P.tw_lo[r & Lm]);
        if (tid < TV) {
            const int64_t rr = (int64_t(tid) * c0) & Nm;
            rowtw[tid] = cmul(P.tw_hi[rr >> P.log2Lo], P.tw_lo[rr & Lm]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
        const int vi = rg + q * rstep;
        if (FULL || vi < TV) {
            float2 y = x[q];
            if (TW) y = cmul(y, cmul(cmul(wc, rowtw[vi]), t4[q]));
            tile[ci * (kMidTile + 1) + vi] = y;
        }
    }
    __syncthreads();
    // write side: thread owns tile column vi and output rows cg + q*cstep
    const int vi = tid & (TV - 1);
    const int cg = tid >> lTV;
    const int cstep = kThreads >> lTV;
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
        const int cj = cg + q * cstep;
        if (FULL || cj < TC) {
            const int64_t u = digmap<GEN>(c0 + cj, P.t, P.m2, P.s2, false);
            P.out[u * P.N1 + v0 + vi] = tile[cj * (kMidTile + 1) + vi];
        }
    }
}

template <bool GEN, bool TW>
__global__ __launch_bounds__(kThreads) void middle_packed_kernel(MiddlePass P)
{
    middle_packed_tile<GEN, TW>(P, blockIdx.x, threadIdx.x);
}

template <bool GEN, bool TW>
__global__ __launch_bounds__(kThreads) void middle_packed2_kernel(MiddlePass P)
{
    middle_packed2_tile<GEN, TW>(P, blockIdx.x, threadIdx.x);
}

}  // namespace

hipError_t launch_middle(const MiddlePass &p, hipStream_t s)
{
    if (p.packed && p.N1 >= 2 * kMidTile && p.N2 >= kMidTile) {
        const int64_t groups = (p.N1 / (2 * kMidTile)) * (p.N2 / kMidTile);
        void (*k)(MiddlePass);
        if (digrev_fast(p.t))
            k = p.twiddle ? middle_packed2_kernel<false, true> : middle_packed2_kernel<false, false>;
        else
            k = p.twiddle ? middle_packed2_kernel<true, true> : middle_packed2_kernel<true, false>;
        hipLaunchKernelGGL(k, dim3(unsigned(groups)), dim3(kThreads), 0, s, p);
        return hipGetLastError();
    }
    if (p.packed) {
        if (p.N1 < kMidTile || p.N2 < kMidTile) return hipErrorInvalidValue;
        const int64_t groups = (p.N1 / kMidTile) * (p.N2 / kMidTile);
        void (*k)(MiddlePass);
        if (digrev_fast(p.t))
            k = p.twiddle ? middle_packed_kernel<false, true> : middle_packed_kernel<false, false>;
        else
            k = p.twiddle ? middle_packed_kernel<true, true> : middle_packed_kernel<true, false>;
        hipLaunchKernelGGL(k, dim3(unsigned(groups)), dim3(kThreads), 0, s, p);
        return hipGetLastError();
    }
    const int64_t TV = p.N1 < kMidTile ? p.N1 : kMidTile, TC = p.N2 < kMidTile ? p.N2 : kMidTile;
    const int64_t groups = (p.N1 / TV) * (p.N2 / TC);
    const bool full = p.N1 >= kMidTile && p.N2 >= kMidTile, tw = p.twiddle != 0;
    void (*k)(MiddlePass);
    if (!digrev_fast(p.t))
        k = tw ? middle_kernel<true, false, true> : middle_kernel<true, false, false>;
    else if (full)
        k = tw ? middle_kernel<false, true, true> : middle_kernel<false, true, false>;
    else
        k = tw ? middle_kernel<false, false, true> : middle_kernel<false, false, false>;
    hipLaunchKernelGGL(k, dim3(unsigned(groups)), dim3(kThreads), 0, s, p);
    return hipGetLastError();
}

}  // namespace paco
