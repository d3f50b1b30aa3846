// Phase II tile bodies of the fused pipeline, shared by the single-transform
// kernels (middle.hip) and the batched persistent kernel (batch.hip).
// COH: device-coherent result stores (st2/st4 in stages.h).
#pragma once

#include "stages.h"

namespace paco {
namespace {

constexpr int kMidThreads = 256;
constexpr int kMidPerThread = kMidTile * kMidTile / kMidThreads;  // 16

// Fused-pipeline variant: ws is the packed slab stored transposed,
// ws[c*N1 + v] = A[v, c] with v the logical first-stage frequency (the pack
// step's row reversal already undone by Phase I's store).  What remains of
// the redistribution is the unpack (row c -> u = pi_{m2}(c)) with the
// twiddle w_N^{-v c}: a streaming row permutation.  A workgroup owns 64 rows
// c x 64 columns v; wave w takes rows c0 + w + 4q, lane = column, so every
// load and store is a 512-byte run and the row index, its digit reversal
// and the per-row twiddle factor are wave-uniform (scalar) values.
template <bool GEN, bool TW, bool COH = false>
__device__ __forceinline__ void middle_packed_tile(const MiddlePass &P, int64_t blk, int tid)
{
    const int64_t nvt = P.N1 >> 6;
    const int64_t ct = blk / nvt;
    const int64_t vt = blk - ct * nvt;
    const int64_t v0 = vt << 6, c0 = ct << 6;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t Nm = (int64_t(1) << P.log2N) - 1;
    const int64_t Lm = (int64_t(1) << P.log2Lo) - 1;

    float2 rw = make_float2(1.f, 0.f);  // w_N^{-vi c0}
    if (TW) {
        const int64_t r = (int64_t(lane) * c0) & Nm;
        rw = cmul(P.tw_hi[r >> P.log2Lo], P.tw_lo[r & Lm]);
    }
    float2 x[kMidPerThread], t4[kMidPerThread];
#pragma unroll
    for (int q = 0; q < kMidPerThread; ++q) {
        const int ci = w + 4 * q;
        x[q] = ld2_last(P.ws + (c0 + ci) * P.N1 + v0 + lane);
        if (TW) t4[q] = P.tw_tile[ci * kTwTile + lane];
    }
#pragma unroll
    for (int q = 0; q < kMidPerThread; ++q) {
        const int64_t c = c0 + w + 4 * q;
        const int64_t u = digmap<GEN>(c, P.t, P.m2, P.s2, false);
        float2 y = x[q];
        if (TW) {
            const int64_t r = (v0 * c) & Nm;  // w_N^{-v0 c}: one value per row
            const float2 wc = cmul(P.tw_hi[r >> P.log2Lo], P.tw_lo[r & Lm]);
            y = cmul(y, cmul(wc, cmul(rw, t4[q])));
        }
        st2<COH>(reinterpret_cast<char *>(P.out + u * P.N1 + v0 + lane), y);
    }
}

// The same with two adjacent columns per lane: a workgroup owns 64 rows x
// 128 columns and every load and store is a 1 KB run of 16-byte accesses.
template <bool GEN, bool TW, bool COH = false>
__device__ __forceinline__ void middle_packed2_tile(const MiddlePass &P, int64_t blk, int tid)
{
    const int64_t nvt = P.N1 >> 7;
    const int64_t ct = blk / nvt;
    const int64_t vt = blk - ct * nvt;
    const int64_t v0 = vt << 7, c0 = ct << 6;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t Nm = (int64_t(1) << P.log2N) - 1;
    const int64_t Lm = (int64_t(1) << P.log2Lo) - 1;
    const int vi = 2 * lane;

    float2 rw0 = make_float2(1.f, 0.f), rw1 = rw0;  // w_N^{-vi c0}, w_N^{-(vi+1) c0}
    if (TW) {
        const int64_t r0 = (int64_t(vi) * c0) & Nm, r1 = (int64_t(vi + 1) * c0) & Nm;
        rw0 = cmul(P.tw_hi[r0 >> P.log2Lo], P.tw_lo[r0 & Lm]);
        rw1 = cmul(P.tw_hi[r1 >> P.log2Lo], P.tw_lo[r1 & Lm]);
    }
    float4 x[kMidPerThread], t4[kMidPerThread];
#pragma unroll
    for (int q = 0; q < kMidPerThread; ++q) {
        const int ci = w + 4 * q;
        x[q] = ld4_last(P.ws + (c0 + ci) * P.N1 + v0 + vi);
        if (TW) t4[q] = *reinterpret_cast<const float4 *>(P.tw_tile + ci * kTwTile + vi);
    }
#pragma unroll
    for (int q = 0; q < kMidPerThread; ++q) {
        const int64_t c = c0 + w + 4 * q;
        const int64_t u = digmap<GEN>(c, P.t, P.m2, P.s2, false);
        float2 y0 = make_float2(x[q].x, x[q].y), y1 = make_float2(x[q].z, x[q].w);
        if (TW) {
            const int64_t r = (v0 * c) & Nm;  // w_N^{-v0 c}: one value per row
            const float2 wc = cmul(P.tw_hi[r >> P.log2Lo], P.tw_lo[r & Lm]);
            y0 = cmul(y0, cmul(wc, cmul(rw0, make_float2(t4[q].x, t4[q].y))));
            y1 = cmul(y1, cmul(wc, cmul(rw1, make_float2(t4[q].z, t4[q].w))));
        }
        st4<COH>(reinterpret_cast<char *>(P.out + u * P.N1 + v0 + vi), make_float4(y0.x, y0.y, y1.x, y1.y));
    }
}

}  // namespace
}  // namespace paco
