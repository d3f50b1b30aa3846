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
// TC items), scales each item by its destination-indexed twiddle,
// transposes the tile in LDS and writes rows u = pi_{m2}(c) (contiguous runs
// of TV items).  With TV | N1/p and TC | N2/p every tile lies inside one
// source/destination slab pair (q, q'), so the launch is the paper's block
// exchange cut into equal tiles.
#include "paco_internal.h"

namespace paco {
namespace {

constexpr int kTile = 64;
constexpr int kThreads = 256;

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ __launch_bounds__(kThreads) void middle_kernel(MiddlePass P)
{
    __shared__ float2 tile[kTile * (kTile + 1)];
    const int lTV = P.N1 < kTile ? __builtin_ctzll(P.N1) : 6;
    const int lTC = P.N2 < kTile ? __builtin_ctzll(P.N2) : 6;
    const int TV = 1 << lTV, TC = 1 << lTC;
    const int64_t nct = P.N2 >> lTC;
    const int64_t vt = blockIdx.x / nct;
    const int64_t ct = blockIdx.x - vt * nct;
    const int64_t v0 = vt << lTV, c0 = ct << lTC;
    const int64_t Nm = (int64_t(1) << P.log2N) - 1;
    const int64_t Lm = (int64_t(1) << P.log2Lo) - 1;
    const int tid = threadIdx.x;

    for (int e = tid; e < TV * TC; e += kThreads) {
        const int vi = e >> lTC, ci = e & (TC - 1);
        const int64_t v = v0 + vi, c = c0 + ci;
        const int64_t a = P.pi1[v];
        float2 x = P.ws[a * P.N2 + c];
        if (P.twiddle) {
            const int64_t r = (v * c) & Nm;
            x = cmul(x, cmul(P.tw_hi[r >> P.log2Lo], P.tw_lo[r & Lm]));
        }
        tile[ci * (kTile + 1) + vi] = x;
    }
    __syncthreads();
    for (int e = tid; e < TV * TC; e += kThreads) {
        const int ci = e >> lTV, vi = e & (TV - 1);
        const int64_t c = c0 + ci;
        const int64_t u = P.pi2[c];
        P.out[u * P.N1 + v0 + vi] = tile[ci * (kTile + 1) + vi];
    }
}

}  // namespace

hipError_t launch_middle(const MiddlePass &p, hipStream_t s)
{
    const int64_t TV = p.N1 < kTile ? p.N1 : kTile, TC = p.N2 < kTile ? p.N2 : kTile;
    const int64_t groups = (p.N1 / TV) * (p.N2 / TC);
    hipLaunchKernelGGL(middle_kernel, dim3(unsigned(groups)), dim3(kThreads), 0, s, p);
    return hipGetLastError();
}

}  // namespace paco
