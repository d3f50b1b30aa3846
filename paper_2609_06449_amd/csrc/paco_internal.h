// Internal declarations shared by the PACO HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace paco {

// Largest transform length one local pass keeps on chip (LDS + registers).
constexpr int kMaxOnChipLog2 = 12;

// One HBM pass of a batched local FFT: the GPU form of a digit-field view
// (paper, appendix A.3-A.4).  The pass runs n_outer * (ncols / T) independent
// groups; group (o, tile) transforms the T contiguous columns
// [tile*T, tile*T + T) of the rows
//     input  row of logical j : o*o_in  + map_in(j)  * j_in
//     output row of logical k : o*o_out + map_out(k) * k_out
// where map_in / map_out are the identity or a base-b digit reversal table.
// A row is ld complex64 items long; the column field C of the paper's view is
// the contiguous run of T items that every access reads or writes whole.
// Before the length-n DFT the input j of group o is scaled by the
// Cooley-Tukey twiddle w_M^{-f(o)*j}, f(o) = o or tw_perm[o] (the
// layout-aware twiddle of appendix A.2), when pre_tw is set.
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
    const int32_t *perm_in;   // nullable
    const int32_t *perm_out;  // nullable
    const float2 *tw;         // w_L^{-r}, r < L = 2^log2L (FP64-generated)
    int32_t log2L;
    int32_t pre_tw;           // 0: none; 1: w_M^{-f(o) j} before the DFT
    int32_t log2M;            // M of the pre-twiddle (M <= L)
    const int32_t *tw_perm;   // nullable: f(o) = tw_perm[o], else f(o) = o
};

// Phase II: out[pi2[c]*N1 + v] = ws[pi1[v]*N2 + c] * w_N^{-(v*c mod N)}, the
// fused middle permutation (section 3.3) written by v = pi_{m1}(a).
struct MiddlePass {
    const float2 *ws;
    float2 *out;
    int64_t N1, N2;
    const int32_t *pi1;       // pi_{m1} over [N1]
    const int32_t *pi2;       // pi_{m2} over [N2]
    const float2 *tw_hi;      // w_N^{-h*Lo}, h < N/Lo
    const float2 *tw_lo;      // w_N^{-l}, l < Lo
    int32_t log2N, log2Lo;
    int32_t twiddle;          // 0: bare permutation
};

// Workgroup geometry a local pass is launched with.
struct LocalLaunch {
    int threads;       // per workgroup
    size_t lds_bytes;  // dynamic LDS per workgroup
    int64_t groups;    // workgroups
};

LocalLaunch local_fft_geometry(const LocalPass &p);
hipError_t local_fft_prepare();  // raises the dynamic-LDS limit of every kernel once
hipError_t launch_local_fft(const LocalPass &p, hipStream_t s);
hipError_t launch_middle(const MiddlePass &p, hipStream_t s);

// Columns per workgroup for an on-chip pass of length 2^log2n over ncols.
int32_t choose_log2T(int32_t log2n, int64_t ncols);

}  // namespace paco
