// The symmetric split form (FP32) for N1 = N2 = 4096.
//
// Both local phases are split once more by Cooley-Tukey (Lemma 1), each with
// one 16-point child, and both 16-point children run in the redistribution
// pass:
//
//   Phase I,   j1 = 16 j + r,    k1 = k + 256 s   (j, k < 256; r, s < 16):
//     A[k1, c]  = sum_r w_16^{-s r} U[c][r][k],
//     U[c][r][k] = w_N1^{-k r} sum_j X[16 j + r, c] w_256^{-k j};
//   Phase III, j2 = jc + 256 rr, k2 = q0 + 16 q  (jc, q < 256; rr, q0 < 16):
//     Y[k2, v]  = sum_jc w_256^{-q jc} W[v][jc][q0],
//     W[v][jc][q0] = w_N2^{-q0 jc} sum_rr Z[v, jc + 256 rr] w_16^{-q0 rr},
//   with Z[v, c] = A[v, c] w_N^{-v c} the twiddled middle stage (section 3.3).
//
// Pass 1 computes U (256-point transforms over rows 16 j + r of x), pass 2
// the 16-point transform over r, the top-level twiddle and the 16-point
// transform over rr, pass 3 the 256-point transforms over jc.  Every tile is
// 16 adjacent columns (or 16 consecutive items) wide, so every HBM access of
// every pass moves whole 128-byte lines; the form it replaces keeps whole
// 4096-point columns of Phase III on chip, which caps its tile at 8 columns
// (64-byte runs).  The digit reversals of the paper's layouts (Phase II's row
// map pi_{m2}(c) and Phase III's input-layout read of row pi_{m2}(j2)) cancel,
// as in the packed form, so neither the layout base b nor the slab count p
// appears in any address.  In a distributed run pass 2's first half (the
// transform over r and the twiddle, local to column c) runs on the source
// slab and its second half (over rr, local to output column v) on the
// destination slab, one exchange between them.
//
// Buffers: x (N1 x N2) -> ws[((k >> 4) N2 + c) 256 + 16 r + (k & 15)] = U[c][r][k]
//          ws          -> out[(16 jc + q0) N1 + v] = W[v][jc][q0]
//          out         -> out[(q0 + 16 q) N1 + v] = Y[q0 + 16 q, v], in place:
//          the tile of pass 3 for (q0, columns) reads rows 16 t + q0 and
//          writes the same rows (t < 256), and reads all of them before its
//          first store.

#include "stages.h"

namespace paco {
namespace {

constexpr int kSymThreads = 256;
// LDS exchange buffers: 16 planes of 16 x 16 items.  The LDS serves a wave's
// 8-byte accesses in two halves of 32 lanes, one 8-byte slot of 32 per lane
// and cycle; the plane strides make every half-wave hit 32 distinct slots:
// 258 (= 2 mod 32 slots) where a half-wave's 16 lanes run across planes and
// 2 along a row (pass 1's stage-2 reads; 260 had measured 3.1M bank-conflict
// cycles per launch), 272 (= 16 mod 32) where 16 lanes run along a row and
// 2 across planes.  Pass 2 keeps 256-item planes (32 KiB, five workgroups
// per CU) and swaps the row pairs of odd planes instead (row a of plane m at
// a ^ (m & 1)), which gives the same.
constexpr int kPlaneK = 258;
constexpr int kPlaneR = 272;

// w_M^{-m} for M = 2^log2M <= L from the table w_L^{-r}
__device__ __forceinline__ float2 root_of(const float2 *tw, int log2L, int log2M, uint32_t m)
{
    return tw[(m & ((1u << log2M) - 1u)) << (log2L - log2M)];
}

// Pass 1.  Workgroup (r, cb) transforms columns c = 16 cb + cl over rows
// 16 j + r, j = jl + 16 jh: radix 16 over jh by thread (cl, jl), twiddle
// w_256^{-jl kl}, radix 16 over jl by thread (kl, cl), k = kl + 16 kh, then
// w_N1^{-k r} = w_N1^{-kl r} w_N1^{-16 kh r}.  Loads: four 128-byte row runs
// per instruction; stores: four 128-byte runs of U (k fastest).  STREAM:
// non-temporal stores (ws is read once, by pass 2: measured 10 us faster
// over the first two passes than plain stores at 2^24).
template <bool STREAM>
__global__ __launch_bounds__(kSymThreads) void sym_first_kernel(SymPass P)
{
    __shared__ float2 lds[16 * kPlaneK];
    const int tid = threadIdx.x;
    const uint32_t N2 = uint32_t(P.N2);
    const uint32_t r = blockIdx.x / (N2 >> 4);
    const int cl = tid & 15, jl = tid >> 4;
    float2 v[16];
    const float2 *src = P.src + addr::sym1_load_base(N2, blockIdx.x, tid);
#pragma unroll
    for (int jh = 0; jh < 16; ++jh) v[jh] = src[addr::sym1_load_off(N2, jh)];
    // every twiddle factor, issued behind the data loads
    float2 t256[16], b[16];
#pragma unroll
    for (int k = 1; k < 16; ++k) t256[k] = root_of(P.tw, P.log2L, 8, uint32_t(jl * k));   // w_256^{-jl kl}
    const int kl = tid & 15, cl2 = tid >> 4;
    const float2 a = root_of(P.tw, P.log2L, 12, uint32_t(kl) * r);                       // w_N1^{-kl r}
#pragma unroll
    for (int kh = 0; kh < 16; ++kh) b[kh] = root_of(P.tw, P.log2L, 12, 16u * kh * r);   // w_N1^{-16 kh r}
    if (P.conj_in) {
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i].y = -v[i].y;
    }
    dft_regs<4>(v);
#pragma unroll
    for (int k = 1; k < 16; ++k) v[k] = cmul(v[k], t256[k]);
#pragma unroll
    for (int k = 0; k < 16; ++k) lds[k * kPlaneK + jl * 16 + cl] = v[k];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = lds[kl * kPlaneK + j * 16 + cl2];
    dft_regs<4>(v);
    float2 *dst = P.dst + addr::sym1_store_base(N2, blockIdx.x, tid);
#pragma unroll
    for (int kh = 0; kh < 16; ++kh) {
        const float2 y = cmul(v[kh], cmul(a, b[kh]));
        float2 *d = dst + addr::sym1_store_off(N2, kh);
        if constexpr (STREAM)
            st2_stream(d, y);
        else
            *d = y;
    }
}

// Pass 2.  Workgroup (jc, kb) owns k = 16 kb + kk and the columns
// c = jc + 256 rr: thread (kk, rr) reads U[c][r][k] (r < 16; a 2 KiB run
// per thread group of 16, last use), transforms over r (-> s,
// v = k + 256 s), applies w_N^{-v c} = w_N^{-k c} w_{16 N2}^{-s jc}
// w_256^{-s rr}; thread (kk, s) then transforms over rr (-> q0), applies
// w_N2^{-q0 jc} and stores W at row 16 jc + q0, columns v (four 128-byte runs
// per instruction).  w_{16 N2}^{-s jc} is the same for the whole workgroup
// and comes from a 16 x 256 table (one scalar load per s).  Measured at 2^24
// against the first version (workspace U[c][r][k] with k contiguous, kb
// fastest, padded LDS, the factor as a product of two-level table entries):
// 54 against 63 us, and pass 1, which now stores 128-byte runs, 45 against
// 50 us.  Five waves per SIMD (96 VGPRs, 32 KiB of LDS).
__global__ __launch_bounds__(kSymThreads) __attribute__((amdgpu_waves_per_eu(5))) void sym_middle_kernel(SymPass P)
{
    __shared__ float2 lds[16 * 256];
    const int tid = threadIdx.x;
    const uint32_t N1 = uint32_t(P.N1), N2 = uint32_t(P.N2);
    const uint32_t blk = addr::sym2_block(blockIdx.x);
    const uint32_t kb = blk & 15, jc = blk >> 4;
    const int kk = tid & 15, rr = tid >> 4;
    const uint32_t c = jc + 256u * rr, k = 16u * kb + kk;
    float2 v[16];
    const float2 *src = P.src + addr::sym2_load_base(N2, blk, tid);
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = ld2_last(src + addr::sym2_load_off(r));  // last use
    const uint32_t nmask = uint32_t((uint64_t(1) << P.log2N) - 1), lomask = (1u << P.log2Lo) - 1u;
    const uint32_t e1 = (k * c) & nmask;
    const float2 h1 = P.tw_hi[e1 >> P.log2Lo], l1 = P.tw_lo[e1 & lomask];
    float2 t2[16], t3[16], t4[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        t2[s] = P.tw_sj[s * 256 + jc];                           // w_{16 N2}^{-s jc}
        t3[s] = root_of(P.tw, P.log2L, 8, uint32_t(s * rr));    // w_256^{-s rr}
        t4[s] = root_of(P.tw, P.log2L, 12, uint32_t(s) * jc);  // w_N2^{-q0 jc}, q0 = s
    }
    dft_regs<4>(v);
    const float2 t1 = cmul(h1, l1);
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        v[s] = cmul(v[s], cmul(t1, cmul(t2[s], t3[s])));
        lds[s * 256 + ((rr ^ (s & 1)) << 4) + kk] = v[s];
    }
    __syncthreads();
    const int s2 = tid >> 4;
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = lds[s2 * 256 + ((i ^ (s2 & 1)) << 4) + kk];
    dft_regs<4>(v);
    float2 *dst = P.dst + addr::sym2_store_base(N1, blk, tid);
#pragma unroll
    for (int q0 = 0; q0 < 16; ++q0) dst[addr::sym2_store_off(N1, q0)] = q0 ? cmul(v[q0], t4[q0]) : v[q0];
}

// Pass 3.  Workgroup (q0, vb) transforms columns v = 16 vb + cl over the rows
// 16 jc + q0, jc = jl + 16 jh: radix 16 over jh by thread (cl, jl), twiddle
// w_256^{-jl kl}, radix 16 over jl by thread (cl, kl), q = kl + 16 kh, stored
// to row q0 + 16 q (four 128-byte runs per instruction).  In place.
__global__ __launch_bounds__(kSymThreads) void sym_last_kernel(SymPass P)
{
    __shared__ float2 lds[16 * kPlaneR];
    const int tid = threadIdx.x;
    const uint32_t N1 = uint32_t(P.N1);
    const int cl = tid & 15, jl = tid >> 4;
    const float2 *src = P.src + addr::sym3_load_base(N1, blockIdx.x, tid);
    float2 v[16];
#pragma unroll
    for (int jh = 0; jh < 16; ++jh) v[jh] = src[addr::sym3_load_off(N1, jh)];
    float2 t256[16];
#pragma unroll
    for (int k = 1; k < 16; ++k) t256[k] = root_of(P.tw, P.log2L, 8, uint32_t(jl * k));
    dft_regs<4>(v);
#pragma unroll
    for (int k = 1; k < 16; ++k) v[k] = cmul(v[k], t256[k]);
#pragma unroll
    for (int k = 0; k < 16; ++k) lds[k * kPlaneR + jl * 16 + cl] = v[k];
    __syncthreads();
    const int kl = tid >> 4;
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = lds[kl * kPlaneR + j * 16 + cl];
    dft_regs<4>(v);
    float2 *dst = P.dst + addr::sym3_store_base(N1, blockIdx.x, tid);
#pragma unroll
    for (int kh = 0; kh < 16; ++kh)
        dst[addr::sym3_store_off(N1, kh)] = P.out_scale != 0.f ? conj_scale(v[kh], P.out_scale) : v[kh];
}

bool sym_shape_ok(const SymPass &p)
{
    return p.N1 == 4096 && p.N2 == 4096 && p.log2L >= 12 && p.log2N == 24 && p.src && p.dst && p.tw && p.tw_hi &&
           p.tw_lo && p.tw_sj;
}

}  // namespace

hipError_t launch_sym_first(const SymPass &p, hipStream_t s)
{
    if (!sym_shape_ok(p)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sym_first_kernel<true>, dim3(addr::sym1_groups(uint32_t(p.N2))), dim3(kSymThreads), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_sym_middle(const SymPass &p, hipStream_t s)
{
    if (!sym_shape_ok(p)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sym_middle_kernel, dim3(addr::sym2_groups(uint32_t(p.N1), uint32_t(p.N2))), dim3(kSymThreads), 0,
                       s, p);
    return hipGetLastError();
}

hipError_t launch_sym_last(const SymPass &p, hipStream_t s)
{
    if (!sym_shape_ok(p)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sym_last_kernel, dim3(addr::sym3_groups(uint32_t(p.N1))), dim3(kSymThreads), 0, s, p);
    return hipGetLastError();
}

}  // namespace paco
