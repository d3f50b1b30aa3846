// The symmetric split form (sym.hip) with every radix-16 butterfly on the
// MFMA units, in the split 16-bit forms of stages.h (FP16x3, BF16x3,
// BF16x6).  Same passes, buffers, twiddles and HBM access pattern as the
// FP32 kernels; only the 16-point transforms differ.
//
// Operand layout.  A wave owns the 64 butterflies of the FP32 kernel's 64
// threads, as four groups G of 16: butterfly 16 G + n of wave w is FP32
// thread 64 w + 16 G + n.  Lane l (n = l & 15, kb = l >> 4) holds, for every
// group, only its 8 real MFMA operands: inputs 8 (kb & 1) .. +8, real parts
// for kb < 2 and imaginary parts otherwise; afterwards it holds the outputs
// m = 4 kb .. 4 kb + 3 of butterfly n.  Stage-0 operands come straight from
// HBM: lanes l and l ^ 32 need the two components of the same 8 items, so
// each loads 4 whole items and the pair swaps the other component through a
// cross-lane shuffle.  Outputs go, with the next stage's twiddle, straight
// to the exchange positions the FP32 kernel uses, and after the second
// stage straight to HBM: the LDS traffic of an FP32 stage, no scratch.
// Butterfly n runs along the 16 adjacent columns (or items) of the HBM
// access, so every load and store instruction still moves whole 128-byte
// runs.

#include "stages.h"

namespace paco {
namespace {

constexpr int kPlaneK = 260;  // the exchange layouts of sym.hip
constexpr int kPlaneR = 272;

__device__ __forceinline__ float2 root_of(const float2 *tw, int log2L, int log2M, uint32_t m)
{
    return tw[(m & ((1u << log2M) - 1u)) << (log2L - log2M)];
}

// The radix-16 DFT matrix as this lane's split A operands: row m = n of
// [Wr, -Wi] (real outputs) and [Wi, Wr] (imaginary outputs), columns
// 8 kb .. 8 kb + 7, W[m][k] = w_16^{-mk}; the FP32 values come from the
// plan's table (w16_operands: evaluated with a lane-dependent index on the
// device, the lookup compiled into hundreds of branches per launch).
template <int PREC>
struct MfW16 {
    MfSplit<PREC> Ar, Ai;
    __device__ MfW16(const float *w16, int lane)
    {
        const float4 *t = reinterpret_cast<const float4 *>(w16 + 16 * lane);
        const float4 a0 = t[0], a1 = t[1], b0 = t[2], b1 = t[3];
        const float ar[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
        const float ai[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
        Ar = mf_split<PREC>(ar);
        Ai = mf_split<PREC>(ai);
    }
    // One group's 16 butterflies: x = this lane's 8 operands, o = its 4
    // outputs m = 4 kb + i.  FP16x3: the butterfly's 32 reals (lanes n,
    // n + 16, n + 32, n + 48) are scaled by one power of two into [1/2, 1)
    // and back (exact).
    __device__ __forceinline__ void dft(float (&x)[8], float2 (&o)[4]) const
    {
        int e = 0;
        if constexpr (PREC == kPrecFP16x3) {
            float amax = 0.f;
#pragma unroll
            for (int i = 0; i < 8; ++i) amax = fmaxf(amax, fabsf(x[i]));
            amax = fmaxf(amax, __shfl_xor(amax, 16));
            amax = fmaxf(amax, __shfl_xor(amax, 32));
            if (amax > 0.f) (void)frexpf(amax, &e);
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = ldexpf(x[i], -e);
        }
        const MfSplit<PREC> B = mf_split<PREC>(x);
        const mf_f32x4 yr = mf_product<PREC>(Ar, B), yi = mf_product<PREC>(Ai, B);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            o[i] = make_float2(yr[i], yi[i]);
            if constexpr (PREC == kPrecFP16x3) o[i] = make_float2(ldexpf(o[i].x, e), ldexpf(o[i].y, e));
        }
    }
};

// Stage-0 operands of one group from four whole items per lane: it[k] is
// item 8 (kb & 1) + (comp ? 4 + k : k) of the lane's butterfly; the pair l,
// l ^ 32 swaps components.  conj: the inverse's input map (negate the
// imaginary parts).
__device__ __forceinline__ void mf_swap_in(const float2 (&it)[4], float (&x)[8], int comp, bool conj)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float recv = __shfl_xor(comp ? it[k].x : it[k].y, 32);
        x[k] = comp ? recv : it[k].x;
        x[4 + k] = comp ? it[k].y : recv;
    }
    if (conj && comp) {
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = -x[i];
    }
}

// Pass 1 (see sym.hip): stage 1 butterfly (cl = n, jl = 4 w + G) over jh,
// stage 2 butterfly (kl = n, cl = 4 w + G) over jl.
template <int PREC>
__global__ __launch_bounds__(256) void sym_first_mf_kernel(SymPass P)
{
    __shared__ float2 lds[16 * kPlaneK];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int n = lane & 15, kb = lane >> 4, comp = kb >> 1, half = kb & 1;
    const uint32_t N2 = uint32_t(P.N2);
    const uint32_t r = blockIdx.x / (N2 >> 4);
    const MfW16<PREC> W(P.w16, lane);
    float x[4][8];
    {
        float2 it[4][4];
#pragma unroll
        for (int G = 0; G < 4; ++G) {
            const float2 *src = P.src + addr::sym1_load_base(N2, blockIdx.x, uint32_t(n + 16 * (4 * w + G)));
#pragma unroll
            for (int k = 0; k < 4; ++k) it[G][k] = src[addr::sym1_load_off(N2, uint32_t(8 * half + (comp ? 4 + k : k)))];
        }
#pragma unroll
        for (int G = 0; G < 4; ++G) mf_swap_in(it[G], x[G], comp, P.conj_in != 0);
    }
    float2 o[4][4];
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        W.dft(x[G], o[G]);
        const int jl = 4 * w + G;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = 4 * kb + i;
            lds[m * kPlaneK + jl * 16 + n] = cmul(o[G][i], root_of(P.tw, P.log2L, 8, uint32_t(jl * m)));
        }
    }
    __syncthreads();
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        const int cl2 = 4 * w + G;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            x[G][i] = reinterpret_cast<const float *>(&lds[n * kPlaneK + (8 * half + i) * 16 + cl2])[comp];
        W.dft(x[G], o[G]);
    }
    // outputs kh = 4 kb + i of butterfly (kl = n, c = 16 cb + cl2), times
    // w_N1^{-k r}, k = n + 16 kh
    const float2 a = root_of(P.tw, P.log2L, 12, uint32_t(n) * r);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t kh = uint32_t(4 * kb + i);
        const float2 t = cmul(a, root_of(P.tw, P.log2L, 12, 16u * kh * r));
#pragma unroll
        for (int G = 0; G < 4; ++G) {
            float2 *d = P.dst + addr::sym1_store_base(N2, blockIdx.x, uint32_t(n + 16 * (4 * w + G)));
            st2_stream(d + addr::sym1_store_off(N2, kh), cmul(o[G][i], t));
        }
    }
}

// Pass 2: stage 1 butterfly (kk = n, rr = 4 w + G) over r, stage 2 butterfly
// (kk = n, s = 4 w + G) over rr.
template <int PREC>
__global__ __launch_bounds__(256) void sym_middle_mf_kernel(SymPass P)
{
    __shared__ float2 lds[16 * 256];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int n = lane & 15, kb = lane >> 4, comp = kb >> 1, half = kb & 1;
    const uint32_t N1 = uint32_t(P.N1), N2 = uint32_t(P.N2);
    const uint32_t blk = addr::sym2_block(blockIdx.x);
    const uint32_t jc = blk >> 4, k = 16u * (blk & 15) + n;
    const MfW16<PREC> W(P.w16, lane);
    float x[4][8];
    {
        float2 it[4][4];
#pragma unroll
        for (int G = 0; G < 4; ++G) {
            const float2 *src = P.src + addr::sym2_load_base(N2, blk, uint32_t(n + 16 * (4 * w + G)));
#pragma unroll
            for (int q = 0; q < 4; ++q) it[G][q] = ld2_last(src + addr::sym2_load_off(uint32_t(8 * half + (comp ? 4 + q : q))));
        }
#pragma unroll
        for (int G = 0; G < 4; ++G) mf_swap_in(it[G], x[G], comp, false);
    }
    const uint32_t nmask = uint32_t((uint64_t(1) << P.log2N) - 1), lomask = (1u << P.log2Lo) - 1u;
    float2 o[4][4];
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        W.dft(x[G], o[G]);
        const uint32_t rr = uint32_t(4 * w + G), c = jc + 256u * rr;
        const uint32_t e1 = (k * c) & nmask;
        const float2 t1 = cmul(P.tw_hi[e1 >> P.log2Lo], P.tw_lo[e1 & lomask]);  // w_N^{-k c}
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int s = 4 * kb + i;
            const float2 t = cmul(t1, cmul(P.tw_sj[s * 256 + jc], root_of(P.tw, P.log2L, 8, uint32_t(s) * rr)));
            lds[s * 256 + ((int(rr) ^ (s & 1)) << 4) + n] = cmul(o[G][i], t);
        }
    }
    __syncthreads();
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        const int s2 = 4 * w + G;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            x[G][i] = reinterpret_cast<const float *>(&lds[s2 * 256 + (((8 * half + i) ^ (s2 & 1)) << 4) + n])[comp];
        W.dft(x[G], o[G]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t q0 = uint32_t(4 * kb + i);
        const float2 t4 = root_of(P.tw, P.log2L, 12, q0 * jc);  // w_N2^{-q0 jc}
#pragma unroll
        for (int G = 0; G < 4; ++G) {
            float2 *d = P.dst + addr::sym2_store_base(N1, blk, uint32_t(n + 16 * (4 * w + G)));
            d[addr::sym2_store_off(N1, q0)] = q0 ? cmul(o[G][i], t4) : o[G][i];
        }
    }
}

// Pass 3: stage 1 butterfly (cl = n, jl = 4 w + G) over jh, stage 2
// butterfly (cl = n, kl = 4 w + G) over jl; in place.
template <int PREC>
__global__ __launch_bounds__(256) void sym_last_mf_kernel(SymPass P)
{
    __shared__ float2 lds[16 * kPlaneR];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int n = lane & 15, kb = lane >> 4, comp = kb >> 1, half = kb & 1;
    const uint32_t N1 = uint32_t(P.N1);
    const MfW16<PREC> W(P.w16, lane);
    float x[4][8];
    {
        float2 it[4][4];
#pragma unroll
        for (int G = 0; G < 4; ++G) {
            const float2 *src = P.src + addr::sym3_load_base(N1, blockIdx.x, uint32_t(n + 16 * (4 * w + G)));
#pragma unroll
            for (int q = 0; q < 4; ++q) it[G][q] = src[addr::sym3_load_off(N1, uint32_t(8 * half + (comp ? 4 + q : q)))];
        }
#pragma unroll
        for (int G = 0; G < 4; ++G) mf_swap_in(it[G], x[G], comp, false);
    }
    float2 o[4][4];
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        W.dft(x[G], o[G]);
        const int jl = 4 * w + G;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = 4 * kb + i;
            lds[m * kPlaneR + jl * 16 + n] = cmul(o[G][i], root_of(P.tw, P.log2L, 8, uint32_t(jl * m)));
        }
    }
    __syncthreads();
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        const int kl = 4 * w + G;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            x[G][i] = reinterpret_cast<const float *>(&lds[kl * kPlaneR + (8 * half + i) * 16 + n])[comp];
        W.dft(x[G], o[G]);
    }
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        float2 *d = P.dst + addr::sym3_store_base(N1, blockIdx.x, uint32_t(n + 16 * (4 * w + G)));
#pragma unroll
        for (int i = 0; i < 4; ++i)
            d[addr::sym3_store_off(N1, uint32_t(4 * kb + i))] =
                P.out_scale != 0.f ? conj_scale(o[G][i], P.out_scale) : o[G][i];
    }
}

template <int PREC>
hipError_t launch_pass(int pass, const SymPass &p, hipStream_t s)
{
    if (pass == 1)
        hipLaunchKernelGGL(sym_first_mf_kernel<PREC>, dim3(addr::sym1_groups(uint32_t(p.N2))), dim3(256), 0, s, p);
    else if (pass == 2)
        hipLaunchKernelGGL(sym_middle_mf_kernel<PREC>, dim3(addr::sym2_groups(uint32_t(p.N1), uint32_t(p.N2))),
                           dim3(256), 0, s, p);
    else
        hipLaunchKernelGGL(sym_last_mf_kernel<PREC>, dim3(addr::sym3_groups(uint32_t(p.N1))), dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace

void w16_operands(float *t)
{
    for (int lane = 0; lane < 64; ++lane) {
        const int n = lane & 15, kb = lane >> 4;
        for (int i = 0; i < 8; ++i) {
            const int k = 8 * kb + i;
            t[16 * lane + i] = kb < 2 ? cos16(n * k) : cos16(n * (k - 16) + 12);
            t[16 * lane + 8 + i] = kb < 2 ? -cos16(n * k + 12) : cos16(n * (k - 16));
        }
    }
}

hipError_t launch_sym_mf(int prec, int pass, const SymPass &p, hipStream_t s)
{
    if (!(p.N1 == 4096 && p.N2 == 4096 && p.log2L >= 12 && p.log2N == 24 && p.src && p.dst && p.tw && p.tw_hi &&
          p.tw_lo && p.tw_sj && p.w16) ||
        pass < 1 || pass > 3)
        return hipErrorInvalidValue;
    switch (prec) {
    case kPrecFP16x3: return launch_pass<kPrecFP16x3>(pass, p, s);
    case kPrecBF16x3: return launch_pass<kPrecBF16x3>(pass, p, s);
    case kPrecBF16x6: return launch_pass<kPrecBF16x6>(pass, p, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace paco
