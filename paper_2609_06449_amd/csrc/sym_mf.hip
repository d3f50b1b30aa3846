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

// Exchange buffers addressed by addr::mf1_*, mf2_* and mf3_* (passes 1, 2
// and 3): bank-conflict free for the stores of stage-1 results and the
// component loads of stage 2.
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
    // outputs m = 4 kb + i.  FP16x3 splits x 2^-e (e: the power of two of
    // the butterfly or of the workgroup's tile) and leaves the outputs in
    // units of 2^e: the caller scales back, mostly inside a twiddle factor
    // it multiplies by anyway.
    __device__ __forceinline__ void dft(const float (&x)[8], float2 (&o)[4], int e = 0) const
    {
        const MfSplit<PREC> B = mf_split<PREC>(x, e);
        const mf_f32x4 yr = mf_product<PREC>(Ar, B), yi = mf_product<PREC>(Ai, B);
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = make_float2(yr[i], yi[i]);
    }
};

// FP16x3 scales of passes 1 and 3: a power of two per workgroup tile
// instead of per butterfly: the tile's operands share one exponent range
// (values far below the tile's largest keep their absolute accuracy, the
// relative one of the largest), the scale costs one reduction per pass
// instead of one per group, and stage 1's outputs feed stage 2 without
// rescaling.  (Pass 2 keeps the scale per butterfly: there the reduction had
// to wait for all of the wave's loads.)  max |x| over the wave's 64 lanes x
// 32 operands:
__device__ __forceinline__ float wave_absmax(const float (&x)[4][8])
{
    float m = 0.f;
#pragma unroll
    for (int G = 0; G < 4; ++G)
#pragma unroll
        for (int i = 0; i < 8; ++i) m = fmaxf(m, fabsf(x[G][i]));
    m = max_over_kb(m);
    // the 16 lanes of a row, with DPP moves (no LDS): swaps of neighbours
    // and of lane pairs (quad_perm [1,0,3,2], [2,3,0,1]), then the mirror of
    // each half row and of the row
    m = fmaxf(m, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(m), 0xB1, 0xF, 0xF, false)));
    m = fmaxf(m, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(m), 0x4E, 0xF, 0xF, false)));
    m = fmaxf(m, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(m), 0x141, 0xF, 0xF, false)));
    m = fmaxf(m, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(m), 0x140, 0xF, 0xF, false)));
    return m;
}
// e with m 2^-e in [1/2, 1) (0 for m = 0; at least -100, so that 2^-e and
// 2^(11-e) stay finite for subnormal tiles), the same in every lane
__device__ __forceinline__ int scale_of(float m)
{
    int e = 0;
    if (m > 0.f) (void)frexpf(m, &e);
    return __builtin_amdgcn_readfirstlane(e < -100 ? -100 : e);
}
// Workgroup scale of passes 1 and 3: the four wave maxima meet in exchange
// slots that stage 1 does not store to (spare: a float2 item index).
__device__ __forceinline__ int tile_scale(const float (&x)[4][8], float2 *lds, int spare, int lane, int w)
{
    float *red = reinterpret_cast<float *>(lds + spare);
    const float m = wave_absmax(x);
    if (lane == 0) red[w] = m;
    __syncthreads();
    return scale_of(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])));
}

// Stage-0 operands of one group (mf_swap_in); conj: the inverse's input map
// (negate the imaginary parts, held by lanes l >= 32).
__device__ __forceinline__ void mf_load_ops(const float2 (&it)[4], float (&x)[8], int comp, bool conj)
{
    mf_swap_in(it, x);
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
    __shared__ float2 lds[addr::kMf1Items];
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
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
        for (int G = 0; G < 4; ++G) mf_load_ops(it[G], x[G], comp, P.conj_in != 0);
    }
    // every twiddle loaded right behind the data (LDS caps the kernel at four
    // waves per SIMD, so the registers are there): stage 1's w_256^{-jl m}
    // and the outputs' w_N1^{-k r}, k = n + 16 kh, kh = 4 kb + i
    float2 t1[4][4], t2[4];
#pragma unroll
    for (int G = 0; G < 4; ++G)
#pragma unroll
        for (int i = 0; i < 4; ++i) t1[G][i] = root_of(P.tw, P.log2L, 8, uint32_t((4 * w + G) * (4 * kb + i)));
    const float2 a = root_of(P.tw, P.log2L, 12, uint32_t(n) * r);
#pragma unroll
    for (int i = 0; i < 4; ++i) t2[i] = root_of(P.tw, P.log2L, 12, 16u * uint32_t(4 * kb + i) * r);
    // FP16x3: one scale for the tile; stage 1's outputs (below 16 in its
    // units) feed stage 2 unscaled, the final twiddle scales back
    const int e = PREC == kPrecFP16x3 ? tile_scale(x, lds, addr::kMf1Spare, lane, w) : 0;
    float2 o[4][4];
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        W.dft(x[G], o[G], e);
        const int jl = 4 * w + G;
#pragma unroll
        for (int i = 0; i < 4; ++i) lds[addr::mf1_store(kb, i, jl, n)] = cmul(o[G][i], t1[G][i]);
    }
    __syncthreads();
    const float *ldf = reinterpret_cast<const float *>(lds) + comp;
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        const int cl2 = 4 * w + G;
#pragma unroll
        for (int i = 0; i < 8; ++i) x[G][i] = ldf[2 * addr::mf1_load(n, half, i, cl2)];
        W.dft(x[G], o[G]);
    }
    // outputs kh = 4 kb + i of butterfly (kl = n, c = 16 cb + cl2)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t kh = uint32_t(4 * kb + i);
        float2 t = cmul(a, t2[i]);
        if constexpr (PREC == kPrecFP16x3) t = make_float2(ldexpf(t.x, e), ldexpf(t.y, e));
#pragma unroll
        for (int G = 0; G < 4; ++G) {
            float2 *d = P.dst + addr::sym1_store_base(N2, blockIdx.x, uint32_t(n + 16 * (4 * w + G)));
            st2_stream(d + addr::sym1_store_off(N2, kh), cmul(o[G][i], t));
        }
    }
}

// Pass 2: stage 1 butterfly (kk = n, rr = 4 w + G) over r, stage 2 butterfly
// (kk = n, s = 4 w + G) over rr.  The twiddle of stage-1 output s of group G
// is w_N^{-c (k + L s)}, c = jc + L rr, s = 4 kb + i: the first (i = 0)
// from the two-level table, each next one times w_{16 N2}^{-c}, which is the
// same for the whole wave (scalar loads).  That keeps the twiddle loads few
// (one pair per group) and issued right behind the data loads; with one
// lookup per output the compiler spread 32 loads, each waited for, between
// the butterflies.
template <int PREC, int LL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PREC == kPrecBF16x6 ? 4 : 5))) void sym_middle_mf_kernel(SymPass P)
{
    __shared__ float2 lds[16 * 256];
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = lane & 15, kb = lane >> 4, comp = kb >> 1, half = kb & 1;
    const uint32_t N1 = uint32_t(P.N1), N2 = uint32_t(P.N2);
    const uint32_t blk = addr::sym2_block(blockIdx.x, LL, LL);
    const uint32_t jc = blk >> (LL - 4), k = 16u * (blk & ((1u << (LL - 4)) - 1u)) + n;
    float2 it[4][4];
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        const float2 *src = P.src + addr::sym2_load_base(N2, blk, uint32_t(n + 16 * (4 * w + G)), LL, LL);
#pragma unroll
        for (int q = 0; q < 4; ++q) it[G][q] = ld2_last(src + addr::sym2_load_off(uint32_t(8 * half + (comp ? 4 + q : q))));
    }
    const uint32_t nmask = uint32_t((uint64_t(1) << P.log2N) - 1), lomask = (1u << P.log2Lo) - 1u;
    float2 th[4], tl[4];  // w_N^{-c (k + 4 L kb)} as its two table factors
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        const uint32_t c = jc + (uint32_t(4 * w + G) << LL);
        const uint32_t e = (c * (k + (uint32_t(kb) << (LL + 2)))) & nmask;
        th[G] = P.tw_hi[e >> P.log2Lo];
        tl[G] = P.tw_lo[e & lomask];
    }
    const MfW16<PREC> W(P.w16, lane);
    float x[4][8];
#pragma unroll
    for (int G = 0; G < 4; ++G) mf_swap_in(it[G], x[G]);
    // FP16x3: one scale per butterfly (mf_scale_exp), scaled back inside the
    // twiddle factor; a scale per wave measured slower here, since no group
    // could start before the wave's last load had arrived
    const float2 sj = P.tw_sj[(1u << LL) + jc];  // w_{16 N2}^{-jc}
    float2 o[4][4];
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        const int e1 = PREC == kPrecFP16x3 ? mf_scale_exp(x[G]) : 0;
        W.dft(x[G], o[G], e1);
        const int rr = 4 * w + G;
        const float2 step = cmul(sj, root_of(P.tw, P.log2L, 8, uint32_t(rr)));  // w_{16 N2}^{-c}
        float2 t = cmul(th[G], tl[G]);
        if constexpr (PREC == kPrecFP16x3) t = make_float2(ldexpf(t.x, e1), ldexpf(t.y, e1));
#pragma unroll
        for (int i = 0; i < 4; ++i) {  // output s = 4 kb + i
            lds[addr::mf2_store(kb, i, rr, n)] = cmul(o[G][i], t);
            if (i < 3) t = cmul(t, step);
        }
    }
    __syncthreads();
    float2 t4[4];  // w_N2^{-q0 jc}, q0 = 4 kb + i
#pragma unroll
    for (int i = 0; i < 4; ++i) t4[i] = root_of(P.tw, P.log2L, LL + 4, uint32_t(4 * kb + i) * jc);
    const float *ldf = reinterpret_cast<const float *>(lds) + comp;
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        const int s2 = 4 * w + G;
#pragma unroll
        for (int i = 0; i < 8; ++i) x[G][i] = ldf[2 * addr::mf2_load(s2, half, i, n)];
        const int e2 = PREC == kPrecFP16x3 ? mf_scale_exp(x[G]) : 0;
        W.dft(x[G], o[G], e2);
        if constexpr (PREC == kPrecFP16x3) {
#pragma unroll
            for (int i = 0; i < 4; ++i) o[G][i] = make_float2(ldexpf(o[G][i].x, e2), ldexpf(o[G][i].y, e2));
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t q0 = uint32_t(4 * kb + i);
#pragma unroll
        for (int G = 0; G < 4; ++G) {
            float2 *d = P.dst + addr::sym2_store_base(N1, blk, uint32_t(n + 16 * (4 * w + G)), LL);
            d[addr::sym2_store_off(N1, q0)] = q0 ? cmul(o[G][i], t4[i]) : o[G][i];
        }
    }
}

// Pass 3: stage 1 butterfly (cl = n, jl = 4 w + G) over jh, stage 2
// butterfly (cl = n, kl = 4 w + G) over jl; in place.
template <int PREC>
__global__ __launch_bounds__(256) void sym_last_mf_kernel(SymPass P)
{
    __shared__ float2 lds[addr::kMf1Items];
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
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
        for (int G = 0; G < 4; ++G) mf_swap_in(it[G], x[G]);
    }
    float2 t1[4][4];  // w_256^{-jl m}, loaded right behind the data (as in pass 1)
#pragma unroll
    for (int G = 0; G < 4; ++G)
#pragma unroll
        for (int i = 0; i < 4; ++i) t1[G][i] = root_of(P.tw, P.log2L, 8, uint32_t((4 * w + G) * (4 * kb + i)));
    // FP16x3: one scale for the tile (as in pass 1), scaled back at the store
    const int e = PREC == kPrecFP16x3 ? tile_scale(x, lds, addr::kMf3Spare, lane, w) : 0;
    float2 o[4][4];
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        W.dft(x[G], o[G], e);
        const int jl = 4 * w + G;
#pragma unroll
        for (int i = 0; i < 4; ++i) lds[addr::mf3_store(kb, i, jl, n)] = cmul(o[G][i], t1[G][i]);
    }
    __syncthreads();
    const float *ldf = reinterpret_cast<const float *>(lds) + comp;
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        const int kl = 4 * w + G;
#pragma unroll
        for (int i = 0; i < 8; ++i) x[G][i] = ldf[2 * addr::mf3_load(kl, half, i, n)];
        W.dft(x[G], o[G]);
    }
    const float osc = ldexpf(1.0f, e);  // 1 except in FP16x3
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        float2 *d = P.dst + addr::sym3_store_base(N1, blockIdx.x, uint32_t(n + 16 * (4 * w + G)));
#pragma unroll
        for (int i = 0; i < 4; ++i)
            d[addr::sym3_store_off(N1, uint32_t(4 * kb + i))] =
                P.out_scale != 0.f ? conj_scale(o[G][i], P.out_scale * osc) : make_float2(o[G][i].x * osc, o[G][i].y * osc);
    }
}

// ---- L = 512 (N1 = N2 = 8192): passes 1 and 3, 512 threads -----------------
// Stage A as at L = 256 (butterfly (cl = n, jl = 4 w + G) over jh, j = jl +
// 32 jh).  Stage B: the 32-point transform over jl = jp + 2 jm of each (ka,
// column) as radix 16 over jm in two MFMA groups G = 2 g + jp of one wave,
// twiddle w_32^{-jp kb'}, and the radix-2 step between the two groups in
// registers (both halves of a transform sit in the same lane): outputs
// kb' + 16 kc, k = ka + 16 (kb' + 16 kc).  FP16x3: one scale for the tile,
// the eight wave maxima met in a small LDS array.

// the tile's scale from its eight waves' maxima
__device__ __forceinline__ int tile_scale8(const float (&x)[4][8], float *red, int lane, int w)
{
    const float m = wave_absmax(x);
    if (lane == 0) red[w] = m;
    __syncthreads();
    float t = red[0];
#pragma unroll
    for (int i = 1; i < 8; ++i) t = fmaxf(t, red[i]);
    return scale_of(t);
}

// stage-B tail of one transform: twiddle its jp = 1 half by w_32^{-kb'}
// (kb' = 4 kb + i; twL: w_512^{-m}) and combine the halves (outputs kb' in
// o0, kb' + 16 in o1)
__device__ __forceinline__ void radix2_pair(float2 (&o0)[4], float2 (&o1)[4], const float2 *twL, uint32_t kb)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float2 y0 = o0[i], y1 = cmul(o1[i], twL[(4 * kb + i) << 4]);
        o0[i] = make_float2(y0.x + y1.x, y0.y + y1.y);
        o1[i] = make_float2(y0.x - y1.x, y0.y - y1.y);
    }
}

// Persistent and software-pipelined like the FP32 kernels of these passes
// (sym.hip): workgroup g of G takes tiles g, g + G, ..., issues the next
// tile's loads right after stage A and keeps the twiddle factors in LDS.
// BF16x6's pass 1 (24 VGPRs of DFT-matrix operands) does not fit the
// 128-VGPR budget of two workgroups per CU without spills, whose reloads
// would wait for the prefetch: it runs one workgroup per CU.
template <int PREC>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(PREC == kPrecBF16x6 ? 2 : 4))) void sym_first_mf_long_kernel(SymPass P,
                                                                                                      uint32_t tiles)
{
    constexpr int LL = 9, L = 1 << LL;
    __shared__ float2 lds[addr::kMfLItems];
    __shared__ float2 twL[L];    // w_512^{-m}
    __shared__ float2 twF[256];  // w_N1^{-m}, m < 256
    __shared__ float red[8];
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = lane & 15, kb = lane >> 4, comp = kb >> 1, half = kb & 1;
    const uint32_t N2 = uint32_t(P.N2);
    const MfW16<PREC> W(P.w16, lane);
    uint32_t t = blockIdx.x;
    float2 it[4][4];
    auto load = [&](uint32_t tile) {
        const uint32_t blk = addr::sym1_block(tile, N2, LL);
#pragma unroll
        for (int G = 0; G < 4; ++G) {
            const uint32_t base = addr::sym1_load_base(N2, blk, uint32_t(n + 16 * (4 * w + G)));
#pragma unroll
            for (int k = 0; k < 4; ++k)
                it[G][k] = *off32(P.src, base + addr::sym1_load_off(N2, uint32_t(8 * half + (comp ? 4 + k : k)), LL));
        }
    };
    int e = 0;  // FP16x3: the tile's scale, from stage A to the stores
    auto stage_a = [&](uint32_t tc) {
        float x[4][8];
#pragma unroll
        for (int G = 0; G < 4; ++G) mf_load_ops(it[G], x[G], comp, P.conj_in != 0);
        e = PREC == kPrecFP16x3 ? tile_scale8(x, red, lane, w) : 0;
        const uint32_t kq = opaque(uint32_t(kb));
#pragma unroll
        for (int G = 0; G < 4; ++G) {
            float2 o[4];
            W.dft(x[G], o, e);
            const int jl = 4 * w + G;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                lds[addr::mf1L_store(kb, i, jl, n)] = cmul(o[i], twL[(uint32_t(jl) * (4 * kq + i)) & (L - 1)]);
        }
        load(tc + gridDim.x < tiles ? tc + gridDim.x : tc);
        __syncthreads();
    };
    load(t < tiles ? t : 0);  // (the launch gives every workgroup a tile)
    twL[tid] = P.tw[uint32_t(tid) << (P.log2L - LL)];
    if (tid < 256) twF[tid] = P.tw[uint32_t(tid) << (P.log2L - LL - 4)];
    __syncthreads();
    if (t < tiles) stage_a(t);
    const float *ldf = reinterpret_cast<const float *>(lds) + comp;
    while (t < tiles) {
        const uint32_t blk = addr::sym1_block(t, N2, LL);
        const uint32_t r = blk / (N2 >> 4);
        float2 o[4][4];
#pragma unroll
        for (int G = 0; G < 4; ++G) {
            float x[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = ldf[2 * addr::mf1L_load(n, half, i, G & 1, 2 * w + (G >> 1))];
            W.dft(x, o[G]);
        }
        const uint32_t kq = opaque(uint32_t(kb));
#pragma unroll
        for (int g = 0; g < 2; ++g) radix2_pair(o[2 * g], o[2 * g + 1], twL, kq);
        // outputs k = ka + 16 (kb' + 16 kc), ka = n, kb' = 4 kb + i, times
        // w_N1^{-k r} = w_N1^{-n r} w_512^{-(kb' + 16 kc) r}
        const float2 a = twF[uint32_t(n) * r];
#pragma unroll
        for (int kc = 0; kc < 2; ++kc)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float2 tw = cmul(a, twL[((4 * kq + i + 16u * kc) * r) & (L - 1)]);
                if constexpr (PREC == kPrecFP16x3) tw = make_float2(ldexpf(tw.x, e), ldexpf(tw.y, e));
#pragma unroll
                for (int g = 0; g < 2; ++g) {
                    const uint32_t d = addr::sym1_store_base(N2, blk, uint32_t(n + 16 * kc + 32 * (2 * w + g)), LL);
                    st2_stream(off32(P.dst, d + addr::sym1_store_off(N2, uint32_t(4 * kb + i))), cmul(o[2 * g + kc][i], tw));
                }
            }
        __syncthreads();
        t += gridDim.x;
        if (t < tiles) stage_a(t);
    }
}

template <int PREC>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void sym_last_mf_long_kernel(SymPass P,
                                                                                                     uint32_t tiles)
{
    constexpr int LL = 9, L = 1 << LL;
    __shared__ float2 lds[addr::kMfLItems];
    __shared__ float2 twL[L];
    __shared__ float red[8];
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = lane & 15, kb = lane >> 4, comp = kb >> 1, half = kb & 1;
    const uint32_t N1 = uint32_t(P.N1);
    const MfW16<PREC> W(P.w16, lane);
    uint32_t t = blockIdx.x;
    float2 it[4][4];
    auto load = [&](uint32_t tile) {
        const uint32_t blk = addr::sym3_block(tile, N1, LL);
#pragma unroll
        for (int G = 0; G < 4; ++G) {
            const uint32_t base = addr::sym3_load_base(N1, blk, uint32_t(n + 16 * (4 * w + G)));
#pragma unroll
            for (int q = 0; q < 4; ++q)
                it[G][q] = *off32(P.src, base + addr::sym3_load_off(N1, uint32_t(8 * half + (comp ? 4 + q : q)), LL));
        }
    };
    int e = 0;
    auto stage_a = [&](uint32_t tc) {
        float x[4][8];
#pragma unroll
        for (int G = 0; G < 4; ++G) mf_swap_in(it[G], x[G]);
        e = PREC == kPrecFP16x3 ? tile_scale8(x, red, lane, w) : 0;
        const uint32_t kq = opaque(uint32_t(kb));
#pragma unroll
        for (int G = 0; G < 4; ++G) {
            float2 o[4];
            W.dft(x[G], o, e);
            const int jl = 4 * w + G;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                lds[addr::mf3L_store(kb, i, jl, n)] = cmul(o[i], twL[(uint32_t(jl) * (4 * kq + i)) & (L - 1)]);
        }
        load(tc + gridDim.x < tiles ? tc + gridDim.x : tc);
        __syncthreads();
    };
    load(t < tiles ? t : 0);
    twL[tid] = P.tw[uint32_t(tid) << (P.log2L - LL)];
    __syncthreads();
    if (t < tiles) stage_a(t);
    const float *ldf = reinterpret_cast<const float *>(lds) + comp;
    while (t < tiles) {
        const uint32_t blk = addr::sym3_block(t, N1, LL);
        const uint32_t kq = opaque(uint32_t(kb));
        const float osc = ldexpf(1.0f, e);  // 1 except in FP16x3
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            float2 o[2][4];
#pragma unroll
            for (int jp = 0; jp < 2; ++jp) {
                float x[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) x[i] = ldf[2 * addr::mf3L_load(2 * w + g, half, i, jp, n)];
                W.dft(x, o[jp]);
            }
            radix2_pair(o[0], o[1], twL, kq);
            // outputs q = ka + 16 (kb' + 16 kc) of column v = 16 vb + n, row q0 + 16 q
#pragma unroll
            for (int kc = 0; kc < 2; ++kc) {
                const uint32_t d = addr::sym3_store_base(N1, blk, uint32_t(n + 16 * kc + 32 * (2 * w + g)), LL);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float2 y = o[kc][i];
                    *off32(P.dst, d + addr::sym3_store_off(N1, uint32_t(4 * kb + i))) =
                        P.out_scale != 0.f ? conj_scale(y, P.out_scale * osc) : make_float2(y.x * osc, y.y * osc);
                }
            }
        }
        __syncthreads();
        t += gridDim.x;
        if (t < tiles) stage_a(t);
    }
}

template <int PREC>
hipError_t launch_pass(int pass, int ll, const SymPass &p, hipStream_t s)
{
    const dim3 g1(addr::sym1_groups(uint32_t(p.N2))), g2(addr::sym2_groups(uint32_t(p.N1), uint32_t(p.N2))),
        g3(addr::sym3_groups(uint32_t(p.N1)));
    if (ll == 8) {
        if (pass == 1)
            hipLaunchKernelGGL(sym_first_mf_kernel<PREC>, g1, dim3(256), 0, s, p);
        else if (pass == 2)
            hipLaunchKernelGGL((sym_middle_mf_kernel<PREC, 8>), g2, dim3(256), 0, s, p);
        else
            hipLaunchKernelGGL(sym_last_mf_kernel<PREC>, g3, dim3(256), 0, s, p);
    } else {
        if (pass == 1)
            hipLaunchKernelGGL(sym_first_mf_long_kernel<PREC>, persistent(g1, p.resident1), dim3(512), 0, s, p, g1.x);
        else if (pass == 2)
            hipLaunchKernelGGL((sym_middle_mf_kernel<PREC, 9>), g2, dim3(256), 0, s, p);
        else
            hipLaunchKernelGGL(sym_last_mf_long_kernel<PREC>, persistent(g3, p.resident3), dim3(512), 0, s, p, g3.x);
    }
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

uint32_t sym_mf_resident_groups(int prec, int pass, const SymPass &p)
{
    if (sym_log2_child(p) != 9 || (pass != 1 && pass != 3)) return 0;
    switch (prec) {
    case kPrecFP16x3:
        return pass == 1 ? resident(sym_first_mf_long_kernel<kPrecFP16x3>, 512) : resident(sym_last_mf_long_kernel<kPrecFP16x3>, 512);
    case kPrecBF16x3:
        return pass == 1 ? resident(sym_first_mf_long_kernel<kPrecBF16x3>, 512) : resident(sym_last_mf_long_kernel<kPrecBF16x3>, 512);
    case kPrecBF16x6:
        return pass == 1 ? resident(sym_first_mf_long_kernel<kPrecBF16x6>, 512) : resident(sym_last_mf_long_kernel<kPrecBF16x6>, 512);
    default: return 0;
    }
}

hipError_t launch_sym_mf(int prec, int pass, const SymPass &p, hipStream_t s)
{
    const int ll = sym_log2_child(p);  // L = 256 or 512 for these forms
    if (!(ll == 8 || ll == 9) || !(p.src && p.dst && p.tw && p.tw_hi && p.tw_lo && p.tw_sj && p.w16) || pass < 1 ||
        pass > 3)
        return hipErrorInvalidValue;
    switch (prec) {
    case kPrecFP16x3: return launch_pass<kPrecFP16x3>(pass, ll, p, s);
    case kPrecBF16x3: return launch_pass<kPrecBF16x3>(pass, ll, p, s);
    case kPrecBF16x6: return launch_pass<kPrecBF16x6>(pass, ll, p, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace paco
