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
#include "paco_internal.h"

namespace paco {
namespace {

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// d * w_16^{-m} for a compile-time m (after unrolling), w_16 = exp(2 pi i/16).
// Constants are cos/sin(2 pi m/16) rounded to float.
__device__ __forceinline__ float2 mul_w16(float2 d, int m)
{
    constexpr float c1 = 0.923879532511286756f;  // cos(pi/8)
    constexpr float s1 = 0.382683432365089772f;  // sin(pi/8)
    constexpr float h = 0.707106781186547524f;   // cos(pi/4)
    switch (m & 15) {
    case 0: return d;
    case 1: return cmul(d, make_float2(c1, -s1));
    case 2: return make_float2(h * (d.x + d.y), h * (d.y - d.x));
    case 3: return cmul(d, make_float2(s1, -c1));
    case 4: return make_float2(d.y, -d.x);
    case 5: return cmul(d, make_float2(-s1, -c1));
    case 6: return make_float2(h * (d.y - d.x), -h * (d.x + d.y));
    case 7: return cmul(d, make_float2(-c1, -s1));
    case 8: return make_float2(-d.x, -d.y);
    case 9: return cmul(d, make_float2(-c1, s1));
    case 10: return make_float2(-h * (d.x + d.y), h * (d.x - d.y));
    case 11: return cmul(d, make_float2(-s1, c1));
    case 12: return make_float2(-d.y, d.x);
    case 13: return cmul(d, make_float2(s1, c1));
    case 14: return make_float2(h * (d.x - d.y), h * (d.x + d.y));
    default: return cmul(d, make_float2(c1, s1));
    }
}

constexpr int bitrev_c(int x, int bits)
{
    int r = 0;
    for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1) << (bits - 1 - i);
    return r;
}

// In-register length-R DFT (R = 2^LR <= 16), natural order in and out:
// radix-2 decimation-in-frequency network, then a compile-time reorder.
template <int LR>
__device__ __forceinline__ void dft_regs(float2 *v)
{
    constexpr int R = 1 << LR;
#pragma unroll
    for (int len = R; len >= 2; len >>= 1) {
        const int half = len >> 1;
#pragma unroll
        for (int base = 0; base < R; base += len) {
#pragma unroll
            for (int k = 0; k < half; ++k) {
                float2 a = v[base + k], b = v[base + k + half];
                v[base + k] = cadd(a, b);
                v[base + k + half] = mul_w16(csub(a, b), k * (16 / len));
            }
        }
    }
    float2 t[R];
#pragma unroll
    for (int k = 0; k < R; ++k) t[k] = v[bitrev_c(k, LR)];
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = t[k];
}

// LDS index with 4 pad items per 64: the radix-16 first-stage writes (row
// stride 16*T items) land on distinct banks.
__device__ __forceinline__ int lpad(int e) { return e + ((e >> 6) << 2); }

// Digit reversal with compile-time digit width TB and digit count ND.
template <int TB, int ND>
__device__ __forceinline__ uint32_t drev(uint32_t x)
{
    uint32_t r = 0;
#pragma unroll
    for (int g = 0; g < ND; ++g) r |= ((x >> (TB * g)) & ((1u << TB) - 1)) << (TB * (ND - 1 - g));
    return r;
}
constexpr int crev(int x, int tb, int nd)
{
    int r = 0;
    for (int g = 0; g < nd; ++g) r |= ((x >> (tb * g)) & ((1 << tb) - 1)) << (tb * (nd - 1 - g));
    return r;
}

// Tile width of the fast kernels: 4096 items per workgroup for short
// transforms, 4 columns (32-byte row runs) for long ones.
constexpr int fast_log2T(int l) { return l >= 10 ? 2 : 12 - l; }

struct Ctx {
    float2 *lds;
    const float2 *twl;
    int tid, nt, log2T;
    char *dst;                 // tile base (column col0 of row 0)
    uint32_t ld8;              // row length in bytes
    uint32_t orow_out, k_out;  // generic: output row = orow_out + pi_out(k) * k_out
    int out_t, out_ell;
};

// Stage S of the Stockham sequence on H column groups.  v[h*EG + i*R + r]
// is operand r of butterfly i of group h; butterfly id g = tid + i*nt of a
// group covers column g mod TG and index j = g / TG (TG columns per group);
// between stages the groups take turns in LDS, which holds n x TG items.
// LT >= 0: compile-time log2 TG.  MODE: -1 generic output rows, 0 digit-
// reversed output rows (Phase I), 1 natural output rows (Phase III), 2 the
// transposed natural output (row = column, n items per row; Phase I of the
// fused pipeline).
template <int LOG2N, int S, int EG, int LT, int MODE, int TB, bool GEN, int H>
__device__ __forceinline__ void run_stage(float2 (&v)[H * EG], const Ctx &c)
{
    constexpr int LR = stage_log2radix(LOG2N, S);
    constexpr int R = 1 << LR;
    constexpr int LNS = stage_log2ns(LOG2N, S);
    constexpr int NB = EG / R;
    constexpr bool last = (S + 1 == stage_count(LOG2N));
    const int log2T = LT >= 0 ? LT : c.log2T;
    const int nt = LT >= 0 ? ((1 << (LOG2N + (LT >= 0 ? LT : 0))) / EG) : c.nt;
    const int Tm = (1 << log2T) - 1;

#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int g = c.tid + i * nt;
        const int j = g >> log2T;
        if constexpr (LNS > 0) {
            // the same twiddles serve every group (same j)
            constexpr int LOW = stage_lo_width(LOG2N, S);
            constexpr int HIW = stage_hi_width(LOG2N, S);
            constexpr int OFF = stage_tw_offset(LOG2N, S);
            const int k = j & ((1 << LNS) - 1);
            const float2 *tlo = c.twl + OFF + (k & (LOW - 1));
            const float2 *thi = c.twl + OFF + (R - 1) * LOW + (k >> 4);
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 w = tlo[(r - 1) * LOW];
                if constexpr (HIW > 0) w = cmul(w, thi[(r - 1) * HIW]);
#pragma unroll
                for (int h = 0; h < H; ++h) v[h * EG + i * R + r] = cmul(v[h * EG + i * R + r], w);
            }
        }
#pragma unroll
        for (int h = 0; h < H; ++h) dft_regs<LR>(&v[h * EG + i * R]);
    }
    if constexpr (!last) {
        constexpr int LR2 = stage_log2radix(LOG2N, S + 1);
        constexpr int R2 = 1 << LR2;
        constexpr int NB2 = EG / R2;
        constexpr int LNR2 = LOG2N - LR2;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            if (S > 0 || h > 0) __syncthreads();  // the previous LDS contents were consumed
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int g = c.tid + i * nt;
                const int t = g & Tm, j = g >> log2T;
                const int idxD = ((j >> LNS) << (LNS + LR)) + (j & ((1 << LNS) - 1));
#pragma unroll
                for (int r = 0; r < R; ++r)
                    c.lds[lpad(((idxD + (r << LNS)) << log2T) + t)] = v[h * EG + i * R + r];
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < NB2; ++i) {
                const int g = c.tid + i * nt;
                const int t = g & Tm, j = g >> log2T;
#pragma unroll
                for (int r = 0; r < R2; ++r)
                    v[h * EG + i * R2 + r] = c.lds[lpad(((j + (r << LNR2)) << log2T) + t)];
            }
        }
        run_stage<LOG2N, S + 1, EG, LT, MODE, TB, GEN, H>(v, c);
    } else {
        // last stage: j < n/R = 2^LNS, outputs are the natural-order rows k = j + r*2^LNS.
        // With H = 2 the groups interleave: group h of tile column t holds
        // column 2t + h, so one 16-byte store writes both groups' items.
        if constexpr (H == 2 && (MODE == 0 || MODE == 1)) {
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int g = c.tid + i * nt;
                const int t = (g & Tm) << 1, j = g >> log2T;
                uint32_t base;
                if constexpr (MODE == 0)
                    base = ((drev<TB, LNS / TB>(j) << LR) * c.ld8) + uint32_t(t) * 8u;
                else
                    base = uint32_t(j) * c.ld8 + uint32_t(t) * 8u;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const uint32_t row_off = MODE == 0 ? uint32_t(crev(r, TB, LR / TB)) * c.ld8 : (uint32_t(r) << LNS) * c.ld8;
                    const float2 a0 = v[i * R + r], a1 = v[EG + i * R + r];
                    *reinterpret_cast<float4 *>(c.dst + base + row_off) = make_float4(a0.x, a0.y, a1.x, a1.y);
                }
            }
            return;
        }
#pragma unroll
        for (int h = 0; h < H; ++h) {
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int g = c.tid + i * nt;
                const int t = H == 2 ? (((g & Tm) << 1) + h) : (g & Tm), j = g >> log2T;
                const float2 *u = &v[h * EG + i * R];
                if constexpr (MODE == 0) {
                    // row pi(k) = pi(j)*2^LR + pi(r)
                    const uint32_t base = ((drev<TB, LNS / TB>(j) << LR) * c.ld8) + uint32_t(t) * 8u;
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        *reinterpret_cast<float2 *>(c.dst + base + uint32_t(crev(r, TB, LR / TB)) * c.ld8) = u[r];
                } else if constexpr (MODE == 2) {
                    // transposed output: row (col0 + t) holds all n frequencies in order
                    const uint32_t base = (uint32_t(t) << (LOG2N + 3)) + uint32_t(j) * 8u;
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        *reinterpret_cast<float2 *>(c.dst + base + (uint32_t(r) << (LNS + 3))) = u[r];
                } else if constexpr (MODE == 1) {
                    const uint32_t base = uint32_t(j) * c.ld8 + uint32_t(t) * 8u;
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        *reinterpret_cast<float2 *>(c.dst + base + (uint32_t(r) << LNS) * c.ld8) = u[r];
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const uint32_t k = j + (r << LNS);
                        const uint32_t m = uint32_t(digrev<GEN>(k, c.out_t, c.out_ell));
                        const uint32_t off = (c.orow_out + m * c.k_out) * c.ld8 + uint32_t(t) * 8u;
                        *reinterpret_cast<float2 *>(c.dst + off) = u[r];
                    }
                }
            }
        }
    }
}

// Tile order: the hardware deals consecutive workgroup ids to the 8 XCDs in
// turn.  Renumber so that the workgroups one XCD receives back to back own
// neighbouring column tiles, which share 128-byte lines in that XCD's L2.
__device__ __forceinline__ int64_t tile_order(int64_t i, int64_t G)
{
    if (G & 7) return i;
    return (i & 7) * (G >> 3) + (i >> 3);
}

__device__ __forceinline__ void copy_twiddles(float2 *twl, const float2 *stw, int n, int tid, int nt)
{
    for (int e = tid; e < n; e += nt) twl[e] = stw[e];  // first read after a barrier
}

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
    run_stage<LOG2N, 0, EG, -1, -1, 1, GEN, 1>(v, c);
}

// Fast single-pass kernel.  MODE 0: natural input rows, digit-reversed
// output rows (Phase I, A = P_pi Omega).  MODE 1: digit-reversed input rows,
// natural output rows (Phase III, B = Omega P_pi).  MODE 2: natural input
// rows, output written transposed in natural frequency order (Phase I of the
// fused pipeline: Lemma 1's output layout composed with the pack step's row
// reversal is the identity, so the packed slab holds frequency k1 at k1).
// b = 2^TB.  H = 2 splits the T columns into two LDS groups: half the LDS
// per workgroup, so two workgroups share a CU and overlap each other's HBM
// traffic and arithmetic.
// EG = 32 (with H = 2) doubles the tile width: 512 threads hold 64 items
// each (two waves per SIMD, 256 VGPRs of budget).
constexpr int fast_tile_log2T(int l, int h, int eg) { return fast_log2T(l) + (h == 2 && eg == 32 ? 1 : 0); }
constexpr int fast_threads(int l, int h, int eg)
{
    return (1 << (l + fast_tile_log2T(l, h, eg))) / (h * eg);
}

template <int LOG2N, int MODE, int TB, int H, int EG>
__global__ __launch_bounds__(fast_threads(LOG2N, H, EG)) void local_fft_fast_kernel(LocalPass P)
{
    constexpr int LT = fast_tile_log2T(LOG2N, H, EG);  // log2 of all columns of the tile
    constexpr int LTG = LT - (H == 2 ? 1 : 0);         // log2 of the columns of one group
    constexpr int NT = (1 << (LOG2N + LTG)) / EG;
    constexpr int LR0 = stage_log2radix(LOG2N, 0);
    constexpr int R0 = 1 << LR0;
    constexpr int NB0 = EG / R0;
    constexpr int LNR0 = LOG2N - LR0;
    constexpr int TWN = stage_tw_total(LOG2N);
    extern __shared__ float2 smem[];
    const int tid = threadIdx.x;
    float2 *twl = smem;
    float2 *lds = smem + ((TWN + 63) & ~63);

    const int64_t col0 = tile_order(blockIdx.x, gridDim.x) << LT;
    const char *src = reinterpret_cast<const char *>(P.src + col0);
    const uint32_t ld8 = uint32_t(P.ld) * 8u;

    // H = 2: group h of tile column t is column 2t + h, and one 16-byte load
    // fetches both groups' items of a row
    float2 v[H * EG];
#pragma unroll
    for (int q = 0; q < NB0; ++q) {
        const int g = tid + q * NT;
        const int t = (g & ((1 << LTG) - 1)) * H, j = g >> LTG;
        uint32_t base;
        if constexpr (MODE == 0 || MODE == 2)
            base = uint32_t(j) * ld8 + uint32_t(t) * 8u;
        else  // row pi(j + r*2^LNR0) = pi(j)*2^LR0 + pi(r)
            base = (drev<TB, LNR0 / TB>(j) << LR0) * ld8 + uint32_t(t) * 8u;
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const uint32_t row_off =
                (MODE == 0 || MODE == 2) ? (uint32_t(r) << LNR0) * ld8 : uint32_t(crev(r, TB, LR0 / TB)) * ld8;
            if constexpr (H == 2) {
                const float4 a = *reinterpret_cast<const float4 *>(src + base + row_off);
                v[q * R0 + r] = make_float2(a.x, a.y);
                v[EG + q * R0 + r] = make_float2(a.z, a.w);
            } else {
                v[q * R0 + r] = *reinterpret_cast<const float2 *>(src + base + row_off);
            }
        }
    }
    copy_twiddles(twl, P.stw, TWN, tid, NT);  // after the data loads are issued
    Ctx c;
    c.lds = lds;
    c.twl = twl;
    c.tid = tid;
    c.nt = NT;
    c.log2T = LTG;
    c.dst = reinterpret_cast<char *>(MODE == 2 ? P.dst + (col0 << LOG2N) : P.dst + col0);
    c.ld8 = ld8;
    c.orow_out = 0;
    c.k_out = 1;
    c.out_t = 0;
    c.out_ell = 0;
    run_stage<LOG2N, 0, EG, LTG, MODE, TB, false, H>(v, c);
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
