// Device code shared by the LocalFFT kernels (local_fft.hip) and the batched
// persistent kernel (batch.hip): radix-16 Stockham stages with LDS
// exchanges, the HBM-boundary row maps of Lemma 1, and one column tile of a
// single-pass local transform.  Included once per translation unit.
#pragma once

#include <type_traits>

#include "paco_internal.h"

namespace paco {
namespace {


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

// A streaming (non-temporal) 8-byte store, for a buffer whose one reader
// streams it back in long contiguous runs (the packed Phase-I buffer and the
// split form's buffer, read by the redistribution pass): HBM serves such
// reads at copy speed, and keeping these lines out of the 256 MiB MALL
// leaves room there for the input of the next transform and for Phase III's
// input.
__device__ __forceinline__ void st2_stream(void *p, float2 v)
{
    typedef float sf2 __attribute__((ext_vector_type(2)));
    sf2 t;
    t.x = v.x;
    t.y = v.y;
    __builtin_nontemporal_store(t, reinterpret_cast<sf2 *>(p));
}

// HBM stores of a tile's results.  COH: a device-coherent store (written
// through this XCD's L2), for results another workgroup of the same launch
// reads after a completion counter says they are there; the 16-byte form
// becomes two such 8-byte stores.
// Loads of data the transform never reads again (Phase II's source buffer):
// non-temporal, so they do not push out of the caches the lines just written
// for the next phase (on a 2^24 transform, whose three 128 MB buffers
// overflow the 256 MB MALL, this keeps Phase III's input resident: measured
// 13% faster end to end; the same hint on other phases' loads or on stores
// measured slower).
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float2 ld2_last(const float2 *p)
{
    const nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2 *>(p));
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ float4 ld4_last(const float2 *p)
{
    const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}

template <bool COH>
__device__ __forceinline__ void st2(char *p, float2 v)
{
    if constexpr (COH) {
        uint64_t bits;
        __builtin_memcpy(&bits, &v, 8);
        __hip_atomic_store(reinterpret_cast<uint64_t *>(p), bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        *reinterpret_cast<float2 *>(p) = v;
    }
}
template <bool COH>
__device__ __forceinline__ void st4(char *p, float4 v)
{
    if constexpr (COH) {
        st2<true>(p, make_float2(v.x, v.y));
        st2<true>(p + 8, make_float2(v.z, v.w));
    } else {
        *reinterpret_cast<float4 *>(p) = v;
    }
}

// LDS index with 4 pad items per 64: the radix-16 first-stage writes (row
// stride 16*T items) land on distinct banks.
__device__ __forceinline__ int lpad(int e) { return e + ((e >> 6) << 2); }

struct Ctx {
    float2 *lds;
    const float2 *twl;
    int tid, nt, log2T;
    char *dst;                 // tile base (column col0 of row 0)
    uint32_t ld8;              // row length in bytes
    uint32_t orow_out, k_out;  // generic: output row = orow_out + pi_out(k) * k_out
    int out_t, out_ell;
    int out_s = 0;             // generic: short top digit of pi_out (mixed radix)
    bool act;                  // runtime tile width: this thread owns butterflies (tid < nt)
    float oscale = 0.f;        // nonzero: every output is stored as conj(y) * oscale
    bool stream = false;       // MODE 2: streaming stores (st2_stream)
};

// conj(v) * s: the inverse transform's output map (s = 1/N, a power of two)
__device__ __forceinline__ float2 conj_scale(float2 v, float s) { return make_float2(v.x * s, -v.y * s); }

// base + idx items through a 32-bit byte offset (buffers below 4 GiB: every
// plan's are, N <= 2^28 complex64): the access then takes a uniform 64-bit
// base and one VGPR of offset instead of a 64-bit address per item.
template <typename T>
__device__ __forceinline__ T *off32(T *base, uint32_t idx)
{
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return reinterpret_cast<T *>(reinterpret_cast<B *>(base) + idx * uint32_t(sizeof(T)));
}

// x, with a value the compiler cannot see through: a lane index taken through
// this inside a loop keeps the index arithmetic that depends on it inside the
// loop (hoisted out of a tile loop, 30 loop-invariant twiddle offsets held in
// registers across it made the kernel spill).  Emits no instruction.
__device__ __forceinline__ uint32_t opaque(uint32_t x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Host side of the persistent passes: the launch over `tiles` tiles (the
// plan's resident workgroup count `groups`, all tiles where it is 0, never
// more than the tiles), and the workgroups of kernel k (threads each) that
// the current device holds at once (0 if the runtime does not say).
inline dim3 persistent(dim3 tiles, uint32_t groups) { return dim3(groups && groups < tiles.x ? groups : tiles.x); }
template <typename K>
uint32_t resident(K k, int threads)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, threads, 0) != hipSuccess)
        return 0;
    return uint32_t(cus > 0 ? cus : 0) * uint32_t(per > 0 ? per : 0);
}

// ---- split-precision MFMA form of the radix-16 butterflies -----------------
// A radix-16 butterfly y = W x, W[m][k] = w_16^{-mk}, is one real contraction
//     [yr; yi] = [[Wr, -Wi], [Wi, Wr]] [xr; xi]          (K = 32),
// so the butterflies of 16 columns are one v_mfma_f32_16x16x32 per output
// half (rows yr, rows yi).  MFMA takes 16-bit operands: each FP32 value is
// split into 16-bit parts and the partial products are summed in FP32:
//   FP16x3: x = s * (hi + 2^-11 lo), s a power of two per butterfly (the
//           butterfly's largest |component| scaled into [1/2, 1)); products
//           hi*hi + 2^-11 (hi*lo + lo*hi)                   (~22 bits)
//   BF16x3: x = hi + lo; products hi*hi + hi*lo + lo*hi     (~16 bits)
//   BF16x6: x = hi + mid + lo; the six products down to 2^-16 (~24 bits).
// Operand layouts of v_mfma_f32_16x16x32_{f16,bf16} (lane l, i < 8):
// A[l & 15][8 (l >> 4) + i], B[8 (l >> 4) + i][l & 15]; result D[4 (l >> 4)
// + i][l & 15], i < 4.  Twiddles stay FP32 (FP64-generated tables).
enum : int { kPrecFP32 = 0, kPrecFP16x3 = 1, kPrecBF16x3 = 2, kPrecBF16x6 = 3 };

typedef __bf16 mf_bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 mf_f16x8 __attribute__((ext_vector_type(8)));
typedef float mf_f32x4 __attribute__((ext_vector_type(4)));

// cos(2 pi r / 16) for any integer r: FP64 values rounded once to FP32.
__host__ __device__ __forceinline__ float cos16(int r)
{
    const int a = r & 7;
    const float v = a == 0   ? 1.0f
                    : a == 1 ? 0.923879532511286756f
                    : a == 2 ? 0.707106781186547524f
                    : a == 3 ? 0.382683432365089772f
                    : a == 4 ? 0.0f
                    : a == 5 ? -0.382683432365089772f
                    : a == 6 ? -0.707106781186547524f
                             : -0.923879532511286756f;
    return (r & 8) ? -v : v;
}

// 16-bit parts of 8 values (see above); lo parts of FP16 carry 2^11.
template <int PREC>
struct MfSplit {
    using T = mf_bf16x8;
    T h, m, l;
};
template <>
struct MfSplit<kPrecFP16x3> {
    using T = mf_f16x8;
    T h, m, l;
};

typedef __bf16 mf_bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 mf_f16x2 __attribute__((ext_vector_type(2)));
typedef float mf_f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t mf_u32x4 __attribute__((ext_vector_type(4)));

// Two FP32 values rounded (to nearest even) into one packed BF16 pair; the
// rounded values back in FP32 are the pair's halves moved into the upper 16
// bits, so one conversion, one shift and one mask per pair.
__device__ __forceinline__ uint32_t bf16_pair(float a, float b, float &ra, float &rb)
{
    const mf_f32x2 v = {a, b};
    const uint32_t p = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, mf_bf16x2));
    ra = __uint_as_float(p << 16);
    rb = __uint_as_float(p & 0xffff0000u);
    return p;
}
__device__ __forceinline__ uint32_t bf16_pair(float a, float b)
{
    const mf_f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, mf_bf16x2));
}

// 16-bit parts of 8 values (see above).  FP16x3 takes x 2^-e (e: the
// butterfly's power-of-two scale, applied here): hi = f16(x 2^-e) and
// lo = f16(x 2^(11-e) - 2^11 hi), the subtraction one mixed-precision FMA on
// the packed hi part.  BF16: hi = bf16(x), the remainders split again.
template <int PREC>
__device__ __forceinline__ MfSplit<PREC> mf_split(const float (&x)[8], int e = 0)
{
    MfSplit<PREC> s;
    if constexpr (PREC == kPrecFP16x3) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const mf_f32x2 y = {ldexpf(x[2 * i], -e), ldexpf(x[2 * i + 1], -e)};
            const float z0 = ldexpf(x[2 * i], 11 - e), z1 = ldexpf(x[2 * i + 1], 11 - e);
            const mf_f16x2 h = __builtin_convertvector(y, mf_f16x2);
            const mf_f32x2 r = {__builtin_fmaf(float(h[0]), -2048.0f, z0), __builtin_fmaf(float(h[1]), -2048.0f, z1)};
            const mf_f16x2 l = __builtin_convertvector(r, mf_f16x2);
            s.h[2 * i] = h[0];
            s.h[2 * i + 1] = h[1];
            s.l[2 * i] = l[0];
            s.l[2 * i + 1] = l[1];
        }
    } else {
        mf_u32x4 hw, mw, lw;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float h0, h1;
            hw[i] = bf16_pair(x[2 * i], x[2 * i + 1], h0, h1);
            float r0 = x[2 * i] - h0, r1 = x[2 * i + 1] - h1;
            if constexpr (PREC == kPrecBF16x6) {
                float m0, m1;
                mw[i] = bf16_pair(r0, r1, m0, m1);
                r0 -= m0;
                r1 -= m1;
            }
            lw[i] = bf16_pair(r0, r1);
        }
        s.h = __builtin_bit_cast(mf_bf16x8, hw);
        if constexpr (PREC == kPrecBF16x6) s.m = __builtin_bit_cast(mf_bf16x8, mw);
        s.l = __builtin_bit_cast(mf_bf16x8, lw);
    }
    return s;
}

// Cross-lane exchanges of the operand layout, on the vector ALU
// (v_permlane32_swap / v_permlane16_swap: the upper 32 (16) lanes of the first
// operand trade places with the lower 32 (16) lanes of the second).
__device__ __forceinline__ void swap32(float &a, float &b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}
// max over lanes l, l ^ 16, l ^ 32, l ^ 48
__device__ __forceinline__ float max_over_kb(float v)
{
    const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = fmaxf(__uint_as_float(a[0]), __uint_as_float(a[1]));
    const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return fmaxf(__uint_as_float(b[0]), __uint_as_float(b[1]));
}

// Stage-0 operands of one group from four whole items per lane: lanes
// l < 32 loaded items q = 0..3 of their 8, lanes l + 32 items 4..7 (it[k]:
// item (l < 32 ? k : 4 + k)); afterwards x[k], x[4 + k] are the real parts
// (l < 32) or the imaginary parts (l >= 32) of items k and 4 + k.
__device__ __forceinline__ void mf_swap_in(const float2 (&it)[4], float (&x)[8])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        float a = it[k].x, b = it[k].y;
        swap32(a, b);
        x[k] = a;
        x[4 + k] = b;
    }
}

// FP16x3: the exponent e with amax 2^-e in [1/2, 1) for the butterfly's 32
// reals (lanes n, n + 16, n + 32, n + 48); 0 for an all-zero butterfly.
// e >= -100 keeps 2^-e and 2^(11-e) finite for butterflies of subnormal
// values (they then stay below 1/2, which loses nothing).
__device__ __forceinline__ int mf_scale_exp(const float (&x)[8])
{
    float amax = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) amax = fmaxf(amax, fabsf(x[i]));
    amax = max_over_kb(amax);
    int e = 0;
    if (amax > 0.f) (void)frexpf(amax, &e);
    return e < -100 ? -100 : e;
}

__device__ __forceinline__ mf_f32x4 mf_mma(mf_bf16x8 a, mf_bf16x8 b, mf_f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ mf_f32x4 mf_mma(mf_f16x8 a, mf_f16x8 b, mf_f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// A * B from the split products.  The products that involve a low part are
// about 2^-8 (BF16) or 2^-11 (FP16) of the result: they are chained through
// one MFMA accumulator, where the hardware's summation rounding is negligible
// at their size.  hi*hi goes into its own accumulator and the two are added
// in FP32 on the vector ALU: chaining hi*hi as well rounded in a way that did
// not average out and piled up at the lowest output frequencies (measured at
// N = 2^24: about 4x larger errors near k = 0 for BF16x6).
template <int PREC>
__device__ __forceinline__ mf_f32x4 mf_product(const MfSplit<PREC> &a, const MfSplit<PREC> &b)
{
    const mf_f32x4 z = {0.f, 0.f, 0.f, 0.f};
    mf_f32x4 small = mf_mma(a.l, b.h, z);
    small = mf_mma(a.h, b.l, small);
    if constexpr (PREC == kPrecBF16x6) {
        small = mf_mma(a.m, b.m, small);
        small = mf_mma(a.m, b.h, small);
        small = mf_mma(a.h, b.m, small);
    }
    const mf_f32x4 main = mf_mma(a.h, b.h, z);
    mf_f32x4 d;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        d[i] = PREC == kPrecFP16x3 ? __builtin_fmaf(small[i], 1.0f / 2048.0f, main[i]) : main[i] + small[i];
    return d;
}

// The 64 butterflies held by one wave (lane l: the 16 inputs u[0..15] of its
// own butterfly, natural order) become their DFTs, in place.  scr is the
// wave's private 1024-item LDS scratch: row b (butterfly of lane b) holds
// item r at b*16 + (r ^ (b & 15)), which spreads the lanes of every access
// over the banks.
template <int PREC>
__device__ __forceinline__ void mfma_dft16(float2 *u, float2 *scr, int lane)
{
    const int n = lane & 15, kb = lane >> 4;
    // A operands: row m = n of [Wr, -Wi] (yr) and [Wi, Wr] (yi), columns k = 8 kb + i
    float ar[8], ai[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int k = 8 * kb + i;
        if (kb < 2) {
            ar[i] = cos16(n * k);           //  Wr =  cos
            ai[i] = -cos16(n * k + 12);     //  Wi = -sin
        } else {
            ar[i] = cos16(n * (k - 16) + 12);  // -Wi =  sin
            ai[i] = cos16(n * (k - 16));       //  Wr
        }
    }
    const MfSplit<PREC> Ar = mf_split<PREC>(ar), Ai = mf_split<PREC>(ai);
    int e = 0;
    if constexpr (PREC == kPrecFP16x3) {
        float amax = 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r) amax = fmaxf(amax, fmaxf(fabsf(u[r].x), fabsf(u[r].y)));
        if (amax > 0.f) (void)frexpf(amax, &e);  // amax * 2^-e in [1/2, 1)
#pragma unroll
        for (int r = 0; r < 16; ++r) u[r] = make_float2(ldexpf(u[r].x, -e), ldexpf(u[r].y, -e));
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) scr[lane * 16 + (r ^ n)] = u[r];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        const int b = 16 * G + n;
        float x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float2 q = scr[b * 16 + ((8 * (kb & 1) + i) ^ n)];
            x[i] = kb < 2 ? q.x : q.y;
        }
        const MfSplit<PREC> B = mf_split<PREC>(x);
        const mf_f32x4 yr = mf_product<PREC>(Ar, B), yi = mf_product<PREC>(Ai, B);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < 4; ++i) scr[b * 16 + ((4 * kb + i) ^ n)] = make_float2(yr[i], yi[i]);
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int m = 0; m < 16; ++m) u[m] = scr[lane * 16 + (m ^ n)];
    if constexpr (PREC == kPrecFP16x3) {
#pragma unroll
        for (int m = 0; m < 16; ++m) u[m] = make_float2(ldexpf(u[m].x, e), ldexpf(u[m].y, e));
    }
}

// Stage S of the Stockham sequence on H column groups.  v[h*EG + i*R + r]
// is operand r of butterfly i of group h; butterfly id g = tid + i*nt of a
// group covers column g mod TG and index j = g / TG (TG columns per group);
// between stages the groups take turns in LDS, which holds n x TG items.
// LT >= 0: compile-time log2 TG.  MODE: -1 generic output rows, 0 digit-
// reversed output rows (Phase I), 1 natural output rows (Phase III), 2 the
// transposed natural output (row = column, n items per row; Phase I of the
// fused pipeline).
template <int LOG2N, int S, int EG, int LT, int MODE, int TB, bool GEN, int H, bool COH = false, int PREC = kPrecFP32>
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
    // with a compile-time tile width every thread of the workgroup owns
    // butterflies; with a runtime one the threads from nt on only take part
    // in the barriers
    const bool act = LT >= 0 || c.act;
    // radix-16 stages of the split-precision forms run on MFMA
    constexpr bool MF = PREC != kPrecFP32 && LR == 4;

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
        if constexpr (!MF) {
#pragma unroll
            for (int h = 0; h < H; ++h) dft_regs<LR>(&v[h * EG + i * R]);
        }
    }
    if constexpr (MF) {
        // the exchange buffer serves as the waves' scratch (1024 items each;
        // the tile has at least 16 items per thread): first every wave has
        // read its inputs out of it
        if constexpr (S > 0) __syncthreads();
        float2 *scr = c.lds + ((c.tid >> 6) << 10);
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int h = 0; h < H; ++h) mfma_dft16<PREC>(&v[h * EG + i * R], scr, c.tid & 63);
    }
    if constexpr (!last) {
        constexpr int LR2 = stage_log2radix(LOG2N, S + 1);
        constexpr int R2 = 1 << LR2;
        constexpr int NB2 = EG / R2;
        constexpr int LNR2 = LOG2N - LR2;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            if (S > 0 || h > 0 || MF) __syncthreads();  // the previous LDS contents were consumed
            if (act) {
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    const int g = c.tid + i * nt;
                    const int t = g & Tm, j = g >> log2T;
                    const int idxD = ((j >> LNS) << (LNS + LR)) + (j & ((1 << LNS) - 1));
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        c.lds[lpad(((idxD + (r << LNS)) << log2T) + t)] = v[h * EG + i * R + r];
                }
            }
            __syncthreads();
            if (act) {
#pragma unroll
                for (int i = 0; i < NB2; ++i) {
                    const int g = c.tid + i * nt;
                    const int t = g & Tm, j = g >> log2T;
#pragma unroll
                    for (int r = 0; r < R2; ++r)
                        v[h * EG + i * R2 + r] = c.lds[lpad(((j + (r << LNR2)) << log2T) + t)];
                }
            }
        }
        run_stage<LOG2N, S + 1, EG, LT, MODE, TB, GEN, H, COH, PREC>(v, c);
    } else {
        // last stage: j < n/R = 2^LNS, outputs are the natural-order rows k = j + r*2^LNS.
        if (!act) return;
        if (c.oscale != 0.f) {
#pragma unroll
            for (int k = 0; k < H * EG; ++k) v[k] = conj_scale(v[k], c.oscale);
        }
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
                    st4<COH>(c.dst + base + row_off, make_float4(a0.x, a0.y, a1.x, a1.y));
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
                        st2<COH>(c.dst + base + uint32_t(crev(r, TB, LR / TB)) * c.ld8, u[r]);
                } else if constexpr (MODE == 2) {
                    // transposed output: row (col0 + t) holds all n frequencies in order
                    const uint32_t base = (uint32_t(t) << (LOG2N + 3)) + uint32_t(j) * 8u;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        if (c.stream)
                            st2_stream(c.dst + base + (uint32_t(r) << (LNS + 3)), u[r]);
                        else
                            st2<COH>(c.dst + base + (uint32_t(r) << (LNS + 3)), u[r]);
                    }
                } else if constexpr (MODE == 1) {
                    const uint32_t base = uint32_t(j) * c.ld8 + uint32_t(t) * 8u;
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        st2<COH>(c.dst + base + (uint32_t(r) << LNS) * c.ld8, u[r]);
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const uint32_t k = j + (r << LNS);
                        const uint32_t m = uint32_t(digmap<GEN>(k, c.out_t, c.out_ell, c.out_s, true));
                        const uint32_t off = (c.orow_out + m * c.k_out) * c.ld8 + uint32_t(t) * 8u;
                        st2<COH>(c.dst + off, u[r]);
                    }
                }
            }
        }
    }
}

__device__ __forceinline__ void copy_twiddles(float2 *twl, const float2 *stw, int n, int tid, int nt)
{
    for (int e = tid; e < n; e += nt) twl[e] = stw[e];  // first read after a barrier
}


constexpr int fast_tile_log2T(int l, int h, int eg) { return fast_log2T(l) + (h == 2 && eg == 32 ? 1 : 0); }
constexpr int fast_threads(int l, int h, int eg)
{
    return (1 << (l + fast_tile_log2T(l, h, eg))) / (h * eg);
}

// The top-level twiddle w_N^{-v j} that a MODE 3 tile applies on load to the
// item of column v and row j = j0 + r n/R0 (r < R0, R0 = the first stage's
// radix), as a product of two FP64-generated FP32 values:
//   a = w_N^{-(v j0 mod N)} = hi[e >> lshift] * lo[e & lomask], e = v j0 mod N,
//   c = w_N^{-v r n/R0} = w_{16 N1}^{-v r 16/R0} = cw[v r 16/R0]  (N = N1 n).
// c depends on the column alone (uniform across a wave when a tile group is
// one column wide), so each item costs one cached load, not two gathers.
struct TopTw {
    const float2 *hi, *lo, *cw;
    uint32_t nmask, lomask, cmask;
    int lshift;
};

// One column tile of a single-pass local transform, the body of the fast
// kernels.  MODE 4: MODE 2 reading its source with last-use (non-temporal)
// loads: Phase I of the two-pass form, whose next pass reads only what this
// one writes (in the three-pass pipeline the same hint measured slower).
// MODE 3: natural input rows scaled by the top-level twiddle on
// load (TopTw), natural output rows: Phase III of the two-pass form, which
// reads the packed Phase-I buffer directly.  MODE 0: natural input rows, digit-reversed
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
// COH: device-coherent result stores (see st2).  PREC: arithmetic of the
// radix-16 butterflies (FP32 VALU, or one of the split MFMA forms).
// LT = log2 of the tile's columns; the caller launches exactly
// 2^(LOG2N + LT - (H == 2)) / EG threads per tile.  srcm/dstm: the matrix
// (row length ld items); col0: the tile's first column.
template <int LOG2N, int MODE, int TB, int H, int EG, int LT, bool COH = false, int PREC = kPrecFP32>
__device__ __forceinline__ void fast_tile(const float2 *srcm, float2 *dstm, uint32_t ld, int64_t col0,
                                          const float2 *stw, float2 *smem, int tid, const TopTw *top = nullptr,
                                          bool conj_in = false, float oscale = 0.f, bool stream_out = false)
{
    constexpr int LTG = LT - (H == 2 ? 1 : 0);         // log2 of the columns of one group
    constexpr int NT = (1 << (LOG2N + LTG)) / EG;
    constexpr int LR0 = stage_log2radix(LOG2N, 0);
    constexpr int R0 = 1 << LR0;
    constexpr int NB0 = EG / R0;
    constexpr int LNR0 = LOG2N - LR0;
    constexpr int TWN = stage_tw_total(LOG2N);
    float2 *twl = smem;
    float2 *lds = smem + ((TWN + 63) & ~63);
    const char *src = reinterpret_cast<const char *>(srcm + col0);
    const uint32_t ld8 = ld * 8u;

    // H = 2: group h of tile column t is column 2t + h, and one 16-byte load
    // fetches both groups' items of a row
    float2 v[H * EG];
#pragma unroll
    for (int q = 0; q < NB0; ++q) {
        const int g = tid + q * NT;
        const int t = (g & ((1 << LTG) - 1)) * H, j = g >> LTG;
        constexpr bool NAT = MODE == 0 || MODE == 2 || MODE == 3 || MODE == 4;  // natural input rows
        uint32_t base;
        if constexpr (NAT)
            base = uint32_t(j) * ld8 + uint32_t(t) * 8u;
        else  // row pi(j + r*2^LNR0) = pi(j)*2^LR0 + pi(r)
            base = (drev<TB, LNR0 / TB>(j) << LR0) * ld8 + uint32_t(t) * 8u;
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const uint32_t row_off = NAT ? (uint32_t(r) << LNR0) * ld8 : uint32_t(crev(r, TB, LR0 / TB)) * ld8;
            const char *pa = src + base + row_off;
            if constexpr (H == 2) {
                const float4 a = MODE == 4 ? ld4_last(reinterpret_cast<const float2 *>(pa))
                                           : *reinterpret_cast<const float4 *>(pa);
                v[q * R0 + r] = make_float2(a.x, a.y);
                v[EG + q * R0 + r] = make_float2(a.z, a.w);
            } else {
                v[q * R0 + r] = MODE == 4 ? ld2_last(reinterpret_cast<const float2 *>(pa))
                                          : *reinterpret_cast<const float2 *>(pa);
            }
        }
        if (conj_in) {  // the inverse transform's input map
#pragma unroll
            for (int k = 0; k < R0; ++k)
#pragma unroll
                for (int h = 0; h < H; ++h) v[h * EG + q * R0 + k].y = -v[h * EG + q * R0 + k].y;
        }
        if constexpr (MODE == 3) {
            // item (row j + r 2^LNR0, column col0 + t + h) times w_N^{-(column * row mod N)}
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const uint32_t col = uint32_t(col0 + t + h);
                const uint32_t e = (col * uint32_t(j)) & top->nmask;
                const float2 a = cmul(top->hi[e >> top->lshift], top->lo[e & top->lomask]);
#pragma unroll
                for (int r = 0; r < R0; ++r) {
                    const float2 c = top->cw[(col * uint32_t(r << (4 - LR0))) & top->cmask];
                    v[h * EG + q * R0 + r] = cmul(v[h * EG + q * R0 + r], cmul(a, c));
                }
            }
        }
    }
    copy_twiddles(twl, stw, TWN, tid, NT);  // after the data loads are issued
    Ctx c;
    c.lds = lds;
    c.twl = twl;
    c.tid = tid;
    c.nt = NT;
    c.log2T = LTG;
    c.dst = reinterpret_cast<char *>(MODE == 2 || MODE == 4 ? dstm + (col0 << LOG2N) : dstm + col0);
    c.ld8 = ld8;
    c.orow_out = 0;
    c.k_out = 1;
    c.out_t = 0;
    c.out_ell = 0;
    c.act = true;
    c.oscale = oscale;
    c.stream = stream_out;
    run_stage<LOG2N, 0, EG, LTG, MODE == 3 ? 1 : (MODE == 4 ? 2 : MODE), TB, false, H, COH, PREC>(v, c);
}

// One column tile of a single-pass transform of n = 16^s points (s <= 3)
// whose butterflies all run on MFMA, in the operand layout throughout: a
// wave owns 64 butterflies as four groups of 16, and lane l (column n = l & 15,
// K slice kb = l >> 4) holds, for each group, only its 8 real MFMA operands
// (components 8 (kb & 1) .. +8 of the real part for kb < 2, of the imaginary
// part otherwise) and afterwards the 4 outputs m = 4 kb .. +4 of its column.
// Stage-0 operands are read straight from HBM rows, later ones from the
// exchange buffer; outputs go straight to their Stockham positions with the
// next stage's twiddle applied (or to HBM rows after the last stage), so a
// stage costs the same LDS traffic as an FP32 stage.  The tile is n x 2^LT
// columns with one 16-item butterfly per thread and stage (EG = 16).
template <int LOG2N, int MODE, int TB, int PREC, int LT = fast_log2T(LOG2N)>
__device__ __forceinline__ void mf_tile(const float2 *srcm, float2 *dstm, uint32_t ld, int64_t col0,
                                        const float2 *stw, float2 *smem, int tid, bool conj_in = false,
                                        float oscale = 0.f)
{
    static_assert(LOG2N % 4 == 0 && LOG2N >= 4 && LOG2N <= 12, "radix-16 stages only");
    constexpr int NS = LOG2N / 4;
    constexpr int Tm = (1 << LT) - 1;
    constexpr int NT = (1 << (LOG2N + LT)) / 16;
    constexpr int LNR = LOG2N - 4;  // input k of a butterfly: row j + k 2^LNR
    constexpr int TWN = stage_tw_total(LOG2N);
    float2 *twl = smem;
    float2 *lds = smem + ((TWN + 63) & ~63);
    const int lane = tid & 63, n = lane & 15, kb = lane >> 4, wbase = (tid >> 6) << 6;
    const int comp = kb >> 1, half = kb & 1;  // real (0) or imaginary (1) part; first or second 8 inputs
    const char *src = reinterpret_cast<const char *>(srcm + col0);
    char *dst = reinterpret_cast<char *>(MODE == 2 ? dstm + (col0 << LOG2N) : dstm + col0);
    const uint32_t ld8 = ld * 8u;

    // A operands: row m = n of [Wr, -Wi] (yr) and [Wi, Wr] (yi), columns 8 kb + i
    float ar[8], ai[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int k = 8 * kb + i;
        if (kb < 2) {
            ar[i] = cos16(n * k);
            ai[i] = -cos16(n * k + 12);
        } else {
            ar[i] = cos16(n * (k - 16) + 12);
            ai[i] = cos16(n * (k - 16));
        }
    }
    const MfSplit<PREC> Ar = mf_split<PREC>(ar), Ai = mf_split<PREC>(ai);

    // stage 0 operands straight from HBM rows.  Lanes l and l ^ 32 hold the
    // real and the imaginary parts of the same 8 items: each loads 4 whole
    // items (8-byte loads) and the pair swaps the other component's halves
    // (measured 13-15% faster end to end than 8 component loads per lane)
    float xin[4][8];
    {
        float2 it[4][4];
#pragma unroll
        for (int G = 0; G < 4; ++G) {
            const int g = wbase + 16 * G + n;
            const int t = g & Tm, j = g >> LT;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int ii = comp ? 4 + k : k;  // this lane's items: the lower or the upper 4
                const uint32_t jj = uint32_t(j + ((8 * half + ii) << LNR));
                const uint32_t row = MODE == 1 ? uint32_t(digrev<false>(jj, TB, LOG2N / TB)) : jj;
                it[G][k] = *reinterpret_cast<const float2 *>(src + row * ld8 + uint32_t(t) * 8u);
            }
        }
#pragma unroll
        for (int G = 0; G < 4; ++G) mf_swap_in(it[G], xin[G]);
    }
    if (conj_in && comp == 1) {  // the inverse transform's input map: negate the imaginary parts
#pragma unroll
        for (int G = 0; G < 4; ++G)
#pragma unroll
            for (int i = 0; i < 8; ++i) xin[G][i] = -xin[G][i];
    }
    copy_twiddles(twl, stw, TWN, tid, NT);  // after the data loads are issued

    float2 o[4][4];  // outputs of this lane: group G, m = 4 kb + i
#pragma unroll
    for (int S = 0; S < NS; ++S) {
        const int LNS = 4 * S;
        // Butterfly g of a stage is (column t, index j); any assignment works
        // as long as one stage uses one.  The last stage of the transposed
        // store (MODE 2) takes j fastest, so each store instruction writes 16
        // consecutive outputs of a column (128-byte runs); elsewhere t is
        // fastest (neighbouring columns of a row are adjacent in HBM and LDS).
        const bool jfast = MODE == 2 && S == NS - 1 && S > 0;
#pragma unroll
        for (int G = 0; G < 4; ++G) {
            if (S > 0) {
                // operands of stage S out of the exchange buffer (already twiddled)
                const int g = wbase + 16 * G + n;
                const int t = jfast ? g >> LNR : g & Tm, j = jfast ? g & ((1 << LNR) - 1) : g >> LT;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int row = j + ((8 * half + i) << LNR);
                    xin[G][i] = reinterpret_cast<const float *>(lds + lpad((row << LT) + t))[comp];
                }
            }
            // FP16x3: per-butterfly power-of-two scale (the column's 32 reals)
            const int e = PREC == kPrecFP16x3 ? mf_scale_exp(xin[G]) : 0;
            const MfSplit<PREC> B = mf_split<PREC>(xin[G], e);
            const mf_f32x4 yr = mf_product<PREC>(Ar, B);
            const mf_f32x4 yi = mf_product<PREC>(Ai, B);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                o[G][i] = make_float2(yr[i], yi[i]);
                if constexpr (PREC == kPrecFP16x3) o[G][i] = make_float2(ldexpf(o[G][i].x, e), ldexpf(o[G][i].y, e));
            }
        }
        if (S + 1 < NS) {
            // outputs to the exchange buffer, scaled by the next stage's twiddle
            const int LNS2 = LNS + 4;
            const int OFF = stage_tw_offset(LOG2N, S + 1);
            const int LOW = stage_lo_width(LOG2N, S + 1), HIW = stage_hi_width(LOG2N, S + 1);
            __syncthreads();  // stage S's operands are read (and the twiddle table is in LDS)
#pragma unroll
            for (int G = 0; G < 4; ++G) {
                const int g = wbase + 16 * G + n;
                const int t = g & Tm, j = g >> LT;
                const int idxD = ((j >> LNS) << (LNS + 4)) + (j & ((1 << LNS) - 1));
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int pos = idxD + ((4 * kb + i) << LNS);
                    const int r2 = pos >> LNR, k2 = (pos & ((1 << LNR) - 1)) & ((1 << LNS2) - 1);
                    float2 w = make_float2(1.f, 0.f);
                    if (r2 > 0) {
                        w = twl[OFF + (r2 - 1) * LOW + (k2 & (LOW - 1))];
                        if (HIW > 0) w = cmul(w, twl[OFF + 15 * LOW + (r2 - 1) * HIW + (k2 >> 4)]);
                    }
                    lds[lpad((pos << LT) + t)] = r2 > 0 ? cmul(o[G][i], w) : o[G][i];
                }
            }
            __syncthreads();
        }
    }
    // last stage: output k = j + m 2^(LOG2N - 4) of every butterfly to its HBM row
    constexpr bool jfast_last = MODE == 2 && NS > 1;
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        const int g = wbase + 16 * G + n;
        const int t = jfast_last ? g >> LNR : g & Tm, j = jfast_last ? g & ((1 << LNR) - 1) : g >> LT;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t k = uint32_t(j + ((4 * kb + i) << (LOG2N - 4)));
            uint32_t off;
            if constexpr (MODE == 2)
                off = (uint32_t(t) << (LOG2N + 3)) + k * 8u;
            else if constexpr (MODE == 0)
                off = uint32_t(digrev<false>(k, TB, LOG2N / TB)) * ld8 + uint32_t(t) * 8u;
            else
                off = k * ld8 + uint32_t(t) * 8u;
            const float2 w = oscale != 0.f ? conj_scale(o[G][i], oscale) : o[G][i];
            if constexpr (MODE == 2)
                st2_stream(dst + off, w);  // the packed buffer, streamed back by Phase II
            else
                st2<false>(dst + off, w);
        }
    }
}

}  // namespace
}  // namespace paco
