// LocalFFT passes (paper, section 4.1 and appendix A) for gfx950.
//
// One workgroup transforms T contiguous columns of an n-row tile (n <= 4096)
// entirely on chip.  The transform is a radix-16 Stockham sequence (one
// radix-2/4/8 stage when log2 n is not a multiple of 4): every thread holds
// E = min(16, n) items in registers; the first stage reads its operands
// straight from HBM rows, the last stage writes its results straight to HBM
// rows, and only the exchanges between stages go through LDS.
//
// The arithmetic order inside a workgroup is free (paper, Lemma 1 holds for
// any digit-aligned split); what the paper fixes is the layout at the HBM
// boundary, which the pass descriptor states: Phase I writes the item of
// logical frequency k to row pi(k) (output layout P_pi Omega), Phase III
// reads logical input j from row pi(j) (input layout Omega P_pi).  Rows are
// contiguous runs of T items, so a digit-reversed row order costs nothing.
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

template <int LOG2N>
struct StagePlan {
    static constexpr int nfull = LOG2N / 4;
    static constexpr int rem = LOG2N % 4;
    static constexpr int count = nfull + (rem ? 1 : 0);
    static constexpr int log2radix(int s) { return s < nfull ? 4 : rem; }
    static constexpr int log2ns(int s)
    {
        int a = 0;
        for (int i = 0; i < s; ++i) a += log2radix(i);
        return a;
    }
    static constexpr int E = LOG2N < 4 ? (1 << LOG2N) : 16;
};

// LDS index with one pad item per 32 (spreads strided stage writes over banks).
__device__ __forceinline__ int lpad(int e) { return e + (e >> 5); }

struct Ctx {
    float2 *lds;
    const float2 *tw;
    int tid, nt, log2T, log2L;
    float2 *dst;
    int64_t ld, orow_out, k_out;
    const int32_t *perm_out;
};

template <int LOG2N, int S>
__device__ __forceinline__ void run_stage(float2 (&v)[StagePlan<LOG2N>::E], const Ctx &c)
{
    using SP = StagePlan<LOG2N>;
    constexpr int E = SP::E;
    constexpr int LR = SP::log2radix(S);
    constexpr int R = 1 << LR;
    constexpr int LNS = SP::log2ns(S);
    constexpr int NB = E / R;
    constexpr int LNR = LOG2N - LR;
    constexpr bool last = (S + 1 == SP::count);
    const int Tm = (1 << c.log2T) - 1;

    if constexpr (S > 0) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int g = c.tid + i * c.nt;
            const int t = g & Tm, j = g >> c.log2T;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i * R + r] = c.lds[lpad(((j + (r << LNR)) << c.log2T) + t)];
        }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int g = c.tid + i * c.nt;
        const int j = g >> c.log2T;
        if constexpr (LNS > 0) {
            const int k = j & ((1 << LNS) - 1);
            const int sh = c.log2L - (LNS + LR);
#pragma unroll
            for (int r = 1; r < R; ++r) v[i * R + r] = cmul(v[i * R + r], c.tw[(k * r) << sh]);
        }
        dft_regs<LR>(&v[i * R]);
    }
    if constexpr (!last) {
        if constexpr (S > 0) __syncthreads();  // all stage-S operands read before overwriting
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int g = c.tid + i * c.nt;
            const int t = g & Tm, j = g >> c.log2T;
            const int idxD = ((j >> LNS) << (LNS + LR)) + (j & ((1 << LNS) - 1));
#pragma unroll
            for (int r = 0; r < R; ++r) c.lds[lpad(((idxD + (r << LNS)) << c.log2T) + t)] = v[i * R + r];
        }
        __syncthreads();
        run_stage<LOG2N, S + 1>(v, c);
    } else {
        // last stage: j < n/R = 2^LNS, outputs are the natural-order rows k = j + r*2^LNS
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int g = c.tid + i * c.nt;
            const int t = g & Tm, j = g >> c.log2T;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int k = j + (r << LNS);
                const int64_t m = c.perm_out ? (int64_t)c.perm_out[k] : (int64_t)k;
                c.dst[(c.orow_out + m * c.k_out) * c.ld + t] = v[i * R + r];
            }
        }
    }
}

// Workgroup order: the hardware deals consecutive workgroup ids to the 8 XCDs
// in turn; renumber so that the groups one XCD receives back to back own
// neighbouring column tiles and share that XCD's L2 lines.
__device__ __forceinline__ int64_t xcd_order(int64_t i, int64_t G)
{
    if (G & 7) return i;
    return (i & 7) * (G >> 3) + (i >> 3);
}

template <int LOG2N>
__global__ __launch_bounds__(1024) void local_fft_kernel(LocalPass P)
{
    using SP = StagePlan<LOG2N>;
    constexpr int E = SP::E;
    constexpr int LR0 = SP::log2radix(0);
    constexpr int R0 = 1 << LR0;
    constexpr int NB0 = E / R0;
    constexpr int LNR0 = LOG2N - LR0;
    extern __shared__ float2 lds[];

    const int log2T = P.log2T;
    const int Tm = (1 << log2T) - 1;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int64_t ntiles = P.ncols >> log2T;
    const int64_t wg = xcd_order(blockIdx.x, gridDim.x);
    const int64_t o = wg / ntiles;
    const int64_t col0 = (wg - o * ntiles) << log2T;
    const float2 *__restrict__ src = P.src + col0;

    float2 v[E];
    const int64_t orow_in = o * P.o_in;
    int64_t f = 0;
    if (P.pre_tw) f = P.tw_perm ? (int64_t)P.tw_perm[o] : o;
    const int64_t Mm = (int64_t(1) << P.log2M) - 1;
    const int shM = P.log2L - P.log2M;
#pragma unroll
    for (int i = 0; i < NB0; ++i) {
        const int g = tid + i * nt;
        const int t = g & Tm, j = g >> log2T;
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int jj = j + (r << LNR0);
            const int64_t m = P.perm_in ? (int64_t)P.perm_in[jj] : (int64_t)jj;
            v[i * R0 + r] = src[(orow_in + m * P.j_in) * P.ld + t];
        }
    }
    if (P.pre_tw) {
#pragma unroll
        for (int i = 0; i < NB0; ++i) {
            const int g = tid + i * nt;
            const int j = g >> log2T;
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const int64_t jj = j + (r << LNR0);
                v[i * R0 + r] = cmul(v[i * R0 + r], P.tw[((f * jj) & Mm) << shM]);
            }
        }
    }
    Ctx c;
    c.lds = lds;
    c.tw = P.tw;
    c.tid = tid;
    c.nt = nt;
    c.log2T = log2T;
    c.log2L = P.log2L;
    c.dst = P.dst + col0;
    c.ld = P.ld;
    c.orow_out = o * P.o_out;
    c.k_out = P.k_out;
    c.perm_out = P.perm_out;
    run_stage<LOG2N, 0>(v, c);
}

template <int LOG2N>
const void *kernel_ptr()
{
    return reinterpret_cast<const void *>(&local_fft_kernel<LOG2N>);
}

const void *kernel_for(int log2n)
{
    switch (log2n) {
    case 1: return kernel_ptr<1>();
    case 2: return kernel_ptr<2>();
    case 3: return kernel_ptr<3>();
    case 4: return kernel_ptr<4>();
    case 5: return kernel_ptr<5>();
    case 6: return kernel_ptr<6>();
    case 7: return kernel_ptr<7>();
    case 8: return kernel_ptr<8>();
    case 9: return kernel_ptr<9>();
    case 10: return kernel_ptr<10>();
    case 11: return kernel_ptr<11>();
    case 12: return kernel_ptr<12>();
    default: return nullptr;
    }
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

LocalLaunch local_fft_geometry(const LocalPass &p)
{
    const int E = p.log2n < 4 ? (1 << p.log2n) : 16;
    const int64_t items = int64_t(1) << (p.log2n + p.log2T);
    LocalLaunch g;
    g.threads = int(items / E);
    g.lds_bytes = size_t(items + (items >> 5) + 1) * sizeof(float2);
    g.groups = p.n_outer * (p.ncols >> p.log2T);
    return g;
}

hipError_t local_fft_prepare()
{
    for (int l = 1; l <= kMaxOnChipLog2; ++l) {
        hipError_t e = hipFuncSetAttribute(kernel_for(l), hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_local_fft(const LocalPass &p, hipStream_t s)
{
    const void *k = kernel_for(p.log2n);
    if (!k) return hipErrorInvalidValue;
    const LocalLaunch g = local_fft_geometry(p);
    void *args[] = {const_cast<LocalPass *>(&p)};
    return hipLaunchKernel(k, dim3(unsigned(g.groups)), dim3(unsigned(g.threads)), args, g.lds_bytes, s);
}

}  // namespace paco
