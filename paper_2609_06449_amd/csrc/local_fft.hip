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
// Two launch shapes.  Short transforms: one tile per workgroup of up to 1024
// threads with 16 items each.  Long transforms (n >= 2^9): persistent
// workgroups of 512 threads with 32 items each (two waves per SIMD, 256
// VGPRs of budget) that walk a sequence of tiles and load the next tile's
// first-stage operands into registers before computing the current one, so
// the HBM traffic of neighbouring tiles overlaps the arithmetic and LDS
// exchanges of the current one.  Stage twiddles come from small factor
// tables copied to LDS once per workgroup (broadcast or contiguous reads);
// row digit reversals are computed with bit operations.
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

struct Ctx {
    float2 *lds;
    const float2 *twl;
    int tid, nt, log2T;
    char *dst;                 // tile base (column col0 of row 0)
    uint32_t ld8;              // row length in bytes
    uint32_t orow_out, k_out;  // output row = orow_out + pi_out(k) * k_out
    int out_t, out_ell;
};

// Stage S of the Stockham sequence.  v[i*R + r] is operand r of butterfly i;
// butterfly id g = tid + i*nt covers column g mod T and index j = g / T.
template <int LOG2N, int S, bool GEN, int EG>
__device__ __forceinline__ void run_stage(float2 (&v)[EG], const Ctx &c)
{
    constexpr int LR = stage_log2radix(LOG2N, S);
    constexpr int R = 1 << LR;
    constexpr int LNS = stage_log2ns(LOG2N, S);
    constexpr int NB = EG / R;
    constexpr bool last = (S + 1 == stage_count(LOG2N));
    const int Tm = (1 << c.log2T) - 1;

#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int g = c.tid + i * c.nt;
        const int j = g >> c.log2T;
        float2 *u = &v[i * R];
        if constexpr (LNS > 0) {
            constexpr int LOW = stage_lo_width(LOG2N, S);
            constexpr int HIW = stage_hi_width(LOG2N, S);
            constexpr int OFF = stage_tw_offset(LOG2N, S);
            const int k = j & ((1 << LNS) - 1);
            const int kl = k & (LOW - 1), kh = k >> 4;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 w = c.twl[OFF + (r - 1) * LOW + kl];
                if constexpr (HIW > 0) w = cmul(w, c.twl[OFF + (R - 1) * LOW + (r - 1) * HIW + kh]);
                u[r] = cmul(u[r], w);
            }
        }
        dft_regs<LR>(u);
    }
    if constexpr (!last) {
        constexpr int LR2 = stage_log2radix(LOG2N, S + 1);
        constexpr int R2 = 1 << LR2;
        constexpr int NB2 = EG / R2;
        constexpr int LNR2 = LOG2N - LR2;
        if constexpr (S > 0) __syncthreads();  // all stage-S operands were read
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int g = c.tid + i * c.nt;
            const int t = g & Tm, j = g >> c.log2T;
            const int idxD = ((j >> LNS) << (LNS + LR)) + (j & ((1 << LNS) - 1));
#pragma unroll
            for (int r = 0; r < R; ++r) c.lds[lpad(((idxD + (r << LNS)) << c.log2T) + t)] = v[i * R + r];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NB2; ++i) {
            const int g = c.tid + i * c.nt;
            const int t = g & Tm, j = g >> c.log2T;
#pragma unroll
            for (int r = 0; r < R2; ++r) v[i * R2 + r] = c.lds[lpad(((j + (r << LNR2)) << c.log2T) + t)];
        }
        run_stage<LOG2N, S + 1, GEN, EG>(v, c);
    } else {
        // last stage: j < n/R = 2^LNS, outputs are the natural-order rows k = j + r*2^LNS
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int g = c.tid + i * c.nt;
            const int t = g & Tm, j = g >> c.log2T;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t k = j + (r << LNS);
                const uint32_t m = uint32_t(digrev<GEN>(k, c.out_t, c.out_ell));
                const uint32_t off = (c.orow_out + m * c.k_out) * c.ld8 + uint32_t(t) * 8u;
                *reinterpret_cast<float2 *>(c.dst + off) = v[i * R + r];
            }
        }
    }
}

// Tile order: the hardware deals consecutive workgroup ids to the 8 XCDs in
// turn, and a workgroup stays on its XCD.  Renumber so that the tiles one
// XCD works on at the same time are neighbouring column tiles, which share
// 128-byte lines in that XCD's L2.  i runs over rounds of `grid` tiles.
__device__ __forceinline__ int64_t tile_order(int64_t i, int64_t G, int64_t grid)
{
    const int64_t s = i / grid, b = i - s * grid;
    if ((grid & 7) || (s + 1) * grid > G) return i;
    return s * grid + (b & 7) * (grid >> 3) + (b >> 3);
}

// First-stage operands of one tile: rows o*o_in + pi_in(jj)*j_in, jj = j +
// r*2^LNR0, column col0 + t.  Byte offsets are 32-bit (buffers < 4 GiB).
template <int LOG2N, bool GEN, int EG>
__device__ __forceinline__ void load_tile(const LocalPass &P, const char *src, uint32_t orow, int tid, int nt,
                                          int log2T, float2 (&v)[EG])
{
    constexpr int LR0 = stage_log2radix(LOG2N, 0);
    constexpr int R0 = 1 << LR0;
    constexpr int NB0 = EG / R0;
    constexpr int LNR0 = LOG2N - LR0;
    const int Tm = (1 << log2T) - 1;
    const uint32_t ld8 = uint32_t(P.ld) * 8u, j_in = uint32_t(P.j_in);
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
}

template <int LOG2N, bool GEN, int EG>
__device__ __forceinline__ void pre_twiddle(const LocalPass &P, int64_t o, int tid, int nt, int log2T,
                                            float2 (&v)[EG])
{
    constexpr int LR0 = stage_log2radix(LOG2N, 0);
    constexpr int R0 = 1 << LR0;
    constexpr int NB0 = EG / R0;
    constexpr int LNR0 = LOG2N - LR0;
    const int64_t f = digrev<GEN>(o, P.tw_t, P.tw_ell);
    const int64_t Mm = (int64_t(1) << P.log2M) - 1;
    const int shM = P.log2L - P.log2M;
#pragma unroll
    for (int q = 0; q < NB0; ++q) {
        const int j = (tid + q * nt) >> log2T;
#pragma unroll
        for (int r = 0; r < R0; ++r) v[q * R0 + r] = cmul(v[q * R0 + r], P.tw[((f * (j + (r << LNR0))) & Mm) << shM]);
    }
}

// One tile per workgroup.
template <int LOG2N, bool PRE, bool GEN, int EG>
__global__ __launch_bounds__(1024) void local_fft_kernel(LocalPass P)
{
    constexpr int TWN = stage_tw_total(LOG2N);
    extern __shared__ float2 smem[];
    const int log2T = P.log2T;
    const int tid = threadIdx.x, nt = blockDim.x;
    float2 *twl = smem;
    float2 *lds = smem + ((TWN + 63) & ~63);
    for (int e = tid; e < TWN; e += nt) twl[e] = P.stw[e];  // first read after a barrier

    const int64_t ntc = P.ncols >> log2T;
    const int64_t tile = tile_order(blockIdx.x, gridDim.x, gridDim.x);
    const int64_t o = tile / ntc;
    const int64_t col0 = (tile - o * ntc) << log2T;

    float2 v[EG];
    load_tile<LOG2N, GEN, EG>(P, reinterpret_cast<const char *>(P.src + col0), uint32_t(o * P.o_in), tid, nt,
                              log2T, v);
    if constexpr (PRE) pre_twiddle<LOG2N, GEN, EG>(P, o, tid, nt, log2T, v);
    Ctx c;
    c.lds = lds;
    c.twl = twl;
    c.tid = tid;
    c.nt = nt;
    c.log2T = log2T;
    c.dst = reinterpret_cast<char *>(P.dst + col0);
    c.ld8 = uint32_t(P.ld) * 8u;
    c.orow_out = uint32_t(o * P.o_out);
    c.k_out = uint32_t(P.k_out);
    c.out_t = P.out_t;
    c.out_ell = P.out_ell;
    run_stage<LOG2N, 0, GEN, EG>(v, c);
}

// Persistent workgroups with a one-tile register prefetch (no pre-twiddle).
template <int LOG2N, bool GEN>
__global__ __launch_bounds__(512) void local_fft_persistent_kernel(LocalPass P)
{
    constexpr int EG = 32;
    constexpr int TWN = stage_tw_total(LOG2N);
    extern __shared__ float2 smem[];
    const int log2T = P.log2T;
    const int nt = blockDim.x;
    float2 *twl = smem;
    float2 *lds = smem + ((TWN + 63) & ~63);
    for (int e = threadIdx.x; e < TWN; e += nt) twl[e] = P.stw[e];

    const int64_t ntc = P.ncols >> log2T;
    const int64_t G = P.n_outer * ntc;
    const int64_t grid = gridDim.x;
    int64_t i = blockIdx.x;
    if (i >= G) return;

    float2 cur[EG], nxt[EG];
    {
        const int64_t tile = tile_order(i, G, grid);
        const int64_t o = tile / ntc, col0 = (tile - o * ntc) << log2T;
        load_tile<LOG2N, GEN, EG>(P, reinterpret_cast<const char *>(P.src + col0), uint32_t(o * P.o_in),
                                  threadIdx.x, nt, log2T, cur);
    }
    for (; i < G; i += grid) {
        // An opaque copy of the thread index per tile keeps thread-invariant
        // addresses and twiddles from being hoisted out of the loop and held
        // in registers across it.
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int64_t tile = tile_order(i, G, grid);
        const int64_t o = tile / ntc, col0 = (tile - o * ntc) << log2T;
        if (i + grid < G) {
            const int64_t tn = tile_order(i + grid, G, grid);
            const int64_t on = tn / ntc, cn = (tn - on * ntc) << log2T;
            load_tile<LOG2N, GEN, EG>(P, reinterpret_cast<const char *>(P.src + cn), uint32_t(on * P.o_in), tid, nt,
                                      log2T, nxt);
        }
        if (i != blockIdx.x) __syncthreads();  // the previous tile's last LDS reads are done
        Ctx c;
        c.lds = lds;
        c.twl = twl;
        c.tid = tid;
        c.nt = nt;
        c.log2T = log2T;
        c.dst = reinterpret_cast<char *>(P.dst + col0);
        c.ld8 = uint32_t(P.ld) * 8u;
        c.orow_out = uint32_t(o * P.o_out);
        c.k_out = uint32_t(P.k_out);
        c.out_t = P.out_t;
        c.out_ell = P.out_ell;
        run_stage<LOG2N, 0, GEN, EG>(cur, c);
#pragma unroll
        for (int e = 0; e < EG; ++e) cur[e] = nxt[e];
    }
}

template <int L, bool PRE, bool GEN>
const void *kptr()
{
    return reinterpret_cast<const void *>(&local_fft_kernel<L, PRE, GEN, (L < 4 ? (1 << L) : 16)>);
}

template <int L, bool GEN>
const void *pptr()
{
    return reinterpret_cast<const void *>(&local_fft_persistent_kernel<L, GEN>);
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

template <bool GEN>
const void *persistent_for(int log2n)
{
    switch (log2n) {
    case 9: return pptr<9, GEN>();
    case 10: return pptr<10, GEN>();
    case 11: return pptr<11, GEN>();
    case 12: return pptr<12, GEN>();
    default: return nullptr;
    }
}

const void *kernel_for(int log2n, bool pre, bool gen, bool persist)
{
    if (persist) return pre ? nullptr : (gen ? persistent_for<true>(log2n) : persistent_for<false>(log2n));
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

bool local_fft_has_persistent(int32_t log2n) { return kernel_for(log2n, false, false, true) != nullptr; }

LocalLaunch local_fft_geometry(const LocalPass &p)
{
    const int EG = p.persist ? 32 : (p.log2n < 4 ? (1 << p.log2n) : 16);
    const int64_t items = int64_t(1) << (p.log2n + p.log2T);
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
        for (int v = 0; v < 8; ++v) {
            const void *k = kernel_for(l, v & 1, v & 2, v & 4);
            if (!k) continue;
            hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

int local_fft_occupancy(const LocalPass &p)
{
    const void *k = kernel_for(p.log2n, p.pre_tw != 0, pass_needs_gen(p), p.persist != 0);
    if (!k) return 0;
    const LocalLaunch g = local_fft_geometry(p);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, g.threads, g.lds_bytes) != hipSuccess) return 0;
    return nb;
}

hipError_t launch_local_fft(const LocalPass &p, hipStream_t s)
{
    const void *k = kernel_for(p.log2n, p.pre_tw != 0, pass_needs_gen(p), p.persist != 0);
    if (!k) return hipErrorInvalidValue;
    const LocalLaunch g = local_fft_geometry(p);
    if (g.tiles < 1 || g.tiles > 0x7fffffff) return hipErrorInvalidValue;
    int64_t grid = g.tiles;
    if (p.persist && p.grid > 0 && p.grid < grid) grid = p.grid;
    void *args[] = {const_cast<LocalPass *>(&p)};
    return hipLaunchKernel(k, dim3(unsigned(grid)), dim3(unsigned(g.threads)), args, g.lds_bytes, s);
}

}  // namespace paco
