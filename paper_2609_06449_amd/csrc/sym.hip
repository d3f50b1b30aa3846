// The symmetric split form (FP32), N1 = 16 L1 and N2 = 16 L2 with L1, L2 in
// {256, 512, 1024}; written out below for N1 = N2 = 4096 (L = 256), the
// other sizes replacing 256 by L1 in Phase I and by L2 in Phase III.
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
    const uint32_t blk = addr::sym1_block(blockIdx.x, N2);
    const uint32_t r = blk / (N2 >> 4);
    const int cl = tid & 15, jl = tid >> 4;
    float2 v[16];
    const float2 *src = P.src + addr::sym1_load_base(N2, blk, tid);
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
    float2 *dst = P.dst + addr::sym1_store_base(N2, blk, tid);
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
// Children L1 = 2^LL1 = N1/16 (Phase I) and L2 = 2^LL2 = N2/16 (Phase III):
// jc < L2, kb < L1/16, c = jc + L2 rr, v = k + L1 s, and the pass-2 factor
// table holds w_{16 N2}^{-s jc} at [s L2 + jc].  The split of the top-level
// factor holds for any L1, L2: N / L1 = 16 N2 and 16 N2 / L2 = 256.
template <int LL1, int LL2>
__global__ __launch_bounds__(kSymThreads) __attribute__((amdgpu_waves_per_eu(5))) void sym_middle_kernel(SymPass P)
{
    __shared__ float2 lds[16 * 256];
    const int tid = threadIdx.x;
    const uint32_t N1 = uint32_t(P.N1), N2 = uint32_t(P.N2);
    const uint32_t blk = addr::sym2_block(blockIdx.x, LL1, LL2);
    const uint32_t kb = blk & ((1u << (LL1 - 4)) - 1u), jc = blk >> (LL1 - 4);
    const int kk = tid & 15, rr = tid >> 4;
    const uint32_t c = jc + (uint32_t(rr) << LL2), k = 16u * kb + kk;
    float2 v[16];
    const float2 *src = P.src + addr::sym2_load_base(N2, blk, tid, LL1, LL2);
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = ld2_last(src + addr::sym2_load_off(r));  // last use
    const uint32_t nmask = uint32_t((uint64_t(1) << P.log2N) - 1), lomask = (1u << P.log2Lo) - 1u;
    const uint32_t e1 = (k * c) & nmask;
    const float2 h1 = P.tw_hi[e1 >> P.log2Lo], l1 = P.tw_lo[e1 & lomask];
    float2 t2[16], t3[16], t4[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        t2[s] = P.tw_sj[(s << LL2) + jc];                            // w_{16 N2}^{-s jc}
        t3[s] = root_of(P.tw, P.log2L, 8, uint32_t(s * rr));        // w_256^{-s rr}
        t4[s] = root_of(P.tw, P.log2L, LL2 + 4, uint32_t(s) * jc);  // w_N2^{-q0 jc}, q0 = s
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
    float2 *dst = P.dst + addr::sym2_store_base(N1, blk, tid, LL1);
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
    const uint32_t blk = addr::sym3_block(blockIdx.x, N1);
    const float2 *src = P.src + addr::sym3_load_base(N1, blk, tid);
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
    float2 *dst = P.dst + addr::sym3_store_base(N1, blk, tid);
#pragma unroll
    for (int kh = 0; kh < 16; ++kh)
        dst[addr::sym3_store_off(N1, kh)] = P.out_scale != 0.f ? conj_scale(v[kh], P.out_scale) : v[kh];
}

// ---- passes 1 and 3 for L = 512 and 1024 (N1 = N2 = 8192, 16384) ----------
// The L-point transform of a 16-column tile: radix 16 over jh (j = jl + M jh,
// M = L/16) by thread (cl, jl), twiddle w_L^{-jl ka}, exchange; then the
// M-point transform over jl = jp + P jm (P = M/16 = 2 or 4) of each (column,
// ka): radix 16 over jm by thread (jp, ...), twiddle w_M^{-jp kb'}, and radix
// P across the P threads of a transform, which sit 16 lanes apart: a
// v_permlane16_swap (and for P = 4 two v_permlane32_swaps) of a value with
// itself leaves every lane with the values of all P threads.  Thread jp keeps
// the outputs kb' + 16 jp, i.e. k = ka + 16 (kb' + 16 jp) of the L-point
// transform.  The exchange buffer holds 16 planes (ka) of M x 16 items.

template <int PP>
__device__ __forceinline__ float2 radix_across_lanes(float2 y, int jp)
{
    // X_jp = sum_p w_P^{-jp p} y_p, y_p the value of lane group p
    const auto sx = __builtin_amdgcn_permlane16_swap(__float_as_uint(y.x), __float_as_uint(y.x), false, false);
    const auto sy = __builtin_amdgcn_permlane16_swap(__float_as_uint(y.y), __float_as_uint(y.y), false, false);
    float2 a = make_float2(__uint_as_float(sx[0]), __uint_as_float(sy[0]));  // y of the even lane group
    float2 b = make_float2(__uint_as_float(sx[1]), __uint_as_float(sy[1]));  // y of the odd lane group
    if constexpr (PP == 2) {
        const float sg = (jp & 1) ? -1.f : 1.f;
        return make_float2(fmaf(sg, b.x, a.x), fmaf(sg, b.y, a.y));
    } else {
        // after the 32-lane swaps: a = y_0, a2 = y_2, b = y_1, b2 = y_3
        const auto ax = __builtin_amdgcn_permlane32_swap(__float_as_uint(a.x), __float_as_uint(a.x), false, false);
        const auto ay = __builtin_amdgcn_permlane32_swap(__float_as_uint(a.y), __float_as_uint(a.y), false, false);
        const auto bx = __builtin_amdgcn_permlane32_swap(__float_as_uint(b.x), __float_as_uint(b.x), false, false);
        const auto by = __builtin_amdgcn_permlane32_swap(__float_as_uint(b.y), __float_as_uint(b.y), false, false);
        const float2 y0 = make_float2(__uint_as_float(ax[0]), __uint_as_float(ay[0]));
        const float2 y2 = make_float2(__uint_as_float(ax[1]), __uint_as_float(ay[1]));
        const float2 y1 = make_float2(__uint_as_float(bx[0]), __uint_as_float(by[0]));
        const float2 y3 = make_float2(__uint_as_float(bx[1]), __uint_as_float(by[1]));
        // X_t = (y0 + (-1)^t y2) + w_4^{-t} (y1 + (-1)^t y3), w_4^{-1} = -i
        const float sg = (jp & 1) ? -1.f : 1.f;
        const float2 e = make_float2(fmaf(sg, y2.x, y0.x), fmaf(sg, y2.y, y0.y));
        const float2 o = make_float2(fmaf(sg, y3.x, y1.x), fmaf(sg, y3.y, y1.y));
        const float2 r = (jp & 1) ? make_float2(o.y, -o.x) : o;
        const float g = (jp & 2) ? -1.f : 1.f;
        return make_float2(fmaf(g, r.x, e.x), fmaf(g, r.y, e.y));
    }
}

// Stage B on the 16 values v[jm] of item jl = jp + P jm: afterwards v[i] is
// output kb' = i of the thread's M-point transform times nothing, combined
// across its P threads (output i + 16 jp).  tb[i] = w_M^{-jp i}.
template <int PP>
__device__ __forceinline__ void stage_b(float2 (&v)[16], const float2 (&tb)[16], int jp)
{
    dft_regs<4>(v);
#pragma unroll
    for (int i = 1; i < 16; ++i) v[i] = cmul(v[i], tb[i]);
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = radix_across_lanes<PP>(v[i], jp);
}

// Passes 1 and 3 at L = 512 and 1024 run persistent workgroups: workgroup g
// of G takes tiles g, g + G, ... (in the block order addr::sym{1,3}_block
// gives a launch of one workgroup per tile), and issues the loads of its
// next tile right after stage A of the current one, so that they are in
// flight during stage B, the stores and the next barrier.  A tile fills the
// LDS of a CU (1024 threads, 128 KiB at L = 1024) or half of it, so without
// this one tile's loads did not overlap another's arithmetic (L = 1024:
// passes 1 and 3 1233 / 1321 us against 1007 / 1094 us pipelined, 893 /
// 929 us for a copy with the same loads and stores).  The twiddle factors
// sit in LDS (loaded once per workgroup): a global load in the loop would
// wait for the prefetch ahead of it.  G is the number of workgroups the
// device holds at once (plan creation); the last tile reloads itself, which
// keeps the loop one block (its loads are issued before its stores and the
// values are not used).

// Pass 1, L = 2^LL.  Stage-B thread (ka, jp, cl2) = (tid & 15, (tid >> 4) &
// (P-1), tid >> (4 + log2 P)): k fastest, for the 128-byte runs of U.  Plane
// stride L + 1 (odd): a half-wave of stage-B loads (16 ka x 2 jp) hits 32
// distinct 8-byte slots.
template <bool STREAM, int LL>
__global__ __launch_bounds__(1 << LL) __attribute__((amdgpu_waves_per_eu(4))) void sym_first_long_kernel(SymPass P,
                                                                                                        uint32_t tiles)
{
    constexpr int L = 1 << LL, M = L >> 4, PP = M >> 4, S = L + 1;
    __shared__ float2 lds[16 * S];
    __shared__ float2 twL[L];      // w_L^{-m}
    __shared__ float2 twF[256];    // w_N1^{-m}, m < 256 (N1 = 16 L)
    const int tid = threadIdx.x, cl = tid & 15;
    const uint32_t N2 = uint32_t(P.N2);
    uint32_t t = blockIdx.x;
    float2 v[16];
    auto load = [&](uint32_t tile) {
        const uint32_t base = addr::sym1_load_base(N2, addr::sym1_block(tile, N2, LL), tid);
#pragma unroll
        for (int jh = 0; jh < 16; ++jh) v[jh] = *off32(P.src, base + addr::sym1_load_off(N2, jh, LL));
    };
    // stage A of tile tc (radix 16 over jh by thread (cl, jl), twiddle
    // w_L^{-jl ka}) into the exchange buffer, then the next tile's loads
    auto stage_a = [&](uint32_t tc) {
        const uint32_t jl = opaque(uint32_t(tid)) >> 4;
        if (P.conj_in) {
#pragma unroll
            for (int i = 0; i < 16; ++i) v[i].y = -v[i].y;
        }
        dft_regs<4>(v);
#pragma unroll
        for (int k = 1; k < 16; ++k) v[k] = cmul(v[k], twL[(jl * k) & (L - 1)]);
#pragma unroll
        for (int k = 0; k < 16; ++k) lds[k * S + jl * 16 + cl] = v[k];
        load(tc + gridDim.x < tiles ? tc + gridDim.x : tc);
        __syncthreads();
    };
    load(t < tiles ? t : 0);  // (the launch gives every workgroup a tile)
    twL[tid] = P.tw[uint32_t(tid) << (P.log2L - LL)];
    if (tid < 256) twF[tid] = P.tw[uint32_t(tid) << (P.log2L - LL - 4)];
    __syncthreads();
    if (t < tiles) stage_a(t);
    while (t < tiles) {
        const uint32_t blk = addr::sym1_block(t, N2, LL);
        const uint32_t r = blk / (N2 >> 4);
        const uint32_t tt = opaque(uint32_t(tid));
        const uint32_t ka = tt & 15, jp = (tt >> 4) & (PP - 1), cl2 = tt >> (LL - 4);
        float2 u[16], tb[16];
#pragma unroll
        for (int jm = 0; jm < 16; ++jm) u[jm] = lds[ka * S + (jp + PP * jm) * 16 + cl2];
#pragma unroll
        for (int k = 1; k < 16; ++k) tb[k] = twL[((jp * k) << 4) & (L - 1)];  // w_M^{-jp kb'}
        stage_b<PP>(u, tb, int(jp));
        const float2 a = twF[ka * r];  // w_N1^{-ka r}
        const uint32_t dbase = addr::sym1_store_base(N2, blk, tid, LL);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            // w_N1^{-k r}, k = ka + 16 (i + 16 jp): w_N1^{-ka r} w_L^{-(i + 16 jp) r}
            const float2 y = cmul(u[i], cmul(a, twL[((i + 16 * jp) * r) & (L - 1)]));
            float2 *d = off32(P.dst, dbase + addr::sym1_store_off(N2, i));
            if constexpr (STREAM)
                st2_stream(d, y);
            else
                *d = y;
        }
        __syncthreads();
        t += gridDim.x;
        if (t < tiles) stage_a(t);
    }
}

// Pass 3, L = 2^LL, in place (a tile's stores go to the items it loaded,
// and no other workgroup's tile overlaps them).  Stage-B thread (cl, jp,
// ka) = (tid & 15, (tid >> 4) & (P-1), tid >> (4 + log2 P)): column fastest,
// for the 128-byte runs of the rows it stores; a half-wave of stage-B loads
// (16 cl x 2 jp) is 32 consecutive items of one plane, so the planes need no
// padding.  R = 2^LR: the radix of pass 2's Phase III child (rows R t + q0).
template <int LL, int LR>
__global__ __launch_bounds__(1 << LL) __attribute__((amdgpu_waves_per_eu(4))) void sym_last_long_kernel(SymPass P,
                                                                                                       uint32_t tiles)
{
    constexpr int L = 1 << LL, M = L >> 4, PP = M >> 4, S = L;
    __shared__ float2 lds[16 * S];
    __shared__ float2 twL[L];
    const int tid = threadIdx.x, cl = tid & 15;
    const uint32_t N1 = uint32_t(P.N1);
    uint32_t t = blockIdx.x;
    float2 v[16];
    auto load = [&](uint32_t tile) {
        const uint32_t base = addr::sym3r_load_base(N1, addr::sym3r_block(tile, N1, LL, LR), tid, LR);
#pragma unroll
        for (int jh = 0; jh < 16; ++jh) v[jh] = *off32(P.src, base + addr::sym3r_load_off(N1, jh, LL, LR));
    };
    auto stage_a = [&](uint32_t tc) {
        const uint32_t jl = opaque(uint32_t(tid)) >> 4;
        dft_regs<4>(v);
#pragma unroll
        for (int k = 1; k < 16; ++k) v[k] = cmul(v[k], twL[(jl * k) & (L - 1)]);
#pragma unroll
        for (int k = 0; k < 16; ++k) lds[k * S + jl * 16 + cl] = v[k];
        load(tc + gridDim.x < tiles ? tc + gridDim.x : tc);
        __syncthreads();
    };
    load(t < tiles ? t : 0);  // (the launch gives every workgroup a tile)
    twL[tid] = P.tw[uint32_t(tid) << (P.log2L - LL)];
    __syncthreads();
    if (t < tiles) stage_a(t);
    while (t < tiles) {
        const uint32_t blk = addr::sym3r_block(t, N1, LL, LR);
        const uint32_t tt = opaque(uint32_t(tid));
        const uint32_t jp = (tt >> 4) & (PP - 1), ka = tt >> (LL - 4);
        float2 u[16], tb[16];
#pragma unroll
        for (int jm = 0; jm < 16; ++jm) u[jm] = lds[ka * S + (jp + PP * jm) * 16 + cl];
#pragma unroll
        for (int k = 1; k < 16; ++k) tb[k] = twL[((jp * k) << 4) & (L - 1)];
        stage_b<PP>(u, tb, int(jp));
        const uint32_t dbase = addr::sym3r_store_base(N1, blk, tid, LL, LR);
#pragma unroll
        for (int i = 0; i < 16; ++i)
            *off32(P.dst, dbase + addr::sym3r_store_off(N1, i, LR)) =
                P.out_scale != 0.f ? conj_scale(u[i], P.out_scale) : u[i];
        __syncthreads();
        t += gridDim.x;
        if (t < tiles) stage_a(t);
    }
}

// Pass 2 of the wide form (N2 = 32 L2, L2 = 2^LL2): Phase III's child in
// this pass has 32 points, j2 = jc + L2 rr, k2 = q0 + 32 q (rr, q0 < 32).
// Tile (jc, kb) owns k = 16 kb + kk and the columns c = jc + L2 rr: thread
// (kk, rr) of 512 reads U[c][r][k] (r < 16), transforms over r (-> s,
// v = k + L1 s) and applies w_N^{-k c} w_512^{-s rr}; thread (kk, p, s) then
// transforms over rr = p + 2 m: radix 16 over m, twiddle w_32^{-p i}, radix 2
// with the thread 16 lanes away (stage_b), keeping q0 = i + 16 p, and
// applies w_{16 N2}^{-s jc} w_N2^{-q0 jc} (the first factor, the same for
// all rr of the thread's transform, moved past it; together with the
// others it is w_N^{-v c} w_N2^{-q0 jc}, N = 512 L1 L2).  W goes to row
// 32 jc + q0, columns v (four 128-byte runs per instruction).  The exchange
// buffer is [s][rr][kk] (64 KiB: each half-wave writes and reads 32
// consecutive items), so two workgroups fit on a CU; they run persistent
// and pipelined like passes 1 and 3 at L >= 512, issuing the next tile's
// loads after stage A.  The factors that depend on the tile's jc (16 of
// w_{16 N2}, 32 of w_N2) are loaded by threads 0..47 with that tile's data
// and pass through LDS; w_512 sits in LDS for the whole launch.
template <int LL1, int LL2>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void sym_middle_wide_kernel(SymPass P,
                                                                                                     uint32_t tiles)
{
    __shared__ float2 lds[16 * 512];
    __shared__ float2 tw512[512];  // w_512^{-m}
    __shared__ float2 tjc[48];     // the current tile's w_{16 N2}^{-s jc} (s < 16), w_N2^{-q0 jc} (q0 < 32)
    const int tid = threadIdx.x, kk = tid & 15;
    const uint32_t N1 = uint32_t(P.N1), N2 = uint32_t(P.N2);
    const uint32_t nmask = uint32_t((uint64_t(1) << P.log2N) - 1), lomask = (1u << P.log2Lo) - 1u;
    uint32_t t = blockIdx.x;
    float2 v[16], h1, l1, tu;
    auto load = [&](uint32_t tile) {
        const uint32_t blk = addr::sym2_block(tile, LL1, LL2);
        const uint32_t kb = blk & ((1u << (LL1 - 4)) - 1u), jc = blk >> (LL1 - 4);
        const uint32_t c = jc + ((uint32_t(tid) >> 4) << LL2), k = 16u * kb + kk;
        const uint32_t e1 = (k * c) & nmask;
        // threads 48.. repeat the loads of 16..47 (no branch in the loop)
        const uint32_t u = tid < 16 ? uint32_t(tid) : 16u + ((uint32_t(tid) - 16u) & 31u);
        tu = u < 16 ? P.tw_sj[(u << (LL2 + 1)) + jc] : root_of(P.tw, P.log2L, LL2 + 5, (u - 16u) * jc);
        h1 = P.tw_hi[e1 >> P.log2Lo];
        l1 = P.tw_lo[e1 & lomask];
        const uint32_t base = addr::sym2_load_base(N2, blk, tid, LL1, LL2);
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = ld2_last(off32(P.src, base + addr::sym2_load_off(r)));  // last use
    };
    // stage A of tile tc into the exchange buffer, then the next tile's loads
    auto stage_a = [&](uint32_t tc) {
        const uint32_t rr = opaque(uint32_t(tid)) >> 4;
        if (tid < 48) tjc[tid] = tu;
        dft_regs<4>(v);
        const float2 t1 = cmul(h1, l1);  // w_N^{-k c}
#pragma unroll
        for (int s = 0; s < 16; ++s)
            lds[s * 512 + rr * 16 + kk] = cmul(v[s], cmul(t1, tw512[(s * rr) & 511]));  // w_512^{-s rr}
        load(tc + gridDim.x < tiles ? tc + gridDim.x : tc);
        __syncthreads();
    };
    load(t < tiles ? t : 0);  // (the launch gives every workgroup a tile)
    tw512[tid] = P.tw[uint32_t(tid) << (P.log2L - 9)];
    __syncthreads();
    if (t < tiles) stage_a(t);
    while (t < tiles) {
        const uint32_t blk = addr::sym2_block(t, LL1, LL2);
        const uint32_t tt = opaque(uint32_t(tid));
        const uint32_t p = (tt >> 4) & 1u, s2 = tt >> 5;
        float2 u[16], tb[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) u[m] = lds[s2 * 512 + (p + 2 * m) * 16 + kk];
#pragma unroll
        for (int i = 1; i < 16; ++i) tb[i] = tw512[(16 * p * i) & 511];  // w_32^{-p i}
        stage_b<2>(u, tb, int(p));
        const float2 g = tjc[s2];  // w_{16 N2}^{-s jc}
        const uint32_t dbase = addr::sym2w_store_base(N1, blk, tid, LL1);
#pragma unroll
        for (int i = 0; i < 16; ++i)
            *off32(P.dst, dbase + addr::sym2w_store_off(N1, i)) = cmul(u[i], cmul(g, tjc[16 + i + 16 * p]));
        __syncthreads();
        t += gridDim.x;
        if (t < tiles) stage_a(t);
    }
}

bool sym_shape_ok(const SymPass &p, int &ll1, int &ll2, int &lr2)
{
    return sym_children(p, ll1, ll2, lr2) && p.src && p.dst && p.tw && p.tw_hi && p.tw_lo && p.tw_sj;
}

int log2_child(int64_t n) { return n == 4096 ? 8 : n == 8192 ? 9 : n == 16384 ? 10 : 0; }

// pass 2 for L1 = 2^LL1 and L2 = 2^ll2
template <int LL1>
void launch_middle(int ll2, dim3 grid, const SymPass &p, hipStream_t s)
{
    switch (ll2) {
    case 8: hipLaunchKernelGGL((sym_middle_kernel<LL1, 8>), grid, dim3(kSymThreads), 0, s, p); break;
    case 9: hipLaunchKernelGGL((sym_middle_kernel<LL1, 9>), grid, dim3(kSymThreads), 0, s, p); break;
    default: hipLaunchKernelGGL((sym_middle_kernel<LL1, 10>), grid, dim3(kSymThreads), 0, s, p); break;
    }
}

}  // namespace

bool sym_children(const SymPass &p, int &ll1, int &ll2, int &lr2)
{
    ll1 = log2_child(p.N1);
    const bool wide = p.N2 == 32768 && (ll1 == 8 || ll1 == 9);
    ll2 = wide ? 10 : log2_child(p.N2);
    lr2 = wide ? 5 : 4;
    const int lmax = ll1 + 4 > ll2 + lr2 ? ll1 + 4 : ll2 + lr2;
    return ll1 && ll2 && p.log2L >= lmax && p.log2N == ll1 + 4 + ll2 + lr2;
}

int sym_log2_child(const SymPass &p)
{
    int ll1 = 0, ll2 = 0, lr2 = 0;
    return sym_children(p, ll1, ll2, lr2) && ll1 == ll2 && lr2 == 4 ? ll1 : 0;
}

uint32_t sym_resident_groups(int pass, const SymPass &p)
{
    int ll1 = 0, ll2 = 0, lr2 = 0;
    if (!sym_children(p, ll1, ll2, lr2)) return 0;
    if (pass == 2)
        return lr2 != 5 ? 0 : ll1 == 8 ? resident(sym_middle_wide_kernel<8, 10>, 512) : resident(sym_middle_wide_kernel<9, 10>, 512);
    if (pass == 1) {
        switch (ll1) {
        case 9: return resident(sym_first_long_kernel<true, 9>, 512);
        case 10: return resident(sym_first_long_kernel<true, 10>, 1024);
        default: return 0;
        }
    }
    if (lr2 == 5) return resident(sym_last_long_kernel<10, 5>, 1024);
    switch (ll2) {
    case 9: return resident(sym_last_long_kernel<9, 4>, 512);
    case 10: return resident(sym_last_long_kernel<10, 4>, 1024);
    default: return 0;
    }
}

hipError_t launch_sym_first(const SymPass &p, hipStream_t s)
{
    int ll1 = 0, ll2 = 0, lr2 = 0;
    if (!sym_shape_ok(p, ll1, ll2, lr2)) return hipErrorInvalidValue;
    const dim3 grid(addr::sym1_groups(uint32_t(p.N2)));
    switch (ll1) {
    case 8: hipLaunchKernelGGL(sym_first_kernel<true>, grid, dim3(kSymThreads), 0, s, p); break;
    case 9: hipLaunchKernelGGL((sym_first_long_kernel<true, 9>), persistent(grid, p.resident1), dim3(512), 0, s, p, grid.x); break;
    default: hipLaunchKernelGGL((sym_first_long_kernel<true, 10>), persistent(grid, p.resident1), dim3(1024), 0, s, p, grid.x); break;
    }
    return hipGetLastError();
}

hipError_t launch_sym_middle(const SymPass &p, hipStream_t s)
{
    int ll1 = 0, ll2 = 0, lr2 = 0;
    if (!sym_shape_ok(p, ll1, ll2, lr2)) return hipErrorInvalidValue;
    if (lr2 == 5) {
        const dim3 grid(addr::sym2w_groups(uint32_t(p.N1), uint32_t(p.N2)));
        if (ll1 == 8)
            hipLaunchKernelGGL((sym_middle_wide_kernel<8, 10>), persistent(grid, p.resident2), dim3(512), 0, s, p, grid.x);
        else
            hipLaunchKernelGGL((sym_middle_wide_kernel<9, 10>), persistent(grid, p.resident2), dim3(512), 0, s, p, grid.x);
        return hipGetLastError();
    }
    const dim3 grid(addr::sym2_groups(uint32_t(p.N1), uint32_t(p.N2)));
    switch (ll1) {
    case 8: launch_middle<8>(ll2, grid, p, s); break;
    case 9: launch_middle<9>(ll2, grid, p, s); break;
    default: launch_middle<10>(ll2, grid, p, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_sym_last(const SymPass &p, hipStream_t s)
{
    int ll1 = 0, ll2 = 0, lr2 = 0;
    if (!sym_shape_ok(p, ll1, ll2, lr2)) return hipErrorInvalidValue;
    if (lr2 == 5) {
        const dim3 grid(addr::sym3r_groups(uint32_t(p.N1), 5));
        hipLaunchKernelGGL((sym_last_long_kernel<10, 5>), persistent(grid, p.resident3), dim3(1024), 0, s, p, grid.x);
        return hipGetLastError();
    }
    const dim3 grid(addr::sym3_groups(uint32_t(p.N1)));
    switch (ll2) {
    case 8: hipLaunchKernelGGL(sym_last_kernel, grid, dim3(kSymThreads), 0, s, p); break;
    case 9: hipLaunchKernelGGL((sym_last_long_kernel<9, 4>), persistent(grid, p.resident3), dim3(512), 0, s, p, grid.x); break;
    default: hipLaunchKernelGGL((sym_last_long_kernel<10, 4>), persistent(grid, p.resident3), dim3(1024), 0, s, p, grid.x); break;
    }
    return hipGetLastError();
}

}  // namespace paco
