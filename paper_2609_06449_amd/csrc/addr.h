// Address maps of the kernels: which item of which buffer each thread of each
// workgroup loads or stores.  The kernels compute their addresses with these
// functions, and a host audit (tests/audit/addr_audit.cpp) enumerates the
// same functions over every workgroup, thread and item of a pass to check
// that every address lies inside its buffer, every output item is written
// exactly once, in-place passes read and write the same items, and the
// 32-bit byte offsets never wrap.  Plain C++ (no HIP header): compiled for
// the device by the library and for the host by the audit.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define PACO_HD __host__ __device__ __forceinline__
#else
#define PACO_HD inline
#endif

namespace paco {

// ---- digit reversals (appendix A.1) ---------------------------------------

// pi_ell in base b = 2^t: the ell groups of t bits of x in the opposite
// order.  ell == 0 is the identity.
PACO_HD int64_t digit_reverse_bits(int64_t x, int t, int ell)
{
    if (ell == 0) return x;
    int64_t r = 0;
    const int64_t m = (int64_t(1) << t) - 1;
    for (int g = 0; g < ell; ++g) {
        r = (r << t) | (x & m);
        x >>= t;
    }
    return r;
}

// The same permutation for b = 2^t with t in {1, 2, 4, 8} (t*ell <= 32):
// reverse all t*ell bits, then restore the bit order inside each t-bit digit
// with up to three mask swaps.  Branch-free; GEN selects the digit-by-digit
// loop for other t.
template <bool GEN = false>
PACO_HD int64_t digrev(int64_t x, int t, int ell)
{
    if constexpr (GEN) {
        return digit_reverse_bits(x, t, ell);
    } else {
        const int nb = t * ell;
        uint32_t r = __builtin_bitreverse32(uint32_t(x)) >> ((32 - nb) & 31);
        const uint32_t s1 = ((r & 0x55555555u) << 1) | ((r >> 1) & 0x55555555u);
        r = t >= 2 ? s1 : r;
        const uint32_t s2 = ((r & 0x33333333u) << 2) | ((r >> 2) & 0x33333333u);
        r = t >= 4 ? s2 : r;
        const uint32_t s3 = ((r & 0x0F0F0F0Fu) << 4) | ((r >> 4) & 0x0F0F0F0Fu);
        r = t >= 8 ? s3 : r;
        return nb == 0 ? x : int64_t(r);
    }
}

// Mixed-radix digit maps over [0, b^ell 2^s) (0 <= s < t): the digits are
// (b, ..., b, 2^s), least significant first.  The forward map pi reverses
// the digit string and reads it with the radices reversed:
//     pi(x)     = (x >> t ell) + digrev(x mod b^ell) 2^s
//     pi^-1(u)  = digrev(u >> s) + (u mod 2^s) b^ell      (inv = true)
// s = 0: both are digrev (pi_ell is an involution).
template <bool GEN = false>
PACO_HD int64_t digmap(int64_t x, int t, int ell, int s, bool inv)
{
    if (s == 0) return digrev<GEN>(x, t, ell);
    const int nb = t * ell;
    if (inv) return digrev<GEN>(x >> s, t, ell) | ((x & ((int64_t(1) << s) - 1)) << nb);
    return (x >> nb) | (digrev<GEN>(x & ((int64_t(1) << nb) - 1), t, ell) << s);
}

// True when the branch-free digit reversal covers digit width t.
PACO_HD constexpr bool digrev_fast(int t) { return t == 1 || t == 2 || t == 4 || t == 8; }

// Digit reversal with compile-time digit width TB and digit count ND.
template <int TB, int ND>
PACO_HD uint32_t drev(uint32_t x)
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

// Tile order: the hardware deals consecutive workgroup ids to the 8 XCDs in
// turn.  Renumber so that the workgroups one XCD receives back to back own
// neighbouring column tiles, which share 128-byte lines in that XCD's L2.
PACO_HD int64_t tile_order(int64_t i, int64_t G)
{
    if (G & 7) return i;
    return (i & 7) * (G >> 3) + (i >> 3);
}

namespace addr {

// Each map is a per-thread base plus a per-item offset (item indices, not
// bytes, into the pass's source or destination buffer): the kernels form one
// pointer from the base and add the offsets, the audit adds the two.

// ---- the symmetric split form (sym.hip), N1 = N2 = 16 L, L = 2^ll ----------
// (ll = 8, 9, 10: N = 2^24, 2^26, 2^28).  Workgroup blk, L threads (256 for
// ll = 8), item i < 16.  With P = L / 256 threads per M-point stage-B
// transform (M = L / 16): thread tid of passes 1 and 3 is (cl, jl) =
// (tid & 15, tid >> 4) in stage A and, in stage B, k fastest in pass 1
// (ka, jp, cl) = (tid & 15, (tid >> 4) & (P - 1), tid >> (4 + ll - 8)) and
// column fastest in pass 3 (cl, jp, ka) = (tid & 15, (tid >> 4) & (P - 1),
// tid >> (4 + ll - 8)); jp picks the outputs kB = i + 16 jp of the thread.

// Block orders: the hardware's workgroup id g of a pass maps to its tile blk
// (a permutation of [0, groups)); the order decides which tiles run at the
// same time, and so how far apart in HBM their loads and stores fall.
// Measured per L (pass times in us, transform in ms):
//   L = 256  (4096^2):  tile order (cb / vb fastest) in passes 1 and 3, jc
//            fastest in pass 2: 42.0 / 54.3 / 42.4; other orders within 1-2%.
//   L = 512  (8192^2):  the same in passes 1 and 3, kb fastest in pass 2
//            (its stores then fill whole rows): 264 / 212 / 244, 0.706 ms,
//            against 262 / 276 / 243 (0.756) with jc fastest.
//   L = 1024 (16384^2): r (q0) fastest in passes 1 (3), kb fastest in pass 2:
//            1215 / 879 / 1328, 3.43 ms, against 1309 / 922 / 1399 (3.67).
//   L1 = 512 with N2 = 2^15 (8192 x 32768, the wide form): r fastest in
//            pass 1 (974-1014 against 1012-1037 us; at 8192^2 it measured
//            247 against 220 us), vb fastest in pass 3 (sym3r_block: 1157-
//            1172 against 1172-1181 us).
PACO_HD uint32_t sym1_block(uint32_t g, uint32_t N2, uint32_t ll = 8)
{
    const bool r_fastest = ll >= 10 || (ll == 9 && N2 >= 32768u);
    return r_fastest ? (g & 15u) * (N2 >> 4) + (g >> 4) : g;  // r fastest : cb fastest
}
PACO_HD uint32_t sym3_block(uint32_t g, uint32_t N1, uint32_t ll = 8)
{
    return ll >= 10 ? (g & 15u) * (N1 >> 4) + (g >> 4) : g;  // q0 fastest : vb fastest
}

// pass 1: workgroup (r, cb) = (blk / (N2/16), blk mod (N2/16)); thread
// (cl, jl) loads row 16 (jl + (L/16) i) + r, column 16 cb + cl
PACO_HD uint32_t sym1_load_base(uint32_t N2, uint32_t blk, uint32_t tid)
{
    const uint32_t ncb = N2 >> 4, cb = blk % ncb, r = blk / ncb;
    return (16u * (tid >> 4) + r) * N2 + (cb << 4) + (tid & 15u);
}
PACO_HD uint32_t sym1_load_off(uint32_t N2, uint32_t i, uint32_t ll = 8) { return (i << ll) * N2; }
// The workspace between passes 1 and 2 holds U[c][r][k] at
//     ((k >> 4) N2 + c) 256 + 16 r + (k & 15),
// so that pass 2 reads 2 KiB runs (all r of 16 consecutive k of one column).
// Stage-B thread (ka, jp, cl) stores U[c][r][ka + 16 (i + 16 jp)], c = 16 cb + cl.
PACO_HD uint32_t sym1_store_base(uint32_t N2, uint32_t blk, uint32_t tid, uint32_t ll = 8)
{
    const uint32_t ncb = N2 >> 4, cb = blk % ncb, r = blk / ncb;
    const uint32_t jp = (tid >> 4) & ((1u << (ll - 8)) - 1u), cl = tid >> (ll - 4);
    return ((16u * jp * N2 + (cb << 4) + cl) << 8) + 16u * r + (tid & 15u);
}
PACO_HD uint32_t sym1_store_off(uint32_t N2, uint32_t i) { return i * N2 * 256u; }
// pass 2 (children L1 = N1/16 of Phase I, L2 = N2/16 of Phase III; ll1,
// ll2 their log2): tile blk = (L1/16) jc + kb, jc < L2, kb < L1/16.
// L1 = 256: the hardware's workgroup id g maps to (jc, kb) = (g mod L2,
// g / L2) (jc fastest: neighbouring workgroups read neighbouring 2 KiB runs);
// L1 >= 512: blk = g (kb fastest: the running workgroups' stores fill whole
// rows of W).  Thread (kk, rr) loads U[jc + L2 rr][i][16 kb + kk].
PACO_HD uint32_t sym2_block(uint32_t g, uint32_t ll1, uint32_t ll2)
{
    return ll1 == 8 ? ((g & ((1u << ll2) - 1u)) << (ll1 - 4)) | (g >> ll2) : g;
}
PACO_HD uint32_t sym2_load_base(uint32_t N2, uint32_t blk, uint32_t tid, uint32_t ll1, uint32_t ll2)
{
    const uint32_t kb = blk & ((1u << (ll1 - 4)) - 1u), jc = blk >> (ll1 - 4);
    return ((kb * N2 + jc + ((tid >> 4) << ll2)) << 8) + (tid & 15u);
}
PACO_HD uint32_t sym2_load_off(uint32_t i) { return 16u * i; }
// thread (kk, s) stores W at row 16 jc + i, column 16 kb + kk + L1 s
PACO_HD uint32_t sym2_store_base(uint32_t N1, uint32_t blk, uint32_t tid, uint32_t ll1)
{
    const uint32_t kb = blk & ((1u << (ll1 - 4)) - 1u), jc = blk >> (ll1 - 4);
    return 16u * jc * N1 + 16u * kb + (tid & 15u) + ((tid >> 4) << ll1);
}
PACO_HD uint32_t sym2_store_off(uint32_t N1, uint32_t i) { return i * N1; }
// pass 3: workgroup (q0, vb) = (blk / (N1/16), blk mod (N1/16)); thread
// (cl, jl) loads row 16 (jl + (L/16) i) + q0, column 16 vb + cl
PACO_HD uint32_t sym3_load_base(uint32_t N1, uint32_t blk, uint32_t tid)
{
    const uint32_t nvb = N1 >> 4, vb = blk % nvb, q0 = blk / nvb;
    return (16u * (tid >> 4) + q0) * N1 + (vb << 4) + (tid & 15u);
}
PACO_HD uint32_t sym3_load_off(uint32_t N1, uint32_t i, uint32_t ll = 8) { return (i << ll) * N1; }
// stage-B thread (cl, jp, ka) stores row q0 + 16 q, q = ka + 16 (i + 16 jp)
PACO_HD uint32_t sym3_store_base(uint32_t N1, uint32_t blk, uint32_t tid, uint32_t ll = 8)
{
    const uint32_t nvb = N1 >> 4, vb = blk % nvb, q0 = blk / nvb;
    const uint32_t jp = (tid >> 4) & ((1u << (ll - 8)) - 1u), ka = tid >> (ll - 4);
    return (q0 + 16u * ka + 4096u * jp) * N1 + (vb << 4) + (tid & 15u);
}
PACO_HD uint32_t sym3_store_off(uint32_t N1, uint32_t i) { return 256u * i * N1; }
// workgroup counts of the three passes
PACO_HD uint32_t sym1_groups(uint32_t N2) { return 16u * (N2 >> 4); }
PACO_HD uint32_t sym2_groups(uint32_t N1, uint32_t N2) { return (N2 >> 4) * (N1 >> 8); }
PACO_HD uint32_t sym3_groups(uint32_t N1) { return 16u * (N1 >> 4); }

// ---- Phase III child of radix R = 2^lr in pass 2 (lr = 4 as above, or 5) --
// With N2 = R L2 the Phase III split is j2 = jc + L2 rr, k2 = q0 + R q (rr,
// q0 < R; jc, q < L2): pass 2 stores W at row R jc + q0, pass 3 transforms
// rows R t + q0 (t < L2) of each 16-column tile and stores row q0 + R q.
// R = 32 (the wide form) takes N2 = 2^15 with L2 = 1024 on chip; pass 1 and
// its workspace do not depend on R.  For lr = 4 the pass-3 maps below equal
// the sym3_ maps above.
// Pass 2, R = 32: 512 threads per workgroup.  Loads as sym2_load_base with
// thread (kk, rr), rr < 32.  Stores by thread (kk, p, s) = (tid & 15,
// (tid >> 4) & 1, tid >> 5), which holds outputs q0 = i + 16 p of the
// 32-point transform: row 32 jc + 16 p + i, column 16 kb + kk + L1 s.
PACO_HD uint32_t sym2w_store_base(uint32_t N1, uint32_t blk, uint32_t tid, uint32_t ll1)
{
    const uint32_t kb = blk & ((1u << (ll1 - 4)) - 1u), jc = blk >> (ll1 - 4);
    return (32u * jc + 16u * ((tid >> 4) & 1u)) * N1 + 16u * kb + (tid & 15u) + ((tid >> 5) << ll1);
}
PACO_HD uint32_t sym2w_store_off(uint32_t N1, uint32_t i) { return i * N1; }
PACO_HD uint32_t sym2w_groups(uint32_t N1, uint32_t N2) { return (N2 >> 5) * (N1 >> 8); }
// Pass 3 at L = 2^ll >= 512 (the persistent kernels): tile (q0, vb), q0
// fastest at ll >= 10 for R = 16 as in sym3_block, vb fastest otherwise
PACO_HD uint32_t sym3r_block(uint32_t g, uint32_t N1, uint32_t ll, uint32_t lr)
{
    return ll >= 10 && lr == 4 ? (g & 15u) * (N1 >> 4) + (g >> 4) : g;
}
// thread (cl, jl) loads row R (jl + (L/16) i) + q0, column 16 vb + cl
PACO_HD uint32_t sym3r_load_base(uint32_t N1, uint32_t blk, uint32_t tid, uint32_t lr)
{
    const uint32_t nvb = N1 >> 4, vb = blk % nvb, q0 = blk / nvb;
    return (((tid >> 4) << lr) + q0) * N1 + (vb << 4) + (tid & 15u);
}
PACO_HD uint32_t sym3r_load_off(uint32_t N1, uint32_t i, uint32_t ll, uint32_t lr)
{
    return (i << (ll + lr - 4)) * N1;
}
// stage-B thread (cl, jp, ka) stores row q0 + R q, q = ka + 16 (i + 16 jp)
PACO_HD uint32_t sym3r_store_base(uint32_t N1, uint32_t blk, uint32_t tid, uint32_t ll, uint32_t lr)
{
    const uint32_t nvb = N1 >> 4, vb = blk % nvb, q0 = blk / nvb;
    const uint32_t jp = (tid >> 4) & ((1u << (ll - 8)) - 1u), ka = tid >> (ll - 4);
    return (q0 + (ka << lr) + (jp << (lr + 8))) * N1 + (vb << 4) + (tid & 15u);
}
PACO_HD uint32_t sym3r_store_off(uint32_t N1, uint32_t i, uint32_t lr) { return (i << (lr + 4)) * N1; }
PACO_HD uint32_t sym3r_groups(uint32_t N1, uint32_t lr) { return (N1 >> 4) << lr; }

// Exchange buffers of the MFMA passes (sym_mf.hip): 16 rows of 256 items.
// Stage-1 results: lane (n, kb) stores output i of group j, logical row
// 4 kb + i, column 16 j + n (8-byte stores; a half-wave covers two rows).
// Stage-2 operands, one component per 4-byte load: pass 1 lane (n, half)
// loads operand i of group c (row n, column 16 (8 half + i) + c); passes 2
// and 3 lane (n, half) of group row g load row g, column 16 (8 half + i) + n.
// Pass 1 (loads across rows): item (row, col) at row * 260 + col + (col >>
// 7) + 2 (row >> 3 & 1); pass 3: row * 260 + (col ^ 16 (col >> 7)); both
// 4160 items (at most four workgroups per CU, which measured faster for
// these two passes than five).  Pass 2: row * 256 + (col ^ 16 b), b = bit 2
// of row xor bit 7 of col, 4096 items (32 KiB: five workgroups per CU).
// Every store half-wave hits 32 distinct 8-byte slots, every load wave 64
// distinct banks; each lane's addresses are one or two bases plus
// compile-time offsets (i and j are unrolled constants).
constexpr int kMf1Items = 16 * 260;  // passes 1 and 3
// items no stage-1 store of pass 1 (pass 3) touches: two from here on hold
// four floats of workgroup scratch
constexpr int kMf1Spare = 257, kMf3Spare = 256;
PACO_HD int mf1_store(int kb, int i, int j, int n)
{
    return (4 * kb + i) * 260 + 2 * (kb >> 1) + 16 * j + (j >> 3) + n;
}
PACO_HD int mf1_load(int n, int half, int i, int c) { return n * 260 + 2 * (n >> 3) + 129 * half + 16 * i + c; }
PACO_HD int mf3_store(int kb, int i, int j, int n) { return (4 * kb + i) * 260 + ((16 * j) ^ (16 * (j >> 3))) + n; }
PACO_HD int mf3_load(int g, int half, int i, int n)
{
    const int b0 = g * 260 + 144 * half + n;
    return ((i & 1) ? b0 - 32 * half : b0) + 16 * i;
}
// L = 512 (N1 = N2 = 8192): 16 rows of 512 columns, row stride 516.  Stage-B
// butterflies of both passes pair up as groups 2 g + jp (jp: the half of
// the 32-point transform), so their loads add 16 jp to the column: pass 1
// loads row n, column 16 (jp + 2 (8 half + i)) + c; pass 3 loads row g,
// column 16 (jp + 2 (8 half + i)) + n.  Pass 1: item (row, col) at
// row * 516 + col + (col >> 8) + 2 (row >> 3 & 1); pass 3: row * 516 +
// (col ^ 16 (col >> 8)).  Conflict-free as above (checked by the audit).
constexpr int kMfLStride = 516, kMfLItems = 16 * kMfLStride;
PACO_HD int mf1L_store(int kb, int i, int j, int n)
{
    return (4 * kb + i) * kMfLStride + 16 * j + n + (j >> 4) + 2 * (kb >> 1);
}
PACO_HD int mf1L_load(int n, int half, int i, int jp, int c)
{
    return n * kMfLStride + 2 * (n >> 3) + 257 * half + 32 * i + 16 * jp + c;
}
PACO_HD int mf3L_store(int kb, int i, int j, int n) { return (4 * kb + i) * kMfLStride + 16 * (j ^ (j >> 4)) + n; }
PACO_HD int mf3L_load(int g, int half, int i, int jp, int n)
{
    return g * kMfLStride + 256 * half + 32 * i + n + 16 * (jp ^ half);
}
PACO_HD int mf2_store(int kb, int i, int j, int n)
{
    const int f = (kb ^ (j >> 3)) & 1;
    return (4 * kb + i) * 256 + 16 * j + ((j & 1) ? -16 * f : 16 * f) + n;
}
PACO_HD int mf2_load(int g, int half, int i, int n)
{
    const int f = ((g >> 2) ^ half) & 1;
    const int b0 = g * 256 + 128 * half + n + 16 * f;
    return ((i & 1) ? b0 - 32 * f : b0) + 16 * i;
}

// ---- the split form of Phase I (split.hip), N1 = 16 M -------------------------

// pass 1: workgroup (cg, jg) = (blk mod (N2/16), blk / (N2/16)), 256
// threads (cl, jl); thread loads row j + M i (j = 16 jg + jl), column 16 cg + cl
PACO_HD uint32_t split1_load_base(uint32_t N2, uint32_t blk, uint32_t tid)
{
    const uint32_t ncg = N2 >> 4, cg = blk % ncg, jg = blk / ncg;
    return ((jg << 4) + (tid >> 4)) * N2 + (cg << 4) + (tid & 15u);
}
PACO_HD uint32_t split1_load_off(uint32_t N1, uint32_t N2, uint32_t i) { return (N1 >> 4) * i * N2; }
// store q < 16 of thread tid: column 16 cg + q, items 256 jg + tid of its T
PACO_HD uint32_t split1_store_base(uint32_t N1, uint32_t N2, uint32_t blk, uint32_t tid)
{
    const uint32_t ncg = N2 >> 4, cg = blk % ncg, jg = blk / ncg;
    return (cg << 4) * N1 + (jg << 8) + tid;
}
PACO_HD uint32_t split1_store_off(uint32_t N1, uint32_t q) { return q * N1; }
PACO_HD uint32_t split1_groups(uint32_t N1, uint32_t N2) { return (N2 >> 4) * (N1 >> 8); }

// pass 2, N1 = 4096: workgroup c, 256 threads (lo, hi) = (tid & 15, tid >> 4):
// loads T[c][hi + 16 i][lo]; stores row u (the caller's pi_{m2}(c)),
// frequency lo + 16 hi + 256 i
PACO_HD uint32_t split2_load_base(uint32_t N1, uint32_t c, uint32_t tid) { return c * N1 + tid; }
PACO_HD uint32_t split2_load_off(uint32_t i) { return 256u * i; }
PACO_HD uint32_t split2_store_base(uint32_t N1, uint32_t u, uint32_t tid) { return u * N1 + tid; }
PACO_HD uint32_t split2_store_off(uint32_t i) { return 256u * i; }

// pass 2, N1 = 16 M with M = 256 R: workgroup c, M threads, thread
// (k0, jl) = (tid & 15, tid >> 4) loads T[c][jl + (M/16) i][k0]; stage C
// thread (k0, q) stores, for pair i < 16 / R and kc < R, frequency
// k0 + 16 (q + (M/16) i) + 4096 kc of row u
PACO_HD uint32_t split3_load_base(uint32_t N1, uint32_t c, uint32_t tid) { return c * N1 + tid; }
PACO_HD uint32_t split3_load_off(uint32_t N1, uint32_t i) { return (N1 >> 8) * 16u * i; }
PACO_HD uint32_t split3_store_base(uint32_t N1, uint32_t u, uint32_t tid) { return u * N1 + tid; }
PACO_HD uint32_t split3_store_off(uint32_t N1, uint32_t pair, uint32_t kc) { return 16u * (N1 >> 8) * pair + 4096u * kc; }

}  // namespace addr
}  // namespace paco
