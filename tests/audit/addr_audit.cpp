// Host audit of the kernels' address maps (paper_2609_06449_amd/csrc/addr.h):
// for every workgroup, thread and item of a pass, the item index each load
// and store uses is formed by the same functions the kernels call.  Checks:
//   - every index lies inside its buffer;
//   - every output item is written exactly once, every input item read
//     exactly once (the passes are permutations of their buffers);
//   - a pass that runs in place reads and writes the same items in every
//     workgroup (so no workgroup overwrites another's unread input);
//   - base + offset never wraps the 32-bit arithmetic the kernels use, and
//     the byte offset (index * 8) stays below 2^32;
//   - the digit maps are bijections whose inverse direction undoes the
//     forward one, the branch-free and the digit-by-digit forms agree, and
//     the XCD tile order is a permutation of the workgroup ids.
// Prints one line per check and exits non-zero on the first failure.
#include "addr.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

using namespace paco;

namespace {

int g_fail = 0;

#define CHECK(cond, ...)                                       \
    do {                                                       \
        if (!(cond)) {                                         \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__);   \
            std::printf(__VA_ARGS__);                          \
            std::printf("\n");                                 \
            std::exit(1);                                      \
        }                                                      \
    } while (0)

// A bitmap of N items that counts visits 0, 1, more.
struct Cover {
    uint64_t n;
    std::vector<uint64_t> once, twice;
    explicit Cover(uint64_t n_) : n(n_), once((n_ + 63) / 64), twice((n_ + 63) / 64) {}
    void hit(uint64_t i)
    {
        const uint64_t w = i >> 6, b = uint64_t(1) << (i & 63);
        if (once[w] & b) twice[w] |= b;
        once[w] |= b;
    }
    bool exact() const
    {
        for (uint64_t w = 0; w < once.size(); ++w) {
            const uint64_t full = (w + 1) * 64 <= n ? ~uint64_t(0) : ((uint64_t(1) << (n & 63)) - 1);
            if (once[w] != full || twice[w]) return false;
        }
        return true;
    }
};

// base + off as the kernels form it (uint32), checked against the exact sum
uint32_t item(uint32_t base, uint32_t off, uint64_t N, const char *what)
{
    const uint64_t exact = uint64_t(base) + uint64_t(off);
    CHECK(exact < (uint64_t(1) << 32), "%s: base + offset wraps 32 bits", what);
    CHECK(exact < N, "%s: index %llu outside [0, %llu)", what, (unsigned long long)exact, (unsigned long long)N);
    CHECK(exact * 8 < (uint64_t(1) << 32), "%s: byte offset beyond 32 bits", what);
    return uint32_t(exact);
}

// N1 = 16 L1, N2 = R L2 (L1 = 2^ll1, L2 = 2^ll2, R = 2^lr: 16, or 32 in the
// wide form): L1 (L2) threads per workgroup in pass 1 (3), 16 R in pass 2.
// The pass-3 maps of the persistent kernels (sym3r_, L2 >= 512) are checked
// for every R, and for R = 16 also against the sym3_ maps the L = 256 and
// MFMA kernels use, item by item.
void audit_sym(uint32_t ll1, uint32_t ll2, uint32_t lr = 4)
{
    const uint32_t R = 1u << lr, N1 = 16u << ll1, N2 = R << ll2, T1 = 1u << ll1, T3 = 1u << ll2;
    const uint64_t N = uint64_t(N1) * N2;
    const bool wide = lr == 5;
    {
        Cover rd(N), wr(N), blocks(addr::sym1_groups(N2));
        for (uint32_t g = 0; g < addr::sym1_groups(N2); ++g) {
            const uint32_t blk = addr::sym1_block(g, N2, ll1);
            CHECK(blk < addr::sym1_groups(N2), "sym pass 1 block id out of range");
            blocks.hit(blk);
            for (uint32_t tid = 0; tid < T1; ++tid)
                for (uint32_t i = 0; i < 16; ++i) {
                    rd.hit(item(addr::sym1_load_base(N2, blk, tid), addr::sym1_load_off(N2, i, ll1), N, "sym pass 1 load"));
                    wr.hit(item(addr::sym1_store_base(N2, blk, tid, ll1), addr::sym1_store_off(N2, i), N,
                                "sym pass 1 store"));
                }
        }
        CHECK(blocks.exact(), "sym pass 1 block order is not a permutation (%u x %u)", N1, N2);
        CHECK(rd.exact() && wr.exact(), "sym pass 1 is not a permutation (%u x %u)", N1, N2);
    }
    {
        const uint32_t groups = wide ? addr::sym2w_groups(N1, N2) : addr::sym2_groups(N1, N2);
        Cover rd(N), wr(N), blocks(groups);
        for (uint32_t g = 0; g < groups; ++g) {
            const uint32_t blk = addr::sym2_block(g, ll1, ll2);
            CHECK(blk < groups, "sym pass 2 block id out of range");
            blocks.hit(blk);
            for (uint32_t tid = 0; tid < 16 * R; ++tid)
                for (uint32_t i = 0; i < 16; ++i) {
                    rd.hit(item(addr::sym2_load_base(N2, blk, tid, ll1, ll2), addr::sym2_load_off(i), N,
                                "sym pass 2 load"));
                    wr.hit(wide ? item(addr::sym2w_store_base(N1, blk, tid, ll1), addr::sym2w_store_off(N1, i), N,
                                       "sym pass 2 store")
                                : item(addr::sym2_store_base(N1, blk, tid, ll1), addr::sym2_store_off(N1, i), N,
                                       "sym pass 2 store"));
                }
        }
        CHECK(blocks.exact(), "sym pass 2 block order is not a permutation (%u x %u)", N1, N2);
        CHECK(rd.exact() && wr.exact(), "sym pass 2 is not a permutation (%u x %u)", N1, N2);
    }
    for (int maps = wide ? 1 : 0; maps < (ll2 < 9 ? 1 : 2); ++maps) {  // 0: sym3_, 1: sym3r_ (L2 >= 512)
        const bool r = maps == 1;
        const uint32_t groups = r ? addr::sym3r_groups(N1, lr) : addr::sym3_groups(N1);
        Cover rd(N), wr(N), blocks(groups);
        std::vector<uint32_t> a, b;
        for (uint32_t g = 0; g < groups; ++g) {
            const uint32_t blk = r ? addr::sym3r_block(g, N1, ll2, lr) : addr::sym3_block(g, N1, ll2);
            CHECK(blk < groups, "sym pass 3 block id out of range");
            blocks.hit(blk);
            a.clear();
            b.clear();
            for (uint32_t tid = 0; tid < T3; ++tid)
                for (uint32_t i = 0; i < 16; ++i) {
                    const uint32_t ld =
                        r ? item(addr::sym3r_load_base(N1, blk, tid, lr), addr::sym3r_load_off(N1, i, ll2, lr), N,
                                 "sym pass 3 load")
                          : item(addr::sym3_load_base(N1, blk, tid), addr::sym3_load_off(N1, i, ll2), N,
                                 "sym pass 3 load");
                    const uint32_t st =
                        r ? item(addr::sym3r_store_base(N1, blk, tid, ll2, lr), addr::sym3r_store_off(N1, i, lr), N,
                                 "sym pass 3 store")
                          : item(addr::sym3_store_base(N1, blk, tid, ll2), addr::sym3_store_off(N1, i), N,
                                 "sym pass 3 store");
                    if (r && !wide) {
                        CHECK(addr::sym3r_block(g, N1, ll2, lr) == addr::sym3_block(g, N1, ll2) &&
                                  ld == item(addr::sym3_load_base(N1, blk, tid), addr::sym3_load_off(N1, i, ll2), N,
                                             "sym pass 3 load") &&
                                  st == item(addr::sym3_store_base(N1, blk, tid, ll2), addr::sym3_store_off(N1, i), N,
                                             "sym pass 3 store"),
                              "sym pass 3: the R = 16 maps differ from sym3_ (%u x %u)", N1, N2);
                    }
                    a.push_back(ld);
                    b.push_back(st);
                }
            for (uint32_t x : a) rd.hit(x);
            for (uint32_t x : b) wr.hit(x);
            std::sort(a.begin(), a.end());
            std::sort(b.begin(), b.end());
            CHECK(a == b, "sym pass 3 workgroup %u reads and writes different items (in place)", blk);
        }
        CHECK(blocks.exact(), "sym pass 3 block order is not a permutation (%u x %u)", N1, N2);
        CHECK(rd.exact() && wr.exact(), "sym pass 3 is not a permutation (%u x %u)", N1, N2);
    }
    std::printf("ok symmetric split form %u x %u (pass-2 Phase III radix %u): three passes are permutations, "
                "pass 3 in place per workgroup\n",
                N1, N2, R);
}

// the split form of Phase I for N1 = 16 M, every pass over every workgroup;
// pass 2 stores row u = digmap(c, t, m2, s2, forward)
void audit_split(uint32_t N1, uint32_t N2, int t, bool mixed)
{
    const uint64_t N = uint64_t(N1) * N2;
    int l2 = 0;
    while ((uint64_t(1) << l2) < N2) ++l2;
    const int m2 = l2 / t, s2 = l2 % t;
    if (!mixed && s2) return;
    Cover rd1(N), wr1(N);
    for (uint32_t blk = 0; blk < addr::split1_groups(N1, N2); ++blk)
        for (uint32_t tid = 0; tid < 256; ++tid)
            for (uint32_t i = 0; i < 16; ++i) {
                rd1.hit(item(addr::split1_load_base(N2, blk, tid), addr::split1_load_off(N1, N2, i), N, "split pass 1 load"));
                wr1.hit(item(addr::split1_store_base(N1, N2, blk, tid), addr::split1_store_off(N1, i), N,
                             "split pass 1 store"));
            }
    CHECK(rd1.exact() && wr1.exact(), "split pass 1 %ux%u is not a permutation", N1, N2);
    Cover rd2(N), wr2(N), rows(N2);
    const bool gen = !digrev_fast(t);
    for (uint32_t c = 0; c < N2; ++c) {
        const int64_t u64 = gen ? digmap<true>(c, t, m2, s2, false) : digmap<false>(c, t, m2, s2, false);
        CHECK(u64 >= 0 && u64 < int64_t(N2), "pass 2 row map out of range");
        const uint32_t u = uint32_t(u64);
        rows.hit(u);
        if (N1 == 4096) {
            for (uint32_t tid = 0; tid < 256; ++tid)
                for (uint32_t i = 0; i < 16; ++i) {
                    rd2.hit(item(addr::split2_load_base(N1, c, tid), addr::split2_load_off(i), N, "split pass 2 load"));
                    wr2.hit(item(addr::split2_store_base(N1, u, tid), addr::split2_store_off(i), N, "split pass 2 store"));
                }
        } else {
            const uint32_t R = N1 / 4096, npair = 16 / R;
            for (uint32_t tid = 0; tid < N1 / 16; ++tid) {
                for (uint32_t i = 0; i < 16; ++i)
                    rd2.hit(item(addr::split3_load_base(N1, c, tid), addr::split3_load_off(N1, i), N, "split pass 2 load"));
                for (uint32_t pr = 0; pr < npair; ++pr)
                    for (uint32_t kc = 0; kc < R; ++kc)
                        wr2.hit(item(addr::split3_store_base(N1, u, tid), addr::split3_store_off(N1, pr, kc), N,
                                     "split pass 2 store"));
            }
        }
    }
    CHECK(rows.exact(), "pass 2 row map of %u rows (b = 2^%d) is not a permutation", N2, t);
    CHECK(rd2.exact() && wr2.exact(), "split pass 2 %ux%u (b = 2^%d) is not a permutation", N1, N2, t);
    std::printf("ok split form %u x %u, b = 2^%d%s: passes 1 and 2 are permutations\n", N1, N2, t,
                s2 ? " (mixed radix)" : "");
}

void audit_digit_maps()
{
    for (int t = 1; t <= 8; ++t)
        for (int l = 0; l <= 16; ++l) {
            const int ell = l / t, s = l % t;
            const int64_t n = int64_t(1) << l;
            Cover fwd{uint64_t(n)}, inv{uint64_t(n)};
            for (int64_t x = 0; x < n; ++x) {
                const int64_t f = digmap<true>(x, t, ell, s, false), g = digmap<true>(x, t, ell, s, true);
                CHECK(f >= 0 && f < n && g >= 0 && g < n, "digmap out of range");
                CHECK(digmap<true>(f, t, ell, s, true) == x, "digmap inverse does not undo the forward map");
                if (digrev_fast(t)) {
                    CHECK(digmap<false>(x, t, ell, s, false) == f && digmap<false>(x, t, ell, s, true) == g,
                          "branch-free and digit-by-digit digit maps differ (t = %d, l = %d)", t, l);
                }
                fwd.hit(uint64_t(f));
                inv.hit(uint64_t(g));
                if (s == 0) CHECK(f == g, "pi_ell is not an involution");
            }
            CHECK(fwd.exact() && inv.exact(), "digmap is not a bijection (t = %d, l = %d)", t, l);
        }
    // compile-time digit reversal of the fast tiles against the run-time one
    for (uint32_t x = 0; x < 4096; ++x) {
        const uint32_t a = drev<4, 3>(x), b = drev<2, 6>(x), c = drev<1, 12>(x);
        CHECK(a == uint32_t(digrev<true>(x, 4, 3)), "drev with b = 16 differs");
        CHECK(b == uint32_t(digrev<true>(x, 2, 6)), "drev with b = 4 differs");
        CHECK(c == uint32_t(digrev<true>(x, 1, 12)), "drev with b = 2 differs");
    }
    std::printf("ok digit maps: t = 1..8, lengths up to 2^16, bijections, inverse, branch-free = digit-by-digit\n");
    for (int64_t G = 1; G <= 4096; G += (G < 64 ? 1 : 37)) {
        Cover c{uint64_t(G)};
        for (int64_t i = 0; i < G; ++i) {
            const int64_t o = tile_order(i, G);
            CHECK(o >= 0 && o < G, "tile order out of range");
            c.hit(uint64_t(o));
        }
        CHECK(c.exact(), "tile order of %lld workgroups is not a permutation", (long long)G);
    }
    std::printf("ok XCD tile order: a permutation of the workgroup ids\n");
}

}  // namespace

// The MFMA passes' LDS exchange buffers (16 rows of 256 logical items): the
// stage-1 stores of 4 waves x 4 groups x 4 outputs x 64 lanes fill every slot
// once, inside the buffer, and leave the two spare items (the FP16x3 tile
// scale's scratch) alone; every stage-2 component load reads the slot its
// logical item was stored to; and (the layouts' purpose) every store
// half-wave covers 32 distinct 8-byte slots, every load wave 64 distinct
// 4-byte banks.
template <class Store, class Load>
void audit_mf_exchange(const char *name, int items, Store store, Load load, bool load_across_rows, int spare)
{
    std::vector<int> at(items, -1);  // logical item (row * 256 + col) per slot
    std::vector<int> slot_of(16 * 256, -1);
    for (int w = 0; w < 4; ++w)
        for (int G = 0; G < 4; ++G)
            for (int i = 0; i < 4; ++i) {
                const int j = 4 * w + G;
                int slots[64];
                for (int l = 0; l < 64; ++l) {
                    const int n = l & 15, kb = l >> 4;
                    const int a = store(kb, i, j, n);
                    CHECK(a >= 0 && a < items, "%s: store %d outside %d items", name, a, items);
                    CHECK(at[a] < 0, "%s: slot %d stored twice", name, a);
                    CHECK(spare < 0 || a < spare || a >= spare + 2, "%s: store to spare slot %d", name, a);
                    const int logical = (4 * kb + i) * 256 + 16 * j + n;
                    at[a] = logical;
                    slot_of[logical] = a;
                    slots[l] = a & 31;
                }
                for (int h = 0; h < 2; ++h) {
                    uint32_t seen = 0;
                    for (int l = 32 * h; l < 32 * h + 32; ++l) seen |= 1u << slots[l];
                    CHECK(seen == 0xffffffffu, "%s: store half-wave %d of (w %d, G %d, i %d) shares a slot", name, h, w,
                          G, i);
                }
            }
    for (int w = 0; w < 4; ++w)
        for (int G = 0; G < 4; ++G)
            for (int i = 0; i < 8; ++i) {
                const int g = 4 * w + G;
                uint64_t banks = 0;
                for (int l = 0; l < 64; ++l) {
                    const int n = l & 15, kb = l >> 4, half = kb & 1, comp = kb >> 1;
                    const int a = load(load_across_rows ? n : g, half, i, load_across_rows ? g : n);
                    const int logical =
                        load_across_rows ? n * 256 + 16 * (8 * half + i) + g : g * 256 + 16 * (8 * half + i) + n;
                    CHECK(a >= 0 && a < items && at[a] == logical, "%s: load (w %d, G %d, i %d, lane %d) reads slot %d",
                          name, w, G, i, l, a);
                    banks |= uint64_t(1) << ((2 * a + comp) & 63);
                }
                CHECK(banks == ~uint64_t(0), "%s: load wave (w %d, G %d, i %d) shares a bank", name, w, G, i);
            }
    for (int v : slot_of) CHECK(v >= 0, "%s: a logical item is never stored", name);
    std::printf("ok   MFMA exchange buffer %s (%d items)\n", name, items);
}

// The L = 512 exchange buffers (8 waves; stage-B groups 2 g + jp): the same
// checks as audit_mf_exchange.  across: pass 1 (stage-B loads run across
// rows n), else pass 3 (one row g per group).
template <class Store, class Load>
void audit_mf_exchange_512(const char *name, Store store, Load load, bool across)
{
    const int items = addr::kMfLItems;
    std::vector<int> at(items, -1);
    for (int w = 0; w < 8; ++w)
        for (int G = 0; G < 4; ++G)
            for (int i = 0; i < 4; ++i) {
                const int j = 4 * w + G;
                int slots[64];
                for (int l = 0; l < 64; ++l) {
                    const int n = l & 15, kb = l >> 4;
                    const int a = store(kb, i, j, n);
                    CHECK(a >= 0 && a < items, "%s: store %d outside %d items", name, a, items);
                    CHECK(at[a] < 0, "%s: slot %d stored twice", name, a);
                    at[a] = (4 * kb + i) * 512 + 16 * j + n;
                    slots[l] = a & 31;
                }
                for (int h = 0; h < 2; ++h) {
                    uint32_t seen = 0;
                    for (int l = 32 * h; l < 32 * h + 32; ++l) seen |= 1u << slots[l];
                    CHECK(seen == 0xffffffffu, "%s: store half-wave shares a slot", name);
                }
            }
    for (int w = 0; w < 8; ++w)
        for (int G = 0; G < 4; ++G)
            for (int i = 0; i < 8; ++i) {
                const int g = 2 * w + (G >> 1), jp = G & 1;
                uint64_t banks = 0;
                for (int l = 0; l < 64; ++l) {
                    const int n = l & 15, kb = l >> 4, half = kb & 1, comp = kb >> 1;
                    const int col = 16 * (jp + 2 * (8 * half + i)) + (across ? g : n);
                    const int row = across ? n : g;
                    const int a = across ? load(n, half, i, jp, g) : load(g, half, i, jp, n);
                    CHECK(a >= 0 && a < items && at[a] == row * 512 + col, "%s: load reads slot %d", name, a);
                    banks |= uint64_t(1) << ((2 * a + comp) & 63);
                }
                CHECK(banks == ~uint64_t(0), "%s: load wave shares a bank", name);
            }
    int stored = 0;
    for (int v : at) stored += v >= 0;
    CHECK(stored == 16 * 512, "%s: not every logical item stored", name);
    std::printf("ok   MFMA exchange buffer %s (%d items)\n", name, items);
}

int main(int argc, char **argv)
{
    const bool full = argc > 1;  // also the 2^28 shapes (about 2 x 2^28 items per pass)
    audit_digit_maps();
    audit_sym(8, 8);
    audit_sym(9, 9);
    audit_sym(8, 9);
    audit_sym(9, 8);
    audit_sym(8, 10, 5);  // 4096 x 32768, the wide form
    audit_mf_exchange("pass 1", addr::kMf1Items, addr::mf1_store, addr::mf1_load, true, addr::kMf1Spare);
    audit_mf_exchange("pass 2", 16 * 256, addr::mf2_store, addr::mf2_load, false, -1);
    audit_mf_exchange("pass 3", addr::kMf1Items, addr::mf3_store, addr::mf3_load, false, addr::kMf3Spare);
    audit_mf_exchange_512("pass 1, L = 512", addr::mf1L_store, addr::mf1L_load, true);
    audit_mf_exchange_512("pass 3, L = 512", addr::mf3L_store, addr::mf3L_load, false);
    const uint32_t n1s[] = {4096, 8192, 16384};
    const uint32_t n2s[] = {16, 64, 256, 2048, 4096};
    for (uint32_t N1 : n1s)
        for (uint32_t N2 : n2s)
            for (int t : {1, 2, 3, 4})
                audit_split(N1, N2, t, true);
    if (full) {  // the 2^28 shapes the benchmark times, every workgroup
        audit_sym(10, 10);
        audit_sym(8, 10);
        audit_sym(10, 8);
        audit_sym(9, 10);
        audit_sym(10, 9);
        audit_sym(9, 10, 5);  // 8192 x 32768
        audit_split(16384, 16384, 2, false);
        audit_split(16384, 16384, 4, true);
        audit_split(8192, 32768, 1, false);
        audit_split(8192, 32768, 3, false);
        audit_split(4096, 16384, 2, false);
    }
    std::printf("address audit passed\n");
    return g_fail;
}
