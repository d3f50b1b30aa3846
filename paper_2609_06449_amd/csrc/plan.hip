// C ABI of the PACO library: validation, planning and execution on the
// caller's stream.  Host code only; the kernels live in local_fft.hip and
// middle.hip.
#include <cmath>
#include <cstdio>
#include <mutex>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "paco.h"
#include "paco_internal.h"

using paco::LocalPass;
using paco::MiddlePass;

// The workspace of paco_execute_noalloc: one array per GPU, in device memory
// for as long as the process runs.  In host code `scratch` is only a
// stand-in for the symbol: its device address comes from
// hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) float2 scratch[PACO_NOALLOC_MAX_ITEMS];

namespace {

thread_local std::string g_last_error;

paco_status fail(paco_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

paco_status hip_fail(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return PACO_ERR_HIP;
}

int ilog2_exact(int64_t n)
{
    if (n < 1 || (n & (n - 1))) return -1;
    int l = 0;
    while ((int64_t(1) << l) < n) ++l;
    return l;
}

constexpr int kMaxLocalLog2 = 16;  // N1, N2 <= 2^16 (at most two on-chip passes)
constexpr int kMaxTotalLog2 = 28;  // N1*N2 <= 2^28: every buffer < 4 GiB (32-bit byte offsets)

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's scratch array (looked up on the first call
// for that device); nullptr with the reason in `err` on failure.
void *scratch_for_device(int dev, std::string &err)
{
    if (dev < 0 || dev >= kMaxDevices) {
        err = "device ordinal beyond the library's table";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

void paco::set_last_error(const std::string &msg) { g_last_error = msg; }

struct paco_plan_s {
    int64_t N1 = 0, N2 = 0, p = 0;
    int32_t b = 0;
    paco_dtype dt = PACO_C64;
    int t = 0, m1 = 0, m2 = 0, l1 = 0, l2 = 0, lN = 0, lL = 0, lLo = 0;
    int s1 = 0, s2 = 0;  // short top digit of N1 / N2 (mixed-radix plans)
    bool mixed = false;
    int device = 0;
    void *dev_tables = nullptr;
    std::vector<LocalPass> phase1, phase3;  // src/dst filled per execution
    MiddlePass mid{};
    bool fused = false;                     // packed Phase-I buffer (see paco_execute)
    LocalPass phase1_packed{};
    bool two_pass = false;                  // Phase III can read the packed buffer itself
    LocalPass phase1_two{}, phase3_two{};   // the two-pass form's passes
    bool split = false;                     // N1 = 2^12: Phase I split 16 x 256 across passes 1 and 2
    paco::SplitPass split_pass{};           // src/dst filled per execution
    bool sym = false;                       // N1 = N2 = 16 L: the symmetric split form (three passes)
    paco::SymPass sym_pass{};               // src/dst filled per execution
    paco_plan_s *inv = nullptr;             // N2 x N1 passes of the inverse (NULL: square, this plan's)
    void *scratch = nullptr;                // this device's scratch array (paco_execute_noalloc)
    std::string scratch_error;              // why scratch is NULL
    std::string inv_error;                  // non-empty: the inverse passes could not be built
    std::string desc;
};

extern "C" {

const char *paco_status_string(paco_status st)
{
    switch (st) {
    case PACO_OK: return "ok";
    case PACO_ERR_INVALID_ARG: return "invalid argument";
    case PACO_ERR_NOT_POWER_OF_B: return "N1/N2 not a power of b (or b not a power of two >= 2)";
    case PACO_ERR_DIVISIBILITY: return "p must satisfy p >= 2, p | N1 and p | N2";
    case PACO_ERR_UNSUPPORTED: return "size not supported by the library";
    case PACO_ERR_WORKSPACE: return "workspace too small";
    case PACO_ERR_ALLOC: return "allocation failed";
    case PACO_ERR_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char *paco_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace {

paco_status validate_impl(int64_t N1, int64_t N2, int64_t p, int32_t b, paco_dtype dt, bool mixed)
{
    if (dt != PACO_C64 && dt != PACO_C64_MFMA_FP16X3 && dt != PACO_C64_MFMA_BF16X3 && dt != PACO_C64_MFMA_BF16X6)
        return fail(PACO_ERR_INVALID_ARG, "unknown dtype");
    const int t = ilog2_exact(b);
    if (b < 2 || t < 1) return fail(PACO_ERR_NOT_POWER_OF_B, "b must be 2^t with t >= 1");
    const int l1 = ilog2_exact(N1), l2 = ilog2_exact(N2);
    if (mixed) {
        if (N1 < 2 || N2 < 2 || l1 < 0 || l2 < 0)
            return fail(PACO_ERR_NOT_POWER_OF_B, "mixed-radix plans need N1 and N2 powers of two >= 2");
    } else if (N1 < 2 || N2 < 2 || l1 < 0 || l2 < 0 || l1 % t || l2 % t) {
        return fail(PACO_ERR_NOT_POWER_OF_B, "N1 and N2 must be powers of b (b^m with m >= 1)");
    }
    if (p < 2 || N1 % p || N2 % p) return fail(PACO_ERR_DIVISIBILITY, "need p >= 2, p | N1, p | N2");
    if (l1 > kMaxLocalLog2 || l2 > kMaxLocalLog2 || l1 + l2 > kMaxTotalLog2)
        return fail(PACO_ERR_UNSUPPORTED, "the library supports N1, N2 <= 2^16 and N1*N2 <= 2^28");
    if (N1 / p < 16 || N2 / p < 16)
        g_last_error = "note: slab width N1/p or N2/p below 16 items (one 128-byte line)";
    else
        g_last_error.clear();
    return PACO_OK;
}

}  // namespace

extern "C" {

paco_status paco_plan_validate(int64_t N1, int64_t N2, int64_t p, int32_t b, paco_dtype dt)
{
    return validate_impl(N1, N2, p, b, dt, false);
}

paco_status paco_plan_validate_mixed(int64_t N1, int64_t N2, int64_t p, int32_t b, paco_dtype dt)
{
    return validate_impl(N1, N2, p, b, dt, true);
}

}  // extern "C"

namespace {

// Digit-aligned split of a local transform of 2^l = b^m 2^s items into
// on-chip passes: one pass up to 2^12 items, otherwise two passes n1 * n2
// with n1 = b^k 2^s and n2 = b^(m-k) (the short digit of a mixed-radix
// length goes with n1, whose digit maps carry it), k chosen so that the two
// lengths are as close as the digits allow (section 4.1's balanced split;
// for s = 0, n1 = b^ceil(m/2)).  la = 0 when no split fits two passes.
void split_local(int l, int t, int &la, int &lb)
{
    if (l <= paco::kMaxOnChipLog2) {
        la = l;
        lb = 0;
        return;
    }
    const int m = l / t, s = l % t;
    la = 0;
    for (int k = 0; k <= m; ++k) {
        const int a = k * t + s, c = l - a;
        if (a < 1 || c < 1 || a > paco::kMaxOnChipLog2 || c > paco::kMaxOnChipLog2) continue;
        const int d = a > c ? a - c : c - a, dbest = la > l - la ? 2 * la - l : l - 2 * la;
        if (la == 0 || d < dbest || (d == dbest && a > la)) la = a;
    }
    if (la == 0) la = l;  // no two-pass split: rejected by the caller
    lb = l - la;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// Builds the passes and tables of one factorisation N1 x N2 (the forward
// transform's; paco_plan_create builds a second, N2 x N1, for the inverse).
paco_status create_impl(paco_plan **plan, int64_t N1, int64_t N2, int64_t p, int32_t b, paco_dtype dt,
                        const paco_plan_options &opt)
{
    if (!plan) return fail(PACO_ERR_INVALID_ARG, "plan out-pointer is NULL");
    *plan = nullptr;
    const bool mixed = (opt.flags & PACO_PLAN_MIXED) != 0;
    const bool paper_layout = (opt.flags & PACO_PLAN_PAPER_LAYOUT) != 0;
    const bool generic = (opt.flags & PACO_PLAN_GENERIC) != 0;
    const bool no_split = (opt.flags & PACO_PLAN_NO_SPLIT) != 0;
    const bool no_sym = (opt.flags & PACO_PLAN_NO_SYM) != 0;
    paco_status st = validate_impl(N1, N2, p, b, dt, mixed);
    if (st != PACO_OK) return st;

    paco_plan_s *P = new (std::nothrow) paco_plan_s();
    if (!P) return fail(PACO_ERR_ALLOC, "host allocation failed");
    P->N1 = N1;
    P->N2 = N2;
    P->p = p;
    P->b = b;
    P->dt = dt;
    P->t = ilog2_exact(b);
    P->l1 = ilog2_exact(N1);
    P->l2 = ilog2_exact(N2);
    P->m1 = P->l1 / P->t;
    P->m2 = P->l2 / P->t;
    P->s1 = P->l1 % P->t;
    P->s2 = P->l2 % P->t;
    P->mixed = mixed;
    P->lN = P->l1 + P->l2;
    P->lL = P->l1 > P->l2 ? P->l1 : P->l2;
    P->lLo = paco::middle_log2lo(P->lN);

    int a1, b1, a3, b3;
    split_local(P->l1, P->t, a1, b1);
    split_local(P->l2, P->t, a3, b3);
    if (a1 > paco::kMaxOnChipLog2 || b1 > paco::kMaxOnChipLog2 || a3 > paco::kMaxOnChipLog2 ||
        b3 > paco::kMaxOnChipLog2) {
        delete P;
        return fail(PACO_ERR_UNSUPPORTED, "local transform needs more than two on-chip passes");
    }

    // ---- host tables (FP64-generated, rounded once to FP32) ----------------
    const int64_t L = int64_t(1) << P->lL;
    std::vector<float2> tw(L), thi, tlo, ttile, stw, tcw, tsj;
    std::vector<float> tw16;
    for (int64_t r = 0; r < L; ++r) tw[r] = paco::root_neg(r, L);
    // the two-pass form's column factor w_{16 N1}^{-k} (single-pass Phase III
    // over at most 2^12 columns: a table of at most 512 KiB)
    const bool two_pass_tables = dt == PACO_C64 && P->l2 <= paco::kMaxOnChipLog2 && P->l1 <= 12;
    if (two_pass_tables) {
        tcw.resize(size_t(16 * N1));
        for (int64_t k = 0; k < 16 * N1; ++k) tcw[k] = paco::root_neg(k, 16 * N1);
    }
    paco::middle_tables(P->lN, thi, tlo, ttile);
    // the symmetric split form (N1 = 16 L1, N2 = 16 L2; option
    // PACO_PLAN_NO_SYM): square shapes with L = 256 and 512 for every dtype,
    // 1024 in FP32; in FP32 also every non-square pair of N1, N2 in {2^12,
    // 2^13, 2^14} (N1 N2 <= 2^28 by validation), and the wide form N2 = 2^15
    // = 32 L2 (L2 = 1024) with N1 = 2^12 or 2^13
    const auto sym_side = [](int l) { return l >= paco::kSymLog2N && l <= paco::kSymLog2N + 2; };
    const bool sym_square = P->l1 == P->l2 && (P->l1 == paco::kSymLog2N || P->l1 == 13 || (dt == PACO_C64 && P->l1 == 14));
    const bool sym_rect = dt == PACO_C64 && P->l1 != P->l2 && sym_side(P->l1) && sym_side(P->l2);
    const bool sym_wide = dt == PACO_C64 && P->l2 == 15 && (P->l1 == 12 || P->l1 == 13);
    const bool sym_form = !no_split && !no_sym && !paper_layout && !generic && (sym_square || sym_rect || sym_wide);
    if (sym_form) {  // its pass-2 factor w_{16 N2}^{-s j}, s < 16, j < N2 / 16 (jc < L2 <= N2 / 16)
        const int64_t L2 = N2 / 16;
        tsj.resize(size_t(16 * L2));
        for (int64_t sv = 0; sv < 16; ++sv)
            for (int64_t jc = 0; jc < L2; ++jc) tsj[sv * L2 + jc] = paco::root_neg((sv * jc) % (16 * N2), 16 * N2);
        if (dt != PACO_C64) {  // the MFMA lanes' DFT-matrix operands
            tw16.resize(64 * 16);
            paco::w16_operands(tw16.data());
        }
    }
    int64_t stw_off[paco::kMaxOnChipLog2 + 1];
    if (!paco::stage_tables(stw, stw_off)) {
        delete P;
        return fail(PACO_ERR_INVALID_ARG, "internal: stage twiddle layout mismatch");
    }

    // one device allocation, 256-byte aligned pieces
    struct Piece { const void *src; size_t bytes; size_t off; };
    std::vector<Piece> pieces = {{tw.data(), tw.size() * 8, 0},       {thi.data(), thi.size() * 8, 0},
                                 {tlo.data(), tlo.size() * 8, 0},     {ttile.data(), ttile.size() * 8, 0},
                                 {stw.data(), stw.size() * 8, 0},     {tcw.data(), tcw.size() * 8, 0},
                                 {tsj.data(), tsj.size() * 8, 0},     {tw16.data(), tw16.size() * 4, 0}};
    size_t total = 0;
    for (auto &pc : pieces) {
        pc.off = total;
        total += (pc.bytes + 255) & ~size_t(255);
    }
    hipError_t e = hipGetDevice(&P->device);
    if (e != hipSuccess) { delete P; return hip_fail(e, "hipGetDevice"); }
    e = paco::local_fft_prepare();
    if (e == hipSuccess) e = paco::split_prepare();
    if (e != hipSuccess) { delete P; return hip_fail(e, "hipFuncSetAttribute"); }
    // set-up of paco_execute_noalloc: this device's scratch array (a plan that
    // cannot have it still works through the other entry points)
    P->scratch = scratch_for_device(P->device, P->scratch_error);
    e = hipMalloc(&P->dev_tables, total);
    if (e != hipSuccess) { P->dev_tables = nullptr; delete P; return fail(PACO_ERR_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e)); }
    std::vector<unsigned char> staging(total, 0);
    for (auto &pc : pieces)
        if (pc.bytes) std::memcpy(staging.data() + pc.off, pc.src, pc.bytes);
    e = hipMemcpy(P->dev_tables, staging.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) { (void)hipFree(P->dev_tables); delete P; return hip_fail(e, "hipMemcpy"); }
    auto at = [&](int i) { return static_cast<unsigned char *>(P->dev_tables) + pieces[i].off; };
    const float2 *d_tw = reinterpret_cast<const float2 *>(at(0));
    const float2 *d_thi = reinterpret_cast<const float2 *>(at(1));
    const float2 *d_tlo = reinterpret_cast<const float2 *>(at(2));
    const float2 *d_ttile = reinterpret_cast<const float2 *>(at(3));
    const float2 *d_stw = reinterpret_cast<const float2 *>(at(4));
    const float2 *d_tcw = reinterpret_cast<const float2 *>(at(5));
    const float2 *d_tsj = reinterpret_cast<const float2 *>(at(6));
    const float *d_tw16 = reinterpret_cast<const float *>(at(7));

    auto base_pass = [&](int64_t ld, int64_t ncols, int log2n) {
        LocalPass q{};
        q.ld = ld;
        q.ncols = ncols;
        q.log2n = log2n;
        q.log2T = paco::choose_log2T(log2n, ncols);
        q.no_fast = generic ? 1 : 0;
        q.groups = 1;
        // option: columns per workgroup for long single-group transforms
        if (opt.cols_long > 0 && log2n >= 10 && opt.cols_long <= ncols) q.log2T = ilog2_exact(opt.cols_long);
        q.prec = int32_t(dt);  // paco_dtype values are the butterfly arithmetic codes
        q.stw = d_stw + stw_off[log2n];
        q.tw = d_tw;
        q.log2L = P->lL;
        q.n_outer = 1;
        return q;
    };
    const int t = P->t;

    // ---- Phase I: A_{m1} (x) I_{N2}, output layout (Lemma 1) -------------
    if (b1 == 0) {
        LocalPass q = base_pass(N2, N2, a1);
        q.j_in = 1;
        q.k_out = 1;
        q.out_t = t;                        // logical k1 -> row pi_{m1}^-1(k1)
        q.out_ell = P->m1;
        q.out_s = P->s1;
        P->phase1.push_back(q);
    } else {
        // first child: length n1 = 2^a1 over j1 (row stride n2), batch j2;
        // its frequency k1 lands at physical row field pi(k1)
        const int64_t n2 = int64_t(1) << b1;
        LocalPass A = base_pass(N2, N2, a1);
        A.n_outer = n2;
        A.o_in = 1;
        A.j_in = n2;
        A.o_out = 1;
        A.k_out = n2;
        A.out_t = t;
        A.out_ell = a1 / t;                 // n1 = b^(a1/t) 2^s1 carries the short digit
        A.out_s = P->s1;
        // second child: length n2 over j2 for each physical a, twiddle
        // w_{N1}^{-pi(a) j2} from the represented k1 = pi(a) (appendix A.2)
        LocalPass B = base_pass(N2, N2, b1);
        B.n_outer = int64_t(1) << a1;
        B.o_in = n2;
        B.j_in = 1;
        B.o_out = n2;
        B.k_out = 1;
        B.out_t = t;
        B.out_ell = b1 / t;
        B.pre_tw = 1;
        B.log2M = P->l1;
        B.tw_t = t;
        B.tw_ell = a1 / t;
        B.tw_s = P->s1;
        P->phase1.push_back(A);
        P->phase1.push_back(B);
    }
    // ---- Phase III: B_{m2} (x) I_{N1}, input layout ----------------------
    if (b3 == 0) {
        LocalPass q = base_pass(N1, N1, a3);
        q.j_in = 1;
        q.k_out = 1;
        q.in_t = t;                         // logical j2 read from row pi_{m2}(j2)
        q.in_ell = P->m2;
        q.in_s = P->s2;
        P->phase3.push_back(q);
    } else {
        // logical j = j1*s2 + j2 sits at row pi(j2)*s1 + pi(j1)
        const int64_t s1 = int64_t(1) << a3;
        LocalPass A = base_pass(N1, N1, a3);
        A.n_outer = int64_t(1) << b3;
        A.o_in = s1;
        A.j_in = 1;
        A.in_t = t;
        A.in_ell = a3 / t;                  // s1 = b^(a3/t) 2^s2 carries the short digit
        A.in_s = P->s2;
        A.o_out = s1;
        A.k_out = 1;
        LocalPass B = base_pass(N1, N1, b3);
        B.n_outer = s1;
        B.o_in = 1;
        B.j_in = s1;
        B.in_t = t;
        B.in_ell = b3 / t;
        B.pre_tw = 1;
        B.log2M = P->l2;
        B.o_out = 1;
        B.k_out = s1;
        P->phase3.push_back(A);
        P->phase3.push_back(B);
    }
    // Column groups for n >= 2^10 (options groups1 / groups3):
    // 1 = one LDS group of T columns; 2 = two groups of T/2 (half the LDS, two
    // workgroups per CU); 3 = two groups of T, a tile twice as wide (512
    // threads with 64 items each).
    auto pick = [](LocalPass &q, int32_t want, int dflt) {
        int g = want > 0 ? want : dflt;
        if (g < 1 || g > 3 || q.log2n < 10 || q.log2T < 1 || q.no_fast) g = 1;
        // split MFMA forms: no wide tile; 16^s-point passes use the one-group
        // kernel that keeps the MFMA operand layout throughout
        if (q.prec != 0 && !q.no_fast) g = q.log2n % 4 == 0 ? 1 : (g == 3 ? 2 : g);
        if (g == 3) {
            if ((int64_t(1) << (q.log2T + 1)) > q.ncols) g = 2;
            else q.log2T += 1;  // twice as many columns per tile
        }
        q.groups = g;
        if (g > 1 && paco::local_fft_fast_mode(q) < 0) {  // not a fast pass: plain tile
            if (g == 3) q.log2T -= 1;
            q.groups = 1;
        }
    };
    const LocalPass phase1_base = P->phase1[0];
    for (auto &q : P->phase1) pick(q, opt.groups1, q.log2n >= 12 ? 2 : 1);
    const LocalPass phase3_base = P->phase3[0];
    for (auto &q : P->phase3) pick(q, opt.groups3, q.log2n >= 12 ? 3 : 1);
    // generic passes of the split MFMA forms: at most 512 threads per tile
    for (auto *ph : {&P->phase1, &P->phase3})
        for (auto &q : *ph)
            while (q.log2T > 0 && (q.no_fast || paco::local_fft_fast_mode(q) < 0) &&
                   paco::local_fft_geometry(q).threads > paco::generic_max_threads(q.prec))
                --q.log2T;
    // ---- fused pipeline: Phase I writes the packed slab transposed --------
    {
        const bool want = !paper_layout;
        LocalPass q = phase1_base;
        q.out_tr = 1;
        q.out_t = 0;
        q.out_ell = 0;
        q.out_s = 0;
        pick(q, opt.groups1, q.log2n >= 12 ? 2 : 1);
        if (q.prec != 0 && q.log2n >= 4 && q.log2n % 4 == 0)  // the operand-layout tile's own width
            q.log2T = paco::mf_log2T(q.log2n, 2);
        if (want && b1 == 0 && N1 >= paco::kMidTile && N2 >= paco::kMidTile && !q.no_fast &&
            paco::local_fft_fast_mode(q) == 2) {
            P->fused = true;
            P->phase1_packed = q;
        }
    }
    // ---- two-pass form: Phase III reads the packed buffer in natural row
    // order and applies the top-level twiddle on load (no Phase-II pass) ----
    if (P->fused && b3 == 0 && two_pass_tables) {
        LocalPass q = phase3_base;
        q.in_t = 0;
        q.in_ell = 0;
        q.in_s = 0;
        q.top_tw = 1;
        q.top_log2N = P->lN;
        q.top_log2Lo = P->lLo;
        q.top_hi = d_thi;
        q.top_lo = d_tlo;
        q.top_cw = d_tcw;
        pick(q, opt.groups3, q.log2n >= 12 ? 3 : 1);
        if (!q.no_fast && paco::local_fft_fast_mode(q) == 3) {
            P->two_pass = true;
            P->phase3_two = q;
            // its Phase I: the packed pass, reading x for the last time
            P->phase1_two = P->phase1_packed;
            P->phase1_two.src_last = 1;
            if (paco::local_fft_fast_mode(P->phase1_two) != 4) P->phase1_two = P->phase1_packed;
        }
    }
    for (auto *ph : {&P->phase1, &P->phase3})
        for (const auto &q : *ph)
            if (paco::local_fft_geometry(q).lds_bytes > 160 * 1024 || paco::local_fft_geometry(q).threads > 1024) {
                (void)hipFree(P->dev_tables);
                delete P;
                return fail(PACO_ERR_UNSUPPORTED, "local FFT tile does not fit one workgroup");
            }
    // ---- Phase II ---------------------------------------------------------
    P->mid.N1 = N1;
    P->mid.N2 = N2;
    P->mid.t = t;
    P->mid.m1 = P->m1;
    P->mid.m2 = P->m2;
    P->mid.s1 = P->s1;
    P->mid.s2 = P->s2;
    P->mid.tw_hi = d_thi;
    P->mid.tw_lo = d_tlo;
    P->mid.tw_tile = d_ttile;
    P->mid.log2N = P->lN;
    P->mid.log2Lo = P->lLo;
    P->mid.twiddle = 1;

    // ---- split form (FP32, N1 = 2^12 .. 2^14; option PACO_PLAN_NO_SPLIT) ----
    // Measured per transform (MI355X): with plain stores in both forms,
    // N2 = 2^10 49 against 60 us for the packed form, 2^12 183 against
    // 197 us, 2^13 421 against 438 us, 2^14 944 against 926 us; with the
    // streaming stores of the buffer between the first two passes, 2^14
    // 914 against 922 us (b = 4) and 947 against 953 us (b = 2).  Larger N2
    // (up to 2^16) was not measured: N2 <= 2^14.
    {
        const bool want = !no_split && !paper_layout && !generic;
        // N1 = 2^13, 2^14: Phase I takes two on-chip passes there, so the split
        // form also saves one HBM pass (pass 2 runs its M-point transforms in
        // three stages; see split.hip)
        const bool n4096 = P->fused && P->l1 == paco::kSplitLog2N1 && P->l2 <= 14;
        const bool nlong = (P->l1 == 13 || P->l1 == 14) && N2 >= 64;
        if (want && dt == PACO_C64 && (n4096 || nlong) && N2 % 16 == 0 && P->lN <= 32) {
            paco::SplitPass &q = P->split_pass;
            q.N1 = N1;
            q.N2 = N2;
            q.tw = d_tw;
            q.tw_shift = P->lL - P->l1;
            q.tw_hi = d_thi;
            q.tw_lo = d_tlo;
            q.log2N = P->lN;
            q.log2Lo = P->lLo;
            q.t = t;
            q.m2 = P->m2;
            q.s2 = P->s2;
            P->split = true;
        }
    }

    // ---- symmetric split form (N1 = N2 = 16 L; option PACO_PLAN_NO_SYM)
    // Phase III split like Phase I, its 16-point child moved into the
    // redistribution pass: every pass moves whole 128-byte lines
    if (sym_form) {
        paco::SymPass &q = P->sym_pass;
        q.N1 = N1;
        q.N2 = N2;
        q.tw = d_tw;
        q.log2L = P->lL;
        q.tw_hi = d_thi;
        q.tw_lo = d_tlo;
        q.log2N = P->lN;
        q.log2Lo = P->lLo;
        q.tw_sj = d_tsj;
        q.w16 = d_tw16;
        // passes 1 and 3 at L >= 512: one workgroup per resident slot
        q.resident1 = dt == PACO_C64 ? paco::sym_resident_groups(1, q) : paco::sym_mf_resident_groups(int(dt), 1, q);
        q.resident3 = dt == PACO_C64 ? paco::sym_resident_groups(3, q) : paco::sym_mf_resident_groups(int(dt), 3, q);
        q.resident2 = dt == PACO_C64 ? paco::sym_resident_groups(2, q) : 0;
        P->sym = true;
    }

    char buf[512];
    std::string desc;
    for (auto *ph : {&P->phase1, &P->phase3}) {
        desc += ph == &P->phase1 ? "phase1[" : " phase2[tile64x64] phase3[";
        for (const auto &q : *ph) {
            const paco::LocalLaunch g = paco::local_fft_geometry(q);
            std::snprintf(buf, sizeof buf, " n=2^%d T=%d%s outer=%lld wg=%lld thr=%d lds=%zu", q.log2n, 1 << q.log2T,
                          (!q.no_fast && paco::local_fft_fast_mode(q) >= 0) ? "(fast)" : "", (long long)q.n_outer,
                          (long long)g.tiles, g.threads, g.lds_bytes);
            desc += buf;
        }
        desc += " ]";
    }
    if (P->split) {
        std::snprintf(buf, sizeof buf,
                      "split[pass1: phase1 radix-16 stage over 128-byte row runs -> ws; pass2: %lld-point tails + "
                      "row unpack+twiddle] ",
                      (long long)(N1 / 16));
        desc = buf + desc;
    }
    if (P->fused) desc = "fused[phase1 -> packed transposed slab, phase2 row unpack+twiddle] " + desc;
    if (P->sym) {
        const int64_t r2 = sym_wide ? 32 : 16;
        std::snprintf(buf, sizeof buf,
                      "sym[pass1: phase1 %lld-point children over rows 16j+r -> ws; pass2: phase1 radix-16 + twiddle + "
                      "phase3 radix-%lld; pass3: phase3 %lld-point children, in place] ",
                      (long long)(N1 / 16), (long long)r2, (long long)(N2 / r2));
        desc = buf + desc;
    }
    if (P->two_pass) {
        const paco::LocalLaunch g = paco::local_fft_geometry(P->phase3_two);
        std::snprintf(buf, sizeof buf, " two_pass[phase3 twiddle-on-load n=2^%d T=%d wg=%lld thr=%d lds=%zu]",
                      P->phase3_two.log2n, 1 << P->phase3_two.log2T, (long long)g.tiles, g.threads, g.lds_bytes);
        desc += buf;
    }
    if (P->s1 || P->s2) {
        std::snprintf(buf, sizeof buf, " mixed-radix[N1=%lld^%d*2^%d N2=%lld^%d*2^%d]", (long long)b, P->m1, P->s1,
                      (long long)b, P->m2, P->s2);
        desc += buf;
    }
    static const char *kPrecName[] = {"fp32", "fp16x3", "bf16x3", "bf16x6"};
    desc += std::string(" prec=") + kPrecName[int(dt)];
    P->desc = desc;
    if (const char *lg = std::getenv("PACO_LOG"))  // plan summary on stderr
        if (lg[0] == '1')
            std::fprintf(stderr, "paco plan N1=%lld N2=%lld p=%lld b=%d: %s\n", (long long)N1, (long long)N2,
                         (long long)p, b, desc.c_str());
    *plan = P;
    return PACO_OK;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

paco_status create_with_inverse(paco_plan **plan, int64_t N1, int64_t N2, int64_t p, int32_t b, paco_dtype dt,
                                const paco_plan_options &opt)
{
    if (plan) *plan = nullptr;
    if (opt.flags & ~(PACO_PLAN_MIXED | PACO_PLAN_PAPER_LAYOUT | PACO_PLAN_NO_SPLIT | PACO_PLAN_GENERIC | PACO_PLAN_NO_SYM))
        return fail(PACO_ERR_INVALID_ARG, "unknown plan option flag");
    if (opt.groups1 < 0 || opt.groups1 > 3 || opt.groups3 < 0 || opt.groups3 > 3)
        return fail(PACO_ERR_INVALID_ARG, "groups1 / groups3 must be 0 (default), 1, 2 or 3");
    if (opt.cols_long < 0 || (opt.cols_long > 0 && ilog2_exact(opt.cols_long) < 0))
        return fail(PACO_ERR_INVALID_ARG, "cols_long must be 0 (default) or a power of two");
    paco_status st = create_impl(plan, N1, N2, p, b, dt, opt);
    if (st != PACO_OK || N1 == N2) return st;  // square: the inverse reuses the forward passes
    const std::string note = g_last_error;
    paco_plan *inv = nullptr;
    st = create_impl(&inv, N2, N1, p, b, dt, opt);
    if (st != PACO_OK) {
        // the forward plan stands; paco_execute_inverse reports the reason
        (*plan)->inv_error = "inverse (N2 x N1 passes) unavailable: " + g_last_error;
        g_last_error = note;
        return PACO_OK;
    }
    (*plan)->inv = inv;
    g_last_error = note;
    return PACO_OK;
}

}  // namespace

extern "C" {

paco_status paco_plan_create(paco_plan **plan, int64_t N1, int64_t N2, int64_t p, int32_t b,
                             paco_dtype dt)
{
    return create_with_inverse(plan, N1, N2, p, b, dt, paco_plan_options{});
}

paco_status paco_plan_create_mixed(paco_plan **plan, int64_t N1, int64_t N2, int64_t p, int32_t b,
                                   paco_dtype dt)
{
    paco_plan_options o{};
    o.flags = PACO_PLAN_MIXED;
    return create_with_inverse(plan, N1, N2, p, b, dt, o);
}

paco_status paco_plan_create_ex(paco_plan **plan, int64_t N1, int64_t N2, int64_t p, int32_t b, paco_dtype dt,
                                const paco_plan_options *options)
{
    return create_with_inverse(plan, N1, N2, p, b, dt, options ? *options : paco_plan_options{});
}

paco_status paco_plan_workspace_size(const paco_plan *plan, size_t *bytes)
{
    if (!bytes) return fail(PACO_ERR_INVALID_ARG, "bytes out-pointer is NULL");
    *bytes = 0;
    if (!plan) return fail(PACO_ERR_INVALID_ARG, "plan is NULL");
    *bytes = size_t(plan->N1) * size_t(plan->N2) * 8;
    return PACO_OK;
}

paco_status paco_plan_describe(const paco_plan *plan, int32_t *launches, char *buf, size_t buflen)
{
    if (!plan) return fail(PACO_ERR_INVALID_ARG, "plan is NULL");
    if (launches)  // the split form runs its two passes in place of Phase I's passes and Phase II
        *launches = plan->sym ? 3 : int32_t((plan->split ? 2 : plan->phase1.size() + 1) + plan->phase3.size());
    if (buf && buflen) {
        std::strncpy(buf, plan->desc.c_str(), buflen - 1);
        buf[buflen - 1] = 0;
    }
    return PACO_OK;
}

paco_status paco_plan_destroy(paco_plan *plan)
{
    if (!plan) return PACO_OK;
    if (plan->inv) paco_plan_destroy(plan->inv);
    if (plan->dev_tables) (void)hipFree(plan->dev_tables);
    delete plan;
    return PACO_OK;
}

}  // extern "C"

namespace {

bool bad_ptr(const void *p) { return !p || (reinterpret_cast<uintptr_t>(p) & 15); }

paco_status run_local(const std::vector<LocalPass> &passes, const void *src, void *dst, hipStream_t s)
{
    for (size_t i = 0; i < passes.size(); ++i) {
        LocalPass q = passes[i];
        q.src = static_cast<const float2 *>(i == 0 ? src : dst);
        q.dst = static_cast<float2 *>(dst);
        hipError_t e = paco::launch_local_fft(q, s);
        if (e != hipSuccess) return hip_fail(e, "local FFT launch");
    }
    return PACO_OK;
}

paco_status run_middle(const paco_plan *plan, const void *src, void *dst, int twiddle, bool packed, hipStream_t s)
{
    MiddlePass m = plan->mid;
    m.ws = static_cast<const float2 *>(src);
    m.out = static_cast<float2 *>(dst);
    m.twiddle = twiddle;
    m.packed = packed ? 1 : 0;
    hipError_t e = paco::launch_middle(m, s);
    if (e != hipSuccess) return hip_fail(e, "phase II launch");
    return PACO_OK;
}

paco_status check_buffers(const paco_plan *plan, const void *in, void *out, void *workspace, size_t workspace_bytes)
{
    if (!plan) return fail(PACO_ERR_INVALID_ARG, "plan is NULL");
    if (bad_ptr(in) || bad_ptr(out) || bad_ptr(workspace))
        return fail(PACO_ERR_INVALID_ARG, "in/out/workspace must be non-NULL and 16-byte aligned");
    const size_t need = size_t(plan->N1) * size_t(plan->N2) * 8;
    if (workspace_bytes < need) return fail(PACO_ERR_WORKSPACE, "workspace smaller than N1*N2*8 bytes");
    const size_t wb = reinterpret_cast<uintptr_t>(workspace), ib = reinterpret_cast<uintptr_t>(in),
                 ob = reinterpret_cast<uintptr_t>(out);
    if ((wb < ib + need && ib < wb + need) || (wb < ob + need && ob < wb + need))
        return fail(PACO_ERR_INVALID_ARG, "workspace overlaps in or out");
    return PACO_OK;
}

// Pass 1 (pass == 1) or pass 2 of the split form.
paco_status run_split(const paco_plan *plan, int pass, const void *src, void *dst, bool conj_in, hipStream_t s)
{
    paco::SplitPass q = plan->split_pass;
    q.src = static_cast<const float2 *>(src);
    q.dst = static_cast<float2 *>(dst);
    q.conj_in = conj_in ? 1 : 0;
    hipError_t e = pass == 1 ? paco::launch_split_first(q, s) : paco::launch_split_middle(q, s);
    if (e != hipSuccess) return hip_fail(e, pass == 1 ? "split pass 1 launch" : "split pass 2 launch");
    return PACO_OK;
}

// Pass 1, 2 or 3 of the symmetric split form.
paco_status run_sym(const paco_plan *plan, int pass, const void *src, void *dst, bool inverse, hipStream_t s)
{
    paco::SymPass q = plan->sym_pass;
    q.src = static_cast<const float2 *>(src);
    q.dst = static_cast<float2 *>(dst);
    q.conj_in = inverse && pass == 1 ? 1 : 0;
    q.out_scale = inverse && pass == 3 ? 1.0f / float(plan->N1 * plan->N2) : 0.f;  // 2^-log2 N: exact
    hipError_t e = plan->dt != PACO_C64 ? paco::launch_sym_mf(int(plan->dt), pass, q, s)
                   : pass == 1          ? paco::launch_sym_first(q, s)
                   : pass == 2          ? paco::launch_sym_middle(q, s)
                                        : paco::launch_sym_last(q, s);
    if (e != hipSuccess) return hip_fail(e, "symmetric split pass launch");
    return PACO_OK;
}

// The three phases of one plan.  inverse: conj on Phase I's loads, conj and
// 1/N on Phase III's stores, i.e. conj(Omega conj(in)) / N.
paco_status run_three(const paco_plan *plan, const void *in, void *out, void *workspace, hipStream_t s, bool inverse)
{
    if (plan->sym) {
        paco_status st = run_sym(plan, 1, in, workspace, inverse, s);
        if (st == PACO_OK) st = run_sym(plan, 2, workspace, out, inverse, s);
        if (st == PACO_OK) st = run_sym(plan, 3, out, out, inverse, s);
        return st;
    }
    std::vector<LocalPass> p1 = plan->fused ? std::vector<LocalPass>{plan->phase1_packed} : plan->phase1;
    std::vector<LocalPass> p3 = plan->phase3;
    if (inverse) {
        p1.front().conj_in = 1;
        p3.back().out_scale = 1.0f / float(plan->N1 * plan->N2);  // 2^-log2 N: exact
    }
    paco_status st;
    if (plan->split) {
        st = run_split(plan, 1, in, workspace, inverse, s);
        if (st != PACO_OK) return st;
        st = run_split(plan, 2, workspace, out, false, s);
    } else {
        st = run_local(p1, in, workspace, s);
        if (st != PACO_OK) return st;
        st = run_middle(plan, workspace, out, 1, plan->fused, s);
    }
    if (st != PACO_OK) return st;
    return run_local(p3, out, out, s);
}

}  // namespace

extern "C" {

paco_status paco_execute(const paco_plan *plan, const void *in, void *out, void *workspace,
                         size_t workspace_bytes, void *stream)
{
    paco_status st = check_buffers(plan, in, out, workspace, workspace_bytes);
    if (st != PACO_OK) return st;
    return run_three(plan, in, out, workspace, static_cast<hipStream_t>(stream), false);
}

paco_status paco_execute_noalloc(const paco_plan *plan, const void *in, void *out, void *stream)
{
    if (!plan) return fail(PACO_ERR_INVALID_ARG, "plan is NULL");
    if (plan->N1 * plan->N2 > int64_t(PACO_NOALLOC_MAX_ITEMS))
        return fail(PACO_ERR_WORKSPACE, "paco_execute_noalloc: N1*N2 above PACO_NOALLOC_MAX_ITEMS (2^22 items)");
    if (!plan->scratch) return fail(PACO_ERR_HIP, "paco_execute_noalloc: no scratch array: " + plan->scratch_error);
    paco_status st = check_buffers(plan, in, out, plan->scratch, size_t(PACO_NOALLOC_MAX_ITEMS) * 8);
    if (st != PACO_OK) return st;
    return run_three(plan, in, out, plan->scratch, static_cast<hipStream_t>(stream), false);
}

paco_status paco_execute_inverse(const paco_plan *plan, const void *in, void *out, void *workspace,
                                 size_t workspace_bytes, void *stream)
{
    paco_status st = check_buffers(plan, in, out, workspace, workspace_bytes);
    if (st != PACO_OK) return st;
    if (!plan->inv_error.empty()) return fail(PACO_ERR_UNSUPPORTED, plan->inv_error);
    return run_three(plan->inv ? plan->inv : plan, in, out, workspace, static_cast<hipStream_t>(stream), true);
}

paco_status paco_execute_two_pass(const paco_plan *plan, const void *in, void *out, void *workspace,
                                  size_t workspace_bytes, void *stream)
{
    if (!plan) return fail(PACO_ERR_INVALID_ARG, "plan is NULL");
    if (!plan->two_pass)
        return fail(PACO_ERR_UNSUPPORTED, "two-pass form needs the fused FP32 pipeline with a single-pass Phase III");
    paco_status st = check_buffers(plan, in, out, workspace, workspace_bytes);
    if (st != PACO_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = run_local({plan->phase1_two}, in, workspace, s);
    if (st != PACO_OK) return st;
    return run_local({plan->phase3_two}, workspace, out, s);
}

paco_status paco_plan_has_two_pass(const paco_plan *plan, int32_t *yes)
{
    if (!yes) return fail(PACO_ERR_INVALID_ARG, "yes out-pointer is NULL");
    *yes = 0;
    if (!plan) return fail(PACO_ERR_INVALID_ARG, "plan is NULL");
    *yes = plan->two_pass ? 1 : 0;
    return PACO_OK;
}

paco_status paco_plan_has_split(const paco_plan *plan, int32_t *yes)
{
    if (!yes) return fail(PACO_ERR_INVALID_ARG, "yes out-pointer is NULL");
    *yes = 0;
    if (!plan) return fail(PACO_ERR_INVALID_ARG, "plan is NULL");
    *yes = plan->sym ? 2 : (plan->split ? 1 : 0);
    return PACO_OK;
}

paco_status paco_execute_stage(const paco_plan *plan, int stage, int flags, const void *src, void *dst,
                               void *stream)
{
    if (!plan) return fail(PACO_ERR_INVALID_ARG, "plan is NULL");
    if (bad_ptr(src) || bad_ptr(dst)) return fail(PACO_ERR_INVALID_ARG, "src/dst must be non-NULL and 16-byte aligned");
    if (flags & ~(PACO_NO_TWIDDLE | PACO_PACKED | PACO_TWO_PASS | PACO_SPLIT))
        return fail(PACO_ERR_INVALID_ARG, "unknown flags");
    if (flags & PACO_SPLIT) {
        if (flags != PACO_SPLIT || stage < 1 || stage > (plan->sym ? 3 : 2))
            return fail(PACO_ERR_INVALID_ARG, "PACO_SPLIT applies alone to stage 1 or 2 (3 in the symmetric form)");
        if (!plan->split && !plan->sym) return fail(PACO_ERR_UNSUPPORTED, "this plan has no split form");
        const size_t need = size_t(plan->N1) * size_t(plan->N2) * 8;
        const uintptr_t a = reinterpret_cast<uintptr_t>(src), b = reinterpret_cast<uintptr_t>(dst);
        if (a < b + need && b < a + need && !(stage == 3 && a == b))
            return fail(PACO_ERR_INVALID_ARG, "split stages 1 and 2 are out of place (stage 3: in place or disjoint)");
        if (plan->sym) return run_sym(plan, stage, src, dst, false, static_cast<hipStream_t>(stream));
        return run_split(plan, stage, src, dst, false, static_cast<hipStream_t>(stream));
    }
    if ((flags & PACO_TWO_PASS) && !(stage == 1 && (flags & PACO_PACKED)))
        return fail(PACO_ERR_INVALID_ARG, "PACO_TWO_PASS applies to stage 1 with PACO_PACKED");
    if ((flags & PACO_TWO_PASS) && !plan->two_pass) return fail(PACO_ERR_UNSUPPORTED, "this plan has no two-pass form");
    const bool packed = (flags & PACO_PACKED) != 0;
    if (packed && !plan->fused) return fail(PACO_ERR_UNSUPPORTED, "this plan has no packed Phase-I buffer");
    if (packed && stage == 3 && !plan->two_pass)
        return fail(PACO_ERR_UNSUPPORTED, "this plan has no two-pass Phase III");
    if ((flags & PACO_NO_TWIDDLE) && stage != 2) return fail(PACO_ERR_INVALID_ARG, "PACO_NO_TWIDDLE applies to stage 2");
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (stage) {
    case 1: {
        if (packed && src == dst) return fail(PACO_ERR_INVALID_ARG, "packed stage 1 is out of place");
        if (flags & PACO_TWO_PASS) return run_local({plan->phase1_two}, src, dst, s);
        return packed ? run_local({plan->phase1_packed}, src, dst, s) : run_local(plan->phase1, src, dst, s);
    }
    case 2: {
        const size_t need = size_t(plan->N1) * size_t(plan->N2) * 8;
        const uintptr_t a = reinterpret_cast<uintptr_t>(src), b = reinterpret_cast<uintptr_t>(dst);
        if (a < b + need && b < a + need) return fail(PACO_ERR_INVALID_ARG, "stage 2 src and dst overlap");
        return run_middle(plan, src, dst, (flags & PACO_NO_TWIDDLE) ? 0 : 1, packed, s);
    }
    case 3: return packed ? run_local({plan->phase3_two}, src, dst, s) : run_local(plan->phase3, src, dst, s);
    default: return fail(PACO_ERR_INVALID_ARG, "stage must be 1, 2 or 3");
    }
}

}  // extern "C"
