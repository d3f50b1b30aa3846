// Batched form: many independent transforms of power-of-two sizes, each run
// through the three phases of the paper (LocalFFT in output layout, the fused
// global permutation with the top-level twiddle, LocalFFT in input layout),
// all inside ONE persistent kernel launch.
//
// Work is cut into tasks: one column tile of Phase I, one 64-row tile of
// Phase II, one column tile of Phase III of one transform ("jobs" are the
// (transform, phase) pairs), and, for transforms of at most 2^12 items, the
// whole transform in one workgroup (its three phases separated by workgroup
// barriers, the intermediates staying in L2).  A resident workgroup claims
// the next task number from an atomic ticket counter.  A Phase II task waits
// until every tile of its transform's Phase I job is done, a Phase III task
// for Phase II, on per-job completion counters: the producer writes those
// tiles with device-coherent stores, waits for them to complete and then
// increments the counter; the consumer reads the counter with a device-scope
// acquire load (which also drops stale cache lines) before touching the data.
//
// Forward progress: tickets are claimed in increasing order by workgroups
// that are already running, and a task only waits for jobs whose tasks all
// have smaller tickets.  The smallest unfinished ticket therefore never
// waits on anything unfinished, so every wait ends; each wait also gives up
// after a bounded number of polls and counts the event, so no wave can spin
// forever.  The schedule interleaves jobs so that a dependent job is usually
// emitted a couple of grid-widths of tiles after the job it waits for.
//
// The last workgroup to leave resets the ticket and completion counters, so
// the launch can be replayed (e.g. from a captured graph) without any memset.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <fstream>
#include <map>
#include <new>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "paco.h"
#include "middle_dev.h"
#include "stages.h"

namespace paco {
namespace {

constexpr int kBT = 256;             // threads per workgroup of the persistent kernel
constexpr int kBatchMinLog2 = 2;     // N >= 4 (N1, N2 >= 2)
constexpr int kBatchMaxLog2 = 20;    // local lengths <= 2^10
constexpr int kSmallMaxLog2 = 12;    // whole transform inside one workgroup
constexpr int kBigMinLocal = 6;      // Phase II tiles need N1, N2 >= 64
constexpr int kBigMaxLocal = 10;
constexpr uint32_t kSpinLimit = 1u << 22;
// s_waitcnt operand that waits for vmcnt = 0 only (gfx9 encoding: vmcnt in
// bits 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at their maxima)
constexpr int kWaitStores = 0x0F70;
// s_getreg operand of the XCC_ID hardware register (id 20), bits 3:0: the
// XCD the reading wave runs on
constexpr int kHwRegXccId = 20 | (0 << 6) | ((4 - 1) << 11);
constexpr int kMaxQueues = 16;
constexpr int kTicketStride = 64;  // counters 256 bytes apart

enum : int32_t { kSmall = 0, kP1 = 1, kP2 = 2, kP3 = 3 };

struct alignas(8) BatchJob {
    int64_t base;            // first item of the transform in in / out / workspace
    int32_t kind;            // kSmall, kP1, kP2, kP3
    int32_t l1, l2, t;       // N1 = 2^l1, N2 = 2^l2, b = 2^t
    int32_t v1, v3;          // tile variants of Phase I / Phase III
    int32_t dep, dep_tiles;  // job this one waits for (-1: none) and its tile count
    int32_t ntiles;          // tasks of this job
    int32_t tab;             // Phase-II table set of the transform size
    int32_t signal;          // 1: a later job waits for this one
    int32_t pad;
};

static_assert(sizeof(BatchJob) == 56, "job layout");

struct BatchTables {
    const float2 *hi, *lo, *tile;
    int32_t log2N, log2Lo;
};

// One task: the tile number and a copy of its job (one 64-byte scalar load).
struct BatchTask {
    BatchJob J;
    uint32_t job, tile;
};

static_assert(sizeof(BatchTask) == 64, "task layout");

struct BatchArgs {
    const float2 *in;
    float2 *out;
    float2 *ws;
    const BatchTask *tasks;
    const BatchJob *jobs;
    const BatchTables *tabs;
    const float2 *stw;
    int32_t stw_off[kMaxOnChipLog2 + 1];
    uint32_t njobs;
    uint32_t nq;           // work queues: one per XCD, or one shared queue
    const uint32_t *qbeg;  // tasks of queue q: [qbeg[q], qbeg[q + 1])
    uint32_t *tickets;     // one counter per queue, kTicketStride apart
    uint32_t *exits, *done, *errors;
    uint32_t spin_limit;   // polls before a completion wait gives up (kSpinLimit)
};

// Tile variant v of a local length 2^l: 2^(12 - l + v) columns per tile;
// v = 0 one LDS group, v = 1 two groups (16-byte accesses move both).
// Every variant runs exactly kBT threads with 16 items each.
constexpr int var_log2T(int l, int v) { return kMaxOnChipLog2 - l + v; }

// ---- Phase I / Phase III column tiles --------------------------------------
template <int L, int V, bool COH>
__device__ __forceinline__ void p1_tile(const BatchArgs &A, const BatchJob &J, uint32_t tile, float2 *smem, int tid)
{
    constexpr int LT = var_log2T(L, V), H = V ? 2 : 1, EG = 16;
    static_assert((1 << (L + LT - (H == 2 ? 1 : 0))) / EG == kBT, "tile geometry");
    fast_tile<L, 2, 1, H, EG, LT, COH>(A.in + J.base, A.ws + J.base, 1u << J.l2, int64_t(tile) << LT, A.stw + A.stw_off[L],
                                  smem, tid);
}

template <int L, int V, int TB>
__device__ __forceinline__ void p3_tile(const BatchArgs &A, const BatchJob &J, uint32_t tile, float2 *smem, int tid)
{
    constexpr int LT = var_log2T(L, V), H = V ? 2 : 1, EG = 16;
    static_assert((1 << (L + LT - (H == 2 ? 1 : 0))) / EG == kBT, "tile geometry");
    if constexpr (L % TB == 0) {
        fast_tile<L, 1, TB, H, EG, LT>(A.out + J.base, A.out + J.base, 1u << J.l1, int64_t(tile) << LT,
                                       A.stw + A.stw_off[L], smem, tid);
    }
}

template <int L, bool COH>
__device__ __forceinline__ void p1_len(const BatchArgs &A, const BatchJob &J, uint32_t tile, float2 *smem, int tid)
{
    if (J.v1 == 0) p1_tile<L, 0, COH>(A, J, tile, smem, tid);
    else p1_tile<L, 1, COH>(A, J, tile, smem, tid);
}

template <int L, int V>
__device__ __forceinline__ void p3_var(const BatchArgs &A, const BatchJob &J, uint32_t tile, float2 *smem, int tid)
{
    switch (J.t) {
    case 1: p3_tile<L, V, 1>(A, J, tile, smem, tid); break;
    case 2: p3_tile<L, V, 2>(A, J, tile, smem, tid); break;
    default: p3_tile<L, V, 4>(A, J, tile, smem, tid); break;
    }
}

template <int L>
__device__ __forceinline__ void p3_len(const BatchArgs &A, const BatchJob &J, uint32_t tile, float2 *smem, int tid)
{
    if (J.v3 == 0) p3_var<L, 0>(A, J, tile, smem, tid);
    else p3_var<L, 1>(A, J, tile, smem, tid);
}

template <bool COH>
__device__ __forceinline__ void run_p1(const BatchArgs &A, const BatchJob &J, uint32_t tile, float2 *smem, int tid)
{
    switch (J.l1) {
    case 6: p1_len<6, COH>(A, J, tile, smem, tid); break;
    case 7: p1_len<7, COH>(A, J, tile, smem, tid); break;
    case 8: p1_len<8, COH>(A, J, tile, smem, tid); break;
    case 9: p1_len<9, COH>(A, J, tile, smem, tid); break;
    default: p1_len<10, COH>(A, J, tile, smem, tid); break;
    }
}

__device__ __forceinline__ void run_p3(const BatchArgs &A, const BatchJob &J, uint32_t tile, float2 *smem, int tid)
{
    switch (J.l2) {
    case 6: p3_len<6>(A, J, tile, smem, tid); break;
    case 7: p3_len<7>(A, J, tile, smem, tid); break;
    case 8: p3_len<8>(A, J, tile, smem, tid); break;
    case 9: p3_len<9>(A, J, tile, smem, tid); break;
    default: p3_len<10>(A, J, tile, smem, tid); break;
    }
}

__device__ __forceinline__ MiddlePass middle_of(const BatchArgs &A, const BatchJob &J)
{
    const BatchTables T = A.tabs[J.tab];
    MiddlePass M;
    M.ws = A.ws + J.base;
    M.out = A.out + J.base;
    M.N1 = int64_t(1) << J.l1;
    M.N2 = int64_t(1) << J.l2;
    M.t = J.t;
    M.m1 = J.l1 / J.t;
    M.m2 = J.l2 / J.t;
    M.s1 = 0;  // the batched plans use bases that divide both exponents
    M.s2 = 0;
    M.tw_hi = T.hi;
    M.tw_lo = T.lo;
    M.tw_tile = T.tile;
    M.log2N = T.log2N;
    M.log2Lo = T.log2Lo;
    M.twiddle = 1;
    M.packed = 1;
    return M;
}

// Phase II of the fused pipeline: the same tile bodies as the single-transform
// kernels (64 rows x 128 columns when N1 >= 128, else 64 x 64).
template <bool COH>
__device__ __forceinline__ void run_p2(const BatchArgs &A, const BatchJob &J, uint32_t tile, int tid)
{
    const MiddlePass M = middle_of(A, J);
    if (J.l1 >= 7) middle_packed2_tile<false, true, COH>(M, tile, tid);
    else middle_packed_tile<false, true, COH>(M, tile, tid);
}

// ---- whole small transform in one workgroup --------------------------------
// One local phase over all columns at once: n = 2^LOG2N rows, 2^log2T
// columns, row length ld.  MODE 2: natural input rows, packed transposed
// output (Phase I); MODE 1: input row of logical j is pi(j) in base 2^in_t
// over in_ell digits, natural output rows (Phase III).
template <int LOG2N, int MODE>
__device__ __forceinline__ void small_local(const float2 *src, float2 *dst, uint32_t ld, int log2T, int in_t,
                                            int in_ell, const float2 *stw, float2 *smem, int tid)
{
    constexpr int EG = LOG2N < 4 ? (1 << LOG2N) : 16;
    constexpr int LR0 = stage_log2radix(LOG2N, 0);
    constexpr int R0 = 1 << LR0;
    constexpr int NB0 = EG / R0;
    constexpr int LNR0 = LOG2N - LR0;
    constexpr int TWN = stage_tw_total(LOG2N);
    float2 *twl = smem;
    float2 *lds = smem + ((TWN + 63) & ~63);
    const int nt = (1 << (LOG2N + log2T)) / EG;  // threads that own butterflies (<= kBT)
    const bool act = tid < nt;
    const int Tm = (1 << log2T) - 1;
    const char *s = reinterpret_cast<const char *>(src);
    const uint32_t ld8 = ld * 8u;
    float2 v[EG];
#pragma unroll
    for (int e = 0; e < EG; ++e) v[e] = make_float2(0.f, 0.f);
    if (act) {
#pragma unroll
        for (int q = 0; q < NB0; ++q) {
            const int g = tid + q * nt;
            const int t = g & Tm, j = g >> log2T;
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const uint32_t jj = uint32_t(j + (r << LNR0));
                const uint32_t row = MODE == 1 ? uint32_t(digrev<false>(jj, in_t, in_ell)) : jj;
                v[q * R0 + r] = *reinterpret_cast<const float2 *>(s + row * ld8 + uint32_t(t) * 8u);
            }
        }
    }
    copy_twiddles(twl, stw, TWN, tid, kBT);
    Ctx c;
    c.lds = lds;
    c.twl = twl;
    c.tid = tid;
    c.nt = nt;
    c.log2T = log2T;
    c.dst = reinterpret_cast<char *>(dst);
    c.ld8 = ld8;
    c.orow_out = 0;
    c.k_out = 1;
    c.out_t = 0;
    c.out_ell = 0;
    c.act = act;
    run_stage<LOG2N, 0, EG, -1, MODE, 1, false, 1>(v, c);
}

template <int MODE>
__device__ __forceinline__ void small_phase(int l, const float2 *src, float2 *dst, uint32_t ld, int log2T, int in_t,
                                            int in_ell, const BatchArgs &A, float2 *smem, int tid)
{
    switch (l) {
    case 1: small_local<1, MODE>(src, dst, ld, log2T, in_t, in_ell, A.stw + A.stw_off[1], smem, tid); break;
    case 2: small_local<2, MODE>(src, dst, ld, log2T, in_t, in_ell, A.stw + A.stw_off[2], smem, tid); break;
    case 3: small_local<3, MODE>(src, dst, ld, log2T, in_t, in_ell, A.stw + A.stw_off[3], smem, tid); break;
    case 4: small_local<4, MODE>(src, dst, ld, log2T, in_t, in_ell, A.stw + A.stw_off[4], smem, tid); break;
    case 5: small_local<5, MODE>(src, dst, ld, log2T, in_t, in_ell, A.stw + A.stw_off[5], smem, tid); break;
    default: small_local<6, MODE>(src, dst, ld, log2T, in_t, in_ell, A.stw + A.stw_off[6], smem, tid); break;
    }
}

__device__ __forceinline__ void run_small(const BatchArgs &A, const BatchJob &J, float2 *smem, int tid)
{
    const float2 *x = A.in + J.base;
    float2 *w = A.ws + J.base;
    float2 *y = A.out + J.base;
    const int l1 = J.l1, l2 = J.l2, lN = l1 + l2;
    // Phase I: N1-point DFTs of the N2 columns, packed slab written transposed
    small_phase<2>(l1, x, w, 1u << l2, l2, 0, 0, A, smem, tid);
    __syncthreads();
    // Phase II: row c -> pi_{m2}(c), item v scaled by w_N^{-v c}
    const BatchTables T = A.tabs[J.tab];
    const uint32_t N = 1u << lN, n1m = (1u << l1) - 1, lom = (1u << T.log2Lo) - 1;
    for (uint32_t e = tid; e < N; e += kBT) {
        const uint32_t c = e >> l1, v = e & n1m;
        const uint32_t u = uint32_t(digrev<false>(c, J.t, l2 / J.t));
        const uint32_t r = (v * c) & (N - 1);
        y[(u << l1) + v] = cmul(w[e], cmul(T.hi[r >> T.log2Lo], T.lo[r & lom]));
    }
    __syncthreads();
    // Phase III: N2-point DFTs of the N1 columns, input rows pi_{m2}, in place
    small_phase<1>(l2, y, y, 1u << l1, l1, J.t, l2 / J.t, A, smem, tid);
}

// Polls with relaxed loads (an acquire load also drops this XCD's cached
// lines, which would slow every other workgroup on it while one waits), then
// one device-scope acquire fence once the count is reached.
__device__ __forceinline__ void wait_for(const BatchArgs &A, int32_t dep, uint32_t need)
{
    uint32_t spins = 0;
    while (__hip_atomic_load(A.done + dep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        __builtin_amdgcn_s_sleep(8);
        if (++spins >= A.spin_limit) {
            atomicAdd(A.errors, 1u);
            break;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// COH = false: one work queue per XCD.  A workgroup serves the queue of the
// XCD it runs on (read from the hardware), and every task of a transform sits
// in one queue, so producer and consumer tiles share that XCD's L2: ordinary
// stores, completed (vmcnt 0) before the counter moves, are what the
// consumer reads after its acquire fence (which drops stale L1 lines).
// COH = true: one queue shared by all XCDs; the tiles other tasks read are
// written with device-coherent stores instead.
template <bool COH>
__global__ __launch_bounds__(kBT) void batch_kernel(BatchArgs A)
{
    extern __shared__ float2 smem[];
    __shared__ uint32_t s_ticket;
    __shared__ int s_last;
    const int tid = threadIdx.x;
    const uint32_t q = COH ? 0u : uint32_t(__builtin_amdgcn_s_getreg(kHwRegXccId)) % A.nq;
    uint32_t *ticket = A.tickets + q * kTicketStride;
    const uint32_t beg = A.qbeg[q], end = A.qbeg[q + 1];
    if (tid == 0) s_ticket = beg + atomicAdd(ticket, 1u);
    __syncthreads();
    uint32_t tk = __builtin_amdgcn_readfirstlane(s_ticket);
    for (;;) {
        if (tk >= end) break;
        const BatchTask task = A.tasks[tk];
        const BatchJob &J = task.J;
        // the next ticket is claimed now and read after the task, so the
        // atomic's round trip overlaps the work
        uint32_t next = 0;
        if (tid == 0) next = beg + atomicAdd(ticket, 1u);
        if (J.dep >= 0) {
            if (tid == 0) wait_for(A, J.dep, uint32_t(J.dep_tiles));
            __syncthreads();
        }
        // The thread id goes through an empty asm in every iteration: the
        // compiler then cannot hoist the per-thread address arithmetic of all
        // task variants out of the loop, which would keep every variant's
        // values live at once.
        int ltid = tid;
        __asm__ volatile("" : "+v"(ltid));
        switch (J.kind) {
        case kP1: run_p1<COH>(A, J, task.tile, smem, ltid); break;
        case kP2: run_p2<COH>(A, J, task.tile, ltid); break;
        case kP3: run_p3(A, J, task.tile, smem, ltid); break;
        default: run_small(A, J, smem, ltid); break;
        }
        // Completion: once every wave has seen its stores complete (vmcnt 0)
        // a relaxed device-scope increment publishes the tile (the ordering a
        // release gives, without writing back the whole L2 of the XCD).
        if (J.signal) __builtin_amdgcn_s_waitcnt(kWaitStores);
        if (tid == 0) s_ticket = next;
        __syncthreads();  // LDS free for the next task; s_ticket written
        if (J.signal && tid == 0) __hip_atomic_fetch_add(A.done + task.job, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        tk = __builtin_amdgcn_readfirstlane(s_ticket);
        __syncthreads();  // every wave has read s_ticket before thread 0 writes it again
    }
    if (tid == 0) {
        const uint32_t before = __hip_atomic_fetch_add(A.exits, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = before + 1 == gridDim.x;
    }
    __syncthreads();
    if (s_last) {  // everyone else has left: rearm the counters for the next launch
        // a queue whose ticket never reached its length had tasks no
        // workgroup ran (no workgroup landed on its XCD): count them
        for (uint32_t j = tid; j < A.nq; j += kBT) {
            const uint32_t got = __hip_atomic_load(A.tickets + j * kTicketStride, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t len = A.qbeg[j + 1] - A.qbeg[j];
            if (got < len) atomicAdd(A.errors, len - got);
        }
        __syncthreads();  // every queue checked before its ticket is rearmed
        for (uint32_t j = tid; j < A.njobs; j += kBT) A.done[j] = 0;
        for (uint32_t j = tid; j < A.nq; j += kBT) A.tickets[j * kTicketStride] = 0;
        if (tid == 0) *A.exits = 0;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct SizePlan {
    int l1 = 0, l2 = 0, t = 1, v1 = 0, v3 = 0;
};

int ilog2_pow2(int64_t n)
{
    if (n < 1 || (n & (n - 1))) return -1;
    int l = 0;
    while ((int64_t(1) << l) < n) ++l;
    return l;
}

bool is_small(int k) { return k <= kSmallMaxLog2; }

// Valid per-size plans, default first.
std::vector<SizePlan> candidates(int k)
{
    std::vector<SizePlan> out;
    auto variants = [](int l, int lcols) {
        std::vector<int> v;
        for (int x = 0; x <= 1; ++x)
            if (var_log2T(l, x) <= lcols) v.push_back(x);
        return v;
    };
    std::vector<int> splits;
    if (is_small(k)) {
        splits = {(k + 1) / 2, k / 2};
        if (splits[0] == splits[1]) splits.pop_back();
    } else {
        const int lo = std::max(kBigMinLocal, k - kBigMaxLocal), hi = std::min(kBigMaxLocal, k - kBigMinLocal);
        int mid = (k + 1) / 2;
        mid = std::min(std::max(mid, lo), hi);
        splits.push_back(mid);
        for (int l = lo; l <= hi; ++l)
            if (l != mid) splits.push_back(l);
    }
    for (int l1 : splits) {
        const int l2 = k - l1;
        for (int t : {1, 2, 4}) {
            if (l1 % t || l2 % t) continue;
            if (is_small(k)) {
                SizePlan sp;
                sp.l1 = l1;
                sp.l2 = l2;
                sp.t = t;
                out.push_back(sp);
                continue;
            }
            for (int v1 : variants(l1, l2))
                for (int v3 : variants(l2, l1)) {
                    SizePlan sp;
                    sp.l1 = l1;
                    sp.l2 = l2;
                    sp.t = t;
                    sp.v1 = v1;
                    sp.v3 = v3;
                    out.push_back(sp);
                }
        }
    }
    // default first: balanced split, b = 2, two LDS groups for the long lengths
    const int pref = splits.front();
    auto score = [&](const SizePlan &s) {
        const int dv = is_small(k) ? 0 : int(s.v1 != (s.l1 >= 9 ? 1 : 0)) + int(s.v3 != (s.l2 >= 9 ? 1 : 0));
        return (s.l1 != pref) * 8 + (s.t != 1) * 4 + dv;
    };
    std::stable_sort(out.begin(), out.end(), [&](const SizePlan &a, const SizePlan &b) { return score(a) < score(b); });
    return out;
}

size_t lds_bytes_for(int maxl)
{
    int64_t twn = 0;
    for (int l = 1; l <= maxl; ++l) twn = std::max<int64_t>(twn, stage_tw_total(l));
    const int64_t items = int64_t(1) << kMaxOnChipLog2;  // one LDS group holds 4096 items
    return size_t(((twn + 63) & ~int64_t(63)) + items + ((items >> 6) << 2) + 4) * sizeof(float2);
}

}  // namespace
}  // namespace paco

using paco::BatchArgs;
using paco::BatchJob;
using paco::BatchTables;
using paco::BatchTask;
using paco::SizePlan;

struct paco_batch_plan_s {
    int32_t count = 0;
    std::vector<int64_t> N, offset;
    std::map<int, SizePlan> plans;  // by log2 N
    int64_t total = 0;
    int device = 0;
    void *dev = nullptr;
    BatchArgs args{};
    int grid = 0;
    size_t lds = 0;
    int64_t gap = 0;
    int nq = 1;        // work queues
    bool coh = false;  // one queue served by several XCDs: coherent stores
    paco_batch_options opt{};
    std::string desc;
};

namespace {

paco_status bfail(paco_status st, const std::string &msg)
{
    paco::set_last_error(msg);
    return st;
}

paco_status bhip(hipError_t e, const char *what)
{
    paco::set_last_error(std::string(what) + ": " + hipGetErrorString(e));
    return PACO_ERR_HIP;
}

const void *kernel_of(bool coh)
{
    return coh ? reinterpret_cast<const void *>(paco::batch_kernel<true>)
               : reinterpret_cast<const void *>(paco::batch_kernel<false>);
}

int resident_workgroups(bool coh, size_t lds)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const hipError_t e = coh ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, paco::batch_kernel<true>, paco::kBT, lds)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, paco::batch_kernel<false>, paco::kBT, lds);
    if (e != hipSuccess) return 0;
    return cus * std::max(per, 1);
}

// Work queues: one per XCD of the device (the option PACO_BATCH_ONE_QUEUE
// forces one shared queue with device-coherent stores).
int queue_count(const paco_batch_options &opt)
{
    int dev = 0, nx = 0;
    if (opt.flags & PACO_BATCH_ONE_QUEUE) return 1;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess) return 1;
    return (nx >= 1 && nx <= paco::kMaxQueues) ? nx : 1;
}

// Builds jobs, the task order and the device tables of a batch whose
// per-size plans are fixed.  Returns PACO_OK or an error with the detail set.
paco_status build_batch(paco_batch_plan_s *P)
{
    using namespace paco;
    const int32_t count = P->count;
    // ---- per-size Phase II tables and the stage tables -----------------------
    std::vector<int> ks;
    for (auto &kv : P->plans) ks.push_back(kv.first);
    std::map<int, int> tab_of;
    std::vector<std::vector<float2>> his, los, tiles;
    for (int k : ks) {
        tab_of[k] = int(his.size());
        std::vector<float2> hi, lo, tile;
        middle_tables(k, hi, lo, tile);
        his.push_back(std::move(hi));
        los.push_back(std::move(lo));
        tiles.push_back(std::move(tile));
    }
    std::vector<float2> stw;
    int64_t stw_off[kMaxOnChipLog2 + 1];
    if (!stage_tables(stw, stw_off)) return bfail(PACO_ERR_INVALID_ARG, "internal: stage twiddle layout mismatch");

    // ---- queues: transforms to XCDs, largest first onto the least loaded ------
    int nx = queue_count(P->opt);
    int dev = 0, nxcd = 1;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&nxcd, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess)
        nxcd = 0;  // unknown: one shared, coherent queue
    P->coh = nx == 1 && nxcd != 1;  // several XCDs serve one queue
    P->nq = nx;
    std::vector<int32_t> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return P->N[a] > P->N[b]; });
    std::vector<int64_t> load(nx, 0);
    std::vector<std::vector<int32_t>> qorder(nx);
    for (int32_t i : order) {
        const int qi = int(std::min_element(load.begin(), load.end()) - load.begin());
        load[qi] += P->N[i];
        qorder[qi].push_back(i);
    }

    // ---- jobs ---------------------------------------------------------------
    std::vector<BatchJob> jobs;
    struct Chain { int32_t first; };  // P1 job of a large transform (P2 = +1, P3 = +2)
    std::vector<std::vector<Chain>> chains(nx);
    std::vector<std::vector<int32_t>> smalls(nx);
    int maxl = 1;
    for (int qi = 0; qi < nx; ++qi)
    for (int32_t i : qorder[qi]) {
        const int k = ilog2_pow2(P->N[i]);
        const SizePlan &sp = P->plans[k];
        BatchJob J{};
        J.base = P->offset[i];
        J.l1 = sp.l1;
        J.l2 = sp.l2;
        J.t = sp.t;
        J.v1 = sp.v1;
        J.v3 = sp.v3;
        J.tab = tab_of[k];
        J.dep = -1;
        maxl = std::max(maxl, std::max(sp.l1, sp.l2));
        if (is_small(k)) {
            J.kind = kSmall;
            J.ntiles = 1;
            smalls[qi].push_back(int32_t(jobs.size()));
            jobs.push_back(J);
            continue;
        }
        const int32_t first = int32_t(jobs.size());
        BatchJob a = J, m = J, c = J;
        a.kind = kP1;
        a.ntiles = int32_t((int64_t(1) << sp.l2) >> var_log2T(sp.l1, sp.v1));
        a.signal = 1;
        m.kind = kP2;
        m.ntiles = int32_t(((int64_t(1) << sp.l1) >> (sp.l1 >= 7 ? 7 : 6)) * ((int64_t(1) << sp.l2) >> 6));
        m.dep = first;
        m.dep_tiles = a.ntiles;
        m.signal = 1;
        c.kind = kP3;
        c.ntiles = int32_t((int64_t(1) << sp.l1) >> var_log2T(sp.l2, sp.v3));
        c.dep = first + 1;
        c.dep_tiles = m.ntiles;
        jobs.push_back(a);
        jobs.push_back(m);
        jobs.push_back(c);
        chains[qi].push_back({first});
    }

    // ---- launch geometry -----------------------------------------------------
    P->lds = lds_bytes_for(std::min(maxl, kMaxOnChipLog2));
    hipError_t e = hipFuncSetAttribute(kernel_of(P->coh), hipFuncAttributeMaxDynamicSharedMemorySize, int(P->lds));
    if (e != hipSuccess) return bhip(e, "hipFuncSetAttribute");
    const int resident = resident_workgroups(P->coh, P->lds);
    if (resident <= 0) return bfail(PACO_ERR_HIP, "occupancy query failed");
    // per queue: a job's successor is emitted about `gap` tiles after it, a
    // few times the workgroups that serve the queue
    P->gap = 4 * int64_t(resident) / nx;
    if (P->opt.flags & PACO_BATCH_SET_GAP) P->gap = P->opt.gap;

    // ---- task order, queue by queue ------------------------------------------
    std::vector<BatchTask> tasks;
    std::vector<uint32_t> qbeg;
    for (int qi = 0; qi < nx; ++qi) {
        qbeg.push_back(uint32_t(tasks.size()));
        const int64_t base = int64_t(tasks.size());
        std::deque<std::pair<int64_t, int32_t>> pending;  // (ready position, job)
        auto emit = [&](int32_t j) {
            for (int32_t t = 0; t < jobs[j].ntiles; ++t) tasks.push_back({jobs[j], uint32_t(j), uint32_t(t)});
            if (jobs[j].kind == kP1 || jobs[j].kind == kP2)
                pending.push_back({int64_t(tasks.size()) - base + P->gap, j + 1});
        };
        auto pos = [&]() { return int64_t(tasks.size()) - base; };
        size_t next_small = 0;
        const std::vector<int32_t> &sm = smalls[qi];
        for (const Chain &ch : chains[qi]) {
            while (!pending.empty() && pending.front().first <= pos()) {
                const int32_t j = pending.front().second;
                pending.pop_front();
                emit(j);
            }
            emit(ch.first);
        }
        while (!pending.empty()) {
            if (pending.front().first > pos() && next_small < sm.size()) {
                emit(sm[next_small++]);
                continue;
            }
            const int32_t j = pending.front().second;
            pending.pop_front();
            emit(j);
        }
        while (next_small < sm.size()) emit(sm[next_small++]);
    }
    qbeg.push_back(uint32_t(tasks.size()));
    if (tasks.size() >= 0xffffffffull) return bfail(PACO_ERR_UNSUPPORTED, "too many tasks");

    // ---- one device allocation ----------------------------------------------
    struct Piece { const void *src; size_t bytes; size_t off; };
    std::vector<Piece> pieces;
    auto add = [&](const void *src, size_t bytes) {
        pieces.push_back({src, bytes, 0});
        return pieces.size() - 1;
    };
    const size_t i_stw = add(stw.data(), stw.size() * 8);
    std::vector<size_t> i_hi, i_lo, i_tile;
    for (size_t s = 0; s < his.size(); ++s) {
        i_hi.push_back(add(his[s].data(), his[s].size() * 8));
        i_lo.push_back(add(los[s].data(), los[s].size() * 8));
        i_tile.push_back(add(tiles[s].data(), tiles[s].size() * 8));
    }
    std::vector<BatchTables> tabs(his.size());
    const size_t i_tabs = add(nullptr, tabs.size() * sizeof(BatchTables));
    const size_t i_jobs = add(jobs.data(), jobs.size() * sizeof(BatchJob));
    const size_t i_tasks = add(tasks.data(), tasks.size() * sizeof(BatchTask));
    const size_t i_qbeg = add(qbeg.data(), qbeg.size() * 4);
    const size_t i_tick = add(nullptr, size_t(nx) * kTicketStride * 4);  // one 256-byte block per queue
    const size_t i_cnt = add(nullptr, 256 * 2);                          // exits, errors
    const size_t i_done = add(nullptr, jobs.size() * 4);
    size_t total = 0;
    for (auto &pc : pieces) {
        pc.off = total;
        total += (pc.bytes + 255) & ~size_t(255);
    }
    e = hipMalloc(&P->dev, total);
    if (e != hipSuccess) {
        P->dev = nullptr;
        return bfail(PACO_ERR_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    auto at = [&](size_t i) { return static_cast<unsigned char *>(P->dev) + pieces[i].off; };
    for (size_t s = 0; s < his.size(); ++s) {
        tabs[s].hi = reinterpret_cast<const float2 *>(at(i_hi[s]));
        tabs[s].lo = reinterpret_cast<const float2 *>(at(i_lo[s]));
        tabs[s].tile = reinterpret_cast<const float2 *>(at(i_tile[s]));
        tabs[s].log2N = ks[s];
        tabs[s].log2Lo = middle_log2lo(ks[s]);
    }
    pieces[i_tabs].src = tabs.data();
    std::vector<unsigned char> staging(total, 0);  // counters start at zero
    for (auto &pc : pieces)
        if (pc.src) std::memcpy(staging.data() + pc.off, pc.src, pc.bytes);
    e = hipMemcpy(P->dev, staging.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) return bhip(e, "hipMemcpy");

    BatchArgs &A = P->args;
    A.tasks = reinterpret_cast<const BatchTask *>(at(i_tasks));
    A.jobs = reinterpret_cast<const BatchJob *>(at(i_jobs));
    A.tabs = reinterpret_cast<const BatchTables *>(at(i_tabs));
    A.stw = reinterpret_cast<const float2 *>(at(i_stw));
    for (int l = 0; l <= kMaxOnChipLog2; ++l) A.stw_off[l] = int32_t(stw_off[l]);
    A.njobs = uint32_t(jobs.size());
    A.nq = uint32_t(nx);
    A.qbeg = reinterpret_cast<const uint32_t *>(at(i_qbeg));
    A.tickets = reinterpret_cast<uint32_t *>(at(i_tick));
    A.exits = reinterpret_cast<uint32_t *>(at(i_cnt));
    A.errors = reinterpret_cast<uint32_t *>(at(i_cnt) + 256);
    // option: a tiny poll limit forces the give-up path from the host
    // (every wave still exits; results are then unspecified)
    A.spin_limit = P->opt.spin_limit ? P->opt.spin_limit : kSpinLimit;
    A.done = reinterpret_cast<uint32_t *>(at(i_done));
    // at least one workgroup per queue: workgroups are dealt to the XCDs in
    // turn, so every XCD's queue has a server (the exit check of the kernel
    // counts any queue left unserved anyway)
    P->grid = int(std::max<int64_t>(std::min<int64_t>(int64_t(resident), int64_t(tasks.size())), int64_t(nx)));

    char buf[256];
    std::snprintf(buf, sizeof buf,
                  "batch[%d transforms, %lld items, %zu jobs, %zu tasks, %d %s, grid %d x %d, lds %zu, gap %lld]",
                  count, (long long)P->total, jobs.size(), tasks.size(), nx,
                  P->coh ? "shared queue (coherent stores)" : "queues (one per XCD)", P->grid, kBT, P->lds,
                  (long long)P->gap);
    P->desc = buf;
    for (auto &kv : P->plans) {
        const SizePlan &sp = kv.second;
        std::snprintf(buf, sizeof buf, " 2^%d:%dx%d,b=%d,T1=%d,T3=%d%s", kv.first, 1 << sp.l1, 1 << sp.l2, 1 << sp.t,
                      1 << var_log2T(sp.l1, sp.v1), 1 << var_log2T(sp.l2, sp.v3), is_small(kv.first) ? "(wg)" : "");
        P->desc += buf;
    }
    if (const char *lg = std::getenv("PACO_LOG"))  // plan summary on stderr
        if (lg[0] == '1') std::fprintf(stderr, "paco batch plan: %s\n", P->desc.c_str());
    return PACO_OK;
}

hipError_t launch_batch(const paco_batch_plan_s *P, const void *in, void *out, void *ws, hipStream_t s)
{
    BatchArgs A = P->args;
    A.in = static_cast<const float2 *>(in);
    A.out = static_cast<float2 *>(out);
    A.ws = static_cast<float2 *>(ws);
    void *args[] = {&A};
    return hipLaunchKernel(kernel_of(P->coh), dim3(unsigned(P->grid)), dim3(paco::kBT), args, P->lds, s);
}

void free_plan(paco_batch_plan_s *P)
{
    if (!P) return;
    if (P->dev) (void)hipFree(P->dev);
    delete P;
}

// ---- autotuner -----------------------------------------------------------------
// For every transform size of the batch, each candidate (split, b, tile
// variants) runs a batch of copies of that size (about 2^24 items) through
// the persistent kernel; the fastest of three timed launches wins.
paco_status tune(std::map<int, SizePlan> &plans, const std::vector<int> &ks)
{
    const int64_t items = int64_t(1) << 24;
    void *buf = nullptr;
    hipError_t e = hipMalloc(&buf, size_t(items) * 8 * 3);
    if (e != hipSuccess) return bfail(PACO_ERR_ALLOC, std::string("tuning buffers: ") + hipGetErrorString(e));
    float2 *in = static_cast<float2 *>(buf), *out = in + items, *ws = out + items;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    paco_status st = PACO_OK;
    if ((e = hipMemset(buf, 0, size_t(items) * 8 * 3)) != hipSuccess || (e = hipStreamCreate(&s)) != hipSuccess ||
        (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        st = bhip(e, "tuning set-up");
    }
    for (size_t ki = 0; st == PACO_OK && ki < ks.size(); ++ki) {
        const int k = ks[ki];
        const int64_t copies = std::min<int64_t>(std::max<int64_t>(1, items >> k), 16384);
        float best = 1e30f;
        for (const SizePlan &sp : paco::candidates(k)) {
            paco_batch_plan_s *T = new (std::nothrow) paco_batch_plan_s();
            if (!T) { st = bfail(PACO_ERR_ALLOC, "host allocation failed"); break; }
            T->count = int32_t(copies);
            for (int64_t i = 0; i < copies; ++i) {
                T->N.push_back(int64_t(1) << k);
                T->offset.push_back(i << k);
            }
            T->total = copies << k;
            T->plans[k] = sp;
            st = build_batch(T);
            float ms = 1e30f;
            for (int rep = 0; st == PACO_OK && rep < 4; ++rep) {
                if ((e = hipEventRecord(e0, s)) != hipSuccess || (e = launch_batch(T, in, out, ws, s)) != hipSuccess ||
                    (e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess) {
                    st = bhip(e, "tuning launch");
                    break;
                }
                float t = 0.f;
                (void)hipEventElapsedTime(&t, e0, e1);
                if (rep > 0) ms = std::min(ms, t);  // the first launch warms up
            }
            free_plan(T);
            if (st != PACO_OK) break;
            if (ms < best) {
                best = ms;
                plans[k] = sp;
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(buf);
    return st;
}

bool valid_plan(int k, const SizePlan &sp)
{
    for (const SizePlan &c : paco::candidates(k))
        if (c.l1 == sp.l1 && c.l2 == sp.l2 && c.t == sp.t && c.v1 == sp.v1 && c.v3 == sp.v3) return true;
    return false;
}

// The device a tuning cache was measured on: its entries are reused only on
// the same architecture, CU count and cache format.
std::string cache_key()
{
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string arch = prop.gcnArchName;
    for (char &ch : arch)
        if (ch == ' ') ch = '_';
    return arch + " cus=" + std::to_string(prop.multiProcessorCount) + " format=1";
}

// Tuning cache: a "key <device key>" line, then lines "log2N l1 l2 t v1 v3";
// '#' starts a comment.  A file with another key (or none) is ignored, and
// rewritten after tuning.
void read_cache(const char *path, const std::string &key, std::map<int, SizePlan> &plans)
{
    std::ifstream f(path);
    std::string line;
    bool keyed = false;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        if (line.compare(0, 4, "key ") == 0) {
            keyed = line.substr(4) == key;
            continue;
        }
        if (!keyed) continue;
        std::istringstream is(line);
        int k;
        SizePlan sp;
        if (is >> k >> sp.l1 >> sp.l2 >> sp.t >> sp.v1 >> sp.v3)
            if (k >= paco::kBatchMinLog2 && k <= paco::kBatchMaxLog2 && valid_plan(k, sp)) plans[k] = sp;
    }
}

bool write_cache(const char *path, const std::string &key, const std::map<int, SizePlan> &plans)
{
    std::ofstream f(path);
    if (!f) return false;
    f << "# paco batched plan cache: log2N l1 l2 t v1 v3 (N1 = 2^l1, N2 = 2^l2, b = 2^t, tile variants)\n";
    f << "key " << key << '\n';
    for (auto &kv : plans)
        f << kv.first << ' ' << kv.second.l1 << ' ' << kv.second.l2 << ' ' << kv.second.t << ' ' << kv.second.v1 << ' '
          << kv.second.v3 << '\n';
    return bool(f);
}

bool bad_ptr16(const void *p) { return !p || (reinterpret_cast<uintptr_t>(p) & 15); }

}  // namespace

extern "C" {

paco_status paco_batch_plan_create(paco_batch_plan **bp, int32_t count, const int64_t *N, paco_dtype dt,
                                   const char *tune_cache_path)
{
    return paco_batch_plan_create_ex(bp, count, N, dt, tune_cache_path, nullptr);
}

paco_status paco_batch_plan_create_ex(paco_batch_plan **bp, int32_t count, const int64_t *N, paco_dtype dt,
                                      const char *tune_cache_path, const paco_batch_options *options)
{
    if (!bp) return bfail(PACO_ERR_INVALID_ARG, "plan out-pointer is NULL");
    *bp = nullptr;
    const paco_batch_options opt = options ? *options : paco_batch_options{};
    if (opt.flags & ~(PACO_BATCH_NO_TUNE | PACO_BATCH_ONE_QUEUE | PACO_BATCH_SET_GAP))
        return bfail(PACO_ERR_INVALID_ARG, "unknown batch option flag");
    if ((opt.flags & PACO_BATCH_SET_GAP) && opt.gap < 0) return bfail(PACO_ERR_INVALID_ARG, "gap must be >= 0");
    if (opt.spin_limit >= (1u << 31)) return bfail(PACO_ERR_INVALID_ARG, "spin_limit must be below 2^31");
    if (dt == PACO_C64_MFMA_FP16X3 || dt == PACO_C64_MFMA_BF16X3 || dt == PACO_C64_MFMA_BF16X6)
        return bfail(PACO_ERR_UNSUPPORTED, "the batched form runs the FP32 arithmetic only");
    if (dt != PACO_C64) return bfail(PACO_ERR_INVALID_ARG, "unknown dtype");
    if (count < 1 || !N) return bfail(PACO_ERR_INVALID_ARG, "need count >= 1 and a size array");
    paco_batch_plan_s *P = new (std::nothrow) paco_batch_plan_s();
    if (!P) return bfail(PACO_ERR_ALLOC, "host allocation failed");
    P->count = count;
    P->opt = opt;
    std::vector<int> ks;
    for (int32_t i = 0; i < count; ++i) {
        const int k = paco::ilog2_pow2(N[i]);
        if (k < 0) {
            free_plan(P);
            return bfail(PACO_ERR_NOT_POWER_OF_B, "every size must be a power of two");
        }
        if (k < paco::kBatchMinLog2 || k > paco::kBatchMaxLog2) {
            free_plan(P);
            return bfail(PACO_ERR_UNSUPPORTED, "batched sizes must lie in [2^2, 2^20]");
        }
        P->N.push_back(N[i]);
        P->offset.push_back(P->total);
        P->total += N[i];
        if (std::find(ks.begin(), ks.end(), k) == ks.end()) ks.push_back(k);
    }
    std::sort(ks.begin(), ks.end());
    hipError_t e = hipGetDevice(&P->device);
    if (e != hipSuccess) {
        free_plan(P);
        return bhip(e, "hipGetDevice");
    }
    e = paco::local_fft_prepare();
    if (e != hipSuccess) {
        free_plan(P);
        return bhip(e, "hipFuncSetAttribute");
    }
    // per-size plans: cache file, then tuning (unless PACO_BATCH_NO_TUNE), else defaults
    std::map<int, SizePlan> plans;
    const std::string key = cache_key();
    if (tune_cache_path) read_cache(tune_cache_path, key, plans);
    std::vector<int> missing;
    for (int k : ks)
        if (!plans.count(k)) missing.push_back(k);
    const bool tuning = !(opt.flags & PACO_BATCH_NO_TUNE);
    if (!missing.empty() && tuning) {
        paco_status st = tune(plans, missing);
        if (st != PACO_OK) {
            free_plan(P);
            return st;
        }
    }
    for (int k : ks)
        if (!plans.count(k)) plans[k] = paco::candidates(k).front();
    for (int k : ks) P->plans[k] = plans[k];
    if (tune_cache_path && !missing.empty() && tuning && !write_cache(tune_cache_path, key, plans)) {
        free_plan(P);
        return bfail(PACO_ERR_INVALID_ARG, std::string("cannot write the tuning cache ") + tune_cache_path);
    }
    paco_status st = build_batch(P);
    if (st != PACO_OK) {
        free_plan(P);
        return st;
    }
    paco::set_last_error("");
    *bp = P;
    return PACO_OK;
}

paco_status paco_batch_workspace_size(const paco_batch_plan *bp, size_t *bytes)
{
    if (!bytes) return bfail(PACO_ERR_INVALID_ARG, "bytes out-pointer is NULL");
    *bytes = 0;
    if (!bp) return bfail(PACO_ERR_INVALID_ARG, "plan is NULL");
    *bytes = size_t(bp->total) * 8;
    return PACO_OK;
}

paco_status paco_execute_batched(const paco_batch_plan *bp, const void *in, void *out, void *workspace,
                                 size_t workspace_bytes, void *stream)
{
    if (!bp) return bfail(PACO_ERR_INVALID_ARG, "plan is NULL");
    if (bad_ptr16(in) || bad_ptr16(out) || bad_ptr16(workspace))
        return bfail(PACO_ERR_INVALID_ARG, "in/out/workspace must be non-NULL and 16-byte aligned");
    const size_t need = size_t(bp->total) * 8;
    if (workspace_bytes < need) return bfail(PACO_ERR_WORKSPACE, "workspace smaller than the total items * 8 bytes");
    const uintptr_t wb = reinterpret_cast<uintptr_t>(workspace), ib = reinterpret_cast<uintptr_t>(in),
                    ob = reinterpret_cast<uintptr_t>(out);
    if ((wb < ib + need && ib < wb + need) || (wb < ob + need && ob < wb + need))
        return bfail(PACO_ERR_INVALID_ARG, "workspace overlaps in or out");
    if (ib != ob && ib < ob + need && ob < ib + need) return bfail(PACO_ERR_INVALID_ARG, "in and out overlap partially");
    hipError_t e = launch_batch(bp, in, out, workspace, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return bhip(e, "batched launch");
    return PACO_OK;
}

paco_status paco_batch_plan_describe(const paco_batch_plan *bp, int32_t index, int64_t *N1, int64_t *N2, int64_t *p,
                                     int32_t *b, char *buf, size_t buflen)
{
    if (!bp) return bfail(PACO_ERR_INVALID_ARG, "plan is NULL");
    if (index >= bp->count) return bfail(PACO_ERR_INVALID_ARG, "index out of range");
    if (index >= 0) {
        const int k = paco::ilog2_pow2(bp->N[index]);
        const SizePlan &sp = bp->plans.at(k);
        const int64_t n1 = int64_t(1) << sp.l1, n2 = int64_t(1) << sp.l2;
        if (N1) *N1 = n1;
        if (N2) *N2 = n2;
        // p has no effect on one device (the output is the same for every
        // valid p); the plan reports the largest p with slabs of at least 16
        // items (one 128-byte line), and at least 2
        if (p) *p = std::max<int64_t>(2, std::min(n1, n2) / 16);
        if (b) *b = 1 << sp.t;
    }
    if (buf && buflen) {
        std::strncpy(buf, bp->desc.c_str(), buflen - 1);
        buf[buflen - 1] = 0;
    }
    return PACO_OK;
}

paco_status paco_batch_errors(const paco_batch_plan *bp, uint32_t *count)
{
    if (!bp || !count) return bfail(PACO_ERR_INVALID_ARG, "plan or count is NULL");
    *count = 0;
    hipError_t e = hipMemcpy(count, bp->args.errors, sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return bhip(e, "hipMemcpy");
    return PACO_OK;
}

paco_status paco_batch_plan_destroy(paco_batch_plan *bp)
{
    free_plan(bp);
    return PACO_OK;
}

}  // extern "C"
