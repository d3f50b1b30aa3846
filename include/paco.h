/*
 * paco.h -- C ABI of the MI355X (gfx950) PACO transform library.
 *
 * PACO computes the canonical forward DFT
 *     y = Omega_N x,   (Omega_N)_{k,j} = w_N^{-kj},   w_N = exp(2*pi*i/N)
 * (paper, section 2: negative exponent, no normalisation) as three phases
 * (section 3, eq. paco-composite-op):
 *     Phase I   LocalFFT in output layout  A_{m1} (x) I_{N2},  A = P_pi Omega
 *     Phase II  one fused permutation pi_m(a ++ c) = pi_{m2}(c) ++ pi_{m1}(a)
 *               with the top-level twiddle w_N^{-pi_{m1}(a) c}
 *     Phase III LocalFFT in input layout   B_{m2} (x) I_{N1},  B = Omega P_pi
 * On one GPU the paper's p processors are p column slabs of the matrices
 * below, all resident in the same HBM.
 *
 * Data layout (section 2, eqs. input-slab-owner, factor-swapped-output-view,
 * output-slab-owner):
 *   in   N1 x N2 row-major complex64 (interleaved float re, im):
 *        in[j1*N2 + j2] = x[j1*N2 + j2]  -- i.e. simply x.
 *        Source slab q = columns [q*N2/p, (q+1)*N2/p).
 *   out  N2 x N1 row-major complex64:  out[k2*N1 + k1] = y[k1 + k2*N1]
 *        -- i.e. simply y in natural order.
 *        Target slab q' = columns [q'*N1/p, (q'+1)*N1/p).
 *   workspace  N1*N2 complex64 (N*8 bytes) of device memory.
 *
 * Ownership: the caller allocates and owns in, out, workspace (device
 * memory) and the stream.  A plan owns only its small device tables
 * (twiddle-factor tables generated in FP64 on the host and rounded once to
 * FP32; digit reversals are computed in the kernels from the indices),
 * allocated by paco_plan_create and released by
 * paco_plan_destroy.  A plan is immutable after creation and may be shared
 * by threads; executions that share a workspace must not overlap.
 *
 * Errors: every call returns paco_status (0 == PACO_OK); no exception
 * crosses the ABI.  On failure out-parameters are set to NULL/0 and nothing
 * leaks; paco_last_error() returns a thread-local detail string.  Execute
 * calls only enqueue work on the given stream and never synchronise: a
 * device fault surfaces at the caller's next synchronisation.  Arguments
 * are checked (null or misaligned pointers, undersized workspace) before
 * anything is enqueued.
 */
#ifndef PACO_H
#define PACO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PACO_OK = 0,
    PACO_ERR_INVALID_ARG = 1,   /* null/misaligned pointer, bad stage, p < 2 ... */
    PACO_ERR_NOT_POWER_OF_B = 2,/* N1 or N2 not a power of b, or b not 2^t >= 2 */
    PACO_ERR_DIVISIBILITY = 3,  /* p does not divide N1 and N2                   */
    PACO_ERR_UNSUPPORTED = 4,   /* valid for the paper, not built here (size)    */
    PACO_ERR_WORKSPACE = 5,     /* workspace smaller than paco_plan_workspace_size */
    PACO_ERR_ALLOC = 6,         /* device or host allocation failed              */
    PACO_ERR_HIP = 7            /* a HIP runtime call failed (detail in last_error) */
} paco_status;

/* Arithmetic of a plan; I/O is always complex64 (interleaved FP32 re, im).
 * The split forms run every radix-16 butterfly of the local FFTs as a real
 * contraction [Wr, -Wi; Wi, Wr][xr; xi] (K = 32) on the MFMA units, with each
 * FP32 operand split into 16-bit parts and the partial products summed in
 * FP32; twiddle multiplications stay FP32 (tables generated in FP64).  Not in
 * the paper: its DFT is exact in exact arithmetic; these trade accuracy for
 * matrix-core arithmetic, and their error against FP64 is a measured figure
 * (no bound is claimed). */
typedef enum {
    PACO_C64 = 0,               /* FP32 arithmetic on the vector ALUs                  */
    PACO_C64_MFMA_FP16X3 = 1,   /* FP16 hi + 2^11-scaled lo, per-butterfly power-of-two
                                   scale, products hi*hi + hi*lo + lo*hi (~22 bits)      */
    PACO_C64_MFMA_BF16X3 = 2,   /* BF16 hi + lo, products hi*hi + hi*lo + lo*hi (~16 bits) */
    PACO_C64_MFMA_BF16X6 = 3    /* BF16 hi + mid + lo, six products (~24 bits)           */
} paco_dtype;

/* paco_execute_stage flags */
#define PACO_NO_TWIDDLE 1       /* stage 2 only: apply the bare permutation pi_m */
#define PACO_PACKED 2           /* the fused pipeline's Phase-I buffer (below) */
#define PACO_TWO_PASS 4         /* with PACO_PACKED, stage 1: the two-pass form's Phase I */
#define PACO_SPLIT 8            /* alone: pass 1, 2 (or 3) of the plan's split form */

typedef struct paco_plan_s paco_plan;

/* Checks the problem contract of section 2 with the proofs' divisibility
 * condition (eq. exact-divisibility): b = 2^t with t >= 1; N1 = b^m1 and
 * N2 = b^m2 with m1, m2 >= 1; p >= 2 with p | N1 and p | N2 (p itself need
 * not be a power of b; the balance argument of section 4.2 uses only the
 * divisibility).  Pure host code: no HIP call, usable without a GPU.
 * Returns PACO_ERR_UNSUPPORTED for sizes the library has no kernels for
 * (N1 or N2 above 2^16, or N1*N2 above 2^28: every buffer stays below
 * 4 GiB, so the kernels address it with 32-bit byte offsets). */
paco_status paco_plan_validate(int64_t N1, int64_t N2, int64_t p, int32_t b, paco_dtype dt);

/* Validates, builds the pass plan and uploads the plan's tables to the
 * current HIP device.  *plan is NULL on failure.  A plan is meant for the
 * device current at its creation: its tables live there, and the persistent
 * passes of the symmetric form at N1 = N2 >= 8192 launch as many workgroups
 * as that device holds at once (counted here). */
paco_status paco_plan_create(paco_plan **plan, int64_t N1, int64_t N2, int64_t p, int32_t b,
                             paco_dtype dt);

/* Mixed-radix sizes, outside the paper's preconditions (section 5,
 * Limitations name sizes that are not powers of b): N1 and N2 any powers of
 * two >= 2, b = 2^t, N_i = b^{m_i} 2^{s_i} with 0 <= s_i < t.  An index of
 * [0, N_i) then has the digit radices (b, ..., b, 2^{s_i}), least
 * significant first, and pi_{m_i} of appendix A.1 becomes the reversal of
 * that digit string read back with the radices reversed, (2^{s_i}, b, ...,
 * b); it is no longer an involution, and each layout uses it in the
 * direction its definition asks for (Phase-I row a holds frequency pi(a),
 * Phase II moves (a, c) to (pi(c), pi(a)), Phase III reads logical j at row
 * pi(j)).  With s1 = s2 = 0 the plan equals paco_plan_create's.  Two-pass
 * local phases put the short digit into their first pass.  Otherwise as
 * paco_plan_create / paco_plan_validate; every entry point that takes a
 * plan accepts these. */
paco_status paco_plan_validate_mixed(int64_t N1, int64_t N2, int64_t p, int32_t b, paco_dtype dt);
paco_status paco_plan_create_mixed(paco_plan **plan, int64_t N1, int64_t N2, int64_t p, int32_t b,
                                   paco_dtype dt);

/* Plan-creation options.  Every field at zero selects the default, which is
 * what paco_plan_create builds; a plan never depends on the process
 * environment (the one exception, PACO_LOG=1, only prints each plan's pass
 * summary on stderr).  The alternatives exist for stage-wise checks of the
 * paper's own layouts and for measurement. */
typedef struct {
    uint32_t flags;        /* PACO_PLAN_* bits below                                  */
    int32_t groups1;       /* 0: default; 1, 2 or 3 LDS column groups of Phase I's
                              single-pass tile (3: two groups of a tile twice as wide) */
    int32_t groups3;       /* 0: default; the same for Phase III                     */
    int32_t cols_long;     /* 0: default; else the columns per workgroup (a power of
                              two) of a single-group pass of 2^10 or more points      */
} paco_plan_options;

#define PACO_PLAN_MIXED 1u         /* mixed-radix sizes (as paco_plan_create_mixed)        */
#define PACO_PLAN_PAPER_LAYOUT 2u  /* the paper's Phase-I layout Atilde and a Phase II that
                                      applies the whole pi_m (no packed buffer, no split
                                      form, no two-pass form)                              */
#define PACO_PLAN_NO_SPLIT 4u      /* no split form (the packed form, or the two on-chip
                                      passes of Phase I plus Phase II)                     */
#define PACO_PLAN_GENERIC 8u       /* descriptor-driven kernels only (no fast tiles, no
                                      split form); same arithmetic order as the fast tiles */
#define PACO_PLAN_NO_SYM 16u       /* no symmetric split form: the split form of Phase I
                                      alone (Phase III keeps whole columns on chip)         */

/* paco_plan_create / paco_plan_create_mixed with options (NULL: defaults).
 * Errors as paco_plan_create; PACO_ERR_INVALID_ARG for an unknown flag or a
 * field out of range. */
paco_status paco_plan_create_ex(paco_plan **plan, int64_t N1, int64_t N2, int64_t p, int32_t b, paco_dtype dt,
                                const paco_plan_options *options);

/* Bytes of device workspace paco_execute needs (N1*N2*8 for PACO_C64). */
paco_status paco_plan_workspace_size(const paco_plan *plan, size_t *bytes);

/* Runs Phase I (in -> workspace), Phase II (workspace -> out) and Phase III
 * (out -> out, in place) on `stream` (a hipStream_t; NULL = default stream).
 * in == out is allowed.  in, out and workspace are device pointers, 16-byte
 * aligned (kernels move two complex64 items per 16-byte access), of N1*N2 complex64 each (workspace: at least the reported size).
 *
 * Workspace layout.  With the paper's layouts (section 4.2) the workspace
 * holds the Phase-I buffer Atilde[a, c] = A[pi_{m1}(a), c] and Phase II packs
 * (rows a -> v = pi_{m1}(a)), exchanges, transposes and unpacks.  When the
 * plan is "fused" (single-pass Phase I, N1, N2 >= 64, b in {2, 4, 16}) the
 * pack and the block transpose move into Phase I's store: pi_{m1} composed
 * with itself is the identity (appendix A.1), so the packed slab holds
 * frequency k1 at row k1, and Phase I writes it transposed,
 *     workspace[c*N1 + k1] = A[k1, c]   (the "packed" buffer),
 * with contiguous runs on both sides of every HBM pass but Phase I's reads and
 * Phase III's writes.  Phase II is then the unpack (rows c -> pi_{m2}(c)) with
 * the top-level twiddle.  paco_plan_describe names the mode; the plan option
 * PACO_PLAN_PAPER_LAYOUT selects the paper's layouts.
 *
 * Split form.  A fused PACO_C64 plan with N1 = 2^12 and 16 | N2 <= 2^14, and
 * a PACO_C64 plan with N1 = 2^13 or 2^14 and 64 <= N2, 16 | N2, splits each
 * Phase-I column transform once more by Lemma 1, N1 = 16 x M (row
 * j1 = j + M r, frequency k1 = k0 + 16 k).  Pass 1 computes
 *     T[c][j][k0] = w_N1^{-j k0} sum_r X[j + M r, c] w_16^{-r k0}
 * into workspace[c*N1 + 16 j + k0], reading x in whole 128-byte row runs
 * (16 columns at a time; the packed Phase I reads 32-byte runs).  Pass 2
 * reads column c's T (contiguous), finishes A[k1, c] = sum_j w_M^{-j k}
 * T[c][j][k0] and writes Phase II's result row pi_{m2}(c) of out with the
 * twiddle w_N^{-k1 c}.  Phase III and out are unchanged.  With N1 = 2^12
 * the HBM passes stay three and only how Phase I's arithmetic is divided
 * between the first two differs; with N1 = 2^13 or 2^14, where Phase I takes
 * two on-chip passes otherwise, the split form saves one HBM pass.
 * paco_plan_has_split tells; the plan option PACO_PLAN_NO_SPLIT keeps the
 * other plan.
 *
 * Symmetric split form.  A plan with N1 = 16 L1 and N2 = 16 L2, L1 and L2
 * in {256, 512, 1024} (any valid b and p; square shapes with L1 = L2 = 256
 * or 512 in every dtype, the split MFMA forms running each 16-point
 * transform on MFMA in the operand layout; L1 = L2 = 1024 and the
 * non-square shapes in PACO_C64) splits Phase III the same way, with its
 * 16-point child moved into the redistribution pass (Lemma 1 on both local
 * phases; Phase I: j1 = 16 j + r, k1 = k + L1 s; Phase III:
 * j2 = jc + L2 rr, k2 = q0 + 16 q):
 *   pass 1: workspace[((k >> 4)*N2 + c)*256 + 16 r + (k & 15)] = U[c][r][k]
 *           = w_N1^{-k r} sum_j X[16 j + r, c] w_L1^{-k j}
 *   pass 2: A[k + L1 s, c] = sum_r w_16^{-s r} U[c][r][k],
 *           Z[v, c] = A[v, c] w_N^{-v c},
 *           out[(16 jc + q0)*N1 + v] = W[v][jc][q0]
 *           = w_N2^{-q0 jc} sum_rr Z[v, jc + L2 rr] w_16^{-q0 rr}
 *   pass 3: out[(q0 + 16 q)*N1 + v] = Y[q0 + 16 q, v]
 *           = sum_jc w_L2^{-q jc} W[v][jc][q0]   (in place)
 * so that every pass reads and writes whole 128-byte lines; the paper's
 * digit reversals cancel between the redistribution and Phase III's input
 * layout, as in the packed form.  Three HBM passes, the same workspace and
 * out.  In PACO_C64 the wide variant takes N2 = 2^15 = 32 L2 (L2 = 1024)
 * with N1 = 2^12 or 2^13: Phase III splits as j2 = jc + L2 rr, k2 = q0 +
 * 32 q (rr, q0 < 32), pass 2 stores W at out[(32 jc + q0)*N1 + v] after a
 * 32-point transform over rr, and pass 3 transforms rows 32 t + q0 into
 * out[(q0 + 32 q)*N1 + v]; pass 1 is the same.  paco_plan_has_split
 * reports 2; the option PACO_PLAN_NO_SYM keeps the split form of Phase I
 * alone. */
paco_status paco_execute(const paco_plan *plan, const void *in, void *out, void *workspace,
                         size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * transform of paco_execute, with the workspace held in the library's own
 * file-scope device array of PACO_NOALLOC_MAX_ITEMS complex64 items (32 MiB).
 * Each GPU the library runs on holds one such array from the first plan
 * created on it until the process ends; the plan records its address at
 * creation.  The call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine); in and out are as for paco_execute (in == out allowed).
 * Plans with N1*N2 above PACO_NOALLOC_MAX_ITEMS get PACO_ERR_WORKSPACE before
 * anything is enqueued.  Every call on one GPU shares that GPU's array, which
 * keeps the last call's contents (nothing in it needs clearing: every item is
 * written before it is read): calls that can overlap in time on one GPU
 * (streams without an order between them) race and their results are
 * undefined; calls issued on one stream are ordered. */
#define PACO_NOALLOC_MAX_ITEMS (1 << 22)
paco_status paco_execute_noalloc(const paco_plan *plan, const void *in, void *out, void *stream);

/* The inverse transform x = Omega_N^{-1} y, x[j] = (1/N) sum_k y[k] w_N^{+jk}
 * (the paper names the inverse in sections 1 and 5 without specifying it;
 * this is the textbook inverse of section 2's convention).  in = y in natural
 * order, the buffer paco_execute writes; out = x in natural order, the
 * layout paco_execute reads; the forward plan's arguments, alignment,
 * workspace and overlap rules apply.
 *
 * Ownership.  The forward transform leaves y in the factor-swapped
 * ownership: output slab q holds columns [q N1/p, (q+1) N1/p) of the N2 x N1
 * matrix Y (section 2, eq. output-slab-owner).  The inverse runs the PACO
 * phases on the swapped factorisation N2 x N1 (the plan builds its passes at
 * creation; a square plan reuses its own), so its input slabs are exactly
 * those output slabs and its output slabs, columns of the N1 x N2 matrix X,
 * are exactly the forward input's: the ownership is restored by the inverse
 * itself, with no further exchange.  The arithmetic is conj(Omega_N conj(y))
 * / N, the two conjugations and the 1/N scale (a power of two, exact) folded
 * into Phase I's loads and Phase III's stores: the same launches as
 * paco_execute.  All dtypes.  Returns PACO_ERR_UNSUPPORTED (the forward
 * plan still works) if the N2 x N1 passes could not be built at plan
 * creation (e.g. device memory for their tables). */
paco_status paco_execute_inverse(const paco_plan *plan, const void *in, void *out, void *workspace,
                                 size_t workspace_bytes, void *stream);

/* The same transform in two HBM passes instead of three (an ablation of the
 * paper's pass structure, not the paper's schedule).  Phase I writes the
 * packed buffer workspace[c*N1 + k1] = A[k1, c] as in paco_execute; Phase III
 * then reads that buffer itself.  Phase III's input-layout read of row
 * pi_{m2}(j) of Zhat[u, v] = Z[v, pi_{m2}(u)] (the theorem on the fused global
 * permutation, section 4.2) finds Z[v, j], pi_{m2} being an involution, so
 * its tile for columns v takes packed rows j in natural order and forms
 * Z[v, j] = A[v, j] w_N^{-vj} on load.
 * Twiddle and digit reversal thus happen in registers, and Phase II's HBM
 * round trip (16 of the 48 bytes per item of the three passes) is gone.
 * out = y in natural order, as paco_execute.  Arguments, alignment,
 * workspace and overlap rules as paco_execute (in == out allowed: Phase III
 * writes out only after Phase I has read all of in).  Needs a fused
 * PACO_C64 plan whose Phase III is one on-chip pass (N1 <= 2^12);
 * paco_plan_has_two_pass tells; otherwise PACO_ERR_UNSUPPORTED. */
paco_status paco_execute_two_pass(const paco_plan *plan, const void *in, void *out, void *workspace,
                                  size_t workspace_bytes, void *stream);

/* *yes = 1 when paco_execute_two_pass runs for this plan, else 0. */
paco_status paco_plan_has_two_pass(const paco_plan *plan, int32_t *yes);

/* *yes = 2 when paco_execute (and paco_execute_inverse of a square plan)
 * runs the symmetric split form for this plan, 1 for the split form of
 * Phase I alone, else 0. */
paco_status paco_plan_has_split(const paco_plan *plan, int32_t *yes);

/* Runs one phase alone, for stage-wise checks and per-phase timing, always
 * in the paper's layouts unless flags holds PACO_PACKED:
 *   stage 1: src (N1 x N2, x) -> dst (N1 x N2, Phase-I layout Atilde);
 *            PACO_PACKED: dst = the packed buffer dst[c*N1 + k1] = A[k1, c]
 *            (src and dst must differ)
 *   stage 2: src (N1 x N2, Atilde; PACO_PACKED: the packed buffer) -> dst
 *            (N2 x N1, Zhat); flags may also hold PACO_NO_TWIDDLE; src and
 *            dst must not overlap
 *   stage 3: src (N2 x N1, Zhat) -> dst (N2 x N1, Y); src == dst allowed;
 *            PACO_PACKED: src = the packed buffer, Phase III of
 *            paco_execute_two_pass (twiddle on load), src == dst allowed
 * Stage 1 also allows src == dst.  PACO_PACKED on a plan that is not fused
 * (stage 3: that has no two-pass form) returns PACO_ERR_UNSUPPORTED;
 * PACO_NO_TWIDDLE on stage 1 or 3 returns PACO_ERR_INVALID_ARG.
 * Stage 1 with PACO_PACKED | PACO_TWO_PASS is the two-pass form's Phase I:
 * the same output as PACO_PACKED alone, its source read with last-use
 * (non-temporal) loads (PACO_ERR_UNSUPPORTED without a two-pass form;
 * PACO_TWO_PASS elsewhere: PACO_ERR_INVALID_ARG).
 * PACO_SPLIT (alone) runs the split form's pass 1 (stage 1: src = x, dst =
 * the split buffer T) or pass 2 (stage 2: src = T, dst = Zhat, the same
 * result as stage 2 of paco_execute); src and dst must not overlap;
 * PACO_ERR_UNSUPPORTED without a split form, PACO_ERR_INVALID_ARG with
 * other flags or stage 3.  On a plan with the symmetric split form
 * PACO_SPLIT runs its passes instead: stage 1 (src = x, dst = the buffer U),
 * stage 2 (src = U, dst = the buffer W, see paco_execute) and stage 3
 * (src = W, dst = out = y; src == dst allowed); stages 1 and 2 out of
 * place. */
paco_status paco_execute_stage(const paco_plan *plan, int stage, int flags, const void *src,
                               void *dst, void *stream);

/* Number of device kernel launches paco_execute enqueues for this plan, and
 * a short human-readable description of the pass plan. */
paco_status paco_plan_describe(const paco_plan *plan, int32_t *launches, char *buf, size_t buflen);

paco_status paco_plan_destroy(paco_plan *plan);

/* ---- batched form ---------------------------------------------------------
 * Many independent transforms, transform i of N[i] = 2^k items (2 <= k <= 20),
 * each computed as y_i = Omega_{N_i} x_i through the same three phases
 * (section 3) with its own factorisation N_i = N1 * N2, base b and tile
 * widths, all inside ONE kernel launch (a persistent grid that takes tiles
 * from a work queue).  Layout: the transforms are packed back to back, x_i at
 * items [off_i, off_i + N[i]) of `in`, off_i = N[0] + ... + N[i-1]; y_i is
 * written in natural order at the same items of `out`.
 */
typedef struct paco_batch_plan_s paco_batch_plan;

/* Plans `count` transforms of sizes N[0..count-1] (copied; the caller keeps
 * N).  The per-size choices (N1 = 2^l1 with N2 = N/N1, b in {2, 4, 16}
 * dividing both exponents, tile widths) come from, in order: the tuning
 * cache file tune_cache_path (text, one line per size, written by an earlier
 * call), else timing every candidate on the current device (allocates about
 * 400 MB of device memory for a moment; the option PACO_BATCH_NO_TUNE of
 * paco_batch_plan_create_ex skips the timing and takes the defaults), after which
 * the cache file, if named, is (re)written.  NULL: tune now, no file.
 * dt must be PACO_C64 (the split MFMA forms are single-transform only).
 * Errors: NOT_POWER_OF_B (a size not a power of two), UNSUPPORTED (a size
 * outside [2^2, 2^20], or another dt), INVALID_ARG (count < 1, NULL N, an
 * unknown dt, unwritable cache). */
paco_status paco_batch_plan_create(paco_batch_plan **bp, int32_t count, const int64_t *N, paco_dtype dt,
                                   const char *tune_cache_path);

/* Batch-plan options (every field zero: the defaults of
 * paco_batch_plan_create). */
typedef struct {
    uint32_t flags;        /* PACO_BATCH_* bits below                              */
    uint32_t spin_limit;   /* 0: default (2^22); polls before a completion wait
                              gives up and is counted by paco_batch_errors          */
    int64_t gap;           /* with PACO_BATCH_SET_GAP: tiles between a job and its
                              successor in a queue (default: 4 x the resident
                              workgroups per queue)                                  */
} paco_batch_options;

#define PACO_BATCH_NO_TUNE 1u      /* default per-size plans, no timing (a cache file is
                                      still read if named, never written)               */
#define PACO_BATCH_ONE_QUEUE 2u    /* one shared work queue with device-coherent stores
                                      instead of one queue per XCD                      */
#define PACO_BATCH_SET_GAP 4u      /* use options->gap                                  */

/* paco_batch_plan_create with options (NULL: defaults); INVALID_ARG for an
 * unknown flag or a negative gap. */
paco_status paco_batch_plan_create_ex(paco_batch_plan **bp, int32_t count, const int64_t *N, paco_dtype dt,
                                      const char *tune_cache_path, const paco_batch_options *options);

/* Bytes of device workspace paco_execute_batched needs: 8 * sum N[i]. */
paco_status paco_batch_workspace_size(const paco_batch_plan *bp, size_t *bytes);

/* Runs every transform of the plan with one kernel launch on `stream`.
 * in, out and workspace are 16-byte aligned device buffers of sum N[i]
 * complex64 items (workspace: at least the reported size); in == out is
 * allowed, any other overlap is rejected.  The call enqueues exactly one
 * kernel and no memset or allocation, so it may be captured into a HIP
 * graph and replayed.  Executions of one batch plan must not overlap in
 * time (they share the plan's work-queue counters): issue them on one
 * stream.  A completion wait that exceeds its poll limit is counted (see
 * paco_batch_errors) instead of hanging; the launch then still completes,
 * with unspecified results.  The limit is 2^22 polls; the option spin_limit
 * of paco_batch_plan_create_ex sets another (testing). */
paco_status paco_execute_batched(const paco_batch_plan *bp, const void *in, void *out, void *workspace,
                                 size_t workspace_bytes, void *stream);

/* Per-transform plan of transform `index` (N1, N2, the reported slab count p
 * and b; any pointer may be NULL; index < 0 fills only buf) and a short
 * description of the whole batch plan in buf. */
paco_status paco_batch_plan_describe(const paco_batch_plan *bp, int32_t index, int64_t *N1, int64_t *N2, int64_t *p,
                                     int32_t *b, char *buf, size_t buflen);

/* Number of completion waits that gave up since the plan was created
 * (0 in every correct run).  Synchronous: copies one counter to the host. */
paco_status paco_batch_errors(const paco_batch_plan *bp, uint32_t *count);

paco_status paco_batch_plan_destroy(paco_batch_plan *bp);

const char *paco_status_string(paco_status st);
const char *paco_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PACO_H */
