/*
 * rplu.h -- C ABI of the MI355X (gfx950) Randomly Pivoted LU library.
 *
 * Randomly Pivoted LU (Gilles & Wilber, "Low-Rank Approximation by Randomly
 * Pivoted LU") builds a rank-k approximation A ~ L U by k steps of Gaussian
 * elimination in which the pivot (i, j) of step t is drawn with probability
 * |S_ij|^2 / ||S||_F^2 from the current Schur complement S = A^(t)
 * (Sec. 1, the RPLU distribution; Alg. 1). The library runs each step on the
 * device in four parts: reduce |S_ij|^2 into row masses; draw the row, then
 * the column of that row, by inverse-CDF sampling on a counter-based Philox
 * stream (two-stage sampling, Sec. 4.1); copy the pivot row into U and the
 * scaled pivot column into L; apply the rank-1 update
 * S <- S - L(:,t) U(t,:) (eq. residual_update) while accumulating the next
 * step's masses in the same pass.
 *
 * Two forms:
 *   rplu_dense   S is stored in device memory and swept once per step.
 *   rplu_cauchy  S is Cauchy-like (eq. cauchy-like): s_ij = (G_i,: B_:,j) /
 *                (x_i - y_j). Only the generators G, B are stored and updated
 *                (eqs. generator_update_g/_b, Alg. 3); entries are regenerated
 *                on the fly and the row masses are computed exactly.
 * plus rplu_batched (many independent dense instances in one persistent
 * launch) and a continuous-batching server (rplu_server_*).
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers owned by the caller; the
 *     library never frees them. Host pointers are named *_host.
 *   - Indices are 0-based. piv[2t] = i_t, piv[2t+1] = j_t.
 *   - L is n x k column-major: column t starts at L + t*ldl (ldl >= n).
 *   - U is k x m row-major: row t starts at U + t*ldu (ldu >= m).
 *   - A is n x m row-major with leading dimension lda >= m. It is
 *     OVERWRITTEN with the final Schur complement S^(rank) (unless
 *     RPLU_FLAG_KEEP_INPUT).
 *   - Complex data are interleaved (re, im) pairs. Masses are |z|^2, U is not
 *     conjugated, L(:,t) = S_:,j / S_ij with L(i_t, t) = 1.
 *   - Pivot row and column of each update are set to exactly 0.
 *   - Random numbers: Philox4x64-10 with key (seed, 0) and counter
 *     (t, stream, 0, 0); u1 = (w0 >> 11) 2^-53 draws the row, u2 =
 *     (w1 >> 11) 2^-53 the column. A drawn index is the first whose
 *     inclusive prefix of masses exceeds u * (last prefix), so an index of
 *     zero mass is never drawn.
 *   - Stop test, before each draw, with T = ||S^(t)||_F^2 and T0 = ||A||_F^2:
 *     T == 0 -> EXHAUSTED; rel_tol > 0 and T <= rel_tol^2 T0 -> TOL;
 *     optional stall rule -> STALL (RPLU_FLAG_STALL_STOP);
 *     t == kmax -> RANK (TOL_UNREACHED if rel_tol > 0), where
 *     kmax = min(n, m) if max_rank == 0, else min(max_rank, n, m).
 *   - Calls that take a hip_stream (a hipStream_t; NULL = default stream)
 *     enqueue on it and synchronise with it once per chunk of steps (to stop
 *     early) and at the end (to fill info). By default the step loop is
 *     captured once into hipGraphs (a chunk of steps and the remainder) on a
 *     context-owned stream and replayed on hip_stream; the instantiated
 *     graphs are cached in the context and reused by calls with the same
 *     buffers, sizes and options.
 *   - Errors return a negative rplu_status; rplu_last_error() gives a
 *     thread-local message. No call aborts or throws across the ABI.
 */
#ifndef RPLU_H
#define RPLU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rplu_status;

enum {
    RPLU_OK = 0,
    RPLU_PENDING = 1,          /* server: job admitted or queued, not done  */
    RPLU_E_ARG = -1,           /* invalid argument (shape, pointer, dtype)  */
    RPLU_E_NOMEM = -2,         /* device workspace could not be allocated   */
    RPLU_E_HIP = -3,           /* a HIP runtime call failed                 */
    RPLU_E_NONFINITE = -4,     /* NaN/Inf in the input or a pivot           */
    RPLU_E_BUSY = -5,          /* server queue full                         */
    RPLU_E_UNSUPPORTED = -6,   /* valid but not implemented combination     */
    RPLU_E_ZERO_PIVOT = -7,    /* a forced pivot has S_ij == 0              */
    RPLU_E_BOUND = -8          /* RPLU_FLAG_BOUNDS: no row accepted in
                                  RPLU_BOUND_MAX_TRIALS trials (a bound
                                  below a row mass)                         */
};

typedef enum {
    RPLU_R32 = 1,    /* float                       */
    RPLU_R64 = 2,    /* double                      */
    RPLU_C64 = 3,    /* complex float  (re, im)     */
    RPLU_C128 = 4    /* complex double (re, im)     */
} rplu_dtype;

enum {
    RPLU_STOP_RANK = 1,
    RPLU_STOP_TOL = 2,
    RPLU_STOP_EXHAUSTED = 3,
    RPLU_STOP_TOL_UNREACHED = 4,
    RPLU_STOP_STALL = 5,       /* RPLU_FLAG_STALL_STOP: T stopped falling      */
    RPLU_STOP_REFRESH = 6      /* internal: a residual replacement is due
                                  (RPLU_FLAG_REFRESH); never returned          */
};

enum {
    RPLU_FLAG_COLMASS = 1u << 0,  /* also reduce column masses in each sweep  */
    RPLU_FLAG_GRAPH = 1u << 1,    /* replay the step loop as a hipGraph (the
                                     default; accepted for clarity)            */
    RPLU_FLAG_NO_GRAPH = 1u << 2, /* plain kernel launches, no hipGraph        */
    RPLU_FLAG_STALL_STOP = 1u << 3, /* stall rule (below), for tolerance runs
                                     whose target may lie under the rounding
                                     floor of single precision                */
    RPLU_FLAG_SPLIT_SAMPLER = 1u << 4, /* dense: draw each pivot with the two
                                     wide kernels used for n or m > 12288
                                     (row draw; pivot row and column draw)
                                     also when n, m <= 12288, where one
                                     fused workgroup kernel is the default;
                                     every output is the same bit for bit.
                                     The Cauchy-like path has one form.      */
    RPLU_FLAG_C2PLU = 1u << 5,      /* dense and Cauchy-like: complete 2-norm
                                     pivoting (Sec. 2.3.3) instead of the
                                     random draws: i = the first row of
                                     largest mass, then j = the first column
                                     of largest |S_ij| in that row (ties go
                                     to the smallest index); same update and
                                     stop test, seed and stream unused.
                                     rplu_batched and rplu_server_submit
                                     reject it in a job (RPLU_E_ARG).        */
    RPLU_FLAG_KEEP_INPUT = 1u << 8, /* rplu_dense / rplu_cauchy: run on a copy
                                     of A (of G and B) in the context's
                                     workspace; the caller's arrays are not
                                     modified and the final Schur complement
                                     (generators) is not returned. With
                                     RPLU_FLAG_REFRESH and no opts.A_orig, A
                                     itself is the original. Not accepted by
                                     rplu_dense_noalloc.                     */
    RPLU_FLAG_LAZY_SWEEP = 1u << 9, /* dense: the deferred sweep (S read every
                                     step, written back every RPLU_LAZY_STEPS
                                     steps, the pending updates applied on
                                     the fly in the same order: the same
                                     results bit for bit) also below its
                                     default size; needs L and U, not with
                                     RPLU_FLAG_COLMASS (then eager)          */
    RPLU_FLAG_EAGER_SWEEP = 1u << 10, /* dense: read and write S every step
                                     (the default below RPLU_LAZY_MIN_BYTES) */
    RPLU_FLAG_BOUNDS = 1u << 12,    /* rplu_cauchy: Alg. 3 as printed: certified
                                     row-norm upper bounds u_i with
                                     ||S_i,:||^2 <= u_i <= nu ||S_i,:||^2
                                     (App. C: quadtrees and interaction lists
                                     built once per run on the host, bounds
                                     per step on the device) in place of the
                                     exact all-pairs masses, and the row
                                     drawn by rejection: trial q of step t
                                     draws i from u with word w0 of Philox
                                     counter (t, stream, q, 0) and accepts
                                     when v u_i < ||S_i,:||^2, v from its word
                                     w2 (at most RPLU_BOUND_MAX_TRIALS); the
                                     column draw keeps w1 of trial 0. The stop
                                     test runs on sum(u): the tolerance stop
                                     is sum(u) <= (rel_tol^2 / nu) sum(u_0),
                                     which certifies ||S|| <= rel_tol ||A||;
                                     info.a_fro2 / res_fro2 are then the
                                     bound sums, info.trials the trials.
                                     opts.bound_nu (0: 5) and bound_leaf
                                     (0: 32, at most 64). Not with
                                     RPLU_FLAG_COLMASS; rplu_cauchy only.   */
    RPLU_FLAG_MAXMASS_STOP = 1u << 13, /* rplu_dense / rplu_cauchy: the tolerance
                                     stop compares the largest row mass
                                     (bound, with RPLU_FLAG_BOUNDS) with
                                     rel_tol^2 times its value at step 0
                                     (the stop rule of Alg. 4) instead of
                                     the total                              */
    RPLU_FLAG_CPLU = 1u << 11,      /* dense (rplu_dense): complete pivoting
                                     (Sec. 1; Sec. 2.3.2) instead of the
                                     random draws: (i, j) = the entry of
                                     largest |S_ij|^2 (FP64) over all of S,
                                     the first in row-major order among
                                     equal ones. Each sweep also keeps the
                                     largest |S_ij|^2 of every row; i is the
                                     first row of largest such value, j the
                                     first column of largest |S_ij| in it.
                                     Same update and stop test, seed and
                                     stream unused. Not with RPLU_FLAG_C2PLU
                                     (RPLU_E_ARG) or RPLU_FLAG_COLMASS;
                                     rplu_cauchy, rplu_batched and the
                                     server reject it (RPLU_E_UNSUPPORTED,
                                     RPLU_E_ARG).                            */
    RPLU_FLAG_CERTIFY = 1u << 7,    /* server, dense R32/R64 jobs: after the run,
                                     ||A - L U||_F^2 is formed in FP64 on the
                                     matrix cores from the original A and
                                     returned in info.err_fro2 (needs L, U) */
    RPLU_FLAG_REFRESH = 1u << 6     /* dense R32/R64 (rplu_dense, batches, the
                                     server): residual replacement. Before
                                     the draw of step t, when ||S||^2 has
                                     fallen to RPLU_REFRESH_DROP2 times its
                                     value at the start or at the previous
                                     replacement, or when the stall rule
                                     fires above rel_tol, S is replaced by
                                     the true residual A - L U of the t steps
                                     taken, formed in FP64 with the matrix
                                     cores from the original matrix
                                     (opts.A_orig / job.A_orig) and rounded to
                                     the element type (every entry: earlier
                                     pivot rows and columns keep the errors
                                     the stored factors leave there and may
                                     be drawn again); the run goes on from
                                     step t (same Philox stream, stall window
                                     restarted), at most RPLU_MAX_REFRESH
                                     times. The rounding errors of earlier
                                     steps then no longer stay in S, so a
                                     single-precision sweep draws its pivots
                                     from a residual accurate to its own
                                     precision at every level and reaches
                                     tolerances near its rounding floor. A
                                     tolerance stop on a swept S is taken
                                     again on the replaced residual (whose
                                     total is the true error of the stored
                                     factors), so res_fro2 at a TOL stop is
                                     ||A - L U||_F^2 up to the rounding of
                                     the residual. Needs L and U.            */
};

/* Deferred dense sweep: steps per write-back of S, and the size of S
 * (n * lda * element bytes) from which rplu_dense uses it by default when L
 * and U are stored. */
#define RPLU_LAZY_STEPS 4
#define RPLU_LAZY_MIN_BYTES ((size_t)64 << 20)

/* Residual replacements per run under RPLU_FLAG_REFRESH, and the fall of
 * ||S||_F^2 between two of them that triggers one. */
#define RPLU_MAX_REFRESH 8
#define RPLU_REFRESH_DROP2 1e-4

/* Stall rule (a library extension, not from the paper): with
 * RPLU_FLAG_STALL_STOP the run keeps the best total T_best and the step
 * t_best where T last fell below (63/64) T_best (at the start T_best = T0,
 * t_best = 0), and stops with RPLU_STOP_STALL at step t once
 * t - t_best >= RPLU_STALL_WINDOW. A transient rise of T (one step can
 * increase the residual) does not end the run; a residual at the rounding
 * floor of the working precision does. Tested after the tolerance and before
 * the rank limit. */
#define RPLU_STALL_WINDOW 64

/* Per-step trace words (opts.trace, RPLU_TRACE_WORDS doubles per step t):
 *  0 T        total mass ||S^(t)||_F^2 (last row prefix)
 *  1 u1*T     row draw target
 *  2 lo_i     lower CDF edge of the row bin used (prefix before i)
 *  3 hi_i     upper CDF edge of the row bin used (prefix at i)
 *  4 T_i      pivot row's own total (last prefix of |S_i,:|^2)
 *  5 u2*T_i   column draw target
 *  6 lo_j     lower CDF edge of the column bin used
 *  7 hi_j     upper CDF edge of the column bin used
 *  8 a.re     pivot entry S_ij (real part)
 *  9 a.im     pivot entry (imaginary part, 0 for real dtypes)
 * 10 i        pivot row (as a double)
 * 11 j        pivot column (as a double)                                   */
#define RPLU_TRACE_WORDS 12

/* RPLU_FLAG_BOUNDS: defaults and limits. */
#define RPLU_BOUND_NU_DEFAULT 5.0
#define RPLU_BOUND_LEAF_DEFAULT 32
#define RPLU_BOUND_LEAF_MAX 64
#define RPLU_BOUND_MAX_TRIALS 256

typedef struct {
    int64_t max_rank;       /* k; 0 => min(n, m)                                */
    double rel_tol;         /* stop when ||S||_F <= rel_tol ||A||_F; 0 => off   */
    uint64_t seed;          /* Philox key word 0                                */
    uint64_t stream;        /* Philox counter word 1 (instance / request id)    */
    uint32_t flags;         /* RPLU_FLAG_*                                      */
    uint32_t reserved;
    const int32_t* forced;  /* device, 2*kmax ints: use (i_t, j_t) instead of the
                               draws (draws are still traced); NULL = sample    */
    double* trace;          /* device, kmax*RPLU_TRACE_WORDS doubles, or NULL   */
    double* rowmass_out;    /* device, kmax*n doubles: the row masses each draw
                               used (dense: per row; Cauchy: per row), or NULL  */
    double* colmass_out;    /* device, kmax*m doubles: column masses of S^(t),
                               needs RPLU_FLAG_COLMASS, or NULL                  */
    const void* A_orig;     /* device: the unmodified input (RPLU_FLAG_REFRESH),
                               n x m row-major with lda_orig >= m, not
                               overlapping A; otherwise ignored                 */
    int64_t lda_orig;
    double bound_nu;        /* RPLU_FLAG_BOUNDS: the factor nu >= 1 (0: 5)      */
    int32_t bound_leaf;     /* RPLU_FLAG_BOUNDS: quadtree leaf size, 1..64 (0: 32) */
    uint32_t reserved2;
} rplu_opts;

typedef struct {
    int64_t rank;           /* pivots taken                                     */
    int32_t stop;           /* RPLU_STOP_*                                      */
    int32_t status;         /* this run's rplu_status: RPLU_OK or an RPLU_E_*
                               code (per instance for rplu_batched)            */
    double a_fro2;          /* ||A||_F^2 as reduced on the device               */
    double res_fro2;        /* ||S^(rank)||_F^2 at the final stop test          */
    double err_fro2;        /* server jobs with RPLU_FLAG_CERTIFY: ||A - L U||_F^2
                               in FP64 from the original A (rplu_verify's
                               contraction); -1 otherwise                      */
    int32_t refreshes;      /* residual replacements made (RPLU_FLAG_REFRESH)   */
    int32_t first_refresh;  /* step of the first one, or -1                    */
    int64_t trials;         /* RPLU_FLAG_BOUNDS: row trials over all steps      */
} rplu_info;

typedef struct rplu_ctx_s* rplu_ctx;

/* Context: device workspace (row masses, step state, partial sums), a pinned
 * host staging word and the batched-launch tuning table. Not thread-safe; use
 * one context per host thread. hbm_budget_bytes caps the device workspace the
 * context may hold (grow-only; a call that would need more fails with
 * RPLU_E_NOMEM before anything is enqueued); 0 = no cap. The workspace of a
 * dense run is about 8 n + 16 (n + m) / 512 bytes plus, with
 * RPLU_FLAG_KEEP_INPUT, a copy of A; of a Cauchy-like run about
 * 8 n (splits + 1) bytes plus, with RPLU_FLAG_KEEP_INPUT, a copy of G and B. */
rplu_status rplu_create(int device, size_t hbm_budget_bytes, rplu_ctx* out);
rplu_status rplu_destroy(rplu_ctx ctx);

/* Dense RPLU (Alg. 1 with two-stage exact sampling, Sec. 4.1).
 * A: n x m, dtype, row-major, lda >= m; overwritten by S^(rank).
 * piv: 2*kmax int32. L: n x kmax col-major (ldl >= n). U: kmax x m row-major
 * (ldu >= m). L or U may be NULL to skip storing that factor (the update still
 * runs; U row t is then kept in workspace). info: host pointer, required.
 * Real dtypes R32/R64 and complex C64/C128 are supported; R32/C64 sweep in
 * single precision with FP64 masses, prefix sums, totals and pivot reciprocal. */
rplu_status rplu_dense(rplu_ctx ctx, rplu_dtype dtype, int64_t n, int64_t m,
                       void* A, int64_t lda, const rplu_opts* opts,
                       int32_t* piv, void* L, int64_t ldl, void* U, int64_t ldu,
                       rplu_info* info, void* hip_stream);

/* RPLU in CUR form (Alg. 2, Sec. 4.1): the approximation is kept as
 * A[:, J] U A[I, :] with the core U = A[I, J]^{-1}, grown each step by block
 * inversion (eq. block-inverse-update); the residual A - A[:, J] U A[I, :] is
 * never formed, its row norms are updated from products with A (Sec. 4.1,
 * row-norm updates). A is only READ: n x m, dtype, row-major, lda >= m.
 * Each step reads A once (the rows not yet selected) plus O(k m + n k)
 * other data. The draws, stop test and stall rule are those of rplu_dense on
 * the row-norm estimates (info.a_fro2 = their sum at step 0 = ||A||_F^2,
 * info.res_fro2 = their sum at the stop test).
 * piv: 2*kmax int32: piv[2t] = i_t (I in selection order), piv[2t+1] = j_t.
 * Ucore: kmax x kmax row-major, ldc >= kmax, FP64 for R32/R64 and complex
 * FP64 for C64/C128; on return its leading rank x rank block is
 * A[I, J]^{-1}. All arithmetic other than the storage of A is FP64.
 * kmax <= RPLU_CUR_MAX_RANK. Flags: RPLU_FLAG_C2PLU (greedy choices, Sec.
 * 2.3.3), RPLU_FLAG_STALL_STOP, RPLU_FLAG_NO_GRAPH; RPLU_FLAG_KEEP_INPUT is
 * implied; RPLU_FLAG_COLMASS, _REFRESH and _CPLU are rejected
 * (RPLU_E_UNSUPPORTED). opts.forced, opts.trace and opts.rowmass_out (the
 * estimates before each draw) as for rplu_dense. Workspace: about
 * n (9 + kmax s) + 16 kmax^2 + 48 (m + kmax) bytes (s = element size of A;
 * it holds the compact copy of A[:, J] and the transpose of the core).
 * The row-norm estimates are accurate to about 1e-16 ||A||_F^2 (rounding of
 * the updates); a drawn row whose residual row is exactly 0 ends the run
 * with RPLU_E_ZERO_PIVOT. */
#define RPLU_CUR_MAX_RANK 2048
rplu_status rplu_cur(rplu_ctx ctx, rplu_dtype dtype, int64_t n, int64_t m, const void* A,
                     int64_t lda, const rplu_opts* opts, int32_t* piv, void* Ucore,
                     int64_t ldc, rplu_info* info, void* hip_stream);

/* CUR-AAA (Alg. 4, Sec. 5.3): a rational approximation
 * r(z) = sum_j w_j f(t_j) / (z - t_j) / sum_j w_j / (z - t_j) of samples
 * (z_q, f_q), q < m (device, complex FP64), from a CUR decomposition of the
 * Loewner matrix of a random split of the samples. The split: sample q gets
 * the key w0 of Philox4x64-10 with key (seed, 1) and counter (q, 0, 0, 0);
 * the ceil(m/2) smallest keys (ties by index) form X, the others Y, each in
 * sample order. The generators G = [f^x / alpha, alpha], B = [alpha;
 * -f^y / alpha] with alpha = sqrt(max |f|) (eq. loewner-generators) go
 * through rplu_cauchy (p = 2, seed, stream 0) until the largest row mass is
 * at most eps^2 times its initial value (RPLU_FLAG_MAXMASS_STOP), at most
 * max_support steps. The selected rows and the selected columns each serve
 * as support points: the weights are the right singular vector of the
 * smallest singular value of the Loewner matrix of eq. Laaa over the other
 * samples (one-sided Jacobi rotations on the device), and the fit with the
 * smaller largest error |f - r| over all samples is returned (the rows on
 * ties): support (device, max_support int32: indices into z) and weights
 * (device, max_support complex FP64), k in info. flags: RPLU_FLAG_C2PLU,
 * RPLU_FLAG_BOUNDS (bound_opts->bound_nu / bound_leaf; bound_opts may be
 * NULL), RPLU_FLAG_NO_GRAPH. Synchronous; allocates its own device
 * buffers. */
typedef struct {
    int64_t k;              /* support points returned (= rank)                 */
    int64_t rank;           /* steps of the CUR run                             */
    int64_t trials;         /* rejection trials (RPLU_FLAG_BOUNDS)              */
    int32_t which;          /* 0: the selected rows (points of X), 1: columns   */
    int32_t stop;           /* the CUR run's RPLU_STOP_*                        */
    double max_err;         /* max over the samples of |f - r|                  */
    double err_rows;        /* the same for the fit on the rows                 */
    double err_cols;        /* and on the columns                               */
} rplu_aaa_info;
rplu_status rplu_cur_aaa(rplu_ctx ctx, int64_t m, const void* z, const void* f, double eps,
                         uint64_t seed, int64_t max_support, uint32_t flags,
                         const rplu_opts* bound_opts, int32_t* support, void* weights,
                         rplu_aaa_info* info, void* hip_stream);

/* Cauchy-like RPLU (Alg. 3 with exact row masses, Sec. 5.1), C128 only.
 * x: n complex nodes, y: m complex nodes (x_i != y_j required), G: n x p
 * row-major, B: p x m row-major, 1 <= p <= 4. G and B are OVERWRITTEN with the
 * generators of S^(rank) (eqs. generator_update_g/_b). L, U, piv as for
 * rplu_dense; U(t,:) is the regenerated pivot row, L(:,t) the pivot column
 * divided by the pivot. No n x m array is ever stored. With
 * RPLU_FLAG_COLMASS and opts.colmass_out, row t of colmass_out receives the
 * exact column masses sum_i |s_ij|^2 of S^(t) (the same all-pairs pass with
 * rows and columns exchanged, which doubles the mass work of a step). */
rplu_status rplu_cauchy(rplu_ctx ctx, rplu_dtype dtype, int64_t n, int64_t m,
                        int32_t p, const void* x, const void* y, void* G, void* B,
                        const rplu_opts* opts, int32_t* piv, void* L, int64_t ldl,
                        void* U, int64_t ldu, rplu_info* info, void* hip_stream);

/* Allocation-free dense RPLU, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc). Same arguments, results and errors as rplu_dense (bit for bit:
 * the same kernels in plain launches), without a context. The step state,
 * row masses and chunk totals live in a fixed device array of
 * RPLU_NOALLOC_SCRATCH_BYTES that the library defines once per device and
 * keeps until the process ends; this call and what it calls allocate nothing
 * (no hipMalloc, hipFree or graph instantiation; the state is read back into
 * pageable host memory on the caller's stream). Runs on the current device.
 * A problem whose scratch (rplu_dense_noalloc_bytes) exceeds the array is
 * rejected with RPLU_E_ARG before anything is enqueued; without U and with
 * RPLU_FLAG_COLMASS the scratch also holds a U row and the column partials.
 * RPLU_FLAG_NO_GRAPH is implied. Calls on one device share the array: calls
 * that overlap in time on one device (other host threads, other streams)
 * race and must be serialised by the caller. */
#define RPLU_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
rplu_status rplu_dense_noalloc(rplu_dtype dtype, int64_t n, int64_t m, void* A, int64_t lda,
                               const rplu_opts* opts, int32_t* piv, void* L, int64_t ldl,
                               void* U, int64_t ldu, rplu_info* info, void* hip_stream);
/* Scratch bytes rplu_dense_noalloc needs for this problem (has_U: U is not
 * NULL); 0 for an invalid dtype or shape. */
size_t rplu_dense_noalloc_bytes(int dtype, int64_t n, int64_t m, uint32_t flags, int has_U);

/* ------------------------------------------------------------- batched */

enum { RPLU_JOB_DENSE = 1, RPLU_JOB_CAUCHY = 2 };

/* One independent problem. Dense fields: A, lda. Cauchy fields: p, x, y, G, B.
 * Outputs piv/L/U as for the single-instance calls (device pointers). */
typedef struct {
    int32_t kind;           /* RPLU_JOB_DENSE or RPLU_JOB_CAUCHY               */
    int32_t dtype;          /* rplu_dtype                                      */
    int64_t n, m;
    void* A;                /* dense input, overwritten by S^(rank)            */
    int64_t lda;
    int32_t p;              /* Cauchy displacement rank                        */
    uint32_t flags;         /* RPLU_FLAG_STALL_STOP and RPLU_FLAG_REFRESH
                               honoured; RPLU_FLAG_C2PLU rejected
                               (RPLU_E_ARG); others ignored                   */
    const void* x;          /* Cauchy nodes and generators                     */
    const void* y;
    void* G;
    void* B;
    int32_t* piv;           /* outputs                                         */
    void* L;
    int64_t ldl;
    void* U;
    int64_t ldu;
    int64_t max_rank;
    double rel_tol;
    uint64_t seed;
    uint64_t stream;
    const void* A_orig;     /* dense, RPLU_FLAG_REFRESH: the unmodified input
                               (lda_orig >= m); the server uses A itself      */
    int64_t lda_orig;
    void* ready_event;      /* server: a hipEvent_t recorded (on the
                               submitter's stream) after the job's inputs are
                               written; the admission copy waits for it. NULL:
                               the inputs are ready at submit. It must stay
                               valid until poll stops returning RPLU_PENDING. */
} rplu_job;

/* Batched launch configuration. None of these fields changes the arithmetic:
 * an instance's reduction order depends only on its shape, so every
 * configuration returns bitwise the same results.
 *   rows_per_pass  rows one wave sweeps at once: 1, 2, 4, 8
 *   wg_per_cu      resident workgroups per compute unit (grid = CUs x this,
 *                  at most the number of jobs), 1..8 within occupancy
 *   order          queue order: RPLU_ORDER_AREA (n*m descending, the default),
 *                  RPLU_ORDER_CUBE (n*m*kmax descending), RPLU_ORDER_GIVEN
 * A field left 0 takes the tuned (or default) value. */
enum { RPLU_ORDER_AREA = 1, RPLU_ORDER_CUBE = 2, RPLU_ORDER_GIVEN = 3 };
typedef struct {
    int32_t rows_per_pass;
    int32_t wg_per_cu;
    int32_t order;
    int32_t reserved;
} rplu_batch_cfg;

/* Runs `count` dense jobs (host array `jobs`) in ONE persistent launch: every
 * workgroup takes instances from a device work queue (largest estimated cost
 * first) and runs each instance's whole step loop with workgroup barriers
 * (Alg. 1 with two-stage sampling, Sec. 4.1). R32 or R64 jobs only, all of
 * one dtype, 1 <= n, m <= 8192, and n * (12 + element size) bytes of LDS
 * per workgroup; piv is required, L and U may be NULL; max_rank, rel_tol,
 * seed and stream are per job. Results are bitwise those of rplu_dense on each
 * job alone (for finite data; rows already pivoted are skipped, which leaves
 * their exact zeros unchanged). infos_host: count entries, each with its own status; the call
 * returns RPLU_OK, or the status of the first failing job (by index).
 *
 * rplu_batched picks the configuration from the context's tuning table,
 * keyed by (dtype, count, largest n and m, mean n*m) rounded to powers of
 * two; on the first call with a new key it runs rplu_batched_tune first.
 * Tuning runs candidate configurations on device copies of the inputs (every
 * job, or a cost-stratified subset when the copies would exceed 8 GiB or a
 * quarter of free device memory), so the caller's buffers are untouched
 * until the real run. */
rplu_status rplu_batched(rplu_ctx ctx, int64_t count, const rplu_job* jobs,
                         rplu_info* infos_host, void* hip_stream);
/* Same with an explicit configuration (NULL = as rplu_batched). */
rplu_status rplu_batched_ex(rplu_ctx ctx, int64_t count, const rplu_job* jobs,
                            rplu_info* infos_host, const rplu_batch_cfg* cfg,
                            void* hip_stream);
/* Autotuner: times the candidate configurations on copies of the jobs (inputs
 * are not modified), stores the fastest in the context's table and returns it
 * in best_out; best_ms_out (may be NULL) gets its device time. */
rplu_status rplu_batched_tune(rplu_ctx ctx, int64_t count, const rplu_job* jobs,
                              rplu_batch_cfg* best_out, double* best_ms_out,
                              void* hip_stream);

/* ------------------------------------------------------------- server */

/* Continuous-batching server for arriving dense and Cauchy-like jobs.
 *
 * Admission: submitted jobs wait in FIFO order; the head is admitted while
 * its footprint fits in the server's slot pool (one device allocation of
 * hbm_budget_bytes, sub-allocated first-fit) and fewer than max_slots jobs
 * are running. A job's footprint is everything it touches on the device
 * besides its read-only inputs: a work block (the copy of the input the run
 * overwrites: dense A, Cauchy G and B; the run's workspace: step state,
 * masses, chunk totals, Cauchy split partials; the certification partials)
 * and, when the server owns the outputs (job.piv == NULL), an output block
 * (piv, L, U of kmax steps), allocated at admission. The work block returns
 * to the pool when the job finishes, the output block at
 * rplu_server_release. The caller's inputs are never modified.
 * Execution, overlapping on the device:
 *   - step-level batching: every admitted dense R32/R64 job with n, m <=
 *     batch_max_dim joins the resident set of the tick thread; each tick is
 *     one launch of the batched kernel over all resident jobs, advancing
 *     each by up to tick_steps steps (a job pauses at a step boundary and
 *     resumes in the next tick), so an arriving job starts at the next step
 *     boundary and a finished one leaves at once;
 *   - `workers` threads, each with its own stream, run larger dense jobs
 *     and Cauchy-like jobs alone (rplu_dense / rplu_cauchy steps, plain
 *     launches).
 * A job's results are those it gets alone (rplu_dense / rplu_cauchy, bit for
 * bit): the batched kernel reproduces rplu_dense, pauses change no bit, slots
 * keep each input's row pitch and 16-byte offset, and RPLU_FLAG_REFRESH acts
 * at the same step in both. Honoured job flags: RPLU_FLAG_STALL_STOP,
 * RPLU_FLAG_REFRESH (dense R32/R64: the caller's A is the original),
 * RPLU_FLAG_CERTIFY (dense R32/R64). */
typedef struct {
    size_t hbm_budget_bytes;   /* slot pool size                               */
    int32_t max_slots;         /* most jobs running at once (<= 0: no limit)   */
    int32_t queue_capacity;    /* most jobs waiting; beyond -> RPLU_E_BUSY     */
    int32_t workers;           /* worker threads/streams (<= 0: 3)             */
    int32_t batch_max_dim;     /* dense R32/R64 jobs with n, m <= this go to
                                  the step ticks (<= 0: 2048; at most 8192)    */
    uint32_t flags;            /* RPLU_SERVER_SIMULATE                         */
    int32_t tick_steps;        /* steps per tick (<= 0: 32)                    */
} rplu_server_cfg;

/* Host-only mode for testing the queueing logic without a device: the pool is
 * host memory, no HIP call is made, inputs are not read. A worker job "runs"
 * for footprint / 1e10 seconds; a tick advances every resident job by
 * tick_steps steps and takes the sum of footprint * steps / kmax / 1e10
 * seconds. Jobs complete with rank kmax and RPLU_STOP_RANK. */
#define RPLU_SERVER_SIMULATE 1u

typedef struct {
    int64_t submitted, completed, rejected, queued, active;
    double p50_ms, p99_ms;             /* submit -> completion latency       */
    double p50_dense_ms, p99_dense_ms;
    double p50_cauchy_ms, p99_cauchy_ms;
    double busy_s;                     /* wall time with >= 1 admitted job   */
    size_t hbm_in_use;                 /* bytes of the pool held by blocks   */
    size_t hbm_peak;                   /* largest hbm_in_use so far          */
    int64_t ticks;                     /* batched step ticks launched        */
    int64_t tick_jobs;                 /* jobs completed through the ticks   */
    int64_t refreshes;                 /* residual replacements (ticks)      */
} rplu_server_stats_t;

typedef struct rplu_server_s* rplu_server;

/* ctx names the device (its workspace is not used; the tick thread and each
 * worker make their own context); it may be NULL with RPLU_SERVER_SIMULATE. */
rplu_status rplu_server_create(rplu_ctx ctx, const rplu_server_cfg* cfg,
                               rplu_server* out);
/* Non-blocking, thread-safe. Copies the descriptor and returns a ticket;
 * RPLU_E_BUSY when queue_capacity jobs are waiting, RPLU_E_ARG for a job that
 * can never be admitted (footprint above the pool) or is malformed.
 * Outputs: job.piv/L/U given (caller-owned, written by the run), or all three
 * NULL (server-owned, in the job's output block: rplu_server_outputs). The
 * job's input buffers must stay valid and unmodified until poll returns
 * something other than RPLU_PENDING; if they are written on a stream, record
 * job.ready_event after the writes (the admission copy waits for it). */
rplu_status rplu_server_submit(rplu_server srv, const rplu_job* job,
                               uint64_t* ticket);
/* RPLU_PENDING until the job finished; then its status (RPLU_OK or an error)
 * and info. A ticket with caller-owned outputs (or a failed job) is then
 * forgotten (a later poll: RPLU_E_ARG); one with server-owned outputs stays
 * until rplu_server_release. Thread-safe. */
rplu_status rplu_server_poll(rplu_server srv, uint64_t ticket, rplu_info* info);
/* Device pointers of a finished job's server-owned outputs: piv (2 kmax
 * int32), L (n x kmax column-major, *ldl = n), U (kmax x m row-major,
 * *ldu = m); valid until rplu_server_release. RPLU_PENDING while running. */
rplu_status rplu_server_outputs(rplu_server srv, uint64_t ticket, int32_t** piv, void** L,
                                int64_t* ldl, void** U, int64_t* ldu);
/* Returns a finished job's output block to the pool and forgets the ticket. */
rplu_status rplu_server_release(rplu_server srv, uint64_t ticket);
rplu_status rplu_server_stats(rplu_server srv, rplu_server_stats_t* out);
/* Drains every submitted job, stops the threads and frees the pool (outputs
 * not yet released go with it). */
rplu_status rplu_server_destroy(rplu_server srv);

/* -------------------------------------------------------- verification */

/* Check of a rank-k factorisation with FP64 matrix cores (off the step loop).
 * After k steps the residual is S = A - L U (eqs. residual_update and
 * approximation_update), so ||A - L U||_F is the approximation error and
 * ||A - L U - S||_F is zero up to rounding for a consistent L, U, S.
 * A: n x m row-major (lda >= m), the ORIGINAL matrix; L: n x k column-major
 * (ldl >= n); U: k x m row-major (ldu >= m); S: n x m row-major (lds >= m)
 * or NULL. R32 inputs are widened to FP64 before the products; every sum is
 * FP64 and its order is fixed, so repeated calls give the same bits. Nothing
 * is modified. Real dtypes (R32, R64) only. Blocks until out is filled. */
typedef struct {
    double a_fro2;          /* ||A||_F^2                                       */
    double err_fro2;        /* ||A - L U||_F^2                                 */
    double schur_gap_fro2;  /* ||A - L U - S||_F^2 (0 when S is NULL)          */
} rplu_verify_out;
rplu_status rplu_verify(rplu_ctx ctx, rplu_dtype dtype, int64_t n, int64_t m, int64_t k,
                        const void* A, int64_t lda, const void* L, int64_t ldl,
                        const void* U, int64_t ldu, const void* S, int64_t lds,
                        rplu_verify_out* out, void* hip_stream);

/* ------------------------------------------------------------- profiling */

/* Device time per kernel class, measured with HIP events recorded on the
 * caller's stream around every launch between rplu_profile_begin and
 * rplu_profile_end. While profiling is on, runs use plain launches (events
 * time individual kernels; a replayed graph cannot be timed per kernel).
 * Class 0: the hot kernel (dense sweep / Cauchy all-pairs mass / the batched
 * persistent kernel, queue reset included / the CUR form's pass over A),
 * 1: the pivot draws (with the kernels that produce their chunk totals: the
 * Cauchy-like row-mass reduction and pivot-row regeneration, the CUR form's
 * residual pivot row), 2: the Cauchy-like generator update, the dense
 * column-mass reduction, the CUR form's k-vector and core-update kernels,
 * 3: initial mass pass. */
#define RPLU_PROFILE_CLASSES 4
typedef struct {
    int64_t launches[RPLU_PROFILE_CLASSES];
    double ms[RPLU_PROFILE_CLASSES];
} rplu_profile;
rplu_status rplu_profile_begin(rplu_ctx ctx);
/* Synchronises with the recorded events and returns the sums. */
rplu_status rplu_profile_end(rplu_ctx ctx, rplu_profile* out);

const char* rplu_status_str(rplu_status s);
const char* rplu_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RPLU_H */
