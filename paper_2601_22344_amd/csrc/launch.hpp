// Host-side launch descriptors and launchers of the RPLU kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "rplu.h"

namespace rplu {

struct StepState;

// Rows and threads per workgroup of the dense sweep (row masses only / with
// column masses, whose per-row-block partials favour taller blocks).
constexpr int DENSE_ROWS = 4;
constexpr int DENSE_THREADS = 512;
constexpr int DENSE_ROWS_COLMASS = 16;
constexpr int DENSE_THREADS_COLMASS = 256;
constexpr int DENSE_LAZY_ROWS = 4;        // rows per workgroup of the deferred sweep

// Deferred ("lazy") dense sweep: S in memory is written back every LAZY_B
// steps; in between each sweep reads it and applies the pending rank-1
// updates in registers in the eager sweep's order (dense.hip).
constexpr int LAZY_B = RPLU_LAZY_STEPS;

struct DenseArgs {
    int dtype;
    int lazy;            // deferred sweep (needs L and U stored, ldu >= m)
    int64_t n, m;
    void* S;
    int64_t lda;
    void* U;             // U rows (caller's U, or a one-row workspace with ldu = 0)
    int64_t ldu;
    void* L;             // may be null
    int64_t ldl;
    int32_t* piv;
    StepState* st;
    double* rowmass;     // n
    double* rowmax;      // n: largest |S_ij|^2 of each row (RPLU_FLAG_CPLU), or null
    double* ct_col;      // chunk totals of the pivot row's masses
    double* colpart;     // ceil(n / DENSE_ROWS_COLMASS) * m, when colmass
    bool colmass;
    bool vec_ok;         // 16-byte packs are aligned for S and U
    double* colmass_out;
    double* rowmass_out;
    double* trace;
    const int32_t* forced;
    uint64_t seed, stream;
    int64_t kmax;
    double tol2;
};

// The one-launch step of small dense runs (dense.hip, k_dense_step): n and
// m limit, and rows swept per workgroup.
constexpr int DENSE_STEP_MAX = 1024;
constexpr int DENSE_STEP_ROWS = 4;

struct SampleArgs;
struct DenseStepArgs {
    StepState* states;   // one private step state per workgroup (slot 0 is read back)
    double* masses;      // 2 x n: the row masses of steps t (slot t mod 2) and t + 1
    void* urows;         // workgroups 1..: their own copy of the pivot row (ldur)
    int64_t ldur;
    uint8_t* dead;       // n: row already pivoted (its owner no longer sweeps it)
    int groups;          // workgroups: ceil(n / DENSE_STEP_ROWS)
};
void launch_dense_step_init(const DenseArgs& a, const DenseStepArgs& d, hipStream_t s);
void launch_dense_step(const DenseArgs& a, const SampleArgs& sa, const DenseStepArgs& d,
                       hipStream_t s);
void launch_dense_step_finish(const DenseArgs& a, const DenseStepArgs& d, hipStream_t s);

// n and m limit of the fused one-workgroup pivot draw of the dense path
// (pivot.hpp); above it the draws run as wide kernels. Measured on MI355X:
// per step the fused draw takes 15.7 us against 18.8 at 512^2 and 20.3
// against 22.3 at 8192^2, the wide one 24.4 against 25.3 at 16384^2 and
// 25.2 against 31.9 at 32768^2.
constexpr int PIVOT_FUSED_MAX = 12288;

// Pivot sampling (sample.hip), shared by both forms.
struct SampleArgs {
    int dtype;           // element type of U
    int p;               // 0: dense; >= 1: Cauchy-like displacement rank
    int64_t n, m;
    const double* rowmass;
    const double* rowmax;   // greedy == 2: largest |S_ij|^2 of each row
    double* ct_row;      // chunk totals of the row masses
    double* ct_col;      // chunk totals of the pivot row's masses
    StepState* st;
    int32_t* piv;
    void* U;
    int64_t ldu;
    const void* G;       // Cauchy: generators (copies of G_i,: and B_:,j)
    const void* B;
    uint64_t seed, stream;
    int64_t kmax;
    double tol2;
    int stall;           // RPLU_FLAG_STALL_STOP
    const int32_t* forced;
    double* trace;
    double* rowmass_out;
    int fused;           // dense: one fused pivot kernel per step (n, m <= PIVOT_FUSED_MAX)
    int maxmass;         // RPLU_FLAG_MAXMASS_STOP: tolerance on the largest row mass
    int greedy;          // 1: C2PLU, the largest masses instead of the draws;
                         // 2: CPLU, the row of the largest entry (rowmax), then
                         // the largest entry of that row
};

void launch_state_init(StepState* st, hipStream_t s, int refresh_on = 0);
void launch_state_resume(StepState* st, int refresh_on, hipStream_t s);
void launch_rows_draw(const SampleArgs& a, hipStream_t s);

void launch_dense_sweep(const DenseArgs& a, bool init, hipStream_t s);
// Deferred sweep: S^(st->t) written back after the run if the last
// write-back is older (no-op for the eager sweep).
void launch_dense_flush(const DenseArgs& a, hipStream_t s);
void launch_dense_pivrow_draw(const DenseArgs& a, const SampleArgs& sa, hipStream_t s);
void launch_colmass_reduce(const DenseArgs& a, bool after_step, hipStream_t s);
// Row st->t of out (ld_out per row, rows below rows_cap) = sum over b in
// order of part[b][0..m); skipped once the run is done.
void launch_colmass_sum(const double* part, int nb, int64_t m, StepState* st, double* out,
                        int64_t ld_out, int64_t rows_cap, hipStream_t s);
void launch_dense_pivot(const DenseArgs& a, const SampleArgs& sa, hipStream_t s);
int dense_row_block(bool colmass);

struct CauchyArgs {
    int64_t n, m;
    int p;
    const void* x;
    const void* y;
    void* G;
    void* B;
    void* U;
    int64_t ldu;
    void* L;
    int64_t ldl;
    int32_t* piv;
    StepState* st;
    double* partial;     // splits * n
    void* mcol;          // p = 1: per-column data of the mass kernel (m entries)
    void* mframe;        // p = 1: the bounding box of y and its centre
    int splits;
    int cols_per_split;  // columns of y per workgroup column of the mass kernel
    double* rowmass;     // n (reduced masses)
    double* ct_col;      // chunk totals of the regenerated pivot row
    double* colmass_out; // column masses per step (RPLU_FLAG_COLMASS), or null;
                         // part of the graph-cache key like every pointer here
    double* trace;
    const int32_t* forced;
    uint64_t seed, stream;
    int64_t kmax;
    double tol2;
};

struct BoundsPlan;
struct HostBoundsPlan;
// Copies a host bound plan into dev (bounds_plan_bytes bytes) on stream s;
// staging holds host data the copies read (keep it until they have run).
hipError_t upload_bounds_plan(const HostBoundsPlan& P, int64_t n, int p, char* dev, hipStream_t s,
                              std::vector<int32_t>* staging, BoundsPlan* out);
// RPLU_FLAG_BOUNDS (cauchy_bounds.hip): the bounds u of the step, and the
// rejection loop after the trial-0 row draw.
void launch_bh_bounds(const BoundsPlan& bp, const CauchyArgs& a, hipStream_t s);
void launch_bh_reject(const BoundsPlan& bp, const CauchyArgs& a, const SampleArgs& sa,
                      hipStream_t s);
void launch_cauchy_frame(const CauchyArgs& a, hipStream_t s);
void launch_cauchy_transpose(const CauchyArgs& a, void* Gt, void* Bt, hipStream_t s);
void launch_cauchy_mass(const CauchyArgs& a, hipStream_t s);
size_t cauchy_mass_col_bytes(int p, int64_t m);
size_t cauchy_mass_frame_bytes(int p);
void launch_cauchy_reduce_draw(const CauchyArgs& a, const SampleArgs& sa, hipStream_t s);
void launch_cauchy_rowgen_draw(const CauchyArgs& a, const SampleArgs& sa, hipStream_t s);
void launch_cauchy_update(const CauchyArgs& a, hipStream_t s);
int cauchy_rows_per_block();

// RPLU in CUR form (cur.hip). W below is the FP64 form of the element type
// (double, or complex FP64 for complex inputs).
struct CurArgs {
    int dtype;
    int vec_ok;          // rows of A 16-byte aligned
    int64_t n, m, kmax;
    const void* A;       // n x m row-major (lda), read only
    int64_t lda;
    void* Uc;            // the core U_k (W), row-major, ldc
    int64_t ldc;
    void* Ut;            // its transpose (W), kmax x kmax
    void* C;             // A[:, J] row-major n x kmax, element type
    double* nrm;         // n row-norm estimates (the draws' row masses)
    uint8_t* selr;       // n: row selected
    uint8_t* selc;       // m: column selected
    void* rhat;          // m (W): the residual's pivot row
    void* l;             // m (W): rhat / rhat_j
    void* zv;            // kmax (W): A[i, J]
    void* zU;            // kmax (W): z^T U_k
    void* gI;            // kmax (W): (A conj(l))[I]
    void* wv;            // kmax (W): A[I, j]
    void* y;             // kmax (W): U_k gI
    void* Uw;            // kmax (W): U_k w
    double* l2part;      // cur_l_blocks(m) partial sums of |l|^2
    double* ct_col;
    int32_t* piv;
    StepState* st;
};

// The kernels of a step after the row draw, in four parts launched in this
// order: the pivot row and column draw (k_cur_zu, k_cur_pivrow_draw), the
// k-vectors (k_cur_l_gi, k_cur_core_mv), the pass over A (k_cur_sweep), the
// core update (k_cur_core_update).
enum { CUR_PART_PIVOT = 0, CUR_PART_VECTORS = 1, CUR_PART_SWEEP = 2, CUR_PART_CORE = 3 };
void launch_cur_part(const CurArgs& a, const SampleArgs& sa, int part, hipStream_t s);
int cur_l_blocks(int64_t m);

// Batched dense instances (batched.hip): one workgroup runs a whole instance.
constexpr int RPLU_BATCH_MAX_DIM = 8192;

struct BatchJob {
    void* A;             // n x m row-major, lda
    void* L;             // n x kmax col-major (ldl), or null
    void* U;             // kmax x m row-major (ldu), or null: a per-workgroup row
    int32_t* piv;        // 2 * kmax, or null (required when t0 > 0)
    int64_t lda, ldl, ldu;
    int32_t n, m, kmax;
    int32_t vec;         // 16-byte packs aligned for A and U (as rplu_dense decides)
    int32_t stall;       // RPLU_FLAG_STALL_STOP
    // Resumption (the server's step ticks): the run starts at step t0 on an A
    // that already holds S^(t0) (pivots 0..t0-1 in piv), with the original
    // total T0_in and the stall state (Tbest_in, tbest_in; Tbest_in < 0:
    // restart the stall window at t0), and pauses (stop 0) when it reaches
    // step t_end > t0 without another stop. t0 = t_end = 0: a whole run.
    int32_t t0, t_end;
    int32_t tbest_in;
    int32_t refresh_on;  // RPLU_FLAG_REFRESH with replacements left: stop with
                         // RPLU_STOP_REFRESH when T <= RPLU_REFRESH_DROP2 T_ref
    double Tbest_in, T0_in;
    double Tref_in;      // T_ref at t0 (< 0: take the total at t0)
    double tol2;
    uint64_t seed, stream;
};

struct BatchInfo {
    int64_t rank;
    int32_t stop, error;    // stop 0 and no error: paused at t_end
    double a_fro2, res_fro2;
    double T_best;          // stall and replacement state at the last stop test
    double T_ref;           // (for resumption)
    int32_t t_best, pad;
};

struct BatchLaunch {
    int dtype;           // RPLU_R32 or RPLU_R64
    int rows;            // rows per lane-group pass: 1, 2, 4 or 8
    int grid;            // resident workgroups
    int maxn;            // largest n in the batch (LDS rows)
    int count;
    const BatchJob* jobs;
    const int32_t* order;   // queue position -> job index
    int* queue;
    void* uscratch;      // grid rows of uscr_ld elements
    int64_t uscr_ld;
    BatchInfo* infos;
};

void launch_batched(const BatchLaunch& a, hipStream_t s);

// Factorisation check (verify.hip): ||A||^2, ||A - L U||^2, ||A - L U - S||^2.
struct VerifyArgs {
    int dtype;           // RPLU_R32 or RPLU_R64
    int64_t n, m, k;
    const void* A;
    int64_t lda;
    const void* L;       // n x k column-major (ldl)
    int64_t ldl;
    const void* U;       // k x m row-major (ldu)
    int64_t ldu;
    const void* S;       // n x m row-major (lds), or null
    int64_t lds;
    double* partial;     // verify_tiles(n, m) * 3
    double* out;         // 3
};
void launch_verify(const VerifyArgs& a, hipStream_t s);

// Residual replacement (verify.hip): S = A - L(:,0:t) U(0:t,:) formed in FP64
// with the matrix cores and rounded to the element type, every entry (the
// rows and columns of earlier pivots keep the rounding errors the stored
// factors leave there, so the total of S is the error of the factors).
struct RefreshArgs {
    int dtype;           // RPLU_R32 or RPLU_R64
    int64_t n, m, t;
    const void* A;       // the original matrix, lda
    int64_t lda;
    const void* L;       // n x >= t column-major (ldl)
    int64_t ldl;
    const void* U;       // >= t x m row-major (ldu)
    int64_t ldu;
    void* S;             // n x m row-major (lds), overwritten
    int64_t lds;
    const int32_t* piv;  // 2 t (unused)
};
void launch_refresh(const RefreshArgs& a, hipStream_t s);
int64_t verify_tiles(int64_t n, int64_t m);
size_t batched_lds_bytes(int dtype, int maxn);
constexpr size_t BT_STATIC_LDS = 8192;   // bound on k_batched's static LDS (checked there)
int batched_max_resident(int dtype, int rows, int maxn);

}  // namespace rplu
