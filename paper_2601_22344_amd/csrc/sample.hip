// Pivot sampling (two-stage exact sampling, Sec. 4.1): the step state and
// the wide row draw over a stored mass vector (pivot.hpp has the pieces).
//
//   k_state_init   zeroes the step state (t = 0, not done, counter 0)
//   k_rows_draw    wide: chunk totals of the row masses; the last workgroup
//                  takes the total T, runs the stop test and draws the row
//                  i = first prefix > u1 T with u1 from the Philox stream
//
// Step protocol on the device state: the row draw reads t, runs the stop
// test (setting done) or records cur = t and i; the column draw (a kernel of
// each path, after the pivot row is in U(t,:)) records j, a, 1/a and sets
// t = t + 1. Every later kernel of the step reads cur, i, j.
#include "common.hpp"
#include "cdf.hpp"
#include "launch.hpp"
#include "pivot.hpp"

namespace rplu {

__global__ __launch_bounds__(CDF_THREADS) void k_rows_draw(PivotArgs pa, double* __restrict__ ct) {
    __shared__ WideShared sh;
    if (pa.st->done) return;
    const int t = pa.st->t;
    const StopInputs in = stop_inputs(pa.st);
    wide_keep_words(sh, step_words(pa, t));
    const int e = blockIdx.x * WIDE_ELEMS + threadIdx.x;
    wide_chunk_totals(sh, e < pa.n ? pa.rowmass[e] : 0.0, pa.n, ct);
    if (!wide_arrive_last(sh, &pa.st->arrive)) return;
    pivot_row_draw_ct(sh.cdf, &sh.flag, pa, ct, t, wide_words(sh), in, RowMassGlobal{pa.rowmass});
}

__global__ void k_state_init(StepState* st, int refresh_on) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        StepState z{};
        z.refresh_on = refresh_on;
        *st = z;
    }
}

// After a residual replacement at step t (RPLU_FLAG_REFRESH): the run goes
// on from t with the stall window and the replacement reference restarted
// (inf: the next stop test records its total, at step t); refresh_on = 0
// once no replacement is left.
__global__ void k_state_resume(StepState* st, int refresh_on) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->done = 0;
        st->stop = 0;
        st->T_best = __builtin_inf();
        st->t_best = st->t;
        st->T_ref = __builtin_inf();
        st->refresh_on = refresh_on;
        st->t_base = st->t;             // the replaced S is S^(t) in memory
        st->flushed = st->t;
        st->arrive = 0;
    }
}

// ---------------------------------------------------------------- launchers

void launch_state_resume(StepState* st, int refresh_on, hipStream_t s) {
    hipLaunchKernelGGL(k_state_resume, dim3(1), dim3(64), 0, s, st, refresh_on);
}

void launch_state_init(StepState* st, hipStream_t s, int refresh_on) {
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st, refresh_on);
}

void launch_rows_draw(const SampleArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_rows_draw, dim3(wide_blocks(a.n)), dim3(CDF_THREADS), 0, s,
                       pivot_args(a), a.ct_row);
}

}  // namespace rplu
