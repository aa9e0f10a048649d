// Pivot sampling (two-stage exact sampling, Sec. 4.1), shared by the dense
// and the Cauchy-like paths.
//
//   k_ct_vec       wide: chunk totals of a mass vector (the row masses)
//   k_sample_row   one workgroup: total T from the chunk totals, stop test,
//                  Philox draw u1, row i = first prefix > u1 T
//   (a wide kernel of each path then writes the pivot row into U(t,:) and
//    the chunk totals of |U(t,e)|^2)
//   k_sample_col   one workgroup: T_i, draw u2, column j, pivot a = U(t,j)
//                  and its FP64 reciprocal, pivot record and trace
//
// Step protocol on the device state: k_sample_row reads t, runs the stop
// test (setting done) or records cur = t and i; k_sample_col records j, a,
// 1/a and sets t = t + 1. Every later kernel of the step reads cur, i, j.
#include "common.hpp"
#include "cdf.hpp"
#include "launch.hpp"

namespace rplu {

__global__ __launch_bounds__(256) void k_ct_vec(const double* __restrict__ v, int len,
                                                double* __restrict__ ct,
                                                const StepState* __restrict__ st) {
    if (st->done) return;
    cdf_chunk_totals_wave(len, ct, [&](int e) { return v[e]; });
}

__global__ __launch_bounds__(CDF_THREADS) void k_sample_row(
    const double* __restrict__ rowmass, const double* __restrict__ ct, int n,
    StepState* __restrict__ st, uint64_t seed, uint64_t stream, int kmax, double tol2,
    int stall, const int32_t* __restrict__ forced, double* __restrict__ rowmass_out) {
    __shared__ CdfShared sh;
    __shared__ int s_flag;
    if (st->done) return;
    const int t = st->t;
    const int K = cdf_chunks(n);
    const double T = cdf_levels(sh, ct, K);
    if (threadIdx.x == 0) {
        int stop = 0, err = 0;
        const double T0 = (t == 0) ? T : st->T0;
        if (stall) {
            if (t == 0) { st->T_best = T; st->t_best = 0; }
            else if (T < RPLU_STALL_RATIO * st->T_best) { st->T_best = T; st->t_best = t; }
        }
        if (!isfinite(T)) err = RPLU_E_NONFINITE;
        else if (T == 0.0) stop = RPLU_STOP_EXHAUSTED;
        else if (tol2 > 0.0 && T <= tol2 * T0) stop = RPLU_STOP_TOL;
        else if (stall && t - st->t_best >= RPLU_STALL_WINDOW) stop = RPLU_STOP_STALL;
        else if (t >= kmax) stop = tol2 > 0.0 ? RPLU_STOP_TOL_UNREACHED : RPLU_STOP_RANK;
        st->T = T;
        if (t == 0) st->T0 = T;
        if (err || stop) { st->error = err; st->stop = stop; st->done = 1; }
        s_flag = (err || stop) ? 1 : 0;
    }
    __syncthreads();
    if (s_flag) return;
    if (rowmass_out != nullptr)
        for (int e = threadIdx.x; e < n; e += CDF_THREADS) rowmass_out[(int64_t)t * n + e] = rowmass[e];
    const Philox4 rnd = philox4x64_10((uint64_t)t, stream, 0, 0, seed, 0);
    const double tgt = unit_from_word(rnd.w[0]) * T;
    const CdfPick p = cdf_draw(sh, ct, K, n, [&](int e) { return rowmass[e]; }, tgt);
    if (threadIdx.x == 0) {
        const int i = forced ? forced[2 * t] : p.idx;
        if (i < 0 || i >= n) {
            st->error = RPLU_E_ARG;
            st->done = 1;
        } else {
            st->cur = t;
            st->i = i;
            st->row_tgt = tgt;
            st->row_lo = p.lo;
            st->row_hi = p.hi;
        }
    }
}

// P == 0: dense; P >= 1: Cauchy-like, whose generator update also needs
// copies of G_i,: and B_:,j taken before any generator changes.
template <class T, int P>
__global__ __launch_bounds__(CDF_THREADS) void k_sample_col(
    const T* __restrict__ U, int64_t ldu, const double* __restrict__ ct, int m,
    StepState* __restrict__ st, int32_t* __restrict__ piv, uint64_t seed, uint64_t stream,
    const int32_t* __restrict__ forced, double* __restrict__ trace,
    const cf64* __restrict__ G, const cf64* __restrict__ B) {
    __shared__ CdfShared sh;
    if (st->done) return;
    const int t = st->cur;
    const T* Ut = U + (int64_t)t * ldu;
    const int K = cdf_chunks(m);
    const double Ti = cdf_levels(sh, ct, K);
    const Philox4 rnd = philox4x64_10((uint64_t)t, stream, 0, 0, seed, 0);
    const double tgt = unit_from_word(rnd.w[1]) * Ti;
    CdfPick p{0, 0.0, 0.0};
    if (Ti > 0.0 && isfinite(Ti)) p = cdf_draw(sh, ct, K, m, [&](int e) { return Sc<T>::mag2(Ut[e]); }, tgt);
    if (threadIdx.x == 0) {
        const int j = forced ? forced[2 * t + 1] : p.idx;
        if (j < 0 || j >= m) {
            st->error = RPLU_E_ARG;
            st->done = 1;
            return;
        }
        const T a = Ut[j];
        const double a2 = Sc<T>::mag2(a);
        if (!(a2 > 0.0)) {
            st->error = isfinite(a2) ? RPLU_E_ZERO_PIVOT : RPLU_E_NONFINITE;
            st->done = 1;
            return;
        }
        const typename Sc<T>::W inv = winv(Sc<T>::widen(a));
        const int i = st->i;
        st->j = j;
        st->a_re = Sc<T>::re(a);
        st->a_im = Sc<T>::im(a);
        if constexpr (Sc<T>::cplx) { st->inv_re = inv.re; st->inv_im = inv.im; }
        else { st->inv_re = inv; st->inv_im = 0.0; }
        if constexpr (P > 0) {
            for (int l = 0; l < P; ++l) {
                const cf64 g = G[(int64_t)i * P + l];
                const cf64 b = B[(int64_t)l * m + j];
                st->gi[2 * l] = g.re; st->gi[2 * l + 1] = g.im;
                st->bj[2 * l] = b.re; st->bj[2 * l + 1] = b.im;
            }
        }
        piv[2 * t] = i;
        piv[2 * t + 1] = j;
        if (trace != nullptr) {
            double* tr = trace + (int64_t)t * RPLU_TRACE_WORDS;
            tr[0] = st->T; tr[1] = st->row_tgt; tr[2] = st->row_lo; tr[3] = st->row_hi;
            tr[4] = Ti; tr[5] = tgt; tr[6] = p.lo; tr[7] = p.hi;
            tr[8] = Sc<T>::re(a); tr[9] = Sc<T>::im(a);
            tr[10] = (double)i; tr[11] = (double)j;
        }
        st->t = t + 1;
    }
}

__global__ void k_state_init(StepState* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        StepState z{};
        *st = z;
    }
}

// ---------------------------------------------------------------- launchers

void launch_state_init(StepState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st);
}

void launch_ct_vec(const double* v, int64_t len, double* ct, StepState* st, hipStream_t s) {
    const int waves = cdf_chunks((int)len);
    hipLaunchKernelGGL(k_ct_vec, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, v, (int)len,
                       ct, st);
}

void launch_sample_row(const SampleArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_sample_row, dim3(1), dim3(CDF_THREADS), 0, s, a.rowmass, a.ct_row,
                       (int)a.n, a.st, a.seed, a.stream, (int)a.kmax, a.tol2, a.stall, a.forced,
                       a.rowmass_out);
}

template <class T, int P>
static void sample_col_t(const SampleArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_sample_col<T, P>), dim3(1), dim3(CDF_THREADS), 0, s, (const T*)a.U,
                       a.ldu, a.ct_col, (int)a.m, a.st, a.piv, a.seed, a.stream, a.forced,
                       a.trace, (const cf64*)a.G, (const cf64*)a.B);
}

void launch_sample_col(const SampleArgs& a, hipStream_t s) {
    if (a.p == 0) {
        switch (a.dtype) {
            case RPLU_R32: sample_col_t<float, 0>(a, s); break;
            case RPLU_R64: sample_col_t<double, 0>(a, s); break;
            case RPLU_C64: sample_col_t<cf32, 0>(a, s); break;
            case RPLU_C128: sample_col_t<cf64, 0>(a, s); break;
        }
    } else {
        switch (a.p) {
            case 1: sample_col_t<cf64, 1>(a, s); break;
            case 2: sample_col_t<cf64, 2>(a, s); break;
            case 3: sample_col_t<cf64, 3>(a, s); break;
            case 4: sample_col_t<cf64, 4>(a, s); break;
        }
    }
}

}  // namespace rplu
