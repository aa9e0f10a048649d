// Plain C++17 FP64 / complex128 oracle for Randomly Pivoted LU, with OpenMP
// over rows for the O(nm) passes.
//
// TEST INFRASTRUCTURE. Only tests, the smoke check and the bench's CPU
// baseline load this library; the product path never does, and it shares no
// code (no header, helper or constant table) with the HIP library.
//
// It follows the numpy oracle (oracle/rplu.py) step for step and computes the
// same thing (Gilles & Wilber, "Low-Rank Approximation by Randomly Pivoted
// LU"):
//   * Dense RPLU, Alg. 1, with two-stage exact sampling (Sec. 4.1): row i with
//     probability ||S_i,:||^2 / ||S||_F^2, then column j of that row with
//     probability |S_ij|^2 / ||S_i,:||^2; L(:,t) = S_:,j / S_ij with
//     L(i,t) = 1, U(t,:) = S_i,:, S <- S - L(:,t) U(t,:)
//     (eq. residual_update), row i and column j then set to exactly 0.
//   * Cauchy-like RPLU, Alg. 3 with exact row masses: entries
//     s_ij = (G_i,: B_:,j) / (x_i - y_j) (eq. cauchy-like), row masses
//     sum_j |G_i,: B_:,j|^2 / |x_i - y_j|^2 (Sec. 5.1, row-norm formula),
//     generator updates G <- G - (1/a) c G_i,:, B <- B - (1/a) B_:,j r
//     (eqs. generator_update_g, generator_update_b), G_i,: and B_:,j zeroed.
//   * C2PLU (complete 2-norm pivoting, Sec. 2.3.3) in place of the draws:
//     the first row of largest mass, then the first column of largest
//     |S_ij|^2 in it.
// Conventions (the readings the numpy oracle states): inclusive prefix sums
// left to right, T = the last prefix, the drawn index is the first whose
// prefix exceeds u*T; the column draw uses the pivot row's own total; the
// stop test before each draw is T == 0 -> EXHAUSTED, tol > 0 and
// T <= tol^2 T0 -> TOL, the optional stall rule, t == kmax -> RANK (or
// TOL_UNREACHED with tol > 0). Random numbers: Philox4x64-10 (Salmon et al.,
// SC'11) with key (seed, 0) and counter (t, stream, 0, 0), u = (w >> 11) 2^-53
// from words 0 (row) and 1 (column).
//
// Complex arrays are interleaved (re, im) doubles. Matrices are row-major;
// L is returned n x kmax column-major (column t at L + t n); U kmax x m
// row-major. Sums are plain left-to-right sums in FP64 (per row; OpenMP only
// splits rows among threads, so results do not depend on the thread count).
#include <omp.h>
#include <stdint.h>

#include <cmath>
#include <cstring>
#include <vector>

namespace {

constexpr int STOP_RANK = 1, STOP_TOL = 2, STOP_EXHAUSTED = 3, STOP_TOL_UNREACHED = 4,
              STOP_STALL = 5;
constexpr int ERR_NONFINITE = -4, ERR_ZERO_PIVOT = -7, ERR_ARG = -1;
constexpr int STALL_WINDOW = 64;
constexpr double STALL_RATIO = 63.0 / 64.0;
constexpr int TRACE_WORDS = 12;

// --- Philox4x64-10 from its published definition ---------------------------
void mulhilo(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
    const unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1,
            uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += W0; k1 += W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo(M0, c0, &hi0, &lo0);
        mulhilo(M1, c2, &hi1, &lo1);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double unit(uint64_t w) { return (double)(w >> 11) * 0x1p-53; }

void step_uniforms(uint64_t seed, uint64_t stream, int64_t t, double* u1, double* u2) {
    uint64_t w[4];
    philox((uint64_t)t, stream, 0, 0, seed, 0, w);
    *u1 = unit(w[0]);
    *u2 = unit(w[1]);
}

// --- inverse CDF and argmax ---------------------------------------------------
struct Draw {
    int64_t drawn = -1, used = -1;
    double total = 0, target = NAN, lo = NAN, hi = NAN;
};

// Inclusive prefix P of w (left to right), T = P[len-1]; drawn = the first
// idx with P[idx] > u T; lo/hi = the edges of the used index's bin.
Draw inverse_cdf(const double* w, int64_t len, double u, int64_t forced) {
    std::vector<double> P((size_t)len);
    double run = 0.0;
    for (int64_t q = 0; q < len; ++q) { run += w[q]; P[(size_t)q] = run; }
    Draw d;
    d.total = P[(size_t)len - 1];
    d.target = u * d.total;
    int64_t idx = 0;
    while (idx < len && !(P[(size_t)idx] > d.target)) ++idx;
    d.drawn = idx < len ? idx : -1;
    d.used = forced >= 0 ? forced : d.drawn;
    if (d.used >= 0 && d.used < len) {
        d.lo = d.used > 0 ? P[(size_t)d.used - 1] : 0.0;
        d.hi = P[(size_t)d.used];
    }
    return d;
}

Draw largest(const double* w, int64_t len, int64_t forced) {
    Draw d;
    int64_t best = 0;
    double sum = 0.0;
    for (int64_t q = 0; q < len; ++q) {
        sum += w[q];
        if (w[q] > w[best]) best = q;
    }
    d.drawn = best;
    d.used = forced >= 0 ? forced : best;
    d.total = sum;
    return d;
}

int stop_reason(int64_t t, double T, double T0, int64_t kmax, double tol, bool stall,
                double* T_best, int64_t* t_best) {
    if (T == 0.0) return STOP_EXHAUSTED;
    if (tol > 0.0 && T <= (tol * tol) * T0) return STOP_TOL;
    if (stall) {
        if (t == 0) { *T_best = T; *t_best = 0; }
        else if (T < STALL_RATIO * *T_best) { *T_best = T; *t_best = t; }
        if (t - *t_best >= STALL_WINDOW) return STOP_STALL;
    }
    if (t == kmax) return tol > 0.0 ? STOP_TOL_UNREACHED : STOP_RANK;
    return 0;
}

// complex helpers on (re, im) pairs
inline double mag2(double re, double im) { return re * re + im * im; }

// q = x / y for complex numbers by Smith's algorithm (R. L. Smith, "Algorithm
// 116: Complex division", CACM 1962).
inline void cdiv(double xr, double xi, double yr, double yi, double* qr, double* qi) {
    if (std::fabs(yr) >= std::fabs(yi)) {
        const double r = yi / yr, den = yr + yi * r;
        *qr = (xr + xi * r) / den;
        *qi = (xi - xr * r) / den;
    } else {
        const double r = yr / yi, den = yr * r + yi;
        *qr = (xr * r + xi) / den;
        *qi = (xi * r - xr) / den;
    }
}

void record_trace(double* tr, const Draw& rd, const Draw& cd, double are, double aim, int64_t i,
                  int64_t j) {
    tr[0] = rd.total; tr[1] = rd.target; tr[2] = rd.lo; tr[3] = rd.hi;
    tr[4] = cd.total; tr[5] = cd.target; tr[6] = cd.lo; tr[7] = cd.hi;
    tr[8] = are; tr[9] = aim; tr[10] = (double)i; tr[11] = (double)j;
}

int64_t kmax_of(int64_t n, int64_t m, int64_t k) {
    const int64_t mn = n < m ? n : m;
    return k <= 0 ? mn : (k < mn ? k : mn);
}

}  // namespace

extern "C" {

int ref_threads(void) { return omp_get_max_threads(); }

void ref_philox(uint64_t seed, uint64_t stream, int64_t t, uint64_t* out4) {
    philox((uint64_t)t, stream, 0, 0, seed, 0, out4);
}

// Dense RPLU (Alg. 1). S: n x m row-major (cplx: interleaved complex128),
// overwritten by the final Schur complement. forced: 2*kmax ints (i, j; a
// negative i draws freely at that step) or NULL. Outputs: piv (2*kmax), L
// (n x kmax column-major), U (kmax x m), trace (kmax x 12) and rowmass_out
// (kmax x n) may be NULL; res: rank, stop, T0, T. Returns 0 or an error
// (-4 non-finite, -7 zero forced pivot, -1 argument).
int ref_rplu_dense(int cplx, int64_t n, int64_t m, double* S, int64_t k, double tol,
                   uint64_t seed, uint64_t stream, int stall, int greedy, const int32_t* forced,
                   int32_t* piv, double* L, double* U, double* trace, double* rowmass_out,
                   int64_t* rank_out, int32_t* stop_out, double* T0_out, double* T_out) {
    if (n < 1 || m < 1 || S == nullptr) return ERR_ARG;
    const int64_t kmax = kmax_of(n, m, k);
    const int64_t cw = cplx ? 2 : 1;             // doubles per element
    std::vector<double> rowmass((size_t)n), wrow((size_t)m), l((size_t)(n * cw)),
        u((size_t)(m * cw));
    double T0 = 0.0, T = 0.0, T_best = 0.0;
    int64_t t_best = 0, t = 0;
    int stop = 0;
    for (;;) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            const double* r = S + i * m * cw;
            double s = 0.0;
            if (cplx) for (int64_t q = 0; q < m; ++q) s += mag2(r[2 * q], r[2 * q + 1]);
            else for (int64_t q = 0; q < m; ++q) s += r[q] * r[q];
            rowmass[(size_t)i] = s;
        }
        double run = 0.0;
        for (int64_t i = 0; i < n; ++i) run += rowmass[(size_t)i];
        T = run;
        if (!std::isfinite(T)) return ERR_NONFINITE;
        if (t == 0) T0 = T;
        stop = stop_reason(t, T, T0, kmax, tol, stall != 0, &T_best, &t_best);
        if (stop) break;
        if (rowmass_out) std::memcpy(rowmass_out + t * n, rowmass.data(), (size_t)n * 8);
        double u1, u2;
        step_uniforms(seed, stream, t, &u1, &u2);
        const int64_t fi = (forced && forced[2 * t] >= 0) ? forced[2 * t] : -1;
        const int64_t fj = (forced && forced[2 * t] >= 0) ? forced[2 * t + 1] : -1;
        if (fi >= n || fj >= m) return ERR_ARG;
        const Draw rd = greedy ? largest(rowmass.data(), n, fi) : inverse_cdf(rowmass.data(), n, u1, fi);
        const int64_t i = rd.used;
        const double* ri = S + i * m * cw;
        for (int64_t q = 0; q < m; ++q)
            wrow[(size_t)q] = cplx ? mag2(ri[2 * q], ri[2 * q + 1]) : ri[q] * ri[q];
        const Draw cd = greedy ? largest(wrow.data(), m, fj) : inverse_cdf(wrow.data(), m, u2, fj);
        const int64_t j = cd.used;
        const double are = ri[j * cw], aim = cplx ? ri[j * cw + 1] : 0.0;
        if (are == 0.0 && aim == 0.0) return ERR_ZERO_PIVOT;
        std::memcpy(u.data(), ri, (size_t)(m * cw) * 8);
        for (int64_t r = 0; r < n; ++r) {
            const double* e = S + (r * m + j) * cw;
            if (cplx) cdiv(e[0], e[1], are, aim, &l[(size_t)(2 * r)], &l[(size_t)(2 * r + 1)]);
            else l[(size_t)r] = e[0] / are;
        }
        l[(size_t)(i * cw)] = 1.0;
        if (cplx) l[(size_t)(2 * i + 1)] = 0.0;
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < n; ++r) {
            double* row = S + r * m * cw;
            if (cplx) {
                const double lr = l[(size_t)(2 * r)], li = l[(size_t)(2 * r + 1)];
                for (int64_t q = 0; q < m; ++q) {
                    const double ur = u[(size_t)(2 * q)], ui = u[(size_t)(2 * q + 1)];
                    row[2 * q] -= lr * ur - li * ui;
                    row[2 * q + 1] -= lr * ui + li * ur;
                }
            } else {
                const double lr = l[(size_t)r];
                for (int64_t q = 0; q < m; ++q) row[q] -= lr * u[(size_t)q];
            }
            row[j * cw] = 0.0;
            if (cplx) row[j * cw + 1] = 0.0;
        }
        std::memset(S + i * m * cw, 0, (size_t)(m * cw) * 8);
        if (L) std::memcpy(L + t * n * cw, l.data(), (size_t)(n * cw) * 8);
        if (U) std::memcpy(U + t * m * cw, u.data(), (size_t)(m * cw) * 8);
        if (piv) { piv[2 * t] = (int32_t)i; piv[2 * t + 1] = (int32_t)j; }
        if (trace) record_trace(trace + t * TRACE_WORDS, rd, cd, are, aim, i, j);
        ++t;
    }
    *rank_out = t;
    *stop_out = stop;
    *T0_out = T0;
    *T_out = T;
    return 0;
}

// Exact row masses of the Cauchy-like matrix (Sec. 5.1):
// out[i] = sum_j |G_i,: B_:,j|^2 / |x_i - y_j|^2, left to right in j.
void ref_cauchy_row_masses(int64_t n, int64_t m, int p, const double* x, const double* y,
                           const double* G, const double* B, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double xr = x[2 * i], xi = x[2 * i + 1];
        double s = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            double nr = 0.0, ni = 0.0;
            for (int l = 0; l < p; ++l) {
                const double gr = G[2 * (i * p + l)], gi = G[2 * (i * p + l) + 1];
                const double br = B[2 * (l * m + j)], bi = B[2 * (l * m + j) + 1];
                nr += gr * br - gi * bi;
                ni += gr * bi + gi * br;
            }
            const double dr = xr - y[2 * j], di = xi - y[2 * j + 1];
            s += mag2(nr, ni) / mag2(dr, di);
        }
        out[i] = s;
    }
}

// Cauchy-like RPLU (Alg. 3, exact masses). x (n), y (m) complex nodes; G n x p
// and B p x m row-major complex, overwritten with the final generators.
// mass_steps: kmax+1 flags (1 = compute the row masses at that step), or NULL
// for every step; a step without masses must be forced. Outputs as in
// ref_rplu_dense (L, U complex).
int ref_rplu_cauchy(int64_t n, int64_t m, int p, const double* x, const double* y, double* G,
                    double* B, int64_t k, double tol, uint64_t seed, uint64_t stream, int stall,
                    int greedy, const int32_t* forced, const uint8_t* mass_steps, int32_t* piv,
                    double* L, double* U, double* trace, double* rowmass_out, int64_t* rank_out,
                    int32_t* stop_out, double* T0_out, double* T_out) {
    if (n < 1 || m < 1 || p < 1) return ERR_ARG;
    const int64_t kmax = kmax_of(n, m, k);
    std::vector<double> rowmass((size_t)n), w((size_t)m), r((size_t)(2 * m)), c((size_t)(2 * n)),
        gi((size_t)(2 * p)), bj((size_t)(2 * p));
    double T0 = 0.0, T = NAN, T_best = 0.0;
    int64_t t_best = 0, t = 0;
    int stop = 0;
    // entry (a, b) of the current generators: (G_a,: B_:,b) / (x_a - y_b)
    auto entry = [&](int64_t a, int64_t b, double* er, double* ei) {
        double nr = 0.0, ni = 0.0;
        for (int l = 0; l < p; ++l) {
            const double gr = G[2 * (a * p + l)], gim = G[2 * (a * p + l) + 1];
            const double br = B[2 * (l * m + b)], bim = B[2 * (l * m + b) + 1];
            nr += gr * br - gim * bim;
            ni += gr * bim + gim * br;
        }
        cdiv(nr, ni, x[2 * a] - y[2 * b], x[2 * a + 1] - y[2 * b + 1], er, ei);
    };
    for (;;) {
        const bool need = mass_steps == nullptr || t == 0 || mass_steps[t] != 0;
        if (need) {
            ref_cauchy_row_masses(n, m, p, x, y, G, B, rowmass.data());
            double run = 0.0;
            for (int64_t i = 0; i < n; ++i) run += rowmass[(size_t)i];
            T = run;
            if (!std::isfinite(T)) return ERR_NONFINITE;
            if (t == 0) T0 = T;
            stop = stop_reason(t, T, T0, kmax, tol, stall != 0, &T_best, &t_best);
        } else {
            stop = (t == kmax) ? STOP_RANK : 0;
        }
        if (stop) break;
        double u1, u2;
        step_uniforms(seed, stream, t, &u1, &u2);
        const int64_t fi = (forced && forced[2 * t] >= 0) ? forced[2 * t] : -1;
        const int64_t fj = (forced && forced[2 * t] >= 0) ? forced[2 * t + 1] : -1;
        if (fi >= n || fj >= m) return ERR_ARG;
        if (!need && fi < 0) return ERR_ARG;
        Draw rd;
        if (need) {
            if (rowmass_out) std::memcpy(rowmass_out + t * n, rowmass.data(), (size_t)n * 8);
            rd = greedy ? largest(rowmass.data(), n, fi) : inverse_cdf(rowmass.data(), n, u1, fi);
        } else {
            rd.used = fi;
        }
        const int64_t i = rd.used;
        for (int64_t b = 0; b < m; ++b) {
            entry(i, b, &r[(size_t)(2 * b)], &r[(size_t)(2 * b + 1)]);
            w[(size_t)b] = mag2(r[(size_t)(2 * b)], r[(size_t)(2 * b + 1)]);
        }
        const Draw cd = greedy ? largest(w.data(), m, fj) : inverse_cdf(w.data(), m, u2, fj);
        const int64_t j = cd.used;
        const double are = r[(size_t)(2 * j)], aim = r[(size_t)(2 * j + 1)];
        if (are == 0.0 && aim == 0.0) return ERR_ZERO_PIVOT;
        for (int64_t a = 0; a < n; ++a) entry(a, j, &c[(size_t)(2 * a)], &c[(size_t)(2 * a + 1)]);
        for (int l = 0; l < p; ++l) {
            gi[(size_t)(2 * l)] = G[2 * (i * p + l)];
            gi[(size_t)(2 * l + 1)] = G[2 * (i * p + l) + 1];
            bj[(size_t)(2 * l)] = B[2 * (l * m + j)];
            bj[(size_t)(2 * l + 1)] = B[2 * (l * m + j) + 1];
        }
        // G <- G - (1/a) c G_i,:   and   B <- B - (1/a) B_:,j r
        for (int64_t a = 0; a < n; ++a)
            for (int l = 0; l < p; ++l) {
                double pr = c[(size_t)(2 * a)] * gi[(size_t)(2 * l)] - c[(size_t)(2 * a + 1)] * gi[(size_t)(2 * l + 1)];
                double pi = c[(size_t)(2 * a)] * gi[(size_t)(2 * l + 1)] + c[(size_t)(2 * a + 1)] * gi[(size_t)(2 * l)];
                double qr, qi;
                cdiv(pr, pi, are, aim, &qr, &qi);
                G[2 * (a * p + l)] -= qr;
                G[2 * (a * p + l) + 1] -= qi;
            }
        for (int l = 0; l < p; ++l)
            for (int64_t b = 0; b < m; ++b) {
                double pr = bj[(size_t)(2 * l)] * r[(size_t)(2 * b)] - bj[(size_t)(2 * l + 1)] * r[(size_t)(2 * b + 1)];
                double pi = bj[(size_t)(2 * l)] * r[(size_t)(2 * b + 1)] + bj[(size_t)(2 * l + 1)] * r[(size_t)(2 * b)];
                double qr, qi;
                cdiv(pr, pi, are, aim, &qr, &qi);
                B[2 * (l * m + b)] -= qr;
                B[2 * (l * m + b) + 1] -= qi;
            }
        for (int l = 0; l < p; ++l) {
            G[2 * (i * p + l)] = 0.0;
            G[2 * (i * p + l) + 1] = 0.0;
            B[2 * (l * m + j)] = 0.0;
            B[2 * (l * m + j) + 1] = 0.0;
        }
        if (L) {
            double* col = L + t * n * 2;
            for (int64_t a = 0; a < n; ++a)
                cdiv(c[(size_t)(2 * a)], c[(size_t)(2 * a + 1)], are, aim, &col[2 * a], &col[2 * a + 1]);
            col[2 * i] = 1.0;
            col[2 * i + 1] = 0.0;
        }
        if (U) std::memcpy(U + t * m * 2, r.data(), (size_t)(2 * m) * 8);
        if (piv) { piv[2 * t] = (int32_t)i; piv[2 * t + 1] = (int32_t)j; }
        if (trace) record_trace(trace + t * TRACE_WORDS, rd, cd, are, aim, i, j);
        ++t;
    }
    *rank_out = t;
    *stop_out = stop;
    *T0_out = T0;
    *T_out = T;
    return 0;
}

}  // extern "C"
