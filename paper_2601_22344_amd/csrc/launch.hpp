// Host-side launch descriptors and launchers of the RPLU kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rplu.h"

namespace rplu {

struct StepState;

// Rows per workgroup of the dense sweep (row masses only / with column masses).
constexpr int DENSE_ROWS = 8;
constexpr int DENSE_ROWS_COLMASS = 16;

struct DenseArgs {
    int dtype;
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

void launch_state_init(StepState* st, hipStream_t s);
void launch_dense_sweep(const DenseArgs& a, bool init, hipStream_t s);
void launch_dense_sample(const DenseArgs& a, hipStream_t s);
void launch_colmass_reduce(const DenseArgs& a, bool after_step, hipStream_t s);
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
    int splits;
    double* rowmass;     // n (reduced masses, written by the sampler)
    double* rowmass_out;
    double* trace;
    const int32_t* forced;
    uint64_t seed, stream;
    int64_t kmax;
    double tol2;
};

void launch_cauchy_mass(const CauchyArgs& a, hipStream_t s);
void launch_cauchy_sample(const CauchyArgs& a, hipStream_t s);
void launch_cauchy_update(const CauchyArgs& a, hipStream_t s);
int cauchy_rows_per_block();

}  // namespace rplu
