// BLAS-1 launch interface (SCG vector work and conversions).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgfas {

enum { kOpGamma = 0, kOpBeta = 1, kOpAlpha = 2, kOpNorm2 = 3, kOpStore = 4 };

// All vectors are [nrhs][n]; partial sums live at partial[rhs * 1024 + block] and the SCG
// scalars at scal[rhs * 8 + k].
// second-stage reduction of one (or, for kOpBeta, two: partial and partial2) sums per rhs
void finish(int nblocks, int nrhs, const double* partial, const double* partial2, int op, double* scal, double* out,
            hipStream_t st, int pstride = 1024);
// p = z (first) or p = beta p + z, with the previous iteration's x += alpha p_old when x is set
template <typename T>
void pupdate(int64_t n, int nrhs, const T* z, T* p, T* x, const double* scal, int first, hipStream_t st);
// x += alpha p
template <typename T>
void xupdate(int64_t n, int nrhs, T* x, const T* p, const double* scal, hipStream_t st);
// y += (double)(x + alpha p)
void xupdate_acc(int64_t n, int nrhs, const float* x, const float* p, const double* scal, double* y, hipStream_t st);
// rout = rin - alpha q with sum rout^2 partials
template <typename T>
void cg_update(int64_t n, int nrhs, const T* rin, T* rout, const T* q, const double* scal, double* partial,
               int nblocks, hipStream_t st);
template <typename T>
void dot_partials(int64_t n, int nrhs, const T* a, const T* b, const T* c, double* partial, int nblocks,
                  hipStream_t st);
template <typename TI, typename TO>
void convert(int64_t n, const TI* x, TO* y, int accumulate, hipStream_t st);
void fill(int64_t n, double* y, double v, hipStream_t st);
// v -= mean(v) per right-hand side (vectors [nrhs][n]); partial: [nrhs][1024] scratch
void project_mean(int64_t n, int nrhs, double* v, double* partial, hipStream_t st);
void mask_mul(int64_t n, double* y, const double* m, hipStream_t st);   // y *= m
void fill(int64_t n, float* y, float v, hipStream_t st);

}  // namespace dgfas
