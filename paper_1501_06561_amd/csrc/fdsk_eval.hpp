// Launchers of the error-evaluation kernels (covariance and projection error).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdsk {

hipError_t eval_colgram(const void* X, int dt, int64_t ldx, int64_t rows, int d, double sign,
                        int accumulate, double* M, double* ws, int nsplit_max, hipStream_t s);
hipError_t eval_symv(const double* M, int d, const double* x, double* y, hipStream_t s);
hipError_t eval_gram_op(const void* X, int dt, int64_t ldx, int64_t rows, int d, double sign,
                        int accumulate, const double* x, double* y, double* t, double* part,
                        int nz_max, hipStream_t s);
hipError_t eval_lanczos_step(const double* Q, int d, int j, double* y, double* h1, double* h2,
                             double* alpha, double* beta, double* qnext, double floor_abs,
                             hipStream_t s);
hipError_t eval_build_tridiag(const double* alpha, const double* beta, int K, double* T, int ldt,
                              hipStream_t s);
hipError_t eval_extremes(const double* v, int n, int k, double* out, hipStream_t s);
hipError_t eval_fro2(const void* X, int dt, int64_t ldx, int64_t rows, int d, double* part,
                     double* out, hipStream_t s);
hipError_t eval_rowspace(const double* lam, const double* U, int l, int mp, const double* B,
                         int64_t ldb, int d, double rtol, int* perm, int* nrank, double* Vt,
                         hipStream_t s);
hipError_t eval_proj_mass(const void* X, int dt, int64_t ldx, int64_t rows, int d, const double* Vt,
                          const int* nrank, int k, double* part, double* out2, hipStream_t s);
hipError_t eval_start_vector(double* q, int d, hipStream_t s);
hipError_t eval_finish(const double* ext_M, const double* ext_A, int k, const double* fro2A,
                       const double* mass, double* out, hipStream_t s);

}  // namespace fdsk
