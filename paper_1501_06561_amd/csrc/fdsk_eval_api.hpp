// Host-side entry of the device evaluator (see eval_host.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdsk {

struct EvalResult {
  double cov_err, proj_err_k, proj_full, lambda_max, lambda_min, tail_k, fro2_A, fro2_B;
  int rank_b, eig_unconverged, barrier_error;
};

// A: n x d (dtype a_dt, leading dim lda) and B: rows_b x d FP64 (ldb), both on
// the device.  method 0 = dense d x d operator, 1 = matrix-free.
hipError_t evaluate_device(const void* A, int a_dt, int64_t n, int64_t lda, const double* B,
                           int64_t rows_b, int64_t ldb, int d, int k, int method, hipStream_t s,
                           EvalResult* res, const char** msg);

}  // namespace fdsk
