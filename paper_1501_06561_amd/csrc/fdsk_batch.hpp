// Descriptors of the many-sketch persistent kernel (kernels_batch.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fdsk_kernels.hpp"

namespace fdsk {

constexpr int kBatchMaxRows = 256;    // buffer rows m supported by the batched kernel

// Per sketch, per call: input rows and the sketch's device workspace.
struct BatchDesc {
  const void* rows;      // n x d input rows of this call (device)
  int64_t stride;        // leading dimension of rows (elements)
  int64_t n;             // rows in this call
  int dt;                // input dtype
  int d, ldc, l, m, mp;
  RuleParams rp;
  double* C0;            // mp x ldc buffers (double-buffered rebuild)
  double* C1;
  double* G;             // mp x mp
  double* W;             // mp x mp (one-sided Jacobi)
  double* V;             // mp x mp eigenvectors (column-major)
  double* Ut;            // mp x mp rebuild operator
  double* lam;           // mp
  double* rownorm;       // mp
  DevStats* st;
  void* out;             // finalize: l x d output (device), leading dim ldb
  int64_t ldb;
  int out_dt;
  int pad;
};

// Per sketch state kept on the device between calls.
struct BatchState {
  int occ;    // occupied rows
  int cur;    // which buffer holds the sketch
  int new0;   // first row appended since the last ReduceRank
  int pad;
};

hipError_t launch_batch_run(const BatchDesc* descs, BatchState* states, const int* order, int nsk,
                            int* counter, int finalize, int grid, hipStream_t s);

}  // namespace fdsk
