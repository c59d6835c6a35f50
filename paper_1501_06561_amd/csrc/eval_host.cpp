// Host driver of the Section 1.1 error measures (sketch_error, fdsk_evaluate).
//
// Every number is computed by device kernels; the host only sequences
// launches, owns the workspace and copies the final scalars back.
//   1. ||A||_F^2 (FP64).
//   2. Operator for A^T A: dense d x d column Gram (method 0) or two passes
//      over A per product (method 1, matrix-free).
//   3. Lanczos with full reorthogonalisation (K = min(d, 256) steps) on A^T A
//      -> top-k Ritz values -> ||A - A_k||_F^2 = ||A||_F^2 - their sum.
//   4. The same on A^T A - B^T B -> largest and smallest eigenvalue ->
//      cov-err = max(|lmax|, |lmin|) / ||A||_F^2.
//   5. Eigenpairs of B B^T -> orthonormal row-space directions of B (largest
//      first) -> ||A V_k||_F^2 and ||A V_B||_F^2 -> both projection errors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "fdsk_eval.hpp"
#include "fdsk_kernels.hpp"
#include "fdsk_eval_api.hpp"

namespace fdsk {
namespace {

struct Arena {
  void* base = nullptr;
  size_t off = 0, cap = 0;
  ~Arena() {
    if (base) (void)hipFree(base);
  }
  template <class T>
  T* take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) / 256 * 256;
    T* p = reinterpret_cast<T*>(static_cast<char*>(base) + off);
    off += bytes;
    return p;
  }
};

size_t al(size_t bytes) { return (bytes + 255) / 256 * 256; }

}  // namespace

#define EVCHK(expr)                                   \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) {                           \
      *msg = #expr;                                   \
      return e_;                                      \
    }                                                 \
  } while (0)

// Lanczos on op() for K steps from a fixed start vector; returns the Ritz
// values' summary (ext: max, min, k largest) on the device.
template <class Op>
static hipError_t lanczos(Op op, int d, int K, int k, double* Q, double* y, double* h1, double* h2,
                          double* alpha, double* beta, double* T, int mpT, double* lamT,
                          double* VT, EigWork wk, double* ext, hipStream_t s, const char** msg) {
  EVCHK(eval_start_vector(Q, d, s));
  for (int j = 0; j < K; ++j) {
    EVCHK(op(Q + static_cast<int64_t>(j) * d, y));
    EVCHK(eval_lanczos_step(Q, d, j, y, h1, h2, alpha, beta, Q + static_cast<int64_t>(j + 1) * d,
                            1e-290, s));
  }
  EVCHK(hipMemsetAsync(T, 0, static_cast<size_t>(mpT) * mpT * sizeof(double), s));
  EVCHK(eval_build_tridiag(alpha, beta, K, T, mpT, s));
  EVCHK(launch_eig(T, K, mpT, lamT, VT, wk, s));
  EVCHK(eval_extremes(lamT, K, k, ext, s));
  return hipSuccess;
}

hipError_t evaluate_device(const void* A, int a_dt, int64_t n, int64_t lda, const double* B,
                           int64_t rows_b, int64_t ldb, int d, int k, int method, hipStream_t s,
                           EvalResult* res, const char** msg) {
  *msg = "";
  const int K = std::min(d, 256);
  const int mpT = (K + 31) / 32 * 32;
  const int lb = static_cast<int>(std::max<int64_t>(rows_b, 1));
  const int mpB = (lb + 31) / 32 * 32;
  const int ldcB = (d + 63) / 64 * 64;
  const int kk = std::max(0, std::min(k, d));
  const bool dense = (method == 0);
  const int64_t dd = static_cast<int64_t>(d) * d;
  const int T_ = (d + 31) / 32;
  const int ntiles = T_ * (T_ + 1) / 2;
  const int nsplit_max = dense ? std::max(1, std::min<int>(64, (1024 + ntiles - 1) / ntiles)) : 0;
  const int nz_max = 256;

  Arena ar;
  size_t need = 0;
  need += dense ? al(dd * 8) * (1 + nsplit_max) : 0;                // M, partials
  need += al(static_cast<size_t>(K + 1) * d * 8) + 3 * al(d * 8);    // Q, y, (tmp)
  need += 4 * al(static_cast<size_t>(K + 1) * 8);                    // h1 h2 alpha beta
  need += 5 * al(static_cast<size_t>(mpT) * mpT * 8) + al(mpT * 8);  // T, VT, W, S1, S2, lamT
  need += dense ? 0 : al(static_cast<size_t>(std::max<int64_t>(n, rows_b)) * 8) +
                          al(static_cast<size_t>(nz_max) * d * 8);
  need += 2 * al(static_cast<size_t>(mpB) * ldcB * 8);               // padded B, unused
  need += 6 * al(static_cast<size_t>(mpB) * mpB * 8) + al(mpB * 8) + al(mpB * 4);  // GB, part, VB, WB, S1, S2, lamB, perm
  need += al(static_cast<size_t>(mpB) * d * 8);                      // Vt
  need += al(4096 * 2 * 8) + al(64 * 8) + 4 * al(sizeof(DevStats)) + al(64) + al(64 * 4) + al(16 * 8);
  need += al(static_cast<size_t>(2 + std::max(kk, 1)) * 8) * 2;
  if (hipMalloc(&ar.base, need) != hipSuccess) {
    *msg = "evaluator workspace allocation failed";
    return hipErrorOutOfMemory;
  }
  ar.cap = need;
  double* M = dense ? ar.take<double>(dd) : nullptr;
  double* Mpart = dense ? ar.take<double>(dd * nsplit_max) : nullptr;
  double* Q = ar.take<double>(static_cast<size_t>(K + 1) * d);
  double* y = ar.take<double>(d);
  double* y2 = ar.take<double>(d);
  ar.take<double>(d);
  double* h1 = ar.take<double>(K + 1);
  double* h2 = ar.take<double>(K + 1);
  double* alpha = ar.take<double>(K + 1);
  double* beta = ar.take<double>(K + 1);
  double* T = ar.take<double>(static_cast<size_t>(mpT) * mpT);
  double* VT = ar.take<double>(static_cast<size_t>(mpT) * mpT);
  double* WT = ar.take<double>(static_cast<size_t>(mpT) * mpT);
  double* S1T = ar.take<double>(static_cast<size_t>(mpT) * mpT);
  double* S2T = ar.take<double>(static_cast<size_t>(mpT) * mpT);
  double* lamT = ar.take<double>(mpT);
  double* tvec = dense ? nullptr : ar.take<double>(std::max<int64_t>(n, rows_b));
  double* part = dense ? nullptr : ar.take<double>(static_cast<size_t>(nz_max) * d);
  double* Bp = ar.take<double>(static_cast<size_t>(mpB) * ldcB);
  ar.take<double>(static_cast<size_t>(mpB) * ldcB);
  double* GB = ar.take<double>(static_cast<size_t>(mpB) * mpB);
  double* GBpart = ar.take<double>(static_cast<size_t>(mpB) * mpB);
  double* VB = ar.take<double>(static_cast<size_t>(mpB) * mpB);
  double* WB = ar.take<double>(static_cast<size_t>(mpB) * mpB);
  double* S1B = ar.take<double>(static_cast<size_t>(mpB) * mpB);
  double* S2B = ar.take<double>(static_cast<size_t>(mpB) * mpB);
  double* lamB = ar.take<double>(mpB);
  int* perm = ar.take<int>(mpB);
  double* Vt = ar.take<double>(static_cast<size_t>(mpB) * d);
  double* mpart = ar.take<double>(4096 * 2);
  double* scal = ar.take<double>(64);
  DevStats* ds = ar.take<DevStats>(4);
  unsigned* bar = ar.take<unsigned>(16);
  int* rot = ar.take<int>(64);
  double* out = ar.take<double>(16);
  double* extA = ar.take<double>(2 + std::max(kk, 1));
  double* extM = ar.take<double>(2 + std::max(kk, 1));
  int* nrank = reinterpret_cast<int*>(scal + 32);
  EVCHK(hipMemsetAsync(ar.base, 0, ar.off, s));

  // Both eigensolves take the tridiagonal route (ordinary launches only).
  EigWork wkT{WT, bar, rot, ds, S1T, S2T, EIG_AUTO};

  // 1. ||A||_F^2
  EVCHK(eval_fro2(A, a_dt, lda, n, d, mpart, scal + 0, s));

  // 2-3. A^T A and its top-k eigenvalues.
  if (dense) {
    EVCHK(eval_colgram(A, a_dt, lda, n, d, 1.0, 0, M, Mpart, nsplit_max, s));
    auto opA = [&](const double* x, double* yy) { return eval_symv(M, d, x, yy, s); };
    EVCHK(lanczos(opA, d, K, kk, Q, y, h1, h2, alpha, beta, T, mpT, lamT, VT, wkT, extA, s, msg));
    // 4. M = A^T A - B^T B
    if (rows_b > 0) EVCHK(eval_colgram(B, 0, ldb, rows_b, d, -1.0, 1, M, Mpart, nsplit_max, s));
    auto opM = [&](const double* x, double* yy) { return eval_symv(M, d, x, yy, s); };
    EVCHK(lanczos(opM, d, K, kk, Q, y, h1, h2, alpha, beta, T, mpT, lamT, VT, wkT, extM, s, msg));
  } else {
    auto opA = [&](const double* x, double* yy) {
      return eval_gram_op(A, a_dt, lda, n, d, 1.0, 0, x, yy, tvec, part, nz_max, s);
    };
    EVCHK(lanczos(opA, d, K, kk, Q, y, h1, h2, alpha, beta, T, mpT, lamT, VT, wkT, extA, s, msg));
    auto opM = [&](const double* x, double* yy) {
      hipError_t e = eval_gram_op(A, a_dt, lda, n, d, 1.0, 0, x, yy, tvec, part, nz_max, s);
      if (e == hipSuccess && rows_b > 0)
        e = eval_gram_op(B, 0, ldb, rows_b, d, -1.0, 1, x, yy, tvec, part, nz_max, s);
      return e;
    };
    EVCHK(lanczos(opM, d, K, kk, Q, y, h1, h2, alpha, beta, T, mpT, lamT, VT, wkT, extM, s, msg));
  }
  (void)y2;

  // 5. B's row space, largest directions first.
  if (rows_b > 0) {
    EVCHK(hipMemsetAsync(Bp, 0, static_cast<size_t>(mpB) * ldcB * 8, s));
    EVCHK(hipMemcpy2DAsync(Bp, ldcB * 8, B, ldb * 8, static_cast<size_t>(d) * 8, rows_b,
                           hipMemcpyDeviceToDevice, s));
    EVCHK(launch_gram(Bp, ldcB, mpB, GBpart, 1, GB, s));
    EigWork wkB{WB, bar, rot, ds, S1B, S2B, EIG_AUTO};
    EVCHK(launch_eig(GB, lb, mpB, lamB, VB, wkB, s));
    EVCHK(eval_rowspace(lamB, VB, lb, mpB, B, ldb, d, 1e-12, perm, nrank, Vt, s));
    EVCHK(eval_proj_mass(A, a_dt, lda, n, d, Vt, nrank, kk, mpart, scal + 8, s));
  } else {
    EVCHK(hipMemsetAsync(scal + 8, 0, 2 * sizeof(double), s));
  }
  EVCHK(eval_fro2(B, 0, ldb, rows_b, d, mpart, scal + 1, s));
  EVCHK(eval_finish(extM, extA, kk, scal + 0, scal + 8, out, s));

  double host_out[6], host_sc[2];
  int host_rank = 0;
  DevStats hds{};
  EVCHK(hipMemcpyAsync(host_out, out, sizeof host_out, hipMemcpyDeviceToHost, s));
  EVCHK(hipMemcpyAsync(host_sc, scal, sizeof host_sc, hipMemcpyDeviceToHost, s));
  EVCHK(hipMemcpyAsync(&host_rank, nrank, sizeof host_rank, hipMemcpyDeviceToHost, s));
  EVCHK(hipMemcpyAsync(&hds, ds, sizeof hds, hipMemcpyDeviceToHost, s));
  EVCHK(hipStreamSynchronize(s));
  res->cov_err = host_out[0];
  res->proj_err_k = host_out[1];
  res->proj_full = host_out[2];
  res->lambda_max = host_out[3];
  res->lambda_min = host_out[4];
  res->tail_k = host_out[5];
  res->fro2_A = host_sc[0];
  res->fro2_B = host_sc[1];
  res->rank_b = host_rank;
  res->eig_unconverged = hds.eig_unconv;
  res->barrier_error = hds.bar_err;
  return hipSuccess;
}

}  // namespace fdsk
