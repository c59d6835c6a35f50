// Host-visible declarations of the device kernels' launchers and the small
// structs shared between the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <algorithm>

namespace fdsk {

// FP64 accumulators kept on the device (updated in stream order, no host sync).
struct DevStats {
  double fro2A;      // ||A||_F^2 of every appended row
  double Delta;      // sum of delta_i
  double Stot;       // squared mass removed by the ReduceRank rules
  long long n_rr;    // ReduceRank steps
  int nonfinite;     // a NaN/Inf reached the accumulators or the spectrum
  int bar_err;       // a grid barrier timed out
  int eig_unconv;    // eigensolves that hit their sweep cap
  int pad;
  unsigned long long eig_sweeps;  // Jacobi sweeps summed over eigensolves
};

// ReduceRank rule: delta = lambda_t (1-based t); indices < r are untouched;
// variant 1 (iSVD) keeps the first l-1 and zeroes the rest; variant 4
// (SpaceSaving Directions) moves lambda_{l-1} onto the l-th direction;
// keep = t-1 rows survive.
//
// comp != 0 turns the stage into Compensative FD's last step (Section 3.1):
// every one of the first l squared values is raised by the accumulated Delta
// and keep = l rows are written; comp = 1 applies the FD rule first (the
// reduction just run is re-evaluated from the same spectrum), comp = 2 takes
// the spectrum as it is.  Only the shrink total and fro2A are updated.
//
// mass != 0 (reduced-precision products): the shrink leaves the shrink total
// alone; it is measured instead as the buffer's squared Frobenius norm before
// the reduction minus that of the rebuilt rows, both in FP64 from the rows
// themselves (launch_row_mass / launch_mass_close), so that
// ||A||_F^2 - ||B||_F^2 equals it however far the approximate Gram's
// eigenvalues are off.
struct RuleParams {
  int variant;
  int l;
  int t;
  int r;
  int keep;
  int comp;
  int mass;
};

// Squared singular values at or below this fraction of the largest are
// treated as directions outside the buffer's row space.
constexpr double kNullRel = 1e-12;

hipError_t launch_ingest(const void* src, int dt, int64_t stride, int f, int d, double* C, int ldc,
                         int row0, double* rownorm, hipStream_t s);
// Split-K count of the single-buffer Gram when none is requested: enough
// K slices to give about 256 workgroups over ntiles output tiles, each slice
// at least 256 columns.
inline int gram_ksplit_default(int ntiles, int ldc) {
  int k = (256 + ntiles - 1) / ntiles;
  const int cap = ldc / 256 > 1 ? ldc / 256 : 1;
  return k < cap ? k : cap;
}
// Gram G = C C^T of an mp-row buffer: ksplit_req K slices (0: the default
// above), at most ksplit_max (Gpart holds ksplit_max mp x mp partials); the
// slice length is rounded up to the kernel's K step, which may lower the
// count.
hipError_t launch_gram(const double* C, int ldc, int mp, double* Gpart, int ksplit_max, double* G,
                       hipStream_t s, int ksplit_req = 0);
hipError_t launch_gram_reduce(const double* Gpart, int ksplit, int mp, double* G, hipStream_t s);
// BF16 matrix-core Gram / rebuild on the FP64 buffer; npass 1 = hi*hi,
// 3 = hi*hi + hi*lo + lo*hi (split-bf16 compensation), FP32 accumulation.
// bfw: workspace of bf16_workspace_bytes(mp, ldc) for the buffer's pre-split
// hi/lo halves (written by the Gram, read by the rebuild of the same
// ReduceRank), or null to split inside the products.
hipError_t launch_gram_lowp(const double* C, int ldc, int mp, double* Gpart, int ksplit_max, double* G,
                            int npass, void* bfw, hipStream_t s, int ksplit_req = 0);
size_t bf16_workspace_bytes(int mp, int ldc);
// The buffer's hi/lo bf16 halves into bfw (for a rebuild whose Gram did not
// write them: the FP8 path).
hipError_t launch_split_bf16(const double* C, int ldc, int mp, void* bfw, hipStream_t s);
// FP8 (e4m3) compensated Gram: per-row scaled hi/lo codes of C in q8
// (fp8_workspace_bytes), then three FP8 products per tile.
hipError_t launch_gram_fp8(const double* C, int ldc, int mp, void* q8, double* Gpart, int ksplit_max,
                           double* G, hipStream_t s, int ksplit_req = 0);
size_t fp8_workspace_bytes(int mp, int ldc);
// Rebuilds out[0:keep] = Ut[0:keep] C with rt (32 or 64) output rows per
// workgroup (the lowp path without pre-split halves always uses 32).
hipError_t launch_rebuild_lowp(const double* Ut, const double* C, int ldc, int mp, int keep, double* out,
                               int npass, const void* bfw, hipStream_t s, int rt = 32);
hipError_t launch_shrink(const double* lam, const double* V, int m, int mp, RuleParams rp,
                         const double* rownorm, int new0, int new1, double* Ut, DevStats* st,
                         hipStream_t s);
hipError_t launch_rebuild(const double* Ut, const double* C, int ldc, int mp, int keep, double* out,
                          hipStream_t s, int rt = 32);
hipError_t launch_zero_rows(double* C, int ldc, int r0, int r1, hipStream_t s);
// out[i] = ||C_i||^2 (FP64) for rows i < rows of a buffer with d columns.
hipError_t launch_row_mass(const double* C, int ldc, int rows, int d, double* out, hipStream_t s);
// st->Stot += sum(before[0:nb]) - sum(after[0:na]) (fixed order).
hipError_t launch_mass_close(const double* before, int nb, const double* after, int na, DevStats* st,
                             hipStream_t s);
hipError_t launch_add_pending_norms(const double* rownorm, int new0, int new1, DevStats* st,
                                    hipStream_t s);
hipError_t launch_merge_stats(DevStats* dst, const DevStats* src, const double* src_rownorm, int new0,
                              int new1, hipStream_t s);
// out (mp x mp) = in^T for the leading n x n block of an mp x mp matrix.
hipError_t launch_transpose(const double* in, int mp, int n, double* out, hipStream_t s);
// out (rows x d, ld d, FP64) = X converted from dtype dt (ld ldx).
hipError_t launch_convert_f64(const void* X, int dt, int64_t ldx, int64_t rows, int d, double* out,
                              hipStream_t s);
hipError_t launch_copy_out(const double* C, int ldc, int valid_rows, int l, int d, void* out,
                           int64_t ldb, int out_dt, hipStream_t s);

// Symmetric eigensolver for the m x m Gram matrix (G is mp x mp, zero padded).
// Output: lam[j] (j < m) and V column-major (column j = eigenvector j, ld mp,
// entries of rows >= m zero).  ws: workspace of eig_workspace_doubles(mp).
struct EigWork {
  double* W;        // mp x mp
  unsigned* bar;    // 2 counters (grid barrier)
  int* rot;         // per-sweep rotation counts (kMaxSweeps)
  DevStats* st;
  double* S1;       // mp x mp scratch (divide and conquer)
  double* S2;       // mp x mp scratch
  int method;       // EIG_AUTO or EIG_JACOBI
};
enum { EIG_AUTO = 0, EIG_JACOBI = 1 };
constexpr int kMaxSweeps = 40;
constexpr int kLdsEigMax = 100;   // single-workgroup solver limit (G and V in LDS)
constexpr int kTridMax = 200;     // back-transformation with the reflectors staged in LDS
constexpr int kTridGlobalMax = 1024; // tridiagonal route (packed triangle above 208 rows, the full
                                     // matrix in the S1 workspace above kTridLargeMin)
constexpr int kTridLargeMin = 256;   // orders above this reduce one column per two launches
constexpr int kBatchMax = 256;    // buffer rows of a batched sketch
constexpr int kDcMax = 1024;      // divide and conquer: O(n) state in LDS
// Eigen-decomposition of the symmetric m x m G (leading dimension mp): lam
// (m values, any order) and V (column j = eigenvector of lam[j], leading
// dimension mp).  m <= kTridGlobalMax goes through the tridiagonal route unless
// wk.method is EIG_JACOBI; larger m through the Jacobi solvers.
hipError_t launch_eig(const double* G, int m, int mp, double* lam, double* V, EigWork wk,
                      hipStream_t s);
hipError_t launch_eig_jacobi(const double* G, int m, int mp, double* lam, double* V, EigWork wk,
                             hipStream_t s);
hipError_t launch_eig_trid(const double* G, int m, int mp, double* lam, double* V, EigWork wk,
                           hipStream_t s);
// The three kernels of the tridiagonal route on their own (same arguments).
hipError_t launch_tridiag(const double* G, int m, int mp, EigWork wk, hipStream_t s);
// nvec: eigenvectors wanted (those of the nvec largest eigenvalues; the
// others are left undefined); m or less than 1 for all.
hipError_t launch_dc(int m, int mp, double* lam, double* V, EigWork wk, hipStream_t s, int nvec);
hipError_t launch_backtr(int m, int mp, double* V, EigWork wk, hipStream_t s);
// The message sketch_last_error(NULL) returns (entry points without a
// sketch object).
void set_last_error(const char* msg);

inline bool eig_uses_trid(int m, const EigWork& wk) {
  return wk.method != EIG_JACOBI && m <= kTridGlobalMax && wk.S1 && wk.S2;
}

}  // namespace fdsk
