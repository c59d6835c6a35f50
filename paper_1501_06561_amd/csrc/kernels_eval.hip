// Error measures of Section 1.1, evaluated on the device in FP64:
//   cov-err  = ||A^T A - B^T B||_2 / ||A||_F^2
//   proj-err = ||A - pi_{B_k}(A)||_F^2 / ||A - A_k||_F^2
//   ||A - pi_B(A)||_F^2 / ||A||_F^2
// The spectral norm and the top-k eigenvalues of A^T A come from Lanczos with
// full reorthogonalisation (dense d x d operator, or matrix-free passes over
// A); the small tridiagonal matrix is diagonalised by the library's Jacobi
// solver.  B's top right singular vectors come from the eigenpairs of B B^T.
#include "fdsk_device.hpp"
#include "fdsk_kernels.hpp"
#include "fdsk_eval.hpp"

namespace fdsk {

// ---------------------------------------------------------- column Gram
// Mpart[z] (d x d, lower 32x32 tiles) = sum over the z-th row range of X[r]^T X[r].
__global__ __launch_bounds__(256) void k_colgram(const void* __restrict__ X, int dt, int64_t ldx,
                                                 int64_t rows, int d, int64_t rchunk,
                                                 double* __restrict__ Mpart) {
  const int tile = blockIdx.x;
  int ti = static_cast<int>((sqrtf(8.0f * tile + 1.0f) - 1.0f) * 0.5f);
  while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
  while (ti * (ti + 1) / 2 > tile) --ti;
  const int tj = tile - ti * (ti + 1) / 2;
  const int64_t r0 = blockIdx.y * rchunk;
  const int64_t r1 = min(rows, r0 + rchunk);
  __shared__ double Xi[32][33];
  __shared__ double Xj[32][33];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w >> 1, wj = w & 1;
  const int li = lane & 15, lk = lane >> 4;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  const int ci0 = ti * 32, cj0 = tj * 32;
  for (int64_t rr = r0; rr < r1; rr += 32) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int idx = threadIdx.x + e * 256;
      int r = idx >> 5, c = idx & 31;
      int64_t row = rr + r;
      double vi = 0.0, vj = 0.0;
      if (row < r1) {
        if (ci0 + c < d) vi = load_as_f64(X, row * ldx + ci0 + c, dt);
        if (cj0 + c < d) vj = load_as_f64(X, row * ldx + cj0 + c, dt);
      }
      Xi[r][c] = vi;
      Xj[r][c] = vj;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < 8; ++k4) {
      double a = Xi[k4 * 4 + lk][wi * 16 + li];   // A[i][k] = X[r0+k][ci0+i]
      double b = Xj[k4 * 4 + lk][wj * 16 + li];   // B[k][j] = X[r0+k][cj0+j]
      acc = mfma_f64(a, b, acc);
    }
    __syncthreads();
  }
  const int64_t dd = static_cast<int64_t>(d);
  double* out = Mpart + static_cast<int64_t>(blockIdx.y) * dd * dd;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    int row = ci0 + wi * 16 + lk + 4 * v;
    int col = cj0 + wj * 16 + li;
    if (row < d && col < d) out[row * dd + col] = acc[v];
  }
}

// M (+)= sign * sum_z Mpart[z], lower triangle mirrored (fixed order).
__global__ void k_colgram_reduce(const double* __restrict__ Mpart, int nsplit, int d, double sign,
                                 int accumulate, double* __restrict__ M) {
  const int64_t dd = d;
  const int64_t n = dd * dd;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int r = static_cast<int>(e / d), c = static_cast<int>(e % d);
    if (r < c) continue;
    double v = 0.0;
    for (int z = 0; z < nsplit; ++z) v += Mpart[z * n + e];
    v *= sign;
    if (accumulate) v += M[e];
    M[e] = v;
    M[static_cast<int64_t>(c) * d + r] = v;
  }
}

// ------------------------------------------------------ Lanczos pieces
// y = M x for dense symmetric M (d x d); a wave per row.
__global__ __launch_bounds__(256) void k_symv(const double* __restrict__ M, int d,
                                              const double* __restrict__ x, double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= d) return;
  const double* mr = M + static_cast<int64_t>(row) * d;
  double s = 0.0;
  for (int c = lane; c < d; c += 64) s += mr[c] * x[c];
  s = wave_sum(s);
  if (lane == 0) y[row] = s;
}

// t[r] = X[r] . x for r < rows (a wave per row).
__global__ __launch_bounds__(256) void k_gemv_rows(const void* __restrict__ X, int dt, int64_t ldx,
                                                   int64_t rows, int d, const double* __restrict__ x,
                                                   double* __restrict__ t) {
  const int lane = threadIdx.x & 63;
  const int64_t row = blockIdx.x * 4LL + (threadIdx.x >> 6);
  if (row >= rows) return;
  double s = 0.0;
  for (int c = lane; c < d; c += 64) s += load_as_f64(X, row * ldx + c, dt) * x[c];
  s = wave_sum(s);
  if (lane == 0) t[row] = s;
}

// part[z][c] = sum over the z-th row range of X[r][c] * t[r].
__global__ __launch_bounds__(256) void k_gemv_cols(const void* __restrict__ X, int dt, int64_t ldx,
                                                   int64_t rows, int d, int64_t rchunk,
                                                   const double* __restrict__ t,
                                                   double* __restrict__ part) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= d) return;
  const int64_t r0 = blockIdx.y * rchunk;
  const int64_t r1 = min(rows, r0 + rchunk);
  double s = 0.0;
  for (int64_t r = r0; r < r1; ++r) s += load_as_f64(X, r * ldx + c, dt) * t[r];
  part[static_cast<int64_t>(blockIdx.y) * d + c] = s;
}

// y[c] = sign * sum_z part[z][c] (+ y[c] if accumulate).
__global__ void k_sum_parts(const double* __restrict__ part, int nz, int d, double sign,
                            int accumulate, double* __restrict__ y) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d) return;
  double s = 0.0;
  for (int z = 0; z < nz; ++z) s += part[static_cast<int64_t>(z) * d + c];
  s *= sign;
  y[c] = accumulate ? y[c] + s : s;
}

// h[i] = Q[i] . y for i < nq (one workgroup per i).
__global__ __launch_bounds__(256) void k_dots(const double* __restrict__ Q, int d, int nq,
                                              const double* __restrict__ y, double* __restrict__ h) {
  const int i = blockIdx.x;
  if (i >= nq) return;
  const double* q = Q + static_cast<int64_t>(i) * d;
  double s = 0.0;
  for (int c = threadIdx.x; c < d; c += 256) s += q[c] * y[c];
  __shared__ double red[4];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) h[i] = (red[0] + red[1]) + (red[2] + red[3]);
}

// y -= Q^T h over the first nq rows of Q.
__global__ void k_axpy_many(const double* __restrict__ Q, int d, int nq, const double* __restrict__ h,
                            double* __restrict__ y) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d) return;
  double s = y[c];
  for (int i = 0; i < nq; ++i) s -= h[i] * Q[static_cast<int64_t>(i) * d + c];
  y[c] = s;
}

// alpha[j] = h1[j] + h2[j]; beta[j] = ||y||; q_next = y / beta (0 if beta tiny).
__global__ __launch_bounds__(1024) void k_lanczos_close(const double* __restrict__ h1,
                                                        const double* __restrict__ h2, int j,
                                                        double* __restrict__ y, int d,
                                                        double* __restrict__ alpha,
                                                        double* __restrict__ beta,
                                                        double* __restrict__ qnext,
                                                        double scale_floor) {
  __shared__ double red[16];
  __shared__ double bsh;
  double s = 0.0;
  for (int c = threadIdx.x; c < d; c += blockDim.x) s += y[c] * y[c];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) t += red[w];
    double b = sqrt(t);
    alpha[j] = h1[j] + h2[j];
    beta[j] = b;
    bsh = b;
  }
  __syncthreads();
  const double b = bsh;
  const double inv = (b > scale_floor) ? 1.0 / b : 0.0;
  for (int c = threadIdx.x; c < d; c += blockDim.x) qnext[c] = y[c] * inv;
}

// Dense K x K tridiagonal T from alpha, beta (beta[j] couples j and j+1).
__global__ void k_build_tridiag(const double* __restrict__ alpha, const double* __restrict__ beta,
                                int K, double* __restrict__ T, int ldt) {
  const int64_t n = static_cast<int64_t>(K) * K;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int i = static_cast<int>(e / K), j = static_cast<int>(e % K);
    double v = 0.0;
    if (i == j) v = alpha[i];
    else if (j == i + 1) v = beta[i];
    else if (i == j + 1) v = beta[j];
    T[static_cast<int64_t>(i) * ldt + j] = v;
  }
}

// Summaries of n values: out[0] = max, out[1] = min, out[2 + i] = i-th largest (i < k).
__global__ __launch_bounds__(1024) void k_extremes(const double* __restrict__ v, int n, int k,
                                                   double* __restrict__ out) {
  __shared__ double vals[1024];
  for (int i = threadIdx.x; i < n; i += blockDim.x) vals[i] = v[i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double x = vals[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) rank += (vals[j] > x) || (vals[j] == x && j < i);
    if (rank == 0) out[0] = x;
    if (rank == n - 1) out[1] = x;
    if (rank < k) out[2 + rank] = x;
  }
}

// Squared Frobenius norm of X (rows x d), partial sums per block.
__global__ __launch_bounds__(256) void k_fro2_rows(const void* __restrict__ X, int dt, int64_t ldx,
                                                   int64_t rows, int d, double* __restrict__ part) {
  double s = 0.0;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x)
    for (int c = threadIdx.x; c < d; c += 256) {
      double v = load_as_f64(X, r * ldx + c, dt);
      s += v * v;
    }
  __shared__ double red[4];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_sum_scalar(const double* __restrict__ part, int n, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = s;
  }
}

// Rank the eigenvalues of B B^T (descending, NaN last): perm[q] = index of
// the q-th largest; *nrank = how many exceed rtol * largest.
__global__ __launch_bounds__(1024) void k_rank_desc(const double* __restrict__ lam, int l, double rtol,
                                                    int* __restrict__ perm, int* __restrict__ nrank) {
  __shared__ double lv[1024];
  __shared__ int cnt;
  for (int i = threadIdx.x; i < l; i += blockDim.x) {
    double x = lam[i];
    lv[i] = (x == x) ? x : -INFINITY;
  }
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  double top = -INFINITY;
  for (int i = 0; i < l; ++i) top = fmax(top, lv[i]);
  for (int i = threadIdx.x; i < l; i += blockDim.x) {
    double x = lv[i];
    int rank = 0;
    for (int j = 0; j < l; ++j) rank += (lv[j] > x) || (lv[j] == x && j < i);
    perm[rank] = i;
    if (top > 0.0 && x > rtol * top) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) *nrank = cnt;
}

// Vt[q] = B^T u_{perm[q]} / sqrt(lam_{perm[q]}) for q < nrank: orthonormal
// directions spanning B's row space, largest singular value first.
__global__ __launch_bounds__(256) void k_rowspace_vt(const double* __restrict__ lam,
                                                     const double* __restrict__ U, int mp,
                                                     const double* __restrict__ B, int64_t ldb,
                                                     int l, int d, const int* __restrict__ perm,
                                                     const int* __restrict__ nrank,
                                                     double* __restrict__ Vt) {
  const int q = blockIdx.x;
  if (q >= *nrank) return;
  const int col = perm[q];
  const double inv = 1.0 / sqrt(lam[col]);
  const double* u = U + static_cast<int64_t>(col) * mp;
  for (int c = threadIdx.x; c < d; c += 256) {
    double s = 0.0;
    for (int i = 0; i < l; ++i) s += B[i * ldb + c] * u[i];
    Vt[static_cast<int64_t>(q) * d + c] = s * inv;
  }
}

// part[2*blk] = sum over rows of sum_{q < k} (X[r] . Vt[q])^2 and
// part[2*blk+1] = the same over q < nrank (nrank read on the device).
__global__ __launch_bounds__(256) void k_proj_mass(const void* __restrict__ X, int dt, int64_t ldx,
                                                   int64_t rows, int d, const double* __restrict__ Vt,
                                                   const int* __restrict__ nrank, int k,
                                                   double* __restrict__ part) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nv = *nrank;
  double acc_k = 0.0, acc_all = 0.0;
  for (int64_t r = blockIdx.x * 4LL + w; r < rows; r += gridDim.x * 4LL) {
    for (int q = 0; q < nv; ++q) {
      const double* v = Vt + static_cast<int64_t>(q) * d;
      double s = 0.0;
      for (int c = lane; c < d; c += 64) s += load_as_f64(X, r * ldx + c, dt) * v[c];
      s = wave_sum(s);
      acc_all += s * s;
      if (q < k) acc_k += s * s;
    }
  }
  __shared__ double red[8];
  if (lane == 0) { red[w] = acc_k; red[4 + w] = acc_all; }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    part[2 * blockIdx.x + 1] = (red[4] + red[5]) + (red[6] + red[7]);
  }
}

__global__ void k_sum_pairs(const double* __restrict__ part, int n, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < n; ++i) { a += part[2 * i]; b += part[2 * i + 1]; }
    out[0] = a;
    out[1] = b;
  }
}

// Deterministic start vector (splitmix64 hash of the index, then normalised
// by the first Lanczos step's caller): q[c] in [-1, 1).
__global__ void k_start_vector(double* __restrict__ q, int d) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d) return;
  unsigned long long z = 0x9E3779B97F4A7C15ull * (static_cast<unsigned long long>(c) + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  q[c] = static_cast<double>(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ __launch_bounds__(1024) void k_normalize(double* __restrict__ q, int d) {
  __shared__ double red[16];
  __shared__ double inv;
  double s = 0.0;
  for (int c = threadIdx.x; c < d; c += blockDim.x) s += q[c] * q[c];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) t += red[w];
    inv = t > 0.0 ? 1.0 / sqrt(t) : 0.0;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < d; c += blockDim.x) q[c] *= inv;
}

// Report scalars from the device values: sc = [fro2A, fro2B, lmax, lmin,
// topk_sum(A^T A), mass_k, mass_all, nrank]; writes out[0..2] = cov-err,
// proj-err_k, proj-full / ||A||^2.
__global__ void k_finish_report(const double* __restrict__ ext_M, const double* __restrict__ ext_A,
                                int k, const double* __restrict__ fro2A,
                                const double* __restrict__ mass, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double fa = *fro2A;
  const double lmax = ext_M[0], lmin = ext_M[1];
  double topk = 0.0;
  for (int i = 0; i < k; ++i) topk += ext_A[2 + i];
  const double tail = fa - topk;
  out[0] = fmax(fabs(lmax), fabs(lmin)) / fa;
  out[1] = (fa - mass[0]) / tail;
  out[2] = (fa - mass[1]) / fa;
  out[3] = lmax;
  out[4] = lmin;
  out[5] = tail;
}

// ============================================================== host side
namespace {

int blocks_for(int64_t n, int per = 256, int cap = 4096) {
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, cap)));
}

}  // namespace

// Column Gram (+/-) of X into M (d x d).  ws must hold nsplit * d * d doubles.
hipError_t eval_colgram(const void* X, int dt, int64_t ldx, int64_t rows, int d, double sign,
                        int accumulate, double* M, double* ws, int nsplit_max, hipStream_t s) {
  const int T = (d + 31) / 32;
  const int ntiles = T * (T + 1) / 2;
  int nsplit = std::max(1, std::min<int>(nsplit_max, (1024 + ntiles - 1) / ntiles));
  int64_t rchunk = (rows + nsplit - 1) / nsplit;
  rchunk = (rchunk + 31) / 32 * 32;
  nsplit = static_cast<int>(std::max<int64_t>(1, (rows + rchunk - 1) / rchunk));
  if (rows > 0) {
    hipLaunchKernelGGL(k_colgram, dim3(ntiles, nsplit), dim3(256), 0, s, X, dt, ldx, rows, d, rchunk,
                       ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  } else {
    nsplit = 0;
  }
  hipLaunchKernelGGL(k_colgram_reduce, dim3(blocks_for(static_cast<int64_t>(d) * d)), dim3(256), 0, s,
                     ws, nsplit, d, sign, accumulate, M);
  return hipGetLastError();
}

hipError_t eval_symv(const double* M, int d, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_symv, dim3((d + 3) / 4), dim3(256), 0, s, M, d, x, y);
  return hipGetLastError();
}

hipError_t eval_gram_op(const void* X, int dt, int64_t ldx, int64_t rows, int d, double sign,
                        int accumulate, const double* x, double* y, double* t, double* part,
                        int nz_max, hipStream_t s) {
  if (rows <= 0) {
    if (!accumulate) return hipMemsetAsync(y, 0, d * sizeof(double), s);
    return hipSuccess;
  }
  hipLaunchKernelGGL(k_gemv_rows, dim3(static_cast<unsigned>((rows + 3) / 4)), dim3(256), 0, s, X, dt,
                     ldx, rows, d, x, t);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int nz = static_cast<int>(std::min<int64_t>(nz_max, std::max<int64_t>(1, rows / 256)));
  int64_t rchunk = (rows + nz - 1) / nz;
  nz = static_cast<int>((rows + rchunk - 1) / rchunk);
  hipLaunchKernelGGL(k_gemv_cols, dim3((d + 255) / 256, nz), dim3(256), 0, s, X, dt, ldx, rows, d,
                     rchunk, t, part);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_parts, dim3((d + 255) / 256), dim3(256), 0, s, part, nz, d, sign, accumulate,
                     y);
  return hipGetLastError();
}

hipError_t eval_lanczos_step(const double* Q, int d, int j, double* y, double* h1, double* h2,
                             double* alpha, double* beta, double* qnext, double floor_abs,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_dots, dim3(j + 1), dim3(256), 0, s, Q, d, j + 1, y, h1);
  hipLaunchKernelGGL(k_axpy_many, dim3((d + 255) / 256), dim3(256), 0, s, Q, d, j + 1, h1, y);
  hipLaunchKernelGGL(k_dots, dim3(j + 1), dim3(256), 0, s, Q, d, j + 1, y, h2);
  hipLaunchKernelGGL(k_axpy_many, dim3((d + 255) / 256), dim3(256), 0, s, Q, d, j + 1, h2, y);
  hipLaunchKernelGGL(k_lanczos_close, dim3(1), dim3(1024), 0, s, h1, h2, j, y, d, alpha, beta, qnext,
                     floor_abs);
  return hipGetLastError();
}

hipError_t eval_build_tridiag(const double* alpha, const double* beta, int K, double* T, int ldt,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_build_tridiag, dim3(blocks_for(static_cast<int64_t>(K) * K)), dim3(256), 0, s,
                     alpha, beta, K, T, ldt);
  return hipGetLastError();
}

hipError_t eval_extremes(const double* v, int n, int k, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_extremes, dim3(1), dim3(1024), 0, s, v, n, k, out);
  return hipGetLastError();
}

hipError_t eval_fro2(const void* X, int dt, int64_t ldx, int64_t rows, int d, double* part,
                     double* out, hipStream_t s) {
  int nb = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(rows, 2048)));
  if (rows <= 0) return hipMemsetAsync(out, 0, sizeof(double), s);
  hipLaunchKernelGGL(k_fro2_rows, dim3(nb), dim3(256), 0, s, X, dt, ldx, rows, d, part);
  hipLaunchKernelGGL(k_sum_scalar, dim3(1), dim3(64), 0, s, part, nb, out);
  return hipGetLastError();
}

hipError_t eval_rowspace(const double* lam, const double* U, int l, int mp, const double* B,
                         int64_t ldb, int d, double rtol, int* perm, int* nrank, double* Vt,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_rank_desc, dim3(1), dim3(1024), 0, s, lam, l, rtol, perm, nrank);
  hipLaunchKernelGGL(k_rowspace_vt, dim3(l), dim3(256), 0, s, lam, U, mp, B, ldb, l, d, perm, nrank,
                     Vt);
  return hipGetLastError();
}

hipError_t eval_proj_mass(const void* X, int dt, int64_t ldx, int64_t rows, int d, const double* Vt,
                          const int* nrank, int k, double* part, double* out2, hipStream_t s) {
  if (rows <= 0) return hipMemsetAsync(out2, 0, 2 * sizeof(double), s);
  int nb = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((rows + 3) / 4, 2048)));
  hipLaunchKernelGGL(k_proj_mass, dim3(nb), dim3(256), 0, s, X, dt, ldx, rows, d, Vt, nrank, k, part);
  hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(64), 0, s, part, nb, out2);
  return hipGetLastError();
}

hipError_t eval_start_vector(double* q, int d, hipStream_t s) {
  hipLaunchKernelGGL(k_start_vector, dim3((d + 255) / 256), dim3(256), 0, s, q, d);
  hipLaunchKernelGGL(k_normalize, dim3(1), dim3(1024), 0, s, q, d);
  return hipGetLastError();
}

hipError_t eval_finish(const double* ext_M, const double* ext_A, int k, const double* fro2A,
                       const double* mass, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_report, dim3(1), dim3(64), 0, s, ext_M, ext_A, k, fro2A, mass, out);
  return hipGetLastError();
}

}  // namespace fdsk
