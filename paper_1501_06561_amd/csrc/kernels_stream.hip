// Streaming-path kernels: row ingest, FP64 Gram (matrix cores), shrink
// (ReduceRank rules), rebuild (matrix cores), finalize helpers.
//
// Buffer layout: C is mp x ldc FP64 row-major; mp = m rounded up to 32 rows
// (rows >= m are zero forever), ldc = d rounded up to 64 columns (columns >= d
// are zero).  Rows [0, occ) are occupied.
#include "fdsk_device.hpp"
#include "fdsk_kernels.hpp"
#include "fdsk_batch.hpp"

namespace fdsk {

// ----------------------------------------------------------------- ingest
// One workgroup per row: convert to FP64, zero the pad columns, and store the
// row's squared norm (FP64) for the ||A||_F^2 accumulator.
// With H (and L) set, the row's split-BF16 halves are written there too
// (same row, leading dimension ldc).
__device__ __forceinline__ void ingest_body(const void* __restrict__ src, int dt, int64_t stride, int d,
                                            double* __restrict__ C, int ldc, int row0,
                                            double* __restrict__ rownorm, int i,
                                            uint16_t* __restrict__ H = nullptr,
                                            uint16_t* __restrict__ L = nullptr, bool w64 = true) {
  const int64_t base = static_cast<int64_t>(i) * stride;
  const int64_t ro = static_cast<int64_t>(row0 + i) * ldc;
  double* dst = C + ro;
  double acc = 0.0;
  for (int c = threadIdx.x; c < ldc; c += blockDim.x) {
    double v = (c < d) ? load_as_f64(src, base + c, dt) : 0.0;
    if (w64) dst[c] = v;
    acc += v * v;
    if (H) {
      uint16_t hb, lb;
      split_bits(v, hb, lb);
      H[ro + c] = hb;
      L[ro + c] = lb;
    }
  }
  __shared__ double red[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) rownorm[row0 + i] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_ingest(const void* __restrict__ src, int dt,
                                                int64_t stride, int d, double* __restrict__ C,
                                                int ldc, int row0, double* __restrict__ rownorm) {
  ingest_body(src, dt, stride, d, C, ldc, row0, rownorm, blockIdx.x);
}

// ------------------------------------------------------------------- Gram
// G = C C^T on lower-triangular 32x32 tiles with split-K.  Four waves per
// workgroup, each owning a 16x16 sub-tile fed by 16x16x4 FP64 MFMA.
constexpr int GT = 32;   // output tile
constexpr int GK = 32;   // K chunk staged in LDS

__device__ __forceinline__ void gram_body(const double* __restrict__ C, int ldc, int mp, int kchunk,
                                          double* __restrict__ Gpart, int tile, int ks) {
  int ti = static_cast<int>((sqrtf(8.0f * tile + 1.0f) - 1.0f) * 0.5f);
  while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
  while (ti * (ti + 1) / 2 > tile) --ti;
  const int tj = tile - ti * (ti + 1) / 2;
  const int k0 = ks * kchunk;
  const int k1 = min(ldc, k0 + kchunk);

  __shared__ double As[GT][GK + 1];
  __shared__ double Bs[GT][GK + 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w >> 1, wj = w & 1;
  const int li = lane & 15, lk = lane >> 4;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  const double* Ca = C + static_cast<int64_t>(ti * GT) * ldc;
  const double* Cb = C + static_cast<int64_t>(tj * GT) * ldc;

  for (int kk = k0; kk < k1; kk += GK) {
    // 32 rows x 32 cols per operand: 256 threads x 4 doubles.
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int idx = threadIdx.x + e * 256;
      int r = idx >> 5, c = idx & 31;
      As[r][c] = Ca[static_cast<int64_t>(r) * ldc + kk + c];
      Bs[r][c] = Cb[static_cast<int64_t>(r) * ldc + kk + c];
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < GK / 4; ++k4) {
      double a = As[wi * 16 + li][k4 * 4 + lk];
      double b = Bs[wj * 16 + li][k4 * 4 + lk];
      acc = mfma_f64(a, b, acc);
    }
    __syncthreads();
  }
  double* out = Gpart + static_cast<int64_t>(ks) * mp * mp;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    int row = ti * GT + wi * 16 + lk + 4 * v;
    int col = tj * GT + wj * 16 + li;
    out[static_cast<int64_t>(row) * mp + col] = acc[v];
  }
}

__global__ __launch_bounds__(256) void k_gram_f64(const double* __restrict__ C, int ldc,
                                                  int mp, int kchunk, double* __restrict__ Gpart) {
  gram_body(C, ldc, mp, kchunk, Gpart, blockIdx.x, blockIdx.y);
}

// Sum the split-K partials in a fixed order and mirror the lower triangle.
__device__ __forceinline__ void gram_reduce_body(const double* __restrict__ Gpart, int ksplit, int mp,
                                                 double* __restrict__ G, int bx, int nbx) {
  const int64_t n = static_cast<int64_t>(mp) * mp;
  for (int64_t e = bx * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(nbx) * blockDim.x) {
    int r = static_cast<int>(e / mp), c = static_cast<int>(e % mp);
    if ((r >> 5) < (c >> 5)) continue;   // upper tiles are written by the mirror
    double v = 0.0;
    for (int k = 0; k < ksplit; ++k) v += Gpart[static_cast<int64_t>(k) * n + e];
    if (r >= c) {
      G[static_cast<int64_t>(r) * mp + c] = v;
      G[static_cast<int64_t>(c) * mp + r] = v;
    }
  }
}

__global__ void k_gram_reduce(const double* __restrict__ Gpart, int ksplit, int mp,
                              double* __restrict__ G) {
  gram_reduce_body(Gpart, ksplit, mp, G, blockIdx.x, gridDim.x);
}

// ----------------------------------------------------------------- shrink
// One workgroup.  Ranks the eigenvalues (descending, ties by index), applies
// the variant's ReduceRank rule in FP64, updates the accumulators and writes
// Ut = diag(rho) * U^T for the keep surviving rows, rho_j = sigma'_j/sigma_j.
// With Uh set, Ut's rows also go out as their split-BF16 halves (hi rows in
// Uh, lo rows mp x mp further on), for a rebuild that reads them directly.
__device__ __forceinline__ void shrink_body(const double* __restrict__ lam_raw,
                                            const double* __restrict__ V, int m, int mp, RuleParams rp,
                                            const double* __restrict__ rownorm, int new0, int new1,
                                            double* __restrict__ Ut, DevStats* __restrict__ st,
                                            uint16_t* __restrict__ Uh = nullptr) {
  __shared__ double lam[1024];
  __shared__ int perm[1024];
  __shared__ double rho[1024];
  __shared__ double red[1024];
  __shared__ double red2[1024];
  __shared__ double raw[1024];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  __syncthreads();
  // NaN is ranked as -inf so the ranking stays a permutation (indices read
  // through perm[] are always in range); the flag reports it.
  for (int j = tid; j < m; j += blockDim.x) {
    double x = lam_raw[j];
    if (!(x == x) || isinf(x)) bad = 1;
    raw[j] = (x == x) ? x : -INFINITY;
  }
  __syncthreads();
  for (int j = tid; j < m; j += blockDim.x) {
    double x = raw[j];
    int rank = 0;
    for (int i = 0; i < m; ++i) {
      double y = raw[i];
      rank += (y > x) || (y == x && i < j);
    }
    perm[rank] = j;
  }
  __syncthreads();
  for (int q = tid; q < m; q += blockDim.x) lam[q] = fmax(raw[perm[q]], 0.0);
  __syncthreads();
  double delta = (rp.t - 1 < m) ? lam[rp.t - 1] : 0.0;
  const double lnull = kNullRel * lam[0];
  // SpaceSaving Directions: nothing moves when the l-th direction is outside
  // the row space (then the buffer already has a free row).
  const bool ssd_move = rp.variant == 4 && lam[rp.l - 1] > lnull;
  if (rp.variant == 4) delta = ssd_move ? lam[rp.l - 2] : 0.0;
  // Compensative FD: the accumulated Delta after the latest reduction.
  const double Dtot = rp.comp ? st->Delta : 0.0;
  double removed = 0.0;
  for (int q = tid; q < m; q += blockDim.x) {
    double x = lam[q];
    double y;
    bool untouched;
    if (rp.comp == 2) {               // the spectrum as it is
      untouched = false;
      y = x;
    } else if (rp.variant == 1) {     // iSVD: keep the first l-1, drop the rest
      untouched = q < rp.l - 1;
      y = untouched ? x : 0.0;
    } else if (rp.variant == 4) {     // SSD: lambda_{l-1} moves onto the l-th direction
      untouched = !ssd_move || q < rp.l - 2;
      y = untouched ? x : (q == rp.l - 2 ? 0.0 : x + delta);
    } else {                          // FD / alpha / fast alpha / CFD: shrink from index r on
      untouched = q < rp.r;
      y = untouched ? x : fmax(x - delta, 0.0);
    }
    if (rp.comp) {
      // Output value y + Delta on the first l directions in the row space;
      // the shrink total falls by what is added back.
      double yh = (q < rp.l && x > lnull) ? y + Dtot : 0.0;
      removed += y - yh;
      rho[q] = yh > 0.0 ? sqrt(yh / x) : 0.0;
    } else {
      removed += x - y;
      rho[q] = untouched ? 1.0 : ((x > 0.0 && y > 0.0) ? sqrt(y / x) : 0.0);
    }
  }
  // SSD: the merged direction takes the freed slot l-2 of the kept rows.
  __syncthreads();
  if (ssd_move && tid == 0) {
    perm[rp.l - 2] = perm[rp.l - 1];
    rho[rp.l - 2] = rho[rp.l - 1];
  }
  // Squared norms of the rows appended since the last reduction, summed by
  // the block alongside the removed mass.
  double nrm_part = 0.0;
  for (int i = new0 + tid; i < new1; i += blockDim.x) nrm_part += rownorm[i];
  red[tid] = removed;
  red2[tid] = nrm_part;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if (tid < s) {
      red[tid] += red[tid + s];
      red2[tid] += red2[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double nrm = red2[0];
    st->fro2A += nrm;
    if (!rp.mass) st->Stot += red[0];
    if (!rp.comp) {
      st->Delta += delta;
      st->n_rr += 1;
    }
    if (bad || !(nrm == nrm)) st->nonfinite = 1;
  }
  // Ut rows [0, keep) ; rows up to the next multiple of 32 are zero.  A
  // wave per row, lanes across it.
  const int rows = (rp.keep + 31) & ~31;
  const int lane = tid & 63, nwave = blockDim.x >> 6;
  for (int q = tid >> 6; q < rows; q += nwave) {
    const bool live = q < rp.keep && q < m;
    const double r = live ? rho[q] : 0.0;
    const double* src = V + static_cast<int64_t>(live ? perm[q] : 0) * mp;
    double* dst = Ut + static_cast<int64_t>(q) * mp;
    for (int i = lane; i < mp; i += 64) {
      const double u = (live && i < m) ? r * src[i] : 0.0;
      dst[i] = u;
      if (Uh) {
        uint16_t hb, lb;
        split_bits(u, hb, lb);
        Uh[static_cast<int64_t>(q) * mp + i] = hb;
        Uh[static_cast<int64_t>(mp) * mp + static_cast<int64_t>(q) * mp + i] = lb;
      }
    }
  }
}

__global__ __launch_bounds__(1024) void k_shrink(const double* __restrict__ lam_raw,
                                                 const double* __restrict__ V, int m, int mp,
                                                 RuleParams rp, const double* __restrict__ rownorm,
                                                 int new0, int new1, double* __restrict__ Ut,
                                                 DevStats* __restrict__ st) {
  shrink_body(lam_raw, V, m, mp, rp, rownorm, new0, new1, Ut, st);
}

// ---------------------------------------------------------------- rebuild
// out[0:keep, :] = Ut[0:keep, 0:mp] * C[0:mp, :].  Tile RT rows (32 or 64) x
// 64 cols; wave w owns rows (w>>1)*RT/2.. and cols (w&1)*32.. as RT/32 x 2
// 16x16 MFMA tiles, so a 64-row tile reads each column slab of C once for
// twice the rows.  Ut rows past mp (the last tile of a 64-row launch) load
// as zero; output rows past keep are not written.
template <int RT>
__device__ __forceinline__ void rebuild_body(const double* __restrict__ Ut, const double* __restrict__ C,
                                             int ldc, int mp, int keep, double* __restrict__ out, int bx,
                                             int by) {
  static_assert(RT == 32 || RT == 64, "rebuild rows per workgroup");
  constexpr int RA = RT / 32;
  const int r0 = by * RT, c0 = bx * 64;
  __shared__ double As[RT][33];
  __shared__ double Bs[32][65];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w >> 1, wj = w & 1;
  const int li = lane & 15, lk = lane >> 4;
  f64x4 acc[RA][2];
#pragma unroll
  for (int a = 0; a < RA; ++a) acc[a][0] = acc[a][1] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < mp; k0 += 32) {
#pragma unroll
    for (int e = 0; e < RT / 8; ++e) {
      int idx = threadIdx.x + e * 256;
      int r = idx >> 5, c = idx & 31;
      As[r][c] = (r0 + r < mp) ? Ut[static_cast<int64_t>(r0 + r) * mp + k0 + c] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      int idx = threadIdx.x + e * 256;
      int r = idx >> 6, c = idx & 63;
      Bs[r][c] = C[static_cast<int64_t>(k0 + r) * ldc + c0 + c];
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < 8; ++k4) {
      double b0 = Bs[k4 * 4 + lk][wj * 32 + li];
      double b1 = Bs[k4 * 4 + lk][wj * 32 + 16 + li];
#pragma unroll
      for (int a = 0; a < RA; ++a) {
        double av = As[wi * (RT / 2) + a * 16 + li][k4 * 4 + lk];
        acc[a][0] = mfma_f64(av, b0, acc[a][0]);
        acc[a][1] = mfma_f64(av, b1, acc[a][1]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < RA; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int row = r0 + wi * (RT / 2) + a * 16 + lk + 4 * v;
      if (row < keep) {
        int64_t o = static_cast<int64_t>(row) * ldc + c0 + wj * 32 + li;
        out[o] = acc[a][0][v];
        out[o + 16] = acc[a][1][v];
      }
    }
}

template <int RT>
__global__ __launch_bounds__(256) void k_rebuild_f64(const double* __restrict__ Ut,
                                                     const double* __restrict__ C, int ldc,
                                                     int mp, int keep, double* __restrict__ out) {
  rebuild_body<RT>(Ut, C, ldc, mp, keep, out, blockIdx.x, blockIdx.y);
}

// --------------------------------------------------------------- helpers
__global__ void k_zero_rows(double* __restrict__ C, int ldc, int r0, int r1) {
  const int64_t n = static_cast<int64_t>(r1 - r0) * ldc;
  double* p = C + static_cast<int64_t>(r0) * ldc;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[e] = 0.0;
}

__global__ void k_add_pending_norms(const double* __restrict__ rownorm, int new0, int new1,
                                    DevStats* __restrict__ st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double nrm = 0.0;
    for (int i = new0; i < new1; ++i) nrm += rownorm[i];
    st->fro2A += nrm;
    if (!(nrm == nrm) || isinf(nrm)) st->nonfinite = 1;
  }
}

__global__ void k_copy_out(const double* __restrict__ C, int ldc, int valid_rows, int l, int d,
                           void* __restrict__ out, int64_t ldb, int out_dt) {
  const int64_t n = static_cast<int64_t>(l) * d;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int r = static_cast<int>(e / d), c = static_cast<int>(e % d);
    double v = (r < valid_rows) ? C[static_cast<int64_t>(r) * ldc + c] : 0.0;
    if (out_dt == DT_F64)
      static_cast<double*>(out)[r * ldb + c] = v;
    else
      static_cast<float*>(out)[r * ldb + c] = static_cast<float>(v);
  }
}

__global__ void k_transpose(const double* __restrict__ in, int mp, int n, double* __restrict__ out) {
  const int64_t tot = static_cast<int64_t>(n) * n;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < tot;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int i = static_cast<int>(e / n), j = static_cast<int>(e % n);
    out[static_cast<int64_t>(i) * mp + j] = in[static_cast<int64_t>(j) * mp + i];
  }
}

__global__ void k_convert_f64(const void* __restrict__ X, int dt, int64_t ldx, int64_t rows, int d,
                              double* __restrict__ out) {
  const int64_t n = rows * d;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int64_t r = e / d;
    int c = static_cast<int>(e % d);
    out[e] = load_as_f64(X, r * ldx + c, dt);
  }
}

// ------------------------------------------------------------ launchers
hipError_t launch_convert_f64(const void* X, int dt, int64_t ldx, int64_t rows, int d, double* out,
                              hipStream_t s) {
  int64_t n = rows * d;
  int blocks = static_cast<int>(std::min<int64_t>((n + 255) / 256, 4096));
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert_f64, dim3(blocks), dim3(256), 0, s, X, dt, ldx, rows, d, out);
  return hipGetLastError();
}

hipError_t launch_transpose(const double* in, int mp, int n, double* out, hipStream_t s) {
  int64_t tot = static_cast<int64_t>(n) * n;
  int blocks = static_cast<int>(std::min<int64_t>((tot + 255) / 256, 4096));
  hipLaunchKernelGGL(k_transpose, dim3(blocks), dim3(256), 0, s, in, mp, n, out);
  return hipGetLastError();
}

hipError_t launch_ingest(const void* src, int dt, int64_t stride, int f, int d, double* C,
                         int ldc, int row0, double* rownorm, hipStream_t s) {
  if (f <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ingest, dim3(f), dim3(256), 0, s, src, dt, stride, d, C, ldc, row0, rownorm);
  return hipGetLastError();
}

hipError_t launch_gram(const double* C, int ldc, int mp, double* Gpart, int ksplit_max, double* G,
                       hipStream_t s, int ksplit_req) {
  const int T = mp / GT;
  const int ntiles = T * (T + 1) / 2;
  int ksplit = ksplit_req > 0 ? ksplit_req : gram_ksplit_default(ntiles, ldc);
  ksplit = std::max(1, std::min(ksplit, ksplit_max));
  int kchunk = (ldc + ksplit - 1) / ksplit;
  kchunk = (kchunk + GK - 1) / GK * GK;
  ksplit = (ldc + kchunk - 1) / kchunk;
  hipLaunchKernelGGL(k_gram_f64, dim3(ntiles, ksplit), dim3(256), 0, s, C, ldc, mp, kchunk, Gpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_gram_reduce(Gpart, ksplit, mp, G, s);
}

hipError_t launch_gram_reduce(const double* Gpart, int ksplit, int mp, double* G, hipStream_t s) {
  const int64_t n = static_cast<int64_t>(mp) * mp;
  int blocks = static_cast<int>(std::min<int64_t>((n + 255) / 256, 2048));
  hipLaunchKernelGGL(k_gram_reduce, dim3(blocks), dim3(256), 0, s, Gpart, ksplit, mp, G);
  return hipGetLastError();
}

hipError_t launch_shrink(const double* lam, const double* V, int m, int mp, RuleParams rp,
                         const double* rownorm, int new0, int new1, double* Ut, DevStats* st,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_shrink, dim3(1), dim3(1024), 0, s, lam, V, m, mp, rp, rownorm, new0, new1,
                     Ut, st);
  return hipGetLastError();
}

hipError_t launch_rebuild(const double* Ut, const double* C, int ldc, int mp, int keep, double* out,
                          hipStream_t s, int rt) {
  if (keep <= 0) return hipSuccess;
  if (rt != 32 && rt != 64) return hipErrorInvalidValue;
  dim3 grid(ldc / 64, (keep + rt - 1) / rt);
  if (rt == 64)
    hipLaunchKernelGGL(k_rebuild_f64<64>, grid, dim3(256), 0, s, Ut, C, ldc, mp, keep, out);
  else
    hipLaunchKernelGGL(k_rebuild_f64<32>, grid, dim3(256), 0, s, Ut, C, ldc, mp, keep, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_row_mass(const double* __restrict__ C, int ldc, int d,
                                                 double* __restrict__ out) {
  __shared__ double red[4];
  const double* c = C + static_cast<int64_t>(blockIdx.x) * ldc;
  double v = 0.0;
  for (int j = threadIdx.x; j < d; j += 256) v = fma(c[j], c[j], v);
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_mass_close(const double* __restrict__ before, int nb, const double* __restrict__ after, int na,
                             DevStats* __restrict__ st) {
  if (threadIdx.x != 0) return;
  double b = 0.0, a = 0.0;
  for (int i = 0; i < nb; ++i) b += before[i];
  for (int i = 0; i < na; ++i) a += after[i];
  st->Stot += b - a;
}

hipError_t launch_row_mass(const double* C, int ldc, int rows, int d, double* out, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_mass, dim3(rows), dim3(256), 0, s, C, ldc, d, out);
  return hipGetLastError();
}

hipError_t launch_mass_close(const double* before, int nb, const double* after, int na, DevStats* st,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_mass_close, dim3(1), dim3(64), 0, s, before, nb, after, na, st);
  return hipGetLastError();
}

hipError_t launch_zero_rows(double* C, int ldc, int r0, int r1, hipStream_t s) {
  if (r1 <= r0) return hipSuccess;
  int64_t n = static_cast<int64_t>(r1 - r0) * ldc;
  int blocks = static_cast<int>(std::min<int64_t>((n + 255) / 256, 4096));
  hipLaunchKernelGGL(k_zero_rows, dim3(blocks), dim3(256), 0, s, C, ldc, r0, r1);
  return hipGetLastError();
}

hipError_t launch_add_pending_norms(const double* rownorm, int new0, int new1, DevStats* st,
                                    hipStream_t s) {
  hipLaunchKernelGGL(k_add_pending_norms, dim3(1), dim3(64), 0, s, rownorm, new0, new1, st);
  return hipGetLastError();
}

// Merge: dst's accumulators absorb src's, including the squared norms of
// src's rows appended since its last reduction (not yet in src's fro2A).
__global__ void k_merge_stats(DevStats* __restrict__ dst, const DevStats* __restrict__ src,
                              const double* __restrict__ src_rownorm, int new0, int new1) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double nrm = 0.0;
    for (int i = new0; i < new1; ++i) nrm += src_rownorm[i];
    dst->fro2A += src->fro2A + nrm;
    dst->Delta += src->Delta;
    dst->Stot += src->Stot;
    dst->n_rr += src->n_rr;
    dst->eig_unconv += src->eig_unconv;
    dst->eig_sweeps += src->eig_sweeps;
    if (src->nonfinite || !(nrm == nrm) || isinf(nrm)) dst->nonfinite = 1;
    if (src->bar_err) dst->bar_err = 1;
  }
}

hipError_t launch_merge_stats(DevStats* dst, const DevStats* src, const double* src_rownorm, int new0,
                              int new1, hipStream_t s) {
  hipLaunchKernelGGL(k_merge_stats, dim3(1), dim3(64), 0, s, dst, src, src_rownorm, new0, new1);
  return hipGetLastError();
}

hipError_t launch_copy_out(const double* C, int ldc, int valid_rows, int l, int d, void* out,
                           int64_t ldb, int out_dt, hipStream_t s) {
  int64_t n = static_cast<int64_t>(l) * d;
  int blocks = static_cast<int>(std::min<int64_t>((n + 255) / 256, 4096));
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_out, dim3(blocks), dim3(256), 0, s, C, ldc, valid_rows, l, d, out, ldb,
                     out_dt);
  return hipGetLastError();
}

// ------------------------------------------------------ grouped (batches)
// One task per entry of the grid's last dimension; blocks past the task's
// own extent return at once (before any barrier).
__global__ __launch_bounds__(256) void kg_ingest(const GroupSketch* __restrict__ SK,
                                                 const GroupIngest* __restrict__ T, int dt) {
  const GroupIngest t = T[blockIdx.y];
  if (static_cast<int>(blockIdx.x) >= t.f) return;
  const GroupSketch& s = SK[t.sk];
  uint16_t* H = s.npass ? (t.cur ? s.bh1 : s.bh0) : nullptr;
  uint16_t* L = H ? H + static_cast<int64_t>((s.mp + 63) / 64 * 64) * s.ldc : nullptr;
  ingest_body(t.src, dt, t.stride, s.d, t.cur ? s.C1 : s.C0, s.ldc, t.row0, s.rownorm, blockIdx.x, H, L,
              t.w64 != 0 || s.npass == 0);
}

// Split-K: K slice blockIdx.y of the task's slice length (task_kchunk) into
// partial blockIdx.y of its Gp; slices past the task's row length return.
__global__ __launch_bounds__(256) void kg_gram(const GroupSketch* __restrict__ SK,
                                               const GroupRR* __restrict__ T, int kc) {
  const GroupRR t = T[blockIdx.z];
  const GroupSketch& s = SK[t.sk];
  if (s.npass != 0) return;
  const int nt = s.mp / GT;
  if (static_cast<int>(blockIdx.x) >= nt * (nt + 1) / 2) return;
  const int kchunk = task_kchunk(kc >= 0 ? kc : s.kchunk, s.ldc);
  if (static_cast<int>(blockIdx.y) * kchunk >= s.ldc) return;
  gram_body(t.cur ? s.C1 : s.C0, s.ldc, s.mp, kchunk, s.Gp, blockIdx.x, blockIdx.y);
}

// Sum each task's partials in order and mirror the lower triangle into G.
__global__ __launch_bounds__(256) void kg_mirror(const GroupSketch* __restrict__ SK,
                                                 const GroupRR* __restrict__ T, int kc) {
  const GroupSketch& s = SK[T[blockIdx.y].sk];
  const int kchunk = task_kchunk(kc >= 0 ? kc : s.kchunk, s.ldc);
  gram_reduce_body(s.Gp, (s.ldc + kchunk - 1) / kchunk, s.mp, s.G, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(1024) void kg_shrink(const GroupSketch* __restrict__ SK,
                                                  const GroupRR* __restrict__ T) {
  const GroupRR t = T[blockIdx.x];
  const GroupSketch& s = SK[t.sk];
  shrink_body(s.lam, s.V, s.m, s.mp, s.rp, s.rownorm, t.new0, t.new1, s.Ut, s.st, s.npass ? s.uh : nullptr);
}

template <int RT>
__global__ __launch_bounds__(256) void kg_rebuild(const GroupSketch* __restrict__ SK,
                                                  const GroupRR* __restrict__ T) {
  const GroupRR t = T[blockIdx.z];
  const GroupSketch& s = SK[t.sk];
  if (s.npass != 0) return;
  if (static_cast<int>(blockIdx.x) >= s.ldc / 64 || static_cast<int>(blockIdx.y) * RT >= s.rp.keep) return;
  rebuild_body<RT>(s.Ut, t.cur ? s.C1 : s.C0, s.ldc, s.mp, s.rp.keep, t.cur ? s.C0 : s.C1, blockIdx.x,
                   blockIdx.y);
}

__global__ __launch_bounds__(256) void kg_zero(const GroupSketch* __restrict__ SK,
                                               const GroupSpan* __restrict__ T) {
  const GroupSpan t = T[blockIdx.y];
  const GroupSketch& s = SK[t.sk];
  double* p = (t.cur ? s.C1 : s.C0) + static_cast<int64_t>(t.r0) * s.ldc;
  const int64_t n = static_cast<int64_t>(t.r1 - t.r0) * s.ldc;
  for (int64_t e = blockIdx.x * 256LL + threadIdx.x; e < n; e += 256LL * gridDim.x) p[e] = 0.0;
  if (s.npass) {     // and the rows' bf16 halves
    uint16_t* H = (t.cur ? s.bh1 : s.bh0) + static_cast<int64_t>(t.r0) * s.ldc;
    uint16_t* L = H + static_cast<int64_t>((s.mp + 63) / 64 * 64) * s.ldc;
    for (int64_t e = blockIdx.x * 256LL + threadIdx.x; e < n; e += 256LL * gridDim.x) H[e] = L[e] = 0;
  }
}

__global__ void kg_pending(const GroupSketch* __restrict__ SK, const GroupSpan* __restrict__ T, int nt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  const GroupSpan t = T[i];
  const GroupSketch& s = SK[t.sk];
  double nrm = 0.0;
  for (int r = t.r0; r < t.r1; ++r) nrm += s.rownorm[r];
  s.st->fro2A += nrm;
  if (!(nrm == nrm) || isinf(nrm)) s.st->nonfinite = 1;
}

hipError_t launch_group_ingest(const GroupSketch* sk, const GroupIngest* t, int nt, int max_f, int dt,
                               hipStream_t s) {
  if (nt <= 0 || max_f <= 0) return hipSuccess;
  hipLaunchKernelGGL(kg_ingest, dim3(max_f, nt), dim3(256), 0, s, sk, t, dt);
  return hipGetLastError();
}

hipError_t launch_group_gram(const GroupSketch* sk, const GroupRR* t, int nt, int max_mp, bool fp64, int ks,
                             int kc, hipStream_t s) {
  if (nt <= 0) return hipSuccess;
  if (ks < 1 || ks > kGpParts || (kc > 0 && kc % 64)) return hipErrorInvalidValue;
  const int T = max_mp / GT;
  if (fp64) hipLaunchKernelGGL(kg_gram, dim3(T * (T + 1) / 2, ks, nt), dim3(256), 0, s, sk, t, kc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nb = std::max(1, std::min(64, (max_mp * max_mp + 255) / 256));
  hipLaunchKernelGGL(kg_mirror, dim3(nb, nt), dim3(256), 0, s, sk, t, kc);
  return hipGetLastError();
}

hipError_t launch_group_shrink(const GroupSketch* sk, const GroupRR* t, int nt, hipStream_t s) {
  if (nt <= 0) return hipSuccess;
  hipLaunchKernelGGL(kg_shrink, dim3(nt), dim3(1024), 0, s, sk, t);
  return hipGetLastError();
}

hipError_t launch_group_rebuild(const GroupSketch* sk, const GroupRR* t, int nt, int max_ldc, int max_keep,
                                int rt, hipStream_t s) {
  if (nt <= 0 || max_keep <= 0) return hipSuccess;
  if (rt == 64)
    hipLaunchKernelGGL(kg_rebuild<64>, dim3(max_ldc / 64, (max_keep + 63) / 64, nt), dim3(256), 0, s, sk, t);
  else if (rt == 32)
    hipLaunchKernelGGL(kg_rebuild<32>, dim3(max_ldc / 64, (max_keep + 31) / 32, nt), dim3(256), 0, s, sk, t);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_group_zero(const GroupSketch* sk, const GroupSpan* t, int nt, hipStream_t s) {
  if (nt <= 0) return hipSuccess;
  hipLaunchKernelGGL(kg_zero, dim3(16, nt), dim3(256), 0, s, sk, t);
  return hipGetLastError();
}

hipError_t launch_group_pending(const GroupSketch* sk, const GroupSpan* t, int nt, hipStream_t s) {
  if (nt <= 0) return hipSuccess;
  hipLaunchKernelGGL(kg_pending, dim3((nt + 255) / 256), dim3(256), 0, s, sk, t, nt);
  return hipGetLastError();
}

}  // namespace fdsk
