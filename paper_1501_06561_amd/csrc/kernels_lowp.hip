// Reduced-precision Gram and rebuild products (BF16 matrix cores, FP32
// accumulation).  The sketch buffer stays FP64; each operand element x is
// split into hi = bf16(x) and lo = bf16(x - hi).  One pass uses hi*hi only;
// the compensated form adds the two cross terms hi*lo + lo*hi, which recovers
// about 16 significant bits per product (the dropped lo*lo term is below the
// FP32 accumulation error).  Eigensolve, shrink and accumulators stay FP64.
#include "fdsk_device.hpp"
#include "fdsk_kernels.hpp"
#include "fdsk_batch.hpp"

namespace fdsk {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split_bf16(double x, __bf16& hi, __bf16& lo) {
  const uint16_t hb = f32_to_bf16_bits(static_cast<float>(x));
  const float hf = bf16_bits_to_f32(hb);
  const uint16_t lb = f32_to_bf16_bits(static_cast<float>(x - static_cast<double>(hf)));
  hi = __builtin_bit_cast(__bf16, hb);
  lo = __builtin_bit_cast(__bf16, lb);
}

// 16x16x32 BF16 matrix-core step: lane = i + 16*q holds A[i][8q..8q+7] and
// B[8q..8q+7][i]; the result lane = j + 16*q holds D[4q + v][j] in element v.
__device__ __forceinline__ f32x4 mfma_bf16(bf16x8_t a, bf16x8_t b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int NPASS>
__device__ __forceinline__ f32x4 mfma_split(const bf16x8_t& ah, const bf16x8_t& al, const bf16x8_t& bh,
                                            const bf16x8_t& bl, f32x4 acc) {
  acc = mfma_bf16(ah, bh, acc);
  if (NPASS == 3) {
    acc = mfma_bf16(ah, bl, acc);
    acc = mfma_bf16(al, bh, acc);
  }
  return acc;
}

// G partials on lower-triangular 32x32 tiles with split-K (see k_gram_f64).
template <int NPASS>
__device__ __forceinline__ void gram_bf16_body(const double* __restrict__ C, int ldc, int mp, int kchunk,
                                               double* __restrict__ Gpart, int tile, int ks) {
  int ti = static_cast<int>((sqrtf(8.0f * tile + 1.0f) - 1.0f) * 0.5f);
  while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
  while (ti * (ti + 1) / 2 > tile) --ti;
  const int tj = tile - ti * (ti + 1) / 2;
  const int k0 = ks * kchunk;
  const int k1 = min(ldc, k0 + kchunk);
  __shared__ double As[32][33];
  __shared__ double Bs[32][33];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w >> 1, wj = w & 1;
  const int li = lane & 15, lq = lane >> 4;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  const double* Ca = C + static_cast<int64_t>(ti * 32) * ldc;
  const double* Cb = C + static_cast<int64_t>(tj * 32) * ldc;
  for (int kk = k0; kk < k1; kk += 32) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int idx = threadIdx.x + e * 256;
      int r = idx >> 5, c = idx & 31;
      As[r][c] = Ca[static_cast<int64_t>(r) * ldc + kk + c];
      Bs[r][c] = Cb[static_cast<int64_t>(r) * ldc + kk + c];
    }
    __syncthreads();
    bf16x8_t ah, al, bh, bl;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      __bf16 h, l;
      split_bf16(As[wi * 16 + li][8 * lq + t], h, l);
      ah[t] = h;
      al[t] = l;
      split_bf16(Bs[wj * 16 + li][8 * lq + t], h, l);
      bh[t] = h;
      bl[t] = l;
    }
    acc = mfma_split<NPASS>(ah, al, bh, bl, acc);
    __syncthreads();
  }
  double* out = Gpart + static_cast<int64_t>(ks) * mp * mp;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    int row = ti * 32 + wi * 16 + 4 * lq + v;
    int col = tj * 32 + wj * 16 + li;
    out[static_cast<int64_t>(row) * mp + col] = static_cast<double>(acc[v]);
  }
}

template <int NPASS>
__global__ __launch_bounds__(256) void k_gram_bf16(const double* __restrict__ C, int ldc, int mp,
                                                   int kchunk, double* __restrict__ Gpart) {
  gram_bf16_body<NPASS>(C, ldc, mp, kchunk, Gpart, blockIdx.x, blockIdx.y);
}

// out[0:keep, :] = Ut[0:keep, 0:mp] * C (see k_rebuild_f64), BF16 products.
template <int NPASS>
__device__ __forceinline__ void rebuild_bf16_body(const double* __restrict__ Ut, const double* __restrict__ C,
                                                  int ldc, int mp, int keep, double* __restrict__ out, int bx,
                                                  int by) {
  const int r0 = by * 32, c0 = bx * 64;
  __shared__ double As[32][33];
  __shared__ double Bs[32][65];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w >> 1, wj = w & 1;
  const int li = lane & 15, lq = lane >> 4;
  f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < mp; k0 += 32) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int idx = threadIdx.x + e * 256;
      int r = idx >> 5, c = idx & 31;
      As[r][c] = Ut[static_cast<int64_t>(r0 + r) * mp + k0 + c];
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      int idx = threadIdx.x + e * 256;
      int r = idx >> 6, c = idx & 63;
      Bs[r][c] = C[static_cast<int64_t>(k0 + r) * ldc + c0 + c];
    }
    __syncthreads();
    bf16x8_t ah, al, b0h, b0l, b1h, b1l;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      __bf16 h, l;
      split_bf16(As[wi * 16 + li][8 * lq + t], h, l);
      ah[t] = h;
      al[t] = l;
      split_bf16(Bs[8 * lq + t][wj * 32 + li], h, l);
      b0h[t] = h;
      b0l[t] = l;
      split_bf16(Bs[8 * lq + t][wj * 32 + 16 + li], h, l);
      b1h[t] = h;
      b1l[t] = l;
    }
    acc0 = mfma_split<NPASS>(ah, al, b0h, b0l, acc0);
    acc1 = mfma_split<NPASS>(ah, al, b1h, b1l, acc1);
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    int row = r0 + wi * 16 + 4 * lq + v;
    if (row < keep) {
      int64_t o = static_cast<int64_t>(row) * ldc + c0 + wj * 32 + li;
      out[o] = static_cast<double>(acc0[v]);
      out[o + 16] = static_cast<double>(acc1[v]);
    }
  }
}

template <int NPASS>
__global__ __launch_bounds__(256) void k_rebuild_bf16(const double* __restrict__ Ut,
                                                      const double* __restrict__ C, int ldc, int mp,
                                                      int keep, double* __restrict__ out) {
  rebuild_bf16_body<NPASS>(Ut, C, ldc, mp, keep, out, blockIdx.x, blockIdx.y);
}

hipError_t launch_gram_lowp(const double* C, int ldc, int mp, double* Gpart, int ksplit_max, double* G,
                            int npass, hipStream_t s) {
  const int T = mp / 32;
  const int ntiles = T * (T + 1) / 2;
  int ksplit = (256 + ntiles - 1) / ntiles;
  ksplit = std::min(ksplit, std::max(1, ldc / 256));
  ksplit = std::min(ksplit, ksplit_max);
  int kchunk = (ldc + ksplit - 1) / ksplit;
  kchunk = (kchunk + 31) / 32 * 32;
  ksplit = (ldc + kchunk - 1) / kchunk;
  if (npass == 3)
    hipLaunchKernelGGL(k_gram_bf16<3>, dim3(ntiles, ksplit), dim3(256), 0, s, C, ldc, mp, kchunk, Gpart);
  else
    hipLaunchKernelGGL(k_gram_bf16<1>, dim3(ntiles, ksplit), dim3(256), 0, s, C, ldc, mp, kchunk, Gpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_gram_reduce(Gpart, ksplit, mp, G, s);
}

hipError_t launch_rebuild_lowp(const double* Ut, const double* C, int ldc, int mp, int keep, double* out,
                               int npass, hipStream_t s) {
  if (keep <= 0) return hipSuccess;
  dim3 grid(ldc / 64, (keep + 31) / 32);
  if (npass == 3)
    hipLaunchKernelGGL(k_rebuild_bf16<3>, grid, dim3(256), 0, s, Ut, C, ldc, mp, keep, out);
  else
    hipLaunchKernelGGL(k_rebuild_bf16<1>, grid, dim3(256), 0, s, Ut, C, ldc, mp, keep, out);
  return hipGetLastError();
}

// ------------------------------------------------------ grouped (batches)
// Tasks of sketches with another precision return at once (the FP64 kernels
// of kernels_stream.hip take those).
template <int NPASS>
__global__ __launch_bounds__(256) void kg_gram_bf16(const GroupSketch* __restrict__ SK,
                                                    const GroupRR* __restrict__ T) {
  const GroupRR t = T[blockIdx.z];
  const GroupSketch& s = SK[t.sk];
  if (s.npass != NPASS) return;
  const int nt = s.mp / 32;
  if (static_cast<int>(blockIdx.x) >= nt * (nt + 1) / 2) return;
  gram_bf16_body<NPASS>(t.cur ? s.C1 : s.C0, s.ldc, s.mp, s.ldc, s.Gp, blockIdx.x, 0);
}

template <int NPASS>
__global__ __launch_bounds__(256) void kg_rebuild_bf16(const GroupSketch* __restrict__ SK,
                                                       const GroupRR* __restrict__ T) {
  const GroupRR t = T[blockIdx.z];
  const GroupSketch& s = SK[t.sk];
  if (s.npass != NPASS) return;
  if (static_cast<int>(blockIdx.x) >= s.ldc / 64 || static_cast<int>(blockIdx.y) * 32 >= s.rp.keep) return;
  rebuild_bf16_body<NPASS>(s.Ut, t.cur ? s.C1 : s.C0, s.ldc, s.mp, s.rp.keep, t.cur ? s.C0 : s.C1,
                           blockIdx.x, blockIdx.y);
}

hipError_t launch_group_gram_lowp(const GroupSketch* sk, const GroupRR* t, int nt, int max_mp, bool one,
                                  bool three, hipStream_t s) {
  if (nt <= 0) return hipSuccess;
  const int T = max_mp / 32;
  const dim3 g(T * (T + 1) / 2, 1, nt);
  if (one) hipLaunchKernelGGL(kg_gram_bf16<1>, g, dim3(256), 0, s, sk, t);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && three) {
    hipLaunchKernelGGL(kg_gram_bf16<3>, g, dim3(256), 0, s, sk, t);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_group_rebuild_lowp(const GroupSketch* sk, const GroupRR* t, int nt, int max_ldc,
                                     int max_keep, bool one, bool three, hipStream_t s) {
  if (nt <= 0 || max_keep <= 0) return hipSuccess;
  const dim3 g(max_ldc / 64, (max_keep + 31) / 32, nt);
  if (one) hipLaunchKernelGGL(kg_rebuild_bf16<1>, g, dim3(256), 0, s, sk, t);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && three) {
    hipLaunchKernelGGL(kg_rebuild_bf16<3>, g, dim3(256), 0, s, sk, t);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace fdsk
