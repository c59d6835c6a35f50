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

// ------------------------------------------------ pre-split BF16 operands
// The buffer's hi and lo halves, H = bf16(C) and L = bf16(C - H), written
// once per ReduceRank (rows64 = mp rounded up to 64; rows >= mp are zero)
// and read by the Gram and the rebuild below instead of splitting FP64
// operands inside their loops.
size_t bf16_workspace_bytes(int mp, int ldc) {
  const size_t rows64 = static_cast<size_t>((mp + 63) / 64 * 64);
  return 2 * rows64 * static_cast<size_t>(ldc) * sizeof(uint16_t);
}

// Row r, columns bx*256 + tid (+ nbx*256 ...).
__device__ __forceinline__ void split_bf16_body(const double* __restrict__ C, int ldc, int mp,
                                                uint16_t* __restrict__ H, uint16_t* __restrict__ L,
                                                int bx, int r, int nbx) {
  for (int c = bx * 256 + threadIdx.x; c < ldc; c += nbx * 256) {
    uint16_t hb = 0, lb = 0;
    if (r < mp) split_bits(C[static_cast<int64_t>(r) * ldc + c], hb, lb);
    H[static_cast<int64_t>(r) * ldc + c] = hb;
    L[static_cast<int64_t>(r) * ldc + c] = lb;
  }
}

__global__ __launch_bounds__(256) void k_split_bf16(const double* __restrict__ C, int ldc, int mp,
                                                    uint16_t* __restrict__ H, uint16_t* __restrict__ L) {
  split_bf16_body(C, ldc, mp, H, L, blockIdx.x, blockIdx.y, gridDim.x);
}

// G partials on lower-triangular 64x64 tiles of the pre-split buffer, split-K
// in chunks of kchunk (a multiple of 64).  Four waves; wave (wi, wj) owns the
// 32x32 block at (32 wi, 32 wj) as 2x2 16x16 tiles.  A 64-column K slab of
// the hi (and lo) rows of both tile rows is staged in LDS per step.
constexpr int kBt = 64, kBk = 64, kBpad = 8;

template <int NPASS>
__device__ __forceinline__ void gram_bf16t_body(const uint16_t* __restrict__ H, const uint16_t* __restrict__ L,
                                                int ldc, int mp, int kchunk, double* __restrict__ Gpart,
                                                int tile, int ks) {
  int ti = static_cast<int>((sqrtf(8.0f * tile + 1.0f) - 1.0f) * 0.5f);
  while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
  while (ti * (ti + 1) / 2 > tile) --ti;
  const int tj = tile - ti * (ti + 1) / 2;
  const int k0 = ks * kchunk;
  const int k1 = min(ldc, k0 + kchunk);
  __shared__ __attribute__((aligned(16))) uint16_t Ah[kBt][kBk + kBpad], Bh[kBt][kBk + kBpad];
  __shared__ __attribute__((aligned(16))) uint16_t Al[NPASS == 3 ? kBt : 1][kBk + kBpad];
  __shared__ __attribute__((aligned(16))) uint16_t Bl[NPASS == 3 ? kBt : 1][kBk + kBpad];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wi = w >> 1, wj = w & 1, li = lane & 15, lq = lane >> 4;
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t ra = static_cast<int64_t>(ti * kBt) * ldc, rb = static_cast<int64_t>(tj * kBt) * ldc;
  for (int kk = k0; kk < k1; kk += kBk) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int idx = tid + 256 * p, r = idx >> 3, c = (idx & 7) * 8;
      const int64_t o = static_cast<int64_t>(r) * ldc + kk + c;
      *reinterpret_cast<uint4*>(&Ah[r][c]) = *reinterpret_cast<const uint4*>(H + ra + o);
      *reinterpret_cast<uint4*>(&Bh[r][c]) = *reinterpret_cast<const uint4*>(H + rb + o);
      if (NPASS == 3) {
        *reinterpret_cast<uint4*>(&Al[r][c]) = *reinterpret_cast<const uint4*>(L + ra + o);
        *reinterpret_cast<uint4*>(&Bl[r][c]) = *reinterpret_cast<const uint4*>(L + rb + o);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k2 = 0; k2 < kBk; k2 += 32) {
      bf16x8_t ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int r = wi * 32 + a * 16 + li;
        ah[a] = *reinterpret_cast<const bf16x8_t*>(&Ah[r][k2 + 8 * lq]);
        if (NPASS == 3) al[a] = *reinterpret_cast<const bf16x8_t*>(&Al[r][k2 + 8 * lq]);
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int r = wj * 32 + b * 16 + li;
        bh[b] = *reinterpret_cast<const bf16x8_t*>(&Bh[r][k2 + 8 * lq]);
        if (NPASS == 3) bl[b] = *reinterpret_cast<const bf16x8_t*>(&Bl[r][k2 + 8 * lq]);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma_split<NPASS>(ah[a], al[a], bh[b], bl[b], acc[a][b]);
    }
    __syncthreads();
  }
  double* out = Gpart + static_cast<int64_t>(ks) * mp * mp;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = ti * kBt + wi * 32 + a * 16 + 4 * lq + v;
        const int col = tj * kBt + wj * 32 + b * 16 + li;
        if (row < mp && col < mp) out[static_cast<int64_t>(row) * mp + col] = static_cast<double>(acc[a][b][v]);
      }
}

template <int NPASS>
__global__ __launch_bounds__(256) void k_gram_bf16t(const uint16_t* __restrict__ H, const uint16_t* __restrict__ L,
                                                    int ldc, int mp, int kchunk, double* __restrict__ Gpart) {
  gram_bf16t_body<NPASS>(H, L, ldc, mp, kchunk, Gpart, blockIdx.x, blockIdx.y);
}

// out[0:keep, :] = Ut[0:keep, 0:mp] * C with C's hi/lo from the pre-split
// arrays (Ut is split in the loop: it is small).  Tile RT rows (32 or 64) x
// 64 columns; wave w owns rows (w>>1)*RT/2.. as RT/32 16-row MFMA tiles.
// C's 32x64 slab is staged transposed in LDS so that each B fragment is one
// 16-byte read.  Ut rows past mp load as zero.
template <int NPASS, int RT>
__device__ __forceinline__ void rebuild_bf16t_body(const double* __restrict__ Ut, const uint16_t* __restrict__ H,
                                                   const uint16_t* __restrict__ L, int ldc, int mp, int keep,
                                                   double* __restrict__ out, int bx, int by,
                                                   uint16_t* __restrict__ Ho = nullptr,
                                                   uint16_t* __restrict__ Lo = nullptr) {
  static_assert(RT == 32 || RT == 64, "rebuild rows per workgroup");
  constexpr int RA = RT / 32;
  const int r0 = by * RT, c0 = bx * 64;
  __shared__ double As[RT][33];
  __shared__ __attribute__((aligned(16))) uint16_t BhT[64][32 + kBpad];
  __shared__ __attribute__((aligned(16))) uint16_t BlT[NPASS == 3 ? 64 : 1][32 + kBpad];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wi = w >> 1, wj = w & 1, li = lane & 15, lq = lane >> 4;
  f32x4 acc[RA][2];
#pragma unroll
  for (int a = 0; a < RA; ++a) acc[a][0] = acc[a][1] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < mp; k0 += 32) {
#pragma unroll
    for (int e = 0; e < RT / 8; ++e) {
      const int idx = tid + e * 256, r = idx >> 5, c = idx & 31;
      As[r][c] = (r0 + r < mp) ? Ut[static_cast<int64_t>(r0 + r) * mp + k0 + c] : 0.0;
    }
    {
      const int kr = tid >> 3, nc = (tid & 7) * 8;
      const int64_t o = static_cast<int64_t>(k0 + kr) * ldc + c0 + nc;
      const uint4 hv = *reinterpret_cast<const uint4*>(H + o);
      const uint16_t* hs = reinterpret_cast<const uint16_t*>(&hv);
#pragma unroll
      for (int t = 0; t < 8; ++t) BhT[nc + t][kr] = hs[t];
      if (NPASS == 3) {
        const uint4 lv = *reinterpret_cast<const uint4*>(L + o);
        const uint16_t* ls = reinterpret_cast<const uint16_t*>(&lv);
#pragma unroll
        for (int t = 0; t < 8; ++t) BlT[nc + t][kr] = ls[t];
      }
    }
    __syncthreads();
    const int n0 = wj * 32 + li, n1 = n0 + 16;
    const bf16x8_t b0h = *reinterpret_cast<const bf16x8_t*>(&BhT[n0][8 * lq]);
    const bf16x8_t b1h = *reinterpret_cast<const bf16x8_t*>(&BhT[n1][8 * lq]);
    bf16x8_t b0l = b0h, b1l = b1h;
    if (NPASS == 3) {
      b0l = *reinterpret_cast<const bf16x8_t*>(&BlT[n0][8 * lq]);
      b1l = *reinterpret_cast<const bf16x8_t*>(&BlT[n1][8 * lq]);
    }
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      bf16x8_t ah, al;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        __bf16 h, l;
        split_bf16(As[wi * (RT / 2) + a * 16 + li][8 * lq + t], h, l);
        ah[t] = h;
        al[t] = l;
      }
      acc[a][0] = mfma_split<NPASS>(ah, al, b0h, b0l, acc[a][0]);
      acc[a][1] = mfma_split<NPASS>(ah, al, b1h, b1l, acc[a][1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < RA; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = r0 + wi * (RT / 2) + a * 16 + 4 * lq + v;
      if (row < keep) {
        const int64_t o = static_cast<int64_t>(row) * ldc + c0 + wj * 32 + li;
        const double x0 = static_cast<double>(acc[a][0][v]), x1 = static_cast<double>(acc[a][1][v]);
        out[o] = x0;
        out[o + 16] = x1;
        if (Ho) {
          uint16_t hb, lb;
          split_bits(x0, hb, lb);
          Ho[o] = hb;
          Lo[o] = lb;
          split_bits(x1, hb, lb);
          Ho[o + 16] = hb;
          Lo[o + 16] = lb;
        }
      }
    }
}

// The same product with Ut also pre-split (hi rows in Uh, lo rows mp x mp
// further on, written by the shrink): each A fragment is one 16-byte load of
// 8 consecutive bf16 of a Ut row, straight from global memory, so no Ut
// staging or split runs in the loop.  Rows of Uh at or past keep hold
// whatever they hold; they only reach output rows past keep, which are not
// stored.
template <int NPASS, int RT>
__device__ __forceinline__ void rebuild_bf16u_body(const uint16_t* __restrict__ Uh, const uint16_t* __restrict__ H,
                                                   const uint16_t* __restrict__ L, int ldc, int mp, int keep,
                                                   double* __restrict__ out, int bx, int by,
                                                   uint16_t* __restrict__ Ho, uint16_t* __restrict__ Lo, bool w64) {
  static_assert(RT == 32 || RT == 64, "rebuild rows per workgroup");
  constexpr int RA = RT / 32;
  const int r0 = by * RT, c0 = bx * 64;
  __shared__ __attribute__((aligned(16))) uint16_t BhT[64][32 + kBpad];
  __shared__ __attribute__((aligned(16))) uint16_t BlT[NPASS == 3 ? 64 : 1][32 + kBpad];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wi = w >> 1, wj = w & 1, li = lane & 15, lq = lane >> 4;
  const uint16_t* Ul = Uh + static_cast<int64_t>(mp) * mp;
  f32x4 acc[RA][2];
#pragma unroll
  for (int a = 0; a < RA; ++a) acc[a][0] = acc[a][1] = f32x4{0.f, 0.f, 0.f, 0.f};
  int64_t ua[RA];
#pragma unroll
  for (int a = 0; a < RA; ++a) {
    const int row = min(r0 + wi * (RT / 2) + a * 16 + li, mp - 1);
    ua[a] = static_cast<int64_t>(row) * mp + 8 * lq;
  }
  for (int k0 = 0; k0 < mp; k0 += 32) {
    bf16x8_t ah[RA], al[RA];
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      ah[a] = *reinterpret_cast<const bf16x8_t*>(Uh + ua[a] + k0);
      al[a] = (NPASS == 3) ? *reinterpret_cast<const bf16x8_t*>(Ul + ua[a] + k0) : ah[a];
    }
    {
      const int kr = tid >> 3, nc = (tid & 7) * 8;
      const int64_t o = static_cast<int64_t>(k0 + kr) * ldc + c0 + nc;
      const uint4 hv = *reinterpret_cast<const uint4*>(H + o);
      const uint16_t* hs = reinterpret_cast<const uint16_t*>(&hv);
#pragma unroll
      for (int t = 0; t < 8; ++t) BhT[nc + t][kr] = hs[t];
      if (NPASS == 3) {
        const uint4 lv = *reinterpret_cast<const uint4*>(L + o);
        const uint16_t* ls = reinterpret_cast<const uint16_t*>(&lv);
#pragma unroll
        for (int t = 0; t < 8; ++t) BlT[nc + t][kr] = ls[t];
      }
    }
    __syncthreads();
    const int n0 = wj * 32 + li, n1 = n0 + 16;
    const bf16x8_t b0h = *reinterpret_cast<const bf16x8_t*>(&BhT[n0][8 * lq]);
    const bf16x8_t b1h = *reinterpret_cast<const bf16x8_t*>(&BhT[n1][8 * lq]);
    bf16x8_t b0l = b0h, b1l = b1h;
    if (NPASS == 3) {
      b0l = *reinterpret_cast<const bf16x8_t*>(&BlT[n0][8 * lq]);
      b1l = *reinterpret_cast<const bf16x8_t*>(&BlT[n1][8 * lq]);
    }
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      acc[a][0] = mfma_split<NPASS>(ah[a], al[a], b0h, b0l, acc[a][0]);
      acc[a][1] = mfma_split<NPASS>(ah[a], al[a], b1h, b1l, acc[a][1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < RA; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = r0 + wi * (RT / 2) + a * 16 + 4 * lq + v;
      if (row < keep) {
        const int64_t o = static_cast<int64_t>(row) * ldc + c0 + wj * 32 + li;
        const double x0 = static_cast<double>(acc[a][0][v]), x1 = static_cast<double>(acc[a][1][v]);
        if (w64) {
          out[o] = x0;
          out[o + 16] = x1;
        }
        uint16_t hb, lb;
        split_bits(x0, hb, lb);
        Ho[o] = hb;
        Lo[o] = lb;
        split_bits(x1, hb, lb);
        Ho[o + 16] = hb;
        Lo[o + 16] = lb;
      }
    }
}

template <int NPASS, int RT>
__global__ __launch_bounds__(256) void k_rebuild_bf16t(const double* __restrict__ Ut, const uint16_t* __restrict__ H,
                                                       const uint16_t* __restrict__ L, int ldc, int mp, int keep,
                                                       double* __restrict__ out) {
  rebuild_bf16t_body<NPASS, RT>(Ut, H, L, ldc, mp, keep, out, blockIdx.x, blockIdx.y);
}

hipError_t launch_split_bf16(const double* C, int ldc, int mp, void* bfw, hipStream_t s) {
  const int rows64 = (mp + 63) / 64 * 64;
  uint16_t* H = static_cast<uint16_t*>(bfw);
  uint16_t* L = H + static_cast<size_t>(rows64) * ldc;
  hipLaunchKernelGGL(k_split_bf16, dim3((ldc + 255) / 256, rows64), dim3(256), 0, s, C, ldc, mp, H, L);
  return hipGetLastError();
}

hipError_t launch_gram_lowp(const double* C, int ldc, int mp, double* Gpart, int ksplit_max, double* G,
                            int npass, void* bfw, hipStream_t s, int ksplit_req) {
  if (bfw) {
    const int rows64 = (mp + 63) / 64 * 64;
    uint16_t* H = static_cast<uint16_t*>(bfw);
    uint16_t* L = H + static_cast<size_t>(rows64) * ldc;
    hipLaunchKernelGGL(k_split_bf16, dim3((ldc + 255) / 256, rows64), dim3(256), 0, s, C, ldc, mp, H, L);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int T = rows64 / kBt;
    const int ntiles = T * (T + 1) / 2;
    int ksplit = ksplit_req > 0 ? ksplit_req : gram_ksplit_default(ntiles, ldc);
    ksplit = std::max(1, std::min(ksplit, ksplit_max));
    int kchunk = (ldc + ksplit - 1) / ksplit;
    kchunk = (kchunk + kBk - 1) / kBk * kBk;
    ksplit = (ldc + kchunk - 1) / kchunk;
    if (npass == 3)
      hipLaunchKernelGGL(k_gram_bf16t<3>, dim3(ntiles, ksplit), dim3(256), 0, s, H, L, ldc, mp, kchunk, Gpart);
    else
      hipLaunchKernelGGL(k_gram_bf16t<1>, dim3(ntiles, ksplit), dim3(256), 0, s, H, L, ldc, mp, kchunk, Gpart);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_gram_reduce(Gpart, ksplit, mp, G, s);
  }
  const int T = mp / 32;
  const int ntiles = T * (T + 1) / 2;
  int ksplit = ksplit_req > 0 ? ksplit_req : gram_ksplit_default(ntiles, ldc);
  ksplit = std::max(1, std::min(ksplit, ksplit_max));
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
                               int npass, const void* bfw, hipStream_t s, int rt) {
  if (keep <= 0) return hipSuccess;
  if (rt != 32 && rt != 64) return hipErrorInvalidValue;
  if (bfw) {
    const int rows64 = (mp + 63) / 64 * 64;
    const uint16_t* H = static_cast<const uint16_t*>(bfw);
    const uint16_t* L = H + static_cast<size_t>(rows64) * ldc;
    const dim3 g(ldc / 64, (keep + rt - 1) / rt);
    if (npass == 3 && rt == 64)
      hipLaunchKernelGGL((k_rebuild_bf16t<3, 64>), g, dim3(256), 0, s, Ut, H, L, ldc, mp, keep, out);
    else if (npass == 3)
      hipLaunchKernelGGL((k_rebuild_bf16t<3, 32>), g, dim3(256), 0, s, Ut, H, L, ldc, mp, keep, out);
    else if (rt == 64)
      hipLaunchKernelGGL((k_rebuild_bf16t<1, 64>), g, dim3(256), 0, s, Ut, H, L, ldc, mp, keep, out);
    else
      hipLaunchKernelGGL((k_rebuild_bf16t<1, 32>), g, dim3(256), 0, s, Ut, H, L, ldc, mp, keep, out);
    return hipGetLastError();
  }
  // Without pre-split halves: 32-row tiles, C split inside the product.
  dim3 grid(ldc / 64, (keep + 31) / 32);
  if (npass == 3)
    hipLaunchKernelGGL(k_rebuild_bf16<3>, grid, dim3(256), 0, s, Ut, C, ldc, mp, keep, out);
  else
    hipLaunchKernelGGL(k_rebuild_bf16<1>, grid, dim3(256), 0, s, Ut, C, ldc, mp, keep, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------- FP8
// Per-row e4m3 split of the FP64 buffer: hi = e4m3(x / s) with s = amax/240,
// lo = e4m3((x - s hi) / t) with t the same for the residual (240 keeps every
// value inside the e4m3 range whichever bias the hardware format uses).  The
// Gram G_ij = s_i s_j (hi_i . hi_j) + s_i t_j (hi_i . lo_j) + t_i s_j (lo_i .
// hi_j): three FP8 matrix-core products, FP32 accumulation, scales in FP64.
constexpr double kFp8Range = 240.0;

// Byte u (0..3) of a word of e4m3 codes as a float.
__device__ __forceinline__ float fp8_byte(int w, int u) {
  switch (u) {
    case 0: return __builtin_amdgcn_cvt_f32_fp8(w, 0);
    case 1: return __builtin_amdgcn_cvt_f32_fp8(w, 1);
    case 2: return __builtin_amdgcn_cvt_f32_fp8(w, 2);
    default: return __builtin_amdgcn_cvt_f32_fp8(w, 3);
  }
}

__device__ __forceinline__ double block_max_256(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  return m;
}

// One workgroup per buffer row; four consecutive elements per thread and
// pass (packed into one 32-bit word of e4m3 codes).
__global__ __launch_bounds__(256) void k_quant_fp8(const double* __restrict__ C, int ldc,
                                                   uint32_t* __restrict__ Qh, uint32_t* __restrict__ Ql,
                                                   double* __restrict__ sc, int mp) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  const double* x = C + static_cast<int64_t>(r) * ldc;
  double amax = 0.0;
  for (int c = threadIdx.x; c < ldc; c += 256) amax = fmax(amax, fabs(x[c]));
  amax = block_max_256(amax, red);
  const double s = (amax > 0.0) ? amax / kFp8Range : 1.0;
  const double inv_s = 1.0 / s;
  const int nw = ldc / 4;
  double rmax = 0.0;
  for (int q = threadIdx.x; q < nw; q += 256) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = x[4 * q + u];
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(static_cast<float>(v[0] * inv_s), static_cast<float>(v[1] * inv_s), 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(static_cast<float>(v[2] * inv_s), static_cast<float>(v[3] * inv_s), w, true);
    Qh[static_cast<int64_t>(r) * nw + q] = static_cast<uint32_t>(w);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double hv = static_cast<double>(fp8_byte(w, u)) * s;
      rmax = fmax(rmax, fabs(v[u] - hv));
    }
  }
  rmax = block_max_256(rmax, red);
  const double t = (rmax > 0.0) ? rmax / kFp8Range : 1.0;
  const double inv_t = 1.0 / t;
  for (int q = threadIdx.x; q < nw; q += 256) {
    const int w = static_cast<int>(Qh[static_cast<int64_t>(r) * nw + q]);
    float res[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      res[u] = static_cast<float>((x[4 * q + u] - static_cast<double>(fp8_byte(w, u)) * s) * inv_t);
    int wl = __builtin_amdgcn_cvt_pk_fp8_f32(res[0], res[1], 0, false);
    wl = __builtin_amdgcn_cvt_pk_fp8_f32(res[2], res[3], wl, true);
    Ql[static_cast<int64_t>(r) * nw + q] = static_cast<uint32_t>(wl);
  }
  if (threadIdx.x == 0) {
    sc[r] = s;
    sc[mp + r] = t;
  }
}

__device__ __forceinline__ f32x4 mfma_fp8(long a, long b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
}

// G partials on lower-triangular 32x32 tiles with split-K (see k_gram_f64);
// 16x16x32 FP8 steps: lane = i + 16 q holds A[i][8q..8q+7] and B[8q..8q+7][i]
// (eight e4m3 codes in one 64-bit word); the result lane = j + 16 q holds
// D[4q + v][j] in element v.
__global__ __launch_bounds__(256) void k_gram_fp8(const uint8_t* __restrict__ Qh,
                                                  const uint8_t* __restrict__ Ql,
                                                  const double* __restrict__ sc, int ldc, int mp,
                                                  int kchunk, double* __restrict__ Gpart) {
  const int tile = blockIdx.x;
  int ti = static_cast<int>((sqrtf(8.0f * tile + 1.0f) - 1.0f) * 0.5f);
  while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
  while (ti * (ti + 1) / 2 > tile) --ti;
  const int tj = tile - ti * (ti + 1) / 2;
  const int k0 = blockIdx.y * kchunk;
  const int k1 = min(ldc, k0 + kchunk);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wi = w >> 1, wj = w & 1;
  const int li = lane & 15, lq = lane >> 4;
  const int ra = ti * 32 + wi * 16 + li, rb = tj * 32 + wj * 16 + li;
  const long* ah_p = reinterpret_cast<const long*>(Qh + static_cast<int64_t>(ra) * ldc);
  const long* al_p = reinterpret_cast<const long*>(Ql + static_cast<int64_t>(ra) * ldc);
  const long* bh_p = reinterpret_cast<const long*>(Qh + static_cast<int64_t>(rb) * ldc);
  const long* bl_p = reinterpret_cast<const long*>(Ql + static_cast<int64_t>(rb) * ldc);
  f32x4 hh = {0.f, 0.f, 0.f, 0.f}, hl = hh, lh = hh;
  for (int kk = k0; kk < k1; kk += 32) {
    const int o = (kk >> 3) + lq;
    const long ah = ah_p[o], al = al_p[o], bh = bh_p[o], bl = bl_p[o];
    hh = mfma_fp8(ah, bh, hh);
    hl = mfma_fp8(ah, bl, hl);
    lh = mfma_fp8(al, bh, lh);
  }
  double* out = Gpart + static_cast<int64_t>(blockIdx.y) * mp * mp;
  const int col = tj * 32 + wj * 16 + li;
  const double scol = sc[col], tcol = sc[mp + col];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = ti * 32 + wi * 16 + 4 * lq + v;
    const double srow = sc[row], trow = sc[mp + row];
    out[static_cast<int64_t>(row) * mp + col] =
        srow * scol * static_cast<double>(hh[v]) + srow * tcol * static_cast<double>(hl[v]) +
        trow * scol * static_cast<double>(lh[v]);
  }
}

hipError_t launch_gram_fp8(const double* C, int ldc, int mp, void* q8, double* Gpart, int ksplit_max,
                           double* G, hipStream_t s, int ksplit_req) {
  uint8_t* Qh = static_cast<uint8_t*>(q8);
  uint8_t* Ql = Qh + static_cast<size_t>(mp) * ldc;
  double* sc = reinterpret_cast<double*>(Ql + static_cast<size_t>(mp) * ldc);
  hipLaunchKernelGGL(k_quant_fp8, dim3(mp), dim3(256), 0, s, C, ldc, reinterpret_cast<uint32_t*>(Qh),
                     reinterpret_cast<uint32_t*>(Ql), sc, mp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int T = mp / 32;
  const int ntiles = T * (T + 1) / 2;
  int ksplit = ksplit_req > 0 ? ksplit_req : gram_ksplit_default(ntiles, ldc);
  ksplit = std::max(1, std::min(ksplit, ksplit_max));
  int kchunk = (ldc + ksplit - 1) / ksplit;
  kchunk = (kchunk + 31) / 32 * 32;
  ksplit = (ldc + kchunk - 1) / kchunk;
  hipLaunchKernelGGL(k_gram_fp8, dim3(ntiles, ksplit), dim3(256), 0, s, Qh, Ql, sc, ldc, mp, kchunk, Gpart);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_gram_reduce(Gpart, ksplit, mp, G, s);
}

size_t fp8_workspace_bytes(int mp, int ldc) {
  return 2 * static_cast<size_t>(mp) * ldc + 2 * static_cast<size_t>(mp) * 8;
}

// ------------------------------------------------------ grouped (batches)
// Tasks of sketches with another precision return at once (the FP64 kernels
// of kernels_stream.hip take those).  Each buffer keeps its bf16 halves
// beside its FP64 rows (s.bh0 for C0, s.bh1 for C1: hi rows then lo rows,
// rows64 x ldc each): the ingest and the rebuild write them with the rows
// (the same split as k_split_bf16, so the same bits), and the Gram and the
// next rebuild read them; no separate split pass runs.
// Split-K as the FP64 grouped Gram: K slice blockIdx.y of the task's slice
// length into partial blockIdx.y of its Gp.
template <int NPASS>
__global__ __launch_bounds__(256) void kg_gram_bf16(const GroupSketch* __restrict__ SK,
                                                    const GroupRR* __restrict__ T, int kc) {
  const GroupRR t = T[blockIdx.z];
  const GroupSketch& s = SK[t.sk];
  if (s.npass != NPASS) return;
  const int rows64 = (s.mp + 63) / 64 * 64, nt = rows64 / kBt;
  if (static_cast<int>(blockIdx.x) >= nt * (nt + 1) / 2) return;
  const int kchunk = task_kchunk(kc >= 0 ? kc : s.kchunk, s.ldc);
  if (static_cast<int>(blockIdx.y) * kchunk >= s.ldc) return;
  const uint16_t* H = t.cur ? s.bh1 : s.bh0;
  gram_bf16t_body<NPASS>(H, H + static_cast<int64_t>(rows64) * s.ldc, s.ldc, s.mp, kchunk, s.Gp, blockIdx.x,
                         blockIdx.y);
}

template <int NPASS, int RT>
__global__ __launch_bounds__(256) void kg_rebuild_bf16(const GroupSketch* __restrict__ SK,
                                                       const GroupRR* __restrict__ T) {
  const GroupRR t = T[blockIdx.z];
  const GroupSketch& s = SK[t.sk];
  if (s.npass != NPASS) return;
  if (static_cast<int>(blockIdx.x) >= s.ldc / 64 || static_cast<int>(blockIdx.y) * RT >= s.rp.keep) return;
  const int64_t half = static_cast<int64_t>((s.mp + 63) / 64 * 64) * s.ldc;
  const uint16_t* H = t.cur ? s.bh1 : s.bh0;
  uint16_t* Ho = t.cur ? s.bh0 : s.bh1;
  rebuild_bf16u_body<NPASS, RT>(s.uh, H, H + half, s.ldc, s.mp, s.rp.keep, t.cur ? s.C0 : s.C1, blockIdx.x,
                                blockIdx.y, Ho, Ho + half, t.w64 != 0);
}

hipError_t launch_group_gram_lowp(const GroupSketch* sk, const GroupRR* t, int nt, int max_mp, int max_ldc,
                                  bool one, bool three, int ks, int kc, hipStream_t s) {
  if (nt <= 0) return hipSuccess;
  if (ks < 1 || ks > kGpParts || (kc > 0 && kc % 64)) return hipErrorInvalidValue;
  const int rows64 = (max_mp + 63) / 64 * 64, T = rows64 / kBt;
  hipError_t e = hipSuccess;
  const dim3 g(T * (T + 1) / 2, ks, nt);
  if (e == hipSuccess && one) {
    hipLaunchKernelGGL(kg_gram_bf16<1>, g, dim3(256), 0, s, sk, t, kc);
    e = hipGetLastError();
  }
  if (e == hipSuccess && three) {
    hipLaunchKernelGGL(kg_gram_bf16<3>, g, dim3(256), 0, s, sk, t, kc);
    e = hipGetLastError();
  }
  return e;
}

template <int RT>
hipError_t group_rebuild_lowp_rt(const GroupSketch* sk, const GroupRR* t, int nt, int max_ldc, int max_keep,
                                 bool one, bool three, hipStream_t s) {
  const dim3 g(max_ldc / 64, (max_keep + RT - 1) / RT, nt);
  if (one) hipLaunchKernelGGL((kg_rebuild_bf16<1, RT>), g, dim3(256), 0, s, sk, t);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && three) {
    hipLaunchKernelGGL((kg_rebuild_bf16<3, RT>), g, dim3(256), 0, s, sk, t);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_group_rebuild_lowp(const GroupSketch* sk, const GroupRR* t, int nt, int max_ldc,
                                     int max_keep, bool one, bool three, int rt, hipStream_t s) {
  if (nt <= 0 || max_keep <= 0) return hipSuccess;
  if (rt == 64) return group_rebuild_lowp_rt<64>(sk, t, nt, max_ldc, max_keep, one, three, s);
  if (rt == 32) return group_rebuild_lowp_rt<32>(sk, t, nt, max_ldc, max_keep, one, three, s);
  return hipErrorInvalidValue;
}

}  // namespace fdsk
