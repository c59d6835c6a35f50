// Jacobi building blocks of the Jacobi eigensolvers (device code only).
//
// The buffer's SVD (Algorithm 1) is reached through G = C C^T = U diag(lambda) U^T:
// sigma_j^2 = lambda_j and the rebuilt rows are diag(sigma'/sigma) U^T C.
#pragma once
#include "fdsk_device.hpp"
#include "fdsk_kernels.hpp"

namespace fdsk {

constexpr int LN = kLdsEigMax;       // largest n of the LDS-resident solver
constexpr int LLD = LN + 1;          // padded leading dimension in LDS
constexpr double kLdsTol = 1e-15;    // rotate (p,q) only if |g_pq| > tol*sqrt(|g_pp g_qq|)
constexpr int BW = 8;                // block width; a panel task owns 2 blocks = 16 columns
constexpr double kOuterTol = 1e-14;  // one-sided: columns orthogonal to this relative level
constexpr double kInnerTol = 1e-15;
constexpr int kInnerSweeps = 1;

// Round-robin ("circle") ordering of n (even) indices: step s pairs position
// k with position n-1-k of [0, 1+(s mod n-1), 1+(s+1 mod n-1), ...].
__device__ __forceinline__ int rr_slot(int pos, int step, int n) {
  return pos == 0 ? 0 : 1 + (pos - 1 + step) % (n - 1);
}
// Same without integer division (step < n - 1).
__device__ __forceinline__ int rr_fast(int pos, int step, int n) {
  if (pos == 0) return 0;
  int s = pos - 1 + step;
  if (s >= n - 1) s -= n - 1;
  return 1 + s;
}

// LDS scratch of the LDS-resident two-sided solver.
struct LdsEigSmem {
  double* Gs;     // LN * LLD
  double* Vs;     // LN * LLD, column-major (column j contiguous)
  double* cs;     // LN: c values then s values
  short* pi;      // LN / 2
  short* qi;      // LN / 2
  int* nrot;
  double* gmax;
};

// Cyclic two-sided Jacobi on the m x m symmetric G (row-major, ld mp) with G
// and V in LDS, executed by the whole workgroup (any blockDim multiple of 64).
// Each step rotates n/2 disjoint index pairs; every 2x2 block of G is
// updated independently.  A sweep without any rotation ends the solve.
// Output: lam[j] = final diagonal, Vout column-major (ld mp), zero padded.
__device__ void eig_lds_body(const double* __restrict__ G, int m, int mp, double* __restrict__ lam,
                             double* __restrict__ Vout, DevStats* __restrict__ st, LdsEigSmem sm) {
  double* Gs = sm.Gs;
  double* Vs = sm.Vs;
  double* cs = sm.cs;
  const int n = (m + 1) & ~1;
  const int np2 = n / 2;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int rows_per = nt >> 5;       // thread grid nt/32 x 32 for the 2x2 blocks
  const int vgroups = nt >> 7;        // V: groups of 128 lanes along a column pair
  if (tid == 0) *sm.gmax = 0.0;
  __syncthreads();
  double lmax = 0.0;
  for (int e = tid; e < n * n; e += nt) {
    int i = e / n, j = e % n;
    double g = (i < m && j < m) ? G[static_cast<int64_t>(i) * mp + j] : 0.0;
    Gs[i * LLD + j] = g;
    Vs[j * LLD + i] = (i == j) ? 1.0 : 0.0;
    lmax = fmax(lmax, fabs(g));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) lmax = fmax(lmax, __shfl_xor(lmax, off, 64));
  if ((tid & 63) == 0)   // non-negative doubles order as integers
    atomicMax(reinterpret_cast<unsigned long long*>(sm.gmax), __double_as_longlong(lmax));
  __syncthreads();
  // Entries below this are rounding noise of the largest one; never rotate on them.
  const double floor_abs = 1e-300 + 1e-17 * (*sm.gmax);

  int sweep = 0;
  for (; sweep < kMaxSweeps; ++sweep) {
    if (tid == 0) *sm.nrot = 0;
    __syncthreads();
    for (int step = 0; step < n - 1; ++step) {
      if (tid < np2) {
        int p = rr_fast(tid, step, n), q = rr_fast(n - 1 - tid, step, n);
        double app = Gs[p * LLD + p], aqq = Gs[q * LLD + q], apq = Gs[p * LLD + q];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > floor_abs && apq * apq > (kLdsTol * kLdsTol) * fabs(app * aqq)) {
          jacobi_rotation(app, aqq, apq, c, s);
          *sm.nrot = 1;
        }
        cs[tid] = c;
        cs[LN / 2 + tid] = s;
        sm.pi[tid] = static_cast<short>(p);
        sm.qi[tid] = static_cast<short>(q);
      }
      __syncthreads();
      // G <- J^T G J on 2x2 blocks (a <= b; the mirror block is written too).
      for (int a = tid >> 5; a < np2; a += rows_per) {
        const int pa = sm.pi[a], qa = sm.qi[a];
        const double ca = cs[a], sa = cs[LN / 2 + a];
        for (int b = tid & 31; b < np2; b += 32) {
          if (b < a) continue;
          const int pb = sm.pi[b], qb = sm.qi[b];
          const double cb = cs[b], sb = cs[LN / 2 + b];
          double g11 = Gs[pa * LLD + pb], g12 = Gs[pa * LLD + qb];
          double g21 = Gs[qa * LLD + pb], g22 = Gs[qa * LLD + qb];
          double r11 = ca * g11 - sa * g21, r12 = ca * g12 - sa * g22;
          double r21 = sa * g11 + ca * g21, r22 = sa * g12 + ca * g22;
          double n11 = cb * r11 - sb * r12, n12 = sb * r11 + cb * r12;
          double n21 = cb * r21 - sb * r22, n22 = sb * r21 + cb * r22;
          Gs[pa * LLD + pb] = n11;
          Gs[pa * LLD + qb] = n12;
          Gs[qa * LLD + pb] = n21;
          Gs[qa * LLD + qb] = n22;
          if (b != a) {
            Gs[pb * LLD + pa] = n11;
            Gs[qb * LLD + pa] = n12;
            Gs[pb * LLD + qa] = n21;
            Gs[qb * LLD + qa] = n22;
          }
        }
      }
      // V <- V J: lanes run along a column pair, so accesses are contiguous.
      for (int b = tid >> 7; b < np2; b += vgroups) {
        const int pb = sm.pi[b], qb = sm.qi[b];
        const double cb = cs[b], sb = cs[LN / 2 + b];
        for (int i = tid & 127; i < n; i += 128) {
          double vp = Vs[pb * LLD + i], vq = Vs[qb * LLD + i];
          Vs[pb * LLD + i] = cb * vp - sb * vq;
          Vs[qb * LLD + i] = sb * vp + cb * vq;
        }
      }
      __syncthreads();
    }
    const int rotated = *sm.nrot;
    __syncthreads();            // every thread has read nrot before it is reset
    if (rotated == 0) break;
  }
  if (tid == 0) {
    atomicAdd(&st->eig_sweeps, static_cast<unsigned long long>(sweep + 1));
    if (sweep == kMaxSweeps) atomicAdd(&st->eig_unconv, 1);
  }
  for (int j = tid; j < m; j += nt) lam[j] = Gs[j * LLD + j];
  for (int64_t e = tid; e < static_cast<int64_t>(mp) * mp; e += nt) {
    int j = static_cast<int>(e / mp), i = static_cast<int>(e % mp);
    Vout[e] = (i < m && j < m) ? Vs[j * LLD + i] : 0.0;
  }
}

// Wave-synchronous phase separator: LDS operations of one wave complete in
// order, so a compiler fence is enough between phases of a single wave.
__device__ __forceinline__ void wave_sync() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// One sweep of two-sided Jacobi on the 16x16 H (LDS, ld 17) accumulating Q,
// executed by a single wave (lane = threadIdx.x & 63).  The outer one-sided
// iteration revisits the panel until its columns are orthogonal.
__device__ void inner_jacobi16(double* Hs, double* Qs, double* cs) {
  const int lane = threadIdx.x & 63;
  for (int e = lane; e < 256; e += 64) Qs[(e >> 4) * 17 + (e & 15)] = ((e >> 4) == (e & 15)) ? 1.0 : 0.0;
  wave_sync();
  for (int sw = 0; sw < kInnerSweeps; ++sw) {
    for (int step = 0; step < 15; ++step) {
      if (lane < 8) {
        int p = rr_fast(lane, step, 16), q = rr_fast(15 - lane, step, 16);
        double hpq = Hs[p * 17 + q], hpp = Hs[p * 17 + p], hqq = Hs[q * 17 + q];
        double c = 1.0, sn = 0.0;
        if (hpq * hpq > (0.0625 * kInnerTol * kInnerTol) * fabs(hpp * hqq)) jacobi_rotation(hpp, hqq, hpq, c, sn);
        cs[lane] = c;
        cs[8 + lane] = sn;
      }
      wave_sync();
      {
        const int a = lane >> 3, b = lane & 7;
        const int pa = rr_fast(a, step, 16), qa = rr_fast(15 - a, step, 16);
        const int pb = rr_fast(b, step, 16), qb = rr_fast(15 - b, step, 16);
        const double ca = cs[a], sa = cs[8 + a], cb = cs[b], sb = cs[8 + b];
        double g11 = Hs[pa * 17 + pb], g12 = Hs[pa * 17 + qb], g21 = Hs[qa * 17 + pb], g22 = Hs[qa * 17 + qb];
        double r11 = ca * g11 - sa * g21, r12 = ca * g12 - sa * g22;
        double r21 = sa * g11 + ca * g21, r22 = sa * g12 + ca * g22;
        const int i0 = lane >> 3;   // Q <- Q J for rows i0 and i0 + 8, pair b
        double v0p = Qs[i0 * 17 + pb], v0q = Qs[i0 * 17 + qb];
        double v1p = Qs[(i0 + 8) * 17 + pb], v1q = Qs[(i0 + 8) * 17 + qb];
        wave_sync();
        Hs[pa * 17 + pb] = cb * r11 - sb * r12;
        Hs[pa * 17 + qb] = sb * r11 + cb * r12;
        Hs[qa * 17 + pb] = cb * r21 - sb * r22;
        Hs[qa * 17 + qb] = sb * r21 + cb * r22;
        Qs[i0 * 17 + pb] = cb * v0p - sb * v0q;
        Qs[i0 * 17 + qb] = sb * v0p + cb * v0q;
        Qs[(i0 + 8) * 17 + pb] = cb * v1p - sb * v1q;
        Qs[(i0 + 8) * 17 + qb] = sb * v1p + cb * v1q;
      }
      wave_sync();
    }
  }
}

// Column index of panel column c (0..15) for blocks bi, bj.
__device__ __forceinline__ int panel_col(int c, int bi, int bj) {
  return (c < 8) ? bi * BW + c : bj * BW + (c - 8);
}

// One wave: Ps[c*ldp + i] = X[col(c)*mp + i] (column-major X, mp x mp).
__device__ __forceinline__ void wave_load_panel(const double* __restrict__ X, int mp, int ldp, int bi,
                                                int bj, double* __restrict__ Ps) {
  const int lane = threadIdx.x & 63;
  const int half = mp >> 1;
  const int total = 16 * half;
  for (int base = lane; base < total; base += 64 * 8) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * 64;
      if (e < total) {
        int c = e / half, i2 = e - c * half;
        v[u] = reinterpret_cast<const double2*>(X + static_cast<int64_t>(panel_col(c, bi, bj)) * mp)[i2];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * 64;
      if (e < total) {
        int c = e / half, i2 = e - c * half;
        Ps[c * ldp + 2 * i2] = v[u].x;
        Ps[c * ldp + 2 * i2 + 1] = v[u].y;
      }
    }
  }
}

// One wave: H (16x16, ld 17) = P^T P over the panel's mp rows (matrix cores).
__device__ __forceinline__ void wave_panel_gram(const double* Ps, int ldp, int mp, double* Hs) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < mp; k0 += 4) {
    double a = Ps[li * ldp + k0 + lk];
    acc = mfma_f64(a, a, acc);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) Hs[(lk + 4 * v) * 17 + li] = acc[v];
}

// One wave: out[:, cols] = P Q for the mp x 16 panel (matrix cores).
__device__ __forceinline__ void wave_panel_times_q(const double* Ps, int ldp, int mp, const double* Qs,
                                                   double* out, int bi, int bj) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int col = panel_col(li, bi, bj);
  for (int i0 = 0; i0 < mp; i0 += 16) {
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < 16; k0 += 4) {
      double a = Ps[(k0 + lk) * ldp + i0 + li];
      double b = Qs[(k0 + lk) * 17 + li];
      acc = mfma_f64(a, b, acc);
    }
    double* o = out + static_cast<int64_t>(col) * mp + i0 + lk;
#pragma unroll
    for (int v = 0; v < 4; ++v) o[4 * v] = acc[v];
  }
}

// Does the 16x16 panel Gram show a pair of columns that is not orthogonal?
__device__ __forceinline__ bool wave_panel_needs_rotation(const double* Hs) {
  const int lane = threadIdx.x & 63;
  bool need = false;
  for (int e = lane; e < 256; e += 64) {
    int p = e >> 4, q = e & 15;
    if (p < q) {
      double hpq = Hs[p * 17 + q], hpp = Hs[p * 17 + p], hqq = Hs[q * 17 + q];
      if (hpp > 0.0 && hqq > 0.0 && hpq * hpq > (kOuterTol * kOuterTol) * (hpp * hqq)) need = true;
    }
  }
  return __any(need);
}

}  // namespace fdsk
