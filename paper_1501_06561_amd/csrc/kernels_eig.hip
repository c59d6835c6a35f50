// FP64 symmetric eigensolvers for the m x m Gram matrix of the sketch buffer.
//
// The buffer's SVD (Algorithm 1) is reached through G = C C^T = U diag(lambda) U^T:
// sigma_j^2 = lambda_j and the rebuilt rows are diag(sigma'/sigma) U^T C.
//
// * k_eig_lds  (m <= 100): cyclic two-sided Jacobi in one workgroup with G and
//   V resident in LDS; each step rotates n/2 disjoint index pairs (round-robin
//   ordering) and updates every 2x2 block of G independently.
// * k_eig_blk  (m <= 1024): one-sided block Jacobi (Hestenes) on W = G with
//   V accumulated.  A task orthogonalises a 16-column panel (two 8-column
//   blocks): H = P^T P on matrix cores, a two-sided Jacobi on the 16x16 H in
//   LDS gives Q, then P <- P Q and V_panel <- V_panel Q on matrix cores.
//   mp/16 workgroups run the disjoint block pairs of one round-robin step in
//   parallel, with a grid barrier between steps; a sweep with no rotation ends
//   the solve.  At convergence W = V diag(lambda) and lambda_j = v_j . w_j.
#include "fdsk_device.hpp"
#include "fdsk_kernels.hpp"

namespace fdsk {

// Round-robin ("circle") ordering of n (even) indices: step s pairs position
// k with position n-1-k of [0, 1+(s mod n-1), 1+(s+1 mod n-1), ...].
__device__ __forceinline__ int rr_slot(int pos, int step, int n) {
  return pos == 0 ? 0 : 1 + (pos - 1 + step) % (n - 1);
}

// ------------------------------------------------------------- LDS solver
constexpr int LN = kLdsEigMax;       // max n
constexpr int LLD = LN + 1;
constexpr double kLdsTol = 1e-15;    // rotate (p,q) only if |g_pq| > tol*sqrt(|g_pp g_qq|)

// Index at slot `pos` of the round-robin ordering (no integer division).
__device__ __forceinline__ int rr_fast(int pos, int step, int n) {
  if (pos == 0) return 0;
  int s = pos - 1 + step;
  if (s >= n - 1) s -= n - 1;
  return 1 + s;
}

__global__ __launch_bounds__(1024) void k_eig_lds(const double* __restrict__ G, int m, int mp,
                                                  double* __restrict__ lam,
                                                  double* __restrict__ Vout,
                                                  DevStats* __restrict__ st) {
  __shared__ double Gs[LN * LLD];
  __shared__ double Vs[LN * LLD];
  __shared__ double cs[LN];
  __shared__ short pi[LN / 2], qi[LN / 2];
  __shared__ int nrot;
  __shared__ double gmax;
  const int n = (m + 1) & ~1;
  const int np2 = n / 2;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) gmax = 0.0;
  __syncthreads();
  double lmax = 0.0;
  for (int e = tid; e < n * n; e += nt) {
    int i = e / n, j = e % n;
    double g = (i < m && j < m) ? G[static_cast<int64_t>(i) * mp + j] : 0.0;
    Gs[i * LLD + j] = g;
    Vs[j * LLD + i] = (i == j) ? 1.0 : 0.0;   // column-major: column j contiguous
    lmax = fmax(lmax, fabs(g));
  }
  lmax = fmax(lmax, __shfl_xor(lmax, 32, 64));
  lmax = fmax(lmax, __shfl_xor(lmax, 16, 64));
  lmax = fmax(lmax, __shfl_xor(lmax, 8, 64));
  lmax = fmax(lmax, __shfl_xor(lmax, 4, 64));
  lmax = fmax(lmax, __shfl_xor(lmax, 2, 64));
  lmax = fmax(lmax, __shfl_xor(lmax, 1, 64));
  if ((tid & 63) == 0) atomicMax(reinterpret_cast<unsigned long long*>(&gmax),
                                 __double_as_longlong(lmax));   // non-negative doubles order as integers
  __syncthreads();
  // Entries below this are rounding noise of the largest one; never rotate on them.
  const double floor_abs = 1e-300 + 1e-17 * gmax;

  int sweep = 0;
  for (; sweep < kMaxSweeps; ++sweep) {
    if (tid == 0) nrot = 0;
    __syncthreads();
    for (int step = 0; step < n - 1; ++step) {
      if (tid < np2) {
        int p = rr_fast(tid, step, n), q = rr_fast(n - 1 - tid, step, n);
        double app = Gs[p * LLD + p], aqq = Gs[q * LLD + q], apq = Gs[p * LLD + q];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > floor_abs && apq * apq > (kLdsTol * kLdsTol) * fabs(app * aqq)) {
          jacobi_rotation(app, aqq, apq, c, s);
          nrot = 1;
        }
        cs[tid] = c;
        cs[LN / 2 + tid] = s;
        pi[tid] = static_cast<short>(p);
        qi[tid] = static_cast<short>(q);
      }
      __syncthreads();
      // G <- J^T G J on 2x2 blocks (a <= b; the mirror block is written too).
      for (int a = tid >> 5; a < np2; a += 32) {
        const int pa = pi[a], qa = qi[a];
        const double ca = cs[a], sa = cs[LN / 2 + a];
        for (int b = (tid & 31) + 0; b < np2; b += 32) {
          if (b < a) continue;
          const int pb = pi[b], qb = qi[b];
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
      for (int b = tid >> 7; b < np2; b += 8) {
        const int pb = pi[b], qb = qi[b];
        const double cb = cs[b], sb = cs[LN / 2 + b];
        for (int i = tid & 127; i < n; i += 128) {
          double vp = Vs[pb * LLD + i], vq = Vs[qb * LLD + i];
          Vs[pb * LLD + i] = cb * vp - sb * vq;
          Vs[qb * LLD + i] = sb * vp + cb * vq;
        }
      }
      __syncthreads();
    }
    const int rotated = nrot;
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

// ------------------------------------------------------- block solver
constexpr int BW = 8;            // block width; a task owns 2 blocks = 16 columns
constexpr int PMAX = 1024;       // largest mp
constexpr double kOuterTol = 1e-14;
constexpr double kInnerTol = 1e-15;
constexpr int kInnerSweeps = 1;

struct BlkArgs {
  const double* G;
  int m, mp;
  double* W;
  double* V;
  double* lam;
  GridBar bar;
  int* rot;
  DevStats* st;
};

// Inner two-sided Jacobi on the 16x16 H (LDS), accumulating Q, run by wave 0
// alone (wave-synchronous: LDS operations of one wave complete in order, so a
// compiler fence is enough between phases).  One sweep per call; the outer
// iteration revisits the pair until it is orthogonal.
__device__ __forceinline__ void wave_sync() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ void inner_jacobi16(double (*Hs)[17], double (*Qs)[17], double* cs) {
  const int lane = threadIdx.x;          // caller guarantees threadIdx.x < 64
  for (int e = lane; e < 256; e += 64) Qs[e >> 4][e & 15] = ((e >> 4) == (e & 15)) ? 1.0 : 0.0;
  wave_sync();
  for (int sw = 0; sw < kInnerSweeps; ++sw) {
    for (int step = 0; step < 15; ++step) {
      if (lane < 8) {
        int p = rr_slot(lane, step, 16), q = rr_slot(15 - lane, step, 16);
        double hpq = Hs[p][q], hpp = Hs[p][p], hqq = Hs[q][q];
        double c = 1.0, sn = 0.0;
        if (hpq * hpq > (0.0625 * kInnerTol * kInnerTol) * fabs(hpp * hqq)) jacobi_rotation(hpp, hqq, hpq, c, sn);
        cs[lane] = c;
        cs[8 + lane] = sn;
      }
      wave_sync();
      {
        const int a = lane >> 3, b = lane & 7;
        const int pa = rr_slot(a, step, 16), qa = rr_slot(15 - a, step, 16);
        const int pb = rr_slot(b, step, 16), qb = rr_slot(15 - b, step, 16);
        const double ca = cs[a], sa = cs[8 + a], cb = cs[b], sb = cs[8 + b];
        double g11 = Hs[pa][pb], g12 = Hs[pa][qb], g21 = Hs[qa][pb], g22 = Hs[qa][qb];
        double r11 = ca * g11 - sa * g21, r12 = ca * g12 - sa * g22;
        double r21 = sa * g11 + ca * g21, r22 = sa * g12 + ca * g22;
        // Q <- Q J for rows (lane >> 3) and (lane >> 3) + 8, pair b.
        const int i0 = lane >> 3;
        double v0p = Qs[i0][pb], v0q = Qs[i0][qb], v1p = Qs[i0 + 8][pb], v1q = Qs[i0 + 8][qb];
        wave_sync();
        Hs[pa][pb] = cb * r11 - sb * r12;
        Hs[pa][qb] = sb * r11 + cb * r12;
        Hs[qa][pb] = cb * r21 - sb * r22;
        Hs[qa][qb] = sb * r21 + cb * r22;
        Qs[i0][pb] = cb * v0p - sb * v0q;
        Qs[i0][qb] = sb * v0p + cb * v0q;
        Qs[i0 + 8][pb] = cb * v1p - sb * v1q;
        Qs[i0 + 8][qb] = sb * v1p + cb * v1q;
      }
      wave_sync();
    }
  }
}

// out[:, cols] = P * Q for the mp x 16 panel in LDS (column c at Ps[c*ldp+i]).
__device__ void panel_times_q(const double* Ps, int ldp, int mp, double (*Qs)[17], double* out,
                              const int* cols) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  for (int i0 = w * 16; i0 < mp; i0 += 64) {
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < 16; k0 += 4) {
      double a = Ps[(k0 + lk) * ldp + i0 + li];
      double b = Qs[k0 + lk][li];
      acc = mfma_f64(a, b, acc);
    }
    double* o = out + static_cast<int64_t>(cols[li]) * mp + i0 + lk;
#pragma unroll
    for (int v = 0; v < 4; ++v) o[4 * v] = acc[v];
  }
}

// Ps[c*ldp + i] = X[col(c)*mp + i] for the two 8-column blocks bi, bj of a
// column-major mp x mp matrix; 16-byte loads, 8 in flight per thread.
__device__ __forceinline__ void load_panel(const double* __restrict__ X, int mp, int ldp, int bi,
                                           int bj, double* __restrict__ Ps) {
  const int half = mp >> 1;                       // double2 per column
  const int total = 16 * half;
  for (int base = threadIdx.x; base < total; base += 256 * 8) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * 256;
      if (e < total) {
        int c = e / half, i2 = e - c * half;
        int col = (c < 8) ? bi * BW + c : bj * BW + (c - 8);
        v[u] = reinterpret_cast<const double2*>(X + static_cast<int64_t>(col) * mp)[i2];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * 256;
      if (e < total) {
        int c = e / half, i2 = e - c * half;
        Ps[c * ldp + 2 * i2] = v[u].x;
        Ps[c * ldp + 2 * i2 + 1] = v[u].y;
      }
    }
  }
}

// PREF: the V panel (mp <= 512) is fetched into registers together with the W
// panel, so its latency overlaps the Gram and inner solve.
template <bool PREF>
__global__ __launch_bounds__(256) void k_eig_blk(BlkArgs A) {
  const int mp = A.mp;
  const int ldp = mp + 1;
  const int nb = mp / BW;
  const unsigned nwg = gridDim.x;
  __shared__ double Ps[16 * (PMAX + 1)];
  __shared__ double Hp[4][256];
  __shared__ double Hs[16][17];
  __shared__ double Qs[16][17];
  __shared__ double cs[16];
  __shared__ int cols[16];
  __shared__ int flag;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;

  // W = G (symmetric, so row-major G is column-major W); V = I.
  const int64_t nn = static_cast<int64_t>(mp) * mp;
  for (int64_t e = blockIdx.x * 256LL + tid; e < nn; e += 256LL * nwg) {
    A.W[e] = A.G[e];
    A.V[e] = ((e / mp) == (e % mp)) ? 1.0 : 0.0;
  }
  if (blockIdx.x == 0 && tid < kMaxSweeps) A.rot[tid] = 0;
  grid_barrier(A.bar, nwg);

  int sweep = 0;
  for (; sweep < kMaxSweeps; ++sweep) {
    for (int step = 0; step < nb - 1; ++step) {
      const int bi = rr_slot(blockIdx.x, step, nb);
      const int bj = rr_slot(nb - 1 - blockIdx.x, step, nb);
      // Stage the W panel: every load is issued before any is consumed.
      double2 vreg[PREF ? 16 : 1];
      const int half = mp >> 1;
      if (PREF) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          int e = tid + u * 256;
          if (e < 16 * half) {
            int c = e / half, i2 = e - c * half;
            int col = (c < 8) ? bi * BW + c : bj * BW + (c - 8);
            vreg[u] = reinterpret_cast<const double2*>(A.V + static_cast<int64_t>(col) * mp)[i2];
          }
        }
      }
      load_panel(A.W, mp, ldp, bi, bj, Ps);
      if (tid < 16) cols[tid] = (tid < 8) ? bi * BW + tid : bj * BW + (tid - 8);
      __syncthreads();
      // H = P^T P, split over the four waves along the rows.
      {
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
        const int span = mp / 4;
        for (int k0 = w * span; k0 < (w + 1) * span; k0 += 4) {
          double a = Ps[li * ldp + k0 + lk];
          acc = mfma_f64(a, a, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) Hp[w][(lk + 4 * v) * 16 + li] = acc[v];
      }
      if (tid == 0) flag = 0;
      __syncthreads();
      {
        double h = (Hp[0][tid] + Hp[1][tid]) + (Hp[2][tid] + Hp[3][tid]);
        Hs[tid >> 4][tid & 15] = h;
      }
      __syncthreads();
      {
        int p = tid >> 4, q = tid & 15;
        if (p < q) {
          double hpq = Hs[p][q], hpp = Hs[p][p], hqq = Hs[q][q];
          if (hpp > 0.0 && hqq > 0.0 && hpq * hpq > (kOuterTol * kOuterTol) * (hpp * hqq)) flag = 1;
        }
      }
      __syncthreads();
      if (flag) {
        if (tid < 64) inner_jacobi16(Hs, Qs, cs);
        __syncthreads();
        panel_times_q(Ps, ldp, mp, Qs, A.W, cols);
        __syncthreads();
        if (PREF) {
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            int e = tid + u * 256;
            if (e < 16 * half) {
              int c = e / half, i2 = e - c * half;
              Ps[c * ldp + 2 * i2] = vreg[u].x;
              Ps[c * ldp + 2 * i2 + 1] = vreg[u].y;
            }
          }
        } else {
          load_panel(A.V, mp, ldp, bi, bj, Ps);
        }
        __syncthreads();
        panel_times_q(Ps, ldp, mp, Qs, A.V, cols);
        if (tid == 0) atomicAdd(&A.rot[sweep], 1);
      }
      grid_barrier(A.bar, nwg);
    }
    int r = __hip_atomic_load(&A.rot[sweep], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    if (r == 0) break;
  }
  if (blockIdx.x == 0 && tid == 0) {
    atomicAdd(&A.st->eig_sweeps, static_cast<unsigned long long>(sweep + 1));
    if (sweep == kMaxSweeps) atomicAdd(&A.st->eig_unconv, 1);
  }
  if (blockIdx.x == 0 && tid == 0) {
    int e = __hip_atomic_load(A.bar.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (e) A.st->bar_err = 1;
  }
  // lambda_j = v_j . w_j  (Rayleigh quotient with the converged V).
  for (int j = blockIdx.x * 4 + w; j < A.m; j += nwg * 4) {
    const double* vj = A.V + static_cast<int64_t>(j) * mp;
    const double* wj = A.W + static_cast<int64_t>(j) * mp;
    double s = 0.0;
    for (int i = lane; i < mp; i += 64) s += vj[i] * wj[i];
    s = wave_sum(s);
    if (lane == 0) A.lam[j] = s;
  }
}

hipError_t launch_eig(const double* G, int m, int mp, double* lam, double* V, EigWork wk,
                      hipStream_t s) {
  const int n = (m + 1) & ~1;
  if (n <= kLdsEigMax) {
    hipLaunchKernelGGL(k_eig_lds, dim3(1), dim3(1024), 0, s, G, m, mp, lam, V, wk.st);
    return hipGetLastError();
  }
  if (mp > PMAX || (mp % 32) != 0) return hipErrorInvalidValue;
  BlkArgs a;
  a.G = G; a.m = m; a.mp = mp; a.W = wk.W; a.V = V; a.lam = lam;
  a.bar.count = wk.bar; a.bar.gen = wk.bar + 1; a.bar.err = reinterpret_cast<int*>(wk.bar + 2);
  a.rot = wk.rot; a.st = wk.st;
  void* args[] = {&a};
  void* fn = (mp <= 512) ? reinterpret_cast<void*>(k_eig_blk<true>)
                         : reinterpret_cast<void*>(k_eig_blk<false>);
  return hipLaunchCooperativeKernel(fn, dim3(mp / 16), dim3(256), args, 0, s);
}

}  // namespace fdsk
