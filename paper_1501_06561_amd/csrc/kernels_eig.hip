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

__global__ __launch_bounds__(1024) void k_eig_lds(const double* __restrict__ G, int m, int mp,
                                                  double* __restrict__ lam,
                                                  double* __restrict__ Vout,
                                                  DevStats* __restrict__ st) {
  __shared__ double Gs[LN * LLD];
  __shared__ double Vs[LN * LLD];
  __shared__ double cs[LN];
  __shared__ double red[32];
  __shared__ int done;
  const int n = (m + 1) & ~1;
  const int np2 = n / 2;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < n * n; e += nt) {
    int i = e / n, j = e % n;
    Gs[i * LLD + j] = (i < m && j < m) ? G[static_cast<int64_t>(i) * mp + j] : 0.0;
    Vs[i * LLD + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();

  int sweep = 0;
  for (; sweep < kMaxSweeps; ++sweep) {
    // Convergence: off-diagonal mass against the whole matrix.
    double off = 0.0, all = 0.0;
    for (int e = tid; e < n * n; e += nt) {
      int i = e / n, j = e % n;
      double g = Gs[i * LLD + j];
      all += g * g;
      if (i != j) off += g * g;
    }
    off = wave_sum(off);
    all = wave_sum(all);
    if ((tid & 63) == 0) { red[tid >> 6] = off; red[16 + (tid >> 6)] = all; }
    __syncthreads();
    if (tid == 0) {
      double o = 0.0, a = 0.0;
      for (int w = 0; w < nt / 64; ++w) { o += red[w]; a += red[16 + w]; }
      done = (o <= 1e-30 * a) ? 1 : 0;
    }
    __syncthreads();
    if (done) break;

    for (int step = 0; step < n - 1; ++step) {
      if (tid < np2) {
        int p = rr_slot(tid, step, n), q = rr_slot(n - 1 - tid, step, n);
        double c, s;
        jacobi_rotation(Gs[p * LLD + p], Gs[q * LLD + q], Gs[p * LLD + q], c, s);
        cs[tid] = c;
        cs[np2 + tid] = s;
      }
      __syncthreads();
      for (int e = tid; e < np2 * np2; e += nt) {
        int a = e / np2, b = e % np2;
        int pa = rr_slot(a, step, n), qa = rr_slot(n - 1 - a, step, n);
        int pb = rr_slot(b, step, n), qb = rr_slot(n - 1 - b, step, n);
        double ca = cs[a], sa = cs[np2 + a], cb = cs[b], sb = cs[np2 + b];
        double g11 = Gs[pa * LLD + pb], g12 = Gs[pa * LLD + qb];
        double g21 = Gs[qa * LLD + pb], g22 = Gs[qa * LLD + qb];
        double r11 = ca * g11 - sa * g21, r12 = ca * g12 - sa * g22;
        double r21 = sa * g11 + ca * g21, r22 = sa * g12 + ca * g22;
        Gs[pa * LLD + pb] = cb * r11 - sb * r12;
        Gs[pa * LLD + qb] = sb * r11 + cb * r12;
        Gs[qa * LLD + pb] = cb * r21 - sb * r22;
        Gs[qa * LLD + qb] = sb * r21 + cb * r22;
      }
      for (int e = tid; e < n * np2; e += nt) {
        int i = e / np2, b = e % np2;
        int pb = rr_slot(b, step, n), qb = rr_slot(n - 1 - b, step, n);
        double cb = cs[b], sb = cs[np2 + b];
        double vp = Vs[i * LLD + pb], vq = Vs[i * LLD + qb];
        Vs[i * LLD + pb] = cb * vp - sb * vq;
        Vs[i * LLD + qb] = sb * vp + cb * vq;
      }
      __syncthreads();
    }
  }
  if (sweep == kMaxSweeps && tid == 0) atomicAdd(&st->eig_unconv, 1);
  for (int j = tid; j < m; j += nt) lam[j] = Gs[j * LLD + j];
  for (int64_t e = tid; e < static_cast<int64_t>(mp) * mp; e += nt) {
    int j = static_cast<int>(e / mp), i = static_cast<int>(e % mp);
    Vout[e] = (i < m && j < m) ? Vs[i * LLD + j] : 0.0;
  }
}

// ------------------------------------------------------- block solver
constexpr int BW = 8;            // block width; a task owns 2 blocks = 16 columns
constexpr int PMAX = 1024;       // largest mp
constexpr double kOuterTol = 1e-14;
constexpr double kInnerTol = 1e-15;
constexpr int kInnerSweeps = 8;

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

// Inner two-sided Jacobi on the 16x16 H (LDS), accumulating Q.  All 256
// threads call it; returns after convergence or kInnerSweeps sweeps.
__device__ void inner_jacobi16(double (*Hs)[17], double (*Qs)[17], double* cs, int* flag) {
  const int tid = threadIdx.x;
  for (int e = tid; e < 256; e += blockDim.x) Qs[e >> 4][e & 15] = ((e >> 4) == (e & 15)) ? 1.0 : 0.0;
  __syncthreads();
  for (int sw = 0; sw < kInnerSweeps; ++sw) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    if (tid < 256) {
      int p = tid >> 4, q = tid & 15;
      if (p < q) {
        double hpq = Hs[p][q], hpp = Hs[p][p], hqq = Hs[q][q];
        if (fabs(hpq) > kInnerTol * sqrt(fabs(hpp) * fabs(hqq))) *flag = 1;
      }
    }
    __syncthreads();
    if (*flag == 0) break;
    for (int step = 0; step < 15; ++step) {
      if (tid < 8) {
        int p = rr_slot(tid, step, 16), q = rr_slot(15 - tid, step, 16);
        double hpq = Hs[p][q], hpp = Hs[p][p], hqq = Hs[q][q];
        double c = 1.0, s = 0.0;
        if (fabs(hpq) > 0.25 * kInnerTol * sqrt(fabs(hpp) * fabs(hqq))) jacobi_rotation(hpp, hqq, hpq, c, s);
        cs[tid] = c;
        cs[8 + tid] = s;
      }
      __syncthreads();
      if (tid < 64) {
        int a = tid >> 3, b = tid & 7;
        int pa = rr_slot(a, step, 16), qa = rr_slot(15 - a, step, 16);
        int pb = rr_slot(b, step, 16), qb = rr_slot(15 - b, step, 16);
        double ca = cs[a], sa = cs[8 + a], cb = cs[b], sb = cs[8 + b];
        double g11 = Hs[pa][pb], g12 = Hs[pa][qb], g21 = Hs[qa][pb], g22 = Hs[qa][qb];
        double r11 = ca * g11 - sa * g21, r12 = ca * g12 - sa * g22;
        double r21 = sa * g11 + ca * g21, r22 = sa * g12 + ca * g22;
        Hs[pa][pb] = cb * r11 - sb * r12;
        Hs[pa][qb] = sb * r11 + cb * r12;
        Hs[qa][pb] = cb * r21 - sb * r22;
        Hs[qa][qb] = sb * r21 + cb * r22;
      } else if (tid < 192) {
        int e = tid - 64;
        int i = e >> 3, b = e & 7;
        int pb = rr_slot(b, step, 16), qb = rr_slot(15 - b, step, 16);
        double cb = cs[b], sb = cs[8 + b];
        double vp = Qs[i][pb], vq = Qs[i][qb];
        Qs[i][pb] = cb * vp - sb * vq;
        Qs[i][qb] = sb * vp + cb * vq;
      }
      __syncthreads();
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
  __shared__ int iflag;
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
      if (tid < 16) cols[tid] = (tid < 8) ? bi * BW + tid : bj * BW + (tid - 8);
      __syncthreads();
      // Stage the W panel.
      for (int e = tid; e < 16 * mp; e += 256) {
        int c = e / mp, i = e % mp;
        Ps[c * ldp + i] = A.W[static_cast<int64_t>(cols[c]) * mp + i];
      }
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
          if (hpp > 0.0 && hqq > 0.0 && fabs(hpq) > kOuterTol * sqrt(hpp * hqq)) flag = 1;
        }
      }
      __syncthreads();
      if (flag) {
        inner_jacobi16(Hs, Qs, cs, &iflag);
        panel_times_q(Ps, ldp, mp, Qs, A.W, cols);
        __syncthreads();
        for (int e = tid; e < 16 * mp; e += 256) {
          int c = e / mp, i = e % mp;
          Ps[c * ldp + i] = A.V[static_cast<int64_t>(cols[c]) * mp + i];
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
  if (sweep == kMaxSweeps && blockIdx.x == 0 && tid == 0) atomicAdd(&A.st->eig_unconv, 1);
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
  return hipLaunchCooperativeKernel(reinterpret_cast<void*>(k_eig_blk), dim3(mp / 16), dim3(256),
                                    args, 0, s);
}

}  // namespace fdsk
