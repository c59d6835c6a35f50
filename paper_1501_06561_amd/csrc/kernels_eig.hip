// FP64 symmetric eigensolvers for the m x m Gram matrix of the sketch buffer.
//
// * k_eig_lds  (m <= 100): cyclic two-sided Jacobi in one workgroup with G and
//   V resident in LDS (eig_lds_body).
// * k_eig_blk  (m <= 1024): one-sided block Jacobi (Hestenes) on W = G with
//   V accumulated.  A task orthogonalises a 16-column panel (two 8-column
//   blocks): H = P^T P on matrix cores, a two-sided Jacobi sweep on the 16x16
//   H gives Q, then P <- P Q and V_panel <- V_panel Q on matrix cores.
//   mp/16 workgroups run the disjoint block pairs of one round-robin step in
//   parallel, with a grid barrier between steps; a sweep with no rotation ends
//   the solve.  At convergence W = V diag(lambda) and lambda_j = v_j . w_j.
#include "fdsk_jacobi.hpp"

namespace fdsk {

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
  eig_lds_body(G, m, mp, lam, Vout, st, LdsEigSmem{Gs, Vs, cs, pi, qi, &nrot, &gmax});
}

constexpr int PMAX = 1024;       // largest mp of the block solver

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

// out[:, cols] = P * Q for the mp x 16 panel in LDS, four waves.
__device__ void block_panel_times_q(const double* Ps, int ldp, int mp, const double* Qs, double* out,
                                    const int* cols) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  for (int i0 = w * 16; i0 < mp; i0 += 64) {
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < 16; k0 += 4) {
      double a = Ps[(k0 + lk) * ldp + i0 + li];
      double b = Qs[(k0 + lk) * 17 + li];
      acc = mfma_f64(a, b, acc);
    }
    double* o = out + static_cast<int64_t>(cols[li]) * mp + i0 + lk;
#pragma unroll
    for (int v = 0; v < 4; ++v) o[4 * v] = acc[v];
  }
}

// Ps[c*ldp + i] = X[col(c)*mp + i]; 16-byte loads, 8 in flight per thread.
__device__ __forceinline__ void load_panel(const double* __restrict__ X, int mp, int ldp, int bi,
                                           int bj, double* __restrict__ Ps) {
  const int half = mp >> 1;
  const int total = 16 * half;
  for (int base = threadIdx.x; base < total; base += 256 * 8) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * 256;
      if (e < total) {
        int c = e / half, i2 = e - c * half;
        v[u] = reinterpret_cast<const double2*>(X + static_cast<int64_t>(panel_col(c, bi, bj)) * mp)[i2];
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
  __shared__ double Hs[16 * 17];
  __shared__ double Qs[16 * 17];
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
        Hs[(tid >> 4) * 17 + (tid & 15)] = h;
      }
      __syncthreads();
      {
        int p = tid >> 4, q = tid & 15;
        if (p < q) {
          double hpq = Hs[p * 17 + q], hpp = Hs[p * 17 + p], hqq = Hs[q * 17 + q];
          if (hpp > 0.0 && hqq > 0.0 && hpq * hpq > (kOuterTol * kOuterTol) * (hpp * hqq)) flag = 1;
        }
      }
      __syncthreads();
      if (flag) {
        if (tid < 64) inner_jacobi16(Hs, Qs, cs);
        __syncthreads();
        block_panel_times_q(Ps, ldp, mp, Qs, A.W, cols);
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
        block_panel_times_q(Ps, ldp, mp, Qs, A.V, cols);
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
