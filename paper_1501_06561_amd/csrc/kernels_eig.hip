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

// out[:, cols] = Pn Q for the mp x P panel in LDS (four waves split the rows).
template <int P>
__device__ void block_panel_times_q(const double* Ps, int ldp, int mp, const double* Qs, double* out,
                                    const int* cols) {
  constexpr int LDH = P + 1;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  for (int i0 = w * 16; i0 < mp; i0 += 64) {
#pragma unroll
    for (int ct = 0; ct < P / 16; ++ct) {
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k0 = 0; k0 < P; k0 += 4) {
        double a = Ps[(k0 + lk) * ldp + i0 + li];
        double b = Qs[(k0 + lk) * LDH + ct * 16 + li];
        acc = mfma_f64(a, b, acc);
      }
      double* o = out + static_cast<int64_t>(cols[ct * 16 + li]) * mp + i0 + lk;
#pragma unroll
      for (int v = 0; v < 4; ++v) o[4 * v] = acc[v];
    }
  }
}

// Ps[c*ldp + i] = X[col(c)*mp + i] for the P panel columns (two blocks of
// P/2); 16-byte loads, 8 in flight per thread.
template <int P>
__device__ __forceinline__ void load_panel(const double* __restrict__ X, int mp, int ldp, int bi,
                                           int bj, double* __restrict__ Ps) {
  constexpr int HB = P / 2;
  const int half = mp >> 1;
  const int total = P * half;
  for (int base = threadIdx.x; base < total; base += 256 * 8) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int e = base + u * 256;
      if (e < total) {
        int c = e / half, i2 = e - c * half;
        int col = (c < HB) ? bi * HB + c : bj * HB + (c - HB);
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

// One sweep of two-sided Jacobi on the P x P panel Gram H (LDS, ld P+1),
// accumulating Q, executed by the whole workgroup (256 threads).
template <int P>
__device__ void inner_jacobi_wg(double* Hs, double* Qs, double* cs) {
  constexpr int LDH = P + 1, NP = P / 2;
  const int tid = threadIdx.x;
  for (int e = tid; e < P * P; e += 256) Qs[(e / P) * LDH + (e % P)] = ((e / P) == (e % P)) ? 1.0 : 0.0;
  __syncthreads();
  for (int sw = 0; sw < kInnerSweeps; ++sw) {
    for (int step = 0; step < P - 1; ++step) {
      if (tid < NP) {
        int p = rr_fast(tid, step, P), q = rr_fast(P - 1 - tid, step, P);
        double hpq = Hs[p * LDH + q], hpp = Hs[p * LDH + p], hqq = Hs[q * LDH + q];
        double c = 1.0, sn = 0.0;
        if (hpq * hpq > (0.0625 * kInnerTol * kInnerTol) * fabs(hpp * hqq)) jacobi_rotation(hpp, hqq, hpq, c, sn);
        cs[tid] = c;
        cs[NP + tid] = sn;
      }
      __syncthreads();
      for (int e = tid; e < NP * NP; e += 256) {
        const int a = e / NP, b = e % NP;
        const int pa = rr_fast(a, step, P), qa = rr_fast(P - 1 - a, step, P);
        const int pb = rr_fast(b, step, P), qb = rr_fast(P - 1 - b, step, P);
        const double ca = cs[a], sa = cs[NP + a], cb = cs[b], sb = cs[NP + b];
        double g11 = Hs[pa * LDH + pb], g12 = Hs[pa * LDH + qb], g21 = Hs[qa * LDH + pb], g22 = Hs[qa * LDH + qb];
        double r11 = ca * g11 - sa * g21, r12 = ca * g12 - sa * g22;
        double r21 = sa * g11 + ca * g21, r22 = sa * g12 + ca * g22;
        Hs[pa * LDH + pb] = cb * r11 - sb * r12;
        Hs[pa * LDH + qb] = sb * r11 + cb * r12;
        Hs[qa * LDH + pb] = cb * r21 - sb * r22;
        Hs[qa * LDH + qb] = sb * r21 + cb * r22;
      }
      for (int e = tid; e < P * NP; e += 256) {
        const int i = e / NP, b = e % NP;
        const int pb = rr_fast(b, step, P), qb = rr_fast(P - 1 - b, step, P);
        const double cb = cs[b], sb = cs[NP + b];
        double vp = Qs[i * LDH + pb], vq = Qs[i * LDH + qb];
        Qs[i * LDH + pb] = cb * vp - sb * vq;
        Qs[i * LDH + qb] = sb * vp + cb * vq;
      }
      __syncthreads();
    }
  }
}

// P: panel width (16 or 32 columns = two blocks of P/2).  PREF: the V panel
// is fetched into registers together with the W panel, so its latency
// overlaps the Gram and inner solve (mp <= 512).
template <int P, bool PREF>
__global__ __launch_bounds__(256) void k_eig_blk(BlkArgs A) {
  constexpr int HB = P / 2;
  constexpr int LDH = P + 1;
  constexpr int PM = (P == 32) ? 512 : PMAX;    // largest mp for this panel width
  constexpr int VR = PREF ? (P * 256 / 256) : 1; // double2 per thread for mp <= 512
  const int mp = A.mp;
  const int ldp = mp + 1;
  const int nb = mp / HB;
  const unsigned nwg = gridDim.x;
  __shared__ double Ps[P * (PM + 1)];
  __shared__ double Hp[(P == 16) ? 4 * 256 : 1];
  __shared__ double Hs[P * LDH];
  __shared__ double Qs[P * LDH];
  __shared__ double cs[P];
  __shared__ int cols[P];
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
      double2 vreg[VR];
      const int half = mp >> 1;
      if (PREF) {
#pragma unroll
        for (int u = 0; u < VR; ++u) {
          int e = tid + u * 256;
          if (e < P * half) {
            int c = e / half, i2 = e - c * half;
            int col = (c < HB) ? bi * HB + c : bj * HB + (c - HB);
            vreg[u] = reinterpret_cast<const double2*>(A.V + static_cast<int64_t>(col) * mp)[i2];
          }
        }
      }
      load_panel<P>(A.W, mp, ldp, bi, bj, Ps);
      if (tid < P) cols[tid] = (tid < HB) ? bi * HB + tid : bj * HB + (tid - HB);
      __syncthreads();
      // H = P^T P on matrix cores.
      if (P == 16) {
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
        const int span = mp / 4;
        for (int k0 = w * span; k0 < (w + 1) * span; k0 += 4) {
          double a = Ps[li * ldp + k0 + lk];
          acc = mfma_f64(a, a, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) Hp[w * 256 + (lk + 4 * v) * 16 + li] = acc[v];
        __syncthreads();
        Hs[(tid >> 4) * LDH + (tid & 15)] = (Hp[tid] + Hp[256 + tid]) + (Hp[512 + tid] + Hp[768 + tid]);
      } else {
        const int ti = w >> 1, tj = w & 1;       // one 16x16 tile of the 32x32 H per wave
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < mp; k0 += 4) {
          double a = Ps[(ti * 16 + li) * ldp + k0 + lk];
          double b = Ps[(tj * 16 + li) * ldp + k0 + lk];
          acc = mfma_f64(a, b, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) Hs[(ti * 16 + lk + 4 * v) * LDH + tj * 16 + li] = acc[v];
      }
      if (tid == 0) flag = 0;
      __syncthreads();
      for (int e = tid; e < P * P; e += 256) {
        int p = e / P, q = e % P;
        if (p < q) {
          double hpq = Hs[p * LDH + q], hpp = Hs[p * LDH + p], hqq = Hs[q * LDH + q];
          if (hpp > 0.0 && hqq > 0.0 && hpq * hpq > (kOuterTol * kOuterTol) * (hpp * hqq)) flag = 1;
        }
      }
      __syncthreads();
      if (flag) {
        if (P == 16) {
          if (tid < 64) inner_jacobi16(Hs, Qs, cs);
          __syncthreads();
        } else {
          inner_jacobi_wg<P>(Hs, Qs, cs);
        }
        block_panel_times_q<P>(Ps, ldp, mp, Qs, A.W, cols);
        __syncthreads();
        if (PREF) {
#pragma unroll
          for (int u = 0; u < VR; ++u) {
            int e = tid + u * 256;
            if (e < P * half) {
              int c = e / half, i2 = e - c * half;
              Ps[c * ldp + 2 * i2] = vreg[u].x;
              Ps[c * ldp + 2 * i2 + 1] = vreg[u].y;
            }
          }
        } else {
          load_panel<P>(A.V, mp, ldp, bi, bj, Ps);
        }
        __syncthreads();
        block_panel_times_q<P>(Ps, ldp, mp, Qs, A.V, cols);
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
  if (eig_uses_trid(m, wk)) return launch_eig_trid(G, m, mp, lam, V, wk, s);
  return launch_eig_jacobi(G, m, mp, lam, V, wk, s);
}

hipError_t launch_eig_jacobi(const double* G, int m, int mp, double* lam, double* V, EigWork wk,
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
  void* fn;
  int grid;
  if (mp <= 512) {
    fn = reinterpret_cast<void*>(k_eig_blk<32, true>);
    grid = mp / 32;
  } else {
    fn = reinterpret_cast<void*>(k_eig_blk<16, false>);
    grid = mp / 16;
  }
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(256), args, 0, s);
}

}  // namespace fdsk
