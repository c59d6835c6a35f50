// Many independent sketches in one persistent launch.
//
// Every workgroup claims the next sketch from a device queue (an atomic
// counter over a cost-sorted order) and runs that sketch's whole schedule of
// Algorithm 1 by itself: ingest, and for every full buffer the Gram product,
// the FP64 eigensolve, the ReduceRank rule and the rebuild -- then claims the
// next sketch.  Sketches never wait for each other and the launch drains when
// the queue is empty.  Arithmetic per sketch is identical whichever workgroup
// runs it, so results do not depend on the grid size.
#include "fdsk_batch.hpp"
#include "fdsk_jacobi.hpp"

namespace fdsk {

constexpr int NT = 512;                 // threads per workgroup (8 waves)
constexpr int SMEM_DOUBLES = 20400;     // 163,200 bytes of LDS
constexpr int MAXT = 9;                 // 16x16 Gram tiles per wave and pass

// ----------------------------------------------------------------- ingest
__device__ void b_ingest(const BatchDesc& D, int64_t r0, int f, int occ, double* C) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = w; i < f; i += NT / 64) {
    const int64_t base = (r0 + i) * D.stride;
    double* dst = C + static_cast<int64_t>(occ + i) * D.ldc;
    double acc = 0.0;
    for (int c = lane; c < D.ldc; c += 64) {
      double v = (c < D.d) ? load_as_f64(D.rows, base + c, D.dt) : 0.0;
      dst[c] = v;
      acc += v * v;
    }
    acc = wave_sum(acc);
    if (lane == 0) D.rownorm[occ + i] = acc;
  }
  __syncthreads();
}

// ------------------------------------------------------------------- Gram
// G = C C^T on 16x16 lower tiles; each 32-column chunk of C is staged once in
// LDS per pass and every wave accumulates up to MAXT tiles (matrix cores).
__device__ __forceinline__ void tri_decode(int idx, int& a, int& b) {
  a = static_cast<int>((sqrtf(8.0f * idx + 1.0f) - 1.0f) * 0.5f);
  while ((a + 1) * (a + 2) / 2 <= idx) ++a;
  while (a * (a + 1) / 2 > idx) --a;
  b = idx - a * (a + 1) / 2;
}

__device__ void b_gram(const double* __restrict__ C, int ldc, int mp, double* __restrict__ G,
                       double* smem) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int T = mp / 16;
  const int ntiles = T * (T + 1) / 2;
  constexpr int NW = NT / 64;
  double* Cs = smem;                    // mp x 33
  for (int pass0 = 0; pass0 < ntiles; pass0 += NW * MAXT) {
    f64x4 acc[MAXT];
#pragma unroll
    for (int t = 0; t < MAXT; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < ldc; k0 += 32) {
      for (int e = threadIdx.x; e < mp * 32; e += NT) {
        int r = e >> 5, c = e & 31;
        Cs[r * 33 + c] = C[static_cast<int64_t>(r) * ldc + k0 + c];
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        const int idx = pass0 + w + t * NW;
        if (idx < ntiles) {
          int ta, tb;
          tri_decode(idx, ta, tb);
#pragma unroll
          for (int k4 = 0; k4 < 8; ++k4) {
            double a = Cs[(ta * 16 + li) * 33 + k4 * 4 + lk];
            double b = Cs[(tb * 16 + li) * 33 + k4 * 4 + lk];
            acc[t] = mfma_f64(a, b, acc[t]);
          }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      const int idx = pass0 + w + t * NW;
      if (idx < ntiles) {
        int ta, tb;
        tri_decode(idx, ta, tb);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          int row = ta * 16 + lk + 4 * v, col = tb * 16 + li;
          G[static_cast<int64_t>(row) * mp + col] = acc[t][v];
          G[static_cast<int64_t>(col) * mp + row] = acc[t][v];
        }
      }
    }
  }
  __syncthreads();
}

// ------------------------------------------------ eigensolve, m in (100, 256]
// One-sided block Jacobi on W = G with V accumulated, inside one workgroup:
// four waves each own a 16-column panel task of the current round-robin step
// (panel, 16x16 Gram, inner sweep and panel updates all wave-local), the
// workgroup synchronises between steps.
__device__ void b_eig_wg(const double* __restrict__ G, int m, int mp, double* __restrict__ W,
                         double* __restrict__ V, double* __restrict__ lam, DevStats* st,
                         double* smem) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ldp = mp + 1;
  const int per_wave = 16 * ldp + 2 * 272 + 16;
  int* rotcount = reinterpret_cast<int*>(smem + 4 * per_wave);
  const int64_t nn = static_cast<int64_t>(mp) * mp;
  for (int64_t e = threadIdx.x; e < nn; e += NT) {
    W[e] = G[e];
    V[e] = ((e / mp) == (e % mp)) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int nb = mp / BW;
  double* Ps = smem + w * per_wave;
  double* Hs = Ps + 16 * ldp;
  double* Qs = Hs + 272;
  double* cs = Qs + 272;
  int sweep = 0;
  for (; sweep < kMaxSweeps; ++sweep) {
    if (threadIdx.x == 0) *rotcount = 0;
    __syncthreads();
    for (int step = 0; step < nb - 1; ++step) {
      if (w < 4) {
        for (int task = w; task < nb / 2; task += 4) {
          const int bi = rr_slot(task, step, nb), bj = rr_slot(nb - 1 - task, step, nb);
          wave_load_panel(W, mp, ldp, bi, bj, Ps);
          wave_sync();
          wave_panel_gram(Ps, ldp, mp, Hs);
          wave_sync();
          if (wave_panel_needs_rotation(Hs)) {
            inner_jacobi16(Hs, Qs, cs);
            wave_sync();
            wave_panel_times_q(Ps, ldp, mp, Qs, W, bi, bj);
            wave_sync();
            wave_load_panel(V, mp, ldp, bi, bj, Ps);
            wave_sync();
            wave_panel_times_q(Ps, ldp, mp, Qs, V, bi, bj);
            if (lane == 0) atomicAdd(rotcount, 1);
          }
          wave_sync();
        }
      }
      __syncthreads();
    }
    const int r = *rotcount;
    __syncthreads();
    if (r == 0) break;
  }
  if (threadIdx.x == 0) {
    atomicAdd(&st->eig_sweeps, static_cast<unsigned long long>(sweep + 1));
    if (sweep == kMaxSweeps) atomicAdd(&st->eig_unconv, 1);
  }
  for (int j = w; j < m; j += NT / 64) {
    const double* vj = V + static_cast<int64_t>(j) * mp;
    const double* wj = W + static_cast<int64_t>(j) * mp;
    double s = 0.0;
    for (int i = lane; i < mp; i += 64) s += vj[i] * wj[i];
    s = wave_sum(s);
    if (lane == 0) lam[j] = s;
  }
  __syncthreads();
}

// ----------------------------------------------------------------- shrink
// Rank the eigenvalues, apply the variant's rule in FP64, update the
// accumulators and write Ut = diag(rho) U^T for the kept rows.
__device__ void b_shrink(const BatchDesc& D, int new0, int new1, double* smem) {
  const int m = D.m, mp = D.mp;
  const RuleParams rp = D.rp;
  double* raw = smem;
  double* lam = raw + 256;
  double* rho = lam + 256;
  double* red = rho + 256;
  int* perm = reinterpret_cast<int*>(red + NT);
  int* bad = perm + 256;
  const int tid = threadIdx.x;
  if (tid == 0) *bad = 0;
  __syncthreads();
  for (int j = tid; j < m; j += NT) {
    double x = D.lam[j];
    if (!(x == x) || isinf(x)) *bad = 1;
    raw[j] = (x == x) ? x : -INFINITY;
  }
  __syncthreads();
  for (int j = tid; j < m; j += NT) {
    double x = raw[j];
    int rank = 0;
    for (int i = 0; i < m; ++i) rank += (raw[i] > x) || (raw[i] == x && i < j);
    perm[rank] = j;
  }
  __syncthreads();
  for (int q = tid; q < m; q += NT) lam[q] = fmax(raw[perm[q]], 0.0);
  __syncthreads();
  const double delta = (rp.t - 1 < m) ? lam[rp.t - 1] : 0.0;
  double removed = 0.0;
  for (int q = tid; q < m; q += NT) {
    double x = lam[q], y;
    bool untouched;
    if (rp.variant == 1) {
      untouched = q < rp.l - 1;
      y = untouched ? x : 0.0;
    } else {
      untouched = q < rp.r;
      y = untouched ? x : fmax(x - delta, 0.0);
    }
    removed += x - y;
    rho[q] = untouched ? 1.0 : ((x > 0.0 && y > 0.0) ? sqrt(y / x) : 0.0);
  }
  red[tid] = removed;
  __syncthreads();
  for (int s = NT >> 1; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) {
    double nrm = 0.0;
    for (int i = new0; i < new1; ++i) nrm += D.rownorm[i];
    D.st->fro2A += nrm;
    D.st->Delta += delta;
    D.st->Stot += red[0];
    D.st->n_rr += 1;
    if (*bad || !(nrm == nrm)) D.st->nonfinite = 1;
  }
  const int rows = (rp.keep + 15) & ~15;
  for (int64_t e = tid; e < static_cast<int64_t>(rows) * mp; e += NT) {
    int q = static_cast<int>(e / mp), i = static_cast<int>(e % mp);
    double v = 0.0;
    if (q < rp.keep && q < m && i < m) v = rho[q] * D.V[static_cast<int64_t>(perm[q]) * mp + i];
    D.Ut[e] = v;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- rebuild
// out[0:keep, :] = Ut[0:keep, :] C.  Wave pair p (waves p and p+4) owns the
// 16-row blocks rb = p, p+4, ...; the block's Ut rows are staged in LDS and
// the two waves split the 16-column output tiles, streaming C from memory.
__device__ void b_rebuild(const double* __restrict__ Ut, const double* __restrict__ C, int ldc,
                          int mp, int keep, double* __restrict__ out, double* smem) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int pair = w & 3, half = w >> 2;
  const int ldu = mp + 2;
  double* Us = smem + pair * 16 * ldu;
  const int nrb = (keep + 15) / 16;
  const int iters = (nrb + 3) / 4;
  for (int it = 0; it < iters; ++it) {
    const int rb = pair + 4 * it;
    if (rb < nrb) {
      for (int e = half * 64 + lane; e < 16 * mp; e += 128) {
        int r = e / mp, k = e - r * mp;
        Us[r * ldu + k] = Ut[static_cast<int64_t>(rb * 16 + r) * mp + k];
      }
    }
    __syncthreads();
    if (rb < nrb) {
      for (int ct = half; ct < ldc / 16; ct += 2) {
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
        const double* Cb = C + ct * 16 + li;
        for (int k0 = 0; k0 < mp; k0 += 4) {
          double a = Us[li * ldu + k0 + lk];
          double b = Cb[static_cast<int64_t>(k0 + lk) * ldc];
          acc = mfma_f64(a, b, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          int row = rb * 16 + lk + 4 * v;
          if (row < keep) out[static_cast<int64_t>(row) * ldc + ct * 16 + li] = acc[v];
        }
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------- one sketch
__device__ void b_reduce(const BatchDesc& D, BatchState& S, double* smem) {
  double* C = S.cur ? D.C1 : D.C0;
  double* Cn = S.cur ? D.C0 : D.C1;
  b_gram(C, D.ldc, D.mp, D.G, smem);
  if (((D.m + 1) & ~1) <= kLdsEigMax) {
    LdsEigSmem sm{smem, smem + LN * LLD, smem + 2 * LN * LLD,
                  reinterpret_cast<short*>(smem + 2 * LN * LLD + LN),
                  reinterpret_cast<short*>(smem + 2 * LN * LLD + LN) + LN / 2,
                  reinterpret_cast<int*>(smem + 2 * LN * LLD + LN + 32),
                  smem + 2 * LN * LLD + LN + 34};
    eig_lds_body(D.G, D.m, D.mp, D.lam, D.V, D.st, sm);
    __syncthreads();
  } else {
    b_eig_wg(D.G, D.m, D.mp, D.W, D.V, D.lam, D.st, smem);
  }
  b_shrink(D, S.new0, S.occ, smem);
  b_rebuild(D.Ut, C, D.ldc, D.mp, D.rp.keep, Cn, smem);
  S.cur ^= 1;
  S.occ = D.rp.keep;
  S.new0 = S.occ;
}

__device__ void b_run_sketch(const BatchDesc& D, BatchState* Sg, int finalize, double* smem) {
  BatchState S = *Sg;
  __syncthreads();
  int64_t r = 0;
  while (r < D.n) {
    const int f = static_cast<int>(min(static_cast<int64_t>(D.m - S.occ), D.n - r));
    b_ingest(D, r, f, S.occ, S.cur ? D.C1 : D.C0);
    S.occ += f;
    r += f;
    if (S.occ == D.m) b_reduce(D, S, smem);
  }
  if (finalize) {
    double* C = S.cur ? D.C1 : D.C0;
    if (S.occ > D.l) {
      const int64_t nz = static_cast<int64_t>(D.m - S.occ) * D.ldc;
      double* p = C + static_cast<int64_t>(S.occ) * D.ldc;
      for (int64_t e = threadIdx.x; e < nz; e += NT) p[e] = 0.0;
      __syncthreads();
      b_reduce(D, S, smem);
    } else {
      if (threadIdx.x == 0) {
        double nrm = 0.0;
        for (int i = S.new0; i < S.occ; ++i) nrm += D.rownorm[i];
        D.st->fro2A += nrm;
        if (!(nrm == nrm) || isinf(nrm)) D.st->nonfinite = 1;
      }
      S.new0 = S.occ;
    }
    C = S.cur ? D.C1 : D.C0;
    const int valid = min(S.occ, D.l);
    const int64_t tot = static_cast<int64_t>(D.l) * D.d;
    for (int64_t e = threadIdx.x; e < tot; e += NT) {
      int rr = static_cast<int>(e / D.d), c = static_cast<int>(e % D.d);
      double v = (rr < valid) ? C[static_cast<int64_t>(rr) * D.ldc + c] : 0.0;
      if (D.out_dt == DT_F64)
        static_cast<double*>(D.out)[rr * D.ldb + c] = v;
      else
        static_cast<float*>(D.out)[rr * D.ldb + c] = static_cast<float>(v);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *Sg = S;
}

__global__ __launch_bounds__(NT) void k_batch_run(const BatchDesc* __restrict__ descs,
                                                  BatchState* __restrict__ states,
                                                  const int* __restrict__ order, int nsk,
                                                  int* __restrict__ counter, int finalize) {
  __shared__ double smem[SMEM_DOUBLES];
  __shared__ int job;
  for (;;) {
    if (threadIdx.x == 0) job = atomicAdd(counter, 1);
    __syncthreads();
    const int j = job;
    __syncthreads();              // every thread has read job before it changes
    if (j >= nsk) break;
    const int i = order[j];
    BatchDesc D = descs[i];
    b_run_sketch(D, &states[i], finalize, smem);
  }
}

__global__ void k_zero_int(int* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

hipError_t launch_batch_run(const BatchDesc* descs, BatchState* states, const int* order, int nsk,
                            int* counter, int finalize, int grid, hipStream_t s) {
  // The queue counter is cleared by a kernel (not a memset) so the launch pair
  // can be captured into a graph.
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, counter, 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nsk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_run, dim3(grid), dim3(NT), 0, s, descs, states, order, nsk, counter,
                     finalize);
  return hipGetLastError();
}

}  // namespace fdsk
