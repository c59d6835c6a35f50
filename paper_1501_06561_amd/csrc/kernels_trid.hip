// FP64 symmetric eigensolver by tridiagonal reduction and divide and conquer.
//
// The m x m Gram matrix G of a ReduceRank (m <= kTridGlobalMax) goes through
// three kernels, all in FP64 and all in stream order:
//
// * k_tridiag_reg / k_tridiag: Householder reduction Q^T G Q = T (T
//   tridiagonal) in one workgroup, the matrix held in registers across the
//   workgroup (m <= kTridRegMax).  Above that, k_tridiag takes the first
//   m - kTridRegMax columns with the lower triangle packed by columns in the
//   workspace W itself (L2-resident), and the register kernel the rest.  Reflector
//   H_k = I - tau_k u_k u_k^T with u_k = (0,..,0, 1, v_k) zeroes column k below
//   the subdiagonal; the trailing block is updated by the symmetric rank-2
//   form A <- A - v w^T - w v^T, w = p - (tau/2)(p.v) v, p = tau A v.
//
// * k_dc: eigen-decomposition T = Z diag(lambda) Z^T by Cuppen's divide and
//   conquer, bottom up from 4 x 4 blocks (each diagonalised by a few cyclic
//   Jacobi sweeps in one thread).  Every off-diagonal e_b between two blocks
//   is a tear: the two neighbouring diagonal entries lose |e_b|, and merging the blocks on
//   both sides of b is the rank-one problem D + rho z z^T with rho = |e_b| and
//   z = (last row of the left block's eigenvectors, sign(e_b) x first row of
//   the right block's).  Per merge: sort, deflate (negligible rho z_i, or two
//   close d's after a Givens rotation), solve the secular equation
//   1 + rho sum_j z_j^2 / (d_j - lambda) = 0 for each remaining root (each root
//   kept as an offset tau from its nearer pole so that lambda - d_j is exact),
//   recompute z from the roots (Gu-Eisenstat) so the vectors
//   u_i = z_i / (d_i - lambda) are orthogonal to working precision, and
//   multiply them into the block's eigenvectors on matrix cores.  All merges
//   of one level run together.
//
// * k_backtr: V = H_0 H_1 ... H_{m-3} Z, one wave per eigenvector with the
//   column in registers and the reflectors staged in LDS.
#include "fdsk_device.hpp"
#include "fdsk_kernels.hpp"
#include "fdsk_batch.hpp"

namespace fdsk {

namespace {

constexpr int TNT = 1024;                       // threads of the one-workgroup kernels
constexpr int TRI_PACK = kTridMax * (kTridMax + 1) / 2;

__device__ __forceinline__ int colstart(int j, int n) { return j * n - (j * (j - 1)) / 2; }

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

}  // namespace

// ----------------------------------------------------------------- reduce
// Output in W (doubles): [0, P) packed columns (column k holds v_k below the
// subdiagonal, P = n(n+1)/2), then tau[n], d[n], e[n], scale.  d and e are of
// G * 2^-s (an exact power-of-two scaling by the largest |g|); scale = 2^s.
// With kend < n - 2 only columns [0, kend) are reduced: W then holds their
// reflectors, d, e and tau, the scale, and the updated trailing block
// (columns >= kend of the packed triangle), which the register kernel
// finishes (its argument h = kend).
//
// Blocked by panels of HNB columns (the blocked form of the Householder
// tridiagonal reduction): within a panel the packed triangle keeps its
// values from the panel's start, A_0, and the reflectors' v and
// w = p - (tau/2)(p.v) v are collected in LDS; column k of the current matrix
// is A_0(:,k) - sum_q (v_q w_q(k) + w_q v_q(k)), and p = tau (A_0 v -
// sum_q (v_q (w_q.v) + w_q (v_q.v))).  The trailing block is written once
// per panel (A -= V W^T + W V^T).  Per column the triangle is only read, one
// wave per column (every HW-th), with each lane keeping the rows
// lane + 64 t (t < HT, so n <= 64 HT).  512 threads, two barriers per
// column.  Requires n > 64 (the unclamped loads below stay inside W).
constexpr int HNT = 512;                        // threads of the packed-triangle reduction
constexpr int HW = HNT / 64;                    // its waves
constexpr int HNB = 8;                          // panel width (<= HW)

template <int HT>
__device__ __forceinline__ void tridiag_body(const double* __restrict__ G, int n, int ldg,
                                             double* __restrict__ W, int kend) {
  constexpr int NM = 64 * HT;
  constexpr int UNR = HT <= 4 ? 4 : 2;          // columns per pass of the product
  constexpr int TG = HT <= 4 ? 4 : 2;           // row chunks per pass of the panel update
  __shared__ double Vp[HNB][NM];     // the panel's v
  __shared__ double Wq[HNB][NM];     // the panel's w
  __shared__ double ys[HW][NM];      // per-wave partial A_0 v
  // The current column and v are bitwise equal in every wave (each forms
  // them the same way), so the waves share one copy: every wave writes all
  // of it before reading, and any value it reads is its own or an equal one.
  __shared__ double colw[NM];
  __shared__ double vw[NM];
  __shared__ double pl[NM];
  __shared__ double ac[NM];          // next column: A_0 minus the older corrections
  __shared__ double sdp[4][NM];      // row-group partials of sum_{i >= jc} A_0(i,jc) v_i
  __shared__ double dg0[NM];         // diagonal of A_0
  __shared__ double cs[2][HNB];                  // w_q.v and v_q.v
  __shared__ double pd[HT];
  __shared__ double red[HW];
  static_assert(HNB <= HW, "one wave per panel column in the corrections");
  double* const A = W;
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int P = n * (n + 1) / 2;
  // The lower triangle, read by rows (coalesced): its largest magnitude,
  // then scaled into the packed columns.
  double amax = 0.0;
  for (int i = wv; i < n; i += HW) {
    const double* gi = G + static_cast<int64_t>(i) * ldg;
    for (int j = lane; j <= i; j += 64) amax = fmax(amax, fabs(gi[j]));
  }
  amax = wave_max(amax);
  if (lane == 0) red[wv] = amax;
  for (int e = tid; e < HNB * NM; e += HNT) {
    (&Vp[0][0])[e] = 0.0;
    (&Wq[0][0])[e] = 0.0;
  }
  __syncthreads();
  double gmax = 0.0;
  for (int i = 0; i < HW; ++i) gmax = fmax(gmax, red[i]);
  const int sexp = (gmax > 0.0 && gmax < INFINITY) ? ilogb(gmax) : 0;
  const double sc = ldexp(1.0, -sexp);
  for (int i = wv; i < n; i += HW) {
    const double* gi = G + static_cast<int64_t>(i) * ldg;
    for (int j = lane; j <= i; j += 64) A[colstart(j, n) + i - j] = gi[j] * sc;
    if (lane == 0) dg0[i] = gi[i] * sc;
  }
  __syncthreads();
  double* tauG = W + P;
  double* dG = tauG + n;
  double* eG = dG + n;
  const int kstop = min(kend, n - 2);
  double* const cw = colw;
  double* const vv = vw;
  // a: column k of the current matrix (rows lane + 64 t, zero above k and
  // at n and beyond); vprev/wprev: this wave's v and w of the previous step.
  double a[HT], vprev[HT], wprev[HT];
#pragma unroll
  for (int t = 0; t < HT; ++t) {
    const int i = lane + 64 * t;
    const double x = A[min(i, n - 1)];
    a[t] = (i < n) ? x : 0.0;
    vprev[t] = 0.0;
    wprev[t] = 0.0;
  }
  for (int k0 = 0; k0 < kstop; k0 += HNB) {
    const int nb = min(HNB, kstop - k0);
    for (int j = 0; j < nb; ++j) {
      const int k = k0 + j, k1 = k + 1;
      // Reflector, formed by every wave in the same order.
#pragma unroll
      for (int t = 0; t < HT; ++t) cw[lane + 64 * t] = a[t];
      __builtin_amdgcn_wave_barrier();
      const double alpha = cw[k1], dk = cw[k];
      double s2 = 0.0;
#pragma unroll
      for (int t = 0; t < HT; ++t) {
        const double x = (lane + 64 * t >= k + 2) ? a[t] : 0.0;
        s2 = fma(x, x, s2);
      }
      s2 = wave_sum(s2);
      double tau = 0.0, beta = alpha, scale = 0.0;
      if (s2 > 0.0) {
        const double mu = sqrt(alpha * alpha + s2);
        beta = (alpha >= 0.0) ? -mu : mu;
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      double v[HT];
#pragma unroll
      for (int t = 0; t < HT; ++t) {
        const int i = lane + 64 * t;
        v[t] = (i > k1) ? a[t] * scale : ((i == k1) ? 1.0 : 0.0);
        vv[i] = v[t];
      }
      __builtin_amdgcn_wave_barrier();
      if (wv == 0) {
#pragma unroll
        for (int t = 0; t < HT; ++t) Vp[j][lane + 64 * t] = v[t];
      }
      // Partial A_0 v over this wave's columns jc = k+1+wv, k+1+wv+HW, ...:
      // A_0(i, jc) v_jc into row i, and sum_{i > jc} A_0(i, jc) v_i into
      // row jc (the upper part, by symmetry).
      // Four columns per pass, their loads issued together.  Column jc's
      // entries sit at a uniform base plus the row, so the loads need no
      // per-lane clamping: rows above jc or at n and beyond read other
      // entries of the workspace (in bounds for n > 64), which the select
      // discards.  The transposed sums (diagonal included, removed when p is
      // assembled) leave as row-group partials through LDS.
      double acc[HT];
#pragma unroll
      for (int t = 0; t < HT; ++t) acc[t] = 0.0;
      for (int jc0 = k1 + wv; jc0 < n; jc0 += UNR * HW) {
        double x[UNR][HT];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int jcc = min(jc0 + u * HW, n - 1);
          const double* col = A + (colstart(jcc, n) - jcc);
#pragma unroll
          for (int t = 0; t < HT; ++t) x[u][t] = col[lane + 64 * t];
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int jc = jc0 + u * HW;
          const double vj = vv[min(jc, n - 1)];
          double sd = 0.0;
#pragma unroll
          for (int t = 0; t < HT; ++t) {
            const int i = lane + 64 * t;
            const double xm = (i >= jc && i < n) ? x[u][t] : 0.0;
            acc[t] = fma(xm, vj, acc[t]);
            sd = fma(xm, v[t], sd);
          }
          sd = row16_sum(sd);
          if ((lane & 15) == 0 && jc < n) sdp[lane >> 4][jc] = sd;
        }
      }
#pragma unroll
      for (int t = 0; t < HT; ++t) ys[wv][lane + 64 * t] = acc[t];
      // w_q.v and v_q.v for the panel's earlier columns, one wave each; the
      // previous step's pair is this wave's own registers.
      if (wv < j) {
        double s1 = 0.0, sv = 0.0;
        if (wv == j - 1) {
#pragma unroll
          for (int t = 0; t < HT; ++t) {
            s1 = fma(wprev[t], v[t], s1);
            sv = fma(vprev[t], v[t], sv);
          }
        } else {
#pragma unroll
          for (int t = 0; t < HT; ++t) {
            const int i = lane + 64 * t;
            s1 = fma(Wq[wv][i], v[t], s1);
            sv = fma(Vp[wv][i], v[t], sv);
          }
        }
        s1 = wave_sum(s1);
        sv = wave_sum(sv);
        if (lane == 0) {
          cs[0][wv] = s1;
          cs[1][wv] = sv;
        }
      }
      __syncthreads();
      // p for rows 64 wv + lane (waves below HT), its part of p.v, and the
      // next column of the panel less the corrections known so far.
      if (wv < HT) {
        const int i = 64 * wv + lane;
        double y = -dg0[i] * vv[i];
        for (int q = 0; q < HW; ++q) y += ys[q][i];
        for (int g = 0; g < 4; ++g) y += sdp[g][i];
        for (int q = 0; q < j; ++q) y -= fma(Vp[q][i], cs[0][q], Wq[q][i] * cs[1][q]);
        const double pi = (i > k && i < n) ? tau * y : 0.0;
        pl[i] = pi;
        const double d = wave_sum(pi * vv[i]);
        if (lane == 0) pd[wv] = d;
        if (j + 1 < nb) {
          const double raw = A[colstart(k1, n) + min(max(i, k1), n - 1) - k1];
          double x = (i >= k1 && i < n) ? raw : 0.0;
          for (int q = 0; q < j; ++q) x -= fma(Vp[q][i], Wq[q][k1], Wq[q][i] * Vp[q][k1]);
          ac[i] = (i >= k1) ? x : 0.0;
        }
      }
      // The reflector into column k (no wave reads column k any more).
      if (wv == 0) {
        const int ck = colstart(k, n);
#pragma unroll
        for (int t = 0; t < HT; ++t) {
          const int i = lane + 64 * t;
          if (i >= k + 2 && i < n) A[ck + i - k] = v[t];
        }
        if (lane == 0) {
          A[ck] = dk;
          A[ck + 1] = 1.0;
          dG[k] = dk;
          eG[k] = beta;
          tauG[k] = tau;
        }
      }
      __syncthreads();
      double dot = 0.0;
#pragma unroll
      for (int t = 0; t < HT; ++t) dot += pd[t];
      const double c = 0.5 * tau * dot;
      double w[HT];
#pragma unroll
      for (int t = 0; t < HT; ++t) w[t] = fma(-c, v[t], pl[lane + 64 * t]);
      if (wv == 0) {
#pragma unroll
        for (int t = 0; t < HT; ++t) Wq[j][lane + 64 * t] = w[t];
      }
      if (j + 1 < nb) {
        // Column k+1 of the current matrix: the q = j term is v w(k1) + w
        // (v(k1) = 1).
        const double wk1 = pl[k1] - c;
#pragma unroll
        for (int t = 0; t < HT; ++t) {
          const int i = lane + 64 * t;
          a[t] = (i >= k1 && i < n) ? ac[i] - fma(v[t], wk1, w[t]) : 0.0;
        }
      }
#pragma unroll
      for (int t = 0; t < HT; ++t) {
        vprev[t] = v[t];
        wprev[t] = w[t];
      }
    }
    // The panel's update of the trailing block: columns >= kt, one wave per
    // column, A -= V W^T + W V^T.  Each lane keeps its rows of V and W; a
    // column's coefficients are read once.  Loads are unconditional as in
    // the product above; only rows jc..n-1 are stored.
    __syncthreads();
    const int kt = k0 + nb;
#pragma unroll
    for (int tg = 0; tg < HT; tg += TG) {
      // Row chunks tg .. tg+TG-1.
      if (64 * (tg + TG) <= kt || 64 * tg >= n) continue;
      double vq[TG][HNB], wq[TG][HNB];
#pragma unroll
      for (int t = 0; t < TG; ++t)
#pragma unroll
        for (int q = 0; q < HNB; ++q) {
          vq[t][q] = (q < nb) ? Vp[q][lane + 64 * (tg + t)] : 0.0;
          wq[t][q] = (q < nb) ? Wq[q][lane + 64 * (tg + t)] : 0.0;
        }
      const int jend = min(n, 64 * (tg + TG));
      for (int jc = kt + wv; jc < jend; jc += HW) {
        double cwq[HNB], cvq[HNB];
#pragma unroll
        for (int q = 0; q < HNB; ++q) {
          cwq[q] = Wq[q][jc];
          cvq[q] = Vp[q][jc];
        }
        double* col = A + (colstart(jc, n) - jc);
        double x[TG];
#pragma unroll
        for (int t = 0; t < TG; ++t) x[t] = col[lane + 64 * (tg + t)];
#pragma unroll
        for (int t = 0; t < TG; ++t) {
          const int i = lane + 64 * (tg + t);
          double y = x[t];
#pragma unroll
          for (int q = 0; q < HNB; ++q) y -= fma(vq[t][q], cwq[q], wq[t][q] * cvq[q]);
          if (i >= jc && i < n) col[i] = y;
        }
      }
    }
    __syncthreads();
    for (int i = kt + tid; i < n; i += HNT) dg0[i] = A[colstart(i, n)];
    if (kt < kstop) {
      const int ct = colstart(kt, n);
#pragma unroll
      for (int t = 0; t < HT; ++t) {
        const int i = lane + 64 * t;
        const double x = A[ct + min(max(i, kt), n - 1) - kt];
        a[t] = (i >= kt && i < n) ? x : 0.0;
        vprev[t] = 0.0;
        wprev[t] = 0.0;
      }
    }
  }
  if (tid == 0) {
    if (kend >= n - 2) {
      if (n >= 2) {
        const int c2 = colstart(n - 2, n);
        dG[n - 2] = A[c2];
        eG[n - 2] = A[c2 + 1];
        tauG[n - 2] = 0.0;
      }
      dG[n - 1] = A[colstart(n - 1, n)];
      tauG[n - 1] = 0.0;
      eG[n - 1] = 0.0;
    }
    W[P + 3 * n] = ldexp(1.0, sexp);
  }
}

template <int HT>
__global__ __launch_bounds__(HNT) void k_tridiag(const double* __restrict__ G, int n, int ldg,
                                                 double* __restrict__ W, int kend) {
  tridiag_body<HT>(G, n, ldg, W, kend);
}

// ------------------------------------------------- reduce, in registers
// The same reduction with the matrix held in registers (n <= 32*RP and
// n <= 16*CP).  512 threads; thread (ti, tk) with ti = 4*wave + lane/16 in
// [0, 32) and tk = lane%16 keeps A(ti + 32a, tk + 16b), a < RP, b < CP, of
// the full symmetric matrix.  Per column k:
//  * every wave forms the reflector from column k (in LDS) itself, in the
//    same order, so all waves hold bitwise-equal tau and scale;
//  * p = tau A v: each thread sums its own columns, the 16 lanes of a row
//    group finish the row by a DPP butterfly, and one lane stores p_i;
//  * every wave forms c = (tau/2) p.v, then each thread applies
//    A -= v w^T + w v^T to its own elements, w = p - c v, with no LDS
//    traffic for A; the owners of column k+1 store it for the next step.
// Two barriers per column.  Column slots b < k1/16 hold finished columns
// only and are skipped.  The columns are taken in groups of 16 with the
// same first live slot B0, and each group is its own instantiation, so the
// slot loops carry no per-column tests: the product reads its slots of v at
// once, the update streams (v, p) three slots ahead.  Elements of finished
// rows (and the finished columns of slot B0) take meaningless but finite
// values: a finished row i has v_i = 0, so it is only multiplied by the
// reflector (A_i <- A_i - tau (A_i v) v^T), and every later v is zero on
// finished columns, so those elements are only ever multiplied by zero.
// With h > 0 the kernel continues a reduction that k_tridiag took through
// columns [0, h): it loads the trailing (ng-h) x (ng-h) block, already
// scaled, from W's packed triangle and writes reflectors h.. in place.
constexpr int RNT = 512;
constexpr int kTridRegMax = 208;   // 32 * 7 rows, 16 * 13 columns

template <int RP, int CP>
struct RegTrid {
  static constexpr int NB = (32 * RP > 16 * CP) ? 32 * RP : 16 * CP;
  static constexpr int NL = (NB + 63) / 64;    // strided entries per lane
  double* colb0;    // column k (k even) / k+1 (k odd), 64 NL rows
  double* colb1;
  double* pv;       // p = tau A v
  double* vv;       // this wave's copy of v
  double* dsh;      // d, e and tau of each column, written out at the end
  double* esh;
  double* tsh;
  double* W;        // packed reflectors (column h + k at colstart(h + k, ng))
  int n, ng, h, bend, ti, tk, lane, wv;
};

// Columns k in [kb, ke) (all with k+1 in slot B0).
template <int RP, int CP, int B0>
__device__ __forceinline__ void tridiag_reg_cols(const RegTrid<RP, CP>& c, double (&A)[RP][CP], int kb,
                                                 int ke) {
  constexpr int NL = RegTrid<RP, CP>::NL;
  constexpr int NS = CP - B0;        // live slots
  constexpr int PF = NS < 3 ? NS : 3;  // update prefetch distance
  const int lane = c.lane, wv = c.wv, ti = c.ti, tk = c.tk, n = c.n;
  double* const vv = c.vv;
  double* const pv = c.pv;
  for (int k = kb; k < ke; ++k) {
    const double* cb = (k & 1) ? c.colb1 : c.colb0;
    double* nb = (k & 1) ? c.colb0 : c.colb1;
    const int k1 = k + 1, tk1 = k1 & 15;
    double xs[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) xs[q] = cb[lane + 64 * q];
    const double alpha = cb[k1];
    double s2 = 0.0;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const double x = (lane + 64 * q >= k + 2) ? xs[q] : 0.0;
      s2 = fma(x, x, s2);
    }
    s2 = wave_sum(s2);
    double tau = 0.0, beta = alpha, scale = 0.0;
    if (s2 > 0.0) {
      const double mu = sqrt(alpha * alpha + s2);
      beta = (alpha >= 0.0) ? -mu : mu;
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    // This wave's copy of v: 0 up to k, 1 at k+1, x*scale below (0 beyond n,
    // where x = 0).  LDS operations of one wave complete in order, so the
    // wave reads its copy back after a wave barrier only (which keeps the
    // compiler from moving the reads above the writes).
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int t = lane + 64 * q;
      vv[t] = (t > k1) ? xs[q] * scale : ((t == k1) ? 1.0 : 0.0);
    }
    __builtin_amdgcn_wave_barrier();
    // The reflector's entries below the subdiagonal: wave q stores rows
    // lane + 64 q (every wave holds the same values).
    {
      const int ck = colstart(c.h + k, c.ng);
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int t = lane + 64 * q;
        if (wv == q && t >= k + 2 && t < n) c.W[ck + t - k] = xs[q] * scale;
      }
    }
    if (wv == RNT / 64 - 1 && lane == 0) {
      c.dsh[k] = cb[k];
      c.esh[k] = beta;
      c.tsh[k] = tau;
    }
    if (tau != 0.0) {                  // the same in every wave
      // p = tau A v over the live slots (v is zero on finished columns).
      double vk[NS];
#pragma unroll
      for (int j = 0; j < NS; ++j) vk[j] = vv[tk + 16 * (B0 + j)];
      double sp[RP];
#pragma unroll
      for (int a = 0; a < RP; ++a) sp[a] = 0.0;
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        if (B0 + j < c.bend) {
#pragma unroll
          for (int a = 0; a < RP; ++a) sp[a] = fma(A[a][B0 + j], vk[j], sp[a]);
        }
      }
#pragma unroll
      for (int a = 0; a < RP; ++a) {
        const double t = row16_sum(sp[a]);
        if (tk == 0) pv[ti + 32 * a] = tau * t;
      }
      __syncthreads();
      // c = (tau/2) p.v (v is zero up to k and beyond n).
      double dot = 0.0;
#pragma unroll
      for (int q = 0; q < NL; ++q) dot = fma(pv[lane + 64 * q], vv[lane + 64 * q], dot);
      dot = wave_sum(dot);
      const double cc = 0.5 * tau * dot;
      // A -= v w^T + w v^T with w = p - c v.
      double vr[RP], wr[RP];
#pragma unroll
      for (int a = 0; a < RP; ++a) {
        vr[a] = vv[ti + 32 * a];
        wr[a] = pv[ti + 32 * a];
      }
#pragma unroll
      for (int a = 0; a < RP; ++a) wr[a] = fma(-cc, vr[a], wr[a]);
      double nv[PF], np[PF];
#pragma unroll
      for (int j = 0; j < PF; ++j) {
        nv[j] = vv[tk + 16 * (B0 + j)];
        np[j] = pv[tk + 16 * (B0 + j)];
      }
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        const double vk1 = nv[j % PF], pk1 = np[j % PF];
        if (j + PF < NS) {
          nv[j % PF] = vv[tk + 16 * (B0 + j + PF)];
          np[j % PF] = pv[tk + 16 * (B0 + j + PF)];
        }
        if (B0 + j < c.bend) {
          const double wk = fma(-cc, vk1, pk1);
#pragma unroll
          for (int a = 0; a < RP; ++a) A[a][B0 + j] = fma(-vr[a], wk, fma(-wr[a], vk1, A[a][B0 + j]));
        }
        if (j == 0 && tk == tk1) {
#pragma unroll
          for (int a = 0; a < RP; ++a) nb[ti + 32 * a] = A[a][B0];
        }
      }
    } else {
      if (tk == tk1) {
#pragma unroll
        for (int a = 0; a < RP; ++a) nb[ti + 32 * a] = A[a][B0];
      }
    }
    __syncthreads();
  }
}

// Slot groups B0, B0+1, ..: the columns k with (k+1)/16 == B0.
template <int RP, int CP, int B0>
__device__ __forceinline__ void tridiag_reg_groups(const RegTrid<RP, CP>& c, double (&A)[RP][CP]) {
  if constexpr (B0 < CP) {
    const int kb = max(0, 16 * B0 - 1), ke = min(c.n - 2, 16 * B0 + 15);
    if (kb >= ke) return;
    tridiag_reg_cols<RP, CP, B0>(c, A, kb, ke);
    tridiag_reg_groups<RP, CP, B0 + 1>(c, A);
  }
}

template <int RP, int CP>
__device__ __forceinline__ void tridiag_reg_body(const double* __restrict__ G, int ng, int ldg,
                                                 double* __restrict__ W, int h) {
  using C = RegTrid<RP, CP>;
  constexpr int NL = C::NL;
  const int n = ng - h;                 // order of the block reduced here
  __shared__ double colb[2][64 * NL];
  __shared__ double pv[64 * NL];
  __shared__ double vwave[RNT / 64][64 * NL];   // each wave's copy of v
  __shared__ double dsh[64 * NL], esh[64 * NL], tsh[64 * NL];
  __shared__ double red[RNT / 64];
  // The wave index is made a scalar so that the slot tests below are
  // uniform branches.
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ti = 4 * wv + (lane >> 4), tk = lane & 15;
  for (int e = tid; e < 64 * NL; e += RNT) {
    colb[0][e] = 0.0;
    colb[1][e] = 0.0;
    pv[e] = 0.0;
  }
  double A[RP][CP];
  double amax = 0.0;
#pragma unroll
  for (int a = 0; a < RP; ++a) {
    const int i = ti + 32 * a;
#pragma unroll
    for (int b = 0; b < CP; ++b) {
      const int k = tk + 16 * b;
      double g = 0.0;
      if (i < n && k < n) {
        if (h == 0)
          g = (i >= k) ? G[static_cast<int64_t>(i) * ldg + k] : G[static_cast<int64_t>(k) * ldg + i];
        else
          g = (i >= k) ? W[colstart(h + k, ng) + i - k] : W[colstart(h + i, ng) + k - i];
      }
      A[a][b] = g;
      amax = fmax(amax, fabs(g));
    }
  }
  amax = wave_max(amax);
  if (lane == 0) red[wv] = amax;
  __syncthreads();
  double gmax = 0.0;
  for (int i = 0; i < RNT / 64; ++i) gmax = fmax(gmax, red[i]);
  const int sexp = (gmax > 0.0 && gmax < INFINITY) ? ilogb(gmax) : 0;
  const double sc = (h == 0) ? ldexp(1.0, -sexp) : 1.0;
#pragma unroll
  for (int a = 0; a < RP; ++a)
#pragma unroll
    for (int b = 0; b < CP; ++b) A[a][b] *= sc;
  if (tk == 0) {
#pragma unroll
    for (int a = 0; a < RP; ++a) {
      const int i = ti + 32 * a;
      if (i < n) colb[0][i] = A[a][0];
    }
  }
  __syncthreads();
  const int P = ng * (ng + 1) / 2;
  double* tauG = W + P;
  double* dG = tauG + ng;
  double* eG = dG + ng;
  C c;
  c.colb0 = colb[0];
  c.colb1 = colb[1];
  c.pv = pv;
  c.vv = vwave[wv];
  c.dsh = dsh;
  c.esh = esh;
  c.tsh = tsh;
  c.W = W;
  c.n = n;
  c.ng = ng;
  c.h = h;
  c.bend = (n + 15) >> 4;               // column slots b < bend hold a column < n
  c.ti = ti;
  c.tk = tk;
  c.lane = lane;
  c.wv = wv;
  tridiag_reg_groups<RP, CP, 0>(c, A);
  // d, e and tau of columns [0, n-2), and each packed column's head
  // (diagonal entry, then the reflector's leading 1).
  for (int k = tid; k < n - 2; k += RNT) {
    const int ck = colstart(h + k, ng);
    W[ck] = dsh[k];
    W[ck + 1] = 1.0;
    dG[h + k] = dsh[k];
    eG[h + k] = esh[k];
    tauG[h + k] = tsh[k];
  }
  // Column n-2 is in colb[(n-2) & 1] (n >= 2); A(n-1, n-1) is with its owner.
  if (tid == 0) {
    if (n >= 2) {
      const double* cb = colb[(n - 2) & 1];
      dG[ng - 2] = cb[n - 2];
      eG[ng - 2] = cb[n - 1];
      tauG[ng - 2] = 0.0;
      W[colstart(ng - 2, ng)] = cb[n - 2];
      W[colstart(ng - 2, ng) + 1] = cb[n - 1];
    }
    tauG[ng - 1] = 0.0;
    eG[ng - 1] = 0.0;
    if (h == 0) W[P + 3 * ng] = ldexp(1.0, sexp);
  }
#pragma unroll
  for (int a = 0; a < RP; ++a)
#pragma unroll
    for (int b = 0; b < CP; ++b)
      if (ti + 32 * a == n - 1 && tk + 16 * b == n - 1) {
        dG[ng - 1] = A[a][b];
        W[colstart(ng - 1, ng)] = A[a][b];
      }
}

template <int RP, int CP>
__global__ __launch_bounds__(RNT) void k_tridiag_reg(const double* __restrict__ G, int n, int ldg,
                                                     double* __restrict__ W, int h) {
  tridiag_reg_body<RP, CP>(G, n, ldg, W, h);
}

// ------------------------------------------------------ divide and conquer
namespace {

template <int NMAX>
struct DcSmem {
  double D[NMAX];      // eigenvalues per position of the current blocks
  double Ds[NMAX];     // sorted d (deflation rotations applied), then the roots
  double Zs[NMAX];     // sorted z
  double dh[NMAX];     // compact non-deflated d
  double zh[NMAX];     // compact non-deflated z
  double zg[NMAX];     // z recomputed from the roots
  double ddf[NMAX];    // compact deflated eigenvalues
  double rc[NMAX];     // deflation rotations of a merge, in scan order
  double rs[NMAX];
  double tau[NMAX];    // root offsets from their poles
  short rp[NMAX];      // rotation operands (sorted positions)
  short rj[NMAX];
  short perm[NMAX];    // sorted position -> local column
  short dest[NMAX];    // sorted position -> compact column
  short org[NMAX];     // root -> compact index of its pole
  short src[NMAX];     // compact column -> local column of the level's input
  int kk[NMAX / 2];    // non-deflated count per merge
  int nrot[NMAX / 2];  // deflation rotations per merge
  int tile0[NMAX / 2 + 1];
  int rot_any[NMAX / 2];  // the merge needs the sequential deflation scan
  char zdef[NMAX];        // 1 z-deflated, 2 rotation candidate, 0 otherwise
  double rv[NMAX];        // last merge: final eigenvalue of each column (ranking)
  char want[NMAX];        // last merge: the column's eigenvector is wanted
  int clo;                  // last merge: first wanted non-deflated column
  int cfirst;               // last merge: first column tile of its products
};

// Merge b of the level with half-size s: block [a, a+k1+k2).
__device__ __forceinline__ void merge_geom(int b, int s, int n, int& a, int& k1, int& k2) {
  a = 2 * s * b;
  k1 = min(s, n - a);
  k2 = max(0, min(s, n - a - s));
}

// Root `i` of 1 + rho sum_j zz_j^2 / (dd_j - lambda) = 0 over the sorted,
// non-deflated poles dd (kk of them, rho > 0): lambda_i lies in (dd_i,
// dd_{i+1}), the last one in (dd_{kk-1}, dd_{kk-1} + rho |zz|^2).  The root
// is kept as an offset tau from its nearer pole dd_o, so that every
// dd_j - lambda = (dd_j - dd_o) - tau is formed without cancellation.  Each
// step fits psi (poles up to i) and phi (poles above i) with one simple
// pole each at dd_i and dd_{i+1}, matching value and slope, and solves the
// resulting quadratic (the two-pole rational model of the secular-equation
// literature); the first iterate comes from the same model at the midpoint,
// where the origin is chosen.  Steps leaving the bracket fall back to
// geometric or plain bisection; the loop stops when g is at the rounding
// level of its own evaluation or the step is below 2 eps |tau|.  Four lanes
// (q = 0..3) share a root; returns o and writes tau.
__device__ int secular_root(const double* dd, const double* zz, int kk, int i, double rho, int q,
                            double& tau_out) {
  const double eps = 1.1102230246251565e-16;
  const double irho = 1.0 / rho;
  // Split sums at offset t from d0: p1 = sum_{j<=i} z_j^2/delta_j and its
  // slope dp1 = sum z_j^2/delta_j^2, p2 and dp2 over j > i.
  auto sums = [&](double d0, double t, double& p1, double& dp1, double& p2, double& dp2) {
    double a1 = 0.0, b1 = 0.0, a2 = 0.0, b2 = 0.0;
    for (int j = q; j <= i; j += 4) {
      const double r = zz[j] * rcp_nr((dd[j] - d0) - t);
      a1 = fma(zz[j], r, a1);
      b1 = fma(r, r, b1);
    }
    for (int j = i + 1 + ((q - i - 1) & 3); j < kk; j += 4) {
      const double r = zz[j] * rcp_nr((dd[j] - d0) - t);
      a2 = fma(zz[j], r, a2);
      b2 = fma(r, r, b2);
    }
    p1 = quad_sum(a1);
    dp1 = quad_sum(b1);
    p2 = quad_sum(a2);
    dp2 = quad_sum(b2);
  };
  // Step eta of the two-pole model from offset t (g = 1 + rho (p1 + p2)).
  auto model = [&](double d0, double t, double g, double p1, double dp1, double p2, double dp2,
                   double& eta) -> bool {
    const double Di = (dd[i] - d0) - t;
    if (i < kk - 1) {
      const double Di1 = (dd[i + 1] - d0) - t;
      const double C = irho + (p1 - dp1 * Di) + (p2 - dp2 * Di1);
      const double b = C * (Di + Di1) + dp1 * Di * Di + dp2 * Di1 * Di1;
      const double c0 = Di * Di1 * g * irho;
      const double disc = b * b - 4.0 * C * c0;
      if (!(disc >= 0.0)) return false;
      double e1, e2;
      if (C == 0.0) {
        if (b == 0.0) return false;
        e1 = e2 = c0 / b;
      } else {
        const double qq = 0.5 * (b + copysign(sqrt(disc), b));
        if (qq == 0.0) {
          e1 = e2 = 0.5 * b / C;
        } else {
          e1 = qq / C;
          e2 = c0 / qq;
        }
      }
      if (e1 > Di && e1 < Di1) { eta = e1; return true; }
      if (e2 > Di && e2 < Di1) { eta = e2; return true; }
      return false;
    }
    const double C = irho + (p1 - dp1 * Di);
    if (!(C > 0.0)) return false;
    eta = Di + dp1 * Di * Di / C;
    return true;
  };
  int o;
  double lo, hi, t, d0;
  if (i < kk - 1) {
    const double h = 0.5 * (dd[i + 1] - dd[i]);
    double p1, dp1, p2, dp2;
    sums(dd[i], h, p1, dp1, p2, dp2);
    const double g = 1.0 + rho * (p1 + p2);
    if (g >= 0.0) {
      o = i; lo = 0.0; hi = h; t = h;
    } else {
      o = i + 1; lo = -h; hi = 0.0; t = -h;
    }
    d0 = dd[o];
    double eta;
    double tn = model(d0, t, g, p1, dp1, p2, dp2, eta) ? t + eta : 0.5 * (lo + hi);
    if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
    t = tn;
  } else {
    double z2 = 0.0;
    for (int j = q; j < kk; j += 4) z2 = fma(zz[j], zz[j], z2);
    o = kk - 1; lo = 0.0; hi = rho * quad_sum(z2); t = 0.5 * hi;
    d0 = dd[o];
  }
  for (int it = 0; it < 100; ++it) {
    double p1, dp1, p2, dp2;
    sums(d0, t, p1, dp1, p2, dp2);
    const double g = 1.0 + rho * (p1 + p2);
    if (fabs(g) <= 8.0 * eps * (1.0 + rho * (fabs(p1) + fabs(p2)))) break;
    if (g > 0.0) hi = t; else lo = t;
    double eta;
    if (!model(d0, t, g, p1, dp1, p2, dp2, eta)) eta = -g / (rho * (dp1 + dp2));
    double tn = t + eta;
    if (fabs(eta) <= 2.0 * eps * fabs(t)) { t = tn; break; }
    if (!(tn > lo && tn < hi)) {
      if (lo > 0.0 && hi > 16.0 * lo) tn = sqrt(lo * hi);
      else if (hi < 0.0 && lo < 16.0 * hi) tn = -sqrt(lo * hi);
      else tn = 0.5 * (lo + hi);
    }
    if (tn == t || !(hi - lo > 2.0 * eps * fmax(fabs(lo), fabs(hi)))) { t = tn; break; }
    t = tn;
  }
  tau_out = t;
  return o;
}

}  // namespace

// T = Z diag(lambda) Z^T for the tridiagonal (d, e) written by k_tridiag in W.
// Z (n x n, column-major, leading dimension ldz) and lambda are the outputs;
// Qc, U (ldz) are scratch.  Only the eigenvectors of the nvec largest
// eigenvalues (descending, ties to the lower index, NaN last: the order the
// shrink ranks them in) are wanted; the last merge forms only those of its
// non-deflated roots (they are a suffix: the roots ascend), and the wanted
// columns are flagged (1.0 / 0.0) at W[P + 3n + 1 + j] for the
// back-transformation.  Other columns of Z are left undefined.
template <int NMAX, int NT>
__device__ __forceinline__ void dc_body(double* __restrict__ W, int n, double* __restrict__ Z, int ldz,
                                        double* __restrict__ Qc, double* __restrict__ U,
                                        double* __restrict__ lam, DevStats* __restrict__ st, int nvec) {
  __shared__ DcSmem<NMAX> S;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int P = n * (n + 1) / 2;
  const double* dG = W + P + n;
  const double* eG = dG + n;
  const double scale = W[P + 3 * n];
  // The eigenvectors of the current blocks alternate between Z and Qc from
  // level to level (each level reads one and writes the other), starting in
  // the one that makes the last level write Z.  Both start as I: a level
  // reads, within its merge blocks, entries that no earlier level wrote
  // (between two blocks of the level before), and those must be zero.
  // The first two levels are replaced by blocks of 4 (the last one possibly
  // smaller) solved directly below, so the merge levels start from blocks
  // of 4.
  int levels = 0;
  for (int s = 4; s < n; s *= 2) ++levels;
  int cur = levels & 1;
  for (int c = w; c < n; c += NT / 64)
    for (int r = lane; r < n; r += 64) {
      Z[static_cast<int64_t>(c) * ldz + r] = (r == c) ? 1.0 : 0.0;
      Qc[static_cast<int64_t>(c) * ldz + r] = (r == c) ? 1.0 : 0.0;
    }
  for (int i = tid; i < n; i += NT) {
    const double el = (i > 0) ? fabs(eG[i - 1]) : 0.0;
    const double er = (i < n - 1) ? fabs(eG[i]) : 0.0;
    S.D[i] = dG[i] - el - er;
  }
  __syncthreads();
  // Block p (rows 4p .. 4p + k - 1, k <= 4) with its inner off-diagonals
  // restored, diagonalised by one thread with cyclic Jacobi: six sweeps
  // over the six planes, rotation (cs, sn) from zeta = (a_qq - a_pp) / 2a_pq
  // and t the smaller root of t^2 + 2 zeta t = 1 (quadratic convergence:
  // four by four blocks reach rounding level in about three sweeps).
  {
    double* In0 = cur ? Qc : Z;
    for (int p = tid; 4 * p < n; p += NT) {
      const int i0 = 4 * p, k = min(4, n - i0);
      double A[4][4], V[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          A[r][c] = 0.0;
          V[r][c] = (r == c) ? 1.0 : 0.0;
        }
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (j < k) {
          const double inl = (j > 0) ? fabs(eG[i0 + j - 1]) : 0.0;
          const double inr = (j < k - 1) ? fabs(eG[i0 + j]) : 0.0;
          A[j][j] = S.D[i0 + j] + inl + inr;
          if (j < k - 1) A[j][j + 1] = A[j + 1][j] = eG[i0 + j];
        }
      for (int sweep = 0; sweep < 6; ++sweep) {
#pragma unroll
        for (int pq = 0; pq < 6; ++pq) {
          const int pp = pq < 3 ? 0 : (pq < 5 ? 1 : 2);
          const int qq = pq < 3 ? pq + 1 : (pq < 5 ? pq - 1 : 3);
          const double apq = A[pp][qq];
          if (qq < k && apq != 0.0) {
            const double zeta = (A[qq][qq] - A[pp][pp]) / (2.0 * apq);
            const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(fma(zeta, zeta, 1.0)));
            const double cs = 1.0 / sqrt(fma(t, t, 1.0)), sn = t * cs;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              if (r != pp && r != qq) {
                const double arp = A[r][pp], arq = A[r][qq];
                A[r][pp] = A[pp][r] = cs * arp - sn * arq;
                A[r][qq] = A[qq][r] = sn * arp + cs * arq;
              }
            }
            A[pp][pp] -= t * apq;
            A[qq][qq] += t * apq;
            A[pp][qq] = A[qq][pp] = 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const double vrp = V[r][pp], vrq = V[r][qq];
              V[r][pp] = cs * vrp - sn * vrq;
              V[r][qq] = sn * vrp + cs * vrq;
            }
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (j < k) {
          S.D[i0 + j] = A[j][j];
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (r < k) In0[static_cast<int64_t>(i0 + j) * ldz + i0 + r] = V[r][j];
        }
    }
  }
  __syncthreads();
  const double eps = 1.1102230246251565e-16;
  // Four lanes per root in the per-root steps.
  const int g4 = tid >> 2, q4 = tid & 3;
  for (int s = 4; s < n; s *= 2, cur ^= 1) {
    // Selected, not indexed from a local array, so that the loads below
    // stay global (flat loads would also count against the LDS counter).
    const double* In = cur ? Qc : Z;
    double* Out = cur ? Z : Qc;
    const int nm = (n + 2 * s - 1) / (2 * s);
    // 1. z from the boundary rows, sorted by eigenvalue within each merge.
    for (int g = tid; g < n; g += NT) {
      const int b = g / (2 * s);
      int a, k1, k2;
      merge_geom(b, s, n, a, k1, k2);
      if (k2 == 0) continue;
      const int k = k1 + k2, j = g - a;
      const double beta = eG[a + k1 - 1];
      const double zj = (j < k1) ? In[static_cast<int64_t>(a + j) * ldz + a + k1 - 1]
                                 : ((beta >= 0.0) ? 1.0 : -1.0) * In[static_cast<int64_t>(a + j) * ldz + a + k1];
      const double dj = S.D[g];
      int rank = 0;
      for (int i = 0; i < k; ++i) {
        const double di = S.D[a + i];
        rank += (di < dj) || (di == dj && i < j);
      }
      S.perm[a + rank] = static_cast<short>(j);
      S.Ds[a + rank] = dj;
      S.Zs[a + rank] = zj * 0.70710678118654752440;
    }
    __syncthreads();
    // 2. Deflation.  a) z-deflation flags (negligible rho |z_j|) and, for the
    //    other entries, whether the previous such entry is close enough for a
    //    Givens rotation (tested on the unrotated values).
    for (int g = tid; g < n; g += NT) {
      const int b = g / (2 * s);
      int a, k1, k2;
      merge_geom(b, s, n, a, k1, k2);
      if (k2 == 0) continue;
      const int k = k1 + k2, j = g - a;
      const double rho = 2.0 * fabs(eG[a + k1 - 1]);
      const double tol = 8.0 * eps * fmax(fmax(fabs(S.Ds[a]), fabs(S.Ds[a + k - 1])), rho);
      const bool zd = rho * fabs(S.Zs[g]) <= tol;
      S.zdef[g] = zd ? 1 : 0;
      if (j == 0) S.rot_any[b] = 0;
      if (zd) continue;
      int p = j - 1;
      while (p >= 0 && rho * fabs(S.Zs[a + p]) <= tol) --p;
      if (p < 0) continue;
      const double zl = S.Zs[a + p], zj = S.Zs[g];
      const double th = hypot(zl, zj);
      const double c = zj / th, sn = zl / th;
      if (fabs((S.Ds[g] - S.Ds[a + p]) * c * sn) <= tol) S.zdef[g] = 2;
    }
    __syncthreads();
    for (int g = tid; g < n; g += NT) {
      const int b = g / (2 * s);
      if (S.zdef[g] == 2) S.rot_any[b] = 1;
    }
    __syncthreads();
    //    b) Merges without a rotation: compact in parallel (non-deflated
    //    first, in sorted order, then the deflated ones).  Merges with one:
    //    the sequential scan below, where each rotation changes the pending
    //    entry's d and z.
    for (int g = tid; g < n; g += NT) {
      const int b = g / (2 * s);
      int a, k1, k2;
      merge_geom(b, s, n, a, k1, k2);
      if (k2 == 0 || S.rot_any[b]) continue;
      const int k = k1 + k2, j = g - a;
      int before = 0, total = 0;
      for (int i = 0; i < k; ++i) {
        const int nd_i = (S.zdef[a + i] == 0) ? 1 : 0;
        total += nd_i;
        before += (i < j) ? nd_i : 0;
      }
      if (S.zdef[g] == 0) {
        S.dest[g] = static_cast<short>(before);
        S.dh[a + before] = S.Ds[g];
        S.zh[a + before] = S.Zs[g];
      } else {
        const int di = j - before;
        S.dest[g] = static_cast<short>(total + di);
        S.ddf[a + di] = S.Ds[g];
      }
      if (j == 0) {
        S.kk[b] = total;
        S.nrot[b] = 0;
      }
    }
    for (int b = tid; b < nm; b += NT) {
      int a, k1, k2;
      merge_geom(b, s, n, a, k1, k2);
      if (k2 == 0 || !S.rot_any[b]) continue;
      const int k = k1 + k2;
      const double rho = 2.0 * fabs(eG[a + k1 - 1]);
      const double tol = 8.0 * eps * fmax(fmax(fabs(S.Ds[a]), fabs(S.Ds[a + k - 1])), rho);
      int nk = 0, nd = 0, nr = 0, last = -1;
      for (int j = 0; j < k; ++j) {
        const int pj = a + j;
        if (rho * fabs(S.Zs[pj]) <= tol) {
          S.dest[pj] = static_cast<short>(-1 - nd);
          S.ddf[a + nd] = S.Ds[pj];
          ++nd;
          continue;
        }
        if (last >= 0) {
          const int pl = a + last;
          const double zl = S.Zs[pl], zj = S.Zs[pj];
          const double th = hypot(zl, zj);
          const double c = zj / th, sn = zl / th;
          const double t = S.Ds[pj] - S.Ds[pl];
          if (fabs(t * c * sn) <= tol) {
            const double dl = S.Ds[pl], dj = S.Ds[pj];
            S.Ds[pl] = c * c * dl + sn * sn * dj;
            S.Ds[pj] = sn * sn * dl + c * c * dj;
            S.Zs[pj] = th;
            S.Zs[pl] = 0.0;
            S.rp[a + nr] = static_cast<short>(pl);
            S.rj[a + nr] = static_cast<short>(pj);
            S.rc[a + nr] = c;
            S.rs[a + nr] = sn;
            ++nr;
            S.dest[pl] = static_cast<short>(-1 - nd);
            S.ddf[a + nd] = S.Ds[pl];
            ++nd;
            last = j;
            continue;
          }
          S.dest[pl] = static_cast<short>(nk);
          S.dh[a + nk] = S.Ds[pl];
          S.zh[a + nk] = S.Zs[pl];
          ++nk;
        }
        last = j;
      }
      if (last >= 0) {
        const int pl = a + last;
        S.dest[pl] = static_cast<short>(nk);
        S.dh[a + nk] = S.Ds[pl];
        S.zh[a + nk] = S.Zs[pl];
        ++nk;
      }
      for (int j = 0; j < k; ++j)
        if (S.dest[a + j] < 0) S.dest[a + j] = static_cast<short>(nk + (-1 - S.dest[a + j]));
      S.kk[b] = nk;
      S.nrot[b] = nr;
    }
    __syncthreads();
    // The last merge covers the whole matrix; with nvec < n it forms only
    // the wanted eigenvectors.
    const bool part = (2 * s >= n) && nvec < n;
    if (tid == 0) {
      int acc = 0;
      for (int b = 0; b < nm; ++b) {
        int a, k1, k2;
        merge_geom(b, s, n, a, k1, k2);
        S.tile0[b] = acc;
        if (k2 > 0) acc += ((k1 + k2 + 31) / 32) * ((S.kk[b] + 15) / 16);
      }
      S.tile0[nm] = acc;
      S.clo = n;
      S.cfirst = 0;
    }
    // 3. Compact column dest[j] of the merge is the input's local column
    //    perm[j]; the products below read the input through this map.
    for (int g = tid; g < n; g += NT) {
      const int b = g / (2 * s);
      int a, k1, k2;
      merge_geom(b, s, n, a, k1, k2);
      if (k2 == 0) continue;
      S.src[a + S.dest[g]] = S.perm[g];
    }
    // 4. Secular roots, four lanes per root.
    for (int g = g4; g < n; g += NT / 4) {
      const int b = g / (2 * s);
      int a, k1, k2;
      merge_geom(b, s, n, a, k1, k2);
      if (k2 == 0) continue;
      const int i = g - a;
      const int nk = S.kk[b];
      if (i >= nk) continue;
      const double rho = 2.0 * fabs(eG[a + k1 - 1]);
      double t;
      const int o = secular_root(S.dh + a, S.zh + a, nk, i, rho, q4, t);
      if (q4 == 0) {
        S.org[g] = static_cast<short>(o);
        S.tau[g] = t;
      }
    }
    __syncthreads();
    if (part) {
      // Rank every final eigenvalue (the same expressions as below, so the
      // same doubles) and mark the nvec largest.
      const int nk0 = S.kk[0];
      for (int c = tid; c < n; c += NT) {
        const double v = (c < nk0) ? S.dh[S.org[c]] + S.tau[c] : S.ddf[c - nk0];
        S.rv[c] = (v == v) ? v : -INFINITY;
      }
      __syncthreads();
      for (int c = tid; c < n; c += NT) {
        const double vc = S.rv[c];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
          const double vj = S.rv[j];
          rank += (vj > vc) || (vj == vc && j < c);
        }
        const bool wt = rank < nvec;
        S.want[c] = wt ? 1 : 0;
        if (wt && c < nk0) atomicMin(&S.clo, c);
      }
      __syncthreads();
      if (tid == 0) {
        int a, k1, k2;
        merge_geom(0, s, n, a, k1, k2);
        const int nct = (nk0 + 15) / 16, cf = min(S.clo, nk0) / 16;
        S.cfirst = cf;
        S.tile0[1] = ((k1 + k2 + 31) / 32) * max(0, nct - cf);
      }
    }
    // 3b. Deflation rotations, in place on the input's columns (read only
    //    by the products and copies below), one thread per row.
    for (int g = tid; g < n; g += NT) {
      const int b = g / (2 * s);
      int a, k1, k2;
      merge_geom(b, s, n, a, k1, k2);
      if (k2 == 0) continue;
      const int nr = S.nrot[b];
      double* InW = cur ? Qc : Z;
      for (int t = 0; t < nr; ++t) {
        double* xp = InW + static_cast<int64_t>(a + S.perm[S.rp[a + t]]) * ldz + g;
        double* xj = InW + static_cast<int64_t>(a + S.perm[S.rj[a + t]]) * ldz + g;
        const double c = S.rc[a + t], sn = S.rs[a + t];
        const double x = *xp, y = *xj;
        *xp = c * x - sn * y;
        *xj = sn * x + c * y;
      }
    }
    // 5. z recomputed from the roots (Gu-Eisenstat), signs of z kept:
    //    rho z_i^2 = prod_j (lambda_j - d_i) / prod_{j != i} (d_j - d_i).
    for (int g = g4; g < n; g += NT / 4) {
      const int b = g / (2 * s);
      int a, k1, k2;
      merge_geom(b, s, n, a, k1, k2);
      if (k2 == 0) continue;
      const int i = g - a;
      const int nk = S.kk[b];
      if (i >= nk) continue;
      const double rho = 2.0 * fabs(eG[a + k1 - 1]);
      const double* dd = S.dh + a;
      const double di = dd[i];
      double prod = (q4 == 0) ? ((dd[S.org[g]] - di) + S.tau[g]) / rho : 1.0;
      for (int j = q4; j < nk; j += 4) {
        if (j == i) continue;
        prod *= ((dd[S.org[a + j]] - di) + S.tau[a + j]) / (dd[j] - di);
      }
      prod = quad_prod(prod);
      const double zn = sqrt(fabs(prod));
      if (q4 == 0) S.zg[g] = (S.zh[g] >= 0.0) ? zn : -zn;
    }
    __syncthreads();
    // 6. Secular eigenvectors, four lanes per root: U(i, j) = z_i / (d_i -
    //    lambda_j), normalised; U row-major within the merge's block.
    for (int g = g4; g < n; g += NT / 4) {
      const int b = g / (2 * s);
      int a, k1, k2;
      merge_geom(b, s, n, a, k1, k2);
      if (k2 == 0) continue;
      const int j = g - a;
      const int nk = S.kk[b];
      if (j >= nk) continue;
      const double* dd = S.dh + a;
      const double dj = dd[S.org[g]], tj = S.tau[g];
      if (q4 == 0) S.Ds[g] = dj + tj;                  // the root
      if (part && j < S.clo) continue;                 // eigenvector not wanted
      double nrm = 0.0;
      for (int i = q4; i < nk; i += 4) {
        const double u = S.zg[a + i] * rcp_nr((dd[i] - dj) - tj);
        nrm = fma(u, u, nrm);
      }
      const double inv = rsq_nr(quad_sum(nrm));
      for (int i = q4; i < nk; i += 4) {
        const double u = S.zg[a + i] * rcp_nr((dd[i] - dj) - tj);
        U[static_cast<int64_t>(a + i) * ldz + a + j] = u * inv;
      }
    }
    __syncthreads();
    // 7. Output block = (input columns src[0:nk]) U on matrix cores.  A wave
    //    computes two vertically adjacent 16 x 16 tiles (sharing the U
    //    fragment).
    const int ntile = S.tile0[nm];
    for (int t = w; t < ntile; t += NT / 64) {
      int b = 0;
      while (S.tile0[b + 1] <= t) ++b;
      int a, k1, k2;
      merge_geom(b, s, n, a, k1, k2);
      const int k = k1 + k2, nk = S.kk[b];
      const int cf = part ? S.cfirst : 0;
      const int nct = (nk + 15) / 16 - cf;
      const int tl = t - S.tile0[b];
      const int r0 = (tl / nct) * 32, c0 = (cf + tl % nct) * 16;
      const int li = lane & 15, lk = lane >> 4;
      f64x4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
      const bool rok0 = (r0 + li) < k, rok1 = (r0 + 16 + li) < k, cok = (c0 + li) < nk;
      // Row and column indices are clamped into the block, so every load is
      // unconditional and reads a finite entry of the block; the padding is
      // zeroed by multiplying with 0/1 at the product, which lets the next
      // 16-deep slab stay in flight while the current one goes through the
      // matrix cores.
      const double* Ab0 = In + static_cast<int64_t>(a) * ldz + a + min(r0 + li, k - 1);
      const double* Ab1 = In + static_cast<int64_t>(a) * ldz + a + min(r0 + 16 + li, k - 1);
      const double* Bb = U + static_cast<int64_t>(a) * ldz + a + min(c0 + li, nk - 1);
      const double m0 = rok0 ? 1.0 : 0.0, m1 = rok1 ? 1.0 : 0.0, mc = cok ? 1.0 : 0.0;
      auto slab = [&](int i0, double (&x0)[4], double (&x1)[4], double (&y)[4]) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int ic = min(i0 + 4 * u + lk, nk - 1);
          const int64_t oa = static_cast<int64_t>(S.src[a + ic]) * ldz;
          x0[u] = Ab0[oa];
          x1[u] = Ab1[oa];
          y[u] = Bb[static_cast<int64_t>(ic) * ldz];
        }
      };
      double x0[4], x1[4], y[4];
      slab(0, x0, x1, y);
      for (int i0 = 0; i0 < nk; i0 += 16) {
        double n0[4], n1[4], ny[4];
        slab(i0 + 16, n0, n1, ny);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double mk = (i0 + 4 * u + lk < nk) ? 1.0 : 0.0;
          const double yu = y[u] * (mc * mk);
          acc0 = mfma_f64(x0[u] * m0, yu, acc0);
          acc1 = mfma_f64(x1[u] * m1, yu, acc1);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          x0[u] = n0[u];
          x1[u] = n1[u];
          y[u] = ny[u];
        }
      }
      if (cok) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = r0 + lk + 4 * v;
          double* zc = Out + static_cast<int64_t>(a + c0 + li) * ldz + a;
          if (row < k) zc[row] = acc0[v];
          if (row + 16 < k) zc[row + 16] = acc1[v];
        }
      }
    }
    // Deflated columns (compact index >= kk) are copied unchanged, and so
    // are the columns of a block with no partner at this level.
    for (int g = w; g < n; g += NT / 64) {
      const int b = g / (2 * s);
      int a, k1, k2;
      merge_geom(b, s, n, a, k1, k2);
      int k, from;
      if (k2 == 0) {
        k = k1;
        from = g;
      } else {
        if (g - a < S.kk[b]) continue;
        k = k1 + k2;
        from = a + S.src[g];
      }
      const double* src = In + static_cast<int64_t>(from) * ldz + a;
      double* dst = Out + static_cast<int64_t>(g) * ldz + a;
      for (int r = lane; r < k; r += 64) dst[r] = src[r];
    }
    __syncthreads();
    for (int g = tid; g < n; g += NT) {
      const int b = g / (2 * s);
      int a, k1, k2;
      merge_geom(b, s, n, a, k1, k2);
      if (k2 == 0) continue;
      const int j = g - a;
      const int nk = S.kk[b];
      S.D[g] = (j < nk) ? S.Ds[g] : S.ddf[a + (j - nk)];
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += NT) lam[i] = S.D[i] * scale;
  const bool flagged = n >= 2 && nvec < n;
  for (int i = tid; i < n; i += NT) W[P + 3 * n + 1 + i] = (!flagged || S.want[i]) ? 1.0 : 0.0;
  if (tid == 0 && st) atomicAdd(&st->eig_sweeps, 1ull);
}

template <int NMAX>
__global__ __launch_bounds__(TNT) void k_dc(double* __restrict__ W, int n, double* __restrict__ Z, int ldz,
                                            double* __restrict__ Qc, double* __restrict__ U,
                                            double* __restrict__ lam, DevStats* __restrict__ st, int nvec) {
  dc_body<NMAX, TNT>(W, n, Z, ldz, Qc, U, lam, st, nvec);
}

// ---------------------------------------------------------- back-transform
// Z <- H_0 H_1 ... H_{n-3} Z for every wanted column (flagged by the divide
// and conquer), in place: one wave per column, NPL elements per lane, the
// packed reflectors staged in LDS.  A column's reflectors are a sequential
// chain, so the time is that of one wave's chain: blocks have one wave per
// SIMD, and wave w of block cb takes the (4 cb + w)-th wanted column.
constexpr int BNT = 256;

// The t-th (0-based) column flagged in W[F .. F+n), or -1; also the count.
__device__ __forceinline__ int nth_flagged(const double* __restrict__ flags, int n, int t, int& count) {
  const int lane = threadIdx.x & 63;
  int col = -1, seen = 0;
  for (int c0 = 0; c0 < n; c0 += 64) {
    const bool f = (c0 + lane < n) && flags[c0 + lane] != 0.0;
    const unsigned long long m = __ballot(f);
    const int cnt = __popcll(m);
    if (col < 0 && t >= seen && t < seen + cnt) {
      const int before = __popcll(m & ((1ull << lane) - 1ull));
      const unsigned long long hit = __ballot(f && (seen + before == t));
      col = c0 + __ffsll(static_cast<long long>(hit)) - 1;
    }
    seen += cnt;
  }
  count = seen;
  return col;
}

// Packed reflectors of an order up to 64*NPL, staged in LDS (n <= kTridMax).
constexpr int bt_pack(int npl) {
  return (64 * npl) * (64 * npl + 1) / 2 < TRI_PACK ? (64 * npl) * (64 * npl + 1) / 2 : TRI_PACK;
}

// NT threads per block, one wave per wanted column: block cb takes wanted
// columns cb*NT/64 .. cb*NT/64 + NT/64 - 1.
template <int NPL, bool GA, int NT = BNT>
__device__ __forceinline__ void backtr_body(const double* __restrict__ W, int n, double* __restrict__ Z,
                                            int ldz, int cb) {
  __shared__ double R_lds[GA ? 1 : bt_pack(NPL)];
  __shared__ double tau_lds[64 * NPL];
  const double* const R = GA ? W : R_lds;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int P = n * (n + 1) / 2;
  int nw;
  const int col = nth_flagged(W + P + 3 * n + 1, n, cb * (NT / 64) + w, nw);
  if (cb * (NT / 64) >= nw) return;      // the whole block: no wanted column left
  if (!GA)
    for (int e = tid; e < P; e += NT) R_lds[e] = W[e];
  for (int e = tid; e < n; e += NT) tau_lds[e] = W[P + e];
  __syncthreads();
  if (col < 0) return;
  double z[NPL];
  double* zc = Z + static_cast<int64_t>(col) * ldz;
#pragma unroll
  for (int t = 0; t < NPL; ++t) {
    const int i = lane + 64 * t;
    z[t] = (i < n) ? zc[i] : 0.0;
  }
  // Reflector k's v (and tau) are fetched while reflector k+1 is applied.
  auto fetch = [&](int k, double* v) {
    const int ck = colstart(k, n);
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int i = lane + 64 * t;
      const double x = R[ck + min(max(i - k, 0), n - 1 - k)];
      v[t] = (i == k + 1) ? 1.0 : ((i > k + 1 && i < n) ? x : 0.0);
    }
  };
  double v[NPL];
  if (n >= 3) fetch(n - 3, v);
  for (int k = n - 3; k >= 0; --k) {
    const double tk = tau_lds[k];
    double cv[NPL];
#pragma unroll
    for (int t = 0; t < NPL; ++t) cv[t] = v[t];
    if (k > 0) fetch(k - 1, v);
    if (tk == 0.0) continue;
    double dot = 0.0;
#pragma unroll
    for (int t = 0; t < NPL; ++t) dot = fma(cv[t], z[t], dot);
    dot = wave_sum(dot) * tk;
#pragma unroll
    for (int t = 0; t < NPL; ++t) z[t] = fma(-dot, cv[t], z[t]);
  }
#pragma unroll
  for (int t = 0; t < NPL; ++t) {
    const int i = lane + 64 * t;
    if (i < n) zc[i] = z[t];
  }
}

template <int NPL, bool GA>
__global__ __launch_bounds__(BNT) void k_backtr(const double* __restrict__ W, int n,
                                                double* __restrict__ Z, int ldz) {
  backtr_body<NPL, GA>(W, n, Z, ldz, blockIdx.x);
}

// The same product in blocks of 16 reflectors (compact WY form): the
// reflectors k0 .. k0+15 multiply to I - V T V^T, with V their vectors
// (n x 16) and T upper triangular, T_jj = tau_j and column i above the
// diagonal -tau_i T(0:i, 0:i) V(:, 0:i)^T v_i.  Q Z = H_0 H_1 ... H_{n-3} Z
// applies the blocks from the last to the first, each as
// Z -= V (T (V^T Z)), all three products on FP64 matrix cores.  A wave holds
// 16 wanted columns of Z in registers for the whole product, as MFMA
// accumulators: lane l keeps rows 16r + l/16 + 4v (v = 0..3) of column l%16
// for row tile r.  Entry v of that tile is also the B operand of the K
// slice of rows 16r + 4v .. 16r + 4v + 3, so V^T Z reads Z from the
// accumulators directly.  Rows of V above k0 + 1 are zero and their tiles
// are skipped.  Block cb takes the wanted columns 16 NWV cb .. ; RTM row
// tiles cover n <= 16 RTM.
template <int RTM, int NWV>
__device__ __forceinline__ void backtr_wy_body(const double* __restrict__ W, int n, double* __restrict__ Z,
                                               int ldz, int cb) {
  constexpr int NT = 64 * NWV;
  __shared__ double Vs[16 * RTM][17];
  __shared__ double Gp[NWV][16][17];
  __shared__ double Gs[16][17];
  __shared__ double Ts[16][17];
  __shared__ double tau_s[16];
  __shared__ int cols[NWV][16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int P = n * (n + 1) / 2;
  const double* flags = W + P + 3 * n + 1;
  // This wave's 16 wanted columns: wanted columns 16 (NWV cb + w) + j.
  const int base = 16 * (NWV * cb + w);
  if (lane < 16) cols[w][lane] = -1;
  int seen = 0;
  for (int c0 = 0; c0 < n; c0 += 64) {
    const bool f = (c0 + lane < n) && flags[c0 + lane] != 0.0;
    const unsigned long long msk = __ballot(f);
    const int pos = seen + __popcll(msk & ((1ull << lane) - 1ull));
    if (f && pos >= base && pos < base + 16) cols[w][pos - base] = c0 + lane;
    seen += __popcll(msk);
  }
  if (16 * NWV * cb >= seen) return;     // the whole block: no wanted column (uniform)
  __syncthreads();
  const int rt = (n + 15) / 16;
  const int col = cols[w][li];
  f64x4 Zt[RTM];
#pragma unroll
  for (int r = 0; r < RTM; ++r) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * r + lk + 4 * v;
      Zt[r][v] = (r < rt && col >= 0 && row < n) ? Z[static_cast<int64_t>(col) * ldz + row] : 0.0;
    }
  }
  const int nref = n - 2;
  // A block's V (rows 16 rlo .. 16 rt, consecutive threads on consecutive
  // rows of one packed column) and tau, fetched into registers one block
  // ahead: the next block's loads are in flight while this block's products
  // run, and are stored to LDS after them.
  constexpr int PRE = (256 * RTM + NT - 1) / NT;
  double pre[PRE];
  double pre_tau = 0.0;
  auto fetch = [&](int kb) {
    const int rl = (kb + 1) / 16, rows = 16 * (rt - rl);
#pragma unroll
    for (int j = 0; j < PRE; ++j) {
      const int e = tid + j * NT;
      double v = 0.0;
      if (e < 16 * rows) {
        const int q = e / rows, i = 16 * rl + e % rows, k = kb + q;
        if (k < nref && i < n) v = (i == k + 1) ? 1.0 : (i > k + 1 ? W[colstart(k, n) + i - k] : 0.0);
      }
      pre[j] = v;
    }
    if (tid < 16) pre_tau = (kb + tid < nref) ? W[P + kb + tid] : 0.0;
  };
  auto store = [&](int kb) {
    const int rl = (kb + 1) / 16, rows = 16 * (rt - rl);
#pragma unroll
    for (int j = 0; j < PRE; ++j) {
      const int e = tid + j * NT;
      if (e < 16 * rows) Vs[16 * rl + e % rows][e / rows] = pre[j];
    }
    if (tid < 16) tau_s[tid] = pre_tau;
  };
  const int kfirst = ((nref - 1) / 16) * 16;
  if (nref > 0) {
    fetch(kfirst);
    store(kfirst);
  }
  __syncthreads();
  for (int k0 = kfirst; nref > 0 && k0 >= 0; k0 -= 16) {
    const int rlo = (k0 + 1) / 16;     // first row tile holding a nonzero of V
    // G = V^T V on matrix cores: each wave sums its share of the row tiles
    // (A = V^T and B = V take the same value per lane), then the partials
    // are added in wave order.
    {
      f64x4 g = {0.0, 0.0, 0.0, 0.0};
      for (int r = rlo + w; r < rt; r += NWV) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double x = Vs[16 * r + 4 * u + lk][li];
          g = mfma_f64(x, x, g);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) Gp[w][lk + 4 * v][li] = g[v];
    }
    __syncthreads();
    for (int e = tid; e < 256; e += NT) {
      double g = 0.0;
#pragma unroll
      for (int q = 0; q < NWV; ++q) g += Gp[q][e / 16][e % 16];
      Gs[e / 16][e % 16] = g;
    }
    __syncthreads();
    // T, one row per lane: T(j, i) needs only row j's earlier entries.
    if (tid < 16) {
      const int j = tid;
      double trow[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) trow[i] = 0.0;
      trow[j] = tau_s[j];
#pragma unroll
      for (int i = 1; i < 16; ++i) {
        if (i > j) {
          double acc = 0.0;
#pragma unroll
          for (int q = 0; q < 16; ++q)
            if (q >= j && q < i) acc = fma(trow[q], Gs[q][i], acc);
          trow[i] = -tau_s[i] * acc;
        }
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) Ts[j][i] = trow[i];
    }
    __syncthreads();
    if (k0 >= 16) fetch(k0 - 16);
    // Wt = V^T Z, Yt = T Wt, Z -= V Yt.  Four partial Wt (one per K slice
    // of a row tile) keep four products in flight.
    f64x4 Wp[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) Wp[u] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < RTM; ++r)
      if (r >= rlo && r < rt) {
#pragma unroll
        for (int u = 0; u < 4; ++u) Wp[u] = mfma_f64(Vs[16 * r + 4 * u + lk][li], Zt[r][u], Wp[u]);
      }
    const f64x4 Wt = (Wp[0] + Wp[1]) + (Wp[2] + Wp[3]);
    f64x4 Yt = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 4; ++u) Yt = mfma_f64(Ts[li][4 * u + lk], Wt[u], Yt);
#pragma unroll
    for (int r = 0; r < RTM; ++r)
      if (r >= rlo && r < rt) {
#pragma unroll
        for (int u = 0; u < 4; ++u) Zt[r] = mfma_f64(-Vs[16 * r + li][4 * u + lk], Yt[u], Zt[r]);
      }
    __syncthreads();
    if (k0 >= 16) {
      store(k0 - 16);
      __syncthreads();
    }
  }
  if (col >= 0) {
#pragma unroll
    for (int r = 0; r < RTM; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * r + lk + 4 * v;
        if (r < rt && row < n) Z[static_cast<int64_t>(col) * ldz + row] = Zt[r][v];
      }
  }
}


// ------------------------------------------- reduce, large orders (> 512)
// The same Householder reduction for buffers too large for one CU's
// registers: the full symmetric matrix (scaled by 2^-s) lives in the S1
// workspace (row-major, leading dimension mp) and every column takes two
// ordinary launches over blocks of LRB rows; the kernel boundaries are the
// only synchronisation.  Block b always owns rows [LRB b, LRB b + LRB), so
// the same rows stay on the same XCD (and in its L2) from column to column.
//  * k_ltr_reflect: every block forms the reflector of column k from row k
//    (the column by symmetry) in the same order, so all hold bitwise-equal
//    tau and v; the block owning row k+1 writes the packed reflector, tau,
//    d_k and e_k (the layout of the other reductions) and v; each block then
//    forms p_i = tau (A v)_i for its rows and its rows' share of p.v.
//  * k_ltr_update: c = (tau/2) p.v from the shares (added in block order),
//    w = p - c v, and A -= v w^T + w v^T on the block's rows of the trailing
//    block.
// Scratch: v, p and the shares in S2.
constexpr int LRB = 8;          // rows per block
constexpr int LNT = 256;        // threads per block

// Deterministic block sum (fixed order), returned to every thread.
__device__ __forceinline__ double ltr_block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < LNT / 64; ++q) t += red[q];
  return t;
}

__global__ __launch_bounds__(1024) void k_ltr_scale(const double* __restrict__ G, int n, int ldg,
                                                    double* __restrict__ W) {
  __shared__ double red[16];
  double amax = 0.0;
  for (int i = threadIdx.x >> 6; i < n; i += 16)
    for (int j = threadIdx.x & 63; j <= i; j += 64) amax = fmax(amax, fabs(G[static_cast<int64_t>(i) * ldg + j]));
  amax = wave_max(amax);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = amax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double g = 0.0;
    for (int q = 0; q < 16; ++q) g = fmax(g, red[q]);
    const int sexp = (g > 0.0 && g < INFINITY) ? ilogb(g) : 0;
    W[n * (n + 1) / 2 + 3 * n] = ldexp(1.0, sexp);
  }
}

// A (row-major, lda) = the symmetric matrix whose lower triangle is G's,
// times 2^-s; one block per row.
__global__ __launch_bounds__(LNT) void k_ltr_load(const double* __restrict__ G, int n, int ldg,
                                                  const double* __restrict__ W, double* __restrict__ A, int lda) {
  const int i = blockIdx.x;
  const double sc = 1.0 / W[n * (n + 1) / 2 + 3 * n];   // an exact power of two
  for (int j = threadIdx.x; j < n; j += LNT) {
    const double g = (j <= i) ? G[static_cast<int64_t>(i) * ldg + j] : G[static_cast<int64_t>(j) * ldg + i];
    A[static_cast<int64_t>(i) * lda + j] = g * sc;
  }
}

__global__ __launch_bounds__(LNT) void k_ltr_reflect(double* __restrict__ A, int lda, int n, int k,
                                                     double* __restrict__ W, double* __restrict__ S2) {
  __shared__ double vs[kTridGlobalMax];
  __shared__ double red[LNT / 64];
  __shared__ double prow[LRB][LNT / LRB];
  const int r0 = blockIdx.x * LRB;
  if (r0 + LRB <= k + 1) return;                 // every row of the block is finished
  const int tid = threadIdx.x, k1 = k + 1;
  const int P = n * (n + 1) / 2;
  const double* rk = A + static_cast<int64_t>(k) * lda;
  double s2 = 0.0;
  for (int j = k + 2 + tid; j < n; j += LNT) s2 = fma(rk[j], rk[j], s2);
  s2 = ltr_block_sum(s2, red);
  const double alpha = rk[k1];
  double tau = 0.0, beta = alpha, scale = 0.0;
  if (s2 > 0.0) {
    const double mu = sqrt(alpha * alpha + s2);
    beta = (alpha >= 0.0) ? -mu : mu;
    tau = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  for (int j = k1 + tid; j < n; j += LNT) vs[j] = (j == k1) ? 1.0 : rk[j] * scale;
  __syncthreads();
  double* vg = S2;                // v
  double* pg = S2 + lda;          // p
  double* sh = S2 + 2 * lda;      // shares of p.v, one per block
  if (blockIdx.x == k1 / LRB) {
    const int ck = colstart(k, n);
    for (int j = k1 + tid; j < n; j += LNT) {
      vg[j] = vs[j];
      if (j >= k + 2) W[ck + j - k] = vs[j];
    }
    if (tid == 0) {
      const double dk = rk[k];
      W[ck] = dk;
      W[ck + 1] = 1.0;
      W[P + k] = tau;
      W[P + n + k] = dk;
      W[P + 2 * n + k] = beta;
    }
  }
  // p_i for the block's rows: LNT/LRB threads per row, then a fixed-order
  // sum of their partials.
  const int r = tid / (LNT / LRB), q = tid % (LNT / LRB);
  const int i = r0 + r;
  double acc = 0.0;
  if (i > k && i < n) {
    const double* ai = A + static_cast<int64_t>(i) * lda;
    for (int j = k1 + q; j < n; j += LNT / LRB) acc = fma(ai[j], vs[j], acc);
  }
  prow[r][q] = acc;
  __syncthreads();
  if (tid < LRB) {
    const int ir = r0 + tid;
    double y = 0.0;
    for (int t = 0; t < LNT / LRB; ++t) y += prow[tid][t];
    const double p = (ir > k && ir < n) ? tau * y : 0.0;
    if (ir < n) pg[ir] = p;
    prow[tid][0] = (ir > k && ir < n) ? p * vs[ir] : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double d = 0.0;
    for (int t = 0; t < LRB; ++t) d += prow[t][0];
    sh[blockIdx.x] = d;
  }
}

__global__ __launch_bounds__(LNT) void k_ltr_update(double* __restrict__ A, int lda, int n, int k,
                                                    const double* __restrict__ W, const double* __restrict__ S2) {
  __shared__ double ws[kTridGlobalMax];
  __shared__ double vsh[kTridGlobalMax];
  const int r0 = blockIdx.x * LRB;
  if (r0 + LRB <= k + 1) return;
  const int tid = threadIdx.x, k1 = k + 1;
  const int P = n * (n + 1) / 2;
  const double tau = W[P + k];
  if (tau == 0.0) return;                        // H_k = I: nothing to update
  const double* vg = S2;
  const double* pg = S2 + lda;
  const double* sh = S2 + 2 * lda;
  double dot = 0.0;
  for (int b = k1 / LRB; b < static_cast<int>(gridDim.x); ++b) dot += sh[b];
  const double c = 0.5 * tau * dot;
  for (int j = k1 + tid; j < n; j += LNT) {
    const double v = vg[j];
    vsh[j] = v;
    ws[j] = fma(-c, v, pg[j]);
  }
  __syncthreads();
  for (int r = 0; r < LRB; ++r) {
    const int i = r0 + r;
    if (i <= k || i >= n) continue;
    const double vi = vsh[i], wi = ws[i];
    double* ai = A + static_cast<int64_t>(i) * lda;
    for (int j = k1 + tid; j < n; j += LNT) ai[j] = fma(-vi, ws[j], fma(-wi, vsh[j], ai[j]));
  }
}

__global__ void k_ltr_finish(const double* __restrict__ A, int lda, int n, double* __restrict__ W) {
  if (threadIdx.x != 0) return;
  const int P = n * (n + 1) / 2;
  const double d2 = A[static_cast<int64_t>(n - 2) * lda + n - 2];
  const double e2 = A[static_cast<int64_t>(n - 1) * lda + n - 2];
  const double d1 = A[static_cast<int64_t>(n - 1) * lda + n - 1];
  W[P + n + n - 2] = d2;
  W[P + 2 * n + n - 2] = e2;
  W[P + n - 2] = 0.0;
  W[colstart(n - 2, n)] = d2;
  W[colstart(n - 2, n) + 1] = e2;
  W[P + n + n - 1] = d1;
  W[P + n - 1] = 0.0;
  W[P + 2 * n + n - 1] = 0.0;
  W[colstart(n - 1, n)] = d1;
}

hipError_t launch_tridiag_large(const double* G, int m, int mp, EigWork wk, hipStream_t s) {
  if (m < 3 || m > kTridGlobalMax || mp < m) return hipErrorInvalidValue;
  const int nb = (m + LRB - 1) / LRB;
  if (2 * mp + nb > mp * mp) return hipErrorInvalidValue;   // S2 holds v, p and the shares
  hipLaunchKernelGGL(k_ltr_scale, dim3(1), dim3(1024), 0, s, G, m, mp, wk.W);
  hipLaunchKernelGGL(k_ltr_load, dim3(m), dim3(LNT), 0, s, G, m, mp, wk.W, wk.S1, mp);
  for (int k = 0; k + 2 < m; ++k) {
    hipLaunchKernelGGL(k_ltr_reflect, dim3(nb), dim3(LNT), 0, s, wk.S1, mp, m, k, wk.W, wk.S2);
    hipLaunchKernelGGL(k_ltr_update, dim3(nb), dim3(LNT), 0, s, wk.S1, mp, m, k, wk.W, wk.S2);
  }
  hipLaunchKernelGGL(k_ltr_finish, dim3(1), dim3(64), 0, s, wk.S1, mp, m, wk.W);
  return hipGetLastError();
}

hipError_t launch_tridiag(const double* G, int m, int mp, EigWork wk, hipStream_t s) {
  if (m < 1 || m > kTridGlobalMax || mp < m) return hipErrorInvalidValue;
  if (m <= 64)
    hipLaunchKernelGGL((k_tridiag_reg<2, 4>), dim3(1), dim3(RNT), 0, s, G, m, mp, wk.W, 0);
  else if (m <= 128)
    hipLaunchKernelGGL((k_tridiag_reg<4, 8>), dim3(1), dim3(RNT), 0, s, G, m, mp, wk.W, 0);
  else if (m <= 192)
    hipLaunchKernelGGL((k_tridiag_reg<6, 12>), dim3(1), dim3(RNT), 0, s, G, m, mp, wk.W, 0);
  else if (m <= kTridRegMax)
    hipLaunchKernelGGL((k_tridiag_reg<7, 13>), dim3(1), dim3(RNT), 0, s, G, m, mp, wk.W, 0);
  else {
    // The first m - kTridRegMax columns on the packed triangle in W, the
    // rest in registers (m <= kTridLargeMin = 256 = 64 * 4 rows here).
    if (m > kTridLargeMin) return launch_tridiag_large(G, m, mp, wk, s);
    static_assert(kTridLargeMin <= 64 * 4, "the head's instance holds 256 rows");
    const int h = m - kTridRegMax;
    hipLaunchKernelGGL(k_tridiag<4>, dim3(1), dim3(HNT), 0, s, G, m, mp, wk.W, h);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_tridiag_reg<7, 13>), dim3(1), dim3(RNT), 0, s, G, m, mp, wk.W, h);
  }
  return hipGetLastError();
}

hipError_t launch_dc(int m, int mp, double* lam, double* V, EigWork wk, hipStream_t s, int nvec) {
  if (m < 1 || m > kDcMax || mp < m) return hipErrorInvalidValue;
  if (m <= 512)
    hipLaunchKernelGGL(k_dc<512>, dim3(1), dim3(TNT), 0, s, wk.W, m, V, mp, wk.S1, wk.S2, lam, wk.st,
                       nvec < 1 ? m : nvec);
  else
    hipLaunchKernelGGL(k_dc<kDcMax>, dim3(1), dim3(TNT), 0, s, wk.W, m, V, mp, wk.S1, wk.S2, lam, wk.st,
                       nvec < 1 ? m : nvec);
  return hipGetLastError();
}

hipError_t launch_backtr(int m, int mp, double* V, EigWork wk, hipStream_t s) {
  if (m < 1 || m > kTridGlobalMax || mp < m) return hipErrorInvalidValue;
  const int grid = (m + BNT / 64 - 1) / (BNT / 64);
  if (m <= 64)
    hipLaunchKernelGGL((k_backtr<1, false>), dim3(grid), dim3(BNT), 0, s, wk.W, m, V, mp);
  else if (m <= 128)
    hipLaunchKernelGGL((k_backtr<2, false>), dim3(grid), dim3(BNT), 0, s, wk.W, m, V, mp);
  else if (m <= kTridMax)
    hipLaunchKernelGGL((k_backtr<4, false>), dim3(grid), dim3(BNT), 0, s, wk.W, m, V, mp);
  else if (m <= 256)
    hipLaunchKernelGGL((k_backtr<4, true>), dim3(grid), dim3(BNT), 0, s, wk.W, m, V, mp);
  else if (m <= 512)
    hipLaunchKernelGGL((k_backtr<8, true>), dim3(grid), dim3(BNT), 0, s, wk.W, m, V, mp);
  else
    hipLaunchKernelGGL((k_backtr<16, true>), dim3(grid), dim3(BNT), 0, s, wk.W, m, V, mp);
  return hipGetLastError();
}

hipError_t launch_eig_trid(const double* G, int m, int mp, double* lam, double* V, EigWork wk,
                           hipStream_t s) {
  hipError_t e = launch_tridiag(G, m, mp, wk, s);
  if (e == hipSuccess) e = launch_dc(m, mp, lam, V, wk, s, m);
  if (e == hipSuccess) e = launch_backtr(m, mp, V, wk, s);
  return e;
}

// ------------------------------------------------------ grouped (batches)
// One launch per stage over the tasks of a round.  The host groups sketches
// into classes of buffer rows (<= 64, <= 128, <= 208, <= 256) and launches
// each class on its own, so every launch below is instantiated for its
// class: the small classes do not carry the register footprint of the large
// ones.  Buffers above the register capacity continue the packed-triangle
// head.
template <int RP, int CP>
__global__ __launch_bounds__(RNT) void kg_tridiag_reg(const GroupSketch* __restrict__ SK,
                                                      const GroupRR* __restrict__ T) {
  const GroupSketch& s = SK[T[blockIdx.x].sk];
  const int h = max(0, s.m - kTridRegMax), n = s.m - h;
  // The host launches each class with the instance that holds its largest
  // block, so this never skips a task; it keeps the register indexing in range.
  if (n > 32 * RP || n > 16 * CP) return;
  tridiag_reg_body<RP, CP>(s.G, s.m, s.mp, s.W, h);
}

// The head of the reduction of buffers above the register capacity.
__global__ __launch_bounds__(HNT) void kg_tridiag(const GroupSketch* __restrict__ SK,
                                                  const GroupRR* __restrict__ T) {
  const GroupSketch& s = SK[T[blockIdx.x].sk];
  if (s.m <= kTridRegMax) return;        // the register variant's task
  tridiag_body<4>(s.G, s.m, s.mp, s.W, s.m - kTridRegMax);
}

// Divide and conquer per size class: LDS state for NMAX rows and NT = 4 NMAX
// threads (one four-lane group per root of the widest merge), so the small
// classes neither hold the large class's LDS nor wait on its barriers.
template <int NMAX, int NT>
__global__ __launch_bounds__(NT) void kg_dc(const GroupSketch* __restrict__ SK,
                                            const GroupRR* __restrict__ T) {
  const GroupSketch& s = SK[T[blockIdx.x].sk];
  if (s.m > NMAX) return;     // the host picks NMAX >= every task's order
  dc_body<NMAX, NT>(s.W, s.m, s.V, s.mp, s.S1, s.S2, s.lam, s.st, min(s.m, s.l));
}

// Size class [LO, HI] of buffer rows, with the LDS staging sized for it;
// tasks of other classes return at once.  Classes that stage the reflectors
// in LDS run 16 waves per block (NT = 1024), so one staging serves 16
// columns and a CU holds enough waves to hide each column's chain.
template <int NPL, bool GA, int LO, int HI, int NT>
__global__ __launch_bounds__(NT) void kg_backtr(const GroupSketch* __restrict__ SK,
                                                const GroupRR* __restrict__ T) {
  const GroupSketch& s = SK[T[blockIdx.y].sk];
  if (s.m < LO || s.m > HI) return;
  if (static_cast<int>(blockIdx.x) * (NT / 64) >= s.m) return;
  backtr_body<NPL, GA, NT>(s.W, s.m, s.V, s.mp, blockIdx.x);
}

// The blocked back-transformation per size class [LO, HI]: RTM row tiles,
// NWV waves (16 wanted columns each) per workgroup.
template <int RTM, int NWV, int LO, int HI>
__global__ __launch_bounds__(64 * NWV) void kg_backtr_wy(const GroupSketch* __restrict__ SK,
                                                         const GroupRR* __restrict__ T) {
  const GroupSketch& s = SK[T[blockIdx.y].sk];
  if (s.m < LO || s.m > HI) return;
  if (static_cast<int>(blockIdx.x) * 16 * NWV >= min(s.m, s.l)) return;
  backtr_wy_body<RTM, NWV>(s.W, s.m, s.V, s.mp, blockIdx.x);
}

template <int RTM, int NWV, int LO, int HI>
hipError_t launch_group_backtr_wy(const GroupSketch* sk, const GroupRR* t, int nt, int max_m, int max_c,
                                  hipStream_t s) {
  if (max_m < LO) return hipSuccess;
  const dim3 g((max_c + 16 * NWV - 1) / (16 * NWV), nt);
  hipLaunchKernelGGL((kg_backtr_wy<RTM, NWV, LO, HI>), g, dim3(64 * NWV), 0, s, sk, t);
  return hipGetLastError();
}

template <int NPL, bool GA, int LO, int HI>
hipError_t launch_group_backtr(const GroupSketch* sk, const GroupRR* t, int nt, int max_m, hipStream_t s) {
  constexpr int NT = GA ? BNT : 1024;
  if (max_m < LO) return hipSuccess;
  const int top = min(max_m, HI);
  const dim3 g((top + NT / 64 - 1) / (NT / 64), nt);
  hipLaunchKernelGGL((kg_backtr<NPL, GA, LO, HI, NT>), g, dim3(NT), 0, s, sk, t);
  return hipGetLastError();
}

hipError_t launch_group_tridiag_head(const GroupSketch* sk, const GroupRR* t, int nt, int max_m,
                                     hipStream_t s) {
  if (nt <= 0 || max_m <= kTridRegMax) return hipSuccess;
  if (max_m > kBatchMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kg_tridiag, dim3(nt), dim3(HNT), 0, s, sk, t);
  return hipGetLastError();
}

hipError_t launch_group_tridiag(const GroupSketch* sk, const GroupRR* t, int nt, int max_m, hipStream_t s) {
  if (nt <= 0) return hipSuccess;
  if (max_m > kBatchMax) return hipErrorInvalidValue;
  if (max_m <= 64)
    hipLaunchKernelGGL((kg_tridiag_reg<2, 4>), dim3(nt), dim3(RNT), 0, s, sk, t);
  else if (max_m <= 128)
    hipLaunchKernelGGL((kg_tridiag_reg<4, 8>), dim3(nt), dim3(RNT), 0, s, sk, t);
  else
    hipLaunchKernelGGL((kg_tridiag_reg<7, 13>), dim3(nt), dim3(RNT), 0, s, sk, t);
  return hipGetLastError();
}

hipError_t launch_group_dc(const GroupSketch* sk, const GroupRR* t, int nt, int max_m, hipStream_t s) {
  if (nt <= 0) return hipSuccess;
  if (max_m > kBatchMax) return hipErrorInvalidValue;
  if (max_m <= 64)
    hipLaunchKernelGGL((kg_dc<64, 256>), dim3(nt), dim3(256), 0, s, sk, t);
  else if (max_m <= 128)
    hipLaunchKernelGGL((kg_dc<128, 512>), dim3(nt), dim3(512), 0, s, sk, t);
  else
    hipLaunchKernelGGL((kg_dc<kBatchMax, TNT>), dim3(nt), dim3(TNT), 0, s, sk, t);
  return hipGetLastError();
}

hipError_t launch_group_backtr(const GroupSketch* sk, const GroupRR* t, int nt, int max_m, int max_c,
                               hipStream_t s) {
  if (nt <= 0) return hipSuccess;
  if (max_m > kBatchMax) return hipErrorInvalidValue;
  hipError_t e = launch_group_backtr<1, false, 1, 64>(sk, t, nt, max_m, s);
  if (e == hipSuccess) e = launch_group_backtr_wy<8, 4, 65, 128>(sk, t, nt, max_m, max_c, s);
  if (e == hipSuccess) e = launch_group_backtr_wy<13, 4, 129, 208>(sk, t, nt, max_m, max_c, s);
  if (e == hipSuccess) e = launch_group_backtr_wy<16, 4, 209, kBatchMax>(sk, t, nt, max_m, max_c, s);
  return e;
}

}  // namespace fdsk
