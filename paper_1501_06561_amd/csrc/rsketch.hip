// Hashing, OSNAP, Priority and VarOpt streaming sketches (Sections 2.2 and
// 3.2 of the paper), the hashing and sampling competitors of the Frequent
// Directions family: kernels, host state and the rsketch_* C ABI (see
// include/fdsketch.h for the exact definitions).
//
// All four read every row once from HBM; their work per row is O(d).
//  * Hashing / OSNAP: one kernel per append call.  A block takes a few rows;
//    its threads stride over the columns, read each row once (coalesced)
//    and add sign * row / sqrt(s) into the row's bucket of every instance
//    with FP64 atomics (B stays in L2).  The same block adds the rows'
//    squared norms into ||A||_F^2.
//  * Priority / VarOpt: per append call, (1) a row-norm kernel over the
//    call's rows (the HBM pass) writes each candidate's weight and, for
//    Priority, its priority w/u; (2) when the reservoir plus the call's
//    rows exceed l, one block decides which candidates stay (Priority: an
//    MSB-first radix select of the l-th largest priority on its IEEE bits;
//    VarOpt: the threshold of the candidates by fixed-point iteration, then
//    systematic sampling below it), writing the kept candidates' positions
//    in candidate order; (3) a gather kernel builds the new reservoir.
// Random numbers come from the counter-based SplitMix64 construction stated
// in the header (Steele, Lea and Flood, 2014), evaluated per row index.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fdsk_device.hpp"
#include "fdsketch.h"

namespace {

using fdsk::load_as_f64;

// ------------------------------------------------------------ generator
__device__ __forceinline__ uint64_t sm_mix(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t sm_bits(uint64_t key, uint64_t i, uint64_t j) {
  return sm_mix(sm_mix(key ^ i) ^ j);
}
__device__ __forceinline__ double sm_uniform(uint64_t key, uint64_t i) {
  return (static_cast<double>(sm_bits(key, i, 0) >> 11) + 0.5) * 0x1p-53;
}

// ------------------------------------------------------------ hashing
constexpr int HROWS = 4;    // rows per block
constexpr int HNT = 256;

__global__ __launch_bounds__(HNT) void k_hash_rows(const void* __restrict__ X, int dt, int64_t ldx, int n,
                                                   int d, int64_t row0, uint64_t key, int inst, int rows,
                                                   double scale, double* __restrict__ B,
                                                   double* __restrict__ fro2) {
  __shared__ int bk[HROWS][8];
  __shared__ double sg[HROWS][8];
  __shared__ double red[HNT / 64];
  const int r0 = blockIdx.x * HROWS;
  const int tid = threadIdx.x;
  if (tid < HROWS * inst) {
    const int r = tid / inst, j = tid % inst;
    const uint64_t i = static_cast<uint64_t>(row0 + r0 + r);
    bk[r][j] = j * rows + static_cast<int>(((sm_bits(key, i, 2ull * j) >> 32) * static_cast<uint64_t>(rows)) >> 32);
    sg[r][j] = (sm_bits(key, i, 2ull * j + 1) >> 63) ? -scale : scale;
  }
  __syncthreads();
  double nrm = 0.0;
  for (int r = 0; r < HROWS; ++r) {
    const int rr = r0 + r;
    if (rr >= n) break;
    const int64_t base = static_cast<int64_t>(rr) * ldx;
    for (int c = tid; c < d; c += HNT) {
      const double x = load_as_f64(X, base + c, dt);
      nrm = fma(x, x, nrm);
      for (int j = 0; j < inst; ++j)
        unsafeAtomicAdd(B + static_cast<int64_t>(bk[r][j]) * d + c, sg[r][j] * x);
    }
  }
  nrm = fdsk::wave_sum(nrm);
  if ((tid & 63) == 0) red[tid >> 6] = nrm;
  __syncthreads();
  if (tid == 0) unsafeAtomicAdd(fro2, red[0] + red[1] + red[2] + red[3]);
}

// ------------------------------------------------------------ sampling
// Candidate arrays: w (squared norm), key (Priority: priority; VarOpt:
// adjusted weight), idx (stream index).  Reservoir candidates first.
__global__ __launch_bounds__(HNT) void k_norms(const void* __restrict__ X, int dt, int64_t ldx, int n, int d,
                                               int64_t row0, uint64_t key, int priority, int cand0,
                                               double* __restrict__ cw, double* __restrict__ ckey,
                                               long long* __restrict__ cidx, double* __restrict__ fro2) {
  __shared__ double red[HNT / 64];
  const int r = blockIdx.x;
  const int64_t base = static_cast<int64_t>(r) * ldx;
  double s = 0.0;
  for (int c = threadIdx.x; c < d; c += HNT) {
    const double x = load_as_f64(X, base + c, dt);
    s = fma(x, x, s);
  }
  s = fdsk::wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double w = (red[0] + red[1]) + (red[2] + red[3]);
    const long long i = row0 + r;
    cw[cand0 + r] = w;
    ckey[cand0 + r] = priority ? w / sm_uniform(key, static_cast<uint64_t>(i)) : w;
    cidx[cand0 + r] = i;
    unsafeAtomicAdd(fro2, w);
  }
}

constexpr int SNT = 1024;   // the selection block

// Exclusive block scan of one int per thread; returns the total.
__device__ int block_scan_excl(int v, int* sh, int& excl) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < SNT; off <<= 1) {
    const int t = (tid >= off) ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += t;
    __syncthreads();
  }
  const int incl = sh[tid];
  const int total = sh[SNT - 1];
  __syncthreads();
  excl = incl - v;
  return total;
}

// Same for doubles (fixed order: a Hillis-Steele scan).
__device__ double block_scan_excl_f64(double v, double* sh, double& excl) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < SNT; off <<= 1) {
    const double t = (tid >= off) ? sh[tid - off] : 0.0;
    __syncthreads();
    sh[tid] += t;
    __syncthreads();
  }
  const double incl = sh[tid];
  const double total = sh[SNT - 1];
  __syncthreads();
  excl = incl - v;
  return total;
}

__device__ double block_sum_f64(double v, double* sh) {
  double e;
  return block_scan_excl_f64(v, sh, e);
}

// Priority: keep the l candidates of largest priority (ties: earlier
// candidates first), in candidate order; tau = max(tau, largest dropped).
__global__ __launch_bounds__(SNT) void k_select_priority(const double* __restrict__ ckey, int N, int l,
                                                         int* __restrict__ keep, double* __restrict__ tau) {
  __shared__ int hist[256];
  __shared__ int shi[SNT];
  __shared__ double shd[SNT];
  __shared__ unsigned long long s_prefix;
  __shared__ int s_rank, s_greater;
  const int tid = threadIdx.x;
  const int seg = (N + SNT - 1) / SNT, lo = min(N, tid * seg), hi = min(N, lo + seg);
  if (tid == 0) {
    s_prefix = 0;
    s_rank = l;        // 1-based rank of the wanted key among those matching the prefix
    s_greater = 0;
  }
  // MSB-first radix select, 8 bits per pass.
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 56 - 8 * pass;
    for (int b = tid; b < 256; b += SNT) hist[b] = 0;
    __syncthreads();
    const unsigned long long pre = s_prefix;
    for (int c = lo; c < hi; ++c) {
      const unsigned long long k = static_cast<unsigned long long>(__double_as_longlong(ckey[c]));
      if (pass == 0 || (k >> (shift + 8)) == pre) atomicAdd(&hist[(k >> shift) & 255], 1);
    }
    __syncthreads();
    if (tid == 0) {
      int rank = s_rank, acc = 0, dgt = 255;
      for (; dgt >= 0; --dgt) {
        if (acc + hist[dgt] >= rank) break;
        acc += hist[dgt];
      }
      s_greater += acc;
      s_rank = rank - acc;
      s_prefix = (pre << 8) | static_cast<unsigned long long>(dgt);
    }
    __syncthreads();
  }
  const unsigned long long T = s_prefix;
  const int ties_kept = l - s_greater;    // >= 1 keys equal to T are kept, in candidate order
  // Stable compaction: flags per candidate.
  int mine_eq = 0;
  for (int c = lo; c < hi; ++c) {
    const unsigned long long k = static_cast<unsigned long long>(__double_as_longlong(ckey[c]));
    mine_eq += (k == T);
  }
  int eq_before;
  block_scan_excl(mine_eq, shi, eq_before);
  int kept_local = 0;
  {
    int e = eq_before;
    for (int c = lo; c < hi; ++c) {
      const unsigned long long k = static_cast<unsigned long long>(__double_as_longlong(ckey[c]));
      kept_local += (k > T) || (k == T && e < ties_kept);
      e += (k == T);
    }
  }
  int out;
  block_scan_excl(kept_local, shi, out);
  double dropmax = 0.0;
  {
    int e = eq_before;
    for (int c = lo; c < hi; ++c) {
      const double kv = ckey[c];
      const unsigned long long k = static_cast<unsigned long long>(__double_as_longlong(kv));
      const bool kp = (k > T) || (k == T && e < ties_kept);
      e += (k == T);
      if (kp) keep[out++] = c;
      else dropmax = fmax(dropmax, kv);
    }
  }
  shd[tid] = dropmax;
  __syncthreads();
  if (tid == 0) {
    double m = *tau;
    for (int t = 0; t < SNT; ++t) m = fmax(m, shd[t]);
    *tau = m;
  }
}

// VarOpt: the candidates' threshold tau (sum min(1, key/tau) = l) by the
// fixed-point iteration tau <- (sum of keys below tau) / (l - count of keys
// at or above tau) from tau = total / l (tau does not increase and the set
// above it only grows; it stops when the count repeats; the small keys are
// summed directly, not as total minus the large ones, which would cancel); candidates at or above tau stay; below it, l - t are chosen by
// systematic sampling with offset u over p = key / tau in candidate order:
// positions (q + u) C/(l - t), q = 0 .. l-t-1, C = sum p, each picks the
// candidate whose interval (C_{j-1}, C_j] of the running sum holds it.
// Chosen candidates' keys become tau.
__global__ __launch_bounds__(SNT) void k_select_varopt(double* __restrict__ ckey, int N, int l, double u,
                                                       int* __restrict__ keep, double* __restrict__ tau_out) {
  __shared__ int shi[SNT];
  __shared__ double shd[SNT];
  const int tid = threadIdx.x;
  const int seg = (N + SNT - 1) / SNT, lo = min(N, tid * seg), hi = min(N, lo + seg);
  double part = 0.0;
  for (int c = lo; c < hi; ++c) part += ckey[c];
  const double total = block_sum_f64(part, shd);
  double tau = total / l;
  int t_prev = -1;
  for (int it = 0; it <= l; ++it) {
    double small = 0.0;
    int cnt = 0;
    for (int c = lo; c < hi; ++c) {
      const double k = ckey[c];
      if (k >= tau) ++cnt;
      else small += k;
    }
    const double S = block_sum_f64(small, shd);
    int e;
    const int t = block_scan_excl(cnt, shi, e);
    if (t == t_prev || t >= l) break;
    t_prev = t;
    tau = S / (l - t);
  }
  // Systematic sampling below tau.
  int t_local = 0;
  double p_local = 0.0;
  for (int c = lo; c < hi; ++c) {
    const double k = ckey[c];
    if (k >= tau) ++t_local;
    else p_local += k / tau;
  }
  int e;
  const int t = block_scan_excl(t_local, shi, e);
  double C0;
  const double Ctot = block_scan_excl_f64(p_local, shd, C0);
  const int kq = l - t;
  const double spacing = Ctot / kq;
  int kept_local = 0;
  {
    double C = C0;
    for (int c = lo; c < hi; ++c) {
      const double k = ckey[c];
      if (k >= tau) {
        ++kept_local;
        continue;
      }
      const double Cprev = C;
      C += k / tau;
      // The one q (if any) whose position lies in (Cprev, C].
      const double q0 = floor(Cprev / spacing - u);
      for (int dq = 0; dq < 3; ++dq) {
        const double q = q0 + dq;
        if (q < 0.0 || q >= kq) continue;
        const double pos = (q + u) * spacing;
        if (pos > Cprev && pos <= C) {
          ++kept_local;
          break;
        }
      }
    }
  }
  int out;
  block_scan_excl(kept_local, shi, out);
  {
    double C = C0;
    for (int c = lo; c < hi; ++c) {
      const double k = ckey[c];
      if (k >= tau) {
        keep[out++] = c;
        continue;
      }
      const double Cprev = C;
      C += k / tau;
      const double q0 = floor(Cprev / spacing - u);
      for (int dq = 0; dq < 3; ++dq) {
        const double q = q0 + dq;
        if (q < 0.0 || q >= kq) continue;
        const double pos = (q + u) * spacing;
        if (pos > Cprev && pos <= C) {
          keep[out++] = c;
          ckey[c] = tau;
          break;
        }
      }
    }
  }
  if (tid == 0) *tau_out = tau;
}

// New reservoir: kept candidate q is old reservoir row c (c < nres) or row
// c - nres of the call's rows.  A position outside [0, N) (a selection that
// came up short, which exact arithmetic rules out) gives a zero row.
__global__ __launch_bounds__(HNT) void k_gather(const int* __restrict__ keep, int nres, int N,
                                                const double* __restrict__ Rold,
                                                const void* __restrict__ X, int dt, int64_t ldx, int d,
                                                double* __restrict__ Rnew, const double* __restrict__ cw,
                                                const double* __restrict__ ckey, const long long* __restrict__ cidx,
                                                double* __restrict__ nw, double* __restrict__ nkey,
                                                long long* __restrict__ nidx) {
  const int q = blockIdx.x;
  const int c = keep[q];
  double* dst = Rnew + static_cast<int64_t>(q) * d;
  if (c < 0 || c >= N) {
    for (int j = threadIdx.x; j < d; j += HNT) dst[j] = 0.0;
    if (threadIdx.x == 0) {
      nw[q] = 0.0;
      nkey[q] = 0.0;
      nidx[q] = -1;
    }
    return;
  }
  if (c < nres) {
    const double* src = Rold + static_cast<int64_t>(c) * d;
    for (int j = threadIdx.x; j < d; j += HNT) dst[j] = src[j];
  } else {
    const int64_t base = static_cast<int64_t>(c - nres) * ldx;
    for (int j = threadIdx.x; j < d; j += HNT) dst[j] = load_as_f64(X, base + j, dt);
  }
  if (threadIdx.x == 0) {
    nw[q] = cw[c];
    nkey[q] = ckey[c];
    nidx[q] = cidx[c];
  }
}

__global__ void k_fill_keep(int* __restrict__ keep, int l) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < l) keep[i] = -1;
}

// Every call's rows are kept (the reservoir is not full): append them.
__global__ __launch_bounds__(HNT) void k_append_rows(const void* __restrict__ X, int dt, int64_t ldx, int d,
                                                     double* __restrict__ R, int r0) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * ldx;
  double* dst = R + static_cast<int64_t>(r0 + blockIdx.x) * d;
  for (int j = threadIdx.x; j < d; j += HNT) dst[j] = load_as_f64(X, base + j, dt);
}

// Output: row q = reservoir row q * sqrt(w^ / w) (mode 1 Priority:
// w^ = max(w, tau); mode 0 VarOpt: the adjusted weight; mode 2 hashing:
// the row as it is), rows >= cnt zero.
__global__ __launch_bounds__(HNT) void k_rs_out(const double* __restrict__ R, int cnt, int l, int d,
                                                const double* __restrict__ w, const double* __restrict__ key,
                                                const double* __restrict__ tau, int mode,
                                                void* __restrict__ out, int64_t ldo, int odt) {
  const int q = blockIdx.x;
  double f = 0.0;
  if (q < cnt) {
    if (mode == 2) {
      f = 1.0;
    } else {
      const double wq = w[q];
      const double wh = mode == 1 ? fmax(wq, *tau) : key[q];
      f = wq > 0.0 ? sqrt(wh / wq) : 0.0;
    }
  }
  for (int j = threadIdx.x; j < d; j += HNT) {
    const double v = (q < cnt) ? R[static_cast<int64_t>(q) * d + j] * f : 0.0;
    if (odt == 0) static_cast<double*>(out)[static_cast<int64_t>(q) * ldo + j] = v;
    else static_cast<float*>(out)[static_cast<int64_t>(q) * ldo + j] = static_cast<float>(v);
  }
}

__global__ void k_rs_weights(const double* __restrict__ w, const double* __restrict__ key, const double* __restrict__ tau,
                             int cnt, int priority, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int q = 0; q < cnt; ++q) s += priority ? fmax(w[q], *tau) : key[q];
  *out = s;
}

}  // namespace

struct fdsk_rsketch {
  int kind = 0, d = 0, l = 0, inst = 1, rows = 0;
  uint64_t key = 0;
  hipStream_t stream = nullptr;
  double* B = nullptr;          // hashing: l x d
  double* acc = nullptr;        // [0] ||A||_F^2, [1] tau, [2] weight sum
  // sampling: double-buffered reservoir and its scalars
  double* R[2] = {nullptr, nullptr};
  double* w[2] = {nullptr, nullptr};
  double* kv[2] = {nullptr, nullptr};
  long long* ix[2] = {nullptr, nullptr};
  int cur = 0, cnt = 0;
  // candidates of one call
  double* cw = nullptr;
  double* ckey = nullptr;
  long long* cidx = nullptr;
  int* keep = nullptr;
  size_t cand_cap = 0;
  void* stage = nullptr;
  size_t stage_bytes = 0;
  int64_t n_rows = 0;
  int64_t chunks = 0;
  bool finalized = false;
  int err = 0;
  std::string msg;
};

namespace {

thread_local std::string g_rs_err;

int rs_err(fdsk_rsketch* s, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (s) {
    s->err = code;
    s->msg = buf;
  } else {
    g_rs_err = buf;
  }
  return code;
}

size_t dt_size(int dt) { return dt == FDSK_F64 ? 8 : dt == FDSK_F32 ? 4 : dt == FDSK_BF16 ? 2 : 0; }

void free_all(fdsk_rsketch* s) {
  void* ptrs[] = {s->B, s->acc, s->R[0], s->R[1], s->w[0], s->w[1], s->kv[0], s->kv[1], s->ix[0], s->ix[1],
                  s->cw, s->ckey, s->cidx, s->keep, s->stage};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

// Candidate arrays for the reservoir plus n rows.
int ensure_candidates(fdsk_rsketch* s, size_t n) {
  const size_t need = static_cast<size_t>(s->l) + n;
  if (need <= s->cand_cap) return 0;
  (void)hipStreamSynchronize(s->stream);
  if (s->cw) (void)hipFree(s->cw);
  if (s->ckey) (void)hipFree(s->ckey);
  if (s->cidx) (void)hipFree(s->cidx);
  s->cw = s->ckey = nullptr;
  s->cidx = nullptr;
  s->cand_cap = 0;
  if (hipMalloc(&s->cw, need * 8) != hipSuccess || hipMalloc(&s->ckey, need * 8) != hipSuccess ||
      hipMalloc(&s->cidx, need * 8) != hipSuccess)
    return rs_err(s, FDSK_ENOMEM, "candidate arrays for %zu rows", need);
  s->cand_cap = need;
  return 0;
}

#define RSCHK(s, expr)                                                                     \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return rs_err((s), FDSK_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

double host_uniform(uint64_t key, uint64_t i) {
  auto mix = [](uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  return (static_cast<double>(mix(mix(key ^ i) ^ 0ull) >> 11) + 0.5) * 0x1p-53;
}

int append_device(fdsk_rsketch* s, const void* X, int64_t n, int64_t ldx, int dt) {
  const int d = s->d;
  if (s->kind == FDSK_RS_HASH || s->kind == FDSK_RS_OSNAP) {
    const int blocks = static_cast<int>((n + HROWS - 1) / HROWS);
    hipLaunchKernelGGL(k_hash_rows, dim3(blocks), dim3(HNT), 0, s->stream, X, dt, ldx, static_cast<int>(n), d,
                       s->n_rows, s->key, s->inst, s->rows, 1.0 / std::sqrt(static_cast<double>(s->inst)), s->B,
                       s->acc);
    RSCHK(s, hipGetLastError());
  } else {
    const bool pri = s->kind == FDSK_RS_PRIORITY;
    int rc = ensure_candidates(s, static_cast<size_t>(n));
    if (rc) return rc;
    const int nres = s->cnt, N = nres + static_cast<int>(n);
    // Reservoir candidates first (their weights, keys and indices), then the
    // call's rows.
    if (nres > 0) {
      RSCHK(s, hipMemcpyAsync(s->cw, s->w[s->cur], nres * 8, hipMemcpyDeviceToDevice, s->stream));
      RSCHK(s, hipMemcpyAsync(s->ckey, s->kv[s->cur], nres * 8, hipMemcpyDeviceToDevice, s->stream));
      RSCHK(s, hipMemcpyAsync(s->cidx, s->ix[s->cur], nres * 8, hipMemcpyDeviceToDevice, s->stream));
    }
    hipLaunchKernelGGL(k_norms, dim3(static_cast<unsigned>(n)), dim3(HNT), 0, s->stream, X, dt, ldx,
                       static_cast<int>(n), d, s->n_rows, s->key, pri ? 1 : 0, nres, s->cw, s->ckey, s->cidx,
                       s->acc);
    RSCHK(s, hipGetLastError());
    if (N <= s->l) {
      // Everything fits: the rows go after the reservoir's.
      hipLaunchKernelGGL(k_append_rows, dim3(static_cast<unsigned>(n)), dim3(HNT), 0, s->stream, X, dt, ldx, d,
                         s->R[s->cur], nres);
      RSCHK(s, hipGetLastError());
      RSCHK(s, hipMemcpyAsync(s->w[s->cur] + nres, s->cw + nres, n * 8, hipMemcpyDeviceToDevice, s->stream));
      RSCHK(s, hipMemcpyAsync(s->kv[s->cur] + nres, s->ckey + nres, n * 8, hipMemcpyDeviceToDevice, s->stream));
      RSCHK(s, hipMemcpyAsync(s->ix[s->cur] + nres, s->cidx + nres, n * 8, hipMemcpyDeviceToDevice, s->stream));
      s->cnt = N;
    } else {
      hipLaunchKernelGGL(k_fill_keep, dim3((s->l + 255) / 256), dim3(256), 0, s->stream, s->keep, s->l);
      if (pri) {
        hipLaunchKernelGGL(k_select_priority, dim3(1), dim3(SNT), 0, s->stream, s->ckey, N, s->l, s->keep,
                           s->acc + 1);
      } else {
        const double u = host_uniform(s->key, (1ull << 62) + static_cast<uint64_t>(s->chunks));
        hipLaunchKernelGGL(k_select_varopt, dim3(1), dim3(SNT), 0, s->stream, s->ckey, N, s->l, u, s->keep,
                           s->acc + 1);
      }
      RSCHK(s, hipGetLastError());
      const int nx = 1 - s->cur;
      hipLaunchKernelGGL(k_gather, dim3(s->l), dim3(HNT), 0, s->stream, s->keep, nres, N, s->R[s->cur], X, dt, ldx,
                         d, s->R[nx], s->cw, s->ckey, s->cidx, s->w[nx], s->kv[nx], s->ix[nx]);
      RSCHK(s, hipGetLastError());
      s->cur = nx;
      s->cnt = s->l;
    }
  }
  s->n_rows += n;
  s->chunks += 1;
  return 0;
}

}  // namespace

extern "C" {

const char* rsketch_last_error(const fdsk_rsketch* s) { return s ? s->msg.c_str() : g_rs_err.c_str(); }

int rsketch_create(int32_t kind, int64_t d, int32_t l, int32_t s_inst, uint64_t key, void* hip_stream,
                   fdsk_rsketch** out) {
  if (!out) return rs_err(nullptr, FDSK_EINVAL, "null output");
  *out = nullptr;
  if (kind < FDSK_RS_HASH || kind > FDSK_RS_VAROPT) return rs_err(nullptr, FDSK_EINVAL, "unknown kind %d", kind);
  if (d < 1 || d > 65536 || l < 1) return rs_err(nullptr, FDSK_EINVAL, "bad sizes");
  const int inst = kind == FDSK_RS_OSNAP ? s_inst : 1;
  if (kind == FDSK_RS_OSNAP && (s_inst < 1 || s_inst > 8 || l % s_inst != 0))
    return rs_err(nullptr, FDSK_EINVAL, "OSNAP needs 1 <= s <= 8 dividing l");
  if (l > (1 << 24)) return rs_err(nullptr, FDSK_EUNSUPPORTED, "l above 2^24");
  fdsk_rsketch* s = new fdsk_rsketch;
  s->kind = kind;
  s->d = static_cast<int>(d);
  s->l = l;
  s->inst = inst;
  s->rows = l / inst;
  s->key = key;
  s->stream = static_cast<hipStream_t>(hip_stream);
  const size_t ld = static_cast<size_t>(l) * d;
  hipError_t e = hipMalloc(&s->acc, 3 * 8);
  if (e == hipSuccess) {
    if (kind == FDSK_RS_HASH || kind == FDSK_RS_OSNAP) {
      e = hipMalloc(&s->B, ld * 8);
      if (e == hipSuccess) e = hipMemsetAsync(s->B, 0, ld * 8, s->stream);
    } else {
      for (int b = 0; b < 2 && e == hipSuccess; ++b) {
        e = hipMalloc(&s->R[b], ld * 8);
        if (e == hipSuccess) e = hipMalloc(&s->w[b], static_cast<size_t>(l) * 8);
        if (e == hipSuccess) e = hipMalloc(&s->kv[b], static_cast<size_t>(l) * 8);
        if (e == hipSuccess) e = hipMalloc(&s->ix[b], static_cast<size_t>(l) * 8);
      }
      if (e == hipSuccess) e = hipMalloc(&s->keep, static_cast<size_t>(l) * 4);
    }
  }
  if (e == hipSuccess) e = hipMemsetAsync(s->acc, 0, 3 * 8, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) {
    free_all(s);
    delete s;
    return rs_err(nullptr, FDSK_ENOMEM, "rsketch workspace: %s", hipGetErrorString(e));
  }
  *out = s;
  return 0;
}

int rsketch_append(fdsk_rsketch* s, const void* rows, int64_t n, int64_t stride, fdsk_dtype dtype, fdsk_mem mem) {
  if (!s) return rs_err(nullptr, FDSK_EINVAL, "null sketch");
  if (s->err) return s->err;
  if (s->finalized) return rs_err(s, FDSK_ESTATE, "append after finalize");
  if (n < 0) return rs_err(s, FDSK_EINVAL, "n < 0");
  if (n == 0) return 0;
  if (!rows) return rs_err(s, FDSK_EINVAL, "null rows");
  const size_t es = dt_size(dtype);
  if (es == 0) return rs_err(s, FDSK_EINVAL, "bad dtype");
  if (stride < s->d) return rs_err(s, FDSK_EINVAL, "stride < d");
  if (n > (1 << 30)) return rs_err(s, FDSK_EUNSUPPORTED, "more than 2^30 rows in one call");
  if (mem == FDSK_MEM_DEVICE) return append_device(s, rows, n, stride, dtype);
  if (mem != FDSK_MEM_HOST) return rs_err(s, FDSK_EINVAL, "bad mem kind");
  const size_t bytes = static_cast<size_t>(n) * s->d * es;
  if (s->stage_bytes < bytes) {
    RSCHK(s, hipStreamSynchronize(s->stream));
    if (s->stage) (void)hipFree(s->stage);
    s->stage = nullptr;
    s->stage_bytes = 0;
    if (hipMalloc(&s->stage, bytes) != hipSuccess) return rs_err(s, FDSK_ENOMEM, "staging host rows");
    s->stage_bytes = bytes;
  }
  RSCHK(s, hipMemcpy2DAsync(s->stage, s->d * es, rows, stride * es, s->d * es, n, hipMemcpyHostToDevice,
                            s->stream));
  int rc = append_device(s, s->stage, n, s->d, dtype);
  if (rc) return rc;
  RSCHK(s, hipStreamSynchronize(s->stream));
  return 0;
}

int rsketch_finalize(fdsk_rsketch* s, void* B_out, int64_t ldb, fdsk_dtype out_dtype, fdsk_mem mem,
                     int64_t* index_out, int32_t* rows_out) {
  if (!s) return rs_err(nullptr, FDSK_EINVAL, "null sketch");
  if (s->err) return s->err;
  if (s->finalized) return rs_err(s, FDSK_ESTATE, "finalize called twice");
  if (!B_out || ldb < s->d) return rs_err(s, FDSK_EINVAL, "bad output");
  if (out_dtype != FDSK_F64 && out_dtype != FDSK_F32) return rs_err(s, FDSK_EINVAL, "output dtype must be F64 or F32");
  if (mem != FDSK_MEM_DEVICE && mem != FDSK_MEM_HOST) return rs_err(s, FDSK_EINVAL, "bad mem kind");
  const size_t es = dt_size(out_dtype);
  const bool hashing = s->kind == FDSK_RS_HASH || s->kind == FDSK_RS_OSNAP;
  void* dst = B_out;
  void* tmp = nullptr;
  int64_t ld = ldb;
  if (mem == FDSK_MEM_HOST) {
    if (hipMalloc(&tmp, static_cast<size_t>(s->l) * s->d * es) != hipSuccess)
      return rs_err(s, FDSK_ENOMEM, "output staging");
    dst = tmp;
    ld = s->d;
  }
  hipError_t e = hipSuccess;
  if (hashing) {
    hipLaunchKernelGGL(k_rs_out, dim3(s->l), dim3(HNT), 0, s->stream, s->B, s->l, s->l, s->d, nullptr, nullptr,
                       nullptr, 2, dst, ld, out_dtype == FDSK_F64 ? 0 : 1);
  } else {
    hipLaunchKernelGGL(k_rs_out, dim3(s->l), dim3(HNT), 0, s->stream, s->R[s->cur], s->cnt, s->l, s->d,
                       s->w[s->cur], s->kv[s->cur], s->acc + 1, s->kind == FDSK_RS_PRIORITY ? 1 : 0, dst, ld,
                       out_dtype == FDSK_F64 ? 0 : 1);
    e = hipGetLastError();
    if (e == hipSuccess)
      hipLaunchKernelGGL(k_rs_weights, dim3(1), dim3(64), 0, s->stream, s->w[s->cur], s->kv[s->cur], s->acc + 1,
                         s->cnt, s->kind == FDSK_RS_PRIORITY ? 1 : 0, s->acc + 2);
  }
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess && mem == FDSK_MEM_HOST)
    e = hipMemcpy2DAsync(B_out, ldb * es, tmp, s->d * es, s->d * es, s->l, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess && index_out && !hashing && s->cnt > 0)
    e = hipMemcpyAsync(index_out, s->ix[s->cur], static_cast<size_t>(s->cnt) * 8,
                       mem == FDSK_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (tmp) (void)hipFree(tmp);
  if (e != hipSuccess) return rs_err(s, FDSK_EDEVICE, "finalize: %s", hipGetErrorString(e));
  s->finalized = true;
  if (rows_out) *rows_out = hashing ? s->l : s->cnt;
  return 0;
}

int rsketch_stats(const fdsk_rsketch* cs, fdsk_rs_stats* out) {
  fdsk_rsketch* s = const_cast<fdsk_rsketch*>(cs);
  if (!s || !out) return rs_err(s, FDSK_EINVAL, "null argument");
  double h[3] = {0, 0, 0};
  RSCHK(s, hipMemcpyAsync(h, s->acc, sizeof h, hipMemcpyDeviceToHost, s->stream));
  RSCHK(s, hipStreamSynchronize(s->stream));
  std::memset(out, 0, sizeof *out);
  out->fro2_A = h[0];
  out->tau = h[1];
  out->weight_sum = s->finalized ? h[2] : std::nan("");
  out->n_rows = s->n_rows;
  out->rows_kept = (s->kind == FDSK_RS_HASH || s->kind == FDSK_RS_OSNAP) ? s->l : s->cnt;
  return 0;
}

void rsketch_destroy(fdsk_rsketch* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  free_all(s);
  delete s;
}

}  // extern "C"
