// Host side of the many-sketch batch (see include/fdsketch.h and
// kernels_batch.hip): workspace layout, descriptor upload, queue order and
// the C ABI entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "fdsk_batch.hpp"
#include "fdsketch.h"

using namespace fdsk;

struct fdsk_batch {
  int S = 0;
  hipStream_t stream = nullptr;
  std::vector<fdsk_config> cfg;
  std::vector<BatchDesc> desc;     // host copy; per-call fields are rewritten
  void* arena = nullptr;
  BatchDesc* d_desc = nullptr;
  BatchState* d_state = nullptr;
  int* d_order = nullptr;
  int* d_counter = nullptr;
  DevStats* d_stats = nullptr;
  std::vector<int64_t> rows_in;    // rows appended so far per sketch
  std::vector<int32_t> rows_out;
  bool finalized = false;
  int cus = 256;
  int err = 0;
  std::string msg;
};

namespace {

// The persistent many-sketch launch is switched off: its first GPU run ended
// in a device memory fault whose cause has not been shown (a CPU emulation of
// the kernel under AddressSanitizer finds every access in bounds).  Creation
// and stats work; append/finalize report FDSK_EUNSUPPORTED until then.
constexpr bool kBatchLaunchEnabled = false;

thread_local std::string g_batch_err;

int berr(fdsk_batch* b, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (b) {
    b->err = code;
    b->msg = buf;
  } else {
    g_batch_err = buf;
  }
  return code;
}

int rup(int x, int a) { return (x + a - 1) / a * a; }

RuleParams rule_for(const fdsk_config& c) {
  RuleParams rp{};
  rp.variant = static_cast<int>(c.variant);
  rp.l = c.l;
  int s = static_cast<int>(std::ceil(c.alpha * c.l * (1.0 - 1e-12)));
  s = std::min(std::max(s, 1), c.l);
  int r = c.l - s;
  switch (c.variant) {
    case FDSK_FD: rp.t = c.l; rp.r = 0; break;
    case FDSK_ISVD: rp.t = c.l; rp.r = c.l - 1; break;
    case FDSK_ALPHA: rp.t = c.l; rp.r = r; break;
    case FDSK_FAST_ALPHA: rp.t = r + (s + 1) / 2; rp.r = r; break;
  }
  rp.keep = rp.t - 1;
  return rp;
}

// Launch with a queue order that starts with the most expensive sketches
// (estimated ReduceRank count times the cost of one ReduceRank).
int launch(fdsk_batch* b, const std::vector<int64_t>& n, int finalize, int grid_size) {
  if (!kBatchLaunchEnabled)
    return berr(b, FDSK_EUNSUPPORTED, "the persistent many-sketch launch is disabled in this build");
  std::vector<double> cost(b->S);
  for (int i = 0; i < b->S; ++i) {
    const BatchDesc& D = b->desc[i];
    double rr = static_cast<double>(n[i]) / std::max(1, D.m - D.rp.keep) + (finalize ? 1.0 : 0.0);
    double per = 30.0 * D.m * D.m * static_cast<double>(D.m) + 3.0 * D.m * D.m * static_cast<double>(D.d);
    cost[i] = rr * per;
  }
  std::vector<int> order(b->S);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] > cost[c]; });
  hipError_t e = hipMemcpyAsync(b->d_desc, b->desc.data(), sizeof(BatchDesc) * b->S,
                                hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_order, order.data(), sizeof(int) * b->S, hipMemcpyHostToDevice, b->stream);
  int grid = grid_size > 0 ? grid_size : std::min(b->S, b->cus);
  grid = std::max(1, std::min(grid, b->S));
  if (e == hipSuccess)
    e = launch_batch_run(b->d_desc, b->d_state, b->d_order, b->S, b->d_counter, finalize, grid, b->stream);
  // The descriptor array is read by the kernel; keep the host copy stable
  // until the launch has consumed it.
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return berr(b, FDSK_EDEVICE, "batch launch: %s", hipGetErrorString(e));
  return 0;
}

}  // namespace

extern "C" {

const char* sketch_batch_last_error(const fdsk_batch* b) {
  return b ? b->msg.c_str() : g_batch_err.c_str();
}

int sketch_batch_create(int32_t S, const fdsk_config* cfgs, void* hip_stream, fdsk_batch** out) {
  if (!out || !cfgs || S < 1) return berr(nullptr, FDSK_EINVAL, "bad arguments");
  *out = nullptr;
  for (int i = 0; i < S; ++i) {
    const fdsk_config& c = cfgs[i];
    int m = c.buffer_rows == 0 ? 2 * c.l : c.buffer_rows;
    if (c.d < 1 || c.d > 65536 || c.l < 1 || m < c.l)
      return berr(nullptr, FDSK_EINVAL, "sketch %d: bad sizes", i);
    if (m > kBatchMaxRows) return berr(nullptr, FDSK_EUNSUPPORTED, "sketch %d: m = %d > %d", i, m, kBatchMaxRows);
    if (c.variant < FDSK_FD || c.variant > FDSK_FAST_ALPHA) return berr(nullptr, FDSK_EINVAL, "bad variant");
    if ((c.variant == FDSK_ALPHA || c.variant == FDSK_FAST_ALPHA) && !(c.alpha > 0.0 && c.alpha <= 1.0))
      return berr(nullptr, FDSK_EINVAL, "sketch %d: alpha must lie in (0, 1]", i);
    if (c.precision != FDSK_P_FP64 || c.flags != 0)
      return berr(nullptr, FDSK_EUNSUPPORTED, "sketch %d: batched sketches are FP64 without flags", i);
  }
  fdsk_batch* b = new fdsk_batch;
  b->S = S;
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->cfg.assign(cfgs, cfgs + S);
  b->desc.resize(S);
  b->rows_in.assign(S, 0);
  b->rows_out.assign(S, 0);
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      b->cus = cus;
  }
  // One arena: per-sketch buffers, then descriptors, states, order, counter, stats.
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  std::vector<size_t> oC0(S), oC1(S), oG(S), oW(S), oV(S), oUt(S), oL(S), oR(S);
  for (int i = 0; i < S; ++i) {
    const fdsk_config& c = cfgs[i];
    BatchDesc& D = b->desc[i];
    std::memset(&D, 0, sizeof D);
    D.d = static_cast<int>(c.d);
    D.l = c.l;
    D.m = c.buffer_rows == 0 ? 2 * c.l : c.buffer_rows;
    D.mp = rup(D.m, 32);
    D.ldc = rup(D.d, 64);
    D.rp = rule_for(c);
    const size_t cb = static_cast<size_t>(D.mp) * D.ldc * 8, g = static_cast<size_t>(D.mp) * D.mp * 8;
    oC0[i] = take(cb);
    oC1[i] = take(cb);
    oG[i] = take(g);
    oW[i] = take(g);
    oV[i] = take(g);
    oUt[i] = take(g);
    oL[i] = take(D.mp * 8);
    oR[i] = take(D.mp * 8);
  }
  size_t oDesc = take(sizeof(BatchDesc) * S), oState = take(sizeof(BatchState) * S),
         oOrder = take(sizeof(int) * S), oCnt = take(64), oStats = take(sizeof(DevStats) * S);
  hipError_t e = hipMalloc(&b->arena, off);
  if (e != hipSuccess) {
    delete b;
    return berr(nullptr, FDSK_ENOMEM, "batch workspace of %zu bytes: %s", off, hipGetErrorString(e));
  }
  char* a = static_cast<char*>(b->arena);
  b->d_desc = reinterpret_cast<BatchDesc*>(a + oDesc);
  b->d_state = reinterpret_cast<BatchState*>(a + oState);
  b->d_order = reinterpret_cast<int*>(a + oOrder);
  b->d_counter = reinterpret_cast<int*>(a + oCnt);
  b->d_stats = reinterpret_cast<DevStats*>(a + oStats);
  for (int i = 0; i < S; ++i) {
    BatchDesc& D = b->desc[i];
    D.C0 = reinterpret_cast<double*>(a + oC0[i]);
    D.C1 = reinterpret_cast<double*>(a + oC1[i]);
    D.G = reinterpret_cast<double*>(a + oG[i]);
    D.W = reinterpret_cast<double*>(a + oW[i]);
    D.V = reinterpret_cast<double*>(a + oV[i]);
    D.Ut = reinterpret_cast<double*>(a + oUt[i]);
    D.lam = reinterpret_cast<double*>(a + oL[i]);
    D.rownorm = reinterpret_cast<double*>(a + oR[i]);
    D.st = b->d_stats + i;
  }
  e = hipMemsetAsync(b->arena, 0, off, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    (void)hipFree(b->arena);
    delete b;
    return berr(nullptr, FDSK_EDEVICE, "batch init: %s", hipGetErrorString(e));
  }
  *out = b;
  return 0;
}

int sketch_batch_append(fdsk_batch* b, const void* const* rows, const int64_t* n_rows,
                        const int64_t* strides, fdsk_dtype dtype, fdsk_mem mem, int32_t grid_size) {
  if (!b) return berr(nullptr, FDSK_EINVAL, "null batch");
  if (b->err) return b->err;
  if (b->finalized) return berr(b, FDSK_ESTATE, "append after finalize");
  if (!rows || !n_rows || !strides) return berr(b, FDSK_EINVAL, "null argument");
  if (mem != FDSK_MEM_DEVICE) return berr(b, FDSK_EUNSUPPORTED, "batched rows must be on the device");
  if (dtype != FDSK_F64 && dtype != FDSK_F32 && dtype != FDSK_BF16) return berr(b, FDSK_EINVAL, "bad dtype");
  std::vector<int64_t> n(b->S);
  for (int i = 0; i < b->S; ++i) {
    if (n_rows[i] < 0) return berr(b, FDSK_EINVAL, "sketch %d: n_rows < 0", i);
    if (n_rows[i] > 0 && (!rows[i] || strides[i] < b->desc[i].d))
      return berr(b, FDSK_EINVAL, "sketch %d: bad rows or stride", i);
    BatchDesc& D = b->desc[i];
    D.rows = rows[i];
    D.stride = strides[i];
    D.n = n_rows[i];
    D.dt = static_cast<int>(dtype);
    D.out = nullptr;
    n[i] = n_rows[i];
  }
  int rc = launch(b, n, 0, grid_size);
  if (rc) return rc;
  for (int i = 0; i < b->S; ++i) b->rows_in[i] += n[i];
  return 0;
}

int sketch_batch_finalize(fdsk_batch* b, void* const* B_out, const int64_t* ldb, fdsk_dtype out_dtype,
                          fdsk_mem mem, int32_t grid_size, int32_t* rows_out) {
  if (!b) return berr(nullptr, FDSK_EINVAL, "null batch");
  if (b->err) return b->err;
  if (b->finalized) return berr(b, FDSK_ESTATE, "finalize called twice");
  if (!B_out || !ldb) return berr(b, FDSK_EINVAL, "null argument");
  if (mem != FDSK_MEM_DEVICE) return berr(b, FDSK_EUNSUPPORTED, "batched outputs must be on the device");
  if (out_dtype != FDSK_F64 && out_dtype != FDSK_F32) return berr(b, FDSK_EINVAL, "output dtype");
  std::vector<int64_t> n(b->S, 0);
  for (int i = 0; i < b->S; ++i) {
    if (!B_out[i] || ldb[i] < b->desc[i].d) return berr(b, FDSK_EINVAL, "sketch %d: bad output", i);
    BatchDesc& D = b->desc[i];
    D.rows = nullptr;
    D.n = 0;
    D.out = B_out[i];
    D.ldb = ldb[i];
    D.out_dt = static_cast<int>(out_dtype);
  }
  int rc = launch(b, n, 1, grid_size);
  if (rc) return rc;
  b->finalized = true;
  std::vector<BatchState> st(b->S);
  std::vector<DevStats> ds(b->S);
  hipError_t e = hipMemcpyAsync(st.data(), b->d_state, sizeof(BatchState) * b->S, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ds.data(), b->d_stats, sizeof(DevStats) * b->S, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return berr(b, FDSK_EDEVICE, "batch finalize: %s", hipGetErrorString(e));
  int bad = -1;
  for (int i = 0; i < b->S; ++i) {
    b->rows_out[i] = std::min(st[i].occ, b->desc[i].l);
    if (rows_out) rows_out[i] = b->rows_out[i];
    if (ds[i].nonfinite && bad < 0) bad = i;
  }
  if (bad >= 0) return berr(b, FDSK_ENONFINITE, "sketch %d: a NaN or Inf reached the sketch", bad);
  return 0;
}

int sketch_batch_stats(const fdsk_batch* cb, int32_t index, fdsk_report* out) {
  fdsk_batch* b = const_cast<fdsk_batch*>(cb);
  if (!b || !out || index < 0 || index >= b->S) return berr(b, FDSK_EINVAL, "bad arguments");
  DevStats h{};
  hipError_t e = hipMemcpyAsync(&h, b->d_stats + index, sizeof h, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return berr(b, FDSK_EDEVICE, "batch stats: %s", hipGetErrorString(e));
  std::memset(out, 0, sizeof *out);
  out->fro2_A = h.fro2A;
  out->delta_sum = h.Delta;
  out->shrink_total = h.Stot;
  out->n_rows = b->rows_in[index];
  out->n_reduce = h.n_rr;
  out->rows_out = b->rows_out[index];
  out->eig_unconverged = h.eig_unconv;
  out->eig_sweeps = static_cast<int64_t>(h.eig_sweeps);
  out->cov_err = out->proj_err_k = out->proj_full_over_fro2 = std::nan("");
  out->fro2_B = out->lambda_max = out->lambda_min = std::nan("");
  return 0;
}

void sketch_batch_destroy(fdsk_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  if (b->arena) (void)hipFree(b->arena);
  delete b;
}

}  // extern "C"
