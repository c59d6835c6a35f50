// Host runtime and C ABI of libfdsketch.so (see include/fdsketch.h).
//
// A sketch owns an m-row FP64 buffer on the device (double-buffered for the
// rebuild), the Gram / eigen / rebuild workspaces and FP64 accumulators.  The
// schedule of Algorithm 1 is data independent (rows go after the first t-1
// surviving rows; a ReduceRank runs when all m rows are occupied), so the host
// plans every launch without reading anything back: ingest, Gram, eigensolve,
// shrink and rebuild are enqueued on the sketch's stream in order and the
// host only synchronises in finalize / stats / error.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fdsk_kernels.hpp"
#include "fdsk_eval.hpp"
#include "fdsk_eval_api.hpp"
#include "fdsk_tune.hpp"
#include "fdsketch.h"

using namespace fdsk;

struct fdsk_sketch {
  fdsk_config cfg;
  int d = 0, l = 0, m = 0, mp = 0, ldc = 0;
  RuleParams rp{};
  hipStream_t stream = nullptr;
  void* arena = nullptr;
  double* C[2] = {nullptr, nullptr};
  int cur = 0;
  double *G = nullptr, *Gpart = nullptr, *W = nullptr, *V = nullptr, *lam = nullptr,
         *Ut = nullptr, *rownorm = nullptr, *S1 = nullptr, *S2 = nullptr;
  double *mass_b = nullptr, *mass_a = nullptr;   // row masses before / after a reduction
  void* q8 = nullptr;   // FP8 codes and scales of the buffer (FDSK_P_FP8X3)
  void* bfw = nullptr;  // the buffer's bf16 hi/lo halves (every reduced precision)
  int ksplit_max = 1;   // Gram partials the workspace holds
  int ksplit = 0;       // tuned Gram split-K count (0: the launch's default)
  int rt = 32;          // tuned rebuild rows per workgroup
  DevStats* st = nullptr;
  unsigned* bar = nullptr;
  int* rot = nullptr;
  void* stage = nullptr;
  size_t stage_bytes = 0;
  int occ = 0;      // occupied rows
  int new0 = 0;     // first row appended since the last ReduceRank
  int64_t n_rows = 0;
  int64_t n_rr_host = 0;
  bool finalized = false;
  int rows_out = 0;
  int err = 0;
  std::string msg;
  // Stage profiling (FDSK_FLAG_PROFILE): event pairs recorded on the stream.
  bool profile = false;
  std::vector<hipEvent_t> ev_pool;
  struct Mark { int stage; hipEvent_t a, b; double work; };
  std::vector<Mark> marks;
};

namespace {

thread_local std::string g_last_error;

int set_err(fdsk_sketch* s, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (s) {
    s->err = code;
    s->msg = buf;
  } else {
    g_last_error = buf;
  }
  return code;
}

#define HIPCHK(s, expr)                                                                    \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return set_err((s), FDSK_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
  } while (0)

size_t dtype_size(fdsk_dtype dt) {
  switch (dt) {
    case FDSK_F64: return 8;
    case FDSK_F32: return 4;
    case FDSK_BF16: return 2;
  }
  return 0;
}

int round_up(int x, int a) { return (x + a - 1) / a * a; }

RuleParams make_rule(const fdsk_config& c) {
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
    case FDSK_SSD: rp.t = c.l; rp.r = 0; break;
    case FDSK_CFD: rp.t = c.l; rp.r = 0; break;
  }
  rp.keep = rp.t - 1;
  // Reduced-precision products: the shrink total is measured from the rows
  // (see RuleParams).  Compensative FD keeps the spectral count, its last
  // step adding mass back from the previous reduction's spectrum.
  rp.mass = (c.precision != FDSK_P_FP64 && c.variant != FDSK_CFD) ? 1 : 0;
  return rp;
}

hipEvent_t take_event(fdsk_sketch* s) {
  hipEvent_t e = nullptr;
  if (!s->ev_pool.empty()) {
    e = s->ev_pool.back();
    s->ev_pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    e = nullptr;
  }
  return e;
}

// Record an event on the stream (profiling only); returns it or nullptr.
hipEvent_t mark(fdsk_sketch* s) {
  if (!s->profile) return nullptr;
  hipEvent_t e = take_event(s);
  if (e && hipEventRecord(e, s->stream) != hipSuccess) return nullptr;
  return e;
}

void add_mark(fdsk_sketch* s, int stage, hipEvent_t a, hipEvent_t b, double work) {
  if (a && b) s->marks.push_back({stage, a, b, work});
}

// Algorithmic work of the stages of one ReduceRank on m buffer rows (the
// figures sketch_profile reports, see the header).
double passes(const fdsk_sketch* s) { return s->cfg.precision == FDSK_P_FP64 ? 1.0 : 3.0; }
double work_gram(const fdsk_sketch* s) { return passes(s) * s->m * (s->m + 1.0) * s->d; }
double work_tridiag(const fdsk_sketch* s) { return 4.0 / 3.0 * s->m * s->m * (double)s->m; }
double work_dc(const fdsk_sketch* s) { return 4.0 / 3.0 * s->m * s->m * (double)s->m; }
double work_backtr(const fdsk_sketch* s) {
  return 2.0 * s->m * s->m * (double)std::min(s->m, s->l);
}

// The Gram of buffer C in the sketch's precision with ksplit K slices (0:
// the launch's default count).
hipError_t gram_launch(fdsk_sketch* s, const double* C, int ksplit) {
  if (s->cfg.precision == FDSK_P_FP64)
    return launch_gram(C, s->ldc, s->mp, s->Gpart, s->ksplit_max, s->G, s->stream, ksplit);
  if (s->cfg.precision == FDSK_P_FP8X3)
    return launch_gram_fp8(C, s->ldc, s->mp, s->q8, s->Gpart, s->ksplit_max, s->G, s->stream, ksplit);
  const int npass = s->cfg.precision == FDSK_P_BF16 ? 1 : 3;
  return launch_gram_lowp(C, s->ldc, s->mp, s->Gpart, s->ksplit_max, s->G, npass, s->bfw, s->stream, ksplit);
}

// Precision tag of the tuning keys: the Gram's arithmetic, and the rebuild's
// (FP8X3 rebuilds with split-BF16 x3).
int gram_tag(const fdsk_sketch* s) {
  switch (s->cfg.precision) {
    case FDSK_P_FP64: return 0;
    case FDSK_P_BF16: return 1;
    case FDSK_P_FP8X3: return 8;
    default: return 3;
  }
}
int rebuild_tag(const fdsk_sketch* s) { return s->cfg.precision == FDSK_P_FP64 ? 0 : 3; }

// Pick the Gram's split-K count and the rebuild's rows per workgroup for
// this sketch's sizes (see fdsk_tune.hpp).  Runs on the new sketch's zeroed
// workspaces, which the candidates overwrite with zeros.
int tune_shapes(fdsk_sketch* s) {
  if (tune_mode() == TUNE_OFF) return 0;
  const std::string dev = tune_device_tag();
  const std::string sizes = "|m" + std::to_string(s->mp) + "|d" + std::to_string(tune_bucket(s->ldc));
  // Gram: the default count and every power of two the workspace holds.
  const int tile = s->cfg.precision == FDSK_P_FP64 || s->cfg.precision == FDSK_P_FP8X3 ? 32 : 64;
  const int T = (s->mp + tile - 1) / tile;
  const int dflt = std::min(gram_ksplit_default(T * (T + 1) / 2, s->ldc), s->ksplit_max);
  std::vector<int> cand{dflt};
  for (int k = 1; k <= s->ksplit_max; k *= 2)
    if (k != dflt) cand.push_back(k);
  s->ksplit = tune_pick(dev + "|gram|p" + std::to_string(gram_tag(s)) + sizes, cand, dflt, s->stream,
                        [s](int k) { return gram_launch(s, s->C[0], k); });
  // Rebuild: 32 or 64 rows per workgroup (64 only when more than 32 rows
  // are kept).
  const int keep = s->rp.keep;
  if (keep > 32) {
    const int npass = s->cfg.precision == FDSK_P_BF16 ? 1 : 3;
    s->rt = tune_pick(dev + "|rebuild|p" + std::to_string(rebuild_tag(s)) + sizes, {32, 64}, 32, s->stream,
                      [s, keep, npass](int rt) {
                        if (s->cfg.precision == FDSK_P_FP64)
                          return launch_rebuild(s->Ut, s->C[0], s->ldc, s->mp, keep, s->C[1], s->stream, rt);
                        return launch_rebuild_lowp(s->Ut, s->C[0], s->ldc, s->mp, keep, s->C[1], npass, s->bfw,
                                                   s->stream, rt);
                      });
  }
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return 0;
}

// Gram and eigensolve of the current buffer: lam and V on the device.
int spectrum(fdsk_sketch* s) {
  EigWork wk{s->W, s->bar, s->rot, s->st, s->S1, s->S2,
             (s->cfg.flags & FDSK_FLAG_EIG_JACOBI) ? EIG_JACOBI : EIG_AUTO};
  hipEvent_t e0 = mark(s);
  HIPCHK(s, gram_launch(s, s->C[s->cur], s->ksplit));
  hipEvent_t e1 = mark(s);
  if (eig_uses_trid(s->m, wk)) {
    HIPCHK(s, launch_tridiag(s->G, s->m, s->mp, wk, s->stream));
    hipEvent_t t1 = mark(s);
    // Every rule reads at most the eigenvectors of the l largest values.
    HIPCHK(s, launch_dc(s->m, s->mp, s->lam, s->V, wk, s->stream, std::min(s->m, s->l)));
    hipEvent_t t2 = mark(s);
    HIPCHK(s, launch_backtr(s->m, s->mp, s->V, wk, s->stream));
    hipEvent_t t3 = mark(s);
    add_mark(s, FDSK_STAGE_TRIDIAG, e1, t1, work_tridiag(s));
    add_mark(s, FDSK_STAGE_DC, t1, t2, work_dc(s));
    add_mark(s, FDSK_STAGE_BACKTR, t2, t3, work_backtr(s));
  } else {
    HIPCHK(s, launch_eig(s->G, s->m, s->mp, s->lam, s->V, wk, s->stream));
  }
  hipEvent_t e2 = mark(s);
  add_mark(s, FDSK_STAGE_GRAM, e0, e1, work_gram(s));
  add_mark(s, FDSK_STAGE_EIG, e1, e2, work_tridiag(s) + work_dc(s) + work_backtr(s));
  return 0;
}

// Shrink with rule rp and rebuild rp.keep rows of src into dst.
int shrink_rebuild(fdsk_sketch* s, const RuleParams& rp, int new0, int new1, const double* src,
                   double* dst) {
  const int npass = s->cfg.precision == FDSK_P_BF16 ? 1 : 3;
  hipEvent_t e2 = mark(s);
  if (rp.mass) HIPCHK(s, launch_row_mass(src, s->ldc, s->m, s->d, s->mass_b, s->stream));
  HIPCHK(s, launch_shrink(s->lam, s->V, s->m, s->mp, rp, s->rownorm, new0, new1, s->Ut, s->st,
                          s->stream));
  hipEvent_t e3 = mark(s);
  if (s->cfg.precision == FDSK_P_FP64)
    HIPCHK(s, launch_rebuild(s->Ut, src, s->ldc, s->mp, rp.keep, dst, s->stream, s->rt));
  else {
    // The bf16 paths read the halves the Gram of the same buffer wrote (src
    // is that buffer for every caller); the FP8 Gram wrote none, so FP8X3
    // splits the buffer first and rebuilds with split-BF16 x3.
    if (s->cfg.precision == FDSK_P_FP8X3) HIPCHK(s, launch_split_bf16(src, s->ldc, s->mp, s->bfw, s->stream));
    HIPCHK(s, launch_rebuild_lowp(s->Ut, src, s->ldc, s->mp, rp.keep, dst, npass, s->bfw, s->stream, s->rt));
  }
  if (rp.mass) {
    HIPCHK(s, launch_row_mass(dst, s->ldc, rp.keep, s->d, s->mass_a, s->stream));
    HIPCHK(s, launch_mass_close(s->mass_b, s->m, s->mass_a, rp.keep, s->st, s->stream));
  }
  add_mark(s, FDSK_STAGE_SHRINK, e2, e3, 0.0);
  add_mark(s, FDSK_STAGE_REBUILD, e3, mark(s), passes(s) * 2.0 * rp.keep * s->m * (double)s->d);
  return 0;
}

int reduce(fdsk_sketch* s) {
  int rc = spectrum(s);
  if (rc) return rc;
  rc = shrink_rebuild(s, s->rp, s->new0, s->occ, s->C[s->cur], s->C[1 - s->cur]);
  if (rc) return rc;
  s->cur = 1 - s->cur;
  s->occ = s->rp.keep;
  s->new0 = s->occ;
  s->n_rr_host += 1;
  return 0;
}

// Algorithm 1's insertion of n rows.  count = false inserts another
// sketch's rows (a merge): their squared norms are zeroed so that they do not
// enter ||A||_F^2, and they are not counted as stream rows.
int ingest_device(fdsk_sketch* s, const char* src, int64_t n, int64_t stride, fdsk_dtype dt,
                  bool count = true) {
  const size_t es = dtype_size(dt);
  int64_t i = 0;
  while (i < n) {
    int f = static_cast<int>(std::min<int64_t>(s->m - s->occ, n - i));
    hipEvent_t a = mark(s);
    HIPCHK(s, launch_ingest(src + i * stride * es, static_cast<int>(dt), stride, f, s->d,
                            s->C[s->cur], s->ldc, s->occ, s->rownorm, s->stream));
    if (!count) HIPCHK(s, launch_zero_rows(s->rownorm, 1, s->occ, s->occ + f, s->stream));
    add_mark(s, FDSK_STAGE_INGEST, a, mark(s), static_cast<double>(f) * s->d * (es + 8.0));
    s->occ += f;
    i += f;
    if (count) s->n_rows += f;
    if (s->occ == s->m) {
      int rc = reduce(s);
      if (rc) return rc;
    }
  }
  return 0;
}

// Compensative FD's last step (Section 3.1): B = S^ V^T of the latest
// reduction with sigma^_j^2 = sigma'_j^2 + Delta on the first l directions.
// When no row arrived after the latest reduction, its spectrum (lam, V) and the
// buffer it factored (the other half of the double buffer) are still on the
// device and the l output rows are rebuilt from them.  Otherwise the current
// buffer is factored (after one more FD reduction when more than l rows are
// occupied, which brings back the first case) and compensated as it is.
int finalize_cfd(fdsk_sketch* s) {
  if (s->n_rows == 0) return 0;
  if (s->occ > s->l) {
    HIPCHK(s, launch_zero_rows(s->C[s->cur], s->ldc, s->occ, s->m, s->stream));
    int rc = reduce(s);
    if (rc) return rc;
  }
  RuleParams rp = s->rp;
  rp.keep = s->l;
  int rc;
  if (s->n_rr_host > 0 && s->occ == s->new0) {
    rp.comp = 1;
    rc = shrink_rebuild(s, rp, s->new0, s->new0, s->C[1 - s->cur], s->C[s->cur]);
  } else {
    HIPCHK(s, launch_zero_rows(s->C[s->cur], s->ldc, s->occ, s->m, s->stream));
    rc = spectrum(s);
    if (rc) return rc;
    rp.comp = 2;
    rc = shrink_rebuild(s, rp, s->new0, s->occ, s->C[s->cur], s->C[1 - s->cur]);
    s->cur = 1 - s->cur;
  }
  if (rc) return rc;
  s->occ = s->l;
  s->new0 = s->occ;
  return 0;
}

int check_device_flags(fdsk_sketch* s) {
  DevStats h{};
  HIPCHK(s, hipMemcpyAsync(&h, s->st, sizeof h, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  if (h.bar_err) return set_err(s, FDSK_EDEVICE, "grid barrier timed out in the eigensolver");
  if (h.nonfinite) return set_err(s, FDSK_ENONFINITE, "a NaN or Inf reached the sketch");
  return 0;
}

}  // namespace

void fdsk::set_last_error(const char* msg) { g_last_error = msg ? msg : ""; }

extern "C" {

const char* fdsk_version(void) {
  return "fdsketch 0.3 (gfx950; FP64 / BF16 / BF16x3 Gram and rebuild; FP64 tridiagonal divide-and-conquer "
         "and Jacobi eigensolvers)";
}

const char* sketch_last_error(const fdsk_sketch* s) {
  if (!s) return g_last_error.c_str();
  return s->msg.c_str();
}

int sketch_create(const fdsk_config* cfg, void* hip_stream, fdsk_sketch** out) {
  if (!cfg || !out) return set_err(nullptr, FDSK_EINVAL, "null argument");
  *out = nullptr;
  const fdsk_config& c = *cfg;
  if (c.d < 1 || c.d > 65536) return set_err(nullptr, FDSK_EINVAL, "d must be in [1, 65536]");
  if (c.l < 1) return set_err(nullptr, FDSK_EINVAL, "l must be >= 1");
  int m = c.buffer_rows == 0 ? 2 * c.l : c.buffer_rows;
  if (m < c.l) return set_err(nullptr, FDSK_EINVAL, "buffer_rows must be 0 or >= l");
  if (m > 1024) return set_err(nullptr, FDSK_EUNSUPPORTED, "buffer rows %d > 1024", m);
  if (c.variant < FDSK_FD || c.variant > FDSK_CFD)
    return set_err(nullptr, FDSK_EINVAL, "unknown variant");
  if (c.variant == FDSK_SSD && (m != c.l || c.l < 2))
    return set_err(nullptr, FDSK_EINVAL, "SSD needs buffer_rows == l and l >= 2");
  if ((c.variant == FDSK_ALPHA || c.variant == FDSK_FAST_ALPHA) && !(c.alpha > 0.0 && c.alpha <= 1.0))
    return set_err(nullptr, FDSK_EINVAL, "alpha must lie in (0, 1]");
  if (c.precision != FDSK_P_FP64 && c.precision != FDSK_P_BF16 && c.precision != FDSK_P_BF16X3 &&
      c.precision != FDSK_P_FP8X3)
    return set_err(nullptr, FDSK_EINVAL, "unknown precision %d", (int)c.precision);
  // One uncompensated BF16 pass keeps ~8 significant bits per operand; the
  // covariance error it reaches misses the 1e-3 (of ||A||_F^2) bar set for
  // reduced-precision sketches, so it is offered by fdsk_gram only.
  if (c.precision == FDSK_P_BF16)
    return set_err(nullptr, FDSK_EUNSUPPORTED,
                   "single-pass BF16 is not a sketching precision (use FDSK_P_BF16X3)");
  if (c.flags & ~(FDSK_FLAG_PROFILE | FDSK_FLAG_EIG_JACOBI))
    return set_err(nullptr, FDSK_EINVAL, "unknown flags");

  fdsk_sketch* s = new fdsk_sketch;
  s->cfg = c;
  s->d = static_cast<int>(c.d);
  s->l = c.l;
  s->m = m;
  s->mp = round_up(m, 32);
  s->ldc = round_up(s->d, 64);
  s->rp = make_rule(c);
  s->stream = static_cast<hipStream_t>(hip_stream);
  s->profile = (c.flags & FDSK_FLAG_PROFILE) != 0;
  // Gram partials: up to 16 K slices of at least 128 columns (the tuner's
  // candidates).
  s->ksplit_max = std::max(1, std::min(16, s->ldc / 128));

  const size_t mp2 = static_cast<size_t>(s->mp) * s->mp;
  const size_t cbuf = static_cast<size_t>(s->mp) * s->ldc;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  size_t oC0 = take(cbuf * 8), oC1 = take(cbuf * 8), oG = take(mp2 * 8),
         oGp = take(mp2 * 8 * s->ksplit_max), oW = take(mp2 * 8), oV = take(mp2 * 8),
         oUt = take(mp2 * 8), oLam = take(s->mp * 8), oRn = take(s->mp * 8),
         oSt = take(sizeof(DevStats)), oBar = take(4 * sizeof(unsigned)),
         oRot = take(kMaxSweeps * sizeof(int)), oS1 = take(mp2 * 8), oS2 = take(mp2 * 8),
         oMb = take(s->mp * 8), oMa = take(s->mp * 8),
         oQ8 = take(c.precision == FDSK_P_FP8X3 ? fp8_workspace_bytes(s->mp, s->ldc) : 0),
         oBf = take(c.precision != FDSK_P_FP64 ? bf16_workspace_bytes(s->mp, s->ldc) : 0);
  hipError_t e = hipMalloc(&s->arena, off);
  if (e != hipSuccess) {
    delete s;
    return set_err(nullptr, FDSK_ENOMEM, "hipMalloc(%zu) failed: %s", off, hipGetErrorString(e));
  }
  char* a = static_cast<char*>(s->arena);
  s->C[0] = reinterpret_cast<double*>(a + oC0);
  s->C[1] = reinterpret_cast<double*>(a + oC1);
  s->G = reinterpret_cast<double*>(a + oG);
  s->Gpart = reinterpret_cast<double*>(a + oGp);
  s->W = reinterpret_cast<double*>(a + oW);
  s->V = reinterpret_cast<double*>(a + oV);
  s->Ut = reinterpret_cast<double*>(a + oUt);
  s->lam = reinterpret_cast<double*>(a + oLam);
  s->rownorm = reinterpret_cast<double*>(a + oRn);
  s->st = reinterpret_cast<DevStats*>(a + oSt);
  s->bar = reinterpret_cast<unsigned*>(a + oBar);
  s->rot = reinterpret_cast<int*>(a + oRot);
  s->S1 = reinterpret_cast<double*>(a + oS1);
  s->S2 = reinterpret_cast<double*>(a + oS2);
  s->mass_b = reinterpret_cast<double*>(a + oMb);
  s->mass_a = reinterpret_cast<double*>(a + oMa);
  s->q8 = (c.precision == FDSK_P_FP8X3) ? static_cast<void*>(a + oQ8) : nullptr;
  s->bfw = (c.precision != FDSK_P_FP64) ? static_cast<void*>(a + oBf) : nullptr;
  e = hipMemsetAsync(s->arena, 0, off, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) {
    (void)hipFree(s->arena);
    delete s;
    return set_err(nullptr, FDSK_EDEVICE, "initialising sketch memory failed: %s",
                   hipGetErrorString(e));
  }
  if (tune_shapes(s)) {
    g_last_error = s->msg;
    (void)hipFree(s->arena);
    delete s;
    return FDSK_EDEVICE;
  }
  *out = s;
  return 0;
}

int sketch_append_rows(fdsk_sketch* s, const void* rows, int64_t n_rows, int64_t row_stride,
                       fdsk_dtype dtype, fdsk_mem mem) {
  if (!s) return set_err(nullptr, FDSK_EINVAL, "null sketch");
  if (s->err) return s->err;
  if (s->finalized) return set_err(s, FDSK_ESTATE, "append after finalize");
  if (n_rows < 0) return set_err(s, FDSK_EINVAL, "n_rows < 0");
  if (n_rows == 0) return 0;
  if (!rows) return set_err(s, FDSK_EINVAL, "null rows");
  if (dtype_size(dtype) == 0) return set_err(s, FDSK_EINVAL, "bad dtype");
  if (row_stride < s->d) return set_err(s, FDSK_EINVAL, "row_stride < d");
  if (mem == FDSK_MEM_DEVICE)
    return ingest_device(s, static_cast<const char*>(rows), n_rows, row_stride, dtype);
  if (mem != FDSK_MEM_HOST) return set_err(s, FDSK_EINVAL, "bad mem kind");
  // Host rows: staged through a device buffer, chunk by chunk.
  const size_t es = dtype_size(dtype);
  const size_t row_bytes = static_cast<size_t>(s->d) * es;
  int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(n_rows, (64 << 20) / row_bytes));
  if (s->stage_bytes < chunk * row_bytes) {
    HIPCHK(s, hipStreamSynchronize(s->stream));
    if (s->stage) HIPCHK(s, hipFree(s->stage));
    s->stage = nullptr;
    s->stage_bytes = 0;
    hipError_t e = hipMalloc(&s->stage, chunk * row_bytes);
    if (e != hipSuccess) return set_err(s, FDSK_ENOMEM, "staging buffer: %s", hipGetErrorString(e));
    s->stage_bytes = chunk * row_bytes;
  }
  const char* h = static_cast<const char*>(rows);
  for (int64_t i = 0; i < n_rows; i += chunk) {
    int64_t c = std::min(chunk, n_rows - i);
    HIPCHK(s, hipMemcpy2DAsync(s->stage, row_bytes, h + i * row_stride * es, row_stride * es,
                               row_bytes, c, hipMemcpyHostToDevice, s->stream));
    int rc = ingest_device(s, static_cast<const char*>(s->stage), c, s->d, dtype);
    if (rc) return rc;
  }
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return 0;
}

int sketch_merge(fdsk_sketch* dst, fdsk_sketch* src) {
  if (!dst || !src) return set_err(dst, FDSK_EINVAL, "null sketch");
  if (dst == src) return set_err(dst, FDSK_EINVAL, "a sketch cannot absorb itself");
  if (dst->err) return dst->err;
  if (src->err) return set_err(dst, FDSK_EINVAL, "the source sketch is in an error state");
  if (dst->finalized || src->finalized) return set_err(dst, FDSK_ESTATE, "merge after finalize");
  const fdsk_config& a = dst->cfg;
  const fdsk_config& b = src->cfg;
  const bool uses_alpha = a.variant == FDSK_ALPHA || a.variant == FDSK_FAST_ALPHA;
  if (a.d != b.d || a.l != b.l || dst->m != src->m || a.variant != b.variant ||
      a.precision != b.precision || (uses_alpha && a.alpha != b.alpha))
    return set_err(dst, FDSK_EINVAL, "merge needs sketches of the same configuration");
  // dst's stream waits for src's work; src's stream then waits for dst's
  // reads of src's buffer.
  hipEvent_t ev = nullptr;
  HIPCHK(dst, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  hipError_t e = hipEventRecord(ev, src->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(dst->stream, ev, 0);
  if (e == hipSuccess) e = launch_merge_stats(dst->st, src->st, src->rownorm, src->new0, src->occ, dst->stream);
  if (e != hipSuccess) {
    (void)hipEventDestroy(ev);
    return set_err(dst, FDSK_EDEVICE, "merge: %s", hipGetErrorString(e));
  }
  int rc = ingest_device(dst, reinterpret_cast<const char*>(src->C[src->cur]), src->occ, src->ldc,
                         FDSK_F64, false);
  if (rc == 0) {
    e = hipEventRecord(ev, dst->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(src->stream, ev, 0);
    if (e != hipSuccess) rc = set_err(dst, FDSK_EDEVICE, "merge: %s", hipGetErrorString(e));
  }
  (void)hipEventDestroy(ev);
  if (rc) return rc;
  dst->n_rows += src->n_rows;
  return 0;
}

int sketch_finalize(fdsk_sketch* s, void* B_out, int64_t ldb, fdsk_dtype out_dtype, fdsk_mem mem,
                    int32_t* rows_out) {
  if (!s) return set_err(nullptr, FDSK_EINVAL, "null sketch");
  if (s->err) return s->err;
  if (s->finalized) return set_err(s, FDSK_ESTATE, "finalize called twice");
  if (!B_out) return set_err(s, FDSK_EINVAL, "null B_out");
  if (ldb < s->d) return set_err(s, FDSK_EINVAL, "ldb < d");
  if (out_dtype != FDSK_F64 && out_dtype != FDSK_F32)
    return set_err(s, FDSK_EINVAL, "output dtype must be F64 or F32");
  if (s->cfg.variant == FDSK_CFD) {
    int rc = finalize_cfd(s);
    if (rc) return rc;
  } else if (s->occ > s->l) {
    HIPCHK(s, launch_zero_rows(s->C[s->cur], s->ldc, s->occ, s->m, s->stream));
    int rc = reduce(s);
    if (rc) return rc;
  } else if (s->occ > s->new0) {
    HIPCHK(s, launch_add_pending_norms(s->rownorm, s->new0, s->occ, s->st, s->stream));
    s->new0 = s->occ;
  }
  s->finalized = true;
  s->rows_out = std::min(s->occ, s->l);
  const size_t es = dtype_size(out_dtype);
  if (mem == FDSK_MEM_DEVICE) {
    HIPCHK(s, launch_copy_out(s->C[s->cur], s->ldc, s->rows_out, s->l, s->d, B_out, ldb,
                              static_cast<int>(out_dtype), s->stream));
  } else {
    void* tmp = nullptr;
    size_t bytes = static_cast<size_t>(s->l) * s->d * es;
    hipError_t e = hipMalloc(&tmp, bytes);
    if (e != hipSuccess) return set_err(s, FDSK_ENOMEM, "output staging: %s", hipGetErrorString(e));
    e = launch_copy_out(s->C[s->cur], s->ldc, s->rows_out, s->l, s->d, tmp, s->d,
                        static_cast<int>(out_dtype), s->stream);
    if (e == hipSuccess)
      e = hipMemcpy2DAsync(B_out, ldb * es, tmp, s->d * es, s->d * es, s->l,
                           hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return set_err(s, FDSK_EDEVICE, "copy-out: %s", hipGetErrorString(e));
  }
  if (rows_out) *rows_out = s->rows_out;
  return check_device_flags(s);
}

int sketch_stats(const fdsk_sketch* cs, fdsk_report* out) {
  fdsk_sketch* s = const_cast<fdsk_sketch*>(cs);
  if (!s || !out) return set_err(s, FDSK_EINVAL, "null argument");
  DevStats h{};
  HIPCHK(s, hipMemcpyAsync(&h, s->st, sizeof h, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  std::memset(out, 0, sizeof *out);
  out->fro2_A = h.fro2A;
  out->delta_sum = h.Delta;
  out->shrink_total = h.Stot;
  out->n_rows = s->n_rows;
  out->n_reduce = h.n_rr;
  out->rows_out = s->finalized ? s->rows_out : std::min(s->occ, s->l);
  out->eig_unconverged = h.eig_unconv;
  out->eig_sweeps = static_cast<int64_t>(h.eig_sweeps);
  out->cov_err = out->proj_err_k = out->proj_full_over_fro2 = std::nan("");
  out->fro2_B = std::nan("");
  out->lambda_max = out->lambda_min = std::nan("");
  return 0;
}

int sketch_reset(fdsk_sketch* s) {
  if (!s) return set_err(nullptr, FDSK_EINVAL, "null sketch");
  // Counters of the grid barrier and the buffers' zero padding are kept; the
  // accumulators and occupancy start over.  Rows beyond occ are never read
  // before they are written again, so the buffers need no clearing.
  HIPCHK(s, hipMemsetAsync(s->st, 0, sizeof(DevStats), s->stream));
  s->cur = 0;
  s->occ = 0;
  s->new0 = 0;
  s->n_rows = 0;
  s->n_rr_host = 0;
  s->finalized = false;
  s->rows_out = 0;
  s->err = 0;
  s->msg.clear();
  return 0;
}

int sketch_profile(fdsk_sketch* s, fdsk_profile* out) {
  if (!s || !out) return set_err(s, FDSK_EINVAL, "null argument");
  HIPCHK(s, hipStreamSynchronize(s->stream));
  std::memset(out, 0, sizeof *out);
  for (auto& mk : s->marks) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, mk.a, mk.b) == hipSuccess) {
      out->ms[mk.stage] += ms;
      out->launches[mk.stage] += 1;
      out->work[mk.stage] += mk.work;
    }
  }
  // Events are shared between neighbouring marks; return each once.
  std::vector<hipEvent_t> seen;
  for (auto& mk : s->marks) {
    seen.push_back(mk.a);
    seen.push_back(mk.b);
  }
  std::sort(seen.begin(), seen.end());
  seen.erase(std::unique(seen.begin(), seen.end()), seen.end());
  for (auto e : seen) s->ev_pool.push_back(e);
  s->marks.clear();
  return 0;
}

void sketch_destroy(fdsk_sketch* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  for (auto& mk : s->marks) {
    s->ev_pool.push_back(mk.a);
    s->ev_pool.push_back(mk.b);
  }
  std::sort(s->ev_pool.begin(), s->ev_pool.end());
  s->ev_pool.erase(std::unique(s->ev_pool.begin(), s->ev_pool.end()), s->ev_pool.end());
  for (auto e : s->ev_pool) (void)hipEventDestroy(e);
  if (s->stage) (void)hipFree(s->stage);
  if (s->arena) (void)hipFree(s->arena);
  delete s;
}

}  // extern "C"

namespace {

// Run the device evaluator; A may be on the host (staged to the device).
int run_evaluator(fdsk_sketch* owner, const void* A, int64_t n, int64_t lda, fdsk_dtype a_dt,
                  fdsk_mem mem, const double* Bdev, int64_t rows_b, int64_t ldb, int d, int k,
                  int method, hipStream_t st, fdsk_report* out) {
  if (n < 1) return set_err(owner, FDSK_EINVAL, "A has no rows");
  if (lda < d) return set_err(owner, FDSK_EINVAL, "lda < d");
  if (k < 0) return set_err(owner, FDSK_EINVAL, "k < 0");
  if (method != 0 && method != 1) return set_err(owner, FDSK_EINVAL, "method must be 0 or 1");
  if (method == 0 && d > 8192) return set_err(owner, FDSK_EUNSUPPORTED, "dense evaluation needs d <= 8192");
  if (rows_b > 1024) return set_err(owner, FDSK_EUNSUPPORTED, "B has more than 1024 rows");
  const size_t es = dtype_size(a_dt);
  if (es == 0) return set_err(owner, FDSK_EINVAL, "bad dtype");
  const void* Adev = A;
  void* stage = nullptr;
  int64_t ld = lda;
  if (mem == FDSK_MEM_HOST) {
    size_t bytes = static_cast<size_t>(n) * d * es;
    if (hipMalloc(&stage, bytes) != hipSuccess) return set_err(owner, FDSK_ENOMEM, "staging A");
    hipError_t e = hipMemcpy2DAsync(stage, d * es, A, lda * es, d * es, n, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
      (void)hipFree(stage);
      return set_err(owner, FDSK_EDEVICE, "copying A: %s", hipGetErrorString(e));
    }
    Adev = stage;
    ld = d;
  } else if (mem != FDSK_MEM_DEVICE) {
    return set_err(owner, FDSK_EINVAL, "bad mem kind");
  }
  EvalResult r{};
  const char* msg = "";
  hipError_t e = evaluate_device(Adev, static_cast<int>(a_dt), n, ld, Bdev, rows_b, ldb, d, k,
                                 method, st, &r, &msg);
  if (stage) {
    (void)hipStreamSynchronize(st);
    (void)hipFree(stage);
  }
  if (e != hipSuccess)
    return set_err(owner, e == hipErrorOutOfMemory ? FDSK_ENOMEM : FDSK_EDEVICE, "evaluator: %s: %s",
                   msg, hipGetErrorString(e));
  if (r.barrier_error) return set_err(owner, FDSK_EDEVICE, "evaluator: grid barrier timed out");
  if (!(r.fro2_A > 0.0)) return set_err(owner, FDSK_EINVAL, "||A||_F = 0: cov-err is undefined");
  out->cov_err = r.cov_err;
  out->proj_err_k = r.tail_k > 0.0 ? r.proj_err_k : std::nan("");
  out->proj_full_over_fro2 = r.proj_full;
  out->fro2_A = r.fro2_A;
  out->fro2_B = r.fro2_B;
  out->lambda_max = r.lambda_max;
  out->lambda_min = r.lambda_min;
  out->k = k;
  out->eig_unconverged += r.eig_unconverged;
  if (!(r.cov_err == r.cov_err)) return set_err(owner, FDSK_ENONFINITE, "non-finite error measure");
  return 0;
}

}  // namespace

extern "C" int sketch_error(fdsk_sketch* s, const void* A, int64_t n, int64_t lda, fdsk_dtype dtype,
                            fdsk_mem mem, int32_t k, int32_t method, fdsk_report* out) {
  if (!s || !A || !out) return set_err(s, FDSK_EINVAL, "null argument");
  if (s->err) return s->err;
  if (!s->finalized) return set_err(s, FDSK_ESTATE, "sketch_error needs a finalized sketch");
  int rc = sketch_stats(s, out);
  if (rc) return rc;
  return run_evaluator(s, A, n, lda, dtype, mem, s->C[s->cur], s->rows_out, s->ldc, s->d, k,
                       method, s->stream, out);
}

extern "C" int fdsk_evaluate(const void* A, int64_t n, int64_t lda, fdsk_dtype a_dtype,
                             const void* B, int64_t rows_b, int64_t ldb, fdsk_dtype b_dtype,
                             int64_t d, fdsk_mem mem, int32_t k, int32_t method, void* hip_stream,
                             fdsk_report* out) {
  if (!A || !out || (rows_b > 0 && !B)) return set_err(nullptr, FDSK_EINVAL, "null argument");
  if (d < 1 || d > 65536 || rows_b < 0 || (rows_b > 0 && ldb < d))
    return set_err(nullptr, FDSK_EINVAL, "bad sizes");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  std::memset(out, 0, sizeof *out);
  out->delta_sum = out->shrink_total = std::nan("");
  // B as FP64 on the device.
  const size_t esb = dtype_size(b_dtype);
  if (rows_b > 0 && (esb == 0 || b_dtype == FDSK_BF16))
    return set_err(nullptr, FDSK_EINVAL, "B must be F64 or F32");
  double* Bd = nullptr;
  size_t bbytes = static_cast<size_t>(std::max<int64_t>(rows_b, 1)) * d * 8;
  if (hipMalloc(&Bd, bbytes) != hipSuccess) return set_err(nullptr, FDSK_ENOMEM, "staging B");
  hipError_t e = hipSuccess;
  if (rows_b > 0) {
    if (b_dtype == FDSK_F64) {
      e = hipMemcpy2DAsync(Bd, d * 8, B, ldb * 8, d * 8, rows_b,
                           mem == FDSK_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, st);
    } else {
      const void* Bsrc = B;
      void* tmp = nullptr;
      if (mem == FDSK_MEM_HOST) {
        e = hipMalloc(&tmp, static_cast<size_t>(rows_b) * d * 4);
        if (e == hipSuccess)
          e = hipMemcpy2DAsync(tmp, d * 4, B, ldb * 4, d * 4, rows_b, hipMemcpyHostToDevice, st);
        Bsrc = tmp;
      }
      int64_t ld = (mem == FDSK_MEM_HOST) ? d : ldb;
      if (e == hipSuccess) e = launch_convert_f64(Bsrc, FDSK_F32, ld, rows_b, static_cast<int>(d), Bd, st);
      if (tmp) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(tmp);
      }
    }
  }
  int rc = 0;
  if (e != hipSuccess) {
    rc = set_err(nullptr, FDSK_EDEVICE, "staging B: %s", hipGetErrorString(e));
  } else {
    fdsk_report rep{};
    rc = run_evaluator(nullptr, A, n, lda, a_dtype, mem, Bd, rows_b, d, static_cast<int>(d), k,
                       method, st, &rep);
    rep.delta_sum = rep.shrink_total = std::nan("");
    rep.n_rows = n;
    rep.rows_out = static_cast<int32_t>(rows_b);
    *out = rep;
  }
  (void)hipStreamSynchronize(st);
  (void)hipFree(Bd);
  return rc;
}

namespace {
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() { if (p) (void)hipFree(p); }
};
}  // namespace

extern "C" int fdsk_gram(const double* C, int32_t rows, int64_t d, int64_t ldc, double* G,
                         int64_t ldg, fdsk_precision prec, void* hip_stream) {
  if (prec != FDSK_P_FP64 && prec != FDSK_P_BF16 && prec != FDSK_P_BF16X3 && prec != FDSK_P_FP8X3)
    return set_err(nullptr, FDSK_EINVAL, "fdsk_gram: unknown precision");
  if (!C || !G || rows < 1 || rows > 1024 || d < 1 || d > 65536 || ldc < d || ldg < rows)
    return set_err(nullptr, FDSK_EINVAL, "fdsk_gram: bad arguments");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int mp = round_up(rows, 32), ld = round_up(static_cast<int>(d), 64);
  const int T = mp / 32, ntiles = T * (T + 1) / 2;
  const int ks = std::max(1, std::min({(256 + ntiles - 1) / ntiles, ld / 256, 16}));
  DevBuf buf;
  const size_t nC = static_cast<size_t>(mp) * ld, nG = static_cast<size_t>(mp) * mp;
  const size_t q8b = (prec == FDSK_P_FP8X3) ? fp8_workspace_bytes(mp, ld)
                     : (prec != FDSK_P_FP64) ? bf16_workspace_bytes(mp, ld) : 0;
  if (hipMalloc(&buf.p, (nC + nG * (1 + ks)) * 8 + q8b) != hipSuccess)
    return set_err(nullptr, FDSK_ENOMEM, "fdsk_gram: workspace");
  double* Cp = static_cast<double*>(buf.p);
  double* Gp = Cp + nC;
  double* Gpart = Gp + nG;
  void* q8 = Gpart + nG * ks;
  HIPCHK(nullptr, hipMemsetAsync(Cp, 0, nC * 8, st));
  HIPCHK(nullptr, hipMemcpy2DAsync(Cp, ld * 8, C, ldc * 8, d * 8, rows, hipMemcpyDeviceToDevice, st));
  if (prec == FDSK_P_FP64)
    HIPCHK(nullptr, launch_gram(Cp, ld, mp, Gpart, ks, Gp, st));
  else if (prec == FDSK_P_FP8X3)
    HIPCHK(nullptr, launch_gram_fp8(Cp, ld, mp, q8, Gpart, ks, Gp, st));
  else
    HIPCHK(nullptr, launch_gram_lowp(Cp, ld, mp, Gpart, ks, Gp, prec == FDSK_P_BF16 ? 1 : 3, q8, st));
  HIPCHK(nullptr, hipMemcpy2DAsync(G, ldg * 8, Gp, mp * 8, rows * 8, rows, hipMemcpyDeviceToDevice, st));
  HIPCHK(nullptr, hipStreamSynchronize(st));
  return 0;
}

extern "C" int fdsk_eigh(const double* G, int32_t m, int64_t ldg, double* lam, double* V,
                         int64_t ldv, int32_t method, void* hip_stream) {
  if (!G || !lam || !V || m < 1 || ldg < m || ldv < m)
    return set_err(nullptr, FDSK_EINVAL, "fdsk_eigh: bad arguments");
  if (method != FDSK_EIG_AUTO && method != FDSK_EIG_JACOBI)
    return set_err(nullptr, FDSK_EINVAL, "fdsk_eigh: unknown method %d", (int)method);
  if (m > 1024) return set_err(nullptr, FDSK_EUNSUPPORTED, "fdsk_eigh: m > 1024");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int mp = round_up(m, 32);
  const size_t nG = static_cast<size_t>(mp) * mp;
  DevBuf buf;
  const size_t bytes = (6 * nG + mp) * 8 + sizeof(DevStats) + 4 * sizeof(unsigned) +
                       kMaxSweeps * sizeof(int) + 256;
  if (hipMalloc(&buf.p, bytes) != hipSuccess) return set_err(nullptr, FDSK_ENOMEM, "fdsk_eigh: workspace");
  HIPCHK(nullptr, hipMemsetAsync(buf.p, 0, bytes, st));
  double* Gp = static_cast<double*>(buf.p);
  double* Wp = Gp + nG;
  double* Vp = Wp + nG;
  double* Vt = Vp + nG;
  double* S1 = Vt + nG;
  double* S2 = S1 + nG;
  double* lp = S2 + nG;
  DevStats* ds = reinterpret_cast<DevStats*>(lp + mp);
  unsigned* bar = reinterpret_cast<unsigned*>(ds + 1);
  int* rot = reinterpret_cast<int*>(bar + 4);
  HIPCHK(nullptr, hipMemcpy2DAsync(Gp, mp * 8, G, ldg * 8, m * 8, m, hipMemcpyDeviceToDevice, st));
  EigWork wk{Wp, bar, rot, ds, S1, S2, method == FDSK_EIG_JACOBI ? EIG_JACOBI : EIG_AUTO};
  HIPCHK(nullptr, launch_eig(Gp, m, mp, lp, Vp, wk, st));
  // V is column-major inside the library; hand it out row-major.
  HIPCHK(nullptr, launch_transpose(Vp, mp, m, Vt, st));
  HIPCHK(nullptr, hipMemcpyAsync(lam, lp, m * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(nullptr, hipMemcpy2DAsync(V, ldv * 8, Vt, mp * 8, m * 8, m, hipMemcpyDeviceToDevice, st));
  DevStats h{};
  HIPCHK(nullptr, hipMemcpyAsync(&h, ds, sizeof h, hipMemcpyDeviceToHost, st));
  HIPCHK(nullptr, hipStreamSynchronize(st));
  if (h.bar_err) return set_err(nullptr, FDSK_EDEVICE, "fdsk_eigh: grid barrier timed out");
  return 0;
}
