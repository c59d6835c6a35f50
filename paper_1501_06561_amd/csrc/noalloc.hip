// fdsk_eigh_noalloc: the eigensolve entry point without device allocation
// (see include/fdsketch.h).  Its workspace is the file-scope device array
// `scratch` below.  In host code that name is only a stand-in for the
// device symbol, so it is never passed anywhere: on the first call on each
// device (with that device current) its device address is looked up with
// hipGetSymbolAddress and kept per device, and only that address reaches the
// kernels.  Every call on one GPU shares the array and leaves its contents
// behind; what must start at zero is cleared by a fill kernel on the
// caller's stream (no hipMemsetAsync, so the call can be captured into a
// HIP graph).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>

#include "fdsk_kernels.hpp"
#include "fdsketch.h"

using namespace fdsk;

namespace {

constexpr size_t kScratchBytes = FDSK_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

__global__ void k_fill_zero(double* __restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Device address of this device's scratch array (looked up once per device).
hipError_t scratch_ptr(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

int fail(int code, const char* msg) {
  set_last_error(msg);
  return code;
}

// Bytes of scratch one call on m rows uses.
size_t eigh_noalloc_bytes(int32_t m) {
  if (m < 1) return 0;
  const size_t mp = static_cast<size_t>((m + 31) / 32 * 32);
  const size_t nG = mp * mp;
  return align256(6 * nG * 8) + align256(mp * 8) + align256(sizeof(DevStats)) + align256(4 * sizeof(unsigned)) +
         align256(kMaxSweeps * sizeof(int));
}

}  // namespace

extern "C" int fdsk_eigh_noalloc(const double* G, int32_t m, int64_t ldg, double* lam, double* V, int64_t ldv,
                                 void* hip_stream) {
  if (!G || !lam || !V || m < 1 || ldg < m || ldv < m) return fail(FDSK_EINVAL, "fdsk_eigh_noalloc: bad arguments");
  if (m > FDSK_NOALLOC_EIGH_MAX) return fail(FDSK_EUNSUPPORTED, "fdsk_eigh_noalloc: m above the scratch limit");
  const size_t need = eigh_noalloc_bytes(m);
  if (need > kScratchBytes) return fail(FDSK_EUNSUPPORTED, "fdsk_eigh_noalloc: scratch too small");
  void* base = nullptr;
  hipError_t e = scratch_ptr(&base);
  if (e != hipSuccess) return fail(FDSK_EDEVICE, "fdsk_eigh_noalloc: scratch symbol lookup failed");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int mp = (m + 31) / 32 * 32;
  const size_t nG = static_cast<size_t>(mp) * mp;
  char* c = static_cast<char*>(base);
  double* Gp = reinterpret_cast<double*>(c);
  double* Wp = Gp + nG;
  double* Vp = Wp + nG;
  double* Vt = Vp + nG;
  double* S1 = Vt + nG;
  double* S2 = S1 + nG;
  size_t off = align256(6 * nG * 8);
  double* lp = reinterpret_cast<double*>(c + off);
  off += align256(mp * 8);
  DevStats* ds = reinterpret_cast<DevStats*>(c + off);
  off += align256(sizeof(DevStats));
  unsigned* bar = reinterpret_cast<unsigned*>(c + off);
  off += align256(4 * sizeof(unsigned));
  int* rot = reinterpret_cast<int*>(c + off);
  // The previous call's contents are still there: clear the whole region
  // this call uses (padding of G and V, statistics) with a fill kernel.
  const size_t nd = need / 8;
  hipLaunchKernelGGL(k_fill_zero, dim3(static_cast<unsigned>(std::min<size_t>((nd + 255) / 256, 2048))),
                     dim3(256), 0, st, reinterpret_cast<double*>(base), nd);
  e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(Gp, mp * 8, G, ldg * 8, m * 8, m, hipMemcpyDeviceToDevice, st);
  EigWork wk{Wp, bar, rot, ds, S1, S2, EIG_AUTO};
  if (e == hipSuccess) e = launch_eig(Gp, m, mp, lp, Vp, wk, st);
  // V is column-major inside the library; hand it out row-major.
  if (e == hipSuccess) e = launch_transpose(Vp, mp, m, Vt, st);
  if (e == hipSuccess) e = hipMemcpyAsync(lam, lp, m * 8, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpy2DAsync(V, ldv * 8, Vt, mp * 8, m * 8, m, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return fail(FDSK_EDEVICE, "fdsk_eigh_noalloc: launch failed");
  return 0;
}
