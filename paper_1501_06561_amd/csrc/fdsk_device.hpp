// Device-side helpers shared by the FD-family kernels (gfx950 / CDNA4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));

namespace fdsk {

// Row dtypes accepted at the boundary (mirrors fdsk_dtype in fdsketch.h).
enum { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2 };

__device__ __forceinline__ double load_as_f64(const void* p, int64_t i, int dt) {
  if (dt == DT_F64) return static_cast<const double*>(p)[i];
  if (dt == DT_F32) return static_cast<double>(static_cast<const float*>(p)[i]);
  uint32_t b = static_cast<uint32_t>(static_cast<const uint16_t*>(p)[i]) << 16;
  return static_cast<double>(__uint_as_float(b));
}

// Round-to-nearest-even float -> bfloat16 bits.
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) {
  return __uint_as_float(static_cast<uint32_t>(b) << 16);
}
// The split-BF16 halves of a double: hi = bf16(float(x)), lo = bf16(float(x - hi)).
__device__ __forceinline__ void split_bits(double x, uint16_t& hb, uint16_t& lb) {
  hb = f32_to_bf16_bits(static_cast<float>(x));
  lb = f32_to_bf16_bits(static_cast<float>(x - static_cast<double>(bf16_bits_to_f32(hb))));
}

// Data-parallel-primitive (DPP) move of a double: both 32-bit halves go
// through the same lane permutation.  Lanes whose row is masked off (or whose
// source does not exist) get `old`.
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ double dpp_f64(double v, double old) {
  const long long u = __double_as_longlong(v), o = __double_as_longlong(old);
  const int lo = __builtin_amdgcn_update_dpp(static_cast<int>(o), static_cast<int>(u), CTRL, ROWMASK,
                                             0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(static_cast<int>(o >> 32), static_cast<int>(u >> 32), CTRL,
                                             ROWMASK, 0xF, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<long long>(static_cast<unsigned>(lo)));
}

// The same move for a control that writes every lane (a quad permutation or
// a row mirror, all rows and banks enabled): no lane keeps an old value, so
// none is supplied and the compiler does not have to initialise one.
template <int CTRL>
__device__ __forceinline__ double dpp_perm_f64(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(u), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<long long>(static_cast<unsigned>(lo)));
}

// Sum over each quad of lanes (4i .. 4i+3); every lane of the quad gets it.
__device__ __forceinline__ double quad_sum(double v) {
  v += dpp_perm_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_perm_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  return v;
}
__device__ __forceinline__ double quad_prod(double v) {
  v *= dpp_perm_f64<0xB1>(v);
  v *= dpp_perm_f64<0x4E>(v);
  return v;
}

// Sum over each row of 16 lanes, returned in every lane of the row (a
// butterfly: each step adds the same two operands on both partners, so the
// 16 results are bitwise equal).
__device__ __forceinline__ double row16_sum(double v) {
  v = quad_sum(v);
  v += dpp_perm_f64<0x141>(v);          // row_half_mirror
  v += dpp_perm_f64<0x140>(v);          // row_mirror
  return v;
}

// Wave-wide (64 lanes, all active) sum, returned in every lane: quad
// butterflies and row mirrors give each row of 16 its total, two row
// broadcasts accumulate the rows into lane 63, which is read back.
__device__ __forceinline__ double wave_sum(double v) {
  v = quad_sum(v);
  v += dpp_perm_f64<0x141>(v);          // row_half_mirror
  v += dpp_perm_f64<0x140>(v);          // row_mirror
  v += dpp_f64<0x142, 0xA>(v, 0.0);     // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xC>(v, 0.0);     // row_bcast:31 into rows 2 and 3
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(u), 63);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(u >> 32), 63);
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<long long>(static_cast<unsigned>(lo)));
}

// 16x16x4 FP64 matrix-core step: D(16x16) += A(16x4) * B(4x16).
// Lane layout (wave64): lane = i + 16*k holds A[i][k] and B[k][i];
// the result lane = j + 16*q holds D[q + 4v][j] in element v (rows of a lane
// group are interleaved by 4 for the FP64 instruction).
__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Grid-wide barrier for a cooperatively launched grid.  Generation counter
// scheme: counters return to zero at every completed barrier, so the pair can
// be reused by later launches without a reset.  The spin is bounded: on
// timeout an error bit is set and the wave proceeds, so the grid always drains.
struct GridBar {
  unsigned* count;
  unsigned* gen;
  int* err;
};

__device__ __forceinline__ void grid_barrier(const GridBar& b, unsigned nblocks) {
  // Every wave waits for its own stores to complete (they are then in L2);
  // one thread publishes the workgroup's writes to the device with an
  // agent-scope release, arrives, waits, and acquires (which also drops stale
  // lines of this CU's caches for every wave of the workgroup).
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned g = __hip_atomic_load(b.gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned arrived = __hip_atomic_fetch_add(b.count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(b.count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(b.gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      // Once any barrier has timed out every later one falls through at once.
      long spins = 0;
      while (__hip_atomic_load(b.gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 1023) == 0 &&
            __hip_atomic_load(b.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
          break;
        if (spins > (1L << 25)) {
          __hip_atomic_fetch_or(b.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
    }
    __threadfence();
  }
  __syncthreads();
}

// Reciprocal and reciprocal square root from the hardware estimates refined
// by two Newton steps (each doubles the correct bits), in place of the longer
// IEEE-exact division and square-root sequences.  Arguments are >= 1 or
// well inside the normal range where they are used.
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}

// Stable Jacobi rotation (Rutishauser) annihilating the (p,q) entry of the
// symmetric 2x2 [[app, apq], [apq, aqq]]:  J = [[c, s], [-s, c]], and
// J^T [[app, apq],[apq, aqq]] J is diagonal.  With zeta = (aqq-app)/(2 apq),
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)) is the smaller root of
// t^2 + 2 zeta t - 1 = 0, c = 1/sqrt(1+t^2), s = t c.
__device__ __forceinline__ void jacobi_rotation(double app, double aqq, double apq,
                                                double& c, double& s) {
  if (apq == 0.0) { c = 1.0; s = 0.0; return; }
  const double diff = aqq - app;
  double t;
  if (fabs(diff) > 1e150 * fabs(apq)) {
    t = apq / diff;                       // |zeta| huge: t -> 1/(2 zeta)
  } else {
    const double zeta = diff * rcp_nr(2.0 * apq);
    const double z2 = fma(zeta, zeta, 1.0);
    const double w = z2 * rsq_nr(z2);    // sqrt(1 + zeta^2)
    t = rcp_nr(fabs(zeta) + w);
    if (zeta < 0.0) t = -t;
  }
  c = rsq_nr(fma(t, t, 1.0));
  s = t * c;
}

}  // namespace fdsk
