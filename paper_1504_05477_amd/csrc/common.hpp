// Shared definitions of the gfx950 Block Krylov library: element types,
// the device status word, launch helpers and the BF16 / OCP-e4m3 codecs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstddef>

#include "bk.h"

namespace bk {

using bf16_t = uint16_t;  // raw bfloat16 bits
using fp8_t = uint8_t;    // raw OCP e4m3 bits

// Device status word, one per solve, in the workspace.  Kernels raise flags
// with atomics; the host reads it once the stream has drained.
struct Ctrl {
  int32_t flags;        // CTRL_* bits
  int32_t q_eff;        // atomicMin'ed by the breakdown test
  int32_t csr_bad;      // CSR validation failures
  int32_t pad0;
  unsigned long long offmax;  // bit pattern of the largest relative
                              // off-diagonal seen in the current sweep
  unsigned long long pad1;
};

enum : int32_t {
  CTRL_RANK = 1,       // block 0 rank deficient
  CTRL_NONFINITE = 2,  // NaN / Inf in a Gram matrix
  CTRL_STALL = 4,      // a grid barrier gave up waiting (the device stalled)
};

#define BK_TRY(expr)                          \
  do {                                        \
    hipError_t _e = (expr);                   \
    if (_e != hipSuccess) return BK_EHIP;     \
  } while (0)

#define BK_TRY_LAUNCH()                                      \
  do {                                                       \
    hipError_t _e = hipGetLastError();                       \
    if (_e != hipSuccess) return BK_EHIP;                    \
  } while (0)

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------- codecs --
__host__ __device__ inline float bf16_to_f32(bf16_t v) {
  union {
    uint32_t u;
    float f;
  } c;
  c.u = static_cast<uint32_t>(v) << 16;
  return c.f;
}

// Round to nearest even; NaN stays a quiet NaN.
__host__ __device__ inline bf16_t f32_to_bf16(float x) {
  union {
    uint32_t u;
    float f;
  } c;
  c.f = x;
  if ((c.u & 0x7FFFFFFFu) > 0x7F800000u) return 0x7FC0;
  uint32_t r = c.u + 0x7FFFu + ((c.u >> 16) & 1u);
  return static_cast<bf16_t>(r >> 16);
}

// OCP e4m3 (bias 7, no infinities, 0x7F / 0xFF = NaN, largest finite 448).
__host__ __device__ inline float e4m3_to_f32(fp8_t v) {
  const uint32_t s = (v & 0x80u) << 24;
  const uint32_t e = (v >> 3) & 0xFu;
  const uint32_t m = v & 0x7u;
  union {
    uint32_t u;
    float f;
  } c;
  if (e == 15u && m == 7u) {
    c.u = 0x7FC00000u | s;
  } else if (e == 0u) {
    c.f = static_cast<float>(m) * 0.001953125f;  // m * 2^-9
    c.u |= s;
  } else {
    c.u = s | ((e + 120u) << 23) | (m << 20);  // (e - 7 + 127)
  }
  return c.f;
}

// Round to nearest even, saturating to +-448 (never produces NaN from a
// finite input).
__host__ __device__ inline fp8_t f32_to_e4m3(float x) {
  union {
    uint32_t u;
    float f;
  } c;
  c.f = x;
  const uint8_t s = static_cast<uint8_t>((c.u >> 24) & 0x80u);
  const float a = fabsf(x);
  if (!(a == a)) return 0x7F;
  if (a >= 448.0f) return s | 0x7E;
  if (a < 0.015625f) {  // below the smallest normal 2^-6: units of 2^-9
    float qv = rintf(a * 512.0f);
    return s | static_cast<uint8_t>(qv);  // 8 -> 0x08 = 2^-6, still right
  }
  union {
    uint32_t u;
    float f;
  } b;
  b.f = a;
  uint32_t r = b.u + 0x7FFFFu + ((b.u >> 20) & 1u);  // RNE to 3 mantissa bits
  uint32_t e = (r >> 23) - 120u;                      // -127 + 7
  uint32_t m = (r >> 20) & 7u;
  if (e > 15u || (e == 15u && m > 6u)) return s | 0x7E;
  return static_cast<uint8_t>(s | (e << 3) | m);
}

// Element loaders used by the generic (VALU) kernels.
template <typename T>
struct Elem;
template <>
struct Elem<double> {
  __device__ static double load(const double* p, int64_t i) { return p[i]; }
};
template <>
struct Elem<float> {
  __device__ static float load(const float* p, int64_t i) { return p[i]; }
};
template <>
struct Elem<bf16_t> {
  __device__ static float load(const bf16_t* p, int64_t i) {
    return bf16_to_f32(p[i]);
  }
};
template <>
struct Elem<fp8_t> {
  __device__ static float load(const fp8_t* p, int64_t i) {
    return e4m3_to_f32(p[i]);
  }
};

// Non-negative doubles order like their bit patterns: atomicMax on the bits.
__device__ inline void atomic_max_nonneg(unsigned long long* p, double v) {
  if (!(v >= 0.0)) v = 1.0e300;  // NaN counts as "not converged"
  atomicMax(p, static_cast<unsigned long long>(__double_as_longlong(v)));
}

}  // namespace bk
