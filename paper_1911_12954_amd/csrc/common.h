// Shared device/host helpers of libtrg (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

namespace trg {

// ---------------------------------------------------------------------------
// Errors: host code throws trg::Error; the C-ABI layer converts to codes.
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define TRG_HIP_CHECK(expr)                                                              \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::trg::Error(-3, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

#define TRG_REQUIRE(cond, msg)                                                           \
  do {                                                                                   \
    if (!(cond)) throw ::trg::Error(-1, msg);                                            \
  } while (0)

// ---------------------------------------------------------------------------
// Fast 32-bit unsigned division by a runtime-invariant divisor (round-up
// multiplier method of Granlund and Montgomery, 1994): q = (mulhi(n, mult) +
// n) >> shift with shift = ceil(log2 d) and mult = floor(2^32 (2^shift - d)
// / d) + 1; exact for all n < 2^32 and 1 <= d <= 2^31.
// ---------------------------------------------------------------------------
struct FastDiv {
  uint32_t d, mult, shift;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t s = 0;
  while ((uint64_t(1) << s) < d) ++s;
  f.shift = s;
  f.mult = uint32_t(((uint64_t(1) << 32) * ((uint64_t(1) << s) - d)) / d + 1);
  return f;
}

__host__ __device__ inline uint32_t fast_div(uint32_t n, const FastDiv &f) {
#ifdef __HIP_DEVICE_COMPILE__
  uint32_t hi = __umulhi(n, f.mult);
#else
  uint32_t hi = uint32_t((uint64_t(n) * f.mult) >> 32);
#endif
  return uint32_t((uint64_t(hi) + n) >> f.shift);
}

// ---------------------------------------------------------------------------
// bf16 split of an FP64 value: hi = RNE_bf16(float(a)), lo = RNE_bf16(float(a) - hi).
// ---------------------------------------------------------------------------
__device__ inline uint16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return uint16_t(u >> 16);
}

__device__ inline float bf16_to_f32(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

inline size_t round_up(size_t x, size_t m) { return (x + m - 1) / m * m; }

}  // namespace trg
