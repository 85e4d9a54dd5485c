// Internal helpers shared by the gfx950 kernels and the host runtime of the
// Lanczos GW self-energy library.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "gwl.h"

namespace gwl {

// ---------------------------------------------------------------- errors
// Thread-local message returned by gwl_last_error().
void set_error(const std::string& msg);

struct Error {
  gwl_status code;
  std::string msg;
};

#define GWL_HIP(call)                                                            \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess)                                                        \
      throw ::gwl::Error{GWL_EDEVICE, std::string(#call) + ": " +                \
                                          hipGetErrorString(e_)};                \
  } while (0)

#define GWL_CHECK(cond, code, msg)                                               \
  do {                                                                           \
    if (!(cond)) throw ::gwl::Error{(code), (msg)};                              \
  } while (0)

// ---------------------------------------------------------------- types
typedef uint16_t bf16_t;  // raw bfloat16 bits

__host__ __device__ inline bf16_t f32_to_bf16(float f) {
  // round to nearest even; inputs here are finite
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (bf16_t)(u >> 16);
}

__host__ __device__ inline float bf16_to_f32(bf16_t h) {
  uint32_t u = ((uint32_t)h) << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

// raw IEEE binary16 bits (a distinct type so that overloads can tell it from
// bfloat16); conversions round to nearest even
struct f16_t {
  uint16_t bits;
};

__host__ __device__ inline f16_t f32_to_f16(float f) {
  const _Float16 h = (_Float16)f;
  f16_t r;
  __builtin_memcpy(&r.bits, &h, 2);
  return r;
}

__host__ __device__ inline float f16_to_f32(f16_t v) {
  _Float16 h;
  __builtin_memcpy(&h, &v.bits, 2);
  return (float)h;
}

// Power-of-two scale of the second GEMM's FP16 operand phi_v(r) V_b(r) for
// one pair vector b: with vmax >= max_r |V_b(r)| and pmax = max |phi_v| (both
// as stored, i.e. with their own scales), vmax = m_v 2^ev and pmax = m_p 2^ep
// (m in [0.5, 1)), the scale 2^(14 - ev - ep) keeps every product below 2^14,
// inside FP16's range.  Returns the exponent.
__host__ __device__ inline int f16_operand_exp(float vmax, int ep) {
  int ev = 0;
  if (vmax > 0.0f && vmax <= 3.0e38f) (void)frexpf(vmax, &ev);
  int e = 14 - ev - ep;
  return e < -100 ? -100 : (e > 100 ? 100 : e);
}

template <typename T>
struct cplx {
  T x, y;
};

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }
inline long round_up(long a, long b) { return ((a + b - 1) / b) * b; }

constexpr double kHartreeEv = 27.211386245988;  // CODATA 2018
constexpr double kPi = 3.14159265358979323846;

}  // namespace gwl
