// Shared definitions of the libdk HIP sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

namespace dk {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kFdRadius = 6;  // twelfth-order central differences

// Sticky device error bits (OR-ed by kernels, checked by the host at the end of a call).
enum : unsigned {
  kErrNotSpd = 1u,
  kErrNonFinite = 2u,
  kErrFermi = 4u,
  kErrConvergence = 8u,
  kErrDegree = 16u,  // host-detected: the degree tail rule found no degree
};

// Degree of the density-kernel expansion when the caller passes n_pl = 0: the
// first of 32, 64, ... whose coefficient tail sum_{n < j <= 4n} |c_j(mu)| is
// at most kTailTol at that degree's Fermi level.
constexpr int kTailStart = 32;
constexpr int kTailCap = 256;
constexpr double kTailTol = 1e-12;

// Pulay mixing: at most this many stored difference pairs; the normal
// equations carry a shift kPulayReg * trace / m.
constexpr int kPulayMaxHistory = 8;
constexpr double kPulayReg = 1e-12;

inline int ceil_div(long a, long b) { return int((a + b - 1) / b); }

// -------------------------------------------------------------- MFMA --

// D(16x16) += A(16x4) B(4x16), FP64.  Lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; register r of lane l holds D[l/16 + 4r][l%16] (measured on
// gfx950: the FP64 form interleaves rows, unlike the FP32 forms below).
__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Same shape, FP32: register r of lane l holds D[4*(l/16) + r][l%16].
__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// D(16x16) += A(16x32) B(32x16), BF16 inputs, FP32 accumulation.  Lane l
// supplies A[l%16][8*(l/16)+v] and B[8*(l/16)+v][l%16] for v = 0..7; the
// output layout is that of the 16x16x4 forms.
__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Round-to-nearest-even float -> bf16 (finite inputs).
__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }

// x = hi + mid + lo + O(2^-24 |x|) with each piece representable in bf16.
__device__ __forceinline__ void split3_bf16(float x, __bf16& hi, __bf16& mid, __bf16& lo) {
  hi = (__bf16)x;
  const float r = x - (float)hi;
  mid = (__bf16)r;
  lo = (__bf16)(r - (float)mid);
}

// x = hi + lo + O(2^-16 |x|) with hi, lo representable in bf16.
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = to_bf16(x);
  lo = to_bf16(x - (float)hi);
}

}  // namespace dk
