// Device helpers shared by the multigrid kernel files: storage conversions
// (FP64 / FP32 / BF16 with round-to-nearest-even), the interior-node test and
// bilinear prolongation of a coarse correction.
#pragma once

#include "irk_internal.h"

namespace irk {
namespace {

constexpr int NT = 256;

__device__ __forceinline__ float bf2f(uint16_t u) { return __uint_as_float(((uint32_t)u) << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest even (inputs are finite)
  uint32_t b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

template <typename TC>
__device__ __forceinline__ TC ld(const double* p) { return (TC)*p; }
template <typename TC>
__device__ __forceinline__ TC ld(const float* p) { return (TC)*p; }
template <typename TC>
__device__ __forceinline__ TC ld(const bf16* p) { return (TC)bf2f(p->u); }

__device__ __forceinline__ void st(double* p, double v) { *p = v; }
__device__ __forceinline__ void st(double* p, float v) { *p = (double)v; }
__device__ __forceinline__ void st(float* p, float v) { *p = v; }
__device__ __forceinline__ void st(float* p, double v) { *p = (float)v; }
__device__ __forceinline__ void st(bf16* p, float v) { p->u = f2bf(v); }
__device__ __forceinline__ void st(bf16* p, double v) { p->u = f2bf((float)v); }

__device__ __forceinline__ bool interior(int i, int j, int N) { return i >= 1 && i <= N - 1 && j >= 1 && j <= N - 1; }

// bilinear interpolation of the coarse correction at fine interior node (i, j):
// weights 1, 1/2, 1/4 by parity; all four coarse values are loaded (always in bounds)
template <typename TS, typename TC>
__device__ __forceinline__ TC prolong_at(const TS* __restrict__ e, int pc, int i, int j) {
  const TS* b = e + (long)(j >> 1) * pc + (i >> 1);
  const TC e00 = ld<TC>(b), e10 = ld<TC>(b + 1), e01 = ld<TC>(b + pc), e11 = ld<TC>(b + pc + 1);
  const TC wx = (i & 1) ? (TC)0.5 : (TC)0, wy = (j & 1) ? (TC)0.5 : (TC)0;
  return ((TC)1 - wx) * ((TC)1 - wy) * e00 + wx * ((TC)1 - wy) * e10 + ((TC)1 - wx) * wy * e01 + wx * wy * e11;
}

}  // namespace
}  // namespace irk
