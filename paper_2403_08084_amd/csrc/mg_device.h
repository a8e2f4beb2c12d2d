// Device helpers shared by the multigrid kernel files: storage conversions
// (FP64 / FP32 / BF16 with round-to-nearest-even), the interior-node test and
// bilinear prolongation of a coarse correction.
#pragma once

#include "irk_internal.h"

namespace irk {
namespace {

__device__ __forceinline__ float bf2f(uint16_t u) { return __uint_as_float(((uint32_t)u) << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest even (inputs are finite)
  uint32_t b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

// 1/x for the smoothers' diagonal scalings: v_rcp_f32 (within 1 ulp) in the FP32 compute type, where the
// correctly rounded division costs about ten instructions; exact division in FP64
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

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
  // a 32-bit element offset from the (uniform) base, then constant offsets from the two row pointers: the
  // compiler can pair the loads of horizontally adjacent values
  const TS* q0 = e + ((unsigned)(j >> 1) * (unsigned)pc + (unsigned)(i >> 1));
  const TS* q1 = q0 + pc;
  const TC e00 = ld<TC>(q0), e10 = ld<TC>(q0 + 1), e01 = ld<TC>(q1), e11 = ld<TC>(q1 + 1);
  const TC wx = (i & 1) ? (TC)0.5 : (TC)0, wy = (j & 1) ? (TC)0.5 : (TC)0;
  return ((TC)1 - wx) * ((TC)1 - wy) * e00 + wx * ((TC)1 - wy) * e10 + ((TC)1 - wx) * wy * e01 + wx * wy * e11;
}

// Tile loads are staged through registers with fully unrolled loops, so every
// thread has all of its global loads in flight before the first LDS store.
template <typename TC, typename TK, int KX, int KY, int NT>
__device__ __forceinline__ void load_kappa_tile(TC* sK, const TK* __restrict__ kap, int ox, int oy, const Geom& g) {
  constexpr int CNT = KX * KY, NL = (CNT + NT - 1) / NT;
  TC v[NL];
#pragma unroll
  for (int r = 0; r < NL; ++r) {
    const int idx = threadIdx.x + r * NT;
    const int b = idx / KX, a = idx - b * KX;
    const int ex = ox - 1 + a, ey = oy - 1 + b;
    const bool ok = idx < CNT && ex >= 0 && ex < g.N && ey >= 0 && ey < g.N;
    // unconditional load from a clamped address keeps all loads in flight; the select zeroes the rest
    const TC val = (TC)kap[ok ? (unsigned)ey * g.pitch + ex : 0u];
    v[r] = ok ? val : (TC)0;
  }
#pragma unroll
  for (int r = 0; r < NL; ++r) {
    const int idx = threadIdx.x + r * NT;
    if (idx < CNT) sK[idx] = v[r];
  }
}

}  // namespace
}  // namespace irk
