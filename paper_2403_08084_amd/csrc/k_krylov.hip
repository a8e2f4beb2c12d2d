// Multi-vector Krylov pass for FGMRES (classical Gram-Schmidt).
//
// One pass streams a set of basis vectors V_0..V_{nv-1} and the vector w once:
//   optionally  w <- w - sum_k c_k V_k          (projection / combination)
//   optionally  d_k = V_k . w                   (projection coefficients)
//   always      |w|^2
// so a classical Gram-Schmidt step with re-orthogonalisation costs two or three
// streaming passes over the basis, each fusing the axpy of one projection with
// the dot products of the next. Reductions are deterministic: every block
// reduces its share in a fixed order (wavefront shuffles, then LDS), writes one
// partial row, and the last block to finish (device-scope counter) sums the
// partial rows in block order and writes the results, the optional inverse norm
// and the optional re-orthogonalisation flag. No floating-point atomics.
#include "irk_internal.h"

namespace irk {
namespace {

constexpr int NT = 256;
constexpr int NW = NT / 64;
constexpr int kStride = kMaxRestart + 1;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

template <int MAXV>
__global__ __launch_bounds__(NT) void ortho_kernel(OrthoArgs a, ReduceWork rw) {
  if (a.skip && *a.skip == 0) return;
  const int nv = a.nv;
  const bool do_axpy = a.coef != nullptr;
  const bool do_dots = a.want_dots != 0;
  double c[MAXV];
#pragma unroll
  for (int k = 0; k < MAXV; ++k) {
    double v = 0.0;
    if (do_axpy && k < nv) v = a.coef_sign * a.coef[k] * (a.vscale ? a.vscale[k] : 1.0);
    c[k] = v;
  }
  double d[MAXV];
#pragma unroll
  for (int k = 0; k < MAXV; ++k) d[k] = 0.0;
  double nrm = 0.0;
  const long stride = (long)gridDim.x * NT;
  for (long q = (long)blockIdx.x * NT + threadIdx.x; q < a.len; q += stride) {
    double wv = a.w[q];
    if (do_axpy) {
      double v[MAXV];
#pragma unroll
      for (int k = 0; k < MAXV; ++k)
        if (k < nv) v[k] = a.V[k * a.vstride + q];
#pragma unroll
      for (int k = 0; k < MAXV; ++k)
        if (k < nv) wv -= c[k] * v[k];
      a.w[q] = wv;
      if (do_dots) {
#pragma unroll
        for (int k = 0; k < MAXV; ++k)
          if (k < nv) d[k] += v[k] * wv;
      }
    } else if (do_dots) {
#pragma unroll
      for (int k = 0; k < MAXV; ++k)
        if (k < nv) d[k] += a.V[k * a.vstride + q] * wv;
    }
    nrm += wv * wv;
  }
  // block reduction: wavefront shuffle, then across the NW wavefronts
  __shared__ double red[(MAXV + 1) * NW];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < MAXV; ++k) {
    if (k < nv && do_dots) {
      const double s = wave_sum(d[k]);
      if (lane == 0) red[k * NW + wid] = s;
    }
  }
  {
    const double s = wave_sum(nrm);
    if (lane == 0) red[MAXV * NW + wid] = s;
  }
  __syncthreads();
  double* part = rw.partial + (long)blockIdx.x * kStride;
  for (int k = threadIdx.x; k <= nv; k += NT) {
    const int slot = (k == nv) ? MAXV : k;
    if (k < nv && !do_dots) {
      part[k] = 0.0;
      continue;
    }
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[slot * NW + w];
    part[k] = s;
  }
  __threadfence();
  __shared__ int is_last;
  if (threadIdx.x == 0) is_last = (atomicAdd(rw.counter, 1u) == gridDim.x - 1);
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  const int nb = gridDim.x;
  for (int k = threadIdx.x; k <= nv; k += NT) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += rw.partial[(long)b * kStride + k];
    if (k < nv) {
      a.result[k] = s * (a.vscale ? a.vscale[k] : 1.0);
    } else {
      a.result[nv] = s;
      if (a.sigma_out) *a.sigma_out = 1.0 / sqrt(s);
      if (a.flag_out) *a.flag_out = (s < a.eta2 * (*a.ref)) ? 1 : 0;
    }
  }
  if (threadIdx.x == 0) *rw.counter = 0u;
}

}  // namespace

void launch_ortho(const OrthoArgs& a, const ReduceWork& rw, hipStream_t st) {
  long blocks = (a.len + NT - 1) / NT;
  if (blocks > rw.max_blocks) blocks = rw.max_blocks;
  if (blocks < 1) blocks = 1;
  const int nb = (int)blocks;
  if (a.nv <= 0) {
    ortho_kernel<1><<<nb, NT, 0, st>>>(a, rw);
  } else if (a.nv <= 8) {
    ortho_kernel<8><<<nb, NT, 0, st>>>(a, rw);
  } else if (a.nv <= 16) {
    ortho_kernel<16><<<nb, NT, 0, st>>>(a, rw);
  } else {
    ortho_kernel<32><<<nb, NT, 0, st>>>(a, rw);
  }
}

}  // namespace irk
