// Multi-vector Krylov passes for FGMRES: classical Gram-Schmidt with re-orthogonalisation (CGS2),
// and its delayed one-reduction form (DCGS2).
//
// One pass streams a set of basis vectors V_0..V_{nv-1} and the vector w once:
//   optionally  w <- w - sum_k c_k V_k          (projection / combination)
//   optionally  d_k = V_k . w                   (projection coefficients)
//   always      |w|^2
// so a classical Gram-Schmidt step with re-orthogonalisation costs two or three
// streaming passes over the basis, each fusing the axpy of one projection with
// the dot products of the next. The vector count is a compile-time parameter
// (one instantiation per count and mode) so every loop unrolls without
// guards and each thread keeps all of its loads in flight.
//
// Reductions are deterministic: every block reduces its share in a fixed order
// (wavefront shuffles, then LDS) and writes one partial per value; a one-block
// finishing kernel sums the partials with all its threads in a fixed strided
// order followed by the same tree, and writes the results, the optional inverse
// norm and the optional re-orthogonalisation flag. No atomics, no fences.
#include <hip/hip_ext.h>

#include "irk_internal.h"

namespace irk {
namespace {

constexpr int NT = 256;
constexpr int NW = NT / 64;

enum Mode { NORM = 0, DOTS = 1, AXPY_DOTS = 2, AXPY = 3 };

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Reduce vals[0..CNT) over the block into out_smem[0..CNT) (fixed order).
template <int CNT>
__device__ __forceinline__ void block_reduce(const double (&vals)[CNT], double* red, double* out_smem) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < CNT; ++k) {
    const double s = wave_sum(vals[k]);
    if (lane == 0) red[k * NW + wid] = s;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < CNT; k += NT) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[k * NW + w];
    out_smem[k] = s;
  }
  __syncthreads();
}

template <int NV, int MODE, int U, bool VF>
__device__ __forceinline__ void process(const OrthoArgs& a, const double (&c)[NV > 0 ? NV : 1], long q0, long stride,
                                        double (&acc)[NV + 1]) {
  constexpr bool AX = (MODE == AXPY_DOTS || MODE == AXPY);
  constexpr bool DT = (MODE == AXPY_DOTS || MODE == DOTS);
  constexpr bool NEEDV = AX || DT;
  constexpr int NVV = NV > 0 ? NV : 1;
  double wv[U];
  double v[U][NVV];
#pragma unroll
  for (int u = 0; u < U; ++u) wv[u] = (AX && a.assign) ? 0.0 : a.w[q0 + u * stride];
  if (NEEDV) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NV; ++k)
        v[u][k] = VF ? (double)a.Vf[k * a.vstride + q0 + u * stride] : a.V[k * a.vstride + q0 + u * stride];
  }
  if (AX) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int k = 0; k < NV; ++k) wv[u] -= c[k] * v[u][k];
      a.w[q0 + u * stride] = wv[u];
    }
  }
  if (DT) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NV; ++k) acc[k] += v[u][k] * wv[u];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) acc[NV] += wv[u] * wv[u];
}

template <int NV, int MODE, bool VF>
__global__ __launch_bounds__(NT) void ortho_kernel(OrthoArgs a, ReduceWork rw) {
  if (a.skip && *a.skip == 0) return;
  constexpr bool AX = (MODE == AXPY_DOTS || MODE == AXPY);
  constexpr int NVV = NV > 0 ? NV : 1;
  constexpr int U = NV <= 2 ? 4 : (NV <= 8 ? 2 : 1);
  double c[NVV];
#pragma unroll
  for (int k = 0; k < NVV; ++k) c[k] = (AX && k < NV) ? a.coef_sign * a.coef[k] * (a.vscale ? a.vscale[k] : 1.0) : 0.0;
  double acc[NV + 1];
#pragma unroll
  for (int k = 0; k <= NV; ++k) acc[k] = 0.0;
  const long stride = (long)gridDim.x * NT;
  const long len = a.len;
  long q0 = (long)blockIdx.x * NT + threadIdx.x;
  for (; q0 + (U - 1) * stride < len; q0 += U * stride) process<NV, MODE, U, VF>(a, c, q0, stride, acc);
  for (; q0 < len; q0 += stride) process<NV, MODE, 1, VF>(a, c, q0, stride, acc);

  __shared__ double red[(NV + 1) * NW];
  __shared__ double tot[NV + 1];
  block_reduce<NV + 1>(acc, red, tot);
  const int mb = rw.max_blocks;
  for (int k = threadIdx.x; k <= NV; k += NT) rw.partial[(long)k * mb + blockIdx.x] = tot[k];
}

// Second stage (one block of NF threads, nb <= NF): thread b loads partial b of every value,
// then a fixed-order tree. The kernel boundary makes the partials visible, so no device-scope
// fence (which would write back and invalidate the L2 of every block's XCD) is needed.
constexpr int NF = 1024;
constexpr int NFW = NF / 64;

template <int NV>
__global__ __launch_bounds__(NF) void finish_kernel(OrthoArgs a, ReduceWork rw, int nb) {
  if (a.skip && *a.skip == 0) return;
  const int mb = rw.max_blocks;
  const int b = threadIdx.x;
  double fin[NV + 1];
#pragma unroll
  for (int k = 0; k <= NV; ++k) fin[k] = rw.partial[(long)k * mb + (b < nb ? b : 0)];
#pragma unroll
  for (int k = 0; k <= NV; ++k)
    if (b >= nb) fin[k] = 0.0;
  __shared__ double red[(NV + 1) * NFW];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k <= NV; ++k) {
    const double s = wave_sum(fin[k]);
    if (lane == 0) red[k * NFW + wid] = s;
  }
  __syncthreads();
  for (int k = threadIdx.x; k <= NV; k += NF) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NFW; ++w) s += red[k * NFW + w];
    if (k < NV) {
      a.result[k] = s * (a.vscale ? a.vscale[k] : 1.0);
    } else {
      a.result[NV] = s;
      if (a.sigma_out) *a.sigma_out = 1.0 / sqrt(s);
      if (a.flag_out) *a.flag_out = (s < a.eta2 * (*a.ref)) ? 1 : 0;
    }
  }
}

// ---------------------------------------------------------------- DCGS2
//
// Delayed CGS2 (Swirydowicz, Langou, Ananthan, Yang and Thomas, "Low synchronization Gram-Schmidt and
// GMRES algorithms", Numer. Linear Algebra Appl. 2021): at Arnoldi step j the new direction w and the
// previous direction u (projected once, not yet re-orthogonalised or normalised) are treated together,
// one reduction giving Q^T u, Q^T w, u.u, u.w, w.w; u is then re-orthogonalised and normalised into
// q_j and w projected against Q and q_j in one streaming update pass.

constexpr int NF2 = 1024;  // threads of the DCGS2 finishing kernel (one wave per reduced value)

template <int NV, int U>
__device__ __forceinline__ void process2(const D2Args& a, long q0, long stride, double (&acc)[2 * NV + 3]) {
  double uv[U], wv[U];
#pragma unroll
  for (int t = 0; t < U; ++t) {
    uv[t] = a.u[q0 + t * stride];
    wv[t] = a.w[q0 + t * stride];
  }
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const double v = a.V[k * a.vstride + q0 + t * stride];
      acc[k] += v * uv[t];
      acc[NV + k] += v * wv[t];
    }
#pragma unroll
  for (int t = 0; t < U; ++t) {
    acc[2 * NV] += uv[t] * uv[t];
    acc[2 * NV + 1] += uv[t] * wv[t];
    acc[2 * NV + 2] += wv[t] * wv[t];
  }
}

// The grid holds 4 waves per SIMD (dcgs2_blocks), so the kernel may take up to 128 VGPRs: the 2NV+3 FP64
// accumulators then leave room for all NV+2 loads of an element to be in flight at once (capped at 64 VGPRs
// for 8 waves, the pass fell from 5.3 to 3.7 TB/s at NV = 10..14).
template <int NV>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 4))) void dots2_kernel(D2Args a,
                                                                                             ReduceWork rw) {
  constexpr int CNT = 2 * NV + 3;
  constexpr int U = NV <= 2 ? 4 : (NV <= 8 ? 2 : 1);
  double acc[CNT];
#pragma unroll
  for (int k = 0; k < CNT; ++k) acc[k] = 0.0;
  const long stride = (long)gridDim.x * NT;
  const long len = a.len;
  long q0 = (long)blockIdx.x * NT + threadIdx.x;
  for (; q0 + (U - 1) * stride < len; q0 += U * stride) process2<NV, U>(a, q0, stride, acc);
  for (; q0 < len; q0 += stride) process2<NV, 1>(a, q0, stride, acc);
  __shared__ double red[CNT * NW];
  __shared__ double tot[CNT];
  block_reduce<CNT>(acc, red, tot);
  const int mb = rw.max_blocks;
  for (int k = threadIdx.x; k < CNT; k += NT) rw.partial[(long)k * mb + blockIdx.x] = tot[k];
}

// Sums the partials in a fixed order and derives the step's coefficients:
//   res[0..NV) = a = Q^T u, res[NV..2NV) = s = Q^T w, then u.u, u.w, w.w,
//   beta = |u - Q a| = sqrt(u.u - |a|^2), 1/beta, h = q_j . w = (u.w - a.s) / beta,
//   nu = w.w - |s|^2 - h^2 (the squared norm of the next direction before its re-orthogonalisation),
//   flag (1 if beta is not a positive finite number).
template <int NV>
__global__ __launch_bounds__(NF2) void dcgs2_finish_kernel(D2Args a, ReduceWork rw, int nb) {
  constexpr int CNT = 2 * NV + 3;
  constexpr int W2 = NF2 / 64;
  const int mb = rw.max_blocks;
  __shared__ double tot[CNT];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // wave w sums the partials of values w, w + W2, ...: every lane adds its partials (independent loads, all
  // in flight at once), then the wave reduces across lanes
  for (int k = wid; k < CNT; k += W2) {
    const double* p = rw.partial + (long)k * mb;
    double sm = 0.0;
    for (int b0 = 0; b0 < nb; b0 += 1024) {
      double v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int b = b0 + lane + 64 * i;
        v[i] = b < nb ? p[b] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) sm += v[i];
    }
    sm = wave_sum(sm);
    if (lane == 0) {
      tot[k] = sm;
      a.res[k] = sm;
      if (a.mirror) a.mirror[k] = sm;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double na = 0.0, as = 0.0, ns = 0.0;
    for (int k = 0; k < NV; ++k) {
      na += tot[k] * tot[k];
      as += tot[k] * tot[NV + k];
      ns += tot[NV + k] * tot[NV + k];
    }
    const double b2 = tot[2 * NV] - na;
    const bool ok = b2 > 0.0 && b2 < 1.0e300;
    const double beta = ok ? sqrt(b2) : 0.0;
    const double ib = ok ? 1.0 / beta : 0.0;
    const double h = (tot[2 * NV + 1] - as) * ib;
    const double tail[5] = {beta, ib, h, tot[2 * NV + 2] - ns - h * h, ok ? 0.0 : 1.0};
#pragma unroll
    for (int k = 0; k < 5; ++k) a.res[CNT + k] = tail[k];
    if (a.mirror)
#pragma unroll
      for (int k = 0; k < 5; ++k) a.mirror[CNT + k] = tail[k];
  }
  // No system-scope fence after the mirror stores: the host reads the mirror only after waiting for the event
  // recorded behind this step, and the kernel's completion makes its stores to the coherent host memory visible
  // (the fence, a round trip to host memory, cost about 3.5 us per Arnoldi step).
}

template <int NV, int U>
__device__ __forceinline__ void process_upd(const D2Args& a, const double (&c1)[NV > 0 ? NV : 1],
                                            const double (&c2)[NV > 0 ? NV : 1], double ib, double h, long q0,
                                            long stride) {
  double uv[U], wv[U];
#pragma unroll
  for (int t = 0; t < U; ++t) {
    uv[t] = a.u[q0 + t * stride];
    wv[t] = a.w[q0 + t * stride];
  }
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const double v = a.V[k * a.vstride + q0 + t * stride];
      uv[t] -= c1[k] * v;
      wv[t] -= c2[k] * v;
    }
#pragma unroll
  for (int t = 0; t < U; ++t) {
    const double qn = uv[t] * ib;
    a.u[q0 + t * stride] = qn;
    a.w[q0 + t * stride] = wv[t] - h * qn;
  }
}

// u <- (u - Q a) / beta  (the finished q_j);  w <- w - Q s - h q_j  (the next direction)
template <int NV>
__global__ __launch_bounds__(NT) void dcgs2_update_kernel(D2Args a) {
  constexpr int NVV = NV > 0 ? NV : 1;
  constexpr int U = NV <= 2 ? 4 : (NV <= 8 ? 2 : 1);
  constexpr int CNT = 2 * NV + 3;
  double c1[NVV], c2[NVV];
#pragma unroll
  for (int k = 0; k < NVV; ++k) {
    c1[k] = k < NV ? a.res[k] : 0.0;
    c2[k] = k < NV ? a.res[NV + k] : 0.0;
  }
  const double ib = a.res[CNT + 1], h = a.res[CNT + 2];
  const long stride = (long)gridDim.x * NT;
  const long len = a.len;
  long q0 = (long)blockIdx.x * NT + threadIdx.x;
  for (; q0 + (U - 1) * stride < len; q0 += U * stride) process_upd<NV, U>(a, c1, c2, ib, h, q0, stride);
  for (; q0 < len; q0 += stride) process_upd<NV, 1>(a, c1, c2, ib, h, q0, stride);
}

using D2Fn = void (*)(D2Args, ReduceWork);
using D2FinFn = void (*)(D2Args, ReduceWork, int);
using D2UpdFn = void (*)(D2Args);

template <int... I>
struct Table2 {
  static D2Fn dots(int nv) {
    D2Fn out = nullptr;
    ((nv == I ? (out = dots2_kernel<I>, 0) : 0), ...);
    return out;
  }
  static D2FinFn fin(int nv) {
    D2FinFn out = nullptr;
    ((nv == I ? (out = dcgs2_finish_kernel<I>, 0) : 0), ...);
    return out;
  }
  static D2UpdFn upd(int nv) {
    D2UpdFn out = nullptr;
    ((nv == I ? (out = dcgs2_update_kernel<I>, 0) : 0), ...);
    return out;
  }
};

template <int... I>
Table2<I...> make_table2(std::integer_sequence<int, I...>);

using KernelFn = void (*)(OrthoArgs, ReduceWork);
using FinishFn = void (*)(OrthoArgs, ReduceWork, int);

template <int NV>
KernelFn pick(int mode, bool vf) {
  if (vf) return ortho_kernel<NV, AXPY, true>;  // FP32 basis: update passes only
  switch (mode) {
    case DOTS: return ortho_kernel<NV, DOTS, false>;
    case AXPY_DOTS: return ortho_kernel<NV, AXPY_DOTS, false>;
    default: return ortho_kernel<NV, AXPY, false>;
  }
}

template <int... I>
struct Table {
  static KernelFn get(int nv, int mode, bool vf) {
    KernelFn out = nullptr;
    ((nv == I + 1 ? (out = pick<I + 1>(mode, vf), 0) : 0), ...);
    return out;
  }
  static FinishFn fin(int nv) {
    FinishFn out = nullptr;
    ((nv == I + 1 ? (out = finish_kernel<I + 1>, 0) : 0), ...);
    return out;
  }
};

template <int... I>
Table<I...> make_table(std::integer_sequence<int, I...>);

}  // namespace

void launch_ortho(const OrthoArgs& a, const ReduceWork& rw, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  long blocks = (a.len + NT - 1) / NT;
  if (blocks > rw.max_blocks) blocks = rw.max_blocks;
  if (blocks > NF) blocks = NF;
  if (blocks < 1) blocks = 1;
  const int nb = (int)blocks;
  const bool ax = a.coef != nullptr, dt = a.want_dots != 0;
  if (a.nv <= 0 || (!ax && !dt)) {
    OrthoArgs b = a;
    b.nv = 0;
    // with events, they are attached to the dispatch itself (kernel start/end timestamps)
    if (ev0)
      hipExtLaunchKernelGGL(ortho_kernel<0, NORM, false>, dim3(nb), dim3(NT), 0, st, ev0, ev1, 0, b, rw);
    else
      ortho_kernel<0, NORM, false><<<nb, NT, 0, st>>>(b, rw);
    launch_k(finish_kernel<0>, dim3(1), dim3(NF), st, b, rw, nb);
    return;
  }
  const int mode = (ax && dt) ? AXPY_DOTS : (ax ? AXPY : DOTS);
  // an FP32 basis is read by update passes alone (the solution update x = Z y)
  const bool vf = a.Vf != nullptr && mode == AXPY;
  using T = decltype(make_table(std::make_integer_sequence<int, 32>{}));
  if (ev0)
    hipExtLaunchKernelGGL(T::get(a.nv, mode, vf), dim3(nb), dim3(NT), 0, st, ev0, ev1, 0, a, rw);
  else
    hipLaunchKernelGGL(T::get(a.nv, mode, vf), dim3(nb), dim3(NT), 0, st, a, rw);
  launch_k(T::fin(a.nv), dim3(1), dim3(NF), st, a, rw, nb);
}

int dcgs2_blocks(long len, const ReduceWork& rw) {
  long blocks = (len + NT - 1) / NT;
  if (blocks > rw.max_blocks) blocks = rw.max_blocks;
  if (blocks < 1) blocks = 1;
  return (int)blocks;
}

void launch_dcgs2_dots(const D2Args& a, const ReduceWork& rw, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  using T = decltype(make_table2(std::make_integer_sequence<int, kMaxDcgs2 + 1>{}));
  const int nb = dcgs2_blocks(a.len, rw);
  if (ev0)
    hipExtLaunchKernelGGL(T::dots(a.nv), dim3(nb), dim3(NT), 0, st, ev0, ev1, 0, a, rw);
  else
    hipLaunchKernelGGL(T::dots(a.nv), dim3(nb), dim3(NT), 0, st, a, rw);
  launch_k(T::fin(a.nv), dim3(1), dim3(NF2), st, a, rw, nb);
}

void launch_dcgs2_update(const D2Args& a, const ReduceWork& rw, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  using T = decltype(make_table2(std::make_integer_sequence<int, kMaxDcgs2 + 1>{}));
  const int nb = dcgs2_blocks(a.len, rw);
  if (ev0)
    hipExtLaunchKernelGGL(T::upd(a.nv), dim3(nb), dim3(NT), 0, st, ev0, ev1, 0, a);
  else
    hipLaunchKernelGGL(T::upd(a.nv), dim3(nb), dim3(NT), 0, st, a);
}

}  // namespace irk
