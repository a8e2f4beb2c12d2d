// Monolithic multigrid kernels for the stage-coupled operator (Section 3.3).
//
// A level operator acts on s stage planes at once,
//   (Acal x)_q = sum_r cm[q][r] M x_r + dt * sum_r ck[q][r] K x_r,
// with (cm, ck) = (I, A) for the AI form and (A^{-1}, I) for the IA form (transposed
// for the adjoint). The relaxation is additive Schwarz over the vertex patches of all
// stages (eq:Cinv, eq:bigdecomp): at every interior node the s x s patch block
//   C_v = cm * M_vv + dt * ck * K_vv,   M_vv = 16 h^2/36,  K_vv = (2/3) * (sum of the 4 kappa),
// is solved in registers (Gaussian elimination with partial pivoting), inside a Chebyshev
// iteration. One thread owns one node and all of its stages, so the s x s stage mixing
// never leaves registers.
//
// Kernels per level of a V-cycle: one Chebyshev step per smoothing step (stencil, block
// solve, recurrence), the residual, the full-weighting restriction, the bilinear
// prolongation-and-correction, and on the coarsest level a dense inverse.
#include "mg_device.h"

namespace irk {
namespace {

constexpr int MX = 64, MY = 4;  // thread block of the nodal kernels

__device__ __forceinline__ bool mmg_node(const Geom& g, int& i, int& j) {
  i = 1 + blockIdx.x * MX + threadIdx.x;
  j = 1 + blockIdx.y * MY + threadIdx.y;
  return i <= g.N - 1 && j <= g.N - 1;
}

dim3 mmg_grid(const Geom& g) { return dim3((g.N - 1 + MX - 1) / MX, (g.N - 1 + MY - 1) / MY); }

template <typename TC>
struct Stencil {
  TC kSW, kSE, kNW, kNE;
  __device__ __forceinline__ TC kdiag() const { return (TC)(2.0 / 3.0) * (kSW + kSE + kNW + kNE); }
};

template <typename TC>
__device__ __forceinline__ Stencil<TC> load_stencil(const TC* __restrict__ kap, long p, int P) {
  // elements around node p: SW at p - P - 1, SE at p - P, NW at p - 1, NE at p
  Stencil<TC> k;
  k.kSW = kap[p - P - 1];
  k.kSE = kap[p - P];
  k.kNW = kap[p - 1];
  k.kNE = kap[p];
  return k;
}

// M x and K x at node p of one plane
template <typename TS, typename TC>
__device__ __forceinline__ void mk_at(const TS* __restrict__ x, long p, int P, const Stencil<TC>& k, TC m, TC& Mx,
                                      TC& Kx) {
  const TC xc = ld<TC>(x + p), xE = ld<TC>(x + p + 1), xW = ld<TC>(x + p - 1), xN = ld<TC>(x + p + P),
           xS = ld<TC>(x + p - P);
  const TC xNE = ld<TC>(x + p + P + 1), xNW = ld<TC>(x + p + P - 1), xSE = ld<TC>(x + p - P + 1),
           xSW = ld<TC>(x + p - P - 1);
  Kx = (TC)(2.0 / 3.0) * (k.kSW + k.kSE + k.kNW + k.kNE) * xc -
       (TC)(1.0 / 6.0) * ((k.kNE + k.kSE) * xE + (k.kNW + k.kSW) * xW + (k.kNE + k.kNW) * xN + (k.kSE + k.kSW) * xS) -
       (TC)(1.0 / 3.0) * (k.kNE * xNE + k.kNW * xNW + k.kSE * xSE + k.kSW * xSW);
  Mx = m * ((TC)16 * xc + (TC)4 * (xE + xW + xN + xS) + (xNE + xNW + xSE + xSW));
}

// r = ts * t - Acal x at node p (x == nullptr: x = 0; t == nullptr: t = 0)
template <typename TT, typename TS, typename TC, int S>
__device__ __forceinline__ void residual_at(const TT* __restrict__ t, TC ts, const TS* __restrict__ x, long p,
                                            const Geom& g, const Stencil<TC>& k, const MMGCoef& c, TC r[S]) {
  const TC m = (TC)c.m, dt = (TC)c.dt;
#pragma unroll
  for (int q = 0; q < S; ++q) r[q] = t ? ts * ld<TC>(t + q * g.plane + p) : (TC)0;
  if (!x) return;
  TC Mx[S], Kx[S];
#pragma unroll
  for (int q = 0; q < S; ++q) mk_at<TS, TC>(x + q * g.plane, p, g.pitch, k, m, Mx[q], Kx[q]);
#pragma unroll
  for (int q = 0; q < S; ++q) {
    TC acc = (TC)0;
#pragma unroll
    for (int rr = 0; rr < S; ++rr) acc += (TC)c.cm[q * kMMGMax + rr] * Mx[rr] + dt * (TC)c.ck[q * kMMGMax + rr] * Kx[rr];
    r[q] -= acc;
  }
}

// the patch block C_v at a node with K_vv = kd
template <typename TC, int S>
__device__ __forceinline__ void patch_block(const MMGCoef& c, TC kd, TC C[S][S]) {
  const TC mv = (TC)16 * (TC)c.m, dtk = (TC)c.dt * kd;
#pragma unroll
  for (int q = 0; q < S; ++q)
#pragma unroll
    for (int rr = 0; rr < S; ++rr) C[q][rr] = (TC)c.cm[q * kMMGMax + rr] * mv + (TC)c.ck[q * kMMGMax + rr] * dtk;
}

// z = C^{-1} r in place (Gaussian elimination with partial pivoting, fully unrolled)
template <typename TC, int S>
__device__ __forceinline__ void block_solve(TC C[S][S], TC r[S]) {
#pragma unroll
  for (int k = 0; k < S; ++k) {
    // pivot: swap row k with the row of largest |C[i][k]|, i >= k (selects keep everything in registers)
#pragma unroll
    for (int i = k + 1; i < S; ++i) {
      const bool sw = fabs((double)C[i][k]) > fabs((double)C[k][k]);
#pragma unroll
      for (int j = 0; j < S; ++j) {
        const TC a = C[k][j], b = C[i][j];
        C[k][j] = sw ? b : a;
        C[i][j] = sw ? a : b;
      }
      const TC a = r[k], b = r[i];
      r[k] = sw ? b : a;
      r[i] = sw ? a : b;
    }
    const TC inv = (TC)1 / C[k][k];
#pragma unroll
    for (int i = k + 1; i < S; ++i) {
      const TC f = C[i][k] * inv;
#pragma unroll
      for (int j = k + 1; j < S; ++j) C[i][j] -= f * C[k][j];
      r[i] -= f * r[k];
    }
  }
#pragma unroll
  for (int k = S - 1; k >= 0; --k) {
    TC v = r[k];
#pragma unroll
    for (int j = k + 1; j < S; ++j) v -= C[k][j] * r[j];
    r[k] = v / C[k][k];
  }
}

// One Chebyshev step of the additive-Schwarz-preconditioned iteration on a level:
//   step 0:  out = xc + c0 C^{-1} (ts t - Acal xc)               (xc == nullptr: xc = 0)
//   step k:  out = xc + beta_k (xc - xp) + gam_k C^{-1} (ts t - Acal xc)   (xp == nullptr: xp = 0)
// out may alias xp (read and written only at the thread's own node).
template <typename TT, typename TS, typename TO, typename TC, int S>
__global__ __launch_bounds__(MX* MY) void mmg_step_kernel(const TT* __restrict__ t, const double* __restrict__ tscale,
                                                          const TS* __restrict__ xc, const TS* xp, TO* out,
                                                          const TC* __restrict__ kap, Geom g, MMGCoef c, int step) {
  int i, j;
  if (!mmg_node(g, i, j)) return;
  const long p = (long)j * g.pitch + i;
  const Stencil<TC> k = load_stencil(kap, p, g.pitch);
  const TC ts = tscale ? (TC)(*tscale) : (TC)1;
  TC r[S];
  residual_at<TT, TS, TC, S>(t, ts, xc, p, g, k, c, r);
  TC C[S][S];
  patch_block<TC, S>(c, k.kdiag(), C);
  block_solve<TC, S>(C, r);
  if (step == 0) {
    const TC c0 = (TC)c.c0;
#pragma unroll
    for (int q = 0; q < S; ++q) {
      const TC x0 = xc ? ld<TC>(xc + q * g.plane + p) : (TC)0;
      st(out + q * g.plane + p, x0 + c0 * r[q]);
    }
  } else {
    const TC beta = (TC)c.beta[step], gam = (TC)c.gam[step];
#pragma unroll
    for (int q = 0; q < S; ++q) {
      const TC x1 = ld<TC>(xc + q * g.plane + p);
      const TC x0 = xp ? ld<TC>(xp + q * g.plane + p) : (TC)0;
      st(out + q * g.plane + p, x1 + beta * (x1 - x0) + gam * r[q]);
    }
  }
}

// r = ts t - Acal x into level storage
template <typename TT, typename TS, typename TC, int S>
__global__ __launch_bounds__(MX* MY) void mmg_residual_kernel(const TT* __restrict__ t, const double* __restrict__ tscale,
                                                              const TS* __restrict__ x, TS* __restrict__ rout,
                                                              const TC* __restrict__ kap, Geom g, MMGCoef c) {
  int i, j;
  if (!mmg_node(g, i, j)) return;
  const long p = (long)j * g.pitch + i;
  const Stencil<TC> k = load_stencil(kap, p, g.pitch);
  const TC ts = tscale ? (TC)(*tscale) : (TC)1;
  TC r[S];
  residual_at<TT, TS, TC, S>(t, ts, x, p, g, k, c, r);
#pragma unroll
  for (int q = 0; q < S; ++q) st(rout + q * g.plane + p, r[q]);
}

// coarse right-hand side = (I (x) P^T) r, full weighting around fine node (2I, 2J)
template <typename TS, typename TC, int S>
__global__ __launch_bounds__(MX* MY) void mmg_restrict_kernel(const TS* __restrict__ r, TS* __restrict__ tc, Geom g,
                                                              Geom gc) {
  int I, J;
  if (!mmg_node(gc, I, J)) return;
  const int P = g.pitch;
  const long f = (long)(2 * J) * P + 2 * I;
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const TS* R = r + q * g.plane + f;
    const TC v = ld<TC>(R) + (TC)0.5 * (ld<TC>(R + 1) + ld<TC>(R - 1) + ld<TC>(R + P) + ld<TC>(R - P)) +
                 (TC)0.25 * (ld<TC>(R + P + 1) + ld<TC>(R + P - 1) + ld<TC>(R - P + 1) + ld<TC>(R - P - 1));
    st(tc + q * gc.plane + (long)J * gc.pitch + I, v);
  }
}

// x += (I (x) P) e
template <typename TS, typename TC, int S>
__global__ __launch_bounds__(MX* MY) void mmg_prolong_kernel(const TS* __restrict__ e, TS* __restrict__ x, Geom g,
                                                             Geom gc) {
  int i, j;
  if (!mmg_node(g, i, j)) return;
  const long p = (long)j * g.pitch + i;
#pragma unroll
  for (int q = 0; q < S; ++q) {
    TS* xp = x + q * g.plane + p;
    st(xp, ld<TC>(xp) + prolong_at<TS, TC>(e + q * gc.plane, gc.pitch, i, j));
  }
}

// Coarsest level: out = Cinv * t over the s*(N-1)^2 <= kMaxCoarse stage-major unknowns. One
// wavefront per row, all row and right-hand-side loads in flight, fixed-order reduction.
template <typename TI, typename TO, typename TC>
__global__ __launch_bounds__(256) void mmg_coarse_kernel(const TI* __restrict__ t, const double* __restrict__ tscale,
                                                         TO* __restrict__ out, const TC* __restrict__ Cinv, Geom g,
                                                         int s) {
  const int m = g.N - 1;
  const int nc = m * m, n = s * nc;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const TC* rw = Cinv + (long)row * n;
  constexpr int U = kMaxCoarse / 64;
  TC bv[U], tv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int col = lane + 64 * u;
    const int cc = col < n ? col : 0;
    const int q = cc / nc, node = cc - q * nc;
    const int j = node / m + 1, i = node - (j - 1) * m + 1;
    bv[u] = rw[cc];
    tv[u] = ld<TC>(t + q * g.plane + (long)j * g.pitch + i);
  }
  TC acc = (TC)0;
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (lane + 64 * u < n) acc += bv[u] * tv[u];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) {
    const TC tsc = tscale ? (TC)(*tscale) : (TC)1;
    const int q = row / nc, node = row - q * nc;
    const int j = node / m + 1, i = node - (j - 1) * m + 1;
    st(out + q * g.plane + (long)j * g.pitch + i, acc * tsc);
  }
}

// FP64 set-up operators: mode 0 out = C^{-1} Acal x, 1 out = Acal x, 2 out = C x
template <int S>
__global__ __launch_bounds__(MX* MY) void mmg_apply_kernel(const double* __restrict__ x, double* __restrict__ out,
                                                           const double* __restrict__ kap, Geom g, MMGCoef c,
                                                           int mode) {
  int i, j;
  if (!mmg_node(g, i, j)) return;
  const long p = (long)j * g.pitch + i;
  const Stencil<double> k = load_stencil(kap, p, g.pitch);
  double C[S][S];
  patch_block<double, S>(c, k.kdiag(), C);
  double r[S];
  if (mode == 2) {
#pragma unroll
    for (int q = 0; q < S; ++q) {
      double acc = 0.0;
#pragma unroll
      for (int rr = 0; rr < S; ++rr) acc += C[q][rr] * x[rr * g.plane + p];
      r[q] = acc;
    }
  } else {
    residual_at<double, double, double, S>(nullptr, 1.0, x, p, g, k, c, r);
#pragma unroll
    for (int q = 0; q < S; ++q) r[q] = -r[q];
    if (mode == 0) block_solve<double, S>(C, r);
  }
#pragma unroll
  for (int q = 0; q < S; ++q) out[q * g.plane + p] = r[q];
}

// ---------------------------------------------------------------- launch dispatch

template <typename TT, typename TS, typename TO, typename TC>
void step_t(const void* t, const double* ts, const void* xc, const void* xp, void* out, const void* kap, Geom g,
            const MMGCoef& c, int step, hipStream_t st) {
  const dim3 grid = mmg_grid(g), blk(MX, MY);
  const TT* tt = (const TT*)t;
  const TS *a = (const TS*)xc, *b = (const TS*)xp;
  TO* o = (TO*)out;
  const TC* k = (const TC*)kap;
  switch (c.s) {
    case 1: mmg_step_kernel<TT, TS, TO, TC, 1><<<grid, blk, 0, st>>>(tt, ts, a, b, o, k, g, c, step); break;
    case 2: mmg_step_kernel<TT, TS, TO, TC, 2><<<grid, blk, 0, st>>>(tt, ts, a, b, o, k, g, c, step); break;
    case 3: mmg_step_kernel<TT, TS, TO, TC, 3><<<grid, blk, 0, st>>>(tt, ts, a, b, o, k, g, c, step); break;
    default: mmg_step_kernel<TT, TS, TO, TC, 4><<<grid, blk, 0, st>>>(tt, ts, a, b, o, k, g, c, step); break;
  }
}

template <typename TT, typename TS, typename TC>
void residual_t(const void* t, const double* ts, const void* x, void* r, const void* kap, Geom g, const MMGCoef& c,
                hipStream_t st) {
  const dim3 grid = mmg_grid(g), blk(MX, MY);
  const TT* tt = (const TT*)t;
  const TS* xx = (const TS*)x;
  TS* rr = (TS*)r;
  const TC* k = (const TC*)kap;
  switch (c.s) {
    case 1: mmg_residual_kernel<TT, TS, TC, 1><<<grid, blk, 0, st>>>(tt, ts, xx, rr, k, g, c); break;
    case 2: mmg_residual_kernel<TT, TS, TC, 2><<<grid, blk, 0, st>>>(tt, ts, xx, rr, k, g, c); break;
    case 3: mmg_residual_kernel<TT, TS, TC, 3><<<grid, blk, 0, st>>>(tt, ts, xx, rr, k, g, c); break;
    default: mmg_residual_kernel<TT, TS, TC, 4><<<grid, blk, 0, st>>>(tt, ts, xx, rr, k, g, c); break;
  }
}

template <typename TS, typename TC>
void transfer_t(bool restrict_, const void* a, void* b, Geom g, Geom gc, int s, hipStream_t st) {
  const dim3 blk(MX, MY);
  if (restrict_) {
    const dim3 grid = mmg_grid(gc);
    const TS* r = (const TS*)a;
    TS* tc = (TS*)b;
    switch (s) {
      case 1: mmg_restrict_kernel<TS, TC, 1><<<grid, blk, 0, st>>>(r, tc, g, gc); break;
      case 2: mmg_restrict_kernel<TS, TC, 2><<<grid, blk, 0, st>>>(r, tc, g, gc); break;
      case 3: mmg_restrict_kernel<TS, TC, 3><<<grid, blk, 0, st>>>(r, tc, g, gc); break;
      default: mmg_restrict_kernel<TS, TC, 4><<<grid, blk, 0, st>>>(r, tc, g, gc); break;
    }
  } else {
    const dim3 grid = mmg_grid(g);
    const TS* e = (const TS*)a;
    TS* x = (TS*)b;
    switch (s) {
      case 1: mmg_prolong_kernel<TS, TC, 1><<<grid, blk, 0, st>>>(e, x, g, gc); break;
      case 2: mmg_prolong_kernel<TS, TC, 2><<<grid, blk, 0, st>>>(e, x, g, gc); break;
      case 3: mmg_prolong_kernel<TS, TC, 3><<<grid, blk, 0, st>>>(e, x, g, gc); break;
      default: mmg_prolong_kernel<TS, TC, 4><<<grid, blk, 0, st>>>(e, x, g, gc); break;
    }
  }
}

}  // namespace

// prec: 0 FP64, 1 FP32, 2 BF16 storage with FP32 compute (kappa and Cinv in the compute type).
// t_f64 / out_f64: t or out is an FP64 Krylov vector instead of level storage.
void launch_mmg_step(int prec, bool t_f64, bool out_f64, const void* t, const double* tscale, const void* xc,
                     const void* xp, void* out, const void* kap, Geom g, const MMGCoef& c, int step, hipStream_t st) {
  if (prec == 0) {
    step_t<double, double, double, double>(t, tscale, xc, xp, out, kap, g, c, step, st);
  } else if (prec == 1) {
    if (t_f64 && out_f64) step_t<double, float, double, float>(t, tscale, xc, xp, out, kap, g, c, step, st);
    else if (t_f64) step_t<double, float, float, float>(t, tscale, xc, xp, out, kap, g, c, step, st);
    else if (out_f64) step_t<float, float, double, float>(t, tscale, xc, xp, out, kap, g, c, step, st);
    else step_t<float, float, float, float>(t, tscale, xc, xp, out, kap, g, c, step, st);
  } else {
    if (t_f64 && out_f64) step_t<double, bf16, double, float>(t, tscale, xc, xp, out, kap, g, c, step, st);
    else if (t_f64) step_t<double, bf16, bf16, float>(t, tscale, xc, xp, out, kap, g, c, step, st);
    else if (out_f64) step_t<bf16, bf16, double, float>(t, tscale, xc, xp, out, kap, g, c, step, st);
    else step_t<bf16, bf16, bf16, float>(t, tscale, xc, xp, out, kap, g, c, step, st);
  }
}

void launch_mmg_residual(int prec, bool t_f64, const void* t, const double* tscale, const void* x, void* r,
                         const void* kap, Geom g, const MMGCoef& c, hipStream_t st) {
  if (prec == 0) residual_t<double, double, double>(t, tscale, x, r, kap, g, c, st);
  else if (prec == 1) {
    if (t_f64) residual_t<double, float, float>(t, tscale, x, r, kap, g, c, st);
    else residual_t<float, float, float>(t, tscale, x, r, kap, g, c, st);
  } else {
    if (t_f64) residual_t<double, bf16, float>(t, tscale, x, r, kap, g, c, st);
    else residual_t<bf16, bf16, float>(t, tscale, x, r, kap, g, c, st);
  }
}

void launch_mmg_restrict(int prec, const void* r, void* tc, Geom g, Geom gc, int s, hipStream_t st) {
  if (prec == 0) transfer_t<double, double>(true, r, tc, g, gc, s, st);
  else if (prec == 1) transfer_t<float, float>(true, r, tc, g, gc, s, st);
  else transfer_t<bf16, float>(true, r, tc, g, gc, s, st);
}

void launch_mmg_prolong(int prec, const void* e, void* x, Geom g, Geom gc, int s, hipStream_t st) {
  if (prec == 0) transfer_t<double, double>(false, e, x, g, gc, s, st);
  else if (prec == 1) transfer_t<float, float>(false, e, x, g, gc, s, st);
  else transfer_t<bf16, float>(false, e, x, g, gc, s, st);
}

void launch_mmg_coarse(int prec, bool t_f64, bool out_f64, const void* t, const double* tscale, void* out,
                       const void* Cinv, Geom g, int s, hipStream_t st) {
  const int n = s * (g.N - 1) * (g.N - 1);
  const dim3 grid((n + 3) / 4), blk(256);
  if (prec == 0) {
    mmg_coarse_kernel<double, double, double><<<grid, blk, 0, st>>>((const double*)t, tscale, (double*)out,
                                                                     (const double*)Cinv, g, s);
  } else if (prec == 1) {
    const float* C = (const float*)Cinv;
    if (t_f64 && out_f64) mmg_coarse_kernel<double, double, float><<<grid, blk, 0, st>>>((const double*)t, tscale, (double*)out, C, g, s);
    else if (t_f64) mmg_coarse_kernel<double, float, float><<<grid, blk, 0, st>>>((const double*)t, tscale, (float*)out, C, g, s);
    else if (out_f64) mmg_coarse_kernel<float, double, float><<<grid, blk, 0, st>>>((const float*)t, tscale, (double*)out, C, g, s);
    else mmg_coarse_kernel<float, float, float><<<grid, blk, 0, st>>>((const float*)t, tscale, (float*)out, C, g, s);
  } else {
    const float* C = (const float*)Cinv;
    if (t_f64 && out_f64) mmg_coarse_kernel<double, double, float><<<grid, blk, 0, st>>>((const double*)t, tscale, (double*)out, C, g, s);
    else if (t_f64) mmg_coarse_kernel<double, bf16, float><<<grid, blk, 0, st>>>((const double*)t, tscale, (bf16*)out, C, g, s);
    else if (out_f64) mmg_coarse_kernel<bf16, double, float><<<grid, blk, 0, st>>>((const bf16*)t, tscale, (double*)out, C, g, s);
    else mmg_coarse_kernel<bf16, bf16, float><<<grid, blk, 0, st>>>((const bf16*)t, tscale, (bf16*)out, C, g, s);
  }
}

void launch_mmg_apply(const double* x, double* out, const double* kap, Geom g, const MMGCoef& c, int mode,
                      hipStream_t st) {
  const dim3 grid = mmg_grid(g), blk(MX, MY);
  switch (c.s) {
    case 1: mmg_apply_kernel<1><<<grid, blk, 0, st>>>(x, out, kap, g, c, mode); break;
    case 2: mmg_apply_kernel<2><<<grid, blk, 0, st>>>(x, out, kap, g, c, mode); break;
    case 3: mmg_apply_kernel<3><<<grid, blk, 0, st>>>(x, out, kap, g, c, mode); break;
    default: mmg_apply_kernel<4><<<grid, blk, 0, st>>>(x, out, kap, g, c, mode); break;
  }
}

}  // namespace irk
