// Layout conversions and FP64 Q1 stencil kernels on padded planes.
//
// The Q1 stiffness and mass operators are applied matrix-free through their
// 9-point stencils at interior node c with the four surrounding elements
// SW, SE, NW, NE (element diffusivities k..):
//   (K x)_c = 2/3 (kSW+kSE+kNW+kNE) x_c
//             - 1/6 [(kNE+kSE) x_E + (kNW+kSW) x_W + (kNE+kNW) x_N + (kSE+kSW) x_S]
//             - 1/3 (kNE x_NE + kNW x_NW + kSE x_SE + kSW x_SW)
//   (M x)_c = h^2/36 [16 x_c + 4 (x_E+x_W+x_N+x_S) + (x_NE+x_NW+x_SE+x_SW)]
// which is the element-by-element assembly of the bilinear element matrices
// (Section 2, eq:heat/eq:rkheat discretised with Q1) with the boundary rows and
// columns removed (homogeneous "DAE-type" Dirichlet data, Section 2.1).
#include "irk_internal.h"

namespace irk {
namespace {

constexpr int BX = 64;  // one wavefront along x
constexpr int BY = 4;

struct Nb {
  double c, e, w, n, s, ne, nw, se, sw;
};

template <typename TX>
__device__ __forceinline__ Nb load_nb(const TX* __restrict__ x, long p, int P) {
  Nb v;
  v.c = x[p];
  v.e = x[p + 1];
  v.w = x[p - 1];
  v.n = x[p + P];
  v.s = x[p - P];
  v.ne = x[p + P + 1];
  v.nw = x[p + P - 1];
  v.se = x[p - P + 1];
  v.sw = x[p - P - 1];
  return v;
}

struct Kap {
  double sw, se, nw, ne;
};

__device__ __forceinline__ Kap load_kap(const double* __restrict__ kap, long p, int P) {
  Kap k;
  k.sw = kap[p - P - 1];
  k.se = kap[p - P];
  k.nw = kap[p - 1];
  k.ne = kap[p];
  return k;
}

__device__ __forceinline__ double stiff(const Nb& x, const Kap& k) {
  const double c23 = 2.0 / 3.0, c16 = 1.0 / 6.0, c13 = 1.0 / 3.0;
  return c23 * (k.sw + k.se + k.nw + k.ne) * x.c -
         c16 * ((k.ne + k.se) * x.e + (k.nw + k.sw) * x.w + (k.ne + k.nw) * x.n + (k.se + k.sw) * x.s) -
         c13 * (k.ne * x.ne + k.nw * x.nw + k.se * x.se + k.sw * x.sw);
}

__device__ __forceinline__ double mass(const Nb& x, double m) {
  return m * (16.0 * x.c + 4.0 * (x.e + x.w + x.n + x.s) + (x.ne + x.nw + x.se + x.sw));
}

// interior node of the thread, or false
__device__ __forceinline__ bool node_of_thread(const Geom& g, int& i, int& j) {
  i = 1 + blockIdx.x * BX + threadIdx.x;
  j = 1 + blockIdx.y * BY + threadIdx.y;
  return i <= g.N - 1 && j <= g.N - 1;
}

dim3 stencil_grid(const Geom& g) { return dim3((g.N - 1 + BX - 1) / BX, (g.N - 1 + BY - 1) / BY); }

// ------------------------------------------------------------------ layout

__global__ void pack_kernel(const double* __restrict__ src, double* __restrict__ dst, Geom g) {
  const long plane = g.plane;
  const int m = g.N - 1;
  const double* s = src + (long)blockIdx.y * m * m;
  double* d = dst + (long)blockIdx.y * plane;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < plane; idx += (long)gridDim.x * blockDim.x) {
    const int j = (int)(idx / g.pitch);
    const int i = (int)(idx - (long)j * g.pitch);
    double v = 0.0;
    if (i >= 1 && i <= m && j >= 1 && j <= m) v = s[(long)(j - 1) * m + (i - 1)];
    d[idx] = v;
  }
}

__global__ void unpack_kernel(const double* __restrict__ src, double* __restrict__ dst, Geom g) {
  const int m = g.N - 1;
  const long n = (long)m * m;
  const double* s = src + (long)blockIdx.y * g.plane;
  double* d = dst + (long)blockIdx.y * n;
  for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
    const int j = (int)(q / m) + 1;
    const int i = (int)(q - (long)(j - 1) * m) + 1;
    d[q] = s[(long)j * g.pitch + i];
  }
}

__global__ void pack_elem_kernel(const double* __restrict__ src, double* __restrict__ dst, Geom g) {
  const long total = (long)g.N * g.pitch;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const int ey = (int)(idx / g.pitch);
    const int ex = (int)(idx - (long)ey * g.pitch);
    dst[idx] = (ex < g.N) ? src[(long)ey * g.N + ex] : 0.0;
  }
}

__global__ void unpack_elem_kernel(const double* __restrict__ src, double* __restrict__ dst, Geom g) {
  const long n = (long)g.N * g.N;
  for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
    const int ey = (int)(q / g.N);
    const int ex = (int)(q - (long)ey * g.N);
    dst[q] = src[(long)ey * g.pitch + ex];
  }
}

__global__ void check_kappa_kernel(const double* __restrict__ k, int count, int* bad) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < count; q += gridDim.x * blockDim.x) {
    const double v = k[q];
    if (!(v > 0.0) || !(v < INFINITY)) atomicOr(bad, 1);
  }
}

__global__ void cast_f32_kernel(const double* __restrict__ s, float* __restrict__ d, long n) {
  for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x)
    d[q] = (float)s[q];
}

__global__ void coarsen_kappa_kernel(const double* __restrict__ f, double* __restrict__ c, Geom gf, Geom gc) {
  const long total = (long)gc.N * gc.pitch;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const int ey = (int)(idx / gc.pitch);
    const int ex = (int)(idx - (long)ey * gc.pitch);
    double v = 0.0;
    if (ex < gc.N) {
      const long b = (long)(2 * ey) * gf.pitch + 2 * ex;
      v = 0.25 * (f[b] + f[b + 1] + f[b + gf.pitch] + f[b + gf.pitch + 1]);
    }
    c[idx] = v;
  }
}

// ------------------------------------------------------------------ stencils

// Stage operator, register-blocked: each thread owns RB consecutive nodes of one column, so the three rows
// of every 9-point stencil and the element diffusivities are loaded once per column segment
// ((RB + 2) * 3 values per plane and 2 (RB + 1) diffusivities for RB nodes); tiles in XCD-aware order.
constexpr int RB = 4;
constexpr int SBY = 4;  // wavefronts per block

template <int S, bool IA, typename TX>
__global__ __launch_bounds__(BX* SBY) void stage_operator_kernel(const TX* __restrict__ x, double* __restrict__ y,
                                                                const double* __restrict__ f,
                                                                const double* __restrict__ kap, Geom g, Coefs a,
                                                                double dt) {
  const int N = g.N, P = g.pitch;
  const int ntx = (N - 1 + BX - 1) / BX;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int i = 1 + (t % ntx) * BX + threadIdx.x;
  const int j0 = 1 + (t / ntx) * (SBY * RB) + threadIdx.y * RB;
  if (i > N - 1 || j0 > N - 1) return;
  const double m = g.h * g.h / 36.0;
  // element rows j0-1 .. j0+RB-1 and node rows j0-1 .. j0+RB, clamped to the array (values past the
  // last interior row are loaded but not used)
  double kw[RB + 1], ke[RB + 1];
#pragma unroll
  for (int r = 0; r <= RB; ++r) {
    const int er = min(j0 - 1 + r, N - 1);
    kw[r] = kap[(long)er * P + i - 1];
    ke[r] = kap[(long)er * P + i];
  }
  double Kx[S][RB], Mx[S][RB];
#pragma unroll
  for (int q = 0; q < S; ++q) {
    double xw[RB + 2], xc[RB + 2], xe[RB + 2];
#pragma unroll
    for (int r = 0; r < RB + 2; ++r) {
      const int nr = min(j0 - 1 + r, N);
      const long pr = q * g.plane + (long)nr * P + i;
      xw[r] = (double)x[pr - 1];
      xc[r] = (double)x[pr];
      xe[r] = (double)x[pr + 1];
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      Kap k;
      k.sw = kw[r];
      k.se = ke[r];
      k.nw = kw[r + 1];
      k.ne = ke[r + 1];
      Nb v;
      v.c = xc[r + 1];
      v.e = xe[r + 1];
      v.w = xw[r + 1];
      v.n = xc[r + 2];
      v.s = xc[r];
      v.ne = xe[r + 2];
      v.nw = xw[r + 2];
      v.se = xe[r];
      v.sw = xw[r];
      Kx[q][r] = stiff(v, k);
      Mx[q][r] = mass(v, m);
    }
  }
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int j = j0 + r;
    if (j > N - 1) break;
    const long p = (long)j * P + i;
#pragma unroll
    for (int qo = 0; qo < S; ++qo) {
      double acc = 0.0, val;
      if (IA) {
        // (A^{-1} (x) M + dt I (x) K) x: stage mixing on the mass term
#pragma unroll
        for (int q = 0; q < S; ++q) acc += a.a[qo * kMaxStages + q] * Mx[q][r];
        val = acc + dt * Kx[qo][r];
      } else {
#pragma unroll
        for (int q = 0; q < S; ++q) acc += a.a[qo * kMaxStages + q] * Kx[q][r];
        val = Mx[qo][r] + dt * acc;
      }
      if (f)
        y[qo * g.plane + p] = f[qo * g.plane + p] - val;
      else
        y[qo * g.plane + p] = val;
    }
  }
}

__global__ __launch_bounds__(BX* BY) void stage_rhs_kernel(const double* __restrict__ u, const double* __restrict__ F,
                                                           double* __restrict__ f, const double* __restrict__ kap,
                                                           Geom g, int s, double* __restrict__ f2) {
  int i, j;
  if (!node_of_thread(g, i, j)) return;
  const int P = g.pitch;
  const long p = (long)j * P + i;
  double v = -stiff(load_nb(u, p, P), load_kap(kap, p, P));
  if (F) v += F[p];
  for (int r = 0; r < s; ++r) f[r * g.plane + p] = v;
  if (f2)
    for (int r = 0; r < s; ++r) f2[r * g.plane + p] = v;
}

__global__ __launch_bounds__(BX* BY) void mass_kernel(const double* __restrict__ x, double* __restrict__ y, Geom g) {
  int i, j;
  if (!node_of_thread(g, i, j)) return;
  const long p = (long)j * g.pitch + i;
  y[p] = mass(load_nb(x, p, g.pitch), g.h * g.h / 36.0);
}

__global__ __launch_bounds__(BX* BY) void stiff_kernel(const double* __restrict__ x, double* __restrict__ y,
                                                       const double* __restrict__ kap, Geom g) {
  int i, j;
  if (!node_of_thread(g, i, j)) return;
  const long p = (long)j * g.pitch + i;
  y[p] = stiff(load_nb(x, p, g.pitch), load_kap(kap, p, g.pitch));
}

template <typename TZ>
__global__ __launch_bounds__(BX* BY) void gs_couple_kernel(const double* __restrict__ v, const double* __restrict__ vscale,
                                                           const TZ* __restrict__ z, int ns, Coefs row, double dt,
                                                           const double* __restrict__ kap, double* __restrict__ t,
                                                           Geom g, int use_mass, double vmul) {
  int i, j;
  if (!node_of_thread(g, i, j)) return;
  const int P = g.pitch;
  const long p = (long)j * P + i;
  const Kap k = load_kap(kap, p, P);
  const double m = g.h * g.h / 36.0;
  double acc = 0.0;
  for (int q = 0; q < ns; ++q) {
    const Nb nb = load_nb(z + q * g.plane, p, P);
    acc += row.a[q] * (use_mass ? mass(nb, m) : stiff(nb, k));
  }
  t[p] = vmul * (vscale ? *vscale : 1.0) * v[p] - dt * acc;
}

__global__ void update_kernel(double* __restrict__ u, const double* __restrict__ k, int s, Coefs b, double dt,
                              long plane) {
  for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < plane; q += (long)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int r = 0; r < s; ++r) acc += b.a[r] * k[r * plane + q];
    u[q] += dt * acc;
  }
}

__global__ void adjoint_rhs_kernel(const double* __restrict__ lam, double* __restrict__ f, int s, Coefs b, double dt,
                                   long plane) {
  for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < plane; q += (long)gridDim.x * blockDim.x) {
    const double l = lam[q];
    for (int r = 0; r < s; ++r) f[r * plane + q] = dt * b.a[r] * l;
  }
}

__global__ __launch_bounds__(BX* BY) void lambda_update_kernel(double* __restrict__ lam, const double* __restrict__ nu,
                                                               int s, const double* __restrict__ kap, Geom g) {
  int i, j;
  if (!node_of_thread(g, i, j)) return;
  const int P = g.pitch;
  const long p = (long)j * P + i;
  const Kap k = load_kap(kap, p, P);
  double acc = 0.0;
  for (int r = 0; r < s; ++r) acc += stiff(load_nb(nu + r * g.plane, p, P), k);
  lam[p] -= acc;
}

// one thread per element; local nodes (0,0),(1,0),(1,1),(0,1)
__global__ void kappa_grad_kernel(double* __restrict__ grad, const double* __restrict__ u, const double* __restrict__ k,
                                  const double* __restrict__ nu, const double* __restrict__ kap, Geom g, int s, Coefs a,
                                  double dt) {
  const int ex = blockIdx.x * blockDim.x + threadIdx.x;
  const int ey = blockIdx.y * blockDim.y + threadIdx.y;
  if (ex >= g.N || ey >= g.N) return;
  const int P = g.pitch;
  const long n0 = (long)ey * P + ex;
  const long nd[4] = {n0, n0 + 1, n0 + P + 1, n0 + P};
  const double Kr[4][4] = {{4, -1, -2, -1}, {-1, 4, -1, -2}, {-2, -1, 4, -1}, {-1, -2, -1, 4}};
  double un[4];
  for (int q = 0; q < 4; ++q) un[q] = u[nd[q]];
  double kn[kMaxStages][4];
  for (int r = 0; r < s; ++r)
    for (int q = 0; q < 4; ++q) kn[r][q] = k[r * g.plane + nd[q]];
  double acc = 0.0;
  for (int r = 0; r < s; ++r) {
    double U[4], nv[4];
    for (int q = 0; q < 4; ++q) {
      double w = 0.0;
      for (int c = 0; c < s; ++c) w += a.a[r * kMaxStages + c] * kn[c][q];
      U[q] = un[q] + dt * w;
      nv[q] = nu[r * g.plane + nd[q]];
    }
    for (int q = 0; q < 4; ++q) {
      double t = 0.0;
      for (int c = 0; c < 4; ++c) t += Kr[q][c] * U[c];
      acc += nv[q] * t;
    }
  }
  grad[n0] -= kap[n0] * acc / 6.0;
}

__global__ __launch_bounds__(BX* BY) void level_apply_kernel(const double* __restrict__ x, double* __restrict__ y,
                                                             const double* __restrict__ kap, Geom g, double alpha,
                                                             int mode) {
  int i, j;
  if (!node_of_thread(g, i, j)) return;
  const int P = g.pitch;
  const long p = (long)j * P + i;
  const Kap k = load_kap(kap, p, P);
  const double m = g.h * g.h / 36.0;
  const double D = 16.0 * m + alpha * (2.0 / 3.0) * (k.sw + k.se + k.nw + k.ne);
  if (mode == 2) {
    y[p] = D * x[p];
    return;
  }
  const Nb v = load_nb(x, p, P);
  const double Bx = mass(v, m) + alpha * stiff(v, k);
  y[p] = (mode == 1) ? Bx / D : Bx;
}

// SplitMix64 (Steele, Lea & Flood 2014), written from its published definition
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(BX* BY) void start_vector_kernel(double* __restrict__ x, Geom g, int level,
                                                              uint64_t offset) {
  int i, j;
  if (!node_of_thread(g, i, j)) return;
  const uint64_t dof = (uint64_t)(j - 1) * (uint64_t)(g.N - 1) + (uint64_t)(i - 1) + offset;
  const uint64_t r = splitmix64(dof + ((uint64_t)level << 32));
  x[(long)j * g.pitch + i] = 2.0 * ((double)(r >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
}

__global__ void scale_kernel(double* __restrict__ x, long n, const double* __restrict__ nrm2) {
  const double f = 1.0 / sqrt(*nrm2);
  for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) x[q] *= f;
}

// Streaming copy, the reference kernel for the bandwidth ceiling and for scaling the HBM byte counters: one 16-byte
// load and one store per thread over a grid that covers the vector (an odd last value is copied by the first
// thread); pointers that are not 16-byte aligned take the scalar grid-stride form.
__global__ __launch_bounds__(256) void device_copy_kernel(const double2* __restrict__ x, double2* __restrict__ y,
                                                          long n2, const double* __restrict__ xs,
                                                          double* __restrict__ ys, long n) {
  const long q = (long)blockIdx.x * 256 + threadIdx.x;
  if (q < n2) y[q] = x[q];
  if ((n & 1) && q == 0) ys[n - 1] = xs[n - 1];
}

__global__ __launch_bounds__(256) void device_copy_scalar_kernel(const double* __restrict__ x, double* __restrict__ y,
                                                                 long n) {
  for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) y[q] = x[q];
}

int flat_blocks(long n) {
  long b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

void launch_device_copy(const double* x, double* y, long n, hipStream_t st) {
  if (n <= 0) return;
  if (((uintptr_t)x | (uintptr_t)y) & 15) {
    launch_k(device_copy_scalar_kernel, flat_blocks(n), 256, st, x, y, n);
    return;
  }
  const long n2 = n / 2;
  const long blocks = n2 > 0 ? (n2 + 255) / 256 : 1;
  launch_k(device_copy_kernel, dim3((unsigned)blocks), 256, st, (const double2*)x, (double2*)y, n2, x, y, n);
}

void launch_pack(const double* src, double* dst, Geom g, int nplanes, hipStream_t st) {
  launch_k(pack_kernel, dim3(flat_blocks(g.plane), nplanes), 256, st, src, dst, g);
}
void launch_unpack(const double* src, double* dst, Geom g, int nplanes, hipStream_t st) {
  launch_k(unpack_kernel, dim3(flat_blocks((long)(g.N - 1) * (g.N - 1)), nplanes), 256, st, src, dst, g);
}
void launch_pack_elem(const double* src, double* dst, Geom g, hipStream_t st) {
  launch_k(pack_elem_kernel, flat_blocks((long)g.N * g.pitch), 256, st, src, dst, g);
}
void launch_unpack_elem(const double* src, double* dst, Geom g, hipStream_t st) {
  launch_k(unpack_elem_kernel, flat_blocks((long)g.N * g.N), 256, st, src, dst, g);
}
void launch_check_kappa(const double* kappa, int count, int* bad, hipStream_t st) {
  launch_k(check_kappa_kernel, flat_blocks(count), 256, st, kappa, count, bad);
}
void launch_cast_f32(const double* src, float* dst, long count, hipStream_t st) {
  launch_k(cast_f32_kernel, flat_blocks(count), 256, st, src, dst, count);
}
void launch_coarsen_kappa(const double* fine, double* coarse, Geom gf, Geom gc, hipStream_t st) {
  launch_k(coarsen_kappa_kernel, flat_blocks((long)gc.N * gc.pitch), 256, st, fine, coarse, gf, gc);
}

template <bool IA, typename TX>
void stage_operator_t(const TX* x, double* y, const double* f, const double* kappa, Geom g, int s, const Coefs& a,
                      double dt, hipStream_t st) {
  const int ntx = (g.N - 1 + BX - 1) / BX, nty = (g.N - 1 + SBY * RB - 1) / (SBY * RB);
  const dim3 grid(ntx * nty), blk(BX, SBY);
  switch (s) {
    case 1: launch_k(stage_operator_kernel<1, IA, TX>, grid, blk, st, x, y, f, kappa, g, a, dt); break;
    case 2: launch_k(stage_operator_kernel<2, IA, TX>, grid, blk, st, x, y, f, kappa, g, a, dt); break;
    case 3: launch_k(stage_operator_kernel<3, IA, TX>, grid, blk, st, x, y, f, kappa, g, a, dt); break;
    case 4: launch_k(stage_operator_kernel<4, IA, TX>, grid, blk, st, x, y, f, kappa, g, a, dt); break;
    case 5: launch_k(stage_operator_kernel<5, IA, TX>, grid, blk, st, x, y, f, kappa, g, a, dt); break;
    case 6: launch_k(stage_operator_kernel<6, IA, TX>, grid, blk, st, x, y, f, kappa, g, a, dt); break;
    case 7: launch_k(stage_operator_kernel<7, IA, TX>, grid, blk, st, x, y, f, kappa, g, a, dt); break;
    default: launch_k(stage_operator_kernel<8, IA, TX>, grid, blk, st, x, y, f, kappa, g, a, dt); break;
  }
}

void launch_stage_operator(const double* x, double* y, const double* f, const double* kappa, Geom g, int s,
                           const Coefs& a, double dt, hipStream_t st, bool ia) {
  if (ia)
    stage_operator_t<true>(x, y, f, kappa, g, s, a, dt, st);
  else
    stage_operator_t<false>(x, y, f, kappa, g, s, a, dt, st);
}
void launch_stage_operator(const float* x, double* y, const double* f, const double* kappa, Geom g, int s,
                           const Coefs& a, double dt, hipStream_t st, bool ia) {
  if (ia)
    stage_operator_t<true>(x, y, f, kappa, g, s, a, dt, st);
  else
    stage_operator_t<false>(x, y, f, kappa, g, s, a, dt, st);
}
void launch_stage_rhs(const double* u, const double* F, double* f, const double* kappa, Geom g, int s, hipStream_t st,
                      double* f2) {
  launch_k(stage_rhs_kernel, stencil_grid(g), dim3(BX, BY), st, u, F, f, kappa, g, s, f2);
}
void launch_mass(const double* x, double* y, Geom g, hipStream_t st) {
  launch_k(mass_kernel, stencil_grid(g), dim3(BX, BY), st, x, y, g);
}
void launch_stiff(const double* x, double* y, const double* kappa, Geom g, hipStream_t st) {
  launch_k(stiff_kernel, stencil_grid(g), dim3(BX, BY), st, x, y, kappa, g);
}
void launch_gs_couple(const double* v, const double* vscale, const double* z, int nz, const Coefs& row, double dt,
                      const double* kappa, double* t, Geom g, hipStream_t st, int mass, double vmul) {
  launch_k(gs_couple_kernel<double>, stencil_grid(g), dim3(BX, BY), st, v, vscale, z, nz, row, dt, kappa, t, g, mass,
           vmul);
}
void launch_gs_couple(const double* v, const double* vscale, const float* z, int nz, const Coefs& row, double dt,
                      const double* kappa, double* t, Geom g, hipStream_t st, int mass, double vmul) {
  launch_k(gs_couple_kernel<float>, stencil_grid(g), dim3(BX, BY), st, v, vscale, z, nz, row, dt, kappa, t, g, mass,
           vmul);
}
void launch_update(double* u, const double* k, int s, const Coefs& b, double dt, Geom g, hipStream_t st) {
  launch_k(update_kernel, flat_blocks(g.plane), 256, st, u, k, s, b, dt, g.plane);
}
void launch_adjoint_rhs(const double* lam, double* f, int s, const Coefs& b, double dt, Geom g, hipStream_t st) {
  launch_k(adjoint_rhs_kernel, flat_blocks(g.plane), 256, st, lam, f, s, b, dt, g.plane);
}
void launch_lambda_update(double* lam, const double* nu, int s, const double* kappa, Geom g, hipStream_t st) {
  launch_k(lambda_update_kernel, stencil_grid(g), dim3(BX, BY), st, lam, nu, s, kappa, g);
}
void launch_kappa_grad(double* grad, const double* u, const double* k, const double* nu, const double* kappa, Geom g,
                       int s, const Coefs& a, double dt, hipStream_t st) {
  const dim3 blk(64, 4), grid((g.N + 63) / 64, (g.N + 3) / 4);
  launch_k(kappa_grad_kernel, grid, blk, st, grad, u, k, nu, kappa, g, s, a, dt);
}
void launch_level_apply(const double* x, double* y, const double* kappa, Geom g, double alpha, int mode,
                        hipStream_t st) {
  launch_k(level_apply_kernel, stencil_grid(g), dim3(BX, BY), st, x, y, kappa, g, alpha, mode);
}
void launch_start_vector(double* x, Geom g, int level, hipStream_t st, uint64_t offset) {
  launch_k(start_vector_kernel, stencil_grid(g), dim3(BX, BY), st, x, g, level, offset);
}
void launch_scale(double* x, long n, const double* nrm2, hipStream_t st) {
  launch_k(scale_kernel, flat_blocks(n), 256, st, x, n, nrm2);
}

}  // namespace irk
