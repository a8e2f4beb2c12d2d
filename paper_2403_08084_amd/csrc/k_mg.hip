// Geometric multigrid V-cycle kernels for one diagonal stage block
// B = M + dt*a_ii*K (Section 3.1: the diagonal blocks of the block Jacobi /
// Gauss-Seidel stage preconditioners are approximated by multigrid).
//
// One level of the V-cycle is two LDS-tiled kernels:
//   DOWN: Jacobi-Chebyshev pre-smoothing from a zero guess, fused with the
//         residual t - B x and its restriction P^T (full weighting) to the
//         next coarser level; writes x (needed again on the way up) and the
//         coarse right-hand side. Reads t and kappa once.
//   UP:   bilinear prolongation and correction x + P e, fused with
//         Jacobi-Chebyshev post-smoothing; writes the level's result.
// Each block stages a tile of TX x TY nodes plus a halo (one node per fused
// stencil application) of the fields in LDS; the valid region shrinks by one
// node per stencil application until it is the tile. The diagonal D of B is
// recomputed from the four element diffusivities wherever it is needed.
// The coarsest level is solved with a precomputed dense inverse.
//
// Storage type TS (FP64, FP32 or BF16) holds the level vectors; arithmetic and
// kappa use TC (FP64, or FP32 for both reduced-precision forms). TV is the type
// of the finest level's right-hand side and result (the FP64 Krylov vectors).
#include "mg_device.h"

namespace irk {
namespace {

// threads per block of the level kernels: a tile phase has up to (TX + 2H)(TY + 2H) nodes, and 16 waves per
// block shorten each phase of these latency-bound kernels (measured: 1024 threads 9% faster than 256)
constexpr int NT = 1024;

// B x and D at LDS node (li, lj); X has row length RX, K (element field) row length KX = RX + 1
template <typename TC, int RX, int KX>
__device__ __forceinline__ void bx_d(const TC* X, const TC* K, int li, int lj, TC m, TC alpha, TC& Bx, TC& D) {
  const int p = lj * RX + li;
  const int q = lj * KX + li;
  const TC kSW = K[q], kSE = K[q + 1], kNW = K[q + KX], kNE = K[q + KX + 1];
  const TC xc = X[p], xE = X[p + 1], xW = X[p - 1], xN = X[p + RX], xS = X[p - RX];
  const TC xNE = X[p + RX + 1], xNW = X[p + RX - 1], xSE = X[p - RX + 1], xSW = X[p - RX - 1];
  const TC ks = kSW + kSE + kNW + kNE;
  const TC Kx = (TC)(2.0 / 3.0) * ks * xc -
                (TC)(1.0 / 6.0) * ((kNE + kSE) * xE + (kNW + kSW) * xW + (kNE + kNW) * xN + (kSE + kSW) * xS) -
                (TC)(1.0 / 3.0) * (kNE * xNE + kNW * xNW + kSE * xSE + kSW * xSW);
  const TC Mx = m * ((TC)16 * xc + (TC)4 * (xE + xW + xN + xS) + (xNE + xNW + xSE + xSW));
  Bx = Mx + alpha * Kx;
  D = (TC)16 * m + alpha * (TC)(2.0 / 3.0) * ks;
}

template <typename TC, int KX>
__device__ __forceinline__ TC diag_at(const TC* K, int li, int lj, TC m, TC alpha) {
  const int q = lj * KX + li;
  return (TC)16 * m + alpha * (TC)(2.0 / 3.0) * (K[q] + K[q + 1] + K[q + KX] + K[q + KX + 1]);
}




// Block-triangular stage coupling inside the finest-level tiles: w = sum_q a_q z_q is loaded on the
// region plus one node (row length RX + 2) together with the other tile loads, staged in LDS,
// and t -= dt * K w (AI form, with the region's kappa tile) or t -= M w (IA form) is applied on the
// region.
template <typename TC, int RX, int RY>
struct CoupleLoad {
  static constexpr int WX = RX + 2, CNT = WX * (RY + 2), NL = (CNT + NT - 1) / NT;
  TC v[NL];
  __device__ __forceinline__ void load(const Couple& cp, int ox, int oy, const Geom& g) {
#pragma unroll
    for (int r = 0; r < NL; ++r) {
      const int idx = threadIdx.x + r * NT;
      const int lj = idx / WX, li = idx - lj * WX;
      const int i = ox - 1 + li, j = oy - 1 + lj;
      const bool ok = idx < CNT && interior(i, j, g.N);
      const long p = ok ? (long)j * g.pitch + i : 0;
      double acc = 0.0;
      for (int q = 0; q < cp.nz; ++q) acc += cp.a[q] * cp.z[q * cp.zstride + p];
      v[r] = ok ? (TC)acc : (TC)0;
    }
  }
  __device__ __forceinline__ void store(TC* sW) const {
#pragma unroll
    for (int r = 0; r < NL; ++r) {
      const int idx = threadIdx.x + r * NT;
      if (idx < CNT) sW[idx] = v[r];
    }
  }
};

template <typename TC, int RX, int RY, int KX>
__device__ __forceinline__ void couple_apply(TC* sT, const TC* sW, const TC* sK, const Couple& cp, int ox, int oy,
                                             const Geom& g) {
  constexpr int WX = RX + 2;
  const TC dt = (TC)cp.dt;
  for (int idx = threadIdx.x; idx < RX * RY; idx += NT) {
    const int lj = idx / RX, li = idx - lj * RX;
    if (!interior(ox + li, oy + lj, g.N)) continue;
    const int p = (lj + 1) * WX + (li + 1);
    const int q = lj * KX + li;
    const TC kSW = sK[q], kSE = sK[q + 1], kNW = sK[q + KX], kNE = sK[q + KX + 1];
    TC opw;
    if (cp.mass) {
      opw = (TC)cp.mh * ((TC)16 * sW[p] + (TC)4 * (sW[p + 1] + sW[p - 1] + sW[p + WX] + sW[p - WX]) +
                         (sW[p + WX + 1] + sW[p + WX - 1] + sW[p - WX + 1] + sW[p - WX - 1]));
    } else {
      opw = (TC)(2.0 / 3.0) * (kSW + kSE + kNW + kNE) * sW[p] -
            (TC)(1.0 / 6.0) * ((kNE + kSE) * sW[p + 1] + (kNW + kSW) * sW[p - 1] + (kNE + kNW) * sW[p + WX] +
                               (kSE + kSW) * sW[p - WX]) -
            (TC)(1.0 / 3.0) * (kNE * sW[p + WX + 1] + kNW * sW[p + WX - 1] + kSE * sW[p - WX + 1] +
                               kSW * sW[p - WX - 1]);
    }
    sT[idx] -= dt * opw;
  }
}

// tout (optional): the level's right-hand side as the smoother sees it (scaled, coupling applied), stored on the
// tile in the compute type so that the UP kernel of the same V-cycle reads it instead of recomputing it
template <typename TV, typename TS, typename TC, int DEG, int TX, int TY, bool COUPLE>
__global__ __launch_bounds__(NT) void mg_down_kernel(const TV* __restrict__ t, const double* __restrict__ tscale, TS* __restrict__ xout,
                                                     TS* __restrict__ tc, TC* __restrict__ tout,
                                                     const TC* __restrict__ kap, Geom g, Geom gc, MGCoef cf,
                                                     Couple cp) {
  constexpr int H = DEG + 1;
  constexpr int RX = TX + 2 * H, RY = TY + 2 * H;
  constexpr int KX = RX + 1, KY = RY + 1;
  __shared__ TC sK[KX * KY];
  __shared__ TC sT[RX * RY];
  __shared__ TC sA[COUPLE ? (RX + 2) * (RY + 2) : RX * RY];  // also stages the coupling field
  __shared__ TC sB[RX * RY];
  const int N = g.N;
  // tiles on a 1-D grid in XCD-aware order: neighbouring tiles (shared halos) run on the same XCD
  const int ntx = (g.N - 1 + TX - 1) / TX;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int i0 = 1 + (tile % ntx) * TX, j0 = 1 + (tile / ntx) * TY;
  const int ox = i0 - H, oy = j0 - H;
  const TC m = (TC)cf.m, alpha = (TC)cf.alpha, ts = (TC)((tscale ? *tscale : 1.0) * cp.vmul);

  {
    constexpr int CNT = RX * RY, NL = (CNT + NT - 1) / NT;
    TC tv[NL];
#pragma unroll
    for (int r = 0; r < NL; ++r) {
      const int idx = threadIdx.x + r * NT;
      const int lj = idx / RX, li = idx - lj * RX;
      const int i = ox + li, j = oy + lj;
      const bool ok = idx < CNT && interior(i, j, N);
      const TC val = ld<TC>(t + (ok ? (long)j * g.pitch + i : 0));
      tv[r] = ok ? val * ts : (TC)0;
    }
    CoupleLoad<TC, RX, RY> w;
    if (COUPLE) w.load(cp, ox, oy, g);
    load_kappa_tile<TC, TC, KX, KY, NT>(sK, kap, ox, oy, g);
#pragma unroll
    for (int r = 0; r < NL; ++r) {
      const int idx = threadIdx.x + r * NT;
      if (idx < CNT) sT[idx] = tv[r];
    }
    if (COUPLE) w.store(sA);
  }
  __syncthreads();
  if (COUPLE) {
    couple_apply<TC, RX, RY, KX>(sT, sA, sK, cp, ox, oy, g);
    __syncthreads();
  }
  // first Chebyshev step from x0 = 0 is pointwise: x1 = c0 D^{-1} t (x_prev = 0 in sA)
  {
    const TC c0 = (TC)cf.c0;
    for (int idx = threadIdx.x; idx < RX * RY; idx += NT) {
      const int lj = idx / RX, li = idx - lj * RX;
      TC v = (TC)0;
      if (interior(ox + li, oy + lj, N)) v = c0 * sT[idx] * recip(diag_at<TC, KX>(sK, li, lj, m, alpha));
      sB[idx] = v;
      sA[idx] = (TC)0;
    }
  }
  __syncthreads();
  TC* cur = sB;
  TC* prv = sA;
#pragma unroll
  for (int k = 1; k < DEG; ++k) {
    const TC beta = (TC)cf.beta[k], gam = (TC)cf.gam[k];
    const int w = RX - 2 * k, hgt = RY - 2 * k;
    for (int idx = threadIdx.x; idx < w * hgt; idx += NT) {
      const int lj = k + idx / w, li = k + idx % w;
      if (!interior(ox + li, oy + lj, N)) continue;
      TC Bx, D;
      bx_d<TC, RX, KX>(cur, sK, li, lj, m, alpha, Bx, D);
      const int p = lj * RX + li;
      prv[p] = cur[p] + beta * (cur[p] - prv[p]) + gam * (sT[p] - Bx) * recip(D);
    }
    __syncthreads();
    TC* tmp = cur;
    cur = prv;
    prv = tmp;
  }
  // smoothed x (and the right-hand side) on the tile
  for (int idx = threadIdx.x; idx < TX * TY; idx += NT) {
    const int lj = H + idx / TX, li = H + idx % TX;
    const int i = ox + li, j = oy + lj;
    if (interior(i, j, N)) {
      st(xout + (long)j * g.pitch + i, cur[lj * RX + li]);
      if (tout) tout[(long)j * g.pitch + i] = sT[lj * RX + li];
    }
  }
  // residual on the tile plus one node
  {
    const int w = TX + 2, hgt = TY + 2;
    for (int idx = threadIdx.x; idx < w * hgt; idx += NT) {
      const int lj = H - 1 + idx / w, li = H - 1 + idx % w;
      const int p = lj * RX + li;
      TC r = (TC)0;
      if (interior(ox + li, oy + lj, N)) {
        TC Bx, D;
        bx_d<TC, RX, KX>(cur, sK, li, lj, m, alpha, Bx, D);
        r = sT[p] - Bx;
      }
      prv[p] = r;
    }
  }
  __syncthreads();
  // full-weighting restriction (P^T of bilinear interpolation) to coarse nodes centred in the tile
  {
    constexpr int CX = TX / 2, CY = TY / 2;
    const int I0 = (i0 + 1) / 2, J0 = (j0 + 1) / 2;
    for (int idx = threadIdx.x; idx < CX * CY; idx += NT) {
      const int I = I0 + idx % CX, J = J0 + idx / CX;
      if (I > gc.N - 1 || J > gc.N - 1) continue;
      const int li = 2 * I - ox, lj = 2 * J - oy;
      const TC* R = prv + lj * RX + li;
      const TC v = R[0] + (TC)0.5 * (R[1] + R[-1] + R[RX] + R[-RX]) +
                   (TC)0.25 * (R[RX + 1] + R[RX - 1] + R[-RX + 1] + R[-RX - 1]);
      st(tc + (long)J * gc.pitch + I, v);
    }
  }
}

// t: the level's right-hand side (finest level: the one the DOWN kernel stored, already scaled and coupled)
template <typename TT, typename TS, typename TO, typename TC, int DEG, int TX, int TY>
__global__ __launch_bounds__(NT) void mg_up_kernel(const TT* __restrict__ t, const TS* __restrict__ x,
                                                   const TS* __restrict__ e, TO* __restrict__ out,
                                                   const TC* __restrict__ kap, Geom g, Geom gc, MGCoef cf) {
  constexpr int H = DEG;
  constexpr int RX = TX + 2 * H, RY = TY + 2 * H;
  constexpr int KX = RX + 1, KY = RY + 1;
  __shared__ TC sK[KX * KY];
  __shared__ TC sT[RX * RY];
  __shared__ TC sA[RX * RY];
  __shared__ TC sB[RX * RY];
  const int N = g.N;
  // tiles on a 1-D grid in XCD-aware order: neighbouring tiles (shared halos) run on the same XCD
  const int ntx = (g.N - 1 + TX - 1) / TX;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int i0 = 1 + (tile % ntx) * TX, j0 = 1 + (tile / ntx) * TY;
  const int ox = i0 - H, oy = j0 - H;
  const TC m = (TC)cf.m, alpha = (TC)cf.alpha;

  {
    constexpr int CNT = RX * RY, NL = (CNT + NT - 1) / NT;
    TC tv[NL], xv[NL];
#pragma unroll
    for (int r = 0; r < NL; ++r) {
      const int idx = threadIdx.x + r * NT;
      const int lj = idx / RX, li = idx - lj * RX;
      const int i = ox + li, j = oy + lj;
      const bool ok = idx < CNT && interior(i, j, N);
      const int ic = ok ? i : 1, jc = ok ? j : 1;
      const long p = (long)jc * g.pitch + ic;
      const TC a = ld<TC>(t + p);
      const TC b = ld<TC>(x + p) + prolong_at<TS, TC>(e, gc.pitch, ic, jc);
      tv[r] = ok ? a : (TC)0;
      xv[r] = ok ? b : (TC)0;
    }
    load_kappa_tile<TC, TC, KX, KY, NT>(sK, kap, ox, oy, g);
#pragma unroll
    for (int r = 0; r < NL; ++r) {
      const int idx = threadIdx.x + r * NT;
      if (idx < CNT) {
        sT[idx] = tv[r];
        sA[idx] = xv[r];
      }
    }
  }
  __syncthreads();
  // first step from the corrected x0: x1 = x0 + c0 D^{-1} (t - B x0), written on the whole
  // inner region (zero outside the domain); the region's edge ring of sB is never read again
  {
    const TC c0 = (TC)cf.c0;
    const int w = RX - 2, hgt = RY - 2;
    for (int idx = threadIdx.x; idx < w * hgt; idx += NT) {
      const int lj = 1 + idx / w, li = 1 + idx % w;
      const int p = lj * RX + li;
      TC v = (TC)0;
      if (interior(ox + li, oy + lj, N)) {
        TC Bx, D;
        bx_d<TC, RX, KX>(sA, sK, li, lj, m, alpha, Bx, D);
        v = sA[p] + c0 * (sT[p] - Bx) * recip(D);
      }
      sB[p] = v;
    }
  }
  __syncthreads();
  TC* cur = sB;
  TC* prv = sA;
#pragma unroll
  for (int k = 1; k < DEG; ++k) {
    const TC beta = (TC)cf.beta[k], gam = (TC)cf.gam[k];
    const int w = RX - 2 * (k + 1), hgt = RY - 2 * (k + 1);
    for (int idx = threadIdx.x; idx < w * hgt; idx += NT) {
      const int lj = k + 1 + idx / w, li = k + 1 + idx % w;
      if (!interior(ox + li, oy + lj, N)) continue;
      TC Bx, D;
      bx_d<TC, RX, KX>(cur, sK, li, lj, m, alpha, Bx, D);
      const int p = lj * RX + li;
      prv[p] = cur[p] + beta * (cur[p] - prv[p]) + gam * (sT[p] - Bx) * recip(D);
    }
    __syncthreads();
    TC* tmp = cur;
    cur = prv;
    prv = tmp;
  }
  for (int idx = threadIdx.x; idx < TX * TY; idx += NT) {
    const int lj = H + idx / TX, li = H + idx % TX;
    const int i = ox + li, j = oy + lj;
    if (interior(i, j, N)) st(out + (long)j * g.pitch + i, cur[lj * RX + li]);
  }
}

// Coarsest level: out = Binv * t on the n = (N-1)^2 <= 1024 interior nodes. One wavefront per
// row; each lane issues all of its (at most 16) coalesced row loads and right-hand-side loads
// before accumulating, then a fixed-order wavefront reduction.
// Blocks of NTC = 256 threads (four rows each): spreading the rows over many CUs matters more here than
// the level kernels' large blocks.
constexpr int NTC = 256;
template <typename TI, typename TO, typename TC>
__global__ __launch_bounds__(NTC) void mg_coarse_kernel(const TI* __restrict__ t, const double* __restrict__ tscale,
                                                        TO* __restrict__ out, const TC* __restrict__ Binv, Geom g) {
  const int m = g.N - 1;
  const int n = m * m;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (NTC / 64) + (threadIdx.x >> 6);
  if (row >= n) return;
  const TC* r = Binv + (long)row * n;
  constexpr int U = kMaxCoarse / 64;
  TC bv[U], tv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int c = lane + 64 * u;
    const int cc = c < n ? c : 0;
    const int j = cc / m + 1, i = cc - (j - 1) * m + 1;
    bv[u] = r[cc];
    tv[u] = ld<TC>(t + (long)j * g.pitch + i);
  }
  TC acc = (TC)0;
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (lane + 64 * u < n) acc += bv[u] * tv[u];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) {
    const TC tsc = tscale ? (TC)(*tscale) : (TC)1;
    const int j = row / m + 1, i = row % m + 1;
    st(out + (long)j * g.pitch + i, acc * tsc);
  }
}

// Tiles: 64 x 16 on large levels (coalesced rows, small halo share); on levels below 512^2, where a
// level is latency-bound, 32 x 8 tiles spread the work of each smoothing phase over four times more
// waves.
constexpr int TXD = 64, TYD = 16, TXS = 32, TYS = 8;
constexpr int kSmallLevel = 512;

template <typename TV, typename TS, typename TC, bool CP, int TX, int TY>
void down_tiles(const TV* tt, const double* tscale, TS* xx, TS* cc, TC* to, const TC* kk, Geom g, Geom gc,
                const MGCoef& c, const Couple& cp, hipStream_t st) {
  const dim3 grid(((g.N - 1 + TX - 1) / TX) * ((g.N - 1 + TY - 1) / TY));
  switch (c.deg) {
    case 1:
      mg_down_kernel<TV, TS, TC, 1, TX, TY, CP><<<grid, NT, 0, st>>>(tt, tscale, xx, cc, to, kk, g, gc, c, cp);
      break;
    case 2:
      mg_down_kernel<TV, TS, TC, 2, TX, TY, CP><<<grid, NT, 0, st>>>(tt, tscale, xx, cc, to, kk, g, gc, c, cp);
      break;
    default:
      mg_down_kernel<TV, TS, TC, 3, TX, TY, CP><<<grid, NT, 0, st>>>(tt, tscale, xx, cc, to, kk, g, gc, c, cp);
      break;
  }
}

template <typename TV, typename TS, typename TC, bool CP>
void down_launch(const TV* tt, const double* tscale, TS* xx, TS* cc, TC* to, const TC* kk, Geom g, Geom gc,
                 const MGCoef& c, const Couple& cp, hipStream_t st) {
  if (g.N < kSmallLevel)
    down_tiles<TV, TS, TC, CP, TXS, TYS>(tt, tscale, xx, cc, to, kk, g, gc, c, cp, st);
  else
    down_tiles<TV, TS, TC, CP, TXD, TYD>(tt, tscale, xx, cc, to, kk, g, gc, c, cp, st);
}

template <typename TV, typename TS, typename TC>
void down_t(const void* t, const double* tscale, void* x, void* tc, void* tout, const void* kap, Geom g, Geom gc,
            const MGCoef& c, const Couple& cp, hipStream_t st) {
  if (cp.nz > 0)
    down_launch<TV, TS, TC, true>((const TV*)t, tscale, (TS*)x, (TS*)tc, (TC*)tout, (const TC*)kap, g, gc, c, cp, st);
  else
    down_launch<TV, TS, TC, false>((const TV*)t, tscale, (TS*)x, (TS*)tc, (TC*)tout, (const TC*)kap, g, gc, c, cp, st);
}

template <typename TT, typename TS, typename TO, typename TC, int TX, int TY>
void up_tiles(const TT* tt, const TS* xx, const TS* ee, TO* oo, const TC* kk, Geom g, Geom gc, const MGCoef& c,
              hipStream_t st) {
  const dim3 grid(((g.N - 1 + TX - 1) / TX) * ((g.N - 1 + TY - 1) / TY));
  switch (c.deg) {
    case 1: mg_up_kernel<TT, TS, TO, TC, 1, TX, TY><<<grid, NT, 0, st>>>(tt, xx, ee, oo, kk, g, gc, c); break;
    case 2: mg_up_kernel<TT, TS, TO, TC, 2, TX, TY><<<grid, NT, 0, st>>>(tt, xx, ee, oo, kk, g, gc, c); break;
    default: mg_up_kernel<TT, TS, TO, TC, 3, TX, TY><<<grid, NT, 0, st>>>(tt, xx, ee, oo, kk, g, gc, c); break;
  }
}

template <typename TT, typename TS, typename TO, typename TC>
void up_t(const void* t, const void* x, const void* e, void* out, const void* kap, Geom g, Geom gc, const MGCoef& c,
          hipStream_t st) {
  if (g.N < kSmallLevel)
    up_tiles<TT, TS, TO, TC, TXS, TYS>((const TT*)t, (const TS*)x, (const TS*)e, (TO*)out, (const TC*)kap, g, gc, c,
                                       st);
  else
    up_tiles<TT, TS, TO, TC, TXD, TYD>((const TT*)t, (const TS*)x, (const TS*)e, (TO*)out, (const TC*)kap, g, gc, c,
                                       st);
}

}  // namespace

void launch_mg_down(int prec, bool t_is_f64, const void* t, const double* tscale, void* x, void* tc, void* tout,
                    const void* kappa, Geom g, Geom gc, const MGCoef& c, const Couple& cp, hipStream_t st) {
  if (prec == 0) {
    down_t<double, double, double>(t, tscale, x, tc, tout, kappa, g, gc, c, cp, st);
  } else if (prec == 1) {
    if (t_is_f64)
      down_t<double, float, float>(t, tscale, x, tc, tout, kappa, g, gc, c, cp, st);
    else
      down_t<float, float, float>(t, tscale, x, tc, tout, kappa, g, gc, c, cp, st);
  } else {
    if (t_is_f64)
      down_t<double, bf16, float>(t, tscale, x, tc, tout, kappa, g, gc, c, cp, st);
    else
      down_t<bf16, bf16, float>(t, tscale, x, tc, tout, kappa, g, gc, c, cp, st);
  }
}

void launch_mg_up(int prec, bool finest, const void* t, const void* x, const void* e, void* out, const void* kappa,
                  Geom g, Geom gc, const MGCoef& c, hipStream_t st) {
  if (prec == 0) {
    up_t<double, double, double, double>(t, x, e, out, kappa, g, gc, c, st);
  } else if (prec == 1) {
    if (finest)
      up_t<float, float, double, float>(t, x, e, out, kappa, g, gc, c, st);
    else
      up_t<float, float, float, float>(t, x, e, out, kappa, g, gc, c, st);
  } else {
    if (finest)
      up_t<float, bf16, double, float>(t, x, e, out, kappa, g, gc, c, st);
    else
      up_t<bf16, bf16, bf16, float>(t, x, e, out, kappa, g, gc, c, st);
  }
}

void launch_mg_coarse(int prec, bool io_is_f64, const void* t, const double* tscale, void* out, const void* Binv, Geom g,
                      hipStream_t st) {
  const int n = (g.N - 1) * (g.N - 1);
  const dim3 grid((n + NTC / 64 - 1) / (NTC / 64));
  if (prec == 0) {
    mg_coarse_kernel<double, double, double><<<grid, NTC, 0, st>>>((const double*)t, tscale, (double*)out,
                                                                 (const double*)Binv, g);
  } else if (io_is_f64) {
    mg_coarse_kernel<double, double, float><<<grid, NTC, 0, st>>>((const double*)t, tscale, (double*)out,
                                                                (const float*)Binv, g);
  } else if (prec == 1) {
    mg_coarse_kernel<float, float, float><<<grid, NTC, 0, st>>>((const float*)t, tscale, (float*)out,
                                                              (const float*)Binv, g);
  } else {
    mg_coarse_kernel<bf16, bf16, float><<<grid, NTC, 0, st>>>((const bf16*)t, tscale, (bf16*)out, (const float*)Binv,
                                                            g);
  }
}

}  // namespace irk

