// Geometric multigrid V-cycle kernels for one diagonal stage block
// B = M + dt*a_ii*K (Section 3.1: the diagonal blocks of the block Jacobi /
// Gauss-Seidel stage preconditioners are approximated by multigrid).
//
// One level of the V-cycle is two kernels:
//   DOWN: Jacobi-Chebyshev pre-smoothing from a zero guess, fused with the
//         residual t - B x and its restriction P^T (full weighting) to the
//         next coarser level; writes x (needed again on the way up) and the
//         coarse right-hand side. Reads t and kappa once.
//   UP:   bilinear prolongation and correction x + P e, fused with
//         Jacobi-Chebyshev post-smoothing; writes the level's result.
// The coarsest level is solved with a precomputed dense inverse.
//
// Column-segment tiling. A block of NW wavefronts covers a region of 64 node
// columns x RY = NW*RW node rows: lane l of every wavefront owns column l, and
// wavefront w owns the RW consecutive rows from w*RW. A lane keeps everything
// about its own nodes in registers -- the right-hand side, the iterates and the
// nine weights of B's stencil (with 1/D), built once per launch from the four
// element diffusivities it loads straight from global memory -- so only the
// iterate being smoothed is exchanged through LDS, one buffer per Chebyshev
// step. Each stencil application invalidates one more node ring at the region's
// edge, so the tile a block writes is the region less a halo of H nodes (one per
// fused stencil application); the halo rings are recomputed by the neighbouring
// blocks. LDS rows are 64 values wide, so a wavefront's 64 lanes read
// consecutive words of one row (no bank conflicts).
//
// Storage type TS (FP64, FP32 or BF16) holds the level vectors; arithmetic and
// kappa use TC (FP64, or FP32 for both reduced-precision forms). TV is the type
// of the finest level's right-hand side and result (the FP64 Krylov vectors).
#include "mg_device.h"

namespace irk {
namespace {

constexpr int WL = 64;  // lanes per wavefront = region columns

// The nine stencil weights of B = m*(16,4,4,4,4,1,1,1,1) + alpha*K at one node and 1/D (D = the centre weight),
// from the diffusivities of the four elements around it (K's 9-point stencil: 2/3 sum(k) at the centre,
// -1/6 (sum of the two elements sharing an edge) at an edge neighbour, -1/3 k at a diagonal neighbour).
template <typename TC>
struct W9 {
  TC c, e, w, n, s, ne, nw, se, sw, dinv;
};

template <typename TC>
__device__ __forceinline__ W9<TC> stencil_weights(TC kSW, TC kSE, TC kNW, TC kNE, TC m, TC alpha) {
  const TC a6 = alpha * (TC)(1.0 / 6.0), a3 = alpha * (TC)(1.0 / 3.0);
  W9<TC> q;
  q.c = (TC)16 * m + alpha * (TC)(2.0 / 3.0) * (kSW + kSE + kNW + kNE);
  q.e = (TC)4 * m - a6 * (kNE + kSE);
  q.w = (TC)4 * m - a6 * (kNW + kSW);
  q.n = (TC)4 * m - a6 * (kNE + kNW);
  q.s = (TC)4 * m - a6 * (kSE + kSW);
  q.ne = m - a3 * kNE;
  q.nw = m - a3 * kNW;
  q.se = m - a3 * kSE;
  q.sw = m - a3 * kSW;
  q.dinv = recip(q.c);
  return q;
}

// LDS plane of the region with one spare row above and below and one spare word before and after, so that every
// neighbour address of a region node is inside the array (the spare words are zeroed once per launch)
template <int RY>
struct Plane {
  static constexpr int SIZE = (RY + 2) * WL + 2;
  __device__ static __forceinline__ int at(int r, int c) { return (r + 1) * WL + c + 1; }
};

template <typename TC, int RY>
__device__ __forceinline__ void zero_spare(TC* X) {
  const int t = threadIdx.x;
  if (t < WL + 1) X[t] = (TC)0;                               // word before and row above
  if (t < WL + 1) X[Plane<RY>::at(RY, 0) + t] = (TC)0;        // row below and word after
}

// Bx at this lane's RW nodes (column l, rows r0 .. r0+RW-1) from the iterate in LDS; own is the lane's own
// column of that iterate for those rows (the same values), so only the rows r0-1 and r0+RW of the own column
// and the two neighbour columns are read from LDS.
template <typename TC, int RY, int RW>
__device__ __forceinline__ void apply_b(const TC* X, int l, int r0, const W9<TC> (&w)[RW], const TC (&own)[RW],
                                        TC (&bx)[RW]) {
  using PL = Plane<RY>;
  TC sW = X[PL::at(r0 - 1, l - 1)], sC = X[PL::at(r0 - 1, l)], sE = X[PL::at(r0 - 1, l + 1)];
  TC cW = X[PL::at(r0, l - 1)], cE = X[PL::at(r0, l + 1)];
  TC cC = own[0];
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    const TC nW = X[PL::at(r0 + r + 1, l - 1)], nE = X[PL::at(r0 + r + 1, l + 1)];
    const TC nC = (r + 1 < RW) ? own[r + 1] : X[PL::at(r0 + RW, l)];
    bx[r] = w[r].c * cC + w[r].e * cE + w[r].w * cW + w[r].n * nC + w[r].s * sC + w[r].ne * nE + w[r].nw * nW +
            w[r].se * sE + w[r].sw * sW;
    sW = cW;
    sC = cC;
    sE = cE;
    cW = nW;
    cC = nC;
    cE = nE;
  }
}

template <typename TC, int RY, int RW>
__device__ __forceinline__ void store_rows(TC* X, int l, int r0, const TC (&v)[RW]) {
#pragma unroll
  for (int r = 0; r < RW; ++r) X[Plane<RY>::at(r0 + r, l)] = v[r];
}

// Element diffusivities around this lane's nodes: columns i-1 (kw) and i (ke), element rows j-1 .. j+RW-1 for the
// lane's first node row j; zero outside the N x N elements. All loads are issued before any is used.
template <typename TC, int RW>
__device__ __forceinline__ void load_kappa_cols(const TC* __restrict__ kap, int i, int jfirst, const Geom& g,
                                                TC (&kw)[RW + 1], TC (&ke)[RW + 1]) {
#pragma unroll
  for (int q = 0; q <= RW; ++q) {
    const int ey = jfirst - 1 + q;
    const bool oky = ey >= 0 && ey < g.N;
    const bool okw = oky && i - 1 >= 0 && i - 1 < g.N, oke = oky && i >= 0 && i < g.N;
    const TC a = kap[okw ? (long)ey * g.pitch + i - 1 : 0];
    const TC b = kap[oke ? (long)ey * g.pitch + i : 0];
    kw[q] = okw ? a : (TC)0;
    ke[q] = oke ? b : (TC)0;
  }
}

// Block-triangular stage coupling of the finest level (P_L, P_LD, P_U and the IA forms): the right-hand side
// becomes t - dt * K w (AI: K with the element diffusivities) or t - M w (IA) for w = sum_q a_q z_q, with w staged
// in LDS. Valid one node in from the region's edge.
template <typename TC, int RY, int RW>
__device__ __forceinline__ void couple_rows(const TC* W, int l, int r0, const TC (&wown)[RW], const TC (&kw)[RW + 1],
                                            const TC (&ke)[RW + 1], const Couple& cp, TC (&t)[RW]) {
  using PL = Plane<RY>;
  const TC dt = (TC)cp.dt, mh = (TC)cp.mh;
  TC sW = W[PL::at(r0 - 1, l - 1)], sC = W[PL::at(r0 - 1, l)], sE = W[PL::at(r0 - 1, l + 1)];
  TC cW = W[PL::at(r0, l - 1)], cE = W[PL::at(r0, l + 1)];
  TC cC = wown[0];
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    const TC nW = W[PL::at(r0 + r + 1, l - 1)], nE = W[PL::at(r0 + r + 1, l + 1)];
    const TC nC = (r + 1 < RW) ? wown[r + 1] : W[PL::at(r0 + RW, l)];
    TC op;
    if (cp.mass) {
      op = mh * ((TC)16 * cC + (TC)4 * (cE + cW + nC + sC) + (nE + nW + sE + sW));
    } else {
      const TC kSW = kw[r], kSE = ke[r], kNW = kw[r + 1], kNE = ke[r + 1];
      op = (TC)(2.0 / 3.0) * (kSW + kSE + kNW + kNE) * cC -
           (TC)(1.0 / 6.0) * ((kNE + kSE) * cE + (kNW + kSW) * cW + (kNE + kNW) * nC + (kSE + kSW) * sC) -
           (TC)(1.0 / 3.0) * (kNE * nE + kNW * nW + kSE * sE + kSW * sW);
    }
    t[r] -= dt * op;
    sW = cW;
    sC = cC;
    sE = cE;
    cW = nW;
    cC = nC;
    cE = nE;
  }
}

// DOWN. H = DEG + 1 halo rings (DEG stencil applications in the smoother and the residual take one ring each, the
// full-weighting restriction one more), one more with the stage coupling. The tile is even in both directions, so
// the coarse nodes of a tile (fine positions 2I, 2J) are whole.
// tout (optional): the level's right-hand side as the smoother sees it (scaled, coupling applied), stored on the
// tile in the compute type for the UP kernel of the same V-cycle.
template <typename TV, typename TS, typename TC, int DEG, int NW, int RW, bool COUPLE>
__global__ __launch_bounds__(NW* WL) void mg_down_kernel(const TV* __restrict__ t, const double* __restrict__ tscale,
                                                         TS* __restrict__ xout, TS* __restrict__ tc,
                                                         TC* __restrict__ tout, const TC* __restrict__ kap, Geom g,
                                                         Geom gc, MGCoef cf, Couple cp) {
  constexpr int RY = NW * RW;
  constexpr int H = DEG + 1 + (COUPLE ? 1 : 0);
  constexpr int TX = WL - 2 * H, TY = RY - 2 * H;
  static_assert(TX % 2 == 0 && TY > 0 && TY % 2 == 0, "tile must be even");
  using PL = Plane<RY>;
  __shared__ TC sA[PL::SIZE];
  __shared__ TC sB[PL::SIZE];
  const int N = g.N;
  const int l = threadIdx.x & (WL - 1), r0 = (threadIdx.x / WL) * RW;
  // tiles on a 1-D grid in XCD-aware order: neighbouring tiles (shared halos) run on the same XCD
  const int ntx = (N - 1 + TX - 1) / TX;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int i0 = 1 + (tile % ntx) * TX, j0 = 1 + (tile / ntx) * TY;
  const int ox = i0 - H, oy = j0 - H;
  const int i = ox + l, jf = oy + r0;
  const TC m = (TC)cf.m, alpha = (TC)cf.alpha;
  const TC ts = (TC)((tscale ? *tscale : 1.0) * cp.vmul);

  bool in[RW];
  long p[RW];
  TC tv[RW], kw[RW + 1], ke[RW + 1], wv[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    in[r] = interior(i, jf + r, N);
    p[r] = in[r] ? (long)(jf + r) * g.pitch + i : 0;
    tv[r] = ld<TC>(t + p[r]);
  }
  load_kappa_cols<TC, RW>(kap, i, jf, g, kw, ke);
  if (COUPLE) {
    // w = sum_q a_q z_q in FP64; the stage loop is unrolled over its bound with a uniform guard, so the loads of
    // all rows of a stage plane are in flight together
    double acc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) acc[r] = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxStages - 1; ++q) {
      if (q < cp.nz) {
        const double* zq = cp.z + q * cp.zstride;
        double zv[RW];
#pragma unroll
        for (int r = 0; r < RW; ++r) zv[r] = zq[p[r]];
#pragma unroll
        for (int r = 0; r < RW; ++r) acc[r] += cp.a[q] * zv[r];
      }
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) wv[r] = in[r] ? (TC)acc[r] : (TC)0;
  }
  zero_spare<TC, RY>(sA);
  zero_spare<TC, RY>(sB);
#pragma unroll
  for (int r = 0; r < RW; ++r) tv[r] = in[r] ? tv[r] * ts : (TC)0;
  if (COUPLE) {
    store_rows<TC, RY, RW>(sB, l, r0, wv);
    __syncthreads();
    couple_rows<TC, RY, RW>(sB, l, r0, wv, kw, ke, cp, tv);
  }
  W9<TC> w[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) w[r] = stencil_weights<TC>(kw[r], ke[r], kw[r + 1], ke[r + 1], m, alpha);
  // first Chebyshev step from x0 = 0 is pointwise: x1 = c0 D^{-1} t
  TC xc[RW], xp[RW], bx[RW];
  {
    const TC c0 = (TC)cf.c0;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      xc[r] = in[r] ? c0 * w[r].dinv * tv[r] : (TC)0;
      xp[r] = (TC)0;
    }
  }
  TC* cur = sA;
  TC* nxt = sB;
  store_rows<TC, RY, RW>(cur, l, r0, xc);
  __syncthreads();
#pragma unroll
  for (int k = 1; k < DEG; ++k) {
    const TC beta = (TC)cf.beta[k], gam = (TC)cf.gam[k];
    apply_b<TC, RY, RW>(cur, l, r0, w, xc, bx);
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const TC xn = in[r] ? xc[r] + beta * (xc[r] - xp[r]) + gam * (tv[r] - bx[r]) * w[r].dinv : (TC)0;
      xp[r] = xc[r];
      xc[r] = xn;
    }
    store_rows<TC, RY, RW>(nxt, l, r0, xc);
    __syncthreads();
    TC* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  // smoothed x (and the right-hand side) on the tile; the residual t - B x into the free buffer
  apply_b<TC, RY, RW>(cur, l, r0, w, xc, bx);
  const bool col_in_tile = l >= H && l < WL - H;
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    const int rr = r0 + r;
    if (col_in_tile && rr >= H && rr < RY - H && in[r]) {
      st(xout + p[r], xc[r]);
      if (tout) tout[p[r]] = tv[r];
    }
    bx[r] = in[r] ? tv[r] - bx[r] : (TC)0;
  }
  store_rows<TC, RY, RW>(nxt, l, r0, bx);
  __syncthreads();
  // full-weighting restriction (P^T of bilinear interpolation) to the coarse nodes of the tile
  {
    constexpr int CX = TX / 2, CY = TY / 2;
    const int I0 = (i0 + 1) / 2, J0 = (j0 + 1) / 2;
    for (int idx = threadIdx.x; idx < CX * CY; idx += NW * WL) {
      const int I = I0 + idx % CX, J = J0 + idx / CX;
      if (I > gc.N - 1 || J > gc.N - 1) continue;
      const TC* R = nxt + PL::at(2 * J - oy, 2 * I - ox);
      const TC v = R[0] + (TC)0.5 * (R[1] + R[-1] + R[WL] + R[-WL]) +
                   (TC)0.25 * (R[WL + 1] + R[WL - 1] + R[-WL + 1] + R[-WL - 1]);
      st(tc + (long)J * gc.pitch + I, v);
    }
  }
}

// UP. H = DEG halo rings (one per smoothing step). t: the level's right-hand side (finest level: the one the DOWN
// kernel stored, already scaled and coupled).
template <typename TT, typename TS, typename TO, typename TC, int DEG, int NW, int RW>
__global__ __launch_bounds__(NW* WL) void mg_up_kernel(const TT* __restrict__ t, const TS* __restrict__ x,
                                                       const TS* __restrict__ e, TO* __restrict__ out,
                                                       const TC* __restrict__ kap, Geom g, Geom gc, MGCoef cf) {
  constexpr int RY = NW * RW;
  constexpr int H = DEG;
  constexpr int TX = WL - 2 * H, TY = RY - 2 * H;
  static_assert(TY > 0, "region too small");
  using PL = Plane<RY>;
  __shared__ TC sA[PL::SIZE];
  __shared__ TC sB[PL::SIZE];
  const int N = g.N;
  const int l = threadIdx.x & (WL - 1), r0 = (threadIdx.x / WL) * RW;
  const int ntx = (N - 1 + TX - 1) / TX;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int i0 = 1 + (tile % ntx) * TX, j0 = 1 + (tile / ntx) * TY;
  const int ox = i0 - H, oy = j0 - H;
  const int i = ox + l, jf = oy + r0;
  const TC m = (TC)cf.m, alpha = (TC)cf.alpha;

  bool in[RW];
  TC tv[RW], xc[RW], xp[RW], bx[RW], kw[RW + 1], ke[RW + 1];
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    in[r] = interior(i, jf + r, N);
    const int ic = in[r] ? i : 1, jc = in[r] ? jf + r : 1;
    const long p = (long)jc * g.pitch + ic;
    const TC a = ld<TC>(t + p);
    const TC b = ld<TC>(x + p) + prolong_at<TS, TC>(e, gc.pitch, ic, jc);
    tv[r] = in[r] ? a : (TC)0;
    xp[r] = in[r] ? b : (TC)0;
  }
  load_kappa_cols<TC, RW>(kap, i, jf, g, kw, ke);
  zero_spare<TC, RY>(sA);
  zero_spare<TC, RY>(sB);
  store_rows<TC, RY, RW>(sA, l, r0, xp);
  W9<TC> w[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) w[r] = stencil_weights<TC>(kw[r], ke[r], kw[r + 1], ke[r + 1], m, alpha);
  __syncthreads();
  // first step from the corrected x0: x1 = x0 + c0 D^{-1} (t - B x0)
  apply_b<TC, RY, RW>(sA, l, r0, w, xp, bx);
  {
    const TC c0 = (TC)cf.c0;
#pragma unroll
    for (int r = 0; r < RW; ++r) xc[r] = in[r] ? xp[r] + c0 * (tv[r] - bx[r]) * w[r].dinv : (TC)0;
  }
  TC* cur = sA;
  TC* nxt = sB;
#pragma unroll
  for (int k = 1; k < DEG; ++k) {
    store_rows<TC, RY, RW>(nxt, l, r0, xc);
    __syncthreads();
    TC* tmp = cur;
    cur = nxt;
    nxt = tmp;
    const TC beta = (TC)cf.beta[k], gam = (TC)cf.gam[k];
    apply_b<TC, RY, RW>(cur, l, r0, w, xc, bx);
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const TC xn = in[r] ? xc[r] + beta * (xc[r] - xp[r]) + gam * (tv[r] - bx[r]) * w[r].dinv : (TC)0;
      xp[r] = xc[r];
      xc[r] = xn;
    }
  }
  const bool col_in_tile = l >= H && l < WL - H;
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    const int rr = r0 + r;
    if (col_in_tile && rr >= H && rr < RY - H && in[r]) st(out + (long)(jf + r) * g.pitch + i, xc[r]);
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

// Region shapes (NW wavefronts, RW rows per lane) by level size: enough blocks to occupy every CU, few enough that
// they are all resident at once, and regions tall enough that the halo rows stay a small share.
constexpr int kBigLevel = 1024, kMidLevel = 512;
constexpr int DNWB = 16, DRWB = 3, UNWB = 16, URWB = 3;  // N >= 1024 (DOWN, UP)
constexpr int DNWM = 8, DRWM = 2, UNWM = 8, URWM = 2;  // 512 <= N < 1024
constexpr int DNWS = 8, DRWS = 2, UNWS = 8, URWS = 2;  // N < 512

template <int NW, int RW, int H>
dim3 level_grid(const Geom& g) {
  constexpr int TX = WL - 2 * H, TY = NW * RW - 2 * H;
  return dim3(((g.N - 1 + TX - 1) / TX) * ((g.N - 1 + TY - 1) / TY));
}

template <typename TV, typename TS, typename TC, bool CP, int NW, int RW>
void down_shape(const TV* tt, const double* tscale, TS* xx, TS* cc, TC* to, const TC* kk, Geom g, Geom gc,
                const MGCoef& c, const Couple& cp, hipStream_t st) {
  constexpr int B = NW * WL, C = CP ? 1 : 0;
  switch (c.deg) {
    case 1:
      launch_k(mg_down_kernel<TV, TS, TC, 1, NW, RW, CP>, level_grid<NW, RW, 2 + C>(g), B, st, tt, tscale, xx, cc, to, kk, g, gc, c, cp);
      break;
    case 2:
      launch_k(mg_down_kernel<TV, TS, TC, 2, NW, RW, CP>, level_grid<NW, RW, 3 + C>(g), B, st, tt, tscale, xx, cc, to, kk, g, gc, c, cp);
      break;
    default:
      launch_k(mg_down_kernel<TV, TS, TC, 3, NW, RW, CP>, level_grid<NW, RW, 4 + C>(g), B, st, tt, tscale, xx, cc, to, kk, g, gc, c, cp);
      break;
  }
}

template <typename TV, typename TS, typename TC, bool CP>
void down_launch(const TV* tt, const double* tscale, TS* xx, TS* cc, TC* to, const TC* kk, Geom g, Geom gc,
                 const MGCoef& c, const Couple& cp, hipStream_t st) {
  if (g.N >= kBigLevel)
    down_shape<TV, TS, TC, CP, DNWB, DRWB>(tt, tscale, xx, cc, to, kk, g, gc, c, cp, st);
  else if (g.N >= kMidLevel)
    down_shape<TV, TS, TC, CP, DNWM, DRWM>(tt, tscale, xx, cc, to, kk, g, gc, c, cp, st);
  else
    down_shape<TV, TS, TC, CP, DNWS, DRWS>(tt, tscale, xx, cc, to, kk, g, gc, c, cp, st);
}

template <typename TV, typename TS, typename TC>
void down_t(const void* t, const double* tscale, void* x, void* tc, void* tout, const void* kap, Geom g, Geom gc,
            const MGCoef& c, const Couple& cp, hipStream_t st) {
  if (cp.nz > 0)
    down_launch<TV, TS, TC, true>((const TV*)t, tscale, (TS*)x, (TS*)tc, (TC*)tout, (const TC*)kap, g, gc, c, cp, st);
  else
    down_launch<TV, TS, TC, false>((const TV*)t, tscale, (TS*)x, (TS*)tc, (TC*)tout, (const TC*)kap, g, gc, c, cp, st);
}

template <typename TT, typename TS, typename TO, typename TC, int NW, int RW>
void up_shape(const TT* tt, const TS* xx, const TS* ee, TO* oo, const TC* kk, Geom g, Geom gc, const MGCoef& c,
              hipStream_t st) {
  constexpr int B = NW * WL;
  switch (c.deg) {
    case 1:
      launch_k(mg_up_kernel<TT, TS, TO, TC, 1, NW, RW>, level_grid<NW, RW, 1>(g), B, st, tt, xx, ee, oo, kk, g, gc, c);
      break;
    case 2:
      launch_k(mg_up_kernel<TT, TS, TO, TC, 2, NW, RW>, level_grid<NW, RW, 2>(g), B, st, tt, xx, ee, oo, kk, g, gc, c);
      break;
    default:
      launch_k(mg_up_kernel<TT, TS, TO, TC, 3, NW, RW>, level_grid<NW, RW, 3>(g), B, st, tt, xx, ee, oo, kk, g, gc, c);
      break;
  }
}

template <typename TT, typename TS, typename TO, typename TC>
void up_t(const void* t, const void* x, const void* e, void* out, const void* kap, Geom g, Geom gc, const MGCoef& c,
          hipStream_t st) {
  if (g.N >= kBigLevel)
    up_shape<TT, TS, TO, TC, UNWB, URWB>((const TT*)t, (const TS*)x, (const TS*)e, (TO*)out, (const TC*)kap, g, gc, c,
                                       st);
  else if (g.N >= kMidLevel)
    up_shape<TT, TS, TO, TC, UNWM, URWM>((const TT*)t, (const TS*)x, (const TS*)e, (TO*)out, (const TC*)kap, g, gc, c,
                                       st);
  else
    up_shape<TT, TS, TO, TC, UNWS, URWS>((const TT*)t, (const TS*)x, (const TS*)e, (TO*)out, (const TC*)kap, g, gc, c,
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
    launch_k(mg_coarse_kernel<double, double, double>, grid, NTC, st, (const double*)t, tscale, (double*)out,
                                                                 (const double*)Binv, g);
  } else if (io_is_f64) {
    launch_k(mg_coarse_kernel<double, double, float>, grid, NTC, st, (const double*)t, tscale, (double*)out,
                                                                (const float*)Binv, g);
  } else if (prec == 1) {
    launch_k(mg_coarse_kernel<float, float, float>, grid, NTC, st, (const float*)t, tscale, (float*)out,
                                                              (const float*)Binv, g);
  } else {
    launch_k(mg_coarse_kernel<bf16, bf16, float>, grid, NTC, st, (const bf16*)t, tscale, (bf16*)out, (const float*)Binv,
                                                            g);
  }
}

}  // namespace irk
