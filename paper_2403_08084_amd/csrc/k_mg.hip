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
// of the finest level's right-hand side (the FP64 Krylov vector); the finest
// result TO is FP64, or FP32 for the reduced-precision forms' flexible basis
// (it holds the TC values either way), and TZ the type of the coupled stages.
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

// Keeps the weights' computation ahead of the next barrier: left alone, the compiler sinks it to the first use
// after the barrier, where it can no longer overlap the global loads still in flight (an empty statement that
// only reads the values; it emits no instruction).
template <typename TC, int RW>
__device__ __forceinline__ void weights_ready(const W9<TC> (&w)[RW]) {
#pragma unroll
  for (int r = 0; r < RW; ++r)
    asm volatile("" ::"v"(w[r].c), "v"(w[r].e), "v"(w[r].w), "v"(w[r].n), "v"(w[r].s), "v"(w[r].ne), "v"(w[r].nw),
                 "v"(w[r].se), "v"(w[r].sw), "v"(w[r].dinv));
}

// A value from the adjacent lane of the wavefront (DPP wavefront shift by one lane: kDppFromLower gives lane l the
// value of lane l - 1, kDppFromUpper that of lane l + 1; the lane without a source gets 0)
constexpr int kDppFromLower = 0x138, kDppFromUpper = 0x130;
template <typename TC, int CTRL>
__device__ __forceinline__ TC lane_shift(TC v);
template <>
__device__ __forceinline__ float lane_shift<float, kDppFromLower>(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), kDppFromLower, 0xF, 0xF, false));
}
template <>
__device__ __forceinline__ float lane_shift<float, kDppFromUpper>(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), kDppFromUpper, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift_f64(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xFFFFFFFFll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
template <>
__device__ __forceinline__ double lane_shift<double, kDppFromLower>(double v) { return lane_shift_f64<kDppFromLower>(v); }
template <>
__device__ __forceinline__ double lane_shift<double, kDppFromUpper>(double v) { return lane_shift_f64<kDppFromUpper>(v); }

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
    const TC a = kap[okw ? (unsigned)ey * g.pitch + i - 1 : 0];
    const TC b = kap[oke ? (unsigned)ey * g.pitch + i : 0];
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
template <typename TV, typename TS, typename TC, int DEG, int NW, int RW, bool COUPLE, typename TZ>
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
  unsigned p[RW];
  TC tv[RW], kw[RW + 1], ke[RW + 1], wv[RW];
  // diffusivities first: the stencil weights are formed while the right-hand side's loads are still in flight
  load_kappa_cols<TC, RW>(kap, i, jf, g, kw, ke);
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    in[r] = interior(i, jf + r, N);
    p[r] = in[r] ? (unsigned)(jf + r) * g.pitch + i : 0;
    tv[r] = ld<TC>(t + p[r]);
  }
  if (COUPLE) {
    // w = sum_q a_q z_q in FP64; the stage loop is unrolled over its bound with a uniform guard, so the loads of
    // all rows of a stage plane are in flight together (loading two planes ahead of the guard would take the
    // kernel past 64 registers, half the occupancy)
    double acc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) acc[r] = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxStages - 1; ++q) {
      if (q < cp.nz) {
        const TZ* zq = (const TZ*)cp.z + q * cp.zstride;
        double zv[RW];
#pragma unroll
        for (int r = 0; r < RW; ++r) zv[r] = (double)zq[p[r]];
#pragma unroll
        for (int r = 0; r < RW; ++r) acc[r] += cp.a[q] * zv[r];
      }
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) wv[r] = in[r] ? (TC)acc[r] : (TC)0;
  }
  // the stencil weights need only the diffusivities, loaded first: without coupling they are formed while the
  // right-hand side's loads are in flight; with it, after the coupling (earlier, the kernel would need more than
  // 64 registers, half the occupancy)
  W9<TC> w[RW];
  if constexpr (!COUPLE) {
#pragma unroll
    for (int r = 0; r < RW; ++r) w[r] = stencil_weights<TC>(kw[r], ke[r], kw[r + 1], ke[r + 1], m, alpha);
    weights_ready<TC, RW>(w);
  }
  zero_spare<TC, RY>(sA);
  zero_spare<TC, RY>(sB);
#pragma unroll
  for (int r = 0; r < RW; ++r) tv[r] = in[r] ? tv[r] * ts : (TC)0;
  if constexpr (COUPLE) {
    store_rows<TC, RY, RW>(sB, l, r0, wv);
    __syncthreads();
    couple_rows<TC, RY, RW>(sB, l, r0, wv, kw, ke, cp, tv);
#pragma unroll
    for (int r = 0; r < RW; ++r) w[r] = stencil_weights<TC>(kw[r], ke[r], kw[r + 1], ke[r + 1], m, alpha);
  }
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
  // full-weighting restriction (P^T of bilinear interpolation) to the coarse nodes of the tile. The wavefront spans
  // the region's 64 columns, so each lane's row neighbours come from the adjacent lanes by wavefront shifts (no LDS
  // reads at stride 2, which would put two lanes on each bank); the coarse columns' row sums go to a compact plane
  // (row stride CS, rows two apart half the banks apart) in the buffer of the previous iterate, free now, and each
  // half-wavefront then weights three rows of that plane for one coarse row.
  {
    constexpr int CX = TX / 2, CY = TY / 2, CS = 48;
    static_assert(CX <= 32 && RY * CS <= PL::SIZE, "compact restriction plane");
    const int I0 = (i0 + 1) / 2, J0 = (j0 + 1) / 2;
    const int c0 = 2 * I0 - ox;  // local column of the tile's first coarse column
    const bool ccol = l >= c0 && l < c0 + 2 * CX && ((l - c0) & 1) == 0;
    const int cc = (l - c0) >> 1;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const TC left = lane_shift<TC, kDppFromLower>(bx[r]), right = lane_shift<TC, kDppFromUpper>(bx[r]);
      if (ccol) nxt[(r0 + r) * CS + cc] = bx[r] + (TC)0.5 * (left + right);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 32 * CY; k += NW * WL) {
      const int kc = k & 31, cj = k >> 5;
      const int I = I0 + kc, J = J0 + cj;
      if (kc >= CX || I > gc.N - 1 || J > gc.N - 1) continue;
      const TC* hrow = nxt + (2 * J - oy) * CS + kc;
      st(tc + (unsigned)J * gc.pitch + I, hrow[0] + (TC)0.5 * (hrow[-CS] + hrow[CS]));
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
  // diffusivities first: the stencil weights are formed while the iterate's loads are still in flight
  load_kappa_cols<TC, RW>(kap, i, jf, g, kw, ke);
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    in[r] = interior(i, jf + r, N);
    const int ic = in[r] ? i : 1, jc = in[r] ? jf + r : 1;
    const unsigned p = (unsigned)jc * g.pitch + ic;
    const TC a = ld<TC>(t + p);
    const TC b = ld<TC>(x + p) + prolong_at<TS, TC>(e, gc.pitch, ic, jc);
    tv[r] = in[r] ? a : (TC)0;
    xp[r] = in[r] ? b : (TC)0;
  }
  W9<TC> w[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) w[r] = stencil_weights<TC>(kw[r], ke[r], kw[r + 1], ke[r + 1], m, alpha);
  weights_ready<TC, RW>(w);
  zero_spare<TC, RY>(sA);
  zero_spare<TC, RY>(sB);
  store_rows<TC, RY, RW>(sA, l, r0, xp);
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
    if (col_in_tile && rr >= H && rr < RY - H && in[r]) st(out + (unsigned)(jf + r) * g.pitch + i, xc[r]);
  }
}

// ---------------------------------------------------------------- three levels in one launch
// The levels above the coarsest, A, B = A/2 and C = B/2 (256², 128², 64² over the 32² coarsest solve of a 1024²
// grid), are short chains of dependent phases whose cost is mostly the launch and the round trips through global
// memory. DOWN3 does their three DOWN steps in one launch: it smooths A on a 64-column region in column segments (as
// mg_down_kernel), restricts the residual into an LDS region of B, smooths that, restricts into an LDS region of C,
// smooths that and restricts C's residual to D. UP3 does the three UP steps from D's correction to A. Each block's
// regions are deep enough that it needs nothing from its neighbours: the tiles nest (a C tile of CT nodes, a B tile
// of 2CT, an A tile of 4CT for DOWN3), and the halo rings of every level are recomputed by the neighbouring blocks.
// The two lower levels are stored flat in LDS (W x W nodes, row stride W; element tile (W+1) x (W+1) from one
// element below-left of the region), one node per thread and loop step.

// B x at flat node (li, lj) (and the diagonal D)
template <typename TC, int W>
__device__ __forceinline__ TC flat_bx(const TC* X, const TC* K, int li, int lj, TC m, TC alpha, TC& D) {
  const int p = lj * W + li, q = lj * (W + 1) + li;
  const TC kSW = K[q], kSE = K[q + 1], kNW = K[q + W + 1], kNE = K[q + W + 2];
  const TC xc = X[p], xE = X[p + 1], xW = X[p - 1], xN = X[p + W], xS = X[p - W];
  const TC xNE = X[p + W + 1], xNW = X[p + W - 1], xSE = X[p - W + 1], xSW = X[p - W - 1];
  const TC ks = kSW + kSE + kNW + kNE;
  const TC Kx = (TC)(2.0 / 3.0) * ks * xc -
                (TC)(1.0 / 6.0) * ((kNE + kSE) * xE + (kNW + kSW) * xW + (kNE + kNW) * xN + (kSE + kSW) * xS) -
                (TC)(1.0 / 3.0) * (kNE * xNE + kNW * xNW + kSE * xSE + kSW * xSW);
  const TC Mx = m * ((TC)16 * xc + (TC)4 * (xE + xW + xN + xS) + (xNE + xNW + xSE + xSW));
  D = (TC)16 * m + alpha * (TC)(2.0 / 3.0) * ks;
  return Mx + alpha * Kx;
}

// element tile of a flat region at level origin (ox, oy): (W+1) x (HM+1) diffusivities from element (ox-1, oy-1),
// all loads issued before the first store
template <typename TC, int W, int HM, int NT>
__device__ __forceinline__ void flat_kappa(TC* K, const TC* __restrict__ kap, int ox, int oy, const Geom& g) {
  constexpr int CNT = (W + 1) * (HM + 1), NL = (CNT + NT - 1) / NT;
  TC v[NL];
#pragma unroll
  for (int r = 0; r < NL; ++r) {
    const int idx = threadIdx.x + r * NT;
    const int b = idx / (W + 1), a = idx - b * (W + 1);
    const int ex = ox - 1 + a, ey = oy - 1 + b;
    const bool ok = idx < CNT && ex >= 0 && ex < g.N && ey >= 0 && ey < g.N;
    const TC x = kap[ok ? (unsigned)ey * g.pitch + ex : 0];
    v[r] = ok ? x : (TC)0;
  }
#pragma unroll
  for (int r = 0; r < NL; ++r) {
    const int idx = threadIdx.x + r * NT;
    if (idx < CNT) K[idx] = v[r];
  }
}

// DOWN smoothing on a flat Rx x Ry region (row stride W, at most HM rows) with right-hand side T: Chebyshev from
// zero, then the residual. Returns through x and r the buffers (of P0, P1) holding x_deg (valid from ring deg - 1)
// and the residual (valid from ring deg). Ends with a barrier.
template <typename TC, int W, int HM, int NT>
__device__ void flat_down(const TC* T, TC* P0, TC* P1, const TC* K, int Rx, int Ry, int ox, int oy, int N,
                          const MGCoef& cf, TC*& x, TC*& r) {
  const TC m = (TC)cf.m, alpha = (TC)cf.alpha, c0 = (TC)cf.c0;
  for (int idx = threadIdx.x; idx < W * HM; idx += NT) {
    const int lj = idx / W, li = idx - lj * W;
    if (li >= Rx || lj >= Ry) continue;
    const int q = lj * (W + 1) + li;
    TC v = (TC)0;
    if (interior(ox + li, oy + lj, N)) {
      const TC D = (TC)16 * m + alpha * (TC)(2.0 / 3.0) * (K[q] + K[q + 1] + K[q + W + 1] + K[q + W + 2]);
      v = c0 * T[idx] * recip(D);
    }
    P0[idx] = v;
    P1[idx] = (TC)0;
  }
  __syncthreads();
  TC* cur = P0;
  TC* prv = P1;
  for (int k = 1; k < cf.deg; ++k) {
    const TC beta = (TC)cf.beta[k], gam = (TC)cf.gam[k];
    for (int idx = threadIdx.x; idx < W * HM; idx += NT) {
      const int lj = idx / W, li = idx - lj * W;
      if (li < k || li >= Rx - k || lj < k || lj >= Ry - k || !interior(ox + li, oy + lj, N)) continue;
      TC D;
      const TC bx = flat_bx<TC, W>(cur, K, li, lj, m, alpha, D);
      prv[idx] = cur[idx] + beta * (cur[idx] - prv[idx]) + gam * (T[idx] - bx) * recip(D);
    }
    __syncthreads();
    TC* tmp = cur;
    cur = prv;
    prv = tmp;
  }
  const int dg = cf.deg;
  for (int idx = threadIdx.x; idx < W * HM; idx += NT) {
    const int lj = idx / W, li = idx - lj * W;
    if (li < dg || li >= Rx - dg || lj < dg || lj >= Ry - dg) continue;
    TC v = (TC)0;
    if (interior(ox + li, oy + lj, N)) {
      TC D;
      v = T[idx] - flat_bx<TC, W>(cur, K, li, lj, m, alpha, D);
    }
    prv[idx] = v;
  }
  __syncthreads();
  x = cur;
  r = prv;
}

// UP smoothing on a flat Rx x Ry region from x0 in P0 (Chebyshev steps with right-hand side T). Returns the buffer
// holding the result (valid from ring deg). Ends with a barrier.
template <typename TC, int W, int HM, int NT>
__device__ TC* flat_up(const TC* T, TC* P0, TC* P1, const TC* K, int Rx, int Ry, int ox, int oy, int N,
                       const MGCoef& cf) {
  const TC m = (TC)cf.m, alpha = (TC)cf.alpha, c0 = (TC)cf.c0;
  for (int idx = threadIdx.x; idx < W * HM; idx += NT) {
    const int lj = idx / W, li = idx - lj * W;
    if (li < 1 || li >= Rx - 1 || lj < 1 || lj >= Ry - 1) continue;
    TC v = (TC)0;
    if (interior(ox + li, oy + lj, N)) {
      TC D;
      const TC bx = flat_bx<TC, W>(P0, K, li, lj, m, alpha, D);
      v = P0[idx] + c0 * (T[idx] - bx) * recip(D);
    }
    P1[idx] = v;
  }
  __syncthreads();
  TC* cur = P1;
  TC* prv = P0;
  for (int k = 1; k < cf.deg; ++k) {
    const TC beta = (TC)cf.beta[k], gam = (TC)cf.gam[k];
    for (int idx = threadIdx.x; idx < W * HM; idx += NT) {
      const int lj = idx / W, li = idx - lj * W;
      if (li < k + 1 || li >= Rx - k - 1 || lj < k + 1 || lj >= Ry - k - 1 || !interior(ox + li, oy + lj, N))
        continue;
      TC D;
      const TC bx = flat_bx<TC, W>(cur, K, li, lj, m, alpha, D);
      prv[idx] = cur[idx] + beta * (cur[idx] - prv[idx]) + gam * (T[idx] - bx) * recip(D);
    }
    __syncthreads();
    TC* tmp = cur;
    cur = prv;
    prv = tmp;
  }
  return cur;
}

// full weighting of the residual region R (row stride W, level origin (ox, oy)) at coarse node (I, J)
template <typename TC, int W>
__device__ __forceinline__ TC flat_restrict(const TC* R, int ox, int oy, int I, int J) {
  const TC* c = R + (2 * J - oy) * W + (2 * I - ox);
  return c[0] + (TC)0.5 * (c[1] + c[-1] + c[W] + c[-W]) + (TC)0.25 * (c[W + 1] + c[W - 1] + c[-W + 1] + c[-W - 1]);
}

// bilinear interpolation at fine node (i, j) of a coarse field stored flat (row stride W, level origin (ox, oy))
template <typename TC, int W>
__device__ __forceinline__ TC flat_prolong(const TC* E, int ox, int oy, int i, int j) {
  const TC* b = E + ((j >> 1) - oy) * W + ((i >> 1) - ox);
  const TC wx = (i & 1) ? (TC)0.5 : (TC)0, wy = (j & 1) ? (TC)0.5 : (TC)0;
  return ((TC)1 - wx) * ((TC)1 - wy) * b[0] + wx * ((TC)1 - wy) * b[1] + ((TC)1 - wx) * wy * b[W] + wx * wy * b[W + 1];
}

// DOWN3 geometry: C tile CT (even), flat regions RC, RB, the A region RA <= 64 columns
template <int DEG>
struct Down3 {
  static constexpr int H = DEG + 1;
  static constexpr int CT = ((WL - 8 * H - 6 * DEG - 3) / 4) & ~1;
  static constexpr int RC = CT + 2 * H, RB = 2 * RC + 1 + 2 * DEG, RA = 2 * RB + 1 + 2 * DEG;
  static_assert(CT >= 2 && RA <= WL, "three-level region does not fit");
};

template <typename TS, typename TC, int DEG, int NW, int RW>
__global__ __launch_bounds__(NW* WL) void mg_down3_kernel(const TS* __restrict__ tA, TS* __restrict__ xA,
                                                          TS* __restrict__ tB, TS* __restrict__ xB,
                                                          TS* __restrict__ tC, TS* __restrict__ xC,
                                                          TS* __restrict__ tD, const TC* __restrict__ kA,
                                                          const TC* __restrict__ kB, const TC* __restrict__ kC,
                                                          Geom gA, Geom gB, Geom gC, Geom gD, MGCoef cA, MGCoef cB,
                                                          MGCoef cC) {
  using G = Down3<DEG>;
  constexpr int NT = NW * WL, RY = NW * RW, H = G::H, CT = G::CT, RC = G::RC, RB = G::RB;
  static_assert(RY >= G::RA, "three-level region does not fit the rows");
  using PL = Plane<RY>;
  __shared__ TC sA[PL::SIZE];
  __shared__ TC sA2[PL::SIZE];
  __shared__ TC sKB[(RB + 1) * (RB + 1)];
  __shared__ TC sTB[RB * RB];
  __shared__ TC sB0[RB * RB];
  __shared__ TC sB1[RB * RB];
  __shared__ TC sKC[(RC + 1) * (RC + 1)];
  __shared__ TC sTC[RC * RC];
  __shared__ TC sC0[RC * RC];
  __shared__ TC sC1[RC * RC];
  // nested tiles; the tile count follows the A level so that every node of A, B, C and D is covered
  const int ntx = (gA.N - 1 + 4 * CT - 1) / (4 * CT);
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int iC0 = 1 + (tile % ntx) * CT, jC0 = 1 + (tile / ntx) * CT;
  const int iB0 = 2 * iC0 - 1, jB0 = 2 * jC0 - 1, iA0 = 2 * iB0 - 1, jA0 = 2 * jB0 - 1;
  const int oCx = iC0 - H, oCy = jC0 - H;
  const int oBx = 2 * oCx - 1 - DEG, oBy = 2 * oCy - 1 - DEG;
  const int oAx = 2 * oBx - 1 - DEG, oAy = 2 * oBy - 1 - DEG;

  // ---- level A (column segments)
  const int l = threadIdx.x & (WL - 1), r0 = (threadIdx.x / WL) * RW;
  const int i = oAx + l, jf = oAy + r0;
  const TC m = (TC)cA.m, alpha = (TC)cA.alpha;
  bool in[RW];
  unsigned p[RW];
  TC tv[RW], kw[RW + 1], ke[RW + 1];
  // A's diffusivities first: its stencil weights are formed while the right-hand side's loads are in flight
  load_kappa_cols<TC, RW>(kA, i, jf, gA, kw, ke);
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    in[r] = interior(i, jf + r, gA.N);
    p[r] = in[r] ? (unsigned)(jf + r) * gA.pitch + i : 0;
    tv[r] = ld<TC>(tA + p[r]);
  }
  W9<TC> w[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) w[r] = stencil_weights<TC>(kw[r], ke[r], kw[r + 1], ke[r + 1], m, alpha);
  weights_ready<TC, RW>(w);
  flat_kappa<TC, RB, RB, NT>(sKB, kB, oBx, oBy, gB);
  flat_kappa<TC, RC, RC, NT>(sKC, kC, oCx, oCy, gC);
  zero_spare<TC, RY>(sA);
  zero_spare<TC, RY>(sA2);
#pragma unroll
  for (int r = 0; r < RW; ++r) tv[r] = in[r] ? tv[r] : (TC)0;
  TC xc[RW], xp[RW], bx[RW];
  {
    const TC c0 = (TC)cA.c0;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      xc[r] = in[r] ? c0 * w[r].dinv * tv[r] : (TC)0;
      xp[r] = (TC)0;
    }
  }
  TC* cur = sA;
  TC* nxt = sA2;
  store_rows<TC, RY, RW>(cur, l, r0, xc);
  __syncthreads();
#pragma unroll
  for (int k = 1; k < DEG; ++k) {
    const TC beta = (TC)cA.beta[k], gam = (TC)cA.gam[k];
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
  apply_b<TC, RY, RW>(cur, l, r0, w, xc, bx);
  {
    const int ax = iA0 - oAx, ay = jA0 - oAy;
    const bool col_in_tile = l >= ax && l < ax + 4 * CT;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int rr = r0 + r;
      if (col_in_tile && rr >= ay && rr < ay + 4 * CT && in[r]) st(xA + p[r], xc[r]);
      bx[r] = in[r] ? tv[r] - bx[r] : (TC)0;
    }
  }
  store_rows<TC, RY, RW>(nxt, l, r0, bx);
  __syncthreads();
  // ---- restriction A -> right-hand side of B on the B region (and to global on the B tile)
  for (int idx = threadIdx.x; idx < RB * RB; idx += NT) {
    const int lj = idx / RB, li = idx - lj * RB;
    const int I = oBx + li, J = oBy + lj;
    TC v = (TC)0;
    if (interior(I, J, gB.N)) {
      const TC* c = nxt + PL::at(2 * J - oAy, 2 * I - oAx);
      v = c[0] + (TC)0.5 * (c[1] + c[-1] + c[WL] + c[-WL]) +
          (TC)0.25 * (c[WL + 1] + c[WL - 1] + c[-WL + 1] + c[-WL - 1]);
      if (I >= iB0 && I < iB0 + 2 * CT && J >= jB0 && J < jB0 + 2 * CT) st(tB + (unsigned)J * gB.pitch + I, v);
    }
    sTB[lj * RB + li] = v;
  }
  __syncthreads();
  // ---- level B
  TC *bxv, *brv;
  flat_down<TC, RB, RB, NT>(sTB, sB0, sB1, sKB, RB, RB, oBx, oBy, gB.N, cB, bxv, brv);
  for (int idx = threadIdx.x; idx < 4 * CT * CT; idx += NT) {
    const int I = iB0 + idx % (2 * CT), J = jB0 + idx / (2 * CT);
    if (interior(I, J, gB.N)) st(xB + (unsigned)J * gB.pitch + I, bxv[(J - oBy) * RB + (I - oBx)]);
  }
  // ---- restriction B -> right-hand side of C on the C region (and to global on the C tile)
  for (int idx = threadIdx.x; idx < RC * RC; idx += NT) {
    const int lj = idx / RC, li = idx - lj * RC;
    const int I = oCx + li, J = oCy + lj;
    TC v = (TC)0;
    if (interior(I, J, gC.N)) {
      v = flat_restrict<TC, RB>(brv, oBx, oBy, I, J);
      if (I >= iC0 && I < iC0 + CT && J >= jC0 && J < jC0 + CT) st(tC + (unsigned)J * gC.pitch + I, v);
    }
    sTC[lj * RC + li] = v;
  }
  __syncthreads();
  // ---- level C
  TC *cxv, *crv;
  flat_down<TC, RC, RC, NT>(sTC, sC0, sC1, sKC, RC, RC, oCx, oCy, gC.N, cC, cxv, crv);
  for (int idx = threadIdx.x; idx < CT * CT; idx += NT) {
    const int I = iC0 + idx % CT, J = jC0 + idx / CT;
    if (interior(I, J, gC.N)) st(xC + (unsigned)J * gC.pitch + I, cxv[(J - oCy) * RC + (I - oCx)]);
  }
  // ---- restriction C -> right-hand side of D on the D nodes of the C tile
  for (int idx = threadIdx.x; idx < (CT / 2) * (CT / 2); idx += NT) {
    const int I = (iC0 + 1) / 2 + idx % (CT / 2), J = (jC0 + 1) / 2 + idx / (CT / 2);
    if (I > gD.N - 1 || J > gD.N - 1) continue;
    st(tD + (unsigned)J * gD.pitch + I, flat_restrict<TC, RC>(crv, oCx, oCy, I, J));
  }
}

// UP3 geometry: A region of 64 columns x RY rows (tile less DEG halo rings), the largest flat regions of B and C
template <int DEG, int RY>
struct Up3 {
  static constexpr int TA = WL - 2 * DEG, TAY = RY - 2 * DEG;
  static constexpr int RBM = WL / 2 + 2 * DEG + 3, RBH = RY / 2 + 2 * DEG + 3;
  static constexpr int RCM = RBM / 2 + 2 * DEG + 3, RCH = RBH / 2 + 2 * DEG + 3;
};

// t and x of a flat region from global memory (zero outside the interior), optionally x + P e for the coarse
// correction e one level down; all loads issued before the first store
template <typename TS, typename TC, int W, int HM, int NT, bool PROLONG>
__device__ __forceinline__ void flat_load_tx(TC* T, TC* X, const TS* __restrict__ t, const TS* __restrict__ x,
                                             const TS* __restrict__ e, int Rx, int Ry, int ox, int oy, const Geom& g,
                                             const Geom& ge) {
  constexpr int CNT = W * HM, NL = (CNT + NT - 1) / NT;
  TC tv[NL], xv[NL];
#pragma unroll
  for (int r = 0; r < NL; ++r) {
    const int idx = threadIdx.x + r * NT;
    const int lj = idx / W, li = idx - lj * W;
    const int I = ox + li, J = oy + lj;
    const bool ok = idx < CNT && li < Rx && lj < Ry && interior(I, J, g.N);
    const int Ic = ok ? I : 1, Jc = ok ? J : 1;
    const unsigned q = (unsigned)Jc * g.pitch + Ic;
    const TC a = ld<TC>(t + q);
    TC b = ld<TC>(x + q);
    if (PROLONG) b += prolong_at<TS, TC>(e, ge.pitch, Ic, Jc);
    tv[r] = ok ? a : (TC)0;
    xv[r] = ok ? b : (TC)0;
  }
#pragma unroll
  for (int r = 0; r < NL; ++r) {
    const int idx = threadIdx.x + r * NT;
    if (idx < CNT) {
      T[idx] = tv[r];
      X[idx] = xv[r];
    }
  }
}

template <typename TS, typename TC, int DEG, int NW, int RW>
__global__ __launch_bounds__(NW* WL) void mg_up3_kernel(const TS* __restrict__ eD, const TS* __restrict__ tC,
                                                        const TS* __restrict__ xC, const TS* __restrict__ tB,
                                                        const TS* __restrict__ xB, const TS* __restrict__ tA,
                                                        const TS* __restrict__ xA, TS* __restrict__ outA,
                                                        const TC* __restrict__ kA, const TC* __restrict__ kB,
                                                        const TC* __restrict__ kC, Geom gA, Geom gB, Geom gC, Geom gD,
                                                        MGCoef cA, MGCoef cB, MGCoef cC) {
  constexpr int NT = NW * WL, RY = NW * RW;
  using G = Up3<DEG, RY>;
  constexpr int TA = G::TA, TAY = G::TAY, RBM = G::RBM, RBH = G::RBH, RCM = G::RCM, RCH = G::RCH;
  using PL = Plane<RY>;
  __shared__ TC sA[PL::SIZE];
  __shared__ TC sA2[PL::SIZE];
  __shared__ TC sKB[(RBM + 1) * (RBH + 1)];
  __shared__ TC sTB[RBM * RBH];
  __shared__ TC sB0[RBM * RBH];
  __shared__ TC sB1[RBM * RBH];
  __shared__ TC sKC[(RCM + 1) * (RCH + 1)];
  __shared__ TC sTC[RCM * RCH];
  __shared__ TC sC0[RCM * RCH];
  __shared__ TC sC1[RCM * RCH];
  const int ntx = (gA.N - 1 + TA - 1) / TA;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int iA0 = 1 + (tile % ntx) * TA, jA0 = 1 + (tile / ntx) * TAY;
  const int oAx = iA0 - DEG, oAy = jA0 - DEG;
  // B nodes whose result the A region's prolongation reads, and the B region (DEG rings more) that produces them
  const int bLx = oAx >> 1, bLy = oAy >> 1;
  const int oBx = bLx - DEG, oBy = bLy - DEG;
  const int RBx = ((oAx + WL - 1) >> 1) + 2 - bLx + 2 * DEG, RBy = ((oAy + RY - 1) >> 1) + 2 - bLy + 2 * DEG;
  // the same one level down
  const int cLx = oBx >> 1, cLy = oBy >> 1;
  const int oCx = cLx - DEG, oCy = cLy - DEG;
  const int RCx = ((oBx + RBx - 1) >> 1) + 2 - cLx + 2 * DEG, RCy = ((oBy + RBy - 1) >> 1) + 2 - cLy + 2 * DEG;

  // ---- loads: A rows (column segments), the B and C regions (flat), their diffusivities
  const int l = threadIdx.x & (WL - 1), r0 = (threadIdx.x / WL) * RW;
  const int i = oAx + l, jf = oAy + r0;
  bool in[RW];
  unsigned p[RW];
  TC tv[RW], xa[RW], kw[RW + 1], ke[RW + 1];
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    in[r] = interior(i, jf + r, gA.N);
    p[r] = in[r] ? (unsigned)(jf + r) * gA.pitch + i : 0;
    tv[r] = ld<TC>(tA + p[r]);
    xa[r] = ld<TC>(xA + p[r]);
  }
  load_kappa_cols<TC, RW>(kA, i, jf, gA, kw, ke);
  flat_kappa<TC, RBM, RBH, NT>(sKB, kB, oBx, oBy, gB);
  flat_kappa<TC, RCM, RCH, NT>(sKC, kC, oCx, oCy, gC);
  flat_load_tx<TS, TC, RBM, RBH, NT, false>(sTB, sB1, tB, xB, nullptr, RBx, RBy, oBx, oBy, gB, gC);
  flat_load_tx<TS, TC, RCM, RCH, NT, true>(sTC, sC0, tC, xC, eD, RCx, RCy, oCx, oCy, gC, gD);
  __syncthreads();
  // ---- level C: post-smoothing from x_C + P e_D
  const TC* cout = flat_up<TC, RCM, RCH, NT>(sTC, sC0, sC1, sKC, RCx, RCy, oCx, oCy, gC.N, cC);
  // ---- level B: x_B + P (C result), post-smoothing
  for (int idx = threadIdx.x; idx < RBM * RBH; idx += NT) {
    const int lj = idx / RBM, li = idx - lj * RBM;
    if (li >= RBx || lj >= RBy) continue;
    const int I = oBx + li, J = oBy + lj;
    TC v = (TC)0;
    if (interior(I, J, gB.N)) v = sB1[idx] + flat_prolong<TC, RCM>(cout, oCx, oCy, I, J);
    sB0[idx] = v;
  }
  __syncthreads();
  const TC* bout = flat_up<TC, RBM, RBH, NT>(sTB, sB0, sB1, sKB, RBx, RBy, oBx, oBy, gB.N, cB);
  // ---- level A: x_A + P (B result), post-smoothing in column segments, result on the A tile
  const TC m = (TC)cA.m, alpha = (TC)cA.alpha;
  W9<TC> w[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) w[r] = stencil_weights<TC>(kw[r], ke[r], kw[r + 1], ke[r + 1], m, alpha);
  TC xc[RW], xp[RW], bx[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) xp[r] = in[r] ? xa[r] + flat_prolong<TC, RBM>(bout, oBx, oBy, i, jf + r) : (TC)0;
  zero_spare<TC, RY>(sA);
  zero_spare<TC, RY>(sA2);
  store_rows<TC, RY, RW>(sA, l, r0, xp);
  __syncthreads();
  apply_b<TC, RY, RW>(sA, l, r0, w, xp, bx);
  {
    const TC c0 = (TC)cA.c0;
#pragma unroll
    for (int r = 0; r < RW; ++r) xc[r] = in[r] ? xp[r] + c0 * (tv[r] - bx[r]) * w[r].dinv : (TC)0;
  }
  TC* cur = sA;
  TC* nxt = sA2;
#pragma unroll
  for (int k = 1; k < DEG; ++k) {
    store_rows<TC, RY, RW>(nxt, l, r0, xc);
    __syncthreads();
    TC* tmp = cur;
    cur = nxt;
    nxt = tmp;
    const TC beta = (TC)cA.beta[k], gam = (TC)cA.gam[k];
    apply_b<TC, RY, RW>(cur, l, r0, w, xc, bx);
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const TC xn = in[r] ? xc[r] + beta * (xc[r] - xp[r]) + gam * (tv[r] - bx[r]) * w[r].dinv : (TC)0;
      xp[r] = xc[r];
      xc[r] = xn;
    }
  }
  const bool col_in_tile = l >= DEG && l < WL - DEG;
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    const int rr = r0 + r;
    if (col_in_tile && rr >= DEG && rr < RY - DEG && in[r]) st(outA + p[r], xc[r]);
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

template <typename TV, typename TS, typename TC, bool CP, typename TZ, int NW, int RW>
void down_shape(const TV* tt, const double* tscale, TS* xx, TS* cc, TC* to, const TC* kk, Geom g, Geom gc,
                const MGCoef& c, const Couple& cp, hipStream_t st) {
  constexpr int B = NW * WL, C = CP ? 1 : 0;
  switch (c.deg) {
    case 1:
      launch_k(mg_down_kernel<TV, TS, TC, 1, NW, RW, CP, TZ>, level_grid<NW, RW, 2 + C>(g), B, st, tt, tscale, xx, cc, to, kk, g, gc, c, cp);
      break;
    case 2:
      launch_k(mg_down_kernel<TV, TS, TC, 2, NW, RW, CP, TZ>, level_grid<NW, RW, 3 + C>(g), B, st, tt, tscale, xx, cc, to, kk, g, gc, c, cp);
      break;
    default:
      launch_k(mg_down_kernel<TV, TS, TC, 3, NW, RW, CP, TZ>, level_grid<NW, RW, 4 + C>(g), B, st, tt, tscale, xx, cc, to, kk, g, gc, c, cp);
      break;
  }
}

template <typename TV, typename TS, typename TC, bool CP, typename TZ>
void down_launch(const TV* tt, const double* tscale, TS* xx, TS* cc, TC* to, const TC* kk, Geom g, Geom gc,
                 const MGCoef& c, const Couple& cp, hipStream_t st) {
  if (g.N >= kBigLevel)
    down_shape<TV, TS, TC, CP, TZ, DNWB, DRWB>(tt, tscale, xx, cc, to, kk, g, gc, c, cp, st);
  else if (g.N >= kMidLevel)
    down_shape<TV, TS, TC, CP, TZ, DNWM, DRWM>(tt, tscale, xx, cc, to, kk, g, gc, c, cp, st);
  else
    down_shape<TV, TS, TC, CP, TZ, DNWS, DRWS>(tt, tscale, xx, cc, to, kk, g, gc, c, cp, st);
}

template <typename TV, typename TS, typename TC>
void down_t(const void* t, const double* tscale, void* x, void* tc, void* tout, const void* kap, Geom g, Geom gc,
            const MGCoef& c, const Couple& cp, hipStream_t st) {
  if (cp.nz > 0 && cp.z_f32)
    down_launch<TV, TS, TC, true, float>((const TV*)t, tscale, (TS*)x, (TS*)tc, (TC*)tout, (const TC*)kap, g, gc, c,
                                         cp, st);
  else if (cp.nz > 0)
    down_launch<TV, TS, TC, true, double>((const TV*)t, tscale, (TS*)x, (TS*)tc, (TC*)tout, (const TC*)kap, g, gc, c,
                                          cp, st);
  else
    down_launch<TV, TS, TC, false, double>((const TV*)t, tscale, (TS*)x, (TS*)tc, (TC*)tout, (const TC*)kap, g, gc, c,
                                           cp, st);
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

// three-level kernels: DOWN3 on 64-row A regions of 16 wavefronts with 4 rows per lane (the nested tiles need the
// height); UP3 on 16-row regions of 16 wavefronts with one row per lane (swept: more blocks, and more threads for
// the flat B and C regions, shorten its chain the most; 2.6% off the step against 32-row regions of 8 wavefronts)
constexpr int NW3 = 16, RW3 = 4, NWU3 = 16, RWU3 = 1;

template <typename TS, typename TC>
void down3_t(const ThreeLevels& z, hipStream_t st) {
  const Geom& gA = z.g[0];
  auto grid = [&](int ct) { const int n = (gA.N - 1 + 4 * ct - 1) / (4 * ct); return dim3(n * n); };
  const TS* tA = (const TS*)z.t[0];
  TS *xA = (TS*)z.x[0], *tB = (TS*)z.t[1], *xB = (TS*)z.x[1], *tC = (TS*)z.t[2], *xC = (TS*)z.x[2], *tD = (TS*)z.t[3];
  const TC *kA = (const TC*)z.kap[0], *kB = (const TC*)z.kap[1], *kC = (const TC*)z.kap[2];
  switch (z.c[0].deg) {
    case 1:
      launch_k(mg_down3_kernel<TS, TC, 1, NW3, RW3>, grid(Down3<1>::CT), dim3(NW3 * WL), st, tA, xA, tB, xB, tC, xC, tD,
               kA, kB, kC, z.g[0], z.g[1], z.g[2], z.g[3], z.c[0], z.c[1], z.c[2]);
      break;
    case 2:
      launch_k(mg_down3_kernel<TS, TC, 2, NW3, RW3>, grid(Down3<2>::CT), dim3(NW3 * WL), st, tA, xA, tB, xB, tC, xC, tD,
               kA, kB, kC, z.g[0], z.g[1], z.g[2], z.g[3], z.c[0], z.c[1], z.c[2]);
      break;
    default:
      launch_k(mg_down3_kernel<TS, TC, 3, NW3, RW3>, grid(Down3<3>::CT), dim3(NW3 * WL), st, tA, xA, tB, xB, tC, xC, tD,
               kA, kB, kC, z.g[0], z.g[1], z.g[2], z.g[3], z.c[0], z.c[1], z.c[2]);
      break;
  }
}

template <typename TS, typename TC>
void up3_t(const ThreeLevels& z, hipStream_t st) {
  const Geom& gA = z.g[0];
  auto grid = [&](int deg) {
    const int tx = WL - 2 * deg, ty = NWU3 * RWU3 - 2 * deg;
    return dim3(((gA.N - 1 + tx - 1) / tx) * ((gA.N - 1 + ty - 1) / ty));
  };
  const TS* eD = (const TS*)z.e[3];
  const TS *tC = (const TS*)z.t[2], *xC = (const TS*)z.x[2], *tB = (const TS*)z.t[1], *xB = (const TS*)z.x[1];
  const TS *tA = (const TS*)z.t[0], *xA = (const TS*)z.x[0];
  TS* outA = (TS*)z.e[0];
  const TC *kA = (const TC*)z.kap[0], *kB = (const TC*)z.kap[1], *kC = (const TC*)z.kap[2];
  switch (z.c[0].deg) {
    case 1:
      launch_k(mg_up3_kernel<TS, TC, 1, NWU3, RWU3>, grid(1), dim3(NWU3 * WL), st, eD, tC, xC, tB, xB, tA, xA, outA, kA, kB,
               kC, z.g[0], z.g[1], z.g[2], z.g[3], z.c[0], z.c[1], z.c[2]);
      break;
    case 2:
      launch_k(mg_up3_kernel<TS, TC, 2, NWU3, RWU3>, grid(2), dim3(NWU3 * WL), st, eD, tC, xC, tB, xB, tA, xA, outA, kA, kB,
               kC, z.g[0], z.g[1], z.g[2], z.g[3], z.c[0], z.c[1], z.c[2]);
      break;
    default:
      launch_k(mg_up3_kernel<TS, TC, 3, NWU3, RWU3>, grid(3), dim3(NWU3 * WL), st, eD, tC, xC, tB, xB, tA, xA, outA, kA, kB,
               kC, z.g[0], z.g[1], z.g[2], z.g[3], z.c[0], z.c[1], z.c[2]);
      break;
  }
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
                  Geom g, Geom gc, const MGCoef& c, hipStream_t st, bool out_f32) {
  if (prec == 0) {
    up_t<double, double, double, double>(t, x, e, out, kappa, g, gc, c, st);
  } else if (prec == 1) {
    if (finest && !out_f32)
      up_t<float, float, double, float>(t, x, e, out, kappa, g, gc, c, st);
    else
      up_t<float, float, float, float>(t, x, e, out, kappa, g, gc, c, st);
  } else {
    if (finest && out_f32)
      up_t<float, bf16, float, float>(t, x, e, out, kappa, g, gc, c, st);
    else if (finest)
      up_t<float, bf16, double, float>(t, x, e, out, kappa, g, gc, c, st);
    else
      up_t<bf16, bf16, bf16, float>(t, x, e, out, kappa, g, gc, c, st);
  }
}

void launch_mg_coarse(int prec, bool io_is_f64, const void* t, const double* tscale, void* out, const void* Binv, Geom g,
                      hipStream_t st, bool out_f32) {
  const int n = (g.N - 1) * (g.N - 1);
  const dim3 grid((n + NTC / 64 - 1) / (NTC / 64));
  if (prec == 0) {
    launch_k(mg_coarse_kernel<double, double, double>, grid, NTC, st, (const double*)t, tscale, (double*)out,
                                                                 (const double*)Binv, g);
  } else if (io_is_f64 && out_f32) {
    launch_k(mg_coarse_kernel<double, float, float>, grid, NTC, st, (const double*)t, tscale, (float*)out,
                                                               (const float*)Binv, g);
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

void launch_mg_down3(int prec, const ThreeLevels& z, hipStream_t st) {
  if (prec == 0)
    down3_t<double, double>(z, st);
  else if (prec == 1)
    down3_t<float, float>(z, st);
  else
    down3_t<bf16, float>(z, st);
}

void launch_mg_up3(int prec, const ThreeLevels& z, hipStream_t st) {
  if (prec == 0)
    up3_t<double, double>(z, st);
  else if (prec == 1)
    up3_t<float, float>(z, st);
  else
    up3_t<bf16, float>(z, st);
}

}  // namespace irk
