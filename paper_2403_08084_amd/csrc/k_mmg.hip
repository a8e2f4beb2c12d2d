// Monolithic multigrid kernels for the stage-coupled operator (Section 3.2).
//
// A level operator acts on s stage planes at once,
//   (Acal x)_q = sum_r cm[q][r] M x_r + dt * sum_r ck[q][r] K x_r,
// with (cm, ck) = (I, A) for the AI form and (A^{-1}, I) for the IA form (transposed
// for the adjoint). The relaxation is additive Schwarz over the vertex patches of all
// stages (eq:Cinv, eq:bigdecomp): at every interior node the s x s patch block
//   C_v = cm * M_vv + dt * ck * K_vv,   M_vv = 16 h^2/36,  K_vv = (2/3) * (sum of the 4 kappa),
// is solved in registers inside a Chebyshev iteration. Every patch block has the form
// (1/w)(I + tau B) with one fixed s x s matrix B per level and a scalar tau from the node's
// diffusivity, so its inverse is applied in closed form, w adj(I + tau B) / det(I + tau B), with the
// adjugate and determinant as polynomials in tau whose coefficients the host computes once per level
// (Faddeev-LeVerrier). One thread owns one node and all of its stages, so the s x s stage mixing
// never leaves registers.
//
// Kernels per level of a V-cycle: a fused DOWN (pre-smoothing, residual, restriction) and a
// fused UP (prolongation and correction, post-smoothing), both LDS-tiled; on the coarsest level
// a dense inverse.
#include "mg_device.h"

namespace irk {
namespace {

// threads per block of the fused level kernels (512: eight waves share a tile's phases; 1024 would cap
// the registers of the s-plane kernels and spill)
constexpr int NT = 512;
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

// z = C_v^{-1} r in place from the closed form w adj(I + tau B) / det(I + tau B) (coefficients precomputed
// per level on the host); kd = K_vv of the node
template <typename TC, int S>
__device__ __forceinline__ void patch_apply(const MMGCoef& c, TC kd, TC r[S]) {
  const TC ikd = c.ia ? recip(kd) : (TC)1;
  const TC tau = c.ia ? (TC)c.tfac * ikd : (TC)c.tfac * kd;
  const TC w = (TC)c.wfac * ikd;
  TC d = (TC)c.det[S];
#pragma unroll
  for (int k = S - 1; k >= 0; --k) d = d * tau + (TC)c.det[k];
  const TC f = w * recip(d);
  TC z[S];
#pragma unroll
  for (int q = 0; q < S; ++q) {
    TC acc = (TC)0;
#pragma unroll
    for (int rr = 0; rr < S; ++rr) {
      TC a = (TC)c.adj[(S - 1) * kMMGMax * kMMGMax + q * kMMGMax + rr];
#pragma unroll
      for (int k = S - 2; k >= 0; --k) a = a * tau + (TC)c.adj[k * kMMGMax * kMMGMax + q * kMMGMax + rr];
      acc += a * r[rr];
    }
    z[q] = f * acc;
  }
#pragma unroll
  for (int q = 0; q < S; ++q) r[q] = z[q];
}

// ---------------------------------------------------------------- fused, LDS-tiled levels
//
// One level of the V-cycle is two kernels, as for the single-stage cycle:
//   DOWN: Chebyshev pre-smoothing from zero, the residual and its restriction (I (x) P^T);
//         writes the smoothed iterate and the coarse right-hand side.
//   UP:   prolongation and correction x + (I (x) P) e, then Chebyshev post-smoothing.
// A block stages a TX x TY tile plus a halo of all s planes (right-hand side and two iterates)
// and the element diffusivities in LDS; the valid region shrinks by one node per stencil.

// (Acal x)_q at LDS node (li, lj) of S planes (plane stride PA, row length RX); kd = K_vv
template <typename TC, int S, int RX, int KX, int PA>
__device__ __forceinline__ void lds_apply(const TC* X, const TC* sK, int li, int lj, const MMGCoef& c, TC out[S],
                                          TC& kd) {
  const int p = lj * RX + li;
  const int q = lj * KX + li;
  const TC kSW = sK[q], kSE = sK[q + 1], kNW = sK[q + KX], kNE = sK[q + KX + 1];
  const TC ks = kSW + kSE + kNW + kNE;
  kd = (TC)(2.0 / 3.0) * ks;
  const TC m = (TC)c.m, dt = (TC)c.dt;
  TC Mx[S], Kx[S];
#pragma unroll
  for (int r = 0; r < S; ++r) {
    const TC* x = X + r * PA + p;
    const TC xc = x[0], xE = x[1], xW = x[-1], xN = x[RX], xS = x[-RX];
    const TC xNE = x[RX + 1], xNW = x[RX - 1], xSE = x[-RX + 1], xSW = x[-RX - 1];
    Kx[r] = kd * xc -
            (TC)(1.0 / 6.0) * ((kNE + kSE) * xE + (kNW + kSW) * xW + (kNE + kNW) * xN + (kSE + kSW) * xS) -
            (TC)(1.0 / 3.0) * (kNE * xNE + kNW * xNW + kSE * xSE + kSW * xSW);
    Mx[r] = m * ((TC)16 * xc + (TC)4 * (xE + xW + xN + xS) + (xNE + xNW + xSE + xSW));
  }
  // one of the two mixing matrices is the identity: AI (I, ck), IA (cm, I)
  if (c.ia) {
#pragma unroll
    for (int qq = 0; qq < S; ++qq) {
      TC acc = dt * Kx[qq];
#pragma unroll
      for (int r = 0; r < S; ++r) acc += (TC)c.cm[qq * kMMGMax + r] * Mx[r];
      out[qq] = acc;
    }
  } else {
#pragma unroll
    for (int qq = 0; qq < S; ++qq) {
      TC acc = (TC)0;
#pragma unroll
      for (int r = 0; r < S; ++r) acc += (TC)c.ck[qq * kMMGMax + r] * Kx[r];
      out[qq] = Mx[qq] + dt * acc;
    }
  }
}

template <typename TC, int KX>
__device__ __forceinline__ TC lds_kdiag(const TC* sK, int li, int lj) {
  const int q = lj * KX + li;
  return (TC)(2.0 / 3.0) * (sK[q] + sK[q + 1] + sK[q + KX] + sK[q + KX + 1]);
}

// Tiles: on large levels 64 wide (coalesced rows) and tall enough to amortise the halo while keeping the
// three S-plane LDS fields within about 80 KB; on levels below 512^2 a 32 x 8 tile spreads the
// latency-bound work over four times more waves.
template <typename TC, int S, bool SMALL>
struct MTile {
  static constexpr int TX = SMALL ? 32 : 64;
  static constexpr int TY = 8;
};
constexpr int kSmallLevel = 512;

template <typename TT, typename TS, typename TC, int S, int DEG, int TX, int TY>
__global__ __launch_bounds__(NT) void mmg_down_kernel(const TT* __restrict__ t, const double* __restrict__ tscale,
                                                      TS* __restrict__ xout, TS* __restrict__ tc,
                                                      const TC* __restrict__ kap, Geom g, Geom gc, MMGCoef c) {
  constexpr int H = DEG + 1;
  constexpr int RX = TX + 2 * H, RY = TY + 2 * H;
  constexpr int KX = RX + 1, KY = RY + 1;
  constexpr int PA = RX * RY;
  __shared__ TC sK[KX * KY];
  __shared__ TC sT[S * PA];
  __shared__ TC sA[S * PA];
  __shared__ TC sB[S * PA];
  const int N = g.N;
  // tiles on a 1-D grid in XCD-aware order: neighbouring tiles (shared halos) run on the same XCD
  const int ntx = (g.N - 1 + TX - 1) / TX;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int i0 = 1 + (tile % ntx) * TX, j0 = 1 + (tile / ntx) * TY;
  const int ox = i0 - H, oy = j0 - H;
  const TC ts = tscale ? (TC)(*tscale) : (TC)1;
  {
    constexpr int NL = (PA + NT - 1) / NT;
    TC tv[S][NL];
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
      for (int r = 0; r < NL; ++r) {
        const int idx = threadIdx.x + r * NT;
        const int lj = idx / RX, li = idx - lj * RX;
        const int i = ox + li, j = oy + lj;
        const bool ok = idx < PA && interior(i, j, N);
        const TC val = ld<TC>(t + q * g.plane + (ok ? (long)j * g.pitch + i : 0));
        tv[q][r] = ok ? val * ts : (TC)0;
      }
    load_kappa_tile<TC, TC, KX, KY, NT>(sK, kap, ox, oy, g);
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
      for (int r = 0; r < NL; ++r) {
        const int idx = threadIdx.x + r * NT;
        if (idx < PA) sT[q * PA + idx] = tv[q][r];
      }
  }
  __syncthreads();
  // step 0 from x = 0 is pointwise: x1 = c0 C^{-1} t on the whole region
  {
    const TC c0 = (TC)c.c0;
    for (int idx = threadIdx.x; idx < PA; idx += NT) {
      const int lj = idx / RX, li = idx - lj * RX;
      TC r[S];
#pragma unroll
      for (int q = 0; q < S; ++q) r[q] = sT[q * PA + idx];
      const bool in = interior(ox + li, oy + lj, N);
      if (in) patch_apply<TC, S>(c, lds_kdiag<TC, KX>(sK, li, lj), r);
#pragma unroll
      for (int q = 0; q < S; ++q) {
        sB[q * PA + idx] = in ? c0 * r[q] : (TC)0;
        sA[q * PA + idx] = (TC)0;
      }
    }
  }
  __syncthreads();
  TC* cur = sB;
  TC* prv = sA;
#pragma unroll
  for (int k = 1; k < DEG; ++k) {
    const TC beta = (TC)c.beta[k], gam = (TC)c.gam[k];
    const int w = RX - 2 * k, hgt = RY - 2 * k;
    for (int idx = threadIdx.x; idx < w * hgt; idx += NT) {
      const int lj = k + idx / w, li = k + idx % w;
      if (!interior(ox + li, oy + lj, N)) continue;
      const int p = lj * RX + li;
      TC ax[S], kd;
      lds_apply<TC, S, RX, KX, PA>(cur, sK, li, lj, c, ax, kd);
      TC r[S];
#pragma unroll
      for (int q = 0; q < S; ++q) r[q] = sT[q * PA + p] - ax[q];
      patch_apply<TC, S>(c, kd, r);
#pragma unroll
      for (int q = 0; q < S; ++q) {
        const TC x1 = cur[q * PA + p];
        prv[q * PA + p] = x1 + beta * (x1 - prv[q * PA + p]) + gam * r[q];
      }
    }
    __syncthreads();
    TC* tmp = cur;
    cur = prv;
    prv = tmp;
  }
  // smoothed iterate on the tile
  for (int idx = threadIdx.x; idx < TX * TY; idx += NT) {
    const int lj = H + idx / TX, li = H + idx % TX;
    const int i = ox + li, j = oy + lj;
    if (interior(i, j, N)) {
#pragma unroll
      for (int q = 0; q < S; ++q) st(xout + q * g.plane + (long)j * g.pitch + i, cur[q * PA + lj * RX + li]);
    }
  }
  // residual on the tile plus one node
  {
    const int w = TX + 2, hgt = TY + 2;
    for (int idx = threadIdx.x; idx < w * hgt; idx += NT) {
      const int lj = H - 1 + idx / w, li = H - 1 + idx % w;
      const int p = lj * RX + li;
      TC r[S];
#pragma unroll
      for (int q = 0; q < S; ++q) r[q] = (TC)0;
      if (interior(ox + li, oy + lj, N)) {
        TC ax[S], kd;
        lds_apply<TC, S, RX, KX, PA>(cur, sK, li, lj, c, ax, kd);
#pragma unroll
        for (int q = 0; q < S; ++q) r[q] = sT[q * PA + p] - ax[q];
      }
#pragma unroll
      for (int q = 0; q < S; ++q) prv[q * PA + p] = r[q];
    }
  }
  __syncthreads();
  // full-weighting restriction of every plane to the coarse nodes centred in the tile
  {
    constexpr int CX = TX / 2, CY = TY / 2;
    const int I0 = (i0 + 1) / 2, J0 = (j0 + 1) / 2;
    for (int idx = threadIdx.x; idx < CX * CY; idx += NT) {
      const int I = I0 + idx % CX, J = J0 + idx / CX;
      if (I > gc.N - 1 || J > gc.N - 1) continue;
      const int li = 2 * I - ox, lj = 2 * J - oy;
#pragma unroll
      for (int q = 0; q < S; ++q) {
        const TC* R = prv + q * PA + lj * RX + li;
        const TC v = R[0] + (TC)0.5 * (R[1] + R[-1] + R[RX] + R[-RX]) +
                     (TC)0.25 * (R[RX + 1] + R[RX - 1] + R[-RX + 1] + R[-RX - 1]);
        st(tc + q * gc.plane + (long)J * gc.pitch + I, v);
      }
    }
  }
}

template <typename TT, typename TS, typename TO, typename TC, int S, int DEG, int TX, int TY>
__global__ __launch_bounds__(NT) void mmg_up_kernel(const TT* __restrict__ t, const double* __restrict__ tscale,
                                                    const TS* __restrict__ x, const TS* __restrict__ e,
                                                    TO* __restrict__ out, const TC* __restrict__ kap, Geom g, Geom gc,
                                                    MMGCoef c) {
  constexpr int H = DEG;
  constexpr int RX = TX + 2 * H, RY = TY + 2 * H;
  constexpr int KX = RX + 1, KY = RY + 1;
  constexpr int PA = RX * RY;
  __shared__ TC sK[KX * KY];
  __shared__ TC sT[S * PA];
  __shared__ TC sA[S * PA];
  __shared__ TC sB[S * PA];
  const int N = g.N;
  // tiles on a 1-D grid in XCD-aware order: neighbouring tiles (shared halos) run on the same XCD
  const int ntx = (g.N - 1 + TX - 1) / TX;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int i0 = 1 + (tile % ntx) * TX, j0 = 1 + (tile / ntx) * TY;
  const int ox = i0 - H, oy = j0 - H;
  const TC ts = tscale ? (TC)(*tscale) : (TC)1;
  {
    constexpr int NL = (PA + NT - 1) / NT;
    TC tv[S][NL], xv[S][NL];
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
      for (int r = 0; r < NL; ++r) {
        const int idx = threadIdx.x + r * NT;
        const int lj = idx / RX, li = idx - lj * RX;
        const int i = ox + li, j = oy + lj;
        const bool ok = idx < PA && interior(i, j, N);
        const int ic = ok ? i : 1, jc = ok ? j : 1;
        const long p = (long)jc * g.pitch + ic;
        const TC a = ld<TC>(t + q * g.plane + p) * ts;
        const TC b = ld<TC>(x + q * g.plane + p) + prolong_at<TS, TC>(e + q * gc.plane, gc.pitch, ic, jc);
        tv[q][r] = ok ? a : (TC)0;
        xv[q][r] = ok ? b : (TC)0;
      }
    load_kappa_tile<TC, TC, KX, KY, NT>(sK, kap, ox, oy, g);
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
      for (int r = 0; r < NL; ++r) {
        const int idx = threadIdx.x + r * NT;
        if (idx < PA) {
          sT[q * PA + idx] = tv[q][r];
          sA[q * PA + idx] = xv[q][r];
        }
      }
  }
  __syncthreads();
  // step 0 from the corrected iterate: x1 = x0 + c0 C^{-1} (t - Acal x0) on the inner region
  {
    const TC c0 = (TC)c.c0;
    const int w = RX - 2, hgt = RY - 2;
    for (int idx = threadIdx.x; idx < w * hgt; idx += NT) {
      const int lj = 1 + idx / w, li = 1 + idx % w;
      const int p = lj * RX + li;
      if (interior(ox + li, oy + lj, N)) {
        TC ax[S], kd;
        lds_apply<TC, S, RX, KX, PA>(sA, sK, li, lj, c, ax, kd);
        TC r[S];
#pragma unroll
        for (int q = 0; q < S; ++q) r[q] = sT[q * PA + p] - ax[q];
        patch_apply<TC, S>(c, kd, r);
#pragma unroll
        for (int q = 0; q < S; ++q) sB[q * PA + p] = sA[q * PA + p] + c0 * r[q];
      } else {
#pragma unroll
        for (int q = 0; q < S; ++q) sB[q * PA + p] = (TC)0;
      }
    }
  }
  __syncthreads();
  TC* cur = sB;
  TC* prv = sA;
#pragma unroll
  for (int k = 1; k < DEG; ++k) {
    const TC beta = (TC)c.beta[k], gam = (TC)c.gam[k];
    const int w = RX - 2 * (k + 1), hgt = RY - 2 * (k + 1);
    for (int idx = threadIdx.x; idx < w * hgt; idx += NT) {
      const int lj = k + 1 + idx / w, li = k + 1 + idx % w;
      if (!interior(ox + li, oy + lj, N)) continue;
      const int p = lj * RX + li;
      TC ax[S], kd;
      lds_apply<TC, S, RX, KX, PA>(cur, sK, li, lj, c, ax, kd);
      TC r[S];
#pragma unroll
      for (int q = 0; q < S; ++q) r[q] = sT[q * PA + p] - ax[q];
      patch_apply<TC, S>(c, kd, r);
#pragma unroll
      for (int q = 0; q < S; ++q) {
        const TC x1 = cur[q * PA + p];
        prv[q * PA + p] = x1 + beta * (x1 - prv[q * PA + p]) + gam * r[q];
      }
    }
    __syncthreads();
    TC* tmp = cur;
    cur = prv;
    prv = tmp;
  }
  for (int idx = threadIdx.x; idx < TX * TY; idx += NT) {
    const int lj = H + idx / TX, li = H + idx % TX;
    const int i = ox + li, j = oy + lj;
    if (interior(i, j, N)) {
#pragma unroll
      for (int q = 0; q < S; ++q) st(out + q * g.plane + (long)j * g.pitch + i, cur[q * PA + lj * RX + li]);
    }
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

template <typename TT, typename TS, typename TC, int S, int DEG, bool SMALL>
void down_k(const void* t, const double* ts, void* x, void* tc, const void* kap, Geom g, Geom gc, const MMGCoef& c,
            hipStream_t st) {
  constexpr int TX = MTile<TC, S, SMALL>::TX, TY = MTile<TC, S, SMALL>::TY;
  const dim3 grid(((g.N - 1 + TX - 1) / TX) * ((g.N - 1 + TY - 1) / TY));
  launch_k(mmg_down_kernel<TT, TS, TC, S, DEG, TX, TY>, grid, NT, st, (const TT*)t, ts, (TS*)x, (TS*)tc, (const TC*)kap,
                                                                   g, gc, c);
}

template <typename TT, typename TS, typename TO, typename TC, int S, int DEG, bool SMALL>
void up_k(const void* t, const double* ts, const void* x, const void* e, void* out, const void* kap, Geom g, Geom gc,
          const MMGCoef& c, hipStream_t st) {
  constexpr int TX = MTile<TC, S, SMALL>::TX, TY = MTile<TC, S, SMALL>::TY;
  const dim3 grid(((g.N - 1 + TX - 1) / TX) * ((g.N - 1 + TY - 1) / TY));
  launch_k(mmg_up_kernel<TT, TS, TO, TC, S, DEG, TX, TY>, grid, NT, st, (const TT*)t, ts, (const TS*)x, (const TS*)e,
                                                                     (TO*)out, (const TC*)kap, g, gc, c);
}

template <typename TT, typename TS, typename TC, int S, int DEG>
void down_s(const void* t, const double* ts, void* x, void* tc, const void* kap, Geom g, Geom gc, const MMGCoef& c,
            hipStream_t st) {
  if (g.N < kSmallLevel)
    down_k<TT, TS, TC, S, DEG, true>(t, ts, x, tc, kap, g, gc, c, st);
  else
    down_k<TT, TS, TC, S, DEG, false>(t, ts, x, tc, kap, g, gc, c, st);
}

template <typename TT, typename TS, typename TO, typename TC, int S, int DEG>
void up_s(const void* t, const double* ts, const void* x, const void* e, void* out, const void* kap, Geom g, Geom gc,
          const MMGCoef& c, hipStream_t st) {
  if (g.N < kSmallLevel)
    up_k<TT, TS, TO, TC, S, DEG, true>(t, ts, x, e, out, kap, g, gc, c, st);
  else
    up_k<TT, TS, TO, TC, S, DEG, false>(t, ts, x, e, out, kap, g, gc, c, st);
}

template <typename TT, typename TS, typename TC, int S>
void down_d(const void* t, const double* ts, void* x, void* tc, const void* kap, Geom g, Geom gc, const MMGCoef& c,
            hipStream_t st) {
  switch (c.deg) {
    case 1: down_s<TT, TS, TC, S, 1>(t, ts, x, tc, kap, g, gc, c, st); break;
    case 2: down_s<TT, TS, TC, S, 2>(t, ts, x, tc, kap, g, gc, c, st); break;
    default: down_s<TT, TS, TC, S, 3>(t, ts, x, tc, kap, g, gc, c, st); break;
  }
}

template <typename TT, typename TS, typename TO, typename TC, int S>
void up_d(const void* t, const double* ts, const void* x, const void* e, void* out, const void* kap, Geom g, Geom gc,
          const MMGCoef& c, hipStream_t st) {
  switch (c.deg) {
    case 1: up_s<TT, TS, TO, TC, S, 1>(t, ts, x, e, out, kap, g, gc, c, st); break;
    case 2: up_s<TT, TS, TO, TC, S, 2>(t, ts, x, e, out, kap, g, gc, c, st); break;
    default: up_s<TT, TS, TO, TC, S, 3>(t, ts, x, e, out, kap, g, gc, c, st); break;
  }
}

template <typename TT, typename TS, typename TC>
void down_t(const void* t, const double* ts, void* x, void* tc, const void* kap, Geom g, Geom gc, const MMGCoef& c,
            hipStream_t st) {
  switch (c.s) {
    case 1: down_d<TT, TS, TC, 1>(t, ts, x, tc, kap, g, gc, c, st); break;
    case 2: down_d<TT, TS, TC, 2>(t, ts, x, tc, kap, g, gc, c, st); break;
    case 3: down_d<TT, TS, TC, 3>(t, ts, x, tc, kap, g, gc, c, st); break;
    default: down_d<TT, TS, TC, 4>(t, ts, x, tc, kap, g, gc, c, st); break;
  }
}

template <typename TT, typename TS, typename TO, typename TC>
void up_t(const void* t, const double* ts, const void* x, const void* e, void* out, const void* kap, Geom g, Geom gc,
          const MMGCoef& c, hipStream_t st) {
  switch (c.s) {
    case 1: up_d<TT, TS, TO, TC, 1>(t, ts, x, e, out, kap, g, gc, c, st); break;
    case 2: up_d<TT, TS, TO, TC, 2>(t, ts, x, e, out, kap, g, gc, c, st); break;
    case 3: up_d<TT, TS, TO, TC, 3>(t, ts, x, e, out, kap, g, gc, c, st); break;
    default: up_d<TT, TS, TO, TC, 4>(t, ts, x, e, out, kap, g, gc, c, st); break;
  }
}

}  // namespace

// prec: 0 FP64, 1 FP32, 2 BF16 storage with FP32 compute (kappa and Cinv in the compute type).
// t_f64: t (and, for UP, out) is an FP64 Krylov vector (the finest level) instead of level storage.
void launch_mmg_down(int prec, bool t_f64, const void* t, const double* tscale, void* x, void* tc, const void* kap,
                     Geom g, Geom gc, const MMGCoef& c, hipStream_t st) {
  if (prec == 0) down_t<double, double, double>(t, tscale, x, tc, kap, g, gc, c, st);
  else if (prec == 1) {
    if (t_f64) down_t<double, float, float>(t, tscale, x, tc, kap, g, gc, c, st);
    else down_t<float, float, float>(t, tscale, x, tc, kap, g, gc, c, st);
  } else {
    if (t_f64) down_t<double, bf16, float>(t, tscale, x, tc, kap, g, gc, c, st);
    else down_t<bf16, bf16, float>(t, tscale, x, tc, kap, g, gc, c, st);
  }
}

void launch_mmg_up(int prec, bool io_f64, const void* t, const double* tscale, const void* x, const void* e, void* out,
                   const void* kap, Geom g, Geom gc, const MMGCoef& c, hipStream_t st, bool out_f32) {
  if (prec == 0) up_t<double, double, double, double>(t, tscale, x, e, out, kap, g, gc, c, st);
  else if (prec == 1) {
    if (io_f64 && out_f32) up_t<double, float, float, float>(t, tscale, x, e, out, kap, g, gc, c, st);
    else if (io_f64) up_t<double, float, double, float>(t, tscale, x, e, out, kap, g, gc, c, st);
    else up_t<float, float, float, float>(t, tscale, x, e, out, kap, g, gc, c, st);
  } else {
    if (io_f64 && out_f32) up_t<double, bf16, float, float>(t, tscale, x, e, out, kap, g, gc, c, st);
    else if (io_f64) up_t<double, bf16, double, float>(t, tscale, x, e, out, kap, g, gc, c, st);
    else up_t<bf16, bf16, bf16, float>(t, tscale, x, e, out, kap, g, gc, c, st);
  }
}

void launch_mmg_coarse(int prec, bool t_f64, bool out_f64, const void* t, const double* tscale, void* out,
                       const void* Cinv, Geom g, int s, hipStream_t st, bool out_f32) {
  const int n = s * (g.N - 1) * (g.N - 1);
  const dim3 grid((n + 3) / 4), blk(256);
  if (prec != 0 && t_f64 && out_f32) {
    launch_k(mmg_coarse_kernel<double, float, float>, grid, blk, st, (const double*)t, tscale, (float*)out,
                                                                   (const float*)Cinv, g, s);
  } else if (prec == 0) {
    launch_k(mmg_coarse_kernel<double, double, double>, grid, blk, st, (const double*)t, tscale, (double*)out,
                                                                     (const double*)Cinv, g, s);
  } else if (prec == 1) {
    const float* C = (const float*)Cinv;
    if (t_f64 && out_f64) launch_k(mmg_coarse_kernel<double, double, float>, grid, blk, st, (const double*)t, tscale, (double*)out, C, g, s);
    else if (t_f64) launch_k(mmg_coarse_kernel<double, float, float>, grid, blk, st, (const double*)t, tscale, (float*)out, C, g, s);
    else if (out_f64) launch_k(mmg_coarse_kernel<float, double, float>, grid, blk, st, (const float*)t, tscale, (double*)out, C, g, s);
    else launch_k(mmg_coarse_kernel<float, float, float>, grid, blk, st, (const float*)t, tscale, (float*)out, C, g, s);
  } else {
    const float* C = (const float*)Cinv;
    if (t_f64 && out_f64) launch_k(mmg_coarse_kernel<double, double, float>, grid, blk, st, (const double*)t, tscale, (double*)out, C, g, s);
    else if (t_f64) launch_k(mmg_coarse_kernel<double, bf16, float>, grid, blk, st, (const double*)t, tscale, (bf16*)out, C, g, s);
    else if (out_f64) launch_k(mmg_coarse_kernel<bf16, double, float>, grid, blk, st, (const bf16*)t, tscale, (double*)out, C, g, s);
    else launch_k(mmg_coarse_kernel<bf16, bf16, float>, grid, blk, st, (const bf16*)t, tscale, (bf16*)out, C, g, s);
  }
}

void launch_mmg_apply(const double* x, double* out, const double* kap, Geom g, const MMGCoef& c, int mode,
                      hipStream_t st) {
  const dim3 grid = mmg_grid(g), blk(MX, MY);
  switch (c.s) {
    case 1: launch_k(mmg_apply_kernel<1>, grid, blk, st, x, out, kap, g, c, mode); break;
    case 2: launch_k(mmg_apply_kernel<2>, grid, blk, st, x, out, kap, g, c, mode); break;
    case 3: launch_k(mmg_apply_kernel<3>, grid, blk, st, x, out, kap, g, c, mode); break;
    default: launch_k(mmg_apply_kernel<4>, grid, blk, st, x, out, kap, g, c, mode); break;
  }
}

}  // namespace irk
