// Internal declarations of the MI355X stage solver: data layout, kernel launch
// wrappers and the runtime objects behind the C ABI of include/irk.h.
//
// Device data layout ("padded planes"). A level with N elements per side stores
// a nodal field as (N+1) rows of `pitch` values (pitch = N+1 rounded up to a
// multiple of 16, so every row starts on a 128-byte boundary for FP64). Node
// (i, j) lives at j*pitch + i for 0 <= i, j <= N; the boundary ring and the row
// padding hold zeros at all times, so every 9-point stencil at an interior node
// reads valid memory without branches, and whole-vector Krylov operations can
// run over the flat array. A stage block is s planes back to back. A per-element
// field uses N rows of the same pitch: element (ex, ey) at ey*pitch + ex.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace irk {

constexpr int kMaxStages = 8;
constexpr int kMaxDeg = 3;
constexpr int kMaxRestart = 64;
constexpr int kMaxCoarse = 1024;  // unknowns of the dense coarsest-level solve
constexpr int kMMGMax = 4;        // stages supported by the monolithic multigrid cycle

struct bf16 {
  uint16_t u;
};

struct Geom {
  int N;       // elements per side
  int pitch;   // values per row
  long plane;  // (N+1)*pitch values per nodal plane
  double h;    // 1/N
};

inline int pitch_for(int N) { return ((N + 1 + 15) / 16) * 16; }
inline Geom make_geom(int N) {
  Geom g;
  g.N = N;
  g.pitch = pitch_for(N);
  g.plane = (long)(N + 1) * g.pitch;
  g.h = 1.0 / N;
  return g;
}

// XCD-aware tile order. Workgroups of a launch are dealt round-robin to the chip's 8 XCDs, each with its own L2;
// tile = xcd_tile(linear block id, block count) gives every XCD a contiguous range of tiles, so neighbouring tiles
// (which read each other's halo rows) share one L2. A bijection of [0, nb) for any nb.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb / kXcds, r = nb % kXcds;
  const int x = b % kXcds, k = b / kXcds;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// s x s coefficient matrix passed by value to kernels
struct Coefs {
  double a[kMaxStages * kMaxStages];
};

// Chebyshev-Jacobi smoothing coefficients for one (level, diagonal block).
// x_1 = x_0 + c0 D^{-1} r_0;  x_{k+1} = x_k + beta[k] (x_k - x_{k-1}) + gam[k] D^{-1} r_k.
struct MGCoef {
  double alpha;  // dt * a_ii
  double m;      // h^2 / 36 (mass stencil scale)
  double c0;
  double beta[kMaxDeg];
  double gam[kMaxDeg];
  int deg;
};

// One level of the monolithic cycle (Section 3.2): operator cm (x) M + dt ck (x) K on s planes,
// additive Schwarz patch blocks cm M_vv + dt ck K_vv, Chebyshev coefficients as in MGCoef.
struct MMGCoef {
  int s;
  int deg;
  double m;   // h^2 / 36 of the level
  double dt;
  double c0;
  double beta[kMaxDeg];
  double gam[kMaxDeg];
  double cm[kMMGMax * kMMGMax];  // row-major, row stride kMMGMax
  double ck[kMMGMax * kMMGMax];
  // patch blocks in closed form: C_v = (1/w) (I + tau B) with B the non-identity mixing matrix,
  // AI: tau = tfac * K_vv, w = wfac; IA: tau = tfac / K_vv, w = wfac / K_vv; then
  // C_v^{-1} = w adj(I + tau B) / det(I + tau B), adj = sum_k tau^k adj_k, det = sum_k tau^k det_k
  int ia;
  double tfac, wfac;
  double adj[kMMGMax * kMMGMax * kMMGMax];  // [k][q][r]
  double det[kMMGMax + 1];
};

// ---------------------------------------------------------------- measurement hook
// Start/stop events that the next launch of a wrapper attaches to its dispatch (kernel start and end
// timestamps); the runtime sets them just before calling the wrapper, whose first launch consumes them.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchEvents g_launch_ev;

template <typename K, typename... A>
inline void launch_k(K kernel, dim3 grid, dim3 block, hipStream_t st, A... args) {
  const LaunchEvents ev = g_launch_ev;
  g_launch_ev = LaunchEvents{};
  if (ev.start)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, ev.start, ev.stop, 0, args...);
  else
    kernel<<<grid, block, 0, st>>>(args...);
}

// ---------------------------------------------------------------- layout (k_stencil.hip)
void launch_pack(const double* src, double* dst, Geom g, int nplanes, hipStream_t st);
void launch_unpack(const double* src, double* dst, Geom g, int nplanes, hipStream_t st);
void launch_pack_elem(const double* src, double* dst, Geom g, hipStream_t st);
void launch_unpack_elem(const double* src, double* dst, Geom g, hipStream_t st);
void launch_check_kappa(const double* kappa, int count, int* bad, hipStream_t st);
void launch_cast_f32(const double* src, float* dst, long count, hipStream_t st);
void launch_coarsen_kappa(const double* fine, double* coarse, Geom gf, Geom gc, hipStream_t st);
void launch_device_copy(const double* x, double* y, long n, hipStream_t st);

// ---------------------------------------------------------------- stencils (k_stencil.hip)
// y = (I (x) M + dt*A (x) K) x  (coefficients `a`, row-major s x s); if f != nullptr: y = f - that.
// ia: y = (A (x) M + dt*I (x) K) x instead (the IA form passes A^{-1} as `a`).
void launch_stage_operator(const double* x, double* y, const double* f, const double* kappa, Geom g, int s,
                           const Coefs& a, double dt, hipStream_t st, bool ia = false);
// the same with FP32 x (the mixed form's flexible basis), read into FP64 arithmetic
void launch_stage_operator(const float* x, double* y, const double* f, const double* kappa, Geom g, int s,
                           const Coefs& a, double dt, hipStream_t st, bool ia = false);
// f_i = -K u + F (F may be null), i = 0..s-1
// f (and f2 if not NULL: a second copy) = -K u + F in every stage plane
void launch_stage_rhs(const double* u, const double* F, double* f, const double* kappa, Geom g, int s, hipStream_t st,
                      double* f2 = nullptr);
// y = M x or y = K x
void launch_mass(const double* x, double* y, Geom g, hipStream_t st);
void launch_stiff(const double* x, double* y, const double* kappa, Geom g, hipStream_t st);
// t = vmul * vscale * v - dt * Op * sum_{q<nz} row[q] z_q  (z_q planes at z + q*plane; vscale: device scalar or
// null = 1; Op = K, or M if mass)
void launch_gs_couple(const double* v, const double* vscale, const double* z, int nz, const Coefs& row, double dt,
                      const double* kappa, double* t, Geom g, hipStream_t st, int mass = 0, double vmul = 1.0);
// the same with FP32 z planes
void launch_gs_couple(const double* v, const double* vscale, const float* z, int nz, const Coefs& row, double dt,
                      const double* kappa, double* t, Geom g, hipStream_t st, int mass = 0, double vmul = 1.0);
// u += dt * sum_i b_i k_i
void launch_update(double* u, const double* k, int s, const Coefs& b, double dt, Geom g, hipStream_t st);
// f_i = dt * b_i * lam
void launch_adjoint_rhs(const double* lam, double* f, int s, const Coefs& b, double dt, Geom g, hipStream_t st);
// lam -= K * sum_i nu_i
void launch_lambda_update(double* lam, const double* nu, int s, const double* kappa, Geom g, hipStream_t st);
// g_e -= kappa_e * sum_i nu_i|_e^T Kref (u + dt sum_j a_ij k_j)|_e   (g padded element layout)
void launch_kappa_grad(double* grad, const double* u, const double* k, const double* nu, const double* kappa, Geom g,
                       int s, const Coefs& a, double dt, hipStream_t st);
// power iteration helpers (FP64, setup): mode 0: y = B x, 1: y = D^{-1} B x, 2: y = D x
void launch_level_apply(const double* x, double* y, const double* kappa, Geom g, double alpha, int mode,
                        hipStream_t st);
// SplitMix64 start vector on the interior nodes; the value index is the compact node index + offset
void launch_start_vector(double* x, Geom g, int level, hipStream_t st, uint64_t offset = 0);
void launch_scale(double* x, long n, const double* inv_norm2_src, hipStream_t st);

// ---------------------------------------------------------------- multigrid (k_mg.hip)
// Block Gauss-Seidel coupling folded into the finest-level kernels: their right-hand side becomes
// t = tscale * v - dt * K * sum_{q<nz} a[q] z_q  (z_q = z + q*zstride, FP64 padded planes).
struct Couple {
  const void* z = nullptr;    // first coupled stage plane
  int z_f32 = 0;              // the coupled planes are FP32 (the mixed form's flexible basis), else FP64
  long zstride = 0;
  int nz = 0;                 // number of coupled stages; 0: no coupling
  int mass = 0;               // coupling operator: 0 = stiffness K (element kappa), 1 = mass M
  double dt = 0;              // t -= dt * Op(sum_q a_q z_q)
  double mh = 0;              // h^2/36 of the level (mass stencil)
  double vmul = 1.0;          // the right-hand side t is scaled by vmul (and the device scalar)
  double a[kMaxStages] = {};
};
// prec: 0 = FP64 storage/compute, 1 = FP32, 2 = BF16 storage / FP32 compute.
// DOWN: pre-smooth from zero on the fine level, write x, restrict the residual into tc (coarse).
// t_is_f64: t is the FP64 Krylov vector (scaled by the device scalar *tscale; null = 1) instead of level storage.
// tout (optional, compute type, finest level): receives the right-hand side the smoother used (scaled, coupled).
void launch_mg_down(int prec, bool t_is_f64, const void* t, const double* tscale, void* x, void* tc, void* tout,
                    const void* kappa, Geom g, Geom gc, const MGCoef& c, const Couple& cp, hipStream_t st);
// UP: x0 = x + P e, post-smooth, write out. finest: t is the compute-type right-hand side stored by DOWN and out
// is the FP64 result (FP32 with out_f32: the mixed form's flexible basis, which holds the same values, since the
// smoother computes in FP32); otherwise t and out are level storage.
void launch_mg_up(int prec, bool finest, const void* t, const void* x, const void* e, void* out, const void* kappa,
                  Geom g, Geom gc, const MGCoef& c, hipStream_t st, bool out_f32 = false);
// coarsest level: out = Binv * t on the interior nodes (io_is_f64: FP64 t and out; out FP32 with out_f32)
void launch_mg_coarse(int prec, bool io_is_f64, const void* t, const double* tscale, void* out, const void* Binv, Geom g,
                      hipStream_t st, bool out_f32 = false);

// The three levels A, B = A/2, C = B/2 above the coarsest level D in one launch each way. Index 0..3 = A..D.
// DOWN3 reads t[0] and writes x[0..2], t[1..3]; UP3 reads e[3], t[0..2], x[0..2] and writes e[0].
struct ThreeLevels {
  Geom g[4];
  MGCoef c[3];
  void* t[4];
  void* x[3];
  void* e[4];
  const void* kap[3];
};
void launch_mg_down3(int prec, const ThreeLevels& z, hipStream_t st);
void launch_mg_up3(int prec, const ThreeLevels& z, hipStream_t st);

// ---------------------------------------------------------------- monolithic multigrid (k_mmg.hip)
// prec as above; t_f64 / io_f64: t (and out) is an FP64 Krylov vector (s planes) instead of level storage.
// DOWN: Chebyshev pre-smoothing from zero of Acal x = ts t, writes x and the restricted residual tc.
void launch_mmg_down(int prec, bool t_f64, const void* t, const double* tscale, void* x, void* tc, const void* kap,
                     Geom g, Geom gc, const MMGCoef& c, hipStream_t st);
// UP: x0 = x + (I (x) P) e, Chebyshev post-smoothing, writes out (with io_f64 and out_f32: FP32 out).
void launch_mmg_up(int prec, bool io_f64, const void* t, const double* tscale, const void* x, const void* e, void* out,
                   const void* kap, Geom g, Geom gc, const MMGCoef& c, hipStream_t st, bool out_f32 = false);
// coarsest level: out = Cinv (ts t) over the s (N-1)^2 stage-major unknowns (<= kMaxCoarse); out_f32 (with t_f64):
// FP32 out whatever the storage type
void launch_mmg_coarse(int prec, bool t_f64, bool out_f64, const void* t, const double* tscale, void* out,
                       const void* Cinv, Geom g, int s, hipStream_t st, bool out_f32 = false);
// FP64 set-up: mode 0 out = C^{-1} Acal x, 1 out = Acal x, 2 out = C x
void launch_mmg_apply(const double* x, double* out, const double* kap, Geom g, const MMGCoef& c, int mode,
                      hipStream_t st);

// ---------------------------------------------------------------- Krylov (k_krylov.hip)
struct OrthoArgs {
  const double* V;       // basis vectors V_k = V + k*vstride
  const float* Vf;       // if set (update passes only, coef set, no dots): the basis is FP32 at Vf + k*vstride
  long vstride;
  int nv;                // number of basis vectors (0..kMaxRestart)
  double* w;             // vector updated in place when coef != nullptr
  long len;              // values per vector
  const double* coef;    // if set: w -= coef_sign * sum_k coef[k]*vscale[k]*V_k first
  int assign;            // with coef: w = -coef_sign * sum_k ... (w is not read: it may hold anything)
  double coef_sign;
  const double* vscale;  // per-vector scale (nullptr = 1)
  int want_dots;         // compute dots[k] = vscale[k] * V_k . w (after the update)
  const int* skip;       // if set and *skip == 0 the pass does nothing
  double* result;        // [nv+1]: dots then |w|^2
  double* sigma_out;     // if set: *sigma_out = 1/sqrt(|w|^2)
  int* flag_out;         // if set: *flag_out = (|w|^2 < eta2 * *ref)
  const double* ref;
  double eta2;
};
struct ReduceWork {
  double* partial;     // [max_blocks * (kMaxRestart+1)]
  unsigned* counter;   // one zeroed counter
  int max_blocks;
};
// ev0/ev1 (optional): start/stop events of the streaming pass's own dispatch on st (not the finish)
void launch_ortho(const OrthoArgs& a, const ReduceWork& w, hipStream_t st, hipEvent_t ev0 = nullptr,
                  hipEvent_t ev1 = nullptr);

// Delayed CGS2 (one reduction per Arnoldi step). Q = V_0..V_{nv-1} (finished), u (previous direction),
// w (new direction). res receives [Q^T u (nv), Q^T w (nv), u.u, u.w, w.w, beta, 1/beta, h, nu, flag].
constexpr int kMaxDcgs2 = 31;
constexpr int kDcgs2Res = 2 * (kMaxDcgs2 + 1) + 8;
struct D2Args {
  const double* V;
  long vstride;
  int nv;
  double* u;
  double* w;
  long len;
  double* res;
  // optional: the same coefficients written a second time into pinned host memory (the device address of
  // a hipHostMalloc'ed, coherent buffer), so that the host reads them once the step's event has completed
  double* mirror = nullptr;
};
void launch_dcgs2_dots(const D2Args& a, const ReduceWork& rw, hipStream_t st, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr);
// u <- (u - Q a)/beta, w <- w - Q s - h u (coefficients read from res on the device)
void launch_dcgs2_update(const D2Args& a, const ReduceWork& rw, hipStream_t st, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);

}  // namespace irk
