// Host runtime behind the C ABI: problem and stepper objects, multigrid setup,
// the FGMRES driver, the time loop and the adjoint with binomial checkpointing.
// Every floating-point step of the solve runs in the kernels of k_*.hip; the
// host only orchestrates launches, runs the (m+1) x m Hessenberg least-squares
// update, and makes the convergence decisions.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/irk.h"
#include "host_math.h"
#include "irk_internal.h"

using namespace irk;

thread_local irk::LaunchEvents irk::g_launch_ev;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(IRK_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define CHK(expr)              \
  do {                         \
    int r_ = (expr);           \
    if (r_ != IRK_OK) return r_; \
  } while (0)

int dev_alloc(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(IRK_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
  }
  return IRK_OK;
}

void dev_free(void* p) {
  if (p) (void)hipFree(p);
}

hipStream_t S(void* s) { return (hipStream_t)s; }

int check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(IRK_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return IRK_OK;
}

size_t storage_bytes(int prec) { return prec == 0 ? 8 : (prec == 1 ? 4 : 2); }

}  // namespace

struct irk_problem {
  int N = 0;
  int dev = 0;  // device current at creation
  Geom g{};
  double* kappa = nullptr;  // padded element layout, FP64
  int* bad = nullptr;       // device flag of the kappa check (create and irk_problem_set_kappa)
  // staging of irk_apply_mass / irk_apply_stiffness: two padded planes, allocated by the first such call
  mutable double* stage = nullptr;
  mutable std::mutex stage_mu;
};

namespace {

struct Level {
  Geom g{};
  double* kap64 = nullptr;  // FP64 diffusivity (level 0: the problem's)
  void* kapc = nullptr;     // diffusivity in the multigrid compute type
  void* t = nullptr;        // right-hand side (levels >= 1)
  void* x = nullptr;        // pre-smoothed iterate (levels < L-1)
  void* e = nullptr;        // level result / coarse correction (levels >= 1)
  void* tp = nullptr;       // finest level: the smoother's right-hand side in the compute type (DOWN -> UP)
  bool own64 = false;
};

}  // namespace

struct irk_stepper {
  const irk_problem* prob = nullptr;
  int s = 0;
  double A[kMaxStages * kMaxStages] = {};
  double b[kMaxStages] = {};
  double c[kMaxStages] = {};
  double dt = 0;
  // preconditioner matrix Atil (lower triangular, row-major) for the forward [0] and transposed [1]
  // systems, and its diagonal (the diagonal blocks M + dt*pd_i*K)
  double Pt[2][kMaxStages * kMaxStages] = {};
  double pd[kMaxStages] = {};
  // stage formulation: AI (unknowns k) or IA (unknowns w = (A (x) I) k)
  bool ia = false;
  double Op[2][kMaxStages * kMaxStages] = {};  // operator mixing: AI A / A^T (on K), IA A^{-1} / A^{-T} (on M)
  double Ci[2][kMaxStages * kMaxStages] = {};  // IA preconditioner coupling Atil^{-1} (forward / transposed)
  double bw[kMaxStages] = {};                  // update weights on the unknowns: AI b, IA A^{-T} b
  irk_options opt{};
  int prec = 0;
  Geom g{};
  long vlen = 0;  // s * plane
  std::vector<Level> lv;
  std::vector<MGCoef> coef;   // [stage * L + level]
  std::vector<double> mu;     // [stage * L + level]
  std::vector<void*> binv;    // per stage, coarsest-level inverse in the compute type
  // monolithic multigrid (IRK_PC_MONOLITHIC): levels with s-plane buffers, per-level coefficients and the
  // dense inverse of the coarsest coupled operator, for the forward [0] and transposed [1] systems
  std::vector<Level> ml;
  std::vector<MMGCoef> mcoef[2];
  std::vector<double> mmu[2];
  void* mcinv[2] = {nullptr, nullptr};
  // Krylov workspace
  double* V = nullptr;    // (m+1) vectors
  double* Z = nullptr;    // m vectors
  double* f = nullptr;    // right-hand side (s planes)
  double* k = nullptr;    // solution (s planes)
  double* tmp = nullptr;  // s planes
  double* tmp2 = nullptr; // s planes
  double* u = nullptr;    // state plane
  double* Fp = nullptr;   // forcing plane
  double* dres = nullptr; // device results: [4][kMaxRestart+1] + sigma[kMaxRestart+1] + y[kMaxRestart]
  int* dflag = nullptr;
  double* hres = nullptr; // pinned host mirror of dres
  ReduceWork rw{};
  bool have_prev = false;
  hipStream_t cap = nullptr;              // library-owned stream used only to capture graphs
  // Arnoldi steps may run one ahead of the host: step j leaves its reduction in slot j % 2 of dres and
  // of the pinned, device-visible mirror hmir, and the host waits for step j's event alone
  double* hmir = nullptr;      // host address of the mirror (2 slots of kDcgs2Res)
  double* hmir_dev = nullptr;  // its device address
  hipEvent_t step_ev[2] = {nullptr, nullptr};  // recorded on the solver's stream after step j
  hipEvent_t norm_ev = nullptr;                // behind the initial norms of a solve
  int last_its[2 + kMaxStages] = {};           // iterations of the last solve per system (as graphs[])
  // measurement hook: start/stop events on every dispatch of the timed kernel families (eager launches only),
  // with each dispatch's family and the algorithmic bytes it moves (two counts: the per-pass model, and the
  // minimum of the fused kernels)
  int timer_family = -1;                  // -1 off, a family, or IRK_KFAM_ALL
  std::vector<hipEvent_t> timer_ev;       // pairs (start, end)
  std::vector<int> timer_tag;             // family of each pair
  size_t timer_used = 0;
  double timer_bytes[IRK_KFAM_COUNT] = {};
  double timer_bytes_min[IRK_KFAM_COUNT] = {};
  int timer_launches[IRK_KFAM_COUNT] = {};
  // one graph per Arnoldi index j, per system: [0] coupled forward, [1] coupled transposed,
  // [2 + i] the single-stage system of DIRK stage i
  std::vector<hipGraphExec_t> graphs[2 + kMaxStages];
  bool dirk = false;  // stage-by-stage solves for a lower-triangular A (Section 2.3)
  // set by the time step when its right-hand side kernel also wrote f into V_0: the next DCGS2 solve of st->f
  // without a guess then needs no copy (cleared by every solve)
  bool v0_is_f = false;
  // the mixed form keeps its flexible basis Z in FP32: the preconditioner's output is computed in FP32, so the
  // stored values are the same, at half the bytes for the finest UP, the operator, the stage coupling and the
  // solution update
  bool zf32 = false;
  int sys = -1;       // system the Krylov solver works on: -1 the coupled one, i >= 0 DIRK stage i
  // adjoint workspace, allocated by the first irk_adjoint call: checkpoint planes (grown when a call needs
  // more slots), the adjoint state, the padded gradient and two stage vectors
  double* adj_snaps = nullptr;
  int adj_slots = 0;
  double* adj_lam = nullptr;
  double* adj_grad = nullptr;
  double* adj_nu = nullptr;
  double* adj_kstep = nullptr;
};

namespace {

// a step is launched ahead only while the predicted residual estimate exceeds this multiple of the target
constexpr double kLookaheadMargin = 4.0;
constexpr int RSTRIDE = kMaxRestart + 2;
double* res_slot(irk_stepper* st, int which) { return st->dres + (long)which * RSTRIDE; }
double* sigma_dev(irk_stepper* st) { return st->dres + 4L * RSTRIDE; }
double* ycoef_dev(irk_stepper* st) { return st->dres + 5L * RSTRIDE; }
double* dcgs2_dev(irk_stepper* st, int slot) { return st->dres + 6L * RSTRIDE + (long)slot * kDcgs2Res; }
constexpr long DRES_LEN = 6L * RSTRIDE + 2L * kDcgs2Res;

// length of the Krylov vectors of the current system
long sys_len(const irk_stepper* st) { return st->sys < 0 ? st->vlen : st->g.plane; }

// stage-operator mixing coefficients for the forward or transposed system
Coefs coefs_of(const irk_stepper* st, bool trans) {
  Coefs a{};
  for (int i = 0; i < st->s; ++i)
    for (int j = 0; j < st->s; ++j) a.a[i * kMaxStages + j] = st->Op[trans ? 1 : 0][i * st->s + j];
  return a;
}

// stage values U_i = u + dt sum_j mix_ij x_j in terms of the unknowns x: AI mix = A, IA mix = I
Coefs mix_of(const irk_stepper* st) {
  Coefs a{};
  for (int i = 0; i < st->s; ++i)
    for (int j = 0; j < st->s; ++j) a.a[i * kMaxStages + j] = st->ia ? (i == j ? 1.0 : 0.0) : st->A[i * st->s + j];
  return a;
}

Coefs ptil_of(const irk_stepper* st, bool trans) {
  Coefs a{};
  for (int i = 0; i < st->s; ++i)
    for (int j = 0; j < st->s; ++j) a.a[i * kMaxStages + j] = st->Pt[trans ? 1 : 0][i * st->s + j];
  return a;
}

Coefs b_of(const irk_stepper* st) {
  Coefs b{};
  for (int i = 0; i < st->s; ++i) b.a[i] = st->bw[i];
  return b;
}

// ------------------------------------------------------------------ reductions

// Next (start, end) event pair of the measurement hook for one dispatch of `family` moving `bytes` (per-pass
// model) and `bytes_min` (fused minimum) algorithmic bytes, or nulls when the family is not timed.
int timer_pair(irk_stepper* st, int family, double bytes, double bytes_min, hipEvent_t* e0, hipEvent_t* e1) {
  *e0 = *e1 = nullptr;
  if (st->timer_family != family && st->timer_family != IRK_KFAM_ALL) return IRK_OK;
  if (st->timer_used + 2 > st->timer_ev.size()) {
    for (int q = 0; q < 256; ++q) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      st->timer_ev.push_back(e);
    }
  }
  if (st->timer_tag.size() < st->timer_ev.size() / 2) st->timer_tag.resize(st->timer_ev.size() / 2);
  st->timer_tag[st->timer_used / 2] = family;
  *e0 = st->timer_ev[st->timer_used++];
  *e1 = st->timer_ev[st->timer_used++];
  st->timer_launches[family]++;
  st->timer_bytes[family] += bytes;
  st->timer_bytes_min[family] += bytes_min;
  return IRK_OK;
}

// the same, handed to the next launch of a wrapper (launch_k)
int timer_arm(irk_stepper* st, int family, double bytes, double bytes_min) {
  hipEvent_t e0, e1;
  CHK(timer_pair(st, family, bytes, bytes_min, &e0, &e1));
  g_launch_ev.start = e0;
  g_launch_ev.stop = e1;
  return IRK_OK;
}

// interior nodes of a level
double nodes(const Geom& g) { return (double)(g.N - 1) * (double)(g.N - 1); }

// Algorithmic bytes of the multigrid kernels, as (per-pass model, fused minimum). The per-pass model counts what
// the V-cycle moves when every smoothing, residual and transfer pass streams its vectors (per node: 5p for
// Chebyshev(2) pre-smoothing, 3p + p/4 for the residual and its restriction, 2p + p/4 for the prolongation and
// correction, 6p for the post-smoothing, with p the bytes of a stored value, plus the element diffusivity once
// per smoother pass); the fused minimum counts what the fused level kernels read and write once.
struct Bytes {
  double model, min;
};
double compute_bytes(const irk_stepper* st) { return st->prec == 0 ? 8.0 : 4.0; }

// single-stage DOWN on level l (nz coupled stage planes of zb bytes a value read at the finest level)
Bytes mg_down_bytes(const irk_stepper* st, int l, int nz, double zb = 8.0) {
  const double n = nodes(st->lv[l].g), p = (double)storage_bytes(st->prec), c = compute_bytes(st);
  const double tin = l == 0 ? 8.0 : p, tout = l == 0 ? c : 0.0;
  return {n * (8.25 * p + 2 * c + zb * nz), n * (tin + c + p + 0.25 * p + tout + zb * nz)};
}

// single-stage UP on level l (the finest writes ob bytes a value)
Bytes mg_up_bytes(const irk_stepper* st, int l, double ob = 8.0) {
  const double n = nodes(st->lv[l].g), p = (double)storage_bytes(st->prec), c = compute_bytes(st);
  const double tin = l == 0 ? c : p, out = l == 0 ? ob : p;
  return {n * (8.25 * p + 2 * c), n * (tin + p + 0.25 * p + c + out)};
}

// three levels A = a, a+1, a+2 in one launch: the per-pass model of the three single-level kernels; the fused
// minimum reads A's right-hand side and the three diffusivities, writes the three iterates and the right-hand
// sides of B, C and D (the intermediate right-hand sides are not read back)
Bytes mg_down3_bytes(const irk_stepper* st, int a) {
  const double p = (double)storage_bytes(st->prec), c = compute_bytes(st);
  Bytes b{0, 0};
  for (int q = 0; q < 3; ++q) {
    const double n = nodes(st->lv[a + q].g);
    b.model += mg_down_bytes(st, a + q, 0).model;
    b.min += n * ((q == 0 ? p : 0.0) + c + p + 0.25 * p);
  }
  return b;
}

// the converse: reads D's correction, the right-hand sides, iterates and diffusivities of the three levels and
// writes A's result (the intermediate results stay in the block)
Bytes mg_up3_bytes(const irk_stepper* st, int a) {
  const double p = (double)storage_bytes(st->prec), c = compute_bytes(st);
  Bytes b{0, 0};
  for (int q = 0; q < 3; ++q) {
    const double n = nodes(st->lv[a + q].g);
    b.model += mg_up_bytes(st, a + q).model;
    b.min += n * (2 * p + c + (q == 0 ? p : 0.0) + (q == 2 ? 0.25 * p : 0.0));
  }
  return b;
}

// dense coarsest solve on nv unknowns: the inverse once, the right-hand side and the result (io64: an FP64
// right-hand side and a result of ob bytes a value)
Bytes coarse_bytes(const irk_stepper* st, double nv, bool io64, double ob = 8.0) {
  const double c = compute_bytes(st), io = io64 ? 8.0 + ob : 2.0 * (double)storage_bytes(st->prec);
  const double b = nv * nv * c + nv * io;
  return {b, b};
}

// monolithic DOWN / UP on level l (s planes)
Bytes mmg_down_bytes(const irk_stepper* st, int l) {
  const double n = nodes(st->ml[l].g), p = (double)storage_bytes(st->prec), c = compute_bytes(st), s = st->s;
  const double tin = l == 0 ? 8.0 : p;
  return {n * (s * 8.25 * p + 2 * c), n * (s * tin + c + s * p + s * 0.25 * p)};
}

Bytes mmg_up_bytes(const irk_stepper* st, int l, double ob = 8.0) {
  const double n = nodes(st->ml[l].g), p = (double)storage_bytes(st->prec), c = compute_bytes(st), s = st->s;
  const double io = l == 0 ? 8.0 : p, out = l == 0 ? ob : p;
  return {n * (s * 8.25 * p + 2 * c), n * (s * io + s * p + s * 0.25 * p + c + s * out)};
}

int arm(irk_stepper* st, int family, const Bytes& b) { return timer_arm(st, family, b.model, b.min); }

// Algorithmic bytes of one streaming Gram-Schmidt pass over s*n interior values:
// the basis vectors it reads, w read (not when the pass assigns w), and w written when it updates w.
double ortho_bytes(const irk_stepper* st, const OrthoArgs& a) {
  const double vec = 8.0 * (double)(a.len / st->g.plane) * (double)(st->prob->N - 1) * (st->prob->N - 1);
  const bool ax = a.coef != nullptr, dt = a.want_dots != 0;
  const int nvec = (a.nv > 0 && (ax || dt)) ? a.nv : 0;
  return vec * ((a.Vf ? 0.5 : 1.0) * nvec + ((ax && a.assign) ? 0 : 1) + (ax ? 1 : 0));
}

// Algorithmic bytes of the two DCGS2 passes over nv finished vectors: the reduction reads Q, u and w;
// the update reads them and writes u and w.
double dcgs2_bytes(const irk_stepper* st, int nv, long len, bool update) {
  const double vec = 8.0 * (double)(len / st->g.plane) * (double)(st->prob->N - 1) * (st->prob->N - 1);
  return vec * (nv + 2 + (update ? 2 : 0));
}

int ortho(irk_stepper* st, const OrthoArgs& a, hipStream_t s) {
  if (a.Vf && (a.coef == nullptr || a.want_dots)) return fail(IRK_EINVAL, "an FP32 basis is read by update passes only");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  // only passes over the Krylov vectors are timed (not the setup's per-level norms); with DCGS2 the timed
  // family is its reduction and update passes alone
  if (a.len == sys_len(st)) {
    const double b = ortho_bytes(st, a);
    CHK(timer_pair(st, IRK_KFAM_GRAM_SCHMIDT, b, b, &e0, &e1));
    CHK(timer_arm(st, IRK_KFAM_REDUCE_FINISH, 0, 0));
  }
  launch_ortho(a, st->rw, s, e0, e1);
  return check_launch();
}

OrthoArgs ortho_base() {
  OrthoArgs a{};
  a.coef_sign = 1.0;
  a.eta2 = 0.5;
  return a;
}

// |x|^2 into res (device), optionally 1/|x| into sig
int norm2(irk_stepper* st, const double* x, long len, double* res, double* sig, hipStream_t s) {
  OrthoArgs a = ortho_base();
  a.nv = 0;
  a.w = const_cast<double*>(x);
  a.len = len;
  a.result = res;
  a.sigma_out = sig;
  return ortho(st, a, s);
}

// res[0] = x . y
int dot(irk_stepper* st, const double* x, const double* y, long len, double* res, hipStream_t s) {
  OrthoArgs a = ortho_base();
  a.V = x;
  a.vstride = 0;
  a.nv = 1;
  a.w = const_cast<double*>(y);
  a.len = len;
  a.want_dots = 1;
  a.result = res;
  return ortho(st, a, s);
}

// ------------------------------------------------------------------ multigrid setup

void cheb_coef(double mu, const irk_options& o, MGCoef& c) {
  c.deg = o.cheb_degree;
  host::chebyshev_coefficients(o.cheb_lo * mu, o.cheb_hi * mu, o.cheb_degree, kMaxDeg, &c.c0, c.beta, c.gam);
}

// Largest eigenvalue of D^{-1}B on one level by power iteration from the SplitMix64 start vector.
int power_mu(irk_stepper* st, int level, double alpha, double* mu_out, hipStream_t s) {
  const Level& L = st->lv[level];
  const Geom& g = L.g;
  double* x = st->tmp;
  double* y = st->tmp + g.plane;
  double* z = st->tmp2;
  HIPCHK(hipMemsetAsync(x, 0, g.plane * sizeof(double), s));
  HIPCHK(hipMemsetAsync(y, 0, g.plane * sizeof(double), s));
  HIPCHK(hipMemsetAsync(z, 0, g.plane * sizeof(double), s));
  launch_start_vector(x, g, level, s);
  double* r = res_slot(st, 0);
  for (int it = 0; it < st->opt.power_its; ++it) {
    launch_level_apply(x, y, L.kap64, g, alpha, 1, s);
    CHK(norm2(st, y, g.plane, r, nullptr, s));
    launch_scale(y, g.plane, r, s);
    std::swap(x, y);
  }
  launch_level_apply(x, y, L.kap64, g, alpha, 0, s);  // B x
  launch_level_apply(x, z, L.kap64, g, alpha, 2, s);  // D x
  CHK(dot(st, x, y, g.plane, res_slot(st, 1), s));
  CHK(dot(st, x, z, g.plane, res_slot(st, 2), s));
  CHK(check_launch());
  double h[2];
  HIPCHK(hipMemcpyAsync(&h[0], res_slot(st, 1), sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&h[1], res_slot(st, 2), sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *mu_out = h[0] / h[1];
  if (!(std::isfinite(*mu_out) && *mu_out > 0)) return fail(IRK_EINVAL, "power iteration produced a non-positive mu");
  return IRK_OK;
}

// Dense inverse of the coarsest-level block M + alpha*K (interior nodes): banded Cholesky (half-bandwidth N)
int coarse_inverse(const std::vector<double>& kap, int N, double alpha, std::vector<double>& inv) {
  const int m = N - 1, n = m * m;
  std::vector<double> K((size_t)n * n, 0.0), B((size_t)n * n, 0.0);
  host::assemble_q1(kap.data(), N, N, K.data(), B.data());
  for (size_t q = 0; q < B.size(); ++q) B[q] += alpha * K[q];
  inv.assign((size_t)n * n, 0.0);
  if (host::spd_band_inverse(B.data(), n, m + 1, inv.data()) != 0)
    return fail(IRK_EINVAL, "coarsest-level block is not positive definite");
  return IRK_OK;
}

int setup_multigrid(irk_stepper* st, hipStream_t s) {
  const irk_problem* p = st->prob;
  std::vector<int> sizes{p->N};
  while (sizes.back() % 2 == 0 && sizes.back() > st->opt.mg_coarse_n) sizes.push_back(sizes.back() / 2);
  const int Nc = sizes.back();
  if ((long)(Nc - 1) * (Nc - 1) > kMaxCoarse)
    return fail(IRK_EINVAL, "multigrid needs N = Nc * 2^L with (Nc-1)^2 <= 1024; N = " + std::to_string(p->N) +
                                " stops at a " + std::to_string(Nc) + "^2 coarsest grid");
  const int L = (int)sizes.size();
  const size_t tsz = storage_bytes(st->prec);
  st->lv.resize(L);
  for (int l = 0; l < L; ++l) {
    Level& lev = st->lv[l];
    lev.g = make_geom(sizes[l]);
    const long kcount = (long)lev.g.N * lev.g.pitch;
    // buffers are allocated by the first call only (a refresh after a change of kappa reuses them)
    if (l == 0) {
      lev.kap64 = p->kappa;
    } else {
      if (!lev.kap64) CHK(dev_alloc((void**)&lev.kap64, kcount * sizeof(double)));
      lev.own64 = true;
      launch_coarsen_kappa(st->lv[l - 1].kap64, lev.kap64, st->lv[l - 1].g, lev.g, s);
    }
    if (st->prec == 0) {
      lev.kapc = lev.kap64;
    } else {
      if (!lev.kapc) CHK(dev_alloc(&lev.kapc, kcount * sizeof(float)));
      launch_cast_f32(lev.kap64, (float*)lev.kapc, kcount, s);
    }
    const size_t pb = lev.g.plane * tsz;
    if (l >= 1) {
      if (!lev.t) CHK(dev_alloc(&lev.t, pb));
      if (!lev.e) CHK(dev_alloc(&lev.e, pb));
      HIPCHK(hipMemsetAsync(lev.t, 0, pb, s));
      HIPCHK(hipMemsetAsync(lev.e, 0, pb, s));
    }
    if (l < L - 1) {
      if (!lev.x) CHK(dev_alloc(&lev.x, pb));
      HIPCHK(hipMemsetAsync(lev.x, 0, pb, s));
    }
    if (l == 0 && L > 1) {
      const size_t tb = lev.g.plane * (st->prec == 0 ? sizeof(double) : sizeof(float));
      if (!lev.tp) CHK(dev_alloc(&lev.tp, tb));
      HIPCHK(hipMemsetAsync(lev.tp, 0, tb, s));
    }
  }
  CHK(check_launch());
  // Chebyshev coefficients per (stage, level) from power-iteration estimates
  st->coef.assign((size_t)st->s * L, MGCoef{});
  st->mu.assign((size_t)st->s * L, 0.0);
  for (int i = 0; i < st->s; ++i) {
    const double alpha = st->dt * st->pd[i];
    for (int l = 0; l < L; ++l) {
      MGCoef& c = st->coef[(size_t)i * L + l];
      c.alpha = alpha;
      c.m = st->lv[l].g.h * st->lv[l].g.h / 36.0;
      c.deg = st->opt.cheb_degree;
      if (l < L - 1) {
        // reuse the estimate of an earlier stage with the same diagonal entry
        double mu = 0;
        for (int i2 = 0; i2 < i; ++i2)
          if (st->pd[i2] == st->pd[i]) mu = st->mu[(size_t)i2 * L + l];
        if (mu == 0) CHK(power_mu(st, l, alpha, &mu, s));
        st->mu[(size_t)i * L + l] = mu;
        cheb_coef(mu, st->opt, c);
      }
    }
  }
  // the power iterations used tmp / tmp2 with coarse-level layouts: restore the all-zero boundary ring and
  // padding of the finest layout, which the interior-only kernels writing into them rely on
  const size_t tb = (size_t)std::max(st->s, 2) * st->g.plane * sizeof(double);
  HIPCHK(hipMemsetAsync(st->tmp, 0, tb, s));
  HIPCHK(hipMemsetAsync(st->tmp2, 0, tb, s));
  // coarsest-level inverses
  const Level& lc = st->lv[L - 1];
  std::vector<double> kpad((size_t)lc.g.N * lc.g.pitch), kc((size_t)lc.g.N * lc.g.N);
  HIPCHK(hipMemcpyAsync(kpad.data(), lc.kap64, kpad.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int ey = 0; ey < lc.g.N; ++ey)
    for (int ex = 0; ex < lc.g.N; ++ex) kc[(size_t)ey * lc.g.N + ex] = kpad[(size_t)ey * lc.g.pitch + ex];
  if (st->binv.empty()) st->binv.assign(st->s, nullptr);
  const int nc = (lc.g.N - 1) * (lc.g.N - 1);
  for (int i = 0; i < st->s; ++i) {
    std::vector<double> inv;
    CHK(coarse_inverse(kc, lc.g.N, st->dt * st->pd[i], inv));
    if (st->prec == 0) {
      if (!st->binv[i]) CHK(dev_alloc(&st->binv[i], (size_t)nc * nc * sizeof(double)));
      HIPCHK(hipMemcpy(st->binv[i], inv.data(), (size_t)nc * nc * sizeof(double), hipMemcpyHostToDevice));
    } else {
      std::vector<float> f(inv.begin(), inv.end());
      if (!st->binv[i]) CHK(dev_alloc(&st->binv[i], (size_t)nc * nc * sizeof(float)));
      HIPCHK(hipMemcpy(st->binv[i], f.data(), (size_t)nc * nc * sizeof(float), hipMemcpyHostToDevice));
    }
  }
  return IRK_OK;
}

// ------------------------------------------------------------------ monolithic multigrid setup

// the level operator's stage mixing: AI (I, Op), IA (Op, I), with Op = A, A^T or A^{-1}, A^{-T}
void mmg_mixing(const irk_stepper* st, int trans, MMGCoef& c) {
  const int s = st->s;
  for (int q = 0; q < s; ++q)
    for (int r = 0; r < s; ++r) {
      const double op = st->Op[trans][q * s + r], id = (q == r) ? 1.0 : 0.0;
      c.cm[q * kMMGMax + r] = st->ia ? op : id;
      c.ck[q * kMMGMax + r] = st->ia ? id : op;
    }
  // closed form of the patch-block inverse: adj(I + tau B) and det(I + tau B) as polynomials in tau for B = Op
  // (Faddeev-LeVerrier recursion for the characteristic polynomial and adjugate of B)
  double B[kMMGMax * kMMGMax] = {};
  for (int q = 0; q < s; ++q)
    for (int r = 0; r < s; ++r) B[q * kMMGMax + r] = st->Op[trans][q * s + r];
  host::faddeev_leverrier(B, s, kMMGMax, c.adj, c.det);
  c.ia = st->ia ? 1 : 0;
  const double mv = 16.0 * c.m;  // M_vv
  c.tfac = st->ia ? mv / st->dt : st->dt / mv;
  c.wfac = st->ia ? 1.0 / st->dt : 1.0 / mv;
}

// Levels, Chebyshev coefficients (power iteration on C^{-1} Acal per level, both systems) and the coarsest
// inverse of the monolithic cycle.
int setup_mmg(irk_stepper* st, hipStream_t s) {
  const irk_problem* p = st->prob;
  const int ns = st->s;
  std::vector<int> sizes{p->N};
  while (sizes.back() % 2 == 0 &&
         (sizes.back() > st->opt.mg_coarse_n || (long)ns * (sizes.back() - 1) * (sizes.back() - 1) > kMaxCoarse))
    sizes.push_back(sizes.back() / 2);
  const int Nc = sizes.back();
  if ((long)ns * (Nc - 1) * (Nc - 1) > kMaxCoarse)
    return fail(IRK_EINVAL, "monolithic multigrid needs N = Nc * 2^L with s (Nc-1)^2 <= 1024");
  const int L = (int)sizes.size();
  const size_t tsz = storage_bytes(st->prec);
  st->ml.resize(L);
  for (int l = 0; l < L; ++l) {
    Level& lev = st->ml[l];
    lev.g = make_geom(sizes[l]);
    const long kcount = (long)lev.g.N * lev.g.pitch;
    // buffers are allocated by the first call only (a refresh after a change of kappa reuses them)
    if (l == 0) {
      lev.kap64 = p->kappa;
    } else {
      if (!lev.kap64) CHK(dev_alloc((void**)&lev.kap64, kcount * sizeof(double)));
      lev.own64 = true;
      launch_coarsen_kappa(st->ml[l - 1].kap64, lev.kap64, st->ml[l - 1].g, lev.g, s);
    }
    if (st->prec == 0) {
      lev.kapc = lev.kap64;
    } else {
      if (!lev.kapc) CHK(dev_alloc(&lev.kapc, kcount * sizeof(float)));
      launch_cast_f32(lev.kap64, (float*)lev.kapc, kcount, s);
    }
    const size_t pb = (size_t)ns * lev.g.plane * tsz;
    auto zalloc = [&](void** q) -> int {
      if (!*q) CHK(dev_alloc(q, pb));
      HIPCHK(hipMemsetAsync(*q, 0, pb, s));
      return IRK_OK;
    };
    if (l >= 1) {
      CHK(zalloc(&lev.t));
      CHK(zalloc(&lev.e));
    }
    if (l < L - 1) CHK(zalloc(&lev.x));
  }
  CHK(check_launch());
  // FP64 power iterations in Krylov workspace (cleared again afterwards)
  double* x = st->V;
  double* y = st->V + st->vlen;
  double* z = st->Z;
  for (int tr = 0; tr < 2; ++tr) {
    st->mcoef[tr].assign(L, MMGCoef{});
    st->mmu[tr].assign(L, 0.0);
    for (int l = 0; l < L; ++l) {
      MMGCoef& c = st->mcoef[tr][l];
      c.s = ns;
      c.deg = st->opt.cheb_degree;
      c.m = st->ml[l].g.h * st->ml[l].g.h / 36.0;
      c.dt = st->dt;
      mmg_mixing(st, tr, c);
      if (l == L - 1) continue;
      const Geom& g = st->ml[l].g;
      const long len = (long)ns * g.plane;
      const long nl = (long)(g.N - 1) * (g.N - 1);
      HIPCHK(hipMemsetAsync(x, 0, len * sizeof(double), s));
      HIPCHK(hipMemsetAsync(y, 0, len * sizeof(double), s));
      HIPCHK(hipMemsetAsync(z, 0, len * sizeof(double), s));
      for (int q = 0; q < ns; ++q) launch_start_vector(x + q * g.plane, g, l, s, (uint64_t)(q * nl));
      double* r = res_slot(st, 0);
      double* xx = x;
      double* yy = y;
      for (int it = 0; it < st->opt.power_its; ++it) {
        launch_mmg_apply(xx, yy, st->ml[l].kap64, g, c, 0, s);
        CHK(norm2(st, yy, len, r, nullptr, s));
        launch_scale(yy, len, r, s);
        std::swap(xx, yy);
      }
      launch_mmg_apply(xx, yy, st->ml[l].kap64, g, c, 1, s);  // Acal x
      launch_mmg_apply(xx, z, st->ml[l].kap64, g, c, 2, s);   // C x
      CHK(dot(st, xx, yy, len, res_slot(st, 1), s));
      CHK(dot(st, xx, z, len, res_slot(st, 2), s));
      CHK(check_launch());
      double h[2];
      HIPCHK(hipMemcpyAsync(&h[0], res_slot(st, 1), sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(&h[1], res_slot(st, 2), sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      const double mu = h[0] / h[1];
      if (!(std::isfinite(mu) && mu > 0)) return fail(IRK_EINVAL, "monolithic power iteration produced mu <= 0");
      st->mmu[tr][l] = mu;
      MGCoef cc{};
      cheb_coef(mu, st->opt, cc);
      c.c0 = cc.c0;
      for (int k = 0; k < kMaxDeg; ++k) {
        c.beta[k] = cc.beta[k];
        c.gam[k] = cc.gam[k];
      }
    }
  }
  HIPCHK(hipMemsetAsync(st->V, 0, st->vlen * sizeof(double) * (st->opt.restart + 1), s));
  HIPCHK(hipMemsetAsync(st->Z, 0, st->vlen * sizeof(double) * st->opt.restart, s));
  // coarsest coupled operator cm (x) M + dt ck (x) K, its inverse, and the transposed system's (the transpose)
  const Level& lc = st->ml[L - 1];
  const int N = lc.g.N, m = N - 1, nc = m * m, n = ns * nc;
  std::vector<double> kpad((size_t)N * lc.g.pitch);
  HIPCHK(hipMemcpyAsync(kpad.data(), lc.kap64, kpad.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<double> Mc((size_t)nc * nc, 0.0), Kc((size_t)nc * nc, 0.0);
  host::assemble_q1(kpad.data(), lc.g.pitch, N, Kc.data(), Mc.data());
  const MMGCoef& c0 = st->mcoef[0][L - 1];
  std::vector<double> W((size_t)n * n, 0.0), inv;
  for (int q = 0; q < ns; ++q)
    for (int r = 0; r < ns; ++r) {
      const double a = c0.cm[q * kMMGMax + r], b = st->dt * c0.ck[q * kMMGMax + r];
      if (a == 0.0 && b == 0.0) continue;
      for (int i = 0; i < nc; ++i)
        for (int j = 0; j < nc; ++j)
          W[(size_t)(q * nc + i) * n + r * nc + j] = a * Mc[(size_t)i * nc + j] + b * Kc[(size_t)i * nc + j];
    }
  inv.assign((size_t)n * n, 0.0);
  if (host::dense_inverse(W.data(), n, inv.data()) != 0) return fail(IRK_EINVAL, "singular coarsest coupled operator");
  for (int tr = 0; tr < 2; ++tr) {
    std::vector<double> use(inv.size());
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) use[(size_t)i * n + j] = tr ? inv[(size_t)j * n + i] : inv[(size_t)i * n + j];
    if (st->prec == 0) {
      if (!st->mcinv[tr]) CHK(dev_alloc(&st->mcinv[tr], use.size() * sizeof(double)));
      HIPCHK(hipMemcpy(st->mcinv[tr], use.data(), use.size() * sizeof(double), hipMemcpyHostToDevice));
    } else {
      std::vector<float> f(use.begin(), use.end());
      if (!st->mcinv[tr]) CHK(dev_alloc(&st->mcinv[tr], f.size() * sizeof(float)));
      HIPCHK(hipMemcpy(st->mcinv[tr], f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
    }
  }
  return IRK_OK;
}

// out = one monolithic V-cycle for the coupled system (forward or transposed) applied to tscale * t
// (FP64 padded stage blocks)
int mmg_vcycle(irk_stepper* st, const double* t, const double* tscale, void* out, bool out_f32, bool trans,
               hipStream_t s) {
  std::vector<Level>& ml = st->ml;
  const int L = (int)ml.size();
  const int pr = st->prec, ns = st->s;
  const MMGCoef* cf = st->mcoef[trans ? 1 : 0].data();
  const void* cinv = st->mcinv[trans ? 1 : 0];
  const double nc = (double)ns * nodes(ml[L - 1].g);
  if (L == 1) {
    CHK(arm(st, IRK_KFAM_COARSE_SOLVE, coarse_bytes(st, nc, true, out_f32 ? 4.0 : 8.0)));
    launch_mmg_coarse(pr, true, true, t, tscale, out, cinv, ml[0].g, ns, s, out_f32);
    return check_launch();
  }
  for (int l = 0; l < L - 1; ++l) {
    CHK(arm(st, l == 0 ? IRK_KFAM_MG_FINE : IRK_KFAM_MG_COARSE, mmg_down_bytes(st, l)));
    launch_mmg_down(pr, l == 0, l == 0 ? (const void*)t : ml[l].t, l == 0 ? tscale : nullptr, ml[l].x, ml[l + 1].t,
                    ml[l].kapc, ml[l].g, ml[l + 1].g, cf[l], s);
  }
  CHK(arm(st, IRK_KFAM_COARSE_SOLVE, coarse_bytes(st, nc, false)));
  launch_mmg_coarse(pr, false, false, ml[L - 1].t, nullptr, ml[L - 1].e, cinv, ml[L - 1].g, ns, s);
  for (int l = L - 2; l >= 0; --l) {
    CHK(arm(st, l == 0 ? IRK_KFAM_MG_FINE : IRK_KFAM_MG_COARSE, mmg_up_bytes(st, l, out_f32 ? 4.0 : 8.0)));
    launch_mmg_up(pr, l == 0, l == 0 ? (const void*)t : ml[l].t, l == 0 ? tscale : nullptr, ml[l].x, ml[l + 1].e,
                  l == 0 ? out : ml[l].e, ml[l].kapc, ml[l].g, ml[l + 1].g, cf[l], s, l == 0 && out_f32);
  }
  return check_launch();
}

// ------------------------------------------------------------------ preconditioner

// out = one V-cycle for block `stage` applied to tscale * t (FP64 padded planes; out FP32 with out_f32)
int vcycle(irk_stepper* st, int stage, const double* t, const double* tscale, void* out, bool out_f32, hipStream_t s,
           const Couple* cpl = nullptr) {
  const int L = (int)st->lv.size();
  Couple none{};
  const Couple& cp = cpl ? *cpl : none;
  const MGCoef* cf = &st->coef[(size_t)stage * L];
  const int pr = st->prec;
  if (L == 1) {
    CHK(arm(st, IRK_KFAM_COARSE_SOLVE, coarse_bytes(st, nodes(st->lv[0].g), true, out_f32 ? 4.0 : 8.0)));
    launch_mg_coarse(pr, true, t, tscale, out, st->binv[stage], st->lv[0].g, s, out_f32);
    return check_launch();
  }
  std::vector<Level>& lv = st->lv;
  // the three levels above the coarsest run as one DOWN and one UP launch when they are not the finest level
  const int A3 = L - 4;
  const bool three = A3 >= 1;
  ThreeLevels z{};
  if (three) {
    for (int q = 0; q < 4; ++q) {
      const Level& lq = lv[A3 + q];
      z.g[q] = lq.g;
      z.t[q] = lq.t;
      z.e[q] = lq.e;
      if (q < 3) {
        z.c[q] = cf[A3 + q];
        z.x[q] = lq.x;
        z.kap[q] = lq.kapc;
      }
    }
  }
  // the finest DOWN stores the right-hand side it smoothed (scaled, with the stage coupling) for the finest UP
  CHK(arm(st, IRK_KFAM_MG_FINE, mg_down_bytes(st, 0, cp.nz, cp.z_f32 ? 4.0 : 8.0)));
  launch_mg_down(pr, true, t, tscale, lv[0].x, lv[1].t, lv[0].tp, lv[0].kapc, lv[0].g, lv[1].g, cf[0], cp, s);
  for (int l = 1; l < (three ? A3 : L - 1); ++l) {
    CHK(arm(st, IRK_KFAM_MG_COARSE, mg_down_bytes(st, l, 0)));
    launch_mg_down(pr, false, lv[l].t, nullptr, lv[l].x, lv[l + 1].t, nullptr, lv[l].kapc, lv[l].g, lv[l + 1].g, cf[l],
                   none, s);
  }
  if (three) {
    CHK(arm(st, IRK_KFAM_MG_COARSE, mg_down3_bytes(st, A3)));
    launch_mg_down3(pr, z, s);
  }
  CHK(arm(st, IRK_KFAM_COARSE_SOLVE, coarse_bytes(st, nodes(lv[L - 1].g), false)));
  launch_mg_coarse(pr, false, lv[L - 1].t, nullptr, lv[L - 1].e, st->binv[stage], lv[L - 1].g, s);
  if (three) {
    CHK(arm(st, IRK_KFAM_MG_COARSE, mg_up3_bytes(st, A3)));
    launch_mg_up3(pr, z, s);
  }
  for (int l = (three ? A3 - 1 : L - 2); l >= 1; --l) {
    CHK(arm(st, IRK_KFAM_MG_COARSE, mg_up_bytes(st, l)));
    launch_mg_up(pr, false, lv[l].t, lv[l].x, lv[l + 1].e, lv[l].e, lv[l].kapc, lv[l].g, lv[l + 1].g, cf[l], s);
  }
  CHK(arm(st, IRK_KFAM_MG_FINE, mg_up_bytes(st, 0, out_f32 ? 4.0 : 8.0)));
  launch_mg_up(pr, true, lv[0].tp, lv[0].x, lv[1].e, out, lv[0].kapc, lv[0].g, lv[1].g, cf[0], s, out_f32);
  return check_launch();
}

// z = P^{-1} (vscale * v) for the block-triangular stage preconditioner (vscale: device scalar or null).
// AI form: P = I (x) M + dt Atil (x) K, z_i = B_i^{-1} (v_i - dt K sum_j atil_ij z_j).
// IA form: P = Atil^{-1} (x) M + dt I (x) K, z_i = atil_ii B_i^{-1} (v_i - M sum_j c_ij z_j) with
// C = Atil^{-1}, B_i = M + dt atil_ii K (one V-cycle is linear, so atil_ii scales its input).
// z: FP64 planes, or FP32 planes with zf (the stage coupling then reads them as FP32)
int precondition(irk_stepper* st, const double* v, const double* vscale, void* z, bool zf, bool trans, hipStream_t s) {
  if (st->sys >= 0) return vcycle(st, st->sys, v, vscale, z, zf, s);  // one DIRK stage: one V-cycle
  if (st->opt.precond == IRK_PC_MONOLITHIC) return mmg_vcycle(st, v, vscale, z, zf, trans, s);
  const long plane = st->g.plane;
  // stage plane q of z
  auto zplane = [&](int q) -> void* {
    return zf ? (void*)((float*)z + (long)q * plane) : (void*)((double*)z + (long)q * plane);
  };
  const int ns = st->s;
  const Coefs a = ptil_of(st, trans);
  const double* Ci = st->Ci[trans ? 1 : 0];
  // Atil is lower triangular (forward substitution) except for P_U (backward substitution), and the
  // transposed system uses Atil^T (the other way round); stage i is coupled to the nc stages solved
  // before it, which sit contiguously from stage j0 on
  const bool upper = (st->opt.precond == IRK_PC_GS_UPPER) != trans;
  for (int step = 0; step < ns; ++step) {
    const int i = upper ? ns - 1 - step : step;
    const int j0 = upper ? i + 1 : 0;
    const int nc = (st->opt.precond == IRK_PC_JACOBI) ? 0 : step;
    const double vmul = st->ia ? st->pd[i] : 1.0;
    const double* vi = v + i * plane;
    void* zi = zplane(i);
    double row[kMaxStages] = {};
    for (int q = 0; q < nc; ++q)
      row[q] = st->ia ? vmul * Ci[i * ns + j0 + q] : a.a[i * kMaxStages + j0 + q];
    if (nc > 0 || vmul != 1.0) {
      if (st->lv.size() > 1) {
        // the coupling and the scale are applied inside the finest-level kernels
        Couple cp{};
        cp.z = zplane(j0);
        cp.z_f32 = zf ? 1 : 0;
        cp.zstride = plane;
        cp.nz = nc;
        cp.mass = st->ia ? 1 : 0;
        cp.dt = st->ia ? 1.0 : st->dt;
        cp.mh = st->g.h * st->g.h / 36.0;
        cp.vmul = vmul;
        for (int q = 0; q < nc; ++q) cp.a[q] = row[q];
        CHK(vcycle(st, i, vi, vscale, zi, zf, s, &cp));
      } else {
        Coefs r{};
        for (int q = 0; q < nc; ++q) r.a[q] = row[q];
        double* t = st->tmp2;
        const double gb = nodes(st->g) * (24.0 + (zf ? 4.0 : 8.0) * nc);
        CHK(timer_arm(st, IRK_KFAM_OTHER, gb, gb));
        if (zf)
          launch_gs_couple(vi, vscale, (const float*)zplane(j0), nc, r, st->ia ? 1.0 : st->dt, st->prob->kappa, t,
                           st->g, s, st->ia ? 1 : 0, vmul);
        else
          launch_gs_couple(vi, vscale, (const double*)zplane(j0), nc, r, st->ia ? 1.0 : st->dt, st->prob->kappa, t,
                           st->g, s, st->ia ? 1 : 0, vmul);
        CHK(vcycle(st, i, t, nullptr, zi, zf, s));
      }
    } else {
      CHK(vcycle(st, i, vi, vscale, zi, zf, s));
    }
  }
  return check_launch();
}

// y = Acal x (y = f - Acal x with f); xf: x is FP32 (a vector of the mixed form's flexible basis) at xf instead
int apply_op(irk_stepper* st, const double* x, double* y, const double* f, bool trans, hipStream_t s,
             const float* xf = nullptr) {
  const int ns = st->sys >= 0 ? 1 : st->s;
  const double ob = nodes(st->g) * ((xf ? 4.0 : 8.0) * ns + 8.0 * ns + 8.0 + (f ? 8.0 * ns : 0.0));
  CHK(timer_arm(st, IRK_KFAM_OPERATOR, ob, ob));
  Coefs a{};
  if (st->sys >= 0) a.a[0] = st->A[st->sys * st->s + st->sys];  // one DIRK stage: M + dt a_ii K (symmetric)
  const Coefs& c = st->sys >= 0 ? a : coefs_of(st, trans);
  const bool ia = st->sys < 0 && st->ia;
  if (xf)
    launch_stage_operator(xf, y, f, st->prob->kappa, st->g, ns, c, st->dt, s, ia);
  else
    launch_stage_operator(x, y, f, st->prob->kappa, st->g, ns, c, st->dt, s, ia);
  return check_launch();
}

// ------------------------------------------------------------------ Arnoldi step

// Everything one FGMRES iteration j enqueues between two host decisions:
// Z_j = P^{-1}(sigma_j V_j), w = Acal Z_j into V_{j+1}, then classical Gram-Schmidt
// with re-orthogonalisation (passes A, B, C) against V_0..V_j. Scales are read
// from device memory, so the sequence is replayable as a graph.
int arnoldi_body(irk_stepper* st, int j, bool trans, hipStream_t s) {
  const long n = sys_len(st);
  double* sig = sigma_dev(st);
  double* Vj = st->V + (long)j * n;
  double* Vn = st->V + (long)(j + 1) * n;
  double* Zj = st->Z + (long)j * n;
  if (st->opt.orth == IRK_ORTH_DCGS2) {
    // Z_j = P^{-1} u_j (u_j = V_j: the previous direction, projected once), w = Acal Z_j into V_{j+1},
    // then one reduction and one update pass: V_j <- q_j, V_{j+1} <- the next direction
    CHK(precondition(st, Vj, nullptr, Zj, st->zf32, trans, s));
    CHK(apply_op(st, Zj, Vn, nullptr, trans, s, st->zf32 ? (const float*)Zj : nullptr));
    D2Args d{st->V, n, j, Vj, Vn, n, dcgs2_dev(st, j & 1), st->hmir_dev + (long)(j & 1) * kDcgs2Res};
    hipEvent_t e0, e1, e2, e3;
    const double b0 = dcgs2_bytes(st, j, n, false), b1 = dcgs2_bytes(st, j, n, true);
    CHK(timer_pair(st, IRK_KFAM_GRAM_SCHMIDT, b0, b0, &e0, &e1));
    CHK(timer_arm(st, IRK_KFAM_REDUCE_FINISH, 0, 0));
    launch_dcgs2_dots(d, st->rw, s, e0, e1);
    CHK(timer_pair(st, IRK_KFAM_GRAM_SCHMIDT, b1, b1, &e2, &e3));
    launch_dcgs2_update(d, st->rw, s, e2, e3);
    return check_launch();
  }
  CHK(precondition(st, Vj, sig + j, Zj, st->zf32, trans, s));
  CHK(apply_op(st, Zj, Vn, nullptr, trans, s, st->zf32 ? (const float*)Zj : nullptr));
  // pass A: h = V^T w, |w|^2
  OrthoArgs a = ortho_base();
  a.V = st->V;
  a.vstride = n;
  a.nv = j + 1;
  a.w = Vn;
  a.len = n;
  a.vscale = sig;
  a.want_dots = 1;
  a.result = res_slot(st, 0);
  CHK(ortho(st, a, s));
  // pass B: w -= V h; h2 = V^T w; |w|^2; flag = |w|^2 < eta^2 |w_before|^2
  OrthoArgs b = a;
  b.coef = res_slot(st, 0);
  b.result = res_slot(st, 1);
  b.sigma_out = sig + (j + 1);
  b.flag_out = st->dflag;
  b.ref = res_slot(st, 0) + (j + 1);
  b.eta2 = 0.5;
  CHK(ortho(st, b, s));
  // pass C: w -= V h2; |w|^2 (skipped unless needed for the selective variant)
  OrthoArgs c = a;
  c.coef = res_slot(st, 1);
  c.want_dots = 0;
  c.result = res_slot(st, 2);
  c.sigma_out = sig + (j + 1);
  c.skip = st->opt.orth == IRK_ORTH_CGS_SELECTIVE ? st->dflag : nullptr;
  CHK(ortho(st, c, s));
  return IRK_OK;
}

// Enqueue Arnoldi step j on s: replay its captured graph (captured on first use), or eagerly.
int run_arnoldi(irk_stepper* st, int j, bool trans, hipStream_t s) {
  if (!st->opt.use_graphs || st->timer_family >= 0) return arnoldi_body(st, j, trans, s);
  std::vector<hipGraphExec_t>& gs = st->graphs[st->sys >= 0 ? 2 + st->sys : (trans ? 1 : 0)];
  if (gs.empty()) gs.assign(st->opt.restart, nullptr);
  if (!gs[j]) {
    HIPCHK(hipStreamBeginCapture(st->cap, hipStreamCaptureModeRelaxed));
    const int rc = arnoldi_body(st, j, trans, st->cap);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(st->cap, &graph);
    if (rc != IRK_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail(IRK_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    hipGraphExec_t ge = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) return fail(IRK_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e2));
    gs[j] = ge;
  }
  HIPCHK(hipGraphLaunch(gs[j], s));
  return IRK_OK;
}

// ------------------------------------------------------------------ FGMRES

struct SolveInfo {
  int its = 0, restarts = 0;
  double rel = 0;
  int solves = 0, its_max = 0;
  int discarded = 0;  // Arnoldi steps launched ahead of the host's decision and not used
};

// the flexible basis as the basis of an update pass (x = Z y): Z_j starts n FP64 values after Z_{j-1}, so an FP32
// basis has a stride of 2n values
void set_z_basis(const irk_stepper* st, OrthoArgs& a, long n) {
  if (st->zf32) {
    a.V = nullptr;
    a.Vf = (const float*)st->Z;
    a.vstride = 2 * n;
  } else {
    a.V = st->Z;
    a.vstride = n;
  }
}

// FGMRES with the delayed CGS2 Arnoldi process. The Hessenberg column of step j is provisional until
// step j+1 re-orthogonalises and normalises the direction it produced: then the column gains the
// re-orthogonalisation coefficients and its subdiagonal entry becomes that direction's exact norm
// (the provisional entry is the norm predicted from the reduction of step j).
int fgmres_dcgs2(irk_stepper* st, const double* f, bool trans, bool use_guess, SolveInfo& info, hipStream_t s,
                 double* x, bool v0_is_f) {
  const int m = st->opt.restart;
  const long n = sys_len(st);
  double* h = st->hres;
  info = SolveInfo{};
  // Enqueue step k and an event behind it: the host can wait for step k alone (its reduction lands in
  // mirror slot k % 2) while later work is already queued behind it.
  auto launch_step = [&](int k) -> int {
    CHK(run_arnoldi(st, k, trans, s));
    HIPCHK(hipEventRecord(st->step_ev[k & 1], s));
    return IRK_OK;
  };
  // |f| and the initial residual r_0 = V_0 (= f without a guess). Step 0 needs neither norm on the host
  // (it normalises u_0 from its own reduction), so it is queued before the host waits for them.
  CHK(norm2(st, f, n, res_slot(st, 0), nullptr, s));
  // without a guess x is not cleared: the first cycle's solution update assigns x = Z y (x_unset)
  bool x_unset = !use_guess;
  if (use_guess) {
    CHK(apply_op(st, x, st->V, f, trans, s));
    CHK(norm2(st, st->V, n, res_slot(st, 0) + 1, nullptr, s));
  } else if (!v0_is_f) {
    HIPCHK(hipMemcpyAsync(st->V, f, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  HIPCHK(hipMemcpyAsync(h, res_slot(st, 0), 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipEventRecord(st->norm_ev, s));
  const int look = st->opt.lookahead;
  // step 1 goes in with step 0 when the last solve of this system needed three or more iterations
  const int key = st->sys >= 0 ? 2 + st->sys : (trans ? 1 : 0);
  const bool two = m > 1 && st->opt.max_it >= 2 &&
                   (look == IRK_LOOKAHEAD_ALWAYS || (look == IRK_LOOKAHEAD_ADAPTIVE && st->last_its[key] >= 3));
  bool step0_queued = look != IRK_LOOKAHEAD_OFF;
  if (step0_queued) CHK(launch_step(0));
  if (step0_queued && two) CHK(launch_step(1));
  HIPCHK(hipEventSynchronize(st->norm_ev));
  const double fnorm = std::sqrt(h[0]);
  if (!std::isfinite(fnorm)) return fail(IRK_EBREAKDOWN, "non-finite right-hand side");
  if (fnorm == 0.0) {
    HIPCHK(hipMemsetAsync(x, 0, n * sizeof(double), s));
    info.discarded = step0_queued ? (two ? 2 : 1) : 0;
    return IRK_OK;
  }
  double beta = use_guess ? std::sqrt(h[1]) : fnorm;
  const double target = st->opt.rtol * fnorm;
  if (beta <= target) {
    if (x_unset) HIPCHK(hipMemsetAsync(x, 0, n * sizeof(double), s));
    info.rel = beta / fnorm;
    info.discarded = step0_queued ? (two ? 2 : 1) : 0;
    st->last_its[key] = 0;
    return IRK_OK;
  }
  std::vector<double> H((size_t)(m + 1) * m), y(m);
  while (true) {
    std::fill(H.begin(), H.end(), 0.0);
    double g0 = beta;
    int jdone = 0;
    double est_prev = beta;
    int launched = 0;  // highest step enqueued in this cycle
    if (step0_queued) {
      launched = two ? 1 : 0;
    } else {
      CHK(launch_step(0));
    }
    step0_queued = false;
    int read = 0;      // highest step whose reduction the host has taken
    for (int j = 0; j < m; ++j) {
      HIPCHK(hipEventSynchronize(st->step_ev[j & 1]));
      read = j;
      const double* hj_res = st->hmir + (long)(j & 1) * kDcgs2Res;
      const int cnt = 2 * j + 3;
      bool finite = true;
      for (int i = 0; i < cnt + 5; ++i) finite = finite && std::isfinite(hj_res[i]);
      if (!finite) return fail(IRK_EBREAKDOWN, "non-finite Hessenberg entry in FGMRES");
      const double* a = hj_res;
      const double* sw = hj_res + j;
      const double bj = hj_res[cnt], hj = hj_res[cnt + 2], nu = hj_res[cnt + 3];
      if (hj_res[cnt + 4] != 0.0) {
        // the direction u_j vanished: the Krylov space is invariant and column j-1 is exact
        if (j == 0) return fail(IRK_EBREAKDOWN, "zero initial direction in FGMRES");
        for (int i = 0; i < j; ++i) H[(size_t)i * m + (j - 1)] += a[i];
        H[(size_t)j * m + (j - 1)] = 0.0;
        break;
      }
      if (j == 0) {
        g0 = bj;
        est_prev = bj;
      } else {
        for (int i = 0; i < j; ++i) H[(size_t)i * m + (j - 1)] += a[i];
        H[(size_t)j * m + (j - 1)] = bj;
      }
      for (int i = 0; i < j; ++i) H[(size_t)i * m + j] = sw[i];
      H[(size_t)j * m + j] = hj;
      H[(size_t)(j + 1) * m + j] = std::sqrt(std::max(nu, 0.0));
      info.its++;
      jdone = j + 1;
      const double est = host::hessenberg_ls(H.data(), m, jdone, g0, nullptr);
      if (est <= target || H[(size_t)(j + 1) * m + j] <= 1e-300 * std::fabs(hj)) break;
      if (info.its >= st->opt.max_it) break;
      if (j + 1 < m && launched == j) {
        CHK(launch_step(j + 1));
        launched = j + 1;
      }
      // Step j+2 goes in behind step j+1 when the last reduction factor, applied once more, still leaves
      // the estimate well above the target: the host then decides on step j+1 while step j+2 runs.
      // A step launched this way and not needed is discarded (it writes only V_{j+2}, V_{j+3}, Z_{j+2}).
      const double rate = est_prev > 0 ? est / est_prev : 1.0;
      est_prev = est;
      const bool ahead = look == IRK_LOOKAHEAD_ALWAYS ||
                         (look == IRK_LOOKAHEAD_ADAPTIVE && est * std::min(rate, 1.0) > kLookaheadMargin * target);
      if (launched == j + 1 && j + 2 < m && info.its + 2 <= st->opt.max_it && ahead) {
        CHK(launch_step(j + 2));
        launched = j + 2;
      }
    }
    info.discarded += launched - read;
    if (jdone > 0) {
      host::hessenberg_ls(H.data(), m, jdone, g0, y.data());
      std::copy(y.begin(), y.begin() + jdone, h);
      HIPCHK(hipMemcpyAsync(ycoef_dev(st), h, jdone * sizeof(double), hipMemcpyHostToDevice, s));
      OrthoArgs ax = ortho_base();
      set_z_basis(st, ax, n);
      ax.nv = jdone;
      ax.w = x;
      ax.len = n;
      ax.coef = ycoef_dev(st);
      ax.coef_sign = -1.0;
      ax.assign = x_unset ? 1 : 0;
      ax.result = res_slot(st, 3);
      CHK(ortho(st, ax, s));
      x_unset = false;
    }
    if (x_unset) {
      HIPCHK(hipMemsetAsync(x, 0, n * sizeof(double), s));
      x_unset = false;
    }
    CHK(apply_op(st, x, st->V, f, trans, s));
    CHK(norm2(st, st->V, n, res_slot(st, 0), nullptr, s));
    HIPCHK(hipMemcpyAsync(h, res_slot(st, 0), sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    beta = std::sqrt(h[0]);
    info.rel = beta / fnorm;
    if (!std::isfinite(beta)) return fail(IRK_EBREAKDOWN, "non-finite residual in FGMRES");
    st->last_its[key] = info.its;
    if (beta <= target) return IRK_OK;
    if (info.its >= st->opt.max_it) {
      char buf[160];
      snprintf(buf, sizeof buf, "FGMRES reached max_it = %d with relative residual %.3e > rtol %.3e", st->opt.max_it,
               info.rel, st->opt.rtol);
      return fail(IRK_ENOCONV, buf);
    }
    info.restarts++;
  }
}

// Solve Acal x = f (padded planes) for the current system; x defaults to st->k. If use_guess, x holds
// the initial guess.
int fgmres(irk_stepper* st, const double* f, bool trans, bool use_guess, SolveInfo& info, hipStream_t s,
           double* x = nullptr) {
  if (!x) x = st->k;
  const bool v0_is_f = st->v0_is_f && f == st->f;
  st->v0_is_f = false;
  if (st->opt.orth == IRK_ORTH_DCGS2) return fgmres_dcgs2(st, f, trans, use_guess, info, s, x, v0_is_f);
  const int m = st->opt.restart;
  const long n = sys_len(st);
  double* sig = sigma_dev(st);
  double* h = st->hres;
  info = SolveInfo{};
  // |f|
  CHK(norm2(st, f, n, res_slot(st, 0), nullptr, s));
  HIPCHK(hipMemcpyAsync(h, res_slot(st, 0), sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double fnorm = std::sqrt(h[0]);
  if (!std::isfinite(fnorm)) return fail(IRK_EBREAKDOWN, "non-finite right-hand side");
  if (fnorm == 0.0) {
    HIPCHK(hipMemsetAsync(x, 0, n * sizeof(double), s));
    return IRK_OK;
  }
  // initial residual into V_0
  if (use_guess) {
    CHK(apply_op(st, x, st->V, f, trans, s));
  } else {
    HIPCHK(hipMemsetAsync(x, 0, n * sizeof(double), s));
    HIPCHK(hipMemcpyAsync(st->V, f, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  CHK(norm2(st, st->V, n, res_slot(st, 0), sig, s));
  HIPCHK(hipMemcpyAsync(h, res_slot(st, 0), sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double beta = std::sqrt(h[0]);
  const double target = st->opt.rtol * fnorm;
  if (beta <= target) {
    info.rel = beta / fnorm;
    return IRK_OK;
  }
  const bool selective = st->opt.orth == IRK_ORTH_CGS_SELECTIVE;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), sig_h(m + 1), y(m);
  while (true) {
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    sig_h[0] = 1.0 / beta;
    int jdone = 0;
    bool converged_est = false;
    for (int j = 0; j < m; ++j) {
      CHK(run_arnoldi(st, j, trans, s));
      HIPCHK(hipMemcpyAsync(h, st->dres, 3L * RSTRIDE * sizeof(double), hipMemcpyDeviceToHost, s));
      int flag = 1;
      if (selective) HIPCHK(hipMemcpyAsync(&flag, st->dflag, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      const bool reorth = !selective || flag != 0;
      const double* rA = h;
      const double* rB = h + RSTRIDE;
      const double* rC = h + 2 * RSTRIDE;
      double* col = &H[(size_t)j];  // column j, row stride m
      for (int i = 0; i <= j; ++i) col[(size_t)i * m] = rA[i] + (reorth ? rB[i] : 0.0);
      const double hn = std::sqrt(reorth ? rC[j + 1] : rB[j + 1]);
      bool finite = std::isfinite(hn);
      for (int i = 0; i <= j; ++i) finite = finite && std::isfinite(col[(size_t)i * m]);
      if (!finite) return fail(IRK_EBREAKDOWN, "non-finite Hessenberg entry in FGMRES");
      sig_h[j + 1] = 1.0 / hn;
      // Givens rotations
      for (int i = 0; i < j; ++i) {
        const double t0 = cs[i] * col[(size_t)i * m] + sn[i] * col[(size_t)(i + 1) * m];
        const double t1 = -sn[i] * col[(size_t)i * m] + cs[i] * col[(size_t)(i + 1) * m];
        col[(size_t)i * m] = t0;
        col[(size_t)(i + 1) * m] = t1;
      }
      const double hj = col[(size_t)j * m];
      const double r = std::hypot(hj, hn);
      cs[j] = hj / r;
      sn[j] = hn / r;
      col[(size_t)j * m] = r;
      col[(size_t)(j + 1) * m] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      info.its++;
      jdone = j + 1;
      if (std::fabs(gv[j + 1]) <= target || hn <= 1e-300 * std::max(1.0, r)) {
        converged_est = true;
        break;
      }
      if (info.its >= st->opt.max_it) break;
    }
    // y = R^{-1} g
    for (int i = jdone - 1; i >= 0; --i) {
      double v = gv[i];
      for (int c2 = i + 1; c2 < jdone; ++c2) v -= H[(size_t)i * m + c2] * y[c2];
      y[i] = v / H[(size_t)i * m + i];
    }
    // k += Z y
    std::copy(y.begin(), y.begin() + jdone, h);
    HIPCHK(hipMemcpyAsync(ycoef_dev(st), h, jdone * sizeof(double), hipMemcpyHostToDevice, s));
    {
      OrthoArgs a = ortho_base();
      set_z_basis(st, a, n);
      a.nv = jdone;
      a.w = x;
      a.len = n;
      a.coef = ycoef_dev(st);
      a.coef_sign = -1.0;
      a.result = res_slot(st, 3);
      CHK(ortho(st, a, s));
    }
    // true residual r = f - Acal k into V_0
    CHK(apply_op(st, x, st->V, f, trans, s));
    CHK(norm2(st, st->V, n, res_slot(st, 0), sig, s));
    HIPCHK(hipMemcpyAsync(h, res_slot(st, 0), sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    beta = std::sqrt(h[0]);
    info.rel = beta / fnorm;
    if (!std::isfinite(beta)) return fail(IRK_EBREAKDOWN, "non-finite residual in FGMRES");
    if (beta <= target) return IRK_OK;
    if (info.its >= st->opt.max_it) {
      char buf[160];
      snprintf(buf, sizeof buf, "FGMRES reached max_it = %d with relative residual %.3e > rtol %.3e", st->opt.max_it,
               info.rel, st->opt.rtol);
      return fail(IRK_ENOCONV, buf);
    }
    (void)converged_est;
    info.restarts++;
  }
}

void add_stats(irk_stats* stats, const SolveInfo& si) {
  if (!stats) return;
  stats->fgmres_its_total += si.its;
  stats->fgmres_its_max = std::max(stats->fgmres_its_max, std::max(si.its_max, si.solves ? 0 : si.its));
  stats->restarts_total += si.restarts;
  stats->arnoldi_discarded += si.discarded;
  stats->solves += std::max(1, si.solves);
  stats->last_rel_resid = si.rel;
}

// Solve the stage system (I (x) M + dt A (x) K) k = f (A^T if trans) into st->k: one FGMRES on the coupled
// system, or, for a DIRK stepper, block substitution with one single-stage FGMRES per stage (Section 2.3):
// (M + dt a_ii K) k_i = f_i - dt K sum_{j<i} a_ij k_j (transposed: backwards, j > i with a_ji).
// The interior-only kernels (stage operator, stage right-hand side, multigrid levels) rely on every padded plane
// holding zeros in its boundary ring and padding. The flat vector kernels (Arnoldi updates, solution update) write
// those entries as 0 * c, which stays zero only while every coefficient c is finite. After a breakdown on
// non-finite data (including Arnoldi steps queued ahead of the host's check), the work planes are cleared to the
// state set-up left, so the stepper's next solve is unaffected. The state plane u is left alone (it holds the
// last good state the caller gets back).
int clear_work(irk_stepper* st, hipStream_t s) {
  const size_t vb = st->vlen * sizeof(double);
  const size_t tb = (size_t)std::max(st->s, 2) * st->g.plane * sizeof(double);
  auto clr = [&](void* q, size_t bytes) -> int {
    if (q) HIPCHK(hipMemsetAsync(q, 0, bytes, s));
    return IRK_OK;
  };
  CHK(clr(st->V, vb * (st->opt.restart + 1)));
  CHK(clr(st->Z, vb * st->opt.restart));
  CHK(clr(st->f, vb));
  CHK(clr(st->k, vb));
  CHK(clr(st->tmp, tb));
  CHK(clr(st->tmp2, tb));
  const size_t tsz = storage_bytes(st->prec);
  for (const Level& lev : st->lv) {
    const size_t pb = lev.g.plane * tsz;
    CHK(clr(lev.t, pb));
    CHK(clr(lev.e, pb));
    CHK(clr(lev.x, pb));
    CHK(clr(lev.tp, lev.g.plane * (st->prec == 0 ? sizeof(double) : sizeof(float))));
  }
  for (const Level& lev : st->ml) {
    const size_t pb = (size_t)st->s * lev.g.plane * tsz;
    CHK(clr(lev.t, pb));
    CHK(clr(lev.e, pb));
    CHK(clr(lev.x, pb));
  }
  return IRK_OK;
}

int stage_solve_run(irk_stepper* st, const double* f, bool trans, bool use_guess, SolveInfo& info, hipStream_t s);

int stage_solve(irk_stepper* st, const double* f, bool trans, bool use_guess, SolveInfo& info, hipStream_t s) {
  const int rc = stage_solve_run(st, f, trans, use_guess, info, s);
  if (rc == IRK_EBREAKDOWN) {
    const std::string keep = g_err;
    (void)clear_work(st, s);
    g_err = keep;
  }
  return rc;
}

int stage_solve_run(irk_stepper* st, const double* f, bool trans, bool use_guess, SolveInfo& info, hipStream_t s) {
  if (!st->dirk) return fgmres(st, f, trans, use_guess, info, s);
  info = SolveInfo{};
  const int ns = st->s;
  const long plane = st->g.plane;
  for (int step = 0; step < ns; ++step) {
    const int i = trans ? ns - 1 - step : step;
    const int j0 = trans ? i + 1 : 0;
    const double* rhs = f + i * plane;
    if (step > 0) {
      Coefs row{};
      for (int q = 0; q < step; ++q)
        row.a[q] = trans ? st->A[(j0 + q) * ns + i] : st->A[i * ns + j0 + q];
      launch_gs_couple(f + i * plane, nullptr, st->k + j0 * plane, step, row, st->dt, st->prob->kappa, st->tmp2,
                       st->g, s);
      CHK(check_launch());
      rhs = st->tmp2;
    }
    SolveInfo si;
    st->sys = i;
    const int rc = fgmres(st, rhs, false, use_guess, si, s, st->k + i * plane);
    st->sys = -1;
    info.its += si.its;
    info.restarts += si.restarts;
    info.discarded += si.discarded;
    info.its_max = std::max(info.its_max, si.its);
    info.rel = std::max(info.rel, si.rel);
    info.solves++;
    if (rc != IRK_OK) return rc;
  }
  return IRK_OK;
}

void init_stats(irk_stats* stats) {
  if (!stats) return;
  std::memset(stats, 0, sizeof(*stats));
  stats->failed_step = -1;
}

// one forward step on st->u (padded); stage derivatives left in st->k
int forward_step(irk_stepper* st, const double* Fp, SolveInfo& si, hipStream_t s) {
  const double n = nodes(st->g), rb = n * (16.0 + (Fp ? 8.0 : 0.0) + 8.0 * st->s), ub = n * (8.0 * st->s + 16.0);
  const bool guess = st->opt.initial_guess == IRK_GUESS_PREV && st->have_prev;
  // the coupled DCGS2 solve without a guess starts from V_0 = f: the kernel writes that copy too
  const bool f_to_v0 = !guess && !st->dirk && st->opt.orth == IRK_ORTH_DCGS2;
  CHK(timer_arm(st, IRK_KFAM_OTHER, rb + (f_to_v0 ? n * 8.0 * st->s : 0.0), rb + (f_to_v0 ? n * 8.0 * st->s : 0.0)));
  launch_stage_rhs(st->u, Fp, st->f, st->prob->kappa, st->g, st->s, s, f_to_v0 ? st->V : nullptr);
  st->v0_is_f = f_to_v0;
  CHK(stage_solve(st, st->f, false, guess, si, s));
  st->have_prev = true;
  CHK(timer_arm(st, IRK_KFAM_OTHER, ub, ub));
  launch_update(st->u, st->k, st->s, b_of(st), st->dt, st->g, s);
  return check_launch();
}

// ------------------------------------------------------------------ binomial checkpointing

// y = M x (op 0) or K x (op 1) on one compact nodal vector, through two padded staging planes at xp (the pack
// kernel writes every value of the first plane, boundary ring and padding as zeros; the stencil writes the
// interior of the second, the only part unpack reads), enqueued on s
int apply_nodal(const irk_problem* p, int op, const double* x, double* y, double* xp, hipStream_t s) {
  double* yp = xp + p->g.plane;
  launch_pack(x, xp, p->g, 1, s);
  if (op == 0)
    launch_mass(xp, yp, p->g, s);
  else
    launch_stiff(xp, yp, p->kappa, p->g, s);
  launch_unpack(yp, y, p->g, 1, s);
  return check_launch();
}

// the problem's staging planes (allocated by the first call that needs them)
int problem_stage(const irk_problem* p, double** out) {
  std::lock_guard<std::mutex> lk(p->stage_mu);
  if (!p->stage) CHK(dev_alloc((void**)&p->stage, 2 * p->g.plane * sizeof(double)));
  *out = p->stage;
  return IRK_OK;
}

// Staging of irk_apply_mass_noalloc: a static device array (two padded planes at N = kScratchMaxN), which every
// GPU the library runs on holds until the process ends. In host code its name is only a stand-in: the device
// address is looked up once per device (hipGetSymbolAddress, with that device current) and used from then on.
constexpr int kScratchMaxN = 1024;
constexpr long kScratchDoubles = 2L * (kScratchMaxN + 1) * ((kScratchMaxN + 1 + 15) / 16 * 16);
static __device__ __align__(256) double scratch[kScratchDoubles];
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;

int scratch_of_device(int dev, double** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != dev)
      return fail(IRK_EINVAL, "the problem's device (" + std::to_string(dev) + ") must be current on the first call");
    void* a = nullptr;
    HIPCHK(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = (double*)a;
  }
  *out = g_scratch_ptr[dev];
  return IRK_OK;
}

// Checks kappa (N * N element values, device) and, only if every value is finite and positive, packs it into the
// problem's padded layout; waits for the stream (the check's verdict is read on the host).
int load_kappa(irk_problem* p, const double* kappa, hipStream_t s) {
  const int N = p->N;
  int hbad = 0;
  hipError_t e = hipMemsetAsync(p->bad, 0, sizeof(int), s);
  if (e == hipSuccess) {
    launch_check_kappa(kappa, N * N, p->bad, s);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&hbad, p->bad, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(IRK_EHIP, std::string("kappa check: ") + hipGetErrorString(e));
  if (hbad) return fail(IRK_EINVAL, "kappa must be finite and positive everywhere");
  launch_pack_elem(kappa, p->kappa, p->g, s);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(IRK_EHIP, std::string("kappa packing: ") + hipGetErrorString(e));
  return IRK_OK;
}

int validate_stepper(const irk_stepper* st) {
  if (!st) return fail(IRK_EINVAL, "stepper is NULL");
  return IRK_OK;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

const char* irk_last_error(void) { return g_err.c_str(); }

void irk_options_default(irk_options* o) {
  if (!o) return;
  o->precond = IRK_PC_GS_LOWER;
  o->rtol = 1e-10;
  o->restart = 30;
  o->max_it = 300;
  o->mg_coarse_n = 32;
  o->cheb_degree = 2;
  o->cheb_lo = 0.25;
  o->cheb_hi = 1.1;
  o->power_its = 15;
  o->mg_precision = IRK_F64;
  o->orth = IRK_ORTH_DCGS2;
  o->initial_guess = IRK_GUESS_ZERO;
  o->use_graphs = 1;
  o->splitting = IRK_SPLIT_AI;
  o->stage_type = IRK_STAGE_COUPLED;
  o->lookahead = IRK_LOOKAHEAD_ADAPTIVE;
  o->basis_f64 = 0;
}

int irk_problem_create(irk_problem** out, int N, const double* kappa, void* stream) {
  g_err.clear();
  if (!out) return fail(IRK_EINVAL, "out is NULL");
  *out = nullptr;
  if (N < 2 || N > 16384) return fail(IRK_EINVAL, "N must be in [2, 16384]");
  if (!kappa) return fail(IRK_EINVAL, "kappa is NULL");
  irk_problem* p = new irk_problem();
  p->N = N;
  p->g = make_geom(N);
  if (hipGetDevice(&p->dev) != hipSuccess) {
    delete p;
    return fail(IRK_EHIP, "hipGetDevice failed");
  }
  const long kc = (long)N * p->g.pitch;
  int rc = dev_alloc((void**)&p->kappa, kc * sizeof(double));
  if (rc == IRK_OK) rc = dev_alloc((void**)&p->bad, sizeof(int));
  if (rc == IRK_OK) rc = load_kappa(p, kappa, S(stream));
  if (rc != IRK_OK) {
    const std::string keep = g_err;
    irk_problem_destroy(p);
    g_err = keep;
    return rc;
  }
  *out = p;
  return IRK_OK;
}

int irk_problem_set_kappa(irk_problem* p, const double* kappa, void* stream) {
  g_err.clear();
  if (!p || !p->kappa) return fail(IRK_EINVAL, "NULL problem");
  if (!kappa) return fail(IRK_EINVAL, "kappa is NULL");
  return load_kappa(p, kappa, S(stream));
}

void irk_problem_destroy(irk_problem* p) {
  if (!p) return;
  dev_free(p->kappa);
  dev_free(p->bad);
  dev_free(p->stage);
  delete p;
}

int irk_apply_mass(const irk_problem* p, const double* x, double* y, void* stream) {
  g_err.clear();
  if (!p || !x || !y) return fail(IRK_EINVAL, "NULL argument");
  double* xp = nullptr;
  CHK(problem_stage(p, &xp));
  return apply_nodal(p, 0, x, y, xp, S(stream));
}

int irk_apply_stiffness(const irk_problem* p, const double* x, double* y, void* stream) {
  g_err.clear();
  if (!p || !x || !y) return fail(IRK_EINVAL, "NULL argument");
  double* xp = nullptr;
  CHK(problem_stage(p, &xp));
  return apply_nodal(p, 1, x, y, xp, S(stream));
}

int irk_apply_mass_noalloc(const irk_problem* p, const double* x, double* y, void* stream) {
  g_err.clear();
  if (!p || !x || !y) return fail(IRK_EINVAL, "NULL argument");
  if (2 * p->g.plane > kScratchDoubles)
    return fail(IRK_EINVAL, "irk_apply_mass_noalloc supports N <= " + std::to_string(kScratchMaxN) + " (N = " +
                                std::to_string(p->N) + "); use irk_apply_mass");
  double* xp = nullptr;
  CHK(scratch_of_device(p->dev, &xp));
  return apply_nodal(p, 0, x, y, xp, S(stream));
}

void irk_stepper_destroy(irk_stepper* st) {
  if (!st) return;
  for (size_t l = 0; l < st->lv.size(); ++l) {
    Level& L = st->lv[l];
    if (L.kapc && L.kapc != L.kap64) dev_free(L.kapc);
    if (L.own64) dev_free(L.kap64);
    dev_free(L.t);
    dev_free(L.x);
    dev_free(L.e);
    dev_free(L.tp);
  }
  for (void* p : st->binv) dev_free(p);
  for (size_t l = 0; l < st->ml.size(); ++l) {
    Level& L = st->ml[l];
    if (L.kapc && L.kapc != L.kap64) dev_free(L.kapc);
    if (L.own64) dev_free(L.kap64);
    dev_free(L.t);
    dev_free(L.x);
    dev_free(L.e);
  }
  dev_free(st->mcinv[0]);
  dev_free(st->mcinv[1]);
  dev_free(st->V);
  dev_free(st->Z);
  dev_free(st->f);
  dev_free(st->k);
  dev_free(st->tmp);
  dev_free(st->tmp2);
  dev_free(st->u);
  dev_free(st->Fp);
  dev_free(st->dres);
  dev_free(st->dflag);
  dev_free(st->rw.partial);
  dev_free(st->rw.counter);
  dev_free(st->adj_snaps);
  dev_free(st->adj_lam);
  dev_free(st->adj_grad);
  dev_free(st->adj_nu);
  dev_free(st->adj_kstep);
  for (auto& v : st->graphs)
    for (hipGraphExec_t g : v)
      if (g) (void)hipGraphExecDestroy(g);
  for (hipEvent_t e : st->timer_ev) (void)hipEventDestroy(e);
  if (st->cap) (void)hipStreamDestroy(st->cap);
  for (int i = 0; i < 2; ++i)
    if (st->step_ev[i]) (void)hipEventDestroy(st->step_ev[i]);
  if (st->norm_ev) (void)hipEventDestroy(st->norm_ev);
  if (st->hmir) {
    (void)hipDeviceSynchronize();
    (void)hipHostFree(st->hmir);
  }
  if (st->hres) (void)hipHostFree(st->hres);
  delete st;
}

int irk_stepper_create(irk_stepper** out, const irk_problem* p, const irk_tableau* tab, double dt,
                       const irk_options* opts, void* stream) {
  g_err.clear();
  if (!out) return fail(IRK_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p || !tab || !tab->A || !tab->b) return fail(IRK_EINVAL, "NULL problem or tableau");
  if (tab->s < 1 || tab->s > kMaxStages) return fail(IRK_EINVAL, "tableau must have 1..8 stages");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(IRK_EINVAL, "dt must be finite and positive");
  irk_options o;
  irk_options_default(&o);
  if (opts) o = *opts;
  if (o.precond < IRK_PC_JACOBI || o.precond > IRK_PC_MONOLITHIC) return fail(IRK_EINVAL, "unknown precond");
  if (o.precond == IRK_PC_MONOLITHIC && tab->s > kMMGMax)
    return fail(IRK_EINVAL, "the monolithic multigrid cycle supports up to 4 stages");
  if (o.restart < 1 || o.restart > 32) return fail(IRK_EINVAL, "restart must be in 1..32");
  if (o.max_it < 1) return fail(IRK_EINVAL, "max_it must be >= 1");
  if (!(o.rtol > 0) || !(o.rtol < 1)) return fail(IRK_EINVAL, "rtol must be in (0, 1)");
  if (o.cheb_degree < 1 || o.cheb_degree > kMaxDeg) return fail(IRK_EINVAL, "cheb_degree must be 1..3");
  if (!(o.cheb_lo > 0) || !(o.cheb_hi > o.cheb_lo)) return fail(IRK_EINVAL, "need 0 < cheb_lo < cheb_hi");
  if (o.power_its < 1 || o.power_its > 1000) return fail(IRK_EINVAL, "power_its must be 1..1000");
  if (o.mg_precision < IRK_F64 || o.mg_precision > IRK_BF16) return fail(IRK_EINVAL, "unknown mg_precision");
  if (o.orth != IRK_ORTH_CGS2 && o.orth != IRK_ORTH_CGS_SELECTIVE && o.orth != IRK_ORTH_DCGS2)
    return fail(IRK_EINVAL, "unknown orth");
  if (o.initial_guess != IRK_GUESS_ZERO && o.initial_guess != IRK_GUESS_PREV)
    return fail(IRK_EINVAL, "unknown initial_guess");
  if (o.mg_coarse_n < 1) return fail(IRK_EINVAL, "mg_coarse_n must be >= 1");
  if (o.splitting != IRK_SPLIT_AI && o.splitting != IRK_SPLIT_IA) return fail(IRK_EINVAL, "unknown splitting");
  if (o.stage_type != IRK_STAGE_COUPLED && o.stage_type != IRK_STAGE_DIRK) return fail(IRK_EINVAL, "unknown stage_type");
  if (o.lookahead < IRK_LOOKAHEAD_OFF || o.lookahead > IRK_LOOKAHEAD_ALWAYS) return fail(IRK_EINVAL, "unknown lookahead");
  if (o.basis_f64 != 0 && o.basis_f64 != 1) return fail(IRK_EINVAL, "basis_f64 must be 0 or 1");
  if (o.stage_type == IRK_STAGE_DIRK) {
    if (o.splitting != IRK_SPLIT_AI) return fail(IRK_EINVAL, "the DIRK stage type solves the AI form");
    for (int i = 0; i < tab->s; ++i)
      for (int j = i + 1; j < tab->s; ++j)
        if (tab->A[i * tab->s + j] != 0.0) return fail(IRK_EINVAL, "the DIRK stage type needs a lower-triangular A");
  }
  const int s = tab->s;
  for (int i = 0; i < s * s; ++i)
    if (!std::isfinite(tab->A[i])) return fail(IRK_EINVAL, "non-finite tableau entry");
  for (int i = 0; i < s; ++i) {
    if (!std::isfinite(tab->b[i])) return fail(IRK_EINVAL, "non-finite tableau entry");
    if (!(tab->A[i * s + i] > 0))
      return fail(IRK_EINVAL, "every diagonal entry a_ii must be > 0 (the diagonal blocks M + dt*a_ii*K must be SPD)");
  }
  if (p->N < 2) return fail(IRK_EINVAL, "bad problem");
  irk_stepper* st = new irk_stepper();
  st->prob = p;
  st->s = s;
  for (int i = 0; i < s * s; ++i) st->A[i] = tab->A[i];
  for (int i = 0; i < s; ++i) {
    st->b[i] = tab->b[i];
    st->c[i] = tab->c ? tab->c[i] : 0.0;
  }
  st->dt = dt;
  st->opt = o;
  {
    // Atil: D, L + D, U + D (additive split, eq:pcbjac / eq:pcbgs and its upper variant) or L1 D of
    // A = L1 D U1 (eq:pcranald); the transposed system is preconditioned by the transpose of the forward
    // preconditioner, I (x) M + dt Atil^T (x) K (IA: Atil^{-T} (x) M + dt I (x) K), with the same diagonal
    double L1[kMaxStages * kMaxStages] = {}, U1[kMaxStages * kMaxStages] = {}, D[kMaxStages] = {};
    if (o.precond == IRK_PC_RANA_LD) {
      double W[kMaxStages * kMaxStages];
      for (int i = 0; i < s * s; ++i) W[i] = tab->A[i];
      for (int k = 0; k < s; ++k) {
        D[k] = W[k * s + k];
        if (!(D[k] > 0)) {
          delete st;
          return fail(IRK_EINVAL, "Rana-LD needs A = L D U with positive pivots D");
        }
        L1[k * s + k] = U1[k * s + k] = 1.0;
        for (int i = k + 1; i < s; ++i) {
          L1[i * s + k] = W[i * s + k] / D[k];
          U1[k * s + i] = W[k * s + i] / D[k];
        }
        for (int i = k + 1; i < s; ++i)
          for (int j = k + 1; j < s; ++j) W[i * s + j] -= L1[i * s + k] * D[k] * U1[k * s + j];
      }
    }
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j) {
        double f = 0;
        if (o.precond == IRK_PC_JACOBI || o.precond == IRK_PC_MONOLITHIC)
          f = (i == j) ? tab->A[i * s + i] : 0.0;
        else if (o.precond == IRK_PC_GS_LOWER)
          f = (j <= i) ? tab->A[i * s + j] : 0.0;
        else if (o.precond == IRK_PC_GS_UPPER)
          f = (j >= i) ? tab->A[i * s + j] : 0.0;
        else
          f = (j <= i) ? L1[i * s + j] * D[j] : 0.0;
        st->Pt[0][i * s + j] = f;
      }
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j) st->Pt[1][i * s + j] = st->Pt[0][j * s + i];
    for (int i = 0; i < s; ++i) st->pd[i] = st->Pt[0][i * s + i];
  }
  st->ia = o.splitting == IRK_SPLIT_IA;
  st->dirk = o.stage_type == IRK_STAGE_DIRK;
  {
    double Ainv[kMaxStages * kMaxStages];
    if (st->ia && !host::small_inverse(tab->A, s, Ainv)) {
      delete st;
      return fail(IRK_EINVAL, "the IA splitting needs an invertible A");
    }
    for (int i = 0; i < s; ++i) {
      for (int j = 0; j < s; ++j) {
        st->Op[0][i * s + j] = st->ia ? Ainv[i * s + j] : tab->A[i * s + j];
        st->Op[1][i * s + j] = st->ia ? Ainv[j * s + i] : tab->A[j * s + i];
      }
      double bw = tab->b[i];
      if (st->ia) {
        bw = 0.0;
        for (int j = 0; j < s; ++j) bw += Ainv[j * s + i] * tab->b[j];
      }
      st->bw[i] = bw;
    }
    if (st->ia)
      for (int t = 0; t < 2; ++t)
        if (!host::small_inverse(st->Pt[t], s, st->Ci[t])) {
          delete st;
          return fail(IRK_EINVAL, "singular preconditioner matrix");
        }
  }
  st->prec = o.mg_precision;
  st->zf32 = st->prec != 0 && o.basis_f64 == 0;
  st->g = p->g;
  st->vlen = (long)s * p->g.plane;
  hipStream_t hs = S(stream);
  const int m = o.restart;
  const size_t vb = st->vlen * sizeof(double);
  int rc = IRK_OK;
  auto alloc_zero = [&](double** ptr, size_t bytes) {
    if (rc != IRK_OK) return;
    rc = dev_alloc((void**)ptr, bytes);
    if (rc == IRK_OK && hipMemsetAsync(*ptr, 0, bytes, hs) != hipSuccess) rc = fail(IRK_EHIP, "memset failed");
  };
  alloc_zero(&st->V, vb * (m + 1));
  alloc_zero(&st->Z, vb * m);
  alloc_zero(&st->f, vb);
  alloc_zero(&st->k, vb);
  // scratch planes; at least two, the power iteration keeps x and y in tmp
  const size_t tb = (size_t)std::max(s, 2) * p->g.plane * sizeof(double);
  alloc_zero(&st->tmp, tb);
  alloc_zero(&st->tmp2, tb);
  alloc_zero(&st->u, p->g.plane * sizeof(double));
  alloc_zero(&st->Fp, p->g.plane * sizeof(double));
  alloc_zero(&st->dres, DRES_LEN * sizeof(double));
  if (rc == IRK_OK) rc = dev_alloc((void**)&st->dflag, sizeof(int));
  st->rw.max_blocks = 1024;
  alloc_zero(&st->rw.partial, (size_t)st->rw.max_blocks * (kMaxRestart + 1) * sizeof(double));
  if (rc == IRK_OK) {
    rc = dev_alloc((void**)&st->rw.counter, 64);
    if (rc == IRK_OK && hipMemsetAsync(st->rw.counter, 0, 64, hs) != hipSuccess) rc = fail(IRK_EHIP, "memset");
  }
  if (rc == IRK_OK && hipHostMalloc((void**)&st->hres, DRES_LEN * sizeof(double)) != hipSuccess)
    rc = fail(IRK_ENOMEM, "hipHostMalloc failed");
  if (rc == IRK_OK && hipStreamCreateWithFlags(&st->cap, hipStreamNonBlocking) != hipSuccess)
    rc = fail(IRK_EHIP, "stream creation failed");
  if (rc == IRK_OK && (hipHostMalloc((void**)&st->hmir, 2 * kDcgs2Res * sizeof(double), hipHostMallocCoherent) !=
                            hipSuccess ||
                        hipHostGetDevicePointer((void**)&st->hmir_dev, st->hmir, 0) != hipSuccess))
    rc = fail(IRK_ENOMEM, "pinned coefficient mirror allocation failed");
  for (int i = 0; i < 2 && rc == IRK_OK; ++i)
    if (hipEventCreateWithFlags(&st->step_ev[i], hipEventDisableTiming) != hipSuccess)
      rc = fail(IRK_EHIP, "event creation failed");
  if (rc == IRK_OK && hipEventCreateWithFlags(&st->norm_ev, hipEventDisableTiming) != hipSuccess)
    rc = fail(IRK_EHIP, "event creation failed");
  if (rc == IRK_OK) rc = setup_multigrid(st, hs);
  if (rc == IRK_OK && o.precond == IRK_PC_MONOLITHIC) rc = setup_mmg(st, hs);
  if (rc == IRK_OK && hipStreamSynchronize(hs) != hipSuccess) rc = fail(IRK_EHIP, "setup synchronisation failed");
  if (rc != IRK_OK) {
    std::string keep = g_err;
    irk_stepper_destroy(st);
    g_err = keep;
    return rc;
  }
  *out = st;
  return IRK_OK;
}

int irk_stepper_refresh(irk_stepper* st, void* stream) {
  g_err.clear();
  CHK(validate_stepper(st));
  hipStream_t hs = S(stream);
  // nothing of the stepper may still run while its kappa-dependent state is rebuilt
  HIPCHK(hipStreamSynchronize(hs));
  // the captured Arnoldi graphs hold the old Chebyshev coefficients as kernel arguments: capture again
  for (auto& v : st->graphs) {
    for (hipGraphExec_t g : v)
      if (g) (void)hipGraphExecDestroy(g);
    v.clear();
  }
  st->have_prev = false;
  for (int& it : st->last_its) it = 0;
  int rc = setup_multigrid(st, hs);
  if (rc == IRK_OK && st->opt.precond == IRK_PC_MONOLITHIC) rc = setup_mmg(st, hs);
  if (rc == IRK_OK && hipStreamSynchronize(hs) != hipSuccess) rc = fail(IRK_EHIP, "refresh synchronisation failed");
  return rc;
}

int irk_stepper_sizes(const irk_stepper* st, int* N, int* s, int* levels) {
  CHK(validate_stepper(st));
  if (N) *N = st->prob->N;
  if (s) *s = st->s;
  if (levels) *levels = (int)st->lv.size();
  return IRK_OK;
}

int irk_stepper_mu(const irk_stepper* st, int stage, int level, double* mu) {
  CHK(validate_stepper(st));
  const int L = (int)st->lv.size();
  if (stage < 0 || stage >= st->s || level < 0 || level >= L || !mu) return fail(IRK_EINVAL, "bad stage/level");
  *mu = st->mu[(size_t)stage * L + level];
  return IRK_OK;
}

int irk_stepper_mmg_mu(const irk_stepper* st, int transpose, int level, double* mu, int* levels) {
  CHK(validate_stepper(st));
  if (st->opt.precond != IRK_PC_MONOLITHIC) return fail(IRK_EINVAL, "not a monolithic-multigrid stepper");
  const int L = (int)st->ml.size();
  if (levels) *levels = L;
  if (mu) {
    if (level < 0 || level >= L) return fail(IRK_EINVAL, "bad level");
    *mu = st->mmu[transpose ? 1 : 0][level];
  }
  return IRK_OK;
}

int irk_stage_rhs(const irk_stepper* cst, const double* u, const double* F, double* f, void* stream) {
  g_err.clear();
  CHK(validate_stepper(cst));
  if (!u || !f) return fail(IRK_EINVAL, "NULL argument");
  irk_stepper* st = const_cast<irk_stepper*>(cst);
  hipStream_t s = S(stream);
  launch_pack(u, st->u, st->g, 1, s);
  if (F) launch_pack(F, st->Fp, st->g, 1, s);
  launch_stage_rhs(st->u, F ? st->Fp : nullptr, st->f, st->prob->kappa, st->g, st->s, s);
  launch_unpack(st->f, f, st->g, st->s, s);
  return check_launch();
}

int irk_apply_stage_operator(const irk_stepper* cst, const double* x, double* y, int transpose, void* stream) {
  g_err.clear();
  CHK(validate_stepper(cst));
  if (!x || !y) return fail(IRK_EINVAL, "NULL argument");
  irk_stepper* st = const_cast<irk_stepper*>(cst);
  hipStream_t s = S(stream);
  launch_pack(x, st->tmp, st->g, st->s, s);
  CHK(apply_op(st, st->tmp, st->f, nullptr, transpose != 0, s));
  launch_unpack(st->f, y, st->g, st->s, s);
  return check_launch();
}

int irk_apply_preconditioner(const irk_stepper* cst, const double* v, double* z, int transpose, void* stream) {
  g_err.clear();
  CHK(validate_stepper(cst));
  if (!v || !z) return fail(IRK_EINVAL, "NULL argument");
  irk_stepper* st = const_cast<irk_stepper*>(cst);
  hipStream_t s = S(stream);
  launch_pack(v, st->f, st->g, st->s, s);
  CHK(precondition(st, st->f, nullptr, st->k, false, transpose != 0, s));
  launch_unpack(st->k, z, st->g, st->s, s);
  return check_launch();
}

int irk_vcycle(const irk_stepper* cst, int stage, const double* t, double* z, void* stream) {
  g_err.clear();
  CHK(validate_stepper(cst));
  if (!t || !z) return fail(IRK_EINVAL, "NULL argument");
  if (stage < 0 || stage >= cst->s) return fail(IRK_EINVAL, "stage out of range");
  irk_stepper* st = const_cast<irk_stepper*>(cst);
  hipStream_t s = S(stream);
  launch_pack(t, st->f, st->g, 1, s);
  CHK(vcycle(st, stage, st->f, nullptr, st->k, false, s));
  launch_unpack(st->k, z, st->g, 1, s);
  return check_launch();
}

int irk_solve_stages(irk_stepper* st, const double* f, double* k, int transpose, irk_stats* stats, void* stream) {
  g_err.clear();
  init_stats(stats);
  CHK(validate_stepper(st));
  if (!f || !k) return fail(IRK_EINVAL, "NULL argument");
  hipStream_t s = S(stream);
  launch_pack(f, st->f, st->g, st->s, s);
  CHK(check_launch());
  SolveInfo si;
  const int rc = stage_solve(st, st->f, transpose != 0, false, si, s);
  add_stats(stats, si);
  if (rc != IRK_OK) {
    if (stats) stats->failed_step = 0;
    return rc;
  }
  launch_unpack(st->k, k, st->g, st->s, s);
  HIPCHK(hipStreamSynchronize(s));
  return check_launch();
}

int irk_advance(irk_stepper* st, double* u, const double* F, int nsteps, irk_stats* stats, void* stream) {
  g_err.clear();
  init_stats(stats);
  CHK(validate_stepper(st));
  if (!u) return fail(IRK_EINVAL, "u is NULL");
  if (nsteps < 0) return fail(IRK_EINVAL, "nsteps must be >= 0");
  hipStream_t s = S(stream);
  launch_pack(u, st->u, st->g, 1, s);
  if (F) launch_pack(F, st->Fp, st->g, 1, s);
  CHK(check_launch());
  st->have_prev = false;
  for (int n = 0; n < nsteps; ++n) {
    SolveInfo si;
    const int rc = forward_step(st, F ? st->Fp : nullptr, si, s);
    add_stats(stats, si);
    if (rc != IRK_OK) {
      // the update only runs after a converged solve: st->u is the last good state
      if (stats) stats->failed_step = n;
      std::string keep = g_err;
      launch_unpack(st->u, u, st->g, 1, s);
      (void)hipStreamSynchronize(s);
      g_err = keep;
      return rc;
    }
    if (stats) stats->steps_done = n + 1;
  }
  launch_unpack(st->u, u, st->g, 1, s);
  HIPCHK(hipStreamSynchronize(s));
  return check_launch();
}

int irk_revolve_schedule(int nsteps, int nsnap, int* actions, int cap, int* count, int* advances) {
  g_err.clear();
  if (nsteps < 0 || nsnap < 1) return fail(IRK_EINVAL, "need nsteps >= 0 and nsnap >= 1");
  long adv = 0;
  std::vector<host::Action> sch = host::revolve_schedule(nsteps, std::min(nsnap, std::max(nsteps, 1)), adv);
  if (count) *count = (int)sch.size();
  if (advances) *advances = (int)adv;
  if (!actions) return IRK_OK;
  if ((int)sch.size() > cap) return fail(IRK_EINVAL, "action buffer too small");
  for (size_t i = 0; i < sch.size(); ++i) {
    actions[2 * i] = sch[i].kind;
    actions[2 * i + 1] = sch[i].arg;
  }
  return IRK_OK;
}

int irk_adjoint(irk_stepper* st, const double* u0, int nsteps, int nsnap, const double* lambda_T, double* lambda_0,
                double* grad_logkappa, irk_stats* stats, void* stream) {
  g_err.clear();
  init_stats(stats);
  CHK(validate_stepper(st));
  if (!u0 || !lambda_T) return fail(IRK_EINVAL, "NULL argument");
  if (nsteps < 0 || nsnap < 1) return fail(IRK_EINVAL, "need nsteps >= 0 and nsnap >= 1");
  hipStream_t s = S(stream);
  const Geom& g = st->g;
  const int slots = std::min(nsnap, std::max(nsteps, 1));
  const long gcount = (long)g.N * g.pitch;
  // the stepper's workspace: allocated by the first call, the checkpoint planes grown when more slots are needed
  int rc = IRK_OK;
  if (slots > st->adj_slots) {
    // every earlier call waited for its own work before returning, so the old planes are idle
    dev_free(st->adj_snaps);
    st->adj_snaps = nullptr;
    st->adj_slots = 0;
    CHK(dev_alloc((void**)&st->adj_snaps, (size_t)slots * g.plane * sizeof(double)));
    st->adj_slots = slots;
  }
  if (!st->adj_lam) CHK(dev_alloc((void**)&st->adj_lam, g.plane * sizeof(double)));
  if (!st->adj_grad) CHK(dev_alloc((void**)&st->adj_grad, gcount * sizeof(double)));
  if (!st->adj_nu) CHK(dev_alloc((void**)&st->adj_nu, st->vlen * sizeof(double)));
  if (!st->adj_kstep) CHK(dev_alloc((void**)&st->adj_kstep, st->vlen * sizeof(double)));
  double* snaps = st->adj_snaps;
  double* lam = st->adj_lam;
  double* grad = st->adj_grad;
  double* nu = st->adj_nu;
  double* kstep = st->adj_kstep;
  if (hipMemsetAsync(grad, 0, gcount * sizeof(double), s) != hipSuccess) rc = fail(IRK_EHIP, "memset");
  launch_pack(u0, st->u, g, 1, s);
  launch_pack(lambda_T, lam, g, 1, s);
  long adv = 0;
  std::vector<host::Action> sch = host::revolve_schedule(nsteps, slots, adv);
  const Coefs at = mix_of(st);
  const Coefs bb = b_of(st);
  st->have_prev = false;
  int done = 0;
  for (size_t q = 0; q < sch.size() && rc == IRK_OK; ++q) {
    const host::Action& act = sch[q];
    if (act.kind == 0) {
      for (int r = 0; r < act.arg && rc == IRK_OK; ++r) {
        SolveInfo si;
        rc = forward_step(st, nullptr, si, s);
        add_stats(stats, si);
      }
    } else if (act.kind == 1) {
      if (hipMemcpyAsync(snaps + (long)act.arg * g.plane, st->u, g.plane * sizeof(double), hipMemcpyDeviceToDevice,
                         s) != hipSuccess)
        rc = fail(IRK_EHIP, "snapshot copy failed");
    } else if (act.kind == 2) {
      if (hipMemcpyAsync(st->u, snaps + (long)act.arg * g.plane, g.plane * sizeof(double), hipMemcpyDeviceToDevice,
                         s) != hipSuccess)
        rc = fail(IRK_EHIP, "snapshot copy failed");
    } else {
      // reverse step act.arg from u_n = st->u: recompute its stages, then the adjoint step
      SolveInfo si;
      launch_stage_rhs(st->u, nullptr, st->f, st->prob->kappa, g, st->s, s);
      rc = stage_solve(st, st->f, false, false, si, s);
      add_stats(stats, si);
      if (rc != IRK_OK) break;
      if (hipMemcpyAsync(kstep, st->k, st->vlen * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) {
        rc = fail(IRK_EHIP, "copy failed");
        break;
      }
      launch_adjoint_rhs(lam, st->f, st->s, bb, st->dt, g, s);
      SolveInfo sa;
      rc = stage_solve(st, st->f, true, false, sa, s);
      add_stats(stats, sa);
      if (rc != IRK_OK) break;
      if (hipMemcpyAsync(nu, st->k, st->vlen * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) {
        rc = fail(IRK_EHIP, "copy failed");
        break;
      }
      launch_kappa_grad(grad, st->u, kstep, nu, st->prob->kappa, g, st->s, at, st->dt, s);
      launch_lambda_update(lam, nu, st->s, st->prob->kappa, g, s);
      rc = check_launch();
      ++done;
    }
  }
  if (rc == IRK_OK) {
    if (lambda_0) launch_unpack(lam, lambda_0, g, 1, s);
    if (grad_logkappa) launch_unpack_elem(grad, grad_logkappa, g, s);
    rc = check_launch();
    if (rc == IRK_OK && hipStreamSynchronize(s) != hipSuccess) rc = fail(IRK_EHIP, "synchronisation failed");
  } else {
    std::string keep = g_err;
    (void)hipStreamSynchronize(s);
    g_err = keep;
  }
  if (stats) {
    stats->forward_advances = (int)adv;
    stats->steps_done = done;
    if (rc != IRK_OK) stats->failed_step = nsteps - 1 - done;
  }
  return rc;
}

int irk_kernel_timer(irk_stepper* st, int family, int enable) {
  g_err.clear();
  CHK(validate_stepper(st));
  if (!(family >= 0 && family < IRK_KFAM_COUNT) && family != IRK_KFAM_ALL)
    return fail(IRK_EINVAL, "unknown kernel family " + std::to_string(family));
  st->timer_family = enable ? family : -1;
  st->timer_used = 0;
  for (int f = 0; f < IRK_KFAM_COUNT; ++f) {
    st->timer_bytes[f] = st->timer_bytes_min[f] = 0;
    st->timer_launches[f] = 0;
  }
  return IRK_OK;
}

int irk_kernel_timer_family(irk_stepper* st, int family, int* launches, double* total_ms, double* bytes,
                            double* bytes_min) {
  g_err.clear();
  CHK(validate_stepper(st));
  if (!(family >= 0 && family < IRK_KFAM_COUNT) && family != IRK_KFAM_ALL)
    return fail(IRK_EINVAL, "unknown kernel family " + std::to_string(family));
  double ms = 0, by = 0, bymin = 0;
  int n = 0;
  for (size_t q = 0; q + 1 < st->timer_used; q += 2) {
    if (family != IRK_KFAM_ALL && st->timer_tag[q / 2] != family) continue;
    HIPCHK(hipEventSynchronize(st->timer_ev[q + 1]));
    float f = 0;
    HIPCHK(hipEventElapsedTime(&f, st->timer_ev[q], st->timer_ev[q + 1]));
    ms += f;
  }
  for (int f = 0; f < IRK_KFAM_COUNT; ++f)
    if (family == IRK_KFAM_ALL || family == f) {
      by += st->timer_bytes[f];
      bymin += st->timer_bytes_min[f];
      n += st->timer_launches[f];
    }
  if (launches) *launches = n;
  if (total_ms) *total_ms = ms;
  if (bytes) *bytes = by;
  if (bytes_min) *bytes_min = bymin;
  return IRK_OK;
}

int irk_kernel_timer_read(irk_stepper* st, int* launches, double* total_ms, double* bytes) {
  return irk_kernel_timer_family(st, IRK_KFAM_ALL, launches, total_ms, bytes, nullptr);
}

int irk_device_copy(const double* x, double* y, long long n, void* stream) {
  g_err.clear();
  if (n < 0) return fail(IRK_EINVAL, "n must be >= 0");
  if (n == 0) return IRK_OK;
  if (!x || !y) return fail(IRK_EINVAL, "NULL argument");
  const uintptr_t xa = (uintptr_t)x, ya = (uintptr_t)y, nb = (uintptr_t)n * sizeof(double);
  if (xa < ya + nb && ya < xa + nb) return fail(IRK_EINVAL, "x and y overlap");
  launch_device_copy(x, y, (long)n, S(stream));
  return check_launch();
}

}  // extern "C"
