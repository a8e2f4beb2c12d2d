// Checks of the library's host-side routines (paper_2403_08084_amd/csrc/host_math.cpp) against properties that
// fix their results: inverses reproduce the identity, the Faddeev-LeVerrier polynomials give the adjugate and the
// determinant, the FGMRES least-squares update satisfies the normal equations, the Chebyshev coefficients
// reproduce the scaled Chebyshev polynomial, and the binomial checkpointing schedule reverses every step once with
// Griewank's minimal number of forward steps. Built and run under the address and undefined-behaviour sanitizers
// by tests/test_host_sanitize.py; exits non-zero on the first failed check.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "host_math.h"

using namespace irk::host;

static int g_fail = 0;
static void check(bool ok, const char* what, double v = 0) {
  if (!ok) {
    std::printf("FAIL %s (%g)\n", what, v);
    g_fail = 1;
  }
}

// deterministic pseudo-random numbers in [-1, 1) (a linear congruential generator; inputs only)
static unsigned long long g_state = 12345;
static double rnd() {
  g_state = g_state * 6364136223846793005ULL + 1442695040888963407ULL;
  return (double)(g_state >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static double identity_error(const std::vector<double>& A, const std::vector<double>& X, int n) {
  double worst = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double acc = 0;
      for (int k = 0; k < n; ++k) acc += A[(size_t)i * n + k] * X[(size_t)k * n + j];
      worst = std::fmax(worst, std::fabs(acc - (i == j ? 1.0 : 0.0)));
    }
  return worst;
}

static void check_q1_inverse() {
  for (int N : {2, 3, 8, 13}) {
    const int m = N - 1, n = m * m;
    std::vector<double> kap((size_t)N * N), K((size_t)n * n, 0.0), M((size_t)n * n, 0.0);
    for (auto& k : kap) k = std::exp(rnd());
    assemble_q1(kap.data(), N, N, K.data(), M.data());
    // symmetric, and the mass matrix of the whole interior reproduces the closed-form diagonal 4h^2/9
    const double h = 1.0 / N;
    for (int i = 0; i < n; ++i) {
      check(std::fabs(M[(size_t)i * n + i] - 4 * h * h / 9) < 1e-15, "mass diagonal");
      for (int j = 0; j < n; ++j)
        check(K[(size_t)i * n + j] == K[(size_t)j * n + i] && M[(size_t)i * n + j] == M[(size_t)j * n + i],
              "symmetric assembly");
    }
    const double alpha = 0.37;
    std::vector<double> B((size_t)n * n), B0, W, inv((size_t)n * n), inv2((size_t)n * n);
    for (size_t q = 0; q < B.size(); ++q) B[q] = M[q] + alpha * K[q];
    B0 = B;
    W = B;
    check(spd_band_inverse(B.data(), n, m + 1, inv.data()) == 0, "banded Cholesky succeeds");
    const double e = identity_error(B0, inv, n);
    check(e < 1e-9, "B * inv(B) = I", e);
    check(dense_inverse(W.data(), n, inv2.data()) == 0, "Gauss-Jordan succeeds");
    double d = 0, s = 0;
    for (size_t q = 0; q < inv.size(); ++q) {
      d = std::fmax(d, std::fabs(inv[q] - inv2[q]));
      s = std::fmax(s, std::fabs(inv2[q]));
    }
    check(d < 1e-12 * s, "banded Cholesky inverse = Gauss-Jordan inverse", d / s);
  }
  // an indefinite matrix is rejected
  std::vector<double> B = {1, 2, 2, 1}, inv(4);
  check(spd_band_inverse(B.data(), 2, 1, inv.data()) == -1, "indefinite matrix rejected");
}

static void check_dense_and_small() {
  const int n = 40;
  std::vector<double> W((size_t)n * n), W0, inv((size_t)n * n);
  std::vector<double> Zs((size_t)9, 0.0), Zinv(9);
  check(dense_inverse(Zs.data(), 3, Zinv.data()) == -1, "zero matrix rejected");
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) W[(size_t)i * n + j] = rnd() + (i == j ? 8.0 : 0.0);
  W0 = W;
  check(dense_inverse(W.data(), n, inv.data()) == 0, "general inverse succeeds");
  const double e = identity_error(W0, inv, n);
  check(e < 1e-12, "W * inv(W) = I", e);
  std::vector<double> S = {1, 2, 3, 2, 4, 6, 1, 1, 1}, Sinv(9);  // rank 2
  check(!small_inverse(S.data(), 3, Sinv.data()), "singular small matrix rejected");
  for (int s = 1; s <= 8; ++s) {
    std::vector<double> A((size_t)s * s), Ai((size_t)s * s);
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j) A[(size_t)i * s + j] = rnd() + (i == j ? 3.0 : 0.0);
    check(small_inverse(A.data(), s, Ai.data()), "small inverse succeeds");
    const double es = identity_error(A, Ai, s);
    check(es < 1e-13, "A * inv(A) = I (small)", es);
  }
}

static void check_faddeev_leverrier() {
  const int ld = 4;
  for (int s = 1; s <= 4; ++s) {
    double B[ld * ld] = {}, adj[ld * ld * ld], det[ld + 1];
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j) B[i * ld + j] = rnd();
    faddeev_leverrier(B, s, ld, adj, det);
    for (double tau : {0.0, 0.3, -1.7, 25.0}) {
      // C = I + tau B; P = adj(C) from the polynomial; C * P must equal det(C) I
      double C[ld * ld] = {}, P[ld * ld] = {}, dC = 0, tk = 1;
      for (int i = 0; i < s; ++i)
        for (int j = 0; j < s; ++j) C[i * ld + j] = (i == j ? 1.0 : 0.0) + tau * B[i * ld + j];
      for (int k = 0; k < s; ++k, tk *= tau)
        for (int i = 0; i < s; ++i)
          for (int j = 0; j < s; ++j) P[i * ld + j] += tk * adj[k * ld * ld + i * ld + j];
      tk = 1;
      for (int k = 0; k <= s; ++k, tk *= tau) dC += tk * det[k];
      double scale = 1;
      for (int i = 0; i < s * s; ++i) scale = std::fmax(scale, std::fabs(P[i]));
      for (int i = 0; i < s; ++i)
        for (int j = 0; j < s; ++j) {
          double acc = 0;
          for (int k = 0; k < s; ++k) acc += C[i * ld + k] * P[k * ld + j];
          const double want = (i == j) ? dC : 0.0;
          check(std::fabs(acc - want) < 1e-11 * scale * (1 + std::fabs(tau)), "C adj(C) = det(C) I",
                acc - want);
        }
      // determinant by cofactor expansion for s <= 3
      if (s <= 3) {
        double d;
        if (s == 1)
          d = C[0];
        else if (s == 2)
          d = C[0] * C[ld + 1] - C[1] * C[ld];
        else
          d = C[0] * (C[ld + 1] * C[2 * ld + 2] - C[ld + 2] * C[2 * ld + 1]) -
              C[1] * (C[ld] * C[2 * ld + 2] - C[ld + 2] * C[2 * ld]) +
              C[2] * (C[ld] * C[2 * ld + 1] - C[ld + 1] * C[2 * ld]);
        check(std::fabs(d - dC) < 1e-11 * (1 + std::fabs(d)), "det(I + tau B)", d - dC);
      }
    }
  }
}

static void check_hessenberg() {
  const int ld = 9;
  for (int ncol = 1; ncol <= 8; ++ncol) {
    std::vector<double> H((size_t)(ld + 1) * ld, 0.0), y(ncol);
    for (int i = 0; i <= ncol; ++i)
      for (int j = 0; j < ncol; ++j)
        if (i <= j + 1) H[(size_t)i * ld + j] = rnd() + (i == j ? 2.0 : 0.0);
    const double g0 = 1.5;
    const double est = hessenberg_ls(H.data(), ld, ncol, g0, y.data());
    // r = g0 e_1 - H y: |r| equals the estimate and H^T r = 0 (normal equations of the least-squares problem)
    std::vector<double> r(ncol + 1);
    double rn = 0;
    for (int i = 0; i <= ncol; ++i) {
      double acc = (i == 0) ? g0 : 0.0;
      for (int j = 0; j < ncol; ++j) acc -= H[(size_t)i * ld + j] * y[j];
      r[i] = acc;
      rn += acc * acc;
    }
    check(std::fabs(std::sqrt(rn) - est) < 1e-12, "least-squares residual estimate", std::sqrt(rn) - est);
    for (int j = 0; j < ncol; ++j) {
      double acc = 0;
      for (int i = 0; i <= ncol; ++i) acc += H[(size_t)i * ld + j] * r[i];
      check(std::fabs(acc) < 1e-12, "normal equations H^T r = 0", acc);
    }
  }
}

static void check_chebyshev() {
  const int cap = 3;
  for (int deg = 1; deg <= 3; ++deg) {
    const double lo = 0.25, hi = 1.1;
    double c0, beta[cap], gam[cap];
    chebyshev_coefficients(lo, hi, deg, cap, &c0, beta, gam);
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    for (double lam : {0.25, 0.4, 0.9, 1.1, 0.05}) {
      // error recurrence of the iteration for D^{-1}B = lam, from e_0 = 1
      double ep = 1.0, e = 1.0 - c0 * lam;
      for (int k = 1; k < deg; ++k) {
        const double en = e + beta[k] * (e - ep) - gam[k] * lam * e;
        ep = e;
        e = en;
      }
      // T_deg((theta - lam)/delta) / T_deg(sigma)
      const double x = (theta - lam) / delta;
      double t0 = 1, t1 = x, s0 = 1, s1 = sigma;
      for (int k = 1; k < deg; ++k) {
        const double t2 = 2 * x * t1 - t0, s2 = 2 * sigma * s1 - s0;
        t0 = t1;
        t1 = t2;
        s0 = s1;
        s1 = s2;
      }
      check(std::fabs(e - t1 / s1) < 1e-14, "Chebyshev error polynomial", e - t1 / s1);
    }
  }
}

static void check_revolve() {
  check(binom_sat(10, 8) == 45 && binom_sat(5, 0) == 1 && binom_sat(3, 5) == 0, "binomial coefficients");
  check(revolve_cost(40, 8) == 70, "F(40, 8) = 70", (double)revolve_cost(40, 8));
  check(revolve_cost(10, 1) == 45, "single slot cost", (double)revolve_cost(10, 1));
  for (int nsteps : {1, 2, 7, 40, 100}) {
    for (int nsnap : {1, 2, 3, 8}) {
      long adv = 0;
      const std::vector<Action> sch = revolve_schedule(nsteps, nsnap, adv);
      // simulate: slot contents (the step index of the stored state), current state index
      std::vector<int> slot(nsnap + 1, -1);
      int cur = 0, next_reverse = nsteps - 1;
      long fwd = 0;
      bool ok = true;
      for (const Action& a : sch) {
        if (a.kind == 0) {
          cur += a.arg;
          fwd += a.arg;
          ok = ok && a.arg > 0 && cur < nsteps;
        } else if (a.kind == 1) {
          ok = ok && a.arg >= 0 && a.arg < nsnap;
          if (ok) slot[a.arg] = cur;
        } else if (a.kind == 2) {
          ok = ok && a.arg >= 0 && a.arg < nsnap && slot[a.arg] >= 0;
          if (ok) cur = slot[a.arg];
        } else {
          ok = ok && a.arg == next_reverse && cur == a.arg;
          --next_reverse;
        }
      }
      check(ok && next_reverse == -1, "schedule reverses every step once, in order");
      check(fwd == adv, "advances counted");
      check(adv == revolve_cost(nsteps, nsnap), "schedule is optimal", (double)(adv - revolve_cost(nsteps, nsnap)));
    }
  }
}

int main() {
  check_q1_inverse();
  check_dense_and_small();
  check_faddeev_leverrier();
  check_hessenberg();
  check_chebyshev();
  check_revolve();
  if (!g_fail) std::printf("host_math checks passed\n");
  return g_fail;
}
