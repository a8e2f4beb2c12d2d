// Host-side numerical and scheduling routines (declarations and contracts in host_math.h).
#include "host_math.h"

#include <algorithm>
#include <cmath>
#include <cstddef>

namespace irk {
namespace host {

void assemble_q1(const double* kap, int ldk, int N, double* K, double* M) {
  // bilinear element matrices with local nodes (0,0), (1,0), (1,1), (0,1): K_e = kappa/6 Kr, M_e = h^2/36 Mr
  static const double Kr[4][4] = {{4, -1, -2, -1}, {-1, 4, -1, -2}, {-2, -1, 4, -1}, {-1, -2, -1, 4}};
  static const double Mr[4][4] = {{4, 2, 1, 2}, {2, 4, 2, 1}, {1, 2, 4, 2}, {2, 1, 2, 4}};
  static const int dx[4] = {0, 1, 1, 0}, dy[4] = {0, 0, 1, 1};
  const int m = N - 1;
  const size_t n = (size_t)m * m;
  const double h = 1.0 / N;
  for (int ey = 0; ey < N; ++ey)
    for (int ex = 0; ex < N; ++ex) {
      long idx[4];
      for (int a = 0; a < 4; ++a) {
        const int i = ex + dx[a], j = ey + dy[a];
        idx[a] = (i >= 1 && i <= m && j >= 1 && j <= m) ? (long)(j - 1) * m + (i - 1) : -1;
      }
      const double ke = kap[(size_t)ey * ldk + ex];
      for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 4; ++c)
          if (idx[a] >= 0 && idx[c] >= 0) {
            K[(size_t)idx[a] * n + idx[c]] += ke * Kr[a][c] / 6.0;
            M[(size_t)idx[a] * n + idx[c]] += h * h * Mr[a][c] / 36.0;
          }
    }
}

int spd_band_inverse(double* B, int n, int bw, double* inv) {
  // Cholesky B = L L^T within the band (fill stays inside it); L in the lower triangle of B
  for (int j = 0; j < n; ++j) {
    const int k0 = std::max(0, j - bw);
    double* Bj = B + (size_t)j * n;
    double d = Bj[j];
    for (int k = k0; k < j; ++k) d -= Bj[k] * Bj[k];
    if (!(d > 0)) return -1;
    d = std::sqrt(d);
    Bj[j] = d;
    const int i1 = std::min(n - 1, j + bw);
    for (int i = j + 1; i <= i1; ++i) {
      double* Bi = B + (size_t)i * n;
      double v = Bi[j];
      for (int k = std::max(k0, i - bw); k < j; ++k) v -= Bi[k] * Bj[k];
      Bi[j] = v / d;
    }
  }
  // U = L^T stored row-major over the band, so that both triangular solves stream rows
  std::vector<double> U((size_t)n * (bw + 1), 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = i; k <= std::min(n - 1, i + bw); ++k) U[(size_t)i * (bw + 1) + (k - i)] = B[(size_t)k * n + i];
  std::vector<double> y(n);
  for (int c = 0; c < n; ++c) {
    // L y = e_c: y vanishes above row c
    std::fill(y.begin(), y.begin() + c, 0.0);
    for (int i = c; i < n; ++i) {
      const double* Bi = B + (size_t)i * n;
      double v = (i == c) ? 1.0 : 0.0;
      for (int k = std::max(c, i - bw); k < i; ++k) v -= Bi[k] * y[k];
      y[i] = v / Bi[i];
    }
    // L^T x = y, overwriting y
    for (int i = n - 1; i >= 0; --i) {
      const double* Ui = U.data() + (size_t)i * (bw + 1);
      double v = y[i];
      const int k1 = std::min(n - 1, i + bw);
      for (int k = i + 1; k <= k1; ++k) v -= Ui[k - i] * y[k];
      y[i] = v / Ui[0];
    }
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + c] = y[i];
  }
  return 0;
}

int dense_inverse(double* W, int n, double* inv) {
  std::fill(inv, inv + (size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int k = 0; k < n; ++k) {
    int pr = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(W[(size_t)i * n + k]) > std::fabs(W[(size_t)pr * n + k])) pr = i;
    if (!(std::fabs(W[(size_t)pr * n + k]) > 0)) return -1;
    if (pr != k)
      for (int j = 0; j < n; ++j) {
        std::swap(W[(size_t)k * n + j], W[(size_t)pr * n + j]);
        std::swap(inv[(size_t)k * n + j], inv[(size_t)pr * n + j]);
      }
    const double d = 1.0 / W[(size_t)k * n + k];
    for (int j = 0; j < n; ++j) {
      W[(size_t)k * n + j] *= d;
      inv[(size_t)k * n + j] *= d;
    }
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const double f = W[(size_t)i * n + k];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        W[(size_t)i * n + j] -= f * W[(size_t)k * n + j];
        inv[(size_t)i * n + j] -= f * inv[(size_t)k * n + j];
      }
    }
  }
  return 0;
}

bool small_inverse(const double* A, int s, double* inv) {
  std::vector<double> W((size_t)s * 2 * s);
  double nrm = 0;
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) {
      W[(size_t)i * 2 * s + j] = A[i * s + j];
      W[(size_t)i * 2 * s + s + j] = (i == j) ? 1.0 : 0.0;
      nrm = std::max(nrm, std::fabs(A[i * s + j]));
    }
  for (int k = 0; k < s; ++k) {
    int pr = k;
    for (int i = k + 1; i < s; ++i)
      if (std::fabs(W[(size_t)i * 2 * s + k]) > std::fabs(W[(size_t)pr * 2 * s + k])) pr = i;
    if (!(std::fabs(W[(size_t)pr * 2 * s + k]) > 1e-13 * nrm)) return false;
    if (pr != k)
      for (int j = 0; j < 2 * s; ++j) std::swap(W[(size_t)k * 2 * s + j], W[(size_t)pr * 2 * s + j]);
    const double d = W[(size_t)k * 2 * s + k];
    for (int j = 0; j < 2 * s; ++j) W[(size_t)k * 2 * s + j] /= d;
    for (int i = 0; i < s; ++i) {
      if (i == k) continue;
      const double f = W[(size_t)i * 2 * s + k];
      if (f != 0.0)
        for (int j = 0; j < 2 * s; ++j) W[(size_t)i * 2 * s + j] -= f * W[(size_t)k * 2 * s + j];
    }
  }
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) inv[i * s + j] = W[(size_t)i * 2 * s + s + j];
  return true;
}

void chebyshev_coefficients(double lo, double hi, int deg, int cap, double* c0, double* beta, double* gam) {
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  *c0 = 1.0 / theta;
  for (int k = 0; k < cap; ++k) {
    beta[k] = 0.0;
    gam[k] = 0.0;
  }
  double rho = 1.0 / sigma;
  for (int k = 1; k < deg && k < cap; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    beta[k] = rn * rho;
    gam[k] = 2.0 * rn / delta;
    rho = rn;
  }
}

void faddeev_leverrier(const double* B, int s, int ld, double* adj, double* det) {
  // with N_0 = I, c_k = -tr(B N_{k-1}) / k and N_k = B N_{k-1} + c_k I: det(lambda I - B) = sum_k c_k lambda^{s-k}
  // and adj(lambda I - B) = sum_k N_k lambda^{s-1-k}; at lambda = -1/tau, scaled by (-tau)^s:
  // det(I + tau B) = sum_k c_k (-tau)^k, adj(I + tau B) = sum_k (-tau)^k N_k
  std::vector<double> N((size_t)ld * ld, 0.0), BN((size_t)ld * ld, 0.0);
  for (int i = 0; i < s; ++i) N[(size_t)i * ld + i] = 1.0;
  std::fill(adj, adj + (size_t)s * ld * ld, 0.0);
  std::fill(det, det + s + 1, 0.0);
  det[0] = 1.0;
  double sign = 1.0;
  for (int k = 0; k < s; ++k) {
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j) adj[(size_t)k * ld * ld + (size_t)i * ld + j] = sign * N[(size_t)i * ld + j];
    double tr = 0.0;
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j) {
        double acc = 0.0;
        for (int l = 0; l < s; ++l) acc += B[i * ld + l] * N[(size_t)l * ld + j];
        BN[(size_t)i * ld + j] = acc;
      }
    for (int i = 0; i < s; ++i) tr += BN[(size_t)i * ld + i];
    const double ck = -tr / (k + 1);
    sign = -sign;
    det[k + 1] = sign * ck;
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j) N[(size_t)i * ld + j] = BN[(size_t)i * ld + j] + (i == j ? ck : 0.0);
  }
}

double hessenberg_ls(const double* H, int ld, int ncol, double g0, double* y) {
  std::vector<double> R(H, H + (size_t)(ncol + 1) * ld), g(ncol + 1, 0.0);
  g[0] = g0;
  for (int j = 0; j < ncol; ++j) {
    const double a = R[(size_t)j * ld + j], b = R[(size_t)(j + 1) * ld + j];
    const double r = std::hypot(a, b);
    const double c = r > 0 ? a / r : 1.0, sn = r > 0 ? b / r : 0.0;
    for (int k = j; k < ncol; ++k) {
      const double t0 = c * R[(size_t)j * ld + k] + sn * R[(size_t)(j + 1) * ld + k];
      const double t1 = -sn * R[(size_t)j * ld + k] + c * R[(size_t)(j + 1) * ld + k];
      R[(size_t)j * ld + k] = t0;
      R[(size_t)(j + 1) * ld + k] = t1;
    }
    const double t0 = c * g[j] + sn * g[j + 1], t1 = -sn * g[j] + c * g[j + 1];
    g[j] = t0;
    g[j + 1] = t1;
  }
  if (y)
    for (int i = ncol - 1; i >= 0; --i) {
      double v = g[i];
      for (int k = i + 1; k < ncol; ++k) v -= R[(size_t)i * ld + k] * y[k];
      y[i] = v / R[(size_t)i * ld + i];
    }
  return std::fabs(g[ncol]);
}

long binom_sat(long n, long k) {
  if (k < 0 || k > n) return 0;
  k = std::min(k, n - k);
  double r = 1.0;
  for (long i = 1; i <= k; ++i) {
    r = r * (double)(n - k + i) / (double)i;
    if (r > 4e18) return (long)4e18;
  }
  return (long)std::llround(r);
}

long revolve_cost(long l, long c) {
  if (l <= 1) return 0;
  if (c <= 1) return l * (l - 1) / 2;
  long r = 0;
  while (binom_sat(c + r, c) < l) ++r;
  return r * l - binom_sat(c + r, c + 1);
}

namespace {

// reverse steps [a, a+l) with the state u_a in slot `slot`, `c` slots usable from `slot` on
void revolve_rec(int a, int l, int c, int slot, int& cur, std::vector<Action>& out, long& adv) {
  if (l <= 0) return;
  if (l == 1) {
    if (cur != a) out.push_back({2, slot});
    cur = a;
    out.push_back({3, a});
    return;
  }
  if (c == 1) {
    for (int stp = a + l - 1; stp >= a; --stp) {
      if (cur != a) out.push_back({2, slot});
      cur = a;
      if (stp > a) {
        out.push_back({0, stp - a});
        adv += stp - a;
        cur = stp;
      }
      out.push_back({3, stp});
    }
    return;
  }
  int best = 1;
  long bestc = -1;
  for (int k2 = 1; k2 < l; ++k2) {
    const long cost = k2 + revolve_cost(l - k2, c - 1) + revolve_cost(k2, c);
    if (bestc < 0 || cost < bestc) {
      bestc = cost;
      best = k2;
    }
  }
  if (cur != a) out.push_back({2, slot});
  out.push_back({0, best});
  adv += best;
  cur = a + best;
  out.push_back({1, slot + 1});
  revolve_rec(a + best, l - best, c - 1, slot + 1, cur, out, adv);
  revolve_rec(a, best, c, slot, cur, out, adv);
}

}  // namespace

std::vector<Action> revolve_schedule(int nsteps, int nsnap, long& adv) {
  std::vector<Action> out;
  adv = 0;
  int cur = 0;
  out.push_back({1, 0});
  revolve_rec(0, nsteps, nsnap, 0, cur, out, adv);
  return out;
}

}  // namespace host
}  // namespace irk
