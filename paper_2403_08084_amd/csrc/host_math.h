// Host-side numerical and scheduling routines of the stage solver: the dense coarsest-level inverses, small
// s x s inverses, Chebyshev smoothing coefficients, the closed form of the monolithic cycle's patch inverses, the
// FGMRES least-squares update and the binomial checkpointing schedule of the adjoint.
//
// Plain C++ (no GPU code): the library compiles this file with the rest, and a CPU test builds it on its own
// with the address and undefined-behaviour sanitizers.
#pragma once

#include <vector>

namespace irk {
namespace host {

// Q1 stiffness (unit diffusivity factor kap per element) and mass matrices on the (N-1)^2 interior nodes of the
// uniform N x N grid of the unit square, dense and row-major, node (i, j) at (j-1)(N-1) + (i-1). kap holds the
// N x N element diffusivities with row stride ldk (element (ex, ey) at ey*ldk + ex). K and M must hold n*n zeros.
void assemble_q1(const double* kap, int ldk, int N, double* K, double* M);

// Inverse of a symmetric positive definite n x n matrix B (row-major) whose nonzeros lie within bw of the
// diagonal, by a banded Cholesky factorisation (B is overwritten by the factor) and n banded triangular solves.
// Returns 0, or -1 if B is not positive definite.
int spd_band_inverse(double* B, int n, int bw, double* inv);

// Inverse of a general n x n row-major matrix W (overwritten) by Gauss-Jordan elimination with partial pivoting.
// Returns 0, or -1 if W is singular.
int dense_inverse(double* W, int n, double* inv);

// Inverse of a small s x s row-major matrix (Gauss-Jordan, partial pivoting); false if a pivot is negligible
// against the largest entry.
bool small_inverse(const double* A, int s, double* inv);

// Chebyshev iteration on [lo, hi] in the three-term form of Saad, Iterative Methods, Alg. 12.1:
// x_1 = x_0 + c0 r_0 (preconditioned), x_{k+1} = x_k + beta[k] (x_k - x_{k-1}) + gam[k] r_k for k = 1..deg-1.
// beta and gam have at least `cap` entries; entries from deg on (and entry 0) are set to zero.
void chebyshev_coefficients(double lo, double hi, int deg, int cap, double* c0, double* beta, double* gam);

// Faddeev-LeVerrier recursion for the s x s matrix B (row stride ld): adj(I + tau B) = sum_k tau^k adj_k and
// det(I + tau B) = sum_k tau^k det_k, k = 0..s. adj receives s matrices adj_0..adj_{s-1} of row stride ld, each
// ld*ld entries apart (adj_s = 0); det receives s + 1 values.
void faddeev_leverrier(const double* B, int s, int ld, double* adj, double* det);

// Least-squares update of FGMRES with the (ncol+1) x ncol Hessenberg matrix H (row stride ld): Givens QR from
// scratch; returns the residual estimate |g_ncol| and, if y is not null, the solution of R y = g (ncol entries).
double hessenberg_ls(const double* H, int ld, int ncol, double g0, double* y);

// Binomial checkpointing (Griewank & Walther, "revolve"): C(n, k) saturated at 4e18; the minimal number of
// forward steps to reverse l steps with c snapshot slots; and a schedule of actions
//   kind 0: advance arg steps, 1: store the current state in slot arg, 2: restore slot arg,
//   3: reverse step arg (recompute its stages from the current state and take its adjoint step)
// reversing nsteps steps with nsnap slots (slot 0 holds the initial state); adv receives the forward steps it
// takes.
long binom_sat(long n, long k);
long revolve_cost(long l, long c);
struct Action {
  int kind, arg;
};
std::vector<Action> revolve_schedule(int nsteps, int nsnap, long& adv);

}  // namespace host
}  // namespace irk
