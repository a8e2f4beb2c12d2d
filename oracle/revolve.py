"""Optimal binomial checkpointing cost (CPU).

Test infrastructure only (see the package docstring).

The paper does not treat adjoints or checkpointing. The reverse sweep of the
adjoint needs u_n at every step n in reverse order; with c snapshot slots (one
of them holding u_0) the states are recomputed from snapshots. The cost model is
that of Griewank & Walther's binomial checkpointing ("revolve", ACM TOMS 26,
2000): reversing one step (recomputing its stages from u_n and solving its
adjoint) counts as the reversal itself, and every other forward step counts
one advance.

  * dynamic programming (the definition): F(1, c) = 0, F(l, 1) = l(l-1)/2,
    F(l, c) = min_{1<=k<l} [ k + F(l-k, c-1) + F(k, c) ]
    (advance k steps, store the state, reverse the tail with one slot fewer,
    then reverse the head).
  * closed form (Griewank 1992): with beta(c, r) = C(c+r, c) and r the least
    integer with beta(c, r) >= l, F(l, c) = r*l - beta(c+1, r-1).
"""
from __future__ import annotations

from functools import lru_cache
from math import comb


def min_advances_dp(l: int, c: int) -> int:
    """Minimal number of forward advances to reverse l steps with c slots (DP)."""
    if c < 1:
        raise ValueError("need at least one snapshot slot")

    @lru_cache(maxsize=None)
    def F(ll: int, cc: int) -> int:
        if ll <= 1:
            return 0
        if cc == 1:
            return ll * (ll - 1) // 2
        return min(k + F(ll - k, cc - 1) + F(k, cc) for k in range(1, ll))

    return F(l, c)


def min_advances_closed_form(l: int, c: int) -> int:
    """Griewank's closed form r*l - beta(c+1, r-1) for the same cost."""
    if l <= 1:
        return 0
    r = 0
    while comb(c + r, c) < l:
        r += 1
    return r * l - comb(c + 1 + r - 1, c + 1)
