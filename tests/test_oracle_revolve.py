"""Pins for oracle.revolve: dynamic programme vs Griewank's closed form."""
import pytest

from oracle import revolve


def test_dp_equals_closed_form():
    for l in range(1, 80):
        for c in range(1, 12):
            assert revolve.min_advances_dp(l, c) == revolve.min_advances_closed_form(l, c), (l, c)


def test_known_values():
    assert revolve.min_advances_dp(40, 8) == 70  # 40 steps, 8 slots including u_0
    for l in range(1, 30):
        assert revolve.min_advances_dp(l, l) == l - 1  # store-all
        assert revolve.min_advances_dp(l, 1) == l * (l - 1) // 2  # recompute everything from u_0


def test_needs_a_slot():
    with pytest.raises(ValueError):
        revolve.min_advances_dp(5, 0)
