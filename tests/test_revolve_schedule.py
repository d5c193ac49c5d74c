"""Host logic of binomial checkpointing (no GPU): the schedule's closed-form
recompute count and its split against a brute-force minimisation of the
same recursion (reverse L substeps from a held state with c more slots:
recompute everything, or advance m, store, reverse L - m with c - 1 slots,
then m with c)."""
from functools import lru_cache

import pytest

from paper_1810_01054_amd import _lib


@lru_cache(None)
def brute(L, c):
    if L <= 1:
        return 0
    if c == 0:
        return L * (L - 1) // 2
    return min(m + brute(L - m, c - 1) + brute(m, c) for m in range(1, L))


def test_recompute_count_is_the_minimum_of_the_recursion():
    L_ = _lib.lib()
    for L in range(0, 140):
        for c in range(0, 7):
            assert L_.mpm_revolve_steps(L, c) == brute(L, c), (L, c)


def test_split_attains_the_minimum():
    L_ = _lib.lib()
    for L in range(2, 140):
        for c in range(1, 7):
            m = L_.mpm_revolve_split(L, c)
            assert 1 <= m < L
            assert m + brute(L - m, c - 1) + brute(m, c) == brute(L, c), (L, c, m)


def test_special_cases_and_arguments():
    L_ = _lib.lib()
    # one slot per substep: nothing is recomputed beyond the first advance
    for L in range(2, 30):
        assert L_.mpm_revolve_steps(L, L) == L - 1
    # no slot: the quadratic recompute from the held state
    assert L_.mpm_revolve_steps(100, 0) == 4950
    # large T stays cheap to schedule; with 16 slots 10^5 substeps recompute
    # t = 6 passes at most (C(17 + 6, 6) = 100,947 >= 10^5)
    assert 5 * 100000 < L_.mpm_revolve_steps(100000, 16) < 6 * 100000
    assert L_.mpm_revolve_steps(-1, 2) == -1
    assert L_.mpm_revolve_split(1, 2) == -1
    assert L_.mpm_revolve_split(5, 0) == -1
