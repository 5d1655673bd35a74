"""The binomial checkpointing schedule of the path adjoint (host logic, no GPU).

Pin: Griewank & Walther (ACM TOMS 26, 2000, Prop. 1) give the minimal number of forward
steps to reverse l steps with c checkpoints (the initial state among them) as
t(l, c) = r l - beta(c + 1, r - 1), beta(c, r) = (c + r)! / (c! r!), with r the repetition
number beta(c, r - 1) < l <= beta(c, r).  Our count adds the l re-runs of the step being
reversed (u_n is recovered by solving step n again), so it must equal t(l, c) + l with
c = slots + 1.  A simulation of the recursion checks that steps are reversed last to
first, each from the state right before it, with at most slots + 1 states held."""
from math import comb

import pytest

from paper_2604_22087_amd.adjoint import _revolve, revolve_cost


def _griewank(l, c):
    beta = lambda cc, rr: comb(cc + rr, cc)
    r = 0
    while beta(c, r) < l:
        r += 1
    return r * l - beta(c + 1, r - 1)


@pytest.mark.parametrize("slots", [0, 1, 2, 3, 5])
def test_cost_matches_closed_form(slots):
    for l in range(1, 41):
        assert revolve_cost(l, slots) == _griewank(l, slots + 1) + l, (l, slots)


def _simulate(l, slots):
    """Run the recursion on step indices only: `held` are the stored states (the initial
    one first), `work` the one state being advanced; every advance must start from one of
    them and every reversed step from the state right before it."""
    held, work = [0], [None]
    reversed_steps, solves, peak = [], [0], [1]

    def advance(first, last):
        assert first in held or work[0] == first
        solves[0] += last - first
        work[0] = last

    def rev(first, last, c):
        if last - first == 1:
            assert first in held or work[0] == first
            advance(first, last)
            reversed_steps.append(last)
            work[0] = None
            return
        if c == 0:
            for t in range(last, first, -1):
                advance(first, t - 1)
                rev(t - 1, t, 0)
            return
        k = _revolve(last - first, c)[1]
        assert 1 <= k < last - first
        advance(first, first + k)
        held.append(first + k)
        peak[0] = max(peak[0], len(held))
        rev(first + k, last, c - 1)
        held.pop()
        rev(first, first + k, c)

    rev(0, l, slots)
    return reversed_steps, solves[0], peak[0]


@pytest.mark.parametrize("l,slots", [(1, 0), (5, 0), (5, 1), (10, 2), (17, 3), (30, 4)])
def test_schedule_reverses_in_order_within_memory(l, slots):
    order, solves, peak = _simulate(l, slots)
    assert order == list(range(l, 0, -1))
    assert solves == revolve_cost(l, slots)
    assert peak <= slots + 1
