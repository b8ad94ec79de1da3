"""CPU checks of the outcome comparison used by the GPU parity tests: on a
synthetic 20-qubit state (CDF steps near 2^-20, the same order as the
complex64 tolerance delta = 1e-6) it accepts only the two picks on either
side of a boundary the threshold lies next to, and rejects every other
outcome, a neighbour across a large step included."""
import numpy as np
import pytest

from outcomes import check_outcomes, outcome_ok

DELTA = 1e-6


@pytest.fixture(scope="module")
def state20():
    rng = np.random.default_rng(2024)
    psi = rng.normal(size=1 << 20) + 1j * rng.normal(size=1 << 20)
    psi /= np.linalg.norm(psi)
    return psi, np.cumsum(np.abs(psi) ** 2)


def _oracle_pick(pre, t):
    return int(np.searchsorted(pre, t, side="right"))


def test_adjacent_boundary_pick_accepted(state20):
    psi, pre = state20
    # a boundary x0 whose two neighbouring steps are both large (> 3 delta)
    p = np.diff(pre, prepend=0.0)
    x0 = next(x for x in range(400000, 500000) if p[x] > 3 * DELTA and p[x + 1] > 3 * DELTA)
    u = pre[x0] + 0.2 * DELTA  # threshold just above prefix(x0)
    want = _oracle_pick(pre, u)
    assert want == x0 + 1
    assert outcome_ok(psi, u, x0, want, DELTA)          # the rounding neighbour
    assert outcome_ok(psi, u, want, want, DELTA)


def test_non_adjacent_and_far_picks_rejected(state20):
    psi, pre = state20
    p = np.diff(pre, prepend=0.0)
    x0 = next(x for x in range(400000, 500000) if p[x] > 3 * DELTA and p[x + 1] > 3 * DELTA)
    u = pre[x0] + 0.2 * DELTA
    want = _oracle_pick(pre, u)
    # one past the oracle's pick: prefix(want) is a large step above u T
    assert not outcome_ok(psi, u, want + 1, want, DELTA)
    # two below: prefix(x0 - 1) is a large step below u T
    assert not outcome_ok(psi, u, x0 - 1, want, DELTA)
    # far away, although some prefix near u T exists (a check that only
    # asks whether the threshold is close to any boundary would pass these)
    assert not outcome_ok(psi, u, 0, want, DELTA)
    assert not outcome_ok(psi, u, (1 << 20) - 1, want, DELTA)
    # out of range
    assert not outcome_ok(psi, u, 1 << 20, want, DELTA)


def test_threshold_far_from_boundaries_allows_no_mismatch(state20):
    psi, pre = state20
    p = np.diff(pre, prepend=0.0)
    x = next(x for x in range(300000, 400000) if p[x] > 5 * DELTA)
    u = pre[x] - 0.5 * p[x]  # mid-step: 2 delta or more from either boundary
    want = _oracle_pick(pre, u)
    assert want == x
    assert not outcome_ok(psi, u, x - 1, want, DELTA)
    assert not outcome_ok(psi, u, x + 1, want, DELTA)


def test_check_outcomes_counts_and_caps(state20):
    psi, pre = state20
    p = np.diff(pre, prepend=0.0)
    x0 = next(x for x in range(400000, 500000) if p[x] > 3 * DELTA and p[x + 1] > 3 * DELTA)
    u = pre[x0] + 0.2 * DELTA
    want = _oracle_pick(pre, u)
    states = [psi] * 4
    us = [u] * 4
    # one valid boundary leaf among four: counted
    assert check_outcomes([x0, want, want, want], [want] * 4, states, us, DELTA) == 1
    # an invalid pick fails
    with pytest.raises(AssertionError):
        check_outcomes([want + 1, want, want, want], [want] * 4, states, us, DELTA)
    # more valid boundary leaves than the cap fails
    with pytest.raises(AssertionError):
        check_outcomes([x0] * 4, [want] * 4, states, us, DELTA, cap=2)
