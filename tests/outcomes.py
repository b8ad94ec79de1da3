"""Outcome comparison of the GPU path against the oracle (test helper).

One outcome per leaf is the inverse-CDF pick x = min{x : prefix(x) > u T}
in FP64 over the final state (Sec. 2.2 measurement from the final state;
Sec. 3.1 one outcome per leaf).  Both sides take the same uniform, so the
outcomes are equal unless the two prefix sums, which differ by rounding,
put the threshold on different sides of a boundary.  A GPU outcome that
differs from the oracle's is accepted only when it is what the oracle
itself would pick under a threshold moved by at most delta * T: every
oracle prefix from min(x_gpu, x_oracle) to max(x_gpu, x_oracle) - 1 lies
within delta * T of u T.  Any other outcome, however close in index, fails.
"""
import math

import numpy as np


def outcome_ok(psi, u, got, want, delta):
    """True when `got` is a valid pick for state `psi` and uniform `u` under
    a threshold moved by at most delta * T from the oracle's u * T."""
    got, want = int(got), int(want)
    if got == want:
        return True
    p = np.abs(np.asarray(psi)) ** 2
    if got < 0 or got >= p.size:
        return False
    tot = float(p.sum())
    pre = np.cumsum(p)
    lo, hi = min(got, want), max(got, want)
    return bool(np.all(np.abs(pre[lo:hi] - u * tot) <= delta * tot))


def check_outcomes(got, want, states, leaf_u, delta, cap=None):
    """Identical outcomes except at CDF-boundary leaves, which must pass
    `outcome_ok`; their count is returned and must not exceed `cap`
    (default: 2 plus 1% of the leaves)."""
    got = np.asarray(got, np.uint64)
    want = np.asarray(want, np.uint64)
    assert got.shape == want.shape, (got.shape, want.shape)
    bad = np.nonzero(got != want)[0]
    for i in bad:
        assert outcome_ok(states[i], float(leaf_u[i]), got[i], want[i], delta), \
            ("outcome is not a valid boundary pick", int(i), int(got[i]), int(want[i]))
    if cap is None:
        cap = 2 + math.ceil(0.01 * got.size)
    assert bad.size <= cap, ("too many boundary leaves", int(bad.size), cap)
    return bad.size


def rel_l2(amps, ref):
    """Largest per-leaf relative 2-norm error ||a - r||_2 / ||r||_2."""
    a = np.asarray(amps).reshape(len(ref), -1)
    r = np.asarray(ref).reshape(len(ref), -1)
    return float(np.max(np.linalg.norm(a - r, axis=1) / np.linalg.norm(r, axis=1)))
