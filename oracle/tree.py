"""Tree arithmetic, Dynamic Circuit Partition and fidelity metrics.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Written from the paper's equations, in the paper's order:
* Sec. 3.1 (tree organisation): instances of subcircuit l = prod_{j<=l} A_j
  (0-based levels; the printed product bound is read for 1-based subcircuits),
  outcomes = prod A_j.
* Sec. 3.2 (Dynamic Circuit Partition): the error-rate product, the
  sample-size bound for A_0, the equal remaining arity A_r and its adjustment.
* Sec. 3.6: the maximum speedup of k equal subcircuits, kN / ((k-1) + N).
* Sec. 4.1: state fidelity F_s and normalised fidelity F.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


# ------------------------------------------------------------ tree shape --

def instances(arity):
    """Number of simulated instances of each subcircuit (Sec. 3.1)."""
    out, p = [], 1
    for a in arity:
        p *= int(a)
        out.append(p)
    return out


def outcomes(arity) -> int:
    return int(np.prod([int(a) for a in arity], dtype=object))


def node_count(arity, include_root: bool = True) -> int:
    """Nodes of the simulation tree; the paper's figures count the initial
    state as one extra node."""
    return sum(instances(arity)) + (1 if include_root else 0)


def ancestor(arity, level: int, leaf: int) -> int:
    """Index (within its level) of a leaf's ancestor at ``level``."""
    below = 1
    for a in arity[level + 1:]:
        below *= int(a)
    return leaf // below


def work_ratio_equal(arity) -> float:
    """Subcircuit runs of per-shot simulation over those of the tree, for
    equal-length subcircuits: k * N / sum_l I_l."""
    k = len(arity)
    return k * outcomes(arity) / sum(instances(arity))


def max_speedup_equal(k: int, N: int) -> float:
    """Sec. 3.6: the largest speedup of k equal-length subcircuits."""
    return k * N / ((k - 1) + N)


# ------------------------------------------------------------------- DCP --

def first_error_rate(error_rates) -> float:
    """Sec. 3.2.3: error rate of the first subcircuit, 1 - prod (1 - e_i)."""
    prod = 1.0
    for e in error_rates:
        prod *= (1.0 - float(e))
    return 1.0 - prod


def sample_size(p_hat: float, z: float, eps: float, N=None) -> float:
    """Sec. 3.2.3: the minimum A_0; with N=None the finite-population
    correction is dropped (N -> infinity)."""
    n0 = z * z * p_hat * (1.0 - p_hat) / (eps * eps)
    if N is None:
        return n0
    return n0 / (1.0 + n0 / N)


def int_root_floor(x: Fraction, k: int) -> int:
    """floor(x^(1/k)) for a positive rational x, exactly."""
    a = int(math.floor(float(x) ** (1.0 / k))) + 2
    while a > 0 and Fraction(a) ** k > x:
        a -= 1
    return a


def dcp(error_rates, N: int, z: float = 1.96, eps: float = 0.01,
        copy_cost: float = 1.0, max_levels=None, A0_min=None):
    """Dynamic Circuit Partition (Sec. 3.2).

    1. The first subcircuit is the shortest that amortises a state copy:
       L0 = max(1, ceil(copy_cost)) gates.
    2. Its error rate p_hat = 1 - prod (1 - e_i).
    3. A0_min = ceil(sample-size bound) (or the given ``A0_min``).
    4. k = the most remaining subcircuits with A_r = floor((N/A0_min)^(1/k))
       >= 2, capped by the gate budget floor((G - L0) / max(1, copy_cost)) and
       by ``max_levels - 1``; A_0 is then raised to ceil(N / A_r^k) so the
       tree has at least N outcomes; the remaining gates are split into k
       equal parts (larger parts first).
    Returns (arity, cut); a tree of one level is the per-shot form.
    """
    G = len(error_rates)
    N = int(N)
    if G == 0 or N < 1:
        raise ValueError("empty circuit or no shots")
    L0 = max(1, int(math.ceil(copy_cost)))
    if L0 >= G:
        return [N], [0, G]
    if A0_min is None:
        p_hat = first_error_rate(error_rates[:L0])
        A0_min = int(math.ceil(sample_size(p_hat, z, eps, N)))
    A0_min = min(max(int(A0_min), 1), N)
    ratio = Fraction(N, A0_min)
    k_shots = 0
    while int_root_floor(ratio, k_shots + 1) >= 2:
        k_shots += 1
    k_gates = int(math.floor((G - L0) / max(1.0, float(copy_cost))))
    k = min(k_shots, k_gates)
    if max_levels is not None:
        k = min(k, int(max_levels) - 1)
    if k < 1:
        return [N], [0, G]
    Ar = int_root_floor(ratio, k)
    A0 = -(-N // Ar ** k)
    rest = G - L0
    sizes = [rest // k + (1 if i < rest % k else 0) for i in range(k)]
    cut = [0, L0]
    for s in sizes:
        cut.append(cut[-1] + s)
    return [A0] + [Ar] * k, cut


def equal_cuts(G: int, levels: int):
    """Equal gate counts per subcircuit (larger parts first)."""
    sizes = [G // levels + (1 if i < G % levels else 0) for i in range(levels)]
    cut = [0]
    for s in sizes:
        cut.append(cut[-1] + s)
    return cut


# -------------------------------------------------------------- fidelity --

def hist_probs(outcomes_arr, n: int) -> np.ndarray:
    """Empirical distribution over 2^n outcomes."""
    cnt = np.bincount(np.asarray(outcomes_arr, np.int64), minlength=1 << n)
    return cnt / max(1, cnt.sum())


def fidelity_s(p_ideal, p_out) -> float:
    """Sec. 4.1: F_s = (sum_x sqrt(P_ideal(x) P_out(x)))^2."""
    return float(np.sum(np.sqrt(np.asarray(p_ideal) * np.asarray(p_out))) ** 2)


def fidelity_norm(p_ideal, p_out) -> float:
    """Sec. 4.1: normalised fidelity, (F_s(P, Q) - F_s(P, U)) / (1 - F_s(P, U))
    with U uniform; undefined (nan) when P itself is uniform."""
    p_ideal = np.asarray(p_ideal, np.float64)
    uni = np.full_like(p_ideal, 1.0 / p_ideal.size)
    fu = fidelity_s(p_ideal, uni)
    if abs(1.0 - fu) < 1e-15:
        return float("nan")
    return (fidelity_s(p_ideal, p_out) - fu) / (1.0 - fu)


def tv_distance(p, q) -> float:
    return 0.5 * float(np.sum(np.abs(np.asarray(p) - np.asarray(q))))
