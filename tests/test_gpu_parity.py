"""GPU parity: the HIP path against the CPU oracle, element by element.

Both sides read the same seeded circuit; each side draws the noise
insertion list with its own implementation of the same counter-based
generator (bit-identity of the two lists is a host test), or both read an
explicit list written by the test.  Amplitudes agree to 1e-5 (complex64)
and 1e-12 (complex128) max-abs; outcomes are identical except at leaves
where the GPU's pick is the oracle's own pick under a threshold moved by at
most delta * T (delta 1e-6 for complex64, 1e-12 for complex128): every
oracle prefix between the two outcomes lies within delta * T of u * T.
Such boundary leaves are counted and capped (tests/outcomes.py).
"""
import math
import os

import numpy as np
import pytest

import oracle
from outcomes import check_outcomes, rel_l2
from paper_2203_13892_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "c128": 1e-12}
DELTA = {"c64": 1e-6, "c128": 1e-12}
U = {"c64": 2.0 ** -24, "c128": 2.0 ** -53}


def rel_bound(prec, gates):
    """Relative 2-norm bound on a trajectory after `gates` unitary steps:
    rounding errors of unit roundoff u add up like a random walk, about
    u sqrt(G) in the 2-norm (measured: 0.45-1.25 u sqrt(G) at 20-26 qubits
    in both precisions); three times that is the bound."""
    return 3.0 * U[prec] * math.sqrt(gates)


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2203_13892_amd import tqsim
    return tqsim


def run_both(T, wc, tree, seed, prec, leaves, tuning=None, noise_arrays=None):
    c = T.Circuit.from_workload(wc)
    if noise_arrays is None:
        nz = T.Noise.sample(c, tree, seed)
        onz = oracle.sample_noise(wc.gates, tree, seed)
    else:
        nz = T.Noise.from_arrays(c, tree, *noise_arrays)
        onz = oracle.Noise(*[np.asarray(a) for a in noise_arrays])
    plan = T.Plan(c, tree, prec, tuning)
    out, amps = T.run_capture(plan, nz, leaves)
    oout, ost = oracle.run_leaves(wc.n, wc.gates, tree, onz, leaves, states=True)
    return out, amps, oout, ost, onz


def event_arrays(wc, tree, rng, rate=0.3):
    """An explicit insertion list with events on a fraction of gate slots."""
    A, cut = tree
    node_off, eg, ec = [0], [], []
    for l in range(len(A)):
        I = int(np.prod(A[:l + 1]))
        for _ in range(I):
            for g in range(cut[l], cut[l + 1]):
                if rng.random() < rate:
                    eg.append(g)
                    ec.append(int(rng.integers(1, 4 ** len(wc.gates[g][0]))))
            node_off.append(len(eg))
    leaves = int(np.prod(A))
    return (np.array(node_off, np.uint64), np.array(eg, np.uint32), np.array(ec, np.uint8),
            rng.random(leaves))


# Hadamard and its sign variants: every entry +-1/sqrt(2) (the specialised
# kernels' sign-only butterflies)
_BUTTERFLIES = [np.array(m, complex) / math.sqrt(2.0) for m in
                ([[1, 1], [1, -1]], [[1, -1], [1, 1]], [[-1, 1], [1, 1]], [[1, 1], [-1, 1]])]


def mixed_gates(n, count, rng):
    """Every op class: dense 1q, Hadamard-like 1q, diagonal 1q/2q,
    controlled, dense 2q, swap, on low / high / mixed qubit positions."""
    c = W.Circuit(n)
    for i in range(count):
        kind = i % 8
        if kind == 7:
            c.add((int(rng.integers(n)),), _BUTTERFLIES[int(rng.integers(4))])
        elif kind == 0:
            c.add((int(rng.integers(n)),), W.haar_unitary(2, rng))
        elif kind == 1:
            c.add((int(rng.integers(n)),), W.phase(float(rng.uniform(0, 6))))
        else:
            a, b = [int(x) for x in rng.choice(n, 2, replace=False)]
            if kind == 2:
                c.add((a, b), W.cphase(float(rng.uniform(0, 6))))
            elif kind == 3:
                c.add((a, b), W.cx())
            elif kind == 4:
                c.add((a, b), W.haar_unitary(4, rng))
            elif kind == 5:
                c.add((a, b), W.swap())
            else:
                c.add((a, b), W.rzz(float(rng.uniform(0, 6))))
    return c


@pytest.mark.parametrize("jit", [1, 2])
@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("n", [1, 2, 5, 9, 14])
def test_every_op_class_with_forced_noise(T, prec, n, jit):
    rng = np.random.default_rng(100 + n)
    wc = mixed_gates(n, 60, rng) if n > 1 else W.Circuit(1, [((0,), W.haar_unitary(2, rng), None)] * 3)
    if n == 1:
        wc.add((0,), W.phase(0.3))
    tree = ([6], [0, len(wc)])
    arr = event_arrays(wc, tree, rng)
    out, amps, oout, ost, _ = run_both(T, wc, tree, 0, prec, np.arange(6), noise_arrays=arr,
                                       tuning={"jit": jit})
    assert np.max(np.abs(amps - ost)) < TOL[prec]
    check_outcomes(out, oout, ost, arr[3], DELTA[prec])


def longest_phase_run(plan):
    """Gates of the plan's longest run of diagonal gates whose noise events
    act inside the run (all but its last gate), from the plan's text form:
    'pass p' lines, 'diag slot0 slot1' ops, 'gate g pass slot-after' lines."""
    runs, where, p = [], {}, -1
    for line in plan.describe().splitlines():
        f = line.split()
        if f[0] == "pass":
            p = int(f[1])
        elif f[0] == "diag":
            runs.append((int(f[2]) - int(f[1]), p, int(f[1]), int(f[2])))
        elif f[0] == "gate":
            where[int(f[1])] = (int(f[2]), int(f[3]))
    _, p, s0, s1 = max(runs)
    return sorted(g for g, (gp, gs) in where.items() if gp == p and s0 < gs < s1)


@pytest.mark.parametrize("jit", [1, 2])
@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_phase_run_with_up_to_five_events_inside(T, prec, jit):
    # one long run of diagonal gates on lane, register and fixed qubits;
    # leaf i carries counts[i] events inside it, so the run is applied
    # whole, in two to four frames, and gate by gate
    rng = np.random.default_rng(11)
    n = 13
    wc = W.Circuit(n)
    for q in range(n):
        wc.add((q,), W.haar_unitary(2, rng))
    for i in range(48):
        if i % 4 == 3:
            wc.add((int(rng.integers(n)),), W.phase(float(rng.uniform(0, 6))))
        else:
            a, b = [int(x) for x in rng.choice(n, 2, replace=False)]
            wc.add((a, b), W.cphase(float(rng.uniform(0, 6))) if i % 4 < 2 else W.rzz(float(rng.uniform(0, 6))))
    for q in range(n):
        wc.add((q,), W.haar_unitary(2, rng))
    tree = ([8], [0, len(wc)])
    run = longest_phase_run(T.Plan(T.Circuit.from_workload(wc), tree, prec))
    assert len(run) >= 30
    assert all(np.allclose(np.diag(np.diag(wc.gates[g][1])), wc.gates[g][1]) for g in run)
    counts = [0, 1, 2, 3, 4, 5, 1, 3]
    node_off, eg, ec = [0], [], []
    for k in counts:
        for g in sorted(rng.choice(run, k, replace=False)):
            eg.append(int(g))
            ec.append(int(rng.integers(1, 4 ** len(wc.gates[g][0]))))
        node_off.append(len(eg))
    arr = (np.array(node_off, np.uint64), np.array(eg, np.uint32), np.array(ec, np.uint8), rng.random(8))
    out, amps, oout, ost, _ = run_both(T, wc, tree, 0, prec, np.arange(8), noise_arrays=arr,
                                       tuning={"jit": jit})
    assert np.max(np.abs(amps - ost)) < TOL[prec]
    check_outcomes(out, oout, ost, arr[3], DELTA[prec])


@pytest.mark.parametrize("jit", [1, 2])
@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_tree_levels_ragged_chunks(T, prec, jit):
    rng = np.random.default_rng(7)
    n = 13
    wc = mixed_gates(n, 45, rng)
    tree = ([3, 4, 5], [0, 10, 27, 45])
    arr = event_arrays(wc, tree, rng, rate=0.15)
    leaves = np.arange(60)
    out, amps, oout, ost, _ = run_both(T, wc, tree, 0, prec, leaves,
                                       tuning={"chunk_states": 7, "max_ops_per_pass": 5, "jit": jit},
                                       noise_arrays=arr)
    assert np.max(np.abs(amps - ost)) < TOL[prec]
    check_outcomes(out, oout, ost, arr[3], DELTA[prec])


def test_c1_qft10_per_shot_c128_all_leaves(T):
    # 10-qubit QFT, depolarizing 1e-3 / 1e-2, 1000 shots, per-shot, seed 0
    wc = W.qft(10).with_depolarizing(1e-3, 1e-2)
    tree = ([1000], [0, len(wc)])
    leaves = np.arange(1000)
    out, amps, oout, ost, onz = run_both(T, wc, tree, 0, "c128", leaves)
    assert np.max(np.abs(amps - ost)) < 1e-12
    assert rel_l2(amps, ost) < rel_bound("c128", len(wc))
    nb = check_outcomes(out, oout, ost, onz.leaf_u, DELTA["c128"])
    assert nb <= 2


def test_c1_qft10_per_shot_c64(T):
    wc = W.qft(10).with_depolarizing(1e-3, 1e-2)
    tree = ([1000], [0, len(wc)])
    leaves = np.arange(0, 1000, 7)
    out, amps, oout, ost, onz = run_both(T, wc, tree, 0, "c64", leaves)
    assert np.max(np.abs(amps - ost)) < 1e-5
    check_outcomes(out[leaves], oout, ost, onz.leaf_u[leaves], DELTA["c64"])


def test_outcomes_all_leaves_c64_small(T):
    # every leaf's outcome at complex64 against the oracle (boundary leaves counted)
    wc = W.concat(W.ghz(8), W.random_circuit(8, 30, seed=3)).with_depolarizing(0.01, 0.05)
    tree = ([8, 4, 4], [0, 12, 25, len(wc)])
    c = T.Circuit.from_workload(wc)
    nz = T.Noise.sample(c, tree, 11)
    out = T.run(T.Plan(c, tree, "c64"), nz)
    onz = oracle.sample_noise(wc.gates, tree, 11)
    oout, ost = oracle.run_leaves(8, wc.gates, tree, onz, states=True)
    nb = check_outcomes(out, oout, ost, onz.leaf_u, DELTA["c64"])
    assert nb <= 3


@pytest.mark.parametrize("n,blog", [(7, 8), (9, 8), (13, 12), (14, 8), (16, 12)])
def test_sampling_under_permuted_positions(T, n, blog):
    # swap gates only relabel positions, so the final state sits in memory
    # with logical qubits at permuted bit positions (a reversal, then seeded
    # random swaps); sampling and read-out still run in logical order
    rng = np.random.default_rng(31 * n + blog)
    wc = W.Circuit(n)
    for q in range(n):
        wc.add((q,), W.haar_unitary(2, rng))
    for q in range(n - 1):
        wc.add((q, q + 1), W.haar_unitary(4, rng))
    for i in range(n // 2):
        wc.add((i, n - 1 - i), W.swap())
    for _ in range(2 * n):
        a, b = [int(x) for x in rng.choice(n, 2, replace=False)]
        wc.add((a, b), W.swap())
    wc.add((0,), W.haar_unitary(2, rng))
    wc = wc.with_depolarizing(1e-2, 5e-2)
    tree = ([24], [0, len(wc)])
    out, amps, oout, ost, onz = run_both(T, wc, tree, 3, "c64", np.arange(24),
                                         tuning={"sample_block_log": blog})
    assert np.max(np.abs(amps - ost)) < TOL["c64"]
    check_outcomes(out, oout, ost, onz.leaf_u, DELTA["c64"])


def _c2_case(family):
    if family == "qft":
        wc = W.qft(20).with_depolarizing(1e-3, 1e-2)
    else:
        wc = W.brickwall(20, 20, seed=1).with_depolarizing(1e-3, 1e-2)
    G = len(wc)
    return wc, ([16, 32, 32], [0, G // 3, 2 * G // 3, G])


# 20 qubits, 16384 leaves of the (16, 32, 32) tree at complex64 (the
# headline workload and its brick-wall partner).  The oracle recomputes
# every leaf of level-0 subtree 0 (its 1024 leaves: 32 sibling groups whose
# ancestors are shared, spanning state chunks) in four parts, then 64 random
# leaves of the other subtrees.  Each leaf's amplitudes agree to 1e-5
# max-abs and to 3 u sqrt(G) in relative 2-norm (2.7e-6 for the 220-gate
# QFT, 2.5e-6 for the 190-gate brick-wall); outcomes are identical except
# at valid boundary picks, at most 2 + 1% of the leaves.
C2_PARTS = [("sub0", k) for k in range(4)] + [("random", 0)]


@pytest.mark.parametrize("part", C2_PARTS, ids=lambda p: "%s%d" % p)
@pytest.mark.parametrize("family", ["qft", "bw"])
def test_c2_20q_tree_leaves(T, family, part):
    wc, tree = _c2_case(family)
    kind, k = part
    if kind == "sub0":
        leaves = np.arange(256 * k, 256 * (k + 1))
    else:
        leaves = np.sort(np.random.default_rng(5).choice(np.arange(1024, 16384), 64, replace=False))
    out, amps, oout, ost, onz = run_both(T, wc, tree, 0, "c64", leaves)
    err, rel = float(np.max(np.abs(amps - ost))), rel_l2(amps, ost)
    nb = check_outcomes(out[leaves], oout, ost, onz.leaf_u[leaves], DELTA["c64"])
    print(family, part, "max-abs %.3g rel-l2 %.3g boundary leaves %d" % (err, rel, nb))
    assert err < 1e-5
    assert rel < rel_bound("c64", len(wc))


def test_range_runs_equal_full_run(T):
    wc = W.qft(12).with_depolarizing(0.01, 0.03)
    tree = ([6, 5, 4], [0, 30, 60, len(wc)])
    c = T.Circuit.from_workload(wc)
    nz = T.Noise.sample(c, tree, 2)
    plan = T.Plan(c, tree, "c64", {"chunk_states": 9})
    full = T.run(plan, nz)
    parts = [T.run(plan, nz, subtrees=(a, b)) for a, b in [(0, 1), (1, 4), (4, 6)]]
    assert np.array_equal(np.concatenate(parts), full)


def test_deterministic(T):
    wc = W.brickwall(16, 8, seed=3).with_depolarizing(0.01, 0.02)
    tree = ([8, 16], [0, 30, len(wc)])
    c = T.Circuit.from_workload(wc)
    nz = T.Noise.sample(c, tree, 4)
    plan = T.Plan(c, tree, "c64")
    a = T.run(plan, nz)
    b = T.run(plan, nz)
    assert np.array_equal(a, b)


def test_noiseless_ghz_outcomes(T):
    # closed form: every outcome is 0..0 or 1..1
    n = 16
    wc = W.ghz(n)
    c = T.Circuit.from_workload(wc)
    tree = ([64, 8], [0, 5, n])
    out = T.run(T.Plan(c, tree), T.Noise.sample(c, tree, 0))
    assert set(np.unique(out).tolist()) <= {0, (1 << n) - 1}
    frac = np.mean(out == 0)
    assert abs(frac - 0.5) < 4 * math.sqrt(0.25 / out.size)


def test_tree_histogram_vs_density_matrix(T):
    # statistics: tree estimate of the outcome distribution within a clustered
    # bound of the exact density-matrix distribution
    from oracle import density, tree as otree
    n = 4
    wc = W.concat(W.ghz(n), W.random_circuit(n, 8, seed=2)).with_depolarizing(0.05, 0.1)
    p_dm = np.real(np.diag(density.dm_run(n, wc.gates)))
    A = [256, 4, 4]
    tree = (A, [0, 5, 9, len(wc)])
    c = T.Circuit.from_workload(wc)
    out = T.run(T.Plan(c, tree), T.Noise.sample(c, tree, 1))
    p_hat = otree.hist_probs(out, n)
    bound = 0.5 * np.sum(np.sqrt(p_dm * (1 - p_dm) / A[0]))
    assert otree.tv_distance(p_hat, p_dm) < 3 * bound


@pytest.mark.parametrize("prec,tile", [("c64", 10), ("c64", 11), ("c64", 12), ("c128", 10), ("c128", 11)])
def test_qft_closed_form_every_tile(T, prec, tile):
    # noiseless QFT|x> against the DFT closed form, with qubits outside the
    # tile (fixed per tile) at several widths and pass splits
    for n in (11, 13, 16, 20):
        if n < tile:
            continue
        x = (0x5A5A5 >> (20 - n)) & ((1 << n) - 1)
        wc = W.concat(W.basis_prep(n, x), W.qft(n))
        c = T.Circuit.from_workload(wc)
        tree = ([1], [0, len(wc)])
        y = np.arange(1 << n)
        want = np.exp(2j * np.pi * x * y / (1 << n)) / math.sqrt(1 << n)
        for cost in (80, 100000):
            plan = T.Plan(c, tree, prec, {"tile_qubits": tile, "pass_cost": cost})
            _, amps = T.run_capture(plan, T.Noise.sample(c, tree, 0), [0])
            assert np.max(np.abs(amps[0] - want)) < TOL[prec], (n, cost)


def _diag_case(n, gates, rng):
    c = W.Circuit(n)
    for q in range(n):
        c.add((q,), W.haar_unitary(2, rng))
    for q, m in gates:
        c.add(q, m)
    return c


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_phase_run_term_groups(T, prec):
    # n = 12 with 10-qubit tiles: the second pass has register qubits
    # 6, 7, 10, 11, fixed qubits 8, 9 and lanes 0..5, so these runs exercise
    # every term group, several terms per register bit included
    rng = np.random.default_rng(0)

    def rd(k):
        return np.diag(np.exp(1j * rng.uniform(-np.pi, np.pi, k)))

    def cp(m, j):
        return ((m, j), W.cphase(np.pi / 2 ** (j - m)))

    cases = [
        [((9, 11), rd(4)), ((8, 11), rd(4))],                 # two fixed+register, same bit
        [((11, 9), rd(4)), ((8, 10), rd(4)), ((9, 10), rd(4))],
        [cp(m, 11) for m in range(10, -1, -1)],                # a whole QFT row
        [((8, 9), rd(4)), ((9,), rd(2)), ((8, 9), rd(4))],     # fixed only
        [((2, 9), rd(4)), ((9, 3), rd(4)), ((1, 4), rd(4)), ((5,), rd(2))],   # lane terms
        [((1, 7), rd(4)), ((2, 7), rd(4)), ((7, 3), rd(4))],   # lane+register, same bit
        [((6, 7), rd(4)), ((10,), rd(2)), ((11, 6), rd(4))],   # register only (table)
    ]
    for k, gates in enumerate(cases):
        wc = _diag_case(12, gates, rng)
        c = T.Circuit.from_workload(wc)
        tree = ([1], [0, len(wc)])
        for jit in (1, 2):
            plan = T.Plan(c, tree, prec, {"tile_qubits": 10, "pass_cost": 100000, "jit": jit})
            _, amps = T.run_capture(plan, T.Noise.sample(c, tree, 0), [0])
            _, ref = oracle.run_events(12, wc.gates)
            assert np.max(np.abs(amps[0] - ref)) < TOL[prec], (k, jit)


def test_tree_fidelity_loss_is_small(T):
    # the tree's normalised fidelity against per-shot sampling on a peaked
    # output (QFT round trip from a basis state), over noise seeds: the mean
    # difference stays within the paper's worst case (0.016) plus 3 SE
    from oracle import tree as otree
    n, shots = 12, 4096
    x = 0xA5A & ((1 << n) - 1)
    wc = W.concat(W.basis_prep(n, x), W.qft(n), W.inverse(W.qft(n))).with_depolarizing(5e-4, 5e-3)
    G = len(wc)
    c = T.Circuit.from_workload(wc)
    p_ideal = np.zeros(1 << n)
    p_ideal[x] = 1.0
    F = {}
    for name, tree in (("pershot", ([shots], [0, G])), ("tree", ([16, 16, 16], [0, G // 3, 2 * G // 3, G]))):
        plan = T.Plan(c, tree, "c64")
        vals = []
        for s in range(6):
            o = T.run(plan, T.Noise.sample(c, tree, s))
            vals.append(otree.fidelity_norm(p_ideal, otree.hist_probs(o, n)))
        F[name] = np.array(vals)
    d = F["tree"] - F["pershot"]
    se = d.std(ddof=1) / math.sqrt(d.size)
    assert 0.2 < F["pershot"].mean() < 0.99
    assert abs(d.mean()) <= 0.016 + 3 * se, (d.mean(), se)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_damping_channels(T, prec):
    # depolarizing plus twirled amplitude damping and phase damping on each
    # gate's qubits (one Pauli channel per gate), a 13-qubit brick-wall in a
    # 3-level tree, at rates high enough that most nodes draw events
    # (and thermal relaxation over the gate times, twirled the same way)
    for wc in (W.brickwall(13, 10, seed=4).with_noise(0.01, 0.05, gamma=0.05, lam=0.03),
               W.qft(12).with_thermal_relaxation(0.005, 0.02, 0.05, 0.3, 8.0, 6.0)):
        G = len(wc)
        tree = ([4, 3, 3], [0, G // 3, 2 * G // 3, G])
        out, amps, oout, ost, onz = run_both(T, wc, tree, 9, prec, np.arange(36))
        assert np.max(np.abs(amps - ost)) < TOL[prec]
        check_outcomes(out, oout, ost, onz.leaf_u, DELTA[prec])


def test_c4_precision_brickwall_22q(T):
    # the precision-sweep circuit family at 22 qubits: depth-24 brick-wall,
    # p2 = 1e-2 with twirled amplitude damping gamma = 1e-2; two leaves of a
    # (8, 32, 32) tree at complex64 (FP64 CDF) and complex128 against the
    # FP64 oracle
    n = 22
    wc = W.brickwall(n, 24, seed=1).with_noise(0.0, 1e-2, gamma=1e-2)
    G = len(wc)
    tree = ([8, 32, 32], [0, G // 3, 2 * G // 3, G])
    leaves = np.array([0, 8191], np.uint64)
    c = T.Circuit.from_workload(wc)
    nz = T.Noise.sample(c, tree, 3)
    onz = oracle.sample_noise(wc.gates, tree, 3)
    oout, ost = oracle.run_leaves(n, wc.gates, tree, onz, leaves, states=True)
    for prec in ("c64", "c128"):
        out, amps = T.run_capture(T.Plan(c, tree, prec), nz, leaves)
        err = np.max(np.abs(amps - ost))
        print(prec, "max-abs error vs oracle", err)
        assert err < TOL[prec]
        check_outcomes(out[leaves.astype(np.int64)], oout, ost, onz.leaf_u[leaves.astype(np.int64)], DELTA[prec])


@pytest.fixture(scope="module")
def c4_26q():
    """The precision sweep's circuit at its own size: 26 qubits, depth-24
    brick-wall, p2 = 1e-2 with twirled amplitude damping gamma = 1e-2, in a
    six-level tree with the sweep's equal cuts; the FP64 oracle's first and
    last leaf (computed once for both precisions)."""
    n = 26
    wc = W.brickwall(n, 24, seed=1).with_noise(0.0, 1e-2, gamma=1e-2)
    G = len(wc)
    shape = [2, 2, 2, 2, 2, 2]
    cut = [round(j * G / len(shape)) for j in range(len(shape) + 1)]
    tree = (shape, cut)
    leaves = np.array([0, 63], np.uint64)
    onz = oracle.sample_noise(wc.gates, tree, 3)
    oout, ost = oracle.run_leaves(n, wc.gates, tree, onz, leaves, states=True)
    return wc, tree, leaves, onz, oout, ost


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_c4_precision_brickwall_26q(T, c4_26q, prec):
    # error against the FP64 oracle at the precision sweep's own size
    # (512 MiB complex64 / 1 GiB complex128 states): complex64 evolution
    # with FP64 partial sums and CDF, and complex128 throughout
    wc, tree, leaves, onz, oout, ost = c4_26q
    c = T.Circuit.from_workload(wc)
    nz = T.Noise.sample(c, tree, 3)
    out, amps = T.run_capture(T.Plan(c, tree, prec), nz, leaves)
    err, rel = float(np.max(np.abs(amps - ost))), rel_l2(amps, ost)
    li = leaves.astype(np.int64)
    nb = check_outcomes(out[li], oout, ost, onz.leaf_u[li], DELTA[prec])
    print(prec, "26q max-abs %.3g rel-l2 %.3g boundary leaves %d" % (err, rel, nb))
    assert err < TOL[prec]
    assert rel < rel_bound(prec, len(wc))


def test_perceptron_kernels_against_oracle(T):
    # forward, loss gradient and Adam of the shape perceptron (float32 HIP
    # kernels) against the float64 oracle, batch not a multiple of the tile
    import torch
    from oracle import mlp as omlp
    d_in, h, d_out, B = 11, 128, 2, 37
    rng = np.random.default_rng(8)
    net = T.Perceptron(d_in, h, d_out, seed=4)
    p0 = net.params.cpu().numpy().astype(np.float64)
    x = rng.normal(size=(B, d_in)).astype(np.float32)
    t = rng.normal(size=(B, d_out)).astype(np.float32)
    w = np.array([1.0, 0.5], np.float32)
    y = net.forward(x).cpu().numpy()
    yo = omlp.forward(p0, x, d_in, h, d_out)
    assert np.max(np.abs(y - yo)) < 1e-4 * max(1.0, np.max(np.abs(yo)))
    loss = net.loss_grad(x, t, w)
    torch.cuda.synchronize()
    Lo, go = omlp.loss_grad(p0, x, t, w, d_in, h, d_out)
    assert abs(float(loss.cpu()) - Lo) < 1e-4 * max(1.0, Lo)
    g = net.grad.cpu().numpy()
    assert np.max(np.abs(g - go)) < 1e-4 * max(1.0, np.max(np.abs(go)))
    net.adam(lr=1e-2)
    po, _, _ = omlp.adam(p0, go, np.zeros_like(p0), np.zeros_like(p0), 1, 1e-2)
    assert np.max(np.abs(net.params.cpu().numpy() - po)) < 1e-5


def test_learned_shape_against_partition_heuristic(T):
    # the committed shape model (trained on the simulator's own runs of 12-22
    # qubit circuits) against the DCP shape on a circuit it has not seen:
    # measured time per leaf and the design effect of the fidelity estimate
    import torch
    from paper_2203_13892_amd import learned as Lm
    model = Lm.ShapeModel.load(T)
    wc = W.brickwall(18, 18, seed=11).with_noise(1e-3, 1e-2)
    shots = 8192
    (shape, _), src = Lm.choose_shape(T, model, wc, shots)
    assert src == "learned"
    c = T.Circuit.from_workload(wc)
    # DCP's own trees (arities and cuts): a separate state copy costing 26
    # gates, and the copy fused into the child's first pass (about one gate)
    dshape, dcut = T.dcp(c, shots, 1.96, 0.01, 26.0, 8)
    fshape, fcut = T.dcp(c, shots, 1.96, 0.01, 1.0, 8)
    p_ideal = Lm.ideal_probs(T, wc)
    t_d, deff_d, ws = Lm.measure(T, torch, wc, c, dshape, shots, p_ideal, 1, cut=dcut)
    t_f, deff_f, ws = Lm.measure(T, torch, wc, c, fshape, shots, p_ideal, 1, ws, cut=fcut)
    t_l, deff_l, ws = Lm.measure(T, torch, wc, c, shape, shots, p_ideal, 1, ws)
    print("learned", shape, t_l, deff_l, "dcp", dshape, dcut, t_d, deff_d, "dcp_fused", fshape, fcut, t_f, deff_f)
    assert t_l < 0.8 * t_d
    assert deff_l < 12.0
    # far outside the training range: the heuristic decides
    big = W.brickwall(30, 4, seed=1).with_noise(1e-3, 1e-2)
    assert Lm.choose_shape(T, model, big, shots)[1] == "dcp"


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_batch_equals_separate_runs(T, prec):
    # runs of different circuits, qubit counts, trees and noise advanced
    # together give exactly the outcomes of the same runs made one by one,
    # and every run matches the oracle
    rng = np.random.default_rng(12)
    specs = [(W.qft(10).with_depolarizing(1e-2, 5e-2), ([40], None)),
             (W.ghz(12).with_depolarizing(1e-2, 5e-2), ([4, 4, 3], None)),
             (W.brickwall(14, 8, seed=3).with_noise(0.0, 3e-2, gamma=2e-2), ([8, 8], None)),
             (W.qaoa(12, 2, seed=5).with_depolarizing(1e-2, 3e-2), ([6, 5], None)),
             (W.random_circuit(11, 60, seed=9).with_depolarizing(2e-2, 5e-2), ([3, 3, 3, 3], None))]
    plans, noises, wcs, trees = [], [], [], []
    for i, (wc, (A, _)) in enumerate(specs):
        G = len(wc)
        tree = (A, [round(j * G / len(A)) for j in range(len(A) + 1)])
        c = T.Circuit.from_workload(wc)
        plans.append(T.Plan(c, tree, prec, {"chunk_states": 7}))
        noises.append(T.Noise.sample(c, tree, 20 + i))
        wcs.append(wc)
        trees.append(tree)
    b = T.Batch(plans, noises)
    assert b.info()["steps"] > 1
    outs = b.run()
    for i in range(len(specs)):
        want = T.run(plans[i], noises[i])
        assert np.array_equal(outs[i], want), i
    # every run against the oracle: the batch's outcomes on every leaf, and
    # the amplitudes of every leaf of the same plan and insertion list
    for i in range(len(specs)):
        onz = oracle.sample_noise(wcs[i].gates, trees[i], 20 + i)
        oout, ost = oracle.run_leaves(wcs[i].n, wcs[i].gates, trees[i], onz, states=True)
        check_outcomes(outs[i], oout, ost, onz.leaf_u, DELTA[prec])
        _, amps = T.run_capture(plans[i], noises[i], np.arange(outs[i].size))
        assert np.max(np.abs(amps - ost)) < TOL[prec], i


def _repeating_events(wc, tree, rng, rate=0.05, copy=0.35):
    """Insertion list where many siblings repeat an earlier sibling's events
    (or have none), so that merged states are common."""
    A, cut = tree
    node_off, eg, ec = [0], [], []
    for l in range(len(A)):
        I = int(np.prod(A[:l + 1]))
        prev = None
        for m in range(I):
            if prev is not None and m % A[l] != 0 and rng.random() < copy:
                ev = prev
            else:
                ev = [(g, int(rng.integers(1, 4 ** len(wc.gates[g][0]))))
                      for g in range(cut[l], cut[l + 1]) if rng.random() < rate]
            for g, k in ev:
                eg.append(g)
                ec.append(k)
            node_off.append(len(eg))
            prev = ev
    return (np.array(node_off, np.uint64), np.array(eg, np.uint32), np.array(ec, np.uint8),
            rng.random(int(np.prod(A))))


def _distinct_histories(tree, arr):
    """Nodes per level minus distinct (parent class, own event set) classes."""
    A, _ = tree
    node_off, eg, ec = arr[0].astype(np.int64), arr[1], arr[2]
    merged, cls_prev, nu = 0, None, 0
    for l in range(len(A)):
        I = int(np.prod(A[:l + 1]))
        ids, cls = {}, []
        for m in range(I):
            par = 0 if l == 0 else cls_prev[m // A[l]]
            ev = tuple(sorted(zip(eg[node_off[nu]:node_off[nu + 1]].tolist(),
                                  ec[node_off[nu]:node_off[nu + 1]].tolist())))
            cls.append(ids.setdefault((par, ev), len(ids)))
            nu += 1
        merged += I - len(ids)
        cls_prev = cls
    return merged


@pytest.mark.parametrize("jit", [1, 2])
@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_merged_states_equal_separate_states(T, prec, jit):
    # nodes with equal parent state, frame and events share one state: the
    # outcomes are bit-identical to computing every node, the captured
    # leaves match the oracle, and at least every repeated history is
    # merged (one chunk per level here; events after a level's last op may
    # merge more)
    rng = np.random.default_rng(31)
    wc = mixed_gates(12, 48, rng)
    tree = ([4, 8, 8], [0, 16, 32, 48])
    arr = _repeating_events(wc, tree, rng)
    c = T.Circuit.from_workload(wc)
    nz = T.Noise.from_arrays(c, tree, *arr)
    merged_plan = T.Plan(c, tree, prec, {"chunk_states": 512, "jit": jit})
    plain_plan = T.Plan(c, tree, prec, {"chunk_states": 512, "no_merge": 1, "jit": jit})
    out_m, st_m = T.run(merged_plan, nz, stats=True)
    out_p, st_p = T.run(plain_plan, nz, stats=True)
    assert np.array_equal(out_m, out_p)
    assert st_p["nodes_merged"] == 0
    want = _distinct_histories(tree, arr)
    assert want > 100
    assert st_m["nodes_merged"] >= want
    assert st_m["pass_states"] < st_p["pass_states"]
    leaves = np.arange(256)
    out, amps, oout, ost, _ = run_both(T, wc, tree, 0, prec, leaves, noise_arrays=arr, tuning={"jit": jit})
    assert np.max(np.abs(amps - ost)) < TOL[prec]
    check_outcomes(out, oout, ost, arr[3], DELTA[prec])


def test_merged_states_small_chunks_and_ranges(T):
    # merging inside small ragged chunks, and over subtree ranges, gives the
    # unmerged outcomes
    rng = np.random.default_rng(32)
    wc = mixed_gates(11, 45, rng)
    tree = ([5, 6, 7], [0, 12, 30, 45])
    arr = _repeating_events(wc, tree, rng, rate=0.04)
    c = T.Circuit.from_workload(wc)
    nz = T.Noise.from_arrays(c, tree, *arr)
    base = T.run(T.Plan(c, tree, "c64", {"chunk_states": 5, "no_merge": 1}), nz)
    plan = T.Plan(c, tree, "c64", {"chunk_states": 5, "max_ops_per_pass": 6})
    out, st = T.run(plan, nz, stats=True)
    assert st["nodes_merged"] > 0
    assert np.array_equal(out, base)
    parts = [T.run(plan, nz, subtrees=(a, b)) for a, b in [(0, 2), (2, 3), (3, 5)]]
    assert np.array_equal(np.concatenate(parts), base)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_readout_flips_on_device(T, prec):
    # read-out flips XOR the measured bits on the device: outcomes equal the
    # oracle's (trajectory, measurement, then flips), also for leaves that
    # share a merged state, in single runs and in a batch
    wc = W.qft(12).with_depolarizing(2e-3, 2e-2).with_readout(np.linspace(0.0, 0.3, 12))
    G = len(wc)
    tree = ([4, 8, 16], [0, G // 3, 2 * G // 3, G])
    c = T.Circuit.from_workload(wc)
    nz = T.Noise.sample(c, tree, 4)
    onz = oracle.sample_noise(wc.gates, tree, 4, readout=wc.readout)
    assert np.array_equal(nz.flips(), onz.leaf_flip)
    plan = T.Plan(c, tree, prec)
    out, st = T.run(plan, nz, stats=True)
    assert st["nodes_merged"] > 0
    oout, ost = oracle.run_leaves(wc.n, wc.gates, tree, onz, states=True)
    bad = check_outcomes(out ^ onz.leaf_flip, oout ^ onz.leaf_flip, ost, onz.leaf_u, DELTA[prec])
    assert bad <= 2
    c0 = T.Circuit.from_workload(wc)
    c0.set_readout(None)
    plain = T.run(T.Plan(c0, tree, prec), T.Noise.sample(c0, tree, 4))
    assert np.array_equal(out, plain ^ onz.leaf_flip.astype(np.uint64))
    outs = T.Batch([plan, plan], [nz, nz]).run()
    assert np.array_equal(outs[0], out) and np.array_equal(outs[1], out)


def test_batch_graph_replay_equals_plain_launches(T):
    # the recorded launches replayed several times, with other device work
    # and synchronisations in between, and again after a workspace change,
    # give the plain launches' outcomes every time
    import torch
    specs = [(W.qft(10).with_depolarizing(1e-2, 5e-2), [32]),
             (W.ghz(12).with_depolarizing(1e-2, 5e-2), [4, 4, 2]),
             (W.brickwall(11, 6, seed=2).with_depolarizing(1e-2, 3e-2), [6, 6])]
    plans, noises = [], []
    for i, (wc, A) in enumerate(specs):
        G = len(wc)
        tree = (A, [round(j * G / len(A)) for j in range(len(A) + 1)])
        c = T.Circuit.from_workload(wc)
        plans.append(T.Plan(c, tree, "c64", {"chunk_states": 5}))
        noises.append(T.Noise.sample(c, tree, 40 + i))
    b = T.Batch(plans, noises)
    need = b.info()["workspace_bytes"]
    ws = T.Workspace(need)
    want = b.run(ws)
    b.use_graph(True)
    other = T.Plan(T.Circuit.from_workload(specs[0][0]), ([8], [0, len(specs[0][0])]), "c64")
    other_nz = T.Noise.sample(T.Circuit.from_workload(specs[0][0]), ([8], [0, len(specs[0][0])]), 3)
    for rep in range(3):
        got = b.run(ws)
        assert all(np.array_equal(g, w) for g, w in zip(got, want)), rep
        T.run(other, other_nz)
        torch.cuda.synchronize()
    ws2 = T.Workspace(need)
    for rep in range(2):
        got = b.run(ws2)
        assert all(np.array_equal(g, w) for g, w in zip(got, want)), rep
    b.use_graph(False)
    got = b.run(ws)
    assert all(np.array_equal(g, w) for g, w in zip(got, want))


@pytest.mark.parametrize("case", ["qft14", "bw13", "swaps16"])
def test_partials_from_last_pass_equal_separate_sampling(T, case):
    # the last leaf pass writes the sampling partials (per tile, in the
    # final layout); outcomes equal the separate partials kernel's and the
    # oracle's except at CDF-boundary leaves
    rng = np.random.default_rng(50)
    if case == "qft14":
        wc = W.qft(14).with_depolarizing(2e-3, 2e-2)
    elif case == "bw13":
        wc = W.brickwall(13, 10, seed=4).with_depolarizing(2e-3, 2e-2)
    else:
        wc = mixed_gates(16, 50, rng)
        for i in range(8):
            wc.add((i, 15 - i), W.swap())
    G = len(wc)
    tree = ([4, 4, 4], [0, G // 3, 2 * G // 3, G])
    c = T.Circuit.from_workload(wc)
    arr = event_arrays(wc, tree, rng, rate=0.02) if case == "swaps16" else None
    nz = T.Noise.from_arrays(c, tree, *arr) if arr is not None else T.Noise.sample(c, tree, 6)
    fused = T.Plan(c, tree, "c64", {"sample_block_log": 8})
    assert [ln for ln in fused.describe().split("\n") if ln.startswith("sampling")][0].split()[1] == "1"
    sep = T.Plan(c, tree, "c64", {"sample_block_log": 8, "separate_sampling": 1})
    a, b = T.run(fused, nz), T.run(sep, nz)
    onz = oracle.Noise(*[np.asarray(x) for x in arr]) if arr is not None else oracle.sample_noise(wc.gates, tree, 6)
    oout, ost = oracle.run_leaves(wc.n, wc.gates, tree, onz, states=True)
    check_outcomes(a, oout, ost, onz.leaf_u, DELTA["c64"])
    check_outcomes(b, oout, ost, onz.leaf_u, DELTA["c64"])
    assert np.sum(a != b) <= 2


def test_largest_sizes(T):
    # 30 qubits at complex64 (8 GiB states) and 29 at complex128: GHZ
    # outcomes are all-zeros or all-ones before the read-out flips; a
    # 28-qubit QFT round trip returns its input on every shot
    for n, prec in ((30, "c64"), (29, "c128")):
        wc = W.ghz(n).with_readout(0.25)
        G = len(wc)
        tree = ([2, 2], [0, G // 2, G])
        c = T.Circuit.from_workload(wc)
        nz = T.Noise.sample(c, tree, 1)
        out = T.run(T.Plan(c, tree, prec), nz)
        flips = nz.flips().astype(np.uint64)
        base = out ^ flips
        assert np.all((base == 0) | (base == (1 << n) - 1)), (n, base)
        del nz, c
    n, x = 28, 0xA5C3E1F & ((1 << 28) - 1)
    wc = W.concat(W.basis_prep(n, x), W.qft(n), W.inverse(W.qft(n)))
    G = len(wc)
    tree = ([3], [0, G])
    c = T.Circuit.from_workload(wc)
    out = T.run(T.Plan(c, tree, "c64"), T.Noise.sample(c, tree, 0))
    assert np.all(out == x), out


@pytest.mark.parametrize("jit", [1, 2])
@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_degenerate_trees(T, prec, jit):
    # arity-1 levels, a level of swap gates only (a pass with no ops), a
    # one-gate level, and a list without events: outcomes and amplitudes
    # match the oracle
    rng = np.random.default_rng(61)
    wc = mixed_gates(12, 20, rng)
    wc.add((0, 7), W.swap())
    wc.add((3, 11), W.swap())
    wc.add((5,), W.haar_unitary(2, rng))
    G = len(wc)
    for tree in (([1, 1, 3], [0, 10, 20, G]), ([2, 3, 2], [0, 20, 22, G]), ([1], [0, G])):
        arr = event_arrays(wc, tree, rng, rate=0.3)
        leaves = np.arange(int(np.prod(tree[0])))
        out, amps, oout, ost, _ = run_both(T, wc, tree, 0, prec, leaves, noise_arrays=arr,
                                           tuning={"jit": jit})
        assert np.max(np.abs(amps - ost)) < TOL[prec]
        check_outcomes(out, oout, ost, arr[3], DELTA[prec])
    tree = ([4, 4], [0, 10, G])
    none = (np.zeros(1 + 4 + 16, np.uint64), np.zeros(0, np.uint32), np.zeros(0, np.uint8), rng.random(16))
    out, amps, oout, ost, _ = run_both(T, wc, tree, 0, prec, np.arange(16), noise_arrays=none,
                                       tuning={"jit": jit})
    assert np.max(np.abs(amps - ost)) < TOL[prec]
    check_outcomes(out, oout, ost, none[3], DELTA[prec])


def test_c2_20q_tree_sampled_leaves_c128(T):
    # the same 20-qubit QFT tree in complex128 (16 MiB states) on a handful
    # of leaves: amplitudes within 1e-12 of the oracle
    wc = W.qft(20).with_depolarizing(1e-3, 1e-2)
    G = len(wc)
    tree = ([16, 32, 32], [0, G // 3, 2 * G // 3, G])
    leaves = np.array([0, 1, 5000, 16383])
    out, amps, oout, ost, onz = run_both(T, wc, tree, 0, "c128", leaves)
    assert np.max(np.abs(amps - ost)) < 1e-12
    assert rel_l2(amps, ost) < rel_bound("c128", len(wc))
    check_outcomes(out[leaves], oout, ost, onz.leaf_u[leaves], DELTA["c128"])


@pytest.mark.parametrize("seed", range(32))
def test_random_configurations(T, seed):
    # random circuits (every op class, swap networks), trees, tunings
    # (level-end exchanges on for half the seeds), insertion lists with
    # repeated histories, and read-out flips: every leaf's amplitudes and
    # outcome against the oracle
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(11, 15))
    wc = mixed_gates(n, int(rng.integers(30, 70)), rng)
    for i in range(int(rng.integers(0, n // 2))):
        a, b = [int(x) for x in rng.choice(n, 2, replace=False)]
        wc.add((a, b), W.swap())
    G = len(wc)
    levels = int(rng.integers(1, 4))
    cut = [0] + sorted(rng.choice(np.arange(1, G), levels - 1, replace=False).tolist()) + [G]
    A = [int(a) for a in rng.integers(2, 6, levels)]
    tree = (A, cut)
    tuning = {"chunk_states": int(rng.integers(1, 8)), "tile_qubits": int(rng.choice([10, 11])),
              "sample_block_log": int(rng.integers(8, 13)), "separate_sampling": int(rng.integers(0, 2)),
              "no_merge": int(rng.integers(0, 2)), "pass_cost": int(rng.choice([120, 480])),
              "jit": 1 + seed % 2, "mfma_min_ops": (1, 2, 1000)[seed % 3],
              "level_exchange": 1 + (seed // 2) % 2}
    arr = _repeating_events(wc, tree, rng, rate=float(rng.uniform(0.01, 0.1)))
    flips = rng.integers(0, 1 << n, arr[3].size).astype(np.uint32) if seed % 2 else None
    c = T.Circuit.from_workload(wc)
    nz = T.Noise.from_arrays(c, tree, *arr, leaf_flip=flips)
    prec = "c128" if seed % 3 == 0 else "c64"
    plan = T.Plan(c, tree, prec, tuning)
    leaves = np.arange(int(np.prod(A)))
    out, amps = T.run_capture(plan, nz, leaves)
    onz = oracle.Noise(*[np.asarray(x) for x in arr], flips)
    oout, ost = oracle.run_leaves(wc.n, wc.gates, tree, onz, leaves, states=True)
    assert np.max(np.abs(amps - ost)) < TOL[prec], tuning
    f = np.zeros(leaves.size, np.uint64) if flips is None else flips.astype(np.uint64)
    check_outcomes(out ^ f, oout ^ f, ost, arr[3], DELTA[prec])


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_events_after_the_last_op_share_states(T, prec):
    # events on trailing relabelled swap gates (after a level's last op)
    # change only the end frame: such nodes share their sibling's state, and
    # outcomes and amplitudes (frame applied) still match the oracle
    rng = np.random.default_rng(70)
    wc = mixed_gates(12, 30, rng)
    for i in range(5):
        wc.add((i, 11 - i), W.swap())
    G = len(wc)
    tree = ([3, 8], [0, 15, G])
    # every leaf: one event on a trailing swap, or none
    node_off, eg, ec = [0, 0, 0, 0], [], []
    for m in range(24):
        if m % 3:
            eg.append(G - 1 - (m % 5))
            ec.append(int(rng.integers(1, 16)))
        node_off.append(len(eg))
    arr = (np.array(node_off, np.uint64), np.array(eg, np.uint32), np.array(ec, np.uint8), rng.random(24))
    c = T.Circuit.from_workload(wc)
    nz = T.Noise.from_arrays(c, tree, *arr)
    plan = T.Plan(c, tree, prec, {"chunk_states": 64})
    out, st = T.run(plan, nz, stats=True)
    # the 3 roots have no events and share one state, so all 24 leaves start
    # from it and share one state whatever their trailing events
    assert st["nodes_merged"] == 2 + 23
    plain = T.run(T.Plan(c, tree, prec, {"chunk_states": 64, "no_merge": 1}), nz)
    assert np.array_equal(out, plain)
    out2, amps, oout, ost, _ = run_both(T, wc, tree, 0, prec, np.arange(24), noise_arrays=arr)
    assert np.max(np.abs(amps - ost)) < TOL[prec]
    check_outcomes(out2, oout, ost, arr[3], DELTA[prec])


@pytest.mark.parametrize("case", ["qft20", "bw20", "mixed14"])
def test_specialised_kernels_match_generic(T, case):
    # the plan-specialised pass kernels against the generic kernel on the
    # same plan and insertion list: every leaf's outcome and sampled leaves'
    # amplitudes; the run statistics show which kernel took how many states
    # (nodes with more than three events inside a phase run, or a frame
    # change between a run's register-only gates, go to the generic kernel)
    rng = np.random.default_rng(77)
    if case == "qft20":
        wc = W.qft(20).with_depolarizing(1e-3, 1e-2)
        A = [16, 32, 32]
    elif case == "bw20":
        wc = W.brickwall(20, 20, seed=1).with_depolarizing(1e-3, 1e-2)
        A = [8, 16, 16]
    else:
        wc = mixed_gates(14, 80, rng).with_depolarizing(2e-2, 8e-2)
        A = [8, 8, 8]
    G = len(wc)
    tree = (A, [round(j * G / len(A)) for j in range(len(A) + 1)])
    c = T.Circuit.from_workload(wc)
    nz = T.Noise.sample(c, tree, 9)
    leaves = np.sort(rng.choice(int(np.prod(A)), 12, replace=False))
    res = {}
    for jit in (1, 2):
        plan = T.Plan(c, tree, "c64", {"jit": jit})
        out, st = T.run(plan, nz, stats=True)
        _, amps = T.run_capture(plan, nz, leaves)
        res[jit] = (out, st, amps)
    (o1, s1, a1), (o2, s2, a2) = res[1], res[2]
    print(case, "specialised launches", s1["jit_launches"], "states", s1["jit_states"], "of", s1["pass_states"])
    assert s2["jit_launches"] == 0
    assert s1["jit_launches"] > 0 and s1["jit_states"] >= 0.5 * s1["pass_states"]
    assert np.max(np.abs(a1 - a2)) < 1e-6
    assert np.mean(o1 == o2) > 0.99


@pytest.mark.parametrize("min_ops", [1, 2])
@pytest.mark.parametrize("n", [11, 14])
def test_fused_register_blocks_on_matrix_cores(T, n, min_ops):
    # runs of dense ops on the five register qubits fused into 32x32
    # unitaries and applied with MFMA (complex64): amplitudes and outcomes
    # against the oracle, with events before, after and between the fused
    # ops (nodes with events between them take the generic kernel), frames
    # with X and Z parts on register qubits, and a lane exchange in between
    rng = np.random.default_rng(300 + n + min_ops)
    wc = W.Circuit(n)
    for q in range(n):
        wc.add((q,), W.haar_unitary(2, rng))
    for layer in range(8):
        for a in range(layer % 2, n - 1, 2):
            wc.add((a, a + 1), W.haar_unitary(4, rng))
        wc.add((int(rng.integers(n)),), W.haar_unitary(2, rng))
    G = len(wc)
    tree = ([4, 6], [0, G // 2, G])
    c = T.Circuit.from_workload(wc)
    plan = T.Plan(c, tree, "c64", {"jit": 1, "mfma_min_ops": min_ops})
    blocks = [ln for ln in plan.describe().splitlines() if ln.startswith("block")]
    assert blocks, "no fused block"
    arr = event_arrays(wc, tree, rng, rate=0.04)
    out, amps, oout, ost, _ = run_both(T, wc, tree, 0, "c64", np.arange(24), noise_arrays=arr,
                                       tuning={"jit": 1, "mfma_min_ops": min_ops})
    print("fused blocks", len(blocks), "max-abs %.3g" % np.max(np.abs(amps - ost)))
    assert np.max(np.abs(amps - ost)) < TOL["c64"]
    check_outcomes(out, oout, ost, arr[3], DELTA["c64"])
    # the same list through the generic kernel only: equal outcomes
    nz = T.Noise.from_arrays(c, tree, *arr)
    base = T.run(T.Plan(c, tree, "c64", {"jit": 2}), nz)
    fused, st = T.run(plan, nz, stats=True)
    assert st["jit_launches"] > 0
    assert np.mean(base == fused) > 0.9


@pytest.mark.parametrize("n,tile", [(7, 11), (10, 11), (11, 11), (12, 11), (14, 11), (13, 10)])
def test_levels_in_lds(T, n, tile):
    # generic complex64 kernels with every pass of a level in one launch and
    # the state in LDS between passes (tuning lds_levels = 1; levels of two
    # or more passes): every
    # op class, events inside and between passes, shared states, a ragged
    # last chunk and partial tiles (n < 11), against the oracle and against
    # the same plan run pass by pass
    rng = np.random.default_rng(500 + n)
    wc = mixed_gates(n, 60, rng)
    tree = ([3, 4, 6], [0, 14, 35, 60])
    arr = event_arrays(wc, tree, rng, rate=0.08)
    leaves = np.arange(72)
    tun = {"chunk_states": 5, "max_ops_per_pass": 6, "tile_qubits": tile, "jit": 2}
    out, amps, oout, ost, _ = run_both(T, wc, tree, 0, "c64", leaves, tuning=dict(tun, lds_levels=1),
                                       noise_arrays=arr)
    c = T.Circuit.from_workload(wc)
    plan = T.Plan(c, tree, "c64", dict(tun, lds_levels=1))
    passes = [plan.info(l)["passes_level"] for l in range(3)]
    assert max(passes) >= 2, passes
    print("n", n, "passes per level", passes, "max-abs %.3g" % np.max(np.abs(amps - ost)))
    assert np.max(np.abs(amps - ost)) < TOL["c64"]
    check_outcomes(out, oout, ost, arr[3], DELTA["c64"])
    # the same plan pass by pass: the same ops, compiled in another kernel,
    # so amplitudes agree to rounding and outcomes up to CDF boundaries
    nz = T.Noise.from_arrays(c, tree, *arr)
    base_plan = T.Plan(c, tree, "c64", dict(tun, lds_levels=2))
    base, st_b = T.run(base_plan, nz, stats=True)
    lds, st_l = T.run(plan, nz, stats=True)
    _, amps_b = T.run_capture(base_plan, nz, leaves)
    assert np.max(np.abs(amps_b - amps)) < 1e-6
    check_outcomes(base, oout, ost, arr[3], DELTA["c64"])
    check_outcomes(lds, oout, ost, arr[3], DELTA["c64"])
    print("launches pass by pass", st_b["pass_launches"], "with levels in LDS", st_l["pass_launches"])
    assert st_l["pass_launches"] < st_b["pass_launches"]


@pytest.mark.parametrize("family", ["qft", "bw"])
def test_level_exchange_20q(T, family):
    # tuning level_exchange = 1: lane exchanges at the end of a level's last
    # pass (QFT-20: level 1 in one pass instead of two; brick-wall: another
    # layout at every level) against the oracle, on the first two sibling
    # groups of subtree 0 and 64 random leaves
    wc, tree = _c2_case(family)
    c = T.Circuit.from_workload(wc)
    on = T.Plan(c, tree, "c64", {"level_exchange": 1})
    off = T.Plan(c, tree, "c64", {"level_exchange": 2})
    p_on = [on.info(l)["passes_level"] for l in range(3)]
    p_off = [off.info(l)["passes_level"] for l in range(3)]
    assert on.describe() != off.describe()
    if family == "qft":
        assert p_on == [1, 1, 1] and p_off == [1, 2, 1]
    leaves = np.concatenate([np.arange(64), np.sort(np.random.default_rng(6).choice(
        np.arange(1024, 16384), 64, replace=False))])
    out, amps, oout, ost, onz = run_both(T, wc, tree, 0, "c64", leaves, tuning={"level_exchange": 1})
    err, rel = float(np.max(np.abs(amps - ost))), rel_l2(amps, ost)
    nb = check_outcomes(out[leaves], oout, ost, onz.leaf_u[leaves], DELTA["c64"])
    print(family, "passes per level", p_on, "(off:", p_off, ")", "max-abs %.3g rel-l2 %.3g boundary leaves %d"
          % (err, rel, nb))
    assert err < 1e-5
    assert rel < rel_bound("c64", len(wc))


@pytest.mark.parametrize("prec,jit", [("c64", 1), ("c64", 2), ("c128", 2)])
def test_level_exchange_mixed_events(T, prec, jit):
    # level-end exchanges on 13 qubits in 10-qubit tiles, every op class,
    # events in every level (also on the gates just before an exchange),
    # ragged chunks, in the specialised and the generic kernels
    rng = np.random.default_rng(77)
    n = 13
    wc = mixed_gates(n, 60, rng)
    tree = ([3, 4, 6], [0, 14, 35, 60])
    arr = event_arrays(wc, tree, rng, rate=0.08)
    leaves = np.arange(72)
    tun = {"chunk_states": 5, "tile_qubits": 10, "jit": jit, "level_exchange": 1}
    c = T.Circuit.from_workload(wc)
    assert T.Plan(c, tree, prec, tun).describe() != T.Plan(c, tree, prec, dict(tun, level_exchange=2)).describe()
    out, amps, oout, ost, _ = run_both(T, wc, tree, 0, prec, leaves, tuning=tun, noise_arrays=arr)
    err = float(np.max(np.abs(amps - ost)))
    print(prec, "jit", jit, "max-abs %.3g" % err)
    assert err < TOL[prec]
    check_outcomes(out, oout, ost, arr[3], DELTA[prec])
