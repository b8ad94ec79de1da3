"""Host-side checks of the library (no GPU): the C ABI loads and exports every
declared symbol, the host noise sampler and DCP agree with the oracle's
independent implementations, and argument errors map to the documented
status codes."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from oracle import tree as otree
from paper_2203_13892_amd import tqsim as T
from paper_2203_13892_amd import workloads as W
from paper_2203_13892_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "tqsim.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tqs_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = header_functions()
    assert len(names) >= 20
    L = ctypes.CDLL(T.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    # and the binding declares a signature for each of them
    assert set(names) == set(T.SIGNATURES)


def _same_noise(a, o):
    node_off, ev_gate, ev_code, leaf_u = a
    return (np.array_equal(node_off, o.node_off) and np.array_equal(ev_gate, o.ev_gate)
            and np.array_equal(ev_code, o.ev_code) and np.array_equal(leaf_u, o.leaf_u))


@pytest.mark.parametrize("case", range(6))
def test_noise_sampler_matches_oracle(case):
    rng = np.random.default_rng(case)
    n = int(rng.integers(2, 7))
    wc = W.random_circuit(n, int(rng.integers(5, 40)), seed=case,
                          p1=float(rng.uniform(0, 0.3)), p2=float(rng.uniform(0, 0.5)))
    G = len(wc)
    levels = int(rng.integers(1, min(4, G) + 1))
    cut = [0] + sorted(rng.choice(np.arange(1, G), levels - 1, replace=False).tolist()) + [G]
    A = [int(a) for a in rng.integers(1, 6, levels)]
    seed = int(rng.integers(1 << 62))
    c = T.Circuit.from_workload(wc)
    assert _same_noise(T.Noise.sample(c, (A, cut), seed).arrays(),
                       oracle.sample_noise(wc.gates, (A, cut), seed))


def test_noise_sampler_matches_oracle_qft20_tree():
    wc = W.qft(20).with_depolarizing(1e-3, 1e-2)
    c = T.Circuit.from_workload(wc)
    tree = ([16, 32, 32], [0, 74, 147, 220])
    assert _same_noise(T.Noise.sample(c, tree, 0).arrays(), oracle.sample_noise(wc.gates, tree, 0))


def test_set_depolarizing_equals_explicit_probabilities():
    wc = W.qft(6)
    a = T.Circuit.from_workload(wc).set_depolarizing(0.01, 0.05)
    b = T.Circuit.from_workload(wc.with_depolarizing(0.01, 0.05))
    t = ([200], [0, len(wc)])
    for x, y in zip(T.Noise.sample(a, t, 5).arrays(), T.Noise.sample(b, t, 5).arrays()):
        assert np.array_equal(x, y)


def test_noise_import_roundtrip_and_validation():
    wc = W.random_circuit(4, 12, seed=1, p1=0.3, p2=0.3)
    c = T.Circuit.from_workload(wc)
    tree = ([2, 3], [0, 5, 12])
    arr = T.Noise.sample(c, tree, 9).arrays()
    back = T.Noise.from_arrays(c, tree, *arr).arrays()
    for x, y in zip(arr, back):
        assert np.array_equal(x, y)
    node_off = np.zeros(9, np.uint64)
    node_off[1:] = 1
    with pytest.raises(T.TqsError) as e:   # event gate outside node 0's subcircuit
        T.Noise.from_arrays(c, tree, node_off, [7], [1], np.zeros(6))
    assert e.value.status == -1
    node_off = np.zeros(9, np.uint64)
    with pytest.raises(T.TqsError):        # leaf uniform out of range
        T.Noise.from_arrays(c, tree, node_off, [], [], np.ones(6))


def test_dcp_matches_oracle():
    rng = np.random.default_rng(2)
    for _ in range(100):
        n = int(rng.integers(2, 8))
        G = int(rng.integers(1, 120))
        wc = W.random_circuit(n, G, seed=int(rng.integers(1000)), p1=float(rng.uniform(0, .01)),
                              p2=float(rng.uniform(0, .05)))
        N = int(rng.integers(1, 50000))
        C = float(rng.uniform(0, 12))
        ml = int(rng.integers(1, 10))
        got = T.dcp(T.Circuit.from_workload(wc), N, 1.96, 0.01, C, ml)
        want = otree.dcp(wc.error_rates(), N, 1.96, 0.01, C, ml)
        assert got == (list(want[0]), list(want[1]))


def test_dcp_printed_shapes_from_library():
    c = T.Circuit.from_workload(W.Circuit(4, [((0,), W.H, W.depolarizing_probs(1e-3, 1))] * 120))
    assert T.dcp(c, 1000, 1.96, 0.01, 6)[0] == [250, 2, 2]
    c = T.Circuit.from_workload(W.Circuit(4, [((0,), W.H, W.depolarizing_probs(1e-3, 1))] * 472))
    assert T.dcp(c, 32000, 1.96, 0.01, 8)[0] == [500] + [2] * 6


def test_argument_errors():
    with pytest.raises(T.TqsError) as e:
        T.Circuit(0)
    assert e.value.status == -6
    c = T.Circuit(3)
    with pytest.raises(T.TqsError) as e:
        c.add_gate((3,), W.H)
    assert e.value.status == -1
    with pytest.raises(T.TqsError):
        c.add_gate((0,), np.array([[1, 1], [0, 1]]))        # not unitary
    with pytest.raises(T.TqsError):
        c.add_gate((1, 1), W.cx())                          # repeated qubit
    with pytest.raises(T.TqsError):
        c.add_gate((0,), W.H, [0.5, 0.5, 0.5, 0.0])         # probabilities sum to 1.5
    c.add_gate((0,), W.H).add_gate((0, 1), W.cx())
    for A, cut in [([2, 2], [0, 1, 1]), ([0], [0, 2]), ([2], [0, 1]), ([2], [1, 2])]:
        with pytest.raises(T.TqsError) as e:
            T.Plan(c, (A, cut))
        assert e.value.status == -2
    with pytest.raises(T.TqsError):
        T.Plan(c, ([2], [0, 2]), tuning={"tile_qubits": 3})


def test_workspace_too_small_is_reported_before_device_work():
    wc = W.qft(5).with_depolarizing(0.01, 0.01)
    c = T.Circuit.from_workload(wc)
    tree = ([4, 2], [0, 5, len(wc)])
    p = T.Plan(c, tree)
    nz = T.Noise.sample(c, tree, 0)
    need = p.workspace_bytes(nz)
    assert need <= p.workspace_bytes(None)
    out = np.zeros(8, np.uint64)
    st = T.lib.tqs_run(p.h, nz.h, ctypes.c_void_p(1 << 20), need - 1, None,
                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), None)
    assert st == -3 and "workspace" in T.lib.tqs_last_error().decode()
    st = T.lib.tqs_run(p.h, nz.h, ctypes.c_void_p((1 << 20) + 8), need, None,
                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), None)
    assert st == -3   # misaligned
    # noise sampled for another tree is rejected
    nz2 = T.Noise.sample(c, ([8], [0, len(wc)]), 0)
    st = T.lib.tqs_run(p.h, nz2.h, ctypes.c_void_p(1 << 20), need, None,
                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), None)
    assert st == -1


def test_histogram():
    v, c = T.histogram([5, 1, 5, 5, 0, 1])
    assert v.tolist() == [0, 1, 5] and c.tolist() == [1, 2, 3]
    v, c = T.histogram([])
    assert v.size == 0


def test_plan_passes_respect_tile_capacity():
    # every gate lands in some pass; pass counts shrink with a larger tile
    wc = W.qft(20)
    c = T.Circuit.from_workload(wc)
    tree = ([4], [0, len(wc)])
    big = 1 << 30   # no work bound: passes limited by tile capacity only
    p10 = T.Plan(c, tree, tuning={"tile_qubits": 10, "pass_cost": big}).info(0)
    p12 = T.Plan(c, tree, tuning={"tile_qubits": 12, "pass_cost": big}).info(0)
    assert p12["passes_level"] <= p10["passes_level"]
    p1 = T.Plan(c, tree, tuning={"max_ops_per_pass": 1}).info(0)
    # swap gates relabel qubit positions and take no pass of their own
    n_swap = sum(1 for q, m, _ in wc.gates if len(q) == 2 and np.array_equal(m, W.swap()))
    assert n_swap == 10
    assert p1["passes_level"] == len(wc) - n_swap


def test_swap_gates_take_no_pass():
    # a level made of swaps only still has its one (copy) pass
    wc = W.Circuit(12)
    for i in range(6):
        wc.add((i, 11 - i), W.swap())
    wc = wc.with_depolarizing(1e-3, 1e-2)
    c = T.Circuit.from_workload(wc)
    assert T.Plan(c, ([8], [0, len(wc)])).info(0)["passes_level"] == 1
    assert T.Plan(c, ([2, 2], [0, 3, len(wc)])).info(1)["passes_level"] == 1


def test_perceptron_sizes_and_argument_errors():
    # parameter count of the layout W1 b1 W2 b2 W3 b3; bad sizes fail before
    # any device work
    lib = T.lib
    assert lib.tqs_mlp_param_count(11, 128, 2) == 11 * 128 + 128 + 128 * 128 + 128 + 128 * 2 + 2
    assert lib.tqs_mlp_scratch_floats(11, 128, 2, 10) == 10 * (4 * 128 + 2 * 2 + 1)
    st = lib.tqs_mlp_forward(None, 0, 128, 2, None, 1, None, None, None)
    assert st == -1 and b"positive" in lib.tqs_last_error()
    st = lib.tqs_mlp_adam(None, None, None, None, 0, 1e-3, 0.9, 0.999, 1e-8, 1, None)
    assert st == -1


# ------------------------------------------------------ planner emulation --
def _parse_plan(text):
    lines = text.strip().split("\n")
    n = int(lines[0].split()[1])
    lay = [int(v) for v in lines[1].split()[1:]]
    gates, passes = {}, []
    for ln in lines[2:]:
        head, _, rest = ln.partition("|")
        f = head.split()
        if f[0] == "gate":
            g, p, pos, a, q0, q1 = map(int, f[1:])
            gates[g] = (p, pos, a, q0, q1)
        elif f[0] == "pass":
            passes.append([])
        elif f[0] == "dense":
            nq, p0, p1, s0, s1 = map(int, f[1:])
            v = np.array(rest.split(), float)
            m = (v[0::2] + 1j * v[1::2]).reshape(1 << nq, 1 << nq)
            passes[-1].append(("dense", s0, [(((p0, p1)[:nq]), m)]))
        elif f[0] == "diag":
            s0, s1 = int(f[1]), int(f[2])
            gl = []
            for seg in ln.split("|")[1:]:
                v = seg.split()
                nq, p0, p1 = int(v[0]), int(v[1]), int(v[2])
                d = np.array(v[3:], float)
                gl.append(((p0, p1)[:nq], np.diag(d[0::2] + 1j * d[1::2])))
            passes[-1].append(("diag", s0, gl))
    return n, lay, gates, passes


def _emulate(text, events):
    """Run the described plan gate by gate on a physical-order state, with
    each noise event (gate, code) applied at its planned position."""
    n, lay, gates, passes = _parse_plan(text)
    psi = np.zeros(1 << n, np.complex128)
    psi[0] = 1.0
    evs = sorted(((gates[g][0] << 16) | gates[g][1], i, g, c) for i, (g, c) in enumerate(events))
    k = 0

    def flush(key):
        nonlocal k
        while k < len(evs) and evs[k][0] <= key:
            _, _, g, c = evs[k]
            p, pos, a, q0, q1 = gates[g]
            oracle.apply_pauli(psi, [q0, q1][:a], c)
            k += 1

    for pi, ops in enumerate(passes):
        flush((pi << 16) - 1)
        for kind, s0, gl in ops:
            for j, (qs, m) in enumerate(gl):
                flush((pi << 16) | (s0 + j))
                oracle.apply_gate(psi, list(qs), m)
    flush(1 << 62)
    idx = [sum(((y >> q) & 1) << lay[q] for q in range(n)) for y in range(1 << n)]
    return psi[idx]


def _random_gates(n, count, rng):
    c = W.Circuit(n)
    for i in range(count):
        kind = i % 7
        if kind == 0:
            c.add((int(rng.integers(n)),), W.haar_unitary(2, rng))
        elif kind == 1:
            c.add((int(rng.integers(n)),), W.phase(float(rng.uniform(0, 6))))
        else:
            a, b = [int(x) for x in rng.choice(n, 2, replace=False)]
            m = {2: W.cphase(float(rng.uniform(0, 6))), 3: W.cx(), 4: W.haar_unitary(4, rng),
                 5: W.swap(), 6: W.rzz(float(rng.uniform(0, 6)))}[kind]
            c.add((a, b), m)
    return c


@pytest.mark.parametrize("n,tree,tuning", [
    (7, ([5], None), None),
    (8, ([3, 2], None), {"max_ops_per_pass": 3}),
    (9, ([2, 2, 2], None), None),
    (10, ([4, 2], None), {"tile_qubits": 10}),
    (10, ([3], None), {"pass_cost": 60}),
    (11, ([2, 3], None), None),
    # more qubits than one tile holds: exchanges at a level's end prepare
    # the next level's qubits
    (12, ([2, 3], None), {"tile_qubits": 10, "level_exchange": 1}),
    (12, ([3, 2], None), {"level_exchange": 1}),
    (13, ([2, 2, 2], None), {"tile_qubits": 10, "level_exchange": 1}),
    (14, ([2, 2], None), {"tile_qubits": 10, "level_exchange": 1}),
    (14, ([2, 2], None), {"tile_qubits": 10}),
])
def test_planner_schedule_reproduces_trajectories(n, tree, tuning):
    # the plan's ops in its order (gates reordered, swaps relabelled, lane
    # exchanges inserted), noise events at their planned positions, and the
    # final layout reproduce every leaf's oracle trajectory
    rng = np.random.default_rng(40 + n)
    wc = _random_gates(n, 70, rng).with_depolarizing(0.1, 0.2)
    G = len(wc)
    A = tree[0]
    cut = [round(i * G / len(A)) for i in range(len(A) + 1)]
    tr = (A, cut)
    c = T.Circuit.from_workload(wc)
    text = T.Plan(c, tr, "c64", tuning).describe()
    nz = oracle.sample_noise(wc.gates, tr, 5)
    leaves = int(np.prod(A))
    _, st = oracle.run_leaves(n, wc.gates, tr, nz, np.arange(leaves, dtype=np.uint64), states=True)
    off = np.cumsum([0] + [int(np.prod(A[:l + 1])) for l in range(len(A))])
    for lam in range(leaves):
        events = []
        for l in range(len(A)):
            node = int(off[l]) + lam // int(np.prod(A[l + 1:], dtype=np.int64))
            for e in range(int(nz.node_off[node]), int(nz.node_off[node + 1])):
                events.append((int(nz.ev_gate[e]), int(nz.ev_code[e])))
        assert np.max(np.abs(_emulate(text, events) - st[lam])) < 1e-12


def test_level_end_exchange_qft20():
    # QFT-20 cut in three levels: level 1 changes six qubits outside the lanes
    # (one more than the register slots).  With level_exchange on, level 0's
    # pass ends with a lane exchange and every level is one pass; level 1
    # changes no more than the tile holds afterwards, so its pass ends with no
    # exchange.  Off, level 1 takes two passes and no pass holds an exchange.
    # The default keeps the exchanges only when they save a tenth of the
    # passes weighted by their levels' nodes: here they save 3%, so it is off.
    wc = W.qft(20).with_depolarizing(1e-3, 1e-2)
    G = len(wc)
    cut = [0, 74, 147, G]
    c = T.Circuit.from_workload(wc)
    swap = np.eye(4)[[0, 2, 1, 3]]

    def is_exchange(op):
        kind, _, gl = op
        return kind == "dense" and len(gl[0][0]) == 2 and np.array_equal(gl[0][1], swap)

    off = T.Plan(c, ([16, 32, 32], cut), "c64", {"level_exchange": 2}).describe()
    assert [ln for ln in off.splitlines() if ln.startswith("level")] == ["level 0 0 1", "level 1 1 2",
                                                                         "level 2 3 1"]
    assert not any(is_exchange(op) for ops in _parse_plan(off)[3] for op in ops)
    assert T.Plan(c, ([16, 32, 32], cut), "c64").describe() == off
    text = T.Plan(c, ([16, 32, 32], cut), "c64", {"level_exchange": 1}).describe()
    lines = text.splitlines()
    assert [ln for ln in lines if ln.startswith("level")] == ["level 0 0 1", "level 1 1 1", "level 2 2 1"]
    n, lay, gates, passes = _parse_plan(text)
    # a lane position and a register position
    assert is_exchange(passes[0][-1])
    qs = passes[0][-1][2][0][0]
    assert min(qs) < 6 <= max(qs)
    assert not any(is_exchange(op) for op in passes[1] + passes[2])
    # the final layout is still a permutation of the 20 positions
    assert sorted(lay) == list(range(20))
    with pytest.raises(T.TqsError, match="level_exchange"):
        T.Plan(c, ([16, 32, 32], cut), "c64", {"level_exchange": 3})


@pytest.mark.parametrize("shape,expect_on", [([16, 32, 32], False), ([8, 8, 16, 16], True)])
def test_default_level_exchange_choice(shape, expect_on):
    # the default plans a tree both ways and keeps the exchanges when they
    # save at least a tenth of the passes weighted by their levels' nodes:
    # the 20-qubit brick-wall saves 28% with them in the (8, 8, 16, 16) tree,
    # none in the (16, 32, 32) tree
    wc = W.brickwall(20, 20, seed=1).with_depolarizing(1e-3, 1e-2)
    G = len(wc)
    L = len(shape)
    cut = [G * l // L for l in range(L)] + [G]
    c = T.Circuit.from_workload(wc)
    tr = (shape, cut)
    plans = {v: T.Plan(c, tr, "c64", {"level_exchange": v}) for v in (1, 2)}
    weight = {v: sum(int(np.prod(shape[:l + 1])) * p.info(l)["passes_level"] for l in range(L))
              for v, p in plans.items()}
    assert (weight[1] <= 0.9 * weight[2]) == expect_on
    assert T.Plan(c, tr, "c64").describe() == plans[1 if expect_on else 2].describe()


def test_one_hip_runtime_per_process():
    # the library binds to the HIP runtime torch loaded, so that streams and
    # device pointers from torch belong to the runtime the library calls
    maps = open("/proc/self/maps").read().splitlines()
    hip = {ln.split()[-1] for ln in maps if "libamdhip64" in ln}
    assert len(hip) == 1, hip


def test_readout_flips_match_oracle():
    # the library's sampler draws the same read-out flips as the oracle's
    wc = W.random_circuit(6, 40, seed=8, p1=0.1, p2=0.2).with_readout([0.02, 0.1, 0.3, 0.5, 0.0, 1.0])
    tree = ([4, 6, 5], [0, 10, 25, 40])
    c = T.Circuit.from_workload(wc)
    nz = T.Noise.sample(c, tree, 123)
    o = oracle.sample_noise(wc.gates, tree, 123, readout=wc.readout)
    assert _same_noise(nz.arrays(), o)
    assert np.array_equal(nz.flips(), o.leaf_flip)
    # without the channel there are no masks; explicit masks round-trip
    c.set_readout(None)
    nz2 = T.Noise.sample(c, tree, 123)
    assert nz2.flips() is None and _same_noise(nz2.arrays(), o)
    nz3 = T.Noise.from_arrays(c, tree, *nz2.arrays(), leaf_flip=o.leaf_flip)
    assert np.array_equal(nz3.flips(), o.leaf_flip)
    with pytest.raises(T.TqsError):
        c.set_readout([0.1, 0.2, 0.3, 0.4, 0.5, 1.5])
    # masks with bits beyond the circuit's qubits are refused before any run
    bad = o.leaf_flip.copy()
    bad[3] = 1 << 6
    nz4 = T.Noise.from_arrays(c, tree, *nz2.arrays(), leaf_flip=bad)
    with pytest.raises(T.TqsError, match="beyond qubit"):
        T.Plan(c, tree, "c64").workspace_bytes(nz4)


def _tiled_block_masses(text, psi_phys, b):
    """Block masses from per-tile partials built as the described plan says
    the last leaf pass writes them (lane positions, then registers), summed
    over tiles that differ in in-block positions only."""
    lines = text.strip().split("\n")
    n = int(lines[0].split()[1])
    lay = [int(v) for v in lines[1].split()[1:]]
    regs = [int(v) for v in [ln for ln in lines if ln.startswith("pass ")][-1].split()[4:]]
    head, _, rest = [ln for ln in lines if ln.startswith("sampling")][0].partition("|")
    tiled, kv, nfree, tfree, psum = map(int, head.split()[1:])
    bsrc = [int(v) for v in rest.split()]
    assert tiled == 1
    fold_l, fold_r = psum & 0xFF, (psum >> 8) & 0xFF
    fixed = [q for q in range(n) if q >= 6 and q not in regs]
    assert len(fixed) == nfree
    part = np.zeros((1 << nfree) << kv)
    p = np.abs(psi_phys) ** 2
    for x in range(1 << n):
        lane = x & 63
        tile = sum(((x >> P) & 1) << t for t, P in enumerate(fixed))
        pat, k = 0, 0
        for bb in range(6):
            if not (fold_l >> bb) & 1:
                pat |= ((lane >> bb) & 1) << k
                k += 1
        for i, P in enumerate(regs):
            if not (fold_r >> i) & 1:
                pat |= ((x >> P) & 1) << k
                k += 1
        part[(tile << kv) | pat] += p[x]
    nb = 1 << (n - b)
    S = np.zeros(nb)
    for B in range(nb):
        jv, tfix = 0, 0
        for i, src in enumerate(bsrc):
            bit = (B >> i) & 1
            if src & 0x80:
                jv |= bit << (src & 0x7F)
            else:
                tfix |= bit << src
        sub = 0
        while True:
            S[B] += part[((tfix | sub) << kv) | jv]
            sub = (sub - tfree) & tfree
            if sub == 0:
                break
    return S


@pytest.mark.parametrize("n,count,seed", [(13, 40, 1), (14, 60, 2), (12, 30, 3)])
def test_tiled_sampling_partials_give_block_masses(n, count, seed):
    # the plan's map from per-tile partials to logical blocks reproduces the
    # block masses of the logical-order state (random state, layouts moved
    # by swap gates and lane exchanges)
    rng = np.random.default_rng(seed)
    wc = _random_gates(n, count, rng)
    for i in range(n // 2):
        wc.add((i, n - 1 - i), W.swap())
    c = T.Circuit.from_workload(wc)
    G = len(wc)
    text = T.Plan(c, ([2, 2], [0, G // 2, G]), "c64", {"sample_block_log": 8}).describe()
    lay = [int(v) for v in text.split("\n")[1].split()[1:]]
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi_phys = np.zeros_like(psi)
    for y in range(1 << n):
        psi_phys[sum(((y >> q) & 1) << lay[q] for q in range(n))] = psi[y]
    S = _tiled_block_masses(text, psi_phys, 8)
    want = (np.abs(psi) ** 2).reshape(-1, 1 << 8).sum(1)
    assert np.allclose(S, want, rtol=1e-12, atol=0)


@pytest.mark.parametrize("seed", range(4))
def test_workspace_bound_holds_for_any_list(seed):
    # the list-free workspace size bounds the exact size of any list, with
    # shared states on or off and either sampling form
    rng = np.random.default_rng(seed)
    n = int(rng.integers(8, 15))
    wc = _random_gates(n, int(rng.integers(20, 60)), rng)
    G = len(wc)
    A = [int(a) for a in rng.integers(1, 6, 3)]
    tree = (A, [0, G // 3, 2 * G // 3, G])
    c = T.Circuit.from_workload(wc.with_depolarizing(0.2, 0.3))
    for tun in ({}, {"no_merge": 1}, {"separate_sampling": 1}, {"chunk_states": 2}):
        p = T.Plan(c, tree, "c64", tun)
        bound = p.workspace_bytes(None)
        for s in range(3):
            assert p.workspace_bytes(T.Noise.sample(c, tree, s)) <= bound


def test_missing_library_fails_loudly(tmp_path):
    # without the built library the binding raises at import: there is no
    # fallback path
    import shutil
    import subprocess
    import sys
    env = dict(os.environ)
    # a copy of the package without the shared library
    pkg = tmp_path / "paper_2203_13892_amd"
    shutil.copytree(os.path.join(ROOT, "paper_2203_13892_amd"), pkg,
                    ignore=shutil.ignore_patterns("*.so", "__pycache__", "csrc", "data"))
    code = "import sys; sys.path.insert(0, %r)\nimport paper_2203_13892_amd.tqsim\n" % str(tmp_path)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode != 0
    assert "libtqsim.so is not built" in r.stderr


def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    # the planner, noise sampler, importer, DCP and histogram (pure host
    # code) on random circuits, trees and tunings, built with g++ under
    # AddressSanitizer and UndefinedBehaviorSanitizer; any report aborts
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "host_sanitize")
    csrc = os.path.join(ROOT, "paper_2203_13892_amd", "csrc")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-I", csrc,
           os.path.join(csrc, "plan.cpp"), os.path.join(csrc, "host.cpp"),
           os.path.join(ROOT, "tests", "host_sanitize.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    # (another preloaded library may come before the sanitizer runtime)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0")
    r = subprocess.run([exe, "300"], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "cases 300" in r.stdout
def test_executor_host_steps_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    # the executor's host side (frames and events per node, the chunk
    # schedule with shared states and its key table, the routing of states
    # to the specialised kernels with their frame tables and generated
    # source, layout and metadata packing) on random circuits, trees, tunings and noise, with the
    # schedule's invariants checked; built by hipcc with the sanitizers on
    # the host code only (the kernels are compiled but never launched)
    import subprocess
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "executor_sanitize")
    csrc = os.path.join(ROOT, "paper_2203_13892_amd", "csrc")
    cmd = [hipcc, "--offload-arch=gfx950", "-std=c++17", "-O1", "-g", "-Xarch_device", "-O3", "-Xarch_device", "-g0",
           "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-mllvm", "-simplifycfg-sink-common=false", "-Wno-unused-command-line-argument",
           "-I", os.path.join(ROOT, "include"), "-I", csrc,
           os.path.join(ROOT, "tests", "executor_sanitize.hip"), os.path.join(csrc, "plan.cpp"),
           os.path.join(csrc, "host.cpp"), os.path.join(csrc, "jit.cpp"), "-I", os.path.dirname(build.write_jit_headers()),
           "-lrocprofiler-sdk-roctx", "-lhiprtc", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=900)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0")
    r = subprocess.run([exe, "2000"], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-1000:] + r.stderr[-2000:]
    assert "cases 2000 runs 4000 fails 0" in r.stdout, r.stdout


