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
