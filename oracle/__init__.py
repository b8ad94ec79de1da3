"""CPU oracle for tree-based noisy trajectory simulation (TQSim, arXiv 2203.13892).

TEST INFRASTRUCTURE ONLY.  The product package never imports this module; only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` do.

* ``orc.c`` (built into ``liborc.so``): complex128 per-leaf trajectories, one
  gate at a time, the seeded noise insertion list, FP64 inverse-CDF sampling.
* ``density.py``: density-matrix evolution and exact Pauli-pattern enumeration
  for at most 6 qubits (numpy).
* ``tree.py``: tree arithmetic, Dynamic Circuit Partition, fidelity metrics.

A circuit is given as ``(n, gates)`` where every gate is a triple
``(qubits, matrix, probs)``: ``qubits`` a tuple of 1 or 2 qubit indices,
``matrix`` a complex (2^a x 2^a) array whose local index bit j is qubits[j],
``probs`` None (noiseless) or the 4^a Pauli-code probabilities
(code = sum_j c_j 4^j, c: 0 I, 1 X, 2 Y, 3 Z; entry 0 is the identity).
A tree is ``(arity, cut)``: arities A_0..A_{k-1} and strictly increasing
gate cuts with cut[0] = 0 and cut[k] = number of gates.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liborc.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``orc.c`` with gcc into ``liborc.so`` (plain -O2, no fast-math)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-ffp-contract=off", "-o", tmp,
                               os.path.join(_HERE, "orc.c"), "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = C.CDLL(_SO)
        u64, i64, dbl, i32 = C.c_uint64, C.c_int64, C.c_double, C.c_int
        P = C.c_void_p
        L.orc_draw.restype = u64
        L.orc_draw.argtypes = [u64, u64, u64]
        L.orc_uniform.restype = dbl
        L.orc_uniform.argtypes = [u64, u64, u64]
        L.orc_noise_count.restype = i32
        L.orc_noise_count.argtypes = [u64, i32, P, P, P, P, P, P]
        L.orc_noise_fill.restype = i32
        L.orc_noise_fill.argtypes = [u64, i32, P, P, P, P, P, P, P, P, P]
        L.orc_readout_fill.restype = i32
        L.orc_readout_fill.argtypes = [u64, i32, P, P, P, P, P, i32, P, P]
        L.orc_apply_gate.restype = None
        L.orc_apply_gate.argtypes = [i32, P, i32, P, P]
        L.orc_apply_pauli.restype = None
        L.orc_apply_pauli.argtypes = [i32, P, i32, P, i32]
        L.orc_sample_state.restype = u64
        L.orc_sample_state.argtypes = [i32, P, dbl]
        L.orc_run_leaves.restype = i32
        L.orc_run_leaves.argtypes = [i32, P, P, P, P, i32, P, P, P, P, P, P, P, u64, P, P, i32]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


@dataclass
class Flat:
    """Gate list flattened into the arrays the C oracle reads."""
    arity: np.ndarray      # int32 [G]
    qubits: np.ndarray     # int32 [2G]
    mats: np.ndarray       # float64, interleaved complex
    mat_off: np.ndarray    # int64 [G], in doubles
    probs: np.ndarray      # float64
    prob_off: np.ndarray   # int64 [G], -1 = noiseless


def flatten(gates) -> Flat:
    G = len(gates)
    arity = np.zeros(G, np.int32)
    qubits = np.zeros(2 * G, np.int32)
    mat_off = np.zeros(G, np.int64)
    prob_off = np.full(G, -1, np.int64)
    mats, probs = [], []
    mo = po = 0
    for g, (q, m, p) in enumerate(gates):
        a = len(q)
        arity[g] = a
        qubits[2 * g:2 * g + a] = q
        m = np.ascontiguousarray(np.asarray(m, np.complex128).reshape(1 << a, 1 << a))
        mats.append(m.view(np.float64).ravel())
        mat_off[g] = mo
        mo += 2 * (1 << (2 * a))
        if p is not None:
            p = np.asarray(p, np.float64).ravel()
            assert p.size == 1 << (2 * a)
            probs.append(p)
            prob_off[g] = po
            po += p.size
    mats = np.ascontiguousarray(np.concatenate(mats)) if mats else np.zeros(1)
    probs = np.ascontiguousarray(np.concatenate(probs)) if probs else np.zeros(1)
    return Flat(arity, qubits, mats, mat_off, probs, prob_off)


@dataclass
class Noise:
    """Noise insertion list in CSR form over global tree-node ids."""
    node_off: np.ndarray   # uint64 [nodes+1]
    ev_gate: np.ndarray    # uint32 [events]
    ev_code: np.ndarray    # uint8  [events]
    leaf_u: np.ndarray     # float64 [leaves]
    leaf_flip: np.ndarray = None  # uint32 [leaves] read-out flip masks, or None


def tree_arrays(tree):
    A = np.ascontiguousarray(np.asarray(tree[0], np.uint64))
    cut = np.ascontiguousarray(np.asarray(tree[1], np.uint64))
    assert cut.size == A.size + 1
    return A, cut


def n_nodes(A) -> int:
    tot, p = 0, 1
    for a in A:
        p *= int(a)
        tot += p
    return tot


def sample_noise(gates, tree, seed: int, readout=None) -> Noise:
    """The seeded insertion list (definition in the header of orc.c);
    ``readout`` (per-qubit flip probabilities, Sec. 4.3 read-out channel)
    adds each leaf's flip mask."""
    L = lib()
    f = flatten(gates)
    A, cut = tree_arrays(tree)
    nodes = n_nodes(A)
    leaves = int(np.prod([int(a) for a in A]))
    node_off = np.zeros(nodes + 1, np.uint64)
    L.orc_noise_count(seed, A.size, _p(A), _p(cut), _p(f.arity), _p(f.probs),
                      _p(f.prob_off), _p(node_off))
    ne = int(node_off[-1])
    ev_gate = np.zeros(max(ne, 1), np.uint32)
    ev_code = np.zeros(max(ne, 1), np.uint8)
    leaf_u = np.zeros(leaves, np.float64)
    L.orc_noise_fill(seed, A.size, _p(A), _p(cut), _p(f.arity), _p(f.probs),
                     _p(f.prob_off), _p(node_off), _p(ev_gate), _p(ev_code), _p(leaf_u))
    flips = None
    if readout is not None:
        r = np.ascontiguousarray(np.asarray(readout, np.float64))
        flips = np.zeros(leaves, np.uint32)
        L.orc_readout_fill(seed, A.size, _p(A), _p(cut), _p(f.arity), _p(f.probs),
                           _p(f.prob_off), r.size, _p(r), _p(flips))
    return Noise(node_off, ev_gate[:ne], ev_code[:ne], leaf_u, flips)


def run_leaves(n, gates, tree, noise: Noise, leaves=None, states=False, threads=None):
    """Simulate the listed leaves from scratch, one full trajectory each,
    and apply their read-out flips if the list has them.

    Returns (outcomes uint64 [len(leaves)], states complex128 [len, 2^n] or None).
    """
    L = lib()
    f = flatten(gates)
    A, cut = tree_arrays(tree)
    n_leaf = int(np.prod([int(a) for a in A]))
    if leaves is None:
        leaves = np.arange(n_leaf, dtype=np.uint64)
    leaves = np.ascontiguousarray(np.asarray(leaves, np.uint64))
    outcomes = np.zeros(max(leaves.size, 1), np.uint64)
    st = np.zeros((leaves.size, 1 << n), np.complex128) if states else None
    if threads is None:
        threads = max(1, min(len(os.sched_getaffinity(0)), 16))
    ev_gate = np.ascontiguousarray(noise.ev_gate, np.uint32)
    ev_code = np.ascontiguousarray(noise.ev_code, np.uint8)
    if ev_gate.size == 0:
        ev_gate, ev_code = np.zeros(1, np.uint32), np.zeros(1, np.uint8)
    node_off = np.ascontiguousarray(noise.node_off, np.uint64)
    leaf_u = np.ascontiguousarray(noise.leaf_u, np.float64)
    rc = L.orc_run_leaves(n, _p(f.arity), _p(f.qubits), _p(f.mats), _p(f.mat_off),
                          A.size, _p(A), _p(cut), _p(node_off), _p(ev_gate), _p(ev_code),
                          _p(leaf_u), _p(leaves), leaves.size, _p(outcomes),
                          _p(st) if st is not None else None, int(threads))
    if rc != 0:
        raise RuntimeError("oracle run failed")
    outcomes = outcomes[:leaves.size]
    if noise.leaf_flip is not None:
        # read-out channel: the measured bits flip after the measurement
        outcomes = outcomes ^ np.asarray(noise.leaf_flip, np.uint64)[leaves.astype(np.int64)]
    return outcomes, st


def run_events(n, gates, events=(), u: float = 0.0, state=True):
    """One trajectory of the whole circuit with an explicit event list
    [(gate, code), ...] (sorted by gate) and measurement uniform u."""
    ev = sorted(events, key=lambda e: e[0])
    noise = Noise(np.array([0, len(ev)], np.uint64),
                  np.array([e[0] for e in ev], np.uint32),
                  np.array([e[1] for e in ev], np.uint8),
                  np.array([u], np.float64))
    out, st = run_leaves(n, gates, ([1], [0, len(gates)]), noise, [0], states=state,
                         threads=1)
    return int(out[0]), (st[0] if st is not None else None)


def apply_gate(psi: np.ndarray, qubits, mat) -> None:
    """psi <- U psi in place (psi complex128 of length 2^n)."""
    L = lib()
    n = int(psi.size).bit_length() - 1
    q = np.ascontiguousarray(np.asarray(qubits, np.int32))
    m = np.ascontiguousarray(np.asarray(mat, np.complex128))
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous
    L.orc_apply_gate(n, _p(psi), q.size, _p(q), _p(m))


def apply_pauli(psi: np.ndarray, qubits, code: int) -> None:
    L = lib()
    n = int(psi.size).bit_length() - 1
    q = np.ascontiguousarray(np.asarray(qubits, np.int32))
    L.orc_apply_pauli(n, _p(psi), q.size, _p(q), int(code))


def sample_state(psi: np.ndarray, u: float) -> int:
    L = lib()
    n = int(psi.size).bit_length() - 1
    psi = np.ascontiguousarray(psi, np.complex128)
    return int(L.orc_sample_state(n, _p(psi), float(u)))


def draw(seed: int, node: int, j: int) -> int:
    return int(lib().orc_draw(seed, node, j))


def uniform(seed: int, node: int, j: int) -> float:
    return float(lib().orc_uniform(seed, node, j))
