"""Density-matrix oracle and exact Pauli-pattern enumeration (n <= 6).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``dm_run`` evolves the mixed state rho under each gate and then under that
  gate's Pauli channel, rho <- sum_c p_c P_c rho P_c^dagger (Sec. 2.3.1: the
  density-matrix formalism, O(4^n) memory, hence the 6-qubit limit).
* ``enumerate_mixture`` forms the exact average over every Pauli pattern the
  trajectories can draw, each pattern simulated by the C trajectory oracle.
  Agreement of the two (to rounding) pins the trajectory code against an
  independent implementation of the same channel (Sec. 2.4.1: trajectories
  converge to the density matrix).
"""
from __future__ import annotations

import itertools

import numpy as np

from . import run_events

MAX_QUBITS = 6

_P1 = [np.eye(2, dtype=np.complex128),
       np.array([[0, 1], [1, 0]], np.complex128),
       np.array([[0, -1j], [1j, 0]], np.complex128),
       np.array([[1, 0], [0, -1]], np.complex128)]


def embed(n: int, qubits, mat) -> np.ndarray:
    """The full 2^n x 2^n operator of a gate, written from its definition:
    <y|U|x> = mat[l(y), l(x)] when y and x agree off the gate's qubits, where
    l(.) collects bit qubits[j] into local bit j; 0 otherwise."""
    mat = np.asarray(mat, np.complex128)
    dim = 1 << n
    mask = 0
    for q in qubits:
        mask |= 1 << q
    U = np.zeros((dim, dim), np.complex128)

    def local(x):
        return sum(((x >> q) & 1) << j for j, q in enumerate(qubits))

    for y in range(dim):
        for x in range(dim):
            if (x & ~mask) == (y & ~mask):
                U[y, x] = mat[local(y), local(x)]
    return U


def pauli_matrix(arity: int, code: int) -> np.ndarray:
    """Local 2^a x 2^a matrix of a Pauli code (local bit j <- factor j)."""
    m = np.ones((1, 1), np.complex128)
    for j in range(arity):
        c = (code >> (2 * j)) & 3
        m = np.kron(_P1[c], m)  # factor j acts on local bit j
    return m


def dm_run(n: int, gates) -> np.ndarray:
    """Final density matrix of the noisy circuit, starting from |0..0>."""
    if n > MAX_QUBITS:
        raise ValueError("density-matrix oracle limited to %d qubits" % MAX_QUBITS)
    dim = 1 << n
    rho = np.zeros((dim, dim), np.complex128)
    rho[0, 0] = 1.0
    for q, m, p in gates:
        U = embed(n, q, m)
        rho = U @ rho @ U.conj().T
        if p is not None:
            p = np.asarray(p, np.float64)
            new = np.zeros_like(rho)
            for c, pc in enumerate(p):
                if pc == 0.0:
                    continue
                P = embed(n, q, pauli_matrix(len(q), c))
                new += pc * (P @ rho @ P.conj().T)
            rho = new
    return rho


def enumerate_mixture(n: int, gates, max_noisy: int = 6) -> np.ndarray:
    """Exact mixture over all Pauli patterns (the trajectory ensemble's limit).

    Each pattern picks one code per noisy gate (identity included) with
    probability prod p_g[c_g]; its pure state comes from the C trajectory
    oracle with the matching explicit event list."""
    noisy = [g for g, (_, _, p) in enumerate(gates) if p is not None]
    if len(noisy) > max_noisy:
        raise ValueError("too many noisy gates to enumerate")
    dim = 1 << n
    rho = np.zeros((dim, dim), np.complex128)
    choices = [range(len(gates[g][2])) for g in noisy]
    for pattern in itertools.product(*choices):
        w = 1.0
        ev = []
        for g, c in zip(noisy, pattern):
            w *= float(gates[g][2][c])
            if c:
                ev.append((g, c))
        if w == 0.0:
            continue
        _, psi = run_events(n, gates, ev)
        rho += w * np.outer(psi, psi.conj())
    return rho
