"""Seeded synthetic workloads: circuits and noise-model parameters.

This module only *defines inputs*.  It holds none of the simulation method's
arithmetic (no state evolution, no noise sampling, no measurement), so the
product path and the test oracle can both read its output.

A circuit is ``Circuit(n, gates)``; each gate is a triple
``(qubits, matrix, probs)`` with ``matrix`` a complex128 (2^a x 2^a) array
whose local index bit j is ``qubits[j]``, and ``probs`` either None or the 4^a
Pauli-code probabilities (code = sum_j c_j 4^j, c: 0 I, 1 X, 2 Y, 3 Z).

Families follow the paper's benchmark classes (Sec. 4.2, QFT / QAOA /
quantum-volume-like random circuits); the paper's own circuit files are not
used, these are generated from their textbook definitions.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------- gate library --

H = np.array([[1, 1], [1, -1]], np.complex128) / np.sqrt(2.0)
X = np.array([[0, 1], [1, 0]], np.complex128)
Y = np.array([[0, -1j], [1j, 0]], np.complex128)
Z = np.array([[1, 0], [0, -1]], np.complex128)
I2 = np.eye(2, dtype=np.complex128)


def phase(phi: float) -> np.ndarray:
    return np.diag([1.0, np.exp(1j * phi)]).astype(np.complex128)


def rx(theta: float) -> np.ndarray:
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], np.complex128)


def rz(theta: float) -> np.ndarray:
    return np.diag([np.exp(-0.5j * theta), np.exp(0.5j * theta)]).astype(np.complex128)


def cphase(phi: float) -> np.ndarray:
    """Controlled phase on (q0, q1): diag(1, 1, 1, e^{i phi})."""
    return np.diag([1, 1, 1, np.exp(1j * phi)]).astype(np.complex128)


def cx() -> np.ndarray:
    """CNOT with control qubits[0] (local bit 0) and target qubits[1]."""
    m = np.zeros((4, 4), np.complex128)
    for l in range(4):
        c, t = l & 1, (l >> 1) & 1
        m[(c | ((t ^ c) << 1)), l] = 1.0
    return m


def swap() -> np.ndarray:
    m = np.zeros((4, 4), np.complex128)
    for l in range(4):
        m[((l & 1) << 1) | (l >> 1), l] = 1.0
    return m


def rzz(theta: float) -> np.ndarray:
    """exp(-i theta/2 Z(x)Z)."""
    d = []
    for l in range(4):
        par = (l & 1) ^ (l >> 1)
        d.append(np.exp(-0.5j * theta) if par == 0 else np.exp(0.5j * theta))
    return np.diag(d).astype(np.complex128)


def haar_unitary(dim: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random unitary: QR of a complex Ginibre matrix with the phases of
    R's diagonal moved into Q (Mezzadri 2007), scaled to determinant 1."""
    z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    q = q * (d / np.abs(d))
    det = np.linalg.det(q)
    return (q / det ** (1.0 / dim)).astype(np.complex128)


# ---------------------------------------------------------- noise models --

def depolarizing_probs(p: float, arity: int) -> np.ndarray:
    """Depolarizing channel with total non-identity probability p, spread
    uniformly over the 3 (one qubit) or 15 (two qubits) non-identity Paulis."""
    k = 1 << (2 * arity)
    pr = np.full(k, p / (k - 1), np.float64)
    pr[0] = 1.0 - p
    return pr


def pauli_probs_1q(px: float, py: float, pz: float) -> np.ndarray:
    return np.array([1.0 - px - py - pz, px, py, pz], np.float64)


def amplitude_damping_twirl(gamma: float) -> np.ndarray:
    """Pauli twirl of amplitude damping with decay probability gamma (the
    channel keeps only its Pauli-diagonal part): p_X = p_Y = gamma / 4,
    p_Z = (1 - sqrt(1 - gamma))^2 / 4, p_I = (1 + sqrt(1 - gamma))^2 / 4."""
    a = np.sqrt(1.0 - gamma)
    return np.array([(1.0 + a) ** 2 / 4.0, gamma / 4.0, gamma / 4.0, (1.0 - a) ** 2 / 4.0], np.float64)


def phase_damping_probs(lam: float) -> np.ndarray:
    """Phase damping with parameter lambda is exactly the Z channel with
    p_Z = (1 - sqrt(1 - lambda)) / 2 (it damps coherences by sqrt(1 - lambda))."""
    pz = (1.0 - np.sqrt(1.0 - lam)) / 2.0
    return np.array([1.0 - pz, 0.0, 0.0, pz], np.float64)


def thermal_relaxation_params(t: float, T1: float, T2: float):
    """(gamma, lambda) such that amplitude damping gamma followed by phase
    damping lambda is thermal relaxation over a time t: populations relax
    with e^{-t/T1}, coherences with e^{-t/T2} (requires 0 < T2 <= 2 T1)."""
    if not (T1 > 0 and 0 < T2 <= 2 * T1 and t >= 0):
        raise ValueError("need T1 > 0, 0 < T2 <= 2 T1, t >= 0")
    gamma = 1.0 - float(np.exp(-t / T1))
    # sqrt(1 - gamma) sqrt(1 - lambda) = e^{-t/T2}
    lam = 1.0 - float(np.exp(-2.0 * t / T2 + t / T1))
    return gamma, max(lam, 0.0)


# one-qubit Pauli codes (0 I, 1 X, 2 Y, 3 Z) multiply, up to phase, as their
# (x, z) bit pairs xor: I (0,0), X (1,0), Y (1,1), Z (0,1)
_CODE_XZ = [(0, 0), (1, 0), (1, 1), (0, 1)]
_XZ_CODE = {xz: c for c, xz in enumerate(_CODE_XZ)}


def _pauli_product_code(a: int, b: int, arity: int) -> int:
    out = 0
    for j in range(arity):
        ca, cb = (a >> (2 * j)) & 3, (b >> (2 * j)) & 3
        xa, za = _CODE_XZ[ca]
        xb, zb = _CODE_XZ[cb]
        out |= _XZ_CODE[(xa ^ xb, za ^ zb)] << (2 * j)
    return out


def compose_pauli_channels(p: np.ndarray, q: np.ndarray, arity: int) -> np.ndarray:
    """Probabilities of the product of independent Paulis drawn from p and
    from q (phases cancel in P rho P^dagger): the two channels in sequence."""
    k = 1 << (2 * arity)
    out = np.zeros(k, np.float64)
    for a in range(k):
        for b in range(k):
            out[_pauli_product_code(a, b, arity)] += p[a] * q[b]
    return out


def per_qubit_channel(ch: np.ndarray, arity: int) -> np.ndarray:
    """The same one-qubit Pauli channel on each of a gate's qubits
    (code c0 + 4 c1 for qubits[0], qubits[1])."""
    if arity == 1:
        return np.asarray(ch, np.float64).copy()
    return np.array([ch[c & 3] * ch[c >> 2] for c in range(16)], np.float64)


# --------------------------------------------------------------- circuits --

@dataclass
class Circuit:
    n: int
    gates: list = field(default_factory=list)
    name: str = ""
    readout: object = None  # per-qubit read-out flip probabilities, or None

    def add(self, qubits, mat, probs=None):
        self.gates.append((tuple(int(q) for q in qubits), np.asarray(mat, np.complex128),
                           None if probs is None else np.asarray(probs, np.float64)))
        return self

    def __len__(self):
        return len(self.gates)

    def with_depolarizing(self, p1: float, p2: float) -> "Circuit":
        """Copy with a depolarizing channel after every gate (p1 for one-qubit,
        p2 for two-qubit gates)."""
        out = Circuit(self.n, [], self.name)
        for q, m, _ in self.gates:
            p = p1 if len(q) == 1 else p2
            out.add(q, m, depolarizing_probs(p, len(q)) if p > 0 else None)
        out.readout = self.readout
        return out

    def with_noise(self, p1: float, p2: float, gamma: float = 0.0, lam: float = 0.0) -> "Circuit":
        """Copy with, after every gate, the depolarizing channel (p1 / p2) and
        then on each of its qubits the Pauli-twirled amplitude damping (gamma)
        and phase damping (lambda), combined into one Pauli channel."""
        ch = compose_pauli_channels(amplitude_damping_twirl(gamma), phase_damping_probs(lam), 1)
        out = Circuit(self.n, [], self.name)
        for q, m, _ in self.gates:
            a = len(q)
            dep = depolarizing_probs(p1 if a == 1 else p2, a)
            pr = compose_pauli_channels(dep, per_qubit_channel(ch, a), a)
            out.add(q, m, pr if pr[0] < 1.0 else None)
        out.readout = self.readout
        return out

    def with_thermal_relaxation(self, p1: float, p2: float, t1: float, t2: float,
                                T1: float, T2: float) -> "Circuit":
        """Copy with, after every gate, the depolarizing channel (p1 / p2) and
        then on each of its qubits the Pauli-twirled thermal relaxation over
        the gate's duration (t1 for one-qubit, t2 for two-qubit gates)."""
        out = Circuit(self.n, [], self.name)
        for q, m, _ in self.gates:
            a = len(q)
            g, lam = thermal_relaxation_params(t1 if a == 1 else t2, T1, T2)
            ch = compose_pauli_channels(amplitude_damping_twirl(g), phase_damping_probs(lam), 1)
            dep = depolarizing_probs(p1 if a == 1 else p2, a)
            pr = compose_pauli_channels(dep, per_qubit_channel(ch, a), a)
            out.add(q, m, pr if pr[0] < 1.0 else None)
        out.readout = self.readout
        return out

    def with_readout(self, r) -> "Circuit":
        """Copy with a read-out channel: bit q of each outcome flips with
        probability r[q] (a scalar applies to every qubit)."""
        out = Circuit(self.n, list(self.gates), self.name)
        out.readout = np.broadcast_to(np.asarray(r, np.float64), (self.n,)).copy()
        return out

    def noiseless(self) -> "Circuit":
        return Circuit(self.n, [(q, m, None) for q, m, _ in self.gates], self.name)

    def error_rates(self) -> np.ndarray:
        return np.array([0.0 if p is None else float(np.sum(p[1:])) for _, _, p in self.gates])


def basis_prep(n: int, x: int) -> Circuit:
    """X gates preparing |x> from |0..0> (bit q of x -> qubit q)."""
    c = Circuit(n, [], "prep%d" % x)
    for q in range(n):
        if (x >> q) & 1:
            c.add((q,), X)
    return c


def qft(n: int, swaps: bool = True, decompose: bool = False) -> Circuit:
    """Quantum Fourier transform on n qubits, little-endian:
    |x> -> 2^{-n/2} sum_y exp(2 pi i x y / 2^n) |y>.
    For j = n-1 .. 0: H(j), then CP(pi / 2^{j-m}) on (m, j) for m = j-1 .. 0;
    finally SWAP(i, n-1-i).  With ``decompose`` each CP becomes
    P(phi/2) on both qubits around two CNOTs (gate counts like basis-compiled
    benchmark circuits)."""
    c = Circuit(n, [], "qft%d" % n)
    for j in range(n - 1, -1, -1):
        c.add((j,), H)
        for m in range(j - 1, -1, -1):
            phi = np.pi / (1 << (j - m))
            if decompose:
                c.add((m,), phase(phi / 2))
                c.add((m, j), cx())
                c.add((j,), phase(-phi / 2))
                c.add((m, j), cx())
                c.add((j,), phase(phi / 2))
            else:
                c.add((m, j), cphase(phi))
    if swaps:
        for i in range(n // 2):
            c.add((i, n - 1 - i), swap())
    return c


def ghz(n: int) -> Circuit:
    """H(0) then the CNOT chain 0->1->..->n-1."""
    c = Circuit(n, [], "ghz%d" % n)
    c.add((0,), H)
    for q in range(n - 1):
        c.add((q, q + 1), cx())
    return c


def brickwall(n: int, depth: int, seed: int) -> Circuit:
    """Random brick-wall circuit: layer t applies Haar SU(4) gates on
    (2i, 2i+1) for even t and (2i+1, 2i+2) for odd t."""
    rng = np.random.default_rng(seed)
    c = Circuit(n, [], "bw%d_d%d_s%d" % (n, depth, seed))
    for t in range(depth):
        start = 0 if t % 2 == 0 else 1
        for a in range(start, n - 1, 2):
            c.add((a, a + 1), haar_unitary(4, rng))
    return c


def random_3regular(n: int, rng: np.random.Generator):
    """Random 3-regular simple graph (pairing model with rejection)."""
    if n % 2 or n < 4:
        raise ValueError("3-regular graphs need an even n >= 4")
    for _ in range(10000):
        stubs = np.repeat(np.arange(n), 3)
        rng.shuffle(stubs)
        edges = set()
        ok = True
        for i in range(0, stubs.size, 2):
            a, b = int(stubs[i]), int(stubs[i + 1])
            if a == b or (min(a, b), max(a, b)) in edges:
                ok = False
                break
            edges.add((min(a, b), max(a, b)))
        if ok:
            return sorted(edges)
    raise RuntimeError("no 3-regular graph found")


def qaoa(n: int, p: int, seed: int) -> Circuit:
    """QAOA MaxCut ansatz on a seeded random 3-regular graph: H on all
    qubits, then p rounds of RZZ(gamma) on every edge and RX(2 beta) on every
    qubit; gamma, beta uniform in [0, pi]."""
    rng = np.random.default_rng(seed)
    edges = random_3regular(n, rng)
    gam = rng.uniform(0, np.pi, p)
    bet = rng.uniform(0, np.pi, p)
    c = Circuit(n, [], "qaoa%d_p%d_s%d" % (n, p, seed))
    for q in range(n):
        c.add((q,), H)
    for r in range(p):
        for a, b in edges:
            c.add((a, b), rzz(gam[r]))
        for q in range(n):
            c.add((q,), rx(2 * bet[r]))
    return c


def random_circuit(n: int, n_gates: int, seed: int, p1: float = 0.0, p2: float = 0.0,
                   two_qubit_frac: float = 0.5) -> Circuit:
    """Random 1q/2q Haar gates on random qubits (test workload)."""
    rng = np.random.default_rng(seed)
    c = Circuit(n, [], "rand%d_%d_s%d" % (n, n_gates, seed))
    for _ in range(n_gates):
        if n >= 2 and rng.random() < two_qubit_frac:
            a, b = rng.choice(n, 2, replace=False)
            c.add((int(a), int(b)), haar_unitary(4, rng),
                  depolarizing_probs(p2, 2) if p2 > 0 else None)
        else:
            c.add((int(rng.integers(n)),), haar_unitary(2, rng),
                  depolarizing_probs(p1, 1) if p1 > 0 else None)
    return c


def concat(*cs: Circuit) -> Circuit:
    out = Circuit(cs[0].n, [], "+".join(c.name for c in cs))
    for c in cs:
        assert c.n == out.n
        out.gates.extend(c.gates)
    return out


def inverse(c: Circuit) -> Circuit:
    out = Circuit(c.n, [], c.name + "^-1")
    for q, m, p in reversed(c.gates):
        out.add(q, m.conj().T, p)
    return out
