"""Test infrastructure (oracle): noise channels from their Kraus operators.

Only tests, smoke() and the CPU-baseline leg of the bench use this module.
Written from the definitions, not from the closed forms the product side
uses: amplitude damping (decay probability gamma) and phase damping
(parameter lambda) as Kraus operators and thermal relaxation (T1, T2, gate
time) by its action on matrix elements (the noise models named in Sec. 4.3),
the Pauli twirl as the Pauli-diagonal part of a channel's process matrix,
p_P = sum_k |tr(P^dagger K_k)|^2 / 4, and density-matrix application of a
Kraus channel and of a Pauli channel for checks on small systems.
"""
import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], np.complex128)
Y = np.array([[0, -1j], [1j, 0]], np.complex128)
Z = np.array([[1, 0], [0, -1]], np.complex128)
PAULI = [I2, X, Y, Z]


def kraus_amplitude_damping(gamma):
    """|1> decays to |0> with probability gamma."""
    k0 = np.array([[1, 0], [0, np.sqrt(1 - gamma)]], np.complex128)
    k1 = np.array([[0, np.sqrt(gamma)], [0, 0]], np.complex128)
    return [k0, k1]


def kraus_phase_damping(lam):
    """Coherences lose a factor sqrt(1 - lambda); populations stay."""
    k0 = np.array([[1, 0], [0, np.sqrt(1 - lam)]], np.complex128)
    k1 = np.array([[0, 0], [0, np.sqrt(lam)]], np.complex128)
    return [k0, k1]


def pauli_twirl(kraus):
    """Pauli probabilities (I, X, Y, Z) of the twirled one-qubit channel."""
    return np.array([sum(abs(np.trace(P.conj().T @ K)) ** 2 for K in kraus) / 4.0 for P in PAULI])


def apply_kraus(rho, kraus):
    return sum(K @ rho @ K.conj().T for K in kraus)


def apply_pauli_channel(rho, probs):
    """One-qubit Pauli channel (I, X, Y, Z probabilities) on a 2x2 rho, or a
    two-qubit one (code c0 + 4 c1, c0 on the low qubit) on a 4x4 rho."""
    if rho.shape[0] == 2:
        return sum(p * P @ rho @ P.conj().T for p, P in zip(probs, PAULI))
    out = np.zeros_like(rho)
    for c, p in enumerate(probs):
        # index bit 0 is the first qubit: operator = P_{c1} (x) P_{c0}
        P = np.kron(PAULI[c >> 2], PAULI[c & 3])
        out += p * P @ rho @ P.conj().T
    return out


def thermal_relaxation(rho, t, T1, T2):
    """Thermal relaxation toward |0> for a time t (one qubit, T2 <= 2 T1),
    by its definition on matrix elements: the excited population decays as
    e^{-t/T1} into |0>, coherences decay as e^{-t/T2}."""
    g = 1.0 - np.exp(-t / T1)
    c = np.exp(-t / T2)
    out = np.empty_like(rho)
    out[0, 0] = rho[0, 0] + g * rho[1, 1]
    out[1, 1] = (1.0 - g) * rho[1, 1]
    out[0, 1] = c * rho[0, 1]
    out[1, 0] = c * rho[1, 0]
    return out


def pauli_twirl_of_map(f):
    """Pauli probabilities (I, X, Y, Z) of the twirl of a one-qubit linear
    map f, from its Pauli transfer diagonal lambda_Q = tr(Q f(Q)) / 2:
    p_P = (1/4) sum_Q s(P, Q) lambda_Q, s = +1 if P and Q commute, else -1."""
    lam = [np.real(np.trace(Q @ f(Q))) / 2.0 for Q in PAULI]
    out = np.zeros(4)
    for a, P in enumerate(PAULI):
        for b, Q in enumerate(PAULI):
            sgn = 1.0 if np.allclose(P @ Q, Q @ P) else -1.0
            out[a] += sgn * lam[b] / 4.0
    return out


def twirl_channel(rho, kraus):
    """The twirled channel by its definition: the average over Paulis P of
    P^dagger E(P rho P^dagger) P."""
    return sum(P.conj().T @ apply_kraus(P @ rho @ P.conj().T, kraus) @ P for P in PAULI) / 4.0
