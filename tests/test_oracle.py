"""Pins of the CPU oracle against what the mathematics and the paper fix.

None of these compare the oracle with itself: closed forms (DFT, GHZ),
invariants (unitarity), an independent density-matrix implementation,
exhaustive enumeration, published generator outputs, the paper's printed tree
numbers, and binomial / chi-square statistics.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import density, tree
from paper_2203_13892_amd import workloads as W


# ------------------------------------------------------------- generator --

def test_splitmix64_published_outputs():
    # SplitMix64 seeded with 0 (Steele, Lea & Flood 2014 reference code):
    # node 0's stream is exactly that sequence.
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    assert [oracle.draw(0, 0, j) for j in range(4)] == want


def test_node_streams_are_disjoint_subsequences():
    # node nu starts 2^32 draws further along the same sequence
    assert oracle.draw(5, 1, 0) == oracle.draw(5, 0, 1 << 32)
    assert oracle.draw(5, 3, 7) == oracle.draw(5, 0, (3 << 32) + 7)


def test_uniform_range():
    u = [oracle.uniform(11, nu, j) for nu in range(20) for j in range(50)]
    assert min(u) >= 0.0 and max(u) < 1.0
    assert abs(np.mean(u) - 0.5) < 4 * math.sqrt(1 / 12 / len(u))


# ----------------------------------------------------------- gate apply --

def dft_state(n, x):
    y = np.arange(1 << n)
    return np.exp(2j * np.pi * x * y / (1 << n)) / math.sqrt(1 << n)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 10])
def test_qft_closed_form(n):
    rng = np.random.default_rng(n)
    for x in [0, 1, (1 << n) - 1, int(rng.integers(1 << n))]:
        c = W.concat(W.basis_prep(n, x), W.qft(n))
        _, psi = oracle.run_events(n, c.gates)
        assert np.max(np.abs(psi - dft_state(n, x))) < 1e-12


def test_qft_decomposed_matches_native():
    n = 6
    c1 = W.concat(W.basis_prep(n, 37), W.qft(n))
    c2 = W.concat(W.basis_prep(n, 37), W.qft(n, decompose=True))
    _, a = oracle.run_events(n, c1.gates)
    _, b = oracle.run_events(n, c2.gates)
    assert np.max(np.abs(a - b)) < 1e-12


@pytest.mark.parametrize("n", [2, 5, 9])
def test_ghz_closed_form(n):
    _, psi = oracle.run_events(n, W.ghz(n).gates)
    want = np.zeros(1 << n, np.complex128)
    want[0] = want[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(psi - want)) < 1e-14


def test_apply_gate_against_full_operator():
    # brute force: a gate equals its embedded 2^n x 2^n operator
    rng = np.random.default_rng(3)
    n = 5
    for qubits in [(0,), (4,), (2,), (0, 1), (1, 0), (3, 1), (4, 0), (2, 4)]:
        m = W.haar_unitary(1 << len(qubits), rng)
        psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
        want = density.embed(n, qubits, m) @ psi
        got = psi.copy()
        oracle.apply_gate(got, qubits, m)
        assert np.max(np.abs(got - want)) < 1e-13


def test_pauli_codes():
    # code c_j on qubits[j]: X flips, Z signs, Y = i X Z
    n = 3
    psi = np.arange(1, 9).astype(np.complex128)
    got = psi.copy()
    oracle.apply_pauli(got, (1,), 1)              # X on qubit 1
    assert np.array_equal(got, psi[np.arange(8) ^ 2])
    got = psi.copy()
    oracle.apply_pauli(got, (2,), 3)              # Z on qubit 2
    assert np.array_equal(got, psi * np.where(np.arange(8) & 4, -1, 1))
    got = psi.copy()
    oracle.apply_pauli(got, (0,), 2)              # Y on qubit 0
    y = np.arange(8)
    want = psi[y ^ 1] * np.where(y & 1, 1j, -1j)
    assert np.allclose(got, want, atol=0)
    got = psi.copy()
    oracle.apply_pauli(got, (0, 2), 1 + 4 * 3)    # X on qubit 0, Z on qubit 2
    want = psi[y ^ 1] * np.where((y & 4), -1, 1)
    assert np.array_equal(got, want)


def test_norm_preserved_by_every_gate_and_pauli():
    rng = np.random.default_rng(9)
    n = 8
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    psi /= np.linalg.norm(psi)
    c = W.random_circuit(n, 60, seed=4)
    for q, m, _ in c.gates:
        oracle.apply_gate(psi, q, m)
        assert abs(np.vdot(psi, psi).real - 1) < 1e-13
        oracle.apply_pauli(psi, q, int(rng.integers(1, 4 ** len(q))))
        assert abs(np.vdot(psi, psi).real - 1) < 1e-13


# -------------------------------------------------------------- sampling --

def test_sampling_inverse_cdf_brute_force():
    # probabilities 0.25, 0.25, 0.5, 0 on 2 qubits
    psi = np.array([0.5, 0.5j, -math.sqrt(0.5), 0], np.complex128)
    cases = {0.0: 0, 0.1: 0, 0.2499: 0, 0.25: 1, 0.3: 1, 0.49: 1, 0.5: 2, 0.99: 2,
             0.9999999999: 2}
    for u, x in cases.items():
        assert oracle.sample_state(psi, u) == x
    # unnormalised input: the CDF is scaled by the FP64 total
    assert oracle.sample_state(3 * psi, 0.3) == 1


def test_sampling_matches_distribution():
    rng = np.random.default_rng(1)
    n = 4
    psi = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    p = np.abs(psi) ** 2 / np.sum(np.abs(psi) ** 2)
    us = (np.arange(4000) + 0.5) / 4000
    counts = np.bincount([oracle.sample_state(psi, u) for u in us], minlength=16)
    # stratified uniforms: counts within 1 of 4000 p_x
    assert np.max(np.abs(counts - 4000 * p)) <= 1.0 + 1e-9


# ------------------------------------------------------------ noise list --

def test_noise_event_rates_binomial():
    n = 4
    c = W.random_circuit(n, 40, seed=2, p1=0.05, p2=0.2)
    N = 4000
    nz = oracle.sample_noise(c.gates, ([N], [0, len(c)]), seed=7)
    per_gate = np.bincount(nz.ev_gate, minlength=len(c))
    for g, (_, _, p) in enumerate(c.gates):
        pg = float(np.sum(p[1:]))
        sd = math.sqrt(N * pg * (1 - pg))
        assert abs(per_gate[g] - N * pg) < 4 * sd + 1
    # at most one event per gate per node, events sorted by gate within a node
    for nu in range(N):
        ev = nz.ev_gate[nz.node_off[nu]:nz.node_off[nu + 1]]
        assert np.all(np.diff(ev.astype(np.int64)) > 0)


def test_noise_codes_uniform_chi2():
    from scipy.stats import chi2
    c = W.Circuit(2).add((0, 1), W.cx(), W.depolarizing_probs(0.9, 2))
    nz = oracle.sample_noise(c.gates, ([20000], [0, 1]), seed=3)
    cnt = np.bincount(nz.ev_code, minlength=16)
    assert cnt[0] == 0
    obs = cnt[1:]
    exp = np.full(15, obs.sum() / 15)
    stat = float(np.sum((obs - exp) ** 2 / exp))
    assert stat < chi2.ppf(0.9999, 14)


def test_noise_zero_probability_is_ideal():
    n = 5
    c = W.concat(W.basis_prep(n, 11), W.qft(n)).with_depolarizing(0.0, 0.0)
    nz = oracle.sample_noise(c.gates, ([64], [0, len(c)]), seed=1)
    assert nz.ev_gate.size == 0
    cd = W.concat(W.basis_prep(n, 11), W.qft(n)).with_depolarizing(1e-12, 1e-12)
    nz2 = oracle.sample_noise(cd.gates, ([64], [0, len(cd)]), seed=1)
    assert nz2.ev_gate.size == 0
    # leaf uniforms do not depend on the probabilities (draw positions are fixed)
    assert np.array_equal(nz.leaf_u, nz2.leaf_u)


def test_noise_deterministic_and_seed_dependent():
    c = W.random_circuit(3, 30, seed=5, p1=0.1, p2=0.3)
    t = ([4, 5], [0, 12, 30])
    a = oracle.sample_noise(c.gates, t, 123)
    b = oracle.sample_noise(c.gates, t, 123)
    d = oracle.sample_noise(c.gates, t, 124)
    assert np.array_equal(a.ev_gate, b.ev_gate) and np.array_equal(a.leaf_u, b.leaf_u)
    assert not np.array_equal(a.leaf_u, d.leaf_u)


# ----------------------------------------------- channel / density matrix --

def test_full_depolarizing_1q_is_maximally_mixed():
    c = W.Circuit(1).add((0,), W.H, W.depolarizing_probs(0.75, 1))
    rho = density.dm_run(1, c.gates)
    assert np.max(np.abs(rho - np.eye(2) / 2)) < 1e-15


def test_full_depolarizing_2q_is_maximally_mixed():
    c = W.Circuit(2).add((0,), W.H).add((0, 1), W.cx(), W.depolarizing_probs(15 / 16, 2))
    rho = density.dm_run(2, c.gates)
    assert np.max(np.abs(rho - np.eye(4) / 4)) < 1e-15


def test_enumeration_equals_density_matrix():
    # exact Pauli-pattern mixture (C trajectories) == DM channel (numpy)
    for seed in range(3):
        c = W.random_circuit(4, 12, seed=seed)
        rng = np.random.default_rng(100 + seed)
        gates = list(c.gates)
        noisy = rng.choice(len(gates), 3, replace=False)
        for g in noisy:
            q, m, _ = gates[g]
            p = rng.dirichlet(np.ones(4 ** len(q)))
            gates[g] = (q, m, p)
        rho_dm = density.dm_run(4, gates)
        rho_en = density.enumerate_mixture(4, gates)
        assert np.max(np.abs(rho_dm - rho_en)) < 1e-12


def test_trajectory_average_converges_to_density_matrix():
    n = 4
    c = W.concat(W.ghz(n), W.random_circuit(n, 10, seed=8)).with_depolarizing(0.05, 0.1)
    M = 3000
    nz = oracle.sample_noise(c.gates, ([M], [0, len(c)]), seed=2)
    _, st = oracle.run_leaves(n, c.gates, ([M], [0, len(c)]), nz, states=True)
    p_traj = np.abs(st) ** 2
    mean = p_traj.mean(axis=0)
    se = p_traj.std(axis=0) / math.sqrt(M)
    diag = np.real(np.diag(density.dm_run(n, c.gates)))
    assert np.all(np.abs(mean - diag) <= 4 * se + 1e-12)


# ----------------------------------------------------------------- trees --

def test_tree_leaf_equals_per_shot_with_ancestor_events():
    # a leaf of a tree is one ordinary trajectory whose noise is the union of
    # its ancestors' events
    n = 5
    c = W.random_circuit(n, 24, seed=11, p1=0.2, p2=0.4)
    A, cut = [3, 2, 4], [0, 7, 15, 24]
    nz = oracle.sample_noise(c.gates, (A, cut), seed=9)
    leaves = np.arange(24)
    out, st = oracle.run_leaves(n, c.gates, (A, cut), nz, leaves, states=True)
    offs = [0, 3, 9]
    for lam in leaves:
        ev = []
        for l in range(3):
            nu = offs[l] + tree.ancestor(A, l, int(lam))
            s, e = int(nz.node_off[nu]), int(nz.node_off[nu + 1])
            ev += list(zip(nz.ev_gate[s:e].tolist(), nz.ev_code[s:e].tolist()))
        x, psi = oracle.run_events(n, c.gates, ev, u=float(nz.leaf_u[lam]))
        assert x == out[lam]
        assert np.max(np.abs(psi - st[lam])) == 0.0


def test_printed_tree_numbers():
    # Sec. 3: baseline BV tree (64,1,1) has 193 nodes with the root; DCP tree
    # (16,2,2) has 113 nodes and 64 outcomes
    assert tree.node_count([64, 1, 1]) == 193
    assert tree.node_count([16, 2, 2]) == 113
    assert tree.outcomes([16, 2, 2]) == 64
    # Sec. 3.2.1: UCP (10,10,10) simulates the subcircuits 10, 100, 1000 times
    assert tree.instances([10, 10, 10]) == [10, 100, 1000]


def test_printed_speedup_qft14():
    # Sec. 5.1: QFT_14 with 7 subcircuits and A_0 = 500: theoretical 3.53x
    A = [500] + [2] * 6
    assert tree.outcomes(A) == 32000
    assert round(tree.work_ratio_equal(A), 2) == 3.53


def test_max_speedup_formula_matches_tree():
    # Sec. 3.6: (1, .., 1, N) with k equal subcircuits gives kN / ((k-1) + N)
    for k, N in [(2, 1000), (3, 32000), (7, 50)]:
        A = [1] * (k - 1) + [N]
        assert abs(tree.work_ratio_equal(A) - tree.max_speedup_equal(k, N)) < 1e-12


# ------------------------------------------------------------------- DCP --

def test_sample_size_cochran():
    # p = 0.5, z = 1.96, eps = 0.05, infinite population: 384.16
    assert abs(tree.sample_size(0.5, 1.96, 0.05) - 384.16) < 1e-9
    # finite-population correction
    n0 = 384.16
    assert abs(tree.sample_size(0.5, 1.96, 0.05, 1000) - n0 / (1 + n0 / 1000)) < 1e-9


def test_first_error_rate():
    assert abs(tree.first_error_rate([0.1, 0.2]) - (1 - 0.9 * 0.8)) < 1e-15
    assert tree.first_error_rate([]) == 0.0


def test_dcp_printed_shapes():
    # Sec. 5.6: QPE_9 with 1000 shots -> (250, 2, 2)
    for a0 in (126, 200, 250):
        A, cut = tree.dcp([1e-3] * 120, 1000, copy_cost=8, A0_min=a0)
        assert A == [250, 2, 2]
    # Sec. 5.1: QFT_14 with 32000 shots -> 7 subcircuits, A_0 = 500
    for a0 in (251, 400, 500):
        A, cut = tree.dcp([1e-3] * 472, 32000, copy_cost=8, A0_min=a0)
        assert A == [500] + [2] * 6
        assert len(cut) == 8 and cut[0] == 0 and cut[-1] == 472


def test_dcp_reproduces_shapes_from_error_rates():
    # z = 1.96, eps = 0.01 and 0.1% gate error: first subcircuits of a few
    # gates give both printed shapes
    A, _ = tree.dcp([1e-3] * 120, 1000, z=1.96, eps=0.01, copy_cost=6)
    assert A == [250, 2, 2]
    A, _ = tree.dcp([1e-3] * 472, 32000, z=1.96, eps=0.01, copy_cost=8)
    assert A == [500] + [2] * 6


def test_dcp_invariants():
    rng = np.random.default_rng(0)
    for _ in range(200):
        G = int(rng.integers(1, 400))
        N = int(rng.integers(1, 100000))
        e = rng.uniform(0, 0.02, G)
        C = float(rng.uniform(0, 30))
        A, cut = tree.dcp(e, N, copy_cost=C, max_levels=int(rng.integers(1, 9)))
        assert tree.outcomes(A) >= N
        assert cut[0] == 0 and cut[-1] == G and all(b > a for a, b in zip(cut, cut[1:]))
        assert len(cut) == len(A) + 1
        if len(A) > 1:
            assert all(a == A[1] for a in A[1:]) and A[1] >= 2
            # A_0 is the smallest first arity reaching N outcomes
            assert (A[0] - 1) * A[1] ** (len(A) - 1) < N


# -------------------------------------------------------------- fidelity --

def test_fidelity_metrics():
    p = np.array([0.5, 0.5, 0, 0])
    assert abs(tree.fidelity_s(p, p) - 1) < 1e-15
    assert abs(tree.fidelity_norm(p, p) - 1) < 1e-15
    assert abs(tree.fidelity_norm(p, np.full(4, 0.25))) < 1e-15
    assert math.isnan(tree.fidelity_norm(np.full(4, 0.25), p))
    assert tree.tv_distance(p, np.array([0, 0, 0.5, 0.5])) == 1.0


# ------------------------------------------------------------ channels --
def _random_rho(d, rng):
    a = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    r = a @ a.conj().T
    return r / np.trace(r)


@pytest.mark.parametrize("gamma", [0.0, 1e-3, 0.02, 0.3, 1.0])
def test_amplitude_damping_twirl_from_kraus(gamma):
    from oracle import channels as ch
    tw = ch.pauli_twirl(ch.kraus_amplitude_damping(gamma))
    assert np.allclose(tw, W.amplitude_damping_twirl(gamma), atol=1e-15)
    assert abs(tw.sum() - 1.0) < 1e-14
    # the twirled channel by its definition acts as this Pauli channel
    rng = np.random.default_rng(int(gamma * 1000) + 1)
    rho = _random_rho(2, rng)
    assert np.allclose(ch.twirl_channel(rho, ch.kraus_amplitude_damping(gamma)),
                       ch.apply_pauli_channel(rho, tw), atol=1e-14)


@pytest.mark.parametrize("lam", [0.0, 1e-3, 0.05, 0.5, 1.0])
def test_phase_damping_is_a_z_channel(lam):
    from oracle import channels as ch
    rng = np.random.default_rng(int(lam * 1000) + 7)
    rho = _random_rho(2, rng)
    # phase damping needs no twirl: it already is this Z channel, exactly
    assert np.allclose(ch.apply_kraus(rho, ch.kraus_phase_damping(lam)),
                       ch.apply_pauli_channel(rho, W.phase_damping_probs(lam)), atol=1e-14)
    assert np.allclose(ch.pauli_twirl(ch.kraus_phase_damping(lam)), W.phase_damping_probs(lam), atol=1e-15)


def test_composed_pauli_channels_act_in_sequence():
    from oracle import channels as ch
    rng = np.random.default_rng(5)
    for arity in (1, 2):
        k = 4 ** arity
        p = rng.random(k); p /= p.sum()
        q = rng.random(k); q /= q.sum()
        rho = _random_rho(2 ** arity, rng)
        seq = ch.apply_pauli_channel(ch.apply_pauli_channel(rho, p), q)
        assert np.allclose(ch.apply_pauli_channel(rho, W.compose_pauli_channels(p, q, arity)), seq, atol=1e-14)
    # the per-qubit product is the channel on each qubit in turn
    c1 = W.amplitude_damping_twirl(0.1)
    rho = _random_rho(4, rng)
    two = ch.apply_pauli_channel(rho, W.per_qubit_channel(c1, 2))
    one_each = ch.apply_pauli_channel(rho, np.array([c1[c & 3] * (c >> 2 == 0) for c in range(16)]))
    one_each = ch.apply_pauli_channel(one_each, np.array([c1[c >> 2] * (c & 3 == 0) for c in range(16)]))
    assert np.allclose(two, one_each, atol=1e-14)


def test_damped_circuit_trajectories_match_density_matrix():
    # noise = depolarizing, then twirled amplitude damping and phase damping
    # per qubit: trajectory average of |psi|^2 = density-matrix diagonal
    from oracle import density
    wc = W.brickwall(4, 4, seed=2).with_noise(0.02, 0.05, gamma=0.2, lam=0.1)
    rho = density.dm_run(wc.n, wc.gates)
    tree = ([3000], [0, len(wc)])
    nz = oracle.sample_noise(wc.gates, tree, 11)
    _, st = oracle.run_leaves(wc.n, wc.gates, tree, nz, states=True)
    mean = np.mean(np.abs(st) ** 2, axis=0)
    sd = np.std(np.abs(st) ** 2, axis=0) / np.sqrt(st.shape[0])
    assert np.all(np.abs(mean - np.real(np.diag(rho))) <= 4 * sd + 1e-12)


# ---------------------------------------------------- shape perceptron --
def test_perceptron_gradient_matches_finite_differences():
    from oracle import mlp
    rng = np.random.default_rng(3)
    d_in, h, d_out, B = 5, 7, 2, 9
    n = sum(int(np.prod(s)) for s in mlp.sizes(d_in, h, d_out))
    p = rng.normal(size=n) * 0.5
    x = rng.normal(size=(B, d_in))
    t = rng.normal(size=(B, d_out))
    w = np.array([1.0, 0.3])
    L, g = mlp.loss_grad(p, x, t, w, d_in, h, d_out)
    assert abs(L - mlp.loss(p, x, t, w, d_in, h, d_out)) < 1e-14
    eps = 1e-6
    fd = np.array([(mlp.loss(p + eps * e, x, t, w, d_in, h, d_out) - mlp.loss(p - eps * e, x, t, w, d_in, h, d_out))
                   / (2 * eps) for e in np.eye(n)])
    assert np.max(np.abs(fd - g)) < 1e-7 * max(1.0, np.max(np.abs(g)))


def test_perceptron_linear_regime_closed_form():
    # with every pre-activation positive the network is affine in x, and a
    # one-output squared error has the textbook gradient 2/B sum (y - t) dy/dp
    from oracle import mlp
    d_in, h, d_out = 2, 3, 1
    W1 = np.array([[1.0, 0.5, 0.2], [0.3, 1.0, 0.1]]); b1 = np.ones(3)
    W2 = np.eye(3) * 2.0; b2 = np.ones(3)
    W3 = np.array([[1.0], [-1.0], [0.5]]); b3 = np.array([0.25])
    p = mlp.pack([W1, b1, W2, b2, W3, b3])
    x = np.array([[1.0, 2.0], [0.5, 0.0]])
    y = mlp.forward(p, x, d_in, h, d_out)
    want = ((x @ W1 + b1) @ W2 + b2) @ W3 + b3
    assert np.allclose(y, want, atol=1e-14)
    t = np.zeros((2, 1))
    L, g = mlp.loss_grad(p, x, t, np.ones(1), d_in, h, d_out)
    assert abs(L - np.mean(want[:, 0] ** 2)) < 1e-12
    # gradient wrt b3 is 2 mean(y - t)
    assert abs(g[-1] - 2 * np.mean(want[:, 0])) < 1e-12


def test_adam_first_step_moves_by_lr():
    # after bias correction the first step is lr * g / (|g| + eps)
    from oracle import mlp
    g = np.array([0.5, -2.0, 1e-3])
    p1, m, v = mlp.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p1, -0.01 * g / (np.abs(g) + 1e-8), atol=1e-12)


# ------------------------------------------------------- read-out channel --

def test_readout_extremes_and_unchanged_streams():
    # r = 0 flips nothing, r = 1 flips every bit; the read-out draws come
    # after every other draw of a leaf, so events and measurement uniforms
    # are those of the same list without read-out
    n, x = 5, 0b10110
    wc = W.concat(W.basis_prep(n, x), W.qft(n), W.inverse(W.qft(n))).with_depolarizing(0.0, 0.0)
    tree = ([4, 8], [0, 10, len(wc)])
    base = oracle.sample_noise(wc.gates, tree, 5)
    for r, mask in ((0.0, 0), (1.0, (1 << n) - 1)):
        nz = oracle.sample_noise(wc.gates, tree, 5, readout=[r] * n)
        assert np.array_equal(nz.node_off, base.node_off) and np.array_equal(nz.leaf_u, base.leaf_u)
        assert np.all(nz.leaf_flip == mask)
        out, _ = oracle.run_leaves(n, wc.gates, tree, nz)
        assert np.all(out == (x ^ mask))


def test_readout_draw_positions():
    # leaf nu's flips are its draws j0 .. j0+n-1 with j0 = gates of its
    # subcircuit (one uniform each) + its events (one more each) + 1
    wc = W.random_circuit(4, 30, seed=3, p1=0.2, p2=0.3)
    tree = ([3, 5], [0, 12, 30])
    r = np.array([0.1, 0.5, 0.3, 0.9])
    seed = 77
    nz = oracle.sample_noise(wc.gates, tree, seed, readout=r)
    first_leaf = 3
    for m in range(15):
        nu = first_leaf + m
        ne = int(nz.node_off[nu + 1] - nz.node_off[nu])
        j0 = (30 - 12) + ne + 1
        want = sum(1 << q for q in range(4) if oracle.uniform(seed, nu, j0 + q) < r[q])
        assert int(nz.leaf_flip[m]) == want


def test_readout_histogram_matches_confusion_of_density_matrix():
    # trajectories with read-out flips sample p'(y) = sum_x p(x) prod_q
    # (r_q if x_q != y_q else 1 - r_q), p = diagonal of the noisy density
    # matrix (an implementation independent of the trajectory code)
    wc = W.brickwall(3, 3, seed=4).with_depolarizing(0.05, 0.1).with_readout([0.05, 0.2, 0.35])
    rho = density.dm_run(wc.n, wc.gates)
    p = np.real(np.diag(rho))
    d = 1 << wc.n
    conf = np.ones((d, d))
    for y in range(d):
        for x in range(d):
            for q in range(wc.n):
                conf[y, x] *= wc.readout[q] if ((x ^ y) >> q) & 1 else 1 - wc.readout[q]
    want = conf @ p
    S = 20000
    tree = ([S], [0, len(wc)])
    nz = oracle.sample_noise(wc.gates, tree, 9, readout=wc.readout)
    out, _ = oracle.run_leaves(wc.n, wc.gates, tree, nz)
    cnt = np.bincount(out.astype(np.int64), minlength=d)
    sd = np.sqrt(S * want * (1 - want))
    assert np.all(np.abs(cnt - S * want) <= 5 * sd + 1)
    # and the flip masks alone: bit q set with rate r_q, bits independent
    f = nz.leaf_flip
    for q in range(wc.n):
        k = int(np.sum((f >> q) & 1))
        assert abs(k - S * wc.readout[q]) <= 5 * math.sqrt(S * wc.readout[q] * (1 - wc.readout[q]))
    both = int(np.sum((f & 3) == 3))
    r01 = wc.readout[0] * wc.readout[1]
    assert abs(both - S * r01) <= 5 * math.sqrt(S * r01 * (1 - r01))


@pytest.mark.parametrize("t,T1,T2", [(0.0, 20.0, 15.0), (0.05, 20.0, 15.0), (0.5, 10.0, 20.0),
                                     (2.0, 5.0, 1.0), (1.0, 3.0, 6.0)])
def test_thermal_relaxation_is_damping_in_sequence(t, T1, T2):
    # thermal relaxation by its definition equals amplitude damping then
    # phase damping with the parameters the workloads derive, and its twirl
    # (from the Pauli transfer diagonal) is their composed Pauli channel
    from oracle import channels as ch
    g, lam = W.thermal_relaxation_params(t, T1, T2)
    rng = np.random.default_rng(int(t * 100 + T1))
    rho = _random_rho(2, rng)
    seq = ch.apply_kraus(ch.apply_kraus(rho, ch.kraus_amplitude_damping(g)), ch.kraus_phase_damping(lam))
    assert np.allclose(ch.thermal_relaxation(rho, t, T1, T2), seq, atol=1e-14)
    tw = ch.pauli_twirl_of_map(lambda r: ch.thermal_relaxation(r, t, T1, T2))
    want = W.compose_pauli_channels(W.amplitude_damping_twirl(g), W.phase_damping_probs(lam), 1)
    assert np.allclose(tw, want, atol=1e-14)
    # t = 0 is the identity channel
    if t == 0.0:
        assert np.allclose(tw, [1, 0, 0, 0])


def test_thermal_relaxation_circuit_trajectories_match_density_matrix():
    from oracle import density
    wc = W.brickwall(4, 4, seed=5).with_thermal_relaxation(0.01, 0.02, 0.05, 0.3, 8.0, 6.0)
    rho = density.dm_run(wc.n, wc.gates)
    tree = ([3000], [0, len(wc)])
    nz = oracle.sample_noise(wc.gates, tree, 12)
    _, st = oracle.run_leaves(wc.n, wc.gates, tree, nz, states=True)
    mean = np.mean(np.abs(st) ** 2, axis=0)
    sd = np.std(np.abs(st) ** 2, axis=0) / np.sqrt(st.shape[0])
    assert np.all(np.abs(mean - np.real(np.diag(rho))) <= 4 * sd + 1e-12)
