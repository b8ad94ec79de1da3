"""Learned tree-shape choice: a perceptron that predicts, for a circuit,
its noise, a shot count and a candidate tree shape, the run time per shot
on this GPU and the design effect of the tree's fidelity estimate; it picks
the fastest candidate whose predicted design effect stays within a bound and
falls back to the Dynamic Circuit Partition heuristic (Sec. 3.2) when the
circuit lies outside what it was trained on or no candidate qualifies.

The network runs in the library's own kernels (``tqsim.Perceptron``:
forward, back-propagation and Adam in HIP).  Its training set is made of the
simulator's own runs: the time of each run and, from the run's outcomes, the
design effect deff = Var(tree estimate) / Var(per-shot estimate) of the
mean linear cross-entropy score s = 2^n p_ideal(x) - 1, with the tree's
variance taken over its independent level-0 subtrees.  (Sec. 3.1: the
leaves of one level-0 subtree share their ancestors' noise, so they are not
independent; per-shot sampling has deff = 1.)
"""
from __future__ import annotations

import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL = os.path.join(HERE, "data", "shape_mlp.npz")

CIRCUIT_FEATURES = ("qubits", "gates_1q", "gates_2q", "depth", "err_1q", "err_2q", "log_events", "log2_shots")
SHAPE_FEATURES = ("levels", "log2_root", "log2_branch_mean", "log2_branch_last", "log2_leaves_per_root")
N_IN = len(CIRCUIT_FEATURES) + len(SHAPE_FEATURES)
HIDDEN = 128
OUTPUTS = ("log_s_per_shot_amp", "log_deff")  # log(seconds per shot / 2^n), log(design effect)


# ---------------------------------------------------------------- features --

def circuit_features(wc, shots: int) -> np.ndarray:
    """qubits, 1q / 2q gate counts, depth (greedy layering), mean 1q / 2q
    error rate, log of the expected noise events per trajectory (sum of the
    gates' error rates), log2 shots."""
    n = wc.n
    g1 = g2 = 0
    e1, e2 = [], []
    front = [0] * n
    for q, _, p in wc.gates:
        err = 0.0 if p is None else float(np.sum(p[1:]))
        if len(q) == 1:
            g1 += 1
            e1.append(err)
        else:
            g2 += 1
            e2.append(err)
        lvl = max(front[x] for x in q) + 1
        for x in q:
            front[x] = lvl
    depth = max(front) if front else 0
    events = float(np.sum(e1) + np.sum(e2))
    return np.array([n, g1, g2, depth, np.mean(e1) if e1 else 0.0, np.mean(e2) if e2 else 0.0,
                     math.log(events + 1e-6), math.log2(max(shots, 1))], np.float64)


def shape_features(shape) -> np.ndarray:
    a = [int(x) for x in shape]
    rest = a[1:]
    return np.array([len(a), math.log2(a[0]),
                     float(np.mean([math.log2(x) for x in rest])) if rest else 0.0,
                     math.log2(rest[-1]) if rest else 0.0,
                     float(sum(math.log2(x) for x in rest))], np.float64)


def equal_cuts(G: int, levels: int):
    sizes = [G // levels + (1 if i < G % levels else 0) for i in range(levels)]
    cut = [0]
    for s in sizes:
        cut.append(cut[-1] + s)
    return cut


def candidate_shapes(shots: int, G: int, max_levels: int = 4):
    """Per-shot, and trees of 2..max_levels levels with equal branching b
    (2..32) below a root arity ceil(shots / b^(k-1)), plus two-factor mixes;
    every subcircuit gets at least one gate."""
    out = [[shots]]
    for k in range(2, max_levels + 1):
        if k > G:
            break
        for b in (2, 4, 8, 16, 32):
            root = -(-shots // b ** (k - 1))
            if root < 2:  # the design effect needs independent subtrees
                continue
            out.append([root] + [b] * (k - 1))
            if k >= 3:
                for b2 in (2, 4, 8, 16, 32):
                    if b2 != b:
                        r2 = -(-shots // (b ** (k - 2) * b2))
                        if r2 >= 2:
                            out.append([r2] + [b] * (k - 2) + [b2])
    uniq = []
    for s in out:
        if s not in uniq:
            uniq.append(s)
    return uniq


# ------------------------------------------------------------ measurement --

def ideal_probs(T, wc) -> np.ndarray:
    """|psi_ideal|^2 of the noiseless circuit, from one captured GPU run."""
    c = T.Circuit.from_workload(wc.noiseless())
    G = len(wc)
    plan = T.Plan(c, ([1], [0, G]), "c64")
    nz = T.Noise.sample(c, ([1], [0, G]), 0)
    _, amps = T.run_capture(plan, nz, [0])
    return np.abs(amps[0]) ** 2


def design_effect(scores: np.ndarray, root: int) -> float:
    """Var of the mean over independent level-0 subtrees against the
    independent-sample variance of the same scores (leaves are ordered by
    subtree, each subtree holding the same number of leaves)."""
    N = scores.size
    v = scores.var(ddof=1)
    if root <= 1 or v <= 0:
        return float("nan")
    if root == N:
        return 1.0
    means = scores.reshape(root, N // root).mean(1)
    return float((means.var(ddof=1) / root) / (v / N))


def measure(T, torch, wc, circuit, shape, shots, p_ideal, seed, ws=None, cut=None):
    """One timed run of `shape` (with `cut` as given, else equal cuts);
    returns (seconds per leaf, design effect of the cross-entropy score over
    all leaves)."""
    G = len(wc)
    tree = (list(shape), list(cut) if cut is not None else equal_cuts(G, len(shape)))
    plan = T.Plan(circuit, tree, "c64")
    nz = T.Noise.sample(circuit, tree, seed)
    need = plan.workspace_bytes(nz)
    if ws is None or ws.nbytes < need:
        ws = T.Workspace(need)
    torch.cuda.synchronize()
    out, st = T.run(plan, nz, ws, stats=True)
    leaves = out.size
    s = (2.0 ** wc.n) * p_ideal[out.astype(np.int64)] - 1.0
    return st["ms_device"] * 1e-3 / leaves, design_effect(s, int(shape[0])), ws


# ------------------------------------------------------------------ model --

class ShapeModel:
    """Feature scaling plus the perceptron (library kernels)."""

    def __init__(self, T, params=None, mu=None, sd=None, out_mu=None, out_sd=None, train_range=None, seed=0):
        self.T = T
        self.net = T.Perceptron(N_IN, HIDDEN, len(OUTPUTS), params=params, seed=seed)
        self.mu = np.zeros(N_IN) if mu is None else np.asarray(mu, np.float64)
        self.sd = np.ones(N_IN) if sd is None else np.asarray(sd, np.float64)
        self.out_mu = np.zeros(len(OUTPUTS)) if out_mu is None else np.asarray(out_mu, np.float64)
        self.out_sd = np.ones(len(OUTPUTS)) if out_sd is None else np.asarray(out_sd, np.float64)
        self.train_range = train_range  # (min, max) per circuit feature

    @staticmethod
    def load(T, path=MODEL):
        z = np.load(path, allow_pickle=False)
        return ShapeModel(T, z["params"], z["mu"], z["sd"], z["out_mu"], z["out_sd"],
                          (z["range_lo"], z["range_hi"]))

    def save(self, path=MODEL):
        os.makedirs(os.path.dirname(path), exist_ok=True)
        lo, hi = self.train_range
        np.savez(path, params=self.net.params.cpu().numpy(), mu=self.mu, sd=self.sd, out_mu=self.out_mu,
                 out_sd=self.out_sd, range_lo=lo, range_hi=hi)

    def _x(self, feats):
        return ((np.asarray(feats, np.float64) - self.mu) / self.sd).astype(np.float32)

    def predict(self, feats) -> np.ndarray:
        y = self.net.forward(self._x(feats)).cpu().numpy().astype(np.float64)
        return y * self.out_sd + self.out_mu

    def fit(self, X, Y, steps=3000, batch=256, lr=2e-3, seed=0, log=None):
        """Adam on the weighted squared error of standardised targets, every
        step in the library's kernels; returns the final full-set loss."""
        X = np.asarray(X, np.float64)
        Y = np.asarray(Y, np.float64)
        self.mu, self.sd = X.mean(0), X.std(0) + 1e-9
        self.out_mu, self.out_sd = Y.mean(0), Y.std(0) + 1e-9
        lo = X[:, :len(CIRCUIT_FEATURES)].min(0)
        hi = X[:, :len(CIRCUIT_FEATURES)].max(0)
        self.train_range = (lo, hi)
        xs = self._x(X)
        ys = ((Y - self.out_mu) / self.out_sd).astype(np.float32)
        w = np.ones(len(OUTPUTS), np.float32)
        rng = np.random.default_rng(seed)
        for it in range(steps):
            idx = rng.integers(0, xs.shape[0], min(batch, xs.shape[0]))
            loss = self.net.loss_grad(xs[idx], ys[idx], w)
            self.net.adam(lr=lr * (0.5 ** (it // 1000)))
            if log is not None and (it % 500 == 0 or it == steps - 1):
                log(it, float(loss.cpu()))
        return float(self.net.loss_grad(xs, ys, w).cpu())

    def in_range(self, cf, margin=(6, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0)) -> bool:
        """Circuit features within the training range, widened by a margin
        (in units of the feature's training spread for all but qubits)."""
        if self.train_range is None:
            return False
        lo, hi = self.train_range
        span = np.maximum(hi - lo, 1e-9)
        for i, v in enumerate(cf):
            m = margin[i] if i == 0 else margin[i] * span[i]
            if v < lo[i] - m or v > hi[i] + m:
                return False
        return True


def choose_shape(T, model, wc, shots, copy_cost=1.0, max_deff=4.0, max_levels=4, deff_margin=0.8):
    """The learned choice: the candidate with the smallest predicted time per
    shot among those whose predicted log design effect plus deff_margin (about
    twice the model's error on its training runs) stays <= log(max_deff); the
    DCP tree (at `copy_cost` gates per branch copy: about one here, where the
    copy rides in the child's first pass) when the model is missing, the
    circuit is out of its range or no candidate qualifies.  Returns
    ((arities, cuts), source)."""
    G = len(wc)
    circuit = T.Circuit.from_workload(wc)

    def dcp():
        return T.dcp(circuit, shots, 1.96, 0.01, copy_cost, 8), "dcp"

    if model is None:
        return dcp()
    cf = circuit_features(wc, shots)
    if not model.in_range(cf):
        return dcp()
    cands = candidate_shapes(shots, G, max_levels)
    feats = np.array([np.concatenate([cf, shape_features(s)]) for s in cands])
    pred = model.predict(feats)
    ok = [i for i in range(len(cands)) if pred[i, 1] + deff_margin <= math.log(max_deff)]
    if not ok:
        return dcp()
    best = min(ok, key=lambda i: pred[i, 0])
    s = cands[best]
    return (s, equal_cuts(G, len(s))), "learned"


# ------------------------------------------------------------- evaluation --

def held_out_circuits(n=24):
    """Circuits of a size the model never saw: a depth-24 brick-wall, QAOA
    p = 2 on a random 3-regular graph, and the QFT round trip from a basis
    state at n qubits, and QAOA p = 2 at n + 2 qubits, with depolarizing
    p1 = 1e-3, p2 = 1e-2."""
    from . import workloads as W
    x = 0xA5A5A5 & ((1 << n) - 1)
    return [("brickwall%d" % n, W.brickwall(n, 24, seed=7).with_noise(1e-3, 1e-2)),
            ("qaoa%d" % n, W.qaoa(n, 2, seed=7).with_noise(1e-3, 1e-2)),
            ("qft%d_roundtrip" % n, W.concat(W.basis_prep(n, x), W.qft(n),
                                             W.inverse(W.qft(n))).with_noise(1e-3, 1e-2)),
            ("qaoa%d" % (n + 2), W.qaoa(n + 2, 2, seed=7).with_noise(1e-3, 1e-2))]


def evaluate(T, torch, model, circuits, shots=16384, copy_cost=26.0, max_deff=4.0, seed=0, log=print):
    """Per-shot (the exact reference), two DCP trees and the learned shape on
    each circuit: measured time, and the normalised linear fidelity
    F = (mean p_ideal(x) - 2^-n) / (sum p_ideal^2 - 2^-n) (1 for the ideal
    output, 0 for the uniform one; for a single ideal outcome it is the
    normalised fidelity of Sec. 4.1) with its standard error, clustered over
    level-0 subtrees for trees.

    The DCP trees are the heuristic's own (arities and cuts, Sec. 3.2) at two
    copy costs: `copy_cost` gates ("dcp", a state copy as a separate
    kernel) and one gate ("dcp_fused": this library copies the parent's
    state inside the child's first pass, so a branch costs about one gate
    of memory traffic).  The learned gain is stated against both."""
    out = []
    for name, wc in circuits:
        G = len(wc)
        circuit = T.Circuit.from_workload(wc)
        p_ideal = ideal_probs(T, wc)
        u = 2.0 ** -wc.n
        norm = float(np.sum(p_ideal ** 2)) - u
        ltree, src = choose_shape(T, model, wc, shots, 1.0, max_deff)
        trees = {"pershot": ([shots], [0, G]),
                 "dcp": T.dcp(circuit, shots, 1.96, 0.01, copy_cost, 8),
                 "dcp_fused": T.dcp(circuit, shots, 1.96, 0.01, 1.0, 8),
                 "learned": (list(ltree[0]), list(ltree[1]))}
        rec = {"circuit": name, "qubits": wc.n, "gates": G, "shots": shots, "learned_source": src,
               "copy_cost_gates": copy_cost}
        ws = None
        for form, tree in trees.items():
            plan = T.Plan(circuit, tree, "c64")
            nz = T.Noise.sample(circuit, tree, seed)
            need = plan.workspace_bytes(nz)
            if ws is None or ws.nbytes < need:
                ws = None
                ws = T.Workspace(need)
            torch.cuda.synchronize()
            o, st = T.run(plan, nz, ws, stats=True)
            s = (p_ideal[o.astype(np.int64)] - u) / norm
            root = int(tree[0][0])
            if root == o.size:
                se = float(s.std(ddof=1) / math.sqrt(o.size))
            else:
                m = s.reshape(root, o.size // root).mean(1)
                se = float(m.std(ddof=1) / math.sqrt(root))
            rec[form] = {"shape": list(tree[0]), "cut": list(tree[1]), "s": st["ms_device"] * 1e-3,
                         "leaves": int(o.size), "F": float(s.mean()), "F_se": se}

        def per_leaf(f):
            return rec[f]["s"] / rec[f]["leaves"]

        rec["learned_delta_F_vs_pershot"] = rec["learned"]["F"] - rec["pershot"]["F"]
        se = math.hypot(rec["learned"]["F_se"], rec["pershot"]["F_se"])
        rec["learned_delta_F_se"] = se
        # the fidelity bound of the paper (0.016) plus three standard errors
        rec["learned_within_bound"] = bool(abs(rec["learned_delta_F_vs_pershot"]) <= 0.016 + 3 * se)
        for f in ("dcp", "dcp_fused", "pershot"):
            rec["learned_speedup_vs_" + f] = per_leaf(f) / per_leaf("learned")
        log("%s: pershot %.3f s, dcp %s %.3f s, dcp_fused %s %.3f s, learned %s %.3f s (%s); "
            "F %.4f+-%.4f / %.4f+-%.4f / %.4f+-%.4f / %.4f+-%.4f; learned/dcp_fused %.2fx" % (
                name, rec["pershot"]["s"], rec["dcp"]["shape"], rec["dcp"]["s"], rec["dcp_fused"]["shape"],
                rec["dcp_fused"]["s"], rec["learned"]["shape"], rec["learned"]["s"], src,
                rec["pershot"]["F"], rec["pershot"]["F_se"], rec["dcp"]["F"], rec["dcp"]["F_se"],
                rec["dcp_fused"]["F"], rec["dcp_fused"]["F_se"], rec["learned"]["F"], rec["learned"]["F_se"],
                rec["learned_speedup_vs_dcp_fused"]))
        out.append(rec)
    return out
