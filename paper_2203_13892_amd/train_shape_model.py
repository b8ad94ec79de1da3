"""Generate the shape model's training runs on the GPU and train it.

    python -m paper_2203_13892_amd.train_shape_model [--minutes M] [--steps S]

Runs seeded circuits of 12-22 qubits (brick-wall, QAOA p = 2, GHZ, QFT round
trip, random 1q/2q) under depolarizing noise (sometimes with twirled
amplitude damping) at 2048-16384 shots in per-shot and tree shapes, timing
each run and measuring the design effect of its cross-entropy estimate
(``learned.measure``); writes the runs to data/shape_runs.npz, trains the
perceptron in the library's kernels and writes data/shape_mlp.npz.
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

from . import learned as Lm
from . import workloads as W

DATA = os.path.join(Lm.HERE, "data", "shape_runs.npz")


def circuit_pool(rng):
    fams = []
    for n in (12, 14, 16, 18, 20, 22):
        for s in range(6):
            fams.append(("bw", n, s))
            fams.append(("bw2", n, s))
            fams.append(("qaoa", n, s))
            fams.append(("rand", n, s))
            fams.append(("qftrt", n, s))
        fams.append(("ghz", n, 0))
    rng.shuffle(fams)
    return fams


def make(fam, n, s, rng):
    if fam == "bw":
        wc = W.brickwall(n, n, seed=100 + s)
    elif fam == "bw2":
        wc = W.brickwall(n, 2 * n, seed=150 + s)
    elif fam == "qaoa":
        wc = W.qaoa(n, 2, seed=200 + s)
    elif fam == "rand":
        wc = W.random_circuit(n, 10 * n, seed=300 + s)
    elif fam == "ghz":
        wc = W.ghz(n)
    else:
        x = int(rng.integers(0, 1 << n))
        wc = W.concat(W.basis_prep(n, x), W.qft(n), W.inverse(W.qft(n)))
    p2 = float(rng.choice([1e-3, 3e-3, 1e-2, 3e-2]))
    gamma = float(rng.choice([0.0, 0.0, p2]))
    return wc.with_noise(p2 / 10, p2, gamma=gamma)


def generate(T, torch, minutes, seed=0, log=print):
    rng = np.random.default_rng(seed)
    rows, t_end = [], time.time() + 60 * minutes
    for fam, n, s in circuit_pool(rng):
        if time.time() > t_end:
            break
        wc = make(fam, n, s, rng)
        G = len(wc)
        circuit = T.Circuit.from_workload(wc)
        p_ideal = Lm.ideal_probs(T, wc)
        ws = None
        for shots in ((2048, 4096) if n >= 20 else (2048, 4096, 8192, 16384)):
            cands = Lm.candidate_shapes(shots, G)
            k = 4 if n >= 20 else 7
            pick = [cands[0]] + [cands[i] for i in rng.choice(np.arange(1, len(cands)),
                                                             min(k, len(cands) - 1), replace=False)]
            for shape in pick:
                if time.time() > t_end:
                    break
                sec, deff, ws = Lm.measure(T, torch, wc, circuit, shape, shots, p_ideal,
                                           int(rng.integers(1 << 30)), ws)
                if not (deff > 0 and np.isfinite(deff)):
                    continue
                feat = np.concatenate([Lm.circuit_features(wc, shots), Lm.shape_features(shape)])
                rows.append(np.concatenate([feat, [math.log(sec / 2.0 ** n), math.log(deff)]]))
        log("%s n=%d: %d runs so far" % (fam, n, len(rows)))
    return np.array(rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--minutes", type=float, default=11.0)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--out-dir", default=None, help="write the npz files here instead of data/")
    ap.add_argument("--evaluate", action="store_true",
                    help="only evaluate the stored model on held-out 24-26 qubit circuits")
    ap.add_argument("--model", default=None, help="with --evaluate: the model file (default data/shape_mlp.npz)")
    ap.add_argument("--copy-cost", type=float, default=26.0,
                    help="with --evaluate: copy cost in gates of the separate-copy DCP baseline")
    args = ap.parse_args()
    import torch
    from . import tqsim as T
    torch.cuda.set_device(0)
    if args.evaluate:
        import json
        model = Lm.ShapeModel.load(T, args.model or Lm.MODEL)
        res = Lm.evaluate(T, torch, model, Lm.held_out_circuits(), copy_cost=args.copy_cost,
                          log=lambda m: print(m, flush=True))
        print(json.dumps(res), flush=True)
        return 0
    rows = generate(T, torch, args.minutes, log=lambda m: print(m, flush=True))
    d = args.out_dir or os.path.dirname(DATA)
    os.makedirs(d, exist_ok=True)
    np.savez(os.path.join(d, "shape_runs.npz"), rows=rows,
             columns=np.array(Lm.CIRCUIT_FEATURES + Lm.SHAPE_FEATURES + Lm.OUTPUTS))
    model = Lm.ShapeModel(T, seed=1)
    X, Y = rows[:, :Lm.N_IN], rows[:, Lm.N_IN:]
    loss = model.fit(X, Y, steps=args.steps, log=lambda it, l: print("step %d loss %.4f" % (it, l), flush=True))
    model.save(os.path.join(d, "shape_mlp.npz"))
    print("runs", rows.shape[0], "final loss", loss, flush=True)


if __name__ == "__main__":
    sys.exit(main())
