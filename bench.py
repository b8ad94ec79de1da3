"""Benchmark: noisy shots/s of tree-reuse vs per-shot trajectory simulation.

Workload: 20-qubit QFT (native H / controlled-phase / swap form, 220 gates),
depolarizing p1 = 1e-3 per one-qubit gate and p2 = 1e-2 per two-qubit gate,
16384 shots, complex64 on one GPU; synthetic seeded inputs.  One step is one
full tqs_run: metadata upload, every gate-apply pass of every tree node,
branching, FP64 sampling of every leaf and the outcome download.

Prints one JSON line.  The dominant kernel's roofline figures come from HIP
events recorded by the library on the run's stream around its pass launches
during the timed steps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "tqs_jit_pass_qft20_tree16x32x32_traffic.json")


def profiled_record():
    """The committed rocprofv3 figures of the pass kernel (FETCH/WRITE bytes
    per launch, VALU instructions of the full leaf launches), or None when
    the kernel, planner or executor sources changed since."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_JSON))
        h = hashlib.sha256()
        for s in rec["sources"]:
            h.update(open(os.path.join(ROOT, s), "rb").read())
        if h.hexdigest() != rec["sources_sha256"]:
            return None
        return rec
    except (OSError, KeyError, ValueError):
        return None


def measured_traffic():
    """HBM bytes per pass launch from the committed counters, or None."""
    rec = profiled_record()
    if rec is None:
        return None
    return rec["hbm_read_bytes_per_launch"] + rec["hbm_write_bytes_per_launch"]


def valu_issue_frac():
    """Share of the VALU issue limit used by a full leaf pass launch: its
    VALU instructions x 4 cycles (a wave64 FP32 instruction per SIMD) over
    1024 SIMDs at 2.4 GHz, against its measured duration; None without a
    current profile."""
    rec = profiled_record()
    if rec is None or "leaf_valu_per_wave" not in rec:
        return None
    cycles = rec["leaf_waves"] * rec["leaf_valu_per_wave"] * 4.0 / 1024
    return cycles / 2.4e9 / (rec["leaf_launch_us"] * 1e-6)


def equal_cuts(G, levels):
    sizes = [G // levels + (1 if i < G % levels else 0) for i in range(levels)]
    cut = [0]
    for s in sizes:
        cut.append(cut[-1] + s)
    return cut


def time_form(T, torch, circuit, tree, seed, steps, warmup, tuning=None):
    t0 = time.perf_counter()
    plan = T.Plan(circuit, tree, "c64", tuning)
    t1 = time.perf_counter()
    nz = T.Noise.sample(circuit, tree, seed)
    t2 = time.perf_counter()
    # two workspaces: step k + 1 is started (its host work done and its
    # launches queued) while step k's device work runs, then step k is
    # finished (tqs_run_start / tqs_run_finish)
    need = plan.workspace_bytes(nz)
    wss = [T.Workspace(need), T.Workspace(need)]
    ws = wss[0]
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        T.run(plan, nz, ws, stream)
    torch.cuda.synchronize()
    agg = {"ms_passes": 0.0, "ms_sample": 0.0, "bytes_passes": 0, "bytes_sample": 0,
           "pass_launches": 0, "ms_device": 0.0, "launches": 0, "nodes_merged": 0,
           "ms_jit": 0.0, "bytes_jit": 0, "jit_launches": 0, "jit_states": 0, "pass_states": 0,
           "host_plan_ms": (t1 - t0) * 1e3, "host_noise_ms": (t2 - t1) * 1e3}
    t0 = time.perf_counter()
    pending = None
    done = []
    for k in range(steps + 1):
        nxt = T.run_start(plan, nz, wss[k % 2], stream, stats=True) if k < steps else None
        if pending is not None:
            done.append(pending.finish())
        pending = nxt
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for out, st in done:
        agg["ms_passes"] += st["ms_passes"]
        agg["ms_sample"] += st["ms_sample"]
        agg["bytes_passes"] += st["bytes_passes"]
        agg["bytes_sample"] += st["bytes_sample"]
        agg["ms_device"] += st["ms_device"]
        agg["launches"] += st["launches"]
        agg["pass_launches"] += st["pass_launches"]
        agg["nodes_merged"] = st["nodes_merged"]
        for k in ("ms_jit", "bytes_jit", "jit_launches", "jit_states", "pass_states"):
            agg[k] += st[k]
    passes_total = sum(plan.info(l)["passes_level"] * int(__import__("numpy").prod(tree[0][:l + 1]))
                       for l in range(len(tree[0])))
    agg["pass_launches_per_step"] = sum(
        plan.info(l)["passes_level"] for l in range(len(tree[0])))
    agg["node_passes_per_step"] = passes_total
    return plan.n_leaves * steps / dt, dt * 1000 / steps, agg, out


def fidelity_loss(T, W, torch, seeds, n=20, shots=16384, p1=1e-4, p2=1e-3):
    """Normalised fidelity (Sec. 4.1: F_s of a peaked ideal distribution,
    normalised against the uniform one) of the 20-qubit QFT round trip from a
    basis state (440 gates), trees (16, 32, 32) and (8, 8, 16, 16) against
    per-shot, over noise seeds; the differences +- their standard errors over
    seeds (each seed's level-0 subtrees are independent, so the per-seed
    difference carries the tree's clustering).  The noise rates keep the
    per-shot F inside (0.3, 0.9), where a fidelity loss would show."""
    import numpy as np
    x = 0x5A5A5 & ((1 << n) - 1)
    wc = W.concat(W.basis_prep(n, x), W.qft(n), W.inverse(W.qft(n))).with_depolarizing(p1, p2)
    G = len(wc)
    c = T.Circuit.from_workload(wc)
    u = 2.0 ** -n
    out = {}
    for name, tree in (("pershot", ([shots], [0, G])), ("tree", ([16, 32, 32], equal_cuts(G, 3))),
                       ("tree4b", ([8, 8, 16, 16], equal_cuts(G, 4)))):
        plan = T.Plan(c, tree, "c64")
        ws = None
        vals = []
        for s in range(seeds):
            nz = T.Noise.sample(c, tree, s)
            if ws is None:
                ws = T.Workspace(plan.workspace_bytes(None))
            o = T.run(plan, nz, ws)
            fs = float(np.mean(o == x))          # F_s with P_ideal = delta_x
            vals.append((fs - u) / (1 - u))
        out[name] = np.array(vals)
    d = out["tree"] - out["pershot"]
    d4 = out["tree4b"] - out["pershot"]
    return {"workload": "qft%d round trip from |x>, depolarizing(%g,%g), %d shots" % (n, p1, p2, shots),
            "bound": 0.016,
            "F_pershot": float(out["pershot"].mean()), "F_tree": float(out["tree"].mean()),
            "delta_F": float(d.mean()), "delta_F_se": float(d.std(ddof=1) / np.sqrt(len(d))),
            "F_tree4b": float(out["tree4b"].mean()), "delta_F_tree4b": float(d4.mean()),
            "delta_F_tree4b_se": float(d4.std(ddof=1) / np.sqrt(len(d4))),
            "seeds": seeds}


def precision_sweep(T, W, torch, seed):
    """26-qubit depth-24 brick-wall, depolarizing p2 in {1e-3, 1e-2} plus the
    Pauli-twirled amplitude damping with gamma = p2 on each gate's qubits,
    8192 shots in the tree (8, 4, 4, 4, 4, 4): complex64 evolution (FP64 CDF)
    over all leaves against complex128 over level-0 subtree 0 (1024 leaves).
    Reports rates, how many of the common leaves draw the same outcome, and
    the complex64 amplitude error against complex128 on two captured
    trajectories
    (the complex128 path itself is checked against the FP64 oracle by a GPU
    parity test on the same circuit family at 22 qubits)."""
    import numpy as np
    n, depth, shape = 26, 24, [8, 4, 4, 4, 4, 4]
    out = []
    for p2 in (1e-3, 1e-2):
        wc = W.brickwall(n, depth, seed=1).with_noise(0.0, p2, gamma=p2)
        G = len(wc)
        c = T.Circuit.from_workload(wc)
        tree = (shape, equal_cuts(G, len(shape)))
        nz = T.Noise.sample(c, tree, seed)
        per = int(np.prod(shape[1:]))
        rec = {"p2": p2, "gamma": p2, "qubits": n, "depth": depth, "gates": G, "tree": shape}
        outs = {}
        for prec, (first, last) in (("c64", (0, shape[0])), ("c128", (0, 1))):
            plan = T.Plan(c, tree, prec)
            # the plan's specialised kernels are compiled beforehand, as a
            # plan does once (timed on its own)
            tc = time.perf_counter()
            plan.compile()
            compile_s = time.perf_counter() - tc
            ws = T.Workspace(plan.workspace_bytes(nz))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            o, st = T.run(plan, nz, ws, stats=True, subtrees=(first, last))
            dt = time.perf_counter() - t0
            outs[prec] = o
            rec[prec] = {"leaves": int(o.size), "shots_per_s": o.size / dt, "s": dt, "compile_s": compile_s,
                         "pass_GBps": st["bytes_passes"] / (st["ms_passes"] * 1e-3) / 1e9}
            del ws
        # complex64 against complex128 amplitudes of two trajectories of the
        # same circuit and noise model
        cap = {}
        tree_c = ([2], [0, G])
        nz_c = T.Noise.sample(c, tree_c, seed)
        for prec in ("c64", "c128"):
            _, amps = T.run_capture(T.Plan(c, tree_c, prec), nz_c, [0, 1])
            cap[prec] = amps
        rec["c64_max_abs_error_vs_c128"] = float(np.max(np.abs(cap["c64"] - cap["c128"])))
        rec["max_abs_amplitude"] = float(np.max(np.abs(cap["c128"])))
        del cap
        same = outs["c64"][:per] == outs["c128"]
        rec["outcomes_equal_c64_c128"] = "%d of %d" % (int(same.sum()), per)
        # a rounding-level difference moves the inverse-CDF pick across a
        # neighbouring boundary: the differing outcomes are index neighbours
        gap = np.abs(outs["c64"][:per].astype(np.int64) - outs["c128"].astype(np.int64))
        rec["largest_outcome_index_gap"] = int(gap.max())
        out.append(rec)
        print("# precision p2=%g: c64 %.1f shots/s, c128 %.1f shots/s, equal outcomes %s, largest index gap %d, "
              "c64 amplitude error %.2e" %
              (p2, rec["c64"]["shots_per_s"], rec["c128"]["shots_per_s"], rec["outcomes_equal_c64_c128"],
               rec["largest_outcome_index_gap"], rec["c64_max_abs_error_vs_c128"]), file=sys.stderr, flush=True)
    return out


def batch_workload(W, count=512):
    """512 circuits of 12-22 qubits: QFT, GHZ chains, QAOA p = 2 on seeded
    random 3-regular graphs (angles uniform in [0, pi]), random brick-walls
    (depth = qubits), depolarizing 1e-3 / 1e-2."""
    out = []
    fams = ("qft", "ghz", "qaoa", "bw")
    ns = (12, 14, 16, 18, 20, 22)
    i = 0
    while len(out) < count:
        f, n = fams[i % 4], ns[(i // 4) % 6]
        s = i // 24
        wc = {"qft": lambda: W.qft(n), "ghz": lambda: W.ghz(n), "qaoa": lambda: W.qaoa(n, 2, seed=s),
              "bw": lambda: W.brickwall(n, n, seed=s)}[f]()
        out.append(("%s%d_%d" % (f, n, s), wc.with_depolarizing(1e-3, 1e-2)))
        i += 1
    return out


def memory_probe(torch, gib=4, reps=10):
    """Plain device memory rates on this GPU, beside the roofline: a fill
    (write only) and a copy (read plus write) of `gib` GiB with torch's own
    kernels, best of `reps`."""
    n = gib << 30
    x = torch.empty(n, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)

    def best(fn):
        fn()
        torch.cuda.synchronize()
        b = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            b = min(b, time.perf_counter() - t0)
        return b

    rec = {"fill_write_GBps": n / best(lambda: x.fill_(1)) / 1e9,
           "copy_read_write_GBps": 2 * n / best(lambda: y.copy_(x)) / 1e9, "bytes": n}
    del x, y
    return rec


def small_runs_leg(T, W, torch, seed, shots=2048, max_qubits=14, reps=3):
    """The batched mixed workload's circuits of at most 14 qubits (their
    states fit one workgroup's LDS), per-shot at 2048 shots each: one run
    after another pass by pass (the default), one run after another with
    each level's passes in one launch and the states in LDS, and as batches
    of runs advanced together (plain launches and a replayed graph).  Best
    of `reps` timings per mode."""
    import numpy as np
    circs = [(name, wc) for name, wc in batch_workload(W) if wc.n <= max_qubits]
    items = {}
    for mode, lds in (("pass_by_pass", 2), ("levels_in_lds", 1)):
        its = []
        for i, (name, wc) in enumerate(circs):
            G = len(wc)
            c = T.Circuit.from_workload(wc)
            tree = ([shots], [0, G])
            tun = {"chunk_states": 512, "lds_levels": lds}
            its.append((T.Plan(c, tree, "c64", tun), T.Noise.sample(c, tree, seed + i)))
        items[mode] = its
    ws = T.Workspace(max(p.workspace_bytes(nz) for p, nz in items["pass_by_pass"]))
    rec = {"workload": "%d circuits of 12-14 qubits from the batched mixed workload, %d shots each, per-shot, "
                       "depolarizing(1e-3,1e-2)" % (len(circs), shots), "runs": len(circs),
           "shots_total": shots * len(circs)}
    outs = {}

    def timed(fn):
        best = float("inf")
        out = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best, out

    for mode, its in items.items():
        for p, nz in its[:4]:
            T.run(p, nz, ws)
        dt, outs[mode] = timed(lambda: [T.run(p, nz, ws) for p, nz in its])
        rec[mode + "_s"] = dt
    # batches: the pass-by-pass plans, runs grouped up to 8 GiB of workspace
    its = items["pass_by_pass"]
    groups, cur, cur_b = [], [], 0
    for k, (p, nz) in enumerate(its):
        b = p.workspace_bytes(nz)
        if cur and cur_b + b > (8 << 30):
            groups.append(cur)
            cur, cur_b = [], 0
        cur.append(k)
        cur_b += b
    groups.append(cur)
    batches = [T.Batch([its[k][0] for k in g], [its[k][1] for k in g]) for g in groups]
    bws = T.Workspace(max(bt.info()["workspace_bytes"] for bt in batches))

    def run_batches():
        res = [bt.run(bws) for bt in batches]
        out = [None] * len(its)
        for gi, g in enumerate(groups):
            for j, k in enumerate(g):
                out[k] = res[gi][j]
        return out

    run_batches()
    rec["batched_s"], outs["batched"] = timed(run_batches)
    for bt in batches:
        bt.use_graph(True)
    run_batches()
    rec["batched_graph_s"], outs["batched_graph"] = timed(run_batches)
    rec["batches"] = len(batches)
    base = outs["pass_by_pass"]
    # batches run the same kernels as the runs one after another: identical
    # outcomes; the level kernel's arithmetic agrees to rounding, so a few
    # leaves at a CDF boundary may pick the neighbouring outcome
    rec["outcomes_identical"] = bool(all(all(np.array_equal(a, b) for a, b in zip(base, outs[m]))
                                         for m in ("batched", "batched_graph")))
    rec["levels_in_lds_outcomes_differing"] = int(sum(int(np.sum(a != b))
                                                      for a, b in zip(base, outs["levels_in_lds"])))
    for k in ("pass_by_pass", "levels_in_lds", "batched", "batched_graph"):
        rec[k + "_shots_per_s"] = rec["shots_total"] / rec[k + "_s"]
        rec[k + "_speedup"] = rec["pass_by_pass_s"] / rec[k + "_s"]
    print("# small runs (%d circuits): pass by pass %.3f s, levels in LDS %.3f s (%.2fx), batched %.3f s (%.2fx), "
          "graph %.3f s (%.2fx), batched outcomes identical %s" % (
              len(circs), rec["pass_by_pass_s"], rec["levels_in_lds_s"], rec["levels_in_lds_speedup"],
              rec["batched_s"], rec["batched_speedup"], rec["batched_graph_s"], rec["batched_graph_speedup"],
              rec["outcomes_identical"]), file=sys.stderr, flush=True)
    return rec


def batch_bench(T, W, torch, seed, shots=2048, budget_gib=32, extra=False):
    """The mixed workload per-shot at 2048 shots each: one run after another
    (default tuning) against batches (runs grouped in qubit order up to a
    workspace budget, each batch advancing its runs together), with the
    default tuning and with the tile width and pass bound autotuned per
    family and size, and with the launches replayed from a recorded graph;
    the same runs as (8, 16, 16) trees, one after another and batched; also
    the 12-16 qubit runs alone, where launches, not bytes, dominate."""
    import numpy as np
    from paper_2203_13892_amd import autotune as AT
    circs = batch_workload(W)

    def note(msg):
        print("# batch: " + msg, file=sys.stderr, flush=True)

    def build(tunings, shape=None):
        items = []
        for i, (name, wc) in enumerate(circs):
            G = len(wc)
            c = T.Circuit.from_workload(wc)
            tree = ([shots], [0, G]) if shape is None else (list(shape), equal_cuts(G, len(shape)))
            tun = dict(tunings.get(name.split("_")[0], {}))
            # live states per run: about 256 MiB of states, at most 512
            tun["chunk_states"] = int(max(1, min(512, (256 << 20) // (8 << wc.n))))
            # one run per circuit: the generic kernels (a plan's specialised
            # kernels cost a hipRTC compile of about a second, more than one
            # such run)
            tun["jit"] = 2
            plan = T.Plan(c, tree, "c64", tun)
            items.append((wc.n, plan, T.Noise.sample(c, tree, seed + i), tun.get("tile_qubits", 11)))
        return items

    def pipelined(items):
        # one run after another, each started before the previous one is
        # finished (two workspaces): host work overlaps device work
        wss = [T.Workspace(max(p.workspace_bytes(nz) for _, p, nz, _ in items)) for _ in range(2)]
        for _, p, nz, _ in items[:4]:
            T.run(p, nz, wss[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out, pend = [], None
        for k in range(len(items) + 1):
            nxt = T.run_start(items[k][1], items[k][2], wss[k % 2]) if k < len(items) else None
            if pend is not None:
                out.append(pend.finish())
            pend = nxt
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    def sequential(items):
        ws = T.Workspace(max(p.workspace_bytes(nz) for _, p, nz, _ in items))
        for _, p, nz, _ in items[:4]:
            T.run(p, nz, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = [T.run(p, nz, ws) for _, p, nz, _ in items]
        return time.perf_counter() - t0, out

    def batched(items, graph=False):
        order = sorted(range(len(items)), key=lambda k: (items[k][3], items[k][0]))
        groups, cur, cur_b, cur_t = [], [], 0, None
        for k in order:
            b = items[k][1].workspace_bytes(items[k][2])
            if cur and (cur_b + b > (budget_gib << 30) or items[k][3] != cur_t):
                groups.append(cur)
                cur, cur_b = [], 0
            cur.append(k)
            cur_b += b
            cur_t = items[k][3]
        groups.append(cur)
        batches = [T.Batch([items[k][1] for k in g], [items[k][2] for k in g]) for g in groups]
        ws = T.Workspace(max(bt.info()["workspace_bytes"] for bt in batches))
        if graph:
            # record each batch's launches once; the timed runs replay them
            for bt in batches:
                bt.use_graph(True)
                bt.run(ws)
        else:
            batches[0].run(ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [bt.run(ws) for bt in batches]
        dt = time.perf_counter() - t0
        out = [None] * len(items)
        for gi, g in enumerate(groups):
            for j, k in enumerate(g):
                out[k] = res[gi][j]
        return dt, out, len(batches)

    rec = {"workload": "512 circuits of 12-22 qubits (qft, ghz, qaoa p=2, brick-wall), 2048 shots each, "
                       "per-shot, depolarizing(1e-3,1e-2)", "runs": len(circs), "shots_total": shots * len(circs)}

    items = build({})
    note("%d runs planned" % len(items))
    t_seq, seq = sequential(items)
    note("one after another %.2f s" % t_seq)
    t_pip, pip = pipelined(items)
    note("one after another, pipelined %.2f s" % t_pip)
    t_bat, bat, nb = batched(items)
    note("batched %.2f s in %d batches" % (t_bat, nb))
    rec["sequential_s"], rec["pipelined_s"], rec["batched_s"], rec["batches"] = t_seq, t_pip, t_bat, nb
    # what a plan's specialised kernels would cost first: the hipRTC
    # compile of the four 22-qubit circuits' plans
    comp = []
    for name, wc in [(nm, w) for nm, w in circs if w.n == 22][:4]:
        c = T.Circuit.from_workload(wc)
        plan = T.Plan(c, ([shots], [0, len(wc)]), "c64", {"jit": 1})
        t0 = time.perf_counter()
        plan.compile()
        comp.append(time.perf_counter() - t0)
    rec["jit_compile_s_22q"] = comp
    note("hipRTC compile of 22-qubit plans: %s s" % ", ".join("%.2f" % x for x in comp))
    rec["outcomes_identical"] = bool(all(np.array_equal(a, b) for a, b in zip(seq, bat)))
    rec["pipelined_outcomes_identical"] = bool(all(np.array_equal(a, b) for a, b in zip(seq, pip)))
    t_bg, bat_g, _ = batched(items, graph=True)
    note("batched, graph replay %.2f s" % t_bg)
    rec["batched_graph_s"] = t_bg
    rec["graph_outcomes_identical"] = bool(all(np.array_equal(a, b) for a, b in zip(seq, bat_g)))
    if extra:
        # autotuned tile width and pass bound per family and size
        tunings, t_tune = {}, time.perf_counter()
        for name, wc in circs:
            key = name.split("_")[0]
            if key not in tunings:
                tunings[key], _ = AT.autotune(T, torch, wc)
                note("autotuned %s: %s" % (key, tunings[key]))
        t_tune = time.perf_counter() - t_tune
        items_t = build(tunings)
        t_auto, _, nb_a = batched(items_t)
        note("autotuned batched %.2f s" % t_auto)
        rec["autotuned_batched_s"], rec["autotune_s"], rec["autotuned_batches"] = t_auto, t_tune, nb_a
        rec["tunings"] = tunings
        # the same runs as trees (8, 16, 16): tree reuse and batching together
        items_tree = build({}, (8, 16, 16))
        t_tseq, tseq = sequential(items_tree)
        t_tbat, tbat, _ = batched(items_tree)
        note("trees (8, 16, 16): one after another %.2f s, batched %.2f s" % (t_tseq, t_tbat))
        rec["tree_shape"] = [8, 16, 16]
        rec["tree_sequential_s"], rec["tree_batched_s"] = t_tseq, t_tbat
        rec["tree_outcomes_identical"] = bool(all(np.array_equal(a, b) for a, b in zip(tseq, tbat)))
        del items_tree, tseq, tbat
    # the small runs alone
    small = [it for it in items if it[0] <= 16]
    t_ss, _ = sequential(small)
    t_sb, _, _ = batched(small)
    t_sg, _, _ = batched(small, graph=True)
    rec["small_runs"] = len(small)
    rec["small_sequential_s"], rec["small_batched_s"], rec["small_batched_graph_s"] = t_ss, t_sb, t_sg
    for k in ("sequential", "pipelined", "batched", "batched_graph", "autotuned_batched", "tree_sequential",
              "tree_batched"):
        if k + "_s" in rec:
            rec[k + "_shots_per_s"] = rec["shots_total"] / rec[k + "_s"]
    rec["small_batch_speedup"] = t_ss / t_sb
    rec["small_batch_graph_speedup"] = t_ss / t_sg
    print("# batch: sequential %.2f s, pipelined %.2f s, batched %.2f s (%d batches, identical %s); "
          "12-16q runs: sequential %.3f s, batched %.3f s, graph replay %.3f s" % (
              t_seq, t_pip, t_bat, nb, rec["outcomes_identical"], t_ss, t_sb, t_sg),
          file=sys.stderr, flush=True)
    return rec


def mfma_sweep(T, W, torch, steps=3, shots=4096):
    """Fused 32x32 blocks on the matrix cores against the vector units: a
    20-qubit circuit of k Haar SU(4) gates on random pairs of qubits 6..10
    (the tile's register window; seed 5), noiseless, every state computed,
    one pass; per k the rate with tuning.mfma_min_ops 1000 (off) and 1."""
    import numpy as np
    rng = np.random.default_rng(5)
    out = []
    for k in (4, 8, 16, 32):
        wc = W.Circuit(20)
        for _ in range(k):
            a, b = rng.choice(np.arange(6, 11), 2, replace=False)
            wc.add((int(a), int(b)), W.haar_unitary(4, rng))
        c = T.Circuit.from_workload(wc)
        tree = ([shots], [0, len(wc)])
        nz = T.Noise.sample(c, tree, 0)
        rec = {"su4_gates": k}
        for name, mm in (("vector", 1000), ("mfma", 1)):
            plan = T.Plan(c, tree, "c64", {"mfma_min_ops": mm, "pass_cost": 100000, "no_merge": 1})
            ws = T.Workspace(plan.workspace_bytes(nz))
            T.run(plan, nz, ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                T.run(plan, nz, ws)
            torch.cuda.synchronize()
            rec[name + "_shots_per_s"] = shots * steps / (time.perf_counter() - t0)
            del ws
        rec["mfma_speedup"] = rec["mfma_shots_per_s"] / rec["vector_shots_per_s"]
        print("# mfma: %d SU(4): vector %.1fK shots/s, fused block on MFMA %.1fK shots/s" %
              (k, rec["vector_shots_per_s"] / 1e3, rec["mfma_shots_per_s"] / 1e3), file=sys.stderr, flush=True)
        out.append(rec)
    return out


def parity_sample(T, wc, tree, seed, count=16):
    """The headline run against the oracle on `count` leaves spread over the
    tree: max-abs amplitude error (complex64 against complex128) and how many
    outcomes agree (a disagreement is counted at a CDF boundary only)."""
    import numpy as np
    import oracle
    c = T.Circuit.from_workload(wc)
    plan = T.Plan(c, tree, "c64")
    nz = T.Noise.sample(c, tree, seed)
    leaves = np.linspace(0, plan.n_leaves - 1, count).astype(np.uint64)
    out, amps = T.run_capture(plan, nz, leaves)
    onz = oracle.sample_noise(wc.gates, tree, seed)
    threads = max(1, min(len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS", "16"))))
    oout, ost = oracle.run_leaves(wc.n, wc.gates, tree, onz, leaves, states=True, threads=threads)
    err = float(np.max(np.abs(amps - ost)))
    got = out[leaves.astype(np.int64)]
    same = int(np.sum(got == oout))
    # a differing outcome is a boundary pick when every oracle prefix between
    # the two outcomes lies within 1e-6 T of u T; anything else is invalid
    boundary, invalid = 0, 0
    for i in np.nonzero(got != oout)[0]:
        pr = np.abs(ost[i]) ** 2
        tot, pre = pr.sum(), np.cumsum(pr)
        lo, hi = sorted((int(got[i]), int(oout[i])))
        ok = hi < pr.size and np.all(np.abs(pre[lo:hi] - onz.leaf_u[int(leaves[i])] * tot) <= 1e-6 * tot)
        boundary += int(ok)
        invalid += int(not ok)
    return {"leaves": count, "max_abs_amplitude_error": err, "tolerance": 1e-5,
            "outcomes_equal": "%d of %d" % (same, count), "boundary_leaves": boundary,
            "invalid_outcomes": invalid}


def cpu_baseline(wc, seed, budget_s=15.0):
    """The oracle (per-shot, complex128, threads over shots) on a bounded
    sample of the same workload's shots."""
    import numpy as np
    import oracle
    n = wc.n
    G = len(wc)
    # the host cores this process may use (at most the job's share of 16)
    threads = max(1, min(len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS", "16"))))
    tree = ([16384], [0, G])
    nz = oracle.sample_noise(wc.gates, tree, seed)
    # calibrate on one round of `threads` shots, then fill the budget
    S = threads
    t0 = time.perf_counter()
    oracle.run_leaves(n, wc.gates, tree, nz, np.arange(S, dtype=np.uint64), threads=threads)
    t1 = time.perf_counter() - t0
    rounds = max(1, int(budget_s / max(t1, 1e-3)) - 1)
    S2 = min(16384, threads * rounds)
    t0 = time.perf_counter()
    oracle.run_leaves(n, wc.gates, tree, nz, np.arange(S, S + S2, dtype=np.uint64), threads=threads)
    dt = time.perf_counter() - t0
    # one thread, two trajectories
    t0 = time.perf_counter()
    oracle.run_leaves(n, wc.gates, tree, nz, np.arange(S + S2, S + S2 + 2, dtype=np.uint64), threads=1)
    dt1 = time.perf_counter() - t0
    model = ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": S2 / dt, "unit": "noisy shots/s", "cores": threads, "kind": "oracle",
            "sample": "%d of the 16384 per-shot trajectories of the same workload "
                      "(complex128, %d threads, %.1f s)" % (S2, threads, dt),
            "single_thread_shots_per_s": 2 / dt1, "cpu_model": model}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-dcp", action="store_true",
                    help="skip the copy-cost measurement and the DCP-shaped form")
    ap.add_argument("--forms", default="tree,pershot,tree_nomerge,pershot_nomerge,tree4a,tree4b")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--tile", type=int, default=0, help="tile qubits (0 = library default)")
    ap.add_argument("--pass-cost", type=int, default=0, help="per-pass work bound (0 = default)")
    ap.add_argument("--chunk", type=int, default=0, help="live states per level (0 = default)")
    ap.add_argument("--no-fidelity", action="store_true",
                    help="skip the tree's fidelity loss against per-shot sampling")
    ap.add_argument("--fid-seeds", type=int, default=20)
    ap.add_argument("--no-small-runs", action="store_true",
                    help="skip the leg of the batched mixed workload's 12-14 qubit circuits")
    ap.add_argument("--batch-extra", action="store_true",
                    help="with --batch: also the autotuned tile widths and the (8, 16, 16) trees")
    ap.add_argument("--batch", action="store_true",
                    help="also run the 512-circuit mixed workload one run at a time and batched")
    ap.add_argument("--learned", action="store_true",
                    help="also evaluate the learned tree shape against DCP and per-shot on "
                         "held-out 24-qubit circuits")
    ap.add_argument("--precision", action="store_true",
                    help="also run the 26-qubit complex64 / complex128 precision sweep")
    ap.add_argument("--no-bw", action="store_true",
                    help="skip the 20-qubit brick-wall forms (reported beside the QFT ones)")
    ap.add_argument("--mfma-sweep", action="store_true",
                    help="only compare fused 32x32 blocks on the matrix cores with the vector units "
                         "on register-local SU(4) circuits, and print that record")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(level-0 subtree ranges would be split across GPUs with tqs_run_range)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2203_13892_amd import tqsim as T
    from paper_2203_13892_amd import workloads as W

    torch.cuda.set_device(0)
    if args.mfma_sweep:
        print(json.dumps({"mfma_sweep": mfma_sweep(T, W, torch, args.steps)}), flush=True)
        return
    shots = 16384
    wc = W.qft(20).with_depolarizing(1e-3, 1e-2)
    G = len(wc)
    circuit = T.Circuit.from_workload(wc)
    forms = {
        "tree": ([16, 32, 32], equal_cuts(G, 3)),
        "pershot": ([shots], [0, G]),
        "tree4a": ([32, 8, 8, 8], equal_cuts(G, 4)),
        "tree4b": ([8, 8, 16, 16], equal_cuts(G, 4)),
    }
    # the same shapes with every node's state computed (tree reuse alone,
    # without sharing the states of nodes with equal noise histories)
    forms["tree_nomerge"] = forms["tree"]
    forms["pershot_nomerge"] = forms["pershot"]
    # state copy in gate-equivalents on this GPU (the DCP copy-cost input):
    # one state's read + write at the streaming-copy rate, against the average
    # time per gate execution of a per-shot run
    if not args.no_dcp:
        copy_gbps = T.probe_copy(1 << 30, 10)
        copy_us = 2 * 8 * (1 << 20) / (copy_gbps * 1e3)
        sps_ps, _, agg_ps, _ = time_form(T, torch, circuit, forms["pershot"], args.seed, 1, 1,
                                         {"no_merge": 1})
        gate_us = agg_ps["ms_passes"] * 1e3 / (shots * G)
        copy_cost = copy_us / gate_us
        dcp_shape = T.dcp(circuit, shots, 1.96, 0.01, copy_cost, 8)
        forms["dcp"] = dcp_shape
        # the branch copy rides on the children's first pass here, so its
        # marginal cost is about one gate: DCP with that copy cost
        forms["dcp_fused"] = T.dcp(circuit, shots, 1.96, 0.01, 1.0, 8)
        for f in ("dcp", "dcp_fused"):
            if f not in args.forms.split(","):
                args.forms += "," + f
    results = {}
    for name in args.forms.split(","):
        tree = forms[name]
        tuning = {k: v for k, v in (("tile_qubits", args.tile), ("pass_cost", args.pass_cost),
                                     ("chunk_states", args.chunk)) if v}
        if name.endswith("_nomerge"):
            tuning["no_merge"] = 1
        sps, ms, agg, _ = time_form(T, torch, circuit, tree, args.seed, args.steps, args.warmup,
                                    tuning or None)
        results[name] = {"shots_per_s": sps, "ms_per_step": ms, "shape": tree[0], "cut": tree[1],
                         "pass_GBps": agg["bytes_passes"] / (agg["ms_passes"] * 1e-3) / 1e9,
                         "ms_passes": agg["ms_passes"] / args.steps,
                         "ms_sample": agg["ms_sample"] / args.steps,
                         "launches": agg["launches"] // args.steps,
                         "pass_launches_per_step": agg["pass_launches_per_step"],
                         "pass_launches": agg["pass_launches"],
                         "nodes_merged": agg["nodes_merged"],
                         "host_plan_ms": agg["host_plan_ms"], "host_noise_ms": agg["host_noise_ms"],
                         "bytes_per_launch": agg["bytes_passes"] / max(agg["pass_launches"], 1),
                         "us_per_launch": agg["ms_passes"] * 1e3 / max(agg["pass_launches"], 1),
                         "jit_launches": agg["jit_launches"], "ms_jit": agg["ms_jit"],
                         "bytes_jit": agg["bytes_jit"], "jit_states": agg["jit_states"],
                         "pass_states": agg["pass_states"]}
        print("# %s: %.1f shots/s, %.2f ms/step, pass %.0f GB/s" %
              (name, sps, ms, results[name]["pass_GBps"]), file=sys.stderr, flush=True)
    head = "tree" if "tree" in results else list(results)[0]
    h = results[head]
    # the dominant kernel: the plan-specialised pass kernel, timed with HIP
    # events around each of its launches (the generic kernel takes the
    # nodes it does not: reported beside it)
    jl = max(h["jit_launches"], 1)
    achieved = h["bytes_jit"] / (h["ms_jit"] * 1e-3) / 1e9 if h["ms_jit"] > 0 else h["pass_GBps"]
    prof = profiled_record()
    line = {
        "metric": "noisy shots/s, 20q QFT 16k shots: tree vs per-shot on 1 GPU; % HBM peak",
        "value": h["shots_per_s"],
        "unit": "noisy shots/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "complex64",
        "data": "synthetic",
        "config": {"workload": "qft20 depolarizing(1e-3,1e-2) 16384 shots, tree %s" %
                   "x".join(map(str, h["shape"])), "qubits": 20, "gates": G, "shots": shots,
                   "tree": h["shape"], "cut": h["cut"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "valu_issue_frac": valu_issue_frac(),
                     "kernel": "tqs_jit_p* (plan-specialised pass kernel, float)",
                     "algorithmic_bytes_per_launch": h["bytes_jit"] / jl,
                     "us_per_launch": h["ms_jit"] * 1e3 / jl, "launches": h["jit_launches"],
                     "states_share": h["jit_states"] / max(h["pass_states"], 1),
                     "all_pass_launches_GBps": h["pass_GBps"]},
        "forms": {k: {kk: v[kk] for kk in ("shots_per_s", "ms_per_step", "pass_GBps", "shape", "nodes_merged",
                                           "host_plan_ms", "host_noise_ms")}
                  for k, v in results.items()},
    }
    # like for like: the tree against per-shot with states of equal noise
    # histories shared in both, and with every node computed in both
    if "tree" in results and "pershot" in results:
        line["tree_speedup_vs_pershot"] = results["tree"]["shots_per_s"] / results["pershot"]["shots_per_s"]
    if "tree_nomerge" in results and "pershot_nomerge" in results:
        line["tree_nomerge_speedup_vs_pershot_nomerge"] = (results["tree_nomerge"]["shots_per_s"] /
                                                           results["pershot_nomerge"]["shots_per_s"])
    if not args.no_dcp:
        line["copy_cost_gates"] = copy_cost
        line["copy_GBps"] = copy_gbps
        line["dcp"] = {"tree": dcp_shape[0], "cut": dcp_shape[1], "z": 1.96, "eps": 0.01,
                       "copy_cost_gates": copy_cost}
    if not args.no_bw:
        # the same noise model on a 20-qubit depth-20 brick-wall of Haar SU(4)
        # gates (circuit seed 1): per-shot against tree reuse
        bw = W.brickwall(20, 20, seed=1).with_depolarizing(1e-3, 1e-2)
        Gb = len(bw)
        cb = T.Circuit.from_workload(bw)
        line["brickwall"] = {"workload": "brickwall20 d20 seed 1, depolarizing(1e-3,1e-2) 16384 shots",
                             "gates": Gb, "forms": {}}
        # (tree4b_no_level_exchange: without lane exchanges at the levels'
        # ends, tuning level_exchange = 2; the default plan keeps them here)
        for name, tree, tun in (("pershot", ([shots], [0, Gb]), None),
                                ("tree", ([16, 32, 32], equal_cuts(Gb, 3)), None),
                                ("tree4b", ([8, 8, 16, 16], equal_cuts(Gb, 4)), None),
                                ("tree4b_no_level_exchange", ([8, 8, 16, 16], equal_cuts(Gb, 4)),
                                 {"level_exchange": 2})):
            sps, ms, agg, _ = time_form(T, torch, cb, tree, args.seed, args.steps, args.warmup, tun)
            pl = T.Plan(cb, tree, "c64", tun)
            line["brickwall"]["forms"][name] = {
                "shots_per_s": sps, "ms_per_step": ms, "shape": tree[0],
                "passes_per_level": [pl.info(l)["passes_level"] for l in range(len(tree[0]))],
                "pass_GBps": agg["bytes_passes"] / (agg["ms_passes"] * 1e-3) / 1e9}
            print("# brickwall %s: %.1f shots/s, %.2f ms/step" % (name, sps, ms), file=sys.stderr, flush=True)
    if not args.no_fidelity:
        line["fidelity_loss"] = fidelity_loss(T, W, torch, args.fid_seeds)
        fl = line["fidelity_loss"]
        print("# fidelity: F_pershot %.4f, dF (16,32,32) %+.4f +- %.4f, dF (8,8,16,16) %+.4f +- %.4f" %
              (fl["F_pershot"], fl["delta_F"], fl["delta_F_se"], fl["delta_F_tree4b"], fl["delta_F_tree4b_se"]),
              file=sys.stderr, flush=True)
    line["memory_probe"] = memory_probe(torch)
    if not args.no_small_runs:
        line["small_runs"] = small_runs_leg(T, W, torch, args.seed)
    if args.precision:
        line["precision_sweep"] = precision_sweep(T, W, torch, args.seed)
    if args.batch:
        line["batched_mixed"] = batch_bench(T, W, torch, args.seed, extra=args.batch_extra)
    if args.learned:
        from paper_2203_13892_amd import learned as Lm
        model = Lm.ShapeModel.load(T)
        cc = line.get("copy_cost_gates", 26.0)
        line["learned_shape"] = Lm.evaluate(T, torch, model, Lm.held_out_circuits(), copy_cost=cc,
                                            seed=args.seed,
                                            log=lambda m: print("# learned " + m, file=sys.stderr, flush=True))
    if not args.no_cpu:
        # the oracle leg: its timing, and the headline run checked against it
        line["cpu_baseline"] = cpu_baseline(wc, args.seed, args.cpu_budget)
        line["cpu_baseline"]["gpu_parity"] = parity_sample(T, wc, forms[head], args.seed)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
