"""Pass-shape autotuning: the tile width (lane plus register qubits, i.e.
how many qubits one pass's fused gates may touch) and the per-pass work
bound, chosen per circuit by timing short runs of each candidate on the
GPU (library kernels only; the tuning changes how gates are grouped into
passes, never what a trajectory computes)."""
from __future__ import annotations

CANDIDATES = tuple({"tile_qubits": t, "pass_cost": c} for t in (10, 11) for c in (240, 480, 960))


def autotune(T, torch, wc, shots: int = 256, seed: int = 0, reps: int = 2, candidates=CANDIDATES):
    """Fastest tuning for `wc` on a per-shot run of `shots` trajectories;
    returns (tuning, {candidate index: ms})."""
    circuit = T.Circuit.from_workload(wc)
    G = len(wc)
    tree = ([shots], [0, G])
    nz = T.Noise.sample(circuit, tree, seed)
    times = {}
    ws = None
    for i, tun in enumerate(candidates):
        plan = T.Plan(circuit, tree, "c64", tun)
        need = plan.workspace_bytes(nz)
        if ws is None or ws.nbytes < need:
            ws = None
            ws = T.Workspace(need)
        T.run(plan, nz, ws)
        best = float("inf")
        for _ in range(reps):
            _, st = T.run(plan, nz, ws, stats=True)
            best = min(best, st["ms_device"])
        times[i] = best
    k = min(times, key=times.get)
    return dict(candidates[k]), times
