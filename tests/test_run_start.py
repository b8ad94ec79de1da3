"""Runs in two halves (tqs_run_start / tqs_run_finish): the host work of
the next run overlaps the device work of the one in flight.  Argument
checks on the CPU; on the GPU, runs started back to back on two workspaces
give the outcomes of runs made one at a time, finished in either order, and
a third start while two are in flight is refused."""
import ctypes

import numpy as np
import pytest

from paper_2203_13892_amd import tqsim as T
from paper_2203_13892_amd import workloads as W


def _case(n=5):
    wc = W.qft(n).with_depolarizing(0.01, 0.01)
    c = T.Circuit.from_workload(wc)
    tree = ([4, 2], [0, 5, len(wc)])
    return wc, c, tree


def test_start_argument_checks(monkeypatch):
    wc, c, tree = _case()
    p = T.Plan(c, tree)
    nz = T.Noise.sample(c, tree, 0)
    need = p.workspace_bytes(nz)
    out = np.zeros(8, np.uint64)
    optr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    h = ctypes.c_void_p(123)
    # no output handle, unknown flags, no plan
    assert T.lib.tqs_run_start(p.h, nz.h, ctypes.c_void_p(1 << 20), need, None, optr, 0, None) == -1
    assert T.lib.tqs_run_start(p.h, nz.h, ctypes.c_void_p(1 << 20), need, None, optr, 6, ctypes.byref(h)) == -1
    assert h.value is None
    assert T.lib.tqs_run_start(None, nz.h, ctypes.c_void_p(1 << 20), need, None, optr, 0, ctypes.byref(h)) == -1
    assert T.lib.tqs_run_finish(None, None) == -1
    # a start that fails before any device call leaves nothing to finish
    monkeypatch.setenv("TQS_FAULT", "alloc")
    h = ctypes.c_void_p(123)
    assert T.lib.tqs_run_start(p.h, nz.h, ctypes.c_void_p(1 << 20), need, None, optr, 1, ctypes.byref(h)) == -5
    assert h.value is None
    monkeypatch.delenv("TQS_FAULT")
    # too small a workspace: refused before device work, the plan usable
    assert T.lib.tqs_run_start(p.h, nz.h, ctypes.c_void_p(1 << 20), need - 1, None, optr, 0, ctypes.byref(h)) == -3
    assert p.workspace_bytes(nz) == need


@pytest.mark.gpu
@pytest.mark.parametrize("prec,n", [("c64", 16), ("c128", 12)])
def test_started_runs_equal_runs_one_at_a_time(prec, n):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    wc = W.qft(n).with_depolarizing(0.002, 0.01)
    g = len(wc)
    tree = ([4, 4, 8], [0, g // 3, 2 * g // 3, g])
    c = T.Circuit.from_workload(wc)
    plan = T.Plan(c, tree, prec, {"chunk_states": 16})
    noises = [T.Noise.sample(c, tree, s) for s in range(5)]
    want = [T.run(plan, nz) for nz in noises]
    need = max(plan.workspace_bytes(nz) for nz in noises)
    wss = [T.Workspace(need), T.Workspace(need)]
    # two in flight, finished in reverse order; a third start is refused
    r0 = T.run_start(plan, noises[0], wss[0], stats=True)
    r1 = T.run_start(plan, noises[1], wss[1])
    with pytest.raises(T.TqsError) as ei:
        T.run_start(plan, noises[2], wss[0])
    assert ei.value.status == -1 and "in flight" in str(ei.value)
    assert np.array_equal(r1.finish(), want[1])
    out0, st0 = r0.finish()
    assert np.array_equal(out0, want[0])
    assert st0["ms_device"] > 0 and st0["pass_launches"] > 0
    # a pipeline over the five lists: start k + 1, then finish k
    got, pending = [], None
    for k in range(len(noises) + 1):
        nxt = T.run_start(plan, noises[k], wss[k % 2]) if k < len(noises) else None
        if pending is not None:
            got.append(pending.finish())
        pending = nxt
    for g_, w_ in zip(got, want):
        assert np.array_equal(g_, w_)
    # the plan still runs one at a time afterwards
    assert np.array_equal(T.run(plan, noises[3]), want[3])
