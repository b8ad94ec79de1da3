"""Error paths of a run, driven by the host-side failure injection
(environment variable TQS_FAULT, read by the library on each run; no kernel
is altered).

- alloc: the run's host metadata allocation fails, TQS_E_OOM before any
  device call (so it runs on the CPU too); the plan stays usable.
- launch:K: the K-th pass reports a launch failure, TQS_E_HIP after the
  passes before it were enqueued; the run drains its stream before it
  returns, and resuming with subtree ranges on the same workspace gives the
  outcomes of an undisturbed run.
"""
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


def test_alloc_fault_before_device_work(monkeypatch):
    wc, c, tree = _case()
    p = T.Plan(c, tree)
    nz = T.Noise.sample(c, tree, 0)
    need = p.workspace_bytes(nz)
    out = np.zeros(8, np.uint64)
    optr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    monkeypatch.setenv("TQS_FAULT", "alloc")
    # a well-formed call: an aligned address (never touched: the failure
    # comes before any device call) and a large enough workspace
    st = T.lib.tqs_run(p.h, nz.h, ctypes.c_void_p(1 << 20), need, None, optr, None)
    assert st == -5 and "host allocation" in T.lib.tqs_last_error().decode()
    st = T.lib.tqs_run_range(p.h, nz.h, ctypes.c_void_p(1 << 20), need, None, 1, 3, optr, None)
    assert st == -5
    assert not out.any()
    # argument checks come before the injected failure
    st = T.lib.tqs_run(p.h, nz.h, ctypes.c_void_p(1 << 20), need, None, None, None)
    assert st == -1
    # the plan is intact: its queries answer as before, and it is destroyed
    assert p.workspace_bytes(nz) == need
    assert "pass" in p.describe()
    monkeypatch.delenv("TQS_FAULT")
    del p


def test_unknown_fault_values_are_ignored(monkeypatch):
    # anything but "alloc" or "launch[:K]" injects nothing: the run gets to
    # its workspace check (which fails here on purpose, before device work)
    wc, c, tree = _case()
    p = T.Plan(c, tree)
    nz = T.Noise.sample(c, tree, 0)
    need = p.workspace_bytes(nz)
    out = np.zeros(8, np.uint64)
    optr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    for v in ["", "allocx", "launcher", "oom"]:
        monkeypatch.setenv("TQS_FAULT", v)
        st = T.lib.tqs_run(p.h, nz.h, ctypes.c_void_p(1 << 20), need - 1, None, optr, None)
        assert st == -3, v


@pytest.mark.gpu
@pytest.mark.parametrize("prec,n", [("c64", 16), ("c128", 12)])
def test_launch_fault_then_resume(monkeypatch, prec, n):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    wc = W.qft(n).with_depolarizing(0.002, 0.01)
    g = len(wc)
    tree = ([4, 4, 8], [0, g // 3, 2 * g // 3, g])
    c = T.Circuit.from_workload(wc)
    nz = T.Noise.sample(c, tree, 7)
    plan = T.Plan(c, tree, prec, {"chunk_states": 8})
    ws = T.Workspace(plan.workspace_bytes(nz))
    want = T.run(plan, nz, workspace=ws)
    # this tree's runs take at least six passes (chunks of up to eight
    # computed states, one pass per level): the first, one in the middle
    # level, one at the leaves
    for k in [0, 2, 5]:
        monkeypatch.setenv("TQS_FAULT", "launch:%d" % k)
        with pytest.raises(T.TqsError) as ei:
            T.run(plan, nz, workspace=ws)
        assert ei.value.status == -4 and "TQS_FAULT" in str(ei.value)
        monkeypatch.delenv("TQS_FAULT")
        # resume on the same workspace, right away, in two ranges
        got = np.concatenate([T.run(plan, nz, workspace=ws, subtrees=(0, 1)),
                              T.run(plan, nz, workspace=ws, subtrees=(1, 4))])
        assert np.array_equal(got, want), k
    # K beyond the run's last pass injects nothing
    monkeypatch.setenv("TQS_FAULT", "launch:100000")
    assert np.array_equal(T.run(plan, nz, workspace=ws), want)
    monkeypatch.setenv("TQS_FAULT", "alloc")
    with pytest.raises(T.TqsError) as ei:
        T.run(plan, nz, workspace=ws)
    assert ei.value.status == -5
    monkeypatch.delenv("TQS_FAULT")
    assert np.array_equal(T.run(plan, nz, workspace=ws), want)
