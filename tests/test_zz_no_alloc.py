"""The run entry point that allocates nothing (tqs_run_noalloc), through the
C ABI, against tqs_run with a workspace: identical outcomes on two calls in
a row, the second with a smaller input, then a run too large for the static
scratch is refused."""
import ctypes

import numpy as np
import pytest

from paper_2203_13892_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2203_13892_amd import tqsim
    return tqsim


def _case(T, wc, A, seed, prec):
    G = len(wc)
    tree = (A, [round(j * G / len(A)) for j in range(len(A) + 1)])
    c = T.Circuit.from_workload(wc)
    return T.Plan(c, tree, prec), T.Noise.sample(c, tree, seed), c


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_noalloc_equals_workspace_run(T, prec):
    import torch
    big = _case(T, W.qft(14).with_depolarizing(1e-2, 3e-2), [4, 4, 4], 5, prec)
    small = _case(T, W.brickwall(12, 8, seed=2).with_depolarizing(1e-2, 3e-2), [4, 6], 6, prec)
    for plan, nz, _ in (big, small):
        assert plan.workspace_bytes(nz) <= 64 << 20
        want = T.run(plan, nz)
        out = np.zeros(plan.n_leaves, np.uint64)
        s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        st = T.lib.tqs_run_noalloc(plan.h, nz.h, s, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
        assert st == 0, T.lib.tqs_last_error()
        assert np.array_equal(out, want)
    # the same two calls once more through the binding: the array keeps the
    # last call's contents, and nothing depends on them
    for plan, nz, _ in (big, small):
        assert np.array_equal(T.run_noalloc(plan, nz), T.run(plan, nz))


def test_noalloc_refuses_runs_beyond_the_scratch(T):
    plan, nz, _ = _case(T, W.qft(20).with_depolarizing(1e-3, 1e-2), [4, 4], 0, "c64")
    assert plan.workspace_bytes(nz) > 64 << 20
    with pytest.raises(T.TqsError) as e:
        T.run_noalloc(plan, nz)
    assert e.value.status == -3 and "static scratch" in str(e.value)


def test_noalloc_with_specialised_kernels(T):
    # a plan with specialised kernels: before any run has loaded them the
    # call takes the generic kernels (loading a module allocates), so it
    # equals the plan run with the generic kernels only; once a run has
    # loaded them it takes them, and equals that run
    wc = W.qft(16).with_depolarizing(1e-2, 3e-2)
    G = len(wc)
    tree = ([4, 4, 8], [0, G // 3, 2 * G // 3, G])
    c = T.Circuit.from_workload(wc)
    nz = T.Noise.sample(c, tree, 3)
    plan = T.Plan(c, tree, "c64", {"jit": 1, "chunk_states": 16})
    assert plan.workspace_bytes(nz) <= 64 << 20
    generic = T.run(T.Plan(c, tree, "c64", {"jit": 2, "chunk_states": 16}), nz)
    assert np.array_equal(T.run_noalloc(plan, nz), generic)
    specialised = T.run(plan, nz)
    assert np.array_equal(T.run_noalloc(plan, nz), specialised)
