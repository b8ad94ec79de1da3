"""Python binding of ``libtqsim.so`` (argument marshalling only).

Every simulation step runs in the library's HIP kernels; this module only
converts arrays, owns the opaque handles and lets PyTorch supply the device
workspace and the stream.  The library must have been built
(``python -m paper_2203_13892_amd.build``); importing this module without it
raises immediately -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtqsim.so")

C64, C128 = 0, 1
_PREC = {"c64": C64, "c128": C128, C64: C64, C128: C128}

u32, u64, dbl, i32, vp = C.c_uint32, C.c_uint64, C.c_double, C.c_int, C.c_void_p
P = C.POINTER


class TqsTree(C.Structure):
    _fields_ = [("levels", u32), ("arity", P(u64)), ("cut", P(u32))]


class TqsTuning(C.Structure):
    _fields_ = [("tile_qubits", u32), ("max_ops_per_pass", u32), ("chunk_states", u32),
                ("sample_block_log", u32), ("pass_cost", u32), ("no_merge", u32),
                ("separate_sampling", u32), ("jit", u32), ("mfma_min_ops", u32), ("lds_levels", u32),
                ("level_exchange", u32)]


class TqsRunStats(C.Structure):
    _fields_ = [("ms_wall", dbl), ("ms_device", dbl), ("ms_passes", dbl), ("ms_sample", dbl),
                ("launches", u64), ("pass_launches", u64), ("pass_states", u64), ("bytes_passes", u64),
                ("bytes_sample", u64), ("events", u64), ("nodes_merged", u64), ("jit_launches", u64),
                ("jit_states", u64), ("bytes_jit", u64), ("ms_jit", dbl)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes): every symbol declared in include/tqsim.h
SIGNATURES = {
    "tqs_circuit_create": (i32, [u32, P(vp)]),
    "tqs_circuit_add_gate": (i32, [vp, u32, P(u32), P(dbl), P(dbl)]),
    "tqs_circuit_set_depolarizing": (i32, [vp, dbl, dbl]),
    "tqs_circuit_info": (i32, [vp, P(u32), P(u32)]),
    "tqs_circuit_destroy": (None, [vp]),
    "tqs_dcp": (i32, [vp, u64, dbl, dbl, dbl, u32, P(u32), P(u64), P(u32)]),
    "tqs_noise_sample": (i32, [vp, P(TqsTree), u64, P(vp)]),
    "tqs_noise_import": (i32, [vp, P(TqsTree), P(u64), P(u32), P(C.c_uint8), P(dbl), P(vp)]),
    "tqs_noise_view": (i32, [vp, P(P(u64)), P(P(u32)), P(P(C.c_uint8)), P(P(dbl)), P(u64), P(u64)]),
    "tqs_noise_destroy": (None, [vp]),
    "tqs_plan_create": (i32, [vp, P(TqsTree), i32, P(TqsTuning), P(vp)]),
    "tqs_plan_info": (i32, [vp, u32, P(u32), P(u32), P(u32)]),
    "tqs_workspace_bytes": (i32, [vp, vp, P(u64)]),
    "tqs_plan_destroy": (None, [vp]),
    "tqs_circuit_set_readout": (i32, [vp, P(dbl)]),
    "tqs_noise_set_flips": (i32, [vp, P(u32)]),
    "tqs_noise_flips": (i32, [vp, P(P(u32))]),
    "tqs_run": (i32, [vp, vp, vp, u64, vp, P(u64), P(TqsRunStats)]),
    "tqs_run_range": (i32, [vp, vp, vp, u64, vp, u64, u64, P(u64), P(TqsRunStats)]),
    "tqs_run_start": (i32, [vp, vp, vp, u64, vp, P(u64), u32, P(vp)]),
    "tqs_run_finish": (i32, [vp, P(TqsRunStats)]),
    "tqs_run_capture": (i32, [vp, vp, vp, u64, vp, P(u64), P(u64), u64, P(dbl)]),
    "tqs_run_noalloc": (i32, [vp, vp, vp, P(u64)]),
    "tqs_histogram": (i32, [P(u64), u64, P(u64), P(u64), P(u64)]),
    "tqs_probe_copy": (i32, [vp, u64, u32, vp, P(dbl)]),
    "tqs_plan_describe": (i32, [vp, C.c_char_p, u64, P(u64)]),
    "tqs_plan_compile": (i32, [vp]),
    "tqs_plan_jit_source": (i32, [vp, C.c_char_p, u64, P(u64)]),
    "tqs_batch_create": (i32, [P(vp), P(vp), u32, P(vp)]),
    "tqs_batch_info": (i32, [vp, P(u64), P(u64), P(u32)]),
    "tqs_batch_use_graph": (i32, [vp, u32]),
    "tqs_batch_run": (i32, [vp, vp, u64, vp, P(u64), P(TqsRunStats)]),
    "tqs_batch_destroy": (None, [vp]),
    "tqs_mlp_param_count": (u64, [u32, u32, u32]),
    "tqs_mlp_scratch_floats": (u64, [u32, u32, u32, u32]),
    "tqs_mlp_forward": (i32, [vp, u32, u32, u32, vp, u32, vp, vp, vp]),
    "tqs_mlp_loss_grad": (i32, [vp, u32, u32, u32, vp, vp, vp, u32, vp, vp, vp, vp]),
    "tqs_mlp_adam": (i32, [vp, vp, vp, vp, u64, C.c_float, C.c_float, C.c_float, C.c_float, u32, vp]),
    "tqs_last_error": (C.c_char_p, []),
    "tqs_version": (C.c_char_p, []),
}

STATUS = {0: "TQS_OK", -1: "TQS_E_ARG", -2: "TQS_E_SHAPE", -3: "TQS_E_WORKSPACE",
          -4: "TQS_E_HIP", -5: "TQS_E_OOM", -6: "TQS_E_UNSUPPORTED"}


class TqsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libtqsim.so is not built (%s); run python -m paper_2203_13892_amd.build"
                          % LIB_PATH)
    # Load torch's HIP runtime first so that the library binds to it: one
    # runtime per process, to which the streams and device pointers handed
    # over from torch belong (a second runtime copy cannot open the device).
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


lib = _load()


def _check(st):
    if st != 0:
        raise TqsError(st, lib.tqs_last_error().decode())


def _ptr(a, ct):
    return a.ctypes.data_as(P(ct))


def version() -> str:
    return lib.tqs_version().decode()


# ----------------------------------------------------------------- circuit --

class Circuit:
    """Owned tqs_circuit handle."""

    def __init__(self, n: int):
        h = vp()
        _check(lib.tqs_circuit_create(n, C.byref(h)))
        self.h = h
        self.n = n

    def add_gate(self, qubits, mat, probs=None):
        q = np.ascontiguousarray(np.asarray(qubits, np.uint32))
        m = np.ascontiguousarray(np.asarray(mat, np.complex128)).view(np.float64)
        p = None if probs is None else np.ascontiguousarray(np.asarray(probs, np.float64))
        _check(lib.tqs_circuit_add_gate(self.h, q.size, _ptr(q, u32), _ptr(m, dbl),
                                        None if p is None else _ptr(p, dbl)))
        return self

    def set_depolarizing(self, p1: float, p2: float):
        _check(lib.tqs_circuit_set_depolarizing(self.h, p1, p2))
        return self

    def set_readout(self, p_flip):
        """Per-qubit read-out flip probabilities (None removes the channel)."""
        if p_flip is None:
            _check(lib.tqs_circuit_set_readout(self.h, None))
        else:
            r = np.ascontiguousarray(np.broadcast_to(np.asarray(p_flip, np.float64), (self.n,)))
            _check(lib.tqs_circuit_set_readout(self.h, _ptr(r, dbl)))
        return self

    @property
    def n_gates(self) -> int:
        n, g = u32(), u32()
        _check(lib.tqs_circuit_info(self.h, C.byref(n), C.byref(g)))
        return g.value

    @classmethod
    def from_workload(cls, wc) -> "Circuit":
        """From a ``workloads.Circuit`` (gates with matrices and probabilities)."""
        c = cls(wc.n)
        for q, m, p in wc.gates:
            c.add_gate(q, m, p)
        if getattr(wc, "readout", None) is not None:
            c.set_readout(wc.readout)
        return c

    def __del__(self):
        h = getattr(self, "h", None)
        # (at interpreter exit the module globals may already be gone)
        if h is not None and h.value and lib is not None:
            lib.tqs_circuit_destroy(h)
            self.h = vp()


class _Tree:
    def __init__(self, arity, cut):
        self.A = np.ascontiguousarray(np.asarray(arity, np.uint64))
        self.cut = np.ascontiguousarray(np.asarray(cut, np.uint32))
        self.s = TqsTree(self.A.size, _ptr(self.A, u64), _ptr(self.cut, u32))


def dcp(circuit: Circuit, shots: int, z: float = 1.96, eps: float = 0.01, copy_cost: float = 1.0,
        max_levels: int = 16):
    """Dynamic Circuit Partition; returns (arity list, cut list)."""
    lv = u32()
    A = np.zeros(max_levels, np.uint64)
    cut = np.zeros(max_levels + 1, np.uint32)
    _check(lib.tqs_dcp(circuit.h, shots, z, eps, copy_cost, max_levels, C.byref(lv),
                       _ptr(A, u64), _ptr(cut, u32)))
    k = lv.value
    return [int(a) for a in A[:k]], [int(c) for c in cut[:k + 1]]


# ------------------------------------------------------------------- noise --

class Noise:
    """Owned tqs_noise handle (insertion list + leaf uniforms)."""

    def __init__(self, h):
        self.h = h

    @classmethod
    def sample(cls, circuit: Circuit, tree, seed: int) -> "Noise":
        t = _Tree(*tree)
        h = vp()
        _check(lib.tqs_noise_sample(circuit.h, C.byref(t.s), seed, C.byref(h)))
        return cls(h)

    @classmethod
    def from_arrays(cls, circuit: Circuit, tree, node_off, ev_gate, ev_code, leaf_u,
                    leaf_flip=None) -> "Noise":
        t = _Tree(*tree)
        no = np.ascontiguousarray(np.asarray(node_off, np.uint64))
        eg = np.ascontiguousarray(np.asarray(ev_gate, np.uint32))
        ec = np.ascontiguousarray(np.asarray(ev_code, np.uint8))
        lu = np.ascontiguousarray(np.asarray(leaf_u, np.float64))
        # the library reads node_off[nodes + 1], node_off[-1] events and one
        # uniform per leaf: check the lengths before handing pointers over
        A = [int(a) for a in tree[0]]
        nodes, leaves, width = 0, 1, 1
        for a in A:
            width *= a
            nodes += width
        leaves = width
        if no.ndim != 1 or no.size != nodes + 1:
            raise ValueError("node_off needs %d entries (nodes + 1), got %d" % (nodes + 1, no.size))
        ne = int(no[-1])
        if eg.size < ne or ec.size < ne:
            raise ValueError("node_off[-1] = %d events, ev_gate has %d and ev_code %d" % (ne, eg.size, ec.size))
        if lu.size != leaves:
            raise ValueError("leaf_u needs %d entries (one per leaf), got %d" % (leaves, lu.size))
        if eg.size == 0:
            eg, ec = np.zeros(1, np.uint32), np.zeros(1, np.uint8)
        h = vp()
        _check(lib.tqs_noise_import(circuit.h, C.byref(t.s), _ptr(no, u64), _ptr(eg, u32),
                                    _ptr(ec, C.c_uint8), _ptr(lu, dbl), C.byref(h)))
        nz = cls(h)
        if leaf_flip is not None:
            lf = np.ascontiguousarray(np.asarray(leaf_flip, np.uint32))
            assert lf.size == lu.size
            _check(lib.tqs_noise_set_flips(h, _ptr(lf, u32)))
        return nz

    def flips(self):
        """Copy of the read-out flip masks (uint32 per leaf), or None."""
        f = P(u32)()
        _check(lib.tqs_noise_flips(self.h, C.byref(f)))
        if not f:
            return None
        nl = u64()
        _check(lib.tqs_noise_view(self.h, None, None, None, None, None, C.byref(nl)))
        return np.ctypeslib.as_array(f, (nl.value,)).copy()

    def arrays(self):
        """Copies of (node_off, ev_gate, ev_code, leaf_u)."""
        no, eg, ec, lu = P(u64)(), P(u32)(), P(C.c_uint8)(), P(dbl)()
        nn, nl = u64(), u64()
        _check(lib.tqs_noise_view(self.h, C.byref(no), C.byref(eg), C.byref(ec), C.byref(lu),
                                  C.byref(nn), C.byref(nl)))
        node_off = np.ctypeslib.as_array(no, (nn.value + 1,)).copy()
        ne = int(node_off[-1])
        ev_gate = np.ctypeslib.as_array(eg, (ne,)).copy() if ne else np.zeros(0, np.uint32)
        ev_code = np.ctypeslib.as_array(ec, (ne,)).copy() if ne else np.zeros(0, np.uint8)
        leaf_u = np.ctypeslib.as_array(lu, (nl.value,)).copy()
        return node_off, ev_gate, ev_code, leaf_u

    def __del__(self):
        h = getattr(self, "h", None)
        # (at interpreter exit the module globals may already be gone)
        if h is not None and h.value and lib is not None:
            lib.tqs_noise_destroy(h)
            self.h = vp()


# -------------------------------------------------------------------- plan --

class Plan:
    """Owned tqs_plan handle."""

    def __init__(self, circuit: Circuit, tree, precision="c64", tuning=None):
        t = _Tree(*tree)
        self.tree = (list(map(int, t.A)), list(map(int, t.cut)))
        tu = None
        if tuning:
            tu = TqsTuning(**{k: int(v) for k, v in tuning.items()})
        h = vp()
        _check(lib.tqs_plan_create(circuit.h, C.byref(t.s), _PREC[precision],
                                   C.byref(tu) if tu is not None else None, C.byref(h)))
        self.h = h
        self.n = circuit.n
        self.precision = _PREC[precision]
        self.n_leaves = int(np.prod(self.tree[0], dtype=object))

    def info(self, level: int = 0):
        a, b, c = u32(), u32(), u32()
        _check(lib.tqs_plan_info(self.h, level, C.byref(a), C.byref(b), C.byref(c)))
        return {"passes_level": a.value, "passes_total": b.value, "chunk_states": c.value}

    def describe(self) -> str:
        """The plan as text (format in tqsim.h, tqs_plan_describe)."""
        n = u64()
        _check(lib.tqs_plan_describe(self.h, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib.tqs_plan_describe(self.h, buf, n.value, C.byref(n)))
        return buf.value.decode()

    def compile(self):
        """Compile the plan's specialised pass kernels now (tqs_plan_compile)."""
        _check(lib.tqs_plan_compile(self.h))

    def jit_source(self) -> str:
        """HIP source of the plan's specialised pass kernels."""
        n = u64()
        _check(lib.tqs_plan_jit_source(self.h, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib.tqs_plan_jit_source(self.h, buf, n.value, C.byref(n)))
        return buf.value.decode()

    def workspace_bytes(self, noise: Noise = None) -> int:
        b = u64()
        _check(lib.tqs_workspace_bytes(self.h, noise.h if noise is not None else None, C.byref(b)))
        return b.value

    def __del__(self):
        h = getattr(self, "h", None)
        # (at interpreter exit the module globals may already be gone)
        if h is not None and h.value and lib is not None:
            lib.tqs_plan_destroy(h)
            self.h = vp()


# --------------------------------------------------------------------- run --

class Workspace:
    """Device workspace owned by a torch uint8 tensor, 256-byte aligned."""

    def __init__(self, nbytes: int, device="cuda"):
        import torch
        self.tensor = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.tensor.data_ptr()
        self.ptr = (base + 255) & ~255
        self.nbytes = nbytes


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return vp(stream.cuda_stream)


def run(plan: Plan, noise: Noise, workspace: Workspace = None, stream=None, stats: bool = False,
        subtrees=None):
    """Simulate the tree; returns outcomes (uint64 per leaf) and, with
    ``stats``, a dict of device timings and byte counts."""
    need = plan.workspace_bytes(noise)
    if workspace is None:
        workspace = Workspace(need)
    st = TqsRunStats() if stats else None
    s = _stream(stream)
    if subtrees is None:
        out = np.zeros(plan.n_leaves, np.uint64)
        _check(lib.tqs_run(plan.h, noise.h, vp(workspace.ptr), workspace.nbytes, s,
                           _ptr(out, u64), C.byref(st) if st is not None else None))
    else:
        first, last = subtrees
        per = plan.n_leaves // plan.tree[0][0]
        out = np.zeros((last - first) * per, np.uint64)
        _check(lib.tqs_run_range(plan.h, noise.h, vp(workspace.ptr), workspace.nbytes, s,
                                 first, last, _ptr(out, u64),
                                 C.byref(st) if st is not None else None))
    return (out, st.as_dict()) if stats else out


class PendingRun:
    """A run started with ``run_start``: ``finish()`` waits for it and
    returns its outcomes (and statistics when asked for at the start)."""

    def __init__(self, h, out, stats, keep):
        self.h, self.out, self.stats, self._keep = h, out, stats, keep

    def finish(self):
        if self.h is None:
            raise RuntimeError("run already finished")
        st = TqsRunStats() if self.stats else None
        h, self.h = self.h, None
        _check(lib.tqs_run_finish(h, C.byref(st) if st is not None else None))
        self._keep = None
        return (self.out, st.as_dict()) if self.stats else self.out

    def __del__(self):
        if getattr(self, "h", None) is not None and lib is not None:
            lib.tqs_run_finish(self.h, None)


def run_start(plan: Plan, noise: Noise, workspace: Workspace, stream=None, stats: bool = False) -> PendingRun:
    """Start a run (tqs_run_start): its host work and every launch are done
    when this returns, its device work may still be running.  At most two
    runs of one plan in flight, each with its own workspace."""
    out = np.zeros(plan.n_leaves, np.uint64)
    h = vp()
    _check(lib.tqs_run_start(plan.h, noise.h, vp(workspace.ptr), workspace.nbytes, _stream(stream),
                             _ptr(out, u64), 1 if stats else 0, C.byref(h)))
    # the plan, noise and workspace stay alive while the run is in flight
    return PendingRun(h, out, stats, (plan, noise, workspace))


def run_noalloc(plan: Plan, noise: Noise, stream=None):
    """As ``run``, in the library's static device scratch (64 MiB per GPU):
    no workspace is allocated (tqs_run_noalloc)."""
    out = np.zeros(plan.n_leaves, np.uint64)
    _check(lib.tqs_run_noalloc(plan.h, noise.h, _stream(stream), _ptr(out, u64)))
    return out


def run_capture(plan: Plan, noise: Noise, leaves, workspace: Workspace = None, stream=None):
    """Outcomes of all leaves plus the final complex128 amplitudes of
    ``leaves`` (noise frame applied)."""
    need = plan.workspace_bytes(noise)
    if workspace is None:
        workspace = Workspace(need)
    lv = np.ascontiguousarray(np.asarray(leaves, np.uint64))
    amps = np.zeros((lv.size, 1 << plan.n), np.complex128)
    out = np.zeros(plan.n_leaves, np.uint64)
    _check(lib.tqs_run_capture(plan.h, noise.h, vp(workspace.ptr), workspace.nbytes, _stream(stream),
                               _ptr(out, u64), _ptr(lv, u64), lv.size,
                               amps.view(np.float64).ctypes.data_as(P(dbl))))
    return out, amps


def histogram(outcomes):
    o = np.ascontiguousarray(np.asarray(outcomes, np.uint64))
    n = o.size
    vals = np.zeros(max(n, 1), np.uint64)
    cnts = np.zeros(max(n, 1), np.uint64)
    nu = u64()
    _check(lib.tqs_histogram(_ptr(o, u64), n, _ptr(vals, u64), _ptr(cnts, u64), C.byref(nu)))
    return vals[:nu.value], cnts[:nu.value]


def probe_copy(nbytes: int, reps: int = 10, stream=None) -> float:
    """Device copy bandwidth (GB/s, read + write) of the library's streaming kernel."""
    ws = Workspace(2 * nbytes)
    g = dbl()
    _check(lib.tqs_probe_copy(vp(ws.ptr), nbytes, reps, _stream(stream), C.byref(g)))
    return g.value


class Batch:
    """Owned tqs_batch: several (plan, insertion list) runs advanced together."""

    def __init__(self, plans, noises):
        if len(plans) != len(noises) or not plans:
            raise ValueError("need one insertion list per plan")
        self._keep = (list(plans), list(noises))
        ph = (vp * len(plans))(*[p.h.value for p in plans])
        nh = (vp * len(noises))(*[n.h.value for n in noises])
        h = vp()
        _check(lib.tqs_batch_create(ph, nh, len(plans), C.byref(h)))
        self.h = h
        self.leaf_counts = [p.n_leaves for p in plans]

    def info(self):
        ws, lv, st = u64(), u64(), u32()
        _check(lib.tqs_batch_info(self.h, C.byref(ws), C.byref(lv), C.byref(st)))
        return {"workspace_bytes": ws.value, "leaves": lv.value, "steps": st.value}

    def use_graph(self, on: bool = True):
        """Record the launches once into a HIP graph and replay it on later
        runs (per workspace address)."""
        _check(lib.tqs_batch_use_graph(self.h, 1 if on else 0))
        return self

    def run(self, workspace=None, stream=None, stats=False):
        """Per-run outcome arrays (and the stats dict with ``stats``)."""
        info = self.info()
        if workspace is None:
            workspace = Workspace(info["workspace_bytes"])
        out = np.zeros(info["leaves"], np.uint64)
        st = TqsRunStats() if stats else None
        _check(lib.tqs_batch_run(self.h, vp(workspace.ptr), workspace.nbytes, _stream(stream), _ptr(out, u64),
                                 C.byref(st) if st is not None else None))
        parts, o = [], 0
        for k in self.leaf_counts:
            parts.append(out[o:o + k])
            o += k
        return (parts, st.as_dict()) if stats else parts

    def __del__(self):
        h = getattr(self, "h", None)
        # (at interpreter exit the module globals may already be gone)
        if h is not None and h.value and lib is not None:
            lib.tqs_batch_destroy(h)


class Perceptron:
    """The library's two-hidden-layer perceptron on device tensors (torch
    float32 on the GPU): forward, loss gradient and Adam run in the
    library's kernels; torch only holds the memory."""

    def __init__(self, d_in: int, hidden: int, d_out: int, params=None, seed: int = 0):
        import torch
        self.d_in, self.h, self.d_out = int(d_in), int(hidden), int(d_out)
        self.count = int(lib.tqs_mlp_param_count(self.d_in, self.h, self.d_out))
        if params is None:
            # He-uniform weights, zero biases (host draw, then one copy)
            rng = np.random.default_rng(seed)
            p = np.zeros(self.count, np.float32)
            o = 0
            for fan_in, fan_out in ((self.d_in, self.h), (self.h, self.h), (self.h, self.d_out)):
                lim = np.sqrt(6.0 / fan_in)
                p[o:o + fan_in * fan_out] = rng.uniform(-lim, lim, fan_in * fan_out)
                o += fan_in * fan_out + fan_out
            params = p
        params = np.ascontiguousarray(np.asarray(params, np.float32))
        if params.size != self.count:
            raise ValueError("expected %d parameters, got %d" % (self.count, params.size))
        self.params = torch.from_numpy(params).cuda()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.step = 0
        self._scratch = None

    def _scr(self, batch):
        import torch
        need = int(lib.tqs_mlp_scratch_floats(self.d_in, self.h, self.d_out, batch))
        if self._scratch is None or self._scratch.numel() < need:
            self._scratch = torch.empty(need, dtype=torch.float32, device="cuda")
        return self._scratch

    @staticmethod
    def _dev(a):
        import torch
        t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32)))
        return t.to(device="cuda", dtype=torch.float32).contiguous()

    def forward(self, x):
        import torch
        x = self._dev(x)
        b = x.shape[0]
        y = torch.empty((b, self.d_out), dtype=torch.float32, device="cuda")
        s = _stream(None)
        _check(lib.tqs_mlp_forward(vp(self.params.data_ptr()), self.d_in, self.h, self.d_out,
                                   vp(x.data_ptr()), b, vp(y.data_ptr()), vp(self._scr(b).data_ptr()), s))
        return y

    def loss_grad(self, x, target, weight):
        """Loss (device scalar) and the gradient (into self.grad)."""
        import torch
        x, t, w = self._dev(x), self._dev(target), self._dev(weight)
        b = x.shape[0]
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(lib.tqs_mlp_loss_grad(vp(self.params.data_ptr()), self.d_in, self.h, self.d_out,
                                     vp(x.data_ptr()), vp(t.data_ptr()), vp(w.data_ptr()), b,
                                     vp(self.grad.data_ptr()), vp(loss.data_ptr()),
                                     vp(self._scr(b).data_ptr()), _stream(None)))
        return loss

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        _check(lib.tqs_mlp_adam(vp(self.params.data_ptr()), vp(self.grad.data_ptr()), vp(self.m.data_ptr()),
                                vp(self.v.data_ptr()), self.count, lr, beta1, beta2, eps, self.step,
                                _stream(None)))
