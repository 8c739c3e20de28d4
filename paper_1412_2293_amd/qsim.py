"""ctypes binding of libqsim (include/qsim.h): argument marshalling only.

Every entry point has the same name as its C function without the ``qs_`` prefix.  Device
buffers are torch tensors on a ROCm device; streams are torch streams.  A failing call raises
QsimError with the library's message.  If libqsim.so has not been built this module raises
on first use: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsim.so")

C64, C128 = 0, 1
U1, CP, SWAP, CNOT, U2, FLIP, DIAG = 0, 1, 2, 3, 4, 5, 6
NOISE_NONE, NOISE_ROT, NOISE_PHASE = 0, 1, 2

__all__ = ["QsimError", "lib", "Gate", "Noise", "Plan", "C64", "C128", "gate_array",
           "sv_bytes_required", "StateVector", "apply_gate", "apply_kraus", "fidelity",
           "dm_fidelity", "fidelity_noalloc", "dm_apply_gate", "noise_draw", "traj_bytes_required", "run_trajectories",
           "timing_enable", "timing_read", "plan_describe", "plan_choose", "traj_layout", "timing_reset", "copy", "FixedRank", "trajectory_states",
           "fr_bytes_required", "kraus_cp", "dm_superop", "dm_run_bytes_required", "dm_run", "dm_state", "TrajGraph", "Server", "SrvConfig", "SrvJobInfo", "SrvStats", "LIB_PATH"]


class QsimError(RuntimeError):
    pass


class Gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("q0", ctypes.c_int32), ("q1", ctypes.c_int32),
                ("noise", ctypes.c_int32), ("site", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("theta", ctypes.c_double), ("mask", ctypes.c_uint64), ("value", ctypes.c_uint64),
                ("m", ctypes.c_double * 32)]


class Noise(ctypes.Structure):
    _fields_ = [("e", ctypes.c_double), ("seed", ctypes.c_uint64), ("request", ctypes.c_uint32),
                ("traj_base", ctypes.c_uint32), ("e_per_traj", ctypes.POINTER(ctypes.c_double))]


class Plan(ctypes.Structure):
    _fields_ = [("fuse", ctypes.c_int32), ("tile_bits", ctypes.c_int32),
                ("reg_bits", ctypes.c_int32), ("run_bits", ctypes.c_int32), ("mfma", ctypes.c_int32)]


class SrvConfig(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("max_chunk_traj", ctypes.c_int32), ("reserved", ctypes.c_int32), ("plan", Plan)]


class SrvJobInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_chunks", ctypes.c_int32), ("chunk_traj", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("chunk_bytes", ctypes.c_uint64), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("latency_s", ctypes.c_double),
                ("queue_s", ctypes.c_double)]


class SrvStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("trajectories", ctypes.c_uint64), ("chunks", ctypes.c_uint64),
                ("admission_waits", ctypes.c_uint64), ("pool_bytes", ctypes.c_uint64),
                ("peak_bytes", ctypes.c_uint64), ("in_use_bytes", ctypes.c_uint64),
                ("peak_inflight", ctypes.c_int32), ("inflight", ctypes.c_int32), ("queued", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("busy_s", ctypes.c_double), ("elapsed_s", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise QsimError(f"{LIB_PATH} is missing: build it with paper_1412_2293_amd/build.py "
                        "(or __graft_entry__.build()); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, u64, dbl, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                      ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double,
                                      ctypes.c_size_t)
    st = ctypes.c_int
    sigs = {
        "qs_last_error": ([], ctypes.c_char_p),
        "qs_version": ([], ctypes.c_char_p),
        "qs_sv_bytes_required": ([i32, i32, i32], sz),
        "qs_sv_create": ([i32, i32, i32, P, sz, P, ctypes.POINTER(P)], st),
        "qs_sv_destroy": ([P], st),
        "qs_sv_init_basis": ([P, u64], st),
        "qs_apply_gate": ([P, ctypes.POINTER(Gate), ctypes.POINTER(Noise)], st),
        "qs_apply_kraus": ([P, i32, P, i32, P], st),
        "qs_fidelity": ([P, i32, P, i32, P, P], st),
        "qs_dm_apply_gate": ([P, ctypes.POINTER(Gate), dbl], st),
        "qs_fr_apply_noisy_gate": ([P, ctypes.POINTER(Gate), dbl, dbl, dbl, P], st),
        "qs_dm_fidelity": ([P, P, i32, P, P], st),
        "qs_noise_draw": ([u64, u32, u32, P, i32, u32, i32, P, P], st),
        "qs_traj_bytes_required": ([P, i32, i32, i32, i32, ctypes.POINTER(Plan)], sz),
        "qs_run_trajectories": ([P, i32, i32, u64, i32, ctypes.POINTER(Noise), i32, i64,
                                 ctypes.POINTER(Plan), P, sz, P, P, P, P, P], st),
        "qs_timing_enable": ([i32], st),
        "qs_traj_layout": ([P, i32, i32, i32, i32, ctypes.POINTER(Plan), P], st),
        "qs_plan_describe": ([P, i32, i32, i32, ctypes.POINTER(Plan), ctypes.c_char_p, sz, P], st),
        "qs_plan_choose": ([P, i32, i32, i32, ctypes.POINTER(Plan), ctypes.POINTER(dbl)], st),
        "qs_timing_read": ([ctypes.c_char_p, P, P, P], st),
        "qs_timing_reset": ([], st),
        "qs_copy": ([P, P, sz, P], st),
        "qs_fr_bytes_required": ([i32, i32, i32], sz),
        "qs_fr_create": ([i32, i32, i32, P, sz, P, ctypes.POINTER(P)], st),
        "qs_fr_destroy": ([P], st),
        "qs_fr_init_basis": ([P, u64], st),
        "qs_fr_apply_gate": ([P, ctypes.POINTER(Gate)], st),
        "qs_fr_apply_kraus": ([P, i32, i32, P, dbl, dbl, P], st),
        "qs_fr_apply_kraus2": ([P, i32, i32, i32, P, dbl, dbl, P], st),
        "qs_kraus_cp": ([dbl, dbl, i32, P], st),
        "qs_fidelity_noalloc": ([P, P, i32, i32, P, P], st),
        "qs_dm_superop": ([P, i32, i32, dbl, P, i32, ctypes.POINTER(ctypes.c_int)], st),
        "qs_dm_run_bytes_required": ([P, i32, i32, i32, dbl, ctypes.POINTER(Plan)], sz),
        "qs_dm_run": ([P, i32, i32, u64, i32, dbl, ctypes.POINTER(Plan), P, P, sz, P, P, P, P], st),
        "qs_fr_fidelity": ([P, P, i32, P, P, P], st),
        "qs_fr_info": ([P, P, P, P], st),
        "qs_traj_graph_bytes_required": ([P, i32, i32, i32, i32, ctypes.POINTER(Plan), ctypes.POINTER(sz)], st),
        "qs_traj_graph_create": ([P, i32, i32, i32, i32, ctypes.POINTER(Plan), P, sz, ctypes.POINTER(P)], st),
        "qs_traj_graph_launch": ([P, u64, ctypes.POINTER(Noise), i64, P, P, P, P], st),
        "qs_traj_graph_destroy": ([P], st),
        "qs_srv_create": ([ctypes.POINTER(SrvConfig), P, sz, ctypes.POINTER(P)], st),
        "qs_srv_submit": ([P, P, i32, i32, u64, ctypes.POINTER(Noise), i32, i64, ctypes.POINTER(u64)], st),
        "qs_srv_poll": ([P, u64, ctypes.POINTER(ctypes.c_int)], st),
        "qs_srv_wait": ([P, u64, dbl], st),
        "qs_srv_result": ([P, u64, P, P, P, ctypes.POINTER(SrvJobInfo)], st),
        "qs_srv_stats_get": ([P, ctypes.POINTER(SrvStats)], st),
        "qs_srv_destroy": ([P], st),
    }
    for name, (args, res) in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(status: int, what: str):
    if status != 0:
        msg = lib().qs_last_error().decode(errors="replace")
        raise QsimError(f"{what} failed ({status}): {msg}")


def _ptr(t) -> ctypes.c_void_p:
    if t is None:
        return ctypes.c_void_p(0)
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(ctypes.c_void_p)
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------------------------------
def make_gate(g) -> Gate:
    """Gate struct from any object with the fields of workloads.Gate."""
    out = Gate()
    out.kind, out.q0, out.q1, out.noise = int(g.kind), int(g.q0), int(g.q1), int(g.noise)
    out.site = int(g.site)
    out.theta = float(g.theta)
    out.mask, out.value = int(g.mask), int(g.value)
    if g.m is not None:
        m = np.asarray(g.m, np.complex128).reshape(-1)
        for k, z in enumerate(m):
            out.m[2 * k] = z.real
            out.m[2 * k + 1] = z.imag
    return out


def gate_array(gates) -> ctypes.Array:
    gs = list(gates)
    arr = (Gate * len(gs))()    # may be empty: the library accepts n_gates = 0
    for i, g in enumerate(gs):
        arr[i] = g if isinstance(g, Gate) else make_gate(g)
    return arr


def _noise(e=0.0, seed=0, request=0, traj_base=0, e_per_traj=None):
    nz = Noise()
    nz.e, nz.seed, nz.request, nz.traj_base = float(e), int(seed), int(request), int(traj_base)
    keep = None
    if e_per_traj is not None:
        keep = np.ascontiguousarray(e_per_traj, np.float64)
        nz.e_per_traj = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return nz, keep


# ------------------------------------------------------------------------------------------
def sv_bytes_required(n: int, dtype: int, n_traj: int) -> int:
    return int(lib().qs_sv_bytes_required(n, dtype, n_traj))


class StateVector:
    """n_traj state vectors of n qubits in a torch uint8 device buffer."""

    def __init__(self, n: int, dtype: int = C128, n_traj: int = 1, buf=None, stream=None):
        import torch
        self.n, self.dtype, self.n_traj = n, dtype, n_traj
        nbytes = sv_bytes_required(n, dtype, n_traj)
        if nbytes == 0:
            raise QsimError("sv_bytes_required rejected the arguments")
        self.buf = buf if buf is not None else torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib().qs_sv_create(n, dtype, n_traj, _ptr(self.buf), self.buf.numel() * self.buf.element_size(),
                                  _stream(stream), ctypes.byref(h)), "sv_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().qs_sv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_basis(self, index: int):
        _check(lib().qs_sv_init_basis(self.h, int(index)), "sv_init_basis")

    def amplitudes(self):
        """The states as a complex torch tensor view [n_traj, 2^n] on the device."""
        import torch
        ft = torch.float32 if self.dtype == C64 else torch.float64
        N = 1 << self.n
        v = self.buf[: sv_bytes_required(self.n, self.dtype, self.n_traj)].view(ft)
        return torch.view_as_complex(v.view(self.n_traj, N, 2))


def apply_gate(s: StateVector, g, e: float = 0.0, seed: int = 0, request: int = 0, traj_base: int = 0):
    gs = g if isinstance(g, Gate) else make_gate(g)
    nz, _ = _noise(e, seed, request, traj_base)
    _check(lib().qs_apply_gate(s.h, ctypes.byref(gs), ctypes.byref(nz) if e else None), "apply_gate")


def apply_kraus(rho: StateVector, qubits: Sequence[int], ops):
    ops = np.ascontiguousarray(np.asarray(ops, np.complex128))
    qs = np.ascontiguousarray(qubits, np.int32)
    _check(lib().qs_apply_kraus(rho.h, qs.size, _ptr(qs), ops.shape[0], _ptr(ops.view(np.float64))),
           "apply_kraus")


def dm_apply_gate(rho: StateVector, g, e: float = 0.0):
    gs = g if isinstance(g, Gate) else make_gate(g)
    _check(lib().qs_dm_apply_gate(rho.h, ctypes.byref(gs), float(e)), "dm_apply_gate")


def fidelity(a: StateVector, ta: int, b: StateVector, tb: int):
    f = ctypes.c_double()
    ov = np.zeros(2)
    _check(lib().qs_fidelity(a.h, ta, b.h, tb, ctypes.byref(f), _ptr(ov)), "fidelity")
    return f.value, complex(ov[0], ov[1])


def fidelity_noalloc(a, b, n: int, dtype: int, out, stream=None):
    """qs_fidelity_noalloc on device buffers a, b (torch tensors of one state each) into the
    device tensor out (4 float64: Re <a|b>, Im <a|b>, <a|a>, <b|b>); asynchronous."""
    _check(lib().qs_fidelity_noalloc(_ptr(a), _ptr(b), int(n), int(dtype), _stream(stream), _ptr(out)),
           "fidelity_noalloc")


def dm_fidelity(rho: StateVector, psi: StateVector, tpsi: int = 0):
    f, tr = ctypes.c_double(), ctypes.c_double()
    _check(lib().qs_dm_fidelity(rho.h, psi.h, tpsi, ctypes.byref(f), ctypes.byref(tr)), "dm_fidelity")
    return f.value, tr.value


def noise_draw(seed: int, sites, n_traj: int, traj_base: int = 0, request: int = 0, stream_id: int = 0,
               stream=None):
    """xi[t, s] drawn on the device (float64 torch tensor)."""
    import torch
    sites_t = torch.as_tensor(np.ascontiguousarray(sites, np.uint32).view(np.int32), device="cuda")
    out = torch.empty((n_traj, sites_t.numel()), dtype=torch.float64, device="cuda")
    _check(lib().qs_noise_draw(int(seed), int(request), int(stream_id), _ptr(sites_t), sites_t.numel(),
                               int(traj_base), int(n_traj), _ptr(out), _stream(stream)), "noise_draw")
    return out


def _plan(plan):
    if plan is None:
        return None
    if isinstance(plan, Plan):
        return plan
    p = Plan()
    p.fuse = int(plan.get("fuse", -1))
    p.tile_bits = int(plan.get("tile_bits", 0))
    p.reg_bits = int(plan.get("reg_bits", 0))
    p.run_bits = int(plan.get("run_bits", 0))
    p.mfma = int(plan.get("mfma", 0))
    return p


def traj_bytes_required(gates, n: int, dtype: int, n_traj: int, plan=None) -> int:
    ga = gates if isinstance(gates, ctypes.Array) else gate_array(gates)
    p = _plan(plan)
    return int(lib().qs_traj_bytes_required(ga, len(ga), n, dtype, n_traj,
                                            ctypes.byref(p) if p is not None else None))


def run_trajectories(gates, n: int, init_index: int, dtype: int, n_traj: int, e=0.0, seed: int = 0,
                     request: int = 0, traj_base: int = 0, marked: int = -1, plan=None, buf=None,
                     stream=None, n_gates: Optional[int] = None):
    """Run the ideal circuit and n_traj noisy trajectories; returns a dict with numpy arrays
    F, p (if marked >= 0), norm, layout and the device buffer holding the final states."""
    import torch
    ga = gates if isinstance(gates, ctypes.Array) else gate_array(gates)
    G = len(ga) if n_gates is None else n_gates
    p = _plan(plan)
    e_arr = np.asarray(e, np.float64)
    per = None if e_arr.ndim == 0 else e_arr
    nz, keep = _noise(float(e_arr) if per is None else 0.0, seed, request, traj_base, per)
    need = int(lib().qs_traj_bytes_required(ga, G, n, dtype, n_traj, ctypes.byref(p) if p else None))
    if need == 0:
        raise QsimError("traj_bytes_required rejected the arguments: " + lib().qs_last_error().decode())
    if buf is None:
        buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    F = np.zeros(n_traj)
    P = np.zeros(n_traj)
    norms = np.zeros(n_traj)
    layout = np.zeros(n, np.int32)
    _check(lib().qs_run_trajectories(ga, G, n, int(init_index), dtype, ctypes.byref(nz), n_traj,
                                     int(marked), ctypes.byref(p) if p else None, _ptr(buf),
                                     buf.numel() * buf.element_size(), _stream(stream), _ptr(F),
                                     _ptr(P) if marked >= 0 else None, _ptr(norms), _ptr(layout)),
           "run_trajectories")
    del keep
    return {"F": F, "p": P if marked >= 0 else None, "norm": norms, "layout": layout, "buf": buf}


def dm_superop(gates, n: int, e: float = 0.0) -> ctypes.Array:
    """The noiseless 2n-qubit circuit on vec(rho) that the library builds for a density-matrix
    run of the noisy circuit (qs_dm_superop)."""
    ga = gates if isinstance(gates, ctypes.Array) else gate_array(gates)
    cnt = ctypes.c_int(0)
    _check(lib().qs_dm_superop(ga, len(ga), n, float(e), None, 0, ctypes.byref(cnt)), "dm_superop")
    out = (Gate * max(cnt.value, 1))()
    _check(lib().qs_dm_superop(ga, len(ga), n, float(e), out, len(out), ctypes.byref(cnt)), "dm_superop")
    return (Gate * cnt.value).from_buffer(out) if cnt.value else (Gate * 0)()


def dm_run_bytes_required(gates, n: int, dtype: int, e: float = 0.0, plan=None) -> int:
    ga = gates if isinstance(gates, ctypes.Array) else gate_array(gates)
    p = _plan(plan)
    return int(lib().qs_dm_run_bytes_required(ga, len(ga), n, dtype, float(e), ctypes.byref(p) if p else None))


def dm_run(gates, n: int, init_index: int, dtype: int, psi, e: float = 0.0, plan=None, buf=None, stream=None):
    """Density-matrix run of the noisy circuit (qs_dm_run): returns a dict with F =
    <psi|rho|psi>, trace, layout and the device buffer whose first 4^n amplitudes are vec(rho)
    (row bit q at layout[q] + n, column bit q at layout[q]).  psi: the n-qubit state (device
    tensor or StateVector, logical order) to take the expectation with."""
    import torch
    ga = gates if isinstance(gates, ctypes.Array) else gate_array(gates)
    p = _plan(plan)
    need = int(lib().qs_dm_run_bytes_required(ga, len(ga), n, dtype, float(e), ctypes.byref(p) if p else None))
    if need == 0:
        raise QsimError("dm_run_bytes_required rejected the arguments: " + lib().qs_last_error().decode())
    if buf is None:
        buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    psi_ptr = ctypes.c_void_p(psi.buf.data_ptr()) if isinstance(psi, StateVector) else _ptr(psi)
    f = ctypes.c_double(0.0)
    tr = ctypes.c_double(0.0)
    layout = np.zeros(n, np.int32)
    _check(lib().qs_dm_run(ga, len(ga), n, int(init_index), dtype, float(e), ctypes.byref(p) if p else None,
                           psi_ptr, _ptr(buf), buf.numel() * buf.element_size(), _stream(stream),
                           ctypes.byref(f), ctypes.byref(tr), _ptr(layout)), "dm_run")
    return {"F": f.value, "trace": tr.value, "layout": layout, "buf": buf}


def dm_state(res, n: int, dtype: int):
    """vec(rho) of a dm_run result as a complex torch tensor view [4^n] (physical order)."""
    import torch
    ft = torch.float32 if dtype == C64 else torch.float64
    N = 1 << (2 * n)
    nbytes = N * (8 if dtype == C64 else 16)
    return torch.view_as_complex(res["buf"][:nbytes].view(ft).view(N, 2))


def trajectory_states(res, n: int, dtype: int, n_traj: int):
    """Final states (slot 0 = ideal) as a complex torch tensor view [n_traj + 1, 2^n] in the
    physical qubit order res['layout']."""
    import torch
    ft = torch.float32 if dtype == C64 else torch.float64
    N = 1 << n
    nbytes = (n_traj + 1) * N * (8 if dtype == C64 else 16)
    return torch.view_as_complex(res["buf"][:nbytes].view(ft).view(n_traj + 1, N, 2))


def traj_layout(gates, n: int, dtype: int, n_traj: int, plan=None) -> dict:
    """Byte offsets of the regions of the run_trajectories buffer."""
    ga = gates if isinstance(gates, ctypes.Array) else gate_array(gates)
    p = _plan(plan)
    out = np.zeros(17, np.uint64)
    _check(lib().qs_traj_layout(ga, len(ga), n, dtype, n_traj, ctypes.byref(p) if p else None, _ptr(out)),
           "traj_layout")
    names = ["states", "tab", "gates", "edev", "passes", "stages", "rounds", "ops", "prefs", "jobs",
             "obits", "chains", "wtab", "rec", "partials", "out", "total"]
    return {k: int(v) for k, v in zip(names, out)}


def plan_choose(gates, n: int, dtype: int):
    """The plan the library picks for fuse = -1 and its modelled seconds per state slot."""
    ga = gates if isinstance(gates, ctypes.Array) else gate_array(gates)
    p = Plan()
    cost = ctypes.c_double()
    _check(lib().qs_plan_choose(ga, len(ga), n, dtype, ctypes.byref(p), ctypes.byref(cost)), "plan_choose")
    out = {"fuse": p.fuse, "tile_bits": p.tile_bits, "reg_bits": p.reg_bits, "run_bits": p.run_bits}
    if p.mfma:
        out["mfma"] = 1
    return out, cost.value


def plan_describe(gates, n: int, dtype: int, plan=None) -> dict:
    """The fused-pass program the library builds for this circuit (parsed JSON)."""
    import json
    ga = gates if isinstance(gates, ctypes.Array) else gate_array(gates)
    p = _plan(plan)
    ln = ctypes.c_size_t()
    _check(lib().qs_plan_describe(ga, len(ga), n, dtype, ctypes.byref(p) if p else None, None, 0,
                                  ctypes.byref(ln)), "plan_describe")
    buf = ctypes.create_string_buffer(ln.value + 1)
    _check(lib().qs_plan_describe(ga, len(ga), n, dtype, ctypes.byref(p) if p else None, buf,
                                  ln.value + 1, ctypes.byref(ln)), "plan_describe")
    return json.loads(buf.value.decode())


def timing_enable(on: bool = True):
    _check(lib().qs_timing_enable(1 if on else 0), "timing_enable")


def timing_reset():
    _check(lib().qs_timing_reset(), "timing_reset")


def timing_read(name: str):
    n, ms, b = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    _check(lib().qs_timing_read(name.encode(), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(b)),
           "timing_read")
    return {"launches": n.value, "ms": ms.value, "alg_bytes": b.value}


def copy(dst, src, nbytes: int, stream=None):
    _check(lib().qs_copy(_ptr(dst), _ptr(src), int(nbytes), _stream(stream)), "copy")


def kraus_cp(theta: float, e: float, improved: bool = False) -> np.ndarray:
    """(2, 4, 4) complex128: the noisy controlled phase's Kraus pair built by the library
    (qs_kraus_cp: eq. 9, or eq. 14 when improved)."""
    out = np.zeros((2, 4, 4), np.complex128)
    _check(lib().qs_kraus_cp(float(theta), float(e), int(improved), _ptr(out.view(np.float64))), "kraus_cp")
    return out


def fr_bytes_required(n: int, r: int, dtype: int) -> int:
    return int(lib().qs_fr_bytes_required(n, r, dtype))


class FixedRank:
    """Fixed-rank density matrix: rho = exp(log_trace) sum_j |v_j><v_j|, at most r columns."""

    def __init__(self, n: int, r: int, dtype: int = C128, buf=None, stream=None):
        import torch
        self.n, self.r, self.dtype = n, r, dtype
        nbytes = fr_bytes_required(n, r, dtype)
        if nbytes == 0:
            raise QsimError("fr_bytes_required rejected the arguments")
        self.buf = buf if buf is not None else torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        _check(lib().qs_fr_create(n, r, dtype, _ptr(self.buf), self.buf.numel(), _stream(stream),
                                  ctypes.byref(h)), "fr_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().qs_fr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_basis(self, index: int):
        _check(lib().qs_fr_init_basis(self.h, int(index)), "fr_init_basis")

    def apply_gate(self, g):
        gs = g if isinstance(g, Gate) else make_gate(g)
        _check(lib().qs_fr_apply_gate(self.h, ctypes.byref(gs)), "fr_apply_gate")

    def apply_kraus(self, q: int, ops, tau: float = 1e-9, zero_tol: float = 1e-13) -> int:
        ops = np.ascontiguousarray(np.asarray(ops, np.complex128))
        rank = ctypes.c_int()
        _check(lib().qs_fr_apply_kraus(self.h, int(q), ops.shape[0], _ptr(ops.view(np.float64)),
                                       float(tau), float(zero_tol), ctypes.byref(rank)), "fr_apply_kraus")
        return rank.value

    def apply_kraus2(self, q0: int, q1: int, ops, tau: float = 1e-9, zero_tol: float = 1e-13) -> int:
        ops = np.ascontiguousarray(np.asarray(ops, np.complex128))
        rank = ctypes.c_int()
        _check(lib().qs_fr_apply_kraus2(self.h, int(q0), int(q1), ops.shape[0], _ptr(ops.view(np.float64)),
                                        float(tau), float(zero_tol), ctypes.byref(rank)), "fr_apply_kraus2")
        return rank.value

    def apply_noisy_gate(self, g, e: float, tau: float = 1e-9, zero_tol: float = 1e-13) -> int:
        gs = g if isinstance(g, Gate) else make_gate(g)
        rank = ctypes.c_int()
        _check(lib().qs_fr_apply_noisy_gate(self.h, ctypes.byref(gs), float(e), float(tau), float(zero_tol),
                                            ctypes.byref(rank)), "fr_apply_noisy_gate")
        return rank.value

    def fidelity(self, psi: StateVector, tpsi: int = 0):
        fu, fn, lt = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().qs_fr_fidelity(self.h, psi.h, tpsi, ctypes.byref(fu), ctypes.byref(fn), ctypes.byref(lt)),
               "fr_fidelity")
        return fu.value, fn.value, lt.value

    def info(self):
        rank, lt, ptr = ctypes.c_int(), ctypes.c_double(), ctypes.c_void_p()
        _check(lib().qs_fr_info(self.h, ctypes.byref(rank), ctypes.byref(lt), ctypes.byref(ptr)), "fr_info")
        return rank.value, lt.value

    def columns(self):
        import torch
        ft = torch.float32 if self.dtype == C64 else torch.float64
        N = 1 << self.n
        return torch.view_as_complex(self.buf[: fr_bytes_required(self.n, self.r, self.dtype)]
                                     .view(ft).view(self.r, N, 2))


# ------------------------------------------------------------------------------------------
class TrajGraph:
    """A captured run_trajectories launch sequence for one circuit, n_traj and buffer; launch()
    replays it with new noise parameters, initial index and marked index."""

    def __init__(self, gates, n: int, dtype: int, n_traj: int, plan=None, buf=None):
        import torch
        self.ga = gates if isinstance(gates, ctypes.Array) else gate_array(gates)
        self.n, self.dtype, self.n_traj = n, dtype, n_traj
        p = _plan(plan)
        need = ctypes.c_size_t()
        _check(lib().qs_traj_graph_bytes_required(self.ga, len(self.ga), n, dtype, n_traj,
                                                  ctypes.byref(p) if p else None, ctypes.byref(need)),
               "traj_graph_bytes_required")
        self.buf = buf if buf is not None else torch.empty(need.value, dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        _check(lib().qs_traj_graph_create(self.ga, len(self.ga), n, dtype, n_traj, ctypes.byref(p) if p else None,
                                          _ptr(self.buf), self.buf.numel(), ctypes.byref(h)), "traj_graph_create")
        self.h = h

    def launch(self, init_index: int, e=0.0, seed: int = 0, request: int = 0, traj_base: int = 0,
               marked: int = -1) -> dict:
        e_arr = np.asarray(e, np.float64)
        per = None if e_arr.ndim == 0 else e_arr
        nz, keep = _noise(float(e_arr) if per is None else 0.0, seed, request, traj_base, per)
        T = self.n_traj
        F, P, norms, layout = np.zeros(T), np.zeros(T), np.zeros(T), np.zeros(self.n, np.int32)
        _check(lib().qs_traj_graph_launch(self.h, int(init_index), ctypes.byref(nz), int(marked), _ptr(F),
                                          _ptr(P) if marked >= 0 else None, _ptr(norms), _ptr(layout)),
               "traj_graph_launch")
        del keep
        return {"F": F, "p": P if marked >= 0 else None, "norm": norms, "layout": layout, "buf": self.buf}

    def close(self):
        if getattr(self, "h", None):
            lib().qs_traj_graph_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------------------------
def _struct_dict(x) -> dict:
    return {name: getattr(x, name) for name, _ in x._fields_ if name != "reserved"}


class Server:
    """Continuous-batching request server over one device pool (qs_srv_*).  submit() returns a
    request id; result() blocks until the request has finished and returns F, p, norm and its
    timing."""

    def __init__(self, pool_bytes: int, dtype: int = C64, max_inflight: int = 4,
                 max_chunk_traj: int = 256, plan=None, pool=None):
        import torch
        self.dtype = dtype
        self.pool = pool if pool is not None else torch.empty(int(pool_bytes), dtype=torch.uint8, device="cuda")
        cfg = SrvConfig()
        cfg.dtype = dtype
        cfg.max_inflight = max_inflight
        cfg.max_chunk_traj = max_chunk_traj
        p = _plan(plan)
        if p is not None:
            cfg.plan = p
        else:
            cfg.plan.fuse = -1
        h = ctypes.c_void_p()
        _check(lib().qs_srv_create(ctypes.byref(cfg), _ptr(self.pool), self.pool.numel(), ctypes.byref(h)),
               "srv_create")
        self.h = h
        self._meta = {}

    def submit(self, gates, n: int, init_index: int, n_traj: int, e=0.0, seed: int = 0, request: int = 0,
               traj_base: int = 0, marked: int = -1) -> int:
        ga = gates if isinstance(gates, ctypes.Array) else gate_array(gates)
        e_arr = np.asarray(e, np.float64)
        per = None if e_arr.ndim == 0 else e_arr
        nz, keep = _noise(float(e_arr) if per is None else 0.0, seed, request, traj_base, per)
        jid = ctypes.c_uint64()
        _check(lib().qs_srv_submit(self.h, ga, len(ga), n, int(init_index), ctypes.byref(nz), n_traj,
                                   int(marked), ctypes.byref(jid)), "srv_submit")
        del keep
        self._meta[jid.value] = (n_traj, marked)
        return jid.value

    def poll(self, job: int) -> bool:
        d = ctypes.c_int()
        _check(lib().qs_srv_poll(self.h, job, ctypes.byref(d)), "srv_poll")
        return bool(d.value)

    def wait(self, job: int, timeout: float = -1.0):
        _check(lib().qs_srv_wait(self.h, job, float(timeout)), "srv_wait")

    def result(self, job: int, timeout: float = -1.0) -> dict:
        self.wait(job, timeout)
        n_traj, marked = self._meta.pop(job)
        F, P, norms = np.zeros(n_traj), np.zeros(n_traj), np.zeros(n_traj)
        info = SrvJobInfo()
        _check(lib().qs_srv_result(self.h, job, _ptr(F), _ptr(P) if marked >= 0 else None, _ptr(norms),
                                   ctypes.byref(info)), "srv_result")
        return {"F": F, "p": P if marked >= 0 else None, "norm": norms, "info": _struct_dict(info)}

    def stats(self) -> dict:
        s = SrvStats()
        _check(lib().qs_srv_stats_get(self.h, ctypes.byref(s)), "srv_stats")
        return _struct_dict(s)

    def close(self):
        if getattr(self, "h", None):
            _check(lib().qs_srv_destroy(self.h), "srv_destroy")
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
