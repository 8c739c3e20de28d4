"""CPU FP64 oracle for the noisy quantum-circuit method of arXiv:1412.2293.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the CPU-baseline
leg of the benchmark, never by the HIP library or its Python binding.  It shares no code
with the HIP path; both sides read the same seeded circuit description from ``workloads``.

Parts:
  * ``qsim_oracle.c`` (plain C loops, built into ``liboracle.so``): Philox4x32-10, the
    Box-Muller normal deviate, Monte Carlo state-vector trajectories (Section 2, eq. 1-2),
    the exact density matrix with Kraus channels (Section 3, eq. 3, 6, 9).
  * ``fixed_rank.py`` (numpy): the fixed-rank density-matrix approximation (Section 3.2).

Parity pinned by the not-gpu tests: Philox words against rocRAND's Philox4x32-10, the
normal transform against libm and its moments, gates against Kronecker-product matrices,
Grover and QFT closed forms, the noisy-QFT product closed form per trajectory, trace and
norm preservation, the Kraus channel against the Monte Carlo mean, eq. (10) for rank 1.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qsim_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile qsim_oracle.c with gcc into liboracle.so (next to the source)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, u64, u32, i32, dbl = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32,
                                   ctypes.c_int, ctypes.c_double)
        L.or_philox_batch.argtypes = [i64, P, P, P]
        L.or_log.argtypes = [dbl]
        L.or_log.restype = dbl
        L.or_cos2pi.argtypes = [dbl]
        L.or_cos2pi.restype = dbl
        L.or_normal.argtypes = [u64, u32, u32, u32, u32]
        L.or_normal.restype = dbl
        L.or_normals.argtypes = [u64, u32, u32, i64, P, i64, P, P]
        circ = [i64, P, P, P, P, P, P, P, P, P]
        L.or_sv_apply_circuit.argtypes = [i32] + circ + [dbl, u64, u32, u32, P]
        L.or_sv_apply_circuit.restype = i32
        L.or_sv_run.argtypes = [i32] + circ + [dbl, u64, u32, u32, u64, P]
        L.or_sv_run.restype = i32
        L.or_inner.argtypes = [i64, P, P, P, P, P, P]
        L.or_dm_apply_kraus.argtypes = [i32, P, i32, P, i32, P]
        L.or_dm_apply_kraus.restype = i32
        L.or_dm_run.argtypes = [i32, i64, P, P, P, P, P, P, P, P, dbl, u64, P]
        L.or_dm_run.restype = i32
        L.or_dm_expect.argtypes = [i32, P, P, P, P, P, P]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class FlatCircuit:
    """The oracle's own flat-array view of a ``workloads.Circuit``."""

    def __init__(self, circuit):
        G = len(circuit.gates)
        self.n = circuit.n
        self.kind = np.zeros(G, np.int32)
        self.q0 = np.zeros(G, np.int32)
        self.q1 = np.zeros(G, np.int32)
        self.noise = np.zeros(G, np.int32)
        self.site = np.zeros(G, np.uint32)
        self.mats = np.zeros((G, 32), np.float64)
        self.theta = np.zeros(G, np.float64)
        self.mask = np.zeros(G, np.uint64)
        self.value = np.zeros(G, np.uint64)
        for i, g in enumerate(circuit.gates):
            self.kind[i], self.q0[i], self.q1[i] = g.kind, g.q0, g.q1
            self.noise[i], self.site[i], self.theta[i] = g.noise, g.site, g.theta
            self.mask[i], self.value[i] = g.mask, g.value
            if g.m is not None:
                m = np.asarray(g.m, np.complex128).reshape(-1)
                self.mats[i, : 2 * m.size : 2] = m.real
                self.mats[i, 1 : 2 * m.size : 2] = m.imag
        self.n_gates = G

    def args(self):
        return [ctypes.c_int64(self.n_gates), _ptr(self.kind), _ptr(self.q0), _ptr(self.q1),
                _ptr(self.noise), _ptr(self.site), _ptr(self.mats), _ptr(self.theta),
                _ptr(self.mask), _ptr(self.value)]


# ------------------------------------------------------------------------------------------
# Noise draws
# ------------------------------------------------------------------------------------------
def philox(ctrs: np.ndarray, keys: np.ndarray) -> np.ndarray:
    """Philox4x32-10 words for each row of ctrs (k x 4 uint32) under keys (k x 2 uint32)."""
    ctrs = np.ascontiguousarray(ctrs, np.uint32).reshape(-1, 4)
    keys = np.ascontiguousarray(keys, np.uint32).reshape(-1, 2)
    assert ctrs.shape[0] == keys.shape[0]
    out = np.zeros_like(ctrs)
    lib().or_philox_batch(ctrs.shape[0], _ptr(ctrs), _ptr(keys), _ptr(out))
    return out


def normals(seed: int, sites, trajs, request: int = 0, stream: int = 0) -> np.ndarray:
    """xi[t, s] for the given trajectory ids and site ids (float64)."""
    sites = np.ascontiguousarray(sites, np.uint32)
    trajs = np.ascontiguousarray(trajs, np.uint32)
    out = np.zeros((trajs.size, sites.size), np.float64)
    lib().or_normals(ctypes.c_uint64(seed), request, stream, sites.size, _ptr(sites),
                     trajs.size, _ptr(trajs), _ptr(out))
    return out


def log(x: float) -> float:
    return lib().or_log(x)


def cos2pi(u: float) -> float:
    return lib().or_cos2pi(u)


# ------------------------------------------------------------------------------------------
# State-vector level
# ------------------------------------------------------------------------------------------
def sv_run(circuit, e: float = 0.0, seed: int = 0, traj: int = 0, request: int = 0,
           init_index=None, flat: FlatCircuit = None) -> np.ndarray:
    """Final state of one Monte Carlo trajectory (e = 0: the ideal circuit)."""
    flat = flat or FlatCircuit(circuit)
    init = circuit.init_index if init_index is None else init_index
    psi = np.zeros(1 << circuit.n, np.complex128)
    st = lib().or_sv_run(circuit.n, *flat.args(), ctypes.c_double(e), ctypes.c_uint64(seed),
                         request, traj, ctypes.c_uint64(init), _ptr(psi))
    if st != 0:
        raise ValueError("oracle sv_run rejected its arguments")
    return psi


def sv_apply(circuit, psi: np.ndarray, e: float = 0.0, seed: int = 0, traj: int = 0,
             request: int = 0) -> np.ndarray:
    """Apply the circuit to a copy of psi."""
    flat = FlatCircuit(circuit)
    out = np.array(psi, np.complex128, copy=True)
    st = lib().or_sv_apply_circuit(circuit.n, *flat.args(), ctypes.c_double(e),
                                   ctypes.c_uint64(seed), request, traj, _ptr(out))
    if st != 0:
        raise ValueError("oracle sv_apply rejected its arguments")
    return out


def inner(a: np.ndarray, b: np.ndarray):
    """(<a|b>, <a|a>, <b|b>) summed in index order."""
    a = np.ascontiguousarray(a, np.complex128)
    b = np.ascontiguousarray(b, np.complex128)
    re, im, na, nb = (ctypes.c_double() for _ in range(4))
    lib().or_inner(a.size, _ptr(a), _ptr(b), ctypes.byref(re), ctypes.byref(im),
                   ctypes.byref(na), ctypes.byref(nb))
    return complex(re.value, im.value), na.value, nb.value


def fidelity(ideal: np.ndarray, psi: np.ndarray) -> float:
    """|<ideal|psi>|^2 / (<ideal|ideal> <psi|psi>)."""
    z, na, nb = inner(ideal, psi)
    return (z.real * z.real + z.imag * z.imag) / (na * nb)


def run_trajectories(circuit, e, seed: int, trajs, request: int = 0, keep_states: bool = False):
    """Fidelity to the ideal state and marked-index probability for each trajectory id.

    ``e`` is a scalar or one noise strength per trajectory.
    """
    flat = FlatCircuit(circuit)
    ideal = sv_run(circuit, 0.0, flat=flat)
    trajs = list(trajs)
    es = np.broadcast_to(np.asarray(e, np.float64), (len(trajs),))
    F = np.zeros(len(trajs))
    p = np.zeros(len(trajs))
    states = []
    for k, t in enumerate(trajs):
        psi = sv_run(circuit, float(es[k]), seed, t, request, flat=flat)
        F[k] = fidelity(ideal, psi)
        if circuit.marked is not None:
            a = psi[circuit.marked]
            p[k] = a.real * a.real + a.imag * a.imag
        if keep_states:
            states.append(psi)
    return (F, p, ideal, states) if keep_states else (F, p)


# ------------------------------------------------------------------------------------------
# Density-matrix level
# ------------------------------------------------------------------------------------------
def dm_run(circuit, e: float, init_index=None) -> np.ndarray:
    """Exact rho (2^n x 2^n) after the circuit with every noisy gate as its Kraus channel."""
    n = circuit.n
    flat = FlatCircuit(circuit)
    init = circuit.init_index if init_index is None else init_index
    rho = np.zeros((1 << n) * (1 << n), np.complex128)
    st = lib().or_dm_run(n, ctypes.c_int64(flat.n_gates), _ptr(flat.kind), _ptr(flat.q0),
                         _ptr(flat.q1), _ptr(flat.noise), _ptr(flat.mats), _ptr(flat.theta),
                         _ptr(flat.mask), _ptr(flat.value), ctypes.c_double(e),
                         ctypes.c_uint64(init), _ptr(rho))
    if st != 0:
        raise ValueError("oracle dm_run rejected its arguments")
    return rho.reshape(1 << n, 1 << n)


def dm_apply_kraus(rho: np.ndarray, n: int, qubits, ops) -> np.ndarray:
    """sum_k E_k rho E_k^dagger for a Kraus set on one or two qubits (eq. 3)."""
    out = np.array(rho, np.complex128, copy=True).reshape(-1)
    qs = np.ascontiguousarray(qubits, np.int32)
    ops = np.ascontiguousarray(np.asarray(ops, np.complex128))
    st = lib().or_dm_apply_kraus(n, _ptr(out), qs.size, _ptr(qs), ops.shape[0], _ptr(ops))
    if st != 0:
        raise ValueError("oracle dm_apply_kraus rejected its arguments")
    return out.reshape(rho.shape)


def dm_expect(rho: np.ndarray, psi: np.ndarray):
    """(<psi|rho|psi>, Tr rho) as complex numbers."""
    n = int(np.log2(psi.size))
    r = np.ascontiguousarray(rho, np.complex128).reshape(-1)
    p = np.ascontiguousarray(psi, np.complex128)
    vals = [ctypes.c_double() for _ in range(4)]
    lib().or_dm_expect(n, _ptr(r), _ptr(p), *[ctypes.byref(v) for v in vals])
    return complex(vals[0].value, vals[1].value), complex(vals[2].value, vals[3].value)


def kraus_rot(u: np.ndarray, e: float) -> np.ndarray:
    """Kraus set of the eq. (1) noisy one-qubit gate u: {u E1, u E2} with E1, E2 of eq. (6)."""
    l1 = 0.5 * (1.0 + np.exp(-2.0 * e * e))
    l2 = 0.5 * (1.0 - np.exp(-2.0 * e * e))
    E1 = np.sqrt(l1) * np.eye(2)
    E2 = np.sqrt(l2) * np.array([[0.0, 1.0], [-1.0, 0.0]])
    return np.stack([u @ E1, u @ E2]).astype(np.complex128)


def kraus_phase(theta: float, e: float) -> np.ndarray:
    """Kraus set of the noisy controlled phase: {U_theta E1, U_theta E2} with eq. (9)."""
    P = np.exp(-e * e)
    ph = np.exp(-1j * theta)
    E1 = np.diag([1.0, 1.0, 1.0, ph * np.sqrt(P)])
    E2 = np.diag([0.0, 0.0, 0.0, ph * np.sqrt(1.0 - P)])
    return np.stack([E1, E2]).astype(np.complex128)


def cp_mixing_f(e: float) -> float:
    """The parameter f of eq. (13) for P = exp(-e^2): (sqrt(1 + 3P) - P - 1) / sqrt(P (1 - P)),
    0 in the limit P -> 1 (no noise)."""
    P = math.exp(-e * e)
    if P >= 1.0:
        return 0.0
    return (math.sqrt(1.0 + 3.0 * P) - P - 1.0) / math.sqrt(P * (1.0 - P))


def kraus_phase_improved(theta: float, e: float) -> np.ndarray:
    """The noisy controlled phase with the Kraus operators of eq. (14): the eq. (9) pair mixed by
    the unitary of eq. (13), {U_theta E~1, U_theta E~2}, with E~1 = diag(1, 1, 1, sqrt(P) +
    f sqrt(1-P)) / sqrt(1+f^2) and E~2 = diag(-f, -f, -f, -f sqrt(P) + sqrt(1-P)) / sqrt(1+f^2).
    A unitary mixture of Kraus operators describes the same channel."""
    P = math.exp(-e * e)
    f = cp_mixing_f(e)
    c = 1.0 / math.sqrt(1.0 + f * f)
    ph = np.exp(-1j * theta)
    E1 = c * np.diag([1.0, 1.0, 1.0, ph * (math.sqrt(P) + f * math.sqrt(1.0 - P))])
    E2 = c * np.diag([-f, -f, -f, ph * (-f * math.sqrt(P) + math.sqrt(1.0 - P))])
    return np.stack([E1, E2]).astype(np.complex128)


# ------------------------------------------------------------------------------------------
# Choi-Jamiolkowski relative states (Section 4, eq. 16-17)
# ------------------------------------------------------------------------------------------
def _gate_unitary(g):
    """(qubits, unitary) of a gate of the circuit description, for a one-operator Kraus step."""
    from workloads import CNOT, CP, SWAP, U1, U2
    if g.kind == U1:
        return [g.q0], np.asarray(g.m, np.complex128)
    if g.kind == U2:
        return [g.q0, g.q1], np.asarray(g.m, np.complex128)
    if g.kind == CNOT:   # control q0, target q1; local index bit(q0) + 2 bit(q1)
        return [g.q0, g.q1], np.array([[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0], [0, 1, 0, 0]], np.complex128)
    if g.kind == CP:
        return [g.q0, g.q1], np.diag([1, 1, 1, np.exp(-1j * g.theta)]).astype(np.complex128)
    if g.kind == SWAP:
        return [g.q0, g.q1], np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], np.complex128)
    raise ValueError("gate kind not supported in relative-state programs")


def choi_state(prog) -> np.ndarray:
    """rho_E of eq. (17) for the register and its references: |0><0|, the entangling gates of
    eq. (16), then the program's gates (U rho U^dagger) and channels (sum_k E_k rho E_k^dagger)."""
    from workloads import Channel, choi_preparation
    N = prog.total_qubits()
    rho = np.zeros((1 << N, 1 << N), np.complex128)
    rho[0, 0] = 1.0
    for st in choi_preparation(prog) + list(prog.steps):
        if isinstance(st, Channel):
            rho = dm_apply_kraus(rho, N, list(st.qubits), st.ops)
        else:
            qs, U = _gate_unitary(st)
            rho = dm_apply_kraus(rho, N, qs, U[None])
    return rho


def choi_target(prog, index: int) -> np.ndarray:
    """The ideal relative state with the ancillas in the basis values of `index`."""
    from workloads import Circuit, choi_preparation
    N = prog.total_qubits()
    c = Circuit(N, choi_preparation(prog) + list(prog.ideal), init_index=index)
    return sv_run(c, 0.0)


def choi_fidelity(prog):
    """Relative-state fidelity sum_a <target_a|rho_E|target_a> over the ancilla assignments a
    (the ancillas traced out), and Tr rho_E."""
    from workloads import ancilla_indices
    rho = choi_state(prog)
    F = 0.0
    for idx in ancilla_indices(prog):
        f, tr = dm_expect(rho, choi_target(prog, idx))
        F += f.real
    return F, dm_expect(rho, choi_target(prog, 0))[1].real
