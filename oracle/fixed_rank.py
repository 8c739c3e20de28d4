"""Fixed-rank density-matrix approximation (Section 3.2), numpy FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

rho is kept as rho = exp(log_trace) * sum_j |v_j><v_j| with at most r orthogonal columns
v_j and sum_j <v_j|v_j> = 1.  The paper's steps, in its order:
  * the run starts from the pure state |psi0> (rank 1);
  * a unitary gate acts on every v_j and cannot raise the rank;
  * a noisy gate with Kraus set {K_m} (eq. 3) maps rho to sum_m K_m rho K_m^dagger, whose
    factor is W = [K_m v_j]_{m,j}: the rank grows at most by the number of Kraus operators;
  * after that step rho is approximated by a matrix of the fixed rank r through its spectral
    decomposition: the eigen-decomposition of the Gram matrix G = W^dagger W gives the
    non-zero spectrum of W W^dagger, and W q_k are its eigenvectors;
  * the kept part is renormalised to unit trace; the removed weight is booked in log_trace,
    so exp(log_trace) * <psi|rho|psi> is the paper's unnormalised fidelity and
    <psi|rho|psi> the normalised one.

Readings where the paper is silent (listed with the other readings of the paper):
  * truncation happens only when a Kraus step leaves more than r non-zero eigenvalues;
  * eigenvalues at most ``zero_tol * mu_max`` are numerically zero and dropped;
  * ties at the cut: if mu_r - mu_{r+1} <= tau * mu_max the whole cluster of tied
    eigenvalues straddling the cut is dropped (rank <= r, result unique).
The eigen-decomposition is numpy.linalg.eigh (a library primitive).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _ptr, lib


def _apply_op(v: np.ndarray, n: int, qubits, K: np.ndarray) -> np.ndarray:
    """K (2x2 or 4x4, any matrix) applied to qubits of the vector v via the oracle's loops."""
    out = np.array(v, np.complex128, copy=True)
    k = len(qubits)
    kind = np.array([0 if k == 1 else 4], np.int32)
    q0 = np.array([qubits[0]], np.int32)
    q1 = np.array([qubits[1] if k == 2 else 0], np.int32)
    zi = np.zeros(1, np.int32)
    site = np.zeros(1, np.uint32)
    mats = np.zeros(32, np.float64)
    flatK = np.asarray(K, np.complex128).reshape(-1)
    mats[0:2 * flatK.size:2] = flatK.real
    mats[1:2 * flatK.size:2] = flatK.imag
    th = np.zeros(1, np.float64)
    mk = np.zeros(1, np.uint64)
    st = lib().or_sv_apply_circuit(n, ctypes.c_int64(1), _ptr(kind), _ptr(q0), _ptr(q1), _ptr(zi),
                                   _ptr(site), _ptr(mats), _ptr(th), _ptr(mk), _ptr(mk),
                                   ctypes.c_double(0.0), ctypes.c_uint64(0), 0, 0, _ptr(out))
    assert st == 0
    return out


def select(mu: np.ndarray, r: int, tau: float, zero_tol: float):
    """Indices (into mu sorted descending) that the truncation keeps."""
    mu_max = float(mu[0]) if mu.size else 0.0
    if mu_max <= 0.0:
        return 0
    nz = int(np.count_nonzero(mu > zero_tol * mu_max))
    keep = min(nz, r)
    if nz > r:
        while keep > 0 and mu[keep - 1] - mu[keep] <= tau * mu_max:
            keep -= 1
    return keep


class FixedRank:
    def __init__(self, n: int, r: int, init_index: int = 0, tau: float = 1e-9,
                 zero_tol: float = 1e-13):
        self.n, self.r, self.tau, self.zero_tol = n, r, tau, zero_tol
        v = np.zeros(1 << n, np.complex128)
        v[init_index] = 1.0
        self.V = [v]
        self.log_trace = 0.0
        self.ranks = []

    def apply_unitary(self, qubits, U):
        self.V = [_apply_op(v, self.n, qubits, U) for v in self.V]

    def apply_flip(self, mask: int, value: int):
        idx = np.arange(1 << self.n, dtype=np.uint64)
        sel = (idx & np.uint64(mask)) == np.uint64(value)
        for v in self.V:
            v[sel] = -v[sel]

    def apply_diag(self, mask: int, value: int, f: complex):
        idx = np.arange(1 << self.n, dtype=np.uint64)
        sel = (idx & np.uint64(mask)) == np.uint64(value)
        for v in self.V:
            v[sel] = v[sel] * f

    def apply_kraus(self, qubits, ops):
        W = [_apply_op(v, self.n, qubits, K) for K in ops for v in self.V]
        Wm = np.stack(W, axis=1)                      # N x (m * rank)
        G = Wm.conj().T @ Wm                          # Gram matrix W^dagger W
        mu, Q = np.linalg.eigh(G)
        order = np.argsort(mu)[::-1]
        mu, Q = mu[order], Q[:, order]
        keep = select(mu, self.r, self.tau, self.zero_tol)
        Vn = Wm @ Q[:, :keep]                         # eigenvectors of W W^dagger, norms^2 = mu
        kept = float(np.sum(mu[:keep]))
        Vn = Vn / np.sqrt(kept)
        self.log_trace += float(np.log(kept))
        self.V = [Vn[:, k].copy() for k in range(keep)]
        self.ranks.append(keep)
        return keep

    def fidelity(self, psi: np.ndarray):
        """(unnormalised F, normalised F, log_trace) against the pure state psi."""
        fn = float(sum(abs(np.vdot(psi, v)) ** 2 for v in self.V))
        return fn * float(np.exp(self.log_trace)), fn, self.log_trace

    def rho(self) -> np.ndarray:
        Vm = np.stack(self.V, axis=1)
        return np.exp(self.log_trace) * (Vm @ Vm.conj().T)


def run_circuit(circuit, e: float, r: int, tau: float = 1e-9, zero_tol: float = 1e-13,
                init_index=None, max_gates=None) -> FixedRank:
    """Run a workloads.Circuit in the fixed-rank form: ROT-tagged one-qubit gates and
    PHASE-tagged controlled phases become their Kraus channels (eq. 6, eq. 9)."""
    from . import kraus_phase, kraus_rot
    init = circuit.init_index if init_index is None else init_index
    fr = FixedRank(circuit.n, r, init, tau, zero_tol)
    gates = circuit.gates if max_gates is None else circuit.gates[:max_gates]
    for g in gates:
        noisy = e != 0.0
        if g.kind == 0:
            if noisy and g.noise == 1:
                fr.apply_kraus([g.q0], kraus_rot(np.asarray(g.m), e))
            else:
                fr.apply_unitary([g.q0], np.asarray(g.m))
        elif g.kind == 1:
            if noisy and g.noise == 2:
                fr.apply_kraus([g.q0, g.q1], kraus_phase(g.theta, e))
            else:
                fr.apply_unitary([g.q0, g.q1], np.diag([1, 1, 1, np.exp(-1j * g.theta)]))
        elif g.kind == 2:
            fr.apply_unitary([g.q0, g.q1], np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0],
                                                     [0, 0, 0, 1]], np.complex128))
        elif g.kind == 3:
            fr.apply_unitary([g.q0, g.q1], np.array([[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0],
                                                     [0, 1, 0, 0]], np.complex128))
        elif g.kind == 4:
            fr.apply_unitary([g.q0, g.q1], np.asarray(g.m))
        elif g.kind == 5:
            fr.apply_flip(g.mask, g.value)
        elif g.kind == 6:
            fr.apply_diag(g.mask, g.value, complex(np.asarray(g.m).reshape(-1)[0]))
    return fr
