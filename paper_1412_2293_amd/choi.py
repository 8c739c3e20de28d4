"""Choi-Jamiolkowski relative states (Section 4, eq. 16-17) on the density-matrix path.

A program's register and its reference qubits start in |0...0><0...0|; the gates of eq. (16)
entangle each logical qubit with its reference, then the program's gates and Kraus channels act
on the register (eq. 17).  Every step is a call into the library (``dm_apply_gate`` for gates,
``apply_kraus`` for channels, ``dm_fidelity`` for the overlaps); this module only sequences them.
"""
from __future__ import annotations

from . import qsim as q


def relative_state(prog, dtype: int = q.C128, stream=None) -> "q.StateVector":
    """vec(rho_E) of the program (a 2N-qubit state vector, N = register + references)."""
    from workloads import Channel, choi_preparation
    N = prog.total_qubits()
    rho = q.StateVector(2 * N, dtype, 1, stream=stream)
    rho.init_basis(0)
    for st in choi_preparation(prog) + list(prog.steps):
        if isinstance(st, Channel):
            q.apply_kraus(rho, list(st.qubits), st.ops)
        else:
            q.dm_apply_gate(rho, st, 0.0)
    return rho


def relative_state_fidelity(prog, dtype: int = q.C128, stream=None):
    """(F, Tr rho_E): F = sum over the ancilla assignments a of <target_a|rho_E|target_a>, the
    target being the entangled input mapped by the program's ideal gates."""
    from workloads import ancilla_indices, choi_preparation
    N = prog.total_qubits()
    rho = relative_state(prog, dtype, stream)
    target = q.StateVector(N, dtype, 1, stream=stream)
    F, tr = 0.0, 0.0
    try:
        for idx in ancilla_indices(prog):
            target.init_basis(idx)
            for g in choi_preparation(prog) + list(prog.ideal):
                q.apply_gate(target, g)
            f, tr = q.dm_fidelity(rho, target, 0)
            F += f
    finally:
        target.close()
        rho.close()
    return F, tr
