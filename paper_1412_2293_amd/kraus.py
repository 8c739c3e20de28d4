"""Kraus operators that callers hand to `apply_kraus` or `FixedRank.apply_kraus2`.

`cp_kraus_improved` is the noisy controlled phase in the form of Section 3.3: the two operators
of eq. (9) mixed by the unitary of eq. (13), which gives the pair of eq. (14), orthogonal in the
Hilbert-Schmidt sense.  It describes the same channel as eq. (9) (`dm_apply_gate` applies that
one with diagonal sweeps), so either path gives the same density matrix.  The operators are
built by the library (qs_kraus_cp); this module only marshals.
"""
import numpy as np

from .qsim import kraus_cp

__all__ = ["cp_kraus", "cp_kraus_improved"]


def cp_kraus(theta: float, e: float) -> np.ndarray:
    """(2, 4, 4) complex128: the eq. (9) pair times the ideal phase exp(-i theta) on |11>."""
    return kraus_cp(theta, e, improved=False)


def cp_kraus_improved(theta: float, e: float) -> np.ndarray:
    """(2, 4, 4) complex128: the controlled phase exp(-i theta) on |11> times each operator of
    eq. (14), for `apply_kraus` on (control, target) (local index bit(q0) + 2 bit(q1); the
    operators are diagonal, so the order of the two qubits does not matter)."""
    return kraus_cp(theta, e, improved=True)
