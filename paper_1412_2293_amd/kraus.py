"""Kraus operators that callers hand to `apply_kraus` (host-side parameters; the sweeps run in
libqsim's kernels).

`cp_kraus_improved` is the noisy controlled phase in the form of Section 3.3: the two operators
of eq. (9) mixed by the unitary of eq. (13), which gives the pair of eq. (14), orthogonal in the
Hilbert-Schmidt sense.  It describes the same channel as eq. (9) (`dm_apply_gate` applies that
one with diagonal sweeps), so either path gives the same density matrix.
"""
import math

import numpy as np

__all__ = ["cp_mixing", "cp_kraus_improved"]


def cp_mixing(e: float) -> float:
    """f of eq. (13) for the phase-noise strength e (P = exp(-e^2)); its limit 0 at e = 0."""
    p = math.exp(-e * e)
    if p >= 1.0:
        return 0.0
    return (math.sqrt(1.0 + 3.0 * p) - 1.0 - p) / math.sqrt(p * (1.0 - p))


def cp_kraus_improved(theta: float, e: float) -> np.ndarray:
    """(2, 4, 4) complex128: the controlled phase exp(-i theta) on |11> times each operator of
    eq. (14), for `apply_kraus` on (control, target) (local index bit(q0) + 2 bit(q1); the
    operators are diagonal, so the order of the two qubits does not matter)."""
    p = math.exp(-e * e)
    f = cp_mixing(e)
    norm = 1.0 / math.sqrt(1.0 + f * f)
    u11 = complex(math.cos(theta), -math.sin(theta))
    ops = np.zeros((2, 4, 4), np.complex128)
    for k in range(3):
        ops[0, k, k] = norm
        ops[1, k, k] = -f * norm
    ops[0, 3, 3] = u11 * (math.sqrt(p) + f * math.sqrt(1.0 - p)) * norm
    ops[1, 3, 3] = u11 * (math.sqrt(1.0 - p) - f * math.sqrt(p)) * norm
    return ops
