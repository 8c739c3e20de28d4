"""The oracle's relative states (Section 4, eq. 16-17) against closed forms."""
import math

import numpy as np
import pytest

import oracle
import workloads as w


def test_toffoli_decomposition_is_exact():
    for idx in range(8):
        c = w.Circuit(3, w._renumber_sites(w.toffoli_gates(1, 2, 0)), init_index=idx)
        psi = oracle.sv_run(c, 0.0)
        want = idx ^ 1 if ((idx >> 1) & 1 and (idx >> 2) & 1) else idx
        ref = np.zeros(8, np.complex128)
        ref[want] = 1.0
        assert np.linalg.norm(psi - ref) < 1e-12, idx


@pytest.mark.parametrize("p", [0.0, 0.01, 0.1, 0.3, 0.5])
def test_phase_code_fidelity_is_one_minus_two_or_more_errors(p):
    """Independent phase errors of probability p on the three code qubits: the majority
    correction fails exactly when two or more occur, and a logical Z has zero overlap with the
    entangled input, so F = 1 - 3p^2 + 2p^3 (the paper's eq. (18) is its square root)."""
    F, tr = oracle.choi_fidelity(w.phase_code(p))
    assert abs(F - (1 - 3 * p * p + 2 * p ** 3)) < 1e-13
    assert abs(tr - 1.0) < 1e-13
    assert abs(math.sqrt(F) - math.sqrt(1 - 3 * p ** 2 + 2 * p ** 3)) < 1e-12


@pytest.mark.parametrize("p,g", [(0.2, 0.0), (0.0, 0.3), (0.1, 0.25)])
def test_one_qubit_channels(p, g):
    """Entanglement fidelity of a one-qubit channel: sum_k |Tr E_k / 2|^2."""
    T1 = -1.0 / math.log(1.0 - g) if g > 0 else 1e300
    steps = [w.Channel((0,), w.amplitude_damping(1.0, T1)), w.Channel((0,), w.dephasing(p))]
    F, tr = oracle.choi_fidelity(w.ChoiProgram(1, [0], steps, []))
    s = math.sqrt(1.0 - g)
    want = (1 - p) * ((1 + s) / 2) ** 2 + p * ((1 - s) / 2) ** 2
    assert abs(F - want) < 1e-13 and abs(tr - 1.0) < 1e-13


def test_eq19_probability():
    """T2 = -t / ln(1 - 2p) (eq. 19): the dephasing built from (t, T2) has that p."""
    p = 0.07
    T2 = -1.0 / math.log(1 - 2 * p)
    np.testing.assert_allclose(w.dephasing_from_T2(1.0, T2), w.dephasing(p), atol=1e-15)


def test_noiseless_program_has_unit_fidelity():
    prog = w.qft_relaxation(3, 1e300, 1e300)
    prog = w.ChoiProgram(prog.n, prog.logical, list(prog.ideal), list(prog.ideal))
    F, tr = oracle.choi_fidelity(prog)
    assert abs(F - 1.0) < 1e-13 and abs(tr - 1.0) < 1e-13


def test_relaxation_lowers_qft_fidelity_monotonically():
    Fs = [oracle.choi_fidelity(w.qft_relaxation(3, T, T))[0] for T in (5.0, 20.0, 100.0, 1e6)]
    assert Fs[0] < Fs[1] < Fs[2] < Fs[3] and abs(Fs[3] - 1.0) < 1e-4


def test_shor_code_phase_errors():
    """Under phase errors alone each block of Shor's code carries a phase flip when an odd number
    of its qubits is hit, q = 3p(1-p)^2 + p^3, and the outer code corrects one flipped block:
    F = 1 - 3q^2 + 2q^3."""
    p = 0.07
    F, tr = oracle.choi_fidelity(w.shor_code(p))
    qb = 3 * p * (1 - p) ** 2 + p ** 3
    assert abs(F - (1 - 3 * qb * qb + 2 * qb ** 3)) < 1e-12 and abs(tr - 1.0) < 1e-12


def test_codes_under_relaxation_reduce_to_the_phase_error_forms():
    """With no amplitude relaxation (T1 = inf) the relaxation builders give the phase-error codes
    with p from eq. (19), whose overlaps are 1 - 3p^2 + 2p^3 (three-qubit code) and
    1 - 3q^2 + 2q^3, q = 3p(1-p)^2 + p^3 (Shor's code)."""
    T2 = 12.0
    p = 0.5 * (1.0 - math.exp(-1.0 / T2))
    F, tr = oracle.choi_fidelity(w.phase_code_relaxation(math.inf, T2))
    assert abs(F - (1 - 3 * p * p + 2 * p ** 3)) < 1e-13 and abs(tr - 1.0) < 1e-13
    F, tr = oracle.choi_fidelity(w.shor_code_relaxation(math.inf, T2))
    qb = 3 * p * (1 - p) ** 2 + p ** 3
    assert abs(F - (1 - 3 * qb * qb + 2 * qb ** 3)) < 1e-12 and abs(tr - 1.0) < 1e-12


def test_phase_code_under_relaxation_is_trace_preserving_and_monotone():
    """Amplitude relaxation (which the phase code does not correct) only lowers the overlap, the
    more the shorter T1; the trace stays 1."""
    Fs = []
    for T1 in (5.0, 20.0, 100.0, math.inf):
        F, tr = oracle.choi_fidelity(w.phase_code_relaxation(T1, 50.0))
        assert abs(tr - 1.0) < 1e-13
        Fs.append(F)
    assert Fs[0] < Fs[1] < Fs[2] < Fs[3] < 1.0
