"""GPU relative states (Section 4) against closed forms and the oracle."""
import math

import numpy as np
import pytest

import oracle
import workloads as w

torch = pytest.importorskip("torch")
import paper_1412_2293_amd as q  # noqa: E402
from paper_1412_2293_amd import choi  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
def test_phase_code_against_closed_form(dtype):
    for p in (0.0, 0.05, 0.2, 0.5):
        F, tr = choi.relative_state_fidelity(w.phase_code(p), dtype)
        tol = 1e-12 if dtype == q.C128 else 2e-6
        assert abs(F - (1 - 3 * p * p + 2 * p ** 3)) <= tol, (p, F)
        assert abs(tr - 1.0) <= tol


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
@pytest.mark.parametrize("n,T1,T2", [(3, 30.0, 20.0), (5, 10.0, 5.0), (5, 100.0, 70.0)])
def test_qft_relaxation_against_oracle(dtype, n, T1, T2):
    prog = w.qft_relaxation(n, T1, T2)
    rho = choi.relative_state(prog, dtype)
    torch.cuda.synchronize()
    got = rho.amplitudes()[0].cpu().numpy().astype(np.complex128)
    rho.close()
    ref = oracle.choi_state(prog).reshape(-1)
    tol = 1e-12 if dtype == q.C128 else 3e-6
    assert np.linalg.norm(got - ref) <= tol * np.linalg.norm(ref)
    F, tr = choi.relative_state_fidelity(prog, dtype)
    F_ref, _ = oracle.choi_fidelity(prog)
    assert abs(F - F_ref) <= (1e-12 if dtype == q.C128 else 2e-6)
    assert abs(tr - 1.0) <= (1e-12 if dtype == q.C128 else 2e-6)


def test_one_qubit_channel_closed_form():
    p, g = 0.1, 0.25
    steps = [w.Channel((0,), w.amplitude_damping(1.0, -1.0 / math.log(1.0 - g))), w.Channel((0,), w.dephasing(p))]
    F, tr = choi.relative_state_fidelity(w.ChoiProgram(1, [0], steps, []), q.C128)
    s = math.sqrt(1.0 - g)
    assert abs(F - ((1 - p) * ((1 + s) / 2) ** 2 + p * ((1 - s) / 2) ** 2)) <= 1e-12


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
def test_shor_code_against_closed_form(dtype):
    """Shor's code under phase errors: F = 1 - 3q^2 + 2q^3, q = 3p(1-p)^2 + p^3 (eight traced-out
    qubits, 2^20-entry vec(rho))."""
    for p in (0.0, 0.02, 0.1):
        F, tr = choi.relative_state_fidelity(w.shor_code(p), dtype)
        qb = 3 * p * (1 - p) ** 2 + p ** 3
        tol = 1e-12 if dtype == q.C128 else 5e-6
        assert abs(F - (1 - 3 * qb * qb + 2 * qb ** 3)) <= tol, (p, F)
        assert abs(tr - 1.0) <= tol


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
def test_codes_under_relaxation_against_oracle(dtype):
    """The three-qubit and Shor codes with amplitude and phase relaxation on every code qubit:
    relative-state overlaps against the oracle's, and with T1 = inf the closed forms of the
    phase-error codes (p from eq. 19)."""
    tol = 1e-12 if dtype == q.C128 else 5e-6
    for T1, T2 in ((30.0, 20.0), (10.0, 5.0)):
        for build in (w.phase_code_relaxation, w.shor_code_relaxation):
            prog = build(T1, T2)
            F, tr = choi.relative_state_fidelity(prog, dtype)
            F_ref, _ = oracle.choi_fidelity(prog)
            assert abs(F - F_ref) <= tol, (prog.name, F, F_ref)
            assert abs(tr - 1.0) <= tol
    T2 = 12.0
    p = 0.5 * (1.0 - math.exp(-1.0 / T2))
    F, _ = choi.relative_state_fidelity(w.phase_code_relaxation(math.inf, T2), dtype)
    assert abs(F - (1 - 3 * p * p + 2 * p ** 3)) <= tol
