"""GPU parity of the fixed-rank form's two-qubit Kraus steps (Section 3.2 with the noisy
controlled phase of eq. 9): the library through the C ABI against the numpy oracle
(oracle/fixed_rank.py), which is pinned on the CPU to the exact density matrix at full rank.

Tolerances: complex<double> columns 1e-11 on fidelities and log-traces and 1e-12 on the entries
of rho; complex<float> columns (FP64 Gram and eigen-decomposition) 1e-5 on fidelities.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import fixed_rank
from workloads import U1, Gate, qft

torch = pytest.importorskip("torch")
import paper_1412_2293_amd as q  # noqa: E402

pytestmark = pytest.mark.gpu


def _zero_tol(dtype):
    return 1e-13 if dtype == q.C128 else 1e-6


def _upload(psi: np.ndarray, dtype) -> "q.StateVector":
    n = int(np.log2(psi.size))
    sv = q.StateVector(n, dtype, 1)
    amps = sv.amplitudes()
    amps.copy_(torch.as_tensor(psi.astype(np.complex64 if dtype == q.C64 else np.complex128)).to(amps.device))
    torch.cuda.synchronize()
    return sv


def _rho(fr: "q.FixedRank") -> np.ndarray:
    rank, lt = fr.info()
    V = fr.columns()[:rank].cpu().numpy().astype(np.complex128).T
    return math.exp(lt) * (V @ V.conj().T)


def _check(fr, ref, ideal, dtype, ranks=None):
    sv = _upload(ideal, dtype)
    fu, fn, lt = fr.fidelity(sv)
    fu_ref, fn_ref, lt_ref = ref.fidelity(ideal)
    if dtype == q.C128:
        if ranks is not None:
            assert ranks[-1] == len(ref.V)
        assert abs(fu - fu_ref) <= 1e-11 and abs(fn - fn_ref) <= 1e-11 and abs(lt - lt_ref) <= 1e-11
        np.testing.assert_allclose(_rho(fr), ref.rho(), atol=1e-12)
    else:
        assert abs(fu - fu_ref) <= 1e-5 and abs(fn - fn_ref) <= 1e-5


@pytest.mark.parametrize("dtype", [q.C128, q.C64], ids=["c128", "c64"])
def test_fixed_rank_noisy_controlled_phases_against_oracle(dtype):
    """QFT n = 8 with noisy Hadamards (eq. 6) and noisy controlled phases (eq. 9): every CP is a
    two-qubit Kraus step with truncation back to r = 8."""
    n, e, r = 8, 0.08, 8
    c = qft(n, seed=4)
    fr = q.FixedRank(n, r, dtype)
    fr.init_basis(c.init_index)
    ranks = [fr.apply_noisy_gate(g, e, tau=1e-9, zero_tol=_zero_tol(dtype)) for g in c.gates]
    assert max(ranks) == r
    ref = fixed_rank.run_circuit(c, e, r, tau=1e-9, zero_tol=1e-13)
    _check(fr, ref, oracle.sv_run(c, 0.0), dtype, ranks)


def _random_kraus2(rng, n_ops):
    """A random complete two-qubit Kraus set: blocks of an isometry from QR."""
    z = rng.standard_normal((4 * n_ops, 4)) + 1j * rng.standard_normal((4 * n_ops, 4))
    Q, _ = np.linalg.qr(z)
    return Q.reshape(n_ops, 4, 4)


@pytest.mark.parametrize("n", [5, 8, 14])
@pytest.mark.parametrize("dtype", [q.C128, q.C64], ids=["c128", "c64"])
def test_fixed_rank_general_two_qubit_kraus_sets(n, dtype):
    """Dense (non-diagonal) Kraus sets of 2-4 operators on qubit pairs in both orders, low and
    high bits; n = 5 takes the one-block Gram kernel, 8 the matrix-core kernel with one block,
    14 with several blocks."""
    rng = np.random.default_rng(100 + n)
    r = 8
    fr = q.FixedRank(n, r, dtype)
    ref = fixed_rank.FixedRank(n, r, init_index=3, tau=1e-9, zero_tol=1e-13)
    fr.init_basis(3)
    pairs = [(0, 1), (n - 1, 0), (2, n - 2), (1, 3), (n - 2, n - 1)]
    ranks = []
    for k, (a, b) in enumerate(pairs):
        # a Haar layer first, so the columns are complex and spread
        for qb in range(n):
            U = np.linalg.qr(rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)))[0]
            fr.apply_gate(Gate(U1, q0=qb, m=U))
            ref.apply_unitary([qb], U)
        ops = _random_kraus2(rng, 2 + k % 3)
        ranks.append(fr.apply_kraus2(a, b, ops, tau=1e-9, zero_tol=_zero_tol(dtype)))
        ref.apply_kraus([a, b], ops)
        if dtype == q.C128:
            assert ranks[-1] == len(ref.V)
    psi = np.exp(1j * rng.uniform(0, 2 * np.pi, 1 << n)) / math.sqrt(1 << n)
    _check(fr, ref, psi, dtype)


def test_fixed_rank_kraus2_rejects_bad_arguments():
    fr = q.FixedRank(4, 2, q.C128)
    fr.init_basis(0)
    ops = np.stack([np.eye(4)]).astype(np.complex128)
    for args in [(1, 1), (0, 4), (-1, 2)]:
        with pytest.raises(q.QsimError):
            fr.apply_kraus2(args[0], args[1], ops)
    with pytest.raises(q.QsimError):
        fr.apply_kraus2(0, 1, np.zeros((5, 4, 4), np.complex128))
    bad = ops.copy()
    bad[0, 0, 0] = np.nan
    with pytest.raises(q.QsimError):
        fr.apply_kraus2(0, 1, bad)
    assert fr.info()[0] == 1


@pytest.mark.parametrize("dtype", [q.C128, q.C64], ids=["c128", "c64"])
def test_fixed_rank_mixed_circuit_with_diagonal_gates(dtype):
    """Every gate kind in the fixed-rank form (unitary steps on each column, Kraus steps with
    truncation for the noisy ones), including diagonal patterns with complex factors, against the
    numpy oracle."""
    from workloads import DIAG, Circuit, random_mixed_circuit
    n, e, r = 7, 0.1, 8
    c = random_mixed_circuit(n, 70, seed=21)
    rng = np.random.default_rng(21)
    gates = list(c.gates)
    for _ in range(6):
        mask = int(rng.integers(1, 1 << n))
        f = complex(np.exp(1j * rng.uniform(0, 2 * np.pi)))
        gates.insert(int(rng.integers(0, len(gates) + 1)),
                     Gate(DIAG, m=np.array([f]), mask=mask, value=int(rng.integers(0, 1 << n)) & mask))
    c = Circuit(n, gates, name="mixed7+diag", init_index=c.init_index)
    fr = q.FixedRank(n, r, dtype)
    fr.init_basis(c.init_index)
    ranks = [fr.apply_noisy_gate(g, e, tau=1e-9, zero_tol=_zero_tol(dtype)) for g in c.gates]
    ref = fixed_rank.run_circuit(c, e, r, tau=1e-9, zero_tol=1e-13)
    _check(fr, ref, oracle.sv_run(c, 0.0), dtype, ranks)
