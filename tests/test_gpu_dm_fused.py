"""GPU parity of the density-matrix runs through the fused passes (qs_dm_run): the noisy circuit
becomes a noiseless circuit on vec(rho) (eq. 6 Kraus pairs as dense two-qubit gates on a row
and a column bit, the eq. 9 average as diagonal patterns) that the trajectory machinery runs as
one slot.  Small sizes: every entry of rho against the oracle's Kraus-channel run; full size
(n = 13, 2^26 entries): the closed forms and invariants the oracle is pinned to.

Tolerances: complex<double> 1e-12 relative (2-norm over the norm, and on F); complex<float>
2e-5 relative on rho and |dF| <= 1e-5.
"""
import math

import numpy as np
import pytest

import oracle
from workloads import DIAG, FLIP, Circuit, Gate, grover, qft, random_mixed_circuit

torch = pytest.importorskip("torch")
import paper_1412_2293_amd as q  # noqa: E402

pytestmark = pytest.mark.gpu


def rel_err(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def ideal_state(n, dtype, psi):
    sv = q.StateVector(n, dtype, 1)
    amps = sv.amplitudes()
    amps.copy_(torch.as_tensor(psi[None, :].astype(np.complex64 if dtype == q.C64 else np.complex128)).to(amps.device))
    torch.cuda.synchronize()
    return sv


def rho_logical(res, n, dtype):
    """rho[i, j] from vec(rho) stored with row bit q at layout[q] + n, column bit q at layout[q]."""
    v = q.dm_state(res, n, dtype).cpu().numpy().astype(np.complex128)
    idx = np.arange(1 << n, dtype=np.int64)
    phys = np.zeros_like(idx)
    for b in range(n):
        phys |= ((idx >> b) & 1) << int(res["layout"][b])
    return v[(phys[:, None] << n) | phys[None, :]]


def with_diag_gates(c: Circuit, seed: int) -> Circuit:
    rng = np.random.default_rng(seed)
    N = 1 << c.n
    gates = list(c.gates)
    for _ in range(5):
        mask = int(rng.integers(1, N))
        value = int(rng.integers(0, N)) & mask
        f = complex(np.exp(1j * rng.uniform(0, 2 * math.pi)))
        gates.insert(int(rng.integers(0, len(gates) + 1)), Gate(DIAG, m=np.array([f]), mask=mask, value=value))
    return Circuit(c.n, gates, name=c.name + "+diag", init_index=c.init_index)


CIRCUITS = {
    "grover6": (lambda: grover(6, seed=4), 0.08),
    "qft6_noisy_cp": (lambda: qft(6, seed=3, x=37), 0.15),
    "qft7_noisy_cp": (lambda: qft(7, seed=5, x=77), 0.05),
    "mixed6_diag": (lambda: with_diag_gates(random_mixed_circuit(6, 60, seed=9), 9), 0.1),
}
PLANS = {
    "fused": {"fuse": 1},
    "t8": {"fuse": 1, "tile_bits": 8, "reg_bits": 3, "run_bits": 2},
    "t9r2": {"fuse": 1, "tile_bits": 9, "reg_bits": 2, "run_bits": 3},
    "t11r3": {"fuse": 1, "tile_bits": 11, "reg_bits": 3, "run_bits": 3},
    "unfused": {"fuse": 0},
    "auto": None,
}


@pytest.mark.parametrize("dtype", [q.C128, q.C64], ids=["c128", "c64"])
@pytest.mark.parametrize("plan", list(PLANS), ids=list(PLANS))
@pytest.mark.parametrize("name", list(CIRCUITS), ids=list(CIRCUITS))
def test_fused_dm_against_oracle(name, plan, dtype):
    make, e = CIRCUITS[name]
    c = make()
    n = c.n
    print(f"[dm_run] {name} plan={plan} dtype={dtype}", flush=True)
    psi = oracle.sv_run(c, 0.0)
    ideal = ideal_state(n, dtype, psi)
    res = q.dm_run(c.gates, n, c.init_index, dtype, ideal, e=e, plan=PLANS[plan])
    ref = oracle.dm_run(c, e)
    got = rho_logical(res, n, dtype)
    f_ref, tr_ref = oracle.dm_expect(ref, psi)
    tol = 1e-12 if dtype == q.C128 else 2e-5
    assert rel_err(got, ref) <= tol, (name, plan)
    if dtype == q.C128:
        assert abs(res["F"] - f_ref.real) <= tol * abs(f_ref.real)
    else:
        assert abs(res["F"] - f_ref.real) <= 1e-5
    assert abs(res["trace"] - tr_ref.real) <= (tol if dtype == q.C128 else 1e-5)
    ideal.close()


def test_swaps_relabel_both_halves_alike():
    """A fused QFT turns its final SWAPs into a relabelling: the run reports it, and rho read
    through it is the oracle's."""
    c = qft(6, seed=3, x=21)
    psi = oracle.sv_run(c, 0.0)
    ideal = ideal_state(6, q.C128, psi)
    res = q.dm_run(c.gates, 6, c.init_index, q.C128, ideal, e=0.1, plan={"fuse": 1, "tile_bits": 8,
                                                                          "reg_bits": 3, "run_bits": 2})
    assert sorted(res["layout"]) == list(range(6))
    assert list(res["layout"]) != list(range(6))
    assert rel_err(rho_logical(res, 6, q.C128), oracle.dm_run(c, 0.1)) <= 1e-12


@pytest.mark.parametrize("dtype", [q.C128, q.C64], ids=["c128", "c64"])
def test_degenerate_circuits(dtype):
    """No gates: rho = |init><init| and F = |psi_init|^2; one qubit; noise off (e = 0) equals the
    pure state's projector."""
    n = 4
    rng = np.random.default_rng(3)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi /= np.linalg.norm(psi)
    ideal = ideal_state(n, dtype, psi)
    res = q.dm_run([], n, 5, dtype, ideal, e=0.3, plan={"fuse": 1})
    got = rho_logical(res, n, dtype)
    ref = np.zeros((1 << n, 1 << n), np.complex128)
    ref[5, 5] = 1.0
    assert np.max(np.abs(got - ref)) <= 1e-6
    assert abs(res["F"] - abs(psi[5]) ** 2) <= 1e-6 and abs(res["trace"] - 1.0) <= 1e-6
    ideal.close()
    c1 = Circuit(1, [Gate(0, q0=0, m=np.array([[1, 1], [1, -1]]) / math.sqrt(2), noise=1)], name="h1")
    p1 = oracle.sv_run(c1, 0.0)
    i1 = ideal_state(1, dtype, p1)
    for plan in ({"fuse": 1}, {"fuse": 0}):
        r1 = q.dm_run(c1.gates, 1, 0, dtype, i1, e=0.4, plan=plan)
        ref1 = oracle.dm_run(c1, 0.4)
        assert np.max(np.abs(rho_logical(r1, 1, dtype) - ref1)) <= 1e-6
    i1.close()
    c = grover(5, seed=1)
    p = oracle.sv_run(c, 0.0)
    i5 = ideal_state(5, dtype, p)
    r = q.dm_run(c.gates, 5, 0, dtype, i5, e=0.0, plan={"fuse": 1})
    tol = 1e-12 if dtype == q.C128 else 2e-5
    assert rel_err(rho_logical(r, 5, dtype), np.outer(p, p.conj())) <= tol
    assert abs(r["F"] - 1.0) <= (1e-12 if dtype == q.C128 else 1e-5)
    i5.close()


def test_dm_run_rejects_bad_arguments():
    c = grover(4, seed=1)
    ideal = ideal_state(4, q.C128, oracle.sv_run(c, 0.0))
    with pytest.raises(q.QsimError):
        q.dm_run(c.gates, 4, 16, q.C128, ideal, e=0.1)            # init_index out of range
    with pytest.raises(q.QsimError):
        q.dm_run(c.gates, 4, 0, q.C128, ideal, e=-1.0)
    with pytest.raises(q.QsimError):
        q.dm_run(c.gates, 18, 0, q.C128, ideal, e=0.1)
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(q.QsimError):
        q.dm_run(c.gates, 4, 0, q.C128, ideal, e=0.1, buf=small)
    ideal.close()


# ----------------------------------------------------------------------------------------
# Full size: n = 13, vec(rho) of 2^26 entries.
def qft_ideal_state(n, x):
    N = 1 << n
    ex = np.zeros(N, np.complex128)
    ex[x] = 1.0
    return np.fft.fft(ex) / math.sqrt(N)


@pytest.mark.parametrize("dtype", [q.C128, q.C64], ids=["c128", "c64"])
def test_fused_dm_qft13_full_size_against_closed_form(dtype):
    """QFT at n = 13 with noisy Hadamards (eq. 6) and noisy controlled phases (eq. 9): the exact
    fidelity to the ideal output equals prod_t (1 + exp(-2e^2) exp(-e^2 m_t / 2)) / 2
    (m_t = ones of x below t), for inputs with few and many ones; Tr rho = 1."""
    import sys
    import os
    sys.path.insert(0, os.path.dirname(__file__))
    from paper_forms import qft_expected_fidelity
    n, e = 13, 0.05
    for x in (1, (1 << n) - 2, 0x0A5B):
        print(f"[dm_run] qft13 x={x} dtype={dtype}", flush=True)
        c = qft(n, seed=1, x=x)
        ideal = ideal_state(n, dtype, qft_ideal_state(n, x))
        res = q.dm_run(c.gates, n, x, dtype, ideal, e=e)
        F = qft_expected_fidelity(n, x, e)
        if dtype == q.C128:
            assert abs(res["F"] - F) <= 1e-12 * F, (x, res["F"], F)
            assert abs(res["trace"] - 1.0) <= 1e-12
        else:
            assert abs(res["F"] - F) <= 1e-5, (x, res["F"], F)
            assert abs(res["trace"] - 1.0) <= 1e-5
        ideal.close()
        del res
        torch.cuda.empty_cache()


def test_fused_dm_grover13_full_size():
    """Grover at n = 13 (every Hadamard noisy, eq. 6): a prefix on the lowest, a middle and the
    highest qubit plus the oracle flip against the oracle entry by entry; the whole circuit
    through its invariants: Tr rho = 1, and <psi|rho|psi> equals the mean fidelity of Monte Carlo
    trajectories of the same circuit within 5 standard errors (the channel is the exact average
    over xi of eq. 1)."""
    n, e = 13, 0.02
    c = grover(n, seed=5)
    hs = {g.q0: g for g in c.gates[:n]}
    flip = next(g for g in c.gates if g.kind == FLIP)
    prefix = Circuit(n, [hs[0], hs[n - 1], hs[6], flip], name="g13prefix", init_index=0, marked=c.marked)
    psi_p = oracle.sv_run(prefix, 0.0)
    ideal = ideal_state(n, q.C128, psi_p)
    print("[dm_run] grover13 prefix", flush=True)
    res = q.dm_run(prefix.gates, n, 0, q.C128, ideal, e=e)
    ref = oracle.dm_run(prefix, e)
    assert rel_err(rho_logical(res, n, q.C128), ref) <= 1e-12
    del ref, res
    ideal.close()
    torch.cuda.empty_cache()
    print("[dm_run] grover13 full", flush=True)
    ideal = ideal_state(n, q.C128, oracle.sv_run(c, 0.0))
    res = q.dm_run(c.gates, n, 0, q.C128, ideal, e=e)
    assert abs(res["trace"] - 1.0) <= 1e-11
    T = 2048
    mc = q.run_trajectories(c.gates, n, 0, q.C128, T, e=e, seed=21)
    m, se = float(np.mean(mc["F"])), float(np.std(mc["F"]) / math.sqrt(T))
    assert abs(res["F"] - m) <= 5 * se, (res["F"], m, se)
    ideal.close()
