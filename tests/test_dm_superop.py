"""The density-matrix circuit the library builds for vec(rho) (qs_dm_superop, host only: no GPU
needed) against the oracle's density-matrix run, and the diagonal gate kind in the oracle.

The library's superoperator gates are applied to |init, init> with the oracle's state-vector
runner on 2n qubits; the result must equal the oracle's Kraus-channel run of the noisy circuit
(Section 3: eq. 6 for the rotation noise, eq. 9 for the controlled-phase noise) entry by entry.
"""
import ctypes
import math

import numpy as np
import pytest

import oracle
import paper_1412_2293_amd as q
from workloads import (CP, DIAG, FLIP, NOISE_PHASE, NOISE_ROT, U1, Circuit, Gate, grover, qft,
                       random_mixed_circuit)


def to_workload_gate(g) -> Gate:
    """A library Gate struct as a workloads.Gate (for the oracle)."""
    m = np.array([complex(g.m[2 * k], g.m[2 * k + 1]) for k in range(16)])
    kind = int(g.kind)
    if kind == U1:
        mat = m[:4].reshape(2, 2)
    elif kind == 4:
        mat = m.reshape(4, 4)
    elif kind == DIAG:
        mat = m[:1]
    else:
        mat = None
    return Gate(kind, q0=int(g.q0), q1=int(g.q1), m=mat, theta=float(g.theta), noise=int(g.noise),
                site=int(g.site), mask=int(g.mask), value=int(g.value))


def superop_rho(c: Circuit, e: float) -> np.ndarray:
    n = c.n
    sg = q.dm_superop(c.gates, n, e)
    assert all(int(g.noise) == 0 for g in sg)
    big = Circuit(2 * n, [to_workload_gate(g) for g in sg], name="superop",
                  init_index=c.init_index * ((1 << n) + 1))
    return oracle.sv_run(big, 0.0).reshape(1 << n, 1 << n)


def with_diag_gates(c: Circuit, seed: int) -> Circuit:
    """c with a few DIAG gates (random patterns and unit or non-unit factors) spliced in."""
    rng = np.random.default_rng(seed)
    N = 1 << c.n
    gates = list(c.gates)
    for k in range(4):
        mask = int(rng.integers(1, N))
        value = int(rng.integers(0, N)) & mask
        f = complex(np.exp(1j * rng.uniform(0, 2 * math.pi)) * (1.0 if k % 2 == 0 else 0.7))
        gates.insert(int(rng.integers(0, len(gates) + 1)), Gate(DIAG, m=np.array([f]), mask=mask, value=value))
    return Circuit(c.n, gates, name=c.name + "+diag", init_index=c.init_index)


CASES = [
    ("grover3", lambda: grover(3, seed=2), 0.1),
    ("qft3_noisy_cp", lambda: qft(3, seed=1, x=5), 0.2),
    ("qft4_noisy_cp", lambda: qft(4, seed=2, x=9), 0.07),
    ("mixed4", lambda: random_mixed_circuit(4, 40, seed=3), 0.15),
    ("mixed4_diag", lambda: with_diag_gates(random_mixed_circuit(4, 30, seed=6), 6), 0.1),
]


@pytest.mark.parametrize("name,make,e", CASES, ids=[x[0] for x in CASES])
@pytest.mark.parametrize("noisy", [False, True])
def test_superop_circuit_equals_the_oracle_density_matrix(name, make, e, noisy):
    c = make()
    e = e if noisy else 0.0
    got = superop_rho(c, e)
    ref = oracle.dm_run(c, e)
    assert np.max(np.abs(got - ref)) <= 1e-13, name
    if name != "mixed4_diag":       # the non-unit diagonal factors there change the trace
        assert abs(np.trace(got) - 1.0) <= 1e-13


def test_superop_gate_counts():
    """A noisy rotation is one dense gate on (q, q + n); a noisy controlled phase three diagonal
    patterns; every other gate a pair (row bits, then column bits)."""
    n, e = 3, 0.1
    h = np.array([[1, 1], [1, -1]]) / math.sqrt(2)
    gates = [Gate(U1, q0=1, m=h, noise=NOISE_ROT), Gate(U1, q0=2, m=h), Gate(CP, q0=0, q1=2, theta=0.3,
                                                                            noise=NOISE_PHASE),
             Gate(CP, q0=0, q1=1, theta=0.4), Gate(FLIP, mask=5, value=4)]
    sg = q.dm_superop(gates, n, e)
    kinds = [int(g.kind) for g in sg]
    assert kinds == [4, U1, U1, DIAG, DIAG, DIAG, CP, CP, FLIP, FLIP]
    assert (sg[0].q0, sg[0].q1) == (1, 1 + n)
    assert (sg[1].q0, sg[2].q0) == (2 + n, 2)
    assert [(int(g.mask), int(g.value)) for g in sg[3:6]] == [(5 << n, 5 << n), (5, 5), (5 | 5 << n,) * 2]
    assert math.isclose(sg[5].m[0], math.exp(e * e)) and sg[5].m[1] == 0.0
    assert (sg[6].theta, sg[7].theta) == (0.4, -0.4)
    assert [(int(g.mask), int(g.value)) for g in sg[8:]] == [(5 << n, 4 << n), (5, 4)]
    # at e = 0 the noisy gates are their ideal pairs
    assert [int(g.kind) for g in q.dm_superop(gates, n, 0.0)] == [U1, U1, U1, U1, CP, CP, CP, CP, FLIP, FLIP]


def test_superop_rejects_bad_arguments():
    g = [Gate(U1, q0=0, m=np.eye(2))]
    L = q.lib()
    cnt = ctypes.c_int(0)
    ga = q.gate_array(g)
    assert L.qs_dm_superop(ga, 1, 0, 0.0, None, 0, cnt) != 0
    assert L.qs_dm_superop(ga, 1, 18, 0.0, None, 0, cnt) != 0
    assert L.qs_dm_superop(ga, 1, 2, -0.1, None, 0, cnt) != 0
    assert L.qs_dm_superop(ga, 1, 2, float("nan"), None, 0, cnt) != 0
    assert L.qs_dm_superop(ga, 1, 2, 0.1, None, 0, None) != 0
    assert L.qs_dm_superop(ga, 1, 2, 0.0, None, 0, cnt) == 0 and cnt.value == 2
    out = (q.Gate * 1)()
    assert L.qs_dm_superop(ga, 1, 2, 0.0, out, 1, cnt) != 0     # cap below the two gates
    bad = q.gate_array([Gate(DIAG, m=np.array([1j]), mask=1, value=2)])      # value outside mask
    assert L.qs_dm_superop(bad, 1, 2, 0.0, None, 0, cnt) != 0
    assert q.dm_run_bytes_required(g, 0, q.C128) == 0
    assert q.dm_run_bytes_required(g, 2, q.C128, e=0.1) > 0


# ----------------------------------------------------------------------------------------
# The diagonal gate kind in the oracle, pinned to the gates it generalises and to D rho D^+.
def test_oracle_diag_reduces_to_cp_and_flip():
    rng = np.random.default_rng(1)
    n = 4
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    theta = 0.77
    cp = Circuit(n, [Gate(CP, q0=1, q1=3, theta=theta)], name="cp")
    dg = Circuit(n, [Gate(DIAG, m=np.array([np.exp(-1j * theta)]), mask=0b1010, value=0b1010)], name="d")
    assert np.max(np.abs(oracle.sv_apply(cp, psi.copy()) - oracle.sv_apply(dg, psi.copy()))) <= 1e-15
    fl = Circuit(n, [Gate(FLIP, mask=0b0110, value=0b0100)], name="f")
    dm = Circuit(n, [Gate(DIAG, m=np.array([-1.0 + 0j]), mask=0b0110, value=0b0100)], name="d")
    assert np.max(np.abs(oracle.sv_apply(fl, psi.copy()) - oracle.sv_apply(dm, psi.copy()))) <= 1e-15


def test_oracle_dm_diag_is_d_rho_d_dagger():
    n = 3
    N = 1 << n
    f = 0.6 * np.exp(0.4j)
    mask, value = 0b101, 0b001
    c = Circuit(n, [Gate(U1, q0=k, m=np.array([[1, 1], [1, -1]]) / math.sqrt(2)) for k in range(n)]
                + [Gate(U1, q0=1, m=np.array([[1, 0], [0, 1j]]))]
                + [Gate(DIAG, m=np.array([f]), mask=mask, value=value)], name="hd", init_index=3)
    got = oracle.dm_run(c, 0.0)
    pre = Circuit(n, c.gates[:-1], name="h", init_index=3)
    psi = oracle.sv_run(pre, 0.0)
    d = np.array([f if (i & mask) == value else 1.0 for i in range(N)])
    D = np.diag(d)
    rho = np.outer(psi, psi.conj())
    assert np.max(np.abs(got - D @ rho @ D.conj().T)) <= 1e-15
