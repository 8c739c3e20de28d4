"""Pins for the oracle's state-vector, density-matrix and fixed-rank levels."""
import math

import numpy as np
import pytest

import oracle
from oracle import fixed_rank
from workloads import (CP, FLIP, NOISE_NONE, NOISE_PHASE, NOISE_ROT, U1, Circuit, Gate,
                       grover, qft, random_layers, random_mixed_circuit)

from paper_forms import (first_layer_pairs, pair_product_amplitudes, pair_product_fidelity, eq10, eq11, eq15, full_gate_matrix, grover_ideal, grover_p_ideal,
                         lambdas, qft_expected_fidelity, qft_ideal, qft_noisy_closed_form)


def _rand_state(n, rng):
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_gates_match_kronecker_matrices(n):
    rng = np.random.default_rng(n)
    circ = random_mixed_circuit(n, 60, seed=10 + n)
    for g in circ.gates:
        psi = _rand_state(n, rng)
        one = Circuit(n, [g])
        got = oracle.sv_apply(one, psi, e=0.0)
        ref = full_gate_matrix(n, g) @ psi
        np.testing.assert_allclose(got, ref, atol=1e-13)


def test_noisy_gates_are_u_times_v_and_shifted_phase():
    """eq. (1): U * V(e xi); after eq. (2): theta -> theta + e xi on |11>."""
    n, e, seed, traj = 3, 0.37, 99, 5
    rng = np.random.default_rng(3)
    from workloads import haar_2x2
    gates = [Gate(U1, q0=1, m=haar_2x2(rng), noise=NOISE_ROT, site=11),
             Gate(CP, q0=0, q1=2, theta=0.7, noise=NOISE_PHASE, site=12)]
    xi = oracle.normals(seed, [11, 12], [traj], request=4)[0]
    psi = _rand_state(n, rng)
    got = oracle.sv_apply(Circuit(n, gates), psi, e=e, seed=seed, traj=traj, request=4)
    a = e * xi[0]
    V = np.array([[math.cos(a), math.sin(a)], [-math.sin(a), math.cos(a)]])
    g0 = Gate(U1, q0=1, m=gates[0].m @ V)
    g1 = Gate(CP, q0=0, q1=2, theta=0.7 + e * xi[1])
    ref = full_gate_matrix(n, g1) @ (full_gate_matrix(n, g0) @ psi)
    np.testing.assert_allclose(got, ref, atol=1e-13)


@pytest.mark.parametrize("n", [2, 3, 5, 8, 10])
def test_grover_ideal_closed_form(n):
    c = grover(n, seed=n)
    j = c.meta["iterations"]
    psi = oracle.sv_run(c, 0.0)
    np.testing.assert_allclose(psi, grover_ideal(n, c.marked, j), atol=1e-13)
    assert abs(abs(psi[c.marked]) ** 2 - grover_p_ideal(n, j)) < 1e-13


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 8])
def test_qft_ideal_is_dft(n):
    for x in sorted({0, 1, (1 << n) - 1, (5 * n) % (1 << n)}):
        c = qft(n, seed=0, x=x)
        np.testing.assert_allclose(oracle.sv_run(c, 0.0), qft_ideal(n, x), atol=1e-13)


@pytest.mark.parametrize("n,e", [(4, 0.3), (6, 0.3), (8, 0.05), (10, 0.01)])
def test_noisy_qft_matches_product_closed_form(n, e):
    c = qft(n, seed=n + 100)
    seed = 42
    sites = [g.site for g in c.gates]
    trajs = [0, 3, 17]
    xi = oracle.normals(seed, sites, trajs)
    ideal = oracle.sv_run(c, 0.0)
    for k, t in enumerate(trajs):
        psi = oracle.sv_run(c, e, seed=seed, traj=t)
        F_cf, psi_cf = qft_noisy_closed_form(c, dict(zip(sites, xi[k])), e)
        np.testing.assert_allclose(psi, psi_cf, atol=1e-13)
        assert abs(oracle.fidelity(ideal, psi) - F_cf) < 1e-13


@pytest.mark.parametrize("n", [6, 10])
def test_first_random_layer_is_a_product_of_pair_states(n):
    """One layer of Haar gates (rotation noise) and brickwork CZ (phase noise) from |0>: every
    amplitude and F factor over the CZ pairs (the closed form the n = 32 GPU test uses)."""
    from workloads import random_layers
    e, seed = 0.07, 4
    c = random_layers(n, 1, seed, pairing="brickwork")
    for t in range(3):
        xi = oracle.normals(seed, [g.site for g in c.gates], [t])[0]
        pairs = first_layer_pairs(c, {g.site: float(x) for g, x in zip(c.gates, xi)}, e)
        psi = oracle.sv_run(c, e, seed=seed, traj=t)
        np.testing.assert_allclose(pair_product_amplitudes(pairs, np.arange(1 << n)), psi, atol=1e-14)
        F, _ = oracle.run_trajectories(c, e, seed, [t])
        assert abs(F[0] - pair_product_fidelity(first_layer_pairs(c, {}, 0.0), pairs)) <= 1e-13


def test_norm_preserved_by_noisy_trajectories():
    c = random_layers(6, 8, seed=1)
    for t in range(4):
        psi = oracle.sv_run(c, 0.05, seed=3, traj=t)
        assert abs(np.vdot(psi, psi).real - 1.0) < 1e-13


@pytest.mark.parametrize("n", [1, 2, 3])
def test_kraus_sandwich_matches_full_matrices(n):
    rng = np.random.default_rng(20 + n)
    N = 1 << n
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    rho = A @ A.conj().T
    rho /= np.trace(rho)
    for q in range(n):
        ops = rng.standard_normal((3, 2, 2)) + 1j * rng.standard_normal((3, 2, 2))
        got = oracle.dm_apply_kraus(rho, n, [q], ops)
        ref = sum(full_gate_matrix(n, Gate(U1, q0=q, m=K)) @ rho @ full_gate_matrix(n, Gate(U1, q0=q, m=K)).conj().T
                  for K in ops)
        np.testing.assert_allclose(got, ref, atol=1e-12)
    if n >= 2:
        from workloads import U2
        ops = rng.standard_normal((2, 4, 4)) + 1j * rng.standard_normal((2, 4, 4))
        got = oracle.dm_apply_kraus(rho, n, [n - 1, 0], ops)
        ref = sum(full_gate_matrix(n, Gate(U2, q0=n - 1, q1=0, m=K)) @ rho
                  @ full_gate_matrix(n, Gate(U2, q0=n - 1, q1=0, m=K)).conj().T for K in ops)
        np.testing.assert_allclose(got, ref, atol=1e-12)


def test_dm_unitary_circuit_equals_pure_state():
    c = random_mixed_circuit(3, 40, seed=77)
    psi = oracle.sv_run(c, 0.0)
    rho = oracle.dm_run(c, 0.0)
    np.testing.assert_allclose(rho, np.outer(psi, psi.conj()), atol=1e-13)


@pytest.mark.parametrize("n,e", [(3, 0.2), (5, 0.1), (6, 0.05)])
def test_dm_qft_fidelity_equals_expected_closed_form(n, e):
    """F_DM = E_xi[F_MC], and for QFT on |x> that expectation has the closed product form."""
    for x in [0, 1, (1 << n) - 1, 5 % (1 << n)]:
        c = qft(n, seed=0, x=x)
        rho = oracle.dm_run(c, e)
        f, tr = oracle.dm_expect(rho, qft_ideal(n, x))
        assert abs(tr - 1.0) < 1e-13
        assert abs(f.real - qft_expected_fidelity(n, x, e)) < 1e-13


def test_qft_bounds_ordering():
    """Eq. (11) <= eq. (15) <= exact mean fidelity (averaged over inputs)."""
    for n, e in [(8, 0.01), (8, 0.05), (12, 0.01)]:
        mean_exact = np.mean([qft_expected_fidelity(n, x, e) for x in range(1 << n)])
        assert eq11(n, e) <= eq15(n, e) <= mean_exact


@pytest.mark.parametrize("n,e", [(3, 0.2), (4, 0.1)])
def test_dm_grover_invariants_and_lower_bound(n, e):
    c = grover(n, seed=1)
    rho = oracle.dm_run(c, e)
    assert abs(np.trace(rho) - 1.0) < 1e-13
    np.testing.assert_allclose(rho, rho.conj().T, atol=1e-14)
    assert np.linalg.eigvalsh(rho).min() > -1e-13
    NH = n + 2 * n * c.meta["iterations"]
    l1 = lambdas(e)[0]
    ideal = oracle.sv_run(c, 0.0)
    f, _ = oracle.dm_expect(rho, ideal)
    assert f.real >= l1 ** NH - 1e-14
    assert rho[c.marked, c.marked].real >= l1 ** NH * grover_p_ideal(n, c.meta["iterations"]) - 1e-14


def test_monte_carlo_mean_converges_to_kraus_channel():
    """E over xi of the trajectory projector equals the Kraus-channel density matrix."""
    n, e, T = 2, 0.4, 20000
    c = random_mixed_circuit(n, 12, seed=5)
    rho = oracle.dm_run(c, e)
    acc = np.zeros((1 << n, 1 << n), np.complex128)
    acc2 = np.zeros((1 << n, 1 << n))
    flat = oracle.FlatCircuit(c)
    for t in range(T):
        psi = oracle.sv_run(c, e, seed=11, traj=t, flat=flat)
        P = np.outer(psi, psi.conj())
        acc += P
        acc2 += np.abs(P) ** 2
    mean = acc / T
    sd = np.sqrt(np.maximum(acc2 / T - np.abs(mean) ** 2, 1e-12))
    assert np.all(np.abs(mean - rho) <= 5 * sd / math.sqrt(T) + 1e-12)
    assert np.max(np.abs(mean - rho)) > 0   # the check is not vacuous


def test_fixed_rank_full_rank_equals_exact_dm():
    c = random_mixed_circuit(3, 25, seed=8)
    e = 0.3
    fr = fixed_rank.run_circuit(c, e, r=64)
    np.testing.assert_allclose(fr.rho(), oracle.dm_run(c, e), atol=1e-12)


def test_fixed_rank_full_rank_noisy_qft_equals_exact_dm():
    """Every controlled phase a two-qubit Kraus step (eq. 9), every Hadamard a one-qubit one
    (eq. 6): at a rank bound above the reachable rank nothing is truncated, so the factored rho
    is the exact density matrix (which the closed-form QFT noise average pins)."""
    c = qft(4, seed=1)
    fr = fixed_rank.run_circuit(c, 0.3, r=256)
    np.testing.assert_allclose(fr.rho(), oracle.dm_run(c, 0.3), atol=1e-13)
    assert max(fr.ranks) > 2


@pytest.mark.parametrize("n,e", [(5, 0.2), (8, 0.05), (10, 0.01)])
def test_fixed_rank_rank1_grover_is_eq10(n, e):
    c = grover(n, seed=2)
    fr = fixed_rank.run_circuit(c, e, r=1)
    j = c.meta["iterations"]
    w = np.zeros(1 << n, np.complex128)
    w[c.marked] = 1
    p_unnorm, p_norm, _ = fr.fidelity(w)
    assert abs(p_unnorm - eq10(n, j, e)) <= 1e-12 * eq10(n, j, e)
    assert abs(p_norm - grover_p_ideal(n, j)) < 1e-12


def test_fixed_rank_invariants():
    n, e, r = 6, 0.1, 4
    c = grover(n, seed=3, iterations=2)
    fr = fixed_rank.FixedRank(n, r)
    prev_lt = 0.0
    for g in c.gates:
        if g.kind == 0:
            fr.apply_kraus([g.q0], oracle.kraus_rot(np.asarray(g.m), e))
            Vm = np.stack(fr.V, 1)
            np.testing.assert_allclose(Vm.conj().T @ Vm, np.diag(np.diag(Vm.conj().T @ Vm)), atol=1e-13)
            assert abs(np.sum(np.abs(Vm) ** 2) - 1.0) < 1e-12
            assert len(fr.V) <= r
            assert fr.log_trace <= prev_lt + 1e-15
            prev_lt = fr.log_trace
        elif g.kind == 5:
            fr.apply_flip(g.mask, g.value)


def test_cluster_drop_rule():
    mu = np.array([1.0, 0.5, 0.25, 0.25, 0.25, 0.1])
    assert fixed_rank.select(mu, 3, 1e-9, 1e-13) == 2      # the tie straddles the cut
    assert fixed_rank.select(mu, 5, 1e-9, 1e-13) == 5
    assert fixed_rank.select(mu, 2, 1e-9, 1e-13) == 2
    assert fixed_rank.select(np.array([1.0, 1e-15, 0.0]), 4, 1e-9, 1e-13) == 1
