"""GPU parity: the HIP path through the C ABI against the CPU oracle (and, at full size, the
closed forms the oracle is pinned to).

Tolerances: complex<double> states within 1e-12 relative (2-norm of the difference over the
norm) and fidelities within 1e-12 relative; complex<float> amplitudes (with FP64 reductions)
within |dF| <= 1e-5 absolute, the bound stated for the single-precision path.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import fixed_rank
from workloads import (CP, FLIP, H_MATRIX, NOISE_PHASE, NOISE_ROT, U1, Circuit, Gate, chain_heavy_circuit,
                       grover, qft, random_layers, random_mixed_circuit)

from paper_forms import (eq10, first_layer_pairs, grover_p_ideal, pair_product_amplitudes,
                         pair_product_fidelity, qft_noisy_amplitudes)

torch = pytest.importorskip("torch")
import paper_1412_2293_amd as q  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {q.C128: 1e-12, q.C64: 1e-5}
NAMES = {q.C128: "c128", q.C64: "c64"}


def rel_err(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def unpermute(state: np.ndarray, layout, n):
    """Logical-order amplitudes from a state stored with logical qubit q at bit layout[q]."""
    idx = np.arange(1 << n, dtype=np.int64)
    phys = np.zeros_like(idx)
    for qb in range(n):
        phys |= ((idx >> qb) & 1) << int(layout[qb])
    return state[phys]


def to_device_states(sv: "q.StateVector", states: np.ndarray):
    amps = sv.amplitudes()
    t = torch.as_tensor(states.astype(np.complex64 if sv.dtype == q.C64 else np.complex128))
    amps.copy_(t.to(amps.device))
    torch.cuda.synchronize()


def from_device(sv):
    torch.cuda.synchronize()
    return sv.amplitudes().cpu().numpy().astype(np.complex128)


# ----------------------------------------------------------------------------------------
def test_noise_draws_bit_exact():
    sites = np.arange(0, 1500, dtype=np.uint32) * 7 + 3
    for seed, request, tb, T in [(0, 0, 0, 64), ((1 << 40) + 5, 7, 1000, 32), (0xFFFFFFFFFFFFFFFF, 3, 2**31, 8)]:
        got = q.noise_draw(seed, sites, T, traj_base=tb, request=request).cpu().numpy()
        ref = oracle.normals(seed, sites, np.arange(tb, tb + T, dtype=np.uint64).astype(np.uint32), request=request)
        assert got.shape == ref.shape
        mism = np.count_nonzero(got.view(np.uint64) != ref.view(np.uint64))
        assert mism == 0, f"{mism} of {got.size} deviates differ (max |d| {np.max(np.abs(got - ref)):.3e})"


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 9, 13])
def test_apply_gate_every_kind_and_position(dtype, n):
    rng = np.random.default_rng(100 + n)
    T = 3
    circ = random_mixed_circuit(n, 40 if n > 1 else 10, seed=200 + n)
    # make sure both end qubits are hit by dense one-qubit gates
    from workloads import haar_2x2
    circ.gates += [Gate(U1, q0=0, m=haar_2x2(rng), noise=NOISE_ROT), Gate(U1, q0=n - 1, m=haar_2x2(rng), noise=NOISE_ROT)]
    for i, g in enumerate(circ.gates):
        g.site = i
    psi0 = rng.standard_normal((T, 1 << n)) + 1j * rng.standard_normal((T, 1 << n))
    psi0 /= np.linalg.norm(psi0, axis=1, keepdims=True)
    sv = q.StateVector(n, dtype, T)
    to_device_states(sv, psi0)
    e, seed, request, tb = 0.2, 77, 5, 11
    ref = psi0.copy()
    for g in circ.gates:
        q.apply_gate(sv, g, e=e, seed=seed, request=request, traj_base=tb)
        one = Circuit(n, [g])
        for t in range(T):
            ref[t] = oracle.sv_apply(one, ref[t], e=e, seed=seed, traj=tb + t, request=request)
    got = from_device(sv)
    for t in range(T):
        err = rel_err(got[t], ref[t])
        assert err <= (1e-12 if dtype == q.C128 else 2e-5), (NAMES[dtype], n, t, err)
    sv.close()


@pytest.mark.parametrize("fuse", [0, 1])
@pytest.mark.parametrize("dtype", [q.C128, q.C64])
def test_grover_n10_200_trajectories(dtype, fuse):
    """Plain-method workload: Grover n = 10, 200 trajectories, e = 0.01, seed 0."""
    c = grover(10, seed=0)
    T, e, seed = 200, 0.01, 0
    res = q.run_trajectories(c.gates, c.n, c.init_index, dtype, T, e=e, seed=seed, marked=c.marked,
                             plan={"fuse": fuse})
    F_ref, p_ref = oracle.run_trajectories(c, e, seed, range(T))
    if dtype == q.C128:
        assert np.max(np.abs(res["F"] - F_ref) / F_ref) <= 1e-12
        assert np.max(np.abs(res["p"] - p_ref) / p_ref) <= 1e-12
    else:
        assert np.max(np.abs(res["F"] - F_ref)) <= 1e-5
        assert np.max(np.abs(res["p"] - p_ref)) <= 1e-5
    assert np.all(np.abs(res["norm"] - 1.0) <= TOL[dtype] * 10)


PLANS = [
    {"fuse": 0},
    {"fuse": 1},
    {"fuse": 1, "tile_bits": 8, "reg_bits": 2, "run_bits": 2},
    {"fuse": 1, "tile_bits": 9, "reg_bits": 3, "run_bits": 3},
    {"fuse": 1, "tile_bits": 7, "reg_bits": 4, "run_bits": 1},
    {"fuse": 1, "tile_bits": 6, "reg_bits": 2, "run_bits": 2},
]


@pytest.mark.parametrize("plan", PLANS, ids=lambda p: "-".join(f"{k}{v}" for k, v in p.items()))
@pytest.mark.parametrize("dtype", [q.C128, q.C64])
@pytest.mark.parametrize("n", [11, 14])
def test_mixed_circuits_every_plan(n, dtype, plan):
    c = random_mixed_circuit(n, 90, seed=300 + n)
    T, e, seed = 3, 0.15, 9
    res = q.run_trajectories(c.gates, n, c.init_index, dtype, T, e=e, seed=seed, plan=plan, traj_base=4)
    F_ref, _, ideal, states = oracle.run_trajectories(c, e, seed, range(4, 4 + T), keep_states=True)
    st = q.trajectory_states(res, n, dtype, T).cpu().numpy().astype(np.complex128)
    tol = 1e-12 if dtype == q.C128 else 3e-5
    assert rel_err(unpermute(st[0], res["layout"], n), ideal) <= tol
    for t in range(T):
        assert rel_err(unpermute(st[t + 1], res["layout"], n), states[t]) <= tol
    assert np.max(np.abs(res["F"] - F_ref)) <= (1e-12 if dtype == q.C128 else 1e-5)


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
@pytest.mark.parametrize("n,plan", [(14, {"fuse": 1}), (15, {"fuse": 1}), (13, {"fuse": 0}),
                                    (12, {"fuse": 1, "tile_bits": 10, "reg_bits": 4}),
                                    (12, {"fuse": 1, "tile_bits": 6, "reg_bits": 1, "run_bits": 2})])
def test_qft_states_and_fidelities(n, plan, dtype):
    c = qft(n, seed=n)
    T, e, seed = 3, 0.05, 21
    res = q.run_trajectories(c.gates, n, c.init_index, dtype, T, e=e, seed=seed, plan=plan)
    F_ref, _, ideal, states = oracle.run_trajectories(c, e, seed, range(T), keep_states=True)
    st = q.trajectory_states(res, n, dtype, T).cpu().numpy().astype(np.complex128)
    tol = 1e-12 if dtype == q.C128 else 3e-5
    assert rel_err(unpermute(st[0], res["layout"], n), ideal) <= tol
    for t in range(T):
        assert rel_err(unpermute(st[t + 1], res["layout"], n), states[t]) <= tol
    assert np.max(np.abs(res["F"] - F_ref)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
@pytest.mark.parametrize("plan", [{"fuse": 1}, {"fuse": 1, "tile_bits": 8, "reg_bits": 3, "run_bits": 2},
                                  {"fuse": 1, "tile_bits": 6, "reg_bits": 2, "run_bits": 2}],
                         ids=["default", "t8r3", "t6r2"])
def test_qft_basis_folded_phases_every_input(dtype, plan):
    """The QFT's controlled phases fold into the target's Hadamard as one factor per tile taken
    from the run's basis bits (the control is still untouched there): inputs with no ones, all
    ones, alternating bits and a random index, every amplitude of every trajectory against the
    oracle."""
    n = 13
    c0 = qft(n, seed=8)
    d = q.plan_describe(c0.gates, n, dtype, plan)
    assert any(ph[0] == 3 for p in d["passes"] for st in p["stages"] for rd in st["rounds"]
               for op in rd["ops"] for ph in op["phases"])
    T, e, seed = 3, 0.08, 13
    for x in (0, (1 << n) - 1, 0x0AAA, 0x1555, c0.init_index):
        c = Circuit(n, c0.gates, name=c0.name, init_index=x)
        res = q.run_trajectories(c.gates, n, x, dtype, T, e=e, seed=seed, plan=plan)
        F_ref, _, ideal, states = oracle.run_trajectories(c, e, seed, range(T), keep_states=True)
        st = q.trajectory_states(res, n, dtype, T).cpu().numpy().astype(np.complex128)
        tol = 1e-12 if dtype == q.C128 else 3e-5
        assert rel_err(unpermute(st[0], res["layout"], n), ideal) <= tol, x
        for t in range(T):
            assert rel_err(unpermute(st[t + 1], res["layout"], n), states[t]) <= tol, (x, t)
        assert np.max(np.abs(res["F"] - F_ref)) <= TOL[dtype], x


@pytest.mark.parametrize("n,plan", [(13, {"fuse": 1, "tile_bits": 12, "reg_bits": 4, "run_bits": 4}),
                                    (14, {"fuse": 1, "tile_bits": 8, "reg_bits": 4, "run_bits": 2}),
                                    (16, {"fuse": 1, "tile_bits": 12, "reg_bits": 4, "run_bits": 4}),
                                    (18, {"fuse": 1, "tile_bits": 10, "reg_bits": 4, "run_bits": 2})],
                         ids=["n13t12", "n14t8", "n16t12", "n18t10"])
@pytest.mark.parametrize("dtype", [q.C128, q.C64])
def test_straight_line_rounds_full_states(n, plan, dtype):
    """16-register tiles run the rounds of the QFT's passes (untouched targets, register bits
    3..0) and of Grover's (touched targets, bits 0..3, and at n = 16 and 18 two such runs around
    the oracle's or the diffusion's sign flip) straight-line: every amplitude of every trajectory
    against the oracle."""
    seqs = set()
    tol = 1e-12 if dtype == q.C128 else 3e-5
    for c in (qft(n, seed=n + 20), grover(n, seed=n + 20, iterations=3)):
        d = q.plan_describe(c.gates, n, dtype, plan)
        seqs |= {rd["seq"] for p in d["passes"] for st in p["stages"] for rd in st["rounds"]}
        T, e, seed = 3, 0.1, 31
        res = q.run_trajectories(c.gates, n, c.init_index, dtype, T, e=e, seed=seed, plan=plan)
        F_ref, _, ideal, states = oracle.run_trajectories(c, e, seed, range(T), keep_states=True)
        st = q.trajectory_states(res, n, dtype, T).cpu().numpy().astype(np.complex128)
        assert rel_err(unpermute(st[0], res["layout"], n), ideal) <= tol, c.name
        for t in range(T):
            assert rel_err(unpermute(st[t + 1], res["layout"], n), states[t]) <= tol, (c.name, t)
        assert np.max(np.abs(res["F"] - F_ref)) <= TOL[dtype], c.name
    assert 4 in seqs and (n < 16 or 9 in seqs)


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
def test_grover20_full_size(dtype):
    """Grover n = 20 with its full 804 iterations through the fused passes (two per iteration,
    list-scheduled; rounds straight-line around the sign flips): the ideal slot's probabilities
    against the closed form sin^2((2j+1)asin 2^-n/2) on the marked index and its complement
    spread evenly over the others; the noisy trajectories' fidelities and marked probabilities
    against the same circuit as per-gate sweeps (complex<double>), and against the complex<double>
    fused run (complex<float>).  The bounds are those of 33,788 gate updates in sequence: about
    that many roundings of the working precision (2e-11 for complex<double>, where one gate's
    bound is 1e-12).  In complex<float> the norm drifts by about 1e-3 over the run (one rounding
    of each Hadamard's 1/sqrt(2) per gate, accumulating in one direction), so its probabilities are
    compared after normalising the state, as the fidelities already are."""
    from paper_forms import grover_p_ideal
    n = 20
    c = grover(n, seed=2)
    j = (len(c.gates) - n) // (2 * n + 2)
    N = 1 << n
    T, e, seed = 3, 0.01, 41
    print(f"[grover20] dtype={dtype}", flush=True)
    res = q.run_trajectories(c.gates, n, 0, dtype, T, e=e, seed=seed, marked=c.marked)
    st = q.trajectory_states(res, n, dtype, T)
    prob = (st[0].abs() ** 2).cpu().numpy().astype(np.float64)
    norm = float(prob.sum())
    print(f"[grover20] ideal slot norm^2 {norm:.9f}", flush=True)
    if dtype == q.C64:
        assert abs(norm - 1.0) <= 5e-3
        prob /= norm
    phys = 0
    for qb in range(n):
        phys |= ((c.marked >> qb) & 1) << int(res["layout"][qb])
    p = grover_p_ideal(n, j)
    tol = 2e-11 if dtype == q.C128 else 2e-5
    print(f"[grover20] |dp| {abs(prob[phys] - p):.3e}", flush=True)
    assert abs(prob[phys] - p) <= tol, (prob[phys], p)
    rest = np.delete(prob, phys)
    print(f"[grover20] rest max |d| {np.max(np.abs(rest - (1.0 - p) / (N - 1))):.3e}", flush=True)
    assert np.max(np.abs(rest - (1.0 - p) / (N - 1))) <= tol / N * 8
    del st
    if dtype == q.C128:
        ref = q.run_trajectories(c.gates, n, 0, q.C128, T, e=e, seed=seed, marked=c.marked, plan={"fuse": 0})
        print(f"[grover20] fused vs sweeps max rel dF {np.max(np.abs(res['F'] - ref['F']) / ref['F']):.3e}", flush=True)
        assert np.max(np.abs(res["F"] - ref["F"]) / ref["F"]) <= 2e-11
        assert np.max(np.abs(res["p"] - ref["p"]) / ref["p"]) <= 2e-11
    else:
        ref = q.run_trajectories(c.gates, n, 0, q.C128, T, e=e, seed=seed, marked=c.marked)
        print(f"[grover20] c64 vs c128 max |dF| {np.max(np.abs(res['F'] - ref['F'])):.3e}", flush=True)
        assert np.max(np.abs(res["F"] - ref["F"])) <= 1e-5
        # p is the unnormalised marked probability, so it carries the norm drift
        assert np.max(np.abs(res["p"] - ref["p"])) <= 5e-3 * np.max(ref["p"])
    torch.cuda.empty_cache()


def test_random_layers_n28_full_size_fused_against_sweeps():
    """Eight random layers at n = 28 (brickwork CZ, noisy one-qubit gates and CZ phases): the
    fused run, whose passes and register rounds are list-scheduled out of circuit order, against
    the same circuit as per-gate sweeps in complex<double> (fidelities and norms, 1e-12 relative),
    and the complex<float> fused run against both within the single-precision bound."""
    n = 28
    c = random_layers(n, 8, seed=12, pairing="brickwork")
    T, e, seed = 2, 0.02, 17
    print("[random28] fused c128", flush=True)
    f128 = q.run_trajectories(c.gates, n, c.init_index, q.C128, T, e=e, seed=seed)
    torch.cuda.empty_cache()
    print("[random28] sweeps c128", flush=True)
    s128 = q.run_trajectories(c.gates, n, c.init_index, q.C128, T, e=e, seed=seed, plan={"fuse": 0})
    torch.cuda.empty_cache()
    print("[random28] fused c64", flush=True)
    f64 = q.run_trajectories(c.gates, n, c.init_index, q.C64, T, e=e, seed=seed)
    torch.cuda.empty_cache()
    assert np.max(np.abs(f128["F"] - s128["F"]) / s128["F"]) <= 1e-12
    assert np.max(np.abs(f128["norm"] - s128["norm"])) <= 1e-12
    assert np.max(np.abs(f64["F"] - f128["F"])) <= 1e-5
    assert np.all(np.abs(f64["norm"] - 1.0) <= 1e-4)


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
def test_random_layers_against_oracle(dtype):
    c = random_layers(12, 6, seed=5, pairing="random")
    T = 4
    for plan in ({"fuse": 0}, {"fuse": 1}):
        res = q.run_trajectories(c.gates, 12, 0, dtype, T, e=0.05, seed=3, plan=plan)
        F_ref, _ = oracle.run_trajectories(c, 0.05, 3, range(T))
        assert np.max(np.abs(res["F"] - F_ref)) <= TOL[dtype]


def test_per_trajectory_noise_strength():
    c = qft(10, seed=1)
    es = np.array([0.0, 0.001, 0.01, 0.1, 0.3])
    res = q.run_trajectories(c.gates, 10, c.init_index, q.C128, len(es), e=es, seed=2)
    for t, e in enumerate(es):
        F_ref, _ = oracle.run_trajectories(c, float(e), 2, [t])
        assert abs(res["F"][t] - F_ref[0]) <= 1e-12
    assert abs(res["F"][0] - 1.0) <= 1e-13


# ----------------------------------------------------------------------------------------
# Full-size QFT (n = 26, 64 trajectories per e in one launch): the per-trajectory product
# closed form, evaluated with the oracle's noise draws, pins every fidelity and sampled
# amplitudes.
#
# The unfused cases (one sweep kernel per gate) use enough slots that the sweeps' grids reach
# their 2^21-block cap and every thread block walks the state in its grid-stride loop: the dense
# one-qubit sweep takes 512 work items per block, 2^25 (complex<double>) or 2^24
# (complex<float>, two amplitudes per item) per slot, so 41 and 73 slots need 41 * 2^16 and
# 73 * 2^15 blocks; the two-qubit sweeps (256 items per block, 2^24 or 2^23 per slot) the same.
@pytest.mark.parametrize("dtype,fuse,T", [(q.C64, 1, 128), (q.C128, 1, 16), (q.C64, 0, 72), (q.C128, 0, 40)],
                         ids=["c64-fused", "c128-fused", "c64-unfused", "c128-unfused"])
def test_qft26_full_size_against_closed_form(dtype, fuse, T):
    n = 26
    c = qft(n, seed=1)
    es = np.array([0.001] * (T // 2) + [0.01] * (T // 2))
    seed = 1
    if fuse == 0:
        items_per_block = 512
        per_slot = (1 << (n - 1)) // (2 if dtype == q.C64 else 1)
        assert (T + 1) * per_slot // items_per_block > (1 << 21)   # the grid-stride loop runs
    print(f"qft26 {NAMES[dtype]} fuse={fuse} T={T}", flush=True)
    res = q.run_trajectories(c.gates, n, c.init_index, dtype, T, e=es, seed=seed, plan={"fuse": fuse})
    sites = [g.site for g in c.gates]
    xi = oracle.normals(seed, sites, np.arange(T, dtype=np.uint32))
    st = q.trajectory_states(res, n, dtype, T)
    rng = np.random.default_rng(0)
    sample = rng.integers(0, 1 << n, size=64)
    phys = np.zeros_like(sample)
    for qb in range(n):
        phys |= ((sample >> qb) & 1) << int(res["layout"][qb])
    phys_t = torch.as_tensor(phys, device=st.device)
    for t in range(T):
        F_cf, amp_cf = qft_noisy_amplitudes(c, dict(zip(sites, xi[t])), float(es[t]), sample)
        if dtype == q.C128:
            assert abs(res["F"][t] - F_cf) <= 1e-12 * F_cf, (t, res["F"][t], F_cf)
        else:
            assert abs(res["F"][t] - F_cf) <= 1e-5, (t, res["F"][t], F_cf)
        if t % 16 == 0 or t == T - 1:
            amps = st[t + 1].index_select(0, phys_t).cpu().numpy().astype(np.complex128)
            ref = amp_cf
            assert np.max(np.abs(amps - ref)) <= (1e-14 if dtype == q.C128 else 2e-8) , t
    assert np.all(np.abs(res["norm"] - 1.0) <= (1e-12 if dtype == q.C128 else 1e-4))
    del res, st
    torch.cuda.empty_cache()


# ----------------------------------------------------------------------------------------
# Density matrices and the fixed-rank form.
@pytest.mark.parametrize("dtype", [q.C128, q.C64])
def test_dm_grover_against_oracle(dtype):
    n, e = 6, 0.08
    c = grover(n, seed=4)
    rho = q.StateVector(2 * n, dtype, 1)
    rho.init_basis(0)
    for g in c.gates:
        q.dm_apply_gate(rho, g, e)
    ideal_sv = q.StateVector(n, dtype, 1)
    to_device_states(ideal_sv, oracle.sv_run(c, 0.0)[None, :])
    f, tr = q.dm_fidelity(rho, ideal_sv, 0)
    rho_ref = oracle.dm_run(c, e)
    f_ref, tr_ref = oracle.dm_expect(rho_ref, oracle.sv_run(c, 0.0))
    got = from_device(rho)[0].reshape(1 << n, 1 << n)
    tol = 1e-12 if dtype == q.C128 else 2e-5
    assert rel_err(got, rho_ref) <= tol
    assert abs(f - f_ref.real) <= tol * 10
    assert abs(tr - 1.0) <= tol * 10


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
def test_dm_qft_with_noisy_controlled_phases(dtype):
    """Noisy Hadamards (eq. 6) and noisy controlled phases (eq. 9) on vec(rho) against the
    oracle's Kraus channels, entry by entry."""
    n, e = 6, 0.15
    c = qft(n, seed=3)
    rho = q.StateVector(2 * n, dtype, 1)
    rho.init_basis(c.init_index * ((1 << n) + 1))     # |x><x|: index x * 2^n + x
    for g in c.gates:
        q.dm_apply_gate(rho, g, e)
    ref = oracle.dm_run(c, e)
    got = from_device(rho)[0].reshape(1 << n, 1 << n)
    tol = 1e-12 if dtype == q.C128 else 2e-5
    assert rel_err(got, ref) <= tol
    ideal_sv = q.StateVector(n, dtype, 1)
    to_device_states(ideal_sv, oracle.sv_run(c, 0.0)[None, :])
    f, tr = q.dm_fidelity(rho, ideal_sv, 0)
    f_ref, _ = oracle.dm_expect(ref, oracle.sv_run(c, 0.0))
    assert abs(f - f_ref.real) <= 10 * tol and abs(tr - 1.0) <= 10 * tol


def test_random_layer_n32_full_size_against_closed_form():
    """n = 32 complex<float> (two 32 GiB slots, the shape of the 40-layer large-state run): the
    first layer of the random circuit (Haar gates with rotation noise, then noisy CZ on the
    brickwork pairs) leaves a product of two-qubit states, so sampled amplitudes and the
    fidelity have closed forms given the oracle's noise draws."""
    n, e, seed = 32, 0.05, 4
    c = random_layers(n, 1, seed, pairing="brickwork")
    T = 1
    res = q.run_trajectories(c.gates, n, 0, q.C64, T, e=e, seed=seed)
    assert list(res["layout"]) == list(range(n))
    xi = oracle.normals(seed, [g.site for g in c.gates], [0])[0]
    xi_by_site = {g.site: float(x) for g, x in zip(c.gates, xi)}
    pairs = first_layer_pairs(c, xi_by_site, e)
    ideal = first_layer_pairs(c, {}, 0.0)
    assert abs(res["F"][0] - pair_product_fidelity(ideal, pairs)) <= 1e-5
    assert abs(res["norm"][0] - 1.0) <= 1e-5
    rng = np.random.default_rng(5)
    idx = np.concatenate([[0, (1 << n) - 1, 0x55555555, 0xAAAAAAAA], rng.integers(0, 1 << n, 4092)])
    states = q.trajectory_states(res, n, q.C64, T)
    got = states[1][torch.as_tensor(idx, device=states.device)].cpu().numpy().astype(np.complex128)
    ref = pair_product_amplitudes(pairs, idx)
    got0 = states[0][torch.as_tensor(idx, device=states.device)].cpu().numpy().astype(np.complex128)
    ref0 = pair_product_amplitudes(ideal, idx)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-5 * scale
    assert np.max(np.abs(got0 - ref0)) <= 1e-5 * np.max(np.abs(ref0))


def test_dm_grover13_full_size():
    """vec(rho) at the full n = 13 (2^26 complex<double> entries).  A prefix of gates on the
    lowest, middle and highest qubit plus the oracle flip is compared entry by entry with the
    oracle; the whole circuit is checked through properties that hold at any size: the trace
    stays 1 and <psi|rho|psi> equals the mean fidelity of Monte Carlo trajectories of the same
    circuit (the Kraus channel of eq. 6 is the exact average over xi of eq. 1) within 5
    standard errors."""
    from workloads import Circuit
    n, e = 13, 0.02
    c = grover(n, seed=5)
    hs = {g.q0: g for g in c.gates[:n]}
    flip = next(g for g in c.gates if g.kind == FLIP)
    prefix = Circuit(n, [hs[0], hs[n - 1], hs[6], flip], name="g13prefix", init_index=0, marked=c.marked)
    rho = q.StateVector(2 * n, q.C128, 1)
    rho.init_basis(0)
    for g in prefix.gates:
        q.dm_apply_gate(rho, g, e)
    ref = oracle.dm_run(prefix, e)
    got = from_device(rho)[0].reshape(1 << n, 1 << n)
    assert rel_err(got, ref) <= 1e-12
    del got, ref
    rho.init_basis(0)
    for g in c.gates:
        q.dm_apply_gate(rho, g, e)
    ideal = q.StateVector(n, q.C128, 1)
    to_device_states(ideal, oracle.sv_run(c, 0.0)[None, :])
    f, tr = q.dm_fidelity(rho, ideal, 0)
    assert abs(tr - 1.0) <= 1e-11
    T = 2048
    res = q.run_trajectories(c.gates, n, 0, q.C128, T, e=e, seed=21)
    mc, se = float(np.mean(res["F"])), float(np.std(res["F"]) / math.sqrt(T))
    assert abs(f - mc) <= 5 * se, (f, mc, se)


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
def test_apply_kraus_random_sets(dtype):
    n = 7
    rng = np.random.default_rng(8)
    N = 1 << n
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    rho0 = A @ A.conj().T
    rho0 /= np.trace(rho0)
    sv = q.StateVector(2 * n, dtype, 1)
    to_device_states(sv, rho0.reshape(1, -1))
    ref = rho0
    for qb in [0, 3, n - 1]:
        ops = (rng.standard_normal((3, 2, 2)) + 1j * rng.standard_normal((3, 2, 2))) / 2
        q.apply_kraus(sv, [qb], ops)
        ref = oracle.dm_apply_kraus(ref, n, [qb], ops)
    got = from_device(sv)[0].reshape(N, N)
    assert rel_err(got, ref) <= (1e-12 if dtype == q.C128 else 2e-5)


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
def test_apply_kraus_random_two_qubit_sets(dtype):
    """Two-qubit Kraus sets (the 16 x 16 superoperator sweep on four index bits) against the
    oracle's E rho E^dagger sums, for qubit pairs in both orders, adjacent and far apart."""
    n = 7
    rng = np.random.default_rng(18)
    N = 1 << n
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    rho0 = A @ A.conj().T
    rho0 /= np.trace(rho0)
    sv = q.StateVector(2 * n, dtype, 1)
    to_device_states(sv, rho0.reshape(1, -1))
    ref = rho0
    for pair in [(0, 3), (5, 1), (6, 2), (3, 4), (0, 6)]:
        ops = (rng.standard_normal((3, 4, 4)) + 1j * rng.standard_normal((3, 4, 4))) / 3
        q.apply_kraus(sv, list(pair), ops)
        ref = oracle.dm_apply_kraus(ref, n, list(pair), ops)
    got = from_device(sv)[0].reshape(N, N)
    assert rel_err(got, ref) <= (1e-12 if dtype == q.C128 else 2e-5)


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
@pytest.mark.parametrize("n", [10, 13])
def test_fixed_rank_r1_grover_is_eq10(n, dtype):
    e = 0.02
    c = grover(n, seed=2)
    fr = q.FixedRank(n, 1, dtype)
    fr.init_basis(0)
    for g in c.gates:
        fr.apply_noisy_gate(g, e, tau=1e-9 if dtype == q.C128 else 1e-5,
                            zero_tol=1e-13 if dtype == q.C128 else 1e-6)
    w = q.StateVector(n, dtype, 1)
    w.init_basis(c.marked)
    pu, pn, lt = fr.fidelity(w)
    j = c.meta["iterations"]
    ref = eq10(n, j, e)
    tol = 1e-12 if dtype == q.C128 else 1e-5
    assert abs(pu - ref) <= tol * ref, (pu, ref)
    assert abs(pn - grover_p_ideal(n, j)) <= tol


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
def test_fixed_rank_full_size_n24(dtype):
    """The fixed-rank configuration's size, n = 24.  Rank 1: every Kraus step keeps the
    dominant branch, so p(marked) after j Grover iterations is eq. (10) for any j (here 3).
    Rank 8: invariants of the truncated form — rank <= 8, trace <= 1, orthogonal stored
    columns of total weight 1, F_unnorm = exp(log_trace) F_norm."""
    n, e = 24, 0.02
    c = grover(n, seed=7, iterations=3)
    tau = 1e-9 if dtype == q.C128 else 1e-5
    zt = 1e-13 if dtype == q.C128 else 1e-6
    tol = 1e-12 if dtype == q.C128 else 1e-5
    w = q.StateVector(n, dtype, 1)
    w.init_basis(c.marked)
    fr = q.FixedRank(n, 1, dtype)
    fr.init_basis(0)
    for g in c.gates:
        fr.apply_noisy_gate(g, e, tau=tau, zero_tol=zt)
    pu, pn, lt = fr.fidelity(w)
    assert abs(pu - eq10(n, 3, e)) <= tol * eq10(n, 3, e)
    assert abs(pn - grover_p_ideal(n, 3)) <= tol
    fr.close()
    g1 = grover(n, seed=7, iterations=1)
    fr = q.FixedRank(n, 8, dtype)
    fr.init_basis(0)
    ranks = [fr.apply_noisy_gate(g, e, tau=tau, zero_tol=zt) for g in g1.gates]
    rank, lt = fr.info()
    assert max(ranks) <= 8 and rank == ranks[-1] and lt <= 1e-12
    V = fr.columns()[:rank]
    G = (V.conj() @ V.T).cpu().numpy().astype(np.complex128) if dtype == q.C128 else \
        (V.to(torch.complex128).conj() @ V.to(torch.complex128).T).cpu().numpy()
    gtol = 1e-12 if dtype == q.C128 else 1e-5
    assert abs(np.trace(G).real - 1.0) <= gtol
    assert np.max(np.abs(G - np.diag(np.diag(G)))) <= gtol
    pu, pn, lt2 = fr.fidelity(w)
    assert lt2 == lt and abs(pu - math.exp(lt) * pn) <= 1e-12 and 0.0 <= pn <= 1.0 + gtol


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
def test_fixed_rank_r8_against_oracle(dtype):
    n, e, r = 8, 0.05, 8
    c = grover(n, seed=6, iterations=4)
    tau = 1e-9
    zt = 1e-13 if dtype == q.C128 else 1e-6
    fr = q.FixedRank(n, r, dtype)
    fr.init_basis(0)
    ranks = []
    for g in c.gates:
        ranks.append(fr.apply_noisy_gate(g, e, tau=tau, zero_tol=zt))
    ref = fixed_rank.run_circuit(c, e, r, tau=tau, zero_tol=1e-13)
    ideal = oracle.sv_run(c, 0.0)
    psi = q.StateVector(n, dtype, 1)
    to_device_states(psi, ideal[None, :])
    fu, fn, lt = fr.fidelity(psi)
    fu_ref, fn_ref, lt_ref = ref.fidelity(ideal)
    if dtype == q.C128:
        assert ranks[-1] == len(ref.V)
        assert abs(fu - fu_ref) <= 1e-11 and abs(fn - fn_ref) <= 1e-11 and abs(lt - lt_ref) <= 1e-11
        rank, _ = fr.info()
        V = fr.columns()[:rank].cpu().numpy().T
        np.testing.assert_allclose(np.exp(lt) * V @ V.conj().T, ref.rho(), atol=1e-12)
    else:
        assert abs(fu - fu_ref) <= 1e-5 and abs(fn - fn_ref) <= 1e-5


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
def test_fixed_rank_complex_amplitudes_against_oracle(dtype):
    """Haar-random one-qubit gates make every amplitude complex, so the imaginary part of the
    Gram matrix (and its orientation) matters; Grover alone stays real.  The CZs keep their
    phase noise: each is a two-qubit Kraus step (eq. 9) with truncation."""
    n, e, r = 9, 0.05, 8
    c = random_layers(n, 3, seed=12, pairing="random")
    tau = 1e-9
    zt = 1e-13 if dtype == q.C128 else 1e-6
    fr = q.FixedRank(n, r, dtype)
    fr.init_basis(c.init_index)
    ranks = [fr.apply_noisy_gate(g, e, tau=tau, zero_tol=zt) for g in c.gates]
    ref = fixed_rank.run_circuit(c, e, r, tau=tau, zero_tol=1e-13)
    ideal = oracle.sv_run(c, 0.0)
    psi = q.StateVector(n, dtype, 1)
    to_device_states(psi, ideal[None, :])
    fu, fn, lt = fr.fidelity(psi)
    fu_ref, fn_ref, lt_ref = ref.fidelity(ideal)
    if dtype == q.C128:
        assert ranks[-1] == len(ref.V) == r
        assert abs(fu - fu_ref) <= 1e-11 and abs(fn - fn_ref) <= 1e-11 and abs(lt - lt_ref) <= 1e-11
        rank, _ = fr.info()
        V = fr.columns()[:rank].cpu().numpy().T
        np.testing.assert_allclose(np.exp(lt) * V @ V.conj().T, ref.rho(), atol=1e-12)
    else:
        assert abs(fu - fu_ref) <= 1e-5 and abs(fn - fn_ref) <= 1e-5


# ----------------------------------------------------------------------------------------
def test_timing_records_kernels():
    c = qft(12, seed=0)
    q.timing_reset()
    q.timing_enable(True)
    q.run_trajectories(c.gates, 12, c.init_index, q.C64, 4, e=0.01, seed=0, plan={"fuse": 1})
    q.timing_enable(False)
    t = q.timing_read("fused")
    assert t["launches"] >= 1 and t["ms"] > 0 and t["alg_bytes"] > 0
    q.timing_reset()


def partially_touched_circuit(n: int, n_gates: int, active, seed: int):
    """Random gates whose non-diagonal targets all lie in `active`; controlled phases, sign flips
    and SWAPs may involve every qubit.  The other qubits keep the initial index's values (up to
    relabelling), so fused passes leave tiles and amplitudes outside that support alone and the
    first pass stores the zero tiles."""
    from workloads import CNOT, NOISE_NONE, SWAP, U2, _renumber_sites, haar_2x2, random_unitary
    rng = np.random.default_rng(seed)
    N = 1 << n
    act = list(active)
    gates = []
    for _ in range(n_gates):
        k = int(rng.integers(0, 7))
        if k <= 2:
            gates.append(Gate(U1, q0=int(rng.choice(act)), m=haar_2x2(rng), noise=NOISE_ROT))
        elif k == 3:
            a, b = (int(v) for v in rng.choice(n, size=2, replace=False))
            gates.append(Gate(CP, q0=a, q1=b, theta=float(rng.uniform(0, 2 * math.pi)), noise=NOISE_PHASE))
        elif k == 4:
            a, b = (int(v) for v in rng.choice(act, size=2, replace=False))
            gates.append(Gate(U2, q0=a, q1=b, m=random_unitary(4, rng)) if rng.random() < 0.5
                         else Gate(CNOT, q0=a, q1=b))
        elif k == 5:
            mask = int(rng.integers(0, N)) | (1 << int(rng.integers(0, n)))
            gates.append(Gate(FLIP, mask=mask, value=int(rng.integers(0, N)) & mask))
        else:
            # a SWAP moves the roles of qubits: keep the active set closed under it
            a, b = (int(v) for v in rng.choice(act, size=2, replace=False))
            gates.append(Gate(SWAP, q0=a, q1=b))
    return Circuit(n, _renumber_sites(gates), name=f"partial{n}", init_index=int(rng.integers(0, N)))


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
@pytest.mark.parametrize("plan", [{"fuse": 1}, {"fuse": 1, "tile_bits": 6, "reg_bits": 2, "run_bits": 2},
                                  {"fuse": 1, "tile_bits": 8, "reg_bits": 3, "run_bits": 3}],
                         ids=["default", "t6r2", "t8r3"])
def test_untouched_qubits_full_states(dtype, plan):
    """Circuits that leave qubits untouched by non-diagonal gates: every amplitude of every
    trajectory (including those the passes never compute, stored as zeros by the first pass)
    against the oracle, for several initial indices."""
    engaged = False
    for n, active, seed in ((12, [0, 3, 4, 9, 10], 1), (13, [1, 2, 5, 6, 7, 11, 12], 2), (14, [13, 12, 8], 3)):
        c = partially_touched_circuit(n, 60, active, seed)
        desc = q.plan_describe(c.gates, n, dtype, plan)
        engaged |= any(p["classical"] for p in desc["passes"][1:]) or desc["passes"][0]["zero_fill"] == 1
        T, e, s = 3, 0.1, 5
        for init in (c.init_index, (1 << n) - 1, 0):
            res = q.run_trajectories(c.gates, n, init, dtype, T, e=e, seed=s, plan=plan)
            ci = Circuit(n, c.gates, name=c.name, init_index=init)
            F_ref, _, ideal, states = oracle.run_trajectories(ci, e, s, range(T), keep_states=True)
            st = q.trajectory_states(res, n, dtype, T).cpu().numpy().astype(np.complex128)
            tol = 1e-12 if dtype == q.C128 else 3e-5
            assert rel_err(unpermute(st[0], res["layout"], n), ideal) <= tol, (n, init)
            for t in range(T):
                assert rel_err(unpermute(st[t + 1], res["layout"], n), states[t]) <= tol, (n, init, t)
            assert np.max(np.abs(res["F"] - F_ref)) <= TOL[dtype]
    assert engaged


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
def test_dm_qft13_full_size_against_closed_form(dtype):
    """Density-matrix QFT at n = 13 (vec(rho) of 2^26 entries), noisy Hadamards (eq. 6) and noisy
    controlled phases (eq. 9): the fidelity to the ideal output equals the noise average of the
    trajectory fidelity, prod_t (1 + exp(-2e^2) exp(-e^2 m_t / 2)) / 2 (m_t = ones of x below
    t), for inputs with few and many ones; Tr rho = 1."""
    from paper_forms import qft_expected_fidelity
    n, e = 13, 0.05
    for x in (1, (1 << n) - 2, 0x0A5B):
        c = qft(n, seed=1)
        c = Circuit(n, c.gates, name=c.name, init_index=x)
        rho = q.StateVector(2 * n, dtype, 1)
        rho.init_basis(x * ((1 << n) + 1))
        for g in c.gates:
            q.dm_apply_gate(rho, g, e)
        ideal = q.StateVector(n, dtype, 1)
        to_device_states(ideal, qft_ideal_state(n, x)[None, :])
        f, tr = q.dm_fidelity(rho, ideal, 0)
        F = qft_expected_fidelity(n, x, e)
        tol = 1e-12 if dtype == q.C128 else 2e-5
        assert abs(f - F) <= tol * F if dtype == q.C128 else abs(f - F) <= tol, (x, f, F)
        assert abs(tr - 1.0) <= tol, (x, tr)
        rho.close()
        ideal.close()


def qft_ideal_state(n, x):
    """QFT|x> = N^-1/2 sum_y exp(-2 pi i x y / N)|y>, the transform's ideal output (numpy FFT)."""
    N = 1 << n
    ex = np.zeros(N, np.complex128)
    ex[x] = 1.0
    return np.fft.fft(ex) / math.sqrt(N)


def test_fixed_rank_unnormalised_never_exceeds_the_density_matrix():
    """Truncation removes a positive semidefinite part at every Kraus step and the later channels
    are positive maps, so the unnormalised fixed-rank <w|rho_r|w> can only fall short of the
    exact density-matrix value, for every r; rank 1 is eq. (10) exactly."""
    n, e = 10, 0.05
    c = grover(n, seed=8, iterations=6)
    w = q.StateVector(n, q.C128, 1)
    w.init_basis(c.marked)
    rho = q.StateVector(2 * n, q.C128, 1)
    rho.init_basis(0)
    for g in c.gates:
        q.dm_apply_gate(rho, g, e)
    p_dm, tr = q.dm_fidelity(rho, w, 0)
    assert abs(tr - 1.0) <= 1e-12
    prev = None
    for r in (1, 2, 4, 8):
        fr = q.FixedRank(n, r, q.C128)
        fr.init_basis(0)
        for g in c.gates:
            fr.apply_noisy_gate(g, e)
        fu, fn, lt = fr.fidelity(w)
        assert fu <= p_dm * (1 + 1e-12), (r, fu, p_dm)
        assert lt <= 1e-12
        if r == 1:
            assert abs(fu - eq10(n, c.meta["iterations"], e)) <= 1e-12 * eq10(n, c.meta["iterations"], e)
        prev = fu
        fr.close()
    assert prev > 0.5 * p_dm   # r = 8 keeps most of it
    rho.close()
    w.close()


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
@pytest.mark.parametrize("plan", [{"fuse": 1}, {"fuse": 1, "tile_bits": 6, "reg_bits": 2, "run_bits": 2},
                                  {"fuse": 1, "tile_bits": 9, "reg_bits": 3, "run_bits": 2}],
                         ids=["default", "t6r2", "t9r3"])
def test_phase_chains_full_states(dtype, plan):
    """Complex one-qubit gates applied as real rotations after an input phase, the leftover
    phases carried along each wire (across diagonal gates, CNOT controls and SWAPs) into the
    chain's last gate: every amplitude of every trajectory against the oracle."""
    for n, seed in ((11, 1), (13, 2)):
        c = chain_heavy_circuit(n, 160, seed)
        desc = q.plan_describe(c.gates, n, dtype, plan)
        assert max(len(ch) for ch in desc["chains"]) >= 5
        T, e, s = 3, 0.2, 8
        res = q.run_trajectories(c.gates, n, c.init_index, dtype, T, e=e, seed=s, plan=plan)
        F_ref, _, ideal, states = oracle.run_trajectories(c, e, s, range(T), keep_states=True)
        st = q.trajectory_states(res, n, dtype, T).cpu().numpy().astype(np.complex128)
        tol = 1e-12 if dtype == q.C128 else 3e-5
        assert rel_err(unpermute(st[0], res["layout"], n), ideal) <= tol, n
        for t in range(T):
            assert rel_err(unpermute(st[t + 1], res["layout"], n), states[t]) <= tol, (n, t)
        assert np.max(np.abs(res["F"] - F_ref)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
def test_dm_qft_with_the_improved_cp_kraus_set(dtype):
    """The controlled phases of a noisy QFT on vec(rho) applied as the eq. (14) Kraus pair
    through the general Kraus sweep give, entry by entry, the state of the eq. (9) path (the two
    sets are one channel), and the oracle's."""
    n, e = 6, 0.2
    c = qft(n, seed=5)
    a = q.StateVector(2 * n, dtype, 1)
    b = q.StateVector(2 * n, dtype, 1)
    for r in (a, b):
        r.init_basis(c.init_index * ((1 << n) + 1))
    for g in c.gates:
        q.dm_apply_gate(a, g, e)
        if g.kind == CP:
            q.apply_kraus(b, [g.q0, g.q1], q.cp_kraus_improved(g.theta, e))
        else:
            q.dm_apply_gate(b, g, e)
    ra = from_device(a)[0].reshape(1 << n, 1 << n)
    rb = from_device(b)[0].reshape(1 << n, 1 << n)
    tol = 1e-12 if dtype == q.C128 else 2e-5
    assert rel_err(rb, ra) <= tol
    assert rel_err(rb, oracle.dm_run(c, e)) <= tol


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
@pytest.mark.parametrize("plan", [{"fuse": 1}, {"fuse": 1, "tile_bits": 8, "reg_bits": 3, "run_bits": 3}],
                         ids=["default", "t8r3"])
def test_random_layers_uniform_factor_variant_full_states(dtype, plan):
    """Random layers, whose folded CZ phases are mostly conditioned on register or tile-number
    bits, run most passes in the kernel variant that reads those blocks' factors uniformly:
    every amplitude of every trajectory against the oracle."""
    n = 14
    c = random_layers(n, 5, seed=1, pairing="random")
    desc = q.plan_describe(c.gates, n, dtype, plan)
    assert any(p["uni_kernel"] for p in desc["passes"]) and not all(p["uni_kernel"] for p in desc["passes"])
    T, e, s = 3, 0.1, 12
    res = q.run_trajectories(c.gates, n, c.init_index, dtype, T, e=e, seed=s, plan=plan)
    F_ref, _, ideal, states = oracle.run_trajectories(c, e, s, range(T), keep_states=True)
    st = q.trajectory_states(res, n, dtype, T).cpu().numpy().astype(np.complex128)
    tol = 1e-12 if dtype == q.C128 else 3e-5
    assert rel_err(unpermute(st[0], res["layout"], n), ideal) <= tol
    for t in range(T):
        assert rel_err(unpermute(st[t + 1], res["layout"], n), states[t]) <= tol, t
    assert np.max(np.abs(res["F"] - F_ref)) <= TOL[dtype]


def test_apply_kraus_rejects_bad_sets_before_device_work():
    """k outside 1..2 is unsupported; equal or out-of-range qubits and non-finite entries are
    invalid; the density matrix is left untouched."""
    n = 3
    sv = q.StateVector(2 * n, q.C128, 1)
    sv.init_basis(0)
    before = from_device(sv).copy()
    ops2 = np.stack([np.eye(4, dtype=np.complex128)])
    for qubits, ops, code in (([0, 1, 2], np.stack([np.eye(8, dtype=np.complex128)]), -4),
                              ([1, 1], ops2, -1), ([0, 3], ops2, -1),
                              ([0, 1], np.full((1, 4, 4), np.nan, np.complex128), -1)):
        with pytest.raises(q.QsimError) as ei:
            q.apply_kraus(sv, qubits, ops)
        assert f"({code})" in str(ei.value), str(ei.value)
    assert np.array_equal(from_device(sv), before)


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
@pytest.mark.parametrize("T", [1, 6, 9])
def test_fused_last_pass_overlaps_edge_cases(dtype, T):
    """The fused runs form the overlaps with the ideal slot inside their last pass (the ideal
    slot alone first, then the others tile-major); the unfused runs keep the separate reduction.
    Covered: one noisy trajectory, slot counts that are not powers of two, programs whose only
    pass is also the first (zero tiles outside the support), a marked amplitude."""
    n = 9
    circuits = [
        Circuit(n, [Gate(U1, q0=3, m=H_MATRIX.copy(), noise=NOISE_ROT)], name="one-h", init_index=5),
        Circuit(n, [Gate(U1, q0=q, m=H_MATRIX.copy(), noise=NOISE_ROT) for q in range(n)] +
                [Gate(CP, q0=0, q1=4, theta=0.7, noise=NOISE_PHASE)], name="h-layer"),
        qft(n, seed=3),
    ]
    marked = 13   # inside the support of the one-gate circuit (|5> and |13>)
    for c in circuits:
        c.marked = marked
        F_ref, p_ref, ideal, states = oracle.run_trajectories(c, 0.1, 4, range(T), keep_states=True)
        out = {}
        for fuse in (0, 1):
            out[fuse] = q.run_trajectories(c.gates, n, c.init_index, dtype, T, e=0.1, seed=4, marked=marked,
                                           plan={"fuse": fuse, "tile_bits": 6, "reg_bits": 2, "run_bits": 2}
                                           if fuse else {"fuse": 0})
        for fuse, res in out.items():
            assert np.max(np.abs(res["F"] - F_ref)) <= TOL[dtype], (c.name, fuse)
            assert np.max(np.abs(res["p"] - p_ref)) <= TOL[dtype], (c.name, fuse)
            norms = [np.vdot(s, s).real for s in states]
            assert np.max(np.abs(res["norm"] - norms)) <= TOL[dtype] * 10, (c.name, fuse)
        assert np.max(np.abs(out[1]["F"] - out[0]["F"])) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [q.C128, q.C64])
@pytest.mark.parametrize("n", [10, 14])
def test_trajectory_results_do_not_depend_on_the_batch(n, dtype):
    """A trajectory's fidelity, marked probability and norm are the same bits whether it runs in
    a batch of 64 or of 5: its noise comes from its own counter, and the overlap sums of a slot do
    not depend on how many slots share the launch.  n = 10 (one 2^10-amplitude tile per slot)
    runs every slot's last pass in one launch and sums the overlaps from the stored states;
    n = 14 in complex<float> (128 KiB per slot) forms them inside the last pass, after slot 0."""
    c = grover(n, seed=3, iterations=3)
    e, seed = 0.02, 21
    full = q.run_trajectories(c.gates, n, c.init_index, dtype, 64, e=e, seed=seed, marked=c.marked)
    for base, T in ((0, 5), (37, 5), (63, 1)):
        part = q.run_trajectories(c.gates, n, c.init_index, dtype, T, e=e, seed=seed, marked=c.marked,
                                  traj_base=base)
        for key in ("F", "p", "norm"):
            assert np.array_equal(part[key], full[key][base:base + T]), (key, base, T)
    # and the batch agrees with the oracle on its first eight trajectories
    F_ref, p_ref = oracle.run_trajectories(c, e, seed, range(8))
    if dtype == q.C128:
        assert np.allclose(full["F"][:8], F_ref, rtol=1e-12, atol=0)
        assert np.allclose(full["p"][:8], p_ref, rtol=1e-12, atol=1e-15)
    else:
        assert np.max(np.abs(full["F"][:8] - F_ref)) <= 1e-5
        assert np.max(np.abs(full["p"][:8] - p_ref)) <= 1e-5
