"""GPU parity of the fused passes whose register rounds run as dense 16 x 16 blocks on the FP32
matrix cores (plan field mfma = 1, complex<float>): every amplitude of every trajectory against
the oracle at n = 12-14, and the 32-qubit random layer against its closed form.

Tolerances as for every complex<float> path: states within 3e-5 relative, |dF| <= 1e-5."""
import numpy as np
import pytest

import oracle
from workloads import qft, random_layers, random_mixed_circuit

from paper_forms import first_layer_pairs, pair_product_amplitudes, pair_product_fidelity

torch = pytest.importorskip("torch")
import paper_1412_2293_amd as q  # noqa: E402

pytestmark = pytest.mark.gpu


def rel_err(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def unpermute(state, layout, n):
    idx = np.arange(1 << n, dtype=np.int64)
    phys = np.zeros_like(idx)
    for qb in range(n):
        phys |= ((idx >> qb) & 1) << int(layout[qb])
    return state[phys]


def block_rounds(c, plan):
    d = q.plan_describe(c.gates, c.n, q.C64, plan)
    return sum(1 for p in d["passes"] for st in p["stages"] for rd in st["rounds"] if rd["block_rec"] >= 0)


CASES = [("random14", lambda: random_layers(14, 5, seed=31, pairing="random")),
         ("brick13", lambda: random_layers(13, 3, seed=32)),
         ("mixed14", lambda: random_mixed_circuit(14, 200, seed=33)),
         ("qft13", lambda: qft(13, seed=34))]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("plan", [{"fuse": 1, "mfma": 1}, {"fuse": 1, "tile_bits": 10, "reg_bits": 4, "run_bits": 2,
                                                           "mfma": 1}], ids=["t12", "t10"])
def test_block_rounds_full_states(name, make, plan):
    c = make()
    if not name.startswith("mixed"):
        # dense two-qubit gates and standalone diagonals break a mixed circuit's rounds
        assert block_rounds(c, plan) >= 1
    T, e, seed = 3, 0.1, 17
    print(f"mfma {name} plan={plan}", flush=True)
    res = q.run_trajectories(c.gates, c.n, c.init_index, q.C64, T, e=e, seed=seed, plan=plan, traj_base=2)
    F_ref, _, ideal, states = oracle.run_trajectories(c, e, seed, range(2, 2 + T), keep_states=True)
    st = q.trajectory_states(res, c.n, q.C64, T).cpu().numpy().astype(np.complex128)
    assert rel_err(unpermute(st[0], res["layout"], c.n), ideal) <= 3e-5
    for t in range(T):
        assert rel_err(unpermute(st[t + 1], res["layout"], c.n), states[t]) <= 3e-5
    assert np.max(np.abs(res["F"] - F_ref)) <= 1e-5


def test_block_rounds_equal_their_graph_replay():
    c = random_layers(12, 4, seed=35, pairing="random")
    plan = {"fuse": 1, "mfma": 1}
    assert block_rounds(c, plan) >= 1
    with q.TrajGraph(c.gates, c.n, q.C64, 4, plan=plan) as g:
        for init in (0, 77):
            a = g.launch(init, e=0.05, seed=3)
            b = q.run_trajectories(c.gates, c.n, init, q.C64, 4, e=0.05, seed=3, plan=plan)
            assert np.array_equal(a["F"], b["F"])


def test_block_rounds_random_layer_n32_full_size():
    """The first random layer at n = 32 (two 32 GiB slots) on block rounds against the pair
    product closed form."""
    n, e, seed = 32, 0.05, 4
    c = random_layers(n, 1, seed, pairing="brickwork")
    plan = {"fuse": 1, "mfma": 1}
    assert block_rounds(c, plan) >= 1
    res = q.run_trajectories(c.gates, n, 0, q.C64, 1, e=e, seed=seed, plan=plan)
    xi = oracle.normals(seed, [g.site for g in c.gates], [0])[0]
    xi_by_site = {g.site: float(x) for g, x in zip(c.gates, xi)}
    pairs = first_layer_pairs(c, xi_by_site, e)
    ideal = first_layer_pairs(c, {}, 0.0)
    assert abs(res["F"][0] - pair_product_fidelity(ideal, pairs)) <= 1e-5
    rng = np.random.default_rng(6)
    idx = np.concatenate([[0, (1 << n) - 1, 0x55555555, 0xAAAAAAAA], rng.integers(0, 1 << n, 4092)])
    states = q.trajectory_states(res, n, q.C64, 1)
    phys = np.zeros_like(idx)
    for qb in range(n):
        phys |= ((idx >> qb) & 1) << int(res["layout"][qb])
    got = states[1][torch.as_tensor(phys, device=states.device)].cpu().numpy().astype(np.complex128)
    ref = pair_product_amplitudes(pairs, idx)
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))
    del res, states
    torch.cuda.empty_cache()
