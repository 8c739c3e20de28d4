"""Full-size parity of the dense two-qubit sweeps (per-gate plan) at n = 28: a layer of random
4 x 4 unitaries on disjoint qubit pairs leaves a product of two-qubit states, so every amplitude
has a closed form (the product of one entry of each pair's first column).  Adjacent pairs
(2i, 2i + 1) put the lower qubit among a wave's lane bits for the first pairs (the lane-exchange
kernel) and above them for the rest; far pairs (i, i + 14) the same with long strides.  The slots
are enough that both kernels' grids reach their 2^21-block cap and walk the state in their
grid-stride loops.

Tolerances: complex<double> 1e-14 absolute on amplitudes of size 2^-14, complex<float> 2e-8; F = 1
for every slot (the gates are noiseless) within 1e-12 / 1e-5.
"""
import numpy as np
import pytest

from workloads import U2, Circuit, Gate

torch = pytest.importorskip("torch")
import paper_1412_2293_amd as q  # noqa: E402

pytestmark = pytest.mark.gpu


def _unitary4(rng):
    z = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    Q, R = np.linalg.qr(z)
    return Q * (np.diag(R) / np.abs(np.diag(R)))


@pytest.mark.parametrize("pairing", ["adjacent", "far"])
@pytest.mark.parametrize("dtype,T", [(q.C64, 16), (q.C128, 8)], ids=["c64", "c128"])
def test_dense_pairs_n28_unfused_against_product_closed_form(dtype, T, pairing):
    n = 28
    rng = np.random.default_rng(7 if pairing == "adjacent" else 8)
    pairs = [(2 * i, 2 * i + 1) for i in range(14)] if pairing == "adjacent" else [(i, i + 14) for i in range(14)]
    # every other pair in reversed order, so both operand orders of the gate occur
    pairs = [(a, b) if k % 2 == 0 else (b, a) for k, (a, b) in enumerate(pairs)]
    mats = [_unitary4(rng) for _ in pairs]
    c = Circuit(n, [Gate(U2, q0=a, q1=b, m=m) for (a, b), m in zip(pairs, mats)], name=f"u2pairs-{pairing}")
    vec = 2 if dtype == q.C64 else 1
    # one item per thread of 256-thread blocks: the lane kernel has 2^(n - 1) / vec items per slot
    # (vectors with the upper qubit clear), the other 2^(n - 2) / vec (groups of four vectors)
    assert (T + 1) * (1 << (n - 2)) // vec // 256 > (1 << 21)
    print(f"[full size] {c.name} {'c64' if dtype == q.C64 else 'c128'} T={T}", flush=True)
    res = q.run_trajectories(c.gates, n, 0, dtype, T, plan={"fuse": 0})
    assert np.all(np.abs(res["F"] - 1.0) <= (1e-12 if dtype == q.C128 else 1e-5))
    idx = np.concatenate([[0, 1, (1 << n) - 1, 0x5555555, 0xAAAAAAA], rng.integers(0, 1 << n, 1019)]).astype(np.int64)
    ref = np.ones(idx.size, np.complex128)
    for (a, b), m in zip(pairs, mats):
        local = ((idx >> a) & 1) + 2 * ((idx >> b) & 1)     # local index bit(q0) + 2 bit(q1)
        ref *= m[local, 0]
    st = q.trajectory_states(res, n, dtype, T)
    for s in (0, T):
        got = st[s].index_select(0, torch.as_tensor(idx, device=st.device)).cpu().numpy().astype(np.complex128)
        assert np.max(np.abs(got - ref)) <= (1e-14 if dtype == q.C128 else 2e-8), s
    del res, st
    torch.cuda.empty_cache()
