"""GPU tests of the request server (qs_srv_*): continuous batching must not change any result.

Each request's per-trajectory fidelity, success probability and norm, served in a mix with
other requests, split into batches and overlapped on several streams, must equal bit for bit
the same request run alone through qs_run_trajectories, which the parity tests tie to the
oracle.  The pool must never hold more than its size.
"""
import numpy as np
import pytest

import oracle
from workloads import grover, qft, random_layers, random_mixed_circuit

torch = pytest.importorskip("torch")
import paper_1412_2293_amd as q  # noqa: E402

pytestmark = pytest.mark.gpu


def _requests():
    """A small mixed stream: Grover, QFT, random layers and mixed circuits of 9..14 qubits."""
    rng = np.random.default_rng(11)
    circs = [grover(10, 1, iterations=6), qft(14, 2), random_layers(12, 8, 3, pairing="random"),
             random_mixed_circuit(13, 60, 4), grover(9, 5), qft(11, 6), random_layers(10, 6, 7)]
    reqs = []
    for i, c in enumerate(circs):
        T = int(rng.integers(5, 41))
        e = float(rng.uniform(0.001, 0.05))
        marked = c.marked if c.marked is not None else -1
        reqs.append(dict(circ=c, T=T, e=e, seed=1000 + i, request=i, marked=marked))
    return reqs


def _alone(r, dtype):
    c = r["circ"]
    return q.run_trajectories(c.gates, c.n, c.init_index, dtype, r["T"], e=r["e"], seed=r["seed"],
                              request=r["request"], marked=r["marked"])


def _same(a, b):
    return np.array_equal(a, b) and not np.any(np.isnan(a))


@pytest.mark.parametrize("dtype", [q.C64, q.C128])
def test_mix_equals_alone_bitwise(dtype):
    reqs = _requests()
    alone = [_alone(r, dtype) for r in reqs]
    torch.cuda.synchronize()
    # small batches force several batches per request and interleaving across streams
    with q.Server(pool_bytes=256 << 20, dtype=dtype, max_inflight=4, max_chunk_traj=7) as srv:
        ids = [srv.submit(r["circ"].gates, r["circ"].n, r["circ"].init_index, r["T"], e=r["e"], seed=r["seed"],
                          request=r["request"], marked=r["marked"]) for r in reqs]
        out = [srv.result(j, timeout=120.0) for j in ids]
        st = srv.stats()
    for r, a, o in zip(reqs, alone, out):
        name = r["circ"].name
        assert o["info"]["status"] == 0, name
        assert o["info"]["n_chunks"] == -(-r["T"] // 7), name
        assert _same(o["F"], a["F"]), name
        assert _same(o["norm"], a["norm"]), name
        if r["marked"] >= 0:
            assert _same(o["p"], a["p"]), name
        inf = o["info"]
        assert 0.0 <= inf["t_submit"] <= inf["t_admit"] <= inf["t_done"]
        assert inf["latency_s"] >= inf["queue_s"] >= 0.0
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["trajectories"] == sum(r["T"] for r in reqs)
    assert st["peak_bytes"] <= st["pool_bytes"]
    assert st["peak_inflight"] >= 2, "batches of different requests never overlapped"
    assert st["in_use_bytes"] == 0


def test_mix_matches_oracle_on_a_small_request():
    c = grover(8, 21, iterations=4)
    T, e = 12, 0.03
    with q.Server(pool_bytes=64 << 20, dtype=q.C128, max_inflight=3, max_chunk_traj=5) as srv:
        other = srv.submit(qft(12, 3).gates, 12, qft(12, 3).init_index, 9, e=0.01, seed=4)
        j = srv.submit(c.gates, c.n, c.init_index, T, e=e, seed=77, request=2, marked=c.marked)
        got = srv.result(j, timeout=60.0)
        srv.result(other, timeout=60.0)
    F, p = oracle.run_trajectories(c, e, seed=77, trajs=range(T), request=2)
    assert np.max(np.abs(got["F"] - F) / F) <= 1e-12
    assert np.max(np.abs(got["p"] - p) / np.maximum(p, 1e-300)) <= 1e-12


def test_admission_never_exceeds_the_pool():
    c = qft(16, 5)
    one = q.traj_bytes_required(c.gates, c.n, q.C64, 8)
    pool = int(one * 2.5)          # room for two 8-trajectory batches at a time
    reqs = [(c, 24, 100 + i) for i in range(4)]
    alone = [q.run_trajectories(cc.gates, cc.n, cc.init_index, q.C64, T, e=0.02, seed=s) for cc, T, s in reqs]
    with q.Server(pool_bytes=pool, dtype=q.C64, max_inflight=6, max_chunk_traj=8) as srv:
        ids = [srv.submit(cc.gates, cc.n, cc.init_index, T, e=0.02, seed=s) for cc, T, s in reqs]
        out = [srv.result(j, timeout=120.0) for j in ids]
        st = srv.stats()
    for a, o in zip(alone, out):
        assert _same(o["F"], a["F"])
    assert st["peak_bytes"] <= pool
    assert st["peak_inflight"] <= 2
    assert st["admission_waits"] >= 1
    assert st["chunks"] == 4 * 3


def test_batch_size_shrinks_to_fit_the_pool_and_oversize_is_rejected():
    c = grover(12, 8, iterations=3)
    one = q.traj_bytes_required(c.gates, c.n, q.C64, 1)
    four = q.traj_bytes_required(c.gates, c.n, q.C64, 4)
    with q.Server(pool_bytes=four + 256, dtype=q.C64, max_inflight=2, max_chunk_traj=64) as srv:
        j = srv.submit(c.gates, c.n, c.init_index, 30, e=0.01, seed=5, marked=c.marked)
        got = srv.result(j, timeout=60.0)
        assert got["info"]["chunk_traj"] == 4
        assert got["info"]["n_chunks"] == 8
        alone = q.run_trajectories(c.gates, c.n, c.init_index, q.C64, 30, e=0.01, seed=5, marked=c.marked)
        assert _same(got["F"], alone["F"]) and _same(got["p"], alone["p"])
    with q.Server(pool_bytes=one // 2, dtype=q.C64, max_inflight=1) as srv:
        with pytest.raises(q.QsimError, match="more than the pool"):
            srv.submit(c.gates, c.n, c.init_index, 4, e=0.01, seed=5)


def test_per_trajectory_noise_strengths_follow_their_trajectories():
    c = random_layers(11, 5, 9)
    e = np.linspace(0.0, 0.05, 19)
    alone = q.run_trajectories(c.gates, c.n, c.init_index, q.C64, 19, e=e, seed=3)
    with q.Server(pool_bytes=64 << 20, dtype=q.C64, max_inflight=3, max_chunk_traj=4) as srv:
        got = srv.result(srv.submit(c.gates, c.n, c.init_index, 19, e=e, seed=3), timeout=60.0)
    assert _same(got["F"], alone["F"])
    assert got["F"][0] == 1.0 or abs(got["F"][0] - 1.0) < 1e-6
