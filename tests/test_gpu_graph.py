"""GPU: captured trajectory runs (qs_traj_graph_*) replay bit for bit what the eager launch
sequence computes, run after run with new per-run values and eager work in between."""
import numpy as np
import pytest

from workloads import grover, qft, random_layers, random_mixed_circuit

torch = pytest.importorskip("torch")
import paper_1412_2293_amd as q  # noqa: E402

pytestmark = pytest.mark.gpu


def _same(a, b):
    return np.array_equal(a, b) and not np.any(np.isnan(a))


@pytest.mark.parametrize("dtype", [q.C64, q.C128])
@pytest.mark.parametrize("plan", [None, {"fuse": 0}, {"fuse": 1, "tile_bits": 9, "reg_bits": 3, "run_bits": 3}])
def test_replays_equal_eager_runs(dtype, plan):
    c = random_mixed_circuit(13, 50, 9)
    T = 9
    with q.TrajGraph(c.gates, c.n, dtype, T, plan=plan) as g:
        runs = [dict(init=c.init_index, e=0.02, seed=1, request=0, tb=0, marked=5),
                dict(init=17, e=np.linspace(0, 0.05, T), seed=99, request=3, tb=40, marked=-1),
                dict(init=0, e=0.0, seed=2, request=1, tb=0, marked=8191),
                dict(init=c.init_index, e=0.02, seed=1, request=0, tb=0, marked=5)]
        first = None
        for k, r in enumerate(runs):
            got = g.launch(r["init"], e=r["e"], seed=r["seed"], request=r["request"], traj_base=r["tb"],
                           marked=r["marked"])
            # eager work on the default stream between replays
            ref = q.run_trajectories(c.gates, c.n, r["init"], dtype, T, e=r["e"], seed=r["seed"],
                                     request=r["request"], traj_base=r["tb"], marked=r["marked"], plan=plan)
            assert _same(got["F"], ref["F"]), k
            assert _same(got["norm"], ref["norm"]), k
            assert np.array_equal(got["layout"], ref["layout"])
            if r["marked"] >= 0:
                assert _same(got["p"], ref["p"]), k
            if k == 0:
                first = got["F"].copy()
        assert _same(got["F"], first)      # the last run repeats the first


def test_graph_of_grover_and_qft():
    for c, T in ((grover(11, 3, iterations=4), 16), (qft(15, 4), 8), (random_layers(14, 12, 5), 5)):
        marked = c.marked if c.marked is not None else -1
        with q.TrajGraph(c.gates, c.n, q.C64, T) as g:
            got = g.launch(c.init_index, e=0.03, seed=7, marked=marked)
        ref = q.run_trajectories(c.gates, c.n, c.init_index, q.C64, T, e=0.03, seed=7, marked=marked)
        assert _same(got["F"], ref["F"]), c.name


@pytest.mark.parametrize("dtype", [q.C64, q.C128])
def test_qft_graph_with_new_initial_states(dtype):
    """A QFT from a basis state leaves most tile-number bits untouched until its last pass, so
    the passes walk only the tiles that agree with the initial index there, and the per-tile
    phase products depend on it: one graph replayed from several initial indices matches eager
    runs from the same indices."""
    c = qft(15, 4)
    T = 6
    plan = {"fuse": 1, "tile_bits": 8, "reg_bits": 3, "run_bits": 2}
    with q.TrajGraph(c.gates, c.n, dtype, T, plan=plan) as g:
        for init in (c.init_index, 0, (1 << 15) - 1, 0x5A5A & 0x7FFF):
            got = g.launch(init, e=0.04, seed=3)
            ref = q.run_trajectories(c.gates, c.n, init, dtype, T, e=0.04, seed=3, plan=plan)
            assert _same(got["F"], ref["F"]), init
            assert _same(got["norm"], ref["norm"]), init
