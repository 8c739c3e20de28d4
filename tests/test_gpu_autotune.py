"""GPU: the measured autotuner times the candidate shapes, caches the fastest, and the cached
plan gives the same results (to the FP32 bound) as the library's automatic choice."""
import numpy as np
import pytest

from workloads import qft

torch = pytest.importorskip("torch")
import paper_1412_2293_amd as q  # noqa: E402
from paper_1412_2293_amd import autotune  # noqa: E402

pytestmark = pytest.mark.gpu


def test_tune_caches_the_fastest_plan(tmp_path):
    c = qft(16, 4)
    path = str(tmp_path / "plans.json")
    entry = autotune.tune(c.gates, c.n, q.C64, init_index=c.init_index, n_traj=8, reps=1, path=path)
    secs = [x["seconds"] for x in entry["candidates"]]
    assert entry["seconds"] == min(secs) and len(secs) >= 4
    plan = autotune.lookup(c.gates, c.n, q.C64, path)
    assert plan == entry["plan"]
    a = q.run_trajectories(c.gates, c.n, c.init_index, q.C64, 8, e=0.01, seed=2, plan=plan)
    b = q.run_trajectories(c.gates, c.n, c.init_index, q.C64, 8, e=0.01, seed=2)
    assert np.max(np.abs(a["F"] - b["F"])) <= 1e-5
