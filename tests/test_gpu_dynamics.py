"""Per-iteration dynamics of noisy Grover search (Section 3.2, the paper's comparison of Monte
Carlo, fixed-rank and exact density-matrix evolution): after every iteration the library's exact
density matrix against the oracle's, rank 1 against eq. (10), higher ranks against the
inequality unnormalised <= exact, and the Monte Carlo trajectories against the oracle's, with
their mean within five standard errors of the exact density matrix."""
import math

import numpy as np
import pytest

import oracle
from workloads import Circuit, grover

from paper_forms import eq10, grover_p_ideal

torch = pytest.importorskip("torch")
import paper_1412_2293_amd as q  # noqa: E402

pytestmark = pytest.mark.gpu


def test_grover_dynamics_every_iteration():
    n, e, seed, T = 7, 0.05, 3, 1024
    c = grover(n, seed=seed)
    j = c.meta["iterations"]
    per = 2 * n + 2
    ends = [n + k * per for k in range(j + 1)]
    ga = q.gate_array(c.gates)
    w = q.StateVector(n, q.C128, 1)
    w.init_basis(c.marked)
    rho = q.StateVector(2 * n, q.C128, 1)
    rho.init_basis(0)
    frs = {r: q.FixedRank(n, r, q.C128) for r in (1, 2, 4, 8)}
    for fr in frs.values():
        fr.init_basis(0)
    g0 = 0
    for k, end in enumerate(ends):
        for g in ga[g0:end]:
            q.dm_apply_gate(rho, g, e)
            for fr in frs.values():
                fr.apply_noisy_gate(g, e)
        g0 = end
        prefix = Circuit(n, c.gates[:end], init_index=c.init_index, marked=c.marked)
        p_dm = q.dm_fidelity(rho, w, 0)[0]
        ref = oracle.dm_run(prefix, e)
        p_ref = float(ref[c.marked, c.marked].real)
        assert abs(p_dm - p_ref) <= 1e-12 * max(p_ref, 1e-300), (k, p_dm, p_ref)
        fu, fn, _ = frs[1].fidelity(w)
        assert abs(fu - eq10(n, k, e)) <= 1e-12 * eq10(n, k, e), (k, fu, eq10(n, k, e))
        assert abs(fn - grover_p_ideal(n, k)) <= 1e-12, k
        for r in (2, 4, 8):
            fu_r = frs[r].fidelity(w)[0]
            assert fu_r <= p_dm + 1e-12, (k, r, fu_r, p_dm)
        res = q.run_trajectories(ga[:end], n, c.init_index, q.C128, T, e=e, seed=seed, marked=c.marked)
        p = np.asarray(res["p"])
        _, p_or = oracle.run_trajectories(prefix, e, seed, range(8))
        np.testing.assert_allclose(p[:8], p_or, rtol=1e-12, atol=1e-15)
        sem = p.std(ddof=1) / math.sqrt(T)
        assert abs(p.mean() - p_dm) <= 5 * sem + 1e-12, (k, p.mean(), p_dm, sem)
