"""Maximum sizes: index arithmetic past 2^32 amplitudes per slot and byte offsets past 2^36.

* A QFT on n = 33 qubits (2^33 complex<float> amplitudes, 64 GiB per slot, ideal + one noisy
  trajectory) through the fused passes, against the per-trajectory product closed form (the
  oracle's noise draws): the fidelity and sampled amplitudes, including the last index.
* A density-matrix QFT on n = 17 qubits: vec(rho) of 2^34 complex<float> entries (128 GiB, the
  library's largest state) through the fused density-matrix run, against the closed-form noise
  average of the fidelity, prod_t (1 + exp(-2e^2) exp(-e^2 m_t / 2)) / 2, and Tr rho = 1.

Tolerances as for every complex<float> path: |dF| <= 1e-5; amplitudes within 2e-8 absolute
(their size is 2^-16.5).
"""
import math

import numpy as np
import pytest

import oracle
from workloads import qft

from paper_forms import qft_expected_fidelity, qft_noisy_amplitudes

torch = pytest.importorskip("torch")
import paper_1412_2293_amd as q  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.bigmem]


def test_qft33_fused_full_size_against_closed_form():
    torch.cuda.empty_cache()
    n, T, e, seed = 33, 1, 0.01, 7
    c = qft(n, seed=3)
    print(f"[max size] qft{n} c64 fused T={T}", flush=True)
    res = q.run_trajectories(c.gates, n, c.init_index, q.C64, T, e=e, seed=seed, plan={"fuse": 1})
    sites = [g.site for g in c.gates]
    xi = oracle.normals(seed, sites, np.arange(T, dtype=np.uint32))
    rng = np.random.default_rng(1)
    sample = np.concatenate([[0, 1, (1 << 32) - 1, 1 << 32, (1 << n) - 1],
                             rng.integers(0, 1 << n, size=59)]).astype(np.int64)
    F_cf, amp_cf = qft_noisy_amplitudes(c, dict(zip(sites, xi[0])), e, sample)
    assert abs(res["F"][0] - F_cf) <= 1e-5, (res["F"][0], F_cf)
    assert abs(res["norm"][0] - 1.0) <= 1e-4
    phys = np.zeros_like(sample)
    for qb in range(n):
        phys |= ((sample >> qb) & 1) << int(res["layout"][qb])
    st = q.trajectory_states(res, n, q.C64, T)
    amps = st[1].index_select(0, torch.as_tensor(phys, device=st.device)).cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(amps - amp_cf)) <= 2e-8
    del res, st
    torch.cuda.empty_cache()


def test_dm_qft17_fused_full_size_against_closed_form():
    torch.cuda.empty_cache()
    n, e = 17, 0.03
    x = 0x1B2D5
    c = qft(n, seed=1, x=x)
    N = 1 << n
    ex = np.zeros(N, np.complex128)
    ex[x] = 1.0
    psi = np.fft.fft(ex) / math.sqrt(N)
    ideal = q.StateVector(n, q.C64, 1)
    amps = ideal.amplitudes()
    amps.copy_(torch.as_tensor(psi[None, :].astype(np.complex64)).to(amps.device))
    torch.cuda.synchronize()
    print(f"[max size] dm qft{n} c64 fused (vec rho of 2^{2 * n} entries)", flush=True)
    res = q.dm_run(c.gates, n, x, q.C64, ideal, e=e)
    F = qft_expected_fidelity(n, x, e)
    assert abs(res["F"] - F) <= 1e-5, (res["F"], F)
    assert abs(res["trace"] - 1.0) <= 1e-5
    ideal.close()
    del res
    torch.cuda.empty_cache()
