"""Pins for the oracle's noise draws (Section 2, eq. (1): xi ~ N(0,1)).

* Philox4x32-10 words against rocRAND's independent implementation of the same generator.
* The series logarithm and the reduced cosine against libm.
* The Box-Muller deviate against the formula evaluated from the raw words, and its moments.
* Gauss-Hermite quadrature of the eq. (1) and eq. (2) noise reproduces the Kraus weights of
  eq. (6) and eq. (9): E[cos 2 e xi] = exp(-2 e^2), E[exp(-i e xi)] = exp(-e^2 / 2) = sqrt(P).
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "ref")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", "-o", exe,
                           os.path.join(HERE, "rocrand_philox_ref.hip")])
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(1234)
    M = 20000
    ctr = rng.integers(0, 2**32, size=(M, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:, 1] &= np.uint32((1 << 30) - 1)      # offset = 4 * (c1:c0) must fit 64 bits
    key = rng.integers(0, 2**32, size=(M, 2), dtype=np.uint64).astype(np.uint32)
    # structured corners: all-zero, all-ones-ish, small counters as used by the noise stream
    ctr[0] = 0; key[0] = 0
    ctr[1] = [0xFFFFFFFF, (1 << 30) - 1, 0xFFFFFFFF, 0xFFFFFFFF]; key[1] = [0xFFFFFFFF, 0xFFFFFFFF]
    for i in range(2, 200):
        ctr[i] = [i, i % 7, 0, 0]; key[i] = [i * 13, 0]
    text = "\n".join(" ".join(f"{int(v):x}" for v in (*c, *k)) for c, k in zip(ctr, key))
    out = subprocess.run([rocrand_ref], input=text, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(w, 16) for w in line.split()] for line in out.strip().splitlines()],
                   dtype=np.uint32)
    mine = oracle.philox(ctr, key)
    assert ref.shape == mine.shape
    assert np.array_equal(ref, mine)


def test_log_against_libm():
    rng = np.random.default_rng(5)
    xs = np.concatenate([
        (rng.integers(1, 2**53, size=20000).astype(np.float64) + 1.0) * 2.0**-53,
        np.array([2.0**-53, 2.0**-52, 0.5, 1.0 - 2.0**-53, 1.0, math.sqrt(0.5), math.sqrt(2.0) / 2 * 1.0000001]),
        np.exp(rng.uniform(-700, 700, size=2000)),
    ])
    for x in xs:
        got = oracle.log(float(x))
        ref = math.log(float(x))
        assert abs(got - ref) <= 4 * math.ulp(ref) + 1e-300, (x, got, ref)
    assert oracle.log(1.0) == 0.0


def test_cos2pi_against_libm():
    rng = np.random.default_rng(6)
    us = np.concatenate([rng.integers(0, 2**53, size=20000).astype(np.float64) * 2.0**-53,
                         np.array([0.0, 0.125, 0.25, 0.375, 0.5, 0.625, 0.75, 0.875, 1.0 - 2.0**-53])])
    # reference in x87 extended precision (64-bit significand): 2*pi*u without double rounding
    two_pi = np.longdouble("6.283185307179586476925286766559005768")
    for u in us:
        got = oracle.cos2pi(float(u))
        ref = float(np.cos(two_pi * np.longdouble(float(u))))
        assert abs(got - ref) <= 2.5e-16, (u, got, ref)
    assert oracle.cos2pi(0.0) == 1.0
    assert oracle.cos2pi(0.5) == -1.0


def test_normal_is_box_muller_of_the_words():
    seed = 0x1234_5678_9ABC_DEF0
    sites = np.arange(0, 300, dtype=np.uint32)
    trajs = np.array([0, 1, 7, 199, 65535], dtype=np.uint32)
    xi = oracle.normals(seed, sites, trajs, request=3, stream=0)
    for ti, t in enumerate(trajs):
        ctr = np.stack([sites, np.full_like(sites, t), np.zeros_like(sites), np.full_like(sites, 3)], 1)
        key = np.tile(np.array([seed & 0xFFFFFFFF, seed >> 32], np.uint32), (sites.size, 1))
        w = oracle.philox(ctr, key).astype(np.uint64)
        a = ((w[:, 0] << np.uint64(32)) | w[:, 1]) >> np.uint64(11)
        b = ((w[:, 2] << np.uint64(32)) | w[:, 3]) >> np.uint64(11)
        u1 = (a.astype(np.float64) + 1.0) * 2.0**-53
        u2 = b.astype(np.float64) * 2.0**-53
        ref = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
        np.testing.assert_allclose(xi[ti], ref, rtol=1e-14, atol=1e-14)


def test_normal_moments_and_distribution():
    from scipy import stats
    M = 400_000
    xi = oracle.normals(7, np.arange(M // 4, dtype=np.uint32), np.arange(4, dtype=np.uint32)).ravel()
    assert abs(xi.mean()) < 5.0 / math.sqrt(M)
    assert abs(xi.var() - 1.0) < 5.0 * math.sqrt(2.0 / M)
    k = stats.kurtosis(xi, fisher=False)
    assert abs(k - 3.0) < 5.0 * math.sqrt(24.0 / M)
    assert stats.kstest(xi, "norm").pvalue > 1e-4
    # distinct counters give distinct deviates; the same counter the same deviate
    again = oracle.normals(7, np.arange(16, dtype=np.uint32), np.arange(4, dtype=np.uint32))
    assert np.array_equal(again.ravel()[:16], oracle.normals(7, np.arange(16, dtype=np.uint32),
                                                             np.array([0], np.uint32)).ravel())


@pytest.mark.parametrize("e", [0.001, 0.005, 0.01, 0.02, 0.05, 0.3])
def test_noise_averages_by_quadrature(e):
    x, w = np.polynomial.hermite_e.hermegauss(80)
    w = w / math.sqrt(2.0 * math.pi)
    # eq. (6): lambda_1 = E[cos^2 e xi] = (1 + exp(-2 e^2)) / 2, lambda_2 = E[sin^2 e xi]
    l1 = float(np.sum(w * np.cos(e * x) ** 2))
    l2 = float(np.sum(w * np.sin(e * x) ** 2))
    assert abs(l1 - 0.5 * (1 + math.exp(-2 * e * e))) < 1e-15
    assert abs(l2 - 0.5 * (1 - math.exp(-2 * e * e))) < 1e-15
    assert abs(float(np.sum(w * np.sin(e * x) * np.cos(e * x)))) < 1e-15
    # eq. (9): E[exp(-i e xi)] = exp(-e^2/2) = sqrt(P), P = exp(-e^2)
    m = complex(np.sum(w * np.exp(-1j * e * x)))
    assert abs(m - math.sqrt(math.exp(-e * e))) < 1e-15


def test_kraus_sets_are_trace_preserving():
    rng = np.random.default_rng(0)
    from workloads import haar_2x2
    for e in [0.0, 0.01, 0.3, 1.0]:
        for _ in range(5):
            K = oracle.kraus_rot(haar_2x2(rng), e)
            np.testing.assert_allclose(sum(k.conj().T @ k for k in K), np.eye(2), atol=1e-15)
            K = oracle.kraus_phase(float(rng.uniform(0, 2 * math.pi)), e)
            np.testing.assert_allclose(sum(k.conj().T @ k for k in K), np.eye(4), atol=1e-15)


def _superop(K):
    return sum(np.kron(k, k.conj()) for k in K)


def test_improved_cp_kraus_is_the_orthogonal_form_of_eq9():
    """Eq. (14): the eq. (9) operators mixed by the unitary of eq. (13).  Same channel (equal
    superoperators), complete, and Hilbert-Schmidt orthogonal with squared norms equal to the
    squared singular values of the matrix of eq. (12) (its rows are the diagonals of the eq. (9)
    operators), taken from numpy's SVD; those are the lambda_1,2 = 2 +- sqrt(1 + 3P) of the
    text."""
    rng = np.random.default_rng(4)
    for e in [0.0, 0.01, 0.1, 0.3, 1.0, 2.0]:
        P = math.exp(-e * e)
        for theta in [0.0, math.pi, float(rng.uniform(0, 2 * math.pi))]:
            K9 = oracle.kraus_phase(theta, e)
            K14 = oracle.kraus_phase_improved(theta, e)
            np.testing.assert_allclose(sum(k.conj().T @ k for k in K14), np.eye(4), atol=1e-14)
            np.testing.assert_allclose(_superop(K14), _superop(K9), atol=1e-14)
        K14 = oracle.kraus_phase_improved(0.0, e)
        gram = np.array([[np.trace(a.conj().T @ b) for b in K14] for a in K14])
        psi12 = np.array([[1, 1, 1, math.sqrt(P)], [0, 0, 0, math.sqrt(1 - P)]])
        sv2 = np.linalg.svd(psi12, compute_uv=False) ** 2
        np.testing.assert_allclose(gram, np.diag(sv2), atol=1e-13)
        np.testing.assert_allclose(sv2, [2 + math.sqrt(1 + 3 * P), 2 - math.sqrt(1 + 3 * P)], atol=1e-13)


def test_library_improved_cp_kraus_matches_the_oracle():
    """The operators the library builds behind the C ABI (qs_kraus_cp, host-only) equal the
    oracle's eq. (9) and eq. (14) sets."""
    import paper_1412_2293_amd as q
    rng = np.random.default_rng(9)
    for e in [0.0, 0.02, 0.2, 1.5]:
        for theta in [0.0, 1.0, float(rng.uniform(0, 2 * math.pi))]:
            np.testing.assert_allclose(q.cp_kraus_improved(theta, e), oracle.kraus_phase_improved(theta, e),
                                       atol=1e-15)
            np.testing.assert_allclose(q.cp_kraus(theta, e), oracle.kraus_phase(theta, e), atol=1e-15)


def test_library_cp_kraus_rejects_bad_arguments():
    import paper_1412_2293_amd as q
    for args in [(math.nan, 0.1, 0), (0.0, -0.1, 0), (0.0, math.inf, 1), (0.0, 0.1, 2)]:
        with pytest.raises(q.QsimError):
            q.kraus_cp(args[0], args[1], args[2])
