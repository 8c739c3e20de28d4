"""The allocation-free fidelity entry point against qs_fidelity, through the C ABI.

qs_fidelity_noalloc runs the same reductions in the same order as qs_fidelity with its partial
sums in the library's fixed device array, so the overlap and both norms agree bit for bit.  Two
calls in a row (the second on a smaller state) check that the shared array keeps no state that
changes a later result.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_1412_2293_amd as q  # noqa: E402

pytestmark = pytest.mark.gpu


def _random_state(sv: "q.StateVector", seed: int):
    rng = np.random.default_rng(seed)
    N = 1 << sv.n
    z = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    z /= np.linalg.norm(z)
    amps = sv.amplitudes()
    amps.copy_(torch.as_tensor(z.astype(np.complex64 if sv.dtype == q.C64 else np.complex128)[None, :]).to(amps.device))


@pytest.mark.parametrize("dtype", [q.C128, q.C64], ids=["c128", "c64"])
def test_fidelity_noalloc_equals_fidelity(dtype):
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    for k, n in enumerate((21, 12)):          # the second call on a smaller state
        print(f"noalloc dtype={dtype} n={n}", flush=True)
        a, b = q.StateVector(n, dtype, 1), q.StateVector(n, dtype, 1)
        _random_state(a, 10 + k)
        _random_state(b, 20 + k)
        torch.cuda.synchronize()
        f_ref, ov_ref = q.fidelity(a, 0, b, 0)
        out.fill_(float("nan"))
        q.fidelity_noalloc(a.buf, b.buf, n, dtype, out)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        assert o[0] == ov_ref.real and o[1] == ov_ref.imag
        f = (o[0] * o[0] + o[1] * o[1]) / (o[2] * o[3])
        assert f == f_ref
        assert abs(o[2] - 1.0) <= (1e-12 if dtype == q.C128 else 1e-5)
        assert abs(o[3] - 1.0) <= (1e-12 if dtype == q.C128 else 1e-5)


def test_fidelity_noalloc_rejects_bad_arguments():
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    a = q.StateVector(4, q.C64, 1)
    for n, dt in [(0, q.C64), (35, q.C64), (4, 7)]:
        with pytest.raises(q.QsimError):
            q.fidelity_noalloc(a.buf, a.buf, n, dt, out)
    with pytest.raises(q.QsimError):
        q.fidelity_noalloc(None, a.buf, 4, q.C64, out)
