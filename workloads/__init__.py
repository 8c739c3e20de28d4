"""Seeded synthetic circuits: the shared input to both the HIP path and the CPU oracle.

This module only *describes* circuits (which gate acts on which qubits, with which ideal
matrix or angle, and which gates are noisy).  It holds none of the simulation arithmetic:
no amplitude update, no noise draw, no fidelity.  The noise samples xi are drawn by each
side from its own Philox4x32-10 implementation, keyed by the per-gate ``site`` id below.

Conventions (shared vocabulary of the circuit description):
  * qubit q is bit q of the amplitude index (qubit 0 = least significant bit);
  * U1    dense one-qubit gate, 2x2 complex matrix ``m`` (row-major), target ``q0``;
  * CP    controlled phase of eq. (2): the |11> amplitude of (q0, q1) gets exp(-i*theta);
          CZ is CP with theta = pi;
  * SWAP  exchange of qubits q0 and q1;
  * CNOT  control q0, target q1;
  * U2    dense two-qubit gate, 4x4 complex matrix, local index bit(q0) + 2*bit(q1);
  * FLIP  negate every amplitude whose index i satisfies (i & mask) == value
          (the Grover oracle and the reflection about |0>, both noiseless);
  * noise tag ROT   : the gate becomes U * V(e*xi) with V of eq. (1);
    noise tag PHASE : theta -> theta + e*xi on the |11> element (Section 2, after eq. (2)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

U1, CP, SWAP, CNOT, U2, FLIP = 0, 1, 2, 3, 4, 5
KIND_NAMES = {U1: "U1", CP: "CP", SWAP: "SWAP", CNOT: "CNOT", U2: "U2", FLIP: "FLIP"}
NOISE_NONE, NOISE_ROT, NOISE_PHASE = 0, 1, 2

H_MATRIX = np.array([[1.0, 1.0], [1.0, -1.0]], dtype=np.complex128) / math.sqrt(2.0)


@dataclass
class Gate:
    kind: int
    q0: int = 0
    q1: int = 0
    m: Optional[np.ndarray] = None      # 2x2 (U1) or 4x4 (U2) complex128
    theta: float = 0.0                  # CP angle
    noise: int = NOISE_NONE
    site: int = 0                       # Philox counter word 0 for this gate's noise draw
    mask: int = 0                       # FLIP
    value: int = 0                      # FLIP


@dataclass
class Circuit:
    n: int
    gates: List[Gate]
    name: str = ""
    init_index: int = 0                 # the circuit acts on the basis state |init_index>
    marked: Optional[int] = None        # Grover marked index (success probability p = |psi_w|^2)
    meta: dict = field(default_factory=dict)

    def __len__(self):
        return len(self.gates)

    def count(self, kind: int) -> int:
        return sum(1 for g in self.gates if g.kind == kind)

    def amplitude_updates(self) -> int:
        """Amplitudes rewritten by one pass of the circuit over one state vector.

        Dense one-qubit and dense two-qubit gates rewrite N amplitudes, a controlled phase
        N/4, a SWAP or CNOT N/2, and a FLIP the amplitudes it selects.
        """
        N = 1 << self.n
        tot = 0
        for g in self.gates:
            if g.kind in (U1, U2):
                tot += N
            elif g.kind == CP:
                tot += N // 4
            elif g.kind in (SWAP, CNOT):
                tot += N // 2
            elif g.kind == FLIP:
                tot += N >> bin(g.mask).count("1")
        return tot


def _renumber_sites(gates: List[Gate]) -> List[Gate]:
    for i, g in enumerate(gates):
        g.site = i
    return gates


def grover_iterations(n: int) -> int:
    """floor(pi/4 * sqrt(2^n)) Grover iterations."""
    return int(math.floor(math.pi / 4.0 * math.sqrt(2.0 ** n)))


def grover(n: int, seed: int, iterations: Optional[int] = None, marked: Optional[int] = None) -> Circuit:
    """Grover search on n qubits.

    Preparation H^n, then per iteration: oracle O_w (sign flip of |w>), H^n, reflection R_0
    (sign flip of |0>), H^n.  Every Hadamard is tagged for the eq. (1) rotation noise, so the
    number of noisy Hadamards is n + 2*n*j, the count in the exponent of eq. (10).  The two
    reflections are exact one-amplitude sign flips; H R_0 H equals minus the Grover diffusion,
    so each iteration carries a global phase of -1.
    """
    rng = np.random.default_rng(seed)
    N = 1 << n
    w = int(rng.integers(0, N)) if marked is None else int(marked)
    j = grover_iterations(n) if iterations is None else int(iterations)
    gates: List[Gate] = []
    full = N - 1

    def hlayer():
        for q in range(n):
            gates.append(Gate(U1, q0=q, m=H_MATRIX.copy(), noise=NOISE_ROT))

    hlayer()
    for _ in range(j):
        gates.append(Gate(FLIP, mask=full, value=w))
        hlayer()
        gates.append(Gate(FLIP, mask=full, value=0))
        hlayer()
    return Circuit(n, _renumber_sites(gates), name=f"grover{n}", init_index=0, marked=w,
                   meta={"iterations": j, "seed": seed})


def qft(n: int, seed: int, x: Optional[int] = None, swaps: bool = True, noisy_h: bool = True) -> Circuit:
    """Quantum Fourier transform on the basis input |x>, built from H and controlled phases.

    Most-significant qubit first: for t = n-1 .. 0, H on t, then CP(c, t) with
    theta = 2*pi / 2^(t-c+1) for c = t-1 .. 0; finally SWAP(q, n-1-q).  With the exp(-i*theta)
    phase of eq. (2) the output is N^(-1/2) sum_y exp(-2*pi*i*x*y/N) |y>.
    Controlled phases carry the phase noise; Hadamards carry the eq. (1) rotation noise unless
    ``noisy_h`` is False.
    """
    rng = np.random.default_rng(seed)
    N = 1 << n
    x = int(rng.integers(0, N)) if x is None else int(x)
    gates: List[Gate] = []
    for t in range(n - 1, -1, -1):
        gates.append(Gate(U1, q0=t, m=H_MATRIX.copy(), noise=NOISE_ROT if noisy_h else NOISE_NONE))
        for c in range(t - 1, -1, -1):
            gates.append(Gate(CP, q0=c, q1=t, theta=2.0 * math.pi / float(1 << (t - c + 1)),
                              noise=NOISE_PHASE))
    if swaps:
        for q in range(n // 2):
            gates.append(Gate(SWAP, q0=q, q1=n - 1 - q))
    return Circuit(n, _renumber_sites(gates), name=f"qft{n}", init_index=x,
                   meta={"x": x, "seed": seed})


def haar_2x2(rng: np.random.Generator) -> np.ndarray:
    """Haar-random 2x2 unitary: QR of a complex Ginibre matrix with the phases of R's diagonal
    moved into Q (Mezzadri, Notices AMS 2007)."""
    z = (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    ph = d / np.abs(d)
    return (q * ph[None, :]).astype(np.complex128)


def random_layers(n: int, depth: int, seed: int, pairing: str = "brickwork") -> Circuit:
    """Random circuit: each layer is a Haar one-qubit gate on every qubit (rotation noise),
    then CZ gates (phase noise) on disjoint pairs.

    ``pairing="brickwork"``: pairs (2i, 2i+1) on even layers, (2i+1, 2i+2) on odd layers.
    ``pairing="random"``: floor(n/2) disjoint pairs from a fresh shuffle each layer.
    """
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    for layer in range(depth):
        for q in range(n):
            gates.append(Gate(U1, q0=q, m=haar_2x2(rng), noise=NOISE_ROT))
        if pairing == "brickwork":
            start = layer % 2
            pairs = [(a, a + 1) for a in range(start, n - 1, 2)]
        else:
            perm = rng.permutation(n)
            pairs = [(int(min(perm[2 * i], perm[2 * i + 1])), int(max(perm[2 * i], perm[2 * i + 1])))
                     for i in range(n // 2)]
        for a, b in pairs:
            gates.append(Gate(CP, q0=a, q1=b, theta=math.pi, noise=NOISE_PHASE))
    return Circuit(n, _renumber_sites(gates), name=f"random{n}x{depth}", init_index=0,
                   meta={"depth": depth, "seed": seed, "pairing": pairing})


def random_unitary(dim: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random dim x dim unitary (same QR construction as haar_2x2)."""
    z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return (q * (d / np.abs(d))[None, :]).astype(np.complex128)


def random_mixed_circuit(n: int, n_gates: int, seed: int) -> Circuit:
    """A seeded mix of every gate kind on random qubits (for gate-level parity tests)."""
    rng = np.random.default_rng(seed)
    N = 1 << n
    gates: List[Gate] = []
    kinds = [U1, U1, U1, CP, CP, SWAP, CNOT, U2, FLIP] if n >= 2 else [U1, FLIP]
    for _ in range(n_gates):
        k = kinds[int(rng.integers(0, len(kinds)))]
        if k == U1:
            gates.append(Gate(U1, q0=int(rng.integers(0, n)), m=haar_2x2(rng),
                              noise=NOISE_ROT if rng.random() < 0.7 else NOISE_NONE))
        elif k == FLIP:
            mask = int(rng.integers(0, N)) | (1 << int(rng.integers(0, n)))
            gates.append(Gate(FLIP, mask=mask, value=int(rng.integers(0, N)) & mask))
        else:
            a, b = (int(v) for v in rng.choice(n, size=2, replace=False))
            if k == CP:
                gates.append(Gate(CP, q0=a, q1=b, theta=float(rng.uniform(0, 2 * math.pi)),
                                  noise=NOISE_PHASE if rng.random() < 0.7 else NOISE_NONE))
            elif k == U2:
                gates.append(Gate(U2, q0=a, q1=b, m=random_unitary(4, rng)))
            else:
                gates.append(Gate(k, q0=a, q1=b))
    return Circuit(n, _renumber_sites(gates), name=f"mixed{n}x{n_gates}",
                   init_index=int(rng.integers(0, N)), meta={"seed": seed})


# ------------------------------------------------------------------------------------------
SERVING_KINDS = ("grover", "qft", "random")


@dataclass
class Request:
    """One request of a serving stream: which circuit, how many trajectories, which noise."""
    index: int
    arrival: float            # arrival time in units of the mean inter-arrival gap
    kind: str
    n: int
    T: int
    e: float
    seed: int

    def circuit(self) -> Circuit:
        if self.kind == "grover":
            # iterations capped at 10 n, the budget of the random-layer circuits (~20 n^2 gates)
            return grover(self.n, self.seed, iterations=min(grover_iterations(self.n), 10 * self.n))
        if self.kind == "qft":
            return qft(self.n, self.seed)
        return random_layers(self.n, 20 * self.n, self.seed, pairing="random")


def serving_stream(n_requests: int = 2000, seed: int = 3, n_min: int = 12, n_max: int = 28,
                   t_min: int = 16, t_max: int = 256, e_min: float = 0.001, e_max: float = 0.05) -> List[Request]:
    """Seeded request stream: Poisson arrivals (exponential gaps of mean 1; the caller scales
    them to a rate), qubit count uniform in [n_min, n_max], circuit kind uniform over Grover,
    QFT and random layers of depth 20 n, trajectories uniform in [t_min, t_max], noise strength
    uniform in [e_min, e_max].  Request i uses circuit seed seed * 100003 + i and Philox request
    word i."""
    rng = np.random.default_rng([seed, 2])
    gaps = rng.exponential(1.0, n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    ns = rng.integers(n_min, n_max + 1, n_requests)
    kinds = rng.integers(0, len(SERVING_KINDS), n_requests)
    Ts = rng.integers(t_min, t_max + 1, n_requests)
    es = rng.uniform(e_min, e_max, n_requests)
    return [Request(i, float(arrivals[i]), SERVING_KINDS[int(kinds[i])], int(ns[i]), int(Ts[i]), float(es[i]),
                    seed * 100003 + i) for i in range(n_requests)]
