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
  * DIAG  multiply every amplitude whose index i satisfies (i & mask) == value by the
          complex factor m[0] (noiseless; a phase on any set of controls);
  * noise tag ROT   : the gate becomes U * V(e*xi) with V of eq. (1);
    noise tag PHASE : theta -> theta + e*xi on the |11> element (Section 2, after eq. (2)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

U1, CP, SWAP, CNOT, U2, FLIP, DIAG = 0, 1, 2, 3, 4, 5, 6
KIND_NAMES = {U1: "U1", CP: "CP", SWAP: "SWAP", CNOT: "CNOT", U2: "U2", FLIP: "FLIP", DIAG: "DIAG"}
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
    mask: int = 0                       # FLIP, DIAG
    value: int = 0                      # FLIP, DIAG


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
            elif g.kind in (FLIP, DIAG):
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


# ------------------------------------------------------------------------------------------
# Choi-Jamiolkowski relative states (Section 4): a register of qubits, the qubits whose input is
# entangled with a reference (eq. 16), the noisy steps (gates and Kraus channels), the ideal
# gates that define the target, and the ancillas that are traced out at the end.
# ------------------------------------------------------------------------------------------
@dataclass
class Channel:
    """A Kraus channel {E_k} on one or two qubits (sum_k E_k^dagger E_k = I); 4x4 operators use
    the local index bit(qubits[0]) + 2 * bit(qubits[1])."""
    qubits: tuple
    ops: np.ndarray


@dataclass
class ChoiProgram:
    n: int                      # register qubits (references are added after them)
    logical: List[int]          # register qubits entangled with reference n + k (eq. 16)
    steps: list                 # Gate or Channel, applied to the register (eq. 17)
    ideal: List[Gate]           # gates that map the entangled input to the target
    ancillas: List[int] = field(default_factory=list)   # traced out in the fidelity
    name: str = ""
    meta: dict = field(default_factory=dict)

    def total_qubits(self) -> int:
        return self.n + len(self.logical)


def amplitude_damping(t: float, T1: float) -> np.ndarray:
    """Amplitude relaxation over time t (textbook channel): gamma = 1 - exp(-t / T1)."""
    g = 1.0 - math.exp(-t / T1)
    return np.array([[[1, 0], [0, math.sqrt(1 - g)]], [[0, math.sqrt(g)], [0, 0]]], np.complex128)


def dephasing(p: float) -> np.ndarray:
    """Phase error with probability p: {sqrt(1 - p) I, sqrt(p) Z}."""
    return np.array([[[math.sqrt(1 - p), 0], [0, math.sqrt(1 - p)]],
                     [[math.sqrt(p), 0], [0, -math.sqrt(p)]]], np.complex128)


def dephasing_from_T2(t: float, T2: float) -> np.ndarray:
    """Phase relaxation over time t with the probability of eq. (19): T2 = -t / ln(1 - 2p)."""
    return dephasing(0.5 * (1.0 - math.exp(-t / T2)))


def _u1(q: int, m) -> Gate:
    return Gate(U1, q0=q, m=np.asarray(m, np.complex128))


_T = np.diag([1.0, np.exp(1j * math.pi / 4)])
_TDG = np.diag([1.0, np.exp(-1j * math.pi / 4)])


def toffoli_gates(c1: int, c2: int, t: int) -> List[Gate]:
    """Toffoli (controls c1, c2, target t) as Hadamards, T / T^dagger and six CNOTs (the standard
    exact decomposition)."""
    return [_u1(t, H_MATRIX), Gate(CNOT, q0=c2, q1=t), _u1(t, _TDG), Gate(CNOT, q0=c1, q1=t), _u1(t, _T),
            Gate(CNOT, q0=c2, q1=t), _u1(t, _TDG), Gate(CNOT, q0=c1, q1=t), _u1(c2, _T), _u1(t, _T),
            _u1(t, H_MATRIX), Gate(CNOT, q0=c1, q1=c2), _u1(c1, _T), _u1(c2, _TDG), Gate(CNOT, q0=c1, q1=c2)]


def relaxation_channels(qubits, T1: float, T2: float, t: float = 1.0) -> List[Channel]:
    """Amplitude then phase relaxation over time t on each of `qubits` (T1 or T2 = inf: none)."""
    out: List[Channel] = []
    for q in qubits:
        out.append(Channel((q,), amplitude_damping(t, T1)))
        out.append(Channel((q,), dephasing_from_T2(t, T2)))
    return out


def _phase_code(noise: list, name: str, meta: dict) -> ChoiProgram:
    enc = [Gate(CNOT, q0=0, q1=1), Gate(CNOT, q0=0, q1=2)] + [_u1(q, H_MATRIX) for q in range(3)]
    dec = [_u1(q, H_MATRIX) for q in range(3)] + [Gate(CNOT, q0=0, q1=1), Gate(CNOT, q0=0, q1=2)]
    dec += toffoli_gates(1, 2, 0)
    return ChoiProgram(3, [0], enc + noise + dec, [], ancillas=[1, 2], name=name, meta=meta)


def phase_code(p: float) -> ChoiProgram:
    """Three-qubit phase-error code (Section 4.1) on the logical qubit 0: encode (CNOTs then
    Hadamards), a phase error with probability p on each code qubit, decode (Hadamards, CNOTs,
    and the majority correction as a Toffoli controlled by the syndrome qubits 1 and 2).  The
    target is the identity on the logical qubit; the syndrome qubits are traced out."""
    return _phase_code([Channel((q,), dephasing(p)) for q in range(3)], f"phase_code p={p}", {"p": p})


def phase_code_relaxation(T1: float, T2: float, t: float = 1.0) -> ChoiProgram:
    """The three-qubit phase-error code with amplitude and phase relaxation (T1, T2 over a time t,
    eq. 19 for the phase part) on each code qubit in place of the phase errors."""
    return _phase_code(relaxation_channels(range(3), T1, T2, t), f"phase_code T1={T1} T2={T2}",
                       {"T1": T1, "T2": T2, "t": t})


def qft_relaxation(n: int, T1: float, T2: float, t: float = 1.0) -> ChoiProgram:
    """QFT on n qubits (Section 4.3; the noiseless gates of ``qft``) with amplitude and phase
    relaxation on every qubit after every gate, each gate lasting t."""
    gates = [Gate(g.kind, q0=g.q0, q1=g.q1, m=g.m, theta=g.theta) for g in qft(n, 0, noisy_h=False).gates]
    steps = []
    for g in gates:
        steps.append(g)
        for q in range(n):
            steps.append(Channel((q,), amplitude_damping(t, T1)))
            steps.append(Channel((q,), dephasing_from_T2(t, T2)))
    return ChoiProgram(n, list(range(n)), steps, gates, name=f"qft{n} T1={T1} T2={T2}",
                       meta={"T1": T1, "T2": T2, "t": t})


def choi_preparation(prog: ChoiProgram) -> List[Gate]:
    """Gates that make the maximally entangled input of eq. (16) from |0...0>: a Hadamard on
    each logical qubit and a CNOT onto its reference qubit n + k."""
    out: List[Gate] = []
    for k, l in enumerate(prog.logical):
        out.append(_u1(l, H_MATRIX))
        out.append(Gate(CNOT, q0=l, q1=prog.n + k))
    return out


def ancilla_indices(prog: ChoiProgram) -> List[int]:
    """Basis indices of every assignment of the traced-out ancillas (all other qubits 0)."""
    out = []
    for a in range(1 << len(prog.ancillas)):
        idx = 0
        for b, q in enumerate(prog.ancillas):
            if (a >> b) & 1:
                idx |= 1 << q
        out.append(idx)
    return out


def shor_code(p: float) -> ChoiProgram:
    """Shor's nine-qubit code (Section 4.2) on the logical qubit 0 with a phase error of
    probability p on every code qubit.  Encode: CNOTs 0 -> 3, 6, Hadamards on 0, 3, 6, then
    CNOTs b -> b+1, b+2 in each block b = 0, 3, 6.  Decode: in each block the CNOTs again and a
    Toffoli controlled by b+1, b+2 onto b (bit correction), then Hadamards on 0, 3, 6, CNOTs
    0 -> 3, 6 and a Toffoli controlled by 3, 6 onto 0 (phase correction).  The target is the
    identity on the logical qubit; the other eight qubits are traced out."""
    return _shor_code([Channel((q,), dephasing(p)) for q in range(9)], f"shor_code p={p}", {"p": p})


def shor_code_relaxation(T1: float, T2: float, t: float = 1.0) -> ChoiProgram:
    """Shor's nine-qubit code with amplitude and phase relaxation (T1, T2 over a time t) on each
    code qubit in place of the phase errors."""
    return _shor_code(relaxation_channels(range(9), T1, T2, t), f"shor_code T1={T1} T2={T2}",
                      {"T1": T1, "T2": T2, "t": t})


def _shor_code(noise: list, name: str, meta: dict) -> ChoiProgram:
    enc = [Gate(CNOT, q0=0, q1=3), Gate(CNOT, q0=0, q1=6)] + [_u1(b, H_MATRIX) for b in (0, 3, 6)]
    for b in (0, 3, 6):
        enc += [Gate(CNOT, q0=b, q1=b + 1), Gate(CNOT, q0=b, q1=b + 2)]
    dec = []
    for b in (0, 3, 6):
        dec += [Gate(CNOT, q0=b, q1=b + 1), Gate(CNOT, q0=b, q1=b + 2)] + toffoli_gates(b + 1, b + 2, b)
    dec += [_u1(b, H_MATRIX) for b in (0, 3, 6)] + [Gate(CNOT, q0=0, q1=3), Gate(CNOT, q0=0, q1=6)]
    dec += toffoli_gates(3, 6, 0)
    return ChoiProgram(9, [0], enc + noise + dec, [], ancillas=list(range(1, 9)), name=name, meta=meta)


def chain_heavy_circuit(n: int, n_gates: int, seed: int):
    """Mostly complex one-qubit gates, so that long phase chains form, with every gate that a
    chain crosses (controlled phases, sign flips, SWAPs, CNOT controls) or that ends one (real
    gates, CNOT targets, dense two-qubit gates) in between, some of the one-qubit gates
    noiseless and diagonal (T-like)."""
    rng = np.random.default_rng(seed)
    N = 1 << n
    hm = np.array([[1, 1], [1, -1]], np.complex128) / math.sqrt(2.0)
    gates = []
    for _ in range(n_gates):
        k = int(rng.integers(0, 20))
        qa = int(rng.integers(0, n))
        if k < 11:
            gates.append(Gate(U1, q0=qa, m=haar_2x2(rng), noise=NOISE_ROT))
        elif k == 11:
            ph = np.exp(1j * rng.uniform(0, 2 * math.pi))
            gates.append(Gate(U1, q0=qa, m=np.diag([1.0, ph]).astype(np.complex128), noise=NOISE_NONE))
        elif k == 12:
            gates.append(Gate(U1, q0=qa, m=hm, noise=NOISE_ROT))
        elif k in (13, 14):
            a, b = (int(v) for v in rng.choice(n, size=2, replace=False))
            gates.append(Gate(CP, q0=a, q1=b, theta=float(rng.uniform(0, 2 * math.pi)), noise=NOISE_PHASE))
        elif k == 15:
            a, b = (int(v) for v in rng.choice(n, size=2, replace=False))
            gates.append(Gate(SWAP, q0=a, q1=b))
        elif k == 16:
            a, b = (int(v) for v in rng.choice(n, size=2, replace=False))
            gates.append(Gate(CNOT, q0=a, q1=b))
        elif k == 17:
            a, b = (int(v) for v in rng.choice(n, size=2, replace=False))
            gates.append(Gate(U2, q0=a, q1=b, m=random_unitary(4, rng)))
        else:
            mask = int(rng.integers(0, N)) | (1 << qa)
            gates.append(Gate(FLIP, mask=mask, value=int(rng.integers(0, N)) & mask))
    return Circuit(n, _renumber_sites(gates), name=f"chains{n}", init_index=int(rng.integers(0, N)))

