"""Closed forms used as pins, derived independently of the oracle's loops.

* Grover at e = 0 (textbook): with theta0 = asin(N^-1/2), after j iterations the marked
  amplitude is sin((2j+1) theta0) and every other cos((2j+1) theta0)/sqrt(N-1), up to the
  global phase (-1)^j that H R_0 H = -(2|s><s| - I) contributes per iteration.
* QFT at e = 0 on |x>: N^-1/2 exp(-2 pi i x y / N), i.e. numpy.fft.fft(e_x) / sqrt(N).
* Noisy QFT on a basis input (controls of target t are qubits c < t, still basis states when
  their controlled phases act, so the state stays a product state): qubit t ends in
  D(Phi_t) H V(e xi_t) |x_t>, D(Phi) = diag(1, exp(-i Phi)),
  Phi_t = sum_{c<t, x_c=1} (theta_{c,t} + e xi_{c,t}); the per-trajectory fidelity is
  prod_t (1 + cos(2 e xi_t) cos(phi_t)) / 2 with phi_t = e sum_{c<t, x_c=1} xi_{c,t}, and
  its expectation prod_t (1 + exp(-2e^2) exp(-e^2 m_t / 2)) / 2, m_t = #{c < t: x_c = 1}.
* Eq. (10) (Section 3.3): p_noise(j) = lambda_1^(n + 2 n j) p_ideal(j).
* Eq. (11) and eq. (15) (Section 3.3): QFT lower bounds.
"""
import math

import numpy as np


def lambdas(e):
    return 0.5 * (1.0 + math.exp(-2 * e * e)), 0.5 * (1.0 - math.exp(-2 * e * e))


def grover_ideal(n, w, j):
    N = 1 << n
    th = math.asin(N ** -0.5)
    psi = np.full(N, math.cos((2 * j + 1) * th) / math.sqrt(N - 1), np.complex128)
    psi[w] = math.sin((2 * j + 1) * th)
    return psi * (-1) ** j


def grover_p_ideal(n, j):
    return math.sin((2 * j + 1) * math.asin(2.0 ** (-n / 2))) ** 2


def qft_ideal(n, x):
    N = 1 << n
    ex = np.zeros(N, np.complex128)
    ex[x] = 1.0
    return np.fft.fft(ex) / math.sqrt(N)


def qft_noisy_qubits(circuit, xi_by_site, e):
    """(F, per-qubit final states) of one noisy QFT trajectory; xi_by_site: site -> xi."""
    n, x = circuit.n, circuit.init_index
    h_site, cp_site = {}, {}
    for g in circuit.gates:
        if g.kind == 0:
            h_site[g.q0] = g.site
        elif g.kind == 1:
            cp_site[(g.q0, g.q1)] = g.site
    H = np.array([[1, 1], [1, -1]], np.complex128) / math.sqrt(2)
    F = 1.0
    qubit_states = {}
    for t in range(n):
        xt = (x >> t) & 1
        a = e * xi_by_site[h_site[t]]
        V = np.array([[math.cos(a), math.sin(a)], [-math.sin(a), math.cos(a)]])
        Phi, phi = 0.0, 0.0
        for c in range(t):
            if (x >> c) & 1:
                dx = e * xi_by_site[cp_site[(c, t)]]
                Phi += 2 * math.pi / (1 << (t - c + 1)) + dx
                phi += dx
        F *= 0.5 * (1.0 + math.cos(2 * a) * math.cos(phi))
        qubit_states[t] = np.diag([1.0, np.exp(-1j * Phi)]) @ H @ V[:, xt]
    return F, qubit_states


def qft_noisy_closed_form(circuit, xi_by_site, e):
    """(F, psi) of one noisy QFT trajectory (full state; small n only)."""
    n = circuit.n
    F, qs_ = qft_noisy_qubits(circuit, xi_by_site, e)
    # the final SWAP layer puts qubit t at output bit n-1-t; kron: most significant first
    psi = np.array([1.0 + 0j])
    for b in range(n - 1, -1, -1):
        psi = np.kron(psi, qs_[n - 1 - b])
    return F, psi


def qft_noisy_amplitudes(circuit, xi_by_site, e, indices):
    """(F, amplitudes at the given output indices) of one noisy QFT trajectory."""
    n = circuit.n
    F, qs_ = qft_noisy_qubits(circuit, xi_by_site, e)
    idx = np.asarray(indices, np.int64)
    amp = np.ones(idx.size, np.complex128)
    for b in range(n):
        st = qs_[n - 1 - b]
        amp *= np.where((idx >> b) & 1, st[1], st[0])
    return F, amp


def qft_expected_fidelity(n, x, e):
    F = 1.0
    for t in range(n):
        m = bin(x & ((1 << t) - 1)).count("1")
        F *= 0.5 * (1.0 + math.exp(-2 * e * e) * math.exp(-e * e * m / 2))
    return F


def eq10(n, j, e):
    return lambdas(e)[0] ** (n + 2 * n * j) * grover_p_ideal(n, j)


def eq11(n, e):
    PH = 0.5 * (1 + math.exp(-2 * e * e))
    PR = math.exp(-e * e)
    return PH ** n * PR ** (n * (n - 1) / 8)


def eq15(n, e):
    PH = 0.5 * (1 + math.exp(-2 * e * e))
    P = math.exp(-e * e)
    f = (math.sqrt(1 + 3 * P) - P - 1) / math.sqrt(P * (1 - P))
    PRt = (math.sqrt(P) + f * math.sqrt(1 - P)) ** 2 / (1 + f * f) ** 4
    return PH ** n * PRt ** (n * (n - 1) / 8)


def full_gate_matrix(n, g):
    """The gate as a 2^n x 2^n matrix by Kronecker products (qubit 0 = rightmost factor)."""
    N = 1 << n
    if g.kind == 0:
        ops = [np.eye(2)] * n
        ops = list(ops)
        ops[g.q0] = g.m
        M = np.array([[1.0 + 0j]])
        for q in range(n - 1, -1, -1):
            M = np.kron(M, ops[q])
        return M
    # generic: build column by column from the basis action
    M = np.zeros((N, N), np.complex128)
    for col in range(N):
        if g.kind == 1:
            ph = np.exp(-1j * g.theta) if ((col >> g.q0) & 1) and ((col >> g.q1) & 1) else 1.0
            M[col, col] = ph
        elif g.kind == 2:
            a, b = (col >> g.q0) & 1, (col >> g.q1) & 1
            row = col & ~((1 << g.q0) | (1 << g.q1)) | (b << g.q0) | (a << g.q1)
            M[row, col] = 1.0
        elif g.kind == 3:
            row = col ^ (1 << g.q1) if (col >> g.q0) & 1 else col
            M[row, col] = 1.0
        elif g.kind == 4:
            loc = ((col >> g.q0) & 1) + 2 * ((col >> g.q1) & 1)
            base = col & ~((1 << g.q0) | (1 << g.q1))
            for r in range(4):
                row = base | ((r & 1) << g.q0) | (((r >> 1) & 1) << g.q1)
                M[row, col] += g.m[r, loc]
        elif g.kind == 5:
            M[col, col] = -1.0 if (col & g.mask) == g.value else 1.0
    return M


def first_layer_pairs(circuit, xi_by_site, e):
    """Per-pair two-qubit states of one trajectory of a circuit made of one dense one-qubit
    gate per qubit (rotation noise, eq. 1: U V(e xi) with V = [[c, s], [-s, c]]) followed by
    controlled phases on disjoint pairs covering every qubit (phase noise: theta + e xi), from
    |0...0>.  Returns {(a, b): 4-vector over (bit a) + 2 (bit b)}."""
    col = {}
    for g in circuit.gates:
        if g.kind == 0:
            a = e * xi_by_site.get(g.site, 0.0) if g.noise == 1 else 0.0
            V = np.array([[math.cos(a), math.sin(a)], [-math.sin(a), math.cos(a)]])
            col[g.q0] = (np.asarray(g.m) @ V)[:, 0]
    pairs = {}
    for g in circuit.gates:
        if g.kind == 1:
            th = g.theta + (e * xi_by_site.get(g.site, 0.0) if g.noise == 2 else 0.0)
            v = np.kron(col[g.q1], col[g.q0]).astype(np.complex128)   # index bit(q0) + 2 bit(q1)
            v[3] *= np.exp(-1j * th)
            pairs[(g.q0, g.q1)] = v
    return pairs


def pair_product_amplitudes(pairs, indices):
    idx = np.asarray(indices, np.int64)
    amp = np.ones(idx.size, np.complex128)
    for (a, b), v in pairs.items():
        amp *= v[((idx >> a) & 1) + 2 * ((idx >> b) & 1)]
    return amp


def pair_product_fidelity(pairs_ideal, pairs):
    F = 1.0
    for k, v in pairs.items():
        F *= abs(np.vdot(pairs_ideal[k], v)) ** 2 / (np.vdot(v, v).real * np.vdot(pairs_ideal[k], pairs_ideal[k]).real)
    return F
