"""Host-side check of the fusion planner: the fused-pass program the library builds
(qs_plan_describe) is executed tile by tile in numpy, with the same tile-local semantics as
the GPU kernel (register rounds, folded controlled phases conditioned on register, thread or
tile-number bits, diagonal ops, SWAP relabelling), and compared with the oracle."""
import math

import numpy as np
import pytest

import oracle
import paper_1412_2293_amd as q
from workloads import (CNOT, CP, FLIP, NOISE_PHASE, NOISE_ROT, SWAP, U1, U2, Circuit, chain_heavy_circuit, grover,
                       qft, random_layers, random_mixed_circuit)

CNOT4 = np.array([[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0], [0, 1, 0, 0]], np.complex128)


def gate_operators(circuit, e, seed, traj):
    """Per gate: the operator the method applies in this trajectory (eq. 1, eq. 2)."""
    sites = [g.site for g in circuit.gates]
    xi = oracle.normals(seed, sites, [traj])[0] if e else np.zeros(len(sites))
    ops = {}
    for gi, g in enumerate(circuit.gates):
        if g.kind == U1:
            M = np.asarray(g.m, np.complex128)
            if e and g.noise == NOISE_ROT:
                a = e * xi[gi]
                M = M @ np.array([[math.cos(a), math.sin(a)], [-math.sin(a), math.cos(a)]])
            ops[gi] = M
        elif g.kind == CP:
            th = g.theta + (e * xi[gi] if e and g.noise == NOISE_PHASE else 0.0)
            ops[gi] = np.exp(-1j * th)
        elif g.kind == U2:
            ops[gi] = np.asarray(g.m, np.complex128)
        elif g.kind == CNOT:
            ops[gi] = CNOT4
    return ops


def _unit(z):
    return z / abs(z) if z != 0 else 1.0 + 0j


def chain_operators(ops, chains):
    """The phase-chain rewrite of the operators: along each chain every inner gate becomes a
    real matrix after an input phase d (M = p diag(1, b) Rm diag(1, d), with b carried into
    the next gate's |1> column and p into the global phase), and the last gate takes the carried
    phase and the global phase.  Inner entries become ("chain", Rm, d)."""
    out = dict(ops)
    for ch in chains:
        carry, glob = 1.0 + 0j, 1.0 + 0j
        for k, g in enumerate(ch):
            M = np.array(ops[g], np.complex128)
            M[:, 1] *= carry
            if k == len(ch) - 1:
                out[g] = glob * M
                break
            p = _unit(M[0, 0])
            d = _unit(M[0, 1]) / p
            b = (_unit(M[1, 1]) / (p * d) if abs(M[1, 1]) >= abs(M[1, 0]) else -_unit(M[1, 0]) / p)
            ph = np.array([[p, p * d], [p * b, p * b * d]])
            Rm = (M / ph).real
            assert np.abs((M / ph).imag).max() < 1e-14
            out[g] = ("chain", Rm, d)
            carry, glob = b, glob * p
    return out


def block_round(v, rnd, regbits, tbits, ar, outer, basis, ops):
    """A round run as one dense block (the kernel's matrix-core path): every op's phases
    conditioned outside the registers on its target's |1> states first, then the ops in order with
    their phases conditioned on register bits (the block), then the outside output phases."""
    def cond_of(kind, bit, idx):
        if kind == 0:
            return (idx >> regbits[bit]) & 1
        if kind == 1:
            return (idx >> tbits[bit]) & 1
        if kind == 3:
            return np.full(idx.size, (basis >> bit) & 1)
        return np.full(idx.size, (outer >> bit) & 1)

    def phases(v, op, post, inside):
        j = regbits[op["p0"]]
        l1 = ar[((ar >> j) & 1) == 1]
        w = np.ones(l1.size, np.complex128)
        for kind, pst, bit, cpg in op["phases"]:
            if pst == post and (kind == 0) == inside:
                w = w * np.where(cond_of(kind, bit, l1) == 1, ops[cpg], 1.0)
        v[l1] *= w

    v = v.copy()
    for op in rnd["ops"]:
        assert op["type"] == 0 and not (op["flags"] & 2)
        phases(v, op, 0, False)
    for op in rnd["ops"]:
        phases(v, op, 0, True)
        j = regbits[op["p0"]]
        l0 = ar[((ar >> j) & 1) == 0]
        l1 = l0 | (1 << j)
        M = ops[op["gate"]]
        x0, x1 = v[l0].copy(), v[l1].copy()
        v[l0] = M[0, 0] * x0 + M[0, 1] * x1
        v[l1] = M[1, 0] * x0 + M[1, 1] * x1
        phases(v, op, 1, True)
    for op in rnd["ops"]:
        phases(v, op, 1, False)
    return v


def emulate(circuit, prog, e=0.0, seed=0, traj=0):
    """Run the program the way the kernel does, on memory that starts as garbage (NaN): the
    first pass makes the basis state in its tile, a pass works only on the tiles that can hold
    amplitude and reads only the amplitudes of the support (every one of them must have been
    written by an earlier pass), and the first pass stores the other tiles as zeros only when
    the program asks for it.  At the end every amplitude must have been written."""
    n = circuit.n
    ops = chain_operators(gate_operators(circuit, e, seed, traj), prog["chains"])
    b = circuit.init_index
    psi = np.full(1 << n, np.nan, np.complex128)
    all_idx = np.arange(1 << n, dtype=np.int64)
    for pi, pas in enumerate(prog["passes"]):
        first = pi == 0
        cl, lc = pas["classical"], pas["lclassical"]
        qpos = pas["q_pos"]
        K = len(qpos)
        assert (cl & ~pas["outer_mask"]) == 0 and lc < (1 << K)
        # Before the pass, amplitudes outside the support (untouched qubits hold b's values:
        # the classical tile-number bits and the tile-local classical bits) are zero wherever
        # they have been written.
        untouched = cl | sum(1 << qpos[j] for j in range(K) if (lc >> j) & 1)
        outside = psi[((all_idx ^ b) & untouched) != 0]
        assert np.all(np.isnan(outside) | (outside == 0)), (pi, "support")
        ar = np.arange(1 << K, dtype=np.int64)
        loc = np.zeros(1 << K, np.int64)
        blocal = 0
        for j, qb in enumerate(qpos):
            loc |= ((ar >> j) & 1) << qb
            blocal |= ((b >> qb) & 1) << j
        readable = ((ar ^ blocal) & lc) == 0
        obits = [bb for bb in range(n) if (pas["outer_mask"] >> bb) & 1]
        for tile in range(1 << (n - K)):
            outer = 0
            for k, bb in enumerate(obits):
                if (tile >> k) & 1:
                    outer |= 1 << bb
            idx = outer | loc
            if (outer ^ b) & cl:
                if first and pas["zero_fill"]:
                    psi[idx] = 0.0
                continue
            if first:
                v = (idx == b).astype(np.complex128)
            else:
                v = np.zeros(1 << K, np.complex128)
                vals = psi[idx[readable]]
                assert np.all(np.isfinite(vals)), (pi, "read of an amplitude no pass wrote")
                v[readable] = vals
            for stage in pas["stages"]:
                for rnd in stage["rounds"]:
                    m = rnd["reg_mask"]
                    regbits = [j for j in range(K) if (m >> j) & 1]
                    tbits = [j for j in range(K) if not (m >> j) & 1]
                    if rnd.get("block_rec", -1) >= 0:
                        v = block_round(v, rnd, regbits, tbits, ar, outer, b, ops)
                        continue
                    for op in rnd["ops"]:
                        if op["type"] == 0:
                            # creg: register bits no earlier gate touched; amplitudes that
                            # disagree with the basis index there must be zero
                            for k, jj in enumerate(regbits):
                                if (op["creg"] >> k) & 1:
                                    off = ((ar ^ blocal) >> jj) & 1 == 1
                                    assert np.all(v[off] == 0), (pi, "creg")
                            j = regbits[op["p0"]]
                            l0 = ar[((ar >> j) & 1) == 0]
                            l1 = l0 | (1 << j)
                            w = [np.ones(l0.size, np.complex128), np.ones(l0.size, np.complex128)]
                            for kind, post, bit, cpg in op["phases"]:
                                if kind == 0:
                                    cond = (l0 >> regbits[bit]) & 1
                                elif kind == 1:
                                    cond = (l0 >> tbits[bit]) & 1
                                elif kind == 3:
                                    # a basis-bit condition: the tile-local qubit is untouched,
                                    # so the amplitudes that disagree with the basis there are
                                    # zero (the phase is one factor, or none, for the block)
                                    jl = qpos.index(bit)
                                    off = ((ar ^ blocal) >> jl) & 1 == 1
                                    assert np.all(v[off] == 0), (pi, "basis condition")
                                    cond = np.full(l0.size, (b >> bit) & 1)
                                else:
                                    cond = np.full(l0.size, (outer >> bit) & 1)
                                w[post] = w[post] * np.where(cond == 1, ops[cpg], 1.0)
                            M = ops[op["gate"]]
                            # a block flagged uniform has no thread-conditioned phase; one flagged
                            # one-factor (64) no register-conditioned output phase
                            for post, flag in ((0, 16), (1, 32)):
                                if op["flags"] & flag:
                                    assert not any(ph[0] == 1 and ph[1] == post for ph in op["phases"])
                            if op["flags"] & 64:
                                assert not any(ph[0] == 0 and ph[1] == 1 for ph in op["phases"])
                            assert bool(op["flags"] & 2) == isinstance(M, tuple)
                            if op["flags"] & 2:
                                # inner chain member: a real matrix after a uniform input phase
                                if op["flags"] & 4:
                                    assert not any(ph[1] == 0 for ph in op["phases"])
                                _, M, d = M
                                w[0] = w[0] * d
                            x0, x1 = v[l0], v[l1] * w[0]
                            v[l0] = M[0, 0] * x0 + M[0, 1] * x1
                            v[l1] = (M[1, 0] * x0 + M[1, 1] * x1) * w[1]
                        elif op["type"] == 1:
                            j0, j1 = regbits[op["p0"]], regbits[op["p1"]]
                            base = ar[(((ar >> j0) & 1) == 0) & (((ar >> j1) & 1) == 0)]
                            quad = [base, base | (1 << j0), base | (1 << j1), base | (1 << j0) | (1 << j1)]
                            x = np.stack([v[t] for t in quad])
                            y = ops[op["gate"]] @ x
                            for r in range(4):
                                v[quad[r]] = y[r]
                        else:
                            if (outer & op["omask"]) != op["ovalue"]:
                                continue
                            f = -1.0 if op["diag_kind"] == 0 else ops[op["gate"]]
                            sel = (ar & op["lmask"]) == op["lvalue"]
                            v[sel] *= f
            psi[idx] = v
    assert np.all(np.isfinite(psi)), "amplitudes no pass wrote"
    return psi, prog["layout"]


def unpermute(state, layout, n):
    idx = np.arange(1 << n, dtype=np.int64)
    phys = np.zeros_like(idx)
    for qb in range(n):
        phys |= ((idx >> qb) & 1) << int(layout[qb])
    return state[phys]


PLANS = [{"fuse": 1},
         {"fuse": 1, "tile_bits": 4, "reg_bits": 2, "run_bits": 1},
         {"fuse": 1, "tile_bits": 5, "reg_bits": 3, "run_bits": 2},
         {"fuse": 1, "tile_bits": 6, "reg_bits": 2, "run_bits": 2},
         {"fuse": 1, "tile_bits": 8, "reg_bits": 2, "run_bits": 2},
         {"fuse": 1, "tile_bits": 7, "reg_bits": 4, "run_bits": 1}]


def circuits():
    yield random_mixed_circuit(7, 150, seed=1)
    yield random_mixed_circuit(9, 120, seed=2)
    yield random_mixed_circuit(11, 90, seed=311)
    yield qft(8, seed=3)
    yield grover(6, seed=4, iterations=3)
    yield random_layers(8, 5, seed=5, pairing="random")
    yield chain_heavy_circuit(9, 140, seed=1)


@pytest.mark.parametrize("plan", PLANS, ids=lambda p: "-".join(f"{k}{v}" for k, v in p.items()))
def test_planner_program_matches_oracle(plan):
    for c in circuits():
        if plan.get("tile_bits", 12) > c.n and plan.get("reg_bits", 3) > c.n:
            continue
        prog = q.plan_describe(c.gates, c.n, q.C128, plan)
        for e, traj in ((0.0, 0), (0.2, 3)):
            psi, layout = emulate(c, prog, e, seed=7, traj=traj)
            ref = oracle.sv_run(c, e, seed=7, traj=traj)
            err = np.linalg.norm(unpermute(psi, layout, c.n) - ref)
            assert err < 1e-12, (c.name, plan, e, err)


MFMA_PLANS = [{"fuse": 1, "mfma": 1},
              {"fuse": 1, "tile_bits": 10, "reg_bits": 4, "run_bits": 2, "mfma": 1}]


@pytest.mark.parametrize("plan", MFMA_PLANS, ids=["default", "t10r4"])
def test_block_rounds_match_oracle(plan):
    """Rounds run as dense blocks: the outside phases moved before and after the block, the ops
    and their register-conditioned phases in order inside it; against the oracle."""
    cases = [random_layers(12, 4, seed=21, pairing="random"), random_layers(13, 3, seed=22),
             random_mixed_circuit(12, 160, seed=23), qft(12, seed=24)]
    blocks = 0
    for c in cases:
        prog = q.plan_describe(c.gates, c.n, q.C64, plan)
        assert prog["mfma"] == 1 and not prog["chains"]
        blocks += sum(1 for pas in prog["passes"] for st in pas["stages"] for rd in st["rounds"]
                      if rd["block_rec"] >= 0)
        for e, traj in ((0.0, 0), (0.2, 5)):
            psi, layout = emulate(c, prog, e, seed=9, traj=traj)
            ref = oracle.sv_run(c, e, seed=9, traj=traj)
            assert np.linalg.norm(unpermute(psi, layout, c.n) - ref) < 1e-12, (c.name, plan, e)
    assert blocks >= 6


def test_stages_split_long_passes():
    c = random_mixed_circuit(7, 400, seed=9)
    prog = q.plan_describe(c.gates, 7, q.C64, {"fuse": 1})
    assert len(prog["passes"]) == 1 and len(prog["passes"][0]["stages"]) > 2
    psi, layout = emulate(c, prog, 0.1, seed=1, traj=2)
    ref = oracle.sv_run(c, 0.1, seed=1, traj=2)
    assert np.linalg.norm(unpermute(psi, layout, 7) - ref) < 1e-12


def test_program_ranges_are_consistent():
    """Every pass and stage covers its own contiguous slice of rounds, ops and outer jobs."""
    for c in circuits():
        for plan in PLANS:
            if plan.get("tile_bits", 12) > c.n and plan.get("reg_bits", 3) > c.n:
                continue
            prog = q.plan_describe(c.gates, c.n, q.C64, plan)
            op_at = round_at = job_at = 0
            for pas in prog["passes"]:
                # the pass's load layout is the rounds-array entry just before its rounds
                assert pas["load_round"] == round_at
                K = len(pas["q_pos"])
                # the load/store layout: RB register bits, none of them among the low run bits
                # (consecutive lanes cover contiguous rows), and the first or the last round's
                # layout when that one qualifies
                lm = pas["load_reg_mask"]
                assert bin(lm).count("1") == prog["RB"] and lm < (1 << K)
                whole = K == c.n
                run_mask = 0 if whole else (1 << min(prog["run_bits"], K)) - 1
                assert lm & run_mask == 0
                rmasks = [rd["reg_mask"] for st in pas["stages"] for rd in st["rounds"]]
                if rmasks[0] & run_mask == 0:
                    assert lm == rmasks[0]
                elif rmasks[-1] & run_mask == 0:
                    assert lm == rmasks[-1]
                # stored from the last round's layout when that one qualifies, else the load one
                sm = pas["store_reg_mask"]
                assert sm & run_mask == 0
                assert sm == (rmasks[-1] if rmasks[-1] & run_mask == 0 else lm)
                round_at += 1
                assert pas["op_begin"] == op_at and pas["round_begin"] == round_at
                assert pas["job_begin"] == job_at
                rec_at = 0
                for st in pas["stages"]:
                    assert st["op_begin"] == op_at and st["round_begin"] == round_at
                    assert st["job_begin"] == job_at and st["rec_begin"] == rec_at
                    for rd in st["rounds"]:
                        # every register layout holds exactly RB tile-local bits (the kernel
                        # inserts one zero bit per register bit to place the thread id)
                        assert bin(rd["reg_mask"]).count("1") == prog["RB"] and rd["reg_mask"] < (1 << K)
                        for op in rd["ops"]:
                            assert op["rec"] >= rec_at
                        op_at += len(rd["ops"])
                        round_at += 1
                    job_at = st["job_end"]
                    rec_at = st["rec_end"]
                    assert st["rec_end"] - st["rec_begin"] <= 4096
                assert pas["op_end"] == op_at and pas["round_end"] == round_at
                assert pas["job_end"] == job_at and pas["rec_size"] == rec_at


def pass_targets(pas):
    """Physical qubits targeted by the non-diagonal ops of a pass (register bit -> tile-local
    bit -> physical bit)."""
    out = 0
    K = len(pas["q_pos"])
    for st in pas["stages"]:
        for rd in st["rounds"]:
            regbits = [j for j in range(K) if (rd["reg_mask"] >> j) & 1]
            for op in rd["ops"]:
                if op["type"] == 0:
                    out |= 1 << pas["q_pos"][regbits[op["p0"]]]
                elif op["type"] == 1:
                    out |= 1 << pas["q_pos"][regbits[op["p0"]]]
                    out |= 1 << pas["q_pos"][regbits[op["p1"]]]
    return out


@pytest.mark.parametrize("plan", PLANS, ids=lambda p: "-".join(f"{k}{v}" for k, v in p.items()))
def test_classical_bits_are_the_untouched_tile_number_bits(plan):
    for c in circuits():
        if plan.get("tile_bits", 12) > c.n and plan.get("reg_bits", 3) > c.n:
            continue
        prog = q.plan_describe(c.gates, c.n, q.C64, plan)
        touched = 0
        for pas in prog["passes"]:
            assert pas["classical"] == pas["outer_mask"] & ~touched, (c.name, plan)
            touched |= pass_targets(pas)


def test_pass_kernel_variant_flags():
    """The per-pass flags that pick a kernel variant agree with the pass's ops: zin_ops says
    whether none (0), some (1) or all (2) of its one-qubit ops find their target untouched, and
    mixed_ops whether it holds any other op (a variant without those paths must never run one)."""
    seen = set()
    for c in circuits():
        for plan in PLANS:
            if plan.get("tile_bits", 12) > c.n and plan.get("reg_bits", 3) > c.n:
                continue
            prog = q.plan_describe(c.gates, c.n, q.C64, plan)
            for pas in prog["passes"]:
                ops = [op for st in pas["stages"] for rd in st["rounds"] for op in rd["ops"]]
                u1 = [op for op in ops if op["type"] == 0]
                zin = sum((op["creg"] >> op["p0"]) & 1 for op in u1)
                expect = 0 if zin == 0 else 2 if zin == len(u1) else 1
                # 3: all untouched, and every op real (1), no chain (2, 4), no input phases, any
                # output phases one uniform factor (64, 32)
                simple = all(op["flags"] & 1 and not op["flags"] & 6 and not any(ph[1] == 0 for ph in op["phases"])
                             and (not any(ph[1] == 1 for ph in op["phases"]) or (op["flags"] & 96) == 96)
                             for op in u1)
                if expect == 2 and simple and len(u1) == len(ops) and not pas["blocks"]:
                    expect = 3
                # 4: none untouched, every one-qubit op real, no chain, no folded phase
                plain = all(op["flags"] & 1 and not op["flags"] & 6 and not op["phases"] for op in u1)
                if expect == 0 and plain and u1 and not pas["blocks"]:
                    expect = 4
                if not u1 and ops and not pas["blocks"]:
                    expect = 5
                assert pas["zin_ops"] == expect, (c.name, plan)
                assert pas["mixed_ops"] == (1 if len(u1) < len(ops) else 0), (c.name, plan)
                seen.add((pas["zin_ops"], pas["mixed_ops"]))
    assert {0, 1, 3} <= {z for z, _ in seen} and {0, 1} <= {m for _, m in seen}
    # every pass of a QFT from a basis state holds only real one-qubit ops on untouched targets
    # with uniform output factors
    c = qft(14, seed=6)
    for pas in q.plan_describe(c.gates, c.n, q.C64, {"fuse": 1, "tile_bits": 6, "reg_bits": 2,
                                                     "run_bits": 2})["passes"]:
        assert (pas["zin_ops"], pas["mixed_ops"]) == (3, 0)


def test_straight_line_rounds():
    """A round is marked for the straight-line path (seq = k) exactly when its pass is of the
    simple untouched-target kind and its k ops are one-qubit ops on register bits k-1, ..., 0 in
    that order; the QFT's rounds all are."""
    marked = 0
    for c in list(circuits()) + [qft(26, seed=1), grover(16, seed=2, iterations=4)]:
        for plan in PLANS[:1] + [{"fuse": 1, "tile_bits": 12, "reg_bits": 4, "run_bits": 4}]:
            if plan.get("tile_bits", 12) > c.n:
                continue
            prog = q.plan_describe(c.gates, c.n, q.C64, plan)
            for pas in prog["passes"]:
                for st in pas["stages"]:
                    for rd in st["rounds"]:
                        ops = rd["ops"]
                        k = len(ops)
                        want = 0
                        if pas["zin_ops"] == 3 and 0 < k <= 4:
                            if all(op["type"] == 0 and op["p0"] == k - 1 - i for i, op in enumerate(ops)):
                                want = k
                        elif pas["zin_ops"] == 4 and prog["RB"] == 4:
                            if 0 < k <= 4 and all(op["type"] == 0 and op["p0"] == i for i, op in enumerate(ops)):
                                want = k
                            elif (k == 9 and ops[4]["type"] == 2
                                  and all(ops[i]["type"] == 0 and ops[i]["p0"] == i and ops[5 + i]["type"] == 0
                                          and ops[5 + i]["p0"] == i for i in range(4))):
                                want = 9
                        assert rd["seq"] == want, (c.name, plan)
                        marked += rd["seq"] > 0
    assert marked >= 12


def test_qft_second_pass_has_a_support_bound():
    """On a QFT from a basis state the low qubits are transformed last, so the second pass still
    has classical tile-number bits: most of its tiles hold zeros and are left alone."""
    c = qft(14, seed=6)
    plan = {"fuse": 1, "tile_bits": 6, "reg_bits": 2, "run_bits": 2}
    prog = q.plan_describe(c.gates, c.n, q.C64, plan)
    assert len(prog["passes"]) >= 3
    assert prog["passes"][0]["classical"] == prog["passes"][0]["outer_mask"]
    assert prog["passes"][1]["classical"] != 0
    psi, layout = emulate(c, prog, 0.1, seed=2, traj=1)
    ref = oracle.sv_run(c, 0.1, seed=2, traj=1)
    assert np.linalg.norm(unpermute(psi, layout, c.n) - ref) < 1e-12


def test_phase_chains_follow_the_wire():
    """Runs of complex one-qubit gates on one physical bit form a chain across diagonal gates, a
    CNOT control and a SWAP (which keeps the physical bit); a real gate, a CNOT target or a
    dense two-qubit gate ends it, and a lone complex gate is no chain."""
    from workloads import Circuit, Gate, haar_2x2
    rng = np.random.default_rng(12)
    Hm = np.array([[1, 1], [1, -1]], np.complex128) / math.sqrt(2.0)

    def u(qb):
        return Gate(U1, q0=qb, m=haar_2x2(rng), noise=NOISE_ROT)

    g = [u(0),                                # 0
         Gate(CP, q0=0, q1=1, theta=0.3),     # 1  diagonal
         Gate(CNOT, q0=0, q1=2),              # 2  q0 is the control
         u(0),                                # 3  continues 0
         Gate(SWAP, q0=0, q1=3),              # 4  logical 3 now sits on the physical bit of 0
         u(3),                                # 5  continues 0, 3
         u(1),                                # 6
         Gate(CNOT, q0=0, q1=1),              # 7  q1 is the target: ends the run of 6 alone
         u(1),                                # 8
         Gate(U1, q0=1, m=Hm),                # 9  real: ends 8 alone
         u(2), u(2),                          # 10, 11
         Gate(U2, q0=2, q1=1, m=np.eye(4, dtype=np.complex128)),   # 12 ends 10, 11
         u(2)]                                # 13 alone
    for i, gg in enumerate(g):
        gg.site = i
    c = Circuit(4, g, name="chains4")
    prog = q.plan_describe(c.gates, c.n, q.C128, {"fuse": 1, "tile_bits": 4, "reg_bits": 2, "run_bits": 1})
    assert sorted(prog["chains"]) == [[0, 3, 5], [10, 11]]
    for e, traj in ((0.0, 0), (0.3, 2)):
        psi, layout = emulate(c, prog, e, seed=5, traj=traj)
        ref = oracle.sv_run(c, e, seed=5, traj=traj)
        assert np.linalg.norm(unpermute(psi, layout, c.n) - ref) < 1e-12


@pytest.mark.parametrize("dtype", [q.C64, q.C128])
def test_stage_records_fit_the_lds_stage(dtype):
    """Every stage's records (matrices, uniform input phases of chain members, phase blocks)
    fit the LDS area the kernel stages them in."""
    cs = list(circuits()) + [chain_heavy_circuit(11, 160, 1), chain_heavy_circuit(13, 160, 2)]
    for c in cs:
        for plan in PLANS + [{"fuse": 1, "tile_bits": 9, "reg_bits": 3, "run_bits": 2}]:
            if plan.get("tile_bits", 12) > c.n and plan.get("reg_bits", 3) > c.n:
                continue
            prog = q.plan_describe(c.gates, c.n, dtype, plan)
            cap = prog["stage_rec_cap"]
            for pas in prog["passes"]:
                for st in pas["stages"]:
                    assert st["rec_end"] - st["rec_begin"] <= cap, (c.name, plan)
                    for rd in st["rounds"]:
                        for op in rd["ops"]:
                            size = {0: 5 if op["flags"] & 4 else 4, 1: 16, 2: 1}[op["type"]]
                            assert st["rec_begin"] <= op["rec"] and op["rec"] + size <= st["rec_end"]


def _in_order_passes(circuit, K, run_bits):
    """Passes the planner's target rule gives when gates are taken strictly in circuit order
    (a pass ends at the first gate whose targets do not fit)."""
    n = circuit.n
    whole = n == K
    cap = K if whole else K - run_bits
    perm = list(range(n))
    passes, targets, high = 1, set(), 0
    for g in circuit.gates:
        if g.kind == SWAP:
            perm[g.q0], perm[g.q1] = perm[g.q1], perm[g.q0]
            continue
        need = []
        if g.kind == U1:
            need = [perm[g.q0]]
        elif g.kind in (U2, CNOT):
            need = [perm[g.q0], perm[g.q1]]
        extra = sum(1 for x in need if x not in targets and (whole or x >= run_bits))
        if high + extra > cap:
            passes, targets, high = passes + 1, set(), 0
        for x in need:
            if x not in targets:
                targets.add(x)
                high += whole or x >= run_bits
    return passes


@pytest.mark.parametrize("make,plan", [
    (lambda: grover(10, seed=4, iterations=6), {"fuse": 1, "tile_bits": 7, "reg_bits": 3, "run_bits": 2}),
    (lambda: random_layers(12, 6, seed=5, pairing="brickwork"), {"fuse": 1, "tile_bits": 6, "reg_bits": 2,
                                                                  "run_bits": 2}),
    (lambda: random_mixed_circuit(11, 160, seed=8), {"fuse": 1, "tile_bits": 6, "reg_bits": 3, "run_bits": 1}),
], ids=["grover10", "brick12", "mixed11"])
def test_passes_are_list_scheduled(make, plan):
    """Gates that commute (disjoint qubits, or both diagonal) may change order so that a pass
    keeps taking gates that fit: fewer passes than taking the circuit strictly in order (a Grover
    iteration in two passes), every qubit's non-diagonal gates still in circuit order, and the
    program's state equal to the oracle's."""
    c = make()
    prog = q.plan_describe(c.gates, c.n, q.C64, plan)
    npass = len(prog["passes"])
    assert npass < _in_order_passes(c, plan["tile_bits"], plan["run_bits"])
    if c.name.startswith("grover"):
        assert npass <= 2 * 6 + 2
    # per physical qubit, the non-diagonal ops appear in increasing gate index
    last = {}
    for pas in prog["passes"]:
        K = len(pas["q_pos"])
        for st in pas["stages"]:
            for rd in st["rounds"]:
                regbits = [j for j in range(K) if (rd["reg_mask"] >> j) & 1]
                for op in rd["ops"]:
                    if op["type"] == 2:
                        continue
                    qbs = [pas["q_pos"][regbits[op["p0"]]]]
                    if op["type"] == 1:
                        qbs.append(pas["q_pos"][regbits[op["p1"]]])
                    for qb in qbs:
                        assert op["gate"] > last.get(qb, -1), (qb, op["gate"])
                        last[qb] = op["gate"]
    for e, traj in ((0.0, 0), (0.2, 3)):
        psi, layout = emulate(c, prog, e, seed=7, traj=traj)
        ref = oracle.sv_run(c, e, seed=7, traj=traj)
        assert np.linalg.norm(unpermute(psi, layout, c.n) - ref) < 1e-12


def test_qft_phases_fold_on_basis_bits():
    """A QFT from a basis state meets every controlled phase while its control is still untouched:
    each is folded into the target's Hadamard as an output phase conditioned on the basis bit
    (kind 3) or on a tile-number bit, so no block has a per-register or per-thread factor, and
    the program still gives the oracle's state for inputs with many and few ones."""
    for n, plan in ((12, {"fuse": 1, "tile_bits": 6, "reg_bits": 2, "run_bits": 2}),
                    (13, {"fuse": 1, "tile_bits": 8, "reg_bits": 3, "run_bits": 2})):
        c = qft(n, seed=2)
        prog = q.plan_describe(c.gates, n, q.C64, plan)
        kinds = set()
        for pas in prog["passes"]:
            for st in pas["stages"]:
                for rd in st["rounds"]:
                    for op in rd["ops"]:
                        kinds |= {ph[0] for ph in op["phases"]}
                        if any(ph[1] == 1 for ph in op["phases"]):
                            assert op["flags"] & 64 and op["flags"] & 32
                        assert not any(ph[1] == 0 for ph in op["phases"])
        assert 3 in kinds and not kinds & {0, 1}
        for init in (c.init_index, (1 << n) - 1, 1):
            ci = Circuit(n, c.gates, name=c.name, init_index=init)
            for e, traj in ((0.0, 0), (0.1, 2)):
                psi, layout = emulate(ci, prog, e, seed=3, traj=traj)
                ref = oracle.sv_run(ci, e, seed=3, traj=traj)
                assert np.linalg.norm(unpermute(psi, layout, n) - ref) < 1e-12
