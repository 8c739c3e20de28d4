#!/usr/bin/env python3
"""Benchmark of the noisy state-vector hot path on one MI355X.

Workload (one "step"): QFT on n = 26 qubits from a seeded basis state, 128 Monte Carlo
trajectories in one batch (64 with e = 0.001 and 64 with e = 0.01; Hadamards carry the eq. (1)
rotation noise, controlled phases the theta -> theta + e xi noise), plus the ideal circuit,
complex<float> amplitudes with FP64 fidelity reductions, fused passes.  The step ends when the
128 fidelities are on the host.

Reported: amplitude-updates/s (dense one-qubit gate: 2^n, controlled phase: 2^n / 4,
SWAP: 2^n / 2 per trajectory), trajectories/s, the roofline of the dominant kernel from HIP
events recorded on its stream during the timed steps, the same workload as plain per-gate
sweeps in complex<double>, the unfused sweep kernels at n = 28, and the CPU oracle on a
bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
METRIC = "amplitude-updates/s & %HBM peak; MC trajectories/s; p50/p99 request latency"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fused_qft26.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash():
    h = hashlib.sha256()
    for f in ("fused.hip", "planner.cpp"):
        with open(os.path.join(ROOT, "paper_1412_2293_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=26)
    ap.add_argument("--traj-per-e", type=int, default=64)
    ap.add_argument("--no-extras", action="store_true", help="headline only (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain copy of 1 GiB (for HBM counter calibration)")
    ap.add_argument("--plan", default="", help="tile_bits,reg_bits,run_bits of the fused plan")
    ap.add_argument("--serving-requests", type=int, default=150,
                    help="requests of the seeded serving stream to replay (0: skip)")
    ap.add_argument("--serving-inflight", type=int, default=4)
    ap.add_argument("--leg", default="",
                    help="run only this side measurement (large_state_n32, graph_replay, dm13, dm_qft13, "
                         "fr24, fr_vs_dm12, choi, sweeps_n28, sweeps_n30, grover12_dynamics, grover10_c1, "
                         "serving_full_range, fr24_full, block_rounds_n30) and print its JSON")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported in this build "
              "(trajectories shard trivially across GPUs, see the design notes)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1412_2293_amd as q
    from workloads import qft

    leg_names = ("large_state_n32", "graph_replay", "dm13", "dm_qft13", "dm_qft17", "fr24", "fr_vs_dm12", "choi", "sweeps_n28", "sweeps_n30",
                 "grover12_dynamics", "grover10_c1", "grover20", "serving_full_range", "fr24_full", "block_rounds_n30")
    if a.leg and a.leg not in leg_names:
        print(f"unknown leg {a.leg}; one of {', '.join(leg_names)}", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if a.leg:
        legs = {"large_state_n32": lambda: large_state_bench(q, torch), "graph_replay": lambda: graph_bench(q, torch),
                "dm13": lambda: dm13_bench(q, torch), "dm_qft13": lambda: dm_qft13_bench(q, torch),
                "dm_qft17": lambda: dm_qft17_bench(q, torch),
                "fr24": lambda: fr24_bench(q, torch), "fr_vs_dm12": lambda: fr_vs_dm12_bench(q, torch),
                "choi": lambda: choi_bench(q, torch), "sweeps_n28": lambda: sweeps(q),
                "sweeps_n30": lambda: sweeps(q, 30),
                "grover12_dynamics": lambda: grover12_dynamics_bench(q, torch),
                "grover10_c1": lambda: grover10_c1_bench(q, torch),
                "grover20": lambda: grover20_bench(q, torch),
                "serving_full_range": lambda: serving_full_range_bench(q, torch),
                "fr24_full": lambda: fr24_bench(q, torch, iterations=None),
                "block_rounds_n30": lambda: block_rounds_bench(q, torch)}
        print(json.dumps({a.leg: legs[a.leg]()}), flush=True)
        if a.copy_calibration:
            copy_calibration(q, torch)
        return
    n, Te = a.n, a.traj_per_e
    T = 2 * Te
    es = np.array([0.001] * Te + [0.01] * Te)
    seed = 1
    c = qft(n, seed=seed)
    ga = q.gate_array(c.gates)
    plan = {"fuse": -1}    # the library's automatic choice (cost model)
    if a.plan:
        kb, rb, runb = (int(x) for x in a.plan.split(","))
        plan = {"fuse": 1, "tile_bits": kb, "reg_bits": rb, "run_bits": runb}
    chosen = q.plan_choose(ga, n, q.C64)[0] if plan["fuse"] == -1 else plan
    need = q.traj_bytes_required(ga, n, q.C64, T, plan)
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    updates_per_traj = c.amplitude_updates()

    def step():
        return q.run_trajectories(ga, n, c.init_index, q.C64, T, e=es, seed=seed, plan=plan, buf=buf,
                                  stream=stream)

    log(f"[bench] qft{n} T={T} c64 fused: warmup {a.warmup}")
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    q.timing_reset()
    q.timing_enable(True)
    log(f"[bench] timed {a.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        res = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    q.timing_enable(False)
    ms_step = (t1 - t0) * 1e3 / a.steps
    fused = q.timing_read("fused")
    kernels = {k: q.timing_read(k) for k in ("fused", "noise", "chains", "prep", "jobs", "init", "reduce")}
    value = updates_per_traj * T / (ms_step / 1e3)
    F_c64 = res["F"].copy()
    launch_ms = fused["ms"] / max(fused["launches"], 1)
    launch_bytes = fused["alg_bytes"] / max(fused["launches"], 1)
    achieved = launch_bytes / (launch_ms / 1e3) / 1e9
    traffic = None
    valu_busy = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("source_hash") == source_hash() and tr.get("n") == n and tr.get("T") == T:
            traffic = tr.get("hbm_bytes_per_launch")
            valu_busy = tr.get("valu_busy_by_pass")
    # Algorithmic bytes of a pass count the tiles that can hold amplitude and the support
    # amplitudes read inside them (a run starts from a basis state); the pass that dominates
    # the step is bound by vector-instruction issue, whose profiled busy fraction is given
    # beside the HBM figures.
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_fused<float,RB>", "launches_per_step": fused["launches"] / a.steps,
                "avg_launch_ms": round(launch_ms, 4), "alg_bytes_per_launch": launch_bytes,
                "valu_busy_by_pass_profiled": valu_busy}
    out = {
        "metric": METRIC, "value": value, "unit": "amplitude-updates/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"qft{n}: {T} noisy trajectories (64 at e=0.001, 64 at e=0.01) + ideal, "
                               "complex64 amplitudes, FP64 fidelities, fused passes",
                   "n_qubits": n, "trajectories": T, "gates": len(c.gates), "seed": seed,
                   "plan": plan, "plan_chosen": chosen},
        "trajectories_per_s": T / (ms_step / 1e3),
        "hbm_frac_step": None,
        # the paper's figures, with their hardware: context only (it gives no runtimes)
        "paper_figures": [
            {"what": "largest state-vector simulation", "value": "39 qubits",
             "hardware": "Lomonosov, MVS-100K and MVS-10P supercomputers (distributed state)"},
            {"what": "speed-up of the active-message programming model", "value": "about 10x",
             "hardware": "the same supercomputers (baseline not stated)"},
            {"what": "largest Kraus-operator (density-matrix) simulation", "value": "17 qubits",
             "hardware": "Lomonosov"},
            {"what": "here, on one MI355X", "value": "state vectors up to 34 qubits (complex64, 128 GiB per "
             "slot; 33 checked against a closed form), density matrices up to 17 qubits (the dm_qft17 leg)"}],
        "roofline": roofline,
        "kernels_ms_per_step": {k: v["ms"] / a.steps for k, v in kernels.items()},
    }
    # whole-step HBM fraction: algorithmic bytes of every kernel over the step time
    step_bytes = sum(v["alg_bytes"] for v in kernels.values()) / a.steps
    out["hbm_frac_step"] = round(step_bytes / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    del res
    if a.copy_calibration:
        copy_calibration(q, torch)

    if not a.no_extras:
        del buf
        torch.cuda.empty_cache()
        out["fp64_unfused"] = fp64_unfused(q, c, ga, n, T, es, seed, F_c64, value)
        torch.cuda.empty_cache()
        out["sweeps_n28"] = sweeps(q)
        torch.cuda.empty_cache()
        out["sweeps_n30"] = sweeps(q, 30)
        torch.cuda.empty_cache()
        out["large_state_n32"] = large_state_bench(q, torch)
        torch.cuda.empty_cache()
        out["graph_replay"] = graph_bench(q, torch)
        out["dm13"] = dm13_bench(q, torch)
        torch.cuda.empty_cache()
        out["dm_qft13"] = dm_qft13_bench(q, torch)
        torch.cuda.empty_cache()
        out["dm_qft17"] = dm_qft17_bench(q, torch)
        torch.cuda.empty_cache()
        out["fr24"] = fr24_bench(q, torch)
        torch.cuda.empty_cache()
        out["fr_vs_dm12"] = fr_vs_dm12_bench(q, torch)
        torch.cuda.empty_cache()
        out["grover12_dynamics"] = grover12_dynamics_bench(q, torch)
        torch.cuda.empty_cache()
        out["choi"] = choi_bench(q, torch)
        torch.cuda.empty_cache()
        out["grover10_c1"] = grover10_c1_bench(q, torch)
        torch.cuda.empty_cache()
        out["grover20"] = grover20_bench(q, torch)
        torch.cuda.empty_cache()
        if a.serving_requests > 0:
            out["serving"] = serving_bench(q, torch, a.serving_requests, a.serving_inflight)
            torch.cuda.empty_cache()
            out["serving_full_range"] = serving_full_range_bench(q, torch)
            torch.cuda.empty_cache()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c)
    print(json.dumps(out), flush=True)


def fp64_unfused(q, c, ga, n, T, es, seed, F_c64, fused_value):
    """The same step as plain per-gate sweeps in complex<double> (one timed run), and fused in
    complex<double> (one timed run after a warm-up)."""
    import numpy as np
    import torch
    log("[bench] fp64 unfused per-gate comparison (1 run)")
    plan = {"fuse": 0}
    need = q.traj_bytes_required(ga, n, q.C128, T, plan)
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    q.timing_reset()
    q.timing_enable(True)
    t0 = time.perf_counter()
    res = q.run_trajectories(ga, n, c.init_index, q.C128, T, e=es, seed=seed, plan=plan, buf=buf)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    q.timing_enable(False)
    ms = (t1 - t0) * 1e3
    per = {k: q.timing_read(k) for k in ("sweep_u1", "sweep_cp", "sweep_swap")}
    v = c.amplitude_updates() * T / (ms / 1e3)
    dF = float(np.max(np.abs(res["F"] - F_c64)))
    F64 = res["F"].copy()
    del res
    # the same step fused in complex<double> (automatic plan), on the same buffer size class
    fplan = {"fuse": -1}
    need_f = q.traj_bytes_required(ga, n, q.C128, T, fplan)
    if need_f > buf.numel():
        del buf
        torch.cuda.empty_cache()
        buf = torch.empty(need_f, dtype=torch.uint8, device="cuda")
    q.run_trajectories(ga, n, c.init_index, q.C128, T, e=es, seed=seed, plan=fplan, buf=buf)   # warm-up
    torch.cuda.synchronize()
    q.timing_reset()
    q.timing_enable(True)
    f0 = time.perf_counter()
    resf = q.run_trajectories(ga, n, c.init_index, q.C128, T, e=es, seed=seed, plan=fplan, buf=buf)
    torch.cuda.synchronize()
    f1 = time.perf_counter()
    q.timing_enable(False)
    fz = q.timing_read("fused")
    fused64 = {"ms_per_step": (f1 - f0) * 1e3, "value": c.amplitude_updates() * T / (f1 - f0),
               "plan": q.plan_choose(ga, n, q.C128)[0], "passes": fz["launches"],
               "fused_avg_ms": fz["ms"] / max(fz["launches"], 1),
               "fused_GBps": round(fz["alg_bytes"] / (fz["ms"] / 1e3) / 1e9, 1) if fz["ms"] else None,
               "max_abs_dF_vs_unfused_f64": float(np.max(np.abs(resf["F"] - F64))),
               "max_abs_dF_vs_fused_f32": float(np.max(np.abs(resf["F"] - F_c64)))}
    del resf, buf
    sweeps_ = {}
    for k, d in per.items():
        if d["launches"]:
            sweeps_[k] = {"launches": d["launches"], "avg_ms": d["ms"] / d["launches"],
                          "GB/s": d["alg_bytes"] / (d["ms"] / 1e3) / 1e9,
                          "frac": d["alg_bytes"] / (d["ms"] / 1e3) / 1e9 / HBM_PEAK_GBS}
    return {"dtype": "f64", "ms_per_step": ms, "value": v, "unit": "amplitude-updates/s",
            "speedup_fused_f32_over_unfused_f64": fused_value / v,
            "max_abs_dF_f32_fused_vs_f64_unfused": dF, "kernels": sweeps_, "fused_f64": fused64}


def copy_calibration(q, torch):
    """One plain copy of 1 GiB (the library's copy kernel): 1 GiB read and 1 GiB written, the
    reference for scaling the HBM byte counters of a profiled run."""
    nb = 1 << 30
    src = torch.empty(nb, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nb, dtype=torch.uint8, device="cuda")
    q.copy(dst, src, nb, torch.cuda.current_stream())
    torch.cuda.synchronize()
    del src, dst


def sweeps(q, n=28):
    """Unfused sweep kernels on one state + 1 more trajectory of n qubits, both dtypes: dense
    one-qubit gates on low, middle and top qubits; controlled phases, SWAPs, CNOTs and dense
    two-qubit gates on low pairs (runs of 2^lo contiguous amplitudes: short rows) and on high
    pairs (long rows).  Algorithmic bytes: what the gate must read and write (N amplitudes for
    dense gates, N/4 for a controlled phase, N/2 for a SWAP or CNOT)."""
    import torch
    from workloads import CNOT, CP, Gate, SWAP, U1, U2, haar_2x2
    import numpy as np
    log(f"[bench] unfused sweeps at n={n}")
    rng = np.random.default_rng(0)

    def haar4():
        z = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
        qm, r = np.linalg.qr(z)
        return qm * (np.diag(r) / np.abs(np.diag(r)))

    out = {}
    T = 2
    top = n - 1
    for dt, name in ((q.C64, "c64"), (q.C128, "c128")):
        sv = q.StateVector(n, dt, T)
        sv.init_basis(0)
        res = {}
        cases = [(f"u1_q{k}", Gate(U1, q0=k, m=haar_2x2(rng))) for k in range(n)]
        cases += [("cp_3_20", Gate(CP, q0=3, q1=20, theta=0.3)), ("swap_2_25", Gate(SWAP, q0=2, q1=25)),
                 ("u2_3_20", Gate(U2, q0=3, q1=20, m=haar4())),
                 (f"cp_18_{top}", Gate(CP, q0=18, q1=top, theta=0.3)),
                 (f"swap_20_{top}", Gate(SWAP, q0=20, q1=top)),
                 (f"cnot_19_{top - 1}", Gate(CNOT, q0=19, q1=top - 1)),
                 (f"u2_20_{top}", Gate(U2, q0=20, q1=top, m=haar4()))]
        for label, g in cases:
            kname = {U1: "sweep_u1", CP: "sweep_cp", SWAP: "sweep_swap", CNOT: "sweep_swap",
                     U2: "sweep_2q"}[g.kind]
            q.apply_gate(sv, g)
            torch.cuda.synchronize()
            q.timing_reset()
            q.timing_enable(True)
            for _ in range(5):
                q.apply_gate(sv, g)
            torch.cuda.synchronize()
            q.timing_enable(False)
            d = q.timing_read(kname)
            gbs = d["alg_bytes"] / (d["ms"] / 1e3) / 1e9
            res[label] = {"avg_ms": round(d["ms"] / d["launches"], 4), "GB/s": round(gbs, 1),
                          "frac": round(gbs / HBM_PEAK_GBS, 4)}
        out[name] = res
        sv.close()
        del sv
        torch.cuda.empty_cache()
    return out


def large_state_bench(q, torch, prefixes=(2, 4)):
    """One large state: n = 32 complex64 (32 GiB per slot), 40 layers of Haar one-qubit gates
    and brickwork CZ, e = 0.005, 4 trajectories + ideal (160 GiB), run in full twice: fused passes
    op by op on the vector ALUs (automatic plan) and fused passes whose register rounds run as
    dense 16 x 16 blocks on the FP32 matrix cores (mfma = 1).  Beside them the first 2 and 4
    layers as per-gate sweeps and as fused passes: the difference of the two prefixes is the
    per-layer time past the first layers (where a basis-state start still leaves tiles empty),
    whose ratio is the steady-state speed-up of fusion over per-gate sweeps."""
    import numpy as np
    from workloads import Circuit, random_layers
    n, depth, T, e, seed = 32, 40, 4, 0.005, 4
    c = random_layers(n, depth, seed, pairing="brickwork")
    ga = q.gate_array(c.gates)
    plan = q.plan_choose(ga, n, q.C64)[0]
    need = q.traj_bytes_required(ga, n, q.C64, T, {"fuse": 1, "mfma": 1})
    need = max(need, q.traj_bytes_required(ga, n, q.C64, T))
    log(f"[bench] large state n={n}: {len(c.gates)} gates, {need / 2**30:.1f} GiB")
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    runs = {}
    for name, pl in (("valu", {"fuse": -1}), ("mfma", {"fuse": 1, "mfma": 1})):
        q.timing_reset()
        q.timing_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = q.run_trajectories(ga, n, 0, q.C64, T, e=e, seed=seed, plan=pl, buf=buf)
        t1 = time.perf_counter()
        q.timing_enable(False)
        fz = q.timing_read("fused")
        runs[name] = {"plan": pl if name == "mfma" else plan, "wall_s": t1 - t0, "passes": fz["launches"],
                      "fused_avg_ms": fz["ms"] / max(fz["launches"], 1),
                      "fused_GBps": round(fz["alg_bytes"] / (fz["ms"] / 1e3) / 1e9, 1),
                      "F": res["F"].tolist(), "norm": res["norm"].tolist()}
        del res
    runs["mfma"]["max_abs_dF_vs_valu"] = float(np.max(np.abs(np.array(runs["mfma"]["F"]) - np.array(runs["valu"]["F"]))))
    per_layer = len(c.gates) // depth
    pref = {}
    for L in prefixes:
        pre = Circuit(n, c.gates[:L * per_layer], name="prefix")
        pga = q.gate_array(pre.gates)
        for name, pl in (("fused", {"fuse": -1}), ("unfused", {"fuse": 0})):
            q.timing_reset()
            q.timing_enable(True)
            torch.cuda.synchronize()
            a0 = time.perf_counter()
            r = q.run_trajectories(pga, n, 0, q.C64, T, e=e, seed=seed, plan=pl, buf=buf)
            pref[(L, name)] = (time.perf_counter() - a0, r["F"].copy())
            q.timing_enable(False)
            if name == "unfused":
                sw = q.timing_read("sweep_u1")
            del r
    del buf
    a, b = prefixes
    u1_gbs = sw["alg_bytes"] / (sw["ms"] / 1e3) / 1e9 if sw["ms"] else 0.0
    steady_fused = (pref[(b, "fused")][0] - pref[(a, "fused")][0]) / (b - a)
    steady_unfused = (pref[(b, "unfused")][0] - pref[(a, "unfused")][0]) / (b - a)
    v = runs["valu"]
    return {"workload": f"random{n}x{depth} brickwork, complex64, {T} trajectories + ideal, e={e}",
            "bytes": need, "plan": plan, "passes": v["passes"], "wall_s": v["wall_s"],
            "fused_avg_ms": v["fused_avg_ms"], "fused_GBps": v["fused_GBps"],
            "fused_hbm_frac": round(v["fused_GBps"] / HBM_PEAK_GBS, 4), "F": v["F"], "norm": v["norm"],
            "mfma": runs["mfma"],
            "prefix_s": {f"{L}_{name}": t for (L, name), (t, _) in pref.items()},
            "prefix_speedup": pref[(a, "unfused")][0] / pref[(a, "fused")][0],
            "steady_state_s_per_layer": {"fused": steady_fused, "unfused": steady_unfused},
            "steady_state_speedup": steady_unfused / steady_fused,
            "prefix_max_abs_dF_fused_vs_unfused": float(max(np.max(np.abs(pref[(L, "fused")][1] - pref[(L, "unfused")][1]))
                                                            for L in prefixes)),
            "unfused_u1_GBps": round(u1_gbs, 1), "unfused_u1_hbm_frac": round(u1_gbs / HBM_PEAK_GBS, 4)}


def block_rounds_bench(q, torch, n=30, depth=8, T=4):
    """Random layers (Haar one-qubit gates, noisy brickwork CZ, e = 0.005) on n = 30 complex64
    (8 GiB per slot), T trajectories + ideal, fused op by op on the vector ALUs and with every
    register round as a dense 16 x 16 block on the FP32 matrix cores (mfma = 1): time per pass
    and |dF| between the two.  A short run for counter profiles of both kernel variants."""
    import numpy as np
    from workloads import random_layers
    c = random_layers(n, depth, 4, pairing="brickwork")
    ga = q.gate_array(c.gates)
    out = {"workload": f"random{n}x{depth} brickwork, complex64, {T} trajectories + ideal, e=0.005"}
    F = {}
    for name, pl in (("valu", {"fuse": 1}), ("mfma", {"fuse": 1, "mfma": 1})):
        need = q.traj_bytes_required(ga, n, q.C64, T, pl)
        buf = torch.empty(need, dtype=torch.uint8, device="cuda")
        q.run_trajectories(ga, n, 0, q.C64, T, e=0.005, seed=4, plan=pl, buf=buf)   # warm-up
        torch.cuda.synchronize()
        q.timing_reset()
        q.timing_enable(True)
        t0 = time.perf_counter()
        res = q.run_trajectories(ga, n, 0, q.C64, T, e=0.005, seed=4, plan=pl, buf=buf)
        t1 = time.perf_counter()
        q.timing_enable(False)
        fz = q.timing_read("fused")
        F[name] = res["F"].copy()
        out[name] = {"wall_s": t1 - t0, "passes": fz["launches"], "fused_avg_ms": fz["ms"] / max(fz["launches"], 1),
                     "fused_GBps": round(fz["alg_bytes"] / (fz["ms"] / 1e3) / 1e9, 1)}
        del res, buf
        torch.cuda.empty_cache()
    out["max_abs_dF"] = float(np.max(np.abs(F["mfma"] - F["valu"])))
    return out


def graph_bench(q, torch, reps=20):
    """A launch-bound run: random layers on n = 14 (depth 60, random pairs), 16 trajectories,
    complex64, hundreds of short fused passes.  Eager launches vs one captured-graph replay per
    run; the results are identical."""
    import numpy as np
    from workloads import random_layers
    c = random_layers(14, 60, 8, pairing="random")
    ga = q.gate_array(c.gates)
    T = 16
    need = q.traj_bytes_required(ga, c.n, q.C64, T)
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    eager = q.run_trajectories(ga, c.n, 0, q.C64, T, e=0.01, seed=1, buf=buf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(reps):
        q.run_trajectories(ga, c.n, 0, q.C64, T, e=0.01, seed=1 + k, buf=buf)
    t_eager = (time.perf_counter() - t0) / reps
    with q.TrajGraph(ga, c.n, q.C64, T) as g:
        got = g.launch(0, e=0.01, seed=1)
        same = bool(np.array_equal(got["F"], eager["F"]))
        t0 = time.perf_counter()
        for k in range(reps):
            g.launch(0, e=0.01, seed=1 + k)
        t_graph = (time.perf_counter() - t0) / reps
    passes = len(q.plan_describe(ga, c.n, q.C64)["passes"])
    return {"workload": f"random14x60 (random pairs), T={T}, complex64", "fused_passes": passes,
            "kernel_launches": 2 * passes + 3, "eager_ms": t_eager * 1e3, "graph_ms": t_graph * 1e3,
            "speedup": t_eager / t_graph, "results_identical": same}


def dm13_bench(q, torch):
    """Density-matrix Grover on n = 13 (vec rho: 2^26 complex<double>, 1 GiB), every Hadamard
    as its two-operator Kraus channel (eq. 6, e = 0.02) applied as one superoperator sweep,
    the sign flips exact; fidelity <psi_ideal|rho|psi_ideal> in FP64.  Beside it the mean
    fidelity of 2048 Monte Carlo trajectories of the same circuit, which the channel is the
    exact average of."""
    import numpy as np
    from workloads import grover
    n, e = 13, 0.02
    c = grover(n, seed=5)
    ga = q.gate_array(c.gates)
    log(f"[bench] dm13: {len(c.gates)} gates on vec(rho) of 2^{2 * n} entries")
    rho = q.StateVector(2 * n, q.C128, 1)
    ideal = q.StateVector(n, q.C128, 1)
    # ideal state through the same library (noise off)
    ideal.init_basis(0)
    for g in ga:
        q.apply_gate(ideal, g)
    rho.init_basis(0)
    q.dm_apply_gate(rho, ga[0], e)          # warm-up of the kernels
    rho.init_basis(0)
    torch.cuda.synchronize()
    q.timing_reset()
    q.timing_enable(True)
    t0 = time.perf_counter()
    for g in ga:
        q.dm_apply_gate(rho, g, e)
    f, tr = q.dm_fidelity(rho, ideal, 0)
    t1 = time.perf_counter()
    q.timing_enable(False)
    k = q.timing_read("sweep_2q")
    sweeps = k["launches"]
    gbs = k["alg_bytes"] / (k["ms"] / 1e3) / 1e9 if k["ms"] else 0.0
    rho.close()
    torch.cuda.empty_cache()
    # the same channel through the fused passes: the superoperator circuit on vec(rho) run as one
    # slot of the trajectory machinery (plan picked by the library, and two fixed shapes)
    fused = {}
    sg = q.dm_superop(ga, n, e)
    for dt, dname in ((q.C128, "c128"), (q.C64, "c64")):
        ideal_d = ideal if dt == q.C128 else q.StateVector(n, q.C64, 1)
        if dt == q.C64:
            ideal_d.amplitudes().copy_(ideal.amplitudes().to(torch.complex64))
        plans = [("auto", None)]
        if dt == q.C128:
            plans += [("t11r3", {"fuse": 1, "tile_bits": 11, "reg_bits": 3, "run_bits": 3}),
                      ("t12r4", {"fuse": 1, "tile_bits": 12, "reg_bits": 4, "run_bits": 3})]
        for pname, plan in plans:
            need = q.dm_run_bytes_required(ga, n, dt, e, plan)
            buf = torch.empty(need, dtype=torch.uint8, device="cuda")
            q.dm_run(ga, n, c.init_index, dt, ideal_d, e=e, plan=plan, buf=buf)      # warm-up (plan cache)
            torch.cuda.synchronize()
            # the automatic plan: median of five runs; the fixed shapes: one
            walls = []
            for rep in range(5 if pname == "auto" else 1):
                q.timing_reset()
                q.timing_enable(True)
                t2 = time.perf_counter()
                r = q.dm_run(ga, n, c.init_index, dt, ideal_d, e=e, plan=plan, buf=buf)
                t3 = time.perf_counter()
                q.timing_enable(False)
                walls.append(t3 - t2)
            wall = float(np.median(walls))
            kf = q.timing_read("fused")
            desc = q.plan_describe(sg, 2 * n, dt, plan)
            fgbs = kf["alg_bytes"] / (kf["ms"] / 1e3) / 1e9 if kf["ms"] else 0.0
            fused[f"{dname}_{pname}"] = {
                "plan": {"fused": desc["fused"], "tile_bits": desc["K"], "reg_bits": desc["RB"],
                         "run_bits": desc["run_bits"]},
                "passes": len(desc["passes"]), "wall_s": wall, "runs": len(walls), "fused_ms": kf["ms"],
                "pass_avg_ms": kf["ms"] / max(kf["launches"], 1), "pass_GBps": round(fgbs, 1),
                "pass_hbm_frac": round(fgbs / HBM_PEAK_GBS, 4), "fidelity": r["F"], "trace": r["trace"],
                "fidelity_minus_sweeps": r["F"] - f}
            log(f"[bench] dm13 fused {dname} {pname}: {wall:.4f} s, {len(desc['passes'])} passes, "
                f"F = {r['F']:.12f}")
            del buf, r
            torch.cuda.empty_cache()
        if dt == q.C64:
            ideal_d.close()
    res = q.run_trajectories(ga, n, c.init_index, q.C128, 2048, e=e, seed=11)
    mc = float(np.mean(res["F"]))
    mc_err = float(np.std(res["F"]) / np.sqrt(2048))
    out = {"workload": f"grover{n} (j={c.meta['iterations']}), vec(rho) complex128, e={e}",
           "gates": len(c.gates), "superoperator_gates": len(sg), "superoperator_sweeps": sweeps,
           "wall_s": t1 - t0, "sweep_avg_ms": k["ms"] / max(sweeps, 1), "sweep_GBps": round(gbs, 1),
           "sweep_hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "fidelity": f, "trace": tr,
           "fused": fused, "mc_mean_fidelity_T2048": mc, "mc_stderr": mc_err,
           "dm_minus_mc_in_stderr": (f - mc) / mc_err if mc_err > 0 else None}
    ideal.close()
    return out


def dm_qft17_bench(q, torch, e=0.01):
    """The largest density matrix the library takes: a QFT on n = 17 qubits, vec(rho) of 2^34
    complex64 entries (128 GiB), noisy Hadamards (eq. 6) and noisy controlled phases (eq. 9),
    through the fused density-matrix run (automatic plan); the exact fidelity beside its closed
    form, the noise average of the trajectory fidelity prod_t (1 + exp(-2e^2) exp(-e^2 m_t/2))/2."""
    import math

    import numpy as np
    from workloads import qft
    n = 17
    c = qft(n, seed=17)
    x = c.init_index
    N = 1 << n
    ex = np.zeros(N, np.complex128)
    ex[x] = 1.0
    psi = np.fft.fft(ex) / math.sqrt(N)
    ideal = q.StateVector(n, q.C64, 1)
    ideal.amplitudes().copy_(torch.as_tensor(psi[None, :].astype(np.complex64)).to("cuda"))
    ga = q.gate_array(c.gates)
    need = q.dm_run_bytes_required(ga, n, q.C64, e)
    log(f"[bench] dm_qft17: vec(rho) of 2^{2 * n} complex64 entries ({need / 2**30:.1f} GiB buffer)")
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    q.dm_run(ga, n, x, q.C64, ideal, e=e, buf=buf)      # warm-up (plan cache)
    torch.cuda.synchronize()
    q.timing_reset()
    q.timing_enable(True)
    t0 = time.perf_counter()
    r = q.dm_run(ga, n, x, q.C64, ideal, e=e, buf=buf)
    t1 = time.perf_counter()
    q.timing_enable(False)
    kf = q.timing_read("fused")
    gbs = kf["alg_bytes"] / (kf["ms"] / 1e3) / 1e9 if kf["ms"] else 0.0
    F = 1.0
    for t in range(n):
        m = bin(x & ((1 << t) - 1)).count("1")
        F *= 0.5 * (1.0 + math.exp(-2 * e * e) * math.exp(-e * e * m / 2))
    sg = q.dm_superop(ga, n, e)
    desc = q.plan_describe(sg, 2 * n, q.C64, None)
    out = {"workload": f"qft{n} (x={x}) on vec(rho) of 2^{2 * n} entries, complex64, e={e}, noisy H (eq. 6) "
                       "and controlled phases (eq. 9), fused density-matrix run",
           "gates": len(c.gates), "superoperator_gates": len(sg), "passes": len(desc["passes"]),
           "plan": {"tile_bits": desc["K"], "reg_bits": desc["RB"], "run_bits": desc["run_bits"]},
           "wall_s": t1 - t0, "fused_ms": kf["ms"], "pass_GBps": round(gbs, 1),
           "pass_hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "fidelity": r["F"], "fidelity_closed_form": F,
           "abs_dF": abs(r["F"] - F), "trace": r["trace"],
           "paper": "17-qubit Kraus-operator simulation on the Lomonosov supercomputer (no runtime given)"}
    del buf, r
    ideal.close()
    torch.cuda.empty_cache()
    return out


def dm_qft13_bench(q, torch, es=(0.005, 0.01, 0.02, 0.05), n_inputs=4):
    """Density-matrix QFT on n = 13 (vec rho: 2^26 complex<double>), noisy Hadamards as their
    eq. (6) channel and noisy controlled phases as their eq. (9) channel, for a seeded sample of
    basis inputs and several noise strengths: the exact fidelity <psi_ideal|rho|psi_ideal> of
    each, their mean, and beside it the Section 3.3 lower estimates eq. (11) and eq. (15) (a
    synthetic counterpart of the paper's QFT fidelity figure)."""
    import math

    import numpy as np
    from workloads import qft
    n = 13
    rng = np.random.default_rng(13)
    inputs = [int(x) for x in rng.integers(0, 1 << n, size=n_inputs)]
    log(f"[bench] dm_qft13: {len(es)} noise strengths x {n_inputs} inputs on vec(rho) of 2^{2 * n} entries")

    def eq11(e):
        PH = 0.5 * (1 + math.exp(-2 * e * e))
        PR = math.exp(-e * e)
        return PH ** n * PR ** (n * (n - 1) / 8)

    def eq15(e):
        PH = 0.5 * (1 + math.exp(-2 * e * e))
        P = math.exp(-e * e)
        f = (math.sqrt(1 + 3 * P) - P - 1) / math.sqrt(P * (1 - P))
        PRt = (math.sqrt(P) + f * math.sqrt(1 - P)) ** 2 / (1 + f * f) ** 4
        return PH ** n * PRt ** (n * (n - 1) / 8)

    rho = q.StateVector(2 * n, q.C128, 1)
    ideal = q.StateVector(n, q.C128, 1)
    rows = []
    q.timing_reset()
    q.timing_enable(True)
    t0 = time.perf_counter()
    for e in es:
        fs = []
        for x in inputs:
            ga = q.gate_array(qft(n, seed=1).gates)
            ideal.init_basis(x)
            for g in ga:
                q.apply_gate(ideal, g)
            rho.init_basis(x * ((1 << n) + 1))
            for g in ga:
                q.dm_apply_gate(rho, g, e)
            f, tr = q.dm_fidelity(rho, ideal, 0)
            fs.append(f)
        rows.append({"e": e, "fidelity_by_input": fs, "fidelity_mean": float(np.mean(fs)),
                     "eq11": eq11(e), "eq15": eq15(e)})
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    q.timing_enable(False)
    k = q.timing_read("sweep_2q")
    gbs = k["alg_bytes"] / (k["ms"] / 1e3) / 1e9 if k["ms"] else 0.0
    rho.close()
    ideal.close()
    return {"workload": f"qft{n} on vec(rho) complex128, noisy H (eq. 6) and controlled phases (eq. 9)",
            "inputs": inputs, "by_e": rows, "wall_s": t1 - t0, "runs": len(es) * len(inputs),
            "sweep_GBps": round(gbs, 1), "sweep_hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}


def fr_vs_dm12_bench(q, torch, ranks=(1, 2, 4, 8)):
    """Fixed rank against the exact density matrix on the paper's small case (Grover n = 12,
    e = 0.01, the whole circuit): the marked probability, unnormalised (can only fall short of
    the exact value) and normalised, for several ranks, and the exact value from vec(rho)."""
    from workloads import grover
    n, e = 12, 0.01
    c = grover(n, seed=12)
    ga = q.gate_array(c.gates)
    log(f"[bench] fr_vs_dm12: ranks {ranks}, {len(c.gates)} gates")
    w = q.StateVector(n, q.C128, 1)
    w.init_basis(c.marked)
    rho = q.StateVector(2 * n, q.C128, 1)
    rho.init_basis(0)
    t0 = time.perf_counter()
    for g in ga:
        q.dm_apply_gate(rho, g, e)
    p_dm, tr = q.dm_fidelity(rho, w, 0)
    t_dm = time.perf_counter() - t0
    rows = []
    for r in ranks:
        fr = q.FixedRank(n, r, q.C128)
        fr.init_basis(0)
        t0 = time.perf_counter()
        for g in ga:
            fr.apply_noisy_gate(g, e)
        fu, fn, lt = fr.fidelity(w)
        rows.append({"r": r, "p_unnormalised": fu, "p_normalised": fn, "log_trace": lt,
                     "abs_err_unnormalised": abs(fu - p_dm), "abs_err_normalised": abs(fn - p_dm),
                     "wall_s": time.perf_counter() - t0})
        fr.close()
    rho.close()
    w.close()
    return {"workload": f"grover{n} (j={c.meta['iterations']}), e={e}, complex128", "p_exact_dm": p_dm,
            "trace_dm": tr, "dm_wall_s": t_dm, "by_rank": rows}


def grover_dynamics(q, n, e, seed, ranks=(1, 2, 4, 8), T=256, keep=8):
    """The marked-state probability after every Grover iteration (Section 3.2, the comparison of
    the paper's 12-qubit figure): the exact density matrix (vec(rho), every noisy Hadamard its
    eq. (6) Kraus channel), the fixed-rank form at several ranks (unnormalised and normalised),
    and Monte Carlo trajectories (eq. 1), whose state after iteration k is the same circuit cut
    after that iteration (the noise counters are the gates' positions, so a prefix replays the
    trajectory's first k iterations exactly).  Beside them eq. (10), lambda_1^(n + 2nk) times the
    ideal probability, which rank 1 reproduces."""
    import math

    import numpy as np
    from workloads import grover
    c = grover(n, seed=seed)
    j = c.meta["iterations"]
    per = 2 * n + 2
    ends = [n + k * per for k in range(j + 1)]     # gate count after iteration k (k = 0: after H^n)
    ga = q.gate_array(c.gates)
    w = q.StateVector(n, q.C128, 1)
    w.init_basis(c.marked)
    lam1 = 0.5 * (1.0 + math.exp(-2.0 * e * e))
    p_ideal = [math.sin((2 * k + 1) * math.asin(2.0 ** (-n / 2))) ** 2 for k in range(j + 1)]
    eq10 = [lam1 ** (n + 2 * n * k) * p_ideal[k] for k in range(j + 1)]
    t0 = time.perf_counter()
    rho = q.StateVector(2 * n, q.C128, 1)
    rho.init_basis(0)
    p_dm, g0 = [], 0
    for end in ends:
        for g in ga[g0:end]:
            q.dm_apply_gate(rho, g, e)
        g0 = end
        p_dm.append(q.dm_fidelity(rho, w, 0)[0])
    rho.close()
    t_dm = time.perf_counter() - t0
    fr_rows = []
    for r in ranks:
        fr = q.FixedRank(n, r, q.C128)
        fr.init_basis(0)
        pu, pn, g0 = [], [], 0
        for end in ends:
            for g in ga[g0:end]:
                fr.apply_noisy_gate(g, e)
            g0 = end
            fu, fn, _ = fr.fidelity(w)
            pu.append(fu)
            pn.append(fn)
        fr_rows.append({"r": r, "p_unnormalised": pu, "p_normalised": pn})
        fr.close()
    w.close()
    t0 = time.perf_counter()
    mc_mean, mc_sem, mc_traj = [], [], []
    for end in ends:
        res = q.run_trajectories(ga[:end], n, c.init_index, q.C128, T, e=e, seed=seed, marked=c.marked)
        p = np.asarray(res["p"])
        mc_mean.append(float(p.mean()))
        mc_sem.append(float(p.std(ddof=1) / math.sqrt(T)))
        mc_traj.append([float(x) for x in p[:keep]])
    t_mc = time.perf_counter() - t0
    return {"n": n, "e": e, "iterations": j, "marked": c.marked, "p_ideal": p_ideal, "eq10": eq10,
            "p_dm": p_dm, "fixed_rank": fr_rows, "mc_trajectories": T, "mc_mean": mc_mean, "mc_sem": mc_sem,
            "mc_first_trajectories": [list(x) for x in zip(*mc_traj)], "dm_wall_s": t_dm, "mc_wall_s": t_mc}


def grover12_dynamics_bench(q, torch):
    """grover_dynamics on the paper's case: n = 12, e = 0.01, r = 1, 2, 4, 8, 256 trajectories."""
    log("[bench] grover12 dynamics")
    d = grover_dynamics(q, 12, 0.01, seed=12)
    last = d["iterations"]
    d["summary"] = {
        "final_p_dm": d["p_dm"][last], "final_mc_mean": d["mc_mean"][last], "final_eq10": d["eq10"][last],
        "final_fixed_rank": {row["r"]: [row["p_unnormalised"][last], row["p_normalised"][last]]
                             for row in d["fixed_rank"]},
        "max_unnormalised_minus_dm": max(u - p for row in d["fixed_rank"]
                                         for u, p in zip(row["p_unnormalised"], d["p_dm"])),
    }
    return d


def choi_bench(q, torch):
    """Choi-Jamiolkowski relative states (Section 4) on the density-matrix path: the three-qubit
    phase-error code against the phase-error probability p, with eq. (18) beside it (the paper
    states its fidelity as the square root of the overlap), Shor's nine-qubit code under the same
    errors (with the three-qubit code and an unprotected qubit beside it), and the five-qubit QFT
    under amplitude and phase relaxation (T1, T2 in units of one gate time)."""
    import math

    import workloads as w
    from paper_1412_2293_amd import choi
    log("[bench] choi: phase code and QFT5 relative states")
    t0 = time.perf_counter()
    code = []
    for p in (0.01, 0.05, 0.1, 0.2, 0.3):
        F, tr = choi.relative_state_fidelity(w.phase_code(p), q.C128)
        code.append({"p": p, "overlap": F, "sqrt_overlap": math.sqrt(max(F, 0.0)),
                     "eq18_F_min": math.sqrt(1 - 3 * p * p + 2 * p ** 3), "trace": tr})
    shor = []
    for p in (0.001, 0.01, 0.05, 0.1):
        F, tr = choi.relative_state_fidelity(w.shor_code(p), q.C128)
        shor.append({"p": p, "overlap": F, "sqrt_overlap": math.sqrt(max(F, 0.0)), "trace": tr,
                     "phase_code_overlap": 1 - 3 * p * p + 2 * p ** 3, "unprotected_overlap": 1 - p})
    qft, codes_relax = [], []
    for T1, T2 in ((10.0, 5.0), (30.0, 20.0), (100.0, 70.0), (300.0, 200.0), (1000.0, 700.0)):
        t1 = time.perf_counter()
        F, tr = choi.relative_state_fidelity(w.qft_relaxation(5, T1, T2), q.C128)
        qft.append({"T1": T1, "T2": T2, "overlap": F, "trace": tr, "wall_s": time.perf_counter() - t1})
        Fp, _ = choi.relative_state_fidelity(w.phase_code_relaxation(T1, T2), q.C128)
        Fs, _ = choi.relative_state_fidelity(w.shor_code_relaxation(T1, T2), q.C128)
        # one unprotected qubit over the same time: sum_k |Tr E_k / 2|^2
        g, pz = 1.0 - math.exp(-1.0 / T1), 0.5 * (1.0 - math.exp(-1.0 / T2))
        s1 = math.sqrt(1.0 - g)
        F1 = (1 - pz) * ((1 + s1) / 2) ** 2 + pz * ((1 - s1) / 2) ** 2
        codes_relax.append({"T1": T1, "T2": T2, "phase_code_overlap": Fp, "shor_code_overlap": Fs,
                            "unprotected_overlap": F1})
    return {"workload": "relative states on vec(rho) complex128: phase code (3 + 1 reference qubits), "
                        "Shor's code (9 + 1), both under phase errors and under T1/T2 relaxation of "
                        "one gate time, qft5 with relaxation after every gate (5 + 5 reference qubits, "
                        "2^20 entries)",
            "phase_code": code, "shor_code": shor, "codes_T1T2": codes_relax, "qft5": qft,
            "wall_s": time.perf_counter() - t0}


def fr24_bench(q, torch, iterations=10):
    """Fixed-rank density matrix (r = 8, complex<float> columns, FP64 Gram and eigen-solve) for
    Grover on n = 24, e = 0.02: a bounded prefix of the circuit (the preparation layer and
    `iterations` Grover iterations); the full circuit has 154,392 Kraus steps."""
    from workloads import grover, grover_iterations
    n, r, e = 24, 8, 0.02
    c = grover(n, seed=7, iterations=iterations)
    ga = q.gate_array(c.gates)
    fr = q.FixedRank(n, r, q.C64)
    fr.init_basis(0)
    fr.apply_noisy_gate(ga[0], e, tau=1e-5, zero_tol=1e-6)
    fr.init_basis(0)
    torch.cuda.synchronize()
    q.timing_reset()
    q.timing_enable(True)
    t0 = time.perf_counter()
    ranks = [fr.apply_noisy_gate(g, e, tau=1e-5, zero_tol=1e-6) for g in ga]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    q.timing_enable(False)
    w = q.StateVector(n, q.C64, 1)
    w.init_basis(c.marked)
    fu, fn, lt = fr.fidelity(w)
    kr = {k: q.timing_read(k) for k in ("fr_gram", "fr_recombine")}
    steps = sum(1 for g in c.gates if g.kind == 0)
    full_steps = n + 2 * n * grover_iterations(n)
    per_step = (t1 - t0) / steps
    part = "full circuit" if iterations is None else f"prefix: {iterations} iterations"
    out = {"workload": f"grover{n} {part} (j={c.meta['iterations']}), r={r}, complex64 columns, e={e}",
           "kraus_steps": steps, "wall_s": t1 - t0, "ms_per_kraus_step": per_step * 1e3,
           "max_rank": max(ranks), "p_marked_unnormalised": fu, "p_marked_normalised": fn,
           "log_trace": lt, "full_circuit_kraus_steps": full_steps,
           "projected_full_circuit_s": per_step * full_steps}
    for k, v in kr.items():
        if v["launches"]:
            gbs = v["alg_bytes"] / (v["ms"] / 1e3) / 1e9
            out[k] = {"launches": v["launches"], "avg_ms": v["ms"] / v["launches"], "GB/s": round(gbs, 1),
                      "frac": round(gbs / HBM_PEAK_GBS, 4)}
    if kr["fr_gram"]["launches"]:
        # Gram of the 2r half-columns on the FP64 matrix cores: three real 16 x 16 x 4 products
        # per four pairs, 768 flops per amplitude index executed (mfma_frac against the FP64
        # matrix peak); the method's own count is 544 (the 136 independent entries of a
        # Hermitian 16 x 16, four real multiply-adds each, per pair of indices)
        g = kr["fr_gram"]
        sec = g["ms"] / g["launches"] / 1e3
        tf = 768.0 * (1 << n) / sec / 1e12
        out["fr_gram"].update({"mfma_TFLOPs": round(tf, 2), "alg_TFLOPs": round(544.0 * (1 << n) / sec / 1e12, 2),
                               "fp64_peak_TFLOPs": FP64_PEAK_TFLOPS, "mfma_frac": round(tf / FP64_PEAK_TFLOPS, 4)})
    fr.close()
    w.close()
    return out


def serving_bench(q, torch, n_requests, inflight):
    """Replay the first n_requests of the seeded serving stream (seed 3) with qubit counts capped
    at 20 through the native server: once with every request at t = 0 (sustainable rate), then
    with Poisson arrivals at 0.8x, 0.5x and 1.0x that rate."""
    from paper_1412_2293_amd import serving
    from workloads import serving_stream
    reqs = serving_stream(seed=3, n_max=20)[:n_requests]
    log(f"[bench] serving: building {len(reqs)} requests")
    P = serving.prepare(reqs, q.C64)
    pool_bytes = 16 << 30
    pool = torch.empty(pool_bytes, dtype=torch.uint8, device="cuda")
    cfg = dict(pool_bytes=pool_bytes, dtype=q.C64, max_inflight=inflight, max_chunk_traj=256, pool=pool)
    # warm-up: the kernels' first launches load code objects
    with q.Server(**cfg) as srv:
        serving.replay(srv, P[:8], rate=None)
    log("[bench] serving: calibration (all requests at t = 0)")
    with q.Server(**cfg) as srv:
        cal = serving.replay(srv, P, rate=None)["summary"]
    rate = cal["requests_per_s"]
    out = {"workload": f"first {len(reqs)} requests of the seeded serving stream (seed 3): Poisson arrivals, "
                       "n uniform in [12, 20] (capped from [12, 28]), Grover / QFT / random layers of depth 20n, "
                       "T uniform in [16, 256], e uniform in [0.001, 0.05], complex64, FP64 fidelities",
           "pool_bytes": pool_bytes, "max_inflight": inflight, "calibration": cal,
           "sustainable_requests_per_s": rate}
    for f in (0.8, 0.5, 1.0):
        log(f"[bench] serving: Poisson arrivals at {f} x {rate:.2f} req/s")
        with q.Server(**cfg) as srv:
            out[f"rate_{f}"] = serving.replay(srv, P, rate=f * rate)["summary"]
    main = out["rate_0.8"]
    out.update(latency_p50_s=main["latency_p50_s"], latency_p99_s=main["latency_p99_s"],
               trajectories_per_s=main["trajectories_per_s"], hbm_frac=main["hbm_frac"],
               arrival_rate_per_s=0.8 * rate)
    del pool
    return out


def grover10_c1_bench(q, torch, T=200, runs=10):
    """The plain method at CPU size (Fig. 1): Grover n = 10 (marked index from seed 0, 25
    iterations), 200 noisy trajectories with the eq. (1) rotation after every Hadamard (e = 0.01,
    Philox seed 0) and the ideal circuit in one launch (the whole state sits in one tile), in
    complex<double>.  Median of `runs` timed runs after 3 warm-ups; the distribution of 1 - F
    over the trajectories, eq. (10) and the rigorous lower bound lambda_1^(n + 2nj) beside the
    mean marked probability."""
    import math

    import numpy as np
    from workloads import grover
    c = grover(10, seed=0)
    ga = q.gate_array(c.gates)
    e, seed = 0.01, 0
    plan = {"fuse": -1}
    chosen = q.plan_choose(ga, c.n, q.C128)[0]
    need = q.traj_bytes_required(ga, c.n, q.C128, T, plan)
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    log("[bench] grover10 C1 (200 trajectories)")
    for _ in range(3):
        q.run_trajectories(ga, c.n, c.init_index, q.C128, T, e=e, seed=seed, plan=plan, marked=c.marked, buf=buf)
    torch.cuda.synchronize()
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        res = q.run_trajectories(ga, c.n, c.init_index, q.C128, T, e=e, seed=seed, plan=plan, marked=c.marked,
                                 buf=buf)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    F, p = np.asarray(res["F"]), np.asarray(res["p"])
    j = c.meta["iterations"]
    lam1 = 0.5 * (1.0 + math.exp(-2.0 * e * e))
    p_ideal = math.sin((2 * j + 1) * math.asin(2.0 ** (-c.n / 2))) ** 2
    hist, edges = np.histogram(1.0 - F, bins=12)
    return {"workload": f"grover10 (j={j}, marked {c.marked}), {T} trajectories + ideal, e={e}, complex128, one launch",
            "plan": chosen, "median_s": dt, "trajectories_per_s": T / dt,
            "amplitude_updates_per_s": c.amplitude_updates() * T / dt,
            "F_mean": float(F.mean()), "p_mean": float(p.mean()), "p_ideal": p_ideal,
            "eq10": lam1 ** (c.n + 2 * c.n * j) * p_ideal, "lower_bound_lambda1_pow": lam1 ** (c.n + 2 * c.n * j),
            "one_minus_F_hist": {"counts": hist.tolist(), "edges": [float(x) for x in edges]}}


def grover20_bench(q, torch, T=64):
    """Grover at a size bound by HBM: n = 20 (marked index from seed 20, 804 iterations, every
    Hadamard noisy with e = 0.01), 64 trajectories + ideal in complex<float> (FP64 reductions),
    automatic plan; amplitude-updates/s, trajectories/s, the fused passes' algorithmic bandwidth
    against the HBM peak, and the mean marked probability beside eq. (10)."""
    import math

    import numpy as np
    from workloads import grover
    c = grover(20, seed=20)
    ga = q.gate_array(c.gates)
    e = 0.01
    need = q.traj_bytes_required(ga, c.n, q.C64, T, None)
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    log(f"[bench] grover20 ({len(c.gates)} gates, {T} trajectories)")
    q.run_trajectories(ga, c.n, c.init_index, q.C64, T, e=e, seed=20, marked=c.marked, buf=buf)
    torch.cuda.synchronize()
    q.timing_reset()
    q.timing_enable(True)
    t0 = time.perf_counter()
    res = q.run_trajectories(ga, c.n, c.init_index, q.C64, T, e=e, seed=20, marked=c.marked, buf=buf)
    t1 = time.perf_counter()
    q.timing_enable(False)
    fz = q.timing_read("fused")
    gbs = fz["alg_bytes"] / (fz["ms"] / 1e3) / 1e9 if fz["ms"] else 0.0
    j = c.meta["iterations"]
    lam1 = 0.5 * (1.0 + math.exp(-2.0 * e * e))
    p_ideal = math.sin((2 * j + 1) * math.asin(2.0 ** (-c.n / 2))) ** 2
    out = {"workload": f"grover20 (j={j}), {T} trajectories + ideal, e={e}, complex64, FP64 reductions",
           "plan": q.plan_choose(ga, c.n, q.C64)[0], "wall_s": t1 - t0, "passes": fz["launches"],
           "amplitude_updates_per_s": c.amplitude_updates() * T / (t1 - t0), "trajectories_per_s": T / (t1 - t0),
           "fused_GBps": round(gbs, 1), "fused_hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
           "p_mean": float(np.mean(res["p"])), "eq10": lam1 ** (c.n + 2 * c.n * j) * p_ideal, "p_ideal": p_ideal}
    del buf, res
    return out


def serving_full_range_bench(q, torch, inflight=4, first=60, max_model_s=1.0, pool_gib=32):
    """The serving stream over its full qubit range [12, 28]: of the first `first` requests of the
    seeded stream (seed 3, in arrival order) every one whose modelled time (the library's cost
    model, qs_plan_choose, times its T + 1 slots) is under max_model_s; the others (Grover and
    random layers at n >= 22, up to minutes each) are listed.  The pool is small enough that the
    large requests split into batches and wait for memory (admission waits)."""
    from paper_1412_2293_amd import serving
    from workloads import serving_stream
    reqs = serving_stream(seed=3)[:first]
    keep, skipped, model_total = [], [], 0.0
    for r in reqs:
        c = r.circuit()
        s = q.plan_choose(q.gate_array(c.gates), c.n, q.C64)[1] * (r.T + 1)
        if s <= max_model_s:
            keep.append(r)
            model_total += s
        else:
            skipped.append({"index": r.index, "kind": r.kind, "n": r.n, "T": r.T, "model_s": round(s, 1)})
    log(f"[bench] serving full range: {len(keep)} of {first} requests (n up to 28), pool {pool_gib} GiB")
    P = serving.prepare(keep, q.C64)
    pool_bytes = pool_gib << 30
    pool = torch.empty(pool_bytes, dtype=torch.uint8, device="cuda")
    cfg = dict(pool_bytes=pool_bytes, dtype=q.C64, max_inflight=inflight, max_chunk_traj=256, pool=pool)
    with q.Server(**cfg) as srv:
        serving.replay(srv, P[:4], rate=None)
    with q.Server(**cfg) as srv:
        cal = serving.replay(srv, P, rate=None)["summary"]
    rate = cal["requests_per_s"]
    with q.Server(**cfg) as srv:
        main = serving.replay(srv, P, rate=0.8 * rate)
    del pool
    recs = main["records"]
    return {"workload": f"requests of the first {first} of the seeded serving stream (seed 3, n uniform in [12, 28]) "
                        f"with modelled time <= {max_model_s} s: {len(keep)} kept, n up to {max(r.n for r in keep)}, "
                        "Poisson arrivals at 0.8x the sustainable rate, complex64, FP64 fidelities",
            "pool_bytes": pool_bytes, "max_inflight": inflight, "modelled_s": model_total, "skipped": skipped,
            "calibration": cal, "arrival_rate_per_s": 0.8 * rate, "summary": main["summary"],
            "largest": sorted(({"n": r["n"], "kind": r["kind"], "T": r["T"], "chunks": r["chunks"],
                                "latency_s": round(r["latency_s"], 3), "queue_s": round(r["queue_s"], 3)}
                               for r in recs), key=lambda x: -x["n"])[:6]}


def cpu_baseline(c, prefix=None, workers=None):
    """The CPU oracle on a bounded sample of the workload: one noisy trajectory (e = 0.01) of the
    same circuit (all gates unless `prefix` is given) per host core, each an oracle call in a
    child process of its own (about 15 s each), all cores at once.  Value: the amplitude updates
    of all of them over the wall time; beside it the single-core rate (mean over the children)."""
    import numpy as np
    from workloads import Circuit
    if workers is None:
        # the host's CPU share for one GPU is 16 cores, whatever the machine reports
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
    log(f"[bench] cpu baseline (oracle, {workers} processes, one thread each)")
    n = c.n
    N = 1 << n
    prefix = len(c.gates) if prefix is None else prefix
    part = Circuit(n, c.gates[:prefix], init_index=c.init_index)
    updates = sum({0: N, 1: N // 4, 2: N // 2}.get(g.kind, N) for g in part.gates)
    child = ("import sys, time; sys.path.insert(0, {root!r}); import oracle; from workloads import qft, Circuit; "
             "c = qft({n}, seed={seed}); p = Circuit({n}, c.gates[:{prefix}], init_index=c.init_index); "
             "oracle.lib(); t0 = time.perf_counter(); oracle.sv_run(p, 0.01, seed=1, traj={traj}); "
             "print(time.perf_counter() - t0)")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    t0 = time.perf_counter()
    procs = [subprocess.Popen([sys.executable, "-c", child.format(root=ROOT, n=n, seed=c.meta.get("seed", 1),
                                                                   prefix=prefix, traj=64 + k)],
                              stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env)
             for k in range(workers)]
    times = []
    for pr in procs:
        out, err = pr.communicate()
        if pr.returncode != 0:
            raise RuntimeError(f"cpu baseline child failed ({pr.returncode}): {err[-400:]}")
        times.append(float(out.strip().split()[-1]))
    wall = time.perf_counter() - t0
    return {"value": workers * updates / wall, "unit": "amplitude-updates/s", "cores": workers,
            "kind": "oracle", "host_cores": os.cpu_count(),
            "single_core_value": float(np.mean([updates / t for t in times])),
            "sample": f"qft{n}: {workers} noisy trajectories (e=0.01, trajectory counters 64..{63 + workers}), one "
                      f"per process and core, each the first {prefix} of {len(c.gates)} gates "
                      f"({part.count(0)} H, {part.count(1)} controlled phases) in complex128 plain loops; "
                      f"wall {wall:.1f} s, per process {min(times):.1f}-{max(times):.1f} s"}


if __name__ == "__main__":
    main()
