"""Measured autotuning of the fused-pass shape, kept in a JSON cache.

The library's own choice for ``fuse = -1`` (``plan_choose``) comes from a cost model.  This
module times the candidate shapes (and unfused sweeps) on the device for one circuit and
records the fastest under a key made of the device architecture, n, the dtype and the
circuit's class (its mix of gate kinds).  Looking a plan up is a pure function of that key
and the cache file; tuning is an explicit, separate step.
"""
from __future__ import annotations

import json
import os
import time
from typing import Optional

import numpy as np

from . import qsim as q

CANDIDATES = {
    q.C64: [(12, 4, 5), (12, 4, 4), (12, 3, 5), (12, 3, 4), (12, 3, 3), (11, 3, 4), (11, 2, 3), (10, 2, 3)],
    q.C128: [(11, 3, 4), (11, 3, 3), (11, 2, 4), (11, 2, 3), (10, 2, 3), (10, 1, 3)],
}
DTYPE_NAMES = {q.C64: "c64", q.C128: "c128"}


def circuit_class(gates) -> str:
    """Gate-kind mix rounded to tenths: U1 with real / complex matrices, CP, SWAP, CNOT, U2, FLIP."""
    counts = {"u1r": 0, "u1c": 0, "cp": 0, "swap": 0, "cnot": 0, "u2": 0, "flip": 0}
    total = 0
    for g in gates:
        total += 1
        if g.kind == q.U1:
            im = any(abs(g.m[2 * k + 1]) > 0 for k in range(4)) if isinstance(g, q.Gate) else \
                bool(np.any(np.imag(np.asarray(g.m)) != 0))
            counts["u1c" if im else "u1r"] += 1
        else:
            counts[{q.CP: "cp", q.SWAP: "swap", q.CNOT: "cnot", q.U2: "u2", q.FLIP: "flip"}[g.kind]] += 1
    if total == 0:
        return "empty"
    return ",".join(f"{k}:{round(v / total, 1):.1f}" for k, v in counts.items() if v)


def cache_key(n: int, dtype: int, gates, arch: str) -> str:
    return f"{arch}/{DTYPE_NAMES[dtype]}/n{n}/{circuit_class(gates)}"


def device_arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def load_cache(path: str) -> dict:
    if path and os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def lookup(gates, n: int, dtype: int, path: str, arch: Optional[str] = None) -> Optional[dict]:
    """The cached plan for this circuit's key, or None."""
    entry = load_cache(path).get(cache_key(n, dtype, gates, arch or device_arch()))
    return None if entry is None else dict(entry["plan"])


def plan_for(gates, n: int, dtype: int, path: Optional[str] = None, arch: Optional[str] = None) -> dict:
    """The cached plan if there is one, else the library's automatic choice."""
    hit = lookup(gates, n, dtype, path, arch) if path else None
    return hit if hit is not None else {"fuse": -1}


def tune(gates, n: int, dtype: int, init_index: int = 0, n_traj: int = 16, reps: int = 3,
         path: Optional[str] = None, include_unfused: bool = True, e: float = 0.01) -> dict:
    """Time every candidate shape on this circuit (n_traj trajectories, best of `reps`) and
    store the fastest in the cache at `path` (if given).  Returns the cache entry."""
    import torch
    ga = gates if hasattr(gates, "_type_") else q.gate_array(gates)
    plans = [{"fuse": 1, "tile_bits": k, "reg_bits": r, "run_bits": b} for k, r, b in CANDIDATES[dtype]]
    if include_unfused:
        plans.append({"fuse": 0})
    results = []
    for plan in plans:
        try:
            need = q.traj_bytes_required(ga, n, dtype, n_traj, plan)
        except q.QsimError:
            continue
        if need == 0:
            continue
        buf = torch.empty(need, dtype=torch.uint8, device="cuda")
        q.run_trajectories(ga, n, init_index, dtype, n_traj, e=e, plan=plan, buf=buf)   # warm-up
        best = float("inf")
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            q.run_trajectories(ga, n, init_index, dtype, n_traj, e=e, plan=plan, buf=buf)
            best = min(best, time.perf_counter() - t0)
        results.append((best, plan))
        del buf
    results.sort(key=lambda x: x[0])
    model_plan, model_cost = q.plan_choose(ga, n, dtype)
    entry = {"plan": results[0][1], "seconds": results[0][0], "n_traj": n_traj,
             "model_plan": model_plan, "model_s_per_slot": model_cost,
             "candidates": [{"plan": p, "seconds": t} for t, p in results]}
    if path:
        cache = load_cache(path)
        cache[cache_key(n, dtype, ga, device_arch())] = entry
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return entry
