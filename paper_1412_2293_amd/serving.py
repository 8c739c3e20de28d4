"""Request-stream driver for the native server (qs_srv_*): replays a seeded stream of requests
with Poisson arrivals against a Server and summarises latency and throughput.

The server does all the scheduling (admission by footprint, batching, streams); this module
only submits each request at its arrival time from a host thread and collects the results.
"""
from __future__ import annotations

import threading
import time
from typing import List, Optional

import numpy as np

from . import qsim as q


def state_bytes_per_slot(desc: dict, n: int, amp: int) -> float:
    """Algorithmic HBM bytes of one slot's state traffic under a plan, as the library counts
    them for a fused plan: a pass writes the tiles that can hold amplitude (all of them when the
    first pass stores the zeros) and, after the first, reads the support amplitudes inside them."""
    N = float(1 << n)
    total = 0.0
    for i, p in enumerate(desc["passes"]):
        first = i == 0
        tiles = 1.0 if (first and p["zero_fill"]) else 2.0 ** -bin(p["classical"]).count("1")
        reads = 0.0 if first else 2.0 ** -bin(p["lclassical"]).count("1")
        total += (1.0 + reads) * tiles * N * amp
    return total


def prepare(requests, dtype: int = q.C64, plan=None) -> List[dict]:
    """Build every request's circuit and gate array up front (outside any timed region) and its
    algorithmic HBM bytes: (T + 1) states x the state traffic of its plan."""
    amp = 8 if dtype == q.C64 else 16
    out = []
    for r in requests:
        c = r.circuit()
        ga = q.gate_array(c.gates)
        desc = q.plan_describe(ga, c.n, dtype, plan)
        passes = len(desc["passes"]) if desc["fused"] else len(c.gates)
        per_slot = state_bytes_per_slot(desc, c.n, amp) if desc["fused"] else 2.0 * (1 << c.n) * amp * len(c.gates)
        out.append({"req": r, "circ": c, "ga": ga, "passes": passes,
                    "alg_bytes": per_slot * (r.T + 1),
                    "marked": c.marked if c.marked is not None else -1})
    return out


def replay(server: "q.Server", prepared: List[dict], rate: Optional[float] = None,
           timeout: float = 900.0) -> dict:
    """Submit request i at arrival_i / rate seconds after the start (all at once when rate is
    None) and wait for every result.  Returns per-request records and the summary."""
    n = len(prepared)
    ids: List[Optional[int]] = [None] * n
    submitted = threading.Semaphore(0)
    errors = []
    t_start = time.perf_counter()

    def arrivals():
        try:
            for i, p in enumerate(prepared):
                if rate is not None:
                    due = t_start + p["req"].arrival / rate
                    delay = due - time.perf_counter()
                    if delay > 0:
                        time.sleep(delay)
                r = p["req"]
                ids[i] = server.submit(p["ga"], r.n, p["circ"].init_index, r.T, e=r.e, seed=r.seed,
                                       request=r.index, marked=p["marked"])
                submitted.release()
        except Exception as ex:  # surfaced by the collector below
            errors.append(ex)
            submitted.release()

    th = threading.Thread(target=arrivals, daemon=True)
    th.start()
    records = []
    for i in range(n):
        submitted.acquire()
        if errors:
            th.join()
            raise errors[0]
        res = server.result(ids[i], timeout=timeout)
        info = res["info"]
        p = prepared[i]
        records.append({"index": p["req"].index, "kind": p["req"].kind, "n": p["req"].n, "T": p["req"].T,
                        "latency_s": info["latency_s"], "queue_s": info["queue_s"],
                        "t_submit": info["t_submit"], "t_done": info["t_done"], "chunks": info["n_chunks"],
                        "alg_bytes": p["alg_bytes"], "F_mean": float(np.mean(res["F"]))})
    th.join()
    return {"records": records, "summary": summarise(records, server.stats())}


def summarise(records: List[dict], stats: dict) -> dict:
    lat = np.array([r["latency_s"] for r in records])
    wait = np.array([r["queue_s"] for r in records])
    t0 = min(r["t_submit"] for r in records)
    t1 = max(r["t_done"] for r in records)
    span = t1 - t0
    traj = sum(r["T"] for r in records)
    alg = sum(r["alg_bytes"] for r in records)
    return {"requests": len(records), "makespan_s": span,
            "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
            "latency_mean_s": float(lat.mean()), "queue_p50_s": float(np.percentile(wait, 50)),
            "queue_p99_s": float(np.percentile(wait, 99)), "requests_per_s": len(records) / span,
            "trajectories_per_s": traj / span, "alg_bytes": alg, "alg_GBps": alg / span / 1e9,
            "hbm_frac": alg / span / 8e12, "admission_waits": stats["admission_waits"],
            "chunks": stats["chunks"], "peak_inflight": stats["peak_inflight"],
            "peak_pool_bytes": stats["peak_bytes"], "pool_bytes": stats["pool_bytes"]}
