"""Serving driver: open-loop Poisson arrivals of SELECT SUM(col2) WHERE col1 op c
queries over prefixes of one resident encrypted table, fed to the library's
continuous-batching server (``sql_server_*``).

Arrival times are drawn up front (seeded exponential gaps at rate lam); the
loop submits every query whose arrival time has passed, runs one server tick
(the next circuit level of every active query, batched together), and records
each query's completion time.  Latency = completion - arrival.
"""
from __future__ import annotations

import math
import time

import numpy as np

from ._lib import Server


def poisson_arrivals(seed, count, lam):
    """Seeded open-loop arrival times (s) with exponential gaps of mean 1/lam."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / lam, size=count))


def run(ctx, queries, arrivals, budget_bytes, max_batch=65536, log=None, timeout_s=600.0):
    """queries: list of dicts (col, sum_col, rows, w, op, lit_a, lit_b, out).
    Returns per-query records with arrival, completion and latency (s)."""
    srv = Server(ctx, budget_bytes, max_batch)
    n = len(queries)
    ids = [None] * n
    done_at = [None] * n
    nxt = 0
    ticks = gates_total = 0
    t0 = time.perf_counter()
    pending = set()
    while True:
        now = time.perf_counter() - t0
        while nxt < n and arrivals[nxt] <= now:
            q = queries[nxt]
            ids[nxt] = srv.submit(q["col"], q["sum_col"], q["rows"], q["w"], q["op"], q["lit_a"], q["out"],
                                  lit_b=q.get("lit_b"))
            pending.add(nxt)
            nxt += 1
        if not pending:
            if nxt >= n:
                break
            time.sleep(max(0.0, min(arrivals[nxt] - now, 0.05)))
            continue
        g, _, _ = srv.step()
        ticks += 1
        gates_total += g
        now = time.perf_counter() - t0
        for i in list(pending):
            if srv.done(ids[i]):
                done_at[i] = now
                pending.discard(i)
                if log:
                    log(f"query {i} ({queries[i]['rows']} rows) done at {now:.2f} s")
        if now > timeout_s:
            raise RuntimeError("serving run exceeded its time limit")
    makespan = time.perf_counter() - t0
    srv.close()
    recs = [{"arrival": float(arrivals[i]), "done": done_at[i], "latency": done_at[i] - float(arrivals[i]),
             "rows": queries[i]["rows"]} for i in range(n)]
    if log:
        log(f"served {n} queries in {makespan:.2f} s, {ticks} ticks, {gates_total} gates")
    return recs, {"makespan": makespan, "ticks": ticks, "gates": gates_total}


def summarize(recs, stats):
    lat = np.array([r["latency"] for r in recs])
    rows = sum(r["rows"] for r in recs)
    return {"queries": len(recs), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "makespan_s": stats["makespan"],
            "rows_per_s": rows / stats["makespan"], "gates_per_s": stats["gates"] / stats["makespan"],
            "ticks": stats["ticks"]}


def sum_bits(w, rows):
    return w + (math.ceil(math.log2(rows)) if rows > 1 else 0)
