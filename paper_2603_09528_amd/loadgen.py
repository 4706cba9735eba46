"""Load generator for the serving loop (tpt_server_*): closed-loop throughput
and open-loop Poisson arrivals with p50/p99 latency.

Every request solves one problem of one of the grid families with a fixed
seeded right-hand side; output buffers come from a per-family pool and are
reused once their request has completed.  Latency is measured by the
library's own clock (submit -> completion detected by the server thread).
"""
from __future__ import annotations

import time
from typing import Dict, List, Sequence

import numpy as np


def _pools(families, rhs_list, per_family):
    import torch
    pools = []
    for p, f in zip(families, rhs_list):
        outs = [torch.empty(p.shape, dtype=torch.float64, device="cuda") for _ in range(per_family)]
        pools.append({"rhs": f, "free": list(range(per_family)), "outs": outs})
    return pools


def run(families: Sequence, rhs_list: Sequence, plans: Sequence, *, n_requests: int, warmup: int,
        rate: float | None, seed: int = 5, max_slots: int = 4, per_family: int = 6,
        budget_bytes: int = 0, weights: Sequence[float] | None = None, keep_outputs: bool = False) -> Dict:
    """Serve n_requests (+ warmup) requests over the families.

    rate None: closed loop (keep max_slots*2 requests in flight) -> throughput.
    rate > 0: open loop with exponential inter-arrival times (Poisson process).
    Returns a dict with solves/s, GDOF/s, p50/p99/max latency in ms; with
    keep_outputs also "_outputs": {family index: the output tensor of that
    family's last completed request} (every request of a family solves the
    same right-hand side).
    """
    import paper_2603_09528_amd as T
    rng = np.random.default_rng(seed)
    nf = len(families)
    w = np.ones(nf) / nf if weights is None else np.asarray(weights, dtype=float) / np.sum(weights)
    total = warmup + n_requests
    choice = rng.choice(nf, size=total, p=w)
    gaps = rng.exponential(1.0 / rate, size=total) if rate else np.zeros(total)
    arrivals = np.cumsum(gaps)
    pools = _pools(families, rhs_list, per_family)
    srv = T.Server(hbm_budget_bytes=budget_bytes, max_slots=max_slots)
    inflight: Dict[int, tuple] = {}
    last_slot: Dict[int, int] = {}
    lat: List[float] = []
    dofs = 0
    t_first = None
    t_last = 0.0
    k = 0
    t0 = time.perf_counter()
    max_inflight = 2 * max_slots if rate is None else 10 ** 9

    def reap(block: bool):
        nonlocal t_first, t_last, dofs
        while True:
            done_any = False
            for t in list(inflight.keys()):
                r = srv.poll(t)
                if r is None:
                    continue
                info, ts, tstart, tdone = r
                idx, fam, slot = inflight.pop(t)
                pools[fam]["free"].append(slot)
                last_slot[fam] = slot
                done_any = True
                if idx >= warmup:
                    lat.append((tdone - ts) * 1e3)
                    dofs += families[fam].dof
                    if t_first is None:
                        t_first = ts
                    t_last = max(t_last, tdone)
            if done_any or not block or not inflight:
                return
            time.sleep(0.0002)

    first_measured_submit = None
    while k < total:
        now = time.perf_counter() - t0
        fam = int(choice[k])
        if rate and now < arrivals[k]:
            reap(False)
            time.sleep(min(0.0005, max(0.0, arrivals[k] - now)))
            continue
        if len(inflight) >= max_inflight or not pools[fam]["free"]:
            reap(True)
            continue
        slot = pools[fam]["free"].pop()
        t = srv.submit(plans[fam], pools[fam]["rhs"], pools[fam]["outs"][slot])
        if k == warmup:
            first_measured_submit = time.perf_counter()
        inflight[t] = (k, fam, slot)
        k += 1
        reap(False)
    while inflight:
        reap(True)
    t_end = time.perf_counter()
    srv.drain()
    wall = t_end - (first_measured_submit or t0)
    lat_a = np.array(lat)
    out = {
        "requests": n_requests,
        "warmup": warmup,
        "rate_per_s": rate,
        "solves_per_s": n_requests / wall,
        "gdofs": dofs / wall / 1e9,
        "p50_ms": float(np.percentile(lat_a, 50)),
        "p99_ms": float(np.percentile(lat_a, 99)),
        "max_ms": float(lat_a.max()),
        "mean_ms": float(lat_a.mean()),
        "slots": max_slots,
    }
    if keep_outputs:
        out["_outputs"] = {fam: pools[fam]["outs"][slot] for fam, slot in last_slot.items()}
    del srv
    return out
