"""Seeded Poisson load generator for the serving loop (fsim_server_*).

Jobs draw a design from a list, an instance count log-uniform in
[inst_lo, inst_hi] and a cycle budget log-uniform in [cyc_lo, cyc_hi]
(arrival seed and job-parameter seed fixed), arrive as a Poisson process of
rate lam jobs/s, and are submitted to the server as they arrive.  Reports
latency percentiles of (done - arrival) and aggregate instance-cycles/s.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import fibersim as F


def draw_jobs(n_jobs, designs, inst_lo=1, inst_hi=1024, cyc_lo=10_000, cyc_hi=1_000_000,
              param_seed=8):
    rng = np.random.default_rng(param_seed)
    jobs = []
    for k in range(n_jobs):
        d = int(rng.integers(0, len(designs)))
        inst = int(round(math.exp(rng.uniform(math.log(inst_lo), math.log(inst_hi)))))
        cyc = int(round(math.exp(rng.uniform(math.log(cyc_lo), math.log(cyc_hi)))))
        jobs.append(dict(design=d, instances=max(1, inst), cycles=max(1, cyc), seed=0x5EED0000 + 4096 * k))
    return jobs


def arrivals(n_jobs, lam, arrival_seed=7):
    rng = np.random.default_rng(arrival_seed)
    return np.cumsum(rng.exponential(1.0 / lam, n_jobs))


def run(server: F.Server, designs, jobs, arrival_times, timeout_s=600.0, poll_s=0.001, progress=None):
    """Submits jobs at their arrival times (seconds from now), waits for all,
    returns per-job records and a summary.  With `progress` (a text file), a
    line per submitted and per finished job is written to it."""
    t0 = time.perf_counter()
    ids = []
    submit_at = []
    for job, at in zip(jobs, arrival_times):
        now = time.perf_counter() - t0
        if at > now:
            time.sleep(at - now)
        submit_at.append(time.perf_counter() - t0)
        ids.append(server.submit(designs[job["design"]], job["instances"], job["cycles"], job["seed"]))
        if progress:
            print(f"serve: t={submit_at[-1]:.1f}s submitted job {len(ids) - 1}", file=progress, flush=True)
    for k, jid in enumerate(ids):
        server.wait(jid, timeout_s)
        if progress:
            print(f"serve: t={time.perf_counter() - t0:.1f}s job {k} done", file=progress, flush=True)
    wall = time.perf_counter() - t0
    recs = []
    for job, jid in zip(jobs, ids):
        st = server.poll(jid)
        recs.append(dict(job, id=jid, state=st["state"], latency=st["t_done"] - st["t_submit"],
                         queue_wait=st["t_start"] - st["t_submit"] if st["t_start"] >= 0 else None))
    lat = np.array([r["latency"] for r in recs if r["state"] == F.JOB_DONE])
    inst_cycles = sum(r["instances"] * r["cycles"] for r in recs if r["state"] == F.JOB_DONE)
    summary = dict(jobs=len(jobs), completed=int(len(lat)), wall_s=wall,
                   p50_s=float(np.percentile(lat, 50)) if len(lat) else None,
                   p99_s=float(np.percentile(lat, 99)) if len(lat) else None,
                   mean_s=float(lat.mean()) if len(lat) else None,
                   instance_cycles=inst_cycles, instance_cycles_per_s=inst_cycles / wall if wall > 0 else None,
                   total_work_instance_cycles=sum(j["instances"] * j["cycles"] for j in jobs))
    return recs, summary
