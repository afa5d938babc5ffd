#!/usr/bin/env python3
"""Benchmark: simulated cycles/s x instances of the per-cycle BSP evaluation
of a fiber-partitioned netlist (Parendi's method) on one MI355X.

One step = one pass of the hot path over one batch of synthetic input: the
single-core workload (about 20k registers, 200k word operators, depth 40,
two 4096 x 64 memories, one instance) simulated for 100,000 cycles with the
on-device stimulus.  Compilation (fiber extraction, packing, encoding) and
autotuning happen once, before the timed region.

Prints ONE JSON line.  Also reports the roofline of the dominant kernel and
the oracle's CPU rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X published HBM3E bandwidth


def algorithmic_bytes_per_cycle(nl, n_live_ops, n_instances=1):
    """Bytes the method itself must move per simulated cycle: read the
    current state and write the next state once at declared widths, 2 reads +
    1 write of 8 bytes per memory, per instance, plus the program once
    (8 bytes per live operator)."""
    import numpy as np
    state_bytes = int(np.ceil(int(nl.reg_width.astype(np.int64).sum()) / 8))
    per_inst = 2 * state_bytes + 24 * nl.n_mems
    return per_inst * n_instances + 8 * n_live_ops, state_bytes


def cpu_baseline(nl, seed, budget_s=12.0):
    """The oracle as it stands, single thread, on a bounded prefix."""
    from oracle import oracle as orc
    sim = orc.Sim(nl, seed=seed)
    t0 = time.perf_counter()
    sim.step(20)
    per = (time.perf_counter() - t0) / 20
    n = max(50, int(budget_s / max(per, 1e-9)))
    t0 = time.perf_counter()
    sim.step(n)
    dt = time.perf_counter() - t0
    return dict(value=n / dt, unit="instance-cycles/s", cores=1, kind="oracle",
                sample=f"{nl.name}: 1 instance, cycles 20..{20 + n} of the same stimulus, "
                       f"single-threaded C oracle ({dt:.1f} s)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cycles", type=int, default=100_000, help="cycles per step")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--retune", action="store_true", help="ignore the autotuner cache")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); "
              "multi-GPU sharding is described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2403_04714_amd import fibersim as F
    if not os.path.exists(F.LIB_PATH):
        from paper_2403_04714_amd import build as B
        B.build()
    from paper_2403_04714_amd import netgen as g
    from paper_2403_04714_amd import tune

    seed = g.STIM_SEED_BASE
    t0 = time.time()
    nl = g.workload("core")
    gen_s = time.time() - t0
    ctx = F.Context(0)
    t0 = time.time()
    best, _ = tune.tune_plain(ctx, nl, targets=(128, 256, 512), threads=(64, 256),
                              launches=(F.LAUNCH_PERSISTENT, F.LAUNCH_GRAPH), cycles=2000,
                              use_cache=not args.retune)
    tune_s = time.time() - t0
    d = F.Design(ctx, nl, pack=F.PACK_SLB, target_processes=best["target"])
    info = d.info()
    sim = F.Sim(d, 1, launch=best["launch"], wg_threads=best["threads"], seed=seed)
    lay = sim.layout()
    stream = ctx.torch_stream
    for _ in range(args.warmup):
        sim.step(args.cycles)
    sim.sync()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        sim.step(args.cycles)
    e1.record(stream)
    e1.synchronize()
    sim.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    gpu_s = e0.elapsed_time(e1) / 1e3
    total_cycles = args.steps * args.cycles
    value = total_cycles * 1 / gpu_s
    ms_per_step = gpu_s * 1e3 / args.steps

    bpc, state_bytes = algorithmic_bytes_per_cycle(nl, info["n_live_ops"])
    if best["launch"] == F.LAUNCH_PERSISTENT:
        kernel = "plain_persistent"
        cycles_per_launch = min(args.cycles, 1 << 20)
        launch_s = gpu_s / args.steps * cycles_per_launch / args.cycles
    else:
        kernel = "plain_cycle"
        cycles_per_launch = 1
        launch_s = gpu_s / total_cycles       # upper bound: includes the graph's launch gaps
    achieved = bpc * cycles_per_launch / launch_s / 1e9
    out = {
        "metric": "simulated cycles/s x instances",
        "value": round(value, 1),
        "unit": "instance-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "single-core netlist, plain form",
                   "registers": int(nl.n_regs), "word_ops": int(nl.n_comb_ops()),
                   "depth": int(info["max_depth"]), "memories": "2 x 4096 x 64b",
                   "instances": 1, "cycles_per_step": args.cycles, "netlist_seed": 1,
                   "stimulus_seed": seed},
        "roofline": {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 3),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
                     "traffic": None,
                     "bytes_per_cycle": bpc, "cycles_per_launch": cycles_per_launch,
                     "launch_ms": round(launch_s * 1e3, 4),
                     "note": "latency-bound: levels x per-level latency + barrier; see latency"},
        "latency": {"us_per_cycle": round(gpu_s / total_cycles * 1e6, 3),
                    "process_levels": int(info["max_process_levels"]) + 2,
                    "ns_per_level_if_all_latency": round(gpu_s / total_cycles * 1e9 /
                                                          (info["max_process_levels"] + 2), 1)},
        "design": {"processes": int(info["n_processes"]), "dup_fiber": round(info["dup_fiber"], 4),
                   "dup_process": round(info["dup_process"], 4), "live_ops": int(info["n_live_ops"]),
                   "max_fiber_cost": int(info["max_fiber_cost"]),
                   "max_process_cost": int(info["max_process_cost"]),
                   "program_bytes": int(info["program_bytes"]),
                   "compile_s": round(info["compile_seconds"], 2), "generate_s": round(gen_s, 2),
                   "autotune_s": round(tune_s, 2), "state_bytes_packed": state_bytes},
        "launch": {"mode": {1: "persistent", 2: "per_cycle", 3: "graph"}[best["launch"]],
                   "workgroups": lay["workgroups"], "threads": lay["threads"],
                   "instructions_in_lds": lay["staged"]},
        "wall_s_timed": round(wall, 3),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(nl, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
