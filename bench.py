#!/usr/bin/env python3
"""Benchmark: simulated cycles/s x instances of the per-cycle BSP evaluation
of a fiber-partitioned netlist (Parendi's method) on one MI355X.

One step = one pass of the hot path over one batch of synthetic input: the
48-tile SoC (48 copies of the single-core netlist on an 8 x 6 mesh of
registered 32-bit links: 960,576 registers, 9.45M word operators, 96
memories of 4096 x 64, one instance) simulated for 20,000 cycles with the
on-device stimulus, at the fixed launch configuration of
``configs.SOC48_PLAIN``.  Compilation (fiber extraction, packing, encoding)
happens once, before the timed region.

Prints ONE JSON line.  Beside the headline it reports the roofline of the
dominant kernel, the per-cycle barrier cost and the duplication overhead,
the oracle's CPU rate on a bounded sample (one host thread and all host
threads), and, measured in the same run at the fixed configurations of
``configs``: the 48-tile SoC batched x64, the single core plain x1 and
batched x1024, the 8-tile SoC plain x1 and batched x256, the single core
with clock domains, and a served Poisson stream of jobs with p50/p99
latency.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X published HBM3E bandwidth
CPU_THREADS_CAP = 16      # host threads of the all-core baseline (the GPU machine's CPU share)

# packing policies the autotuner tries: bottom-up SLB (Sec. 5.1) and the
# hypergraph alternative (Sec. 6.6)
PACKS = (0, 3)
PACK_NAMES = {0: "slb", 1: "fibers", 2: "single", 3: "hypergraph"}
LAUNCH_MODE = {1: "persistent", 2: "per_cycle", 3: "graph"}


def algorithmic_bytes_per_cycle(nl, n_live_ops, n_instances=1):
    """Bytes the method itself must move per simulated cycle: read the
    current state and write the next state once at declared widths, 2 reads +
    1 write of 8 bytes per memory, per instance, plus the program once
    (8 bytes per live operator)."""
    import numpy as np
    state_bytes = int(np.ceil(int(nl.reg_width.astype(np.int64).sum()) / 8))
    per_inst = 2 * state_bytes + 24 * nl.n_mems
    return per_inst * n_instances + 8 * n_live_ops, state_bytes


def kernel_source_hash():
    """Hash of the plain-form device code (the kernel file and the helpers it
    shares with the batched form), comments and blank lines left out."""
    import hashlib
    import re
    h = hashlib.sha1()
    for name in ("kernels_plain.hip", "device_common.h"):
        with open(os.path.join(ROOT, "paper_2403_04714_amd", "csrc", name)) as f:
            for line in f:
                code = re.sub(r"//.*", "", line).strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:12]


def profile_record(prefix, kernel, workload, processes, threads):
    """The `<prefix>_json:` record of the committed rocprofv3 summary
    profiles/<prefix>_<kernel>_<workload>.md, or None when there is none for
    this configuration or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{prefix}_{kernel}_{workload}.md")
    tag = f"{prefix}_json: "
    try:
        with open(path) as f:
            line = next(l for l in f if l.startswith(tag))
        rec = json.loads(line[len(tag):])
    except (OSError, StopIteration, ValueError):
        return None
    if (rec.get("kernel_source") != kernel_source_hash() or rec.get("processes") != processes
            or rec.get("threads") != threads):
        return None
    return rec


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"model": model, "logical_cpus_available": len(os.sched_getaffinity(0))}


def cpu_baseline(nl, seed, budget_s=15.0):
    """The oracle as it stands on a bounded sample of the workload: one host
    thread stepping instance 0, then one oracle instance per host thread
    (instances are independent), each stepping its own seed for budget_s."""
    from oracle import oracle as orc
    block = 2 if nl.n_nodes > 2_000_000 else 100
    sim = orc.Sim(nl, seed=seed)
    sim.step(block)
    n, dt, t0 = 0, 0.0, time.perf_counter()
    while dt < budget_s:
        sim.step(block)
        n += block
        dt = time.perf_counter() - t0
    single = n / dt
    del sim
    P = max(1, min(CPU_THREADS_CAP, len(os.sched_getaffinity(0))))
    done = [0] * P
    start = threading.Barrier(P + 1)

    def run(k):
        s = orc.Sim(nl, seed=seed + k)
        s.step(block)
        start.wait()
        # each thread's own deadline, taken after the common start
        end = time.perf_counter() + budget_s
        while time.perf_counter() < end:
            s.step(block)
            done[k] += block

    ths = [threading.Thread(target=run, args=(k,)) for k in range(P)]
    for t in ths:
        t.start()
    start.wait()
    t0 = time.perf_counter()
    for t in ths:
        t.join()
    wall = time.perf_counter() - t0
    all_rate = sum(done) / wall
    return dict(value=round(all_rate, 2), unit="instance-cycles/s", cores=P, kind="oracle",
                sample=f"{nl.name}: {P} oracle instances (seeds {seed:#x}+i), one per host thread, "
                       f"{sum(done)} instance-cycles in {wall:.1f} s after {block} warm-up cycles each",
                single_thread={"value": round(single, 3), "unit": "instance-cycles/s", "cores": 1,
                               "sample": f"instance 0, cycles {block}..{block + n} ({dt:.1f} s)"},
                host=host_cpu(), oracle_build="gcc -O2, plain C, single-threaded per instance")


def time_sim(sim, stream, cycles, warm):
    """Seconds of GPU time for `cycles` cycles after `warm` untimed ones
    (HIP events on the library's stream)."""
    import torch
    if warm:
        sim.step(warm)
    sim.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(cycles)
    e1.record(stream)
    e1.synchronize()
    sim.sync()
    return e0.elapsed_time(e1) / 1e3


def design_stats(info):
    return {"pack": PACK_NAMES.get(int(info.get("pack", -1)), None),
            "processes": int(info["n_processes"]), "live_ops": int(info["n_live_ops"]),
            "dup_fiber": round(info["dup_fiber"], 4), "dup_process": round(info["dup_process"], 4),
            "duplicated_ops_per_cycle": int(round((info["dup_process"] - 1) * info["n_live_ops"])),
            "max_fiber_cost": int(info["max_fiber_cost"]), "max_process_cost": int(info["max_process_cost"]),
            "process_levels": int(info["max_process_levels"]) + 2,
            "program_bytes": int(info["program_bytes"]), "compile_s": round(info["compile_seconds"], 2)}


def barrier_estimate(sim, cycles=24):
    """Per-cycle cost outside the slowest workgroup's compute, from the phase
    timestamps: cycle period minus the slowest workgroup's compute span
    (start to commit).  With graph launches this is the launch gap and the
    start skew; with the persistent kernel, the grid barrier."""
    import numpy as np
    sim.enable_trace(cycles)
    sim.step(cycles)
    tr = sim.trace().astype(np.int64)
    stride = tr.shape[2]
    period = np.diff(tr[:, :, 0].min(axis=1)) * 10 / 1000
    comp = (tr[:, :, stride - 2] - tr[:, :, 0]).max(axis=1) * 10 / 1000
    return {"traced_period_us": round(float(np.median(period)), 3),
            "slowest_compute_us": round(float(np.median(comp[1:])), 3),
            "outside_compute_us": round(float(np.median(period) - np.median(comp[1:])), 3)}


def empty_design_barrier(F, g, ctx, workgroups, cfg, seed, cycles=4000):
    """Pure synchronization per cycle: a design without operators (every
    register keeps its value through its own next-value node), one register
    per workgroup, run like the headline (same launch mode and threads)."""
    import numpy as np
    b = g.Builder()
    for r in range(workgroups):
        b.add_reg(1, r & 1)
        b.set_next(r, b.reg(r))
    d = F.Design(ctx, b.build("empty"), partition=np.arange(workgroups, dtype=np.uint32))
    sim = F.Sim(d, 1, launch=cfg.launch, wg_threads=cfg.threads, seed=seed, stage=cfg.stage)
    us = time_sim(sim, ctx.torch_stream, cycles, 200) / cycles * 1e6
    sim.close()
    d.close()
    return round(us, 3)


def plain_record(F, ctx, cfg, nl, cycles, warm, seed, design=None, trace=False):
    """Plain form, one instance, at a fixed configuration."""
    d = design or cfg.design(ctx, nl)
    info = d.info()
    info["pack"] = cfg.pack
    sim = cfg.sim(d, seed)
    gpu_s = time_sim(sim, ctx.torch_stream, cycles, warm)
    lay = sim.layout()
    rec = {"workload": f"{nl.name} x1", "instances": 1, "cycles": cycles,
           "value": round(cycles / gpu_s, 1), "unit": "instance-cycles/s",
           "us_per_cycle": round(gpu_s / cycles * 1e6, 3), "config": cfg.label(),
           "workgroups": lay["workgroups"], "threads": lay["threads"],
           "instructions_in_lds": lay["staged"], "design": design_stats(info)}
    if trace:
        rec["sync"] = barrier_estimate(sim)
    sim.close()
    if design is None:
        d.close()
    return rec


def batched_record(F, ctx, cfg, nl, cycles, warm, seed, plain_rate=None):
    """Batched form: cfg.instances instances in one launch per cycle
    (hipGraph), at a fixed configuration."""
    d = cfg.design(ctx, nl)
    info = d.info()
    info["pack"] = cfg.pack
    sim = cfg.sim(d, seed)
    gpu_s = time_sim(sim, ctx.torch_stream, cycles, warm)
    bpc, _ = algorithmic_bytes_per_cycle(nl, info["n_live_ops"], cfg.instances)
    achieved = bpc / (gpu_s / cycles) / 1e9
    lay = sim.layout()
    bi = d.batched_info()
    value = cfg.instances * cycles / gpu_s
    rec = {"workload": f"{nl.name} x{cfg.instances}", "instances": cfg.instances, "cycles": cycles,
           "value": round(value, 1), "unit": "instance-cycles/s",
           "us_per_cycle": round(gpu_s / cycles * 1e6, 2), "config": cfg.label(),
           "roofline": {"bound": "alu", "kernel": "batched_cycle2" if cfg.tiles_per_wave == 2 else "batched_cycle",
                        "hbm_achieved_GBs": round(achieved, 2), "hbm_frac": round(achieved / HBM_PEAK_GBS, 5),
                        "bytes_per_cycle": bpc},
           "workgroups": lay["workgroups"], "threads": lay["threads"],
           "wave_lds_bytes": int(bi["wave_lds_bytes"]) * cfg.tiles_per_wave, "instructions": int(bi["n_instr"]),
           "design": design_stats(info)}
    if plain_rate:
        rec["vs_plain_x1"] = round(value / plain_rate, 2)
    sim.close()
    d.close()
    return rec


def bench_served(F, g, configs, ctx, n_jobs, lam, inst_hi, cyc_lo, cyc_hi):
    """Served Poisson stream over the single-core and 8-tile SoC designs."""
    from paper_2403_04714_amd import serve
    designs = [F.Design(ctx, g.workload(w), pack=pk, target_processes=t) for w, pk, t in configs.SERVED]
    jobs = serve.draw_jobs(n_jobs, designs, inst_lo=1, inst_hi=inst_hi, cyc_lo=cyc_lo, cyc_hi=cyc_hi)
    arr = serve.arrivals(n_jobs, lam=lam)
    srv = F.Server(ctx, 64 << 30, quantum_cycles=256)
    recs, summ = serve.run(srv, designs, jobs, arr, timeout_s=600)
    st = srv.stats()
    srv.close()
    out = {"designs": [f"{w} ({d.info()['n_processes']} processes, {PACK_NAMES[pk]} packing)"
                       for (w, pk, _), d in zip(configs.SERVED, designs)],
           "jobs": n_jobs, "arrival_rate_per_s": lam, "instances": f"log-uniform [1, {inst_hi}]",
           "cycles": f"log-uniform [{cyc_lo}, {cyc_hi}]",
           "scale_vs_serving_config": ("scaled down to fit the benchmark run: the serving configuration "
                                       "draws cycle budgets log-uniform in [10k, 1M] and sweeps 200 jobs "
                                       "per arrival rate (bench.py --study serving-c3 runs budgets from "
                                       "its 10k floor)"),
           "completed": summ["completed"], "p50_s": round(summ["p50_s"], 4), "p99_s": round(summ["p99_s"], 4),
           "mean_s": round(summ["mean_s"], 4), "wall_s": round(summ["wall_s"], 3),
           "value": round(summ["instance_cycles_per_s"], 1), "unit": "instance-cycles/s",
           "total_work_instance_cycles": int(summ["total_work_instance_cycles"]),
           "quanta": int(st["quanta"]), "device_busy_s": round(st["busy_seconds"], 3)}
    for d in designs:
        d.close()
    return out


def study_serving(F, g, configs, ctx, n_jobs=24, lams=(1.0, 2.0, 4.0, 8.0, 16.0, 64.0), cyc_lo=100,
                  cyc_hi=2000):
    """The serving mix swept over the mean arrival rate: p50/p99 of (done -
    arrival) and aggregate instance-cycles/s per rate, one fresh server per
    rate over the same compiled designs and the same job draw."""
    from paper_2403_04714_amd import serve
    designs = [F.Design(ctx, g.workload(w), pack=pk, target_processes=t) for w, pk, t in configs.SERVED]
    jobs = serve.draw_jobs(n_jobs, designs, inst_lo=1, inst_hi=1024, cyc_lo=cyc_lo, cyc_hi=cyc_hi)
    work = sum(j["instances"] * j["cycles"] for j in jobs)
    print(json.dumps({"serving_study": {"jobs": n_jobs, "total_work_instance_cycles": int(work),
                                        "cycles": f"log-uniform [{cyc_lo}, {cyc_hi}]"}}), file=sys.stderr,
          flush=True)
    rows = []
    for lam in lams:
        srv = F.Server(ctx, 64 << 30, quantum_cycles=256)
        recs, summ = serve.run(srv, designs, jobs, serve.arrivals(n_jobs, lam=lam), timeout_s=1800,
                               progress=sys.stderr)
        st = srv.stats()
        srv.close()
        waits = sorted(r["queue_wait"] for r in recs if r["queue_wait"] is not None)
        rows.append({"arrival_rate_per_s": lam, "offered_instance_cycles_per_s": round(work * lam / n_jobs, 1),
                     "completed": summ["completed"], "p50_s": round(summ["p50_s"], 4),
                     "p99_s": round(summ["p99_s"], 4), "mean_s": round(summ["mean_s"], 4),
                     "max_queue_wait_s": round(waits[-1], 4) if waits else None,
                     "wall_s": round(summ["wall_s"], 3), "instance_cycles_per_s": round(summ["instance_cycles_per_s"], 1),
                     "device_busy_s": round(st["busy_seconds"], 3)})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    out = {"jobs": n_jobs, "total_work_instance_cycles": int(work),
           "designs": [f"{w} ({d.info()['n_processes']} processes, {PACK_NAMES[pk]} packing)"
                       for (w, pk, _), d in zip(configs.SERVED, designs)],
           "instances": "log-uniform [1, 1024]", "cycles": f"log-uniform [{cyc_lo}, {cyc_hi}]", "rows": rows}
    for d in designs:
        d.close()
    return out


def study_prng(F, g, ctx, cycles=2000, warm=200):
    """The synchronization experiment of Sec. 4.1 on this GPU: independent
    xorshift32 fibers (no communication), a fixed number of fibers per
    workgroup (7, 56, 448), workgroups swept from 64 upwards; each series'
    rate is normalised to its rate at 64 workgroups.  Both barriers are
    measured: the persistent kernel's grid barrier and per-cycle launches in
    a hipGraph."""
    import numpy as np
    rows = []
    for k in (7, 56, 448):
        for G in (64, 128, 256, 512, 1024, 2048):
            n = k * G
            nl = g.prng_array(n)
            d = F.Design(ctx, nl, partition=np.arange(n, dtype=np.uint32) // k)
            for launch in (F.LAUNCH_PERSISTENT, F.LAUNCH_GRAPH):
                try:
                    sim = F.Sim(d, 1, launch=launch, wg_threads=64)
                except F.FsimError:
                    continue                       # not co-resident: no grid barrier possible
                gpu_s = time_sim(sim, ctx.torch_stream, cycles, warm)
                rows.append({"fibers_per_wg": k, "workgroups": G,
                             "launch": "persistent" if launch == F.LAUNCH_PERSISTENT else "graph",
                             "rate_hz": round(cycles / gpu_s, 1), "us_per_cycle": round(gpu_s / cycles * 1e6, 3)})
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
                sim.close()
            d.close()
    for r in rows:
        base = [x for x in rows if x["fibers_per_wg"] == r["fibers_per_wg"] and x["launch"] == r["launch"]
                and x["workgroups"] == 64]
        r["normalised"] = round(r["rate_hz"] / base[0]["rate_hz"], 4) if base else None
    return rows


def trace_split(sim, cycles=24):
    """Phase timestamps of `cycles` cycles: cycle period, slowest and median
    workgroup compute span (start to commit) and the level-0 span (register
    gathers), medians over cycles, in us."""
    import numpy as np
    sim.enable_trace(cycles)
    sim.step(cycles)
    tr = sim.trace().astype(np.int64)
    stride = tr.shape[2]
    period = np.diff(tr[:, :, 0].min(axis=1)) * 10 / 1000
    comp = (tr[:, :, stride - 2] - tr[:, :, 0]) * 10 / 1000
    lvl0 = (tr[:, :, 1] - tr[:, :, 0]) * 10 / 1000
    return {"period_us": round(float(np.median(period)), 3),
            "compute_max_us": round(float(np.median(comp[1:].max(axis=1))), 3),
            "compute_median_us": round(float(np.median(comp[1:])), 3),
            "gather_us": round(float(np.median(lvl0[1:])), 3)}


def study_packing(F, g, tune, ctx):
    """Bottom-up SLB (Sec. 5.1) against hypergraph packing (Sec. 6.6) on the
    single-core and 8-tile designs: duplication, straggler cost, compile
    time, and the rate of the plain form (one instance, one-wave processes,
    instructions from global memory, graph launches) and of the batched
    form (single-core x1024, 8-tile x256)."""
    rows = []
    cases = (("core", (1024, 2048, 4096), 1024, (2048, 4096, 8192)),
             ("soc8", (2048, 4096), 256, (16384, 32768)))
    for name, ptargets, n_inst, btargets in cases:
        nl = g.workload(name)
        for t in sorted(set(ptargets) | set(btargets)):
            for pk in PACKS:
                t0 = time.time()
                d = F.Design(ctx, nl, pack=pk, target_processes=t)
                comp = time.time() - t0
                info = d.info()
                rec = {"design": name, "target": t, "pack": PACK_NAMES[pk], "processes": int(info["n_processes"]),
                       "dup_process": round(info["dup_process"], 4),
                       "max_process_cost": int(info["max_process_cost"]),
                       "max_fiber_cost": int(info["max_fiber_cost"]), "compile_s": round(comp, 2)}
                if t in ptargets:
                    s = tune.time_plain(ctx, d, F.LAUNCH_GRAPH, 64, 3000 if name == "core" else 1500,
                                        stage=F.STAGE_GLOBAL, reps=3)
                    rec["plain_khz"] = round(1 / s / 1e3, 2)
                if t in btargets:
                    s = tune.time_batched(ctx, d, n_inst, 256, 128 if name == "core" else 64)
                    rec[f"batched_x{n_inst}_M"] = round(n_inst / s / 1e6, 4)
                rows.append(rec)
                print(json.dumps(rec), file=sys.stderr, flush=True)
                d.close()
    return {"rows": rows}


def study_scaling(F, g, tune, ctx, seed):
    """The scaling study of Sec. 6.3 on this GPU.  Strong scaling: the
    single-core design at a growing number of one-wave processes, split into
    compute (slowest workgroup), register gathers (the exchange: level 0) and
    the rest of the cycle (launch gap, i.e. synchronization).  Weak scaling:
    meshes of 1 to 48 core tiles at a fixed number of processes per tile."""
    strong = []
    nl = g.workload("core")
    for P in (64, 128, 256, 512, 1024, 2048, 4096, 8192):
        d = F.Design(ctx, nl, pack=F.PACK_SLB, target_processes=P)
        info = d.info()
        best = None
        for st in (F.STAGE_LDS, F.STAGE_GLOBAL):
            try:
                sim = F.Sim(d, 1, launch=F.LAUNCH_GRAPH, wg_threads=64, seed=seed, stage=st)
            except F.FsimError:
                continue
            us = time_sim(sim, ctx.torch_stream, 2000, 200) / 2000 * 1e6
            if best is None or us < best[0]:
                if best is not None:
                    best[2].close()
                best = (us, st, sim)
            else:
                sim.close()
        us, st, sim = best
        rec = {"processes": int(info["n_processes"]), "us_per_cycle": round(us, 2),
               "rate_khz": round(1e3 / us, 2), "instructions_in_lds": st == F.STAGE_LDS,
               "dup_process": round(info["dup_process"], 4), "max_process_cost": int(info["max_process_cost"])}
        rec.update(trace_split(sim))
        strong.append(rec)
        print(json.dumps({"strong": rec}), file=sys.stderr, flush=True)
        sim.close()
        d.close()
    weak = []
    core = g.gen_core(seed=1)
    for rows, cols in ((1, 1), (1, 2), (2, 2), (2, 4), (4, 4), (8, 6)):
        nlw = g.gen_soc(rows, cols, core, mesh_seed=2) if rows * cols > 1 else core
        t0 = time.time()
        d = F.Design(ctx, nlw, pack=F.PACK_SLB, target_processes=512 * rows * cols)
        compile_s = time.time() - t0
        info = d.info()
        sim = F.Sim(d, 1, launch=F.LAUNCH_GRAPH, wg_threads=64, seed=seed, stage=F.STAGE_GLOBAL)
        us = time_sim(sim, ctx.torch_stream, 500, 50) / 500 * 1e6
        rec = {"tiles": rows * cols, "word_ops": int(nlw.n_comb_ops()), "processes": int(info["n_processes"]),
               "us_per_cycle": round(us, 2), "rate_khz": round(1e3 / us, 2),
               "dup_process": round(info["dup_process"], 4), "compile_s": round(compile_s, 1)}
        rec.update(trace_split(sim))
        weak.append(rec)
        print(json.dumps({"weak": rec}), file=sys.stderr, flush=True)
        sim.close()
        d.close()
    return {"strong": strong, "weak": weak}


def profile_run(F, g, configs, ctx, name, cycles=32):
    """A short fixed run for hardware counters: the named configuration of
    `configs`, one launch per simulated cycle (so each dispatch is one
    cycle), `cycles` cycles."""
    import numpy as np
    seed = g.STIM_SEED_BASE
    if name == "plain-prng":
        d = F.Design(ctx, g.prng_array(7 * 64), partition=np.arange(7 * 64, dtype=np.uint32) // 7)
        sim = F.Sim(d, 1, launch=F.LAUNCH_PER_CYCLE, wg_threads=64, seed=seed)
    else:
        cfg = getattr(configs, name.replace("-", "_").upper())
        d = cfg.design(ctx, g.workload(cfg.workload))
        if isinstance(cfg, configs.Plain):
            sim = F.Sim(d, 1, launch=F.LAUNCH_PER_CYCLE, wg_threads=cfg.threads, seed=seed, stage=cfg.stage,
                        form=F.FORM_PLAIN)
        else:
            sim = F.Sim(d, cfg.instances, launch=F.LAUNCH_PER_CYCLE, wg_threads=cfg.threads, seed=seed,
                        tiles_per_wave=cfg.tiles_per_wave, form=F.FORM_BATCHED)
    sim.step(cycles)
    sim.sync()
    print(json.dumps({"profile_run": name, "layout": sim.layout(), "processes": d.info()["n_processes"],
                      "cycles": cycles}), flush=True)
    sim.close()
    d.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cycles", type=int, default=20_000, help="simulated cycles per step")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="headline only: skip the batched, single-core, 8-tile and served sections")
    ap.add_argument("--retune", action="store_true",
                    help="run the autotuner for the headline instead of its fixed configuration")
    ap.add_argument("--profile-run", default=None,
                    help="a short fixed run for hardware counters: the name of a configuration in "
                         "configs.py written in lower case with dashes (soc48-plain, soc48-batched, "
                         "core-plain, core-batched, ...) or plain-prng (64 one-wave processes of 7 "
                         "independent PRNG fibers)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a device copy of known size (the reference for HBM byte counters)")
    ap.add_argument("--study", choices=["prng", "scaling", "serving", "serving-c3", "packing"], default=None,
                    help="run a study instead of the benchmark (prng: the barrier sweep of Sec. 4.1; "
                         "scaling: strong and weak scaling of Sec. 6.3; serving: the served mix swept "
                         "over the arrival rate, budgets log-uniform [100, 2000]; serving-c3: the same "
                         "from the serving configuration's 10k-cycle floor, budgets log-uniform "
                         "[10k, 100k]; packing: SLB against hypergraph packing, Sec. 6.6)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); "
              "multi-GPU sharding is described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np  # noqa: F401
    import torch
    from paper_2403_04714_amd import fibersim as F
    if not os.path.exists(F.LIB_PATH):
        from paper_2403_04714_amd import build as B
        B.build()
    from paper_2403_04714_amd import configs
    from paper_2403_04714_amd import netgen as g
    from paper_2403_04714_amd import tune

    ctx = F.Context(0)
    if args.profile_run:
        profile_run(F, g, configs, ctx, args.profile_run)
        return
    if args.copy_calibration:
        n = 512 << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read": n, "bytes_written": n, "launches": 3}}), flush=True)
        return
    if args.study:
        if args.study == "prng":
            res = {"study": "prng barrier sweep (Sec. 4.1)", "rows": study_prng(F, g, ctx)}
        elif args.study == "serving":
            res = {"study": "serving sweep", **study_serving(F, g, configs, ctx)}
        elif args.study == "serving-c3":
            res = {"study": "serving sweep from the 10k-cycle floor",
                   **study_serving(F, g, configs, ctx, n_jobs=24, lams=(0.2, 0.5, 1.0), cyc_lo=10_000,
                                   cyc_hi=100_000)}
        elif args.study == "packing":
            res = {"study": "packing: SLB vs hypergraph (Sec. 6.6)", **study_packing(F, g, tune, ctx)}
        else:
            res = {"study": "scaling (Sec. 6.3)", **study_scaling(F, g, tune, ctx, g.STIM_SEED_BASE)}
        print(json.dumps(res), flush=True)
        F.close_all()
        return

    seed = g.STIM_SEED_BASE
    t0 = time.time()
    nl = g.workload("soc48")
    gen_s = time.time() - t0
    cfg = configs.SOC48_PLAIN
    t0 = time.time()
    if args.retune:
        best, _ = tune.tune_plain(ctx, nl, targets=(4096, 8192, 16384), threads=(64,), launches=(F.LAUNCH_GRAPH,),
                                  cycles=500, use_cache=False, packs=PACKS)
        cfg = configs.Plain("soc48", best["pack"], best["target"], best["threads"], best["launch"], best["stage"])
    tune_s = time.time() - t0
    d = cfg.design(ctx, nl)
    info = d.info()
    info["pack"] = cfg.pack
    sim = cfg.sim(d, seed)
    lay = sim.layout()
    stream = ctx.torch_stream
    print(json.dumps({"headline": cfg.label(), "processes": int(info["n_processes"]),
                      "compile_s": round(info["compile_seconds"], 1)}), file=sys.stderr, flush=True)
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
    value = total_cycles / gpu_s
    ms_per_step = gpu_s * 1e3 / args.steps

    bpc, state_bytes = algorithmic_bytes_per_cycle(nl, info["n_live_ops"])
    one_wave = lay["threads"] == 64
    suffix = "" if lay["staged"] else "_g"
    if cfg.launch == F.LAUNCH_PERSISTENT:
        kernel = ("plain_wave_persistent" if one_wave else "plain_persistent") + suffix
        cycles_per_launch = min(args.cycles, 1 << 20)
    else:
        kernel = ("plain_wave_cycle" if one_wave else "plain_cycle") + suffix
        cycles_per_launch = 1
    # average launch duration from the events over the timed region (with
    # one launch per cycle this includes the graph's launch gaps)
    launch_s = gpu_s / total_cycles * cycles_per_launch
    achieved = bpc * cycles_per_launch / launch_s / 1e9
    traffic = profile_record("traffic", kernel, "soc48", int(info["n_processes"]), lay["threads"])
    util = profile_record("util", kernel, "soc48", int(info["n_processes"]), lay["threads"])
    sync = barrier_estimate(sim)
    sim.close()
    sync["empty_design_us_per_cycle"] = empty_design_barrier(F, g, ctx, int(info["n_processes"]), cfg, seed)
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
        "config": {"workload": "48-tile SoC netlist (8 x 6 mesh of single-core tiles), plain form, one instance",
                   "registers": int(nl.n_regs), "word_ops": int(nl.n_comb_ops()),
                   "depth": int(info["max_depth"]), "memories": f"{nl.n_mems} x 4096 x 64b",
                   "instances": 1, "cycles_per_step": args.cycles, "netlist_seed": 1, "mesh_seed": 4,
                   "stimulus_seed": seed},
        "roofline": {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 3),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
                     "traffic": traffic["bytes_per_launch"] if traffic else None,
                     "bytes_per_cycle": bpc, "cycles_per_launch": cycles_per_launch,
                     "launch_us": round(launch_s * 1e6, 3),
                     "valu_lds_utilisation": ({k: util[k] for k in ("valu_busy_frac", "lds_busy_frac",
                                                                    "salu_busy_frac")} if util else None),
                     "note": "algorithmic bytes: 2 x packed state + 24 B per memory + 8 B per live operator"},
        "latency": {"us_per_cycle": round(gpu_s / total_cycles * 1e6, 3),
                    "process_levels": int(info["max_process_levels"]) + 2,
                    "ns_per_level_if_all_latency": round(gpu_s / total_cycles * 1e9 /
                                                          (info["max_process_levels"] + 2), 1)},
        "sync": sync,
        "design": dict(design_stats(info), state_bytes_packed=state_bytes, generate_s=round(gen_s, 2),
                       autotune_s=round(tune_s, 2)),
        "launch": {"config": cfg.label(), "mode": LAUNCH_MODE[cfg.launch], "workgroups": lay["workgroups"],
                   "threads": lay["threads"], "instructions_in_lds": lay["staged"]},
        "wall_s_timed": round(wall, 3),
    }
    d.close()
    if not args.no_extra:
        extra_t0 = time.time()
        out["batched_soc48"] = batched_record(F, ctx, configs.SOC48_BATCHED, nl, 100, 8, seed, plain_rate=value)
        print(json.dumps({"batched_soc48": out["batched_soc48"]}), file=sys.stderr, flush=True)
        core = g.workload("core")
        out["plain_core"] = plain_record(F, ctx, configs.CORE_PLAIN, core, 20_000, 2000, seed, trace=True)
        out["batched_core"] = batched_record(F, ctx, configs.CORE_BATCHED, core, 256, 32, seed,
                                             plain_rate=out["plain_core"]["value"])
        soc8 = g.workload("soc8")
        out["plain_soc8"] = plain_record(F, ctx, configs.SOC8_PLAIN, soc8, 5000, 500, seed)
        out["batched_soc8"] = batched_record(F, ctx, configs.SOC8_BATCHED, soc8, 128, 16, seed,
                                             plain_rate=out["plain_soc8"]["value"])
        out["plain_core_clocks"] = plain_record(F, ctx, configs.CORE_CLOCKS_PLAIN, g.workload("core_clocks"),
                                                5000, 500, seed)
        out["served"] = bench_served(F, g, configs, ctx, n_jobs=24, lam=4.0, inst_hi=1024, cyc_lo=100,
                                     cyc_hi=2000)
        out["extra_sections_s"] = round(time.time() - extra_t0, 1)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(nl, seed)
    F.close_all()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
