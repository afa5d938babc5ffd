#!/usr/bin/env python3
"""Benchmark: simulated cycles/s x instances of the per-cycle BSP evaluation
of a fiber-partitioned netlist (Parendi's method) on one MI355X.

One step = one pass of the hot path over one batch of synthetic input: the
single-core workload (about 20k registers, 200k word operators, depth 40,
two 4096 x 64 memories, one instance) simulated for 100,000 cycles with the
on-device stimulus.  Compilation (fiber extraction, packing, encoding) and
autotuning happen once, before the timed region.

Prints ONE JSON line.  Also reports the roofline of the dominant kernel and
the oracle's CPU rate on a bounded sample, and, measured in the same run at
bounded cycle counts: the batched form (many independent stimulus instances
per launch) on the single-core and 8-tile SoC workloads, the plain form on
the 8-tile SoC, and a served Poisson stream of jobs with p50/p99 latency.
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

# packing policies the autotuner tries: bottom-up SLB (Sec. 5.1) and the
# hypergraph alternative (Sec. 6.6)
PACKS = (0, 3)
PACK_NAMES = {0: "slb", 1: "fibers", 2: "single", 3: "hypergraph"}


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


def measured_traffic(kernel, workload, processes, threads):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the same counters over a
    device copy of known size), or None when there is no summary for this
    configuration or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.md")
    try:
        with open(path) as f:
            line = next(l for l in f if l.startswith("traffic_json: "))
        rec = json.loads(line[len("traffic_json: "):])
    except (OSError, StopIteration, ValueError):
        return None
    if (rec.get("kernel_source") != kernel_source_hash() or rec.get("processes") != processes
            or rec.get("threads") != threads):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(nl, seed, budget_s=15.0):
    """The oracle as it stands, single thread, on a bounded prefix: 20
    warm-up cycles, then blocks of 100 cycles until budget_s has passed."""
    from oracle import oracle as orc
    sim = orc.Sim(nl, seed=seed)
    sim.step(20)
    n, dt = 0, 0.0
    t0 = time.perf_counter()
    while dt < budget_s:
        sim.step(100)
        n += 100
        dt = time.perf_counter() - t0
    return dict(value=n / dt, unit="instance-cycles/s", cores=1, kind="oracle",
                sample=f"{nl.name}: 1 instance, cycles 20..{20 + n} of the same stimulus, "
                       f"single-threaded C oracle ({dt:.1f} s)")


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


def bench_batched(F, g, tune, ctx, name, n_inst, targets, threads, cycles, warm, seed):
    """Batched form: n_inst instances in one launch per cycle (hipGraph),
    packing target and threads per workgroup autotuned."""
    nl = g.workload(name)
    t0 = time.time()
    designs = {(pk, t): F.Design(ctx, nl, pack=pk, target_processes=t) for pk in PACKS for t in targets}
    compile_s = time.time() - t0
    best, _ = tune.tune_batched(ctx, nl, n_inst, targets=targets, threads=threads, cycles=32,
                                use_cache=False, designs=designs, packs=PACKS)
    d = designs.pop((best["pack"], best["target"]))
    designs.clear()
    tw = best.get("tiles_per_wave", 1)
    sim = F.Sim(d, n_inst, launch=F.LAUNCH_GRAPH, wg_threads=best["threads"], seed=seed, tiles_per_wave=tw)
    gpu_s = time_sim(sim, ctx.torch_stream, cycles, warm)
    info = d.info()
    bpc, _ = algorithmic_bytes_per_cycle(nl, info["n_live_ops"], n_inst)
    achieved = bpc / (gpu_s / cycles) / 1e9
    lay = sim.layout()
    bi = d.batched_info()
    out = {"workload": f"{nl.name} x{n_inst}", "instances": n_inst, "cycles": cycles,
           "value": round(n_inst * cycles / gpu_s, 1), "unit": "instance-cycles/s",
           "us_per_cycle": round(gpu_s / cycles * 1e6, 2),
           "roofline": {"bound": "alu", "kernel": "batched_cycle2" if tw == 2 else "batched_cycle",
                        "hbm_achieved_GBs": round(achieved, 2),
                        "hbm_frac": round(achieved / HBM_PEAK_GBS, 5), "bytes_per_cycle": bpc},
           "pack": PACK_NAMES[best["pack"]], "processes": int(info["n_processes"]),
           "dup_process": round(info["dup_process"], 4),
           "workgroups": lay["workgroups"], "threads": lay["threads"], "tiles_per_wave": tw,
           "wave_lds_bytes": int(bi["wave_lds_bytes"]) * tw, "instructions": int(bi["n_instr"]),
           "compile_s": round(compile_s, 2)}
    del sim, d
    return out


def bench_plain_tuned(F, g, tune, ctx, name, targets, threads, cycles, warm, seed):
    """Plain form, one instance, packing target and threads autotuned (graph
    launches: beyond a hundred or so workgroups the per-cycle launch is the
    cheaper barrier)."""
    nl = g.workload(name)
    t0 = time.time()
    best, _ = tune.tune_plain(ctx, nl, targets=targets, threads=threads, launches=(F.LAUNCH_GRAPH,),
                              cycles=500, use_cache=False, packs=PACKS)
    tune_s = time.time() - t0
    d = F.Design(ctx, nl, pack=best["pack"], target_processes=best["target"])
    sim = F.Sim(d, 1, launch=best["launch"], wg_threads=best["threads"], seed=seed,
                stage=best.get("stage", F.STAGE_AUTO))
    gpu_s = time_sim(sim, ctx.torch_stream, cycles, warm)
    info = d.info()
    lay = sim.layout()
    out = {"workload": f"{nl.name} x1", "instances": 1, "cycles": cycles,
           "value": round(cycles / gpu_s, 1), "unit": "instance-cycles/s",
           "us_per_cycle": round(gpu_s / cycles * 1e6, 2), "pack": PACK_NAMES[best["pack"]],
           "processes": int(info["n_processes"]),
           "workgroups": lay["workgroups"], "threads": lay["threads"],
           "process_levels": int(info["max_process_levels"]) + 2,
           "dup_process": round(info["dup_process"], 4), "compile_s": round(info["compile_seconds"], 2),
           "autotune_s": round(tune_s, 1)}
    del sim, d
    return out


def barrier_estimate(F, sim, cycles=24):
    """Per-cycle cost outside the slowest workgroup's compute, from the phase
    timestamps: cycle period minus the slowest workgroup's compute span
    (start to commit).  In graph mode this is the launch gap; in persistent
    mode the grid barrier."""
    import numpy as np
    sim.enable_trace(cycles)
    sim.step(cycles)
    tr = sim.trace().astype(np.int64)
    stride = tr.shape[2]
    period = np.diff(tr[:, :, 0].min(axis=1)) * 10 / 1000
    comp = (tr[:, :, stride - 2] - tr[:, :, 0]).max(axis=1) * 10 / 1000
    return {"period_us": round(float(np.median(period)), 3),
            "slowest_compute_us": round(float(np.median(comp[1:])), 3),
            "barrier_us": round(float(np.median(period) - np.median(comp[1:])), 3)}


def bench_soc48(F, g, ctx, seed, plain_cfgs=((8192, 64),), batched_target=32768, cycles=200,
                batched_packs=(0, 3)):
    """The 48-tile SoC: compile statistics (duplication overhead), the plain
    form at one instance and the batched form at 64 instances.  A plain
    config is (target, threads[, stage[, pack]])."""
    nl = g.workload("soc48")
    out = {"workload": nl.name, "registers": int(nl.n_regs), "word_ops": int(nl.n_comb_ops()),
           "memories": int(nl.n_mems), "plain": [], "batched": None}
    designs = {}
    for cfg in plain_cfgs:
        target, threads = cfg[0], cfg[1]
        stage = cfg[2] if len(cfg) > 2 else F.STAGE_AUTO
        pack = cfg[3] if len(cfg) > 3 else F.PACK_SLB
        if (pack, target) not in designs:
            designs[(pack, target)] = F.Design(ctx, nl, pack=pack, target_processes=target)
        d = designs[(pack, target)]
        info = d.info()
        sim = F.Sim(d, 1, launch=F.LAUNCH_GRAPH, wg_threads=threads, seed=seed, stage=stage)
        gpu_s = time_sim(sim, ctx.torch_stream, cycles, 20)
        rec = {"pack": PACK_NAMES[pack], "processes": int(info["n_processes"]), "threads": threads,
               "instructions_in_lds": bool(sim.layout()["staged"]),
               "value": round(cycles / gpu_s, 1), "unit": "instance-cycles/s",
               "us_per_cycle": round(gpu_s / cycles * 1e6, 2), "compile_s": round(info["compile_seconds"], 1),
               "dup_fiber": round(info["dup_fiber"], 4), "dup_process": round(info["dup_process"], 4),
               "duplicated_ops": int(round((info["dup_process"] - 1) * info["n_live_ops"])),
               "process_levels": int(info["max_process_levels"]) + 2}
        rec.update(barrier_estimate(F, sim))
        out["plain"].append(rec)
        print(json.dumps({"soc48_plain": rec}), file=sys.stderr, flush=True)
        del sim
    out["batched"] = []
    for bp in batched_packs:
        if (bp, batched_target) not in designs:
            designs[(bp, batched_target)] = F.Design(ctx, nl, pack=bp, target_processes=batched_target)
        d = designs[(bp, batched_target)]
        sim = F.Sim(d, 64, launch=F.LAUNCH_GRAPH, seed=seed)
        bc = max(8, cycles // 10)
        gpu_s = time_sim(sim, ctx.torch_stream, bc, 4)
        info = d.info()
        bpc, _ = algorithmic_bytes_per_cycle(nl, info["n_live_ops"], 64)
        out["batched"].append({"instances": 64, "pack": PACK_NAMES[bp], "processes": int(info["n_processes"]),
                               "cycles": bc, "value": round(64 * bc / gpu_s, 1), "unit": "instance-cycles/s",
                               "us_per_cycle": round(gpu_s / bc * 1e6, 1),
                               "hbm_achieved_GBs": round(bpc / (gpu_s / bc) / 1e9, 2),
                               "dup_process": round(info["dup_process"], 4),
                               "wave_lds_bytes": int(d.batched_info()["wave_lds_bytes"])})
        del sim
    print(json.dumps({"soc48_batched": out["batched"]}), file=sys.stderr, flush=True)
    return out


def bench_served(F, g, ctx, n_jobs, lam, inst_hi, cyc_lo, cyc_hi):
    """Served Poisson stream over the single-core and 8-tile SoC designs."""
    from paper_2403_04714_amd import serve
    designs = [F.Design(ctx, g.workload("core"), pack=F.PACK_HYPER, target_processes=2048),
               F.Design(ctx, g.workload("soc8"), pack=F.PACK_HYPER, target_processes=16384)]
    jobs = serve.draw_jobs(n_jobs, designs, inst_lo=1, inst_hi=inst_hi, cyc_lo=cyc_lo, cyc_hi=cyc_hi)
    arr = serve.arrivals(n_jobs, lam=lam)
    srv = F.Server(ctx, 64 << 30, quantum_cycles=256)
    recs, summ = serve.run(srv, designs, jobs, arr, timeout_s=600)
    st = srv.stats()
    srv.close()
    return {"designs": [f"core ({designs[0].info()['n_processes']} processes, hypergraph packing)",
                        f"soc8 ({designs[1].info()['n_processes']} processes, hypergraph packing)"], "jobs": n_jobs,
            "arrival_rate_per_s": lam, "instances": f"log-uniform [1, {inst_hi}]",
            "cycles": f"log-uniform [{cyc_lo}, {cyc_hi}]",
            "completed": summ["completed"], "p50_s": round(summ["p50_s"], 4), "p99_s": round(summ["p99_s"], 4),
            "mean_s": round(summ["mean_s"], 4), "wall_s": round(summ["wall_s"], 3),
            "value": round(summ["instance_cycles_per_s"], 1), "unit": "instance-cycles/s",
            "total_work_instance_cycles": int(summ["total_work_instance_cycles"]),
            "quanta": int(st["quanta"]), "device_busy_s": round(st["busy_seconds"], 3)}


def study_serving(F, g, ctx, n_jobs=24, lams=(1.0, 2.0, 4.0, 8.0, 16.0, 64.0)):
    """The serving mix swept over the mean arrival rate: p50/p99 of (done -
    arrival) and aggregate instance-cycles/s per rate, one fresh server per
    rate over the same compiled designs and the same job draw."""
    from paper_2403_04714_amd import serve
    designs = [F.Design(ctx, g.workload("core"), pack=F.PACK_HYPER, target_processes=2048),
               F.Design(ctx, g.workload("soc8"), pack=F.PACK_HYPER, target_processes=16384)]
    jobs = serve.draw_jobs(n_jobs, designs, inst_lo=1, inst_hi=1024, cyc_lo=100, cyc_hi=2000)
    work = sum(j["instances"] * j["cycles"] for j in jobs)
    rows = []
    for lam in lams:
        srv = F.Server(ctx, 64 << 30, quantum_cycles=256)
        recs, summ = serve.run(srv, designs, jobs, serve.arrivals(n_jobs, lam=lam), timeout_s=600)
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
    return {"jobs": n_jobs, "total_work_instance_cycles": int(work),
            "designs": [f"core ({designs[0].info()['n_processes']} processes, hypergraph packing)",
                        f"soc8 ({designs[1].info()['n_processes']} processes, hypergraph packing)"],
            "instances": "log-uniform [1, 1024]", "cycles": "log-uniform [100, 2000]", "rows": rows}


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
                del sim
            del d
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
                del d
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
                best = (us, st, sim)
            else:
                del sim
        us, st, sim = best
        rec = {"processes": int(info["n_processes"]), "us_per_cycle": round(us, 2),
               "rate_khz": round(1e3 / us, 2), "instructions_in_lds": st == F.STAGE_LDS,
               "dup_process": round(info["dup_process"], 4), "max_process_cost": int(info["max_process_cost"])}
        rec.update(trace_split(sim))
        strong.append(rec)
        print(json.dumps({"strong": rec}), file=sys.stderr, flush=True)
        del sim, d
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
        del sim, d
    return {"strong": strong, "weak": weak}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cycles", type=int, default=100_000, help="cycles per step")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--retune", action="store_true", help="ignore the autotuner cache")
    ap.add_argument("--soc48", action="store_true",
                    help="also measure the 48-tile SoC (compiling it takes about a minute)")
    ap.add_argument("--soc48-plain", default="16384:64:2:0,16384:64:2:3,8192:64:2:3",
                    help="plain configurations for --soc48, target:threads[:stage[:pack]][,...] "
                         "(stage 1: instructions in LDS, 2: from global memory; pack 0 SLB, 3 "
                         "hypergraph)")
    ap.add_argument("--plain-config", default=None,
                    help="target:threads:launch[:stage[:pack]] for the headline plain run, skipping "
                         "the autotuner (launch 1 persistent, 3 graph; stage 1 LDS, 2 global; pack 0 "
                         "SLB, 3 hypergraph); used for profiling runs")
    ap.add_argument("--profile-run", choices=["batched-core", "plain-core", "plain-prng"], default=None,
                    help="a short fixed run for hardware counters (per-cycle launches, hypergraph "
                         "packing): batched single-core x1024 at target 4096, plain single-core at "
                         "target 2048 in one-wave processes reading instructions from global memory, "
                         "or 64 one-wave "
                         "processes of 7 independent PRNG fibers")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a device copy of known size (the reference for HBM byte counters)")
    ap.add_argument("--study", choices=["prng", "scaling", "serving", "packing"], default=None,
                    help="run a study instead of the benchmark (prng: the barrier sweep of Sec. 4.1; "
                         "scaling: strong and weak scaling of Sec. 6.3; serving: the served mix "
                         "swept over the arrival rate; packing: SLB against hypergraph packing, "
                         "Sec. 6.6)")
    ap.add_argument("--no-extra", action="store_true",
                    help="headline only: skip the batched, 8-tile plain and served sections")
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

    if args.profile_run:
        ctx = F.Context(0)
        if args.profile_run == "batched-core":
            d = F.Design(ctx, g.workload("core"), pack=F.PACK_HYPER, target_processes=4096)
            sim = F.Sim(d, 1024, launch=F.LAUNCH_PER_CYCLE, wg_threads=64, seed=g.STIM_SEED_BASE)
        elif args.profile_run == "plain-core":
            d = F.Design(ctx, g.workload("core"), pack=F.PACK_HYPER, target_processes=2048)
            sim = F.Sim(d, 1, launch=F.LAUNCH_PER_CYCLE, wg_threads=64, seed=g.STIM_SEED_BASE,
                        stage=F.STAGE_LDS)
        else:
            import numpy as np
            d = F.Design(ctx, g.prng_array(7 * 64), partition=np.arange(7 * 64, dtype=np.uint32) // 7)
            sim = F.Sim(d, 1, launch=F.LAUNCH_PER_CYCLE, wg_threads=64, seed=g.STIM_SEED_BASE)
        sim.step(32)
        sim.sync()
        print(json.dumps({"profile_run": args.profile_run, "layout": sim.layout(),
                          "processes": d.info()["n_processes"], "cycles": 32}), flush=True)
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
    if args.study == "prng":
        ctx = F.Context(0)
        print(json.dumps({"study": "prng barrier sweep (Sec. 4.1)", "rows": study_prng(F, g, ctx)}), flush=True)
        return
    if args.study == "serving":
        ctx = F.Context(0)
        print(json.dumps({"study": "serving sweep", **study_serving(F, g, ctx)}), flush=True)
        return
    if args.study == "packing":
        ctx = F.Context(0)
        print(json.dumps({"study": "packing: SLB vs hypergraph (Sec. 6.6)",
                          **study_packing(F, g, tune, ctx)}), flush=True)
        return
    if args.study == "scaling":
        ctx = F.Context(0)
        print(json.dumps({"study": "scaling (Sec. 6.3)",
                          **study_scaling(F, g, tune, ctx, g.STIM_SEED_BASE)}), flush=True)
        return

    seed = g.STIM_SEED_BASE
    t0 = time.time()
    nl = g.workload("core")
    gen_s = time.time() - t0
    ctx = F.Context(0)
    t0 = time.time()
    if args.plain_config:
        vals = [int(v) for v in args.plain_config.split(":")]
        best = {"target": vals[0], "threads": vals[1], "launch": vals[2],
                "stage": vals[3] if len(vals) > 3 else F.STAGE_AUTO,
                "pack": vals[4] if len(vals) > 4 else F.PACK_SLB}
    else:
        best, _ = tune.tune_plain(ctx, nl, targets=(512, 1024, 2048, 4096), threads=(64, 256),
                                  launches=(F.LAUNCH_GRAPH,), cycles=2000, use_cache=not args.retune,
                                  packs=PACKS)
    tune_s = time.time() - t0
    d = F.Design(ctx, nl, pack=best["pack"], target_processes=best["target"])
    info = d.info()
    sim = F.Sim(d, 1, launch=best["launch"], wg_threads=best["threads"], seed=seed,
                stage=best.get("stage", F.STAGE_AUTO))
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
    one_wave = lay["threads"] == 64
    suffix = "" if lay["staged"] else "_g"
    if best["launch"] == F.LAUNCH_PERSISTENT:
        kernel = ("plain_wave_persistent" if one_wave else "plain_persistent") + suffix
        cycles_per_launch = min(args.cycles, 1 << 20)
        launch_s = gpu_s / args.steps * cycles_per_launch / args.cycles
    else:
        kernel = ("plain_wave_cycle" if one_wave else "plain_cycle") + suffix
        cycles_per_launch = 1
        launch_s = gpu_s / total_cycles       # upper bound: includes the graph's launch gaps
    achieved = bpc * cycles_per_launch / launch_s / 1e9
    traffic = measured_traffic(kernel, "core", info["n_processes"], lay["threads"])
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
                     "traffic": traffic,
                     "bytes_per_cycle": bpc, "cycles_per_launch": cycles_per_launch,
                     "launch_ms": round(launch_s * 1e3, 4),
                     "note": "latency-bound: levels x per-level latency + barrier; see latency"},
        "latency": {"us_per_cycle": round(gpu_s / total_cycles * 1e6, 3),
                    "process_levels": int(info["max_process_levels"]) + 2,
                    "ns_per_level_if_all_latency": round(gpu_s / total_cycles * 1e9 /
                                                          (info["max_process_levels"] + 2), 1)},
        "design": {"pack": PACK_NAMES[best["pack"]], "processes": int(info["n_processes"]),
                   "dup_fiber": round(info["dup_fiber"], 4),
                   "dup_process": round(info["dup_process"], 4), "live_ops": int(info["n_live_ops"]),
                   "max_fiber_cost": int(info["max_fiber_cost"]),
                   "max_process_cost": int(info["max_process_cost"]),
                   "program_bytes": int(info["program_bytes"]),
                   "compile_s": round(info["compile_seconds"], 2), "generate_s": round(gen_s, 2),
                   "autotune_s": round(tune_s, 2), "state_bytes_packed": state_bytes},
        "launch": {"mode": {1: "persistent", 2: "per_cycle", 3: "graph"}[best["launch"]],
                   "workgroups": lay["workgroups"], "threads": lay["threads"],
                   "instructions_in_lds": lay["staged"],
                   # the same run again: bench.py --plain-config <this>
                   "plain_config": f"{best['target']}:{best['threads']}:{best['launch']}:"
                                   f"{F.STAGE_LDS if lay['staged'] else F.STAGE_GLOBAL}:{best['pack']}"},
        "wall_s_timed": round(wall, 3),
    }
    if not args.no_extra:
        del sim
        extra_t0 = time.time()
        out["batched"] = [
            bench_batched(F, g, tune, ctx, "core", 1024, (2048, 4096, 8192), (64, 256), 512, 64, seed),
            bench_batched(F, g, tune, ctx, "soc8", 256, (16384, 32768), (64, 256), 256, 32, seed),
        ]
        out["plain_soc8"] = bench_plain_tuned(F, g, tune, ctx, "soc8", (1024, 2048, 4096), (64, 256),
                                              5000, 500, seed)
        # the single-core design with half of its registers on gated or divided clocks
        out["plain_core_clocks"] = bench_plain_tuned(F, g, tune, ctx, "core_clocks", (1024, 2048, 4096),
                                                     (64,), 5000, 500, seed)
        out["served"] = bench_served(F, g, ctx, n_jobs=24, lam=4.0, inst_hi=1024, cyc_lo=100, cyc_hi=2000)
        out["extra_sections_s"] = round(time.time() - extra_t0, 1)
    if args.soc48:
        cfgs = tuple(tuple(int(v) for v in c.split(":")) for c in args.soc48_plain.split(","))
        out["soc48"] = bench_soc48(F, g, ctx, seed, plain_cfgs=cfgs)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(nl, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
