"""Autotuner: picks the launch configuration of a design by timing short runs.

The simulation rate is not monotone in the number of processes (Parendi
Sec. 6.3: the "staircase" of equal-size stragglers, and Sec. 4: t_sync and
t_comm grow with parallelism while t_comp falls), so the configuration is
measured rather than derived.  Knobs: packing target (processes = workgroups
of the plain kernel), threads per workgroup, launch mode (persistent kernel
with grid barrier, or per-cycle launches captured in a hipGraph).  Results are
cached per (design hash, instances, device name) in a JSON file.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from . import fibersim as F

CACHE = os.environ.get("FSIM_TUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                         "tune_cache.json"))


def design_hash(nl) -> str:
    h = hashlib.sha1()
    for f in ("op", "width", "arg", "imm", "reg_width", "reg_init", "reg_next", "in_width",
              "out_node", "mem_depth", "mem_width", "wp_mem", "wp_en", "wp_addr", "wp_data"):
        h.update(np.ascontiguousarray(getattr(nl, f)).tobytes())
    en = getattr(nl, "reg_en", None)
    if en is not None:
        h.update(b"reg_en" + np.ascontiguousarray(en, np.uint32).tobytes())
    return h.hexdigest()[:16]


def _device_name():
    import torch
    return torch.cuda.get_device_name(0)


def _load_cache():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(c):
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def time_plain(ctx, design, launch, threads, cycles, seed=0x5EED0000, reps=2, stage=F.STAGE_AUTO):
    """Seconds per simulated cycle (best of reps), torch events on ctx's stream."""
    import torch
    s = F.Sim(design, 1, launch=launch, wg_threads=threads, seed=seed, stage=stage)
    s.step(min(200, cycles))
    s.sync()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.torch_stream)
        s.step(cycles)
        e1.record(ctx.torch_stream)
        e1.synchronize()
        s.sync()
        best = min(best, e0.elapsed_time(e1) / 1e3 / cycles)
    del s
    return best


def tune_plain(ctx, nl, targets=(16, 32, 64, 128, 256), threads=(256, 512, 1024),
               launches=(F.LAUNCH_PERSISTENT, F.LAUNCH_GRAPH), cycles=2000, use_cache=True,
               verbose=False, packs=(F.PACK_SLB,)):
    """Returns (best, trials): best = dict(pack, target, threads, launch,
    stage, s_per_cycle)."""
    key = f"plain/{design_hash(nl)}/{'-'.join(map(str, packs))}/{_device_name()}"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return cache[key], []
    trials = []
    best = None
    for pk, t in [(pk, t) for pk in packs for t in targets]:
        try:
            d = F.Design(ctx, nl, pack=pk, target_processes=t)
        except F.FsimError as e:
            if verbose:
                print(f"tune: pack {pk} target {t}: {e}", flush=True)
            continue
        for th in threads:
            # one-wave processes: instructions staged in LDS or read from global memory
            stages = (F.STAGE_LDS, F.STAGE_GLOBAL) if th == 64 else (F.STAGE_AUTO,)
            for la, st in [(la, st) for la in launches for st in stages]:
                try:
                    spc = time_plain(ctx, d, la, th, cycles, stage=st)
                except F.FsimError as e:
                    if verbose:
                        print(f"tune: target {t} threads {th} launch {la} stage {st}: {e}", flush=True)
                    continue
                rec = dict(pack=pk, target=t, processes=d.info()["n_processes"], threads=th, launch=la,
                           stage=st, s_per_cycle=spc)
                trials.append(rec)
                if verbose:
                    print(f"tune: {rec}  ({1/spc/1e3:.1f} kHz)", flush=True)
                if best is None or spc < best["s_per_cycle"]:
                    best = rec
        del d
    if best is None:
        raise RuntimeError("autotuner found no runnable configuration")
    if use_cache:
        cache = _load_cache()
        cache[key] = best
        _save_cache(cache)
    return best, trials


def time_batched(ctx, design, n_inst, threads, cycles, seed=0x5EED0000, reps=2, tiles_per_wave=0):
    """Seconds per simulated cycle of the batched form (all n_inst instances)."""
    import torch
    s = F.Sim(design, n_inst, launch=F.LAUNCH_GRAPH, wg_threads=threads, seed=seed,
              tiles_per_wave=tiles_per_wave)
    s.step(min(64, cycles))
    s.sync()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.torch_stream)
        s.step(cycles)
        e1.record(ctx.torch_stream)
        e1.synchronize()
        s.sync()
        best = min(best, e0.elapsed_time(e1) / 1e3 / cycles)
    del s
    return best


def tune_batched(ctx, nl, n_inst, targets=(256, 512, 1024, 2048), threads=(64, 128, 256),
                 cycles=256, use_cache=True, verbose=False, designs=None, tiles=(1, 2),
                 packs=(F.PACK_SLB,)):
    """Batched-form autotuner: packing policy and target, tiles of 64
    instances per workgroup and per wave.  designs: optional {(pack,
    target): Design} already compiled.  Returns (best, trials); best has
    s_per_cycle for all instances."""
    key = f"batched/{design_hash(nl)}/{n_inst}/{'-'.join(map(str, packs))}/{_device_name()}"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return cache[key], []
    trials, best = [], None
    for pk, t in [(pk, t) for pk in packs for t in targets]:
        try:
            d = designs[(pk, t)] if designs and (pk, t) in designs else \
                F.Design(ctx, nl, pack=pk, target_processes=t)
        except F.FsimError as e:
            if verbose:
                print(f"tune: pack {pk} target {t}: {e}", flush=True)
            continue
        for th, tw in [(th, tw) for th in threads for tw in tiles]:
            if th * tw > 64 * ((n_inst + 63) // 64):
                continue
            try:
                spc = time_batched(ctx, d, n_inst, th, cycles, tiles_per_wave=tw)
            except F.FsimError as e:
                if verbose:
                    print(f"tune: target {t} threads {th} tiles/wave {tw}: {e}", flush=True)
                continue
            rec = dict(pack=pk, target=t, processes=d.info()["n_processes"], threads=th, tiles_per_wave=tw,
                       s_per_cycle=spc, inst_cycles_per_s=n_inst / spc)
            trials.append(rec)
            if verbose:
                print(f"tune: {rec}", flush=True)
            if best is None or spc < best["s_per_cycle"]:
                best = rec
        del d
    if best is None:
        raise RuntimeError("autotuner found no runnable configuration")
    if use_cache:
        cache = _load_cache()
        cache[key] = best
        _save_cache(cache)
    return best, trials
