"""Writes tests/golden/oracle_refs.json: oracle results of the long parity
runs (see tests/oracle_refs.py for the stored form).

It calls only the CPU oracle (oracle/) and the seeded input generator
(paper_2403_04714_amd/netgen.py, which holds none of the method's
arithmetic).  Instance i of a record runs with stimulus seed
0x5EED0000 + i.  Runs are independent, so they go to a pool of host
threads (the oracle's C calls release the interpreter lock).

    python tests/golden/make_oracle_refs.py [--threads N] [--only NAME,...]

About 10 minutes on 8 host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

from oracle import oracle as O  # noqa: E402
from paper_2403_04714_amd import netgen as g  # noqa: E402

import oracle_refs as R  # noqa: E402

# name: (workload, instance indices, cycles, digest block, memories stored)
RECORDS = {
    # the single core's full 100,000-cycle run
    "core_x1_100k": ("core", [0], 100_000, 1000, True),
    # every instance of the single core batched x1024
    "core_x1024_1000": ("core", list(range(1024)), 1000, 100, False),
    # the 8-tile SoC: one instance, every instance of x256, a longer sample
    "soc8_x1_2000": ("soc8", [0], 2000, 100, True),
    "soc8_x256_500": ("soc8", list(range(256)), 500, 100, False),
    "soc8_sample_1000": ("soc8", [0, 1, 127, 255], 1000, 100, True),
    # the 48-tile SoC: one instance; every instance of x64, memories included
    "soc48_x1_500": ("soc48", [0], 500, 100, True),
    "soc48_x64_1000": ("soc48", list(range(64)), 1000, 100, True),
}
HEAD = 4          # digests kept in the clear per instance (records of <= 4 instances)


def run_one(nl, seed, cycles, mems):
    sim = O.Sim(nl, seed=seed)
    d = sim.step(cycles, digests=True)
    out = {"regs": R.h64(sim.regs()), "outputs": R.h64(sim.outputs())}
    if mems:
        out["mems"] = [R.h64(sim.mem(m)) for m in range(nl.n_mems)]
    return d, out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=min(8, len(os.sched_getaffinity(0))))
    ap.add_argument("--only", default=None)
    args = ap.parse_args()
    names = args.only.split(",") if args.only else list(RECORDS)
    try:
        with open(R.REFS_PATH) as f:
            refs = json.load(f)
    except OSError:
        refs = {}
    nets = {w: g.workload(w) for w in sorted({RECORDS[n][0] for n in names})}
    jobs = []
    for n in names:
        w, insts, cycles, block, mems = RECORDS[n]
        for i in insts:
            jobs.append((n, i))
    # longest runs first, so the pool ends evenly
    cost = {"core": 1, "soc8": 12, "soc48": 95}
    jobs.sort(key=lambda j: -RECORDS[j[0]][2] * cost[RECORDS[j[0]][0]])
    t0 = time.time()
    results = {}

    def work(job):
        n, i = job
        w, insts, cycles, block, mems = RECORDS[n]
        d, out = run_one(nets[w], g.STIM_SEED_BASE + i, cycles, mems)
        out["digest_blocks"] = R.block_hashes(d, block)
        if len(insts) <= 4:
            out["head"] = [f"{int(x):016x}" for x in d[:HEAD]]
        return job, out

    with ThreadPoolExecutor(args.threads) as ex:
        for k, (job, out) in enumerate(ex.map(work, jobs)):
            results[job] = out
            if (k + 1) % 64 == 0 or k + 1 == len(jobs):
                print(f"{k + 1}/{len(jobs)} runs, {time.time() - t0:.0f} s", flush=True)
    for n in names:
        w, insts, cycles, block, mems = RECORDS[n]
        refs[n] = {"name": n, "workload": w, "netlist": R.fingerprint(nets[w]), "seed_base": g.STIM_SEED_BASE,
                   "cycles": cycles, "block": block,
                   "instances": {str(i): results[(n, i)] for i in insts}}
    tmp = R.REFS_PATH + ".tmp"
    with open(tmp, "w") as f:
        json.dump(refs, f, indent=0, sort_keys=True)
    os.replace(tmp, R.REFS_PATH)
    print(f"wrote {R.REFS_PATH} ({len(names)} records, {time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
