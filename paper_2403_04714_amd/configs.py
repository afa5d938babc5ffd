"""Fixed launch configurations of the measured workloads.

The benchmark times every workload at the configuration listed here, with no
tuning sweep in the timed run, and the parity tests run exactly these
configurations against the oracle.  The values are what the autotuner
(tune.py) settles on for each workload on MI355X; re-running it is a study
of its own (``bench.py --retune``).

A plain configuration: packing policy and target process count (fibers
packed into processes, Sec. 5.1 / Sec. 6.6), threads per workgroup, launch
mode, and where a one-wave workgroup reads its instructions from.  A batched
configuration: the same packing plus instances, threads per workgroup (64 per
tile of 64 instances) and tiles per wave.
"""
from __future__ import annotations

import dataclasses

from . import fibersim as F


@dataclasses.dataclass(frozen=True)
class Plain:
    workload: str
    pack: int
    target: int
    threads: int = 64
    launch: int = F.LAUNCH_GRAPH
    stage: int = F.STAGE_AUTO

    def design(self, ctx, nl):
        return F.Design(ctx, nl, pack=self.pack, target_processes=self.target)

    def sim(self, design, seed=None):
        return F.Sim(design, 1, launch=self.launch, wg_threads=self.threads, seed=seed, stage=self.stage,
                     form=F.FORM_PLAIN)

    def label(self):
        return (f"{PACK_NAMES[self.pack]} packing at target {self.target}, {self.threads} threads, "
                f"{LAUNCH_NAMES[self.launch]} launches, instructions {STAGE_NAMES[self.stage]}")


@dataclasses.dataclass(frozen=True)
class Batched:
    workload: str
    instances: int
    pack: int
    target: int
    threads: int = 64
    tiles_per_wave: int = 1

    def design(self, ctx, nl):
        return F.Design(ctx, nl, pack=self.pack, target_processes=self.target)

    def sim(self, design, seed=None):
        return F.Sim(design, self.instances, launch=F.LAUNCH_GRAPH, wg_threads=self.threads, seed=seed,
                     tiles_per_wave=self.tiles_per_wave, form=F.FORM_BATCHED)

    def label(self):
        return (f"{PACK_NAMES[self.pack]} packing at target {self.target}, {self.threads} threads, "
                f"{self.tiles_per_wave} tile(s) of 64 instances per wave, graph launches")


PACK_NAMES = {F.PACK_SLB: "SLB", F.PACK_FIBERS: "one-fiber", F.PACK_SINGLE: "single", F.PACK_HYPER: "hypergraph"}
LAUNCH_NAMES = {F.LAUNCH_PERSISTENT: "persistent", F.LAUNCH_PER_CYCLE: "per-cycle", F.LAUNCH_GRAPH: "graph"}
STAGE_NAMES = {F.STAGE_AUTO: "auto", F.STAGE_LDS: "staged in LDS", F.STAGE_GLOBAL: "from global memory"}

# the 48-tile SoC, one instance: the headline
SOC48_PLAIN = Plain("soc48", F.PACK_HYPER, 4096, stage=F.STAGE_GLOBAL)
# the 48-tile SoC, 64 instances
SOC48_BATCHED = Batched("soc48", 64, F.PACK_HYPER, 32768)
# the single core, one instance
CORE_PLAIN = Plain("core", F.PACK_HYPER, 2048, stage=F.STAGE_GLOBAL)
# the single core, 1024 instances
CORE_BATCHED = Batched("core", 1024, F.PACK_HYPER, 4096)
# the 8-tile SoC, one instance and 256 instances
SOC8_PLAIN = Plain("soc8", F.PACK_HYPER, 4096, stage=F.STAGE_GLOBAL)
SOC8_BATCHED = Batched("soc8", 256, F.PACK_HYPER, 16384)
# the single core with clock domains, one instance
CORE_CLOCKS_PLAIN = Plain("core_clocks", F.PACK_HYPER, 2048, stage=F.STAGE_GLOBAL)
# served designs (batched form inside the server)
SERVED = (("core", F.PACK_HYPER, 2048), ("soc8", F.PACK_HYPER, 16384))
