"""Oracle runs of many independent instances in host threads.

Instances of the oracle share no state, and its C calls release the Python
interpreter lock, so one thread per instance runs them side by side.  Test
infrastructure only, like the oracle itself."""
import os
from concurrent.futures import ThreadPoolExecutor

from oracle import oracle as O


def workers(cap: int = 16) -> int:
    return max(1, min(cap, len(os.sched_getaffinity(0))))


def run_instances(nl, seeds, cycles, mems=(), cap=16):
    """For each seed: (per-cycle digests, final registers, final outputs,
    {m: final memory m for m in mems}) after `cycles` cycles."""
    def one(seed):
        ref = O.Sim(nl, seed=seed)
        d = ref.step(cycles, digests=True)
        return d, ref.regs(), ref.outputs(), {m: ref.mem(m) for m in mems}

    with ThreadPoolExecutor(workers(cap)) as ex:
        return list(ex.map(one, seeds))
