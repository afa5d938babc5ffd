"""The 8-tile SoC (eight copies of the single-core netlist on a 2 x 4 mesh of
registered 32-bit links, about 1.6M operators and 16 memories of 4096 x 64)
at full size on the GPU against the oracle, in the launch configurations
the benchmark's tuner settles on for it:

- plain, one instance: 4096 one-wave processes reading their instructions
  from global memory, graph launches; every cycle's digest over 1,000
  cycles, then registers, outputs and every memory;
- batched, 256 instances: 32768 processes, 64 threads; every instance's
  per-cycle digests, registers and outputs over the first 12 cycles, then a
  fixed sample of instances over 200 cycles with every memory.

The oracle needs about 20 ms per cycle at this size; instances run in host
threads."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2403_04714_amd import netgen as g

from oracle_pool import run_instances

pytestmark = pytest.mark.gpu

SEED = g.STIM_SEED_BASE
SAMPLE = (0, 1, 127, 255)


@pytest.fixture(scope="module")
def F():
    from paper_2403_04714_amd import fibersim
    return fibersim


@pytest.fixture(scope="module")
def soc8(F):
    print("case soc8: generate", flush=True)
    return g.workload("soc8"), F.Context(0)


@pytest.mark.timeout(600)
def test_soc8_plain_one_instance(F, soc8):
    nl, ctx = soc8
    d = F.Design(ctx, nl, pack=F.PACK_SLB, target_processes=4096)
    cycles = 1000
    s = F.Sim(d, 1, launch=F.LAUNCH_GRAPH, wg_threads=64, seed=SEED, stage=F.STAGE_GLOBAL)
    lay = s.layout()
    print(f"case soc8: plain x1, {d.info()['n_processes']} processes, {lay}", flush=True)
    assert lay["threads"] == 64 and not lay["staged"]
    s.enable_digest(cycles)
    s.step(cycles)
    ref = O.Sim(nl, seed=SEED)
    rd = ref.step(cycles, digests=True)
    bad = np.nonzero(s.digests()[:, 0] != rd)[0]
    assert bad.size == 0, f"first digest mismatch at cycle {bad[0]} of {cycles}"
    assert np.array_equal(s.regs(), ref.regs())
    assert np.array_equal(s.outputs(), ref.outputs())
    for m in range(nl.n_mems):
        assert np.array_equal(s.mem(m), ref.mem(m)), f"memory {m}"


@pytest.mark.timeout(600)
def test_soc8_batched_256(F, soc8):
    nl, ctx = soc8
    d = F.Design(ctx, nl, pack=F.PACK_SLB, target_processes=32768)
    n_inst, first, cycles = 256, 12, 200
    s = F.Sim(d, n_inst, launch=F.LAUNCH_GRAPH, wg_threads=64, seed=SEED)
    print(f"case soc8: batched x{n_inst}, {d.info()['n_processes']} processes, {s.layout()}", flush=True)
    s.enable_digest(cycles)
    s.step(first)
    s.sync()
    regs = [s.regs(i) for i in range(n_inst)]
    outs = [s.outputs(i) for i in range(n_inst)]
    print(f"case soc8: oracle, {n_inst} instances x {first} cycles", flush=True)
    refs = run_instances(nl, [SEED + i for i in range(n_inst)], first)
    dg = s.digests()
    for i, (rd, rr, ro, _) in enumerate(refs):
        bad = np.nonzero(dg[:first, i] != rd)[0]
        assert bad.size == 0, f"instance {i}: first digest mismatch at cycle {bad[0]}"
        assert np.array_equal(regs[i], rr), f"instance {i} registers"
        assert np.array_equal(outs[i], ro), f"instance {i} outputs"
    s.step(cycles - first)
    print(f"case soc8: oracle, instances {SAMPLE} x {cycles} cycles", flush=True)
    refs = run_instances(nl, [SEED + i for i in SAMPLE], cycles, mems=range(nl.n_mems))
    dg = s.digests()
    for i, (rd, rr, ro, rm) in zip(SAMPLE, refs):
        bad = np.nonzero(dg[:, i] != rd)[0]
        assert bad.size == 0, f"instance {i}: first digest mismatch at cycle {bad[0]}"
        assert np.array_equal(s.regs(i), rr), f"instance {i} registers"
        assert np.array_equal(s.outputs(i), ro), f"instance {i} outputs"
        for m, v in rm.items():
            assert np.array_equal(s.mem(m, i), v), f"instance {i} memory {m}"
