"""The 48-tile SoC (8 x 6 mesh, about 9.4M operators, 960k registers, 96
memories of 4096 x 64) at full size on the GPU against the oracle: the plain
form with one instance and the batched form with 64 instances, every cycle's
digest, registers and outputs of every instance, and every memory of a fixed
sample of instances, over a short run (the oracle needs about a tenth of a
second per cycle at this size; instances run in host threads).  Compilation
alone takes about a minute on the host."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2403_04714_amd import netgen as g

from oracle_pool import run_instances

pytestmark = pytest.mark.gpu

SEED = g.STIM_SEED_BASE
SAMPLE = (0, 31, 63)


@pytest.fixture(scope="module")
def F():
    from paper_2403_04714_amd import fibersim
    return fibersim


@pytest.fixture(scope="module")
def soc48(F):
    print("case soc48: generate and compile (8192 processes)", flush=True)
    nl = g.workload("soc48")
    ctx = F.Context(0)
    d = F.Design(ctx, nl, pack=F.PACK_SLB, target_processes=8192)
    info = d.info()
    print(f"case soc48: {info['n_processes']} processes, D_f {info['dup_fiber']:.3f}, "
          f"D_p {info['dup_process']:.3f}, compile {info['compile_seconds']:.1f} s", flush=True)
    return nl, ctx, d


@pytest.mark.timeout(900)
def test_soc48_plain_one_instance(F, soc48):
    nl, ctx, d = soc48
    cycles = 6
    print("case soc48: plain x1, graph launches, 64 threads", flush=True)
    s = F.Sim(d, 1, launch=F.LAUNCH_GRAPH, wg_threads=64, seed=SEED)
    s.enable_digest(cycles)
    s.step(cycles)
    ref = O.Sim(nl, seed=SEED)
    rd = ref.step(cycles, digests=True)
    assert np.array_equal(s.digests()[:, 0], rd)
    assert np.array_equal(s.regs(), ref.regs())
    assert np.array_equal(s.outputs(), ref.outputs())
    for m in (0, 47, 95):
        assert np.array_equal(s.mem(m), ref.mem(m)), f"memory {m}"


@pytest.mark.timeout(900)
def test_soc48_batched_64(F, soc48):
    nl, ctx, d = soc48
    cycles = 3
    print("case soc48: batched x64", flush=True)
    s = F.Sim(d, 64, launch=F.LAUNCH_GRAPH, seed=SEED)
    s.enable_digest(cycles)
    s.step(cycles)
    dg = s.digests()
    print("case soc48: oracle, 64 instances", flush=True)
    refs = run_instances(nl, [SEED + i for i in range(64)], cycles)
    for i, (rd, rr, ro, _) in enumerate(refs):
        assert np.array_equal(dg[:, i], rd), f"instance {i}"
        assert np.array_equal(s.regs(i), rr), f"instance {i} registers"
        assert np.array_equal(s.outputs(i), ro), f"instance {i} outputs"
    refs = run_instances(nl, [SEED + i for i in SAMPLE], cycles, mems=range(nl.n_mems))
    for i, (_, _, _, rm) in zip(SAMPLE, refs):
        for m, v in rm.items():
            assert np.array_equal(s.mem(m, i), v), f"instance {i} memory {m}"
