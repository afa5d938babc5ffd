"""The 8-tile SoC (eight copies of the single-core netlist on a 2 x 4 mesh of
registered 32-bit links, 1.57M operators and 16 memories of 4096 x 64) at
full size on the GPU, at the benchmark's launch configurations
(configs.SOC8_PLAIN and configs.SOC8_BATCHED), against oracle results stored
by tests/golden/make_oracle_refs.py:

- plain, one instance: every cycle's digest over 2,000 cycles, then the
  registers, outputs and every memory;
- batched, 256 instances: every instance's per-cycle digests, registers and
  outputs over the first 500 cycles, then instances {0, 1, 127, 255} over
  1,000 cycles with every memory;
- and, against the oracle run live, the plain form under bottom-up SLB
  packing at 4096 processes (the other packing policy) for 300 cycles."""
import numpy as np
import pytest

import oracle_refs as R
from oracle import oracle as O
from paper_2403_04714_amd import netgen as g

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
    nl = g.workload("soc8")
    ctx = F.Context(0)
    yield nl, ctx
    F.close_all()


@pytest.mark.timeout(600)
def test_soc8_plain_config(F, soc8):
    from paper_2403_04714_amd import configs
    nl, ctx = soc8
    rec = R.load("soc8_x1_2000")
    R.check_netlist(rec, nl)
    cfg = configs.SOC8_PLAIN
    d = cfg.design(ctx, nl)
    s = cfg.sim(d, SEED)
    print(f"case soc8 plain x1: {cfg.label()}, {d.info()['n_processes']} processes, {s.layout()}", flush=True)
    s.enable_digest(rec["cycles"])
    s.step(rec["cycles"])
    R.compare_instance(rec, 0, digests=s.digests()[:, 0], regs=s.regs(), outputs=s.outputs(),
                       mems={m: s.mem(m) for m in range(nl.n_mems)})
    s.close()
    d.close()


@pytest.mark.timeout(600)
def test_soc8_plain_slb_live_oracle(F, soc8):
    nl, ctx = soc8
    cycles = 300
    d = F.Design(ctx, nl, pack=F.PACK_SLB, target_processes=4096)
    s = F.Sim(d, 1, launch=F.LAUNCH_GRAPH, wg_threads=64, seed=SEED, stage=F.STAGE_GLOBAL)
    print(f"case soc8 plain x1 SLB: {d.info()['n_processes']} processes, {s.layout()}", flush=True)
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
    s.close()
    d.close()


@pytest.mark.timeout(600)
def test_soc8_batched_256_config(F, soc8):
    from paper_2403_04714_amd import configs
    nl, ctx = soc8
    first, sample = R.load("soc8_x256_500"), R.load("soc8_sample_1000")
    R.check_netlist(first, nl)
    cfg = configs.SOC8_BATCHED
    d = cfg.design(ctx, nl)
    s = cfg.sim(d, SEED)
    print(f"case soc8 batched x256: {cfg.label()}, {d.info()['n_processes']} processes, {s.layout()}",
          flush=True)
    s.enable_digest(sample["cycles"])
    s.step(first["cycles"])
    dg = s.digests()
    for i in range(cfg.instances):
        R.compare_instance(first, i, digests=dg[:first["cycles"], i], regs=s.regs(i), outputs=s.outputs(i))
    print(f"case soc8 batched x256: instances {SAMPLE} to cycle {sample['cycles']}", flush=True)
    s.step(sample["cycles"] - first["cycles"])
    dg = s.digests()
    for i in SAMPLE:
        R.compare_instance(sample, i, digests=dg[:, i], regs=s.regs(i), outputs=s.outputs(i),
                           mems={m: s.mem(m, i) for m in range(nl.n_mems)})
    s.close()
    d.close()
