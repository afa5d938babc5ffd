"""The 48-tile SoC (8 x 6 mesh, 9.45M operators, 960,576 registers, 96
memories of 4096 x 64) at full size on the GPU, at the benchmark's own
launch configurations (configs.SOC48_PLAIN, the headline, and
configs.SOC48_BATCHED), against oracle results stored by
tests/golden/make_oracle_refs.py (the oracle needs about 0.1-0.4 s per cycle
at this size, so the long runs are computed once on the host):

- plain, one instance: every cycle's digest over 500 cycles, then the
  registers, outputs and all 96 memories;
- batched, 64 instances: every instance's per-cycle digests over 1,000
  cycles, then its registers, outputs and all 96 memories.

Compiling the design takes about a minute on the host."""
import numpy as np
import pytest

import oracle_refs as R
from paper_2403_04714_amd import netgen as g

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module")
def F():
    from paper_2403_04714_amd import fibersim
    return fibersim


@pytest.fixture(scope="module")
def soc48(F):
    print("case soc48: generate", flush=True)
    nl = g.workload("soc48")
    ctx = F.Context(0)
    yield nl, ctx
    F.close_all()


@pytest.mark.timeout(900)
def test_soc48_plain_headline_config(F, soc48):
    from paper_2403_04714_amd import configs
    nl, ctx = soc48
    rec = R.load("soc48_x1_500")
    R.check_netlist(rec, nl)
    cfg = configs.SOC48_PLAIN
    print(f"case soc48 plain x1: compile ({cfg.label()})", flush=True)
    d = cfg.design(ctx, nl)
    s = cfg.sim(d, g.STIM_SEED_BASE)
    print(f"case soc48 plain x1: {d.info()['n_processes']} processes, {s.layout()}, {rec['cycles']} cycles",
          flush=True)
    s.enable_digest(rec["cycles"])
    s.step(rec["cycles"])
    R.compare_instance(rec, 0, digests=s.digests()[:, 0], regs=s.regs(), outputs=s.outputs(),
                       mems={m: s.mem(m) for m in range(nl.n_mems)})
    s.close()
    d.close()


@pytest.mark.timeout(900)
def test_soc48_batched_64_config(F, soc48):
    from paper_2403_04714_amd import configs
    nl, ctx = soc48
    rec = R.load("soc48_x64_1000")
    R.check_netlist(rec, nl)
    cfg = configs.SOC48_BATCHED
    print(f"case soc48 batched x64: compile ({cfg.label()})", flush=True)
    d = cfg.design(ctx, nl)
    s = cfg.sim(d, g.STIM_SEED_BASE)
    print(f"case soc48 batched x64: {d.info()['n_processes']} processes, {s.layout()}, {rec['cycles']} cycles",
          flush=True)
    s.enable_digest(rec["cycles"])
    s.step(rec["cycles"])
    dg = s.digests()
    for i in range(cfg.instances):
        R.compare_instance(rec, i, digests=dg[:, i], regs=s.regs(i), outputs=s.outputs(i),
                           mems={m: s.mem(m, i) for m in range(nl.n_mems)})
    s.close()
    d.close()
