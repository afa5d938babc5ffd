"""The single-core design (20,000 registers, about 197k operators, two
4096 x 64 memories) at the benchmark's launch configurations
(configs.CORE_PLAIN and configs.CORE_BATCHED), against oracle results stored
by tests/golden/make_oracle_refs.py:

- plain, one instance: every cycle's digest over all 100,000 cycles of the
  configuration, then the registers, outputs and both memories;
- batched, 1024 instances: every instance's per-cycle digests, registers and
  outputs over 1,000 cycles."""
import pytest

import oracle_refs as R
from paper_2403_04714_amd import netgen as g

pytestmark = pytest.mark.gpu

SEED = g.STIM_SEED_BASE


@pytest.fixture(scope="module")
def F():
    from paper_2403_04714_amd import fibersim
    return fibersim


@pytest.fixture(scope="module")
def core(F):
    nl = g.workload("core")
    ctx = F.Context(0)
    yield nl, ctx
    F.close_all()


@pytest.mark.timeout(600)
def test_core_plain_config_100k_cycles(F, core):
    from paper_2403_04714_amd import configs
    nl, ctx = core
    rec = R.load("core_x1_100k")
    R.check_netlist(rec, nl)
    cfg = configs.CORE_PLAIN
    d = cfg.design(ctx, nl)
    s = cfg.sim(d, SEED)
    print(f"case core plain x1: {cfg.label()}, {d.info()['n_processes']} processes, {s.layout()}, "
          f"{rec['cycles']} cycles", flush=True)
    s.enable_digest(rec["cycles"])
    for _ in range(rec["cycles"] // 10_000):
        s.step(10_000)
    R.compare_instance(rec, 0, digests=s.digests()[:, 0], regs=s.regs(), outputs=s.outputs(),
                       mems={m: s.mem(m) for m in range(nl.n_mems)})
    s.close()
    d.close()


@pytest.mark.timeout(600)
def test_core_batched_1024_config(F, core):
    from paper_2403_04714_amd import configs
    nl, ctx = core
    rec = R.load("core_x1024_1000")
    R.check_netlist(rec, nl)
    cfg = configs.CORE_BATCHED
    d = cfg.design(ctx, nl)
    s = cfg.sim(d, SEED)
    print(f"case core batched x1024: {cfg.label()}, {d.info()['n_processes']} processes, {s.layout()}",
          flush=True)
    s.enable_digest(rec["cycles"])
    s.step(rec["cycles"])
    dg = s.digests()
    for i in range(cfg.instances):
        R.compare_instance(rec, i, digests=dg[:, i], regs=s.regs(i), outputs=s.outputs(i))
    s.close()
    d.close()
