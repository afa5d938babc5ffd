"""The autotuner (tune.py) on a reduced core: it times the configurations it
is given and returns the fastest runnable one, and the sim it picks is
bit-exact against the oracle.  The staircase of Sec. 6.3 is why the rate is
measured rather than derived, so whichever configuration wins, its result
must not change."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2403_04714_amd import netgen as g

pytestmark = pytest.mark.gpu

SEED = g.STIM_SEED_BASE


@pytest.fixture(scope="module")
def F():
    from paper_2403_04714_amd import fibersim
    return fibersim


@pytest.fixture(scope="module")
def ctx(F):
    c = F.Context(0)
    yield c
    F.close_all()


def small_core(seed=5):
    p = g.CoreParams(n_regs_1=1400, n_regs_32=300, n_regs_64=300, target_ops=20000,
                     mem_depth=256, reg_locality=96)
    return g.gen_core(seed, p)


def test_tune_plain_then_parity(F, ctx):
    from paper_2403_04714_amd import tune
    nl = small_core()
    print("case tuner: plain, reduced core", flush=True)
    best, trials = tune.tune_plain(ctx, nl, targets=(16, 64), threads=(64, 256),
                                   launches=(F.LAUNCH_PERSISTENT, F.LAUNCH_GRAPH), cycles=200, use_cache=False,
                                   packs=(F.PACK_SLB, F.PACK_HYPER))
    assert trials and best["s_per_cycle"] == min(t["s_per_cycle"] for t in trials)
    assert {t["pack"] for t in trials} == {F.PACK_SLB, F.PACK_HYPER}
    print(f"case tuner: plain picked {best}", flush=True)
    d = F.Design(ctx, nl, pack=best["pack"], target_processes=best["target"])
    s = F.Sim(d, 1, launch=best["launch"], wg_threads=best["threads"], seed=SEED, stage=best["stage"])
    cycles = 400
    s.enable_digest(cycles)
    s.step(cycles)
    ref = O.Sim(nl, seed=SEED)
    rd = ref.step(cycles, digests=True)
    assert np.array_equal(s.digests()[:, 0], rd)
    assert np.array_equal(s.regs(), ref.regs())
    for m in range(nl.n_mems):
        assert np.array_equal(s.mem(m), ref.mem(m))
    s.close()
    d.close()


def test_tune_batched_then_parity(F, ctx):
    from paper_2403_04714_amd import tune
    nl = small_core()
    n_inst = 130
    print("case tuner: batched x130, reduced core", flush=True)
    best, trials = tune.tune_batched(ctx, nl, n_inst, targets=(64, 256), threads=(64, 128), cycles=32,
                                     use_cache=False, tiles=(1, 2), packs=(F.PACK_SLB, F.PACK_HYPER))
    assert trials and best["s_per_cycle"] == min(t["s_per_cycle"] for t in trials)
    assert {t["tiles_per_wave"] for t in trials} == {1, 2}
    print(f"case tuner: batched picked {best}", flush=True)
    d = F.Design(ctx, nl, pack=best["pack"], target_processes=best["target"])
    s = F.Sim(d, n_inst, launch=F.LAUNCH_GRAPH, wg_threads=best["threads"], seed=SEED,
              tiles_per_wave=best["tiles_per_wave"])
    cycles = 150
    s.enable_digest(cycles)
    s.step(cycles)
    dg = s.digests()
    for i in (0, 63, 64, 129):
        ref = O.Sim(nl, seed=SEED + i)
        rd = ref.step(cycles, digests=True)
        assert np.array_equal(dg[:, i], rd), f"instance {i}"
        assert np.array_equal(s.regs(i), ref.regs()), f"instance {i}"
    s.close()
    d.close()
