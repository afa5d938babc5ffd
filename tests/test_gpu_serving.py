"""Serving on the GPU: a job's results are the same alone and in a mix of
jobs of other designs, sizes and arrival times (continuous batching), and
equal to the oracle; a seeded Poisson stream completes with latencies."""
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2403_04714_amd import netgen as g
from paper_2403_04714_amd import serve

pytestmark = pytest.mark.gpu

SEED = g.STIM_SEED_BASE


@pytest.fixture(scope="module")
def F():
    from paper_2403_04714_amd import fibersim
    return fibersim


@pytest.fixture(scope="module")
def ctx(F):
    return F.Context(0)


def small_core(seed=5):
    p = g.CoreParams(n_regs_1=1400, n_regs_32=300, n_regs_64=300, target_ops=20000,
                     mem_depth=256, reg_locality=96)
    return g.gen_core(seed, p)


@pytest.fixture(scope="module")
def designs(F, ctx):
    nl_a, nl_b = small_core(), g.gen_tiny(0)
    return (nl_a, F.Design(ctx, nl_a, target_processes=64)), (nl_b, F.Design(ctx, nl_b, target_processes=8))


def results(srv, job, d, insts):
    return {i: srv.result(job, i, d) for i in insts}


def test_alone_equals_in_mix(F, ctx, designs):
    (nl_a, da), (nl_b, db) = designs
    insts = [0, 33, 69]
    print("case serving: job A alone", flush=True)
    srv = F.Server(ctx, 8 << 30, quantum_cycles=64)
    a = srv.submit(da, 70, 300, SEED)
    srv.wait(a, 120)
    alone = results(srv, a, da, insts)
    srv.close()
    print("case serving: job A in a mix", flush=True)
    srv = F.Server(ctx, 8 << 30, quantum_cycles=64)
    b = srv.submit(db, 200, 1000, SEED + 1000)
    time.sleep(0.01)
    a2 = srv.submit(da, 70, 300, SEED)
    c = srv.submit(da, 5, 50, SEED + 77)
    time.sleep(0.02)
    e = srv.submit(db, 1, 777, SEED + 5)
    for j in (a2, b, c, e):
        srv.wait(j, 120)
        assert srv.poll(j)["state"] == F.JOB_DONE
    mix = results(srv, a2, da, insts)
    for i in insts:
        assert np.array_equal(alone[i][0], mix[i][0]) and np.array_equal(alone[i][1], mix[i][1])
    # against the oracle
    for i in (0, 69):
        ref = O.Sim(nl_a, seed=SEED + i)
        ref.step(300)
        assert np.array_equal(mix[i][0], ref.regs())
        assert np.array_equal(mix[i][1], ref.outputs())
    # the other jobs against standalone batched sims of the same parameters
    for job, d, nl, n, cyc, seed, probe in ((b, db, nl_b, 200, 1000, SEED + 1000, [0, 199]),
                                             (c, da, nl_a, 5, 50, SEED + 77, [4]),
                                             (e, db, nl_b, 1, 777, SEED + 5, [0])):
        s = F.Sim(d, n, form=F.FORM_BATCHED, seed=seed)
        s.step(cyc)
        for i in probe:
            r, o = srv.result(job, i, d)
            assert np.array_equal(r, s.regs(i)) and np.array_equal(o, s.outputs(i))
    st = srv.stats()
    assert st["completed"] == 4 and st["hbm_used"] == 0
    srv.close()


def test_poisson_stream(F, ctx, designs):
    (nl_a, da), (nl_b, db) = designs
    jobs = serve.draw_jobs(24, [da, db], inst_lo=1, inst_hi=256, cyc_lo=100, cyc_hi=2000)
    arr = serve.arrivals(24, lam=200.0)
    print("case serving: 24-job Poisson stream", flush=True)
    srv = F.Server(ctx, 4 << 30, quantum_cycles=128)
    recs, summ = serve.run(srv, [da, db], jobs, arr, timeout_s=300)
    assert summ["completed"] == 24
    assert summ["p50_s"] <= summ["p99_s"]
    # spot-check one job against the oracle
    r0 = recs[0]
    nl = (nl_a, nl_b)[r0["design"]]
    regs, _ = srv.result(r0["id"], 0, (da, db)[r0["design"]])
    ref = O.Sim(nl, seed=r0["seed"])
    ref.step(r0["cycles"])
    assert np.array_equal(regs, ref.regs())
    srv.close()


def test_alone_equals_in_mix_served_designs(F, ctx):
    """The benchmark's served designs (configs.SERVED: the single core and
    the 8-tile SoC under hypergraph packing) in one batched_multi launch per
    tick: a single-core job gives the same registers and outputs alone and
    in a mix with an 8-tile SoC job and a second single-core job, and both
    designs' jobs equal the oracle."""
    from paper_2403_04714_amd import configs
    nets = {w: g.workload(w) for w, _, _ in configs.SERVED}
    print("case serving: compile the served designs", flush=True)
    ds = {w: F.Design(ctx, nets[w], pack=pk, target_processes=t) for w, pk, t in configs.SERVED}
    core, soc8 = ds["core"], ds["soc8"]
    insts = [0, 41, 69]
    print("case serving: single-core job alone", flush=True)
    srv = F.Server(ctx, 32 << 30, quantum_cycles=64)
    a = srv.submit(core, 70, 300, SEED)
    srv.wait(a, 300)
    alone = results(srv, a, core, insts)
    srv.close()
    print("case serving: single-core job in a mix with an 8-tile SoC job", flush=True)
    srv = F.Server(ctx, 32 << 30, quantum_cycles=64)
    b = srv.submit(soc8, 16, 100, SEED + 500)
    a2 = srv.submit(core, 70, 300, SEED)
    time.sleep(0.01)
    c = srv.submit(core, 3, 130, SEED + 900)
    for j in (a2, b, c):
        srv.wait(j, 300)
        assert srv.poll(j)["state"] == F.JOB_DONE
    mix = results(srv, a2, core, insts)
    for i in insts:
        assert np.array_equal(alone[i][0], mix[i][0]) and np.array_equal(alone[i][1], mix[i][1]), i
    for i in (0, 69):
        ref = O.Sim(nets["core"], seed=SEED + i)
        ref.step(300)
        assert np.array_equal(mix[i][0], ref.regs()) and np.array_equal(mix[i][1], ref.outputs()), i
    for i in (0, 15):
        ref = O.Sim(nets["soc8"], seed=SEED + 500 + i)
        ref.step(100)
        r, o = srv.result(b, i, soc8)
        assert np.array_equal(r, ref.regs()) and np.array_equal(o, ref.outputs()), f"soc8 instance {i}"
    ref = O.Sim(nets["core"], seed=SEED + 900 + 2)
    ref.step(130)
    r, o = srv.result(c, 2, core)
    assert np.array_equal(r, ref.regs()) and np.array_equal(o, ref.outputs())
    srv.close()
    for d in ds.values():
        d.close()
