"""Parity of the plain form (one instance, level-parallel workgroups) on the
GPU against the oracle: per-cycle digests and full state, bit-exact, across
packings (single process, one fiber per process, SLB merge), launch modes
(persistent with grid barrier, one launch per cycle, hipGraph) and the
circuits with known behaviour."""
import itertools

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
    return F.Context(0)


def say(*a):
    print(*a, flush=True)


def run_both(F, ctx, nl, cycles, pack, target=0, launch=None, threads=0, seed=SEED, chunks=(None,), stage=0):
    launch = F.LAUNCH_PERSISTENT if launch is None else launch
    say(f"case {nl.name}: pack={pack} target={target} launch={launch} threads={threads} stage={stage} "
        f"cycles={cycles}")
    d = F.Design(ctx, nl, pack=pack, target_processes=target)
    s = F.Sim(d, 1, launch=launch, wg_threads=threads, seed=seed, stage=stage)
    s.enable_digest(cycles)
    done = 0
    for c in chunks:
        n = cycles - done if c is None else c
        s.step(n)
        done += n
    assert done == cycles
    dg = s.digests()[:, 0]
    ref = O.Sim(nl, seed=seed)
    rd = ref.step(cycles, digests=True)
    bad = np.nonzero(dg != rd)[0]
    assert bad.size == 0, f"first digest mismatch at cycle {bad[0]} of {cycles}"
    assert np.array_equal(s.regs(), ref.regs())
    assert np.array_equal(s.outputs(), ref.outputs())
    for m in range(nl.n_mems):
        assert np.array_equal(s.mem(m), ref.mem(m)), f"memory {m}"
    return d, s


def test_tiny_single_process_10k_cycles(F, ctx):
    run_both(F, ctx, g.gen_tiny(0), 10_000, F.PACK_SINGLE)


@pytest.mark.parametrize("pack,target", [(1, 0), (0, 8), (0, 33)])
def test_tiny_packings(F, ctx, pack, target):
    run_both(F, ctx, g.gen_tiny(1), 2000, pack, target)


@pytest.mark.parametrize("launch", [2, 3])
def test_tiny_launch_modes(F, ctx, launch):
    run_both(F, ctx, g.gen_tiny(2), 1000, 0, 16, launch=launch, chunks=(3, 130, 500, None))


@pytest.mark.parametrize("threads", [64, 128, 1024])
def test_tiny_workgroup_sizes(F, ctx, threads):
    run_both(F, ctx, g.gen_tiny(3), 1000, 0, 5, threads=threads)


def test_persistent_chunks_and_odd_steps(F, ctx):
    run_both(F, ctx, g.gen_tiny(4), 777, 0, 12, chunks=(1, 2, 3, 100, None))


def small_core(seed=5):
    p = g.CoreParams(n_regs_1=1400, n_regs_32=300, n_regs_64=300, target_ops=20000,
                     mem_depth=256, reg_locality=96)
    return g.gen_core(seed, p)


@pytest.mark.parametrize("target,threads", [(6, 0), (24, 0), (200, 0), (24, 64), (200, 64)])
def test_small_core_with_memories(F, ctx, target, threads):
    """threads 64: one wave per process, the flat chunk loop."""
    run_both(F, ctx, small_core(), 400, 0, target, threads=threads)


def test_oversized_processes_fall_back_to_batched(F, ctx):
    """One process holding 9,000 independent fibers keeps 9,000 next values
    live until its store level, beyond the plain form's 8191 LDS slots: the
    design loads, a plain sim is refused with FSIM_E_CAPACITY, and the
    automatic form runs one instance in the batched form (which stores each
    value right after computing it), matching the oracle."""
    nl = g.prng_array(9000)
    d = F.Design(ctx, nl, pack=F.PACK_SINGLE)
    with pytest.raises(F.FsimError) as e:
        F.Sim(d, 1, form=F.FORM_PLAIN)
    assert e.value.code == F.E_CAPACITY
    s = F.Sim(d, 1, seed=SEED)
    s.enable_digest(50)
    s.step(50)
    ref = O.Sim(nl, seed=SEED)
    assert np.array_equal(s.digests()[:, 0], ref.step(50, digests=True))
    assert np.array_equal(s.regs(), ref.regs())


@pytest.mark.parametrize("launch", [1, 3])
def test_single_wave_launch_modes(F, ctx, launch):
    """The one-wave kernel under the grid barrier and under graph launches,
    with steps that cut graphs and persistent launches unevenly."""
    run_both(F, ctx, g.gen_tiny(6), 700, 0, 9, launch=launch, threads=64, chunks=(1, 64, 129, None))


def test_core_full_size_2000_cycles(F, ctx):
    """The single-core workload at full size (~200k operators, depth 40, two
    4096 x 64 memories), one fiber per register merged to 256 processes;
    2,000 cycles compared per cycle (the oracle needs ~6 ms per cycle)."""
    run_both(F, ctx, g.workload("core"), 2000, 0, 256)


@pytest.mark.parametrize("launch", [1, 2, 3])
def test_single_wave_instructions_from_global(F, ctx, launch):
    """The one-wave kernel reading its instructions from global memory (a
    group of chunks ahead) instead of an LDS copy."""
    run_both(F, ctx, g.gen_tiny(7), 600, 0, 9, launch=launch, threads=64, chunks=(1, 130, None), stage=2)


@pytest.mark.parametrize("target", [24, 200])
def test_small_core_instructions_from_global(F, ctx, target):
    run_both(F, ctx, small_core(), 300, 0, target, launch=3, threads=64, stage=2)


def test_core_full_size_single_wave(F, ctx):
    """The single-core workload at 1024 one-wave processes (the flat chunk
    loop), 1,000 cycles compared per cycle."""
    run_both(F, ctx, g.workload("core"), 1000, 0, 1024, launch=3, threads=64)
    run_both(F, ctx, g.workload("core"), 500, 0, 2048, launch=3, threads=64, stage=2)


@pytest.mark.parametrize("launch,stage,threads", [(3, 1, 64), (3, 2, 64), (1, 1, 64), (1, 2, 64), (3, 0, 256)])
def test_phase_timestamps(F, ctx, launch, stage, threads):
    """Phase timestamps (the traced kernel variants): results stay bit-exact
    with tracing on, then off again, and each workgroup's stamps of a cycle
    are ordered: start <= end of each level <= commit <= cycle end."""
    nl = small_core()
    cycles = 60
    say(f"case trace: launch={launch} stage={stage} threads={threads}")
    d = F.Design(ctx, nl, pack=F.PACK_SLB, target_processes=24)
    s = F.Sim(d, 1, launch=launch, wg_threads=threads, seed=SEED, stage=stage)
    s.enable_digest(2 * cycles)
    s.enable_trace(cycles)
    s.step(cycles)
    tr = s.trace().astype(np.int64)            # [cycles][workgroups][stride]
    s.enable_trace(0)
    s.step(cycles)
    ref = O.Sim(nl, seed=SEED)
    assert np.array_equal(s.digests()[:, 0], ref.step(2 * cycles, digests=True))
    assert np.array_equal(s.regs(), ref.regs())
    start, commit, end = tr[:, :, 0], tr[:, :, -2], tr[:, :, -1]
    assert (start > 0).all() and (commit >= start).all() and (end >= commit).all()
    if threads == 64:
        n_lv = int(d.info()["max_process_levels"])
        for c in range(cycles):
            for w in range(tr.shape[1]):
                row = tr[c, w, 1:min(n_lv, tr.shape[2] - 2)]
                row = row[row != 0]
                assert (np.diff(row) >= 0).all() and (row >= start[c, w]).all() and (row <= commit[c, w]).all()


@pytest.mark.parametrize("target,stage", [(24, 2), (200, 1)])
def test_hypergraph_packing_small_core(F, ctx, target, stage):
    """Hypergraph packing (the alternative of Sec. 6.6) through the one-wave
    kernel, memories included."""
    run_both(F, ctx, small_core(), 300, F.PACK_HYPER, target, launch=3, threads=64, stage=stage)


def test_hypergraph_packing_core_full_size(F, ctx):
    run_both(F, ctx, g.workload("core"), 500, F.PACK_HYPER, 2048, launch=3, threads=64, stage=2)


def _pairs_inputs(n=4):
    pairs = list(itertools.product(range(2**n), repeat=2))
    return pairs, np.array(pairs, np.uint64)


@pytest.mark.parametrize("builder,check", [
    (g.ripple_adder, lambda a, b, r: int(r[0]) == a + b),
    (g.array_multiplier, lambda a, b, r: int(r[0]) == a * b),
    (g.comparators, lambda a, b, r: int(r[0]) == int(a == b) and int(r[1]) == int(a < b)),
])
def test_bruteforce_circuits_explicit_inputs(F, ctx, builder, check):
    nl = builder(4)
    say(f"case {nl.name}: explicit inputs, all 256 pairs")
    pairs, vals = _pairs_inputs()
    for pack in (F.PACK_SINGLE, F.PACK_FIBERS):
        d = F.Design(ctx, nl, pack=pack)
        s = F.Sim(d, 1)
        s.set_inputs(0, vals)
        for (a, b) in pairs:
            s.step(1)
            assert check(a, b, s.regs()), (nl.name, a, b)


def test_closed_forms(F, ctx):
    say("case counters/lfsr/xorshift")
    for w in (1, 8, 64):
        d = F.Design(ctx, g.counter(w))
        s = F.Sim(d, 1)
        s.step(1000)
        assert int(s.regs()[0]) == 1000 % 2**w
    d = F.Design(ctx, g.lfsr(12, [12, 11, 10, 4]), pack=F.PACK_FIBERS)
    s = F.Sim(d, 1)
    r0 = s.regs().copy()
    s.step(2**12 - 1)
    assert np.array_equal(s.regs(), r0)
    d = F.Design(ctx, g.xorshift32())
    s = F.Sim(d, 1)
    s.step(1)
    assert int(s.regs()[0]) == 723471715


def test_explicit_input_window_error(F, ctx):
    nl = g.ripple_adder(4)
    d = F.Design(ctx, nl)
    s = F.Sim(d, 1)
    s.set_inputs(0, np.zeros((10, 2), np.uint64))
    s.step(10)
    with pytest.raises(F.FsimError) as e:
        s.step(1)
    assert e.value.code == F.E_ARG
    s.step(0)


def test_checkpoint_resume(F, ctx):
    """Run N, checkpoint (registers, memories, cycle), restore into a fresh sim,
    run M: equal to an uninterrupted N + M run."""
    nl = small_core(9)
    say("case checkpoint/resume on small core")
    d = F.Design(ctx, nl, target_processes=16)
    a = F.Sim(d, 1, seed=SEED)
    a.step(150)
    regs, mems, cyc = a.regs().copy(), [a.mem(m).copy() for m in range(nl.n_mems)], a.cycle
    a.step(251)
    b = F.Sim(d, 1, seed=SEED)
    b.write_regs(regs)
    for m, v in enumerate(mems):
        b.write_mem(m, v)
    b.set_cycle(cyc)
    b.step(251)
    assert np.array_equal(a.regs(), b.regs())
    for m in range(nl.n_mems):
        assert np.array_equal(a.mem(m), b.mem(m))


def test_context_released_before_its_design_and_sim(F):
    """The caller may release handles in any order: with the context's own
    handle released first, its sim still steps and reads back, the design and
    sim are released afterwards, and a fresh context works with no error
    left behind (a design or sim holds the context until it is released)."""
    nl = g.gen_tiny(seed=8)
    print("case release order: context first", flush=True)
    ctx = F.Context(0)
    d = F.Design(ctx, nl, pack=F.PACK_SLB, target_processes=4)
    s = F.Sim(d, 1, seed=SEED)
    ctx.close()
    s.enable_digest(50)
    s.step(50)
    ref = O.Sim(nl, seed=SEED)
    assert np.array_equal(s.digests()[:, 0], ref.step(50, digests=True))
    s.close()
    d.close()
    ctx2 = F.Context(0)
    d2 = F.Design(ctx2, nl, pack=F.PACK_SLB, target_processes=4)
    s2 = F.Sim(d2, 1, seed=SEED)
    s2.step(10)
    ref2 = O.Sim(nl, seed=SEED)
    ref2.step(10)
    assert np.array_equal(s2.regs(), ref2.regs())
    s2.close()
    d2.close()
    ctx2.close()
