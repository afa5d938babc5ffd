"""Parity of the batched form (one lane per instance, many independent
stimulus instances in one launch) against the oracle: instance i of a
batched run equals the oracle run with seed_base + i, every cycle (digests)
and in full final state; ragged instance counts, workgroup shapes, launch
modes, explicit per-instance inputs, memories, and batched == plain."""
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


def check_batched(F, ctx, nl, n_inst, cycles, target=0, threads=0, launch=0, full_state=None,
                  chunks=(None,), seed=SEED, digest_insts=None, tiles_per_wave=0, pack=None):
    say(f"case {nl.name}: batched n_inst={n_inst} target={target} threads={threads} "
        f"launch={launch} tiles_per_wave={tiles_per_wave} cycles={cycles}")
    d = F.Design(ctx, nl, pack=F.PACK_SLB if pack is None else pack, target_processes=target)
    s = F.Sim(d, n_inst, launch=launch, wg_threads=threads, seed=seed, tiles_per_wave=tiles_per_wave)
    s.enable_digest(cycles)
    done = 0
    for c in chunks:
        n = cycles - done if c is None else c
        s.step(n)
        done += n
    dg = s.digests()
    insts = range(n_inst) if digest_insts is None else digest_insts
    for i in insts:
        ref = O.Sim(nl, seed=seed + i)
        rd = ref.step(cycles, digests=True)
        bad = np.nonzero(dg[:, i] != rd)[0]
        assert bad.size == 0, f"instance {i}: first digest mismatch at cycle {bad[0]}"
        if full_state is None or i in full_state:
            assert np.array_equal(s.regs(i), ref.regs()), f"instance {i} registers"
            assert np.array_equal(s.outputs(i), ref.outputs()), f"instance {i} outputs"
            for m in range(nl.n_mems):
                assert np.array_equal(s.mem(m, i), ref.mem(m)), f"instance {i} memory {m}"
    return d, s


def test_tiny_ragged_instances(F, ctx):
    check_batched(F, ctx, g.gen_tiny(0), 200, 300, target=16, full_state={0, 63, 64, 199})


@pytest.mark.parametrize("n_inst", [2, 64, 65, 130])
def test_tiny_instance_counts(F, ctx, n_inst):
    check_batched(F, ctx, g.gen_tiny(5), n_inst, 150, target=9, full_state={0, n_inst - 1})


@pytest.mark.parametrize("threads", [64, 128, 256])
def test_workgroup_shapes(F, ctx, threads):
    check_batched(F, ctx, g.gen_tiny(6), 256, 120, target=5, threads=threads, full_state={3, 200})


def test_per_cycle_launches_and_chunks(F, ctx):
    check_batched(F, ctx, g.gen_tiny(7), 96, 200, target=12, launch=2, chunks=(1, 5, 64, None),
                  full_state={95})


def test_graph_launch_chunks(F, ctx):
    check_batched(F, ctx, g.gen_tiny(8), 80, 333, target=7, launch=3, chunks=(7, 128, None),
                  full_state={0, 79})


def small_core(seed=5):
    p = g.CoreParams(n_regs_1=1400, n_regs_32=300, n_regs_64=300, target_ops=20000,
                     mem_depth=256, reg_locality=96)
    return g.gen_core(seed, p)


def test_small_core_memories(F, ctx):
    check_batched(F, ctx, small_core(), 70, 150, target=40, full_state={0, 69})


def test_core_full_size_sampled(F, ctx):
    """Full single-core netlist, 128 instances, 60 cycles: digests of a sample
    of instances every cycle and their full state."""
    check_batched(F, ctx, g.workload("core"), 128, 60, target=512, full_state={0, 127},
                  digest_insts=[0, 1, 77, 127])


# two tiles (128 instances) per wave: instance counts that fill both tiles,
# leave the second tile of the last wave empty (ragged: 1, 3 or 5 tiles), or
# end inside a tile; workgroups of 1, 2 and 4 waves; memories; full size
@pytest.mark.parametrize("n_inst,threads", [(1, 0), (64, 0), (65, 64), (130, 0), (200, 128), (320, 256)])
def test_two_tiles_per_wave(F, ctx, n_inst, threads):
    check_batched(F, ctx, g.gen_tiny(9), n_inst, 140, target=7, threads=threads, tiles_per_wave=2,
                  full_state={0, n_inst - 1})


def test_two_tiles_per_wave_memories_and_chunks(F, ctx):
    check_batched(F, ctx, small_core(), 190, 150, target=40, launch=3, chunks=(3, 64, None),
                  tiles_per_wave=2, full_state={0, 64, 127, 128, 189})


def test_two_tiles_per_wave_core_full_size(F, ctx):
    check_batched(F, ctx, g.workload("core"), 256, 40, target=4096, threads=256, tiles_per_wave=2,
                  full_state={0, 255}, digest_insts=[0, 63, 64, 127, 128, 255])


def test_two_tiles_per_wave_explicit_inputs(F, ctx):
    """Gate-level 4-bit adder with explicit per-instance inputs, 200 instances
    (the last wave's second tile half full)."""
    nl = g.ripple_adder(4)
    d = F.Design(ctx, nl, pack=F.PACK_SINGLE)
    n = 200
    s = F.Sim(d, n, tiles_per_wave=2)
    T = 8
    rng = np.random.default_rng(4)
    vals = rng.integers(0, 16, (T, 2, n)).astype(np.uint64)
    s.set_inputs(0, vals)
    for t in range(T):
        s.step(1)
        for i in (0, 63, 64, 127, 128, 199):
            assert int(s.regs(i)[0]) == int(vals[t, 0, i] + vals[t, 1, i]), (t, i)


def test_hypergraph_packing(F, ctx):
    """Hypergraph packing in the batched form: memories, a ragged instance
    count, and the full single-core design."""
    check_batched(F, ctx, small_core(), 70, 150, target=40, pack=F.PACK_HYPER, full_state={0, 69})
    check_batched(F, ctx, g.workload("core"), 128, 40, target=2048, pack=F.PACK_HYPER, full_state={0, 127},
                  digest_insts=[0, 64, 127])


def test_batched_single_instance_equals_plain(F, ctx):
    nl = small_core(11)
    d = F.Design(ctx, nl, target_processes=30)
    a = F.Sim(d, 1, form=F.FORM_BATCHED, seed=SEED)
    b = F.Sim(d, 1, form=F.FORM_PLAIN, launch=F.LAUNCH_PERSISTENT, seed=SEED)
    a.step(123)
    b.step(123)
    assert np.array_equal(a.regs(), b.regs())
    for m in range(nl.n_mems):
        assert np.array_equal(a.mem(m), b.mem(m))


def test_explicit_inputs_per_instance(F, ctx):
    """Gate-level 4-bit adder, 256 instances, instance i drives pairs (a, b)
    from its own row; every instance's register equals a + b each cycle."""
    nl = g.ripple_adder(4)
    say("case adder4 batched explicit inputs")
    d = F.Design(ctx, nl, pack=F.PACK_SINGLE)
    n = 256
    s = F.Sim(d, n)
    T = 16
    rng = np.random.default_rng(3)
    vals = rng.integers(0, 16, (T, 2, n)).astype(np.uint64)
    s.set_inputs(0, vals)
    for t in range(T):
        s.step(1)
        for i in (0, 1, 63, 64, 200, 255):
            assert int(s.regs(i)[0]) == int(vals[t, 0, i] + vals[t, 1, i]), (t, i)


def test_write_regs_per_instance(F, ctx):
    nl = g.counter(16)
    d = F.Design(ctx, nl)
    s = F.Sim(d, 100)
    s.step(10)
    s.write_regs([1000], 37)
    s.step(5)
    assert int(s.regs(37)[0]) == 1005
    assert int(s.regs(36)[0]) == 15
    assert int(s.regs(99)[0]) == 15
