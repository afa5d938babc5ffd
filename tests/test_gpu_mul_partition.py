"""Two inputs of the problem statement that the seeded workloads do not
exercise, on the GPU against the oracle:

- word-level multipliers (the optional MUL operator) at widths 1, 7, 32, 33
  and 64, where products wrap past 64 bits and are masked back, in the
  plain and the batched form;
- fiber partitions supplied by the caller (Sec. 3.2: the design is loaded
  "with its fiber partition"): the independent PRNG fibers of the
  synchronization experiment of Sec. 4.1 with 7 fibers per process, and a
  random valid partition of a reduced core with memories (processes merged
  at random from the one-fiber-per-process packing, so every memory's
  readers stay with its write ports).  Fiber-partitioned evaluation must
  equal the monolithic oracle whatever the partition (Sec. 3.2)."""
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


def check_plain(F, nl, d, cycles, launch, threads=64, stage=0):
    s = F.Sim(d, 1, launch=launch, wg_threads=threads, seed=SEED, stage=stage, form=F.FORM_PLAIN)
    s.enable_digest(cycles)
    s.step(cycles)
    ref = O.Sim(nl, seed=SEED)
    rd = ref.step(cycles, digests=True)
    bad = np.nonzero(s.digests()[:, 0] != rd)[0]
    assert bad.size == 0, f"{nl.name}: first digest mismatch at cycle {bad[0]}"
    assert np.array_equal(s.regs(), ref.regs())
    assert np.array_equal(s.outputs(), ref.outputs())
    for m in range(nl.n_mems):
        assert np.array_equal(s.mem(m), ref.mem(m)), f"memory {m}"
    s.close()


def check_batched(F, nl, d, n_inst, cycles, probe):
    s = F.Sim(d, n_inst, launch=F.LAUNCH_GRAPH, seed=SEED, form=F.FORM_BATCHED)
    s.enable_digest(cycles)
    s.step(cycles)
    dg = s.digests()
    for i in probe:
        ref = O.Sim(nl, seed=SEED + i)
        rd = ref.step(cycles, digests=True)
        bad = np.nonzero(dg[:, i] != rd)[0]
        assert bad.size == 0, f"{nl.name} instance {i}: first digest mismatch at cycle {bad[0]}"
        assert np.array_equal(s.regs(i), ref.regs()), f"instance {i}"
        assert np.array_equal(s.outputs(i), ref.outputs()), f"instance {i}"
    s.close()


@pytest.mark.parametrize("pack", ["single", "fibers", "slb"])
def test_mul_plain(F, ctx, pack):
    nl = g.mul_mix()
    p = {"single": F.PACK_SINGLE, "fibers": F.PACK_FIBERS, "slb": F.PACK_SLB}[pack]
    print(f"case mul_mix plain, {pack} packing", flush=True)
    d = F.Design(ctx, nl, pack=p, target_processes=4)
    for launch in (F.LAUNCH_PER_CYCLE, F.LAUNCH_GRAPH):
        check_plain(F, nl, d, 300, launch)
    d.close()


def test_mul_batched(F, ctx):
    nl = g.mul_mix()
    print("case mul_mix batched x70", flush=True)
    d = F.Design(ctx, nl, pack=F.PACK_SLB, target_processes=4)
    check_batched(F, nl, d, 70, 300, (0, 1, 63, 64, 69))
    d.close()


def test_partition_prng_array(F, ctx):
    """The Sec. 4.1 workload as the barrier sweep runs it: n independent
    xorshift fibers, 7 per process, given as the caller's partition."""
    k, G = 7, 64
    nl = g.prng_array(k * G)
    part = np.arange(k * G, dtype=np.uint32) // k
    print("case partition: prng array, 7 fibers per process", flush=True)
    d = F.Design(ctx, nl, partition=part)
    assert d.info()["n_processes"] == G
    stp, _, _ = d.partition()
    assert np.array_equal(stp, part)
    for launch in (F.LAUNCH_PERSISTENT, F.LAUNCH_GRAPH):
        check_plain(F, nl, d, 500, launch)
    check_batched(F, nl, d, 130, 200, (0, 64, 129))
    d.close()


def small_core(seed=5):
    p = g.CoreParams(n_regs_1=1400, n_regs_32=300, n_regs_64=300, target_ops=20000,
                     mem_depth=256, reg_locality=96)
    return g.gen_core(seed, p)


@pytest.mark.parametrize("k", [8, 40])
def test_partition_random_merge(F, ctx, k):
    nl = small_core()
    fib = F.Design(None, nl, pack=F.PACK_FIBERS)
    stp, _, _ = fib.partition()
    n_fib = int(stp.max()) + 1
    rng = np.random.default_rng(100 + k)
    merge = rng.integers(0, k, n_fib)
    ids, part = np.unique(merge[stp], return_inverse=True)
    part = part.astype(np.uint32)
    print(f"case partition: reduced core, {n_fib} one-fiber processes merged at random into {len(ids)}",
          flush=True)
    d = F.Design(ctx, nl, partition=part)
    assert d.info()["n_processes"] == len(ids)
    check_plain(F, nl, d, 300, F.LAUNCH_GRAPH, threads=64, stage=F.STAGE_GLOBAL)
    check_plain(F, nl, d, 300, F.LAUNCH_PER_CYCLE, threads=256)
    check_batched(F, nl, d, 65, 120, (0, 64))
    d.close()
    fib.close()
