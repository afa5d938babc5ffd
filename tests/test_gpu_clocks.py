"""Gated and divided clocks (Sec. 5.3) on the GPU, bit-exact against the
oracle: the per-register enables become multiplexers in the compiler, so both
kernel forms run them unchanged.  Small circuits with closed forms, the
random test design with clock domains under several packings, and the full
single-core design with half of its registers on divided or gated clocks, in
the plain form (one instance) and the batched form (many instances)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2403_04714_amd import netgen as g
from tests.test_gpu_batched import check_batched
from tests.test_gpu_plain import run_both

pytestmark = pytest.mark.gpu

SEED = g.STIM_SEED_BASE


@pytest.fixture(scope="module")
def F():
    from paper_2403_04714_amd import fibersim
    return fibersim


@pytest.fixture(scope="module")
def ctx(F):
    return F.Context(0)


@pytest.mark.parametrize("k", [2, 3, 8])
def test_divided_counter_plain(F, ctx, k):
    nl = g.divided_counter(8, k)
    d, s = run_both(F, ctx, nl, 1000, F.PACK_FIBERS)
    assert int(s.regs()[1]) == (1000 // k) % 256


def test_multibit_enable_plain_and_batched(F, ctx):
    """An enable wider than one bit ticks on any non-zero value."""
    from tests.test_oracle_clocks import wide_enable_counter
    nl = wide_enable_counter(5)
    d, s = run_both(F, ctx, nl, 600, F.PACK_FIBERS)
    assert int(s.regs()[1]) == 600 - (600 + 4) // 5
    check_batched(F, ctx, nl, 65, 200, full_state={0, 64})


def test_gated_counter_plain_and_batched(F, ctx):
    nl = g.gated_counter(12)
    run_both(F, ctx, nl, 700, F.PACK_SINGLE)
    check_batched(F, ctx, nl, 70, 300, full_state={0, 69})


@pytest.mark.parametrize("pack,target", [(1, 0), (0, 9), (3, 9)])
def test_clock_domains_tiny_plain(F, ctx, pack, target):
    nl = g.add_clock_domains(g.gen_tiny(4), seed=3)
    run_both(F, ctx, nl, 1500, pack, target)


@pytest.mark.parametrize("launch", [2, 3])
def test_clock_domains_tiny_launch_modes(F, ctx, launch):
    nl = g.add_clock_domains(g.gen_tiny(5), seed=9, divisors=(2, 5))
    run_both(F, ctx, nl, 600, 0, 12, launch=launch, chunks=(1, 7, 200, None))


def test_clock_domains_tiny_batched(F, ctx):
    nl = g.add_clock_domains(g.gen_tiny(6), seed=4)
    check_batched(F, ctx, nl, 130, 200, target=11, full_state={0, 64, 129})


def test_clock_domains_tiny_batched_two_tiles(F, ctx):
    nl = g.add_clock_domains(g.gen_tiny(7), seed=5)
    # one wave per workgroup: two tiles of this design's slots need 40 KiB of LDS
    check_batched(F, ctx, nl, 200, 150, target=6, threads=64, tiles_per_wave=2,
                  full_state={0, 127, 199})


def test_core_with_clock_domains_plain_full_size(F, ctx):
    """The full single-core design, half of its registers on clocks divided
    by 2, 3 and 8 or gated by a stimulus bit: hypergraph packing at the
    benchmark's 2048 processes, instructions from global memory, graph
    launches, 300 cycles."""
    nl = g.workload("core_clocks")
    run_both(F, ctx, nl, 300, F.PACK_HYPER, 2048, launch=F.LAUNCH_GRAPH, threads=64, stage=2)


def test_core_with_clock_domains_batched(F, ctx):
    nl = g.workload("core_clocks")
    check_batched(F, ctx, nl, 96, 40, target=1024, pack=F.PACK_HYPER, full_state={0, 95},
                  digest_insts=[0, 1, 64, 95])
