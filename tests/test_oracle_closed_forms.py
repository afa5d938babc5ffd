"""Whole-cycle semantics against closed forms: a w-bit counter holds
N mod 2^w after N cycles; maximal-length LFSRs (published taps) have period
exactly 2^n - 1; the xorshift32 netlist follows Marsaglia's recurrence (the
PRNG fibers of Parendi Sec. 4.1); two registers that swap alternate (both
take their next values at once, Sec. 3.2)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2403_04714_amd import netgen as g
from tests.conftest import golden_lines


@pytest.mark.parametrize("w", [1, 3, 8, 32, 63, 64])
def test_counter(w):
    sim = O.Sim(g.counter(w))
    done = 0
    for n in (1, 5, 250, 1000):
        sim.step(n - done)
        done = n
        assert int(sim.regs()[0]) == n % 2**w
        assert int(sim.outputs()[0]) == (n - 1) % 2**w   # output of the last cycle


def test_counter_wraps():
    sim = O.Sim(g.counter(4))
    sim.step(16)
    assert int(sim.regs()[0]) == 0
    sim.step(21)
    assert int(sim.regs()[0]) == 37 % 16


def _taps():
    out = {}
    for ln in golden_lines("lfsr_maximal_taps.txt"):
        n, t = ln.split(":")
        out[int(n)] = [int(x) for x in t.split()]
    return out


@pytest.mark.parametrize("n", list(range(3, 17)))
def test_lfsr_period(n):
    taps = _taps()[n]
    sim = O.Sim(g.lfsr(n, taps))
    s0 = sim.regs().copy()
    period = 2**n - 1
    d = sim.step(period, digests=True)
    d0 = sim.digest()
    # back at the start after exactly 2^n - 1 cycles ...
    assert np.array_equal(sim.regs(), s0)
    # ... and never before (the digest of the start state appears once)
    assert int(np.count_nonzero(d == np.uint64(d0))) == 1


def test_lfsr_nonmaximal_taps_have_short_period():
    # taps (4, 2) are not primitive: the period must be shorter than 15
    sim = O.Sim(g.lfsr(4, [4, 2]))
    s0 = sim.regs().copy()
    for k in range(1, 16):
        sim.step(1)
        if np.array_equal(sim.regs(), s0):
            break
    assert k < 15


def test_xorshift32_matches_marsaglia():
    seed = int(golden_lines("xorshift32.txt")[0].split()[1])
    first = int(golden_lines("xorshift32.txt")[1].split()[1])
    sim = O.Sim(g.xorshift32(seed))
    sim.step(1)
    assert int(sim.regs()[0]) == first
    # 10^4 further cycles against the software recurrence
    y = first
    for _ in range(10_000):
        y ^= (y << 13) & 0xFFFFFFFF
        y ^= y >> 17
        y ^= (y << 5) & 0xFFFFFFFF
    sim.step(10_000)
    assert int(sim.regs()[0]) == y


def test_swap_pair_alternates():
    sim = O.Sim(g.swap_pair(16, 0x1234, 0xBEEF))
    for k in range(1, 8):
        sim.step(1)
        r = [int(x) for x in sim.regs()]
        assert r == ([0xBEEF, 0x1234] if k % 2 else [0x1234, 0xBEEF])
