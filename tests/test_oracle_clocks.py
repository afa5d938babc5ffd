"""Pins of the oracle's gated and divided clocks (Sec. 5.3, Limitations: one
top clock plus any number of gated or divided ones), read as a per-register
enable of the top clock.

- closed forms: a counter on a clock divided by k holds floor(t / k) after
  t cycles; a counter gated by an input bit holds the prefix sum of that bit;
- time dilation: an LFSR of maximal length (taps from the published table)
  moved wholesale onto a clock divided by k visits, at cycle t, the state the
  undivided LFSR has at cycle floor(t / k), and holds it in between;
- special cases: an enable that is constantly 1 is the top clock, one that is
  constantly 0 freezes the register at its initial value, and a multi-bit
  enable ticks on any non-zero value (not on its low bit);
- BSP: evaluating every fiber (or a random grouping of fibers) on its own
  gives the monolithic result, so the enable belongs to the register's cone;
  a fiber that left the enable out would miss an operand and fail.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2403_04714_amd import netgen as g
from tests.conftest import golden_lines


def lfsr_taps():
    out = {}
    for ln in golden_lines("lfsr_maximal_taps.txt"):
        n, t = ln.split(":")
        out[int(n)] = [int(x) for x in t.split()]
    return out


@pytest.mark.parametrize("w,k", [(8, 2), (8, 3), (4, 7), (16, 8), (3, 255)])
def test_divided_counter_closed_form(w, k):
    nl = g.divided_counter(w, k)
    s = O.Sim(nl)
    for t in range(1, 3 * k + 300):
        s.step(1)
        r = s.regs()
        assert int(r[0]) == t % k, t
        assert int(r[1]) == (t // k) % (1 << w), t


def test_gated_counter_prefix_sum():
    nl = g.gated_counter(6)
    rng = np.random.default_rng(11)
    bits = rng.integers(0, 2, (500, 1)).astype(np.uint64)
    s = O.Sim(nl)
    s.set_inputs(0, bits)
    total = 0
    for t in range(500):
        s.step(1)
        total += int(bits[t, 0])
        assert int(s.regs()[0]) == total % 64, t


def test_gated_counter_with_stimulus_bit():
    """The enable also sees the seeded stimulus: the counter counts the cycles
    whose stimulus word for port 0 is odd (the port is 1 bit wide)."""
    nl = g.gated_counter(16)
    s = O.Sim(nl, seed=99)
    s.step(400)
    want = sum(O.stim(99, 0, t) & 1 for t in range(400))
    assert int(s.regs()[0]) == want


@pytest.mark.parametrize("n,k", [(5, 2), (7, 3), (9, 4)])
def test_divided_lfsr_is_time_dilated(n, k):
    plain = g.lfsr(n, lfsr_taps()[n])
    slow = g.add_clock_domains(plain, divisors=(k,), n_gated=0, frac=1.0)
    assert slow.meta["gated_regs"] == n
    T = (1 << n) + 5
    a, b = O.Sim(plain), O.Sim(slow)
    states = [a.regs().copy()]
    for _ in range(T):
        a.step(1)
        states.append(a.regs().copy())
    for t in range(1, k * T + 1):
        b.step(1)
        assert np.array_equal(b.regs()[:n], states[t // k]), t
    # the undivided LFSR is maximal: its period is 2^n - 1 (a check on the taps)
    first = [tuple(x) for x in states[: (1 << n)]]
    assert len(set(first[:-1])) == (1 << n) - 1 and first[-1] == first[0]


def with_const_enable(nl, value):
    """nl with one extra CONST node of the given value as every register's enable."""
    op = np.append(nl.op, np.uint8(g.OPS["CONST"]))
    width = np.append(nl.width, np.uint8(1))
    arg = np.vstack([nl.arg, np.full((1, 3), g.NONE, np.uint32)])
    imm = np.append(nl.imm, np.uint64(value))
    en = np.full(nl.n_regs, len(nl.op), np.uint32)
    import dataclasses
    return dataclasses.replace(nl, op=op, width=width, arg=arg, imm=imm, reg_en=en)


def test_enable_one_is_top_clock_and_zero_freezes():
    nl = g.gen_tiny(3)
    ref = O.Sim(nl, seed=5)
    d_ref = ref.step(200, digests=True)
    one = O.Sim(with_const_enable(nl, 1), seed=5)
    assert np.array_equal(one.step(200, digests=True), d_ref)
    assert np.array_equal(one.outputs(), ref.outputs())
    zero = O.Sim(with_const_enable(nl, 0), seed=5)
    zero.step(50)
    assert np.array_equal(zero.regs(), nl.reg_init)
    # an enable array of all NONE is the same as no array at all
    import dataclasses
    none = O.Sim(dataclasses.replace(nl, reg_en=np.full(nl.n_regs, g.NONE, np.uint32)), seed=5)
    assert np.array_equal(none.step(200, digests=True), d_ref)


def test_enable_out_of_range_is_rejected():
    import dataclasses
    nl = g.gen_tiny(0)
    en = np.full(nl.n_regs, g.NONE, np.uint32)
    en[3] = nl.n_nodes
    with pytest.raises(O.OracleError):
        O.Sim(dataclasses.replace(nl, reg_en=en))


@pytest.mark.parametrize("groups", [0, 5, 17])
def test_partitioned_with_clock_domains_equals_monolithic(groups):
    nl = g.add_clock_domains(g.gen_tiny(4), seed=3)
    assert nl.meta["gated_regs"] > 0
    n_sinks = nl.n_sinks
    if groups == 0:
        stp = np.arange(n_sinks, dtype=np.uint32)         # one fiber per process
    else:
        stp = np.random.default_rng(groups).integers(0, groups, n_sinks).astype(np.uint32)
    a, b = O.Sim(nl, seed=8), O.Sim(nl, seed=8)
    da = a.step(300, digests=True)
    db = b.step_partitioned(300, stp, digests=True)
    assert np.array_equal(da, db)
    assert np.array_equal(a.outputs(), b.outputs())


def test_clock_domains_change_the_trajectory():
    """Guard against a transform that silently did nothing: the gated design
    leaves the top-clock design's trajectory within a few cycles."""
    base = g.gen_tiny(4)
    nl = g.add_clock_domains(base, seed=3)
    a, b = O.Sim(base, seed=8), O.Sim(nl, seed=8)
    a.step(20)
    b.step(20)
    assert not np.array_equal(a.regs(), b.regs()[: base.n_regs])


def wide_enable_counter(k, w=12):
    """A counter whose enable is an 8-bit divider's whole value (not one bit):
    it ticks in every cycle whose divider value is non-zero."""
    b = g.Builder()
    d = b.add_reg(8, 0)
    r = b.add_reg(w, 0)
    wrap = b.op2("EQ", b.reg(d), b.const(8, k - 1))
    b.set_next(d, b.mux(wrap, b.const(8, 0), b.op2("ADD", b.reg(d), b.const(8, 1)), w=8))
    b.set_next(r, b.op2("ADD", b.reg(r), b.const(w, 1)))
    b.set_enable(r, b.reg(d))
    return b.build(name=f"wide_enable_counter{k}")


@pytest.mark.parametrize("k", [2, 5, 9])
def test_enable_is_any_nonzero_value(k):
    """The enable is 'non-zero', not 'bit 0': with the divider's value as
    enable (multi-bit, even values included) the counter misses exactly the
    cycles whose divider value is 0, i.e. t - ceil(t / k) ticks in t cycles."""
    nl = wide_enable_counter(k)
    s = O.Sim(nl)
    for t in range(1, 4 * k + 100):
        s.step(1)
        assert int(s.regs()[1]) == t - (t + k - 1) // k, t
