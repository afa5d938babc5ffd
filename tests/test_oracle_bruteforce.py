"""Brute force over tiny gate-level circuits built only from 1-bit
AND/OR/XOR/NOT (plus the shift/and plumbing that splits a port into bits):
every one of the 2^8 input pairs against integer +, *, == and <.  This pins
the 1-bit logic and the netlist plumbing (operand order, register update,
explicit inputs) of the oracle."""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_2403_04714_amd import netgen as g


def run_pairs(nl, n=4):
    pairs = list(itertools.product(range(2**n), repeat=2))
    vals = np.array(pairs, np.uint64)
    sim = O.Sim(nl)
    sim.set_inputs(0, vals)
    out = []
    for _ in pairs:
        sim.step(1)
        out.append(sim.regs().copy())
    return pairs, out


def test_ripple_adder4():
    pairs, out = run_pairs(g.ripple_adder(4))
    for (a, b), r in zip(pairs, out):
        assert int(r[0]) == a + b, (a, b, r)


def test_array_multiplier4():
    pairs, out = run_pairs(g.array_multiplier(4))
    for (a, b), r in zip(pairs, out):
        assert int(r[0]) == a * b, (a, b, r)


def test_comparators4():
    pairs, out = run_pairs(g.comparators(4))
    for (a, b), r in zip(pairs, out):
        assert int(r[0]) == int(a == b) and int(r[1]) == int(a < b), (a, b, r)


@pytest.mark.parametrize("n", [2, 3, 5])
def test_adder_other_widths(n):
    pairs, out = run_pairs(g.ripple_adder(n), n)
    assert all(int(r[0]) == a + b for (a, b), r in zip(pairs, out))
