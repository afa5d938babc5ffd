"""Operator semantics of the oracle against the unbounded-integer statement
of the same operators (oracle/pyref.py): exhaustive over every operand pair
for narrow widths, seeded random operands at the edge widths, and the shift
guards (amounts >= width and >= 64 give zero)."""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from oracle.pyref import OPS, ref_op

COMB = ["AND", "OR", "XOR", "NOT", "ADD", "SUB", "MUX", "SHL", "SHR", "EQ", "LT", "MUL"]


@pytest.mark.parametrize("name", COMB)
def test_exhaustive_narrow(name):
    op = OPS[name]
    for w in range(1, 5):
        for a, b in itertools.product(range(16), repeat=2):
            cs = (0, 5) if name == "MUX" else (0,)
            for c in cs:
                got = O.eval_op(op, w, a, b, c)
                assert got == ref_op(op, w, a, b, c), (name, w, a, b, c, got)


EDGE_W = [1, 2, 31, 32, 33, 63, 64]


@pytest.mark.parametrize("name", COMB)
def test_random_edge_widths(name):
    op = OPS[name]
    rng = np.random.default_rng(OPS[name])
    specials = [0, 1, 2**31 - 1, 2**31, 2**32 - 1, 2**32, 2**63 - 1, 2**63, 2**64 - 1]
    for w in EDGE_W:
        vals = specials + [int(x) for x in rng.integers(0, 2**63, 60, dtype=np.int64)] \
            + [int(x) | 2**63 for x in rng.integers(0, 2**63, 20, dtype=np.int64)]
        for a in vals:
            for j in rng.integers(0, len(vals), 8):
                b = vals[int(j)]
                c = vals[int(rng.integers(0, len(vals)))]
                assert O.eval_op(op, w, a, b, c) == ref_op(op, w, a, b, c), (name, w, a, b, c)


@pytest.mark.parametrize("w", [1, 7, 32, 63, 64])
def test_shift_guards(w):
    a = 2**w - 1
    for amt in [w - 1, w, w + 1, 63, 64, 65, 2**32, 2**63, 2**64 - 1]:
        shl = O.eval_op(OPS["SHL"], w, a, amt)
        shr = O.eval_op(OPS["SHR"], w, a, amt)
        assert shl == ref_op(OPS["SHL"], w, a, amt)
        assert shr == ref_op(OPS["SHR"], w, a, amt)
        if amt >= 64:
            assert shl == 0 and shr == 0
        if amt >= w:
            assert shl == 0


def test_result_always_masked():
    rng = np.random.default_rng(5)
    for _ in range(2000):
        op = OPS[COMB[int(rng.integers(0, len(COMB)))]]
        w = int(rng.integers(1, 65))
        a, b, c = (int(x) for x in rng.integers(0, 2**63, 3, dtype=np.int64))
        assert O.eval_op(op, w, a, b, c) < 2**w
