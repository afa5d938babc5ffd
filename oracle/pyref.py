"""Arbitrary-precision statement of the word-level operators -- TEST
INFRASTRUCTURE ONLY.

The paper works on Verilator's AST and prints no operator table, so the
operators are read as unsigned Verilog expressions whose operands are
zero-extended and whose result is truncated to the node width (the reading
recorded beside the oracle).  Here each operator is written with Python's
unbounded integers straight from that textbook meaning -- "the sum modulo
2**w", "the product modulo 2**w", "a shifted left by b places, modulo 2**w" --
with no 64-bit machine arithmetic, no masks built from shifts and no special
cases for large shift amounts: a left shift by b >= w simply leaves no bits
below 2**w.  That makes it an independent statement against which the C
oracle's 64-bit formulas (which need explicit guards) are checked.
"""
from __future__ import annotations

OPS = dict(CONST=0, INPUT=1, REG=2, MEMRD=3, AND=4, OR=5, XOR=6, NOT=7,
           ADD=8, SUB=9, MUX=10, SHL=11, SHR=12, EQ=13, LT=14, MUL=15)


def ref_op(op: int, w: int, a: int, b: int = 0, c: int = 0) -> int:
    """Value of one operator of width w on unsigned operands a, b, c."""
    M = 2 ** w
    if op == OPS["AND"]:
        r = a & b
    elif op == OPS["OR"]:
        r = a | b
    elif op == OPS["XOR"]:
        r = a ^ b
    elif op == OPS["NOT"]:
        r = (2 ** 64 - 1) - a          # complement of the 64-bit zero-extension
    elif op == OPS["ADD"]:
        r = a + b
    elif op == OPS["SUB"]:
        r = a - b                      # Python's % below maps negatives into [0, M)
    elif op == OPS["MUX"]:
        r = b if a != 0 else c
    elif op == OPS["SHL"]:
        r = a * pow(2, b, M)           # a * 2**b reduced mod 2**w
    elif op == OPS["SHR"]:
        r = a >> b                     # floor(a / 2**b) for unbounded ints
    elif op == OPS["EQ"]:
        r = int(a == b)
    elif op == OPS["LT"]:
        r = int(a < b)
    elif op == OPS["MUL"]:
        r = a * b
    else:
        raise ValueError(op)
    return r % M
