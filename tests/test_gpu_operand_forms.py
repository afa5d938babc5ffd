"""Operand forms the encoders special-case, on the GPU against the oracle,
bit-exact, every cycle:
- plain form: a narrow value (at most 32 bits) is kept in one 4-byte LDS unit
  unless an instruction reading it depends on its upper half (comparisons,
  right shifts, shift amounts, multiplexer selects, memory addresses, write
  ports, wide results, stores into registers wider than 32 bits); the design
  below reads narrow values in every one of those roles and in the tolerant
  ones;
- batched form: 1-bit operators become whole-mask operations, including
  products and shifts of 1-bit values and comparisons with constants, and
  must not where a constant or shifted operand has more than bit 0 set.

Every node feeds a register, so every result is checked through the
per-cycle digests and the final state."""
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


def operand_forms():
    b = g.Builder()
    i1, i3, i8, i40 = b.add_input(1), b.add_input(3), b.add_input(8), b.add_input(40)
    # state that changes every cycle: narrow and wide registers mixed with inputs
    a1, c1 = b.add_reg(1, 1), b.add_reg(1, 0)
    x8, y7, z32 = b.add_reg(8, 3), b.add_reg(7, 5), b.add_reg(32, 123456)
    w64, v33 = b.add_reg(64, 2**63 + 11), b.add_reg(33, 2**32 + 1)
    b.set_next(a1, b.op2("XOR", b.reg(a1), b.input(i1)))
    b.set_next(c1, b.op2("XOR", b.reg(a1), b.op2("AND", b.reg(c1), b.input(i3, 1), w=1)))
    b.set_next(x8, b.op2("ADD", b.reg(x8), b.input(i8), w=8))
    b.set_next(y7, b.op2("XOR", b.reg(y7), b.input(i3), w=7))
    b.set_next(z32, b.op2("ADD", b.op2("MUL", b.reg(z32), b.const(32, 1103515245), w=32), b.input(i8), w=32))
    b.set_next(w64, b.op2("XOR", b.op2("SHL", b.reg(w64), b.const(6, 13)), b.op2("SHR", b.reg(w64), b.const(6, 7))))
    b.set_next(v33, b.op2("ADD", b.reg(v33), b.input(i40), w=33))
    k = {v: b.const(1 if v < 2 else 8, v) for v in (0, 1, 2, 5)}
    k64 = b.const(64, 2**40 + 3)
    results = [
        # plain form: narrow operands in roles that need their upper half zero
        b.op2("ADD", b.reg(x8), b.reg(w64), w=64),          # wide result
        b.op2("SUB", b.reg(z32), b.reg(x8), w=64),
        b.op2("EQ", b.reg(x8), b.reg(y7)),                   # comparisons
        b.op2("LT", b.reg(y7), b.reg(v33)),
        b.op2("LT", b.reg(z32), b.reg(x8)),
        b.op2("SHR", b.reg(z32), b.reg(y7), w=32),           # right shift of a narrow value
        b.op2("SHL", b.reg(w64), b.reg(y7), w=64),           # narrow shift amount
        b.op2("SHL", b.reg(x8), b.reg(c1), w=16),            # narrow shifted operand (tolerant)
        b.mux(b.reg(a1), b.reg(x8), b.reg(w64), w=64),       # narrow select, wide data
        b.mux(b.reg(x8), b.reg(y7), b.reg(z32), w=32),       # 8-bit select
        b.op2("AND", b.reg(x8), b.reg(z32), w=32),           # tolerant narrow results
        b.op2("OR", b.reg(y7), b.reg(x8), w=8),
        b.op2("MUL", b.reg(x8), b.reg(z32), w=32),
        b.not_(b.reg(y7), w=32),
        b.op2("XOR", b.reg(z32), b.reg(v33), w=33),
        b.op2("ADD", b.reg(x8), k64, w=20),
        # batched form: 1-bit operators with 1-bit operands and constants
        b.op2("SHL", b.reg(a1), b.reg(c1), w=1),
        b.op2("SHR", b.reg(a1), b.reg(c1), w=1),
        b.op2("MUL", b.reg(a1), b.reg(c1), w=1),
        b.op2("SHL", k[5], b.reg(c1), w=1),                  # wide constant shifted left: bit 0 only
        b.op2("SHR", k[2], b.reg(c1), w=1),                  # wide constant shifted right: not a mask form
        b.op2("SHR", b.reg(a1), k[2], w=1),                  # shift by 2
        b.op2("SHL", b.reg(a1), k[1], w=1),
        b.op2("MUL", b.reg(a1), k[5], w=1),
        b.op2("EQ", b.reg(a1), k[1]),
        b.op2("EQ", b.reg(a1), k[5]),                        # 1-bit value against a wide constant
        b.op2("LT", b.reg(a1), k[2]),
        b.op2("LT", k[1], b.reg(c1)),
        b.op2("LT", k[0], b.reg(c1)),
        b.op2("EQ", b.reg(a1), b.reg(c1)),
        b.mux(b.reg(c1), k[1], b.reg(a1), w=1),
        b.op2("ADD", b.reg(a1), b.reg(c1), w=1),
        b.op2("SUB", b.reg(a1), k[1], w=1),
    ]
    for n in results:
        r = b.add_reg(b.width_of(n), 0)
        b.set_next(r, n)
    # stores of narrow values into wide registers and outputs
    r64 = b.add_reg(64, 0)
    b.set_next(r64, b.reg(x8))
    r40 = b.add_reg(40, 0)
    b.set_next(r40, b.op2("ADD", b.reg(y7), b.reg(x8), w=8))
    b.output(b.reg(x8))
    b.output(b.op2("XOR", b.reg(y7), b.reg(x8), w=8))
    # a memory addressed and written through narrow values
    m = b.add_mem(5, 16, np.arange(5, dtype=np.uint64) * 7)
    rd = b.memrd(m, b.reg(x8))
    rm = b.add_reg(16, 0)
    b.set_next(rm, b.op2("ADD", rd, b.reg(y7), w=16))
    b.wport(m, b.reg(a1), b.reg(y7), b.op2("XOR", b.reg(x8), b.reg(z32), w=16))
    return b.build("operand_forms")


CYCLES = 300


def reference(nl, seed, cycles):
    ref = O.Sim(nl, seed=seed)
    return ref, ref.step(cycles, digests=True)


@pytest.mark.parametrize("tree", ["low", "high"])
@pytest.mark.parametrize("pack", [0, 1, 2, 3])
def test_plain_operand_forms(F, ctx, pack, tree, monkeypatch):
    """Both opcode-tree thresholds (the one for few waves per SIMD and the
    one for many), whatever the design's size, so every operator chunk runs
    the tree, the per-opcode tests and the single-opcode form."""
    monkeypatch.setenv("FSIM_TREE", tree)
    nl = operand_forms()
    print(f"case operand_forms: plain pack={pack} tree={tree}", flush=True)
    d = F.Design(ctx, nl, pack=pack)
    s = F.Sim(d, 1, seed=SEED, wg_threads=64)
    s.enable_digest(CYCLES)
    s.step(CYCLES)
    ref, rd = reference(nl, SEED, CYCLES)
    assert np.array_equal(s.digests()[:, 0], rd)
    assert np.array_equal(s.regs(), ref.regs())
    assert np.array_equal(s.outputs(), ref.outputs())
    assert np.array_equal(s.mem(0), ref.mem(0))


def test_batched_operand_forms(F, ctx):
    nl = operand_forms()
    n_inst = 70
    print(f"case operand_forms: batched n_inst={n_inst}", flush=True)
    d = F.Design(ctx, nl, pack=F.PACK_SLB)
    s = F.Sim(d, n_inst, seed=SEED)
    s.enable_digest(CYCLES)
    s.step(CYCLES)
    dg = s.digests()
    for i in range(n_inst):
        ref, rd = reference(nl, SEED + i, CYCLES)
        assert np.array_equal(dg[:, i], rd), f"instance {i}"
        assert np.array_equal(s.regs(i), ref.regs()), f"instance {i} registers"
        assert np.array_equal(s.outputs(i), ref.outputs()), f"instance {i} outputs"
        assert np.array_equal(s.mem(0, i), ref.mem(0)), f"instance {i} memory"
