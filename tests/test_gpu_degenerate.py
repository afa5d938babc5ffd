"""Degenerate designs on the GPU against the oracle, bit-exact:
- a design with no combinational operator at all;
- cones that are a single leaf or a single constant;
- 64-bit wrap-around and shifts by >= 64;
- a memory of depth 1 and one of depth 3, where the address is taken mod
  depth and the depth is not a power of two;
- outputs taken straight from a constant, an input and a register.

Each runs in the plain form (single process, one fiber per process, SLB) and
in the batched form with a ragged instance count."""
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


def no_operators():
    """Registers that hold, or copy each other and the inputs: no operator."""
    b = g.Builder()
    b.add_input(5)
    r = [b.add_reg(w, init) for w, init in ((5, 3), (64, 2**64 - 1), (1, 1), (64, 7))]
    b.set_next(r[0], b.input(0))
    b.set_next(r[1], b.reg(r[1]))            # holds
    b.set_next(r[2], b.reg(r[2]))
    b.set_next(r[3], b.reg(r[1]))            # copies r1
    b.output(b.reg(r[0]))
    b.output(b.input(0))
    return b.build("no_operators")


def edge_cases():
    b = g.Builder()
    b.add_input(3)
    b.add_input(8)
    r0 = b.add_reg(7, 0)
    r1 = b.add_reg(64, 2**64 - 3)
    r2 = b.add_reg(1, 0)
    r3 = b.add_reg(64, 1)
    r4 = b.add_reg(64, 0)
    r5 = b.add_reg(13, 0)
    r6 = b.add_reg(64, 0)
    b.set_next(r0, b.const(7, 5))                                   # constant cone
    b.set_next(r1, b.op2("ADD", b.reg(r1), b.const(64, 1)))           # wraps through 2^64
    b.set_next(r2, b.input(0, 1))                                    # 3-bit port read as 1 bit
    b.set_next(r3, b.op2("SUB", b.reg(r3), b.reg(r1)))
    sh = b.input(1)                                                  # 0..255: >= 64 often
    b.set_next(r4, b.op2("XOR", b.op2("SHL", b.reg(r3), sh), b.op2("SHR", b.reg(r1), b.const(8, 64))))
    m1 = b.add_mem(1, 64, np.array([0xDEADBEEF], np.uint64))
    m3 = b.add_mem(3, 13, np.array([1, 2, 3], np.uint64))
    rd1 = b.memrd(m1, b.reg(r3))
    rd3 = b.memrd(m3, b.reg(r1))                                      # address mod 3
    b.set_next(r5, b.op2("ADD", rd3, b.reg(r5), w=13))
    b.set_next(r6, b.op2("ADD", rd1, b.reg(r6)))
    b.wport(m1, b.const(1, 1), b.reg(r3), b.reg(r1))
    b.wport(m3, b.reg(r2), b.reg(r3), b.op2("XOR", b.reg(r5), b.reg(r1), w=13))
    b.wport(m3, b.input(0), b.reg(r1), b.reg(r3))                     # later port wins on a tie
    b.output(b.const(9, 300))
    b.output(b.input(1))
    b.output(b.reg(r4))
    return b.build("edge_cases")


def check_plain(F, ctx, nl, pack, cycles, threads=0):
    print(f"case {nl.name}: plain pack={pack} threads={threads} cycles={cycles}", flush=True)
    d = F.Design(ctx, nl, pack=pack)
    s = F.Sim(d, 1, seed=SEED, wg_threads=threads)
    s.enable_digest(cycles)
    s.step(cycles)
    ref = O.Sim(nl, seed=SEED)
    rd = ref.step(cycles, digests=True)
    assert np.array_equal(s.digests()[:, 0], rd)
    assert np.array_equal(s.regs(), ref.regs())
    assert np.array_equal(s.outputs(), ref.outputs())
    for m in range(nl.n_mems):
        assert np.array_equal(s.mem(m), ref.mem(m)), f"memory {m}"


def check_batched(F, ctx, nl, n_inst, cycles):
    print(f"case {nl.name}: batched n_inst={n_inst} cycles={cycles}", flush=True)
    d = F.Design(ctx, nl, pack=F.PACK_SLB)
    s = F.Sim(d, n_inst, seed=SEED)
    s.enable_digest(cycles)
    s.step(cycles)
    dg = s.digests()
    for i in range(n_inst):
        ref = O.Sim(nl, seed=SEED + i)
        rd = ref.step(cycles, digests=True)
        assert np.array_equal(dg[:, i], rd), f"instance {i}"
        assert np.array_equal(s.regs(i), ref.regs()), f"instance {i} registers"
        assert np.array_equal(s.outputs(i), ref.outputs()), f"instance {i} outputs"
        for m in range(nl.n_mems):
            assert np.array_equal(s.mem(m, i), ref.mem(m)), f"instance {i} memory {m}"


@pytest.mark.parametrize("make", [no_operators, edge_cases])
@pytest.mark.parametrize("pack", [0, 1, 2])
@pytest.mark.parametrize("threads", [64, 256])
def test_plain_degenerate(F, ctx, make, pack, threads):
    check_plain(F, ctx, make(), pack, 257, threads)


@pytest.mark.parametrize("make", [no_operators, edge_cases])
def test_batched_degenerate(F, ctx, make):
    check_batched(F, ctx, make(), 67, 129)
