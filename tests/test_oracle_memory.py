"""Memory semantics (the readings recorded with the oracle): reads see the
memory as it was at the start of the cycle; enabled writes commit at the end
of the cycle in port order, so the higher port wins on the same address;
addresses wrap modulo the depth.  Checked on hand scenarios and on seeded
random traffic against a Python dictionary model of a RAM."""
import numpy as np

from oracle import oracle as O
from paper_2403_04714_amd import netgen as g

DEPTH, W = 8, 16


def ram_netlist():
    """Inputs: en0 addr0 data0 en1 addr1 data1 raddr0 raddr1 (ports 0..7).
    Two registered read ports (registers 0, 1), two write ports."""
    b = g.Builder()
    widths = [1, 8, W, 1, 8, W, 8, 8]
    for w in widths:
        b.add_input(w)
    m = b.add_mem(DEPTH, W, np.arange(DEPTH, dtype=np.uint64) * 3)
    ins = [b.input(p) for p in range(8)]
    b.wport(m, ins[0], ins[1], ins[2])
    b.wport(m, ins[3], ins[4], ins[5])
    r0, r1 = b.add_reg(W, 0), b.add_reg(W, 0)
    b.set_next(r0, b.memrd(m, ins[6]))
    b.set_next(r1, b.memrd(m, ins[7]))
    return b.build(name="ram")


def run(rows):
    sim = O.Sim(ram_netlist())
    sim.set_inputs(0, np.array(rows, np.uint64))
    regs = []
    for _ in rows:
        sim.step(1)
        regs.append([int(x) for x in sim.regs()])
    return sim, regs


def test_read_old_then_new():
    # cycle 0: write 0xAAAA to 2 and read 2 -> old value (6)
    # cycle 1: read 2 -> new value
    sim, regs = run([[1, 2, 0xAAAA, 0, 0, 0, 2, 2],
                     [0, 0, 0, 0, 0, 0, 2, 5]])
    assert regs[0] == [6, 6]
    assert regs[1] == [0xAAAA, 15]


def test_higher_port_wins():
    sim, regs = run([[1, 4, 0x1111, 1, 4, 0x2222, 0, 0],
                     [0, 0, 0, 0, 0, 0, 4, 4]])
    assert regs[1] == [0x2222, 0x2222]
    assert int(sim.mem(0)[4]) == 0x2222


def test_disabled_port_and_wrap():
    # address 11 wraps to 3 (depth 8); a disabled port writes nothing
    sim, regs = run([[1, 11, 0x3333, 0, 3, 0x4444, 0, 0],
                     [0, 0, 0, 0, 0, 0, 3, 11]])
    assert regs[1] == [0x3333, 0x3333]


def test_random_traffic_vs_dict_model():
    rng = np.random.default_rng(11)
    T = 500
    rows = np.stack([rng.integers(0, 2, T), rng.integers(0, 256, T), rng.integers(0, 2**16, T),
                     rng.integers(0, 2, T), rng.integers(0, 256, T), rng.integers(0, 2**16, T),
                     rng.integers(0, 256, T), rng.integers(0, 256, T)], axis=1)
    sim, regs = run(rows)
    mem = {a: (3 * a) for a in range(DEPTH)}
    for t in range(T):
        en0, a0, d0, en1, a1, d1, ra0, ra1 = (int(x) for x in rows[t])
        want = [mem[ra0 % DEPTH], mem[ra1 % DEPTH]]
        if en0:
            mem[a0 % DEPTH] = d0
        if en1:
            mem[a1 % DEPTH] = d1
        assert regs[t] == want, t
    assert [int(x) for x in sim.mem(0)] == [mem[a] for a in range(DEPTH)]
