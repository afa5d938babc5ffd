"""The seeded generators produce the workload shapes they promise (sizes,
widths, depth, activity), deterministically."""
import numpy as np

from oracle import oracle as O
from paper_2403_04714_amd import netgen as g


def comb_depth(nl):
    d = np.zeros(nl.n_nodes, np.int64)
    for n in range(nl.n_nodes):                    # builders emit operands first
        if nl.op[n] >= g.OPS["MEMRD"]:
            d[n] = 1 + max(d[a] for a in nl.arg[n] if a != g.NONE)
    return d


def test_tiny_shape():
    nl = g.gen_tiny(0)
    assert nl.n_regs == 64 and nl.n_inputs == 8
    assert nl.n_comb_ops() == 1000
    assert 1 <= nl.reg_width.min() and nl.reg_width.max() <= 32
    assert comb_depth(nl).max() <= 16
    ar = (nl.arg != g.NONE).sum(axis=1)[nl.op >= g.OPS["AND"]]
    assert set(np.unique(ar)) <= {1, 2, 3}


def test_deterministic():
    a, b = g.gen_tiny(5), g.gen_tiny(5)
    for f in ("op", "width", "arg", "imm", "reg_init", "reg_next"):
        assert np.array_equal(getattr(a, f), getattr(b, f))


def test_core_shape_and_activity():
    nl = g.gen_core(1)
    s = nl.summary()
    assert s["regs"] == 20000 and s["regs_1b"] == 14000
    assert 180_000 <= s["comb_ops"] <= 220_000
    assert s["mems"] == 2 and s["wports"] == 2
    assert 30 <= comb_depth(nl).max() <= 48
    # activity: most registers toggle within the first cycles
    sim = O.Sim(nl, seed=g.STIM_SEED_BASE)
    r0 = sim.regs().copy()
    changed = np.zeros(nl.n_regs, bool)
    for _ in range(20):
        sim.step(1)
        r = sim.regs()
        changed |= r != r0
        r0 = r.copy()
    assert changed.mean() > 0.3, changed.mean()


def test_soc_replicates_core():
    core = g.gen_core(1, g.CoreParams(n_regs_1=350, n_regs_32=75, n_regs_64=75,
                                      target_ops=5000, mem_depth=64, reg_locality=32))
    soc = g.gen_soc(2, 2, core, mesh_seed=2)
    assert soc.n_regs == 4 * core.n_regs + 4 * 4 * 3
    assert soc.n_mems == 4 * core.n_mems and soc.n_inputs == 4 * core.n_inputs
    sim = O.Sim(soc, seed=1)      # valid: acyclic, indices in range
    sim.step(20)


def test_prng_array_is_independent_xorshift32():
    """Each register of the PRNG array follows Marsaglia's xorshift32
    recurrence on its own (the synchronization experiment of Sec. 4.1)."""
    from oracle import oracle as O
    nl = g.prng_array(37, seed=3)
    assert nl.n_comb_ops() == 6 * 37
    ref = O.Sim(nl, seed=1)
    ref.step(11)
    def xs(v):
        v ^= (v << 13) & 0xFFFFFFFF
        v ^= v >> 17
        v ^= (v << 5) & 0xFFFFFFFF
        return v
    x = [int(v) for v in nl.reg_init]
    for _ in range(11):
        x = [xs(v) for v in x]
    assert [int(v) for v in ref.regs()] == x


def test_clock_domains_structure():
    """add_clock_domains keeps the design, adds one divider register per
    divisor and one 1-bit gate port per gated domain, and gives half of the
    original registers an enable that is a 1-bit node of one of the domains."""
    base = g.gen_tiny(3)
    nl = g.add_clock_domains(base, seed=5, divisors=(2, 3, 8), n_gated=1, frac=0.5)
    R0, N0 = base.n_regs, base.n_nodes
    assert nl.n_regs == R0 + 3 and nl.n_inputs == base.n_inputs + 1
    for f in ("op", "width", "imm"):
        assert np.array_equal(getattr(nl, f)[:N0], getattr(base, f))
    assert np.array_equal(nl.arg[:N0], base.arg)
    assert np.array_equal(nl.reg_next[:R0], base.reg_next)
    en = nl.reg_en
    gated = np.flatnonzero(en[:R0] != g.NONE)
    assert len(gated) == round(0.5 * R0) == nl.meta["gated_regs"]
    assert (en[R0:] == g.NONE).all()                  # dividers run on the top clock
    domains = set(int(x) for x in en[gated])
    assert len(domains) == 4                          # three dividers and one gate
    for e in domains:
        assert e >= N0 and nl.width[e] == 1
        assert nl.op[e] in (g.OPS["EQ"], g.OPS["INPUT"])
    # deterministic
    again = g.add_clock_domains(base, seed=5, divisors=(2, 3, 8), n_gated=1, frac=0.5)
    assert np.array_equal(again.reg_en, en)


def test_core_clocks_workload():
    nl = g.workload("core_clocks")
    assert nl.n_regs == 20003 and nl.meta["gated_regs"] == 10000
    assert nl.reg_en is not None and len(nl.reg_en) == nl.n_regs


def test_core_memory_init_draws_every_bit():
    """Random memory initialisation covers the whole 64-bit word: every bit
    position, the lowest and the highest included, is set in about half of
    the words (a bit stuck at zero would hide read-path errors on that bit
    until the word is first written)."""
    nl = g.gen_core(1)
    w = nl.mem_init
    assert w.size == 2 * 4096
    bits = (w[:, None] >> np.arange(64, dtype=np.uint64)[None, :]) & np.uint64(1)
    frac = bits.mean(axis=0)
    assert frac.min() > 0.45 and frac.max() < 0.55, (frac.min(), frac.max())
