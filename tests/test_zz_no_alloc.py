"""fsim_read_regs_noalloc, the register readback for callers that cannot
allocate device memory, against fsim_read_regs through the C-ABI: two
calls in a row on batched sims (the second on a smaller design, so it reads
a shorter prefix of the static staging array the first call filled), the
plain form, and the size limit."""
import ctypes as C

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
    c = F.Context(0)
    yield c
    F.close_all()


def noalloc(F, sim, inst, n):
    out = np.zeros(max(n, 1), np.uint64)
    rc = F.lib().fsim_read_regs_noalloc(sim._h, inst, C.c_void_p(out.ctypes.data))
    return rc, out[:n]


def small_core(seed=5):
    p = g.CoreParams(n_regs_1=1400, n_regs_32=300, n_regs_64=300, target_ops=20000,
                     mem_depth=256, reg_locality=96)
    return g.gen_core(seed, p)


def test_noalloc_equals_read_regs_twice_then_smaller(F, ctx):
    big, small = small_core(), g.gen_tiny(0)
    print("case no-alloc: batched reduced core x130, then tiny x65", flush=True)
    d1 = F.Design(ctx, big, target_processes=64)
    s1 = F.Sim(d1, 130, seed=SEED, form=F.FORM_BATCHED)
    s1.step(57)
    for inst in (77, 129):
        rc, got = noalloc(F, s1, inst, d1.n_regs)
        assert rc == F.OK, F.lib().fsim_last_error()
        assert np.array_equal(got, s1.regs(inst)), f"instance {inst}"
    ref = O.Sim(big, seed=SEED + 77)
    ref.step(57)
    assert np.array_equal(noalloc(F, s1, 77, d1.n_regs)[1], ref.regs())
    d2 = F.Design(ctx, small, pack=F.PACK_SINGLE)
    s2 = F.Sim(d2, 65, seed=SEED + 3, form=F.FORM_BATCHED)
    s2.step(33)
    for inst in (64, 0):
        rc, got = noalloc(F, s2, inst, d2.n_regs)
        assert rc == F.OK, F.lib().fsim_last_error()
        assert np.array_equal(got, s2.regs(inst)), f"instance {inst}"
    assert np.array_equal(s2.regs_noalloc(5), s2.regs(5))
    s1.close()
    s2.close()
    d1.close()
    d2.close()


def test_noalloc_plain_form(F, ctx):
    nl = g.gen_tiny(2)
    d = F.Design(ctx, nl, target_processes=4)
    s = F.Sim(d, 1, seed=SEED, form=F.FORM_PLAIN, launch=F.LAUNCH_GRAPH, wg_threads=64)
    s.step(101)
    rc, got = noalloc(F, s, 0, d.n_regs)
    assert rc == F.OK
    assert np.array_equal(got, s.regs())
    assert noalloc(F, s, 1, d.n_regs)[0] == F.E_ARG       # instance out of range
    s.close()
    d.close()


def identity_regs(n):
    """n one-bit registers that keep their initial value: register r's next
    value is its own REG node r."""
    idx = np.arange(n, dtype=np.uint64)
    return g.Netlist(
        op=np.full(n, g.OPS["REG"], np.uint8), width=np.ones(n, np.uint8),
        arg=np.full((n, 3), g.NONE, np.uint32), imm=idx, reg_width=np.ones(n, np.uint8),
        reg_init=idx & np.uint64(1), reg_next=idx.astype(np.uint32), in_width=np.zeros(0, np.uint8),
        out_node=np.zeros(0, np.uint32), mem_depth=np.zeros(0, np.uint32), mem_width=np.zeros(0, np.uint8),
        mem_init=np.zeros(0, np.uint64), wp_mem=np.zeros(0, np.uint32), wp_en=np.zeros(0, np.uint32),
        wp_addr=np.zeros(0, np.uint32), wp_data=np.zeros(0, np.uint32), name=f"identity{n}")


def test_noalloc_size_limit(F, ctx):
    n = (1 << 20) + 1
    print("case no-alloc: 1,048,577 registers (one past the static array)", flush=True)
    nl = identity_regs(n)
    d = F.Design(ctx, nl, partition=np.arange(n, dtype=np.uint32) // 1024)
    s = F.Sim(d, 1, seed=SEED, form=F.FORM_BATCHED)
    s.step(2)
    rc, _ = noalloc(F, s, 0, n)
    assert rc == F.E_CAPACITY
    assert np.array_equal(s.regs(0), nl.reg_init)
    s.close()
    d.close()
    # the largest design it takes: exactly 1,048,576 registers
    nl = identity_regs(n - 1)
    d = F.Design(ctx, nl, partition=np.arange(n - 1, dtype=np.uint32) // 1024)
    s = F.Sim(d, 1, seed=SEED, form=F.FORM_BATCHED)
    s.step(3)
    rc, got = noalloc(F, s, 0, n - 1)
    assert rc == F.OK
    assert np.array_equal(got, nl.reg_init)
    s.close()
    d.close()
