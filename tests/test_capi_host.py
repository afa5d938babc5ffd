"""Host-side checks of libfibersim through its C-ABI, no GPU needed: the
library loads and exports every symbol the header declares; designs compile
on the host (ctx = NULL) with the right status codes; the compiler's
per-process node lists, run through the oracle's partitioned mode, give the
monolithic result (cone completeness); and the packer reproduces the paper's
worked examples (the staircase of Sec. 6.3 and the memory pre-merge bound of
Sec. 5.1) and the submodular cost identity of Sec. 4.3."""
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2403_04714_amd import fibersim as F
from paper_2403_04714_amd import netgen as g
from tests.conftest import ROOT, golden_lines

HEADER = os.path.join(ROOT, "include", "fibersim.h")


def header_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fsim_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = F.lib()
    syms = header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(L, s), s
        assert s in F.SIGNATURES, f"binding lacks {s}"


def host_design(nl, **kw):
    return F.Design(None, nl, **kw)


def test_host_compile_info_tiny():
    nl = g.gen_tiny(0)
    d = host_design(nl, pack=F.PACK_SINGLE)
    info = d.info()
    assert info["n_processes"] == 1
    assert info["n_regs"] == 64 and info["n_sinks"] == 64 + 4
    assert info["max_depth"] <= 16
    assert info["dup_process"] == pytest.approx(1.0)
    assert info["dup_fiber"] >= 1.0
    assert info["program_bytes"] > 0


def test_error_codes():
    b = g.Builder()
    r = b.add_reg(4, 0)
    x = b.op2("ADD", b.reg(r), b.const(4, 1))
    y = b.op2("XOR", x, x)
    b.set_next(r, y)
    nl = b.build()
    nl.arg[x, 1] = y
    with pytest.raises(F.FsimError) as e:
        host_design(nl)
    assert e.value.code == F.E_COMB_LOOP
    bad = g.counter(8); bad.width[1] = 65
    with pytest.raises(F.FsimError) as e:
        host_design(bad)
    assert e.value.code == F.E_UNSUPPORTED
    bad = g.counter(8); bad.width[1] = 0
    with pytest.raises(F.FsimError) as e:
        host_design(bad)
    assert e.value.code == F.E_NETLIST
    bad = g.counter(8); bad.arg[2, 1] = 999
    with pytest.raises(F.FsimError) as e:
        host_design(bad)
    assert e.value.code == F.E_NETLIST
    bad = g.counter(8); bad.op[2] = 31
    with pytest.raises(F.FsimError) as e:
        host_design(bad)
    assert e.value.code == F.E_UNSUPPORTED
    with pytest.raises(F.FsimError) as e:
        host_design(g.counter(8), partition=[0, 0, 0])
    assert e.value.code == F.E_ARG
    assert "n_sinks" in str(e.value)


def small_core(seed=5):
    p = g.CoreParams(n_regs_1=700, n_regs_32=150, n_regs_64=150, target_ops=10000,
                     mem_depth=64, reg_locality=64)
    return g.gen_core(seed, p)


def test_partition_must_colocate_memory_ports():
    nl = small_core()
    stp = np.arange(nl.n_sinks, dtype=np.uint32)     # every sink alone
    with pytest.raises(F.FsimError) as e:
        host_design(nl, partition=stp)
    assert e.value.code == F.E_ARG


@pytest.mark.parametrize("pack,target", [(F.PACK_SINGLE, 0), (F.PACK_FIBERS, 0),
                                         (F.PACK_SLB, 7), (F.PACK_SLB, 64),
                                         (F.PACK_HYPER, 7), (F.PACK_HYPER, 64)])
def test_compiler_node_lists_reproduce_monolithic(pack, target):
    for nl in (g.gen_tiny(2), small_core(5)):
        d = host_design(nl, pack=pack, target_processes=target)
        stp, off, nodes = d.partition()
        info = d.info()
        if pack in (F.PACK_SLB, F.PACK_HYPER):
            assert info["n_processes"] <= target
        s0 = O.Sim(nl, seed=3)
        d0 = s0.step(60, digests=True)
        s1 = O.Sim(nl, seed=3)
        d1 = s1.step_partitioned(60, stp, off, nodes, digests=True)
        assert np.array_equal(d0, d1)
        for m in range(nl.n_mems):
            assert np.array_equal(s0.mem(m), s1.mem(m))


def test_node_lists_are_closed_cones():
    nl = g.gen_tiny(7)
    d = host_design(nl, pack=F.PACK_SLB, target_processes=9)
    stp, off, nodes = d.partition()
    for p in range(len(off) - 1):
        have = set(int(x) for x in nodes[off[p]:off[p + 1]])
        for x in have:
            for a in nl.arg[x]:
                if a != g.NONE:
                    assert int(a) in have


def union_cost(nl, nodes):
    """tau of a node set in the compiler's cost unit (Sec. 4.3): constants
    0, register and input leaves 1, operators and memory reads 2 above 32
    bits and 1 otherwise."""
    c = 0
    for x in nodes:
        op = int(nl.op[x])
        if op in (1, 2):
            c += 1
        elif op >= 3:
            c += 2 if int(nl.width[x]) > 32 else 1
    return c


@pytest.mark.parametrize("target", [3, 16, 50])
def test_hypergraph_packing_is_valid(target):
    """Hypergraph packing: every sink in one process, memory groups kept,
    at most `target` processes, each process's node list the union of its
    fibers' cones (checked against a brute-force crawl), and the reported
    duplication and straggler equal to what the node lists give."""
    nl = small_core(5)
    d = host_design(nl, pack=F.PACK_HYPER, target_processes=target)
    stp, off, nodes = d.partition()
    info = d.info()
    P = len(off) - 1
    assert info["n_processes"] == P <= target
    assert stp.min() >= 0 and stp.max() < P
    # the union of cones by brute force
    R, W = nl.n_regs, len(nl.wp_mem)
    def cone(roots):
        seen, st = set(), list(roots)
        while st:
            x = st.pop()
            if x in seen:
                continue
            seen.add(x)
            st.extend(int(a) for a in nl.arg[x] if a != g.NONE)
        return seen
    roots = [[int(nl.reg_next[s])] for s in range(R)]
    roots += [[int(nl.wp_en[k]), int(nl.wp_addr[k]), int(nl.wp_data[k])] for k in range(W)]
    roots += [[int(o)] for o in nl.out_node]
    want = [set() for _ in range(P)]
    for s, r in enumerate(roots):
        want[int(stp[s])] |= cone(r)
    for p in range(P):
        assert set(int(x) for x in nodes[off[p]:off[p + 1]]) == want[p]
    # memory co-location: every reader of a written memory shares the
    # process of its write ports
    for m in range(nl.n_mems):
        ports = [R + k for k in range(W) if int(nl.wp_mem[k]) == m]
        if not ports:
            continue
        home = {int(stp[s]) for s in ports}
        assert len(home) == 1
        for s, r in enumerate(roots):
            if any(int(nl.op[x]) == 3 and int(nl.imm[x]) == m for x in cone(r)):
                assert int(stp[s]) in home
    costs = [union_cost(nl, want[p]) for p in range(P)]
    assert info["max_process_cost"] == max(costs)


def test_hypergraph_packing_beats_fiber_duplication():
    """On the single-core workload, hypergraph packing replicates less than
    one fiber per process does (D_p < D_f) and never exceeds the target."""
    nl = g.workload("core")
    d = host_design(nl, pack=F.PACK_HYPER, target_processes=1024)
    info = d.info()
    assert info["n_processes"] <= 1024
    assert 1.0 <= info["dup_process"] < info["dup_fiber"]
    assert info["max_process_cost"] >= info["max_fiber_cost"]


def equal_fibers(n_fibers, ops_each, width=16):
    """n disjoint registers, each x' = x + c applied ops_each times (equal cones)."""
    b = g.Builder()
    for i in range(n_fibers):
        r = b.add_reg(width, i)
        x = b.reg(r)
        for k in range(ops_each):
            x = b.op2("ADD", x, b.const(width, k + 1))
        b.set_next(r, x)
    return b.build(name="equal_fibers")


def test_staircase_example():
    """Sec. 6.3: twelve equal fibers on 4/5/6 processes -> 3/3/2 fibers in the
    largest process."""
    lines = golden_lines("staircase.txt")
    n = int(lines[0].split()[1])
    nl = equal_fibers(n, 5)
    one = host_design(nl, pack=F.PACK_FIBERS).info()["max_process_cost"]
    for ln in lines[1:]:
        procs, largest = (int(x) for x in ln.split())
        info = host_design(nl, pack=F.PACK_SLB, target_processes=procs).info()
        assert info["n_processes"] == procs
        assert info["max_process_cost"] == largest * one, (procs, info["max_process_cost"], one)


def test_submodular_cost_identity():
    """Sec. 4.3: tau(f1 u f2) = t1 + t2 - tau(f1 n f2): checked on operator
    counts against a brute-force intersection of the two cones."""
    rng = np.random.default_rng(0)
    for trial in range(5):
        b = g.Builder()
        r1, r2 = b.add_reg(8, 1), b.add_reg(8, 2)
        shared = b.reg(r1)
        for k in range(int(rng.integers(1, 6))):
            shared = b.op2("XOR", shared, b.const(8, k))
        x1, x2 = shared, shared
        for k in range(int(rng.integers(1, 6))):
            x1 = b.op2("ADD", x1, b.reg(r2))
        for k in range(int(rng.integers(1, 6))):
            x2 = b.op2("SUB", x2, b.const(8, 3))
        b.set_next(r1, x1)
        b.set_next(r2, x2)
        nl = b.build()

        def cone(root):
            seen, st = set(), [int(root)]
            while st:
                x = st.pop()
                if x in seen:
                    continue
                seen.add(x)
                st.extend(int(a) for a in nl.arg[x] if a != g.NONE)
            return {x for x in seen if nl.op[x] >= g.OPS["MEMRD"]}

        c1, c2 = cone(nl.reg_next[0]), cone(nl.reg_next[1])
        fib = host_design(nl, pack=F.PACK_FIBERS).info()
        one = host_design(nl, pack=F.PACK_SINGLE).info()
        assert fib["sum_process_ops"] == len(c1) + len(c2)
        assert one["sum_process_ops"] == len(c1) + len(c2) - len(c1 & c2)
        assert one["sum_process_ops"] == len(c1 | c2)


def test_memory_premerge_bound():
    """Sec. 5.1 footnote: one 256 KiB array and four 64 KiB arrays, three
    equal fibers each, three processes: no process may need more than
    384 KiB of array memory, and every array lives in exactly one process."""
    kv = {ln.split()[0]: [int(x) for x in ln.split()[1:]] for ln in golden_lines("premerge.txt")}
    sizes_kib = kv["arrays_kib"]
    per = kv["fibers_per_array"][0]
    nproc = kv["processes"][0]
    bound = kv["bound_with_premerge_kib"][0]
    b = g.Builder()
    b.add_input(16)
    mems = [b.add_mem(kib * 1024 // 8, 64) for kib in sizes_kib]
    for m in mems:
        for k in range(per):
            r = b.add_reg(64, 0)
            addr = b.op2("ADD", b.input(0), b.const(16, k))
            b.set_next(r, b.memrd(m, addr))
        b.wport(m, b.const(1, 1), b.input(0), b.op2("XOR", b.reg(r), b.const(64, 5)))
    nl = b.build()
    d = host_design(nl, pack=F.PACK_SLB, target_processes=nproc)
    stp, off, nodes = d.partition()
    assert d.info()["n_processes"] == nproc
    owner = {}
    for p in range(nproc):
        mem_here = {int(nl.imm[x]) for x in nodes[off[p]:off[p + 1]] if nl.op[x] == g.OPS["MEMRD"]}
        for m in mem_here:
            assert m not in owner
            owner[m] = p
        assert sum(sizes_kib[m] for m in mem_here) <= bound
    assert sorted(owner) == list(range(len(mems)))


@pytest.mark.parametrize("pack", [F.PACK_SLB, F.PACK_HYPER])
def test_capacity_limit_respected(pack):
    nl = g.gen_tiny(1)
    d = host_design(nl, pack=pack, target_processes=20, max_process_nodes=400)
    stp, off, nodes = d.partition()
    assert np.diff(off).max() <= 400
    with pytest.raises(F.FsimError) as e:
        host_design(nl, pack=pack, target_processes=1, max_process_nodes=50)
    assert e.value.code == F.E_CAPACITY


# every packing the GPU tests ask for compiles on the host (so that a GPU run
# never spends its time on a design that cannot be built)
@pytest.mark.parametrize("make,pack,target", [
    ("tiny0", 2, 0), ("tiny1", 1, 0), ("tiny1", 0, 8), ("tiny1", 0, 33), ("tiny2", 0, 16),
    ("tiny3", 0, 5), ("tiny4", 0, 12), ("tiny6", 0, 9),
    ("small_core", 0, 4), ("small_core", 0, 6), ("small_core", 0, 24), ("small_core", 0, 200),
    ("core", 0, 256), ("core", 0, 1024), ("core", 0, 2048),
])
def test_gpu_test_designs_compile(make, pack, target):
    from paper_2403_04714_amd import fibersim as F
    if make.startswith("tiny"):
        nl = g.gen_tiny(int(make[4:]))
    elif make == "small_core":
        p = g.CoreParams(n_regs_1=1400, n_regs_32=300, n_regs_64=300, target_ops=20000,
                         mem_depth=256, reg_locality=96)
        nl = g.gen_core(5, p)
    else:
        nl = g.workload(make)
    d = F.Design(None, nl, pack=pack, target_processes=target)
    assert d.info()["n_processes"] >= 1
    d.batched_info()


def lowered(nl):
    """nl with every register enable written out as the header numbers it:
    per enabled register, in register order, a REG leaf then
    MUX(en, next, leaf) after the netlist's own nodes."""
    import dataclasses
    op, width, arg, imm = list(nl.op), list(nl.width), [list(a) for a in nl.arg], list(nl.imm)
    nxt = nl.reg_next.copy()
    for r in np.flatnonzero(nl.reg_en != g.NONE):
        leaf = len(op)
        op += [g.OPS["REG"], g.OPS["MUX"]]
        width += [nl.reg_width[r]] * 2
        arg += [[g.NONE] * 3, [nl.reg_en[r], nl.reg_next[r], leaf]]
        imm += [r, 0]
        nxt[r] = leaf + 1
    return dataclasses.replace(nl, op=np.array(op, np.uint8), width=np.array(width, np.uint8),
                               arg=np.array(arg, np.uint32), imm=np.array(imm, np.uint64),
                               reg_next=nxt, reg_en=None)


@pytest.mark.parametrize("pack,target", [(F.PACK_FIBERS, 0), (F.PACK_SLB, 9), (F.PACK_HYPER, 9)])
def test_clock_enables_lowered_by_the_compiler(pack, target):
    """Gated and divided clocks (Sec. 5.3): the compiler's processes, run by
    the oracle's partitioned mode on the netlist with its enables written out
    as multiplexers, give the oracle's own enable semantics; the compiled node
    count includes the two nodes per enabled register."""
    nl = g.add_clock_domains(g.gen_tiny(6), seed=4)
    n_en = int((nl.reg_en != g.NONE).sum())
    d = host_design(nl, pack=pack, target_processes=target)
    assert d.info()["n_nodes"] == nl.n_nodes + 2 * n_en
    stp, off, nodes = d.partition()
    s0 = O.Sim(nl, seed=2)
    d0 = s0.step(120, digests=True)
    s1 = O.Sim(lowered(nl), seed=2)
    d1 = s1.step_partitioned(120, stp, off, nodes, digests=True)
    assert np.array_equal(d0, d1)


def test_clock_enable_out_of_range_rejected():
    import dataclasses
    nl = g.gen_tiny(0)
    en = np.full(nl.n_regs, g.NONE, np.uint32)
    en[5] = nl.n_nodes + 1
    with pytest.raises(F.FsimError) as e:
        host_design(dataclasses.replace(nl, reg_en=en))
    assert e.value.code == F.E_NETLIST


def test_plain_slots_follow_liveness():
    """The plain form gives LDS slots by liveness: a value's slot is reused
    after the last level that reads it, so a process needs fewer slots than
    nodes, and never fewer than the next values it keeps for its store
    level (one per register it owns)."""
    nl = g.workload("core")
    d = host_design(nl, pack=F.PACK_HYPER, target_processes=2048)
    info = d.info()
    stp, off, nodes = d.partition()
    regs_per_proc = np.bincount(stp[: nl.n_regs], minlength=info["n_processes"])
    assert regs_per_proc.max() <= info["plain_max_slots"] < info["max_process_nodes"]


@pytest.mark.parametrize("make,pack,target", [
    (lambda: g.gen_tiny(3), F.PACK_SLB, 4),
    (lambda: g.gen_tiny(11), F.PACK_HYPER, 9),
    (lambda: g.workload("core"), F.PACK_HYPER, 2048),
    (lambda: g.workload("core"), F.PACK_SLB, 512),
    (lambda: g.workload("core_clocks"), F.PACK_HYPER, 2048),
    (lambda: g.workload("soc8"), F.PACK_HYPER, 4096),
])
def test_plain_unit_allocation_self_check(monkeypatch, make, pack, target):
    """The plain encoder's LDS units, checked against its own liveness: no
    two values hold a unit at a common position, and the unit above a
    one-unit operator result (which the result's 8-byte store overwrites at
    its step) holds no live value then.  The library checks this itself
    when FSIM_CHECK_UNITS is set and fails the compile with E_INTERNAL."""
    monkeypatch.setenv("FSIM_CHECK_UNITS", "1")
    d = host_design(make(), pack=pack, target_processes=target)
    assert d.info()["plain_max_slots"] > 0
