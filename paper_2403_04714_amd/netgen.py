"""Seeded synthetic netlists and small test circuits.

This module only *builds inputs*: flat word-level netlists as numpy arrays.
It evaluates nothing (no operator semantics, no stimulus hash, no simulation),
so both the GPU library and the CPU oracle can take their inputs from it
without sharing any of the method's arithmetic.

Netlist format (structure of arrays; one netlist is one flat graph, no
hierarchy):

  op[n] u8, width[n] u8 (1..64), arg[n,3] u32 (NONE = unused), imm[n] u64
      CONST: imm = value; INPUT: imm = port; REG: imm = register;
      MEMRD: imm = memory, arg0 = address node; MUX: arg = (sel, a, b)
  reg_width[R] u8, reg_init[R] u64, reg_next[R] u32 (node giving the next value)
  in_width[I] u8; out_node[O] u32
  mem_depth[M] u32, mem_width[M] u8, mem_init[sum(depth)] u64
  wp_mem/wp_en/wp_addr/wp_data[W] u32 (write ports, applied in index order)
  reg_en[R] u32 or None: per register an enable node (NONE = top clock); a
      register with an enable keeps its value in cycles where that node is 0
      (gated and divided clocks, Sec. 5.3)

The synthetic designs stand in for the paper's benchmark SoCs (Sec. 6: a
Constellation 2D mesh of Rocket tiles, Chipyard) whose RTL is not available.
They reproduce structure only: replicated cores on a 2D mesh with registered
32-bit links, a skewed fiber-depth distribution with a few deep stragglers
(Sec. 4.3, straggler discussion), and locality, so that cones stay bounded as
in a floor-plannable design (Sec. 6.7).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

NONE = 0xFFFFFFFF
OPS = dict(CONST=0, INPUT=1, REG=2, MEMRD=3, AND=4, OR=5, XOR=6, NOT=7,
           ADD=8, SUB=9, MUX=10, SHL=11, SHR=12, EQ=13, LT=14, MUL=15)
OPNAMES = {v: k for k, v in OPS.items()}
COMB11 = ["AND", "OR", "XOR", "NOT", "ADD", "SUB", "MUX", "SHL", "SHR", "EQ", "LT"]


@dataclasses.dataclass
class Netlist:
    op: np.ndarray
    width: np.ndarray
    arg: np.ndarray
    imm: np.ndarray
    reg_width: np.ndarray
    reg_init: np.ndarray
    reg_next: np.ndarray
    in_width: np.ndarray
    out_node: np.ndarray
    mem_depth: np.ndarray
    mem_width: np.ndarray
    mem_init: np.ndarray
    wp_mem: np.ndarray
    wp_en: np.ndarray
    wp_addr: np.ndarray
    wp_data: np.ndarray
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)
    reg_en: np.ndarray | None = None

    @property
    def n_nodes(self):
        return len(self.op)

    @property
    def n_regs(self):
        return len(self.reg_width)

    @property
    def n_inputs(self):
        return len(self.in_width)

    @property
    def n_outputs(self):
        return len(self.out_node)

    @property
    def n_mems(self):
        return len(self.mem_depth)

    @property
    def n_wports(self):
        return len(self.wp_mem)

    @property
    def n_sinks(self):
        return self.n_regs + self.n_wports + self.n_outputs

    def n_comb_ops(self) -> int:
        return int(np.count_nonzero(self.op >= OPS["MEMRD"]))

    def summary(self) -> dict:
        w = self.reg_width
        return dict(name=self.name, nodes=self.n_nodes, comb_ops=self.n_comb_ops(),
                    regs=self.n_regs, regs_1b=int((w == 1).sum()),
                    regs_le32=int(((w > 1) & (w <= 32)).sum()), regs_gt32=int((w > 32).sum()),
                    inputs=self.n_inputs, outputs=self.n_outputs, mems=self.n_mems,
                    wports=self.n_wports, **self.meta)


class Builder:
    """Incremental netlist construction for test circuits and generators."""

    def __init__(self):
        self.op, self.w, self.a0, self.a1, self.a2, self.imm = [], [], [], [], [], []
        self.reg_w, self.reg_init, self.reg_next, self._reg_node = [], [], [], []
        self.reg_en = []
        self.in_w, self.outs = [], []
        self.mem_depth, self.mem_w, self.mem_init = [], [], []
        self.wp = []

    # -- nodes
    def _node(self, op, w, a=(), imm=0):
        assert 1 <= w <= 64, w
        a = list(a) + [NONE] * (3 - len(a))
        self.op.append(OPS[op] if isinstance(op, str) else op)
        self.w.append(w)
        self.a0.append(a[0]); self.a1.append(a[1]); self.a2.append(a[2])
        self.imm.append(int(imm) & (2**64 - 1))
        return len(self.op) - 1

    def width_of(self, n):
        return self.w[n]

    def const(self, w, v):
        return self._node("CONST", w, (), v)

    def add_input(self, w):
        self.in_w.append(w)
        return len(self.in_w) - 1

    def input(self, port, w=None):
        return self._node("INPUT", self.in_w[port] if w is None else w, (), port)

    def add_reg(self, w, init=0):
        self.reg_w.append(w)
        self.reg_init.append(int(init) & ((1 << w) - 1))
        self.reg_next.append(NONE)
        self.reg_en.append(NONE)
        self._reg_node.append(None)
        return len(self.reg_w) - 1

    def reg(self, r):
        """The (single, shared) REG node reading register r's current value."""
        if self._reg_node[r] is None:
            self._reg_node[r] = self._node("REG", self.reg_w[r], (), r)
        return self._reg_node[r]

    def set_next(self, r, node):
        self.reg_next[r] = node

    def set_enable(self, r, node):
        """Register r takes its next value only in cycles where node != 0."""
        self.reg_en[r] = node

    def op2(self, op, a, b, w=None):
        if w is None:
            w = 1 if op in ("EQ", "LT") else max(self.w[a], self.w[b])
        return self._node(op, w, (a, b))

    def not_(self, a, w=None):
        return self._node("NOT", self.w[a] if w is None else w, (a,))

    def mux(self, s, a, b, w=None):
        return self._node("MUX", max(self.w[a], self.w[b]) if w is None else w, (s, a, b))

    def add_mem(self, depth, w, init=None):
        self.mem_depth.append(depth)
        self.mem_w.append(w)
        init = np.zeros(depth, np.uint64) if init is None else np.asarray(init, np.uint64)
        assert len(init) == depth
        self.mem_init.append(init)
        return len(self.mem_depth) - 1

    def memrd(self, m, addr, w=None):
        return self._node("MEMRD", self.mem_w[m] if w is None else w, (addr,), m)

    def wport(self, m, en, addr, data):
        self.wp.append((m, en, addr, data))
        return len(self.wp) - 1

    def output(self, node):
        self.outs.append(node)
        return len(self.outs) - 1

    def build(self, name="", **meta) -> Netlist:
        n = len(self.op)
        arg = np.stack([np.array(self.a0, np.uint32), np.array(self.a1, np.uint32),
                        np.array(self.a2, np.uint32)], axis=1) if n else np.zeros((0, 3), np.uint32)
        wp = np.array(self.wp, np.uint32).reshape(-1, 4)
        rn = np.array(self.reg_next, np.uint32)
        assert not (rn == NONE).any(), "register without a next value"
        en = np.array(self.reg_en, np.uint32)
        return Netlist(
            op=np.array(self.op, np.uint8), width=np.array(self.w, np.uint8), arg=arg,
            imm=np.array(self.imm, np.uint64),
            reg_width=np.array(self.reg_w, np.uint8), reg_init=np.array(self.reg_init, np.uint64),
            reg_next=rn, in_width=np.array(self.in_w, np.uint8),
            out_node=np.array(self.outs, np.uint32),
            mem_depth=np.array(self.mem_depth, np.uint32), mem_width=np.array(self.mem_w, np.uint8),
            mem_init=(np.concatenate(self.mem_init) if self.mem_init else np.zeros(0, np.uint64)),
            wp_mem=wp[:, 0].copy(), wp_en=wp[:, 1].copy(), wp_addr=wp[:, 2].copy(),
            wp_data=wp[:, 3].copy(), name=name, meta=dict(meta),
            reg_en=en if (en != NONE).any() else None)


def _shift_mask(w):
    """Largest 2**k - 1 below w: an AND with it keeps a shift amount < w."""
    return (1 << int(math.floor(math.log2(w)))) - 1 if w > 1 else 0


# --------------------------------------------------------------------------
# Tiny random netlist: 64 registers of widths U[1,32], 1,000 combinational
# operators of fan-in 2-3 over the 11-operator mix, depth <= 16, 8 inputs.
# --------------------------------------------------------------------------
def gen_tiny(seed=0, n_regs=64, n_ops=1000, depth=16, n_inputs=8, n_outputs=4,
             max_w=32) -> Netlist:
    rng = np.random.default_rng(seed)
    b = Builder()
    regs = [b.add_reg(int(rng.integers(1, max_w + 1)), int(rng.integers(0, 2**63)))
            for _ in range(n_regs)]
    for _ in range(n_inputs):
        b.add_input(int(rng.integers(1, max_w + 1)))
    levels = [[b.reg(r) for r in regs] + [b.input(p) for p in range(n_inputs)]
              + [b.const(int(rng.integers(1, max_w + 1)), int(rng.integers(0, 2**32)))
                 for _ in range(8)]]
    per_level = [n_ops // depth + (1 if i < n_ops % depth else 0) for i in range(depth)]
    for lv in range(1, depth + 1):
        cur = []
        below = [x for L in levels for x in L]
        prev = levels[-1]
        made = 0
        while made < per_level[lv - 1]:
            op = COMB11[int(rng.integers(0, len(COMB11)))]
            a = prev[int(rng.integers(0, len(prev)))]          # keeps the depth exact
            bb = below[int(rng.integers(0, len(below)))]
            if op == "NOT":
                n = b.not_(a)
            elif op == "MUX":
                s = below[int(rng.integers(0, len(below)))]
                n = b.mux(s, a, bb)
            elif op in ("SHL", "SHR"):
                if rng.random() < 0.9 and made + 2 <= per_level[lv - 1] and lv >= 2:
                    # the masking AND takes an amount from two levels down, so
                    # the shift still lands on this level
                    low = [x for L in levels[: lv - 1] for x in L]
                    bb = low[int(rng.integers(0, len(low)))]
                    msk = b.const(b.width_of(bb), _shift_mask(b.width_of(a)))
                    bb = b.op2("AND", bb, msk)
                    made += 1
                n = b.op2(op, a, bb, w=b.width_of(a))
            else:
                n = b.op2(op, a, bb)
            cur.append(n)
            made += 1
        levels.append(cur)
    top = [x for L in levels[-4:] for x in L]
    for r in regs:
        b.set_next(r, top[int(rng.integers(0, len(top)))])
    for _ in range(n_outputs):
        b.output(top[int(rng.integers(0, len(top)))])
    return b.build(name=f"tiny(seed={seed})", seed=seed)


# --------------------------------------------------------------------------
# Core: the single-core-shaped netlist.  Registers are 70% 1-bit and 30%
# 32/64-bit; every register's next value is a chain of operators whose depth
# follows a skewed distribution (mostly shallow, a few deep stragglers up to
# ~40).  Side operands come from leaves near the register (register-index
# locality), the inputs, constants, or recently built nodes (which creates the
# shared logic that makes fibers overlap).  Two 4096 x 64 memories with two
# registered read ports and one write port each; four 32-bit link registers
# that a mesh can rewire.
# --------------------------------------------------------------------------
@dataclasses.dataclass
class CoreParams:
    n_regs_1: int = 14000
    n_regs_32: int = 3000
    n_regs_64: int = 3000
    target_ops: int = 200_000
    max_depth: int = 40
    n_inputs: int = 8
    n_mems: int = 2
    mem_depth: int = 4096
    mem_width: int = 64
    n_links: int = 4
    n_outputs: int = 8
    p_share: float = 0.25        # side operand from the recent-node window
    window: int = 48
    reg_locality: int = 256


def _depth_targets(rng, n, max_depth):
    u = rng.random(n)
    d = np.where(u < 0.85, rng.integers(2, 12, n),
                 np.where(u < 0.99, rng.integers(12, 28, n), rng.integers(28, max_depth + 1, n)))
    return d


def gen_core(seed=1, params: CoreParams | None = None) -> Netlist:
    P = params or CoreParams()
    rng = np.random.default_rng(seed)
    b = Builder()
    widths = np.array([1] * P.n_regs_1 + [32] * P.n_regs_32 + [64] * P.n_regs_64)
    rng.shuffle(widths)
    R = len(widths)
    inits = rng.integers(0, 2**63, R, dtype=np.int64).astype(np.uint64) * np.uint64(2) \
        + rng.integers(0, 2, R).astype(np.uint64)
    regs = [b.add_reg(int(w), int(i) & ((1 << int(w)) - 1)) for w, i in zip(widths, inits)]
    in_w = [1, 1, 8, 16, 32, 32, 64, 64][: P.n_inputs] + [32] * max(0, P.n_inputs - 8)
    for w in in_w:
        b.add_input(w)
    inputs = [b.input(p) for p in range(P.n_inputs)]
    # special registers: link registers (32-bit) and memory read-data (64-bit)
    idx32 = [i for i in range(R) if widths[i] == 32]
    idx64 = [i for i in range(R) if widths[i] == 64]
    link_regs = idx32[: P.n_links]
    rd_regs = idx64[: 2 * P.n_mems]
    special = set(link_regs) | set(rd_regs)
    mems = []
    for m in range(P.n_mems):
        # every bit of every word is drawn, bit 0 and bit 63 included
        init = rng.integers(0, 2**64, P.mem_depth, dtype=np.uint64)
        mems.append(b.add_mem(P.mem_depth, P.mem_width, init))

    recent = []          # (node, depth) window of recently built operators
    depth_of = {}

    def dep(n):
        return depth_of.get(n, 0)

    def near_reg(r, want_w):
        lo, hi = max(0, r - P.reg_locality), min(R, r + P.reg_locality)
        for _ in range(8):
            q = int(rng.integers(lo, hi))
            if want_w is None or (widths[q] == 1) == (want_w == 1):
                return b.reg(q)
        return b.reg(q)

    consts = {}

    def const_of(w):
        # a small pool of constants per width keeps the node count honest
        key = (w, int(rng.integers(0, 4)))
        if key not in consts:
            consts[key] = b.const(w, int(rng.integers(0, 2**64, dtype=np.uint64)) & ((1 << w) - 1))
        return consts[key]

    def side(r, chain, cw, maxd):
        """A side operand: a recent node, a nearby register, an input or a constant."""
        u = rng.random()
        if u < P.p_share and recent:
            for _ in range(4):
                n, d = recent[int(rng.integers(0, len(recent)))]
                if d < maxd:
                    return n
        if u < 0.75:
            return near_reg(r, cw)
        if u < 0.9:
            return inputs[int(rng.integers(0, len(inputs)))]
        return const_of(cw)

    def chain_for(r, w, target):
        cur = side(r, None, w, 1) if rng.random() < 0.5 else near_reg(r, w)
        cur_d = dep(cur)
        steps = 0
        while cur_d < target or steps == 0:
            op = COMB11[int(rng.integers(0, len(COMB11)))]
            cw = max(b.width_of(cur), 1)
            x = side(r, cur, w if w > 1 else cw, cur_d + 1)
            if op == "NOT":
                n = b.not_(cur)
            elif op == "MUX":
                s = side(r, cur, 1, cur_d + 1)
                if b.width_of(s) != 1:
                    s2 = b.op2("LT", s, x)
                    depth_of[s2] = 1 + max(dep(s), dep(x))
                    s = s2
                n = b.mux(s, cur, x) if rng.random() < 0.5 else b.mux(s, x, cur)
            elif op in ("SHL", "SHR"):
                amt = x
                if rng.random() < 0.9:
                    msk = const_of_mask(b.width_of(amt), _shift_mask(b.width_of(cur)))
                    amt = b.op2("AND", amt, msk)
                    depth_of[amt] = 1 + dep(x)
                n = b.op2(op, cur, amt, w=b.width_of(cur))
            elif op in ("EQ", "LT"):
                n = b.op2(op, cur, x) if rng.random() < 0.5 else b.op2(op, x, cur)
            else:
                n = b.op2(op, cur, x) if rng.random() < 0.5 else b.op2(op, x, cur)
            d = 1 + max(dep(a) for a in (b.a0[n], b.a1[n], b.a2[n]) if a != NONE)
            depth_of[n] = d
            recent.append((n, d))
            if len(recent) > P.window:
                recent.pop(0)
            cur, cur_d = n, d
            steps += 1
            # widen a 1-bit chain of a wide register back to its width
            if w > 1 and b.width_of(cur) == 1 and cur_d < target:
                y = near_reg(r, w)
                n = b.op2("ADD", cur, y)
                depth_of[n] = 1 + max(cur_d, dep(y))
                cur, cur_d = n, depth_of[n]
        return cur

    mask_consts = {}

    def const_of_mask(w, v):
        key = (w, v)
        if key not in mask_consts:
            mask_consts[key] = b.const(w, v & ((1 << w) - 1))
        return mask_consts[key]

    targets = _depth_targets(rng, R, P.max_depth)
    # scale the depth targets so that the operator count lands near the target
    order = list(range(R))
    for r in order:
        if r in special:
            continue
        b.set_next(r, chain_for(r, int(widths[r]), int(targets[r])))
    # memories: two registered read ports and one write port each
    for m in range(P.n_mems):
        r0 = rd_regs[2 * m]
        for k in range(2):
            rr = rd_regs[2 * m + k]
            addr = chain_for(rr, 32, 4)
            b.set_next(rr, b.memrd(mems[m], addr))
        en = chain_for(r0, 1, 3)
        wa = chain_for(r0, 32, 4)
        wd = chain_for(r0, 64, 6)
        b.wport(mems[m], en, wa, wd)
    link_out = []
    for i, lr in enumerate(link_regs):
        lo = chain_for(lr, 32, 6)
        link_out.append(lo)
        b.set_next(lr, lo)           # loopback when the core stands alone
    for _ in range(P.n_outputs):
        r = int(rng.integers(0, R))
        b.output(chain_for(r, 32, 3))
    nl = b.build(name=f"core(seed={seed})", seed=seed)
    nl.meta["link_regs"] = link_regs
    nl.meta["link_out"] = link_out
    return nl


# --------------------------------------------------------------------------
# Replicated-tile SoC: copies of one core on a rows x cols mesh.  Each tile's
# four link registers take the facing link output of the neighbouring tile (a
# registered 32-bit hop); a small router per tile and direction adds a
# registered valid bit, a registered data stage and an arbitration mux.
# --------------------------------------------------------------------------
def gen_soc(rows, cols, core: Netlist, mesh_seed=2) -> Netlist:
    rng = np.random.default_rng(mesh_seed)
    T = rows * cols
    N, R, I, O = core.n_nodes, core.n_regs, core.n_inputs, core.n_outputs
    Mm, W = core.n_mems, core.n_wports
    link_regs = core.meta["link_regs"]
    link_out = core.meta["link_out"]
    # router per tile: per direction d: valid (1b), data (32b), arb (1b)
    # nodes appended after all tile copies
    rb = Builder()
    # replicate the tiles with index offsets (vectorised)
    def rep(a, off_per_tile, none_keep=False):
        a = np.asarray(a)
        out = np.concatenate([a.astype(np.uint64) + np.uint64(off_per_tile * t) for t in range(T)])
        if none_keep:
            mask = np.tile(a.astype(np.uint64) == NONE, T)
            out[mask] = NONE
        return out

    op = np.tile(core.op, T)
    width = np.tile(core.width, T)
    arg = rep(core.arg.reshape(-1), N, none_keep=True).astype(np.uint32).reshape(-1, 3)
    imm = np.tile(core.imm, T).copy()
    # leaves carry indices in imm: registers, inputs and memories shift per tile
    tile_of = np.repeat(np.arange(T, dtype=np.uint64), N)
    for code, per in ((OPS["REG"], R), (OPS["INPUT"], I), (OPS["MEMRD"], Mm)):
        sel = op == code
        imm[sel] = imm[sel] + tile_of[sel] * np.uint64(per)
    reg_width = np.tile(core.reg_width, T)
    reg_init = np.tile(core.reg_init, T)
    reg_next = rep(core.reg_next, N).astype(np.uint32)
    in_width = np.tile(core.in_width, T)
    out_node = rep(core.out_node, N).astype(np.uint32)
    mem_depth = np.tile(core.mem_depth, T)
    mem_width = np.tile(core.mem_width, T)
    mem_init = np.tile(core.mem_init, T)
    wp_mem = rep(core.wp_mem, Mm).astype(np.uint32)
    wp_en = rep(core.wp_en, N).astype(np.uint32)
    wp_addr = rep(core.wp_addr, N).astype(np.uint32)
    wp_data = rep(core.wp_data, N).astype(np.uint32)

    # router logic, built with a Builder whose node/register indices are then
    # offset behind the tiles
    base_node, base_reg = T * N, T * R
    dirs = [(-1, 0), (0, 1), (1, 0), (0, -1)]      # N E S W
    opp = [2, 3, 0, 1]
    rregs = {}
    for t in range(T):
        for d in range(4):
            v = rb.add_reg(1, int(rng.integers(0, 2)))
            dd = rb.add_reg(32, int(rng.integers(0, 2**32)))
            a = rb.add_reg(1, int(rng.integers(0, 2)))
            rregs[(t, d)] = (v, dd, a)
    # external references into the tiles are expressed as placeholder REG
    # nodes of the tile registers; they are rewritten below
    ext = {}

    def tile_reg_node(t, r):
        key = (t, r)
        if key not in ext:
            ext[key] = rb._node("REG", int(core.reg_width[r]), (), 0)
        return ext[key]

    for t in range(T):
        rr, cc = divmod(t, cols)
        for d, (dr, dc) in enumerate(dirs):
            v, dd, a = rregs[(t, d)]
            # arbitration: alternate between the tile's own link output and
            # the data stage arriving from the next direction
            nxt_d = (d + 1) % 4
            _, dd2, _ = rregs[(t, nxt_d)]
            own = tile_reg_node(t, link_regs[d])
            arb_next = rb.op2("XOR", rb.not_(rb.reg(a)), rb.reg(v))
            rb.set_next(a, arb_next)
            sel = rb.mux(rb.reg(a), own, rb.reg(dd2))
            rb.set_next(dd, rb.op2("XOR", sel, rb.op2("ADD", rb.reg(dd), rb.const(32, 0x9E37 + d))))
            rb.set_next(v, rb.op2("OR", rb.op2("EQ", sel, rb.reg(dd)), rb.op2("LT", rb.reg(dd), own)))
    rnl = rb.build(name="router")
    # offset router arrays
    r_op, r_w, r_arg, r_imm = rnl.op, rnl.width, rnl.arg.astype(np.uint64), rnl.imm.copy()
    r_arg_off = np.where(r_arg == NONE, NONE, r_arg + base_node).astype(np.uint32)
    r_imm = r_imm.copy()
    is_reg = r_op == OPS["REG"]
    r_imm[is_reg] += np.uint64(base_reg)
    for (t, r), n in ext.items():
        r_imm[n] = np.uint64(t * R + r)
    op = np.concatenate([op, r_op])
    width = np.concatenate([width, r_w])
    arg = np.concatenate([arg, r_arg_off])
    imm = np.concatenate([imm, r_imm])
    reg_width = np.concatenate([reg_width, rnl.reg_width])
    reg_init = np.concatenate([reg_init, rnl.reg_init])
    reg_next = np.concatenate([reg_next, (rnl.reg_next.astype(np.uint64) + base_node).astype(np.uint32)])
    # link registers: tile t's link register for direction d takes the router
    # data stage of the neighbour facing it (a registered hop); at the mesh
    # edge it keeps the loopback of the standalone core
    x_op, x_w, x_arg, x_imm = [], [], [], []
    nxt = len(op)
    for t in range(T):
        rr, cc = divmod(t, cols)
        for d, (dr, dc) in enumerate(dirs):
            r2, c2 = rr + dr, cc + dc
            if 0 <= r2 < rows and 0 <= c2 < cols:
                nb = r2 * cols + c2
                _, dd_nb, _ = rregs[(nb, opp[d])]
                node = nxt
                x_op.append(OPS["REG"]); x_w.append(32); x_arg.append((NONE, NONE, NONE))
                x_imm.append(base_reg + dd_nb)
                x_op.append(OPS["XOR"]); x_w.append(32)
                x_arg.append((node, N * t + link_out[d], NONE)); x_imm.append(0)
                reg_next[t * R + link_regs[d]] = nxt + 1
                nxt += 2
    if x_op:
        op = np.concatenate([op, np.array(x_op, np.uint8)])
        width = np.concatenate([width, np.array(x_w, np.uint8)])
        arg = np.concatenate([arg, np.array(x_arg, np.uint32).reshape(-1, 3)])
        imm = np.concatenate([imm, np.array(x_imm, np.uint64)])
    nl = Netlist(op=op.astype(np.uint8), width=width.astype(np.uint8), arg=arg.astype(np.uint32),
                 imm=imm.astype(np.uint64), reg_width=reg_width.astype(np.uint8),
                 reg_init=reg_init.astype(np.uint64), reg_next=reg_next.astype(np.uint32),
                 in_width=in_width.astype(np.uint8), out_node=out_node.astype(np.uint32),
                 mem_depth=mem_depth.astype(np.uint32), mem_width=mem_width.astype(np.uint8),
                 mem_init=mem_init.astype(np.uint64), wp_mem=wp_mem, wp_en=wp_en,
                 wp_addr=wp_addr, wp_data=wp_data, name=f"soc({rows}x{cols})",
                 meta=dict(tiles=T, rows=rows, cols=cols, mesh_seed=mesh_seed))
    return nl


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------
def workload(name: str, **kw) -> Netlist:
    """tiny | core | soc8 | soc48, with the fixed seeds of the workload table."""
    if name == "tiny":
        return gen_tiny(seed=kw.get("seed", 0))
    if name == "core":
        return gen_core(seed=kw.get("seed", 1))
    if name == "soc8":
        return gen_soc(2, 4, gen_core(seed=1), mesh_seed=2)
    if name == "soc48":
        return gen_soc(8, 6, gen_core(seed=1), mesh_seed=4)
    if name == "core_clocks":
        return add_clock_domains(gen_core(seed=1), seed=kw.get("seed", 7))
    raise KeyError(name)


def add_clock_domains(nl: Netlist, seed=7, divisors=(2, 3, 8), n_gated=1, frac=0.5) -> Netlist:
    """A copy of nl in which a share `frac` of the registers, drawn at random,
    runs on a divided or gated clock instead of the top clock (Sec. 5.3:
    one top clock and any number of gated or divided ones).

    Per divisor k one 8-bit divider register counts 0..k-1 on the top clock;
    its domain's enable is (divider == k-1), one tick every k cycles.  Per
    gated domain one new 1-bit input port is the enable (a testbench-driven
    clock gate).  The domains are spread uniformly over the chosen registers;
    registers that already had an enable keep it."""
    assert nl.reg_en is None or len(nl.reg_en) == nl.n_regs
    rng = np.random.default_rng(seed)
    b = Builder()
    R0, N0, I0 = nl.n_regs, nl.n_nodes, nl.n_inputs
    enables = []
    div_regs = []
    for k in divisors:
        assert 2 <= k <= 255
        d = b.add_reg(8, 0)
        cur = b.reg(d)
        tick = b.op2("EQ", cur, b.const(8, k - 1))
        b.set_next(d, b.mux(tick, b.const(8, 0), b.op2("ADD", cur, b.const(8, 1)), w=8))
        enables.append(tick)
        div_regs.append(d)
    for _ in range(n_gated):
        enables.append(b.input(b.add_input(1)))
    tail = b.build()
    # renumber the new nodes, registers and ports after nl's own
    op = np.concatenate([nl.op, tail.op])
    width = np.concatenate([nl.width, tail.width])
    targ = tail.arg.astype(np.uint64)
    targ = np.where(targ == NONE, NONE, targ + N0).astype(np.uint32)
    arg = np.concatenate([nl.arg, targ.reshape(-1, 3)])
    timm = tail.imm.copy()
    timm[tail.op == OPS["REG"]] += np.uint64(R0)
    timm[tail.op == OPS["INPUT"]] += np.uint64(I0)
    imm = np.concatenate([nl.imm, timm])
    reg_next = np.concatenate([nl.reg_next, (tail.reg_next.astype(np.uint64) + N0).astype(np.uint32)])
    en = np.full(R0 + tail.n_regs, NONE, np.uint32)
    if nl.reg_en is not None:
        en[:R0] = nl.reg_en
    free = np.flatnonzero(en[:R0] == NONE)
    pick = rng.permutation(free)[: int(round(frac * len(free)))]
    dom = rng.integers(0, len(enables), len(pick))
    en[pick] = np.array(enables, np.uint64)[dom].astype(np.uint32) + np.uint32(N0)
    meta = dict(nl.meta, clock_domains=[f"div{k}" for k in divisors] + ["gated"] * n_gated,
                gated_regs=int(len(pick)), divider_regs=[R0 + d for d in div_regs])
    return Netlist(
        op=op, width=width, arg=arg, imm=imm,
        reg_width=np.concatenate([nl.reg_width, tail.reg_width]),
        reg_init=np.concatenate([nl.reg_init, tail.reg_init]),
        reg_next=reg_next, in_width=np.concatenate([nl.in_width, tail.in_width]),
        out_node=nl.out_node.copy(), mem_depth=nl.mem_depth.copy(), mem_width=nl.mem_width.copy(),
        mem_init=nl.mem_init.copy(), wp_mem=nl.wp_mem.copy(), wp_en=nl.wp_en.copy(),
        wp_addr=nl.wp_addr.copy(), wp_data=nl.wp_data.copy(),
        name=(nl.name + "+clocks") if nl.name else "clocks", meta=meta, reg_en=en)


STIM_SEED_BASE = 0x5EED0000


# --------------------------------------------------------------------------
# Small circuits with known behaviour (used by the pins and parity tests)
# --------------------------------------------------------------------------
def counter(w) -> Netlist:
    b = Builder()
    r = b.add_reg(w, 0)
    b.set_next(r, b.op2("ADD", b.reg(r), b.const(w, 1)))
    b.output(b.reg(r))
    return b.build(name=f"counter{w}")


def divided_counter(w, k) -> Netlist:
    """A w-bit counter on a clock divided by k: register 0 counts 0..k-1 on the
    top clock, register 1 adds 1 only in cycles where register 0 is k-1, so
    after t cycles it holds floor(t / k) mod 2**w."""
    b = Builder()
    d = b.add_reg(8, 0)
    r = b.add_reg(w, 0)
    tick = b.op2("EQ", b.reg(d), b.const(8, k - 1))
    b.set_next(d, b.mux(tick, b.const(8, 0), b.op2("ADD", b.reg(d), b.const(8, 1)), w=8))
    b.set_next(r, b.op2("ADD", b.reg(r), b.const(w, 1)))
    b.set_enable(r, tick)
    b.output(b.reg(r))
    return b.build(name=f"divided_counter{w}_{k}")


def gated_counter(w) -> Netlist:
    """A w-bit counter whose clock is gated by the 1-bit input port 0: it
    counts the cycles in which the port was 1."""
    b = Builder()
    g = b.add_input(1)
    r = b.add_reg(w, 0)
    b.set_next(r, b.op2("ADD", b.reg(r), b.const(w, 1)))
    b.set_enable(r, b.input(g))
    return b.build(name=f"gated_counter{w}")


def lfsr(n, taps) -> Netlist:
    """Fibonacci LFSR of n 1-bit registers s[0..n-1], shifting towards higher
    indices: s[0]' = XOR of the tapped bits (1-based tap positions), s[i]' = s[i-1]."""
    b = Builder()
    s = [b.add_reg(1, 1 if i == 0 else 0) for i in range(n)]
    fb = b.reg(s[taps[0] - 1])
    for t in taps[1:]:
        fb = b.op2("XOR", fb, b.reg(s[t - 1]))
    b.set_next(s[0], fb)
    for i in range(1, n):
        b.set_next(s[i], b.reg(s[i - 1]))
    return b.build(name=f"lfsr{n}")


def xorshift32(seed=2463534242) -> Netlist:
    """One 32-bit register updated by x ^= x<<13; x ^= x>>17; x ^= x<<5."""
    b = Builder()
    r = b.add_reg(32, seed)
    x = b.reg(r)
    x = b.op2("XOR", x, b.op2("SHL", x, b.const(32, 13), w=32))
    x = b.op2("XOR", x, b.op2("SHR", x, b.const(32, 17), w=32))
    x = b.op2("XOR", x, b.op2("SHL", x, b.const(32, 5), w=32))
    b.set_next(r, x)
    return b.build(name="xorshift32")


def prng_array(n, seed=0x5EED) -> Netlist:
    """n independent xorshift32 generators (three shifts and three XORs each,
    the synchronization experiment of Parendi Sec. 4.1): every register is a
    fiber on its own and no fiber reads another's state.  Built directly as
    arrays (n reaches a million)."""
    n_nodes = 3 + 7 * n
    op = np.empty(n_nodes, np.uint8)
    arg = np.full((n_nodes, 3), NONE, np.uint32)
    imm = np.zeros(n_nodes, np.uint64)
    op[:3] = OPS["CONST"]
    imm[:3] = (13, 17, 5)
    base = 3 + 7 * np.arange(n, dtype=np.int64)
    op[base] = OPS["REG"]
    imm[base] = np.arange(n, dtype=np.uint64)
    for k, (o, a0, a1) in enumerate([("SHL", 0, None), ("XOR", 0, 1), ("SHR", 2, None),
                                      ("XOR", 2, 3), ("SHL", 4, None), ("XOR", 4, 5)], start=1):
        op[base + k] = OPS[o]
        arg[base + k, 0] = base + a0
        # shift amounts are the shared constants 13, 17, 5
        arg[base + k, 1] = (base + a1) if a1 is not None else {1: 0, 3: 1, 5: 2}[k]
    rng = np.random.default_rng(seed)
    init = rng.integers(1, 2**32, n, dtype=np.uint64)
    return Netlist(
        op=op, width=np.full(n_nodes, 32, np.uint8), arg=arg, imm=imm,
        reg_width=np.full(n, 32, np.uint8), reg_init=init, reg_next=(base + 6).astype(np.uint32),
        in_width=np.zeros(0, np.uint8), out_node=np.zeros(0, np.uint32),
        mem_depth=np.zeros(0, np.uint32), mem_width=np.zeros(0, np.uint8), mem_init=np.zeros(0, np.uint64),
        wp_mem=np.zeros(0, np.uint32), wp_en=np.zeros(0, np.uint32), wp_addr=np.zeros(0, np.uint32),
        wp_data=np.zeros(0, np.uint32), name=f"prng{n}", meta=dict(seed=seed))


def mul_mix(seed=11, widths=(1, 7, 32, 33, 64), per_width=8) -> Netlist:
    """Word-level multipliers (the optional MUL operator) at widths 1, 7,
    32, 33 and 64: per width, per_width registers each take
    ADD(MUL(MUL(x, y), port), MUL(own, odd constant)) of two other
    registers x, y of the width and the width's input port, so that products
    wrap past 64 bits and are masked back to narrow widths every cycle.  A
    MUL of operands of different widths and one register of every width
    feeding an output exercise the zero extension."""
    rng = np.random.default_rng(seed)
    b = Builder()
    ports = {w: b.add_input(w) for w in widths}
    regs = {w: [b.add_reg(w, int(rng.integers(0, 2**64, dtype=np.uint64))) for _ in range(per_width)]
            for w in widths}
    for w in widths:
        rs = regs[w]
        for k, r in enumerate(rs):
            x, y = b.reg(rs[(k + 1) % per_width]), b.reg(rs[(k + 3) % per_width])
            p = b.op2("MUL", b.op2("MUL", x, y, w=w), b.input(ports[w]), w=w)
            odd = int(rng.integers(0, 2**64, dtype=np.uint64)) | 1
            b.set_next(r, b.op2("ADD", p, b.op2("MUL", b.reg(r), b.const(w, odd), w=w), w=w))
        b.output(b.reg(rs[0]))
    # mixed widths: a 33-bit value times a 64-bit one, kept at 7 bits
    m = b.op2("MUL", b.reg(regs[33][1]), b.reg(regs[64][2]), w=7)
    b.output(m)
    return b.build(name=f"mul_mix(seed={seed})")


def swap_pair(w=16, a0=0x1234, b0=0xBEEF) -> Netlist:
    b = Builder()
    ra, rb_ = b.add_reg(w, a0), b.add_reg(w, b0)
    b.set_next(ra, b.reg(rb_))
    b.set_next(rb_, b.reg(ra))
    return b.build(name="swap")


def _bits_in(b, port, n):
    """n single-bit nodes taken from an n-bit input port (bit i via shift+and)."""
    x = b.input(port)
    one = b.const(1, 1)
    out = []
    for i in range(n):
        sh = b.op2("SHR", x, b.const(8, i), w=b.width_of(x))
        out.append(b.op2("AND", sh, one, w=1))
    return out


def _bits_out(b, bits):
    """Assemble single bits into a word: sum of bit_i << i."""
    w = len(bits)
    acc = None
    for i, bit in enumerate(bits):
        term = b.op2("SHL", bit, b.const(8, i), w=w) if i else b.op2("OR", bit, b.const(w, 0), w=w)
        acc = term if acc is None else b.op2("OR", acc, term, w=w)
    return acc


def ripple_adder(n=4) -> Netlist:
    """Gate-level n-bit ripple-carry adder from 1-bit AND/OR/XOR.  Inputs: port 0
    = a (n bits), port 1 = b (n bits).  One (n+1)-bit register holds a + b."""
    b = Builder()
    b.add_input(n); b.add_input(n)
    A, B = _bits_in(b, 0, n), _bits_in(b, 1, n)
    c = b.const(1, 0)
    s = []
    for i in range(n):
        t = b.op2("XOR", A[i], B[i])
        s.append(b.op2("XOR", t, c))
        c = b.op2("OR", b.op2("AND", A[i], B[i]), b.op2("AND", t, c))
    s.append(c)
    r = b.add_reg(n + 1, 0)
    b.set_next(r, _bits_out(b, s))
    return b.build(name=f"adder{n}")


def array_multiplier(n=4) -> Netlist:
    """Gate-level n x n array multiplier: partial products with AND, rows
    accumulated by ripple-carry adders of 1-bit gates.  One 2n-bit register."""
    b = Builder()
    b.add_input(n); b.add_input(n)
    A, B = _bits_in(b, 0, n), _bits_in(b, 1, n)
    zero = b.const(1, 0)
    acc = [zero] * (2 * n)
    for j in range(n):
        pp = [zero] * (2 * n)
        for i in range(n):
            pp[i + j] = b.op2("AND", A[i], B[j])
        c = zero
        out = []
        for k in range(2 * n):
            t = b.op2("XOR", acc[k], pp[k])
            out.append(b.op2("XOR", t, c))
            c = b.op2("OR", b.op2("AND", acc[k], pp[k]), b.op2("AND", t, c))
        acc = out
    r = b.add_reg(2 * n, 0)
    b.set_next(r, _bits_out(b, acc))
    return b.build(name=f"mult{n}")


def comparators(n=4) -> Netlist:
    """Gate-level n-bit equality and unsigned less-than from 1-bit
    AND/OR/XOR/NOT.  Two 1-bit registers: eq, lt."""
    b = Builder()
    b.add_input(n); b.add_input(n)
    A, B = _bits_in(b, 0, n), _bits_in(b, 1, n)
    eq = b.const(1, 1)
    lt = b.const(1, 0)
    for i in reversed(range(n)):            # from the most significant bit
        same = b.not_(b.op2("XOR", A[i], B[i]))
        a_lt_b = b.op2("AND", b.not_(A[i]), B[i])
        lt = b.op2("OR", lt, b.op2("AND", eq, a_lt_b))
        eq = b.op2("AND", eq, same)
    re, rl = b.add_reg(1, 0), b.add_reg(1, 0)
    b.set_next(re, eq)
    b.set_next(rl, lt)
    return b.build(name=f"cmp{n}")
