"""ctypes wrapper around oracle.c -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It never touches the GPU library and the
GPU library never touches it.

The oracle is the plain definition of cycle-accurate full-cycle simulation
(Parendi Sec. 3 and Sec. 3.2): a single-threaded topological-order interpreter
over the data-dependence graph whose registers are split into current and next
values.  See oracle.c for the semantics it implements.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_ARG, E_NETLIST, E_COMB_LOOP, E_UNSUPPORTED, E_CONE = 0, -1, -2, -3, -4, -5


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc -O2 into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Netlist(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_uint32), ("op", C.c_void_p), ("width", C.c_void_p),
        ("arg", C.c_void_p), ("imm", C.c_void_p),
        ("n_regs", C.c_uint32), ("reg_width", C.c_void_p), ("reg_init", C.c_void_p),
        ("reg_next", C.c_void_p),
        ("n_inputs", C.c_uint32), ("in_width", C.c_void_p),
        ("n_outputs", C.c_uint32), ("out_node", C.c_void_p),
        ("n_mems", C.c_uint32), ("mem_depth", C.c_void_p), ("mem_width", C.c_void_p),
        ("mem_init", C.c_void_p),
        ("n_wports", C.c_uint32), ("wp_mem", C.c_void_p), ("wp_en", C.c_void_p),
        ("wp_addr", C.c_void_p), ("wp_data", C.c_void_p),
        ("reg_en", C.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        u64, u32, p = C.c_uint64, C.c_uint32, C.c_void_p
        _lib.orc_hash.restype = u64
        _lib.orc_hash.argtypes = [u64]
        _lib.orc_stim.restype = u64
        _lib.orc_stim.argtypes = [u64, u32, u64]
        _lib.orc_eval.restype = u64
        _lib.orc_eval.argtypes = [u32, u32, u64, u64, u64]
        _lib.orc_new.restype = C.c_int
        _lib.orc_new.argtypes = [C.POINTER(_Netlist), u64, C.POINTER(p)]
        _lib.orc_free.argtypes = [p]
        _lib.orc_set_seed.argtypes = [p, u64]
        _lib.orc_set_inputs.argtypes = [p, u64, u64, p]
        _lib.orc_step.restype = C.c_int
        _lib.orc_step.argtypes = [p, u64, p]
        _lib.orc_step_partitioned.restype = C.c_int
        _lib.orc_step_partitioned.argtypes = [p, u64, u32, p, p, p, p]
        _lib.orc_cycle.restype = u64
        _lib.orc_cycle.argtypes = [p]
        _lib.orc_set_cycle.argtypes = [p, u64]
        _lib.orc_digest.restype = u64
        _lib.orc_digest.argtypes = [p]
        for f in ("orc_read_regs", "orc_write_regs", "orc_read_outputs"):
            getattr(_lib, f).argtypes = [p, p]
        for f in ("orc_read_mem", "orc_write_mem"):
            getattr(_lib, f).restype = C.c_int
            getattr(_lib, f).argtypes = [p, u32, p]
    return _lib


def hash64(x: int) -> int:
    return lib().orc_hash(x & (2**64 - 1))


def stim(seed: int, port: int, t: int) -> int:
    return lib().orc_stim(seed & (2**64 - 1), port, t)


def eval_op(op: int, w: int, a: int, b: int = 0, c: int = 0) -> int:
    return lib().orc_eval(op, w, a, b, c)


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


class Sim:
    """One simulated instance.  ``nl`` is any object with the netlist arrays
    (the attribute names of the seeded generator's Netlist)."""

    def __init__(self, nl, seed: int = 0, order_seed: int = 0):
        L = lib()
        self.nl = nl
        # keep contiguous copies alive for the duration of orc_new
        keep = dict(
            op=np.ascontiguousarray(nl.op, np.uint8),
            width=np.ascontiguousarray(nl.width, np.uint8),
            arg=np.ascontiguousarray(nl.arg, np.uint32),
            imm=np.ascontiguousarray(nl.imm, np.uint64),
            reg_width=np.ascontiguousarray(nl.reg_width, np.uint8),
            reg_init=np.ascontiguousarray(nl.reg_init, np.uint64),
            reg_next=np.ascontiguousarray(nl.reg_next, np.uint32),
            in_width=np.ascontiguousarray(nl.in_width, np.uint8),
            out_node=np.ascontiguousarray(nl.out_node, np.uint32),
            mem_depth=np.ascontiguousarray(nl.mem_depth, np.uint32),
            mem_width=np.ascontiguousarray(nl.mem_width, np.uint8),
            mem_init=np.ascontiguousarray(nl.mem_init, np.uint64),
            wp_mem=np.ascontiguousarray(nl.wp_mem, np.uint32),
            wp_en=np.ascontiguousarray(nl.wp_en, np.uint32),
            wp_addr=np.ascontiguousarray(nl.wp_addr, np.uint32),
            wp_data=np.ascontiguousarray(nl.wp_data, np.uint32),
        )
        en = getattr(nl, "reg_en", None)
        if en is not None:
            keep["reg_en"] = np.ascontiguousarray(en, np.uint32)
            assert keep["reg_en"].shape == keep["reg_width"].shape
        s = _Netlist()
        s.n_nodes = len(keep["op"])
        s.n_regs = len(keep["reg_width"])
        s.n_inputs = len(keep["in_width"])
        s.n_outputs = len(keep["out_node"])
        s.n_mems = len(keep["mem_depth"])
        s.n_wports = len(keep["wp_mem"])
        for k, v in keep.items():
            setattr(s, k, _ptr(v))
        h = C.c_void_p()
        rc = L.orc_new(C.byref(s), order_seed, C.byref(h))
        if rc != OK:
            raise OracleError(rc, "orc_new")
        self._h = h
        self.n_regs, self.n_outputs, self.n_inputs = s.n_regs, s.n_outputs, s.n_inputs
        self.n_wports = s.n_wports
        self.mem_depth = keep["mem_depth"].copy()
        L.orc_set_seed(h, seed)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_free(h)
            self._h = None

    def set_seed(self, seed: int):
        lib().orc_set_seed(self._h, seed & (2**64 - 1))

    def set_inputs(self, first_cycle: int, vals: np.ndarray):
        """vals: [n_cycles][n_inputs] uint64, applied from first_cycle."""
        v = np.ascontiguousarray(vals, np.uint64)
        lib().orc_set_inputs(self._h, first_cycle, v.shape[0], _ptr(v))

    def step(self, n_cycles: int, digests: bool = False):
        d = np.zeros(max(n_cycles, 1), np.uint64) if digests else None
        rc = lib().orc_step(self._h, n_cycles, _ptr(d))
        if rc != OK:
            raise OracleError(rc, "orc_step")
        return d[:n_cycles] if digests else None

    def step_partitioned(self, n_cycles: int, sink_to_proc, proc_off=None,
                         proc_nodes=None, digests: bool = False):
        stp = np.ascontiguousarray(sink_to_proc, np.uint32)
        n_proc = int(stp.max()) + 1 if stp.size else 1
        off = nodes = None
        if proc_off is not None:
            off = np.ascontiguousarray(proc_off, np.uint32)
            nodes = np.ascontiguousarray(proc_nodes, np.uint32)
            n_proc = len(off) - 1
        d = np.zeros(max(n_cycles, 1), np.uint64) if digests else None
        rc = lib().orc_step_partitioned(self._h, n_cycles, n_proc, _ptr(stp),
                                        _ptr(off) if off is not None else None,
                                        _ptr(nodes) if nodes is not None else None,
                                        _ptr(d))
        if rc != OK:
            raise OracleError(rc, "orc_step_partitioned")
        return d[:n_cycles] if digests else None

    @property
    def cycle(self) -> int:
        return lib().orc_cycle(self._h)

    def set_cycle(self, c: int):
        lib().orc_set_cycle(self._h, c)

    def digest(self) -> int:
        return lib().orc_digest(self._h)

    def regs(self) -> np.ndarray:
        out = np.zeros(max(self.n_regs, 1), np.uint64)
        lib().orc_read_regs(self._h, _ptr(out))
        return out[: self.n_regs]

    def write_regs(self, vals):
        v = np.ascontiguousarray(vals, np.uint64)
        lib().orc_write_regs(self._h, _ptr(v))

    def outputs(self) -> np.ndarray:
        out = np.zeros(max(self.n_outputs, 1), np.uint64)
        lib().orc_read_outputs(self._h, _ptr(out))
        return out[: self.n_outputs]

    def mem(self, m: int) -> np.ndarray:
        out = np.zeros(int(self.mem_depth[m]), np.uint64)
        rc = lib().orc_read_mem(self._h, m, _ptr(out))
        if rc != OK:
            raise OracleError(rc, "orc_read_mem")
        return out

    def write_mem(self, m: int, vals):
        v = np.ascontiguousarray(vals, np.uint64)
        rc = lib().orc_write_mem(self._h, m, _ptr(v))
        if rc != OK:
            raise OracleError(rc, "orc_write_mem")
