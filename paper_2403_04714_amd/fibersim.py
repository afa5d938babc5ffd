"""Python binding of libfibersim (include/fibersim.h): argument marshalling
only.  Every step of the simulation runs in the library's HIP kernels; torch
supplies device memory (workspaces, digest buffers) and the stream.

Importing this module loads ``libfibersim.so`` from the package directory and
fails loudly when it is missing: there is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfibersim.so")

OK = 0
E_ARG, E_NETLIST, E_COMB_LOOP, E_UNSUPPORTED, E_CAPACITY, E_DEVICE, E_STATE, E_BUSY, E_INTERNAL = \
    -1, -2, -3, -4, -5, -6, -7, -8, -9
PACK_SLB, PACK_FIBERS, PACK_SINGLE, PACK_HYPER = 0, 1, 2, 3
LAUNCH_AUTO, LAUNCH_PERSISTENT, LAUNCH_PER_CYCLE, LAUNCH_GRAPH = 0, 1, 2, 3
FORM_AUTO, FORM_BATCHED, FORM_PLAIN = 0, 1, 2
STAGE_AUTO, STAGE_LDS, STAGE_GLOBAL = 0, 1, 2


class FsimError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


class Netlist(C.Structure):
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


class Partition(C.Structure):
    _fields_ = [("n_sinks", C.c_uint32), ("sink_to_process", C.c_void_p)]


class CompileOpts(C.Structure):
    _fields_ = [("pack", C.c_uint32), ("target_processes", C.c_uint32),
                ("max_process_nodes", C.c_uint32)]


class DesignInfo(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_uint32), ("n_live_ops", C.c_uint32), ("n_regs", C.c_uint32),
        ("n_sinks", C.c_uint32), ("n_processes", C.c_uint32), ("max_depth", C.c_uint32),
        ("sum_fiber_ops", C.c_uint64), ("sum_process_ops", C.c_uint64),
        ("dup_fiber", C.c_double), ("dup_process", C.c_double),
        ("max_fiber_cost", C.c_uint64), ("max_process_cost", C.c_uint64),
        ("program_bytes", C.c_uint64), ("max_process_levels", C.c_uint32),
        ("max_process_nodes", C.c_uint32), ("compile_seconds", C.c_double),
        ("plain_max_slots", C.c_uint32), ("plain_max_chunks", C.c_uint32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SimOpts(C.Structure):
    _fields_ = [("launch", C.c_uint32), ("wg_threads", C.c_uint32), ("grid", C.c_uint32),
                ("graph_cycles", C.c_uint32), ("form", C.c_uint32), ("stage", C.c_uint32),
                ("tiles_per_wave", C.c_uint32)]


# every symbol include/fibersim.h declares, with its signature
_P, _U32, _U64, _I = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
SIGNATURES = {
    "fsim_last_error": (C.c_char_p, []),
    "fsim_ctx_create": (_I, [C.c_int, _P, _P]),
    "fsim_ctx_destroy": (None, [_P]),
    "fsim_ctx_device": (_I, [_P, _P, _P, _P]),
    "fsim_design_load": (_I, [_P, _P, _P, _P, _P]),
    "fsim_design_info": (_I, [_P, _P]),
    "fsim_design_info_get": (_I, [_P, _P]),
    "fsim_design_partition": (_I, [_P, _P, _P, _P]),
    "fsim_design_free": (None, [_P]),
    "fsim_design_batched_info": (_I, [_P, _P, _P, _P, _P, _P]),
    "fsim_sim_footprint": (_I, [_P, _U32, _P]),
    "fsim_sim_create": (_I, [_P, _U32, _P, C.c_size_t, _P, _P]),
    "fsim_sim_destroy": (None, [_P]),
    "fsim_set_stimulus_seed": (_I, [_P, _U64]),
    "fsim_set_inputs": (_I, [_P, _U64, _U32, _P]),
    "fsim_step": (_I, [_P, _U64]),
    "fsim_sync": (_I, [_P]),
    "fsim_cycle": (_U64, [_P]),
    "fsim_read_regs": (_I, [_P, _U32, _P]),
    "fsim_read_regs_noalloc": (_I, [_P, _U32, _P]),
    "fsim_write_regs": (_I, [_P, _U32, _P]),
    "fsim_read_outputs": (_I, [_P, _U32, _P]),
    "fsim_read_mem": (_I, [_P, _U32, _U32, _P]),
    "fsim_write_mem": (_I, [_P, _U32, _U32, _P]),
    "fsim_set_cycle": (_I, [_P, _U64]),
    "fsim_enable_digest": (_I, [_P, _P, _U64]),
    "fsim_enable_trace": (_I, [_P, _P, _U64, _P]),
    "fsim_sim_layout": (_I, [_P, _P, _P, _P, _P]),
    "fsim_server_create": (_I, [_P, C.c_size_t, _P, _P]),
    "fsim_server_submit": (_I, [_P, _P, _U32, _U64, _U64, _P]),
    "fsim_server_poll": (_I, [_P, _U64, _P]),
    "fsim_server_wait": (_I, [_P, _U64, C.c_double]),
    "fsim_server_result": (_I, [_P, _U64, _U32, _P, _P]),
    "fsim_server_cancel": (_I, [_P, _U64]),
    "fsim_server_release": (_I, [_P, _U64]),
    "fsim_server_stats_get": (_I, [_P, _P]),
    "fsim_server_destroy": (None, [_P]),
}

JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_CANCELLED, JOB_FAILED = 0, 1, 2, 3, 4


class ServerOpts(C.Structure):
    _fields_ = [("quantum_cycles", C.c_uint32), ("max_jobs", C.c_uint32), ("max_queue", C.c_uint32),
                ("host_cycle_ns", C.c_uint32)]


class JobStatus(C.Structure):
    _fields_ = [("state", C.c_int32), ("n_instances", C.c_uint32), ("cycles_done", C.c_uint64),
                ("n_cycles", C.c_uint64), ("device_bytes", C.c_uint64), ("t_submit", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [(k, C.c_uint64) for k in ("submitted", "completed", "cancelled", "rejected", "failed",
                                          "running", "queued", "quanta", "instance_cycles")] + \
               [("busy_seconds", C.c_double), ("elapsed_seconds", C.c_double),
                ("hbm_used", C.c_uint64), ("hbm_budget", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2403_04714_amd.build` (no fallback exists)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc, where):
    if rc != OK:
        msg = lib().fsim_last_error().decode(errors="replace")
        raise FsimError(rc, where, msg)


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


def _netlist_struct(nl):
    keep = dict(
        op=np.ascontiguousarray(nl.op, np.uint8), width=np.ascontiguousarray(nl.width, np.uint8),
        arg=np.ascontiguousarray(nl.arg, np.uint32), imm=np.ascontiguousarray(nl.imm, np.uint64),
        reg_width=np.ascontiguousarray(nl.reg_width, np.uint8),
        reg_init=np.ascontiguousarray(nl.reg_init, np.uint64),
        reg_next=np.ascontiguousarray(nl.reg_next, np.uint32),
        in_width=np.ascontiguousarray(nl.in_width, np.uint8),
        out_node=np.ascontiguousarray(nl.out_node, np.uint32),
        mem_depth=np.ascontiguousarray(nl.mem_depth, np.uint32),
        mem_width=np.ascontiguousarray(nl.mem_width, np.uint8),
        mem_init=np.ascontiguousarray(nl.mem_init, np.uint64),
        wp_mem=np.ascontiguousarray(nl.wp_mem, np.uint32), wp_en=np.ascontiguousarray(nl.wp_en, np.uint32),
        wp_addr=np.ascontiguousarray(nl.wp_addr, np.uint32),
        wp_data=np.ascontiguousarray(nl.wp_data, np.uint32))
    en = getattr(nl, "reg_en", None)
    if en is not None:
        keep["reg_en"] = np.ascontiguousarray(en, np.uint32)
        if keep["reg_en"].shape != keep["reg_width"].shape:
            raise ValueError("reg_en needs one entry per register")
    s = Netlist()
    s.n_nodes, s.n_regs = len(keep["op"]), len(keep["reg_width"])
    s.n_inputs, s.n_outputs = len(keep["in_width"]), len(keep["out_node"])
    s.n_mems, s.n_wports = len(keep["mem_depth"]), len(keep["wp_mem"])
    for k, v in keep.items():
        setattr(s, k, _ptr(v))
    return s, keep


# Live handles by kind.  They are destroyed in dependency order -- servers,
# sims, designs, contexts -- by close() or, for whatever is still open, by
# an exit handler that runs before the interpreter and the HIP runtime shut
# down.  During interpreter finalization __del__ makes no library call: by
# then torch may have released a workspace or stream that a handle borrows.
_LIVE = {k: weakref.WeakSet() for k in ("server", "sim", "design", "ctx")}
_exit_hook = False


def _track(kind, obj):
    global _exit_hook
    _LIVE[kind].add(obj)
    if not _exit_hook:
        # registered after torch is imported, so it runs before torch's own
        # exit handlers
        atexit.register(close_all)
        _exit_hook = True


def close_all():
    """Destroy every open server, sim, design and context, in that order."""
    for kind in ("server", "sim", "design", "ctx"):
        for obj in list(_LIVE[kind]):
            obj.close()


def _finalizing():
    return sys.is_finalizing()


class Context:
    """A HIP device plus the stream every call is ordered on (torch's current
    stream by default, so torch.cuda.Event timing sees the kernels)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.torch_stream = stream
        h = C.c_void_p()
        _check(lib().fsim_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(h)), "fsim_ctx_create")
        self._h = h
        self.device = device
        _track("ctx", self)

    def info(self):
        cus, lds, wgs = C.c_uint32(), C.c_uint32(), C.c_uint32()
        _check(lib().fsim_ctx_device(self._h, C.byref(cus), C.byref(lds), C.byref(wgs)), "fsim_ctx_device")
        return dict(n_cus=cus.value, lds_bytes=lds.value, max_coresident_wgs=wgs.value)

    def close(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            self._h = None
            _lib.fsim_ctx_destroy(h)

    def __del__(self):
        if not _finalizing():
            self.close()


class Design:
    """A compiled design.  ctx=None compiles on the host only (partition and
    statistics; no sims)."""

    def __init__(self, ctx, nl, partition=None, pack=PACK_SLB, target_processes=0,
                 max_process_nodes=0):
        s, keep = _netlist_struct(nl)
        p = None
        if partition is not None:
            stp = np.ascontiguousarray(partition, np.uint32)
            self._stp = stp
            p = Partition(len(stp), _ptr(stp))
        o = CompileOpts(pack, target_processes, max_process_nodes)
        h = C.c_void_p()
        rc = lib().fsim_design_load(ctx._h if ctx is not None else None, C.byref(s),
                                    C.byref(p) if p is not None else None, C.byref(o), C.byref(h))
        _check(rc, "fsim_design_load")
        self._h = h
        self.ctx = ctx
        self.nl = nl
        self.n_regs, self.n_outputs, self.n_inputs = s.n_regs, s.n_outputs, s.n_inputs
        self.mem_depth = keep["mem_depth"].copy()
        self.n_sinks = s.n_regs + s.n_wports + s.n_outputs
        _track("design", self)

    def info(self) -> dict:
        i = DesignInfo()
        _check(lib().fsim_design_info(self._h, C.byref(i)), "fsim_design_info")
        return i.as_dict()

    def batched_info(self) -> dict:
        sb, sw, sd = C.c_uint32(), C.c_uint32(), C.c_uint32()
        ni, wb = C.c_uint64(), C.c_uint64()
        _check(lib().fsim_design_batched_info(self._h, C.byref(sb), C.byref(sw), C.byref(sd),
                                              C.byref(ni), C.byref(wb)), "fsim_design_batched_info")
        return dict(slots_b=sb.value, slots_w=sw.value, slots_d=sd.value, n_instr=ni.value,
                    wave_lds_bytes=wb.value)

    def partition(self):
        info = self.info()
        stp = np.zeros(max(self.n_sinks, 1), np.uint32)
        off = np.zeros(info["n_processes"] + 1, np.uint32)
        _check(lib().fsim_design_partition(self._h, _ptr(stp), _ptr(off), None), "fsim_design_partition")
        nodes = np.zeros(max(int(off[-1]), 1), np.uint32)
        _check(lib().fsim_design_partition(self._h, None, None, _ptr(nodes)), "fsim_design_partition")
        return stp[: self.n_sinks], off, nodes[: int(off[-1])]

    def close(self):
        """Release this handle (sims created from the design keep it alive
        inside the library until they are destroyed)."""
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            self._h = None
            _lib.fsim_design_free(h)

    def __del__(self):
        if not _finalizing():
            self.close()


class Sim:
    """n_instances copies of a design's state on the device.  The workspace is
    a torch uint8 tensor sized by fsim_sim_footprint (torch owns the memory)."""

    def __init__(self, design: Design, n_instances: int = 1, launch=LAUNCH_AUTO,
                 wg_threads=0, grid=0, graph_cycles=0, seed=None, use_torch_workspace=True,
                 form=FORM_AUTO, stage=STAGE_AUTO, tiles_per_wave=0):
        import torch
        self.design = design
        self.n_instances = n_instances
        fp = C.c_size_t()
        _check(lib().fsim_sim_footprint(design._h, n_instances, C.byref(fp)), "fsim_sim_footprint")
        self.footprint = fp.value
        ws_ptr, ws_bytes = None, 0
        if use_torch_workspace:
            self._ws = torch.empty(fp.value + 256, dtype=torch.uint8, device=f"cuda:{design.ctx.device}")
            base = self._ws.data_ptr()
            ws_ptr = (base + 255) // 256 * 256
            ws_bytes = fp.value
        o = SimOpts(launch, wg_threads, grid, graph_cycles, form, stage, tiles_per_wave)
        h = C.c_void_p()
        _check(lib().fsim_sim_create(design._h, n_instances, ws_ptr, ws_bytes, C.byref(o), C.byref(h)),
               "fsim_sim_create")
        self._h = h
        self._digest = None
        _track("sim", self)
        if seed is not None:
            self.set_seed(seed)

    def set_seed(self, seed_base: int):
        _check(lib().fsim_set_stimulus_seed(self._h, seed_base & (2**64 - 1)), "fsim_set_stimulus_seed")

    def set_inputs(self, first_cycle: int, vals):
        """vals: [n_cycles][n_inputs][n_instances] (or [n_cycles][n_inputs] for one instance)."""
        v = np.ascontiguousarray(vals, np.uint64)
        if v.ndim == 2:
            v = v[:, :, None]
        _check(lib().fsim_set_inputs(self._h, first_cycle, v.shape[0], _ptr(v)), "fsim_set_inputs")

    def step(self, n_cycles: int):
        _check(lib().fsim_step(self._h, n_cycles), "fsim_step")

    def sync(self):
        _check(lib().fsim_sync(self._h), "fsim_sync")

    @property
    def cycle(self) -> int:
        return lib().fsim_cycle(self._h)

    def set_cycle(self, c: int):
        _check(lib().fsim_set_cycle(self._h, c), "fsim_set_cycle")

    def regs(self, inst: int = 0) -> np.ndarray:
        out = np.zeros(max(self.design.n_regs, 1), np.uint64)
        _check(lib().fsim_read_regs(self._h, inst, _ptr(out)), "fsim_read_regs")
        return out[: self.design.n_regs]

    def regs_noalloc(self, inst: int = 0) -> np.ndarray:
        """Registers of one instance through fsim_read_regs_noalloc (no device
        allocation; a static staging array shared by all calls on the GPU)."""
        out = np.zeros(max(self.design.n_regs, 1), np.uint64)
        _check(lib().fsim_read_regs_noalloc(self._h, inst, _ptr(out)), "fsim_read_regs_noalloc")
        return out[: self.design.n_regs]

    def write_regs(self, vals, inst: int = 0):
        v = np.ascontiguousarray(vals, np.uint64)
        _check(lib().fsim_write_regs(self._h, inst, _ptr(v)), "fsim_write_regs")

    def outputs(self, inst: int = 0) -> np.ndarray:
        out = np.zeros(max(self.design.n_outputs, 1), np.uint64)
        _check(lib().fsim_read_outputs(self._h, inst, _ptr(out)), "fsim_read_outputs")
        return out[: self.design.n_outputs]

    def mem(self, m: int, inst: int = 0) -> np.ndarray:
        out = np.zeros(int(self.design.mem_depth[m]), np.uint64)
        _check(lib().fsim_read_mem(self._h, inst, m, _ptr(out)), "fsim_read_mem")
        return out

    def write_mem(self, m: int, vals, inst: int = 0):
        v = np.ascontiguousarray(vals, np.uint64)
        _check(lib().fsim_write_mem(self._h, inst, m, _ptr(v)), "fsim_write_mem")

    def enable_digest(self, max_cycles: int):
        """Per-cycle digests into a torch buffer [max_cycles][n_instances]."""
        import torch
        if max_cycles == 0:
            _check(lib().fsim_enable_digest(self._h, None, 0), "fsim_enable_digest")
            self._digest = None
            return
        self._digest = torch.zeros(max_cycles * self.n_instances, dtype=torch.int64,
                                   device=f"cuda:{self.design.ctx.device}")
        _check(lib().fsim_enable_digest(self._h, C.c_void_p(self._digest.data_ptr()), max_cycles),
               "fsim_enable_digest")

    def layout(self) -> dict:
        g_, t_, l_, s_ = C.c_uint32(), C.c_uint32(), C.c_uint32(), C.c_uint32()
        _check(lib().fsim_sim_layout(self._h, C.byref(g_), C.byref(t_), C.byref(l_), C.byref(s_)),
               "fsim_sim_layout")
        return dict(workgroups=g_.value, threads=t_.value, launch=l_.value, staged=bool(s_.value))

    def enable_trace(self, max_cycles: int):
        """Phase timestamps (100 MHz counter) per cycle, workgroup and level."""
        import torch
        lay = self.layout()
        stride = C.c_uint32()
        _check(lib().fsim_enable_trace(self._h, None, 0, C.byref(stride)), "fsim_enable_trace")
        self._trace_shape = (max_cycles, lay["workgroups"], stride.value)
        self._trace = torch.zeros(max_cycles * lay["workgroups"] * stride.value, dtype=torch.int64,
                                  device=f"cuda:{self.design.ctx.device}")
        _check(lib().fsim_enable_trace(self._h, C.c_void_p(self._trace.data_ptr()), max_cycles, None),
               "fsim_enable_trace")

    def trace(self) -> np.ndarray:
        self.sync()
        return self._trace.cpu().numpy().view(np.uint64).reshape(self._trace_shape)

    def digests(self) -> np.ndarray:
        self.sync()
        d = self._digest.cpu().numpy().view(np.uint64)
        return d.reshape(-1, self.n_instances)

    def close(self):
        """Destroy the sim (waits for its queued work), then drop the torch
        buffers it borrowed."""
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            self._h = None
            _lib.fsim_sim_destroy(h)
        self._ws = self._digest = self._trace = None

    def __del__(self):
        if not _finalizing():
            self.close()


class Server:
    """Continuous-batching request loop (fsim_server_*).  ctx=None gives the
    host-only executor that advances cycle counters without simulating."""

    def __init__(self, ctx, hbm_budget: int, quantum_cycles=0, max_jobs=0, max_queue=0, host_cycle_ns=0):
        o = ServerOpts(quantum_cycles, max_jobs, max_queue, host_cycle_ns)
        h = C.c_void_p()
        _check(lib().fsim_server_create(ctx._h if ctx is not None else None, hbm_budget, C.byref(o),
                                        C.byref(h)), "fsim_server_create")
        self._h = h
        self.ctx = ctx
        self._designs = []
        _track("server", self)

    def submit(self, design: Design, n_instances: int, n_cycles: int, seed_base: int) -> int:
        jid = C.c_uint64()
        _check(lib().fsim_server_submit(self._h, design._h, n_instances, n_cycles, seed_base & (2**64 - 1),
                                        C.byref(jid)), "fsim_server_submit")
        self._designs.append(design)      # keep the Python object alive
        return jid.value

    def poll(self, job: int) -> dict:
        st = JobStatus()
        _check(lib().fsim_server_poll(self._h, job, C.byref(st)), "fsim_server_poll")
        return st.as_dict()

    def wait(self, job: int, timeout: float = -1.0):
        _check(lib().fsim_server_wait(self._h, job, timeout), "fsim_server_wait")

    def result(self, job: int, inst: int, design: Design):
        regs = np.zeros(max(design.n_regs, 1), np.uint64)
        outs = np.zeros(max(design.n_outputs, 1), np.uint64)
        _check(lib().fsim_server_result(self._h, job, inst, _ptr(regs), _ptr(outs)), "fsim_server_result")
        return regs[: design.n_regs], outs[: design.n_outputs]

    def cancel(self, job: int):
        _check(lib().fsim_server_cancel(self._h, job), "fsim_server_cancel")

    def release(self, job: int):
        _check(lib().fsim_server_release(self._h, job), "fsim_server_release")

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().fsim_server_stats_get(self._h, C.byref(st)), "fsim_server_stats_get")
        return st.as_dict()

    def close(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            self._h = None
            _lib.fsim_server_destroy(h)

    def __del__(self):
        if not _finalizing():
            self.close()
