"""Stored oracle results for long parity runs -- TEST INFRASTRUCTURE ONLY.

The oracle needs 4 ms (single core) to 360 ms (48-tile SoC) per simulated
cycle on a host core, so the long runs that check the GPU at the
benchmark's own configurations (100,000 cycles of the single core, every
instance of the batched SoCs) are computed once, on the host, by
``tests/golden/make_oracle_refs.py``, which calls only ``oracle/`` and the
seeded input generator.  What is stored is compact but exact: for every
instance, SHA-256 prefixes of its per-cycle digest sequence in blocks of
cycles, of its final registers, final outputs and final memories.  A GPU
run matches a record exactly when every one of those hashes is equal; a
mismatch names the instance and the first block of cycles that differs.

Every record also stores the fingerprint of the netlist it was made from,
so a change of the generator shows up as a stale record rather than as a
parity failure, and the first few digests in the clear, which the CPU suite
recomputes with the oracle (``tests/test_oracle_refs.py``).
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
REFS_PATH = os.path.join(HERE, "golden", "oracle_refs.json")

NETLIST_FIELDS = ("op", "width", "arg", "imm", "reg_width", "reg_init", "reg_next", "in_width",
                  "out_node", "mem_depth", "mem_width", "mem_init", "wp_mem", "wp_en", "wp_addr",
                  "wp_data")


def h64(a) -> str:
    """First 16 hex digits of SHA-256 over the little-endian uint64 bytes."""
    b = np.ascontiguousarray(np.asarray(a, dtype=np.uint64).astype("<u8")).tobytes()
    return hashlib.sha256(b).hexdigest()[:16]


def fingerprint(nl) -> str:
    h = hashlib.sha256()
    for f in NETLIST_FIELDS:
        a = np.ascontiguousarray(getattr(nl, f))
        h.update(f.encode() + str(a.dtype).encode() + str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()[:16]


def block_hashes(digests, block: int) -> list:
    d = np.asarray(digests, dtype=np.uint64)
    return [h64(d[k:k + block]) for k in range(0, len(d), block)]


def load(name: str) -> dict:
    with open(REFS_PATH) as f:
        return json.load(f)[name]


def check_netlist(rec: dict, nl):
    fp = fingerprint(nl)
    assert fp == rec["netlist"], (
        f"stored oracle record '{rec['name']}' was made from netlist {rec['netlist']}, the generator now "
        f"gives {fp}: rerun tests/golden/make_oracle_refs.py")


def compare_instance(rec: dict, inst: int, digests=None, regs=None, outputs=None, mems=None):
    """Compare one instance of a GPU run with the stored record.  digests:
    the instance's per-cycle digests from the record's first cycle (all
    of the record's cycles); regs/outputs: final values after the record's
    cycles; mems: {m: words}.  Any argument may be None to skip it."""
    r = rec["instances"][str(inst)]
    if digests is not None:
        d = np.asarray(digests, dtype=np.uint64)
        assert len(d) == rec["cycles"], (len(d), rec["cycles"])
        got = block_hashes(d, rec["block"])
        bad = [k for k, (a, b) in enumerate(zip(got, r["digest_blocks"])) if a != b]
        assert not bad, (f"{rec['name']} instance {inst}: digests differ from the oracle in cycles "
                         f"[{bad[0] * rec['block']}, {(bad[0] + 1) * rec['block']})")
    if regs is not None:
        assert h64(regs) == r["regs"], f"{rec['name']} instance {inst}: final registers differ"
    if outputs is not None:
        assert h64(outputs) == r["outputs"], f"{rec['name']} instance {inst}: final outputs differ"
    if mems is not None:
        for m, words in mems.items():
            assert h64(words) == r["mems"][m], f"{rec['name']} instance {inst}: memory {m} differs"
