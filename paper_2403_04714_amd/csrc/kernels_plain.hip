// kernels_plain.hip -- gfx950 device code of libfibersim: the plain form.
//
// Plain form (one instance): a workgroup runs one process (a set of fibers,
// Parendi Sec. 3.2).  Per simulated cycle it evaluates the process step by
// step -- a step's operators are independent, one per lane (the compiler's
// list schedule), and values live in 4-byte LDS units -- stores the next
// values of the registers it owns
// into the "next" half of a double-buffered state array, commits memory
// writes after every read, and then crosses a grid-wide barrier.  The
// barrier plus the buffer swap is the exchange of Sec. 3.2: the current and
// next copies never alias within a cycle, so one barrier per cycle suffices
// where the IPU needs two (Sec. 4.1).
//
// Two kernels implement it.  plain_wave_* gives each process one 64-thread
// wave: a wave's LDS operations complete in order, so the levels need no
// barrier and the chunks of all levels run as one flat loop.  Its
// instructions are either staged in LDS at launch or read from global memory
// a few chunks ahead (then LDS holds only the value slots, and more
// workgroups are resident at once).  plain_* runs one process on a
// multi-wave workgroup, with a workgroup barrier between levels.  The
// kernel boundary of per-cycle launches (captured in a hipGraph) serves as
// the grid barrier.  It is cheaper on this chip than the flag barrier of
// the persistent launch once there are more than a few dozen workgroups.
//
// The barrier (Sec. 4.1 measures the same cost on the IPU and on x64) uses
// one epoch flag per workgroup: arrivals are plain stores to distinct words,
// so no read-modify-write serialises them.  The first workgroup of every
// group of 64 polls its group's flags and then stores a group flag; every
// workgroup polls the group flags, so a poll round reads G / 64 words per
// workgroup instead of G.  Cross-XCD visibility of the next-state stores
// comes from agent-scope releases before the flag stores and agent-scope
// acquires after the polls.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_common.h"

namespace fsim {

__device__ __forceinline__ uint32_t rfl(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ uint64_t rfl64(uint64_t v) {
  return ((uint64_t)rfl((uint32_t)(v >> 32)) << 32) | rfl((uint32_t)v);
}

// LDS addresses: ds instructions take a 32-bit byte address within the
// workgroup's allocation, so the value area is named by its LDS address
// (`base`) and an access builds its pointer from base + offset.  Where the
// value area starts at address 0 (no static LDS) the addition folds away.
typedef __attribute__((address_space(3))) uint32_t lds_u32_t;
typedef __attribute__((address_space(3))) uint64_t lds_u64_t;
__device__ __forceinline__ lds_u32_t* lds32(uint32_t a) { return (lds_u32_t*)(size_t)a; }
__device__ __forceinline__ lds_u64_t* lds64(uint32_t a) { return (lds_u64_t*)(size_t)a; }
// the LDS address of a __shared__ object
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(size_t)(const __attribute__((address_space(3))) char*)p;
}

// LDS value access by byte offset.  A value is read as 8 bytes.  A value in
// one 4-byte unit (at most 32 bits, read only where its upper half does not
// matter) then comes with the next unit, which belongs to another value, as
// its upper half; a value in two units (wide, or narrow and kept
// zero-extended) is an 8-byte aligned pair.
__device__ __forceinline__ uint64_t ld_raw(uint32_t base, uint32_t off) {
  const lds_u32_t* p = lds32(base + off);
  return (uint64_t)p[0] | ((uint64_t)p[1] << 32);
}
// A store of either size without a branch: the low half goes to its unit,
// the high half to the next unit for a two-unit value and to the spare unit
// at `trash` (never read as a value) for a one-unit one.
__device__ __forceinline__ void st_val(uint32_t base, uint32_t off, uint64_t v, bool one, uint32_t trash) {
  *lds32(base + off) = (uint32_t)v;
  *lds32(base + (one ? trash : off + 4)) = (uint32_t)(v >> 32);
}
// the spare unit: the last 4 bytes of the value area
__device__ __forceinline__ uint32_t trash_off(const PlainArgs& A) { return A.slot_words * 8 - 4; }

// The process a workgroup runs.  The dispatcher deals workgroups to the 8
// XCDs in turn (workgroup b lands on XCD b mod 8, each XCD with an L2 of its
// own); processes are numbered in packing order, where neighbours share
// registers and cone logic, so each XCD takes one contiguous range of
// processes and its L2 serves their shared leaf reads.  A bijection on
// [0, G) for any G.
__device__ __forceinline__ uint32_t process_of(uint32_t b, uint32_t G) {
  const uint32_t x = b & 7, q = G >> 3, r = G & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// Per-cycle state shared by the chunk handlers of both plain kernels.
struct PlainCycle {
  const uint64_t* cur;     // current register values
  uint64_t* nxt;           // next register values
  uint64_t cyc;            // absolute cycle
  uint64_t dacc;           // this lane's digest terms
};

// A leaf-load or sink-store chunk: up to four instructions per lane (lane +
// 64 q), every load issued before the first result is used.  `raw` is the
// lane's first instruction (already fetched); Is the process's
// instructions; base the LDS value area.
__device__ __forceinline__ void plain_wide_chunk(const PlainArgs& A, PlainCycle& C, const uint64_t* Is,
                                                 uint64_t cw, uint64_t raw, uint32_t lane, uint32_t base) {
  const uint32_t start = (uint32_t)cw & 0xFFFF, cnt = ((uint32_t)(cw >> 16) & 0xFF) + 1;
  const uint32_t op = (uint32_t)(cw >> 24) & 0xFF;
  uint64_t rq[4], v[4];
#pragma unroll
  for (uint32_t q = 0; q < 4; ++q) {
    const uint32_t e = lane + 64 * q;
    if (e < cnt) {
      rq[q] = q == 0 ? raw : Is[start + e];
      const uint32_t lo = (uint32_t)rq[q], hi = (uint32_t)(rq[q] >> 32);
      const uint64_t ix = pw_index(lo, hi);
      if (op == I_LDREG) {
        v[q] = C.cur[ix];
      } else if (op == I_LDIN) {
        if (A.in_vals) {
          if (C.cyc < A.in_first || C.cyc >= A.in_first + A.in_count) { atomicOr(&A.error[1], 1u); v[q] = 0; }
          else v[q] = A.in_vals[(C.cyc - A.in_first) * A.I + ix];
        } else {
          v[q] = hmix(A.in_keys[ix] ^ C.cyc);
        }
      } else {
        v[q] = ld_raw(base, pw_f0(lo));
      }
    }
  }
#pragma unroll
  for (uint32_t q = 0; q < 4; ++q) {
    const uint32_t e = lane + 64 * q;
    if (e < cnt) {
      const uint32_t lo = (uint32_t)rq[q], hi = (uint32_t)(rq[q] >> 32);
      const uint64_t x = v[q] & pw_mask(lo);   // LDIN widths fold in the port width
      if (op == I_LDREG || op == I_LDIN) {
        st_val(base, pw_f0(lo), x, pw_one0(hi), trash_off(A));
      } else if (op == I_STREG) {
        const uint64_t r = pw_index(lo, hi);
        C.nxt[r] = x;
        if (A.digest_part) C.dacc += hmix(r ^ hmix(x));
      } else {
        A.outputs[pw_index(lo, hi)] = x;
      }
    }
  }
}

// An operator chunk: one instruction per lane, every operand read before any
// lane computes.  Lanes past the chunk's end hold its last instruction: they
// read the same operands and store the same value to the same place, so the
// store needs no guard.  `cw` is the chunk word (wave-uniform); `dense_flag`
// the chunk flag that selects the opcode-bit tree for this launch.  Every
// result is stored as 8 bytes: a one-unit result's upper half lands on the
// unit above it, which the encoder keeps free at that step.  Chunks holding
// most opcodes are tested for first (nearly every chunk of a large process).
__device__ __forceinline__ void plain_alu_chunk(uint64_t cw, uint64_t raw, uint32_t base, uint32_t dense_flag) {
  const uint32_t lo = (uint32_t)raw, hi = (uint32_t)(raw >> 32);
  const uint32_t flags = (uint32_t)(cw >> 48), present = (uint32_t)(cw >> 32) & 0xFFFF;
  uint64_t a = ld_raw(base, pw_f1(lo, hi)), b = ld_raw(base, pw_f2(hi)), c = ld_raw(base, pw_f3(hi));
  asm volatile("; operands of an operator chunk ready" : "+v"(a), "+v"(b), "+v"(c));
  uint64_t r;
  if (__builtin_expect((flags & dense_flag) != 0, 1)) r = alu_dense(pw_op(lo), pw_mask(lo), a, b, c);
  else if ((present & (present - 1)) == 0) r = alu_single(__builtin_ctz(present | (1u << 31)), pw_mask(lo), a, b, c);
  else r = alu_select(present, pw_op(lo), pw_mask(lo), a, b, c);
  lds_u32_t* const d = lds32(base + pw_f0(lo));
  d[0] = (uint32_t)r;
  d[1] = (uint32_t)(r >> 32);
}

// A memory-read chunk.  Lanes past the chunk's end repeat its last read.
__device__ __forceinline__ void plain_memrd(const PlainArgs& A, uint64_t raw, uint32_t base) {
  const uint32_t lo = (uint32_t)raw, hi = (uint32_t)(raw >> 32);
  const uint64_t addr_v = ld_raw(base, pw_f1(lo, hi));
  const uint32_t m = pw_mem38(hi);
  // addr_v mod depth without a branch (lanes may read different memories):
  // q = floor(addr_v * magic / 2^64) is at most two below the quotient
  const uint64_t depth = A.mem_depth[m];
  const uint64_t q = __umul64hi(addr_v, A.mem_magic[m]);
  uint64_t addr = addr_v - q * depth;
  addr = addr >= depth ? addr - depth : addr;
  addr = addr >= depth ? addr - depth : addr;
  st_val(base, pw_f0(lo), A.mem[A.mem_off[m] + addr] & pw_mask(lo), pw_one0(hi), trash_off(A));
}

// Register or output stores written out among the operator levels: one per
// lane.  Lanes past the chunk's end repeat its last store (the same value to
// the same place) and add nothing to the digest.
__device__ __forceinline__ void plain_store64(const PlainArgs& A, PlainCycle& C, uint64_t cw, uint64_t raw,
                                              uint32_t lane, uint32_t base) {
  const uint32_t lo = (uint32_t)raw, hi = (uint32_t)(raw >> 32);
  const uint64_t x = ld_raw(base, pw_f0(lo)) & pw_mask(lo);
  const uint64_t ix = pw_index(lo, hi);
  if (((uint32_t)(cw >> 24) & 0xFF) == I_STREG) {
    C.nxt[ix] = x;
    if (A.digest_part) C.dacc += lane <= ((uint32_t)(cw >> 16) & 0xFF) ? hmix(ix ^ hmix(x)) : 0;
  } else {
    A.outputs[ix] = x;
  }
}

// A chunk of the operator levels: operators, memory reads, and register
// and output stores written out before the last level; one instruction per
// lane and no branch that differs between lanes.
__device__ __forceinline__ void plain_op_level_chunk(const PlainArgs& A, PlainCycle& C, uint64_t cw, uint64_t raw,
                                                     uint32_t lane, uint32_t base) {
  // operator chunks carry no kOtherKind flag, so the common case costs one
  // test of the chunk word's sign (taken on its high half, a scalar test)
  uint32_t cw_hi = (uint32_t)(cw >> 32);
  asm("" : "+s"(cw_hi));
  if (__builtin_expect((int32_t)cw_hi >= 0, 1)) plain_alu_chunk(cw, raw, base, A.dense_flag);
  else if (((uint32_t)(cw >> 24) & 0xFF) == I_MEMRD) plain_memrd(A, raw, base);
  else plain_store64(A, C, cw, raw, lane, base);
}

// Any chunk (the multi-wave kernel, which runs every level alike).
__device__ __forceinline__ void plain_level_chunk(const PlainArgs& A, PlainCycle& C, const uint64_t* Is, uint64_t cw,
                                                  uint64_t raw, uint32_t lane, uint32_t base) {
  const uint32_t kind = (uint32_t)(cw >> 24) & 0xFF;
  if (kind == I_ALU) plain_alu_chunk(cw, raw, base, A.dense_flag);
  else if (kind == I_MEMRD) plain_memrd(A, raw, base);
  else plain_wide_chunk(A, C, Is, cw, raw, lane, base);
}

// The write-port commit: after every read of the cycle, in port order, by
// one lane.
__device__ __forceinline__ void plain_commit(const PlainArgs& A, const uint64_t* Is, const PlainProc& pp, uint32_t base) {
  for (uint32_t k = 0; k < pp.n_wp; ++k) {
    const uint64_t w = Is[pp.n_instr + k];
    const uint32_t lo = (uint32_t)w, hi = (uint32_t)(w >> 32);
    if (ld_raw(base, pw_f0(lo)) != 0) {
      const uint32_t m = pw_mem50(hi);
      const uint64_t depth = A.mem_depth[m], av = ld_raw(base, pw_f1(lo, hi));
      const uint64_t addr = (depth & (depth - 1)) ? av % depth : (av & (depth - 1));
      A.mem[A.mem_off[m] + addr] = ld_raw(base, pw_f2(hi)) & pw_mask(lo);
    }
  }
}

// The constant prologue: every constant into its LDS place, once per launch.
// A constant is a destination word followed by its value.
__device__ __forceinline__ void plain_consts(const PlainArgs& A, const PlainProc& pp, uint32_t tid, uint32_t nthr,
                                             uint32_t base) {
  for (uint32_t i = tid; i < pp.n_consts; i += nthr) {
    const uint64_t w = A.code[pp.const_off + 2 * i], v = A.code[pp.const_off + 2 * i + 1];
    st_val(base, pw_f0((uint32_t)w), v, pw_one0((uint32_t)(w >> 32)), trash_off(A));
  }
}

// One-wave leaf level, in batches of kLeafQ leaf loads per lane (lane +
// 64 q): a batch's gathers are issued together, and the next batch's words
// are fetched while they are in flight.
constexpr uint32_t kLeafQ = 4;
__device__ __forceinline__ void leaf_words(const uint64_t* Ig, uint32_t b0, uint32_t n, uint32_t lane,
                                           uint64_t (&w)[kLeafQ]) {
#pragma unroll
  for (uint32_t q = 0; q < kLeafQ; ++q) {
    const uint32_t i = b0 + lane + 64 * q;
    w[q] = i < n ? Ig[i] : 0;
  }
}
// `w` holds the first batch's words on entry
__device__ __forceinline__ void leaf_level(const PlainArgs& A, const PlainCycle& C, const uint64_t* Ig,
                                           uint64_t (&w)[kLeafQ], uint32_t n, uint32_t lane, uint32_t base) {
  // inputs: the stimulus hash of the port's key (the key is gathered like a
  // register), or a row of caller-supplied values
  const bool expl = A.in_vals != nullptr;
  const bool in_window = C.cyc >= A.in_first && C.cyc < A.in_first + A.in_count;
  const uint64_t* const in_src = expl ? (in_window ? A.in_vals + (C.cyc - A.in_first) * A.I : C.cur) : A.in_keys;
  for (uint32_t b0 = 0; b0 < n; b0 += 64 * kLeafQ) {
    uint64_t v[kLeafQ];
    bool any_in = false;
#pragma unroll
    for (uint32_t q = 0; q < kLeafQ; ++q) {
      const uint32_t lo = (uint32_t)w[q], hi = (uint32_t)(w[q] >> 32);
      const bool live = b0 + lane + 64 * q < n, inp = lo & 1;
      any_in |= inp && live;
      v[q] = live ? (inp ? in_src : C.cur)[pw_index(lo, hi)] : 0;
    }
    uint64_t wn[kLeafQ];
    leaf_words(Ig, b0 + 64 * kLeafQ, n, lane, wn);
    if (__any(any_in)) {
      if (expl && !in_window && any_in) atomicOr(&A.error[1], 1u);
#pragma unroll
      for (uint32_t q = 0; q < kLeafQ; ++q)
        if ((uint32_t)w[q] & 1) v[q] = expl ? (in_window ? v[q] : 0) : hmix(v[q] ^ C.cyc);
    }
#pragma unroll
    for (uint32_t q = 0; q < kLeafQ; ++q) {
      const uint32_t lo = (uint32_t)w[q], hi = (uint32_t)(w[q] >> 32);
      // LDIN widths fold in the port width
      if (b0 + lane + 64 * q < n) st_val(base, pw_f0(lo), v[q] & pw_mask(lo), pw_one0(hi), trash_off(A));
    }
#pragma unroll
    for (uint32_t q = 0; q < kLeafQ; ++q) w[q] = wn[q];
  }
}

// One-wave final store level: kStQ store words per lane in flight.
constexpr uint32_t kStQ = 4;
__device__ __forceinline__ void final_stores(const PlainArgs& A, PlainCycle& C, const uint64_t* Is, uint32_t first,
                                             uint32_t n, uint32_t lane, uint32_t base) {
  for (uint32_t b0 = first; b0 < n; b0 += 64 * kStQ) {
    uint64_t w[kStQ];
#pragma unroll
    for (uint32_t q = 0; q < kStQ; ++q) {
      const uint32_t i = b0 + lane + 64 * q;
      w[q] = i < n ? Is[i] : 0;
    }
#pragma unroll
    for (uint32_t q = 0; q < kStQ; ++q) {
      if (b0 + lane + 64 * q < n) {
        const uint32_t lo = (uint32_t)w[q], hi = (uint32_t)(w[q] >> 32);
        const uint64_t x = ld_raw(base, pw_f0(lo)) & pw_mask(lo);
        const uint64_t ix = pw_index(lo, hi);
        if (lo & 1) {
          A.outputs[ix] = x;
        } else {
          C.nxt[ix] = x;
          if (A.digest_part) C.dacc += hmix(ix ^ hmix(x));
        }
      }
    }
  }
}

// Multi-wave workgroups: the chunks of a level are spread over the waves,
// with a workgroup barrier between levels.  Chunk words are read from
// global memory; the instructions from global memory or (STAGED) from an
// LDS copy made at launch.
template <bool PERSISTENT, bool STAGED>
__device__ void plain_body(const PlainArgs& A) {
  extern __shared__ uint64_t lds[];
  __shared__ int abort_flag;
  __shared__ uint64_t red[16];
  const uint32_t tid = threadIdx.x, nthr = blockDim.x;
  const uint32_t lane = tid & 63, wave = tid >> 6, nwaves = (nthr + 63) >> 6;
  const PlainProc pp = A.procs[process_of(blockIdx.x, gridDim.x)];
  const uint32_t base = lds_addr(lds);
  const uint32_t n_all = pp.n_instr + pp.n_wp;
  const uint64_t* const Ig = A.code + pp.instr_off;
  uint64_t* const Ist = lds + A.slot_words;
  if (STAGED)
    for (uint32_t i = tid; i < n_all; i += nthr) Ist[i] = Ig[i];
  const uint64_t* const Is = STAGED ? Ist : Ig;
  plain_consts(A, pp, tid, nthr, base);
  if (tid == 0) abort_flag = 0;
  __syncthreads();
  const uint64_t* const chunks = A.chunks + pp.chunk_off;
  const uint32_t* const lv = A.levels + pp.lvl_off;
  const uint64_t cyc0 = A.cycle_ptr ? *A.cycle_ptr + A.cycle0 : A.cycle0;
  uint64_t* trace_row = nullptr;
  for (uint32_t t = 0; t < A.n_cycles; ++t) {
    PlainCycle C;
    C.cyc = cyc0 + t;
    C.cur = A.state + (C.cyc & 1) * A.R;
    C.nxt = A.state + ((C.cyc + 1) & 1) * A.R;
    C.dacc = 0;
    if (A.trace && tid == 0) {
      const uint64_t k = C.cyc - A.trace_first;
      trace_row = k < A.trace_max ? A.trace + (k * gridDim.x + blockIdx.x) * A.trace_stride : nullptr;
      if (trace_row) trace_row[0] = __builtin_amdgcn_s_memrealtime();
    }
    for (uint32_t L = 0; L < pp.n_lvls; ++L) {
      const uint32_t c_hi = lv[L + 1];
      for (uint32_t c = rfl(lv[L] + wave); c < c_hi; c += nwaves) {
        const uint64_t cw = rfl64(chunks[c]);
        const uint32_t m = (uint32_t)(cw >> 16) & 0xFF;
        const uint64_t raw = Is[((uint32_t)cw & 0xFFFF) + (lane < m ? lane : m)];
        plain_level_chunk(A, C, Is, cw, raw, lane, base);
      }
      __syncthreads();
      if (trace_row && L + 2 < A.trace_stride) trace_row[L + 1] = __builtin_amdgcn_s_memrealtime();
    }
    if (tid == 0) plain_commit(A, Is, pp, base);
    if (A.digest_part) {
      uint64_t dacc = C.dacc;
      for (int off = 32; off > 0; off >>= 1) dacc += __shfl_xor(dacc, off);
      if (lane == 0) red[wave] = dacc;
      __syncthreads();
      if (tid == 0) {
        uint64_t s = 0;
        for (uint32_t k = 0; k < nwaves; ++k) s += red[k];
        const uint64_t k = C.cyc - A.digest_first;
        if (k < A.digest_max) A.digest_part[k * gridDim.x + blockIdx.x] = s;
      }
    }
    if (trace_row) trace_row[A.trace_stride - 2] = __builtin_amdgcn_s_memrealtime();
    if (PERSISTENT) {
      if (gridDim.x > 1) {
        if (!grid_barrier(A.flags, A.error, gridDim.x, A.epoch0 + t + 1, &abort_flag)) return;
      } else {
        __syncthreads();
      }
    } else {
      __syncthreads();
    }
    if (trace_row) trace_row[A.trace_stride - 1] = __builtin_amdgcn_s_memrealtime();
  }
}

// Single-wave processes (64 threads).  LDS operations of one wave complete
// in order, so the levels need no barrier.  LDS holds the values, the chunk
// table (zero past the last chunk) and, when STAGED, a copy of the process's
// instructions made at launch; otherwise the instructions are read from
// global memory.  A cycle runs in three phases: the leaf level (register and
// input loads, kLeafQ per lane in flight, their words always read from
// global memory), the operator levels, the final store level (kStQ per lane
// in flight).
//   STAGED: the operator levels run chunk by chunk, the next chunk's
//   instruction read from LDS while the current chunk's operands are read.
//   Otherwise: in groups of kGroup chunks, and when a group starts the first
//   instruction of every chunk of the next group is fetched, so that each
//   global fetch has a whole group's time to land.  The first group is
//   fetched before the leaf level.
template <bool PERSISTENT, bool STAGED, bool TRACE>
__device__ void plain_wave_body(const PlainArgs& A) {
  // no static LDS: the value area starts at address 0, so value offsets are
  // LDS addresses; its first 8 bytes (reserved units) hold the abort flag of
  // the grid barrier
  extern __shared__ uint64_t lds[];
  int* const abort_flag = reinterpret_cast<int*>(lds);
  const uint32_t lane = threadIdx.x;
  const PlainProc pp = A.procs[process_of(blockIdx.x, gridDim.x)];
  const uint32_t base = 0;   // the value area's LDS address
  const uint32_t n_all = pp.n_instr + pp.n_wp;
  const uint64_t* const Ig = A.code + pp.instr_off;
  uint64_t* const ctab = lds + A.slot_words;
  uint64_t* const Ist = ctab + A.ctab_words;
  // set-up in one round trip: the first leaf batch (read from global memory
  // also when staged), the lane's first chunk word and constant, and the
  // first staging block are all in flight together; tables longer than 64
  // entries take more rounds
  const uint32_t n_leaf = pp.n_leaf, n_ch = pp.n_chunks, n_k = pp.n_consts;
  uint64_t lw[kLeafQ];
  leaf_words(Ig, 0, n_leaf, lane, lw);
  const uint64_t* const K = A.code + pp.const_off;
  // the chunk table: entries from the store phase on repeat the last
  // operator chunk, so the operator loop reads ahead without a bound
  const uint32_t c_ops = pp.c_ops, c_st = pp.c_st;
  const uint32_t c_rep = c_st > c_ops ? c_st - 1 : n_ch;
  auto ctab_entry = [&](uint32_t i) -> uint64_t {
    const uint32_t j = i < c_rep ? i : c_rep;
    return j < n_ch ? A.chunks[pp.chunk_off + j] : 0;
  };
  const uint64_t cw0 = ctab_entry(lane);
  const uint64_t kw0 = lane < n_k ? K[2 * lane] : 0, kv0 = lane < n_k ? K[2 * lane + 1] : 0;
  // staging, eight loads in flight per lane
  for (uint32_t b0 = 0; STAGED && b0 < n_all; b0 += 512) {
    uint64_t t[8];
#pragma unroll
    for (uint32_t q = 0; q < 8; ++q) {
      const uint32_t i = b0 + lane + 64 * q;
      t[q] = i < n_all ? Ig[i] : 0;
    }
#pragma unroll
    for (uint32_t q = 0; q < 8; ++q) {
      const uint32_t i = b0 + lane + 64 * q;
      if (i < n_all) Ist[i] = t[q];
    }
  }
  const uint64_t* const Is = STAGED ? Ist : Ig;
  if (lane < A.ctab_words) ctab[lane] = cw0;
  for (uint32_t i = lane + 64; i < A.ctab_words; i += 64) ctab[i] = ctab_entry(i);
  if (lane < n_k) st_val(base, pw_f0((uint32_t)kw0), kv0, pw_one0((uint32_t)(kw0 >> 32)), trash_off(A));
  for (uint32_t i = lane + 64; i < n_k; i += 64)
    st_val(base, pw_f0((uint32_t)K[2 * i]), K[2 * i + 1], pw_one0((uint32_t)(K[2 * i] >> 32)), trash_off(A));
  // level starts, for the phase timestamps only
  const uint32_t n_lvls = pp.n_lvls;
  const uint32_t lv_lo = TRACE && lane <= n_lvls ? A.levels[pp.lvl_off + lane] : 0;
  // one wave: its LDS operations complete in order, so the set-up's stores
  // need no barrier before the reads below
  if (lane == 0) *abort_flag = 0;
  // a chunk word (wave-uniform, kept in scalar registers) and the lane's
  // instruction of that chunk; lanes past the chunk's end take its last one
  auto op_chunk = [&](uint32_t c) -> uint64_t { return rfl64(ctab[c]); };
  auto op_instr = [&](uint64_t cw) -> uint64_t {
    const uint32_t m = (uint32_t)(cw >> 16) & 0xFF;
    return Is[((uint32_t)cw & 0xFFFF) + (lane < m ? lane : m)];
  };
  const uint64_t cyc0 = A.cycle_ptr ? *A.cycle_ptr + A.cycle0 : A.cycle0;
  uint64_t* trace_row = nullptr;
  for (uint32_t t = 0; t < A.n_cycles; ++t) {
    PlainCycle C;
    C.cyc = cyc0 + t;
    C.cur = A.state + (C.cyc & 1) * A.R;
    C.nxt = A.state + ((C.cyc + 1) & 1) * A.R;
    C.dacc = 0;
    if (TRACE && A.trace) {
      const uint64_t k = C.cyc - A.trace_first;
      trace_row = k < A.trace_max ? A.trace + (k * gridDim.x + blockIdx.x) * A.trace_stride : nullptr;
      if (trace_row && lane == 0) trace_row[0] = __builtin_amdgcn_s_memrealtime();
    }
    uint32_t L_next = 1;   // next level whose end is timestamped
    auto stamp = [&](uint32_t done) {
      // stamp the end of every level that ends before chunk `done` (levels
      // beyond the 63rd are not stamped)
      while (L_next < 64 && L_next <= n_lvls &&
             done >= (uint32_t)__builtin_amdgcn_readlane((int)lv_lo, (int)L_next)) {
        if (lane == 0 && L_next + 1 < A.trace_stride) trace_row[L_next] = __builtin_amdgcn_s_memrealtime();
        ++L_next;
      }
    };
    // global instructions: the first group of operator chunks is fetched
    // before the leaf level
    uint64_t cw[kGroup], ins[kGroup];
    if (!STAGED && c_ops < c_st) {
#pragma unroll
      for (uint32_t k = 0; k < kGroup; ++k) {
        cw[k] = op_chunk(c_ops + k);
        ins[k] = op_instr(cw[k]);
      }
    }
    // the leaf level
    if (t > 0) leaf_words(Ig, 0, n_leaf, lane, lw);
    leaf_level(A, C, Ig, lw, n_leaf, lane, base);
    if (TRACE && trace_row) stamp(c_ops);
    if (STAGED && c_ops < c_st) {
      // the next chunk's instruction and the chunk word after it are read
      // while a chunk runs
      uint64_t sw = op_chunk(c_ops), swn = op_chunk(c_ops + 1);
      uint64_t sins = op_instr(sw);
      for (uint32_t c = c_ops; c < c_st; ++c) {
        const uint64_t nins = op_instr(swn);
        const uint64_t swnn = op_chunk(c + 2);
        plain_op_level_chunk(A, C, sw, sins, lane, base);
        sw = swn;
        swn = swnn;
        sins = nins;
        if (TRACE && trace_row) stamp(c + 1);
      }
    } else if (!STAGED) {
      for (uint32_t c = c_ops; c < c_st; c += kGroup) {
        uint64_t nw[kGroup], nins[kGroup];
#pragma unroll
        for (uint32_t k = 0; k < kGroup; ++k) {
          nw[k] = op_chunk(c + kGroup + k);
          nins[k] = op_instr(nw[k]);
        }
#pragma unroll
        for (uint32_t k = 0; k < kGroup; ++k) {
          if (c + k < c_st) {
            plain_op_level_chunk(A, C, cw[k], ins[k], lane, base);
            if (TRACE && trace_row) stamp(c + k + 1);
          }
        }
#pragma unroll
        for (uint32_t k = 0; k < kGroup; ++k) {
          cw[k] = nw[k];
          ins[k] = nins[k];
        }
      }
    }
    final_stores(A, C, Is, pp.st_first, pp.n_instr, lane, base);
    if (TRACE && trace_row) stamp(n_ch);
    if (lane == 0) plain_commit(A, Is, pp, base);
    if (A.digest_part) {
      uint64_t dacc = C.dacc;
      for (int off = 32; off > 0; off >>= 1) dacc += __shfl_xor(dacc, off);
      const uint64_t k = C.cyc - A.digest_first;
      if (lane == 0 && k < A.digest_max) A.digest_part[k * gridDim.x + blockIdx.x] = dacc;
    }
    if (trace_row && lane == 0) trace_row[A.trace_stride - 2] = __builtin_amdgcn_s_memrealtime();
    if (PERSISTENT) {
      if (gridDim.x > 1) {
        if (!grid_barrier(A.flags, A.error, gridDim.x, A.epoch0 + t + 1, abort_flag)) return;
      } else {
        asm volatile("" ::: "memory");
      }
    } else {
      asm volatile("" ::: "memory");
    }
    if (trace_row && lane == 0) trace_row[A.trace_stride - 1] = __builtin_amdgcn_s_memrealtime();
  }
}

__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) plain_wave_persistent(PlainArgs A) { plain_wave_body<true, true, false>(A); }
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) plain_wave_cycle(PlainArgs A) { plain_wave_body<false, true, false>(A); }
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) plain_wave_persistent_g(PlainArgs A) { plain_wave_body<true, false, false>(A); }
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) plain_wave_cycle_g(PlainArgs A) { plain_wave_body<false, false, false>(A); }
// the same with phase timestamps (a sim with tracing enabled): the untraced
// kernels carry no per-chunk test for it
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) plain_wave_persistent_trace(PlainArgs A) { plain_wave_body<true, true, true>(A); }
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) plain_wave_cycle_trace(PlainArgs A) { plain_wave_body<false, true, true>(A); }
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) plain_wave_persistent_g_trace(PlainArgs A) {
  plain_wave_body<true, false, true>(A);
}
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) plain_wave_cycle_g_trace(PlainArgs A) { plain_wave_body<false, false, true>(A); }

__global__ void __launch_bounds__(1024) plain_persistent(PlainArgs A) { plain_body<true, true>(A); }
__global__ void __launch_bounds__(1024) plain_cycle(PlainArgs A) { plain_body<false, true>(A); }
__global__ void __launch_bounds__(1024) plain_persistent_g(PlainArgs A) { plain_body<true, false>(A); }
__global__ void __launch_bounds__(1024) plain_cycle_g(PlainArgs A) { plain_body<false, false>(A); }

// digest[k] = sum over workgroups of the partials of cycle k
__global__ void digest_reduce(const uint64_t* part, uint32_t G, uint64_t n, uint64_t* out) {
  uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  uint64_t s = 0;
  for (uint32_t g = 0; g < G; ++g) s += part[k * G + g];
  out[k] += s;
}

__global__ void add_u64(uint64_t* p, uint64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p += v;
}

// stimulus keys, instance-minor: keys[p * n_inst + i] = H(H(seed_base + i) ^ p)
__global__ void stim_keys(uint64_t* keys, uint64_t seed_base, uint32_t n_inst, uint32_t I) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_inst * I) return;
  uint32_t i = k % n_inst, p = k / n_inst;
  keys[k] = hmix(hmix(seed_base + i) ^ (uint64_t)p);
}

}  // namespace fsim

// ---------------------------------------------------------------- launches
namespace fsim {

hipError_t launch_plain(const PlainArgs& a, uint32_t G, uint32_t threads, size_t lds_bytes,
                        bool persistent, hipStream_t s) {
  if (a.single_wave) {
    const bool tr = a.trace != nullptr;
    if (persistent) {
      void* args[] = {const_cast<PlainArgs*>(&a)};
      const void* k = a.stage_instr ? (tr ? (const void*)plain_wave_persistent_trace : (const void*)plain_wave_persistent)
                                    : (tr ? (const void*)plain_wave_persistent_g_trace
                                          : (const void*)plain_wave_persistent_g);
      return hipLaunchCooperativeKernel(k, dim3(G), dim3(64), args, (unsigned)lds_bytes, s);
    }
    if (a.stage_instr) {
      if (tr) hipLaunchKernelGGL(plain_wave_cycle_trace, dim3(G), dim3(64), lds_bytes, s, a);
      else hipLaunchKernelGGL(plain_wave_cycle, dim3(G), dim3(64), lds_bytes, s, a);
    } else {
      if (tr) hipLaunchKernelGGL(plain_wave_cycle_g_trace, dim3(G), dim3(64), lds_bytes, s, a);
      else hipLaunchKernelGGL(plain_wave_cycle_g, dim3(G), dim3(64), lds_bytes, s, a);
    }
    return hipGetLastError();
  }
  if (persistent) {
    void* args[] = {const_cast<PlainArgs*>(&a)};
    return hipLaunchCooperativeKernel(a.stage_instr ? (const void*)plain_persistent : (const void*)plain_persistent_g,
                                      dim3(G), dim3(threads), args, (unsigned)lds_bytes, s);
  }
  if (a.stage_instr) hipLaunchKernelGGL(plain_cycle, dim3(G), dim3(threads), lds_bytes, s, a);
  else hipLaunchKernelGGL(plain_cycle_g, dim3(G), dim3(threads), lds_bytes, s, a);
  return hipGetLastError();
}

hipError_t plain_occupancy(int* blocks_per_cu, uint32_t threads, size_t lds_bytes, bool staged,
                           bool single_wave) {
  // the traced variants use the most registers: a grid sized by them stays
  // co-resident with tracing on or off
  if (single_wave)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu,
                                                        staged ? plain_wave_persistent_trace
                                                               : plain_wave_persistent_g_trace,
                                                        64, lds_bytes);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, staged ? plain_persistent : plain_persistent_g,
                                                      (int)threads, lds_bytes);
}

hipError_t launch_digest_reduce(const uint64_t* part, uint32_t G, uint64_t n, uint64_t* out,
                                hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(digest_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, G, n, out);
  return hipGetLastError();
}

hipError_t launch_add_u64(uint64_t* p, uint64_t v, hipStream_t s) {
  hipLaunchKernelGGL(add_u64, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_stim_keys(uint64_t* keys, uint64_t seed_base, uint32_t n_inst, uint32_t I,
                            hipStream_t s) {
  uint32_t n = n_inst * I;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(stim_keys, dim3((n + 255) / 256), dim3(256), 0, s, keys, seed_base, n_inst, I);
  return hipGetLastError();
}

}  // namespace fsim
