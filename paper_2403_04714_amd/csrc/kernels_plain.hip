// kernels_plain.hip -- gfx950 device code of libfibersim: the plain form.
//
// Plain form (one instance): a workgroup runs one process (a set of fibers,
// Parendi Sec. 3.2).  Per simulated cycle it evaluates the process level by
// level -- lanes take the independent operators of a level in parallel,
// values live in LDS slots -- stores the next values of the registers it owns
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

template <bool PERSISTENT, bool STAGED>
__device__ void plain_body(const PlainArgs& A) {
  extern __shared__ uint64_t lds[];
  __shared__ int abort_flag;
  __shared__ uint64_t red[16];
  const uint32_t tid = threadIdx.x, nthr = blockDim.x;
  const uint32_t lane = tid & 63, wave = tid >> 6, nwaves = (nthr + 63) >> 6;
  const PlainProc pp = A.procs[blockIdx.x];
  // value slots: instruction operands are byte offsets into the slot area
  char* const slot_base = reinterpret_cast<char*>(lds);
  auto at = [slot_base](uint32_t off) -> uint64_t& { return *reinterpret_cast<uint64_t*>(slot_base + off); };
  const uint32_t n_all = pp.n_instr + pp.n_wp;
  const uint4* Ig = reinterpret_cast<const uint4*>(A.instr) + pp.instr_off;
  uint4* Is = reinterpret_cast<uint4*>(lds + A.slot_words);
  uint32_t* chunks = reinterpret_cast<uint32_t*>(Is + (STAGED ? A.instr_words : 0));
  uint32_t* lvs = chunks + A.chunk_words;
  if (STAGED)
    for (uint32_t i = tid; i < n_all; i += nthr) Is[i] = Ig[i];
  for (uint32_t i = tid; i < pp.n_chunks; i += nthr) chunks[i] = A.chunks[pp.chunk_off + i];
  for (uint32_t L = tid; L <= pp.n_lvls; L += nthr) lvs[L] = A.levels[pp.lvl_off + L];
  for (uint32_t i = tid; i < pp.n_consts; i += nthr) {
    const Instr in = A.instr[pp.const_off + i];
    at(in.dst) = A.consts[in.aux];
  }
  if (tid == 0) abort_flag = 0;
  __syncthreads();
  auto fetch = [&](uint32_t i) -> uint4 { return STAGED ? Is[i] : Ig[i]; };
  const uint32_t n_lvls = pp.n_lvls;
  // the level table (chunk index where each level starts) lives in the lanes
  // of two registers and is read with v_readlane; deeper processes fall back
  // to the LDS copy
  const uint32_t lv_lo = lane <= n_lvls ? lvs[lane] : 0;
  const uint32_t lv_hi = lane + 64 <= n_lvls ? lvs[lane + 64] : 0;
  auto lvl = [&](uint32_t L) -> uint32_t {
    if (L < 64) return (uint32_t)__builtin_amdgcn_readlane((int)lv_lo, (int)L);
    if (L < 128) return (uint32_t)__builtin_amdgcn_readlane((int)lv_hi, (int)(L - 64));
    return lvs[L];
  };
  // one wave: LDS operations of a wave complete in order, so a level needs no
  // s_barrier, only a compiler barrier
  const bool one_wave = nthr <= 64;
  const uint64_t cyc0 = A.cycle_ptr ? *A.cycle_ptr + A.cycle0 : A.cycle0;
  // phase timestamps: [cycle][workgroup][trace_stride] of the 100 MHz
  // realtime counter: cycle start, end of every level, commit, barrier
  uint64_t* trace_row = nullptr;
  for (uint32_t t = 0; t < A.n_cycles; ++t) {
    const uint64_t cyc = cyc0 + t;
    const uint64_t* cur = A.state + (cyc & 1) * A.R;
    uint64_t* nxt = A.state + ((cyc + 1) & 1) * A.R;
    uint64_t dacc = 0;
    if (A.trace && tid == 0) {
      const uint64_t k = cyc - A.trace_first;
      trace_row = k < A.trace_max ? A.trace + (k * gridDim.x + blockIdx.x) * A.trace_stride : nullptr;
      if (trace_row) trace_row[0] = __builtin_amdgcn_s_memrealtime();
    }
    // this wave's first chunk of level 0 and its instruction, and the first
    // chunk word of level 1 (a level always exists after the leaf level)
    uint32_t c_lo = lvl(0), c_hi = lvl(1);
    uint32_t ch_first = c_lo + wave < c_hi ? chunks[c_lo + wave] : 0;
    ch_first = __builtin_amdgcn_readfirstlane(ch_first);
    uint4 raw_first = make_uint4(0, 0, 0, 0);
    if (c_lo + wave < c_hi && lane <= ((ch_first >> 16) & 0xFF)) raw_first = fetch((ch_first & 0xFFFF) + lane);
    uint32_t n_lo = c_hi, n_hi = n_lvls > 1 ? lvl(2) : c_hi;
    uint32_t ch_next = __builtin_amdgcn_readfirstlane(n_lo + wave < n_hi ? chunks[n_lo + wave] : 0);
    for (uint32_t L = 0; L < n_lvls; ++L) {
      // Prefetch, issued with this level's operand reads so that the
      // latencies overlap: the next level's first instruction for this wave
      // and the first chunk word two levels ahead.  Instructions and chunk
      // words never change during the launch.
      const bool have_next = n_lo + wave < n_hi;
      uint4 raw_next = make_uint4(0, 0, 0, 0);
      if (have_next && lane <= ((ch_next >> 16) & 0xFF)) raw_next = fetch((ch_next & 0xFFFF) + lane);
      const uint32_t m_lo = n_hi, m_hi = L + 2 < n_lvls ? lvl(L + 3) : n_hi;
      const uint32_t ch_after = m_lo + wave < m_hi ? chunks[m_lo + wave] : 0;
      bool first = true;
      for (uint32_t c = c_lo + wave; c < c_hi; c += nwaves) {
        uint32_t ch = first ? ch_first : __builtin_amdgcn_readfirstlane(chunks[c]);
        const uint32_t start = ch & 0xFFFF, cnt = ((ch >> 16) & 0xFF) + 1, op = ch >> 24;
        if (op == I_ALU) {
          // operators of mixed opcodes: every operand is read before any lane
          // computes, so the level costs one LDS round trip; the opcode
          // switch then runs on registers only
          if (lane < cnt) {
            const Dec in = decode(first ? raw_first : fetch(start + lane));
            uint64_t a = at(in.a), b = at(in.b), cc = at(in.c);
            asm volatile("; operands of a mixed chunk ready" : "+v"(a), "+v"(b), "+v"(cc));
            const uint32_t present = __builtin_amdgcn_readfirstlane(in.aux);
            at(in.dst) = alu_mixed(present, in.op, in.w, a, b, cc);
          }
        } else if (op == I_LDREG || op == I_LDIN || op == I_STREG || op == I_STOUT) {
          // up to four instructions per lane; all loads are issued before the
          // first result is used
          Dec in[4];
          uint64_t v[4];
#pragma unroll
          for (uint32_t q = 0; q < 4; ++q) {
            const uint32_t e = lane + 64 * q;
            if (e < cnt) {
              in[q] = decode(q == 0 && first ? raw_first : fetch(start + e));
              if (op == I_LDREG) {
                v[q] = cur[in[q].aux];
              } else if (op == I_LDIN) {
                if (A.in_vals) {
                  if (cyc < A.in_first || cyc >= A.in_first + A.in_count) { atomicOr(&A.error[1], 1u); v[q] = 0; }
                  else v[q] = A.in_vals[(cyc - A.in_first) * A.I + in[q].aux];
                } else {
                  v[q] = hmix(A.in_keys[in[q].aux] ^ cyc);
                }
              } else {
                v[q] = at(in[q].a);
              }
            }
          }
#pragma unroll
          for (uint32_t q = 0; q < 4; ++q) {
            const uint32_t e = lane + 64 * q;
            if (e < cnt) {
              const uint64_t x = v[q] & wmask(in[q].w);   // LDIN widths fold in the port width
              if (op == I_LDREG || op == I_LDIN) {
                at(in[q].dst) = x;
              } else if (op == I_STREG) {
                nxt[in[q].aux] = x;
                if (A.digest_part) dacc += hmix((uint64_t)in[q].aux ^ hmix(x));
              } else {
                A.outputs[in[q].aux] = x;
              }
            }
          }
        } else if (op == I_MEMRD) {
          if (lane < cnt) {
            const Dec in = decode(first ? raw_first : fetch(start + lane));
            const uint64_t a = at(in.a);
            const uint64_t depth = A.mem_depth[in.aux];
            const uint64_t addr = (depth & (depth - 1)) ? a % depth : (a & (depth - 1));
            at(in.dst) = A.mem[A.mem_off[in.aux] + addr] & wmask(in.w);
          }
        }
        first = false;
      }
      ch_first = ch_next;
      raw_first = raw_next;
      ch_next = __builtin_amdgcn_readfirstlane(ch_after);
      c_lo = n_lo;
      c_hi = n_hi;
      n_lo = m_lo;
      n_hi = m_hi;
      if (one_wave) asm volatile("" ::: "memory");
      else __syncthreads();
      if (trace_row && L + 2 < A.trace_stride) trace_row[L + 1] = __builtin_amdgcn_s_memrealtime();
    }
    // memory commit after every read of this cycle, in port order
    if (tid == 0) {
      for (uint32_t k = 0; k < pp.n_wp; ++k) {
        const Dec in = decode(fetch(pp.n_instr + k));
        if (at(in.a) != 0) {
          const uint32_t m = in.aux;
          const uint64_t depth = A.mem_depth[m], av = at(in.b);
          const uint64_t addr = (depth & (depth - 1)) ? av % depth : (av & (depth - 1));
          A.mem[A.mem_off[m] + addr] = at(in.c) & wmask(in.w);
        }
      }
    }
    if (A.digest_part) {
      // workgroup reduction of the digest terms; partial per workgroup
      for (int off = 32; off > 0; off >>= 1) dacc += __shfl_xor(dacc, off);
      if (lane == 0) red[wave] = dacc;
      __syncthreads();
      if (tid == 0) {
        uint64_t s = 0;
        for (uint32_t k = 0; k < nwaves; ++k) s += red[k];
        const uint64_t k = cyc - A.digest_first;
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
    }
    if (trace_row) trace_row[A.trace_stride - 1] = __builtin_amdgcn_s_memrealtime();
  }
}

// Single-wave processes (64 threads): LDS operations of one wave complete in
// order, so the levels need no barrier and the chunks of all levels run as
// one flat sequence.  The chunk words sit in an LDS table after the value
// slots, each read with one broadcast LDS read a few chunks ahead, and the
// first instruction of a later chunk is fetched while the current one runs.
// STAGED: the process's instructions are copied into LDS at launch and read
// from there.  Otherwise they are read from global memory, the first
// instruction of each chunk kWaveSlots chunks ahead, and the workgroup's LDS
// holds only the value slots and the chunk table, so that many more
// workgroups are resident at once (large designs) and nothing is copied per
// launch.
template <bool PERSISTENT, bool STAGED, bool TRACE>
__device__ void plain_wave_body(const PlainArgs& A) {
  extern __shared__ uint64_t lds[];
  __shared__ int abort_flag;
  const uint32_t lane = threadIdx.x;
  const PlainProc pp = A.procs[blockIdx.x];
  // value slots: instruction operands are byte offsets into the slot area
  char* const slot_base = reinterpret_cast<char*>(lds);
  auto at = [slot_base](uint32_t off) -> uint64_t& { return *reinterpret_cast<uint64_t*>(slot_base + off); };
  const uint32_t n_all = pp.n_instr + pp.n_wp;
  const uint4* Ig = reinterpret_cast<const uint4*>(A.instr) + pp.instr_off;
  // after the slots: the process's chunk words (zero past the last chunk,
  // read a few chunks ahead with one broadcast LDS read each), then the
  // staged instructions
  uint32_t* const ctab = reinterpret_cast<uint32_t*>(lds + A.slot_words);
  char* const ibase = reinterpret_cast<char*>(ctab) + 4 * A.ctab_words;
  // instruction i of the process (LDS copy or global memory)
  const uint4* const Is = STAGED ? reinterpret_cast<const uint4*>(ibase) : Ig;
  // staging, eight loads in flight per lane (one memory latency per 512
  // instructions; the per-cycle launch modes stage on every launch)
  // (plain 16-byte words, not uint4: an array of the vector type is kept in
  // scratch memory by the compiler)
  const IWord* Igw = reinterpret_cast<const IWord*>(Ig);
  IWord* Isw = reinterpret_cast<IWord*>(ibase);
  for (uint32_t base = 0; STAGED && base < n_all; base += 512) {
    IWord t[8];
#pragma unroll
    for (uint32_t q = 0; q < 8; ++q) {
      const uint32_t i = base + lane + 64 * q;
      t[q] = i < n_all ? Igw[i] : IWord{0, 0, 0, 0};
    }
#pragma unroll
    for (uint32_t q = 0; q < 8; ++q) {
      const uint32_t i = base + lane + 64 * q;
      if (i < n_all) Isw[i] = t[q];
    }
  }
  for (uint32_t i = lane; i < pp.n_consts; i += 64) {
    const Instr in = A.instr[pp.const_off + i];
    at(in.dst) = A.consts[in.aux];
  }
  const uint32_t n_ch = pp.n_chunks;
  for (uint32_t i = lane; i < A.ctab_words; i += 64) ctab[i] = i < n_ch ? A.chunks[pp.chunk_off + i] : 0;
  // level starts, for the phase timestamps only
  const uint32_t n_lvls = pp.n_lvls;
  const uint32_t lv_lo = TRACE && lane <= n_lvls ? A.levels[pp.lvl_off + lane] : 0;
  if (lane == 0) abort_flag = 0;
  __syncthreads();
  // the first instruction of a chunk for this lane; lanes past the chunk's
  // end get its last instruction (valid slots to read; an operator chunk
  // stores their result, the same value to the same slot as the last lane,
  // other chunks guard by count).  No condition: the load stays in the basic block of the
  // operand reads it overlaps.  For "no chunk" (word 0) it reads entry 0.
  auto first_instr = [&](uint32_t chw) -> uint4 {
    const uint32_t m = (chw >> 16) & 0xFF;
    return Is[(chw & 0xFFFF) + (lane < m ? lane : m)];
  };
  const uint64_t cyc0 = A.cycle_ptr ? *A.cycle_ptr + A.cycle0 : A.cycle0;
  uint64_t* trace_row = nullptr;
  for (uint32_t t = 0; t < A.n_cycles; ++t) {
    const uint64_t cyc = cyc0 + t;
    const uint64_t* cur = A.state + (cyc & 1) * A.R;
    uint64_t* nxt = A.state + ((cyc + 1) & 1) * A.R;
    uint64_t dacc = 0;
    if (TRACE && A.trace) {
      const uint64_t k = cyc - A.trace_first;
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
    uint32_t c = 0;
    // chunk word cc, as a wave-uniform value (the read is issued where the
    // word is loaded, the scalar copy taken where it is needed)
    auto rfl = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); };
    // a leaf-load, sink-store or memory-read chunk whose first instruction
    // for this lane is `raw`
    auto other_chunk = [&](const uint4 raw, const uint32_t ch) {
      const uint32_t start = ch & 0xFFFF, cnt = ((ch >> 16) & 0xFF) + 1, op = ch >> 24;
      if (op == I_MEMRD) {
        if (lane < cnt) {
          const Dec in = decode(raw);
          const uint64_t a = at(in.a);
          const uint64_t depth = A.mem_depth[in.aux];
          const uint64_t addr = (depth & (depth - 1)) ? a % depth : (a & (depth - 1));
          at(in.dst) = A.mem[A.mem_off[in.aux] + addr] & wmask(in.w);
        }
      } else {
        // leaf loads and sink stores, up to four per lane, loads all issued
        // before the first is used (the raw instructions are kept, not their
        // decoded fields, to spare registers)
        uint4 rq[4];
        uint64_t v[4];
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
          const uint32_t e = lane + 64 * q;
          if (e < cnt) {
            rq[q] = q == 0 ? raw : Is[start + e];
            const Dec in = decode(rq[q]);
            if (op == I_LDREG) {
              v[q] = cur[in.aux];
            } else if (op == I_LDIN) {
              if (A.in_vals) {
                if (cyc < A.in_first || cyc >= A.in_first + A.in_count) { atomicOr(&A.error[1], 1u); v[q] = 0; }
                else v[q] = A.in_vals[(cyc - A.in_first) * A.I + in.aux];
              } else {
                v[q] = hmix(A.in_keys[in.aux] ^ cyc);
              }
            } else {
              v[q] = at(in.a);
            }
          }
        }
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
          const uint32_t e = lane + 64 * q;
          if (e < cnt) {
            const Dec in = decode(rq[q]);
            const uint64_t x = v[q] & wmask(in.w);
            if (op == I_LDREG || op == I_LDIN) {
              at(in.dst) = x;
            } else if (op == I_STREG) {
              nxt[in.aux] = x;
              if (A.digest_part) dacc += hmix((uint64_t)in.aux ^ hmix(x));
            } else {
              A.outputs[in.aux] = x;
            }
          }
        }
      }
    };
    if (STAGED) {
      // the next chunk's first instruction is read while this one runs, and
      // the chunk word two ahead
      uint32_t ch = rfl(ctab[0]), chn = rfl(ctab[1]);
      uint4 raw = first_instr(ch);
      while (c < n_ch) {
        if ((ch >> 24) == I_ALU) {
          // a run of operator chunks: operand reads, then the next chunk's
          // first instruction; only the operands are waited for
          do {
            const Dec in = decode(raw);
            uint64_t a = at(in.a), b = at(in.b), cc = at(in.c);
            const uint4 rn = first_instr(chn);
            const uint32_t w2 = ctab[c + 2];
            asm volatile("; operands of a mixed chunk ready" : "+v"(a), "+v"(b), "+v"(cc));
            const uint32_t present = __builtin_amdgcn_readfirstlane(in.aux);
            // lanes past the chunk's end repeat its last instruction on the
            // same operands, so their store writes the same value to the
            // same slot and needs no guard
            at(in.dst) = alu_mixed(present, in.op, in.w, a, b, cc);
            ++c;
            ch = chn;
            chn = rfl(w2);
            raw = rn;
            if (TRACE && trace_row) stamp(c);
            // the chunk table is zero past the last chunk (kind 0), so the
            // run also ends at the end of the process
          } while ((ch >> 24) == I_ALU);
          continue;
        }
        const uint4 rn = first_instr(chn);
        const uint32_t w2 = ctab[c + 2];
        other_chunk(raw, ch);
        ++c;
        ch = chn;
        chn = rfl(w2);
        raw = rn;
        if (TRACE && trace_row) stamp(c);
      }
    } else {
      // instructions from global memory: kWaveSlots slots hold the first
      // instructions of chunks c .. c + kWaveSlots - 1; a chunk decodes its
      // slot and refills it with chunk c + kWaveSlots's, so every load has
      // kWaveSlots chunks' time to land.  The loop is unrolled by kWaveSlots
      // so that no slot is ever copied while its load is in flight (a copy
      // would wait for it at once).  cw holds the wave-uniform chunk words
      // c .. c + kWaveSlots.
      constexpr uint32_t K = kWaveSlots;
      static_assert(K >= 2 && K <= 4, "two to four slots");
      uint32_t cw[K + 1];
#pragma unroll
      for (uint32_t k = 0; k <= K; ++k) cw[k] = rfl(ctab[k]);
      uint4 s0 = first_instr(cw[0]), s1 = first_instr(cw[1]);
      uint4 s2 = K > 2 ? first_instr(cw[2]) : uint4{0, 0, 0, 0};
      uint4 s3 = K > 3 ? first_instr(cw[3]) : uint4{0, 0, 0, 0};
      auto one = [&](uint4& slot) {
        const uint32_t wn = ctab[c + K + 1];
        const uint32_t ch = cw[0];
        if ((ch >> 24) == I_ALU) {
          const Dec in = decode(slot);
          uint64_t a = at(in.a), b = at(in.b), cc = at(in.c);
          slot = first_instr(cw[K]);
          asm volatile("; operands of a mixed chunk ready" : "+v"(a), "+v"(b), "+v"(cc));
          const uint32_t present = __builtin_amdgcn_readfirstlane(in.aux);
          // unguarded store: lanes past the chunk's end repeat its last
          // instruction (same operands, same slot, same value)
          at(in.dst) = alu_mixed(present, in.op, in.w, a, b, cc);
        } else {
          const uint4 raw = slot;
          slot = first_instr(cw[K]);
          other_chunk(raw, ch);
        }
        ++c;
#pragma unroll
        for (uint32_t k = 0; k < K; ++k) cw[k] = cw[k + 1];
        cw[K] = rfl(wn);
        if (TRACE && trace_row) stamp(c);
      };
      while (c < n_ch) {
        one(s0);
        if (c >= n_ch) break;
        one(s1);
        if (c >= n_ch) break;
        if constexpr (K > 2) {
          one(s2);
          if (c >= n_ch) break;
        }
        if constexpr (K > 3) {
          one(s3);
          if (c >= n_ch) break;
        }
      }
    }
    if (lane == 0) {
      for (uint32_t k = 0; k < pp.n_wp; ++k) {
        const Dec in = decode(Is[pp.n_instr + k]);
        if (at(in.a) != 0) {
          const uint32_t m = in.aux;
          const uint64_t depth = A.mem_depth[m], av = at(in.b);
          const uint64_t addr = (depth & (depth - 1)) ? av % depth : (av & (depth - 1));
          A.mem[A.mem_off[m] + addr] = at(in.c) & wmask(in.w);
        }
      }
    }
    if (A.digest_part) {
      for (int off = 32; off > 0; off >>= 1) dacc += __shfl_xor(dacc, off);
      const uint64_t k = cyc - A.digest_first;
      if (lane == 0 && k < A.digest_max) A.digest_part[k * gridDim.x + blockIdx.x] = dacc;
    }
    if (trace_row && lane == 0) trace_row[A.trace_stride - 2] = __builtin_amdgcn_s_memrealtime();
    if (PERSISTENT) {
      if (gridDim.x > 1) {
        if (!grid_barrier(A.flags, A.error, gridDim.x, A.epoch0 + t + 1, &abort_flag)) return;
      } else {
        asm volatile("" ::: "memory");
      }
    }
    if (trace_row && lane == 0) trace_row[A.trace_stride - 1] = __builtin_amdgcn_s_memrealtime();
  }
}

__global__ void __launch_bounds__(64) plain_wave_persistent(PlainArgs A) { plain_wave_body<true, true, false>(A); }
__global__ void __launch_bounds__(64) plain_wave_cycle(PlainArgs A) { plain_wave_body<false, true, false>(A); }
__global__ void __launch_bounds__(64) plain_wave_persistent_g(PlainArgs A) { plain_wave_body<true, false, false>(A); }
__global__ void __launch_bounds__(64) plain_wave_cycle_g(PlainArgs A) { plain_wave_body<false, false, false>(A); }
// the same with phase timestamps (a sim with tracing enabled): the untraced
// kernels carry no per-chunk test for it
__global__ void __launch_bounds__(64) plain_wave_persistent_trace(PlainArgs A) { plain_wave_body<true, true, true>(A); }
__global__ void __launch_bounds__(64) plain_wave_cycle_trace(PlainArgs A) { plain_wave_body<false, true, true>(A); }
__global__ void __launch_bounds__(64) plain_wave_persistent_g_trace(PlainArgs A) {
  plain_wave_body<true, false, true>(A);
}
__global__ void __launch_bounds__(64) plain_wave_cycle_g_trace(PlainArgs A) { plain_wave_body<false, false, true>(A); }

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
