// kernels.h -- argument blocks and launch entry points of the device code
// (host and device visible).  Internal to libfibersim.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "isa.h"

namespace fsim {

// One-wave plain kernel: the operator levels run in groups of this many
// chunks, and the instructions of the next group are fetched when a group
// starts, so a fetch has a whole group's time to land.  The LDS chunk table
// has room for 2 kGroup entries past a process's last chunk (the read-ahead),
// which repeat its last operator chunk.
constexpr uint32_t kGroup = 2;

// Words of the grid barrier's flag array for G workgroups: one epoch flag per
// workgroup, then one per group of 64 workgroups.
constexpr uint32_t barrier_words(uint32_t G) { return G + (G + 63) / 64; }

struct PlainArgs {
  const uint64_t* code;        // instruction words (isa.h)
  const uint32_t* levels;      // per process: chunk index where each level starts
  const uint64_t* chunks;      // chunk words
  const PlainProc* procs;
  uint64_t* state;            // [2][R]: cur = cycle & 1
  uint64_t* outputs;          // [O]
  uint64_t* mem;              // all memories, back to back
  const uint64_t* mem_off;    // [M]
  const uint32_t* mem_depth;  // [M]
  const uint64_t* mem_magic;  // [M]: floor((2^64 - 1) / depth)
  const uint8_t* in_width;    // [I]
  const uint64_t* in_keys;    // [I]: H(H(seed) ^ p)
  const uint64_t* in_vals;    // explicit inputs [n][I], or null
  uint64_t in_first, in_count;
  uint64_t* digest_part;      // [max_cycles][G] or null
  uint64_t digest_first, digest_max;
  uint64_t* trace;            // phase timestamps [max][G][trace_stride], or null
  uint64_t trace_first, trace_max;
  uint32_t trace_stride;      // levels + 3
  uint32_t* flags;            // [G] barrier epochs
  uint32_t* error;            // [0] barrier timeout, [1] input window
  uint32_t R, I;
  uint32_t stage_instr;       // instructions staged in LDS
  uint32_t slot_words;        // u64 words of LDS reserved for slots
  uint32_t ctab_words;        // one-wave kernel: u64 entries of the LDS chunk table after the slots
                              // (the most chunks of any process + 2 kGroup read-ahead entries)
  uint32_t instr_words;       // instruction words staged in LDS (after the chunk table)
  uint64_t cycle0;            // absolute cycle at the first cycle of this launch
  uint32_t n_cycles;
  uint32_t epoch0;            // barrier epoch before this launch
  const uint64_t* cycle_ptr;  // graph mode: absolute base cycle in device memory
  uint32_t single_wave;       // 64-thread workgroups: the one-wave kernel
  uint32_t dense_flag;        // the chunk flag that selects the opcode-bit tree (kDenseChunk or kDenseLow)
};

// Batched form: one wave per (process, tile of 64 instances).  State is kept
// per register class: 1-bit registers as 64-instance masks [reg][tile],
// narrow ones as u32 [reg][instance], wide ones as u64 [reg][instance], each
// double-buffered by cycle parity.
struct BatchArgs {
  const Instr* instr;
  uint64_t n_instr_total;     // instructions in the whole program array
  const BatchProc* procs;
  const uint64_t* consts;
  uint64_t* stB;              // [2][nB][n_tiles]
  uint32_t* stW;              // [2][nW][n_pad]
  uint64_t* stD;              // [2][nD][n_pad]
  uint64_t* outputs;          // [O][n_pad]
  uint64_t* mem;              // [words][n_pad]
  const uint64_t* mem_off;    // [M]
  const uint32_t* mem_depth;  // [M]
  const uint64_t* keys;       // [I][n_pad]: H(H(seed_i) ^ p)
  const uint64_t* in_vals;    // explicit [n][I][n_inst] or null
  uint64_t in_first, in_count;
  uint64_t* digest;           // [max][n_inst] or null
  uint64_t digest_first, digest_max;
  uint32_t* error;
  const uint64_t* cycle_ptr;  // graph mode: base cycle in device memory
  uint64_t cycle0;
  uint32_t P, n_tiles, tpw, n_inst, n_pad, I;
  uint32_t nB, nW, nD;
  uint32_t wave_bytes;        // LDS bytes of one tile's region (multiple of 16)
  uint32_t twave;             // tiles of 64 instances per wave (1 or 2)
};

hipError_t launch_batched(const BatchArgs& a, uint32_t grid, uint32_t threads, size_t lds_bytes,
                          hipStream_t s);
hipError_t launch_batched_multi(const BatchArgs* jobs, const uint32_t* wg_start, const uint64_t* cycle_base,
                                const uint32_t* ticks, uint32_t n_jobs, uint32_t tick, uint32_t grid,
                                size_t lds_bytes, hipStream_t s);
hipError_t launch_plain(const PlainArgs& a, uint32_t G, uint32_t threads, size_t lds_bytes,
                        bool persistent, hipStream_t s);
hipError_t plain_occupancy(int* blocks_per_cu, uint32_t threads, size_t lds_bytes, bool staged,
                           bool single_wave);
hipError_t launch_digest_reduce(const uint64_t* part, uint32_t G, uint64_t n, uint64_t* out,
                                hipStream_t s);
hipError_t launch_stim_keys(uint64_t* keys, uint64_t seed_base, uint32_t n_inst, uint32_t I,
                            hipStream_t s);
hipError_t launch_add_u64(uint64_t* p, uint64_t v, hipStream_t s);
// column `col` of a row-major [rows][pitch] table of 4- or 8-byte values
// copied into the contiguous vector `vec` (to_table false) or from it (true)
hipError_t launch_column_copy(void* table, uint32_t elem, uint64_t pitch, uint64_t col, uint64_t rows,
                              void* vec, bool to_table, hipStream_t s);

}  // namespace fsim
