// kernels.h -- argument blocks and launch entry points of the device code
// (host and device visible).  Internal to libfibersim.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "isa.h"

namespace fsim {

struct PlainArgs {
  const Instr* instr;
  const uint32_t* levels;
  const PlainProc* procs;
  const uint64_t* consts;
  uint64_t* state;            // [2][R]: cur = cycle & 1
  uint64_t* outputs;          // [O]
  uint64_t* mem;              // all memories, back to back
  const uint64_t* mem_off;    // [M]
  const uint32_t* mem_depth;  // [M]
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
  uint32_t instr_words;       // 16-byte instruction slots staged in LDS
  uint64_t cycle0;            // absolute cycle at the first cycle of this launch
  uint32_t n_cycles;
  uint32_t epoch0;            // barrier epoch before this launch
  const uint64_t* cycle_ptr;  // graph mode: absolute base cycle in device memory
};

hipError_t launch_plain(const PlainArgs& a, uint32_t G, uint32_t threads, size_t lds_bytes,
                        bool persistent, hipStream_t s);
hipError_t plain_occupancy(int* blocks_per_cu, uint32_t threads, size_t lds_bytes, bool staged);
hipError_t launch_digest_reduce(const uint64_t* part, uint32_t G, uint64_t n, uint64_t* out,
                                hipStream_t s);
hipError_t launch_stim_keys(uint64_t* keys, uint64_t seed_base, uint32_t n_inst, uint32_t I,
                            hipStream_t s);
hipError_t launch_add_u64(uint64_t* p, uint64_t v, hipStream_t s);

}  // namespace fsim
