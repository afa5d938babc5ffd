// device_common.h -- device helpers shared by the plain and the batched
// kernels of libfibersim: the stimulus hash, width masks, the operator
// evaluation, the grid barrier and the instruction decoding.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "isa.h"
#include "kernels.h"

namespace fsim {

// SplitMix64 output function: the first output of a SplitMix64 generator whose
// state is x (Steele, Lea and Flood, OOPSLA 2014; published constants).
__device__ __forceinline__ uint64_t hmix(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t wmask(uint32_t w) { return ~0ull >> (64u - w); }

// One operator per lane, all lanes of one opcode `k` (wave-uniform): one
// dispatch on k with scalar branches.  The result is cut to the operator's
// width by `mask`.
__device__ __forceinline__ uint64_t alu_single(uint32_t k, uint64_t mask, uint64_t a, uint64_t b, uint64_t c) {
  uint64_t r = 0;
  // the empty asm keeps the dispatch a tree of real (scalar) branches
  switch (k) {
    case I_AND: asm volatile(""); r = a & b; break;
    case I_OR:  asm volatile(""); r = a | b; break;
    case I_XOR: asm volatile(""); r = a ^ b; break;
    case I_NOT: asm volatile(""); r = ~a; break;
    case I_ADD: asm volatile(""); r = a + b; break;
    case I_SUB: asm volatile(""); r = a - b; break;
    case I_MUX: asm volatile(""); r = a ? b : c; break;
    case I_SHL: asm volatile(""); r = b >= 64 ? 0 : (a << (b & 63)); break;
    case I_SHR: asm volatile(""); r = b >= 64 ? 0 : (a >> (b & 63)); break;
    case I_EQ:  asm volatile(""); r = a == b; break;
    case I_LT:  asm volatile(""); r = a < b; break;
    case I_MUL: asm volatile(""); r = a * b; break;
    default: break;
  }
  return r & mask;
}

// One operator per lane, opcodes differing between lanes.  `present` (wave
// uniform) holds the opcodes that occur in the chunk; each is evaluated for
// every lane and selected where it is the lane's own: a few vector
// instructions per opcode present and no divergent branch.  (Running each
// opcode under an execution mask of its lanes instead saves the selects but
// adds scalar mask work and a branch per opcode; it measured 1-2% slower on
// every workload.)  An opcode's block follows its test in the code, so an
// opcode present costs no taken branch.
__device__ __forceinline__ uint64_t alu_select(uint32_t present, uint32_t op, uint64_t mask, uint64_t a, uint64_t b,
                                               uint64_t c) {
  uint64_t r = 0;
  // the empty asm keeps each test a real (scalar) branch, so opcodes absent
  // from the chunk cost two scalar instructions instead of being computed
#define FSIM_MIXED(OPC, EXPR) \
  if (__builtin_expect((present & (1u << (OPC))) != 0, 1)) { asm volatile(""); r = op == (OPC) ? (uint64_t)(EXPR) : r; }
  FSIM_MIXED(I_AND, a & b)
  FSIM_MIXED(I_OR, a | b)
  FSIM_MIXED(I_XOR, a ^ b)
  FSIM_MIXED(I_NOT, ~a)
  FSIM_MIXED(I_ADD, a + b)
  FSIM_MIXED(I_SUB, a - b)
  FSIM_MIXED(I_MUX, a ? b : c)
  FSIM_MIXED(I_SHL, b >= 64 ? 0 : (a << (b & 63)))
  FSIM_MIXED(I_SHR, b >= 64 ? 0 : (a >> (b & 63)))
  FSIM_MIXED(I_EQ, a == b)
  FSIM_MIXED(I_LT, a < b)
  FSIM_MIXED(I_MUL, a * b)
#undef FSIM_MIXED
  return r & mask;
}

// The same for a chunk holding most opcodes and no MUL: every opcode is
// evaluated for every lane without a test (a test costs two scalar
// instructions, more than evaluating the few opcodes such a chunk lacks),
// and the lane's own result
// is picked by a selection tree on the bits of its opcode (AND = 4 .. LT =
// 14): ten 64-bit selects under four lane masks computed up front.
__device__ __forceinline__ uint64_t alu_dense(uint32_t op, uint64_t mask, uint64_t a, uint64_t b, uint64_t c) {
  const bool o0 = op & 1, o1 = op & 2, ge8 = op >= 8, ge12 = op >= 12;
  const bool big = b >= 64;
  const uint64_t x_and = a & b, x_or = a | b, x_xor = a ^ b, x_not = ~a;
  const uint64_t x_add = a + b, x_sub = a - b, x_mux = a ? b : c;
  const uint64_t x_shl = big ? 0 : a << (b & 63), x_shr = big ? 0 : a >> (b & 63);
  const uint64_t x_eq = a == b, x_lt = a < b;
  // (such a chunk holds no MUL: leaf 15 is never picked)
  const uint64_t p4 = o0 ? x_or : x_and, p6 = o0 ? x_not : x_xor;
  const uint64_t p8 = o0 ? x_sub : x_add, p10 = o0 ? x_shl : x_mux;
  const uint64_t p12 = o0 ? x_eq : x_shr, p14 = x_lt;
  uint64_t q4 = o1 ? p6 : p4, q8 = o1 ? p10 : p8, q12 = o1 ? p14 : p12;
  // the empty asm has every lane compute all three before the last two
  // selects, which would otherwise become a lane-divergent branch
  asm volatile("" : "+v"(q4), "+v"(q8), "+v"(q12));
  const uint64_t r = ge12 ? q12 : (ge8 ? q8 : q4);
  return r & mask;
}

static constexpr long kSpinLimit = 1l << 22;

// Polls n epoch flags (one per lane, strided by 64) until every one has
// reached `epoch`.  Gives up, returning false, once another workgroup has
// raised the error word or the poll has exceeded its bound (then it raises
// the error word itself).
__device__ __forceinline__ bool poll_flags(const uint32_t* f, uint32_t n, uint32_t epoch, uint32_t* error) {
  long spins = 0;
  for (;;) {
    bool mine = true;
    for (uint32_t g = threadIdx.x; g < n; g += 64) {
      const uint32_t v = __hip_atomic_load(&f[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if ((int32_t)(v - epoch) < 0) mine = false;
    }
    if (__all(mine)) return true;
    __builtin_amdgcn_s_sleep(1);
    if ((++spins & 1023) == 0) {
      if (__hip_atomic_load(&error[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
      if (spins > kSpinLimit) {
        if (threadIdx.x == 0) atomicOr(&error[0], 1u);
        return false;
      }
    }
  }
}

// Grid-wide barrier over G workgroups (see the file comment), in two levels:
// each workgroup stores its epoch flag; the first workgroup of every group
// of 64 waits for its group's flags and then stores the group's flag; every
// workgroup waits for the group flags.  Returns false if a poll exceeded its
// bound or another workgroup already gave up; the caller then leaves its
// cycle loop so that every wave exits.
__device__ __forceinline__ bool grid_barrier(uint32_t* flags, uint32_t* error, uint32_t G,
                                             uint32_t epoch, int* lds_abort) {
  __syncthreads();
  if (threadIdx.x < 64) {
    uint32_t* const group_flags = flags + G;
    const uint32_t grp = blockIdx.x / 64;
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&flags[blockIdx.x], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    bool ok = true;
    if (blockIdx.x % 64 == 0) {
      const uint32_t n = G - 64 * grp < 64 ? G - 64 * grp : 64;
      ok = poll_flags(flags + 64 * grp, n, epoch, error);
      // what the group's workgroups wrote before their flags is published
      // again with the group flag
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (ok && threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&group_flags[grp], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (ok) ok = poll_flags(group_flags, (G + 63) / 64, epoch, error);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x == 0) *lds_abort = ok ? 0 : 1;
  }
  __syncthreads();
  return *lds_abort == 0;
}

// Fields of a plain-form instruction word (isa.h), from its low and high
// halves.  Fields come out as LDS byte offsets (unit x 4).
__device__ __forceinline__ uint32_t pw_op(uint32_t lo) { return lo & 15; }
// the mask of the value's width (the field holds 64 - width)
__device__ __forceinline__ uint64_t pw_mask(uint32_t lo) { return ~0ull >> ((lo >> 4) & 63); }
__device__ __forceinline__ uint32_t pw_f0(uint32_t lo) { return (lo >> 12) & 0x3FFC; }
__device__ __forceinline__ uint32_t pw_f1(uint32_t lo, uint32_t hi) {
  return (uint32_t)((((uint64_t)hi << 32) | lo) >> 24) & 0x3FFC;
}
__device__ __forceinline__ uint32_t pw_f2(uint32_t hi) { return (hi >> 4) & 0x3FFC; }
__device__ __forceinline__ uint32_t pw_f3(uint32_t hi) { return (hi >> 16) & 0x3FFC; }
// whether the destination in field 0 takes one unit (the high half's sign)
__device__ __forceinline__ bool pw_one0(uint32_t hi) { return (int32_t)hi < 0; }
// register, port, output or constant index (bits 26..61)
__device__ __forceinline__ uint64_t pw_index(uint32_t lo, uint32_t hi) {
  return (((uint64_t)(hi & 0x3FFFFFFFu)) << 6) | (lo >> 26);
}
// memory of a MEMRD (bits 38..61) and of a WPORT (bits 50..61)
__device__ __forceinline__ uint32_t pw_mem38(uint32_t hi) { return (hi >> 6) & 0xFFFFFF; }
__device__ __forceinline__ uint32_t pw_mem50(uint32_t hi) { return (hi >> 18) & 0xFFF; }

// one 16-byte batched-form instruction as four plain words: x = op | w << 8
// | cls << 16 | flags << 24, y = dst | a << 16, z = b | c << 16, w = aux
struct IWord { uint32_t x, y, z, w; };

}  // namespace fsim
