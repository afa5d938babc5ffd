// kernels.hip -- gfx950 device code of libfibersim.
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
// The barrier (Sec. 4.1 measures the same cost on the IPU and on x64) uses
// one epoch flag per workgroup: arrivals are plain stores to distinct words
// and every workgroup polls all flags, so no read-modify-write serialises
// the arrivals.  Cross-XCD visibility of the next-state stores comes from an
// agent-scope release before the flag store and an agent-scope acquire after
// the poll.
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

// One combinational operator on zero-extended operands, masked to w.
__device__ __forceinline__ uint64_t alu(uint32_t op, uint32_t w, uint64_t a, uint64_t b, uint64_t c) {
  uint64_t r;
  switch (op) {
    case I_AND: r = a & b; break;
    case I_OR:  r = a | b; break;
    case I_XOR: r = a ^ b; break;
    case I_NOT: r = ~a; break;
    case I_ADD: r = a + b; break;
    case I_SUB: r = a - b; break;
    case I_MUX: r = a ? b : c; break;
    case I_SHL: r = b >= 64 ? 0 : (a << b); break;   // explicit: the hardware
    case I_SHR: r = b >= 64 ? 0 : (a >> b); break;   // takes amounts mod 64
    case I_EQ:  r = a == b; break;
    case I_LT:  r = a < b; break;
    case I_MUL: r = a * b; break;
    default:    r = 0; break;
  }
  return r & wmask(w);
}

static constexpr long kSpinLimit = 1l << 22;

// Grid-wide barrier over G workgroups (see the file comment).  Returns false
// if the poll exceeded its bound or another workgroup already gave up; the
// caller then leaves its cycle loop so that every wave exits.
__device__ __forceinline__ bool grid_barrier(uint32_t* flags, uint32_t* error, uint32_t G,
                                             uint32_t epoch, int* lds_abort) {
  __syncthreads();
  if (threadIdx.x < 64) {
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&flags[blockIdx.x], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    long spins = 0;
    bool ok = true;
    for (;;) {
      bool mine = true;
      for (uint32_t g = threadIdx.x; g < G; g += 64) {
        uint32_t v = __hip_atomic_load(&flags[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((int32_t)(v - epoch) < 0) mine = false;
      }
      if (__all(mine)) break;
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 1023) == 0) {
        if (__hip_atomic_load(&error[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) { ok = false; break; }
        if (spins > kSpinLimit) {
          if (threadIdx.x == 0) atomicOr(&error[0], 1u);
          ok = false;
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x == 0) *lds_abort = ok ? 0 : 1;
  }
  __syncthreads();
  return *lds_abort == 0;
}

struct Dec {
  uint32_t op, w, dst, a, b, c, aux;
};

// The 16-byte instruction is read with one 128-bit load and decoded from
// registers: x = op | w << 8 | cls << 16 | flags << 24, y = dst | a << 16,
// z = b | c << 16, w = aux.
__device__ __forceinline__ Dec decode(uint4 r) {
  Dec d;
  d.op = r.x & 0xFF; d.w = (r.x >> 8) & 0xFF;
  d.dst = r.y & 0xFFFF; d.a = r.y >> 16;
  d.b = r.z & 0xFFFF; d.c = r.z >> 16;
  d.aux = r.w;
  return d;
}

template <bool PERSISTENT, bool STAGED>
__device__ void plain_body(const PlainArgs& A) {
  extern __shared__ uint64_t lds[];
  __shared__ int abort_flag;
  __shared__ uint64_t red[16];
  const uint32_t tid = threadIdx.x, nthr = blockDim.x;
  const PlainProc pp = A.procs[blockIdx.x];
  uint64_t* slot = lds;
  const uint32_t ibase = A.levels[pp.lvl_off];           // first level instruction
  const uint32_t n_instr_all = A.levels[pp.lvl_off + pp.n_lvls] - ibase + pp.n_wp;
  const uint4* Ig = reinterpret_cast<const uint4*>(A.instr) + ibase;
  uint4* Is = reinterpret_cast<uint4*>(lds + A.slot_words);
  // level table (relative to ibase) after the staged instructions
  uint32_t* lvs = reinterpret_cast<uint32_t*>(Is + (STAGED ? A.instr_words : 0));
  if (STAGED)
    for (uint32_t i = tid; i < n_instr_all; i += nthr) Is[i] = Ig[i];
  for (uint32_t L = tid; L <= pp.n_lvls; L += nthr) lvs[L] = A.levels[pp.lvl_off + L] - ibase;
  for (uint32_t i = tid; i < pp.n_consts; i += nthr) {
    const Instr in = A.instr[pp.const_off + i];
    slot[in.dst] = A.consts[in.aux];
  }
  if (tid == 0) abort_flag = 0;
  __syncthreads();
  auto fetch = [&](uint32_t i) -> uint4 { return STAGED ? Is[i] : Ig[i]; };
  const uint32_t n_lvls = pp.n_lvls;
  // the level table lives in the lanes of two registers and is read with
  // v_readlane (no LDS round trip on the level-to-level critical path);
  // deeper processes fall back to the LDS copy
  const uint32_t lane = tid & 63;
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
    uint32_t lo = lvl(0), hi = lvl(1);
    uint4 raw = (lo + tid < hi) ? fetch(lo + tid) : make_uint4(0, 0, 0, 0);
    for (uint32_t L = 0; L < n_lvls; ++L) {
      // next level's bounds and this thread's first instruction there, issued
      // before this level's operand reads so that their wait covers it
      const uint32_t nhi = L + 1 < n_lvls ? lvl(L + 2) : hi;
      const bool have_next = L + 1 < n_lvls && hi + tid < nhi;
      uint4 raw_next = have_next ? fetch(hi + tid) : raw;
      if (L == 0) {
        // leaf level: current register values and this cycle's inputs
        for (uint32_t i = lo + tid; i < hi; i += nthr) {
          if (i != lo + tid) raw = fetch(i);
          const Dec in = decode(raw);
          uint64_t v;
          if (in.op == I_LDREG) {
            v = cur[in.aux];
          } else if (A.in_vals) {
            if (cyc < A.in_first || cyc >= A.in_first + A.in_count) { atomicOr(&A.error[1], 1u); v = 0; }
            else v = A.in_vals[(cyc - A.in_first) * A.I + in.aux];
          } else {
            v = hmix(A.in_keys[in.aux] ^ cyc);
          }
          slot[in.dst] = v & wmask(in.w);   // LDIN widths fold in the port width
        }
      } else if (L + 1 < n_lvls) {
        // operator level: every operand slot is valid (unused ones repeat a),
        // so the three LDS reads issue together and one wait covers them
        for (uint32_t i = lo + tid; i < hi; i += nthr) {
          if (i != lo + tid) raw = fetch(i);
          const Dec in = decode(raw);
          uint64_t a = slot[in.a], b = slot[in.b], c = slot[in.c];
          // keep the three reads (and their single wait) ahead of the
          // per-opcode branches: without this the compiler sinks each read
          // into the cases that use it and every case then waits on its own
          asm volatile("" : "+v"(a), "+v"(b), "+v"(c));
          if (in.op == I_MEMRD) {
            const uint64_t depth = A.mem_depth[in.aux];
            const uint64_t addr = (depth & (depth - 1)) ? a % depth : (a & (depth - 1));
            slot[in.dst] = A.mem[A.mem_off[in.aux] + addr] & wmask(in.w);
          } else {
            slot[in.dst] = alu(in.op, in.w, a, b, c);
          }
        }
      } else {
        // store level: next register values and outputs
        for (uint32_t i = lo + tid; i < hi; i += nthr) {
          if (i != lo + tid) raw = fetch(i);
          const Dec in = decode(raw);
          const uint64_t v = slot[in.a] & wmask(in.w);
          if (in.op == I_STREG) {
            nxt[in.aux] = v;
            if (A.digest_part) dacc += hmix((uint64_t)in.aux ^ hmix(v));
          } else {
            A.outputs[in.aux] = v;
          }
        }
      }
      raw = raw_next;
      lo = hi;
      hi = nhi;
      if (one_wave) asm volatile("" ::: "memory");
      else __syncthreads();
      if (trace_row && L + 2 < A.trace_stride) trace_row[L + 1] = __builtin_amdgcn_s_memrealtime();
    }
    // memory commit after every read of this cycle, in port order
    if (tid == 0) {
      const uint32_t wlo = lvs[n_lvls];
      for (uint32_t k = 0; k < pp.n_wp; ++k) {
        const Dec in = decode(fetch(wlo + k));
        if (slot[in.a] != 0) {
          const uint32_t m = in.aux;
          const uint64_t depth = A.mem_depth[m], av = slot[in.b];
          const uint64_t addr = (depth & (depth - 1)) ? av % depth : (av & (depth - 1));
          A.mem[A.mem_off[m] + addr] = slot[in.c] & wmask(in.w);
        }
      }
    }
    if (A.digest_part) {
      // workgroup reduction of the digest terms; partial per workgroup
      for (int off = 32; off > 0; off >>= 1) dacc += __shfl_xor(dacc, off);
      if ((tid & 63) == 0) red[tid >> 6] = dacc;
      __syncthreads();
      if (tid == 0) {
        uint64_t s = 0;
        for (uint32_t k = 0; k < (nthr + 63) / 64; ++k) s += red[k];
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

// stimulus keys: keys[i * I + p] = H(H(seed_base + i) ^ p)
__global__ void stim_keys(uint64_t* keys, uint64_t seed_base, uint32_t n_inst, uint32_t I) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_inst * I) return;
  uint32_t i = k / I, p = k % I;
  keys[k] = hmix(hmix(seed_base + i) ^ (uint64_t)p);
}

}  // namespace fsim

// ---------------------------------------------------------------- launches
namespace fsim {

hipError_t launch_plain(const PlainArgs& a, uint32_t G, uint32_t threads, size_t lds_bytes,
                        bool persistent, hipStream_t s) {
  if (persistent) {
    void* args[] = {const_cast<PlainArgs*>(&a)};
    return hipLaunchCooperativeKernel(a.stage_instr ? (const void*)plain_persistent : (const void*)plain_persistent_g,
                                      dim3(G), dim3(threads), args, (unsigned)lds_bytes, s);
  }
  if (a.stage_instr) hipLaunchKernelGGL(plain_cycle, dim3(G), dim3(threads), lds_bytes, s, a);
  else hipLaunchKernelGGL(plain_cycle_g, dim3(G), dim3(threads), lds_bytes, s, a);
  return hipGetLastError();
}

hipError_t plain_occupancy(int* blocks_per_cu, uint32_t threads, size_t lds_bytes, bool staged) {
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
