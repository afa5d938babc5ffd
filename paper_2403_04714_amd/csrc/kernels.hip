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

template <bool PERSISTENT>
__device__ void plain_body(const PlainArgs& A) {
  extern __shared__ uint64_t lds[];
  __shared__ int abort_flag;
  __shared__ uint64_t red[16];
  const uint32_t tid = threadIdx.x, nthr = blockDim.x;
  const PlainProc pp = A.procs[blockIdx.x];
  uint64_t* slot = lds;
  const uint32_t n_instr_all = A.levels[pp.lvl_off + pp.n_lvls] - A.levels[pp.lvl_off] + pp.n_wp;
  const uint32_t ibase = A.levels[pp.lvl_off];           // first level instruction
  const Instr* I = A.instr + ibase;
  Instr* Is = reinterpret_cast<Instr*>(lds + A.slot_words);
  if (A.stage_instr) {
    // stage the level and commit instructions (contiguous) in LDS
    for (uint32_t i = tid; i < n_instr_all; i += nthr) Is[i] = I[i];
    I = Is;
  }
  for (uint32_t i = tid; i < pp.n_consts; i += nthr) {
    const Instr in = A.instr[pp.const_off + i];
    slot[in.dst] = A.consts[in.aux];
  }
  if (tid == 0) abort_flag = 0;
  __syncthreads();
  const uint32_t* lv = A.levels + pp.lvl_off;
  const uint64_t cyc0 = A.cycle_ptr ? *A.cycle_ptr + A.cycle0 : A.cycle0;
  for (uint32_t t = 0; t < A.n_cycles; ++t) {
    const uint64_t cyc = cyc0 + t;
    const uint64_t* cur = A.state + (cyc & 1) * A.R;
    uint64_t* nxt = A.state + ((cyc + 1) & 1) * A.R;
    uint64_t dacc = 0;
    for (uint32_t L = 0; L < pp.n_lvls; ++L) {
      const uint32_t lo = lv[L] - ibase, hi = lv[L + 1] - ibase;
      for (uint32_t i = lo + tid; i < hi; i += nthr) {
        const Instr in = I[i];
        const uint32_t op = in.op, w = in.w;
        if (op <= I_MUL && op >= I_AND) {
          uint64_t a = slot[in.a];
          uint64_t b = in.b != 0xFFFF ? slot[in.b] : 0;
          uint64_t c = in.c != 0xFFFF ? slot[in.c] : 0;
          slot[in.dst] = alu(op, w, a, b, c);
        } else if (op == I_LDREG) {
          slot[in.dst] = cur[in.aux] & wmask(w);
        } else if (op == I_LDIN) {
          uint64_t x;
          if (A.in_vals) {
            if (cyc < A.in_first || cyc >= A.in_first + A.in_count) { atomicOr(&A.error[1], 1u); x = 0; }
            else x = A.in_vals[(cyc - A.in_first) * A.I + in.aux];
          } else {
            x = hmix(A.in_keys[in.aux] ^ cyc);
          }
          slot[in.dst] = x & wmask(A.in_width[in.aux]) & wmask(w);
        } else if (op == I_MEMRD) {
          const uint32_t m = in.aux;
          const uint64_t addr = slot[in.a] % A.mem_depth[m];
          slot[in.dst] = A.mem[A.mem_off[m] + addr] & wmask(w);
        } else if (op == I_STREG) {
          const uint64_t v = slot[in.a] & wmask(w);
          nxt[in.aux] = v;
          if (A.digest_part) dacc += hmix((uint64_t)in.aux ^ hmix(v));
        } else if (op == I_STOUT) {
          A.outputs[in.aux] = slot[in.a];
        }
      }
      __syncthreads();
    }
    // memory commit after every read of this cycle, in port order
    if (tid == 0) {
      const uint32_t wlo = lv[pp.n_lvls] - ibase;
      for (uint32_t k = 0; k < pp.n_wp; ++k) {
        const Instr in = I[wlo + k];
        if (slot[in.a] != 0) {
          const uint32_t m = in.aux;
          A.mem[A.mem_off[m] + slot[in.b] % A.mem_depth[m]] = slot[in.c] & wmask(in.w);
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
    if (PERSISTENT) {
      if (gridDim.x > 1) {
        if (!grid_barrier(A.flags, A.error, gridDim.x, A.epoch0 + t + 1, &abort_flag)) return;
      } else {
        __syncthreads();
      }
    }
  }
}

__global__ void __launch_bounds__(1024) plain_persistent(PlainArgs A) { plain_body<true>(A); }
__global__ void __launch_bounds__(1024) plain_cycle(PlainArgs A) { plain_body<false>(A); }

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
    return hipLaunchCooperativeKernel((const void*)plain_persistent, dim3(G), dim3(threads), args,
                                      (unsigned)lds_bytes, s);
  }
  hipLaunchKernelGGL(plain_cycle, dim3(G), dim3(threads), lds_bytes, s, a);
  return hipGetLastError();
}

hipError_t plain_occupancy(int* blocks_per_cu, uint32_t threads, size_t lds_bytes) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, plain_persistent, (int)threads,
                                                      lds_bytes);
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
