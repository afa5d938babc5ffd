// kernels_batched.hip -- gfx950 device code of libfibersim: the batched form
// (many independent stimulus instances of one design per launch) and the
// serving launch that advances every resident job by one cycle.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_common.h"

namespace fsim {


// ------------------------------------------------------------ batched form
//
// A wave evaluates one process for 64 instances (one lane per instance,
// Sec. 6.4's many-independent-tests scenario).  The instruction stream is
// wave-uniform, so it is fetched with scalar loads and dispatched with scalar
// branches.  Values live in LDS slots per class: a 1-bit value is one 64-lane
// ballot mask, a narrow value one u32 per lane, a wide value one u64 per lane.
// Operators whose operands and result are all 1-bit work on the masks
// directly.

// Read-only for the whole launch (program, constant pool, memory tables, the
// current half of the state): reading through the constant address space lets
// the compiler use scalar loads for wave-uniform addresses instead of a vector
// load plus a wait for every interpreted instruction.
template <class T>
using cptr = const __attribute__((address_space(4))) T*;
template <class T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
  return (cptr<T>)(p);
}

// One operand of a per-lane operator, zero-extended to 64 bits.  `off` is a
// byte offset into the wave's LDS region; the class picks the lane stride
// (1-bit masks and constants: every lane reads the same word; u32 and u64
// rows: one element per lane) and the extraction.  Rows of u32 are read as
// two u32 words so that only 4-byte alignment is assumed.
__device__ __forceinline__ uint64_t lread(const char* base, uint32_t cls, uint32_t off, uint32_t lane) {
  const uint32_t stride = (0x0840u >> (cls * 4)) & 0xF;      // B 0, W 4, D 8, K 0
  const uint32_t* p = reinterpret_cast<const uint32_t*>(base + off + lane * stride);
  const uint64_t v = (uint64_t)p[0] | ((uint64_t)p[1] << 32);
  const uint32_t sh = cls == C_B ? lane : 0;
  const uint64_t m = cls == C_B ? 1ull : cls == C_W ? 0xFFFFFFFFull : ~0ull;
  return (v >> sh) & m;
}

// Store a per-lane value into a slot of class cls (never a constant).
__device__ __forceinline__ void lwrite(char* base, uint32_t cls, uint32_t off, uint32_t lane, uint64_t v) {
  if (cls == C_B) {
    *reinterpret_cast<uint64_t*>(base + off) = __ballot(v & 1);   // the same mask from every lane
  } else if (cls == C_W) {
    reinterpret_cast<uint32_t*>(base + off)[lane] = (uint32_t)v;
  } else {
    reinterpret_cast<uint64_t*>(base + off)[lane] = v;
  }
}

// The instruction stream reaches the wave in blocks of 64 instructions: lane
// k holds instruction k of the block in four registers (one vector load per
// block, issued a whole block ahead), and the wave-uniform instruction is
// taken out with v_readlane.  Streaming the program through the scalar data
// cache instead costs a cache miss every few instructions once several
// waves per CU run different processes.
__device__ __forceinline__ IWord lane_word(const uint4& b, uint32_t l) {
  return IWord{(uint32_t)__builtin_amdgcn_readlane((int)b.x, (int)l), (uint32_t)__builtin_amdgcn_readlane((int)b.y, (int)l),
               (uint32_t)__builtin_amdgcn_readlane((int)b.z, (int)l), (uint32_t)__builtin_amdgcn_readlane((int)b.w, (int)l)};
}

__device__ __forceinline__ uint64_t mread(const char* base, uint32_t off) {
  return *reinterpret_cast<const uint64_t*>(base + off);
}

__device__ __forceinline__ uint32_t rlane(uint32_t v, uint32_t l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
}

// Raw operand load of a per-lane operator by class: a u64 row element (D), a
// u32 row element (W) or a wave-uniform word (a B mask or a K constant).  The
// value is not used here, so the loads of all operands are in flight before
// the first wait.  lane4 and lane8 are the lane's byte offsets in W and D rows.
__device__ __forceinline__ uint64_t vload(const char* base, uint32_t cls, uint32_t off, uint32_t lane4,
                                          uint32_t lane8) {
  if (cls == C_D) return *reinterpret_cast<const uint64_t*>(base + off + lane8);
  if (cls == C_W) return *reinterpret_cast<const uint32_t*>(base + off + lane4);
  return *reinterpret_cast<const uint64_t*>(base + off);
}

// The lane's bit of a loaded mask (class B); other classes pass unchanged.
__device__ __forceinline__ uint64_t vbit(uint32_t cls, uint64_t v, uint32_t lane) {
  return cls == C_B ? (v >> lane) & 1 : v;
}

// A per-lane operator on zero-extended operands (not yet masked to its
// width), for each of a wave's TW tiles, as one tree of uniform tests; cheap
// neighbours are selected, not branched to.
template <uint32_t TW>
__device__ __forceinline__ void alu_tree(uint32_t op, const uint64_t (&a)[TW], const uint64_t (&b)[TW],
                                         const uint64_t (&c)[TW], uint64_t (&r)[TW]) {
  if (op <= I_NOT) {
    if (op <= I_OR) {
#pragma unroll
      for (uint32_t t = 0; t < TW; ++t) r[t] = op == I_AND ? (a[t] & b[t]) : (a[t] | b[t]);
    } else {
#pragma unroll
      for (uint32_t t = 0; t < TW; ++t) r[t] = op == I_XOR ? (a[t] ^ b[t]) : ~a[t];
    }
  } else if (op <= I_MUX) {
    if (op == I_ADD) {
#pragma unroll
      for (uint32_t t = 0; t < TW; ++t) r[t] = a[t] + b[t];
    } else if (op == I_SUB) {
#pragma unroll
      for (uint32_t t = 0; t < TW; ++t) r[t] = a[t] - b[t];
    } else {
#pragma unroll
      for (uint32_t t = 0; t < TW; ++t) r[t] = a[t] ? b[t] : c[t];
    }
  } else if (op <= I_SHR) {
#pragma unroll
    for (uint32_t t = 0; t < TW; ++t)
      r[t] = b[t] >= 64 ? 0 : (op == I_SHL ? a[t] << (b[t] & 63) : a[t] >> (b[t] & 63));
  } else if (op <= I_LT) {
#pragma unroll
    for (uint32_t t = 0; t < TW; ++t) r[t] = op == I_EQ ? (uint64_t)(a[t] == b[t]) : (uint64_t)(a[t] < b[t]);
  } else {
#pragma unroll
    for (uint32_t t = 0; t < TW; ++t) r[t] = a[t] * b[t];
  }
}

// Store a per-lane result into a slot of class cls (never a constant).
__device__ __forceinline__ void vstore(char* base, uint32_t cls, uint32_t off, uint64_t v, uint32_t lane4,
                                       uint32_t lane8, uint32_t lane) {
  if (cls == C_D) {
    *reinterpret_cast<uint64_t*>(base + off + lane8) = v;
  } else if (cls == C_W) {
    *reinterpret_cast<uint32_t*>(base + off + lane4) = (uint32_t)v;
  } else {
    // every lane stores the same mask: no change of the execution mask
    *reinterpret_cast<uint64_t*>(base + off) = __ballot(v & 1);
  }
}

// One simulated cycle of one (process, tile group) work item of a batched
// sim.  Each wave interprets the process's instruction stream once for TW
// tiles of 64 instances: fetch, decode and dispatch (the scalar work, which
// bounds this kernel) are shared by the tiles, and only the per-lane data
// work is repeated per tile.  A tile past the last one (ragged tile count)
// repeats the last tile's reads and stores nothing.
template <uint32_t TW>
__device__ __forceinline__ void batched_body(const BatchArgs& A, uint32_t block, uint64_t cyc, char* lds) {
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t p = block % A.P, grp = block / A.P;
  const uint32_t tile0 = (grp * A.tpw + wave) * TW;
  if (tile0 >= A.n_tiles) return;                // no barriers below: a wave may leave early
  uint32_t tile[TW], inst[TW];
  bool live[TW], real[TW];
  char* base[TW];
#pragma unroll
  for (uint32_t t = 0; t < TW; ++t) {
    live[t] = tile0 + t < A.n_tiles;             // wave-uniform
    tile[t] = live[t] ? tile0 + t : A.n_tiles - 1;
    inst[t] = tile[t] * 64 + lane;               // < n_pad
    real[t] = live[t] && inst[t] < A.n_inst;
    base[t] = lds + (size_t)(wave * TW + t) * A.wave_bytes;
  }
  const BatchProc bp = A.procs[p];
  const uint4* prog = reinterpret_cast<const uint4*>(A.instr);
  // block b of this process: instructions instr_off + 64 b .. + 63, zero past
  // the end of the program array
  auto load_blk = [&](uint32_t b) -> uint4 {
    const uint64_t j = (uint64_t)bp.instr_off + 64ull * b + lane;
    return j < A.n_instr_total ? prog[j] : make_uint4(0, 0, 0, 0);
  };
  const cptr<uint64_t> mem_off = as_const(A.mem_off);
  const cptr<uint32_t> mem_depth = as_const(A.mem_depth);
  // each tile's region: the two constant masks, then the process's constants
#pragma unroll
  for (uint32_t t = 0; t < TW; ++t) {
    if (lane < 2) reinterpret_cast<uint64_t*>(base[t])[lane] = lane ? ~0ull : 0ull;
    for (uint32_t k = lane; k < bp.n_consts; k += 64)
      reinterpret_cast<uint64_t*>(base[t] + bp.kbase)[k] = A.consts[bp.const_off + k];
  }
  const uint32_t cur = cyc & 1, nxt = cur ^ 1;
  const cptr<uint64_t> stB_cur = as_const(A.stB + (size_t)cur * A.nB * A.n_tiles);
  uint64_t* stB_nxt = A.stB + (size_t)nxt * A.nB * A.n_tiles;
  const uint32_t* stW_cur = A.stW + (size_t)cur * A.nW * A.n_pad;
  uint32_t* stW_nxt = A.stW + (size_t)nxt * A.nW * A.n_pad;
  const uint64_t* stD_cur = A.stD + (size_t)cur * A.nD * A.n_pad;
  uint64_t* stD_nxt = A.stD + (size_t)nxt * A.nD * A.n_pad;
  uint64_t dacc[TW];
#pragma unroll
  for (uint32_t t = 0; t < TW; ++t) dacc[t] = 0;
  const uint32_t lane4 = 4 * lane, lane8 = 8 * lane;
  uint32_t i = 0;
  uint4 bc = load_blk(0);
  for (uint32_t blk = 0; i < bp.n_instr; ++blk) {
    // the next block is in flight while this one runs; it is waited for only
    // where a leaf run reaches into it, or when it becomes the current block
    // (a step advances i by at most 16, so it crosses at most one block)
    const uint4 bn = load_blk(blk + 1);
    // instruction j of the process, j in the current or the next block
    auto instr = [&](uint32_t j) -> IWord { return lane_word((j >> 6) == blk ? bc : bn, j & 63); };
    const uint32_t blk_end = bp.n_instr < 64 * (blk + 1) ? bp.n_instr : 64 * (blk + 1);
    while (i < blk_end) {
      const uint32_t l = i & 63;
      const uint32_t x = rlane(bc.x, l);
      const uint32_t op = x & 0xFF;
      uint32_t step = 1;
      // Uniform if/else trees throughout, each handler falling through to the
      // common step: switch statements and early exits cost a cascade of
      // scalar flag blocks per interpreted instruction on this target.
      if (op >= K_MASK_AND && op <= K_MASK_MUX) {
        // every operand and the result are 64-instance masks
        const uint32_t y = rlane(bc.y, l), z = rlane(bc.z, l);
        uint64_t ma[TW], mb[TW], r[TW];
#pragma unroll
        for (uint32_t t = 0; t < TW; ++t) {
          ma[t] = mread(base[t], y >> 16);
          mb[t] = mread(base[t], z & 0xFFFF);
        }
        if (op < K_MASK_NOT) {
          if (op == K_MASK_AND) {
#pragma unroll
            for (uint32_t t = 0; t < TW; ++t) r[t] = ma[t] & mb[t];
          } else if (op == K_MASK_OR) {
#pragma unroll
            for (uint32_t t = 0; t < TW; ++t) r[t] = ma[t] | mb[t];
          } else {
#pragma unroll
            for (uint32_t t = 0; t < TW; ++t) r[t] = ma[t] ^ mb[t];   // also 1-bit ADD and SUB (sums mod 2)
          }
        } else if (op < K_MASK_LT) {
#pragma unroll
          for (uint32_t t = 0; t < TW; ++t) r[t] = op == K_MASK_NOT ? ~ma[t] : ~(ma[t] ^ mb[t]);
        } else if (op == K_MASK_LT) {
#pragma unroll
          for (uint32_t t = 0; t < TW; ++t) r[t] = ~ma[t] & mb[t];
        } else {
#pragma unroll
          for (uint32_t t = 0; t < TW; ++t) r[t] = (ma[t] & mb[t]) | (~ma[t] & mread(base[t], z >> 16));   // MUX
        }
        // every lane stores the same mask: no change of the execution mask
#pragma unroll
        for (uint32_t t = 0; t < TW; ++t) *reinterpret_cast<uint64_t*>(base[t] + (y & 0xFFFF)) = r[t];
      } else if (op >= I_AND && op <= I_MUL) {
        // one value per lane: every operand load is issued before the first
        // is used, then 1-bit operands are taken out of their masks
        const uint32_t y = rlane(bc.y, l), z = rlane(bc.z, l);
        const uint32_t cls = (x >> 16) & 0xFF, w = (x >> 8) & 0xFF;
        const uint32_t ca = (cls >> 2) & 3, cb = (cls >> 4) & 3, cc = cls >> 6;
        uint64_t a[TW], b[TW], c[TW], r[TW];
#pragma unroll
        for (uint32_t t = 0; t < TW; ++t) {
          a[t] = vload(base[t], ca, y >> 16, lane4, lane8);
          b[t] = vload(base[t], cb, z & 0xFFFF, lane4, lane8);
          c[t] = 0;
        }
        if (op == I_MUX) {
#pragma unroll
          for (uint32_t t = 0; t < TW; ++t) c[t] = vload(base[t], cc, z >> 16, lane4, lane8);
        }
#pragma unroll
        for (uint32_t t = 0; t < TW; ++t) {
          a[t] = vbit(ca, a[t], lane);
          b[t] = vbit(cb, b[t], lane);
        }
        if (op == I_MUX) {
#pragma unroll
          for (uint32_t t = 0; t < TW; ++t) c[t] = vbit(cc, c[t], lane);
        }
        alu_tree<TW>(op, a, b, c, r);
        if (w < 64) {
#pragma unroll
          for (uint32_t t = 0; t < TW; ++t) r[t] &= wmask(w);
        }
        const uint32_t cd = cls & 3, dst = y & 0xFFFF;
#pragma unroll
        for (uint32_t t = 0; t < TW; ++t) vstore(base[t], cd, dst, r[t], lane4, lane8, lane);
      } else if (op == K_LDB_BATCH) {
        // loads of 1-bit registers, one lane per load: lane k takes
        // instruction k of the block (its register and mask slot)
        const uint32_t n = (x >> 24) & 0xFF;
        if (lane >= l && lane < l + n) {
          const uint32_t r = bc.w, o = bc.y & 0xFFFF;
          uint64_t m[TW];
#pragma unroll
          for (uint32_t t = 0; t < TW; ++t) m[t] = A.stB[(size_t)cur * A.nB * A.n_tiles + (size_t)r * A.n_tiles + tile[t]];
#pragma unroll
          for (uint32_t t = 0; t < TW; ++t) *reinterpret_cast<uint64_t*>(base[t] + o) = m[t];
        }
        step = n;
      } else if (op >= K_LDREG_B) {
        // a run of same-class register loads inside the current block: the
        // register index (aux) and the slot offset (dst) of each load come
        // straight from the block registers; loads first, then the stores
        const uint32_t n = (x >> 24) & 0xFF;
        uint64_t v[kLeafRun][TW];
#pragma unroll
        for (uint32_t k = 0; k < kLeafRun; ++k) {
          if (k < n) {
            const uint32_t r = (uint32_t)__builtin_amdgcn_readlane((int)bc.w, (int)((i + k) & 63));
#pragma unroll
            for (uint32_t t = 0; t < TW; ++t) {
              if (op == K_LDREG_D) v[k][t] = (stD_cur + (size_t)r * A.n_pad)[inst[t]];
              else if (op == K_LDREG_W) v[k][t] = (stW_cur + (size_t)r * A.n_pad)[inst[t]];
              else v[k][t] = stB_cur[(size_t)r * A.n_tiles + tile[t]];
            }
          }
        }
#pragma unroll
        for (uint32_t k = 0; k < kLeafRun; ++k) {
          if (k < n) {
            const uint32_t o = (uint32_t)__builtin_amdgcn_readlane((int)bc.y, (int)((i + k) & 63)) & 0xFFFF;
#pragma unroll
            for (uint32_t t = 0; t < TW; ++t) {
              if (op == K_LDREG_D) *reinterpret_cast<uint64_t*>(base[t] + o + lane8) = v[k][t];
              else if (op == K_LDREG_W) *reinterpret_cast<uint32_t*>(base[t] + o + lane4) = (uint32_t)v[k][t];
              else *reinterpret_cast<uint64_t*>(base[t] + o) = v[k][t];   // the same mask from every lane
            }
          }
        }
        step = n;
      } else {
        const IWord q = lane_word(bc, l);
        const uint32_t y = q.y, z = q.z, aux = q.w;
        const uint32_t w = (x >> 8) & 0xFF, cls = (x >> 16) & 0xFF;
        const uint32_t cd = cls & 3, ca = (cls >> 2) & 3, cb = (cls >> 4) & 3, cc = (cls >> 6) & 3;
        const uint32_t dst = y & 0xFFFF, oa = y >> 16, ob = z & 0xFFFF, oc = z >> 16;
        if (op == I_LDREG || op == I_LDIN) {
          // a run of up to kLeafRun leaf loads (length in flags): every load is
          // issued before any result is used, so the run costs one memory
          // latency.  A shorter run repeats its last leaf (the same value to
          // the same slot): every unrolled load is then used on every path,
          // where a load left unused on some path would make every later
          // handler wait for all outstanding memory operations.
          const uint32_t n = ((x >> 24) & 0xFF) ? ((x >> 24) & 0xFF) : 1;
          uint64_t val[kLeafRun][TW];
#pragma unroll
          for (uint32_t k = 0; k < kLeafRun; ++k) {
            const IWord qk = instr(i + (k < n ? k : n - 1));
            const uint32_t xk = qk.x, auxk = qk.w;
            const uint32_t cak = (xk >> 18) & 3;
#pragma unroll
            for (uint32_t t = 0; t < TW; ++t) {
              if ((xk & 0xFF) == I_LDREG) {
                val[k][t] = cak == C_B ? stB_cur[(size_t)auxk * A.n_tiles + tile[t]]
                          : cak == C_W ? (uint64_t)stW_cur[(size_t)auxk * A.n_pad + inst[t]]
                                       : stD_cur[(size_t)auxk * A.n_pad + inst[t]];
              } else if (A.in_vals) {
                val[k][t] = (real[t] && cyc >= A.in_first && cyc < A.in_first + A.in_count)
                                ? A.in_vals[((cyc - A.in_first) * A.I + auxk) * A.n_inst + inst[t]] : 0;
              } else {
                val[k][t] = A.keys[(size_t)auxk * A.n_pad + inst[t]];
              }
            }
          }
#pragma unroll
          for (uint32_t k = 0; k < kLeafRun; ++k) {
            const IWord qk = instr(i + (k < n ? k : n - 1));
            const uint32_t xk = qk.x, yk = qk.y;
            const uint32_t wk = (xk >> 8) & 0xFF, cdk = (xk >> 16) & 3, cak = (xk >> 18) & 3;
            const uint32_t dk = yk & 0xFFFF;
#pragma unroll
            for (uint32_t t = 0; t < TW; ++t) {
              if ((xk & 0xFF) == I_LDREG) {
                if (cak == C_B) {
                  if (cdk == C_B) {
                    // the mask is wave-uniform: taken into scalar registers,
                    // and every lane stores the same mask
                    const uint64_t m = ((uint64_t)rlane((uint32_t)(val[k][t] >> 32), 0) << 32) |
                                       rlane((uint32_t)val[k][t], 0);
                    *reinterpret_cast<uint64_t*>(base[t] + dk) = m;
                  } else {
                    lwrite(base[t], cdk, dk, lane, (val[k][t] >> lane) & 1);
                  }
                } else {
                  lwrite(base[t], cdk, dk, lane, val[k][t] & wmask(wk));
                }
              } else {
                if (A.in_vals) {
                  if (live[t] && (cyc < A.in_first || cyc >= A.in_first + A.in_count)) atomicOr(&A.error[1], 1u);
                  lwrite(base[t], cdk, dk, lane, val[k][t] & wmask(wk));
                } else {
                  lwrite(base[t], cdk, dk, lane, hmix(val[k][t] ^ cyc) & wmask(wk));
                }
              }
            }
          }
          step = n;
        } else if (op == I_MEMRD) {
#pragma unroll
          for (uint32_t t = 0; t < TW; ++t) {
            const uint64_t a = lread(base[t], ca, oa, lane);
            const uint64_t depth = mem_depth[aux];
            const uint64_t addr = (depth & (depth - 1)) ? a % depth : (a & (depth - 1));
            lwrite(base[t], cd, dst, lane, A.mem[(mem_off[aux] + addr) * A.n_pad + inst[t]] & wmask(w));
          }
        } else if (op == I_STREG) {
          // cd: class of the register's state array, ca: class of the value
#pragma unroll
          for (uint32_t t = 0; t < TW; ++t) {
            const uint64_t v = lread(base[t], ca, oa, lane) & wmask(w);
            if (cd == C_B) {
              const uint64_t m = __ballot(v & 1);
              if (live[t] && lane == 0) stB_nxt[(size_t)aux * A.n_tiles + tile[t]] = m;
            } else if (cd == C_W) {
              if (live[t]) stW_nxt[(size_t)aux * A.n_pad + inst[t]] = (uint32_t)v;
            } else {
              if (live[t]) stD_nxt[(size_t)aux * A.n_pad + inst[t]] = v;
            }
            if (A.digest) dacc[t] += hmix((uint64_t)(ob | (oc << 16)) ^ hmix(v));
          }
        } else if (op == I_STOUT) {
#pragma unroll
          for (uint32_t t = 0; t < TW; ++t) {
            const uint64_t v = lread(base[t], ca, oa, lane) & wmask(w);
            if (live[t]) A.outputs[(size_t)aux * A.n_pad + inst[t]] = v;
          }
        } else if (op == I_WPORT) {
#pragma unroll
          for (uint32_t t = 0; t < TW; ++t) {
            const uint64_t en = lread(base[t], ca, oa, lane), a = lread(base[t], cb, ob, lane);
            const uint64_t v = lread(base[t], cc, oc, lane);
            if (live[t] && en) {
              const uint64_t depth = mem_depth[aux];
              const uint64_t addr = (depth & (depth - 1)) ? a % depth : (a & (depth - 1));
              A.mem[(mem_off[aux] + addr) * A.n_pad + inst[t]] = v & wmask(w);
            }
          }
        }
      }
      i += step;
    }
    bc = bn;
  }
  if (A.digest) {
    const uint64_t k = cyc - A.digest_first;
#pragma unroll
    for (uint32_t t = 0; t < TW; ++t)
      if (real[t] && k < A.digest_max)
        atomicAdd((unsigned long long*)&A.digest[k * A.n_inst + inst[t]], (unsigned long long)dacc[t]);
  }
}

__global__ void __launch_bounds__(256) batched_cycle(BatchArgs A) {
  extern __shared__ uint64_t lds[];
  const uint64_t cyc = A.cycle_ptr ? *A.cycle_ptr + A.cycle0 : A.cycle0;
  batched_body<1>(A, blockIdx.x, cyc, reinterpret_cast<char*>(lds));
}

// two tiles (128 instances) per wave
__global__ void __launch_bounds__(256) batched_cycle2(BatchArgs A) {
  extern __shared__ uint64_t lds[];
  const uint64_t cyc = A.cycle_ptr ? *A.cycle_ptr + A.cycle0 : A.cycle0;
  batched_body<2>(A, blockIdx.x, cyc, reinterpret_cast<char*>(lds));
}

// Serving: one launch advances every resident job by one cycle.  Job j owns
// workgroups [wg_start[j], wg_start[j + 1]); a job whose budget for this
// quantum is spent (tick >= ticks[j]) does nothing.  All jobs share the
// launch's LDS size (the largest job's) and 64 threads per workgroup.
__global__ void __launch_bounds__(64) batched_multi(const BatchArgs* __restrict__ jobs,
                                                    const uint32_t* __restrict__ wg_start,
                                                    const uint64_t* __restrict__ cycle_base,
                                                    const uint32_t* __restrict__ ticks, uint32_t n_jobs,
                                                    uint32_t tick) {
  extern __shared__ uint64_t lds[];
  // the job of this workgroup: binary search over the prefix table
  uint32_t lo = 0, hi = n_jobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (wg_start[mid] <= blockIdx.x) lo = mid; else hi = mid;
  }
  const uint32_t j = lo;
  if (tick >= ticks[j]) return;
  const BatchArgs A = jobs[j];
  batched_body<1>(A, blockIdx.x - wg_start[j], cycle_base[j] + tick, reinterpret_cast<char*>(lds));
}

// One instance's column of an instance-minor [rows][pitch] table, gathered
// into a contiguous [rows] vector or scattered back from one, so that a
// readback or write of one instance's registers, outputs or memory is one
// contiguous host copy rather than a strided copy of `rows` tiny rows.
template <typename T>
__global__ __launch_bounds__(256) void column_copy(T* table, uint64_t pitch, uint64_t col, uint64_t rows,
                                                  T* vec, int to_table) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += stride) {
    if (to_table) table[r * pitch + col] = vec[r];
    else vec[r] = table[r * pitch + col];
  }
}

}  // namespace fsim

// ---------------------------------------------------------------- launches
namespace fsim {

hipError_t launch_batched(const BatchArgs& a, uint32_t grid, uint32_t threads, size_t lds_bytes,
                          hipStream_t s) {
  if (a.twave == 2) hipLaunchKernelGGL(batched_cycle2, dim3(grid), dim3(threads), lds_bytes, s, a);
  else hipLaunchKernelGGL(batched_cycle, dim3(grid), dim3(threads), lds_bytes, s, a);
  return hipGetLastError();
}

hipError_t launch_batched_multi(const BatchArgs* jobs, const uint32_t* wg_start, const uint64_t* cycle_base,
                                const uint32_t* ticks, uint32_t n_jobs, uint32_t tick, uint32_t grid,
                                size_t lds_bytes, hipStream_t s) {
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(batched_multi, dim3(grid), dim3(64), lds_bytes, s, jobs, wg_start, cycle_base, ticks,
                     n_jobs, tick);
  return hipGetLastError();
}

hipError_t launch_column_copy(void* table, uint32_t elem, uint64_t pitch, uint64_t col, uint64_t rows,
                              void* vec, bool to_table, hipStream_t s) {
  if (rows == 0) return hipSuccess;
  if ((elem != 4 && elem != 8) || col >= pitch) return hipErrorInvalidValue;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((rows + 255) / 256, 4096);
  if (elem == 8)
    hipLaunchKernelGGL(column_copy<uint64_t>, dim3(grid), dim3(256), 0, s, static_cast<uint64_t*>(table),
                       pitch, col, rows, static_cast<uint64_t*>(vec), (int)to_table);
  else
    hipLaunchKernelGGL(column_copy<uint32_t>, dim3(grid), dim3(256), 0, s, static_cast<uint32_t*>(table),
                       pitch, col, rows, static_cast<uint32_t*>(vec), (int)to_table);
  return hipGetLastError();
}

}  // namespace fsim
