// isa.h -- the device instruction formats shared by the host encoder and the
// HIP kernels of libfibersim: 8-byte words in the plain form, 16-byte
// instructions in the batched form.
//
// A process (a set of fibers, Parendi Sec. 3.2) is encoded as a straight-line,
// call-free stream (Sec. 5.2 "aggressive inline": the device program has no
// calls).  Combinational operators keep the netlist's opcode numbers; the
// stream adds leaf loads, sink stores and the memory write-port commit.
#pragma once
#include <cstdint>

namespace fsim {

enum : uint8_t {
  I_MEMRD = 3,
  I_AND = 4, I_OR = 5, I_XOR = 6, I_NOT = 7, I_ADD = 8, I_SUB = 9, I_MUX = 10,
  I_SHL = 11, I_SHR = 12, I_EQ = 13, I_LT = 14, I_MUL = 15,
  I_LDREG = 16,    // dst <- current value of register aux
  I_LDIN = 17,     // dst <- input port aux of this cycle
  I_LDCONST = 18,  // dst <- consts[aux]
  I_STREG = 19,    // next value of register aux <- a (masked to w)
  I_STOUT = 20,    // output aux <- a
  I_WPORT = 21,    // if a != 0: mem[aux][b mod depth] <- c (port order)
  I_NUM = 22,
  I_ALU = 23       // plain-form chunk of operators of mixed opcodes (AND .. MUL)
};

// Slot classes of the batched form: 1-bit values are 64-lane ballot masks,
// narrow values one u32 per lane, wide values one u64 per lane; class K is an
// operand read from the process's constant pool (wave-uniform).
enum : uint8_t { C_B = 0, C_W = 1, C_D = 2, C_K = 3 };
inline uint8_t class_of_width(uint32_t w) { return w == 1 ? C_B : (w <= 32 ? C_W : C_D); }

struct Instr {
  uint8_t op;     // I_*
  uint8_t w;      // result width 1..64 (STREG: register width; WPORT: memory width)
  uint8_t cls;    // batched: class of dst | a << 2 | b << 4 | c << 6
  uint8_t flags;
  uint16_t dst, a, b, c;   // slot indices
  uint32_t aux;            // register / port / output / memory / constant index
};
static_assert(sizeof(Instr) == 16, "Instr must be 16 bytes");

// Plain form: per process, a constant prologue (run once per launch: pairs
// of a destination word and the constant's value), then
// levels 0..n_lvls-1 (leaf loads, operator levels, the store level).  The
// instructions of a level are cut into chunks: a chunk of operators (I_ALU)
// holds up to 64 instructions of any opcodes, one per lane, whose operands
// are all read before any lane computes; leaf-load and store chunks hold up
// to 256 instructions of one opcode, four per lane, all issued before the
// first is used; memory reads come in chunks of up to 64.  After the levels
// comes the write-port commit, run in order by one thread after every read
// of the cycle.  Chunks [0, c_ops) are the leaf level, [c_ops, c_st) the
// operator levels (operator and memory-read chunks, and register and output
// stores written out early, all of them at most 64 instructions, one per
// lane) and [c_st, n_chunks) the final store level.
struct PlainProc {
  uint32_t lvl_off;    // index into the level table: n_lvls + 1 chunk indices
  uint32_t n_lvls;
  uint32_t const_off;  // prologue: n_consts pairs (destination word, value)
  uint32_t n_consts;
  uint32_t instr_off;  // first level instruction
  uint32_t n_instr;    // level instructions; the commit follows them
  uint32_t chunk_off;  // first chunk
  uint32_t n_chunks;
  uint32_t n_wp;       // commit instructions
  uint32_t n_slots;    // u64 LDS slots used
  uint32_t c_ops;      // first chunk of the operator levels
  uint32_t c_st;       // first chunk of the store level
  uint32_t n_leaf;     // leaf-load instructions: level instructions [0, n_leaf)
  uint32_t st_first;   // final-store instructions: level instructions [st_first, n_instr)
};
static_assert(sizeof(PlainProc) == 56, "PlainProc must be 56 bytes");

// A plain-form instruction is one 64-bit word.  Values live in LDS in
// 4-byte units: a value of at most 32 bits takes one unit (or two, kept
// zero-extended, where a reader needs its upper half), a wider one two (an
// even pair); a field names a unit (12 bits).
//   bits  0..3   opcode & 15 (operators 4..15; other instructions take their
//                kind from the chunk)
//   bits  4..10  64 - width, for width 1..64 (STREG: the register's; LDIN:
//                the smaller of the node's and the port's; WPORT: the
//                memory's), so the width's mask is ~0 >> this field
//   bits 14..25  field 0        bits 26..37  field 1
//   bits 38..49  field 2        bits 50..61  field 3
//   bit  63      the destination in field 0 takes one unit (the sign bit of
//                the high half, so a kernel tests it with one compare)
// Operators: destination, then operands a, b, c in fields 0..3 (an unused
// operand repeats a).  Leaf loads (LDREG, LDIN) and the prologue (LDCONST):
// the destination in field 0 (bit 63 gives its size),
// the register or port index in bits 26..61, and bit 0 set for an input port.
// Stores (STREG, STOUT): the source in field 0, the register or output index
// in bits 26..61, and bit 0 set for an output.  MEMRD: destination and address, the memory
// in bits 38..61.  WPORT: enable, address and data, the memory in bits
// 50..61.
constexpr uint32_t kUnitBits = 12;
// units 0 and 1 (the first 8 bytes of a process's LDS) hold no value: the
// one-wave kernel keeps its barrier abort flag there
constexpr uint32_t kPlainUnitBase = 2;
constexpr uint32_t kMaxPlainUnits = (1u << kUnitBits) - 1;
constexpr uint32_t kMaxWportMems = 1u << 12;
inline uint64_t plain_word(uint32_t op, uint32_t w, uint64_t f0, uint64_t f1, uint64_t f2, uint64_t f3,
                           bool one0 = false) {
  return (op & 15) | (uint64_t)(64u - w) << 4 | f0 << 14 | f1 << 26 | f2 << 38 | f3 << 50 | (uint64_t)one0 << 63;
}
inline uint64_t plain_index(uint32_t w, uint64_t f0, uint64_t index, bool one0 = false) {
  return (uint64_t)(64u - w) << 4 | f0 << 14 | index << 26 | (uint64_t)one0 << 63;
}

// A chunk word: start (16 bits, relative to the first level instruction) |
// (count - 1) << 16 | kind << 24 | the set of opcodes in an operator chunk
// (bit k for opcode k) << 32 | flags << 48: kDenseChunk (an operator chunk
// holding at least kDenseOps of the opcodes AND .. LT and no MUL),
// kDenseLow (the same from kDenseOpsLow opcodes: with few waves per SIMD
// the branch-free tree's shorter latency wins earlier), kOtherKind (any
// chunk but an operator chunk: the chunk word's sign bit).
constexpr uint32_t kDenseChunk = 16, kDenseLow = 32, kOtherKind = 0x8000;
constexpr uint32_t kDenseOps = 7, kDenseOpsLow = 2;
inline uint64_t make_chunk(uint32_t start, uint32_t count, uint32_t kind, uint32_t present = 0, uint32_t flags = 0) {
  return start | ((uint64_t)(count - 1) << 16) | ((uint64_t)kind << 24) | ((uint64_t)present << 32) |
         ((uint64_t)flags << 48);
}
inline uint32_t chunk_capacity(uint32_t op) {
  return (op == I_LDREG || op == I_LDIN || op == I_STREG || op == I_STOUT) ? 256 : 64;
}

// Batched form: per process, one sequential stream evaluated by a wave for
// 64 instances at a time; slots are per class.  After encoding, the opcode
// byte names the handler and every operand is an LDS byte offset within the
// wave's region:
//   [0, 16)           two 1-bit masks: all zeros, all ones
//   [16, kbase)       1-bit value slots (one u64 mask each)
//   [kbase, rbase)    the process's constants (u64 each, staged per wave)
//   [rbase, end)      256-byte pages of per-lane values: a <=32-bit value
//                     takes one (64 x u32), a <=64-bit value two adjacent
//                     ones (64 x u64)
// with the bounds of each process's own needs, so that a wave's region is
// the largest single process's need.
// Operators on per-lane values keep their opcode (I_AND .. I_MUL, with the
// operand classes in cls); operators whose operands and result are all 1-bit
// become whole-mask handlers.
// longest run of leaf loads (other than 1-bit register loads) the batched
// encoder forms and the kernel issues back to back before waiting: longer
// runs hide more memory latency, shorter ones keep fewer values live
constexpr uint32_t kLeafRun = 2;
enum : uint8_t {
  K_MASK_AND = 24, K_MASK_OR = 25, K_MASK_XOR = 26, K_MASK_NOT = 27,
  K_MASK_EQ = 28, K_MASK_LT = 29, K_MASK_MUX = 30,
  // a run of register loads of one class whose slot class and width match
  // the register's (run length in flags, never crossing a 64-instruction
  // block of the process's stream)
  K_LDREG_B = 40, K_LDREG_W = 41, K_LDREG_D = 42,
  // up to 64 loads of 1-bit registers into 1-bit values, starting at a
  // 64-instruction block boundary of the process's stream (count in the
  // first one's flags): one lane per load
  K_LDB_BATCH = 43
};
struct BatchProc {
  uint32_t instr_off;
  uint32_t n_instr;
  uint32_t mask_slots; // 8-byte slots of 1-bit masks
  uint32_t row_pages;  // 256-byte pages of per-lane values (<=32-bit: one, <=64-bit: two)
  uint32_t pad;
  uint32_t const_off;  // constant pool of the process (class K operands)
  uint32_t n_consts;
  uint32_t kbase;      // LDS byte offset of the staged constants
};
static_assert(sizeof(BatchProc) == 32, "BatchProc must be 32 bytes");

}  // namespace fsim
