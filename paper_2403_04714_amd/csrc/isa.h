// isa.h -- the device instruction format shared by the host encoder and the
// HIP kernels of libfibersim.  One instruction is 16 bytes.
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

// Plain form: per process, a constant prologue (run once per launch), then
// levels 0..n_lvls-1 (leaf loads, operator levels, the store level).  The
// instructions of a level are cut into chunks: a chunk of operators (I_ALU)
// holds up to 64 instructions of any opcodes, one per lane, whose operands
// are all read before any lane computes; leaf-load and store chunks hold up
// to 256 instructions of one opcode, four per lane, all issued before the
// first is used; memory reads come in chunks of up to 64.  A chunk is one
// u32: start (16 bits, relative to the first level instruction) |
// (count - 1) << 16 (8 bits) | opcode << 24.  After the levels comes the
// write-port commit, run in order by one thread after every read of the
// cycle.
struct PlainProc {
  uint32_t lvl_off;    // index into the level table: n_lvls + 1 chunk indices
  uint32_t n_lvls;
  uint32_t const_off;  // prologue instructions
  uint32_t n_consts;
  uint32_t instr_off;  // first level instruction
  uint32_t n_instr;    // level instructions; the commit follows them
  uint32_t chunk_off;  // first chunk
  uint32_t n_chunks;
  uint32_t n_wp;       // commit instructions
  uint32_t n_slots;    // u64 LDS slots used
  uint32_t pad[2];
};
static_assert(sizeof(PlainProc) == 48, "PlainProc must be 48 bytes");

inline uint32_t make_chunk(uint32_t start, uint32_t count, uint32_t op) {
  return start | ((count - 1) << 16) | (op << 24);
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
enum : uint8_t {
  K_MASK_AND = 24, K_MASK_OR = 25, K_MASK_XOR = 26, K_MASK_NOT = 27,
  K_MASK_EQ = 28, K_MASK_LT = 29, K_MASK_MUX = 30,
  // a run of register loads of one class whose slot class and width match
  // the register's (run length in flags, never crossing a 64-instruction
  // block of the process's stream)
  K_LDREG_B = 40, K_LDREG_W = 41, K_LDREG_D = 42
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
