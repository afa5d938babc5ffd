// compiler.h -- host-side preparation of a design: validation, fiber
// extraction, packing of fibers into processes, levelization and encoding
// of the device instruction streams.  Internal to libfibersim.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fibersim.h"
#include "isa.h"

namespace fsim {

// A validated private copy of the netlist plus everything derived from it.
struct Design {
  // ---- netlist (copied)
  uint32_t N = 0, R = 0, I = 0, O = 0, M = 0, W = 0;
  std::vector<uint8_t> op, width;
  std::vector<uint32_t> arg;            // [N][3]
  std::vector<uint64_t> imm;
  std::vector<uint8_t> reg_width;
  std::vector<uint64_t> reg_init;
  std::vector<uint32_t> reg_next;
  std::vector<uint8_t> in_width;
  std::vector<uint32_t> out_node;
  std::vector<uint32_t> mem_depth;
  std::vector<uint8_t> mem_width;
  std::vector<uint64_t> mem_init;       // sum(depth) words
  std::vector<uint64_t> mem_off;        // [M + 1]
  std::vector<uint32_t> wp_mem, wp_en, wp_addr, wp_data;

  // ---- analysis
  std::vector<uint32_t> level;          // ASAP level; leaves are 0
  std::vector<uint32_t> cost;           // per node packing cost (A-10 reading)
  uint32_t n_sinks() const { return R + W + O; }

  // ---- partition (processes)
  uint32_t P = 0;
  std::vector<uint32_t> sink_proc;      // [n_sinks]
  std::vector<uint32_t> proc_off;       // [P + 1] CSR into proc_nodes
  std::vector<uint32_t> proc_nodes;     // union of cones, sorted by level then node
  std::vector<uint32_t> psink_off;      // [P + 1] CSR into psinks
  std::vector<uint32_t> psinks;         // sinks of each process, ascending

  // ---- statistics
  uint64_t n_live_ops = 0, sum_fiber_ops = 0, sum_process_ops = 0;
  uint64_t max_fiber_cost = 0, max_process_cost = 0;
  uint32_t max_depth = 0, max_process_levels = 0, max_process_nodes = 0;
  double compile_seconds = 0;

  // ---- encoded plain-form program (one process per workgroup)
  std::vector<PlainProc> plain_procs;   // [P]
  std::vector<uint32_t> plain_levels;   // per process: chunk index where each level starts
  std::vector<uint64_t> plain_chunks;   // chunk words (make_chunk)
  std::vector<uint64_t> plain_instr;    // 64-bit instruction words (plain_op, plain_aux, ...)
  uint32_t plain_max_slots = 0;
  uint32_t plain_max_instr = 0;
  uint32_t plain_max_chunks = 0;
  uint32_t max_plain_lvls = 0;

  // ---- encoded batched-form program (one wave per instance tile)
  std::vector<BatchProc> batch_procs;   // [P]
  std::vector<Instr> batch_instr;
  std::vector<uint64_t> batch_consts;   // per-process constant pools, back to back
  uint32_t batch_slots[3] = {0, 0, 0};  // max live slots per class over procs
  uint32_t batch_wave_bytes = 0;        // LDS bytes of one wave's region (the largest process's need)
  // processes are ordered by their LDS need, ascending: batch_need[i] bytes
  // of one wave's region for process i (a sim may run a prefix of them in a
  // launch of its own, with more waves resident per CU)
  std::vector<uint32_t> batch_need;
  bool batch_encoded = false;
  // internal register numbering of the batched layout: class + index
  std::vector<uint32_t> reg_cls_idx;    // (class << 30) | index
  uint32_t reg_count[3] = {0, 0, 0};
};

// Status + message helpers shared by the library's host code.
struct Status {
  int code = FSIM_OK;
  std::string msg;
  bool ok() const { return code == FSIM_OK; }
  static Status err(int c, std::string m) { return Status{c, std::move(m)}; }
};

Status copy_and_validate(const fsim_netlist* nl, Design& d);
Status partition_design(Design& d, const fsim_partition* part,
                        const fsim_compile_opts& opts, uint32_t default_target,
                        uint32_t default_max_nodes);
Status encode_plain(Design& d, uint32_t max_slots);
Status encode_batched(Design& d, uint32_t max_slots_per_class[3]);

}  // namespace fsim
