// runtime_internal.h -- objects behind the C-ABI handles, shared by the
// runtime (sims) and the server.  Internal to libfibersim.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fibersim.h"
#include "compiler.h"
#include "kernels.h"

namespace fsim {

// Records the calling thread's error text and returns the code.
int fail(int code, const std::string& msg);
inline int fail(const Status& s) { return fail(s.code, s.msg); }

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::fsim::fail(FSIM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// A device buffer the library owns.
struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { if (p) (void)hipFree(p); }
  hipError_t alloc(size_t bytes) {
    if (p) { (void)hipFree(p); p = nullptr; }
    n = bytes;
    return hipMalloc(&p, bytes ? bytes : 256);
  }
  void release() { if (p) (void)hipFree(p); p = nullptr; n = 0; }
};

}  // namespace fsim

// A context is reference-counted: the caller's handle and every design and
// server made on it each hold one reference, so whatever order the caller
// releases them in, a design or server never outlives its context.
struct fsim_ctx {
  std::atomic<int> refs{1};
  int device = 0;
  hipStream_t stream = nullptr;
  uint32_t n_cus = 0, lds_bytes = 0;
  std::mutex mu;
};

struct fsim_design {
  std::atomic<int> refs{1};
  fsim_ctx* ctx = nullptr;          // null: compiled on the host only
  fsim::Design d;
  struct fsim_design_info info{};
  // plain-form program on the device
  fsim::DevBuf instr, levels, chunks, procs, mem_off, mem_depth, mem_magic, in_width;
  uint32_t slot_words = 0, max_proc_instr = 0, max_lvls = 0, max_chunks = 0;
  bool plain_ok = true;             // false: a process exceeds the plain form's limits
  std::string plain_error;          // why (reported when a plain sim is asked for)
  // batched-form program, encoded on first use
  std::mutex batch_mu;
  bool batch_ready = false;
  fsim::DevBuf b_instr, b_procs, b_consts;
  fsim::DevBuf b_regidx;            // per register: class << 30 | index in its class
};

struct fsim_sim {
  fsim_design* d = nullptr;
  uint32_t n_inst = 1;
  bool batched = false;
  uint32_t n_tiles = 1, n_pad = 64, tpw = 1, twave = 1;
  uint64_t *stB = nullptr, *stD = nullptr;
  uint32_t* stW = nullptr;
  uint32_t G = 1, threads = 256, launch = FSIM_LAUNCH_PERSISTENT, graph_cycles = 64;
  size_t lds_bytes = 0;
  // batched: processes [0, split) run in a launch of their own with
  // wave_bytes_small bytes per wave region (0: one launch for all)
  uint32_t split = 0, wave_bytes_small = 0;
  bool stage_instr = false;
  bool single_wave = false;    // plain form: the flat one-wave kernel
  bool poisoned = false;
  uint64_t cycle = 0, seed = 0;
  uint32_t epoch = 0;
  // device memory: workspace (owned or borrowed) and its carve-up
  fsim::DevBuf own_ws;
  char* ws = nullptr;
  uint64_t *state = nullptr, *outputs = nullptr, *mem = nullptr, *keys = nullptr, *cyc_dev = nullptr;
  uint32_t *flags = nullptr, *error = nullptr;
  // explicit inputs
  fsim::DevBuf in_vals;
  uint64_t in_first = 0, in_count = 0;
  bool explicit_inputs = false;
  // digests
  uint64_t* dig_out = nullptr;
  uint64_t dig_first = 0, dig_max = 0;
  fsim::DevBuf dig_part;
  // staging for one instance's column in the batched layout (readback, writes)
  fsim::DevBuf xfer;
  // phase timestamps
  uint64_t* trace = nullptr;
  uint64_t trace_first = 0, trace_max = 0;
  // graph mode
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  ~fsim_sim() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};


namespace fsim {
int check_inst(fsim_sim* s, uint32_t inst);
BatchArgs batch_args(fsim_sim* s);
uint32_t batch_grid(const fsim_sim* s);
size_t batched_wave_bytes(const Design& D);
int ensure_batched(fsim_design* d);
void design_retain(fsim_design* d);
void design_release(fsim_design* d);
void ctx_retain(fsim_ctx* c);
void ctx_release(fsim_ctx* c);
}  // namespace fsim
