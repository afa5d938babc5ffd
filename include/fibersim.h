/*
 * fibersim.h -- C-ABI of libfibersim, per-cycle bulk-synchronous simulation
 * of a fiber-partitioned RTL netlist on one MI355X (gfx950).
 *
 * The method is Parendi's (Emami, Bourgeat, Larus, ASPLOS 2025):
 *   - Sec. 3.2: the design is a data-dependence graph in which every register
 *     is split into a read-only current value and a write-only next value;
 *     a fiber is the set of nodes that produces one register's next value;
 *     processes are sets of fibers, shared nodes are duplicated, and one
 *     simulated cycle is "compute, barrier, exchange, barrier";
 *   - Sec. 5.1: fibers are found by a reverse crawl from every sink and merged
 *     into processes by a four-stage partitioner (large-array pre-merge,
 *     multi-chip cut, conservative bottom-up merge, forced merge);
 *   - Sec. 5.3: compilation fails on combinational loops and on designs that
 *     exceed the target's capacity; the test driver runs on the device.
 *
 * Conventions for every call:
 *   - return value 0 (FSIM_OK) or a negative FSIM_E_* status; nothing throws
 *     across the ABI and nothing aborts.  fsim_last_error() describes the last
 *     failure of the calling thread.
 *   - Host pointers are borrowed for the duration of the call and copied.
 *     Device pointers (fsim_sim_create's workspace, fsim_enable_digest's
 *     buffer) are borrowed for the lifetime of the object; the caller keeps
 *     them alive (e.g. as torch tensors) and frees them afterwards.
 *   - Handles are opaque; the caller destroys what it creates.  A design is
 *     reference counted: sims and servers keep it alive after
 *     fsim_design_free().
 *   - Values cross the ABI as one uint64_t per register / output / memory
 *     word, masked to the declared width.
 *   - A device error poisons the sim: later calls on it return FSIM_E_STATE.
 *   - One sim must not be used by two host threads at once; a server is
 *     thread-safe.
 */
#ifndef FIBERSIM_H
#define FIBERSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ----------------------------------------------------------------- status */
#define FSIM_OK              0
#define FSIM_E_ARG          -1   /* bad argument, call-order or size error    */
#define FSIM_E_NETLIST      -2   /* bad opcode arity, width 0, index range    */
#define FSIM_E_COMB_LOOP    -3   /* combinational cycle (Sec. 5.3)            */
#define FSIM_E_UNSUPPORTED  -4   /* width > 64, unknown opcode                */
#define FSIM_E_CAPACITY     -5   /* LDS / HBM budget exceeded (Sec. 5.3)      */
#define FSIM_E_DEVICE       -6   /* HIP runtime or kernel error               */
#define FSIM_E_STATE        -7   /* poisoned sim, or object in the wrong state*/
#define FSIM_E_BUSY         -8   /* server queue full                         */
#define FSIM_E_INTERNAL     -9   /* a self-check of the compiler failed       */
                                 /* (environment FSIM_CHECK_UNITS=1)          */

/* Text of the calling thread's last failure; valid until its next call. */
const char* fsim_last_error(void);

/* --------------------------------------------------------------- netlist
 * Node opcodes (a file format: the numbering is fixed).  Operands are the
 * values of other nodes, zero-extended to 64 bits; every result is masked to
 * the node width w (1..64).  Shift amounts >= 64 give 0.  EQ/LT are unsigned
 * and give 0 or 1.  MUX(sel, a, b) = sel != 0 ? a : b.  Leaves read the
 * current register value (REG, imm = register), an input port (INPUT,
 * imm = port), a constant (CONST, imm = value); MEMRD (imm = memory,
 * arg0 = address) reads the memory as it was at the start of the cycle, at
 * address mod depth.  */
enum {
  FSIM_OP_CONST = 0, FSIM_OP_INPUT = 1, FSIM_OP_REG = 2, FSIM_OP_MEMRD = 3,
  FSIM_OP_AND = 4, FSIM_OP_OR = 5, FSIM_OP_XOR = 6, FSIM_OP_NOT = 7,
  FSIM_OP_ADD = 8, FSIM_OP_SUB = 9, FSIM_OP_MUX = 10, FSIM_OP_SHL = 11,
  FSIM_OP_SHR = 12, FSIM_OP_EQ = 13, FSIM_OP_LT = 14, FSIM_OP_MUL = 15
};
#define FSIM_NONE 0xFFFFFFFFu

/* A flattened word-level netlist (the data-dependence graph of Sec. 3.2),
 * structure of arrays, all host memory, borrowed for the call.
 *   arg:       [n_nodes][3] node indices, FSIM_NONE where unused.
 *   reg_next:  node whose value becomes the register's next value.
 *   mem_init:  all memories back to back (sum of depths words), or NULL = 0.
 *   write ports (wp_*): node indices of enable, address and data; ports are
 *   applied at the end of the cycle in index order (the highest port wins).
 *   reg_en:    NULL, or per register a node index or FSIM_NONE.  A register
 *   with an enable node takes its next value only in cycles where that node
 *   is non-zero and keeps its value otherwise: a gated or divided clock
 *   (Sec. 5.3) expressed as an enable of the single top clock.  FSIM_NONE
 *   (and a NULL array) means the register follows the top clock. */
typedef struct fsim_netlist {
  uint32_t n_nodes;
  const uint8_t* op;
  const uint8_t* width;
  const uint32_t* arg;
  const uint64_t* imm;
  uint32_t n_regs;
  const uint8_t* reg_width;
  const uint64_t* reg_init;
  const uint32_t* reg_next;
  uint32_t n_inputs;
  const uint8_t* in_width;
  uint32_t n_outputs;
  const uint32_t* out_node;
  uint32_t n_mems;
  const uint32_t* mem_depth;
  const uint8_t* mem_width;
  const uint64_t* mem_init;
  uint32_t n_wports;
  const uint32_t* wp_mem;
  const uint32_t* wp_en;
  const uint32_t* wp_addr;
  const uint32_t* wp_data;
  const uint32_t* reg_en;
} fsim_netlist;

/* Sinks are numbered registers 0..R-1, then write ports, then outputs.
 * sink_to_process[s] names the process (Sec. 3.2 "process", Sec. 5.1) that
 * produces sink s.  Every sink whose cone reads memory m must share a process
 * with m's write ports (the memory commit stays inside one process). */
typedef struct fsim_partition {
  uint32_t n_sinks;
  const uint32_t* sink_to_process;
} fsim_partition;

/* Packing policy when no partition is given. */
#define FSIM_PACK_SLB      0   /* Sec. 5.1 stages 1, 3, 4: bottom-up merge   */
#define FSIM_PACK_FIBERS   1   /* one fiber per process (memory groups kept) */
#define FSIM_PACK_SINGLE   2   /* one process holding every fiber            */
#define FSIM_PACK_HYPER    3   /* hypergraph packing, the alternative of
                                  Sec. 6.6 (fibers as nodes, shared cone
                                  nodes as hyperedges): runs of units in
                                  node order, then moves that lower total
                                  replication under the straggler bound    */

typedef struct fsim_compile_opts {
  uint32_t pack;              /* FSIM_PACK_*                                 */
  uint32_t target_processes;  /* SLB / hypergraph target process count;
                                 0 = device CUs                              */
  uint32_t max_process_nodes; /* capacity of one process (Sec. 5.1 memory
                                 limit); 0 = derived from the LDS size       */
} fsim_compile_opts;

/* Statistics of a compiled design (the fibers of Sec. 3.2, the processes
 * of Sec. 5.1 and the straggler bound of Sec. 4.3).  The struct and the
 * query that fills it share the name fsim_design_info, as POSIX's struct stat
 * and stat() do, so the struct is always written with its tag. */
struct fsim_design_info {
  uint32_t n_nodes, n_live_ops, n_regs, n_sinks, n_processes, max_depth;
  uint64_t sum_fiber_ops;     /* sum over sinks of combinational cone size  */
  uint64_t sum_process_ops;   /* sum over processes of union cone size      */
  double dup_fiber;           /* D_f = sum_fiber_ops / n_live_ops           */
  double dup_process;         /* D_p = sum_process_ops / n_live_ops         */
  uint64_t max_fiber_cost;    /* straggler bound of Sec. 4.3                */
  uint64_t max_process_cost;  /* t_comp proxy: costliest process            */
  uint64_t program_bytes;     /* encoded plain-form program                 */
  uint32_t max_process_levels;
  uint32_t max_process_nodes;
  double compile_seconds;
  uint32_t plain_max_slots;   /* plain form: 4-byte LDS units of live values
                                 of the largest process (a value of at most
                                 32 bits takes one, a wider one two),
                                 allocated by liveness                       */
  uint32_t plain_max_chunks;  /* plain form: chunks of the longest process   */
};

typedef struct fsim_ctx fsim_ctx;
typedef struct fsim_design fsim_design;
typedef struct fsim_sim fsim_sim;

/* Context on one HIP device.  hip_stream is a borrowed hipStream_t (e.g.
 * torch.cuda.current_stream().cuda_stream); NULL = the null stream. */
int fsim_ctx_create(int hip_device, void* hip_stream, fsim_ctx** out);
void fsim_ctx_destroy(fsim_ctx* ctx);
/* Device facts used by the autotuner: CUs, LDS bytes per workgroup,
 * co-resident workgroups of the plain kernel at 256 threads. */
int fsim_ctx_device(fsim_ctx* ctx, uint32_t* n_cus, uint32_t* lds_bytes,
                    uint32_t* max_coresident_wgs);

/* Validate (Sec. 5.3: comb loops rejected), extract fibers by reverse crawl
 * (Sec. 5.1), pack them into processes (Sec. 5.1, or the given partition),
 * levelize and encode, and upload the program.  partition and opts may be
 * NULL.  A process of more than 8191 live nodes does not fit the plain
 * form's operand encoding: the design still loads (the batched form has no
 * such limit), a plain sim of it fails with FSIM_E_CAPACITY, and
 * FSIM_FORM_AUTO then picks the batched form for one instance too. */
int fsim_design_load(fsim_ctx* ctx, const fsim_netlist* nl,
                     const fsim_partition* partition,
                     const fsim_compile_opts* opts, fsim_design** out);
/* Fill *out with the design's statistics: fibers (Sec. 3.2), processes and
 * the duplication they cost (Sec. 3.2: shared nodes are recomputed in every
 * process that needs them; D_f and D_p below), the straggler bound and the
 * costliest process (Sec. 4.3), depth and program size.  FSIM_E_ARG on a
 * NULL argument.  fsim_design_info_get is the same call under another
 * name. */
int fsim_design_info(const fsim_design* d, struct fsim_design_info* out);
int fsim_design_info_get(const fsim_design* d, struct fsim_design_info* out);
/* The process of every sink (n_sinks entries) and each process's node list
 * (CSR: proc_off[n_processes + 1], proc_nodes[proc_off[n_processes]]), as
 * compiled.  Any pointer may be NULL to skip it.  Every register with an
 * enable (reg_en) adds two nodes after the netlist's own, in register order:
 * a REG leaf of that register at n_nodes + 2k and MUX(en, next, leaf) at
 * n_nodes + 2k + 1, k counting enabled registers; info.n_nodes counts them. */
int fsim_design_partition(const fsim_design* d, uint32_t* sink_to_process,
                          uint32_t* proc_off, uint32_t* proc_nodes);
void fsim_design_free(fsim_design* d);
/* Batched-form encoding (done on first use, also on a host-only design): the
 * most live LDS slots any process needs per class (1-bit masks, <= 32-bit,
 * <= 64-bit values), the instruction count, and the LDS bytes one wave of 64
 * instances needs.  Any output pointer may be NULL. */
int fsim_design_batched_info(fsim_design* d, uint32_t* slots_b, uint32_t* slots_w,
                             uint32_t* slots_d, uint64_t* n_instr, uint64_t* wave_lds_bytes);

/* ------------------------------------------------------------ simulation
 * A sim holds n_instances independent copies of the design state.  One
 * instance runs the plain form (lanes of a workgroup evaluate one process's
 * level in parallel); more than one runs the batched form (one lane per
 * instance, Sec. 6.4 "many short tests" / prior art on batch stimulus). */

#define FSIM_LAUNCH_AUTO        0
#define FSIM_LAUNCH_PERSISTENT  1  /* one cooperative launch, grid barrier per cycle */
#define FSIM_LAUNCH_PER_CYCLE   2  /* one launch per cycle (kernel boundary = barrier) */
#define FSIM_LAUNCH_GRAPH       3  /* per-cycle launches captured in a hipGraph */

#define FSIM_FORM_AUTO     0   /* plain for one instance, batched for more   */
#define FSIM_FORM_BATCHED  1   /* one lane per instance, even for one        */
#define FSIM_FORM_PLAIN    2   /* level-parallel workgroups (one instance)   */

/* Where a plain-form workgroup reads its process's instructions from. */
#define FSIM_STAGE_AUTO    0   /* LDS copy when it fits beside the slots     */
#define FSIM_STAGE_LDS     1   /* copied into LDS at launch (error if too big)*/
#define FSIM_STAGE_GLOBAL  2   /* read from global memory, prefetched; LDS
                                  then holds only the value slots, so more
                                  workgroups are resident at once            */

typedef struct fsim_sim_opts {
  uint32_t launch;          /* FSIM_LAUNCH_*; the batched form always ends a
                               cycle at a kernel boundary (PER_CYCLE/GRAPH)  */
  uint32_t wg_threads;      /* plain: threads per workgroup (64..1024);
                               batched: 64 x tiles of 64 instances per
                               workgroup (64..256); 0 = auto                 */
  uint32_t grid;            /* workgroups of the persistent kernel, 0 = auto*/
  uint32_t graph_cycles;    /* cycles per captured graph (GRAPH mode)       */
  uint32_t form;            /* FSIM_FORM_*                                  */
  uint32_t stage;           /* plain form: FSIM_STAGE_*                     */
  uint32_t tiles_per_wave;  /* batched form: tiles of 64 instances one wave
                               interprets the program for (1 or 2; 0 = 1).
                               With 2, fetch, decode and dispatch are shared
                               by 128 instances and each wave needs twice
                               the LDS                                       */
} fsim_sim_opts;

/* Device bytes a sim needs for n_instances (state x2, memories, outputs,
 * stimulus keys, scratch); what fsim_sim_create's workspace must hold.  For
 * one instance it covers both forms. */
int fsim_sim_footprint(const fsim_design* d, uint32_t n_instances, size_t* device_bytes);

/* Create a sim of n_instances independent state copies of the design.
 * workspace: caller-owned device memory of at least fsim_sim_footprint()
 * bytes, 256-byte aligned (e.g. a torch uint8 tensor), or NULL to let the
 * library allocate.  The one workspace region holds every per-sim device
 * buffer (state halves, memories, outputs, stimulus keys, barrier flags),
 * so a caller hands over one allocation instead of a table of buffers.
 * opts may be NULL.  FSIM_E_CAPACITY when the form asked for cannot run the
 * design (LDS, co-residency of a persistent launch), FSIM_E_ARG for bad
 * options or a short or misaligned workspace. */
int fsim_sim_create(fsim_design* d, uint32_t n_instances, void* workspace,
                    size_t workspace_bytes, const fsim_sim_opts* opts, fsim_sim** out);
void fsim_sim_destroy(fsim_sim* s);

/* Device-side stimulus (Sec. 5.3: the test driver runs on the device):
 * instance i, port p, cycle t gets mask(w_p, H(H(H(seed_base + i) ^ p) ^ t)),
 * H = SplitMix64's output function.  This is the default mode. */
int fsim_set_stimulus_seed(fsim_sim* s, uint64_t seed_base);
/* Explicit inputs for cycles [first_cycle, first_cycle + n_cycles):
 * vals[n_cycles][n_inputs][n_instances]; stepping outside that window
 * fails with FSIM_E_ARG. */
int fsim_set_inputs(fsim_sim* s, uint64_t first_cycle, uint32_t n_cycles,
                    const uint64_t* vals);

/* Advance n_cycles simulated cycles, asynchronously on the context's
 * stream.  Each cycle is one bulk-synchronous superstep of Sec. 3.2: every
 * process evaluates its fibers from the current register copy and writes
 * the next one, memory writes commit after every read, and one barrier (the
 * kernel boundary, or the grid barrier of the persistent launch) ends the
 * cycle; the parity swap of the two state halves is the exchange.  Returns
 * FSIM_E_ARG when explicit inputs do not cover the cycles, FSIM_E_DEVICE when
 * a launch fails (the sim is then poisoned), FSIM_E_STATE on a poisoned sim.
 * Errors raised by the device during the cycles are reported by the next
 * fsim_sync. */
int fsim_step(fsim_sim* s, uint64_t n_cycles);
/* Wait for the sim's queued cycles.  FSIM_E_DEVICE (and a poisoned sim) when
 * the device reported a failure: a grid barrier that exceeded its bounded
 * wait, or a runtime error; FSIM_E_ARG when a cycle found no explicit
 * inputs. */
int fsim_sync(fsim_sim* s);
/* Cycles simulated so far (the t of Sec. 3.2's R_t); 0 for a NULL sim. */
uint64_t fsim_cycle(const fsim_sim* s);

/* State access, the "read register and output state" of the problem
 * statement: the current register copy R_t of Sec. 3.2, the outputs of the
 * last simulated cycle, and the arrays (the memories of Sec. 5.1 stage 1)
 * as they stand after that cycle's writes.  Each call synchronises first
 * and returns what fsim_sync would on a device error; FSIM_E_ARG for an
 * instance or memory out of range or a NULL buffer.  Writes mask every value
 * to its declared width.  out/in hold n_regs, n_outputs or the memory's
 * depth values, one uint64_t each, caller-owned host memory.
 * In the batched form one instance's values are gathered (or scattered) on
 * the device through a staging buffer that the sim allocates on first use,
 * sized for the largest column read so far, and frees with the sim. */
int fsim_read_regs(fsim_sim* s, uint32_t inst, uint64_t* out);
/* fsim_read_regs for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same result, but a batched instance's column is gathered into a
 * static device array of 8 MiB that the library holds on every GPU it runs
 * on until the process ends, so the call makes no allocation (fsim_read_regs
 * allocates its staging buffer on first use).  FSIM_E_CAPACITY when the
 * design has more than 1,048,576 registers (use fsim_read_regs then).  The
 * array is shared by every call on one GPU: calls that overlap on the same
 * GPU (from two host threads) race on it. */
int fsim_read_regs_noalloc(fsim_sim* s, uint32_t inst, uint64_t* out);
int fsim_write_regs(fsim_sim* s, uint32_t inst, const uint64_t* in);
int fsim_read_outputs(fsim_sim* s, uint32_t inst, uint64_t* out);
int fsim_read_mem(fsim_sim* s, uint32_t inst, uint32_t mem, uint64_t* out);
int fsim_write_mem(fsim_sim* s, uint32_t inst, uint32_t mem, const uint64_t* in);
/* Set the cycle counter (restoring a checkpoint: regs + mems + cycle). */
int fsim_set_cycle(fsim_sim* s, uint64_t cycle);

/* Verification digests (not part of the paper's method; an order-free
 * summary of R_{t+1} of Sec. 3.2, so that a run can be compared with the
 * oracle every cycle without reading the state back): after every
 * simulated cycle the device adds, per instance, D = sum_r H(r ^ H(R[r]))
 * mod 2^64, H = SplitMix64's output function, into
 * dev_out[(cycle - first) * n_instances + inst], where first is the cycle
 * at which digests were enabled.  dev_out is caller device memory of
 * max_cycles * n_instances uint64, zeroed by this call; NULL disables. */
int fsim_enable_digest(fsim_sim* s, uint64_t* dev_out, uint64_t max_cycles);

/* Phase timestamps, for the per-cycle time breakdown of Parendi Sec. 4
 * (Eq. sim_rate: t_sync + t_comm + t_comp).  For every simulated cycle from
 * the current one and every workgroup, the device writes the 100 MHz
 * realtime counter to dev_out[(k * workgroups + wg) * stride + j]: j = 0 at
 * the cycle start, j = L + 1 after level L of the process, j = stride - 2
 * after the memory commit, j = stride - 1 after the grid barrier.  dev_out
 * is caller device memory of max_cycles * workgroups * stride uint64; the
 * stride is returned.  NULL disables. */
int fsim_enable_trace(fsim_sim* s, uint64_t* dev_out, uint64_t max_cycles, uint32_t* stride);
/* Launch shape chosen for the sim: workgroups, threads per workgroup,
 * launch mode, and whether the process instructions are staged in LDS. */
int fsim_sim_layout(const fsim_sim* s, uint32_t* workgroups, uint32_t* threads,
                    uint32_t* launch, uint32_t* staged);

/* ---------------------------------------------------------------- serving
 * A request loop with continuous batching (the many-short-tests scenario of
 * Sec. 6.4 sharing one GPU).  Jobs (design, instances, cycle budget, stimulus
 * seed) are admitted while their device footprint (fsim_sim_footprint) fits
 * the HBM budget -- first fit in arrival order, a long-blocked head job stops
 * later ones from overtaking it -- keep their state resident, and advance
 * together: each tick is one launch in which every resident job simulates one
 * cycle (batched form).  Every quantum_cycles cycles finished jobs retire
 * (final registers and outputs copied to host memory, device memory freed)
 * and queued jobs are admitted.  A job's results do not depend on the other
 * jobs in the mix.  ctx = NULL gives a host-only executor that advances cycle
 * counters without simulating (for testing the scheduling logic); it keeps
 * no results.  All server calls are thread-safe. */
typedef struct fsim_server fsim_server;

#define FSIM_JOB_QUEUED     0
#define FSIM_JOB_RUNNING    1
#define FSIM_JOB_DONE       2
#define FSIM_JOB_CANCELLED  3
#define FSIM_JOB_FAILED     4

typedef struct fsim_server_opts {
  uint32_t quantum_cycles;  /* cycles between retire/admit points (256)     */
  uint32_t max_jobs;        /* resident jobs at once (64)                   */
  uint32_t max_queue;       /* queued jobs before FSIM_E_BUSY (4096)        */
  uint32_t host_cycle_ns;   /* host-only executor: wall time per simulated
                               cycle of a quantum (1000)                    */
} fsim_server_opts;

typedef struct fsim_job_status {
  int32_t state;            /* FSIM_JOB_*                                    */
  uint32_t n_instances;
  uint64_t cycles_done, n_cycles;
  uint64_t device_bytes;    /* footprint counted against the budget          */
  double t_submit, t_start, t_done;   /* seconds since server creation; -1 = not yet */
} fsim_job_status;

typedef struct fsim_server_stats {
  uint64_t submitted, completed, cancelled, rejected, failed, running, queued;
  uint64_t quanta;
  uint64_t instance_cycles; /* simulated cycles x instances executed         */
  double busy_seconds;      /* wall time of quanta with device work          */
  double elapsed_seconds;   /* since creation                                */
  uint64_t hbm_used, hbm_budget;
} fsim_server_stats;

int fsim_server_create(fsim_ctx* ctx, size_t hbm_budget, const fsim_server_opts* opts,
                       fsim_server** out);
/* Non-blocking.  FSIM_E_CAPACITY if the job can never fit the budget,
 * FSIM_E_BUSY if the queue is full.  The design stays referenced until the
 * job is released. */
int fsim_server_submit(fsim_server* s, fsim_design* d, uint32_t n_instances, uint64_t n_cycles,
                       uint64_t seed_base, uint64_t* job_id);
int fsim_server_poll(fsim_server* s, uint64_t job_id, fsim_job_status* st);
/* Blocks until the job is done, cancelled or failed; timeout_s < 0 waits
 * forever; FSIM_E_BUSY on timeout. */
int fsim_server_wait(fsim_server* s, uint64_t job_id, double timeout_s);
/* Final registers (n_regs) and outputs (n_outputs) of one instance of a
 * finished job; either pointer may be NULL. */
int fsim_server_result(fsim_server* s, uint64_t job_id, uint32_t inst, uint64_t* regs_out,
                       uint64_t* outputs_out);
/* A queued job is dropped at once, a running one at the next quantum end. */
int fsim_server_cancel(fsim_server* s, uint64_t job_id);
/* Forget a finished job and its stored results. */
int fsim_server_release(fsim_server* s, uint64_t job_id);
int fsim_server_stats_get(fsim_server* s, fsim_server_stats* out);
void fsim_server_destroy(fsim_server* s);

#ifdef __cplusplus
}
#endif
#endif /* FIBERSIM_H */
