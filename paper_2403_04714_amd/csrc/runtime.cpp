// runtime.cpp -- the C-ABI of libfibersim (include/fibersim.h): contexts,
// design loading, sims, stepping, state access and verification digests.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "runtime_internal.h"

using fsim::Design;
using fsim::Status;

namespace fsim {
namespace {
thread_local std::string g_last_error;
}
int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}
}  // namespace fsim

using fsim::fail;
using fsim::DevBuf;
using fsim::align256;
using fsim::batch_args;
using fsim::batch_grid;
using fsim::batched_wave_bytes;
using fsim::ensure_batched;
using fsim::check_inst;

extern "C" const char* fsim_last_error(void) { return fsim::g_last_error.c_str(); }

// ------------------------------------------------------------------ context
extern "C" int fsim_ctx_create(int hip_device, void* hip_stream, fsim_ctx** out) {
  if (!out) return fail(FSIM_E_ARG, "out is NULL");
  *out = nullptr;
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (hip_device < 0 || hip_device >= n) return fail(FSIM_E_ARG, "no such HIP device");
  HIP_TRY(hipSetDevice(hip_device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, hip_device));
  auto* c = new fsim_ctx;
  c->device = hip_device;
  c->stream = (hipStream_t)hip_stream;
  c->n_cus = (uint32_t)prop.multiProcessorCount;
  c->lds_bytes = (uint32_t)prop.sharedMemPerBlock;
  *out = c;
  return FSIM_OK;
}

void fsim::ctx_retain(fsim_ctx* c) { if (c) c->refs++; }
void fsim::ctx_release(fsim_ctx* c) {
  if (c && --c->refs == 0) delete c;
}

extern "C" void fsim_ctx_destroy(fsim_ctx* ctx) { fsim::ctx_release(ctx); }

extern "C" int fsim_ctx_device(fsim_ctx* ctx, uint32_t* n_cus, uint32_t* lds_bytes,
                               uint32_t* max_coresident_wgs) {
  if (!ctx) return fail(FSIM_E_ARG, "ctx is NULL");
  HIP_TRY(hipSetDevice(ctx->device));
  if (n_cus) *n_cus = ctx->n_cus;
  if (lds_bytes) *lds_bytes = ctx->lds_bytes;
  if (max_coresident_wgs) {
    int b = 0;
    HIP_TRY(fsim::plain_occupancy(&b, 256, 0, true, false));
    *max_coresident_wgs = (uint32_t)b * ctx->n_cus;
  }
  return FSIM_OK;
}

// ------------------------------------------------------------------- design
static constexpr uint32_t kDefaultLds = 160 * 1024;
static constexpr uint32_t kStaticLds = 1024;     // abort flag, reduction scratch
// u64 entries of the one-wave kernel's LDS chunk table: every chunk of the
// largest process and the zero entries of the two groups it reads ahead
// order each XCD's range of the plain process table longest first
constexpr bool kLongestFirst = true;

static uint32_t wave_ctab_words(const fsim_design* d) { return d->max_chunks + 2 * fsim::kGroup; }

template <class T>
static int upload(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
  HIP_TRY(b.alloc(v.size() * sizeof(T)));
  if (!v.empty()) HIP_TRY(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return FSIM_OK;
}

extern "C" int fsim_design_load(fsim_ctx* ctx, const fsim_netlist* nl, const fsim_partition* part,
                                const fsim_compile_opts* opts, fsim_design** out) {
  if (!out) return fail(FSIM_E_ARG, "out is NULL");
  *out = nullptr;
  auto t0 = std::chrono::steady_clock::now();
  auto dz = std::make_unique<fsim_design>();
  fsim_compile_opts o{};
  if (opts) o = *opts;
  if (o.pack > FSIM_PACK_HYPER) return fail(FSIM_E_ARG, "unknown packing policy");
  Design& d = dz->d;
  Status s = fsim::copy_and_validate(nl, d);
  if (!s.ok()) return fail(s);
  const uint32_t lds = ctx ? ctx->lds_bytes : kDefaultLds;
  const uint32_t max_slots = (lds - kStaticLds) / 8;
  const uint32_t default_target = ctx ? ctx->n_cus : 256;
  // default node cap of a process: its slots (at most 8 B per node) and its
  // staged instructions (8 B each, about 1.25 per node counting the stores)
  // fit in LDS together with room to spare, so every process can run from
  // LDS-staged instructions
  const uint32_t default_nodes = std::min<uint32_t>((lds - kStaticLds) / 28, 0xFFFE);
  s = fsim::partition_design(d, part, o, default_target, default_nodes);
  if (s.code == FSIM_E_CAPACITY && o.max_process_nodes == 0 && !part) {
    // too few processes for that cap: allow processes whose instructions
    // are read from global memory instead (slots alone must fit) ...
    s = fsim::partition_design(d, part, o, default_target, std::min<uint32_t>(max_slots / 2, 8191));
    // ... or, failing that, processes only the batched form can run
    if (s.code == FSIM_E_CAPACITY)
      s = fsim::partition_design(d, part, o, default_target, 1u << 30);
  }
  if (!s.ok()) return fail(s);
  s = fsim::encode_plain(d, std::min<uint32_t>(2 * max_slots, fsim::kMaxPlainUnits));
  if (s.code == FSIM_E_CAPACITY) {
    // the design still loads: the batched form has no such limit, and a
    // plain sim asked for later reports this error
    dz->plain_ok = false;
    dz->plain_error = "plain form: " + s.msg;
    d.plain_procs.clear(); d.plain_levels.clear(); d.plain_chunks.clear(); d.plain_instr.clear();
    d.plain_max_slots = d.plain_max_instr = d.plain_max_chunks = d.max_plain_lvls = 0;
  } else if (!s.ok()) {
    return fail(s);
  }
  // per-process spans, for the LDS layout
  dz->max_proc_instr = d.plain_max_instr;
  dz->max_lvls = d.max_plain_lvls;
  dz->max_chunks = d.plain_max_chunks;
  // 4-byte units as u64 words, and one unit to spare: a narrow value's
  // operand read takes 8 bytes (the upper half is dropped)
  dz->slot_words = d.plain_max_slots / 2 + 1;
  d.compile_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  struct fsim_design_info& I = dz->info;
  I.n_nodes = d.N;
  I.n_live_ops = (uint32_t)d.n_live_ops;
  I.n_regs = d.R;
  I.n_sinks = d.n_sinks();
  I.n_processes = d.P;
  I.max_depth = d.max_depth;
  I.sum_fiber_ops = d.sum_fiber_ops;
  I.sum_process_ops = d.sum_process_ops;
  I.dup_fiber = d.n_live_ops ? (double)d.sum_fiber_ops / (double)d.n_live_ops : 1.0;
  I.dup_process = d.n_live_ops ? (double)d.sum_process_ops / (double)d.n_live_ops : 1.0;
  I.max_fiber_cost = d.max_fiber_cost;
  I.max_process_cost = d.max_process_cost;
  I.program_bytes = d.plain_instr.size() * 8 + d.plain_levels.size() * 4 + d.plain_chunks.size() * 8 +
                    d.plain_procs.size() * sizeof(fsim::PlainProc);
  I.max_process_levels = d.max_process_levels;
  I.max_process_nodes = d.max_process_nodes;
  I.compile_seconds = d.compile_seconds;
  I.plain_max_slots = d.plain_max_slots;
  I.plain_max_chunks = d.plain_max_chunks;
  if (ctx) {
    dz->ctx = ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    int rc;
    if ((rc = upload(dz->instr, d.plain_instr, st))) return rc;
    if ((rc = upload(dz->levels, d.plain_levels, st))) return rc;
    if ((rc = upload(dz->chunks, d.plain_chunks, st))) return rc;
    {
      // dispatch order: workgroup b runs table entry process_of(b, P), so
      // XCD x runs one contiguous range of the table, in order of
      // dispatch; each range lists its longest processes (most operator
      // chunks) first, so the workgroups that start last have the least to
      // do.  Processes are independent within a cycle: any order is valid.
      std::vector<fsim::PlainProc> tab(d.plain_procs);
      const uint32_t P = (uint32_t)tab.size(), q = P / 8, r = P % 8;
      for (uint32_t x = 0, lo = 0; kLongestFirst && x < 8; ++x) {
        const uint32_t hi = lo + q + (x < r ? 1 : 0);
        std::stable_sort(tab.begin() + lo, tab.begin() + hi, [](const fsim::PlainProc& a, const fsim::PlainProc& b) {
          return a.c_st - a.c_ops > b.c_st - b.c_ops;
        });
        lo = hi;
      }
      if ((rc = upload(dz->procs, tab, st))) return rc;
    }
    std::vector<uint64_t> moff(d.mem_off.begin(), d.mem_off.end() - (d.M ? 1 : 0));
    if (d.M == 0) moff.clear();
    if ((rc = upload(dz->mem_off, moff, st))) return rc;
    if ((rc = upload(dz->mem_depth, d.mem_depth, st))) return rc;
    // per memory, floor((2^64 - 1) / depth): the plain kernel reduces an
    // address mod depth with it, without a division
    std::vector<uint64_t> magic(d.M);
    for (uint32_t m = 0; m < d.M; ++m) magic[m] = ~0ull / d.mem_depth[m];
    if ((rc = upload(dz->mem_magic, magic, st))) return rc;
    if ((rc = upload(dz->in_width, d.in_width, st))) return rc;
    HIP_TRY(hipStreamSynchronize(st));
  }
  fsim::ctx_retain(dz->ctx);        // held until the design is freed
  *out = dz.release();
  return FSIM_OK;
}

extern "C" int fsim_design_info(const fsim_design* d, struct fsim_design_info* out) {
  if (!d || !out) return fail(FSIM_E_ARG, "NULL argument");
  *out = d->info;
  return FSIM_OK;
}

extern "C" int fsim_design_info_get(const fsim_design* d, struct fsim_design_info* out) {
  return fsim_design_info(d, out);
}

extern "C" int fsim_design_partition(const fsim_design* dd, uint32_t* sink_to_process,
                                     uint32_t* proc_off, uint32_t* proc_nodes) {
  if (!dd) return fail(FSIM_E_ARG, "design is NULL");
  const Design& d = dd->d;
  if (sink_to_process) std::copy(d.sink_proc.begin(), d.sink_proc.end(), sink_to_process);
  if (proc_off) std::copy(d.proc_off.begin(), d.proc_off.end(), proc_off);
  if (proc_nodes) std::copy(d.proc_nodes.begin(), d.proc_nodes.end(), proc_nodes);
  return FSIM_OK;
}

void fsim::design_retain(fsim_design* d) { if (d) d->refs++; }
void fsim::design_release(fsim_design* d) {
  if (d && --d->refs == 0) {
    fsim_ctx* c = d->ctx;
    delete d;                       // frees the design's device buffers first
    fsim::ctx_release(c);
  }
}

extern "C" void fsim_design_free(fsim_design* d) { fsim::design_release(d); }

// ---------------------------------------------------------------------- sim
namespace {
struct Layout {
  size_t state, stB, stW, stD, outputs, mem, keys, flags, error, cyc, total;
};

// Plain form: state u64 [2][R]; outputs [O]; memories [words]; keys [I].
// Batched form: state per register class, 1-bit as masks [2][nB][tiles],
// narrow u32 [2][nW][n_pad], wide u64 [2][nD][n_pad]; outputs [O][n_pad];
// memories [words][n_pad]; keys [I][n_pad].
Layout layout(const Design& d, uint32_t n_inst, uint32_t G, bool batched) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  const size_t n_pad = batched ? ((size_t)n_inst + 63) / 64 * 64 : 1;
  const size_t tiles = n_pad / 64;
  if (batched) {
    size_t nb = 0, nw = 0, nd = 0;
    for (uint32_t r = 0; r < d.R; ++r) {
      uint8_t k = fsim::class_of_width(d.reg_width[r]);
      (k == fsim::C_B ? nb : k == fsim::C_W ? nw : nd)++;
    }
    L.stB = take(2 * nb * tiles * 8);
    L.stW = take(2 * nw * n_pad * 4);
    L.stD = take(2 * nd * n_pad * 8);
  } else {
    L.state = take(2ull * d.R * 8);
  }
  L.outputs = take((size_t)d.O * 8 * n_pad);
  L.mem = take(d.mem_off[d.M] * 8 * n_pad);
  L.keys = take((size_t)d.I * 8 * n_pad);
  L.flags = take((size_t)fsim::barrier_words(std::max(G, 1u)) * 4);
  L.error = take(16);
  L.cyc = take(8);
  L.total = off;
  return L;
}
}  // namespace

extern "C" int fsim_sim_footprint(const fsim_design* d, uint32_t n_instances, size_t* bytes) {
  if (!d || !bytes) return fail(FSIM_E_ARG, "NULL argument");
  if (n_instances == 0) return fail(FSIM_E_ARG, "n_instances must be >= 1");
  // one instance may run either form: report the larger of the two layouts
  *bytes = layout(d->d, n_instances, d->d.P, true).total;
  if (n_instances == 1) *bytes = std::max(*bytes, layout(d->d, 1, d->d.P, false).total);
  return FSIM_OK;
}

static int sim_reset_state(fsim_sim* s) {
  const Design& d = s->d->d;
  hipStream_t st = s->d->ctx->stream;
  if (!s->batched) {
    HIP_TRY(hipMemcpyAsync(s->state, d.reg_init.data(), (size_t)d.R * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemsetAsync(s->state + d.R, 0, (size_t)d.R * 8, st));
    if (d.mem_off[d.M])
      HIP_TRY(hipMemcpyAsync(s->mem, d.mem_init.data(), d.mem_off[d.M] * 8, hipMemcpyHostToDevice, st));
    if (d.O) HIP_TRY(hipMemsetAsync(s->outputs, 0, (size_t)d.O * 8, st));
  } else {
    // every instance starts from the netlist's initial state
    const size_t T = s->n_tiles, NP = s->n_pad;
    std::vector<uint64_t> b(2 * (size_t)d.reg_count[0] * T, 0), dd(2 * (size_t)d.reg_count[2] * NP, 0);
    std::vector<uint32_t> w(2 * (size_t)d.reg_count[1] * NP, 0);
    for (uint32_t r = 0; r < d.R; ++r) {
      const uint32_t k = d.reg_cls_idx[r] >> 30, i = d.reg_cls_idx[r] & 0x3FFFFFFF;
      const uint64_t v = d.reg_init[r];
      if (k == fsim::C_B) std::fill(b.begin() + i * T, b.begin() + (i + 1) * T, (v & 1) ? ~0ull : 0ull);
      else if (k == fsim::C_W) std::fill(w.begin() + i * NP, w.begin() + (i + 1) * NP, (uint32_t)v);
      else std::fill(dd.begin() + i * NP, dd.begin() + (i + 1) * NP, v);
    }
    if (!b.empty()) HIP_TRY(hipMemcpyAsync(s->stB, b.data(), b.size() * 8, hipMemcpyHostToDevice, st));
    if (!w.empty()) HIP_TRY(hipMemcpyAsync(s->stW, w.data(), w.size() * 4, hipMemcpyHostToDevice, st));
    if (!dd.empty()) HIP_TRY(hipMemcpyAsync(s->stD, dd.data(), dd.size() * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (d.mem_off[d.M]) {
      std::vector<uint64_t> m(d.mem_off[d.M] * NP);
      for (uint64_t a = 0; a < d.mem_off[d.M]; ++a) std::fill(m.begin() + a * NP, m.begin() + (a + 1) * NP, d.mem_init[a]);
      HIP_TRY(hipMemcpyAsync(s->mem, m.data(), m.size() * 8, hipMemcpyHostToDevice, st));
      HIP_TRY(hipStreamSynchronize(st));
    }
    if (d.O) HIP_TRY(hipMemsetAsync(s->outputs, 0, (size_t)d.O * 8 * NP, st));
  }
  HIP_TRY(hipMemsetAsync(s->flags, 0, (size_t)fsim::barrier_words(s->G) * 4, st));
  HIP_TRY(hipMemsetAsync(s->error, 0, 16, st));
  HIP_TRY(hipMemsetAsync(s->cyc_dev, 0, 8, st));
  HIP_TRY(hipStreamSynchronize(st));
  return FSIM_OK;
}

extern "C" int fsim_set_stimulus_seed(fsim_sim* s, uint64_t seed_base) {
  if (!s) return fail(FSIM_E_ARG, "sim is NULL");
  if (s->poisoned) return fail(FSIM_E_STATE, "sim is poisoned by an earlier device error");
  s->seed = seed_base;
  s->explicit_inputs = false;
  HIP_TRY(fsim::launch_stim_keys(s->keys, seed_base, s->batched ? s->n_pad : 1, s->d->d.I, s->d->ctx->stream));
  return FSIM_OK;
}

int fsim::ensure_batched(fsim_design* d) {
  std::lock_guard<std::mutex> g(d->batch_mu);
  if (d->batch_ready) return FSIM_OK;
  Design& D = d->d;
  if (!D.batch_encoded) {
    Status st = fsim::encode_batched(D, nullptr);
    if (!st.ok()) return fail(st);
  }
  if (!d->ctx) return FSIM_OK;           // host-only design: encoded, not uploaded
  hipStream_t s = d->ctx->stream;
  int rc;
  if ((rc = upload(d->b_instr, D.batch_instr, s))) return rc;
  if ((rc = upload(d->b_procs, D.batch_procs, s))) return rc;
  if ((rc = upload(d->b_consts, D.batch_consts, s))) return rc;
  if ((rc = upload(d->b_regidx, D.reg_cls_idx, s))) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  d->batch_ready = true;
  return FSIM_OK;
}


extern "C" int fsim_design_batched_info(fsim_design* d, uint32_t* slots_b, uint32_t* slots_w,
                                        uint32_t* slots_d, uint64_t* n_instr, uint64_t* wave_lds_bytes) {
  if (!d) return fail(FSIM_E_ARG, "design is NULL");
  int rc = ensure_batched(d);
  if (rc) return rc;
  const Design& D = d->d;
  if (slots_b) *slots_b = D.batch_slots[0];
  if (slots_w) *slots_w = D.batch_slots[1];
  if (slots_d) *slots_d = D.batch_slots[2];
  if (n_instr) *n_instr = D.batch_instr.size();
  if (wave_lds_bytes) *wave_lds_bytes = batched_wave_bytes(D);
  return FSIM_OK;
}

size_t fsim::batched_wave_bytes(const Design& D) {
  return D.batch_wave_bytes;
}

static int sim_create_batched(fsim_sim* s, void* workspace, size_t ws_bytes, const fsim_sim_opts& o) {
  fsim_design* d = s->d;
  HIP_TRY(hipSetDevice(d->ctx->device));
  int rc = ensure_batched(d);
  if (rc) return rc;
  const Design& D = d->d;
  s->G = 1;
  s->n_pad = (s->n_inst + 63) / 64 * 64;
  s->n_tiles = s->n_pad / 64;
  s->tpw = o.wg_threads ? o.wg_threads / 64 : std::min<uint32_t>(s->n_tiles, 4);
  if (s->tpw < 1 || s->tpw > 4 || (o.wg_threads && o.wg_threads % 64))
    return fail(FSIM_E_ARG, "batched form: wg_threads must be 64, 128, 192 or 256");
  s->threads = 64 * s->tpw;
  s->twave = o.tiles_per_wave ? o.tiles_per_wave : 1;
  if (s->twave > 2) return fail(FSIM_E_ARG, "batched form: tiles_per_wave must be 1 or 2");
  s->launch = o.launch ? o.launch : FSIM_LAUNCH_GRAPH;
  if (s->launch == FSIM_LAUNCH_PERSISTENT) s->launch = FSIM_LAUNCH_GRAPH;   // kernel boundary is the barrier
  s->graph_cycles = o.graph_cycles ? o.graph_cycles : 64;
  s->lds_bytes = batched_wave_bytes(D) * s->tpw * s->twave;
  if (s->lds_bytes > d->ctx->lds_bytes)
    return fail(FSIM_E_CAPACITY, "batched form: a process's live values exceed LDS (" +
                                     std::to_string(s->lds_bytes) + " bytes); use more processes");
  // Split the processes (ordered by LDS need) into a prefix of 7/8 of them,
  // launched with the smaller region that prefix needs (more waves resident
  // per CU), and the rest.  Measured over split points from 5/8 to 15/16 on
  // the single-core, 8-tile and 48-tile batched configurations, 7/8 was best
  // or within the run-to-run spread of the best on each; a cost model in
  // whole rounds of resident workgroups chose worse splits.
  if (D.P >= 2) {
    const uint32_t pa = (uint32_t)((uint64_t)D.P * 7 / 8);
    if (pa > 0 && D.batch_need[pa - 1] < D.batch_need[D.P - 1]) {
      s->split = pa;
      s->wave_bytes_small = D.batch_need[pa - 1];
    }
  }
  if (getenv("FSIM_VERBOSE"))
    fprintf(stderr, "fsim sim: batched split %u of %u processes, small region %u bytes\n", s->split, D.P,
            s->wave_bytes_small);
  Layout L = layout(D, s->n_inst, 1, true);
  if (workspace) {
    if (ws_bytes < L.total) return fail(FSIM_E_ARG, "workspace smaller than fsim_sim_footprint()");
    if ((uintptr_t)workspace % 256) return fail(FSIM_E_ARG, "workspace must be 256-byte aligned");
    s->ws = (char*)workspace;
  } else {
    HIP_TRY(s->own_ws.alloc(L.total));
    s->ws = (char*)s->own_ws.p;
  }
  s->stB = (uint64_t*)(s->ws + L.stB);
  s->stW = (uint32_t*)(s->ws + L.stW);
  s->stD = (uint64_t*)(s->ws + L.stD);
  s->outputs = (uint64_t*)(s->ws + L.outputs);
  s->mem = (uint64_t*)(s->ws + L.mem);
  s->keys = (uint64_t*)(s->ws + L.keys);
  s->flags = (uint32_t*)(s->ws + L.flags);
  s->error = (uint32_t*)(s->ws + L.error);
  s->cyc_dev = (uint64_t*)(s->ws + L.cyc);
  if ((rc = sim_reset_state(s))) return rc;
  return fsim_set_stimulus_seed(s, 0);
}

extern "C" int fsim_sim_create(fsim_design* d, uint32_t n_instances, void* workspace, size_t ws_bytes,
                               const fsim_sim_opts* opts, fsim_sim** out) {
  if (!d || !out) return fail(FSIM_E_ARG, "NULL argument");
  *out = nullptr;
  if (!d->ctx) return fail(FSIM_E_STATE, "design was compiled without a device context");
  if (n_instances == 0) return fail(FSIM_E_ARG, "n_instances must be >= 1");
  fsim_sim_opts o{};
  if (opts) o = *opts;
  auto s = std::make_unique<fsim_sim>();
  s->d = d;
  s->n_inst = n_instances;
  s->batched = o.form == FSIM_FORM_BATCHED ||
               (o.form == FSIM_FORM_AUTO && (n_instances > 1 || !d->plain_ok));
  if (!s->batched && !d->plain_ok) return fail(FSIM_E_CAPACITY, d->plain_error);
  if (!s->batched && n_instances != 1) return fail(FSIM_E_ARG, "the plain form runs exactly one instance");
  if (s->batched) {
    int rc = sim_create_batched(s.get(), workspace, ws_bytes, o);
    if (rc) return rc;
    d->refs++;
    *out = s.release();
    return FSIM_OK;
  }
  s->G = d->d.P;
  s->threads = o.wg_threads ? o.wg_threads : 256;
  if (s->threads < 64 || s->threads > 1024 || s->threads % 64)
    return fail(FSIM_E_ARG, "wg_threads must be a multiple of 64 in [64, 1024]");
  if (o.grid && o.grid != s->G)
    return fail(FSIM_E_ARG, "plain form: grid must equal the design's process count");
  s->launch = o.launch ? o.launch : FSIM_LAUNCH_PERSISTENT;
  if (s->launch > FSIM_LAUNCH_GRAPH) return fail(FSIM_E_ARG, "unknown launch mode");
  if (o.form > FSIM_FORM_PLAIN) return fail(FSIM_E_ARG, "unknown form");
  s->graph_cycles = o.graph_cycles ? o.graph_cycles : 64;
  if (s->graph_cycles % 2) s->graph_cycles++;      // keeps the state parity of the base cycle even
  HIP_TRY(hipSetDevice(d->ctx->device));
  // LDS: the value slots; the one-wave kernel adds its chunk table; the
  // process's instructions follow when they are staged (and fit)
  const size_t lds_limit = d->ctx->lds_bytes - kStaticLds;
  if (o.stage > FSIM_STAGE_GLOBAL) return fail(FSIM_E_ARG, "unknown stage mode");
  s->single_wave = s->threads == 64;
  const size_t base = (size_t)d->slot_words * 8 + (s->single_wave ? (size_t)wave_ctab_words(d) * 8 : 0);
  const size_t instr = (size_t)d->max_proc_instr * 8;
  const bool fits = base + instr <= lds_limit;
  if (o.stage == FSIM_STAGE_LDS && !fits)
    return fail(FSIM_E_CAPACITY, "plain form: a process's instructions do not fit in LDS beside its slots");
  s->stage_instr = fits && o.stage != FSIM_STAGE_GLOBAL;
  const size_t lds = base + (s->stage_instr ? instr : 0);
  if (lds > lds_limit) return fail(FSIM_E_CAPACITY, "process does not fit in LDS");
  s->lds_bytes = lds;
  if (s->launch == FSIM_LAUNCH_PERSISTENT) {
    int b = 0;
    HIP_TRY(fsim::plain_occupancy(&b, s->threads, lds, s->stage_instr, s->single_wave));
    if ((uint64_t)b * d->ctx->n_cus < s->G)
      return fail(FSIM_E_CAPACITY, "persistent launch: " + std::to_string(s->G) +
                                       " workgroups are not co-resident; use fewer processes");
  }
  Layout L = layout(d->d, n_instances, s->G, false);
  if (workspace) {
    if (ws_bytes < L.total) return fail(FSIM_E_ARG, "workspace smaller than fsim_sim_footprint()");
    if ((uintptr_t)workspace % 256) return fail(FSIM_E_ARG, "workspace must be 256-byte aligned");
    s->ws = (char*)workspace;
  } else {
    HIP_TRY(s->own_ws.alloc(L.total));
    s->ws = (char*)s->own_ws.p;
  }
  s->state = (uint64_t*)(s->ws + L.state);
  s->outputs = (uint64_t*)(s->ws + L.outputs);
  s->mem = (uint64_t*)(s->ws + L.mem);
  s->keys = (uint64_t*)(s->ws + L.keys);
  s->flags = (uint32_t*)(s->ws + L.flags);
  s->error = (uint32_t*)(s->ws + L.error);
  s->cyc_dev = (uint64_t*)(s->ws + L.cyc);
  int rc = sim_reset_state(s.get());
  if (rc) return rc;
  if ((rc = fsim_set_stimulus_seed(s.get(), 0))) return rc;
  d->refs++;
  *out = s.release();
  return FSIM_OK;
}

extern "C" void fsim_sim_destroy(fsim_sim* s) {
  if (!s) return;
  if (s->d && s->d->ctx) {
    (void)hipSetDevice(s->d->ctx->device);
    (void)hipStreamSynchronize(s->d->ctx->stream);
  }
  fsim_design* d = s->d;
  delete s;
  fsim::design_release(d);
}

extern "C" int fsim_set_inputs(fsim_sim* s, uint64_t first_cycle, uint32_t n_cycles, const uint64_t* vals) {
  if (!s || (!vals && n_cycles)) return fail(FSIM_E_ARG, "NULL argument");
  if (s->poisoned) return fail(FSIM_E_STATE, "sim is poisoned by an earlier device error");
  const Design& d = s->d->d;
  size_t bytes = (size_t)n_cycles * d.I * s->n_inst * 8;
  HIP_TRY(hipStreamSynchronize(s->d->ctx->stream));
  HIP_TRY(s->in_vals.alloc(bytes));
  if (bytes) HIP_TRY(hipMemcpy(s->in_vals.p, vals, bytes, hipMemcpyHostToDevice));
  s->in_first = first_cycle;
  s->in_count = n_cycles;
  s->explicit_inputs = true;
  return FSIM_OK;
}

static fsim::PlainArgs plain_args(fsim_sim* s) {
  const fsim_design* dd = s->d;
  fsim::PlainArgs a{};
  a.code = (const uint64_t*)dd->instr.p;
  a.levels = (const uint32_t*)dd->levels.p;
  a.chunks = (const uint64_t*)dd->chunks.p;
  a.procs = (const fsim::PlainProc*)dd->procs.p;
  a.state = s->state;
  a.outputs = s->outputs;
  a.mem = s->mem;
  a.mem_off = (const uint64_t*)dd->mem_off.p;
  a.mem_depth = (const uint32_t*)dd->mem_depth.p;
  a.mem_magic = (const uint64_t*)dd->mem_magic.p;
  a.in_width = (const uint8_t*)dd->in_width.p;
  a.in_keys = s->keys;
  a.in_vals = s->explicit_inputs ? (const uint64_t*)s->in_vals.p : nullptr;
  a.in_first = s->in_first;
  a.in_count = s->in_count;
  a.digest_part = s->dig_out ? (uint64_t*)s->dig_part.p : nullptr;
  a.digest_first = s->dig_first;
  a.digest_max = s->dig_max;
  a.trace = s->trace;
  a.trace_first = s->trace_first;
  a.trace_max = s->trace_max;
  a.trace_stride = dd->max_lvls + 3;
  a.flags = s->flags;
  a.error = s->error;
  a.R = dd->d.R;
  a.I = dd->d.I;
  a.stage_instr = s->stage_instr ? 1 : 0;
  a.slot_words = dd->slot_words;
  a.ctab_words = wave_ctab_words(dd);
  a.instr_words = dd->max_proc_instr;
  a.single_wave = s->single_wave ? 1 : 0;
  a.cycle_ptr = nullptr;
  // with at most two waves per SIMD (one-wave workgroups over 4 SIMDs per
  // CU) each wave's latency sets the pace, and the branch-free tree pays
  // from two opcodes on; with more waves, vector issue is shared and the
  // tree pays from seven
  const uint64_t waves = (uint64_t)s->G * ((s->threads + 63) / 64);
  a.dense_flag = waves <= 8ull * dd->ctx->n_cus ? fsim::kDenseLow : fsim::kDenseChunk;
  // tests run either threshold on any design: FSIM_TREE=low or high
  if (const char* e = getenv("FSIM_TREE")) a.dense_flag = e[0] == 'l' ? fsim::kDenseLow : fsim::kDenseChunk;
  return a;
}

fsim::BatchArgs fsim::batch_args(fsim_sim* s) {
  const fsim_design* dd = s->d;
  const Design& D = dd->d;
  fsim::BatchArgs a{};
  a.instr = (const fsim::Instr*)dd->b_instr.p;
  a.n_instr_total = D.batch_instr.size();
  a.procs = (const fsim::BatchProc*)dd->b_procs.p;
  a.consts = (const uint64_t*)dd->b_consts.p;
  a.stB = s->stB; a.stW = s->stW; a.stD = s->stD;
  a.outputs = s->outputs;
  a.mem = s->mem;
  a.mem_off = (const uint64_t*)dd->mem_off.p;
  a.mem_depth = (const uint32_t*)dd->mem_depth.p;
  a.keys = s->keys;
  a.in_vals = s->explicit_inputs ? (const uint64_t*)s->in_vals.p : nullptr;
  a.in_first = s->in_first; a.in_count = s->in_count;
  a.digest = s->dig_out;
  a.digest_first = s->dig_first; a.digest_max = s->dig_max;
  a.error = s->error;
  a.cycle_ptr = nullptr;
  a.P = D.P; a.n_tiles = s->n_tiles; a.tpw = s->tpw; a.n_inst = s->n_inst; a.n_pad = s->n_pad; a.I = D.I;
  a.nB = D.reg_count[0]; a.nW = D.reg_count[1]; a.nD = D.reg_count[2];
  a.wave_bytes = D.batch_wave_bytes;
  a.twave = s->twave;
  return a;
}

uint32_t fsim::batch_grid(const fsim_sim* s) {
  const uint32_t per_wg = s->tpw * s->twave;   // tiles per workgroup
  return s->d->d.P * ((s->n_tiles + per_wg - 1) / per_wg);
}

// One batched cycle: the processes whose wave region fits the small size in
// one launch (more waves resident per CU), the rest in a second launch.
// Processes of one cycle are independent, so the order of the launches is
// free; a design whose processes all fall on one side takes one launch.
static hipError_t launch_batched_cycle(fsim_sim* s, const fsim::BatchArgs& ba, hipStream_t st) {
  const Design& D = s->d->d;
  const uint32_t per_wg = s->tpw * s->twave;
  const uint32_t groups = (s->n_tiles + per_wg - 1) / per_wg;
  const uint32_t pa = s->split;
  if (pa == 0 || pa >= D.P) return fsim::launch_batched(ba, batch_grid(s), s->threads, s->lds_bytes, st);
  fsim::BatchArgs a = ba;
  a.P = pa;
  a.wave_bytes = s->wave_bytes_small;
  hipError_t e = fsim::launch_batched(a, pa * groups, s->threads, (size_t)s->wave_bytes_small * per_wg, st);
  if (e != hipSuccess) return e;
  fsim::BatchArgs b = ba;
  b.procs = ba.procs + pa;
  b.P = D.P - pa;
  return fsim::launch_batched(b, (D.P - pa) * groups, s->threads, s->lds_bytes, st);
}

static int build_graph(fsim_sim* s) {
  hipStream_t st = s->d->ctx->stream;
  hipStream_t cap;
  HIP_TRY(hipStreamCreate(&cap));
  fsim::PlainArgs a = plain_args(s);
  a.cycle_ptr = s->cyc_dev;
  a.n_cycles = 1;
  fsim::BatchArgs ba = batch_args(s);
  ba.cycle_ptr = s->cyc_dev;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  for (uint32_t k = 0; e == hipSuccess && k < s->graph_cycles; ++k) {
    if (s->batched) {
      ba.cycle0 = k;
      e = launch_batched_cycle(s, ba, cap);
    } else {
      a.cycle0 = k;
      e = fsim::launch_plain(a, s->G, s->threads, s->lds_bytes, false, cap);
    }
  }
  if (e == hipSuccess) e = fsim::launch_add_u64(s->cyc_dev, s->graph_cycles, cap);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(cap, &g);
  (void)hipStreamDestroy(cap);
  (void)st;
  if (e != hipSuccess || e2 != hipSuccess)
    return fail(FSIM_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
  s->graph = g;
  HIP_TRY(hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0));
  return FSIM_OK;
}

extern "C" int fsim_step(fsim_sim* s, uint64_t n_cycles) {
  if (!s) return fail(FSIM_E_ARG, "sim is NULL");
  if (s->poisoned) return fail(FSIM_E_STATE, "sim is poisoned by an earlier device error");
  if (n_cycles == 0) return FSIM_OK;
  if (s->explicit_inputs &&
      (s->cycle < s->in_first || s->cycle + n_cycles > s->in_first + s->in_count))
    return fail(FSIM_E_ARG, "explicit inputs do not cover the requested cycles");
  fsim_design* dd = s->d;
  hipStream_t st = dd->ctx->stream;
  HIP_TRY(hipSetDevice(dd->ctx->device));
  const uint64_t c_begin = s->cycle;
  uint64_t left = n_cycles;
  fsim::PlainArgs a = plain_args(s);
  if (s->launch == FSIM_LAUNCH_PERSISTENT) {
    while (left) {
      uint32_t n = (uint32_t)std::min<uint64_t>(left, 1u << 20);
      a.cycle0 = s->cycle;
      a.n_cycles = n;
      a.epoch0 = s->epoch;
      hipError_t e = fsim::launch_plain(a, s->G, s->threads, s->lds_bytes, true, st);
      if (e != hipSuccess) { s->poisoned = true; return fail(FSIM_E_DEVICE, std::string("launch: ") + hipGetErrorString(e)); }
      s->epoch += n;
      s->cycle += n;
      left -= n;
    }
  } else {
    // graph mode needs the device-side cycle counter in step with the host's
    bool graph = s->launch == FSIM_LAUNCH_GRAPH && !s->explicit_inputs;
    if (graph && !s->gexec) {
      int rc = build_graph(s);
      if (rc) return rc;
    }
    while (left) {
      if (graph && left >= s->graph_cycles && (s->cycle % 2) == 0) {
        // device counter holds the base cycle of the next graph
        uint64_t c = s->cycle;
        HIP_TRY(hipMemcpyAsync(s->cyc_dev, &c, 8, hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
        while (left >= s->graph_cycles) {
          HIP_TRY(hipGraphLaunch(s->gexec, st));
          s->cycle += s->graph_cycles;
          left -= s->graph_cycles;
        }
        continue;
      }
      hipError_t e;
      if (s->batched) {
        fsim::BatchArgs ba = batch_args(s);
        ba.cycle0 = s->cycle;
        e = launch_batched_cycle(s, ba, st);
      } else {
        a.cycle0 = s->cycle;
        a.n_cycles = 1;
        e = fsim::launch_plain(a, s->G, s->threads, s->lds_bytes, false, st);
      }
      if (e != hipSuccess) { s->poisoned = true; return fail(FSIM_E_DEVICE, std::string("launch: ") + hipGetErrorString(e)); }
      s->cycle += 1;
      left -= 1;
    }
  }
  if (s->dig_out && !s->batched) {
    uint64_t lo = std::max(c_begin, s->dig_first), hi = std::min(s->cycle, s->dig_first + s->dig_max);
    if (hi > lo) {
      uint64_t k0 = lo - s->dig_first;
      HIP_TRY(fsim::launch_digest_reduce((const uint64_t*)s->dig_part.p + k0 * s->G, s->G, hi - lo,
                                         s->dig_out + k0, st));
    }
  }
  return FSIM_OK;
}

extern "C" int fsim_sync(fsim_sim* s) {
  if (!s) return fail(FSIM_E_ARG, "sim is NULL");
  if (s->poisoned) return fail(FSIM_E_STATE, "sim is poisoned by an earlier device error");
  HIP_TRY(hipSetDevice(s->d->ctx->device));
  hipError_t e = hipStreamSynchronize(s->d->ctx->stream);
  if (e != hipSuccess) { s->poisoned = true; return fail(FSIM_E_DEVICE, hipGetErrorString(e)); }
  uint32_t err[2] = {0, 0};
  e = hipMemcpy(err, s->error, 8, hipMemcpyDeviceToHost);
  if (e != hipSuccess) { s->poisoned = true; return fail(FSIM_E_DEVICE, hipGetErrorString(e)); }
  if (err[0]) { s->poisoned = true; return fail(FSIM_E_DEVICE, "grid barrier timed out"); }
  if (err[1]) { s->poisoned = true; return fail(FSIM_E_ARG, "explicit inputs missing for a simulated cycle"); }
  return FSIM_OK;
}

extern "C" uint64_t fsim_cycle(const fsim_sim* s) { return s ? s->cycle : 0; }

int fsim::check_inst(fsim_sim* s, uint32_t inst) {
  if (!s) return fail(FSIM_E_ARG, "sim is NULL");
  if (inst >= s->n_inst) return fail(FSIM_E_ARG, "instance out of range");
  return fsim_sync(s);
}

// batched layout helpers: one instance's column of a [rows][pitch] array,
// gathered or scattered on the device through the sim's staging buffer, so
// the host copy is one contiguous transfer
static int col_xfer(fsim_sim* s, size_t bytes) {
  if (s->xfer.n < bytes) HIP_TRY(s->xfer.alloc(bytes));
  return FSIM_OK;
}
static int col_read(fsim_sim* s, const void* base, size_t elem, size_t pitch_elems, size_t col, size_t rows,
                    void* out) {
  if (!rows) return FSIM_OK;
  int rc = col_xfer(s, rows * elem);
  if (rc) return rc;
  const hipStream_t st = s->d->ctx->stream;
  HIP_TRY(hipSetDevice(s->d->ctx->device));
  HIP_TRY(fsim::launch_column_copy(const_cast<void*>(base), (uint32_t)elem, pitch_elems, col, rows, s->xfer.p,
                                   false, st));
  HIP_TRY(hipMemcpyAsync(out, s->xfer.p, rows * elem, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return FSIM_OK;
}
static int col_write(fsim_sim* s, void* base, size_t elem, size_t pitch_elems, size_t col, size_t rows,
                     const void* in) {
  if (!rows) return FSIM_OK;
  int rc = col_xfer(s, rows * elem);
  if (rc) return rc;
  const hipStream_t st = s->d->ctx->stream;
  HIP_TRY(hipSetDevice(s->d->ctx->device));
  HIP_TRY(hipMemcpyAsync(s->xfer.p, in, rows * elem, hipMemcpyHostToDevice, st));
  HIP_TRY(fsim::launch_column_copy(base, (uint32_t)elem, pitch_elems, col, rows, s->xfer.p, true, st));
  HIP_TRY(hipStreamSynchronize(st));
  return FSIM_OK;
}

// the current-parity register state of one batched instance, per class
struct BatchedRegs {
  std::vector<uint64_t> b, d;
  std::vector<uint32_t> w;
};
static int batched_regs_read(fsim_sim* s, uint32_t inst, BatchedRegs& R) {
  const Design& D = s->d->d;
  const size_t cur = s->cycle & 1, T = s->n_tiles, NP = s->n_pad;
  R.b.assign(D.reg_count[0], 0); R.w.assign(D.reg_count[1], 0); R.d.assign(D.reg_count[2], 0);
  int rc;
  if ((rc = col_read(s, s->stB + cur * D.reg_count[0] * T, 8, T, inst / 64, D.reg_count[0], R.b.data()))) return rc;
  if ((rc = col_read(s, s->stW + cur * D.reg_count[1] * NP, 4, NP, inst, D.reg_count[1], R.w.data()))) return rc;
  if ((rc = col_read(s, s->stD + cur * D.reg_count[2] * NP, 8, NP, inst, D.reg_count[2], R.d.data()))) return rc;
  return FSIM_OK;
}

extern "C" int fsim_read_regs(fsim_sim* s, uint32_t inst, uint64_t* out) {
  int rc = check_inst(s, inst);
  if (rc) return rc;
  if (!out && s->d->d.R) return fail(FSIM_E_ARG, "out is NULL");
  const uint32_t R = s->d->d.R;
  if (!s->batched) {
    HIP_TRY(hipMemcpy(out, s->state + (s->cycle & 1) * R, (size_t)R * 8, hipMemcpyDeviceToHost));
    return FSIM_OK;
  }
  BatchedRegs B;
  if ((rc = batched_regs_read(s, inst, B))) return rc;
  const Design& D = s->d->d;
  for (uint32_t r = 0; r < R; ++r) {
    const uint32_t k = D.reg_cls_idx[r] >> 30, i = D.reg_cls_idx[r] & 0x3FFFFFFF;
    out[r] = k == fsim::C_B ? (B.b[i] >> (inst % 64)) & 1 : k == fsim::C_W ? B.w[i] : B.d[i];
  }
  return FSIM_OK;
}

extern "C" int fsim_write_regs(fsim_sim* s, uint32_t inst, const uint64_t* in) {
  int rc = check_inst(s, inst);
  if (rc) return rc;
  const Design& d = s->d->d;
  if (!in && d.R) return fail(FSIM_E_ARG, "in is NULL");
  std::vector<uint64_t> v(in, in + d.R);
  for (uint32_t r = 0; r < d.R; ++r) v[r] &= ~0ull >> (64 - d.reg_width[r]);
  if (!s->batched) {
    HIP_TRY(hipMemcpy(s->state + (s->cycle & 1) * d.R, v.data(), (size_t)d.R * 8, hipMemcpyHostToDevice));
    return FSIM_OK;
  }
  BatchedRegs B;
  if ((rc = batched_regs_read(s, inst, B))) return rc;
  for (uint32_t r = 0; r < d.R; ++r) {
    const uint32_t k = d.reg_cls_idx[r] >> 30, i = d.reg_cls_idx[r] & 0x3FFFFFFF;
    if (k == fsim::C_B) B.b[i] = (B.b[i] & ~(1ull << (inst % 64))) | ((v[r] & 1) << (inst % 64));
    else if (k == fsim::C_W) B.w[i] = (uint32_t)v[r];
    else B.d[i] = v[r];
  }
  const size_t cur = s->cycle & 1, T = s->n_tiles, NP = s->n_pad;
  if ((rc = col_write(s, s->stB + cur * d.reg_count[0] * T, 8, T, inst / 64, d.reg_count[0], B.b.data()))) return rc;
  if ((rc = col_write(s, s->stW + cur * d.reg_count[1] * NP, 4, NP, inst, d.reg_count[1], B.w.data()))) return rc;
  if ((rc = col_write(s, s->stD + cur * d.reg_count[2] * NP, 8, NP, inst, d.reg_count[2], B.d.data()))) return rc;
  return FSIM_OK;
}

extern "C" int fsim_read_outputs(fsim_sim* s, uint32_t inst, uint64_t* out) {
  int rc = check_inst(s, inst);
  if (rc) return rc;
  const uint32_t O = s->d->d.O;
  if (!out && O) return fail(FSIM_E_ARG, "out is NULL");
  if (!s->batched) {
    if (O) HIP_TRY(hipMemcpy(out, s->outputs, (size_t)O * 8, hipMemcpyDeviceToHost));
    return FSIM_OK;
  }
  return col_read(s, s->outputs, 8, s->n_pad, inst, O, out);
}

extern "C" int fsim_read_mem(fsim_sim* s, uint32_t inst, uint32_t m, uint64_t* out) {
  int rc = check_inst(s, inst);
  if (rc) return rc;
  const Design& d = s->d->d;
  if (m >= d.M) return fail(FSIM_E_ARG, "memory out of range");
  if (!out) return fail(FSIM_E_ARG, "out is NULL");
  if (!s->batched) {
    HIP_TRY(hipMemcpy(out, s->mem + d.mem_off[m], (size_t)d.mem_depth[m] * 8, hipMemcpyDeviceToHost));
    return FSIM_OK;
  }
  return col_read(s, s->mem + d.mem_off[m] * s->n_pad, 8, s->n_pad, inst, d.mem_depth[m], out);
}

extern "C" int fsim_write_mem(fsim_sim* s, uint32_t inst, uint32_t m, const uint64_t* in) {
  int rc = check_inst(s, inst);
  if (rc) return rc;
  const Design& d = s->d->d;
  if (m >= d.M) return fail(FSIM_E_ARG, "memory out of range");
  if (!in) return fail(FSIM_E_ARG, "in is NULL");
  std::vector<uint64_t> v(in, in + d.mem_depth[m]);
  for (auto& x : v) x &= ~0ull >> (64 - d.mem_width[m]);
  if (!s->batched) {
    HIP_TRY(hipMemcpy(s->mem + d.mem_off[m], v.data(), v.size() * 8, hipMemcpyHostToDevice));
    return FSIM_OK;
  }
  return col_write(s, s->mem + d.mem_off[m] * s->n_pad, 8, s->n_pad, inst, d.mem_depth[m], v.data());
}

extern "C" int fsim_set_cycle(fsim_sim* s, uint64_t cycle) {
  int rc = check_inst(s, 0);
  if (rc) return rc;
  const Design& d = s->d->d;
  if ((cycle & 1) != (s->cycle & 1)) {
    const size_t from = s->cycle & 1, to = cycle & 1;
    if (!s->batched) {
      if (d.R) HIP_TRY(hipMemcpy(s->state + to * d.R, s->state + from * d.R, (size_t)d.R * 8, hipMemcpyDeviceToDevice));
    } else {
      const size_t nb = (size_t)d.reg_count[0] * s->n_tiles, nw = (size_t)d.reg_count[1] * s->n_pad,
                   nd = (size_t)d.reg_count[2] * s->n_pad;
      if (nb) HIP_TRY(hipMemcpy(s->stB + to * nb, s->stB + from * nb, nb * 8, hipMemcpyDeviceToDevice));
      if (nw) HIP_TRY(hipMemcpy(s->stW + to * nw, s->stW + from * nw, nw * 4, hipMemcpyDeviceToDevice));
      if (nd) HIP_TRY(hipMemcpy(s->stD + to * nd, s->stD + from * nd, nd * 8, hipMemcpyDeviceToDevice));
    }
  }
  s->cycle = cycle;
  return FSIM_OK;
}

extern "C" int fsim_enable_digest(fsim_sim* s, uint64_t* dev_out, uint64_t max_cycles) {
  if (!s) return fail(FSIM_E_ARG, "sim is NULL");
  if (s->poisoned) return fail(FSIM_E_STATE, "sim is poisoned by an earlier device error");
  hipStream_t st = s->d->ctx->stream;
  HIP_TRY(hipStreamSynchronize(st));
  if (!dev_out || max_cycles == 0) {
    s->dig_out = nullptr;
    s->dig_max = 0;
    return FSIM_OK;
  }
  if (!s->batched) {           // plain: per-workgroup partials, reduced after each step
    HIP_TRY(s->dig_part.alloc((size_t)max_cycles * s->G * 8));
    HIP_TRY(hipMemsetAsync(s->dig_part.p, 0, (size_t)max_cycles * s->G * 8, st));
  }
  HIP_TRY(hipMemsetAsync(dev_out, 0, (size_t)max_cycles * 8 * s->n_inst, st));
  HIP_TRY(hipStreamSynchronize(st));
  s->dig_out = dev_out;
  s->dig_first = s->cycle;
  s->dig_max = max_cycles;
  if (s->gexec) {               // the captured graph has digests baked out
    (void)hipGraphExecDestroy(s->gexec);
    (void)hipGraphDestroy(s->graph);
    s->gexec = nullptr;
    s->graph = nullptr;
  }
  return FSIM_OK;
}

extern "C" int fsim_enable_trace(fsim_sim* s, uint64_t* dev_out, uint64_t max_cycles, uint32_t* stride) {
  if (!s) return fail(FSIM_E_ARG, "sim is NULL");
  if (s->poisoned) return fail(FSIM_E_STATE, "sim is poisoned by an earlier device error");
  HIP_TRY(hipStreamSynchronize(s->d->ctx->stream));
  if (stride) *stride = s->d->max_lvls + 3;
  s->trace = max_cycles ? dev_out : nullptr;
  s->trace_first = s->cycle;
  s->trace_max = dev_out ? max_cycles : 0;
  if (s->gexec) {
    (void)hipGraphExecDestroy(s->gexec);
    (void)hipGraphDestroy(s->graph);
    s->gexec = nullptr;
    s->graph = nullptr;
  }
  return FSIM_OK;
}

extern "C" int fsim_sim_layout(const fsim_sim* s, uint32_t* workgroups, uint32_t* threads,
                               uint32_t* launch, uint32_t* staged) {
  if (!s) return fail(FSIM_E_ARG, "sim is NULL");
  if (workgroups) *workgroups = s->batched ? batch_grid(s) : s->G;
  if (threads) *threads = s->threads;
  if (launch) *launch = s->launch;
  if (staged) *staged = s->stage_instr ? 1 : 0;
  return FSIM_OK;
}
