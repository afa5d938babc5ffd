// serve.cpp -- a request loop with continuous batching of simulation jobs.
//
// Many short, independent tests of one or more designs are the nightly-
// regression scenario of Parendi Sec. 6.4; here they share one GPU.  A job is
// (design, instances, cycle budget, stimulus seed).  Jobs are admitted while
// their device footprint fits the HBM budget (first fit in arrival order; a
// head job blocked for long enough stops later jobs from overtaking it), keep
// their state resident between quanta, and are co-scheduled: each tick is one
// launch in which every resident job advances one cycle, so their work
// overlaps on the device.  At quantum boundaries finished jobs retire (final
// state copied to host, device memory freed) and queued jobs are admitted.
// With no device context the server runs a host-only executor that advances
// cycle counters without simulating, for testing the scheduling logic.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <thread>

#include "runtime_internal.h"

using fsim::fail;

namespace {

struct Job {
  uint64_t id = 0;
  fsim_design* d = nullptr;
  uint32_t n_inst = 1;
  uint64_t n_cycles = 0, seed = 0;
  int state = FSIM_JOB_QUEUED;
  bool cancel = false;
  uint64_t done_cycles = 0;
  size_t footprint = 0;
  double t_submit = 0, t_start = -1, t_done = -1;
  fsim_sim* sim = nullptr;
  uint32_t blocked_quanta = 0;
  // final state, per register class, copied at retirement
  std::vector<uint64_t> fb, fd, fout;
  std::vector<uint32_t> fw;
  uint32_t n_tiles = 0, n_pad = 0;
  std::string error;
};

constexpr uint32_t kAgingQuanta = 8;

}  // namespace

struct fsim_server {
  fsim_ctx* ctx = nullptr;
  size_t budget = 0, used = 0;
  uint32_t K = 256, max_jobs = 64, max_queue = 4096, host_cycle_ns = 1000;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  std::deque<uint64_t> queue;
  std::vector<uint64_t> running;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread th;
  uint64_t quanta = 0, inst_cycles = 0, submitted = 0, completed = 0, cancelled = 0, rejected = 0, failed = 0;
  double busy_s = 0;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  fsim::DevBuf d_jobs, d_wg, d_base, d_ticks;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

// creates the job's sim (batched form, 64-thread workgroups, stimulus seed)
int job_start(fsim_server* S, Job* j) {
  if (!S->ctx) return FSIM_OK;
  fsim_sim_opts o{};
  o.launch = FSIM_LAUNCH_PER_CYCLE;
  o.wg_threads = 64;
  o.form = FSIM_FORM_BATCHED;
  int rc = fsim_sim_create(j->d, j->n_inst, nullptr, 0, &o, &j->sim);
  if (rc) return rc;
  return fsim_set_stimulus_seed(j->sim, j->seed);
}

// copies the final register state and outputs to host memory, frees the sim
int job_retire(fsim_server* S, Job* j, bool keep_results) {
  if (!j->sim) return FSIM_OK;
  fsim_sim* s = j->sim;
  int rc = fsim_sync(s);
  if (!rc && keep_results) {
    const fsim::Design& D = s->d->d;
    const size_t cur = s->cycle & 1, T = s->n_tiles, NP = s->n_pad;
    const size_t nb = (size_t)D.reg_count[0] * T, nw = (size_t)D.reg_count[1] * NP, nd = (size_t)D.reg_count[2] * NP;
    j->fb.resize(nb); j->fw.resize(nw); j->fd.resize(nd); j->fout.resize((size_t)D.O * NP);
    j->n_tiles = (uint32_t)T; j->n_pad = (uint32_t)NP;
    hipError_t e = hipSuccess;
    if (nb && e == hipSuccess) e = hipMemcpy(j->fb.data(), s->stB + cur * nb, nb * 8, hipMemcpyDeviceToHost);
    if (nw && e == hipSuccess) e = hipMemcpy(j->fw.data(), s->stW + cur * nw, nw * 4, hipMemcpyDeviceToHost);
    if (nd && e == hipSuccess) e = hipMemcpy(j->fd.data(), s->stD + cur * nd, nd * 8, hipMemcpyDeviceToHost);
    if (D.O && e == hipSuccess) e = hipMemcpy(j->fout.data(), s->outputs, j->fout.size() * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = fail(FSIM_E_DEVICE, std::string("retire: ") + hipGetErrorString(e));
  }
  fsim_sim_destroy(s);
  j->sim = nullptr;
  (void)S;
  return rc;
}

// first fit in arrival order; a head job blocked for kAgingQuanta quanta
// stops later jobs from overtaking it
void admit(fsim_server* S) {
  bool head_blocked = false;
  for (auto it = S->queue.begin(); it != S->queue.end();) {
    if (S->running.size() >= S->max_jobs) break;
    Job* j = S->jobs[*it].get();
    const bool fits = S->used + j->footprint <= S->budget;
    if (!fits) {
      if (it == S->queue.begin() && ++j->blocked_quanta >= kAgingQuanta) head_blocked = true;
      if (head_blocked) break;
      ++it;
      continue;
    }
    int rc = job_start(S, j);
    if (rc) {
      j->state = FSIM_JOB_FAILED;
      j->error = fsim_last_error();
      j->t_done = S->now();
      S->failed++;
      it = S->queue.erase(it);
      S->done_cv.notify_all();
      continue;
    }
    S->used += j->footprint;
    j->state = FSIM_JOB_RUNNING;
    j->t_start = S->now();
    S->running.push_back(j->id);
    it = S->queue.erase(it);
  }
}

// one quantum: every running job advances min(K, remaining) cycles; one
// launch per tick covers all of them
int run_quantum(fsim_server* S, const std::vector<Job*>& run, const std::vector<uint32_t>& ticks) {
  const size_t n = run.size();
  uint32_t max_ticks = 0;
  for (size_t i = 0; i < n; ++i) max_ticks = std::max(max_ticks, ticks[i]);
  if (max_ticks == 0) return FSIM_OK;
  if (!S->ctx) {              // host-only executor: the quantum only takes time
    const double t0 = S->now();
    std::this_thread::sleep_for(std::chrono::nanoseconds((uint64_t)max_ticks * S->host_cycle_ns));
    S->busy_s += S->now() - t0;
    return FSIM_OK;
  }
  std::vector<fsim::BatchArgs> args(n);
  std::vector<uint32_t> wg(n + 1, 0);
  std::vector<uint64_t> base(n);
  size_t lds = 0;
  for (size_t i = 0; i < n; ++i) {
    fsim_sim* s = run[i]->sim;
    args[i] = fsim::batch_args(s);
    wg[i + 1] = wg[i] + fsim::batch_grid(s);
    base[i] = s->cycle;
    lds = std::max(lds, s->lds_bytes);
  }
  hipStream_t st = S->ctx->stream;
  HIP_TRY(hipSetDevice(S->ctx->device));
  if (S->d_jobs.n < n * sizeof(fsim::BatchArgs)) HIP_TRY(S->d_jobs.alloc(std::max<size_t>(n, 16) * 2 * sizeof(fsim::BatchArgs)));
  if (S->d_wg.n < (n + 1) * 4) HIP_TRY(S->d_wg.alloc((std::max<size_t>(n, 16) * 2 + 1) * 4));
  if (S->d_base.n < n * 8) HIP_TRY(S->d_base.alloc(std::max<size_t>(n, 16) * 2 * 8));
  if (S->d_ticks.n < n * 4) HIP_TRY(S->d_ticks.alloc(std::max<size_t>(n, 16) * 2 * 4));
  HIP_TRY(hipMemcpyAsync(S->d_jobs.p, args.data(), n * sizeof(fsim::BatchArgs), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(S->d_wg.p, wg.data(), (n + 1) * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(S->d_base.p, base.data(), n * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(S->d_ticks.p, ticks.data(), n * 4, hipMemcpyHostToDevice, st));
  const double t0 = S->now();
  for (uint32_t t = 0; t < max_ticks; ++t)
    HIP_TRY(fsim::launch_batched_multi((const fsim::BatchArgs*)S->d_jobs.p, (const uint32_t*)S->d_wg.p,
                                       (const uint64_t*)S->d_base.p, (const uint32_t*)S->d_ticks.p,
                                       (uint32_t)n, t, wg[n], lds, st));
  HIP_TRY(hipStreamSynchronize(st));
  S->busy_s += S->now() - t0;
  for (size_t i = 0; i < n; ++i) run[i]->sim->cycle += ticks[i];
  return FSIM_OK;
}

void scheduler(fsim_server* S) {
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    S->cv.wait(lk, [&] { return S->stop || !S->queue.empty() || !S->running.empty(); });
    if (S->stop) break;
    admit(S);
    if (S->running.empty()) {
      // everything queued is blocked (cannot happen while footprints fit the
      // budget); wait for a change
      S->cv.wait_for(lk, std::chrono::milliseconds(5));
      continue;
    }
    std::vector<Job*> run;
    std::vector<uint32_t> ticks;
    for (uint64_t id : S->running) {
      Job* j = S->jobs[id].get();
      run.push_back(j);
      ticks.push_back(j->cancel ? 0 : (uint32_t)std::min<uint64_t>(S->K, j->n_cycles - j->done_cycles));
    }
    lk.unlock();
    int rc = run_quantum(S, run, ticks);
    std::string err = rc ? fsim_last_error() : "";
    lk.lock();
    S->quanta++;
    const double t = S->now();
    std::vector<uint64_t> still;
    for (size_t i = 0; i < run.size(); ++i) {
      Job* j = run[i];
      int next = FSIM_JOB_RUNNING;
      if (rc) {
        next = FSIM_JOB_FAILED;
        j->error = err;
      } else {
        j->done_cycles += ticks[i];
        S->inst_cycles += (uint64_t)ticks[i] * j->n_inst;
        if (j->cancel) next = FSIM_JOB_CANCELLED;
        else if (j->done_cycles >= j->n_cycles) next = FSIM_JOB_DONE;
      }
      if (next == FSIM_JOB_RUNNING) { still.push_back(j->id); continue; }
      // the job stays "running" to other threads until its results are copied
      lk.unlock();
      int rr = job_retire(S, j, next == FSIM_JOB_DONE);
      std::string rerr = rr ? fsim_last_error() : "";
      lk.lock();
      if (rr && next == FSIM_JOB_DONE) { next = FSIM_JOB_FAILED; j->error = rerr; }
      j->state = next;
      j->t_done = t;
      S->used -= j->footprint;
      if (next == FSIM_JOB_DONE) S->completed++;
      else if (next == FSIM_JOB_CANCELLED) S->cancelled++;
      else S->failed++;
    }
    S->running.swap(still);
    S->done_cv.notify_all();
  }
}

Job* find(fsim_server* S, uint64_t id) {
  auto it = S->jobs.find(id);
  return it == S->jobs.end() ? nullptr : it->second.get();
}

}  // namespace

extern "C" int fsim_server_create(fsim_ctx* ctx, size_t hbm_budget, const fsim_server_opts* opts,
                                  fsim_server** out) {
  if (!out) return fail(FSIM_E_ARG, "out is NULL");
  *out = nullptr;
  if (hbm_budget == 0) return fail(FSIM_E_ARG, "hbm_budget must be > 0");
  auto S = std::make_unique<fsim_server>();
  S->ctx = ctx;
  fsim::ctx_retain(ctx);
  S->budget = hbm_budget;
  if (opts) {
    if (opts->quantum_cycles) S->K = opts->quantum_cycles;
    if (opts->max_jobs) S->max_jobs = opts->max_jobs;
    if (opts->max_queue) S->max_queue = opts->max_queue;
    if (opts->host_cycle_ns) S->host_cycle_ns = opts->host_cycle_ns;
  }
  fsim_server* raw = S.get();
  S->th = std::thread(scheduler, raw);
  *out = S.release();
  return FSIM_OK;
}

extern "C" int fsim_server_submit(fsim_server* S, fsim_design* d, uint32_t n_instances, uint64_t n_cycles,
                                  uint64_t seed_base, uint64_t* job_id) {
  if (!S || !d || !job_id) return fail(FSIM_E_ARG, "NULL argument");
  if (n_instances == 0 || n_cycles == 0) return fail(FSIM_E_ARG, "n_instances and n_cycles must be >= 1");
  if (S->ctx && d->ctx != S->ctx) return fail(FSIM_E_ARG, "design was loaded on another context");
  size_t fp = 0;
  int rc = fsim_sim_footprint(d, n_instances, &fp);
  if (rc) return rc;
  if (S->ctx) {
    // the batched encoding must exist before the footprint is final
    if ((rc = fsim::ensure_batched(d))) return rc;
  }
  std::lock_guard<std::mutex> g(S->mu);
  if (fp > S->budget) {
    S->rejected++;
    return fail(FSIM_E_CAPACITY, "job footprint " + std::to_string(fp) + " bytes exceeds the HBM budget");
  }
  if (S->queue.size() >= S->max_queue) {
    S->rejected++;
    return fail(FSIM_E_BUSY, "server queue is full");
  }
  auto j = std::make_unique<Job>();
  j->id = S->next_id++;
  j->d = d;
  fsim::design_retain(d);
  j->n_inst = n_instances;
  j->n_cycles = n_cycles;
  j->seed = seed_base;
  j->footprint = fp;
  j->t_submit = S->now();
  *job_id = j->id;
  S->queue.push_back(j->id);
  S->jobs[j->id] = std::move(j);
  S->submitted++;
  S->cv.notify_all();
  return FSIM_OK;
}

extern "C" int fsim_server_poll(fsim_server* S, uint64_t job_id, fsim_job_status* st) {
  if (!S || !st) return fail(FSIM_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> g(S->mu);
  Job* j = find(S, job_id);
  if (!j) return fail(FSIM_E_ARG, "no such job");
  st->state = j->state;
  st->cycles_done = j->done_cycles;
  st->n_cycles = j->n_cycles;
  st->n_instances = j->n_inst;
  st->device_bytes = j->footprint;
  st->t_submit = j->t_submit;
  st->t_start = j->t_start;
  st->t_done = j->t_done;
  return FSIM_OK;
}

extern "C" int fsim_server_wait(fsim_server* S, uint64_t job_id, double timeout_s) {
  if (!S) return fail(FSIM_E_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(S->mu);
  Job* j = find(S, job_id);
  if (!j) return fail(FSIM_E_ARG, "no such job");
  auto finished = [&] { return j->state != FSIM_JOB_QUEUED && j->state != FSIM_JOB_RUNNING; };
  if (timeout_s < 0) S->done_cv.wait(lk, finished);
  else if (!S->done_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), finished))
    return fail(FSIM_E_BUSY, "job not finished within the timeout");
  return FSIM_OK;
}

extern "C" int fsim_server_result(fsim_server* S, uint64_t job_id, uint32_t inst, uint64_t* regs_out,
                                  uint64_t* outputs_out) {
  if (!S) return fail(FSIM_E_ARG, "server is NULL");
  std::lock_guard<std::mutex> g(S->mu);
  Job* j = find(S, job_id);
  if (!j) return fail(FSIM_E_ARG, "no such job");
  if (j->state != FSIM_JOB_DONE) return fail(FSIM_E_STATE, "job has not completed");
  if (!S->ctx) return fail(FSIM_E_STATE, "a host-only server keeps no simulation results");
  if (inst >= j->n_inst) return fail(FSIM_E_ARG, "instance out of range");
  const fsim::Design& D = j->d->d;
  if (regs_out) {
    for (uint32_t r = 0; r < D.R; ++r) {
      const uint32_t k = D.reg_cls_idx[r] >> 30, i = D.reg_cls_idx[r] & 0x3FFFFFFF;
      regs_out[r] = k == fsim::C_B ? (j->fb[(size_t)i * j->n_tiles + inst / 64] >> (inst % 64)) & 1
                  : k == fsim::C_W ? j->fw[(size_t)i * j->n_pad + inst]
                                   : j->fd[(size_t)i * j->n_pad + inst];
    }
  }
  if (outputs_out)
    for (uint32_t o = 0; o < D.O; ++o) outputs_out[o] = j->fout[(size_t)o * j->n_pad + inst];
  return FSIM_OK;
}

extern "C" int fsim_server_cancel(fsim_server* S, uint64_t job_id) {
  if (!S) return fail(FSIM_E_ARG, "server is NULL");
  std::lock_guard<std::mutex> g(S->mu);
  Job* j = find(S, job_id);
  if (!j) return fail(FSIM_E_ARG, "no such job");
  if (j->state == FSIM_JOB_QUEUED) {
    S->queue.erase(std::find(S->queue.begin(), S->queue.end(), job_id));
    j->state = FSIM_JOB_CANCELLED;
    j->t_done = S->now();
    S->cancelled++;
    S->done_cv.notify_all();
  } else if (j->state == FSIM_JOB_RUNNING) {
    j->cancel = true;           // retired at the end of the current quantum
  }
  return FSIM_OK;
}

extern "C" int fsim_server_release(fsim_server* S, uint64_t job_id) {
  if (!S) return fail(FSIM_E_ARG, "server is NULL");
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->jobs.find(job_id);
  if (it == S->jobs.end()) return fail(FSIM_E_ARG, "no such job");
  Job* j = it->second.get();
  if (j->state == FSIM_JOB_QUEUED || j->state == FSIM_JOB_RUNNING)
    return fail(FSIM_E_STATE, "job is still queued or running");
  fsim::design_release(j->d);
  S->jobs.erase(it);
  return FSIM_OK;
}

extern "C" int fsim_server_stats_get(fsim_server* S, fsim_server_stats* out) {
  if (!S || !out) return fail(FSIM_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> g(S->mu);
  out->submitted = S->submitted;
  out->completed = S->completed;
  out->cancelled = S->cancelled;
  out->rejected = S->rejected;
  out->failed = S->failed;
  out->running = S->running.size();
  out->queued = S->queue.size();
  out->quanta = S->quanta;
  out->instance_cycles = S->inst_cycles;
  out->busy_seconds = S->busy_s;
  out->elapsed_seconds = S->now();
  out->hbm_used = S->used;
  out->hbm_budget = S->budget;
  return FSIM_OK;
}

extern "C" void fsim_server_destroy(fsim_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  for (auto& kv : S->jobs) {
    Job* j = kv.second.get();
    if (j->sim) fsim_sim_destroy(j->sim);
    fsim::design_release(j->d);
  }
  fsim_ctx* c = S->ctx;
  delete S;
  fsim::ctx_release(c);
}
