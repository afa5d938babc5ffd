// compiler.cpp -- host-side preparation of a design (once per design).
//
//   copy_and_validate   operator/width/index checks; Kahn topological order;
//                       combinational loops rejected (Parendi Sec. 5.3);
//                       ASAP levels.
//   partition_design    fibers = reverse crawl from every sink (Sec. 5.1);
//                       stage 1: co-locate every fiber that touches a memory
//                       with that memory's write ports (adapted from the
//                       large-array pre-merge of Sec. 5.1); stages 3-4: the
//                       bottom-up submodular load-balancing merge of Sec. 5.1
//                       with the cost tau(P) = sum of the costs of the union
//                       of the cones (Sec. 4.3).
//   encode_plain        per process: constant prologue, leaf-load level,
//                       operator levels (sorted by opcode so that wavefronts
//                       run one operator at a time), store level, write-port
//                       commit.
//   encode_batched      per process: one sequential stream in depth-first
//                       order with liveness-based slot reuse per class.
#include "compiler.h"

#include <algorithm>
#include <map>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <queue>
#include <set>
#include <unordered_set>

namespace fsim {

// phase timing of the compiler, printed to stderr when FSIM_VERBOSE is set
static void phase(const char* what) {
  static const bool on = getenv("FSIM_VERBOSE") != nullptr;
  static auto t0 = std::chrono::steady_clock::now();
  if (!on) return;
  auto t = std::chrono::steady_clock::now();
  fprintf(stderr, "fsim compile: %-28s %8.3f s\n", what, std::chrono::duration<double>(t - t0).count());
  t0 = t;
}

static inline int arity(uint8_t op) {
  switch (op) {
    case FSIM_OP_CONST: case FSIM_OP_INPUT: case FSIM_OP_REG: return 0;
    case FSIM_OP_MEMRD: case FSIM_OP_NOT: return 1;
    case FSIM_OP_MUX: return 3;
    default: return 2;
  }
}

static std::string fmt(const char* f, unsigned long long a = 0, unsigned long long b = 0, unsigned long long c = 0,
                       unsigned long long e = 0) {
  char buf[256];
  snprintf(buf, sizeof buf, f, a, b, c, e);
  return buf;
}

Status copy_and_validate(const fsim_netlist* nl, Design& d) {
  if (!nl) return Status::err(FSIM_E_ARG, "netlist is NULL");
  auto need = [&](const void* p, uint64_t n, const char* what) -> Status {
    if (n && !p) return Status::err(FSIM_E_ARG, std::string(what) + " is NULL");
    return {};
  };
  Status s;
  if (!(s = need(nl->op, nl->n_nodes, "op")).ok()) return s;
  if (!(s = need(nl->width, nl->n_nodes, "width")).ok()) return s;
  if (!(s = need(nl->arg, nl->n_nodes, "arg")).ok()) return s;
  if (!(s = need(nl->imm, nl->n_nodes, "imm")).ok()) return s;
  if (!(s = need(nl->reg_width, nl->n_regs, "reg_width")).ok()) return s;
  if (!(s = need(nl->reg_init, nl->n_regs, "reg_init")).ok()) return s;
  if (!(s = need(nl->reg_next, nl->n_regs, "reg_next")).ok()) return s;
  if (!(s = need(nl->in_width, nl->n_inputs, "in_width")).ok()) return s;
  if (!(s = need(nl->out_node, nl->n_outputs, "out_node")).ok()) return s;
  if (!(s = need(nl->mem_depth, nl->n_mems, "mem_depth")).ok()) return s;
  if (!(s = need(nl->mem_width, nl->n_mems, "mem_width")).ok()) return s;
  for (auto* p : {nl->wp_mem, nl->wp_en, nl->wp_addr, nl->wp_data})
    if (!(s = need(p, nl->n_wports, "write port array")).ok()) return s;
  if (nl->n_nodes >= 0x7FFFFFFFu) return Status::err(FSIM_E_CAPACITY, "too many nodes");

  d.N = nl->n_nodes; d.R = nl->n_regs; d.I = nl->n_inputs; d.O = nl->n_outputs;
  d.M = nl->n_mems; d.W = nl->n_wports;
  d.op.assign(nl->op, nl->op + d.N);
  d.width.assign(nl->width, nl->width + d.N);
  d.arg.assign(nl->arg, nl->arg + 3ull * d.N);
  d.imm.assign(nl->imm, nl->imm + d.N);
  d.reg_width.assign(nl->reg_width, nl->reg_width + d.R);
  d.reg_init.assign(nl->reg_init, nl->reg_init + d.R);
  d.reg_next.assign(nl->reg_next, nl->reg_next + d.R);
  d.in_width.assign(nl->in_width, nl->in_width + d.I);
  d.out_node.assign(nl->out_node, nl->out_node + d.O);
  d.mem_depth.assign(nl->mem_depth, nl->mem_depth + d.M);
  d.mem_width.assign(nl->mem_width, nl->mem_width + d.M);
  d.wp_mem.assign(nl->wp_mem, nl->wp_mem + d.W);
  d.wp_en.assign(nl->wp_en, nl->wp_en + d.W);
  d.wp_addr.assign(nl->wp_addr, nl->wp_addr + d.W);
  d.wp_data.assign(nl->wp_data, nl->wp_data + d.W);

  for (uint32_t n = 0; n < d.N; ++n) {
    uint8_t op = d.op[n], w = d.width[n];
    if (op > FSIM_OP_MUL) return Status::err(FSIM_E_UNSUPPORTED, fmt("node %llu: unknown opcode %llu", n, op));
    if (w == 0) return Status::err(FSIM_E_NETLIST, fmt("node %llu: width 0", n));
    if (w > 64) return Status::err(FSIM_E_UNSUPPORTED, fmt("node %llu: width %llu > 64", n, w));
    for (int k = 0; k < arity(op); ++k)
      if (d.arg[3ull * n + k] >= d.N)
        return Status::err(FSIM_E_NETLIST, fmt("node %llu: operand %llu out of range", n, k));
    if (op == FSIM_OP_INPUT && d.imm[n] >= d.I) return Status::err(FSIM_E_NETLIST, fmt("node %llu: bad input port", n));
    if (op == FSIM_OP_REG && d.imm[n] >= d.R) return Status::err(FSIM_E_NETLIST, fmt("node %llu: bad register", n));
    if (op == FSIM_OP_MEMRD && d.imm[n] >= d.M) return Status::err(FSIM_E_NETLIST, fmt("node %llu: bad memory", n));
  }
  for (uint32_t r = 0; r < d.R; ++r) {
    if (d.reg_width[r] == 0) return Status::err(FSIM_E_NETLIST, fmt("register %llu: width 0", r));
    if (d.reg_width[r] > 64) return Status::err(FSIM_E_UNSUPPORTED, fmt("register %llu: width > 64", r));
    if (d.reg_next[r] >= d.N) return Status::err(FSIM_E_NETLIST, fmt("register %llu: next node out of range", r));
  }
  for (uint32_t p = 0; p < d.I; ++p)
    if (d.in_width[p] == 0 || d.in_width[p] > 64)
      return Status::err(d.in_width[p] ? FSIM_E_UNSUPPORTED : FSIM_E_NETLIST, fmt("input %llu: bad width", p));
  for (uint32_t o = 0; o < d.O; ++o)
    if (d.out_node[o] >= d.N) return Status::err(FSIM_E_NETLIST, fmt("output %llu: node out of range", o));
  d.mem_off.assign(d.M + 1, 0);
  for (uint32_t m = 0; m < d.M; ++m) {
    if (d.mem_depth[m] == 0) return Status::err(FSIM_E_NETLIST, fmt("memory %llu: depth 0", m));
    if (d.mem_width[m] == 0 || d.mem_width[m] > 64)
      return Status::err(d.mem_width[m] ? FSIM_E_UNSUPPORTED : FSIM_E_NETLIST, fmt("memory %llu: bad width", m));
    d.mem_off[m + 1] = d.mem_off[m] + d.mem_depth[m];
  }
  d.mem_init.assign(d.mem_off[d.M], 0);
  if (nl->mem_init)
    for (uint32_t m = 0; m < d.M; ++m) {
      uint64_t msk = ~0ull >> (64 - d.mem_width[m]);
      for (uint64_t a = d.mem_off[m]; a < d.mem_off[m + 1]; ++a) d.mem_init[a] = nl->mem_init[a] & msk;
    }
  for (uint32_t k = 0; k < d.W; ++k)
    if (d.wp_mem[k] >= d.M || d.wp_en[k] >= d.N || d.wp_addr[k] >= d.N || d.wp_data[k] >= d.N)
      return Status::err(FSIM_E_NETLIST, fmt("write port %llu: index out of range", k));
  for (uint32_t r = 0; r < d.R; ++r) d.reg_init[r] &= ~0ull >> (64 - d.reg_width[r]);

  // Gated and divided clocks (Sec. 5.3) arrive as a per-register enable of
  // the top clock.  Lower each one to next' = MUX(en, next, REG r) at the
  // register's width, so the register keeps its value in cycles where the
  // enable is zero.  The two new nodes go after the netlist's own, in
  // register order; fibers, packing and both kernel forms then see an
  // ordinary netlist.
  if (nl->reg_en) {
    const uint32_t n0 = d.N;
    uint64_t n_en = 0;
    for (uint32_t r = 0; r < d.R; ++r) {
      uint32_t e = nl->reg_en[r];
      if (e == FSIM_NONE) continue;
      if (e >= n0) return Status::err(FSIM_E_NETLIST, fmt("register %llu: enable node out of range", r));
      ++n_en;
    }
    if (n0 + 2 * n_en >= 0x7FFFFFFFull) return Status::err(FSIM_E_CAPACITY, "too many nodes");
    for (uint32_t r = 0; r < d.R; ++r) {
      uint32_t e = nl->reg_en[r];
      if (e == FSIM_NONE) continue;
      const uint32_t leaf = d.N, mux = d.N + 1;
      d.op.push_back(FSIM_OP_REG); d.width.push_back(d.reg_width[r]);
      d.arg.insert(d.arg.end(), {FSIM_NONE, FSIM_NONE, FSIM_NONE}); d.imm.push_back(r);
      d.op.push_back(FSIM_OP_MUX); d.width.push_back(d.reg_width[r]);
      d.arg.insert(d.arg.end(), {e, d.reg_next[r], leaf}); d.imm.push_back(0);
      d.reg_next[r] = mux;
      d.N += 2;
    }
  }

  // Kahn's algorithm; ASAP level = 1 + max operand level, leaves at 0.
  std::vector<uint32_t> indeg(d.N, 0), ucount(d.N + 1, 0);
  for (uint32_t n = 0; n < d.N; ++n)
    for (int k = 0; k < arity(d.op[n]); ++k) { ucount[d.arg[3ull * n + k] + 1]++; indeg[n]++; }
  for (uint32_t n = 0; n < d.N; ++n) ucount[n + 1] += ucount[n];
  std::vector<uint32_t> users(ucount[d.N]), fill(ucount.begin(), ucount.end() - 1);
  for (uint32_t n = 0; n < d.N; ++n)
    for (int k = 0; k < arity(d.op[n]); ++k) users[fill[d.arg[3ull * n + k]]++] = n;
  d.level.assign(d.N, 0);
  std::vector<uint32_t> q;
  q.reserve(d.N);
  for (uint32_t n = 0; n < d.N; ++n) if (!indeg[n]) q.push_back(n);
  for (size_t h = 0; h < q.size(); ++h) {
    uint32_t x = q[h];
    for (uint32_t e = ucount[x]; e < ucount[x + 1]; ++e) {
      uint32_t y = users[e];
      d.level[y] = std::max(d.level[y], d.level[x] + 1);
      if (--indeg[y] == 0) q.push_back(y);
    }
  }
  if (q.size() != d.N) return Status::err(FSIM_E_COMB_LOOP, "combinational loop in the netlist");
  phase("validate + levels");
  d.cost.assign(d.N, 0);
  for (uint32_t n = 0; n < d.N; ++n) {
    uint8_t op = d.op[n];
    if (op == FSIM_OP_CONST) d.cost[n] = 0;
    else if (op == FSIM_OP_REG || op == FSIM_OP_INPUT) d.cost[n] = 1;
    else d.cost[n] = d.width[n] > 32 ? 2 : 1;
  }
  return {};
}

// ------------------------------------------------------------- partition

namespace {

struct UF {
  std::vector<uint32_t> p;
  explicit UF(size_t n) : p(n) { std::iota(p.begin(), p.end(), 0u); }
  uint32_t find(uint32_t x) {
    while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
    return x;
  }
  void unite(uint32_t a, uint32_t b) {
    a = find(a); b = find(b);
    if (a != b) p[std::max(a, b)] = std::min(a, b);
  }
};

uint32_t sink_roots(const Design& d, uint32_t s, uint32_t roots[3]) {
  if (s < d.R) { roots[0] = d.reg_next[s]; return 1; }
  if (s < d.R + d.W) {
    uint32_t k = s - d.R;
    roots[0] = d.wp_en[k]; roots[1] = d.wp_addr[k]; roots[2] = d.wp_data[k];
    return 3;
  }
  roots[0] = d.out_node[s - d.R - d.W];
  return 1;
}

uint64_t set_cost(const Design& d, const std::vector<uint32_t>& v) {
  uint64_t c = 0;
  for (uint32_t n : v) c += d.cost[n];
  return c;
}

// cost and size of the union of two sorted node sets
void union_stats(const Design& d, const std::vector<uint32_t>& a, const std::vector<uint32_t>& b,
                 uint64_t& cost, uint64_t& size) {
  size_t i = 0, j = 0;
  cost = 0; size = 0;
  while (i < a.size() || j < b.size()) {
    uint32_t x;
    if (j == b.size() || (i < a.size() && a[i] < b[j])) x = a[i++];
    else if (i == a.size() || b[j] < a[i]) x = b[j++];
    else { x = a[i]; ++i; ++j; }
    cost += d.cost[x]; ++size;
  }
}

std::vector<uint32_t> set_union(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
  std::vector<uint32_t> out;
  out.reserve(a.size() + b.size());
  std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(out));
  return out;
}


// Bottom-up merge of Sec. 5.1 (stages 3 and 4) under a cost bound B: take the
// cheapest process; merge it into the process it communicates with whose
// union is cheapest, if that stays within B and within the node capacity;
// otherwise into the costliest process that still fits under B (best fit);
// otherwise skip it.  Stops when every process was considered or the target
// count is reached.
struct SlbResult {
  uint32_t n_alive = 0;
  std::vector<uint32_t> proc_of_sink;
  // the surviving processes, for a later stage to continue from
  std::vector<std::vector<uint32_t>> nodes, sinks;
  std::vector<uint64_t> cost;
};

// who reads each register: the processes whose node sets hold its REG node
std::vector<std::vector<uint32_t>> register_readers(const Design& d,
                                                    const std::vector<std::vector<uint32_t>>& nodes) {
  std::vector<std::vector<uint32_t>> readers(d.R);
  for (uint32_t p = 0; p < (uint32_t)nodes.size(); ++p)
    for (uint32_t x : nodes[p])
      if (d.op[x] == FSIM_OP_REG) readers[d.imm[x]].push_back(p);
  return readers;
}

SlbResult slb_merge(const Design& d, const std::vector<std::vector<uint32_t>>& nodes0,
                    const std::vector<uint64_t>& cost0, const std::vector<std::vector<uint32_t>>& sinks0,
                    const std::vector<std::vector<uint32_t>>& readers, uint64_t B, uint32_t target,
                    uint64_t max_nodes) {
  const uint32_t P0 = (uint32_t)nodes0.size();
  std::vector<std::vector<uint32_t>> nodes(nodes0), sinks(sinks0);
  std::vector<uint64_t> cost(cost0);
  std::vector<uint32_t> owner_init(d.R, UINT32_MAX);
  for (uint32_t p = 0; p < P0; ++p)
    for (uint32_t s : sinks0[p]) if (s < d.R) owner_init[s] = p;
  UF puf(P0);
  std::vector<uint8_t> alive(P0, 1), done(P0, 0);
  std::multiset<std::pair<uint64_t, uint32_t>> by_cost;
  for (uint32_t p = 0; p < P0; ++p) by_cost.emplace(cost[p], p);
  uint32_t n_alive = P0;
  const size_t K = P0 > 200000 ? 4 : 8;
  std::vector<uint32_t> cand, mark(P0, UINT32_MAX);
  uint32_t iter = 0;
  // processes not yet considered, cheapest first
  std::set<std::pair<uint64_t, uint32_t>> todo(by_cost.begin(), by_cost.end());
  auto merge = [&](uint32_t p, uint32_t q) {
    by_cost.erase(by_cost.find({cost[p], p}));
    by_cost.erase(by_cost.find({cost[q], q}));
    todo.erase({cost[q], q});
    bool p_todo = todo.erase({cost[p], p}) > 0;
    nodes[p] = set_union(nodes[p], nodes[q]);
    std::vector<uint32_t>().swap(nodes[q]);
    sinks[p].insert(sinks[p].end(), sinks[q].begin(), sinks[q].end());
    std::vector<uint32_t>().swap(sinks[q]);
    cost[p] = set_cost(d, nodes[p]);
    alive[q] = 0;
    puf.p[q] = p;
    puf.p[p] = p;
    by_cost.emplace(cost[p], p);
    if (p_todo) todo.emplace(cost[p], p);
    n_alive--;
  };
  while (n_alive > target && !todo.empty()) {
    auto [c, p] = *todo.begin();
    todo.erase(todo.begin());
    ++iter;
    cand.clear();
    for (uint32_t x : nodes[p]) {
      if (cand.size() >= K) break;
      if (d.op[x] != FSIM_OP_REG) continue;
      uint32_t o = owner_init[(uint32_t)d.imm[x]];
      if (o == UINT32_MAX) continue;
      uint32_t q = puf.find(o);
      if (q != p && alive[q] && mark[q] != iter) { mark[q] = iter; cand.push_back(q); }
    }
    for (uint32_t s : sinks[p]) {
      if (cand.size() >= K || s >= d.R) break;
      const auto& rd = readers[s];
      for (size_t i = 0; i < rd.size() && i < 32 && cand.size() < K; ++i) {
        uint32_t q = puf.find(rd[i]);
        if (q != p && alive[q] && mark[q] != iter) { mark[q] = iter; cand.push_back(q); }
      }
    }
    uint32_t best = UINT32_MAX;
    uint64_t best_cost = UINT64_MAX;
    for (uint32_t q : cand) {
      uint64_t uc, us;
      union_stats(d, nodes[p], nodes[q], uc, us);
      if (us > max_nodes || uc > B) continue;
      if (uc < best_cost) { best_cost = uc; best = q; }
    }
    if (best == UINT32_MAX && cost[p] <= B) {
      // best fit: the costliest process q with cost(q) <= B - cost(p)
      auto it = by_cost.upper_bound({B - cost[p], UINT32_MAX});
      int tries = 0;
      while (it != by_cost.begin() && tries < 4) {
        --it;
        uint32_t q = it->second;
        if (q == p) continue;
        ++tries;
        uint64_t uc, us;
        union_stats(d, nodes[p], nodes[q], uc, us);
        if (us <= max_nodes && uc <= B) { best = q; break; }
      }
    }
    if (best != UINT32_MAX) {
      merge(best, p);           // p joins best; best stays where it was in the order
      if (alive[best] && !done[best]) {
        // the grown process may still take more work: consider it again
        todo.emplace(cost[best], best);
      }
    } else {
      done[p] = 1;
    }
  }
  SlbResult r;
  r.n_alive = 0;
  r.proc_of_sink.assign(d.n_sinks(), 0);
  for (uint32_t p = 0; p < P0; ++p)
    if (alive[p]) {
      for (uint32_t s : sinks[p]) r.proc_of_sink[s] = r.n_alive;
      r.n_alive++;
      r.nodes.push_back(std::move(nodes[p]));
      r.sinks.push_back(std::move(sinks[p]));
      r.cost.push_back(cost[p]);
    }
  return r;
}

// ---- hypergraph packing (the alternative to bottom-up SLB that Sec. 6.6
// compares against: fibers are the hypergraph's nodes, and the fibers
// sharing a combinational node form a hyperedge of weight c(node)).  A
// partition replicates every node once per process its hyperedge spans, so
// its total replication is sum_P tau(P) minus the design's cost.  Units are
// the stage-1 groups (memory co-location).
//  1. Units are ordered by the median node of their cones (netlists keep
//     related logic close in node order) and cut into consecutive runs
//     whose union cost tau stays within a bound; the smallest bound that
//     gives at most `target` runs is searched (geometric steps, then
//     bisection), and runs also respect the node cap.
//  2. FM-style passes move a unit to the process it shares the most cost
//     with whenever that lowers total replication and keeps the receiving
//     process within the bound and the node cap.  Nodes shared by very many
//     processes are replicated everywhere anyway and are left out of the
//     shared-cost estimate, which only makes a move look costlier.
// Returns the process of every unit, ids compacted; more than `target`
// processes when the node cap leaves no other way.
std::vector<uint32_t> hyper_pack(const Design& d, const std::vector<std::vector<uint32_t>>& unit_nodes,
                                 uint32_t target, uint64_t max_nodes, uint32_t* n_procs) {
  const uint32_t U = (uint32_t)unit_nodes.size();
  std::vector<uint64_t> ucost(U);
  uint64_t max_unit = 0;
  for (uint32_t u = 0; u < U; ++u) {
    ucost[u] = set_cost(d, unit_nodes[u]);
    max_unit = std::max(max_unit, ucost[u]);
  }
  std::vector<uint32_t> order(U);
  std::iota(order.begin(), order.end(), 0u);
  auto key = [&](uint32_t u) -> uint32_t {
    const auto& v = unit_nodes[u];
    return v.empty() ? 0u : v[v.size() / 2];
  };
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return key(a) < key(b); });
  // Register and input leaves cost no operator but each is a value a process
  // loads and keeps live (an LDS value of the plain form from the first
  // level on).  Logic of many small fibers that read many registers (a
  // router, say) is cheap in operators but heavy in leaves, so once a cut
  // under the cost bound alone is known, a process's leaves are capped at
  // 1.15 x their mean over that cut, as long as the target count can still be
  // met.
  auto is_leaf = [&](uint32_t x) { return d.op[x] == FSIM_OP_REG || d.op[x] == FSIM_OP_INPUT; };
  std::vector<uint32_t> uleaves(U, 0);
  uint64_t max_unit_leaves = 0;
  for (uint32_t u = 0; u < U; ++u) {
    for (uint32_t x : unit_nodes[u]) uleaves[u] += is_leaf(x);
    max_unit_leaves = std::max<uint64_t>(max_unit_leaves, uleaves[u]);
  }
  // ---- 1. runs under a union-cost bound (and the leaf cap)
  std::vector<uint32_t> stamp(d.N, UINT32_MAX), proc(U, 0);
  uint64_t max_leaves = UINT64_MAX, leaf_sum = 0;
  auto cut = [&](uint64_t bound, std::vector<uint32_t>* assign) -> uint32_t {
    std::fill(stamp.begin(), stamp.end(), UINT32_MAX);
    uint32_t run = 0;
    uint64_t tau = 0, nodes = 0, leaves = 0;
    leaf_sum = 0;
    for (uint32_t u : order) {
      uint64_t add = 0, addn = 0, addl = 0;
      for (uint32_t x : unit_nodes[u])
        if (stamp[x] != run) { add += d.cost[x]; ++addn; addl += is_leaf(x); }
      if (nodes > 0 && (tau + add > bound || nodes + addn > max_nodes || leaves + addl > max_leaves)) {
        ++run;
        tau = 0;
        nodes = 0;
        leaves = 0;
        add = ucost[u];
        addn = unit_nodes[u].size();
        addl = uleaves[u];
      }
      for (uint32_t x : unit_nodes[u]) stamp[x] = run;
      tau += add;
      nodes += addn;
      leaves += addl;
      leaf_sum += addl;
      if (assign) (*assign)[u] = run;
    }
    return run + 1;
  };
  uint64_t total = 0;
  for (uint64_t c : ucost) total += c;
  // the smallest bound that gives at most `target` runs: geometric steps,
  // then bisection
  auto search = [&]() -> uint64_t {
    uint64_t lo = std::max<uint64_t>(max_unit, 1), hi = 0;
    for (uint64_t B = lo;; B = std::max<uint64_t>(B + 1, B + B / 8)) {
      if (cut(B, nullptr) <= target) { hi = B; break; }
      lo = B + 1;
      if (B >= total) { hi = total; break; }
    }
    for (int it = 0; it < 24 && lo < hi; ++it) {
      const uint64_t mid = lo + (hi - lo) / 2;
      if (cut(mid, nullptr) <= target) hi = mid; else lo = mid + 1;
    }
    return hi;
  };
  uint64_t bound = search();
  {
    const uint32_t runs = cut(bound, nullptr);
    max_leaves = std::max<uint64_t>(max_unit_leaves, leaf_sum * 115 / (100ull * runs) + 1);
    if (cut(total, nullptr) <= target) bound = search();
    else max_leaves = UINT64_MAX;            // the cap would not let the target be met
  }
  const uint32_t P = cut(bound, &proc);
  // ---- incidence: for every node, the processes holding it and how many of
  // their units contain it
  struct Inc { uint32_t p, n; };
  std::vector<std::vector<Inc>> inc(d.N);
  std::vector<uint64_t> tau(P, 0), pnodes(P, 0), pleaves(P, 0);
  auto add = [&](uint32_t u, uint32_t p) {
    for (uint32_t x : unit_nodes[u]) {
      bool found = false;
      for (Inc& e : inc[x]) if (e.p == p) { ++e.n; found = true; break; }
      if (!found) { inc[x].push_back({p, 1}); tau[p] += d.cost[x]; ++pnodes[p]; pleaves[p] += is_leaf(x); }
    }
  };
  auto remove = [&](uint32_t u, uint32_t p) {
    for (uint32_t x : unit_nodes[u]) {
      auto& v = inc[x];
      for (size_t i = 0; i < v.size(); ++i) {
        if (v[i].p != p) continue;
        if (--v[i].n == 0) { v[i] = v.back(); v.pop_back(); tau[p] -= d.cost[x]; --pnodes[p]; pleaves[p] -= is_leaf(x); }
        break;
      }
    }
  };
  for (uint32_t u = 0; u < U; ++u) add(u, proc[u]);
  // ---- 2. refinement
  constexpr size_t kWide = 32;             // nodes in more processes than this: left out of the estimate
  std::vector<uint64_t> shared_c(P, 0), shared_n(P, 0), shared_l(P, 0);
  std::vector<uint32_t> touched;
  for (int pass = 0; pass < 6; ++pass) {
    uint64_t moved = 0;
    for (uint32_t u : order) {
      const uint32_t a = proc[u];
      uint64_t save = 0;                   // cost freed in a by taking u out
      touched.clear();
      for (uint32_t x : unit_nodes[u]) {
        const auto& v = inc[x];
        for (const Inc& e : v) {
          if (e.p == a) { if (e.n == 1) save += d.cost[x]; continue; }
          if (v.size() > kWide) continue;
          if (!shared_c[e.p] && !shared_n[e.p]) touched.push_back(e.p);
          shared_c[e.p] += d.cost[x];
          ++shared_n[e.p];
          shared_l[e.p] += is_leaf(x);
        }
      }
      uint32_t best = UINT32_MAX;
      int64_t best_delta = 0;
      for (uint32_t b : touched) {
        const uint64_t addc = ucost[u] - shared_c[b], addn = unit_nodes[u].size() - shared_n[b];
        const uint64_t addl = uleaves[u] - shared_l[b];
        const int64_t delta = (int64_t)addc - (int64_t)save;   // change of total replication
        if (delta < best_delta && tau[b] + addc <= bound && pnodes[b] + addn <= max_nodes &&
            pleaves[b] + addl <= max_leaves) {
          best_delta = delta;
          best = b;
        }
      }
      for (uint32_t b : touched) shared_c[b] = shared_n[b] = shared_l[b] = 0;
      if (best != UINT32_MAX) {
        remove(u, a);
        add(u, best);
        proc[u] = best;
        ++moved;
      }
    }
    if (!moved) break;
  }
  // ---- compact ids (a process may have lost all its units)
  std::vector<uint32_t> id(P, UINT32_MAX);
  uint32_t n = 0;
  for (uint32_t u : order) {
    if (id[proc[u]] == UINT32_MAX) id[proc[u]] = n++;
    proc[u] = id[proc[u]];
  }
  *n_procs = n;
  return proc;
}

}  // namespace

Status partition_design(Design& d, const fsim_partition* part, const fsim_compile_opts& opts,
                        uint32_t default_target, uint32_t default_max_nodes) {
  const uint32_t S = d.n_sinks();
  // ---- fibers: reverse crawl from every sink (Sec. 5.1)
  std::vector<uint64_t> cone_off(S + 1, 0);
  std::vector<uint32_t> cone;             // sorted per sink
  std::vector<uint32_t> stamp(d.N, UINT32_MAX), stack;
  std::vector<uint8_t> live(d.N, 0);
  std::vector<std::vector<uint32_t>> mem_readers(d.M);
  d.sum_fiber_ops = 0; d.max_fiber_cost = 0; d.max_depth = 0;
  for (uint32_t s = 0; s < S; ++s) {
    uint32_t roots[3], nr = sink_roots(d, s, roots);
    size_t start = cone.size();
    for (uint32_t k = 0; k < nr; ++k)
      if (stamp[roots[k]] != s) { stamp[roots[k]] = s; stack.push_back(roots[k]); }
    while (!stack.empty()) {
      uint32_t x = stack.back(); stack.pop_back();
      cone.push_back(x);
      for (int k = 0; k < arity(d.op[x]); ++k) {
        uint32_t y = d.arg[3ull * x + k];
        if (stamp[y] != s) { stamp[y] = s; stack.push_back(y); }
      }
    }
    std::sort(cone.begin() + start, cone.end());
    uint64_t c = 0, ops = 0;
    for (size_t i = start; i < cone.size(); ++i) {
      uint32_t x = cone[i];
      c += d.cost[x];
      live[x] = 1;
      if (d.op[x] >= FSIM_OP_MEMRD) {
        ops++;
        d.max_depth = std::max(d.max_depth, d.level[x]);
      }
      if (d.op[x] == FSIM_OP_MEMRD) {
        auto& v = mem_readers[d.imm[x]];
        if (v.empty() || v.back() != s) v.push_back(s);
      }
    }
    d.sum_fiber_ops += ops;
    d.max_fiber_cost = std::max(d.max_fiber_cost, c);
    cone_off[s + 1] = cone.size();
  }
  d.n_live_ops = 0;
  for (uint32_t n = 0; n < d.N; ++n) if (live[n] && d.op[n] >= FSIM_OP_MEMRD) d.n_live_ops++;
  phase("fibers (reverse crawl)");

  // ---- stage 1: every sink that reads memory m shares a process with m's
  // write ports, so the end-of-cycle commit never races a read elsewhere
  UF uf(S);
  std::vector<int64_t> mem_anchor(d.M, -1);
  for (uint32_t k = 0; k < d.W; ++k) {
    uint32_t m = d.wp_mem[k];
    if (mem_anchor[m] < 0) mem_anchor[m] = d.R + k; else uf.unite((uint32_t)mem_anchor[m], d.R + k);
  }
  for (uint32_t m = 0; m < d.M; ++m) {
    if (mem_anchor[m] < 0) continue;      // never written: read-only, no constraint
    for (uint32_t s : mem_readers[m]) uf.unite((uint32_t)mem_anchor[m], s);
  }

  d.sink_proc.assign(S, 0);
  if (part) {
    if (part->n_sinks != S || (S && !part->sink_to_process))
      return Status::err(FSIM_E_ARG, "partition: n_sinks does not match the netlist");
    // compact the caller's ids, in first-appearance order
    std::vector<uint32_t> remap;
    std::vector<uint32_t> ids(part->sink_to_process, part->sink_to_process + S);
    uint32_t mx = 0;
    for (uint32_t x : ids) mx = std::max(mx, x);
    if (S && mx > 16u * S) return Status::err(FSIM_E_ARG, "partition: process id out of range");
    remap.assign(S ? mx + 1 : 1, UINT32_MAX);
    uint32_t P = 0;
    for (uint32_t s = 0; s < S; ++s) {
      if (remap[ids[s]] == UINT32_MAX) remap[ids[s]] = P++;
      d.sink_proc[s] = remap[ids[s]];
    }
    for (uint32_t s = 0; s < S; ++s)
      if (d.sink_proc[uf.find(s)] != d.sink_proc[s])
        return Status::err(FSIM_E_ARG,
                           fmt("partition: sink %llu reads or writes a memory whose other ports are in another process", s));
    d.P = std::max(P, 1u);
  } else if (opts.pack == FSIM_PACK_SINGLE) {
    d.P = 1;
  } else {
    // initial processes: the stage-1 groups (one fiber each otherwise)
    std::vector<uint32_t> root_id(S, UINT32_MAX);
    uint32_t P0 = 0;
    for (uint32_t s = 0; s < S; ++s) {
      uint32_t r = uf.find(s);
      if (root_id[r] == UINT32_MAX) root_id[r] = P0++;
      d.sink_proc[s] = root_id[r];
    }
    d.P = std::max(P0, 1u);
    uint32_t target = opts.target_processes ? opts.target_processes : default_target;
    uint64_t max_nodes = opts.max_process_nodes ? opts.max_process_nodes : default_max_nodes;
    if (opts.pack == FSIM_PACK_HYPER && P0 > target) {
      std::vector<std::vector<uint32_t>> unodes(P0);
      {
        std::vector<std::vector<uint32_t>> usinks(P0);
        for (uint32_t s = 0; s < S; ++s) usinks[d.sink_proc[s]].push_back(s);
        for (uint32_t p = 0; p < P0; ++p) {
          std::vector<uint32_t> acc;
          for (uint32_t s : usinks[p]) {
            std::vector<uint32_t> c(cone.begin() + cone_off[s], cone.begin() + cone_off[s + 1]);
            acc = acc.empty() ? std::move(c) : set_union(acc, c);
          }
          unodes[p] = std::move(acc);
        }
      }
      phase("initial processes");
      uint32_t n = 0;
      std::vector<uint32_t> up = hyper_pack(d, unodes, target, max_nodes, &n);
      if (n > target)
        return Status::err(FSIM_E_CAPACITY,
            fmt("cannot pack the design into %llu processes of at most %llu nodes", target, max_nodes));
      for (uint32_t s = 0; s < S; ++s) d.sink_proc[s] = up[d.sink_proc[s]];
      d.P = std::max(n, 1u);
      phase("hypergraph packing");
    } else if (opts.pack == FSIM_PACK_SLB && P0 > target) {
      std::vector<std::vector<uint32_t>> nodes0(P0), sinks0(P0);
      for (uint32_t s = 0; s < S; ++s) sinks0[d.sink_proc[s]].push_back(s);
      std::vector<uint64_t> cost0(P0);
      uint64_t straggler = 0, total = 0;
      for (uint32_t p = 0; p < P0; ++p) {
        std::vector<uint32_t> acc;
        for (uint32_t s : sinks0[p]) {
          std::vector<uint32_t> c(cone.begin() + cone_off[s], cone.begin() + cone_off[s + 1]);
          acc = acc.empty() ? std::move(c) : set_union(acc, c);
        }
        nodes0[p] = std::move(acc);
        cost0[p] = set_cost(d, nodes0[p]);
        straggler = std::max(straggler, cost0[p]);
        total += cost0[p];
      }
      std::vector<std::vector<uint32_t>> readers = register_readers(d, nodes0);
      phase("initial processes");
      SlbResult best;
      // stage 3: conservative merge, the straggler bound stays put
      SlbResult r3 = slb_merge(d, nodes0, cost0, sinks0, readers, straggler, target, max_nodes);
      phase("stage 3");
      if (r3.n_alive <= target) {
        best = std::move(r3);
      } else {
        // stage 4 continues from stage 3's processes; the straggler may now
        // grow.  The smallest bound under which the merge reaches the target
        // is searched upward from max(straggler, total / target):
        // geometrically, then by bisection between the last failing and the
        // first passing bound.
        std::vector<std::vector<uint32_t>> n3 = std::move(r3.nodes), s3 = std::move(r3.sinks);
        std::vector<uint64_t> c3 = std::move(r3.cost);
        const uint32_t P3 = (uint32_t)n3.size();
        uint64_t total3 = 0;
        for (uint64_t x : c3) total3 += x;
        std::vector<std::vector<uint32_t>> readers3 = register_readers(d, n3);
        uint64_t lo = std::max<uint64_t>(straggler, (total3 + target - 1) / target), hi = 0;
        bool found = false;
        const double grow = P3 > 20000 ? 1.04 : 1.1;
        // a larger bound that no longer lowers the process count means the
        // node cap, not the bound, is what stops the merge: three such trials
        // in a row end the search (the final unbounded trial decides)
        uint32_t prev_alive = UINT32_MAX, stalled = 0;
        for (uint64_t B = lo; B <= total3; B = std::max<uint64_t>(B + 1, (uint64_t)(B * grow))) {
          SlbResult t = slb_merge(d, n3, c3, s3, readers3, B, target, max_nodes);
          phase("stage 4 trial");
          if (t.n_alive <= target) { hi = B; best = std::move(t); found = true; break; }
          lo = B + 1;
          stalled = t.n_alive >= prev_alive ? stalled + 1 : 0;
          prev_alive = std::min(prev_alive, t.n_alive);
          if (stalled >= 3) break;
          if (B == total3) break;
          if (B * grow >= total3) B = total3 - 1;
        }
        if (!found) {
          SlbResult t = slb_merge(d, n3, c3, s3, readers3, total3, target, max_nodes);
          if (t.n_alive > target)
            return Status::err(FSIM_E_CAPACITY,
                fmt("cannot pack the design into %llu processes of at most %llu nodes", target, max_nodes));
          best = std::move(t);
          hi = total3;
        }
        const int max_bisect = P3 > 20000 ? 3 : 16;
        for (int it = 0; it < max_bisect && lo < hi; ++it) {
          uint64_t mid = lo + (hi - lo) / 2;
          SlbResult t = slb_merge(d, n3, c3, s3, readers3, mid, target, max_nodes);
          if (t.n_alive <= target) { hi = mid; best = std::move(t); }
          else lo = mid + 1;
        }
      }
      for (uint32_t s = 0; s < S; ++s) d.sink_proc[s] = best.proc_of_sink[s];
      d.P = std::max(best.n_alive, 1u);
      phase("stage 4");
    }
  }

  phase("packing");
  // ---- process node lists: union of member cones, ordered by level
  d.psink_off.assign(d.P + 1, 0);
  for (uint32_t s = 0; s < S; ++s) d.psink_off[d.sink_proc[s] + 1]++;
  for (uint32_t p = 0; p < d.P; ++p) d.psink_off[p + 1] += d.psink_off[p];
  d.psinks.assign(S, 0);
  {
    std::vector<uint32_t> f(d.psink_off.begin(), d.psink_off.end() - 1);
    for (uint32_t s = 0; s < S; ++s) d.psinks[f[d.sink_proc[s]]++] = s;
  }
  d.proc_off.assign(d.P + 1, 0);
  d.proc_nodes.clear();
  std::fill(stamp.begin(), stamp.end(), UINT32_MAX);
  d.sum_process_ops = 0; d.max_process_cost = 0; d.max_process_levels = 0; d.max_process_nodes = 0;
  for (uint32_t p = 0; p < d.P; ++p) {
    size_t start = d.proc_nodes.size();
    for (uint32_t i = d.psink_off[p]; i < d.psink_off[p + 1]; ++i) {
      uint32_t s = d.psinks[i];
      for (uint64_t j = cone_off[s]; j < cone_off[s + 1]; ++j) {
        uint32_t x = cone[j];
        if (stamp[x] != p) { stamp[x] = p; d.proc_nodes.push_back(x); }
      }
    }
    std::sort(d.proc_nodes.begin() + start, d.proc_nodes.end(), [&](uint32_t a, uint32_t b) {
      if (d.level[a] != d.level[b]) return d.level[a] < d.level[b];
      return a < b;
    });
    uint64_t c = 0, ops = 0;
    uint32_t maxl = 0;
    for (size_t i = start; i < d.proc_nodes.size(); ++i) {
      uint32_t x = d.proc_nodes[i];
      c += d.cost[x];
      if (d.op[x] >= FSIM_OP_MEMRD) { ops++; maxl = std::max(maxl, d.level[x]); }
    }
    d.sum_process_ops += ops;
    d.max_process_cost = std::max(d.max_process_cost, c);
    d.max_process_levels = std::max(d.max_process_levels, maxl);
    d.max_process_nodes = std::max<uint32_t>(d.max_process_nodes, (uint32_t)(d.proc_nodes.size() - start));
    d.proc_off[p + 1] = (uint32_t)d.proc_nodes.size();
  }
  return {};
}

// --------------------------------------------------------- plain encoding

static Instr make(uint8_t op, uint8_t w, uint16_t dst, uint16_t a, uint16_t b, uint16_t c, uint32_t aux) {
  Instr in;
  in.op = op; in.w = w; in.cls = 0; in.flags = 0;
  in.dst = dst; in.a = a; in.b = b; in.c = c; in.aux = aux;
  return in;
}

namespace {

// LDS of one plain-form process in 4-byte units: a narrow value (at most 32
// bits) takes one unit, a wide one an even pair.  Released units are reused;
// a released unit whose partner is free makes a free pair again.  Free lists
// may hold stale entries; the unit states decide.
//
// An operator's result is always stored as 8 bytes: a result in one unit u
// also writes the unit above it, u + 1, with its upper half, which is
// garbage.  So such a result goes where u + 1 is free, and u + 1 is given to
// no value of the same step (whose store could come before or after the
// garbage).  Every allocation names its step; units that take garbage in a
// step are marked with it.
class UnitAlloc {
 public:
  // units below `base` are reserved (never handed out)
  void reset(uint32_t base) {
    st_.assign(base, kUsed);
    g_.assign(base, 0);
    one_.clear();
    two_.clear();
  }
  uint32_t top() const { return (uint32_t)st_.size(); }
  // a unit (or an even pair) for a value defined in step s; `garbage`: a
  // one-unit value whose store also writes the unit above it
  uint32_t take(bool wide, uint32_t s, bool garbage = false) {
    const uint32_t m = s + 1;   // marks: 0 = none
    uint32_t u = UINT32_MAX;
    if (!wide) {
      while (!one_.empty()) {
        const uint32_t v = one_.back();
        one_.pop_back();
        if (st_[v] != kFree) continue;
        if (g_[v] != m && (!garbage || v + 1 >= top() || st_[v + 1] == kFree)) { u = v; break; }
        stash_.push_back(v);
      }
      if (u == UINT32_MAX && pop_pair(m, u)) one_.push_back(u + 1);
      if (u == UINT32_MAX) { grow(); u = top() - 1; }
      st_[u] = kUsed;
    } else {
      if (!pop_pair(m, u)) {
        if (top() & 1) { grow(); one_.push_back(top() - 1); }
        grow();
        grow();
        u = top() - 2;
      }
      st_[u] = st_[u + 1] = kUsed;
    }
    if (garbage) {
      if (u + 1 >= top()) { grow(); one_.push_back(u + 1); }
      g_[u + 1] = m;
    }
    for (uint32_t v : stash_) one_.push_back(v);
    stash_.clear();
    return u;
  }
  void give(uint32_t u, bool wide) {
    st_[u] = kFree;
    if (wide) {
      st_[u + 1] = kFree;
      two_.push_back(u);
      return;
    }
    const uint32_t v = u ^ 1;
    if (v < top() && st_[v] == kFree) two_.push_back(u & ~1u);
    else one_.push_back(u);
  }

 private:
  enum : uint8_t { kUsed = 0, kFree = 1 };
  void grow() {
    st_.push_back(kFree);
    g_.push_back(0);
  }
  // a free even pair neither of whose units took garbage in the step marked m
  bool pop_pair(uint32_t m, uint32_t& u) {
    while (!two_.empty()) {
      const uint32_t v = two_.back();
      two_.pop_back();
      if (st_[v] != kFree || st_[v + 1] != kFree) continue;
      if (g_[v] != m && g_[v + 1] != m) { u = v; flush_pairs(); return true; }
      pstash_.push_back(v);
    }
    flush_pairs();
    return false;
  }
  void flush_pairs() {
    for (uint32_t v : pstash_) two_.push_back(v);
    pstash_.clear();
  }
  std::vector<uint8_t> st_;
  std::vector<uint32_t> g_, one_, two_, stash_, pstash_;
};

// pending register and output stores are written out early, in a store level
// of their own, once this many have accumulated (one full store chunk)
constexpr size_t kStoreFlush = 256;

}  // namespace

// Operator steps of one plain-form process, by list scheduling: a step
// holds at most 64 operators and 64 memory reads, every one of them after the
// steps of its operands, so a step is one chunk of each kind.  Ready
// operators go to the earliest step with room, the longest remaining path
// first; a process takes max(depth, operators / 64) steps or close to it
// instead of one chunk per level and per 64 operators of a level.  Sets
// loc[x] (0 for leaves and constants, 1..K for operators); returns K.
struct StepScratch {
  explicit StepScratch(size_t n) : lid(n, UINT32_MAX) {}
  std::vector<uint32_t> lid;                 // node -> index among the process's operators
  std::vector<uint32_t> ops, height, indeg, succ_off, succ, take, ready;
  std::vector<uint8_t> picked;
};

static uint32_t steps_of(const Design& d, uint32_t lo, uint32_t hi, std::vector<uint32_t>& loc, StepScratch& S) {
  auto is_op = [&](uint32_t x) { return d.op[x] >= FSIM_OP_MEMRD; };
  S.ops.clear();
  for (uint32_t i = lo; i < hi; ++i) {
    const uint32_t x = d.proc_nodes[i];
    if (is_op(x)) { S.lid[x] = (uint32_t)S.ops.size(); S.ops.push_back(x); }
    else loc[x] = 0;
  }
  const uint32_t n = (uint32_t)S.ops.size();
  S.height.assign(n, 0);
  S.indeg.assign(n, 0);
  S.succ_off.assign(n + 1, 0);
  // the process's nodes are in level order, so a reverse pass sees every
  // user of an operator before the operator
  for (uint32_t k = n; k-- > 0;) {
    const uint32_t x = S.ops[k];
    for (int a = 0; a < arity(d.op[x]); ++a) {
      const uint32_t y = d.arg[3ull * x + a];
      if (!is_op(y)) continue;
      S.height[S.lid[y]] = std::max(S.height[S.lid[y]], S.height[k] + 1);
      S.indeg[k]++;
      S.succ_off[S.lid[y] + 1]++;
    }
  }
  for (uint32_t k = 0; k < n; ++k) S.succ_off[k + 1] += S.succ_off[k];
  S.succ.assign(S.succ_off[n], 0);
  {
    std::vector<uint32_t> f(S.succ_off.begin(), S.succ_off.end() - 1);
    for (uint32_t k = 0; k < n; ++k) {
      const uint32_t x = S.ops[k];
      for (int a = 0; a < arity(d.op[x]); ++a) {
        const uint32_t y = d.arg[3ull * x + a];
        if (is_op(y)) S.succ[f[S.lid[y]]++] = k;
      }
    }
  }
  // steps: at least the depth, and enough for 64 operators a step; an
  // operator of height h must run by step K - h (its latest step)
  uint32_t n_alu = 0, depth = 0;
  for (uint32_t k = 0; k < n; ++k) {
    if (d.op[S.ops[k]] != FSIM_OP_MEMRD) n_alu++;
    depth = std::max(depth, S.height[k] + 1);
  }
  const uint32_t K = std::max(depth, (n_alu + 63) / 64);
  S.ready.clear();
  for (uint32_t k = 0; k < n; ++k)
    if (S.indeg[k] == 0) S.ready.push_back(k);
  uint32_t step = 0, done = 0;
  while (done < n) {
    ++step;
    // ready operators by latest step, then opcode, then index
    auto latest = [&](uint32_t k) { return K > S.height[k] ? K - S.height[k] : 1u; };
    std::sort(S.ready.begin(), S.ready.end(), [&](uint32_t a, uint32_t b) {
      const uint32_t la = latest(a), lb = latest(b);
      if (la != lb) return la < lb;
      if (d.op[S.ops[a]] != d.op[S.ops[b]]) return d.op[S.ops[a]] < d.op[S.ops[b]];
      return a < b;
    });
    S.take.clear();
    uint32_t used = 0, cnt_rd = 0, ops_in = 0;
    uint32_t cnt[16] = {0};
    S.picked.assign(S.ready.size(), 0);
    // every memory read that is ready, and the operators due by this step
    // (the longest remaining paths first)
    for (size_t i = 0; i < S.ready.size(); ++i) {
      const uint32_t k = S.ready[i], op = d.op[S.ops[k]];
      if (op == FSIM_OP_MEMRD) {
        if (cnt_rd < 64) { cnt_rd++; S.take.push_back(k); S.picked[i] = 1; }
      } else if (latest(k) <= step && used < 64) {
        used++;
        if (!(ops_in & (1u << op))) ops_in |= 1u << op;
        S.take.push_back(k);
        S.picked[i] = 1;
      }
    }
    // fill the step with operators that have slack, preferring opcodes
    // already in it, then the opcodes with the most ready operators, so a
    // step holds few distinct opcodes
    if (used < 64) {
      for (size_t i = 0; i < S.ready.size(); ++i)
        if (!S.picked[i] && d.op[S.ops[S.ready[i]]] != FSIM_OP_MEMRD) cnt[d.op[S.ops[S.ready[i]]]]++;
      while (used < 64) {
        int best = -1;
        for (int op = 0; op < 16; ++op) {
          if (!cnt[op]) continue;
          if (best < 0) { best = op; continue; }
          const bool in_b = ops_in & (1u << best), in_o = ops_in & (1u << op);
          if (in_o != in_b ? in_o : cnt[op] > cnt[best]) best = op;
        }
        if (best < 0) break;
        for (size_t i = 0; i < S.ready.size() && used < 64; ++i) {
          if (S.picked[i] || d.op[S.ops[S.ready[i]]] != (uint32_t)best) continue;
          S.picked[i] = 1;
          S.take.push_back(S.ready[i]);
          used++;
          cnt[best]--;
        }
        ops_in |= 1u << best;
        cnt[best] = 0;
      }
    }
    // the rest stays ready
    size_t w = 0;
    for (size_t i = 0; i < S.ready.size(); ++i)
      if (!S.picked[i]) S.ready[w++] = S.ready[i];
    S.ready.resize(w);
    for (uint32_t k : S.take) {
      loc[S.ops[k]] = step;
      done++;
      for (uint32_t e = S.succ_off[k]; e < S.succ_off[k + 1]; ++e)
        if (--S.indeg[S.succ[e]] == 0) S.ready.push_back(S.succ[e]);
    }
  }
  for (uint32_t x : S.ops) S.lid[x] = UINT32_MAX;
  return step;
}

Status encode_plain(Design& d, uint32_t max_units) {
  phase("process node lists");
  d.plain_procs.assign(d.P, PlainProc{});
  d.plain_levels.clear();
  d.plain_instr.clear();
  d.plain_chunks.clear();
  d.plain_max_slots = 0;
  d.plain_max_instr = 0;
  d.plain_max_chunks = 0;
  d.max_plain_lvls = 0;
  std::vector<uint32_t> unit(d.N, UINT32_MAX), lpos(d.N, 0), loc(d.N, 0);
  std::vector<uint8_t> zx(d.N, 0);                      // narrow value kept zero-extended in two units
  std::vector<uint32_t> lv_start;                       // per local level: first index into ord
  std::vector<uint32_t> ord;                            // the process's nodes by local level
  StepScratch sched(d.N);
  std::vector<std::vector<uint32_t>> flush;             // per local level: sinks stored right after it
  std::vector<std::pair<uint32_t, uint32_t>> by_last;
  UnitAlloc alloc;
  auto narrow = [&](uint32_t x) { return d.width[x] <= 32; };
  const bool check_units = getenv("FSIM_CHECK_UNITS") && atoi(getenv("FSIM_CHECK_UNITS")) != 0;
  for (uint32_t p = 0; p < d.P; ++p) {
    const uint32_t lo = d.proc_off[p], hi = d.proc_off[p + 1];
    // ---- local levels: 0 holds the leaves and constants, 1..K the steps of
    // the operators (steps_of); ord lists the nodes by level
    const uint32_t K = steps_of(d, lo, hi, loc, sched);
    ord.assign(d.proc_nodes.begin() + lo, d.proc_nodes.begin() + hi);
    std::stable_sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) { return loc[a] < loc[b]; });
    lv_start.assign(K + 2, 0);
    for (uint32_t x : ord) lv_start[loc[x] + 1]++;
    for (uint32_t j = 0; j <= K; ++j) lv_start[j + 1] += lv_start[j];
    // ---- where each register and output sink is stored: with the sinks of
    // its level and earlier ones once kStoreFlush are pending, else in the
    // final store level after level K
    flush.assign(K + 1, {});
    {
      std::vector<std::vector<uint32_t>> by_level(K + 1);
      for (uint32_t k = d.psink_off[p]; k < d.psink_off[p + 1]; ++k) {
        const uint32_t s = d.psinks[k];
        if (s < d.R) by_level[loc[d.reg_next[s]]].push_back(s);
        else if (s >= d.R + d.W) by_level[loc[d.out_node[s - d.R - d.W]]].push_back(s);
      }
      std::vector<uint32_t> pending;
      for (uint32_t j = 0; j <= K; ++j) {
        pending.insert(pending.end(), by_level[j].begin(), by_level[j].end());
        if (j == K || pending.size() >= kStoreFlush) {
          flush[j].swap(pending);
          pending.clear();
        }
      }
    }
    auto root = [&](uint32_t s) { return s < d.R ? d.reg_next[s] : d.out_node[s - d.R - d.W]; };
    // ---- liveness in positions: local level j runs at 2j, the stores after
    // it at 2j + 1, the write-port commit at 2K + 2.  A value's units can be
    // taken by a value defined after the last position that reads it (never
    // by one of the same level, whose chunks may still be reading).
    for (uint32_t i = lo; i < hi; ++i) {
      const uint32_t x = d.proc_nodes[i];
      for (int k = 0; k < arity(d.op[x]); ++k) {
        const uint32_t y = d.arg[3ull * x + k];
        lpos[y] = std::max(lpos[y], 2 * loc[x]);
      }
    }
    for (uint32_t j = 0; j <= K; ++j)
      for (uint32_t s : flush[j]) lpos[root(s)] = std::max(lpos[root(s)], 2 * j + 1);
    for (uint32_t k = d.psink_off[p]; k < d.psink_off[p + 1]; ++k) {
      const uint32_t s = d.psinks[k];
      if (s >= d.R && s < d.R + d.W) {
        const uint32_t q = s - d.R;
        for (uint32_t y : {d.wp_en[q], d.wp_addr[q], d.wp_data[q]}) lpos[y] = 2 * K + 2;
      }
    }
    // ---- which narrow values are kept zero-extended (two units): those
    // read by an instruction whose result depends on their upper half.  A
    // narrow value in one unit is read as 8 bytes whose upper half belongs
    // to another value; that is harmless where only the low 32 bits of the
    // operand reach a result of at most 32 bits (bitwise operators, adds,
    // subtracts, multiplies, the shifted operand of a left shift, the data
    // inputs of a multiplexer) and for stores of at most 32 bits.
    auto need_zext = [&](uint32_t y) { if (narrow(y)) zx[y] = 1; };
    for (uint32_t x : ord) {
      const uint8_t op = d.op[x];
      if (op < FSIM_OP_MEMRD) continue;
      const bool small = d.width[x] <= 32;
      for (int k = 0; k < arity(op); ++k) {
        const uint32_t y = d.arg[3ull * x + k];
        bool tolerant;
        switch (op) {
          case FSIM_OP_AND: case FSIM_OP_OR: case FSIM_OP_XOR: case FSIM_OP_NOT:
          case FSIM_OP_ADD: case FSIM_OP_SUB: case FSIM_OP_MUL: tolerant = small; break;
          case FSIM_OP_SHL: tolerant = small && k == 0; break;
          case FSIM_OP_MUX: tolerant = small && k > 0; break;
          default: tolerant = false;   // SHR, EQ, LT, the address of a memory read
        }
        if (!tolerant) need_zext(y);
      }
    }
    for (uint32_t k = d.psink_off[p]; k < d.psink_off[p + 1]; ++k) {
      const uint32_t s = d.psinks[k];
      if (s < d.R) {
        if (d.reg_width[s] > 32) need_zext(d.reg_next[s]);
      } else if (s < d.R + d.W) {
        const uint32_t q = s - d.R;
        for (uint32_t y : {d.wp_en[q], d.wp_addr[q], d.wp_data[q]}) need_zext(y);
      }
    }
    auto one = [&](uint32_t x) { return narrow(x) && !zx[x]; };
    // ---- units: constants first (loaded once per launch, never released),
    // then every value in order of definition, after releasing the values
    // whose last read comes before it
    alloc.reset(kPlainUnitBase);
    for (uint32_t x : ord)
      if (d.op[x] == FSIM_OP_CONST) unit[x] = alloc.take(!one(x), 0);
    by_last.clear();
    for (uint32_t x : ord)
      if (d.op[x] != FSIM_OP_CONST) by_last.push_back({lpos[x], x});
    std::sort(by_last.begin(), by_last.end());
    size_t rel = 0;
    for (uint32_t x : ord) {
      if (d.op[x] == FSIM_OP_CONST) continue;
      while (rel < by_last.size() && by_last[rel].first < 2 * loc[x]) {
        const uint32_t y = by_last[rel++].second;
        alloc.give(unit[y], !one(y));
      }
      // operators store 8 bytes (the upper half of a one-unit result is
      // garbage); leaves and memory reads store a one-unit value's upper
      // half to the spare unit
      unit[x] = alloc.take(!one(x), loc[x], d.op[x] > FSIM_OP_MEMRD && one(x));
    }
    const uint32_t n = alloc.top();
    if (check_units) {
      // the allocation's invariants, checked from the definition: units are
      // held from a value's definition (position 2 loc; constants from the
      // start) to its last read; (1) no two values hold a unit at a common
      // position; (2) the unit above a one-unit operator result, which its
      // 8-byte store overwrites at its step, is held by no other value then
      struct Iv { uint32_t from, to, x; };
      std::vector<std::vector<Iv>> held(n + 2);
      for (uint32_t x : ord) {
        const uint32_t u = unit[x];
        const bool c = d.op[x] == FSIM_OP_CONST;
        const uint32_t from = c ? 0 : 2 * loc[x], to = c ? UINT32_MAX : std::max(lpos[x], from);
        for (uint32_t k = 0; k < (one(x) ? 1u : 2u); ++k) held[u + k].push_back({from, to, x});
      }
      for (uint32_t u = 0; u < n; ++u)
        for (size_t i = 0; i < held[u].size(); ++i)
          for (size_t j = i + 1; j < held[u].size(); ++j) {
            const Iv &a = held[u][i], &b = held[u][j];
            if (a.from <= b.to && b.from <= a.to)
              return Status::err(FSIM_E_INTERNAL, fmt("process %llu: nodes %llu and %llu share LDS unit %llu while "
                                                      "both are live", p, a.x, b.x, u));
          }
      for (uint32_t x : ord) {
        if (d.op[x] <= FSIM_OP_MEMRD || !one(x)) continue;
        const uint32_t at = 2 * loc[x];
        for (const Iv& b : held[unit[x] + 1])
          if (b.x != x && b.from <= at && at <= b.to)
            return Status::err(FSIM_E_INTERNAL, fmt("process %llu: the 8-byte store of node %llu overwrites node "
                                                    "%llu, live in unit %llu", p, x, b.x, unit[x] + 1));
      }
    }
    if (n > max_units || n > kMaxPlainUnits)
      return Status::err(FSIM_E_CAPACITY,
                         fmt("process %llu needs %llu LDS units of live values; use more processes", p, n));
    PlainProc& pp = d.plain_procs[p];
    pp.n_slots = n;
    // ---- constant prologue: destination word, value
    pp.const_off = (uint32_t)d.plain_instr.size();
    for (uint32_t i = lo; i < hi; ++i) {
      uint32_t x = d.proc_nodes[i];
      if (d.op[x] != FSIM_OP_CONST) continue;
      d.plain_instr.push_back(plain_index(d.width[x], unit[x], 0, one(x)));
      d.plain_instr.push_back(d.imm[x] & (~0ull >> (64 - d.width[x])));
    }
    pp.n_consts = ((uint32_t)d.plain_instr.size() - pp.const_off) / 2;
    pp.instr_off = (uint32_t)d.plain_instr.size();
    pp.chunk_off = (uint32_t)d.plain_chunks.size();
    pp.lvl_off = (uint32_t)d.plain_levels.size();
    // one level from its instruction words, each with its kind and whether
    // its result takes one unit; operators of any opcode share I_ALU chunks,
    // other kinds get chunks of their own
    struct PI {
      uint64_t word;
      uint32_t kind;
      bool out_narrow;
    };
    std::vector<PI> ins;
    uint32_t n_lvls = 0;
    // stores written out among the operator levels go one per lane (64 to a
    // chunk), like the operators around them
    bool in_ops = false;
    auto emit_level = [&]() {
      d.plain_levels.push_back((uint32_t)d.plain_chunks.size() - pp.chunk_off);
      std::stable_sort(ins.begin(), ins.end(), [](const PI& a, const PI& b) {
        return (a.word & 15) != (b.word & 15) ? (a.word & 15) < (b.word & 15) : a.out_narrow > b.out_narrow;
      });
      std::stable_sort(ins.begin(), ins.end(), [](const PI& a, const PI& b) { return a.kind < b.kind; });
      size_t k = 0;
      while (k < ins.size()) {
        const uint32_t kk = ins[k].kind, cap = in_ops ? 64 : chunk_capacity(kk);
        size_t e = k;
        while (e < ins.size() && e - k < cap && ins[e].kind == kk) ++e;
        const uint32_t start = (uint32_t)d.plain_instr.size() - pp.instr_off;
        uint32_t present = 0, flags = 0;
        for (size_t j = k; j < e; ++j) {
          if (kk == I_ALU) present |= 1u << (ins[j].word & 15);
          d.plain_instr.push_back(ins[j].word);
        }
        const uint32_t and_to_lt = ((1u << (I_LT + 1)) - 1) & ~((1u << I_AND) - 1);
        const uint32_t n_tree = (uint32_t)__builtin_popcount(present & and_to_lt);
        if (kk == I_ALU && !(present & (1u << I_MUL))) {
          if (n_tree >= kDenseOps) flags |= kDenseChunk;
          if (n_tree >= kDenseOpsLow) flags |= kDenseLow;
        }
        if (kk != I_ALU) flags |= kOtherKind;
        d.plain_chunks.push_back(make_chunk(start, (uint32_t)(e - k), kk, present, flags));
        k = e;
      }
      ins.clear();
      n_lvls++;
    };
    auto emit_stores = [&](const std::vector<uint32_t>& sinks) {
      for (uint32_t s : sinks) {
        const uint32_t x = root(s);
        if (s < d.R)
          ins.push_back({plain_index(d.reg_width[s], unit[x], s), I_STREG, true});
        else
          ins.push_back({plain_index(d.width[x], unit[x], s - d.R - d.W) | 1, I_STOUT, true});
      }
      emit_level();
    };
    // level 0: register and input loads (always present, possibly empty)
    for (uint32_t i = lv_start[0]; i < lv_start[1]; ++i) {
      const uint32_t x = ord[i];
      // the sign bit gives the destination's size (an input's width
      // also folds in the port's own width)
      if (d.op[x] == FSIM_OP_REG)
        ins.push_back({plain_index(d.width[x], unit[x], d.imm[x], one(x)), I_LDREG, one(x)});
      else if (d.op[x] == FSIM_OP_INPUT)
        ins.push_back({plain_index(std::min<uint8_t>(d.width[x], d.in_width[d.imm[x]]), unit[x], d.imm[x], one(x)) | 1,
                       I_LDIN, one(x)});
    }
    emit_level();
    pp.n_leaf = (uint32_t)d.plain_instr.size() - pp.instr_off;
    pp.c_ops = (uint32_t)d.plain_chunks.size() - pp.chunk_off;
    in_ops = true;
    for (uint32_t j = 0; j <= K; ++j) {
      if (j > 0) {
        for (uint32_t i = lv_start[j]; i < lv_start[j + 1]; ++i) {
          const uint32_t x = ord[i];
          const uint8_t op = d.op[x];
          const uint32_t* a = &d.arg[3ull * x];
          if (op == FSIM_OP_MEMRD) {
            ins.push_back({plain_word(0, d.width[x], unit[x], unit[a[0]], d.imm[x] & 0xFFF, d.imm[x] >> 12, one(x)),
                           I_MEMRD, one(x)});
          } else {
            // an unused operand repeats a
            auto opnd = [&](int k) { return a[k < arity(op) ? k : 0]; };
            ins.push_back({plain_word(op, d.width[x], unit[x], unit[opnd(0)], unit[opnd(1)], unit[opnd(2)], one(x)),
                           I_ALU, one(x)});
          }
        }
        emit_level();
      }
      if (j == K) {
        pp.c_st = (uint32_t)d.plain_chunks.size() - pp.chunk_off;
        pp.st_first = (uint32_t)d.plain_instr.size() - pp.instr_off;
        in_ops = false;
      }
      if (!flush[j].empty() || j == K) emit_stores(flush[j]);
    }
    d.plain_levels.push_back((uint32_t)d.plain_chunks.size() - pp.chunk_off);
    pp.n_lvls = n_lvls;
    pp.n_chunks = (uint32_t)d.plain_chunks.size() - pp.chunk_off;
    pp.n_instr = (uint32_t)d.plain_instr.size() - pp.instr_off;
    if (pp.n_instr > 0xFFFF)
      return Status::err(FSIM_E_CAPACITY, fmt("process %llu has %llu instructions; use more processes", p, pp.n_instr));
    // write-port commit, in port order
    for (uint32_t k = d.psink_off[p]; k < d.psink_off[p + 1]; ++k) {
      uint32_t s = d.psinks[k];
      if (s >= d.R && s < d.R + d.W) {
        uint32_t q = s - d.R;
        if (d.wp_mem[q] >= kMaxWportMems)
          return Status::err(FSIM_E_CAPACITY, fmt("plain form: memory %llu is past the %llu write-port memories "
                                                  "its encoding holds", d.wp_mem[q], kMaxWportMems));
        const uint32_t en = d.wp_en[q], ad = d.wp_addr[q], da = d.wp_data[q];
        d.plain_instr.push_back(plain_word(0, d.mem_width[d.wp_mem[q]], unit[en], unit[ad], unit[da], d.wp_mem[q]));
      }
    }
    pp.n_wp = (uint32_t)d.plain_instr.size() - pp.instr_off - pp.n_instr;
    d.plain_max_slots = std::max(d.plain_max_slots, n);
    d.plain_max_instr = std::max(d.plain_max_instr, pp.n_instr + pp.n_wp);
    d.plain_max_chunks = std::max(d.plain_max_chunks, pp.n_chunks);
    d.max_plain_lvls = std::max(d.max_plain_lvls, n_lvls);
    for (uint32_t j = lo; j < hi; ++j) {
      unit[d.proc_nodes[j]] = UINT32_MAX;
      lpos[d.proc_nodes[j]] = 0;
      zx[d.proc_nodes[j]] = 0;
    }
  }
  phase("encode plain");
  if (getenv("FSIM_VERBOSE") && d.P) {
    std::vector<uint32_t> ns;
    for (const PlainProc& q : d.plain_procs) ns.push_back(q.n_slots);
    std::sort(ns.begin(), ns.end());
    fprintf(stderr, "fsim compile: plain LDS units per process: p50 %u p90 %u p99 %u max %u\n", ns[ns.size() / 2],
            ns[ns.size() * 9 / 10], ns[ns.size() * 99 / 100], ns.back());
    uint64_t n_alu = 0, lanes_alu = 0, distinct = 0, dense = 0, n_memrd = 0, n_flush = 0, single_op = 0,
             op_chunks[16] = {0};
    for (const PlainProc& q : d.plain_procs)
      for (uint32_t c = q.c_ops; c < q.c_st; ++c) {
        const uint64_t cw = d.plain_chunks[q.chunk_off + c];
        const uint32_t kind = (uint32_t)(cw >> 24) & 0xFF, fl = (uint32_t)(cw >> 48);
        if (kind == I_ALU) {
          n_alu++;
          lanes_alu += ((cw >> 16) & 0xFF) + 1;
          distinct += __builtin_popcount((uint32_t)(cw >> 32) & 0xFFFF);
          if (__builtin_popcount((uint32_t)(cw >> 32) & 0xFFFF) == 1) single_op++;
          for (int k = 0; k < 16; ++k) op_chunks[k] += (cw >> (32 + k)) & 1;
          if (fl & kDenseChunk) dense++;
        } else if (kind == I_MEMRD) n_memrd++;
        else n_flush++;
      }
    fprintf(stderr, "fsim compile: plain operator chunks %llu: lanes/chunk %.1f, opcodes/chunk %.2f; memory-read chunks "
            "%llu, early store chunks %llu\n", (unsigned long long)n_alu, n_alu ? (double)lanes_alu / n_alu : 0.0,
            n_alu ? (double)distinct / n_alu : 0.0, (unsigned long long)n_memrd, (unsigned long long)n_flush);
    fprintf(stderr, "fsim compile: plain operator chunks with one opcode: %.1f%%, with most opcodes (dense): %.1f%%\n",
            n_alu ? 100.0 * single_op / n_alu : 0.0, n_alu ? 100.0 * dense / n_alu : 0.0);
    {
      std::vector<uint32_t> steps;
      for (const PlainProc& q : d.plain_procs) steps.push_back(q.c_st - q.c_ops);
      std::sort(steps.begin(), steps.end());
      if (!steps.empty())
        fprintf(stderr, "fsim compile: operator-phase chunks per process: p10 %u p50 %u p90 %u p99 %u max %u\n",
                steps[steps.size() / 10], steps[steps.size() / 2], steps[steps.size() * 9 / 10],
                steps[steps.size() * 99 / 100], steps.back());
    }
    fprintf(stderr, "fsim compile: plain operator chunks holding opcode k (%%):");
    for (int k = I_AND; k <= I_MUL; ++k) fprintf(stderr, " %d:%.0f", k, n_alu ? 100.0 * op_chunks[k] / n_alu : 0.0);
    fprintf(stderr, "\n");
    uint64_t wc = 0, wl = 0, ws = 0, ww = 0, cl = 0, cs = 0;
    for (const PlainProc& q : d.plain_procs) {
      wc += 2 * q.n_consts;
      ww += q.n_wp;
      for (uint32_t c = 0; c < q.n_chunks; ++c) {
        const uint64_t cw = d.plain_chunks[q.chunk_off + c];
        const uint32_t cnt = (uint32_t)((cw >> 16) & 0xFF) + 1;
        if (c < q.c_ops) { wl += cnt; cl++; }
        else if (c >= q.c_st) { ws += cnt; cs++; }
      }
    }
    fprintf(stderr, "fsim compile: plain words: consts %llu leaves %llu (%llu chunks) ops+flushes %llu "
            "final stores %llu (%llu chunks) write ports %llu; chunks %zu\n", (unsigned long long)wc,
            (unsigned long long)wl, (unsigned long long)cl, (unsigned long long)(d.plain_instr.size() - wc - wl - ws - ww),
            (unsigned long long)ws, (unsigned long long)cs, (unsigned long long)ww, d.plain_chunks.size());
    for (uint32_t p = 0; p < d.P; ++p)
      if (d.plain_procs[p].n_slots + 64 > ns.back())
        fprintf(stderr, "fsim compile:   process %u: %u units, %u nodes, %u sinks, %u levels, %u chunks\n", p,
                d.plain_procs[p].n_slots, d.proc_off[p + 1] - d.proc_off[p], d.psink_off[p + 1] - d.psink_off[p],
                d.plain_procs[p].n_lvls, d.plain_procs[p].n_chunks);
  }
  return {};
}

// Batched form: each process becomes one sequential, wave-uniform stream.
// Order: for every sink in turn, a depth-first post-order of its cone (the
// operand with the deeper subtree first, so fewer values are live at once);
// each node is emitted once, leaves just before their first use.  Slots are
// allocated per class (1-bit masks, <= 32-bit, <= 64-bit) by liveness; a slot
// is released after its last use.  Constants are not given slots: an operand
// of class K names an entry of the constant pool.  Register stores follow the
// instruction that produces the value; the memory write ports come last.
Status encode_batched(Design& d, uint32_t max_slots_per_class[3]) {
  d.batch_procs.assign(d.P, BatchProc{});
  d.batch_instr.clear();
  d.batch_consts.clear();
  d.batch_slots[0] = d.batch_slots[1] = d.batch_slots[2] = 0;
  // internal register numbering: per class, in register order
  d.reg_cls_idx.assign(d.R, 0);
  d.reg_count[0] = d.reg_count[1] = d.reg_count[2] = 0;
  for (uint32_t r = 0; r < d.R; ++r) {
    uint8_t k = class_of_width(d.reg_width[r]);
    d.reg_cls_idx[r] = ((uint32_t)k << 30) | d.reg_count[k]++;
  }
  std::vector<uint32_t> emitted(d.N, UINT32_MAX);   // instruction index per node (this process)
  std::vector<uint32_t> last_use(d.N, 0), slot_of(d.N, UINT32_MAX), kidx(d.N, UINT32_MAX);
  std::vector<uint32_t> order, stack;
  std::vector<uint8_t> cls_of(d.N, 0);
  std::vector<uint32_t> sub(d.N, 0);                // subtree size estimate for ordering
  for (uint32_t n = 0; n < d.N; ++n) {
    cls_of[n] = class_of_width(d.width[n]);
    uint32_t s = 1;
    for (int k = 0; k < arity(d.op[n]); ++k) s += std::min<uint32_t>(sub[d.arg[3ull * n + k]], 1u << 20);
    sub[n] = std::min<uint32_t>(s, 1u << 20);       // nodes precede their users in level order only,
  }                                                  // so this is a rough size (operands may follow)
  for (uint32_t p = 0; p < d.P; ++p) {
    BatchProc& bp = d.batch_procs[p];
    bp.instr_off = (uint32_t)d.batch_instr.size();
    bp.const_off = (uint32_t)d.batch_consts.size();
    order.clear();
    // ---- order: DFS post-order from each sink
    auto visit = [&](uint32_t root) {
      if (emitted[root] != UINT32_MAX) return;
      stack.push_back(root);
      while (!stack.empty()) {
        uint32_t x = stack.back();
        if (emitted[x] != UINT32_MAX) { stack.pop_back(); continue; }
        // push operands not yet emitted, larger subtree last (visited first)
        uint32_t ops[3]; int na = 0;
        for (int k = 0; k < arity(d.op[x]); ++k) {
          uint32_t y = d.arg[3ull * x + k];
          if (emitted[y] == UINT32_MAX) ops[na++] = y;
        }
        if (na == 0) {
          stack.pop_back();
          emitted[x] = (uint32_t)order.size();
          order.push_back(x);
          continue;
        }
        std::sort(ops, ops + na, [&](uint32_t a, uint32_t b) { return sub[a] < sub[b]; });
        for (int k = 0; k < na; ++k) stack.push_back(ops[k]);
      }
    };
    for (uint32_t k = d.psink_off[p]; k < d.psink_off[p + 1]; ++k) {
      uint32_t s = d.psinks[k];
      if (s < d.R) visit(d.reg_next[s]);
      else if (s < d.R + d.W) { uint32_t q = s - d.R; visit(d.wp_en[q]); visit(d.wp_addr[q]); visit(d.wp_data[q]); }
      else visit(d.out_node[s - d.R - d.W]);
    }
    // ---- leaf loads in groups: the order is cut into segments holding at
    // most kGroup register/input leaves, and each segment's leaves move to its
    // start (a leaf has no operands, so any earlier position is valid).  The
    // kernel then issues a group's loads back to back and waits once, instead
    // of one full memory latency per leaf.
    {
      const size_t kGroup = kLeafRun;
      std::vector<uint32_t> out, leaves, rest;
      out.reserve(order.size());
      auto flush = [&]() {
        out.insert(out.end(), leaves.begin(), leaves.end());
        out.insert(out.end(), rest.begin(), rest.end());
        leaves.clear(); rest.clear();
      };
      // within a group, inputs first, then registers by state class, so that
      // register loads of one class form runs
      auto leaf_key = [&](uint32_t x) -> uint32_t {
        return d.op[x] == FSIM_OP_INPUT ? 0u : 1u + class_of_width(d.reg_width[d.imm[x]]);
      };
      auto flush_sorted = [&]() {
        std::stable_sort(leaves.begin(), leaves.end(),
                         [&](uint32_t a, uint32_t b) { return leaf_key(a) < leaf_key(b); });
        flush();
      };
      for (uint32_t x : order) {
        const bool leaf = d.op[x] == FSIM_OP_REG || d.op[x] == FSIM_OP_INPUT;
        if (leaf && leaves.size() == kGroup) flush_sorted();
        (leaf ? leaves : rest).push_back(x);
      }
      flush_sorted();
      order.swap(out);
    }
    // ---- loads of 1-bit registers into 1-bit values lead the stream: the
    // kernel takes up to 64 of them (a block of the stream) with one vector
    // load, one lane per leaf, and each holds only an 8-byte mask slot
    auto is_bleaf = [&](uint32_t x) {
      return d.op[x] == FSIM_OP_REG && d.width[x] == 1 && d.reg_width[d.imm[x]] == 1;
    };
    std::stable_partition(order.begin(), order.end(), is_bleaf);
    uint32_t n_bleaf = 0;
    while (n_bleaf < order.size() && is_bleaf(order[n_bleaf])) ++n_bleaf;
    for (uint32_t i = 0; i < (uint32_t)order.size(); ++i) emitted[order[i]] = i;
    // ---- liveness (positions in order; sinks read at the end)
    const uint32_t n_ord = (uint32_t)order.size();
    for (uint32_t i = 0; i < n_ord; ++i) last_use[order[i]] = i;
    for (uint32_t i = 0; i < n_ord; ++i) {
      uint32_t x = order[i];
      for (int k = 0; k < arity(d.op[x]); ++k) last_use[d.arg[3ull * x + k]] = std::max(last_use[d.arg[3ull * x + k]], i);
    }
    // register and output stores follow the instruction that produces the
    // value (short live ranges); write ports need their values until the end.
    // A store of a 1-bit register load from the leading batch follows the
    // whole batch (the batch must stay contiguous), and the value lives until
    // then.
    std::vector<std::vector<uint32_t>> stores_after(n_ord);
    auto store_pos = [&](uint32_t root) -> uint32_t {
      const uint32_t e = emitted[root];
      if (e >= n_bleaf) return e;
      last_use[root] = std::max(last_use[root], n_bleaf);
      return n_bleaf - 1;
    };
    for (uint32_t k = d.psink_off[p]; k < d.psink_off[p + 1]; ++k) {
      uint32_t s = d.psinks[k];
      if (s < d.R) stores_after[store_pos(d.reg_next[s])].push_back(s);
      else if (s < d.R + d.W) {
        uint32_t q = s - d.R;
        last_use[d.wp_en[q]] = last_use[d.wp_addr[q]] = last_use[d.wp_data[q]] = n_ord;
      } else {
        stores_after[store_pos(d.out_node[s - d.R - d.W])].push_back(s);
      }
    }
    // ---- slot allocation and emission.  1-bit masks get 8-byte slots of
    // their own; per-lane values share one arena of 256-byte pages, where a
    // <=32-bit value takes one page and a <=64-bit value two adjacent ones
    // (first fit from the bottom), so the region follows the bytes live at
    // once rather than the per-class peaks.
    std::vector<uint32_t> free_masks;
    std::vector<uint8_t> page_busy;
    uint32_t used[3] = {0, 0, 0}, live[3] = {0, 0, 0}, pages = 0;
    std::vector<std::vector<uint32_t>> release_at(n_ord + 1);
    for (uint32_t i = 0; i < n_ord; ++i) {
      uint32_t x = order[i];
      if (d.op[x] == FSIM_OP_CONST) continue;
      release_at[std::min(last_use[x], n_ord)].push_back(x);
    }
    uint32_t masks = 0;
    auto get_slot = [&](uint8_t k) -> uint32_t {
      used[k] = std::max(used[k], ++live[k]);
      if (k == C_B) {
        if (!free_masks.empty()) { uint32_t s = free_masks.back(); free_masks.pop_back(); return s; }
        return masks++;
      }
      const uint32_t n = k == C_D ? 2 : 1;
      // first s whose n pages are free (pages past the arena's end are free)
      auto busy = [&](uint32_t j) { return j < page_busy.size() && page_busy[j]; };
      uint32_t s = 0;
      while (busy(s) || (n == 2 && busy(s + 1))) ++s;
      if (page_busy.size() < s + n) page_busy.resize(s + n, 0);
      for (uint32_t j = 0; j < n; ++j) page_busy[s + j] = 1;
      pages = std::max(pages, s + n);
      return s;
    };
    auto put_slot = [&](uint8_t k, uint32_t s) {
      --live[k];
      if (k == C_B) { free_masks.push_back(s); return; }
      page_busy[s] = 0;
      if (k == C_D) page_busy[s + 1] = 0;
    };
    auto operand = [&](uint32_t y, uint8_t& cls) -> uint16_t {
      if (d.op[y] == FSIM_OP_CONST) { cls = 3; return (uint16_t)kidx[y]; }
      cls = cls_of[y];
      return (uint16_t)slot_of[y];
    };
    for (uint32_t i = 0; i < n_ord; ++i) {
      uint32_t x = order[i];
      uint8_t op = d.op[x];
      if (op == FSIM_OP_CONST) {
        uint32_t ci = (uint32_t)d.batch_consts.size() - bp.const_off;
        if (ci > 0xFFFF) return Status::err(FSIM_E_CAPACITY, fmt("process %llu has too many constants", p));
        kidx[x] = ci;
        d.batch_consts.push_back(d.imm[x] & (~0ull >> (64 - d.width[x])));
      } else {
        // operands are read before the destination slot is taken, so a slot
        // freed by this instruction's last operand use may be reused by it
        Instr in = make(0, d.width[x], 0, 0, 0, 0, 0);
        uint8_t ca = 0, cb = 0, cc = 0;
        const uint32_t* a = &d.arg[3ull * x];
        if (op == FSIM_OP_REG) {
          const uint32_t r = (uint32_t)d.imm[x];
          in.op = I_LDREG;
          in.aux = d.reg_cls_idx[r] & 0x3FFFFFFF;
          in.b = (uint16_t)(r & 0xFFFF); in.c = (uint16_t)(r >> 16);
          ca = class_of_width(d.reg_width[r]);            // the state array it comes from
        } else if (op == FSIM_OP_INPUT) {
          in.op = I_LDIN;
          in.w = std::min<uint8_t>(d.width[x], d.in_width[d.imm[x]]);
          in.aux = (uint32_t)d.imm[x];
        } else if (op == FSIM_OP_MEMRD) {
          in.op = I_MEMRD; in.aux = (uint32_t)d.imm[x];
          in.a = operand(a[0], ca);
        } else {
          in.op = op;
          in.a = operand(a[0], ca);
          if (arity(op) > 1) in.b = operand(a[1], cb); else { in.b = in.a; cb = ca; }
          if (arity(op) > 2) in.c = operand(a[2], cc); else { in.c = in.a; cc = ca; }
        }
        for (uint32_t y : release_at[i])
          if (y != x && slot_of[y] < UINT32_MAX - 1) put_slot(cls_of[y], slot_of[y]);
        const uint8_t kd = cls_of[x];
        slot_of[x] = get_slot(kd);
        in.dst = (uint16_t)slot_of[x];
        in.cls = (uint8_t)(kd | (ca << 2) | (cb << 4) | (cc << 6));
        d.batch_instr.push_back(in);
        if (last_use[x] == i && d.op[x] != FSIM_OP_CONST) {
          // dead on arrival (only a sink's store reads it): released after the stores
        }
      }
      for (uint32_t s : stores_after[i]) {
        uint8_t ca;
        uint16_t sa = operand(s < d.R ? d.reg_next[s] : d.out_node[s - d.R - d.W], ca);
        if (s < d.R) {
          Instr st = make(I_STREG, d.reg_width[s], 0, sa, (uint16_t)(s & 0xFFFF), (uint16_t)(s >> 16),
                          d.reg_cls_idx[s] & 0x3FFFFFFF);
          st.cls = (uint8_t)(class_of_width(d.reg_width[s]) | (ca << 2));
          d.batch_instr.push_back(st);
        } else {
          uint32_t o = s - d.R - d.W;
          Instr st = make(I_STOUT, d.width[d.out_node[o]], 0, sa, 0, 0, o);
          st.cls = (uint8_t)(ca << 2);
          d.batch_instr.push_back(st);
        }
      }
      if (last_use[x] == i && slot_of[x] != UINT32_MAX && d.op[x] != FSIM_OP_CONST) {
        put_slot(cls_of[x], slot_of[x]);
        slot_of[x] = UINT32_MAX - 1;       // released (value no longer needed)
      }
    }
    // write ports, in port order, after every read of the process
    for (uint32_t k = d.psink_off[p]; k < d.psink_off[p + 1]; ++k) {
      uint32_t s = d.psinks[k];
      if (s < d.R || s >= d.R + d.W) continue;
      uint32_t q = s - d.R;
      uint8_t ca, cb, cc;
      uint16_t sa = operand(d.wp_en[q], ca), sb = operand(d.wp_addr[q], cb), sc = operand(d.wp_data[q], cc);
      Instr wp = make(I_WPORT, d.mem_width[d.wp_mem[q]], 0, sa, sb, sc, d.wp_mem[q]);
      wp.cls = (uint8_t)((ca << 2) | (cb << 4) | (cc << 6));
      d.batch_instr.push_back(wp);
    }
    bp.n_instr = (uint32_t)d.batch_instr.size() - bp.instr_off;
    bp.n_consts = (uint32_t)d.batch_consts.size() - bp.const_off;
    // runs of consecutive leaf loads (at most kLeafRun, never crossing a block of
    // 64 instructions): the first carries the run length in flags, the
    // kernel executes the run as one group.  A run of register loads of one
    // class whose slot class and width match the register's gets its own
    // opcode (K_LDREG_*), executed without per-load class tests.
    for (uint32_t j0 = 0; j0 < n_bleaf; j0 += 64) {
      const uint32_t n = std::min<uint32_t>(64, n_bleaf - j0);
      for (uint32_t k = 0; k < n; ++k) d.batch_instr[bp.instr_off + j0 + k].op = K_LDB_BATCH;
      d.batch_instr[bp.instr_off + j0].flags = (uint8_t)n;
    }
    for (uint32_t i = bp.instr_off + n_bleaf; i < bp.instr_off + bp.n_instr;) {
      auto is_leaf = [&](uint32_t j) { return d.batch_instr[j].op == I_LDREG || d.batch_instr[j].op == I_LDIN; };
      auto fast_kind = [&](uint32_t j) -> uint32_t {   // 0: not a plain same-class register load
        const Instr& in = d.batch_instr[j];
        if (in.op != I_LDREG) return 0;
        const uint32_t r = in.b | ((uint32_t)in.c << 16);
        const uint8_t cd = in.cls & 3, ca = (in.cls >> 2) & 3;
        if (cd != ca || in.w != d.reg_width[r]) return 0;
        return K_LDREG_B + ca;
      };
      if (!is_leaf(i)) { ++i; continue; }
      const uint32_t fk = fast_kind(i);
      uint32_t j = i + 1;
      while (j < bp.instr_off + bp.n_instr && j - i < kLeafRun && is_leaf(j) && (j - bp.instr_off) % 64 != 0 &&
             fast_kind(j) == fk)
        ++j;
      d.batch_instr[i].flags = (uint8_t)(j - i);
      if (fk)
        for (uint32_t k = i; k < j; ++k) d.batch_instr[k].op = (uint8_t)fk;
      i = j;
    }
    bp.mask_slots = masks;
    bp.row_pages = pages;
    for (int k = 0; k < 3; ++k) {
      d.batch_slots[k] = std::max(d.batch_slots[k], used[k]);
      if (max_slots_per_class && used[k] > max_slots_per_class[k])
        return Status::err(FSIM_E_CAPACITY,
                           fmt("process %llu needs %llu live slots of one class; use more processes", p, used[k]));
    }
    for (uint32_t i = 0; i < n_ord; ++i) { emitted[order[i]] = UINT32_MAX; slot_of[order[i]] = UINT32_MAX; kidx[order[i]] = UINT32_MAX; last_use[order[i]] = 0; }
  }
  // ---- final form: handler kinds and LDS byte offsets, laid out per process
  d.batch_wave_bytes = 0;
  std::vector<uint32_t> wave_bytes_of;
  for (uint32_t p = 0; p < d.P; ++p) {
    BatchProc& bp = d.batch_procs[p];
    const uint32_t kbase = 16 + 8 * bp.mask_slots;
    const uint32_t rbase = (kbase + 8 * bp.n_consts + 15) & ~15u;
    const uint32_t end = rbase + 256 * bp.row_pages + 16;     // + slack for 8-byte reads of u32 rows
    if (end > 0xFFFF)
      return Status::err(FSIM_E_CAPACITY, fmt("batched form: %llu bytes of live values per wave exceed the "
                                              "16-bit offsets; use more processes", end));
    bp.kbase = kbase;
    d.batch_wave_bytes = std::max(d.batch_wave_bytes, end);
    wave_bytes_of.push_back(end);
    for (uint32_t i = bp.instr_off; i < bp.instr_off + bp.n_instr; ++i) {
      Instr& in = d.batch_instr[i];
      const uint8_t cd = in.cls & 3, ca = (in.cls >> 2) & 3, cb = (in.cls >> 4) & 3, cc = (in.cls >> 6) & 3;
      auto off = [&](uint8_t cls, uint16_t idx) -> uint16_t {
        switch (cls) {
          case C_B: return (uint16_t)(16 + 8 * idx);
          case C_W:
          case C_D: return (uint16_t)(rbase + 256 * idx);
          default:  return (uint16_t)(kbase + 8 * idx);
        }
      };
      // a constant operand of a 1-bit operator becomes the all-zeros or
      // all-ones mask
      auto moff = [&](uint8_t cls, uint16_t idx) -> uint16_t {
        if (cls == C_K) return (d.batch_consts[bp.const_off + idx] & 1) ? 8 : 0;
        return off(cls, idx);
      };
      const uint8_t op = in.op;
      if (op == I_LDREG || op == I_LDIN || (op >= K_LDREG_B && op <= K_LDB_BATCH)) { in.dst = off(cd, in.dst); }
      else if (op == I_MEMRD) { in.dst = off(cd, in.dst); in.a = off(ca, in.a); }
      else if (op == I_STREG || op == I_STOUT) { in.a = off(ca, in.a); }
      else if (op == I_WPORT) { in.a = off(ca, in.a); in.b = off(cb, in.b); in.c = off(cc, in.c); }
      else {
        const bool bk_a = ca == C_B || ca == C_K, bk_b = cb == C_B || cb == C_K, bk_c = cc == C_B || cc == C_K;
        // a constant whose whole value is 0 or 1 (where more than bit 0 of
        // the operand decides the result)
        auto bit_k = [&](uint8_t cls, uint16_t idx) {
          return cls == C_B || (cls == C_K && d.batch_consts[bp.const_off + idx] <= 1);
        };
        // 1-bit results of 1-bit operands: a product is an AND; a shift by a
        // 1-bit amount keeps a only when the amount is 0 (a AND NOT b; a
        // right shift needs all of a to be bit 0, a left shift only bit 0)
        const bool mask_ok = cd == C_B &&
            (((op == I_AND || op == I_OR || op == I_XOR || op == I_ADD || op == I_SUB || op == I_MUL) && bk_a &&
              bk_b) ||
             (op == I_NOT && bk_a) ||
             ((op == I_EQ || op == I_LT) && bit_k(ca, in.a) && bit_k(cb, in.b)) ||
             (op == I_SHL && bk_a && bit_k(cb, in.b)) ||
             (op == I_SHR && bit_k(ca, in.a) && bit_k(cb, in.b)) ||
             (op == I_MUX && ca == C_B && bk_b && bk_c));
        if (mask_ok) {
          in.op = (op == I_AND || op == I_MUL) ? K_MASK_AND : op == I_OR ? K_MASK_OR
                : (op == I_XOR || op == I_ADD || op == I_SUB) ? K_MASK_XOR
                : op == I_NOT ? K_MASK_NOT : op == I_EQ ? K_MASK_EQ
                : (op == I_LT || op == I_SHL || op == I_SHR) ? K_MASK_LT : K_MASK_MUX;
          in.a = moff(ca, in.a); in.b = moff(cb, in.b); in.c = moff(cc, in.c);
          // NOT b AND a is the LT handler (NOT first operand AND second)
          if (op == I_SHL || op == I_SHR) std::swap(in.a, in.b);
          in.dst = off(C_B, in.dst);
        } else {
          in.a = off(ca, in.a); in.b = off(cb, in.b); in.c = off(cc, in.c);
          in.dst = off(cd, in.dst);
        }
      }
    }
  }
  // processes by LDS need (each process's stream, constants and layout are
  // its own, so their order is free), and the split point
  {
    std::vector<uint32_t> ord(d.P);
    std::iota(ord.begin(), ord.end(), 0u);
    std::stable_sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) { return wave_bytes_of[a] < wave_bytes_of[b]; });
    std::vector<BatchProc> sorted(d.P);
    d.batch_need.assign(d.P, 0);
    for (uint32_t i = 0; i < d.P; ++i) {
      sorted[i] = d.batch_procs[ord[i]];
      d.batch_need[i] = wave_bytes_of[ord[i]];
    }
    d.batch_procs.swap(sorted);
  }
  if (getenv("FSIM_VERBOSE") && !wave_bytes_of.empty()) {
    std::sort(wave_bytes_of.begin(), wave_bytes_of.end());
    const size_t n = wave_bytes_of.size();
    fprintf(stderr, "fsim compile: batched LDS bytes per wave: p50 %u p90 %u p99 %u max %u\n", wave_bytes_of[n / 2],
            wave_bytes_of[n * 9 / 10], wave_bytes_of[n * 99 / 100], wave_bytes_of.back());
  }
  if (getenv("FSIM_VERBOSE")) {
    std::map<uint32_t, uint64_t> kinds;
    for (const Instr& in : d.batch_instr) {
      uint32_t k = in.op;
      if (in.op >= I_AND && in.op <= I_MUL) k = 1000 + (uint32_t)in.cls;    // per-lane operator by classes
      kinds[k]++;
    }
    std::vector<std::pair<uint64_t, uint32_t>> v;
    for (auto& kv : kinds) v.push_back({kv.second, kv.first});
    std::sort(v.rbegin(), v.rend());
    fprintf(stderr, "fsim compile: batched instructions %zu; top kinds:", d.batch_instr.size());
    for (size_t i = 0; i < v.size() && i < 24; ++i) {
      if (v[i].second >= 1000) {
        const uint32_t c = v[i].second - 1000;
        fprintf(stderr, " alu[%c%c%c>%c]=%llu", "BWDK"[(c >> 2) & 3], "BWDK"[(c >> 4) & 3], "BWDK"[c >> 6],
                "BWDK"[c & 3], (unsigned long long)v[i].first);
      } else {
        fprintf(stderr, " op%u=%llu", v[i].second, (unsigned long long)v[i].first);
      }
    }
    fprintf(stderr, "\n");
  }
  // one trailing instruction: the kernel fetches instruction i + 1 while it
  // executes instruction i
  d.batch_instr.push_back(Instr{});
  d.batch_encoded = true;
  return {};
}

}  // namespace fsim
