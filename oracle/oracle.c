/*
 * oracle.c -- plain, single-threaded CPU reference simulator.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * GPU library; it has its own netlist reader (the orc_netlist struct below,
 * filled from plain arrays) and its own stimulus hash.
 *
 * What it computes (Parendi, Sec. 3 "Parallel RTL Simulation"):
 *   - cycle-accurate, zero-delay, full-cycle simulation: the whole circuit is
 *     evaluated every cycle, no activity tracking (Sec. 3, opening paragraphs);
 *   - the data-dependence-graph view of Sec. 3.2: every register is split into
 *     a read-only "current" value and a write-only "next" value, and the
 *     stateless combinational nodes between them are evaluated from the
 *     current values only.  All registers then take their next values at
 *     once (the BSP exchange of Sec. 3.2 reduces to this simultaneous update);
 *   - a fiber (Sec. 3.2, last paragraphs) is the set of nodes that produces one
 *     register's next value; Sec. 5.1 finds it by walking the graph backwards
 *     from each sink.  orc_step_partitioned() evaluates each fiber or each
 *     group of fibers (a BSP process) on its own, with a fresh value table,
 *     which is how the paper's processes run.  Its result must equal the
 *     monolithic evaluation of orc_step() for any partition.
 *
 * The method (fibers + packing + BSP) reaches exactly the result of plain
 * sequential evaluation, so this file is that plain definition written out:
 *
 *   per cycle t:
 *     I_t[p]  = mask(w_p, stim(seed, p, t))       (or explicit input values)
 *     for every combinational node n in a topological order:
 *         v[n] = mask(w_n, f_op(v[args]))
 *         leaves: REG -> R[r], INPUT -> I_t[p], CONST -> imm,
 *                 MEMRD -> M[m][v[addr] mod depth]   (reads see M_t)
 *     R'[r]   = mask(w_r, v[reg_next[r]])         (all registers at once)
 *               if r has no enable or v[reg_en[r]] != 0, else R[r]
 *     O_t[o]  = v[out_node[o]]
 *     for write port k in index order:             (after every read)
 *         if v[en_k] != 0: M[m_k][v[addr_k] mod depth] = mask(w_m, v[data_k])
 *     R = R'; t = t + 1
 *     digest_t = sum_r H(r xor H(R[r]))  mod 2^64
 *
 * Readings where the paper is silent (the paper works on Verilator's AST and
 * gives no word-level operator table):
 *   - unsigned Verilog-like operators on operands zero-extended to 64 bits,
 *     result masked to the node width; shift amounts >= 64 give 0, as a
 *     Verilog shift by more than the operand width does;
 *   - memory reads see the state at the start of the cycle; writes commit at
 *     the end of the cycle in port order, so the highest port index wins when
 *     two enabled ports hit one address; addresses wrap modulo the depth;
 *   - gated and divided clocks (Sec. 5.3, Limitations: one top clock plus
 *     any number of gated or divided ones) are modelled as a per-register
 *     enable of the top clock: in a cycle where the enable node is zero the
 *     register keeps its value.  A divided clock is a gate driven by the
 *     divider's own state; the design builds that logic from ordinary nodes;
 *   - the on-device test driver of Sec. 5.3 (Limitations) is modelled as a
 *     counter-based stimulus stim = H(H(H(seed) xor p) xor t), H being the
 *     SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>

/* ---- opcodes (the netlist interchange format; the GPU library defines the
 *      same numbering independently because it is a file format) ---------- */
enum {
  ORC_CONST = 0, ORC_INPUT = 1, ORC_REG = 2, ORC_MEMRD = 3,
  ORC_AND = 4, ORC_OR = 5, ORC_XOR = 6, ORC_NOT = 7, ORC_ADD = 8, ORC_SUB = 9,
  ORC_MUX = 10, ORC_SHL = 11, ORC_SHR = 12, ORC_EQ = 13, ORC_LT = 14,
  ORC_MUL = 15, ORC_NUM_OPS = 16
};

enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_NETLIST = -2, ORC_E_COMB_LOOP = -3,
       ORC_E_UNSUPPORTED = -4, ORC_E_CONE = -5 };

#define ORC_NONE 0xFFFFFFFFu

typedef struct {
  uint32_t n_nodes;
  const uint8_t *op, *width;
  const uint32_t *arg;          /* [n_nodes][3] */
  const uint64_t *imm;
  uint32_t n_regs;
  const uint8_t *reg_width;
  const uint64_t *reg_init;
  const uint32_t *reg_next;
  uint32_t n_inputs;
  const uint8_t *in_width;
  uint32_t n_outputs;
  const uint32_t *out_node;
  uint32_t n_mems;
  const uint32_t *mem_depth;
  const uint8_t *mem_width;
  const uint64_t *mem_init;     /* all memories back to back, mem 0 first */
  uint32_t n_wports;
  const uint32_t *wp_mem, *wp_en, *wp_addr, *wp_data;
  const uint32_t *reg_en;       /* NULL, or per register a node / ORC_NONE */
} orc_netlist;

/* ---------------------------------------------------------------- helpers */

static uint64_t mask_w(unsigned w, uint64_t x) {
  return x & (~0ull >> (64u - w));        /* w in 1..64: no shift by 64 */
}

/* SplitMix64 output function applied to x (the first output of a SplitMix64
 * generator whose state is x): add the golden gamma, then the variant-13
 * finaliser with shifts 30/27/31 (Steele, Lea and Flood, OOPSLA 2014; the
 * constants are the published ones). */
uint64_t orc_hash(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t orc_stim(uint64_t seed, uint32_t port, uint64_t t) {
  return orc_hash(orc_hash(orc_hash(seed) ^ (uint64_t)port) ^ t);
}

static int arity(unsigned op) {
  switch (op) {
    case ORC_CONST: case ORC_INPUT: case ORC_REG: return 0;
    case ORC_MEMRD: case ORC_NOT: return 1;
    case ORC_MUX: return 3;
    default: return 2;
  }
}

/* One combinational operator on operands that are already zero-extended. */
uint64_t orc_eval(uint32_t op, uint32_t w, uint64_t a, uint64_t b, uint64_t c) {
  uint64_t r;
  switch (op) {
    case ORC_AND: r = a & b; break;
    case ORC_OR:  r = a | b; break;
    case ORC_XOR: r = a ^ b; break;
    case ORC_NOT: r = ~a; break;
    case ORC_ADD: r = a + b; break;           /* mod 2^64 */
    case ORC_SUB: r = a - b; break;           /* mod 2^64 */
    case ORC_MUX: r = (a != 0) ? b : c; break; /* MUX(sel, x, y) */
    case ORC_SHL: r = (b >= 64) ? 0 : (a << b); break;
    case ORC_SHR: r = (b >= 64) ? 0 : (a >> b); break;
    case ORC_EQ:  r = (a == b) ? 1 : 0; break;
    case ORC_LT:  r = (a < b) ? 1 : 0; break;
    case ORC_MUL: r = a * b; break;           /* low 64 bits */
    default: r = 0; break;
  }
  return mask_w(w, r);
}

/* ------------------------------------------------------------- simulator */

typedef struct {
  orc_netlist nl;               /* private copies of every array */
  uint32_t *topo;               /* combinational nodes, topological order */
  uint32_t n_topo;
  uint64_t *mem_off;            /* start of memory m in mem */
  uint64_t *R, *Rn, *O, *M, *v, *I;
  uint64_t seed, cycle;
  /* explicit input window: vals[(t - in_first) * n_inputs + p] */
  uint64_t *in_vals, in_first, in_count;
  int explicit_inputs;
} orc_sim;

static void *dup(const void *p, size_t bytes) {
  if (bytes == 0) return calloc(1, 8);
  void *q = malloc(bytes);
  if (q && p) memcpy(q, p, bytes); else if (q) memset(q, 0, bytes);
  return q;
}

static int validate(const orc_netlist *nl) {
  for (uint32_t n = 0; n < nl->n_nodes; ++n) {
    unsigned op = nl->op[n], w = nl->width[n];
    if (op >= ORC_NUM_OPS) return ORC_E_UNSUPPORTED;
    if (w < 1 || w > 64) return w > 64 ? ORC_E_UNSUPPORTED : ORC_E_NETLIST;
    for (int k = 0; k < arity(op); ++k)
      if (nl->arg[3 * n + k] >= nl->n_nodes) return ORC_E_NETLIST;
    if (op == ORC_INPUT && nl->imm[n] >= nl->n_inputs) return ORC_E_NETLIST;
    if (op == ORC_REG && nl->imm[n] >= nl->n_regs) return ORC_E_NETLIST;
    if (op == ORC_MEMRD && nl->imm[n] >= nl->n_mems) return ORC_E_NETLIST;
  }
  for (uint32_t r = 0; r < nl->n_regs; ++r) {
    if (nl->reg_width[r] < 1 || nl->reg_width[r] > 64) return ORC_E_NETLIST;
    if (nl->reg_next[r] >= nl->n_nodes) return ORC_E_NETLIST;
    if (nl->reg_en && nl->reg_en[r] != ORC_NONE && nl->reg_en[r] >= nl->n_nodes)
      return ORC_E_NETLIST;
  }
  for (uint32_t p = 0; p < nl->n_inputs; ++p)
    if (nl->in_width[p] < 1 || nl->in_width[p] > 64) return ORC_E_NETLIST;
  for (uint32_t o = 0; o < nl->n_outputs; ++o)
    if (nl->out_node[o] >= nl->n_nodes) return ORC_E_NETLIST;
  for (uint32_t m = 0; m < nl->n_mems; ++m)
    if (nl->mem_depth[m] == 0 || nl->mem_width[m] < 1 || nl->mem_width[m] > 64)
      return ORC_E_NETLIST;
  for (uint32_t k = 0; k < nl->n_wports; ++k)
    if (nl->wp_mem[k] >= nl->n_mems || nl->wp_en[k] >= nl->n_nodes ||
        nl->wp_addr[k] >= nl->n_nodes || nl->wp_data[k] >= nl->n_nodes)
      return ORC_E_NETLIST;
  return ORC_OK;
}

/* Kahn's algorithm over every node (leaves have no incoming edges).  With
 * order_seed != 0 the ready node is picked at random (a different, equally
 * valid order); with 0 it is a FIFO.  A node left unordered means a cycle. */
static int topo_sort(const orc_netlist *nl, uint64_t order_seed,
                     uint32_t *out, uint32_t *n_out) {
  uint32_t n = nl->n_nodes;
  uint32_t *indeg = calloc(n ? n : 1, sizeof(uint32_t));
  uint32_t *cnt = calloc(n + 1, sizeof(uint32_t));
  uint32_t *users = NULL, *ready = malloc((n ? n : 1) * sizeof(uint32_t));
  uint64_t edges = 0;
  for (uint32_t i = 0; i < n; ++i)
    for (int k = 0; k < arity(nl->op[i]); ++k) { cnt[nl->arg[3 * i + k]]++; edges++; }
  uint64_t *start = calloc(n + 1, sizeof(uint64_t));
  for (uint32_t i = 0; i < n; ++i) start[i + 1] = start[i] + cnt[i];
  users = malloc((edges ? edges : 1) * sizeof(uint32_t));
  memset(cnt, 0, (n + 1) * sizeof(uint32_t));
  for (uint32_t i = 0; i < n; ++i)
    for (int k = 0; k < arity(nl->op[i]); ++k) {
      uint32_t a = nl->arg[3 * i + k];
      users[start[a] + cnt[a]++] = i;
      indeg[i]++;
    }
  uint32_t head = 0, tail = 0, done = 0;
  for (uint32_t i = 0; i < n; ++i) if (indeg[i] == 0) ready[tail++] = i;
  uint64_t s = order_seed;
  while (head < tail) {
    if (order_seed) {                     /* random pick among ready nodes */
      s = orc_hash(s);
      uint32_t j = head + (uint32_t)(s % (tail - head));
      uint32_t t = ready[head]; ready[head] = ready[j]; ready[j] = t;
    }
    uint32_t x = ready[head++];
    out[done++] = x;
    for (uint64_t e = start[x]; e < start[x + 1]; ++e)
      if (--indeg[users[e]] == 0) ready[tail++] = users[e];
  }
  free(indeg); free(cnt); free(users); free(ready); free(start);
  *n_out = done;
  return done == n ? ORC_OK : ORC_E_COMB_LOOP;
}

void orc_free(orc_sim *s) {
  if (!s) return;
  free((void *)s->nl.op); free((void *)s->nl.width); free((void *)s->nl.arg);
  free((void *)s->nl.imm); free((void *)s->nl.reg_width);
  free((void *)s->nl.reg_init); free((void *)s->nl.reg_next);
  free((void *)s->nl.in_width); free((void *)s->nl.out_node);
  free((void *)s->nl.mem_depth); free((void *)s->nl.mem_width);
  free((void *)s->nl.mem_init); free((void *)s->nl.wp_mem);
  free((void *)s->nl.wp_en); free((void *)s->nl.wp_addr);
  free((void *)s->nl.wp_data); free((void *)s->nl.reg_en);
  free(s->topo); free(s->mem_off); free(s->R); free(s->Rn); free(s->O);
  free(s->M); free(s->v); free(s->I); free(s->in_vals);
  free(s);
}

/* Copies the netlist, validates it, orders it and resets the state. */
int orc_new(const orc_netlist *src, uint64_t order_seed, orc_sim **out) {
  if (!src || !out) return ORC_E_ARG;
  *out = NULL;
  int rc = validate(src);
  if (rc) return rc;
  orc_sim *s = calloc(1, sizeof(orc_sim));
  orc_netlist *nl = &s->nl;
  *nl = *src;
  uint32_t n = src->n_nodes;
  nl->op = dup(src->op, n);
  nl->width = dup(src->width, n);
  nl->arg = dup(src->arg, 3ull * n * 4);
  nl->imm = dup(src->imm, 8ull * n);
  nl->reg_width = dup(src->reg_width, src->n_regs);
  nl->reg_init = dup(src->reg_init, 8ull * src->n_regs);
  nl->reg_next = dup(src->reg_next, 4ull * src->n_regs);
  nl->in_width = dup(src->in_width, src->n_inputs);
  nl->out_node = dup(src->out_node, 4ull * src->n_outputs);
  nl->mem_depth = dup(src->mem_depth, 4ull * src->n_mems);
  nl->mem_width = dup(src->mem_width, src->n_mems);
  uint64_t total = 0;
  s->mem_off = calloc(src->n_mems + 1, sizeof(uint64_t));
  for (uint32_t m = 0; m < src->n_mems; ++m) {
    s->mem_off[m] = total;
    total += src->mem_depth[m];
  }
  s->mem_off[src->n_mems] = total;
  nl->mem_init = dup(src->mem_init, 8ull * total);
  nl->wp_mem = dup(src->wp_mem, 4ull * src->n_wports);
  nl->wp_en = dup(src->wp_en, 4ull * src->n_wports);
  nl->wp_addr = dup(src->wp_addr, 4ull * src->n_wports);
  nl->wp_data = dup(src->wp_data, 4ull * src->n_wports);
  nl->reg_en = src->reg_en ? dup(src->reg_en, 4ull * src->n_regs) : NULL;
  s->topo = malloc((n ? n : 1) * sizeof(uint32_t));
  rc = topo_sort(nl, order_seed, s->topo, &s->n_topo);
  if (rc) { orc_free(s); return rc; }
  s->R = calloc(src->n_regs + 1, 8);
  s->Rn = calloc(src->n_regs + 1, 8);
  s->O = calloc(src->n_outputs + 1, 8);
  s->M = calloc(total + 1, 8);
  s->v = calloc(n + 1, 8);
  s->I = calloc(src->n_inputs + 1, 8);
  for (uint32_t r = 0; r < src->n_regs; ++r)
    s->R[r] = mask_w(nl->reg_width[r], nl->reg_init[r]);
  for (uint32_t m = 0; m < src->n_mems; ++m)
    for (uint32_t a = 0; a < src->mem_depth[m]; ++a)
      s->M[s->mem_off[m] + a] = src->mem_init
          ? mask_w(nl->mem_width[m], nl->mem_init[s->mem_off[m] + a]) : 0;
  *out = s;
  return ORC_OK;
}

void orc_set_seed(orc_sim *s, uint64_t seed) { s->seed = seed; s->explicit_inputs = 0; }

/* Explicit mode: vals[(t - first) * n_inputs + p] for t in [first, first+n). */
int orc_set_inputs(orc_sim *s, uint64_t first, uint64_t n, const uint64_t *vals) {
  free(s->in_vals);
  s->in_vals = dup(vals, 8ull * n * s->nl.n_inputs);
  s->in_first = first; s->in_count = n; s->explicit_inputs = 1;
  return ORC_OK;
}

static int load_inputs(orc_sim *s) {
  const orc_netlist *nl = &s->nl;
  for (uint32_t p = 0; p < nl->n_inputs; ++p) {
    uint64_t x;
    if (s->explicit_inputs) {
      if (s->cycle < s->in_first || s->cycle >= s->in_first + s->in_count)
        return ORC_E_ARG;
      x = s->in_vals[(s->cycle - s->in_first) * nl->n_inputs + p];
    } else {
      x = orc_stim(s->seed, p, s->cycle);
    }
    s->I[p] = mask_w(nl->in_width[p], x);
  }
  return ORC_OK;
}

/* Value of node n given a value table that already holds every operand. */
static uint64_t node_value(const orc_sim *s, const uint64_t *v, uint32_t n) {
  const orc_netlist *nl = &s->nl;
  unsigned op = nl->op[n], w = nl->width[n];
  const uint32_t *a = &nl->arg[3 * n];
  switch (op) {
    case ORC_CONST: return mask_w(w, nl->imm[n]);
    case ORC_INPUT: return mask_w(w, s->I[nl->imm[n]]);
    case ORC_REG:   return mask_w(w, s->R[nl->imm[n]]);
    case ORC_MEMRD: {
      uint32_t m = (uint32_t)nl->imm[n];
      uint64_t addr = v[a[0]] % nl->mem_depth[m];
      return mask_w(w, s->M[s->mem_off[m] + addr]);
    }
    case ORC_NOT: return orc_eval(op, w, v[a[0]], 0, 0);
    case ORC_MUX: return orc_eval(op, w, v[a[0]], v[a[1]], v[a[2]]);
    default:      return orc_eval(op, w, v[a[0]], v[a[1]], 0);
  }
}

static uint64_t digest(const orc_sim *s) {
  uint64_t d = 0;
  for (uint32_t r = 0; r < s->nl.n_regs; ++r)
    d += orc_hash((uint64_t)r ^ orc_hash(s->R[r]));
  return d;
}

uint64_t orc_digest(const orc_sim *s) { return digest(s); }

/* Whether register r's clock ticks this cycle (Sec. 5.3: a gated or divided
 * clock is the top clock with an enable). */
static int clock_enabled(const orc_netlist *nl, uint32_t r, const uint64_t *v) {
  uint32_t e = nl->reg_en ? nl->reg_en[r] : ORC_NONE;
  return e == ORC_NONE || v[e] != 0;
}

/* Register update, outputs and memory commit from a complete value table. */
static void end_of_cycle(orc_sim *s, const uint64_t *v) {
  const orc_netlist *nl = &s->nl;
  for (uint32_t r = 0; r < nl->n_regs; ++r)
    s->Rn[r] = clock_enabled(nl, r, v)
        ? mask_w(nl->reg_width[r], v[nl->reg_next[r]]) : s->R[r];
  for (uint32_t o = 0; o < nl->n_outputs; ++o) s->O[o] = v[nl->out_node[o]];
  for (uint32_t k = 0; k < nl->n_wports; ++k) {
    if (v[nl->wp_en[k]] == 0) continue;
    uint32_t m = nl->wp_mem[k];
    uint64_t addr = v[nl->wp_addr[k]] % nl->mem_depth[m];
    s->M[s->mem_off[m] + addr] = mask_w(nl->mem_width[m], v[nl->wp_data[k]]);
  }
  uint64_t *t = s->R; s->R = s->Rn; s->Rn = t;
  s->cycle++;
}

/* Monolithic evaluation: every node, in topological order, every cycle.
 * digests (nullable) receives the digest of R after each cycle. */
int orc_step(orc_sim *s, uint64_t n_cycles, uint64_t *digests) {
  for (uint64_t c = 0; c < n_cycles; ++c) {
    int rc = load_inputs(s);
    if (rc) return rc;
    for (uint32_t i = 0; i < s->n_topo; ++i) {
      uint32_t n = s->topo[i];
      s->v[n] = node_value(s, s->v, n);
    }
    end_of_cycle(s, s->v);
    if (digests) digests[c] = digest(s);
  }
  return ORC_OK;
}

/* ---------------------------------------------------- partitioned (BSP) mode
 * Sinks are numbered: registers 0..R-1, then write ports R..R+W-1, then
 * outputs R+W..R+W+O-1 (one write port -- en, addr and data -- is one sink).
 * sink_to_proc[s] names the process that produces sink s.  Each process
 * evaluates only the nodes it is given:
 *   - node lists NULL: the union of the cones of its sinks, found here by a
 *     reverse crawl from each sink (Sec. 5.1);
 *   - node lists given (proc_off / proc_nodes, CSR form): exactly those
 *     nodes, so that a partition computed elsewhere can be checked; a node
 *     whose operand is not in the list fails with ORC_E_CONE.
 * Each process starts from a fresh value table and sees only R_t, M_t, I_t,
 * so nothing computed by another process can leak in. */

static int cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return x < y ? -1 : x > y;
}

typedef struct {
  uint32_t n_proc;
  uint32_t *off;                /* [n_proc + 1] */
  uint32_t *nodes;              /* per process, topological order */
} orc_plan;

static uint32_t sink_node_list(const orc_netlist *nl, uint32_t sink,
                               uint32_t *roots) {
  uint32_t R = nl->n_regs, W = nl->n_wports;
  if (sink < R) {
    /* a register's fiber also produces its clock enable, if it has one */
    roots[0] = nl->reg_next[sink];
    if (nl->reg_en && nl->reg_en[sink] != ORC_NONE) { roots[1] = nl->reg_en[sink]; return 2; }
    return 1;
  }
  if (sink < R + W) {
    uint32_t k = sink - R;
    roots[0] = nl->wp_en[k]; roots[1] = nl->wp_addr[k]; roots[2] = nl->wp_data[k];
    return 3;
  }
  roots[0] = nl->out_node[sink - R - W];
  return 1;
}

int orc_step_partitioned(orc_sim *s, uint64_t n_cycles, uint32_t n_proc,
                         const uint32_t *sink_to_proc,
                         const uint32_t *proc_off, const uint32_t *proc_nodes,
                         uint64_t *digests) {
  const orc_netlist *nl = &s->nl;
  uint32_t n = nl->n_nodes;
  uint32_t n_sinks = nl->n_regs + nl->n_wports + nl->n_outputs;
  for (uint32_t k = 0; k < n_sinks; ++k)
    if (sink_to_proc[k] >= n_proc) return ORC_E_ARG;
  /* position of every node in the global topological order */
  uint32_t *pos = malloc((n ? n : 1) * sizeof(uint32_t));
  for (uint32_t i = 0; i < s->n_topo; ++i) pos[s->topo[i]] = i;
  orc_plan plan = {n_proc, calloc(n_proc + 1, 4), NULL};
  uint8_t *in_proc = calloc(n ? n : 1, 1);
  uint32_t *stack = malloc((n ? n : 1) * sizeof(uint32_t));
  /* sinks grouped by process */
  uint32_t *sk_off = calloc(n_proc + 1, 4), *sk = malloc((n_sinks ? n_sinks : 1) * 4);
  for (uint32_t k = 0; k < n_sinks; ++k) sk_off[sink_to_proc[k] + 1]++;
  for (uint32_t p = 0; p < n_proc; ++p) sk_off[p + 1] += sk_off[p];
  {
    uint32_t *fill = calloc(n_proc + 1, 4);
    for (uint32_t k = 0; k < n_sinks; ++k) {
      uint32_t p = sink_to_proc[k];
      sk[sk_off[p] + fill[p]++] = k;
    }
    free(fill);
  }
  int rc = ORC_OK;
  if (proc_off) {
    for (uint32_t p = 0; p <= n_proc; ++p) plan.off[p] = proc_off[p];
    uint32_t tot = proc_off[n_proc];
    plan.nodes = malloc((tot ? tot : 1) * 4);
    for (uint32_t i = 0; i < tot; ++i) {
      if (proc_nodes[i] >= n) { rc = ORC_E_ARG; break; }
      plan.nodes[i] = proc_nodes[i];
    }
  } else {
    /* reverse crawl per process; collect, then sort by topological position */
    uint64_t cap = 1024, used = 0;
    plan.nodes = malloc(cap * 4);
    for (uint32_t p = 0; p < n_proc; ++p) {
      plan.off[p] = (uint32_t)used;
      uint32_t sp = 0, first = (uint32_t)used;
      for (uint32_t j = sk_off[p]; j < sk_off[p + 1]; ++j) {
        uint32_t roots[3], nr = sink_node_list(nl, sk[j], roots);
        for (uint32_t q = 0; q < nr; ++q)
          if (!in_proc[roots[q]]) { in_proc[roots[q]] = 1; stack[sp++] = roots[q]; }
        while (sp) {
          uint32_t x = stack[--sp];
          if (used == cap) { cap *= 2; plan.nodes = realloc(plan.nodes, cap * 4); }
          plan.nodes[used++] = x;
          for (int a = 0; a < arity(nl->op[x]); ++a) {
            uint32_t y = nl->arg[3 * x + a];
            if (!in_proc[y]) { in_proc[y] = 1; stack[sp++] = y; }
          }
        }
      }
      for (uint32_t i = first; i < used; ++i) in_proc[plan.nodes[i]] = 0;
    }
    plan.off[n_proc] = (uint32_t)used;
  }
  /* order every process's list by the global topological position */
  if (rc == ORC_OK) {
    uint32_t tot = plan.off[n_proc];
    uint64_t *key = malloc((tot ? tot : 1) * 8);
    for (uint32_t p = 0; p < n_proc && rc == ORC_OK; ++p) {
      uint32_t lo = plan.off[p], hi = plan.off[p + 1];
      for (uint32_t i = lo; i < hi; ++i)
        key[i] = ((uint64_t)pos[plan.nodes[i]] << 32) | plan.nodes[i];
      qsort(key + lo, hi - lo, 8, cmp_u64);
      for (uint32_t i = lo; i < hi; ++i) {
        plan.nodes[i] = (uint32_t)key[i];
        if (i > lo && plan.nodes[i] == plan.nodes[i - 1]) rc = ORC_E_ARG;  /* duplicate */
      }
    }
    free(key);
  }
  /* evaluate */
  uint64_t *v = calloc(n + 1, 8);
  uint8_t *have = calloc(n ? n : 1, 1);
  uint64_t *Rn = calloc(nl->n_regs + 1, 8);
  uint64_t *On = calloc(nl->n_outputs + 1, 8);
  uint8_t *wen = calloc(nl->n_wports + 1, 1);
  uint64_t *waddr = calloc(nl->n_wports + 1, 8), *wdata = calloc(nl->n_wports + 1, 8);
  for (uint64_t c = 0; c < n_cycles && rc == ORC_OK; ++c) {
    rc = load_inputs(s);
    for (uint32_t p = 0; p < n_proc && rc == ORC_OK; ++p) {
      uint32_t lo = plan.off[p], hi = plan.off[p + 1];
      for (uint32_t i = lo; i < hi && rc == ORC_OK; ++i) {
        uint32_t x = plan.nodes[i];
        for (int a = 0; a < arity(nl->op[x]); ++a)
          if (!have[nl->arg[3 * x + a]]) { rc = ORC_E_CONE; break; }
        if (rc) break;
        v[x] = node_value(s, v, x);
        have[x] = 1;
      }
      for (uint32_t j = sk_off[p]; j < sk_off[p + 1] && rc == ORC_OK; ++j) {
        uint32_t k = sk[j], roots[3], nr = sink_node_list(nl, k, roots);
        for (uint32_t q = 0; q < nr; ++q) if (!have[roots[q]]) rc = ORC_E_CONE;
        if (rc) break;
        if (k < nl->n_regs)
          Rn[k] = clock_enabled(nl, k, v) ? mask_w(nl->reg_width[k], v[roots[0]]) : s->R[k];
        else if (k < nl->n_regs + nl->n_wports) {
          uint32_t q = k - nl->n_regs;
          wen[q] = v[roots[0]] != 0; waddr[q] = v[roots[1]]; wdata[q] = v[roots[2]];
        } else On[k - nl->n_regs - nl->n_wports] = v[roots[0]];
      }
      /* fresh table for the next process */
      for (uint32_t i = lo; i < hi; ++i) { have[plan.nodes[i]] = 0; v[plan.nodes[i]] = 0; }
    }
    if (rc) break;
    /* exchange: all next values become current at once; memories commit
     * after every process has read them, in port order */
    for (uint32_t r = 0; r < nl->n_regs; ++r) s->R[r] = Rn[r];
    for (uint32_t o = 0; o < nl->n_outputs; ++o) s->O[o] = On[o];
    for (uint32_t q = 0; q < nl->n_wports; ++q) {
      if (!wen[q]) continue;
      uint32_t m = nl->wp_mem[q];
      s->M[s->mem_off[m] + waddr[q] % nl->mem_depth[m]] = mask_w(nl->mem_width[m], wdata[q]);
    }
    s->cycle++;
    if (digests) digests[c] = digest(s);
  }
  free(v); free(have); free(Rn); free(On); free(wen); free(waddr); free(wdata);
  free(pos); free(plan.off); free(plan.nodes); free(in_proc); free(stack);
  free(sk_off); free(sk);
  return rc;
}

/* ---------------------------------------------------------- state access */
uint64_t orc_cycle(const orc_sim *s) { return s->cycle; }
void orc_read_regs(const orc_sim *s, uint64_t *out) {
  memcpy(out, s->R, 8ull * s->nl.n_regs);
}
void orc_write_regs(orc_sim *s, const uint64_t *in) {
  for (uint32_t r = 0; r < s->nl.n_regs; ++r)
    s->R[r] = mask_w(s->nl.reg_width[r], in[r]);
}
void orc_read_outputs(const orc_sim *s, uint64_t *out) {
  memcpy(out, s->O, 8ull * s->nl.n_outputs);
}
int orc_read_mem(const orc_sim *s, uint32_t m, uint64_t *out) {
  if (m >= s->nl.n_mems) return ORC_E_ARG;
  memcpy(out, s->M + s->mem_off[m], 8ull * s->nl.mem_depth[m]);
  return ORC_OK;
}
int orc_write_mem(orc_sim *s, uint32_t m, const uint64_t *in) {
  if (m >= s->nl.n_mems) return ORC_E_ARG;
  for (uint32_t a = 0; a < s->nl.mem_depth[m]; ++a)
    s->M[s->mem_off[m] + a] = mask_w(s->nl.mem_width[m], in[a]);
  return ORC_OK;
}
void orc_set_cycle(orc_sim *s, uint64_t c) { s->cycle = c; }
