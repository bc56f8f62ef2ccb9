// Host-callable launchers of the device kernels, and the parameter blocks
// they take.  Internal to the library.
#pragma once

#include "dev_common.h"

// The dynamic graph as the kernels see it (internal, label-grouped ids).
// Rows: with edge labels, vertex v has one row per edge label e, row id
// (v << elb) | e, holding its neighbours through edges of label e (sorted by
// internal id).  Without edge labels elb = 0 and the row id is v.
struct GmGraphDev {
  uint32_t n;
  int32_t idbits;                 // bits needed for an id < n
  uint64_t* row_off;              // [n << elb]
  uint32_t* row_len;              // [n << elb]
  uint32_t* col;                  // arena; bit 31 marks batch entries
  uint32_t* ext;                  // parallel arena: external id of each col entry
  const uint16_t* vlabel;         // [n]
  const uint32_t* label_start;    // [label_slots + 1]
  uint32_t label_slots;           // labels >= label_slots occur nowhere
  const uint32_t* new_of_old;     // [n] external -> internal
  const uint32_t* old_of_new;     // [n] internal -> external
  uint32_t elb;                   // edge-label bits of a row id (0: no edge labels)
  uint32_t n_el;                  // edge labels are < n_el (1: no edge labels)
};

// The batch hash: undirected internal edge key -> ord << 1 | sign.
struct GmBatchHash {
  uint64_t* keys;
  uint32_t* vals;
  uint32_t mask;
};

// Device counters of one batch (zeroed before each batch).
struct GmCounters {
  uint32_t err;
  uint32_t n_dup;
  uint32_t n_noop;
  uint32_t pad;
  unsigned long long n_seeds;
  unsigned long long seed_head;
  unsigned long long tuples_found;
  unsigned long long dfs_nodes;
  unsigned long long cand_scanned;
  unsigned long long bytes_alg;
  unsigned long long steals;
  unsigned long long bytes_update;
  unsigned long long cyc[6];      // idle, init, inner, leaf, hand-over cycles; tasks received
  unsigned long long pending;     // work items taken or handed over and not finished
  unsigned int aborted;           // set when a wave passed the deadline; every wave of the launch then exits
  unsigned int timed_out;         // some search launch of the batch passed its deadline (sticky)
  unsigned long long seed_begin;  // first seed of the current search launch (seeds [seed_begin, n_seeds))
  unsigned long long t_start;     // device wall clock when the current search launch began (deadline origin)
};

constexpr uint32_t GM_NO_GROUP = 0xFFFFFFFFu;
struct GmGroupList {
  unsigned long long base;  // arena index of the list's first entry
  uint32_t len;             // entries (GM_NO_GROUP: none)
  uint32_t pad;
};

struct GmDfsParams {
  GmGraphDev G;
  const unsigned long long* lix;  // [rows][lix_slots]: label subrange of each row, start | len << 32
  uint32_t lix_slots;
  const GmPlan* plans;
  const GmQueryDev* queries;
  const uint16_t* cand;           // [nq][n]
  const GmSeed* seeds;
  GmBatchHash H;
  GmCounters* ctr;
  uint32_t flags;
  uint32_t twidth;
  unsigned long long* qres;       // [nq][2][3]: count, hash sum, hash xor
  uint32_t* tuples;
  uint32_t* tmeta;
  uint32_t* tord;
  uint64_t tcap;
  unsigned long long* upd_res;    // [n_canon][3]
  // work hand-over between waves (one mailbox per wave slot)
  uint32_t* mbox;                 // [n_slots][32] task records
  uint32_t* mflag;                // [n_slots] 1 = a task waits in the mailbox
  unsigned long long* idle_bits;  // [ceil(n_slots / 64)] bit set = the wave waits for work
  uint32_t* idle_rep;             // [8 x 32] count of idle waves in 8 copies, 128 B apart (a polling hint)
  uint32_t n_slots;
  uint32_t donate;                // 0 = no hand-over (each wave keeps its seed)
  uint64_t deadline_ticks;        // wall-clock ticks a wave may search (0 = no deadline)
  uint32_t poll_cycles;           // shader cycles between a busy wave's hand-over polls
  uint32_t split_inner;           // smallest inner-level range worth handing over
  uint32_t split_leaf;            // smallest last-level range worth handing over
  uint32_t gate;                  // hand-over attempt probability per idle wave, in 1/1024
  const GmPerm* perms;            // coalesced search: permutation table referenced by plans
  uint32_t coalesce;              // 1: search representative plans only and permute their matches;
                                  // 2: also permute core prefixes (plans with n_cperm >= 2)
  uint32_t shared_leaf;           // 1: a last level that does not depend on level k-2 is walked
                                  // once per level-(k-2) chunk for all its survivors
  uint32_t reenter;               // 1: an inner level that does not depend on the level before
                                  // it keeps its set-up from one survivor of that level to the next
  const uint8_t* qel;             // [nq][16][16] edge label of query edge {u, w} (used when G.elb > 0)
  // per seed, its work items not yet finished (the seed's own item plus one
  // per hand-over of its work); 0xFFFFFFFF = not started.  NULL: untracked.
  // A seed at 0 when the search ends (also past a deadline) is complete.
  uint32_t* seed_open;
  // Update-edge grouping (seeds sharing query, directed query edge and
  // first data vertex a): per seed its group, per group the arena range of
  // a's level-2 candidates, already filtered by the candidate table (len
  // GM_NO_GROUP: level 2 is set up as usual).  NULL: no grouping.
  const uint32_t* seed_group;
  const GmGroupList* group_list;
};

namespace gm {

// graph (k_graph.hip)
void launch_validate_csr(const uint64_t* rp, const uint32_t* col, const uint32_t* labels, const uint32_t* elab,
                         uint32_t n_el, uint32_t n, uint64_t nnz, uint32_t* err, hipStream_t s);
void launch_relabel_keys(const uint32_t* labels, uint32_t n, uint64_t* keys, hipStream_t s);
void launch_relabel_apply(const uint64_t* sorted, uint32_t n, uint32_t* new_of_old,
                          uint32_t* old_of_new, uint16_t* vlabel, hipStream_t s);
void launch_label_start(const uint16_t* vlabel, uint32_t n, uint32_t slots, uint32_t* label_start,
                        hipStream_t s);
// elab (per CSR entry, with elb > 0): the source part becomes the row id map[v] << elb | label
void launch_csr_keys(const uint64_t* row_off, const uint32_t* row_len, const uint64_t* rp,
                     const uint32_t* col, const uint32_t* map, uint32_t n, int idbits,
                     const uint64_t* out_off, uint64_t* keys, hipStream_t s, const uint32_t* elab = nullptr,
                     uint32_t elb = 0);
// row lengths from sorted (row << idbits | neighbour) keys; deg zeroed by the caller
void launch_row_hist(const uint64_t* keys, uint64_t nnz, int idbits, uint64_t* deg, hipStream_t s);
// labelled export: keys old[v] << (idbits + elb) | old[w] << elb | e per row entry, and their split
void launch_row_keys_el(const uint64_t* row_off, const uint32_t* row_len, const uint32_t* col,
                        const uint32_t* old_of_new, uint32_t rows, uint32_t elb, int idbits, const uint64_t* out_off,
                        uint64_t* keys, hipStream_t s);
void launch_keys_split_el(const uint64_t* keys, uint64_t nnz, int idbits, uint32_t elb, uint32_t* col_out,
                          uint32_t* elab_out, hipStream_t s);
// deg_out[map[v]] = total length of v's rows
void launch_deg_rows(const uint32_t* row_len, const uint32_t* map, uint32_t n, uint32_t elb, uint64_t* deg_out,
                     hipStream_t s);
void launch_csr_extract(const uint64_t* keys, uint64_t nnz, uint64_t idmask, uint32_t* col_out,
                        hipStream_t s);
void launch_deg_mapped(const uint64_t* rp, const uint32_t* row_len, const uint32_t* map, uint32_t n,
                       uint64_t* deg_out, hipStream_t s);
void launch_rows_from_scan(const uint64_t* offs, const uint64_t* deg, uint32_t n, uint64_t base,
                           uint64_t* row_off, uint32_t* row_len, hipStream_t s);
void launch_copy_rows(const uint64_t* row_off, const uint32_t* row_len, const uint32_t* src,
                      const uint64_t* new_off, uint32_t* dst, uint32_t n, hipStream_t s);
void launch_u32_to_u64(const uint32_t* in, uint64_t* out, uint32_t n, hipStream_t s);
// vertex deletions: row lengths (err |= GM_ERR_RANGE for ids >= n) with
// each deleted vertex set in the n-bit map `mark` (cleared by the caller);
// explicit insertions touching a marked vertex (err |= GM_ERR_CONFLICT);
// then the incident edges as deletions at offs[i] (external ids)
void launch_vdel_len(GmGraphDev G, const uint32_t* vdel, uint32_t nv, uint64_t* len, uint32_t* mark, uint32_t* err,
                     hipStream_t s);
void launch_vdel_check(const uint32_t* src, const uint32_t* dst, const uint8_t* op, uint32_t n_upd, uint32_t n,
                       const uint32_t* mark, uint32_t* err, hipStream_t s);
void launch_vdel_expand(GmGraphDev G, const uint32_t* vdel, uint32_t nv, const uint64_t* offs, uint32_t* src,
                        uint32_t* dst, uint8_t* op, uint32_t* elab, hipStream_t s);
void launch_gather_ext(const uint32_t* col, const uint32_t* old_of_new, uint64_t nnz, uint32_t* ext,
                       hipStream_t s);

// batch (k_batch.hip)
// keys (lo, hi, e, op) packed as ((lo << eb | hi) << elb | e) << 1 | op; elab may be nullptr
void launch_canon_keys(const uint32_t* src, const uint32_t* dst, const uint8_t* op, const uint32_t* elab,
                       uint32_t n_upd, uint32_t n, int eb, uint32_t elb, uint32_t n_el, uint64_t* keys,
                       GmCounters* ctr, hipStream_t s);
void launch_canon_classify(const uint64_t* keys, uint32_t n_upd, int eb, GmGraphDev G,
                           uint32_t* keep, GmCounters* ctr, hipStream_t s);
void launch_canon_emit(const uint64_t* keys, const uint32_t* keep, const uint32_t* ords,
                       uint32_t n_upd, int eb, GmGraphDev G, uint32_t* canon_lo, uint32_t* canon_hi,
                       uint8_t* canon_sign, uint32_t* canon_a, uint32_t* canon_b, uint32_t* canon_e,
                       GmBatchHash H, uint64_t* dkeys, hipStream_t s);
void launch_runs_flags(const uint64_t* dkeys, uint32_t N, int ib, uint64_t* vals, hipStream_t s);
void launch_runs_fill(const uint64_t* dkeys, const uint64_t* runscan, uint32_t N, int ib,
                      uint32_t* touched, uint32_t* run_start, uint32_t* run_end, hipStream_t s);
void launch_touched_sizes(const uint32_t* touched, const uint32_t* run_start, const uint32_t* run_end,
                          const uint64_t* runscan, uint32_t n_touched, GmGraphDev G, uint64_t* sizes,
                          hipStream_t s);
void launch_merge(const uint64_t* dkeys, const uint64_t* runscan, const uint32_t* touched,
                  const uint32_t* run_start, const uint32_t* run_end, const uint64_t* r1off,
                  uint32_t n_touched, uint64_t r1_total, uint64_t base1, uint64_t base2, int ib,
                  GmGraphDev G, hipStream_t s);
void launch_rows_set(const uint32_t* touched, const uint32_t* run_start, const uint32_t* run_end,
                     const uint64_t* runscan, const uint64_t* r1off, uint32_t n_touched,
                     uint64_t base1, uint64_t base2, GmGraphDev G, uint64_t* r2_off,
                     uint32_t* r2_len, hipStream_t s);
void launch_rows_commit(const uint32_t* touched, const uint64_t* r2_off, const uint32_t* r2_len,
                        uint32_t n_touched, GmGraphDev G, hipStream_t s);
void launch_rows_finish(const uint32_t* touched, const uint64_t* r2_off, const uint32_t* r2_len,
                        const uint64_t* r0_off, const uint32_t* r0_len, uint32_t n_touched, GmGraphDev G,
                        const GmCounters* ctr, uint32_t restore, hipStream_t s);  // restore: roll back
void launch_rows_save(const uint32_t* touched, uint32_t n_touched, GmGraphDev G, uint64_t* r0_off,
                      uint32_t* r0_len, hipStream_t s);

// filter and seeds (k_filter.hip)
// candidate masks of vertices `verts` (or all nv vertices); rows != 0: verts
// holds row ids and each names its vertex
void launch_filter(GmGraphDev G, const uint32_t* verts, uint32_t nv, uint32_t rows, const uint32_t* lab_fstart,
                   const GmFilterEntry* fe, const GmReq* reqs, uint16_t* cand, uint32_t only_q,
                   hipStream_t s);
void launch_pending_init(GmCounters* ctr, hipStream_t s);
// update-edge grouping: keys (position << ib | seed.a), sorted by the caller over the low ib bits,
// then the seeds gathered in key order
void launch_seed_keys(const GmSeed* seeds, uint64_t n, int ib, uint64_t* keys, hipStream_t s);
void launch_seed_gather(const GmSeed* in, const uint64_t* keys, uint64_t n, int ib, GmSeed* out, hipStream_t s);
// opens the seed window of the next search launch: seed_begin = seed_head =
// n_seeds, the deadline origin is now, and an abort of the previous launch
// is moved to the sticky timed_out flag (the next launch runs)
void launch_seed_window(GmCounters* ctr, hipStream_t s);
// Update-edge grouping by (query, directed query edge, a).  keys: qd << (ib +
// pb) | a << pb | position (sorted by the caller over 16 + ib + pb bits);
// gather as for the sort by a (low pb bits = position).
void launch_group_keys(const GmSeed* seeds, uint64_t n, int ib, int pb, uint64_t* keys, hipStream_t s);
void launch_group_gather(const GmSeed* in, const uint64_t* keys, uint64_t n, int pb, GmSeed* out, hipStream_t s);
// after the gather: lead[i] = 1 when seed i starts a group; excl = the
// exclusive scan of lead (a leader's group index)
void launch_group_lead(const uint64_t* keys, uint64_t n, int pb, uint32_t* lead, hipStream_t s);
void launch_group_assign(const uint32_t* excl, const uint32_t* lead, uint64_t n, uint32_t* seed_group,
                         hipStream_t s);
// per group: the length of a's level-2 subrange when the group has >= 2
// seeds and a is a back-neighbour of the plan's level 2, else 0
void launch_group_len(const GmSeed* seeds, const uint32_t* excl, const uint32_t* lead, uint64_t n,
                      const GmPlan* plans, const GmQueryDev* qs, GmGraphDev G, const unsigned long long* lix,
                      uint32_t lix_slots, const uint8_t* qel, unsigned long long* glen, hipStream_t s);
// per group with a length: its candidates written from arena index dst0 +
// goff[g] on (col and ext), those that pass the candidate table for the
// level-2 vertex (any position of its mask); the list records
void launch_group_fill(const GmSeed* seeds, const uint32_t* excl, const uint32_t* lead, uint64_t n,
                       const GmPlan* plans, const GmQueryDev* qs, GmGraphDev G, const unsigned long long* lix,
                       uint32_t lix_slots, const uint8_t* qel, const uint16_t* cand, uint32_t coalesce,
                       const unsigned long long* glen, const unsigned long long* goff, uint64_t dst0,
                       GmGroupList* lists, hipStream_t s);
// label index: for rows `verts` (or all rows), the subrange of each indexed label
void launch_label_index(GmGraphDev G, const uint32_t* verts, uint32_t nv, const uint32_t* slot_labels,
                        uint32_t n_slots, unsigned long long* lix, hipStream_t s);
// canon_e: edge label per canonical edge (nullptr: all 0)
void launch_seeds(const uint32_t* canon_a, const uint32_t* canon_b, const uint8_t* canon_sign,
                  const uint32_t* canon_e, uint32_t n_canon, const GmQueryDev* qs, uint32_t nq, const GmPlan* plans,
                  const uint16_t* cand, uint32_t n, GmSeed* seeds, uint64_t cap, GmCounters* ctr,
                  uint32_t only_q, uint32_t coalesce, hipStream_t s);  // only_q = 0xFFFFFFFF: every query

// search (k_dfs.hip)
void launch_dfs(const GmDfsParams& P, unsigned blocks, hipStream_t s);
// For every seed whose search did not finish (seed_open != 0):
// upd_open[ord] = 1 (if upd_open) and q_open[q] += 1 (if q_open); both must
// be zeroed first
void launch_upd_open(const GmSeed* seeds, const GmCounters* ctr, uint64_t seed_cap, const uint32_t* seed_open,
                     uint8_t* upd_open, unsigned long long* q_open, hipStream_t s);
unsigned dfs_block_threads();
unsigned dfs_resident_waves_per_cu();
unsigned dfs_waves_per_block();
// mailbox slots needed for a grid of `blocks` search blocks
uint32_t dfs_slots(unsigned blocks);

}  // namespace gm
