// Candidate filter and seed generation.
//
// Filter (Sec. IV-B): data vertex v is a candidate of query vertex u when
// L(v) = L(u) and, for every label l among u's query neighbours, v has at
// least as many neighbours of label l as u has.  The paper packs these
// counts into saturating per-label bit fields and ANDs codes; here the exact
// counts are compared, which accepts the same vertices or fewer and is still
// sound (every vertex of a match passes).  Because internal ids are grouped
// by label, |N^l(v)| is the length of a subrange of v's sorted row: two
// binary searches, no scan.  One bit per query vertex, one uint16 per
// (query, data vertex): the candidate table of Sec. IV-B.  During a batch the
// touched rows hold G u I, whose counts bound those of G and of G' from
// above, so the filter stays sound for both search passes.  With edge
// labels a requirement names the edge label too and counts in the row of
// that label; a label the graph has no row for counts zero.
//
// Seeds (Algorithm 1, the loop over query edges and its label test): for
// every canonical batch edge (a, b) and every directed query edge (x, y) of
// every query, (x -> a, y -> b) is a seed when a is a candidate of x and b of
// y (and, with edge labels, the batch edge carries the query edge's label).
// Both orientations of each query edge are plans of their own.
#include "dev_common.h"
#include "kernels.h"

namespace {

__device__ inline uint32_t lb_masked(const uint32_t* col, uint64_t a, uint32_t len, uint32_t key) {
  uint32_t lo = 0, hi = len;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if ((col[a + mid] & GM_IDMASK) < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// verts: vertex ids, or row ids (vertex = row >> elb) when rows != 0; a
// vertex listed twice is recomputed to the same mask.
__global__ void k_filter(GmGraphDev G, const uint32_t* __restrict__ verts, uint32_t nv, uint32_t rows,
                         const uint32_t* __restrict__ lab_fstart, const GmFilterEntry* __restrict__ fe,
                         const GmReq* __restrict__ reqs, uint16_t* __restrict__ cand, uint32_t only_q) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += gridDim.x * blockDim.x) {
    const uint32_t v = verts ? (rows ? verts[i] >> G.elb : verts[i]) : i;
    const uint32_t lab = G.vlabel[v];
    if (lab >= G.label_slots) continue;
    const uint32_t e0 = lab_fstart[lab], e1 = lab_fstart[lab + 1];
    if (e0 == e1) continue;
    uint32_t cur_q = 0xFFFFFFFFu;
    uint32_t mask = 0;
    for (uint32_t e = e0; e < e1; ++e) {
      const GmFilterEntry E = fe[e];
      if (only_q != 0xFFFFFFFFu && E.q != only_q) continue;
      if (E.q != cur_q) {
        if (cur_q != 0xFFFFFFFFu) cand[(uint64_t)cur_q * G.n + v] = (uint16_t)mask;
        cur_q = E.q;
        mask = 0;
      }
      bool ok = true;
      for (uint32_t r = 0; r < E.req_n && ok; ++r) {
        const GmReq R = reqs[E.req_off + r];
        uint32_t have = 0;
        if (R.lab < G.label_slots && R.el < G.n_el) {
          const uint32_t row = (v << G.elb) | R.el;
          const uint64_t off = G.row_off[row];
          const uint32_t len = G.row_len[row];
          uint32_t s0 = lb_masked(G.col, off, len, G.label_start[R.lab]);
          uint32_t s1 = lb_masked(G.col, off, len, G.label_start[R.lab + 1]);
          have = s1 - s0;
        }
        ok = have >= R.cnt;
      }
      if (ok) mask |= 1u << E.u;
    }
    if (cur_q != 0xFFFFFFFFu) cand[(uint64_t)cur_q * G.n + v] = (uint16_t)mask;
  }
}

// Thread per (canonical batch edge, query).
__global__ void k_seeds(const uint32_t* __restrict__ canon_a, const uint32_t* __restrict__ canon_b,
                        const uint8_t* __restrict__ canon_sign, const uint32_t* __restrict__ canon_e,
                        uint32_t n_canon,
                        const GmQueryDev* __restrict__ qs, uint32_t nq, const GmPlan* __restrict__ plans,
                        const uint16_t* __restrict__ cand, uint32_t n, GmSeed* __restrict__ seeds,
                        uint64_t cap, GmCounters* ctr, uint32_t only_q, uint32_t coalesce) {
  const uint32_t nqs = only_q < nq ? 1u : nq;
  const uint64_t total = (uint64_t)n_canon * nqs;
  for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < total;
       w += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t o = (uint32_t)(w / nqs), q = only_q < nq ? only_q : (uint32_t)(w % nqs);
    const uint32_t a = canon_a[o], b = canon_b[o], el = canon_e ? canon_e[o] : 0u;
    const uint32_t ca = cand[(uint64_t)q * n + a], cb = cand[(uint64_t)q * n + b];
    if (!ca || !cb) continue;
    const GmQueryDev Q = qs[q];
    for (uint32_t d = 0; d < Q.n_plans; ++d) {
      const GmPlan& P = plans[Q.plan_base + d];
      if (coalesce && P.n_perm == 0) continue;  // another plan's matches stand for this one's
      if (coalesce >= 2 && P.n_cperm == 0) continue;  // likewise over the core's permutations
      // a representative's seed stands for the seeds of the plans it
      // permutes into: a and b pass the filter of any of their positions
      const bool core = coalesce >= 2 && P.n_cperm >= 2;
      const uint32_t mx = core ? P.omask[P.x] : 1u << P.x, my = core ? P.omask[P.y] : 1u << P.y;
      if ((ca & mx) && (cb & my) && P.el == el) {
        unsigned long long pos = atomicAdd(&ctr->n_seeds, 1ull);
        if (pos < cap) {
          GmSeed sd;
          sd.qd = (q << 8) | d;
          sd.os = (o << 1) | canon_sign[o];
          sd.a = a;
          sd.b = b;
          seeds[pos] = sd;
        }
      }
    }
  }
}

// Label index (thread per (row, indexed label)): the subrange [start,
// start + len) of the row holding neighbours with that label.  Rows are
// sorted by label-grouped ids, so this is two binary searches.  verts holds
// row ids (nullptr: rows 0 .. nv-1).
__global__ void k_label_index(GmGraphDev G, const uint32_t* __restrict__ verts, uint32_t nv,
                              const uint32_t* __restrict__ slot_labels, uint32_t n_slots,
                              unsigned long long* __restrict__ lix) {
  const uint64_t total = (uint64_t)nv * n_slots;
  for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < total;
       w += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t i = (uint32_t)(w / n_slots), sl = (uint32_t)(w % n_slots);
    const uint32_t v = verts ? verts[i] : i;
    const uint32_t lab = slot_labels[sl];
    uint32_t s0 = 0, s1 = 0;
    if (lab < G.label_slots) {
      const uint64_t off = G.row_off[v];
      const uint32_t len = G.row_len[v];
      s0 = lb_masked(G.col, off, len, G.label_start[lab]);
      s1 = s0 + lb_masked(G.col, off + s0, len - s0, G.label_start[lab + 1]);
    }
    lix[(uint64_t)v * n_slots + sl] = (unsigned long long)s0 | ((unsigned long long)(s1 - s0) << 32);
  }
}

// Update-edge grouping: sort keys (position << ib | a) of the seeds, then
// the seeds gathered in key order (a stable sort by a, the first data vertex).
__global__ void k_seed_keys(const GmSeed* __restrict__ seeds, uint64_t n, int ib, uint64_t* __restrict__ keys) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    keys[i] = (i << ib) | seeds[i].a;
}

__global__ void k_seed_gather(const GmSeed* __restrict__ in, const uint64_t* __restrict__ keys, uint64_t n, int ib,
                              GmSeed* __restrict__ out) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = in[keys[i] >> ib];
}

// ---- update-edge grouping (Alg. 1's loop over update edges: seeds that map
// the same directed query edge (x, y) with x onto the same data vertex a
// share every candidate of level 2 that comes from a's row)

__global__ void k_group_keys(const GmSeed* __restrict__ seeds, uint64_t n, int ib, int pb,
                             uint64_t* __restrict__ keys) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    keys[i] = ((uint64_t)(seeds[i].qd & 0xFFFFu) << (ib + pb)) | ((uint64_t)seeds[i].a << pb) | i;
}

__global__ void k_group_lead(const uint64_t* __restrict__ keys, uint64_t n, int pb, uint32_t* __restrict__ lead) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    lead[i] = (i == 0 || (keys[i] >> pb) != (keys[i - 1] >> pb)) ? 1u : 0u;
}

// the arena range of a's label subrange for the level-2 vertex, or len 0
// when level 2 has no list from a
__device__ inline uint32_t group_range(const GmSeed& sd, const GmPlan& P, GmGraphDev G,
                                       const unsigned long long* lix, uint32_t lix_slots, const uint8_t* qel,
                                       uint32_t q, uint64_t& base) {
  if (P.k < 3 || !((P.back[2] >> P.x) & 1u)) return 0u;
  uint32_t row = sd.a;
  if (G.elb) row = (row << G.elb) | qel[(q * GM_MAX_K + P.order[2]) * GM_MAX_K + P.x];
  const unsigned long long li = lix[(uint64_t)row * lix_slots + P.lslot[2]];
  base = G.row_off[row] + (uint32_t)li;
  return (uint32_t)(li >> 32);
}

__global__ void k_group_gather(const GmSeed* __restrict__ in, const uint64_t* __restrict__ keys, uint64_t n, int pb,
                               GmSeed* __restrict__ out) {
  const uint64_t pm = (1ull << pb) - 1ull;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = in[keys[i] & pm];
}

// group of seed i: excl[i] (leaders before i) + lead[i] - 1
__global__ void k_group_assign(const uint32_t* __restrict__ excl, const uint32_t* __restrict__ lead, uint64_t n,
                               uint32_t* __restrict__ seed_group) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    seed_group[i] = excl[i] + lead[i] - 1u;
}

__global__ void k_group_len(const GmSeed* __restrict__ seeds, const uint32_t* __restrict__ excl,
                            const uint32_t* __restrict__ lead, uint64_t n,
                            const GmPlan* __restrict__ plans, const GmQueryDev* __restrict__ qs, GmGraphDev G,
                            const unsigned long long* __restrict__ lix, uint32_t lix_slots,
                            const uint8_t* __restrict__ qel, unsigned long long* __restrict__ glen) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    if (!lead[i]) continue;
    const uint32_t g = excl[i];
    const bool pair = i + 1 < n && !lead[i + 1];
    uint64_t len = 0;
    if (pair) {
      const GmSeed sd = seeds[i];
      const uint32_t q = sd.qd >> 8;
      const GmPlan& P = plans[qs[q].plan_base + (sd.qd & 255u)];
      uint64_t base = 0;
      len = group_range(sd, P, G, lix, lix_slots, qel, q, base);
    }
    glen[g] = len;
  }
}

// one wave per group: its list, compacted in the order of a's row
__global__ void k_group_fill(const GmSeed* __restrict__ seeds, const uint32_t* __restrict__ excl,
                             const uint32_t* __restrict__ lead, uint64_t n, const GmPlan* __restrict__ plans,
                             const GmQueryDev* __restrict__ qs, GmGraphDev G,
                             const unsigned long long* __restrict__ lix, uint32_t lix_slots,
                             const uint8_t* __restrict__ qel, const uint16_t* __restrict__ cand, uint32_t coalesce,
                             const unsigned long long* __restrict__ glen, const unsigned long long* __restrict__ goff,
                             uint64_t dst0, GmGroupList* __restrict__ lists) {
  const int lane = threadIdx.x & 63;
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (uint64_t i = wave; i < n; i += nwaves) {
    if (!lead[i]) continue;
    const uint32_t g = excl[i];
    GmGroupList rec;
    rec.base = dst0 + goff[g];
    rec.len = GM_NO_GROUP;
    rec.pad = 0;
    if (glen[g]) {
      const GmSeed sd = seeds[i];
      const uint32_t q = sd.qd >> 8;
      const GmPlan& P = plans[qs[q].plan_base + (sd.qd & 255u)];
      uint64_t base = 0;
      const uint32_t len = group_range(sd, P, G, lix, lix_slots, qel, q, base);
      const uint32_t u2 = P.order[2];
      const uint32_t om = (coalesce >= 2 && P.n_cperm >= 2) ? P.omask[u2] : (1u << u2);
      uint32_t out = 0;
      for (uint32_t c0 = 0; c0 < len; c0 += 64) {
        const uint32_t idx = c0 + (uint32_t)lane;
        bool keep = false;
        uint32_t e = 0, x = 0;
        if (idx < len) {
          e = G.col[base + idx];
          x = G.ext[base + idx];
          keep = (cand[(uint64_t)q * G.n + (e & GM_IDMASK)] & om) != 0u;
        }
        const uint64_t m = __ballot(keep);
        if (keep) {
          const uint64_t at = rec.base + out + (uint64_t)__popcll(m & lt);
          G.col[at] = e;
          G.ext[at] = x;
        }
        out += (uint32_t)__popcll(m);
      }
      rec.len = out;
    }
    if (lane == 0) lists[g] = rec;
  }
}

// The search starts with one unfinished work item per seed of its window.
__global__ void k_pending_init(GmCounters* ctr) { ctr->pending = ctr->n_seeds - ctr->seed_begin; }

// Seeds appended after this point form the next launch's window.
__global__ void k_seed_window(GmCounters* ctr) {
  if (ctr->aborted) {
    ctr->timed_out = 1u;
    ctr->aborted = 0u;
  }
  ctr->seed_begin = ctr->n_seeds;
  ctr->seed_head = ctr->n_seeds;
  ctr->t_start = wall_clock64();
}

unsigned grid_for(uint64_t work, unsigned per_block) {
  uint64_t b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (unsigned)b;
}

}  // namespace

namespace gm {

void launch_filter(GmGraphDev G, const uint32_t* verts, uint32_t nv, uint32_t rows, const uint32_t* lab_fstart,
                   const GmFilterEntry* fe, const GmReq* reqs, uint16_t* cand, uint32_t only_q,
                   hipStream_t s) {
  if (!nv) return;
  k_filter<<<grid_for(nv, 256), 256, 0, s>>>(G, verts, nv, rows, lab_fstart, fe, reqs, cand, only_q);
}

void launch_pending_init(GmCounters* ctr, hipStream_t s) { k_pending_init<<<1, 1, 0, s>>>(ctr); }

void launch_seed_keys(const GmSeed* seeds, uint64_t n, int ib, uint64_t* keys, hipStream_t s) {
  if (!n) return;
  k_seed_keys<<<grid_for(n, 256), 256, 0, s>>>(seeds, n, ib, keys);
}

void launch_seed_gather(const GmSeed* in, const uint64_t* keys, uint64_t n, int ib, GmSeed* out, hipStream_t s) {
  if (!n) return;
  k_seed_gather<<<grid_for(n, 256), 256, 0, s>>>(in, keys, n, ib, out);
}
void launch_seed_window(GmCounters* ctr, hipStream_t s) { k_seed_window<<<1, 1, 0, s>>>(ctr); }

void launch_group_keys(const GmSeed* seeds, uint64_t n, int ib, int pb, uint64_t* keys, hipStream_t s) {
  if (!n) return;
  k_group_keys<<<grid_for(n, 256), 256, 0, s>>>(seeds, n, ib, pb, keys);
}
void launch_group_lead(const uint64_t* keys, uint64_t n, int pb, uint32_t* lead, hipStream_t s) {
  if (!n) return;
  k_group_lead<<<grid_for(n, 256), 256, 0, s>>>(keys, n, pb, lead);
}
void launch_group_gather(const GmSeed* in, const uint64_t* keys, uint64_t n, int pb, GmSeed* out, hipStream_t s) {
  if (!n) return;
  k_group_gather<<<grid_for(n, 256), 256, 0, s>>>(in, keys, n, pb, out);
}
void launch_group_assign(const uint32_t* excl, const uint32_t* lead, uint64_t n, uint32_t* seed_group,
                         hipStream_t s) {
  if (!n) return;
  k_group_assign<<<grid_for(n, 256), 256, 0, s>>>(excl, lead, n, seed_group);
}
void launch_group_len(const GmSeed* seeds, const uint32_t* excl, const uint32_t* lead, uint64_t n,
                      const GmPlan* plans, const GmQueryDev* qs, GmGraphDev G, const unsigned long long* lix,
                      uint32_t lix_slots, const uint8_t* qel, unsigned long long* glen, hipStream_t s) {
  if (!n) return;
  k_group_len<<<grid_for(n, 256), 256, 0, s>>>(seeds, excl, lead, n, plans, qs, G, lix, lix_slots, qel, glen);
}
void launch_group_fill(const GmSeed* seeds, const uint32_t* excl, const uint32_t* lead, uint64_t n,
                       const GmPlan* plans, const GmQueryDev* qs, GmGraphDev G, const unsigned long long* lix,
                       uint32_t lix_slots, const uint8_t* qel, const uint16_t* cand, uint32_t coalesce,
                       const unsigned long long* glen, const unsigned long long* goff, uint64_t dst0,
                       GmGroupList* lists, hipStream_t s) {
  if (!n) return;
  k_group_fill<<<grid_for(n * 64, 256), 256, 0, s>>>(seeds, excl, lead, n, plans, qs, G, lix, lix_slots, qel, cand,
                                                     coalesce, glen, goff, dst0, lists);
}

void launch_label_index(GmGraphDev G, const uint32_t* verts, uint32_t nv, const uint32_t* slot_labels,
                        uint32_t n_slots, unsigned long long* lix, hipStream_t s) {
  if (!nv || !n_slots) return;
  k_label_index<<<grid_for((uint64_t)nv * n_slots, 256), 256, 0, s>>>(G, verts, nv, slot_labels, n_slots, lix);
}

void launch_seeds(const uint32_t* canon_a, const uint32_t* canon_b, const uint8_t* canon_sign,
                  const uint32_t* canon_e, uint32_t n_canon, const GmQueryDev* qs, uint32_t nq, const GmPlan* plans,
                  const uint16_t* cand, uint32_t n, GmSeed* seeds, uint64_t cap, GmCounters* ctr,
                  uint32_t only_q, uint32_t coalesce, hipStream_t s) {
  if (!n_canon || !nq) return;
  const uint64_t work = (uint64_t)n_canon * (only_q < nq ? 1u : nq);
  k_seeds<<<grid_for(work, 256), 256, 0, s>>>(canon_a, canon_b, canon_sign, canon_e, n_canon, qs, nq, plans, cand, n,
                                              seeds, cap, ctr, only_q, coalesce);
}

}  // namespace gm
