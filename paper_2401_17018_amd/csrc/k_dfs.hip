// The search kernel: depth-first extension of seeds into incremental
// matches (Algorithm 1 of Sec. IV-C, with the order rule stated after it).
//
// One wavefront (64 lanes) owns one task at a time and keeps its whole DFS
// state in LDS (the paper keeps a warp's state in shared memory too).  A task
// is a seed: batch edge e_ord mapped onto the directed query edge (x, y).
// Query vertices are matched in the plan's order; at level l the candidates
// of u = order[l] are the label-l subrange of the shortest neighbour list
// among u's already-matched query neighbours (GenCandidates: candidate table
// bit, then intersection with every matched neighbour's list).  The 64 lanes
// take 64 consecutive entries of that subrange per step (one coalesced
// read); each lane checks its entry against the candidate table, the
// injectivity of the partial match, and membership in every other
// neighbour list (per-lane binary search restricted to the same label
// subrange), and a ballot gives the survivor mask.  The wave then descends
// into survivors one by one (DFS: only the current path is materialised,
// Sec. IV-C), and at the last level every survivor is a match.
//
// Visibility of batch edges (the order rule).  Rows touched by the batch
// hold G u I with batch entries flagged.  An unflagged entry is an edge of
// both G and G'.  A flagged entry is usable by the seed with ord i in pass
// s (1 = insertions, searched on G'; 0 = deletions, searched on G) iff the
// edge's sign is s and its ord is > i: matches are formed from the seed
// towards higher-order batch edges, so each match comes from its
// minimum-ord batch edge exactly once.
#include "dev_common.h"
#include "kernels.h"

namespace {

constexpr int DFS_THREADS = 256;
constexpr int DFS_WAVES = DFS_THREADS / GM_WAVE;
constexpr int MAX_OTH = 120;  // >= |E(Q)| - 1 for any simple query with k <= 16

struct WaveState {
  uint32_t f[GM_MAX_K];    // internal data vertex of each query vertex
  uint32_t fx[GM_MAX_K];   // external id of the same
  uint64_t drv[GM_MAX_K];  // arena index where level l's candidate subrange starts
  uint32_t len[GM_MAX_K];  // length of that subrange
  uint32_t cur[GM_MAX_K];  // next subrange entry to examine
  uint32_t chunk[GM_MAX_K];
  uint64_t mask[GM_MAX_K]; // survivors of the current chunk not descended into yet
  uint32_t drvw[GM_MAX_K]; // query vertex whose list drives level l
  uint32_t oth_n[GM_MAX_K];
  uint64_t hpre;           // hash state over query positions before the last vertex
  uint64_t oth_base[MAX_OTH];
  uint32_t oth_len[MAX_OTH];
  uint32_t oth_w[MAX_OTH];
};

__device__ inline uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline uint64_t uni64(uint64_t x) {
  return ((uint64_t)uni((uint32_t)(x >> 32)) << 32) | uni((uint32_t)x);
}

__device__ inline uint64_t shfl_xor64(uint64_t v, int m) {
  int lo = __shfl_xor((int)(uint32_t)v, m, GM_WAVE);
  int hi = __shfl_xor((int)(uint32_t)(v >> 32), m, GM_WAVE);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
__device__ inline uint64_t wave_sum64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += shfl_xor64(v, m);
  return v;
}
__device__ inline uint64_t wave_xor64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v ^= shfl_xor64(v, m);
  return v;
}

// Wave-cooperative lower bound in a sorted (masked) list: first index whose
// value >= key.  Each step samples 64 evenly spaced entries (64-ary search),
// so a list of length L takes about log64(L) dependent loads.
__device__ inline uint32_t wave_lb(const uint32_t* __restrict__ col, uint64_t base, uint32_t len,
                                   uint32_t key, int lane, uint64_t& bytes) {
  uint32_t lo = 0, hi = len;
  while (hi - lo > GM_WAVE) {
    const uint32_t step = (hi - lo + GM_WAVE - 1) / GM_WAVE;
    const uint32_t pos = lo + (uint32_t)lane * step;
    const bool in = pos < hi;
    uint32_t val = 0;
    if (in) {
      val = col[base + pos] & GM_IDMASK;
      bytes += 4;
    }
    const uint32_t c = (uint32_t)__popcll(__ballot(in && val < key));
    if (c == 0) return lo;
    const uint32_t pos_c = lo + c * step;
    const uint32_t nlo = lo + (c - 1) * step + 1;
    hi = (c < GM_WAVE && pos_c < hi) ? pos_c : hi;
    lo = nlo;
  }
  if (hi > lo) {
    const uint32_t pos = lo + (uint32_t)lane;
    const bool in = pos < hi;
    uint32_t val = 0;
    if (in) {
      val = col[base + pos] & GM_IDMASK;
      bytes += 4;
    }
    lo += (uint32_t)__popcll(__ballot(in && val < key));
  }
  return lo;
}

// Per-lane lower bound (binary search) in a sorted (masked) list.
__device__ inline uint32_t lane_lb(const uint32_t* __restrict__ col, uint64_t base, uint32_t len,
                                   uint32_t key, uint64_t& bytes) {
  uint32_t lo = 0, n = len;
  while (n > 0) {
    const uint32_t half = n >> 1;
    bytes += 4;
    if ((col[base + lo + half] & GM_IDMASK) < key) {
      lo += half + 1;
      n -= half + 1;
    } else {
      n = half;
    }
  }
  return lo;
}

// Is batch edge {a, c} usable by the seed (ord, sign)?
__device__ inline bool visible(const GmBatchHash& H, uint32_t a, uint32_t c, uint32_t ord,
                               uint32_t sign, uint64_t& bytes) {
  const uint64_t key = gm_edge_key(a, c);
  uint32_t slot = gm_hash_slot(key, H.mask);
  for (uint32_t p = 0; p <= H.mask; ++p) {
    const uint64_t k = H.keys[slot];
    bytes += 8;
    if (k == key) {
      const uint32_t v = H.vals[slot];
      bytes += 4;
      return ((v & 1u) == sign) && ((v >> 1) > ord);
    }
    if (k == GM_EMPTY64) return false;
    slot = (slot + 1) & H.mask;
  }
  return false;
}

__device__ inline uint64_t hash_step(uint64_t h, uint32_t v, uint32_t j) {
  return gm_mix64(h ^ ((uint64_t)v + GM_GOLDEN * (uint64_t)(j + 1)));
}

struct Acc {
  uint64_t cnt, sum, xr;
  uint32_t key;
};

__device__ inline void flush_acc(const GmDfsParams& P, Acc& A, int lane) {
  const uint64_t c = wave_sum64(A.cnt);
  const uint64_t s = wave_sum64(A.sum);
  const uint64_t x = wave_xor64(A.xr);
  if (lane == 0 && A.key != 0xFFFFFFFFu && c) {
    unsigned long long* r = P.qres + (uint64_t)A.key * 3;
    atomicAdd(r + 0, (unsigned long long)c);
    atomicAdd(r + 1, (unsigned long long)s);
    atomicXor(r + 2, (unsigned long long)x);
  }
  A.cnt = A.sum = A.xr = 0;
}

// Emit the matches of one ballot: lane bit set <=> (prefix, u -> cx) is a match.
__device__ inline void emit(const GmDfsParams& P, WaveState& S, Acc& A, const GmPlan* pl, uint32_t k,
                            uint32_t u, bool ok, uint64_t m, uint32_t cx, uint64_t hpre, uint32_t q,
                            uint32_t sign, uint32_t ord, int lane, uint64_t lt, uint64_t& bytes) {
  if (ok) A.cnt += 1;
  uint64_t h = 0;
  if (P.flags & (GM_F_HASH | GM_F_PER_UPDATE)) {
    if (ok) {
      h = hash_step(hpre, cx, u);
      for (uint32_t j = u + 1; j < k; ++j) h = hash_step(h, S.fx[j], j);
      A.sum += h;
      A.xr ^= h;
    }
  }
  if (P.flags & GM_F_TUPLES) {
    const uint32_t nok = (uint32_t)__popcll(m);
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&P.ctr->tuples_found, (unsigned long long)nok);
    base = __shfl(base, 0, GM_WAVE);
    const uint64_t pos = base + (uint64_t)__popcll(m & lt);
    if (ok && pos < P.tcap) {
      uint32_t* row = P.tuples + pos * P.twidth;
      for (uint32_t j = 0; j < P.twidth; ++j) row[j] = j < k ? (j == u ? cx : S.fx[j]) : 0xFFFFFFFFu;
      P.tmeta[pos] = (q << 1) | sign;
      if (P.flags & GM_F_SEED_ATTR) P.tord[pos] = ord;
      bytes += 4ull * P.twidth + 8;
    }
  }
  if (P.flags & GM_F_PER_UPDATE) {
    const uint64_t c = (uint64_t)__popcll(m);
    const uint64_t s = wave_sum64(ok ? h : 0);
    const uint64_t x = wave_xor64(ok ? h : 0);
    if (lane == 0 && c) {
      unsigned long long* r = P.upd_res + (uint64_t)ord * 3;
      atomicAdd(r + 0, (unsigned long long)c);
      atomicAdd(r + 1, (unsigned long long)s);
      atomicXor(r + 2, (unsigned long long)x);
    }
  }
}

__global__ __launch_bounds__(DFS_THREADS) void k_dfs(GmDfsParams P) {
  __shared__ WaveState WS[DFS_WAVES];
  const int lane = threadIdx.x & 63;
  WaveState& S = WS[threadIdx.x >> 6];
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  const uint32_t n = P.G.n;
  const uint32_t* __restrict__ col = P.G.col;
  const uint32_t* __restrict__ o2n = P.G.old_of_new;
  Acc A{0, 0, 0, 0xFFFFFFFFu};
  uint64_t st_nodes = 0, st_scan = 0, st_bytes = 0;
  const unsigned long long n_seeds = P.ctr->n_seeds;

  for (;;) {
    unsigned long long t = 0;
    if (lane == 0) t = atomicAdd(&P.ctr->seed_head, 1ull);
    t = __shfl(t, 0, GM_WAVE);
    if (t >= n_seeds) break;
    const GmSeed sd = P.seeds[t];
    const uint32_t q = uni(sd.qd >> 8), dq = uni(sd.qd & 255u);
    const uint32_t ord = uni(sd.os >> 1), sign = uni(sd.os & 1u);
    const uint32_t a = uni(sd.a), b = uni(sd.b);
    const GmPlan* __restrict__ pl = P.plans + P.queries[q].plan_base + dq;
    const uint32_t k = uni(pl->k);
    const uint32_t key = (q << 1) | sign;
    if (key != A.key) {
      flush_acc(P, A, lane);
      A.key = key;
    }
    const uint32_t x = uni(pl->x), y = uni(pl->y);
    const uint32_t ax = uni(o2n[a]), bx = uni(o2n[b]);
    S.f[x] = a;
    S.f[y] = b;
    S.fx[x] = ax;
    S.fx[y] = bx;
    st_bytes += 16 + 8;

    if (k == 2) {
      // the seed itself is the whole match
      uint64_t h = gm_mix64(((uint64_t)q << 1) | sign);
      h = hash_step(h, S.fx[0], 0);
      const bool ok = lane == 0;
      emit(P, S, A, pl, 2, 1, ok, 1ull, S.fx[1], h, q, sign, ord, lane, lt, st_bytes);
      continue;
    }

    // ---- level initialisation: candidate subrange of order[l]
    auto init_level = [&](uint32_t l) -> bool {
      const uint32_t lab = uni(pl->lab[l]);
      if (lab >= P.G.label_slots) return false;
      const uint32_t lo_id = uni(P.G.label_start[lab]);
      const uint32_t hi_id = uni(P.G.label_start[lab + 1]);
      st_bytes += 8;
      if (lo_id >= hi_id) return false;
      const uint32_t ob = uni(pl->bofs[l]);
      uint32_t cnt = 0, best = 0xFFFFFFFFu, besti = 0;
      for (uint32_t bm = uni(pl->back[l]); bm; bm &= bm - 1) {
        const uint32_t w = (uint32_t)__ffs(bm) - 1;
        const uint32_t v = uni(S.f[w]);
        const uint64_t off = uni64(P.G.row_off[v]);
        const uint32_t len = uni(P.G.row_len[v]);
        st_bytes += 12;
        const uint32_t s0 = uni(wave_lb(col, off, len, lo_id, lane, st_bytes));
        const uint32_t s1 = s0 + uni(wave_lb(col, off + s0, len - s0, hi_id, lane, st_bytes));
        const uint32_t sub = s1 - s0;
        if (sub == 0) return false;
        S.oth_base[ob + cnt] = off + s0;
        S.oth_len[ob + cnt] = sub;
        S.oth_w[ob + cnt] = w;
        if (sub < best) {
          best = sub;
          besti = cnt;
        }
        ++cnt;
      }
      S.drv[l] = S.oth_base[ob + besti];
      S.len[l] = best;
      S.drvw[l] = S.oth_w[ob + besti];
      if (besti != cnt - 1) {
        S.oth_base[ob + besti] = S.oth_base[ob + cnt - 1];
        S.oth_len[ob + besti] = S.oth_len[ob + cnt - 1];
        S.oth_w[ob + besti] = S.oth_w[ob + cnt - 1];
      }
      S.oth_n[l] = cnt - 1;
      S.cur[l] = 0;
      S.mask[l] = 0;
      if (lane == 0) ++st_nodes;
      if (l == k - 1) {
        const uint32_t u = uni(pl->order[l]);
        uint64_t h = gm_mix64(((uint64_t)q << 1) | sign);
        for (uint32_t j = 0; j < u; ++j) h = hash_step(h, S.fx[j], j);
        S.hpre = h;
      }
      return true;
    };

    // ---- one chunk of 64 candidates at level l; returns the survivor ballot
    auto eval_chunk = [&](uint32_t l, uint32_t cur, uint32_t& c_out, bool& ok_out) -> uint64_t {
      const uint32_t u = uni(pl->order[l]);
      const uint32_t len = uni(S.len[l]);
      const uint32_t idx = cur + (uint32_t)lane;
      bool ok = idx < len;
      uint32_t e = 0;
      if (ok) {
        e = col[uni64(S.drv[l]) + idx];
        st_bytes += 4;
        ++st_scan;
      }
      const uint32_t c = e & GM_IDMASK;
      for (uint32_t j = 0; j < l; ++j) ok = ok && (c != S.f[pl->order[j]]);
      if (ok && l + 1 < k) {
        ok = (P.cand[(uint64_t)q * n + c] >> u) & 1u;
        st_bytes += 2;
      }
      if (ok && (e & GM_FLAG)) ok = visible(P.H, S.f[S.drvw[l]], c, ord, sign, st_bytes);
      const uint32_t on = uni(S.oth_n[l]);
      const uint32_t ob = uni(pl->bofs[l]);
      for (uint32_t i = 0; i < on; ++i) {
        if (!__ballot(ok)) break;
        if (ok) {
          const uint64_t base = S.oth_base[ob + i];
          const uint32_t olen = S.oth_len[ob + i];
          const uint32_t p = lane_lb(col, base, olen, c, st_bytes);
          if (p >= olen) {
            ok = false;
          } else {
            const uint32_t e2 = col[base + p];
            st_bytes += 4;
            if ((e2 & GM_IDMASK) != c)
              ok = false;
            else if (e2 & GM_FLAG)
              ok = visible(P.H, S.f[S.oth_w[ob + i]], c, ord, sign, st_bytes);
          }
        }
      }
      c_out = c;
      ok_out = ok;
      return __ballot(ok);
    };

    uint32_t l = 2;
    if (!init_level(2)) continue;
    for (;;) {
      uint64_t m = uni64(S.mask[l]);
      if (m == 0) {
        const uint32_t cur = uni(S.cur[l]);
        if (cur >= uni(S.len[l])) {
          if (l == 2) break;
          --l;
          continue;
        }
        S.cur[l] = cur + GM_WAVE;
        S.chunk[l] = cur;
        uint32_t c;
        bool ok;
        m = eval_chunk(l, cur, c, ok);
        if (l == k - 1) {
          if (m) {
            const uint32_t u = uni(pl->order[l]);
            uint32_t cx = 0;
            if (ok && (P.flags & (GM_F_HASH | GM_F_TUPLES | GM_F_PER_UPDATE))) {
              cx = o2n[c];
              st_bytes += 4;
            }
            emit(P, S, A, pl, k, u, ok, m, cx, uni64(S.hpre), q, sign, ord, lane, lt, st_bytes);
          }
          continue;
        }
        S.mask[l] = m;
        if (m == 0) continue;
      }
      const uint32_t bit = (uint32_t)__ffsll((unsigned long long)m) - 1;
      S.mask[l] = m & (m - 1);
      const uint32_t c = uni(col[uni64(S.drv[l]) + uni(S.chunk[l]) + bit] & GM_IDMASK);
      const uint32_t u = uni(pl->order[l]);
      S.f[u] = c;
      S.fx[u] = uni(o2n[c]);
      st_bytes += 8;
      if (init_level(l + 1)) ++l;
    }
  }
  flush_acc(P, A, lane);
  const uint64_t sn = wave_sum64(st_nodes), ss = wave_sum64(st_scan), sb = wave_sum64(st_bytes);
  if (lane == 0) {
    atomicAdd(&P.ctr->dfs_nodes, (unsigned long long)sn);
    atomicAdd(&P.ctr->cand_scanned, (unsigned long long)ss);
    atomicAdd(&P.ctr->bytes_alg, (unsigned long long)sb);
  }
}

}  // namespace

namespace gm {

unsigned dfs_block_threads() { return DFS_THREADS; }

void launch_dfs(const GmDfsParams& P, unsigned blocks, hipStream_t s) {
  k_dfs<<<blocks, DFS_THREADS, 0, s>>>(P);
}

}  // namespace gm
