// The search kernel: depth-first extension of seeds into incremental
// matches (Algorithm 1 of Sec. IV-C, with the order rule stated after it),
// with wavefront-level work hand-over for load balance (Sec. V-A).
//
// One wavefront (64 lanes) owns one work item at a time and keeps its DFS
// state in LDS.  A work item is a seed (batch edge e_ord mapped onto the
// directed query edge (x, y)) or a piece of another wave's search handed
// over to it.  Query vertices are matched in the plan's order; at level l
// the candidates of u = order[l] are the label subrange of the shortest
// neighbour list among u's already-matched query neighbours (GenCandidates:
// candidate-table bit, then intersection with every matched neighbour's
// list).  The 64 lanes take 64 consecutive entries of that subrange per step
// (one coalesced read); each lane checks its entry against the candidate
// table, the injectivity of the partial match and membership in every other
// neighbour list (per-lane binary search restricted to the same label
// subrange), and a ballot gives the survivor mask.  The wave then descends
// into survivors one at a time (only the current path is materialised,
// Sec. IV-C); at the last level every survivor is a match.
//
// Visibility of batch edges (the order rule).  Rows touched by the batch
// hold G u I with batch entries flagged.  An unflagged entry is an edge of
// both G and G'.  A flagged entry is usable by the seed with ord i in pass s
// (1 = insertions, searched on G'; 0 = deletions, searched on G) iff the
// edge's sign is s and its ord is > i, so every match is found once, from
// its minimum-ord batch edge.
//
// Load balance.  The paper balances warps inside a thread block through
// shared memory (Sec. V-A).  A single seed can hold most of a batch's work,
// so here the balancing spans the whole chip: an idle wave advertises itself
// in a global bitmap; a busy wave that sees advertised idle waves (it polls
// a replicated counter every few microseconds) hands over the upper half of
// its shallowest unexplored work - the untouched part of a level's candidate
// range, or half the pending survivors of a level's current chunk - together
// with the partial match above it, through the idle wave's mailbox.
// Termination: `pending` counts unfinished work items (initially the seeds);
// the wave that finishes the last one sends every wave the stop message.
#include "dev_common.h"
#include "handover.h"
#include "kernels.h"

namespace {

constexpr int DFS_THREADS = 256;
constexpr int DFS_WAVES = DFS_THREADS / GM_WAVE;
constexpr int MAX_OTH = 120;  // >= |E(Q)| - 1 for any simple query with k <= 16
constexpr uint32_t MSG_TASK = 1, MSG_STOP = 3;
// the idle count is kept in IDLE_REPS copies, one per 128-byte line; a wave
// polls the copy of its XCD
constexpr uint32_t IDLE_REPS = 8, IDLE_STRIDE = 32;
#ifndef GM_DFS_PROFILE
#define GM_DFS_PROFILE 0
#endif
// GM_DFS_COUNT=1 (instrumented builds only; exclusive with GM_DFS_PROFILE)
// reuses the five cycle tallies as last-level counters: steps, binary-search
// load instructions, lanes entering a list probe, lanes at step start, and
// the summed lengths of the probed lists.
#ifndef GM_DFS_COUNT
#define GM_DFS_COUNT 0
#endif
#ifndef GM_LEAF_UNROLL
#define GM_LEAF_UNROLL 4
#endif
constexpr int LEAF_UNROLL = GM_LEAF_UNROLL;          // last-level chunks examined per step
// survivors of level k-2 whose last-level list is at most this long are
// walked together (packed); longer ones keep their own level so that the
// hand-over can split them
#ifndef GM_PACK_MAX
#define GM_PACK_MAX 512
#endif
constexpr uint32_t PACK_MAX = GM_PACK_MAX;
// the last level polls (deadline, hand-over) once per this many steps
#ifndef GM_POLL_STEPS
#define GM_POLL_STEPS 4
#endif
constexpr uint32_t POLL_STEPS = GM_POLL_STEPS;
// a probed neighbour list of at most this many entries is read into the
// wave's LDS window in one coalesced round trip and searched there
#ifndef GM_WIN_MAX
#define GM_WIN_MAX 256
#endif
constexpr uint32_t WIN_MAX = GM_WIN_MAX;
// a last level shared by the survivors of a level-(k-2) chunk is walked
// once for all of them when its driving list has at most this many
// entries (the walk cannot be handed over, and a chunk's pairs then stay
// within about a millisecond of one wave's time); longer ones take the
// per-survivor descent, whose ranges the hand-over can split
#ifndef GM_SHARED_MAX
#define GM_SHARED_MAX 4096
#endif
constexpr uint32_t SHARED_MAX = GM_SHARED_MAX;

// Algorithmic bytes, counted in eighths of a byte by a fixed model of what
// the method must read, whatever this kernel's layout makes it read: per
// candidate examined, its 4-byte id, a 1-byte label and 1 bit of the
// candidate table; per lower-bound search in another neighbour list of
// length n, ceil(log2 n) + 1 reads of 4 bytes; 16 bytes per batch-hash probe
// of a flagged entry; 4 bytes per tuple element written (and 4 for its
// attributed update).  External ids (a consequence of the label-grouped
// renumbering) and level set-up reads are not counted.
constexpr uint64_t MB_CAND = 41;         // (4 + 1 + 1/8) * 8
constexpr uint64_t MB_HASH_PROBE = 128;  // 16 * 8
constexpr uint64_t MB_WORD = 32;         // 4 * 8
__device__ inline uint32_t mb_search(uint32_t n) {  // ceil(log2 n) + 1 for n >= 1
  return (n > 1 ? 32u - (uint32_t)__clz((int)(n - 1)) : 0u) + 1u;
}

struct WaveState {
  uint32_t f[GM_MAX_K];    // internal data vertex of each query vertex
  uint32_t fo[GM_MAX_K];   // the same by matching position: fo[l] = f[order[l]]
  uint32_t fx[GM_MAX_K];   // external id of the same
  uint64_t drv[GM_MAX_K];  // arena index where level l's candidate subrange starts
  uint32_t len[GM_MAX_K];  // end of the range to examine at level l
  uint32_t cur[GM_MAX_K];  // next subrange entry to examine
  uint32_t chunk[GM_MAX_K];
  uint64_t mask[GM_MAX_K]; // survivors of the current chunk not descended into yet
  uint32_t drvv[GM_MAX_K]; // data vertex whose row drives level l
  uint32_t oth_n[GM_MAX_K];
  uint32_t flen[GM_MAX_K]; // driver length as set up (the hand-over may shorten len)
  uint32_t lvl_ok;         // bit l: level l's set-up was made under the current f(order[0 .. l-2])
  uint64_t hpre;           // checksum salt + element terms of every position but the last vertex
  uint64_t hpp[GM_MAX_PERM]; // the same for each permutation of a coalesced plan
  uint64_t tally[8];       // idle, init, inner, leaf, hand-over cycles; tasks received; hand-overs; nodes
  uint64_t oth_base[MAX_OTH];
  uint32_t oth_len[MAX_OTH];
  uint32_t oth_v[MAX_OTH];  // data vertex whose row holds each probed list
  // Last-level set-up, prepared at the level before it (k >= 4).  The lists
  // of the last vertex's matched neighbours other than order[k-2] do not
  // change while level k-2 is searched ("static"); the survivors of the
  // current level-(k-2) chunk carry their own row's subrange ("pf_*").
  uint64_t st_base[GM_MAX_K];
  uint32_t st_len[GM_MAX_K];
  uint32_t st_v[GM_MAX_K];
  uint32_t st_n;
  uint32_t st_min;         // shortest static list (0xFFFFFFFF: none)
  uint64_t st_h;           // checksum salt + element terms of order[0 .. k-3]
  uint64_t sh_mask;        // with shared = 1: the level-(k-2) survivors that share level k-1
  uint32_t shared;
  uint32_t pf_c[GM_WAVE];  // survivor's internal id
  uint32_t pf_x[GM_WAVE];  // its external id
  uint32_t pf_len[GM_WAVE];
  uint64_t pf_base[GM_WAVE];
  uint64_t pf_h[GM_WAVE];  // its element term
  // coalescing over a core (k-degenerated automorphic subgraph): the core
  // prefix as the search found it, and the permutation now applied to it
  uint32_t fcore[GM_MAX_K];
  uint32_t fxcore[GM_MAX_K];
  uint32_t ccw[GM_MAX_K];  // candidate-filter word of each core vertex's data vertex
  uint32_t pidx;
  uint32_t pvalid;  // bit p: permutation p puts every core data vertex where the filter admits it
  uint32_t win[WIN_MAX];  // a short probed list, copied from HBM for the searches of one step
};

// Plans and query records are never written during a search: reading them
// through the constant address space lets uniform reads use scalar loads.
typedef const __attribute__((address_space(4))) GmPlan* CPlan;
typedef const __attribute__((address_space(4))) GmQueryDev* CQuery;
typedef const __attribute__((address_space(4))) GmPerm* CPerm;

__device__ inline uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline uint64_t uni64(uint64_t x) {
  return ((uint64_t)uni((uint32_t)(x >> 32)) << 32) | uni((uint32_t)x);
}

struct WaveView {
  const WaveState& S;
  __device__ uint32_t cur(uint32_t x) const { return uni(S.cur[x]); }
  __device__ uint32_t len(uint32_t x) const { return uni(S.len[x]); }
  __device__ uint64_t mask(uint32_t x) const { return uni64(S.mask[x]); }
  __device__ uint32_t pvalid() const { return uni(S.pvalid); }
  __device__ uint32_t pidx() const { return uni(S.pidx); }
};
// value of lane i (i uniform)
__device__ inline uint32_t lane_val(uint32_t x, uint32_t i) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, (int)i);
}
// value of lane i (i per lane, 0..63)
__device__ inline uint32_t lane_at(uint32_t x, uint32_t i) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(i << 2), (int)x);
}
__device__ inline uint64_t lane_val64(uint64_t x, uint32_t i) {
  return ((uint64_t)lane_val((uint32_t)(x >> 32), i) << 32) | lane_val((uint32_t)x, i);
}

__device__ inline uint64_t shfl_xor64(uint64_t v, int m) {
  int lo = __shfl_xor((int)(uint32_t)v, m, GM_WAVE);
  int hi = __shfl_xor((int)(uint32_t)(v >> 32), m, GM_WAVE);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
// inclusive prefix sum over the lanes of a wave
__device__ inline uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
  for (int d = 1; d < GM_WAVE; d <<= 1) {
    const uint32_t o = (uint32_t)__shfl_up((int)v, d, GM_WAVE);
    if (lane >= d) v += o;
  }
  return v;
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

__device__ inline uint32_t ld_coherent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t ld_coherent64(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-lane lower bound (binary search) in a sorted (masked) list.
__device__ inline uint32_t lane_lb(const uint32_t* __restrict__ col, uint64_t base, uint32_t len,
                                   uint32_t key) {
  uint32_t lo = 0, n = len;
  while (n > 0) {
    const uint32_t half = n >> 1;
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
                               uint32_t sign) {
  const uint64_t key = gm_edge_key(a, c);
  uint32_t slot = gm_hash_slot(key, H.mask);
  for (uint32_t p = 0; p <= H.mask; ++p) {
    const uint64_t k = H.keys[slot];
    if (k == key) {
      const uint32_t v = H.vals[slot];
      return ((v & 1u) == sign) && ((v >> 1) > ord);
    }
    if (k == GM_EMPTY64) return false;
    slot = (slot + 1) & H.mask;
  }
  return false;
}

// Tuple checksum: h = mix(mix(q << 1 | sign) + sum_j (f_j + 1) K_j), sums and
// products mod 2^64, with the odd position keys K_j = mix(G (j + 1)) | 1.
constexpr uint64_t hk_mix(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}
constexpr uint64_t hk_key(uint32_t j) { return hk_mix(GM_GOLDEN * (uint64_t)(j + 1)) | 1ull; }
static_assert(GM_MAX_K == 16, "position key table sized for 16 query vertices");
__constant__ uint64_t c_hk[GM_MAX_K] = {
    hk_key(0), hk_key(1), hk_key(2),  hk_key(3),  hk_key(4),  hk_key(5),  hk_key(6),  hk_key(7),
    hk_key(8), hk_key(9), hk_key(10), hk_key(11), hk_key(12), hk_key(13), hk_key(14), hk_key(15)};

// Element term of position j: (v + 1) K_j = v K_j + K_j.
__device__ inline uint64_t elem_hash(uint32_t v, uint32_t j) {
  const uint64_t kj = c_hk[j];
  return (uint64_t)v * kj + kj;
}

struct Acc {
  uint64_t cnt, sum, xr;
  uint32_t key;
};

__device__ inline void flush_acc(const GmDfsParams& P, Acc& A, int lane) {
  const uint64_t c = A.cnt;  // wave-uniform
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
// (p2, x2): a prefix position whose external id differs per lane (packed
// last level), or p2 = 0xFFFFFFFF.  pf: for a coalesced plan, the
// permutation pi whose match f o pi is emitted (tuple position j holds
// f(pi(j))), and hu = pi^-1(u), the position the candidate's term takes in
// the checksum (hpre then holds the other positions' terms for pi).
__device__ inline void emit(const GmDfsParams& P, uint32_t flags, WaveState& S, Acc& A, uint32_t k, uint32_t u,
                            bool ok,
                            uint64_t m, uint32_t cx, uint64_t hpre, uint32_t q, uint32_t sign,
                            uint32_t ord, int lane, uint64_t lt, uint64_t& ubytes, uint32_t p2 = 0xFFFFFFFFu,
                            uint32_t x2 = 0, CPerm pf = nullptr, uint32_t hu = 0xFFFFFFFFu) {
  A.cnt += (uint64_t)__popcll(m);  // m: the ballot of ok
  uint64_t h = 0;
  if (flags & (GM_F_HASH | GM_F_PER_UPDATE)) {
    if (ok) {
      h = gm_mix64(hpre + elem_hash(cx, hu == 0xFFFFFFFFu ? u : hu));  // hpre: terms of every other position
      A.sum += h;
      A.xr ^= h;
    }
  }
  if (flags & GM_F_TUPLES) {
    const uint32_t nok = (uint32_t)__popcll(m);
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&P.ctr->tuples_found, (unsigned long long)nok);
    base = lane_val64(base, 0);
    const uint64_t pos = base + (uint64_t)__popcll(m & lt);
    ubytes += MB_WORD * (k + ((flags & GM_F_SEED_ATTR) ? 1u : 0u)) * (uint64_t)__popcll(__ballot(ok && pos < P.tcap));
    if (ok && pos < P.tcap) {
      uint32_t* row = P.tuples + pos * P.twidth;
      for (uint32_t j = 0; j < P.twidth; ++j) {
        const uint32_t src = (pf && j < k) ? pf->fwd[j] : j;
        row[j] = j < k ? (src == u ? cx : (src == p2 ? x2 : S.fx[src])) : 0xFFFFFFFFu;
      }
      P.tmeta[pos] = (q << 1) | sign;
      if (flags & GM_F_SEED_ATTR) P.tord[pos] = ord;
    }
  }
  if (flags & GM_F_PER_UPDATE) {
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

// Tell every wave slot to stop (all work is done; the message carries no data).
__device__ inline void broadcast_stop(const GmDfsParams& P, int lane) {
  for (uint32_t s = (uint32_t)lane; s < P.n_slots; s += GM_WAVE)
    __hip_atomic_store(&P.mflag[s], MSG_STOP, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Register budgets: the lean build is held to 512 / 4 = 128 VGPRs, so four
// waves per SIMD (16 per CU, the default launch) stay resident, which it
// meets without spilling; the full build, which carries every feature, to
// 512 / 3 (three waves per SIMD).
#ifndef GM_DFS_WAVES_PER_EU_LEAN
#define GM_DFS_WAVES_PER_EU_LEAN 4
#endif
#ifndef GM_DFS_WAVES_PER_EU_FULL
#define GM_DFS_WAVES_PER_EU_FULL 3
#endif
#define GM_DFS_ATTR \
  __attribute__((amdgpu_waves_per_eu(FULL ? GM_DFS_WAVES_PER_EU_FULL : GM_DFS_WAVES_PER_EU_LEAN)))

// Two builds of one body.  FULL = false is the lean search: no coalesced
// plans, no edge labels, no tuple output (counts, checksums and per-update
// attribution only), which leaves those paths out of its register budget.
// FULL = true takes every feature.  The host launches the lean one whenever
// a batch needs none of them.
template <bool FULL>
__global__ __launch_bounds__(DFS_THREADS) GM_DFS_ATTR void k_dfs(GmDfsParams P) {
  const uint32_t coal = FULL ? P.coalesce : 0u;
  const uint32_t elb = FULL ? P.G.elb : 0u;
  const uint32_t flags = FULL ? P.flags : (P.flags & ~(uint32_t)(GM_F_TUPLES | GM_F_SEED_ATTR));
  __shared__ WaveState WS[DFS_WAVES];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  WaveState& S = WS[wid];
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  const uint32_t n = P.G.n;
  const uint32_t* __restrict__ col = P.G.col;
  const uint32_t* __restrict__ ext = P.G.ext;
  // slots are numbered so that waves of one XCD (blocks dispatched round
  // robin over 8 XCDs) are contiguous: idle searches start near home
  const uint32_t bpx = (gridDim.x + 7) / 8;
  const uint32_t slot = ((blockIdx.x & 7) * bpx + (blockIdx.x >> 3)) * DFS_WAVES + wid;
  Acc A{0, 0, 0, 0xFFFFFFFFu};
  uint64_t u_scan = 0, u_bytes = 0;  // candidates examined and model bytes (wave-uniform)
  // per-wave tallies live in LDS (keeps scalar registers free).  The cycle
  // split (slots 0-4) is only collected in builds with GM_DFS_PROFILE=1.
  if (lane < 8) S.tally[lane] = 0;
#define TALLY_ALWAYS(i, v)            \
  do {                                \
    if (lane == 0) S.tally[i] += (v); \
  } while (0)
#if GM_DFS_COUNT
#define CNT(i, v) TALLY_ALWAYS(i, v)
#else
#define CNT(i, v) \
  do {            \
  } while (0)
#endif
#if GM_DFS_PROFILE
#define TALLY(i, v) TALLY_ALWAYS(i, v)
#define CYCLES() __builtin_readcyclecounter()
#else
#define TALLY(i, v) \
  do {              \
    (void)(v);      \
  } while (0)
#define CYCLES() 0ull
#endif
  // this launch searches seeds [seed_begin, n_seeds); the seed window kernel
  // set seed_head = seed_begin and the deadline origin before it
  const unsigned long long n_seeds = P.ctr->n_seeds;
  if (n_seeds == P.ctr->seed_begin || P.ctr->aborted) return;  // nothing to do (nobody would send the stop message)
  bool seeds_left = true;
  uint64_t last_poll = __builtin_readcyclecounter();
  const uint64_t t_start = P.ctr->t_start;
  const uint64_t poll_cycles = P.poll_cycles;
  bool abort_now = false;

  for (;;) {
    // ------------------------------------------------------------ obtain work
    uint32_t q, dq, ord, sign, base_l;
    uint32_t tword = 0;  // handed-over work: lane w holds word w of the task record
    bool handed = false;
    bool ptask = false;  // the handed work is a share of another wave's core permutations
    uint32_t item_seed = 0;  // the seed this work item belongs to (completion tracking)
    if (seeds_left) {
      if (P.deadline_ticks && wall_clock64() - t_start > P.deadline_ticks) {
        if (lane == 0) atomicExch(&P.ctr->aborted, 1u);
        break;
      }
      unsigned long long t = 0;
      if (lane == 0) t = atomicAdd(&P.ctr->seed_head, 1ull);
      t = lane_val64(t, 0);
      if (t < n_seeds) {
        item_seed = (uint32_t)t;
        if (P.seed_open && lane == 0) atomicExch(&P.seed_open[t], 1u);
        const GmSeed sd = P.seeds[t];
        q = uni(sd.qd >> 8);
        dq = uni(sd.qd & 255u);
        ord = uni(sd.os >> 1);
        sign = uni(sd.os & 1u);
        CPlan pl = (CPlan)P.plans + ((CQuery)P.queries)[q].plan_base + dq;
        const uint32_t x = uni(pl->x), y = uni(pl->y);
        S.f[x] = uni(sd.a);
        S.f[y] = uni(sd.b);
        base_l = 2;
      } else {
        seeds_left = false;
      }
    }
    if (!seeds_left) {
      if (!P.donate) break;
      // advertise, then wait for a task or the stop message
      // count first (a claimer decrements after claiming), then set our bit
      if ((uint32_t)lane < IDLE_REPS) atomicAdd(&P.idle_rep[lane * IDLE_STRIDE], 1u);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      if (lane == 0) atomicOr(&P.idle_bits[slot >> 6], 1ull << (slot & 63));
      uint32_t msg = 0;
      int nap = 1;
      const uint64_t t_idle0 = CYCLES();
      for (;;) {
        uint32_t ab = 0;
        if (lane == 0) {
          msg = ld_coherent(&P.mflag[slot]);
          ab = ld_coherent(&P.ctr->aborted);
        }
        msg = lane_val(msg, 0);
        if (lane_val(ab, 0)) {
          abort_now = true;
          break;
        }
        if (msg) break;
        for (int i = 0; i < nap; ++i) __builtin_amdgcn_s_sleep(32);
        nap = nap < 16 ? nap * 2 : 16;
      }
      TALLY(0, CYCLES() - t_idle0);
      if (abort_now || msg == MSG_STOP) break;
      TALLY_ALWAYS(5, 1);
      // MSG_TASK: the donor cleared our bit and lowered the idle count;
      // its release store on the flag orders the task record before it
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      tword = lane < HO_WORDS ? P.mbox[(uint64_t)slot * HO_WORDS + lane] : 0;
      if (lane == 0) __hip_atomic_store(&P.mflag[slot], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t w = tword;
      q = lane_val(w, HO_W_QD) >> 8;
      dq = lane_val(w, HO_W_QD) & 255u;
      const uint32_t os = lane_val(w, HO_W_OS);
      ord = os >> 1;
      sign = os & 1u;
      const uint32_t w2 = lane_val(w, HO_W_LV);
      ptask = FULL && (w2 >> 31) != 0u;
      base_l = w2 & 0x7FFFFFFFu;
      item_seed = lane_val(w, HO_W_SEED);
      if (lane >= HO_W_F && lane < HO_W_F + GM_MAX_K) S.f[lane - HO_W_F] = w;
      handed = true;
    }

    CPlan pl = (CPlan)P.plans + ((CQuery)P.queries)[q].plan_base + dq;
    const uint32_t k = uni(pl->k);
    // the seed's group list (update-edge grouping), for a set-up of level 2
    uint32_t grp_len = GM_NO_GROUP;
    uint64_t grp_base = 0;
    bool pre2 = false;  // level 2 drives from the group's prefiltered list
    if (P.seed_group && base_l == 2) {
      const GmGroupList gr = P.group_list[P.seed_group[item_seed]];
      grp_len = uni(gr.len);
      grp_base = uni64(gr.base);
    }
    // coalesced search: this plan's matches stand for nperm permutations
    const uint32_t nperm = coal ? uni(pl->n_perm) : 1u;
    CPerm perm0 = (CPerm)P.perms + (coal ? uni(pl->perm_base) : 0u);
    // coalescing over the core: after the n_core core levels, level L0 is
    // entered once per permutation of the core prefix
    const uint32_t ncp = coal >= 2 ? uni(pl->n_cperm) : 1u;
    const uint32_t L0 = ncp > 1 ? uni(pl->n_core) : 0xFFFFFFFFu;
    const bool core = FULL && ncp > 1;  // (constant false in the lean build)
    CPerm cperm0 = (CPerm)P.perms + (ncp > 1 ? uni(pl->cperm_base) : 0u);
    const uint32_t key = (q << 1) | sign;
    if (key != A.key) {
      flush_acc(P, A, lane);
      A.key = key;
    }
    // external ids of the matched prefix (positions < base_l)
    if ((uint32_t)lane < base_l) {
      const uint32_t u = pl->order[lane];
      const uint32_t fu = S.f[u];
      S.fo[lane] = fu;
      S.fx[u] = P.G.old_of_new[fu];
    }

    if (k == 2) {
      // the seed itself is the whole match (and, coalesced, its mirror image)
      if (nperm == 1) {
        const uint64_t hp = gm_mix64(((uint64_t)q << 1) | sign) + elem_hash(S.fx[0], 0);
        emit(P, flags, S, A, 2, 1, lane == 0, 1ull, S.fx[1], hp, q, sign, ord, lane, lt, u_bytes);
      } else {
        for (uint32_t pi = 0; pi < nperm; ++pi) {
          CPerm pp = perm0 + pi;
          const uint64_t hp = gm_mix64(((uint64_t)q << 1) | sign) + elem_hash(S.fx[0], uni(pp->inv[0]));
          emit(P, flags, S, A, 2, 1, lane == 0, 1ull, S.fx[1], hp, q, sign, ord, lane, lt, u_bytes, 0xFFFFFFFFu, 0, pp,
               uni(pp->inv[1]));
        }
      }
      if (P.seed_open && lane == 0) atomicSub(&P.seed_open[item_seed], 1u);
      if (P.donate) {
        unsigned long long left = 1;
        if (lane == 0) left = atomicAdd(&P.ctr->pending, ~0ull);
        if (lane_val64(left, 0) == 1) broadcast_stop(P, lane);
      }
      continue;
    }

    // ---- level set-up.  The candidates of order[l] lie in the label
    // subrange (label index) of every matched neighbour's row: the shortest
    // list drives the level, the others are probed.  Lane i < nb holds list
    // i as (w = query vertex, base = arena index of the subrange, sub = its
    // length).
    // (a plan that permutes its core prefix keeps it when level k-2 lies
    // past the core, whose levels are all set up again under each
    // permutation; with k-2 inside the core the prefetched state would
    // belong to the identity only)
    const uint32_t pf_lvl = (k >= 4 && (ncp <= 1 || L0 + 2 <= k)) ? k - 2 : 0xFFFFFFFFu;
    // checksum terms of every position but the last vertex's, for each
    // permutation pi of a coalesced plan: position i's vertex f(i) takes
    // position pi^-1(i) in the permuted tuple
    auto perm_prefixes = [&](uint32_t ulast) {
      for (uint32_t pi = 0; pi < nperm; ++pi) {
        CPerm pp = perm0 + pi;
        uint64_t t = 0;
        if ((uint32_t)lane < k && (uint32_t)lane != ulast) t = elem_hash(S.fx[lane], pp->inv[lane]);
        S.hpp[pi] = gm_mix64(((uint64_t)q << 1) | sign) + wave_sum64(t);
      }
    };
    auto finish_level = [&](uint32_t l, uint32_t nb, bool act, uint32_t v, uint64_t base, uint32_t sub) {
      uint32_t best = 0xFFFFFFFFu, bestv = 0xFFFFFFFFu, besti = 0;
      for (uint32_t i = 0; i < nb; ++i) {
        const uint32_t si = lane_val(sub, i), vi = lane_val(v, i);
        if (si < best || (si == best && vi < bestv)) {
          best = si;
          bestv = vi;
          besti = i;
        }
      }
      const uint32_t ob = uni(pl->bofs[l]);
      // every list but the driver is probed; the last list takes the driver's place
      if (act && (uint32_t)lane != besti) {
        const uint32_t at = ob + ((uint32_t)lane == nb - 1 ? besti : (uint32_t)lane);
        S.oth_base[at] = base;
        S.oth_len[at] = sub;
        S.oth_v[at] = v;
      }
      S.drv[l] = lane_val64(base, besti);
      S.len[l] = best;
      S.flen[l] = best;
      S.drvv[l] = lane_val(v, besti);
      S.oth_n[l] = nb - 1;
      S.cur[l] = 0;
      S.mask[l] = 0;
      if (l == k - 1) S.shared = 0u;
    };

    // Lanes 0-31 fetch the lists of order[l] (one memory round trip for
    // all of them); at level k-2 lanes 32-63 fetch, in the same round
    // trip, the static lists of the last level.
    auto init_level_impl = [&](uint32_t l, bool count) -> bool {
      const uint32_t bm = uni(pl->back[l]);
      const uint32_t nb = (uint32_t)__popc(bm);
      const bool pre = l == pf_lvl;
      uint32_t bm1 = 0, nb1 = 0, ls1 = 0;
      if (pre) {
        bm1 = uni(pl->back[k - 1]) & ~(1u << uni(pl->order[l]));
        nb1 = (uint32_t)__popc(bm1);
        ls1 = uni(pl->lslot[k - 1]);
      }
      const bool hi = lane >= 32;
      const uint32_t my_i = (uint32_t)lane & 31u;
      const uint32_t my_n = hi ? nb1 : nb;
      uint32_t t = hi ? bm1 : bm;
      const uint32_t nmax = nb > nb1 ? nb : nb1;
      for (uint32_t i = 0; i < nmax; ++i)
        if (i < my_i) t &= t - 1;  // drop the lower set bits: t's lowest bit is list my_i
      const bool act = my_i < my_n;
      uint32_t v = 0, sub = 0;
      uint64_t base = 0;
      if (act) {
        const uint32_t w = __ffs(t) - 1;
        v = S.f[w];
        // with edge labels the list is the row of f(w) for the label of
        // the query edge between w and the vertex being matched
        uint32_t row = v;
        if (elb) {
          // lanes 32-63 serve the last vertex: select per lane between the
          // two wave-uniform query vertices
          const uint32_t ut = hi ? uni(pl->order[k - 1]) : uni(pl->order[l]);
          row = (v << elb) | P.qel[(q * GM_MAX_K + ut) * GM_MAX_K + w];
        }
        const uint64_t off = P.G.row_off[row];
        const uint64_t li = P.lix[(uint64_t)row * P.lix_slots + (hi ? ls1 : uni(pl->lslot[l]))];
        base = off + (uint32_t)li;
        sub = (uint32_t)(li >> 32);
        // update-edge grouping: level 2's list from a = f(x) is the
        // group's, built once and already filtered by the candidate table
        if (l == 2 && grp_len != GM_NO_GROUP && !hi && w == uni(pl->x)) {
          base = grp_base;
          sub = grp_len;
        }
      }
      if (l == 2) pre2 = grp_len != GM_NO_GROUP;
      // an empty list leaves no candidate (for a static list of the last
      // level: no candidate for any extension of this prefix)
      if (__ballot(act && sub == 0)) return false;
      if (pre) {
        if (hi && act) {
          S.st_base[my_i] = base;
          S.st_len[my_i] = sub;
          S.st_v[my_i] = v;
        }
        S.st_n = nb1;
        uint32_t mn = 0xFFFFFFFFu;
        for (uint32_t i = 0; i < nb1; ++i) mn = min(mn, lane_val(sub, 32 + i));
        S.st_min = mn;
        uint64_t h = gm_mix64(((uint64_t)q << 1) | sign);
        for (uint32_t j = 0; j < l; ++j) {
          const uint32_t uj = uni(pl->order[j]);
          h += elem_hash(uni(S.fx[uj]), uj);
        }
        S.st_h = h;
      }
      finish_level(l, nb, act && !hi, v, base, sub);
      if (count) TALLY_ALWAYS(7, 1);
      if (l == k - 1) {
        const uint32_t u = uni(pl->order[l]);
        uint64_t h = gm_mix64(((uint64_t)q << 1) | sign);
        for (uint32_t j = 0; j < k; ++j)
          if (j != u) h += elem_hash(S.fx[j], j);
        S.hpre = h;
        if (nperm > 1) perm_prefixes(u);
      }
      S.lvl_ok = uni(S.lvl_ok) | (1u << l);
      return true;
    };

    // Re-enter inner level nl (3 <= nl <= k-2) for a new survivor of level
    // nl-1 without setting it up again: when none of its lists comes from
    // order[nl-1] (nor, at level k-2, the last level's static lists), its
    // set-up depends only on f(order[0 .. nl-2]), unchanged since it was
    // made (lvl_ok).  Only the range (which a hand-over may have shortened)
    // and, at level k-2, the checksum terms of the prefix are renewed; the
    // injectivity against the new survivor is checked per candidate anyway.
    auto reenter = [&](uint32_t nl) -> bool {
      if (nl < 3 || nl + 1 >= k || !((uni(S.lvl_ok) >> nl) & 1u)) return false;
      const uint32_t up = uni(pl->order[nl - 1]);
      if ((uni(pl->back[nl]) >> up) & 1u) return false;
      if (nl == pf_lvl) {
        if ((uni(pl->back[k - 1]) >> up) & 1u) return false;
        uint64_t h = gm_mix64(((uint64_t)q << 1) | sign);
        for (uint32_t j = 0; j < nl; ++j) {
          const uint32_t uj = uni(pl->order[j]);
          h += elem_hash(uni(S.fx[uj]), uj);
        }
        S.st_h = h;
      }
      S.len[nl] = uni(S.flen[nl]);
      S.cur[nl] = 0;
      S.mask[nl] = 0;
      TALLY_ALWAYS(7, 1);
      return true;
    };

    // Descend from survivor `bit` of level k-2 into the last level using
    // what that level prepared: no global memory access.
    auto init_leaf_fast = [&](uint32_t bit) -> bool {
      const uint32_t l = k - 1;
      const uint32_t u = uni(pl->order[k - 2]);
      const uint32_t c = uni(S.pf_c[bit]);
      S.f[u] = c;
      S.fo[k - 2] = c;
      S.fx[u] = uni(S.pf_x[bit]);
      const uint32_t nb1 = uni(S.st_n);
      const bool dyn = (uni(pl->back[l]) >> u) & 1u;
      const uint32_t dlen = uni(S.pf_len[bit]);
      if (dyn && dlen == 0) return false;
      const uint32_t nb = nb1 + (dyn ? 1u : 0u);
      uint32_t v = 0, sub = 0;
      uint64_t base = 0;
      if ((uint32_t)lane < nb1) {
        v = S.st_v[lane];
        base = S.st_base[lane];
        sub = S.st_len[lane];
      } else if ((uint32_t)lane == nb1) {
        v = c;
        base = uni64(S.pf_base[bit]);
        sub = dlen;
      }
      finish_level(l, nb, (uint32_t)lane < nb, v, base, sub);
      S.hpre = uni64(S.st_h) + uni64(S.pf_h[bit]);
      if (nperm > 1) perm_prefixes(uni(pl->order[l]));
      TALLY_ALWAYS(7, 1);
      return true;
    };

    // Last level shared by a chunk's survivors.  When none of the last query
    // vertex's lists comes from order[k-2] (its matched neighbours all come
    // earlier in the order), its candidates are the same for every survivor
    // s of a level-(k-2) chunk, but for s itself.  Level k-1 is then set up
    // once from the static lists (the driver picked as for each survivor)
    // and walked once; every candidate that passes is paired with every
    // survivor, (s, c) being a match unless c = s where the labels allow it
    // (leaf_step).  Not for lists longer than SHARED_MAX, whose per-survivor
    // ranges the hand-over can split.
    auto init_leaf_shared = [&](uint64_t m) -> bool {
      const uint32_t nb1 = uni(S.st_n);
      if (nb1 == 0 || uni(S.st_min) > SHARED_MAX) return false;
      uint32_t v = 0, sub = 0;
      uint64_t base = 0;
      if ((uint32_t)lane < nb1) {
        v = S.st_v[lane];
        base = S.st_base[lane];
        sub = S.st_len[lane];
      }
      finish_level(k - 1, nb1, (uint32_t)lane < nb1, v, base, sub);
      S.sh_mask = m;
      S.shared = 1u;
      TALLY_ALWAYS(7, (uint32_t)__popcll(m));
      return true;
    };

    // After a level-(k-2) chunk: every survivor lane records its external id,
    // its element term and (when order[k-2] is a matched neighbour of the
    // last vertex) its own row's subrange for the last vertex's label.
    auto prefetch_leaf = [&](uint32_t l, uint32_t idx, uint32_t c, bool ok) -> uint32_t {
      const uint32_t u = uni(pl->order[l]);
      const bool dyn = (uni(pl->back[k - 1]) >> u) & 1u;
      const uint32_t ls1 = uni(pl->lslot[k - 1]);
      if (ok) {
        const uint32_t x = ext[uni64(S.drv[l]) + idx];
        uint64_t base = 0;
        uint32_t sub = 0;
        if (dyn) {
          uint32_t row = c;
          if (elb) row = (c << elb) | P.qel[(q * GM_MAX_K + uni(pl->order[k - 1])) * GM_MAX_K + u];
          const uint64_t off = P.G.row_off[row];
          const uint64_t li = P.lix[(uint64_t)row * P.lix_slots + ls1];
          base = off + (uint32_t)li;
          sub = (uint32_t)(li >> 32);
        }
        S.pf_c[lane] = c;
        S.pf_x[lane] = x;
        S.pf_base[lane] = base;
        S.pf_len[lane] = sub;
        S.pf_h[lane] = elem_hash(x, u);
        return sub;
      }
      return 0u;
    };

    auto init_level = [&](uint32_t l, bool count) -> bool {
      const uint64_t t0 = CYCLES();
      const bool r = init_level_impl(l, count);
      TALLY(1, CYCLES() - t0);
      return r;
    };

    // ---- one chunk of 64 candidates at level l; returns the survivor ballot
    auto eval_chunk = [&](uint32_t l, uint32_t cur, uint32_t& c_out, uint32_t& e_idx, bool& ok_out) -> uint64_t {
      const uint32_t u = uni(pl->order[l]);
      const uint32_t len = uni(S.len[l]);
      const uint32_t idx = cur + (uint32_t)lane;
      bool ok = idx < len;
      uint32_t e = 0;
      {
        const uint32_t nin = (uint32_t)__popcll(__ballot(ok));
        u_scan += nin;
        u_bytes += MB_CAND * nin;
      }
      if (ok) e = col[uni64(S.drv[l]) + idx];
      const uint32_t c = e & GM_IDMASK;
      // injectivity: only earlier levels with order[l]'s label can collide
      const uint32_t fo_all = S.fo[lane & (GM_MAX_K - 1)];
      for (uint32_t im = uni(pl->injm[l]); im; im &= im - 1) ok = ok && (c != lane_val(fo_all, __builtin_ctz(im)));
      if (ok && l + 1 < k && !(l == 2 && pre2)) {
        // (a representative's core vertex passes for any of its positions)
        const uint32_t om = ncp > 1 ? uni(pl->omask[u]) : 1u << u;
        ok = (P.cand[(uint64_t)q * n + c] & om) != 0u;
      }
      u_bytes += MB_HASH_PROBE * (uint64_t)__popcll(__ballot(ok && (e & GM_FLAG)));
      if (ok && (e & GM_FLAG)) ok = visible(P.H, S.drvv[l], c, ord, sign);
      const uint32_t on = uni(S.oth_n[l]);
      const uint32_t ob = uni(pl->bofs[l]);
      for (uint32_t i = 0; i < on; ++i) {
        const uint64_t act = __ballot(ok);
        if (!act) break;
        const uint32_t olen = uni(S.oth_len[ob + i]);
        u_bytes += MB_WORD * mb_search(olen) * (uint64_t)__popcll(act);
        bool fl = false;
        if (ok) {
          const uint64_t base = S.oth_base[ob + i];
          const uint32_t p = lane_lb(col, base, olen, c);
          if (p >= olen) {
            ok = false;
          } else {
            const uint32_t e2 = col[base + p];
            if ((e2 & GM_IDMASK) != c) {
              ok = false;
            } else if (e2 & GM_FLAG) {
              fl = true;
              ok = visible(P.H, S.oth_v[ob + i], c, ord, sign);
            }
          }
        }
        u_bytes += MB_HASH_PROBE * (uint64_t)__popcll(__ballot(fl));
      }
      c_out = c;
      e_idx = idx;
      ok_out = ok;
      return __ballot(ok);
    };

    // ---- hand the upper half of the shallowest unexplored work to an idle wave
    auto try_donate_impl = [&](uint32_t lcur) {
      // the shallowest splittable work (rules shared with the host model)
      // (a shared last level is not split: its survivors are not in the task record)
      const HoSplit sp = ho_choose(WaveView{S}, base_l, lcur, k, core, L0,
                                   uni(S.shared) ? 0xFFFFFFFFu : P.split_leaf, P.split_inner, ho_rule_default());
      const uint32_t lv = sp.lv, kind = sp.kind;
      const uint64_t give = sp.give;
      if (kind == 0) return;
      // claim an idle wave: scan the bitmap (64 words per coherent load) from
      // a pseudo-random word, clear one set bit with an atomic AND.  No waiting.
      int32_t target = -1;
      const uint32_t nwords = (P.n_slots + 63) / 64;
      const uint32_t start = (uint32_t)(gm_mix64(((uint64_t)slot << 20) ^ __builtin_readcyclecounter()) % nwords);
      for (uint32_t r = 0; r < nwords && target < 0; r += GM_WAVE) {
        const uint32_t wi = (start + r + (uint32_t)lane) % nwords;
        const uint64_t v = (r + (uint32_t)lane < nwords) ? ld_coherent64(&P.idle_bits[wi]) : 0ull;
        uint64_t nz = __ballot(v != 0);
        for (int tries = 0; nz && target < 0 && tries < 2; ++tries) {
          const int ln = __ffsll((unsigned long long)nz) - 1;
          nz &= nz - 1;
          uint64_t vv = lane_val64(v, (uint32_t)ln);
          const uint32_t word = (start + r + (uint32_t)ln) % nwords;
          for (int b_try = 0; vv && target < 0 && b_try < 4; ++b_try) {
            const int b = __ffsll((unsigned long long)vv) - 1;
            unsigned long long old = 0;
            if (lane == 0) old = atomicAnd(&P.idle_bits[word], ~(1ull << b));
            old = lane_val64(old, 0);
            if ((old >> b) & 1ull)
              target = (int32_t)(word * 64 + b);
            else
              vv = old & ~(1ull << b);
          }
        }
      }
      if (target < 0) return;
      if ((uint32_t)lane < IDLE_REPS) atomicSub(&P.idle_rep[lane * IDLE_STRIDE], 1u);
      if (kind == HO_RANGE)
        S.len[lv] = sp.mid;
      else if (kind == HO_SURV)
        S.mask[lv] = uni64(S.mask[lv]) & ~give;
      else
        S.pvalid = uni(S.pvalid) & ~(uint32_t)give;
      // the partial match: the core prefix as found when the work lies in
      // or above a core being permuted
      const uint32_t fi = (lane >= HO_W_F && lane < HO_W_F + GM_MAX_K)
                              ? ((kind == HO_PERMS || (core && lv < L0 && lcur >= L0)) ? S.fcore[lane - HO_W_F]
                                                                                       : S.f[lane - HO_W_F])
                              : 0u;
      const uint32_t w = ho_task_word((uint32_t)lane, q, dq, ord, sign, sp, kind == HO_SURV ? uni(S.chunk[lv]) : 0u,
                                      fi, item_seed);
      if (lane == 0) atomicAdd(&P.ctr->pending, 1ull);
      if (P.seed_open && lane == 0) atomicAdd(&P.seed_open[item_seed], 1u);
      if (lane < HO_WORDS) P.mbox[(uint64_t)target * HO_WORDS + lane] = w;
      if (lane == 0) {
        __hip_atomic_store(&P.mflag[target], MSG_TASK, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        S.tally[6] += 1;
      }
    };

    // ---- keep candidate e[j] (lane, chunk j) only if it is in the sorted
    // list [base, base + olen) of row wv and that entry is visible; the
    // lower-bound searches of the caller's chunks run interleaved.
    auto probe_list = [&](auto& ok, const auto& e, uint64_t base, uint32_t olen, uint32_t wv) {
      constexpr int NU = (int)(sizeof(e) / sizeof(e[0]));  // chunks of the caller's step
      uint32_t n_probe = 0;
#pragma unroll
      for (int j = 0; j < NU; ++j) n_probe += (uint32_t)__popcll(__ballot(ok[j]));
      u_bytes += MB_WORD * n_probe * mb_search(olen);
      CNT(2, n_probe);
      CNT(4, olen);
      uint32_t lo[NU], cnt[NU];
#pragma unroll
      for (int j = 0; j < NU; ++j) {
        lo[j] = 0;
        cnt[j] = ok[j] ? olen : 0u;
      }
      uint32_t e2[NU];
      if (olen <= WIN_MAX) {
        // a short list: all of it into the wave's LDS window (every load
        // issued before any store, so one memory round trip), then the
        // lower-bound searches run on LDS
#pragma unroll
        for (uint32_t r = 0; r < WIN_MAX / GM_WAVE; ++r) {
          const uint32_t i = r * GM_WAVE + (uint32_t)lane;
          if (i < olen) S.win[i] = col[base + i];
        }
        for (;;) {
          bool any = false;
#pragma unroll
          for (int j = 0; j < NU; ++j) {
            if (cnt[j]) {
              any = true;
              const uint32_t half = cnt[j] >> 1;
              if ((S.win[lo[j] + half] & GM_IDMASK) < (e[j] & GM_IDMASK)) {
                lo[j] += half + 1;
                cnt[j] -= half + 1;
              } else {
                cnt[j] = half;
              }
            }
          }
          if (!__ballot(any)) break;
        }
#pragma unroll
        for (int j = 0; j < NU; ++j) {
          const bool in = lo[j] < olen;
          e2[j] = S.win[in ? lo[j] : olen - 1];
          if (ok[j] && (!in || (e2[j] & GM_IDMASK) != (e[j] & GM_IDMASK))) ok[j] = false;
        }
      } else {
        for (;;) {
          uint32_t v[NU];
          bool any = false;
#pragma unroll
          for (int j = 0; j < NU; ++j) {
            // clamped so a finished search still reads inside the list (olen >= 1)
            const uint32_t at = lo[j] + (cnt[j] >> 1);
            v[j] = col[base + (at < olen ? at : olen - 1)] & GM_IDMASK;
          }
          CNT(1, NU);
#pragma unroll
          for (int j = 0; j < NU; ++j) {
            if (cnt[j]) {
              any = true;
              const uint32_t half = cnt[j] >> 1;
              if (v[j] < (e[j] & GM_IDMASK)) {
                lo[j] += half + 1;
                cnt[j] -= half + 1;
              } else {
                cnt[j] = half;
              }
            }
          }
          if (!__ballot(any)) break;
        }
#pragma unroll
        for (int j = 0; j < NU; ++j) {
          const bool in = lo[j] < olen;
          e2[j] = col[base + (in ? lo[j] : olen - 1)];
          if (ok[j] && (!in || (e2[j] & GM_IDMASK) != (e[j] & GM_IDMASK))) ok[j] = false;
        }
      }
      uint32_t nfl = 0;
#pragma unroll
      for (int j = 0; j < NU; ++j) nfl += (uint32_t)__popcll(__ballot(ok[j] && (e2[j] & GM_FLAG)));
      u_bytes += MB_HASH_PROBE * nfl;
#pragma unroll
      for (int j = 0; j < NU; ++j)
        if (ok[j] && (e2[j] & GM_FLAG)) ok[j] = visible(P.H, wv, e[j] & GM_IDMASK, ord, sign);
    };

    // ---- last level: LEAF_UNROLL chunks per step.  Ids and external ids are
    // loaded together, and the binary searches in the other back-neighbour
    // lists run interleaved, so every memory round trip serves 4 chunks.
    auto leaf_step = [&](uint32_t cur) {
      const uint32_t l = k - 1;
      const uint32_t u = uni(pl->order[l]);
      const uint32_t len = uni(S.len[l]);
      const uint64_t drv = uni64(S.drv[l]);
      const uint32_t on = uni(S.oth_n[l]);
      const uint32_t ob = uni(pl->bofs[l]);
      const bool need_x = (flags & (GM_F_HASH | GM_F_TUPLES | GM_F_PER_UPDATE)) != 0;
      uint32_t e[LEAF_UNROLL], x[LEAF_UNROLL];
      bool ok[LEAF_UNROLL];
      // branch-free: lanes past the end read the last entry (len >= 1) and
      // are masked off afterwards
#pragma unroll
      for (int j = 0; j < LEAF_UNROLL; ++j) {
        const uint32_t idx = cur + (uint32_t)(j * GM_WAVE + lane);
        ok[j] = idx < len;
        e[j] = col[drv + (ok[j] ? idx : len - 1)];
      }
      // external ids without a branch around the loads (a branch makes the
      // compiler wait for each load inside it); without a checksum every
      // lane reads entry 0 of the table instead
#pragma unroll
      for (int j = 0; j < LEAF_UNROLL; ++j) {
        const uint32_t idx = cur + (uint32_t)(j * GM_WAVE + lane);
        x[j] = ext[need_x ? drv + (ok[j] ? idx : len - 1) : 0ull];
      }
      // a level shared by several survivors: the byte model counts this
      // step once per survivor, as their own descents would read it
      const bool shared = uni(S.shared) != 0u;
      const uint64_t shm = shared ? uni64(S.sh_mask) : 0ull;
      const uint32_t ns = shared ? (uint32_t)__popcll(shm) : 1u;
      const uint64_t ub0 = u_bytes;
      // candidates scanned and their bytes, counted once per wave
      uint32_t n_in = 0;
#pragma unroll
      for (int j = 0; j < LEAF_UNROLL; ++j) n_in += (uint32_t)__popcll(__ballot(ok[j]));
      u_scan += (uint64_t)n_in * ns;
      u_bytes += (uint64_t)n_in * MB_CAND;
      CNT(0, 1);
      CNT(3, n_in * ns);
      const uint32_t fo_all = S.fo[lane & (GM_MAX_K - 1)];
      // (a shared level leaves the survivor's own position to the pairs)
      for (uint32_t im = uni(pl->injm[l]) & (shared ? ~(1u << (k - 2)) : ~0u); im; im &= im - 1) {
        const uint32_t fv = lane_val(fo_all, __builtin_ctz(im));
#pragma unroll
        for (int j = 0; j < LEAF_UNROLL; ++j) ok[j] = ok[j] && ((e[j] & GM_IDMASK) != fv);
      }
      const uint32_t fdrv = uni(S.drvv[l]);
      {
        uint32_t nfl = 0;
#pragma unroll
        for (int j = 0; j < LEAF_UNROLL; ++j) nfl += (uint32_t)__popcll(__ballot(ok[j] && (e[j] & GM_FLAG)));
        u_bytes += MB_HASH_PROBE * nfl;
      }
#pragma unroll
      for (int j = 0; j < LEAF_UNROLL; ++j)
        if (ok[j] && (e[j] & GM_FLAG)) ok[j] = visible(P.H, fdrv, e[j] & GM_IDMASK, ord, sign);
      for (uint32_t i = 0; i < on; ++i) {
        bool anyok = false;
#pragma unroll
        for (int j = 0; j < LEAF_UNROLL; ++j) anyok = anyok || ok[j];
        if (!__ballot(anyok)) break;
        probe_list(ok, e, uni64(S.oth_base[ob + i]), uni(S.oth_len[ob + i]), uni(S.oth_v[ob + i]));
      }
      if (shared) {
        u_bytes = ub0 + (u_bytes - ub0) * ns;
        // every candidate left pairs with every survivor s (its data vertex
        // and prefix terms sit in lane s), but s itself where order[k-2] and
        // the last vertex share a label; one chunk's term at a time
        const bool inj_s = ((uni(pl->injm[l]) >> (k - 2)) & 1u) != 0u;
        const uint32_t my_c = S.pf_c[lane];
        const uint64_t my_h = uni64(S.st_h) + S.pf_h[lane];
#pragma unroll
        for (int j = 0; j < LEAF_UNROLL; ++j) {
          if (!__ballot(ok[j])) continue;
          const uint64_t t = elem_hash(x[j], u);
          const uint32_t cj = e[j] & GM_IDMASK;
          for (uint64_t mm = shm; mm; mm &= mm - 1) {
            const uint32_t s = (uint32_t)__builtin_ctzll(mm);
            const bool ok2 = ok[j] && !(inj_s && cj == lane_val(my_c, s));
            const uint64_t m2 = __ballot(ok2);
            A.cnt += (uint64_t)__popcll(m2);
            if (flags & (GM_F_HASH | GM_F_PER_UPDATE)) {
              const uint64_t h = ok2 ? gm_mix64(lane_val64(my_h, s) + t) : 0ull;
              A.sum += h;
              A.xr ^= h;
              if (flags & GM_F_PER_UPDATE) {
                const uint64_t ws = wave_sum64(h);
                const uint64_t wx = wave_xor64(h);
                if (lane == 0 && m2) {
                  unsigned long long* r = P.upd_res + (uint64_t)ord * 3;
                  atomicAdd(r + 0, (unsigned long long)__popcll(m2));
                  atomicAdd(r + 1, (unsigned long long)ws);
                  atomicXor(r + 2, (unsigned long long)wx);
                }
              }
            }
          }
        }
      } else if (nperm == 1) {
        const uint64_t hpre = uni64(S.hpre);
#pragma unroll
        for (int j = 0; j < LEAF_UNROLL; ++j) {
          const uint64_t m = __ballot(ok[j]);
          if (m) emit(P, flags, S, A, k, u, ok[j], m, x[j], hpre, q, sign, ord, lane, lt, u_bytes);
        }
      } else {
        // coalesced plan: every match found stands for nperm permuted ones
#pragma unroll
        for (int j = 0; j < LEAF_UNROLL; ++j) {
          const uint64_t m = __ballot(ok[j]);
          if (m)
            for (uint32_t pi = 0; pi < nperm; ++pi) {
              CPerm pp = perm0 + pi;
              emit(P, flags, S, A, k, u, ok[j], m, x[j], uni64(S.hpp[pi]), q, sign, ord, lane, lt, u_bytes, 0xFFFFFFFFu,
                   0, pp, uni(pp->inv[u]));
            }
        }
      }
    };

    auto try_donate = [&](uint32_t lcur) {
      const uint64_t t0 = CYCLES();
      try_donate_impl(lcur);
      TALLY(4, CYCLES() - t0);
    };

    // ---- every poll_cycles: deadline check, then (gated) hand-over of the
    // shallowest splittable work at levels <= lcur.  Returns true to abort.
    auto poll = [&](uint32_t lcur) -> bool {
      const uint64_t now = __builtin_readcyclecounter();
      if (now - last_poll < poll_cycles) return false;
      last_poll = now;
      // cooperative deadline: the first wave past it raises the abort word;
      // every wave checks the word here and leaves
      uint32_t ab = 0;
      if (lane == 0) {
        if (P.deadline_ticks && wall_clock64() - t_start > P.deadline_ticks) atomicExch(&P.ctr->aborted, 1u);
        ab = ld_coherent(&P.ctr->aborted);
      }
      if (lane_val(ab, 0)) return true;
      if (P.donate) {
        // gate: with c idle waves, a busy wave tries with probability
        // min(1, c * gate / 1024), so about c * gate / 1024 of them per period
        const uint32_t c = ld_coherent(&P.idle_rep[(blockIdx.x & (IDLE_REPS - 1)) * IDLE_STRIDE]);
        if (c != 0 && c < 0x80000000u) {
          const uint32_t roll = (uint32_t)gm_mix64(((uint64_t)slot << 32) ^ now) & 1023u;
          if (roll < (c >= 1024u / P.gate ? 1024u : c * P.gate)) try_donate(lcur);
        }
      }
      return false;
    };

    // ---- packed last level.  When the last query vertex's lists include
    // the row of order[k-2], every survivor s of a level-(k-2) chunk whose
    // own list (from its prefetch record) is short and no longer than the
    // static lists drives its last level with that list.  Those lists are
    // walked as one flattened range, 256 candidates per step, lane t taking
    // candidate t of the concatenation; the other survivors are left in
    // the level's mask for the regular descent.  my_len = this lane's
    // survivor list length (0 if not a survivor).
    auto leaf_packed = [&](uint32_t l, uint64_t m, uint32_t my_len) -> bool {
      if (nperm > 1) return false;  // coalesced plans take the regular last level
      const uint32_t lf = k - 1;
      const uint32_t u = uni(pl->order[lf]);
      const uint32_t u2 = uni(pl->order[l]);
      if (!((uni(pl->back[lf]) >> u2) & 1u)) {
        // every list of the last vertex is static: one walk for the chunk
        if (!P.shared_leaf || (flags & GM_F_TUPLES) || !init_leaf_shared(m)) return false;
        S.mask[l] = 0;  // the chunk's survivors are all taken by the shared level
        return true;
      }
      const bool in_m = (m >> lane) & 1ull;
      const uint32_t st_min = uni(S.st_min);
      // survivors with an empty list have no extension at all
      const uint64_t empty = __ballot(in_m && my_len == 0);
      const uint64_t pm = __ballot(in_m && my_len != 0 && my_len <= PACK_MAX && my_len <= st_min);
      S.mask[l] = m & ~pm & ~empty;
      if (!pm) return false;
      TALLY_ALWAYS(7, (uint32_t)__popcll(pm));
      const uint32_t lenv = ((pm >> lane) & 1ull) ? my_len : 0u;
      const uint32_t incl = wave_incl_scan(lenv, lane);  // end of each survivor's range
      const uint32_t excl = incl - lenv;                  // its start
      const uint32_t T = lane_val(incl, GM_WAVE - 1);
      const uint32_t b0 = (uint32_t)__ffsll((unsigned long long)pm) - 1;
      const uint32_t nb1 = uni(S.st_n);
      const uint64_t st_h = uni64(S.st_h);
      const uint32_t fo_all = S.fo[lane & (GM_MAX_K - 1)];
      const bool need_x = (flags & (GM_F_HASH | GM_F_TUPLES | GM_F_PER_UPDATE)) != 0;
      for (uint32_t t0 = 0; t0 < T; t0 += LEAF_UNROLL * GM_WAVE) {
        // the cycle-counter read behind a poll is a scalar memory access:
        // every 4th step is often enough
        if ((t0 & (4 * LEAF_UNROLL * GM_WAVE - 1)) == 0 && poll(l)) {
          abort_now = true;
          return false;
        }
        // survivor of each candidate t: the first lane whose range ends
        // after t, i.e. the number of lanes whose range ends at or before
        // t (incl is non-decreasing over the 64 lanes; lanes that are not
        // packed survivors add 0).  Per chunk [tb, tb + 64): s0 ranges end
        // at or before tb, and the few that end inside the chunk are
        // counted one by one; with many of them, a 6-step binary search
        // over the lanes.  Lanes past T read survivor b0's first entry.
        uint32_t sl[LEAF_UNROLL], off[LEAF_UNROLL];
        bool ok[LEAF_UNROLL];
#pragma unroll
        for (int j = 0; j < LEAF_UNROLL; ++j) {
          const uint32_t tb = t0 + (uint32_t)(j * GM_WAVE);
          const uint32_t t = tb + (uint32_t)lane;
          ok[j] = t < T;
          const uint64_t ends_in = __ballot(incl > tb && incl <= tb + (GM_WAVE - 1));
          uint32_t pos;
          if (__popcll(ends_in) <= 4) {
            pos = (uint32_t)__popcll(__ballot(incl <= tb));
            for (uint64_t m = ends_in; m; m &= m - 1)
              pos += lane_val(incl, (uint32_t)__builtin_ctzll(m)) <= t ? 1u : 0u;
            pos = pos < GM_WAVE ? pos : GM_WAVE - 1;
          } else {
            pos = 0;
#pragma unroll
            for (uint32_t step = GM_WAVE / 2; step; step >>= 1)
              if (lane_at(incl, pos + step - 1) <= t) pos += step;
          }
          const uint32_t lb = lane_at(excl, pos);
          sl[j] = ok[j] ? pos : b0;
          off[j] = ok[j] ? lb : t;
        }
        uint32_t e[LEAF_UNROLL], x[LEAF_UNROLL], cs[LEAF_UNROLL];
#pragma unroll
        for (int j = 0; j < LEAF_UNROLL; ++j) {
          const uint32_t t = t0 + (uint32_t)(j * GM_WAVE + lane);
          const uint64_t at = S.pf_base[sl[j]] + (t - off[j]);
          e[j] = col[at];
          x[j] = ext[need_x ? at : 0ull];  // no branch around the load (see leaf_step)
          cs[j] = S.pf_c[sl[j]];
        }
        uint32_t n_in = 0;
#pragma unroll
        for (int j = 0; j < LEAF_UNROLL; ++j) n_in += (uint32_t)__popcll(__ballot(ok[j]));
        u_scan += n_in;
        u_bytes += (uint64_t)n_in * MB_CAND;
        CNT(0, 1);
        CNT(3, n_in);
        // injectivity against order[0 .. k-3] with the last vertex's label
        // (a neighbour of the survivor is never the survivor itself)
        for (uint32_t im = uni(pl->injm[lf]) & ((1u << l) - 1u); im; im &= im - 1) {
          const uint32_t fv = lane_val(fo_all, __builtin_ctz(im));
#pragma unroll
          for (int j = 0; j < LEAF_UNROLL; ++j) ok[j] = ok[j] && ((e[j] & GM_IDMASK) != fv);
        }
        {
          uint32_t nfl = 0;
#pragma unroll
          for (int j = 0; j < LEAF_UNROLL; ++j) nfl += (uint32_t)__popcll(__ballot(ok[j] && (e[j] & GM_FLAG)));
          u_bytes += MB_HASH_PROBE * nfl;
        }
#pragma unroll
        for (int j = 0; j < LEAF_UNROLL; ++j)
          if (ok[j] && (e[j] & GM_FLAG)) ok[j] = visible(P.H, cs[j], e[j] & GM_IDMASK, ord, sign);
        for (uint32_t i = 0; i < nb1; ++i) {
          bool anyok = false;
#pragma unroll
          for (int j = 0; j < LEAF_UNROLL; ++j) anyok = anyok || ok[j];
          if (!__ballot(anyok)) break;
          probe_list(ok, e, uni64(S.st_base[i]), uni(S.st_len[i]), uni(S.st_v[i]));
        }
#pragma unroll
        for (int j = 0; j < LEAF_UNROLL; ++j) {
          const uint64_t mm = __ballot(ok[j]);
          if (mm) {
            const uint64_t hpre = st_h + S.pf_h[sl[j]];
            const uint32_t x2 = (flags & GM_F_TUPLES) ? S.pf_x[sl[j]] : 0u;
            emit(P, flags, S, A, k, u, ok[j], mm, x[j], hpre, q, sign, ord, lane, lt, u_bytes, u2, x2);
          }
        }
      }
      return false;
    };

    // core permutation p (0: the identity) of the prefix saved in fcore:
    // query vertex v takes fcore[pi(v)]; positions < L0 are the core
    auto apply_cperm = [&](uint32_t p) {
      S.lvl_ok = 0u;  // the prefix moves: every set-up below is stale
      CPerm pp = cperm0 + p;
      uint32_t v = 0, nf = 0, nx = 0;
      if ((uint32_t)lane < L0) {
        v = pl->order[lane];
        const uint32_t src = pp->fwd[v];
        nf = S.fcore[src];
        nx = S.fxcore[src];
      }
      if ((uint32_t)lane < L0) {
        S.f[v] = nf;
        S.fx[v] = nx;
        S.fo[lane] = nf;
      }
    };
    // bit p set: permutation p puts every core vertex's data vertex where
    // the filter admits it.  All permutations at once: lane t checks levels
    // 4 (t & 3) .. 4 (t & 3) + 3 under permutation t / 4 (n_core <= 16 and
    // at most 16 permutations fill the 64 lanes).
    auto cperm_valid = [&]() -> uint32_t {
      const uint32_t p = (uint32_t)lane >> 2;
      bool bad = false;
      if (p < ncp) {
        CPerm pp = cperm0 + p;
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
          const uint32_t i = ((uint32_t)lane & 3u) * 4u + j;
          if (i < L0) {
            const uint32_t v = pl->order[i];
            bad = bad || !((S.ccw[pp->fwd[v]] >> v) & 1u);
          }
        }
      }
      const uint64_t b = __ballot(bad);
      uint32_t ok = 0;
      for (uint32_t q4 = 0; q4 < ncp; ++q4)
        if (((b >> (4 * q4)) & 0xFull) == 0) ok |= 1u << q4;
      return ok;
    };
    // back to the core prefix as found (the identity permutation)
    auto restore_core = [&]() {
      S.lvl_ok = 0u;
      if ((uint32_t)lane < L0) {
        const uint32_t v = pl->order[lane];
        const uint32_t c = S.fcore[v];
        S.f[v] = c;
        S.fx[v] = S.fxcore[v];
        S.fo[lane] = c;
      }
    };

    uint32_t l = base_l;
    bool pf_ok = false;  // level k-2's prefetch records belong to its current chunk
    bool go = false;
    bool entered = false;
    // (core permutation tasks exist in the full build only)
    if constexpr (FULL) {
      if (ptask) {
        // a share of another wave's core permutations: its core prefix (the
        // identity) and the permutations to enter.  Level L0-1 stands used up
        // below it, so that stepping back from L0 ends the task.
        if ((uint32_t)lane < L0) {
          const uint32_t v = pl->order[lane];
          S.fcore[v] = S.f[v];
          S.fxcore[v] = S.fx[v];
        }
        S.pvalid = lane_val(tword, HO_W_GIVE_LO);
        S.pidx = 0xFFFFFFFFu;
        S.lvl_ok = 0u;
        base_l = L0 - 1;
        S.cur[L0 - 1] = 0;
        S.len[L0 - 1] = 0;
        S.mask[L0 - 1] = 0;
        l = L0;
        S.cur[L0] = 0;
        S.len[L0] = 0;
        S.mask[L0] = 0;
        go = true;
        entered = true;
      }
    }
    if (!entered) {
      S.lvl_ok = 0u;
      go = init_level(l, !handed);
    }
    if (!go) {
      // an empty first level (a seed with no extension)
    } else {
      if (handed && !ptask) {
        S.cur[l] = lane_val(tword, HO_W_CUR);
        S.len[l] = lane_val(tword, HO_W_END);
        S.chunk[l] = lane_val(tword, HO_W_CHUNK);
        const uint32_t mlo = lane_val(tword, HO_W_GIVE_LO);
        const uint32_t mhi = lane_val(tword, HO_W_GIVE_HI);
        S.mask[l] = ((uint64_t)mhi << 32) | mlo;
      }
      for (;;) {
        uint64_t m = uni64(S.mask[l]);
        uint32_t nl = 0xFFFFFFFFu;  // the level to set up next (none yet)
        if (m == 0) {
          const uint32_t cur = uni(S.cur[l]);
          // the cycle-counter read behind a poll is a scalar memory access
          // that the step waits for: at the last level, every 4th step is
          // often enough (about 10 % of the mid search time)
          if ((l + 1 < k || (cur & (POLL_STEPS * LEAF_UNROLL * GM_WAVE - 1)) == 0) && poll(l)) {
            abort_now = true;
            break;
          }
          if (cur >= uni(S.len[l])) {
            if (l == base_l) break;
            // the core prefix's next permutation that puts every data
            // vertex where the filter admits it (a received task starting
            // at L0 searches its own permuted prefix only).  pidx + 1 <= 16.
            if (core && l == L0 && (uni(S.pvalid) >> (uni(S.pidx) + 1)) != 0u) {
              const uint32_t p0 = uni(S.pidx) + 1;
              const uint32_t p = p0 + (uint32_t)__builtin_ctz(uni(S.pvalid) >> p0);
              S.pidx = p;
              apply_cperm(p);
              l = L0 - 1;
              nl = L0;
            } else {
              if (core && l == L0) restore_core();
              --l;
              continue;
            }
          } else {
            const uint64_t t_ev = CYCLES();
            if (l == k - 1) {
              S.cur[l] = cur + LEAF_UNROLL * GM_WAVE;
              leaf_step(cur);
              TALLY(3, CYCLES() - t_ev);
              continue;
            }
            S.cur[l] = cur + GM_WAVE;
            S.chunk[l] = cur;
            uint32_t c, eidx;
            bool ok;
            m = eval_chunk(l, cur, c, eidx, ok);
            S.mask[l] = m;
            TALLY(2, CYCLES() - t_ev);
            if (l == pf_lvl) {
              pf_ok = true;
              if (m) {
                const uint32_t my_len = prefetch_leaf(l, eidx, c, ok);
                const uint64_t t_pk = CYCLES();
                const bool sh = leaf_packed(l, m, my_len);
                TALLY(3, CYCLES() - t_pk);
                if (abort_now) break;
                if (sh) {
                  l = k - 1;  // the shared last level, walked from its start
                  continue;
                }
                m = uni64(S.mask[l]);
              }
            }
            if (m == 0) continue;
          }
        }
        if (nl == 0xFFFFFFFFu) {
          const uint32_t bit = (uint32_t)__ffsll((unsigned long long)m) - 1;
          S.mask[l] = m & (m - 1);
          if (l == pf_lvl && pf_ok) {
            const uint64_t t0 = CYCLES();
            const bool r = init_leaf_fast(bit);
            TALLY(1, CYCLES() - t0);
            if (r) ++l;
            continue;
          }
          const uint64_t at = uni64(S.drv[l]) + uni(S.chunk[l]) + bit;
          const uint32_t c = uni(col[at] & GM_IDMASK);
          const uint32_t u = uni(pl->order[l]);
          S.f[u] = c;
          S.fo[l] = c;
          S.fx[u] = uni(ext[at]);
          if (core && l + 1 == L0) {
            // a core match: keep it with its vertices' filter words and
            // stand at level L0 used up under a permutation -1, so that the
            // step back above enters the permutations from the identity on
            if ((uint32_t)lane < L0) {
              const uint32_t v = pl->order[lane];
              const uint32_t fv = S.f[v];
              S.fcore[v] = fv;
              S.fxcore[v] = S.fx[v];
              S.ccw[v] = P.cand[(uint64_t)q * n + fv];
            }
            S.pvalid = cperm_valid();
            S.pidx = 0xFFFFFFFFu;
            l = L0;
            S.cur[L0] = 0;
            S.len[L0] = 0;
            S.mask[L0] = 0;
            continue;
          }
          nl = l + 1;
          // set-ups below nl were made under the previous survivor of level l
          S.lvl_ok = uni(S.lvl_ok) & ((2u << nl) - 1u);
          if (P.reenter && reenter(nl)) {
            l = nl;
            continue;
          }
        }
        // one set-up site for every descent (the set-up is inlined where it
        // is called, and each copy costs registers)
        if (init_level(nl, true)) {
          l = nl;
        } else if (core && nl == L0) {
          // no candidate under this permutation: stand at level L0 used up,
          // so that the next pass tries the next permutation
          l = L0;
          S.cur[L0] = 0;
          S.len[L0] = 0;
          S.mask[L0] = 0;
        }
      }
    }
    if (abort_now) break;
    // ---- work item finished
    if (P.seed_open && lane == 0) atomicSub(&P.seed_open[item_seed], 1u);
    if (P.donate) {
      unsigned long long left = 1;
      if (lane == 0) left = atomicAdd(&P.ctr->pending, ~0ull);
      if (lane_val64(left, 0) == 1) broadcast_stop(P, lane);
    }
  }
  flush_acc(P, A, lane);
#undef TALLY
#undef TALLY_ALWAYS
#undef CYCLES
  const uint64_t ss = u_scan, sb = u_bytes;
  if (lane < 6) atomicAdd(&P.ctr->cyc[lane], (unsigned long long)S.tally[lane]);
  if (lane == 0) {
    atomicAdd(&P.ctr->steals, (unsigned long long)S.tally[6]);
    atomicAdd(&P.ctr->dfs_nodes, (unsigned long long)S.tally[7]);
    atomicAdd(&P.ctr->cand_scanned, (unsigned long long)ss);
    atomicAdd(&P.ctr->bytes_alg, (unsigned long long)sb);
  }
}

__global__ void k_upd_open(const GmSeed* __restrict__ seeds, const GmCounters* __restrict__ ctr, uint64_t seed_cap,
                           const uint32_t* __restrict__ seed_open, uint8_t* __restrict__ upd_open,
                           unsigned long long* __restrict__ q_open) {
  const uint64_t ns = ctr->n_seeds < seed_cap ? ctr->n_seeds : seed_cap;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ns; t += (uint64_t)gridDim.x * blockDim.x)
    if (seed_open[t] != 0u) {
      const GmSeed sd = seeds[t];
      if (upd_open) upd_open[sd.os >> 1] = 1u;
      if (q_open) atomicAdd(&q_open[sd.qd >> 8], 1ull);
    }
}

}  // namespace

namespace gm {

unsigned dfs_block_threads() { return DFS_THREADS; }
// Waves per CU that stay resident with the lean build's register use (the
// default launch width); 12 if the runtime cannot tell.
unsigned dfs_resident_waves_per_cu() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_dfs<false>, DFS_THREADS, 0) != hipSuccess ||
      blocks <= 0) {
    (void)hipGetLastError();
    return 12;
  }
  return (unsigned)blocks * DFS_WAVES;
}
unsigned dfs_waves_per_block() { return DFS_WAVES; }
uint32_t dfs_slots(unsigned blocks) { return 8u * ((blocks + 7) / 8) * DFS_WAVES; }

bool dfs_lean(const GmDfsParams& P) {
  return P.coalesce == 0 && P.G.elb == 0 && (P.flags & (GM_F_TUPLES | GM_F_SEED_ATTR)) == 0;
}

void launch_upd_open(const GmSeed* seeds, const GmCounters* ctr, uint64_t seed_cap, const uint32_t* seed_open,
                     uint8_t* upd_open, unsigned long long* q_open, hipStream_t s) {
  const uint64_t want = (seed_cap + 255) / 256;
  const unsigned blocks = (unsigned)(want < 4096 ? (want ? want : 1) : 4096);
  k_upd_open<<<blocks, 256, 0, s>>>(seeds, ctr, seed_cap, seed_open, upd_open, q_open);
}

void launch_dfs(const GmDfsParams& P, unsigned blocks, hipStream_t s) {
  if (dfs_lean(P))
    k_dfs<false><<<blocks, DFS_THREADS, 0, s>>>(P);
  else
    k_dfs<true><<<blocks, DFS_THREADS, 0, s>>>(P);
}

}  // namespace gm
