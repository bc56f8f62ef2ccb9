// Device-side definitions shared by the HIP kernels and the host runtime of
// the batch-dynamic subgraph matching library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define GM_WAVE 64
#define GM_MAX_K 16
#define GM_FLAG 0x80000000u   // neighbour-list entry belongs to the current batch
#define GM_IDMASK 0x7FFFFFFFu
#define GM_EMPTY64 0xFFFFFFFFFFFFFFFFull

// Device error word bits (set by kernels, read by the host after a sync).
#define GM_ERR_RANGE 1u      // vertex id >= n or label out of range
#define GM_ERR_SELFLOOP 2u
#define GM_ERR_CONFLICT 4u   // +e and -e in one batch
#define GM_ERR_CSR 8u        // malformed CSR (order, symmetry, offsets)
#define GM_ERR_RELABEL 16u   // an inserted pair is present under another edge label

// Flags of the search kernel (mirror the public GAMMA_F_* values).
#define GM_F_HASH 2u
#define GM_F_TUPLES 4u
#define GM_F_SEED_ATTR 8u
#define GM_F_PER_UPDATE 16u

// Matching plan of one directed query edge (x, y): the order in which the
// query vertices are matched (order[0] = x, order[1] = y) and, per level l,
// which already-matched query vertices are neighbours of order[l].
// Every field is a full 32-bit word so that a kernel reading a plan through
// the constant address space gets scalar loads.
struct alignas(16) GmPlan {
  uint32_t k;
  uint32_t x, y;
  uint32_t q;               // query index
  uint32_t order[GM_MAX_K];
  uint32_t back[GM_MAX_K];  // bitmask over query vertex ids
  uint32_t lab[GM_MAX_K];   // label of order[l]
  uint32_t pos[GM_MAX_K];   // pos[u] = level at which query vertex u is matched
  uint32_t bofs[GM_MAX_K];  // first slot of level l's neighbour-list records
  uint32_t lslot[GM_MAX_K]; // label-index slot of order[l]'s label
  // Coalesced search (Sec. V-B): with it on, only representative plans are
  // seeded (n_perm >= 1); every match f found from one stands for the
  // matches f o pi of the perms [perm_base, perm_base + n_perm) (the first
  // is the identity).  n_perm = 0: a plan other plans stand for.
  uint32_t n_perm;
  uint32_t perm_base;
  uint32_t el;  // edge label of the query edge (x, y) (0 without edge labels)
  // Coalesced search over a k-degenerated automorphic subgraph (Sec. V-B,
  // the degree-1 query vertices removed): a plan of a core edge matches the
  // n_core core vertices first; a representative (n_cperm >= 2) then
  // re-enters level n_core once per permutation of its core prefix by the
  // perms [cperm_base, cperm_base + n_cperm) (the first is the identity);
  // n_cperm = 0: a core plan a representative stands for; 1: ordinary.
  uint32_t n_core;
  uint32_t n_cperm;
  uint32_t cperm_base;
  // Candidate test of query vertex u in a representative's core search:
  // the data vertex must pass the filter of some query vertex in omask[u]
  // (the positions pi^-1(u) over its permutations: any of them is where a
  // permuted prefix may put it).  1 << u otherwise.
  uint32_t omask[GM_MAX_K];
  // Injectivity: a candidate of level l carries order[l]'s label, so it can
  // only equal the data vertex of an earlier level with the same label.
  // Bit j (j < l) set: level j's query vertex has order[l]'s label.
  uint32_t injm[GM_MAX_K];
};

#define GM_MAX_PERM 16

// A label-preserving automorphism pi of a query, as its forward map and its
// inverse (query vertex -> query vertex).
struct GmPerm {
  uint32_t fwd[GM_MAX_K];
  uint32_t inv[GM_MAX_K];
};

// Per query: plan range and size.
struct GmQueryDev {
  uint32_t k;
  uint32_t plan_base;  // index of the first GmPlan of this query
  uint32_t n_plans;    // 2 * |E(Q)|
  uint32_t pad;
};

// Candidate-filter requirement list entry: query vertex (q, u) of a given
// label needs at least `cnt` neighbours of label `lab` through edges of
// label `el`.
struct GmReq {
  uint16_t lab;
  uint16_t cnt;
  uint16_t el;
  uint16_t pad;
};
struct GmFilterEntry {
  uint32_t q;
  uint32_t u;
  uint32_t req_off;
  uint32_t req_n;
};

// A search seed: batch edge `ord` (sign in bit 0 of os) mapped onto the
// directed query edge `dqe` of query q, as (x -> a, y -> b).
struct alignas(16) GmSeed {
  uint32_t qd;  // q << 8 | dqe
  uint32_t os;  // ord << 1 | sign (1 = insertion)
  uint32_t a, b;
};

__host__ __device__ inline uint64_t gm_mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

#define GM_GOLDEN 0x9E3779B97F4A7C15ull

// Slot of an undirected edge key in the batch hash.
__device__ inline uint32_t gm_hash_slot(uint64_t key, uint32_t mask) {
  return (uint32_t)(gm_mix64(key ^ 0x5851F42D4C957F2Dull) >> 20) & mask;
}

__device__ inline uint64_t gm_edge_key(uint32_t a, uint32_t b) {
  return a < b ? (((uint64_t)a << 32) | b) : (((uint64_t)b << 32) | a);
}

// ---------------------------------------------------------------------------
// Launch helpers implemented in the .hip files (host-callable).

namespace gm {

// Exclusive scans; out has n + 1 entries, out[n] = total.
void scan_u32(const uint32_t* in, uint32_t* out, size_t n, uint32_t* tmp, hipStream_t s);
void scan_u64(const uint64_t* in, uint64_t* out, size_t n, uint64_t* tmp, hipStream_t s);
size_t scan_tmp_elems(size_t n);

// LSD radix sort of 64-bit keys over their low `bits` bits (stable).
// `keys` and `tmp` hold n keys; the result ends in `keys`.  `hist` needs
// radix_hist_elems(n) uint32 elements.
void radix_sort_u64(uint64_t* keys, uint64_t* tmp, size_t n, int bits, uint32_t* hist,
                    uint32_t* hist_scan, uint32_t* scan_tmp, hipStream_t s);
size_t radix_hist_elems(size_t n);

void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
void fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s);

}  // namespace gm
