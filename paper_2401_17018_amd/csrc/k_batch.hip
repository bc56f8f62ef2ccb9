// Batch pipeline: canonicalisation, batch hash, delta-merge and commit.
//
// A batch (Def. 1) is canonicalised on the device: updates become
// (lo, hi, op) in external ids, are sorted, duplicates collapse, +e/-e pairs
// are rejected and no-ops (+e with e in E, -e with e not in E) are skipped.
// The survivors get ord = rank in ascending (lo, hi) order, the total order
// that the rule after Algorithm 1 (Sec. IV-C) needs.  The batch hash maps an
// undirected internal edge to (ord, sign).  With edge labels an update
// names (lo, hi, e): the key holds e between the pair and the op, two
// updates of one pair must agree in e and op (else the batch conflicts), so
// a pair occurs at most once in the canonical batch and the hash stays keyed
// by the pair; presence is tested in the row of label e, and the directed
// entries go to rows (v << elb) | e.  The graph stays simple: inserting a
// pair that is present under another label is an error.
//
// Delta-merge (the update step of Sec. IV-A): every touched row is written
// twice into fresh arena space: R1 = the row of G u I with batch entries
// flagged (bit 31), searched by both passes, and R2 = the row of G', which
// becomes the row at commit.  Each output entry is placed independently
// (its rank among the row's old entries and the batch entries), so the work
// is load-balanced over all entries of all touched rows.
#include "dev_common.h"
#include "kernels.h"

namespace {

__device__ inline uint64_t lb_row(const uint32_t* col, uint64_t a, uint64_t len, uint32_t key) {
  uint64_t lo = 0, hi = len;
  while (lo < hi) {
    uint64_t mid = lo + ((hi - lo) >> 1);
    if ((col[a + mid] & GM_IDMASK) < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__global__ void k_canon_keys(const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst,
                             const uint8_t* __restrict__ op, const uint32_t* __restrict__ elab, uint32_t n_upd,
                             uint32_t n, int eb, uint32_t elb, uint32_t n_el, uint64_t* __restrict__ keys,
                             GmCounters* ctr) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_upd; i += gridDim.x * blockDim.x) {
    uint32_t s = src[i], d = dst[i];
    const uint32_t el = elab ? elab[i] : 0u;
    uint32_t e = 0;
    if (s >= n || d >= n || el >= n_el) e |= GM_ERR_RANGE;
    if (s == d) e |= GM_ERR_SELFLOOP;
    if (e) {
      atomicOr(&ctr->err, e);
      keys[i] = 0;
      continue;
    }
    uint64_t lo = s < d ? s : d, hi = s < d ? d : s;
    keys[i] = (((((lo << eb) | hi) << elb) | el) << 1) | (uint64_t)(op[i] ? 1 : 0);
  }
}

__global__ void k_canon_classify(const uint64_t* __restrict__ keys, uint32_t n_upd, int eb,
                                 GmGraphDev G, uint32_t* __restrict__ keep, GmCounters* ctr) {
  const uint32_t elb = G.elb;
  const uint64_t tail = (2ull << elb) - 1;  // label and op bits
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n_upd; j += gridDim.x * blockDim.x) {
    uint64_t key = keys[j];
    uint64_t pair = key >> (elb + 1);
    uint32_t op = (uint32_t)(key & 1);
    uint32_t k = 0;
    if (j > 0 && (keys[j - 1] >> (elb + 1)) == pair) {
      if ((keys[j - 1] & tail) != (key & tail))
        atomicOr(&ctr->err, GM_ERR_CONFLICT);
      else
        atomicAdd(&ctr->n_dup, 1u);
    } else {
      uint32_t lo = (uint32_t)(pair >> eb), hi = (uint32_t)(pair & ((1ull << eb) - 1));
      uint32_t a = G.new_of_old[lo], b = G.new_of_old[hi];
      const uint32_t ra = (a << elb) | (uint32_t)((key >> 1) & ((1ull << elb) - 1));
      uint64_t off = G.row_off[ra], len = G.row_len[ra];
      uint64_t p = lb_row(G.col, off, len, b);
      bool present = p < len && (G.col[off + p] & GM_IDMASK) == b;
      // the graph stays simple: an insertion of a pair that another label's
      // row already holds is rejected
      for (uint32_t e2 = 0; op && !present && elb && e2 < G.n_el; ++e2) {
        const uint32_t r2 = (a << elb) | e2;
        if (r2 == ra) continue;
        const uint64_t o2 = G.row_off[r2], l2 = G.row_len[r2];
        const uint64_t p2 = lb_row(G.col, o2, l2, b);
        if (p2 < l2 && (G.col[o2 + p2] & GM_IDMASK) == b) atomicOr(&ctr->err, GM_ERR_RELABEL);
      }
      bool noop = op ? present : !present;
      if (noop)
        atomicAdd(&ctr->n_noop, 1u);
      else
        k = 1;
    }
    keep[j] = k;
  }
}

__device__ inline void hash_insert(GmBatchHash H, uint64_t key, uint32_t val) {
  uint32_t slot = gm_hash_slot(key, H.mask);
  for (uint32_t probe = 0; probe <= H.mask; ++probe) {
    unsigned long long prev =
        atomicCAS((unsigned long long*)&H.keys[slot], (unsigned long long)GM_EMPTY64, (unsigned long long)key);
    if (prev == GM_EMPTY64 || prev == key) {
      H.vals[slot] = val;
      return;
    }
    slot = (slot + 1) & H.mask;
  }
}

__global__ void k_canon_emit(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ keep,
                             const uint32_t* __restrict__ ords, uint32_t n_upd, int eb, GmGraphDev G,
                             uint32_t* __restrict__ canon_lo, uint32_t* __restrict__ canon_hi,
                             uint8_t* __restrict__ canon_sign, uint32_t* __restrict__ canon_a,
                             uint32_t* __restrict__ canon_b, uint32_t* __restrict__ canon_e, GmBatchHash H,
                             uint64_t* __restrict__ dkeys) {
  const int ib = G.idbits;
  const uint32_t elb = G.elb;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n_upd; j += gridDim.x * blockDim.x) {
    if (!keep[j]) continue;
    uint64_t key = keys[j];
    uint32_t o = ords[j];
    uint32_t op = (uint32_t)(key & 1);
    const uint32_t el = (uint32_t)((key >> 1) & ((1ull << elb) - 1));
    uint64_t pair = key >> (elb + 1);
    uint32_t lo = (uint32_t)(pair >> eb), hi = (uint32_t)(pair & ((1ull << eb) - 1));
    uint32_t a = G.new_of_old[lo], b = G.new_of_old[hi];
    canon_lo[o] = lo;
    canon_hi[o] = hi;
    canon_sign[o] = (uint8_t)op;
    canon_a[o] = a;
    canon_b[o] = b;
    if (canon_e) canon_e[o] = el;
    hash_insert(H, gm_edge_key(a, b), (o << 1) | op);
    // directed entries keyed by (row, neighbour, op); the row of a for label el
    const uint64_t ra = ((uint64_t)a << elb) | el, rb = ((uint64_t)b << elb) | el;
    dkeys[2 * (uint64_t)o] = (ra << (ib + 1)) | ((uint64_t)b << 1) | op;
    dkeys[2 * (uint64_t)o + 1] = (rb << (ib + 1)) | ((uint64_t)a << 1) | op;
  }
}

// Sorted directed batch entries (src, dst, op): runs per src.  vals[j] =
// run-start flag | insert flag << 32, scanned to run index and insert rank.
__global__ void k_runs_flags(const uint64_t* __restrict__ dkeys, uint32_t N, int ib,
                             uint64_t* __restrict__ vals) {
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < N; j += gridDim.x * blockDim.x) {
    uint64_t k = dkeys[j];
    uint64_t src = k >> (ib + 1);
    uint64_t start = (j == 0 || (dkeys[j - 1] >> (ib + 1)) != src) ? 1 : 0;
    vals[j] = start | ((k & 1) << 32);
  }
}

__global__ void k_runs_fill(const uint64_t* __restrict__ dkeys, const uint64_t* __restrict__ runscan,
                            uint32_t N, int ib, uint32_t* __restrict__ touched,
                            uint32_t* __restrict__ run_start, uint32_t* __restrict__ run_end) {
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < N; j += gridDim.x * blockDim.x) {
    uint64_t src = dkeys[j] >> (ib + 1);
    uint32_t t = (uint32_t)runscan[j + 1] - 1;
    if (j == 0 || (dkeys[j - 1] >> (ib + 1)) != src) {
      touched[t] = (uint32_t)src;
      run_start[t] = j;
    }
    if (j == N - 1 || (dkeys[j + 1] >> (ib + 1)) != src) run_end[t] = j + 1;
  }
}

__device__ inline uint32_t ins_prefix(const uint64_t* runscan, uint32_t j) {
  return (uint32_t)(runscan[j] >> 32);
}

__global__ void k_touched_sizes(const uint32_t* __restrict__ touched,
                                const uint32_t* __restrict__ run_start,
                                const uint32_t* __restrict__ run_end,
                                const uint64_t* __restrict__ runscan, uint32_t n_touched,
                                GmGraphDev G, uint64_t* __restrict__ sizes) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n_touched; t += gridDim.x * blockDim.x) {
    uint32_t v = touched[t];
    uint32_t rs = run_start[t], re = run_end[t];
    uint32_t ins = ins_prefix(runscan, re) - ins_prefix(runscan, rs);
    sizes[t] = (uint64_t)G.row_len[v] + ins;
  }
}

// Thread per entry of the R1 rows (G u I, flagged) of all touched vertices;
// also writes the matching R2 (G') entry.
__global__ __launch_bounds__(256) void k_merge(const uint64_t* __restrict__ dkeys,
                                               const uint64_t* __restrict__ runscan,
                                               const uint32_t* __restrict__ touched,
                                               const uint32_t* __restrict__ run_start,
                                               const uint32_t* __restrict__ run_end,
                                               const uint64_t* __restrict__ r1off,
                                               uint32_t n_touched, uint64_t r1_total, uint64_t base1,
                                               uint64_t base2, int ib, GmGraphDev G) {
  const uint64_t idmask = (1ull << ib) - 1;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < r1_total;
       j += (uint64_t)gridDim.x * blockDim.x) {
    // touched row t with r1off[t] <= j < r1off[t+1]
    uint32_t lo = 0, hi = n_touched;
    while (hi - lo > 1) {
      uint32_t mid = (lo + hi) >> 1;
      if (r1off[mid] <= j)
        lo = mid;
      else
        hi = mid;
    }
    const uint32_t t = lo;
    const uint64_t jj = j - r1off[t];
    const uint32_t v = touched[t];
    const uint32_t L = G.row_len[v];
    const uint64_t off = G.row_off[v];
    const uint32_t rs = run_start[t], re = run_end[t];
    const uint32_t insb = ins_prefix(runscan, rs);
    const uint64_t o1 = base1 + r1off[t];
    const uint64_t o2 = base2 + r1off[t] - (uint64_t)(rs - insb);  // minus deletions before row t
    if (jj < L) {
      const uint32_t x = G.col[off + jj];
      uint32_t a = rs, b = re;  // first run entry with dst >= x
      while (a < b) {
        uint32_t mid = (a + b) >> 1;
        if (((dkeys[mid] >> 1) & idmask) < x)
          a = mid + 1;
        else
          b = mid;
      }
      const uint32_t r = a - rs;
      const uint32_t ins_lt = ins_prefix(runscan, a) - insb;
      const uint32_t del_lt = r - ins_lt;
      const bool deleted = a < re && ((dkeys[a] >> 1) & idmask) == x && !(dkeys[a] & 1);
      const uint32_t xe = G.ext[off + jj];
      G.col[o1 + jj + ins_lt] = deleted ? (x | GM_FLAG) : x;
      G.ext[o1 + jj + ins_lt] = xe;
      if (!deleted) {
        G.col[o2 + jj + ins_lt - del_lt] = x;
        G.ext[o2 + jj + ins_lt - del_lt] = xe;
      }
    } else {
      const uint32_t i = (uint32_t)(jj - L);  // i-th insertion of the run
      uint32_t a = rs, b = re;                // first entry whose inclusive insert count > i
      while (a < b) {
        uint32_t mid = (a + b) >> 1;
        if (ins_prefix(runscan, mid + 1) - insb <= i)
          a = mid + 1;
        else
          b = mid;
      }
      const uint32_t r = a - rs;
      const uint32_t x = (uint32_t)((dkeys[a] >> 1) & idmask);
      const uint64_t p = lb_row(G.col, off, L, x);
      const uint32_t xe = G.old_of_new[x];
      G.col[o1 + p + i] = x | GM_FLAG;
      G.ext[o1 + p + i] = xe;
      G.col[o2 + p + i - (r - i)] = x;
      G.ext[o2 + p + i - (r - i)] = xe;
    }
  }
}

__global__ void k_rows_set(const uint32_t* __restrict__ touched, const uint32_t* __restrict__ run_start,
                           const uint32_t* __restrict__ run_end, const uint64_t* __restrict__ runscan,
                           const uint64_t* __restrict__ r1off, uint32_t n_touched, uint64_t base1,
                           uint64_t base2, GmGraphDev G, uint64_t* __restrict__ r2_off,
                           uint32_t* __restrict__ r2_len) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n_touched; t += gridDim.x * blockDim.x) {
    uint32_t v = touched[t];
    uint32_t rs = run_start[t], re = run_end[t];
    uint32_t insb = ins_prefix(runscan, rs);
    uint32_t ins = ins_prefix(runscan, re) - insb;
    uint32_t del = (re - rs) - ins;
    uint64_t len1 = r1off[t + 1] - r1off[t];
    r2_off[t] = base2 + r1off[t] - (uint64_t)(rs - insb);
    r2_len[t] = (uint32_t)(len1 - del);
    G.row_off[v] = base1 + r1off[t];
    G.row_len[v] = (uint32_t)len1;
  }
}

__global__ void k_rows_commit(const uint32_t* __restrict__ touched, const uint64_t* __restrict__ r2_off,
                              const uint32_t* __restrict__ r2_len, uint32_t n_touched, GmGraphDev G) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n_touched; t += gridDim.x * blockDim.x) {
    uint32_t v = touched[t];
    G.row_off[v] = r2_off[t];
    G.row_len[v] = r2_len[t];
  }
}

// Commit the G' rows, or put the saved rows back when a search launch of the
// batch passed its deadline.
__global__ void k_rows_finish(const uint32_t* __restrict__ touched, const uint64_t* __restrict__ r2_off,
                              const uint32_t* __restrict__ r2_len, const uint64_t* __restrict__ r0_off,
                              const uint32_t* __restrict__ r0_len, uint32_t n_touched, GmGraphDev G,
                              const GmCounters* __restrict__ ctr, uint32_t restore) {
  const bool back = restore || ctr->aborted != 0 || ctr->timed_out != 0;
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n_touched; t += gridDim.x * blockDim.x) {
    const uint32_t v = touched[t];
    G.row_off[v] = back ? r0_off[t] : r2_off[t];
    G.row_len[v] = back ? r0_len[t] : r2_len[t];
  }
}

__global__ void k_rows_save(const uint32_t* __restrict__ touched, uint32_t n_touched, GmGraphDev G,
                            uint64_t* __restrict__ r0_off, uint32_t* __restrict__ r0_len) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n_touched; t += gridDim.x * blockDim.x) {
    const uint32_t v = touched[t];
    r0_off[t] = G.row_off[v];
    r0_len[t] = G.row_len[v];
  }
}

unsigned grid_for(uint64_t work, unsigned per_block) {
  uint64_t b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (unsigned)b;
}

}  // namespace

namespace gm {

void launch_canon_keys(const uint32_t* src, const uint32_t* dst, const uint8_t* op, const uint32_t* elab,
                       uint32_t n_upd, uint32_t n, int eb, uint32_t elb, uint32_t n_el, uint64_t* keys,
                       GmCounters* ctr, hipStream_t s) {
  if (!n_upd) return;
  k_canon_keys<<<grid_for(n_upd, 256), 256, 0, s>>>(src, dst, op, elab, n_upd, n, eb, elb, n_el, keys, ctr);
}

void launch_canon_classify(const uint64_t* keys, uint32_t n_upd, int eb, GmGraphDev G,
                           uint32_t* keep, GmCounters* ctr, hipStream_t s) {
  if (!n_upd) return;
  k_canon_classify<<<grid_for(n_upd, 256), 256, 0, s>>>(keys, n_upd, eb, G, keep, ctr);
}

void launch_canon_emit(const uint64_t* keys, const uint32_t* keep, const uint32_t* ords,
                       uint32_t n_upd, int eb, GmGraphDev G, uint32_t* canon_lo, uint32_t* canon_hi,
                       uint8_t* canon_sign, uint32_t* canon_a, uint32_t* canon_b, uint32_t* canon_e,
                       GmBatchHash H, uint64_t* dkeys, hipStream_t s) {
  if (!n_upd) return;
  k_canon_emit<<<grid_for(n_upd, 256), 256, 0, s>>>(keys, keep, ords, n_upd, eb, G, canon_lo, canon_hi,
                                                   canon_sign, canon_a, canon_b, canon_e, H, dkeys);
}

void launch_runs_flags(const uint64_t* dkeys, uint32_t N, int ib, uint64_t* vals, hipStream_t s) {
  if (!N) return;
  k_runs_flags<<<grid_for(N, 256), 256, 0, s>>>(dkeys, N, ib, vals);
}

void launch_runs_fill(const uint64_t* dkeys, const uint64_t* runscan, uint32_t N, int ib,
                      uint32_t* touched, uint32_t* run_start, uint32_t* run_end, hipStream_t s) {
  if (!N) return;
  k_runs_fill<<<grid_for(N, 256), 256, 0, s>>>(dkeys, runscan, N, ib, touched, run_start, run_end);
}

void launch_touched_sizes(const uint32_t* touched, const uint32_t* run_start, const uint32_t* run_end,
                          const uint64_t* runscan, uint32_t n_touched, GmGraphDev G, uint64_t* sizes,
                          hipStream_t s) {
  if (!n_touched) return;
  k_touched_sizes<<<grid_for(n_touched, 256), 256, 0, s>>>(touched, run_start, run_end, runscan,
                                                          n_touched, G, sizes);
}

void launch_merge(const uint64_t* dkeys, const uint64_t* runscan, const uint32_t* touched,
                  const uint32_t* run_start, const uint32_t* run_end, const uint64_t* r1off,
                  uint32_t n_touched, uint64_t r1_total, uint64_t base1, uint64_t base2, int ib,
                  GmGraphDev G, hipStream_t s) {
  if (!r1_total) return;
  k_merge<<<grid_for(r1_total, 256), 256, 0, s>>>(dkeys, runscan, touched, run_start, run_end, r1off,
                                                 n_touched, r1_total, base1, base2, ib, G);
}

void launch_rows_set(const uint32_t* touched, const uint32_t* run_start, const uint32_t* run_end,
                     const uint64_t* runscan, const uint64_t* r1off, uint32_t n_touched,
                     uint64_t base1, uint64_t base2, GmGraphDev G, uint64_t* r2_off,
                     uint32_t* r2_len, hipStream_t s) {
  if (!n_touched) return;
  k_rows_set<<<grid_for(n_touched, 256), 256, 0, s>>>(touched, run_start, run_end, runscan, r1off,
                                                     n_touched, base1, base2, G, r2_off, r2_len);
}

void launch_rows_finish(const uint32_t* touched, const uint64_t* r2_off, const uint32_t* r2_len,
                        const uint64_t* r0_off, const uint32_t* r0_len, uint32_t n_touched, GmGraphDev G,
                        const GmCounters* ctr, uint32_t restore, hipStream_t s) {
  if (!n_touched) return;
  k_rows_finish<<<grid_for(n_touched, 256), 256, 0, s>>>(touched, r2_off, r2_len, r0_off, r0_len, n_touched,
                                                         G, ctr, restore);
}

void launch_rows_save(const uint32_t* touched, uint32_t n_touched, GmGraphDev G, uint64_t* r0_off,
                      uint32_t* r0_len, hipStream_t s) {
  if (!n_touched) return;
  k_rows_save<<<grid_for(n_touched, 256), 256, 0, s>>>(touched, n_touched, G, r0_off, r0_len);
}

void launch_rows_commit(const uint32_t* touched, const uint64_t* r2_off, const uint32_t* r2_len,
                        uint32_t n_touched, GmGraphDev G, hipStream_t s) {
  if (!n_touched) return;
  k_rows_commit<<<grid_for(n_touched, 256), 256, 0, s>>>(touched, r2_off, r2_len, n_touched, G);
}

}  // namespace gm
