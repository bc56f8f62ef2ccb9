// Graph loading, relabelling and arena maintenance.
//
// Data layout (device):
//   Vertices are renumbered so that internal ids are grouped by label
//   (internal id = rank of (label, external id)).  Every neighbour list is
//   sorted by internal id, so the neighbours of one label form a contiguous
//   subrange: the candidate lists of the search (candidates must carry the
//   query vertex's label, Def. 2) and the neighbourhood label counts of the
//   candidate filter (Sec. IV-B) are found by binary search instead of a scan.
//   Row v lives at col[row_off[v] .. row_off[v] + row_len[v]) in an arena; a
//   batch writes the rows it changes to fresh arena space (Sec. V-C replaces
//   the paper's packed memory array).  With edge labels (Sec. II-A) vertex v
//   has one row per label e, row id (v << elb) | e, so the neighbours of one
//   vertex label through one edge label are again one contiguous subrange.
#include "dev_common.h"
#include "kernels.h"

namespace {

__device__ inline uint64_t lower_bound_u32(const uint32_t* p, uint64_t lo, uint64_t hi, uint32_t key) {
  while (lo < hi) {
    uint64_t mid = lo + ((hi - lo) >> 1);
    if ((p[mid] & GM_IDMASK) < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// One wave per vertex: offsets, order, range, self loops, symmetry, labels.
// With edge labels (elab != nullptr) the mirror entry must carry the same
// label (the graph stays simple: one edge, with one label, per pair).
__global__ __launch_bounds__(256) void k_validate_csr(const uint64_t* __restrict__ rp,
                                                      const uint32_t* __restrict__ col,
                                                      const uint32_t* __restrict__ labels,
                                                      const uint32_t* __restrict__ elab, uint32_t n_el,
                                                      uint32_t n, uint64_t nnz,
                                                      uint32_t* __restrict__ err) {
  const int lane = threadIdx.x & 63;
  const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t v = gw; v < n; v += nw) {
    uint64_t a = rp[v], b = rp[v + 1];
    if (lane == 0) {
      if (labels[v] > 0xFFFFu) atomicOr(err, GM_ERR_RANGE);
      if (v == 0 && a != 0) atomicOr(err, GM_ERR_CSR);
      if (v == n - 1 && b != nnz) atomicOr(err, GM_ERR_CSR);
    }
    if (a > b || b > nnz) {
      if (lane == 0) atomicOr(err, GM_ERR_CSR);
      continue;
    }
    for (uint64_t j = a + lane; j < b; j += 64) {
      uint32_t x = col[j];
      const uint32_t el = elab ? elab[j] : 0u;
      uint32_t e = 0;
      if (x >= n || el >= n_el) {
        e |= GM_ERR_RANGE;
      } else {
        if (x == v) e |= GM_ERR_SELFLOOP;
        if (j > a && col[j - 1] >= x) e |= GM_ERR_CSR;
        uint64_t xa = rp[x], xb = rp[x + 1];
        if (xa > xb || xb > nnz) {
          e |= GM_ERR_CSR;
        } else {
          uint64_t p = lower_bound_u32(col, xa, xb, (uint32_t)v);
          if (p >= xb || col[p] != (uint32_t)v || (elab && elab[p] != el)) e |= GM_ERR_CSR;
        }
      }
      if (e) atomicOr(err, e);
    }
  }
}

__global__ void k_relabel_keys(const uint32_t* __restrict__ labels, uint32_t n,
                               uint64_t* __restrict__ keys) {
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (uint64_t)gridDim.x * blockDim.x)
    keys[v] = ((uint64_t)(labels[v] & 0xFFFFu) << 32) | v;
}

__global__ void k_relabel_apply(const uint64_t* __restrict__ sorted, uint32_t n,
                                uint32_t* __restrict__ new_of_old, uint32_t* __restrict__ old_of_new,
                                uint16_t* __restrict__ vlabel) {
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t key = sorted[p];
    uint32_t v = (uint32_t)key;
    new_of_old[v] = (uint32_t)p;
    old_of_new[p] = v;
    vlabel[p] = (uint16_t)(key >> 32);
  }
}

// label_start[l] = first internal id whose label is >= l, for l in [0, slots].
__global__ void k_label_start(const uint16_t* __restrict__ vlabel, uint32_t n, uint32_t slots,
                              uint32_t* __restrict__ label_start) {
  for (uint32_t l = blockIdx.x * blockDim.x + threadIdx.x; l <= slots; l += gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
      uint32_t mid = lo + ((hi - lo) >> 1);
      if (vlabel[mid] < l)
        lo = mid + 1;
      else
        hi = mid;
    }
    label_start[l] = lo;
  }
}

// Keys map[src] << idbits | map[dst] for every entry of a CSR (one wave per row).
// With flag_aware, entries carry the batch flag bit, which is stripped.
// With edge labels (elab, elb > 0) the source part is the row id
// (map[src] << elb | label).
__global__ __launch_bounds__(256) void k_csr_keys(const uint64_t* __restrict__ row_off,
                                                  const uint32_t* __restrict__ row_len,
                                                  const uint64_t* __restrict__ rp,
                                                  const uint32_t* __restrict__ col,
                                                  const uint32_t* __restrict__ map, uint32_t n,
                                                  int idbits, const uint64_t* __restrict__ out_off,
                                                  uint64_t* __restrict__ keys, const uint32_t* __restrict__ elab,
                                                  uint32_t elb) {
  const int lane = threadIdx.x & 63;
  const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t v = gw; v < n; v += nw) {
    uint64_t a, len;
    if (rp) {
      a = rp[v];
      len = rp[v + 1] - a;
    } else {
      a = row_off[v];
      len = row_len[v];
    }
    uint64_t src = (uint64_t)map[v] << idbits;
    uint64_t o = out_off ? out_off[v] : a;
    if (elab) {
      for (uint64_t j = lane; j < len; j += 64)
        keys[o + j] = ((((uint64_t)map[v] << elb) | elab[a + j]) << idbits) | map[col[a + j] & GM_IDMASK];
    } else {
      for (uint64_t j = lane; j < len; j += 64) keys[o + j] = src | map[col[a + j] & GM_IDMASK];
    }
  }
}

// Row lengths from sorted keys (row << idbits | neighbour): deg[row] += 1.
__global__ void k_row_hist(const uint64_t* __restrict__ keys, uint64_t nnz, int idbits, uint64_t* __restrict__ deg) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += (uint64_t)gridDim.x * blockDim.x)
    atomicAdd((unsigned long long*)&deg[keys[i] >> idbits], 1ull);
}

// Export keys of every row r = (v << elb) | e (one wave per row):
// old[v] << (idbits + elb) | old[w] << elb | e, placed at out_off[r].
__global__ __launch_bounds__(256) void k_row_keys_el(const uint64_t* __restrict__ row_off,
                                                     const uint32_t* __restrict__ row_len,
                                                     const uint32_t* __restrict__ col,
                                                     const uint32_t* __restrict__ old_of_new, uint32_t rows,
                                                     uint32_t elb, int idbits, const uint64_t* __restrict__ out_off,
                                                     uint64_t* __restrict__ keys) {
  const int lane = threadIdx.x & 63;
  const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t r = gw; r < rows; r += nw) {
    const uint64_t a = row_off[r], o = out_off[r];
    const uint32_t len = row_len[r];
    const uint64_t e = r & ((1ull << elb) - 1);
    const uint64_t src = (uint64_t)old_of_new[r >> elb] << (idbits + elb);
    for (uint32_t j = lane; j < len; j += 64)
      keys[o + j] = src | ((uint64_t)old_of_new[col[a + j] & GM_IDMASK] << elb) | e;
  }
}

__global__ void k_keys_split_el(const uint64_t* __restrict__ keys, uint64_t nnz, int idbits, uint32_t elb,
                                uint32_t* __restrict__ col_out, uint32_t* __restrict__ elab_out) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[i];
    col_out[i] = (uint32_t)((k >> elb) & ((1ull << idbits) - 1));
    elab_out[i] = (uint32_t)(k & ((1ull << elb) - 1));
  }
}

// deg_out[map[v]] = sum of the lengths of v's 2^elb rows.
__global__ void k_deg_rows(const uint32_t* __restrict__ row_len, const uint32_t* __restrict__ map, uint32_t n,
                           uint32_t elb, uint64_t* __restrict__ deg_out) {
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t d = 0;
    for (uint32_t e = 0; e < (1u << elb); ++e) d += row_len[(v << elb) | e];
    deg_out[map ? map[v] : v] = d;
  }
}

__global__ void k_csr_extract(const uint64_t* __restrict__ keys, uint64_t nnz, uint64_t idmask,
                              uint32_t* __restrict__ col_out) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz;
       i += (uint64_t)gridDim.x * blockDim.x)
    col_out[i] = (uint32_t)(keys[i] & idmask);
}

// deg_out[map[v]] = degree of v (from a CSR row_ptr or from row_len).
__global__ void k_deg_mapped(const uint64_t* __restrict__ rp, const uint32_t* __restrict__ row_len,
                             const uint32_t* __restrict__ map, uint32_t n,
                             uint64_t* __restrict__ deg_out) {
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t d = rp ? rp[v + 1] - rp[v] : row_len[v];
    deg_out[map ? map[v] : v] = d;
  }
}

__global__ void k_rows_from_scan(const uint64_t* __restrict__ offs, const uint64_t* __restrict__ deg,
                                 uint32_t n, uint64_t base, uint64_t* __restrict__ row_off,
                                 uint32_t* __restrict__ row_len) {
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (uint64_t)gridDim.x * blockDim.x) {
    row_off[v] = base + offs[v];
    if (row_len) row_len[v] = (uint32_t)deg[v];
  }
}

// Copy every row to its new offset (one wave per row).
__global__ __launch_bounds__(256) void k_copy_rows(const uint64_t* __restrict__ row_off,
                                                   const uint32_t* __restrict__ row_len,
                                                   const uint32_t* __restrict__ src,
                                                   const uint64_t* __restrict__ new_off,
                                                   uint32_t* __restrict__ dst, uint32_t n) {
  const int lane = threadIdx.x & 63;
  const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t v = gw; v < n; v += nw) {
    uint64_t a = row_off[v], o = new_off[v];
    uint32_t len = row_len[v];
    for (uint32_t j = lane; j < len; j += 64) dst[o + j] = src[a + j];
  }
}

__global__ void k_u32_to_u64(const uint32_t* __restrict__ in, uint64_t* __restrict__ out, uint32_t n) {
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (uint64_t)gridDim.x * blockDim.x)
    out[v] = in[v];
}

__global__ void k_gather_ext(const uint32_t* __restrict__ col, const uint32_t* __restrict__ o2n,
                             uint64_t nnz, uint32_t* __restrict__ ext) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz;
       i += (uint64_t)gridDim.x * blockDim.x)
    ext[i] = o2n[col[i] & GM_IDMASK];
}

// Vertex deletion as edge deletions (the paper's reduction, Sec. II-A):
// the row length of every deleted vertex (external id; ids >= n raise the
// range error and count 0), marking it in an n-bit map; then its incident
// edges as (v, w, delete).
__global__ void k_vdel_len(GmGraphDev G, const uint32_t* __restrict__ vdel, uint32_t nv,
                           uint64_t* __restrict__ len, uint32_t* __restrict__ mark, uint32_t* __restrict__ err) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += gridDim.x * blockDim.x) {
    const uint32_t v = vdel[i];
    if (v >= G.n) {
      atomicOr(err, GM_ERR_RANGE);
      len[i] = 0;
    } else {
      const uint32_t vi = G.new_of_old[v];
      uint64_t d = 0;
      for (uint32_t e = 0; e < (1u << G.elb); ++e) d += G.row_len[(vi << G.elb) | e];
      len[i] = d;
      atomicOr(&mark[v >> 5], 1u << (v & 31));
    }
  }
}

// an explicit insertion that touches a deleted vertex cannot be ordered
// against the deletion: conflict (ids >= n are left to the batch's own
// range check)
__global__ void k_vdel_check(const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst,
                             const uint8_t* __restrict__ op, uint32_t n_upd, uint32_t n,
                             const uint32_t* __restrict__ mark, uint32_t* __restrict__ err) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_upd; i += gridDim.x * blockDim.x) {
    if (!op[i]) continue;
    const uint32_t a = src[i], b = dst[i];
    const bool hit = (a < n && ((mark[a >> 5] >> (a & 31)) & 1u)) || (b < n && ((mark[b >> 5] >> (b & 31)) & 1u));
    if (hit) atomicOr(err, GM_ERR_CONFLICT);
  }
}

__global__ void k_vdel_expand(GmGraphDev G, const uint32_t* __restrict__ vdel, uint32_t nv,
                              const uint64_t* __restrict__ offs, uint32_t* __restrict__ src,
                              uint32_t* __restrict__ dst, uint8_t* __restrict__ op, uint32_t* __restrict__ elab) {
  // one wave per deleted vertex, lanes over its rows (one per edge label)
  const uint32_t lane = threadIdx.x & 63;
  for (uint32_t i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < nv; i += (gridDim.x * blockDim.x) >> 6) {
    const uint32_t v = vdel[i];
    if (v >= G.n) continue;
    const uint32_t vi = G.new_of_old[v];
    uint64_t o = offs[i];
    for (uint32_t e = 0; e < (1u << G.elb); ++e) {
      const uint32_t r = (vi << G.elb) | e;
      const uint64_t base = G.row_off[r];
      const uint32_t len = G.row_len[r];
      for (uint32_t j = lane; j < len; j += 64) {
        src[o + j] = v;
        dst[o + j] = G.ext[base + j];
        op[o + j] = 0;
        if (elab) elab[o + j] = e;
      }
      o += len;
    }
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

void launch_validate_csr(const uint64_t* rp, const uint32_t* col, const uint32_t* labels, const uint32_t* elab,
                         uint32_t n_el, uint32_t n, uint64_t nnz, uint32_t* err, hipStream_t s) {
  k_validate_csr<<<grid_for((uint64_t)n * 64, 256), 256, 0, s>>>(rp, col, labels, elab, n_el, n, nnz, err);
}

void launch_row_hist(const uint64_t* keys, uint64_t nnz, int idbits, uint64_t* deg, hipStream_t s) {
  if (!nnz) return;
  k_row_hist<<<grid_for(nnz, 256), 256, 0, s>>>(keys, nnz, idbits, deg);
}

void launch_row_keys_el(const uint64_t* row_off, const uint32_t* row_len, const uint32_t* col,
                        const uint32_t* old_of_new, uint32_t rows, uint32_t elb, int idbits, const uint64_t* out_off,
                        uint64_t* keys, hipStream_t s) {
  k_row_keys_el<<<grid_for((uint64_t)rows * 64, 256), 256, 0, s>>>(row_off, row_len, col, old_of_new, rows, elb,
                                                                   idbits, out_off, keys);
}

void launch_keys_split_el(const uint64_t* keys, uint64_t nnz, int idbits, uint32_t elb, uint32_t* col_out,
                          uint32_t* elab_out, hipStream_t s) {
  if (!nnz) return;
  k_keys_split_el<<<grid_for(nnz, 256), 256, 0, s>>>(keys, nnz, idbits, elb, col_out, elab_out);
}

void launch_deg_rows(const uint32_t* row_len, const uint32_t* map, uint32_t n, uint32_t elb, uint64_t* deg_out,
                     hipStream_t s) {
  k_deg_rows<<<grid_for(n, 256), 256, 0, s>>>(row_len, map, n, elb, deg_out);
}

void launch_relabel_keys(const uint32_t* labels, uint32_t n, uint64_t* keys, hipStream_t s) {
  k_relabel_keys<<<grid_for(n, 256), 256, 0, s>>>(labels, n, keys);
}

void launch_relabel_apply(const uint64_t* sorted, uint32_t n, uint32_t* new_of_old,
                          uint32_t* old_of_new, uint16_t* vlabel, hipStream_t s) {
  k_relabel_apply<<<grid_for(n, 256), 256, 0, s>>>(sorted, n, new_of_old, old_of_new, vlabel);
}

void launch_label_start(const uint16_t* vlabel, uint32_t n, uint32_t slots, uint32_t* label_start,
                        hipStream_t s) {
  k_label_start<<<grid_for((uint64_t)slots + 1, 256), 256, 0, s>>>(vlabel, n, slots, label_start);
}

void launch_csr_keys(const uint64_t* row_off, const uint32_t* row_len, const uint64_t* rp,
                     const uint32_t* col, const uint32_t* map, uint32_t n, int idbits,
                     const uint64_t* out_off, uint64_t* keys, hipStream_t s, const uint32_t* elab, uint32_t elb) {
  k_csr_keys<<<grid_for((uint64_t)n * 64, 256), 256, 0, s>>>(row_off, row_len, rp, col, map, n, idbits,
                                                            out_off, keys, elab, elb);
}

void launch_csr_extract(const uint64_t* keys, uint64_t nnz, uint64_t idmask, uint32_t* col_out,
                        hipStream_t s) {
  k_csr_extract<<<grid_for(nnz, 256), 256, 0, s>>>(keys, nnz, idmask, col_out);
}

void launch_deg_mapped(const uint64_t* rp, const uint32_t* row_len, const uint32_t* map, uint32_t n,
                       uint64_t* deg_out, hipStream_t s) {
  k_deg_mapped<<<grid_for(n, 256), 256, 0, s>>>(rp, row_len, map, n, deg_out);
}

void launch_rows_from_scan(const uint64_t* offs, const uint64_t* deg, uint32_t n, uint64_t base,
                           uint64_t* row_off, uint32_t* row_len, hipStream_t s) {
  k_rows_from_scan<<<grid_for(n, 256), 256, 0, s>>>(offs, deg, n, base, row_off, row_len);
}

void launch_copy_rows(const uint64_t* row_off, const uint32_t* row_len, const uint32_t* src,
                      const uint64_t* new_off, uint32_t* dst, uint32_t n, hipStream_t s) {
  k_copy_rows<<<grid_for((uint64_t)n * 64, 256), 256, 0, s>>>(row_off, row_len, src, new_off, dst, n);
}

void launch_vdel_len(GmGraphDev G, const uint32_t* vdel, uint32_t nv, uint64_t* len, uint32_t* mark, uint32_t* err,
                     hipStream_t s) {
  if (!nv) return;
  k_vdel_len<<<grid_for(nv, 256), 256, 0, s>>>(G, vdel, nv, len, mark, err);
}

void launch_vdel_check(const uint32_t* src, const uint32_t* dst, const uint8_t* op, uint32_t n_upd, uint32_t n,
                       const uint32_t* mark, uint32_t* err, hipStream_t s) {
  if (!n_upd) return;
  k_vdel_check<<<grid_for(n_upd, 256), 256, 0, s>>>(src, dst, op, n_upd, n, mark, err);
}

void launch_vdel_expand(GmGraphDev G, const uint32_t* vdel, uint32_t nv, const uint64_t* offs, uint32_t* src,
                        uint32_t* dst, uint8_t* op, uint32_t* elab, hipStream_t s) {
  if (!nv) return;
  k_vdel_expand<<<grid_for((uint64_t)nv * 64, 256), 256, 0, s>>>(G, vdel, nv, offs, src, dst, op, elab);
}

void launch_gather_ext(const uint32_t* col, const uint32_t* old_of_new, uint64_t nnz, uint32_t* ext,
                       hipStream_t s) {
  if (!nnz) return;
  k_gather_ext<<<grid_for(nnz, 256), 256, 0, s>>>(col, old_of_new, nnz, ext);
}

void launch_u32_to_u64(const uint32_t* in, uint64_t* out, uint32_t n, hipStream_t s) {
  k_u32_to_u64<<<grid_for(n, 256), 256, 0, s>>>(in, out, n);
}

}  // namespace gm
