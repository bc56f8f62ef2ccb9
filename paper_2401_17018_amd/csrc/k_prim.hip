// Data-parallel primitives for the batch pipeline and graph loading:
// exclusive prefix scans and a stable LSD radix sort of 64-bit keys.
// Written for wave64: intra-wave work uses ballots and lane shuffles, and
// blocks are 256 threads (4 waves).
#include "dev_common.h"

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

template <typename T>
__device__ inline T wave_incl_scan(T v, int lane) {
#pragma unroll
  for (int d = 1; d < GM_WAVE; d <<= 1) {
    T o = __shfl_up(v, d, GM_WAVE);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive scan of one tile per block; block total into block_sums[blockIdx].
template <typename T>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_block(const T* __restrict__ in,
                                                             T* __restrict__ out, size_t n,
                                                             T* __restrict__ block_sums) {
  __shared__ T wave_tot[SCAN_THREADS / GM_WAVE];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)tid * SCAN_ITEMS;
  T v[SCAN_ITEMS];
  T sum = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    size_t idx = base + i;
    v[i] = idx < n ? in[idx] : (T)0;
    sum += v[i];
  }
  T incl = wave_incl_scan<T>(sum, lane);
  if (lane == 63) wave_tot[wid] = incl;
  __syncthreads();
  T wave_off = 0;
  for (int w = 0; w < wid; ++w) wave_off += wave_tot[w];
  T run = wave_off + incl - sum;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    size_t idx = base + i;
    if (idx < n) out[idx] = run;
    run += v[i];
  }
  if (tid == SCAN_THREADS - 1) {
    T tot = 0;
    for (int w = 0; w < SCAN_THREADS / GM_WAVE; ++w) tot += wave_tot[w];
    block_sums[blockIdx.x] = tot;
  }
}

template <typename T>
__global__ void k_scan_add(T* __restrict__ out, size_t n, const T* __restrict__ offs) {
  const T add = offs[blockIdx.x];
  const size_t base = (size_t)blockIdx.x * SCAN_TILE;
  for (int i = threadIdx.x; i < SCAN_TILE; i += blockDim.x) {
    size_t idx = base + i;
    if (idx < n) out[idx] += add;
  }
}

template <typename T>
__global__ void k_copy_one(T* dst, const T* src) {
  *dst = *src;
}

template <typename T>
__global__ void k_fill(T* p, T v, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

template <typename T>
void scan_impl(const T* in, T* out, size_t n, T* tmp, hipStream_t s) {
  if (n == 0) {
    k_fill<T><<<1, 1, 0, s>>>(out, (T)0, 1);
    return;
  }
  size_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb == 1) {
    k_scan_block<T><<<1, SCAN_THREADS, 0, s>>>(in, out, n, out + n);
    return;
  }
  T* sums = tmp;
  T* sums_scan = tmp + nb;
  T* rest = tmp + 2 * nb + 1;
  k_scan_block<T><<<(unsigned)nb, SCAN_THREADS, 0, s>>>(in, out, n, sums);
  scan_impl<T>(sums, sums_scan, nb, rest, s);
  k_scan_add<T><<<(unsigned)nb, SCAN_THREADS, 0, s>>>(out, n, sums_scan);
  k_copy_one<T><<<1, 1, 0, s>>>(out + n, sums_scan + nb);
}

// ----------------------------------------------------------------- radix

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 8;
constexpr int RS_WAVES = RS_THREADS / GM_WAVE;
constexpr int RS_WTILE = GM_WAVE * RS_ITEMS;  // keys per wave per tile
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;
constexpr int RS_MAX_BLOCKS = 1024;

struct RsGeom {
  unsigned blocks;
  size_t per;  // keys per block (multiple of RS_TILE)
};

RsGeom rs_geom(size_t n) {
  size_t tiles = (n + RS_TILE - 1) / RS_TILE;
  size_t blocks = tiles < (size_t)RS_MAX_BLOCKS ? tiles : (size_t)RS_MAX_BLOCKS;
  if (blocks == 0) blocks = 1;
  size_t tiles_per = (tiles + blocks - 1) / blocks;
  blocks = (tiles + tiles_per - 1) / tiles_per;
  if (blocks == 0) blocks = 1;
  return RsGeom{(unsigned)blocks, tiles_per * RS_TILE};
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint64_t* __restrict__ keys, size_t n,
                                                        size_t per, int shift,
                                                        uint32_t* __restrict__ hist,
                                                        unsigned nblocks) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  size_t lo = (size_t)blockIdx.x * per;
  size_t hi = lo + per < n ? lo + per : n;
  for (size_t i = lo + threadIdx.x; i < hi; i += RS_THREADS)
    atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  __syncthreads();
  hist[(size_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Lanes holding the same digit as this lane (within `valid`).
__device__ inline uint64_t rs_peers(uint32_t d, uint64_t valid) {
  uint64_t peer = valid;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    uint32_t bit = (d >> b) & 1u;
    uint64_t bb = __ballot(bit);
    peer &= bit ? bb : ~bb;
  }
  return peer;
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const uint64_t* __restrict__ keys,
                                                           uint64_t* __restrict__ out, size_t n,
                                                           size_t per, int shift,
                                                           const uint32_t* __restrict__ hist_scan,
                                                           unsigned nblocks) {
  __shared__ uint32_t goff[256];
  __shared__ uint32_t cnt[RS_WAVES][256];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  goff[tid] = hist_scan[(size_t)tid * nblocks + blockIdx.x];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  size_t lo = (size_t)blockIdx.x * per;
  size_t hi = lo + per < n ? lo + per : n;
  for (size_t t0 = lo; t0 < hi; t0 += RS_TILE) {
    for (int w = 0; w < RS_WAVES; ++w) cnt[w][tid] = 0;
    __syncthreads();
    uint64_t k[RS_ITEMS];
    const size_t wbase = t0 + (size_t)wid * RS_WTILE;
#pragma unroll
    for (int s = 0; s < RS_ITEMS; ++s) {
      size_t idx = wbase + (size_t)s * GM_WAVE + lane;
      bool valid = idx < hi;
      k[s] = valid ? keys[idx] : 0ull;
      uint32_t d = (uint32_t)(k[s] >> shift) & 255u;
      uint64_t vm = __ballot(valid);
      uint64_t peer = rs_peers(d, vm);
      if (valid && lane == __ffsll((unsigned long long)peer) - 1) cnt[wid][d] += __popcll(peer);
    }
    __syncthreads();
    {
      uint32_t run = goff[tid];
      for (int w = 0; w < RS_WAVES; ++w) {
        uint32_t c = cnt[w][tid];
        cnt[w][tid] = run;
        run += c;
      }
      goff[tid] = run;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < RS_ITEMS; ++s) {
      size_t idx = wbase + (size_t)s * GM_WAVE + lane;
      bool valid = idx < hi;
      uint32_t d = (uint32_t)(k[s] >> shift) & 255u;
      uint64_t vm = __ballot(valid);
      uint64_t peer = rs_peers(d, vm);
      if (valid) {
        uint32_t base = cnt[wid][d];
        out[base + __popcll(peer & lt)] = k[s];
      }
      // every lane has read cnt before the leader bumps it
      __builtin_amdgcn_wave_barrier();
      if (valid && lane == __ffsll((unsigned long long)peer) - 1) cnt[wid][d] += __popcll(peer);
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
  }
}

}  // namespace

namespace gm {

size_t scan_tmp_elems(size_t n) {
  size_t total = 0;
  while (true) {
    size_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb <= 1) break;
    total += 2 * nb + 1;
    n = nb;
  }
  return total + 1;
}

void scan_u32(const uint32_t* in, uint32_t* out, size_t n, uint32_t* tmp, hipStream_t s) {
  scan_impl<uint32_t>(in, out, n, tmp, s);
}

void scan_u64(const uint64_t* in, uint64_t* out, size_t n, uint64_t* tmp, hipStream_t s) {
  scan_impl<uint64_t>(in, out, n, tmp, s);
}

size_t radix_hist_elems(size_t n) {
  RsGeom g = rs_geom(n);
  return (size_t)256 * g.blocks + 1;
}

void radix_sort_u64(uint64_t* keys, uint64_t* tmp, size_t n, int bits, uint32_t* hist,
                    uint32_t* hist_scan, uint32_t* scan_tmp, hipStream_t s) {
  if (n < 2 || bits <= 0) return;
  RsGeom g = rs_geom(n);
  uint64_t* src = keys;
  uint64_t* dst = tmp;
  int passes = 0;
  for (int shift = 0; shift < bits; shift += 8) {
    k_rs_hist<<<g.blocks, RS_THREADS, 0, s>>>(src, n, g.per, shift, hist, g.blocks);
    scan_u32(hist, hist_scan, (size_t)256 * g.blocks, scan_tmp, s);
    k_rs_scatter<<<g.blocks, RS_THREADS, 0, s>>>(src, dst, n, g.per, shift, hist_scan, g.blocks);
    uint64_t* t = src;
    src = dst;
    dst = t;
    ++passes;
  }
  if (passes & 1) (void)hipMemcpyAsync(keys, tmp, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
}

void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) {
  if (!n) return;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_fill<uint32_t><<<(unsigned)blocks, 256, 0, s>>>(p, v, n);
}

void fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s) {
  if (!n) return;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_fill<uint64_t><<<(unsigned)blocks, 256, 0, s>>>(p, v, n);
}

}  // namespace gm
