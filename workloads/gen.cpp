// Seeded synthetic input generators shared by the tests, the bench and the
// oracle's callers.  Nothing here performs any step of the matching method:
// it only draws graphs, labels and edge lists.
//
// Every random draw is a pure function of (seed, stream, counter) through the
// SplitMix64 finaliser (Steele, Lea, Flood 2014; Vigna's public-domain
// reference constants), so the output is identical for any thread count.
//
// Build: g++ -O3 -fopenmp -shared -fPIC gen.cpp -o libwlgen.so

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

inline uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

// Counter-based draw: stream key and counter give one 64-bit value.
inline uint64_t draw(uint64_t key, uint64_t ctr) {
  return mix64(key + (ctr + 1) * 0x9E3779B97F4A7C15ull);
}

inline uint64_t stream_key(uint64_t seed, uint64_t tag) {
  return mix64(seed ^ mix64(tag * 0xD1B54A32D192ED03ull + 0x632BE59BD9B4E019ull));
}

// Uniform integer in [0, n) from a 64-bit draw (multiply-high, Lemire 2019).
inline uint64_t bounded(uint64_t r, uint64_t n) {
  return (uint64_t)(((__uint128_t)r * n) >> 64);
}

int nthreads_or(int t) { return t > 0 ? t : omp_get_max_threads(); }

// Stable LSD radix sort of 64-bit keys carrying a 32-bit payload, over the
// low `bits` bits of the key.  Parallel per pass; stable, so equal keys keep
// their input order.
void radix_sort_kv(std::vector<uint64_t>& key, std::vector<uint32_t>& val, int bits,
                   int threads) {
  const size_t n = key.size();
  if (n < 2) return;
  const int R = 11, B = 1 << R;
  std::vector<uint64_t> k2(n);
  std::vector<uint32_t> v2(n);
  const int T = threads;
  std::vector<size_t> hist((size_t)T * B);
  for (int shift = 0; shift < bits; shift += R) {
    std::fill(hist.begin(), hist.end(), 0);
#pragma omp parallel num_threads(T)
    {
      int t = omp_get_thread_num();
      size_t lo = n * t / T, hi = n * (t + 1) / T;
      size_t* h = &hist[(size_t)t * B];
      for (size_t i = lo; i < hi; ++i) h[(key[i] >> shift) & (B - 1)]++;
    }
    size_t run = 0;
    for (int d = 0; d < B; ++d)
      for (int t = 0; t < T; ++t) {
        size_t c = hist[(size_t)t * B + d];
        hist[(size_t)t * B + d] = run;
        run += c;
      }
#pragma omp parallel num_threads(T)
    {
      int t = omp_get_thread_num();
      size_t lo = n * t / T, hi = n * (t + 1) / T;
      size_t* h = &hist[(size_t)t * B];
      for (size_t i = lo; i < hi; ++i) {
        size_t d = (key[i] >> shift) & (B - 1);
        size_t p = h[d]++;
        k2[p] = key[i];
        v2[p] = val[i];
      }
    }
    key.swap(k2);
    val.swap(v2);
  }
}

int bits_for(uint64_t x) {  // number of bits needed to hold values < x
  int b = 0;
  while (b < 64 && (1ull << b) < x) ++b;
  return b;
}

// Keep the first occurrence (by sample index) of each key; then keep the
// `target` keys whose first occurrence is earliest.  Returns the kept keys in
// ascending key order.
std::vector<uint64_t> first_distinct(std::vector<uint64_t>& key, uint64_t target, int keybits,
                                     int threads) {
  std::vector<uint32_t> idx(key.size());
#pragma omp parallel for num_threads(threads)
  for (size_t i = 0; i < key.size(); ++i) idx[i] = (uint32_t)i;
  radix_sort_kv(key, idx, keybits, threads);
  // unique, keeping the first (smallest index: the sort is stable)
  std::vector<uint64_t> uk;
  std::vector<uint32_t> ui;
  uk.reserve(key.size());
  ui.reserve(key.size());
  for (size_t i = 0; i < key.size(); ++i) {
    if (i == 0 || key[i] != key[i - 1]) {
      uk.push_back(key[i]);
      ui.push_back(idx[i]);
    }
  }
  if (uk.size() < target) return {};
  if (uk.size() > target) {
    std::vector<uint32_t> tmp(ui);
    std::nth_element(tmp.begin(), tmp.begin() + (target - 1), tmp.end());
    uint32_t thr = tmp[target - 1];
    size_t w = 0;
    for (size_t i = 0; i < uk.size(); ++i)
      if (ui[i] <= thr) uk[w++] = uk[i];
    uk.resize(w);
  }
  return uk;
}

}  // namespace

extern "C" {

uint64_t wl_mix64(uint64_t z) { return mix64(z); }
uint64_t wl_draw(uint64_t key, uint64_t ctr) { return draw(key, ctr); }
uint64_t wl_stream_key(uint64_t seed, uint64_t tag) { return stream_key(seed, tag); }

// Fill out[i] = draw(key, start + i) for i < n.
void wl_draws(uint64_t key, uint64_t start, uint64_t n, uint64_t* out, int threads) {
  int T = nthreads_or(threads);
#pragma omp parallel for num_threads(T) schedule(static)
  for (uint64_t i = 0; i < n; ++i) out[i] = draw(key, start + i);
}

// Erdos-Renyi G(n, m): uniform pairs u != v, kept without replacement in
// sample order until m distinct undirected edges.  Output canonical (lo < hi)
// edges in ascending (lo, hi) order.  Returns m, or -1 if m is infeasible.
int64_t wl_er_edges(uint32_t n, uint64_t m, uint64_t seed, uint32_t* lo, uint32_t* hi,
                    int threads) {
  int T = nthreads_or(threads);
  if (n < 2 || m > (uint64_t)n * (n - 1) / 2) return -1;
  uint64_t key = stream_key(seed, 1);
  int vb = bits_for(n);
  for (double over = 1.25;; over *= 1.5) {
    uint64_t S = (uint64_t)std::ceil((double)m * over) + 64;
    if (S > 0xFFFFFFFFull) return -1;
    std::vector<uint64_t> k(S);
#pragma omp parallel for num_threads(T) schedule(static)
    for (uint64_t i = 0; i < S; ++i) {
      uint64_t u = bounded(draw(key, 2 * i), n), v = bounded(draw(key, 2 * i + 1), n);
      k[i] = (u == v) ? ~0ull : ((std::min(u, v) << vb) | std::max(u, v));
    }
    size_t w = 0;  // drop rejected samples, keeping sample order
    for (size_t i = 0; i < S; ++i)
      if (k[i] != ~0ull) k[w++] = k[i];
    k.resize(w);
    std::vector<uint64_t> uk = first_distinct(k, m, 2 * vb, T);
    if (uk.size() != m) {
      if (over > 64) return -1;
      continue;
    }
    for (uint64_t i = 0; i < m; ++i) {
      lo[i] = (uint32_t)(uk[i] >> vb);
      hi[i] = (uint32_t)(uk[i] & ((1ull << vb) - 1));
    }
    return (int64_t)m;
  }
}

// R-MAT (Chakrabarti, Zhan, Faloutsos 2004) over 2^scale vertices with
// quadrant probabilities (a, b, c, 1-a-b-c), no noise.  Sample i draws one
// quadrant per level from counter-based draws.  Self-loops are dropped, pairs
// canonicalised to (lo, hi), and the first occurrence of each pair by sample
// index is kept until m distinct pairs exist.  Output ascending (lo, hi).
int64_t wl_rmat_edges(uint32_t scale, uint64_t m, double a, double b, double c, uint64_t seed,
                      uint32_t* lo, uint32_t* hi, int threads) {
  int T = nthreads_or(threads);
  if (scale < 1 || scale > 31) return -1;
  uint64_t key = stream_key(seed, 1);
  // 16-bit thresholds per level
  const uint32_t ta = (uint32_t)std::lround(a * 65536.0);
  const uint32_t tb = (uint32_t)std::lround((a + b) * 65536.0);
  const uint32_t tc = (uint32_t)std::lround((a + b + c) * 65536.0);
  const uint32_t draws_per = (scale + 3) / 4;
  for (double over = 1.3;; over *= 1.4) {
    uint64_t S = (uint64_t)std::ceil((double)m * over) + 1024;
    if (S > 0xFFFFFFFFull) return -1;
    std::vector<uint64_t> k(S);
#pragma omp parallel for num_threads(T) schedule(static)
    for (uint64_t i = 0; i < S; ++i) {
      uint64_t u = 0, v = 0;
      uint32_t lvl = 0;
      for (uint32_t d = 0; d < draws_per; ++d) {
        uint64_t r = draw(key, i * draws_per + d);
        for (int s = 0; s < 4 && lvl < scale; ++s, ++lvl) {
          uint32_t x = (uint32_t)(r >> (16 * s)) & 0xFFFF;
          uint32_t q = x < ta ? 0 : x < tb ? 1 : x < tc ? 2 : 3;
          u = (u << 1) | (q >> 1);
          v = (v << 1) | (q & 1);
        }
      }
      k[i] = (u == v) ? ~0ull : ((std::min(u, v) << scale) | std::max(u, v));
    }
    size_t w = 0;
    for (size_t i = 0; i < S; ++i)
      if (k[i] != ~0ull) k[w++] = k[i];
    k.resize(w);
    std::vector<uint64_t> uk = first_distinct(k, m, 2 * scale, T);
    if (uk.size() != m) {
      if (over > 40) return -1;
      continue;
    }
#pragma omp parallel for num_threads(T) schedule(static)
    for (uint64_t i = 0; i < m; ++i) {
      lo[i] = (uint32_t)(uk[i] >> scale);
      hi[i] = (uint32_t)(uk[i] & ((1ull << scale) - 1));
    }
    return (int64_t)m;
  }
}

// Fisher-Yates permutation of 0..n-1 driven by counter draws.
void wl_permutation(uint32_t n, uint64_t seed, uint64_t tag, uint32_t* perm) {
  uint64_t key = stream_key(seed, tag);
  for (uint32_t i = 0; i < n; ++i) perm[i] = i;
  for (uint64_t i = n; i > 1; --i) {
    uint64_t j = bounded(draw(key, i), i);
    std::swap(perm[i - 1], perm[j]);
  }
}

// Relabel edge endpoints through perm and re-canonicalise to lo < hi.
void wl_apply_perm(uint64_t m, uint32_t* lo, uint32_t* hi, const uint32_t* perm, int threads) {
  int T = nthreads_or(threads);
#pragma omp parallel for num_threads(T) schedule(static)
  for (uint64_t i = 0; i < m; ++i) {
    uint32_t a = perm[lo[i]], b = perm[hi[i]];
    lo[i] = std::min(a, b);
    hi[i] = std::max(a, b);
  }
}

// Deterministic shuffle of an edge list: stable sort by a random key derived
// from (seed, tag, position).
void wl_shuffle_edges(uint64_t m, uint32_t* lo, uint32_t* hi, uint64_t seed, uint64_t tag,
                      int threads) {
  int T = nthreads_or(threads);
  if (m > 0xFFFFFFFFull) return;
  uint64_t key = stream_key(seed, tag);
  std::vector<uint64_t> k(m);
  std::vector<uint32_t> pos(m);
#pragma omp parallel for num_threads(T) schedule(static)
  for (uint64_t i = 0; i < m; ++i) {
    k[i] = draw(key, i);
    pos[i] = (uint32_t)i;
  }
  radix_sort_kv(k, pos, 64, T);
  std::vector<uint32_t> l2(m), h2(m);
#pragma omp parallel for num_threads(T) schedule(static)
  for (uint64_t i = 0; i < m; ++i) {
    l2[i] = lo[pos[i]];
    h2[i] = hi[pos[i]];
  }
  std::memcpy(lo, l2.data(), m * 4);
  std::memcpy(hi, h2.data(), m * 4);
}

// Symmetric CSR with ascending rows from m undirected edges (no duplicates,
// no self-loops assumed).  row_ptr has n+1 entries, col has 2m entries.
int wl_build_csr(uint32_t n, uint64_t m, const uint32_t* lo, const uint32_t* hi,
                 uint64_t* row_ptr, uint32_t* col, int threads) {
  int T = nthreads_or(threads);
  std::vector<uint64_t> deg(n + 1, 0);
  {
    std::vector<std::vector<uint64_t>> part(T, std::vector<uint64_t>());
#pragma omp parallel num_threads(T)
    {
      int t = omp_get_thread_num();
      std::vector<uint64_t>& d = part[t];
      d.assign(n, 0);
      uint64_t a = m * t / T, b = m * (t + 1) / T;
      for (uint64_t i = a; i < b; ++i) {
        d[lo[i]]++;
        d[hi[i]]++;
      }
    }
    for (int t = 0; t < T; ++t)
#pragma omp parallel for num_threads(T) schedule(static)
      for (uint64_t v = 0; v < n; ++v) deg[v] += part[t][v];
  }
  row_ptr[0] = 0;
  for (uint32_t v = 0; v < n; ++v) row_ptr[v + 1] = row_ptr[v] + deg[v];
  std::vector<uint64_t> cur(row_ptr, row_ptr + n);
  // fill in parallel by vertex ranges is awkward; fill sequential-safe with
  // atomics then sort each row (order inside a row is fixed by the sort).
#pragma omp parallel for num_threads(T) schedule(static)
  for (uint64_t i = 0; i < m; ++i) {
    uint64_t p = __atomic_fetch_add(&cur[lo[i]], 1, __ATOMIC_RELAXED);
    col[p] = hi[i];
    uint64_t q = __atomic_fetch_add(&cur[hi[i]], 1, __ATOMIC_RELAXED);
    col[q] = lo[i];
  }
#pragma omp parallel for num_threads(T) schedule(dynamic, 1024)
  for (uint64_t v = 0; v < n; ++v) std::sort(col + row_ptr[v], col + row_ptr[v + 1]);
  return 0;
}

// Vertex labels: i.i.d. uniform over L labels.
void wl_labels_uniform(uint32_t n, uint32_t L, uint64_t seed, uint64_t tag, uint32_t* labels,
                       int threads) {
  int T = nthreads_or(threads);
  uint64_t key = stream_key(seed, tag);
#pragma omp parallel for num_threads(T) schedule(static)
  for (uint64_t v = 0; v < n; ++v) labels[v] = (uint32_t)bounded(draw(key, v), L);
}

// Vertex labels: Zipf with P(l) proportional to (l+1)^-s over L labels.
void wl_labels_zipf(uint32_t n, uint32_t L, double s, uint64_t seed, uint64_t tag,
                    uint32_t* labels, int threads) {
  int T = nthreads_or(threads);
  uint64_t key = stream_key(seed, tag);
  std::vector<double> cdf(L);
  double z = 0;
  for (uint32_t l = 0; l < L; ++l) z += std::pow((double)(l + 1), -s);
  double acc = 0;
  for (uint32_t l = 0; l < L; ++l) {
    acc += std::pow((double)(l + 1), -s) / z;
    cdf[l] = acc;
  }
  cdf[L - 1] = 1.0;
#pragma omp parallel for num_threads(T) schedule(static)
  for (uint64_t v = 0; v < n; ++v) {
    double u = (double)(draw(key, v) >> 11) * (1.0 / 9007199254740992.0);
    uint32_t l = (uint32_t)(std::upper_bound(cdf.begin(), cdf.end(), u) - cdf.begin());
    labels[v] = std::min(l, L - 1);
  }
}

}  // extern "C"
