// Work hand-over rules of the search kernel (load balancing, Sec. V-A),
// written once for the kernel and for a host model of its search loop
// (tests/handover_model.cpp drives them from many host threads).
//
// A busy wave that sees an idle one hands over the upper half of its
// shallowest unexplored work, together with the partial match above it.
// Three kinds of work can be split:
//   RANGE  the untouched part [cur, len) of a level's candidate range;
//   SURV   the survivors of a level's current 64-entry chunk not yet
//          descended into (a bit mask);
//   PERMS  the core permutations of a coalesced plan not yet entered (a bit
//          mask over at most 16 permutations).
// The donor always keeps at least one unit of what it splits (a range of at
// least two entries, at least two survivors or two permutations): a wave
// that receives a single unit polls before entering it and would otherwise
// hand it on again, for as long as some wave is idle.
//
// Task record: HO_WORDS 32-bit words, word i written by lane i of the donor.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define GM_HO_FN __host__ __device__ inline
#else
#define GM_HO_FN inline
#endif

enum : uint32_t {
  HO_NONE = 0,
  HO_RANGE = 1,
  HO_SURV = 2,
  HO_PERMS = 3,
};

enum : uint32_t {
  HO_W_QD = 0,        // query << 8 | directed query edge
  HO_W_OS = 1,        // ord << 1 | sign of the seed
  HO_W_LV = 2,        // level of the split work (| 0x80000000 for PERMS)
  HO_W_CHUNK = 3,     // SURV: first entry of the chunk the survivors belong to
  HO_W_GIVE_LO = 4,   // SURV / PERMS: the bits handed over
  HO_W_GIVE_HI = 5,
  HO_W_CUR = 6,       // RANGE: first entry handed over
  HO_W_END = 7,       // RANGE: end of the range
  HO_W_F = 8,         // 16 words: the partial match f[0..15] (data vertex per query vertex)
  HO_W_SEED = 24,     // the seed the work descends from (completion tracking)
  HO_WORDS = 32,
};

// The split rule.  min_units: the least number of units (survivors,
// permutations) a piece must have to be split; give_ceil: the receiver takes
// the upper ceil(n/2) units instead of floor(n/2).  The search uses
// {2, false}, so the donor keeps at least one; {1, true} is the rule that
// hands on a single unit (kept for the host model, which shows that it does
// not terminate).
struct HoRule {
  uint32_t min_units;
  bool give_ceil;
};
GM_HO_FN HoRule ho_rule_default() { return HoRule{2u, false}; }

struct HoSplit {
  uint32_t lv;    // level of the split work
  uint32_t kind;  // HO_NONE: nothing worth splitting
  uint32_t mid;   // RANGE: the donor keeps [cur, mid), the receiver takes [mid, end)
  uint32_t end;
  uint64_t give;  // SURV / PERMS: the bits the receiver takes
};

GM_HO_FN int ho_popc64(uint64_t m) {
  int c = 0;
  while (m) {
    m &= m - 1;
    ++c;
  }
  return c;
}

// The upper part of a bit set: drop the lower (n - taken) set bits, where
// taken = floor(n / 2) (or ceil with give_ceil).
GM_HO_FN uint64_t ho_upper_part(uint64_t m, const HoRule& r) {
  const int n = ho_popc64(m);
  const int taken = r.give_ceil ? (n + 1) / 2 : n / 2;
  for (int i = 0; i < n - taken; ++i) m &= m - 1;
  return m;
}

// The shallowest splittable work at levels base_l .. lcur.  St gives the
// wave's (uniform) state: cur(x), len(x), mask(x) per level, and pvalid(),
// pidx() for the core permutations of a coalesced plan (level L0; `core`
// false when the plan has none).  Inner levels (x + 1 < k) may also split
// their chunk's survivors; the last level's survivors are matches already.
template <class St>
GM_HO_FN HoSplit ho_choose(const St& st, uint32_t base_l, uint32_t lcur, uint32_t k, bool core, uint32_t L0,
                           uint32_t split_leaf, uint32_t split_inner, HoRule rule) {
  HoSplit s{0xFFFFFFFFu, HO_NONE, 0u, 0u, 0ull};
  for (uint32_t x = base_l; x <= lcur; ++x) {
    if (core && x == L0 && base_l < L0) {
      // permutations after the one being searched (pidx = 0xFFFFFFFF: none entered yet)
      const uint32_t pi = st.pidx();
      const uint32_t rem = st.pvalid() & (pi == 0xFFFFFFFFu ? 0xFFFFFFFFu : ~((2u << pi) - 1u));
      if ((uint32_t)ho_popc64(rem) >= rule.min_units) {
        s.lv = x;
        s.kind = HO_PERMS;
        s.give = ho_upper_part(rem, rule);
        return s;
      }
    }
    const uint32_t cur = st.cur(x), len = st.len(x);
    const uint32_t min_split = (x == k - 1) ? split_leaf : split_inner;
    if (len > cur && len - cur >= min_split && len - cur >= 2) {
      s.lv = x;
      s.kind = HO_RANGE;
      s.mid = cur + ((len - cur) >> 1);
      s.end = len;
      return s;
    }
    if (x + 1 < k) {
      const uint64_t m = st.mask(x);
      if ((uint32_t)ho_popc64(m) >= rule.min_units) {
        s.lv = x;
        s.kind = HO_SURV;
        s.give = ho_upper_part(m, rule);
        return s;
      }
    }
  }
  return s;
}

// Word i of the task record.  f_i: for 8 <= i < 24, the data vertex of query
// vertex i - 8 in the partial match handed over (the core prefix as found
// when the split work lies in or above the core of a coalesced plan).
GM_HO_FN uint32_t ho_task_word(uint32_t i, uint32_t q, uint32_t dq, uint32_t ord, uint32_t sign,
                               const HoSplit& s, uint32_t chunk, uint32_t f_i, uint32_t seed) {
  switch (i) {
    case HO_W_QD: return (q << 8) | dq;
    case HO_W_OS: return (ord << 1) | sign;
    case HO_W_LV: return s.kind == HO_PERMS ? (s.lv | 0x80000000u) : s.lv;
    case HO_W_CHUNK: return s.kind == HO_SURV ? chunk : 0u;
    case HO_W_GIVE_LO: return (uint32_t)s.give;
    case HO_W_GIVE_HI: return (uint32_t)(s.give >> 32);
    case HO_W_CUR: return s.kind == HO_RANGE ? s.mid : 0u;
    case HO_W_END: return s.kind == HO_RANGE ? s.end : 0u;
    case HO_W_SEED: return seed;
    default: return (i >= HO_W_F && i < HO_W_F + 16) ? f_i : 0u;
  }
}
