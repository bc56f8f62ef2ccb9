// Host model of the search kernel's work hand-over (load balancing,
// Sec. V-A), for CPU tests.  Each host thread plays one wavefront and runs
// the kernel's search loop over a synthetic search tree; the split rules and
// the task record come from the kernel's own header (handover.h), and the
// claim / mailbox / termination protocol is the kernel's, on std::atomic.
//
// The search tree: a seed's plan has k levels (2 .. k-1 are searched); the
// node reached above level l (a hash standing for the partial match)
// determines level l's candidate range; an inner level's 64-entry chunk has
// a pseudo-random survivor mask, and every survivor is a child node; at the
// last level the candidates that pass a hash test are matches.  A plan may
// be "coalesced over a core": after level L0 - 1 the core match is entered
// once per valid permutation (at most 16), each a whole subtree, as the
// kernel does for core coalescing.
//
// Output (stdout, one line): matches, sum and xor of match ids, hand-overs by
// kind, the sequential reference's matches, sum and xor, whether every seed's
// open-item counter ended at 0, and "stalled" when the hand-over count
// passed the cap (no progress).
//
// Usage: handover_model threads seeds forced(0/1) perms_rule(0 = kernel's,
//        1 = hand on a single permutation) handover_cap salt [scenario]
// scenario 1: every plan is coalesced over a core with three valid
// permutations (the case in which handing on a single permutation loops).
#include <atomic>
#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "../paper_2401_17018_amd/csrc/handover.h"

namespace {

constexpr uint32_t WAVE = 64, LEAF_STEP = 256, MAXK = 8;
constexpr uint32_t MSG_TASK = 1, MSG_STOP = 3;

uint64_t mix(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

struct Plan {
  uint32_t k;    // levels 0 .. k-1; the seed fixes 0 and 1
  uint32_t L0;   // first level after the core (0: not coalesced)
  uint32_t ncp;  // permutations of the core
};

// scenario 1: every seed's plan has a core whose three permutations are all
// valid, and every level has a single candidate (a survivor), so the core's
// permutations are the only work that can be split; a seed's wave starts
// once every other wave waits for work, and its first split hands one
// permutation on
int g_scenario = 0;

Plan plan_of(uint64_t seed_id, uint64_t salt) {
  const uint64_t h = mix(seed_id * 0x9E3779B97F4A7C15ull ^ salt);
  Plan p;
  if (g_scenario == 1) {
    p.k = 6;
    p.L0 = 3;
    p.ncp = 3;
    return p;
  }
  p.k = 4 + (uint32_t)(h % 4);  // 4 .. 7
  if ((h >> 8) % 3 == 0) {
    p.L0 = 3 + (uint32_t)((h >> 12) % (p.k - 3));  // 3 .. k-1
    p.ncp = 2 + (uint32_t)((h >> 16) % 15);        // 2 .. 16
  } else {
    p.L0 = 0;
    p.ncp = 1;
  }
  return p;
}

uint32_t range_len(uint64_t node, uint32_t l, const Plan& p) {
  if (g_scenario == 1) return 1;
  const uint64_t h = mix(node ^ (0x1234567ull * (l + 1)));
  if (l == p.k - 1) return (h % 13 == 0) ? 1000 + (uint32_t)(h >> 40) % 2000 : (uint32_t)(h >> 20) % 200;
  return (h % 11 == 0) ? 100 + (uint32_t)(h >> 40) % 200 : (uint32_t)(h >> 20) % 24;
}

// survivors of the chunk [chunk, chunk + 64) of a range of length len: each
// entry decides by itself (about 1 in 10 survives)
uint64_t surv_mask(uint64_t node, uint32_t l, uint32_t chunk, uint32_t len) {
  if (g_scenario == 1) return chunk < len ? 1ull : 0ull;
  uint64_t m = 0;
  for (uint32_t b = 0; b < WAVE && chunk + b < len; ++b)
    if (mix(node ^ mix(((uint64_t)l << 32) | (chunk + b))) % 10 == 0) m |= 1ull << b;
  return m;
}

uint64_t child(uint64_t node, uint32_t l, uint32_t idx) { return mix(node * 0x100000001B3ull ^ ((uint64_t)l << 40) ^ idx); }
uint64_t permuted(uint64_t core, uint32_t p) { return mix(core ^ (0xA5A5A5A5ull * (p + 1))); }
uint32_t perm_valid(uint64_t core, uint32_t ncp) {
  if (g_scenario == 1) return (1u << ncp) - 1u;
  uint32_t v = (uint32_t)mix(core ^ 0x77) & ((ncp >= 32 ? 0 : (1u << ncp)) - 1u);
  return v ? v : 1u;
}
bool is_match(uint64_t node, uint32_t idx) { return (mix(node ^ (idx * 0xD6E8FEB86659FD93ull)) & 3u) != 0u; }
uint64_t match_id(uint64_t node, uint32_t idx) { return mix(node + idx * 0x9E3779B97F4A7C15ull); }

struct Totals {
  uint64_t cnt = 0, sum = 0, xr = 0;
  void add(uint64_t id) {
    ++cnt;
    sum += id;
    xr ^= id;
  }
};

// ---------------------------------------------------------------- reference

void visit(uint64_t node, uint32_t l, const Plan& p, Totals& t) {
  const uint32_t len = range_len(node, l, p);
  if (l == p.k - 1) {
    for (uint32_t i = 0; i < len; ++i)
      if (is_match(node, i)) t.add(match_id(node, i));
    return;
  }
  for (uint32_t c = 0; c < len; c += WAVE) {
    uint64_t m = surv_mask(node, l, c, len);
    while (m) {
      const uint32_t b = (uint32_t)__builtin_ctzll(m);
      m &= m - 1;
      const uint64_t ch = child(node, l, c + b);
      if (p.L0 && l + 1 == p.L0) {
        const uint32_t v = perm_valid(ch, p.ncp);
        for (uint32_t q = 0; q < p.ncp; ++q)
          if ((v >> q) & 1u) visit(permuted(ch, q), p.L0, p, t);
      } else {
        visit(ch, l + 1, p, t);
      }
    }
  }
}

// ---------------------------------------------------------------- shared state

struct Shared {
  uint32_t n_waves = 0, n_seeds = 0;
  uint64_t salt = 0;
  bool forced = false;
  HoRule perms_rule{};
  uint64_t cap = 0;
  std::atomic<uint64_t> seed_head{0};
  std::atomic<uint64_t> pending{0};
  std::atomic<uint32_t> idle_count{0};
  std::vector<std::atomic<uint64_t>> idle_bits;
  std::vector<std::atomic<uint32_t>> mflag;
  std::vector<uint32_t> mbox;
  std::vector<std::atomic<uint32_t>> seed_open;
  std::atomic<uint64_t> handovers[4] = {{0}, {0}, {0}, {0}};
  std::atomic<bool> stalled{false};
  std::atomic<uint32_t> went_idle{0};  // waves that have waited for work at least once
};

struct WaveModel {
  Shared& sh;
  uint32_t slot;
  uint64_t rng;
  // per level, as in the kernel's wave state
  uint64_t node[MAXK];
  uint32_t cur[MAXK], len[MAXK], chunk[MAXK];
  uint64_t mask[MAXK];
  uint64_t core = 0;  // the core match being permuted
  uint32_t pvalid = 0, pidx = 0xFFFFFFFFu;
  bool went_idle = false;
  Totals tot;

  struct View {
    const WaveModel& w;
    uint32_t cur(uint32_t x) const { return w.cur[x]; }
    uint32_t len(uint32_t x) const { return w.len[x]; }
    uint64_t mask(uint32_t x) const { return w.mask[x]; }
    uint32_t pvalid() const { return w.pvalid; }
    uint32_t pidx() const { return w.pidx; }
  };

  void setup(uint32_t l, uint64_t nd, const Plan& p) {
    node[l] = nd;
    len[l] = range_len(nd, l, p);
    cur[l] = 0;
    mask[l] = 0;
    chunk[l] = 0;
  }

  void finish_item(uint32_t seed) {
    sh.seed_open[seed].fetch_sub(1, std::memory_order_acq_rel);
    if (sh.pending.fetch_sub(1, std::memory_order_acq_rel) == 1)
      for (uint32_t s = 0; s < sh.n_waves; ++s) sh.mflag[s].store(MSG_STOP, std::memory_order_release);
  }

  // the kernel's try_donate: choose, claim an idle wave, publish the task
  void try_donate(uint32_t lcur, uint32_t base_l, const Plan& p, uint32_t seed) {
    const bool core_plan = p.L0 != 0;
    HoRule rule = ho_rule_default();
    HoSplit sp = ho_choose(View{*this}, base_l, lcur, p.k, core_plan, p.L0, 2u, 2u, rule);
    if (sp.kind == HO_NONE && core_plan && sh.perms_rule.min_units < rule.min_units) {
      // the rule under test for permutations (the kernel's rule handles the rest)
      sp = ho_choose(View{*this}, base_l, lcur, p.k, core_plan, p.L0, 0xFFFFFFFFu, 0xFFFFFFFFu, sh.perms_rule);
      if (sp.kind != HO_PERMS) sp.kind = HO_NONE;
    }
    if (sp.kind == HO_NONE) return;
    if (sp.kind == HO_PERMS && sp.give == 0) return;
    // claim: scan the bitmap from a pseudo-random word, clear one set bit
    const uint32_t nwords = (sh.n_waves + 63) / 64;
    rng = mix(rng + slot);
    const uint32_t start = (uint32_t)(rng % nwords);
    int32_t target = -1;
    for (uint32_t r = 0; r < nwords && target < 0; ++r) {
      const uint32_t wi = (start + r) % nwords;
      uint64_t v = sh.idle_bits[wi].load(std::memory_order_relaxed);
      while (v && target < 0) {
        const int b = __builtin_ctzll(v);
        const uint64_t old = sh.idle_bits[wi].fetch_and(~(1ull << b), std::memory_order_acq_rel);
        if ((old >> b) & 1ull)
          target = (int32_t)(wi * 64 + b);
        else
          v = old & ~(1ull << b);
      }
    }
    if (target < 0) return;
    sh.idle_count.fetch_sub(1, std::memory_order_relaxed);
    if (sp.kind == HO_RANGE)
      len[sp.lv] = sp.mid;
    else if (sp.kind == HO_SURV)
      mask[sp.lv] &= ~sp.give;
    else
      pvalid &= ~(uint32_t)sp.give;
    // the partial match: the node the split level hangs from (the core
    // match for permutations), in place of the data vertices
    const uint64_t nd = sp.kind == HO_PERMS ? core : node[sp.lv];
    for (uint32_t i = 0; i < HO_WORDS; ++i) {
      const uint32_t fi = i == HO_W_F ? (uint32_t)nd : (i == HO_W_F + 1 ? (uint32_t)(nd >> 32) : 0u);
      sh.mbox[(size_t)target * HO_WORDS + i] =
          ho_task_word(i, 0u, 0u, seed, 0u, sp, sp.kind == HO_SURV ? chunk[sp.lv] : 0u, fi, seed);
    }
    sh.pending.fetch_add(1, std::memory_order_acq_rel);
    sh.seed_open[seed].fetch_add(1, std::memory_order_acq_rel);
    sh.mflag[target].store(MSG_TASK, std::memory_order_release);
    const uint64_t total = sh.handovers[sp.kind].fetch_add(1, std::memory_order_relaxed) + 1;
    if (sh.cap && total > sh.cap) sh.stalled.store(true, std::memory_order_relaxed);
  }

  bool poll(uint32_t lcur, uint32_t base_l, const Plan& p, uint32_t seed) {
    if (sh.stalled.load(std::memory_order_relaxed)) return true;
    const uint32_t c = sh.idle_count.load(std::memory_order_relaxed);
    if (c == 0) return false;
    rng = mix(rng ^ 0x5151);
    if (sh.forced || (rng & 7u) == 0) try_donate(lcur, base_l, p, seed);
    return false;
  }

  void run() {
    for (;;) {
      uint32_t seed = 0, base_l = 2, l;
      bool handed = false, ptask = false;
      uint32_t words[HO_WORDS];
      const uint64_t t = sh.seed_head.fetch_add(1, std::memory_order_relaxed);
      if (t < sh.n_seeds) {
        seed = (uint32_t)t;
        sh.seed_open[t].store(1, std::memory_order_release);
        if (g_scenario == 1)
          while (sh.went_idle.load(std::memory_order_relaxed) + sh.n_seeds < sh.n_waves &&
                 !sh.stalled.load(std::memory_order_relaxed))
            std::this_thread::yield();
      } else {
        // advertise, then wait for a task or the stop message
        if (!went_idle) {
          went_idle = true;
          sh.went_idle.fetch_add(1, std::memory_order_relaxed);
        }
        sh.idle_count.fetch_add(1, std::memory_order_relaxed);
        sh.idle_bits[slot >> 6].fetch_or(1ull << (slot & 63), std::memory_order_acq_rel);
        uint32_t msg = 0;
        while ((msg = sh.mflag[slot].load(std::memory_order_acquire)) == 0) {
          if (sh.stalled.load(std::memory_order_relaxed)) return;
          std::this_thread::yield();
        }
        if (msg == MSG_STOP) return;
        for (uint32_t i = 0; i < HO_WORDS; ++i) words[i] = sh.mbox[(size_t)slot * HO_WORDS + i];
        sh.mflag[slot].store(0, std::memory_order_relaxed);
        seed = words[HO_W_SEED];
        base_l = words[HO_W_LV] & 0x7FFFFFFFu;
        ptask = (words[HO_W_LV] >> 31) != 0u;
        handed = true;
      }
      const Plan p = plan_of(seed, sh.salt);
      const bool core_plan = p.L0 != 0;
      const uint32_t L0 = core_plan ? p.L0 : 0xFFFFFFFFu;
      pvalid = 0;
      pidx = 0xFFFFFFFFu;
      if (ptask) {
        core = words[HO_W_F] | ((uint64_t)words[HO_W_F + 1] << 32);
        pvalid = words[HO_W_GIVE_LO];
        base_l = L0 - 1;
        cur[L0 - 1] = len[L0 - 1] = 0;
        mask[L0 - 1] = 0;
        l = L0;
        cur[L0] = len[L0] = 0;
        mask[L0] = 0;
      } else if (handed) {
        l = base_l;
        setup(l, words[HO_W_F] | ((uint64_t)words[HO_W_F + 1] << 32), p);
        cur[l] = words[HO_W_CUR];
        len[l] = words[HO_W_END];
        chunk[l] = words[HO_W_CHUNK];
        mask[l] = words[HO_W_GIVE_LO] | ((uint64_t)words[HO_W_GIVE_HI] << 32);
      } else {
        l = 2;
        setup(l, mix(seed * 0xC2B2AE3D27D4EB4Full + sh.salt), p);
      }
      for (;;) {
        uint64_t m = mask[l];
        uint32_t nl = 0xFFFFFFFFu;
        uint64_t nl_node = 0;
        if (m == 0) {
          if (poll(l, base_l, p, seed)) return;
          if (cur[l] >= len[l]) {
            if (l == base_l) break;
            if (core_plan && l == L0 && (pidx == 0xFFFFFFFFu ? pvalid : (pvalid >> (pidx + 1))) != 0u) {
              const uint32_t p0 = pidx == 0xFFFFFFFFu ? 0u : pidx + 1;
              pidx = p0 + (uint32_t)__builtin_ctz(pvalid >> p0);
              l = L0 - 1;
              nl = L0;
              nl_node = permuted(core, pidx);
            } else {
              --l;
              continue;
            }
          } else {
            const uint32_t c = cur[l];
            if (l == p.k - 1) {
              cur[l] = c + LEAF_STEP;
              const uint32_t e = c + LEAF_STEP < len[l] ? c + LEAF_STEP : len[l];
              for (uint32_t i = c; i < e; ++i)
                if (is_match(node[l], i)) tot.add(match_id(node[l], i));
              continue;
            }
            cur[l] = c + WAVE;
            chunk[l] = c;
            m = surv_mask(node[l], l, c, len[l]);
            mask[l] = m;
            if (m == 0) continue;
          }
        }
        if (nl == 0xFFFFFFFFu) {
          const uint32_t bit = (uint32_t)__builtin_ctzll(m);
          mask[l] = m & (m - 1);
          const uint64_t ch = child(node[l], l, chunk[l] + bit);
          if (core_plan && l + 1 == L0) {
            core = ch;
            pvalid = perm_valid(ch, p.ncp);
            pidx = 0xFFFFFFFFu;
            l = L0;
            cur[L0] = len[L0] = 0;
            mask[L0] = 0;
            continue;
          }
          nl = l + 1;
          nl_node = ch;
        }
        setup(nl, nl_node, p);
        l = nl;
      }
      finish_item(seed);
    }
  }
};

}  // namespace

int main(int argc, char** argv) {
  if (argc < 7) {
    std::fprintf(stderr, "usage: %s threads seeds forced perms_rule cap salt [scenario]\n", argv[0]);
    return 2;
  }
  g_scenario = argc > 7 ? std::atoi(argv[7]) : 0;
  Shared sh;
  sh.n_waves = (uint32_t)std::atoi(argv[1]);
  sh.n_seeds = (uint32_t)std::atoi(argv[2]);
  sh.forced = std::atoi(argv[3]) != 0;
  sh.perms_rule = std::atoi(argv[4]) ? HoRule{1u, true} : ho_rule_default();
  sh.cap = std::strtoull(argv[5], nullptr, 10);
  sh.salt = std::strtoull(argv[6], nullptr, 10);
  sh.idle_bits = std::vector<std::atomic<uint64_t>>((sh.n_waves + 63) / 64);
  sh.mflag = std::vector<std::atomic<uint32_t>>(sh.n_waves);
  sh.mbox.assign((size_t)sh.n_waves * HO_WORDS, 0u);
  sh.seed_open = std::vector<std::atomic<uint32_t>>(sh.n_seeds);
  for (auto& x : sh.idle_bits) x.store(0);
  for (auto& x : sh.mflag) x.store(0);
  for (auto& x : sh.seed_open) x.store(0xFFFFFFFFu);
  sh.pending.store(sh.n_seeds);

  Totals ref;
  for (uint32_t s = 0; s < sh.n_seeds; ++s) {
    const Plan p = plan_of(s, sh.salt);
    visit(mix(s * 0xC2B2AE3D27D4EB4Full + sh.salt), 2, p, ref);
  }

  std::vector<std::thread> th;
  std::vector<Totals> per(sh.n_waves);
  for (uint32_t w = 0; w < sh.n_waves; ++w)
    th.emplace_back([&sh, &per, w]() {
      WaveModel wm{sh, w, mix(w + 1)};
      wm.run();
      per[w] = wm.tot;
    });
  for (auto& t : th) t.join();
  Totals got;
  for (auto& t : per) {
    got.cnt += t.cnt;
    got.sum += t.sum;
    got.xr ^= t.xr;
  }
  bool all_closed = true;
  for (auto& x : sh.seed_open) all_closed = all_closed && x.load() == 0u;
  std::printf("matches %" PRIu64 " sum %" PRIu64 " xor %" PRIu64 " handovers %" PRIu64 " %" PRIu64 " %" PRIu64
              " ref %" PRIu64 " %" PRIu64 " %" PRIu64 " closed %d pending %" PRIu64 " stalled %d\n",
              got.cnt, got.sum, got.xr, sh.handovers[HO_RANGE].load(), sh.handovers[HO_SURV].load(),
              sh.handovers[HO_PERMS].load(), ref.cnt, ref.sum, ref.xr, all_closed ? 1 : 0, sh.pending.load(),
              sh.stalled.load() ? 1 : 0);
  return 0;
}
