// Query validation, matching-order planning and filter tables (host).
#include "host_plan.h"

#include <algorithm>
#include <cstring>
#include <functional>
#include <map>
#include <set>

#include "../../include/gamma.h"

namespace gm {

int validate_query(uint32_t k, const uint32_t* qlabels, uint32_t m, const uint32_t* qedges,
                   std::string* msg) {
  if (k < 2 || k > GM_MAX_K) {
    if (msg) *msg = "query size k must be in [2, 16]";
    return k > GM_MAX_K ? GAMMA_EUNSUPPORTED : GAMMA_EINVAL;
  }
  if (!qlabels || !qedges) {
    if (msg) *msg = "null query array";
    return GAMMA_EINVAL;
  }
  if (m < k - 1 || m > k * (k - 1) / 2) {
    if (msg) *msg = "edge count out of range for a connected simple query";
    return GAMMA_EINVAL;
  }
  for (uint32_t u = 0; u < k; ++u)
    if (qlabels[u] > 0xFFFFu) {
      if (msg) *msg = "query label >= 65536";
      return GAMMA_EINVAL;
    }
  std::set<std::pair<uint32_t, uint32_t>> seen;
  std::vector<std::vector<uint32_t>> adj(k);
  for (uint32_t e = 0; e < m; ++e) {
    uint32_t a = qedges[2 * e], b = qedges[2 * e + 1];
    if (a >= k || b >= k || a == b) {
      if (msg) *msg = "query edge endpoint out of range or self loop";
      return GAMMA_EINVAL;
    }
    auto key = std::make_pair(std::min(a, b), std::max(a, b));
    if (!seen.insert(key).second) {
      if (msg) *msg = "repeated query edge";
      return GAMMA_EINVAL;
    }
    adj[a].push_back(b);
    adj[b].push_back(a);
  }
  std::vector<char> vis(k, 0);
  std::vector<uint32_t> st{0};
  vis[0] = 1;
  uint32_t cnt = 1;
  while (!st.empty()) {
    uint32_t v = st.back();
    st.pop_back();
    for (uint32_t w : adj[v])
      if (!vis[w]) {
        vis[w] = 1;
        ++cnt;
        st.push_back(w);
      }
  }
  if (cnt != k) {
    if (msg) *msg = "query is not connected";
    return GAMMA_EUNSUPPORTED;
  }
  return GAMMA_OK;
}

namespace {

// Matching plan of the directed query edge (x, y).  With core_mask != 0
// (the seed edge inside it) the vertices of core_mask are placed before any
// other vertex.
GmPlan make_plan(const HostQuery& q, uint32_t qindex, uint32_t x, uint32_t y, uint32_t el,
                 const std::vector<uint64_t>& label_count, uint32_t core_mask) {
  const uint32_t k = q.k;
  std::vector<uint32_t> adjm(k, 0), deg(k, 0);
  for (auto& e : q.edges) {
    adjm[e.first] |= 1u << e.second;
    adjm[e.second] |= 1u << e.first;
    deg[e.first]++;
    deg[e.second]++;
  }
  auto lcount = [&](uint32_t u) -> uint64_t {
    uint32_t l = q.labels[u];
    return l < label_count.size() ? label_count[l] : 0;
  };
  GmPlan p;
  std::memset(&p, 0, sizeof(p));
  p.k = k;
  p.x = x;
  p.y = y;
  p.q = qindex;
  p.el = el;
  uint32_t matched = (1u << x) | (1u << y);
  p.order[0] = x;
  p.order[1] = y;
  for (uint32_t l = 2; l < k; ++l) {
    // while core vertices remain unplaced, only they are eligible
    const bool core_first = core_mask && (core_mask & ~matched) != 0;
    int best = -1;
    for (uint32_t u = 0; u < k; ++u) {
      if (matched & (1u << u)) continue;
      if (core_first && !((core_mask >> u) & 1u)) continue;
      uint32_t mn = __builtin_popcount(adjm[u] & matched);
      if (mn == 0) continue;
      if (best < 0) {
        best = (int)u;
        continue;
      }
      uint32_t bm = __builtin_popcount(adjm[best] & matched);
      if (mn != bm) {
        if (mn > bm) best = (int)u;
        continue;
      }
      if (deg[u] != deg[best]) {
        if (deg[u] > deg[best]) best = (int)u;
        continue;
      }
      if (lcount(u) != lcount(best)) {
        if (lcount(u) < lcount(best)) best = (int)u;
        continue;
      }
    }
    p.order[l] = (uint32_t)best;
    matched |= 1u << best;
  }
  uint32_t bofs = 0;
  uint32_t placed = 0;
  for (uint32_t l = 0; l < k; ++l) {
    uint32_t u = p.order[l];
    p.pos[u] = l;
    p.lab[l] = q.labels[u];
    p.back[l] = l >= 2 ? (adjm[u] & placed) : 0;
    p.bofs[l] = bofs;
    if (l >= 2) bofs += __builtin_popcount(p.back[l]);
    p.injm[l] = 0;
    for (uint32_t j = 0; j < l; ++j)
      if (q.labels[p.order[j]] == q.labels[u]) p.injm[l] |= 1u << j;
    placed |= 1u << u;
  }
  p.n_core = k;
  p.n_cperm = 1;
  p.cperm_base = 0;
  for (uint32_t u = 0; u < GM_MAX_K; ++u) p.omask[u] = 1u << u;
  return p;
}

}  // namespace

void plan_query(HostQuery& q, uint32_t qindex, const std::vector<uint64_t>& label_count) {
  q.plans.clear();
  for (size_t i = 0; i < q.edges.size(); ++i) {
    const auto& e = q.edges[i];
    const uint32_t el = i < q.elabels.size() ? q.elabels[i] : 0u;
    q.plans.push_back(make_plan(q, qindex, e.first, e.second, el, label_count, 0));
    q.plans.push_back(make_plan(q, qindex, e.second, e.first, el, label_count, 0));
  }
  coalesce_query(q);
  coalesce_core(q, label_count);
}

namespace {

// Label-preserving automorphisms of q (sigma[i] = image of query vertex i),
// by backtracking: an image must agree in label and degree with the vertex
// and in adjacency, and edge label, to every vertex mapped before it.
// Stops after `cap`.
void automorphisms(const HostQuery& q, size_t cap, std::vector<std::vector<uint32_t>>& out) {
  const uint32_t k = q.k;
  std::vector<uint32_t> adj(k, 0), deg(k, 0), m(k, 0);
  std::vector<uint32_t> el(GM_MAX_K * GM_MAX_K, 0);
  for (size_t i = 0; i < q.edges.size(); ++i) {
    const auto& e = q.edges[i];
    adj[e.first] |= 1u << e.second;
    adj[e.second] |= 1u << e.first;
    const uint32_t l = i < q.elabels.size() ? q.elabels[i] : 0u;
    el[e.first * GM_MAX_K + e.second] = el[e.second * GM_MAX_K + e.first] = l;
  }
  for (uint32_t u = 0; u < k; ++u) deg[u] = (uint32_t)__builtin_popcount(adj[u]);
  uint32_t used = 0;
  std::function<bool(uint32_t)> extend = [&](uint32_t i) -> bool {
    if (i == k) {
      out.push_back(m);
      return out.size() < cap;
    }
    for (uint32_t c = 0; c < k; ++c) {
      if (((used >> c) & 1u) || q.labels[c] != q.labels[i] || deg[c] != deg[i]) continue;
      bool ok = true;
      for (uint32_t j = 0; j < i && ok; ++j) {
        ok = ((adj[i] >> j) & 1u) == ((adj[c] >> m[j]) & 1u);
        if (ok && ((adj[i] >> j) & 1u)) ok = el[i * GM_MAX_K + j] == el[c * GM_MAX_K + m[j]];
      }
      if (!ok) continue;
      m[i] = c;
      used |= 1u << c;
      const bool more = extend(i + 1);
      used &= ~(1u << c);
      if (!more) return false;
    }
    return true;
  };
  extend(0);
}

}  // namespace

void coalesce_query(HostQuery& q) {
  const uint32_t k = q.k;
  q.perms.clear();
  GmPerm id;
  std::memset(&id, 0, sizeof(id));
  for (uint32_t i = 0; i < k; ++i) id.fwd[i] = id.inv[i] = i;
  q.perms.push_back(id);
  for (auto& p : q.plans) {
    p.n_perm = 1;  // by default every plan stands for itself
    p.perm_base = 0;
  }
  std::vector<std::vector<uint32_t>> aut;
  automorphisms(q, 4096, aut);
  if (aut.size() <= 1) return;
  std::map<std::pair<uint32_t, uint32_t>, uint32_t> dir;
  for (uint32_t i = 0; i < q.plans.size(); ++i) dir[{q.plans[i].x, q.plans[i].y}] = i;
  const uint32_t nd = (uint32_t)q.plans.size();
  std::vector<char> seen(nd, 0);
  std::vector<std::vector<uint32_t>> tau(nd);  // tau[d]: automorphism taking the class's first plan to d
  for (uint32_t d0 = 0; d0 < nd; ++d0) {
    if (seen[d0]) continue;
    std::vector<uint32_t> cls{d0};
    seen[d0] = 1;
    tau[d0].assign(id.fwd, id.fwd + k);
    for (size_t h = 0; h < cls.size(); ++h) {
      const uint32_t a = cls[h];
      for (auto& s : aut) {
        const uint32_t b = dir.at({s[q.plans[a].x], s[q.plans[a].y]});
        if (seen[b]) continue;
        seen[b] = 1;
        tau[b].resize(k);
        for (uint32_t i = 0; i < k; ++i) tau[b][i] = s[tau[a][i]];  // s after tau[a]
        cls.push_back(b);
      }
    }
    // groups of at most GM_MAX_PERM plans; the first of a group is searched,
    // pi = tau[r] o tau[m]^-1 takes member m onto the group's first plan r
    for (size_t g0 = 0; g0 < cls.size(); g0 += GM_MAX_PERM) {
      const size_t g1 = std::min(cls.size(), g0 + GM_MAX_PERM);
      const uint32_t r = cls[g0];
      q.plans[r].n_perm = (uint32_t)(g1 - g0);
      q.plans[r].perm_base = (uint32_t)q.perms.size();
      for (size_t j = g0; j < g1; ++j) {
        const uint32_t mb = cls[j];
        std::vector<uint32_t> tinv(k);
        for (uint32_t i = 0; i < k; ++i) tinv[tau[mb][i]] = i;
        GmPerm pi;
        std::memset(&pi, 0, sizeof(pi));
        for (uint32_t i = 0; i < k; ++i) pi.fwd[i] = tau[r][tinv[i]];
        for (uint32_t i = 0; i < k; ++i) pi.inv[pi.fwd[i]] = i;
        q.perms.push_back(pi);
        if (j != g0) q.plans[mb].n_perm = 0;
      }
    }
  }
}

void coalesce_core(HostQuery& q, const std::vector<uint64_t>& label_count) {
  const uint32_t k = q.k;
  q.cperms.clear();
  for (auto& p : q.plans) {
    p.n_core = k;
    p.n_cperm = 1;
    p.cperm_base = 0;
    for (uint32_t u = 0; u < GM_MAX_K; ++u) p.omask[u] = 1u << u;
  }
  if (k < 3) return;
  for (auto& p : q.plans)
    if (p.n_perm != 1) return;  // the whole query is symmetric: the k = 0 case applies
  // the core: the query without its degree-1 vertices
  std::vector<uint32_t> deg(k, 0);
  for (auto& e : q.edges) {
    deg[e.first]++;
    deg[e.second]++;
  }
  std::vector<uint32_t> cid(k, 0xFFFFFFFFu), cv;
  for (uint32_t u = 0; u < k; ++u)
    if (deg[u] >= 2) {
      cid[u] = (uint32_t)cv.size();
      cv.push_back(u);
    }
  // (a core of two vertices would be the seed edge itself, whose level is
  // entered by the seed rather than by a core match: not coalesced)
  if (cv.size() < 3 || cv.size() == k) return;
  HostQuery core;
  core.k = (uint32_t)cv.size();
  for (uint32_t v : cv) core.labels.push_back(q.labels[v]);
  for (size_t i = 0; i < q.edges.size(); ++i) {
    const auto& e = q.edges[i];
    if (cid[e.first] == 0xFFFFFFFFu || cid[e.second] == 0xFFFFFFFFu) continue;
    core.edges.push_back({cid[e.first], cid[e.second]});
    core.elabels.push_back(i < q.elabels.size() ? q.elabels[i] : 0u);
  }
  if (core.edges.empty()) return;
  std::vector<std::vector<uint32_t>> aut;
  automorphisms(core, 4096, aut);
  if (aut.size() <= 1) return;
  uint32_t core_mask = 0;
  for (uint32_t v : cv) core_mask |= 1u << v;
  // core-edge plans match the core first; their groups follow the orbits of
  // the core's directed edges (as for the whole query)
  std::map<std::pair<uint32_t, uint32_t>, uint32_t> dir;  // core ids -> plan index
  for (uint32_t i = 0; i < q.plans.size(); ++i) {
    GmPlan& p = q.plans[i];
    if (!((core_mask >> p.x) & 1u) || !((core_mask >> p.y) & 1u)) continue;
    const uint32_t el = p.el, qi = p.q;
    p = make_plan(q, qi, p.x, p.y, el, label_count, core_mask);
    p.n_perm = 1;
    p.perm_base = 0;
    p.n_core = (uint32_t)cv.size();
    dir[{cid[p.x], cid[p.y]}] = i;
  }
  const uint32_t kc = core.k;
  GmPerm id;
  std::memset(&id, 0, sizeof(id));
  for (uint32_t i = 0; i < GM_MAX_K; ++i) id.fwd[i] = id.inv[i] = i;
  std::map<uint32_t, char> seen;
  for (auto& kv : dir) {
    const uint32_t d0 = kv.second;
    if (seen.count(d0)) continue;
    std::vector<uint32_t> cls{d0};
    std::map<uint32_t, std::vector<uint32_t>> tau;  // plan -> core automorphism taking d0 to it
    seen[d0] = 1;
    tau[d0].resize(kc);
    for (uint32_t i = 0; i < kc; ++i) tau[d0][i] = i;
    for (size_t h = 0; h < cls.size(); ++h) {
      const uint32_t a = cls[h];
      for (auto& sg : aut) {
        const uint32_t b = dir.at({sg[cid[q.plans[a].x]], sg[cid[q.plans[a].y]]});
        if (seen.count(b)) continue;
        seen[b] = 1;
        tau[b].resize(kc);
        for (uint32_t i = 0; i < kc; ++i) tau[b][i] = sg[tau[a][i]];
        cls.push_back(b);
      }
    }
    for (size_t g0 = 0; g0 < cls.size(); g0 += GM_MAX_PERM) {
      const size_t g1 = std::min(cls.size(), g0 + GM_MAX_PERM);
      const uint32_t r = cls[g0];
      q.plans[r].n_cperm = (uint32_t)(g1 - g0);
      q.plans[r].cperm_base = (uint32_t)q.cperms.size();
      for (size_t j = g0; j < g1; ++j) {
        const uint32_t mb = cls[j];
        std::vector<uint32_t> tinv(kc);
        for (uint32_t i = 0; i < kc; ++i) tinv[tau[mb][i]] = i;
        // pi = tau[r] o tau[mb]^-1 on core ids, the identity on the removed vertices
        GmPerm pi = id;
        for (uint32_t i = 0; i < kc; ++i) pi.fwd[cv[i]] = cv[tau[r][tinv[i]]];
        for (uint32_t v = 0; v < k; ++v) pi.inv[pi.fwd[v]] = v;
        q.cperms.push_back(pi);
        if (j != g0) q.plans[mb].n_cperm = 0;
        // the representative's vertex u lands on pi^-1(u)
        for (uint32_t u = 0; u < k; ++u) q.plans[r].omask[u] |= 1u << pi.inv[u];
      }
    }
  }
}

void build_filter_tables(const std::vector<HostQuery>& qs, uint32_t label_slots,
                         std::vector<uint32_t>& lab_fstart, std::vector<GmFilterEntry>& entries,
                         std::vector<GmReq>& reqs) {
  std::vector<std::vector<GmFilterEntry>> per_label(label_slots);
  reqs.clear();
  for (uint32_t qi = 0; qi < qs.size(); ++qi) {
    const HostQuery& q = qs[qi];
    // per query vertex: neighbours needed per (edge label, vertex label)
    std::vector<std::map<std::pair<uint32_t, uint32_t>, uint32_t>> need(q.k);
    for (size_t i = 0; i < q.edges.size(); ++i) {
      const auto& e = q.edges[i];
      const uint32_t el = i < q.elabels.size() ? q.elabels[i] : 0u;
      need[e.first][{el, q.labels[e.second]}]++;
      need[e.second][{el, q.labels[e.first]}]++;
    }
    for (uint32_t u = 0; u < q.k; ++u) {
      uint32_t lab = q.labels[u];
      if (lab >= label_slots) continue;  // no data vertex carries this label
      GmFilterEntry fe;
      fe.q = qi;
      fe.u = u;
      fe.req_off = (uint32_t)reqs.size();
      fe.req_n = (uint32_t)need[u].size();
      for (auto& kv : need[u])
        reqs.push_back(GmReq{(uint16_t)kv.first.second, (uint16_t)kv.second, (uint16_t)kv.first.first, 0});
      per_label[lab].push_back(fe);
    }
  }
  lab_fstart.assign(label_slots + 1, 0);
  entries.clear();
  for (uint32_t l = 0; l < label_slots; ++l) {
    lab_fstart[l] = (uint32_t)entries.size();
    for (auto& fe : per_label[l]) entries.push_back(fe);
  }
  lab_fstart[label_slots] = (uint32_t)entries.size();
  if (reqs.empty()) reqs.push_back(GmReq{0, 0, 0, 0});
  if (entries.empty()) entries.push_back(GmFilterEntry{0, 0, 0, 0});
}

}  // namespace gm
