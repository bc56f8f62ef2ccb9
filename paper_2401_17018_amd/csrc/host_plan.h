// Host-side query validation, matching-order planning and candidate-filter
// tables.  Internal to the library.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "dev_common.h"

namespace gm {

struct HostQuery {
  uint32_t k = 0;
  std::vector<uint32_t> labels;                       // [k]
  std::vector<std::pair<uint32_t, uint32_t>> edges;   // undirected, as given
  std::vector<uint32_t> elabels;                      // [m] edge label per edge (0 without labels)
  std::vector<GmPlan> plans;                          // one per directed edge
  std::vector<GmPerm> perms;                          // coalesced search, referenced by plans
  std::vector<GmPerm> cperms;                         // core-prefix permutations (k > 0 coalescing)
  bool paused = false;                                // kept current but not searched
};

// Validates a query; on failure returns the status code (EINVAL or
// EUNSUPPORTED, as in gamma.h) and a message.
int validate_query(uint32_t k, const uint32_t* qlabels, uint32_t m, const uint32_t* qedges,
                   std::string* msg);

// Matching order per directed query edge (x, y), the order rule of Sec. IV-C
// ("more selective first"): x, y, then repeatedly the unmatched vertex with
// the most matched neighbours; ties go to the higher query degree, then to
// the rarer label (label_count), then to the lower id.
void plan_query(HostQuery& q, uint32_t qindex, const std::vector<uint64_t>& label_count);

// Coalesced search (Sec. V-B) for automorphisms of the whole query: finds
// label-preserving automorphisms (up to a cap), groups the directed query
// edges they map onto each other (groups of at most GM_MAX_PERM), and sets
// each plan's n_perm / perm_base (perm_base indexes q.perms).
void coalesce_query(HostQuery& q);

// Coalesced search over the k-degenerated automorphic subgraph obtained by
// removing the degree-1 query vertices (Sec. V-B), for queries whose own
// automorphism group is trivial: if the remaining core has label- and
// edge-label-preserving automorphisms, core-edge plans are re-planned core
// first and grouped by the orbits of the core's directed edges (n_core,
// n_cperm, cperm_base; cperm_base indexes q.cperms) and each
// representative's omask is set.
void coalesce_core(HostQuery& q, const std::vector<uint64_t>& label_count);

// Candidate-filter tables for all queries over data labels < label_slots:
// entries per data label (sorted by query), each with its neighbour-label
// requirements (Sec. IV-B).
void build_filter_tables(const std::vector<HostQuery>& qs, uint32_t label_slots,
                         std::vector<uint32_t>& lab_fstart, std::vector<GmFilterEntry>& entries,
                         std::vector<GmReq>& reqs);

}  // namespace gm
