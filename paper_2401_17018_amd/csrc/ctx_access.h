// Library-internal read access to a context (for the serving layer).
#pragma once
#include <stdint.h>

struct gamma_ctx;

namespace gm {
// true if a graph is loaded; *n receives its vertex count and *n_el (may
// be null) its number of edge labels
bool ctx_has_graph(const gamma_ctx* c, uint32_t* n, uint32_t* n_el = nullptr);
// the context's tuple buffer capacity (records)
uint64_t ctx_tuple_capacity(const gamma_ctx* c);
}  // namespace gm
