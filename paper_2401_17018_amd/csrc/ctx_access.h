// Library-internal read access to a context (for the serving layer).
#pragma once
#include <stdint.h>

struct gamma_ctx;

namespace gm {
// true if a graph is loaded; *n receives its vertex count
bool ctx_has_graph(const gamma_ctx* c, uint32_t* n);
}  // namespace gm
