// Single-step contractions on small matrices and operators, written as index strings and cached as programs.
#pragma once

#include <initializer_list>
#include <utility>

#include "network.h"

namespace mera {

// Runs the one-line program `spec` (e.g. "G[nq] += -1.0 * W[np] * S[pq]") with the given leg extents and
// tensor bindings (every tensor of the line must be bound).
void mm(Ctx& ctx, const char* spec, std::initializer_list<std::pair<char, int64_t>> dims,
        std::initializer_list<std::pair<const char*, void*>> binds, Prec prec = Prec::F64);

}  // namespace mera
