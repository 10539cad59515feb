// Single-step contractions on small matrices and operators, written as index strings and cached as programs.
#pragma once

#include <initializer_list>
#include <utility>
#include <vector>

#include "network.h"

namespace mera {

// Runs the one-line program `spec` (e.g. "G[nq] += -1.0 * W[np] * S[pq]") with the given leg extents and
// tensor bindings (every tensor of the line must be bound).
void mm(Ctx& ctx, const char* spec, std::initializer_list<std::pair<char, int64_t>> dims,
        std::initializer_list<std::pair<const char*, void*>> binds, Prec prec = Prec::F64);

// The same line for several binding sets of identical extents, in grouped launches of up to kGettMaxGroup sets
// (each set computes exactly what mm computes for it). `names` lists the tensors; sets[j][t] binds names[t].
void mm_group(Ctx& ctx, const char* spec, std::initializer_list<std::pair<char, int64_t>> dims,
              const std::vector<const char*>& names, const std::vector<std::vector<void*>>& sets,
              Prec prec = Prec::F64);

}  // namespace mera
