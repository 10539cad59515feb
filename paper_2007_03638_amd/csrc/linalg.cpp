#include "linalg.h"

#include <algorithm>
#include <mutex>
#include <unordered_map>

namespace mera {

namespace {

// The one-line program of `spec`, parsed once (the external tensors are `names`).
const Program& line_program(const char* spec, const std::vector<std::string>& names) {
  static std::mutex mu;
  static std::unordered_map<std::string, std::unique_ptr<Program>> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(spec);
  if (it == cache.end()) {
    auto p = std::make_unique<Program>(Program::parse(std::string("mm:") + spec, {spec}, names));
    it = cache.emplace(spec, std::move(p)).first;
  }
  return *it->second;
}

}  // namespace

void mm(Ctx& ctx, const char* spec, std::initializer_list<std::pair<char, int64_t>> dims,
        std::initializer_list<std::pair<const char*, void*>> binds, Prec prec) {
  std::vector<std::string> names;
  for (auto& b : binds) names.push_back(b.first);
  const Program* prog = &line_program(spec, names);
  LegDims d;
  d.fill(0);
  for (auto& x : dims) d[(unsigned char)x.first] = x.second;
  std::vector<std::pair<std::string, void*>> b;
  for (auto& x : binds) b.emplace_back(x.first, x.second);
  run_program(ctx, *prog, d, b, prec);
}

void mm_group(Ctx& ctx, const char* spec, std::initializer_list<std::pair<char, int64_t>> dims,
              const std::vector<const char*>& names, const std::vector<std::vector<void*>>& sets, Prec prec) {
  if (sets.empty()) return;
  const std::vector<std::string> nm(names.begin(), names.end());
  const Program& prog = line_program(spec, nm);
  LegDims d;
  d.fill(0);
  for (auto& x : dims) d[(unsigned char)x.first] = x.second;
  std::vector<int> slot(names.size());
  for (size_t t = 0; t < names.size(); ++t) {
    slot[t] = prog.id(names[t]);
    MERA_CHECK(slot[t] >= 0, MERA_EINVAL, std::string("mm_group: unknown tensor ") + names[t]);
  }
  for (size_t j0 = 0; j0 < sets.size(); j0 += kGettMaxGroup) {
    const size_t j1 = std::min(sets.size(), j0 + (size_t)kGettMaxGroup);
    std::vector<Binding> group;
    for (size_t j = j0; j < j1; ++j) {
      MERA_CHECK(sets[j].size() == names.size(), MERA_EINVAL, "mm_group: binding count");
      Binding b;
      b.ctx = &ctx;
      b.ext.assign(prog.tensors.size(), nullptr);
      for (size_t t = 0; t < names.size(); ++t) b.ext[slot[t]] = sets[j][t];
      group.push_back(std::move(b));
    }
    run_group(ctx, prog, d, group, prec, 0, false, nullptr);
  }
}

}  // namespace mera
