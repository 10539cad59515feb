#include "linalg.h"

#include <mutex>
#include <unordered_map>

namespace mera {

void mm(Ctx& ctx, const char* spec, std::initializer_list<std::pair<char, int64_t>> dims,
        std::initializer_list<std::pair<const char*, void*>> binds, Prec prec) {
  static std::mutex mu;
  static std::unordered_map<std::string, std::unique_ptr<Program>> cache;
  const Program* prog;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(spec);
    if (it == cache.end()) {
      std::vector<std::string> names;
      for (auto& b : binds) names.push_back(b.first);
      auto p = std::make_unique<Program>(Program::parse(std::string("mm:") + spec, {spec}, names));
      it = cache.emplace(spec, std::move(p)).first;
    }
    prog = it->second.get();
  }
  LegDims d;
  d.fill(0);
  for (auto& x : dims) d[(unsigned char)x.first] = x.second;
  std::vector<std::pair<std::string, void*>> b;
  for (auto& x : binds) b.emplace_back(x.first, x.second);
  run_program(ctx, *prog, d, b, prec);
}

}  // namespace mera
