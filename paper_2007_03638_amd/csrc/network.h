// Contraction programs: a tensor network written as an ordered list of pairwise contractions
//   C[labels] (+)= alpha * A[labels] * B[labels]
// over named tensors. Each tensor is stored dense and row-major over the leg order in which it is declared
// (the label string of its first appearance, or of its binding for external tensors); the label strings of
// later uses name the same axes positionally, so one buffer can appear with ket labels in one step and bra
// labels in another. A step's legs split into M (A and C only), N (B and C only) and K (A and B only); a
// leg in all three, or in one operand only, is rejected. Every step becomes one GETT launch whose offset
// tables fold the stored leg order of A, B and C into the tile loads and stores.
#pragma once

#include <array>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "gett.h"

namespace mera {

struct StepDef {
  int a, b, c;                    // tensor ids
  std::string la, lb, lc;         // per-use labels (positional)
  double alpha = 1.0;
  bool accumulate = false;        // C += ... instead of C = ...
};

// Slicing: the steps between the lines "@loop <leg>" and "@end" may run in chunks of that leg (to bound the
// size of the intermediates they create). Inside the loop, tensors created in the loop hold one chunk of the leg;
// tensors created before the loop or bound by the caller keep their full extent and are addressed at the
// chunk's offset. Steps in the loop that write a tensor without the leg accumulate over chunks ("+="), and the
// internal accumulators listed on an "@zero <names>" line are cleared before the loop.
struct Program {
  std::string name;
  std::vector<std::string> tensors;    // names
  std::vector<bool> external;          // bound by the caller
  std::vector<std::string> layout;     // declared storage labels
  std::vector<StepDef> steps;
  char slice_leg = 0;
  int loop_begin = -1, loop_end = -1;  // step range [begin, end) of the loop
  std::vector<int> zero_before;        // tensor ids cleared before the loop
  std::vector<int> produced_at;        // step index that first writes each tensor (-1: external)
  bool batch = false;                  // a batcher may group this program across contexts
  // Parse "C[cab] = A[ab] * B[bc]", "C[..] += 0.5 * A[..] * B[..]"; tensors whose name is in `externals`
  // are caller-bound, all others are intermediates owned by the context.
  static Program parse(const std::string& name, const std::vector<std::string>& lines,
                       const std::vector<std::string>& externals);
  int id(const std::string& n) const;
};

// Extent of every leg label for one instantiation of a program.
using LegDims = std::array<int64_t, 128>;

// Offset tables of every planned step, keyed by program, step and extents. Contexts of one server share one
// cache (guarded by `mu`); entries are never removed while it lives, so table pointers stay valid.
struct PlanCache {
  std::mutex mu;
  struct Entry {
    DevBuf tables;
    GettTables t;
    double macs = 0;
    bool swap = false;  // tables built for C^T = B^T A^T: the step's B is the kernel's A operand
  };
  std::unordered_map<std::string, std::unique_ptr<Entry>> map;
};

// Runs `prog` with leg extents `dims`, external tensors bound to `ext` (indexed like prog.tensors; null for
// intermediates), all tensors of element type given by `prec` (float for F32/BF16X3, double for F64).
// Intermediates live in context scratch buffers named after the tensor. `chunk` > 0 runs the program's loop
// in chunks of that many values of the loop leg (it must divide the leg's extent); 0 runs it in one piece.
// With ctx.batcher set, the call is handed to the batcher, which may run it grouped with the same program of
// other contexts (run_group); the result is the same either way.
void run_program(Ctx& ctx, const Program& prog, const LegDims& dims, const std::vector<void*>& ext, Prec prec,
                 int64_t chunk = 0);

// One operand set of a grouped run: the context whose scratch holds the intermediates, and the external
// tensors (indexed like prog.tensors).
struct Binding {
  Ctx* ctx = nullptr;
  std::vector<void*> ext;
};

// Runs `prog` for every binding (at most kGettMaxGroup) as one sequence of launches on lead.stream: step s of
// all bindings is one grouped GETT launch. Binding g's intermediates live in its own context's scratch; plans
// and split-K scratch come from `lead`. The arithmetic of each binding is that of a run of it alone.
// prepare_only allocates every buffer and plan the launches need and launches nothing, so that a following
// run (e.g. under stream capture) makes no allocation. `touched` (nullable) receives every device buffer the
// launches address. Returns the multiply-adds of one binding.
double run_group(Ctx& lead, const Program& prog, const LegDims& dims, const std::vector<Binding>& group, Prec prec,
                 int64_t chunk, bool prepare_only, std::vector<const void*>* touched);

// Receives the run_program calls of contexts that have a batcher (the server's); it must produce the results
// of run_group over that one binding, possibly as part of a larger group.
struct Batcher {
  virtual ~Batcher() = default;
  virtual void run(Ctx& ctx, const Program& prog, const LegDims& dims, const std::vector<void*>& ext, Prec prec,
                   int64_t chunk) = 0;
};

// Same, with each external tensor bound by name.
void run_program(Ctx& ctx, const Program& prog, const LegDims& dims,
                 const std::vector<std::pair<std::string, void*>>& bind, Prec prec, int64_t chunk = 0);

}  // namespace mera
