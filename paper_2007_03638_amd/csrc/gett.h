// Permute-fused tensor contraction (GETT) on the MFMA units.
//
// One pairwise contraction C[m, n] = alpha * sum_k A[m, k] B[k, n] + beta * C[m, n], where m, n, k are
// flattened multi-leg indices. Element addresses come from per-index offset tables:
//   &A[m, k] = A + a_m[m] + a_k[k],   &B[k, n] = B + b_k[k] + b_n[n],   &C[m, n] = C + c_m[m] + c_n[n],
// so any leg permutation of the stored tensors is folded into the tile loads and the epilogue stores; no
// transposed copy is ever written. Tables are padded (offset 0) to the tile multiples so the kernels read them
// without bounds checks; out-of-range elements are masked to zero.
#pragma once

#include "common.h"

namespace mera {

struct GettTables {
  // device int64 tables, padded: m to a multiple of 128, n to 128, k to 32
  const int64_t* a_m = nullptr;
  const int64_t* a_k = nullptr;
  const int64_t* b_k = nullptr;
  const int64_t* b_n = nullptr;
  const int64_t* c_m = nullptr;
  const int64_t* c_n = nullptr;
  int64_t M = 0, N = 0, K = 0;
  bool a_kfast = false;  // A's unit-stride leg is a K leg (load threads walk k), else an M leg
  bool b_kfast = false;  // B's unit-stride leg is a K leg, else an N leg
};

// Largest number of operand sets in one grouped launch.
constexpr int kGettMaxGroup = 8;

struct GettLaunch {
  // `groups` independent operand sets (A[g], B[g], C[g]) contracted with the same tables in one launch; set g
  // computes exactly what a launch of that set alone computes.
  int groups = 1;
  const void* A[kGettMaxGroup] = {};
  const void* B[kGettMaxGroup] = {};
  void* C[kGettMaxGroup] = {};
  double alpha = 1.0, beta = 0.0;
  Prec prec = Prec::F64;
  int splits = 0;             // split-K factor (partials reduced in FP64); 0 chooses it from the extents
  bool prepare_only = false;  // size the split-K scratch and return without launching
};

// Chooses tile shape and split-K and launches on ctx.stream; `ctx` provides the split-K scratch. The choice
// depends only on the tables' extents and the precision, never on `groups`.
void gett_run(Ctx& ctx, const GettTables& t, const GettLaunch& l);

}  // namespace mera
