// Permute-fused tensor contraction (GETT) on the MFMA units.
//
// One pairwise contraction C[m, n] = alpha * sum_k A[m, k] B[k, n] + beta * C[m, n], where m, n, k are
// flattened multi-leg indices. Element addresses are
//   &A[m, k] = A + a_m[m] + a_off(k),   &B[k, n] = B + b_off(k) + b_n[n],   &C[m, n] = C + c_m[m] + c_n[n],
// with per-index offset tables for m and n and the k offsets computed from the K legs' extents and strides, so
// any leg permutation of the stored tensors is folded into the tile loads and the epilogue stores; no transposed
// copy is ever written. Tables are padded (offset 0) to the tile multiples so the kernels read them without bounds
// checks; k past the end is masked to zero.
#pragma once

#include "common.h"

namespace mera {

// K index as a mixed-radix number over the contracted legs, fastest leg first: k = d_0 + ext_0 (d_1 + ext_1 (...)),
// so &A[., k] adds sum_l d_l sa[l] and &B[k, .] adds sum_l d_l sb[l]. The kernels form these offsets
// arithmetically (no table, no memory load): q / ext_l = mulhi(q, mag_l) with mag_l = ceil(2^32 / ext_l), exact
// because every quotient q met satisfies q * ext_l <= 2^32 (checked when the legs are built); the slowest leg has
// mag 0 (its digit is the whole remaining quotient). Legs of extent 1 are dropped and legs contiguous in both
// operands merged; unused entries are zero. Strides are 32-bit (in elements, checked when the legs are built); the
// digits are formed in 32-bit arithmetic and each digit-stride product is accumulated into a 64-bit offset.
constexpr int kGettMaxKLegs = 4;
struct GettKLegs {
  int n = 0;
  uint32_t ext[kGettMaxKLegs] = {};
  uint32_t mag[kGettMaxKLegs] = {};
  uint32_t sa[kGettMaxKLegs] = {};
  uint32_t sb[kGettMaxKLegs] = {};
};

struct GettTables {
  // device int64 tables, padded: m to a multiple of 128, n to 128
  const int64_t* a_m = nullptr;
  const int64_t* b_n = nullptr;
  const int64_t* c_m = nullptr;
  const int64_t* c_n = nullptr;
  GettKLegs kl;
  int64_t M = 0, N = 0, K = 0;
  bool a_kfast = false;  // A's unit-stride leg is a K leg (load threads walk k), else an M leg
  bool b_kfast = false;  // B's unit-stride leg is a K leg, else an N leg
  // Largest vector width w in {1, 2, 4} elements the operand's layout allows for tile loads: its unit-stride leg
  // is the fastest index its loader walks (k when kfast, else m or n), and that leg's extent and every other
  // stride are multiples of w. The kernels load 16 bytes (w = 4 FP32, w = 2 FP64) when both operands allow it.
  int a_vw = 1, b_vw = 1;
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
