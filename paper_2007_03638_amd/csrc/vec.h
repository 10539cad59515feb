// Memory-bound vector and small-matrix kernels: dot products with FP64 accumulation, axpby, conversions,
// symmetrisation, traces, and the cyclic two-sided Jacobi eigensolver for small symmetric matrices.
#pragma once

#include <vector>

#include "common.h"

namespace mera {

// Typed device pointer of either precision.
struct VPtr {
  void* p = nullptr;
  Prec prec = Prec::F64;  // F64: double storage; F32/BF16X3: float storage
  bool dbl() const { return prec == Prec::F64; }
};

double dot(Ctx& ctx, VPtr x, VPtr y, int64_t n);               // sum x*y in FP64 (syncs)
// out[i] = <x_i, y_i> (lengths n_i) for count pairs with one synchronisation; each equals dot(x_i, y_i) bitwise
void dots(Ctx& ctx, const VPtr* x, const VPtr* y, const int64_t* n, int count, double* out);
double nrm2(Ctx& ctx, VPtr x, int64_t n);
void axpby(Ctx& ctx, double a, VPtr x, double b, VPtr y, int64_t n);  // y = a x + b y
// out[j] = <w, v_j>, j < k (host array), FP64 accumulation, one pass over w per 17 vectors (syncs). All vectors of
// one precision.
void multi_dot(Ctx& ctx, const VPtr* v, int k, VPtr w, int64_t n, double* out);
// y <- b y + sum_j c_j v_j (c: host array of k), accumulated in FP64, one pass per 17 vectors (b == 0: y is not
// read). All vectors of one precision; y must not be one of the v_j.
void multi_axpby(Ctx& ctx, const VPtr* v, const double* c, int k, double b, VPtr y, int64_t n);
void scal(Ctx& ctx, double a, VPtr x, int64_t n);
void copy(Ctx& ctx, VPtr dst, VPtr src, int64_t n);            // with conversion
void fill(Ctx& ctx, VPtr x, int64_t n, double v);
// X (dim x dim, row-major) <- (X + X^T)/2
void symmetrize(Ctx& ctx, VPtr x, int64_t dim);
// X_ii += c
void add_diag(Ctx& ctx, VPtr x, int64_t dim, double c);
double trace(Ctx& ctx, VPtr x, int64_t dim);                   // syncs

// The same reductions and updates with FP64 scalars that stay in device memory (no host synchronisation): results
// are written to, and coefficients read from, device addresses; s scales a coefficient read from the device.
void dot_dev(Ctx& ctx, VPtr x, VPtr y, int64_t n, double* out_dev);                       // *out = <x, y>
// FP64 device scalars computed exactly as their host counterparts: <x, y> with the partials added in order, as
// dot() adds them; x <- (num / den) x as scal(num / den); y <- (r p - r q) x + b y as axpby(r p - r q, x, b, y)
void dot_dev_exact(Ctx& ctx, const double* x, const double* y, int64_t n, double* out_dev);
void scal_ratio_dev(Ctx& ctx, const double* num_dev, const double* den_dev, double* x, int64_t n);
void axpby_diff_dev(Ctx& ctx, double r, const double* p_dev, const double* q_dev, const double* x, double b,
                    double* y, int64_t n);
void trace_dev(Ctx& ctx, VPtr x, int64_t dim, double* out_dev);                           // *out = Tr X
void axpby_dev(Ctx& ctx, const double* a_dev, double s, VPtr x, double b, VPtr y, int64_t n);  // y = s*a x + b y
void add_diag_dev(Ctx& ctx, VPtr x, int64_t dim, const double* c_dev, double s);          // X_ii += s*c
void multi_dot_dev(Ctx& ctx, const VPtr* v, int k, VPtr w, int64_t n, double* out_dev);    // out[j] = <w, v_j>
// y <- b y + sum_j (s c[j]) v_j
void multi_axpby_dev(Ctx& ctx, const VPtr* v, const double* c_dev, double s, int k, double b, VPtr y, int64_t n);
// *nrm = |x|, then x <- x / |x| when |x| > 0 (work_dev: one double of scratch)
void normalize_dev(Ctx& ctx, VPtr x, int64_t n, double* nrm_dev, double* work_dev);

// Symmetric eigendecomposition of a dim x dim FP64 matrix (row-major, device) by cyclic two-sided Jacobi
// rotations in tournament order: A = V diag(lam) V^T, eigenvectors in the columns of V. `a` is overwritten.
// v_init: v holds an orthogonal basis Q on entry and a = Q^T A Q; the rotations are then accumulated onto Q, so
// that v returns the eigenvectors of A (few sweeps when Q nearly diagonalises A). Matrices up to 160 x 160 run in one
// launch (one workgroup; A and V in LDS up to 64 x 64); larger ones launch one kernel per round.
void jacobi_eigh(Ctx& ctx, double* a, double* lam, double* v, int dim, double tol = 1e-15, int max_sweeps = 30,
                 bool v_init = false);

// Several independent decompositions (arguments as for jacobi_eigh, distinct buffers): those of matrices up to
// 160 x 160 run together, up to 16 per launch, one workgroup each (up to 64 x 64 with A and V in LDS, above that with
// both in global memory and a 1024-thread workgroup); larger ones launch one kernel per round.
struct JacobiTask {
  double* a;
  double* lam;
  double* v;
  int dim;
  double tol = 1e-15;
  int max_sweeps = 30;
  bool v_init = false;
};
void jacobi_eigh_batch(Ctx& ctx, const std::vector<JacobiTask>& tasks);

// Element-wise helpers for the preconditioner (all FP64, device):
//   M_ij <- M_ij * 2 / (f_i + f_j)
void scale_sylvester(Ctx& ctx, double* m, const double* f, int dim);
//   M_ij <- M_ij * s_j   (column scaling)
void scale_cols(Ctx& ctx, double* m, const double* s, int64_t rows, int cols);
//   dst[i * ldd + j] = a * src[i * lds + j] for a rows x cols block (row-major, strided)
void copy_block(Ctx& ctx, double* dst, int64_t ldd, const double* src, int64_t lds, int rows, int cols, double a);
//   f_i <- sqrt(lam_i^2 + delta^2), g_i <- 1/f_i
void reg_spectrum(Ctx& ctx, const double* lam, double delta, double* f, double* g, int dim);

// Marginals of a 3-site density matrix rho[p q r, P Q R] (b^3 x b^3, float or double):
//   rho1[q, Q]        = sum_{p r} rho[p q r, p Q r]                       (middle site)
//   rho2[x y, X Y]    = ( sum_r rho[x y r, X Y r] + sum_p rho[p x y, p X Y] ) / 2
// outputs FP64 device, b x b and b^2 x b^2.
void rho_marginals(Ctx& ctx, VPtr rho, int b, double* rho1, double* rho2);
// One-site marginal of a two-site density matrix rho[p q, P Q] (b^2 x b^2, FP64), averaged over both sites:
//   rho1[x, X] = ( sum_q rho[x q, X q] + sum_p rho[p x, p X] ) / 2                     (b x b, FP64 device)
void rho_marginal_pair(Ctx& ctx, VPtr rho, int b, double* rho1);

}  // namespace mera
