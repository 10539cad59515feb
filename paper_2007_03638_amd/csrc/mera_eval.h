// Energy and Euclidean gradient of the binary (three-site operators) and ternary (two-site operators) infinite
// MERA (Sec. 4 and App. B of arXiv:2007.03638).
#pragma once

#include <vector>

#include "common.h"
#include "vec.h"

namespace mera {

struct LayerDim {
  int a, b;           // bottom and top leg dimension of the layer
  bool ternary = false;  // ternary geometry: w has three bottom legs, operators act on two sites
  int sites() const { return ternary ? 2 : 3; }
  int64_t wrows() const { return ternary ? (int64_t)a * a * a : (int64_t)a * a; }   // rows of w
  static int64_t pw(int64_t x, int k) { int64_t r = 1; while (k-- > 0) r *= x; return r; }
  int64_t opdim(int x) const { return pw(x, sites()); }          // operator side on x-dimensional sites
  int64_t opsize(int x) const { return pw(x, 2 * sites()); }     // operator element count
};

// Transition layers 0..T-1 then the scale-invariant layer T (a = b = chi). Throws MERA_EINVAL if b_T != chi.
std::vector<LayerDim> layer_dims(const mera_shape& s);

// Krylov dimension used when the caller gives none: 16, or fewer so that the basis (dimension + 1 operators of
// vector_bytes each) stays within 16 GiB, but at least 4. Near a critical point the GMRES solves need about 14 steps
// per evaluation (measured at chi = 24); restarting after 4 costs about 25 % more operator applications there.
int default_krylov_dim(size_t vector_bytes);

// Bytes the binary transition layers' forward activations take when an evaluation keeps them for the derivative
// (0 for the ternary geometry, which does not keep them); kept only when within the context's intermediate limit.
size_t activation_cache_bytes(const std::vector<LayerDim>& dims, size_t eb);

// Device views of one evaluation point, all FP64 row-major (u: a^2 x a^2, w: a^2 x b or a^3 x b).
struct Point {
  std::vector<const double*> u, w;
};

struct Warm {
  int chi = 0;
  bool has_rho = false, has_ht = false;
  DevBuf rho, ht;  // FP64 operators (chi^6 binary, chi^4 ternary) of the last evaluation
  // for extrapolated starts: the solutions of the evaluation before (valid with has_prev) and the tensors of the
  // last two evaluation points, flattened (pts[0] the newer; npts of them valid)
  bool has_prev = false;
  DevBuf rho_prev, ht_prev;
  DevBuf pts[2];
  int npts = 0;
  int64_t pt_elems = 0;
};

struct KrylovOpts {
  int dim = 0;  // 0: default_krylov_dim of the vector size
  int max_restarts = 200;
  double tol = 0.0;  // 0: precision default
  bool extrapolate = true;  // start from the last two solutions extrapolated along the step (needs a Warm)
};

struct EvalOut {
  double energy = 0;
  int app_rho = 0, app_ht = 0;
  double res_rho = 0, res_ht = 0;
  double macs = 0;
};

// Gradient outputs (FP64 device, caller-owned), and optional preconditioner density matrices.
struct GradOut {
  std::vector<double*> Du, Dw;
  std::vector<double*> rho_u, rho_w;  // may be empty
};

EvalOut energy_grad(Ctx& ctx, const mera_shape& shape, const Point& pt, const double* h3, Prec prec, Warm* warm,
                    const KrylovOpts& ko, const GradOut& out);

// One layer map on FP64 device operators (converted internally for FP32/BF16X3).
void ascend_op(Ctx& ctx, const LayerDim& L, const double* u, const double* w, Prec prec, const double* hin,
               double* hout);
void descend_op(Ctx& ctx, const LayerDim& L, const double* u, const double* w, Prec prec, const double* rin,
                double* rout);

// Derivative of Tr[A(h) rho] of one layer with h and rho held fixed (FP64 device operators in and out): Du, Dw
// (Euclidean, FP64), rout (nullable) = D(rho). split: run the forward halves (hout, nullable, receives A(h)) and
// then the reverse halves from the kept activations, as an evaluation does for its binary transition layers;
// otherwise the combined programs, as for the scale-invariant layer (hout must be null).
void layer_grad_op(Ctx& ctx, const LayerDim& L, const double* u, const double* w, Prec prec, bool split,
                   const double* hin, const double* rin, double* hout, double* Du, double* Dw, double* rout);

}  // namespace mera
