// Stiefel-manifold operations, Hilbert-space preconditioner, L-BFGS and the optimisation driver
// (Sec. 2 and Sec. 3 of arXiv:2007.03638). All arithmetic here is FP64 on the device; host code only
// handles scalars (inner products, line-search decisions).
#pragma once

#include <functional>
#include <vector>

#include "common.h"
#include "mera_eval.h"

namespace mera {

struct MatView {
  int n = 0, p = 0;
  double* data = nullptr;
};

// Points and tangent vectors of a product of Stiefel manifolds, stored as one flat FP64 device buffer.
struct Flat {
  std::vector<int> n, p;
  std::vector<int64_t> off;
  int64_t total = 0;
  DevBuf buf;
  Flat() = default;
  Flat(const std::vector<int>& n_, const std::vector<int>& p_) { init(n_, p_); }
  void init(const std::vector<int>& n_, const std::vector<int>& p_);
  int count() const { return (int)n.size(); }
  double* ptr() const { return buf.as<double>(); }
  MatView view(int i) const { return MatView{n[i], p[i], buf.as<double>() + off[i]}; }
  std::vector<MatView> views() const;
};

// G = D - W sym(W^T D)                                      (eq. stiefel_gradient, real case)
void stiefel_project_one(Ctx& ctx, const MatView& W, const MatView& D, const MatView& G);
// W_out = polar(W + alpha X), X_out = dW_out/dalpha (nullable)
void stiefel_retract_one(Ctx& ctx, const MatView& W, const MatView& X, double alpha, const MatView& Wout,
                         const MatView* Xout);
// Projections G_j = D_j - W_j sym(W_j^T D_j) (Grassmann items: without sym) of several items, those of equal shape
// in grouped launches; each item computes exactly what the one-item call computes (G_j may alias D_j).
void project_many(Ctx& ctx, const std::vector<MatView>& W, const std::vector<MatView>& D,
                  const std::vector<MatView>& G, const std::vector<bool>& grassmann);
// The same for several factors at once (each computed exactly as alone; one synchronisation per iteration step)
void stiefel_retract_many(Ctx& ctx, const std::vector<MatView>& W, const std::vector<MatView>& X, double alpha,
                          const std::vector<MatView>& Wout, const std::vector<const MatView*>& Xout);

// G = (1 - W W^T) D: Grassmann tangent projection (eq. grassmann_gradient, real case)
void grassmann_project_one(Ctx& ctx, const MatView& W, const MatView& D, const MatView& G);

// Low-rank form of the generator Q_X of the exponential retraction and transport (Sec. 2.3, eqs. retraction and
// transport): Q_X = U M U^T with U = [W Q], M = [[A, -B^T], [B, 0]], A = W^T X, Z = (1 - W W^T) X = Q B. Q spans
// range(Z) (n x p, columns without a component of Z are zero and have zero rows of B); square W has no Q (m = p).
// E = exp(alpha M) is set per alpha.
struct ExpFrame {
  int n = 0, p = 0, m = 0;
  DevBuf Q, M, E;
  double alpha = 0;
  bool has_alpha = false;
};
void exp_frame_one(Ctx& ctx, const MatView& W, const MatView& X, ExpFrame& fr);
void exp_set_alpha(Ctx& ctx, ExpFrame& fr, double alpha);
// out = exp(alpha Q_X) Y = Y + U (E - 1) U^T Y  (out may alias Y)
void exp_apply_one(Ctx& ctx, const MatView& W, const ExpFrame& fr, const MatView& Y, const MatView& out);
// W_out = exp(alpha Q_X) W with one Newton-Schulz polar refinement (removes accumulated rounding), X_out (nullable)
// = exp(alpha Q_X) X, the curve derivative. The frame must be built for (W, X).
void exp_retract_one(Ctx& ctx, const MatView& W, const MatView& X, ExpFrame& fr, double alpha, const MatView& Wout,
                     const MatView* Xout);

// Evenbly-Vidal local update (App. A): W_out = polar(gamma W rho - D), the polar factor of minus the environment
// of the shifted Hamiltonian H - gamma; polar(Y) = Y (Y^T Y)^{-1/2} from the FP64 Jacobi eigendecomposition of
// Y^T Y, then one Newton-Schulz refinement. W_out must not alias W or D.
void ev_update_one(Ctx& ctx, const MatView& W, const MatView& D, const MatView& rho, double gamma,
                   const MatView& Wout);

// Eigendecompositions of the preconditioner metrics rho_v (one per factor).
struct Metric {
  std::vector<DevBuf> V, lam, f, g;
  std::vector<int> p;
  std::vector<int> warm;  // per factor: decompositions since the last one from scratch (0: no basis kept)
  void compute(Ctx& ctx, const std::vector<MatView>& rho);
  bool empty() const { return p.empty(); }
};
// X_out = preconditioned X for factor i (Sec. 3 eqs. preconditioner / preconditioner_solution); delta < 0
// takes delta = ||X||_F (Sec. 4). X_out may alias X.
void precondition_one(Ctx& ctx, const MatView& W, const MatView& X, Metric& met, int i, double delta,
                      const MatView& Xout);
// The same for several factors (delta[i] >= 0 given per factor), those of equal shape in grouped launches; each
// factor computes exactly what precondition_one computes for it.
void precondition_many(Ctx& ctx, const std::vector<MatView>& W, const std::vector<MatView>& X, Metric& met,
                       const std::vector<double>& delta, const std::vector<MatView>& Xout);

struct Lbfgs {
  int m = 8;
  Flat shape;                    // factor sizes
  std::vector<DevBuf> S, Y;      // ring slots, each `total` doubles
  std::vector<double> r;         // 1 / <s_i, y_i>
  std::vector<int> order;        // slot indices, oldest first
  DevBuf q, z, t;
  void init(Ctx& ctx, const std::vector<int>& n, const std::vector<int>& p, int m);
  void reset() { order.clear(); }
  int size() const { return (int)order.size(); }
  // two-loop recursion; returns slope <G, d>
  double step(Ctx& ctx, const std::vector<MatView>& W, const std::vector<MatView>& G, Metric* met,
              const std::vector<MatView>& dout);
  // After an accepted step: transport the stored pairs with T, form s = T(alpha d), y = G_new - T(G_old), store the
  // pair if <s, y> > 1e-12 |s||y|. T(i, in, out) transports factor i (out may alias in).
  // TM, when given, transports the stored pairs all at once: TM(factor[j], in[j], out[j]) for every item j.
  using Transport = std::function<void(int, const MatView&, const MatView&)>;
  using TransportMany =
      std::function<void(const std::vector<int>&, const std::vector<MatView>&, const std::vector<MatView>&)>;
  bool push(Ctx& ctx, const Transport& T, const std::vector<MatView>& d, double alpha,
            const std::vector<MatView>& Gold, const std::vector<MatView>& Gnew, const TransportMany& TM = nullptr);
  // Same with the projection transport onto the tangent spaces at Wn.
  bool push(Ctx& ctx, const std::vector<MatView>& Wn, const std::vector<MatView>& d, double alpha,
            const std::vector<MatView>& Gold, const std::vector<MatView>& Gnew);
};

double inner(Ctx& ctx, const std::vector<MatView>& X, const std::vector<MatView>& Y);

struct OptResult {
  double energy = 0, gnorm = 0, seconds = 0, macs = 0;
  int iterations = 0, evaluations = 0, status = 0, polish_iter = -1, krylov_apps = 0;
  std::vector<mera_iter_log> log;
};

struct JobSpec {
  mera_shape shape{};
  std::vector<double> h3;                  // d^3 x d^3 host
  std::vector<std::vector<double>> init;   // 2(T+1) host matrices
  Prec prec = Prec::F64;
  int m = 8, max_iter = 100, max_ls_evals = 10;
  double grad_tol = 1e-10, polish_tol = 0.0;
  bool precondition = true;
  int method = 0;                          // 0: L-BFGS, 1: nonlinear CG (Hager-Zhang), 2: Evenbly-Vidal sweeps
  double ev_gamma = 0.0;                   // Evenbly-Vidal shift (inverse step size)
  int retraction = 0;                      // 0: polar + projection transport, 1: exponential (Sec. 2.3)
  bool grassmann_w = false;                // isometries w on Grassmann manifolds (Sec. 4)
  KrylovOpts krylov;
  static JobSpec from_c(const mera_job& j);
};

// Whole optimisation of one job on `ctx` (blocking). Final tensors copied to `final_host` if non-empty.
OptResult optimize(Ctx& ctx, const JobSpec& job, std::vector<double*>* final_host, int log_cap);

// Resumable optimiser state machine used by the server: each call to advance() runs one iteration
// (its evaluations and Stiefel steps) and returns true once the job has finished.
struct Optimizer {
  Ctx* ctx = nullptr;
  JobSpec job;
  std::vector<LayerDim> dims;
  Flat W, G, Wn, Gn, D, Xp, dir, rv, rvn;
  DevBuf h3dev;
  Warm warm;
  Lbfgs hist;
  Metric met;
  // nonlinear CG state: previous direction transported to the current point, y = G - T(G_prev), scratch
  Flat cg_d, cg_y, cg_pg, cg_py;
  std::vector<char> grass;        // factor i is a Grassmann point
  std::vector<ExpFrame> frames;   // exponential retraction: generator of the current direction, per factor
  bool cg_have = false;
  double cg_gold = 0, cg_alpha_prev = 0, cg_slope_prev = 0;
  Prec prec = Prec::F64;
  double f = 0, gnorm = 0, last_alpha = 0;
  int iter = 0, evals = 0, status = -1, polish_iter = -1, krylov_apps = 0;
  bool done = false, started = false;
  double macs0 = 0;
  OptResult result;
  int log_cap = 0;

  void start(Ctx& c, const JobSpec& j, int log_cap_ = 0);
  bool advance();                       // one iteration
  void finish(std::vector<double*>* final_host);
  size_t device_bytes() const;

 private:
  double evaluate(const Flat& X, Flat& Gout, Flat& rvout);   // energy; fills G = P(D) and metrics
  bool need_rv() const { return job.precondition || job.method == 2; }
  void ev_sweep();                // one Evenbly-Vidal sweep over all tensors
  // CG direction into `dir` (Sec. 3, Hager-Zhang coefficient); returns the slope <G, dir>, sets `momentum` when
  // the previous direction was used and `alpha0` to the first trial step
  double cg_direction(Metric* met, bool& momentum, double& alpha0);
  void cg_restart(Metric* met);   // dir = -P G
  void project_factor(int i, const MatView& W, const MatView& D, const MatView& G);
  void build_frames();            // exponential retraction frames for (W, dir)
  // vector transport from W to the accepted point Wn (polar: projection at Wn; exponential: exp(alpha Q_dir))
  void transport_factor(int i, const MatView& in, const MatView& out);
};

}  // namespace mera
