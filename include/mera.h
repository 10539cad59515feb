/*
 * mera.h — C ABI of the MI355X (gfx950) library for Riemannian optimisation of an infinite, scale-invariant
 * binary MERA.
 *
 * Method: Hauru, Van Damme & Haegeman, "Riemannian optimization of isometric tensor networks",
 * arXiv:2007.03638. Section numbers below refer to that paper.
 *
 * Conventions (all calls)
 *   - Every call returns a mera_status; nothing else signals failure, and no exception crosses the ABI.
 *     On error the outputs are unspecified and mera_last_error(ctx) holds a message.
 *   - Matrices (mera_mat) are REAL, FP64, ROW-MAJOR n x p, in DEVICE memory of the context's GPU, and are
 *     owned by the caller. For an isometry the rows index the bottom (incoming) legs and the columns the top
 *     (outgoing) legs: a disentangler u is a^2 x a^2 with rows (bl, br) and columns (tl, tr); an isometry w is
 *     a^2 x b with rows (bl, br) and column t (ternary geometry: a^3 x b, rows (bl, bc, br)). Leg indices are
 *     row-major (first leg slowest).
 *   - Local operators are row-major FP64 matrices on the sites a term covers: d^3 x d^3 for the binary geometry's
 *     three-site terms (rows = ket legs abc, columns = bra legs ABC), d^2 x d^2 for the ternary geometry's two-site
 *     terms (rows ab, columns AB). "h3" arguments below take whichever the shape's geometry uses.
 *   - All device work is ordered on the context's HIP stream. Calls that return host scalars synchronise it.
 *   - The library owns only what its *_create calls allocate and frees it in the matching *_destroy.
 *   - Layer geometry: T transition layers and one scale-invariant layer. Layer 1 has bottom dimension a_1 = d;
 *     layer tau has top dimension b_tau = min(chi, a_tau^2) (binary) or min(chi, a_tau^3) (ternary), a_{tau+1} = b_tau; the scale-invariant layer
 *     has a = b = chi, so b_T must equal chi (MERA_EINVAL otherwise). Tensor arrays are indexed by layer,
 *     0..T-1 for the transition layers and T for the scale-invariant one.
 */
#ifndef MERA_H
#define MERA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MERA_OK = 0,
  MERA_EINVAL = -1,      /* bad argument: shape mismatch, null pointer, unsupported size            */
  MERA_ENOMEM = -2,      /* device allocation failed                                                  */
  MERA_EHIP = -3,        /* a HIP runtime call failed                                                 */
  MERA_ENOCONV = -4,     /* an iteration (Krylov solve, line search) did not reach its tolerance      */
  MERA_ENONFINITE = -5,  /* a NaN or Inf appeared in an energy, a norm or an inner product            */
  MERA_EBUSY = -6        /* the job is still running (server polling)                                 */
} mera_status;

/* Arithmetic of the bulk contractions. FP64: double-precision MFMA throughout. FP32: single-precision
 * MFMA with single-precision accumulation, double-precision dot products, traces and Krylov scalars.
 * BF16X3: each FP32 operand split into bf16 hi + lo parts, products hi*hi + hi*lo + lo*hi on the bf16
 * MFMA units with FP32 accumulation. */
typedef enum { MERA_FP64 = 0, MERA_FP32 = 1, MERA_BF16X3 = 2 } mera_prec;

typedef struct { int n, p; double* data; } mera_mat;

typedef struct {
  int T;         /* number of transition layers (>= 1)                                                  */
  int d;         /* physical site dimension: 4 for two blocked spins (binary), 2 for one spin (ternary)  */
  int chi;       /* bond dimension of the scale-invariant layer                                          */
  int geometry;  /* 0: binary MERA with three-site operators (u a^2 x a^2, w a^2 x b, b = min(chi, a^2));  */
                 /* 1: ternary MERA with two-site operators, the paper's benchmark geometry (Sec. 4):      */
                 /*    u a^2 x a^2, w a^3 x b, b = min(chi, a^3); operators are b^2 x b^2                  */
} mera_shape;

typedef struct mera_ctx mera_ctx;
typedef struct mera_warm mera_warm;
typedef struct mera_lbfgs mera_lbfgs;
typedef struct mera_server mera_server;

/* ---- context ------------------------------------------------------------------------------------------ */

/* Create a context on HIP device `device`. `hip_stream` is a hipStream_t owned by the caller, or NULL for
 * the default stream. */
mera_status mera_ctx_create(int device, void* hip_stream, mera_ctx** out);
void mera_ctx_destroy(mera_ctx* ctx);
const char* mera_last_error(const mera_ctx* ctx);
/* Release the context's cached device workspace (intermediate tensors, offset tables). */
mera_status mera_ctx_trim(mera_ctx* ctx);
/* Multiply-accumulate count of every contraction issued on the context since creation (algorithmic:
 * the product of all leg dimensions of each pairwise step, no padding). */
double mera_ctx_macs(const mera_ctx* ctx);

/* Kernel timing: with profiling on, every contraction launch is bracketed by HIP events on the context
 * stream. mera_ctx_kernel_stats synchronises, aggregates the recorded launches by kernel variant into
 * out[0..cap) (largest total time first), clears the records and returns the number of variants (<0: error). */
typedef struct {
  char kernel[80];   /* kernel variant: precision, tile, operand load order, split-K */
  int launches;
  double seconds;    /* summed launch durations (event to event)                      */
  double flops;      /* summed algorithmic flops, 2 x M x N x K per launch            */
  double bytes;      /* summed algorithmic bytes: A, B and C each moved once          */
} mera_kernel_stat;
mera_status mera_ctx_profile(mera_ctx* ctx, int enable);
int mera_ctx_kernel_stats(mera_ctx* ctx, mera_kernel_stat* out, int cap);

/* Memory bound for the two largest intermediates of a layer program (7-leg tensors of a^6 b elements): when one
 * would exceed `bytes`, the program runs in chunks of a spectator leg so that each chunked intermediate stays
 * within bytes/2 (default 32 GiB; results are unchanged up to rounding order). The same bound decides whether a
 * binary evaluation keeps the transition layers' forward activations for their derivatives (kept when their total,
 * 2 (2 a^6 + a^4 b^2 + a^2 b^4) elements per layer, fits; results equal up to rounding order either way). */
mera_status mera_ctx_set_intermediate_limit(mera_ctx* ctx, size_t bytes);

/* Progress reports on stderr: level > 0 prints a line at every restart of the two Krylov solves of an evaluation
 * (applications so far, relative residual); 0 (default) prints nothing. For long evaluations at large chi. */
mera_status mera_ctx_set_verbose(mera_ctx* ctx, int level);

/* Layer dimensions: a_out[0..T], b_out[0..T] (host arrays of T+1 ints). */
mera_status mera_layer_dims(const mera_shape* shape, int* a_out, int* b_out);

/* ---- model -------------------------------------------------------------------------------------------- */

/* Three-site terms on blocked sites of two spins (d = 4), written to a HOST array of 64*64 doubles.
 * Sec. 4 (cost function): TFIM local term -X X - h Z; XXZ term X X + Y Y + delta Z Z in Pauli units.
 * Blocked site = spins (s1, s2), s1 major; hb = inter-block bond + half of each block's internal terms;
 * h3 = (hb (x) 1 + 1 (x) hb) / 2, so that the sum of h3 over a ring is the spin Hamiltonian. */
mera_status mera_h3_tfim(double h, double* h3_host);
mera_status mera_h3_xxz(double delta, double* h3_host);
/* Two-site terms on unblocked spins (d = 2) for the ternary geometry (Sec. 4): TFIM -X X - h (Z 1 + 1 Z)/2,
 * XXZ X X + Y Y + delta Z Z (Pauli units); summed over the bonds of a chain they give the chain Hamiltonian.
 * Output: 4 x 4 row-major host FP64, basis |s0 s1> with s0 the more significant bit. */
mera_status mera_h2_tfim(double h, double* h2_host);
mera_status mera_h2_xxz(double delta, double* h2_host);

/* ---- energy and Euclidean gradient (Sec. 4, App. B) --------------------------------------------------- */

/* Krylov warm starts kept between evaluations: the scale-invariant density matrix and the operator h~ of
 * the previous call (App. B: "the solution from the previous iteration as the initial guess"). */
mera_status mera_warm_create(mera_ctx* ctx, const mera_shape* shape, mera_warm** out);
void mera_warm_destroy(mera_warm* warm);

typedef struct {
  int krylov_dim;          /* Krylov subspace dimension per restart (App. B suggests 4); 0 -> 16, or    */
                           /* fewer (at least 4) to keep the basis within 16 GiB                       */
  int max_restarts;        /* per solve; 0 -> 200                                                      */
  double tol;              /* relative residual of both solves; 0 -> 1e-13 (FP64) or 1e-7 (FP32/BF16X3)  */
  int extrapolate;         /* with a warm-start object: > 0 (and 0, the default) starts both solves from the */
                           /* solutions of the last two evaluations extrapolated along this evaluation's    */
                           /* step (x1 + t (x1 - x2), t = <P - P1, P1 - P2> / |P1 - P2|^2 over the tensors */
                           /* P of the three points, clamped to [-1, 1]); < 0 starts them from the last    */
                           /* solution alone (App. B)                                                      */
} mera_krylov_opts;

typedef struct {
  double energy;           /* per blocked site, Tr[h_T rho_s]                                           */
  int applications_rho;    /* superoperator applications spent on the fixed point                       */
  int applications_htilde; /* ... on h~                                                                 */
  double residual_rho;     /* final relative residuals                                                  */
  double residual_htilde;
  double macs;             /* multiply-accumulates issued by this call                                  */
} mera_eval_info;

/*
 * mera_energy_grad — energy per blocked site and the Euclidean partial derivatives D_v of every tensor.
 *   Sec. 4 (cost C = <MERA|H|MERA>, D_v = environment of v summed over all its occurrences), App. B (scale-
 *   invariant density matrix as the fixed point of the descending map; derivative through the fixed point by
 *   the deflated series h~ = sum_i <h'|A'^i, A' = A - |rho><1|, h' = h_T - e 1, solved by a Krylov method).
 *   u[0..T], w[0..T]     tensors (device, FP64, see conventions), isometric.
 *   h3                   device FP64 symmetric local term: d^3 x d^3 (binary) or d^2 x d^2 (ternary).
 *   warm                 in/out warm starts, or NULL (then the solves start from 1/chi^k and h', k sites).
 *   energy               host double out.
 *   Du[0..T], Dw[0..T]   caller-allocated device outputs, same shapes as u, w. The scale-invariant D is fixed
 *                        in the gauge Tr[h~ rho_s] = 0 (terms along W S, S symmetric, are not determined).
 *   rho_u, rho_w         optional (NULL) device outputs: the reduced density matrices on the top legs of each
 *                        u (a^2 x a^2) and w (b x b) used by the Hilbert-space preconditioner (Sec. 4,
 *                        eq. mera_diagonal_inner_product).
 *   kopts, info          optional (NULL).
 */
mera_status mera_energy_grad(mera_ctx* ctx, const mera_shape* shape, const mera_mat* u, const mera_mat* w,
                             const double* h3, mera_prec prec, mera_warm* warm, const mera_krylov_opts* kopts,
                             double* energy, mera_mat* Du, mera_mat* Dw, mera_mat* rho_u, mera_mat* rho_w,
                             mera_eval_info* info);

/* Single superoperator applications, for tests and tools (App. B: <h|A raises, A|rho> lowers).
 * layer = 0..T; in/out are device operators of the layer's bottom (a^k x a^k) or top (b^k x b^k) sites, k = 3
 * for the binary and 2 for the ternary geometry. */
mera_status mera_ascend(mera_ctx* ctx, const mera_shape* shape, int layer, const mera_mat* u, const mera_mat* w,
                        mera_prec prec, const double* h_in, double* h_out);
mera_status mera_descend(mera_ctx* ctx, const mera_shape* shape, int layer, const mera_mat* u, const mera_mat* w,
                         mera_prec prec, const double* rho_in, double* rho_out);

/* Derivative of one layer's term Tr[A(h) rho] with h and rho held fixed, for tests and tools (Sec. 4,
 * eq. mera_derivative: the environment of every occurrence of u and w in the layer's diagrams, summed, with the
 * 1/2 (binary) or 1/3 (ternary) of the position average; App. B: the same networks give the descending map).
 *   layer            0..T.  h_in: device FP64 operator on the layer's bottom sites (a^k x a^k, k = 3 binary, 2
 *                    ternary), rho_in: on its top sites (b^k x b^k); both symmetric (the derivative programs use
 *                    the ket/bra symmetry of the network and are wrong for asymmetric operators).
 *   split            0: the combined forward-and-reverse programs (the scale-invariant layer's path in
 *                    mera_energy_grad); 1 (binary geometry only): the forward halves, which keep their
 *                    activations, then the reverse halves (the transition layers' path). Same results up to
 *                    rounding order.
 *   h_out            nullable device FP64 b^k x b^k output A(h); only with split = 1 (MERA_EINVAL otherwise).
 *   Du, Dw           caller-allocated device FP64 outputs, shapes of u and w.
 *   rho_out          nullable device FP64 a^k x a^k output D(rho).
 * Contractions in `prec`; inputs and outputs FP64. Synchronises the context stream. */
mera_status mera_layer_grad(mera_ctx* ctx, const mera_shape* shape, int layer, const mera_mat* u,
                            const mera_mat* w, mera_prec prec, int split, const double* h_in, const double* rho_in,
                            double* h_out, mera_mat* Du, mera_mat* Dw, double* rho_out);

/* ---- Stiefel manifold (Sec. 2) ------------------------------------------------------------------------ */
/* All take `count` matrices (a point of the product manifold, Sec. 2.4) and act factor by factor. count = 0 does
 * nothing and returns MERA_OK (the arrays may then be NULL). */

/* G = D - W (W^T D + D^T W) / 2 (eq. stiefel_gradient, real case). G may alias D. */
mera_status stiefel_project(mera_ctx* ctx, int count, const mera_mat* W, const mera_mat* D, mera_mat* G);
/* stiefel_project without any device allocation, for callers that cannot allocate: code under HIP graph capture,
 * serving loops and harnesses that forbid hipMalloc. Same arguments and result as stiefel_project (up to rounding
 * order). The p x p intermediate W^T D lives in a fixed file-scope device array of 2^20 doubles (8 MiB) per GPU,
 * held until the process ends: every factor must have p * p <= 2^20 (p <= 1024), at most 2097120 rows, and count
 * <= 64, else MERA_EINVAL. The call only launches kernels on the context stream and does not synchronise it (the
 * outputs are ready when the stream is). All calls on one GPU share that array: calls that overlap on one GPU
 * (other streams, other contexts, other threads) race and give wrong results. G may alias D, not W. */
mera_status stiefel_project_noalloc(mera_ctx* ctx, int count, const mera_mat* W, const mera_mat* D, mera_mat* G);
/* Polar retraction W_out = (W + alpha X)(I + alpha^2 X^T X)^{-1/2} computed as the polar factor of
 * Y = W + alpha X, with (Y^T Y)^{-1/2} by a coupled Newton-Schulz iteration in FP64 (retraction as defined in
 * Sec. 2.3; the polar form is this library's choice). X_out (nullable) receives dR/dalpha at alpha, the
 * curve tangent used in the Wolfe slope (Sec. 3). The factors are processed together and every W is read before
 * any output is written, so W_out may alias W; X is read again for X_out, so neither W_out nor X_out may alias
 * any X. */
mera_status stiefel_retract(mera_ctx* ctx, int count, const mera_mat* W, const mera_mat* X, double alpha,
                            mera_mat* W_out, mera_mat* X_out);
/* Vector transport by projection onto the tangent space at W_new. Y_out may alias Y. */
mera_status stiefel_transport(mera_ctx* ctx, int count, const mera_mat* W_new, const mera_mat* Y, mera_mat* Y_out);
/* The paper's exponential retraction (Sec. 2.3, eq. retraction): W_out = exp(alpha Q_X) W with
 * Q_X = [W W_perp] [[A, -B^T], [B, 0]] [W W_perp]^T, X = W A + W_perp B a tangent at W (Stiefel: A skew;
 * Grassmann: A = 0). Evaluated in low-rank form: W_perp B = (1 - W W^T) X is spanned by an orthonormal basis of
 * at most min(p, n - p) columns (from the FP64 Jacobi eigendecomposition of its Gram matrix), the (p + r)-square
 * exponential by scaling and squaring of a degree-14 Taylor polynomial on FP64 MFMA GEMMs; the result gets one
 * Newton-Schulz polar refinement. X_out (nullable) = exp(alpha Q_X) X = dW_out/dalpha. FP64 device buffers,
 * caller-owned; W_out must not alias W or X. MERA_ENONFINITE for a non-finite generator. */
mera_status stiefel_retract_exp(mera_ctx* ctx, int count, const mera_mat* W, const mera_mat* X, double alpha,
                                mera_mat* W_out, mera_mat* X_out);
/* The paper's vector transport (Sec. 2.3, eq. transport): Y_out = exp(alpha Q_X) Y for the retraction of W along
 * X by alpha; it preserves inner products. Y_out may alias Y. */
mera_status stiefel_transport_exp(mera_ctx* ctx, int count, const mera_mat* W, const mera_mat* X, double alpha,
                                  const mera_mat* Y, mera_mat* Y_out);
/* Evenbly-Vidal local update (App. A): W_out = polar(gamma W rho - D) = polar(-D_gamma), D the Euclidean derivative
 * (environment) of the energy with respect to W, rho its p x p reduced density matrix on the top legs, gamma > 0 the
 * shift of H - gamma. The polar factor is Y (Y^T Y)^{-1/2} from the FP64 Jacobi eigendecomposition, refined by one
 * Newton-Schulz step. MERA_ENONFINITE when gamma W rho - D is rank deficient. W_out must not alias W or D. */
mera_status mera_ev_update(mera_ctx* ctx, int count, const mera_mat* W, const mera_mat* D, const mera_mat* rho,
                           double gamma, mera_mat* W_out);
/* Grassmann tangent projection (Sec. 2.2, eq. grassmann_gradient, real case): G = (1 - W W^T) D. G may alias D. */
mera_status grassmann_project(mera_ctx* ctx, int count, const mera_mat* W, const mera_mat* D, mera_mat* G);
/* Hilbert-space preconditioner (Sec. 3 eqs. preconditioner / preconditioner_solution): X = W A + W_perp B
 * maps to W A~ + W_perp B~ with A~ f + f A~ = 2 A, B~ = B f^{-1}, f = (rho^2 + delta^2)^{1/2}; delta < 0 means
 * delta = ||X_v||_F per factor (Sec. 4). rho: count p x p symmetric PSD matrices. */
mera_status stiefel_precondition(mera_ctx* ctx, int count, const mera_mat* W, const mera_mat* X,
                                 const mera_mat* rho, double delta, mera_mat* X_out);
/* Euclidean metric summed over factors: sum_v Tr[X_v^T Y_v] (Sec. 2.2, 2.4). Host result. */
mera_status mera_inner(mera_ctx* ctx, int count, const mera_mat* X, const mera_mat* Y, double* out);

/* ---- L-BFGS (Sec. 3) ---------------------------------------------------------------------------------- */

/* History of up to m pairs for a product manifold with factors of sizes n[i] x p[i]. */
mera_status lbfgs_create(mera_ctx* ctx, int count, const int* n, const int* p, int m, mera_lbfgs** out);
void lbfgs_destroy(mera_lbfgs* lb);
mera_status lbfgs_reset(mera_lbfgs* lb);
int lbfgs_size(const mera_lbfgs* lb);
/* Two-loop recursion: dir_out = -H G with H0 = gamma P, P the preconditioner with rho (NULL: identity),
 * gamma = <s,y>/<y,P y> of the newest pair. slope_out (host) = <G, dir_out>. If the result is not a descent
 * direction the history is cleared and dir_out = -P G. The object keeps the eigenbases of the last rho: the next
 * call decomposes its rho in them (Q^T rho Q, a few Jacobi sweeps when rho changed little; every 32nd decomposition
 * of a factor starts from scratch), as the optimiser does between iterations. */
mera_status lbfgs_step(mera_ctx* ctx, mera_lbfgs* lb, const mera_mat* W, const mera_mat* G, const mera_mat* rho,
                       mera_mat* dir_out, double* slope_out);
/* After an accepted step W_new = R_W(d, alpha): transport the stored pairs to W_new, form
 * s = T(alpha d), y = G_new - T(G_old), store the pair if <s,y> > 1e-12 |s||y| (accepted = 1). */
mera_status lbfgs_push(mera_ctx* ctx, mera_lbfgs* lb, const mera_mat* W_new, const mera_mat* d, double alpha,
                       const mera_mat* G_old, const mera_mat* G_new, int* accepted);

/* ---- whole optimisation ------------------------------------------------------------------------------- */

typedef struct {
  mera_shape shape;
  const double* h3_host;           /* host FP64 local term, d^3 x d^3 (binary) or d^2 x d^2 (ternary)       */
  const double* const* init_host;  /* 2(T+1) host FP64 matrices: u_1, w_1, ..., u_T, w_T, u_s, w_s          */
  mera_prec prec;                  /* contraction arithmetic before polishing                               */
  int lbfgs_m;                     /* memory (8)                                                            */
  int max_iter;
  double grad_tol;                 /* stop at ||G|| <= grad_tol                                             */
  double polish_tol;               /* FP32/BF16X3 forms switch to FP64 below this ||G||, or when a line      */
                                   /* search fails in the reduced precision (0: never; a failed search then */
                                   /* ends the run with status 2)                                           */
  int precondition;                /* 1: Hilbert-space preconditioner as H0 (Sec. 3, Sec. 4)                */
  int max_ls_evals;                /* line-search evaluations per iteration (10)                            */
  mera_krylov_opts krylov;
  int method;                      /* 0: L-BFGS (Sec. 3); 1: nonlinear conjugate gradient with the           */
                                   /* preconditioned Hager-Zhang coefficient (Sec. 3), the previous         */
                                   /* direction carried over by the transport; lbfgs_m is then ignored;     */
                                   /* 2: Evenbly-Vidal sweeps (App. A), one iteration = one sweep updating   */
                                   /* u_1, w_1, ..., u_s, w_s in turn from fresh environments                */
  int retraction;                  /* 0: polar retraction + projection transport; 1: the paper's            */
                                   /* exponential retraction and transport (Sec. 2.3)                       */
  int grassmann_w;                 /* 1: isometries w on Grassmann manifolds (Sec. 4): Grassmann gradient    */
                                   /* projection and projection transport for the w factors                 */
  double ev_gamma;                 /* method 2: shift gamma of H - gamma (inverse step size, App. A), > 0    */
} mera_job;

typedef struct {
  double energy;                   /* per blocked site at the returned point                                */
  double gnorm;                    /* ||G|| of the unpreconditioned Riemannian gradient                      */
  int iterations;
  int evaluations;
  int status;                      /* 0 converged, 1 iteration cap, 2 line search failed, <0 mera_status      */
  int polish_iter;                 /* iteration at which FP64 polishing started, -1 if never                 */
  double seconds;                  /* wall time of the optimisation itself                                  */
  double macs;
  double queued_seconds;           /* server only: time from submission to admission (0 for run_optimize)   */
  int krylov_applications;         /* superoperator applications spent in the two Krylov solves, all evals  */
} mera_result;

typedef struct { int iter; int evals; double energy; double gnorm; double alpha; int prec; } mera_iter_log;

/* Step-wise optimisation: the same algorithm as run_optimize, one iteration per mera_opt_step call.
 * mera_opt_create copies the job, allocates the state on the context's device and evaluates the initial
 * point. mera_opt_step runs one iteration (its line-search evaluations and Stiefel steps); *done becomes 1
 * when the job has converged, hit its iteration cap or failed; `state` (nullable) receives the current
 * energy, ||G||, iteration and evaluation counts. mera_opt_final copies the current tensors to host buffers. */
typedef struct mera_opt mera_opt;
mera_status mera_opt_create(mera_ctx* ctx, const mera_job* job, mera_opt** out);
mera_status mera_opt_step(mera_ctx* ctx, mera_opt* opt, int* done, mera_result* state);
mera_status mera_opt_final(mera_ctx* ctx, mera_opt* opt, double* const* final_host);
void mera_opt_destroy(mera_opt* opt);

/* Blocking single-job optimisation (Sec. 3 L-BFGS with Wolfe / approximate-Wolfe line search on the product
 * of Stiefel manifolds, Sec. 4 MERA cost). final_host (nullable): 2(T+1) host buffers receiving the final
 * tensors. log (nullable): up to log_cap per-iteration records; *log_len (nullable) receives the count. */
mera_status run_optimize(mera_ctx* ctx, const mera_job* job, mera_result* out, double* const* final_host,
                         mera_iter_log* log, int log_cap, int* log_len);

/* ---- serving: continuous batching of optimisation jobs ------------------------------------------------ */

/* A server owns `max_slots` host workers, each with its own HIP stream and workspace on the context's
 * device. Submitted jobs wait in a FIFO queue; the head job is admitted when a worker is free and the summed
 * device-memory footprint of the running jobs plus its own fits `hbm_budget` bytes; the device work of the
 * running jobs overlaps. Contraction programs (ascending / descending maps, gradient networks) that
 * concurrent jobs reach at the same extents are run as one sequence of grouped MFMA launches (up to 8 jobs per
 * launch), and a sequence seen before on the same buffers is replayed from a captured HIP graph. A job
 * computes exactly what run_optimize computes for it alone (same kernels, tiles and reduction order).
 * Destroying the server waits for running jobs and drops queued ones. The server also holds the offset
 * tables of every contraction shape it has run (shared by its workers) until it is destroyed. */
mera_status mera_server_create(mera_ctx* ctx, size_t hbm_budget, int max_slots, mera_server** out);
/* Batching options, before the first submit (MERA_EBUSY afterwards): group_launches != 0 groups the same
 * program across jobs (default on); graph_capture != 0 replays repeated sequences from HIP graphs (default
 * on); max_wait_us >= 0 bounds how long a job waits for others of its shape to reach the same program; a
 * negative value (the default) bounds the wait by a tenth of the program's estimated run time (its multiply-adds
 * at 50e12 per second plus 10 us per kernel launch), at most 2000 us. NaN: MERA_EINVAL. With both options off
 * every job launches its own kernels on its own stream. */
mera_status mera_server_configure(mera_server* srv, int group_launches, int graph_capture, double max_wait_us);
typedef struct {
  int64_t batches;          /* program runs (grouped or not) */
  int64_t grouped_batches;  /* runs that carried more than one job */
  int64_t bindings;         /* job-programs executed (sum of group sizes) */
  int64_t graph_launches;   /* runs replayed from a captured graph */
  int64_t graph_captures;   /* graphs captured */
  int64_t eager_runs;       /* runs launched kernel by kernel */
} mera_server_stats;
/* Counters since creation. */
mera_status mera_server_get_stats(mera_server* srv, mera_server_stats* out);
/* The job is copied (including h3 and initial tensors) before the call returns. */
mera_status mera_server_submit(mera_server* srv, const mera_job* job, uint64_t* job_id);
/* MERA_EBUSY while queued or running; MERA_OK with the result once finished (or the job's error status,
 * with out->status set to it). Time to converged = queued_seconds + seconds. */
mera_status mera_server_poll(mera_server* srv, uint64_t job_id, mera_result* out);
/* Device bytes a job of this shape and precision needs (admission estimate, default Krylov dimension). The server
 * admits a job with polish_tol > 0 at its FP64 size, which it reaches once polishing starts. */
size_t mera_job_footprint(const mera_shape* shape, mera_prec prec);
void mera_server_destroy(mera_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* MERA_H */
