// extern "C" boundary: argument validation, device selection, exception -> status translation.
#include <cmath>
#include <cstring>

#include "common.h"
#include "mera_eval.h"
#include "model.h"
#include "network.h"

namespace mera {
// noalloc.hip
int64_t noalloc_scratch_doubles();
double* noalloc_scratch(int device);
void stiefel_project_noalloc_run(double* S, hipStream_t stream, int count, const int* n, const int* p,
                                 const double* const* W, const double* const* D, double* const* G);
}  // namespace mera


namespace mera {

Ctx::Ctx() : plans(new PlanCache) {}
Ctx::~Ctx() {
  for (auto& r : records) {
    event_pool.push_back(r.start);
    event_pool.push_back(r.stop);
  }
  for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
}

}  // namespace mera

struct mera_ctx {
  mera::Ctx c;
};
struct mera_warm {
  mera::Warm w;
  int device = 0;
};

using namespace mera;

namespace {

template <typename F>
mera_status guarded(mera_ctx* ctx, F&& f) {
  try {
    f();
    return MERA_OK;
  } catch (const Error& e) {
    if (ctx) ctx->c.last_error = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->c.last_error = "host allocation failed";
    return MERA_ENOMEM;
  } catch (const std::exception& e) {
    if (ctx) ctx->c.last_error = e.what();
    return MERA_EINVAL;
  }
}

void check_mats(const mera_mat* m, int count, const char* what) {
  MERA_CHECK(count == 0 || m != nullptr, MERA_EINVAL, std::string(what) + ": null matrix array");
  for (int i = 0; i < count; ++i)
    MERA_CHECK(m[i].data != nullptr && m[i].n > 0 && m[i].p > 0, MERA_EINVAL,
               std::string(what) + ": bad matrix " + std::to_string(i));
}

void check_layer_mats(const mera_shape& s, const mera_mat* u, const mera_mat* w, const char* what) {
  auto dims = layer_dims(s);
  check_mats(u, s.T + 1, what);
  check_mats(w, s.T + 1, what);
  for (int t = 0; t <= s.T; ++t) {
    const int a2 = dims[t].a * dims[t].a;
    const int wn = (int)dims[t].wrows();
    MERA_CHECK(u[t].n == a2 && u[t].p == a2, MERA_EINVAL,
               std::string(what) + ": u[" + std::to_string(t) + "] must be " + std::to_string(a2) + "x" +
                   std::to_string(a2));
    MERA_CHECK(w[t].n == wn && w[t].p == dims[t].b, MERA_EINVAL,
               std::string(what) + ": w[" + std::to_string(t) + "] must be " + std::to_string(wn) + "x" +
                   std::to_string(dims[t].b));
  }
}

Prec to_prec(mera_prec p) {
  MERA_CHECK(p == MERA_FP64 || p == MERA_FP32 || p == MERA_BF16X3, MERA_EINVAL, "unknown precision");
  return p == MERA_FP64 ? Prec::F64 : (p == MERA_FP32 ? Prec::F32 : Prec::BF16X3);
}

}  // namespace

extern "C" {

mera_status mera_ctx_create(int device, void* hip_stream, mera_ctx** out) {
  if (!out) return MERA_EINVAL;
  *out = nullptr;
  mera_ctx* c = nullptr;
  try {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return MERA_EINVAL;
    c = new mera_ctx;
    c->c.device = device;
    c->c.stream = static_cast<hipStream_t>(hip_stream);
    DeviceGuard g(device);
    (void)noalloc_scratch(device);  // this device's copy of the allocation-free entry point's scratch array
    *out = c;
    return MERA_OK;
  } catch (...) {
    delete c;
    return MERA_EHIP;
  }
}

void mera_ctx_destroy(mera_ctx* ctx) {
  if (!ctx) return;
  try {
    DeviceGuard g(ctx->c.device);
    (void)hipStreamSynchronize(ctx->c.stream);
    delete ctx;
  } catch (...) {
  }
}

const char* mera_last_error(const mera_ctx* ctx) { return ctx ? ctx->c.last_error.c_str() : "null context"; }

mera_status mera_ctx_trim(mera_ctx* ctx) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    DeviceGuard g(ctx->c.device);
    ctx->c.sync();
    ctx->c.scratch.clear();
    std::lock_guard<std::mutex> lock(ctx->c.plans->mu);
    ctx->c.plans->map.clear();
  });
}

double mera_ctx_macs(const mera_ctx* ctx) { return ctx ? ctx->c.macs : 0.0; }

mera_status mera_ctx_set_verbose(mera_ctx* ctx, int level) {
  if (!ctx) return MERA_EINVAL;
  ctx->c.verbose = level;
  return MERA_OK;
}

mera_status mera_ctx_set_intermediate_limit(mera_ctx* ctx, size_t bytes) {
  if (!ctx || bytes == 0) return MERA_EINVAL;
  ctx->c.inter_limit = bytes;
  return MERA_OK;
}

mera_status mera_layer_dims(const mera_shape* shape, int* a_out, int* b_out) {
  if (!shape || !a_out || !b_out) return MERA_EINVAL;
  try {
    auto d = layer_dims(*shape);
    for (size_t i = 0; i < d.size(); ++i) {
      a_out[i] = d[i].a;
      b_out[i] = d[i].b;
    }
    return MERA_OK;
  } catch (const Error& e) {
    return e.status;
  }
}

mera_status mera_h3_tfim(double h, double* h3_host) {
  if (!h3_host || !std::isfinite(h)) return MERA_EINVAL;
  build_h3_tfim(h, h3_host);
  return MERA_OK;
}

mera_status mera_h3_xxz(double delta, double* h3_host) {
  if (!h3_host || !std::isfinite(delta)) return MERA_EINVAL;
  build_h3_xxz(delta, h3_host);
  return MERA_OK;
}

mera_status mera_h2_tfim(double h, double* h2_host) {
  if (!h2_host || !std::isfinite(h)) return MERA_EINVAL;
  build_h2_tfim(h, h2_host);
  return MERA_OK;
}

mera_status mera_h2_xxz(double delta, double* h2_host) {
  if (!h2_host || !std::isfinite(delta)) return MERA_EINVAL;
  build_h2_xxz(delta, h2_host);
  return MERA_OK;
}

mera_status mera_warm_create(mera_ctx* ctx, const mera_shape* shape, mera_warm** out) {
  if (!ctx || !shape || !out) return MERA_EINVAL;
  return guarded(ctx, [&] {
    (void)layer_dims(*shape);
    auto* w = new mera_warm;
    w->device = ctx->c.device;
    w->w.chi = shape->chi;
    *out = w;
  });
}

void mera_warm_destroy(mera_warm* warm) {
  if (!warm) return;
  try {
    DeviceGuard g(warm->device);
    delete warm;
  } catch (...) {
  }
}

mera_status mera_energy_grad(mera_ctx* ctx, const mera_shape* shape, const mera_mat* u, const mera_mat* w,
                             const double* h3, mera_prec prec, mera_warm* warm, const mera_krylov_opts* kopts,
                             double* energy, mera_mat* Du, mera_mat* Dw, mera_mat* rho_u, mera_mat* rho_w,
                             mera_eval_info* info) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(shape && h3 && energy, MERA_EINVAL, "null argument");
    DeviceGuard g(ctx->c.device);
    check_layer_mats(*shape, u, w, "mera_energy_grad input");
    check_layer_mats(*shape, Du, Dw, "mera_energy_grad output");
    Point pt;
    GradOut go;
    auto dims = layer_dims(*shape);
    for (int t = 0; t <= shape->T; ++t) {
      pt.u.push_back(u[t].data);
      pt.w.push_back(w[t].data);
      go.Du.push_back(Du[t].data);
      go.Dw.push_back(Dw[t].data);
    }
    if (rho_u || rho_w) {
      MERA_CHECK(rho_u && rho_w, MERA_EINVAL, "rho_u and rho_w must both be given");
      for (int t = 0; t <= shape->T; ++t) {
        const int a2 = dims[t].a * dims[t].a;
        MERA_CHECK(rho_u[t].data && rho_u[t].n == a2 && rho_u[t].p == a2, MERA_EINVAL, "rho_u shape");
        MERA_CHECK(rho_w[t].data && rho_w[t].n == dims[t].b && rho_w[t].p == dims[t].b, MERA_EINVAL,
                   "rho_w shape");
        go.rho_u.push_back(rho_u[t].data);
        go.rho_w.push_back(rho_w[t].data);
      }
    }
    KrylovOpts ko;
    if (kopts) {
      if (kopts->krylov_dim > 0) ko.dim = kopts->krylov_dim;
      if (kopts->extrapolate != 0) ko.extrapolate = kopts->extrapolate > 0;
      if (kopts->max_restarts > 0) ko.max_restarts = kopts->max_restarts;
      if (kopts->tol > 0) ko.tol = kopts->tol;
    }
    MERA_CHECK(!warm || warm->device == ctx->c.device, MERA_EINVAL, "warm start from another device");
    EvalOut r = mera::energy_grad(ctx->c, *shape, pt, h3, to_prec(prec), warm ? &warm->w : nullptr, ko, go);
    *energy = r.energy;
    if (info) {
      info->energy = r.energy;
      info->applications_rho = r.app_rho;
      info->applications_htilde = r.app_ht;
      info->residual_rho = r.res_rho;
      info->residual_htilde = r.res_ht;
      info->macs = r.macs;
    }
    ctx->c.sync();
  });
}

mera_status mera_ascend(mera_ctx* ctx, const mera_shape* shape, int layer, const mera_mat* u, const mera_mat* w,
                        mera_prec prec, const double* h_in, double* h_out) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(shape && u && w && h_in && h_out, MERA_EINVAL, "null argument");
    auto dims = layer_dims(*shape);
    MERA_CHECK(layer >= 0 && layer <= shape->T, MERA_EINVAL, "layer out of range");
    const int a2 = dims[layer].a * dims[layer].a;
    MERA_CHECK(u->data && u->n == a2 && u->p == a2 && w->data && w->n == (int)dims[layer].wrows() &&
                   w->p == dims[layer].b,
               MERA_EINVAL, "tensor shape");
    DeviceGuard g(ctx->c.device);
    ascend_op(ctx->c, dims[layer], u->data, w->data, to_prec(prec), h_in, h_out);
    ctx->c.sync();
  });
}

mera_status mera_descend(mera_ctx* ctx, const mera_shape* shape, int layer, const mera_mat* u, const mera_mat* w,
                         mera_prec prec, const double* rho_in, double* rho_out) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(shape && u && w && rho_in && rho_out, MERA_EINVAL, "null argument");
    auto dims = layer_dims(*shape);
    MERA_CHECK(layer >= 0 && layer <= shape->T, MERA_EINVAL, "layer out of range");
    const int a2 = dims[layer].a * dims[layer].a;
    MERA_CHECK(u->data && u->n == a2 && u->p == a2 && w->data && w->n == (int)dims[layer].wrows() &&
                   w->p == dims[layer].b,
               MERA_EINVAL, "tensor shape");
    DeviceGuard g(ctx->c.device);
    descend_op(ctx->c, dims[layer], u->data, w->data, to_prec(prec), rho_in, rho_out);
    ctx->c.sync();
  });
}

mera_status mera_layer_grad(mera_ctx* ctx, const mera_shape* shape, int layer, const mera_mat* u,
                            const mera_mat* w, mera_prec prec, int split, const double* h_in, const double* rho_in,
                            double* h_out, mera_mat* Du, mera_mat* Dw, double* rho_out) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(shape && u && w && h_in && rho_in && Du && Dw, MERA_EINVAL, "null argument");
    auto dims = layer_dims(*shape);
    MERA_CHECK(layer >= 0 && layer <= shape->T, MERA_EINVAL, "layer out of range");
    const LayerDim& L = dims[layer];
    const int a2 = L.a * L.a;
    MERA_CHECK(u->data && u->n == a2 && u->p == a2 && w->data && w->n == (int)L.wrows() && w->p == L.b,
               MERA_EINVAL, "tensor shape");
    MERA_CHECK(Du->data && Du->n == a2 && Du->p == a2 && Dw->data && Dw->n == (int)L.wrows() && Dw->p == L.b,
               MERA_EINVAL, "gradient shape");
    DeviceGuard g(ctx->c.device);
    layer_grad_op(ctx->c, L, u->data, w->data, to_prec(prec), split != 0, h_in, rho_in, h_out, Du->data,
                  Dw->data, rho_out);
    ctx->c.sync();
  });
}

}  // extern "C"

// ---- Stiefel manifold, L-BFGS, optimiser ---------------------------------------------------------------

#include "optim.h"

struct mera_lbfgs {
  mera::Lbfgs lb;
  mera::Metric met;  // eigenbases of the last preconditioner density matrices (warm starts for the next step)
  int device = 0;
};

namespace mera {
int ctx_device_of(const mera_ctx* ctx) { return ctx->c.device; }
}  // namespace mera

namespace {

std::vector<MatView> views(const mera_mat* m, int count) {
  std::vector<MatView> v;
  for (int i = 0; i < count; ++i) v.push_back(MatView{m[i].n, m[i].p, m[i].data});
  return v;
}

void same_shapes(const mera_mat* a, const mera_mat* b, int count, const char* what) {
  for (int i = 0; i < count; ++i)
    MERA_CHECK(a[i].n == b[i].n && a[i].p == b[i].p, MERA_EINVAL, std::string(what) + ": shape mismatch");
}

void check_isometry_shapes(const mera_mat* W, int count, const char* what) {
  check_mats(W, count, what);
  for (int i = 0; i < count; ++i)
    MERA_CHECK(W[i].n >= W[i].p, MERA_EINVAL, std::string(what) + ": need n >= p");
}

}  // namespace

extern "C" {

mera_status stiefel_project(mera_ctx* ctx, int count, const mera_mat* W, const mera_mat* D, mera_mat* G) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(count >= 0, MERA_EINVAL, "count");
    check_isometry_shapes(W, count, "stiefel_project W");
    check_mats(D, count, "stiefel_project D");
    check_mats(G, count, "stiefel_project G");
    same_shapes(W, D, count, "stiefel_project");
    same_shapes(W, G, count, "stiefel_project");
    DeviceGuard g(ctx->c.device);
    for (int i = 0; i < count; ++i)
      stiefel_project_one(ctx->c, MatView{W[i].n, W[i].p, W[i].data}, MatView{D[i].n, D[i].p, D[i].data},
                          MatView{G[i].n, G[i].p, G[i].data});
    ctx->c.sync();
  });
}

mera_status stiefel_project_noalloc(mera_ctx* ctx, int count, const mera_mat* W, const mera_mat* D, mera_mat* G) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(count >= 0, MERA_EINVAL, "count");
    check_isometry_shapes(W, count, "stiefel_project_noalloc W");
    check_mats(D, count, "stiefel_project_noalloc D");
    check_mats(G, count, "stiefel_project_noalloc G");
    same_shapes(W, D, count, "stiefel_project_noalloc");
    same_shapes(W, G, count, "stiefel_project_noalloc");
    constexpr int kMaxFactors = 64;
    MERA_CHECK(count <= kMaxFactors, MERA_EINVAL, "stiefel_project_noalloc: more than 64 factors in one call");
    int n[kMaxFactors], p[kMaxFactors];
    const double* Wp[kMaxFactors];
    const double* Dp[kMaxFactors];
    double* Gp[kMaxFactors];
    for (int i = 0; i < count; ++i) {
      MERA_CHECK((int64_t)W[i].p * W[i].p <= noalloc_scratch_doubles(), MERA_EINVAL,
                 "stiefel_project_noalloc: factor " + std::to_string(i) + " has p = " + std::to_string(W[i].p) +
                     "; p * p must fit the fixed scratch of " + std::to_string(noalloc_scratch_doubles()) +
                     " doubles (p <= 1024)");
      MERA_CHECK(W[i].n <= 65535 * 32, MERA_EINVAL, "stiefel_project_noalloc: more than 2097120 rows");
      MERA_CHECK(G[i].data != W[i].data, MERA_EINVAL, "stiefel_project_noalloc: G aliases W");
      n[i] = W[i].n;
      p[i] = W[i].p;
      Wp[i] = W[i].data;
      Dp[i] = D[i].data;
      Gp[i] = G[i].data;
    }
    if (count == 0) return;
    DeviceGuard g(ctx->c.device);
    stiefel_project_noalloc_run(noalloc_scratch(ctx->c.device), ctx->c.stream, count, n, p, Wp, Dp, Gp);
  });
}

mera_status stiefel_retract(mera_ctx* ctx, int count, const mera_mat* W, const mera_mat* X, double alpha,
                            mera_mat* W_out, mera_mat* X_out) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(count >= 0 && std::isfinite(alpha), MERA_EINVAL, "count/alpha");
    check_isometry_shapes(W, count, "stiefel_retract W");
    check_mats(X, count, "stiefel_retract X");
    check_mats(W_out, count, "stiefel_retract W_out");
    same_shapes(W, X, count, "stiefel_retract");
    same_shapes(W, W_out, count, "stiefel_retract");
    if (X_out) {
      check_mats(X_out, count, "stiefel_retract X_out");
      same_shapes(W, X_out, count, "stiefel_retract");
    }
    DeviceGuard g(ctx->c.device);
    std::vector<MatView> wv(count), xv(count), wo(count), xo(count);
    std::vector<const MatView*> xop(count, nullptr);
    for (int i = 0; i < count; ++i) {
      wv[i] = MatView{W[i].n, W[i].p, W[i].data};
      xv[i] = MatView{X[i].n, X[i].p, X[i].data};
      wo[i] = MatView{W_out[i].n, W_out[i].p, W_out[i].data};
      if (X_out) {
        xo[i] = MatView{X_out[i].n, X_out[i].p, X_out[i].data};
        xop[i] = &xo[i];
      }
    }
    if (count > 0) stiefel_retract_many(ctx->c, wv, xv, alpha, wo, xop);
    ctx->c.sync();
  });
}

mera_status stiefel_transport(mera_ctx* ctx, int count, const mera_mat* W_new, const mera_mat* Y, mera_mat* Y_out) {
  return stiefel_project(ctx, count, W_new, Y, Y_out);
}

mera_status stiefel_retract_exp(mera_ctx* ctx, int count, const mera_mat* W, const mera_mat* X, double alpha,
                                mera_mat* W_out, mera_mat* X_out) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(count >= 0 && std::isfinite(alpha), MERA_EINVAL, "count/alpha");
    check_isometry_shapes(W, count, "stiefel_retract_exp W");
    check_mats(X, count, "stiefel_retract_exp X");
    check_mats(W_out, count, "stiefel_retract_exp W_out");
    same_shapes(W, X, count, "stiefel_retract_exp");
    same_shapes(W, W_out, count, "stiefel_retract_exp");
    if (X_out) {
      check_mats(X_out, count, "stiefel_retract_exp X_out");
      same_shapes(W, X_out, count, "stiefel_retract_exp");
    }
    for (int i = 0; i < count; ++i)
      MERA_CHECK(W_out[i].data != W[i].data && W_out[i].data != X[i].data, MERA_EINVAL,
                 "stiefel_retract_exp: W_out aliases an input");
    DeviceGuard g(ctx->c.device);
    ExpFrame fr;
    for (int i = 0; i < count; ++i) {
      const MatView Wv{W[i].n, W[i].p, W[i].data}, Xv{X[i].n, X[i].p, X[i].data};
      exp_frame_one(ctx->c, Wv, Xv, fr);
      MatView xo = X_out ? MatView{X_out[i].n, X_out[i].p, X_out[i].data} : MatView{};
      exp_retract_one(ctx->c, Wv, Xv, fr, alpha, MatView{W_out[i].n, W_out[i].p, W_out[i].data},
                      X_out ? &xo : nullptr);
    }
    ctx->c.sync();
  });
}

mera_status stiefel_transport_exp(mera_ctx* ctx, int count, const mera_mat* W, const mera_mat* X, double alpha,
                                  const mera_mat* Y, mera_mat* Y_out) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(count >= 0 && std::isfinite(alpha), MERA_EINVAL, "count/alpha");
    check_isometry_shapes(W, count, "stiefel_transport_exp W");
    for (const mera_mat* M : {X, Y, static_cast<const mera_mat*>(Y_out)}) {
      check_mats(M, count, "stiefel_transport_exp");
      same_shapes(W, M, count, "stiefel_transport_exp");
    }
    DeviceGuard g(ctx->c.device);
    ExpFrame fr;
    for (int i = 0; i < count; ++i) {
      const MatView Wv{W[i].n, W[i].p, W[i].data};
      exp_frame_one(ctx->c, Wv, MatView{X[i].n, X[i].p, X[i].data}, fr);
      exp_set_alpha(ctx->c, fr, alpha);
      exp_apply_one(ctx->c, Wv, fr, MatView{Y[i].n, Y[i].p, Y[i].data}, MatView{Y_out[i].n, Y_out[i].p, Y_out[i].data});
    }
    ctx->c.sync();
  });
}

mera_status mera_ev_update(mera_ctx* ctx, int count, const mera_mat* W, const mera_mat* D, const mera_mat* rho,
                           double gamma, mera_mat* W_out) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(count >= 0 && std::isfinite(gamma) && gamma > 0.0, MERA_EINVAL, "count/gamma");
    check_isometry_shapes(W, count, "mera_ev_update W");
    check_mats(D, count, "mera_ev_update D");
    check_mats(rho, count, "mera_ev_update rho");
    check_mats(W_out, count, "mera_ev_update W_out");
    same_shapes(W, D, count, "mera_ev_update");
    same_shapes(W, W_out, count, "mera_ev_update");
    for (int i = 0; i < count; ++i) {
      MERA_CHECK(rho[i].n == W[i].p && rho[i].p == W[i].p, MERA_EINVAL, "rho must be p x p");
      MERA_CHECK(W_out[i].data != W[i].data && W_out[i].data != D[i].data, MERA_EINVAL,
                 "mera_ev_update: W_out aliases an input");
    }
    DeviceGuard g(ctx->c.device);
    for (int i = 0; i < count; ++i)
      ev_update_one(ctx->c, MatView{W[i].n, W[i].p, W[i].data}, MatView{D[i].n, D[i].p, D[i].data},
                    MatView{rho[i].n, rho[i].p, rho[i].data}, gamma, MatView{W_out[i].n, W_out[i].p, W_out[i].data});
    ctx->c.sync();
  });
}

mera_status grassmann_project(mera_ctx* ctx, int count, const mera_mat* W, const mera_mat* D, mera_mat* G) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(count >= 0, MERA_EINVAL, "count");
    check_isometry_shapes(W, count, "grassmann_project W");
    check_mats(D, count, "grassmann_project D");
    check_mats(G, count, "grassmann_project G");
    same_shapes(W, D, count, "grassmann_project");
    same_shapes(W, G, count, "grassmann_project");
    DeviceGuard g(ctx->c.device);
    for (int i = 0; i < count; ++i)
      grassmann_project_one(ctx->c, MatView{W[i].n, W[i].p, W[i].data}, MatView{D[i].n, D[i].p, D[i].data},
                            MatView{G[i].n, G[i].p, G[i].data});
    ctx->c.sync();
  });
}

mera_status stiefel_precondition(mera_ctx* ctx, int count, const mera_mat* W, const mera_mat* X,
                                 const mera_mat* rho, double delta, mera_mat* X_out) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(count >= 0 && std::isfinite(delta), MERA_EINVAL, "count/delta");
    check_isometry_shapes(W, count, "stiefel_precondition W");
    check_mats(X, count, "stiefel_precondition X");
    check_mats(rho, count, "stiefel_precondition rho");
    check_mats(X_out, count, "stiefel_precondition X_out");
    same_shapes(W, X, count, "stiefel_precondition");
    same_shapes(W, X_out, count, "stiefel_precondition");
    for (int i = 0; i < count; ++i)
      MERA_CHECK(rho[i].n == W[i].p && rho[i].p == W[i].p, MERA_EINVAL, "rho must be p x p");
    DeviceGuard g(ctx->c.device);
    Metric met;
    met.compute(ctx->c, views(rho, count));
    for (int i = 0; i < count; ++i)
      precondition_one(ctx->c, MatView{W[i].n, W[i].p, W[i].data}, MatView{X[i].n, X[i].p, X[i].data}, met, i,
                       delta, MatView{X_out[i].n, X_out[i].p, X_out[i].data});
    ctx->c.sync();
  });
}

mera_status mera_inner(mera_ctx* ctx, int count, const mera_mat* X, const mera_mat* Y, double* out) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(out && count >= 0, MERA_EINVAL, "null output");
    check_mats(X, count, "mera_inner X");
    check_mats(Y, count, "mera_inner Y");
    same_shapes(X, Y, count, "mera_inner");
    DeviceGuard g(ctx->c.device);
    *out = inner(ctx->c, views(X, count), views(Y, count));
  });
}

mera_status lbfgs_create(mera_ctx* ctx, int count, const int* n, const int* p, int m, mera_lbfgs** out) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(out && n && p && count > 0 && m >= 0, MERA_EINVAL, "lbfgs_create arguments");
    for (int i = 0; i < count; ++i) MERA_CHECK(n[i] > 0 && p[i] > 0, MERA_EINVAL, "lbfgs_create sizes");
    DeviceGuard g(ctx->c.device);
    auto* lb = new mera_lbfgs;
    lb->device = ctx->c.device;
    try {
      lb->lb.init(ctx->c, std::vector<int>(n, n + count), std::vector<int>(p, p + count), m);
    } catch (...) {
      delete lb;
      throw;
    }
    *out = lb;
  });
}

void lbfgs_destroy(mera_lbfgs* lb) {
  if (!lb) return;
  try {
    DeviceGuard g(lb->device);
    delete lb;
  } catch (...) {
  }
}

mera_status lbfgs_reset(mera_lbfgs* lb) {
  if (!lb) return MERA_EINVAL;
  lb->lb.reset();
  return MERA_OK;
}

int lbfgs_size(const mera_lbfgs* lb) { return lb ? lb->lb.size() : 0; }

mera_status lbfgs_step(mera_ctx* ctx, mera_lbfgs* lb, const mera_mat* W, const mera_mat* G, const mera_mat* rho,
                       mera_mat* dir_out, double* slope_out) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(lb && slope_out && lb->device == ctx->c.device, MERA_EINVAL, "lbfgs_step arguments");
    const int count = lb->lb.shape.count();
    check_mats(W, count, "lbfgs_step W");
    check_mats(G, count, "lbfgs_step G");
    check_mats(dir_out, count, "lbfgs_step dir_out");
    for (int i = 0; i < count; ++i)
      MERA_CHECK(W[i].n == lb->lb.shape.n[i] && W[i].p == lb->lb.shape.p[i], MERA_EINVAL, "lbfgs_step shape");
    same_shapes(W, G, count, "lbfgs_step");
    same_shapes(W, dir_out, count, "lbfgs_step");
    DeviceGuard g(ctx->c.device);
    if (rho) {
      check_mats(rho, count, "lbfgs_step rho");
      for (int i = 0; i < count; ++i)
        MERA_CHECK(rho[i].n == W[i].p && rho[i].p == W[i].p, MERA_EINVAL, "rho must be p x p");
      lb->met.compute(ctx->c, views(rho, count));
    }
    *slope_out = lb->lb.step(ctx->c, views(W, count), views(G, count), rho ? &lb->met : nullptr,
                             views(dir_out, count));
    ctx->c.sync();
  });
}

mera_status lbfgs_push(mera_ctx* ctx, mera_lbfgs* lb, const mera_mat* W_new, const mera_mat* d, double alpha,
                       const mera_mat* G_old, const mera_mat* G_new, int* accepted) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(lb && lb->device == ctx->c.device && std::isfinite(alpha), MERA_EINVAL, "lbfgs_push arguments");
    const int count = lb->lb.shape.count();
    for (const mera_mat* M : {W_new, d, G_old, G_new}) {
      check_mats(M, count, "lbfgs_push");
      for (int i = 0; i < count; ++i)
        MERA_CHECK(M[i].n == lb->lb.shape.n[i] && M[i].p == lb->lb.shape.p[i], MERA_EINVAL, "lbfgs_push shape");
    }
    DeviceGuard g(ctx->c.device);
    bool ok = lb->lb.push(ctx->c, views(W_new, count), views(d, count), alpha, views(G_old, count),
                          views(G_new, count));
    if (accepted) *accepted = ok ? 1 : 0;
    ctx->c.sync();
  });
}

mera_status run_optimize(mera_ctx* ctx, const mera_job* job, mera_result* out, double* const* final_host,
                         mera_iter_log* log, int log_cap, int* log_len) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(job && out, MERA_EINVAL, "null argument");
    MERA_CHECK(log_cap >= 0 && (log_cap == 0 || log), MERA_EINVAL, "log buffer");
    JobSpec spec = JobSpec::from_c(*job);
    DeviceGuard g(ctx->c.device);
    std::vector<double*> fin;
    if (final_host)
      for (int i = 0; i < 2 * (spec.shape.T + 1); ++i) fin.push_back(final_host[i]);
    OptResult r = optimize(ctx->c, spec, final_host ? &fin : nullptr, log_cap);
    std::memset(out, 0, sizeof(*out));
    out->energy = r.energy;
    out->gnorm = r.gnorm;
    out->iterations = r.iterations;
    out->evaluations = r.evaluations;
    out->status = r.status;
    out->polish_iter = r.polish_iter;
    out->seconds = r.seconds;
    out->macs = r.macs;
    out->krylov_applications = r.krylov_apps;
    for (size_t i = 0; i < r.log.size() && (int)i < log_cap; ++i) log[i] = r.log[i];
    if (log_len) *log_len = (int)std::min<size_t>(r.log.size(), (size_t)log_cap);
  });
}

}  // extern "C"

// ---- profiling and step-wise optimisation ----------------------------------------------------------------

#include <algorithm>
#include <chrono>

struct mera_opt {
  mera::Optimizer o;
  int device = 0;
  mera_ctx* owner = nullptr;
};

extern "C" {

mera_status mera_ctx_profile(mera_ctx* ctx, int enable) {
  if (!ctx) return MERA_EINVAL;
  ctx->c.profiling = enable != 0;
  return MERA_OK;
}

int mera_ctx_kernel_stats(mera_ctx* ctx, mera_kernel_stat* out, int cap) {
  if (!ctx || cap < 0 || (cap > 0 && !out)) return MERA_EINVAL;
  try {
    DeviceGuard g(ctx->c.device);
    ctx->c.sync();
    struct Agg {
      int n = 0;
      double s = 0, f = 0, b = 0;
    };
    std::map<std::string, Agg> agg;
    for (auto& r : ctx->c.records) {
      float ms = 0.f;
      MERA_HIP(hipEventElapsedTime(&ms, r.start, r.stop));
      Agg& a = agg[r.kernel];
      a.n++;
      a.s += ms * 1e-3;
      a.f += r.flops;
      a.b += r.bytes;
      ctx->c.event_pool.push_back(r.start);
      ctx->c.event_pool.push_back(r.stop);
    }
    ctx->c.records.clear();
    std::vector<std::pair<std::string, Agg>> v(agg.begin(), agg.end());
    std::sort(v.begin(), v.end(), [](auto& a, auto& b) { return a.second.s > b.second.s; });
    for (int i = 0; i < (int)v.size() && i < cap; ++i) {
      std::memset(&out[i], 0, sizeof(out[i]));
      std::strncpy(out[i].kernel, v[i].first.c_str(), sizeof(out[i].kernel) - 1);
      out[i].launches = v[i].second.n;
      out[i].seconds = v[i].second.s;
      out[i].flops = v[i].second.f;
      out[i].bytes = v[i].second.b;
    }
    return (int)v.size();
  } catch (const Error& e) {
    ctx->c.last_error = e.what();
    return e.status;
  }
}

mera_status mera_opt_create(mera_ctx* ctx, const mera_job* job, mera_opt** out) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(job && out, MERA_EINVAL, "null argument");
    JobSpec spec = JobSpec::from_c(*job);
    DeviceGuard g(ctx->c.device);
    auto* o = new mera_opt;
    o->device = ctx->c.device;
    o->owner = ctx;
    try {
      o->o.start(ctx->c, spec, 0);
    } catch (...) {
      delete o;
      throw;
    }
    *out = o;
  });
}

mera_status mera_opt_step(mera_ctx* ctx, mera_opt* opt, int* done, mera_result* state) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(opt && opt->owner == ctx, MERA_EINVAL, "optimiser belongs to another context");
    DeviceGuard g(ctx->c.device);
    const bool d = opt->o.advance();
    if (done) *done = d ? 1 : 0;
    if (state) {
      std::memset(state, 0, sizeof(*state));
      state->energy = opt->o.f;
      state->gnorm = opt->o.gnorm;
      state->iterations = opt->o.iter;
      state->evaluations = opt->o.evals;
      state->status = d ? opt->o.status : -1;
      state->polish_iter = opt->o.polish_iter;
      state->macs = ctx->c.macs - opt->o.macs0;
      state->krylov_applications = opt->o.krylov_apps;
    }
  });
}

mera_status mera_opt_final(mera_ctx* ctx, mera_opt* opt, double* const* final_host) {
  if (!ctx) return MERA_EINVAL;
  return guarded(ctx, [&] {
    MERA_CHECK(opt && opt->owner == ctx && final_host, MERA_EINVAL, "mera_opt_final arguments");
    DeviceGuard g(ctx->c.device);
    for (int i = 0; i < opt->o.W.count(); ++i) {
      MatView v = opt->o.W.view(i);
      MERA_HIP(hipMemcpyAsync(final_host[i], v.data, (size_t)v.n * v.p * 8, hipMemcpyDeviceToHost, ctx->c.stream));
    }
    ctx->c.sync();
  });
}

void mera_opt_destroy(mera_opt* opt) {
  if (!opt) return;
  try {
    DeviceGuard g(opt->device);
    delete opt;
  } catch (...) {
  }
}

}  // extern "C"
