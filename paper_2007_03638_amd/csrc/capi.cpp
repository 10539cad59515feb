// extern "C" boundary: argument validation, device selection, exception -> status translation.
#include <cmath>
#include <cstring>

#include "common.h"
#include "mera.h"
#include "model.h"
#include "network.h"


namespace mera {

Ctx::Ctx() : plans(new PlanCache) {}
Ctx::~Ctx() {}

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
  MERA_CHECK(m != nullptr, MERA_EINVAL, std::string(what) + ": null matrix array");
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
    MERA_CHECK(u[t].n == a2 && u[t].p == a2, MERA_EINVAL,
               std::string(what) + ": u[" + std::to_string(t) + "] must be " + std::to_string(a2) + "x" +
                   std::to_string(a2));
    MERA_CHECK(w[t].n == a2 && w[t].p == dims[t].b, MERA_EINVAL,
               std::string(what) + ": w[" + std::to_string(t) + "] must be " + std::to_string(a2) + "x" +
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
    ctx->c.plans->map.clear();
  });
}

double mera_ctx_macs(const mera_ctx* ctx) { return ctx ? ctx->c.macs : 0.0; }

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
    MERA_CHECK(u->data && u->n == a2 && u->p == a2 && w->data && w->n == a2 && w->p == dims[layer].b,
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
    MERA_CHECK(u->data && u->n == a2 && u->p == a2 && w->data && w->n == a2 && w->p == dims[layer].b,
               MERA_EINVAL, "tensor shape");
    DeviceGuard g(ctx->c.device);
    descend_op(ctx->c, dims[layer], u->data, w->data, to_prec(prec), rho_in, rho_out);
    ctx->c.sync();
  });
}

}  // extern "C"
