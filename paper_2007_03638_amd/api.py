"""Python binding of the C ABI (include/mera.h): argument marshalling only.

Every computation runs in the HIP library; torch supplies device memory and the stream. Matrices are torch
float64 CUDA tensors, row-major (contiguous). Names follow the C calls.
"""
import ctypes

import numpy as np
import torch

from . import _lib as L

PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}
STATUS = {0: "MERA_OK", -1: "MERA_EINVAL", -2: "MERA_ENOMEM", -3: "MERA_EHIP", -4: "MERA_ENOCONV",
          -5: "MERA_ENONFINITE", -6: "MERA_EBUSY"}


class MeraError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _prec(p):
    return PREC[p] if isinstance(p, str) else int(p)


def _mats(ts):
    arr = (L.MeraMat * len(ts))()
    for i, t in enumerate(ts):
        if t is None:
            raise ValueError("missing matrix")
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.dim() != 2:
            raise ValueError("matrices must be contiguous 2-D float64 CUDA tensors")
        arr[i] = L.MeraMat(t.shape[0], t.shape[1], t.data_ptr())
    return arr


GEOMETRIES = {"binary": 0, "ternary": 1}


def _shape(T, chi, d=4, geometry="binary"):
    return L.MeraShape(T, d, chi, GEOMETRIES[geometry])


def _sites(geometry):
    return 3 if geometry == "binary" else 2


def h3_tfim(h=1.0):
    out = np.zeros((64, 64))
    st = L.load().mera_h3_tfim(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if st != 0:
        raise MeraError(st, "mera_h3_tfim")
    return out


def h2_tfim(h=1.0):
    """Two-site TFIM term on unblocked spins (ternary geometry)."""
    out = np.zeros((4, 4))
    st = L.load().mera_h2_tfim(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if st != 0:
        raise MeraError(st, "mera_h2_tfim")
    return out


def h2_xxz(delta):
    out = np.zeros((4, 4))
    st = L.load().mera_h2_xxz(delta, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if st != 0:
        raise MeraError(st, "mera_h2_xxz")
    return out


def h3_xxz(delta):
    out = np.zeros((64, 64))
    st = L.load().mera_h3_xxz(delta, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if st != 0:
        raise MeraError(st, "mera_h3_xxz")
    return out


def layer_dims(T, chi, d=4, geometry="binary"):
    a = (ctypes.c_int * (T + 1))()
    b = (ctypes.c_int * (T + 1))()
    sh = _shape(T, chi, d, geometry)
    st = L.load().mera_layer_dims(ctypes.byref(sh), a, b)
    if st != 0:
        raise MeraError(st, "mera_layer_dims")
    return [(a[i], b[i]) for i in range(T + 1)]


class Warm:
    def __init__(self, ctx, T, chi, d=4, geometry="binary"):
        self._lib = L.load()
        self.ptr = ctypes.c_void_p()
        sh = _shape(T, chi, d, geometry)
        ctx._check(self._lib.mera_warm_create(ctx.ptr, ctypes.byref(sh), ctypes.byref(self.ptr)), "warm_create")

    def __del__(self):
        try:
            if self.ptr.value:
                self._lib.mera_warm_destroy(self.ptr)
                self.ptr.value = None
        except Exception:
            pass


class Context:
    """A library context on one device, ordered on torch's current stream of that device."""

    def __init__(self, device=0):
        self._lib = L.load()
        self.device = torch.device("cuda", device)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        self.ptr = ctypes.c_void_p()
        st = self._lib.mera_ctx_create(device, ctypes.c_void_p(stream), ctypes.byref(self.ptr))
        if st != 0:
            raise MeraError(st, "mera_ctx_create")

    def __del__(self):
        try:
            if self.ptr.value:
                self._lib.mera_ctx_destroy(self.ptr)
                self.ptr.value = None
        except Exception:
            pass

    def _check(self, st, what):
        if st != 0:
            raise MeraError(st, f"{what}: {self._lib.mera_last_error(self.ptr).decode()}")

    def macs(self):
        return self._lib.mera_ctx_macs(self.ptr)

    def trim(self):
        self._check(self._lib.mera_ctx_trim(self.ptr), "mera_ctx_trim")

    def set_intermediate_limit(self, nbytes):
        self._check(self._lib.mera_ctx_set_intermediate_limit(self.ptr, int(nbytes)), "mera_ctx_set_intermediate_limit")

    def set_verbose(self, level=1):
        self._check(self._lib.mera_ctx_set_verbose(self.ptr, int(level)), "mera_ctx_set_verbose")

    def profile(self, enable=True):
        self._check(self._lib.mera_ctx_profile(self.ptr, 1 if enable else 0), "mera_ctx_profile")

    def kernel_stats(self, cap=64):
        arr = (L.KernelStat * cap)()
        n = self._lib.mera_ctx_kernel_stats(self.ptr, arr, cap)
        if n < 0:
            self._check(n, "mera_ctx_kernel_stats")
        return [dict(kernel=arr[i].kernel.decode(), launches=arr[i].launches, seconds=arr[i].seconds,
                     flops=arr[i].flops, bytes=arr[i].bytes) for i in range(min(n, cap))]

    def optimizer(self, **job_kwargs):
        return Optimizer(self, **job_kwargs)

    def _dev(self, x):
        return torch.as_tensor(x, dtype=torch.float64).to(self.device).contiguous()

    # ---- energy and gradient ---------------------------------------------------------------------------
    def energy_grad(self, T, chi, u, w, h3, prec="fp64", warm=None, krylov=None, rdms=False, d=4,
                    geometry="binary"):
        dims = layer_dims(T, chi, d, geometry)
        u = [self._dev(x) for x in u]
        w = [self._dev(x) for x in w]
        h3d = self._dev(h3)
        Du = [torch.empty_like(x) for x in u]
        Dw = [torch.empty_like(x) for x in w]
        ru = rw = None
        if rdms:
            ru = [torch.empty((a * a, a * a), dtype=torch.float64, device=self.device) for a, b in dims]
            rw = [torch.empty((b, b), dtype=torch.float64, device=self.device) for a, b in dims]
        e = ctypes.c_double()
        info = L.EvalInfo()
        ko = None
        if krylov is not None:
            ko = L.KrylovOpts(krylov.get("dim", 0), krylov.get("max_restarts", 0), krylov.get("tol", 0.0),
                              krylov.get("extrapolate", 0))
        sh = _shape(T, chi, d, geometry)
        st = self._lib.mera_energy_grad(self.ptr, ctypes.byref(sh), _mats(u), _mats(w), h3d.data_ptr(),
                                        _prec(prec), warm.ptr if warm else None,
                                        ctypes.byref(ko) if ko else None, ctypes.byref(e), _mats(Du), _mats(Dw),
                                        _mats(ru) if rdms else None, _mats(rw) if rdms else None,
                                        ctypes.byref(info))
        self._check(st, "mera_energy_grad")
        out = dict(energy=e.value, Du=Du, Dw=Dw, applications_rho=info.applications_rho,
                   applications_htilde=info.applications_htilde, residual_rho=info.residual_rho,
                   residual_htilde=info.residual_htilde, macs=info.macs)
        if rdms:
            out["rho_u"], out["rho_w"] = ru, rw
        return out

    def ascend(self, T, chi, layer, u, w, h_in, prec="fp64", d=4, geometry="binary"):
        a, b = layer_dims(T, chi, d, geometry)[layer]
        u, w, hi = self._dev(u), self._dev(w), self._dev(h_in)
        k = _sites(geometry)
        ho = torch.empty((b ** k, b ** k), dtype=torch.float64, device=self.device)
        sh = _shape(T, chi, d, geometry)
        self._check(self._lib.mera_ascend(self.ptr, ctypes.byref(sh), layer, _mats([u]), _mats([w]), _prec(prec),
                                          hi.data_ptr(), ho.data_ptr()), "mera_ascend")
        return ho

    def descend(self, T, chi, layer, u, w, rho_in, prec="fp64", d=4, geometry="binary"):
        a, b = layer_dims(T, chi, d, geometry)[layer]
        u, w, ri = self._dev(u), self._dev(w), self._dev(rho_in)
        k = _sites(geometry)
        ro = torch.empty((a ** k, a ** k), dtype=torch.float64, device=self.device)
        sh = _shape(T, chi, d, geometry)
        self._check(self._lib.mera_descend(self.ptr, ctypes.byref(sh), layer, _mats([u]), _mats([w]), _prec(prec),
                                           ri.data_ptr(), ro.data_ptr()), "mera_descend")
        return ro

    def layer_grad(self, T, chi, layer, u, w, h_in, rho_in, prec="fp64", split=False, d=4, geometry="binary"):
        """Derivative of Tr[A(h) rho] for one layer: returns (Du, Dw, rho_out, h_out); h_out is None unless split."""
        dims = layer_dims(T, chi, d, geometry)
        a, b = dims[layer] if 0 <= layer < len(dims) else dims[-1]  # the library rejects a bad layer
        u, w, hi, ri = self._dev(u), self._dev(w), self._dev(h_in), self._dev(rho_in)
        k = _sites(geometry)
        Du, Dw = torch.empty_like(u), torch.empty_like(w)
        ro = torch.empty((a ** k, a ** k), dtype=torch.float64, device=self.device)
        ho = torch.empty((b ** k, b ** k), dtype=torch.float64, device=self.device) if split else None
        sh = _shape(T, chi, d, geometry)
        self._check(self._lib.mera_layer_grad(self.ptr, ctypes.byref(sh), layer, _mats([u]), _mats([w]), _prec(prec),
                                              1 if split else 0, hi.data_ptr(), ri.data_ptr(),
                                              ho.data_ptr() if split else None, _mats([Du]), _mats([Dw]),
                                              ro.data_ptr()), "mera_layer_grad")
        return Du, Dw, ro, ho

    # ---- Stiefel manifold ---------------------------------------------------------------------------------
    def stiefel_project(self, W, D):
        W = [self._dev(x) for x in W]
        D = [self._dev(x) for x in D]
        G = [torch.empty_like(x) for x in D]
        self._check(self._lib.stiefel_project(self.ptr, len(W), _mats(W), _mats(D), _mats(G)), "stiefel_project")
        return G

    def stiefel_project_noalloc(self, W, D, G=None):
        """stiefel_project through the allocation-free entry point. W, D (and G, if given) must already be device
        tensors; the call is only ordered on the context stream (synchronise before reading G)."""
        G = [torch.empty_like(x) for x in D] if G is None else G
        self._check(self._lib.stiefel_project_noalloc(self.ptr, len(W), _mats(W), _mats(D), _mats(G)),
                    "stiefel_project_noalloc")
        return G

    def stiefel_retract(self, W, X, alpha, tangent=True):
        W = [self._dev(x) for x in W]
        X = [self._dev(x) for x in X]
        Wo = [torch.empty_like(x) for x in W]
        Xo = [torch.empty_like(x) for x in W] if tangent else None
        self._check(self._lib.stiefel_retract(self.ptr, len(W), _mats(W), _mats(X), float(alpha), _mats(Wo),
                                              _mats(Xo) if tangent else None), "stiefel_retract")
        return (Wo, Xo) if tangent else Wo

    def stiefel_transport(self, Wn, Y):
        Wn = [self._dev(x) for x in Wn]
        Y = [self._dev(x) for x in Y]
        Yo = [torch.empty_like(x) for x in Y]
        self._check(self._lib.stiefel_transport(self.ptr, len(Wn), _mats(Wn), _mats(Y), _mats(Yo)),
                    "stiefel_transport")
        return Yo

    def stiefel_retract_exp(self, W, X, alpha, tangent=True):
        W = [self._dev(x) for x in W]
        X = [self._dev(x) for x in X]
        Wo = [torch.empty_like(x) for x in W]
        Xo = [torch.empty_like(x) for x in W] if tangent else None
        self._check(self._lib.stiefel_retract_exp(self.ptr, len(W), _mats(W), _mats(X), float(alpha), _mats(Wo),
                                                  _mats(Xo) if tangent else None), "stiefel_retract_exp")
        return (Wo, Xo) if tangent else Wo

    def stiefel_transport_exp(self, W, X, alpha, Y):
        W = [self._dev(x) for x in W]
        X = [self._dev(x) for x in X]
        Y = [self._dev(x) for x in Y]
        Yo = [torch.empty_like(x) for x in Y]
        self._check(self._lib.stiefel_transport_exp(self.ptr, len(W), _mats(W), _mats(X), float(alpha), _mats(Y),
                                                    _mats(Yo)), "stiefel_transport_exp")
        return Yo

    def ev_update(self, W, D, rho, gamma):
        W = [self._dev(x) for x in W]
        D = [self._dev(x) for x in D]
        R = [self._dev(x) for x in rho]
        Wo = [torch.empty_like(x) for x in W]
        self._check(self._lib.mera_ev_update(self.ptr, len(W), _mats(W), _mats(D), _mats(R), float(gamma),
                                             _mats(Wo)), "mera_ev_update")
        return Wo

    def grassmann_project(self, W, D):
        W = [self._dev(x) for x in W]
        D = [self._dev(x) for x in D]
        G = [torch.empty_like(x) for x in D]
        self._check(self._lib.grassmann_project(self.ptr, len(W), _mats(W), _mats(D), _mats(G)), "grassmann_project")
        return G

    def stiefel_precondition(self, W, X, rho, delta=-1.0):
        W = [self._dev(x) for x in W]
        X = [self._dev(x) for x in X]
        R = [self._dev(x) for x in rho]
        Xo = [torch.empty_like(x) for x in X]
        self._check(self._lib.stiefel_precondition(self.ptr, len(W), _mats(W), _mats(X), _mats(R), float(delta),
                                                   _mats(Xo)), "stiefel_precondition")
        return Xo

    def inner(self, X, Y):
        X = [self._dev(x) for x in X]
        Y = [self._dev(x) for x in Y]
        out = ctypes.c_double()
        self._check(self._lib.mera_inner(self.ptr, len(X), _mats(X), _mats(Y), ctypes.byref(out)), "mera_inner")
        return out.value

    # ---- L-BFGS -------------------------------------------------------------------------------------------
    def lbfgs(self, shapes, m=8):
        return LBFGS(self, shapes, m)

    # ---- whole optimisation -------------------------------------------------------------------------------
    def run_optimize(self, T, chi, h3, init, prec="fp64", m=8, max_iter=100, grad_tol=1e-10, polish_tol=0.0,
                     precondition=True, max_ls_evals=10, krylov=None, d=4, log_cap=0, want_final=False,
                     method="lbfgs", retraction="polar", grassmann_w=False, ev_gamma=0.0, geometry="binary"):
        job, keep = make_job(T, chi, h3, init, prec, m, max_iter, grad_tol, polish_tol, precondition,
                             max_ls_evals, krylov, d, method, retraction, grassmann_w, ev_gamma, geometry)
        res = L.Result()
        logs = (L.IterLog * max(log_cap, 1))()
        nlog = ctypes.c_int(0)
        finals = None
        fin_arr = None
        if want_final:
            finals = [np.zeros_like(np.asarray(x, dtype=np.float64)) for x in init]
            fin_arr = (ctypes.POINTER(ctypes.c_double) * len(finals))(
                *[f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for f in finals])
        st = self._lib.run_optimize(self.ptr, ctypes.byref(job), ctypes.byref(res), fin_arr, logs, log_cap,
                                    ctypes.byref(nlog))
        self._check(st, "run_optimize")
        out = result_dict(res)
        out["log"] = [dict(iter=logs[i].iter, evals=logs[i].evals, energy=logs[i].energy, gnorm=logs[i].gnorm,
                           alpha=logs[i].alpha, prec=logs[i].prec) for i in range(nlog.value)]
        if want_final:
            out["final"] = finals
        del keep
        return out


def result_dict(res):
    return dict(energy=res.energy, gnorm=res.gnorm, iterations=res.iterations, evaluations=res.evaluations,
                status=res.status, polish_iter=res.polish_iter, seconds=res.seconds, macs=res.macs,
                queued_seconds=res.queued_seconds, krylov_applications=res.krylov_applications)


def make_job(T, chi, h3, init, prec="fp64", m=8, max_iter=100, grad_tol=1e-10, polish_tol=0.0, precondition=True,
             max_ls_evals=10, krylov=None, d=4, method="lbfgs", retraction="polar", grassmann_w=False,
             ev_gamma=0.0, geometry="binary"):
    """Build a mera_job; returns (job, keepalive) — keep the second item alive while the job is in use."""
    h3c = np.ascontiguousarray(h3, dtype=np.float64)
    mats = [np.ascontiguousarray(x, dtype=np.float64) for x in init]
    ptrs = (ctypes.POINTER(ctypes.c_double) * len(mats))(
        *[x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for x in mats])
    kr = krylov or {}
    job = L.Job(_shape(T, chi, d, geometry), h3c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ptrs, _prec(prec), m,
                max_iter, grad_tol, polish_tol, 1 if precondition else 0, max_ls_evals,
                L.KrylovOpts(kr.get("dim", 0), kr.get("max_restarts", 0), kr.get("tol", 0.0), kr.get("extrapolate", 0)),
                {"lbfgs": 0, "cg": 1, "ev": 2}[method], {"polar": 0, "exp": 1}[retraction],
                1 if grassmann_w else 0, float(ev_gamma))
    return job, (h3c, mats, ptrs)


class Optimizer:
    """Step-wise optimisation (mera_opt_*): one L-BFGS iteration per step()."""

    def __init__(self, ctx, **job_kwargs):
        self.ctx = ctx
        self._lib = ctx._lib
        self.shapes = [np.asarray(x).shape for x in job_kwargs["init"]]
        job, keep = make_job(**job_kwargs)
        self.ptr = ctypes.c_void_p()
        ctx._check(self._lib.mera_opt_create(ctx.ptr, ctypes.byref(job), ctypes.byref(self.ptr)), "mera_opt_create")
        del keep

    def step(self):
        done = ctypes.c_int()
        res = L.Result()
        self.ctx._check(self._lib.mera_opt_step(self.ctx.ptr, self.ptr, ctypes.byref(done), ctypes.byref(res)),
                        "mera_opt_step")
        return bool(done.value), result_dict(res)

    def final(self):
        outs = [np.zeros(s) for s in self.shapes]
        arr = (ctypes.POINTER(ctypes.c_double) * len(outs))(
            *[o.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for o in outs])
        self.ctx._check(self._lib.mera_opt_final(self.ctx.ptr, self.ptr, arr), "mera_opt_final")
        return outs

    def __del__(self):
        try:
            if self.ptr.value:
                self._lib.mera_opt_destroy(self.ptr)
                self.ptr.value = None
        except Exception:
            pass


class LBFGS:
    def __init__(self, ctx, shapes, m=8):
        self.ctx = ctx
        self._lib = ctx._lib
        n = (ctypes.c_int * len(shapes))(*[s[0] for s in shapes])
        p = (ctypes.c_int * len(shapes))(*[s[1] for s in shapes])
        self.ptr = ctypes.c_void_p()
        ctx._check(self._lib.lbfgs_create(ctx.ptr, len(shapes), n, p, m, ctypes.byref(self.ptr)), "lbfgs_create")

    def __del__(self):
        try:
            if self.ptr.value:
                self._lib.lbfgs_destroy(self.ptr)
                self.ptr.value = None
        except Exception:
            pass

    def size(self):
        return self._lib.lbfgs_size(self.ptr)

    def reset(self):
        self.ctx._check(self._lib.lbfgs_reset(self.ptr), "lbfgs_reset")

    def step(self, W, G, rho=None):
        c = self.ctx
        W = [c._dev(x) for x in W]
        G = [c._dev(x) for x in G]
        R = [c._dev(x) for x in rho] if rho is not None else None
        d = [torch.empty_like(x) for x in G]
        slope = ctypes.c_double()
        c._check(self._lib.lbfgs_step(c.ptr, self.ptr, _mats(W), _mats(G), _mats(R) if R else None, _mats(d),
                                      ctypes.byref(slope)), "lbfgs_step")
        return d, slope.value

    def push(self, Wn, d, alpha, G_old, G_new):
        c = self.ctx
        Wn, d, Go, Gn = ([c._dev(x) for x in X] for X in (Wn, d, G_old, G_new))
        acc = ctypes.c_int()
        c._check(self._lib.lbfgs_push(c.ptr, self.ptr, _mats(Wn), _mats(d), float(alpha), _mats(Go), _mats(Gn),
                                      ctypes.byref(acc)), "lbfgs_push")
        return bool(acc.value)


class Server:
    """Continuous-batching job server (mera_server_*)."""

    def __init__(self, ctx, hbm_budget, max_slots, group_launches=True, graph_capture=True, max_wait_us=None):
        self.ctx = ctx
        self._lib = ctx._lib
        self.ptr = ctypes.c_void_p()
        ctx._check(self._lib.mera_server_create(ctx.ptr, int(hbm_budget), int(max_slots), ctypes.byref(self.ptr)),
                   "mera_server_create")
        ctx._check(self._lib.mera_server_configure(self.ptr, int(bool(group_launches)), int(bool(graph_capture)),
                                                   -1.0 if max_wait_us is None else float(max_wait_us)),
                   "mera_server_configure")

    def stats(self):
        st = L.ServerStats()
        self.ctx._check(self._lib.mera_server_get_stats(self.ptr, ctypes.byref(st)), "mera_server_get_stats")
        return {name: int(getattr(st, name)) for name, _ in L.ServerStats._fields_}

    def submit(self, **job_kwargs):
        job, keep = make_job(**job_kwargs)
        jid = ctypes.c_uint64()
        self.ctx._check(self._lib.mera_server_submit(self.ptr, ctypes.byref(job), ctypes.byref(jid)),
                        "mera_server_submit")
        del keep
        return jid.value

    def poll(self, job_id):
        res = L.Result()
        st = self._lib.mera_server_poll(self.ptr, job_id, ctypes.byref(res))
        if st == -6:
            return None
        self.ctx._check(st, "mera_server_poll")
        return result_dict(res)

    def close(self):
        if getattr(self, "ptr", None) is not None and self.ptr.value:
            self._lib.mera_server_destroy(self.ptr)
            self.ptr.value = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def job_footprint(T, chi, prec="fp32", d=4, geometry="binary"):
    sh = _shape(T, chi, d, geometry)
    return L.load().mera_job_footprint(ctypes.byref(sh), _prec(prec))
