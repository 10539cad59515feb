"""Riemannian L-BFGS with a Wolfe / approximate-Wolfe line search (oracle; test infrastructure only).

Sec. 3 of the paper. Readings where the paper leaves details open (constants are "free" in the paper):
  * Wolfe conditions on phi(alpha) = C(R_W(d, alpha)) with slope phi'(alpha) = g(G', X'), X' = dR/dalpha
    (eqs. wolfe_1, wolfe_2). eq. wolfe_1 as printed lacks alpha and its sign allows an increase; it is read as the
    Armijo rule phi(alpha) <= phi(0) + c1 alpha phi'(0). c1 = 1e-4, c2 = 0.9.
  * Approximate-Wolfe switch in the spirit of the Hager-Zhang line search cited in Sec. 3:
    (2 c1 - 1) phi'(0) >= phi'(alpha) >= c2 phi'(0) together with phi(alpha) <= phi(0) + eps |phi(0)|, eps = 1e-6.
  * Trial steps: alpha = 1 first; while no upper bracket exists, double; afterwards a safeguarded secant on the
    slopes, falling back to bisection; at most `max_evals` evaluations.
  * L-BFGS (Sec. 3): two-loop recursion over the last m pairs, transported to the current point; initial inverse
    Hessian gamma * P with P the preconditioner and gamma = <s, y> / <y, P y> from the newest pair;
    s_k = T(alpha d_k), y_k = G_{k+1} - T(G_k); a pair with <s, y> <= 1e-12 |s| |y| is not stored; if the
    direction is not a descent direction the history is dropped and d = -P(G).
  * Evenbly-Vidal update (App. A) as the comparator: for one tensor W with environment D (the Euclidean
    derivative) and rho its reduced density matrix on the top legs, the shifted environment D_gamma = D - gamma W rho
    and W <- polar(-D_gamma); gamma is the free shift of the Hamiltonian, acting as an inverse step size. A sweep
    updates u_1, w_1, ..., u_s, w_s in turn, each with a fresh environment.
  * Nonlinear conjugate gradient (Sec. 3, with the Hager-Zhang coefficient the paper uses): d_{k+1} = -P G_{k+1}
    + beta_k T(d_k), inner products in the metric, the previous direction carried over by the transport; beta_k in
    the preconditioned Hager-Zhang form <y, P g>/<d, y> - 2 <y, P y> <d, g>/<d, y>^2 (y = G_{k+1} - T(G_k), d the
    transported previous direction), truncated below at -1/(|d| min(0.01, |G_k|)) as Hager and Zhang do. A
    non-descent direction restarts from -P G. First trial step: 1 after a (re)start, otherwise
    alpha_{k-1} <G_{k-1}, d_{k-1}> / <G_k, d_k> (the usual scaling for methods without a natural step length).
"""
import math
import numpy as np

from . import manifold as mf
from . import mera as om
from . import ternary as tm


def _axpy(a, X, Y):
    return [y + a * x for x, y in zip(X, Y)]


def _scale(a, X):
    return [a * x for x in X]


class LBFGSHistory:
    """Limited-memory pairs (s_i, y_i) with 1/<s_i, y_i>, oldest first."""

    def __init__(self, m):
        self.m = m
        self.S, self.Y, self.R = [], [], []

    def reset(self):
        self.S, self.Y, self.R = [], [], []

    def direction(self, G, precond):
        """Two-loop recursion: returns d = -H G with H0 = gamma P."""
        q = [g.copy() for g in G]
        alphas = []
        for s, y, r in zip(reversed(self.S), reversed(self.Y), reversed(self.R)):
            a = r * mf.inner(s, q)
            q = _axpy(-a, y, q)
            alphas.append(a)
        z = precond(q)
        if self.S:
            py = precond(self.Y[-1])
            z = _scale(mf.inner(self.S[-1], self.Y[-1]) / mf.inner(self.Y[-1], py), z)
        for (s, y, r), a in zip(zip(self.S, self.Y, self.R), reversed(alphas)):
            b = r * mf.inner(y, z)
            z = _axpy(a - b, s, z)
        return _scale(-1.0, z)

    def transport(self, T):
        """Carry the stored pairs to the new point with the vector transport T (a map on factor lists)."""
        self.S = [T(s) for s in self.S]
        self.Y = [T(y) for y in self.Y]

    def push(self, s, y):
        sy = mf.inner(s, y)
        if sy <= 1e-12 * math.sqrt(mf.inner(s, s) * mf.inner(y, y)):
            return False
        self.S.append(s)
        self.Y.append(y)
        self.R.append(1.0 / sy)
        if len(self.S) > self.m:
            self.S.pop(0)
            self.Y.pop(0)
            self.R.pop(0)
        return True


def line_search(phi, f0, df0, alpha0=1.0, c1=1e-4, c2=0.9, eps=1e-6, max_evals=10):
    """Find alpha meeting the Wolfe or approximate-Wolfe conditions. phi(alpha) -> (f, df, payload).

    Returns (ok, alpha, f, df, payload, evals).
    """
    epsk = eps * abs(f0)
    lo_a, lo_df = 0.0, df0
    hi_a, hi_df = math.inf, None
    alpha = alpha0
    for n in range(1, max_evals + 1):
        f, df, payload = phi(alpha)
        if not (math.isfinite(f) and math.isfinite(df)):
            hi_a, hi_df = alpha, math.inf
        else:
            wolfe = f <= f0 + c1 * alpha * df0 and df >= c2 * df0
            approx = (2.0 * c1 - 1.0) * df0 >= df >= c2 * df0 and f <= f0 + epsk
            if wolfe or approx:
                return True, alpha, f, df, payload, n
            if df >= 0.0 or f > f0 + epsk:
                hi_a, hi_df = alpha, df
            else:
                lo_a, lo_df = alpha, df
        if math.isinf(hi_a):
            alpha = 2.0 * alpha
            continue
        width = hi_a - lo_a
        trial = None
        if hi_df is not None and math.isfinite(hi_df) and hi_df >= 0.0 and hi_df > lo_df:
            trial = (lo_a * hi_df - hi_a * lo_df) / (hi_df - lo_df)
        if trial is None or not (lo_a + 0.1 * width <= trial <= hi_a - 0.1 * width):
            trial = lo_a + 0.5 * width
        alpha = trial
    return False, alpha, None, None, None, max_evals


class Problem:
    """The MERA cost on the product of Stiefel manifolds, flattened as [u_1, w_1, ..., u_s, w_s]. With
    grassmann_w the isometries w are treated as points of Grassmann manifolds (the paper's choice, Sec. 4): their
    gradient and projection transport use the Grassmann projection (1 - W W^T)."""

    def __init__(self, h3, chi, T, d=4, grassmann_w=False, geometry='binary'):
        """h3: the local term (3-site for the binary geometry, 2-site for the ternary one, Sec. 4)."""
        self.h3, self.chi, self.T, self.d = h3, chi, T, d
        self.geo = om if geometry == 'binary' else tm
        self.dims = self.geo.layer_dims(chi, T, d)
        self.evals = 0
        self.grassmann = [grassmann_w and i % 2 == 1 for i in range(2 * len(self.dims))]

    def project(self, i, W, D):
        return mf.grassmann_project(W, D) if self.grassmann[i] else mf.project(W, D)

    def evaluate(self, W):
        params = [(W[2 * i], W[2 * i + 1]) for i in range(len(self.dims))]
        ev = self.geo.evaluate(params, self.h3, self.chi, self.T, self.d)
        self.evals += 1
        D = [m for pair in ev['grads'] for m in pair]
        G = [self.project(i, w, dd) for i, (w, dd) in enumerate(zip(W, D))]
        rdms = self.geo.preconditioner_rdms(ev['rhos'], params, self.dims)
        rv = [m for pair in rdms for m in pair]
        self.last_D = D
        return ev['energy'], G, rv


def _retract(kind, W, X, alpha):
    return mf.retract_exp(W, X, alpha) if kind == 'exp' else mf.retract(W, X, alpha)


def _transport_map(kind, problem, W, d, alpha, Wn):
    """Vector transport from W to Wn = R_W(d, alpha): exp(alpha Q_d) (eq. transport) for the exponential retraction,
    otherwise the projection onto the tangent space at Wn."""
    if kind == 'exp':
        return lambda X: [mf.transport_exp(w, dd, alpha, x) for w, dd, x in zip(W, d, X)]
    return lambda X: [problem.project(i, wn, x) for i, (wn, x) in enumerate(zip(Wn, X))]


def optimize(W0, problem, m=8, max_iter=200, grad_tol=1e-10, use_precond=True, ls_max_evals=10, log=None,
             retraction='polar'):
    """Riemannian L-BFGS driver (Sec. 3) on the flattened parameter list W0. retraction: 'polar' (polar retraction,
    projection transport) or 'exp' (the paper's exponential retraction and transport, Sec. 2.3).
    Returns (W, energy, |G|, info)."""
    W = [w.copy() for w in W0]
    f, G, rv = problem.evaluate(W)
    hist = LBFGSHistory(m)
    it = 0
    status = 'maxiter'
    for it in range(max_iter):
        gnorm = math.sqrt(mf.inner(G, G))
        if log is not None:
            log.append(dict(iter=it, energy=f, gnorm=gnorm, evals=problem.evals))
        if gnorm <= grad_tol:
            status = 'converged'
            break

        def P(X, _W=W, _rv=rv):
            if not use_precond:
                return [x.copy() for x in X]
            return [mf.precondition(w, x, r) for w, x, r in zip(_W, X, _rv)]
        d = hist.direction(G, P)
        slope = mf.inner(G, d)
        if not slope < 0.0:
            hist.reset()
            d = _scale(-1.0, P(G))
            slope = mf.inner(G, d)

        def phi(alpha, _W=W, _dl=[d]):
            pairs = [_retract(retraction, w, x, alpha) for w, x in zip(_W, _dl[0])]
            Wn = [p[0] for p in pairs]
            Xp = [p[1] for p in pairs]
            fn, Gn, rvn = problem.evaluate(Wn)
            return fn, mf.inner(Gn, Xp), (Wn, Gn, rvn)
        dl = [d]
        ok, alpha, fn, dfn, payload, _ = line_search(lambda a: phi(a, _dl=dl), f, slope, max_evals=ls_max_evals)
        if not ok and hist.S:
            hist.reset()
            d = _scale(-1.0, P(G))
            dl[0] = d
            slope = mf.inner(G, d)
            ok, alpha, fn, dfn, payload, _ = line_search(lambda a: phi(a, _dl=dl), f, slope, max_evals=ls_max_evals)
        if not ok:
            status = 'linesearch_failed'
            break
        Wn, Gn, rvn = payload
        T = _transport_map(retraction, problem, W, d, alpha, Wn)
        s = T(_scale(alpha, d))
        y = [gn - tg for gn, tg in zip(Gn, T(G))]
        hist.transport(T)
        hist.push(s, y)
        W, f, G, rv = Wn, fn, Gn, rvn
    else:
        it = max_iter
    gnorm = math.sqrt(mf.inner(G, G))
    return W, f, gnorm, dict(iterations=it, evals=problem.evals, status=status)


def hz_beta(g, pg, y, py, d, g_old_norm, eta=0.01, truncate=True):
    """Hager-Zhang conjugate-gradient coefficient with a preconditioner P (pg = P g, py = P y):
    <y, P g>/<d, y> - 2 <y, P y> <d, g>/<d, y>^2, optionally truncated below at -1/(|d| min(eta, |g_old|)).
    Returns 0 when <d, y> vanishes."""
    dy = mf.inner(d, y)
    if dy == 0.0 or not math.isfinite(dy):
        return 0.0
    beta = mf.inner(y, pg) / dy - 2.0 * mf.inner(y, py) * mf.inner(d, g) / (dy * dy)
    if truncate:
        dn = math.sqrt(mf.inner(d, d))
        if dn > 0.0 and g_old_norm > 0.0:
            beta = max(beta, -1.0 / (dn * min(eta, g_old_norm)))
    return beta


def optimize_cg(W0, problem, max_iter=200, grad_tol=1e-10, use_precond=True, ls_max_evals=10, log=None,
                retraction='polar'):
    """Riemannian nonlinear conjugate gradient (Sec. 3, Hager-Zhang coefficient) on the flattened parameter list W0.
    Returns (W, energy, |G|, info)."""
    W = [w.copy() for w in W0]
    f, G, rv = problem.evaluate(W)
    d_prev = None          # previous direction, transported to the current point
    y = None               # G_k - T(G_{k-1})
    g_old_norm = None
    alpha_prev = slope_prev = None
    it = 0
    status = 'maxiter'
    for it in range(max_iter):
        gnorm = math.sqrt(mf.inner(G, G))
        if log is not None:
            log.append(dict(iter=it, energy=f, gnorm=gnorm, evals=problem.evals))
        if gnorm <= grad_tol:
            status = 'converged'
            break

        def P(X, _W=W, _rv=rv):
            if not use_precond:
                return [x.copy() for x in X]
            return [mf.precondition(w, x, r) for w, x, r in zip(_W, X, _rv)]
        pg = P(G)
        d = _scale(-1.0, pg)
        momentum = False
        if d_prev is not None:
            beta = hz_beta(G, pg, y, P(y), d_prev, g_old_norm)
            d = _axpy(beta, d_prev, d)
            momentum = True
        slope = mf.inner(G, d)
        if not slope < 0.0:
            d = _scale(-1.0, pg)
            slope = mf.inner(G, d)
            momentum = False
        alpha0 = alpha_prev * slope_prev / slope if (momentum and alpha_prev is not None) else 1.0

        dl = [d]

        def phi(alpha, _W=W):
            pairs = [_retract(retraction, w, x, alpha) for w, x in zip(_W, dl[0])]
            Wn = [p[0] for p in pairs]
            Xp = [p[1] for p in pairs]
            fn, Gn, rvn = problem.evaluate(Wn)
            return fn, mf.inner(Gn, Xp), (Wn, Gn, rvn)
        ok, alpha, fn, dfn, payload, _ = line_search(phi, f, slope, alpha0=alpha0, max_evals=ls_max_evals)
        if not ok and momentum:
            d = _scale(-1.0, pg)
            dl[0] = d
            slope = mf.inner(G, d)
            ok, alpha, fn, dfn, payload, _ = line_search(phi, f, slope, alpha0=1.0, max_evals=ls_max_evals)
        if not ok:
            status = 'linesearch_failed'
            break
        Wn, Gn, rvn = payload
        T = _transport_map(retraction, problem, W, d, alpha, Wn)
        d_prev = T(d)
        y = [gn - tg for gn, tg in zip(Gn, T(G))]
        g_old_norm = gnorm
        alpha_prev, slope_prev = alpha, slope
        W, f, G, rv = Wn, fn, Gn, rvn
    else:
        it = max_iter
    gnorm = math.sqrt(mf.inner(G, G))
    return W, f, gnorm, dict(iterations=it, evals=problem.evals, status=status)


def ev_update(W, D, rho, gamma):
    """Evenbly-Vidal local update (App. A): the polar factor of -D_gamma = gamma W rho - D."""
    return mf.polar_factor(gamma * W @ rho - D)


def optimize_ev(W0, problem, gamma, max_iter=20, grad_tol=0.0, log=None):
    """Evenbly-Vidal sweeps (App. A): each iteration updates every tensor in turn (u_1, w_1, ..., u_s, w_s), each
    from a fresh evaluation of its environment. Returns (W, energy, |G|, info)."""
    W = [w.copy() for w in W0]
    f, G, rv = problem.evaluate(W)
    it = 0
    status = 'maxiter'
    for it in range(max_iter):
        gnorm = math.sqrt(mf.inner(G, G))
        if log is not None:
            log.append(dict(iter=it, energy=f, gnorm=gnorm, evals=problem.evals))
        if gnorm <= grad_tol:
            status = 'converged'
            break
        for i in range(len(W)):
            if i > 0:
                f, G, rv = problem.evaluate(W)
            W[i] = ev_update(W[i], problem.last_D[i], rv[i], gamma)
        f, G, rv = problem.evaluate(W)
    else:
        it = max_iter
    gnorm = math.sqrt(mf.inner(G, G))
    return W, f, gnorm, dict(iterations=it, evals=problem.evals, status=status)
