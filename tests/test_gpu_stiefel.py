"""GPU parity of the Stiefel operations and the preconditioner against the oracle (through the C ABI)."""
import numpy as np
import pytest

from gpu_helpers import rel, require_gpu, to_np
from oracle import manifold as mf
from oracle import optim
from paper_2007_03638_amd import inputs

pytestmark = pytest.mark.gpu

# shapes of MERA factors: square disentanglers and tall isometries, several tile sizes and ragged tails; in the
# preconditioner, square factors of 97 (odd) and 144 rows exercise the one-workgroup eigensolver above 64, and 256
# rows the per-round one
SHAPES = [(16, 16), (16, 4), (256, 24), (576, 24), (81, 9), (5, 1), (144, 144), (400, 20), (97, 97), (256, 256)]


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_2007_03638_amd import api
    return api.Context(0)


def _case(seed):
    W = [inputs.haar_params(seed + i, [s])[0] for i, s in enumerate(SHAPES)]
    D = inputs.normal_like(seed + 100, W)
    return W, D


def test_project(ctx):
    W, D = _case(1)
    G = ctx.stiefel_project(W, D)
    for w, d, g in zip(W, D, G):
        ref = mf.project(w, d)
        assert rel(to_np(g), ref) < 1e-13
        S = w.T @ to_np(g)
        assert np.max(np.abs(S + S.T)) < 1e-12


@pytest.mark.parametrize("alpha", [0.0, 1e-3, 0.37, 1.0, 3.0])
def test_retract_and_curve_tangent(ctx, alpha):
    W, D = _case(2)
    X = [mf.project(w, d) / np.linalg.norm(d) for w, d in zip(W, D)]
    Wo, Xo = ctx.stiefel_retract(W, X, alpha)
    for w, x, wo, xo in zip(W, X, Wo, Xo):
        rw, rx = mf.retract(w, x, alpha)
        wo, xo = to_np(wo), to_np(xo)
        print(f"retract {w.shape} alpha={alpha}: W err {rel(wo, rw):.2e} X' err {rel(xo, rx):.2e} "
              f"orth {np.max(np.abs(wo.T @ wo - np.eye(w.shape[1]))):.2e}", flush=True)
        assert np.max(np.abs(wo.T @ wo - np.eye(w.shape[1]))) < 1e-13
        assert rel(wo, rw) < 1e-12
        assert rel(xo, rx) < 1e-10


def test_transport(ctx):
    W, D = _case(3)
    X = [mf.project(w, d) for w, d in zip(W, D)]
    Wn = [to_np(x) for x in ctx.stiefel_retract(W, X, 0.5, tangent=False)]
    Y = [mf.project(w, y) for w, y in zip(W, inputs.normal_like(7, W))]
    T = ctx.stiefel_transport(Wn, Y)
    for wn, y, t in zip(Wn, Y, T):
        assert rel(to_np(t), mf.transport(wn, y)) < 1e-13


@pytest.mark.parametrize("delta", [0.0, 0.05, -1.0])
def test_precondition(ctx, delta):
    W, D = _case(4)
    X = [mf.project(w, d) for w, d in zip(W, D)]
    rho = [inputs.density_matrix(50 + i, w.shape[1]) + 0.01 * np.eye(w.shape[1]) for i, w in enumerate(W)]
    got = ctx.stiefel_precondition(W, X, rho, delta)
    for w, x, r, g in zip(W, X, rho, got):
        ref = mf.precondition(w, x, r, None if delta < 0 else delta)
        err = rel(to_np(g), ref)
        print(f"precondition {w.shape} delta={delta}: {err:.2e}", flush=True)
        assert err < 1e-10


def test_inner(ctx):
    W, D = _case(5)
    assert abs(ctx.inner(W, D) - mf.inner(W, D)) < 1e-12 * max(1.0, abs(mf.inner(W, D)))


EXP_SHAPES = SHAPES + [(12, 5), (9, 6)]   # adds 0 < n - p < p cases


@pytest.mark.parametrize("alpha", [0.0, 0.37, 1.0, 3.0, -2.2])
def test_exponential_retraction(ctx, alpha):
    """eq. retraction (Sec. 2.3) on the GPU against the oracle's QR-based low-rank evaluation."""
    W = [inputs.haar_params(20 + i, [s])[0] for i, s in enumerate(EXP_SHAPES)]
    X = [mf.project(w, d) / np.linalg.norm(d) for w, d in zip(W, inputs.normal_like(21, W))]
    Wo, Xo = ctx.stiefel_retract_exp(W, X, alpha)
    for w, x, wo, xo in zip(W, X, Wo, Xo):
        rw, rx = mf.retract_exp(w, x, alpha)
        wo, xo = to_np(wo), to_np(xo)
        print(f"exp retract {w.shape} alpha={alpha}: W err {rel(wo, rw):.2e} X' err {rel(xo, rx):.2e} "
              f"orth {np.max(np.abs(wo.T @ wo - np.eye(w.shape[1]))):.2e}", flush=True)
        assert np.max(np.abs(wo.T @ wo - np.eye(w.shape[1]))) < 1e-13
        assert rel(wo, rw) < 1e-12
        assert rel(xo, rx) < 1e-12


def test_exponential_transport(ctx):
    """eq. transport (Sec. 2.3): element-wise against the oracle, and inner products are preserved."""
    W = [inputs.haar_params(30 + i, [s])[0] for i, s in enumerate(EXP_SHAPES)]
    X = [mf.project(w, d) for w, d in zip(W, inputs.normal_like(31, W))]
    Y = [mf.project(w, d) for w, d in zip(W, inputs.normal_like(32, W))]
    T = ctx.stiefel_transport_exp(W, X, 0.8, Y)
    for w, x, y, t in zip(W, X, Y, T):
        t = to_np(t)
        assert rel(t, mf.transport_exp(w, x, 0.8, y)) < 1e-12
        assert abs(np.sum(t * t) - np.sum(y * y)) <= 1e-12 * np.sum(y * y)


def test_grassmann_projection_and_geodesic(ctx):
    W = [inputs.haar_params(40 + i, [s])[0] for i, s in enumerate(EXP_SHAPES) if s[0] > s[1]]
    D = inputs.normal_like(41, W)
    G = ctx.grassmann_project(W, D)
    for w, d, g in zip(W, D, G):
        assert rel(to_np(g), mf.grassmann_project(w, d)) < 1e-13
    # a horizontal direction (A = 0): the GPU curve is the oracle's Grassmann geodesic
    X = [mf.grassmann_project(w, d) / np.linalg.norm(d) for w, d in zip(W, D)]
    Wo = ctx.stiefel_retract_exp(W, X, 1.3, tangent=False)
    for w, x, wo in zip(W, X, Wo):
        assert rel(to_np(wo), mf.retract_exp(w, x, 1.3)[0]) < 1e-12


@pytest.mark.parametrize("gamma", [2.0, 20.0])
def test_ev_update(ctx, gamma):
    """Evenbly-Vidal local update (App. A) element-wise against the oracle's SVD polar factor."""
    shapes = [s for s in SHAPES if s[1] > 1]
    W = [inputs.haar_params(50 + i, [s])[0] for i, s in enumerate(shapes)]
    D = inputs.normal_like(51, W)
    rho = [inputs.density_matrix(52 + i, s[1]) + 0.01 * np.eye(s[1]) for i, s in enumerate(shapes)]
    Wo = ctx.ev_update(W, D, rho, gamma)
    for w, d, r, wo in zip(W, D, rho, Wo):
        wo = to_np(wo)
        assert np.max(np.abs(wo.T @ wo - np.eye(w.shape[1]))) < 1e-13
        assert rel(wo, optim.ev_update(w, d, r, gamma)) < 1e-11


@pytest.mark.gpu
def test_ev_update_rank_deficient(ctx):
    """Evenbly-Vidal update when gamma W rho - D has a null space: the result is still an isometry and a polar factor
    of Y = gamma W rho - D (P^T Y = (Y^T Y)^{1/2}, symmetric positive semidefinite), up to the vanishing shift."""
    n, p, gamma = 12, 6, 1.5
    W = inputs.haar_params(60, [(n, p)])[0]
    rho = inputs.density_matrix(61, p) + 0.01 * np.eye(p)
    rng = np.random.default_rng(62)
    Y0 = rng.standard_normal((n, p - 2)) @ rng.standard_normal((p - 2, p))   # rank p - 2
    D = gamma * W @ rho - Y0
    P = to_np(ctx.ev_update([W], [D], [rho], gamma)[0])
    assert np.max(np.abs(P.T @ P - np.eye(p))) < 1e-12
    S = P.T @ Y0
    lam, V = np.linalg.eigh(Y0.T @ Y0)
    absY = (V * np.sqrt(np.clip(lam, 0.0, None))) @ V.T
    assert np.max(np.abs(S - absY)) < 1e-6 * np.linalg.norm(Y0, 2)


def test_empty_factor_lists(ctx):
    """count = 0: the manifold calls do nothing and succeed, and the context keeps working."""
    assert ctx.stiefel_project([], []) == []
    assert ctx.stiefel_retract([], [], 0.5) == ([], [])
    assert ctx.stiefel_transport([], []) == []
    W, D = _case(9)
    G = ctx.stiefel_project(W[:1], D[:1])
    assert rel(to_np(G[0]), mf.project(W[0], D[0])) < 1e-13


def test_zero_tangent(ctx):
    """A zero tangent vector retracts to the point itself with a zero curve tangent, and transports to zero."""
    W, _ = _case(10)
    Z = [np.zeros_like(w) for w in W]
    Wo, Xo = ctx.stiefel_retract(W, Z, 0.8)
    for w, wo, xo in zip(W, Wo, Xo):
        assert np.max(np.abs(to_np(wo) - w)) < 1e-14
        assert not np.any(to_np(xo))
    for t in ctx.stiefel_transport(W, Z):
        assert not np.any(to_np(t))


# the factor sizes of the chi = 24 and chi = 32 binary MERAs: square disentanglers of 576^2 and 1024^2, isometries
# 1024 x 32 and 576 x 24, and a ternary isometry 13824 x 24
FULL = [(576, 576), (1024, 1024), (1024, 32), (576, 24), (13824, 24)]


def _full(seed):
    return [inputs.haar_params(seed + i, [s])[0] for i, s in enumerate(FULL)]


@pytest.mark.parametrize("alpha", [0.37, 2.0])
def test_retract_and_transport_full_size(ctx, alpha):
    W = _full(60)
    X = [mf.project(w, d) / np.linalg.norm(d) for w, d in zip(W, inputs.normal_like(61, W))]
    Wo, Xo = ctx.stiefel_retract(W, X, alpha)
    Wo = [to_np(x) for x in Wo]
    for w, x, wo, xo in zip(W, X, Wo, Xo):
        rw, rx = mf.retract(w, x, alpha)
        xo = to_np(xo)
        orth = np.max(np.abs(wo.T @ wo - np.eye(w.shape[1])))
        print(f"full retract {w.shape} alpha={alpha}: W {rel(wo, rw):.2e} X' {rel(xo, rx):.2e} orth {orth:.2e}",
              flush=True)
        assert orth < 1e-13
        assert rel(wo, rw) < 1e-12
        assert rel(xo, rx) < 1e-10
    Y = [mf.project(w, y) for w, y in zip(W, inputs.normal_like(62, W))]
    T = ctx.stiefel_transport(Wo, Y)
    for wn, y, t in zip(Wo, Y, T):
        assert rel(to_np(t), mf.transport(wn, y)) < 1e-13


def test_preconditioner_full_size_with_warm_eigenbasis(ctx):
    """The preconditioned direction of the two-loop (empty history: d = -P G) for the full-size factors, first with
    a cold Jacobi decomposition of each rho (p = 576, 1024, 32, 24, 24), then with rho changed a little, decomposed
    in the kept eigenbasis (the optimiser's warm start); both against the oracle's eigh-based preconditioner."""
    W = _full(70)
    G = [mf.project(w, d) for w, d in zip(W, inputs.normal_like(71, W))]
    rho1 = [inputs.density_matrix(72 + i, w.shape[1]) + 1e-3 * np.eye(w.shape[1]) / w.shape[1]
            for i, w in enumerate(W)]
    pert = [inputs.symmetric_operator(80 + i, w.shape[1]) for i, w in enumerate(W)]
    rho2 = [r + 1e-3 * np.max(np.abs(r)) * q / np.max(np.abs(q)) for r, q in zip(rho1, pert)]
    lb = ctx.lbfgs(FULL, m=4)
    for tag, rho in (("cold", rho1), ("warm", rho2)):
        d, slope = lb.step(W, G, rho)
        ref = [-mf.precondition(w, g, r) for w, g, r in zip(W, G, rho)]
        for w, a, b in zip(W, d, ref):
            err = rel(to_np(a), b)
            print(f"precondition {tag} {w.shape}: {err:.2e}", flush=True)
            assert err < 1e-10
        assert abs(slope - mf.inner(G, ref)) <= 1e-10 * abs(mf.inner(G, ref))
