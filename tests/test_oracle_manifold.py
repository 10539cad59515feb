"""Pins of the oracle's Stiefel projection, polar retraction, transport and preconditioner."""
import numpy as np
import pytest
import scipy.linalg

from oracle import manifold as mf
from paper_2007_03638_amd import inputs

SHAPES = [(6, 6), (9, 4), (16, 3), (5, 1)]


def _point_and_tangent(seed, n, p):
    W = inputs.haar_params(seed, [(n, p)])[0]
    D = inputs.normal_like(seed + 1, [W])[0]
    return W, D


@pytest.mark.parametrize("n,p", SHAPES)
def test_projection_properties(n, p):
    W, D = _point_and_tangent(1, n, p)
    G = mf.project(W, D)
    S = W.T @ G
    assert np.max(np.abs(S + S.T)) < 1e-14                    # tangent: W^T G skew
    assert np.max(np.abs(mf.project(W, G) - G)) < 1e-14       # idempotent
    X = mf.project(W, inputs.normal_like(7, [W])[0])
    assert abs(np.sum(G * X) - np.sum(D * X)) < 1e-13         # g(G, X) = Tr[D^T X] for tangent X
    Sym = inputs.symmetric_operator(3, p)
    assert np.max(np.abs(mf.project(W, W @ Sym))) < 1e-14      # D = W S, S symmetric -> G = 0


@pytest.mark.parametrize("n,p", SHAPES)
def test_polar_retraction(n, p):
    W, D = _point_and_tangent(2, n, p)
    X = mf.project(W, D)
    for alpha in (0.0, 1e-3, 0.3, 2.0):
        Wn, Xp = mf.retract(W, X, alpha)
        assert np.max(np.abs(Wn.T @ Wn - np.eye(p))) < 1e-13
        # closed form for an exact tangent: (W + aX)(1 + a^2 X^T X)^{-1/2}
        lam, V = np.linalg.eigh(np.eye(p) + alpha ** 2 * X.T @ X)
        ref = (W + alpha * X) @ V @ np.diag(lam ** -0.5) @ V.T
        assert np.max(np.abs(Wn - ref)) < 1e-12
        h = 1e-5
        fd = (mf.retract(W, X, alpha + h)[0] - mf.retract(W, X, alpha - h)[0]) / (2 * h)
        assert np.max(np.abs(fd - Xp)) < 1e-8
    W0, X0 = mf.retract(W, X, 0.0)
    assert np.max(np.abs(W0 - W)) < 1e-14
    assert np.max(np.abs(X0 - X)) < 1e-13


@pytest.mark.parametrize("n,p", SHAPES)
def test_projection_transport(n, p):
    W, D = _point_and_tangent(3, n, p)
    X = mf.project(W, D)
    Wn, _ = mf.retract(W, X, 0.7)
    Y = mf.project(W, inputs.normal_like(9, [W])[0])
    T = mf.transport(Wn, Y)
    S = Wn.T @ T
    assert np.max(np.abs(S + S.T)) < 1e-13
    assert np.max(np.abs(mf.transport(Wn, T) - T)) < 1e-13
    assert np.max(np.abs(mf.transport(W, Y) - Y)) < 1e-13


@pytest.mark.parametrize("n,p", SHAPES)
def test_preconditioner_defining_identity(n, p):
    W, D = _point_and_tangent(4, n, p)
    X = mf.project(W, D)
    rho = inputs.density_matrix(5, p) + 0.05 * np.eye(p)
    Xt = mf.precondition(W, X, rho, delta=0.0)
    St = W.T @ Xt
    assert np.max(np.abs(St + St.T)) < 1e-12                  # result is tangent
    for s in range(3):
        Y = mf.project(W, inputs.normal_like(20 + s, [W])[0])
        assert abs(np.sum(Y * (Xt @ rho)) - np.sum(Y * X)) < 1e-11   # eq. preconditioner
    # positive: g(X, X~) > 0, and with delta the eigenbasis closed form f = sqrt(lam^2 + delta^2) holds
    Xd = mf.precondition(W, X, rho, delta=0.3)
    assert np.sum(X * Xd) > 0
    lam, V = np.linalg.eigh(rho)
    rho_reg = V @ np.diag(np.sqrt(lam ** 2 + 0.09)) @ V.T
    assert np.max(np.abs(mf.precondition(W, X, rho_reg, delta=0.0) - Xd)) < 1e-11


def _full_q(W, X):
    """Q_X of eq. retraction built in full (n x n) from an explicit orthonormal complement W_perp."""
    Wp = scipy.linalg.null_space(W.T)
    A = W.T @ X
    B = Wp.T @ X
    Ub = np.hstack([W, Wp])
    Mb = np.block([[A, -B.T], [B, np.zeros((B.shape[0], B.shape[0]))]])
    return Ub @ Mb @ Ub.T


@pytest.mark.parametrize("n,p", [(12, 5), (9, 6), (7, 7), (16, 4)])
def test_exp_retraction_and_transport_equal_full_exponential(n, p):
    """Brute force of eqs. retraction and transport: the low-rank evaluation equals exp(alpha Q_X) applied to W and
    to Y with the n x n matrix exponential (covers n - p >= p, 0 < n - p < p and square W)."""
    rng = np.random.default_rng(n * 10 + p)
    W = np.linalg.qr(rng.standard_normal((n, p)))[0]
    X = mf.project(W, rng.standard_normal((n, p)))
    Y = mf.project(W, rng.standard_normal((n, p)))
    for alpha in (0.3, -1.1, 2.0):
        E = scipy.linalg.expm(alpha * _full_q(W, X))
        Wn, Xp = mf.retract_exp(W, X, alpha)
        assert np.allclose(Wn, E @ W, atol=1e-12)
        assert np.allclose(Xp, E @ X, atol=1e-12)
        assert np.allclose(mf.transport_exp(W, X, alpha, Y), E @ Y, atol=1e-12)


def test_exp_retraction_properties():
    rng = np.random.default_rng(3)
    W = np.linalg.qr(rng.standard_normal((14, 5)))[0]
    X = mf.project(W, rng.standard_normal((14, 5)))
    assert np.allclose(mf.retract_exp(W, X, 0.0)[0], W, atol=1e-14)
    for alpha in (0.0, 0.4, 1.7):
        Wn, Xp = mf.retract_exp(W, X, alpha)
        assert np.max(np.abs(Wn.T @ Wn - np.eye(5))) < 1e-13
        eps = 1e-5
        fd = (mf.retract_exp(W, X, alpha + eps)[0] - mf.retract_exp(W, X, alpha - eps)[0]) / (2 * eps)
        assert np.allclose(fd, Xp, atol=1e-8)
    # transport: a metric connection (the paper notes it preserves inner products) mapping tangents to tangents
    Y1 = mf.project(W, rng.standard_normal((14, 5)))
    Y2 = mf.project(W, rng.standard_normal((14, 5)))
    Wn = mf.retract_exp(W, X, 0.9)[0]
    T1, T2 = mf.transport_exp(W, X, 0.9, Y1), mf.transport_exp(W, X, 0.9, Y2)
    assert abs(mf.inner([T1], [T2]) - mf.inner([Y1], [Y2])) < 1e-12
    S = Wn.T @ T1
    assert np.max(np.abs(S + S.T)) < 1e-12


def test_exp_retraction_grassmann_geodesic():
    """With A = W^T X = 0 the curve is the Grassmann geodesic W V cos(S alpha) V^T + U sin(S alpha) V^T for the thin
    SVD X = U S V^T (Edelman, Arias and Smith 1998, the closed form the paper's footnote refers to)."""
    rng = np.random.default_rng(4)
    W = np.linalg.qr(rng.standard_normal((15, 4)))[0]
    X = mf.grassmann_project(W, rng.standard_normal((15, 4)))
    assert np.max(np.abs(W.T @ X)) < 1e-13
    U, s, Vt = np.linalg.svd(X, full_matrices=False)
    for alpha in (0.5, 1.3):
        geo = W @ Vt.T @ np.diag(np.cos(s * alpha)) @ Vt + U @ np.diag(np.sin(s * alpha)) @ Vt
        assert np.allclose(mf.retract_exp(W, X, alpha)[0], geo, atol=1e-12)
