"""Pins of the oracle's Stiefel projection, polar retraction, transport and preconditioner."""
import numpy as np
import pytest

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
