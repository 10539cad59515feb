"""GPU parity of the Stiefel operations and the preconditioner against the oracle (through the C ABI)."""
import numpy as np
import pytest

from gpu_helpers import rel, require_gpu, to_np
from oracle import manifold as mf
from paper_2007_03638_amd import inputs

pytestmark = pytest.mark.gpu

# shapes of MERA factors: square disentanglers and tall isometries, several tile sizes and ragged tails
SHAPES = [(16, 16), (16, 4), (256, 24), (576, 24), (81, 9), (5, 1), (144, 144), (400, 20)]


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
