"""GPU parity of the L-BFGS two-loop and pair update against the oracle's history (through the C ABI)."""
import numpy as np
import pytest

from gpu_helpers import rel, require_gpu, to_np
from oracle import manifold as mf
from oracle import optim
from paper_2007_03638_amd import inputs

pytestmark = pytest.mark.gpu

SHAPES = [(16, 16), (16, 4), (64, 8), (9, 3)]


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_2007_03638_amd import api
    return api.Context(0)


@pytest.mark.parametrize("precondition", [False, True])
def test_two_loop_sequence_matches_oracle(ctx, precondition):
    m = 3
    lb = ctx.lbfgs(SHAPES, m=m)
    hist = optim.LBFGSHistory(m)
    W = [inputs.haar_params(i, [s])[0] for i, s in enumerate(SHAPES)]
    rho = [inputs.density_matrix(30 + i, s[1]) + 0.02 * np.eye(s[1]) for i, s in enumerate(SHAPES)]
    G = [mf.project(w, d) for w, d in zip(W, inputs.normal_like(9, W))]
    for k in range(6):
        P = (lambda X, _W=W: [mf.precondition(w, x, r) for w, x, r in zip(_W, X, rho)]) if precondition else \
            (lambda X: [x.copy() for x in X])
        d_ref = hist.direction(G, P)
        slope_ref = mf.inner(G, d_ref)
        if not slope_ref < 0:
            hist.reset()
            d_ref = [-x for x in P(G)]
            slope_ref = mf.inner(G, d_ref)
        d, slope = ctx.lbfgs(SHAPES, m=m).step(W, G, rho if precondition else None) if False else \
            lb.step(W, G, rho if precondition else None)
        print(f"step {k}: history {lb.size()} / {len(hist.S)}, slope {slope:.6e} ref {slope_ref:.6e}", flush=True)
        assert lb.size() == len(hist.S)
        assert abs(slope - slope_ref) <= 1e-10 * abs(slope_ref)
        for a, b in zip(d, d_ref):
            assert rel(to_np(a), b) < 1e-10
        alpha = 0.3 + 0.1 * k
        Wn = [mf.retract(w, x, alpha)[0] for w, x in zip(W, d_ref)]
        Gn = [mf.project(w, x) for w, x in zip(Wn, inputs.normal_like(100 + k, Wn))]
        s = [mf.transport(w, alpha * x) for w, x in zip(Wn, d_ref)]
        y = [gn - mf.transport(w, g) for w, gn, g in zip(Wn, Gn, G)]
        hist.transport(lambda X, _Wn=Wn: [mf.transport(w, x) for w, x in zip(_Wn, X)])
        acc_ref = hist.push(s, y)
        acc = lb.push(Wn, d_ref, alpha, G, Gn)
        assert acc == acc_ref
        W, G = Wn, Gn
