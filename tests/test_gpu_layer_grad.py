"""GPU parity of the single-layer derivative mera_layer_grad (combined and split programs) against the oracle's
explicit per-occurrence environments (Sec. 4, eq. mera_derivative), and of its descended and ascended operators."""
import numpy as np
import pytest

from gpu_helpers import rel, require_gpu, to_np
from oracle import mera as om
from oracle import ternary as ot
from paper_2007_03638_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_2007_03638_amd import api
    return api.Context(0)


# (T, chi, d, layer): ragged tiles, a != b, chi > d^2
CASES = [(1, 3, 3, 1), (2, 4, 4, 1), (1, 5, 5, 0), (2, 6, 3, 1), (1, 7, 7, 1)]
PRECS = [("fp64", 1e-12), ("fp32", 2e-6), ("bf16x3", 1e-4)]


@pytest.mark.parametrize("T,chi,d,layer", CASES)
@pytest.mark.parametrize("prec,tol", PRECS)
@pytest.mark.parametrize("split", [False, True])
def test_layer_grad_binary(ctx, T, chi, d, layer, prec, tol, split):
    a, b = om.layer_dims(chi, T, d)[layer]
    u, w = inputs.mera_init(200 + layer, [(a, b)])[0]
    h = inputs.symmetric_operator(21, a ** 3)
    rho = inputs.density_matrix(22, b ** 3)
    Du_ref, Dw_ref = om.layer_environments(h, rho, u, w, a, b)
    Du, Dw, ro, ho = ctx.layer_grad(T, chi, layer, u, w, h, rho, prec=prec, split=split, d=d)
    errs = (rel(to_np(Du), Du_ref), rel(to_np(Dw), Dw_ref), rel(to_np(ro), om.descend(rho, u, w, a, b)))
    print(f"case T={T} chi={chi} d={d} layer={layer} {prec} split={split}: Du {errs[0]:.2e} Dw {errs[1]:.2e} "
          f"rho {errs[2]:.2e}", flush=True)
    assert max(errs) < tol
    if split:
        assert rel(to_np(ho), om.ascend(h, u, w, a, b)) < tol
    else:
        assert ho is None


@pytest.mark.parametrize("T,chi,layer", [(1, 3, 1), (2, 5, 1), (1, 4, 0)])
@pytest.mark.parametrize("prec,tol", PRECS)
def test_layer_grad_ternary(ctx, T, chi, layer, prec, tol):
    a, b = ot.layer_dims(chi, T)[layer]
    u, w = inputs.mera_init(300 + layer, [(a, b)], w_legs=3)[0]
    h = inputs.symmetric_operator(31, a ** 2)
    rho = inputs.density_matrix(32, b ** 2)
    Du_ref, Dw_ref = ot.layer_environments(h, rho, u, w, a, b)
    Du, Dw, ro, _ = ctx.layer_grad(T, chi, layer, u, w, h, rho, prec=prec, d=2, geometry="ternary")
    errs = (rel(to_np(Du), Du_ref), rel(to_np(Dw), Dw_ref), rel(to_np(ro), ot.descend(rho, u, w, a, b)))
    print(f"ternary T={T} chi={chi} layer={layer} {prec}: Du {errs[0]:.2e} Dw {errs[1]:.2e} rho {errs[2]:.2e}",
          flush=True)
    assert max(errs) < tol


def test_layer_grad_argument_checks(ctx):
    from paper_2007_03638_amd import api
    T, chi, d = 1, 3, 3
    a, b = om.layer_dims(chi, T, d)[1]
    u, w = inputs.mera_init(1, [(a, b)])[0]
    h = inputs.symmetric_operator(1, a ** 3)
    rho = inputs.density_matrix(2, b ** 3)
    with pytest.raises(api.MeraError) as e:
        ctx.layer_grad(T, chi, 2, u, w, h, rho, d=d)
    assert e.value.status == -1
    with pytest.raises(api.MeraError) as e:  # split programs: binary geometry only
        ta, tb = ot.layer_dims(3, 1)[1]
        tu, tw = inputs.mera_init(1, [(ta, tb)], w_legs=3)[0]
        ctx.layer_grad(1, 3, 1, tu, tw, inputs.symmetric_operator(1, ta ** 2), inputs.density_matrix(2, tb ** 2),
                       split=True, d=2, geometry="ternary")
    assert e.value.status == -1
    # the context keeps working
    Du, Dw, ro, _ = ctx.layer_grad(T, chi, 1, u, w, h, rho, d=d)
    assert rel(to_np(Du), om.layer_environments(h, rho, u, w, a, b)[0]) < 1e-12
