"""GPU parity of the ternary MERA (two-site operators, the paper's benchmark geometry) against the oracle."""
import numpy as np
import pytest

from gpu_helpers import rel, require_gpu, to_np
from oracle import model
from oracle import optim
from oracle import ternary as tm
from paper_2007_03638_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_2007_03638_amd import api
    return api.Context(0)


def _params(seed, dims):
    return inputs.mera_init(seed, dims, w_legs=3)


def test_two_site_models(ctx):
    from paper_2007_03638_amd import api
    assert np.max(np.abs(api.h2_tfim(0.7) - tm.tfim_h2(0.7))) == 0.0
    assert np.max(np.abs(api.h2_xxz(0.3) - tm.xxz_h2(0.3))) < 1e-15


@pytest.mark.parametrize("T,chi,layer", [(1, 4, 0), (1, 4, 1), (1, 6, 0), (2, 12, 1), (2, 12, 2)])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 1e-5), ("bf16x3", 1e-3)])
def test_layer_maps(ctx, T, chi, layer, prec, tol):
    """Ascending and descending maps (three diagrams averaged) on random symmetric operators."""
    dims = tm.layer_dims(chi, T)
    a, b = dims[layer]
    u, w = _params(3, dims)[layer]
    h = inputs.symmetric_operator(4, a * a)
    rho = inputs.density_matrix(5, b * b)
    asc = to_np(ctx.ascend(T, chi, layer, u, w, h, prec=prec, d=2, geometry="ternary"))
    des = to_np(ctx.descend(T, chi, layer, u, w, rho, prec=prec, d=2, geometry="ternary"))
    assert rel(asc, tm.ascend(h, u, w, a, b)) < tol
    assert rel(des, tm.descend(rho, u, w, a, b)) < tol


@pytest.mark.parametrize("T,chi,seed", [(1, 4, 0), (1, 6, 1), (2, 9, 2)])
def test_energy_grad_fp64(ctx, T, chi, seed):
    dims = tm.layer_dims(chi, T)
    params = _params(seed, dims)
    h2 = tm.tfim_h2(1.0) if seed != 1 else inputs.symmetric_operator(7, 4)
    ref = tm.evaluate(params, h2, chi, T)
    got = ctx.energy_grad(T, chi, [p[0] for p in params], [p[1] for p in params], h2, prec="fp64", d=2,
                          rdms=True, geometry="ternary")
    print(f"ternary T={T} chi={chi}: e {got['energy']!r} ref {ref['energy']!r} "
          f"apps {got['applications_rho']},{got['applications_htilde']}", flush=True)
    assert abs(got["energy"] - ref["energy"]) <= 1e-12 * abs(ref["energy"])
    for t in range(T + 1):
        for k, key in enumerate(("Du", "Dw")):
            err = rel(to_np(got[key][t]), ref["grads"][t][k])
            assert err < 1e-10, (t, key, err)
    rdm_ref = tm.preconditioner_rdms(ref["rhos"], params, dims)
    for t in range(T + 1):
        assert rel(to_np(got["rho_u"][t]), rdm_ref[t][0]) < 1e-10
        assert rel(to_np(got["rho_w"][t]), rdm_ref[t][1]) < 1e-10


def test_energy_grad_fp32(ctx):
    T, chi = 1, 6
    dims = tm.layer_dims(chi, T)
    params = _params(4, dims)
    h2 = tm.tfim_h2(1.0)
    ref = tm.evaluate(params, h2, chi, T)
    got = ctx.energy_grad(T, chi, [p[0] for p in params], [p[1] for p in params], h2, prec="fp32", d=2,
                          geometry="ternary")
    # a random state's TFIM energy is small (0.027 here); FP32 rounding scales with the size of the local term, so
    # the 1e-6 relative bound is taken against max(|e|, ||h2||_2) (||h2||_2 = 2.2 for the TFIM term at h = 1)
    scale = max(abs(ref["energy"]), np.linalg.norm(h2, 2))
    print(f"fp32 energy error {abs(got['energy'] - ref['energy']):.2e} (scale {scale:.3f})", flush=True)
    assert abs(got["energy"] - ref["energy"]) <= 1e-6 * scale
    for t in range(T + 1):
        assert rel(to_np(got["Du"][t]), ref["grads"][t][0]) < 1e-4
        assert rel(to_np(got["Dw"][t]), ref["grads"][t][1]) < 1e-4


def test_ternary_optimiser_trajectory(ctx):
    """Preconditioned L-BFGS on the ternary geometry against the oracle driver (FP64, first iterations)."""
    chi, T, iters = 4, 1, 6
    dims = tm.layer_dims(chi, T)
    W0 = [m for pair in _params(6, dims) for m in pair]
    h2 = tm.tfim_h2(1.0)
    prob = optim.Problem(h2, chi, T, d=2, geometry="ternary")
    log = []
    _, f_ref, _, _ = optim.optimize(W0, prob, max_iter=iters, log=log)
    got = ctx.run_optimize(T, chi, h2, W0, prec="fp64", max_iter=iters, grad_tol=0.0, log_cap=64, want_final=True,
                           d=2, geometry="ternary")
    print("gpu", [(r["iter"], r["evals"], r["energy"]) for r in got["log"]], flush=True)
    print("ref", [(r["iter"], r["evals"], r["energy"]) for r in log], flush=True)
    for a, b in zip(got["log"], log):
        assert a["evals"] == b["evals"]
        assert abs(a["energy"] - b["energy"]) <= 1e-10 * abs(b["energy"])
    assert abs(got["energy"] - f_ref) <= 1e-10 * abs(f_ref)
    assert got["energy"] > model.tfim_exact_energy_per_spin(1.0)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_degenerate_hamiltonians(ctx, prec, tol):
    """Ternary geometry: h = 0 gives energy 0 and a zero gradient; h = c 1 gives energy c and no Riemannian
    gradient (every layer map sends the identity to the identity)."""
    T, chi = 1, 6
    dims = tm.layer_dims(chi, T)
    params = _params(8, dims)
    u, w = [p[0] for p in params], [p[1] for p in params]
    zero = ctx.energy_grad(T, chi, u, w, np.zeros((4, 4)), prec=prec, d=2, geometry="ternary")
    assert zero["energy"] == 0.0
    for t in range(T + 1):
        assert not np.any(to_np(zero["Du"][t])) and not np.any(to_np(zero["Dw"][t]))
    c = 0.6
    const = ctx.energy_grad(T, chi, u, w, c * np.eye(4), prec=prec, d=2, geometry="ternary")
    assert abs(const["energy"] - c) <= tol * c
    for t in range(T + 1):
        for v, key in ((u[t], "Du"), (w[t], "Dw")):
            D = to_np(const[key][t])
            G = D - v @ (v.T @ D + D.T @ v) / 2
            assert np.max(np.abs(G)) <= tol * c * max(1.0, np.max(np.abs(D))), (t, key)
