"""GPU parity of the layer maps and of mera_energy_grad against the FP64 oracle (through the C ABI)."""
import numpy as np
import pytest

from gpu_helpers import rel, require_gpu, to_np
from oracle import mera as om
from oracle import model
from paper_2007_03638_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_2007_03638_amd import api
    return api.Context(0)


# (T, chi, d, layer) - several tile sizes and ragged tails: a^2 and chi^3 not multiples of the tiles
LAYER_CASES = [(1, 2, 2, 0), (1, 3, 3, 1), (2, 4, 4, 2), (1, 5, 5, 1), (2, 6, 3, 1), (1, 7, 7, 1), (1, 8, 8, 1)]


@pytest.mark.parametrize("T,chi,d,layer", LAYER_CASES)
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-6), ("bf16x3", 1e-4)])
def test_layer_maps(ctx, T, chi, d, layer, prec, tol):
    dims = om.layer_dims(chi, T, d)
    a, b = dims[layer]
    u, w = inputs.mera_init(100 + layer, [(a, b)])[0]
    h = inputs.symmetric_operator(7, a ** 3)
    rho = inputs.density_matrix(8, b ** 3)
    ref_a = om.ascend(h, u, w, a, b)
    ref_d = om.descend(rho, u, w, a, b)
    got_a = to_np(ctx.ascend(T, chi, layer, u, w, h, prec=prec, d=d))
    got_d = to_np(ctx.descend(T, chi, layer, u, w, rho, prec=prec, d=d))
    print(f"case T={T} chi={chi} d={d} layer={layer} prec={prec}: asc {rel(got_a, ref_a):.2e} "
          f"des {rel(got_d, ref_d):.2e}", flush=True)
    assert rel(got_a, ref_a) < tol
    assert rel(got_d, ref_d) < tol


EG_CASES = [(1, 3, 3, 11), (2, 4, 4, 0), (1, 5, 5, 3), (2, 6, 3, 4)]


@pytest.mark.parametrize("T,chi,d,seed", EG_CASES)
def test_energy_grad_fp64(ctx, T, chi, d, seed):
    dims = om.layer_dims(chi, T, d)
    params = inputs.mera_init(seed, dims)
    h3 = model.tfim_h3(1.0) if d == 4 else inputs.symmetric_operator(seed + 1, d ** 3)
    ref = om.evaluate(params, h3, chi, T, d=d)
    got = ctx.energy_grad(T, chi, [p[0] for p in params], [p[1] for p in params], h3, prec="fp64", d=d,
                          rdms=True)
    print(f"case T={T} chi={chi} d={d}: e {got['energy']!r} ref {ref['energy']!r} "
          f"apps {got['applications_rho']},{got['applications_htilde']}", flush=True)
    assert abs(got["energy"] - ref["energy"]) <= 1e-12 * abs(ref["energy"])
    for t in range(T + 1):
        for k, key in enumerate(("Du", "Dw")):
            err = rel(to_np(got[key][t]), ref["grads"][t][k])
            assert err < 1e-10, (t, key, err)
    rdm_ref = om.preconditioner_rdms(ref["rhos"], params, dims)
    for t in range(T + 1):
        assert rel(to_np(got["rho_u"][t]), rdm_ref[t][0]) < 1e-10
        assert rel(to_np(got["rho_w"][t]), rdm_ref[t][1]) < 1e-10


@pytest.mark.parametrize("prec,etol,gtol", [("fp32", 1e-6, 1e-4), ("bf16x3", 1e-4, 1e-2)])
def test_energy_grad_reduced_precision(ctx, prec, etol, gtol):
    T, chi, d = 2, 4, 4
    dims = om.layer_dims(chi, T, d)
    params = inputs.mera_init(5, dims)
    h3 = model.tfim_h3(1.0)
    ref = om.evaluate(params, h3, chi, T, d=d)
    got = ctx.energy_grad(T, chi, [p[0] for p in params], [p[1] for p in params], h3, prec=prec)
    print(f"{prec}: energy err {abs(got['energy'] - ref['energy']) / abs(ref['energy']):.2e}", flush=True)
    assert abs(got["energy"] - ref["energy"]) <= etol * abs(ref["energy"])
    for t in range(T + 1):
        assert rel(to_np(got["Du"][t]), ref["grads"][t][0]) < gtol
        assert rel(to_np(got["Dw"][t]), ref["grads"][t][1]) < gtol


@pytest.mark.parametrize("T,chi,d,limit", [(2, 4, 4, 1), (2, 6, 3, 1_500_000)])
def test_sliced_programs_match(ctx, T, chi, d, limit):
    """Chunked execution of the layer programs (forced by a small intermediate limit: chunks of 1 leg value, and
    of 2 of 6) matches the oracle."""
    dims = om.layer_dims(chi, T, d)
    params = inputs.mera_init(2, dims)
    h3 = model.tfim_h3(1.0) if d == 4 else inputs.symmetric_operator(9, d ** 3)
    ref = om.evaluate(params, h3, chi, T, d=d)
    a, b = dims[T]
    h = inputs.symmetric_operator(3, a ** 3)
    rho = inputs.density_matrix(4, b ** 3)
    try:
        ctx.set_intermediate_limit(limit)
        got = ctx.energy_grad(T, chi, [p[0] for p in params], [p[1] for p in params], h3, prec="fp64", d=d)
        asc = to_np(ctx.ascend(T, chi, T, params[T][0], params[T][1], h, d=d))
        des = to_np(ctx.descend(T, chi, T, params[T][0], params[T][1], rho, d=d))
    finally:
        ctx.set_intermediate_limit(32 << 30)
    assert abs(got["energy"] - ref["energy"]) <= 1e-12 * abs(ref["energy"])
    for t in range(T + 1):
        assert rel(to_np(got["Du"][t]), ref["grads"][t][0]) < 1e-10
        assert rel(to_np(got["Dw"][t]), ref["grads"][t][1]) < 1e-10
    assert rel(asc, om.ascend(h, params[T][0], params[T][1], a, b)) < 1e-13
    assert rel(des, om.descend(rho, params[T][0], params[T][1], a, b)) < 1e-13


@pytest.mark.parametrize("T,chi,d,seed", [(2, 4, 4, 0), (2, 6, 3, 4)])
def test_krylov_dimensions(ctx, T, chi, d, seed):
    """The fixed point and h~ solved with restarted GMRES of dimension 1, 4 and 24 (the last beyond one fused
    Gram-Schmidt launch of 17 vectors) all give the oracle's energy and gradient. A solve that dimension 24 finishes
    without a restart takes no more superoperator applications than with dimension 4: its iterate minimises the
    residual over a Krylov space that contains every restarted iterate of as many steps."""
    dims = om.layer_dims(chi, T, d)
    params = inputs.mera_init(seed, dims)
    h3 = model.tfim_h3(1.0) if d == 4 else inputs.symmetric_operator(seed + 1, d ** 3)
    ref = om.evaluate(params, h3, chi, T, d=d)
    apps = {}
    for m in (1, 4, 24):
        got = ctx.energy_grad(T, chi, [p[0] for p in params], [p[1] for p in params], h3, prec="fp64", d=d,
                              krylov={"dim": m})
        apps[m] = (got["applications_rho"], got["applications_htilde"])
        print(f"case T={T} chi={chi} d={d} dim={m}: apps {got['applications_rho']},{got['applications_htilde']}",
              flush=True)
        assert abs(got["energy"] - ref["energy"]) <= 1e-12 * abs(ref["energy"])
        for t in range(T + 1):
            assert rel(to_np(got["Du"][t]), ref["grads"][t][0]) < 1e-10
            assert rel(to_np(got["Dw"][t]), ref["grads"][t][1]) < 1e-10
    for s in range(2):
        if apps[24][s] <= 25:  # one cycle: the initial residual plus at most 24 Arnoldi steps
            assert apps[24][s] <= apps[4][s]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_degenerate_hamiltonians(ctx, prec, tol):
    """h = 0 gives energy 0 and a zero gradient (the h~ solve then has a zero right-hand side); h = c 1 gives
    energy c per blocked site, since every layer map sends the identity to the identity, and no Riemannian
    gradient, since the energy is then constant on the manifold."""
    T, chi, d = 2, 4, 4
    dims = om.layer_dims(chi, T, d)
    params = inputs.mera_init(6, dims)
    u, w = [p[0] for p in params], [p[1] for p in params]
    zero = ctx.energy_grad(T, chi, u, w, np.zeros((d ** 3, d ** 3)), prec=prec)
    assert zero["energy"] == 0.0
    for t in range(T + 1):
        assert not np.any(to_np(zero["Du"][t])) and not np.any(to_np(zero["Dw"][t]))
    c = 1.7
    const = ctx.energy_grad(T, chi, u, w, c * np.eye(d ** 3), prec=prec)
    print(f"{prec}: energy of c 1 minus c: {const['energy'] - c:.2e}", flush=True)
    assert abs(const["energy"] - c) <= tol * c
    for t in range(T + 1):
        for v, key in ((u[t], "Du"), (w[t], "Dw")):
            D = to_np(const[key][t])
            G = D - v @ (v.T @ D + D.T @ v) / 2
            assert np.max(np.abs(G)) <= tol * c * max(1.0, np.max(np.abs(D))), (t, key)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_product_state_special_case(ctx, prec, tol):
    """u = 1 and w|i> = |i>|0> on every layer drive each site to |0>: the fixed point is |000><000| and the TFIM
    (h = 1, two spins per blocked site) energy is <000|h3|000> = -2 per blocked site."""
    chi, T = 4, 1
    u = np.eye(chi * chi)
    w = np.zeros((chi, chi, chi))
    for i in range(chi):
        w[i, 0, i] = 1.0
    w = w.reshape(chi * chi, chi)
    got = ctx.energy_grad(T, chi, [u, u], [w, w], model.tfim_h3(1.0), prec=prec)
    assert abs(got["energy"] + 2.0) <= 2.0 * tol
