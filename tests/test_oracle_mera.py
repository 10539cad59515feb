"""Pins of the oracle's binary-MERA layer maps, fixed point, energy and Euclidean gradient."""
import numpy as np
import pytest

from oracle import finite, manifold, mera, model
from paper_2007_03638_amd import inputs


def _random_layer(seed, a, b):
    return inputs.mera_init(seed, [(a, b)])[0]


@pytest.mark.parametrize("a,b", [(2, 2), (3, 3), (2, 3), (3, 2)])
def test_layer_maps_unital_adjoint_trace_preserving(a, b):
    u, w = _random_layer(1, a, b)
    h = inputs.symmetric_operator(2, a ** 3)
    rho = inputs.density_matrix(3, b ** 3)
    for net in (mera._NET_L, mera._NET_R):
        assert np.max(np.abs(mera.ascend_one(net, np.eye(a ** 3), u, w, a, b) - np.eye(b ** 3))) < 1e-13
        lhs = np.sum(mera.ascend_one(net, h, u, w, a, b) * rho)
        rhs = np.sum(h * mera.descend_one(net, rho, u, w, a, b))
        assert abs(lhs - rhs) < 1e-13
        assert abs(np.trace(mera.descend_one(net, rho, u, w, a, b)) - 1.0) < 1e-13
        dr = mera.descend_one(net, rho, u, w, a, b)
        assert np.min(np.linalg.eigvalsh(0.5 * (dr + dr.T))) > -1e-13  # positivity is kept


def _ring_state(seed, d, chi):
    """8-site ring, three layers: 8 -> 4 -> 2 -> 1, with a top dimension of 1."""
    rng_params = inputs.haar_params(seed, [(d * d, d * d), (d * d, chi), (chi * chi, chi * chi), (chi * chi, chi),
                                           (chi * chi, chi * chi), (chi * chi, 1)])
    u1, w1, u2, w2, u3, w3 = rng_params
    top = np.ones((1,))
    psi2 = finite.apply_layer(top, u3, w3, chi, 1)            # 2 sites of dim chi
    psi4 = finite.apply_layer(psi2, u2, w2, chi, chi)        # 4 sites of dim chi
    psi8 = finite.apply_layer(psi4, u1, w1, d, chi)          # 8 sites of dim d
    return psi8, psi4, (u1, w1)


def test_finite_ring_state_normalised():
    psi8, psi4, _ = _ring_state(0, 2, 2)
    assert abs(np.sum(psi8 * psi8) - 1.0) < 1e-13
    assert abs(np.sum(psi4 * psi4) - 1.0) < 1e-13


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_descending_diagrams_match_brute_force_rdms(seed):
    d = chi = 2
    psi8, psi4, (u1, w1) = _ring_state(seed, d, chi)
    for j in range(4):
        top = finite.rdm(psi4, [(j - 1) % 4, j, (j + 1) % 4])
        bottom = finite.rdm(psi8, [2 * j, 2 * j + 1, (2 * j + 2) % 8])
        assert np.max(np.abs(mera.descend_one(mera._NET_L, top, u1, w1, d, chi) - bottom)) < 1e-14
        top = finite.rdm(psi4, [j, (j + 1) % 4, (j + 2) % 4])
        bottom = finite.rdm(psi8, [2 * j + 1, (2 * j + 2) % 8, (2 * j + 3) % 8])
        assert np.max(np.abs(mera.descend_one(mera._NET_R, top, u1, w1, d, chi) - bottom)) < 1e-14


def test_brute_force_ring_energy():
    # unblocked TFIM 3-site term on spins: h3 = (hb (x) 1 + 1 (x) hb)/2 with hb = -XX - (Z1 + Z2)/2
    hb = -np.kron(model.PX, model.PX) - 0.5 * (np.kron(model.PZ, model.I2) + np.kron(model.I2, model.PZ))
    h3 = 0.5 * (np.kron(hb, np.eye(2)) + np.kron(np.eye(2), hb))
    d = chi = 2
    psi8, psi4, (u1, w1) = _ring_state(5, d, chi)
    H8 = model.spin_ring_hamiltonian(8, *model.tfim_pair_and_field(1.0))
    v = psi8.reshape(-1)
    e_state = v @ H8 @ v / 8
    rho1 = sum(finite.rdm(psi4, [j, (j + 1) % 4, (j + 2) % 4]) for j in range(4)) / 4
    e_maps = np.sum(h3 * mera.descend(rho1, u1, w1, d, chi))
    e_asc = np.sum(mera.ascend(h3, u1, w1, d, chi) * rho1)
    assert abs(e_state - e_maps) < 1e-14
    assert abs(e_state - e_asc) < 1e-14
    assert abs(finite.ring_energy(psi8, h3) - e_state) < 1e-14


def _tfim_mera(seed, chi, T, d=4):
    dims = mera.layer_dims(chi, T, d)
    return inputs.mera_init(seed, dims), dims


def test_fixed_point_properties():
    chi = 3
    (u, w), = inputs.mera_init(4, [(chi, chi)])
    rho = mera.fixed_point_rho(u, w, chi)
    assert abs(np.trace(rho) - 1.0) < 1e-14
    assert np.max(np.abs(rho - rho.T)) == 0.0
    assert np.min(np.linalg.eigvalsh(rho)) > -1e-13
    assert np.max(np.abs(mera.descend(rho, u, w, chi, chi) - rho)) < 1e-13


def test_fixed_point_product_state_special_case():
    # u = 1 and w|i> = |i>|0>: every site is driven to |0>, rho_s = |000><000| and, for TFIM h = 1 with two
    # spins per blocked site, e = <000|h3|000> = -2 per blocked site (-1 per spin).
    chi = 4
    u = np.eye(chi * chi)
    w = np.zeros((chi, chi, chi))
    for i in range(chi):
        w[i, 0, i] = 1.0
    w = w.reshape(chi * chi, chi)
    rho = mera.fixed_point_rho(u, w, chi)
    ref = np.zeros((chi ** 3, chi ** 3))
    ref[0, 0] = 1.0
    assert np.max(np.abs(rho - ref)) < 1e-12
    params = [(u, w), (u, w)]
    e = mera.energy_only(params, model.tfim_h3(1.0), chi, 1, d=4)
    assert abs(e + 2.0) < 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_variational_bound_and_two_routes(seed):
    params, dims = _tfim_mera(seed, 4, 2)
    h3 = model.tfim_h3(1.0)
    e_top = mera.energy_only(params, h3, 4, 2)
    e_bot = mera.energy_bottom(params, h3, 4, 2)
    assert abs(e_top - e_bot) < 1e-13
    assert e_top / 2 > model.tfim_exact_energy_per_spin(1.0)
    hx = mera.energy_only(params, model.xxz_h3(0.5), 4, 2)
    assert hx / 2 > model.xxz_exact_energy_per_spin(0.5)


def test_htilde_series_equals_solve():
    chi = 2
    (u, w), = inputs.mera_init(7, [(chi, chi)])
    rho = mera.fixed_point_rho(u, w, chi)
    hT = inputs.symmetric_operator(8, chi ** 3)
    s = mera.htilde(hT, rho, u, w, chi, method='series')
    g = mera.htilde(hT, rho, u, w, chi, method='solve')
    assert np.max(np.abs(s - g)) < 1e-11
    assert abs(np.sum(g * rho)) < 1e-13
    # defining relation: h~ - A(h~) + Tr[h~ rho] 1 = h_T - e 1
    e = np.sum(hT * rho)
    lhs = g - mera.ascend(g, u, w, chi, chi) + np.sum(g * rho) * np.eye(chi ** 3)
    assert np.max(np.abs(lhs - (hT - e * np.eye(chi ** 3)))) < 1e-11


def test_energy_invariances():
    chi, T = 4, 2
    params, dims = _tfim_mera(11, chi, T)
    h3 = model.tfim_h3(1.0)
    e0 = mera.energy_only(params, h3, chi, T)
    # shift by a constant
    assert abs(mera.energy_only(params, h3 + 0.37 * np.eye(64), chi, T) - (e0 + 0.37)) < 1e-13
    # sign flips of single tensors
    for t in range(T + 1):
        for k in range(2):
            p2 = [list(p) for p in params]
            p2[t][k] = -p2[t][k]
            assert abs(mera.energy_only([tuple(p) for p in p2], h3, chi, T) - e0) < 1e-13
    # gauge on the top leg of w_1 absorbed by u_2
    O = inputs.haar_isometry(np.random.default_rng(3), chi, chi)
    p2 = [list(p) for p in params]
    p2[0][1] = params[0][1] @ O
    p2[1][0] = np.kron(O, O).T @ params[1][0]
    assert abs(mera.energy_only([tuple(p) for p in p2], h3, chi, T) - e0) < 1e-13
    # gauge of the scale-invariant leg: w_T, w_s -> w O, u_s -> (O (x) O)^T u_s
    p3 = [list(p) for p in params]
    p3[T - 1][1] = params[T - 1][1] @ O
    p3[T][1] = params[T][1] @ O
    p3[T][0] = np.kron(O, O).T @ params[T][0]
    assert abs(mera.energy_only([tuple(p) for p in p3], h3, chi, T) - e0) < 1e-12


def test_transition_gradient_finite_differences():
    chi, T = 3, 2
    dims = mera.layer_dims(chi, T, d=3)
    params = inputs.mera_init(21, dims)
    h3 = inputs.symmetric_operator(22, 27)
    ev = mera.evaluate(params, h3, chi, T, d=3)
    eps = 1e-5
    for t in range(T):
        for k in range(2):
            X = inputs.normal_like(100 + 10 * t + k, [params[t][k]])[0]
            def e_at(s):
                p2 = [list(p) for p in params]
                p2[t][k] = params[t][k] + s * X
                return mera.energy_only([tuple(p) for p in p2], h3, chi, T, d=3)
            fd = (e_at(eps) - e_at(-eps)) / (2 * eps)
            an = np.sum(ev['grads'][t][k] * X)
            assert abs(fd - an) < 1e-8 * max(1.0, abs(an))


def test_scale_invariant_riemannian_gradient_finite_differences():
    chi, T = 3, 1
    dims = mera.layer_dims(chi, T, d=3)
    params = inputs.mera_init(31, dims)
    h3 = inputs.symmetric_operator(32, 27)
    ev = mera.evaluate(params, h3, chi, T, d=3)
    for k in range(2):
        W = params[T][k]
        G = manifold.project(W, ev['grads'][T][k])
        X = manifold.project(W, inputs.normal_like(40 + k, [W])[0])
        def e_at(s):
            p2 = [list(p) for p in params]
            p2[T][k] = manifold.retract(W, X, s)[0]
            return mera.energy_only([tuple(p) for p in p2], h3, chi, T, d=3)
        def cd(h):
            return (e_at(h) - e_at(-h)) / (2 * h)
        h = 1e-3
        rich = (4 * cd(h / 2) - cd(h)) / 3   # Richardson: removes the O(h^2) term
        an = np.sum(G * X)
        assert abs(rich - an) < 1e-9 * max(1.0, abs(an))


def test_gradient_shift_invariance():
    chi, T = 3, 1
    dims = mera.layer_dims(chi, T, d=3)
    params = inputs.mera_init(41, dims)
    h3 = inputs.symmetric_operator(42, 27)
    g1 = mera.evaluate(params, h3, chi, T, d=3)['grads']
    g2 = mera.evaluate(params, h3 + 2.5 * np.eye(27), chi, T, d=3)['grads']
    for t in range(T + 1):
        for k in range(2):
            W = params[t][k]
            assert np.max(np.abs(manifold.project(W, g1[t][k]) - manifold.project(W, g2[t][k]))) < 1e-11


def test_preconditioner_rdms_match_brute_force():
    # rho_w of layer 1 is the one-site density matrix of the 4-site ring above it; rho_u of layer 1 is the
    # two-site density matrix, on the pair a disentangler acts on, of the state between w's and u's.
    d = chi = 2
    psi8, psi4, (u1, w1) = _ring_state(9, d, chi)
    rho1 = sum(finite.rdm(psi4, [j, (j + 1) % 4, (j + 2) % 4]) for j in range(4)) / 4
    rhos = [None, rho1]        # bottom of layer 1 (unused), top of layer 1 (in the slot of rho_s, T = 1)
    dims = [(d, chi), (chi, chi)]
    params = [(u1, w1), (u1, w1)]
    rho_u, rho_w = mera.preconditioner_rdms(rhos, params, dims)[0]
    one_site = sum(finite.rdm(psi4, [j]) for j in range(4)) / 4
    assert np.max(np.abs(rho_w - one_site)) < 1e-14
    mid = finite.apply_layer(psi4, u1, w1, d, chi, isometries_only=True)
    two_site = sum(finite.rdm(mid, [2 * j + 1, (2 * j + 2) % 8]) for j in range(4)) / 4
    assert np.max(np.abs(rho_u - two_site)) < 1e-14


@pytest.mark.parametrize("a,b", [(3, 3), (4, 2), (2, 3)])
def test_ascend_element_matches_full_map(a, b):
    """`ascend_element` (the sampler used for outputs at large bond dimension) against the whole `ascend_one`
    output, at every index."""
    u, w = _random_layer(7, a, b)
    h = inputs.symmetric_operator(8, a ** 3)
    for side, net in (("L", mera._NET_L), ("R", mera._NET_R)):
        full = mera.ascend_one(net, h, u, w, a, b).reshape((b,) * 6)
        for idx in np.ndindex(*(b,) * 6):
            assert abs(mera.ascend_element(side, h, u, w, a, b, idx) - full[idx]) < 1e-13, (side, idx)


def _factor_terms(rng, n, nterms):
    """Sum of products of one-site matrices, closed under transposition so that the operator is symmetric while
    no factor is: A (x) B (x) C + A^T (x) B^T (x) C^T for each random (A, B, C)."""
    out = []
    for _ in range(nterms):
        f = [rng.standard_normal((n, n)) for _ in range(3)]
        out.append(tuple(f))
        out.append(tuple(x.T for x in f))
    return out


@pytest.mark.parametrize("a,b", [(3, 3), (4, 2), (2, 4)])
def test_product_operator_forms_match_dense(a, b):
    """The product-operator forms of the layer maps and environments equal the dense ones on the same operators."""
    rng = np.random.default_rng(11)
    u, w = _random_layer(12, a, b)
    ht = _factor_terms(rng, a, 1)
    rt = _factor_terms(rng, b, 1)
    h = mera.product_operator(ht)
    rho = mera.product_operator(rt)
    assert np.max(np.abs(h - h.T)) < 1e-12 and np.max(np.abs(rho - rho.T)) < 1e-12
    A = mera.ascend_product(ht, u, w, a, b)
    assert np.max(np.abs(A - mera.ascend(h, u, w, a, b))) < 1e-12 * max(1.0, np.max(np.abs(A)))
    D = mera.descend_product(rt, u, w, a, b)
    assert np.max(np.abs(D - mera.descend(rho, u, w, a, b))) < 1e-12 * max(1.0, np.max(np.abs(D)))
    Du, Dw = mera.layer_environments_product(ht, rt, u, w, a, b)
    Du2, Dw2 = mera.layer_environments(h, rho, u, w, a, b)
    scale = max(np.max(np.abs(Du2)), np.max(np.abs(Dw2)))
    assert np.max(np.abs(Du - Du2)) < 1e-12 * scale
    assert np.max(np.abs(Dw - Dw2)) < 1e-12 * scale


@pytest.mark.parametrize("name", ["eval_chi12_T2.npz", "eval_chi12_T2_near.npz"])
def test_stored_chi12_evaluation(name):
    """tests/golden/eval_chi12_T2*.npz (written by tests/golden/make_chi12.py from the oracle): the energy agrees
    with the one obtained by full descent stored beside it, lies above the exact infinite-chain energy (-4/pi per
    spin), and the stored gradients have the layer shapes."""
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", name))
    assert abs(float(g["energy"]) - float(g["energy_bottom"])) < 1e-13
    assert float(g["energy"]) / 2 > model.tfim_exact_energy_per_spin(1.0)
    for t, (a, b) in enumerate(mera.layer_dims(int(g["chi"]), int(g["T"]))):
        assert g[f"Du{t}"].shape == (a * a, a * a) and g[f"Dw{t}"].shape == (a * a, b)
        assert g[f"rho_u{t}"].shape == (a * a, a * a) and g[f"rho_w{t}"].shape == (b, b)
