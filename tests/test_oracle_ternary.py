"""Pins of the oracle's ternary MERA (two-site operators): brute force on an explicit ring, map identities, the
product-state special case, the variational bound and finite differences of the gradient."""
import numpy as np
import pytest

from oracle import finite, manifold as mf, model, ternary as tm
from paper_2007_03638_amd import inputs


def _layer(seed, a, b):
    u, w = inputs.haar_params(seed, [(a * a, a * a), (a ** 3, b)])
    return u, w


@pytest.mark.parametrize("a,b", [(2, 2), (2, 3)])
def test_descending_diagrams_equal_ring_rdms(a, b):
    """Brute force: lower a random state of a 3-site ring through one ternary layer (explicit 9-site state); the
    two-site density matrices on the physical pairs (3k, 3k+1), (3k+1, 3k+2), (3k+2, 3k+3) are D_L, D_C, D_R of
    the two-site density matrices of the upper ring."""
    rng = np.random.default_rng(a * 10 + b)
    u, w = _layer(3, a, b)
    top = rng.standard_normal((b, b, b))
    top /= np.linalg.norm(top)
    low = tm.apply_layer(top, u, w, a, b)
    assert abs(np.linalg.norm(low) - 1.0) < 1e-13
    rho_top = finite.rdm(top, [0, 1])
    assert np.allclose(finite.rdm(low, [3, 4]), tm.descend_one('L', rho_top, u, w, a, b), atol=1e-13)
    assert np.allclose(finite.rdm(low, [1, 2]), tm.descend_one('C', rho_top, u, w, a, b), atol=1e-13)
    assert np.allclose(finite.rdm(low, [2, 3]), tm.descend_one('R', rho_top, u, w, a, b), atol=1e-13)


@pytest.mark.parametrize("a,b", [(2, 2), (2, 3)])
def test_preconditioner_rdms_equal_ring_rdms(a, b):
    """Brute force for the density matrices of the preconditioner (Sec. 4): on an explicit 3-site upper ring,
    rho_w is the mean of the one-site RDMs of the two sites of rho_top, and rho_u is the two-site RDM on the inner
    legs (2, 3) of w_0 (x) w_1 after the isometries alone (disentanglers set to the identity)."""
    rng = np.random.default_rng(a * 7 + b)
    u, w = _layer(11, a, b)
    top = rng.standard_normal((b, b, b))
    top /= np.linalg.norm(top)
    rho_top = finite.rdm(top, [0, 1])
    _, w_si = inputs.haar_params(12, [(b * b, b * b), (b ** 3, b)])
    out = tm.preconditioner_rdms([None, rho_top], [(u, w), (None, w_si)], [(a, b), (b, b)])
    rho_u, rho_w = out[0]
    assert np.allclose(rho_w, 0.5 * (finite.rdm(top, [0]) + finite.rdm(top, [1])), atol=1e-13)
    low_w = tm.apply_layer(top, np.eye(a * a), w, a, b)
    assert np.allclose(rho_u, finite.rdm(low_w, [2, 3]), atol=1e-13)


def test_map_identities():
    a, b = 3, 4
    u, w = _layer(5, a, b)
    h = inputs.symmetric_operator(6, a * a)
    rho = inputs.density_matrix(7, b * b)
    for pos in 'LCR':
        assert np.allclose(tm.ascend_one(pos, np.eye(a * a), u, w, a, b), np.eye(b * b), atol=1e-13)
        assert abs(np.trace(tm.descend_one(pos, rho, u, w, a, b)) - 1.0) < 1e-13
        lhs = np.sum(tm.ascend_one(pos, h, u, w, a, b) * rho)
        rhs = np.sum(h * tm.descend_one(pos, rho, u, w, a, b))
        assert abs(lhs - rhs) < 1e-13


def test_product_state_fixed_point():
    """u = 1 and w|i> = |i 0 0>: the scale-invariant state is the product |0 0 ...>, e = <00|h2|00> = -hx."""
    chi = 2
    u = np.eye(4)
    w = np.zeros((8, 2))
    w[0, 0] = 1.0
    w[4, 1] = 1.0
    rho = tm.fixed_point_rho(u, w, chi)
    ref = np.zeros((4, 4))
    ref[0, 0] = 1.0
    assert np.allclose(rho, ref, atol=1e-12)
    assert abs(np.sum(tm.tfim_h2(1.0) * rho) - (-1.0)) < 1e-12


def test_h2_sums_to_the_chain():
    """Summed over the bonds of a ring, the two-site terms give the TFIM and XXZ chains."""
    for h2, (pair, field) in [(tm.tfim_h2(0.7), model.tfim_pair_and_field(0.7)),
                              (tm.xxz_h2(0.4), model.xxz_pair_and_field(0.4))]:
        n = 6
        H = np.zeros((2 ** n, 2 ** n))
        for s in range(n):
            ops = [np.eye(2)] * n
            # place h2 on (s, s+1) via a permutation of the dense operator
            full = np.kron(h2, np.eye(2 ** (n - 2))).reshape([2] * (2 * n))
            perm = list(range(n))
            perm[0], perm[1] = s, (s + 1) % n
            rest = [k for k in range(n) if k not in (s, (s + 1) % n)]
            perm[2:] = rest
            inv = np.argsort(perm)
            full = np.transpose(full, list(inv) + [n + k for k in inv])
            H += full.reshape(2 ** n, 2 ** n)
        assert np.allclose(H, model.spin_ring_hamiltonian(n, pair, field), atol=1e-12)


def test_energy_bound_and_gradient_fd():
    chi, T = 4, 1
    dims = tm.layer_dims(chi, T)
    assert dims == [(2, 4), (4, 4)]
    params = [tuple(inputs.haar_params(20 + t, [(a * a, a * a), (a ** 3, b)])) for t, (a, b) in enumerate(dims)]
    h2 = tm.tfim_h2(1.0)
    ev = tm.evaluate(params, h2, chi, T)
    assert ev['energy'] > model.tfim_exact_energy_per_spin(1.0)
    # transition layer: Euclidean FD of the polynomial extension
    rng = np.random.default_rng(9)
    for which in (0, 1):
        Dv = ev['grads'][0][which]
        E = rng.standard_normal(Dv.shape)
        eps = 1e-5
        vals = []
        for s in (1, -1):
            p2 = [list(x) for x in params]
            p2[0][which] = p2[0][which] + s * eps * E
            vals.append(tm.energy_only([tuple(x) for x in p2], h2, chi, T))
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(fd - np.sum(Dv * E)) < 1e-8
    # scale-invariant layer: Riemannian FD along a tangent (polar retraction), Richardson
    Wl = [params[T][0], params[T][1]]
    G = [mf.project(Wl[i], ev['grads'][T][i]) for i in range(2)]
    X = [mf.project(Wl[i], rng.standard_normal(Wl[i].shape)) for i in range(2)]

    def f(alpha):
        Wn = [mf.retract(Wl[i], X[i], alpha)[0] for i in range(2)]
        return tm.energy_only(list(params[:T]) + [(Wn[0], Wn[1])], h2, chi, T)
    d1 = (f(3e-4) - f(-3e-4)) / 6e-4      # Richardson: the error falls as eps^4 (4e-11 here)
    d2 = (f(6e-4) - f(-6e-4)) / 1.2e-3
    fd = (4 * d1 - d2) / 3
    assert abs(fd - mf.inner(G, X)) < 1e-9 * max(1.0, abs(fd))


def test_ternary_lbfgs_run_with_preconditioner():
    """The paper's benchmark geometry optimised with the preconditioned L-BFGS: monotone and above the bound; the
    preconditioner metrics are unit-trace PSD matrices of the right sizes."""
    from oracle import optim
    chi, T = 4, 1
    dims = tm.layer_dims(chi, T)
    W0 = [m for t, (a, b) in enumerate(dims) for m in inputs.haar_params(30 + t, [(a * a, a * a), (a ** 3, b)])]
    prob = optim.Problem(tm.tfim_h2(1.0), chi, T, d=2, geometry='ternary')
    _, _, rv = prob.evaluate(W0)
    for r, w in zip(rv, W0):
        assert r.shape == (w.shape[1], w.shape[1])
        assert abs(np.trace(r) - 1.0) < 1e-12 and np.min(np.linalg.eigvalsh(r)) > -1e-12
    log = []
    W, f, gnorm, info = optim.optimize(W0, prob, max_iter=10, log=log)
    energies = [r['energy'] for r in log] + [f]
    assert all(b <= a + 1e-12 for a, b in zip(energies, energies[1:]))
    assert energies[-1] < energies[0] - 0.1
    assert f > model.tfim_exact_energy_per_spin(1.0)
