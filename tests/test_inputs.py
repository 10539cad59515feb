"""The seeded input generators shared by the tests, the benchmark and the oracle's harness: deterministic per seed,
with the structure their users rely on (isometries, the per-layer order and shapes, symmetric operators, density
matrices), and Haar statistics for the isometries."""
import numpy as np

from paper_2007_03638_amd import inputs


def test_isometries_orthonormal_and_deterministic():
    shapes = [(16, 16), (16, 4), (256, 24), (5, 1), (81, 9)]
    a = inputs.haar_params(3, shapes)
    b = inputs.haar_params(3, shapes)
    c = inputs.haar_params(4, shapes)
    for x, y, z, (n, p) in zip(a, b, c, shapes):
        assert x.shape == (n, p)
        assert np.array_equal(x, y)
        assert not np.array_equal(x, z)
        assert np.max(np.abs(x.T @ x - np.eye(p))) < 1e-14


def test_sign_convention_makes_the_map_from_the_gaussian_draw_unique():
    # with the sign of R's diagonal folded into Q, Q^T G is upper triangular with a positive diagonal
    rng = np.random.default_rng(11)
    g = np.random.default_rng(11).standard_normal((12, 5))
    q = inputs.haar_isometry(rng, 12, 5)
    r = q.T @ g
    assert np.max(np.abs(np.tril(r, -1))) < 1e-13
    assert np.all(np.diag(r) > 0)
    assert np.max(np.abs(q @ r - g)) < 1e-13


def test_haar_statistics_of_unit_vectors():
    # columns of Haar isometries are uniform on the sphere: E[x_1] = 0, E[x_1^2] = 1/n, E[x_1^4] = 3/(n(n+2))
    n, draws = 6, 20000
    x = np.array([inputs.haar_params(s, [(n, 1)])[0][0, 0] for s in range(draws)])
    assert abs(x.mean()) < 4 * np.sqrt(1.0 / n / draws)
    assert abs((x ** 2).mean() - 1.0 / n) < 0.01
    assert abs((x ** 4).mean() - 3.0 / (n * (n + 2))) < 0.005


def test_mera_init_order_and_shapes():
    dims = [(4, 16), (16, 24), (24, 24), (24, 24)]
    params = inputs.mera_init(2, dims)
    flat = inputs.haar_params(2, inputs.mera_shapes(dims))
    for t, (a, b) in enumerate(dims):
        u, w = params[t]
        assert u.shape == (a * a, a * a) and w.shape == (a * a, b)
        assert np.array_equal(u, flat[2 * t]) and np.array_equal(w, flat[2 * t + 1])
    ternary = inputs.mera_init(2, [(2, 8), (8, 8)], w_legs=3)
    assert ternary[0][1].shape == (8, 8) and ternary[1][1].shape == (512, 8)


def test_operators_and_density_matrices():
    h = inputs.symmetric_operator(5, 64)
    assert np.array_equal(h, h.T)
    rho = inputs.density_matrix(6, 64)
    assert np.max(np.abs(rho - rho.T)) < 1e-15
    assert abs(np.trace(rho) - 1.0) < 1e-14
    assert np.min(np.linalg.eigvalsh(rho)) > -1e-15
    d = inputs.normal_like(7, [h, rho[:8]])
    assert [x.shape for x in d] == [(64, 64), (8, 64)]
    assert np.array_equal(d[0], inputs.normal_like(7, [h])[0])
