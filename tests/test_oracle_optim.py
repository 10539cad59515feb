"""Pins of the oracle's L-BFGS two-loop, line search and optimisation driver."""
import math

import numpy as np
import pytest

from oracle import manifold as mf
from oracle import mera, model, optim
from paper_2007_03638_amd import inputs


def _explicit_bfgs_inverse(S, Y, gamma, n):
    """Textbook inverse-Hessian recursion H <- (I - r s y^T) H (I - r y s^T) + r s s^T from H0 = gamma I."""
    H = gamma * np.eye(n)
    for s, y in zip(S, Y):
        r = 1.0 / (s @ y)
        V = np.eye(n) - r * np.outer(y, s)
        H = V.T @ H @ V + r * np.outer(s, s)
    return H


def test_two_loop_equals_explicit_bfgs_on_quadratic():
    rng = np.random.default_rng(0)
    n = 7
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    hist = optim.LBFGSHistory(m=4)
    x = rng.standard_normal(n)
    S, Y = [], []
    for _ in range(6):
        step = rng.standard_normal(n)
        s, y = step, A @ step
        assert hist.push([s[:, None]], [y[:, None]])
        S.append(s)
        Y.append(y)
    S, Y = S[-4:], Y[-4:]
    g = A @ x
    d = hist.direction([g[:, None]], lambda v: [t.copy() for t in v])[0][:, 0]
    gamma = (S[-1] @ Y[-1]) / (Y[-1] @ Y[-1])
    ref = -_explicit_bfgs_inverse(S, Y, gamma, n) @ g
    assert np.max(np.abs(d - ref)) < 1e-12
    # secant equation for the newest pair: H y_k = s_k
    Hy = -hist.direction([Y[-1][:, None]], lambda v: [t.copy() for t in v])[0][:, 0]
    assert np.max(np.abs(Hy - S[-1])) < 1e-12


def test_two_loop_empty_history_is_preconditioned_gradient():
    hist = optim.LBFGSHistory(m=8)
    g = [np.arange(6.0).reshape(3, 2)]
    d = hist.direction(g, lambda v: [2.0 * t for t in v])
    assert np.max(np.abs(d[0] + 2.0 * g[0])) == 0.0


def test_history_skips_non_positive_curvature():
    hist = optim.LBFGSHistory(m=2)
    assert not hist.push([np.ones((2, 1))], [-np.ones((2, 1))])
    assert hist.S == []


def test_line_search_wolfe_on_quartic():
    f = lambda a: (a - 3.0) ** 4 - 2.0 * a
    df = lambda a: 4.0 * (a - 3.0) ** 3 - 2.0
    ok, alpha, fa, dfa, _, n = optim.line_search(lambda a: (f(a), df(a), None), f(0.0), df(0.0))
    assert ok
    f0, d0 = f(0.0), df(0.0)
    wolfe = fa <= f0 + 1e-4 * alpha * d0 and dfa >= 0.9 * d0
    approx = (2e-4 - 1.0) * d0 >= dfa >= 0.9 * d0 and fa <= f0 + 1e-6 * abs(f0)
    assert wolfe or approx
    assert n <= 10


def test_line_search_expands_and_bisects():
    # minimum far beyond alpha = 1 forces expansion; a steep wall forces bracketing
    ok, alpha, *_ = optim.line_search(lambda a: ((a - 50.0) ** 2, 2 * (a - 50.0), None), 2500.0, -100.0)
    assert ok and alpha > 1.0
    ok, alpha, *_ = optim.line_search(lambda a: ((a - 0.01) ** 2, 2 * (a - 0.01), None), 1e-4, -0.02)
    assert ok and alpha < 0.1


def test_optimizer_small_run_decreases_energy_above_bound():
    chi, T = 4, 2
    dims = mera.layer_dims(chi, T)
    W0 = [m for pair in inputs.mera_init(0, dims) for m in pair]
    prob = optim.Problem(model.tfim_h3(1.0), chi, T)
    log = []
    W, f, gnorm, info = optim.optimize(W0, prob, m=8, max_iter=12, log=log)
    energies = [r['energy'] for r in log] + [f]
    assert all(b <= a + 1e-12 for a, b in zip(energies, energies[1:]))
    assert f / 2 > model.tfim_exact_energy_per_spin(1.0)
    assert energies[-1] < energies[0] - 0.1
    assert log[-1]['gnorm'] < log[0]['gnorm']
    for w in W:
        assert np.max(np.abs(w.T @ w - np.eye(w.shape[1]))) < 1e-13


def _pcg_with_hz(A, b, M, n_steps):
    """Nonlinear CG with the oracle's Hager-Zhang coefficient and exact line searches on the quadratic
    f(x) = x^T A x / 2 - b^T x (Euclidean, identity transport), preconditioner M."""
    x = np.zeros(len(b))
    g = A @ x - b
    d = -(M @ g)
    grads = [np.linalg.norm(g)]
    for _ in range(n_steps):
        alpha = -(g @ d) / (d @ A @ d)
        x = x + alpha * d
        g_new = A @ x - b
        y = g_new - g
        beta = optim.hz_beta([g_new], [M @ g_new], [y], [M @ y], [d], np.linalg.norm(g))
        d = -(M @ g_new) + beta * d
        g = g_new
        grads.append(np.linalg.norm(g))
    return x, grads


@pytest.mark.parametrize("precond", [False, True])
def test_hz_cg_terminates_on_quadratic(precond):
    """With exact line searches <d, g_new> = 0 and the Hager-Zhang coefficient reduces to the Hestenes-Stiefel one,
    so (preconditioned) nonlinear CG is linear CG: it solves an n-dimensional SPD quadratic in n steps."""
    rng = np.random.default_rng(5)
    n = 7
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    A = Q @ np.diag(np.linspace(1.0, 30.0, n)) @ Q.T
    b = rng.standard_normal(n)
    if precond:
        R = rng.standard_normal((n, n))
        M = R @ R.T / n + 0.5 * np.eye(n)   # an SPD preconditioner unrelated to A
    else:
        M = np.eye(n)
    x, grads = _pcg_with_hz(A, b, M, n)
    assert np.allclose(x, np.linalg.solve(A, b), atol=1e-9)
    assert grads[-1] < 1e-9 * grads[0]
    assert grads[n - 2] > 1e-6 * grads[0]   # not earlier: M A has n distinct eigenvalues


def test_hz_beta_sufficient_descent():
    """Hager-Zhang (2005): with <d, y> != 0 the untruncated coefficient gives <g, -g + beta d> <= -7/8 |g|^2 for
    any g, d, y."""
    rng = np.random.default_rng(6)
    for _ in range(200):
        g, d, y = (rng.standard_normal(9) for _ in range(3))
        beta = optim.hz_beta([g], [g], [y], [y], [d], 1.0, truncate=False)
        assert g @ (-g + beta * d) <= -0.875 * (g @ g) + 1e-12


def test_hz_beta_truncation():
    """The truncated coefficient is max(beta, -1/(|d| min(0.01, |g_old|)))."""
    rng = np.random.default_rng(7)
    g, d, y = (rng.standard_normal(5) for _ in range(3))
    raw = optim.hz_beta([g], [g], [y], [y], [d], 1.0, truncate=False)
    floor = -1.0 / (np.linalg.norm(d) * 0.01)
    assert optim.hz_beta([g], [g], [y], [y], [d], 1.0) == max(raw, floor)
    assert optim.hz_beta([g], [g], [y], [y], [np.zeros(5)], 1.0) == 0.0


def test_cg_small_run_decreases_energy_above_bound():
    chi, T = 4, 2
    dims = mera.layer_dims(chi, T)
    W0 = [m for pair in inputs.mera_init(0, dims) for m in pair]
    prob = optim.Problem(model.tfim_h3(1.0), chi, T)
    log = []
    W, f, gnorm, info = optim.optimize_cg(W0, prob, max_iter=12, log=log)
    energies = [r['energy'] for r in log] + [f]
    assert all(b <= a + 1e-12 for a, b in zip(energies, energies[1:]))
    assert f / 2 > model.tfim_exact_energy_per_spin(1.0)
    assert energies[-1] < energies[0] - 0.1
    for w in W:
        assert np.max(np.abs(w.T @ w - np.eye(w.shape[1]))) < 1e-13


@pytest.mark.parametrize("method,grassmann", [("lbfgs", False), ("lbfgs", True), ("cg", False)])
def test_exponential_retraction_runs(method, grassmann):
    """The paper's own configuration (exponential retraction and transport, Sec. 2.3; Grassmann isometries, Sec. 4):
    monotone, above the bound, isometric, and the Grassmann gradients are horizontal (W^T G = 0)."""
    chi, T = 4, 2
    dims = mera.layer_dims(chi, T)
    W0 = [m for pair in inputs.mera_init(2, dims) for m in pair]
    prob = optim.Problem(model.tfim_h3(1.0), chi, T, grassmann_w=grassmann)
    log = []
    run = optim.optimize if method == "lbfgs" else optim.optimize_cg
    W, f, gnorm, info = run(W0, prob, max_iter=10, log=log, retraction="exp")
    energies = [r['energy'] for r in log] + [f]
    assert all(b <= a + 1e-12 for a, b in zip(energies, energies[1:]))
    assert energies[-1] < energies[0] - 0.1
    assert f / 2 > model.tfim_exact_energy_per_spin(1.0)
    for w in W:
        assert np.max(np.abs(w.T @ w - np.eye(w.shape[1]))) < 1e-12
    if grassmann:
        _, G, _ = prob.evaluate(W)
        for i in range(1, len(W), 2):
            assert np.max(np.abs(W[i].T @ G[i])) < 1e-12


def test_ev_update_fixed_point_and_small_step_limit():
    """App. A: W is a fixed point when D = W P (P symmetric, gamma rho - P positive definite); for large gamma the
    update is preconditioned gradient descent, W' = W - G~/gamma + O(1/gamma^2), with G~ the gradient G = P_W(D)
    preconditioned by rho (eq. preconditioner_solution with delta = 0)."""
    rng = np.random.default_rng(8)
    n, p = 14, 5
    W = inputs.haar_params(8, [(n, p)])[0]
    rho = inputs.density_matrix(9, p) + 0.05 * np.eye(p)
    R = rng.standard_normal((p, p))
    P = 5.0 * rho - (R @ R.T + 0.1 * np.eye(p))             # gamma rho - P symmetric positive definite
    assert np.allclose(optim.ev_update(W, W @ P, rho, 5.0), W, atol=1e-13)
    G = mf.project(W, rng.standard_normal((n, p)))          # a pure gradient, W^T G skew
    Gt = mf.precondition(W, G, rho, delta=0.0)
    errs = []
    for gamma in (1e3, 2e3, 4e3):
        errs.append(np.linalg.norm(optim.ev_update(W, G, rho, gamma) - (W - Gt / gamma)))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5   # second order in 1/gamma


def test_ev_sweeps_decrease_energy():
    chi, T = 4, 2
    dims = mera.layer_dims(chi, T)
    W0 = [m for pair in inputs.mera_init(0, dims) for m in pair]
    prob = optim.Problem(model.tfim_h3(1.0), chi, T)
    log = []
    W, f, gnorm, info = optim.optimize_ev(W0, prob, gamma=20.0, max_iter=3, log=log)
    energies = [r['energy'] for r in log] + [f]
    assert all(b <= a + 1e-12 for a, b in zip(energies, energies[1:]))
    assert f / 2 > model.tfim_exact_energy_per_spin(1.0)
    assert info['evals'] == 1 + 3 * 2 * (T + 1)
    for w in W:
        assert np.max(np.abs(w.T @ w - np.eye(w.shape[1]))) < 1e-13
