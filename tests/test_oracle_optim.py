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
