"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's test harness.

This module holds no arithmetic of the method: it only draws random numbers. Isometries are Haar-distributed
(QR of an n x p standard-normal matrix with the sign of R's diagonal folded into Q, Mezzadri 2007), drawn in the
order the shapes are given, from numpy's default_rng(seed).standard_normal.
"""
import numpy as np


def haar_isometry(rng, n, p):
    """n x p matrix with orthonormal columns, Haar-distributed."""
    g = rng.standard_normal((n, p))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def haar_params(seed, shapes):
    """One Haar isometry per (n, p) in `shapes`, in order, from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return [haar_isometry(rng, n, p) for (n, p) in shapes]


def mera_shapes(dims, w_legs=2):
    """[(n_u, p_u), (n_w, p_w)] per layer for the (a, b) layer dimensions: u is a^2 x a^2, w is a^w_legs x b
    (w_legs = 2 for the binary geometry, 3 for the ternary one)."""
    out = []
    for a, b in dims:
        out.append((a * a, a * a))
        out.append((a ** w_legs, b))
    return out


def mera_init(seed, dims, w_legs=2):
    """Haar initial tensors in the order u_1, w_1, ..., u_T, w_T, u_s, w_s, grouped as [(u, w)] per layer."""
    mats = haar_params(seed, mera_shapes(dims, w_legs))
    return [(mats[2 * i], mats[2 * i + 1]) for i in range(len(dims))]


def normal_like(seed, mats):
    """Standard-normal matrices with the shapes of `mats` (e.g. raw directions before any projection)."""
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(m.shape) for m in mats]


def symmetric_operator(seed, dim):
    """Random real symmetric dim x dim matrix (a generic 3-site operator)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((dim, dim))
    return 0.5 * (g + g.T)


def density_matrix(seed, dim):
    """Random real symmetric positive matrix with unit trace (a generic 3-site density matrix)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((dim, dim))
    r = g @ g.T
    return r / np.trace(r)


def one_site_factors(seed, n, nterms):
    """nterms triples of n x n standard-normal matrices, the one-site factors of a product-operator sum."""
    rng = np.random.default_rng(seed)
    return [tuple(rng.standard_normal((n, n)) for _ in range(3)) for _ in range(nterms)]


def near_identity_isometries(seed, shapes, eps):
    """Isometries near the first p columns of the n x n identity: the Q factor (sign-fixed as above) of
    E + eps G, E = [I_p; 0], G standard normal, one per (n, p) in order from default_rng(seed). With a small eps the
    MERA stays close to a product state, whose energy is far from zero (unlike a Haar-random MERA's)."""
    rng = np.random.default_rng(seed)
    out = []
    for n, p in shapes:
        g = np.eye(n)[:, :p] + eps * rng.standard_normal((n, p))
        q, r = np.linalg.qr(g)
        out.append(q * np.sign(np.diag(r))[None, :])
    return out


def mera_init_near_identity(seed, dims, eps, w_legs=2):
    """near_identity_isometries grouped as [(u, w)] per layer, in the order of mera_init."""
    mats = near_identity_isometries(seed, mera_shapes(dims, w_legs), eps)
    return [(mats[2 * i], mats[2 * i + 1]) for i in range(len(dims))]
