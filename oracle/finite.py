"""Explicit state vector of a small finite periodic binary MERA (oracle; test infrastructure only).

Used to pin the layer maps by brute force: the state of a ring is built top-down, isometries first (w_j sends
site j of the upper ring to sites (2j, 2j+1) below), then the disentanglers on the pairs (2j+1, 2j+2), wrapping
around the ring. Reduced density matrices are taken directly from the state vector.
"""
import numpy as np


def apply_layer(psi, u, w, a, b, isometries_only=False):
    """Lower a ring state by one layer. psi has n legs of dim b (leg k = site k); returns 2n legs of dim a.

    With isometries_only the disentanglers are not applied (the state between the two rows of the layer).
    """
    n = psi.ndim
    Wt = w.reshape(a, a, b)
    U = u.reshape(a, a, a, a)
    for j in range(n):
        # replace leg j (now at position 2j, since earlier legs were doubled) by two legs of dim a
        pos = 2 * j
        psi = np.tensordot(psi, Wt, axes=([pos], [2]))           # new legs appended at the end
        psi = np.moveaxis(psi, [psi.ndim - 2, psi.ndim - 1], [pos, pos + 1])
    if isometries_only:
        return psi
    m = 2 * n
    for j in range(n):
        s1, s2 = (2 * j + 1) % m, (2 * j + 2) % m
        # u[bl, br, tl, tr]: bottom legs on sites (s1, s2), top legs contracted with the state
        psi = np.tensordot(U, psi, axes=([2, 3], [s1, s2]))      # legs: bl, br, rest...
        rest = [k for k in range(m) if k not in (s1, s2)]
        order = [0] * m
        order[s1], order[s2] = 0, 1
        for idx, k in enumerate(rest):
            order[k] = idx + 2
        psi = np.transpose(psi, order)
    return psi


def rdm(psi, sites):
    """Reduced density matrix on the listed sites (in that order), rows = kets, as a matrix."""
    n = psi.ndim
    others = [k for k in range(n) if k not in sites]
    x = np.transpose(psi, list(sites) + others)
    dk = int(np.prod([psi.shape[s] for s in sites]))
    x = x.reshape(dk, -1)
    return x @ x.T


def ring_energy(psi, h3):
    """<psi| sum_s h3(s, s+1, s+2) |psi> / n on a periodic ring, from the dense state."""
    n = psi.ndim
    total = 0.0
    for s in range(n):
        total += np.sum(h3 * rdm(psi, [s, (s + 1) % n, (s + 2) % n]))
    return total / n
