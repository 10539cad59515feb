"""Infinite scale-invariant ternary MERA with two-site operators (oracle; test infrastructure only).

The paper's own benchmark geometry (Sec. 4): every isometry w maps three sites of the layer below to one site above,
disentanglers u act on the two sites where neighbouring isometries meet, and the Hamiltonian is a sum of two-site
terms on unblocked spins (d = 2). Plain numpy/scipy, FP64.

Conventions of this module (readings; the paper's diagrams are not reproduced in the text):
  * w[x, y, z, t]: bottom legs x, y, z (rows, a^3), top leg t (column, b). Isometry w_k covers the sites
    (3k, 3k+1, 3k+2) of the layer below and maps to site k above.
  * u[bl, br, tl, tr]: bottom legs (rows, a^2), top legs (columns, a^2); u_k acts on (3k+2, 3k+3).
  * Operators h[ab, AB] (a^2 x a^2, kets lowercase). A two-site operator on (s, s+1) rises to a two-site operator:
      L: (3k, 3k+1)   -> top (k-1, k), through u_{k-1}, w_{k-1}, w_k
      C: (3k+1, 3k+2) -> top (k, k+1), through u_k, w_k, w_{k+1}
      R: (3k+2, 3k+3) -> top (k, k+1), through u_k, w_k, w_{k+1}
    and A = (A_L + A_C + A_R)/3 (the translation average over the three positions).
  * Layer dimensions: a_1 = d, b_t = min(chi, a_t^3); the scale-invariant layer has a = b = chi.
  * Scale-invariant fixed point, h~ (the deflated series) and the derivative through them exactly as for the binary
    geometry (App. B): rho_s = D_s(rho_s), e = Tr[h_T rho_s], <h~|(1 - A') = <h_T - e 1|.
"""
import numpy as np
from scipy.sparse.linalg import LinearOperator, eigs, gmres

from .mera import _ein

# operand order: h, u, u*, wl, wl*, wr, wr*
_NETS = {
    'L': ['abAB', 'eafc', 'eAFC', 'xyfp', 'xyFP', 'cbzq', 'CBzQ'],
    'C': ['abAB', 'becf', 'BeCF', 'xacp', 'xACP', 'fyzq', 'FyzQ'],
    'R': ['abAB', 'abcd', 'ABCD', 'xycp', 'xyCP', 'dzvq', 'DzvQ'],
}
_TOP = 'pqPQ'
_KINDS = ['h', 'u', 'u', 'wl', 'wl', 'wr', 'wr']


def tfim_h2(hx=1.0):
    """Two-site TFIM term -X X - hx (Z 1 + 1 Z)/2 on unblocked spins (each site's field shared by its two bonds)."""
    X = np.array([[0.0, 1.0], [1.0, 0.0]])
    Z = np.diag([1.0, -1.0])
    I = np.eye(2)
    return -np.kron(X, X) - 0.5 * hx * (np.kron(Z, I) + np.kron(I, Z))


def xxz_h2(delta):
    """Two-site XXZ term XX + YY + delta ZZ (Pauli units; Y Y = -(iY)(iY) is real)."""
    X = np.array([[0.0, 1.0], [1.0, 0.0]])
    iY = np.array([[0.0, 1.0], [-1.0, 0.0]])
    Z = np.diag([1.0, -1.0])
    return np.kron(X, X) - np.kron(iY, iY) + delta * np.kron(Z, Z)


def layer_dims(chi, T, d=2):
    """[(a, b)] for transition layers 1..T and the scale-invariant layer."""
    dims = []
    a = d
    for _ in range(T):
        b = min(chi, a ** 3)
        dims.append((a, b))
        a = b
    if a != chi:
        raise ValueError("the scale-invariant layer needs b_T = chi (choose T larger)")
    dims.append((chi, chi))
    return dims


def _operands(u, w, a, b):
    U = u.reshape(a, a, a, a)
    Wt = w.reshape(a, a, a, b)
    return [U, U, Wt, Wt, Wt, Wt]


def ascend_one(pos, h, u, w, a, b):
    net = _NETS[pos]
    ops = [h.reshape(a, a, a, a)] + _operands(u, w, a, b)
    return _ein(','.join(net) + '->' + _TOP, *ops).reshape(b * b, b * b)


def descend_one(pos, rho, u, w, a, b):
    net = _NETS[pos]
    ops = _operands(u, w, a, b) + [rho.reshape(b, b, b, b)]
    return _ein(','.join(net[1:] + [_TOP]) + '->' + net[0], *ops).reshape(a * a, a * a)


def ascend(h, u, w, a, b):
    return sum(ascend_one(p, h, u, w, a, b) for p in 'LCR') / 3.0


def descend(rho, u, w, a, b):
    return sum(descend_one(p, rho, u, w, a, b) for p in 'LCR') / 3.0


def _sym(m):
    return 0.5 * (m + m.T)


def fixed_point_rho(u, w, chi, tol=0.0):
    """Scale-invariant two-site density matrix: eigenvector of the descending map with eigenvalue 1 (App. B)."""
    n = chi ** 4

    def apply(x):
        return descend(x.reshape(chi * chi, chi * chi), u, w, chi, chi).reshape(-1)
    if n <= 256:
        M = np.stack([apply(e) for e in np.eye(n)], axis=1)
        vals, vecs = np.linalg.eig(M)
        v = vecs[:, np.argmax(np.abs(vals))]
    else:
        op = LinearOperator((n, n), matvec=apply, dtype=np.float64)
        vals, vecs = eigs(op, k=1, which='LM', v0=np.eye(chi * chi).reshape(-1), tol=tol, ncv=min(n, 20),
                          maxiter=10000)
        v = vecs[:, 0]
    rho = np.real(v).reshape(chi * chi, chi * chi)
    return _sym(rho / np.trace(rho))


def htilde(hT, rho, u, w, chi, rtol=1e-14):
    """<h~|(1 - A') = <h_T - e 1| with A' = A - |rho><1| (App. B), by a library GMRES."""
    one = np.eye(chi * chi)
    e = np.sum(hT * rho)
    hp = hT - e * one

    def mv(x):
        X = x.reshape(chi * chi, chi * chi)
        return (X - (ascend(X, u, w, chi, chi) - np.sum(X * rho) * one)).reshape(-1)
    n = chi ** 4
    op = LinearOperator((n, n), matvec=mv, dtype=np.float64)
    x, info = gmres(op, hp.reshape(-1), x0=hp.reshape(-1), rtol=rtol, atol=0.0, restart=min(n, 60), maxiter=2000)
    if info != 0:
        raise RuntimeError(f"GMRES for h~ did not converge (info={info})")
    return x.reshape(chi * chi, chi * chi)


def layer_environments(h, rho, u, w, a, b):
    """Euclidean derivative of Tr[A(h) rho] w.r.t. u and w of one layer: one explicit environment per occurrence
    (ket and bra copies of u, of the left and of the right isometry, in each of the three diagrams), times 1/3."""
    ops = [h.reshape(a, a, a, a)] + _operands(u, w, a, b) + [rho.reshape(b, b, b, b)]
    Du = np.zeros((a, a, a, a))
    Dw = np.zeros((a, a, a, b))
    for pos in 'LCR':
        labels = _NETS[pos] + [_TOP]
        for i, kind in enumerate(_KINDS):
            if kind == 'h':
                continue
            others = [labels[j] for j in range(len(labels)) if j != i]
            env = _ein(','.join(others) + '->' + labels[i], *[ops[j] for j in range(len(ops)) if j != i])
            if kind == 'u':
                Du += env / 3.0
            else:
                Dw += env / 3.0
    return Du.reshape(a * a, a * a), Dw.reshape(a ** 3, b)


def evaluate(params, h2, chi, T, d=2):
    """Energy per site and Euclidean gradient of the infinite ternary MERA (same steps as the binary evaluate)."""
    dims = layer_dims(chi, T, d)
    hs = [h2]
    for t in range(T):
        a, b = dims[t]
        hs.append(_sym(ascend(hs[-1], params[t][0], params[t][1], a, b)))
    us, ws = params[T]
    rho_s = fixed_point_rho(us, ws, chi)
    energy = float(np.sum(hs[T] * rho_s))
    ht = htilde(hs[T], rho_s, us, ws, chi)
    grads = [None] * (T + 1)
    grads[T] = layer_environments(ht, rho_s, us, ws, chi, chi)
    rhos = [None] * (T + 1)
    rhos[T] = rho_s
    for t in range(T - 1, -1, -1):
        a, b = dims[t]
        u, w = params[t]
        grads[t] = layer_environments(hs[t], rhos[t + 1], u, w, a, b)
        rhos[t] = _sym(descend(rhos[t + 1], u, w, a, b))
    return dict(energy=energy, grads=grads, hs=hs, rhos=rhos, rho_s=rho_s, htilde=ht, dims=dims)


def energy_only(params, h2, chi, T, d=2):
    dims = layer_dims(chi, T, d)
    h = h2
    for t in range(T):
        a, b = dims[t]
        h = ascend(h, params[t][0], params[t][1], a, b)
    rho_s = fixed_point_rho(params[T][0], params[T][1], chi)
    return float(np.sum(h * rho_s))


def preconditioner_rdms(rhos, params, dims):
    """rho_v on the top legs of each tensor (Sec. 4): rho_w = one-site marginal of the top two-site rho, averaged
    over both sites; rho_u = the two-site density matrix on (3k+2, 3k+3) between the disentangler and the
    isometries, i.e. rho pushed down through w_k (x) w_{k+1} keeping their inner bottom legs."""
    out = []
    T = len(dims) - 1
    for t, (a, b) in enumerate(dims):
        top = rhos[t + 1] if t < T else rhos[T]
        r4 = top.reshape(b, b, b, b)
        rho_w = 0.5 * (np.einsum('pqPq->pP', r4) + np.einsum('pqpQ->qQ', r4))
        Wt = params[t][1].reshape(a, a, a, b)
        rho_u = np.einsum('xycp,dzvq,pqPQ,xyCP,DzvQ->cdCD', Wt, Wt, r4, Wt, Wt, optimize='greedy')
        out.append((_sym(rho_u.reshape(a * a, a * a)), _sym(rho_w)))
    return out


# ---- explicit finite ring (brute force) ---------------------------------------------------------------------

def apply_layer(psi, u, w, a, b):
    """Lower a periodic ring state by one ternary layer: leg k (dim b) becomes sites (3k, 3k+1, 3k+2) through w,
    then the disentanglers act on the pairs (3k+2, 3k+3), wrapping around."""
    n = psi.ndim
    Wt = w.reshape(a, a, a, b)
    U = u.reshape(a, a, a, a)
    for j in range(n):
        pos = 3 * j
        psi = np.tensordot(psi, Wt, axes=([pos], [3]))
        psi = np.moveaxis(psi, [psi.ndim - 3, psi.ndim - 2, psi.ndim - 1], [pos, pos + 1, pos + 2])
    m = 3 * n
    for j in range(n):
        s1, s2 = (3 * j + 2) % m, (3 * j + 3) % m
        psi = np.tensordot(U, psi, axes=([2, 3], [s1, s2]))
        rest = [k for k in range(m) if k not in (s1, s2)]
        order = [0] * m
        order[s1], order[s2] = 0, 1
        for idx, k in enumerate(rest):
            order[k] = idx + 2
        psi = np.transpose(psi, order)
    return psi
