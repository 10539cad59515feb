"""Infinite scale-invariant binary MERA: layer maps, fixed point, energy and Euclidean gradient (oracle).

Test infrastructure only (see the package header). Plain numpy/scipy, FP64.

What the paper fixes, and how it is read here:
  * Cost function C = <MERA|H|MERA> for a translation-invariant H = sum_i h_i (Sec. 4). Reported per blocked site.
  * Transition layers i with tensors (u_i, w_i), then one scale-invariant layer repeated to infinity (Sec. 4).
  * The ascending superoperator A raises an operator by one layer, its adjoint (left action on rho) lowers a
    density matrix; the scale-invariant density matrix solves A|rho> = |rho> (App. B).
  * The partial derivative D_v of the cost is the environment of v, summed over every occurrence of v (Sec. 4,
    eq. mera_derivative). For the scale-invariant layer the derivative of <h|rho> runs through the fixed point and
    gives the geometric series sum_i <h|A'^i (d_v A)|rho> with A' = A - |rho><1| (App. B, eq.
    scale_invariant_partial), i.e. an operator h~ solving <h~|(1 - A') = <h'|.
  * The paper's network is ternary; the geometry here is the binary MERA (the paper states the generalisation is
    direct and that binary MERAs behave alike). Three-site operators: binary layer maps send a 3-site operator to a
    3-site operator. Tensor layouts: u[bl, br, tl, tr] (rows = bottom legs, columns = top legs, a^2 x a^2 unitary),
    w[bl, br, t] (rows = bottom legs, a^2 x b isometry). Operators h[abc, ABC] with kets lowercase.
  * Isometry w_j covers the two sites (2j, 2j+1) below it; the disentangler of a layer covers (2j+1, 2j+2).
    An operator on sites (2j, 2j+1, 2j+2) rises to top sites (j-1, j, j+1) (left diagram), one on
    (2j+1, 2j+2, 2j+3) to (j, j+1, j+2) (right diagram); averaging the two positions gives A = (A_L + A_R)/2.
"""
import numpy as np
from scipy.sparse.linalg import LinearOperator, eigs, gmres

# Operand order in every network: h, uL, uL*, uR, uR*, w1, w1*, w2, w2*, w3, w3*.
_NET_L = ['abcABC', 'daef', 'dAEF', 'bcgh', 'BCGH', 'xep', 'xEP', 'fgq', 'FGQ', 'hyr', 'HyR']
_NET_R = ['abcABC', 'abef', 'ABEF', 'cdgh', 'CdGH', 'xep', 'xEP', 'fgq', 'FGQ', 'hyr', 'HyR']
_TOP = 'pqrPQR'
_KINDS = ['h', 'u', 'u', 'u', 'u', 'w', 'w', 'w', 'w', 'w', 'w']


def _ein(spec, *ops):
    """Contract a network given as an einsum string, two operands at a time.

    The pair contracted next is the one with the fewest multiply-adds (ties: smaller result), a plain greedy order;
    each pairwise step is one library einsum call. Returns the tensor with the requested output labels.
    """
    lhs, out = spec.split('->')
    labels = lhs.split(',')
    tens = list(ops)
    dim = {}
    for lab, t in zip(labels, tens):
        for c, n in zip(lab, t.shape):
            dim[c] = n
    while len(tens) > 1:
        best = None
        for i in range(len(tens)):
            for j in range(i + 1, len(tens)):
                rest = set(out).union(*[labels[k] for k in range(len(tens)) if k not in (i, j)])
                union = set(labels[i]) | set(labels[j])
                keep = ''.join(c for c in dict.fromkeys(labels[i] + labels[j]) if c in rest)
                cost = float(np.prod([dim[c] for c in union]))
                size = float(np.prod([dim[c] for c in keep])) if keep else 1.0
                if best is None or (cost, size) < best[0]:
                    best = ((cost, size), i, j, keep)
        _, i, j, keep = best
        t = np.einsum(f'{labels[i]},{labels[j]}->{keep}', tens[i], tens[j], optimize=True)
        for k in (j, i):
            del tens[k]
            del labels[k]
        tens.append(t)
        labels.append(keep)
    return np.einsum(f'{labels[0]}->{out}', tens[0])


def _operands(u, w, a, b):
    U = u.reshape(a, a, a, a)
    Wt = w.reshape(a, a, b)
    return [U, U, U, U, Wt, Wt, Wt, Wt, Wt, Wt]


def ascend_one(net, h, u, w, a, b):
    """One binary ascending diagram: 3-site operator on a^3 below -> b^3 above."""
    spec = ','.join(net) + '->' + _TOP
    return _ein(spec, h.reshape((a,) * 6), *_operands(u, w, a, b)).reshape(b ** 3, b ** 3)


def descend_one(net, rho, u, w, a, b):
    """Adjoint of ascend_one: 3-site density matrix on b^3 above -> a^3 below."""
    spec = ','.join([_TOP] + net[1:]) + '->' + net[0]
    return _ein(spec, rho.reshape((b,) * 6), *_operands(u, w, a, b)).reshape(a ** 3, a ** 3)


def ascend_element(side, h, u, w, a, b, idx):
    """One element A_L(h) or A_R(h) at (p, q, r, P, Q, R) = idx, with the isometries' top legs fixed.

    The same networks as `ascend_one`, contracted in a fixed order that keeps every intermediate at most a^6, so
    single outputs can be sampled at large bond dimension (cost ~a^8 per element).
    """
    U = u.reshape(a, a, a, a)
    Wt = w.reshape(a, a, b)
    p, q, r, P, Q, R = idx
    h6 = h.reshape((a,) * 6)
    X1 = np.einsum('xe,xE->eE', Wt[:, :, p], Wt[:, :, P], optimize=True)
    X3 = np.einsum('hy,Hy->hH', Wt[:, :, r], Wt[:, :, R], optimize=True)
    if side == 'L':
        K = np.einsum('daeg,eE->dagE', np.einsum('daef,fg->daeg', U, Wt[:, :, q]), X1, optimize=True)
        Kb = np.einsum('dAEF,FG->dAEG', U, Wt[:, :, Q], optimize=True)
        T = np.einsum('abcABC,bcgh->aABCgh', h6, U, optimize=True)
        T = np.einsum('aABCgh,hH->aABCgH', T, X3, optimize=True)
        T = np.einsum('aABCgH,BCGH->aAgG', T, U, optimize=True)
        T = np.einsum('aAgG,dagE->AGdE', T, K, optimize=True)
        return float(np.einsum('AGdE,dAEG->', T, Kb, optimize=True))
    Rr = np.einsum('cdgH,CdGH->cgCG', np.einsum('cdgh,hH->cdgH', U, X3), U, optimize=True)
    K = np.einsum('abeg,eE->abEg', np.einsum('abef,fg->abeg', U, Wt[:, :, q]), X1, optimize=True)
    Kb = np.einsum('ABEF,FG->ABEG', U, Wt[:, :, Q], optimize=True)
    T = np.einsum('abcABC,cgCG->abABgG', h6, Rr, optimize=True)
    T = np.einsum('abABgG,abEg->ABGE', T, K, optimize=True)
    return float(np.einsum('ABGE,ABEG->', T, Kb, optimize=True))


def ascend(h, u, w, a, b):
    """Ascending superoperator A = (A_L + A_R)/2 of one layer (App. B notation: <h| A)."""
    return 0.5 * (ascend_one(_NET_L, h, u, w, a, b) + ascend_one(_NET_R, h, u, w, a, b))


def descend(rho, u, w, a, b):
    """Descending superoperator, the adjoint of `ascend` (App. B notation: A |rho>)."""
    return 0.5 * (descend_one(_NET_L, rho, u, w, a, b) + descend_one(_NET_R, rho, u, w, a, b))


def layer_dims(chi, T, d=4):
    """(a_tau, b_tau) for the transition layers tau = 1..T and the scale-invariant layer.

    Reading: a_1 = d, b_tau = min(chi, a_tau^2), a_{tau+1} = b_tau; the scale-invariant layer has a = b = chi,
    so b_T must equal chi.
    """
    dims = []
    a = d
    for _ in range(T):
        b = min(chi, a * a)
        dims.append((a, b))
        a = b
    if a != chi:
        raise ValueError(f"top transition dimension {a} != chi {chi}; add transition layers")
    dims.append((chi, chi))
    return dims


def _sym(m):
    return 0.5 * (m + m.T)


def fixed_point_rho(u, w, chi, tol=0.0):
    """Scale-invariant 3-site density matrix: eigenvector of the descending map with eigenvalue 1 (App. B).

    A library eigensolver (dense LAPACK for chi^6 <= 64, ARPACK otherwise) on the descending map; normalised
    to unit trace and symmetrised.
    """
    n = chi ** 6
    def apply(x):
        return descend(x.reshape(chi ** 3, chi ** 3), u, w, chi, chi).reshape(-1)
    if n <= 64:
        M = np.stack([apply(e) for e in np.eye(n)], axis=1)
        vals, vecs = np.linalg.eig(M)
        v = vecs[:, np.argmax(np.abs(vals))]
    else:
        op = LinearOperator((n, n), matvec=apply, dtype=np.float64)
        v0 = np.eye(chi ** 3).reshape(-1)
        vals, vecs = eigs(op, k=1, which='LM', v0=v0, tol=tol, ncv=min(n, 20), maxiter=10000)
        v = vecs[:, 0]
    v = np.real(v)
    rho = v.reshape(chi ** 3, chi ** 3)
    rho = _sym(rho / np.trace(rho))
    return rho


def identity_op(dim):
    return np.eye(dim ** 3)


def htilde(hT, rho, u, w, chi, method='solve', rtol=1e-14, max_terms=20000):
    """Scale-invariant gradient operator h~ = sum_i <h'| A'^i with h' = h_T - <h_T|rho> 1 (App. B).

    Reading of App. B: A' = A - |rho><1|, so <x|A' = A(x) - Tr[x rho] 1, and h~ solves <h~|(1 - A') = <h'|.
    method='series' sums the deflated series term by term until a term is below 1e-16 (small chi only);
    method='solve' uses a library GMRES on (1 - A').
    """
    e = np.sum(hT * rho)
    hp = hT - e * identity_op(chi)

    def aprime(x):
        return ascend(x, u, w, chi, chi) - np.sum(x * rho) * identity_op(chi)
    if method == 'series':
        out = hp.copy()
        term = hp.copy()
        for _ in range(max_terms):
            term = aprime(term)
            out += term
            if np.max(np.abs(term)) < 1e-16:
                break
        return out
    n = chi ** 6

    def mv(x):
        X = x.reshape(chi ** 3, chi ** 3)
        return (X - aprime(X)).reshape(-1)
    op = LinearOperator((n, n), matvec=mv, dtype=np.float64)
    x, info = gmres(op, hp.reshape(-1), x0=hp.reshape(-1), rtol=rtol, atol=0.0, restart=min(n, 60),
                    maxiter=2000)
    if info != 0:
        raise RuntimeError(f"GMRES for h~ did not converge (info={info})")
    return x.reshape(chi ** 3, chi ** 3)


def layer_environments(h, rho, u, w, a, b):
    """Euclidean derivative of Tr[A(h) rho] w.r.t. u and w of one layer, h and rho held fixed.

    One explicit environment per occurrence (sec. 4, eq. mera_derivative): in each of the two diagrams u occurs
    twice in the ket and twice in the bra, w three times in each; the environment of an occurrence is the closed
    network with that tensor removed. D_v is the sum over occurrences, times 1/2 from the position average.
    """
    h6 = h.reshape((a,) * 6)
    r6 = rho.reshape((b,) * 6)
    ops = [h6] + _operands(u, w, a, b) + [r6]
    Du = np.zeros((a, a, a, a))
    Dw = np.zeros((a, a, b))
    for net in (_NET_L, _NET_R):
        labels = net + [_TOP]
        for i, kind in enumerate(_KINDS):
            if kind == 'h':
                continue
            others = [labels[j] for j in range(len(labels)) if j != i]
            spec = ','.join(others) + '->' + labels[i]
            env = _ein(spec, *[ops[j] for j in range(len(ops)) if j != i])
            if kind == 'u':
                Du += 0.5 * env
            else:
                Dw += 0.5 * env
    return Du.reshape(a * a, a * a), Dw.reshape(a * a, b)


def _split3(lab):
    """Labels of a 3-site operator 'abcABC' as three one-site factors ['aA', 'bB', 'cC']."""
    return [lab[0] + lab[3], lab[1] + lab[4], lab[2] + lab[5]]


def layer_environments_product(hterms, rterms, u, w, a, b):
    """`layer_environments` for operators given as sums of products of one-site matrices.

    h = sum_i A_i (x) B_i (x) C_i (each a x a) and rho = sum_j P_j (x) Q_j (x) R_j (each b x b), with
    h[abc, ABC] = A[a, A] B[b, B] C[c, C]. The networks and occurrences are those of `layer_environments` (sec. 4,
    eq. mera_derivative: D_v is the sum over the occurrences of v of the network with v removed, times 1/2 from the
    position average), with each operator entered as its three factors; by linearity the result is summed over all
    pairs of terms. Each network is one library einsum call with its greedy path; without a 6-leg operator in the
    network that path stays near a^6 per occurrence, so full gradients of dense u, w are available at the bond
    dimensions of the benchmark.
    """
    ops_uw = _operands(u, w, a, b)
    Du = np.zeros((a, a, a, a))
    Dw = np.zeros((a, a, b))
    for net in (_NET_L, _NET_R):
        hl = _split3(net[0])
        rl = _split3(_TOP)
        body = net[1:]
        for hf in hterms:
            for rf in rterms:
                labels = hl + body + rl
                ops = list(hf) + ops_uw + list(rf)
                for i, kind in enumerate(_KINDS[1:]):
                    k = 3 + i
                    others = [labels[j] for j in range(len(labels)) if j != k]
                    spec = ','.join(others) + '->' + labels[k]
                    env = np.einsum(spec, *[ops[j] for j in range(len(ops)) if j != k], optimize='greedy')
                    if kind == 'u':
                        Du += 0.5 * env
                    else:
                        Dw += 0.5 * env
    return Du.reshape(a * a, a * a), Dw.reshape(a * a, b)


def ascend_product(hterms, u, w, a, b):
    """Dense A(h) = (A_L(h) + A_R(h))/2 for h = sum_i A_i (x) B_i (x) C_i (one-site factors, a x a).

    The networks of `ascend_one` with h entered as its three factors, each diagram one library einsum call with
    its greedy path (about a^6 b^2 multiply-adds per term, the output being b^6), so that whole outputs can be
    compared at the benchmark's bond dimension.
    """
    ops_uw = _operands(u, w, a, b)
    out = np.zeros((b,) * 6)
    for net in (_NET_L, _NET_R):
        spec = ','.join(_split3(net[0]) + net[1:]) + '->' + _TOP
        for hf in hterms:
            out += 0.5 * np.einsum(spec, *hf, *ops_uw, optimize='greedy')
    return out.reshape(b ** 3, b ** 3)


def descend_product(rterms, u, w, a, b):
    """Dense D(rho) = (D_L(rho) + D_R(rho))/2 for rho = sum_j P_j (x) Q_j (x) R_j (one-site factors, b x b), the
    networks of `descend_one` with rho entered as its factors (one einsum call per diagram and term)."""
    ops_uw = _operands(u, w, a, b)
    out = np.zeros((a,) * 6)
    for net in (_NET_L, _NET_R):
        spec = ','.join(net[1:] + _split3(_TOP)) + '->' + net[0]
        for rf in rterms:
            out += 0.5 * np.einsum(spec, *ops_uw, *rf, optimize='greedy')
    return out.reshape(a ** 3, a ** 3)


def product_operator(terms):
    """Dense 3-site operator sum_i A_i (x) B_i (x) C_i (rows abc, columns ABC)."""
    return sum(np.kron(np.kron(A, B), C) for A, B, C in terms)


def evaluate(params, h3, chi, T, d=4, htilde_method='solve', rho_s=None):
    """Energy per blocked site and Euclidean gradient of an infinite binary MERA.

    params: list of (u, w) matrices for transition layers 1..T followed by the scale-invariant layer.
    Returns dict with energy, grads [(Du, Dw)], ascended h list, rho list (rho[tau] at the top of layer tau,
    index T+1 unused), rho_s and h~.
    Steps (Sec. 4 and App. B): ascend h through the transition layers; scale-invariant fixed point rho_s;
    e = Tr[h_T rho_s]; h~ from the deflated series; environments of the scale-invariant layer from
    Tr[A_s(h~) rho_s]; then from the top down, environments of layer tau from Tr[A_tau(h_{tau-1}) rho_tau]
    and rho_{tau-1} = D_tau(rho_tau).
    """
    dims = layer_dims(chi, T, d)
    hs = [h3]
    for t in range(T):
        a, b = dims[t]
        u, w = params[t]
        hs.append(_sym(ascend(hs[-1], u, w, a, b)))
    us, ws = params[T]
    if rho_s is None:
        rho_s = fixed_point_rho(us, ws, chi)
    energy = float(np.sum(hs[T] * rho_s))
    ht = htilde(hs[T], rho_s, us, ws, chi, method=htilde_method)
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


def energy_only(params, h3, chi, T, d=4):
    """Energy per blocked site Tr[h_T rho_s] (Sec. 4 cost function, App. B fixed point)."""
    dims = layer_dims(chi, T, d)
    h = h3
    for t in range(T):
        a, b = dims[t]
        h = ascend(h, params[t][0], params[t][1], a, b)
    rho_s = fixed_point_rho(params[T][0], params[T][1], chi)
    return float(np.sum(h * rho_s))


def energy_bottom(params, h3, chi, T, d=4):
    """Same energy via full descent: Tr[h3 rho_0] with rho_0 = D_1(...D_T(rho_s))."""
    dims = layer_dims(chi, T, d)
    rho = fixed_point_rho(params[T][0], params[T][1], chi)
    for t in range(T - 1, -1, -1):
        a, b = dims[t]
        rho = descend(rho, params[t][0], params[t][1], a, b)
    return float(np.sum(h3 * rho))


def preconditioner_rdms(rhos, params, dims):
    """Reduced density matrices rho_v on the top legs of each tensor (Sec. 4, eq. mera_diagonal_inner_product).

    rhos[t] is the density matrix at the bottom of layer t (rhos[T] = rho_s), as returned by `evaluate`; the
    top of transition layer t is therefore rhos[t + 1], and the top of the scale-invariant layer is rho_s.
    Reading: rho_w is the one-site marginal (middle site) of the position-averaged 3-site rho at the top of the
    layer; rho_u is the two-site marginal rho2 = (Tr_3 rho + Tr_1 rho)/2 pushed down through w (x) w with the
    outer bottom legs traced, giving an a^2 x a^2 matrix on the two top legs of u.
    """
    out = []
    T = len(dims) - 1
    for t, (a, b) in enumerate(dims):
        top = rhos[t + 1] if t < T else rhos[T]
        r6 = top.reshape((b,) * 6)
        rho_w = np.einsum('pqrpQr->qQ', r6)
        rho2 = 0.5 * (np.einsum('pqrPQr->pqPQ', r6) + np.einsum('pqrpQR->qrQR', r6))
        Wt = params[t][1].reshape(a, a, b)
        rho_u = np.einsum('xep,fyq,pqPQ,xEP,FyQ->efEF', Wt, Wt, rho2, Wt, Wt, optimize='greedy')
        out.append((_sym(rho_u.reshape(a * a, a * a)), _sym(rho_w)))
    return out
