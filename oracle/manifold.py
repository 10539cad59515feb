"""Stiefel-manifold operations for real isometries (oracle; test infrastructure only).

Sec. 2 of the paper, specialised to real matrices (W^T W = 1):
  * tangent space: X = W A + W_perp B with A skew (eq. stiefel_tangent);
  * Euclidean metric g_W(X, Y) = Tr[X^T Y];
  * orthogonal projection of any D onto the tangent space, G = D - W (W^T D + D^T W)/2 (eq. stiefel_gradient);
  * a retraction R_W(X, alpha): a curve through W with initial velocity X that stays on the manifold.
    Reading: the polar retraction R = polar(W + alpha X) is used (the paper uses the exponential one; it notes that
    other retractions have limited effect). Its curve derivative follows the first-order perturbation of the polar
    factor given in App. A (eqs. polar_perturbation / polar_perturbation_dQ).
  * vector transport: projection of the vector onto the tangent space at the new point (reading; the paper's
    exponential transport belongs to its exponential retraction).
  * the paper's own pair (Sec. 2.3, eqs. retraction and transport): R_W(X, alpha) = exp(alpha Q_X) W and
    T(Y) = exp(alpha Q_X) Y with Q_X = [W W_perp] [[A, -B^T], [B, 0]] [W W_perp]^T; W_perp B = Z = (1 - W W^T) X
    comes from a QR decomposition of [W Z] (the footnote to eq. retraction), so only a (p+r)-dimensional exponential
    is needed. The Grassmann case is the same with A = 0.
  * Hilbert-space preconditioner (Sec. 3, eqs. preconditioner / preconditioner_solution): X~ = W A~ + W_perp B~
    with A~ rho + rho A~ = 2A and B~ = B rho^{-1}, rho regularised as (rho^2 + delta^2)^{1/2} (Sec. 3), with
    delta = ||X_v|| (Sec. 4).
"""
import numpy as np
import scipy.linalg


def inner(X, Y):
    """Euclidean metric g(X, Y) = Tr[X^T Y], summed over a list of factors (product manifold, Sec. 2.4)."""
    return float(sum(np.sum(x * y) for x, y in zip(X, Y)))


def project(W, D):
    """Stiefel tangent projection, eq. stiefel_gradient (real case)."""
    S = W.T @ D
    return D - 0.5 * W @ (S + S.T)


def polar_factor(Y):
    """Orthogonal polar factor Q of Y = Q P via the SVD Y = U S V^T, Q = U V^T."""
    U, _, Vt = np.linalg.svd(Y, full_matrices=False)
    return U @ Vt


def retract(W, X, alpha):
    """Polar retraction W' = polar(W + alpha X) and its curve derivative X' = dW'/dalpha.

    The derivative follows App. A's perturbation of the polar decomposition Y = Q P: for dY = X,
    dQ = Q A_X + Q_perp B_X with A_X P + P A_X = Q^T X - X^T Q and Q_perp B_X = (1 - Q Q^T) X P^{-1},
    solved in the eigenbasis of P from the SVD.
    """
    Y = W + alpha * X
    U, s, Vt = np.linalg.svd(Y, full_matrices=False)
    V = Vt.T
    Q = U @ Vt
    C = V.T @ (Q.T @ X - X.T @ Q) @ V
    Ahat = C / (s[:, None] + s[None, :])
    AX = V @ Ahat @ V.T
    Pinv = V @ np.diag(1.0 / s) @ V.T
    dQ = Q @ AX + (X - Q @ (Q.T @ X)) @ Pinv
    return Q, dQ


def transport(Wnew, Y):
    """Projection vector transport of Y to the tangent space at Wnew."""
    return project(Wnew, Y)


def precondition(W, X, rho, delta=None):
    """Hilbert-space preconditioner of Sec. 3 with the regularisation of Sec. 3/Sec. 4.

    Writes X = W A + W_perp B (A = W^T X, W_perp B = X - W A). In the eigenbasis rho = V diag(lam) V^T the
    regularised spectrum is f = sqrt(lam^2 + delta^2); A~_ij = 2 A_ij / (f_i + f_j), B~ = B V diag(1/f) V^T.
    delta defaults to ||X||_F (Sec. 4). delta = 0 gives the exact solution of eq. preconditioner.
    """
    if delta is None:
        delta = np.linalg.norm(X)
    lam, V = np.linalg.eigh(rho)
    f = np.sqrt(lam * lam + delta * delta)
    A = W.T @ X
    Ah = V.T @ A @ V
    At = V @ (2.0 * Ah / (f[:, None] + f[None, :])) @ V.T
    Bpart = X - W @ A
    Bt = Bpart @ (V @ np.diag(1.0 / f) @ V.T)
    return W @ At + Bt


def exp_frame(W, X):
    """Low-rank factors of Q_X (Sec. 2.3, eq. retraction): U = [W Q] with orthonormal columns and the skew matrix
    M = [[A, -B^T], [B, 0]] with Q_X = U M U^T. A = W^T X; Z = X - W A; Q spans the complement part: the columns
    p..p+r of the QR factor of [W Z], r = min(p, n - p), and B = Q^T Z."""
    n, p = W.shape
    A = W.T @ X
    r = min(p, n - p)
    if r == 0:
        return W.copy(), A.copy()
    Z = X - W @ A
    Qf, _ = np.linalg.qr(np.hstack([W, Z]))
    Q = Qf[:, p:p + r]
    B = Q.T @ Z
    M = np.zeros((p + r, p + r))
    M[:p, :p] = A
    M[:p, p:] = -B.T
    M[p:, :p] = B
    return np.hstack([W, Q]), M


def retract_exp(W, X, alpha):
    """Exponential retraction of eq. retraction, R = exp(alpha Q_X) W = U expm(alpha M)[:, :p], and its curve
    derivative dR/dalpha = exp(alpha Q_X) Q_X W = exp(alpha Q_X) X (Q_X W = X).

    Reading: the product U E carries the rounding of the exponential and of W itself, which accumulates over
    iterations (about 1e-12 per step at large alpha); the result is replaced by its polar factor, a change of the
    order of that rounding, so that W^T W = 1 holds to 1e-13 after every retraction."""
    U, M = exp_frame(W, X)
    E = scipy.linalg.expm(alpha * M)
    p = W.shape[1]
    Wn = polar_factor(U @ E[:, :p])
    return Wn, transport_exp(W, X, alpha, X)


def transport_exp(W, X, alpha, Y):
    """Vector transport of eq. transport, T(Y) = exp(alpha Q_X) Y = Y + U (expm(alpha M) - 1) U^T Y."""
    U, M = exp_frame(W, X)
    E = scipy.linalg.expm(alpha * M)
    return Y + U @ ((E - np.eye(E.shape[0])) @ (U.T @ Y))


def grassmann_project(W, D):
    """Grassmann tangent projection (Sec. 2.2, eq. grassmann_gradient, real case): G = (1 - W W^T) D."""
    return D - W @ (W.T @ D)
