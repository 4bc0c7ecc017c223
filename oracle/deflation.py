"""Deflated CG from Ritz vectors of the stored Lanczos basis, in FP64 (TEST INFRASTRUCTURE).

The paper motivates seeding by its implicit deflation of the small eigenvalues of M (section 1)
and keeps the whole Lanczos basis V of the first right-hand side (section 2).  Here that basis is
used once more for the CG that finishes the other right-hand sides:

  * W: the nev lowest Ritz vectors u_k = V^T s_k of the Lanczos tridiagonal T of Eq. (2),
    T s_k = theta_k s_k (V holds the basis vectors as rows);
  * deflated CG (Saad, Yeung, Erhel and Guyomarc'h, SIAM J. Sci. Comput. 21, 2000), with
    G = W^dag M W and Z = M W:
        x_0 = x_-1 + W^T G^{-1} W^dag r_-1,   r_0 = b - M x_0
        mu_j = G^{-1} Z^dag r_j,              p_0 = r_0 - W^T mu_0
        a_j = |r_j|^2 / Re(p_j^dag M p_j),    x_{j+1} = x_j + a_j p_j,   r_{j+1} = r_j - a_j M p_j
        b_j = |r_{j+1}|^2 / |r_j|^2,          p_{j+1} = b_j p_j + r_{j+1} - W^T mu_{j+1}
    so that W^dag r_j = 0 and W^dag M p_j = 0 for every j (the invariants the tests pin);
  * the stop rule of the plain CG in oracle.seedcg: the recursive residual, confirmed by the true
    one (on failure r is replaced by b - M x and the iteration goes on).
"""
import math

import numpy as np

from oracle.seedcg import tridiag


def ritz(V, alpha, beta, nev):
    """The nev lowest Ritz pairs of T (Eq. 2) lifted with the basis: (theta, U), U of shape (nev, N)."""
    T = tridiag(alpha, beta)
    theta, S = np.linalg.eigh(T)
    nev = min(nev, len(theta))
    U = S[:, :nev].T @ np.asarray(V)[: T.shape[0]]
    return theta[:nev], U


def deflated_cg(matvec, b, x0, W, *, tol, max_iter=100000, history=False, precond=None):
    """Deflated CG on M x = b from x0 with deflation vectors W (rows).  Returns (x, iterations,
    true relative residual[, per-iteration (r, p) pairs when history is set]).

    With a preconditioner P (precond(r) = P r, Hermitian positive definite) this is the deflated PCG
    of the same paper: z_j = P r_j takes the place of r_j in the direction, p_0 = z_0 - W^T G^{-1} Z^dag z_0,
    p_{j+1} = z_{j+1} + b_j p_j - W^T G^{-1} Z^dag z_{j+1}, with a_j = r_j^dag z_j / p_j^dag M p_j and
    b_j = r_{j+1}^dag z_{j+1} / r_j^dag z_j; W^dag r_j = 0 and W^dag M p_j = 0 still hold."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128, copy=True)
    W = np.atleast_2d(np.asarray(W, dtype=np.complex128)) if len(W) else np.zeros((0, b.size), np.complex128)
    nw = W.shape[0]
    bn = float(np.linalg.norm(b))
    if nw:
        Z = np.stack([matvec(w) for w in W])          # M W
        G = W.conj() @ Z.T                            # W^dag M W
        Ginv_apply = lambda c: np.linalg.solve(G, c)
        r = b - matvec(x)
        x = x + W.T @ Ginv_apply(W.conj() @ r)        # x_0 = x_-1 + W G^-1 W^dag r_-1
    r = b - matvec(x)
    hist = []
    if float(np.linalg.norm(r)) <= tol * bn:
        out = (x, 0, float(np.linalg.norm(r)) / bn)
        return out + (hist,) if history else out

    def direction(z, p=None, beta=0.0):
        d = z if p is None else z + beta * p
        if nw:
            d = d - W.T @ Ginv_apply(Z.conj() @ z)    # - W mu, mu = G^-1 Z^dag z
        return d

    P = precond if precond is not None else (lambda v: v)
    z = P(r)
    p = direction(z)
    rz = float(np.vdot(r, z).real)
    it = 0
    while it < max_iter:
        if history:
            hist.append((r.copy(), p.copy()))
        q = matvec(p)
        a = rz / float(np.vdot(p, q).real)
        x = x + a * p
        r = r - a * q
        it += 1
        if float(np.linalg.norm(r)) <= tol * bn:
            r = b - matvec(x)
            if float(np.linalg.norm(r)) <= tol * bn:
                break
        z = P(r)
        rz_new = float(np.vdot(r, z).real)
        p = direction(z, p, rz_new / rz)
        rz = rz_new
    res = float(np.linalg.norm(b - matvec(x))) / bn
    out = (x, it, res)
    return out + (hist,) if history else out
