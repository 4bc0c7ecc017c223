"""Seeding the Hermitian-indefinite system gamma5 A x = gamma5 phi through a QR factorisation of the
Lanczos matrix, in FP64 (TEST INFRASTRUCTURE).

Section 2 of the paper solves the systems with the LU of the Lanczos tridiagonal T (Eq. 2) and
notes that for an indefinite matrix a QR or LQ factorisation of T has to replace the LU.  The
even-odd Wilson matrix A is not Hermitian, but H = gamma5 A is (A^dag = gamma5 A gamma5), with
eigenvalues of both signs; A x = phi is H x = c with c = gamma5 phi, and it has the solution of the
normal system M x = A^dag phi without squaring the condition number.

Readings taken here (the paper names the factorisation only):
  * The QR form is that of MINRES (Paige and Saunders, SIAM J. Numer. Anal. 12, 1975).  The
    Lanczos relation H V_i = V_{i+1} Tbar_i has the (i+1) x i matrix Tbar_i with alpha on the
    diagonal and beta below and above it.  Givens rotations G_1..G_i reduce Tbar_i to an upper
    triangular R_i with three bands, r(k,k) = rho_k, r(k-1,k) = delta_k, r(k-2,k) = eps_k.
    Column i needs the two previous rotations, then defines G_i from (gammabar_i, beta_i).
  * RHS 1 (g = beta_0 e_1): x_i = x_0 + V_i y with y minimising ||g - Tbar_i y||, so its residual
    is minimal over the Krylov space.  The update runs through the direction vectors
    w_i = (v_i - eps_i w_{i-2} - delta_i w_{i-1}) / rho_i, which are the columns of V_i R_i^{-1}.
    Then x += tau_i w_i, with tau_i the i-th entry of the rotated right-hand side.  The residual
    estimate after step i is the unrotated remainder |u_{i+1}|.
  * Seeding RHS j >= 2 is the same projection with g^j = V_{i+1}^dag r_0^j in place of beta_0 e_1.
    y^j minimises ||V_{i+1}^dag r_0^j - Tbar_i y||, that is the part of the residual r_0^j - H V_i y
    inside the Lanczos space.  Entry i of the rotated g^j is final once v_{i+1} exists: with
    u^j_1 = v_1^dag r_0^j and eta^j_{i+1} = v_{i+1}^dag r_0^j,
        tau^j_i = c_i u^j_i + s_i eta^j_{i+1},   u^j_{i+1} = -s_i u^j_i + c_i eta^j_{i+1},
    and x^j += tau^j_i w_i.  This replaces the eta recurrence of Algorithm 1's seeding (Eq. 1).
  * Periodic reorthogonalisation is as in Algorithm 1: classical Gram-Schmidt of v_i
    against v_1..v_{i-1}, renormalised, then f against v_1..v_i, with one DGKS repeat.  Column i of
    Tbar needs beta_i, which exists only after the reorthogonalisation.  The QR step, w_i and every iterate update
    of step i therefore use the basis as it stands after the reorthogonalisation.
  * Stopping as Algorithm 1: i_conv is the first step with |u_{i+1}| <= tol ||c^1||, and then
    m = min(ceil(past i_conv), m_max).  A beta_i at rounding level (<= 1e-14 max |alpha|) ends
    the run (invariant subspace).
  * Every system is then finished by plain MINRES on H from its seeded guess.  The stop test is the
    recursive residual estimate, confirmed by the true residual ||c - H x|| <= tol ||c|| (on failure
    MINRES restarts from the current x).  This is the residual of the original system A x = phi,
    since ||gamma5 r|| = ||r||.
"""
import math

import numpy as np

from oracle.seedcg import BREAKDOWN_RTOL, _norm, _orthogonalise


def _givens(a, b):
    """(c, s, r) with [c s; -s c] [a; b] = [r; 0], r >= 0 (a, b real)."""
    r = math.hypot(a, b)
    if r == 0.0:
        return 1.0, 0.0, 0.0
    return a / r, b / r, r


def seed_minres(matvec, C, X0=None, *, k, tol, past=1.5, m_max=2000, m=None):
    """Seeded Lanczos with the QR (MINRES) factorisation of Tbar for the right-hand sides C (nrhs, N)
    of the Hermitian (indefinite) H given by matvec.  k = 0: no reorthogonalisation.  With m given the
    run takes exactly m steps.  Returns dict(X, alpha, beta, rho, cs, sn, est, V, m, i_conv, status)."""
    C = np.atleast_2d(np.asarray(C, dtype=np.complex128))
    nrhs, N = C.shape
    X = np.zeros_like(C) if X0 is None else np.array(X0, dtype=np.complex128, copy=True)
    m_cap = int(m) if m is not None else int(m_max)
    R0 = C - matvec(X) if X0 is not None and np.any(X != 0) else C.copy()
    c1 = _norm(C[0])

    beta0 = _norm(R0[0])
    V = np.empty((m_cap + 1, N), dtype=np.complex128)
    V[0] = R0[0] / beta0
    alpha, beta, rho, cs, sn, est = [], [beta0], [], [], [], []
    u = np.empty(nrhs, dtype=np.complex128)          # unrotated remainder of each rotated g^j
    u[0] = beta0
    if nrhs > 1:
        u[1:] = V[0].conj() @ R0[1:].T
    w1 = w2 = None                                   # w_{i-1}, w_{i-2}
    c_1, s_1, c_2, s_2 = 1.0, 0.0, 1.0, 0.0          # G_{i-1}, G_{i-2}
    i_conv, m_stop, status, m_used = None, m_cap, "ok", 0
    i = 1
    while True:
        v = V[i - 1]
        f = matvec(v)
        if i > 1:
            f = f - beta[i - 1] * V[i - 2]
        a = float(np.vdot(v, f).real)
        f = f - a * v
        alpha.append(a)
        if k and i % k == 0:
            vi, _ = _orthogonalise(V[:i - 1], V[i - 1])
            V[i - 1] = vi / _norm(vi)
            f, _ = _orthogonalise(V[:i], f)
        bi = _norm(f)
        beta.append(bi)
        # column i of Tbar: beta_{i-1} (row i-1; none for i = 1), alpha_i (row i), beta_i (row i+1)
        bprev = beta[i - 1] if i > 1 else 0.0
        eps = s_2 * bprev
        dbar = c_2 * bprev
        delta = c_1 * dbar + s_1 * a
        gbar = -s_1 * dbar + c_1 * a
        c_i, s_i, r_i = _givens(gbar, bi)
        if r_i == 0.0:
            status = "singular"
            break
        rho.append(r_i)
        cs.append(c_i)
        sn.append(s_i)
        vcur = V[i - 1]
        w = vcur.copy()
        if w1 is not None:
            w = w - delta * w1
        if w2 is not None:
            w = w - eps * w2
        w = w / r_i
        if bi > 0.0:
            V[i] = f / bi
            eta = V[i].conj() @ R0.T                 # v_{i+1}^dag r_0^j (zero for j = 1 in exact arithmetic)
        else:
            eta = np.zeros(nrhs, dtype=np.complex128)
        eta[0] = 0.0                                 # RHS 1: g = beta_0 e_1
        tau = c_i * u + s_i * eta
        u = -s_i * u + c_i * eta
        X += tau[:, None] * w[None, :]
        m_used = i
        e = abs(u[0])
        est.append(e / c1)
        if i_conv is None and e <= tol * c1:
            i_conv = i
            if m is None:
                m_stop = min(int(math.ceil(past * i_conv)), m_cap)
        if bi <= BREAKDOWN_RTOL * max(abs(x) for x in alpha):
            status = "breakdown"
            break
        if i >= m_stop:
            if i_conv is None and m is None:
                status = "capped"
            break
        w2, w1 = w1, w
        c_2, s_2, c_1, s_1 = c_1, s_1, c_i, s_i
        i += 1
    return dict(X=X, R0=R0, alpha=np.array(alpha), beta=np.array(beta), rho=np.array(rho), cs=np.array(cs),
                sn=np.array(sn), est=np.array(est), V=V[:m_used], m=m_used, i_conv=i_conv, status=status)


def minres(matvec, c, x0=None, *, tol, max_iter=100000):
    """Plain MINRES on H x = c from x0 (the seed_minres recurrences with one right-hand side and no
    reorthogonalisation).  Stops on the residual estimate, confirmed by the true residual; restarts
    from x when the check fails.  Returns (x, iterations, true relative residual)."""
    c = np.asarray(c, dtype=np.complex128)
    x = np.zeros_like(c) if x0 is None else np.array(x0, dtype=np.complex128, copy=True)
    cn = _norm(c)
    it = 0
    while True:
        r = c - matvec(x)
        rn = _norm(r)
        if rn <= tol * cn or it >= max_iter:
            return x, it, rn / cn
        v_prev = np.zeros_like(c)
        v = r / rn
        b_prev = 0.0
        w1 = np.zeros_like(c)
        w2 = np.zeros_like(c)
        c_1, s_1, c_2, s_2 = 1.0, 0.0, 1.0, 0.0
        u = rn
        while it < max_iter:
            f = matvec(v) - b_prev * v_prev
            a = float(np.vdot(v, f).real)
            f = f - a * v
            bi = _norm(f)
            eps = s_2 * b_prev
            dbar = c_2 * b_prev
            delta = c_1 * dbar + s_1 * a
            gbar = -s_1 * dbar + c_1 * a
            c_i, s_i, r_i = _givens(gbar, bi)
            w = (v - delta * w1 - eps * w2) / r_i
            x = x + (c_i * u) * w
            u = -s_i * u
            it += 1
            if abs(u) <= tol * cn or bi == 0.0:
                break
            v_prev, v = v, f / bi
            b_prev = bi
            w2, w1 = w1, w
            c_2, s_2, c_1, s_1 = c_1, s_1, c_i, s_i


def solve_indefinite(matvec, C, X0=None, *, k, tol, past=1.5, m_max=2000):
    """seed_minres on all right-hand sides, then MINRES on each from its guess.  Returns
    dict(X, m, i_conv, iters=[Lanczos steps + MINRES iterations for RHS 1, MINRES iterations for
    the others], relres=[true relative residuals ||c - H x|| / ||c||])."""
    out = seed_minres(matvec, C, X0, k=k, tol=tol, past=past, m_max=m_max)
    X = out["X"]
    iters, res = [], []
    for j in range(X.shape[0]):
        x, it, rr = minres(matvec, C[j], X[j], tol=tol)
        X[j] = x
        iters.append(it + (out["m"] if j == 0 else 0))
        res.append(rr)
    return dict(X=X, m=out["m"], i_conv=out["i_conv"], iters=iters, relres=np.array(res), seed=out)
