"""Algorithm 1 of the paper (Seed-CG(m, k)) and plain CG, in FP64 (TEST INFRASTRUCTURE).

Seed-CG is written here as one loop over the Lanczos steps i = 1, 2, ...: the three-term
recurrence gives alpha_i, the LU factorisation of the tridiagonal T (Eq. 2) gains one row
(delta_i, gamma_{i-1}, zeta_i) and updates the first system's iterate through w_i, the Galerkin
seeding of Eq. (1) updates every other system through the eta recurrence, the basis is
reorthogonalised every k steps, and beta_i gives the next Lanczos vector and the residual
estimate.

Vectors are flat complex128 arrays of length N; a batch of right-hand sides is (nrhs, N).
`matvec` applies the Hermitian positive-definite M to one vector or to a batch.

Readings of the paper taken here (where it is silent or garbled):
  * The algorithm's start does not form v_2: the end-of-step update v_{i+1} = f / beta_i is
    applied at i = 1 as well, and the first Lanczos step is reorthogonalised and closed like any other.
  * The LU row and the seeding use v_i before the reorthogonalisation changes it; the
    reorthonormalised v_i is what is kept and used as v_{i-1} in the next three-term
    recurrence; alpha, beta (the matrix T) are not recomputed after the reorthogonalisation.
  * The reorthogonalisation is classical Gram-Schmidt: v_i against v_1..v_{i-1}, normalised,
    then f against v_1..v_i; a pass is repeated once (Daniel-Gragg-Kaufman-Stewart) when it
    shrinks the vector's norm below 1/sqrt(2) of its norm before the pass.
  * The initial residuals r_0^j are computed once; the eta recurrence always uses r_0^j.
  * Stopping: the paper fixes m up front.  With past > 0 and no fixed m, the residual
    estimate of D-Lanczos, ||r_i|| = beta_i |zeta_i / delta_i|, decides i_conv, the first
    i with estimate <= tol * ||b^1||, and then m = min(ceil(past * i_conv), m_max).
  * Breakdown: beta_i <= 1e-14 max|alpha| ends the run at m = i (invariant subspace);
    delta_i <= 0 (positive definiteness lost in rounding) ends it at m = i - 1, before
    iteration i changes any iterate.
"""
import math

import numpy as np

BREAKDOWN_RTOL = 1e-14


def _norm(x):
    return float(np.sqrt(np.vdot(x, x).real))


def _cgs_pass_against(Q, x):
    """One classical Gram-Schmidt pass of x against the rows of Q: x - Q^T (conj(Q) x)."""
    if Q.shape[0] == 0:
        return x
    c = Q.conj() @ x
    return x - Q.T @ c


def _orthogonalise(Q, x):
    """CGS with one DGKS repeat; returns the orthogonalised x (not normalised) and the pass count."""
    n0 = _norm(x)
    x = _cgs_pass_against(Q, x)
    n1 = _norm(x)
    passes = 1
    if n1 < n0 / math.sqrt(2.0):
        x = _cgs_pass_against(Q, x)
        passes = 2
    return x, passes


def seed_cg(matvec, B, X0=None, *, k, tol, past=1.5, m_max=2000, m=None, reorth_basis=None):
    """Algorithm 1, Seed-CG(m, k), for the right-hand sides B (nrhs, N).

    k = 0 means no reorthogonalisation (k = infinity).  If m is given the run takes
    exactly m steps (the paper's fixed m); otherwise m = min(ceil(past*i_conv), m_max).
    Returns a dict with X (the RHS-1 iterate and the seeded guesses), the Lanczos
    coefficients alpha_1..alpha_m, beta_0..beta_m, the LU scalars delta, gamma, zeta,
    the basis V (m, N), i_conv, m and a status string.
    reorth_basis (optional): maps the stored basis vectors to the ones the reorthogonalisation
    projects against and subtracts (for instance their FP32 roundings); the stored basis, the
    Lanczos recurrence and the seeding are unchanged.
    """
    B = np.atleast_2d(np.asarray(B, dtype=np.complex128))
    nrhs, N = B.shape
    X = np.zeros_like(B) if X0 is None else np.array(X0, dtype=np.complex128, copy=True)
    m_cap = int(m) if m is not None else int(m_max)

    # initial residuals r_0^j = b^j - M x_0^j
    R0 = B - matvec(X) if X0 is not None and np.any(X != 0) else B.copy()
    b1 = _norm(B[0])

    # the Lanczos start: beta_0 = ||r_0^1||, v_1 = r_0^1 / beta_0
    beta0 = _norm(R0[0])
    V = np.empty((m_cap + 1, N), dtype=np.complex128)
    V[0] = R0[0] / beta0
    alpha, beta, delta, gamma, zeta, est = [], [beta0], [], [0.0], [], []
    eta = np.zeros(nrhs - 1, dtype=np.complex128)
    w_prev = None
    i_conv = None
    m_stop = m_cap
    status = "ok"
    passes = 0
    m_used = 0

    i = 1
    while True:
        v = V[i - 1]
        # three-term recurrence: f = M v_i - beta_{i-1} v_{i-1}; alpha_i = v_i^dag f; f -= alpha_i v_i
        f = matvec(v)
        if i > 1:
            f = f - beta[i - 1] * V[i - 2]
        a = float(np.vdot(v, f).real)
        f = f - a * v
        # one more row of the LU of T (Eq. 2), and the first system's iterate along w_i
        if i == 1:
            g = 0.0
            d = a
            z = beta0
        else:
            g = beta[i - 1] / delta[-1]
            d = a - g * beta[i - 1]
            z = -g * zeta[-1]
        if not (d > 0.0 and math.isfinite(d)):
            status = "indefinite"
            break
        alpha.append(a)
        delta.append(d)
        if i > 1:
            gamma.append(g)
        zeta.append(z)
        w = v / d if i == 1 else (v - beta[i - 1] * w_prev) / d
        X[0] += z * w
        # Galerkin seeding (Eq. 1): eta^j = v_i^dag r_0^j - gamma_{i-1} eta^j; x^j += eta^j w_i
        if nrhs > 1:
            eta = (V[i - 1].conj() @ R0[1:].T) - g * eta
            X[1:] += eta[:, None] * w[None, :]
        m_used = i
        # periodic reorthogonalisation
        if k and i % k == 0:
            Q = (lambda rows: rows) if reorth_basis is None else reorth_basis
            vi, p1 = _orthogonalise(Q(V[:i - 1]), V[i - 1])
            V[i - 1] = vi / _norm(vi)
            f, p2 = _orthogonalise(Q(V[:i]), f)
            passes += p1 + p2
        # beta_i = ||f||, the residual estimate, the stopping rule and v_{i+1} = f / beta_i
        bi = _norm(f)
        beta.append(bi)
        e = bi * abs(z / d)
        est.append(e / b1)
        if i_conv is None and e <= tol * b1:
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
        V[i] = f / bi
        w_prev = w
        i += 1

    return dict(X=X, R0=R0, alpha=np.array(alpha), beta=np.array(beta), delta=np.array(delta),
                gamma=np.array(gamma), zeta=np.array(zeta), est=np.array(est), V=V[:m_used],
                m=m_used, i_conv=i_conv, status=status, reorth_passes=passes)


def tridiag(alpha, beta):
    """The Lanczos matrix T of Eq. (2): alpha on the diagonal, beta_1..beta_{m-1} beside it."""
    m = len(alpha)
    T = np.diag(np.asarray(alpha, dtype=np.float64))
    off = np.asarray(beta[1:m], dtype=np.float64)
    T += np.diag(off, 1) + np.diag(off, -1)
    return T


def cg(matvec, b, x0=None, *, tol, max_iter=100000):
    """Textbook (Hestenes-Stiefel) CG on M x = b from x0.

    The stop test is the recursive residual ||r|| <= tol ||b||, confirmed by the true
    residual b - M x; when the check fails r is replaced by the true residual and CG goes on.
    Returns (x, iterations, true relative residual, list of recursive relative residuals).
    """
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128, copy=True)
    bn = _norm(b)
    r = b - matvec(x)
    rr = float(np.vdot(r, r).real)
    hist = [math.sqrt(rr) / bn]
    it = 0
    if math.sqrt(rr) <= tol * bn:
        return x, 0, math.sqrt(rr) / bn, hist
    p = r.copy()
    while it < max_iter:
        q = matvec(p)
        a = rr / float(np.vdot(p, q).real)
        x = x + a * p
        r = r - a * q
        rr_new = float(np.vdot(r, r).real)
        it += 1
        hist.append(math.sqrt(rr_new) / bn)
        if math.sqrt(rr_new) <= tol * bn:
            r = b - matvec(x)
            rr_new = float(np.vdot(r, r).real)
            if math.sqrt(rr_new) <= tol * bn:
                break
        bcoef = rr_new / rr
        p = r + bcoef * p
        rr = rr_new
    res = b - matvec(x)
    return x, it, _norm(res) / bn, hist


def cg_coefficients(matvec, b, n_iter):
    """The first n_iter step lengths a_j and direction coefficients b_j of plain CG from x0 = 0."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(np.vdot(r, r).real)
    a_list, b_list, r_list = [], [], [r.copy()]
    for _ in range(n_iter):
        q = matvec(p)
        a = rr / float(np.vdot(p, q).real)
        x = x + a * p
        r = r - a * q
        rr_new = float(np.vdot(r, r).real)
        bc = rr_new / rr
        a_list.append(a)
        b_list.append(bc)
        r_list.append(r.copy())
        p = r + bc * p
        rr = rr_new
    return np.array(a_list), np.array(b_list), r_list


def galerkin(matvec, V, R0, X0=None):
    """Galerkin solution of Eq. (1) by a dense solve: x^j = x_0^j + V (V^dag M V)^{-1} V^dag r_0^j."""
    V = np.atleast_2d(V)
    MV = np.stack([matvec(v) for v in V])
    G = V.conj() @ MV.T
    rhs = V.conj() @ np.atleast_2d(R0).T
    Y = np.linalg.solve(G, rhs)
    X = (V.T @ Y).T
    if X0 is not None:
        X = X + X0
    return X


def true_relres(matvec, B, X):
    B = np.atleast_2d(B)
    R = B - matvec(np.atleast_2d(X))
    return np.sqrt(np.sum(np.abs(R) ** 2, axis=1)) / np.sqrt(np.sum(np.abs(B) ** 2, axis=1))


def orth_loss(V):
    """max |V^dag V - I|."""
    G = V.conj() @ V.T
    return float(np.max(np.abs(G - np.eye(G.shape[0]))))


def repeated_seed(matvec, B, X0=None, *, k, tol, m_max=2000):
    """Traditional repeated seeding (section 2 of the paper; the comparison variant): system j runs
    Algorithm 1 from its current guess until its residual estimate meets tol (m = i_conv) and
    seeds systems j+1..n from its own Krylov space; then plain CG finishes any system whose FP64
    true residual is above tol.  Returns dict(X, lanczos=[m_j], cg=[iterations_j], seeded=[...])
    where seeded[j] holds, after run j, the residual of system j+1 (for the Galerkin pin)."""
    B = np.atleast_2d(np.asarray(B, dtype=np.complex128))
    n = B.shape[0]
    X = np.zeros_like(B) if X0 is None else np.array(np.atleast_2d(X0), dtype=np.complex128, copy=True)
    lanczos, seeded, bases = [], [], []
    for j in range(n):
        out = seed_cg(matvec, B[j:], X[j:], k=k, tol=tol, past=1.0, m_max=m_max)
        X[j:] = out["X"]
        lanczos.append(out["m"])
        bases.append(out["V"])
        if j + 1 < n:
            seeded.append(B[j + 1] - matvec(X[j + 1]))
    cg_iters = []
    for j in range(n):
        x, it, _, _ = cg(matvec, B[j], X[j], tol=tol)
        X[j] = x
        cg_iters.append(it)
    return dict(X=X, lanczos=lanczos, cg=cg_iters, seeded=seeded, bases=bases)
