"""FP64 oracle of the learned gauge-covariant preconditioner K (TEST INFRASTRUCTURE).

The paper has no preconditioner; this follows the workload's reading of one:
  * transports on full-lattice 12-spinors, d = 0 .. 8:
      T_0 psi = psi,  T_{+mu} psi(x) = U_mu(x) psi(x+mu),  T_{-mu} psi(x) = U_mu(x-mu)^dag psi(x-mu)
    (d = 1..4 is +x,+y,+z,+t and d = 5..8 is -x,..,-t), with the fermion boundary sign on hops
    across the t boundary, so that T_{+mu}^dag = T_{-mu};
  * a layer (L psi)(x) = sum_d (w_d (x) 1_3)(T_d psi)(x), w_d a 4x4 complex spin matrix;
  * K = R_e L_3 L_2 L_1 E_e and K^dag = R_e L_1^dag L_2^dag L_3^dag E_e, where E_e embeds an
    even-site vector into the full lattice (zero on odd sites), R_e restricts to even sites and
    L^dag = sum_d (w_d^dag (x) 1_3) T_{-d};
  * the preconditioner P = K K^dag, Hermitian positive semi-definite by construction;
  * the loss over training pairs (u_s, y_s = M u_s): mean_s ||K K^dag y_s - u_s||^2 / ||u_s||^2;
  * complex weights, Wirtinger gradients dL/d(conj w), and Adam on Re w and Im w as independent
    reals (dL/dRe w = 2 Re dL/dconj(w), dL/dIm w = 2 Im dL/dconj(w)).
Weights are an array W[layer 0..2][d 0..8][4][4].  Training starts from the first Neumann term of
A^{-1}, K = 1 + kappa^2 H_eo H_oe (neumann_weights); the identity (w_{l,0} = 1, all hops 0) is a
saddle point of the loss.

Parity: pinned by finite differences of the loss, by K = 1 at initialisation, by gauge
covariance and by Hermiticity/positivity of K K^dag on a dense small lattice.
"""
import numpy as np

NDIR = 9
NLAYER = 3


def _coords(dims):
    Lx, Ly, Lz, Lt = dims
    s = np.arange(Lx * Ly * Lz * Lt)
    return np.stack([s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)], axis=1)


class Lattice:
    def __init__(self, links, dims, t_bc=-1):
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.U = np.asarray(links, dtype=np.complex128).reshape(4, self.V, 3, 3)
        C = _coords(self.dims)
        Lx, Ly, Lz, Lt = self.dims
        idx = lambda c: c[:, 0] + Lx * (c[:, 1] + Ly * (c[:, 2] + Lz * c[:, 3]))
        self.fwd = np.empty((4, self.V), dtype=np.int64)
        self.bwd = np.empty((4, self.V), dtype=np.int64)
        self.sf = np.ones((4, self.V))
        self.sb = np.ones((4, self.V))
        for mu in range(4):
            c = C.copy()
            c[:, mu] = (c[:, mu] + 1) % self.dims[mu]
            self.fwd[mu] = idx(c)
            c = C.copy()
            c[:, mu] = (c[:, mu] - 1) % self.dims[mu]
            self.bwd[mu] = idx(c)
        self.sf[3, C[:, 3] == Lt - 1] = t_bc
        self.sb[3, C[:, 3] == 0] = t_bc
        par = C.sum(axis=1) % 2
        self.even = np.nonzero(par == 0)[0]

    def transport(self, psi, d):
        """(T_d psi) for full-lattice psi of shape (..., V, 4, 3)."""
        if d == 0:
            return psi.copy()
        mu = (d - 1) % 4
        if d <= 4:
            nb = psi[..., self.fwd[mu], :, :]
            out = np.einsum("xab,...xsb->...xsa", self.U[mu], nb)
            return out * self.sf[mu][:, None, None]
        nb = psi[..., self.bwd[mu], :, :]
        Ub = self.U[mu][self.bwd[mu]]
        out = np.einsum("xba,...xsb->...xsa", Ub.conj(), nb)
        return out * self.sb[mu][:, None, None]

    def embed(self, x_even):
        out = np.zeros(x_even.shape[:-3] + (self.V, 4, 3), dtype=np.complex128)
        out[..., self.even, :, :] = x_even
        return out

    def restrict(self, psi):
        return psi[..., self.even, :, :]


def adjoint_dir(d):
    return 0 if d == 0 else (d + 4 if d <= 4 else d - 4)


def layer(lat, Wl, psi, dagger=False):
    """L psi = sum_d (w_d x 1) T_d psi;  L^dag psi = sum_d (w_d^dag x 1) T_{-d} psi."""
    out = np.zeros_like(psi)
    for d in range(NDIR):
        w = Wl[d].conj().T if dagger else Wl[d]
        t = lat.transport(psi, adjoint_dir(d) if dagger else d)
        out += np.einsum("ab,...xbc->...xac", w, t)
    return out


def apply_K(lat, W, x_even):
    a = lat.embed(x_even)
    for l in range(NLAYER):
        a = layer(lat, W[l], a)
    return lat.restrict(a)


def apply_Kdag(lat, W, x_even):
    a = lat.embed(x_even)
    for l in reversed(range(NLAYER)):
        a = layer(lat, W[l], a, dagger=True)
    return lat.restrict(a)


def apply_P(lat, W, x_even):
    return apply_K(lat, W, apply_Kdag(lat, W, x_even))


def identity_weights():
    W = np.zeros((NLAYER, NDIR, 4, 4), dtype=np.complex128)
    W[:, 0] = np.eye(4)
    return W


def neumann_weights(kappa):
    """The training start: K = 1 + kappa^2 H_eo H_oe, the first term of the Neumann series of
    A^{-1} = (1 - kappa^2 H_eo H_oe)^{-1} (section 3's even-odd operator).

    Every layer gets w_0 = 1 and the Wilson hop's spin factors w_{+mu} = c (1 - gamma_mu),
    w_{-mu} = c (1 + gamma_mu).  Through E_e and R_e only the paths of zero and two hops reach an
    even site; the two-hop paths come from three layer pairs (w_0 of the third layer, of the second,
    or of the first), so c^2 = kappa^2 / 3.  The identity start (all hops 0) is a saddle point of
    the loss: every surviving hop path carries two hop weights, so the gradient of each one vanishes.
    """
    from oracle.dense import gamma_matrices
    g = gamma_matrices()
    c = kappa / np.sqrt(3.0)
    W = identity_weights()
    for mu in range(4):
        W[:, 1 + mu] = c * (np.eye(4) - g[mu])
        W[:, 5 + mu] = c * (np.eye(4) + g[mu])
    return W


def band_mask(lat, t0, nt):
    """Even sites whose t lies in the band [t0, t0 + nt) mod Lt (the whole lattice for nt = None)."""
    t = _coords(lat.dims)[lat.even, 3]
    if nt is None:
        return np.ones(t.shape, dtype=bool)
    return ((t - t0) % lat.dims[3]) < nt


def loss(lat, W, Y, Uv, band=None):
    """mean_s ||K K^dag y_s - u_s||^2 / ||u_s||^2 for Y, Uv of shape (S, Vh, 4, 3); with band = (t0, nt)
    both norms are taken over the even sites of that band of t-slices only."""
    mask = band_mask(lat, *band) if band else band_mask(lat, 0, None)
    Z = apply_P(lat, W, Y)
    e = (Z - Uv)[:, mask]
    num = np.sum(np.abs(e) ** 2, axis=(1, 2, 3))
    den = np.sum(np.abs(Uv[:, mask]) ** 2, axis=(1, 2, 3))
    return float(np.mean(num / den))


def _outer_grad(g, t):
    """sum over sites and colours of g[x, a, c] conj(t[x, b, c]) -> 4x4 (summed over a batch too)."""
    return np.einsum("xac,xbc->ab", g.reshape(-1, 4, 3), t.reshape(-1, 4, 3).conj())


def grad(lat, W, Y, Uv, band=None):
    """Wirtinger gradient dL/d(conj W), same shape as W, by reverse mode through the six layers (of the
    loss on a band of t-slices when band = (t0, nt) is given)."""
    mask = band_mask(lat, *band) if band else band_mask(lat, 0, None)
    S = Y.shape[0]
    G = np.zeros_like(W)
    # forward, keeping every layer input
    a = [lat.embed(Y)]
    for l in reversed(range(NLAYER)):          # K^dag: layers 3, 2, 1 (adjoints)
        a.append(layer(lat, W[l], a[-1], dagger=True))
    b = [lat.embed(lat.restrict(a[-1]))]
    for l in range(NLAYER):                    # K: layers 1, 2, 3
        b.append(layer(lat, W[l], b[-1]))
    Z = lat.restrict(b[-1])
    den = np.sum(np.abs(Uv[:, mask]) ** 2, axis=(1, 2, 3))
    g_even = (Z - Uv) / (S * den)[:, None, None, None]
    g_even[:, ~mask] = 0.0
    # backward through K
    g = lat.embed(g_even)
    for l in reversed(range(NLAYER)):
        inp = b[l]
        for d in range(NDIR):
            G[l, d] += _outer_grad(g, lat.transport(inp, d))
        g = layer(lat, W[l], g, dagger=True)
    # through E_e R_e
    g = lat.embed(lat.restrict(g))
    # backward through K^dag: a[1] = L3^dag a[0], a[2] = L2^dag a[1], a[3] = L1^dag a[2]
    for step, l in enumerate(range(NLAYER)):   # layers 1, 2, 3 in reverse order of application
        inp = a[NLAYER - 1 - step]
        for d in range(NDIR):
            Gp = _outer_grad(g, lat.transport(inp, adjoint_dir(d)))
            G[l, d] += Gp.conj().T
        g = layer(lat, W[l], g)
    return G


def adam_step(W, G, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on the reals (Re W, Im W); state = dict(m, v, t) of real arrays."""
    g = np.stack([2.0 * G.real, 2.0 * G.imag])
    if not state:
        state.update(m=np.zeros_like(g), v=np.zeros_like(g), t=0)
    state["t"] += 1
    state["m"] = b1 * state["m"] + (1 - b1) * g
    state["v"] = b2 * state["v"] + (1 - b2) * g * g
    mh = state["m"] / (1 - b1 ** state["t"])
    vh = state["v"] / (1 - b2 ** state["t"])
    step = lr * mh / (np.sqrt(vh) + eps)
    return W - (step[0] + 1j * step[1])


def pcg(matvec, precond, b, x0=None, *, tol, max_iter=100000):
    """Preconditioned CG (z = P r) with the same stop rule as plain CG in seedcg.cg."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128, copy=True)
    bn = float(np.linalg.norm(b))
    r = b - matvec(x)
    if np.linalg.norm(r) <= tol * bn:
        return x, 0
    z = precond(r)
    p = z.copy()
    rz = float(np.vdot(r, z).real)
    it = 0
    while it < max_iter:
        q = matvec(p)
        a = rz / float(np.vdot(p, q).real)
        x = x + a * p
        r = r - a * q
        it += 1
        if np.linalg.norm(r) <= tol * bn:
            r = b - matvec(x)
            if np.linalg.norm(r) <= tol * bn:
                break
        z = precond(r)
        rz_new = float(np.vdot(r, z).real)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it
