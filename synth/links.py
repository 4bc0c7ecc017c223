"""Random SU(3) gauge links, APE smearing, a topological flux background and the plaquette diagnostic.

Links are U = exp(i*eps*H) with H a random traceless Hermitian 3x3 matrix whose
entries come from complex Gaussians; APE smearing mixes each link with its six
staples and projects back onto SU(3).  The flux background is a constant abelian field
strength with whole flux quanta through the (x, y) and (z, t) planes of the torus, embedded in
SU(3) as diag(e^{i q_c phi}) with charges q = (1, 1, -2); its topological charge makes the Dirac
operator carry near-zero modes that stand apart from the rest of the spectrum.  All of it is
input generation only.
"""
import numpy as np

_CHUNK = 1 << 20  # matrices per eigen-decomposition batch (bounds peak memory)


def _axis(mu):
    # per-direction arrays are shaped (Lt, Lz, Ly, Lx, 3, 3): x is axis 3, t is axis 0
    return 3 - mu


def _dag(a):
    return np.conj(np.swapaxes(a, -1, -2))


def random_su3_links(dims, eps, rng):
    """U_mu(s) = exp(i*eps*H_mu(s)), H = (Z + Z^dag)/2 - tr(.)/3, Z_ab ~ N(0,1) + i N(0,1).

    Draw order: all real parts for (mu, s, a, b) in C order, then all imaginary parts.
    Returns complex128 (4, V, 3, 3).
    """
    Lx, Ly, Lz, Lt = (int(d) for d in dims)
    V = Lx * Ly * Lz * Lt
    zr = rng.standard_normal((4, V, 3, 3))
    zi = rng.standard_normal((4, V, 3, 3))
    U = np.empty((4 * V, 3, 3), dtype=np.complex128)
    zr = zr.reshape(4 * V, 3, 3)
    zi = zi.reshape(4 * V, 3, 3)
    eye = np.eye(3)
    for lo in range(0, 4 * V, _CHUNK):
        hi = min(lo + _CHUNK, 4 * V)
        Z = zr[lo:hi] + 1j * zi[lo:hi]
        H = 0.5 * (Z + _dag(Z))
        tr = np.trace(H, axis1=1, axis2=2).real / 3.0
        H = H - tr[:, None, None] * eye
        lam, Q = np.linalg.eigh(H)
        U[lo:hi] = (Q * np.exp(1j * eps * lam)[:, None, :]) @ _dag(Q)
    return U.reshape(4, V, 3, 3)


def project_su3(W):
    """Nearest unitary W (W^dag W)^(-1/2), then divide by the principal cube root of det."""
    shape = W.shape
    W = W.reshape(-1, 3, 3)
    out = np.empty_like(W)
    for lo in range(0, W.shape[0], _CHUNK):
        hi = min(lo + _CHUNK, W.shape[0])
        w = W[lo:hi]
        lam, Q = np.linalg.eigh(_dag(w) @ w)
        inv_sqrt = (Q * (1.0 / np.sqrt(lam))[:, None, :]) @ _dag(Q)
        u = w @ inv_sqrt
        phase = np.angle(np.linalg.det(u))
        out[lo:hi] = u * np.exp(-1j * phase / 3.0)[:, None, None]
    return out.reshape(shape)


def _as5(U, dims):
    Lx, Ly, Lz, Lt = (int(d) for d in dims)
    return U.reshape(4, Lt, Lz, Ly, Lx, 3, 3)


def ape_smear(U, dims, alpha, steps):
    """APE smearing: U' = P_SU3[(1-alpha) U_mu + alpha/6 * sum of the 6 staples], all mu at once.

    Staples of U_mu(n) for nu != mu (gauge field periodic in every direction):
      up   U_nu(n) U_mu(n+nu) U_nu(n+mu)^dag
      down U_nu(n-nu)^dag U_mu(n-nu) U_nu(n-nu+mu)
    """
    U5 = _as5(np.array(U, copy=True), dims)
    for _ in range(int(steps)):
        new = np.empty_like(U5)
        for mu in range(4):
            am = _axis(mu)
            S = np.zeros_like(U5[mu])
            for nu in range(4):
                if nu == mu:
                    continue
                an = _axis(nu)
                Unu = U5[nu]
                Umu_pnu = np.roll(U5[mu], -1, axis=an)
                Unu_pmu = np.roll(Unu, -1, axis=am)
                S += Unu @ Umu_pnu @ _dag(Unu_pmu)
                Unu_mnu = np.roll(Unu, 1, axis=an)
                Umu_mnu = np.roll(U5[mu], 1, axis=an)
                Unu_mnu_pmu = np.roll(Unu_mnu, -1, axis=am)
                S += _dag(Unu_mnu) @ Umu_mnu @ Unu_mnu_pmu
            new[mu] = project_su3((1.0 - alpha) * U5[mu] + (alpha / 6.0) * S)
        U5 = new
    return U5.reshape(U.shape)


def flux_background(dims, n01, n23, charges=(1, 1, -2)):
    """A constant field strength on the torus, as SU(3) links (4, V, 3, 3).

    In the (x, y) plane the phase per plaquette is theta = 2 pi n01 / (Lx Ly) (Landau gauge):
    the y link at x carries theta * x, and the x link leaving the last x-slice, x = Lx - 1, carries
    -theta * Lx * y, so that every plaquette, the wrapped ones included, carries theta and the
    plane holds n01 flux quanta.  The (z, t) plane is built the same way from z and t with n23.
    Every other plaquette is 1.  Colour c sees the phase times charges[c] (the charges sum to
    zero, so each link has unit determinant).
    """
    Lx, Ly, Lz, Lt = (int(d) for d in dims)
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    th01 = 2.0 * np.pi * n01 / (Lx * Ly)
    th23 = 2.0 * np.pi * n23 / (Lz * Lt)
    phase = np.zeros((4, Lt, Lz, Ly, Lx))
    phase[0] = np.where(x == Lx - 1, -th01 * Lx * y, 0.0)
    phase[1] = th01 * x
    phase[2] = np.where(z == Lz - 1, -th23 * Lz * t, 0.0)
    phase[3] = th23 * z
    q = np.asarray(charges, dtype=np.float64)
    if abs(q.sum()) > 0:
        raise ValueError("the charges must sum to zero (unit determinant)")
    U = np.zeros((4, Lt * Lz * Ly * Lx, 3, 3), dtype=np.complex128)
    ph = phase.reshape(4, -1)
    for c in range(3):
        U[:, :, c, c] = np.exp(1j * q[c] * ph)
    return U


def plaquette(U, dims):
    """Mean of Re tr[U_mu(n) U_nu(n+mu) U_mu(n+nu)^dag U_nu(n)^dag]/3 over n and mu < nu."""
    U5 = _as5(U, dims)
    acc, cnt = 0.0, 0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            P = (U5[mu] @ np.roll(U5[nu], -1, axis=_axis(mu))
                 @ _dag(np.roll(U5[mu], -1, axis=_axis(nu))) @ _dag(U5[nu]))
            acc += np.trace(P, axis1=-2, axis2=-1).real.mean() / 3.0
            cnt += 1
    return acc / cnt
