/*
 * Plain FP64 Wilson hopping term -- TEST INFRASTRUCTURE ONLY (part of the oracle).
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * The Wilson-Dirac operator in the hopping-parameter normalisation (Wilson r = 1) is
 *     (D psi)(n) = psi(n) - kappa * (H psi)(n),
 *     (H psi)(n) = sum_mu [ (1 - gamma_mu) U_mu(n) psi(n+mu) + (1 + gamma_mu) U_mu(n-mu)^dag psi(n-mu) ],
 * periodic in x, y, z and with a factor t_bc on every hop across the t boundary.
 * H only couples sites of opposite parity, so it splits into H_eo and H_oe, which is
 * the even-odd preconditioning of section 3 of the paper.  This file applies the
 * parity block H_{p,1-p}: it reads a vector on the sites of parity 1-p and writes
 * one on the sites of parity p.  Every product is written out with the full 4x4
 * gamma matrix and the full 3x3 link: no spin projection, no reordering.
 *
 * Layouts: site s = x + Lx*(y + Ly*(z + Lz*t)); a parity-p vector lists the sites of
 * parity p in increasing s, which is index s/2 because Lx is even; each site holds
 * [spin 4][colour 3] complex numbers.  Links U[mu][s][a][b], complex.
 */
#include <complex.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex cplx;

/* Euclidean Hermitian chiral basis:
 *   gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]  (k = 1, 2, 3 -> mu = 0, 1, 2)
 *   gamma_4 = [[0, 1], [1, 0]]                   (mu = 3)
 * so that gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 = diag(1, 1, -1, -1). */
static void gamma_of(int mu, cplx g[4][4])
{
    cplx sigma[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++)
            g[a][b] = 0;
    if (mu == 3) {
        for (int a = 0; a < 2; a++) {
            g[a][a + 2] = 1;
            g[a + 2][a] = 1;
        }
        return;
    }
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
            g[a][b + 2] = -I * sigma[mu][a][b];
            g[a + 2][b] = I * sigma[mu][a][b];
        }
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* out = H_{p,1-p} in, for nvec vectors stored one after another. */
void oracle_hop(const int32_t* dims, int32_t t_bc, const cplx* U, const cplx* in, cplx* out,
                int32_t out_parity, int64_t nvec)
{
    const int64_t L[4] = {dims[0], dims[1], dims[2], dims[3]};
    const int64_t V = L[0] * L[1] * L[2] * L[3];
    const int64_t Vh = V / 2;
    const int64_t Lxh = L[0] / 2;
    cplx one_minus[4][4][4], one_plus[4][4][4];
    for (int mu = 0; mu < 4; mu++) {
        cplx g[4][4];
        gamma_of(mu, g);
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++) {
                cplx id = (a == b) ? 1.0 : 0.0;
                one_minus[mu][a][b] = id - g[a][b];
                one_plus[mu][a][b] = id + g[a][b];
            }
    }

    for (int64_t iv = 0; iv < nvec; iv++) {
        const cplx* src = in + iv * Vh * 12;
        cplx* dst = out + iv * Vh * 12;
#pragma omp parallel for schedule(static) if (Vh >= 4096)  /* small lattices: thread start-up costs more than the sites */
        for (int64_t h = 0; h < Vh; h++) {
            int64_t rest = h / Lxh;
            int64_t c[4];
            c[1] = rest % L[1];
            c[2] = (rest / L[1]) % L[2];
            c[3] = rest / (L[1] * L[2]);
            c[0] = 2 * (h % Lxh) + ((c[1] + c[2] + c[3] + out_parity) & 1);
            const int64_t s = c[0] + L[0] * (c[1] + L[1] * (c[2] + L[2] * c[3]));

            cplx acc[4][3];
            for (int sp = 0; sp < 4; sp++)
                for (int a = 0; a < 3; a++)
                    acc[sp][a] = 0;

            for (int mu = 0; mu < 4; mu++) {
                for (int dir = 0; dir < 2; dir++) {   /* 0: forward, 1: backward */
                    int64_t nb[4] = {c[0], c[1], c[2], c[3]};
                    double sign = 1.0;
                    if (dir == 0) {
                        nb[mu] = (c[mu] + 1) % L[mu];
                        if (mu == 3 && c[3] == L[3] - 1) sign = (double)t_bc;
                    } else {
                        nb[mu] = (c[mu] + L[mu] - 1) % L[mu];
                        if (mu == 3 && c[3] == 0) sign = (double)t_bc;
                    }
                    const int64_t sn = nb[0] + L[0] * (nb[1] + L[1] * (nb[2] + L[2] * nb[3]));
                    const cplx* psi = src + (sn / 2) * 12;

                    /* link: U_mu(n) forward, U_mu(n - mu)^dag backward */
                    cplx link[3][3];
                    if (dir == 0) {
                        const cplx* u = U + (mu * V + s) * 9;
                        for (int a = 0; a < 3; a++)
                            for (int b = 0; b < 3; b++)
                                link[a][b] = u[a * 3 + b];
                    } else {
                        const cplx* u = U + (mu * V + sn) * 9;
                        for (int a = 0; a < 3; a++)
                            for (int b = 0; b < 3; b++)
                                link[a][b] = conj(u[b * 3 + a]);
                    }

                    /* chi[spin][a] = sum_b link[a][b] psi[spin][b] */
                    cplx chi[4][3];
                    for (int sp = 0; sp < 4; sp++)
                        for (int a = 0; a < 3; a++) {
                            cplx t = 0;
                            for (int b = 0; b < 3; b++)
                                t += link[a][b] * psi[sp * 3 + b];
                            chi[sp][a] = t;
                        }

                    /* acc[sp][a] += sign * sum_sp2 (1 -/+ gamma_mu)[sp][sp2] chi[sp2][a] */
                    cplx (*P)[4] = (dir == 0) ? one_minus[mu] : one_plus[mu];
                    for (int sp = 0; sp < 4; sp++)
                        for (int a = 0; a < 3; a++) {
                            cplx t = 0;
                            for (int sp2 = 0; sp2 < 4; sp2++)
                                t += P[sp][sp2] * chi[sp2][a];
                            acc[sp][a] += sign * t;
                        }
                }
            }
            for (int sp = 0; sp < 4; sp++)
                for (int a = 0; a < 3; a++)
                    dst[h * 12 + sp * 3 + a] = acc[sp][a];
        }
    }
}
