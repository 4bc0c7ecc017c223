// Even-odd Wilson hopping term on gfx950 (section 3 of the paper: A = 1 - kappa^2 H_eo H_oe).
//
//   (H psi)(n) = sum_mu (1 - gamma_mu) U_mu(n) psi(n+mu) + (1 + gamma_mu) U_mu(n-mu)^dag psi(n-mu)
//
// One launch applies the parity block H_{p,1-p} to a batch of vectors and fuses the
// combine x - kappa^2 (H ...), the gamma5 of A^dag = gamma5 A gamma5, an extra axpy term and
// one reduction (the CG / Lanczos dot products) into its epilogue.
//
// Work split: TPS threads per output site (1, 2 or 4).  With TPS > 1 the lanes of a site
// take different directions mu, sum their partial results with cross-lane shuffles, and
// each writes 12/TPS of the 12 output components.  This keeps enough wavefronts in flight
// when the half lattice is small (16^3 x 32 has only 64K sites per parity).
//
// Spin projection in the chiral basis: (1 -/+ gamma_mu) psi has only two independent
// spin components, h_0 = psi_0 + c_0 psi_{a_0}, h_1 = psi_1 + c_1 psi_{a_1}; the link
// multiplies those, and the lower two spins are d_0 chi_{b_0}, d_1 chi_{b_1}.  The
// coefficients c, d are units (+-1, +-i); the backward hop negates them.
#include "internal.h"
#include <hip/hip_bf16.h>

namespace scg {

// unit complex number encoded as (re, im) in {-1, 0, 1}
struct Unit {
    int re, im;
};

template <typename T>
__device__ inline cx<T> umul(Unit u, cx<T> a) {
    // (ur + i ui)(ar + i ai)
    return mk<T>((T)u.re * a.re - (T)u.im * a.im, (T)u.re * a.im + (T)u.im * a.re);
}

struct Proj {
    int a0;         // second spin index in h_0 (2 or 3); h_1 uses 5 - a0
    Unit c0, c1;    // projection coefficients (forward hop)
    int b0;         // chi index for spin 2 (spin 3 uses 1 - b0)
    Unit d0, d1;    // reconstruction coefficients (forward hop)
};

__device__ inline Proj proj_of(int mu) {
    // forward hop, (1 - gamma_mu); derived from gamma_k = [[0, -i s_k], [i s_k, 0]], gamma_4 = [[0,1],[1,0]]
    Proj p;
    switch (mu) {
        case 0: p = {3, {0, 1}, {0, 1}, 1, {0, -1}, {0, -1}}; break;
        case 1: p = {3, {1, 0}, {-1, 0}, 1, {-1, 0}, {1, 0}}; break;
        case 2: p = {2, {0, 1}, {0, -1}, 0, {0, -1}, {0, 1}}; break;
        default: p = {2, {-1, 0}, {-1, 0}, 0, {-1, 0}, {-1, 0}}; break;
    }
    return p;
}

// ---- link loads --------------------------------------------------------------------------
template <typename LT>
struct LinkLoad;

template <>
struct LinkLoad<double> {
    using Store = cx<double>;
    template <typename T>
    __device__ static inline cx<T> get(const Store* p) {
        cx<double> v = *p;
        return mk<T>((T)v.re, (T)v.im);
    }
};
template <>
struct LinkLoad<float> {
    using Store = cx<float>;
    template <typename T>
    __device__ static inline cx<T> get(const Store* p) {
        cx<float> v = *p;
        return mk<T>((T)v.re, (T)v.im);
    }
};
// BF16 links: one 32-bit word per complex entry, re in the low half, im in the high half.
struct bf16link {};
template <>
struct LinkLoad<bf16link> {
    using Store = uint32_t;
    template <typename T>
    __device__ static inline cx<T> get(const Store* p) {
        uint32_t w = *p;
        float re = __uint_as_float(w << 16);
        float im = __uint_as_float(w & 0xffff0000u);
        return mk<T>((T)re, (T)im);
    }
};

template <typename T>
struct EpiDev {
    int apply_g5, combine, red, cz_negate;
    T kappa2, sy;
    double cz_host;
    const cx<T>* x;
    const cx<T>* z;
    const double* cz_dev;
    const cx<T>* d;
    double* partials;
    const int32_t* gate_m;
    int32_t gate_i;
    const int32_t* vec_map;
    const CgVec* cg;
};

template <typename T, typename LT, int TPS>
__global__ __launch_bounds__(SCG_BLOCK) void hop_kernel(Geom g, const typename LinkLoad<LT>::Store* __restrict__ links,
                                                        const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                        int p, int nvec, int64_t nsb, EpiDev<T> e) {
    __shared__ double red_lds[SCG_BLOCK / SCG_WAVE];
    if (e.gate_m && e.gate_i > *e.gate_m) return;
    const int64_t nblk = nsb * nvec;
    const int64_t logical = xcd_logical_block(nblk);
    if (logical >= nblk) return;
    const int slot = (int)(logical % nvec);
    const int64_t sb = logical / nvec;
    const int vec = e.vec_map ? e.vec_map[slot] : slot;
    if (e.cg && (e.cg[vec].done || e.cg[vec].frozen)) return;

    const int64_t Vh = g.Vh;
    const int64_t tid = sb * SCG_BLOCK + threadIdx.x;
    const int64_t h = tid / TPS;
    const int sub = (int)(tid % TPS);
    const bool active = h < Vh;
    const cx<T>* src = in + (int64_t)vec * 12 * Vh;

    cx<T> acc[12];
#pragma unroll
    for (int c = 0; c < 12; c++) acc[c] = mk<T>(0, 0);

    if (active) {
        // coordinates of the output site (parity p, checkerboard index h)
        const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
        const int xh = (int)(h % g.Lxh);
        int64_t r = h / g.Lxh;
        const int y = (int)(r % Ly);
        r /= Ly;
        const int z = (int)(r % Lz);
        const int t = (int)(r / Lz);
        const int x = 2 * xh + ((y + z + t + p) & 1);
        const int64_t row = h - xh;  // h of the x = 0,1 pair in this (y,z,t) row

        constexpr int NMU = 4 / TPS;
#pragma unroll 1
        for (int k = 0; k < NMU; k++) {
            const int mu = (TPS == 1) ? k : sub * NMU + k;
            const Proj pr = proj_of(mu);
#pragma unroll
            for (int dir = 0; dir < 2; dir++) {
                // neighbour checkerboard index and boundary sign
                int64_t hn;
                T sign = 1;
                const int step = dir == 0 ? 1 : -1;
                if (mu == 0) {
                    const int xn = (x + step + Lx) % Lx;
                    hn = row + (xn >> 1);
                } else if (mu == 1) {
                    const int yn = (y + step + Ly) % Ly;
                    hn = xh + (int64_t)g.Lxh * (yn + (int64_t)Ly * (z + (int64_t)Lz * t));
                } else if (mu == 2) {
                    const int zn = (z + step + Lz) % Lz;
                    hn = xh + (int64_t)g.Lxh * (y + (int64_t)Ly * (zn + (int64_t)Lz * t));
                } else {
                    const int tn = (t + step + Lt) % Lt;
                    hn = xh + (int64_t)g.Lxh * (y + (int64_t)Ly * (z + (int64_t)Lz * tn));
                    if ((dir == 0 && t == Lt - 1) || (dir == 1 && t == 0)) sign = (T)g.t_bc;
                }
                // neighbour spinor, projected to two spin components
                const cx<T>* ps = src + hn;
                cx<T> psi[12];
#pragma unroll
                for (int c = 0; c < 12; c++) psi[c] = ps[(int64_t)c * Vh];
                const T s = dir == 0 ? (T)1 : (T)-1;
                const Unit c0 = {(int)s * pr.c0.re, (int)s * pr.c0.im};
                const Unit c1 = {(int)s * pr.c1.re, (int)s * pr.c1.im};
                cx<T> hp[2][3];
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    const cx<T> s2 = psi[6 + a], s3 = psi[9 + a];
                    hp[0][a] = psi[a] + umul(c0, pr.a0 == 3 ? s3 : s2);
                    hp[1][a] = psi[3 + a] + umul(c1, pr.a0 == 3 ? s2 : s3);
                }
                // link: U_mu(n) forward (this parity), U_mu(n - mu)^dag backward (other parity)
                const int lp = dir == 0 ? p : 1 - p;
                const int64_t lh = dir == 0 ? h : hn;
                const typename LinkLoad<LT>::Store* lk = links + ((int64_t)(mu * 2 + lp) * 9) * Vh + lh;
                cx<T> u[9];
#pragma unroll
                for (int c = 0; c < 9; c++) u[c] = LinkLoad<LT>::template get<T>(lk + (int64_t)c * Vh);
                cx<T> chi[2][3];
#pragma unroll
                for (int sp = 0; sp < 2; sp++)
#pragma unroll
                    for (int a = 0; a < 3; a++) {
                        cx<T> v = mk<T>(0, 0);
#pragma unroll
                        for (int b = 0; b < 3; b++)
                            v = v + (dir == 0 ? cmul(u[a * 3 + b], hp[sp][b]) : cjmul(u[b * 3 + a], hp[sp][b]));
                        chi[sp][a] = sign * v;
                    }
                const Unit d0 = {(int)s * pr.d0.re, (int)s * pr.d0.im};
                const Unit d1 = {(int)s * pr.d1.re, (int)s * pr.d1.im};
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    acc[a] = acc[a] + chi[0][a];
                    acc[3 + a] = acc[3 + a] + chi[1][a];
                    acc[6 + a] = acc[6 + a] + umul(d0, pr.b0 == 1 ? chi[1][a] : chi[0][a]);
                    acc[9 + a] = acc[9 + a] + umul(d1, pr.b0 == 1 ? chi[0][a] : chi[1][a]);
                }
            }
        }
    }

    // sum the partial results of the TPS lanes of this site
    if (TPS > 1) {
#pragma unroll
        for (int off = 1; off < TPS; off <<= 1)
#pragma unroll
            for (int c = 0; c < 12; c++) {
                acc[c].re += __shfl_xor(acc[c].re, off);
                acc[c].im += __shfl_xor(acc[c].im, off);
            }
    }

    // epilogue on this lane's 12/TPS components
    constexpr int NC = 12 / TPS;
    double part = 0.0;
    if (active) {
        const int64_t vo = (int64_t)vec * 12 * Vh;
        double czd = e.cz_host;
        if (e.cz_dev) czd = e.cz_negate ? -e.cz_dev[vec] : e.cz_dev[vec];
        const T cz = (T)czd;
#pragma unroll
        for (int c = 0; c < NC; c++) {
            const int cc = sub * NC + c;
            cx<T> v = acc[0];
#pragma unroll
            for (int q = 0; q < 12; q++)
                if (q == cc) v = acc[q];
            const int64_t idx = vo + (int64_t)cc * Vh + h;
            cx<T> y = v;
            if (e.combine) {
                const cx<T> xv = e.x[idx];
                y = mk<T>(xv.re - e.kappa2 * v.re, xv.im - e.kappa2 * v.im);
                if (e.apply_g5 && cc >= 6) y = mk<T>(-y.re, -y.im);
            }
            cx<T> o = mk<T>(e.sy * y.re, e.sy * y.im);
            if (e.z) {
                const cx<T> zv = e.z[idx];
                o = mk<T>(o.re + cz * zv.re, o.im + cz * zv.im);
            }
            out[idx] = o;
            if (e.red == 1) {
                const cx<T> dv = e.d[idx];
                part += (double)dv.re * (double)o.re + (double)dv.im * (double)o.im;
            } else if (e.red == 2) {
                part += (double)o.re * (double)o.re + (double)o.im * (double)o.im;
            }
        }
    }
    if (e.red) {
        const double s = block_sum(part, red_lds);
        if (threadIdx.x == 0) e.partials[(int64_t)vec * nsb + sb] = s;
    }
}

int hop_site_blocks(const Geom& g, int tps) { return (int)((g.Vh * tps + SCG_BLOCK - 1) / SCG_BLOCK); }

template <typename T, typename LT>
static void launch_t(const Geom& g, const void* links, const void* in, void* out, int p, int nvec, const HopEpi& epi,
                     int tps, hipStream_t s) {
    EpiDev<T> e;
    e.apply_g5 = epi.apply_g5;
    e.combine = epi.combine;
    e.red = epi.red;
    e.cz_negate = epi.cz_negate;
    e.kappa2 = (T)epi.kappa2;
    e.sy = (T)epi.sy;
    e.cz_host = epi.cz_host;
    e.x = (const cx<T>*)epi.x;
    e.z = (const cx<T>*)epi.z;
    e.cz_dev = epi.cz_dev;
    e.d = (const cx<T>*)epi.d;
    e.partials = epi.partials;
    e.gate_m = epi.gate_m;
    e.gate_i = epi.gate_i;
    e.vec_map = epi.vec_map;
    e.cg = epi.cg;
    const int64_t nsb = hop_site_blocks(g, tps);
    const int64_t grid = xcd_grid(nsb * nvec);
    using S = typename LinkLoad<LT>::Store;
    if (tps == 1)
        hipLaunchKernelGGL((hop_kernel<T, LT, 1>), dim3(grid), dim3(SCG_BLOCK), 0, s, g, (const S*)links,
                           (const cx<T>*)in, (cx<T>*)out, p, nvec, nsb, e);
    else if (tps == 2)
        hipLaunchKernelGGL((hop_kernel<T, LT, 2>), dim3(grid), dim3(SCG_BLOCK), 0, s, g, (const S*)links,
                           (const cx<T>*)in, (cx<T>*)out, p, nvec, nsb, e);
    else
        hipLaunchKernelGGL((hop_kernel<T, LT, 4>), dim3(grid), dim3(SCG_BLOCK), 0, s, g, (const S*)links,
                           (const cx<T>*)in, (cx<T>*)out, p, nvec, nsb, e);
}

void launch_hop(Prec prec, const Geom& g, const void* links, const void* in, void* out, int out_parity, int nvec,
                const HopEpi& epi, int tps, hipStream_t s) {
    if (prec == P64)
        launch_t<double, double>(g, links, in, out, out_parity, nvec, epi, tps, s);
    else if (prec == P32)
        launch_t<float, float>(g, links, in, out, out_parity, nvec, epi, tps, s);
    else
        launch_t<float, bf16link>(g, links, in, out, out_parity, nvec, epi, tps, s);
}

}  // namespace scg
