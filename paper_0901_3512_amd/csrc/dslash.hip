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
#include <cstdlib>
#include <stdexcept>
#include <type_traits>

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
    static constexpr int NE = 9;  // stored complex entries per link
    template <typename T>
    __device__ static inline cx<T> get(const Store* p) {
        cx<double> v = *p;
        return mk<T>((T)v.re, (T)v.im);
    }
    template <typename T>
    __device__ static inline cx<T> get32(const Store* base, uint32_t idx) {
        const cx<double> v = *(const Store*)((const char*)base + idx * (uint32_t)sizeof(Store));
        return mk<T>((T)v.re, (T)v.im);
    }
    template <typename T>
    __device__ static inline cx<T> cvt(Store v) { return mk<T>((T)v.re, (T)v.im); }
};
template <>
struct LinkLoad<float> {
    using Store = cx<float>;
    static constexpr int NE = 9;
    template <typename T>
    __device__ static inline cx<T> get(const Store* p) {
        cx<float> v = *p;
        return mk<T>((T)v.re, (T)v.im);
    }
    template <typename T>
    __device__ static inline cx<T> get32(const Store* base, uint32_t idx) {
        const cx<float> v = *(const Store*)((const char*)base + idx * (uint32_t)sizeof(Store));
        return mk<T>((T)v.re, (T)v.im);
    }
    template <typename T>
    __device__ static inline cx<T> cvt(Store v) { return mk<T>((T)v.re, (T)v.im); }
};
// BF16 links: one 32-bit word per complex entry, re in the low half, im in the high half.
struct bf16link {};
template <>
struct LinkLoad<bf16link> {
    using Store = uint32_t;
    static constexpr int NE = 9;
    template <typename T>
    __device__ static inline cx<T> get(const Store* p) {
        uint32_t w = *p;
        float re = __uint_as_float(w << 16);
        float im = __uint_as_float(w & 0xffff0000u);
        return mk<T>((T)re, (T)im);
    }
    template <typename T>
    __device__ static inline cx<T> get32(const Store* base, uint32_t idx) {
        const uint32_t w = *(const Store*)((const char*)base + idx * (uint32_t)sizeof(Store));
        return mk<T>((T)__uint_as_float(w << 16), (T)__uint_as_float(w & 0xffff0000u));
    }
    template <typename T>
    __device__ static inline cx<T> cvt(Store w) { return mk<T>((T)__uint_as_float(w << 16), (T)__uint_as_float(w & 0xffff0000u)); }
};

// Special-unitary links stored as their first two rows (6 complex entries); the third row is
// rebuilt in registers as conj(row 0 x row 1), which holds for every U in SU(3).
template <typename S>
struct su3rows {};
template <typename S>
struct LinkLoad<su3rows<S>> {
    using Store = cx<S>;
    static constexpr int NE = 6;
    template <typename T>
    __device__ static inline cx<T> get(const Store* p) {
        const cx<S> v = *p;
        return mk<T>((T)v.re, (T)v.im);
    }
    template <typename T>
    __device__ static inline cx<T> get32(const Store* base, uint32_t idx) {
        const cx<S> v = *(const Store*)((const char*)base + idx * (uint32_t)sizeof(Store));
        return mk<T>((T)v.re, (T)v.im);
    }
    template <typename T>
    __device__ static inline cx<T> cvt(Store v) { return mk<T>((T)v.re, (T)v.im); }
};
template <typename T>
__device__ inline cx<T> conjc(cx<T> a) { return mk<T>(a.re, -a.im); }
template <typename T>
__device__ inline void su3_third_row(cx<T> u[9]) {
    u[6] = conjc(cmul(u[1], u[5]) - cmul(u[2], u[4]));
    u[7] = conjc(cmul(u[2], u[3]) - cmul(u[0], u[5]));
    u[8] = conjc(cmul(u[0], u[4]) - cmul(u[1], u[3]));
}
// U of one link: entries c * Vh apart from lk + lane_off (32-bit offsets)
template <typename T, typename LT>
__device__ inline void load_u32(const typename LinkLoad<LT>::Store* __restrict__ lk, uint32_t lane_off, uint32_t Vh, cx<T> u[9]) {
    constexpr int NE = LinkLoad<LT>::NE;
#pragma unroll
    for (int c = 0; c < NE; c++) u[c] = LinkLoad<LT>::template get32<T>(lk, lane_off + (uint32_t)c * Vh);
    if constexpr (NE == 6) su3_third_row(u);
}

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
    const double* kappa2_dev;
    cx<double>* X;     // red 3: CG iterate (always FP64)
    cx<T>* R;          // red 3: CG residual
};

// move every per-configuration pointer of a launch to configuration blockIdx.z
template <typename T, typename PL, typename PI, typename PO>
__device__ inline void zoff_hop(int64_t cs, PL& links, PI& in, PO& out, EpiDev<T>& e) {
    if (cs == 0) return;
    links = zoff(links, cs);
    in = zoff(in, cs);
    out = zoff(out, cs);
    e.x = zoff(e.x, cs);
    e.z = zoff(e.z, cs);
    e.cz_dev = zoff(e.cz_dev, cs);
    e.d = zoff(e.d, cs);
    e.partials = zoff(e.partials, cs);
    e.gate_m = zoff(e.gate_m, cs);
    e.vec_map = zoff(e.vec_map, cs);
    e.cg = zoff(e.cg, cs);
    e.kappa2_dev = zoff(e.kappa2_dev, cs);
    e.X = zoff(e.X, cs);
    e.R = zoff(e.R, cs);
}

// the per-vector coefficient of the epilogue: alpha of the vector's CG record for the fused CG
// update, else cz of the extra vector term
template <typename T>
__device__ inline double epi_coef(const EpiDev<T>& e, int vec) {
    if (e.red == 3) return e.cg[vec].a;
    if (e.cz_dev) return e.cz_negate ? -e.cz_dev[vec] : e.cz_dev[vec];
    return e.cz_host;
}

// Site-block visiting order of the two-lanes-per-site kernels.  A site block (128 sites) lies in
// one t-slice when bps = sites per slice / 128 is whole; blocks are then visited in tiles of
// SB_TILE_T consecutive slices with t fastest, so that the t-neighbours of a block were read by
// the block just before it (instead of a whole slice of blocks earlier) and the z-neighbours a
// few blocks away: both stay in L2.  With bps = 0 the order is the plain one.
constexpr int SB_TILE_T = 4;
__device__ inline int64_t sb_order(int64_t p, int64_t bps, int Lt) {
    if (bps <= 0) return p;
    const int64_t tile = bps * SB_TILE_T;
    const int64_t t0 = (p / tile) * SB_TILE_T;
    const int64_t r = p % tile;
    const int64_t T = (t0 + SB_TILE_T <= Lt) ? SB_TILE_T : (Lt - t0);
    return (t0 + r % T) * bps + r / T;
}

// neighbour (checkerboard index) of site (x,y,z,t) with index h in direction mu, step +-1, and the
// boundary sign of that hop
struct Nb {
    int64_t h;
    int sign;
};
__device__ inline Nb neighbour(const Geom& g, int mu, int step, int x, int y, int z, int t, int xh, int64_t row) {
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
    Nb n;
    n.sign = 1;
    if (mu == 0) {
        const int xn = (x + step + Lx) % Lx;
        n.h = row + (xn >> 1);
    } else if (mu == 1) {
        const int yn = (y + step + Ly) % Ly;
        n.h = xh + (int64_t)g.Lxh * (yn + (int64_t)Ly * (z + (int64_t)Lz * t));
    } else if (mu == 2) {
        const int zn = (z + step + Lz) % Lz;
        n.h = xh + (int64_t)g.Lxh * (y + (int64_t)Ly * (zn + (int64_t)Lz * t));
    } else {
        const int tn = (t + step + Lt) % Lt;
        n.h = xh + (int64_t)g.Lxh * (y + (int64_t)Ly * (z + (int64_t)Lz * tn));
        if ((step == 1 && t == Lt - 1) || (step == -1 && t == 0)) n.sign = g.t_bc;
    }
    return n;
}

template <typename T, typename LT>
__device__ inline void load_link(const typename LinkLoad<LT>::Store* links, int mu, int par, int64_t h, int64_t Vh, cx<T> u[9]) {
    constexpr int NE = LinkLoad<LT>::NE;
    const typename LinkLoad<LT>::Store* lk = links + ((int64_t)(mu * 2 + par) * NE) * Vh + h;
#pragma unroll
    for (int c = 0; c < NE; c++) u[c] = LinkLoad<LT>::template get<T>(lk + (int64_t)c * Vh);
    if constexpr (NE == 6) su3_third_row(u);
}

// acc += (1 -/+ gamma_mu) U psi(neighbour) for one hop (dir 0: forward with U_mu(n), 1: backward
// with U_mu(n - mu)^dag)
template <typename T>
__device__ inline void hop_accumulate(const cx<T>* __restrict__ src, int64_t hn, int64_t Vh, const Proj& pr, int dir, T sign,
                                      const cx<T> u[9], cx<T> acc[12]) {
    // h_0 = psi_0 + c_0 psi_{a0}, h_1 = psi_1 + c_1 psi_{a1}: load the spins pairwise
    const cx<T>* ps = src + hn;
    const int s = dir == 0 ? 1 : -1;
    const Unit c0 = {s * pr.c0.re, s * pr.c0.im};
    const Unit c1 = {s * pr.c1.re, s * pr.c1.im};
    const int64_t oa0 = (int64_t)(3 * pr.a0) * Vh, oa1 = (int64_t)(3 * (5 - pr.a0)) * Vh;
    cx<T> hp[2][3];
#pragma unroll
    for (int a = 0; a < 3; a++) hp[0][a] = ps[(int64_t)a * Vh] + umul(c0, ps[oa0 + (int64_t)a * Vh]);
#pragma unroll
    for (int a = 0; a < 3; a++) hp[1][a] = ps[(int64_t)(3 + a) * Vh] + umul(c1, ps[oa1 + (int64_t)a * Vh]);
    cx<T> chi[2][3];
#pragma unroll
    for (int sp = 0; sp < 2; sp++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            cx<T> v = mk<T>(0, 0);
#pragma unroll
            for (int b = 0; b < 3; b++) v = v + (dir == 0 ? cmul(u[a * 3 + b], hp[sp][b]) : cjmul(u[b * 3 + a], hp[sp][b]));
            chi[sp][a] = sign * v;
        }
    const Unit d0 = {s * pr.d0.re, s * pr.d0.im};
    const Unit d1 = {s * pr.d1.re, s * pr.d1.im};
#pragma unroll
    for (int a = 0; a < 3; a++) {
        acc[a] = acc[a] + chi[0][a];
        acc[3 + a] = acc[3 + a] + chi[1][a];
        acc[6 + a] = acc[6 + a] + umul(d0, pr.b0 == 1 ? chi[1][a] : chi[0][a]);
        acc[9 + a] = acc[9 + a] + umul(d1, pr.b0 == 1 ? chi[0][a] : chi[1][a]);
    }
}

constexpr int HOP_MAX_VB = 32;

// One workgroup = 256/TPS output sites x a group of vb vectors.  The links of the site's
// directions are loaded once and, when they fit in registers (HOIST), reused for every vector
// of the group; the vectors of the group are processed one after another so that the
// neighbour spinors of consecutive sites stay in L2 as for a single vector.
template <typename T, typename LT, int TPS, bool HOIST>
__global__ __launch_bounds__(SCG_BLOCK) void hop_kernel(Geom g, const typename LinkLoad<LT>::Store* __restrict__ links,
                                                        const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                        int p, int nvec, int vb, int64_t nsb, EpiDev<T> e, int64_t cs) {
    constexpr int NMU = 4 / TPS;
    __shared__ double red_lds[HOP_MAX_VB * (SCG_BLOCK / SCG_WAVE)];
    zoff_hop(cs, links, in, out, e);
    if (e.gate_m && e.gate_i > *e.gate_m) return;
    if (e.kappa2_dev) e.kappa2 = (T)*e.kappa2_dev;
    const int nvg = (nvec + vb - 1) / vb;
    const int64_t nblk = nsb * nvg;
    const int64_t logical = xcd_logical_block(nblk);
    if (logical >= nblk) return;
    const int vg = (int)(logical % nvg);
    const int64_t sb = logical / nvg;

    const int64_t Vh = g.Vh;
    const int64_t tid = sb * SCG_BLOCK + threadIdx.x;
    const int64_t h = tid / TPS;
    const int sub = (int)(tid % TPS);
    const bool active = h < Vh;

    // site coordinates, neighbours and (hoisted) links of this lane's directions
    Nb nb[NMU][2];
    cx<T> uh[HOIST ? NMU : 1][2][9];
    int mus[NMU];
    if (active) {
        const int xh = (int)(h % g.Lxh);
        int64_t r = h / g.Lxh;
        const int y = (int)(r % g.L[1]);
        r /= g.L[1];
        const int z = (int)(r % g.L[2]);
        const int t = (int)(r / g.L[2]);
        const int x = 2 * xh + ((y + z + t + p) & 1);
        const int64_t row = h - xh;
#pragma unroll
        for (int k = 0; k < NMU; k++) {
            const int mu = (TPS == 1) ? k : sub * NMU + k;
            mus[k] = mu;
            nb[k][0] = neighbour(g, mu, 1, x, y, z, t, xh, row);
            nb[k][1] = neighbour(g, mu, -1, x, y, z, t, xh, row);
            if constexpr (HOIST) {
                load_link<T, LT>(links, mu, p, h, Vh, uh[k][0]);
                load_link<T, LT>(links, mu, 1 - p, nb[k][1].h, Vh, uh[k][1]);
            }
        }
    }

    constexpr int NC = 12 / TPS;
    for (int vi = 0; vi < vb; vi++) {
        const int slot = vg * vb + vi;
        if (slot >= nvec) break;
        const int vec = e.vec_map ? e.vec_map[slot] : slot;
        if (vec < 0 || (e.cg && (e.cg[vec].done || e.cg[vec].frozen))) continue;
        const cx<T>* src = in + (int64_t)vec * 12 * Vh;

        cx<T> acc[12];
#pragma unroll
        for (int c = 0; c < 12; c++) acc[c] = mk<T>(0, 0);
        if (active) {
#pragma unroll
            for (int k = 0; k < NMU; k++) {
                const Proj pr = proj_of(mus[k]);
#pragma unroll
                for (int dir = 0; dir < 2; dir++) {
                    if constexpr (HOIST) {
                        hop_accumulate<T>(src, nb[k][dir].h, Vh, pr, dir, (T)nb[k][dir].sign, uh[k][dir], acc);
                    } else {
                        cx<T> u[9];
                        load_link<T, LT>(links, mus[k], dir == 0 ? p : 1 - p, dir == 0 ? h : nb[k][1].h, Vh, u);
                        hop_accumulate<T>(src, nb[k][dir].h, Vh, pr, dir, (T)nb[k][dir].sign, u, acc);
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
            // wave sum now, the waves of the workgroup after the vector loop (no barrier per vector)
            for (int off = SCG_WAVE / 2; off > 0; off >>= 1) part += __shfl_xor(part, off);
            if ((threadIdx.x % SCG_WAVE) == 0) red_lds[vi * (SCG_BLOCK / SCG_WAVE) + threadIdx.x / SCG_WAVE] = part;
        }
    }
    if (e.red) {
        __syncthreads();
        const int vi = threadIdx.x;
        if (vi < vb) {
            const int slot = vg * vb + vi;
            if (slot < nvec) {
                const int vec = e.vec_map ? e.vec_map[slot] : slot;
                if (vec >= 0 && !(e.cg && (e.cg[vec].done || e.cg[vec].frozen))) {
                    double s = 0.0;
                    for (int w = 0; w < SCG_BLOCK / SCG_WAVE; w++) s += red_lds[vi * (SCG_BLOCK / SCG_WAVE) + w];
                    e.partials[(int64_t)vec * nsb + sb] = s;
                }
            }
        }
    }
}

// load base[idx] with a 32-bit byte offset, so that a uniform base stays in SGPRs and only the
// offset occupies a VGPR (the global_load saddr form)
template <typename T>
__device__ inline T ld32(const T* base, uint32_t idx) {
    return *(const T*)((const char*)base + idx * (uint32_t)sizeof(T));
}
template <typename T>
__device__ inline void st32(T* base, uint32_t idx, T v) {
    *(T*)((char*)base + idx * (uint32_t)sizeof(T)) = v;
}

// Epilogue of the two-lanes-per-site kernels for one vector (NC of the 12 components, from the
// component offset in lo): out = sy*[gamma5](x - kappa^2 v) +
// cz z, with the reduction partial of Re d^dag out or |out|^2.  Every operand load is issued before
// the first use (independent batches of NC), so the epilogue costs one memory round trip
// instead of one per component and operand.
// red 3 (the CG update fused into the last hop of q = M p): q = out is not stored; with
// a = cz (the vector's alpha), X += a p (p = d), R -= a q, and the partial is |R|^2 -- the same
// arithmetic, in the same precisions, as the separate update kernel.
template <typename T, int NC = 6, bool CGU = false>
__device__ inline double epilogue2(const EpiDev<T>& e, const cx<T>* v, int bwd, size_t vo, int64_t Vh, uint32_t lo, cx<T>* __restrict__ out,
                                   double cz) {
    const T czt = (T)cz;
    cx<T> xv[NC], zv[NC], dv[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) xv[c] = zv[c] = dv[c] = mk<T>(0, 0);
    if (e.combine) {
#pragma unroll
        for (int c = 0; c < NC; c++) xv[c] = ld32(e.x + vo + (size_t)c * Vh, lo);
    }
    if (e.z) {
#pragma unroll
        for (int c = 0; c < NC; c++) zv[c] = ld32(e.z + vo + (size_t)c * Vh, lo);
    }
    if (CGU || e.red == 1) {
#pragma unroll
        for (int c = 0; c < NC; c++) dv[c] = ld32(e.d + vo + (size_t)c * Vh, lo);
    }
    double part = 0.0;
    if constexpr (CGU) {
        cx<T> rv[NC];
        cx<double> sv[NC];
#pragma unroll
        for (int c = 0; c < NC; c++) {
            rv[c] = ld32(e.R + vo + (size_t)c * Vh, lo);
            sv[c] = ld32(e.X + vo + (size_t)c * Vh, lo);
        }
#pragma unroll
        for (int c = 0; c < NC; c++) {
            const cx<T> w = v[c];
            cx<T> y = mk<T>(xv[c].re - e.kappa2 * w.re, xv[c].im - e.kappa2 * w.im);
            if (e.apply_g5 && bwd) y = mk<T>(-y.re, -y.im);
            const cx<T> q = mk<T>(e.sy * y.re, e.sy * y.im);
            st32(e.X + vo + (size_t)c * Vh, lo, mk<double>(sv[c].re + cz * dv[c].re, sv[c].im + cz * dv[c].im));
            const cx<T> rn = mk<T>((T)(rv[c].re - cz * q.re), (T)(rv[c].im - cz * q.im));
            st32(e.R + vo + (size_t)c * Vh, lo, rn);
            part += (double)rn.re * rn.re + (double)rn.im * rn.im;
        }
        return part;
    }
#pragma unroll
    for (int c = 0; c < NC; c++) {
        const cx<T> w = v[c];
        cx<T> y = w;
        if (e.combine) {
            y = mk<T>(xv[c].re - e.kappa2 * w.re, xv[c].im - e.kappa2 * w.im);
            if (e.apply_g5 && bwd) y = mk<T>(-y.re, -y.im);
        }
        cx<T> o = mk<T>(e.sy * y.re, e.sy * y.im);
        if (e.z) o = mk<T>(o.re + czt * zv[c].re, o.im + czt * zv[c].im);
        st32(out + vo + (size_t)c * Vh, lo, o);
        if (e.red == 1)
            part += (double)dv[c].re * (double)o.re + (double)dv[c].im * (double)o.im;
        else if (e.red == 2)
            part += (double)o.re * (double)o.re + (double)o.im * (double)o.im;
    }
    return part;
}

// the same hop with a wave-uniform runtime direction mu (coefficients from proj_of(mu))
template <typename T>
__device__ inline cx<T> fma_u(T sd, Unit u, cx<T> b, cx<T> a) {
    const cx<T> ub = umul(u, b);
    return mk<T>(fma(sd, ub.re, a.re), fma(sd, ub.im, a.im));
}
template <typename T, typename LT>
__device__ inline void hop_dir_rt(const cx<T>* __restrict__ src, const typename LinkLoad<LT>::Store* __restrict__ links, int mu,
                                  uint32_t hn, uint32_t hl, uint32_t lpar, uint32_t Vh, int bwd, T sd, T sign, cx<T> acc[12]) {
    const Proj pr = proj_of(mu);
    const uint32_t a0 = (uint32_t)pr.a0, a1 = 5u - a0;
    cx<T> hp[2][3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        hp[0][a] = fma_u(sd, pr.c0, ld32(src + (size_t)(3 * a0 + a) * Vh, hn), ld32(src + (size_t)a * Vh, hn));
        hp[1][a] = fma_u(sd, pr.c1, ld32(src + (size_t)(3 * a1 + a) * Vh, hn), ld32(src + (size_t)(3 + a) * Vh, hn));
        hp[0][a] = sign * hp[0][a];
        hp[1][a] = sign * hp[1][a];
    }
    constexpr int NE = LinkLoad<LT>::NE;
    const typename LinkLoad<LT>::Store* __restrict__ lk = links + (size_t)(mu * 2) * NE * Vh;
    cx<T> u[9];
    load_u32<T, LT>(lk, lpar * (uint32_t)NE * Vh + hl, Vh, u);
    cx<T> chi[2][3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        cx<T> c0 = mk<T>(0, 0), c1 = mk<T>(0, 0);
#pragma unroll
        for (int b = 0; b < 3; b++) {
            // M[a][b] = U[a][b] (forward) or conj(U[b][a]) (backward)
            cx<T> m = bwd ? u[b * 3 + a] : u[a * 3 + b];
            if (bwd) m.im = -m.im;
            c0 = c0 + cmul(m, hp[0][b]);
            c1 = c1 + cmul(m, hp[1][b]);
        }
        chi[0][a] = c0;
        chi[1][a] = c1;
    }
    const bool b1 = pr.b0 == 1;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        acc[a] = acc[a] + chi[0][a];
        acc[3 + a] = acc[3 + a] + chi[1][a];
        acc[6 + a] = fma_u(sd, pr.d0, b1 ? chi[1][a] : chi[0][a], acc[6 + a]);
        acc[9 + a] = fma_u(sd, pr.d1, b1 ? chi[0][a] : chi[1][a], acc[9 + a]);
    }
}

// Lean variant: two lanes per site, the even lane takes the four forward hops and the odd lane the
// four backward hops (the direction enters as a sign and as U versus U^dag); the mu loop is
// wave-uniform.
// UNR: directions per pass of the mu loop.  1 keeps one direction's loads in flight (fewest
// registers, for grids with many waves per SIMD); 2 and 4 issue the loads of several directions
// together, which shortens the chain of dependent memory round trips when the half lattice gives
// only a couple of waves per SIMD.
template <typename T, typename LT, bool ONE, int UNR>
__global__ __launch_bounds__(SCG_BLOCK) void hop_lean_kernel(Geom g, const typename LinkLoad<LT>::Store* __restrict__ links,
                                                             const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                             int p, int nvec, int vb, int64_t nsb, EpiDev<T> e, int64_t cs,
                                                             int64_t bps) {
    __shared__ double red_lds[HOP_MAX_VB * (SCG_BLOCK / SCG_WAVE)];
    zoff_hop(cs, links, in, out, e);
    if (e.gate_m && e.gate_i > *e.gate_m) return;
    if (e.kappa2_dev) e.kappa2 = (T)*e.kappa2_dev;
    const int nvg = (nvec + vb - 1) / vb;
    const int64_t nblk = nsb * nvg;
    const int64_t logical = xcd_logical_block(nblk);
    if (logical >= nblk) return;
    const int vg = (int)(logical % nvg);
    const int64_t sb = logical / nvg;   // position in the visiting order (partials are indexed by it)
    const int64_t Vh = g.Vh;
    const int64_t tid = sb_order(sb, bps, g.L[3]) * SCG_BLOCK + threadIdx.x;
    const int64_t h = tid >> 1;
    const int bwd = (int)(tid & 1);
    const bool active = h < Vh;
    const int step = bwd ? -1 : 1;
    const T sd = bwd ? (T)-1 : (T)1;

    int x = 0, y = 0, z = 0, t = 0, xh = 0;
    int64_t row = 0;
    if (active) {
        xh = (int)(h % g.Lxh);
        int64_t r = h / g.Lxh;
        y = (int)(r % g.L[1]);
        r /= g.L[1];
        z = (int)(r % g.L[2]);
        t = (int)(r / g.L[2]);
        x = 2 * xh + ((y + z + t + p) & 1);
        row = h - xh;
    }
    const uint32_t lpar = bwd ? 1u - (uint32_t)p : (uint32_t)p;
    const uint32_t Vh32 = (uint32_t)Vh, h32 = (uint32_t)h;

    // ONE: one vector per workgroup (vb == 1); the vectors of a site block are adjacent
    // workgroups on one XCD and share the links through its L2
    const int nloop = ONE ? 1 : vb;
    for (int vi = 0; vi < nloop; vi++) {
        const int slot = vg * vb + vi;
        if (slot >= nvec) break;
        const int vec = e.vec_map ? e.vec_map[slot] : slot;
        if (vec < 0 || (e.cg && (e.cg[vec].done || e.cg[vec].frozen))) continue;
        const cx<T>* src = in + (size_t)vec * 12 * Vh;
        cx<T> acc[12];
#pragma unroll
        for (int c = 0; c < 12; c++) acc[c] = mk<T>(0, 0);
        if (active) {
            // UNR directions per pass (mu is the same for every lane)
#pragma unroll 1
            for (int mu0 = 0; mu0 < 4; mu0 += UNR) {
#pragma unroll
                for (int u = 0; u < UNR; u++) {
                    const int mu = mu0 + u;
                    const Nb n = neighbour(g, mu, step, x, y, z, t, xh, row);
                    const uint32_t hn = (uint32_t)n.h;
                    hop_dir_rt<T, LT>(src, links, mu, hn, bwd ? hn : h32, lpar, Vh32, bwd, sd, (T)n.sign, acc);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 12; c++) {
            acc[c].re += __shfl_xor(acc[c].re, 1);
            acc[c].im += __shfl_xor(acc[c].im, 1);
        }
        double part = 0.0;
        if (active) {
            const size_t vo = (size_t)vec * 12 * Vh;
            const double czd = epi_coef(e, vec);
            const uint32_t lo = (uint32_t)bwd * 6u * Vh32 + h32;
            cx<T> v[6];
#pragma unroll
            for (int c = 0; c < 6; c++) v[c] = bwd ? acc[6 + c] : acc[c];
            part = epilogue2<T>(e, v, bwd, vo, Vh, lo, out, czd);
        }
        if (e.red) {
            for (int off = SCG_WAVE / 2; off > 0; off >>= 1) part += __shfl_xor(part, off);
            if ((threadIdx.x % SCG_WAVE) == 0) red_lds[vi * (SCG_BLOCK / SCG_WAVE) + threadIdx.x / SCG_WAVE] = part;
        }
    }
    if (e.red) {
        __syncthreads();
        const int vi = threadIdx.x;
        if (vi < vb) {
            const int slot = vg * vb + vi;
            if (slot < nvec) {
                const int vec = e.vec_map ? e.vec_map[slot] : slot;
                if (vec >= 0 && !(e.cg && (e.cg[vec].done || e.cg[vec].frozen))) {
                    double s = 0.0;
                    for (int w = 0; w < SCG_BLOCK / SCG_WAVE; w++) s += red_lds[vi * (SCG_BLOCK / SCG_WAVE) + w];
                    e.partials[(int64_t)vec * nsb + sb] = s;
                }
            }
        }
    }
}

// Several vectors per lane: the link of a direction is loaded once and applied to the NV vectors
// of the workgroup's group, so a multi-vector launch reads the links once per site block instead
// of once per vector.  Two lanes per site as in the lean kernel.
template <typename T, typename LT, int NV>
__global__ __launch_bounds__(SCG_BLOCK) void hop_multi_kernel(Geom g, const typename LinkLoad<LT>::Store* __restrict__ links,
                                                              const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                              int p, int nvec, int64_t nsb, EpiDev<T> e, int64_t cs, int64_t bps) {
    __shared__ double red_lds[NV * (SCG_BLOCK / SCG_WAVE)];
    zoff_hop(cs, links, in, out, e);
    if (e.gate_m && e.gate_i > *e.gate_m) return;
    if (e.kappa2_dev) e.kappa2 = (T)*e.kappa2_dev;
    const int nvg = (nvec + NV - 1) / NV;
    const int64_t nblk = nsb * nvg;
    const int64_t logical = xcd_logical_block(nblk);
    if (logical >= nblk) return;
    const int vg = (int)(logical % nvg);
    const int64_t sb = logical / nvg;   // position in the visiting order (partials are indexed by it)
    const int64_t Vh = g.Vh;
    const int64_t tid = sb_order(sb, bps, g.L[3]) * SCG_BLOCK + threadIdx.x;
    const int64_t h = tid >> 1;
    const int bwd = (int)(tid & 1);
    const bool active = h < Vh;
    const int step = bwd ? -1 : 1;
    const T sd = bwd ? (T)-1 : (T)1;

    int x = 0, y = 0, z = 0, t = 0, xh = 0;
    int64_t row = 0;
    if (active) {
        xh = (int)(h % g.Lxh);
        int64_t r = h / g.Lxh;
        y = (int)(r % g.L[1]);
        r /= g.L[1];
        z = (int)(r % g.L[2]);
        t = (int)(r / g.L[2]);
        x = 2 * xh + ((y + z + t + p) & 1);
        row = h - xh;
    }
    const uint32_t lpar = bwd ? 1u - (uint32_t)p : (uint32_t)p;
    const uint32_t Vh32 = (uint32_t)Vh, h32 = (uint32_t)h;

    // the group's vectors (-1: empty slot, or a vector whose CG is done or frozen)
    int vec[NV];
    bool any = false;
#pragma unroll
    for (int v = 0; v < NV; v++) {
        const int slot = vg * NV + v;
        int q = -1;
        if (slot < nvec) {
            q = e.vec_map ? e.vec_map[slot] : slot;
            if (q >= 0 && e.cg && (e.cg[q].done || e.cg[q].frozen)) q = -1;
        }
        vec[v] = q;
        any = any || q >= 0;
    }
    if (!any) return;  // uniform over the workgroup

    cx<T> acc[NV][12];
#pragma unroll
    for (int v = 0; v < NV; v++)
#pragma unroll
        for (int c = 0; c < 12; c++) acc[v][c] = mk<T>(0, 0);
    if (active) {
#pragma unroll 1
        for (int mu = 0; mu < 4; mu++) {
            const Nb n = neighbour(g, mu, step, x, y, z, t, xh, row);
            const uint32_t hn = (uint32_t)n.h;
            const uint32_t hl = bwd ? hn : h32;
            const Proj pr = proj_of(mu);
            const uint32_t a0 = (uint32_t)pr.a0, a1 = 5u - a0;
            // M[a][b] = U[a][b] (forward) or conj(U[b][a]) (backward), loaded once
            constexpr int NE = LinkLoad<LT>::NE;
            const typename LinkLoad<LT>::Store* __restrict__ lk = links + (size_t)(mu * 2) * NE * Vh;
            cx<T> u[9], m[9];
            load_u32<T, LT>(lk, lpar * (uint32_t)NE * Vh32 + hl, Vh32, u);
#pragma unroll
            for (int a = 0; a < 3; a++)
#pragma unroll
                for (int b = 0; b < 3; b++) {
                    cx<T> v = bwd ? u[b * 3 + a] : u[a * 3 + b];
                    if (bwd) v.im = -v.im;
                    m[a * 3 + b] = v;
                }
            const T sign = (T)n.sign;
            const bool b1 = pr.b0 == 1;
#pragma unroll
            for (int v = 0; v < NV; v++) {
                if (vec[v] < 0) continue;
                const cx<T>* src = in + (size_t)vec[v] * 12 * Vh;
                cx<T> hp[2][3];
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    hp[0][a] = sign * fma_u(sd, pr.c0, ld32(src + (size_t)(3 * a0 + a) * Vh, hn), ld32(src + (size_t)a * Vh, hn));
                    hp[1][a] = sign * fma_u(sd, pr.c1, ld32(src + (size_t)(3 * a1 + a) * Vh, hn), ld32(src + (size_t)(3 + a) * Vh, hn));
                }
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    cx<T> c0 = mk<T>(0, 0), c1 = mk<T>(0, 0);
#pragma unroll
                    for (int b = 0; b < 3; b++) {
                        c0 = c0 + cmul(m[a * 3 + b], hp[0][b]);
                        c1 = c1 + cmul(m[a * 3 + b], hp[1][b]);
                    }
                    acc[v][a] = acc[v][a] + c0;
                    acc[v][3 + a] = acc[v][3 + a] + c1;
                    acc[v][6 + a] = fma_u(sd, pr.d0, b1 ? c1 : c0, acc[v][6 + a]);
                    acc[v][9 + a] = fma_u(sd, pr.d1, b1 ? c0 : c1, acc[v][9 + a]);
                }
            }
        }
    }
#pragma unroll
    for (int v = 0; v < NV; v++) {
#pragma unroll
        for (int c = 0; c < 12; c++) {
            acc[v][c].re += __shfl_xor(acc[v][c].re, 1);
            acc[v][c].im += __shfl_xor(acc[v][c].im, 1);
        }
        double part = 0.0;
        if (active && vec[v] >= 0) {
            const size_t vo = (size_t)vec[v] * 12 * Vh;
            const double czd = epi_coef(e, vec[v]);
            const uint32_t lo = (uint32_t)bwd * 6u * Vh32 + h32;
            cx<T> w[6];
#pragma unroll
            for (int c = 0; c < 6; c++) w[c] = bwd ? acc[v][6 + c] : acc[v][c];
            part = epilogue2<T>(e, w, bwd, vo, Vh, lo, out, czd);
        }
        if (e.red) {
            for (int off = SCG_WAVE / 2; off > 0; off >>= 1) part += __shfl_xor(part, off);
            if ((threadIdx.x % SCG_WAVE) == 0) red_lds[v * (SCG_BLOCK / SCG_WAVE) + threadIdx.x / SCG_WAVE] = part;
        }
    }
    if (e.red) {
        __syncthreads();
        const int v = threadIdx.x;
        if (v < NV) {
            int q = -1;
#pragma unroll
            for (int k = 0; k < NV; k++)
                if (k == v) q = vec[k];
            if (q >= 0) {
                double s = 0.0;
                for (int w = 0; w < SCG_BLOCK / SCG_WAVE; w++) s += red_lds[v * (SCG_BLOCK / SCG_WAVE) + w];
                e.partials[(int64_t)q * nsb + sb] = s;
            }
        }
    }
}

// ---- wave-split variant -------------------------------------------------------------------
// The two lanes-per-site kernels above give each site's forward hops to an even lane and its
// backward hops to the odd lane, so every lane selects between U and U^dag, between the signs of
// the two hop directions and between the projection coefficients at run time: on a 16-lane SIMD
// those selects cost as much issue time as the arithmetic itself.  Here whole wavefronts take one
// hop direction: waves 0 and 1 of a workgroup the forward hops of its 128 sites, waves 2 and 3 the
// backward hops of the same sites, and the direction mu is a compile-time constant in each of the
// four unrolled bodies.  Projection and reconstruction coefficients then fold into adds and
// fused multiply-adds, U^dag into operand order and signs.  The two halves of each site's sum meet
// in LDS: every wave hands the six output components that the other wave writes, adds the six it
// receives and runs the epilogue on its own six.

// Raw buffer loads: a descriptor (base and size in bytes) in scalar registers and one 32-bit lane
// offset shared by all component loads of a field, the component's offset going into the scalar
// soffset operand; a 64-bit address per load would cost two VGPRs and a 64-bit add each.  An
// offset beyond the size reads zero instead of faulting.
__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename S, int AUX = 0>
__device__ inline S bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    static_assert(sizeof(S) == 16 || sizeof(S) == 8 || sizeof(S) == 4, "load width");
    if constexpr (sizeof(S) == 16)
        return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX));
    else if constexpr (sizeof(S) == 8)
        return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
    else
        return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
}
// The cache-policy operand of a buffer load: CPOL_NT marks the load non-temporal, so that its lines
// are the first to leave the caches.  A one-vector stencil reads every link exactly once, and when
// the links alone outgrow the memory-side cache they otherwise push out the neighbour spinors that
// the next site blocks read again.
constexpr int CPOL_NT = 2;

// projection coefficients of proj_of(mu) as compile-time constants (forward hop)
template <int MU>
struct PJ;
template <>
struct PJ<0> {
    static constexpr int a0 = 3, c0r = 0, c0i = 1, c1r = 0, c1i = 1, b0 = 1, d0r = 0, d0i = -1, d1r = 0, d1i = -1;
};
template <>
struct PJ<1> {
    static constexpr int a0 = 3, c0r = 1, c0i = 0, c1r = -1, c1i = 0, b0 = 1, d0r = -1, d0i = 0, d1r = 1, d1i = 0;
};
template <>
struct PJ<2> {
    static constexpr int a0 = 2, c0r = 0, c0i = 1, c1r = 0, c1i = -1, b0 = 0, d0r = 0, d0i = -1, d1r = 0, d1i = 1;
};
template <>
struct PJ<3> {
    static constexpr int a0 = 2, c0r = -1, c0i = 0, c1r = -1, c1i = 0, b0 = 0, d0r = -1, d0i = 0, d1r = -1, d1i = 0;
};

// u * a for a compile-time unit u = R + i I (one of R, I is zero): a sign change or a swap, never
// a multiplication (0 * x does not fold away in IEEE arithmetic)
template <int R, int I, typename T>
__device__ inline cx<T> umulc(cx<T> a) {
    static_assert((R == 0) != (I == 0), "unit coefficient");
    if constexpr (I == 0)
        return R > 0 ? a : mk<T>(-a.re, -a.im);
    else
        return I > 0 ? mk<T>(-a.im, a.re) : mk<T>(a.im, -a.re);
}

// w += a * b and w += conj(a) * b as four fused multiply-adds each
template <typename T>
__device__ inline void cmac(cx<T>& w, cx<T> a, cx<T> b) {
    w.re = fma(a.re, b.re, w.re);
    w.re = fma(-a.im, b.im, w.re);
    w.im = fma(a.re, b.im, w.im);
    w.im = fma(a.im, b.re, w.im);
}
template <typename T>
__device__ inline void cjmac(cx<T>& w, cx<T> a, cx<T> b) {
    w.re = fma(a.re, b.re, w.re);
    w.re = fma(a.im, b.im, w.re);
    w.im = fma(a.re, b.im, w.im);
    w.im = fma(-a.im, b.re, w.im);
}

// neighbour index of site h = (x, y, z, t) in direction MU (forward, or backward when BWD) without
// divisions: a step along y, z or t moves h by a fixed stride, wrapping at the boundary
template <int MU, bool BWD>
__device__ inline uint32_t nb_split(const Geom& g, int x, int y, int z, int t, int xh, uint32_t h32, int& sign) {
    sign = 1;
    if constexpr (MU == 0) {
        const int xn = BWD ? (x == 0 ? g.L[0] - 1 : x - 1) : (x == g.L[0] - 1 ? 0 : x + 1);
        return h32 - (uint32_t)xh + (uint32_t)(xn >> 1);
    } else {
        const int c = MU == 1 ? y : (MU == 2 ? z : t);
        const int L = g.L[MU];
        const uint32_t stride = (uint32_t)g.Lxh * (MU >= 2 ? (uint32_t)g.L[1] : 1u) * (MU == 3 ? (uint32_t)g.L[2] : 1u);
        const bool wrap = BWD ? c == 0 : c == L - 1;
        if (MU == 3 && wrap) sign = g.t_bc;
        const uint32_t span = (uint32_t)(L - 1) * stride;
        if constexpr (BWD)
            return wrap ? h32 + span : h32 - stride;
        else
            return wrap ? h32 - span : h32 + stride;
    }
}

// acc += s * w for a runtime sign s = +-1, as fused multiply-adds
template <typename T>
__device__ inline void acc_fma(cx<T>& acc, T s, cx<T> w) {
    acc.re = fma(s, w.re, acc.re);
    acc.im = fma(s, w.im, acc.im);
}

// The input spinors of a tile of xy-rows staged in LDS ([vector][component][staged site]): the x
// and y neighbours of the tile's sites are read from there.  rown is the lane's row in the stage;
// with whole set the stage is the whole xy-plane and y wraps inside it, otherwise it holds one
// halo row on either side of the tile.
template <typename T>
struct Stage {
    const cx<T>* st;
    uint32_t S;   // staged sites
    int rown, whole;
};

// The spinor half of one hop direction of the wave-split kernels for NV vectors: the neighbour's
// spinor (site hn, or staged site ln with LDS) projected with (1 -/+ gamma_mu), multiplied by the
// link u (forward) or u^dag (backward) and reconstructed into acc with the boundary sign.
template <typename T, int NV, int MU, bool BWD, bool LDS>
__device__ __attribute__((always_inline)) inline void split_body(const cx<T> (&u)[9], uint32_t hn, uint32_t ln, T sign,
                                                                 const cx<T>* __restrict__ in, uint32_t Vh32, const int (&vec)[NV],
                                                                 const Stage<T>& sg, cx<T> (&acc)[NV][12]) {
    using C = PJ<MU>;
    constexpr int s = BWD ? -1 : 1;   // the backward hop negates every coefficient
    constexpr int a0 = C::a0, a1 = 5 - C::a0;
    const uint32_t soff = hn * (uint32_t)sizeof(cx<T>);
#pragma unroll
    for (int v = 0; v < NV; v++) {
        if (vec[v] < 0) continue;   // uniform
        cx<T> ps[12];
        if constexpr (LDS) {
#pragma unroll
            for (int c = 0; c < 12; c++) ps[c] = sg.st[(uint32_t)(v * 12 + c) * sg.S + ln];
        } else {
            const auto sr = buf_rsrc(in + (size_t)vec[v] * 12 * Vh32, 12u * Vh32 * (uint32_t)sizeof(cx<T>));
#pragma unroll
            for (int c = 0; c < 12; c++) ps[c] = bload<cx<T>>(sr, soff, (uint32_t)c * Vh32 * (uint32_t)sizeof(cx<T>));
        }
        cx<T> hp[2][3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            hp[0][a] = ps[a] + umulc<s * C::c0r, s * C::c0i>(ps[3 * a0 + a]);
            hp[1][a] = ps[3 + a] + umulc<s * C::c1r, s * C::c1i>(ps[3 * a1 + a]);
        }
#pragma unroll
        for (int a = 0; a < 3; a++) {
            cx<T> ch[2];
#pragma unroll
            for (int sp = 0; sp < 2; sp++) {
                cx<T> w = BWD ? cjmul(u[a], hp[sp][0]) : cmul(u[a * 3], hp[sp][0]);
#pragma unroll
                for (int b = 1; b < 3; b++) {
                    if (BWD)
                        cjmac(w, u[b * 3 + a], hp[sp][b]);
                    else
                        cmac(w, u[a * 3 + b], hp[sp][b]);
                }
                ch[sp] = w;
            }
            acc_fma(acc[v][a], sign, ch[0]);
            acc_fma(acc[v][3 + a], sign, ch[1]);
            acc_fma(acc[v][6 + a], sign, umulc<s * C::d0r, s * C::d0i>(C::b0 == 1 ? ch[1] : ch[0]));
            acc_fma(acc[v][9 + a], sign, umulc<s * C::d1r, s * C::d1i>(C::b0 == 1 ? ch[0] : ch[1]));
        }
    }
}

// The stored link of one hop direction of the wave-split kernels (forward: U_mu at the site;
// backward: U_mu at the neighbour, of the other parity), with the neighbour's index and the
// boundary sign of the hop.
template <typename LT, int MU, bool BWD, int LAUX = 0>
__device__ __attribute__((always_inline)) inline void split_link(const Geom& g, const typename LinkLoad<LT>::Store* __restrict__ links,
                                                                 int p, int x, int y, int z, int t, int xh, uint32_t h32,
                                                                 typename LinkLoad<LT>::Store (&ul)[LinkLoad<LT>::NE], uint32_t& hn,
                                                                 int& nsign) {
    hn = nb_split<MU, BWD>(g, x, y, z, t, xh, h32, nsign);
    const uint32_t Vh32 = (uint32_t)g.Vh;
    const uint32_t lpar = BWD ? 1u - (uint32_t)p : (uint32_t)p;
    using S = typename LinkLoad<LT>::Store;
    constexpr int NE = LinkLoad<LT>::NE;
    const auto lr = buf_rsrc(links + (size_t)(MU * 2 + lpar) * NE * Vh32, (uint32_t)NE * Vh32 * (uint32_t)sizeof(S));
    const uint32_t loff = (BWD ? hn : h32) * (uint32_t)sizeof(S);
#pragma unroll
    for (int c = 0; c < NE; c++) ul[c] = bload<S, LAUX>(lr, loff, (uint32_t)c * Vh32 * (uint32_t)sizeof(S));
}

// the link in the arithmetic precision, its third row rebuilt from the stored two
template <typename T, typename LT>
__device__ __attribute__((always_inline)) inline void split_widen(const typename LinkLoad<LT>::Store (&ul)[LinkLoad<LT>::NE], cx<T> (&u)[9]) {
    constexpr int NE = LinkLoad<LT>::NE;
#pragma unroll
    for (int c = 0; c < NE; c++) u[c] = LinkLoad<LT>::template cvt<T>(ul[c]);
    if constexpr (NE == 6) su3_third_row(u);
}

// One hop direction of the wave-split kernel for NV vectors.  PLANE: x and y neighbours come from
// the LDS stage; LAUX: the cache policy of the link loads.
template <typename T, typename LT, int NV, int MU, bool BWD, bool PLANE, int LAUX = 0>
__device__ __attribute__((always_inline)) inline void split_dir(const Geom& g, const typename LinkLoad<LT>::Store* __restrict__ links, const cx<T>* __restrict__ in,
                                 const int (&vec)[NV], int p, int x, int y, int z, int t, int xh, uint32_t h32,
                                 const Stage<T>& sg, cx<T> (&acc)[NV][12]) {
    constexpr bool LDS = PLANE && MU <= 1;
    uint32_t ln = 0;   // the neighbour's staged site
    if constexpr (LDS) {
        if constexpr (MU == 0) {
            const int xn = BWD ? (x == 0 ? g.L[0] - 1 : x - 1) : (x == g.L[0] - 1 ? 0 : x + 1);
            ln = (uint32_t)(sg.rown * g.Lxh + (xn >> 1));
        } else {
            int rn = BWD ? sg.rown - 1 : sg.rown + 1;
            if (sg.whole) rn = BWD ? (y == 0 ? g.L[1] - 1 : rn) : (y == g.L[1] - 1 ? 0 : rn);
            ln = (uint32_t)(rn * g.Lxh + xh);
        }
    }
    typename LinkLoad<LT>::Store ul[LinkLoad<LT>::NE];
    uint32_t hn;
    int nsign;
    split_link<LT, MU, BWD, LAUX>(g, links, p, x, y, z, t, xh, h32, ul, hn, nsign);
    cx<T> u[9];
    split_widen<T, LT>(ul, u);
    split_body<T, NV, MU, BWD, LDS>(u, hn, ln, (T)nsign, in, (uint32_t)g.Vh, vec, sg, acc);
}

// the four directions of one hop side
template <typename T, typename LT, int NV, bool BWD, bool PLANE>
__device__ __attribute__((always_inline)) inline void split_hops(const Geom& g, const typename LinkLoad<LT>::Store* __restrict__ links, const cx<T>* __restrict__ in,
                                  const int (&vec)[NV], int p, bool active, int x, int y, int z, int t, int xh,
                                  uint32_t h32, const Stage<T>& sg, cx<T> (&acc)[NV][12]) {
    if (active) {
        // straight-line directions; the scheduling fences keep each direction's loads with it, so
        // that the registers in flight are those of one direction
        split_dir<T, LT, NV, 0, BWD, PLANE>(g, links, in, vec, p, x, y, z, t, xh, h32, sg, acc);
        __builtin_amdgcn_sched_barrier(0);
        split_dir<T, LT, NV, 1, BWD, PLANE>(g, links, in, vec, p, x, y, z, t, xh, h32, sg, acc);
        __builtin_amdgcn_sched_barrier(0);
        split_dir<T, LT, NV, 2, BWD, PLANE>(g, links, in, vec, p, x, y, z, t, xh, h32, sg, acc);
        __builtin_amdgcn_sched_barrier(0);
        split_dir<T, LT, NV, 3, BWD, PLANE>(g, links, in, vec, p, x, y, z, t, xh, h32, sg, acc);
    }
}

// hand over the six components the other side writes: xch[vector][side receiving][component][site]
template <typename T, int NV, bool BWD>
__device__ __attribute__((always_inline)) inline void split_handover(const cx<T> (&acc)[NV][12], cx<T>* xch, uint32_t xs, int sl) {
    constexpr int other = BWD ? 0 : 6;
#pragma unroll
    for (int v = 0; v < NV; v++)
#pragma unroll
        for (int c = 0; c < 6; c++) xch[(uint32_t)((v * 2 + (BWD ? 0 : 1)) * 6 + c) * xs + sl] = acc[v][other + c];
}

// the other side's six components added to this side's, then the epilogue on them
template <typename T, int NV, bool BWD, bool CGU>
__device__ __attribute__((always_inline)) inline void split_tail(const EpiDev<T>& e, const int (&vec)[NV], bool active, uint32_t Vh32,
                                                                 uint32_t h32, int sl, int wave, int nwave, const cx<T> (&acc)[NV][12],
                                                                 const cx<T>* xch, uint32_t xs, cx<T>* __restrict__ out, double* red_lds) {
    constexpr int own = BWD ? 6 : 0;
    const uint32_t lo = (uint32_t)own * Vh32 + h32;
#pragma unroll
    for (int v = 0; v < NV; v++) {
        double part = 0.0;
        if (active && vec[v] >= 0) {
            cx<T> w[6];
#pragma unroll
            for (int c = 0; c < 6; c++) w[c] = acc[v][own + c] + xch[(uint32_t)((v * 2 + (BWD ? 1 : 0)) * 6 + c) * xs + sl];
            const size_t vo = (size_t)vec[v] * 12 * Vh32;
            const double czd = epi_coef(e, vec[v]);
            part = epilogue2<T, 6, CGU>(e, w, BWD ? 1 : 0, vo, (int64_t)Vh32, lo, out, czd);
        }
        if (e.red) {
            for (int off = SCG_WAVE / 2; off > 0; off >>= 1) part += __shfl_xor(part, off);
            if ((threadIdx.x % SCG_WAVE) == 0) red_lds[v * nwave + wave] = part;
        }
    }
}

template <typename T, typename LT, int NV, bool CGU = false>
__global__ __launch_bounds__(SCG_BLOCK) void hop_split_kernel(Geom g, const typename LinkLoad<LT>::Store* __restrict__ links,
                                                              const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                              int p, int nvec, int64_t nsb, EpiDev<T> e, int64_t cs, int64_t bps) {
    __shared__ cx<T> xch[NV * 2 * 6 * (SCG_BLOCK / 2)];
    __shared__ double red_lds[NV * (SCG_BLOCK / SCG_WAVE)];
    zoff_hop(cs, links, in, out, e);
    if (e.gate_m && e.gate_i > *e.gate_m) return;
    if (e.kappa2_dev) e.kappa2 = (T)*e.kappa2_dev;
    const int nvg = (nvec + NV - 1) / NV;
    const int64_t nblk = nsb * nvg;
    const int64_t logical = xcd_logical_block(nblk);
    if (logical >= nblk) return;
    const int vg = (int)(logical % nvg);
    const int64_t sb = logical / nvg;   // position in the visiting order (partials are indexed by it)
    const int64_t Vh = g.Vh;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / SCG_WAVE));
    const bool bwd = wave >= 2;                                   // uniform over the wavefront
    const int sl = (wave & 1) * SCG_WAVE + (int)(threadIdx.x % SCG_WAVE);   // site within the block
    const int64_t h = sb_order(sb, bps, g.L[3]) * (SCG_BLOCK / 2) + sl;
    const bool active = h < Vh;

    int x = 0, y = 0, z = 0, t = 0, xh = 0;
    if (active) {   // 32-bit arithmetic: a half lattice has fewer than 2^31 sites
        const uint32_t hu = (uint32_t)h;
        xh = (int)(hu % (uint32_t)g.Lxh);
        uint32_t r = hu / (uint32_t)g.Lxh;
        y = (int)(r % (uint32_t)g.L[1]);
        r /= (uint32_t)g.L[1];
        z = (int)(r % (uint32_t)g.L[2]);
        t = (int)(r / (uint32_t)g.L[2]);
        x = 2 * xh + ((y + z + t + p) & 1);
    }
    const uint32_t Vh32 = (uint32_t)Vh, h32 = (uint32_t)h;

    // the group's vectors (-1: empty slot, or a vector whose CG is done or frozen); uniform
    int vec[NV];
    bool any = false;
#pragma unroll
    for (int v = 0; v < NV; v++) {
        const int slot = vg * NV + v;
        int q = -1;
        if (slot < nvec) {
            q = e.vec_map ? e.vec_map[slot] : slot;
            if (q >= 0 && e.cg && (e.cg[q].done || e.cg[q].frozen)) q = -1;
        }
        vec[v] = __builtin_amdgcn_readfirstlane(q);
        any = any || vec[v] >= 0;
    }
    if (!any) return;  // uniform over the workgroup

    cx<T> acc[NV][12];
#pragma unroll
    for (int v = 0; v < NV; v++)
#pragma unroll
        for (int c = 0; c < 12; c++) acc[v][c] = mk<T>(0, 0);
    const Stage<T> sg{nullptr, 0, 0, 0};
    constexpr uint32_t xs = SCG_BLOCK / 2;
    if (bwd) {
        split_hops<T, LT, NV, true, false>(g, links, in, vec, p, active, x, y, z, t, xh, h32, sg, acc);
        split_handover<T, NV, true>(acc, xch, xs, sl);
    } else {
        split_hops<T, LT, NV, false, false>(g, links, in, vec, p, active, x, y, z, t, xh, h32, sg, acc);
        split_handover<T, NV, false>(acc, xch, xs, sl);
    }
    __syncthreads();

    constexpr int nwave = SCG_BLOCK / SCG_WAVE;
    if (bwd)
        split_tail<T, NV, true, CGU>(e, vec, active, Vh32, h32, sl, wave, nwave, acc, xch, xs, out, red_lds);
    else
        split_tail<T, NV, false, CGU>(e, vec, active, Vh32, h32, sl, wave, nwave, acc, xch, xs, out, red_lds);
    if (e.red) {
        __syncthreads();
        const int v = threadIdx.x;
        if (v < NV) {
            int q = -1;
#pragma unroll
            for (int k = 0; k < NV; k++)
                if (k == v) q = vec[k];
            if (q >= 0) {
                double s = 0.0;
                for (int w = 0; w < SCG_BLOCK / SCG_WAVE; w++) s += red_lds[v * (SCG_BLOCK / SCG_WAVE) + w];
                e.partials[(int64_t)q * nsb + sb] = s;
            }
        }
    }
}

// ---- link-resident multi-vector variant ------------------------------------------------------
// The wave-split kernel for launches of many vectors.  One workgroup per site block runs through
// every vector of the launch, NV at a time, holding the stored form of its side's four links in
// registers all the while: each link is read from memory once per launch instead of once per group
// of NV vectors.  The site blocks (all resident at once, or nearly) advance through the vectors
// together, so a block's z and t neighbours for a vector were fetched for that same vector by the
// blocks around it shortly before, as in a one-vector launch, instead of a whole set of vector groups
// earlier.  The reduction partials are indexed like the wave-split kernel's.
// An empty asm statement that claims to change the held link registers: without it the compiler
// keeps the widened links (nine complex entries per direction) across the vector loop, which costs
// more registers than the stored form it is rebuilt from.
template <typename S>
__device__ __attribute__((always_inline)) inline void opaque(S& v) {
    if constexpr (sizeof(S) == 4) {
        asm volatile("" : "+v"(v));
    } else {
        static_assert(sizeof(S) == 8, "held link entries are 4 or 8 bytes");
        asm volatile("" : "+v"(v.re), "+v"(v.im));
    }
}

template <typename T, typename LT, int NV, bool BWD>
__device__ __attribute__((always_inline)) inline void stream_hops(const typename LinkLoad<LT>::Store (&ul)[4][LinkLoad<LT>::NE],
                                                                  const uint32_t (&hn)[4], const T (&sgn)[4], const cx<T>* __restrict__ in,
                                                                  uint32_t Vh32, const int (&vec)[NV], bool active, cx<T> (&acc)[NV][12]) {
    if (!active) return;
    const Stage<T> sg{nullptr, 0, 0, 0};
    cx<T> u[9];
    split_widen<T, LT>(ul[0], u);
    split_body<T, NV, 0, BWD, false>(u, hn[0], 0, sgn[0], in, Vh32, vec, sg, acc);
    __builtin_amdgcn_sched_barrier(0);
    split_widen<T, LT>(ul[1], u);
    split_body<T, NV, 1, BWD, false>(u, hn[1], 0, sgn[1], in, Vh32, vec, sg, acc);
    __builtin_amdgcn_sched_barrier(0);
    split_widen<T, LT>(ul[2], u);
    split_body<T, NV, 2, BWD, false>(u, hn[2], 0, sgn[2], in, Vh32, vec, sg, acc);
    __builtin_amdgcn_sched_barrier(0);
    split_widen<T, LT>(ul[3], u);
    split_body<T, NV, 3, BWD, false>(u, hn[3], 0, sgn[3], in, Vh32, vec, sg, acc);
}

template <typename LT, bool BWD>
__device__ __attribute__((always_inline)) inline void stream_links(const Geom& g, const typename LinkLoad<LT>::Store* __restrict__ links,
                                                                   int p, int x, int y, int z, int t, int xh, uint32_t h32,
                                                                   typename LinkLoad<LT>::Store (&ul)[4][LinkLoad<LT>::NE],
                                                                   uint32_t (&hn)[4], int (&ns)[4]) {
    split_link<LT, 0, BWD>(g, links, p, x, y, z, t, xh, h32, ul[0], hn[0], ns[0]);
    split_link<LT, 1, BWD>(g, links, p, x, y, z, t, xh, h32, ul[1], hn[1], ns[1]);
    split_link<LT, 2, BWD>(g, links, p, x, y, z, t, xh, h32, ul[2], hn[2], ns[2]);
    split_link<LT, 3, BWD>(g, links, p, x, y, z, t, xh, h32, ul[3], hn[3], ns[3]);
}

template <typename T, typename LT, int NV, bool CGU = false>
__global__ __launch_bounds__(SCG_BLOCK) void hop_stream_kernel(Geom g, const typename LinkLoad<LT>::Store* __restrict__ links,
                                                               const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                               int p, int nvec, int64_t nsb, EpiDev<T> e, int64_t cs, int64_t bps) {
    __shared__ cx<T> xch[NV * 2 * 6 * (SCG_BLOCK / 2)];
    __shared__ double red_lds[NV * (SCG_BLOCK / SCG_WAVE)];
    zoff_hop(cs, links, in, out, e);
    if (e.gate_m && e.gate_i > *e.gate_m) return;
    if (e.kappa2_dev) e.kappa2 = (T)*e.kappa2_dev;
    const int64_t sb = xcd_logical_block(nsb);   // position in the visiting order
    if (sb >= nsb) return;
    const int64_t Vh = g.Vh;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / SCG_WAVE));
    const bool bwd = wave >= 2;                                   // uniform over the wavefront
    const int sl = (wave & 1) * SCG_WAVE + (int)(threadIdx.x % SCG_WAVE);   // site within the block
    const int64_t h = sb_order(sb, bps, g.L[3]) * (SCG_BLOCK / 2) + sl;
    const bool active = h < Vh;

    int x = 0, y = 0, z = 0, t = 0, xh = 0;
    if (active) {
        const uint32_t hu = (uint32_t)h;
        xh = (int)(hu % (uint32_t)g.Lxh);
        uint32_t r = hu / (uint32_t)g.Lxh;
        y = (int)(r % (uint32_t)g.L[1]);
        r /= (uint32_t)g.L[1];
        z = (int)(r % (uint32_t)g.L[2]);
        t = (int)(r / (uint32_t)g.L[2]);
        x = 2 * xh + ((y + z + t + p) & 1);
    }
    const uint32_t Vh32 = (uint32_t)Vh, h32 = (uint32_t)h;

    // this side's four links, read once for the whole launch
    typename LinkLoad<LT>::Store ul[4][LinkLoad<LT>::NE];
    uint32_t hn[4] = {0, 0, 0, 0};
    int ns[4] = {1, 1, 1, 1};
    if (active) {
        if (bwd)
            stream_links<LT, true>(g, links, p, x, y, z, t, xh, h32, ul, hn, ns);
        else
            stream_links<LT, false>(g, links, p, x, y, z, t, xh, h32, ul, hn, ns);
    }
    const T sgn[4] = {(T)ns[0], (T)ns[1], (T)ns[2], (T)ns[3]};

    constexpr int nwave = SCG_BLOCK / SCG_WAVE;
    constexpr uint32_t xs = SCG_BLOCK / 2;
    const int nvg = (nvec + NV - 1) / NV;
    for (int vg = 0; vg < nvg; vg++) {
        // the group's vectors (-1: empty slot, or a vector whose CG is done or frozen); uniform
        int vec[NV];
        bool any = false;
#pragma unroll
        for (int v = 0; v < NV; v++) {
            const int slot = vg * NV + v;
            int q = -1;
            if (slot < nvec) {
                q = e.vec_map ? e.vec_map[slot] : slot;
                if (q >= 0 && e.cg && (e.cg[q].done || e.cg[q].frozen)) q = -1;
            }
            vec[v] = __builtin_amdgcn_readfirstlane(q);
            any = any || vec[v] >= 0;
        }
        if (!any) continue;   // uniform over the workgroup
#pragma unroll
        for (int d = 0; d < 4; d++)
#pragma unroll
            for (int c = 0; c < LinkLoad<LT>::NE; c++) opaque(ul[d][c]);

        cx<T> acc[NV][12];
#pragma unroll
        for (int v = 0; v < NV; v++)
#pragma unroll
            for (int c = 0; c < 12; c++) acc[v][c] = mk<T>(0, 0);
        if (bwd) {
            stream_hops<T, LT, NV, true>(ul, hn, sgn, in, Vh32, vec, active, acc);
            split_handover<T, NV, true>(acc, xch, xs, sl);
        } else {
            stream_hops<T, LT, NV, false>(ul, hn, sgn, in, Vh32, vec, active, acc);
            split_handover<T, NV, false>(acc, xch, xs, sl);
        }
        __syncthreads();
        if (bwd)
            split_tail<T, NV, true, CGU>(e, vec, active, Vh32, h32, sl, wave, nwave, acc, xch, xs, out, red_lds);
        else
            split_tail<T, NV, false, CGU>(e, vec, active, Vh32, h32, sl, wave, nwave, acc, xch, xs, out, red_lds);
        if (e.red) {
            __syncthreads();
            const int v = threadIdx.x;
            if (v < NV) {
                int q = -1;
#pragma unroll
                for (int k = 0; k < NV; k++)
                    if (k == v) q = vec[k];
                if (q >= 0) {
                    double s = 0.0;
                    for (int w = 0; w < nwave; w++) s += red_lds[v * nwave + w];
                    e.partials[(int64_t)q * nsb + sb] = s;
                }
            }
        }
        __syncthreads();   // the exchange and reduction LDS are rewritten by the next group
    }
}

// ---- LDS-staged variant --------------------------------------------------------------------
// The wave-split kernel with the x and y neighbours read from LDS.  A workgroup takes a tile of R
// whole xy-rows of one (z, t) plane (the whole plane when it has at most 256 sites, else tiles of
// balanced size) and first
// stages the input spinors of those rows, plus one halo row on either side, in LDS: every input
// site is then fetched once for the four x and y hops instead of four times, and only the z and t
// neighbours come from L2.  After the hops the same LDS holds the hand-over of the two sides.
__host__ __device__ inline int plane_rows(const Geom& g) {
    const int rmax = g.Lxh >= 256 ? 1 : 256 / g.Lxh;     // rows of at most 256 sites
    const int ntile = (g.L[1] + rmax - 1) / rmax;
    return (g.L[1] + ntile - 1) / ntile;                // balanced tiles
}
__host__ __device__ inline int plane_tiles(const Geom& g) { return (g.L[1] + plane_rows(g) - 1) / plane_rows(g); }
// staged sites of the largest tile
__host__ __device__ inline int plane_stage_sites(const Geom& g) {
    const int R = plane_rows(g);
    return (R >= g.L[1] ? g.L[1] : R + 2) * g.Lxh;
}

template <typename T, typename LT, int NV, bool CGU = false>
__global__ __launch_bounds__(512) void hop_plane_kernel(Geom g, const typename LinkLoad<LT>::Store* __restrict__ links,
                                                        const cx<T>* __restrict__ in, cx<T>* __restrict__ out, int p, int nvec,
                                                        int64_t nsb, EpiDev<T> e, int64_t cs, int Pw) {
    extern __shared__ __align__(16) unsigned char plane_smem[];
    cx<T>* st = reinterpret_cast<cx<T>*>(plane_smem);
    __shared__ double red_lds[NV * 8];
    zoff_hop(cs, links, in, out, e);
    if (e.gate_m && e.gate_i > *e.gate_m) return;
    if (e.kappa2_dev) e.kappa2 = (T)*e.kappa2_dev;
    const int nvg = (nvec + NV - 1) / NV;
    const int64_t nblk = nsb * nvg;
    const int64_t logical = xcd_logical_block(nblk);
    if (logical >= nblk) return;
    const int vg = (int)(logical % nvg);
    const int blk = (int)(logical / nvg);   // tile index (partials are indexed by it)
    const int ntile = plane_tiles(g), R = plane_rows(g);
    const int q = blk / ntile, j = blk - q * ntile;   // plane z + Lz t, tile within it
    const int Lxh = g.Lxh, Ly = g.L[1];
    const bool whole = R >= Ly;
    const int y0 = j * R, Rt = min(R, Ly - y0), St = Rt * Lxh;
    const int nws = Pw / SCG_WAVE;   // wavefronts per side
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / SCG_WAVE));
    const bool bwd = wave >= nws;
    const int sl = (wave - (bwd ? nws : 0)) * SCG_WAVE + (int)(threadIdx.x % SCG_WAVE);   // site within the tile
    const bool active = sl < St;
    const uint32_t Vh32 = (uint32_t)g.Vh;
    const uint32_t base = (uint32_t)q * (uint32_t)(Lxh * Ly);   // first site of the plane
    int x = 0, y = 0, z = 0, t = 0, xh = 0, yl = 0;
    if (active) {
        yl = sl / Lxh;
        xh = sl - yl * Lxh;
        y = y0 + yl;
        z = q % g.L[2];
        t = q / g.L[2];
        x = 2 * xh + ((y + z + t + p) & 1);
    }
    const uint32_t h32 = base + (uint32_t)(y0 * Lxh + sl);

    int vec[NV];
    bool any = false;
#pragma unroll
    for (int v = 0; v < NV; v++) {
        const int slot = vg * NV + v;
        int qv = -1;
        if (slot < nvec) {
            qv = e.vec_map ? e.vec_map[slot] : slot;
            if (qv >= 0 && e.cg && (e.cg[qv].done || e.cg[qv].frozen)) qv = -1;
        }
        vec[v] = __builtin_amdgcn_readfirstlane(qv);
        any = any || vec[v] >= 0;
    }
    if (!any) return;  // uniform over the workgroup

    // stage the tile's rows and halo rows of every vector of the group
    const int nrs = whole ? Ly : Rt + 2;
    const uint32_t S = (uint32_t)(nrs * Lxh);
#pragma unroll
    for (int v = 0; v < NV; v++) {
        if (vec[v] < 0) continue;
        const auto sr = buf_rsrc(in + (size_t)vec[v] * 12 * Vh32, 12u * Vh32 * (uint32_t)sizeof(cx<T>));
        for (uint32_t k = threadIdx.x; k < S; k += blockDim.x) {
            const int r = (int)(k / (uint32_t)Lxh);
            const int yr = whole ? r : (y0 - 1 + r + Ly) % Ly;
            const uint32_t off = (base + (uint32_t)(yr * Lxh) + (k - (uint32_t)(r * Lxh))) * (uint32_t)sizeof(cx<T>);
            cx<T> w[12];
#pragma unroll
            for (int c = 0; c < 12; c++) w[c] = bload<cx<T>>(sr, off, (uint32_t)c * Vh32 * (uint32_t)sizeof(cx<T>));
#pragma unroll
            for (int c = 0; c < 12; c++) st[(uint32_t)(v * 12 + c) * S + k] = w[c];
        }
    }
    __syncthreads();

    const Stage<T> sg{st, S, whole ? y : yl + 1, whole ? 1 : 0};
    cx<T> acc[NV][12];
#pragma unroll
    for (int v = 0; v < NV; v++)
#pragma unroll
        for (int c = 0; c < 12; c++) acc[v][c] = mk<T>(0, 0);
    if (bwd)
        split_hops<T, LT, NV, true, true>(g, links, in, vec, p, active, x, y, z, t, xh, h32, sg, acc);
    else
        split_hops<T, LT, NV, false, true>(g, links, in, vec, p, active, x, y, z, t, xh, h32, sg, acc);
    __syncthreads();   // the stage is read; its LDS now takes the hand-over
    const uint32_t xs = (uint32_t)St;
    if (active) {
        if (bwd)
            split_handover<T, NV, true>(acc, st, xs, sl);
        else
            split_handover<T, NV, false>(acc, st, xs, sl);
    }
    __syncthreads();
    const int nwave = 2 * nws;
    if (bwd)
        split_tail<T, NV, true, CGU>(e, vec, active, Vh32, h32, sl, wave, nwave, acc, st, xs, out, red_lds);
    else
        split_tail<T, NV, false, CGU>(e, vec, active, Vh32, h32, sl, wave, nwave, acc, st, xs, out, red_lds);
    if (e.red) {
        __syncthreads();
        const int v = threadIdx.x;
        if (v < NV) {
            int qv = -1;
#pragma unroll
            for (int k = 0; k < NV; k++)
                if (k == v) qv = vec[k];
            if (qv >= 0) {
                double sum = 0.0;
                for (int w = 0; w < nwave; w++) sum += red_lds[v * nwave + w];
                e.partials[(int64_t)qv * nsb + blk] = sum;
            }
        }
    }
}

// ---- quad-split variant ------------------------------------------------------------------
// One vector per workgroup of 64 sites and four wavefronts: the forward x and y hops, the forward
// z and t hops, and the same two pairs backward, each on a wavefront of its own.  A one-vector
// launch (the Lanczos steps) then has four wavefronts per 64 sites instead of two, each with half
// the dependent loads; the four partial sums meet in LDS and each wavefront writes three of the
// twelve output components.  LAUX: the cache policy of the link loads.
template <typename T, typename LT, bool CGU, int LAUX>
__device__ __attribute__((always_inline)) inline void quad_body(Geom g, const typename LinkLoad<LT>::Store* __restrict__ links,
                                                                const cx<T>* __restrict__ in, cx<T>* __restrict__ out, int p, int nvec,
                                                                int64_t nsb, EpiDev<T> e, int64_t cs, int64_t bps) {
    constexpr int NS = SCG_WAVE;   // sites per workgroup
    __shared__ cx<T> xch[4 * 12 * NS];
    __shared__ double red_lds[SCG_BLOCK / SCG_WAVE];
    zoff_hop(cs, links, in, out, e);
    if (e.gate_m && e.gate_i > *e.gate_m) return;
    if (e.kappa2_dev) e.kappa2 = (T)*e.kappa2_dev;
    const int64_t nblk = nsb * nvec;
    const int64_t logical = xcd_logical_block(nblk);
    if (logical >= nblk) return;
    const int slot = (int)(logical % nvec);
    const int64_t sb = logical / nvec;   // position in the visiting order (partials are indexed by it)
    int q = e.vec_map ? e.vec_map[slot] : slot;
    if (q >= 0 && e.cg && (e.cg[q].done || e.cg[q].frozen)) q = -1;
    const int vec[1] = {__builtin_amdgcn_readfirstlane(q)};
    if (vec[0] < 0) return;   // uniform over the workgroup
    const int grp = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / SCG_WAVE));   // 0 fwd xy, 1 fwd zt, 2 bwd xy, 3 bwd zt
    const int sl = (int)(threadIdx.x % SCG_WAVE);
    const int64_t h = sb_order(sb, bps, g.L[3]) * NS + sl;
    const bool active = h < g.Vh;
    int x = 0, y = 0, z = 0, t = 0, xh = 0;
    if (active) {
        const uint32_t hu = (uint32_t)h;
        xh = (int)(hu % (uint32_t)g.Lxh);
        uint32_t r = hu / (uint32_t)g.Lxh;
        y = (int)(r % (uint32_t)g.L[1]);
        r /= (uint32_t)g.L[1];
        z = (int)(r % (uint32_t)g.L[2]);
        t = (int)(r / (uint32_t)g.L[2]);
        x = 2 * xh + ((y + z + t + p) & 1);
    }
    const uint32_t Vh32 = (uint32_t)g.Vh, h32 = (uint32_t)h;
    const Stage<T> sg{nullptr, 0, 0, 0};
    cx<T> acc[1][12];
#pragma unroll
    for (int c = 0; c < 12; c++) acc[0][c] = mk<T>(0, 0);
    if (active) {
        if (grp == 0) {
            split_dir<T, LT, 1, 0, false, false, LAUX>(g, links, in, vec, p, x, y, z, t, xh, h32, sg, acc);
            __builtin_amdgcn_sched_barrier(0);
            split_dir<T, LT, 1, 1, false, false, LAUX>(g, links, in, vec, p, x, y, z, t, xh, h32, sg, acc);
        } else if (grp == 1) {
            split_dir<T, LT, 1, 2, false, false, LAUX>(g, links, in, vec, p, x, y, z, t, xh, h32, sg, acc);
            __builtin_amdgcn_sched_barrier(0);
            split_dir<T, LT, 1, 3, false, false, LAUX>(g, links, in, vec, p, x, y, z, t, xh, h32, sg, acc);
        } else if (grp == 2) {
            split_dir<T, LT, 1, 0, true, false, LAUX>(g, links, in, vec, p, x, y, z, t, xh, h32, sg, acc);
            __builtin_amdgcn_sched_barrier(0);
            split_dir<T, LT, 1, 1, true, false, LAUX>(g, links, in, vec, p, x, y, z, t, xh, h32, sg, acc);
        } else {
            split_dir<T, LT, 1, 2, true, false, LAUX>(g, links, in, vec, p, x, y, z, t, xh, h32, sg, acc);
            __builtin_amdgcn_sched_barrier(0);
            split_dir<T, LT, 1, 3, true, false, LAUX>(g, links, in, vec, p, x, y, z, t, xh, h32, sg, acc);
        }
    }
#pragma unroll
    for (int c = 0; c < 12; c++) xch[(grp * 12 + c) * NS + sl] = acc[0][c];
    __syncthreads();
    double part = 0.0;
    if (active) {
        cx<T> w[3];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const int cc = 3 * grp + c;
            w[c] = xch[cc * NS + sl] + xch[(12 + cc) * NS + sl] + xch[(24 + cc) * NS + sl] + xch[(36 + cc) * NS + sl];
        }
        const size_t vo = (size_t)vec[0] * 12 * Vh32;
        const double czd = epi_coef(e, vec[0]);
        const uint32_t lo = (uint32_t)(3 * grp) * Vh32 + h32;
        part = epilogue2<T, 3, CGU>(e, w, grp >= 2 ? 1 : 0, vo, (int64_t)Vh32, lo, out, czd);
    }
    if (e.red) {
        for (int off = SCG_WAVE / 2; off > 0; off >>= 1) part += __shfl_xor(part, off);
        if (sl == 0) red_lds[grp] = part;
        __syncthreads();
        if (threadIdx.x == 0) {
            double sum = 0.0;
            for (int w = 0; w < SCG_BLOCK / SCG_WAVE; w++) sum += red_lds[w];
            e.partials[(int64_t)vec[0] * nsb + sb] = sum;
        }
    }
}

template <typename T, typename LT, bool CGU = false>
__global__ __launch_bounds__(SCG_BLOCK) void hop_quad_kernel(Geom g, const typename LinkLoad<LT>::Store* __restrict__ links,
                                                             const cx<T>* __restrict__ in, cx<T>* __restrict__ out, int p, int nvec,
                                                             int64_t nsb, EpiDev<T> e, int64_t cs, int64_t bps) {
    quad_body<T, LT, CGU, 0>(g, links, in, out, p, nvec, nsb, e, cs, bps);
}
// the same with non-temporal link loads (tps 12): for one-vector launches whose links outgrow the
// memory-side cache
template <typename T, typename LT, bool CGU = false>
__global__ __launch_bounds__(SCG_BLOCK) void hop_quad_nt_kernel(Geom g, const typename LinkLoad<LT>::Store* __restrict__ links,
                                                                const cx<T>* __restrict__ in, cx<T>* __restrict__ out, int p, int nvec,
                                                                int64_t nsb, EpiDev<T> e, int64_t cs, int64_t bps) {
    quad_body<T, LT, CGU, CPOL_NT>(g, links, in, out, p, nvec, nsb, e, cs, bps);
}

// LDS bytes of the staged variant for nv vectors of element size es (0 if it does not apply)
static size_t plane_lds_bytes(const Geom& g, int nv, size_t es) {
    if (g.Lxh > 256) return 0;
    return (size_t)nv * 12 * (size_t)plane_stage_sites(g) * es;
}
constexpr size_t PLANE_LDS_MAX = 64 * 1024;

static int norm_vb(int tps, int vb, int nvec) {
    vb = vb < 1 ? 1 : (vb > nvec ? nvec : vb);
    vb = vb > HOP_MAX_VB ? HOP_MAX_VB : vb;
    if (tps == 5 || tps == 6) vb = 1;
    if (tps == 7) vb = vb <= 2 ? 2 : 4;
    if (tps == 8 || tps == 9) vb = vb <= 1 ? 1 : (vb <= 2 ? 2 : 4);
    if (tps == 10 || tps == 12) vb = 1;
    if (tps == 11) vb = vb <= 1 ? 1 : 2;
    return vb;
}

bool hop_shape_ok(const Geom& g, Prec prec, int tps, int vb) {
    if (tps < 1 || tps > 12) return false;
    const size_t es = (prec == P64 || prec == P64R) ? 16 : 8;
    if (tps == 11 && es != 8) return false;   // FP32 arithmetic only (FP64 would not fit in registers)
    if (tps >= 8 && (double)g.Vh * 12.0 * (double)es >= 4294967296.0) return false;
    if (tps == 9) {
        const size_t b = plane_lds_bytes(g, norm_vb(9, vb, 4), es);
        return b > 0 && b <= PLANE_LDS_MAX;
    }
    return true;
}

static int g_order = -1;
static bool getenv_order() {
    if (g_order < 0) {
        const char* v = getenv("SEEDCG_SB_ORDER");
        g_order = v ? atoi(v) : 1;
    }
    return g_order != 0;
}

static int g_hoist = -1;
bool hop_hoist_links() {
    if (g_hoist < 0) {
        const char* v = getenv("SEEDCG_HOIST");
        g_hoist = v ? atoi(v) : 1;
    }
    return g_hoist != 0;
}
void set_hop_hoist_links(bool on) { g_hoist = on ? 1 : 0; }

// tps: 1, 2, 4 lanes per site (direction split), or the lean forward/backward variant (2 lanes)
// with 1 (tps 3), 2 (tps 5) or 4 (tps 6) directions per pass
// tps 7: the multi-vector variant (two lanes per site, links loaded once for vb vectors, vb 2 or 4)
// tps 8: the wave-split variant (forward and backward hops on separate wavefronts, vb 1, 2 or 4
// vectors per workgroup)
// tps 9: the LDS-staged variant (tiles of whole xy-rows, vb 1, 2 or 4); one workgroup per tile
// tps 10: the quad-split variant (four wavefronts per 64 sites, one vector per workgroup)
// tps 11: the link-resident variant (wave-split, one workgroup per site block for every vector of
// the launch, vb 1 or 2 at a time)
// tps 12: the quad-split variant with non-temporal link loads
int hop_threads_per_site(int tps) { return (tps == 10 || tps == 12) ? 4 : ((tps == 3 || tps >= 5) ? 2 : tps); }
int hop_site_blocks(const Geom& g, int tps) {
    if (tps == 9) return g.L[2] * g.L[3] * plane_tiles(g);
    return (int)((g.Vh * hop_threads_per_site(tps) + SCG_BLOCK - 1) / SCG_BLOCK);
}

// the wave-split (tps 8), LDS-staged (9), quad-split (10, 12) and link-resident (11) stencils; CGU: with
// the CG update fused into the epilogue
template <typename T, typename LT, bool CGU>
static void launch_wide(const Geom& g, const typename LinkLoad<LT>::Store* links, const cx<T>* in, cx<T>* out, int p, int nvec,
                        int64_t nsb, const EpiDev<T>& e, int tps, int vb, int64_t grid, int64_t bps, const Launch& L) {
    const hipStream_t s = L.s;
    const dim3 gr((unsigned)grid, 1, L.nz);
    if (tps == 10 || tps == 12) {
        const int64_t slice = g.Vh / g.L[3];
        const int64_t bps64 = (slice % SCG_WAVE == 0 && getenv_order()) ? slice / SCG_WAVE : 0;
        if (tps == 10)
            hipLaunchKernelGGL((hop_quad_kernel<T, LT, CGU>), gr, dim3(SCG_BLOCK), 0, s, g, links, in, out, p, nvec, nsb, e, L.cs, bps64);
        else
            hipLaunchKernelGGL((hop_quad_nt_kernel<T, LT, CGU>), gr, dim3(SCG_BLOCK), 0, s, g, links, in, out, p, nvec, nsb, e, L.cs,
                               bps64);
    } else if (tps == 9) {
        const size_t lds = plane_lds_bytes(g, vb, sizeof(cx<T>));
        if (lds == 0 || lds > PLANE_LDS_MAX) throw std::runtime_error("stencil launch shape does not fit this lattice");
        const int Pw = (plane_rows(g) * g.Lxh + SCG_WAVE - 1) / SCG_WAVE * SCG_WAVE;
        if (vb == 1)
            hipLaunchKernelGGL((hop_plane_kernel<T, LT, 1, CGU>), gr, dim3(2 * Pw), lds, s, g, links, in, out, p, nvec, nsb, e, L.cs, Pw);
        else if (vb == 2)
            hipLaunchKernelGGL((hop_plane_kernel<T, LT, 2, CGU>), gr, dim3(2 * Pw), lds, s, g, links, in, out, p, nvec, nsb, e, L.cs, Pw);
        else
            hipLaunchKernelGGL((hop_plane_kernel<T, LT, 4, CGU>), gr, dim3(2 * Pw), lds, s, g, links, in, out, p, nvec, nsb, e, L.cs, Pw);
    } else if (tps == 11) {
        if constexpr (!std::is_same<T, float>::value)
            throw std::runtime_error("the link-resident stencil runs in FP32 only");
        else if (vb == 1)
            hipLaunchKernelGGL((hop_stream_kernel<T, LT, 1, CGU>), gr, dim3(SCG_BLOCK), 0, s, g, links, in, out, p, nvec, nsb, e, L.cs, bps);
        else
            hipLaunchKernelGGL((hop_stream_kernel<T, LT, 2, CGU>), gr, dim3(SCG_BLOCK), 0, s, g, links, in, out, p, nvec, nsb, e, L.cs, bps);
    } else if (vb == 1)
        hipLaunchKernelGGL((hop_split_kernel<T, LT, 1, CGU>), gr, dim3(SCG_BLOCK), 0, s, g, links, in, out, p, nvec, nsb, e, L.cs, bps);
    else if (vb == 2)
        hipLaunchKernelGGL((hop_split_kernel<T, LT, 2, CGU>), gr, dim3(SCG_BLOCK), 0, s, g, links, in, out, p, nvec, nsb, e, L.cs, bps);
    else
        hipLaunchKernelGGL((hop_split_kernel<T, LT, 4, CGU>), gr, dim3(SCG_BLOCK), 0, s, g, links, in, out, p, nvec, nsb, e, L.cs, bps);
}

template <typename T, typename LT>
static void launch_t(const Geom& g, const void* links, const void* in, void* out, int p, int nvec, const HopEpi& epi,
                     int tps, int vb, const Launch& L) {
    const hipStream_t s = L.s;
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
    e.kappa2_dev = epi.kappa2_dev;
    e.X = (cx<double>*)epi.X;
    e.R = (cx<T>*)epi.R;
    if (epi.red == 3 && (!epi.cg || !epi.d || !epi.X || !epi.R || !epi.combine || epi.z || tps < 8 ||
                         (double)g.Vh * 12.0 * 16.0 >= 4294967296.0))
        throw std::runtime_error("fused CG update: needs cg, p, X, R, the combine and a tps 8 to 11 stencil");
    const int64_t nsb = hop_site_blocks(g, tps);
    vb = norm_vb(tps, vb, nvec);
    // the wave-split kernels address a vector with 32-bit byte offsets, the staged one needs its LDS:
    // the handle's shapes were checked with hop_shape_ok (the reduction partials depend on the shape)
    if (tps >= 8 && (double)g.Vh * 12.0 * (double)sizeof(cx<T>) >= 4294967296.0)
        throw std::runtime_error("stencil launch shape does not fit this lattice");
    const int64_t grid = xcd_grid(tps == 11 ? nsb : nsb * ((nvec + vb - 1) / vb));
    // site blocks per t-slice for the tiled visiting order (two lanes per site, 128 sites a block)
    const int64_t slice = g.Vh / g.L[3];
    const int64_t bps = (slice % (SCG_BLOCK / 2) == 0 && getenv_order()) ? slice / (SCG_BLOCK / 2) : 0;
    using S = typename LinkLoad<LT>::Store;
    // links kept in registers across the vectors of a workgroup when one lane holds one direction
    const bool hoist = tps == 4 && hop_hoist_links();
    if (tps >= 8) {
        if (epi.red == 3)
            launch_wide<T, LT, true>(g, (const S*)links, (const cx<T>*)in, (cx<T>*)out, p, nvec, nsb, e, tps, vb, grid, bps, L);
        else
            launch_wide<T, LT, false>(g, (const S*)links, (const cx<T>*)in, (cx<T>*)out, p, nvec, nsb, e, tps, vb, grid, bps, L);
        return;
    }
    if (tps == 3 && vb == 1)
        hipLaunchKernelGGL((hop_lean_kernel<T, LT, true, 1>), dim3((unsigned)grid, 1, L.nz), dim3(SCG_BLOCK), 0, s, g, (const S*)links,
                           (const cx<T>*)in, (cx<T>*)out, p, nvec, vb, nsb, e, L.cs, bps);
    else if (tps == 3)
        hipLaunchKernelGGL((hop_lean_kernel<T, LT, false, 1>), dim3((unsigned)grid, 1, L.nz), dim3(SCG_BLOCK), 0, s, g, (const S*)links,
                           (const cx<T>*)in, (cx<T>*)out, p, nvec, vb, nsb, e, L.cs, bps);
    else if (tps == 7 && vb == 2)
        hipLaunchKernelGGL((hop_multi_kernel<T, LT, 2>), dim3((unsigned)grid, 1, L.nz), dim3(SCG_BLOCK), 0, s, g, (const S*)links,
                           (const cx<T>*)in, (cx<T>*)out, p, nvec, nsb, e, L.cs, bps);
    else if (tps == 7)
        hipLaunchKernelGGL((hop_multi_kernel<T, LT, 4>), dim3((unsigned)grid, 1, L.nz), dim3(SCG_BLOCK), 0, s, g, (const S*)links,
                           (const cx<T>*)in, (cx<T>*)out, p, nvec, nsb, e, L.cs, bps);
    else if (tps == 5)
        hipLaunchKernelGGL((hop_lean_kernel<T, LT, true, 2>), dim3((unsigned)grid, 1, L.nz), dim3(SCG_BLOCK), 0, s, g, (const S*)links,
                           (const cx<T>*)in, (cx<T>*)out, p, nvec, 1, nsb, e, L.cs, bps);
    else if (tps == 6)
        hipLaunchKernelGGL((hop_lean_kernel<T, LT, true, 4>), dim3((unsigned)grid, 1, L.nz), dim3(SCG_BLOCK), 0, s, g, (const S*)links,
                           (const cx<T>*)in, (cx<T>*)out, p, nvec, 1, nsb, e, L.cs, bps);
    else if (tps == 1)
        hipLaunchKernelGGL((hop_kernel<T, LT, 1, false>), dim3((unsigned)grid, 1, L.nz), dim3(SCG_BLOCK), 0, s, g, (const S*)links,
                           (const cx<T>*)in, (cx<T>*)out, p, nvec, vb, nsb, e, L.cs);
    else if (tps == 2)
        hipLaunchKernelGGL((hop_kernel<T, LT, 2, false>), dim3((unsigned)grid, 1, L.nz), dim3(SCG_BLOCK), 0, s, g, (const S*)links,
                           (const cx<T>*)in, (cx<T>*)out, p, nvec, vb, nsb, e, L.cs);
    else if (hoist)
        hipLaunchKernelGGL((hop_kernel<T, LT, 4, true>), dim3((unsigned)grid, 1, L.nz), dim3(SCG_BLOCK), 0, s, g, (const S*)links,
                           (const cx<T>*)in, (cx<T>*)out, p, nvec, vb, nsb, e, L.cs);
    else
        hipLaunchKernelGGL((hop_kernel<T, LT, 4, false>), dim3((unsigned)grid, 1, L.nz), dim3(SCG_BLOCK), 0, s, g, (const S*)links,
                           (const cx<T>*)in, (cx<T>*)out, p, nvec, vb, nsb, e, L.cs);
}

void launch_hop(Prec prec, const Geom& g, const void* links, const void* in, void* out, int out_parity, int nvec,
                const HopEpi& epi, int tps, int vb, const Launch& L) {
    if (prec == P64)
        launch_t<double, double>(g, links, in, out, out_parity, nvec, epi, tps, vb, L);
    else if (prec == P64R)
        launch_t<double, su3rows<double>>(g, links, in, out, out_parity, nvec, epi, tps, vb, L);
    else if (prec == P32)
        launch_t<float, float>(g, links, in, out, out_parity, nvec, epi, tps, vb, L);
    else if (prec == P32R)
        launch_t<float, su3rows<float>>(g, links, in, out, out_parity, nvec, epi, tps, vb, L);
    else
        launch_t<float, bf16link>(g, links, in, out, out_parity, nvec, epi, tps, vb, L);
}

}  // namespace scg
