// Learned gauge-covariant preconditioner P = K K^dag: forward and adjoint layers, weight
// gradients, Adam, and the Ritz-vector combination that builds its training set.
//
//   (L psi)(x) = sum_{d=0..8} (w_d (x) 1_3)(T_d psi)(x),   T_0 = 1,
//   T_{+mu} psi(x) = U_mu(x) psi(x+mu),  T_{-mu} psi(x) = U_mu(x-mu)^dag psi(x-mu)
//   (fermion boundary sign on hops across the t boundary; d = 1..4 is +x..+t, 5..8 is -x..-t),
//   L^dag = sum_d (w_d^dag (x) 1_3) T_{-d},   K = R_e L_3 L_2 L_1 E_e,   K^dag = R_e L_1^dag L_2^dag L_3^dag E_e.
//
// Full-lattice fields are [vec][parity][12][Vh] complex FP32 (the even block is an even-site
// vector in the library's internal layout); the weights are FP32 for the kernels with an FP64
// master copy for Adam.  Weight gradients are accumulated per direction over sites, colours and
// vectors in FP64 (deterministic block partials, then a fixed-order sum).
#include <stdexcept>

#include "kernels.h"

namespace scg {

__device__ inline int adj_dir(int d) { return d == 0 ? 0 : (d <= 4 ? d + 4 : d - 4); }

struct Site {
    int x, y, z, t, xh;
    int row;
};
// 32-bit site decoding (Vh < 2^31 at every lattice this library accepts)
__device__ inline Site site_of(const Geom& g, int p, int h) {
    Site s;
    const int Lxh = g.Lxh, Ly = g.L[1], Lz = g.L[2];
    s.xh = h % Lxh;
    int r = h / Lxh;
    s.y = r % Ly;
    r /= Ly;
    s.z = r % Lz;
    s.t = r / Lz;
    s.x = 2 * s.xh + ((s.y + s.z + s.t + p) & 1);
    s.row = h - s.xh;
    return s;
}
// checkerboard index of the neighbour in direction mu, step +-1, and the boundary sign
__device__ inline int nb_index(const Geom& g, const Site& s, int mu, int step, float& sign) {
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3], Lxh = g.Lxh;
    sign = 1.f;
    if (mu == 0) {
        int xn = s.x + step;
        xn = xn < 0 ? xn + Lx : (xn >= Lx ? xn - Lx : xn);
        return s.row + (xn >> 1);
    }
    if (mu == 1) {
        int yn = s.y + step;
        yn = yn < 0 ? yn + Ly : (yn >= Ly ? yn - Ly : yn);
        return s.xh + Lxh * (yn + Ly * (s.z + Lz * s.t));
    }
    if (mu == 2) {
        int zn = s.z + step;
        zn = zn < 0 ? zn + Lz : (zn >= Lz ? zn - Lz : zn);
        return s.xh + Lxh * (s.y + Ly * (zn + Lz * s.t));
    }
    if ((step == 1 && s.t == Lt - 1) || (step == -1 && s.t == 0)) sign = (float)g.t_bc;
    int tn = s.t + step;
    tn = tn < 0 ? tn + Lt : (tn >= Lt ? tn - Lt : tn);
    return s.xh + Lxh * (s.y + Ly * (s.z + Lz * tn));
}

// the link of transport d at output site (p, h): U_mu(x) (d = +mu) or U_mu(x - mu) (d = -mu), read once
// per site and direction and applied to every vector of the thread.  NE = 9: links stored whole
// ([mu][parity][9][Vh]); NE = 6: special-unitary links stored as rows 0 and 1 ([mu][parity][6][Vh]),
// row 2 rebuilt as conj(row 0 x row 1)
struct Hop {
    cx<float> u[9];
    int hn;
    float sign;
    bool fwd;
};
__device__ inline cx<float> conj_cx(cx<float> a) { return mk<float>(a.re, -a.im); }

// Raw buffer loads: the base of a field in scalar registers and one 32-bit byte offset per lane, the
// component's offset in the scalar soffset operand, instead of a 64-bit address per component.  The
// bases (a direction's links, one vector's field) are uniform over the workgroup, and every field
// spans fewer than 2^32 bytes (k_layer and k_grad check it).
__device__ inline __amdgpu_buffer_rsrc_t kbuf(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ inline cx<float> kld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(cx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
// one vector's field [2][12][Vh] at base + vec * vs (vs < 24 Vh: the even half only, vs complex)
__device__ inline __amdgpu_buffer_rsrc_t kfield(const cx<float>* base, int vec, int64_t vs, int64_t Vh) {
    const int v = __builtin_amdgcn_readfirstlane(vec);
    return kbuf(base + (int64_t)v * vs, (uint32_t)((vs < 24 * Vh ? vs : 24 * Vh) * (int64_t)sizeof(cx<float>)));
}

template <int NE>
__device__ inline void load_hop(const Geom& g, const cx<float>* __restrict__ links, int p, int h, const Site& s, int d, Hop& o) {
    const uint32_t Vh = (uint32_t)g.Vh;
    const int mu = (d - 1) & 3;
    o.fwd = d <= 4;
    o.hn = nb_index(g, s, mu, o.fwd ? 1 : -1, o.sign);
    const uint32_t lp = (uint32_t)(o.fwd ? p : 1 - p);
    const uint32_t lh = (uint32_t)(o.fwd ? h : o.hn);
    // the links of direction mu, both parities: [parity][NE][Vh]
    const auto lr = kbuf(links + (size_t)mu * 2 * NE * Vh, 2u * NE * Vh * (uint32_t)sizeof(cx<float>));
    const uint32_t voff = (lp * NE * Vh + lh) * (uint32_t)sizeof(cx<float>);
#pragma unroll
    for (int c = 0; c < NE; c++) o.u[c] = kld(lr, voff, (uint32_t)c * Vh * (uint32_t)sizeof(cx<float>));
    if constexpr (NE == 6) {
        o.u[6] = conj_cx(cmul(o.u[1], o.u[5]) - cmul(o.u[2], o.u[4]));
        o.u[7] = conj_cx(cmul(o.u[2], o.u[3]) - cmul(o.u[0], o.u[5]));
        o.u[8] = conj_cx(cmul(o.u[0], o.u[4]) - cmul(o.u[1], o.u[3]));
    }
}
// (T_d src)(p, h) with the link of o; src is the field of one vector, [2][12][Vh]
__device__ inline void apply_hop(const Hop& o, __amdgpu_buffer_rsrc_t src, int p, uint32_t Vh, cx<float> t[12]) {
    const uint32_t voff = ((uint32_t)(1 - p) * 12u * Vh + (uint32_t)o.hn) * (uint32_t)sizeof(cx<float>);
#pragma unroll
    for (int sp = 0; sp < 4; sp++) {
        cx<float> v[3];
#pragma unroll
        for (int b = 0; b < 3; b++) v[b] = kld(src, voff, (uint32_t)(3 * sp + b) * Vh * (uint32_t)sizeof(cx<float>));
#pragma unroll
        for (int a = 0; a < 3; a++) {
            cx<float> acc = mk<float>(0.f, 0.f);
#pragma unroll
            for (int b = 0; b < 3; b++) acc = acc + (o.fwd ? cmul(o.u[a * 3 + b], v[b]) : cjmul(o.u[b * 3 + a], v[b]));
            t[3 * sp + a] = o.sign * acc;
        }
    }
}

// Sites of a launch: the output parities of pmask (1 = even only, 2 = odd only, 3 = both) on the
// band of nt consecutive t-slices starting at slice t0 (wrapping around the lattice; nt = Lt is the
// whole lattice).  A t-slice holds S = Vh / Lt sites of each parity, contiguous in the checkerboard
// index, so the grid index k runs over the selected parities, nt * S sites each.
struct Band {
    int t0, nt;
};
__device__ inline bool site_of_launch(const Geom& g, int pmask, Band b, int64_t k, int& p, int& h) {
    const int S = (int)(g.Vh / g.L[3]);
    const int per = b.nt * S;
    const int np = pmask == 3 ? 2 : 1;
    if (k >= (int64_t)np * per) return false;
    const int kk = (int)k;
    const int pi = kk / per;
    const int rem = kk - pi * per;
    p = pmask == 2 ? 1 : (pmask == 1 ? 0 : pi);
    const int ts = rem / S;
    int t = b.t0 + ts;
    if (t >= g.L[3]) t -= g.L[3];
    h = t * S + (rem - ts * S);
    return true;
}
// with an even-only input (E_e x) the transport T_d vanishes at odd sites for d = 0 and at even
// sites for the hops
__device__ inline bool vanishes(int zero_odd_input, int d, int p) { return zero_odd_input && ((d == 0) ? (p == 1) : (p == 0)); }

// One term of a layer at output site (p, h): acc += (w_d (x) 1) (T_d in) for the NV vectors of vec.
template <int NV, int NE>
__device__ __attribute__((always_inline)) inline void k_layer_term(int d, const Geom& g, const cx<float>* __restrict__ links,
                                                                   const cx<float>* __restrict__ in, const cx<float>* w,
                                                                   const int (&vec)[NV], int zero_odd_input, Band in_band, int p,
                                                                   int h, const Site& s, int Vh, int64_t in_vs, cx<float> (&acc)[NV][12]) {
    if (vanishes(zero_odd_input, d, p)) return;
    // an input known to vanish outside its band of t-slices (a back-propagated gradient): skip the
    // terms that would read it there
    if (in_band.nt < g.L[3]) {
        int tin = s.t;
        if (d == 4) tin = s.t + 1 == g.L[3] ? 0 : s.t + 1;
        if (d == 8) tin = s.t == 0 ? g.L[3] - 1 : s.t - 1;
        const int dt = tin - in_band.t0 < 0 ? tin - in_band.t0 + g.L[3] : tin - in_band.t0;
        if (dt >= in_band.nt) return;
    }
    Hop o;
    if (d) load_hop<NE>(g, links, p, h, s, d, o);
#pragma unroll
    for (int j = 0; j < NV; j++) {
        if (vec[j] < 0) continue;
        const auto src = kfield(in, vec[j], in_vs, Vh);
        cx<float> t[12];
        if (d == 0) {
            const uint32_t voff = ((uint32_t)p * 12u * (uint32_t)Vh + (uint32_t)h) * (uint32_t)sizeof(cx<float>);
#pragma unroll
            for (int c = 0; c < 12; c++) t[c] = kld(src, voff, (uint32_t)c * (uint32_t)Vh * (uint32_t)sizeof(cx<float>));
        } else {
            apply_hop(o, src, p, (uint32_t)Vh, t);
        }
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 4; b++) {
                const cx<float> wab = w[d * 16 + a * 4 + b];
#pragma unroll
                for (int c = 0; c < 3; c++) acc[j][3 * a + c] = acc[j][3 * a + c] + cmul(wab, t[3 * b + c]);
            }
    }
}

// out = L in (dagger = 0) or L^dag in (dagger = 1) on the output parities of pmask, for the vectors
// listed in vmap (or 0..nvec-1): NV vectors per thread, every link read once per site and direction.
// NG = 4: a workgroup takes 64 sites, one wavefront per quarter of the nine terms (the identity and
// the forward x and y transports, forward z and t, backward x and y, backward z and t), so each lane
// follows a quarter of the chain of dependent loads; the other three quarters' sums reach the first
// wavefront through LDS and are added in that order.  NG = 2: 128 sites, waves 0-1 the identity and
// the forward transports, waves 2-3 the backward ones.  The narrow launches of the training take
// NG = 4 (latency-bound), launches of several vector groups NG = 2 (fewer link reads per site
// block).  Workgroup b takes vector group
// b % nvg of site block b / nvg, so the groups of one site block run as neighbouring workgroups and
// find its links in L2.
template <int NV, int NE, int NG>
__global__ __launch_bounds__(256) void k_layer_kernel(Geom g, const cx<float>* __restrict__ links, const cx<float>* __restrict__ in,
                                                      cx<float>* __restrict__ out, const cx<float>* __restrict__ W, int dagger,
                                                      const int32_t* vmap, int nvec, int zero_odd_input, int pmask, Band band,
                                                      Band in_band, int64_t in_vs) {
    static_assert(NG == 2 || NG == 4, "two or four wavefront groups");
    constexpr int K_LAYER_SITES = 256 / NG;
    __shared__ cx<float> w[9 * 16];
    __shared__ cx<float> xch[(NG - 1) * NV * 12 * K_LAYER_SITES];
    for (int k = threadIdx.x; k < 9 * 16; k += blockDim.x) {
        const int d = k / 16, e = k % 16, a = e / 4, b = e % 4;
        if (!dagger) {
            w[k] = W[d * 16 + e];
        } else {  // the hop T_d carries w_{-d}^dag
            const cx<float> v = W[adj_dir(d) * 16 + b * 4 + a];
            w[k] = mk<float>(v.re, -v.im);
        }
    }
    __syncthreads();
    const int nvg = (nvec + NV - 1) / NV;
    const int vg = (int)(blockIdx.x % (unsigned)nvg);
    const int64_t sb = blockIdx.x / (unsigned)nvg;
    const int grp = (int)(threadIdx.x / K_LAYER_SITES);   // uniform over the wavefront
    const int sl = (int)(threadIdx.x % K_LAYER_SITES);
    int p = 0, h = 0;
    const bool valid = site_of_launch(g, pmask, band, sb * K_LAYER_SITES + sl, p, h);
    const int Vh = (int)g.Vh;
    int vec[NV];
#pragma unroll
    for (int j = 0; j < NV; j++) {
        const int slot = vg * NV + j;
        vec[j] = slot < nvec ? (vmap ? vmap[slot] : slot) : -1;
    }
    cx<float> acc[NV][12];
#pragma unroll
    for (int j = 0; j < NV; j++)
#pragma unroll
        for (int c = 0; c < 12; c++) acc[j][c] = mk<float>(0.f, 0.f);
    if (valid) {
        const Site s = site_of(g, p, h);
        // the directions unrolled, so that each one's transport is resolved at compile time
        if (NG == 2 && grp == 0) {
#pragma unroll
            for (int d = 0; d < 5; d++) k_layer_term<NV, NE>(d, g, links, in, w, vec, zero_odd_input, in_band, p, h, s, Vh, in_vs, acc);
        } else if (NG == 2) {
#pragma unroll
            for (int d = 5; d < 9; d++) k_layer_term<NV, NE>(d, g, links, in, w, vec, zero_odd_input, in_band, p, h, s, Vh, in_vs, acc);
        } else if (grp == 0) {
#pragma unroll
            for (int d = 0; d < 3; d++) k_layer_term<NV, NE>(d, g, links, in, w, vec, zero_odd_input, in_band, p, h, s, Vh, in_vs, acc);
        } else if (grp == 1) {
#pragma unroll
            for (int d = 3; d < 5; d++) k_layer_term<NV, NE>(d, g, links, in, w, vec, zero_odd_input, in_band, p, h, s, Vh, in_vs, acc);
        } else if (grp == 2) {
#pragma unroll
            for (int d = 5; d < 7; d++) k_layer_term<NV, NE>(d, g, links, in, w, vec, zero_odd_input, in_band, p, h, s, Vh, in_vs, acc);
        } else {
#pragma unroll
            for (int d = 7; d < 9; d++) k_layer_term<NV, NE>(d, g, links, in, w, vec, zero_odd_input, in_band, p, h, s, Vh, in_vs, acc);
        }
    }
    if (grp > 0) {
#pragma unroll
        for (int j = 0; j < NV; j++)
#pragma unroll
            for (int c = 0; c < 12; c++) xch[(((grp - 1) * NV + j) * 12 + c) * K_LAYER_SITES + sl] = acc[j][c];
    }
    __syncthreads();
    if (grp > 0 || !valid) return;
#pragma unroll
    for (int j = 0; j < NV; j++) {
        if (vec[j] < 0) continue;
        cx<float>* dst = out + (int64_t)vec[j] * 24 * Vh + (int64_t)p * 12 * Vh + h;
#pragma unroll
        for (int c = 0; c < 12; c++) {
            cx<float> o = acc[j][c];
#pragma unroll
            for (int q = 0; q < NG - 1; q++) o = o + xch[((q * NV + j) * 12 + c) * K_LAYER_SITES + sl];
            dst[(int64_t)c * Vh] = o;
        }
    }
}

// the 32-bit byte offsets of the buffer loads: a vector's field (24 Vh complex) and a direction's
// links (2 x 9 Vh complex at most) stay below 2^32 bytes
bool k_offsets_fit(const Geom& g) { return (double)g.Vh * 24.0 * (double)sizeof(cx<float>) < 4294967296.0; }

// the band of t-slices [t0, t0 + nt) (mod Lt); nt <= 0 or nt >= Lt is the whole lattice
Band make_band(const Geom& g, int t0, int nt) {
    if (nt <= 0 || nt >= g.L[3]) return Band{0, g.L[3]};
    t0 %= g.L[3];
    if (t0 < 0) t0 += g.L[3];
    return Band{t0, nt};
}
int64_t k_sites(const Geom& g, int pmask, Band b) { return (int64_t)(pmask == 3 ? 2 : 1) * b.nt * (g.Vh / g.L[3]); }

void k_layer(const Geom& g, KLinks links, const void* in, void* out, const void* W, bool dagger, const int32_t* vmap, int nvec,
             bool zero_odd_input, hipStream_t s, int pmask, int t0, int nt, int in_t0, int in_nt, int64_t in_vstride) {
    // two vectors per thread (four would spill and run one wave per SIMD)
    constexpr int NV = 2;
    const int64_t in_vs = in_vstride ? in_vstride : 24 * g.Vh;
    if (in_vs < 24 * g.Vh && !(zero_odd_input && in_vs >= 12 * g.Vh))
        throw std::invalid_argument("k_layer: an input of even-site vectors must be declared even-only");
    if (links.ne != 6 && links.ne != 9) throw std::invalid_argument("k_layer: links hold 6 or 9 entries");
    if (!k_offsets_fit(g)) throw std::invalid_argument("k_layer: a field of this lattice spans 2^32 bytes or more");
    const Band b = make_band(g, t0, nt), ib = make_band(g, in_t0, in_nt);
    // one vector group: four wavefront groups of 64 sites; several: two of 128
    const int64_t nvg = nvec == 1 ? 1 : (nvec + NV - 1) / NV;
    const int64_t sites_per_wg = nvg == 1 ? 64 : 128;
    const int64_t nsb = (k_sites(g, pmask, b) + sites_per_wg - 1) / sites_per_wg;
    const unsigned grid = (unsigned)(nsb * nvg);
    const auto lk = (const cx<float>*)links.p;
    const auto in32 = (const cx<float>*)in;
    const auto out32 = (cx<float>*)out;
    const auto W32 = (const cx<float>*)W;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, s, g, lk, in32, out32, W32, (int)dagger, vmap, nvec, (int)zero_odd_input,
                           pmask, b, ib, in_vs);
    };
    if (nvec == 1)
        links.ne == 6 ? go(k_layer_kernel<1, 6, 4>) : go(k_layer_kernel<1, 9, 4>);
    else if (nvg == 1)
        links.ne == 6 ? go(k_layer_kernel<NV, 6, 4>) : go(k_layer_kernel<NV, 9, 4>);
    else
        links.ne == 6 ? go(k_layer_kernel<NV, 6, 2>) : go(k_layer_kernel<NV, 9, 2>);
}

// partial sums over the sites of pmask, colours and vectors of g[a][c] conj((T_dt in)[b][c]) for
// direction d = blockIdx.y, with dt = d (layer L) or dt = -d (layer L^dag); each link is read once per
// site for all vectors.  A thread takes spt sites (a workgroup spt consecutive runs of 256; 2, or 1 on
// the narrowest bands) and sums their terms in FP32; the workgroup's sum is FP64.  part[d][block][16] complex.
// (Workgroups of 256 threads: the reduction below assumes it.)
template <int NE>
__global__ __launch_bounds__(256) void k_grad_kernel(Geom g, const cx<float>* __restrict__ links, const cx<float>* __restrict__ gv,
                                                     const cx<float>* __restrict__ in, int dagger, int nvec, int zero_odd_input,
                                                     int pmask, Band band, double* part, int64_t in_vs, int spt) {
    __shared__ double lds[8 * 32];
    __shared__ float tile[256 * 33];
    const int d = blockIdx.y;
    const int dt = dagger ? adj_dir(d) : d;
    const int Vh = (int)g.Vh;
    float acc[32];
#pragma unroll
    for (int e = 0; e < 32; e++) acc[e] = 0.f;
#pragma unroll 1
    for (int r = 0; r < spt; r++) {
        int p, h;
        const int64_t k = ((int64_t)blockIdx.x * spt + r) * blockDim.x + threadIdx.x;
        if (!site_of_launch(g, pmask, band, k, p, h) || vanishes(zero_odd_input, dt, p)) continue;
        const Site s = site_of(g, p, h);
        Hop o;
        if (dt) load_hop<NE>(g, links, p, h, s, dt, o);
#pragma unroll 1
        for (int v = 0; v < nvec; v++) {
            const auto src = kfield(in, v, in_vs, Vh);
            const uint32_t so = (uint32_t)Vh * (uint32_t)sizeof(cx<float>);   // one component
            const uint32_t voff = ((uint32_t)p * 12u * (uint32_t)Vh + (uint32_t)h) * (uint32_t)sizeof(cx<float>);
            cx<float> t[12], q[12];
            if (dt == 0) {
#pragma unroll
                for (int c = 0; c < 12; c++) t[c] = kld(src, voff, (uint32_t)c * so);
            } else {
                apply_hop(o, src, p, (uint32_t)Vh, t);
            }
            const auto gs = kfield(gv, v, 24 * (int64_t)Vh, Vh);
#pragma unroll
            for (int c = 0; c < 12; c++) q[c] = kld(gs, voff, (uint32_t)c * so);
#pragma unroll
            for (int a = 0; a < 4; a++)
#pragma unroll
                for (int b = 0; b < 4; b++) {
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        const cx<float> pr = cjmul(t[3 * b + c], q[3 * a + c]);  // q conj(t)
                        acc[2 * (a * 4 + b)] += pr.re;
                        acc[2 * (a * 4 + b) + 1] += pr.im;
                    }
                }
        }
    }
    // the workgroup's sum through LDS: every thread's 32 values as a row, then 8 groups of 32 rows
    // summed column by column in FP64, then the 8 group sums (fixed order throughout)
#pragma unroll
    for (int e = 0; e < 32; e++) tile[threadIdx.x * 33 + e] = acc[e];
    __syncthreads();
    {
        const int e = threadIdx.x % 32, grp = threadIdx.x / 32;
        double v = 0.0;
        for (int r = 0; r < 32; r++) v += (double)tile[(grp * 32 + r) * 33 + e];
        lds[grp * 32 + e] = v;
    }
    __syncthreads();
    if (threadIdx.x < 32) {
        double v = 0.0;
        for (int grp = 0; grp < 8; grp++) v += lds[grp * 32 + threadIdx.x];
        part[((int64_t)d * gridDim.x + blockIdx.x) * 32 + threadIdx.x] = v;
    }
}

// G[layer][d] += the block sums of every listed gradient of that layer, in list order (dagger layers add
// the conjugate transpose: dL/dconj(w) = G'^dag).  One workgroup of 1024 threads per (direction, layer):
// thread (j, e) adds blocks j, j+32, ... of value e, then the 32 partial sums are added in order
// (deterministic).
__global__ __launch_bounds__(1024) void k_grad_reduce_kernel(const KGradList q, double* G) {
    __shared__ double lds[32 * 32];
    const int d = blockIdx.x, layer = blockIdx.y;
    const int e = threadIdx.x % 32, j = threadIdx.x / 32;
    for (int k = 0; k < q.n; k++) {
        if (q.layer[k] != layer) continue;   // uniform
        const double* part = q.part[k];
        const int64_t nblocks = q.nb[k];
        double s = 0.0;
        for (int64_t b = j; b < nblocks; b += 32) s += part[((int64_t)d * nblocks + b) * 32 + e];
        __syncthreads();
        lds[j * 32 + e] = s;
        __syncthreads();
        if (j == 0) {
            s = 0.0;
            for (int r = 0; r < 32; r++) s += lds[r * 32 + e];
            double* Gl = G + (int64_t)layer * 9 * 32;
            if (!q.dagger[k]) {
                Gl[d * 32 + e] += s;
            } else {
                const int ab = e / 2, comp = e % 2;
                const int a = ab / 4, b = ab % 4;
                Gl[d * 32 + 2 * (b * 4 + a) + comp] += comp ? -s : s;
            }
        }
    }
}

int64_t k_grad_blocks(const Geom& g) { return (2 * g.Vh + 255) / 256; }

int64_t k_grad(const Geom& g, KLinks links, const void* gv, const void* in, bool dagger, int nvec, double* part, hipStream_t s,
               bool zero_odd_input, int pmask, int t0, int nt, int64_t in_vstride) {
    if (links.ne != 6 && links.ne != 9) throw std::invalid_argument("k_grad: links hold 6 or 9 entries");
    if (!k_offsets_fit(g)) throw std::invalid_argument("k_grad: a field of this lattice spans 2^32 bytes or more");
    const Band b = make_band(g, t0, nt);
    const int64_t in_vs = in_vstride ? in_vstride : 24 * g.Vh;
    if (in_vs < 24 * g.Vh && !(zero_odd_input && in_vs >= 12 * g.Vh))
        throw std::invalid_argument("k_grad: an input of even-site vectors must be declared even-only");
    // sites per thread: 2, or 1 where that would leave fewer than 512 workgroups (the narrowest bands)
    const int64_t sites = k_sites(g, pmask, b);
    const int spt = 9 * ((sites + 511) / 512) < 512 ? 1 : 2;
    const int64_t nb = (sites + 256 * spt - 1) / (256 * spt);
    if (links.ne == 6)
        hipLaunchKernelGGL(k_grad_kernel<6>, dim3((unsigned)nb, 9), dim3(256), 0, s, g, (const cx<float>*)links.p,
                           (const cx<float>*)gv, (const cx<float>*)in, (int)dagger, nvec, (int)zero_odd_input, pmask, b, part, in_vs,
                           spt);
    else
        hipLaunchKernelGGL(k_grad_kernel<9>, dim3((unsigned)nb, 9), dim3(256), 0, s, g, (const cx<float>*)links.p,
                           (const cx<float>*)gv, (const cx<float>*)in, (int)dagger, nvec, (int)zero_odd_input, pmask, b, part, in_vs,
                           spt);
    return nb;
}

void k_grad_reduce(const KGradList& q, double* G, hipStream_t s) {
    if (q.n < 1 || q.n > KGradList::MAX) throw std::invalid_argument("k_grad_reduce: 1..6 gradients");
    hipLaunchKernelGGL(k_grad_reduce_kernel, dim3(9, 3), dim3(1024), 0, s, q, G);
}

// field helpers on [vec][2][12][Vh] FP32 fields
template <typename TI>
__global__ void k_embed_kernel(const cx<TI>* __restrict__ x, cx<float>* __restrict__ full, int64_t n, const int32_t* vmap) {
    const int vec = vmap ? vmap[blockIdx.y] : (int)blockIdx.y;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 2 * n) return;
    cx<float> v = mk<float>(0.f, 0.f);
    if (k < n) {
        const cx<TI> a = x[(int64_t)vec * n + k];
        v = mk<float>((float)a.re, (float)a.im);
    }
    full[(int64_t)vec * 2 * n + k] = v;
}
void k_embed(bool x32, const void* x, void* full, int64_t n, const int32_t* vmap, int nvec, hipStream_t s) {
    const dim3 grid((unsigned)((2 * n + 255) / 256), (unsigned)nvec);
    if (x32)
        hipLaunchKernelGGL(k_embed_kernel<float>, grid, dim3(256), 0, s, (const cx<float>*)x, (cx<float>*)full, n, vmap);
    else
        hipLaunchKernelGGL(k_embed_kernel<double>, grid, dim3(256), 0, s, (const cx<double>*)x, (cx<float>*)full, n, vmap);
}
template <typename TO>
__global__ void k_restrict_kernel(const cx<float>* __restrict__ full, cx<TO>* __restrict__ x, int64_t n, const int32_t* vmap) {
    const int vec = vmap ? vmap[blockIdx.y] : (int)blockIdx.y;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const cx<float> a = full[(int64_t)vec * 2 * n + k];
    x[(int64_t)vec * n + k] = mk<TO>((TO)a.re, (TO)a.im);
}
void k_restrict(bool x32, const void* full, void* x, int64_t n, const int32_t* vmap, int nvec, hipStream_t s) {
    const dim3 grid((unsigned)((n + 255) / 256), (unsigned)nvec);
    if (x32)
        hipLaunchKernelGGL(k_restrict_kernel<float>, grid, dim3(256), 0, s, (const cx<float>*)full, (cx<float>*)x, n, vmap);
    else
        hipLaunchKernelGGL(k_restrict_kernel<double>, grid, dim3(256), 0, s, (const cx<float>*)full, (cx<double>*)x, n, vmap);
}
// zero the odd half (E_e R_e)
__global__ void k_zero_odd_kernel(cx<float>* full, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) full[(int64_t)blockIdx.y * 2 * n + n + k] = mk<float>(0.f, 0.f);
}
void k_zero_odd(void* full, int64_t n, int nvec, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_odd_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)nvec), dim3(256), 0, s, (cx<float>*)full, n);
}

// |u|^2 partials over the even sites of a band (the loss's normalisation), one row of blocks per vector
__global__ void k_band_norm_kernel(Geom g, Band b, const cx<float>* __restrict__ u, int64_t n, double* part) {
    __shared__ double lds[4];
    const int v = blockIdx.y;
    int p, h;
    double s = 0.0;
    if (site_of_launch(g, 1, b, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, p, h))
        for (int c = 0; c < 12; c++) {
            const cx<float> a = u[(int64_t)v * n + (int64_t)c * g.Vh + h];
            s += (double)a.re * a.re + (double)a.im * a.im;
        }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) part[(int64_t)v * gridDim.x + blockIdx.x] = s;
}
int64_t k_band_blocks(const Geom& g, int t0, int nt) { return (k_sites(g, 1, make_band(g, t0, nt)) + 255) / 256; }
void k_band_norm(const Geom& g, int t0, int nt, const void* u, int S, double* part, hipStream_t s) {
    const Band b = make_band(g, t0, nt);
    hipLaunchKernelGGL(k_band_norm_kernel, dim3((unsigned)k_band_blocks(g, t0, nt), (unsigned)S), dim3(256), 0, s, g, b,
                       (const cx<float>*)u, 12 * g.Vh, part);
}

// training residual on the even sites of a band: e = z - u there; loss partials |e|^2 / |u|^2; the
// gradient field g = E_e e / (S |u|^2) on the even sites of the band.  Nothing else of g is written:
// the layers and gradients that read g take only its even sites on that band.
__global__ void k_residual_kernel(Geom g, Band b, const cx<float>* __restrict__ zfull, const cx<float>* __restrict__ u,
                                  const double* unorm2, cx<float>* __restrict__ gfull, int64_t n, int S, double* part) {
    __shared__ double lds[4];
    const int v = blockIdx.y;
    const int per = b.nt * (int)(g.Vh / g.L[3]);   // even sites of the band
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e2 = 0.0;
    int p, h;
    if (k < 12 * (int64_t)per && site_of_launch(g, 1, b, k % per, p, h)) {
        const int64_t idx = (k / per) * g.Vh + h;   // component k / per of even site h
        const cx<float> z = zfull[(int64_t)v * 2 * n + idx], uu = u[(int64_t)v * n + idx];
        const double er = (double)z.re - uu.re, ei = (double)z.im - uu.im;
        e2 = er * er + ei * ei;
        const double sc = 1.0 / ((double)S * unorm2[v]);
        gfull[(int64_t)v * 2 * n + idx] = mk<float>((float)(er * sc), (float)(ei * sc));
    }
    const double s = block_sum(e2, lds);
    if (threadIdx.x == 0) part[(int64_t)v * gridDim.x + blockIdx.x] = s / unorm2[v];
}
int64_t k_residual_blocks(const Geom& g, int t0, int nt) { return (12 * k_sites(g, 1, make_band(g, t0, nt)) + 255) / 256; }
void k_residual(const void* zfull, const void* u, const double* unorm2, void* gfull, int64_t n, int S, double* part, hipStream_t s,
                const Geom& g, int t0, int nt) {
    const Band b = make_band(g, t0, nt);
    hipLaunchKernelGGL(k_residual_kernel, dim3((unsigned)k_residual_blocks(g, t0, nt), (unsigned)S), dim3(256), 0, s, g, b,
                       (const cx<float>*)zfull, (const cx<float>*)u, unorm2, (cx<float>*)gfull, n, S, part);
}

// Adam on the reals of 3 x 9 x 16 complex weights (FP64 master, FP32 copy for the kernels);
// the gradient accumulator is cleared for the next step.
__global__ void k_adam_kernel(double* Wm, cx<float>* W32, double* G, double* m, double* v, int t, double lr, double b1, double b2,
                              double eps, int n) {
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const double g = 2.0 * G[k];  // dL/dRe w = 2 Re dL/dconj(w), dL/dIm w = 2 Im dL/dconj(w)
        m[k] = b1 * m[k] + (1.0 - b1) * g;
        v[k] = b2 * v[k] + (1.0 - b2) * g * g;
        Wm[k] -= lr * (m[k] / c1) / (sqrt(v[k] / c2) + eps);
        G[k] = 0.0;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < n / 2; k += blockDim.x) W32[k] = mk<float>((float)Wm[2 * k], (float)Wm[2 * k + 1]);
}
void k_adam(double* Wm, void* W32, double* G, double* m, double* v, int t, double lr, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_adam_kernel, dim3(1), dim3(256), 0, s, Wm, (cx<float>*)W32, G, m, v, t, lr, 0.9, 0.999, 1e-8, n);
}

// X[j] = sum_{r < m} V[r] S[r][j], j < nout (<= 16): Ritz vectors u = V s from the stored basis
template <typename TV, typename TO>
__global__ __launch_bounds__(256) void k_combine_kernel(const cx<TV>* __restrict__ V, int m, const double* __restrict__ S, int nout,
                                                        cx<TO>* __restrict__ X, int64_t n) {
    __shared__ double sl[256 * 16];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double ar[16], ai[16];
#pragma unroll
    for (int j = 0; j < 16; j++) ar[j] = ai[j] = 0.0;
    for (int r0 = 0; r0 < m; r0 += 256) {
        const int nr = min(256, m - r0);
        __syncthreads();
        for (int q = threadIdx.x; q < nr * nout; q += blockDim.x) sl[q] = S[(int64_t)(r0 + q / nout) * nout + q % nout];
        __syncthreads();
        if (k < n)
            for (int q = 0; q < nr; q++) {
                const cx<TV> b = V[(int64_t)(r0 + q) * n + k];
#pragma unroll
                for (int j = 0; j < 16; j++)
                    if (j < nout) {
                        ar[j] += sl[q * nout + j] * (double)b.re;
                        ai[j] += sl[q * nout + j] * (double)b.im;
                    }
            }
    }
    if (k < n)
#pragma unroll
        for (int j = 0; j < 16; j++)
            if (j < nout) X[(int64_t)j * n + k] = mk<TO>((TO)ar[j], (TO)ai[j]);
}
void k_combine(bool v32, const void* V, int m, const double* S, int nout, void* X, int64_t n, hipStream_t s, bool x64) {
    const dim3 grid((unsigned)((n + 255) / 256));
    if (v32 && !x64)
        hipLaunchKernelGGL((k_combine_kernel<float, float>), grid, dim3(256), 0, s, (const cx<float>*)V, m, S, nout, (cx<float>*)X, n);
    else if (v32)
        hipLaunchKernelGGL((k_combine_kernel<float, double>), grid, dim3(256), 0, s, (const cx<float>*)V, m, S, nout, (cx<double>*)X, n);
    else if (!x64)
        hipLaunchKernelGGL((k_combine_kernel<double, float>), grid, dim3(256), 0, s, (const cx<double>*)V, m, S, nout, (cx<float>*)X, n);
    else
        hipLaunchKernelGGL((k_combine_kernel<double, double>), grid, dim3(256), 0, s, (const cx<double>*)V, m, S, nout, (cx<double>*)X, n);
}

}  // namespace scg
