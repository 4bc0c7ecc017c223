// Internal declarations of the Seed-CG library: layouts, geometry, device helpers.
//
// Internal layouts (the C ABI's canonical layouts are repacked at the boundary):
//   spinor field   [12 components][Vh] complex, component = 3*spin + colour; a batch of
//                  vectors is [vec][12][Vh].  Lanes of a wavefront take consecutive sites,
//                  so every component load is a contiguous 64 x 16 B (FP64) segment.
//   gauge links    [mu][parity][9][Vh] complex, entry a*3+b of U_mu at the site of that
//                  parity with checkerboard index h (site s = 2h or 2h+1).
//   Krylov basis   [m][12*Vh] complex, one vector after another.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#define SCG_WAVE 64
#define SCG_BLOCK 256
#define SCG_NXCD 8

namespace scg {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T re, im;
};

template <typename T>
__host__ __device__ inline cx<T> mk(T r, T i) {
    cx<T> c;
    c.re = r;
    c.im = i;
    return c;
}
template <typename T>
__device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return mk<T>(a.re + b.re, a.im + b.im); }
template <typename T>
__device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return mk<T>(a.re - b.re, a.im - b.im); }
template <typename T>
__device__ inline cx<T> operator*(T s, cx<T> a) { return mk<T>(s * a.re, s * a.im); }
template <typename T>
__device__ inline cx<T> cmul(cx<T> a, cx<T> b) {
    return mk<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// conj(a) * b
template <typename T>
__device__ inline cx<T> cjmul(cx<T> a, cx<T> b) {
    return mk<T>(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <typename T>
__device__ inline cx<T> timesI(cx<T> a) { return mk<T>(-a.im, a.re); }
template <typename T>
__device__ inline cx<T> timesMinusI(cx<T> a) { return mk<T>(a.im, -a.re); }

// Lattice geometry of one configuration.
struct Geom {
    int L[4];       // Lx, Ly, Lz, Lt
    int Lxh;        // Lx / 2
    int64_t V, Vh;  // sites, sites per parity
    int t_bc;       // boundary sign in t
};

// XCD-aware block order: the hardware hands consecutive workgroups to the 8 XCDs in turn;
// remapping gives every XCD a contiguous run of logical blocks so that neighbouring sites
// (and the several right-hand sides of one site block) share that XCD's L2.
// The grid is padded to a multiple of 8; a logical id >= nblocks exits.
__device__ inline int64_t xcd_logical_block(int64_t nblocks) {
    const int64_t nb8 = (int64_t)gridDim.x;
    const int64_t per = nb8 / SCG_NXCD;
    const int64_t b = blockIdx.x;
    return (b % SCG_NXCD) * per + b / SCG_NXCD;
}
inline int64_t xcd_grid(int64_t nblocks) { return (nblocks + SCG_NXCD - 1) / SCG_NXCD * SCG_NXCD; }

// A batch of same-shape configurations shares one allocation per buffer family laid out so
// that every per-configuration buffer of configuration c sits exactly c * cs bytes after
// configuration 0's.  A launch then covers all configurations with grid.z = nz, and each
// kernel moves its pointer arguments by blockIdx.z * cs (cs = 0, nz = 1 for a single one).
struct Launch {
    hipStream_t s;
    int nz;
    int64_t cs;
    Launch(hipStream_t s_ = nullptr, int nz_ = 1, int64_t cs_ = 0) : s(s_), nz(nz_), cs(cs_) {}
};
template <typename P>
__device__ inline P* zoff(P* p, int64_t cs) {
    return p ? (P*)((char*)p + (int64_t)blockIdx.z * cs) : p;
}

// Deterministic block reduction of one double (fixed shuffle tree, then waves in order).
__device__ inline double block_sum(double v, double* lds /* >= SCG_BLOCK/SCG_WAVE */) {
    for (int off = SCG_WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x % SCG_WAVE, wave = threadIdx.x / SCG_WAVE;
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x / SCG_WAVE); w++) s += lds[w];
    return s;  // valid in thread 0
}

// Sum n partials in a fixed order with one workgroup; result valid in thread 0.
__device__ inline double block_sum_array(const double* p, int64_t n, double* lds) {
    double v = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) v += p[k];
    return block_sum(v, lds);
}

// Device-side state of Algorithm 1 for one solve.
struct LzState {
    int32_t m;          // last step to run (m_cap until i_conv is known)
    int32_t m_cap;
    int32_t i_conv;     // 0 until the residual estimate meets tol
    int32_t done;       // 1 when the run has ended
    int32_t status;     // 0 ok, 1 breakdown, 2 indefinite, 3 capped
    int32_t passes;     // Gram-Schmidt passes
    int32_t rep_v, rep_f;  // DGKS repeat requested for v_i / f
    int32_t rep_any;       // rep_v | rep_f (gate of the second pass)
    int32_t pad_;
    double beta0, bnorm1, tol, past, max_abs_alpha;
    double f2_before;   // ||f||^2 before the reorthogonalisation of this step
    double v2_before;   // ||v_i||^2 before it
    double nv, e;       // reorth: ||v'|| and (v'^dag f') / ||v'||^2 (re, im in e, e_im)
    double e_im;
    double orth_loss;   // max over the reorthogonalisation passes of max_{j<i} |v_j^dag v_i| / ||v_i||
};

// Device-side scalars of the multi-RHS CG.
struct CgVec {
    double rr, rr_old, pq, a, b, bnorm, tol;
    double rr_reliable;  // true |r|^2 at the previous reliable update (mixed precision)
    double rz;           // Re r^dag z with z = P r (preconditioned CG)
    int32_t iters, done, frozen, restarts;
};

}  // namespace scg

// ---- launchers implemented in the .hip files -------------------------------------------------
namespace scg {

// P64R / P32R: links stored as their first two rows (special unitary fields only)
enum Prec { P64 = 0, P32 = 1, P32BF = 2, P64R = 3, P32R = 4 };

struct HopEpi {
    // y = [gamma5] (x - kappa^2 * hop);  out = sy*y + [cz * z]; optional reduction
    int apply_g5;      // 1: gamma5 on the combined result
    int combine;       // 0: out = hop; 1: y as above
    double kappa2;
    double sy;
    const void* x;     // vectors added in the combine (same batch layout as out)
    const void* z;     // extra vector term
    const double* cz_dev;  // device coefficient per vector (or NULL -> cz_host)
    int cz_negate;     // use -cz_dev[v]
    double cz_host;
    int red;           // 0 none, 1 Re sum conj(d) * out, 2 sum |out|^2, 3 the CG update below
    const void* d;
    double* partials;  // [vec][nblocks_site]
    const int32_t* gate_m;  // if non-null: skip when gate_i > *gate_m
    int32_t gate_i;
    const int32_t* vec_map; // optional: vector slot -> stored vector index (-1: empty slot)
    const CgVec* cg;   // optional: skip vectors whose CG is done or frozen
    const double* kappa2_dev;  // optional: kappa^2 from device memory (per configuration)
    // red 3: out (q) is not stored; instead X += a p and R -= a q with a = cg[vec].a, p = d, and the
    // partials hold |R|^2.  X is FP64, R in the launch precision; needs cg and launch shape tps 8, 9 or 10.
    void* X;
    void* R;
};

// out(parity p) = H_{p,1-p} in, with the epilogue above, for nvec vectors.
// vb: vectors per workgroup (the links of a site are loaded once per workgroup)
void launch_hop(Prec prec, const Geom& g, const void* links, const void* in, void* out, int out_parity,
                int nvec, const HopEpi& epi, int tps, int vb, const Launch& L);
int hop_site_blocks(const Geom& g, int tps);
// whether launch shape (tps, vb) of the stencil can run on this lattice at this precision
bool hop_shape_ok(const Geom& g, Prec prec, int tps, int vb);
bool hop_hoist_links();
void set_hop_hoist_links(bool on);

}  // namespace scg
