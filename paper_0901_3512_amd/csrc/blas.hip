// Vector kernels of Algorithm 1 and of plain CG, and the one-workgroup scalar kernels that
// keep every recurrence on the device (no host round trip inside an iteration).
//
// Every reduction is deterministic: a fixed shuffle tree per block, then the block
// partials are summed in index order by one workgroup.
#include <algorithm>

#include "kernels.h"

namespace scg {

// ---------------------------------------------------------------------------------------------
// layout conversion at the C ABI boundary
// ---------------------------------------------------------------------------------------------
template <typename S>
__device__ inline S conv_link(cx<double> u);
template <>
__device__ inline cx<double> conv_link<cx<double>>(cx<double> u) { return u; }
template <>
__device__ inline cx<float> conv_link<cx<float>>(cx<double> u) { return mk<float>((float)u.re, (float)u.im); }
__device__ inline uint32_t bf16_bits(float f) {
    // round to nearest even
    uint32_t b = __float_as_uint(f);
    uint32_t lsb = (b >> 16) & 1u;
    b += 0x7fffu + lsb;
    return b >> 16;
}
template <>
__device__ inline uint32_t conv_link<uint32_t>(cx<double> u) {
    return bf16_bits((float)u.re) | (bf16_bits((float)u.im) << 16);
}

template <typename S>
__global__ void pack_links_kernel(Geom g, const cx<double>* __restrict__ U, S* __restrict__ out, int ne) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 4 * g.V) return;
    const int mu = (int)(k / g.V);
    const int64_t s = k % g.V;
    const int x = (int)(s % g.L[0]);
    int64_t r = s / g.L[0];
    const int y = (int)(r % g.L[1]);
    r /= g.L[1];
    const int z = (int)(r % g.L[2]);
    const int t = (int)(r / g.L[2]);
    const int par = (x + y + z + t) & 1;
    const int64_t h = s >> 1;
    for (int c = 0; c < ne; c++) out[((int64_t)(mu * 2 + par) * ne + c) * g.Vh + h] = conv_link<S>(U[k * 9 + c]);
}

void pack_links(Prec prec, const Geom& g, const double* U, void* out, hipStream_t s) {
    const int64_t n = 4 * g.V;
    const dim3 grid((unsigned)((n + 255) / 256));
    // the two-row formats keep entries 0..5 (rows 0 and 1) of every link
    const int ne = (prec == P64R || prec == P32R) ? 6 : 9;
    if (prec == P64 || prec == P64R)
        hipLaunchKernelGGL(pack_links_kernel<cx<double>>, grid, dim3(256), 0, s, g, (const cx<double>*)U, (cx<double>*)out, ne);
    else if (prec == P32 || prec == P32R)
        hipLaunchKernelGGL(pack_links_kernel<cx<float>>, grid, dim3(256), 0, s, g, (const cx<double>*)U, (cx<float>*)out, ne);
    else
        hipLaunchKernelGGL(pack_links_kernel<uint32_t>, grid, dim3(256), 0, s, g, (const cx<double>*)U, (uint32_t*)out, ne);
}

// max over links of |row 2 - conj(row 0 x row 1)| and |det U - 1| (canonical FP64 links), per
// block; the two-row link formats are used only when this is at rounding level
__global__ void su3_defect_kernel(const cx<double>* __restrict__ U, int64_t nlinks, double* part) {
    __shared__ double lds[SCG_BLOCK];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double d = 0.0;
    if (k < nlinks) {
        const cx<double>* u = U + k * 9;
        cx<double> r[3];
        r[0] = mk<double>(0, 0);
        // conj(u0 x u1)
        const cx<double> c0 = cmul(u[1], u[5]) - cmul(u[2], u[4]);
        const cx<double> c1 = cmul(u[2], u[3]) - cmul(u[0], u[5]);
        const cx<double> c2 = cmul(u[0], u[4]) - cmul(u[1], u[3]);
        r[0] = u[6] - mk<double>(c0.re, -c0.im);
        r[1] = u[7] - mk<double>(c1.re, -c1.im);
        r[2] = u[8] - mk<double>(c2.re, -c2.im);
        for (int a = 0; a < 3; a++) d = fmax(d, sqrt(r[a].re * r[a].re + r[a].im * r[a].im));
        // det U = row 2 . (row 0 x row 1)
        const cx<double> det = cmul(u[6], c0) + cmul(u[7], c1) + cmul(u[8], c2);
        d = fmax(d, sqrt((det.re - 1.0) * (det.re - 1.0) + det.im * det.im));
        if (!(d == d)) d = 1e300;   // NaN
    }
    lds[threadIdx.x] = d;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) lds[threadIdx.x] = fmax(lds[threadIdx.x], lds[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = lds[0];
}
int64_t su3_defect_blocks(int64_t nlinks) { return (nlinks + SCG_BLOCK - 1) / SCG_BLOCK; }
void su3_defect(const double* U, int64_t nlinks, double* part, hipStream_t s) {
    hipLaunchKernelGGL(su3_defect_kernel, dim3((unsigned)su3_defect_blocks(nlinks)), dim3(SCG_BLOCK), 0, s, (const cx<double>*)U,
                       nlinks, part);
}

// canonical [n][Vh][12] (FP64)  <->  internal [n][12][Vh] (T)
template <typename T>
__global__ void pack_vec_kernel(const cx<double>* __restrict__ in, cx<T>* __restrict__ out, int64_t Vh, int64_t total,
                                const double* const* tab, int64_t cs) {
    if (tab) in = (const cx<double>*)tab[blockIdx.z];
    out = zoff(out, cs);
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (vec, c, h), h fastest
    if (k >= total) return;
    const int64_t h = k % Vh;
    const int64_t c = (k / Vh) % 12;
    const int64_t v = k / (12 * Vh);
    const cx<double> a = in[(v * Vh + h) * 12 + c];
    out[k] = mk<T>((T)a.re, (T)a.im);
}
template <typename T>
__global__ void unpack_vec_kernel(const cx<T>* __restrict__ in, cx<double>* __restrict__ out, int64_t Vh, int64_t total,
                                  double* const* tab, int64_t cs) {
    if (tab) out = (cx<double>*)tab[blockIdx.z];
    in = zoff(in, cs);
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= total) return;
    const int64_t h = k % Vh;
    const int64_t c = (k / Vh) % 12;
    const int64_t v = k / (12 * Vh);
    const cx<T> a = in[k];
    out[(v * Vh + h) * 12 + c] = mk<double>((double)a.re, (double)a.im);
}

void pack_vec(bool fp32, const double* in, void* out, int64_t Vh, int nvec, const Launch& L, const double* const* tab) {
    const int64_t total = 12 * Vh * nvec;
    const dim3 grid((unsigned)((total + 255) / 256), 1, L.nz);
    if (fp32)
        hipLaunchKernelGGL(pack_vec_kernel<float>, grid, dim3(256), 0, L.s, (const cx<double>*)in, (cx<float>*)out, Vh, total, tab, L.cs);
    else
        hipLaunchKernelGGL(pack_vec_kernel<double>, grid, dim3(256), 0, L.s, (const cx<double>*)in, (cx<double>*)out, Vh, total, tab, L.cs);
}
void unpack_vec(bool fp32, const void* in, double* out, int64_t Vh, int nvec, const Launch& L, double* const* tab) {
    const int64_t total = 12 * Vh * nvec;
    const dim3 grid((unsigned)((total + 255) / 256), 1, L.nz);
    if (fp32)
        hipLaunchKernelGGL(unpack_vec_kernel<float>, grid, dim3(256), 0, L.s, (const cx<float>*)in, (cx<double>*)out, Vh, total, tab, L.cs);
    else
        hipLaunchKernelGGL(unpack_vec_kernel<double>, grid, dim3(256), 0, L.s, (const cx<double>*)in, (cx<double>*)out, Vh, total, tab, L.cs);
}

// ---------------------------------------------------------------------------------------------
// small vector helpers
// ---------------------------------------------------------------------------------------------
template <typename TA, typename TB>
__global__ void convert_kernel(const cx<TA>* __restrict__ a, cx<TB>* __restrict__ b, int64_t n, int64_t cs) {
    a = zoff(a, cs);
    b = zoff(b, cs);
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) b[k] = mk<TB>((TB)a[k].re, (TB)a[k].im);
}
void convert(bool from32, bool to32, const void* a, void* b, int64_t n, const Launch& L) {
    const hipStream_t s = L.s;
    const dim3 grid((unsigned)((n + 255) / 256), 1, L.nz);
    if (!from32 && to32)
        hipLaunchKernelGGL((convert_kernel<double, float>), grid, dim3(256), 0, s, (const cx<double>*)a, (cx<float>*)b, n, L.cs);
    else if (from32 && !to32)
        hipLaunchKernelGGL((convert_kernel<float, double>), grid, dim3(256), 0, s, (const cx<float>*)a, (cx<double>*)b, n, L.cs);
    else if (from32)
        hipLaunchKernelGGL((convert_kernel<float, float>), grid, dim3(256), 0, s, (const cx<float>*)a, (cx<float>*)b, n, L.cs);
    else
        hipLaunchKernelGGL((convert_kernel<double, double>), grid, dim3(256), 0, s, (const cx<double>*)a, (cx<double>*)b, n, L.cs);
}

// b_v = a_v (with precision change) for the vectors v of vec_map (-1: empty slot)
template <typename TA, typename TB>
__global__ void convert_map_kernel(const cx<TA>* __restrict__ a, cx<TB>* __restrict__ b, int64_t n, const int32_t* vec_map,
                                   int64_t cs) {
    a = zoff(a, cs);
    b = zoff(b, cs);
    vec_map = zoff(vec_map, cs);
    const int vec = vec_map[blockIdx.y];
    if (vec < 0) return;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const cx<TA> v = a[(int64_t)vec * n + k];
    b[(int64_t)vec * n + k] = mk<TB>((TB)v.re, (TB)v.im);
}
void convert_map(bool from32, bool to32, const void* a, void* b, int64_t n, const int32_t* vec_map, int nact, const Launch& L) {
    const dim3 grid((unsigned)((n + 255) / 256), nact, L.nz);
    if (!from32 && to32)
        hipLaunchKernelGGL((convert_map_kernel<double, float>), grid, dim3(256), 0, L.s, (const cx<double>*)a, (cx<float>*)b, n,
                           vec_map, L.cs);
    else if (!from32 && !to32)
        hipLaunchKernelGGL((convert_map_kernel<double, double>), grid, dim3(256), 0, L.s, (const cx<double>*)a, (cx<double>*)b, n,
                           vec_map, L.cs);
    else if (from32 && to32)
        hipLaunchKernelGGL((convert_map_kernel<float, float>), grid, dim3(256), 0, L.s, (const cx<float>*)a, (cx<float>*)b, n,
                           vec_map, L.cs);
    else
        hipLaunchKernelGGL((convert_map_kernel<float, double>), grid, dim3(256), 0, L.s, (const cx<float>*)a, (cx<double>*)b, n,
                           vec_map, L.cs);
}

// Byte copies between per-configuration buffers and compact staging arrays (4-byte words):
// configuration z copies src + z*src_cs to dst + z*dst_cs.  Kernels rather than memcpy/memset
// calls, so that the same code is safe inside captured graphs.
__global__ void cfg_copy_kernel(const uint32_t* src, int64_t src_cs, uint32_t* dst, int64_t dst_cs, int64_t nwords) {
    src = (const uint32_t*)((const char*)src + (int64_t)blockIdx.z * src_cs);
    dst = (uint32_t*)((char*)dst + (int64_t)blockIdx.z * dst_cs);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nwords; k += (int64_t)gridDim.x * blockDim.x)
        dst[k] = src[k];
}
void cfg_copy(const void* src, int64_t src_cs, void* dst, int64_t dst_cs, int64_t bytes, const Launch& L) {
    const int64_t nw = bytes / 4;
    const unsigned nb = (unsigned)std::min<int64_t>((nw + 255) / 256, 4096);
    hipLaunchKernelGGL(cfg_copy_kernel, dim3(std::max(nb, 1u), 1, L.nz), dim3(256), 0, L.s, (const uint32_t*)src, src_cs,
                       (uint32_t*)dst, dst_cs, nw);
}
__global__ void cfg_zero_kernel(uint32_t* dst, int64_t cs, int64_t nwords) {
    dst = (uint32_t*)((char*)dst + (int64_t)blockIdx.z * cs);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nwords; k += (int64_t)gridDim.x * blockDim.x) dst[k] = 0u;
}
void cfg_zero(void* dst, int64_t bytes, const Launch& L) {
    const int64_t nw = bytes / 4;
    const unsigned nb = (unsigned)std::min<int64_t>((nw + 255) / 256, 4096);
    hipLaunchKernelGGL(cfg_zero_kernel, dim3(std::max(nb, 1u), 1, L.nz), dim3(256), 0, L.s, (uint32_t*)dst, L.cs, nw);
}

// partial sums of |a|^2 per block, for vector v of a batch (grid: blocks x nvec)
template <typename T>
__global__ void norm2_kernel(const cx<T>* __restrict__ a, int64_t n, double* part, int64_t nb, int64_t cs) {
    __shared__ double lds[SCG_BLOCK / SCG_WAVE];
    a = zoff(a, cs);
    part = zoff(part, cs);
    const int64_t v = blockIdx.y;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (k < n) {
        const cx<T> x = a[v * n + k];
        s = (double)x.re * x.re + (double)x.im * x.im;
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) part[v * nb + blockIdx.x] = s;
}
void norm2_partials(bool fp32, const void* a, int64_t n, int nvec, double* part, const Launch& L) {
    const int64_t nb = (n + SCG_BLOCK - 1) / SCG_BLOCK;
    const dim3 grid((unsigned)nb, nvec, L.nz);
    if (fp32)
        hipLaunchKernelGGL(norm2_kernel<float>, grid, dim3(SCG_BLOCK), 0, L.s, (const cx<float>*)a, n, part, nb, L.cs);
    else
        hipLaunchKernelGGL(norm2_kernel<double>, grid, dim3(SCG_BLOCK), 0, L.s, (const cx<double>*)a, n, part, nb, L.cs);
}
int64_t norm2_blocks(int64_t n) { return (n + SCG_BLOCK - 1) / SCG_BLOCK; }

// out[v] = sum_k part[v * nb + k] (one workgroup per v)
__global__ void sum_partials_kernel(const double* part, int64_t nb, double* out, int sqrt_out, int64_t cs) {
    __shared__ double lds[SCG_BLOCK / SCG_WAVE];
    part = zoff(part, cs);
    out = zoff(out, cs);
    const double s = block_sum_array(part + (int64_t)blockIdx.x * nb, nb, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = sqrt_out ? sqrt(s) : s;
}
void sum_partials(const double* part, int64_t nb, int nvec, double* out, bool sqrt_out, const Launch& L) {
    hipLaunchKernelGGL(sum_partials_kernel, dim3(nvec, 1, L.nz), dim3(SCG_BLOCK), 0, L.s, part, nb, out, (int)sqrt_out, L.cs);
}

// ---------------------------------------------------------------------------------------------
// Algorithm 1: Lanczos vectors and the LU recurrences
// ---------------------------------------------------------------------------------------------
// Start: beta_0 = ||r_0^1|| (from partials), v_1 = r_0^1 / beta_0, bnorm1 from its partials.
template <typename T>
__global__ void lz_start_kernel(LzState* st, const double* r2part, int64_t nb, const double* b2part, double* beta, int64_t cs) {
    __shared__ double lds[SCG_BLOCK / SCG_WAVE];
    st = zoff(st, cs);
    r2part = zoff(r2part, cs);
    b2part = zoff(b2part, cs);
    beta = zoff(beta, cs);
    const double r2 = block_sum_array(r2part, nb, lds);
    __syncthreads();
    const double b2 = block_sum_array(b2part, nb, lds);
    if (threadIdx.x == 0) {
        st->beta0 = sqrt(r2);
        st->bnorm1 = sqrt(b2);
        beta[0] = st->beta0;
        if (!(st->beta0 > 0.0)) {  // zero residual: nothing to do
            st->done = 1;
            st->m = 0;
        }
    }
}
void lz_start(LzState* st, const double* r2part, int64_t nb, const double* b2part, double* beta, const Launch& L) {
    hipLaunchKernelGGL(lz_start_kernel<double>, dim3(1, 1, L.nz), dim3(SCG_BLOCK), 0, L.s, st, r2part, nb, b2part, beta, L.cs);
}

template <typename T>
__global__ void scale_from_kernel(const LzState* st, const cx<T>* __restrict__ r, cx<T>* __restrict__ v, int64_t n, int64_t cs) {
    st = zoff(st, cs);
    r = zoff(r, cs);
    v = zoff(v, cs);
    if (st->done) return;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double inv = 1.0 / st->beta0;
    const cx<T> a = r[k];
    v[k] = mk<T>((T)(a.re * inv), (T)(a.im * inv));
}
void lz_first_vector(bool fp32, const LzState* st, const void* r, void* v, int64_t n, const Launch& L) {
    const dim3 grid((unsigned)((n + 255) / 256), 1, L.nz);
    if (fp32)
        hipLaunchKernelGGL(scale_from_kernel<float>, grid, dim3(256), 0, L.s, st, (const cx<float>*)r, (cx<float>*)v, n, L.cs);
    else
        hipLaunchKernelGGL(scale_from_kernel<double>, grid, dim3(256), 0, L.s, st, (const cx<double>*)r, (cx<double>*)v, n, L.cs);
}

// The Lanczos coefficient and the LU row of Eq. (2) in one launch.  alpha_i = v_i^dag M v_i from the stencil's partials, then the LU
// scalars gamma_{i-1} = beta_{i-1}/delta_{i-1}, delta_i = alpha_i - gamma_{i-1} beta_{i-1},
// zeta_i = -gamma_{i-1} zeta_{i-1}: every workgroup sums the partials in the same fixed order and
// so holds the same values; workgroup 0 stores them (and ends the run at step i - 1 when delta_i
// is not positive).  Then f -= alpha_i v_i (with ||f||^2 partials), w_i = (v_i - beta_{i-1} w_{i-1})
// / delta_i and x^1 += zeta_i w_i.
template <typename T>
__global__ void lz_update_kernel(int i, LzState* st, const double* apart, int64_t np, LzArrays a, cx<T>* __restrict__ f,
                                 const cx<T>* __restrict__ v, const cx<T>* __restrict__ wprev, cx<T>* __restrict__ wout,
                                 cx<double>* __restrict__ x1, double* f2part, int64_t n, int64_t cs) {
    __shared__ double lds[SCG_BLOCK / SCG_WAVE];
    __shared__ double sc[4];   // alpha_i, delta_i, zeta_i, 1 if the step goes on
    __shared__ int gate;
    st = zoff(st, cs);
    apart = zoff(apart, cs);
    a = zoff(a, cs);
    f = zoff(f, cs);
    v = zoff(v, cs);
    wprev = zoff(wprev, cs);
    wout = zoff(wout, cs);
    x1 = zoff(x1, cs);
    f2part = zoff(f2part, cs);
    // one read of m for the whole workgroup (workgroup 0 may lower it below, concurrently)
    if (threadIdx.x == 0) gate = i <= st->m;
    __syncthreads();
    if (!gate) return;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    cx<T> vv = mk<T>(0, 0), ff = mk<T>(0, 0), wp = mk<T>(0, 0);
    cx<double> xx = mk<double>(0.0, 0.0);
    if (k < n) {   // this thread's operands are loaded while the scalars are summed
        vv = v[k];
        ff = f[k];
        if (i > 1) wp = wprev[k];
        xx = x1[k];
    }
    const double al = block_sum_array(apart, np, lds);
    if (threadIdx.x == 0) {
        double g, d, z;
        if (i == 1) {
            g = 0.0;
            d = al;
            z = st->beta0;
        } else {
            g = a.beta[i - 1] / a.delta[i - 1];
            d = al - g * a.beta[i - 1];
            z = -g * a.zeta[i - 1];
        }
        const bool ok = d > 0.0 && isfinite(d);   // else definiteness was lost in rounding
        sc[0] = al;
        sc[1] = d;
        sc[2] = z;
        sc[3] = ok ? 1.0 : 0.0;
        if (blockIdx.x == 0) {
            if (ok) {
                a.alpha[i] = al;
                a.delta[i] = d;
                a.gam[i] = g;
                a.zeta[i] = z;
                st->max_abs_alpha = fmax(st->max_abs_alpha, fabs(al));
            } else {   // end before step i changes anything
                st->status = 2;
                st->m = i - 1;
                st->done = 1;
            }
        }
    }
    __syncthreads();
    if (sc[3] == 0.0) return;
    const double d = sc[1], z = sc[2];
    const T alt = (T)sc[0];
    const double bp = i > 1 ? a.beta[i - 1] : 0.0;
    double s = 0.0;
    if (k < n) {
        ff = mk<T>(ff.re - alt * vv.re, ff.im - alt * vv.im);
        f[k] = ff;
        s = (double)ff.re * ff.re + (double)ff.im * ff.im;
        double wr = vv.re, wi = vv.im;
        if (i > 1) {
            wr -= bp * wp.re;
            wi -= bp * wp.im;
        }
        wr /= d;
        wi /= d;
        wout[k] = mk<T>((T)wr, (T)wi);
        x1[k] = mk<double>(xx.re + z * wr, xx.im + z * wi);
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) f2part[blockIdx.x] = s;
}
void lz_update(bool fp32, int i, LzState* st, const double* apart, int64_t np, const LzArrays& a, void* f, const void* v,
               const void* wprev, void* wout, double* x1, double* f2part, int64_t n, const Launch& L) {
    const dim3 grid((unsigned)((n + SCG_BLOCK - 1) / SCG_BLOCK), 1, L.nz);
    if (fp32)
        hipLaunchKernelGGL(lz_update_kernel<float>, grid, dim3(SCG_BLOCK), 0, L.s, i, st, apart, np, a, (cx<float>*)f,
                           (const cx<float>*)v, (const cx<float>*)wprev, (cx<float>*)wout, (cx<double>*)x1, f2part, n, L.cs);
    else
        hipLaunchKernelGGL(lz_update_kernel<double>, grid, dim3(SCG_BLOCK), 0, L.s, i, st, apart, np, a, (cx<double>*)f,
                           (const cx<double>*)v, (const cx<double>*)wprev, (cx<double>*)wout, (cx<double>*)x1, f2part, n,
                           L.cs);
}

// End of a Lanczos step, scalars: beta_i = ||f||, the D-Lanczos residual estimate beta_i |zeta_i/delta_i|, i_conv,
// m = min(ceil(past * i_conv), m_cap), breakdown.
__global__ void lz_beta_kernel(int i, LzState* st, const double* part, int64_t np, LzArrays a, int64_t cs) {
    __shared__ double lds[SCG_BLOCK / SCG_WAVE];
    st = zoff(st, cs);
    part = zoff(part, cs);
    a = zoff(a, cs);
    if (i > st->m) return;
    const double b = sqrt(block_sum_array(part, np, lds));
    if (threadIdx.x != 0) return;
    a.beta[i] = b;
    const double e = b * fabs(a.zeta[i] / a.delta[i]);
    a.est[i] = e / st->bnorm1;
    if (st->i_conv == 0 && e <= st->tol * st->bnorm1) {
        st->i_conv = i;
        if (st->past > 0.0) {
            const int mm = (int)ceil(st->past * (double)i);
            st->m = mm < st->m_cap ? mm : st->m_cap;
        }
    }
    if (b <= 1e-14 * st->max_abs_alpha) {
        st->status = 1;
        st->m = i;
    }
    if (i >= st->m) {
        st->m = i;
        st->done = 1;
        if (st->status == 0 && st->i_conv == 0 && st->past > 0.0) st->status = 3;
    }
}
void lz_beta(int i, LzState* st, const double* part, int64_t np, const LzArrays& a, const Launch& L) {
    hipLaunchKernelGGL(lz_beta_kernel, dim3(1, 1, L.nz), dim3(SCG_BLOCK), 0, L.s, i, st, part, np, a, L.cs);
}

// End of a Lanczos step, vector: v_{i+1} = f / beta_i (only when another step follows).
template <typename T>
__global__ void lz_next_kernel(int i, const LzState* st, const double* beta, const cx<T>* __restrict__ f,
                               cx<T>* __restrict__ vn, int64_t n, int64_t cs) {
    st = zoff(st, cs);
    beta = zoff(beta, cs);
    f = zoff(f, cs);
    vn = zoff(vn, cs);
    if (i >= st->m) return;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double inv = 1.0 / beta[i];
    const cx<T> a = f[k];
    vn[k] = mk<T>((T)(a.re * inv), (T)(a.im * inv));
}
void lz_next(bool fp32, int i, const LzState* st, const double* beta, const void* f, void* vn, int64_t n, const Launch& L) {
    const dim3 grid((unsigned)((n + 255) / 256), 1, L.nz);
    if (fp32)
        hipLaunchKernelGGL(lz_next_kernel<float>, grid, dim3(256), 0, L.s, i, st, beta, (const cx<float>*)f, (cx<float>*)vn, n, L.cs);
    else
        hipLaunchKernelGGL(lz_next_kernel<double>, grid, dim3(256), 0, L.s, i, st, beta, (const cx<double>*)f, (cx<double>*)vn, n, L.cs);
}

// ---------------------------------------------------------------------------------------------
// The seeding recurrence of Eq. (1), blocked: eta^j_i = (V^dag r_0^j)_i - gamma_{i-1} eta^j_{i-1} over the rows of a block,
// then X^j += sum_i eta^j_i w_i.  Rows beyond m (the run ended inside the block) get eta = 0.
// ---------------------------------------------------------------------------------------------
__global__ void seed_eta_kernel(int i0, int nb, int nr, const LzState* st, const double* gam, const cx<double>* P,
                                cx<double>* E, cx<double>* eta_prev, int32_t* nvalid, int64_t cs) {
    st = zoff(st, cs);
    gam = zoff(gam, cs);
    P = zoff(P, cs);
    E = zoff(E, cs);
    eta_prev = zoff(eta_prev, cs);
    nvalid = zoff(nvalid, cs);
    const int j = threadIdx.x;
    const int valid = max(0, min(nb, st->m - i0 + 1));
    if (j == 0) *nvalid = valid;
    if (j >= nr) return;
    cx<double> eta = eta_prev[j];
    for (int r = 0; r < nb; r++) {
        if (r < valid) {
            const double g = gam[i0 + r];
            const cx<double> p = P[r * nr + j];
            eta = mk<double>(p.re - g * eta.re, p.im - g * eta.im);
            E[r * nr + j] = eta;
        } else {
            E[r * nr + j] = mk<double>(0.0, 0.0);
        }
    }
    eta_prev[j] = eta;
}
void seed_eta(int i0, int nb, int nr, const LzState* st, const double* gam, const double* P, double* E, double* eta_prev,
              int32_t* nvalid, const Launch& L) {
    hipLaunchKernelGGL(seed_eta_kernel, dim3(1, 1, L.nz), dim3(64), 0, L.s, i0, nb, nr, st, gam, (const cx<double>*)P, (cx<double>*)E,
                       (cx<double>*)eta_prev, nvalid, L.cs);
}

// X[j] += sum_{r < nrow} W[r] E[r][j]  (flat vectors of n complex; nrow from the device or a constant)
template <typename T, typename TX>
__global__ __launch_bounds__(SCG_BLOCK) void seed_update_kernel(const cx<T>* __restrict__ W, int nw, const cx<double>* __restrict__ E,
                                                                 cx<TX>* __restrict__ X, int nx, int64_t n, const int32_t* nrow_dev,
                                                                 int64_t cs) {
    __shared__ cx<double> e_lds[32 * 48];
    W = zoff(W, cs);
    E = zoff(E, cs);
    X = zoff(X, cs);
    nrow_dev = zoff(nrow_dev, cs);
    const int nrow = nrow_dev ? min(*nrow_dev, nw) : nw;
    if (nrow <= 0) return;
    for (int k = threadIdx.x; k < nrow * nx; k += blockDim.x) e_lds[k] = E[k];
    __syncthreads();
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    cx<T> w[32];
#pragma unroll
    for (int r = 0; r < 32; r++)
        if (r < nrow) w[r] = W[(int64_t)r * n + k];
    for (int j = 0; j < nx; j++) {
        double ar = 0.0, ai = 0.0;
#pragma unroll
        for (int r = 0; r < 32; r++)
            if (r < nrow) {
                const cx<double> e = e_lds[r * nx + j];
                ar += (double)w[r].re * e.re - (double)w[r].im * e.im;
                ai += (double)w[r].re * e.im + (double)w[r].im * e.re;
            }
        cx<TX> x = X[(int64_t)j * n + k];
        X[(int64_t)j * n + k] = mk<TX>((TX)(x.re + ar), (TX)(x.im + ai));
    }
}
void seed_update(bool w32, bool x32, const void* W, int nw, const double* E, void* X, int nx, int64_t n, const int32_t* nrow_dev,
                 const Launch& L) {
    const hipStream_t s = L.s;
    const dim3 grid((unsigned)((n + SCG_BLOCK - 1) / SCG_BLOCK), 1, L.nz);
    if (w32 && x32)
        hipLaunchKernelGGL((seed_update_kernel<float, float>), grid, dim3(SCG_BLOCK), 0, s, (const cx<float>*)W, nw,
                           (const cx<double>*)E, (cx<float>*)X, nx, n, nrow_dev, L.cs);
    else if (w32)
        hipLaunchKernelGGL((seed_update_kernel<float, double>), grid, dim3(SCG_BLOCK), 0, s, (const cx<float>*)W, nw,
                           (const cx<double>*)E, (cx<double>*)X, nx, n, nrow_dev, L.cs);
    else
        hipLaunchKernelGGL((seed_update_kernel<double, double>), grid, dim3(SCG_BLOCK), 0, s, (const cx<double>*)W, nw,
                           (const cx<double>*)E, (cx<double>*)X, nx, n, nrow_dev, L.cs);
}

// ---------------------------------------------------------------------------------------------
// Periodic reorthogonalisation of the pair [v_i, f] by classical Gram-Schmidt (Algorithm 1).
// G = V_{1..i}^dag [v_i, f] comes from the projection kernel.  Pass 1 always runs; pass 2
// (the DGKS repeat) runs only for a vector whose norm fell below 1/sqrt(2) of its norm
// before pass 1.
// ---------------------------------------------------------------------------------------------
__device__ inline bool reorth_gate(int i, int pass, const LzState* st, bool& use_v, bool& use_f) {
    if (i > st->m) return false;
    use_v = pass == 1 || st->rep_v;
    use_f = pass == 1 || st->rep_f;
    return use_v || use_f;
}

// v' = v - V_{1..i-1} c, f' = f - V_{1..i-1} d with c = G[:,0], d = G[:,1]; partials |v'|^2, v'^dag f'.
// TV: the stored basis (FP32 or FP64); T: v and f (FP32 only with an FP32 basis).
template <typename TV, typename T>
__global__ __launch_bounds__(SCG_BLOCK) void reorth_update_kernel(int i, int pass, const LzState* st, const cx<TV>* __restrict__ V,
                                                                   int64_t n, const cx<double>* __restrict__ G,
                                                                   cx<T>* __restrict__ v, cx<T>* __restrict__ f,
                                                                   double* part, int64_t cs) {
    __shared__ cx<double> cd[2 * 1024];
    __shared__ double lds[SCG_BLOCK / SCG_WAVE];
    st = zoff(st, cs);
    V = zoff(V, cs);
    G = zoff(G, cs);
    v = zoff(v, cs);
    f = zoff(f, cs);
    part = zoff(part, cs);
    bool use_v, use_f;
    if (!reorth_gate(i, pass, st, use_v, use_f)) return;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = k < n;
    double vr = 0, vi = 0, fr = 0, fi = 0;
    if (act) {
        const cx<T> a = v[k], b = f[k];
        vr = a.re; vi = a.im; fr = b.re; fi = b.im;
    }
    const int nrows = i - 1;
    for (int r0 = 0; r0 < nrows; r0 += 1024) {
        const int nr = min(1024, nrows - r0);
        __syncthreads();
        for (int q = threadIdx.x; q < nr; q += blockDim.x) {
            cd[2 * q] = use_v ? G[2 * (r0 + q)] : mk<double>(0.0, 0.0);
            cd[2 * q + 1] = use_f ? G[2 * (r0 + q) + 1] : mk<double>(0.0, 0.0);
        }
        __syncthreads();
        if (act) {
            const cx<TV>* Vp = V + (int64_t)r0 * n + k;
#pragma unroll 8
            for (int q = 0; q < nr; q++) {
                const cx<TV> b = Vp[(int64_t)q * n];
                const cx<double> c = cd[2 * q], d = cd[2 * q + 1];
                const double br = b.re, bi = b.im;
                vr -= br * c.re - bi * c.im;
                vi -= br * c.im + bi * c.re;
                fr -= br * d.re - bi * d.im;
                fi -= br * d.im + bi * d.re;
            }
        }
    }
    double p0 = 0, p1 = 0, p2 = 0;
    if (act) {
        const cx<T> a = mk<T>((T)vr, (T)vi), b = mk<T>((T)fr, (T)fi);
        if (use_v) v[k] = a;
        if (use_f) f[k] = b;
        // partials of |v'|^2 and v'^dag f' in the stored precision
        p0 = (double)a.re * a.re + (double)a.im * a.im;
        p1 = (double)a.re * b.re + (double)a.im * b.im;
        p2 = (double)a.re * b.im - (double)a.im * b.re;
    }
    p0 = block_sum(p0, lds);
    __syncthreads();
    p1 = block_sum(p1, lds);
    __syncthreads();
    p2 = block_sum(p2, lds);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = p0;
        part[3 * blockIdx.x + 1] = p1;
        part[3 * blockIdx.x + 2] = p2;
    }
}
void reorth_update(bool fp32, int i, int pass, const LzState* st, const void* V, int64_t n, const double* G, void* v, void* f,
                   double* part, const Launch& L, bool v32) {
    const dim3 grid((unsigned)((n + SCG_BLOCK - 1) / SCG_BLOCK), 1, L.nz);
    if (fp32)
        hipLaunchKernelGGL((reorth_update_kernel<float, float>), grid, dim3(SCG_BLOCK), 0, L.s, i, pass, st, (const cx<float>*)V, n,
                           (const cx<double>*)G, (cx<float>*)v, (cx<float>*)f, part, L.cs);
    else if (v32)
        hipLaunchKernelGGL((reorth_update_kernel<float, double>), grid, dim3(SCG_BLOCK), 0, L.s, i, pass, st, (const cx<float>*)V, n,
                           (const cx<double>*)G, (cx<double>*)v, (cx<double>*)f, part, L.cs);
    else
        hipLaunchKernelGGL((reorth_update_kernel<double, double>), grid, dim3(SCG_BLOCK), 0, L.s, i, pass, st, (const cx<double>*)V, n,
                           (const cx<double>*)G, (cx<double>*)v, (cx<double>*)f, part, L.cs);
}

// nv = ||v'||, e = v'^dag f' / ||v'||^2; the DGKS test for v (pass 1).
__global__ void reorth_scalar_kernel(int i, int pass, LzState* st, const double* part, int64_t nb, const cx<double>* G,
                                     int64_t cs) {
    __shared__ double lds[SCG_BLOCK / SCG_WAVE];
    st = zoff(st, cs);
    part = zoff(part, cs);
    G = zoff(G, cs);
    bool use_v, use_f;
    if (!reorth_gate(i, pass, st, use_v, use_f)) return;
    double s[3];
    for (int q = 0; q < 3; q++) {
        double v = 0.0;
        for (int64_t k = threadIdx.x; k < nb; k += blockDim.x) v += part[3 * k + q];
        s[q] = block_sum(v, lds);
        __syncthreads();
    }
    // loss of orthogonality before this step's pass 1: the largest |v_j^dag v_i| / ||v_i||, j < i
    double mx = 0.0;
    if (pass == 1) {
        for (int q = threadIdx.x; q < i - 1; q += blockDim.x) {
            const cx<double> c = G[2 * q];
            mx = fmax(mx, sqrt(c.re * c.re + c.im * c.im));
        }
        for (int off = SCG_WAVE / 2; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
        if (threadIdx.x % SCG_WAVE == 0) lds[threadIdx.x / SCG_WAVE] = mx;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int w = 0; w < (int)(blockDim.x / SCG_WAVE); w++) mx = fmax(mx, lds[w]);
    }
    if (threadIdx.x != 0) return;
    st->nv = sqrt(s[0]);
    st->e = s[1] / s[0];
    st->e_im = s[2] / s[0];
    if (pass == 1) {
        st->v2_before = G[2 * (i - 1)].re;  // v_i^dag v_i before the pass
        if (st->v2_before > 0.0) st->orth_loss = fmax(st->orth_loss, mx / sqrt(st->v2_before));
        st->passes += 2;
    } else {
        st->passes += (st->rep_v ? 1 : 0) + (st->rep_f ? 1 : 0);
    }
}
void reorth_scalar(int i, int pass, LzState* st, const double* part, int64_t nb, const double* G, const Launch& L) {
    hipLaunchKernelGGL(reorth_scalar_kernel, dim3(1, 1, L.nz), dim3(SCG_BLOCK), 0, L.s, i, pass, st, part, nb, (const cx<double>*)G, L.cs);
}

// v_i = v' / nv; f = f' - e v'; partials of |f|^2 (for beta_i).
template <typename T>
__global__ void reorth_finish_kernel(int i, int pass, const LzState* st, cx<T>* __restrict__ v, cx<T>* __restrict__ f,
                                     double* f2part, int64_t n, int64_t cs) {
    __shared__ double lds[SCG_BLOCK / SCG_WAVE];
    st = zoff(st, cs);
    v = zoff(v, cs);
    f = zoff(f, cs);
    f2part = zoff(f2part, cs);
    bool use_v, use_f;
    if (!reorth_gate(i, pass, st, use_v, use_f)) return;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (k < n) {
        const cx<T> a = v[k];
        cx<T> b = f[k];
        if (use_f) {
            const double br = (double)b.re - (st->e * a.re - st->e_im * a.im);
            const double bi = (double)b.im - (st->e * a.im + st->e_im * a.re);
            b = mk<T>((T)br, (T)bi);
            f[k] = b;
        }
        if (use_v) {
            const double inv = 1.0 / st->nv;
            v[k] = mk<T>((T)(a.re * inv), (T)(a.im * inv));
        }
        s = (double)b.re * b.re + (double)b.im * b.im;
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) f2part[blockIdx.x] = s;
}
void reorth_finish(bool fp32, int i, int pass, const LzState* st, void* v, void* f, double* f2part, int64_t n, const Launch& L) {
    const dim3 grid((unsigned)((n + SCG_BLOCK - 1) / SCG_BLOCK), 1, L.nz);
    if (fp32)
        hipLaunchKernelGGL(reorth_finish_kernel<float>, grid, dim3(SCG_BLOCK), 0, L.s, i, pass, st, (cx<float>*)v, (cx<float>*)f,
                           f2part, n, L.cs);
    else
        hipLaunchKernelGGL(reorth_finish_kernel<double>, grid, dim3(SCG_BLOCK), 0, L.s, i, pass, st, (cx<double>*)v,
                           (cx<double>*)f, f2part, n, L.cs);
}

// After a pass: decide the DGKS repeats (pass 1) or clear them (pass 2).
__global__ void reorth_decide_kernel(int i, int pass, LzState* st, const double* f2_before_part, const double* f2_after_part,
                                     int64_t nb, int64_t cs) {
    __shared__ double lds[SCG_BLOCK / SCG_WAVE];
    st = zoff(st, cs);
    f2_before_part = zoff(f2_before_part, cs);
    f2_after_part = zoff(f2_after_part, cs);
    if (i > st->m) return;
    const double fb = block_sum_array(f2_before_part, nb, lds);
    __syncthreads();
    const double fa = block_sum_array(f2_after_part, nb, lds);
    if (threadIdx.x != 0) return;
    if (pass == 1) {
        st->f2_before = fb;
        st->rep_v = (st->nv * st->nv < 0.5 * st->v2_before) ? 1 : 0;
        st->rep_f = (fa < 0.5 * fb) ? 1 : 0;
    } else {
        st->rep_v = 0;
        st->rep_f = 0;
    }
    st->rep_any = st->rep_v | st->rep_f;
}
void reorth_decide(int i, int pass, LzState* st, const double* f2b, const double* f2a, int64_t nb, const Launch& L) {
    hipLaunchKernelGGL(reorth_decide_kernel, dim3(1, 1, L.nz), dim3(SCG_BLOCK), 0, L.s, i, pass, st, f2b, f2a, nb, L.cs);
}

// ---------------------------------------------------------------------------------------------
// Plain CG on a batch of right-hand sides (one CgVec per right-hand side)
// ---------------------------------------------------------------------------------------------
__device__ inline bool cg_skip(const CgVec& c) { return c.done || c.frozen; }

// a_j = rr_j / Re(p_j^dag q_j)   (preconditioned: rz_j = Re r_j^dag z_j in the numerator)
__global__ void cg_alpha_kernel(CgVec* cg, const double* part, int64_t nb, const int32_t* vec_map, int pc, int64_t cs) {
    __shared__ double lds[SCG_BLOCK / SCG_WAVE];
    cg = zoff(cg, cs);
    part = zoff(part, cs);
    vec_map = zoff(vec_map, cs);
    const int vec = vec_map[blockIdx.x];
    if (vec < 0 || cg_skip(cg[vec])) return;
    const double pq = block_sum_array(part + (int64_t)vec * nb, nb, lds);
    if (threadIdx.x == 0) {
        cg[vec].pq = pq;
        cg[vec].a = (pc ? cg[vec].rz : cg[vec].rr) / pq;
    }
}
void cg_alpha(CgVec* cg, const double* part, int64_t nb, const int32_t* vec_map, int nact, const Launch& L, bool pc) {
    hipLaunchKernelGGL(cg_alpha_kernel, dim3(nact, 1, L.nz), dim3(SCG_BLOCK), 0, L.s, cg, part, nb, vec_map, (int)pc, L.cs);
}

// partials of Re a_v^dag b_v for the vectors of vec_map (grid: blocks x nact)
template <typename T>
__global__ void dot_map_kernel(const cx<T>* __restrict__ a, const cx<T>* __restrict__ b, int64_t n, const int32_t* vec_map,
                               const CgVec* cg, double* part, int64_t nb, int64_t cs) {
    __shared__ double lds[SCG_BLOCK / SCG_WAVE];
    a = zoff(a, cs);
    b = zoff(b, cs);
    vec_map = zoff(vec_map, cs);
    cg = zoff(cg, cs);
    part = zoff(part, cs);
    const int vec = vec_map[blockIdx.y];
    if (vec < 0 || (cg && cg_skip(cg[vec]))) return;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (k < n) {
        const cx<T> x = a[(int64_t)vec * n + k], y = b[(int64_t)vec * n + k];
        s = (double)x.re * y.re + (double)x.im * y.im;
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) part[(int64_t)vec * nb + blockIdx.x] = s;
}
void dot_map(bool fp32, const void* a, const void* b, int64_t n, const int32_t* vec_map, int nact, const CgVec* cg, double* part,
             const Launch& L) {
    const int64_t nb = (n + SCG_BLOCK - 1) / SCG_BLOCK;
    const dim3 grid((unsigned)nb, nact, L.nz);
    if (fp32)
        hipLaunchKernelGGL(dot_map_kernel<float>, grid, dim3(SCG_BLOCK), 0, L.s, (const cx<float>*)a, (const cx<float>*)b, n, vec_map, cg,
                           part, nb, L.cs);
    else
        hipLaunchKernelGGL(dot_map_kernel<double>, grid, dim3(SCG_BLOCK), 0, L.s, (const cx<double>*)a, (const cx<double>*)b, n, vec_map,
                           cg, part, nb, L.cs);
}

// preconditioned CG: rr_new = |r|^2 for the stop test, rz_new = Re r^dag z, b = rz_new / rz
__global__ void cg_beta_pc_kernel(CgVec* cg, const double* rrpart, const double* rzpart, int64_t nb, const int32_t* vec_map, int max_iter,
                                  int64_t cs) {
    __shared__ double lds[SCG_BLOCK / SCG_WAVE];
    cg = zoff(cg, cs);
    rrpart = zoff(rrpart, cs);
    rzpart = zoff(rzpart, cs);
    vec_map = zoff(vec_map, cs);
    const int vec = vec_map[blockIdx.x];
    if (vec < 0 || cg_skip(cg[vec])) return;
    const double rr = block_sum_array(rrpart + (int64_t)vec * nb, nb, lds);
    __syncthreads();
    const double rz = block_sum_array(rzpart + (int64_t)vec * nb, nb, lds);
    if (threadIdx.x != 0) return;
    CgVec& c = cg[vec];
    c.iters += 1;
    if (sqrt(rr) <= c.tol * c.bnorm || c.iters >= max_iter || !isfinite(rr) || !(rz > 0.0)) {
        c.frozen = 1;
        c.pq = rr;
        return;
    }
    c.b = rz / c.rz;
    c.rz = rz;
    c.rr_old = c.rr;
    c.rr = rr;
}
void cg_beta_pc(CgVec* cg, const double* rrpart, const double* rzpart, int64_t nb, const int32_t* vec_map, int nact, int max_iter,
                const Launch& L) {
    hipLaunchKernelGGL(cg_beta_pc_kernel, dim3(nact, 1, L.nz), dim3(SCG_BLOCK), 0, L.s, cg, rrpart, rzpart, nb, vec_map, max_iter, L.cs);
}

// x += a p; r -= a q; partials |r|^2
template <typename T, typename TX>
__global__ void cg_update_kernel(const CgVec* cg, const int32_t* vec_map, int nact, cx<TX>* __restrict__ X, const cx<T>* __restrict__ P,
                                 cx<T>* __restrict__ R, const cx<T>* __restrict__ Q, double* part, int64_t n, int64_t nb,
                                 int64_t cs) {
    __shared__ double lds[SCG_BLOCK / SCG_WAVE];
    cg = zoff(cg, cs);
    vec_map = zoff(vec_map, cs);
    X = zoff(X, cs);
    P = zoff(P, cs);
    R = zoff(R, cs);
    Q = zoff(Q, cs);
    part = zoff(part, cs);
    const int slot = blockIdx.y;
    const int vec = vec_map[slot];
    if (vec < 0 || cg_skip(cg[vec])) return;
    const double a = cg[vec].a;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (k < n) {
        const int64_t o = (int64_t)vec * n + k;
        const cx<T> p = P[o], q = Q[o];
        const cx<TX> x = X[o];
        X[o] = mk<TX>((TX)(x.re + a * p.re), (TX)(x.im + a * p.im));
        const cx<T> r = R[o];
        const cx<T> rn = mk<T>((T)(r.re - a * q.re), (T)(r.im - a * q.im));
        R[o] = rn;
        s = (double)rn.re * rn.re + (double)rn.im * rn.im;
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) part[(int64_t)vec * nb + blockIdx.x] = s;
}
void cg_update(bool fp32, bool x32, const CgVec* cg, const int32_t* vec_map, int nact, void* X, const void* P, void* R,
               const void* Q, double* part, int64_t n, const Launch& L) {
    const hipStream_t s = L.s;
    const int64_t nb = (n + SCG_BLOCK - 1) / SCG_BLOCK;
    const dim3 grid((unsigned)nb, nact, L.nz);
    if (fp32 && x32)
        hipLaunchKernelGGL((cg_update_kernel<float, float>), grid, dim3(SCG_BLOCK), 0, s, cg, vec_map, nact, (cx<float>*)X,
                           (const cx<float>*)P, (cx<float>*)R, (const cx<float>*)Q, part, n, nb, L.cs);
    else if (fp32)
        hipLaunchKernelGGL((cg_update_kernel<float, double>), grid, dim3(SCG_BLOCK), 0, s, cg, vec_map, nact, (cx<double>*)X,
                           (const cx<float>*)P, (cx<float>*)R, (const cx<float>*)Q, part, n, nb, L.cs);
    else
        hipLaunchKernelGGL((cg_update_kernel<double, double>), grid, dim3(SCG_BLOCK), 0, s, cg, vec_map, nact, (cx<double>*)X,
                           (const cx<double>*)P, (cx<double>*)R, (const cx<double>*)Q, part, n, nb, L.cs);
}

// rr_new = |r|^2; stop test on the recursive residual (freeze for a true-residual check);
// b = rr_new / rr
__global__ void cg_beta_kernel(CgVec* cg, const double* part, int64_t nb, const int32_t* vec_map, int max_iter, int64_t cs) {
    __shared__ double lds[SCG_BLOCK / SCG_WAVE];
    cg = zoff(cg, cs);
    part = zoff(part, cs);
    vec_map = zoff(vec_map, cs);
    const int vec = vec_map[blockIdx.x];
    if (vec < 0 || cg_skip(cg[vec])) return;
    const double rr = block_sum_array(part + (int64_t)vec * nb, nb, lds);
    if (threadIdx.x != 0) return;
    CgVec& c = cg[vec];
    c.iters += 1;
    if (sqrt(rr) <= c.tol * c.bnorm || c.iters >= max_iter || !isfinite(rr)) {
        c.frozen = 1;  // the host checks the true residual before going on
        c.pq = rr;
        return;
    }
    c.b = rr / c.rr;
    c.rr_old = c.rr;
    c.rr = rr;
}
void cg_beta(CgVec* cg, const double* part, int64_t nb, const int32_t* vec_map, int nact, int max_iter, const Launch& L) {
    hipLaunchKernelGGL(cg_beta_kernel, dim3(nact, 1, L.nz), dim3(SCG_BLOCK), 0, L.s, cg, part, nb, vec_map, max_iter, L.cs);
}

// p = r + b p
template <typename T>
__global__ void cg_p_kernel(const CgVec* cg, const int32_t* vec_map, cx<T>* __restrict__ P, const cx<T>* __restrict__ R, int64_t n,
                            int ignore_frozen, int64_t cs) {
    cg = zoff(cg, cs);
    vec_map = zoff(vec_map, cs);
    P = zoff(P, cs);
    R = zoff(R, cs);
    const int vec = vec_map[blockIdx.y];
    if (vec < 0 || cg[vec].done || (cg[vec].frozen && !ignore_frozen)) return;
    const double b = cg[vec].b;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t o = (int64_t)vec * n + k;
    const cx<T> p = P[o], r = R[o];
    P[o] = mk<T>((T)(r.re + b * p.re), (T)(r.im + b * p.im));
}
void cg_p(bool fp32, const CgVec* cg, const int32_t* vec_map, int nact, void* P, const void* R, int64_t n, bool ignore_frozen,
          const Launch& L) {
    const dim3 grid((unsigned)((n + 255) / 256), nact, L.nz);
    if (fp32)
        hipLaunchKernelGGL(cg_p_kernel<float>, grid, dim3(256), 0, L.s, cg, vec_map, (cx<float>*)P, (const cx<float>*)R, n,
                           (int)ignore_frozen, L.cs);
    else
        hipLaunchKernelGGL(cg_p_kernel<double>, grid, dim3(256), 0, L.s, cg, vec_map, (cx<double>*)P, (const cx<double>*)R, n,
                           (int)ignore_frozen, L.cs);
}

// Deflated CG (coefficients of the deflation space in a direction or an iterate): one workgroup.
__global__ void defl_mu_kernel(const cx<double>* Ginv, const cx<double>* P, int nev, int ncol, const int32_t* map, int w,
                               const CgVec* cg, double sign, cx<double>* E, int64_t cs) {
    __shared__ int sel[32];
    P = zoff(P, cs);
    E = zoff(E, cs);
    Ginv = zoff(Ginv, cs);
    map = zoff(map, cs);
    cg = zoff(cg, cs);
    if (threadIdx.x < 32) sel[threadIdx.x] = 0;
    __syncthreads();
    if ((int)threadIdx.x < w) {
        const int j = map ? map[threadIdx.x] : (int)threadIdx.x;
        if (j >= 0 && j < ncol && !(cg && (cg[j].done || cg[j].frozen))) sel[j] = 1;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nev * ncol; q += blockDim.x) {
        const int k = q / ncol, j = q % ncol;
        double sr = 0.0, si = 0.0;
        if (sel[j])
            for (int l = 0; l < nev; l++) {
                const cx<double> g = Ginv[k * nev + l], pv = P[l * ncol + j];
                sr += g.re * pv.re - g.im * pv.im;
                si += g.re * pv.im + g.im * pv.re;
            }
        E[q] = mk<double>(sign * sr, sign * si);
    }
}
void defl_mu(const double* Ginv, const double* P, int nev, int ncol, const int32_t* map, int w, const CgVec* cg, double sign,
             double* E, const Launch& L) {
    hipLaunchKernelGGL(defl_mu_kernel, dim3(1, 1, L.nz), dim3(256), 0, L.s, (const cx<double>*)Ginv, (const cx<double>*)P, nev, ncol,
                       map, w, cg, sign, (cx<double>*)E, L.cs);
}

// gamma5 = diag(1, 1, -1, -1): components 6..11 (spins 2, 3) change sign
template <typename T>
__global__ void gamma5_copy_kernel(const cx<T>* a, cx<T>* b, int64_t Vh, int64_t total, int64_t cs) {
    a = zoff(a, cs);
    b = zoff(b, cs);
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= total) return;
    const int64_t c = (k / Vh) % 12;
    const cx<T> v = a[k];
    b[k] = c >= 6 ? mk<T>(-v.re, -v.im) : v;
}
void gamma5_copy(bool fp32, const void* a, void* b, int64_t Vh, int nvec, const Launch& L) {
    const int64_t total = 12 * Vh * nvec;
    const dim3 grid((unsigned)((total + 255) / 256), 1, L.nz);
    if (fp32)
        hipLaunchKernelGGL(gamma5_copy_kernel<float>, grid, dim3(256), 0, L.s, (const cx<float>*)a, (cx<float>*)b, Vh, total, L.cs);
    else
        hipLaunchKernelGGL(gamma5_copy_kernel<double>, grid, dim3(256), 0, L.s, (const cx<double>*)a, (cx<double>*)b, Vh, total, L.cs);
}

}  // namespace scg
