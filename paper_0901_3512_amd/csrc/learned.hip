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
#include "kernels.h"

namespace scg {

__device__ inline int adj_dir(int d) { return d == 0 ? 0 : (d <= 4 ? d + 4 : d - 4); }

struct Site {
    int x, y, z, t, xh;
    int64_t row;
};
__device__ inline Site site_of(const Geom& g, int p, int64_t h) {
    Site s;
    s.xh = (int)(h % g.Lxh);
    int64_t r = h / g.Lxh;
    s.y = (int)(r % g.L[1]);
    r /= g.L[1];
    s.z = (int)(r % g.L[2]);
    s.t = (int)(r / g.L[2]);
    s.x = 2 * s.xh + ((s.y + s.z + s.t + p) & 1);
    s.row = h - s.xh;
    return s;
}
// checkerboard index of the neighbour in direction mu, step +-1, and the boundary sign
__device__ inline int64_t nb_index(const Geom& g, const Site& s, int mu, int step, float& sign) {
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
    sign = 1.f;
    if (mu == 0) return s.row + (((s.x + step + Lx) % Lx) >> 1);
    if (mu == 1) return s.xh + (int64_t)g.Lxh * (((s.y + step + Ly) % Ly) + (int64_t)Ly * (s.z + (int64_t)Lz * s.t));
    if (mu == 2) return s.xh + (int64_t)g.Lxh * (s.y + (int64_t)Ly * (((s.z + step + Lz) % Lz) + (int64_t)Lz * s.t));
    if ((step == 1 && s.t == Lt - 1) || (step == -1 && s.t == 0)) sign = (float)g.t_bc;
    return s.xh + (int64_t)g.Lxh * (s.y + (int64_t)Ly * (s.z + (int64_t)Lz * ((s.t + step + Lt) % Lt)));
}

// (T_d in)(p, h) for one site: 4 spins x 3 colours
__device__ inline void transport(const Geom& g, const cx<float>* __restrict__ links, const cx<float>* __restrict__ in,
                                 int p, int64_t h, const Site& s, int d, cx<float> t[12]) {
    const int64_t Vh = g.Vh;
    if (d == 0) {
        const cx<float>* src = in + (int64_t)p * 12 * Vh;
#pragma unroll
        for (int c = 0; c < 12; c++) t[c] = src[(int64_t)c * Vh + h];
        return;
    }
    const int mu = (d - 1) & 3;
    const bool fwd = d <= 4;
    float sign;
    const int64_t hn = nb_index(g, s, mu, fwd ? 1 : -1, sign);
    const cx<float>* src = in + (int64_t)(1 - p) * 12 * Vh;
    const int lp = fwd ? p : 1 - p;
    const int64_t lh = fwd ? h : hn;
    const cx<float>* lk = links + ((int64_t)(mu * 2 + lp) * 9) * Vh + lh;
    cx<float> u[9];
#pragma unroll
    for (int c = 0; c < 9; c++) u[c] = lk[(int64_t)c * Vh];
#pragma unroll
    for (int sp = 0; sp < 4; sp++) {
        cx<float> v[3];
#pragma unroll
        for (int b = 0; b < 3; b++) v[b] = src[(int64_t)(3 * sp + b) * Vh + hn];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            cx<float> acc = mk<float>(0.f, 0.f);
#pragma unroll
            for (int b = 0; b < 3; b++) acc = acc + (fwd ? cmul(u[a * 3 + b], v[b]) : cjmul(u[b * 3 + a], v[b]));
            t[3 * sp + a] = sign * acc;
        }
    }
}

// out = L in (dagger = 0) or L^dag in (dagger = 1), for the vectors listed in vmap (or 0..nvec-1)
__global__ __launch_bounds__(256) void k_layer_kernel(Geom g, const cx<float>* __restrict__ links, const cx<float>* __restrict__ in,
                                                      cx<float>* __restrict__ out, const cx<float>* __restrict__ W, int dagger,
                                                      const int32_t* vmap, int zero_odd_input) {
    __shared__ cx<float> w[9 * 16];
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
    const int vec = vmap ? vmap[blockIdx.y] : (int)blockIdx.y;
    const int64_t Vh = g.Vh;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 2 * Vh) return;
    const int p = (int)(k / Vh);
    const int64_t h = k % Vh;
    const cx<float>* src = in + (int64_t)vec * 24 * Vh;
    cx<float>* dst = out + (int64_t)vec * 24 * Vh;
    const Site s = site_of(g, p, h);
    cx<float> acc[12];
#pragma unroll
    for (int c = 0; c < 12; c++) acc[c] = mk<float>(0.f, 0.f);
    for (int d = 0; d < 9; d++) {
        // with an even-only input (E_e x) the odd-site terms vanish: skip them
        if (zero_odd_input && ((d == 0) ? (p == 1) : (p == 0))) continue;
        cx<float> t[12];
        transport(g, links, src, p, h, s, d, t);
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 4; b++) {
                const cx<float> wab = w[d * 16 + a * 4 + b];
#pragma unroll
                for (int c = 0; c < 3; c++) acc[3 * a + c] = acc[3 * a + c] + cmul(wab, t[3 * b + c]);
            }
    }
#pragma unroll
    for (int c = 0; c < 12; c++) dst[(int64_t)p * 12 * Vh + (int64_t)c * Vh + h] = acc[c];
}

void k_layer(const Geom& g, const void* links32, const void* in, void* out, const void* W, bool dagger, const int32_t* vmap,
             int nvec, bool zero_odd_input, hipStream_t s) {
    const dim3 grid((unsigned)((2 * g.Vh + 255) / 256), (unsigned)nvec);
    hipLaunchKernelGGL(k_layer_kernel, grid, dim3(256), 0, s, g, (const cx<float>*)links32, (const cx<float>*)in, (cx<float>*)out,
                       (const cx<float>*)W, (int)dagger, vmap, (int)zero_odd_input);
}

// partial sums over sites, colours and vectors of g[a][c] conj((T_dt in)[b][c]) for direction
// d = blockIdx.y, with dt = d (layer L) or dt = -d (layer L^dag).  part[d][block][16] complex.
__global__ __launch_bounds__(256) void k_grad_kernel(Geom g, const cx<float>* __restrict__ links, const cx<float>* __restrict__ gv,
                                                     const cx<float>* __restrict__ in, int dagger, int nvec, double* part) {
    __shared__ double lds[4 * 32];
    const int d = blockIdx.y;
    const int dt = dagger ? adj_dir(d) : d;
    const int64_t Vh = g.Vh;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[32];
#pragma unroll
    for (int e = 0; e < 32; e++) acc[e] = 0.0;
    if (k < 2 * Vh) {
        const int p = (int)(k / Vh);
        const int64_t h = k % Vh;
        const Site s = site_of(g, p, h);
        for (int v = 0; v < nvec; v++) {
            cx<float> t[12], q[12];
            transport(g, links, in + (int64_t)v * 24 * Vh, p, h, s, dt, t);
            const cx<float>* gs = gv + (int64_t)v * 24 * Vh + (int64_t)p * 12 * Vh;
#pragma unroll
            for (int c = 0; c < 12; c++) q[c] = gs[(int64_t)c * Vh + h];
#pragma unroll
            for (int a = 0; a < 4; a++)
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    float re = 0.f, im = 0.f;
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        const cx<float> pr = cjmul(t[3 * b + c], q[3 * a + c]);  // q conj(t)
                        re += pr.re;
                        im += pr.im;
                    }
                    acc[2 * (a * 4 + b)] += re;
                    acc[2 * (a * 4 + b) + 1] += im;
                }
        }
    }
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
    for (int e = 0; e < 32; e++) {
        double v = acc[e];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) lds[wave * 32 + e] = v;
    }
    __syncthreads();
    if (threadIdx.x < 32) {
        const double v = lds[threadIdx.x] + lds[32 + threadIdx.x] + lds[64 + threadIdx.x] + lds[96 + threadIdx.x];
        part[((int64_t)d * gridDim.x + blockIdx.x) * 32 + threadIdx.x] = v;
    }
}

// Gtot[d] += sum over blocks (dagger layers add the conjugate transpose: dL/dconj(w) = G'^dag).
// One workgroup per direction: thread (j, e) adds blocks j, j+8, ... of value e, then the eight
// partial sums are added in order (deterministic).
__global__ void k_grad_reduce_kernel(const double* part, int64_t nblocks, int dagger, double* Gtot) {
    __shared__ double lds[8 * 32];
    const int d = blockIdx.x;
    const int e = threadIdx.x % 32, j = threadIdx.x / 32;
    double s = 0.0;
    for (int64_t b = j; b < nblocks; b += 8) s += part[((int64_t)d * nblocks + b) * 32 + e];
    lds[j * 32 + e] = s;
    __syncthreads();
    if (j != 0) return;
    s = 0.0;
    for (int q = 0; q < 8; q++) s += lds[q * 32 + e];
    const int ab = e / 2, comp = e % 2;
    if (!dagger) {
        Gtot[d * 32 + e] += s;
    } else {
        const int a = ab / 4, b = ab % 4;
        Gtot[d * 32 + 2 * (b * 4 + a) + comp] += comp ? -s : s;
    }
}

int64_t k_grad_blocks(const Geom& g) { return (2 * g.Vh + 255) / 256; }

void k_grad(const Geom& g, const void* links32, const void* gv, const void* in, bool dagger, int nvec, double* part, double* Gtot,
            hipStream_t s) {
    const int64_t nb = k_grad_blocks(g);
    hipLaunchKernelGGL(k_grad_kernel, dim3((unsigned)nb, 9), dim3(256), 0, s, g, (const cx<float>*)links32, (const cx<float>*)gv,
                       (const cx<float>*)in, (int)dagger, nvec, part);
    hipLaunchKernelGGL(k_grad_reduce_kernel, dim3(9), dim3(256), 0, s, part, nb, (int)dagger, Gtot);
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

// training residual: e = z - u on the even sites; loss partials |e|^2 / |u|^2; gradient field
// g = E_e e / (S |u|^2)
__global__ void k_residual_kernel(const cx<float>* __restrict__ zfull, const cx<float>* __restrict__ u, const double* unorm2,
                                  cx<float>* __restrict__ gfull, int64_t n, int S, double* part) {
    __shared__ double lds[4];
    const int v = blockIdx.y;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e2 = 0.0;
    if (k < 2 * n) {
        cx<float> gval = mk<float>(0.f, 0.f);
        if (k < n) {
            const cx<float> z = zfull[(int64_t)v * 2 * n + k], uu = u[(int64_t)v * n + k];
            const double er = (double)z.re - uu.re, ei = (double)z.im - uu.im;
            e2 = er * er + ei * ei;
            const double sc = 1.0 / ((double)S * unorm2[v]);
            gval = mk<float>((float)(er * sc), (float)(ei * sc));
        }
        gfull[(int64_t)v * 2 * n + k] = gval;
    }
    const double s = block_sum(e2, lds);
    if (threadIdx.x == 0) part[(int64_t)v * gridDim.x + blockIdx.x] = s / unorm2[v];
}
void k_residual(const void* zfull, const void* u, const double* unorm2, void* gfull, int64_t n, int S, double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_residual_kernel, dim3((unsigned)((2 * n + 255) / 256), (unsigned)S), dim3(256), 0, s, (const cx<float>*)zfull,
                       (const cx<float>*)u, unorm2, (cx<float>*)gfull, n, S, part);
}
int64_t k_residual_blocks(int64_t n) { return (2 * n + 255) / 256; }

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
