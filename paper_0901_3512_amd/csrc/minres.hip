// Generic FP64 vector kernels of the indefinite (gamma5 A) solver: linear combinations of up to four
// vectors into up to ZLC_MAX outputs per launch, and batched complex dot products.
#include "kernels.h"

#include <algorithm>

namespace scg {

constexpr int ZLC_MAX = 16;
struct ZLCs {
    ZLC o[ZLC_MAX];
};

// out = [out +] sum_t a_t in_t, element by element (an output may be one of its own inputs; no
// output may be an input of another output of the same launch)
__global__ __launch_bounds__(SCG_BLOCK) void zlincomb_kernel(ZLCs d, int64_t n) {
    const ZLC& c = d.o[blockIdx.y];
    const int64_t k = (int64_t)blockIdx.x * SCG_BLOCK + threadIdx.x;
    if (k >= n) return;
    cx<double>* out = (cx<double>*)c.out;
    double re = 0.0, im = 0.0;
    if (c.acc) {
        const cx<double> o = out[k];
        re = o.re;
        im = o.im;
    }
    for (int t = 0; t < c.nt; t++) {
        const cx<double> x = ((const cx<double>*)c.in[t])[k];
        re = fma(c.are[t], x.re, fma(-c.aim[t], x.im, re));
        im = fma(c.are[t], x.im, fma(c.aim[t], x.re, im));
    }
    out[k] = mk<double>(re, im);
}

void zlincomb(const ZLC* o, int nout, int64_t n, hipStream_t s) {
    const int64_t nb = (n + SCG_BLOCK - 1) / SCG_BLOCK;
    for (int b = 0; b < nout; b += ZLC_MAX) {
        ZLCs d{};
        const int cnt = std::min(ZLC_MAX, nout - b);
        for (int j = 0; j < cnt; j++) d.o[j] = o[b + j];
        hipLaunchKernelGGL(zlincomb_kernel, dim3((unsigned)nb, (unsigned)cnt), dim3(SCG_BLOCK), 0, s, d, n);
    }
}

constexpr int ZDOT_MAX = 32;
struct ZDotArgs {
    const void* a[ZDOT_MAX];
    const void* b[ZDOT_MAX];
};

// part[(2 p + 0) nb + block] = Re sum conj(a_p) b_p over the block's elements, (2 p + 1): Im
__global__ __launch_bounds__(SCG_BLOCK) void zdots_kernel(ZDotArgs d, int64_t n, double* part, int64_t nb) {
    __shared__ double lds[SCG_BLOCK / SCG_WAVE];
    const int p = blockIdx.y;
    const int64_t k = (int64_t)blockIdx.x * SCG_BLOCK + threadIdx.x;
    double re = 0.0, im = 0.0;
    if (k < n) {
        const cx<double> x = ((const cx<double>*)d.a[p])[k];
        const cx<double> y = ((const cx<double>*)d.b[p])[k];
        re = x.re * y.re + x.im * y.im;
        im = x.re * y.im - x.im * y.re;
    }
    const double sr = block_sum(re, lds);
    __syncthreads();
    const double si = block_sum(im, lds);
    if (threadIdx.x == 0) {
        part[(2 * (int64_t)p) * nb + blockIdx.x] = sr;
        part[(2 * (int64_t)p + 1) * nb + blockIdx.x] = si;
    }
}

int64_t zdots_blocks(int64_t n) { return (n + SCG_BLOCK - 1) / SCG_BLOCK; }

void zdots(const void* const* a, const void* const* b, int np, int64_t n, double* part, double* out, hipStream_t s) {
    const int64_t nb = zdots_blocks(n);
    for (int q = 0; q < np; q += ZDOT_MAX) {
        ZDotArgs d{};
        const int cnt = std::min(ZDOT_MAX, np - q);
        for (int j = 0; j < cnt; j++) {
            d.a[j] = a[q + j];
            d.b[j] = b[q + j];
        }
        hipLaunchKernelGGL(zdots_kernel, dim3((unsigned)nb, (unsigned)cnt), dim3(SCG_BLOCK), 0, s, d, n, part, nb);
        sum_partials(part, nb, 2 * cnt, out + 2 * q, false, Launch(s));
    }
}

}  // namespace scg
