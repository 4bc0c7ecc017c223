// Dense contraction P = V^dag R on the matrix cores (Algorithm 1 steps 4, 7 and 8).
//
// V is nv vectors, R nr vectors, each n complex numbers stored as interleaved (re, im).
// The complex product is a real GEMM over K = 2n reals:
//     Re P[r][j] = sum_k V[r][k] R[j][k]
//     Im P[r][j] = sum_k V[r][k] R~[j][k],   R~[j][2t] = Im R[j][t],  R~[j][2t+1] = -Re R[j][t]
// so the B operand has 2*nr real columns (Re and Im of every j) and A is V read as stored.
//
// Split-K: a workgroup owns a K-chunk and up to 32 rows of V (two 16-row MFMA tiles) and
// computes all 2*nr columns (up to three 16-column tiles) of its partial product, staging
// 32 complex per row through LDS per step.  Partials go to part[chunk][row][j] and a second
// kernel sums the chunks in a fixed order (deterministic).  FP64 inputs use
// v_mfma_f64_16x16x4; FP32 inputs use v_mfma_f32_16x16x4 with FP32 accumulation.
//
// MFMA operand layout (16x16x4, one block): lane l holds A[l%16][l/16] and B[l/16][l%16];
// the 16x16 result is 4 values per lane in column l%16: rows l/16 + 4q for the FP64
// instruction and rows 4*(l/16) + q for the FP32 one (q = 0..3; checked on gfx950).
#include "kernels.h"

namespace scg {

constexpr int PJ_ROWS = 32;     // rows of V per workgroup
constexpr int PJ_KC = 32;       // complex per LDS step
constexpr int PJ_KR = 2 * PJ_KC; // reals per LDS step
constexpr int PJ_LD = PJ_KR + 1; // padded LDS row (doubles or floats)
constexpr int PJ_MAXR = 24;     // max right-hand sides

template <typename T>
struct MfmaAcc;
template <>
struct MfmaAcc<double> {
    using V4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    __device__ static inline V4 step(double a, double b, V4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static inline int row(int lane, int q) { return (lane >> 4) + 4 * q; }
};
template <>
struct MfmaAcc<float> {
    using V4 = __attribute__((__vector_size__(4 * sizeof(float)))) float;
    __device__ static inline V4 step(float a, float b, V4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static inline int row(int lane, int q) { return 4 * (lane >> 4) + q; }
};

// TS: storage type of V and R; T: compute type (FP32 storage may be contracted in FP64)
template <typename TS, typename T>
__global__ __launch_bounds__(256) void proj_kernel(ProjArgs pa, int64_t cs) {
    using Acc = MfmaAcc<T>;
    using V4 = typename Acc::V4;
    __shared__ T As[PJ_ROWS * PJ_LD];
    __shared__ T Bs[PJ_MAXR * PJ_LD];

    if (cs) {
        pa.V = zoff(pa.V, cs);
        for (int j = 0; j < pa.nr; j++) pa.R[j] = zoff(pa.R[j], cs);
        pa.part = zoff(pa.part, cs);
        pa.st = zoff(pa.st, cs);
        pa.flag = zoff(pa.flag, cs);
    }
    if (pa.st && pa.gate_i > pa.st->m) return;
    if (pa.flag && *pa.flag == 0) return;
    int nvalid = pa.nv;
    if (pa.st && pa.rows_from_m) nvalid = max(0, min(pa.nv, pa.st->m - pa.i0 + 1));
    const int row0 = blockIdx.y * PJ_ROWS;
    const int nrow = min(PJ_ROWS, nvalid - row0);
    if (nrow <= 0) return;

    const TS* V = (const TS*)pa.V;
    const int nr = pa.nr;
    const int ncol = 2 * nr;
    const int ncolt = (ncol + 15) / 16;
    const int nrowt = (nrow + 15) / 16;
    const int ntiles = nrowt * ncolt;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    const int64_t k_begin = (int64_t)blockIdx.x * pa.kchunk;           // complex index
    const int64_t k_end = min(pa.n, k_begin + pa.kchunk);

    V4 acc0, acc1;
    for (int q = 0; q < 4; q++) {
        acc0[q] = 0;
        acc1[q] = 0;
    }

    for (int64_t kb = k_begin; kb < k_end; kb += PJ_KC) {
        const int kc = (int)min((int64_t)PJ_KC, k_end - kb);
        __syncthreads();
        // stage V rows and R vectors: one complex (two reals) per thread per pass
        for (int idx = threadIdx.x; idx < PJ_ROWS * PJ_KC; idx += 256) {
            const int r = idx / PJ_KC, c = idx % PJ_KC;
            T re = 0, im = 0;
            if (r < nrow && c < kc) {
                const TS* p = V + 2 * ((int64_t)(row0 + r) * pa.ldv + kb + c);
                re = (T)p[0];
                im = (T)p[1];
            }
            As[r * PJ_LD + 2 * c] = re;
            As[r * PJ_LD + 2 * c + 1] = im;
        }
        for (int idx = threadIdx.x; idx < nr * PJ_KC; idx += 256) {
            const int j = idx / PJ_KC, c = idx % PJ_KC;
            T re = 0, im = 0;
            if (c < kc) {
                const TS* p = (const TS*)pa.R[j] + 2 * (kb + c);
                re = (T)p[0];
                im = (T)p[1];
            }
            Bs[j * PJ_LD + 2 * c] = re;
            Bs[j * PJ_LD + 2 * c + 1] = im;
        }
        __syncthreads();
        // this wave's output tiles: wave, wave + 4 (at most 6 tiles)
        for (int tsel = 0; tsel < 2; tsel++) {
            const int tile = wave + 4 * tsel;
            if (tile >= ntiles) break;
            const int rt = tile / ncolt, ct = tile % ncolt;
            const int ar = rt * 16 + (lane & 15);
            const int col = ct * 16 + (lane & 15);
            const int j = col >> 1, part = col & 1;
            const bool colok = col < ncol;
            V4 acc = tsel == 0 ? acc0 : acc1;
#pragma unroll 4
            for (int kk = 0; kk < PJ_KR; kk += 4) {
                const int k = kk + (lane >> 4);
                const T a = As[ar * PJ_LD + k];
                T b = 0;
                if (colok) {
                    if (part == 0)
                        b = Bs[j * PJ_LD + k];
                    else
                        b = (k & 1) ? -Bs[j * PJ_LD + k - 1] : Bs[j * PJ_LD + k + 1];
                }
                acc = Acc::step(a, b, acc);
            }
            if (tsel == 0)
                acc0 = acc;
            else
                acc1 = acc;
        }
    }

    // write the partial tiles: part[chunk][row][j] complex (FP64)
    double* out = pa.part + (int64_t)blockIdx.x * pa.part_stride;
    for (int tsel = 0; tsel < 2; tsel++) {
        const int tile = wave + 4 * tsel;
        if (tile >= ntiles) break;
        const int rt = tile / ncolt, ct = tile % ncolt;
        const V4 acc = tsel == 0 ? acc0 : acc1;
        const int col = ct * 16 + (lane & 15);
        if (col >= ncol) continue;
        const int j = col >> 1, part = col & 1;
        for (int q = 0; q < 4; q++) {
            const int r = rt * 16 + Acc::row(lane, q);
            if (r < nrow) out[2 * ((int64_t)(row0 + r) * nr + j) + part] = (double)acc[q];
        }
    }
}

// P[r][j] = sum over chunks of part[chunk][r][j]; one wavefront per output value, lane c adds
// chunks c, c+64, ... and the lanes are combined by a fixed shuffle tree (deterministic).
__global__ void proj_reduce_kernel(const double* part, int64_t nchunks, int64_t stride, int64_t len, double* P,
                                   const LzState* st, int gate_i, const int32_t* flag, int64_t cs) {
    part = zoff(part, cs);
    P = zoff(P, cs);
    st = zoff(st, cs);
    flag = zoff(flag, cs);
    if (st && gate_i > st->m) return;
    if (flag && *flag == 0) return;
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / SCG_WAVE;
    const int lane = threadIdx.x % SCG_WAVE;
    if (k >= len) return;  // uniform per wavefront
    double s = 0.0;
    for (int64_t c = lane; c < nchunks; c += SCG_WAVE) s += part[c * stride + k];
    for (int off = SCG_WAVE / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) P[k] = s;
}

int64_t proj_chunks(int64_t n, int64_t kchunk) { return (n + kchunk - 1) / kchunk; }

void project(bool fp32, const ProjArgs& a, int64_t nrowblocks, double* P, const Launch& L, bool fp64_math) {
    const hipStream_t s = L.s;
    const int64_t nch = proj_chunks(a.n, a.kchunk);
    const dim3 grid((unsigned)nch, (unsigned)nrowblocks, L.nz);
    if (fp32 && fp64_math)
        hipLaunchKernelGGL((proj_kernel<float, double>), grid, dim3(256), 0, s, a, L.cs);
    else if (fp32)
        hipLaunchKernelGGL((proj_kernel<float, float>), grid, dim3(256), 0, s, a, L.cs);
    else
        hipLaunchKernelGGL((proj_kernel<double, double>), grid, dim3(256), 0, s, a, L.cs);
    const int64_t len = 2 * (int64_t)a.nv * a.nr;
    hipLaunchKernelGGL(proj_reduce_kernel, dim3((unsigned)((len * SCG_WAVE + 255) / 256), 1, L.nz), dim3(256), 0, s, a.part, nch,
                       a.part_stride, len, P, a.st, a.gate_i, a.flag, L.cs);
}

}  // namespace scg
