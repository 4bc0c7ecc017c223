// Dense contraction P = V^dag R on the matrix cores (Algorithm 1's seeding projections of Eq. (1) and its
// reorthogonalisation coefficients).
//
// V is nv vectors, R nr vectors, each n complex numbers stored as interleaved (re, im).
// The complex product is a real GEMM over K = 2n reals:
//     Re P[r][j] = sum_k V[r][k] R[j][k]
//     Im P[r][j] = sum_k V[r][k] R~[j][k],   R~[j][2t] = Im R[j][t],  R~[j][2t+1] = -Re R[j][t]
// so the B operand has 2*nr real columns (Re and Im of every j) and A is V read as stored.
//
// Split-K: a workgroup owns a K-chunk and up to 32 rows of V (two 16-row MFMA tiles) and
// computes all 2*nr columns (up to three 16-column tiles) of its partial product, staging
// 32 complex per row through LDS per step; the next two steps' staging is loaded into two
// register sets while the current one is contracted.  Partials go to part[chunk][row][j] and a second
// kernel sums the chunks in a fixed order (deterministic).  FP64 inputs use
// v_mfma_f64_16x16x4; FP32 inputs use v_mfma_f32_16x16x4 with FP32 accumulation.
//
// MFMA operand layout (16x16x4, one block): lane l holds A[l%16][l/16] and B[l/16][l%16];
// the 16x16 result is 4 values per lane in column l%16: rows l/16 + 4q for the FP64
// instruction and rows 4*(l/16) + q for the FP32 one (q = 0..3; checked on gfx950).
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>

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
__global__ __launch_bounds__(256) void proj_kernel(const ProjArgs pa, int64_t cs) {
    using Acc = MfmaAcc<T>;
    using V4 = typename Acc::V4;
    __shared__ T As[PJ_ROWS * PJ_LD];
    __shared__ T Bs[PJ_MAXR * PJ_LD];

    // the argument is only read (a write would make the compiler copy all of it to scratch)
    const LzState* st = zoff(pa.st, cs);
    const int32_t* flag = zoff(pa.flag, cs);
    if (st && pa.gate_i > st->m) return;
    if (flag && *flag == 0) return;
    int nvalid = pa.nv;
    if (st && pa.rows_from_m) nvalid = max(0, min(pa.nv, st->m - pa.i0 + 1));
    const int row0 = blockIdx.y * PJ_ROWS;
    const int nrow = min(PJ_ROWS, nvalid - row0);
    if (nrow <= 0) return;

    const TS* V = (const TS*)zoff(pa.V, cs);
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

    // the staging of steps kb + PJ_KC and kb + 2 PJ_KC is loaded into two register sets while
    // step kb is contracted from LDS, so two steps of global loads are always in flight behind
    // the matrix-core work (one complex per thread and pass)
    constexpr int NVU = PJ_ROWS * PJ_KC / 256;                 // V elements per thread
    constexpr int NRU = (PJ_MAXR * PJ_KC + 255) / 256;         // R elements per thread (at most)
    struct Regs {
        cx<TS> v[NVU], r[NRU];
    };
    Regs ra, rb;
    const TS* vrow[NVU];      // this thread's V rows (null beyond nrow) and R vectors (null beyond nr)
    const TS* rvec[NRU];
#pragma unroll
    for (int u = 0; u < NVU; u++) {
        const int r = (threadIdx.x + 256 * u) / PJ_KC;
        vrow[u] = r < nrow ? V + 2 * (int64_t)(row0 + r) * pa.ldv : nullptr;
    }
#pragma unroll
    for (int u = 0; u < NRU; u++) {
        const int j = (threadIdx.x + 256 * u) / PJ_KC;
        rvec[u] = j < nr ? (const TS*)zoff(pa.R[j], cs) : nullptr;
    }
    const int cth = threadIdx.x % PJ_KC;   // the complex index within a step (256 is a multiple of PJ_KC)
    auto fetch = [&vrow, &rvec, cth, k_end](Regs& g, int64_t kb) {
        const bool cok = kb + cth < k_end;
#pragma unroll
        for (int u = 0; u < NVU; u++)
            g.v[u] = (vrow[u] && cok) ? *(const cx<TS>*)(vrow[u] + 2 * (kb + cth)) : mk<TS>(0, 0);
#pragma unroll
        for (int u = 0; u < NRU; u++)
            g.r[u] = (rvec[u] && cok) ? *(const cx<TS>*)(rvec[u] + 2 * (kb + cth)) : mk<TS>(0, 0);
    };
    // one step: the registers of step kb to LDS, the loads of step kb + 2 PJ_KC into the same
    // registers, then the contraction of step kb
    auto step = [&](Regs& g, int64_t kb) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NVU; u++) {
            const int idx = threadIdx.x + 256 * u;
            const int r = idx / PJ_KC, c = idx % PJ_KC;
            As[r * PJ_LD + 2 * c] = (T)g.v[u].re;
            As[r * PJ_LD + 2 * c + 1] = (T)g.v[u].im;
        }
#pragma unroll
        for (int u = 0; u < NRU; u++) {
            const int idx = threadIdx.x + 256 * u;
            const int j = idx / PJ_KC, c = idx % PJ_KC;
            if (j < nr) {
                Bs[j * PJ_LD + 2 * c] = (T)g.r[u].re;
                Bs[j * PJ_LD + 2 * c + 1] = (T)g.r[u].im;
            }
        }
        __syncthreads();
        if (kb + 2 * PJ_KC < k_end) fetch(g, kb + 2 * PJ_KC);
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
    };
    if (k_begin < k_end) fetch(ra, k_begin);
    if (k_begin + PJ_KC < k_end) fetch(rb, k_begin + PJ_KC);
    for (int64_t kb = k_begin; kb < k_end; kb += 2 * PJ_KC) {
        step(ra, kb);
        if (kb + PJ_KC < k_end) step(rb, kb + PJ_KC);
    }

    // write the partial tiles: part[chunk][row][j] complex (FP64)
    double* out = zoff(pa.part, cs) + (int64_t)blockIdx.x * pa.part_stride;
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

// The reorthogonalisation coefficients V_{1..i}^dag [v_i, f]: at most two columns, which would fill two
// of the sixteen columns of a matrix-core tile, so they are formed on the vector units in FP64 instead.
// A workgroup takes a K-chunk and RP_ROWS rows of V (the row blocks of one chunk run one after another
// on one XCD, so the chunk of R is fetched once into its L2); each thread runs through the chunk with stride
// 256 * EPL, reading EPL consecutive entries (16 bytes of each row of V: one FP64 complex, or two FP32
// ones) of the one or two R vectors once and of the RP_ROWS rows of V (row addresses are uniform; a
// row beyond the last valid one reads the last valid row again and is not written), and keeps FP64
// sums per row and column.  The workgroup's sums are formed in a fixed order through LDS and written
// to part[chunk][row][j] like proj_kernel's, so proj_reduce_kernel finishes them.  TV, TR: storage
// of V and of R (FP32 entries are widened exactly).  With FP32 V the chunk bounds and n are even.
// 8 rows keep 122 VGPRs (4 waves per SIMD) with every load of a step in flight; 16 rows took 240
// and the compiler then issued the loads one at a time
constexpr int RP_ROWS = 8;
template <typename T>
struct Pair16;   // EPL consecutive complex entries as 16-byte loads
template <>
struct Pair16<double> {
    static constexpr int EPL = 1;
    __device__ static inline void load(const cx<double>* p, double (&re)[1], double (&im)[1]) {
        const double2 q = *(const double2*)p;
        re[0] = q.x;
        im[0] = q.y;
    }
};
template <>
struct Pair16<float> {
    static constexpr int EPL = 2;
    __device__ static inline void load(const cx<float>* p, float (&re)[2], float (&im)[2]) {
        const float4 q = *(const float4*)p;
        re[0] = q.x;
        im[0] = q.y;
        re[1] = q.z;
        im[1] = q.w;
    }
};
template <typename TV, typename TR>
__global__ __launch_bounds__(256) void reorth_proj_kernel(const ProjArgs pa, int64_t cs) {
    constexpr int EPL = Pair16<TV>::EPL;
    __shared__ double tile[256 * (RP_ROWS + 1)];
    constexpr int G = 256 / RP_ROWS;   // groups of RP_ROWS threads in the final sums
    __shared__ double grp[256];
    const LzState* st = zoff(pa.st, cs);
    const int32_t* flag = zoff(pa.flag, cs);
    if (st && pa.gate_i > st->m) return;
    if (flag && *flag == 0) return;
    int nvalid = pa.nv;
    if (st && pa.rows_from_m) nvalid = max(0, min(pa.nv, st->m - pa.i0 + 1));
    const int nrb = (pa.nv + RP_ROWS - 1) / RP_ROWS;
    const int64_t nch = (pa.n + pa.kchunk - 1) / pa.kchunk;
    const int64_t w = xcd_logical_block(nch * nrb);
    if (w >= nch * nrb) return;
    const int64_t chunk = w / nrb;
    const int row0 = (int)(w % nrb) * RP_ROWS;
    const int nrow = min(RP_ROWS, nvalid - row0);
    if (nrow <= 0) return;
    const int nr = pa.nr;
    const cx<TR>* R0 = (const cx<TR>*)zoff(pa.R[0], cs);
    const cx<TR>* R1 = (const cx<TR>*)zoff(pa.R[nr > 1 ? 1 : 0], cs);
    const cx<TV>* Vb = (const cx<TV>*)zoff(pa.V, cs);
    const cx<TV>* vrow[RP_ROWS];
#pragma unroll
    for (int r = 0; r < RP_ROWS; r++) vrow[r] = Vb + (int64_t)(row0 + min(r, nrow - 1)) * pa.ldv;
    const int64_t k_begin = chunk * pa.kchunk;
    const int64_t k_end = min(pa.n, k_begin + pa.kchunk);
    // acc[r][0..3]: Re, Im of conj(V_r) R_0 and of conj(V_r) R_1
    double acc[RP_ROWS][4];
#pragma unroll
    for (int r = 0; r < RP_ROWS; r++)
#pragma unroll
        for (int c = 0; c < 4; c++) acc[r][c] = 0.0;
#pragma unroll 1
    for (int64_t k = k_begin + EPL * threadIdx.x; k < k_end; k += EPL * 256) {
        double ar[EPL], ai[EPL], br[EPL], bi[EPL];
#pragma unroll
        for (int e = 0; e < EPL; e++) {
            const cx<TR> a = R0[k + e], b = R1[k + e];
            ar[e] = a.re;
            ai[e] = a.im;
            br[e] = b.re;
            bi[e] = b.im;
        }
        TV vr[RP_ROWS][EPL], vi[RP_ROWS][EPL];   // widened where they are used
#pragma unroll
        for (int r = 0; r < RP_ROWS; r++) Pair16<TV>::load(vrow[r] + k, vr[r], vi[r]);
#pragma unroll
        for (int r = 0; r < RP_ROWS; r++)
#pragma unroll
            for (int e = 0; e < EPL; e++) {
                const double x = vr[r][e], y = vi[r][e];
                acc[r][0] = fma(x, ar[e], fma(y, ai[e], acc[r][0]));
                acc[r][1] = fma(x, ai[e], fma(-y, ar[e], acc[r][1]));
                acc[r][2] = fma(x, br[e], fma(y, bi[e], acc[r][2]));
                acc[r][3] = fma(x, bi[e], fma(-y, br[e], acc[r][3]));
            }
    }
    // per column component c: the 256 threads' row sums through LDS, G groups of RP_ROWS threads summed
    // row by row, then the G group sums (fixed order throughout)
    double* out = zoff(pa.part, cs) + chunk * pa.part_stride;
    const int e = threadIdx.x % RP_ROWS, g = threadIdx.x / RP_ROWS;
#pragma unroll
    for (int c = 0; c < 4; c++) {
        if (c >= 2 * nr) break;   // uniform
#pragma unroll
        for (int r = 0; r < RP_ROWS; r++) tile[threadIdx.x * (RP_ROWS + 1) + r] = acc[r][c];
        __syncthreads();
        double sum = 0.0;
        for (int q = 0; q < RP_ROWS; q++) sum += tile[(g * RP_ROWS + q) * (RP_ROWS + 1) + e];
        grp[g * RP_ROWS + e] = sum;
        __syncthreads();
        if (threadIdx.x < RP_ROWS && (int)threadIdx.x < nrow) {
            double t = 0.0;
            for (int q = 0; q < G; q++) t += grp[q * RP_ROWS + threadIdx.x];
            out[2 * ((int64_t)(row0 + threadIdx.x) * nr + (c >> 1)) + (c & 1)] = t;
        }
        __syncthreads();
    }
}

void reorth_project(bool v32, bool r32, const ProjArgs& a, double* P, const Launch& L) {
    if (a.part == nullptr || P == nullptr) throw std::invalid_argument("reorth_project: partials or output buffer missing");
    if (a.nr < 1 || a.nr > 2) throw std::invalid_argument("reorth_project: one or two columns");
    if (a.part_stride < 2 * (int64_t)a.nv * a.nr) throw std::invalid_argument("reorth_project: partial stride below 2 nv nr");
    if (v32 && (a.n % 2 || a.kchunk % 2 || a.ldv % 2))
        throw std::invalid_argument("reorth_project: an FP32 basis is read in pairs (even n, chunk and row stride)");
    const hipStream_t s = L.s;
    const int64_t nch = proj_chunks(a.n, a.kchunk);
    const dim3 grid((unsigned)xcd_grid(nch * ((a.nv + RP_ROWS - 1) / RP_ROWS)), 1, L.nz);
    if (v32 && r32)
        hipLaunchKernelGGL((reorth_proj_kernel<float, float>), grid, dim3(256), 0, s, a, L.cs);
    else if (v32)
        hipLaunchKernelGGL((reorth_proj_kernel<float, double>), grid, dim3(256), 0, s, a, L.cs);
    else if (!r32)
        hipLaunchKernelGGL((reorth_proj_kernel<double, double>), grid, dim3(256), 0, s, a, L.cs);
    else
        throw std::invalid_argument("reorth_project: an FP64 basis takes FP64 columns");
    const int64_t len = 2 * (int64_t)a.nv * a.nr;
    hipLaunchKernelGGL(proj_reduce_kernel, dim3((unsigned)((len * SCG_WAVE + 255) / 256), 1, L.nz), dim3(256), 0, s, a.part, nch,
                       a.part_stride, len, P, a.st, a.gate_i, a.flag, L.cs);
}

// Split-K partials of the allocation-free contraction (seedcg_project_noalloc): one copy of this
// array per GPU, held by the loaded code object until the process ends.  In host code its name is
// only a stand-in for the device copy; proj_scratch() returns the device address to pass instead.
static __device__ __align__(256) double scratch[PROJ_SCRATCH_DOUBLES];

double* proj_scratch() {
    static std::mutex mu;
    static std::map<int, double*> addr;   // device ordinal -> address of that device's copy
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) throw std::runtime_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) return it->second;
    double* ptr = nullptr;
    e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
        throw std::runtime_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    addr[dev] = ptr;
    return ptr;
}

void project(bool fp32, const ProjArgs& a, int64_t nrowblocks, double* P, const Launch& L, bool fp64_math) {
    // the kernel stages at most PJ_MAXR columns of R and writes its split-K partials to a.part
    if (a.part == nullptr || P == nullptr) throw std::invalid_argument("project: partials or output buffer missing");
    if (a.nr < 1 || a.nr > PJ_MAXR) throw std::invalid_argument("project: 1 <= nr <= 24 columns per contraction");
    if (a.part_stride < 2 * (int64_t)a.nv * a.nr) throw std::invalid_argument("project: partial stride below 2 nv nr");
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
