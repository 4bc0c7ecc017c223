// Launchers of the library's HIP kernels (one declaration per kernel family).
#pragma once
#include "internal.h"

namespace scg {

// Device arrays of the Lanczos recurrences, indexed by the step i (1-based).
struct LzArrays {
    double* alpha;  // alpha_i
    double* beta;   // beta_i (beta[0] = beta_0)
    double* delta;  // delta_i
    double* gam;    // gamma_{i-1}, the coefficient used at step i (gam[1] = 0)
    double* zeta;   // zeta_i
    double* est;    // relative residual estimate after step i
};
__device__ inline LzArrays zoff(LzArrays a, int64_t cs) {
    if (cs == 0) return a;
    return LzArrays{zoff(a.alpha, cs), zoff(a.beta, cs), zoff(a.delta, cs), zoff(a.gam, cs), zoff(a.zeta, cs), zoff(a.est, cs)};
}

// P = V^dag R contraction (split-K partials then a fixed-order reduction)
struct ProjArgs {
    const void* V;          // rows of V, stride ldv complex
    int64_t ldv;
    int nv;                 // rows of V
    const void* R[24];      // the nr vectors of R
    int nr;
    int64_t n;              // complex per vector
    int64_t kchunk;         // complex per workgroup
    double* part;           // [chunk][nv][nr] complex partials
    int64_t part_stride;    // doubles per chunk (>= 2 * nv * nr)
    const LzState* st;      // optional gate: skip when gate_i > st->m
    int gate_i;
    int rows_from_m;        // rows beyond st->m - i0 + 1 are treated as absent
    int i0;
    const int32_t* flag;    // optional gate: skip when *flag == 0
};
// fp32: V and R stored in FP32; fp64_math: contract them on the FP64 matrix cores anyway
void project(bool fp32, const ProjArgs& a, int64_t nrowblocks, double* P, const Launch& L, bool fp64_math = false);
int64_t proj_chunks(int64_t n, int64_t kchunk);
// V^dag R for the reorthogonalisation's one or two columns, FP64 arithmetic on the vector units
// (v32: V stored in FP32; r32: R stored in FP32), partials and output as project()
void reorth_project(bool v32, bool r32, const ProjArgs& a, double* P, const Launch& L);
// Static partials of the allocation-free contraction: PROJ_SCRATCH_DOUBLES doubles (4 MiB) per GPU.
// proj_scratch() returns the current device's copy (its address is looked up once per device).
constexpr int64_t PROJ_SCRATCH_DOUBLES = int64_t(1) << 19;
double* proj_scratch();

void pack_links(Prec prec, const Geom& g, const double* U, void* out, hipStream_t s);
// per-block maxima of the distance of every link from SU(3) as its two-row format sees it
void su3_defect(const double* U, int64_t nlinks, double* part, hipStream_t s);
int64_t su3_defect_blocks(int64_t nlinks);
// tab (optional, device memory): one canonical pointer per configuration of the launch
void pack_vec(bool fp32, const double* in, void* out, int64_t Vh, int nvec, const Launch& L, const double* const* tab = nullptr);
void unpack_vec(bool fp32, const void* in, double* out, int64_t Vh, int nvec, const Launch& L, double* const* tab = nullptr);
void gamma5_copy(bool fp32, const void* a, void* b, int64_t Vh, int nvec, const Launch& L);
void convert(bool from32, bool to32, const void* a, void* b, int64_t n, const Launch& L);
void convert_map(bool from32, bool to32, const void* a, void* b, int64_t n, const int32_t* vec_map, int nact, const Launch& L);
// per-configuration byte copies (bytes a multiple of 4): configuration z moves src + z*src_cs to
// dst + z*dst_cs; cfg_zero clears bytes at dst + z*L.cs
void cfg_copy(const void* src, int64_t src_cs, void* dst, int64_t dst_cs, int64_t bytes, const Launch& L);
void cfg_zero(void* dst, int64_t bytes, const Launch& L);
void norm2_partials(bool fp32, const void* a, int64_t n, int nvec, double* part, const Launch& L);
int64_t norm2_blocks(int64_t n);
void sum_partials(const double* part, int64_t nb, int nvec, double* out, bool sqrt_out, const Launch& L);

void lz_start(LzState* st, const double* r2part, int64_t nb, const double* b2part, double* beta, const Launch& L);
void lz_first_vector(bool fp32, const LzState* st, const void* r, void* v, int64_t n, const Launch& L);
// the Lanczos coefficient alpha_i from the np stencil partials apart, the LU scalars of Eq. (2), and the vector updates
void lz_update(bool fp32, int i, LzState* st, const double* apart, int64_t np, const LzArrays& a, void* f, const void* v,
               const void* wprev, void* wout, double* x1, double* f2part, int64_t n, const Launch& L);
void lz_beta(int i, LzState* st, const double* part, int64_t np, const LzArrays& a, const Launch& L);
void lz_next(bool fp32, int i, const LzState* st, const double* beta, const void* f, void* vn, int64_t n, const Launch& L);

void seed_eta(int i0, int nb, int nr, const LzState* st, const double* gam, const double* P, double* E, double* eta_prev,
              int32_t* nvalid, const Launch& L);
void seed_update(bool w32, bool x32, const void* W, int nw, const double* E, void* X, int nx, int64_t n, const int32_t* nrow_dev,
                 const Launch& L);

// v32: the basis V is stored in FP32 while v and f are FP64 (fp32 false)
void reorth_update(bool fp32, int i, int pass, const LzState* st, const void* V, int64_t n, const double* G, void* v, void* f,
                   double* part, const Launch& L, bool v32 = false);
void reorth_scalar(int i, int pass, LzState* st, const double* part, int64_t nb, const double* G, const Launch& L);
void reorth_finish(bool fp32, int i, int pass, const LzState* st, void* v, void* f, double* f2part, int64_t n, const Launch& L);
void reorth_decide(int i, int pass, LzState* st, const double* f2b, const double* f2a, int64_t nb, const Launch& L);

void cg_alpha(CgVec* cg, const double* part, int64_t nb, const int32_t* vec_map, int nact, const Launch& L, bool pc = false);
void dot_map(bool fp32, const void* a, const void* b, int64_t n, const int32_t* vec_map, int nact, const CgVec* cg, double* part,
             const Launch& L);
void cg_beta_pc(CgVec* cg, const double* rrpart, const double* rzpart, int64_t nb, const int32_t* vec_map, int nact, int max_iter,
                const Launch& L);
void cg_update(bool fp32, bool x32, const CgVec* cg, const int32_t* vec_map, int nact, void* X, const void* P, void* R,
               const void* Q, double* part, int64_t n, const Launch& L);
void cg_beta(CgVec* cg, const double* part, int64_t nb, const int32_t* vec_map, int nact, int max_iter, const Launch& L);
void cg_p(bool fp32, const CgVec* cg, const int32_t* vec_map, int nact, void* P, const void* R, int64_t n, bool ignore_frozen,
          const Launch& L);

// learned preconditioner K (learned.hip); fields are [vec][parity][12][Vh] complex FP32
// pmask: output parities computed (1 even, 2 odd, 3 both); zero_odd_input: the input is E_e x;
// t0, nt: only the band of t-slices [t0, t0 + nt) mod Lt (nt = 0: the whole lattice); in_t0, in_nt: the
// input is zero outside that band (in_nt = 0: no such band)
// FP32 links of K's transports: ne = 9 (whole, [mu][parity][9][Vh]) or 6 (special-unitary links as
// rows 0 and 1, [mu][parity][6][Vh]; row 2 rebuilt in registers)
struct KLinks {
    const void* p;
    int ne;
};
// in_vstride: complex per input vector (0: 24 Vh, a full field; 12 Vh: even-site vectors, for an
// even-only input, zero_odd_input)
void k_layer(const Geom& g, KLinks links, const void* in, void* out, const void* W, bool dagger, const int32_t* vmap,
             int nvec, bool zero_odd_input, hipStream_t s, int pmask = 3, int t0 = 0, int nt = 0, int in_t0 = 0, int in_nt = 0,
             int64_t in_vstride = 0);
// the block partials of one layer's weight gradient, summed over the sites of pmask and the band (where
// the incoming gradient lives), written to part ([9][nb][32] doubles); returns nb.  k_grad_reduce then
// adds the listed gradients to G ([3 layers][9][16] complex) in list order.
int64_t k_grad(const Geom& g, KLinks links, const void* gv, const void* in, bool dagger, int nvec, double* part, hipStream_t s,
               bool zero_odd_input = false, int pmask = 3, int t0 = 0, int nt = 0, int64_t in_vstride = 0);
struct KGradList {
    static constexpr int MAX = 6;
    const double* part[MAX];
    int64_t nb[MAX];
    int dagger[MAX], layer[MAX];
    int n;
};
void k_grad_reduce(const KGradList& q, double* G, hipStream_t s);
// |u|^2 partials of S even-site FP32 vectors over a band of t-slices (k_band_blocks per vector)
void k_band_norm(const Geom& g, int t0, int nt, const void* u, int S, double* part, hipStream_t s);
int64_t k_band_blocks(const Geom& g, int t0, int nt);
int64_t k_grad_blocks(const Geom& g);
void k_embed(bool x32, const void* x, void* full, int64_t n, const int32_t* vmap, int nvec, hipStream_t s);
void k_restrict(bool x32, const void* full, void* x, int64_t n, const int32_t* vmap, int nvec, hipStream_t s);
void k_zero_odd(void* full, int64_t n, int nvec, hipStream_t s);
// the loss residual on the even sites of the band (nt = 0: all of them); the gradient field is written
// there only
void k_residual(const void* zfull, const void* u, const double* unorm2, void* gfull, int64_t n, int S, double* part, hipStream_t s,
                const Geom& g, int t0 = 0, int nt = 0);
int64_t k_residual_blocks(const Geom& g, int t0 = 0, int nt = 0);
void k_adam(double* Wm, void* W32, double* G, double* m, double* v, int t, double lr, int n, hipStream_t s);
// X = V S for nout <= 16 outputs (S: m x nout row-major); X in FP32, or FP64 with x64
void k_combine(bool v32, const void* V, int m, const double* S, int nout, void* X, int64_t n, hipStream_t s, bool x64 = false);
// deflated CG: E[k][j] = sign * sum_l Ginv[k][l] P[l][j] for the columns j listed in map (w entries,
// -1 = none) whose CG record (if cg is given) is neither done nor frozen; 0 in every other column.
// Ginv: nev x nev, P and E: nev x ncol, complex FP64 row-major; ncol <= 32.
void defl_mu(const double* Ginv, const double* P, int nev, int ncol, const int32_t* map, int w, const CgVec* cg, double sign,
             double* E, const Launch& L);

// generic FP64 vector combinations of the indefinite solver (minres.hip): out = [out +] sum_t a_t in_t
// for each of nout outputs (nt <= 4 terms each, complex coefficients a_t = are + i aim)
struct ZLC {
    const void* in[4];
    double are[4], aim[4];
    int nt, acc;
    void* out;
};
void zlincomb(const ZLC* o, int nout, int64_t n, hipStream_t s);
// out[2p], out[2p+1] = Re, Im of a_p^dag b_p for np pairs of n-complex vectors; part holds
// 2 * min(np, 32) * zdots_blocks(n) doubles
void zdots(const void* const* a, const void* const* b, int np, int64_t n, double* part, double* out, hipStream_t s);
int64_t zdots_blocks(int64_t n);

// roofline probes (probe.hip): GB/s of copy (kind 0), FP64 triad (1) or read (2) over buffers of
// `bytes`; TFLOP/s of FP64 (dtype 0) or FP32 (1) matrix-core chains on every SIMD
double probe_bandwidth(int kind, int64_t bytes, int reps, hipStream_t s);
double probe_mfma(int dtype, int iters, hipStream_t s);

}  // namespace scg
