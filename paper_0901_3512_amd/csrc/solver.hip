// Host runtime and C ABI of the Seed-CG library (Algorithm 1 of the paper and plain CG).
//
// The host only enqueues kernels: every scalar recurrence of Algorithm 1 (alpha, beta,
// delta, gamma, zeta, the eta recurrence of step 7, the residual estimate, the choice of m)
// lives in device memory and is updated by one-workgroup kernels, so an iteration never
// waits for the host.  The host reads the device state once every `sync_every` steps to
// learn whether the run has ended; kernels of steps beyond the device's m return at once.
//
// Step 7 is blocked: the projections v_i^dag r_0^j of up to b consecutive steps are one
// MFMA contraction P = V_blk^dag R_0 taken before step 8 touches v_i, and the updates
// x^j += eta^j_i w_i of the block are one pass X += W_blk E over a ring of b w-vectors.
// The result is the paper's step 7 exactly, summed in another order.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kernels.h"
#include "seedcg.h"

using namespace scg;

namespace {

struct HipError {
    std::string what;
};
struct ArgError {
    std::string what;
};
struct StateError {
    std::string what;
};
struct OomError {
    std::string what;
};

#define HIPCHK(call)                                                                                \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            throw HipError{std::string(#call) + ": " + hipGetErrorString(e_)};                      \
    } while (0)

struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void ensure(size_t nbytes) {
        if (nbytes <= bytes && p) return;
        release();
        if (nbytes == 0) nbytes = 256;
        hipError_t e = hipMalloc(&p, nbytes);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            throw OomError{"hipMalloc of " + std::to_string(nbytes) + " bytes failed"};
        }
        bytes = nbytes;
    }
    template <typename T>
    T* as() const {
        return (T*)p;
    }
};

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int env_int(const char* name, int dflt) {
    const char* v = getenv(name);
    return v ? atoi(v) : dflt;
}

}  // namespace

struct seedcg_s {
    seedcg_params p;
    Geom g;
    hipStream_t s = nullptr;
    std::string err;
    bool lo = false;        // FP32 inner vectors (mixed precision)
    Prec lo_prec = P64;     // precision of the inner stencil
    int64_t N = 0;          // complex per vector
    int tps64 = 3, tps_lo = 3;
    int vb64 = 1, vb_lo = 1;      // vectors per stencil workgroup
    int sync_every = 16;
    int debug = 0;

    DBuf links64, links_lo;
    // operator work vectors (FP64), sized for a batch
    DBuf t1_64, u_64, t1_lo, u_lo, g5buf;
    int64_t work_vecs = 0;
    // Algorithm 1
    DBuf basis, wring, f, x1, R0, Bint, Xint, st, arrays, apart, f2a, f2b, rpart, G, projpart, P, E, etaprev, nvalid;
    int32_t m_cap = 0;
    int32_t m_used = 0;
    bool have_seed = false;
    int seed_nrhs = 0;
    // CG
    DBuf cgv, vmap, Pv, Rv, Qv, R64, cgpart, rrpart, respart, norms;
    // sampled timing of the stencil launches (hipEvent pairs on the handle's stream)
    int timing_every = 0;
    int64_t hop_count = 0;
    std::vector<hipEvent_t> ev0, ev1;
    std::vector<double> ev_bytes, ev_flops;
    size_t ev_used = 0;
    double t_ms = 0.0, t_bytes = 0.0, t_flops = 0.0;
    int64_t t_launches = 0;
    ~seedcg_s() {
        for (auto e : ev0) (void)hipEventDestroy(e);
        for (auto e : ev1) (void)hipEventDestroy(e);
    }

    int64_t vec_bytes(bool low) const { return N * (low ? 8 : 16); }
    LzArrays arr() const {
        double* a = arrays.as<double>();
        const int64_t L = (int64_t)m_cap + 2;
        return LzArrays{a, a + L, a + 2 * L, a + 3 * L, a + 4 * L, a + 5 * L};
    }
};

static std::string g_create_error;

// ---------------------------------------------------------------------------------------------
// the operator
// ---------------------------------------------------------------------------------------------
namespace {

void ensure_work(seedcg_s* h, int nvec) {
    if (nvec <= h->work_vecs && h->t1_64.p) return;
    const int64_t n = std::max<int64_t>(nvec, 1);
    h->t1_64.ensure(n * h->vec_bytes(false));
    h->u_64.ensure(n * h->vec_bytes(false));
    h->g5buf.ensure(n * h->vec_bytes(false));
    if (h->lo) {
        h->t1_lo.ensure(n * h->vec_bytes(true));
        h->u_lo.ensure(n * h->vec_bytes(true));
    }
    h->work_vecs = n;
}

// One stencil launch; when timing is on, every timing_every-th launch is bracketed by events and
// its algorithmic bytes are recorded: links 144 reals per output site (read once for the whole
// batch), and per vector the input and output spinors (24 reals each per site) plus every
// epilogue operand (24 reals per site each).
void hop(seedcg_s* h, Prec pr, const void* L, const void* in, void* out, int par, int nvec, const HopEpi& e, int tps) {
    const bool sample = h->timing_every > 0 && (h->hop_count++ % h->timing_every) == 0 && h->ev_used < h->ev0.size();
    if (sample) HIPCHK(hipEventRecord(h->ev0[h->ev_used], h->s));
    launch_hop(pr, h->g, L, in, out, par, nvec, e, tps, pr == P64 ? h->vb64 : h->vb_lo, h->s);
    if (sample) {
        HIPCHK(hipEventRecord(h->ev1[h->ev_used], h->s));
        const double sl = pr == P64 ? 8.0 : (pr == P32 ? 4.0 : 2.0);
        const double ss = pr == P64 ? 8.0 : 4.0;
        const double Vh = (double)h->g.Vh;
        int ops = 2 + (e.combine ? 1 : 0) + (e.z ? 1 : 0) + (e.red == 1 ? 1 : 0);
        h->ev_bytes.push_back(Vh * 144.0 * sl + (double)nvec * Vh * 24.0 * ss * ops);
        h->ev_flops.push_back((double)nvec * Vh * 1320.0);
        h->ev_used++;
    }
}

struct MOpts {
    const void* z = nullptr;      // out = sy * M x + cz * z
    double sy = 1.0;
    const double* cz_dev = nullptr;
    int cz_negate = 0;
    double cz_host = 0.0;
    int red = 0;                  // 1: Re d^dag out, 2: |out|^2
    const void* d = nullptr;
    double* partials = nullptr;
    const int32_t* gate_m = nullptr;
    int gate_i = 0;
    const int32_t* vec_map = nullptr;
    const CgVec* cg = nullptr;
};

// out = M x for nvec vectors (M = A^dag A = gamma5 A gamma5 A), with the epilogue options on
// the last hop.  low = FP32 vectors with the inner links.
void apply_M_int(seedcg_s* h, bool low, const void* x, void* out, int nvec, const MOpts& o) {
    ensure_work(h, nvec);
    const Prec pr = low ? h->lo_prec : P64;
    const void* L = low ? h->links_lo.p : h->links64.p;
    void* t1 = low ? h->t1_lo.p : h->t1_64.p;
    void* u = low ? h->u_lo.p : h->u_64.p;
    const int tps = low ? h->tps_lo : h->tps64;
    const double k2 = h->p.kappa * h->p.kappa;
    HopEpi e{};
    e.gate_m = o.gate_m;
    e.gate_i = o.gate_i;
    e.vec_map = o.vec_map;
    e.cg = o.cg;
    e.sy = 1.0;
    // t1 = H_oe x
    hop(h, pr, L, x, t1, 1, nvec, e, tps);
    // u = gamma5 (x - kappa^2 H_eo t1)
    HopEpi e2 = e;
    e2.combine = 1;
    e2.apply_g5 = 1;
    e2.kappa2 = k2;
    e2.x = x;
    hop(h, pr, L, t1, u, 0, nvec, e2, tps);
    // t1 = H_oe u
    hop(h, pr, L, u, t1, 1, nvec, e, tps);
    // out = sy * gamma5 (u - kappa^2 H_eo t1) + cz z
    HopEpi e4 = e2;
    e4.x = u;
    e4.sy = o.sy;
    e4.z = o.z;
    e4.cz_dev = o.cz_dev;
    e4.cz_negate = o.cz_negate;
    e4.cz_host = o.cz_host;
    e4.red = o.red;
    e4.d = o.d;
    e4.partials = o.partials;
    hop(h, pr, L, t1, out, 0, nvec, e4, tps);
}

// y = A x or A^dag x = gamma5 A gamma5 x (FP64)
void apply_A_int(seedcg_s* h, const void* x, void* out, int nvec, bool dagger) {
    ensure_work(h, nvec);
    const double k2 = h->p.kappa * h->p.kappa;
    const void* in = x;
    if (dagger) {  // A^dag = gamma5 A gamma5: the last gamma5 is the hop epilogue's
        gamma5_copy(false, x, h->g5buf.p, h->g.Vh, nvec, h->s);
        in = h->g5buf.p;
    }
    HopEpi e{};
    e.sy = 1.0;
    launch_hop(P64, h->g, h->links64.p, in, h->t1_64.p, 1, nvec, e, h->tps64, h->vb64, h->s);
    HopEpi e2 = e;
    e2.combine = 1;
    e2.apply_g5 = dagger ? 1 : 0;
    e2.kappa2 = k2;
    e2.x = in;
    launch_hop(P64, h->g, h->links64.p, h->t1_64.p, out, 0, nvec, e2, h->tps64, h->vb64, h->s);
}

void check_launch() { HIPCHK(hipGetLastError()); }

int64_t nsb_of(seedcg_s* h, bool low) { return hop_site_blocks(h->g, low ? h->tps_lo : h->tps64); }

}  // namespace

// ---------------------------------------------------------------------------------------------
// Algorithm 1
// ---------------------------------------------------------------------------------------------
namespace {

int seed_block_of(const seedcg_s* h) {
    int b = h->p.seed_block > 0 ? h->p.seed_block : 32;
    return std::min(std::max(b, 1), 32);
}

int64_t kchunk_for(int64_t n, int64_t target_chunks) {
    int64_t kc = (n + target_chunks - 1) / target_chunks;
    kc = (kc + 31) / 32 * 32;
    return std::max<int64_t>(std::min<int64_t>(kc, 65536), 512);
}

// K-chunk of the reorthogonalisation coefficients V_{1..i}^dag [v_i, f]: about 2048 workgroups
// over the (chunk, 32-row block) grid, at least 96 chunks.
int64_t reorth_kchunk(int64_t n, int i) {
    const int64_t rowblocks = (i + 31) / 32;
    return kchunk_for(n, std::max<int64_t>(96, 2048 / rowblocks));
}

void alloc_seed(seedcg_s* h, int nrhs) {
    const bool lo = h->lo;
    const int64_t N = h->N;
    const int b = seed_block_of(h);
    h->wring.ensure(b * h->vec_bytes(lo));
    h->f.ensure(h->vec_bytes(lo));
    h->x1.ensure(h->vec_bytes(false));
    h->R0.ensure(std::max(1, nrhs - 1) * h->vec_bytes(lo));
    h->Bint.ensure(nrhs * h->vec_bytes(false));
    h->Xint.ensure(nrhs * h->vec_bytes(false));
    h->st.ensure(sizeof(LzState));
    const int64_t nb = norm2_blocks(N);
    const int64_t nsb = std::max(nsb_of(h, lo), nsb_of(h, false));
    h->apart.ensure(std::max<int64_t>(nsb, nb) * nrhs * sizeof(double));
    h->f2a.ensure(std::max<int64_t>(nb, 1) * 2 * sizeof(double));
    h->f2b.ensure(std::max<int64_t>(nb, 1) * sizeof(double));
    h->rpart.ensure(3 * nb * sizeof(double));
    h->P.ensure(2 * 32 * 24 * sizeof(double));
    h->E.ensure(2 * 32 * 24 * sizeof(double));
    h->etaprev.ensure(2 * 24 * sizeof(double));
    h->nvalid.ensure(sizeof(int32_t));
    ensure_work(h, nrhs);

    // basis capacity: params.m_max, or what fits in free HBM (at most 8192 vectors)
    int64_t cap = h->p.m_max;
    if (cap <= 0) {
        size_t freeb = 0, total = 0;
        HIPCHK(hipMemGetInfo(&freeb, &total));
        const int64_t reserve = 2LL << 30;
        const int64_t avail = (int64_t)freeb - reserve + (int64_t)h->basis.bytes;
        cap = std::max<int64_t>(0, (int64_t)(0.9 * (double)avail) / h->vec_bytes(lo));
        cap = std::min<int64_t>(cap, 8192);
        if (cap < 2) throw OomError{"no room for a Krylov basis"};
    }
    h->m_cap = (int32_t)cap;
    h->basis.ensure((size_t)cap * h->vec_bytes(lo));
    h->arrays.ensure(6 * ((int64_t)cap + 2) * sizeof(double));
    h->G.ensure(2 * 2 * ((int64_t)cap + 1) * sizeof(double));
    int64_t part_doubles = proj_chunks(N, kchunk_for(N, 1024)) * 2 * 32 * 24;
    for (int64_t i = 1; i <= cap; i++)
        part_doubles = std::max<int64_t>(part_doubles, proj_chunks(N, reorth_kchunk(N, (int)i)) * 4 * i);
    h->projpart.ensure(part_doubles * sizeof(double));
}

void flush_seed_block(seedcg_s* h, int i0, int i1, int nrhs) {
    if (nrhs <= 1 || i1 < i0) return;
    const bool lo = h->lo;
    const int64_t N = h->N;
    const int nb = i1 - i0 + 1, nr = nrhs - 1;
    ProjArgs a{};
    a.V = (const char*)h->basis.p + (int64_t)(i0 - 1) * h->vec_bytes(lo);
    a.ldv = N;
    a.nv = nb;
    for (int j = 0; j < nr; j++) a.R[j] = (const char*)h->R0.p + (int64_t)j * h->vec_bytes(lo);
    a.nr = nr;
    a.n = N;
    a.kchunk = kchunk_for(N, 1024);
    a.part = h->projpart.as<double>();
    a.part_stride = 2 * 32 * 24;
    a.st = h->st.as<LzState>();
    a.gate_i = i0;
    a.rows_from_m = 1;
    a.i0 = i0;
    project(lo, a, 1, h->P.as<double>(), h->s);
    seed_eta(i0, nb, nr, h->st.as<LzState>(), h->arr().gam, h->P.as<double>(), h->E.as<double>(), h->etaprev.as<double>(),
             h->nvalid.as<int32_t>(), h->s);
    seed_update(lo, false, h->wring.p, nb, h->E.as<double>(), (char*)h->Xint.p + h->vec_bytes(false), nr, N,
                h->nvalid.as<int32_t>(), h->s);
}

void reorthogonalise(seedcg_s* h, int i) {
    const bool lo = h->lo;
    const int64_t N = h->N;
    LzState* st = h->st.as<LzState>();
    void* vi = (char*)h->basis.p + (int64_t)(i - 1) * h->vec_bytes(lo);
    const int64_t nb = norm2_blocks(N);
    for (int pass = 1; pass <= 2; pass++) {
        ProjArgs a{};
        a.V = h->basis.p;
        a.ldv = N;
        a.nv = i;
        a.R[0] = vi;
        a.R[1] = h->f.p;
        a.nr = 2;
        a.n = N;
        a.kchunk = reorth_kchunk(N, i);
        a.part = h->projpart.as<double>();
        a.part_stride = 4 * (int64_t)i;
        a.st = st;
        a.gate_i = i;
        a.flag = pass == 2 ? &st->rep_any : nullptr;
        // the reorthogonalisation coefficients are always accumulated in FP64
        project(lo, a, (i + 31) / 32, h->G.as<double>(), h->s, true);
        reorth_update(lo, i, pass, st, h->basis.p, N, h->G.as<double>(), vi, h->f.p, h->rpart.as<double>(), h->s);
        reorth_scalar(i, pass, st, h->rpart.as<double>(), nb, h->G.as<double>(), h->s);
        reorth_finish(lo, i, pass, st, vi, h->f.p, h->f2b.as<double>(), N, h->s);
        reorth_decide(i, pass, st, h->f2a.as<double>(), h->f2b.as<double>(), nb, h->s);
    }
}

void solve_seed_impl(seedcg_s* h, const double* B, double* X, int nrhs, seedcg_report* rep) {
    if (!B || !X || nrhs < 1) throw ArgError{"solve_seed: null pointer or nrhs < 1"};
    if (nrhs > 25) throw ArgError{"solve_seed: at most 25 right-hand sides (24 seeded)"};
    const double t0 = now_s();
    const bool lo = h->lo;
    const int64_t N = h->N, Vh = h->g.Vh;
    alloc_seed(h, nrhs);
    LzState* st = h->st.as<LzState>();
    const LzArrays A = h->arr();
    const int nr = nrhs - 1;

    pack_vec(false, B, h->Bint.p, Vh, nrhs, h->s);
    pack_vec(false, X, h->Xint.p, Vh, nrhs, h->s);
    // Step 1: r_0^j = b^j - M x_0^j (FP64), kept in the inner precision for the projections;
    // RHS 1's goes straight to v_1 after scaling.
    DBuf r64;
    r64.ensure(nrhs * h->vec_bytes(false));
    {
        MOpts o;
        o.sy = -1.0;
        o.z = h->Bint.p;
        o.cz_host = 1.0;
        apply_M_int(h, false, h->Xint.p, r64.p, nrhs, o);
    }
    if (nr > 0) convert(false, lo, (char*)r64.p + h->vec_bytes(false), h->R0.p, nr * N, h->s);
    HIPCHK(hipMemcpyAsync(h->x1.p, h->Xint.p, h->vec_bytes(false), hipMemcpyDeviceToDevice, h->s));
    HIPCHK(hipMemsetAsync(h->etaprev.p, 0, 2 * 24 * sizeof(double), h->s));
    HIPCHK(hipMemsetAsync(h->arrays.p, 0, h->arrays.bytes, h->s));

    LzState hs{};
    hs.m = h->m_cap;
    hs.m_cap = h->m_cap;
    hs.tol = h->p.tol;
    hs.past = h->p.past_factor;
    HIPCHK(hipMemcpyAsync(st, &hs, sizeof(hs), hipMemcpyHostToDevice, h->s));
    // Step 2: beta_0 = ||r_0^1||, v_1 = r_0^1 / beta_0
    const int64_t nb = norm2_blocks(N);
    norm2_partials(false, r64.p, N, 1, h->f2a.as<double>(), h->s);
    norm2_partials(false, h->Bint.p, N, 1, h->f2a.as<double>() + nb, h->s);
    lz_start(st, h->f2a.as<double>(), nb, h->f2a.as<double>() + nb, A.beta, h->s);
    if (lo) {
        convert(false, true, r64.p, h->f.p, N, h->s);
        lz_first_vector(true, st, h->f.p, h->basis.p, N, h->s);
    } else {
        lz_first_vector(false, st, r64.p, h->basis.p, N, h->s);
    }
    check_launch();

    const int b = seed_block_of(h);
    const int k = h->p.reorth_k;
    const int64_t nsb = nsb_of(h, lo);
    int i0 = 1;          // first step of the pending seeding block
    int last_slot = 0;   // ring slot of w_{i-1}
    int i = 1;
    bool finished = false;
    while (!finished) {
        const int i_end = std::min<int>(h->m_cap, i + h->sync_every - 1);
        for (; i <= i_end; i++) {
            void* vi = (char*)h->basis.p + (int64_t)(i - 1) * h->vec_bytes(lo);
            const void* vprev = i > 1 ? (const char*)h->basis.p + (int64_t)(i - 2) * h->vec_bytes(lo) : nullptr;
            // Step 5: f = M v_i - beta_{i-1} v_{i-1}, alpha_i = v_i^dag f
            MOpts o;
            o.z = vprev;
            o.cz_dev = vprev ? &A.beta[i - 1] : nullptr;
            o.cz_negate = 1;
            o.red = 1;
            o.d = vi;
            o.partials = h->apart.as<double>();
            o.gate_m = &st->m;
            o.gate_i = i;
            apply_M_int(h, lo, vi, h->f.p, 1, o);
            // Step 6: LU scalars; f -= alpha_i v_i; w_i; x^1 += zeta_i w_i
            lz_alpha(i, st, h->apart.as<double>(), nsb, A, h->s);
            const int slot = i - i0;
            void* wout = (char*)h->wring.p + (int64_t)slot * h->vec_bytes(lo);
            const void* wprev = (const char*)h->wring.p + (int64_t)(slot > 0 ? slot - 1 : last_slot) * h->vec_bytes(lo);
            lz_update(lo, i, st, A, h->f.p, vi, wprev, wout, h->x1.as<double>(), h->f2a.as<double>(), N, h->s);
            // Step 7, blocked (before step 8 can touch v_i)
            const bool reorth_now = k > 0 && i % k == 0;
            if (slot + 1 == b || reorth_now) {
                flush_seed_block(h, i0, i, nrhs);
                last_slot = slot;
                i0 = i + 1;
            }
            // Step 8
            if (reorth_now) reorthogonalise(h, i);
            // Step 9
            lz_beta(i, st, reorth_now ? h->f2b.as<double>() : h->f2a.as<double>(), nb, A, h->s);
            lz_next(lo, i, st, A.beta, h->f.p, (char*)h->basis.p + (int64_t)i * h->vec_bytes(lo), N, h->s);
        }
        check_launch();
        HIPCHK(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, h->s));
        HIPCHK(hipStreamSynchronize(h->s));
        if (hs.done || i > h->m_cap) finished = true;
    }
    // the last (partial) seeding block
    if (i0 <= hs.m) flush_seed_block(h, i0, std::min(hs.m, i - 1), nrhs);
    HIPCHK(hipMemcpyAsync(h->Xint.p, h->x1.p, h->vec_bytes(false), hipMemcpyDeviceToDevice, h->s));
    unpack_vec(false, h->Xint.p, X, Vh, nrhs, h->s);
    check_launch();
    HIPCHK(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    h->m_used = hs.m;
    h->have_seed = true;
    h->seed_nrhs = nrhs;
    if (rep) {
        rep->m_used = hs.m;
        rep->i_conv = hs.i_conv;
        rep->seed_status = hs.status;
        rep->reorth_passes = hs.passes;
        rep->t_seed_s = now_s() - t0;
        if (rep->iters) rep->iters[0] = hs.m;
        if (rep->matvecs)
            for (int j = 0; j < nrhs; j++) rep->matvecs[j] = (j == 0 ? hs.m : 0) + 1;
    }
}

// ---------------------------------------------------------------------------------------------
// plain CG on a batch (FP64, or FP32 inner iterations with FP64 reliable updates)
// ---------------------------------------------------------------------------------------------
void true_residual(seedcg_s* h, const std::vector<int>& vecs, void* R64, double* part) {
    if (vecs.empty()) return;
    std::vector<int32_t> vm(vecs.begin(), vecs.end());
    DBuf dmap;
    dmap.ensure(vm.size() * sizeof(int32_t));
    HIPCHK(hipMemcpyAsync(dmap.p, vm.data(), vm.size() * sizeof(int32_t), hipMemcpyHostToDevice, h->s));
    MOpts o;
    o.sy = -1.0;
    o.z = h->Bint.p;
    o.cz_host = 1.0;
    o.red = 2;
    o.partials = part;
    o.vec_map = dmap.as<int32_t>();
    apply_M_int(h, false, h->Xint.p, R64, (int)vm.size(), o);
    HIPCHK(hipStreamSynchronize(h->s));  // dmap must outlive the kernels
}

seedcg_status solve_rest_impl(seedcg_s* h, const double* B, double* X, int nrhs, seedcg_report* rep) {
    if (!B || !X || nrhs < 1) throw ArgError{"solve_rest: null pointer or nrhs < 1"};
    const double t0 = now_s();
    const bool lo = h->lo;
    const int64_t N = h->N, Vh = h->g.Vh;
    h->Bint.ensure(nrhs * h->vec_bytes(false));
    h->Xint.ensure(nrhs * h->vec_bytes(false));
    h->R64.ensure(nrhs * h->vec_bytes(false));
    h->Pv.ensure(nrhs * h->vec_bytes(lo));
    h->Qv.ensure(nrhs * h->vec_bytes(lo));
    if (lo) h->Rv.ensure(nrhs * h->vec_bytes(true));
    h->cgv.ensure(nrhs * sizeof(CgVec));
    h->vmap.ensure(nrhs * sizeof(int32_t));
    const int64_t nsb64 = nsb_of(h, false), nsbl = nsb_of(h, lo), nb = norm2_blocks(N);
    h->cgpart.ensure(nrhs * std::max(nsb64, nsbl) * sizeof(double));
    h->rrpart.ensure(nrhs * std::max(nb, nsb64) * sizeof(double));
    h->norms.ensure(2 * nrhs * sizeof(double));
    ensure_work(h, nrhs);
    void* Rw = lo ? h->Rv.p : h->R64.p;  // the recursive residual

    pack_vec(false, B, h->Bint.p, Vh, nrhs, h->s);
    pack_vec(false, X, h->Xint.p, Vh, nrhs, h->s);
    // ||b_j|| and the true residuals of the starting guesses
    norm2_partials(false, h->Bint.p, N, nrhs, h->rrpart.as<double>(), h->s);
    sum_partials(h->rrpart.as<double>(), nb, nrhs, h->norms.as<double>(), true, h->s);
    std::vector<int> all(nrhs);
    for (int j = 0; j < nrhs; j++) all[j] = j;
    true_residual(h, all, h->R64.p, h->cgpart.as<double>());
    sum_partials(h->cgpart.as<double>(), nsb64, nrhs, h->norms.as<double>() + nrhs, false, h->s);
    std::vector<double> hn(2 * nrhs);
    HIPCHK(hipMemcpyAsync(hn.data(), h->norms.p, 2 * nrhs * sizeof(double), hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));

    std::vector<CgVec> cg(nrhs);
    std::vector<int> matvecs(nrhs, 1);
    const double tol = h->p.tol;
    for (int j = 0; j < nrhs; j++) {
        CgVec& c = cg[j];
        c = CgVec{};
        c.bnorm = hn[j];
        c.tol = tol;
        c.rr = hn[nrhs + j];
        c.done = (std::sqrt(c.rr) <= tol * c.bnorm) ? 1 : 0;
    }
    if (lo) convert(false, true, h->R64.p, h->Rv.p, nrhs * N, h->s);
    convert(lo, lo, Rw, h->Pv.p, nrhs * N, h->s);  // p = r
    HIPCHK(hipMemcpyAsync(h->cgv.p, cg.data(), nrhs * sizeof(CgVec), hipMemcpyHostToDevice, h->s));

    const int max_iter = h->p.max_iter > 0 ? h->p.max_iter : 100000;
    // Mixed precision: reliable updates (Sleijpen and van der Vorst) replace the FP32 recursive
    // residual by the FP64 true residual b - M x whenever the recursive residual norm has fallen
    // a decade below the one at the previous replacement, and at least every reliable_every
    // iterations; the host looks every 4 iterations so that FP32 never tracks more than a few
    // decades on its own.
    const int rel_every = lo ? std::max(1, h->p.reliable_every) : 0;
    const int G = lo ? std::min(h->sync_every, 4) : h->sync_every;
    std::vector<int> it_rel(nrhs, 0);
    for (int j = 0; j < nrhs; j++) cg[j].rr_reliable = cg[j].rr;
    std::vector<int> active;
    bool noconv = false;
    for (;;) {
        active.clear();
        for (int j = 0; j < nrhs; j++)
            if (!cg[j].done) active.push_back(j);
        if (active.empty()) break;
        std::vector<int32_t> vm(active.begin(), active.end());
        HIPCHK(hipMemcpyAsync(h->vmap.p, vm.data(), vm.size() * sizeof(int32_t), hipMemcpyHostToDevice, h->s));
        const int nact = (int)vm.size();
        for (int it = 0; it < G; it++) {
            MOpts o;
            o.red = 1;
            o.d = h->Pv.p;
            o.partials = h->cgpart.as<double>();
            o.vec_map = h->vmap.as<int32_t>();
            o.cg = h->cgv.as<CgVec>();
            apply_M_int(h, lo, h->Pv.p, h->Qv.p, nact, o);
            cg_alpha(h->cgv.as<CgVec>(), h->cgpart.as<double>(), nsbl, h->vmap.as<int32_t>(), nact, h->s);
            cg_update(lo, false, h->cgv.as<CgVec>(), h->vmap.as<int32_t>(), nact, h->Xint.p, h->Pv.p, Rw, h->Qv.p,
                      h->rrpart.as<double>(), N, h->s);
            cg_beta(h->cgv.as<CgVec>(), h->rrpart.as<double>(), nb, h->vmap.as<int32_t>(), nact, max_iter, h->s);
            cg_p(lo, h->cgv.as<CgVec>(), h->vmap.as<int32_t>(), nact, h->Pv.p, Rw, N, false, h->s);
        }
        check_launch();
        HIPCHK(hipMemcpyAsync(cg.data(), h->cgv.p, nrhs * sizeof(CgVec), hipMemcpyDeviceToHost, h->s));
        HIPCHK(hipStreamSynchronize(h->s));
        for (int j : active) matvecs[j] = 1 + cg[j].iters;
        if (h->debug)
            for (int j : active)
                fprintf(stderr, "cg j=%d it=%d rr=%.3e a=%.3e b=%.3e pq=%.3e frozen=%d done=%d restarts=%d\n", j, cg[j].iters,
                        cg[j].rr, cg[j].a, cg[j].b, cg[j].pq, cg[j].frozen, cg[j].done, cg[j].restarts);

        // true residual for frozen vectors and, in mixed precision, the reliable updates
        std::vector<int> check;
        std::vector<char> is_rel(nrhs, 0);
        for (int j : active) {
            const bool rel = rel_every && !cg[j].frozen &&
                             (cg[j].rr <= 1e-2 * cg[j].rr_reliable || cg[j].iters - it_rel[j] >= rel_every);
            if (cg[j].frozen || rel) check.push_back(j);
            is_rel[j] = rel;
        }
        if (check.empty()) continue;
        true_residual(h, check, h->R64.p, h->cgpart.as<double>());
        sum_partials(h->cgpart.as<double>(), nsb64, nrhs, h->norms.as<double>() + nrhs, false, h->s);
        HIPCHK(hipMemcpyAsync(hn.data(), h->norms.p, 2 * nrhs * sizeof(double), hipMemcpyDeviceToHost, h->s));
        HIPCHK(hipStreamSynchronize(h->s));
        std::vector<int> restart;
        for (int j : check) {
            CgVec& c = cg[j];
            const double rr = hn[nrhs + j];
            matvecs[j] += 1;
            if (std::sqrt(rr) <= tol * c.bnorm) {
                c.done = 1;
                c.frozen = 0;
                continue;
            }
            if (c.iters >= max_iter || !std::isfinite(rr)) {
                c.done = 1;
                c.frozen = 0;
                noconv = true;
                continue;
            }
            if (c.frozen) {
                // the recursive residual met tol but the true one did not: go on from r = b - M x
                c.b = rr / c.rr;
                c.frozen = 0;
                restart.push_back(j);
            } else if (is_rel[j] && rr >= c.rr_reliable) {
                // no decrease of the true residual since the previous replacement: the inner
                // operator is too far from M for the old directions; restart with p = r
                c.b = 0.0;
                c.restarts += 1;
                restart.push_back(j);
            }
            c.rr_reliable = rr;
            it_rel[j] = c.iters;
            c.rr = rr;
        }
        // r = b - M x in the working precision, then p = r + b p for the restarted ones
        if (lo) {
            for (int j : check)
                if (!cg[j].done)
                    convert(false, true, (char*)h->R64.p + j * h->vec_bytes(false), (char*)h->Rv.p + j * h->vec_bytes(true), N, h->s);
        }
        HIPCHK(hipMemcpyAsync(h->cgv.p, cg.data(), nrhs * sizeof(CgVec), hipMemcpyHostToDevice, h->s));
        if (!restart.empty()) {
            std::vector<int32_t> rm(restart.begin(), restart.end());
            DBuf dm;
            dm.ensure(rm.size() * sizeof(int32_t));
            HIPCHK(hipMemcpyAsync(dm.p, rm.data(), rm.size() * sizeof(int32_t), hipMemcpyHostToDevice, h->s));
            cg_p(lo, h->cgv.as<CgVec>(), dm.as<int32_t>(), (int)rm.size(), h->Pv.p, Rw, N, false, h->s);
            HIPCHK(hipStreamSynchronize(h->s));
        }
    }
    unpack_vec(false, h->Xint.p, X, Vh, nrhs, h->s);
    // final FP64 true residuals for the report
    true_residual(h, all, h->R64.p, h->cgpart.as<double>());
    sum_partials(h->cgpart.as<double>(), nsb64, nrhs, h->norms.as<double>() + nrhs, false, h->s);
    HIPCHK(hipMemcpyAsync(hn.data(), h->norms.p, 2 * nrhs * sizeof(double), hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    if (rep) {
        for (int j = 0; j < nrhs; j++) {
            if (rep->iters) rep->iters[j] = cg[j].iters;
            if (rep->matvecs) rep->matvecs[j] = matvecs[j];
            if (rep->true_relres) rep->true_relres[j] = std::sqrt(hn[nrhs + j]) / hn[j];
        }
        rep->t_rest_s = now_s() - t0;
    }
    return noconv ? SEEDCG_ERR_NOCONV : SEEDCG_OK;
}

seedcg_status fail(seedcg_s* h, seedcg_status code, const std::string& msg) {
    if (h)
        h->err = msg;
    else
        g_create_error = msg;
    return code;
}

template <typename F>
seedcg_status guarded(seedcg_s* h, F&& f) {
    try {
        return f();
    } catch (const ArgError& e) {
        return fail(h, SEEDCG_ERR_ARG, e.what);
    } catch (const StateError& e) {
        return fail(h, SEEDCG_ERR_STATE, e.what);
    } catch (const OomError& e) {
        return fail(h, SEEDCG_ERR_OOM, e.what);
    } catch (const HipError& e) {
        return fail(h, SEEDCG_ERR_HIP, e.what);
    } catch (const std::bad_alloc&) {
        return fail(h, SEEDCG_ERR_OOM, "host allocation failed");
    } catch (...) {
        return fail(h, SEEDCG_ERR_HIP, "unexpected exception");
    }
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------------------
extern "C" {

void seedcg_default_params(seedcg_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->t_bc = -1;
    p->prec = SEEDCG_FP64;
    p->reorth_k = 10;
    p->past_factor = 1.5;
    p->tol = 1e-10;
    p->reliable_every = 50;
    p->seed_block = 32;
    p->max_iter = 100000;
}

seedcg_status seedcg_create(const seedcg_params* p, const double* links, seedcg_t* out) {
    if (!p || !links || !out) return fail(nullptr, SEEDCG_ERR_ARG, "create: null pointer");
    *out = nullptr;
    for (int d = 0; d < 4; d++)
        if (p->dims[d] < 2 || p->dims[d] % 2) return fail(nullptr, SEEDCG_ERR_ARG, "create: every extent must be even and >= 2");
    if (p->t_bc != 1 && p->t_bc != -1) return fail(nullptr, SEEDCG_ERR_ARG, "create: t_bc must be +1 or -1");
    if (p->prec < 0 || p->prec > 2) return fail(nullptr, SEEDCG_ERR_ARG, "create: unknown precision");
    if (!(p->tol > 0.0)) return fail(nullptr, SEEDCG_ERR_ARG, "create: tol must be > 0");
    if (p->reorth_k < 0) return fail(nullptr, SEEDCG_ERR_ARG, "create: reorth_k must be >= 0");
    seedcg_s* h = new (std::nothrow) seedcg_s;
    if (!h) return fail(nullptr, SEEDCG_ERR_OOM, "create: host allocation failed");
    seedcg_status st = guarded(h, [&]() -> seedcg_status {
        h->p = *p;
        h->s = (hipStream_t)p->stream;
        Geom& g = h->g;
        for (int d = 0; d < 4; d++) g.L[d] = p->dims[d];
        g.Lxh = g.L[0] / 2;
        g.V = (int64_t)g.L[0] * g.L[1] * g.L[2] * g.L[3];
        g.Vh = g.V / 2;
        g.t_bc = p->t_bc;
        h->N = 12 * g.Vh;
        h->lo = p->prec != SEEDCG_FP64;
        h->lo_prec = p->prec == SEEDCG_MIXED_FP32 ? P32 : (p->prec == SEEDCG_MIXED_FP32_BF16LINKS ? P32BF : P64);
        // stencil launch shape: 3 = two lanes per site (forward / backward hops), one vector per
        // workgroup; the vectors of a site block run as adjacent workgroups on one XCD
        h->tps64 = env_int("SEEDCG_TPS", 3);
        h->tps_lo = env_int("SEEDCG_TPS_LO", 3);
        if (h->tps64 < 1 || h->tps64 > 4) h->tps64 = 4;
        if (h->tps_lo < 1 || h->tps_lo > 4) h->tps_lo = 4;
        h->sync_every = std::max(1, env_int("SEEDCG_SYNC_EVERY", 16));
        h->debug = env_int("SEEDCG_DEBUG", 0);
        h->vb64 = std::max(1, env_int("SEEDCG_VB", 1));
        h->vb_lo = std::max(1, env_int("SEEDCG_VB_LO", 1));
        h->links64.ensure(4 * g.V * 9 * 16);
        pack_links(P64, g, links, h->links64.p, h->s);
        if (h->lo) {
            h->links_lo.ensure(4 * g.V * 9 * (h->lo_prec == P32 ? 8 : 4));
            pack_links(h->lo_prec, g, links, h->links_lo.p, h->s);
        }
        check_launch();
        HIPCHK(hipStreamSynchronize(h->s));
        return SEEDCG_OK;
    });
    if (st != SEEDCG_OK) {
        g_create_error = h->err;
        delete h;
        return st;
    }
    *out = h;
    return SEEDCG_OK;
}

seedcg_status seedcg_apply_M(seedcg_t h, const double* x, double* y, int32_t nvec) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "apply_M: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (!x || !y || nvec < 1) throw ArgError{"apply_M: null pointer or nvec < 1"};
        if (x == y) throw ArgError{"apply_M: x and y alias"};
        DBuf xi, yi;
        xi.ensure(nvec * h->vec_bytes(false));
        yi.ensure(nvec * h->vec_bytes(false));
        pack_vec(false, x, xi.p, h->g.Vh, nvec, h->s);
        apply_M_int(h, false, xi.p, yi.p, nvec, MOpts{});
        unpack_vec(false, yi.p, y, h->g.Vh, nvec, h->s);
        check_launch();
        HIPCHK(hipStreamSynchronize(h->s));
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_apply_M_inner(seedcg_t h, const double* x, double* y, int32_t nvec) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "apply_M_inner: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (!x || !y || nvec < 1) throw ArgError{"apply_M_inner: null pointer or nvec < 1"};
        if (x == y) throw ArgError{"apply_M_inner: x and y alias"};
        DBuf xi, yi;
        xi.ensure(nvec * h->vec_bytes(h->lo));
        yi.ensure(nvec * h->vec_bytes(h->lo));
        pack_vec(h->lo, x, xi.p, h->g.Vh, nvec, h->s);
        apply_M_int(h, h->lo, xi.p, yi.p, nvec, MOpts{});
        unpack_vec(h->lo, yi.p, y, h->g.Vh, nvec, h->s);
        check_launch();
        HIPCHK(hipStreamSynchronize(h->s));
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_apply_A(seedcg_t h, const double* x, double* y, int32_t nvec, int32_t dagger) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "apply_A: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (!x || !y || nvec < 1) throw ArgError{"apply_A: null pointer or nvec < 1"};
        if (x == y) throw ArgError{"apply_A: x and y alias"};
        DBuf xi, yi;
        xi.ensure(nvec * h->vec_bytes(false));
        yi.ensure(nvec * h->vec_bytes(false));
        pack_vec(false, x, xi.p, h->g.Vh, nvec, h->s);
        apply_A_int(h, xi.p, yi.p, nvec, dagger != 0);
        unpack_vec(false, yi.p, y, h->g.Vh, nvec, h->s);
        check_launch();
        HIPCHK(hipStreamSynchronize(h->s));
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_solve_seed(seedcg_t h, const double* B, double* X, int32_t nrhs, seedcg_report* r) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "solve_seed: null handle");
    return guarded(h, [&]() -> seedcg_status {
        solve_seed_impl(h, B, X, nrhs, r);
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_solve_rest(seedcg_t h, const double* B, double* X, int32_t nrhs, seedcg_report* r) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "solve_rest: null handle");
    return guarded(h, [&]() -> seedcg_status {
        seedcg_status s = solve_rest_impl(h, B, X, nrhs, r);
        if (s == SEEDCG_ERR_NOCONV) h->err = "solve_rest: max_iter reached before tol";
        return s;
    });
}

seedcg_status seedcg_get_tridiag(seedcg_t h, double* alpha, double* beta, int32_t cap, int32_t* m) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "get_tridiag: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (!h->have_seed) throw StateError{"get_tridiag: no seed solve has run"};
        if (!m) throw ArgError{"get_tridiag: null m"};
        *m = h->m_used;
        if (!alpha || !beta) return SEEDCG_OK;
        if (cap < h->m_used) throw ArgError{"get_tridiag: cap < m"};
        const LzArrays A = h->arr();
        HIPCHK(hipMemcpyAsync(alpha, A.alpha + 1, h->m_used * sizeof(double), hipMemcpyDeviceToHost, h->s));
        HIPCHK(hipMemcpyAsync(beta, A.beta, (h->m_used + 1) * sizeof(double), hipMemcpyDeviceToHost, h->s));
        HIPCHK(hipStreamSynchronize(h->s));
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_get_basis_vector(seedcg_t h, int32_t i, double* v) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "get_basis_vector: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (!h->have_seed || !h->basis.p) throw StateError{"get_basis_vector: no basis"};
        if (i < 1 || i > h->m_used || !v) throw ArgError{"get_basis_vector: index out of range or null pointer"};
        const void* src = (const char*)h->basis.p + (int64_t)(i - 1) * h->vec_bytes(h->lo);
        unpack_vec(h->lo, src, v, h->g.Vh, 1, h->s);
        check_launch();
        HIPCHK(hipStreamSynchronize(h->s));
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_project(seedcg_t h, const double* Vv, int32_t nv, const double* R, int32_t nr, int64_t n, double* P) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "project: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (!Vv || !R || !P || nv < 1 || nr < 1 || n < 1) throw ArgError{"project: null pointer or empty size"};
        if (nr > 24) throw ArgError{"project: at most 24 vectors in R"};
        ProjArgs a{};
        a.V = Vv;
        a.ldv = n;
        a.nv = nv;
        for (int j = 0; j < nr; j++) a.R[j] = R + 2 * (int64_t)j * n;
        a.nr = nr;
        a.n = n;
        a.kchunk = kchunk_for(n, std::max<int64_t>(1, 1024 / ((nv + 31) / 32)));
        const int64_t nch = proj_chunks(n, a.kchunk);
        a.part_stride = 2 * (int64_t)nv * nr;
        DBuf part;
        part.ensure(nch * a.part_stride * sizeof(double));
        a.part = part.as<double>();
        project(false, a, (nv + 31) / 32, P, h->s);
        check_launch();
        HIPCHK(hipStreamSynchronize(h->s));
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_update(seedcg_t h, const double* W, int32_t nw, const double* E, double* X, int32_t nx, int64_t n) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "update: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (!W || !E || !X || nw < 1 || nx < 1 || n < 1) throw ArgError{"update: null pointer or empty size"};
        if (nw > 32 || nx > 48) throw ArgError{"update: at most 32 vectors in W and 48 in X"};
        seed_update(false, false, W, nw, E, X, nx, n, nullptr, h->s);
        check_launch();
        HIPCHK(hipStreamSynchronize(h->s));
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_set_timing(seedcg_t h, int32_t sample_every, int32_t max_samples) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "set_timing: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (sample_every < 0 || max_samples < 0) throw ArgError{"set_timing: negative argument"};
        HIPCHK(hipStreamSynchronize(h->s));
        h->timing_every = sample_every;
        h->hop_count = 0;
        h->ev_used = 0;
        h->ev_bytes.clear();
        h->ev_flops.clear();
        h->t_ms = h->t_bytes = h->t_flops = 0.0;
        h->t_launches = 0;
        while ((int)h->ev0.size() < max_samples) {
            hipEvent_t a, b;
            HIPCHK(hipEventCreate(&a));
            HIPCHK(hipEventCreate(&b));
            h->ev0.push_back(a);
            h->ev1.push_back(b);
        }
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_get_timing(seedcg_t h, double* out) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "get_timing: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (!out) throw ArgError{"get_timing: null pointer"};
        HIPCHK(hipStreamSynchronize(h->s));
        for (size_t k = 0; k < h->ev_used; k++) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, h->ev0[k], h->ev1[k]));
            h->t_ms += ms;
            h->t_bytes += h->ev_bytes[k];
            h->t_flops += h->ev_flops[k];
            h->t_launches++;
        }
        h->ev_used = 0;
        h->ev_bytes.clear();
        h->ev_flops.clear();
        out[0] = (double)h->t_launches;
        out[1] = h->t_ms;
        out[2] = h->t_bytes;
        out[3] = h->t_flops;
        out[4] = (double)h->hop_count;
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_release_basis(seedcg_t h) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "release_basis: null handle");
    return guarded(h, [&]() -> seedcg_status {
        HIPCHK(hipStreamSynchronize(h->s));
        h->basis.release();
        h->wring.release();
        h->projpart.release();
        return SEEDCG_OK;
    });
}

void seedcg_destroy(seedcg_t h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->s);
    delete h;
}

const char* seedcg_last_error(seedcg_t h) { return h ? h->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
