// Host runtime and C ABI of the Seed-CG library (Algorithm 1 of the paper and plain CG).
//
// The host only enqueues kernels: every scalar recurrence of Algorithm 1 (alpha, beta,
// delta, gamma, zeta, the eta recurrence of the seeding, the residual estimate, the choice of m)
// lives in device memory and is updated by one-workgroup kernels, so an iteration never
// waits for the host.  The host reads the device state once every `sync_every` steps to
// learn whether the run has ended; kernels of steps beyond the device's m return at once.
//
// The seeding of Eq. (1) is blocked: the projections v_i^dag r_0^j of up to b consecutive steps are one
// MFMA contraction P = V_blk^dag R_0 taken before the reorthogonalisation touches v_i, and the updates
// x^j += eta^j_i w_i of the block are one pass X += W_blk E over a ring of b w-vectors.
// The result is the paper's seeding update exactly, summed in another order.
#include <algorithm>
#include <array>
#include <chrono>
#include <complex>
#include <map>
#include <mutex>
#include <thread>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <numeric>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

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

struct DBuf;
// Sizing pass of a batch: while a plan is open on this thread, ensure() records the largest
// request of every buffer instead of allocating.
struct Plan {
    std::vector<std::pair<DBuf*, size_t>> req;
    void note(DBuf* b, size_t n) {
        for (auto& r : req)
            if (r.first == b) {
                r.second = std::max(r.second, n);
                return;
            }
        req.push_back({b, n});
    }
};
thread_local Plan* g_plan = nullptr;

struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool view = false;  // a slice of a batch arena (configuration 0's copy), not owned
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p && !view) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        view = false;
    }
    void ensure(size_t nbytes) {
        if (g_plan) {
            g_plan->note(this, nbytes == 0 ? 256 : nbytes);
            return;
        }
        if (view) {
            if (nbytes > bytes) throw StateError{"batch buffer smaller than a request (" + std::to_string(nbytes) + " > " +
                                                 std::to_string(bytes) + " bytes)"};
            return;
        }
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

// A named roctx range over the calling scope: the phases of a solve show up as ranges in a
// rocprofv3 --marker-trace run (and cost a function call otherwise).
struct Phase {
    explicit Phase(const char* name) { roctxRangePushA(name); }
    ~Phase() { roctxRangePop(); }
    Phase(const Phase&) = delete;
    Phase& operator=(const Phase&) = delete;
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
    bool own_stream = false;  // batch classes run on a stream of their own
    int device = 0;
    std::string err;
    bool lo = false;        // FP32 Lanczos basis and seeding (mixed precision)
    bool blo = false;       // the stored basis in FP32 (lo, or FP64 Lanczos with an FP32 copy of each vector)
    bool rcopy = false;     // an FP64 basis plus an FP32 copy of it that only the reorthogonalisation reads
    bool cg_lo = false;     // FP32 CG with FP64 reliable updates (every mixed mode; lo implies it)
    Prec lo_prec = P64;     // precision of the inner stencil
    int64_t N = 0;          // complex per vector
    int tps64 = 3, tps_lo = 3;
    int vb64 = 1, vb_lo = 1;      // vectors per stencil workgroup
    int sync_every = 16;
    int debug = 0;
    // stencil launch shapes for several vectors per launch (the CG phase); the single-vector
    // ones above serve the Lanczos steps
    int tps64_multi = 3, tps_lo_multi = 3;
    int vb64_multi = 1, vb_lo_multi = 1;
    bool tuned = false;
    // batch of same-shape configurations: buffers of configuration c at c * cs bytes from
    // configuration 0's, launches over grid.z = ncfg
    int ncfg = 1;
    int64_t cs = 0;
    DBuf arena;
    std::vector<double> kappas;      // per configuration
    DBuf kap2;                       // kappa^2 per configuration (device)
    DBuf stage;                      // compact staging array, ncfg x (largest per-config record)
    DBuf tabs;                       // per-configuration canonical B / X pointers (device)
    DBuf r64, tmap, rmap;            // FP64 start residuals; vector maps of checks and restarts
    // one CG iteration as a hipGraph per active-set width (not used while timing launches)
    bool use_graphs = true;
    bool fuse_cg = true;    // CG update fused into the last stencil launch of q = M p (where the shape has it)
    hipStream_t cap_stream = nullptr;
    std::map<int, hipGraphExec_t> cg_graphs;
    Launch L() const { return Launch(s, ncfg, cs); }

    DBuf links64, links_lo;      // full 3x3 links (FP64; FP32 or BF16 inner)
    DBuf links64r, links_lor;    // two-row copies for the stencil when the field is special unitary
    Prec hop64 = P64, hop_lo = P64;  // link formats the stencil reads
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
    // learned preconditioner P = K K^dag (FP32 weights, FP64 Adam master copy)
    bool k_ready = false;
    bool k_accepted = false;   // K won the judge against plain CG (solve_rest applies it when asked)
    DBuf kW32, kWm, kG, kAm, kAv, kpart, klinks32, kU, kY, kun2, klpart, kS, kfield, pfa, pfb, Zv, rzpart;
    DBuf vring;         // FP64 Lanczos ring (FP32 copy of an FP64 basis)
    DBuf basis32;       // the FP32 copy of the FP64 basis that the reorthogonalisation reads (rcopy)
    // With params.m_max = 0 (one configuration) the basis grows as the Lanczos run needs it, up to
    // m_cap vectors: basis_phys vectors are allocated.
    bool basis_grow = false;
    int64_t basis_phys = 0;
    // deflated CG: W (the lowest Ritz vectors of T lifted by V), Z = M W, (W^dag M W)^{-1},
    // coefficient blocks, Ritz coefficients
    DBuf dW, dZ, dGinv, dP, dE, dS;
    int nev = 0;
    bool defl_stale = true;   // a seed solve ran since W was built
    std::vector<double> ritz_theta;
    int k_steps = 0, k_train_vecs = 0, k_ritz = 0;
    double k_loss0 = 0.0, k_loss1 = 0.0, k_t_train = 0.0;
    // the judge: seconds and iterations of plain CG, PCG with the start K and with the trained K on one
    // system, the seconds of one application of M and of K K^dag to the seeded systems, the predicted
    // cost of each candidate there; the choice (0 plain CG, 1 start K, 2 trained K) and the judged
    // system's starting residual
    std::vector<double> k_judge = std::vector<double>(11, 0.0);
    int k_choice = 0;
    double k_judge_r0 = 0.0;
    // the judge's verdict on deflating plain CG: -1 none (params.deflate decides), 0 off, 1 on
    int judge_defl = -1;
    double k_judge_cg0_it = 0.0, k_judge_cg0_c = 0.0, k_judge_td = 0.0;
    DBuf klossv, kbn, kbt;   // kbt: |u|^2 of the training pairs per band of the Adam steps
    // sampled timing of the stencil launches (hipEvent pairs on the handle's stream)
    int timing_every = 0;
    int64_t hop_count = 0;
    std::vector<hipEvent_t> ev0, ev1;
    std::vector<double> ev_bytes, ev_flops;
    std::vector<std::array<double, 5>> ev_kind;
    std::map<std::array<double, 5>, std::array<double, 3>> t_kind;   // kind -> launches, ms, bytes
    size_t ev_used = 0;
    double t_ms = 0.0, t_bytes = 0.0, t_flops = 0.0;
    double hop_bytes_all = 0.0;   // algorithmic bytes of every stencil launch issued (sampled or not)
    int64_t t_launches = 0;
    ~seedcg_s() {
        for (auto e : ev0) (void)hipEventDestroy(e);
        for (auto e : ev1) (void)hipEventDestroy(e);
        drop_graphs();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (own_stream && s) (void)hipStreamDestroy(s);
    }
    void drop_graphs() {
        for (auto& kv : cg_graphs) (void)hipGraphExecDestroy(kv.second);
        cg_graphs.clear();
    }

    int64_t vec_bytes(bool low) const { return N * (low ? 8 : 16); }
    LzArrays arr() const {
        double* a = arrays.as<double>();
        const int64_t L = (int64_t)m_cap + 2;
        return LzArrays{a, a + L, a + 2 * L, a + 3 * L, a + 4 * L, a + 5 * L};
    }
};

static std::string g_create_error;

// A batch: one strided handle per lattice shape ("class"), each with its own stream.
struct seedcg_batch_s {
    std::vector<seedcg_s*> cls;
    std::vector<std::vector<int>> members;   // class -> configurations
    int ncfg = 0, nrhs = 0;
    hipStream_t user_stream = nullptr;
    std::string err;
    ~seedcg_batch_s() {
        for (auto h : cls) delete h;
    }
};

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
    if (h->cg_lo) {
        h->t1_lo.ensure(n * h->vec_bytes(true));
        h->u_lo.ensure(n * h->vec_bytes(true));
    }
    h->work_vecs = n;
}

const void* hop_links(const seedcg_s* h, bool low) {
    if (low) return h->hop_lo == P32R ? h->links_lor.p : h->links_lo.p;
    return h->hop64 == P64R ? h->links64r.p : h->links64.p;
}

// One stencil launch; when timing is on, every timing_every-th launch is bracketed by events and
// its algorithmic bytes are recorded: links 144 reals per output site (96 in the two-row format;
// read once for the whole batch), and per vector the input and output spinors (24 reals each per site) plus every
// epilogue operand (24 reals per site each).
void hop(seedcg_s* h, Prec pr, const void* L, const void* in, void* out, int par, int nvec, const HopEpi& e, int tps, int vb) {
    const bool sample = h->timing_every > 0 && (h->hop_count % h->timing_every) == 0 && h->ev_used < h->ev0.size();
    h->hop_count++;
    if (sample) HIPCHK(hipEventRecord(h->ev0[h->ev_used], h->s));
    launch_hop(pr, h->g, L, in, out, par, nvec, e, tps, vb, h->L());
    const double sl = (pr == P64 || pr == P64R) ? 8.0 : (pr == P32BF ? 2.0 : 4.0);
    const double ss = (pr == P64 || pr == P64R) ? 8.0 : 4.0;
    const double lr = (pr == P64R || pr == P32R) ? 96.0 : 144.0;   // link reals per site (two rows or all)
    const double Vh = (double)h->g.Vh * h->ncfg;
    // the fused CG update reads u, p, r and the FP64 x and writes r and x instead of out
    const double per = e.red == 3 ? 5.0 * ss + 2.0 * 8.0 : ss * (2 + (e.combine ? 1 : 0) + (e.z ? 1 : 0) + (e.red == 1 ? 1 : 0));
    const double bytes = Vh * lr * sl + (double)nvec * Vh * 24.0 * per;
    h->hop_bytes_all += bytes;
    if (sample) {
        HIPCHK(hipEventRecord(h->ev1[h->ev_used], h->s));
        h->ev_bytes.push_back(bytes);
        h->ev_flops.push_back((double)nvec * Vh * 1320.0);
        // the launch kind: precision and link format, vectors, fused CG update, lanes per site, vectors per workgroup
        h->ev_kind.push_back({(double)pr, (double)nvec, (double)(e.red == 3), (double)tps, (double)vb});
        h->ev_used++;
    }
}

int64_t nsb_for(seedcg_s* h, bool low, int nvec);

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
    CgVec* cg = nullptr;
    // the CG step fused into M p (cg and vec_map set, red 0): |A p|^2 = p^dag M p is reduced on
    // the second hop into partials, alpha = rr / p^dag M p is set between the hops, and the last
    // hop applies x += alpha p, r -= alpha q without storing q, with the |r|^2 partials in rr_part
    bool cg_fused = false;
    void* X = nullptr;
    void* R = nullptr;
    double* rr_part = nullptr;
};

// out = M x for nvec vectors (M = A^dag A = gamma5 A gamma5 A), with the epilogue options on
// the last hop.  low = FP32 vectors with the inner links.
void apply_M_int(seedcg_s* h, bool low, const void* x, void* out, int nvec, const MOpts& o) {
    ensure_work(h, nvec);
    const Prec pr = low ? h->hop_lo : h->hop64;
    const void* L = hop_links(h, low);
    void* t1 = low ? h->t1_lo.p : h->t1_64.p;
    void* u = low ? h->u_lo.p : h->u_64.p;
    const bool multi = nvec > 1;
    const int tps = low ? (multi ? h->tps_lo_multi : h->tps_lo) : (multi ? h->tps64_multi : h->tps64);
    const int vb = low ? (multi ? h->vb_lo_multi : h->vb_lo) : (multi ? h->vb64_multi : h->vb64);
    const double k2 = h->p.kappa * h->p.kappa;
    HopEpi e{};
    e.kappa2_dev = h->kap2.p ? h->kap2.as<double>() : nullptr;  // batch classes: kappa per configuration
    e.gate_m = o.gate_m;
    e.gate_i = o.gate_i;
    e.vec_map = o.vec_map;
    e.cg = o.cg;
    e.sy = 1.0;
    // t1 = H_oe x
    hop(h, pr, L, x, t1, 1, nvec, e, tps, vb);
    // u = gamma5 (x - kappa^2 H_eo t1)
    HopEpi e2 = e;
    e2.combine = 1;
    e2.apply_g5 = 1;
    e2.kappa2 = k2;
    e2.x = x;
    HopEpi e2r = e2;
    if (o.cg_fused) {
        e2r.red = 2;
        e2r.partials = o.partials;
    }
    hop(h, pr, L, t1, u, 0, nvec, e2r, tps, vb);
    if (o.cg_fused) cg_alpha(o.cg, o.partials, nsb_for(h, low, nvec), o.vec_map, nvec, h->L(), false);
    // t1 = H_oe u
    hop(h, pr, L, u, t1, 1, nvec, e, tps, vb);
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
    if (o.cg_fused) {
        e4.red = 3;
        e4.d = x;
        e4.X = o.X;
        e4.R = o.R;
        e4.partials = o.rr_part;
    }
    hop(h, pr, L, t1, out, 0, nvec, e4, tps, vb);
}

// whether the CG step can be fused into M p: launch shapes 8-10 carry that epilogue, and its FP64
// x must be addressable with 32-bit byte offsets within a vector
bool cg_fusable(const seedcg_s* h, bool low, int nvec) {
    const bool multi = nvec > 1;
    const int tps = low ? (multi ? h->tps_lo_multi : h->tps_lo) : (multi ? h->tps64_multi : h->tps64);
    return h->fuse_cg && tps >= 8 && (double)h->g.Vh * 12.0 * 16.0 < 4294967296.0;
}

// y = A x or A^dag x = gamma5 A gamma5 x (FP64)
void apply_A_int(seedcg_s* h, const void* x, void* out, int nvec, bool dagger) {
    ensure_work(h, nvec);
    const double k2 = h->p.kappa * h->p.kappa;
    const void* in = x;
    if (dagger) {  // A^dag = gamma5 A gamma5: the last gamma5 is the hop epilogue's
        gamma5_copy(false, x, h->g5buf.p, h->g.Vh, nvec, h->L());
        in = h->g5buf.p;
    }
    HopEpi e{};
    e.sy = 1.0;
    e.kappa2_dev = h->kap2.p ? h->kap2.as<double>() : nullptr;
    launch_hop(h->hop64, h->g, hop_links(h, false), in, h->t1_64.p, 1, nvec, e, h->tps64, h->vb64, h->L());
    HopEpi e2 = e;
    e2.combine = 1;
    e2.apply_g5 = dagger ? 1 : 0;
    e2.kappa2 = k2;
    e2.x = in;
    launch_hop(h->hop64, h->g, hop_links(h, false), h->t1_64.p, out, 0, nvec, e2, h->tps64, h->vb64, h->L());
}

void check_launch() { HIPCHK(hipGetLastError()); }

// site blocks of the stencil launch that apply_M_int makes for nvec vectors (its reduction
// partials come one per site block), and the largest over every launch shape (allocation)
int64_t nsb_for(seedcg_s* h, bool low, int nvec) {
    const bool multi = nvec > 1;
    return hop_site_blocks(h->g, low ? (multi ? h->tps_lo_multi : h->tps_lo) : (multi ? h->tps64_multi : h->tps64));
}
int64_t nsb_of(seedcg_s* h, bool) { return std::max(hop_site_blocks(h->g, 4), hop_site_blocks(h->g, 9)); }

// host[c * bytes .. ] -> dev (configuration c's copy), for every configuration
void to_cfg(seedcg_s* h, void* dev, const void* host, size_t bytes) {
    if (h->ncfg == 1) {
        HIPCHK(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, h->s));
        return;
    }
    HIPCHK(hipMemcpyAsync(h->stage.p, host, bytes * h->ncfg, hipMemcpyHostToDevice, h->s));
    cfg_copy(h->stage.p, (int64_t)bytes, dev, h->cs, (int64_t)bytes, h->L());
}
// dev (every configuration's copy) -> host[c * bytes ..]; the caller synchronises
void from_cfg(seedcg_s* h, void* host, const void* dev, size_t bytes) {
    if (h->ncfg == 1) {
        HIPCHK(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, h->s));
        return;
    }
    cfg_copy(dev, h->cs, h->stage.p, (int64_t)bytes, (int64_t)bytes, h->L());
    HIPCHK(hipMemcpyAsync(host, h->stage.p, bytes * h->ncfg, hipMemcpyDeviceToHost, h->s));
}
void copy_cfg(seedcg_s* h, void* dst, const void* src, size_t bytes) { cfg_copy(src, h->cs, dst, h->cs, (int64_t)bytes, h->L()); }
void zero_cfg(seedcg_s* h, void* dst, size_t bytes) { cfg_zero(dst, (int64_t)bytes, h->L()); }

// per-configuration lists of vector indices -> a padded [ncfg][width] map on the device (-1 = none);
// returns the width (0 when every list is empty)
int upload_map(seedcg_s* h, DBuf& map, const std::vector<std::vector<int>>& lists) {
    int w = 0;
    for (const auto& l : lists) w = std::max<int>(w, (int)l.size());
    if (w == 0) return 0;
    std::vector<int32_t> m((size_t)h->ncfg * w, -1);
    for (int c = 0; c < h->ncfg; c++)
        for (size_t k = 0; k < lists[c].size(); k++) m[(size_t)c * w + k] = lists[c][k];
    map.ensure(w * sizeof(int32_t));
    to_cfg(h, map.p, m.data(), w * sizeof(int32_t));
    return w;
}

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

// K-chunk of the reorthogonalisation coefficients V_{1..i}^dag [v_i, f]: about 2048 / ceil(i / 32)
// chunks, at least 96.
int64_t reorth_kchunk(int64_t n, int i) {
    const int64_t rowblocks = (i + 31) / 32;
    return kchunk_for(n, std::max<int64_t>(96, 2048 / rowblocks));
}

void alloc_seed(seedcg_s* h, int nrhs) {
    const bool lo = h->lo, blo = h->blo;
    const int64_t N = h->N;
    const int b = seed_block_of(h);
    h->wring.ensure(b * h->vec_bytes(lo));
    h->f.ensure(h->vec_bytes(lo));
    h->x1.ensure(h->vec_bytes(false));
    // the right-hand sides' residuals are projected against the basis in its stored precision
    h->R0.ensure(std::max(1, nrhs - 1) * h->vec_bytes(blo));
    if (blo && !lo) h->vring.ensure(2 * h->vec_bytes(false));   // v_{i-1}, v_i of the FP64 recurrence
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
    h->r64.ensure(nrhs * h->vec_bytes(false));
    ensure_work(h, nrhs);

    // basis capacity: params.m_max, or 3/4 of the free HBM less 4 GiB (at most 8192 vectors); the
    // rest stays free for the CG vectors, the deflation space and the training of the learned K
    int64_t cap = h->p.m_max;
    if (cap <= 0) {
        size_t freeb = 0, total = 0;
        HIPCHK(hipMemGetInfo(&freeb, &total));
        const int64_t reserve = 4LL << 30;
        const int64_t avail = (int64_t)freeb - reserve + (int64_t)h->basis.bytes + (int64_t)h->basis32.bytes;
        const int64_t per = h->vec_bytes(blo) + (h->rcopy ? h->vec_bytes(true) : 0);
        cap = std::max<int64_t>(0, (int64_t)(0.75 * (double)avail) / per);
        cap = std::min<int64_t>(cap, 8192);
        if (cap < 2) throw OomError{"no room for a Krylov basis"};
    }
    h->m_cap = (int32_t)cap;
    const int64_t vb = h->vec_bytes(blo);
    h->basis_grow = h->p.m_max <= 0 && h->ncfg == 1 && !g_plan;
    if (h->basis_grow) {
        // the first 256 vectors now (SEEDCG_BASIS_FIRST), more at the host's checks as the run
        // proceeds (grow_basis)
        const int64_t first = std::min<int64_t>(cap, std::max(2, env_int("SEEDCG_BASIS_FIRST", 256)));
        if ((int64_t)h->basis.bytes < first * vb) h->basis.ensure((size_t)first * vb);
        h->basis_phys = (int64_t)h->basis.bytes / vb;
        if (h->rcopy) {
            const int64_t vb32 = h->vec_bytes(true);
            if ((int64_t)h->basis32.bytes < first * vb32) h->basis32.ensure((size_t)first * vb32);
            h->basis_phys = std::min<int64_t>(h->basis_phys, (int64_t)h->basis32.bytes / vb32);
        }
    } else {
        h->basis.ensure((size_t)cap * vb);
        if (h->rcopy) h->basis32.ensure((size_t)cap * h->vec_bytes(true));
        h->basis_phys = cap;
    }
    h->arrays.ensure(6 * ((int64_t)cap + 2) * sizeof(double));
    h->G.ensure(2 * 2 * ((int64_t)cap + 1) * sizeof(double));
    int64_t part_doubles = proj_chunks(N, kchunk_for(N, 1024)) * 2 * 32 * 24;
    for (int64_t i = 1; i <= cap; i++)
        part_doubles = std::max<int64_t>(part_doubles, proj_chunks(N, reorth_kchunk(N, (int)i)) * 4 * i);
    h->projpart.ensure(part_doubles * sizeof(double));
}

// Makes room for basis slots 0..need-1 (need <= m_cap) at a host check, when no kernel is in flight:
// a larger allocation (twice the current one, or need), the stored vectors copied over, the old one
// freed.  Returns the vectors now allocated; if HBM cannot hold more, the allocation stays as it was
// and the caller caps the run there.
int64_t grow_basis(seedcg_s* h, int64_t need) {
    if (!h->basis_grow || need <= h->basis_phys) return h->basis_phys;
    const int64_t vb = h->vec_bytes(h->blo), vb32 = h->vec_bytes(true);
    const int64_t to = std::min<int64_t>(h->m_cap, std::max<int64_t>(need, 2 * h->basis_phys));
    void *np = nullptr, *np32 = nullptr;
    if (hipMalloc(&np, (size_t)(to * vb)) != hipSuccess) {
        (void)hipGetLastError();
        return h->basis_phys;
    }
    if (h->rcopy && hipMalloc(&np32, (size_t)(to * vb32)) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(np);
        return h->basis_phys;
    }
    HIPCHK(hipMemcpyAsync(np, h->basis.p, (size_t)(h->basis_phys * vb), hipMemcpyDeviceToDevice, h->s));
    if (h->rcopy)
        HIPCHK(hipMemcpyAsync(np32, h->basis32.p, (size_t)(h->basis_phys * vb32), hipMemcpyDeviceToDevice, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    (void)hipFree(h->basis.p);
    h->basis.p = np;
    h->basis.bytes = (size_t)(to * vb);
    if (h->rcopy) {
        (void)hipFree(h->basis32.p);
        h->basis32.p = np32;
        h->basis32.bytes = (size_t)(to * vb32);
    }
    h->basis_phys = to;
    return to;
}

void flush_seed_block(seedcg_s* h, int i0, int i1, int nrhs) {
    if (nrhs <= 1 || i1 < i0) return;
    const bool lo = h->lo, blo = h->blo;
    const int64_t N = h->N;
    const int nb = i1 - i0 + 1, nr = nrhs - 1;
    ProjArgs a{};
    a.V = (const char*)h->basis.p + (int64_t)(i0 - 1) * h->vec_bytes(blo);
    a.ldv = N;
    a.nv = nb;
    for (int j = 0; j < nr; j++) a.R[j] = (const char*)h->R0.p + (int64_t)j * h->vec_bytes(blo);
    a.nr = nr;
    a.n = N;
    a.kchunk = kchunk_for(N, 1024);
    a.part = h->projpart.as<double>();
    a.part_stride = 2 * 32 * 24;
    a.st = h->st.as<LzState>();
    a.gate_i = i0;
    a.rows_from_m = 1;
    a.i0 = i0;
    // an FP32 copy of an FP64 Lanczos basis is contracted on the FP64 matrix cores
    project(blo, a, 1, h->P.as<double>(), h->L(), blo && !lo);
    seed_eta(i0, nb, nr, h->st.as<LzState>(), h->arr().gam, h->P.as<double>(), h->E.as<double>(), h->etaprev.as<double>(),
             h->nvalid.as<int32_t>(), h->L());
    seed_update(lo, false, h->wring.p, nb, h->E.as<double>(), (char*)h->Xint.p + h->vec_bytes(false), nr, N,
                h->nvalid.as<int32_t>(), h->L());
}

// vi: v_i as the recurrence holds it (the basis slot, or the FP64 ring with an FP32 basis copy)
void reorthogonalise(seedcg_s* h, int i, void* vi) {
    const bool lo = h->lo;
    // the basis vectors it reads: the stored basis, or the FP32 copy of an FP64 one; v_i and f are
    // FP32 only in the FP32 Lanczos (lo)
    const bool v32 = h->blo || h->rcopy;
    void* V = h->rcopy ? h->basis32.p : h->basis.p;
    const int64_t N = h->N;
    LzState* st = h->st.as<LzState>();
    const int64_t nb = norm2_blocks(N);
    for (int pass = 1; pass <= 2; pass++) {
        ProjArgs a{};
        a.V = V;
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
        // the reorthogonalisation coefficients, always accumulated in FP64
        reorth_project(v32, lo, a, h->G.as<double>(), h->L());
        reorth_update(lo, i, pass, st, V, N, h->G.as<double>(), vi, h->f.p, h->rpart.as<double>(), h->L(), v32);
        reorth_scalar(i, pass, st, h->rpart.as<double>(), nb, h->G.as<double>(), h->L());
        reorth_finish(lo, i, pass, st, vi, h->f.p, h->f2b.as<double>(), N, h->L());
        reorth_decide(i, pass, st, h->f2a.as<double>(), h->f2b.as<double>(), nb, h->L());
    }
}

// Caller vectors in the canonical layout: one array for a single configuration, or a device table
// of one pointer per configuration for a batch.
struct Io {
    const double* B = nullptr;
    double* X = nullptr;
    const double* const* Btab = nullptr;
    double* const* Xtab = nullptr;
};
void pack_in(seedcg_s* h, const Io& io, bool x, void* dst, int nrhs) {
    if (h->ncfg > 1)
        pack_vec(false, nullptr, dst, h->g.Vh, nrhs, h->L(), x ? (const double* const*)io.Xtab : io.Btab);
    else
        pack_vec(false, x ? io.X : io.B, dst, h->g.Vh, nrhs, h->L());
}
void unpack_out(seedcg_s* h, const Io& io, const void* src, int nrhs) {
    if (h->ncfg > 1)
        unpack_vec(false, src, nullptr, h->g.Vh, nrhs, h->L(), io.Xtab);
    else
        unpack_vec(false, src, io.X, h->g.Vh, nrhs, h->L());
}

// rep: one report per configuration
void solve_seed_impl(seedcg_s* h, const Io& io, int nrhs, seedcg_report* rep) {
    if (nrhs < 1) throw ArgError{"solve_seed: nrhs < 1"};
    if (nrhs > 25) throw ArgError{"solve_seed: at most 25 right-hand sides (24 seeded)"};
    const double t0 = now_s();
    const bool lo = h->lo;
    const int64_t N = h->N;
    const int C = h->ncfg;
    const Launch L = h->L();
    alloc_seed(h, nrhs);
    LzState* st = h->st.as<LzState>();
    const LzArrays A = h->arr();
    const int nr = nrhs - 1;

    pack_in(h, io, false, h->Bint.p, nrhs);
    pack_in(h, io, true, h->Xint.p, nrhs);
    // initial residuals r_0^j = b^j - M x_0^j (FP64), kept in the inner precision for the projections;
    // RHS 1's goes straight to v_1 after scaling.
    h->r64.ensure(nrhs * h->vec_bytes(false));
    {
        MOpts o;
        o.sy = -1.0;
        o.z = h->Bint.p;
        o.cz_host = 1.0;
        apply_M_int(h, false, h->Xint.p, h->r64.p, nrhs, o);
    }
    {
        // a non-finite entry of B or X makes r_0 non-finite: refuse it before any step runs
        const int64_t nbr = norm2_blocks(N);
        norm2_partials(false, h->r64.p, N, nrhs, h->apart.as<double>(), L);
        sum_partials(h->apart.as<double>(), nbr, nrhs, h->P.as<double>(), false, L);
        std::vector<double> r2((size_t)C * nrhs);
        from_cfg(h, r2.data(), h->P.p, nrhs * sizeof(double));
        HIPCHK(hipStreamSynchronize(h->s));
        for (size_t q = 0; q < r2.size(); q++)
            if (!std::isfinite(r2[q]))
                throw ArgError{"solve_seed: right-hand side or starting guess " + std::to_string(q % nrhs) +
                               " holds a non-finite value"};
    }
    if (nr > 0) convert(false, h->blo, (char*)h->r64.p + h->vec_bytes(false), h->R0.p, nr * N, L);
    copy_cfg(h, h->x1.p, h->Xint.p, h->vec_bytes(false));
    zero_cfg(h, h->etaprev.p, 2 * 24 * sizeof(double));
    zero_cfg(h, h->arrays.p, 6 * ((int64_t)h->m_cap + 2) * sizeof(double));

    std::vector<LzState> hs(C);
    for (auto& x : hs) {
        x = LzState{};
        x.m = h->m_cap;
        x.m_cap = h->m_cap;
        x.tol = h->p.tol;
        x.past = h->p.past_factor;
    }
    to_cfg(h, st, hs.data(), sizeof(LzState));
    // Lanczos start: beta_0 = ||r_0^1||, v_1 = r_0^1 / beta_0
    const int64_t nb = norm2_blocks(N);
    norm2_partials(false, h->r64.p, N, 1, h->f2a.as<double>(), L);
    norm2_partials(false, h->Bint.p, N, 1, h->f2a.as<double>() + nb, L);
    lz_start(st, h->f2a.as<double>(), nb, h->f2a.as<double>() + nb, A.beta, L);
    // with an FP32 copy of an FP64 basis, v_{i-1} and v_i live in a two-vector FP64 ring and every
    // finished v_i is rounded into its basis slot
    const bool split = h->blo && !lo;
    auto vcur = [&](int j) -> void* {   // v_j as the recurrence reads it
        return split ? (char*)h->vring.p + (int64_t)((j - 1) & 1) * h->vec_bytes(false)
                     : (char*)h->basis.p + (int64_t)(j - 1) * h->vec_bytes(lo);
    };
    auto store = [&](int j) {   // round v_j into its slot of the FP32 basis, or of the FP32 copy
        if ((split || h->rcopy) && j <= h->m_cap)
            convert(false, true, vcur(j), (char*)(h->rcopy ? h->basis32.p : h->basis.p) + (int64_t)(j - 1) * h->vec_bytes(true), N,
                    L);
    };
    if (lo) {
        convert(false, true, h->r64.p, h->f.p, N, L);
        lz_first_vector(true, st, h->f.p, h->basis.p, N, L);
    } else {
        lz_first_vector(false, st, h->r64.p, vcur(1), N, L);
        store(1);
    }
    check_launch();

    const int b = seed_block_of(h);
    const int k = h->p.reorth_k;
    const int64_t nsb = nsb_for(h, lo, 1);
    int i0 = 1;          // first step of the pending seeding block
    int last_slot = 0;   // ring slot of w_{i-1}
    int i = 1;
    int m_max = 0;       // largest m over the configurations
    bool finished = false;
    while (!finished) {
        int i_end = std::min<int>(h->m_cap, i + h->sync_every - 1);
        if (h->basis_grow && i_end + 1 > h->basis_phys) {
            // this chunk writes basis slots up to i_end (v_{i_end + 1}); the kernels of the last chunk
            // have finished (the state was read back)
            const int64_t have = grow_basis(h, std::min<int64_t>(h->m_cap, (int64_t)i_end + 1));
            if (have < (int64_t)i_end + 1) {
                // HBM is full: the run ends at the allocated capacity
                h->m_cap = (int32_t)have;
                for (auto& x : hs) {
                    x.m_cap = h->m_cap;
                    x.m = std::min(x.m, h->m_cap);
                }
                to_cfg(h, st, hs.data(), sizeof(LzState));
                i_end = std::min<int>(h->m_cap, i + h->sync_every - 1);
            }
        }
        for (; i <= i_end; i++) {
            void* vi = vcur(i);
            const void* vprev = i > 1 ? vcur(i - 1) : nullptr;
            // three-term recurrence: f = M v_i - beta_{i-1} v_{i-1}, alpha_i = v_i^dag f
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
            // alpha_i and the LU row of Eq. (2); f -= alpha_i v_i; w_i; x^1 += zeta_i w_i
            const int slot = i - i0;
            void* wout = (char*)h->wring.p + (int64_t)slot * h->vec_bytes(lo);
            const void* wprev = (const char*)h->wring.p + (int64_t)(slot > 0 ? slot - 1 : last_slot) * h->vec_bytes(lo);
            lz_update(lo, i, st, h->apart.as<double>(), nsb, A, h->f.p, vi, wprev, wout, h->x1.as<double>(), h->f2a.as<double>(),
                      N, L);
            // seeding of Eq. (1), blocked (before the reorthogonalisation can touch v_i)
            const bool reorth_now = k > 0 && i % k == 0;
            if (slot + 1 == b || reorth_now) {
                flush_seed_block(h, i0, i, nrhs);
                last_slot = slot;
                i0 = i + 1;
            }
            // periodic reorthogonalisation
            if (reorth_now) {
                reorthogonalise(h, i, vi);
                store(i);   // the reorthonormalised v_i replaces its rounded copy
            }
            // beta_i and the next Lanczos vector
            lz_beta(i, st, reorth_now ? h->f2b.as<double>() : h->f2a.as<double>(), nb, A, L);
            if (i < h->m_cap) {
                lz_next(lo, i, st, A.beta, h->f.p, vcur(i + 1), N, L);
                store(i + 1);
            }
        }
        check_launch();
        from_cfg(h, hs.data(), st, sizeof(LzState));
        HIPCHK(hipStreamSynchronize(h->s));
        bool all_done = true;
        for (const auto& x : hs) all_done = all_done && x.done;
        if (all_done || i > h->m_cap) finished = true;
    }
    for (const auto& x : hs) m_max = std::max(m_max, (int)x.m);
    // the last (partial) seeding block; configurations that stopped earlier get no rows from it
    if (i0 <= m_max) flush_seed_block(h, i0, std::min(m_max, i - 1), nrhs);
    copy_cfg(h, h->Xint.p, h->x1.p, h->vec_bytes(false));
    unpack_out(h, io, h->Xint.p, nrhs);
    check_launch();
    from_cfg(h, hs.data(), st, sizeof(LzState));
    HIPCHK(hipStreamSynchronize(h->s));
    h->m_used = m_max;
    h->have_seed = true;
    h->defl_stale = true;
    h->judge_defl = -1;
    h->seed_nrhs = nrhs;
    if (rep) {
        // RHS 1's residual estimate after its last step (Eq. 2), per configuration
        std::vector<double> est_m(C, 0.0);
        for (int c = 0; c < C; c++)
            HIPCHK(hipMemcpyAsync(&est_m[c], (const char*)(A.est + std::max(0, (int)hs[c].m)) + (int64_t)c * h->cs,
                                  sizeof(double), hipMemcpyDeviceToHost, h->s));
        HIPCHK(hipStreamSynchronize(h->s));
        const double t = now_s() - t0;
        for (int c = 0; c < C; c++) {
            seedcg_report& r = rep[c];
            r.orth_loss_max = hs[c].orth_loss;
            if (r.est_relres)
                for (int j = 0; j < nrhs; j++) r.est_relres[j] = j == 0 ? est_m[c] : std::nan("");
            r.m_used = hs[c].m;
            r.i_conv = hs[c].i_conv;
            r.seed_status = hs[c].status;
            r.reorth_passes = hs[c].passes;
            r.t_seed_s = t;
            if (r.iters) r.iters[0] = hs[c].m;
            if (r.matvecs)
                for (int j = 0; j < nrhs; j++) r.matvecs[j] = (j == 0 ? hs[c].m : 0) + 1;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// learned preconditioner P = K K^dag
// ---------------------------------------------------------------------------------------------
constexpr int K_LAYERS = 3, K_NW = 9 * 16;   // complex weights per layer
constexpr int K_NREAL = K_LAYERS * K_NW * 2;  // reals updated by Adam

// FP32 links for the transports of K: the inner stencil's two-row copy where the links are special
// unitary and the inner links FP32, else the inner links when they are FP32, else a copy
KLinks k_links(seedcg_s* h) {
    if (h->cg_lo && h->hop_lo == P32R && h->links_lor.p) return {h->links_lor.p, 6};
    if (h->cg_lo && h->lo_prec == P32) return {h->links_lo.p, 9};
    if (!h->klinks32.p) {
        // repack from the FP64 internal copy: same layout, entry by entry
        h->klinks32.ensure(4 * h->g.V * 9 * 8);
        convert(false, true, h->links64.p, h->klinks32.p, 4 * h->g.V * 9, h->s);
    }
    return {h->klinks32.p, 9};
}

const void* k_weights(seedcg_s* h, int layer) { return (const char*)h->kW32.p + (int64_t)layer * K_NW * 8; }

// z = K K^dag r for the vectors of vmap (r and z in the working precision)
void apply_P(seedcg_s* h, bool low, const void* r, void* z, const int32_t* vmap, int nact, int nalloc) {
    const int64_t N = h->N;
    h->pfa.ensure((int64_t)nalloc * 2 * N * 8);
    h->pfb.ensure((int64_t)nalloc * 2 * N * 8);
    const KLinks L = k_links(h);
    k_embed(low, r, h->pfa.p, N, vmap, nact, h->s);
    // K^dag = R_e L_1^dag L_2^dag L_3^dag E_e: the first layer sees an even-only input and the last
    // one's odd outputs are dropped by R_e, so each of K^dag and K costs four half-lattice hops
    k_layer(h->g, L, h->pfa.p, h->pfb.p, k_weights(h, 2), true, vmap, nact, true, h->s, 3);
    k_layer(h->g, L, h->pfb.p, h->pfa.p, k_weights(h, 1), true, vmap, nact, false, h->s, 3);
    k_layer(h->g, L, h->pfa.p, h->pfb.p, k_weights(h, 0), true, vmap, nact, false, h->s, 1);
    // K = R_e L_3 L_2 L_1 E_e (the zero-odd layer reads only the even half of pfb)
    k_layer(h->g, L, h->pfb.p, h->pfa.p, k_weights(h, 0), false, vmap, nact, true, h->s, 3);
    k_layer(h->g, L, h->pfa.p, h->pfb.p, k_weights(h, 1), false, vmap, nact, false, h->s, 3);
    k_layer(h->g, L, h->pfb.p, h->pfa.p, k_weights(h, 2), false, vmap, nact, false, h->s, 1);
    k_restrict(low, h->pfa.p, z, N, vmap, nact, h->s);
}

// Lowest eigenpairs of the symmetric tridiagonal T (diagonal a[0..m), off-diagonal b[0..m-2]) by
// Sturm-sequence bisection and inverse iteration (Wilkinson's classical method).
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
    int cnt = 0;
    double d = 1.0;
    for (size_t i = 0; i < a.size(); i++) {
        d = a[i] - x - (i ? b[i - 1] * b[i - 1] / d : 0.0);
        if (d == 0.0) d = -1e-300;
        if (d < 0.0) cnt++;
    }
    return cnt;
}

void ritz_lowest(const std::vector<double>& a, const std::vector<double>& b, int want, std::vector<double>& lam,
                 std::vector<double>& vecs /* m x nout, row-major */) {
    const int m = (int)a.size();
    double lo = a[0], hi = a[0];
    for (int i = 0; i < m; i++) {
        const double r = (i ? std::fabs(b[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    const double scale = std::max(std::fabs(lo), std::fabs(hi));
    lam.clear();
    std::vector<std::vector<double>> ys;
    for (int k = 0; k < m && (int)lam.size() < want; k++) {
        double l = lo, u = hi;  // the (k+1)-th smallest eigenvalue lies in [l, u]
        for (int it = 0; it < 200 && u - l > 4e-16 * scale; it++) {
            const double mid = 0.5 * (l + u);
            if (sturm_count(a, b, mid) > k) u = mid; else l = mid;
        }
        const double ev = 0.5 * (l + u);
        if (!lam.empty() && std::fabs(ev - lam.back()) <= 1e-8 * std::max(std::fabs(ev), 1e-300)) continue;  // ghost copy
        // inverse iteration with (T - (ev + tiny) I), Thomas algorithm
        std::vector<double> y(m, 1.0 / std::sqrt((double)m)), c(m), d(m), rhs(m);
        const double shift = ev + 1e-12 * scale;
        for (int it = 0; it < 3; it++) {
            for (int i = 0; i < m; i++) d[i] = a[i] - shift;
            rhs = y;
            for (int i = 1; i < m; i++) {
                const double piv = (d[i - 1] == 0.0) ? 1e-300 : d[i - 1];
                const double f = b[i - 1] / piv;
                d[i] -= f * b[i - 1];
                rhs[i] -= f * rhs[i - 1];
            }
            y[m - 1] = rhs[m - 1] / (d[m - 1] == 0.0 ? 1e-300 : d[m - 1]);
            for (int i = m - 2; i >= 0; i--) y[i] = (rhs[i] - b[i] * y[i + 1]) / (d[i] == 0.0 ? 1e-300 : d[i]);
            double nrm = 0.0;
            for (double v : y) nrm += v * v;
            nrm = std::sqrt(nrm);
            for (double& v : y) v /= nrm;
        }
        lam.push_back(ev);
        ys.push_back(y);
    }
    const int nout = (int)lam.size();
    vecs.assign((size_t)m * nout, 0.0);
    for (int j = 0; j < nout; j++)
        for (int i = 0; i < m; i++) vecs[(size_t)i * nout + j] = ys[j][i];
}

// One pass over training pairs off .. off+S-1 of (kU, kY): the loss of those pairs (their mean) and,
// if `backward`, its gradient accumulated into kG.  Returns the loss when `want_loss` (else 0).
// With band_nt > 0 the loss is taken on the even sites of the t-slices [band_t0, band_t0 + band_nt)
// only, and every layer computes just the slices that loss depends on: K K^dag reaches 6 hops, so
// the j-th of the six layers (K^dag's three, then K's) is needed on the band widened by 6 - j slices
// on either side, and the gradient of its output lives there too.
// band_unorm2 (optional, with a band): |u|^2 of the S pairs on the loss band, computed beforehand.
double k_pass(seedcg_s* h, int off, int S, bool backward, bool want_loss, int band_t0 = 0, int band_nt = 0,
              const double* band_unorm2 = nullptr) {
    const int64_t N = h->N;
    const int Lt = h->g.L[3];
    if (band_nt <= 0 || band_nt + 12 >= Lt) band_nt = 0;   // whole lattice
    const int64_t fb = (int64_t)S * 2 * N * 8;
    h->kfield.ensure(8 * fb);
    auto F = [&](int i) { return (void*)((char*)h->kfield.p + i * fb); };
    void *a1 = F(0), *a2 = F(1), *a3 = F(2), *b1 = F(3), *b2 = F(4), *b3 = F(5), *g = F(6), *gt = F(7);
    const void* Uo = (const char*)h->kU.p + (int64_t)off * N * 8;
    const void* Yo = (const char*)h->kY.p + (int64_t)off * N * 8;
    // the block partials of the six weight gradients of a backward pass, one after another
    h->kpart.ensure(6 * 9 * k_grad_blocks(h->g) * 32 * sizeof(double));
    const int64_t nbb = k_band_blocks(h->g, band_t0, band_nt);
    const KLinks L = k_links(h);
    // the band of layer j = 1..6 (the loss band widened by 6 - j slices each side); 0 slices: whole lattice
    auto bt0 = [&](int j) { return band_nt ? band_t0 - (6 - j) : 0; };
    auto bnt = [&](int j) { return band_nt ? band_nt + 2 * (6 - j) : 0; };
    const int64_t nbr = k_residual_blocks(h->g, bt0(6), bnt(6));
    h->klpart.ensure(std::max({norm2_blocks(N), nbr, nbb}) * S * sizeof(double));
    h->kbn.ensure(32 * sizeof(double));
    auto ks = h->s;
    // |u|^2 on the loss band, the loss's normalisation
    const double* unorm2 = band_nt ? band_unorm2 : nullptr;
    if (!unorm2) {
        k_band_norm(h->g, bt0(6), bnt(6), Uo, S, h->klpart.as<double>(), ks);
        sum_partials(h->klpart.as<double>(), nbb, S, h->kbn.as<double>(), false, ks);
        unorm2 = h->kbn.as<double>();
    }
    // forward: a = K^dag chain on E_e y, b = K chain on E_e R_e a3
    // (odd halves that a later step never reads are not computed: pmask 1 = even outputs only).  E_e y
    // is y itself to a layer told that its input is even-only: the first layer and its gradient read
    // the even-site vectors y directly (vector stride N)
    const void* a0 = Yo;
    k_layer(h->g, L, a0, a1, k_weights(h, 2), true, nullptr, S, true, ks, 3, bt0(1), bnt(1), 0, 0, N);
    k_layer(h->g, L, a1, a2, k_weights(h, 1), true, nullptr, S, false, ks, 3, bt0(2), bnt(2));
    k_layer(h->g, L, a2, a3, k_weights(h, 0), true, nullptr, S, false, ks, 1, bt0(3), bnt(3));
    // E_e R_e a3 is a3 itself for every reader: layer 4 and its gradient take an even-only input
    // (zero_odd_input), so they never read the odd half, which layer 3 did not write
    void* b0 = a3;
    k_layer(h->g, L, b0, b1, k_weights(h, 0), false, nullptr, S, true, ks, 3, bt0(4), bnt(4));
    k_layer(h->g, L, b1, b2, k_weights(h, 1), false, nullptr, S, false, ks, 3, bt0(5), bnt(5));
    k_layer(h->g, L, b2, b3, k_weights(h, 2), false, nullptr, S, false, ks, 1, bt0(6), bnt(6));
    k_residual(b3, Uo, unorm2, g, N, S, h->klpart.as<double>(), ks, h->g, bt0(6), bnt(6));
    double loss = 0.0;
    if (want_loss) {
        h->klossv.ensure(32 * sizeof(double));
        sum_partials(h->klpart.as<double>(), nbr, S, h->klossv.as<double>(), false, ks);
        std::vector<double> lv(S);
        HIPCHK(hipMemcpyAsync(lv.data(), h->klossv.p, S * sizeof(double), hipMemcpyDeviceToHost, ks));
        HIPCHK(hipStreamSynchronize(ks));
        for (double v : lv) loss += v;
        loss /= S;
    }
    if (!backward) return loss;
    // backward through K (layers 3, 2, 1) and then K^dag (1^dag, 2^dag, 3^dag): the gradient of layer
    // j's output lives on band j, and each back-propagated field is zero outside its band (the layer
    // that reads it is told so)
    KGradList q{};
    int64_t used = 0;
    auto grad = [&](int layer, const void* gv, const void* in, bool dagger, bool zero_odd, int pmask, int j, int64_t in_vs = 0) {
        double* part = h->kpart.as<double>() + used;
        q.nb[q.n] = k_grad(h->g, L, gv, in, dagger, S, part, ks, zero_odd, pmask, bt0(j), bnt(j), in_vs);
        used += 9 * q.nb[q.n] * 32;
        q.part[q.n] = part;
        q.dagger[q.n] = dagger;
        q.layer[q.n] = layer;
        q.n++;
    };
    grad(2, g, b2, false, false, 1, 6);
    k_layer(h->g, L, g, gt, k_weights(h, 2), true, nullptr, S, true, ks, 3, bt0(5), bnt(5), bt0(6), bnt(6));
    grad(1, gt, b1, false, false, 3, 5);
    k_layer(h->g, L, gt, g, k_weights(h, 1), true, nullptr, S, false, ks, 3, bt0(4), bnt(4), bt0(5), bnt(5));
    grad(0, g, b0, false, true, 3, 4);
    k_layer(h->g, L, g, gt, k_weights(h, 0), true, nullptr, S, false, ks, 1, bt0(3), bnt(3), bt0(4), bnt(4));
    // through E_e R_e: the odd half of gt (not written above) is read by nobody below
    grad(0, gt, a2, true, false, 1, 3);
    k_layer(h->g, L, gt, g, k_weights(h, 0), false, nullptr, S, true, ks, 3, bt0(2), bnt(2), bt0(3), bnt(3));
    grad(1, g, a1, true, false, 3, 2);
    k_layer(h->g, L, g, gt, k_weights(h, 1), false, nullptr, S, false, ks, 3, bt0(1), bnt(1), bt0(2), bnt(2));
    grad(2, gt, a0, true, true, 3, 1, N);
    // the six gradients into kG, per layer in the order above
    k_grad_reduce(q, h->kG.as<double>(), ks);
    return loss;
}

// mean loss over all S training pairs, taken in minibatches of mb
double k_loss_all(seedcg_s* h, int S, int mb) {
    double sum = 0.0;
    for (int off = 0; off < S; off += mb) {
        const int n = std::min(mb, S - off);
        sum += n * k_pass(h, off, n, false, true);
    }
    return sum / S;
}

void k_alloc_weights(seedcg_s* h) {
    h->kWm.ensure(K_NREAL * sizeof(double));
    h->kW32.ensure(K_NREAL * sizeof(float));
    h->kG.ensure(K_NREAL * sizeof(double));
    h->kAm.ensure(K_NREAL * sizeof(double));
    h->kAv.ensure(K_NREAL * sizeof(double));
}

// host weights (FP64 complex, [layer][d][4][4]) -> device FP64 master and FP32 copy
void k_set_weights(seedcg_s* h, const double* w) {
    k_alloc_weights(h);
    std::vector<float> w32(w, w + K_NREAL);
    HIPCHK(hipMemcpyAsync(h->kWm.p, w, K_NREAL * sizeof(double), hipMemcpyHostToDevice, h->s));
    HIPCHK(hipMemcpyAsync(h->kW32.p, w32.data(), K_NREAL * sizeof(float), hipMemcpyHostToDevice, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
}

// The training start: K = 1 + kappa^2 H_eo H_oe, the first term of the Neumann series of A^{-1}
// (section 3: A = 1 - kappa^2 H_eo H_oe).  Each layer has w_0 = 1 and the Wilson hop's spin factors
// w_{+mu} = c (1 - gamma_mu), w_{-mu} = c (1 + gamma_mu) with c = kappa / sqrt(3): through E_e and R_e
// only paths of zero and two hops reach an even site, and three layer pairs carry the two hops.
// (K = 1 with zero hops is a saddle point: every surviving hop path has two hop weights, so no hop
// weight would ever receive a gradient.)
std::vector<double> k_neumann_weights(double kappa) {
    // Euclidean chiral basis, gamma_5 = diag(1, 1, -1, -1): gamma_k = [[0, -i s_k], [i s_k, 0]],
    // gamma_4 = [[0, 1], [1, 0]]; entries as (re, im) over rows a and columns b
    using C = std::complex<double>;
    const C I(0.0, 1.0);
    const C sig[3][2][2] = {{{0.0, 1.0}, {1.0, 0.0}}, {{0.0, -I}, {I, 0.0}}, {{1.0, 0.0}, {0.0, -1.0}}};
    C gam[4][4][4] = {};
    for (int k = 0; k < 3; k++)
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                gam[k][a][2 + b] = -I * sig[k][a][b];
                gam[k][2 + a][b] = I * sig[k][a][b];
            }
    for (int a = 0; a < 2; a++) gam[3][a][2 + a] = gam[3][2 + a][a] = 1.0;
    const double c = kappa / std::sqrt(3.0);
    std::vector<double> w(K_NREAL, 0.0);
    auto put = [&](int l, int d, int a, int b, C v) {
        w[(size_t)l * K_NW * 2 + 2 * (d * 16 + a * 4 + b)] = v.real();
        w[(size_t)l * K_NW * 2 + 2 * (d * 16 + a * 4 + b) + 1] = v.imag();
    };
    for (int l = 0; l < K_LAYERS; l++)
        for (int a = 0; a < 4; a++) {
            put(l, 0, a, a, 1.0);
            for (int mu = 0; mu < 4; mu++)
                for (int b = 0; b < 4; b++) {
                    const C id = a == b ? 1.0 : 0.0;
                    put(l, 1 + mu, a, b, c * (id - gam[mu][a][b]));
                    put(l, 5 + mu, a, b, c * (id + gam[mu][a][b]));
                }
        }
    return w;
}

seedcg_status solve_rest_impl(seedcg_s* h, const Io& io, int nrhs, seedcg_report* rep);
void deflate_step(seedcg_s* h, bool init, const void* R, int nrhs, const int32_t* map, int w, void* X, bool x32, bool use_cg);

// The judge of the learned K (plain Seed-CG is the fallback and the judge): one system (canonical
// layout b, starting guess x0) until its FP64 true relative residual is at most `target`, with the solver of
// solve_rest (deflated when params.deflate asks for it), with or without K.  Returns the wall seconds
// (infinite when it did not get there) and fills the iterations.
// One judge solve of system b from x0 to target: PCG with the current K (use_k) or plain CG, with
// plain CG's deflation off when defl is false (the built deflation is kept for the later solves).
double k_judge_run(seedcg_s* h, bool use_k, const double* b, const double* x0, double* x, double target, int& iters,
                   bool defl = true, int max_it = 0) {
    HIPCHK(hipMemcpyAsync(x, x0, h->vec_bytes(false), hipMemcpyDeviceToDevice, h->s));
    const seedcg_params saved = h->p;
    const bool acc = h->k_accepted;
    const int jd = h->judge_defl, nev = h->nev;
    const std::vector<double> theta = h->ritz_theta;
    auto restore = [&]() {
        h->p = saved;
        h->k_accepted = acc;
        h->judge_defl = jd;
        if (!defl) {
            h->nev = nev;
            h->ritz_theta = theta;
        }
    };
    h->p.precond = use_k ? 1 : 0;
    h->k_accepted = use_k;
    h->judge_defl = defl ? -1 : 0;
    h->p.tol = std::max(h->p.tol, target);
    if (max_it > 0) h->p.max_iter = std::min(h->p.max_iter, max_it);
    Io io;
    io.B = b;
    io.X = x;
    int32_t it = 0;
    double rr = 0.0;
    seedcg_report rep{};
    rep.iters = &it;
    rep.true_relres = &rr;
    const double t0 = now_s();
    seedcg_status st = SEEDCG_OK;
    try {
        st = solve_rest_impl(h, io, 1, &rep);
    } catch (...) {
        restore();
        throw;
    }
    const double t = now_s() - t0;
    restore();
    iters = it;
    return st == SEEDCG_OK ? t : 1e300;
}

// Trains K by `steps` Adam steps from the Neumann start on pairs (u, y = M u) from the last seed
// solve: the n_ritz lowest Ritz vectors of T and n_lanczos stored basis vectors (normalised CG
// residuals) with their components along those Ritz vectors removed.  Minibatches of two pairs.
// Then the judge solves RHS 2 from its seeded guess with plain CG, PCG with the start K and PCG with
// the trained K, and prices each one's iterations with the time of one application of M (and of K K^dag)
// to all the seeded systems; solve_rest applies K only when one of the K candidates is cheaper.
void train_precond_impl(seedcg_s* h, int steps, int n_ritz, int n_lanczos, double lr) {
    if (!h->have_seed || !h->basis.p) throw StateError{"train_precond: needs the basis of a seed solve"};
    if (h->ncfg != 1) throw StateError{"train_precond: one configuration per handle"};
    if (steps < 0 || n_ritz < 0 || n_lanczos < 0 || n_ritz > 16 || n_ritz + n_lanczos > 32 || n_ritz + n_lanczos < 1)
        throw ArgError{"train_precond: 0 <= n_ritz <= 16, 1 <= n_ritz + n_lanczos <= 32, steps >= 0"};
    const double t0 = now_s();
    const int64_t N = h->N;
    const int m = h->m_used;
    if (m < 2) throw StateError{"train_precond: the seed solve took fewer than 2 steps"};
    const LzArrays A = h->arr();
    std::vector<double> alpha(m), beta(m + 1);
    HIPCHK(hipMemcpyAsync(alpha.data(), A.alpha + 1, m * sizeof(double), hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipMemcpyAsync(beta.data(), A.beta, (m + 1) * sizeof(double), hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    std::vector<double> off(beta.begin() + 1, beta.begin() + m), lam, Sv;
    ritz_lowest(alpha, off, std::min(n_ritz, m), lam, Sv);
    const int nr = (int)lam.size();
    const int nl = std::min(n_lanczos, m);
    const int S = nr + nl;
    h->k_ritz = nr;
    h->k_train_vecs = S;
    h->kU.ensure((int64_t)S * N * 8);
    h->kY.ensure((int64_t)S * N * 8);
    if (nr > 0) {
        h->kS.ensure(Sv.size() * sizeof(double));
        HIPCHK(hipMemcpyAsync(h->kS.p, Sv.data(), Sv.size() * sizeof(double), hipMemcpyHostToDevice, h->s));
        k_combine(h->blo, h->basis.p, m, h->kS.as<double>(), nr, h->kU.p, N, h->s);
    }
    for (int j = 0; j < nl; j++) {  // basis vectors (normalised CG residuals), evenly spread over 1..m
        const int i = nl == 1 ? 1 : 1 + (int)((int64_t)j * (m - 1) / (nl - 1));
        convert(h->blo, true, (const char*)h->basis.p + (int64_t)(i - 1) * h->vec_bytes(h->blo), (char*)h->kU.p + (int64_t)(nr + j) * N * 8,
                N, h->s);
    }
    if (nr > 0 && nl > 0) {
        // u -= W (W^dag u) for the basis vectors, W the Ritz vectors (orthonormal to FP32 rounding)
        for (int j0 = 0; j0 < nl; j0 += 24) {
            const int nj = std::min(24, nl - j0);
            ProjArgs a{};
            a.V = h->kU.p;
            a.ldv = N;
            a.nv = nr;
            for (int j = 0; j < nj; j++) a.R[j] = (const char*)h->kU.p + (int64_t)(nr + j0 + j) * N * 8;
            a.nr = nj;
            a.n = N;
            a.kchunk = kchunk_for(N, 1024);
            a.part_stride = 2 * 32 * 24;
            h->projpart.ensure((size_t)proj_chunks(N, a.kchunk) * a.part_stride * sizeof(double));
            a.part = h->projpart.as<double>();
            h->kS.ensure(std::max(Sv.size(), (size_t)2 * 32 * 24) * sizeof(double));
            project(true, a, 1, h->kS.as<double>(), h->s, true);
            std::vector<double> P((size_t)2 * nr * nj);
            HIPCHK(hipMemcpyAsync(P.data(), h->kS.p, P.size() * sizeof(double), hipMemcpyDeviceToHost, h->s));
            HIPCHK(hipStreamSynchronize(h->s));
            for (double& v : P) v = -v;
            HIPCHK(hipMemcpyAsync(h->kS.p, P.data(), P.size() * sizeof(double), hipMemcpyHostToDevice, h->s));
            seed_update(true, true, h->kU.p, nr, h->kS.as<double>(), (char*)h->kU.p + (int64_t)(nr + j0) * N * 8, nj, N, nullptr,
                        h->s);
        }
    }
    // y = M u with the operator the CG iterates with (the inner precision)
    if (h->cg_lo) {
        apply_M_int(h, true, h->kU.p, h->kY.p, S, MOpts{});
    } else {
        DBuf u64, y64;
        u64.ensure((int64_t)S * h->vec_bytes(false));
        y64.ensure((int64_t)S * h->vec_bytes(false));
        convert(true, false, h->kU.p, u64.p, S * N, h->s);
        apply_M_int(h, false, u64.p, y64.p, S, MOpts{});
        convert(false, true, y64.p, h->kY.p, S * N, h->s);
        HIPCHK(hipStreamSynchronize(h->s));
    }
    const int64_t nbn = norm2_blocks(N);
    h->kun2.ensure(S * sizeof(double));
    h->klpart.ensure(std::max<int64_t>(nbn, k_residual_blocks(h->g)) * S * sizeof(double));
    norm2_partials(true, h->kU.p, N, S, h->klpart.as<double>(), h->s);
    sum_partials(h->klpart.as<double>(), nbn, S, h->kun2.as<double>(), false, h->s);
    // weights: the Neumann start; Adam state cleared
    const std::vector<double> w0 = k_neumann_weights(h->p.kappa);
    k_set_weights(h, w0.data());
    HIPCHK(hipMemsetAsync(h->kG.p, 0, K_NREAL * sizeof(double), h->s));
    HIPCHK(hipMemsetAsync(h->kAm.p, 0, K_NREAL * sizeof(double), h->s));
    HIPCHK(hipMemsetAsync(h->kAv.p, 0, K_NREAL * sizeof(double), h->s));
    const int mb = std::min(2, S);
    h->k_loss0 = k_loss_all(h, S, mb);
    // each Adam step takes the loss on a band of two t-slices, the bands stepping through the lattice;
    // the step size decays from lr to 0 on a half cosine, and the full-lattice loss at four checkpoints
    // decides which weights are kept (the start's, unless one of them is lower)
    const int band = 2;
    const int every = std::max(1, (steps + 3) / 4);
    std::vector<double> best = w0;
    double best_loss = h->k_loss0;
    // |u|^2 of every pair on every band the steps visit (the bands start at multiples of gcd(band, Lt)),
    // computed once: kbt[t0][s]
    const int Lt = h->g.L[3];
    const bool banded = band + 12 < Lt;
    if (banded) {
        const int64_t nbb = k_band_blocks(h->g, 0, band);
        h->kbt.ensure((int64_t)Lt * S * sizeof(double));
        h->klpart.ensure(std::max<int64_t>(nbb * S, h->klpart.bytes / sizeof(double)) * sizeof(double));
        for (int t0 = 0; t0 < Lt; t0 += std::gcd(band, Lt)) {
            k_band_norm(h->g, t0, band, h->kU.p, S, h->klpart.as<double>(), h->s);
            sum_partials(h->klpart.as<double>(), nbb, S, h->kbt.as<double>() + (int64_t)t0 * S, false, h->s);
        }
    }
    for (int step = 0; step < steps; step++) {
        const Phase adam_phase("seedcg_train_precond: Adam step");
        const int o = (int)(((int64_t)step * mb) % S);
        const int t0 = (int)(((int64_t)step * band) % Lt);
        k_pass(h, o, std::min(mb, S - o), true, false, t0, band, banded ? h->kbt.as<double>() + (int64_t)t0 * S + o : nullptr);
        const double lr_t = lr * 0.5 * (1.0 + std::cos(M_PI * step / steps));
        k_adam(h->kWm.as<double>(), h->kW32.p, h->kG.as<double>(), h->kAm.as<double>(), h->kAv.as<double>(), step + 1, lr_t, K_NREAL,
               h->s);
        if ((step & 63) == 63) check_launch();
        if ((step + 1) % every == 0 || step + 1 == steps) {
            check_launch();
            const double l = k_loss_all(h, S, mb);
            if (l < best_loss) {
                best_loss = l;
                HIPCHK(hipMemcpyAsync(best.data(), h->kWm.p, K_NREAL * sizeof(double), hipMemcpyDeviceToHost, h->s));
                HIPCHK(hipStreamSynchronize(h->s));
            }
        }
    }
    check_launch();
    k_set_weights(h, best.data());
    h->k_loss1 = best_loss;
    h->kfield.release();
    h->k_steps = steps;
    h->k_ready = true;
    h->k_t_train = now_s() - t0;
    // the judge: time to solve RHS 2 (RHS 1 with one system) to tol from its seeded guess, with each
    // candidate
    std::vector<double> wt(K_NREAL);
    HIPCHK(hipMemcpyAsync(wt.data(), h->kWm.p, K_NREAL * sizeof(double), hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    const int j = std::min(1, h->seed_nrhs - 1);
    DBuf bj, x0, xj;
    bj.ensure(h->vec_bytes(false));
    x0.ensure(h->vec_bytes(false));
    xj.ensure(h->vec_bytes(false));
    unpack_vec(false, (const char*)h->Bint.p + (int64_t)j * h->vec_bytes(false), bj.as<double>(), h->g.Vh, 1, h->L());
    unpack_vec(false, (const char*)h->Xint.p + (int64_t)j * h->vec_bytes(false), x0.as<double>(), h->g.Vh, 1, h->L());
    {
        // its starting FP64 true relative residual
        MOpts o;
        o.sy = -1.0;
        o.z = (const char*)h->Bint.p + (int64_t)j * h->vec_bytes(false);
        o.cz_host = 1.0;
        apply_M_int(h, false, (const char*)h->Xint.p + (int64_t)j * h->vec_bytes(false), h->r64.p, 1, o);
        norm2_partials(false, h->r64.p, N, 1, h->klpart.as<double>(), h->s);
        norm2_partials(false, (const char*)h->Bint.p + (int64_t)j * h->vec_bytes(false), N, 1, h->klpart.as<double>() + nbn, h->s);
        h->klossv.ensure(32 * sizeof(double));
        sum_partials(h->klpart.as<double>(), nbn, 2, h->klossv.as<double>(), true, h->s);
        double nr2[2];
        HIPCHK(hipMemcpyAsync(nr2, h->klossv.p, 2 * sizeof(double), hipMemcpyDeviceToHost, h->s));
        HIPCHK(hipStreamSynchronize(h->s));
        h->k_judge_r0 = nr2[1] > 0.0 ? nr2[0] / nr2[1] : 0.0;
    }
    Phase judge_phase("seedcg_train_precond: judge");
    const double target = h->p.tol;   // the whole solve: K may help early and lose late (near-zero modes)
    int it_cg = 0, it_start = 0, it_trained = 0, it_cg0 = 0;
    // plain CG with the handle's deflation first (it builds the deflation space)
    h->judge_defl = -1;
    const bool defl_cand = h->p.deflate > 0 && h->seed_nrhs - 1 <= 24;
    const double t_cg = k_judge_run(h, false, bj.as<double>(), x0.as<double>(), xj.as<double>(), target, it_cg);
    // solve_rest iterates on all the seeded systems at once, where M's links are shared by every vector
    // and K's cost is not: the judge's iteration counts are priced with the time of one application of M,
    // of K K^dag and of one deflation step to that many vectors
    const int nb = std::max(1, h->seed_nrhs - 1);
    const bool defl_built = defl_cand && h->nev > 0;
    double t_m = 0.0, t_p = 0.0, t_d = 0.0;
    {
        const bool lo = h->cg_lo;
        DBuf xa, ya;
        xa.ensure((int64_t)nb * h->vec_bytes(lo));
        ya.ensure((int64_t)nb * h->vec_bytes(lo));
        cfg_zero(xa.p, (int64_t)nb * h->vec_bytes(lo), h->L());
        hipEvent_t e0, e1, e2, e3;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventCreate(&e2));
        HIPCHK(hipEventCreate(&e3));
        const int saved = h->timing_every;
        h->timing_every = 0;
        apply_M_int(h, lo, xa.p, ya.p, nb, MOpts{});
        apply_P(h, lo, xa.p, ya.p, nullptr, nb, nb);
        constexpr int reps = 4;
        HIPCHK(hipEventRecord(e0, h->s));
        for (int r = 0; r < reps; r++) apply_M_int(h, lo, xa.p, ya.p, nb, MOpts{});
        HIPCHK(hipEventRecord(e1, h->s));
        for (int r = 0; r < reps; r++) apply_P(h, lo, xa.p, ya.p, nullptr, nb, nb);
        HIPCHK(hipEventRecord(e2, h->s));
        // one deflation of a CG iteration: (M W)^dag r on the matrix cores, then p -= W G^{-1} (M W)^dag r
        if (defl_built)
            for (int r = 0; r < reps; r++) deflate_step(h, false, xa.p, nb, nullptr, nb, ya.p, lo, false);
        HIPCHK(hipEventRecord(e3, h->s));
        HIPCHK(hipEventSynchronize(e3));
        h->timing_every = saved;
        float m1 = 0.f, m2 = 0.f, m3 = 0.f;
        HIPCHK(hipEventElapsedTime(&m1, e0, e1));
        HIPCHK(hipEventElapsedTime(&m2, e1, e2));
        HIPCHK(hipEventElapsedTime(&m3, e2, e3));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipEventDestroy(e2);
        (void)hipEventDestroy(e3);
        t_m = 1e-3 * m1 / reps;
        t_p = 1e-3 * m2 / reps;
        t_d = defl_built ? 1e-3 * m3 / reps : 0.0;
        h->kfield.release();
        h->pfa.release();
        h->pfb.release();
    }
    // then plain CG without deflation, stopped once it has run the iterations that would cost as much
    // as the deflated solve (it can no longer win; its count is then a lower bound)
    double t_cg0 = t_cg;
    it_cg0 = it_cg;
    if (defl_cand) {
        const double c_d = t_cg < 1e299 ? it_cg * (t_m + t_d) : 1e300;
        const int cap = c_d < 1e299 && t_m > 0.0 ? (int)std::min(1e9, std::ceil(c_d / t_m)) + 1 : 0;
        t_cg0 = k_judge_run(h, false, bj.as<double>(), x0.as<double>(), xj.as<double>(), target, it_cg0, false, cap);
    }
    const bool moved = best_loss < h->k_loss0;   // otherwise the kept weights are the start's
    double t_trained = 0.0;
    if (moved) t_trained = k_judge_run(h, true, bj.as<double>(), x0.as<double>(), xj.as<double>(), target, it_trained);
    k_set_weights(h, w0.data());
    const double t_start = k_judge_run(h, true, bj.as<double>(), x0.as<double>(), xj.as<double>(), target, it_start);
    if (!moved) {
        t_trained = t_start;
        it_trained = it_start;
    }
    // per iteration on the seeded systems: M; K K^dag for PCG; the deflation where it is applied
    const double c_cg = t_cg < 1e299 ? it_cg * (t_m + t_d) : 1e300;
    const double c_cg0 = t_cg0 < 1e299 ? it_cg0 * t_m : 1e300;
    const double c_start = t_start < 1e299 ? it_start * (t_m + t_p + t_d) : 1e300;
    const double c_trained = t_trained < 1e299 ? it_trained * (t_m + t_p + t_d) : 1e300;
    h->k_judge = {t_cg, t_start, t_trained, (double)it_cg, (double)it_start, (double)it_trained, t_m, t_p, c_cg, c_start, c_trained};
    h->k_judge_cg0_it = it_cg0;
    h->k_judge_cg0_c = c_cg0;
    h->k_judge_td = t_d;
    if (it_trained < it_start || (it_trained == it_start && t_trained <= t_start)) k_set_weights(h, wt.data());
    const double c_k = std::min(c_start, c_trained);
    const double c_plain = std::min(c_cg, c_cg0);
    h->k_choice = c_k < c_plain ? (c_trained <= c_start ? 2 : 1) : 0;
    h->k_accepted = h->k_choice > 0;
    // plain CG (the fallback) deflates only when that was cheaper; PCG always deflates when asked to
    h->judge_defl = defl_cand ? (c_cg <= c_cg0 ? 1 : 0) : -1;
}

// ---------------------------------------------------------------------------------------------
// plain CG on a batch (FP64, or FP32 inner iterations with FP64 reliable updates)
// ---------------------------------------------------------------------------------------------
// r = b - M x (FP64) and its |r|^2 partials for the listed vectors of every configuration
// Returns the number of |r|^2 partials per vector (0 when nothing was listed).
int64_t true_residual(seedcg_s* h, const std::vector<std::vector<int>>& vecs, void* R64, double* part) {
    const int w = upload_map(h, h->tmap, vecs);
    if (w == 0) return 0;
    MOpts o;
    o.sy = -1.0;
    o.z = h->Bint.p;
    o.cz_host = 1.0;
    o.red = 2;
    o.partials = part;
    o.vec_map = h->tmap.as<int32_t>();
    apply_M_int(h, false, h->Xint.p, R64, w, o);
    return nsb_for(h, false, w);
}

void alloc_rest(seedcg_s* h, int nrhs) {
    const bool lo = h->cg_lo;
    h->Bint.ensure(nrhs * h->vec_bytes(false));
    h->Xint.ensure(nrhs * h->vec_bytes(false));
    h->R64.ensure(nrhs * h->vec_bytes(false));
    h->Pv.ensure(nrhs * h->vec_bytes(lo));
    h->Qv.ensure(nrhs * h->vec_bytes(lo));
    if (lo) h->Rv.ensure(nrhs * h->vec_bytes(true));
    h->cgv.ensure(nrhs * sizeof(CgVec));
    h->vmap.ensure(nrhs * sizeof(int32_t));
    h->tmap.ensure(nrhs * sizeof(int32_t));
    h->rmap.ensure(nrhs * sizeof(int32_t));
    const int64_t nsb64 = nsb_of(h, false), nsbl = nsb_of(h, lo), nb = norm2_blocks(h->N);
    h->cgpart.ensure(nrhs * std::max(nsb64, nsbl) * sizeof(double));
    h->rrpart.ensure(nrhs * std::max(nb, std::max(nsb64, nsbl)) * sizeof(double));
    h->norms.ensure(2 * nrhs * sizeof(double));
    ensure_work(h, nrhs);
}

// ---------------------------------------------------------------------------------------------
// deflated CG from the Ritz vectors of the last seed solve (Saad, Yeung, Erhel and Guyomarc'h):
// W = the nev lowest Ritz vectors V s_k of T, Z = M W, G = W^dag Z;  every direction is made
// M-orthogonal to W by p -= W G^{-1} Z^dag r, and the start is x += W G^{-1} W^dag r.
// ---------------------------------------------------------------------------------------------
std::vector<std::complex<double>> invert_hpd(std::vector<std::complex<double>> A, int n) {
    // Gauss-Jordan with partial pivoting (n <= 24)
    std::vector<std::complex<double>> I((size_t)n * n, 0.0);
    for (int i = 0; i < n; i++) I[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; c++) {
        int piv = c;
        for (int r = c + 1; r < n; r++)
            if (std::abs(A[(size_t)r * n + c]) > std::abs(A[(size_t)piv * n + c])) piv = r;
        if (!(std::abs(A[(size_t)piv * n + c]) > 0.0)) throw StateError{"deflation: W^dag M W is singular"};
        for (int k = 0; k < n; k++) {
            std::swap(A[(size_t)c * n + k], A[(size_t)piv * n + k]);
            std::swap(I[(size_t)c * n + k], I[(size_t)piv * n + k]);
        }
        const std::complex<double> d = 1.0 / A[(size_t)c * n + c];
        for (int k = 0; k < n; k++) {
            A[(size_t)c * n + k] *= d;
            I[(size_t)c * n + k] *= d;
        }
        for (int r = 0; r < n; r++)
            if (r != c) {
                const std::complex<double> f = A[(size_t)r * n + c];
                if (f == 0.0) continue;
                for (int k = 0; k < n; k++) {
                    A[(size_t)r * n + k] -= f * A[(size_t)c * n + k];
                    I[(size_t)r * n + k] -= f * I[(size_t)c * n + k];
                }
            }
    }
    return I;
}

ProjArgs defl_proj_args(seedcg_s* h, const void* rows, int nrows, const void* R, int nr) {
    ProjArgs a{};
    a.V = rows;
    a.ldv = h->N;
    a.nv = nrows;
    for (int j = 0; j < nr; j++) a.R[j] = (const char*)R + (int64_t)j * h->vec_bytes(h->cg_lo);
    a.nr = nr;
    a.n = h->N;
    a.kchunk = kchunk_for(h->N, 1024);
    a.part_stride = 2 * 32 * 24;
    // the partials buffer of the seed solve may have been released with the basis; the
    // deflation space outlives it
    h->projpart.ensure((size_t)proj_chunks(h->N, a.kchunk) * a.part_stride * sizeof(double));
    a.part = h->projpart.as<double>();
    return a;
}

// dP = rows^dag R for the deflation: one or two columns (a single system, the judge's solves) on the
// vector units, more on the matrix cores
void defl_project(seedcg_s* h, const ProjArgs& a) {
    const bool lo = h->cg_lo;   // W, M W and the CG vectors share the CG's precision
    if (a.nr <= 2)
        reorth_project(lo, lo, a, h->dP.as<double>(), h->L());
    else
        project(lo, a, 1, h->dP.as<double>(), h->L(), true);
}

// W, Z = M W and G^{-1} from the tridiagonal and basis of the last seed solve (one configuration)
void build_deflation(seedcg_s* h, int want) {
    h->nev = 0;
    h->ritz_theta.clear();
    const int m = h->m_used;
    want = std::min({want, m, 24});
    if (want <= 0 || !h->basis.p) return;
    const bool lo = h->cg_lo;   // W, M W and the CG vectors share the CG's precision
    const int64_t N = h->N;
    const LzArrays A = h->arr();
    std::vector<double> alpha(m), beta(m + 1);
    HIPCHK(hipMemcpyAsync(alpha.data(), A.alpha + 1, m * sizeof(double), hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipMemcpyAsync(beta.data(), A.beta, (m + 1) * sizeof(double), hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    std::vector<double> off(beta.begin() + 1, beta.begin() + m), lam, Sv;
    ritz_lowest(alpha, off, want, lam, Sv);
    const int nev = (int)lam.size();
    if (nev == 0) return;
    h->dW.ensure((int64_t)nev * h->vec_bytes(lo));
    h->dZ.ensure((int64_t)nev * h->vec_bytes(lo));
    // u_k = V s_k, at most 16 per pass
    for (int k0 = 0; k0 < nev; k0 += 16) {
        const int nk = std::min(16, nev - k0);
        std::vector<double> S((size_t)m * nk);
        for (int i = 0; i < m; i++)
            for (int k = 0; k < nk; k++) S[(size_t)i * nk + k] = Sv[(size_t)i * nev + k0 + k];
        h->dS.ensure(S.size() * sizeof(double));
        HIPCHK(hipMemcpyAsync(h->dS.p, S.data(), S.size() * sizeof(double), hipMemcpyHostToDevice, h->s));
        k_combine(h->blo, h->basis.p, m, h->dS.as<double>(), nk, (char*)h->dW.p + (int64_t)k0 * h->vec_bytes(lo), N, h->s, !lo);
        HIPCHK(hipStreamSynchronize(h->s));  // dS is reused by the next pass
    }
    apply_M_int(h, lo, h->dW.p, h->dZ.p, nev, MOpts{});
    h->dP.ensure((size_t)2 * 32 * 24 * sizeof(double));
    h->dE.ensure((size_t)2 * 32 * 24 * sizeof(double));
    h->dGinv.ensure((size_t)2 * nev * nev * sizeof(double));
    project(lo, defl_proj_args(h, h->dW.p, nev, h->dZ.p, nev), 1, h->dP.as<double>(), h->L(), true);
    std::vector<std::complex<double>> G((size_t)nev * nev);
    HIPCHK(hipMemcpyAsync(G.data(), h->dP.p, G.size() * sizeof(std::complex<double>), hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    for (int i = 0; i < nev; i++)   // G is Hermitian: keep its Hermitian part
        for (int j = i; j < nev; j++) {
            const std::complex<double> g = 0.5 * (G[(size_t)i * nev + j] + std::conj(G[(size_t)j * nev + i]));
            G[(size_t)i * nev + j] = g;
            G[(size_t)j * nev + i] = std::conj(g);
        }
    const std::vector<std::complex<double>> Gi = invert_hpd(G, nev);
    HIPCHK(hipMemcpyAsync(h->dGinv.p, Gi.data(), Gi.size() * sizeof(std::complex<double>), hipMemcpyHostToDevice, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    h->nev = nev;
    h->ritz_theta = lam;
}

// init: X += W G^{-1} W^dag R (all nrhs vectors);  otherwise: X -= W G^{-1} Z^dag R for the vectors
// of map (w entries) whose CG record is running.  R in the working precision.
void deflate_step(seedcg_s* h, bool init, const void* R, int nrhs, const int32_t* map, int w, void* X, bool x32,
                  bool use_cg) {
    const bool lo = h->cg_lo;   // W, M W and the CG vectors share the CG's precision
    defl_project(h, defl_proj_args(h, init ? h->dW.p : h->dZ.p, h->nev, R, nrhs));
    defl_mu(h->dGinv.as<double>(), h->dP.as<double>(), h->nev, nrhs, map, w, (init || !use_cg) ? nullptr : h->cgv.as<CgVec>(),
            init ? 1.0 : -1.0, h->dE.as<double>(), h->L());
    seed_update(lo, x32, h->dW.p, h->nev, h->dE.as<double>(), X, nrhs, h->N, nullptr, h->L());
}

// After a residual replacement: r is b - M x again and no longer exactly orthogonal to W; move the
// listed vectors back, x += W G^{-1} W^dag r and r -= Z G^{-1} W^dag r (Z = M W, so r stays b - M x).
void redeflate(seedcg_s* h, void* Rw, int nrhs, const int32_t* map, int w) {
    const bool lo = h->cg_lo;   // W, M W and the CG vectors share the CG's precision
    defl_project(h, defl_proj_args(h, h->dW.p, h->nev, Rw, nrhs));
    defl_mu(h->dGinv.as<double>(), h->dP.as<double>(), h->nev, nrhs, map, w, nullptr, 1.0, h->dE.as<double>(), h->L());
    seed_update(lo, false, h->dW.p, h->nev, h->dE.as<double>(), h->Xint.p, nrhs, h->N, nullptr, h->L());
    defl_mu(h->dGinv.as<double>(), h->dP.as<double>(), h->nev, nrhs, map, w, nullptr, -1.0, h->dE.as<double>(), h->L());
    seed_update(lo, lo, h->dZ.p, h->nev, h->dE.as<double>(), Rw, nrhs, h->N, nullptr, h->L());
}

// One iteration of (preconditioned) CG on the nact vectors of the device map vmap.
void cg_iteration(seedcg_s* h, bool lo, bool pc, int nact, int nalloc, int64_t nb, int max_iter, void* Rw) {
    const Launch L = h->L();
    const int64_t nsbl = nsb_for(h, lo, nact);
    if (!pc && cg_fusable(h, lo, nact)) {
        MOpts o;
        o.vec_map = h->vmap.as<int32_t>();
        o.cg = h->cgv.as<CgVec>();
        o.partials = h->cgpart.as<double>();
        o.cg_fused = true;
        o.X = h->Xint.p;
        o.R = Rw;
        o.rr_part = h->rrpart.as<double>();
        apply_M_int(h, lo, h->Pv.p, h->Qv.p, nact, o);
        cg_beta(h->cgv.as<CgVec>(), h->rrpart.as<double>(), nsbl, h->vmap.as<int32_t>(), nact, max_iter, L);
        cg_p(lo, h->cgv.as<CgVec>(), h->vmap.as<int32_t>(), nact, h->Pv.p, Rw, h->N, false, L);
        if (h->nev) deflate_step(h, false, Rw, nalloc, h->vmap.as<int32_t>(), nact, h->Pv.p, lo, true);
        return;
    }
    MOpts o;
    o.red = 1;
    o.d = h->Pv.p;
    o.partials = h->cgpart.as<double>();
    o.vec_map = h->vmap.as<int32_t>();
    o.cg = h->cgv.as<CgVec>();
    apply_M_int(h, lo, h->Pv.p, h->Qv.p, nact, o);
    cg_alpha(h->cgv.as<CgVec>(), h->cgpart.as<double>(), nsbl, h->vmap.as<int32_t>(), nact, L, pc);
    cg_update(lo, false, h->cgv.as<CgVec>(), h->vmap.as<int32_t>(), nact, h->Xint.p, h->Pv.p, Rw, h->Qv.p, h->rrpart.as<double>(),
              h->N, L);
    if (pc) {
        apply_P(h, lo, Rw, h->Zv.p, h->vmap.as<int32_t>(), nact, nalloc);
        dot_map(lo, Rw, h->Zv.p, h->N, h->vmap.as<int32_t>(), nact, h->cgv.as<CgVec>(), h->rzpart.as<double>(), L);
        cg_beta_pc(h->cgv.as<CgVec>(), h->rrpart.as<double>(), h->rzpart.as<double>(), nb, h->vmap.as<int32_t>(), nact, max_iter, L);
        cg_p(lo, h->cgv.as<CgVec>(), h->vmap.as<int32_t>(), nact, h->Pv.p, h->Zv.p, h->N, false, L);
        // deflated PCG: p = z + b p - W G^{-1} (M W)^dag z
        if (h->nev) deflate_step(h, false, h->Zv.p, nalloc, h->vmap.as<int32_t>(), nact, h->Pv.p, lo, true);
    } else {
        cg_beta(h->cgv.as<CgVec>(), h->rrpart.as<double>(), nb, h->vmap.as<int32_t>(), nact, max_iter, L);
        cg_p(lo, h->cgv.as<CgVec>(), h->vmap.as<int32_t>(), nact, h->Pv.p, Rw, h->N, false, L);
        if (h->nev) deflate_step(h, false, Rw, nalloc, h->vmap.as<int32_t>(), nact, h->Pv.p, lo, true);
    }
}

// The iteration above captured once per active-set width (on a private stream) and replayed on
// the handle's stream: every argument is a fixed device address, the changing active set is
// read from vmap and the scalars from the CgVec records.  It holds kernel nodes only.
hipGraphExec_t cg_graph(seedcg_s* h, bool lo, int nact, int nalloc, int64_t nb, int max_iter, void* Rw) {
    auto it = h->cg_graphs.find(nact);
    if (it != h->cg_graphs.end()) return it->second;
    if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    const hipStream_t saved = h->s;
    h->s = h->cap_stream;
    hipError_t eb = hipStreamBeginCapture(h->s, hipStreamCaptureModeThreadLocal);
    if (eb != hipSuccess) {
        h->s = saved;
        HIPCHK(eb);
    }
    try {
        cg_iteration(h, lo, false, nact, nalloc, nb, max_iter, Rw);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(h->s, &g);
        if (g) (void)hipGraphDestroy(g);
        h->s = saved;
        throw;
    }
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(h->s, &graph);
    h->s = saved;
    HIPCHK(ee);
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPCHK(ei);
    h->cg_graphs[nact] = exec;
    return exec;
}

// rep: one report per configuration
seedcg_status solve_rest_impl(seedcg_s* h, const Io& io, int nrhs, seedcg_report* rep) {
    if (nrhs < 1) throw ArgError{"solve_rest: nrhs < 1"};
    const double t0 = now_s();
    const bool lo = h->cg_lo;
    const int64_t N = h->N;
    const int C = h->ncfg;
    const Launch L = h->L();
    alloc_rest(h, nrhs);
    const int64_t nb = norm2_blocks(N);
    void* Rw = lo ? h->Rv.p : h->R64.p;  // the recursive residual
    // deflated CG from the Ritz vectors of the last seed solve (one configuration); plain CG skips it
    // when the judge of train_precond found it does not pay
    const bool pc_on = h->p.precond && h->k_accepted;
    const bool want_defl = h->p.deflate > 0 && C == 1 && h->have_seed && (pc_on || h->judge_defl != 0);
    // the deflation projections contract all right-hand sides at once (at most 24 columns)
    if (want_defl && nrhs > 24) throw ArgError{"solve_rest: deflated CG takes at most 24 right-hand sides"};
    if (!want_defl)
        h->nev = 0;
    else if (h->defl_stale || h->nev == 0) {
        build_deflation(h, h->p.deflate);
        h->defl_stale = false;
    }
    // buffers may have moved since the graphs were captured
    h->drop_graphs();

    pack_in(h, io, false, h->Bint.p, nrhs);
    pack_in(h, io, true, h->Xint.p, nrhs);
    // ||b_j|| and the true residuals of the starting guesses
    norm2_partials(false, h->Bint.p, N, nrhs, h->rrpart.as<double>(), L);
    sum_partials(h->rrpart.as<double>(), nb, nrhs, h->norms.as<double>(), true, L);
    std::vector<std::vector<int>> all(C);
    for (int c = 0; c < C; c++)
        for (int j = 0; j < nrhs; j++) all[c].push_back(j);
    int64_t np = true_residual(h, all, h->R64.p, h->cgpart.as<double>());
    sum_partials(h->cgpart.as<double>(), np, nrhs, h->norms.as<double>() + nrhs, false, L);
    std::vector<double> hn((size_t)C * 2 * nrhs);   // [c][ ||b_j|| (nrhs), |r_j|^2 (nrhs) ]
    from_cfg(h, hn.data(), h->norms.p, 2 * nrhs * sizeof(double));
    HIPCHK(hipStreamSynchronize(h->s));
    auto bn = [&](int c, int j) { return hn[(size_t)c * 2 * nrhs + j]; };
    auto rr_of = [&](int c, int j) { return hn[(size_t)c * 2 * nrhs + nrhs + j]; };
    for (int c = 0; c < C; c++)
        for (int j = 0; j < nrhs; j++)
            if (!std::isfinite(bn(c, j)) || !std::isfinite(rr_of(c, j)))
                throw ArgError{"solve_rest: right-hand side or starting guess " + std::to_string(j) + " holds a non-finite value"};
    if (h->nev) {
        // the deflated start x += W G^{-1} W^dag r, then the true residuals again
        if (lo) convert(false, true, h->R64.p, h->Rv.p, nrhs * N, L);
        deflate_step(h, true, Rw, nrhs, nullptr, nrhs, h->Xint.p, false, true);
        np = true_residual(h, all, h->R64.p, h->cgpart.as<double>());
        sum_partials(h->cgpart.as<double>(), np, nrhs, h->norms.as<double>() + nrhs, false, L);
        from_cfg(h, hn.data(), h->norms.p, 2 * nrhs * sizeof(double));
        HIPCHK(hipStreamSynchronize(h->s));
    }

    std::vector<CgVec> cg((size_t)C * nrhs);
    std::vector<int> matvecs((size_t)C * nrhs, 1);
    const double tol = h->p.tol;
    for (int c = 0; c < C; c++)
        for (int j = 0; j < nrhs; j++) {
            CgVec& x = cg[(size_t)c * nrhs + j];
            x = CgVec{};
            x.bnorm = bn(c, j);
            x.tol = tol;
            x.rr = rr_of(c, j);
            x.done = (std::sqrt(x.rr) <= tol * x.bnorm) ? 1 : 0;
        }
    if (lo) convert(false, true, h->R64.p, h->Rv.p, nrhs * N, L);
    // preconditioned CG with the learned P = K K^dag when it has been trained and is asked for
    const bool pc = C == 1 && h->p.precond == 1 && h->k_ready && h->k_accepted;
    if (pc) {
        h->Zv.ensure(nrhs * h->vec_bytes(lo));
        h->rzpart.ensure(nrhs * nb * sizeof(double));
        h->respart.ensure(nrhs * sizeof(double));
    }
    // z = P r and rz = Re r^dag z for the vectors in `vecs` (one configuration); returns rz per vector
    auto precondition = [&](const std::vector<int>& vecs) {
        const int w = upload_map(h, h->rmap, {vecs});
        apply_P(h, lo, Rw, h->Zv.p, h->rmap.as<int32_t>(), w, nrhs);
        dot_map(lo, Rw, h->Zv.p, N, h->rmap.as<int32_t>(), w, nullptr, h->rzpart.as<double>(), L);
        sum_partials(h->rzpart.as<double>(), nb, nrhs, h->respart.as<double>(), false, L);
        std::vector<double> rz(nrhs);
        HIPCHK(hipMemcpyAsync(rz.data(), h->respart.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, h->s));
        HIPCHK(hipStreamSynchronize(h->s));
        return rz;
    };
    if (pc) {
        std::vector<int> live;
        for (int j = 0; j < nrhs; j++)
            if (!cg[j].done) live.push_back(j);
        if (!live.empty()) {
            const std::vector<double> rz = precondition(live);
            for (int j : live) cg[j].rz = rz[j];
        }
        convert(lo, lo, h->Zv.p, h->Pv.p, nrhs * N, L);  // p = z
        if (h->nev) deflate_step(h, false, h->Zv.p, nrhs, nullptr, nrhs, h->Pv.p, lo, false);  // p = z - W mu
    } else {
        convert(lo, lo, Rw, h->Pv.p, nrhs * N, L);  // p = r
        if (h->nev) deflate_step(h, false, Rw, nrhs, nullptr, nrhs, h->Pv.p, lo, false);  // p = r - W mu
    }
    // the device records carry rr_reliable too (every round trip copies them back to the host)
    for (auto& x : cg) x.rr_reliable = x.rr;
    to_cfg(h, h->cgv.p, cg.data(), nrhs * sizeof(CgVec));

    const int max_iter = h->p.max_iter > 0 ? h->p.max_iter : 100000;
    // Mixed precision: reliable updates (Sleijpen and van der Vorst) replace the FP32 recursive
    // residual by the FP64 true residual b - M x whenever the recursive residual norm has fallen
    // a decade below the one at the previous replacement, and at least every reliable_every
    // iterations; the host looks every 4 iterations so that FP32 never tracks more than a few
    // decades on its own.
    const int rel_every = lo ? std::max(1, h->p.reliable_every) : 0;
    const int G = lo ? std::min(h->sync_every, 4) : h->sync_every;
    std::vector<int> it_rel((size_t)C * nrhs, 0);
    bool noconv = false;
    const bool graphs = h->use_graphs && h->timing_every == 0 && !pc;
    for (;;) {
        std::vector<std::vector<int>> active(C);
        bool any = false;
        for (int c = 0; c < C; c++)
            for (int j = 0; j < nrhs; j++)
                if (!cg[(size_t)c * nrhs + j].done) {
                    active[c].push_back(j);
                    any = true;
                }
        if (!any) break;
        const int nact = upload_map(h, h->vmap, active);
        if (graphs) {
            const hipGraphExec_t ge = cg_graph(h, lo, nact, nrhs, nb, max_iter, Rw);
            for (int it = 0; it < G; it++) HIPCHK(hipGraphLaunch(ge, h->s));
        } else {
            for (int it = 0; it < G; it++) cg_iteration(h, lo, pc, nact, nrhs, nb, max_iter, Rw);
        }
        check_launch();
        from_cfg(h, cg.data(), h->cgv.p, nrhs * sizeof(CgVec));
        HIPCHK(hipStreamSynchronize(h->s));
        for (int c = 0; c < C; c++)
            for (int j : active[c]) matvecs[(size_t)c * nrhs + j] = 1 + cg[(size_t)c * nrhs + j].iters;
        if (h->debug)
            for (int c = 0; c < C; c++)
                for (int j : active[c]) {
                    const CgVec& x = cg[(size_t)c * nrhs + j];
                    fprintf(stderr, "cg c=%d j=%d it=%d rr=%.3e a=%.3e b=%.3e pq=%.3e frozen=%d done=%d restarts=%d\n", c, j, x.iters,
                            x.rr, x.a, x.b, x.pq, x.frozen, x.done, x.restarts);
                }

        // true residual for frozen vectors and, in mixed precision, the reliable updates
        std::vector<std::vector<int>> check(C);
        std::vector<char> is_rel((size_t)C * nrhs, 0);
        bool any_check = false;
        for (int c = 0; c < C; c++)
            for (int j : active[c]) {
                const size_t q = (size_t)c * nrhs + j;
                const CgVec& x = cg[q];
                const bool rel = rel_every && !x.frozen && (x.rr <= 1e-2 * x.rr_reliable || x.iters - it_rel[q] >= rel_every);
                if (x.frozen || rel) {
                    check[c].push_back(j);
                    any_check = true;
                }
                is_rel[q] = rel;
            }
        if (!any_check) continue;
        np = true_residual(h, check, h->R64.p, h->cgpart.as<double>());
        sum_partials(h->cgpart.as<double>(), np, nrhs, h->norms.as<double>() + nrhs, false, L);
        from_cfg(h, hn.data(), h->norms.p, 2 * nrhs * sizeof(double));
        HIPCHK(hipStreamSynchronize(h->s));
        std::vector<std::vector<int>> restart(C), reload(C);
        for (int c = 0; c < C; c++)
            for (int j : check[c]) {
                const size_t q = (size_t)c * nrhs + j;
                CgVec& x = cg[q];
                const double rr = rr_of(c, j);
                matvecs[q] += 1;
                if (std::sqrt(rr) <= tol * x.bnorm) {
                    if (x.frozen) x.rr = x.pq;   // the recursive |r|^2 at the freeze (the report's estimate)
                    x.done = 1;
                    x.frozen = 0;
                    continue;
                }
                if (x.iters >= max_iter || !std::isfinite(rr)) {
                    if (x.frozen) x.rr = x.pq;
                    x.done = 1;
                    x.frozen = 0;
                    noconv = true;
                    continue;
                }
                reload[c].push_back(j);
                // no decrease of the true residual since the previous replacement, while the recursive
                // residual (x.rr) has run more than a decade below it: the inner operator is too far
                // from M for the old directions.  (Without that gap the stall is CG's own plateau,
                // which a restart would only prolong.)
                const bool stalled = is_rel[q] && rr >= x.rr_reliable && rr > 100.0 * x.rr;
                if (x.frozen) {
                    // the recursive residual (|r|^2 in pq since the freeze) met tol but the true one
                    // did not: go on from r = b - M x with p = r + b p.  When the true residual is more
                    // than a decade above the recursive one, the old direction belongs to a residual
                    // that no longer exists: restart with p = r.
                    x.b = rr <= 100.0 * x.pq ? rr / x.rr : 0.0;
                    x.frozen = 0;
                    restart[c].push_back(j);
                } else if (stalled) {
                    // restart with p = r
                    x.b = 0.0;
                    x.restarts += 1;
                    restart[c].push_back(j);
                }
                x.rr_reliable = rr;
                it_rel[q] = x.iters;
                x.rr = rr;
            }
        // r = b - M x in the working precision, then p = r + b p for the restarted ones
        if (lo) {
            const int w = upload_map(h, h->tmap, reload);
            if (w) convert_map(false, true, h->R64.p, h->Rv.p, N, h->tmap.as<int32_t>(), w, L);
        }
        if (h->nev) {
            const int w = upload_map(h, h->tmap, reload);
            if (w) redeflate(h, Rw, nrhs, h->tmap.as<int32_t>(), w);
        }
        if (pc && !reload[0].empty()) {
            // z = P r and rz = r^dag z for every replaced residual; the direction is kept (as
            // without the preconditioner) except where it restarts with p = z
            const std::vector<double> rz = precondition(reload[0]);
            for (int j : reload[0]) cg[j].rz = rz[j];
            for (int j : restart[0]) cg[j].b = 0.0;
        }
        to_cfg(h, h->cgv.p, cg.data(), nrhs * sizeof(CgVec));
        const int wr = upload_map(h, h->rmap, restart);
        if (wr) cg_p(lo, h->cgv.as<CgVec>(), h->rmap.as<int32_t>(), wr, h->Pv.p, pc ? h->Zv.p : Rw, N, false, L);
        if (wr && h->nev) deflate_step(h, false, pc ? h->Zv.p : Rw, nrhs, h->rmap.as<int32_t>(), wr, h->Pv.p, lo, true);
    }
    unpack_out(h, io, h->Xint.p, nrhs);
    // final FP64 true residuals for the report
    np = true_residual(h, all, h->R64.p, h->cgpart.as<double>());
    sum_partials(h->cgpart.as<double>(), np, nrhs, h->norms.as<double>() + nrhs, false, L);
    from_cfg(h, hn.data(), h->norms.p, 2 * nrhs * sizeof(double));
    HIPCHK(hipStreamSynchronize(h->s));
    if (rep) {
        const double t = now_s() - t0;
        for (int c = 0; c < C; c++) {
            seedcg_report& r = rep[c];
            for (int j = 0; j < nrhs; j++) {
                const size_t q = (size_t)c * nrhs + j;
                if (r.iters) r.iters[j] = cg[q].iters;
                if (r.matvecs) r.matvecs[j] = matvecs[q];
                if (r.true_relres) r.true_relres[j] = std::sqrt(rr_of(c, j)) / bn(c, j);
                if (r.est_relres) r.est_relres[j] = std::sqrt(std::max(0.0, cg[q].rr)) / bn(c, j);
            }
            r.t_rest_s = t;
            r.t_train_s = pc ? h->k_t_train : 0.0;
        }
    }
    return noconv ? SEEDCG_ERR_NOCONV : SEEDCG_OK;
}

// ---------------------------------------------------------------------------------------------
// handle set-up, stencil autotuning and the batch arena
// ---------------------------------------------------------------------------------------------
void init_geometry(seedcg_s* h, const seedcg_params* p, const int32_t* dims) {
    h->p = *p;
    for (int d = 0; d < 4; d++) h->p.dims[d] = dims[d];
    Geom& g = h->g;
    for (int d = 0; d < 4; d++) g.L[d] = dims[d];
    g.Lxh = g.L[0] / 2;
    g.V = (int64_t)g.L[0] * g.L[1] * g.L[2] * g.L[3];
    g.Vh = g.V / 2;
    g.t_bc = p->t_bc;
    h->N = 12 * g.Vh;
    h->lo = p->prec == SEEDCG_MIXED_FP32 || p->prec == SEEDCG_MIXED_FP32_BF16LINKS;
    h->blo = h->lo || p->basis_fp32 == 1;
    h->rcopy = !h->lo && p->basis_fp32 == 2;
    h->cg_lo = p->prec != SEEDCG_FP64;
    h->lo_prec = p->prec == SEEDCG_MIXED_FP32_BF16LINKS ? P32BF : (h->cg_lo ? P32 : P64);
    // default stencil launch shape: 8 = forward and backward hops on separate wavefronts, one vector
    // per workgroup (the autotuner may pick another); the vectors of a site block run as adjacent
    // workgroups on one XCD
    h->tps64 = env_int("SEEDCG_TPS", 8);
    h->tps_lo = env_int("SEEDCG_TPS_LO", 8);
    if (h->tps64 < 1 || h->tps64 > 12) h->tps64 = 8;
    if (h->tps_lo < 1 || h->tps_lo > 12) h->tps_lo = 8;
    h->vb64 = std::max(1, env_int("SEEDCG_VB", 1));
    h->vb_lo = std::max(1, env_int("SEEDCG_VB_LO", 1));
    // the several-vector launches take the same shape unless the environment names one of their own
    h->tps64_multi = env_int("SEEDCG_TPS_MULTI", h->tps64);
    h->tps_lo_multi = env_int("SEEDCG_TPS_LO_MULTI", h->tps_lo);
    if (h->tps64_multi < 1 || h->tps64_multi > 12) h->tps64_multi = h->tps64;
    if (h->tps_lo_multi < 1 || h->tps_lo_multi > 12) h->tps_lo_multi = h->tps_lo;
    h->vb64_multi = std::max(1, env_int("SEEDCG_VB_MULTI", h->vb64));
    h->vb_lo_multi = std::max(1, env_int("SEEDCG_VB_LO_MULTI", h->vb_lo));
    h->sync_every = std::max(1, env_int("SEEDCG_SYNC_EVERY", 16));
    h->debug = env_int("SEEDCG_DEBUG", 0);
    h->use_graphs = env_int("SEEDCG_GRAPHS", 1) != 0;
    h->fuse_cg = env_int("SEEDCG_FUSE_CG", 1) != 0;
    HIPCHK(hipGetDevice(&h->device));
}

// Largest distance of a link from SU(3) as the two-row format sees it (canonical FP64 links on the
// device); the stencil reads two-row links only when this is at rounding level.
double su3_defect_max(seedcg_s* h, const double* links) {
    const int64_t nl = 4 * h->g.V;
    const int64_t nb = su3_defect_blocks(nl);
    DBuf part;
    part.ensure(nb * sizeof(double));
    su3_defect(links, nl, part.as<double>(), h->s);
    std::vector<double> v(nb);
    HIPCHK(hipMemcpyAsync(v.data(), part.p, nb * sizeof(double), hipMemcpyDeviceToHost, h->s));
    HIPCHK(hipStreamSynchronize(h->s));
    double m = 0.0;
    for (double x : v) m = std::max(m, x);
    return m;
}
constexpr double SU3_DEFECT_TOL = 1e-12;

// link formats of the stencil: two rows when allowed and the field is special unitary
void choose_link_formats(seedcg_s* h, bool special_unitary) {
    const bool rows2 = special_unitary && env_int("SEEDCG_LINK_ROWS", 2) != 9;
    h->hop64 = rows2 ? P64R : P64;
    h->hop_lo = h->lo_prec == P32 ? (rows2 ? P32R : P32) : h->lo_prec;
    // launch shapes taken from the environment must fit this lattice (else the default one)
    auto fit = [h](int& tps, int& vb, Prec pr) {
        if (!hop_shape_ok(h->g, pr, tps, vb)) tps = 3, vb = 1;   // 3 fits every lattice
    };
    fit(h->tps64, h->vb64, h->hop64);
    fit(h->tps64_multi, h->vb64_multi, h->hop64);
    fit(h->tps_lo, h->vb_lo, h->hop_lo);
    fit(h->tps_lo_multi, h->vb_lo_multi, h->hop_lo);
}

bool env_shape_fixed() {
    for (const char* k : {"SEEDCG_TPS", "SEEDCG_TPS_LO", "SEEDCG_VB", "SEEDCG_VB_LO", "SEEDCG_TPS_MULTI", "SEEDCG_TPS_LO_MULTI",
                          "SEEDCG_VB_MULTI", "SEEDCG_VB_LO_MULTI"})
        if (getenv(k)) return true;
    return false;
}

// Process-wide cache of tuned launch shapes: (Lx, Ly, Lz, Lt, precision, configurations, nvec).
std::mutex g_tune_mu;
std::map<std::vector<int>, std::pair<int, int>> g_tune;

// Times M on nvec vectors for every candidate launch shape of the stencil (lanes per site and
// vectors per workgroup) and keeps the fastest for this width class (one vector: the Lanczos
// steps; several: the CG iterations).  x, y: nvec vectors of the precision `low` (all configurations).
void tune_shape(seedcg_s* h, bool low, int nvec, const void* x, void* y) {
    const bool multi = nvec > 1;
    int& tps = low ? (multi ? h->tps_lo_multi : h->tps_lo) : (multi ? h->tps64_multi : h->tps64);
    int& vb = low ? (multi ? h->vb_lo_multi : h->vb_lo) : (multi ? h->vb64_multi : h->vb64);
    const std::vector<int> key{h->g.L[0], h->g.L[1], h->g.L[2], h->g.L[3], low ? (int)h->hop_lo : (int)h->hop64, h->ncfg, nvec};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            tps = it->second.first;
            vb = it->second.second;
            return;
        }
    }
    std::vector<std::pair<int, int>> cand{{10, 1}, {12, 1}, {9, 1}, {8, 1}, {3, 1}, {5, 1}, {6, 1}, {4, 1}, {2, 1}, {1, 1}};
    if (multi) {
        cand.push_back({9, 2});                 // staged x/y neighbours, links once per pair / quad
        cand.push_back({9, 4});
        cand.push_back({8, 2});                 // wave-split, links once per pair / quad of vectors
        cand.push_back({8, 4});
        cand.push_back({4, 2});
        cand.push_back({4, 4});
        cand.push_back({7, 2});                 // links once per pair of vectors
        if (low) cand.push_back({7, 4});        // (four FP64 vectors do not fit in registers)
        cand.push_back({11, 1});                // links once per launch, the vectors streamed
        cand.push_back({11, 2});
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best = 1e30f;
    std::pair<int, int> pick{tps, vb};
    const int timing_saved = h->timing_every;
    h->timing_every = 0;
    try {
        for (const auto& c : cand) {
            if (!hop_shape_ok(h->g, low ? h->hop_lo : h->hop64, c.first, c.second)) continue;
            tps = c.first;
            vb = c.second;
            apply_M_int(h, low, x, y, nvec, MOpts{});  // warm-up
            HIPCHK(hipEventRecord(e0, h->s));
            for (int r = 0; r < 3; r++) apply_M_int(h, low, x, y, nvec, MOpts{});
            HIPCHK(hipEventRecord(e1, h->s));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            // a later candidate must win by 3%: shapes within timing noise of each other (the
            // one-vector FP64 shapes often are) then resolve to the same pick in every process
            if (ms < 0.97f * best || best == 1e30f) {
                best = ms;
                pick = c;
            }
        }
    } catch (...) {
        h->timing_every = timing_saved;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    h->timing_every = timing_saved;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    tps = pick.first;
    vb = pick.second;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = pick;
}

// Tunes the inner-precision shapes of a single-configuration handle on scratch vectors.
void autotune_single(seedcg_s* h, int nvec_multi) {
    if (!h->p.autotune || env_shape_fixed()) return;
    // one vector in the Lanczos precision, several in the CG precision
    const bool low = h->cg_lo;
    DBuf x, y;
    x.ensure(nvec_multi * h->vec_bytes(false));   // large enough for either precision
    y.ensure(nvec_multi * h->vec_bytes(false));
    ensure_work(h, nvec_multi);
    cfg_zero(x.p, nvec_multi * h->vec_bytes(false), h->L());
    tune_shape(h, h->lo, 1, x.p, y.p);
    tune_shape(h, low, nvec_multi, x.p, y.p);
    if (low) {   // the FP64 stencil of the true residuals and reliable updates (several vectors)
        x.ensure(nvec_multi * h->vec_bytes(false));
        y.ensure(nvec_multi * h->vec_bytes(false));
        cfg_zero(x.p, nvec_multi * h->vec_bytes(false), h->L());
        tune_shape(h, false, nvec_multi, x.p, y.p);
    }
    HIPCHK(hipStreamSynchronize(h->s));
    h->tuned = true;
}

// Bytes one configuration of a batch class needs with basis capacity m_cap, and (optionally) the
// buffers with their sizes, from a sizing pass through the allocation code.
size_t plan_layout(seedcg_s* h, int nrhs, int m_cap, std::vector<std::pair<DBuf*, size_t>>* out) {
    Plan pl;
    g_plan = &pl;
    h->p.m_max = m_cap;
    h->work_vecs = 0;
    try {
        h->links64.ensure(4 * h->g.V * 9 * 16);
        if (h->cg_lo) h->links_lo.ensure(4 * h->g.V * 9 * (h->lo_prec == P32 ? 8 : 4));
        if (h->hop64 == P64R) h->links64r.ensure(4 * h->g.V * 6 * 16);
        if (h->hop_lo == P32R) h->links_lor.ensure(4 * h->g.V * 6 * 8);
        h->kap2.ensure(sizeof(double));
        alloc_seed(h, nrhs);
        alloc_rest(h, nrhs);
    } catch (...) {
        g_plan = nullptr;
        throw;
    }
    g_plan = nullptr;
    h->work_vecs = 0;
    size_t off = 0;
    for (const auto& r : pl.req) off = (off + 255) / 256 * 256 + r.second;
    if (out) *out = pl.req;
    return (off + 4095) / 4096 * 4096;
}

void apply_layout(seedcg_s* h, int nrhs, int m_cap) {
    std::vector<std::pair<DBuf*, size_t>> req;
    const size_t per = plan_layout(h, nrhs, m_cap, &req);
    h->arena.ensure(per * (size_t)h->ncfg);
    size_t off = 0;
    for (const auto& r : req) {
        off = (off + 255) / 256 * 256;
        r.first->release();
        r.first->p = (char*)h->arena.p + off;
        r.first->bytes = r.second;
        r.first->view = true;
        off += r.second;
    }
    h->cs = (int64_t)per;
    h->p.m_max = m_cap;
    h->m_cap = m_cap;
    const size_t rec = std::max({sizeof(LzState), (size_t)nrhs * sizeof(CgVec), (size_t)nrhs * 2 * sizeof(double),
                                 (size_t)nrhs * sizeof(int32_t)});
    h->stage.ensure(rec * h->ncfg);
    h->tabs.ensure(2 * sizeof(void*) * h->ncfg);
}

// ---------------------------------------------------------------------------------------------
// The indefinite system H x = gamma5 phi, H = gamma5 A (section 2: a QR factorisation of the
// Lanczos matrix replaces the LU for indefinite matrices).  RHS 1 runs Lanczos on H with the
// MINRES form of that QR (Givens rotations of the (i+1) x i Lanczos matrix), past convergence and
// with periodic reorthogonalisation as in Algorithm 1; every other RHS is seeded from the same
// Lanczos vectors by the minimal-residual projection (the rotations applied to V^dag r_0^j); plain
// MINRES then finishes every system.  FP64 throughout; the scalar recurrences run on the host.
// ---------------------------------------------------------------------------------------------

// out = H x = gamma5 (x - kappa^2 H_eo H_oe x) for the vectors listed in vmap (or the first nvec);
// with d, the partials of Re d^dag out per vector
// (nslots: vectors in x and out, the largest index vmap may list + 1)
void apply_H_int(seedcg_s* h, const void* x, void* out, int nvec, int nslots, const int32_t* vmap, const void* d, double* partials) {
    ensure_work(h, std::max(nvec, nslots));
    const bool multi = nvec > 1;
    const int tps = multi ? h->tps64_multi : h->tps64;
    const int vb = multi ? h->vb64_multi : h->vb64;
    HopEpi e{};
    e.sy = 1.0;
    e.vec_map = vmap;
    const void* L = hop_links(h, false);
    hop(h, h->hop64, L, x, h->t1_64.p, 1, nvec, e, tps, vb);
    HopEpi e2 = e;
    e2.combine = 1;
    e2.apply_g5 = 1;
    e2.kappa2 = h->p.kappa * h->p.kappa;
    e2.x = x;
    e2.red = d ? 1 : 0;
    e2.d = d;
    e2.partials = partials;
    hop(h, h->hop64, L, h->t1_64.p, out, 0, nvec, e2, tps, vb);
}

struct Givens {
    double c = 1.0, s = 0.0;
};

// One column of the QR of the Lanczos matrix: beta_{i-1}, alpha_i, beta_i with the two previous
// rotations g2 = G_{i-2}, g1 = G_{i-1}; returns G_i and rho_i, delta_i, eps_i
struct QrCol {
    Givens g;
    double rho, delta, eps;
};
QrCol qr_column(double bprev, double a, double b, const Givens& g2, const Givens& g1) {
    QrCol q;
    q.eps = g2.s * bprev;
    const double dbar = g2.c * bprev;
    q.delta = g1.c * dbar + g1.s * a;
    const double gbar = -g1.s * dbar + g1.c * a;
    q.rho = std::hypot(gbar, b);
    if (q.rho > 0.0) {
        q.g.c = gbar / q.rho;
        q.g.s = b / q.rho;
    }
    return q;
}

struct IndefWork {
    DBuf V, C, X, R0, Hb, F, W, Va, Vb, Wa, Wb, Wc, part, hpart, scal, P, E, pp, vmap;
};

// returns false when some system reached max_iter before tol (X then holds its last iterate)
bool solve_indefinite_impl(seedcg_s* h, const double* Phi, double* Xout, int nrhs, seedcg_report* rep) {
    using cxd = std::complex<double>;
    if (h->cg_lo) throw StateError{"solve_indefinite: FP64 handles only"};
    if (h->ncfg != 1) throw StateError{"solve_indefinite: one configuration per handle"};
    if (nrhs < 1 || nrhs > 25) throw ArgError{"solve_indefinite: 1 <= nrhs <= 25"};
    const double t0 = now_s();
    const int64_t N = h->N;
    const int64_t vbytes = h->vec_bytes(false);
    const hipStream_t s = h->s;
    const Launch L = h->L();
    const double tol = h->p.tol;
    const int k = h->p.reorth_k;
    const int max_iter = h->p.max_iter;
    int m_cap = h->p.m_max;
    if (m_cap <= 0) {
        size_t freeb = 0, total = 0;
        HIPCHK(hipMemGetInfo(&freeb, &total));
        const double room = 0.75 * ((double)freeb - 4.0 * (1 << 30) - 10.0 * nrhs * vbytes);
        m_cap = (int)std::min<double>(4096.0, std::max(2.0, room / (double)vbytes));
    }
    IndefWork wk;
    wk.V.ensure((size_t)(m_cap + 1) * vbytes);
    for (DBuf* b : {&wk.C, &wk.X, &wk.R0, &wk.Hb, &wk.Va, &wk.Vb, &wk.Wa, &wk.Wb, &wk.Wc}) b->ensure((size_t)nrhs * vbytes);
    wk.F.ensure(vbytes);
    constexpr int WB = 32;   // seeding updates X += W_blk E_blk every WB steps (section 2's x^j updates, blocked)
    wk.W.ensure(WB * vbytes);
    const int64_t nb = zdots_blocks(N);
    wk.part.ensure((size_t)2 * 32 * nb * sizeof(double));
    const int64_t nsb = nsb_of(h, false);
    wk.hpart.ensure((size_t)nrhs * nsb * sizeof(double));
    wk.scal.ensure(256 * sizeof(double));
    wk.vmap.ensure(32 * sizeof(int32_t));
    auto vec = [&](const DBuf& b, int j) { return (void*)((char*)b.p + (int64_t)j * vbytes); };
    auto vcol = [&](int i) { return (void*)((char*)wk.V.p + (int64_t)i * vbytes); };   // v_{i+1}, 0-based
    double* scal = wk.scal.as<double>();
    auto sync = [&]() { HIPCHK(hipStreamSynchronize(s)); };
    auto dots = [&](const std::vector<const void*>& a, const std::vector<const void*>& b) {
        const int np = (int)a.size();
        std::vector<cxd> out(np);
        std::vector<double> raw(2 * np);
        for (int q = 0; q < np; q += 128) {
            const int cnt = std::min(128, np - q);
            zdots(a.data() + q, b.data() + q, cnt, N, wk.part.as<double>(), scal, s);
            HIPCHK(hipMemcpyAsync(raw.data() + 2 * q, scal, 2 * cnt * sizeof(double), hipMemcpyDeviceToHost, s));
            sync();
        }
        for (int q = 0; q < np; q++) out[q] = cxd(raw[2 * q], raw[2 * q + 1]);
        return out;
    };
    auto norm = [&](const void* x) { return std::sqrt(std::max(0.0, dots({x}, {x})[0].real())); };
    auto lin = [&](void* out, bool acc, std::initializer_list<std::pair<const void*, cxd>> terms) {
        ZLC z{};
        int t = 0;
        for (const auto& tm : terms) {
            z.in[t] = tm.first;
            z.are[t] = tm.second.real();
            z.aim[t] = tm.second.imag();
            t++;
        }
        z.nt = t;
        z.acc = acc ? 1 : 0;
        z.out = out;
        return z;
    };
    auto run = [&](const std::vector<ZLC>& zs) {
        if (!zs.empty()) zlincomb(zs.data(), (int)zs.size(), N, s);
    };
    // H on the listed vectors of x (contiguous [nrhs][N]) into out; with red, returns Re x_j^dag H x_j
    int n_apply = 0;
    auto applyH = [&](const DBuf& x, const DBuf& out, const std::vector<int>& js, bool red) {
        std::vector<int32_t> m(js.begin(), js.end());
        HIPCHK(hipMemcpyAsync(wk.vmap.p, m.data(), m.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        apply_H_int(h, x.p, out.p, (int)js.size(), nrhs, wk.vmap.as<int32_t>(), red ? x.p : nullptr,
                    red ? wk.hpart.as<double>() : nullptr);
        n_apply++;
        std::vector<double> a;
        if (red) {
            const int64_t ns = nsb_for(h, false, (int)js.size());
            sum_partials(wk.hpart.as<double>(), ns, nrhs, scal, false, L);
            std::vector<double> all(nrhs);
            HIPCHK(hipMemcpyAsync(all.data(), scal, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
            sync();
            for (int j : js) a.push_back(all[j]);
        }
        return a;
    };
    // x -= V_{0..nv-1} V^dag x, one CGS pass (coefficients on the matrix cores)
    auto cgs_pass = [&](int nv, void* x) {
        if (nv < 1) return;
        ProjArgs a{};
        a.V = wk.V.p;
        a.ldv = N;
        a.nv = nv;
        a.R[0] = x;
        a.nr = 1;
        a.n = N;
        a.kchunk = reorth_kchunk(N, nv);
        const int64_t nch = proj_chunks(N, a.kchunk);
        a.part_stride = 2 * (int64_t)nv;
        wk.pp.ensure((size_t)nch * a.part_stride * sizeof(double));
        a.part = wk.pp.as<double>();
        wk.P.ensure((size_t)2 * nv * sizeof(double));
        wk.E.ensure((size_t)2 * nv * sizeof(double));
        project(false, a, (nv + 31) / 32, wk.P.as<double>(), L, true);
        std::vector<double> c(2 * nv);
        HIPCHK(hipMemcpyAsync(c.data(), wk.P.p, c.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        sync();
        for (double& v : c) v = -v;
        HIPCHK(hipMemcpyAsync(wk.E.p, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice, s));
        sync();
        for (int r0 = 0; r0 < nv; r0 += 32)
            seed_update(false, false, vcol(r0), std::min(32, nv - r0), wk.E.as<double>() + 2 * r0, x, 1, N, nullptr, L);
    };
    int passes = 0;
    auto orthogonalise = [&](int nv, void* x) {   // CGS with one DGKS repeat
        const double n0 = norm(x);
        cgs_pass(nv, x);
        passes++;
        if (norm(x) < n0 / std::sqrt(2.0)) {
            cgs_pass(nv, x);
            passes++;
        }
    };

    // c^j = gamma5 phi^j, x^j from X, r_0^j = c^j - H x^j
    pack_vec(false, Phi, wk.R0.p, h->g.Vh, nrhs, L);
    gamma5_copy(false, wk.R0.p, wk.C.p, h->g.Vh, nrhs, L);
    pack_vec(false, Xout, wk.X.p, h->g.Vh, nrhs, L);
    std::vector<int> all(nrhs);
    for (int j = 0; j < nrhs; j++) all[j] = j;
    applyH(wk.X, wk.Hb, all, false);
    {
        std::vector<ZLC> zs;
        for (int j = 0; j < nrhs; j++) zs.push_back(lin(vec(wk.R0, j), false, {{vec(wk.C, j), 1.0}, {vec(wk.Hb, j), -1.0}}));
        run(zs);
    }
    std::vector<double> cn(nrhs);
    {
        std::vector<const void*> a;
        for (int j = 0; j < nrhs; j++) a.push_back(vec(wk.C, j));
        const auto d = dots(a, a);
        for (int j = 0; j < nrhs; j++) cn[j] = std::sqrt(d[j].real());
    }
    std::vector<int32_t> iters(nrhs, 0), matvecs(nrhs, 1);

    // ---- seeded Lanczos with the QR of Tbar -------------------------------------------------
    const double beta0 = norm(vec(wk.R0, 0));
    int m_used = 0, i_conv = 0, status = 0;
    if (beta0 > 0.0 && cn[0] > 0.0) {
        run({lin(vcol(0), false, {{vec(wk.R0, 0), 1.0 / beta0}})});
        std::vector<cxd> u(nrhs);
        u[0] = beta0;
        if (nrhs > 1) {
            std::vector<const void*> a(nrhs - 1, vcol(0)), b;
            for (int j = 1; j < nrhs; j++) b.push_back(vec(wk.R0, j));
            const auto d = dots(a, b);
            for (int j = 1; j < nrhs; j++) u[j] = d[j - 1];
        }
        std::vector<double> alpha, beta{beta0};
        std::vector<cxd> eblk((size_t)WB * nrhs);
        int nbuf = 0;   // steps whose w_i and tau_i wait in the ring for the next X update
        wk.E.ensure((size_t)2 * WB * nrhs * sizeof(double));
        auto flush = [&]() {
            if (nbuf == 0) return;
            HIPCHK(hipMemcpyAsync(wk.E.p, eblk.data(), (size_t)nbuf * nrhs * sizeof(cxd), hipMemcpyHostToDevice, s));
            sync();
            seed_update(false, false, wk.W.p, nbuf, wk.E.as<double>(), wk.X.p, nrhs, N, nullptr, L);
            nbuf = 0;
        };
        Givens g1, g2;
        int m_stop = m_cap;
        const void* wm1 = nullptr;   // w_{i-1}
        const void* wm2 = nullptr;   // w_{i-2}
        for (int i = 1;; i++) {
            void* v = vcol(i - 1);
            // f = H v_i - beta_{i-1} v_{i-1} - alpha_i v_i, alpha_i = v_i^dag H v_i (fused in the stencil)
            {
                apply_H_int(h, v, wk.F.p, 1, 1, nullptr, v, wk.hpart.as<double>());
                sum_partials(wk.hpart.as<double>(), nsb_for(h, false, 1), 1, scal, false, L);
                double a = 0.0;
                HIPCHK(hipMemcpyAsync(&a, scal, sizeof(double), hipMemcpyDeviceToHost, s));
                sync();
                alpha.push_back(a);
            }
            const double a = alpha.back();
            if (i > 1)
                run({lin(wk.F.p, true, {{v, -a}, {vcol(i - 2), -beta[i - 1]}})});
            else
                run({lin(wk.F.p, true, {{v, -a}})});
            if (k > 0 && i % k == 0) {   // periodic reorthogonalisation
                orthogonalise(i - 1, v);
                const double nv = norm(v);
                run({lin(v, false, {{v, 1.0 / nv}})});
                orthogonalise(i, wk.F.p);
            }
            // beta_i = ||f|| and f^dag r_0^j in one pass
            std::vector<const void*> da{wk.F.p}, db{wk.F.p};
            for (int j = 1; j < nrhs; j++) {
                da.push_back(wk.F.p);
                db.push_back(vec(wk.R0, j));
            }
            const auto d = dots(da, db);
            const double bi = std::sqrt(std::max(0.0, d[0].real()));
            beta.push_back(bi);
            const QrCol q = qr_column(i > 1 ? beta[i - 1] : 0.0, a, bi, g2, g1);
            if (!(q.rho > 0.0)) {
                status = 1;
                break;
            }
            // w_i into ring slot (i - 1) % WB (the previous two slots hold w_{i-1}, w_{i-2}); tau^j_i
            // waits in E_blk until the ring is full
            const int slot = (i - 1) % WB;
            void* w = (char*)wk.W.p + (int64_t)slot * vbytes;
            for (int j = 0; j < nrhs; j++) {
                const cxd eta = (j == 0 || bi == 0.0) ? cxd(0.0) : d[j] / bi;   // v_{i+1}^dag r_0^j
                eblk[(size_t)slot * nrhs + j] = q.g.c * u[j] + q.g.s * eta;
                u[j] = -q.g.s * u[j] + q.g.c * eta;
            }
            std::vector<ZLC> zs;
            if (bi > 0.0) zs.push_back(lin(vcol(i), false, {{wk.F.p, 1.0 / bi}}));
            {
                ZLC z = lin(w, false, {{v, 1.0 / q.rho}});
                if (wm1) {
                    z.in[z.nt] = wm1;
                    z.are[z.nt] = -q.delta / q.rho;
                    z.aim[z.nt] = 0.0;
                    z.nt++;
                }
                if (wm2) {
                    z.in[z.nt] = wm2;
                    z.are[z.nt] = -q.eps / q.rho;
                    z.aim[z.nt] = 0.0;
                    z.nt++;
                }
                zs.push_back(z);
            }
            run(zs);
            if (++nbuf == WB) flush();
            m_used = i;
            const double e = std::abs(u[0]);
            if (i_conv == 0 && e <= tol * cn[0]) {
                i_conv = i;
                m_stop = std::min((int)std::ceil(h->p.past_factor * i_conv), m_cap);
            }
            double amax = 0.0;
            for (double x : alpha) amax = std::max(amax, std::abs(x));
            if (bi <= 1e-14 * amax) {
                status = 1;
                break;
            }
            if (i >= m_stop) {
                if (i_conv == 0) status = 3;
                break;
            }
            wm2 = wm1;
            wm1 = w;
            g2 = g1;
            g1 = q.g;
        }
        flush();
        iters[0] = m_used;
        matvecs[0] += m_used;
    }
    const double t1 = now_s();

    // ---- plain MINRES on every system from its guess, in lockstep ------------------------------
    // v_cur / v_prev alternate between Va and Vb, the direction vectors rotate through Wa, Wb, Wc
    struct St {
        bool active = false, restart = true;
        int it = 0;
        double bprev = 0.0;
        cxd u = 0.0;
        Givens g1, g2;
        bool have_w1 = false, have_w2 = false;
    };
    std::vector<St> st(nrhs);
    std::vector<double> res(nrhs, 0.0);
    DBuf* vcur = &wk.Va;
    DBuf* vprev = &wk.Vb;
    DBuf* wbuf[3] = {&wk.Wa, &wk.Wb, &wk.Wc};
    int wnew = 0;   // the array that takes w_i; (wnew + 2) % 3 holds w_{i-1}, (wnew + 1) % 3 w_{i-2}
    // true residuals of the listed systems into R0 (as r = c - H x) and their norms
    auto residuals = [&](const std::vector<int>& js) {
        applyH(wk.X, wk.Hb, js, false);
        std::vector<ZLC> zs;
        std::vector<const void*> a;
        for (int j : js) {
            zs.push_back(lin(vec(wk.R0, j), false, {{vec(wk.C, j), 1.0}, {vec(wk.Hb, j), -1.0}}));
            a.push_back(vec(wk.R0, j));
        }
        run(zs);
        const auto d = dots(a, a);
        std::vector<double> r;
        for (size_t q = 0; q < js.size(); q++) r.push_back(std::sqrt(std::max(0.0, d[q].real())));
        return r;
    };
    std::vector<int> check = all;
    bool noconv = false;
    for (;;) {
        // confirm or restart the systems whose estimate met tol (all of them at the start)
        if (!check.empty()) {
            const auto r = residuals(check);
            std::vector<ZLC> zs;
            for (size_t q = 0; q < check.size(); q++) {
                const int j = check[q];
                matvecs[j]++;
                const double rel = cn[j] > 0.0 ? r[q] / cn[j] : 0.0;
                res[j] = rel;
                if (rel <= tol || cn[j] == 0.0) {
                    st[j].active = false;
                    continue;
                }
                if (st[j].it >= max_iter) {
                    st[j].active = false;
                    noconv = true;
                    continue;
                }
                st[j] = St{};
                st[j].active = true;
                st[j].u = r[q];
                zs.push_back(lin(vec(*vcur, j), false, {{vec(wk.R0, j), 1.0 / r[q]}}));
                st[j].it = iters[j] - (j == 0 ? m_used : 0);
            }
            run(zs);
            check.clear();
        }
        std::vector<int> act;
        for (int j = 0; j < nrhs; j++)
            if (st[j].active) act.push_back(j);
        if (act.empty()) break;
        // f = H v - alpha v - bprev v_prev (in Hb), alpha fused in the stencil
        const auto al = applyH(*vcur, wk.Hb, act, true);
        {
            std::vector<ZLC> zs;
            for (size_t q = 0; q < act.size(); q++) {
                const int j = act[q];
                if (st[j].bprev > 0.0)
                    zs.push_back(lin(vec(wk.Hb, j), true, {{vec(*vcur, j), -al[q]}, {vec(*vprev, j), -st[j].bprev}}));
                else
                    zs.push_back(lin(vec(wk.Hb, j), true, {{vec(*vcur, j), -al[q]}}));
            }
            run(zs);
        }
        std::vector<const void*> fa;
        for (int j : act) fa.push_back(vec(wk.Hb, j));
        const auto ff = dots(fa, fa);
        std::vector<ZLC> zv, zx;
        std::vector<cxd> tauv(act.size());
        std::vector<QrCol> qs(act.size());
        for (size_t q = 0; q < act.size(); q++) {
            const int j = act[q];
            St& S = st[j];
            const double bi = std::sqrt(std::max(0.0, ff[q].real()));
            const QrCol c = qr_column(S.bprev, al[q], bi, S.g2, S.g1);
            qs[q] = c;
            const cxd tau = c.g.c * S.u;
            S.u = -c.g.s * S.u;
            tauv[q] = tau;
            if (bi > 0.0) zv.push_back(lin(vec(*vprev, j), false, {{vec(wk.Hb, j), 1.0 / bi}}));
            ZLC z = lin(vec(*wbuf[wnew], j), false, {{vec(*vcur, j), 1.0 / c.rho}});
            if (S.have_w1) {
                z.in[z.nt] = vec(*wbuf[(wnew + 2) % 3], j);
                z.are[z.nt] = -c.delta / c.rho;
                z.aim[z.nt] = 0.0;
                z.nt++;
            }
            if (S.have_w2) {
                z.in[z.nt] = vec(*wbuf[(wnew + 1) % 3], j);
                z.are[z.nt] = -c.eps / c.rho;
                z.aim[z.nt] = 0.0;
                z.nt++;
            }
            zv.push_back(z);
            zx.push_back(lin(vec(wk.X, j), true, {{vec(*wbuf[wnew], j), tau}}));
            S.bprev = bi;
            S.g2 = S.g1;
            S.g1 = c.g;
            S.have_w2 = S.have_w1;
            S.have_w1 = true;
            S.it++;
            iters[j]++;
            matvecs[j]++;
            if (std::abs(S.u) <= tol * cn[j] || bi == 0.0 || S.it >= max_iter) check.push_back(j);
        }
        run(zv);   // v_next into the v_prev array, w_i into wbuf[wnew]
        run(zx);   // x += tau w_i
        std::swap(vcur, vprev);
        wnew = (wnew + 1) % 3;
        for (int j : check) st[j].active = false;
    }
    unpack_vec(false, wk.X.p, Xout, h->g.Vh, nrhs, L);
    sync();
    if (rep) {
        for (int j = 0; j < nrhs; j++) {
            if (rep->iters) rep->iters[j] = iters[j];
            if (rep->matvecs) rep->matvecs[j] = matvecs[j];
            if (rep->true_relres) rep->true_relres[j] = res[j];
        }
        rep->m_used = m_used;
        rep->i_conv = i_conv;
        rep->seed_status = status;
        rep->reorth_passes = passes;
        rep->t_seed_s = t1 - t0;
        rep->t_rest_s = now_s() - t1;
    }
    (void)n_apply;
    return !noconv;
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
    } catch (const std::invalid_argument& e) {
        return fail(h, SEEDCG_ERR_ARG, e.what());
    } catch (const std::exception& e) {
        return fail(h, SEEDCG_ERR_HIP, e.what());
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
    p->autotune = 1;
    p->deflate = 0;
}

seedcg_status seedcg_create(const seedcg_params* p, const double* links, seedcg_t* out) {
    if (!p || !links || !out) return fail(nullptr, SEEDCG_ERR_ARG, "create: null pointer");
    *out = nullptr;
    for (int d = 0; d < 4; d++)
        if (p->dims[d] < 2 || p->dims[d] % 2) return fail(nullptr, SEEDCG_ERR_ARG, "create: every extent must be even and >= 2");
    if (p->t_bc != 1 && p->t_bc != -1) return fail(nullptr, SEEDCG_ERR_ARG, "create: t_bc must be +1 or -1");
    if (p->prec < 0 || p->prec > 3) return fail(nullptr, SEEDCG_ERR_ARG, "create: unknown precision");
    if (!(p->tol > 0.0)) return fail(nullptr, SEEDCG_ERR_ARG, "create: tol must be > 0");
    if (p->reorth_k < 0) return fail(nullptr, SEEDCG_ERR_ARG, "create: reorth_k must be >= 0");
    if (p->basis_fp32 < 0 || p->basis_fp32 > 2) return fail(nullptr, SEEDCG_ERR_ARG, "create: basis_fp32 must be 0, 1 or 2");
    seedcg_s* h = new (std::nothrow) seedcg_s;
    if (!h) return fail(nullptr, SEEDCG_ERR_OOM, "create: host allocation failed");
    seedcg_status st = guarded(h, [&]() -> seedcg_status {
        h->s = (hipStream_t)p->stream;
        init_geometry(h, p, p->dims);
        const Geom& g = h->g;
        h->links64.ensure(4 * g.V * 9 * 16);
        pack_links(P64, g, links, h->links64.p, h->s);
        if (h->cg_lo) {
            h->links_lo.ensure(4 * g.V * 9 * (h->lo_prec == P32 ? 8 : 4));
            pack_links(h->lo_prec, g, links, h->links_lo.p, h->s);
        }
        choose_link_formats(h, su3_defect_max(h, links) <= SU3_DEFECT_TOL);
        if (h->hop64 == P64R) {
            h->links64r.ensure(4 * g.V * 6 * 16);
            pack_links(P64R, g, links, h->links64r.p, h->s);
        }
        if (h->hop_lo == P32R) {
            h->links_lor.ensure(4 * g.V * 6 * 8);
            pack_links(P32R, g, links, h->links_lor.p, h->s);
        }
        check_launch();
        autotune_single(h, 12);
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

seedcg_status seedcg_create_batch(int32_t ncfg, const int32_t* dims, const double* kappa, const double* const* links, int32_t nrhs,
                                  const seedcg_params* p, seedcg_batch_t* out) {
    if (!p || !dims || !kappa || !links || !out) return fail(nullptr, SEEDCG_ERR_ARG, "create_batch: null pointer");
    *out = nullptr;
    if (ncfg < 1) return fail(nullptr, SEEDCG_ERR_ARG, "create_batch: ncfg < 1");
    if (p->basis_fp32 && (p->prec == SEEDCG_FP64 || p->prec == SEEDCG_MIXED_FP32_CG))
        return fail(nullptr, SEEDCG_ERR_ARG, "create_batch: an FP32 copy of an FP64 basis is for single configurations");
    if (nrhs < 1 || nrhs > 25) return fail(nullptr, SEEDCG_ERR_ARG, "create_batch: nrhs must be 1..25");
    for (int c = 0; c < ncfg; c++) {
        for (int d = 0; d < 4; d++)
            if (dims[4 * c + d] < 2 || dims[4 * c + d] % 2)
                return fail(nullptr, SEEDCG_ERR_ARG, "create_batch: every extent must be even and >= 2");
        if (!links[c]) return fail(nullptr, SEEDCG_ERR_ARG, "create_batch: null links pointer");
        if (!(kappa[c] > 0.0)) return fail(nullptr, SEEDCG_ERR_ARG, "create_batch: kappa must be > 0");
    }
    if (p->t_bc != 1 && p->t_bc != -1) return fail(nullptr, SEEDCG_ERR_ARG, "create_batch: t_bc must be +1 or -1");
    if (p->prec < 0 || p->prec > 3) return fail(nullptr, SEEDCG_ERR_ARG, "create_batch: unknown precision");
    if (p->prec == SEEDCG_MIXED_FP32_CG && p->deflate > 0)
        return fail(nullptr, SEEDCG_ERR_ARG, "create_batch: MIXED_FP32_CG takes no deflation");
    if (!(p->tol > 0.0)) return fail(nullptr, SEEDCG_ERR_ARG, "create_batch: tol must be > 0");
    if (p->reorth_k < 0) return fail(nullptr, SEEDCG_ERR_ARG, "create_batch: reorth_k must be >= 0");
    if (p->precond != 0) return fail(nullptr, SEEDCG_ERR_ARG, "create_batch: the learned preconditioner is per configuration");
    seedcg_batch_s* b = new (std::nothrow) seedcg_batch_s;
    if (!b) return fail(nullptr, SEEDCG_ERR_OOM, "create_batch: host allocation failed");
    b->ncfg = ncfg;
    b->nrhs = nrhs;
    b->user_stream = (hipStream_t)p->stream;
    seedcg_s tmp;  // collects the error text of the set-up
    const seedcg_status st = guarded(&tmp, [&]() -> seedcg_status {
        // classes in order of first appearance
        for (int c = 0; c < ncfg; c++) {
            int k = 0;
            for (; k < (int)b->members.size(); k++)
                if (std::equal(dims + 4 * c, dims + 4 * c + 4, dims + 4 * b->members[k][0])) break;
            if (k == (int)b->members.size()) b->members.push_back({});
            b->members[k].push_back(c);
        }
        for (const auto& mem : b->members) {
            seedcg_s* h = new seedcg_s;
            b->cls.push_back(h);
            init_geometry(h, p, dims + 4 * mem[0]);
            h->ncfg = (int)mem.size();
            h->p.kappa = kappa[mem[0]];
            for (int c : mem) h->kappas.push_back(kappa[c]);
            HIPCHK(hipStreamCreateWithFlags(&h->s, hipStreamNonBlocking));
            h->own_stream = true;
        }
        // two-row links for a class only when every member's field is special unitary
        for (size_t k = 0; k < b->cls.size(); k++) {
            bool su = true;
            for (int c : b->members[k]) su = su && su3_defect_max(b->cls[k], links[c]) <= SU3_DEFECT_TOL;
            choose_link_formats(b->cls[k], su);
        }
        // one basis capacity for every class: params.m_max, or the largest that fits in 90% of
        // the free HBM less 4 GiB
        size_t freeb = 0, total = 0;
        HIPCHK(hipMemGetInfo(&freeb, &total));
        const double budget = 0.9 * (double)freeb - 4.0 * (1 << 30);
        auto need = [&](int m) {
            double t = 0.0;
            for (auto h : b->cls) t += (double)plan_layout(h, nrhs, m, nullptr) * h->ncfg;
            return t;
        };
        int m_cap = p->m_max;
        if (m_cap > 0) {
            if (need(m_cap) > budget) throw OomError{"create_batch: the Krylov bases of m_max vectors do not fit in HBM"};
        } else {
            int lo = 2, hi = 8192;
            if (need(lo) > budget) throw OomError{"create_batch: no room for the Krylov bases"};
            while (lo < hi) {
                const int mid = (lo + hi + 1) / 2;
                if (need(mid) <= budget)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            m_cap = lo;
        }
        for (size_t k = 0; k < b->cls.size(); k++) {
            seedcg_s* h = b->cls[k];
            apply_layout(h, nrhs, m_cap);
            const Geom& g = h->g;
            std::vector<double> k2;
            for (int i = 0; i < h->ncfg; i++) {
                const int c = b->members[k][i];
                pack_links(P64, g, links[c], (char*)h->links64.p + (int64_t)i * h->cs, h->s);
                if (h->cg_lo) pack_links(h->lo_prec, g, links[c], (char*)h->links_lo.p + (int64_t)i * h->cs, h->s);
                if (h->hop64 == P64R) pack_links(P64R, g, links[c], (char*)h->links64r.p + (int64_t)i * h->cs, h->s);
                if (h->hop_lo == P32R) pack_links(P32R, g, links[c], (char*)h->links_lor.p + (int64_t)i * h->cs, h->s);
                k2.push_back(kappa[c] * kappa[c]);
            }
            to_cfg(h, h->kap2.p, k2.data(), sizeof(double));
            check_launch();
            // launch shapes timed on the batch itself (zeroed vectors of the CG and Lanczos buffers)
            if (h->p.autotune && !env_shape_fixed()) {
                // one vector in the Lanczos precision, several in the CG precision
                zero_cfg(h, h->Pv.p, nrhs * h->vec_bytes(h->cg_lo));
                zero_cfg(h, h->basis.p, h->vec_bytes(h->lo));
                tune_shape(h, h->lo, 1, h->basis.p, h->f.p);
                if (nrhs > 1) tune_shape(h, h->cg_lo, nrhs, h->Pv.p, h->Qv.p);
                if (h->cg_lo && nrhs > 1) {   // the FP64 stencil of the true residuals and reliable updates
                    zero_cfg(h, h->R64.p, nrhs * h->vec_bytes(false));
                    tune_shape(h, false, nrhs, h->R64.p, h->Xint.p);
                }
                h->tuned = true;
            }
            HIPCHK(hipStreamSynchronize(h->s));
        }
        return SEEDCG_OK;
    });
    if (st != SEEDCG_OK) {
        g_create_error = tmp.err;
        delete b;
        return st;
    }
    *out = b;
    return SEEDCG_OK;
}

seedcg_status seedcg_solve_batch(seedcg_batch_t b, const double* const* B, double* const* X, seedcg_report* rep) {
    if (!b) return fail(nullptr, SEEDCG_ERR_ARG, "solve_batch: null batch");
    Phase ph("seedcg_solve_batch");
    if (!B || !X) {
        b->err = "solve_batch: null pointer";
        return SEEDCG_ERR_ARG;
    }
    for (int c = 0; c < b->ncfg; c++)
        if (!B[c] || !X[c]) {
            b->err = "solve_batch: null vector pointer";
            return SEEDCG_ERR_ARG;
        }
    const hipError_t e0 = hipStreamSynchronize(b->user_stream);  // B and X are ready
    if (e0 != hipSuccess) {
        b->err = std::string("solve_batch: ") + hipGetErrorString(e0);
        return SEEDCG_ERR_HIP;
    }
    const int K = (int)b->cls.size(), nrhs = b->nrhs;
    std::vector<seedcg_status> sts(K, SEEDCG_OK);
    std::vector<std::thread> th;
    for (int k = 0; k < K; k++) {
        th.emplace_back([&, k]() {
            seedcg_s* h = b->cls[k];
            const std::vector<int>& mem = b->members[k];
            const int n = (int)mem.size();
            sts[k] = guarded(h, [&]() -> seedcg_status {
                HIPCHK(hipSetDevice(h->device));
                Io io;
                if (n == 1) {
                    io.B = B[mem[0]];
                    io.X = X[mem[0]];
                } else {
                    std::vector<const void*> t(2 * n);
                    for (int i = 0; i < n; i++) {
                        t[i] = B[mem[i]];
                        t[n + i] = X[mem[i]];
                    }
                    HIPCHK(hipMemcpyAsync(h->tabs.p, t.data(), t.size() * sizeof(void*), hipMemcpyHostToDevice, h->s));
                    HIPCHK(hipStreamSynchronize(h->s));
                    io.Btab = (const double* const*)h->tabs.p;
                    io.Xtab = (double* const*)h->tabs.p + n;
                }
                std::vector<int32_t> it_s((size_t)n * nrhs), mv_s((size_t)n * nrhs), it_r((size_t)n * nrhs), mv_r((size_t)n * nrhs);
                std::vector<double> res((size_t)n * nrhs);
                std::vector<seedcg_report> rs(n), rr(n);
                for (int i = 0; i < n; i++) {
                    rs[i] = seedcg_report{};
                    rs[i].iters = &it_s[(size_t)i * nrhs];
                    rs[i].matvecs = &mv_s[(size_t)i * nrhs];
                    rr[i] = seedcg_report{};
                    rr[i].iters = &it_r[(size_t)i * nrhs];
                    rr[i].matvecs = &mv_r[(size_t)i * nrhs];
                    rr[i].true_relres = &res[(size_t)i * nrhs];
                }
                solve_seed_impl(h, io, nrhs, rs.data());
                const seedcg_status s2 = solve_rest_impl(h, io, nrhs, rr.data());
                if (rep)
                    for (int i = 0; i < n; i++) {
                        seedcg_report& u = rep[mem[i]];
                        for (int j = 0; j < nrhs; j++) {
                            const size_t q = (size_t)i * nrhs + j;
                            if (u.iters) u.iters[j] = (j == 0 ? it_s[q] : 0) + it_r[q];
                            if (u.matvecs) u.matvecs[j] = mv_s[q] + mv_r[q];
                            if (u.true_relres) u.true_relres[j] = res[q];
                        }
                        u.m_used = rs[i].m_used;
                        u.i_conv = rs[i].i_conv;
                        u.seed_status = rs[i].seed_status;
                        u.reorth_passes = rs[i].reorth_passes;
                        u.t_seed_s = rs[i].t_seed_s;
                        u.t_rest_s = rr[i].t_rest_s;
                    }
                if (s2 == SEEDCG_ERR_NOCONV) h->err = "solve_batch: max_iter reached before tol";
                return s2;
            });
        });
    }
    for (auto& t : th) t.join();
    for (int k = 0; k < K; k++)
        if (sts[k] != SEEDCG_OK) {
            b->err = b->cls[k]->err;
            return sts[k];
        }
    return SEEDCG_OK;
}

seedcg_status seedcg_batch_info(seedcg_batch_t b, int32_t* nclass, int32_t* class_of, int32_t* m_cap, double* tune) {
    if (!b) return fail(nullptr, SEEDCG_ERR_ARG, "batch_info: null batch");
    if (nclass) *nclass = (int32_t)b->cls.size();
    for (size_t k = 0; k < b->cls.size(); k++) {
        if (class_of)
            for (int c : b->members[k]) class_of[c] = (int32_t)k;
        if (m_cap) m_cap[k] = b->cls[k]->m_cap;
        if (tune) {
            const seedcg_s* h = b->cls[k];
            // one vector in the Lanczos precision, several in the CG precision
            tune[4 * k + 0] = h->lo ? h->tps_lo : h->tps64;
            tune[4 * k + 1] = h->lo ? h->vb_lo : h->vb64;
            tune[4 * k + 2] = h->cg_lo ? h->tps_lo_multi : h->tps64_multi;
            tune[4 * k + 3] = h->cg_lo ? h->vb_lo_multi : h->vb64_multi;
        }
    }
    return SEEDCG_OK;
}

seedcg_status seedcg_batch_set_timing(seedcg_batch_t b, int32_t sample_every, int32_t max_samples) {
    if (!b) return fail(nullptr, SEEDCG_ERR_ARG, "batch_set_timing: null batch");
    for (auto h : b->cls) {
        const seedcg_status st = seedcg_set_timing(h, sample_every, max_samples);
        if (st != SEEDCG_OK) {
            b->err = h->err;
            return st;
        }
    }
    return SEEDCG_OK;
}

seedcg_status seedcg_batch_get_timing(seedcg_batch_t b, double* out) {
    if (!b) return fail(nullptr, SEEDCG_ERR_ARG, "batch_get_timing: null batch");
    if (!out) {
        b->err = "batch_get_timing: null pointer";
        return SEEDCG_ERR_ARG;
    }
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (auto h : b->cls) {
        double o[6];
        const seedcg_status st = seedcg_get_timing(h, o);
        if (st != SEEDCG_OK) {
            b->err = h->err;
            return st;
        }
        for (int k = 0; k < 6; k++) acc[k] += o[k];
    }
    for (int k = 0; k < 6; k++) out[k] = acc[k];
    return SEEDCG_OK;
}

void seedcg_destroy_batch(seedcg_batch_t b) {
    if (!b) return;
    for (auto h : b->cls) (void)hipStreamSynchronize(h->s);
    delete b;
}

const char* seedcg_batch_last_error(seedcg_batch_t b) { return b ? b->err.c_str() : g_create_error.c_str(); }

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
        const bool lo = h->cg_lo;   // the CG's operator (the Lanczos one differs only in MIXED_FP32_CG)
        xi.ensure(nvec * h->vec_bytes(lo));
        yi.ensure(nvec * h->vec_bytes(lo));
        pack_vec(lo, x, xi.p, h->g.Vh, nvec, h->s);
        apply_M_int(h, lo, xi.p, yi.p, nvec, MOpts{});
        unpack_vec(lo, yi.p, y, h->g.Vh, nvec, h->s);
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
    Phase ph("seedcg_solve_seed");
    return guarded(h, [&]() -> seedcg_status {
        if (!B || !X) throw ArgError{"solve_seed: null pointer"};
        Io io;
        io.B = B;
        io.X = X;
        solve_seed_impl(h, io, nrhs, r);
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_solve_rest(seedcg_t h, const double* B, double* X, int32_t nrhs, seedcg_report* r) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "solve_rest: null handle");
    Phase ph("seedcg_solve_rest");
    return guarded(h, [&]() -> seedcg_status {
        if (!B || !X) throw ArgError{"solve_rest: null pointer"};
        Io io;
        io.B = B;
        io.X = X;
        seedcg_status s = solve_rest_impl(h, io, nrhs, r);
        if (s == SEEDCG_ERR_NOCONV) h->err = "solve_rest: max_iter reached before tol";
        return s;
    });
}

seedcg_status seedcg_solve_repeated(seedcg_t h, const double* B, double* X, int32_t nrhs, seedcg_report* r) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "solve_repeated: null handle");
    Phase ph("seedcg_solve_repeated");
    return guarded(h, [&]() -> seedcg_status {
        if (!B || !X || nrhs < 1) throw ArgError{"solve_repeated: null pointer or nrhs < 1"};
        if (nrhs > 25) throw ArgError{"solve_repeated: at most 25 right-hand sides"};
        if (h->ncfg != 1) throw StateError{"solve_repeated: one configuration per handle"};
        const int64_t stride = h->g.Vh * 12 * 2;   // doubles per canonical vector
        std::vector<int32_t> lz(nrhs, 0), lmv(nrhs, 0);
        const double past = h->p.past_factor;
        h->p.past_factor = 1.0;   // every system runs Algorithm 1 just to its own convergence
        try {
            for (int j = 0; j < nrhs; j++) {
                Io io;
                io.B = B + (int64_t)j * stride;
                io.X = X + (int64_t)j * stride;
                seedcg_report rj{};
                solve_seed_impl(h, io, nrhs - j, &rj);
                lz[j] = rj.m_used;
                lmv[j] = rj.m_used + 1;
                if (r && j == 0) {
                    r->i_conv = rj.i_conv;
                    r->seed_status = rj.seed_status;
                }
                if (r) r->reorth_passes += rj.reorth_passes;
            }
        } catch (...) {
            h->p.past_factor = past;
            throw;
        }
        h->p.past_factor = past;
        const double t1 = now_s();
        std::vector<int32_t> it(nrhs), mv(nrhs);
        std::vector<double> res(nrhs);
        seedcg_report rr{};
        rr.iters = it.data();
        rr.matvecs = mv.data();
        rr.true_relres = res.data();
        Io io;
        io.B = B;
        io.X = X;
        const seedcg_status st = solve_rest_impl(h, io, nrhs, &rr);
        if (r) {
            for (int j = 0; j < nrhs; j++) {
                if (r->iters) r->iters[j] = lz[j] + it[j];
                if (r->matvecs) r->matvecs[j] = lmv[j] + mv[j];
                if (r->true_relres) r->true_relres[j] = res[j];
            }
            r->m_used = lz[0];
            r->t_rest_s = now_s() - t1;
        }
        if (st == SEEDCG_ERR_NOCONV) h->err = "solve_repeated: max_iter reached before tol";
        return st;
    });
}

seedcg_status seedcg_solve_indefinite(seedcg_t h, const double* Phi, double* X, int32_t nrhs, seedcg_report* r) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "solve_indefinite: null handle");
    Phase ph("seedcg_solve_indefinite");
    return guarded(h, [&]() -> seedcg_status {
        if (!Phi || !X) throw ArgError{"solve_indefinite: null pointer"};
        if (!solve_indefinite_impl(h, Phi, X, nrhs, r)) {
            h->err = "solve_indefinite: max_iter reached before tol";
            return SEEDCG_ERR_NOCONV;
        }
        return SEEDCG_OK;
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

seedcg_status seedcg_get_ritz(seedcg_t h, double* theta, int32_t cap, int32_t* n) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "get_ritz: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (!n) throw ArgError{"get_ritz: null n"};
        *n = h->nev;
        if (!theta) return SEEDCG_OK;
        if (cap < h->nev) throw ArgError{"get_ritz: cap < n"};
        for (int k = 0; k < h->nev; k++) theta[k] = h->ritz_theta[k];
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_get_basis_vector(seedcg_t h, int32_t i, double* v) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "get_basis_vector: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (!h->have_seed || !h->basis.p) throw StateError{"get_basis_vector: no basis"};
        if (i < 1 || i > h->m_used || !v) throw ArgError{"get_basis_vector: index out of range or null pointer"};
        const void* src = (const char*)h->basis.p + (int64_t)(i - 1) * h->vec_bytes(h->blo);
        unpack_vec(h->blo, src, v, h->g.Vh, 1, h->s);
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

seedcg_status seedcg_project_noalloc(seedcg_t h, const double* Vv, int32_t nv, const double* R, int32_t nr, int64_t n,
                                     double* P) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "project_noalloc: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (!Vv || !R || !P || nv < 1 || nr < 1 || n < 1) throw ArgError{"project_noalloc: null pointer or empty size"};
        if (nr > 24) throw ArgError{"project_noalloc: at most 24 vectors in R"};
        const int64_t per_chunk = 2 * (int64_t)nv * nr;   // partial doubles of one K-chunk
        if (per_chunk > PROJ_SCRATCH_DOUBLES)
            throw ArgError{"project_noalloc: nv * nr = " + std::to_string((int64_t)nv * nr) + " exceeds " +
                           std::to_string(PROJ_SCRATCH_DOUBLES / 2) + " (static partials of " +
                           std::to_string(PROJ_SCRATCH_DOUBLES * 8 >> 20) + " MiB)"};
        ProjArgs a{};
        a.V = Vv;
        a.ldv = n;
        a.nv = nv;
        for (int j = 0; j < nr; j++) a.R[j] = R + 2 * (int64_t)j * n;
        a.nr = nr;
        a.n = n;
        // seedcg_project's K-chunk (so the two agree bit for bit) unless its partials would not fit
        a.kchunk = kchunk_for(n, std::max<int64_t>(1, 1024 / ((nv + 31) / 32)));
        const int64_t max_chunks = PROJ_SCRATCH_DOUBLES / per_chunk;
        if (proj_chunks(n, a.kchunk) > max_chunks) a.kchunk = ((n + max_chunks - 1) / max_chunks + 31) / 32 * 32;
        a.part_stride = per_chunk;
        a.part = proj_scratch();   // the device address of this GPU's copy, never the array's host-side name
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
        h->ev_kind.clear();
        h->t_kind.clear();
        h->t_ms = h->t_bytes = h->t_flops = h->hop_bytes_all = 0.0;
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
            auto& t = h->t_kind[h->ev_kind[k]];
            t[0] += 1.0;
            t[1] += ms;
            t[2] += h->ev_bytes[k];
        }
        h->ev_kind.clear();
        h->ev_used = 0;
        h->ev_bytes.clear();
        h->ev_flops.clear();
        out[0] = (double)h->t_launches;
        out[1] = h->t_ms;
        out[2] = h->t_bytes;
        out[3] = h->t_flops;
        out[4] = (double)h->hop_count;
        out[5] = h->hop_bytes_all;
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_get_timing_kinds(seedcg_t h, double* out, int32_t cap, int32_t* n) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "get_timing_kinds: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (!out || !n || cap < 0) throw ArgError{"get_timing_kinds: null pointer or negative capacity"};
        double tmp[6];
        const seedcg_status st = seedcg_get_timing(h, tmp);   // folds the pending samples in
        if (st != SEEDCG_OK) return st;
        int k = 0;
        for (const auto& kv : h->t_kind) {
            if (k < cap) {
                double* r = out + 8 * (int64_t)k;
                for (int q = 0; q < 5; q++) r[q] = kv.first[q];
                for (int q = 0; q < 3; q++) r[5 + q] = kv.second[q];
            }
            k++;
        }
        *n = k;
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_time_M(seedcg_t h, int32_t inner, int32_t nvec, int32_t reps, double* out) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "time_M: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (!out || nvec < 1 || nvec > 25 || reps < 1) throw ArgError{"time_M: null pointer, nvec not in 1..25 or reps < 1"};
        if (h->ncfg != 1) throw StateError{"time_M: one configuration per handle"};
        const bool low = inner && h->cg_lo;
        DBuf x, y;
        x.ensure(nvec * h->vec_bytes(low));
        y.ensure(nvec * h->vec_bytes(low));
        cfg_zero(x.p, nvec * h->vec_bytes(low), h->L());
        const int saved = h->timing_every;
        h->timing_every = 0;
        apply_M_int(h, low, x.p, y.p, nvec, MOpts{});
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventRecord(e0, h->s));
        for (int r = 0; r < reps; r++) apply_M_int(h, low, (r & 1) ? y.p : x.p, (r & 1) ? x.p : y.p, nvec, MOpts{});
        HIPCHK(hipEventRecord(e1, h->s));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        h->timing_every = saved;
        // algorithmic bytes of one application: each of the four hops reads every link once (in the
        // stored format) for all vectors, and per vector M moves 120 V spinor reals
        const Prec pr = low ? h->hop_lo : h->hop64;
        const double sl = (pr == P64 || pr == P64R) ? 8.0 : (pr == P32BF ? 2.0 : 4.0);
        const double ss = low ? 4.0 : 8.0;
        const double lr = (pr == P64R || pr == P32R) ? 12.0 : 18.0;
        const double V = (double)h->g.V;
        out[0] = ms / reps;
        out[1] = 4.0 * 4.0 * V * lr * sl + 120.0 * V * ss * nvec;
        out[2] = 4.0 * 4.0 * V * 18.0 * sl + 120.0 * V * ss * nvec;
        out[3] = (double)pr;
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_probe_bandwidth(int32_t kind, int64_t bytes, int32_t reps, void* stream, double* gbs) {
    if (!gbs || kind < 0 || kind > 2 || bytes < (1 << 20) || reps < 1)
        return fail(nullptr, SEEDCG_ERR_ARG, "probe_bandwidth: kind 0..2, bytes >= 1 MiB, reps >= 1 and an output pointer");
    try {
        *gbs = probe_bandwidth(kind, bytes, reps, (hipStream_t)stream);
    } catch (const std::bad_alloc&) {
        return fail(nullptr, SEEDCG_ERR_OOM, "probe_bandwidth: the buffers do not fit");
    } catch (const std::exception& e) {
        return fail(nullptr, SEEDCG_ERR_HIP, e.what());
    }
    return SEEDCG_OK;
}

seedcg_status seedcg_probe_mfma(int32_t dtype, int32_t iters, void* stream, double* tflops) {
    if (!tflops || dtype < 0 || dtype > 1 || iters < 1)
        return fail(nullptr, SEEDCG_ERR_ARG, "probe_mfma: dtype 0 or 1, iters >= 1 and an output pointer");
    try {
        *tflops = probe_mfma(dtype, iters, (hipStream_t)stream);
    } catch (const std::bad_alloc&) {
        return fail(nullptr, SEEDCG_ERR_OOM, "probe_mfma: no room for its output");
    } catch (const std::exception& e) {
        return fail(nullptr, SEEDCG_ERR_HIP, e.what());
    }
    return SEEDCG_OK;
}

seedcg_status seedcg_train_precond(seedcg_t h, int32_t steps, int32_t n_ritz, int32_t n_lanczos, double lr, double* out) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "train_precond: null handle");
    Phase ph("seedcg_train_precond");
    return guarded(h, [&]() -> seedcg_status {
        train_precond_impl(h, steps, n_ritz, n_lanczos, lr);
        if (out) {
            out[0] = h->k_loss0;
            out[1] = h->k_loss1;
            out[2] = h->k_t_train;
            out[3] = h->k_ritz;
            out[4] = h->k_train_vecs;
            out[5] = h->k_accepted ? 1.0 : 0.0;
            for (int q = 0; q < 6; q++) out[6 + q] = h->k_judge[q];
            out[12] = h->k_choice;
            for (int q = 0; q < 5; q++) out[13 + q] = h->k_judge[6 + q];
            out[18] = h->k_judge_cg0_it;
            out[19] = h->k_judge_cg0_c;
            out[20] = h->k_judge_td;
            out[21] = h->judge_defl == 0 ? 0.0 : 1.0;
        }
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_use_precond(seedcg_t h, int32_t on) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "use_precond: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (on && !h->k_ready) throw StateError{"use_precond: the preconditioner has no weights"};
        h->p.precond = on ? 1 : 0;
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_set_precond_weights(seedcg_t h, const double* w) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "set_precond_weights: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (!w) throw ArgError{"set_precond_weights: null pointer"};
        k_set_weights(h, w);
        h->k_ready = true;
        h->k_accepted = true;
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_get_precond_weights(seedcg_t h, double* w) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "get_precond_weights: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (!w) throw ArgError{"get_precond_weights: null pointer"};
        if (!h->k_ready) throw StateError{"get_precond_weights: no weights"};
        HIPCHK(hipMemcpyAsync(w, h->kWm.p, K_NREAL * sizeof(double), hipMemcpyDeviceToHost, h->s));
        HIPCHK(hipStreamSynchronize(h->s));
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_apply_P(seedcg_t h, const double* x, double* y, int32_t nvec) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "apply_P: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (!x || !y || nvec < 1) throw ArgError{"apply_P: null pointer or nvec < 1"};
        if (!h->k_ready) throw StateError{"apply_P: the preconditioner has no weights"};
        DBuf xi, yi;
        xi.ensure(nvec * h->vec_bytes(false));
        yi.ensure(nvec * h->vec_bytes(false));
        pack_vec(false, x, xi.p, h->g.Vh, nvec, h->s);
        apply_P(h, false, xi.p, yi.p, nullptr, nvec, nvec);
        unpack_vec(false, yi.p, y, h->g.Vh, nvec, h->s);
        check_launch();
        HIPCHK(hipStreamSynchronize(h->s));
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_precond_loss_grad_band(seedcg_t h, const double* U, const double* Y, int32_t S, int32_t t0, int32_t nt,
                                            double* loss, double* grad) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "precond_loss_grad: null handle");
    return guarded(h, [&]() -> seedcg_status {
        if (!U || !Y || S < 1 || S > 32) throw ArgError{"precond_loss_grad: null pointer or S not in 1..32"};
        if (nt < 0) throw ArgError{"precond_loss_grad: negative band"};
        if (!h->k_ready) throw StateError{"precond_loss_grad: the preconditioner has no weights"};
        const int64_t N = h->N;
        h->kU.ensure((int64_t)S * N * 8);
        h->kY.ensure((int64_t)S * N * 8);
        pack_vec(true, U, h->kU.p, h->g.Vh, S, h->s);
        pack_vec(true, Y, h->kY.p, h->g.Vh, S, h->s);
        HIPCHK(hipMemsetAsync(h->kG.p, 0, K_NREAL * sizeof(double), h->s));
        const double l = k_pass(h, 0, S, grad != nullptr, true, t0, nt);
        if (loss) *loss = l;
        if (grad) {
            HIPCHK(hipMemcpyAsync(grad, h->kG.p, K_NREAL * sizeof(double), hipMemcpyDeviceToHost, h->s));
            HIPCHK(hipMemsetAsync(h->kG.p, 0, K_NREAL * sizeof(double), h->s));
        }
        HIPCHK(hipStreamSynchronize(h->s));
        return SEEDCG_OK;
    });
}

seedcg_status seedcg_precond_loss_grad(seedcg_t h, const double* U, const double* Y, int32_t S, double* loss, double* grad) {
    return seedcg_precond_loss_grad_band(h, U, Y, S, 0, 0, loss, grad);
}

seedcg_status seedcg_release_basis(seedcg_t h) {
    if (!h) return fail(nullptr, SEEDCG_ERR_ARG, "release_basis: null handle");
    return guarded(h, [&]() -> seedcg_status {
        HIPCHK(hipStreamSynchronize(h->s));
        h->basis.release();
        h->wring.release();
        h->projpart.release();
        h->vring.release();
        h->basis32.release();
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
