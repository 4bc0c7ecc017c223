/*
 * seedcg.h -- C ABI of the MI355X (gfx950) Seed-CG library.
 *
 * Solves the multiple right-hand-side systems M x^j = b^j, j = 1..nrhs (section 2 of
 * Abdel-Rehim, Morgan and Wilcox, "Seed methods for linear equations in lattice QCD
 * problems with multiple right-hand sides", LATTICE 2008), where M = A^dag A is the
 * normal operator of the even-odd preconditioned Wilson-Dirac matrix
 * A = 1 - kappa^2 H_eo H_oe (section 3).  The first right-hand side is solved by the
 * Lanczos form of CG run past convergence with periodic reorthogonalisation, every other
 * right-hand side is seeded by the Galerkin projection of Eq. (1) through the LU
 * factorisation of the Lanczos tridiagonal T of Eq. (2) (Algorithm 1, Seed-CG(m, k)),
 * and all of them are then finished with plain CG from the seeded guesses.
 *
 * Conventions shared by every call:
 *  - Array arguments are DEVICE pointers on the handle's device unless a comment says
 *    HOST; the caller owns them and keeps them valid for the duration of the call.
 *  - Complex numbers are interleaved (re, im) doubles.
 *  - Site index s = x + Lx*(y + Ly*(z + Lz*t)), parity (x+y+z+t) mod 2.  An even-site
 *    vector lists the Vh = V/2 even sites in increasing s and holds [spin 4][colour 3]
 *    complex numbers per site (12*Vh complex per vector); a batch of n vectors is n
 *    such vectors back to back.  Spin uses the Euclidean chiral basis
 *    gamma_5 = diag(1, 1, -1, -1).
 *  - Links: U[mu][s][a][b], mu = x, y, z, t, complex, U_mu(s) joins s to s + mu-hat.
 *    The fermion boundary sign in t (params.t_bc) is applied by the library.
 *  - Every call enqueues its GPU work on params.stream and returns when that work is
 *    complete.  One host thread per handle.
 *  - No C++ exception crosses this boundary; failures return a negative status and
 *    seedcg_last_error() describes the last failure of that handle.
 */
#ifndef SEEDCG_H
#define SEEDCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct seedcg_s* seedcg_t;
typedef struct seedcg_batch_s* seedcg_batch_t;

typedef enum {
    SEEDCG_OK = 0,
    SEEDCG_ERR_ARG = -1,        /* invalid argument: null pointer, odd extent, bad size     */
    SEEDCG_ERR_OOM = -2,        /* device allocation failed                                 */
    SEEDCG_ERR_HIP = -3,        /* a HIP runtime call failed                                */
    SEEDCG_ERR_BREAKDOWN = -4,  /* the method broke down and could not recover              */
    SEEDCG_ERR_NOCONV = -5,     /* max_iter reached; X holds the last iterate               */
    SEEDCG_ERR_STATE = -6       /* call out of order (e.g. seed data missing)              */
} seedcg_status;

typedef enum {
    SEEDCG_FP64 = 0,                 /* all vectors, links and arithmetic in FP64            */
    SEEDCG_MIXED_FP32 = 1,           /* FP32 stencil/basis/CG, FP64 reliable updates         */
    SEEDCG_MIXED_FP32_BF16LINKS = 2, /* as MIXED_FP32 with the sloppy links stored as BF16   */
    SEEDCG_MIXED_FP32_CG = 3         /* FP64 Lanczos, basis and seeding (Algorithm 1 as in
                                        FP64); FP32 stencil and CG with FP64 reliable updates.
                                        For operators with near-zero modes, where an FP32
                                        basis loses the seeding gain.  Deflation and the
                                        learned K run in the CG's FP32.                     */
} seedcg_prec;

typedef struct {
    int32_t dims[4];          /* Lx, Ly, Lz, Lt: each even and >= 2                              */
    double kappa;             /* hopping parameter (Wilson r = 1)                                */
    int32_t t_bc;             /* -1: antiperiodic in t, +1: periodic                             */
    int32_t prec;             /* seedcg_prec                                                     */
    int32_t m_max;            /* Krylov basis capacity (vectors); 0 = up to 3/4 of the free HBM
                                 less 4 GiB, at most 8192, allocated as the run needs it (256
                                 vectors first, then doubled at the host's checks; a batch
                                 allocates it all)                                              */
    int32_t reorth_k;         /* periodic reorthogonalisation every k iterations; 0 = never      */
    double past_factor;       /* m = ceil(past_factor * i_conv) (Algorithm 1 run past convergence);
                                 <= 0 means m = m_max exactly (the paper's fixed m)             */
    double tol;               /* relative residual ||b - M x|| / ||b|| judged in FP64            */
    int32_t reliable_every;   /* mixed precision: FP64 r = b - M x every n CG iterations         */
    int32_t seed_block;       /* seeding GEMM block b (1..32); 0 = 32                             */
    int32_t max_iter;         /* CG iterations per right-hand side in solve_rest                 */
    int32_t precond;          /* 0: none; 1: solve_rest runs PCG with the learned K K^dag once
                                 train_precond has accepted a K (seedcg_use_precond sets it)       */
    int32_t autotune;         /* 1: choose the stencil launch shapes (lanes per site, vectors per
                                 workgroup) by timing the candidates once per lattice shape;
                                 0: the fixed default (two lanes per site, one vector each).
                                 The environment can fix them instead (profiler runs, whose
                                 serialised dispatches make timing unreliable): SEEDCG_TPS and
                                 SEEDCG_VB for one-vector FP64 launches, SEEDCG_TPS_MULTI and
                                 SEEDCG_VB_MULTI for several vectors, the same with _LO for the
                                 inner precision                                                  */
    int32_t deflate;          /* 0: plain CG in solve_rest; n > 0: deflated CG (deflated PCG with the
                                 learned K) with the n (<= 24) lowest Ritz vectors of the last
                                 solve_seed's T, lifted by its stored basis; one configuration,
                                 at most 24 right-hand sides per solve_rest.  After train_precond
                                 plain CG deflates only if its judge found that cheaper            */
    void* stream;             /* hipStream_t; NULL = the null stream                             */
    int32_t basis_fp32;       /* FP64 and MIXED_FP32_CG (0 otherwise; 0, 1 or 2, else ERR_ARG):
                                 1 stores the Krylov basis in FP32 while the Lanczos recurrence, its
                                 coefficients and the LU of T stay FP64: each finished v_i is rounded
                                 into its basis slot, the seeding and reorthogonalisation projections
                                 contract the FP32 basis on the FP64 matrix cores, and the updates
                                 subtract the widened FP32 vectors from the FP64 v_i and f.  Half the
                                 basis traffic and twice the capacity.
                                 2 keeps the FP64 basis for everything the method reads from it (the
                                 seeding of Eq. (1), the Ritz vectors, the basis vectors handed out)
                                 and adds an FP32 copy of every finished v_i that only the periodic
                                 reorthogonalisation reads, as 1 does: half its traffic, orthogonality
                                 to FP32 rounding, 1.5x the memory of the FP64 basis.
                                 Single configurations only (create_batch refuses both).         */
} seedcg_params;

typedef struct {
    /* HOST arrays of length nrhs supplied by the caller (each may be NULL) */
    int32_t* iters;           /* CG iterations in solve_rest (Lanczos steps m for RHS 1 in solve_seed) */
    int32_t* matvecs;         /* applications of M                                                     */
    double* true_relres;      /* FP64 ||b - M x|| / ||b|| on return                                    */
    /* filled by the library */
    int32_t m_used;           /* Lanczos steps taken by solve_seed                                     */
    int32_t i_conv;           /* first step whose residual estimate met tol (0 = never)                 */
    int32_t seed_status;      /* 0 ok, 1 breakdown (invariant subspace), 2 indefinite, 3 capped         */
    int32_t reorth_passes;    /* Gram-Schmidt passes (a DGKS repeat counts as a pass)                   */
    double t_seed_s;          /* wall seconds of solve_seed                                            */
    double t_rest_s;          /* wall seconds of solve_rest                                            */
    /* HOST array of length nrhs supplied by the caller (may be NULL): the recursive residual
       estimate at return.  solve_seed: the D-Lanczos estimate beta_m |zeta_m / delta_m| / ||b^1|| of
       RHS 1 (Eq. 2) in entry 0, NaN for the seeded right-hand sides (no recursion ran on them);
       solve_rest: sqrt(r^dag r) / ||b|| of the CG's recursive residual (the FP64 true residual where
       the last check replaced it) */
    double* est_relres;
    /* filled by the library */
    double orth_loss_max;     /* solve_seed: largest |v_j^dag v_i| / ||v_i|| (j < i) met by a
                                 reorthogonalisation pass of Algorithm 1 before it acted; 0 without any pass */
    double t_train_s;         /* solve_rest: seconds of the train_precond whose K it applied (0 if none) */
} seedcg_report;

/* Fills *p with the defaults: t_bc = -1, FP64, m_max = 0, reorth_k = 10, past_factor = 1.5,
   tol = 1e-10, reliable_every = 50, seed_block = 32, max_iter = 100000, precond = 0, autotune = 1,
   deflate = 0. */
void seedcg_default_params(seedcg_params* p);

/* Creates a solver for one gauge configuration.  links: device, 4*V*9 complex (layout above),
   read once and repacked into the library's own copy.  On success *out owns the copy. */
seedcg_status seedcg_create(const seedcg_params* p, const double* links, seedcg_t* out);

/* y = M x for nvec even-site vectors (section 3: M = A^dag A).  x and y may not alias. */
seedcg_status seedcg_apply_M(seedcg_t h, const double* x, double* y, int32_t nvec);

/* y = M x with the inner operator the CG iterates with: FP64 for SEEDCG_FP64; FP32 vectors
   and arithmetic with FP32 or BF16-rounded links for the mixed precisions, MIXED_FP32_CG
   included (x is rounded to FP32 on entry, y is returned widened to FP64).  Same layouts and
   rules as seedcg_apply_M. */
seedcg_status seedcg_apply_M_inner(seedcg_t h, const double* x, double* y, int32_t nvec);

/* y = A x (dagger = 0) or y = A^dag x (dagger = 1), A = 1 - kappa^2 H_eo H_oe (section 3);
   the caller forms the normal-equation right-hand side b = A^dag phi with dagger = 1. */
seedcg_status seedcg_apply_A(seedcg_t h, const double* x, double* y, int32_t nvec, int32_t dagger);

/* Algorithm 1, Seed-CG(m, k): B (nrhs vectors) is read only; X holds x_0^j on entry and, on
   return, the RHS-1 iterate after m Lanczos steps in X[0] and the Galerkin-seeded guesses of
   Eq. (1) in X[1..nrhs-1].  The handle keeps the basis and T for seedcg_get_tridiag.
   A breakdown of the seed (invariant subspace or lost definiteness) is reported in
   r->seed_status and is not an error: solve_rest finishes every right-hand side. */
seedcg_status seedcg_solve_seed(seedcg_t h, const double* B, double* X, int32_t nrhs, seedcg_report* r);

/* Plain CG on every right-hand side whose FP64 true residual exceeds tol, starting from X
   (section 2: the seeded guesses are finished by a standard CG solver).  Returns
   SEEDCG_ERR_NOCONV if some right-hand side reached max_iter; X then holds its last iterate. */
seedcg_status seedcg_solve_rest(seedcg_t h, const double* B, double* X, int32_t nrhs, seedcg_report* r);

/* Traditional repeated seeding (section 2: the variant the improved method is compared with):
   system j = 1..nrhs runs Algorithm 1 from its current guess until its own residual estimate meets
   tol (m = i_conv) and seeds systems j+1..nrhs from its Krylov space; then plain CG (solve_rest)
   finishes every system whose FP64 true residual is above tol.  r->iters[j] = Lanczos steps of
   system j + its CG iterations; r->m_used = the Lanczos steps of system 1.  Same arguments and
   layouts as seedcg_solve_seed; nrhs <= 25. */
seedcg_status seedcg_solve_repeated(seedcg_t h, const double* B, double* X, int32_t nrhs, seedcg_report* r);

/* The indefinite formulation (section 2: for an indefinite matrix a QR or LQ factorisation of the
   Lanczos matrix replaces the LU of Eq. 2).  Solves A x^j = phi^j, A the even-odd Wilson matrix
   (section 3), through the Hermitian indefinite H = gamma5 A (H x = gamma5 phi, the same x as
   M x = A^dag phi without the squared condition number):
     - system 1 runs Lanczos on H with the MINRES form of the QR, past convergence and with periodic
       reorthogonalisation as in Algorithm 1 (m = ceil(past_factor * i_conv), reorth_k, m_max as
       for solve_seed; m_max = 0 takes a basis of up to 4096 vectors that fits in 75% of the free
       HBM);
     - every other system is seeded from the same Lanczos vectors by the minimal-residual projection
       of its residual onto their span;
     - plain MINRES on H finishes every system from its guess, until the FP64 true residual
       ||phi - A x|| / ||phi|| <= tol.
   Phi: device, nrhs canonical vectors [Vh][4][3] complex FP64 (layout as seedcg_solve_seed's B);
   X: device, the initial guesses on entry (zeros for x_0 = 0), the solutions on return.
   r->iters[j]: MINRES iterations (plus m for system 1); r->matvecs[j]: applications of A;
   r->true_relres[j]: ||phi - A x|| / ||phi||; m_used, i_conv, seed_status, reorth_passes, t_seed_s
   (the seeded Lanczos run) and t_rest_s (MINRES) as for solve_seed.  FP64 handles of one
   configuration only (SEEDCG_ERR_STATE otherwise); nrhs <= 25.  Scalar recurrences run on the
   host, with two synchronisations of the stream per iteration.  Returns SEEDCG_ERR_NOCONV when a
   system reached max_iter MINRES iterations first (X then holds its last iterate). */
seedcg_status seedcg_solve_indefinite(seedcg_t h, const double* Phi, double* X, int32_t nrhs, seedcg_report* r);

/* Copies the Lanczos coefficients of the last solve_seed to HOST arrays: alpha_1..alpha_m into
   alpha[0..m-1] and beta_0..beta_m into beta[0..m]; cap is the length of alpha (beta needs cap+1).
   *m receives m.  Eq. (2) defines T from these. */
seedcg_status seedcg_get_tridiag(seedcg_t h, double* alpha, double* beta, int32_t cap, int32_t* m);

/* Deflated CG (params.deflate = n > 0; the paper's motivation: seeding deflates the small
   eigenvalues, section 1): solve_rest takes W = the n lowest Ritz vectors V s_k of the last
   solve_seed's T (T s_k = theta_k s_k, Eq. 2), starts from x += W (W^dag M W)^{-1} W^dag r and keeps
   every CG direction M-orthogonal to W (p = r + b p - W (W^dag M W)^{-1} (M W)^dag r; Saad, Yeung,
   Erhel and Guyomarc'h, 2000).  Copies the Ritz values theta_k of the W in use (ascending) to the
   HOST array theta (cap entries); *n receives how many there are (0 before a deflated solve_rest). */
seedcg_status seedcg_get_ritz(seedcg_t h, double* theta, int32_t cap, int32_t* n);

/* Copies basis vector v_i (1 <= i <= m, as stored after any reorthogonalisation) to the
   device vector v in the even-site layout. */
seedcg_status seedcg_get_basis_vector(seedcg_t h, int32_t i, double* v);

/* Building blocks of Algorithm 1 (seeding of Eq. 1, reorthogonalisation) on flat complex vectors (device pointers,
   any common element order): P = V^dag R, with V nv vectors and R nr vectors of n complex
   each, P an nv x nr row-major complex matrix (device).  This is the dense contraction that
   seeds the other right-hand sides and computes the reorthogonalisation coefficients. */
seedcg_status seedcg_project(seedcg_t h, const double* Vv, int32_t nv, const double* R, int32_t nr,
                             int64_t n, double* P);

/* seedcg_project without any device allocation, for callers that cannot allocate (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
   layouts and result as seedcg_project; the split-K partials live in a static device array of
   4 MiB per GPU (2^19 doubles), allocated with the library's code object and held until the
   process ends, so nv * nr may be at most 262144 (and nr <= 24): larger sizes return
   SEEDCG_ERR_ARG without touching the GPU.  Where seedcg_project's K-chunking fits in the array
   the two return the same bits; otherwise longer K-chunks change only the summation order.
   Every call on one GPU shares that GPU's array: calls that overlap in time on one GPU (other
   host threads, other streams) race on it and must be serialised by the caller. */
seedcg_status seedcg_project_noalloc(seedcg_t h, const double* Vv, int32_t nv, const double* R, int32_t nr,
                                     int64_t n, double* P);

/* X += W E: W nw vectors, E an nw x nx row-major complex matrix (device), X nx vectors,
   n complex each (the seeding update of Eq. (1), x^j += eta^j w_i, blocked). */
seedcg_status seedcg_update(seedcg_t h, const double* W, int32_t nw, const double* E, double* X,
                            int32_t nx, int64_t n);

/* Measurement support: from now on every sample_every-th launch of the stencil kernel (the
   Wilson hop of section 3, the dominant kernel) is bracketed by a pair of hipEvents on the
   handle's stream, up to max_samples pairs; 0 turns sampling off.  Resets the counters. */
seedcg_status seedcg_set_timing(seedcg_t h, int32_t sample_every, int32_t max_samples);

/* Reads the sampled stencil timings into out[6] (HOST): number of sampled launches, their total
   milliseconds, their total algorithmic bytes (links once per launch, every spinor operand once),
   their total flops (1320 per site and vector), the number of stencil launches issued since
   set_timing, and the algorithmic bytes of all of those (sampled or not).  Launches replayed from a
   captured graph are counted once, when captured; sampling turns graph replay off. */
seedcg_status seedcg_get_timing(seedcg_t h, double* out);

/* The sampled stencil launches of get_timing, by launch kind: rows of 8 doubles in out (HOST, cap
   rows): link/spinor format (0 FP64, 1 FP32, 2 FP32 with BF16 links, 3 FP64 two-row links, 4 FP32
   two-row links), vectors per launch, 1 if the CG update is fused into the launch, lanes per site,
   vectors per workgroup, then the sampled launches, their total milliseconds and their total
   algorithmic bytes.  *n receives the number of kinds (rows beyond cap are not written). */
seedcg_status seedcg_get_timing_kinds(seedcg_t h, double* out, int32_t cap, int32_t* n);

/* y = M x applied reps times back to back to nvec (1..25) internal vectors (zeros; the stencil's
   work does not depend on the values) and timed with a pair of hipEvents on the stream: the D^dag D
   rate of section 3's operator in FP64 (inner = 0) or in the CG's inner precision (inner = 1).
   out (HOST, 4 doubles): milliseconds per application, its algorithmic bytes with the links in the
   stored format (each of the four hops reads every link once for all vectors; 120 V spinor reals per
   vector), the same with whole 3x3 links (288 V link reals), and the format code of the links (as in
   seedcg_get_timing_kinds).  One configuration per handle. */
seedcg_status seedcg_time_M(seedcg_t h, int32_t inner, int32_t nvec, int32_t reps, double* out);

/* Roofline probes (measurement, not part of the method): what this GPU achieves with the simplest
   kernels that can reach its ceilings, to read the solver's rates against measured limits beside the
   datasheet's (HBM 8 TB/s; FP64 matrix cores 78.6 TFLOP/s, FP32 157.3).
   probe_bandwidth: kind 0 copy b = a, 1 triad a = b + s c (FP64), 2 read (a sum of a); buffers of
   `bytes` each (>= 1 MiB; allocated and freed by the call, ERR_OOM if they do not fit), one untimed
   pass, then reps passes timed with a pair of hipEvents on `stream` (a hipStream_t; NULL = the null
   stream).  *gbs (HOST) receives GB/s counting each byte read or written once.
   probe_mfma: dtype 0 v_mfma_f64_16x16x4, 1 v_mfma_f32_16x16x4: four wavefronts per SIMD, each running
   eight independent chains of `iters` register-resident products; *tflops (HOST) receives TFLOP/s at
   2 * 16 * 16 * 4 flops per instruction.  Both return ERR_ARG on a bad argument. */
seedcg_status seedcg_probe_bandwidth(int32_t kind, int64_t bytes, int32_t reps, void* stream, double* gbs);
seedcg_status seedcg_probe_mfma(int32_t dtype, int32_t iters, void* stream, double* tflops);

/* ---- learned preconditioner P = K K^dag (an addition to the paper's method) -------------------
   K = R_e L_3 L_2 L_1 E_e on full-lattice 12-spinors: E_e embeds an even-site vector (zero on odd
   sites), R_e restricts to the even sites, and each layer is
       (L psi)(x) = sum_{d=0..8} (w_d (x) 1_colour)(T_d psi)(x),
   T_0 = 1, T_{+mu} psi(x) = U_mu(x) psi(x+mu), T_{-mu} psi(x) = U_mu(x-mu)^dag psi(x-mu) (with the
   t boundary sign), d = 1..4 for +x..+t and 5..8 for -x..-t.  K^dag uses L^dag = sum_d (w_d^dag
   (x) 1) T_{-d}.  Weights are 3 x 9 complex 4x4 spin matrices, [layer][d][a][b], 432 complex
   (interleaved re, im), HOST arrays.  P is applied in FP32. */

/* Trains K by `steps` Adam steps (learning rate lr, betas 0.9 / 0.999, eps 1e-8, minibatches of two
   pairs) on the loss mean_s |K K^dag y_s - u_s|^2 / |u_s|^2 over u_s = the n_ritz lowest Ritz vectors
   of T (V s, T s = theta s, from the last solve_seed) and n_lanczos stored basis vectors (normalised
   CG residuals) with their components along those Ritz vectors removed, y_s = M u_s with the CG's
   operator.  Training starts from K = 1 + kappa^2 H_eo H_oe, the first term of the Neumann series of
   A^{-1} (section 3), in every layer w_0 = 1, w_{+mu} = c (1 - gamma_mu), w_{-mu} = c (1 + gamma_mu),
   c = kappa / sqrt(3).  (K = 1 with zero hops is a saddle point where no hop weight has a gradient.)
   Plain Seed-CG then judges: RHS 2 of the last solve_seed (RHS 1 if it had one) is solved from its
   seeded guess to tol, once with plain CG and once each with PCG (P = K K^dag) under the start and the
   trained weights, by the solver of solve_rest (deflated when params.deflate > 0; plain CG also once
   without deflation then).  solve_rest iterates on all the seeded systems at once, where M's links
   are read once for every vector and K's cost is paid per vector, so each candidate's iterations are
   priced with the time of one application of M (plus one of K K^dag, plus one deflation step where
   it deflates) to that many vectors, timed with events: the cheapest wins.  The K with fewer
   iterations of the two is kept as the weights.  If a K wins it is kept and solve_rest applies it when
   precond is on; otherwise solve_rest runs plain CG (the fallback), deflated only if that was the
   cheaper plain candidate.
   out (HOST, 22 doubles, may be NULL): initial loss, final loss, training seconds, Ritz vectors used,
   training vectors, accepted (1 if a K won), the judge's seconds for plain CG, the start K and the
   trained K on one system, their iterations in the same order, the choice (0 plain CG, 1 start K,
   2 trained K), the seconds of one M and of one K K^dag on the seeded systems, the predicted
   seconds of plain CG, the start K and the trained K there, then plain CG without deflation: its
   iterations and predicted seconds (that solve stops once it has run as many iterations as would
   cost what the deflated one did, and its count is then a lower bound with seconds 1e300), the
   seconds of one deflation step on the seeded systems, and whether plain CG in solve_rest deflates
   (1) or not (0).  Each Adam step takes the loss on a band of
   two t-slices (seedcg_precond_loss_grad_band), the bands stepping through the lattice, with a step
   size that decays from lr to 0 on a half cosine; the whole-lattice loss, taken at four checkpoints,
   picks the trained weights (the start's when no checkpoint is lower, and the judge then runs the
   start K once for both).  The final loss reported is the kept weights' whole-lattice loss.
   Needs the basis of the last solve_seed (SEEDCG_ERR_STATE otherwise); one configuration per handle. */
seedcg_status seedcg_train_precond(seedcg_t h, int32_t steps, int32_t n_ritz, int32_t n_lanczos, double lr, double* out);

/* The kernels of K address a vector's field (24 Vh complex FP32) with 32-bit byte offsets: on a
   lattice with Vh >= 22.4 M sites per parity, train_precond, apply_P, the loss calls and PCG return
   SEEDCG_ERR_ARG. */

/* on != 0: solve_rest runs preconditioned CG with P = K K^dag (needs weights). */
seedcg_status seedcg_use_precond(seedcg_t h, int32_t on);

/* Sets / reads the weights of K (HOST arrays of 3*9*16 complex). */
seedcg_status seedcg_set_precond_weights(seedcg_t h, const double* w);
seedcg_status seedcg_get_precond_weights(seedcg_t h, double* w);

/* y = K K^dag x for nvec even-site vectors (device, canonical layout). */
seedcg_status seedcg_apply_P(seedcg_t h, const double* x, double* y, int32_t nvec);

/* The training loss for pairs (U, Y) of S even-site vectors (device, canonical layout, 1 <= S <= 32)
   at the current weights, and its Wirtinger gradient dL/d(conj w) (HOST, 432 complex, may be NULL). */
seedcg_status seedcg_precond_loss_grad(seedcg_t h, const double* U, const double* Y, int32_t S, double* loss, double* grad);

/* The same loss and gradient with both norms of each pair taken over the even sites of the band of
   t-slices [t0, t0 + nt) mod Lt only, the form each Adam step of train_precond takes (bands of two
   slices stepping through the lattice).  Only the slices that loss depends on are computed: K K^dag
   reaches six hops, so a band wider than Lt - 13 slices is taken as the whole lattice, as is nt = 0. */
seedcg_status seedcg_precond_loss_grad_band(seedcg_t h, const double* U, const double* Y, int32_t S, int32_t t0, int32_t nt,
                                            double* loss, double* grad);

/* ---- batches of configurations (an addition to the paper's method) -------------------------
   Many independent gauge configurations, possibly of different lattice shapes, each with nrhs
   right-hand sides, solved together: per configuration, Algorithm 1 on its first right-hand side
   with Galerkin seeding of the others, then plain CG on all of them, exactly as solve_seed
   followed by solve_rest on a handle of its own.  Configurations of one shape share every launch
   (one kernel covers all of them); shapes run concurrently on streams of their own. */

/* dims: HOST [ncfg][4]; kappa: HOST [ncfg]; links: HOST array of ncfg device pointers (each
   4*V*9 complex, layout above).  p supplies everything else (its dims, kappa and precond are
   ignored; precond must be 0).  Memory for every Krylov basis is reserved here: m_max vectors per
   configuration, or (m_max = 0) the largest common capacity that fits in 90% of the free HBM
   less 4 GiB.  nrhs: right-hand sides per configuration of every solve (1..25). */
seedcg_status seedcg_create_batch(int32_t ncfg, const int32_t* dims, const double* kappa, const double* const* links,
                                  int32_t nrhs, const seedcg_params* p, seedcg_batch_t* out);

/* B, X: HOST arrays of ncfg device pointers, each nrhs even-site vectors of that configuration
   (X holds the starting guesses and receives the solutions).  rep: HOST array of ncfg reports
   (may be NULL); its iters count Lanczos steps plus CG iterations, its matvecs every application
   of M of both phases.  Returns when every configuration is done; SEEDCG_ERR_NOCONV if some
   right-hand side reached max_iter. */
seedcg_status seedcg_solve_batch(seedcg_batch_t b, const double* const* B, double* const* X, seedcg_report* rep);

/* HOST outputs, each may be NULL: the number of shape classes, class_of[ncfg], m_cap[nclass] and
   tune[4*nclass] = the inner stencil's lanes per site and vectors per workgroup for one vector and
   for several vectors. */
seedcg_status seedcg_batch_info(seedcg_batch_t b, int32_t* nclass, int32_t* class_of, int32_t* m_cap, double* tune);

/* seedcg_set_timing / seedcg_get_timing for every shape class of the batch; the six counts and
   sums of get_timing (out[6]) are totals over the classes, whose launches may overlap in time on
   their streams, so that a sampled launch's duration includes what the other classes ran beside it. */
seedcg_status seedcg_batch_set_timing(seedcg_batch_t b, int32_t sample_every, int32_t max_samples);
seedcg_status seedcg_batch_get_timing(seedcg_batch_t b, double* out);

void seedcg_destroy_batch(seedcg_batch_t b);

/* Text of the last failure of the batch (or of the last failed create_batch when b is NULL). */
const char* seedcg_batch_last_error(seedcg_batch_t b);

/* Frees the Krylov basis (the paper allocates it for the first right-hand side only). */
seedcg_status seedcg_release_basis(seedcg_t h);

void seedcg_destroy(seedcg_t h);

/* Text of the last failure on h (or of the last failed create when h is NULL). */
const char* seedcg_last_error(seedcg_t h);

#ifdef __cplusplus
}
#endif

#endif /* SEEDCG_H */
