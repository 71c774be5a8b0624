/*
 * fsmlmc.h -- C ABI of the MI355X (gfx950) Frequency-Splitting MLMC library.
 *
 * The library computes stochastic estimates of Tr(Gamma_n Omega_p D^-1) for the
 * Wilson-Dirac operator D by Frequency Splitting (Whyte, Stathopoulos, Romero,
 * Orginos, "Optimizing Shift Selection in Multilevel Monte Carlo for
 * Disconnected Diagrams in Lattice QCD"): the inverse is split into levels with
 * shifts 0 = sigma_0 < ... < sigma_L (Sec. 2.2, eq. tele_sum_prod_disp), each
 * level is estimated with independent Z4 noise (eq. fs_trace_est) and its
 * variance with eq. practical_variance.  The hot path -- shifted BiCGStab
 * solves, Wilson dslash, BLAS-1, Z4 noise, the Wilson-line displacement and
 * the bilinear reductions -- runs in HIP kernels for gfx950.
 *
 * Conventions shared by every call
 * --------------------------------
 *  * Sites: site = x + Lx*(y + Ly*(z + Lz*t)); mu = 0,1,2,3 is x,y,z,t.
 *  * Canonical layouts (the only layouts that cross this ABI), interleaved
 *    complex128 (re, im pairs of double):
 *      gauge  [mu][site][row][col]       -- 4*V*9 complex
 *      spinor [site][spin][colour]       -- 12*V complex; n_rhs spinors are
 *                                           stored one after another.
 *  * gamma matrices: DeGrand-Rossi basis, gamma_5 = g1 g2 g3 g4 =
 *    diag(1,1,-1,-1).  Gamma_n = g1^b0 g2^b1 g3^b2 g4^b3 for n = sum b_k 2^k;
 *    this 4-bit order is the row order of the paper's appendix speedup table.
 *  * D + sigma: ((D+sigma) psi)(x) = (4 + m0 + sigma) psi(x)
 *      - 1/2 sum_mu [(1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu)],
 *    periodic, optionally antiperiodic in t.
 *  * Omega_p (Introduction: Omega_p = W Pi_p along z):
 *      (Omega_p psi)(x) = U_z(x) U_z(x+z) ... U_z(x+(p-1)z) psi(x+pz).
 *  * Pointers flagged is_device are device pointers on the context's device
 *    (e.g. a torch tensor's data_ptr); otherwise host pointers.  The caller
 *    owns every buffer it passes; the library never frees or keeps them.
 *  * Every call returns fs_status and never aborts or throws across the ABI.
 *    FS_E_ARG is returned before anything is written.  The message of the
 *    last failing call is returned by fs_last_error(NULL) for the calling
 *    thread and by fs_last_error(ctx) for the calls on a context.
 *  * Threads: calls on different contexts may come from different host
 *    threads (the library's device-memory cache is locked); calls on one
 *    context, or on a batch and its contexts, must not overlap.
 *  * Work is issued on the context's HIP stream.  Calls that return results
 *    through host pointers synchronise that stream before returning; calls
 *    whose outputs are device pointers also synchronise (the ABI is
 *    synchronous), so outputs are ready on return.
 */
#ifndef FSMLMC_H
#define FSMLMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FS_OK = 0,
    FS_E_ARG = -1,       /* invalid argument (nothing written)                 */
    FS_E_HIP = -2,       /* HIP runtime error                                  */
    FS_E_OOM = -3,       /* device allocation failed                           */
    FS_E_NOCONV = -4,    /* a solve hit max_iter; outputs and stats still set  */
    FS_E_BREAKDOWN = -5, /* unrecoverable BiCGStab breakdown (NaN/Inf)         */
    FS_E_STATE = -6      /* call out of order (e.g. no gauge uploaded)         */
} fs_status;

typedef enum { FS_F64 = 0, FS_F32 = 1, FS_F16 = 2, FS_BF16 = 3 } fs_prec;

typedef struct fs_ctx_s* fs_ctx;
typedef struct fs_batch_s* fs_batch;

/* Library version string (static storage). */
const char* fs_version(void);

/*
 * fs_struct_sizes -- sizeof of the structs of this header, in the order
 * fs_solve_params, fs_solve_stats, fs_est_params, fs_level_stat,
 * fs_total_stat, fs_est_report, fs_shift_model, into out[0 .. min(n, count)-1]
 * (out may be null); returns the count.  Bindings compare them with their own
 * layouts before the first call that takes a struct.
 */
int32_t fs_struct_sizes(int64_t* out, int32_t n);

/*
 * Message of the last failing call (never NULL; "no error" before any):
 * ctx NULL -- of the calling thread, whatever the call;
 * ctx set  -- of the calls made on that context (those whose first argument
 *             is it, fs_destroy aside).  The string is owned by the library
 *             and stays valid until the next failing call on that thread or
 *             context, or fs_destroy(ctx).
 */
const char* fs_last_error(fs_ctx ctx);

/*
 * fs_create -- one lattice instance on one device.
 *   dims[4]        Lx, Ly, Lz, Lt; each >= 2, at most 29.8M sites in all
 *                  (FS_E_ARG otherwise).
 *   t_antiperiodic 0: periodic in t; 1: antiperiodic in t.
 *   device         HIP device ordinal.
 *   hip_stream     hipStream_t to issue work on (borrowed, never destroyed);
 *                  NULL: the context creates and owns a default-priority stream.
 * The context owns its device gauge copies, work buffers and autotune table.
 */
fs_status fs_create(fs_ctx* out, const int32_t dims[4], int32_t t_antiperiodic,
                    int32_t device, void* hip_stream);
fs_status fs_destroy(fs_ctx ctx);

/* Per-process-unique instance index used in the noise counter (default 0). */
fs_status fs_set_instance(fs_ctx ctx, uint32_t instance);

/*
 * fs_upload_gauge -- copy the links (canonical layout, 4*V*9 complex128) into
 * the context, which keeps FP64, FP32, FP16 and BF16 device copies in its
 * internal structure-of-arrays layout.  Links are used as given (no
 * re-unitarisation).  Must precede every operator call (FS_E_STATE).
 * When every link is special unitary to 1e-9 (its third row equals the
 * conjugated cross product of the first two, checked on the host), the FP32
 * stencils of blocks of 4 or more systems read rows 0-1 only and rebuild row 2
 * (the context also keeps the whole links); other links are read whole.
 */
fs_status fs_upload_gauge(fs_ctx ctx, const double* links, int32_t is_device);

/*
 * fs_set_clover -- use the clover-improved Wilson operator D + C (the
 * operator of the paper's Results section) in every later call on ctx:
 *   C(x) = -(c_sw / 2) sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x),
 *   sigma_{mu nu} = (i/2) [g_mu, g_nu] (DeGrand-Rossi basis),
 *   F_{mu nu}(x)  = traceless part of (Q - Q^dagger) / (8 i), Q the sum of the
 *                   four plaquettes of the (mu, nu) plane at x, each taken
 *                   counter-clockwise.
 * With the forward hop carrying (1 - g_mu) this sign makes c_sw = 1 the
 * tree-level improvement coefficient.  The term is built on the device from the
 * uploaded links (and rebuilt by fs_upload_gauge); c_sw = 0 returns to the
 * plain operator.  Requires even extents.  With a nonzero c_sw, stencils run in
 * FP64 or FP32 storage only and solves need even_odd = 1 (the Schur complement
 * (C_e + a) - D_eo (C_o + a)^-1 D_oe, a = 4 + m0 + sigma, with the inverses
 * formed once per shift in FP64); other settings return FS_E_ARG, and so does
 * a shift at which C_o + a is singular.  The s_min bound behind err_bound then
 * also subtracts max ||C(x)|| (largest absolute row sum of its blocks).
 * Errors: FS_E_STATE before fs_upload_gauge, FS_E_ARG for a non-finite c_sw or
 * odd extents.
 */
fs_status fs_set_clover(fs_ctx ctx, double c_sw);

/*
 * fs_gauge_info -- how the uploaded links are stored.
 *   two_rows    1: FP32 stencils rebuild row 2 of each link from rows 0-1
 *               (the links are special unitary to 1e-9); 0: whole links.
 *   su3_defect  max over links and columns j of |U_2j - conj(U_0 x U_1)_j|.
 * Either output may be NULL.  FS_E_STATE before fs_upload_gauge.
 */
fs_status fs_gauge_info(fs_ctx ctx, int32_t* two_rows, double* su3_defect);

/*
 * fs_apply_dirac -- out = (D + sigma) in for n_rhs spinors (canonical layout);
 * D includes the clover term when fs_set_clover set one.
 * storage: precision the spinors and links are held in while the stencil runs
 * (inputs are rounded to it; FP64 accumulates in FP64, the others in FP32).
 * Used for parity tests and the bandwidth benchmark.
 */
fs_status fs_apply_dirac(fs_ctx ctx, double m0, double sigma, fs_prec storage,
                         const double* in, double* out, int32_t n_rhs, int32_t is_device);

/*
 * fs_apply_dirac_noalloc -- fs_apply_dirac for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same operator, kernels and launch configuration as
 * fs_apply_dirac (equal results bit for bit).
 *   in, out   device pointers on the context's device, n_rhs canonical spinors
 *             each (the caller owns them; nothing is copied to host).
 * The staged block-layout fields and work tables live in a fixed 64 MiB
 * device scratch area that the library holds on every GPU it runs on until the
 * process ends; the call allocates nothing (no hipMalloc, no allocating
 * library routine).  Limit: about 64 MiB / (2 x 192 B) = 174k site-systems in
 * FP64 storage (349k FP32, 699k FP16/BF16) per call; larger inputs return
 * FS_E_ARG before anything runs.  Every call on a GPU shares that GPU's
 * scratch area: calls that overlap on one GPU (other host threads, other
 * streams) race and must be serialised by the caller.  Work is issued on the
 * context's stream, which the call synchronises unless it is capturing a graph.
 */
fs_status fs_apply_dirac_noalloc(fs_ctx ctx, double m0, double sigma, fs_prec storage,
                                 const double* in, double* out, int32_t n_rhs);

/*
 * fs_z4_noise -- the Z4 noise vector for (seed, instance, level, sample) in
 * canonical layout: component c = (site*4+spin)*3+colour takes the 2-bit code
 * k = bits [2(c%32), 2(c%32)+1] of word (c%128)/32 of the Philox4x64-10 block
 * with counter (c/128, sample, level, instance) and key (seed, 0); the value
 * is i^k.  Bit-exact across implementations (paper eq. test: Z4 entries).
 */
fs_status fs_z4_noise(fs_ctx ctx, uint64_t seed, uint32_t instance, uint32_t level,
                      uint64_t sample, double* out, int32_t is_device);

/* fs_displace -- out = Omega_p in (one spinor, canonical layout), p >= 0. */
fs_status fs_displace(fs_ctx ctx, int32_t p, const double* in, double* out, int32_t is_device);

/*
 * fs_bilinear -- out[p][n] = y^dagger Gamma_n Omega_p x for p = 0..p_max and
 * all 16 n (complex128, host pointer), y and x one spinor each (canonical).
 * This is the displaced bilinear of eq. fs_trace_est, computed by the fused
 * hop + 4x4 spin-correlation reduction in FP64.
 */
fs_status fs_bilinear(fs_ctx ctx, int32_t p_max, const double* y, const double* x,
                      double* out, int32_t is_device);

typedef struct {
    double m0;             /* bare mass                                            */
    double tol;            /* stop when FP64 ||b - (D+sigma)x|| / ||b|| <= tol      */
    int32_t max_iter;      /* Krylov iterations per system (all precisions)        */
    fs_prec storage;       /* Krylov storage: FS_F64 plain; FS_F32/F16/BF16 mixed   */
    int32_t rhs_block;     /* RHS per block in batched launches: 1,2,4,8,16; 0=tuned */
    int32_t use_graph;     /* capture the inner iterations in a hipGraph            */
    double reliable_delta; /* mixed: FP64 reliable update when ||r|| drops by this  */
    int32_t check_every;   /* iterations between host convergence checks (0 = 8)    */
    int32_t batched;       /* 0: one system at a time; 1: all systems in one batch  */
    int32_t even_odd;      /* 1: even-odd preconditioning (every extent even): the
                              Krylov solver works on the even-site Schur complement
                              S = a - D_eo D_oe / a (a = 4 + m0 + sigma) and the
                              odd sites follow; the stopping rule is unchanged    */
    int32_t multi_shift;   /* fs_solve_shifted and fs_sample_variances only (0
                              elsewhere, else FS_E_ARG): 1 = one Krylov space per rhs
                              (per sample and source family in the sampling phase)
                              for every shift -- BiCGStab on the smallest shift with
                              the others carried along as shifted systems (their
                              residuals are multiples of the base residual; no
                              operator applications of their own); FP64 storage,
                              even_odd = 0, plain operator, at most 17 shifts; every
                              solution's FP64 true residual is checked at exit
                              (FS_E_NOCONV above tol); iteration counts are each
                              shift's own Krylov steps                             */
} fs_solve_params;

typedef struct {
    int32_t iters;             /* Krylov iterations                              */
    int32_t reliable_updates;  /* FP64 residual recomputations                   */
    int32_t status;            /* FS_OK, FS_E_NOCONV or FS_E_BREAKDOWN            */
    int32_t restarts;          /* breakdown restarts                             */
    double true_rel_residual;  /* FP64 ||b - (D+sigma)x|| / ||b|| at exit        */
} fs_solve_stats;

/*
 * fs_solve_shifted -- X[s][r] = (D + sigma[s])^-1 B[r] for s < n_shift, r < n_rhs
 * (paper eq. shifted_linear_systems), B and X canonical spinors (FP64),
 * X laid out [n_shift][n_rhs][spinor].  stats: [n_shift*n_rhs] or NULL.
 * Returns FS_E_NOCONV if any system missed tol (X still holds its iterate).
 */
fs_status fs_solve_shifted(fs_ctx ctx, const fs_solve_params* prm, const double* sigma,
                           int32_t n_shift, const double* B, int32_t n_rhs, double* X,
                           int32_t is_device, fs_solve_stats* stats);

typedef struct {
    uint64_t seed;           /* noise seed                                          */
    int32_t n_noise;         /* Z4 vectors per level (>= 2 for a variance), unless
                                n_level is given                                    */
    uint16_t gamma_mask;     /* bit n -> report Gamma_n (0 = all 16)                */
    int32_t p_max;           /* displacements p = 0..p_max, p_max < Lz              */
    fs_solve_params solve;   /* solver settings (storage FS_F64 = plain path)       */
    const int32_t* n_level;  /* NULL, or host [L+1]: N_l samples of level l, each in
                                1..2^24 (eq. fs_trace_est; e.g. from eq. num_samples
                                via fs_optimal_samples); n_noise is then ignored     */
    int32_t shared_noise;    /* 0: independent noise z_{s,l} per level (eq.
                                fs_trace_est); 1: one vector z_s for every level,
                                the Z4 vector of key (seed, instance, 0, s), as in the
                                sampling algorithm of Sec. 3.1 (levels then correlate) */
    int32_t report_fp64_error; /* 1: fill fp64_rel_err and err_bound of every level */
    int32_t hpe_order;       /* fs_sample_variances only (0 elsewhere, else FS_E_ARG):
                                k in 1..16 samples V_L of every shift with m0 + s > 0
                                through the hopping parameter expansion of order k
                                (Sec. 3.1); 0: plain samples                        */
    int32_t pad_;            /* reserved, 0                                          */
    int64_t pass_bytes;      /* batched fs_estimate / fs_batch_estimate: upper bound
                                on the device memory one pass of solves may take
                                (the systems are split into passes of equal make-up
                                within it); 0: min(half the free device memory,
                                96 GiB).  Results do not depend on it beyond the
                                rounding order of FP64 sums.                          */
} fs_est_params;

typedef struct {
    double tr_re, tr_im;     /* level mean (1/N) sum X_s                            */
    double var_paper;        /* (1/N) sum |X_s|^2 - |mean|^2 (eq. practical_variance) */
    double var_unbiased;     /* var_paper * N/(N-1)                                 */
    int64_t n;               /* samples                                             */
    double max_rel_residual; /* worst FP64 true residual of this level's solves     */
    /* With report_fp64_error (else 0):
     * fp64_rel_err  |mean - mean_64| / ((1/N) sum_s |X64_s|): deviation of this
     *               level's mean from the same estimate (same noise) solved on the
     *               plain FP64 path, which the call runs for this purpose when the
     *               storage is not FS_F64 (0 for FS_F64 storage);
     * err_bound     an upper bound on |X_s - X_s^exact| for every sample s of the
     *               level, X_s^exact being the sample with exact solves:
     *               |c| (||y~|| e_x + e_y (||x~|| + e_x)) ||Gamma_n Omega_p||, with
     *               e = ||b - (D+sigma)v~|| / s_lo(sigma) for each solve v~ (FP64
     *               true residual), c = sigma_{l+1} - sigma_l (l < L, y from the
     *               sigma_l solve) or c = 1 and e_y = 0 with y = z (l = L).
     *               s_lo(sigma) = 4 + m0 + sigma - 4 u is a lower bound on the
     *               smallest singular value of D + sigma, u the largest spectral
     *               norm of a link (each direction's hopping term is a pair of
     *               orthogonal spin projectors times maps of norm <= u), and
     *               ||Gamma_n Omega_p|| <= u^p.  +Inf when s_lo <= 0.          */
    double fp64_rel_err;
    double err_bound;
} fs_level_stat;

/*
 * fs_level_totals -- per (Gamma_n, p), the combination of the levels of an
 * estimate (paper Sec. 2.3): the FS trace estimate sum_l mean_l (eq.
 * fs_trace_est), V_FS = sum_l V_l / N_l (eq. total_var) and V_total = sum_l V_l
 * (eq. tosv), with V_l the level's eq. practical_variance and, beside them, the
 * same with the (N-1)-normalised variances; err_bound = sum_l err_bound_l.
 * Host arithmetic over the output of fs_estimate / fs_batch_estimate /
 * fs_estimate_probed for one instance: levels [(L+1)][16][p_max+1], out
 * [16][p_max+1] (Gamma_n with n_l = 0 on every level are zeroed).
 */
typedef struct {
    double tr_re, tr_im;     /* sum_l mean_l                                        */
    double v_fs;             /* sum_l var_paper_l / n_l      (eq. total_var)        */
    double v_fs_unbiased;    /* sum_l var_unbiased_l / n_l                          */
    double v_total;          /* sum_l var_paper_l            (eq. tosv)             */
    double v_total_unbiased; /* sum_l var_unbiased_l                                */
    double err_bound;        /* sum_l err_bound_l                                   */
} fs_total_stat;
fs_status fs_level_totals(const fs_level_stat* levels, int32_t L, int32_t p_max, fs_total_stat* out);

/*
 * fs_optimal_samples -- eq. num_samples: N_l = mu sqrt(V_l / C_l) with
 * mu = eps^-2 sum_l sqrt(V_l C_l), the sample counts that reach the target
 * variance V_FS = eps^2 at the least total cost sum_l C_l N_l (eq. ml_cost_shifts).
 * Each N_l is rounded up, and raised to n_min (>= 1; 2 gives every level a
 * variance), so that V_FS <= eps^2.  v_levels, c_levels: host [L+1], V_l >= 0,
 * C_l > 0 (e.g. from fs_select_shifts); eps2 > 0.  n_out: host [L+1];
 * FS_E_ARG if a count exceeds 2^24.  mu_out (nullable): mu.
 */
fs_status fs_optimal_samples(const double* v_levels, const double* c_levels, int32_t L, double eps2,
                             int32_t n_min, int32_t* n_out, double* mu_out);

typedef struct {
    int64_t systems;         /* shifted systems solved                              */
    int64_t iterations;      /* sum of Krylov iterations                            */
    int64_t reliable_updates;
    int64_t dslash_calls;    /* stencil launches (each covers a batch of systems)   */
    double max_rel_residual; /* worst FP64 true residual                            */
    double seconds;          /* wall time of the call                               */
} fs_est_report;

/*
 * fs_estimate -- per-level FS estimates for all requested Gamma_n and
 * p = 0..p_max on this context's lattice.  sigma[0..L] with sigma[0] = 0 and
 * strictly increasing (FS_E_ARG otherwise).  Level l < L uses
 * X = (sigma_{l+1}-sigma_l) y^+ Gamma_n Omega_p x with x = (D+sigma_{l+1})^-1 z,
 * y = g5 (D+sigma_l)^-1 g5 z; level L uses X = z^+ Gamma_n Omega_p (D+sigma_L)^-1 z;
 * z is the Z4 vector (seed, instance, level, sample) -- level 0 for every level
 * with shared_noise -- for samples s = 0..N_l-1 (N_l = n_level[l], or n_noise).
 *   out          [(L+1)][16][p_max+1] fs_level_stat (unrequested Gamma zeroed)
 *   samples_out  NULL or host [(L+1)][N][16][p_max+1] complex128 with N = max_l N_l:
 *                every X_s (entries s >= N_l of level l are zero)
 *   report       NULL or totals of the call
 */
fs_status fs_estimate(fs_ctx ctx, const fs_est_params* prm, const double* sigma, int32_t L,
                      fs_level_stat* out, double* samples_out, fs_est_report* report);

/*
 * fs_sample_variances -- the variance-sampling phase of shift selection (paper
 * Sec. 3.1, "Sampling the Variance", and its algorithm).  One Z4 vector z_k per
 * sample is shared by all sampling shifts: noise key (seed, instance, level
 * 0xFFFFFFFF, sample k), independent of the estimation noise.  For every shift
 * s_i: x_i = (D+s_i)^-1 z_k and y_i = (D+s_i)^-dagger z_k = g5 (D+s_i)^-1 g5 z_k
 * (a second solve: the noise is not spin-diluted).  Then, per (Gamma_n, p):
 *   single[i]     samples z_k^+ Gamma_n Omega_p x_i          (V_L(s_i), eq. sampled_single)
 *   pair[i][j]    samples y_i^+ Gamma_n Omega_p x_j, j >= i  (Vbar_l(s_i, s_j), eq. bar_vl;
 *                 V_l = (s_j - s_i)^2 Vbar_l, eq. sampled_prod)
 * each reported as mean, eq. practical_variance and the (N-1) form.
 * With prm->hpe_order = k > 0 the single samples of every shift with
 * m0 + s_i > 0 are z_k^+ Gamma_n Omega_p (H/a_i)^k x_i, where D + s_i = a_i - H,
 * a_i = 4 + m0 + s_i: the stochastic part of the hopping parameter expansion
 *   (D + s)^-1 = sum_{j<k} (H/a)^j / a + (H/a)^k (D + s)^-1,
 * whose variance is the smaller one when m0 + s is large (Sec. 3.1 uses k = 4).
 * With the clover term it is the generalized expansion: a_i is replaced by the
 * site-local A_i = C + a_i, i.e. (A_i^-1 H)^k (inverse blocks of C + a_i formed in
 * FP64 at every site; FS_E_ARG where one is singular).  The traces of the first
 * k terms are not computed here.
 *   shifts       s[0..m-1] with s[0] = 0, strictly increasing, 1 <= m <= 16
 *   prm          seed, n_noise (the N_s samples, >= 2), gamma_mask, p_max, solver
 *   single       [m][16][p_max+1]
 *   pair         [m][m][16][p_max+1]; entries with j < i are zeroed
 *   samples_out  NULL or host [m + m(m+1)/2][n_noise][16][p_max+1] complex128: the
 *                singles i = 0..m-1, then the pairs (i, j), i = 0..m-1, j = i..m-1
 *   iters_out    NULL or host [m]: mean Krylov iterations of the 2 n_noise systems of
 *                each shift, the sampled r(s_i) of the solver-cost model (Sec. 3.2)
 *   report       NULL or totals of the call
 * FS_E_ARG for invalid arguments (before any device work); FS_E_NOCONV if a
 * solve missed tol (outputs still filled).  All systems are solved in one batch.
 * n_level, shared_noise and report_fp64_error of prm are not used here (the
 * sampling noise is always shared; the error fields are zero).
 */
fs_status fs_sample_variances(fs_ctx ctx, const fs_est_params* prm, const double* shifts, int32_t m,
                              fs_level_stat* single, fs_level_stat* pair, double* samples_out,
                              double* iters_out, fs_est_report* report);

/*
 * Batches of uneven lattice instances that share persistent launches: every
 * stencil, BLAS and reduction launch of fs_batch_estimate covers the systems
 * of all instances.  Contexts must be on the same device and have gauge
 * uploaded; instance k uses noise instance index (its fs_set_instance value).
 *   out          [n][(L+1)][16][p_max+1]
 *   samples_out  NULL or host [n][(L+1)][N][16][p_max+1] complex128 (as fs_estimate)
 */
fs_status fs_batch_create(fs_batch* out, const fs_ctx* ctxs, int32_t n);
fs_status fs_batch_estimate(fs_batch b, const fs_est_params* prm, const double* sigma,
                            int32_t L, fs_level_stat* out, double* samples_out,
                            fs_est_report* report);
fs_status fs_batch_destroy(fs_batch b);

/*
 * Stencil variants (row a4 of the hot path):
 *   0  t-columns: a work-group owns wg consecutive (xyz, rhs) slots and walks
 *      t, carrying the backward-t half spinor and the centre in registers;
 *      x/y/z neighbours are loaded from memory (cache hits across lanes);
 *   1  as 0 with one wave per SIMD and the whole register file;
 *   2  LDS tiles: a work-group owns a TX x TY x TZ tile of sites (powers of
 *      two >= 2 dividing Lx, Ly, Lz; TX*TY*TZ = wg / rhs_block) and walks t;
 *      the centre spinors of each slice are staged in LDS, so only the lanes
 *      on a tile face load their outside neighbour from memory.  Where no
 *      such tile exists (e.g. an odd extent) variant 0 runs instead.
 *
 * fs_autotune -- time the stencil over a batch of n_sys systems (batches above
 * 96 are timed at 96: the resident set is bounded by the chip) for every
 * rhs_block in {1,2,4,8,16} (<= n_sys), work-group size in {64,128,256}, the
 * three variants and a cap of {none,1,2,4} resident waves per SIMD, and
 * keep the fastest (per system) in the context for this storage precision;
 * later solves, estimates and stencil calls with rhs_block/wg = 0 use it.
 * When every extent is even it then tunes the even-odd operator at that rhs
 * block: variant 0 or 2 and residency cap -1, 0, 2, 3 or 4 (fs_set_eo_tuning),
 * timing the hop plus the Schur launch as the even-odd solver issues them.
 * cache_path: text file keyed by (arch, dims, precision, batch class; "eo" and
 * the rhs block for the even-odd entry), read first and appended to; NULL
 * keeps the table in memory only.
 * best_rhs_block / best_wg may be NULL.
 */
fs_status fs_autotune(fs_ctx ctx, fs_prec storage, int32_t n_sys, const char* cache_path,
                      int32_t* best_rhs_block, int32_t* best_wg);

/*
 * fs_set_tuning -- set the stencil configuration for one storage precision
 * by hand (what fs_autotune would store): rhs_block in {1,2,4,8,16}, wg in
 * {64,128,256}, variant in {0,1,2} (see above), occ = cap on resident waves
 * per SIMD in 0..8 (0 = none).  FS_E_ARG otherwise, leaving the context
 * unchanged.  The FP64 reliable-update stencil of a mixed-precision batch
 * uses the variant of the batch's storage precision.
 */
fs_status fs_set_tuning(fs_ctx ctx, fs_prec storage, int32_t rhs_block, int32_t wg, int32_t variant,
                        int32_t occ);

/*
 * fs_time_dslash -- average duration (ms, HIP events on the context's stream)
 * of n_launch back-to-back stencil launches on n_sys systems at the given
 * storage precision, rhs_block (0 = tuned), work-group size wg (0 = tuned),
 * stencil variant ilp (0, 1, 2 as above, -1: tuned) and residency cap occ (waves per SIMD,
 * 0 = none, -1 = tuned); and the algorithmic bytes one launch moves
 * (per site and system 48 stored reals of spinor in and out, plus 72 reals of
 * links per block of rhs_block systems; FP16 adds a 4-byte scale per spinor).
 */
fs_status fs_time_dslash(fs_ctx ctx, fs_prec storage, int32_t n_sys, int32_t rhs_block,
                         int32_t wg, int32_t ilp, int32_t occ, int32_t n_launch,
                         double* avg_ms, double* bytes);

/*
 * fs_time_dslash_eo -- as fs_time_dslash for the even-odd hop D_oe / D_eo (one
 * parity out, one in; the kernel of the even-odd preconditioned solver, in the
 * context's even-odd configuration, fs_set_eo_tuning), on n_sys systems in
 * blocks of rhs_block (0 = tuned), residency cap occ (waves per SIMD, 0 =
 * none, -1 = the one the even-odd solver uses), every extent even.  bytes:
 * per output site and system 48 stored reals (+ FP16 scales), plus every link
 * of the lattice once per block: 4 links of 18 reals per site, or 12 reals per
 * link where the FP32 stencils read two rows (fs_gauge_info, rhs blocks >= 4).
 */
fs_status fs_time_dslash_eo(fs_ctx ctx, fs_prec storage, int32_t n_sys, int32_t rhs_block, int32_t occ,
                            int32_t n_launch, double* avg_ms, double* bytes);

/*
 * fs_time_dslash_eo_each -- the launches of fs_time_dslash_eo (the context's
 * even-odd configuration) timed one by one: ms_each host [n_launch] (HIP
 * events around each launch on the context's stream), for medians.
 */
fs_status fs_time_dslash_eo_each(fs_ctx ctx, fs_prec storage, int32_t n_sys, int32_t rhs_block,
                                 int32_t n_launch, float* ms_each, double* bytes);

/*
 * fs_set_eo_tuning -- the even-odd stencil of every one-parity launch of this
 * storage precision (fs_autotune stores its choice the same way):
 *   variant 0  t-streaming: a workgroup owns columns of one parity class and
 *              walks their output sites t, t+2, ...; neighbours come from memory;
 *   variant 2  x-pairs: a lane owns the two columns (2x, 2x+1) at one (y, z) and
 *              walks every t-slice, computing the output column's site while
 *              its input column's spinor -- the forward-t neighbour loaded a
 *              slice earlier -- is shared through LDS with the x/y/z neighbours
 *              of a tile of (Lx/2) x TY x TZ pairs; where no tile fits the
 *              work-group, variant 0 runs.
 *   occ        cap on resident waves per SIMD, 0..8 (0 = none), -1 = the
 *              variant's default (variant 0: 3 for FP32 rhs block 4, else none;
 *              variant 2: none).
 * The FP64 source and reconstruction kernels always stream (variant 0 mapping).
 */
fs_status fs_set_eo_tuning(fs_ctx ctx, fs_prec storage, int32_t variant, int32_t occ);

/*
 * fs_time_copy -- average duration (ms, HIP events on the context's stream) of
 * n_launch device-to-device copies of `bytes` bytes (rounded down to 16) by a
 * plain streaming kernel (one 16-byte element per lane, non-temporal): the
 * achievable-bandwidth reference for the roofline.
 */
fs_status fs_time_copy(fs_ctx ctx, uint64_t bytes, int32_t n_launch, double* avg_ms);

/* ------------------------------------------------------------------ probing and dilution
 * Paper Background (Probing) and Sec. 3.1/3.4: probing vectors from a
 * displacement-p distance-k colouring, combined with Z4 noise and full
 * spin-colour dilution.
 */

/*
 * fs_probing_colours -- greedy colouring of the symmetric part of Pi_p A^k:
 * sites x != y conflict when y lies within periodic taxicab distance k of
 * x + p z^ or of x - p z^; sites are visited in index order
 * (site = x + Lx (y + Ly (z + Lz t))) and take the smallest colour no earlier
 * conflicting site holds.  Host only.
 *   dims       Lx, Ly, Lz, Lt (each >= 2, volume <= 2^26);  0 <= p < Lz;  0 <= k <= 16
 *   colours    host [volume]: colour per site, 0..n_colours-1
 */
fs_status fs_probing_colours(const int32_t dims[4], int32_t p, int32_t k, int32_t* colours, int32_t* n_colours);

/*
 * fs_estimate_probed -- fs_estimate with probing and full spin-colour
 * dilution.  Sample s of level l sums over the 12 n_colours sources
 *   z^(j,a)(x, b) = xi(x, a) if colours[x] = j and b = a, else 0
 * (a = spin-colour index 3 spin + colour, xi the Z4 vector of key (seed,
 * instance, l, s)):
 *   level l < L:  X = sum_{j,a} (sigma_{l+1}-sigma_l) y^+ Gamma_n Omega_p x,
 *                 x = (D+sigma_{l+1})^-1 z, y = s_a g5 (D+sigma_l)^-1 z
 *                 (s_a = +1 for spins 0, 1 and -1 for spins 2, 3: g5 z = s_a z)
 *   level L:      X = sum_{j,a} z^+ Gamma_n Omega_p (D+sigma_L)^-1 z
 * so each sample costs 12 n_colours (2L+1) solves, all in one batch.
 * n_noise samples per level; n_level, shared_noise and report_fp64_error of prm
 * are not used here (the error fields are zero).
 *   colours      host [volume], values 0..n_colours-1, every colour used (1 <= n_colours <= 4096)
 *   out, samples_out, report as for fs_estimate (samples_out holds the per-sample sums)
 * FS_E_ARG for invalid arguments (before any device work); FS_E_NOCONV if a
 * solve missed tol (outputs still filled).
 */
fs_status fs_estimate_probed(fs_ctx ctx, const fs_est_params* prm, const double* sigma, int32_t L,
                             const int32_t* colours, int32_t n_colours, fs_level_stat* out, double* samples_out,
                             fs_est_report* report);

/* ------------------------------------------------------------------ shift selection
 * Paper Sec. 3.2-3.3.  The sampled variances and iteration counts of
 * fs_sample_variances (one Gamma_n, p) are carried to an evaluation set s by
 * monotone cubic Hermite interpolation (PCHIP, Fritsch-Carlson with
 * Fritsch-Butland slopes; a line through two points) of their logarithms:
 * V_L(s_k) from the m samples V_L(s^_i); Vbar_l by the paper's three-stage
 * 2-D scheme (along the first argument at each sampled second argument s^_j,
 * along the diagonal, then along the second argument at each s_i through the
 * diagonal point and the s^_j > s_i); V_l(s_i, s_k) = (s_k - s_i)^2 Vbar_l
 * (eq. sampled_prod).  Iteration counts: r(s) = r(s^_j) for
 * s^_{j-1} < s <= s^_j (eq. solver_cost_shift, 12c = 1 for undiluted noise).
 * Multilevel cost (eq. ml_cost_shifts, eps = 1):
 *   C_FS = (sum_{l=0}^{L} sqrt(C_l V_l))^2,
 *   C_l = r(sigma_l) + r(sigma_{l+1}) for l < L (a level-l sample solves at
 *   both shifts), C_L = r(sigma_L), with V_l = V_l(sigma_l, sigma_{l+1}) and V_L(sigma_L).
 * All arrays are host memory owned by the caller.
 */
typedef struct {
    int32_t m;              /* sampling shifts, 2..16                                     */
    const double* s_hat;    /* [m]: s_hat[0] = 0, strictly increasing                      */
    const double* v_single; /* [m]: sampled V_L(s_hat_i) > 0                               */
    const double* v_pair;   /* [m][m]: sampled Vbar_l(s_hat_i, s_hat_j) > 0 for j >= i;
                               entries j < i are not read                                 */
    const double* iters;    /* [m]: iteration counts r(s_hat_i) > 0                        */
    int32_t n;              /* evaluation shifts, 2..4096                                  */
    const double* s;        /* [n]: s[0] = 0, strictly increasing, containing every s_hat_i
                               exactly, s[n-1] <= s_hat[m-1] (no extrapolation)            */
} fs_shift_model;

/*
 * fs_eval_grid -- the paper's evaluation set (Sec. 3.3): 0, 4 log-spaced
 * shifts from 1e-5 to 1e-2 and 76 from 0.011 to 1, cut at s_hat[m-1], with the
 * sampling shifts inserted where missing, sorted.  Writes *n_out values to
 * s_out (capacity cap; FS_E_ARG if too small or the sampling set is invalid).
 */
fs_status fs_eval_grid(const double* s_hat, int32_t m, double* s_out, int32_t cap, int32_t* n_out);

/*
 * fs_shift_tables -- the predicted quantities on the evaluation set:
 *   v_pair_eval  NULL or [n][n]: V_l(s_i, s_k) for k > i, zero elsewhere
 *   v_single_eval NULL or [n]: V_L(s_k)
 *   r_eval       NULL or [n]: r(s_k)
 * FS_E_ARG for an invalid model (see fs_shift_model).
 */
fs_status fs_shift_tables(const fs_shift_model* model, double* v_pair_eval, double* v_single_eval, double* r_eval);

/*
 * fs_select_shifts -- eq. opt_shifts: the L shifts sigma_l = s[idx[l]],
 * 0 = idx[0] < idx[1] < ... < idx[L] <= n-1, minimising C_FS, found exactly by
 * dynamic programming over increasing indices (each level term depends on two
 * consecutive shifts), O(L n^2), on the host.  0 <= L <= n-1.
 *   idx       [L+1]
 *   c_fs      the minimum C_FS
 *   v_levels  NULL or [L+1]: V_l of the chosen levels;  c_levels NULL or [L+1]: C_l
 * With tied minima the choice among them is unspecified.
 */
fs_status fs_select_shifts(const fs_shift_model* model, int32_t L, int32_t* idx, double* c_fs, double* v_levels,
                           double* c_levels);

/*
 * fs_sweep_shifts -- the same argmin by the paper's exhaustive search over all
 * C(n-1, L) combinations, on the context's GPU (1 <= L <= 8, n <= 88,
 * C(n-1, L) <= 2^40).  Per-path sums are formed in the same order as in
 * fs_select_shifts, so equal paths give equal c_fs bit for bit; ties go to
 * the lexicographically first index tuple.
 *   idx [L+1], c_fs as above; ms NULL or the sweep kernels' GPU time (HIP events)
 */
fs_status fs_sweep_shifts(fs_ctx ctx, const fs_shift_model* model, int32_t L, int32_t* idx, double* c_fs,
                          double* ms);

#ifdef __cplusplus
}
#endif

#endif /* FSMLMC_H */
