/*
 * rfde.h -- C ABI of the MI355X (gfx950) all-at-once BDF2 solver for the Riesz space-fractional
 * diffusion equation with the eps-circulant parallel-in-time preconditioner.
 *
 * Method: Gu, Zhao, Zhao, Carpentieri, Huang, "A note on parallel preconditioning for the
 * all-at-once solution of Riesz fractional diffusion equations" (arXiv:2003.07020).
 *
 *   model (eq. (1.1) in 1D, eq. (4.1) in 2D):  u_t = kappa d^alpha u / d|x|^alpha + f,
 *       u(., 0) = u0, homogeneous Dirichlet boundary, on (a, b) x (0, T].
 *   space: fractional centred differences (eq. (2.3)-(2.4)), M interior points,
 *       h = (b - a) / (M + 1); A = -kappa h^-alpha T_x with T_x[i][j] = g_|i-j| (eq. (2.9)).
 *   time:  BDF2 with a backward-Euler first step (eq. (1.2a)-(1.2b)), N_t steps, tau = T / N_t.
 *   system (eq. (2.11)-(2.12)):  (C kron I - tau I kron A) U = F,  U = (u^1; ...; u^{N_t}).
 *   solver: flexible GMRES, right preconditioned by
 *       P_eps = C_eps kron I - tau I kron A  (eq. (3.1), the paper's alpha-circulant, here eps),
 *       applied by (a) a scaled FFT over time, (b) independent shifted solves
 *       (lambda_n I - tau A) z2_n = z1_n, (c) the inverse FFT (Section 3.1, 3.2).
 *
 * NAMING: `alpha` is the FRACTIONAL ORDER (the paper's gamma).  The circulant parameter (the
 * paper's alpha) is `circ_eps`.
 *
 * MEMORY: every array argument is a DEVICE pointer (hipMalloc'd or a torch tensor's storage) to
 * contiguous data, owned by the caller, on the plan's device, unless the comment says "host".
 * Real arrays are IEEE float64.  Complex arrays ("c128") are interleaved (re, im) float64 pairs.
 *   1D space-time vector: [N_t][M]      (time level k = 0..N_t-1 holds u at t_{k+1}, space fastest)
 *   2D space-time vector: [N_t][My][Mx] (x fastest)
 *   half spectrum:        [floor(N_t/2)+1][S] c128, S = M (1D) or My*Mx (2D)
 *
 * STREAMS: a plan enqueues all work on the hipStream_t given at creation (NULL = default stream).
 * Calls marked "async" only enqueue; rfde_solve and rfde_plan_create_* return after the work is
 * done.  A plan is not thread-safe: use one plan per host thread / stream.
 *
 * ERRORS: functions return an rfde_status.  Negative codes: nothing was written to the outputs
 * (or their content is undefined).  RFDE_ENOTCONV (positive): U holds the best iterate.
 * Arguments are validated before any device work or allocation.
 */
#ifndef RFDE_H
#define RFDE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rfde_plan_s* rfde_plan;

typedef enum {
  RFDE_OK = 0,
  RFDE_ENOTCONV = 1,     /* solver stopped at maxit; U holds the last iterate          */
  RFDE_EINVAL = -1,      /* invalid argument (range, null pointer, unsupported shape)    */
  RFDE_ENOMEM = -2,      /* device allocation failed or the plan would not fit           */
  RFDE_EHIP = -3,        /* a HIP runtime call failed                                    */
  RFDE_ENAN = -4,        /* non-finite value in the right-hand side or the iteration     */
  RFDE_EUNSUPPORTED = -5 /* valid request this build does not implement                  */
} rfde_status;

/* Spatial solver used in preconditioner step (b). */
typedef enum {
  RFDE_SPATIAL_EXACT = 0, /* 1D: dense LDL^T (no pivoting) of lambda_n I - tau A, MFMA updates */
  RFDE_SPATIAL_TAU = 1,   /* DST-I diagonalisation of the tau approximation (eq. (3.9)-(3.11),
                             eq. (4.5)); the only choice in 2D                               */
  RFDE_SPATIAL_TOEPLITZ = 2 /* 1D, FP64: the same exact solves as EXACT without factors: each
                             lambda_n I - tau A is symmetric Toeplitz, so its inverse follows
                             from its first column (Levinson-Durbin recursion at setup, O(M^2)
                             per block) by the Gohberg-Semencul formula, applied as four
                             triangular Toeplitz products by FFT of length L               */
} rfde_spatial;

typedef struct {
  double tol;          /* stop when ||F - A U|| / ||F|| <= tol (true residual). Default 1e-8   */
  int maxit;           /* max total Arnoldi steps. Default 200                                 */
  int restart;         /* FGMRES restart length m, 1..64. Default 30                           */
  double circ_eps;     /* circulant parameter in (0, 1]; <= 0 selects min(0.5, 0.5 tau)        */
  int precond_bits;    /* 64: FP64 preconditioner; 32: FP32/complex64 preconditioner (time FFTs
                          and shifted solves) inside the FP64 outer iteration. Default 64        */
  int spatial;         /* rfde_spatial. Default RFDE_SPATIAL_EXACT in 1D (TAU is forced in 2D);
                          TOEPLITZ needs precond_bits = 64 (else EUNSUPPORTED)                */
  int inner_iters;     /* 2D step (b) only.  0 (default): the tau solve of eq. (4.5), the
                          paper's method.  k in 1..16: up to k GMRES steps per frequency on the
                          exact shifted operator lambda_n I - tau A from a zero start, right-
                          preconditioned by that frequency's tau solve (an inner iteration the
                          paper leaves open; the flexible outer iteration absorbs it).  Needs
                          precond_bits = 64; 1D plans and batches return EUNSUPPORTED for k > 0.
                          Workspace: (2k + 2) complex vectors of nf x Mx x My               */
  double inner_tol;    /* >= 0.  With inner_iters > 0 and inner_tol > 0 every frequency stops
                          after the first inner step at which each has a GMRES residual
                          <= inner_tol times its right-hand side's norm; the host reads those
                          estimates after each step, so step (b) then synchronises the plan's
                          stream.  0 (default): always inner_iters steps                    */
} rfde_opts;

typedef struct {
  int iters;             /* Arnoldi steps taken (= preconditioner applications)               */
  int restarts;          /* completed restart cycles                                           */
  int converged;         /* 1 if true_rel_res <= tol                                           */
  double true_rel_res;   /* ||F - A U|| / ||F|| recomputed at exit                             */
  double ms_setup;       /* plan setup time (g_k, symbols, lambda, factorisation)              */
  double ms_solve;       /* rfde_solve wall time (RHS + FGMRES + true residual)                */
  int n_pinv;            /* preconditioner applications (steps (a)-(c)) made by the solve       */
  int n_matvec;          /* all-at-once matvecs made by the solve (Arnoldi steps, the guess's
                            residual and the true residual of every restart cycle)             */
  double ms_pinv_est;    /* ESTIMATE of the time inside preconditioner applications: only the
                            first application is timed (HIP events; timing every one would
                            idle the GPU between launches), times n_pinv.  0 for batches       */
  double ms_matvec_est;  /* ESTIMATE of the time inside matvecs, formed the same way            */
  int n_hist;            /* entries used in res_hist                                           */
  double res_hist[256];  /* estimated relative residual after each Arnoldi step (res_hist[0]=1)*/
} rfde_stats;

typedef struct {
  int dim;               /* 1 or 2                                                             */
  int M, Mx, My;         /* spatial sizes (1D: M; 2D: Mx, My, M = Mx*My)                       */
  int Nt;                /* time steps                                                          */
  int n_freq;            /* floor(Nt/2) + 1 shifted systems                                    */
  int L, Lx, Ly;         /* circulant-embedding FFT lengths                                    */
  int Mp;                /* padded order of the factored blocks (multiple of 64; 1D exact only)*/
  double h, hx, hy, tau, circ_eps;
  double coef, coef_x, coef_y; /* tau kappa / h^alpha: step-(b) matrices are lambda_n I + coef T */
  size_t factor_bytes;   /* device bytes held by the factors (0 when spatial = TAU)            */
  size_t workspace_bytes;/* other device bytes held by the plan                                */
  int precond_bits, spatial;
  double ms_setup;       /* wall time of rfde_plan_create_* (all setup steps, synchronised)   */
  double ms_factor;      /* device time of the factorisation launches (HIP events; TOEPLITZ: the
                            Levinson-Durbin recursions and generator transforms), 0 if none */
} rfde_plan_info;

/* Fill *o with the defaults listed above. */
void rfde_opts_default(rfde_opts* o);

/* Message for a status code (static string). */
const char* rfde_strerror(int status);

/*
 * Weights g_0..g_{n-1} of eq. (2.4) (omega_k^(alpha); g_{-k} = g_k by Lemma 2.1), FP64, computed
 * on the device by the ratio recurrence g_{k+1} = g_k (k - alpha/2) / (k + 1 + alpha/2) with
 * g_0 = Gamma(1+alpha) / Gamma(1+alpha/2)^2.  g: device, n doubles.  async.
 * Errors: EINVAL if alpha not in (0, 2], n < 1 or g == NULL.
 */
int rfde_gk(double alpha, int n, double* g, void* hip_stream);

/*
 * Create a 1D plan (Section 2, Section 3).  Computes g_k, the circulant-embedding symbol of
 * T_x (length L = 2^ceil(log2(2M-1)), scaled by tau kappa / h^alpha), eps, s_j = eps^{j/N_t},
 * lambda_n (eq. (3.3)) and, for RFDE_SPATIAL_EXACT, the LDL^T factors of the floor(N_t/2)+1
 * shifted blocks lambda_n I + (tau kappa / h^alpha) T_x.  Synchronous.
 *   alpha in (1, 2], kappa > 0, b > a, 1 <= M <= 4096, T > 0, and N_t >= 2 either a power of
 *   two up to 8192 or any other count up to 4096 (its time DFTs then use Bluestein's chirp-z
 *   form with a power-of-two length >= 2 N_t - 1); opts may be NULL (defaults).
 *   RFDE_SPATIAL_TAU accepts every M: its DST-I runs as one FFT of length 2(M+1) when that is a
 *   power of two, else by the chirp-z form (two cyclic convolutions of a power-of-two length
 *   >= 2M - 1, and a work array of the half spectrum's size).
 * Memory: the factors take nb * T(T+1)/2 * 4096 complex entries (T = ceil(M/64); 16 bytes
 * each in FP64, 8 in FP32; nb = n_freq, or n_freq - 1 for an even N_t, whose real blocks 0 and
 * N_t/2 share one complex-sized block): 69.8 GB for M = 4095, N_t = 1024 in FP64.
 * Errors: EINVAL on any range violation; ENOMEM if factors plus workspace exceed free device memory (checked before allocating);
 * EHIP on a runtime failure.  On error *plan is set to NULL.
 */
int rfde_plan_create_1d(rfde_plan* plan, double alpha, double kappa, double a, double b, int M,
                        int Nt, double T, const rfde_opts* opts, void* hip_stream);

/*
 * Create a 2D plan (eq. (4.1)-(4.5)): A = -(c_x T_x (along x) + c_y T_y (along y)),
 * c = kappa / h^alpha, h_x = (bx-ax)/(Mx+1), h_y = (by-ay)/(My+1); Mx, My in [1, 4096]; step
 * (b) uses the 2D tau/DST diagonalisation (no factors are stored), each axis's DST-I as in the
 * 1D tau solver (FFT of length 2(n+1) or the chirp-z form).  Other arguments as in
 * rfde_plan_create_1d.
 */
int rfde_plan_create_2d(rfde_plan* plan, double alpha_x, double alpha_y, double kappa_x,
                        double kappa_y, double ax, double bx, double ay, double by, int Mx, int My,
                        int Nt, double T, const rfde_opts* opts, void* hip_stream);

/* Release every device buffer the plan owns (to the library's device-memory cache: mapping
 * fresh device memory costs ~10-20 ms per GB, so freed blocks are reused by later plans and
 * batches; see rfde_release_cached_memory).  Accepts NULL. */
int rfde_plan_destroy(rfde_plan plan);

/* Return every cached device block to the HIP runtime (hipFree); returns the bytes released.
 * A failed allocation inside the library does this by itself before giving up. */
size_t rfde_release_cached_memory(void);

/* Sizes and derived parameters of a plan (host struct). */
int rfde_plan_get_info(rfde_plan plan, rfde_plan_info* info);

/* What rfde_plan_export copies out. */
typedef enum {
  RFDE_EXPORT_GK = 0,      /* g_0..g_{M-1} (2D: g^x then g^y), double                         */
  RFDE_EXPORT_SYMBOL = 1,  /* 1D: L/2+1 doubles, the real spectrum of the scaled circulant
                              embedding, already divided by L; 2D: Lx/2+1 then Ly/2+1          */
  RFDE_EXPORT_LAMBDA = 2,  /* n_freq c128: lambda_n, n = 0..floor(N_t/2)                       */
  RFDE_EXPORT_SCALE = 3,   /* N_t doubles: s_j = eps^{j/N_t}                                   */
  RFDE_EXPORT_FACTOR = 4,  /* factor of block `index`: Mp*Mp c128 (FP32 plans: complex64) dense
                              row-major matrix holding unit-lower L (strict lower part) and D
                              (diagonal) with B = L D L^T; upper part zero                      */
  RFDE_EXPORT_TAU_SIGMA = 5,/* tau eigenvalues sigma_i of T (eq. (3.10)), unscaled: M doubles
                              (2D: Mx then My); plans with spatial = TAU only, else EINVAL    */
  RFDE_EXPORT_TOEPLITZ_X = 6/* first column of (lambda_n I + coef T)^{-1} for n = index: M c128;
                              plans with spatial = TOEPLITZ only, else EINVAL                 */
} rfde_export_what;

/* Copy plan data into the device buffer dst (sizes above).  index: block for FACTOR.  async. */
int rfde_plan_export(rfde_plan plan, int what, int index, void* dst);

/* Step (a5): F_1 = tau f^1 + u0, F_2 = tau f^2 - u0/2, F_k = tau f^k (eq. (2.11)).
 * u0: [S], f: [N_t][S] (f^1..f^{N_t}), F: [N_t][S].  F may alias f.  async. */
int rfde_build_rhs(rfde_plan plan, const double* u0, const double* f, double* F);

/* Step (a6): y = (C kron I - tau I kron A) v (Section 3.2).  v, y: [N_t][S], y must not alias v.
 * async. */
int rfde_apply_A(rfde_plan plan, const double* v, double* y);

/* Step (a7), preconditioner step (a): z1_n = sum_j theta^{n j} eps^{j/N_t} v_j,
 * theta = exp(+2 pi i / N_t), n = 0..floor(N_t/2).  v: [N_t][S] real; z1: [n_freq][S] c128.
 * (FP32 plans compute it in FP32 and write it widened to c128.)  async. */
int rfde_pinv_step_a(rfde_plan plan, const double* v, void* z1);

/* Step (a8), preconditioner step (b): z2_n = (lambda_n I + coef T)^{-1} z1_n for every n.
 * z1, z2: [n_freq][S] c128; may alias (in place).  Exact 1D solver with an even N_t: levels 0
 * and N_t/2 are taken as real (as step (a) produces them from real data; their imaginary parts
 * are ignored and written as zero), since those two blocks are real and are solved as a pair
 * in real arithmetic.  2D with opts.inner_iters = k > 0: z2_n is the k-step GMRES solution of
 * the exact shifted system (see rfde_opts).  async, except with inner_tol > 0 (it then
 * synchronises the plan's stream once per inner step). */
int rfde_pinv_step_b(rfde_plan plan, const void* z1, void* z2);

/* Step (a9), preconditioner step (c): extend by z2_{N_t-n} = conj(z2_n) (imaginary parts of
 * z2_0 and, for even N_t, z2_{N_t/2} are ignored), v_j = eps^{-j/N_t} (1/N_t)
 * sum_n theta^{-n j} z2_n.  z2: [n_freq][S] c128; v: [N_t][S] real.  async. */
int rfde_pinv_step_c(rfde_plan plan, const void* z2, double* v);

/* Steps (a7)-(a9): z = P_eps^{-1} v.  v, z: [N_t][S]; z may alias v.  async (as step (b)). */
int rfde_apply_Pinv(rfde_plan plan, const double* v, double* z);

/*
 * Steps (a5)-(a10): solve the all-at-once system with FGMRES(m) right-preconditioned by P_eps.
 * u0: [S], f: [N_t][S], U_init: [N_t][S] initial guess or NULL (zero), U: [N_t][S] output;
 * tol <= 0 uses the plan's opts.tol.  stats: host pointer or NULL.  Synchronous.
 * A guess whose residual ||F - A U_init|| is not below ||F|| is discarded (zero start).
 * Returns OK, ENOTCONV (U = last iterate), ENAN (non-finite F or residual), EINVAL, EHIP.
 */
int rfde_solve(rfde_plan plan, const double* u0, const double* f, const double* U_init,
               double* U, double tol, rfde_stats* stats);


/* ------------------------------------------------------------------------------------------
 * Launch-shape tuning (not in the paper).  Every variant computes the same result; only the
 * work split differs.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
  int time_variant;      /* time FFTs: NB >> v transforms per workgroup (v = 0..2), or 3: NB
                            with 1024 threads and radix-8 passes (power-of-two N_t only);
                            0 takes the half width when the full one leaves CUs idle, and
                            the shape of 3 for FP64 forward transforms at N_t >= 1024        */
  int matvec_variant;    /* 0 three-stage register FFT (L >= 256); LDS Stockham passes with
                            1 the default workgroup size, 2 the other size, 3 radix 8         */
  int trsv_grid_cap;     /* 0 one workgroup per block; else persistent workgroups             */
  int from_cache;        /* bit 0 time, bit 1 matvec, bit 2 trsv: taken from the cache        */
  double ms_time[4];     /* timed forward + inverse time FFT per variant (0 when cached)      */
  double ms_matvec[4];   /* timed matvec per variant                                           */
  int trsv_caps[5];      /* candidate caps                                                      */
  double ms_trsv[5];     /* timed triangular solves per cap (-1: not applicable)               */
} rfde_tune_report;

/*
 * Time every variant of the plan's per-iteration kernels on its own buffers and keep the
 * fastest for later calls on this plan.  Choices are cached per shape in the process and, if
 * the environment variable RFDE_TUNE_CACHE names a file, appended to it and read back by later
 * processes.  Synchronous; overwrites the plan's work buffers (not its factors).  report may be
 * NULL.  Errors: EINVAL (NULL plan), EHIP.
 */
int rfde_plan_autotune(rfde_plan plan, rfde_tune_report* report);

/* Set the variants directly (time_variant 0..3, matvec_variant 0..3, trsv_grid_cap >= 0). */
int rfde_plan_set_variants(rfde_plan plan, int time_variant, int matvec_variant,
                           int trsv_grid_cap);

/* ------------------------------------------------------------------------------------------
 * Batched solves (not in the paper; a growth direction of this library).  Many independent 1D
 * problems of Section 2 with their own alpha, kappa, domain, M, N_t and T, each solved exactly
 * as rfde_solve does (its own epsilon-circulant preconditioner of Section 3, exact shifted
 * solves, FGMRES(m) to the true relative residual), but with every step launched for all
 * instances at once: the factorisations of all blocks of all instances share one launch per
 * tile column; Arnoldi step j of all instances is one HIP graph, replayed across restart
 * cycles; one host synchronisation per Arnoldi step for the whole set.
 * ------------------------------------------------------------------------------------------ */

/* One problem: u_t = kappa R^alpha u + f on (a, b) x (0, T], M interior points, N_t steps. */
typedef struct {
  double alpha, kappa, a, b, T;
  int M, Nt;
} rfde_instance;

typedef struct rfde_batch_* rfde_batch;

typedef struct {
  int count;              /* instances                                                        */
  int waves;              /* memory waves (groups whose factors fit the budget together)      */
  int max_wave;           /* most instances in one wave (<= 64)                               */
  size_t budget_bytes;    /* device-memory budget used to form the waves                      */
  size_t wave_bytes_max;  /* estimated device bytes of the largest wave                        */
  size_t instance_bytes_max; /* estimated device bytes of the largest instance                 */
  size_t device_bytes_max;/* device bytes actually held by the largest wave of the last solve */
  double ms_setup;        /* last rfde_batch_solve, summed over waves: plan setup + factors   */
  double ms_plans;        /* ... of which: creating the instances' plans (allocation, g_k,   */
  double ms_tune;         /*     symbols, lambda) and tuning their launch shapes              */
  double ms_factor;       /* ... device time of the factorisation launches (HIP events)       */
  double ms_solve;        /* ... right-hand sides + FGMRES + true residuals (wall)            */
  int graph_launches;     /* ... Arnoldi-step graphs launched                                 */
} rfde_batch_info;

/*
 * Create a batch of `count` instances.  Every instance is validated as rfde_plan_create_1d
 * validates its arguments (EINVAL, EUNSUPPORTED); opts apply to all of them (spatial must be
 * RFDE_SPATIAL_EXACT, else EUNSUPPORTED).  mem_budget = device bytes the batch may hold at
 * once (0: a quarter of the free memory, or the largest instance if that is more; never more
 * than 95% of it); instances are packed, largest first, into waves of at most 64 instances
 * that fit it; ENOMEM if one instance alone does not fit.  The first rfde_batch_solve maps one
 * device buffer of the largest wave's size, which all waves and later solves reuse; it is
 * released by rfde_batch_destroy.  hip_stream: the caller's stream (rfde_batch_solve
 * synchronises with it on entry and runs on a stream of its own, which graph capture needs).
 */
int rfde_batch_create(rfde_batch* batch, int count, const rfde_instance* inst,
                      const rfde_opts* opts, size_t mem_budget, void* hip_stream);

/*
 * Solve every instance.  u0[i] ([M_i] FP64), f[i] ([N_t,i][M_i] FP64, levels 1..N_t) and U[i]
 * ([N_t,i][M_i] FP64) are device pointers (host arrays of `count` pointers).  stats may be NULL
 * (else `count` entries; ms_setup / ms_solve are those of the instance's wave).  Synchronous.
 * Returns OK when every instance converged, ENOTCONV if some stopped at maxit (their U holds
 * the last iterate), ENAN if some met a non-finite value, EINVAL/ENOMEM/EHIP otherwise.
 */
int rfde_batch_solve(rfde_batch batch, const double* const* u0, const double* const* f,
                     double* const* U, rfde_stats* stats);

/* Grid caps of the batched factor and triangular-solve launches: 0 = one workgroup per work
 * item; c > 0 = at most c persistent workgroups looping over the items. */
int rfde_batch_set_grid_caps(rfde_batch batch, int factor_cap, int trsv_cap);

/* Tune the launch shapes of every instance's time FFTs (what bit 0) and matvec (bit 1) as
 * rfde_plan_autotune does, before its wave is solved (0: built-in shapes, the default). */
int rfde_batch_set_autotune(rfde_batch batch, int what);

/* Wave index of instance `index` (>= 0), or EINVAL. */
int rfde_batch_wave_of(rfde_batch batch, int index);

int rfde_batch_get_info(rfde_batch batch, rfde_batch_info* info);
int rfde_batch_destroy(rfde_batch batch);

/* ------------------------------------------------------------------------------------------
 * Learned initial guess (not in the paper; a growth direction of this library).
 *
 * Because the all-at-once solution (eq. (2.11)) is linear in the data, the solution for data
 * u0 = sum_k a_k sin(k pi x), f = e^{-t} sum_k b_k sin(k pi x) is sum_k c_k G_k with G_k the
 * solution for the k-th unit data component.  A small network predicts the G_k, in the first Ks
 * sine modes of x, from the problem parameters:
 *   phat = (p - mu)/sd; h1 = tanh(W1 phat + b1); h2 = tanh(W2 h1 + b2); g = W3t h2 + b3,
 *   g = (G_1, ..., G_nsrc) each [Nt][Ks], NOUT = nsrc * Nt * Ks; loss = mean (g - y)^2.
 * FP32 master weights; the output layer's products use a BF16 copy of W3t on BF16 MFMAs with
 * FP32 accumulation.  All pointers are device pointers owned by the caller (contiguous,
 * row-major: W1 [H1][Pin], W2 [H2][H1], W3t [NOUT][H2]).  Limits: 1 <= B <= 64, Pin <= 64,
 * H1 <= 256, 16 <= H2 <= 256 with H2 % 16 == 0, NOUT % 16 == 0.  All calls are async on the
 * given stream; `ws` is a device workspace of rfde_mlp_workspace_bytes(m, B) bytes.
 * ---------------------------------------------------------------------------------------- */
typedef struct {
  int Pin, H1, H2, NOUT;
  float *W1, *b1, *W2, *b2, *W3t, *b3;      /* FP32 parameters                             */
  unsigned short* W3t_bf16;                 /* BF16 copy of W3t (kept in step by Adam)     */
  float *mW1, *vW1, *mb1, *vb1, *mW2, *vW2, *mb2, *vb2, *mW3, *vW3, *mb3, *vb3; /* Adam     */
  const float *mu, *sd;                     /* feature standardisation, Pin each           */
} rfde_mlp;

/* Workspace bytes needed for batch size B. */
size_t rfde_mlp_workspace_bytes(const rfde_mlp* m, int B);

/* g[B][NOUT] = network(feats[B][Pin]).  Errors: EINVAL on limits or NULL pointers. */
int rfde_mlp_forward(const rfde_mlp* m, const float* feats, int B, float* g, void* ws,
                     void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, serving loops
 * that produce initial guesses, harnesses that forbid hipMalloc): rfde_mlp_forward without the
 * workspace argument.  Same kernels and result as rfde_mlp_forward (bit for bit); the
 * activations (phat, h1, h2 and h2 in BF16: B (Pin + H1 + H2) 4 + B H2 2 bytes, at most 180 KiB
 * within the limits above) live in a fixed device array of rfde_mlp_forward_noalloc_max_bytes()
 * = 256 KiB per GPU, held until the process ends.  Calls no allocator.  Every call on one GPU
 * shares that array, so calls that overlap on one GPU (concurrent streams or host threads) race;
 * calls in one stream are ordered and safe.  Errors: EINVAL as rfde_mlp_forward (and if the
 * activations would exceed the array), EUNSUPPORTED for a device index >= 64, EHIP if the
 * array's device address cannot be obtained.
 */
int rfde_mlp_forward_noalloc(const rfde_mlp* m, const float* feats, int B, float* g,
                             void* stream);
size_t rfde_mlp_forward_noalloc_max_bytes(void);

/* Forward, loss (device float *loss), and the gradients of the loss in `grads` (flat FP32,
 * order W1, b1, W2, b2, W3t, b3); parameters are not changed. */
int rfde_mlp_grads(const rfde_mlp* m, const float* feats, const float* y, int B, float* g,
                   float* grads, float* loss, void* ws, void* stream);

/* One Adam step (lr, beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias correction with step t >= 1)
 * on targets y[B][NOUT]; *loss receives the loss before the step.  Needs the Adam moments. */
int rfde_mlp_train_step(const rfde_mlp* m, const float* feats, const float* y, int B, float* g,
                        float lr, int t, float* loss, void* ws, void* stream);

/* dst[i] = src[i] rounded to BF16 (round to nearest even), i < n (device). */
int rfde_f32_to_bf16(size_t n, const float* src, unsigned short* dst, void* stream);

/* S[i][s] = sin((s+1) pi (i+1) / (M+1)), i < M, s < Ks <= 256: the DST-I vectors (device). */
int rfde_sine_table(int M, int Ks, double* S, void* stream);

/* U[t][i] = sum_s (sum_k coef_scaled[k] g[k][t][s]) S[i][s]: the guess for data coefficients
 * coef (coef_scaled = coef * per-component output scale), U: [Nt][M] FP64 (device). */
int rfde_guess_assemble(int nsrc, int Nt, int Ks, int M, const float* g, const double* coef_scaled,
                        const double* S, double* U, void* stream);

/* Y[t][s] = factor (2/(M+1)) sum_i U[t][i] S[i][s]: the coefficients of U in the first Ks sine
 * modes, times `factor` (training targets use 1/mode^2). */
int rfde_project_sine(int Nt, int M, int Ks, const double* U, const double* S, double factor,
                      float* Y, void* stream);

/* ------------------------------------------------------------------------------------------
 * Measurement probe (not part of the method): the sustained matrix-core rate of one instruction
 * form, from a kernel that issues only that instruction on register-resident operands (2048
 * workgroups of 4 waves, 8 independent accumulator chains per wave, `iters` rounds), timed with
 * HIP events after one warm-up launch.  kind 0: v_mfma_f64_16x16x4f64 (FP64, the factorisation),
 * 1: v_mfma_f32_16x16x4f32 (FP32 factorisation), 2: v_mfma_f32_16x16x16bf16_1k (the guess
 * network's output layer), 3: v_mfma_f32_16x16x32_bf16.  *tflops: host.  Synchronous; allocates
 * a 2 MiB output buffer on the stream.  Errors: EINVAL (kind, iters outside 1..2^20, NULL), EHIP.
 * ------------------------------------------------------------------------------------------ */
int rfde_probe_mfma(int kind, int iters, double* tflops, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RFDE_H */
