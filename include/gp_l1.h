/*
 * gp_l1.h - C ABI of the MI355X (gfx950) gradient-projection solver for
 * l1-constrained least squares.
 *
 * Problem (the constrained form (2) of Section 1 of Loris, Bertero, De Mol,
 * Zanella, Zanni, "Accelerating gradient projection methods for
 * l1-constrained signal recovery by steplength selection rules"):
 *
 *     x~(rho) = argmin_{ ||x||_1 <= rho }  f(x),   f(x) = ||K x - y||^2
 *
 * with K an n x p matrix, y in R^n, x in R^p.  f carries no 1/2 factor, so
 * grad f(x) = 2 K^T (K x - y).  The method is Algorithm 1 of Section 3
 * (gradient projection along the feasible direction d = P(x - alpha g) - x
 * with an Armijo backtracking line search) driven by the adaptive
 * Barzilai-Borwein alternation of Algorithm 2 (equation (5)), with the
 * parameter values that close Section 3 as defaults.
 *
 * Conventions shared by every call:
 *  - Layout: K is row-major, element (i, j) at K[i * ldk + j], ldk >= p.
 *    Batched right-hand sides and solutions are stored one problem per row:
 *    Y[b * ldy + i], X[b * ldx + j].
 *  - Precision: the dtype names K's storage.  Vectors (y, x0, x_out, Y, X,
 *    v, h) are double for GP_F64 and float for GP_F32 / GP_BF16.  Scalars
 *    (steplengths, threshold sums, line-search tests, objective) are double
 *    on the device for every dtype.  GP_BF16 stores K as raw bfloat16 bits
 *    (uint16) and accumulates products in float.
 *  - Memory: every data pointer is a DEVICE pointer owned by the caller
 *    (for example a torch tensor's data_ptr()), except the ones marked
 *    "host".  The library never frees caller memory.  Inputs are read only;
 *    an output may alias the matching input (x_out == x0).
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 *    stream).  Work is enqueued on it; calls that fill a host result struct
 *    synchronise that stream before returning.
 *  - Errors: every call returns a gp_status.  Values >= 0 are solver
 *    outcomes with a valid x; negative values mean no valid output, and
 *    gp_last_error() describes the problem.  No C++ exception crosses this
 *    boundary.  A handle is used by one host thread at a time.
 */
#ifndef GP_L1_H
#define GP_L1_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { GP_F64 = 0, GP_F32 = 1, GP_BF16 = 2 } gp_dtype;

typedef enum {
    GP_OK_TOL = 0,          /* relative objective change fell below tol        */
    GP_STATIONARY = 1,      /* P(x - alpha g) == x, or grad'd >= 0 in rounding  */
    GP_MAX_ITER = 2,        /* iteration budget used up                         */
    GP_REACHED_TARGET = 3,  /* f(x) <= opts.f_target, checked in double         */
    GP_BACKTRACK_LIMIT = 4, /* Armijo test failed after backtrack_cap reductions */
    GP_E_ARG = -1,          /* bad argument (sizes, rho, tol, null pointer)      */
    GP_E_NONFINITE = -2,    /* NaN/Inf in K, y or arising during the run         */
    GP_E_HIP = -3,          /* a HIP runtime call failed                         */
    GP_E_NOMEM = -4,        /* workspace allocation failed                       */
    GP_E_UNSUPPORTED = -5   /* shape outside what the kernels handle             */
} gp_status;

/* gp_opts.fused_cfg value of the K pass over column panels (two launches,
 * K read twice; see gp_l1_solve). */
#define GP_FUSED_PANELS 13

/* Solver options.  gp_opts_default() fills the values the paper uses for
 * GPSS (end of Section 3): M = 1, theta = 0.5, beta = 1e-4,
 * alpha_min = 1e-10, alpha_max = 1e10, tau1 = 0.5, M_alpha = 2. */
typedef struct {
    int32_t M;            /* line-search memory: f_max over the last M values, 1..16 */
    double theta;         /* backtracking factor, (0,1)                        */
    double beta;          /* sufficient-decrease constant, (0,1)               */
    double alpha_min;     /* steplength clamp, 0 < alpha_min < alpha_max       */
    double alpha_max;
    double tau1;          /* initial alternation threshold, (0,1)              */
    int32_t M_alpha;      /* alpha^(2) window = last M_alpha+1 iterations, 0..3 */
    int32_t max_iter;     /* iteration budget (>= 0)                           */
    double f_target;      /* stop once f <= f_target (ignored if < 0).  The iteration
                             tracks f with FP32-accurate products, so a stop it
                             proposes is checked: f is recomputed in double from
                             the stored K, y and the returned x (narrowed to the
                             vector dtype); if that exceeds f_target the problem
                             iterates on with a lower internal target.  A result
                             with GP_REACHED_TARGET therefore has result.f, the
                             double value, <= f_target. */
    int32_t refresh_every;/* recompute r = Kx - y, g = 2K^T r every R iters (0 = never) */
    int32_t backtrack_cap;/* max reductions of the line-search step            */
    int32_t chunk;        /* iterations enqueued between host status polls     */
    int32_t fused_cfg;    /* tuning: fused K/K^T kernel shape, 1..12, or GP_FUSED_PANELS
                             (0 = automatic) */
    int32_t fused_grid;   /* tuning: workgroups (row slabs) of that kernel (0 = automatic) */
    int32_t profile;      /* k > 0: time the fused K/K^T launch of every k-th iteration with HIP
                             events stamped by the launch itself (result.t_fused_ms over
                             result.n_fused launches); 0 = off */
    int32_t fused_interleave; /* tuning: 1 = row blocks dealt round-robin to workgroups, 0 = slabs */
    const double* f_targets;  /* batched calls: host array of one f_target per problem (NULL = f_target
                                 for all); must stay valid for the call; ignored by gp_l1_solve */
    int32_t x0_fallback;      /* 1: when x0 is given and f(P(x0)) >= f(0) = ||y||^2, start from x = 0
                                 instead (result.x0_rejected = 1).  Shared-K batches test it on the
                                 device in their first residual pass, gp_l1_solve with two extra
                                 residual passes; uneven batches return GP_E_UNSUPPORTED. */
    int32_t graph;            /* 1 = replay a captured HIP graph of one chunk of iterations
                                 (refresh_every iterations, or chunk when refresh_every is 0;
                                 iterations outside whole chunks run as plain launches), with the
                                 status poll after each chunk.  gp_l1_solve keeps its graph in the
                                 handle while the problem's arguments are unchanged; the batched
                                 solvers capture per call (shared K: again whenever finished
                                 problems leave the launches).  Results are identical to graph = 0.
                                 Not with profile. */
    /* tuning of the batched solvers (0 = automatic; the autotuner fills them) */
    int32_t batch_splitk;     /* shared K: reduction chunk of the two GEMMs, a multiple of 32
                                 (about 1024 when 0); rounded down to divide the padded size */
    int32_t batch_rows_t;     /* shared K: threads of the per-problem row kernel: 256, 512, 1024 */
    int32_t batch_cols_t;     /* shared K: threads of the per-problem column kernel: 256, 512, 1024
                                 (a width with no compiled register shape for p: GP_E_ARG) */
    int32_t var_item_rows;    /* uneven batches: rows of K per work item of the fused pass, 16..1024
                                 (64 when 0) */
    int32_t batch_gemm_depth; /* shared bf16 K: k-steps of GEMM loads in flight, 1 or 2 (1 when 0) */
    int32_t batch_gemm_tile;  /* shared bf16 K: the GEMM output tile, 128 x 128 (0 or 128), 256 x 128
                                 (256: one k-step in flight, about half the reduction chunk) or
                                 128 x 64 (64); whatever is set, 128 x 64 once at most 128 problems
                                 run.  Every tile gives the same bits at the same reduction chunk;
                                 batch_gemm_depth = 2 goes with 128 x 128 only (GP_E_ARG). */
    int32_t lookahead;        /* gp_l1_solve without graph: k > 0 = keep at most k iterations enqueued
                                 ahead of the device, which posts every completed update to a
                                 host-mapped word of the handle, and poll the state only once a stop
                                 is posted (a stop leaves at most about k iterations of launches
                                 that return at once, and no status polls before it); 0 = `chunk`
                                 iterations between status polls.  Results are identical. */
    int32_t var_wave_rows;    /* uneven batches with float or bf16 K: 0 or 1 = items of problems with
                                 p <= 1024 run the fused pass one row per wave (dots reduced within
                                 the wave, no barrier per row); -1 = the workgroup-wide pass for
                                 every item.  The two round differently (both FP32-level). */
    double* trace;            /* gp_l1_solve: device ring of trace_cap records of GP_TRACE_FIELDS
                                 doubles, written by the device as it iterates (NULL = off, no
                                 cost).  Update k (1-based) goes to record (k - 1) % trace_cap:
                                 {k, f after the update, alpha of its projection, lambda of the
                                 line search, backtracks, tau and rule of the steplength rule that
                                 gave alpha (Algorithm 2: 0 alpha_max, 1 BB1 alpha^(1), 2 the
                                 windowed alpha^(2); -1 for the first update, whose alpha is
                                 alpha_0), mu of the projection (0 inside the ball), the size of
                                 its active set {|v_i| > mu} (-1 inside the ball), the threshold
                                 search's passes}.  Ignored by the batched solvers. */
    int32_t trace_cap;        /* records in `trace` (> 0 when trace is set)             */
} gp_opts;

/* doubles per record of gp_opts.trace */
#define GP_TRACE_FIELDS 10

typedef struct {
    int32_t status;       /* gp_status                                         */
    int32_t iters;        /* accepted updates                                  */
    int32_t backtracks;   /* total step reductions                             */
    int32_t projected_x0; /* 1 if x0 was outside the ball and was projected    */
    double f;             /* ||K x - y||^2 at the returned x                   */
    double rel_change;    /* (f_prev - f)/f_prev of the last update            */
    double lambda_est;    /* ||K^T (y - K x)||_inf: the lambda paired with rho (Section 1) */
    double l1norm;        /* ||x||_1                                           */
    double t_fused_ms;    /* with opts.profile: summed duration of the fused launches */
    int32_t n_fused;      /* with opts.profile: number of fused launches timed  */
    int32_t proj_passes;  /* threshold-search passes summed over the iterations */
    int32_t x0_rejected;  /* 1 if opts.x0_fallback replaced x0 by 0            */
    int32_t reopened;     /* stops at the target that the double check overturned */
    int32_t reserved_;
} gp_result;

typedef struct gp_handle_s* gp_handle;

/* Fill `o` with the paper's GPSS parameters, max_iter = 100000,
 * f_target = -1 (off), f_targets = NULL, x0_fallback = 0, graph = 0, refresh_every = 0,
 * backtrack_cap = 60, chunk = 64, lookahead = 2, automatic kernel shapes. */
void gp_opts_default(gp_opts* o);

/* Create a handle bound to HIP device `device`; it owns the solver's scratch
 * workspace, which grows on demand and is freed by gp_destroy. */
int gp_create(gp_handle* out, int device);
int gp_destroy(gp_handle h);
/* Message for the last failing call on `h` (never NULL; static if h == NULL). */
const char* gp_last_error(gp_handle h);

/* Euclidean projection onto {||h||_1 <= rho}, the operator P_Omega used by
 * Algorithm 1 (Section 2, item 5, and Section 3):
 * h = sgn(v) max(|v| - mu, 0) with mu >= 0 the threshold for which
 * ||h||_1 = rho, or h = v when ||v||_1 <= rho.
 * vdtype: GP_F64 (double vectors) or GP_F32 (float vectors).  v, h_out:
 * device, p elements; h_out may alias v.  mu_out: host, may be NULL (then the
 * call does not synchronise).  p == 0 is a no-op.  rho < 0 or NaN: GP_E_ARG. */
int gp_l1_project(gp_handle h, gp_dtype vdtype, const void* v, int64_t p,
                  double rho, void* h_out, double* mu_out, void* stream);

/* Solve problem (2) with GPSS.  K: device n x p (ldk).  y: device n.
 * x0: device p, or NULL for x0 = 0 (projected onto the ball if outside).
 * tol: stop when (f_prev - f)/f_prev < tol (0 disables).  x_out: device p.
 * opts: host, NULL = defaults.  res: host, required.
 * Any p < 2^31 (double K: at most 65535 panels).  Up to 8192 (double K) or 16384 (float, bf16) columns one
 * pass over K per iteration forms both K d and K^T K d; wider problems cut
 * the columns into panels of 8192 / 16384 and read K twice per iteration
 * (K d, then K^T of it), with the same results to rounding.  Explicit
 * opts.fused_cfg shapes run one pass up to 16384 / 32768 / 65536 columns
 * (slower there than the panels); one narrower than p gives
 * GP_E_UNSUPPORTED.  opts.fused_cfg = GP_FUSED_PANELS asks for the panel
 * pass at any p.
 * Errors: n <= 0, p <= 0, ldk < p, rho < 0 or not finite, tol < 0 -> GP_E_ARG.
 * rho == 0 returns x = 0 with GP_STATIONARY. */
int gp_l1_solve(gp_handle h, gp_dtype kdtype, const void* K, int64_t n,
                int64_t p, int64_t ldk, const void* y, double rho,
                const void* x0, double tol, void* x_out, const gp_opts* opts,
                gp_result* res, void* stream);

/* Maximum workspace of gp_l1_solve_noalloc, in bytes (32 MiB). */
#define GP_NOALLOC_SCRATCH_BYTES (32u << 20)

/* gp_l1_solve without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, kernels and results as gp_l1_solve; the
 * solver's workspace is a fixed device array of GP_NOALLOC_SCRATCH_BYTES per
 * device (created with the library's code object and held until the process
 * ends; gp_create looks up its address), not the handle's growing workspace.
 * The call makes no hipMalloc/hipFree or other allocating call.
 * Limits: the workspace needed for (kdtype, n, p) must fit the scratch --
 * about (36 + 4G) p + 24 n bytes for float or bf16 K and (36 + 8G) p + 24 n
 * for double K, where G <= 256 is the number of row slabs the K pass uses
 * (256 once K holds 32 MB or more), plus 8 n per column panel of a wide
 * problem, so a 4096 x 16384 float K fits --
 * otherwise GP_E_UNSUPPORTED is returned before anything is launched;
 * opts.graph and opts.profile must be 0 (GP_E_ARG).
 * Every call on one device shares that device's scratch, which keeps the
 * last call's contents (the solver initialises what it reads): calls that
 * overlap in time on one device -- from two host threads, or on two streams
 * without ordering between them -- race and give undefined results. */
int gp_l1_solve_noalloc(gp_handle h, gp_dtype kdtype, const void* K, int64_t n,
                        int64_t p, int64_t ldk, const void* y, double rho,
                        const void* x0, double tol, void* x_out,
                        const gp_opts* opts, gp_result* res, void* stream);

/* B independent problems that share one K (B right-hand sides).
 * Y: device B x n (ldy >= n), rho: host array of B radii, X0: device B x p
 * (ldx >= p) or NULL, X_out: device B x p (ldx).  Each problem runs its own
 * steplength, threshold and line search; finished problems are frozen.
 * res: host array of B results.  Returns the most severe status.
 * K in GP_BF16 or GP_F32 runs on the bf16 matrix cores (an FP32 K as three
 * bf16 planes, products to FP32 accuracy) when p <= 16384; other cases run
 * the single-problem solver once per right-hand side. */
int gp_l1_solve_batched_shared(gp_handle h, gp_dtype kdtype, const void* K,
                               int64_t n, int64_t p, int64_t ldk,
                               const void* Y, int64_t ldy, int64_t B,
                               const double* rho, const void* X0, int64_t ldx,
                               double tol, void* X_out, const gp_opts* opts,
                               gp_result* res, void* stream);

/* One problem of an uneven batch: device pointers, its own sizes and radius. */
typedef struct {
    const void* K;     /* device, n x p row-major with leading dimension ldk */
    const void* y;     /* device, n                                          */
    const void* x0;    /* device, p, or NULL for 0                           */
    void* x_out;       /* device, p                                          */
    int64_t n, p, ldk;
    double rho;
} gp_instance;

/* B independent problems of different sizes, all of dtype kdtype.
 * inst: host array of B descriptors (pointers inside are device pointers).
 * res: host array of B results.  Returns the most severe status. */
int gp_l1_solve_batched_var(gp_handle h, gp_dtype kdtype,
                            const gp_instance* inst, int64_t B, double tol,
                            const gp_opts* opts, gp_result* res, void* stream);

/* ------------------------------------------------------------------------
 * The comparison methods of Section 2 on the same device passes.
 *
 *   GP_ISTA  (item 1):  x <- S_{tau lam}[x + tau K^T (y - K x)]
 *   GP_FISTA (item 2, equation (3)): the ISTA step taken from
 *            z_k = x_k + ((t_k - 1)/t_{k+1}) (x_k - x_{k-1}), t_0 = 1,
 *            t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
 *   GP_PSD   (item 5):  x <- P_Omega[x + beta r], r = K^T (y - K x),
 *            beta = ||r||^2 / ||K r||^2
 * with S_t[v] = sgn(v) max(|v| - t, 0).  ISTA and FISTA minimise the
 * penalised functional (1), F(x) = ||K x - y||^2 + 2 lam ||x||_1 (tau = 1
 * is the paper's form, valid for ||K|| < sqrt(2); in general tau < 2/||K||^2);
 * PSD minimises f over the ball ||x||_1 <= rho, problem (2).
 * ------------------------------------------------------------------------ */
typedef enum { GP_ISTA = 0, GP_FISTA = 1, GP_PSD = 2 } gp_fom_method;

/* Run `iters` iterations of `method` (fewer for PSD if r = 0 or K r = 0:
 * GP_STATIONARY; otherwise GP_MAX_ITER).  K, y, x0 (NULL = 0; PSD projects an
 * x0 outside the ball), x_out as in gp_l1_solve; param = lam for ISTA and
 * FISTA, rho for PSD (finite, >= 0); tau = step scale of ISTA and FISTA
 * (0 = 1, the paper's form), ignored by PSD.  opts: only the kernel-shape and
 * chunk fields are used (NULL = automatic).  res (host): iters, f = the
 * method's objective at the returned x (F for ISTA and FISTA, f for PSD)
 * computed in double from the returned x, l1norm; lambda_est is not set.
 * Any p (the K passes as in gp_l1_solve, column panels past 8192 / 16384
 * columns; PSD's projection streams past 32768 columns, where result.proj_passes
 * is not counted).  Errors as gp_l1_solve (GP_E_ARG for an unknown method). */
int gp_fom_solve(gp_handle h, int32_t method, gp_dtype kdtype, const void* K,
                 int64_t n, int64_t p, int64_t ldk, const void* y, double param,
                 double tau, const void* x0, int32_t iters, void* x_out,
                 const gp_opts* opts, gp_result* res, void* stream);

/* ------------------------------------------------------------------------
 * Learned warm start: an unrolled soft-thresholding network.
 *
 * ISTA (Section 2, item 1) iterates x <- S_lam[x + K^T (y - K x)], i.e. an
 * affine map followed by soft thresholding.  The network keeps that shape
 * with learned matrices and per-layer thresholds:
 *     c = We y,  x_1 = S_{theta_1}(c),  x_t = S_{theta_t}(c + S x_{t-1}),
 * t = 2..layers; We is p x n, S is p x p, theta has `layers` entries.  The
 * warm start of a solve is x0 = P_Omega(x_layers) (projection of Algorithm 1),
 * which lies in the ball as Algorithm 1 requires.
 *
 * Weights are kept on the device as FP32 master copies (with Adam moments)
 * and used as bf16 on the matrix cores; activations enter the products as
 * three bf16 planes, so weight x activation products carry FP32 accuracy.
 * Samples are stored one per row: Y is B x n, X is B x p (row-major, FP32).
 * ------------------------------------------------------------------------ */
typedef struct gp_lista_s* gp_lista;

/* Create a network for n x p problems with `layers` (1..32) layers on the
 * handle's device; weights start at zero.  The network owns its memory. */
int gp_lista_create(gp_handle h, gp_lista* out, int64_t n, int64_t p, int32_t layers);
int gp_lista_destroy(gp_lista net);

/* ISTA initialisation from K (device, FP32, n x p row-major, ldk):
 * We = K^T / L, S = I - K^T K / L, theta_t = lam / L for every layer, where
 * L >= ||K||_2^2 is given by the caller.  Resets the Adam state. */
int gp_lista_init_from_K(gp_lista net, const float* K, int64_t ldk, double L, double lam, void* stream);

/* Copy weights in or out (device FP32): We p x n, S p x p, theta[layers]. */
int gp_lista_set_weights(gp_lista net, const float* We, const float* S, const float* theta, void* stream);
int gp_lista_get_weights(gp_lista net, float* We, float* S, float* theta, void* stream);

/* Weights to and from a file: the 8-byte tag "GPLISTA1", int64 n, int64 p,
 * int32 layers, int32 0, then float32 little-endian W_e^T (n x p, row-major,
 * element (a, i) = W_e[i][a]), S^T (p x p, element (j, i) = S[i][j]) and
 * theta (layers).  load requires the network's n, p and layers, and resets
 * the Adam state.  Errors: GP_E_ARG for a bad path, tag or shape. */
int gp_lista_save(gp_lista net, const char* path);
int gp_lista_load(gp_lista net, const char* path);

/* Activations enter the forward products of gp_lista_forward as `planes`
 * bf16 planes (3, the default: FP32-accurate; 1: bf16 activations, a third of
 * the matrix-core work, enough for a warm start).  Training and
 * gp_lista_gradients always use 3.  planes outside 1..3: GP_E_ARG. */
int gp_lista_set_forward_planes(gp_lista net, int32_t planes);

/* Forward pass on B samples: Y (device, B x n, ldy) -> X_out (device,
 * B x p, ldx).  rho: host array of B radii, or NULL for the raw network
 * output; with rho each row is projected onto its ball. */
int gp_lista_forward(gp_lista net, const float* Y, int64_t ldy, int64_t B, const double* rho,
                     float* X_out, int64_t ldx, void* stream);

/* One training step on B samples (Y: B x n, Xstar: B x p, device): loss
 * (1/(2B)) sum ||x_layers - x*||^2, gradients by reverse accumulation
 * (derivative of S_theta taken as 0 at the kink), Adam with step lr
 * (beta1 = 0.9, beta2 = 0.999, eps = 1e-8) on the FP32 masters.
 * loss_out (host) receives the loss before the update; the call
 * synchronises the stream. */
int gp_lista_train_step(gp_lista net, const float* Y, int64_t ldy, const float* Xstar, int64_t ldx,
                        int64_t B, double lr, double* loss_out, void* stream);

/* Gradients of the loss at the current weights without an update (device
 * FP32 outputs, same shapes as the weights); loss_out as above. */
int gp_lista_gradients(gp_lista net, const float* Y, int64_t ldy, const float* Xstar, int64_t ldx, int64_t B,
                       float* dWe, float* dS, float* dtheta, double* loss_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GP_L1_H */
