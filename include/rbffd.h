/*
 * rbffd.h -- C ABI of the RBF-FD surface-diffusion library for MI355X (gfx950).
 *
 * The library computes RBF-FD weights for the projected (extrinsic) surface
 * Laplacian on scattered nodes with unit normals, and advances
 * du_s/dt = D_s L_X u_s + R_s(u) with the sparse operator L_X.  It follows the
 * paper "A Radial Basis Function (RBF)-Finite Difference (FD) Method for
 * Diffusion and Reaction-Diffusion Equations on Surfaces" (Shankar, Wright,
 * Kirby, Fogelson; arXiv:1404.0812): Sec. 4 (stencils, local interpolant,
 * projected gradients, L_P and first-row weights), Sec. 5 (per-stencil shape
 * parameter for a target condition number) and Sec. 4.2 (method of lines).
 *
 * Conventions for every call:
 *  - Array arguments are DEVICE pointers owned by the caller, unless a
 *    comment says "host".  The library never frees or keeps them.
 *  - Every call is enqueued on the stream given to rbffd_create and returns
 *    before the work completes; synchronise that stream before reading
 *    outputs.  Outputs that are written must not alias inputs.
 *  - Return value: 0 on success, a negative RBFFD_E* code on error.  On
 *    error nothing has been enqueued and rbffd_last_error() holds a message.
 *  - Node arrays are N x 3 row-major FP64 (x0 y0 z0 x1 y1 z1 ...).
 *  - Stencil arrays are N x n row-major: row i lists node i first, then its
 *    n-1 nearest neighbours by Euclidean distance in R^3, ascending by
 *    (squared distance, node index); w[i*n + k] is the weight of node
 *    idx[i*n + k] in the approximation of the surface Laplacian at node i.
 *  - One context per stream; a context is not thread-safe.
 */
#ifndef RBFFD_H
#define RBFFD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rbffd_ctx_s* rbffd_ctx;
typedef struct rbffd_op_s* rbffd_op;

/* error codes */
#define RBFFD_OK 0
#define RBFFD_E_ARG (-1)      /* invalid argument (sizes, enum values, null pointer) */
#define RBFFD_E_HIP (-2)      /* a HIP runtime call failed */
#define RBFFD_E_NOMEM (-3)    /* device allocation of library scratch failed */
#define RBFFD_E_UNSUPPORTED (-4) /* valid request outside what this library implements */
#define RBFFD_E_NONFINITE (-5) /* rbffd_step: the state became non-finite (NaN or Inf) */
#define RBFFD_E_NOCONV (-6)    /* rbffd_step_imex: a linear solve missed its tolerance */

/* radial kernels (Sec. 2) */
#define RBFFD_KERNEL_MQ 0  /* sqrt(1 + (eps r)^2) */
#define RBFFD_KERNEL_IMQ 1 /* 1 / sqrt(1 + (eps r)^2) -- the paper's choice */
#define RBFFD_KERNEL_GA 2  /* exp(-(eps r)^2) */

/* shape-parameter modes (Sec. 5) */
#define RBFFD_EPS_FIXED 0   /* one eps for all stencils: opts.eps_fixed */
#define RBFFD_EPS_GIVEN 1   /* per-stencil eps read from eps_in[N] */
#define RBFFD_EPS_BISECT 2  /* per-stencil bisection on eps to kappa_2 = kappa_target */
#define RBFFD_EPS_LEARNED 3 /* start from eps_in[N] (a prediction); keep it if
                               kappa_2 lies in [band_lo, band_hi], else bisect */

/* per-stencil status codes */
#define RBFFD_ST_OK 0
#define RBFFD_ST_FALLBACK 1   /* LEARNED: prediction outside the band, bisection used */
#define RBFFD_ST_NO_BRACKET 2 /* bisection bracket could not be formed */
#define RBFFD_ST_NONFINITE 3  /* non-finite entries in the local system */
#define RBFFD_ST_SINGULAR 4   /* zero pivot in the tridiagonal solve */
#define RBFFD_ST_DUPLICATE 5  /* two stencil nodes coincide */
#define RBFFD_ST_BAD_INDEX 6  /* a stencil index outside [0, N): weights NaN, stencil skipped */
#define RBFFD_ST_BAD_NORMAL 7 /* a stencil node's normal is zero or not finite (the projection
                                 Pi = I - nu nu^T of Sec. 3 is undefined): eps, kappa and
                                 weights NaN, stencil skipped */

/* reaction terms for rbffd_step */
#define RBFFD_REACT_NONE 0
#define RBFFD_REACT_SCHNAKENBERG 1 /* params: a, b, gamma */
#define RBFFD_REACT_TURING 2       /* params: alpha, beta, gamma, tau1, tau2 (eqs. turing1-2) */

/* state precision for rbffd_step / rbffd_apply */
#define RBFFD_F64 0
#define RBFFD_F32 1

typedef struct {
    int32_t n;            /* stencil size including the centre, 2 <= n <= 128 */
    int32_t kernel;       /* RBFFD_KERNEL_* */
    int32_t poly_degree;  /* 0: the paper's constant border (ones); 1 or 2: monomials
                             in (x - x_1)/rho reduced to an orthonormal basis of
                             their numerical range (columns dropped below rank_tol) */
    int32_t eps_mode;     /* RBFFD_EPS_* */
    double eps_fixed;     /* FIXED mode */
    double kappa_target;  /* BISECT/LEARNED: target 2-norm condition number */
    double eps_tol;       /* bisection stops when hi - lo <= eps_tol (absolute, in eps) */
    double bracket_lo;    /* initial bracket [bracket_lo, bracket_hi] / rho */
    double bracket_hi;
    double band_lo;       /* LEARNED acceptance band for kappa_2; also the band for */
    double band_hi;       /*   band_stop */
    double rank_tol;      /* relative drop tolerance for border columns */
    int32_t band_stop;    /* BISECT and the LEARNED fallback: 1 = stop as soon as kappa_2 is inside the band */
    int32_t max_expand;   /* bracket expansions allowed on each side */
} rbffd_weight_opts;

/* Fill opts with the defaults: n = 31, MQ, degree 2, FIXED eps 2, kappa_target
 * 1e12, eps_tol 1e-4 (Sec. 5), bracket [0.05, 20]/rho, band [1e11, 1e13],
 * rank_tol 1e-10, band_stop 0, max_expand 8.  opts is a HOST pointer. */
void rbffd_default_opts(rbffd_weight_opts* opts);

/* Create a context bound to `stream` (a hipStream_t; NULL = the null stream)
 * on the current device.  *out is a HOST pointer that receives the handle. */
int rbffd_create(rbffd_ctx* out, void* stream);
int rbffd_destroy(rbffd_ctx ctx);
/* Message of the last error on this context (static storage of the context). */
const char* rbffd_last_error(rbffd_ctx ctx);

/*
 * Stencils (Sec. 4; Sec. 4.1 uses a k-d tree, this uses a uniform grid hash).
 * xyz: N x 3 FP64.  idx: N x n int32 output in the layout described above.
 * perm (nullable): N int32 output, the library's spatial order, perm[p] =
 * caller index of the node at position p (cell-sorted, Morton order of cells).
 * Errors: n < 1, n > N, n > 128, N > 2^31 - 1.
 */
int rbffd_knn(rbffd_ctx ctx, int64_t N, const double* xyz, int32_t n, int32_t* idx, int32_t* perm);

/*
 * Weights (Secs. 4 and 5).  xyz, nrm: N x 3 FP64 (normals need not be unit
 * length or consistently oriented; only nu nu^T enters).  idx_in: N x n
 * stencils; if NULL the call computes them first (rbffd_knn) and writes them
 * to idx_out (which must then be non-NULL).  eps_in: N FP64 shape parameters
 * for GIVEN/LEARNED modes (NULL otherwise).
 * Outputs: w (N x n FP64), eps (N, nullable), kappa (N, nullable: kappa_2 of
 * the bordered local matrix at the returned eps; for a LEARNED proposal kept
 * inside the band its eigenvalue search stops at band_lo u relative, u =
 * 2^-53, the level of the ~kappa u the reduction itself allows), status (N int32, nullable),
 * nevals (N int32, nullable: number of kappa_2 evaluations of the stencil).
 * Errors: as rbffd_knn; kernel/degree/mode out of range; n + border > 128.
 */
int rbffd_build_weights(rbffd_ctx ctx, int64_t N, const double* xyz, const double* nrm,
                        const rbffd_weight_opts* opts, const int32_t* idx_in, const double* eps_in,
                        int32_t* idx_out, double* w, double* eps, double* kappa, int32_t* status,
                        int32_t* nevals);

/*
 * Weights in extended precision (Sec. 6.2 computes weights for targets up to
 * kappa_T = 1e20 in quadruple precision): the same quantities as
 * rbffd_build_weights for the paper's own local system -- the constant border
 * (poly_degree 0) with the MQ or IMQ kernel -- with every quantity derived
 * from the FP64 inputs held as a double-double (about 32 digits): kernel
 * values, unit normals, the tridiagonal form and Sturm counts behind kappa_2
 * (so the bisection of Sec. 5 works for kappa_T well beyond 1e16), and a
 * pivoted LU for the solves.  eps, kappa and w are rounded to FP64.  Same
 * arguments as rbffd_build_weights; n + 1 <= 48; eps modes FIXED, GIVEN and
 * BISECT.  One wavefront per stencil, much slower than the FP64 path.
 * Errors: as rbffd_build_weights; RBFFD_E_UNSUPPORTED for another kernel,
 * degree, mode or n + 1 > 48.
 */
int rbffd_build_weights_dd(rbffd_ctx ctx, int64_t N, const double* xyz, const double* nrm,
                           const rbffd_weight_opts* opts, const int32_t* idx_in, const double* eps_in,
                           int32_t* idx_out, double* w, double* eps, double* kappa, int32_t* status,
                           int32_t* nevals);

/*
 * kappa_2 of every stencil's bordered local matrix at the given eps (Sec. 5,
 * eq. target_cond): max|lambda| / min|lambda|.  Inputs as rbffd_build_weights;
 * eps_in is required.  kappa: N FP64 output.
 */
int rbffd_kappa(rbffd_ctx ctx, int64_t N, const double* xyz, const rbffd_weight_opts* opts,
                const int32_t* idx, const double* eps_in, double* kappa);

/* ------------------------------------------------------------------------
 * Batched weights (Secs. 4 and 5 applied to many node sets at once).  The
 * stencils of nsurf surfaces, each with its own N and n, are computed by
 * persistent launches -- one for the surfaces with n + border <= 64 (one
 * wavefront per stencil), one for 64 < n + border <= 128 (four wavefronts per
 * stencil) -- whose workgroups take work items (runs of consecutive stencils
 * of one surface) from an atomic counter until none are left.  Every output
 * is bit-identical to rbffd_build_weights on that surface with the same opts
 * and the surface's n.
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t N;              /* nodes of this surface (0 allowed: skipped) */
    int32_t n;              /* stencil size on this surface (opts->n is ignored) */
    int32_t reserved;
    const double* xyz;      /* N x 3 */
    const double* nrm;      /* N x 3 */
    const int32_t* idx;     /* N x n stencils, or NULL: computed into idx_out first */
    const double* eps_in;   /* N, GIVEN/LEARNED modes */
    int32_t* idx_out;       /* N x n, required when idx is NULL (nullable otherwise) */
    double* w;              /* N x n output */
    double* eps;            /* N outputs, nullable as in rbffd_build_weights */
    double* kappa;
    int32_t* status;
    int32_t* nevals;
} rbffd_surface;

#define RBFFD_BUCKETS 2 /* tuning[0]: n + border <= 64; tuning[1]: 64 < n + border <= 128 */

/* Schedule of one bucket's persistent launch. */
typedef struct {
    int32_t stencils_per_item; /* stencils taken per counter increment, 1..4096 */
    int32_t groups_per_cu;     /* persistent workgroups (four wavefronts) per compute unit, 1 or 2 */
    int32_t order;             /* 0: surfaces by decreasing n, ties as given; 1: as given */
    int32_t reserved;
    double us_per_stencil;     /* set by rbffd_autotune_batched: measured time per sampled stencil */
} rbffd_batch_tuning;

/* surf: HOST array of nsurf descriptors (device pointers inside).  tuning:
 * HOST array of RBFFD_BUCKETS schedules, or NULL for the built-in default
 * (16 stencils per item in bucket 0, 2 in bucket 1, 2 groups per CU, order 0).
 * The call first drains the context's stream (the host waits for work
 * enqueued earlier) and then uploads the work list; the weights themselves
 * are enqueued asynchronously as usual.
 * Errors: as rbffd_build_weights for any surface (the message names it);
 * nsurf < 0; a schedule out of range. */
int rbffd_build_weights_batched(rbffd_ctx ctx, int32_t nsurf, const rbffd_surface* surf,
                                const rbffd_weight_opts* opts, const rbffd_batch_tuning* tuning);

/* Autotuner for rbffd_build_weights_batched.  For each bucket that holds
 * stencils, times every candidate schedule (stencils per item, groups per
 * CU, order) on a sample of the batch (the first stencils of every surface
 * in the bucket, about 32768 stencils in bucket 0 and 8192 in bucket 1) and
 * writes the fastest to tuning[bucket] (HOST, RBFFD_BUCKETS entries; buckets
 * without stencils get the default).  Results are cached per (GPU
 * architecture, kernel, poly_degree, eps_mode, bucket) in memory and, when
 * cache_path (HOST string, nullable) is given, in that JSON file, which is
 * read first and rewritten with the new entries.  retune = 1 ignores cached
 * entries.  The timing runs compute (and overwrite) the outputs of the
 * sampled stencils; stencils are computed into idx_out first where idx is
 * NULL.  The call synchronises the context's stream. */
int rbffd_autotune_batched(rbffd_ctx ctx, int32_t nsurf, const rbffd_surface* surf,
                           const rbffd_weight_opts* opts, const char* cache_path, int32_t retune,
                           rbffd_batch_tuning* tuning);

/*
 * Sparse operator L_X (Sec. 4: row k = weights of stencil k).  Built from
 * caller-order idx/w (N x n); stored internally as sliced ELL (slices of 64
 * rows, slot-major within a slice) in the spatial order `perm` (nullable:
 * identity), in FP64 and, for FP32 stepping, as FP32 off-diagonal weights
 * for the difference form sum_{j != i} w_ij (u_j - u_i).  *out is a HOST
 * pointer.  The operator owns device memory freed by rbffd_op_destroy.
 * Requirements on the rows: slot 0 of row i is node i itself (idx[i*n] ==
 * i, the layout rbffd_knn and rbffd_build_weights produce), and for FP32
 * stepping each row's weights sum to zero (L_X reproduces constants, as the
 * RBF-FD weights of Sec. 4 do): the FP32 form drops slot 0 and uses the
 * differences u_j - u_i, which equals L u only under that condition.
 * Errors: N < 1, n < 2, n > 128, n > N, null idx or w; an idx entry outside
 * [0, N), a row whose slot 0 is not the row itself, or a perm that is not a
 * permutation of 0..N-1 (checked on the device; the call then synchronises
 * and returns RBFFD_E_ARG).
 */
int rbffd_op_create(rbffd_ctx ctx, int64_t N, int32_t n, const int32_t* idx, const double* w,
                    const int32_t* perm, rbffd_op* out);

/* One surface of a batched operator. */
typedef struct {
    int64_t N;            /* rows (nodes) of the surface, >= 1 */
    int32_t n;            /* stencil size, 2..128, <= N */
    int32_t reserved;
    const int32_t* idx;   /* N x n, local node indices 0..N-1 */
    const double* w;      /* N x n weights */
    const int32_t* perm;  /* N, spatial order of the surface (nullable: identity) */
} rbffd_op_surface;

/* Block-diagonal operator of nsurf surfaces with their own N and n: one
 * rbffd_step then advances every surface with one kernel per RK4 stage (and
 * one captured graph per batch of steps), with one dt for all (the caller
 * passes the smallest stable dt of the surfaces).  State arrays hold the
 * surfaces one after another: species s, node i of surface t at
 * s * sum_N + (N_0 + ... + N_{t-1}) + i.  surf is a HOST array.
 * Errors: nsurf < 1 or any surface invalid as in rbffd_op_create. */
int rbffd_op_create_batched(rbffd_ctx ctx, int32_t nsurf, const rbffd_op_surface* surf, rbffd_op* out);
int rbffd_op_destroy(rbffd_op op);

/* Layout statistics of an operator (HOST outputs, each nullable): slices of
 * 64 rows; slices whose FP32 stage reads neighbour values from a halo staged
 * in LDS (at most 640 distinct neighbour rows; the others gather directly),
 * the rows in those slices, and their total halo entries.  Synchronises the
 * context's stream. */
int rbffd_op_stats(rbffd_op op, int64_t* nslices, int64_t* halo_slices, int64_t* halo_rows,
                   int64_t* halo_entries);

/*
 * One operator application Lu = L_X u (caller order, FP64 in and out),
 * computed in FP64 (plain form sum_j w_ij u_j) or FP32 (difference form).
 */
int rbffd_apply(rbffd_ctx ctx, rbffd_op op, int32_t prec, const double* u, double* Lu);

/*
 * rbffd_apply without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels and results (bit for bit)
 * as rbffd_apply; the two internal-order vectors (2 x padded rows x 8 bytes
 * in FP64, x 4 bytes in FP32) live in one fixed device array of
 * RBFFD_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends, instead of
 * the operator's workspace.  Every call on one GPU uses that GPU's array:
 * calls that overlap on one GPU (two streams, two threads) race and must be
 * ordered by the caller.  Nothing in the array needs to start at zero.
 * Errors: as rbffd_apply; RBFFD_E_UNSUPPORTED when the operator needs more
 * than the array holds (FP64: more than 4,194,304 padded rows).
 */
#define RBFFD_NOALLOC_SCRATCH_BYTES (64 * 1024 * 1024)
int rbffd_apply_noalloc(rbffd_ctx ctx, rbffd_op op, int32_t prec, const double* u, double* Lu);

/*
 * Method of lines (Sec. 4.2, eq. kernel_mol) with classical RK4:
 * du_s/dt = D[s] L_X u_s + R_s(u).  state: nspecies x N FP64, caller order,
 * read and overwritten with the state after nsteps steps.  D: nspecies
 * diffusivities (HOST).  params: reaction parameters (HOST, see
 * RBFFD_REACT_*).  prec selects FP64 or FP32 state arithmetic (FP32 uses the
 * difference form).  Steps run as a captured HIP graph of `graph_steps`
 * steps (0 = library default), replayed as needed.  The last stage of every
 * step raises a device flag when a state value is not finite; the flag is
 * copied to the host after each graph replay, further replays are skipped
 * once a copied flag shows it, and the call ends by synchronising the
 * context's stream (unlike the other calls, it returns after the work is
 * done) and returns RBFFD_E_NONFINITE if the flag was raised (state then
 * holds the last, non-finite values).
 * Errors: nspecies not 1 or 2, a reaction needing 2 species given 1, dt <= 0.
 */
int rbffd_step(rbffd_ctx ctx, rbffd_op op, int32_t nspecies, double* state, int32_t prec,
               const double* D, int32_t reaction, const double* params, double dt, int64_t nsteps,
               int32_t graph_steps);

/*
 * rbffd_step with a forcing term f (eq. diffusion_scalar of Sec. 4.2:
 * du/dt = delta L_X u + f) of the separable form of the manufactured
 * solutions of Sec. 6 (eqs. sph_forced, torus_forced):
 *   f_s(t, x_i) = exp(lambda t) forcing[s * N + i],
 * forcing: nspecies x N FP64, caller order (read once per call).  The state
 * is at time t0 on entry; RK4 evaluates f at the stage times t_n, t_n + dt/2,
 * t_n + dt/2, t_n + dt.  Otherwise as rbffd_step.
 * Errors: as rbffd_step; null forcing; t0 or lambda not finite.
 */
int rbffd_step_forced(rbffd_ctx ctx, rbffd_op op, int32_t nspecies, double* state, int32_t prec,
                      const double* D, int32_t reaction, const double* params, double dt, int64_t nsteps,
                      int32_t graph_steps, double t0, const double* forcing, double lambda);

/*
 * Semi-implicit BDF time stepping (SBDF-k, the paper's BDF4 of Sec. 6 for
 * diffusion and SBDF2 of Sec. 7 for reaction-diffusion), FP64:
 *   sum_{j=0}^{k} a_j u^{n+1-j} = dt (D L_X u^{n+1} + f(t_{n+1}) + sum_{j=1}^{k} b_j R(u^{n+1-j}))
 * with the k-step backward difference row a and the extrapolation row b of
 * order k; the diffusion and the forcing f_s(t, x_i) = exp(lambda t)
 * forcing[s * N + i] (nullable) are implicit, the reaction explicit.  Each
 * step solves (I - gamma L_X) u_s = rhs_s, gamma = dt D_s / a_0, per species
 * with unpreconditioned BiCGSTAB (initial guess u^n, restarted from the
 * true residual after a breakdown) to the relative residual tol (the
 * paper: 1e-12), at most maxit iterations in all.  No diagonal scaling: on
 * irregular node sets L_X can have positive diagonal entries, and the
 * diagonal of I - gamma L_X then crosses zero as dt grows.
 * state: nspecies x N FP64 at time t0, caller order, overwritten with the
 * state after nsteps steps.  history (nullable): the states at t0 - dt,
 * t0 - 2 dt, ..., (order - 1) x nspecies x N (the paper starts BDF4 from the
 * exact solution); without it the first steps use orders 1, 2, ... (which
 * limits the global order to 2).  iters_out, relres_out (HOST, nullable):
 * total iterations and the largest final relative residual.  Synchronises
 * the context's stream.
 * Errors: as rbffd_step; order outside 1..4; tol <= 0; maxit < 1;
 * RBFFD_E_NOCONV when a solve misses tol (state holds the steps done);
 * RBFFD_E_NONFINITE when a residual is not finite.
 */
int rbffd_step_imex(rbffd_ctx ctx, rbffd_op op, int32_t nspecies, double* state, const double* D, int32_t reaction,
                    const double* params, double dt, int64_t nsteps, int32_t order, const double* history, double t0,
                    const double* forcing, double lambda, double tol, int32_t maxit, int64_t* iters_out,
                    double* relres_out);

/* ------------------------------------------------------------------------
 * Learned shape parameter.  A 128 -> 128 -> 128 -> 1 ReLU network maps a
 * stencil's tangent-plane offsets to y = log(eps * rho) (rho = stencil
 * radius), trained on eps found by the bisection of Sec. 5 (eq.
 * target_cond).  Its proposal is checked by kappa_2 in
 * rbffd_build_weights (RBFFD_EPS_LEARNED), with bisection as fallback.
 * Parameters: one FP32 array of RBFFD_MLP_PARAMS values: W1[128][128]
 * (out, in), b1[128], W2[128][128], b2[128], w3[128], b3.  Matrix products
 * run on BF16 MFMA with FP32 accumulation; activations are rounded to BF16.
 * ------------------------------------------------------------------------ */
#define RBFFD_MLP_IN 128
#define RBFFD_MLP_HIDDEN 128
#define RBFFD_MLP_PARAMS 33153

typedef struct {
    double lr;        /* Adam step size */
    double beta1;     /* Adam moment decays */
    double beta2;
    double adam_eps;
    int32_t batch;    /* samples per step, a positive multiple of 64 */
    int32_t steps;    /* optimiser steps in this call */
    uint64_t seed;    /* non-zero; batch rows are drawn by a counter-based hash of (seed, step) */
    int64_t step0;    /* index of the first step (Adam bias correction and sampling) */
} rbffd_train_opts;

/* Features of N stencils: feats is N x 128 BF16 (stored as uint16), row s =
 * (s_2, t_2, s_3, t_3, ..., zero padding) with (s_j, t_j) the offsets
 * x_j - x_1 in the tangent frame (tau_1 along the nearest neighbour's
 * projected offset, tau_2 = nu x tau_1) divided by rho.  rho (nullable): N
 * FP64 stencil radii.  Requires 2 <= n <= 64 (RBFFD_E_ARG otherwise). */
int rbffd_mlp_features(rbffd_ctx ctx, int64_t N, const double* xyz, const double* nrm, const int32_t* idx,
                       int32_t n, uint16_t* feats, double* rho);
/* y[B] (FP32) = network(feats[B x 128]). */
int rbffd_mlp_forward(rbffd_ctx ctx, const float* params, int64_t B, const uint16_t* feats, float* y);
/* Gradient of the mean squared error over all B samples: grad[RBFFD_MLP_PARAMS]
 * (FP32, overwritten) and loss[1] (FP32, overwritten). */
int rbffd_mlp_grad(rbffd_ctx ctx, const float* params, int64_t B, const uint16_t* feats, const float* target,
                   float* grad, float* loss);
/* Adam training on (feats, target) pairs (count samples); params, adam_m and
 * adam_v (RBFFD_MLP_PARAMS FP32 each) are updated in place.  loss_per_step
 * (nullable): opts->steps FP32 batch losses. */
int rbffd_mlp_train(rbffd_ctx ctx, float* params, float* adam_m, float* adam_v, int64_t count,
                    const uint16_t* feats, const float* target, const rbffd_train_opts* opts,
                    float* loss_per_step);
/* eps[N] (FP64) = exp(network(features)) / rho for the stencils idx (the
 * features of rbffd_mlp_features: 2 <= n <= 64). */
int rbffd_predict_eps(rbffd_ctx ctx, const float* params, int64_t N, const double* xyz, const double* nrm,
                      const int32_t* idx, int32_t n, double* eps);

#ifdef __cplusplus
}
#endif
#endif /* RBFFD_H */
