// RBF-FD weights for the projected surface Laplacian, per stencil on the GPU.
//
// What is computed (Sec. 4, eqs. f_interp, grad_x_f_interp, surface_lap_P1):
// for stencil P_1 = {x_1..x_n} (centre first) and shape parameter eps, the
// bordered local matrix A~ = [[A, U], [U^T, 0]], A_ij = phi(|x_i - x_j|), the
// projected gradient matrices B^d (rows: [Pi_i grad phi(|x - x_j|)]_d at x_i,
// border columns: [Pi_i grad q_k(x_i)]_d), G^d = B^d A~^{-1}[:, :n] and the
// weights w = first row of L_P = sum_d G^d G^d.  The first row is formed
// without the n x n matrices: g_d = (A~^{-1} b_d)[:n] with b_d the first row
// of B^d, r = sum_d (B^d)^T g_d, w = (A~^{-1} r)[:n] (A~ is symmetric).
//
// Shape parameter (Sec. 5, eq. target_cond): kappa_2(A~) = max|l| / min|l|.
// Bisection on eps toward kappa_target, or a given/learned eps checked
// against a kappa band.
//
// How, on gfx950: the m x m matrix lives in registers.  NB = 1 (m <= 64): one
// wavefront per stencil, lane i holding column i.  NB = 2 (m <= 128): four
// wavefronts per stencil, wave (rb, cb) holding rows 64 rb .. 64 rb + 63 of
// columns 64 cb + lane.  A~ is reduced to tridiagonal form T = Q^T A~ Q by
// Householder reflections; the pivot column of each step is published to LDS
// during the previous step's rank-2 update (row k+1, by symmetry), so no
// register is indexed dynamically, and each reflector is kept in the
// registers of the row it annihilated.  kappa_2 comes from Sturm counts of T
// evaluated at 32 shifts per wave at once (multisection); the solves use
// A~^{-1} = Q T^{-1} Q^T with a pivoted tridiagonal factorisation and one step
// of iterative refinement (the residual re-evaluated from the nodes).  All
// FP64.  The polynomial border (degree 1 or 2) is orthonormalised by modified
// Gram-Schmidt with reorthogonalisation, dropping columns whose residual falls
// below rank_tol of their original norm (on the sphere one quadratic
// combination vanishes identically).
//
// This file is the host side of the plain launch (one workgroup per stencil);
// the kernels are in weights_kernels.hip, the batched launch in batched.cpp.
#include "batched.h"

using namespace rbw;

namespace {

int check_opts(rbffd_ctx ctx, int64_t N, const rbffd_weight_opts* opts, WOpts& o) {
    if (!opts) return set_error(ctx, RBFFD_E_ARG, "null opts");
    o.n = opts->n;
    o.kernel = opts->kernel;
    o.degree = opts->poly_degree;
    o.mode = opts->eps_mode;
    o.eps_fixed = opts->eps_fixed;
    o.kappa_target = opts->kappa_target;
    o.eps_tol = opts->eps_tol;
    o.br_lo = opts->bracket_lo;
    o.br_hi = opts->bracket_hi;
    o.band_lo = opts->band_lo;
    o.band_hi = opts->band_hi;
    o.rank_tol = opts->rank_tol;
    o.band_stop = opts->band_stop;
    o.max_expand = opts->max_expand;
    if (N < 0 || N > 0x7fffffffLL) return set_error(ctx, RBFFD_E_ARG, "N out of range");
    if (o.n < 2 || o.n > 128 || (N > 0 && o.n > N))
        return set_error(ctx, RBFFD_E_ARG, "stencil size n=%d invalid for N=%lld", o.n, (long long)N);
    if (o.kernel < 0 || o.kernel > 2) return set_error(ctx, RBFFD_E_ARG, "unknown kernel %d", o.kernel);
    if (o.degree < 0 || o.degree > 2) return set_error(ctx, RBFFD_E_ARG, "poly_degree must be 0, 1 or 2");
    if (o.mode < 0 || o.mode > 3) return set_error(ctx, RBFFD_E_ARG, "unknown eps_mode %d", o.mode);
    if (o.n + border_cols(o.degree) > 128)
        return set_error(ctx, RBFFD_E_UNSUPPORTED, "n + border = %d exceeds 128", o.n + border_cols(o.degree));
    if (o.mode == RBFFD_EPS_FIXED && !(o.eps_fixed > 0.0)) return set_error(ctx, RBFFD_E_ARG, "eps_fixed must be > 0");
    if ((o.mode == RBFFD_EPS_BISECT || o.mode == RBFFD_EPS_LEARNED) &&
        !(o.kappa_target > 1.0 && o.eps_tol > 0.0 && o.br_lo > 0.0 && o.br_hi > o.br_lo))
        return set_error(ctx, RBFFD_E_ARG, "invalid bisection parameters");
    if ((o.mode == RBFFD_EPS_LEARNED || o.band_stop) && !(o.band_lo > 1.0 && o.band_hi >= o.band_lo))
        return set_error(ctx, RBFFD_E_ARG, "invalid kappa band");
    if (!(o.rank_tol >= 0.0)) return set_error(ctx, RBFFD_E_ARG, "rank_tol must be >= 0");
    // kappa_2 of a stencil accepted inside the band is >= band_lo, so its
    // computed value is uncertain by ~band_lo u anyway (backward error of the
    // tridiagonal reduction); the eigenvalue multisection stops at that
    // level too (reported kappa within ~2 kappa u; the tests allow 20)
    o.band_rel = o.band_lo > 1.0 ? o.band_lo * 0x1p-53 : 0.0;
    if (o.max_expand < 0 || o.max_expand > 64) return set_error(ctx, RBFFD_E_ARG, "max_expand out of range");
    return RBFFD_OK;
}

template <int NB>
void launch_plain(hipStream_t st, const Job& J) {
    switch (J.o.kernel) {
        case RBFFD_KERNEL_MQ: launch_weights<RBFFD_KERNEL_MQ, NB>(st, J); break;
        case RBFFD_KERNEL_IMQ: launch_weights<RBFFD_KERNEL_IMQ, NB>(st, J); break;
        default: launch_weights<RBFFD_KERNEL_GA, NB>(st, J); break;
    }
}

int dispatch(rbffd_ctx ctx, const Job& J) {
    if (J.o.n + border_cols(J.o.degree) <= 64) launch_plain<1>(ctx->stream, J);
    else launch_plain<2>(ctx->stream, J);
    HIP_TRY(ctx, hipGetLastError());
    return RBFFD_OK;
}

}  // namespace

int weights_check_opts(rbffd_ctx ctx, int64_t N, const rbffd_weight_opts* opts, rbw::WOpts& o) {
    return check_opts(ctx, N, opts, o);
}

namespace {

template <int NB>
void launch_batched_nb(hipStream_t st, int kernel, const Job* jobs, const WorkItem* items, int nitems, int* cursor,
                       int grid) {
    switch (kernel) {
        case RBFFD_KERNEL_MQ: launch_weights_batched<RBFFD_KERNEL_MQ, NB>(st, jobs, items, nitems, cursor, grid); break;
        case RBFFD_KERNEL_IMQ: launch_weights_batched<RBFFD_KERNEL_IMQ, NB>(st, jobs, items, nitems, cursor, grid); break;
        default: launch_weights_batched<RBFFD_KERNEL_GA, NB>(st, jobs, items, nitems, cursor, grid); break;
    }
}

}  // namespace

int weights_launch_batched(rbffd_ctx ctx, int kernel, int nb, const Job* jobs, const WorkItem* items, int nitems,
                           int* cursor, int grid) {
    if (nb == 1) launch_batched_nb<1>(ctx->stream, kernel, jobs, items, nitems, cursor, grid);
    else launch_batched_nb<2>(ctx->stream, kernel, jobs, items, nitems, cursor, grid);
    HIP_TRY(ctx, hipGetLastError());
    return RBFFD_OK;
}

extern "C" int rbffd_build_weights(rbffd_ctx ctx, int64_t N, const double* xyz, const double* nrm,
                                   const rbffd_weight_opts* opts, const int32_t* idx_in, const double* eps_in,
                                   int32_t* idx_out, double* w, double* eps, double* kappa, int32_t* status,
                                   int32_t* nevals) {
    if (!ctx) return RBFFD_E_ARG;
    Job J;
    int rc = check_opts(ctx, N, opts, J.o);
    if (rc) return rc;
    if (N == 0) return RBFFD_OK;
    if (!xyz || !nrm || !w) return set_error(ctx, RBFFD_E_ARG, "null pointer");
    if ((J.o.mode == RBFFD_EPS_GIVEN || J.o.mode == RBFFD_EPS_LEARNED) && !eps_in)
        return set_error(ctx, RBFFD_E_ARG, "eps_in required for this eps_mode");
    const int32_t* idx = idx_in;
    if (!idx) {
        if (!idx_out) return set_error(ctx, RBFFD_E_ARG, "idx_out required when idx_in is NULL");
        rc = knn_internal(ctx, N, xyz, J.o.n, idx_out, nullptr);
        if (rc) return rc;
        idx = idx_out;
    } else if (idx_out && idx_out != idx_in) {
        HIP_TRY(ctx, hipMemcpyAsync(idx_out, idx_in, N * J.o.n * sizeof(int32_t), hipMemcpyDeviceToDevice, ctx->stream));
    }
    J.N = N;
    J.xyz = xyz;
    J.nrm = nrm;
    J.idx = idx;
    J.eps_in = eps_in;
    J.w = w;
    J.eps = eps;
    J.kappa = kappa;
    J.status = status;
    J.nevals = nevals;
    J.kappa_only = 0;
    return dispatch(ctx, J);
}

extern "C" int rbffd_kappa(rbffd_ctx ctx, int64_t N, const double* xyz, const rbffd_weight_opts* opts,
                           const int32_t* idx, const double* eps_in, double* kappa) {
    if (!ctx) return RBFFD_E_ARG;
    Job J;
    int rc = check_opts(ctx, N, opts, J.o);
    if (rc) return rc;
    if (N == 0) return RBFFD_OK;
    if (!xyz || !idx || !eps_in || !kappa) return set_error(ctx, RBFFD_E_ARG, "null pointer");
    J.o.mode = RBFFD_EPS_GIVEN;
    J.N = N;
    J.xyz = xyz;
    J.nrm = nullptr;
    J.idx = idx;
    J.eps_in = eps_in;
    J.w = nullptr;
    J.eps = nullptr;
    J.kappa = kappa;
    J.status = nullptr;
    J.nevals = nullptr;
    J.kappa_only = 1;
    return dispatch(ctx, J);
}
