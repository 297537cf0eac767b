// RBF-FD weights for the projected surface Laplacian, one wavefront per stencil.
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
// How, on gfx950: the m x m matrix (m = n + border size <= 64) lives in
// registers, lane i holding column i.  A~ is reduced to tridiagonal form
// T = Q^T A~ Q by Householder reflections (the pivot column of each step is
// published to LDS during the previous step's rank-2 update, so no register
// is ever indexed dynamically); the reflectors stay in the registers of the
// annihilated rows.  kappa_2 comes from Sturm counts of T evaluated by the 64
// lanes at 64 shifts at once (multisection), and the solves use
// A~^{-1} = Q T^{-1} Q^T with a pivoted tridiagonal factorisation.  All of it
// is FP64.  The polynomial border (degree 1 or 2) is orthonormalised by
// modified Gram-Schmidt with reorthogonalisation, dropping columns whose
// residual falls below rank_tol of their original norm: on the sphere one
// quadratic combination vanishes identically and is dropped.
#include "common.h"

#include <cmath>

namespace {

constexpr int MMAX = 64;  // m = n + border <= 64 on this path
constexpr int RMAX = 10;  // border columns (degree-2 monomials in R^3)

struct WOpts {
    int n, kernel, degree, mode;
    double eps_fixed, kappa_target, eps_tol, br_lo, br_hi, band_lo, band_hi, rank_tol;
    int band_stop, max_expand;
};

// ------------------------------------------------------------ reductions ----
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ void wave_sum3(double& a, double& b, double& c) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
        c += __shfl_xor(c, o, 64);
    }
}

// ---------------------------------------------------------- radial kernels ----
template <int K>
__device__ __forceinline__ double rbf_phi(double e2, double r2) {
    double e = e2 * r2;
    if (K == RBFFD_KERNEL_MQ) return sqrt(1.0 + e);
    if (K == RBFFD_KERNEL_IMQ) return 1.0 / sqrt(1.0 + e);
    return exp(-e);
}
// phi'(r)/r
template <int K>
__device__ __forceinline__ double rbf_psi(double e2, double r2) {
    double e = e2 * r2;
    if (K == RBFFD_KERNEL_MQ) return e2 / sqrt(1.0 + e);
    if (K == RBFFD_KERNEL_IMQ) return -e2 / (sqrt(1.0 + e) * (1.0 + e));
    return -2.0 * e2 * exp(-e);
}

// LDS of one stencil (one wavefront per workgroup)
struct Shared {
    double x[MMAX], y[MMAX], z[MMAX];  // stencil node coordinates
    double U[MMAX * RMAX];             // border basis values U[j*RMAX + k]
    double T[RMAX * RMAX];             // monomial coefficients of the border basis T[l*RMAX + k]
    double col[MMAX], vv[MMAX], ww[MMAX];
    double d[MMAX], e[MMAX], e2[MMAX], tau[MMAX];
    double fd[MMAX], fdu[MMAX], fdl[MMAX], ffact[MMAX];  // pivoted tridiagonal factors
    int fswap[MMAX];
    double rhs[3][MMAX];
    double zb[3][MMAX];
    double hx[MMAX], hy[MMAX], hz[MMAX];
    double nrm0[3];
    double rho;
    int m, r, n;
};

// ----------------------------------------------------------- local matrix ----
template <int K>
__device__ __forceinline__ void build_matrix(double (&a)[MMAX], const Shared& S, int lane, double e2) {
    const int n = S.n, m = S.m;
    const double xi = S.x[lane < n ? lane : 0], yi = S.y[lane < n ? lane : 0], zi = S.z[lane < n ? lane : 0];
#pragma unroll
    for (int jj = 0; jj < MMAX; ++jj) {
        double v = 0.0;
        if (jj < n) {
            if (lane < n) {
                double dx = xi - S.x[jj], dy = yi - S.y[jj], dz = zi - S.z[jj];
                double r2 = (dx * dx + dy * dy) + dz * dz;
                v = rbf_phi<K>(e2, r2);
            } else if (lane < m) {
                v = S.U[jj * RMAX + (lane - n)];
            }
        } else if (jj < m) {
            if (lane < n) v = S.U[lane * RMAX + (jj - n)];
        }
        a[jj] = v;
    }
}

// a - (vj*wi + wj*vi) with no contraction: the two products are rounded
// separately and added commutatively, so (i, j) and (j, i) get the same value.
__device__ __forceinline__ double sym_rank2(double a, double vj, double wi, double wj, double vi) {
#pragma clang fp contract(off)
    const double p = vj * wi;
    const double q = wj * vi;
    return a - (p + q);
}

// Householder tridiagonalisation of the m x m leading block of the register
// matrix (lane = column).  On return: S.d[0..m-1], S.e[0..m-2] (and e^2),
// S.tau[0..m-3], and row k of `a` holds the reflector v_k (v_k[k+1] = 1).
__device__ __forceinline__ void tridiagonalise(double (&a)[MMAX], Shared& S, int lane) {
    const int m = S.m;
    S.col[lane] = a[0];
    __syncthreads();
    for (int k = 0; k < m - 2; ++k) {
        const double xi = S.col[lane];
        const double alpha = S.col[k + 1];
        const double dk = S.col[k];
        const bool tail = lane > k + 1 && lane < m;
        const double xnorm2 = wave_sum(tail ? xi * xi : 0.0);
        double tau = 0.0, beta = alpha, scal = 0.0;
        if (xnorm2 > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
            tau = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        const double vi = (lane == k + 1) ? 1.0 : (tail ? xi * scal : 0.0);
        if (lane == 0) {
            S.d[k] = dk;
            S.e[k] = beta;
            S.e2[k] = beta * beta;
            S.tau[k] = tau;
        }
        S.vv[lane] = vi;
        __syncthreads();
        // p = A v (rows > k)
        double p0 = 0.0, p1 = 0.0;
#pragma unroll
        for (int j0 = 0; j0 < MMAX; j0 += 8) {
            if (j0 + 8 > k + 1 && j0 < m) {
#pragma unroll
                for (int t = 0; t < 8; t += 2) {
                    p0 = fma(a[j0 + t], S.vv[j0 + t], p0);
                    p1 = fma(a[j0 + t + 1], S.vv[j0 + t + 1], p1);
                }
            }
        }
        double wi = (lane > k && lane < m) ? tau * (p0 + p1) : 0.0;
        const double s = wave_sum(wi * vi);
        wi = fma(-0.5 * tau * s, vi, wi);
        S.ww[lane] = wi;
        __syncthreads();
        // A -= v w^T + w v^T; store v in row k; publish row k+1 as the next pivot column
#pragma unroll
        for (int j0 = 0; j0 < MMAX; j0 += 8) {
            if (j0 + 8 > k + 1 && j0 < m) {
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    // v_j w_i + w_j v_i from two separately rounded products and a
                    // commutative add: entries (i, j) and (j, i) get bit-identical
                    // updates, so the register matrix stays exactly symmetric
                    a[j0 + t] = sym_rank2(a[j0 + t], S.vv[j0 + t], wi, S.ww[j0 + t], vi);
                }
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                if (j0 + t == k) a[j0 + t] = vi;
                if (j0 + t == k + 1) S.col[lane] = a[j0 + t];
            }
        }
        __syncthreads();
    }
    // trailing 2 x 2 block
#pragma unroll
    for (int jj = 0; jj < MMAX; ++jj)
        if (jj == m - 1) S.ww[lane] = a[jj];
    __syncthreads();
    if (lane == 0) {
        if (m >= 2) {
            S.d[m - 2] = S.col[m - 2];
            S.e[m - 2] = S.col[m - 1];
            S.e2[m - 2] = S.col[m - 1] * S.col[m - 1];
        }
        S.d[m - 1] = S.ww[m - 1];
    }
    __syncthreads();
}

// ------------------------------------------------------------ Sturm counts ----
// number of eigenvalues of T below sigma
__device__ __forceinline__ int sturm(const Shared& S, int m, double sigma, double pivmin) {
    double q = S.d[0] - sigma;
    if (fabs(q) < pivmin) q = -pivmin;
    int c = q < 0.0 ? 1 : 0;
    for (int i = 1; i < m; ++i) {
        q = (S.d[i] - sigma) - S.e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0 ? 1 : 0;
    }
    return c;
}

struct Spectrum {
    double amax;  // max |lambda|
    bool finite;
    double pivmin;
    double gl, gu;
};

__device__ __forceinline__ bool finite_d(double v) { return isfinite(v); }

// Largest |lambda| of T to ~33^-rounds of the Gershgorin width.
__device__ Spectrum spectrum_max(const Shared& S, int lane, int rounds) {
    const int m = S.m;
    Spectrum sp;
    double gl = INFINITY, gu = -INFINITY, emax2 = 0.0;
    bool fin = true;
    for (int i = 0; i < m; ++i) {
        double off = (i > 0 ? fabs(S.e[i - 1]) : 0.0) + (i < m - 1 ? fabs(S.e[i]) : 0.0);
        gl = fmin(gl, S.d[i] - off);
        gu = fmax(gu, S.d[i] + off);
        if (i < m - 1) emax2 = fmax(emax2, S.e2[i]);
        fin = fin && finite_d(S.d[i]) && (i == m - 1 || finite_d(S.e[i]));
    }
    sp.finite = fin;
    sp.pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
    double w = gu - gl;
    gl -= 2.0 * w * 2.2e-16 + 2.0 * sp.pivmin;
    gu += 2.0 * w * 2.2e-16 + 2.0 * sp.pivmin;
    sp.gl = gl;
    sp.gu = gu;
    if (!fin) {
        sp.amax = NAN;
        return sp;
    }
    // lanes 0..31: smallest eigenvalue (index 1); lanes 32..63: largest (index m)
    double lo1 = gl, hi1 = gu, lo2 = gl, hi2 = gu;
    const int g = lane >> 5, t = lane & 31;
    for (int rd = 0; rd < rounds; ++rd) {
        const double lo = g ? lo2 : lo1, hi = g ? hi2 : hi1;
        const double sig = lo + (hi - lo) * (double)(t + 1) / 33.0;
        const int kidx = g ? m : 1;
        const bool below = sturm(S, m, sig, sp.pivmin) < kidx;  // eigenvalue kidx lies above sig
        const uint64_t bal = __ballot(below);
        const int nb1 = __popcll(bal & 0xffffffffull);
        const int nb2 = __popcll(bal >> 32);
        const double n_lo1 = nb1 > 0 ? lo1 + (hi1 - lo1) * (double)nb1 / 33.0 : lo1;
        const double n_hi1 = nb1 < 32 ? lo1 + (hi1 - lo1) * (double)(nb1 + 1) / 33.0 : hi1;
        const double n_lo2 = nb2 > 0 ? lo2 + (hi2 - lo2) * (double)nb2 / 33.0 : lo2;
        const double n_hi2 = nb2 < 32 ? lo2 + (hi2 - lo2) * (double)(nb2 + 1) / 33.0 : hi2;
        lo1 = n_lo1; hi1 = n_hi1; lo2 = n_lo2; hi2 = n_hi2;
    }
    const double lmin = 0.5 * (lo1 + hi1), lmax = 0.5 * (lo2 + hi2);
    sp.amax = fmax(fabs(lmin), fabs(lmax));
    return sp;
}

// #eigenvalues with |lambda| < tau_i for up to two thresholds (lanes 0-1, 2-3)
__device__ __forceinline__ void small_counts(const Shared& S, int lane, const Spectrum& sp, double tau_a,
                                             double tau_b, int& ca, int& cb) {
    const int m = S.m;
    double sig = 0.0;
    if (lane == 0) sig = -tau_a;
    if (lane == 1) sig = tau_a;
    if (lane == 2) sig = -tau_b;
    if (lane == 3) sig = tau_b;
    int c = lane < 4 ? sturm(S, m, sig, sp.pivmin) : 0;
    int c0 = __shfl(c, 0, 64), c1 = __shfl(c, 1, 64), c2 = __shfl(c, 2, 64), c3 = __shfl(c, 3, 64);
    ca = c1 - c0;
    cb = c3 - c2;
}

// Smallest |lambda| (geometric multisection on both sides of zero).
__device__ double spectrum_min_abs(const Shared& S, int lane, const Spectrum& sp, int rounds) {
    const int m = S.m;
    const int nu = sturm(S, m, 0.0, sp.pivmin);  // eigenvalues below zero (uniform)
    const double H = sp.amax * (1.0 + 1e-12) + sp.pivmin;
    const double L = sp.amax * 1e-30 + sp.pivmin;
    double lp = log(L), hp = log(H), ln_ = log(L), hn = log(H);
    const int g = lane >> 5, t = lane & 31;
    for (int rd = 0; rd < rounds; ++rd) {
        const double lo = g ? ln_ : lp, hi = g ? hn : hp;
        const double sig = exp(lo + (hi - lo) * (double)(t + 1) / 33.0);
        bool above;  // target magnitude lies above sig
        if (g == 0) above = sturm(S, m, sig, sp.pivmin) <= nu;        // lambda_{nu+1} > sig
        else above = sturm(S, m, -sig, sp.pivmin) >= nu;              // lambda_nu < -sig
        const uint64_t bal = __ballot(above);
        const int nb1 = __popcll(bal & 0xffffffffull);
        const int nb2 = __popcll(bal >> 32);
        const double a1 = lp + (hp - lp) * (double)nb1 / 33.0, b1 = lp + (hp - lp) * (double)(nb1 + 1) / 33.0;
        const double a2 = ln_ + (hn - ln_) * (double)nb2 / 33.0, b2 = ln_ + (hn - ln_) * (double)(nb2 + 1) / 33.0;
        if (nb1 > 0) lp = a1;
        if (nb1 < 32) hp = b1;
        if (nb2 > 0) ln_ = a2;
        if (nb2 < 32) hn = b2;
    }
    double pos = nu < m ? exp(0.5 * (lp + hp)) : INFINITY;
    double neg = nu > 0 ? exp(0.5 * (ln_ + hn)) : INFINITY;
    return fmin(pos, neg);
}

// ------------------------------------------------------- tridiagonal solve ----
// Gaussian elimination with partial pivoting of T (lane 0); returns false on a zero pivot.
__device__ bool tri_factor(Shared& S) {
    const int m = S.m;
    for (int i = 0; i < m; ++i) {
        S.fd[i] = S.d[i];
        S.fdu[i] = i < m - 1 ? S.e[i] : 0.0;
        S.fdl[i] = i < m - 1 ? S.e[i] : 0.0;  // sub-diagonal, later the second super-diagonal
    }
    for (int i = 0; i < m - 1; ++i) {
        const double sub = S.fdl[i];
        if (fabs(S.fd[i]) >= fabs(sub)) {
            if (S.fd[i] == 0.0) return false;
            const double f = sub / S.fd[i];
            S.fd[i + 1] -= f * S.fdu[i];
            S.fdl[i] = 0.0;
            S.ffact[i] = f;
            S.fswap[i] = 0;
        } else {
            const double f = S.fd[i] / sub;
            S.fd[i] = sub;
            const double tmp = S.fd[i + 1];
            S.fd[i + 1] = S.fdu[i] - f * tmp;
            if (i < m - 2) {
                S.fdl[i] = S.fdu[i + 1];
                S.fdu[i + 1] = -f * S.fdl[i];
            } else {
                S.fdl[i] = 0.0;
            }
            S.fdu[i] = tmp;
            S.ffact[i] = f;
            S.fswap[i] = 1;
        }
    }
    return S.fd[m - 1] != 0.0;
}

__device__ void tri_solve(const Shared& S, double* b) {
    const int m = S.m;
    for (int i = 0; i < m - 1; ++i) {
        const double f = S.ffact[i];
        if (!S.fswap[i]) {
            b[i + 1] -= f * b[i];
        } else {
            const double t = b[i];
            b[i] = b[i + 1];
            b[i + 1] = t - f * b[i + 1];
        }
    }
    b[m - 1] /= S.fd[m - 1];
    if (m > 1) b[m - 2] = (b[m - 2] - S.fdu[m - 2] * b[m - 1]) / S.fd[m - 2];
    for (int i = m - 3; i >= 0; --i) b[i] = (b[i] - S.fdu[i] * b[i + 1] - S.fdl[i] * b[i + 2]) / S.fd[i];
}

// y <- Q^T y for three vectors (lane holds component `lane`)
__device__ __forceinline__ void apply_qt3(const double (&a)[MMAX], const Shared& S, double& y0, double& y1,
                                          double& y2) {
    const int m = S.m;
#pragma unroll
    for (int k = 0; k < MMAX - 2; ++k) {
        if (k < m - 2) {
            const double v = a[k];
            double s0 = v * y0, s1 = v * y1, s2 = v * y2;
            wave_sum3(s0, s1, s2);
            const double t = S.tau[k];
            y0 = fma(-t * s0, v, y0);
            y1 = fma(-t * s1, v, y1);
            y2 = fma(-t * s2, v, y2);
        }
    }
}
__device__ __forceinline__ void apply_q3(const double (&a)[MMAX], const Shared& S, double& y0, double& y1,
                                         double& y2) {
    const int m = S.m;
#pragma unroll
    for (int k = MMAX - 3; k >= 0; --k) {
        if (k < m - 2) {
            const double v = a[k];
            double s0 = v * y0, s1 = v * y1, s2 = v * y2;
            wave_sum3(s0, s1, s2);
            const double t = S.tau[k];
            y0 = fma(-t * s0, v, y0);
            y1 = fma(-t * s1, v, y1);
            y2 = fma(-t * s2, v, y2);
        }
    }
}
__device__ __forceinline__ void apply_qt1(const double (&a)[MMAX], const Shared& S, double& y) {
    const int m = S.m;
#pragma unroll
    for (int k = 0; k < MMAX - 2; ++k) {
        if (k < m - 2) {
            const double v = a[k];
            const double s = wave_sum(v * y);
            y = fma(-S.tau[k] * s, v, y);
        }
    }
}
__device__ __forceinline__ void apply_q1(const double (&a)[MMAX], const Shared& S, double& y) {
    const int m = S.m;
#pragma unroll
    for (int k = MMAX - 3; k >= 0; --k) {
        if (k < m - 2) {
            const double v = a[k];
            const double s = wave_sum(v * y);
            y = fma(-S.tau[k] * s, v, y);
        }
    }
}

// y <- A~^{-1} y for three vectors via Q T^{-1} Q^T (lane holds component `lane`)
__device__ __forceinline__ void solve3(const double (&a)[MMAX], Shared& S, int lane, double& y0, double& y1,
                                       double& y2) {
    const int m = S.m;
    apply_qt3(a, S, y0, y1, y2);
    S.rhs[0][lane] = y0;
    S.rhs[1][lane] = y1;
    S.rhs[2][lane] = y2;
    __syncthreads();
    if (lane < 3) tri_solve(S, S.rhs[lane]);
    __syncthreads();
    y0 = lane < m ? S.rhs[0][lane] : 0.0;
    y1 = lane < m ? S.rhs[1][lane] : 0.0;
    y2 = lane < m ? S.rhs[2][lane] : 0.0;
    __syncthreads();
    apply_q3(a, S, y0, y1, y2);
}

// (A~ z) for up to three vectors; z is read from S.zb, A~ is re-evaluated from the nodes
template <int K, int NV>
__device__ __forceinline__ void matvec_lds(const Shared& S, int lane, double e2, double (&out)[3]) {
    const int n = S.n, m = S.m, r = S.r;
    out[0] = out[1] = out[2] = 0.0;
    if (lane < n) {
        const double xi = S.x[lane], yi = S.y[lane], zi = S.z[lane];
        for (int j = 0; j < n; ++j) {
            const double dx = xi - S.x[j], dy = yi - S.y[j], dz = zi - S.z[j];
            const double a = rbf_phi<K>(e2, (dx * dx + dy * dy) + dz * dz);
#pragma unroll
            for (int v = 0; v < NV; ++v) out[v] = fma(a, S.zb[v][j], out[v]);
        }
        for (int k = 0; k < r; ++k) {
            const double u = S.U[lane * RMAX + k];
#pragma unroll
            for (int v = 0; v < NV; ++v) out[v] = fma(u, S.zb[v][n + k], out[v]);
        }
    } else if (lane < m) {
        const int k = lane - n;
        for (int j = 0; j < n; ++j) {
            const double u = S.U[j * RMAX + k];
#pragma unroll
            for (int v = 0; v < NV; ++v) out[v] = fma(u, S.zb[v][j], out[v]);
        }
    }
}

// One step of iterative refinement: z += A~^{-1} (b - A~ z).  The Householder
// route alone leaves an error several times that of LU with partial pivoting
// on these ill-conditioned saddle systems; one step brings it to that level.
template <int K>
__device__ __forceinline__ void refine3(const double (&a)[MMAX], Shared& S, int lane, double e2, double b0,
                                        double b1, double b2, double& z0, double& z1, double& z2) {
    S.zb[0][lane] = z0;
    S.zb[1][lane] = z1;
    S.zb[2][lane] = z2;
    __syncthreads();
    double az[3];
    matvec_lds<K, 3>(S, lane, e2, az);
    __syncthreads();
    double r0 = lane < S.m ? b0 - az[0] : 0.0, r1 = lane < S.m ? b1 - az[1] : 0.0, r2 = lane < S.m ? b2 - az[2] : 0.0;
    solve3(a, S, lane, r0, r1, r2);
    z0 += r0;
    z1 += r1;
    z2 += r2;
}

// --------------------------------------------------------------- border ----
// Monomials in xi (order: 1, x, y, z, x^2, y^2, z^2, xy, xz, yz), orthonormalised
// by MGS with one reorthogonalisation; kept columns are written to S.U and
// their monomial coefficients to S.T.  Degree 0 is the plain column of ones.
__device__ void build_border(Shared& S, int lane, int degree, double rank_tol, double xi, double yi, double zi) {
    const int n = S.n;
    if (degree == 0) {
        if (lane < n) S.U[lane * RMAX] = 1.0;
        if (lane < RMAX) S.T[lane * RMAX] = lane == 0 ? 1.0 : 0.0;
        if (lane == 0) S.r = 1;
        __syncthreads();
        return;
    }
    const int M = degree == 1 ? 4 : 10;
    const bool act = lane < n;
    double u[RMAX];
    u[0] = 1.0; u[1] = xi; u[2] = yi; u[3] = zi;
    u[4] = xi * xi; u[5] = yi * yi; u[6] = zi * zi; u[7] = xi * yi; u[8] = xi * zi; u[9] = yi * zi;
#pragma unroll
    for (int l = 0; l < RMAX; ++l)
        if (!act) u[l] = 0.0;
    // lane l (< M) holds row l of the coefficient matrix: column q of T in tc[q]
    double tc[RMAX];
#pragma unroll
    for (int q = 0; q < RMAX; ++q) tc[q] = (lane == q) ? 1.0 : 0.0;
    bool keep[RMAX];
    int r = 0;
#pragma unroll
    for (int l = 0; l < RMAX; ++l) {
        keep[l] = false;
        if (l < M) {
            const double on2 = wave_sum(u[l] * u[l]);
#pragma unroll
            for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
                for (int q = 0; q < l; ++q) {
                    if (keep[q]) {
                        const double c = wave_sum(u[q] * u[l]);
                        u[l] = fma(-c, u[q], u[l]);
                        tc[l] = fma(-c, tc[q], tc[l]);
                    }
                }
            }
            const double n2 = wave_sum(u[l] * u[l]);
            if (n2 > rank_tol * rank_tol * on2 && n2 > 0.0) {
                const double inv = 1.0 / sqrt(n2);
                u[l] *= inv;
                tc[l] *= inv;
                keep[l] = true;
                if (act) S.U[lane * RMAX + r] = u[l];
                if (lane < RMAX) S.T[lane * RMAX + r] = tc[l];
                ++r;
            }
        }
    }
    if (lane == 0) S.r = r;
    __syncthreads();
}

// ------------------------------------------------------ kappa evaluations ----
template <int K>
__device__ __forceinline__ Spectrum eval_spectrum(double (&a)[MMAX], Shared& S, int lane, double eps, int rounds) {
    build_matrix<K>(a, S, lane, eps * eps);
    tridiagonalise(a, S, lane);
    return spectrum_max(S, lane, rounds);
}

// kappa > target ?  (non-finite counts as above, like an infinite kappa)
__device__ __forceinline__ bool kappa_above(const Shared& S, int lane, const Spectrum& sp, double target) {
    if (!sp.finite || !(sp.amax > 0.0)) return true;
    int ca, cb;
    small_counts(S, lane, sp, sp.amax / target, sp.amax / target, ca, cb);
    return ca > 0;
}

// ------------------------------------------------------------------ kernel ----
template <int K>
__global__ __launch_bounds__(64) void k_weights(int64_t N, WOpts o, const double* __restrict__ xyz,
                                                const double* __restrict__ nrm, const int32_t* __restrict__ idx,
                                                const double* __restrict__ eps_in, double* __restrict__ w_out,
                                                double* __restrict__ eps_out, double* __restrict__ kappa_out,
                                                int32_t* __restrict__ status_out, int32_t* __restrict__ nevals_out,
                                                int kappa_only) {
    __shared__ Shared S;
    const int lane = threadIdx.x;
    const int64_t s = blockIdx.x;
    if (s >= N) return;
    const int n = o.n;
    // ---- gather the stencil
    const int node = lane < n ? idx[s * n + lane] : 0;
    double px = 0, py = 0, pz = 0, nx = 0, ny = 0, nz = 0;
    if (lane < n) {
        px = xyz[3 * (int64_t)node];
        py = xyz[3 * (int64_t)node + 1];
        pz = xyz[3 * (int64_t)node + 2];
        if (nrm) {
            nx = nrm[3 * (int64_t)node];
            ny = nrm[3 * (int64_t)node + 1];
            nz = nrm[3 * (int64_t)node + 2];
            double nn = sqrt(nx * nx + ny * ny + nz * nz);
            nx /= nn; ny /= nn; nz /= nn;
        }
        S.x[lane] = px;
        S.y[lane] = py;
        S.z[lane] = pz;
    }
    if (lane == 0) {
        S.nrm0[0] = nx; S.nrm0[1] = ny; S.nrm0[2] = nz;
        S.n = n;
    }
    __syncthreads();
    // ---- stencil radius and scaled offsets
    const double dx0 = px - S.x[0], dy0 = py - S.y[0], dz0 = pz - S.z[0];
    const double r20 = lane < n ? (dx0 * dx0 + dy0 * dy0) + dz0 * dz0 : 0.0;
    const bool dup = __ballot(lane > 0 && lane < n && r20 == 0.0) != 0;
    const double rho = sqrt(wave_max(r20));
    const double xi = dx0 / rho, yi = dy0 / rho, zi = dz0 / rho;
    build_border(S, lane, o.degree, o.rank_tol, xi, yi, zi);
    if (lane == 0) S.m = n + S.r;
    __syncthreads();
    const int m = S.m;
    int status = RBFFD_ST_OK;
    int evals = 0;
    double a[MMAX];
    double eps;
    if (dup) status = RBFFD_ST_DUPLICATE;

    // ---- shape parameter
    bool have_final = false;  // `a`/S hold the tridiagonal form at eps
    Spectrum sp;
    if (o.mode == RBFFD_EPS_FIXED) {
        eps = o.eps_fixed;
    } else if (o.mode == RBFFD_EPS_GIVEN) {
        eps = eps_in[s];
    } else {
        bool need_bisect = true;
        if (o.mode == RBFFD_EPS_LEARNED) {
            eps = eps_in[s];
            if (isfinite(eps) && eps > 0.0) {
                sp = eval_spectrum<K>(a, S, lane, eps, 6);
                ++evals;
                if (sp.finite && sp.amax > 0.0) {
                    int c_lo, c_hi;  // |lambda| below amax/band_lo and below amax/band_hi
                    small_counts(S, lane, sp, sp.amax / o.band_lo, sp.amax / o.band_hi, c_lo, c_hi);
                    // kappa > band_lo  and  kappa <= band_hi
                    if (c_lo > 0 && c_hi == 0) {
                        need_bisect = false;
                        have_final = true;
                    }
                }
            }
            if (need_bisect) status = status == RBFFD_ST_OK ? RBFFD_ST_FALLBACK : status;
        }
        if (need_bisect) {
            double lo = o.br_lo / rho, hi = o.br_hi / rho;
            bool ok = true;
            sp = eval_spectrum<K>(a, S, lane, lo, 5);
            ++evals;
            bool ab = kappa_above(S, lane, sp, o.kappa_target);
            for (int t = 0; !ab && t < o.max_expand; ++t) {
                lo *= 0.5;
                sp = eval_spectrum<K>(a, S, lane, lo, 5);
                ++evals;
                ab = kappa_above(S, lane, sp, o.kappa_target);
            }
            ok = ok && ab;
            sp = eval_spectrum<K>(a, S, lane, hi, 5);
            ++evals;
            ab = kappa_above(S, lane, sp, o.kappa_target);
            for (int t = 0; ab && t < o.max_expand; ++t) {
                hi *= 2.0;
                sp = eval_spectrum<K>(a, S, lane, hi, 5);
                ++evals;
                ab = kappa_above(S, lane, sp, o.kappa_target);
            }
            ok = ok && !ab;
            if (!ok && status == RBFFD_ST_OK) status = RBFFD_ST_NO_BRACKET;
            bool stop = false;
            while (hi - lo > o.eps_tol && !stop) {
                const double mid = 0.5 * (lo + hi);
                sp = eval_spectrum<K>(a, S, lane, mid, 5);
                ++evals;
                if (o.band_stop && sp.finite && sp.amax > 0.0) {
                    int c_lo, c_hi;
                    small_counts(S, lane, sp, sp.amax / o.band_lo, sp.amax / o.band_hi, c_lo, c_hi);
                    if (c_lo > 0 && c_hi == 0) {
                        eps = mid;
                        stop = true;
                        have_final = true;
                        break;
                    }
                }
                if (kappa_above(S, lane, sp, o.kappa_target)) lo = mid;
                else hi = mid;
            }
            if (!stop) eps = 0.5 * (lo + hi);
        }
    }
    if (!have_final) {
        sp = eval_spectrum<K>(a, S, lane, eps, 8);
        ++evals;
    }
    // ---- kappa_2 at the final eps
    double kappa = NAN;
    if (sp.finite && sp.amax > 0.0) {
        const double amin = spectrum_min_abs(S, lane, sp, 10);
        kappa = sp.amax / amin;
    } else if (status == RBFFD_ST_OK) {
        status = RBFFD_ST_NONFINITE;
    }
    if (!sp.finite && status == RBFFD_ST_OK) status = RBFFD_ST_NONFINITE;
    if (lane == 0) {
        if (eps_out) eps_out[s] = eps;
        if (kappa_out) kappa_out[s] = kappa;
        if (nevals_out) nevals_out[s] = evals;
    }
    if (kappa_only) {
        if (lane == 0 && status_out) status_out[s] = status;
        return;
    }

    // ---- weights: w = (A~^{-1} r)[:n], r = sum_d (B^d)^T g_d, g_d = (A~^{-1} b_d)[:n]
    __shared__ int fact_ok;
    if (lane == 0) fact_ok = sp.finite ? (int)tri_factor(S) : 0;
    __syncthreads();
    if (!fact_ok) {
        if (status == RBFFD_ST_OK) status = sp.finite ? RBFFD_ST_SINGULAR : RBFFD_ST_NONFINITE;
        if (lane == 0 && status_out) status_out[s] = status;
        if (lane < n) w_out[s * n + lane] = NAN;
        return;
    }
    const double e2 = eps * eps;
    const double n0x = S.nrm0[0], n0y = S.nrm0[1], n0z = S.nrm0[2];
    const double irho = 1.0 / rho;
    // b_d (row 1 of B^d) as an m-vector, component `lane`
    double b0 = 0, b1 = 0, b2 = 0;
    if (lane < n) {
        const double dx = S.x[0] - px, dy = S.y[0] - py, dz = S.z[0] - pz;  // x_1 - x_j
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        const double ps = rbf_psi<K>(e2, r2);
        const double dn = n0x * dx + n0y * dy + n0z * dz;
        b0 = ps * (dx - n0x * dn);
        b1 = ps * (dy - n0y * dn);
        b2 = ps * (dz - n0z * dn);
    } else if (lane < m && o.degree > 0) {
        const int k = lane - n;  // grad q_k at the centre (xi = 0): linear coefficients / rho
        const double gx = S.T[1 * RMAX + k] * irho, gy = S.T[2 * RMAX + k] * irho, gz = S.T[3 * RMAX + k] * irho;
        const double dn = n0x * gx + n0y * gy + n0z * gz;
        b0 = gx - n0x * dn;
        b1 = gy - n0y * dn;
        b2 = gz - n0z * dn;
    }
    {
        const double c0 = b0, c1 = b1, c2 = b2;
        solve3(a, S, lane, b0, b1, b2);
        refine3<K>(a, S, lane, e2, c0, c1, c2, b0, b1, b2);
    }
    // h_i = Pi_i g_i
    double hx = 0, hy = 0, hz = 0;
    if (lane < n) {
        const double dn = nx * b0 + ny * b1 + nz * b2;
        hx = b0 - nx * dn;
        hy = b1 - ny * dn;
        hz = b2 - nz * dn;
    }
    S.hx[lane] = hx;
    S.hy[lane] = hy;
    S.hz[lane] = hz;
    __syncthreads();
    // r_j = sum_i psi(r_ij) (x_i - x_j) . h_i   (j < n)
    double rj = 0.0;
#pragma unroll 4
    for (int i = 0; i < n; ++i) {
        const double dx = S.x[i] - px, dy = S.y[i] - py, dz = S.z[i] - pz;
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        const double ps = rbf_psi<K>(e2, r2);
        rj = fma(ps, dx * S.hx[i] + dy * S.hy[i] + dz * S.hz[i], rj);
    }
    if (lane >= n) rj = 0.0;
    // r_{n+k} = sum_i grad q_k(x_i) . h_i
    if (o.degree > 0) {
        const int r = S.r;
        for (int k = 0; k < r; ++k) {
            double c = 0.0;
            if (lane < n) {
                const double* T = S.T;
                const double t1 = T[1 * RMAX + k], t2 = T[2 * RMAX + k], t3 = T[3 * RMAX + k];
                double gx = t1, gy = t2, gz = t3;
                if (o.degree == 2) {
                    const double t4 = T[4 * RMAX + k], t5 = T[5 * RMAX + k], t6 = T[6 * RMAX + k];
                    const double t7 = T[7 * RMAX + k], t8 = T[8 * RMAX + k], t9 = T[9 * RMAX + k];
                    gx += 2.0 * t4 * xi + t7 * yi + t8 * zi;
                    gy += 2.0 * t5 * yi + t7 * xi + t9 * zi;
                    gz += 2.0 * t6 * zi + t8 * xi + t9 * yi;
                }
                c = (gx * hx + gy * hy + gz * hz) * irho;
            }
            c = wave_sum(c);
            if (lane == n + k) rj = c;
        }
    }
    double wv = rj, d1 = 0.0, d2 = 0.0;
    solve3(a, S, lane, wv, d1, d2);
    d1 = d2 = 0.0;
    refine3<K>(a, S, lane, e2, rj, 0.0, 0.0, wv, d1, d2);
    if (lane < n) w_out[s * n + lane] = wv;
    if (lane == 0 && status_out) status_out[s] = status;
}

template <int K>
void launch_weights(hipStream_t st, int64_t N, const WOpts& o, const double* xyz, const double* nrm,
                    const int32_t* idx, const double* eps_in, double* w, double* eps, double* kappa, int32_t* status,
                    int32_t* nevals, int kappa_only) {
    hipLaunchKernelGGL(k_weights<K>, dim3((unsigned)N), dim3(64), 0, st, N, o, xyz, nrm, idx, eps_in, w, eps,
                       kappa, status, nevals, kappa_only);
}

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
    if (o.n < 2 || o.n > 128 || (N > 0 && o.n > N)) return set_error(ctx, RBFFD_E_ARG, "stencil size n=%d invalid for N=%lld", o.n, (long long)N);
    if (o.kernel < 0 || o.kernel > 2) return set_error(ctx, RBFFD_E_ARG, "unknown kernel %d", o.kernel);
    if (o.degree < 0 || o.degree > 2) return set_error(ctx, RBFFD_E_ARG, "poly_degree must be 0, 1 or 2");
    if (o.mode < 0 || o.mode > 3) return set_error(ctx, RBFFD_E_ARG, "unknown eps_mode %d", o.mode);
    const int border = o.degree == 0 ? 1 : (o.degree == 1 ? 4 : 10);
    if (o.n + border > MMAX)
        return set_error(ctx, RBFFD_E_UNSUPPORTED, "n + border = %d exceeds %d on this path", o.n + border, MMAX);
    if (o.mode == RBFFD_EPS_FIXED && !(o.eps_fixed > 0.0)) return set_error(ctx, RBFFD_E_ARG, "eps_fixed must be > 0");
    if ((o.mode == RBFFD_EPS_BISECT || o.mode == RBFFD_EPS_LEARNED) &&
        !(o.kappa_target > 1.0 && o.eps_tol > 0.0 && o.br_lo > 0.0 && o.br_hi > o.br_lo))
        return set_error(ctx, RBFFD_E_ARG, "invalid bisection parameters");
    if ((o.mode == RBFFD_EPS_LEARNED || o.band_stop) && !(o.band_lo > 1.0 && o.band_hi >= o.band_lo))
        return set_error(ctx, RBFFD_E_ARG, "invalid kappa band");
    if (!(o.rank_tol >= 0.0)) return set_error(ctx, RBFFD_E_ARG, "rank_tol must be >= 0");
    if (o.max_expand < 0 || o.max_expand > 64) return set_error(ctx, RBFFD_E_ARG, "max_expand out of range");
    return RBFFD_OK;
}

int dispatch(rbffd_ctx ctx, int64_t N, const WOpts& o, const double* xyz, const double* nrm, const int32_t* idx,
             const double* eps_in, double* w, double* eps, double* kappa, int32_t* status, int32_t* nevals,
             int kappa_only) {
    hipStream_t st = ctx->stream;
    switch (o.kernel) {
        case RBFFD_KERNEL_MQ:
            launch_weights<RBFFD_KERNEL_MQ>(st, N, o, xyz, nrm, idx, eps_in, w, eps, kappa, status, nevals, kappa_only);
            break;
        case RBFFD_KERNEL_IMQ:
            launch_weights<RBFFD_KERNEL_IMQ>(st, N, o, xyz, nrm, idx, eps_in, w, eps, kappa, status, nevals, kappa_only);
            break;
        default:
            launch_weights<RBFFD_KERNEL_GA>(st, N, o, xyz, nrm, idx, eps_in, w, eps, kappa, status, nevals, kappa_only);
            break;
    }
    HIP_TRY(ctx, hipGetLastError());
    return RBFFD_OK;
}

}  // namespace

extern "C" int rbffd_build_weights(rbffd_ctx ctx, int64_t N, const double* xyz, const double* nrm,
                                   const rbffd_weight_opts* opts, const int32_t* idx_in, const double* eps_in,
                                   int32_t* idx_out, double* w, double* eps, double* kappa, int32_t* status,
                                   int32_t* nevals) {
    if (!ctx) return RBFFD_E_ARG;
    WOpts o;
    int rc = check_opts(ctx, N, opts, o);
    if (rc) return rc;
    if (N == 0) return RBFFD_OK;
    if (!xyz || !nrm || !w) return set_error(ctx, RBFFD_E_ARG, "null pointer");
    if ((o.mode == RBFFD_EPS_GIVEN || o.mode == RBFFD_EPS_LEARNED) && !eps_in)
        return set_error(ctx, RBFFD_E_ARG, "eps_in required for this eps_mode");
    const int32_t* idx = idx_in;
    if (!idx) {
        if (!idx_out) return set_error(ctx, RBFFD_E_ARG, "idx_out required when idx_in is NULL");
        rc = knn_internal(ctx, N, xyz, o.n, idx_out, nullptr);
        if (rc) return rc;
        idx = idx_out;
    } else if (idx_out && idx_out != idx_in) {
        HIP_TRY(ctx, hipMemcpyAsync(idx_out, idx_in, N * o.n * sizeof(int32_t), hipMemcpyDeviceToDevice, ctx->stream));
    }
    return dispatch(ctx, N, o, xyz, nrm, idx, eps_in, w, eps, kappa, status, nevals, 0);
}

extern "C" int rbffd_kappa(rbffd_ctx ctx, int64_t N, const double* xyz, const rbffd_weight_opts* opts,
                           const int32_t* idx, const double* eps_in, double* kappa) {
    if (!ctx) return RBFFD_E_ARG;
    WOpts o;
    int rc = check_opts(ctx, N, opts, o);
    if (rc) return rc;
    if (N == 0) return RBFFD_OK;
    if (!xyz || !idx || !eps_in || !kappa) return set_error(ctx, RBFFD_E_ARG, "null pointer");
    o.mode = RBFFD_EPS_GIVEN;
    return dispatch(ctx, N, o, xyz, nullptr, idx, eps_in, nullptr, nullptr, kappa, nullptr, nullptr, 1);
}
