// Device routines of the per-stencil weights computation (see weights.hip).
#pragma once

#include "common.h"
#include "weights_job.h"

#include <cmath>

namespace rbw {

constexpr int RMAX = RBW_RMAX;  // border columns (degree-2 monomials in R^3)
// Rows per guarded chunk in the tridiagonalisation loops (one wave / four
// waves per stencil): a chunk is skipped once all its rows are reduced, and a
// longer chunk lets its LDS reads be issued together (measured: 8 and 16 are
// 6-11% faster than 4; a single chunk of 64 is 40% slower).
template <int NB>
constexpr int chunk_rows() { return NB == 1 ? 8 : 16; }

// ------------------------------------------------------------ reductions ----
// Wavefront reductions with DPP (within rows of 16 lanes) and the row swaps
// (across the four rows).  Every lane must be active; the result is the same,
// bit for bit, in every lane.
// With every row and bank enabled and a permutation inside full rows, every
// lane reads a valid source lane, so no "old" value is needed (mov_dpp leaves
// it undefined and spares the two moves that would initialise it).
template <int CTRL>
__device__ __forceinline__ double dpp64(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double row_sum16(double v) {
    v += dpp64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp64<0x141>(v);  // row_half_mirror
    v += dpp64<0x140>(v);  // row_mirror
    return v;
}
// Cross-row step with the gfx950 row swaps, staying in vector registers: with
// both operands the same value, permlane16_swap gives every lane of rows
// (0, 1) the pair (r0, r1) and of rows (2, 3) the pair (r2, r3);
// permlane32_swap then pairs the two halves.  Every lane ends with
// (r0 + r1) + (r2 + r3) (op = max: the same association with fmax).
__device__ __forceinline__ void swap16(double v, double& a, double& b) {
    const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    a = __hiloint2double((int)h[0], (int)l[0]);
    b = __hiloint2double((int)h[1], (int)l[1]);
}
__device__ __forceinline__ void swap32(double v, double& a, double& b) {
    const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
    const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    a = __hiloint2double((int)h[0], (int)l[0]);
    b = __hiloint2double((int)h[1], (int)l[1]);
}
__device__ __forceinline__ double rows_total(double v) {
    double a, b;
    swap16(v, a, b);
    swap32(a + b, a, b);
    return a + b;
}
__device__ __forceinline__ double wave_sum(double v) { return rows_total(row_sum16(v)); }
// The same swaps with two different operands x (vdst) and y (vsrc):
// permlane32_swap leaves x = [x lanes 0-31, y lanes 0-31] and
// y = [x lanes 32-63, y lanes 32-63], so their sum folds x into lanes 0-31
// and y into lanes 32-63; permlane16_swap leaves x = [x row 0, y row 0, x row 2,
// y row 2] and y = [x row 1, y row 1, x row 3, y row 3] (rows of 16 lanes).
__device__ __forceinline__ double fold32(double x, double y) {
    const auto l = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(x), (unsigned)__double2loint(y), false,
                                                    false);
    const auto h = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(x), (unsigned)__double2hiint(y), false,
                                                    false);
    return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}
__device__ __forceinline__ double fold16(double x, double y) {
    const auto l = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(x), (unsigned)__double2loint(y), false,
                                                    false);
    const auto h = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(x), (unsigned)__double2hiint(y), false,
                                                    false);
    return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}
__device__ __forceinline__ double readlane64(double v, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}
// Four wavefront sums at once: the folds put a, c, b, d in rows 0..3.
__device__ __forceinline__ void wave_sum4(double& a, double& b, double& c, double& d) {
    const double s = fold32(a, b);
    const double t = fold32(c, d);
    const double u = row_sum16(fold16(s, t));
    a = readlane64(u, 0);
    c = readlane64(u, 16);
    b = readlane64(u, 32);
    d = readlane64(u, 48);
}
// Three wavefront sums at once: a and b share the first fold (a in lanes 0-31,
// b in 32-63), c is folded with itself, the second fold puts a, c, b, c in
// rows 0..3, one row sum finishes all three, and lanes 0, 32, 16 hand them
// to every lane.  About a third of the instructions of three wave_sum calls.
__device__ __forceinline__ void wave_sum3(double& a, double& b, double& c) {
    const double s = fold32(a, b);
    const double t = fold32(c, c);
    const double u = row_sum16(fold16(s, t));
    a = readlane64(u, 0);
    c = readlane64(u, 16);
    b = readlane64(u, 32);
}
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp64<0xB1>(v));
    v = fmax(v, dpp64<0x4E>(v));
    v = fmax(v, dpp64<0x141>(v));
    v = fmax(v, dpp64<0x140>(v));
    double a, b;
    swap16(v, a, b);
    swap32(fmax(a, b), a, b);
    return fmax(a, b);
}
// 1/q: hardware reciprocal and one Newton step (the step squares the hardware
// estimate's relative error).  Used by the Sturm recurrence, whose count only
// needs the sign of each pivot (which the recurrence gets backward-stably),
// by the tridiagonal factorisation, where an error of an ulp or two in a
// multiplier is a backward perturbation of T of the size GEPP itself leaves,
// and by the Householder reduction (tau and the scale of v).
__device__ __forceinline__ double recip(double q) {
    const double r = __builtin_amdgcn_rcp(q);
    return fma(r, fma(-q, r, 1.0), r);
}

// ---------------------------------------------------------- radial kernels ----
// sqrt(x) for x >= 1: the hardware reciprocal square root y ~ 1/sqrt(x),
// then g = x y, h = y / 2 refined by one coupled Newton step and two
// residual corrections g += (x - g^2) h, the last of which rounds correctly.
// The general square root adds a rescaling for tiny arguments and a class
// check (seven more instructions); the radial kernels' argument 1 + eps^2 r^2
// never needs them (for x >= 1 the two give the same bits; a non-finite x
// gives a non-finite result either way).
__device__ __forceinline__ double sqrt_ge1(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    return fma(d, h, g);
}
template <int K>
__device__ __forceinline__ double rbf_phi(double e2, double r2) {
    double e = e2 * r2;
    if (K == RBFFD_KERNEL_MQ) return sqrt_ge1(1.0 + e);
    if (K == RBFFD_KERNEL_IMQ) return 1.0 / sqrt_ge1(1.0 + e);
    return exp(-e);
}
// phi'(r)/r
template <int K>
__device__ __forceinline__ double rbf_psi(double e2, double r2) {
    double e = e2 * r2;
    if (K == RBFFD_KERNEL_MQ) return e2 / sqrt_ge1(1.0 + e);
    if (K == RBFFD_KERNEL_IMQ) return -e2 / (sqrt_ge1(1.0 + e) * (1.0 + e));
    return -2.0 * e2 * exp(-e);
}

// LDS of one stencil
template <int NB>
struct Shared {
    static constexpr int MM = 64 * NB;
    double x[MM], y[MM], z[MM];  // stencil node coordinates
    double U[MM * RMAX];         // border basis values U[j*RMAX + k]
    double T[RMAX * RMAX];       // monomial coefficients of the border basis T[l*RMAX + k]
    double col[MM], vv[MM], ww[MM], vb[MM];
    double pp[NB][MM];           // matvec partial sums per row block
    double red[16];              // cross-wave partial sums, two sets of 8
    double d[MM], e[MM], e2[MM], tau[MM];
    double fd[MM], fdu[MM], fdl[MM], ffact[MM];  // pivoted tridiagonal factors (fd: 1/pivot)
    int fswap[MM];
    double rhs[3][MM];
    double zb[3][MM];
    double hx[MM], hy[MM], hz[MM];
    double G[NB == 1 ? 96 : 1];  // Gram entries of the reflectors in blocks of four (one wave)
    double nrm0[3];
    int m, r, n, fact_ok;
};

// Position of a thread in the stencil's work group.
struct Tid {
    int lane;  // 0..63
    int rb;    // row block (rows 64 rb + jj held in registers)
    int cb;    // column block
    int c;     // column index 64 cb + lane
    int tid;   // 0 .. 64 NB^2 - 1 within the stencil's threads
    mutable int rot = 0;  // reductions done so far (selects the slot set)
};

template <int NB>
__device__ __forceinline__ void bsync() {
    if constexpr (NB == 1) {
        // one wavefront: order LDS accesses and keep the compiler from moving them
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Cross-wave partial sums (NB = 2) go through one of two slot sets, taken in
// turn by successive reductions; every reduction has one barrier between its
// writes and its reads, so by the time a set is written again every thread
// has read it, and no second barrier is needed.
__device__ __forceinline__ double* red_set(double* red, const Tid& t) { return red + 8 * (t.rot++ & 1); }

// Sum over the columns (lane-distributed; each column is held by NB threads).
template <int NB>
__device__ __forceinline__ double sum_cols(double v, Shared<NB>& S, const Tid& t) {
    const double w = wave_sum(v);
    if constexpr (NB == 1) {
        return w;
    } else {
        double* red = red_set(S.red, t);
        if (t.rb == 0 && t.lane == 0) red[t.cb] = w;
        bsync<NB>();
        return red[0] + red[1];
    }
}
template <int NB>
__device__ __forceinline__ void sum_cols3(double& a, double& b, double& c, Shared<NB>& S, const Tid& t) {
    wave_sum3(a, b, c);
    if constexpr (NB == 2) {
        double* red = red_set(S.red, t);
        if (t.rb == 0 && t.lane == 0) {
            red[t.cb] = a;
            red[2 + t.cb] = b;
            red[4 + t.cb] = c;
        }
        bsync<NB>();
        a = red[0] + red[1];
        b = red[2] + red[3];
        c = red[4] + red[5];
    }
}
// Sum over the rows held by lanes (row 64 rb + lane; cb == 0 waves count).
template <int NB>
__device__ __forceinline__ double sum_rows(double v, Shared<NB>& S, const Tid& t) {
    const double w = wave_sum(v);
    if constexpr (NB == 1) {
        return w;
    } else {
        double* red = red_set(S.red, t);
        if (t.cb == 0 && t.lane == 0) red[6 + t.rb] = w;
        bsync<NB>();
        return red[6] + red[7];
    }
}
// Four sums over the rows held by lanes at once (see sum_rows).
template <int NB>
__device__ __forceinline__ void sum_rows4(double& a, double& b, double& c, double& d, Shared<NB>& S, const Tid& t) {
    wave_sum4(a, b, c, d);
    if constexpr (NB == 2) {
        double* red = red_set(S.red, t);
        if (t.cb == 0 && t.lane == 0) {
            red[4 * t.rb] = a;
            red[4 * t.rb + 1] = b;
            red[4 * t.rb + 2] = c;
            red[4 * t.rb + 3] = d;
        }
        bsync<NB>();
        a = red[0] + red[4];
        b = red[1] + red[5];
        c = red[2] + red[6];
        d = red[3] + red[7];
    }
}
template <int NB>
__device__ __forceinline__ double max_cols(double v, Shared<NB>& S, const Tid& t) {
    const double w = wave_max(v);
    if constexpr (NB == 1) {
        return w;
    } else {
        double* red = red_set(S.red, t);
        if (t.rb == 0 && t.lane == 0) red[t.cb] = w;
        bsync<NB>();
        return fmax(red[0], red[1]);
    }
}

// ----------------------------------------------------------- local matrix ----
// Column t.c, rows 64 rb .. 64 rb + 63 of A~(eps).
template <int K, int NB>
__device__ __forceinline__ void build_matrix(double (&a)[64], const Shared<NB>& S, const Tid& t, double e2) {
    const int n = S.n, m = S.m, c = t.c;
    const int cc = c < n ? c : 0;
    const double xi = S.x[cc], yi = S.y[cc], zi = S.z[cc];
    const int r0 = 64 * t.rb;
#pragma unroll
    for (int jj = 0; jj < 64; ++jj) {
        const int j = r0 + jj;
        double v = 0.0;
        if (j < n) {
            if (c < n) {
                const double dx = xi - S.x[j], dy = yi - S.y[j], dz = zi - S.z[j];
                const double r2 = (dx * dx + dy * dy) + dz * dz;
                v = rbf_phi<K>(e2, r2);
            } else if (c < m) {
                v = S.U[j * RMAX + (c - n)];
            }
        } else if (j < m) {
            if (c < n) v = S.U[c * RMAX + (j - n)];
        }
        a[jj] = v;
    }
}

// Householder tridiagonalisation of the m x m leading block (lane = column).
// On return: S.d[0..m-1], S.e[0..m-2] (and e^2), S.tau[0..m-3], and row k of
// the register matrix holds the reflector v_k (v_k[k+1] = 1).
template <int NB>
__device__ __forceinline__ void tridiagonalise(double (&a)[64], Shared<NB>& S, const Tid& t) {
    constexpr int CH = chunk_rows<NB>();
    const int m = S.m, c = t.c, r0 = 64 * t.rb;
    if (t.rb == 0) S.col[c] = a[0];
    bsync<NB>();
    for (int k = 0; k < m - 2; ++k) {
        const double xi = S.col[c];
        const double alpha = S.col[k + 1];
        const double dk = S.col[k];
        const bool tail = c > k + 1 && c < m;
        const double xnorm2 = sum_cols<NB>(tail ? xi * xi : 0.0, S, t);
        double tau = 0.0, beta = alpha, scal = 0.0;
        if (xnorm2 > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
            // reciprocals instead of divisions: an ulp or so in tau and in the
            // scale of v, a perturbation of each reflector's orthogonality of
            // the size its own rounding already leaves
            tau = (beta - alpha) * recip(beta);
            scal = recip(alpha - beta);
        }
        const double vi = (c == k + 1) ? 1.0 : (tail ? xi * scal : 0.0);
        if (t.tid == 0) {
            S.d[k] = dk;
            S.e[k] = beta;
            S.e2[k] = beta * beta;
            S.tau[k] = tau;
        }
        if (t.rb == 0) S.vv[c] = vi;
        bsync<NB>();
        // p = A v over this thread's rows (rows <= k hold zero weight in v)
        double p0 = 0.0, p1 = 0.0;
#pragma unroll
        for (int j0 = 0; j0 < 64; j0 += CH) {
            if (r0 + j0 + CH > k + 1 && r0 + j0 < m) {
#pragma unroll
                for (int q = 0; q < CH; q += 2) {
                    p0 = fma(a[j0 + q], S.vv[r0 + j0 + q], p0);
                    p1 = fma(a[j0 + q + 1], S.vv[r0 + j0 + q + 1], p1);
                }
            }
        }
        double p = p0 + p1;
        if constexpr (NB == 2) {
            S.pp[t.rb][c] = p;
            bsync<NB>();
            p = S.pp[0][c] + S.pp[1][c];
        }
        double wi = (c > k && c < m) ? tau * p : 0.0;
        const double s = sum_cols<NB>(wi * vi, S, t);
        wi = fma(-0.5 * tau * s, vi, wi);
        if (t.rb == 0) S.ww[c] = wi;
        bsync<NB>();
        // A -= v w^T + w v^T; store v in row k; publish row k+1 as the next pivot column
#pragma unroll
        for (int j0 = 0; j0 < 64; j0 += CH) {
            if (r0 + j0 + CH > k + 1 && r0 + j0 < m) {
#pragma unroll
                for (int q = 0; q < CH; ++q)
                    a[j0 + q] = fma(-S.vv[r0 + j0 + q], wi, fma(-S.ww[r0 + j0 + q], vi, a[j0 + q]));
            }
            if (r0 + j0 <= k + 1 && k < r0 + j0 + CH) {  // this chunk holds row k or row k + 1
#pragma unroll
                for (int q = 0; q < CH; ++q) {
                    if (r0 + j0 + q == k) a[j0 + q] = vi;
                    if (r0 + j0 + q == k + 1) S.col[c] = a[j0 + q];
                }
            }
        }
        bsync<NB>();
    }
    // trailing 2 x 2 block
#pragma unroll
    for (int jj = 0; jj < 64; ++jj)
        if (r0 + jj == m - 1) S.ww[c] = a[jj];
    bsync<NB>();
    if (t.tid == 0) {
        if (m >= 2) {
            S.d[m - 2] = S.col[m - 2];
            S.e[m - 2] = S.col[m - 1];
            S.e2[m - 2] = S.col[m - 1] * S.col[m - 1];
        }
        S.d[m - 1] = S.ww[m - 1];
    }
    bsync<NB>();
}

// ------------------------------------------------------------ Sturm counts ----
// Number of eigenvalues of T below sigma.  Wave-local: every wave of a
// stencil may evaluate these (they read only S.d, S.e2).
template <int NB>
__device__ __forceinline__ int sturm(const Shared<NB>& S, int m, double sigma, double pivmin) {
    double q = S.d[0] - sigma;
    if (fabs(q) < pivmin) q = -pivmin;
    int c = q < 0.0 ? 1 : 0;
    for (int i = 1; i < m; ++i) {
        q = fma(-S.e2[i - 1], recip(q), S.d[i] - sigma);
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0 ? 1 : 0;
    }
    return c;
}

struct Spectrum {
    double amax;  // max |lambda| (midpoint estimate)
    bool finite;
    double pivmin;
    // multisection brackets: lambda_1 in [lo1, hi1], lambda_m in [lo2, hi2]
    double lo1, hi1, lo2, hi2;
};

// max |lambda| = max(-lambda_1, lambda_m) lies in [alo, ahi].
__device__ __forceinline__ void amax_bounds(const Spectrum& sp, double& alo, double& ahi) {
    alo = fmax(-sp.hi1, sp.lo2);
    ahi = fmax(-sp.lo1, sp.hi2);
}

// Up to `rounds` more multisection rounds on the brackets of lambda_1 and
// lambda_m.  While both can still be max |lambda| = max(-lambda_1, lambda_m),
// lanes 0..31 split lambda_1's bracket and lanes 32..63 lambda_m's 33 ways;
// once one of them is ruled out (its magnitude bound lies below the other's),
// all 64 lanes split the other's bracket 65 ways.  With rel > 0 the rounds
// stop as soon as the bracket of max |lambda| is within 2 rel of its midpoint
// (midpoint error <= rel relative).  sp.amax is that midpoint.
template <int NB>
__device__ __forceinline__ void spectrum_refine(const Shared<NB>& S, int lane, Spectrum& sp, int rounds,
                                                double rel = 0.0) {
    const int m = S.m;
    double lo1 = sp.lo1, hi1 = sp.hi1, lo2 = sp.lo2, hi2 = sp.hi2;
    for (int rd = 0; rd < rounds; ++rd) {
        // all conditions below are wave-uniform: the brackets are
        const double alo = fmax(-hi1, lo2), ahi = fmax(-lo1, hi2);
        if (rel > 0.0 && ahi - alo <= rel * (alo + ahi)) break;
        const bool need1 = !(lo2 > -lo1);  // lambda_1 can still be the largest in magnitude
        const bool need2 = !(-hi1 > hi2);  // lambda_m can
        if (need1 && need2) {
            const int g = lane >> 5, tt = lane & 31;
            const double lo = g ? lo2 : lo1, hi = g ? hi2 : hi1;
            const double sig = lo + (hi - lo) * (double)(tt + 1) / 33.0;
            const int kidx = g ? m : 1;
            const bool below = sturm<NB>(S, m, sig, sp.pivmin) < kidx;  // eigenvalue kidx lies above sig
            const uint64_t bal = __ballot(below);
            const int nb1 = __popcll(bal & 0xffffffffull);
            const int nb2 = __popcll(bal >> 32);
            const double n_lo1 = nb1 > 0 ? lo1 + (hi1 - lo1) * (double)nb1 / 33.0 : lo1;
            const double n_hi1 = nb1 < 32 ? lo1 + (hi1 - lo1) * (double)(nb1 + 1) / 33.0 : hi1;
            const double n_lo2 = nb2 > 0 ? lo2 + (hi2 - lo2) * (double)nb2 / 33.0 : lo2;
            const double n_hi2 = nb2 < 32 ? lo2 + (hi2 - lo2) * (double)(nb2 + 1) / 33.0 : hi2;
            lo1 = n_lo1; hi1 = n_hi1; lo2 = n_lo2; hi2 = n_hi2;
        } else {
            const double lo = need2 ? lo2 : lo1, hi = need2 ? hi2 : hi1;
            const double sig = lo + (hi - lo) * (double)(lane + 1) / 65.0;
            const bool below = sturm<NB>(S, m, sig, sp.pivmin) < (need2 ? m : 1);
            const int nb = __popcll(__ballot(below));
            const double n_lo = nb > 0 ? lo + (hi - lo) * (double)nb / 65.0 : lo;
            const double n_hi = nb < 64 ? lo + (hi - lo) * (double)(nb + 1) / 65.0 : hi;
            if (need2) {
                lo2 = n_lo;
                hi2 = n_hi;
            } else {
                lo1 = n_lo;
                hi1 = n_hi;
            }
        }
    }
    sp.lo1 = lo1; sp.hi1 = hi1; sp.lo2 = lo2; sp.hi2 = hi2;
    sp.amax = 0.5 * (fmax(-hi1, lo2) + fmax(-lo1, hi2));
}

// Largest |lambda| of T to ~33^-rounds of the Gershgorin width (see
// spectrum_refine for rel).
template <int NB>
__device__ __forceinline__ Spectrum spectrum_max(const Shared<NB>& S, int lane, int rounds, double rel = 0.0) {
    const int m = S.m;
    Spectrum sp;
    // Gershgorin interval of T: each lane takes rows lane, lane + 64, then
    // wavefront min/max (exact, so the same bits as a serial scan)
    // and the extreme diagonal entries, Rayleigh quotients of unit vectors:
    // lambda_1 <= min d_i and lambda_m >= max d_i
    double ngl = -INFINITY, gu = -INFINITY, emax2 = 0.0, dmax = -INFINITY, ndmin = -INFINITY;
    bool fin = true;
    for (int i = lane; i < m; i += 64) {
        const double off = (i > 0 ? fabs(S.e[i - 1]) : 0.0) + (i < m - 1 ? fabs(S.e[i]) : 0.0);
        ngl = fmax(ngl, off - S.d[i]);
        gu = fmax(gu, S.d[i] + off);
        dmax = fmax(dmax, S.d[i]);
        ndmin = fmax(ndmin, -S.d[i]);
        if (i < m - 1) emax2 = fmax(emax2, S.e2[i]);
        fin = fin && isfinite(S.d[i]) && (i == m - 1 || isfinite(S.e[i]));
    }
    double gl = -wave_max(ngl);
    gu = wave_max(gu);
    dmax = wave_max(dmax);
    const double dmin = -wave_max(ndmin);
    emax2 = wave_max(emax2);
    fin = __ballot(!fin) == 0;
    sp.finite = fin;
    sp.pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
    const double w = gu - gl;
    gl -= 2.0 * w * 2.2e-16 + 2.0 * sp.pivmin;
    gu += 2.0 * w * 2.2e-16 + 2.0 * sp.pivmin;
    sp.lo1 = gl;
    sp.hi2 = gu;
    // widened like the Gershgorin ends, for the counts' own rounding
    sp.hi1 = fmin(gu, dmin + 2.0 * w * 2.2e-16 + 2.0 * sp.pivmin);
    sp.lo2 = fmax(gl, dmax - 2.0 * w * 2.2e-16 - 2.0 * sp.pivmin);
    if (!fin) {
        sp.amax = NAN;
        return sp;
    }
    spectrum_refine<NB>(S, lane, sp, rounds, rel);
    return sp;
}

// #eigenvalues with |lambda| < tau for two thresholds (lanes 0-1 and 2-3)
template <int NB>
__device__ __forceinline__ void small_counts(const Shared<NB>& S, int lane, const Spectrum& sp, double tau_a,
                                             double tau_b, int& ca, int& cb) {
    const int m = S.m;
    double sig = 0.0;
    if (lane == 0) sig = -tau_a;
    if (lane == 1) sig = tau_a;
    if (lane == 2) sig = -tau_b;
    if (lane == 3) sig = tau_b;
    const int c = lane < 4 ? sturm<NB>(S, m, sig, sp.pivmin) : 0;
    const int c0 = __shfl(c, 0, 64), c1 = __shfl(c, 1, 64), c2 = __shfl(c, 2, 64), c3 = __shfl(c, 3, 64);
    ca = c1 - c0;
    cb = c3 - c2;
}

// Smallest |lambda| (geometric multisection on both sides of zero) within
// [L, H]; nu = #eigenvalues below zero.  The candidates are lambda_{nu+1} > 0
// and -lambda_nu > 0: while both can be the smaller, lanes 0..31 and 32..63
// split their log brackets 33 ways; once one is ruled out (or does not
// exist), all 64 lanes split the other's 65 ways.  Rounds continue until the
// log bracket of min |lambda| is 2 rel wide (midpoint error <= rel relative),
// at most `rounds`.
template <int NB>
__device__ __forceinline__ double min_abs_refine(const Shared<NB>& S, int lane, const Spectrum& sp, int nu, double lp,
                                                 double hp, double ln_, double hn, int rounds, double rel) {
    const int m = S.m;
    const bool has_pos = nu < m, has_neg = nu > 0;
    for (int rd = 0; rd < rounds; ++rd) {
        // wave-uniform: the brackets are
        const bool need_p = has_pos && !(has_neg && lp > hn);
        const bool need_n = has_neg && !(has_pos && ln_ > hp);
        const double blo = need_p ? (need_n ? fmin(lp, ln_) : lp) : ln_;
        const double bhi = need_p ? (need_n ? fmin(hp, hn) : hp) : hn;
        if (!(bhi - blo > 2.0 * rel)) break;
        if (need_p && need_n) {
            const int g = lane >> 5, tt = lane & 31;
            const double lo = g ? ln_ : lp, hi = g ? hn : hp;
            const double sig = exp(lo + (hi - lo) * (double)(tt + 1) / 33.0);
            bool above;  // target magnitude lies above sig
            if (g == 0) above = sturm<NB>(S, m, sig, sp.pivmin) <= nu;   // lambda_{nu+1} > sig
            else above = sturm<NB>(S, m, -sig, sp.pivmin) >= nu;         // lambda_nu < -sig
            const uint64_t bal = __ballot(above);
            const int nb1 = __popcll(bal & 0xffffffffull);
            const int nb2 = __popcll(bal >> 32);
            const double a1 = lp + (hp - lp) * (double)nb1 / 33.0, b1 = lp + (hp - lp) * (double)(nb1 + 1) / 33.0;
            const double a2 = ln_ + (hn - ln_) * (double)nb2 / 33.0, b2 = ln_ + (hn - ln_) * (double)(nb2 + 1) / 33.0;
            if (nb1 > 0) lp = a1;
            if (nb1 < 32) hp = b1;
            if (nb2 > 0) ln_ = a2;
            if (nb2 < 32) hn = b2;
        } else {
            const double lo = need_p ? lp : ln_, hi = need_p ? hp : hn;
            const double sig = exp(lo + (hi - lo) * (double)(lane + 1) / 65.0);
            const bool above = need_p ? sturm<NB>(S, m, sig, sp.pivmin) <= nu : sturm<NB>(S, m, -sig, sp.pivmin) >= nu;
            const int nb = __popcll(__ballot(above));
            const double a1 = lo + (hi - lo) * (double)nb / 65.0, b1 = lo + (hi - lo) * (double)(nb + 1) / 65.0;
            const double n_lo = nb > 0 ? a1 : lo, n_hi = nb < 64 ? b1 : hi;
            if (need_p) {
                lp = n_lo;
                hp = n_hi;
            } else {
                ln_ = n_lo;
                hn = n_hi;
            }
        }
    }
    const double pos = has_pos ? exp(0.5 * (lp + hp)) : INFINITY;
    const double neg = has_neg ? exp(0.5 * (ln_ + hn)) : INFINITY;
    return fmin(pos, neg);
}

template <int NB>
__device__ __forceinline__ double spectrum_min_abs_in(const Shared<NB>& S, int lane, const Spectrum& sp, int nu,
                                                      double L, double H, int rounds, double rel) {
    return min_abs_refine<NB>(S, lane, sp, nu, log(L), log(H), log(L), log(H), rounds, rel);
}

// The band test of a learned proposal and the first round of its min |lambda|
// search in one Sturm pass: lanes 0-3 count the eigenvalues with
// |lambda| < tau_a and < tau_b, lane 4 those below zero (nu), and lanes 8-35
// / 36-63 split [tau_b, tau_a] (log scale) 29 ways on the positive / negative
// side.  If the proposal is kept (ca > 0, cb == 0), min |lambda| lies in
// [tau_b, tau_a), and the returned log brackets (lp, hp) and (ln_, hn) are
// those after that first round.
template <int NB>
__device__ __forceinline__ void band_counts_min(const Shared<NB>& S, int lane, const Spectrum& sp, double tau_a,
                                                double tau_b, int& ca, int& cb, int& nu, double& lp, double& hp,
                                                double& ln_, double& hn) {
    const int m = S.m;
    const double l0 = log(tau_b), l1 = log(tau_a);
    double sig = 0.0;
    if (lane == 0) sig = -tau_a;
    if (lane == 1) sig = tau_a;
    if (lane == 2) sig = -tau_b;
    if (lane == 3) sig = tau_b;
    const bool pos_lane = lane >= 8 && lane < 36, neg_lane = lane >= 36;
    if (pos_lane) sig = exp(l0 + (l1 - l0) * (double)(lane - 8 + 1) / 29.0);
    if (neg_lane) sig = -exp(l0 + (l1 - l0) * (double)(lane - 36 + 1) / 29.0);
    const int c = (lane < 5 || lane >= 8) ? sturm<NB>(S, m, sig, sp.pivmin) : 0;
    const int c0 = __shfl(c, 0, 64), c1 = __shfl(c, 1, 64), c2 = __shfl(c, 2, 64), c3 = __shfl(c, 3, 64);
    ca = c1 - c0;
    cb = c3 - c2;
    nu = __shfl(c, 4, 64);
    // lambda_{nu+1} > sig (positive lanes), lambda_nu < sig (negative lanes)
    const bool above = pos_lane ? c <= nu : (neg_lane ? c >= nu : false);
    const uint64_t bal = __ballot(above);
    const int nb1 = __popcll((bal >> 8) & 0xfffffffull);
    const int nb2 = __popcll(bal >> 36);
    lp = l0; hp = l1; ln_ = l0; hn = l1;
    if (nb1 > 0) lp = l0 + (l1 - l0) * (double)nb1 / 29.0;
    if (nb1 < 28) hp = l0 + (l1 - l0) * (double)(nb1 + 1) / 29.0;
    if (nb2 > 0) ln_ = l0 + (l1 - l0) * (double)nb2 / 29.0;
    if (nb2 < 28) hn = l0 + (l1 - l0) * (double)(nb2 + 1) / 29.0;
}

// Smallest |lambda| with no prior bracket: [1e-30, 1] x max |lambda|, 7 rounds.
template <int NB>
__device__ __forceinline__ double spectrum_min_abs(const Shared<NB>& S, int lane, const Spectrum& sp) {
    const int nu = sturm<NB>(S, S.m, 0.0, sp.pivmin);  // eigenvalues below zero (uniform)
    return spectrum_min_abs_in<NB>(S, lane, sp, nu, sp.amax * 1e-30 + sp.pivmin,
                                   sp.amax * (1.0 + 1e-12) + sp.pivmin, 7, 0.0);
}

// ------------------------------------------------------- tridiagonal solve ----
// Gaussian elimination with partial pivoting of T (one thread); false on a
// zero pivot.  The diagonal and super-diagonal of the row being eliminated are
// carried in registers, so each step reads LDS only for inputs that do not
// depend on the previous step.
template <int NB>
__device__ __forceinline__ bool tri_factor(Shared<NB>& S) {
    const int m = S.m;
    double dcur = S.d[0];                      // pivot-row diagonal (after earlier steps)
    double ucur = m > 1 ? S.e[0] : 0.0;        // its super-diagonal
    for (int i = 0; i < m - 1; ++i) {
        const double sub = S.e[i];             // sub-diagonal entry below the pivot
        const double dnext = S.d[i + 1];
        const double unext = i < m - 2 ? S.e[i + 1] : 0.0;
        // The pivot's reciprocal (hardware reciprocal + one Newton step) gives
        // the multiplier too, which keeps a full division off the serial chain.
        if (fabs(dcur) >= fabs(sub)) {
            if (dcur == 0.0) return false;
            const double rp = recip(dcur);
            const double f = sub * rp;
            S.fd[i] = rp;                      // reciprocal of the pivot
            S.fdu[i] = ucur;
            S.fdl[i] = 0.0;
            S.ffact[i] = f;
            S.fswap[i] = 0;
            dcur = dnext - f * ucur;
            ucur = unext;
        } else {                               // swap rows i and i + 1
            const double rp = recip(sub);
            const double f = dcur * rp;
            S.fd[i] = rp;
            S.fdu[i] = dnext;
            S.fdl[i] = i < m - 2 ? unext : 0.0;  // second super-diagonal
            S.ffact[i] = f;
            S.fswap[i] = 1;
            dcur = ucur - f * dnext;
            ucur = i < m - 2 ? -f * unext : unext;
        }
    }
    if (dcur == 0.0) return false;
    S.fd[m - 1] = recip(dcur);
    S.fdu[m - 1] = 0.0;
    S.fdl[m - 1] = 0.0;
    return true;
}

// b <- T^{-1} b with the factors of tri_factor (one thread); the running
// entries of b are carried in registers.
template <int NB>
__device__ __forceinline__ void tri_solve(const Shared<NB>& S, double* b) {
    const int m = S.m;
    double bi = b[0];
    for (int i = 0; i < m - 1; ++i) {
        const double f = S.ffact[i];
        const double bn = b[i + 1];
        if (!S.fswap[i]) {
            b[i] = bi;
            bi = bn - f * bi;
        } else {
            b[i] = bn;
            bi = bi - f * bn;
        }
    }
    double x1 = bi * S.fd[m - 1];  // x_{i+1}
    b[m - 1] = x1;
    if (m < 2) return;
    double x2 = x1;                // x_{i+2}
    x1 = (b[m - 2] - S.fdu[m - 2] * x2) * S.fd[m - 2];
    b[m - 2] = x1;
    for (int i = m - 3; i >= 0; --i) {
        const double x = (b[i] - S.fdu[i] * x1 - S.fdl[i] * x2) * S.fd[i];
        b[i] = x;
        x2 = x1;
        x1 = x;
    }
}

// y <- Q^T y (FWD) or y <- Q y, for NV = 1 or 3 vectors (thread holds component
// t.c).  The reflector v_k is register row k (NB = 1) or is published through
// LDS by the row block that holds row k (NB = 2).
template <int NB, int NV, bool FWD>
__device__ __forceinline__ void apply_q(const double (&a)[64], Shared<NB>& S, const Tid& t, double (&y)[3]) {
    const int m = S.m;
    constexpr int MM = 64 * NB;
#pragma unroll
    for (int kk = 0; kk < MM - 2; ++kk) {
        const int k = FWD ? kk : MM - 3 - kk;  // a compile-time constant after unrolling
        if (k < m - 2) {
            double v;
            if constexpr (NB == 1) {
                v = a[k];
            } else {
                if (t.rb == k / 64) S.vb[t.c] = a[k % 64];
                bsync<NB>();
                v = S.vb[t.c];
            }
            if constexpr (NV == 3) {
                double s0 = v * y[0], s1 = v * y[1], s2 = v * y[2];
                sum_cols3<NB>(s0, s1, s2, S, t);  // ends with a barrier when NB = 2
                const double ta = S.tau[k];
                y[0] = fma(-ta * s0, v, y[0]);
                y[1] = fma(-ta * s1, v, y[1]);
                y[2] = fma(-ta * s2, v, y[2]);
            } else {
                const double s0 = sum_cols<NB>(v * y[0], S, t);
                y[0] = fma(-S.tau[k] * s0, v, y[0]);
            }
        }
    }
}

// One wave (NB = 1), NV vectors: Q^T y (FWD) or Q y four reflectors at a time.
// For a block H_{k0} .. H_{k0+3} the four products d_i = v_i . y of a vector
// are reduced together, and the coupling of successive reflectors inside the
// block comes from their Gram entries G_ij = v_i . v_j (S.G, six per block,
// from reflector_gram): applying H_{k0} first, s_i = d_i - sum_{j<i} tau_j s_j G_ij
// and y -= sum_i tau_i s_i v_i (the reverse order for Q y).  Rows past the last
// reflector enter with v = 0 and tau = 0.
template <int NB, int NV, bool FWD>
__device__ __forceinline__ void apply_q_blocked(const double (&a)[64], Shared<NB>& S, double (&y)[3]) {
    static_assert(NB == 1, "one-wave tiling only");
    const int p = S.m - 2;
#pragma unroll
    for (int bb = 0; bb < 16; ++bb) {
        const int b = FWD ? bb : 15 - bb;
        const int k0 = 4 * b;
        if (k0 < p) {
            const double v0 = a[k0], v1 = k0 + 1 < p ? a[k0 + 1] : 0.0;
            const double v2 = k0 + 2 < p ? a[k0 + 2] : 0.0, v3 = k0 + 3 < p ? a[k0 + 3] : 0.0;
            const double t0 = S.tau[k0], t1 = k0 + 1 < p ? S.tau[k0 + 1] : 0.0;
            const double t2 = k0 + 2 < p ? S.tau[k0 + 2] : 0.0, t3 = k0 + 3 < p ? S.tau[k0 + 3] : 0.0;
            double d[NV][4];
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                d[q][0] = v0 * y[q];
                d[q][1] = v1 * y[q];
                d[q][2] = v2 * y[q];
                d[q][3] = v3 * y[q];
            }
#pragma unroll
            for (int q = 0; q < NV; ++q) wave_sum4(d[q][0], d[q][1], d[q][2], d[q][3]);
            const double* G = S.G + 6 * b;  // G01 G02 G03 G12 G13 G23
            const double g01 = G[0], g02 = G[1], g03 = G[2], g12 = G[3], g13 = G[4], g23 = G[5];
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                double s0, s1, s2, s3;
                if (FWD) {
                    s0 = d[q][0];
                    s1 = fma(-t0 * s0, g01, d[q][1]);
                    s2 = fma(-t1 * s1, g12, fma(-t0 * s0, g02, d[q][2]));
                    s3 = fma(-t2 * s2, g23, fma(-t1 * s1, g13, fma(-t0 * s0, g03, d[q][3])));
                } else {
                    s3 = d[q][3];
                    s2 = fma(-t3 * s3, g23, d[q][2]);
                    s1 = fma(-t2 * s2, g12, fma(-t3 * s3, g13, d[q][1]));
                    s0 = fma(-t1 * s1, g01, fma(-t2 * s2, g02, fma(-t3 * s3, g03, d[q][0])));
                }
                y[q] = fma(-t3 * s3, v3, fma(-t2 * s2, v2, fma(-t1 * s1, v1, fma(-t0 * s0, v0, y[q]))));
            }
        }
    }
}

// S.G for apply_q_blocked (one wave, after the final tridiagonalisation).
template <int NB>
__device__ __forceinline__ void reflector_gram(const double (&a)[64], Shared<NB>& S, const Tid& t) {
    static_assert(NB == 1, "one-wave tiling only");
    const int p = S.m - 2;
#pragma unroll
    for (int b = 0; b < 16; ++b) {
        const int k0 = 4 * b;
        if (k0 < p) {
            const double v0 = a[k0], v1 = k0 + 1 < p ? a[k0 + 1] : 0.0;
            const double v2 = k0 + 2 < p ? a[k0 + 2] : 0.0, v3 = k0 + 3 < p ? a[k0 + 3] : 0.0;
            double g01 = v0 * v1, g02 = v0 * v2, g03 = v0 * v3, g12 = v1 * v2;
            double g13 = v1 * v3, g23 = v2 * v3, z0 = 0.0, z1 = 0.0;
            wave_sum4(g01, g02, g03, g12);
            wave_sum4(g13, g23, z0, z1);
            if (t.tid == 0) {
                double* G = S.G + 6 * b;
                G[0] = g01; G[1] = g02; G[2] = g03; G[3] = g12; G[4] = g13; G[5] = g23;
            }
        }
    }
    bsync<NB>();
}

// y <- A~^{-1} y via Q T^{-1} Q^T
template <int NB, int NV>
__device__ __forceinline__ void solve(const double (&a)[64], Shared<NB>& S, const Tid& t, double (&y)[3]) {
    const int m = S.m;
    if constexpr (NB == 1) apply_q_blocked<NB, NV, true>(a, S, y);
    else apply_q<NB, NV, true>(a, S, t, y);
    if (t.rb == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) S.rhs[v][t.c] = y[v];
    }
    bsync<NB>();
    if (t.tid < NV) tri_solve<NB>(S, S.rhs[t.tid]);
    bsync<NB>();
#pragma unroll
    for (int v = 0; v < NV; ++v) y[v] = t.c < m ? S.rhs[v][t.c] : 0.0;
    bsync<NB>();
    if constexpr (NB == 1) apply_q_blocked<NB, NV, false>(a, S, y);
    else apply_q<NB, NV, false>(a, S, t, y);
}

// (A~ z) row t.c for NV vectors read from S.zb; A~ re-evaluated from the nodes
template <int K, int NB, int NV>
__device__ __forceinline__ void matvec_lds(const Shared<NB>& S, const Tid& t, double e2, double (&out)[3]) {
    const int n = S.n, m = S.m, r = S.r, c = t.c;
    out[0] = out[1] = out[2] = 0.0;
    if (c < n) {
        const double xi = S.x[c], yi = S.y[c], zi = S.z[c];
        for (int j = 0; j < n; ++j) {
            const double dx = xi - S.x[j], dy = yi - S.y[j], dz = zi - S.z[j];
            const double av = rbf_phi<K>(e2, (dx * dx + dy * dy) + dz * dz);
#pragma unroll
            for (int v = 0; v < NV; ++v) out[v] = fma(av, S.zb[v][j], out[v]);
        }
        for (int k = 0; k < r; ++k) {
            const double u = S.U[c * RMAX + k];
#pragma unroll
            for (int v = 0; v < NV; ++v) out[v] = fma(u, S.zb[v][n + k], out[v]);
        }
    } else if (c < m) {
        const int k = c - n;
        for (int j = 0; j < n; ++j) {
            const double u = S.U[j * RMAX + k];
#pragma unroll
            for (int v = 0; v < NV; ++v) out[v] = fma(u, S.zb[v][j], out[v]);
        }
    }
}

// Solve with one step of iterative refinement: z = A~^{-1} b, z += A~^{-1}(b - A~ z).
// The Householder route alone leaves an error several times that of LU with
// partial pivoting on these ill-conditioned saddle systems; one step brings it
// to that level.
template <int K, int NB, int NV>
__device__ __forceinline__ void solve_refined(const double (&a)[64], Shared<NB>& S, const Tid& t, double e2,
                                              double (&y)[3]) {
    const double b[3] = {y[0], y[1], y[2]};
    solve<NB, NV>(a, S, t, y);
    if (t.rb == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) S.zb[v][t.c] = y[v];
    }
    bsync<NB>();
    double az[3];
    matvec_lds<K, NB, NV>(S, t, e2, az);
    bsync<NB>();
    double r[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int v = 0; v < NV; ++v) r[v] = t.c < S.m ? b[v] - az[v] : 0.0;
    solve<NB, NV>(a, S, t, r);
#pragma unroll
    for (int v = 0; v < NV; ++v) y[v] += r[v];
}

// --------------------------------------------------------------- border ----
// Monomials in xi (order: 1, x, y, z, x^2, y^2, z^2, xy, xz, yz) at row
// jr = 64 rb + lane, orthonormalised by classical Gram-Schmidt applied twice
// (the projections on all earlier kept columns formed together, four sums at
// a time, then subtracted; once more on the result); kept
// columns go to S.U and their monomial coefficients to S.T.  A column is
// dropped when its residual norm is at most rank_tol times the largest column
// norm, that of the ones column (sqrt n; every |xi| <= 1), the analogue of a
// singular value cut relative to the largest one.  (Relative to the column's
// own norm would miss an exact dependency among small columns: at the poles
// of a fine sphere the z^2 column, of norm ~1e-4 sqrt n, keeps a rounding
// residual of 4e-10 of its norm.)  Degree 0 is the plain column of ones.
template <int NB>
__device__ __forceinline__ void build_border(Shared<NB>& S, const Tid& t, int degree, double rank_tol, double xr, double yr,
                             double zr) {
    const int n = S.n;
    const int jr = 64 * t.rb + t.lane;
    if (degree == 0) {
        if (t.cb == 0 && jr < n) S.U[jr * RMAX] = 1.0;
        if (t.tid < RMAX) S.T[t.tid * RMAX] = t.tid == 0 ? 1.0 : 0.0;
        if (t.tid == 0) S.r = 1;
        bsync<NB>();
        return;
    }
    const int M = degree == 1 ? 4 : 10;
    const bool act = jr < n;
    double u[RMAX];
    u[0] = 1.0; u[1] = xr; u[2] = yr; u[3] = zr;
    u[4] = xr * xr; u[5] = yr * yr; u[6] = zr * zr; u[7] = xr * yr; u[8] = xr * zr; u[9] = yr * zr;
#pragma unroll
    for (int l = 0; l < RMAX; ++l)
        if (!act) u[l] = 0.0;
    // thread l (< M) of the stencil holds row l of the coefficient matrix
    double tc[RMAX];
#pragma unroll
    for (int q = 0; q < RMAX; ++q) tc[q] = (t.tid == q) ? 1.0 : 0.0;
    bool keep[RMAX];
    int r = 0;
#pragma unroll
    for (int l = 0; l < RMAX; ++l) {
        keep[l] = false;
        if (l < M) {
#pragma unroll
            for (int pass = 0; pass < 2; ++pass) {
                double cq[RMAX];
#pragma unroll
                for (int q0 = 0; q0 < l; q0 += 4) {  // constant trip counts: u, tc, keep stay in registers
                    double g[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) g[i] = (q0 + i < l && keep[q0 + i]) ? u[q0 + i] * u[l] : 0.0;
                    sum_rows4<NB>(g[0], g[1], g[2], g[3], S, t);
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (q0 + i < l) cq[q0 + i] = g[i];
                }
#pragma unroll
                for (int q = 0; q < l; ++q) {
                    u[l] = fma(-cq[q], u[q], u[l]);
                    tc[l] = fma(-cq[q], tc[q], tc[l]);
                }
            }
            const double n2 = sum_rows<NB>(u[l] * u[l], S, t);
            if (n2 > rank_tol * rank_tol * (double)n && n2 > 0.0) {
                const double inv = 1.0 / sqrt(n2);
                u[l] *= inv;
                tc[l] *= inv;
                keep[l] = true;
                if (act && t.cb == 0) S.U[jr * RMAX + r] = u[l];
                if (t.tid < RMAX) S.T[t.tid * RMAX + r] = tc[l];
                ++r;
            }
        }
    }
    if (t.tid == 0) S.r = r;
    bsync<NB>();
}

// ------------------------------------------------------ kappa evaluations ----
template <int K, int NB>
__device__ __forceinline__ Spectrum eval_spectrum(double (&a)[64], Shared<NB>& S, const Tid& t, double eps,
                                                  int rounds, double rel = 0.0) {
    build_matrix<K, NB>(a, S, t, eps * eps);
    tridiagonalise<NB>(a, S, t);
    return spectrum_max<NB>(S, t.lane, rounds, rel);
}

// kappa_2(T) > target ?  (non-finite counts as above, like an infinite kappa)
// kappa > target exactly when some |lambda| < max|lambda| / target.  With
// max |lambda| known to lie in [alo, ahi], an eigenvalue below alo / target
// decides "above" and none below ahi / target decides "not above"; only when
// the two counts differ is max |lambda| refined (two multisection rounds at a
// time), so every decision is the one the Sturm counts of T give at the exact
// max |lambda|, up to a bracket of a few ulps.  sp's brackets are refined in place.
template <int NB>
__device__ __forceinline__ bool kappa_above(const Shared<NB>& S, int lane, Spectrum& sp, double target) {
    if (!sp.finite || !(sp.amax > 0.0)) return true;
    for (int it = 0; it < 12; ++it) {
        double alo, ahi;
        amax_bounds(sp, alo, ahi);
        int ca, cb;
        small_counts<NB>(S, lane, sp, alo / target, ahi / target, ca, cb);
        if (ca > 0) return true;
        if (cb == 0) return false;
        if (ahi - alo <= 8.0 * 2.2e-16 * ahi) break;  // bracket at FP64 resolution
        spectrum_refine<NB>(S, lane, sp, 2);
    }
    int ca, cb;
    small_counts<NB>(S, lane, sp, sp.amax / target, sp.amax / target, ca, cb);
    return ca > 0;
}

// --------------------------------------------------------------- stencil ----
// The whole computation for stencil s of job J by the NB^2 waves of one stencil.
template <int K, int NB>
__device__ __forceinline__ void process_stencil(const Job& J, int64_t s, Shared<NB>& S, const Tid& t) {
    const WOpts& o = J.o;
    const int n = o.n;
    const int c = t.c;
    // ---- gather the stencil (thread's column node; rb == 0 threads fill LDS)
    double px = 0, py = 0, pz = 0, nx = 0, ny = 0, nz = 0;
    bool bad = false;   // stencil index outside [0, N): read node 0 instead, flag the stencil
    bool badn = false;  // zero or non-finite normal: Pi_i undefined, flag the stencil
    if (c < n) {
        int64_t node = J.idx[s * n + c];
        bad = node < 0 || node >= J.N;
        if (bad) node = 0;
        px = J.xyz[3 * node];
        py = J.xyz[3 * node + 1];
        pz = J.xyz[3 * node + 2];
        if (J.nrm) {
            nx = J.nrm[3 * node];
            ny = J.nrm[3 * node + 1];
            nz = J.nrm[3 * node + 2];
            const double nn = sqrt(nx * nx + ny * ny + nz * nz);
            badn = !(nn > 0.0 && nn <= 1.79e308);
            const double dn = badn ? 1.0 : nn;
            nx /= dn; ny /= dn; nz /= dn;
        }
        if (t.rb == 0) {
            S.x[c] = px;
            S.y[c] = py;
            S.z[c] = pz;
        }
    }
    if (t.tid == 0) {
        S.nrm0[0] = nx; S.nrm0[1] = ny; S.nrm0[2] = nz;
        S.n = n;
    }
    bsync<NB>();
    // ---- stencil radius, scaled offsets of the thread's column node and row node
    const double dx0 = px - S.x[0], dy0 = py - S.y[0], dz0 = pz - S.z[0];
    const double r20 = c < n ? (dx0 * dx0 + dy0 * dy0) + dz0 * dz0 : 0.0;
    // 3: an index out of range somewhere in the stencil; 2: a zero or
    // non-finite normal; 1: two nodes coincide
    const double flagf =
        max_cols<NB>(bad ? 3.0 : (badn ? 2.0 : ((c > 0 && c < n && r20 == 0.0) ? 1.0 : 0.0)), S, t);
    if (flagf >= 2.0) {
        if (t.tid == 0) {
            if (J.eps) J.eps[s] = NAN;
            if (J.kappa) J.kappa[s] = NAN;
            if (J.nevals) J.nevals[s] = 0;
            if (J.status) J.status[s] = flagf >= 3.0 ? RBFFD_ST_BAD_INDEX : RBFFD_ST_BAD_NORMAL;
        }
        if (!J.kappa_only && c < n && t.rb == 0) J.w[s * n + c] = NAN;
        bsync<NB>();
        return;
    }
    const double dupf = flagf;
    const double rho = sqrt(max_cols<NB>(r20, S, t));
    const double irho = 1.0 / rho;
    const double xi = dx0 / rho, yi = dy0 / rho, zi = dz0 / rho;
    const int jr = 64 * t.rb + t.lane;
    double xr = 0, yr = 0, zr = 0;
    if (jr < n) {
        xr = (S.x[jr] - S.x[0]) / rho;
        yr = (S.y[jr] - S.y[0]) / rho;
        zr = (S.z[jr] - S.z[0]) / rho;
    }
    build_border<NB>(S, t, o.degree, o.rank_tol, xr, yr, zr);
    if (t.tid == 0) S.m = n + S.r;
    bsync<NB>();
    int status = RBFFD_ST_OK;
    int evals = 0;
    double a[64];
    double eps;
    if (dupf > 0.0) status = RBFFD_ST_DUPLICATE;

    // ---- shape parameter
    bool have_final = false;  // registers / S hold the tridiagonal form at eps
    double amin_known = 0.0;  // min |lambda| if already found
    Spectrum sp;
    if (o.mode == RBFFD_EPS_FIXED) {
        eps = o.eps_fixed;
    } else if (o.mode == RBFFD_EPS_GIVEN) {
        eps = J.eps_in[s];
    } else {
        bool need_bisect = true;
        if (o.mode == RBFFD_EPS_LEARNED) {
            eps = J.eps_in[s];
            if (isfinite(eps) && eps > 0.0) {
                // max |lambda| to band_rel: also the reported kappa's if kept
                sp = eval_spectrum<K, NB>(a, S, t, eps, 8, o.band_rel);
                ++evals;
                if (sp.finite && sp.amax > 0.0) {
                    int c_lo, c_hi, nu;  // |lambda| below amax/band_lo and below amax/band_hi
                    const double tau_lo = sp.amax / o.band_lo, tau_hi = sp.amax / o.band_hi;
                    double lp, hp, ln_, hn;
                    band_counts_min<NB>(S, t.lane, sp, tau_lo, tau_hi, c_lo, c_hi, nu, lp, hp, ln_, hn);
                    if (c_lo > 0 && c_hi == 0) {  // band_lo < kappa <= band_hi
                        need_bisect = false;
                        have_final = true;
                        // min |lambda| lies in [tau_hi, tau_lo): its first round is done
                        amin_known = min_abs_refine<NB>(S, t.lane, sp, nu, lp, hp, ln_, hn, 6, o.band_rel);
                    }
                }
            }
            if (need_bisect && status == RBFFD_ST_OK) status = RBFFD_ST_FALLBACK;
        }
        if (need_bisect) {
            double lo = o.br_lo / rho, hi = o.br_hi / rho;
            sp = eval_spectrum<K, NB>(a, S, t, lo, 2);
            ++evals;
            bool ab = kappa_above<NB>(S, t.lane, sp, o.kappa_target);
            for (int q = 0; !ab && q < o.max_expand; ++q) {
                lo *= 0.5;
                sp = eval_spectrum<K, NB>(a, S, t, lo, 2);
                ++evals;
                ab = kappa_above<NB>(S, t.lane, sp, o.kappa_target);
            }
            bool ok = ab;
            sp = eval_spectrum<K, NB>(a, S, t, hi, 2);
            ++evals;
            ab = kappa_above<NB>(S, t.lane, sp, o.kappa_target);
            for (int q = 0; ab && q < o.max_expand; ++q) {
                hi *= 2.0;
                sp = eval_spectrum<K, NB>(a, S, t, hi, 2);
                ++evals;
                ab = kappa_above<NB>(S, t.lane, sp, o.kappa_target);
            }
            ok = ok && !ab;
            if (!ok && status == RBFFD_ST_OK) status = RBFFD_ST_NO_BRACKET;
            bool stop = false;
            while (hi - lo > o.eps_tol && !stop) {
                const double mid = 0.5 * (lo + hi);
                sp = eval_spectrum<K, NB>(a, S, t, mid, 2);
                ++evals;
                if (o.band_stop && sp.finite && sp.amax > 0.0) {
                    int c_lo, c_hi;
                    small_counts<NB>(S, t.lane, sp, sp.amax / o.band_lo, sp.amax / o.band_hi, c_lo, c_hi);
                    if (c_lo > 0 && c_hi == 0) {
                        eps = mid;
                        stop = true;
                        have_final = true;
                        // six more rounds: the same brackets as eight from the start,
                        // full precision for the reported kappa
                        spectrum_refine<NB>(S, t.lane, sp, 6);
                        break;
                    }
                }
                if (kappa_above<NB>(S, t.lane, sp, o.kappa_target)) lo = mid;
                else hi = mid;
            }
            if (!stop) eps = 0.5 * (lo + hi);
        }
    }
    if (!have_final) {
        sp = eval_spectrum<K, NB>(a, S, t, eps, 8);
        ++evals;
    }
    // ---- kappa_2 at the final eps
    double kappa = NAN;
    if (sp.finite && sp.amax > 0.0) {
        const double amin = amin_known > 0.0 ? amin_known : spectrum_min_abs<NB>(S, t.lane, sp);
        kappa = sp.amax / amin;
    } else if (status == RBFFD_ST_OK) {
        status = RBFFD_ST_NONFINITE;
    }
    if (!sp.finite && status == RBFFD_ST_OK) status = RBFFD_ST_NONFINITE;
    if (t.tid == 0) {
        if (J.eps) J.eps[s] = eps;
        if (J.kappa) J.kappa[s] = kappa;
        if (J.nevals) J.nevals[s] = evals;
    }
    if (J.kappa_only) {
        if (t.tid == 0 && J.status) J.status[s] = status;
        bsync<NB>();
        return;
    }

    // ---- weights: w = (A~^{-1} r)[:n], r = sum_d (B^d)^T g_d, g_d = (A~^{-1} b_d)[:n]
    if (t.tid == 0) S.fact_ok = sp.finite ? (int)tri_factor<NB>(S) : 0;
    bsync<NB>();
    const int m = S.m;
    if (!S.fact_ok) {
        if (status == RBFFD_ST_OK) status = sp.finite ? RBFFD_ST_SINGULAR : RBFFD_ST_NONFINITE;
        if (t.tid == 0 && J.status) J.status[s] = status;
        if (c < n && t.rb == 0) J.w[s * n + c] = NAN;
        bsync<NB>();
        return;
    }
    const double e2 = eps * eps;
    const double n0x = S.nrm0[0], n0y = S.nrm0[1], n0z = S.nrm0[2];
    // b_d (row 1 of B^d) as an m-vector, component c
    double b[3] = {0.0, 0.0, 0.0};
    if (c < n) {
        const double dx = S.x[0] - px, dy = S.y[0] - py, dz = S.z[0] - pz;  // x_1 - x_j
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        const double ps = rbf_psi<K>(e2, r2);
        const double dn = n0x * dx + n0y * dy + n0z * dz;
        b[0] = ps * (dx - n0x * dn);
        b[1] = ps * (dy - n0y * dn);
        b[2] = ps * (dz - n0z * dn);
    } else if (c < m && o.degree > 0) {
        const int k = c - n;  // grad q_k at the centre (xi = 0): linear coefficients / rho
        const double gx = S.T[1 * RMAX + k] * irho, gy = S.T[2 * RMAX + k] * irho, gz = S.T[3 * RMAX + k] * irho;
        const double dn = n0x * gx + n0y * gy + n0z * gz;
        b[0] = gx - n0x * dn;
        b[1] = gy - n0y * dn;
        b[2] = gz - n0z * dn;
    }
    if constexpr (NB == 1) reflector_gram<NB>(a, S, t);
    // g_d: plain solve.  Refining this solve as well as the final one does not
    // lower the error of w (measured against 60-digit weights: both ways
    // 0.02-0.07 kappa u at kappa_T = 1e10 and 1e12; without any refinement
    // 0.1-0.28 kappa u), so only the final solve is refined.
    solve<NB, 3>(a, S, t, b);
    // h_i = Pi_i g_i
    double hx = 0, hy = 0, hz = 0;
    if (c < n) {
        const double dn = nx * b[0] + ny * b[1] + nz * b[2];
        hx = b[0] - nx * dn;
        hy = b[1] - ny * dn;
        hz = b[2] - nz * dn;
    }
    if (t.rb == 0) {
        S.hx[c] = hx;
        S.hy[c] = hy;
        S.hz[c] = hz;
    }
    bsync<NB>();
    // r_j = sum_i psi(r_ij) (x_i - x_j) . h_i   (j = c < n)
    double rj = 0.0;
    if (c < n) {
#pragma unroll 4
        for (int i = 0; i < n; ++i) {
            const double dx = S.x[i] - px, dy = S.y[i] - py, dz = S.z[i] - pz;
            const double r2 = (dx * dx + dy * dy) + dz * dz;
            const double ps = rbf_psi<K>(e2, r2);
            rj = fma(ps, dx * S.hx[i] + dy * S.hy[i] + dz * S.hz[i], rj);
        }
    }
    // r_{n+k} = sum_i grad q_k(x_i) . h_i
    if (o.degree > 0) {
        const int r = S.r;
        for (int k = 0; k < r; ++k) {
            double cv = 0.0;
            if (c < n) {
                const double* T = S.T;
                double gx = T[1 * RMAX + k], gy = T[2 * RMAX + k], gz = T[3 * RMAX + k];
                if (o.degree == 2) {
                    const double t4 = T[4 * RMAX + k], t5 = T[5 * RMAX + k], t6 = T[6 * RMAX + k];
                    const double t7 = T[7 * RMAX + k], t8 = T[8 * RMAX + k], t9 = T[9 * RMAX + k];
                    gx += 2.0 * t4 * xi + t7 * yi + t8 * zi;
                    gy += 2.0 * t5 * yi + t7 * xi + t9 * zi;
                    gz += 2.0 * t6 * zi + t8 * xi + t9 * yi;
                }
                cv = (gx * hx + gy * hy + gz * hz) * irho;
            }
            cv = sum_cols<NB>(cv, S, t);
            if (c == n + k) rj = cv;
        }
    }
    double wv[3] = {rj, 0.0, 0.0};
    solve_refined<K, NB, 1>(a, S, t, e2, wv);
    if (c < n && t.rb == 0) J.w[s * n + c] = wv[0];
    if (t.tid == 0 && J.status) J.status[s] = status;
    bsync<NB>();
}

}  // namespace rbw
