// Extended-precision (double-double) RBF-FD weights for target condition
// numbers beyond what FP64 resolves (Sec. 6.2 computes the weights for
// kappa_T up to 1e20 in quadruple precision and then steps in FP64).
//
// Same quantities as the FP64 path (Sec. 4, eq. surface_lap_P1: the first
// row of L_P = sum_d G^d G^d, formed as w = (A~^{-1} r)[:n] with
// r = sum_d (B^d)^T g_d, g_d = (A~^{-1} b_d)[:n]; Sec. 5: eps by bisection on
// kappa_2(A~) = max|lambda| / min|lambda|), for the paper's own local system:
// the constant border (a column of ones) and the multiquadric or inverse
// multiquadric kernel, with every quantity derived from the FP64 inputs
// carried as an unevaluated sum of two doubles (about 32 significant digits):
// coordinate differences (exact two-sums), squared distances, kernel values,
// unit normals, the Householder tridiagonalisation and Sturm counts behind
// kappa_2, and a pivoted LU factorisation for the solves.  Only the final
// weights, eps and kappa_2 are rounded to FP64.
//
// One wavefront per stencil; the local matrix (m = n + 1 <= 48) lives in LDS,
// lane j owning column j.  This path trades speed for precision: it exists
// for the high targets of the convergence studies, not for the point-cloud
// workloads.
#include "common.h"
#include "weights_job.h"

#include <cmath>

#pragma clang fp contract(off)

namespace {

constexpr int DD_MAX = 48;
constexpr int LDA = DD_MAX + 1;

// ------------------------------------------------------ double-double ----
// Unevaluated sums hi + lo with |lo| <= ulp(hi) / 2: the error-free sum of
// two doubles (Knuth's two-sum), the error-free product through FMA, and
// the usual compensated add / multiply / divide / square root built on them.
struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd mk(double a) { return {a, 0.0}; }
__device__ __forceinline__ dd quick_two_sum(double a, double b) {
    const double s = a + b;
    return {s, b - (s - a)};
}
__device__ __forceinline__ dd two_sum(double a, double b) {
    const double s = a + b;
    const double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ dd two_prod(double a, double b) {
    const double p = a * b;
    return {p, __builtin_fma(a, b, -p)};
}
__device__ __forceinline__ dd add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    const dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd neg(dd a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ dd sub(dd a, dd b) { return add(a, neg(b)); }
__device__ __forceinline__ dd mul(dd a, dd b) {
    dd p = two_prod(a.hi, b.hi);
    const double c = a.hi * b.lo;
    const double d = a.lo * b.hi;
    p.lo += c + d;
    return quick_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd mul_d(dd a, double b) {
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return quick_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd dvd(dd a, dd b) {
    const double q1 = a.hi / b.hi;
    dd r = sub(a, mul_d(b, q1));
    const double q2 = r.hi / b.hi;
    r = sub(r, mul_d(b, q2));
    const double q3 = r.hi / b.hi;
    return add(quick_two_sum(q1, q2), mk(q3));
}
__device__ __forceinline__ dd dsqrt(dd a) {
    if (!(a.hi > 0.0)) return mk(a.hi == 0.0 ? 0.0 : NAN);
    const double x = 1.0 / sqrt(a.hi);
    const double ax = a.hi * x;
    const dd e = sub(a, two_prod(ax, ax));
    return two_sum(ax, e.hi * (x * 0.5));
}
__device__ __forceinline__ double to_d(dd a) { return a.hi + a.lo; }
__device__ __forceinline__ bool is_fin(dd a) { return isfinite(a.hi) && isfinite(a.lo); }

__device__ __forceinline__ dd shfl_xor(dd v, int o) { return {__shfl_xor(v.hi, o, 64), __shfl_xor(v.lo, o, 64)}; }
// Sum over the wavefront, the same value in every lane (same association everywhere).
__device__ __forceinline__ dd wsum(dd v) {
    for (int o = 1; o < 64; o <<= 1) {
        const dd u = shfl_xor(v, o);
        // order the operands by lane so that both partners add alike
        v = (threadIdx.x & o) ? add(u, v) : add(v, u);
    }
    return v;
}

__device__ __forceinline__ void fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct DDShared {
    double x[DD_MAX], y[DD_MAX], z[DD_MAX];
    double nh[3][DD_MAX], nl[3][DD_MAX];  // unit normals
    double ah[DD_MAX * LDA], al[DD_MAX * LDA];
    double dh[DD_MAX], dl[DD_MAX], eh[DD_MAX], el[DD_MAX], e2h[DD_MAX], e2l[DD_MAX];
    double vh[DD_MAX], vl[DD_MAX], wh[DD_MAX], wl[DD_MAX];
    double bh[4][DD_MAX], bl[4][DD_MAX];
    int piv[DD_MAX];
};

__device__ __forceinline__ dd ld(const double* h, const double* l, int i) { return {h[i], l[i]}; }
__device__ __forceinline__ void st(double* h, double* l, int i, dd v) {
    h[i] = v.hi;
    l[i] = v.lo;
}
__device__ __forceinline__ dd A(const DDShared& S, int r, int c) { return {S.ah[r * LDA + c], S.al[r * LDA + c]}; }
__device__ __forceinline__ void setA(DDShared& S, int r, int c, dd v) {
    S.ah[r * LDA + c] = v.hi;
    S.al[r * LDA + c] = v.lo;
}

// x_i - x_j as an exact double-double, squared distance
__device__ __forceinline__ void diff3(const DDShared& S, int i, int j, dd (&d)[3]) {
    d[0] = two_sum(S.x[i], -S.x[j]);
    d[1] = two_sum(S.y[i], -S.y[j]);
    d[2] = two_sum(S.z[i], -S.z[j]);
}
__device__ __forceinline__ dd norm2(const dd (&d)[3]) { return add(add(mul(d[0], d[0]), mul(d[1], d[1])), mul(d[2], d[2])); }

// phi and psi = phi'(r)/r from the squared distance (MQ: kernel 0, IMQ: 1)
template <int K>
__device__ __forceinline__ dd phi(dd e2, dd r2) {
    const dd t = add(mk(1.0), mul(e2, r2));
    const dd s = dsqrt(t);
    return K == RBFFD_KERNEL_MQ ? s : dvd(mk(1.0), s);
}
template <int K>
__device__ __forceinline__ dd psi(dd e2, dd r2) {
    const dd t = add(mk(1.0), mul(e2, r2));
    const dd s = dsqrt(t);
    return K == RBFFD_KERNEL_MQ ? dvd(e2, s) : neg(dvd(e2, mul(s, t)));
}

// A~ = [[A, 1], [1^T, 0]] at eps (lane j fills column j)
template <int K>
__device__ void build_dd(DDShared& S, int n, int m, double eps, int j) {
    const dd e2 = two_prod(eps, eps);
    if (j < m) {
        for (int r = 0; r < m; ++r) {
            dd v = mk(0.0);
            if (r < n && j < n) {
                dd d[3];
                diff3(S, r, j, d);
                v = phi<K>(e2, norm2(d));
            } else if (r < n || j < n) {
                v = mk(1.0);
            }
            setA(S, r, j, v);
        }
    }
    fence();
}

// Householder tridiagonalisation of A~ (symmetric, full storage in LDS):
// S.d, S.e (and e^2) hold T.
__device__ void tridiag_dd(DDShared& S, int m, int j) {
    for (int k = 0; k < m - 2; ++k) {
        const dd xr = (j > k + 1 && j < m) ? A(S, j, k) : mk(0.0);
        const dd alpha = A(S, k + 1, k);
        const dd xn2 = wsum(mul(xr, xr));
        dd beta = alpha, tau = mk(0.0), scal = mk(0.0);
        if (xn2.hi > 0.0) {
            const dd nrm = dsqrt(add(mul(alpha, alpha), xn2));
            beta = alpha.hi >= 0.0 ? neg(nrm) : nrm;
            tau = dvd(sub(beta, alpha), beta);
            scal = dvd(mk(1.0), sub(alpha, beta));
        }
        const dd vj = (j == k + 1) ? mk(1.0) : ((j > k + 1 && j < m) ? mul(xr, scal) : mk(0.0));
        if (j == 0) {
            st(S.dh, S.dl, k, A(S, k, k));
            st(S.eh, S.el, k, beta);
        }
        if (j < DD_MAX) st(S.vh, S.vl, j, vj);
        fence();
        // w = tau A v - (tau^2 / 2) (v^T A v) v over the trailing block
        dd p = mk(0.0);
        if (j > k && j < m)
            for (int r = k + 1; r < m; ++r) p = add(p, mul(A(S, r, j), ld(S.vh, S.vl, r)));
        dd wj = (j > k && j < m) ? mul(tau, p) : mk(0.0);
        const dd s = wsum(mul(wj, vj));
        wj = sub(wj, mul(mul_d(mul(tau, s), 0.5), vj));
        if (j < DD_MAX) st(S.wh, S.wl, j, wj);
        fence();
        if (j > k && j < m)
            for (int r = k + 1; r < m; ++r) {
                const dd vr = ld(S.vh, S.vl, r), wr = ld(S.wh, S.wl, r);
                setA(S, r, j, sub(sub(A(S, r, j), mul(vr, wj)), mul(wr, vj)));
            }
        fence();
    }
    if (j == 0) {
        if (m >= 2) {
            st(S.dh, S.dl, m - 2, A(S, m - 2, m - 2));
            st(S.eh, S.el, m - 2, A(S, m - 1, m - 2));
        }
        st(S.dh, S.dl, m - 1, A(S, m - 1, m - 1));
    }
    fence();
    if (j < m - 1) {
        const dd e = ld(S.eh, S.el, j);
        st(S.e2h, S.e2l, j, mul(e, e));
    }
    fence();
}

// #eigenvalues of T below sigma (double-double recurrence, FP64 shift)
__device__ int sturm_dd(const DDShared& S, int m, double sigma, double pivmin) {
    dd q = sub(ld(S.dh, S.dl, 0), mk(sigma));
    if (fabs(q.hi) < pivmin) q = mk(-pivmin);
    int c = q.hi < 0.0 ? 1 : 0;
    for (int i = 1; i < m; ++i) {
        q = sub(sub(ld(S.dh, S.dl, i), mk(sigma)), dvd(ld(S.e2h, S.e2l, i - 1), q));
        if (fabs(q.hi) < pivmin) q = mk(-pivmin);
        c += q.hi < 0.0 ? 1 : 0;
    }
    return c;
}

struct SpecDD {
    double lo1, hi1, lo2, hi2, amax, pivmin;
    bool finite;
};

// brackets of lambda_1 (lanes 0..31) and lambda_m (lanes 32..63), 33-way
// multisection until they are a few ulps wide
__device__ SpecDD spectrum_dd(const DDShared& S, int m, int lane) {
    SpecDD sp;
    double gl = INFINITY, gu = -INFINITY, emax2 = 0.0;
    bool fin = true;
    for (int i = 0; i < m; ++i) {
        const double off = (i > 0 ? fabs(S.eh[i - 1]) : 0.0) + (i < m - 1 ? fabs(S.eh[i]) : 0.0);
        gl = fmin(gl, S.dh[i] - off);
        gu = fmax(gu, S.dh[i] + off);
        if (i < m - 1) emax2 = fmax(emax2, S.e2h[i]);
        fin = fin && isfinite(S.dh[i]) && (i == m - 1 || isfinite(S.eh[i]));
    }
    sp.finite = fin;
    sp.pivmin = 1e-290 * fmax(1.0, emax2);
    const double w = gu - gl;
    gl -= 4.0 * w * 2.3e-16 + 2.0 * sp.pivmin;
    gu += 4.0 * w * 2.3e-16 + 2.0 * sp.pivmin;
    double lo1 = gl, hi1 = gu, lo2 = gl, hi2 = gu;
    const int g = lane >> 5, tt = lane & 31;
    for (int rd = 0; fin && rd < 14; ++rd) {
        if (hi1 - lo1 <= 4e-16 * fmax(fabs(lo1), fabs(hi1)) && hi2 - lo2 <= 4e-16 * fmax(fabs(lo2), fabs(hi2))) break;
        const double lo = g ? lo2 : lo1, hi = g ? hi2 : hi1;
        const double sig = lo + (hi - lo) * (double)(tt + 1) / 33.0;
        const bool below = sturm_dd(S, m, sig, sp.pivmin) < (g ? m : 1);
        const uint64_t bal = __ballot(below);
        const int nb1 = __popcll(bal & 0xffffffffull), nb2 = __popcll(bal >> 32);
        const double a1 = nb1 > 0 ? lo1 + (hi1 - lo1) * (double)nb1 / 33.0 : lo1;
        const double b1 = nb1 < 32 ? lo1 + (hi1 - lo1) * (double)(nb1 + 1) / 33.0 : hi1;
        const double a2 = nb2 > 0 ? lo2 + (hi2 - lo2) * (double)nb2 / 33.0 : lo2;
        const double b2 = nb2 < 32 ? lo2 + (hi2 - lo2) * (double)(nb2 + 1) / 33.0 : hi2;
        lo1 = a1; hi1 = b1; lo2 = a2; hi2 = b2;
    }
    sp.lo1 = lo1; sp.hi1 = hi1; sp.lo2 = lo2; sp.hi2 = hi2;
    sp.amax = fmax(fabs(0.5 * (lo1 + hi1)), fabs(0.5 * (lo2 + hi2)));
    return sp;
}

// #|lambda| < tau (lanes 0..1)
__device__ int count_small(const DDShared& S, int m, const SpecDD& sp, double tau, int lane) {
    const int c = lane < 2 ? sturm_dd(S, m, lane == 0 ? -tau : tau, sp.pivmin) : 0;
    return __shfl(c, 1, 64) - __shfl(c, 0, 64);
}

// kappa_2 > target, decided from the Sturm counts at max|lambda| / target
__device__ bool above_dd(const DDShared& S, int m, const SpecDD& sp, double target, int lane) {
    if (!sp.finite || !(sp.amax > 0.0)) return true;
    const double alo = fmax(-sp.hi1, sp.lo2), ahi = fmax(-sp.lo1, sp.hi2);
    if (count_small(S, m, sp, alo / target, lane) > 0) return true;
    if (count_small(S, m, sp, ahi / target, lane) == 0) return false;
    return count_small(S, m, sp, sp.amax / target, lane) > 0;
}

// smallest |lambda| by geometric multisection on both sides of zero
__device__ double min_abs_dd(const DDShared& S, int m, const SpecDD& sp, int lane) {
    const int nu = sturm_dd(S, m, 0.0, sp.pivmin);
    const double L = sp.amax * 1e-40 + sp.pivmin, H = sp.amax * (1.0 + 1e-14);
    double lp = log(L), hp = log(H), ln_ = log(L), hn = log(H);
    const int g = lane >> 5, tt = lane & 31;
    for (int rd = 0; rd < 16 && fmax(hp - lp, hn - ln_) > 1e-14; ++rd) {
        const double lo = g ? ln_ : lp, hi = g ? hn : hp;
        const double sig = exp(lo + (hi - lo) * (double)(tt + 1) / 33.0);
        const bool above = g == 0 ? sturm_dd(S, m, sig, sp.pivmin) <= nu : sturm_dd(S, m, -sig, sp.pivmin) >= nu;
        const uint64_t bal = __ballot(above);
        const int nb1 = __popcll(bal & 0xffffffffull), nb2 = __popcll(bal >> 32);
        const double a1 = lp + (hp - lp) * (double)nb1 / 33.0, b1 = lp + (hp - lp) * (double)(nb1 + 1) / 33.0;
        const double a2 = ln_ + (hn - ln_) * (double)nb2 / 33.0, b2 = ln_ + (hn - ln_) * (double)(nb2 + 1) / 33.0;
        if (nb1 > 0) lp = a1;
        if (nb1 < 32) hp = b1;
        if (nb2 > 0) ln_ = a2;
        if (nb2 < 32) hn = b2;
    }
    const double pos = nu < m ? exp(0.5 * (lp + hp)) : INFINITY;
    const double ng = nu > 0 ? exp(0.5 * (ln_ + hn)) : INFINITY;
    return fmin(pos, ng);
}

template <int K>
__device__ SpecDD eval_dd(DDShared& S, int n, int m, double eps, int lane) {
    build_dd<K>(S, n, m, eps, lane);
    tridiag_dd(S, m, lane);
    return spectrum_dd(S, m, lane);
}

// LU with partial pivoting of A~ in place; false on a zero pivot
__device__ bool lu_dd(DDShared& S, int m, int lane) {
    for (int k = 0; k < m; ++k) {
        const double v = (lane >= k && lane < m) ? fabs(S.ah[lane * LDA + k]) : -1.0;
        double mx = v;
        for (int o = 1; o < 64; o <<= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
        const uint64_t hit = __ballot(v == mx && v >= 0.0);
        const int p = hit ? __ffsll((long long)hit) - 1 : k;
        if (!(mx > 0.0)) return false;
        if (lane == 0) S.piv[k] = p;
        if (p != k && lane < m) {
            const dd a = A(S, k, lane), b = A(S, p, lane);
            setA(S, k, lane, b);
            setA(S, p, lane, a);
        }
        fence();
        const dd piv = A(S, k, k);
        if (lane > k && lane < m) setA(S, lane, k, dvd(A(S, lane, k), piv));
        fence();
        if (lane > k && lane < m) {
            const dd ukj = A(S, k, lane);
            for (int r = k + 1; r < m; ++r) setA(S, r, lane, sub(A(S, r, lane), mul(A(S, r, k), ukj)));
        }
        fence();
    }
    return true;
}

// b_v <- A~^{-1} b_v for the first nb right-hand sides in S.bh/bl
__device__ void lu_solve_dd(DDShared& S, int m, int nb, int lane) {
    if (lane < nb)
        for (int k = 0; k < m; ++k) {
            const int p = S.piv[k];
            if (p != k) {
                const dd a = ld(S.bh[lane], S.bl[lane], k), b = ld(S.bh[lane], S.bl[lane], p);
                st(S.bh[lane], S.bl[lane], k, b);
                st(S.bh[lane], S.bl[lane], p, a);
            }
        }
    fence();
    for (int k = 0; k < m; ++k) {  // L (unit diagonal)
        if (lane > k && lane < m)
            for (int v = 0; v < nb; ++v)
                st(S.bh[v], S.bl[v], lane, sub(ld(S.bh[v], S.bl[v], lane), mul(A(S, lane, k), ld(S.bh[v], S.bl[v], k))));
        fence();
    }
    for (int k = m - 1; k >= 0; --k) {  // U
        if (lane == k)
            for (int v = 0; v < nb; ++v) st(S.bh[v], S.bl[v], k, dvd(ld(S.bh[v], S.bl[v], k), A(S, k, k)));
        fence();
        if (lane < k)
            for (int v = 0; v < nb; ++v)
                st(S.bh[v], S.bl[v], lane, sub(ld(S.bh[v], S.bl[v], lane), mul(A(S, lane, k), ld(S.bh[v], S.bl[v], k))));
        fence();
    }
}

template <int K>
__global__ __launch_bounds__(64) void k_weights_dd(rbw::Job J) {
    __shared__ DDShared S;
    const int64_t s = blockIdx.x;
    if (s >= J.N) return;
    const rbw::WOpts& o = J.o;
    const int n = o.n, m = n + 1, lane = threadIdx.x;
    // gather: coordinates, unit normals in double-double
    bool bad = false, badn = false;
    if (lane < n) {
        int64_t node = J.idx[s * n + lane];
        bad = node < 0 || node >= J.N;
        if (bad) node = 0;
        S.x[lane] = J.xyz[3 * node];
        S.y[lane] = J.xyz[3 * node + 1];
        S.z[lane] = J.xyz[3 * node + 2];
        const dd nx = mk(J.nrm[3 * node]), ny = mk(J.nrm[3 * node + 1]), nz = mk(J.nrm[3 * node + 2]);
        const dd nn = dsqrt(add(add(mul(nx, nx), mul(ny, ny)), mul(nz, nz)));
        badn = !(nn.hi > 0.0 && isfinite(nn.hi));
        const dd inv = badn ? mk(0.0) : dvd(mk(1.0), nn);
        st(S.nh[0], S.nl[0], lane, mul(nx, inv));
        st(S.nh[1], S.nl[1], lane, mul(ny, inv));
        st(S.nh[2], S.nl[2], lane, mul(nz, inv));
    }
    fence();
    bool dup = false;
    double r20 = 0.0;
    if (lane < n) {
        dd d[3];
        diff3(S, lane, 0, d);
        const dd r2 = norm2(d);
        r20 = r2.hi;
        dup = lane > 0 && r2.hi == 0.0;
    }
    if (__ballot(bad) || __ballot(badn)) {
        if (lane == 0) {
            if (J.eps) J.eps[s] = NAN;
            if (J.kappa) J.kappa[s] = NAN;
            if (J.nevals) J.nevals[s] = 0;
            if (J.status) J.status[s] = __ballot(bad) ? RBFFD_ST_BAD_INDEX : RBFFD_ST_BAD_NORMAL;
        }
        if (lane < n) J.w[s * n + lane] = NAN;
        return;
    }
    int status = __ballot(dup) ? RBFFD_ST_DUPLICATE : RBFFD_ST_OK;
    double rmax = r20;
    for (int o2 = 1; o2 < 64; o2 <<= 1) rmax = fmax(rmax, __shfl_xor(rmax, o2, 64));
    const double rho = sqrt(rmax);
    int evals = 0;
    double eps;
    SpecDD sp;
    if (o.mode == RBFFD_EPS_FIXED) {
        eps = o.eps_fixed;
    } else if (o.mode == RBFFD_EPS_GIVEN) {
        eps = J.eps_in[s];
    } else {
        double lo = o.br_lo / rho, hi = o.br_hi / rho;
        sp = eval_dd<K>(S, n, m, lo, lane);
        ++evals;
        bool ab = above_dd(S, m, sp, o.kappa_target, lane);
        for (int q = 0; !ab && q < o.max_expand; ++q) {
            lo *= 0.5;
            sp = eval_dd<K>(S, n, m, lo, lane);
            ++evals;
            ab = above_dd(S, m, sp, o.kappa_target, lane);
        }
        bool ok = ab;
        sp = eval_dd<K>(S, n, m, hi, lane);
        ++evals;
        ab = above_dd(S, m, sp, o.kappa_target, lane);
        for (int q = 0; ab && q < o.max_expand; ++q) {
            hi *= 2.0;
            sp = eval_dd<K>(S, n, m, hi, lane);
            ++evals;
            ab = above_dd(S, m, sp, o.kappa_target, lane);
        }
        ok = ok && !ab;
        if (!ok && status == RBFFD_ST_OK) status = RBFFD_ST_NO_BRACKET;
        while (hi - lo > o.eps_tol) {
            const double mid = 0.5 * (lo + hi);
            sp = eval_dd<K>(S, n, m, mid, lane);
            ++evals;
            if (above_dd(S, m, sp, o.kappa_target, lane)) lo = mid;
            else hi = mid;
        }
        eps = 0.5 * (lo + hi);
    }
    sp = eval_dd<K>(S, n, m, eps, lane);
    ++evals;
    double kappa = NAN;
    if (sp.finite && sp.amax > 0.0) kappa = sp.amax / min_abs_dd(S, m, sp, lane);
    else if (status == RBFFD_ST_OK) status = RBFFD_ST_NONFINITE;
    if (lane == 0) {
        if (J.eps) J.eps[s] = eps;
        if (J.kappa) J.kappa[s] = kappa;
        if (J.nevals) J.nevals[s] = evals;
    }
    // weights: LU of A~(eps), g_d = (A~^{-1} b_d)[:n], r = sum_d (B^d)^T g_d, w = (A~^{-1} r)[:n]
    build_dd<K>(S, n, m, eps, lane);
    const dd e2 = two_prod(eps, eps);
    const dd n0[3] = {ld(S.nh[0], S.nl[0], 0), ld(S.nh[1], S.nl[1], 0), ld(S.nh[2], S.nl[2], 0)};
    if (lane < m) {
        dd b[3] = {mk(0.0), mk(0.0), mk(0.0)};
        if (lane < n) {  // row 1 of B^d: psi(r_1j) [Pi_1 (x_1 - x_j)]_d; the ones border has zero gradient
            dd d[3];
            diff3(S, 0, lane, d);
            const dd ps = psi<K>(e2, norm2(d));
            const dd dn = add(add(mul(n0[0], d[0]), mul(n0[1], d[1])), mul(n0[2], d[2]));
            for (int c = 0; c < 3; ++c) b[c] = mul(ps, sub(d[c], mul(n0[c], dn)));
        }
        for (int c = 0; c < 3; ++c) st(S.bh[c], S.bl[c], lane, b[c]);
    }
    fence();
    if (!lu_dd(S, m, lane)) {
        if (status == RBFFD_ST_OK) status = RBFFD_ST_SINGULAR;
        if (lane == 0 && J.status) J.status[s] = status;
        if (lane < n) J.w[s * n + lane] = NAN;
        return;
    }
    lu_solve_dd(S, m, 3, lane);
    // h_i = Pi_i g_i, kept in S.v/S.w/S.d (free now) as three vectors
    if (lane < n) {
        dd g[3] = {ld(S.bh[0], S.bl[0], lane), ld(S.bh[1], S.bl[1], lane), ld(S.bh[2], S.bl[2], lane)};
        const dd nu[3] = {ld(S.nh[0], S.nl[0], lane), ld(S.nh[1], S.nl[1], lane), ld(S.nh[2], S.nl[2], lane)};
        const dd dn = add(add(mul(nu[0], g[0]), mul(nu[1], g[1])), mul(nu[2], g[2]));
        st(S.vh, S.vl, lane, sub(g[0], mul(nu[0], dn)));
        st(S.wh, S.wl, lane, sub(g[1], mul(nu[1], dn)));
        st(S.dh, S.dl, lane, sub(g[2], mul(nu[2], dn)));
    }
    fence();
    // r_j = sum_i psi(r_ij) (x_i - x_j) . h_i, r_n = 0
    if (lane < m) {
        dd rj = mk(0.0);
        if (lane < n)
            for (int i = 0; i < n; ++i) {
                dd d[3];
                diff3(S, i, lane, d);
                const dd ps = psi<K>(e2, norm2(d));
                const dd dot = add(add(mul(d[0], ld(S.vh, S.vl, i)), mul(d[1], ld(S.wh, S.wl, i))),
                                   mul(d[2], ld(S.dh, S.dl, i)));
                rj = add(rj, mul(ps, dot));
            }
        st(S.bh[3], S.bl[3], lane, rj);
    }
    fence();
    // the solve for w reads slot 3 only: move it to slot 0
    if (lane < m) st(S.bh[0], S.bl[0], lane, ld(S.bh[3], S.bl[3], lane));
    fence();
    lu_solve_dd(S, m, 1, lane);
    if (lane < n) J.w[s * n + lane] = to_d(ld(S.bh[0], S.bl[0], lane));
    if (lane == 0 && J.status) J.status[s] = status;
}

}  // namespace

int weights_check_opts(rbffd_ctx ctx, int64_t N, const rbffd_weight_opts* opts, rbw::WOpts& o);

extern "C" int rbffd_build_weights_dd(rbffd_ctx ctx, int64_t N, const double* xyz, const double* nrm,
                                      const rbffd_weight_opts* opts, const int32_t* idx_in, const double* eps_in,
                                      int32_t* idx_out, double* w, double* eps, double* kappa, int32_t* status,
                                      int32_t* nevals) {
    if (!ctx) return RBFFD_E_ARG;
    rbw::Job J;
    int rc = weights_check_opts(ctx, N, opts, J.o);
    if (rc) return rc;
    if (J.o.kernel != RBFFD_KERNEL_MQ && J.o.kernel != RBFFD_KERNEL_IMQ)
        return set_error(ctx, RBFFD_E_UNSUPPORTED, "extended-precision weights: MQ or IMQ kernel only");
    if (J.o.degree != 0)
        return set_error(ctx, RBFFD_E_UNSUPPORTED, "extended-precision weights: constant border (degree 0) only");
    if (J.o.n + 1 > DD_MAX)
        return set_error(ctx, RBFFD_E_UNSUPPORTED, "extended-precision weights: n + 1 = %d exceeds %d", J.o.n + 1,
                         DD_MAX);
    if (J.o.mode == RBFFD_EPS_LEARNED)
        return set_error(ctx, RBFFD_E_UNSUPPORTED, "extended-precision weights: fixed, given or bisection eps only");
    if (N == 0) return RBFFD_OK;
    if (!xyz || !nrm || !w) return set_error(ctx, RBFFD_E_ARG, "null pointer");
    if (J.o.mode == RBFFD_EPS_GIVEN && !eps_in) return set_error(ctx, RBFFD_E_ARG, "eps_in required for this eps_mode");
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
    const dim3 g((unsigned)N), b(64);
    if (J.o.kernel == RBFFD_KERNEL_MQ) hipLaunchKernelGGL(k_weights_dd<RBFFD_KERNEL_MQ>, g, b, 0, ctx->stream, J);
    else hipLaunchKernelGGL(k_weights_dd<RBFFD_KERNEL_IMQ>, g, b, 0, ctx->stream, J);
    HIP_TRY(ctx, hipGetLastError());
    return RBFFD_OK;
}
