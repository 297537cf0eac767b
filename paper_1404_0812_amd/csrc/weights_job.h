// Plain-data description of one weights job (host and device).
#pragma once

#include <cstdint>

#define RBW_RMAX 10

namespace rbw {

struct WOpts {
    int n, kernel, degree, mode;
    double eps_fixed, kappa_target, eps_tol, br_lo, br_hi, band_lo, band_hi, rank_tol;
    int band_stop, max_expand;
    double band_rel;  // multisection precision of a kappa found inside the band
};

// One stencil set: inputs, options and outputs (device pointers).
struct Job {
    WOpts o;
    int64_t N;
    const double* xyz;
    const double* nrm;
    const int32_t* idx;
    const double* eps_in;
    double* w;
    double* eps;
    double* kappa;
    int32_t* status;
    int32_t* nevals;
    int kappa_only;
};

inline int border_cols(int degree) { return degree == 0 ? 1 : (degree == 1 ? 4 : 10); }

}  // namespace rbw
