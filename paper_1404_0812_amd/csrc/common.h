// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "rbffd.h"

struct rbffd_ctx_s {
    hipStream_t stream = nullptr;
    int device = 0;
    char err[512] = {0};
    // growable scratch owned by the context
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
};

struct rbffd_op_s {
    rbffd_ctx ctx = nullptr;
    int64_t N = 0;
    int32_t n = 0;
    int32_t* ell_idx = nullptr;   // (n-1) x N slot-major, internal order, off-diagonal slots
    float* ell_w32 = nullptr;     // (n-1) x N FP32 off-diagonal weights
    double* ell_w64 = nullptr;    // n x N slot-major FP64 weights (slot 0 = centre)
    int32_t* ell_idx64 = nullptr; // n x N slot-major, slot 0 = centre (internal order)
    int32_t* perm = nullptr;      // internal position -> caller index
    // state workspace (internal order), allocated on first step
    void* work = nullptr;
    size_t work_bytes = 0;
    // captured graph cache
    hipGraphExec_t graph = nullptr;
    int graph_key_species = -1, graph_key_prec = -1, graph_key_react = -1, graph_key_steps = -1;
    double graph_key_dt = 0.0;
    double graph_key_D[2] = {0, 0};
    double graph_key_params[5] = {0, 0, 0, 0, 0};
};

int set_error(rbffd_ctx ctx, int code, const char* fmt, ...);
// Ensure ctx->scratch holds at least `bytes`; returns 0 or an error code.
int ensure_scratch(rbffd_ctx ctx, size_t bytes);

#define HIP_TRY(ctx, call)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return set_error((ctx), RBFFD_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Internal entry points of the translation units.
int knn_internal(rbffd_ctx ctx, int64_t N, const double* xyz, int32_t n, int32_t* idx,
                 int32_t* perm);
