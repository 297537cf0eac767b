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
    // work list of the batched weights launch (kept apart from scratch, which kNN uses)
    void* batch = nullptr;
    size_t batch_bytes = 0;
};

// One slice of the operator: 64 consecutive internal rows of one surface.
struct OpSlice {
    int64_t off32;  // element offset of the slice in the off-diagonal arrays (n - 1 slots)
    int32_t n;      // stencil size of the slice's rows
    int32_t rows;   // rows in use (64 except at a surface's end)
    int32_t halo;   // distinct neighbour rows of the slice (<= OP_HALO_MAX), -1: too many
    int32_t pad;
};

// Largest slice neighbourhood staged in LDS by the stage kernels.
constexpr int OP_HALO_MAX = 640;

struct rbffd_op_s {
    rbffd_ctx ctx = nullptr;
    int64_t N = 0;        // rows in caller order (sum over surfaces)
    int64_t P = 0;        // internal rows, each surface padded to a multiple of 64
    int32_t n = 0;        // largest stencil size
    int32_t nsurf = 0;
    int64_t nslices = 0;
    OpSlice* slices = nullptr;    // device, nslices
    double* wd64 = nullptr;       // FP64 diagonal weight of every internal row (P)
    int32_t* idx32 = nullptr;     // off-diagonal slots 1..n-1 of row (slice, r) at off32 + slot_pos(k-1, n-1, r)
    double* w64 = nullptr;        // FP64 weights of those slots
    float* w32 = nullptr;         // FP32 weights of those slots (difference form)
    uint16_t* lidx = nullptr;     // slot entries as positions in the slice's halo list
    int32_t* halo = nullptr;      // OP_HALO_MAX sorted distinct neighbour rows per slice
    int32_t* perm = nullptr;      // internal row -> caller row (-1 for padding), P entries
    // state workspace (internal order), allocated on first step
    void* work = nullptr;
    size_t work_bytes = 0;
    // vectors of the implicit (BDF) stepper, allocated on first use
    void* impl = nullptr;
    size_t impl_bytes = 0;
    // captured graph cache
    hipGraphExec_t graph = nullptr;
    // graph of KRYLOV_BATCH implicit-solver iterations, valid while its
    // vectors sit where they were when it was captured (kgraph_key)
    hipGraphExec_t kgraph = nullptr;
    const void* kgraph_key = nullptr;
    int graph_key_species = -1, graph_key_prec = -1, graph_key_react = -1, graph_key_steps = -1;
    double graph_key_dt = 0.0;
    double graph_key_D[2] = {0, 0};
    double graph_key_params[5] = {0, 0, 0, 0, 0};
    int graph_key_forced = 0;
    double graph_key_t0 = 0.0, graph_key_lam = 0.0;
    // device: int64 steps done by the forced stages, then int non-finite flag
    void* counters = nullptr;
    int* nonfinite_host = nullptr;  // pinned host copy of the flag
};

int set_error(rbffd_ctx ctx, int code, const char* fmt, ...);
// Look up the device address of the allocation-free call's array on `device`
// (current); once per device, at context creation.
int noalloc_scratch_setup(rbffd_ctx ctx, int device);
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
