// Internal interface between the batched host code and the weights kernels.
#pragma once

#include "common.h"
#include "weights_job.h"

// A run of `count` consecutive stencils of job `job`, starting at `start`.
struct WorkItem {
    int32_t job;
    int32_t count;
    int64_t start;
};

namespace rbw {
// Kernel launchers, one specialisation per (radial kernel K, tiling NB),
// each defined in its own build of weights_kernels.hip.
template <int K, int NB>
void launch_weights(hipStream_t st, const Job& J);
template <int K, int NB>
void launch_weights_batched(hipStream_t st, const Job* jobs, const WorkItem* items, int nitems, int* cursor,
                            int grid);
}  // namespace rbw

// Validates opts for a set of N nodes and fills o (returns an RBFFD_E_* code).
int weights_check_opts(rbffd_ctx ctx, int64_t N, const rbffd_weight_opts* opts, rbw::WOpts& o);
// Persistent launch over `nitems` items (device arrays) with `grid` workgroups
// of four wavefronts; nb = 1 for m <= 64, 2 for m <= 128.  *cursor must be 0.
int weights_launch_batched(rbffd_ctx ctx, int kernel, int nb, const rbw::Job* jobs, const WorkItem* items,
                           int nitems, int* cursor, int grid);
