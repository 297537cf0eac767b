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
// This file holds the kernels; it is compiled once per (radial kernel K,
// tiling NB) with RBW_K and RBW_NB defined, so the large unrolled kernels
// build in parallel.  The host API is in weights.cpp and batched.cpp.
#include "weights_impl.h"
#include "batched.h"

#ifndef RBW_K
#error "RBW_K (radial kernel) must be defined"
#endif
#ifndef RBW_NB
#error "RBW_NB (1 or 2) must be defined"
#endif

using namespace rbw;

namespace {

template <int NB>
__device__ __forceinline__ Tid make_tid(int threads_base) {
    Tid t;
    if constexpr (NB == 1) {
        // one wavefront per stencil: block indices are compile-time zero
        t.lane = threadIdx.x & 63;
        t.tid = t.lane;
        t.rb = 0;
        t.cb = 0;
        t.c = t.lane;
    } else {
        const int tid = threadIdx.x - threads_base;
        t.tid = tid;
        t.lane = tid & 63;
        const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        t.rb = wave / NB;
        t.cb = wave % NB;
        t.c = 64 * t.cb + t.lane;
    }
    return t;
}

// One workgroup (NB^2 wavefronts) per stencil.
template <int K, int NB>
__global__ __launch_bounds__(64 * NB * NB, 2) void k_weights(Job J) {
    __shared__ Shared<NB> S;
    const int64_t s = blockIdx.x;
    if (s >= J.N) return;
    process_stencil<K, NB>(J, s, S, make_tid<NB>(0));
}

// Persistent launch over many stencil sets.  Each workgroup (four wavefronts)
// takes work items from a global counter until none are left.  An item is a
// run of `count` stencils of one set.  NB = 1 (m <= 64): the four waves take
// every fourth stencil of the item, one wave per stencil.  NB = 2 (m <= 128):
// the four waves do the item's stencils one after another, together.  One
// kernel per NB: the two register tilings in one kernel need more than 256
// VGPRs and spill.
template <int K, int NB>
__global__ __launch_bounds__(256, 2) void k_weights_batched(const Job* __restrict__ jobs,
                                                         const WorkItem* __restrict__ items, int nitems,
                                                         int* __restrict__ cursor) {
    __shared__ Shared<NB> S[NB == 1 ? 4 : 1];
    __shared__ int item_sh;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    for (;;) {
        if (threadIdx.x == 0) item_sh = atomicAdd(cursor, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(item_sh);  // uniform: item fields go to SGPRs
        __syncthreads();
        if (it >= nitems) break;
        const WorkItem w = items[it];
        const Job& J = jobs[w.job];
        if constexpr (NB == 1) {
            for (int q = wave; q < w.count; q += 4) process_stencil<K, 1>(J, w.start + q, S[wave], make_tid<1>(64 * wave));
        } else {
            for (int q = 0; q < w.count; ++q) process_stencil<K, 2>(J, w.start + q, S[0], make_tid<2>(0));
        }
        __syncthreads();
    }
}

}  // namespace

namespace rbw {

template <int K, int NB>
void launch_weights(hipStream_t st, const Job& J) {
    const dim3 g((unsigned)J.N), b(64 * NB * NB);
    hipLaunchKernelGGL((k_weights<K, NB>), g, b, 0, st, J);
}

template <int K, int NB>
void launch_weights_batched(hipStream_t st, const Job* jobs, const WorkItem* items, int nitems, int* cursor,
                            int grid) {
    hipLaunchKernelGGL((k_weights_batched<K, NB>), dim3((unsigned)grid), dim3(256), 0, st, jobs, items, nitems,
                       cursor);
}

template void launch_weights<RBW_K, RBW_NB>(hipStream_t, const Job&);
template void launch_weights_batched<RBW_K, RBW_NB>(hipStream_t, const Job*, const WorkItem*, int, int*, int);

}  // namespace rbw
