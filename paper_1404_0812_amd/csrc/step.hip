// Sparse operator L_X and the method-of-lines time stepper (Sec. 4.2,
// eq. kernel_mol): du_s/dt = D_s L_X u_s + R_s(u), classical RK4.
//
// Layout: sliced ELL with slices of 64 rows (one wavefront), slot-major
// inside a slice: slot k of row r of a slice sits at off + 64 k + r, so the
// loads of the weights and indices of one wavefront are one contiguous run.
// Every row of a surface has exactly n entries (Sec. 4), so a slice holds no
// padding except past a surface's last row.  Rows are in the library's
// spatial order, so the gathered neighbour values are close in memory.  Many
// surfaces (each with its own N and n) form one block-diagonal operator:
// each surface starts on a fresh slice and each slice carries its own n.
// Both precisions store the n - 1 off-diagonal slots of every row in the same
// layout (FP32 and FP64 weights side by side, one index array) and read the
// neighbour values through the slice's halo staged in LDS.  FP64 state uses
// the plain form w_ii u_i + sum_{j != i} w_ij u_j (the diagonal weight kept
// per row), exact for any weights.  FP32 state uses the difference form
// sum_{j != i} w_ij (u_j - u_i) with FP32 weights; it equals L u because the
// rows of L_X sum to zero (constants are reproduced), and it keeps L 1 = 0
// exact in FP32.
//
// One RK4 stage is one kernel: it applies L to the stage input of every
// species with one read of the row, adds the reaction, and writes the next
// stage input and the RK accumulator; stage 4 writes the new state.  The
// steps are captured in a HIP graph and replayed.
#include "common.h"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <cstring>
#include <new>
#include <vector>

namespace {

constexpr int BLK = 256;

// Element offset, inside a slice of `ns` slots, of slot k of lane r: the first
// 4 (ns / 4) slots go in groups of four with a lane's four slots adjacent (one
// 16-byte load per lane for FP32, two for FP64), the remaining slots one
// 64-element run each.  A slice holds 64 ns elements either way.
__host__ __device__ __forceinline__ int64_t slot_pos(int k, int ns, int r) {
    const int G = ns >> 2;
    return k < 4 * G ? 256 * (int64_t)(k >> 2) + 4 * r + (k & 3) : 256 * (int64_t)G + 64 * (int64_t)(k - 4 * G) + r;
}

// iperm[perm[p]] = p for one surface (perm nullable: identity); iperm starts
// at -1, and a perm entry outside [0, N) sets *bad instead of being written.
__global__ void k_inverse_perm(int64_t N, const int32_t* __restrict__ perm, int32_t* __restrict__ iperm,
                               int* __restrict__ bad) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t v = perm ? perm[p] : p;
    if (v >= 0 && v < N) iperm[v] = (int32_t)p;
    else *bad = 1;
}

// Rows of one surface into the slices.  row0: first internal row of the
// surface, col0: its first caller row; gperm: internal row -> caller row.
// A stencil entry outside [0, N), or a row that perm does not reach, sets
// *bad; the slot then points at the row itself with weight 0 (the operator is
// discarded by the caller, but nothing reads out of bounds meanwhile).
__global__ void k_build_sell(int64_t N, int n, int64_t row0, int64_t col0, const int32_t* __restrict__ idx,
                             const double* __restrict__ w, const int32_t* __restrict__ perm,
                             const int32_t* __restrict__ iperm, const OpSlice* __restrict__ slices,
                             double* __restrict__ wd64, double* __restrict__ w64, int32_t* __restrict__ idx32,
                             float* __restrict__ w32, int32_t* __restrict__ gperm, int* __restrict__ bad) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= N) return;
    int64_t i = perm ? perm[p] : p;
    if (i < 0 || i >= N || iperm[p] < 0) {  // out of range, or perm misses caller row p
        *bad = 1;
        i = i < 0 || i >= N ? 0 : i;
    }
    const int64_t q = row0 + p;
    const OpSlice sl = slices[q >> 6];
    const int r = (int)(q & 63);
    // slot 0 must be the row's own node: the FP32 difference form drops it
    if (idx[i * n] != i) *bad = 1;
    for (int k = 0; k < n; ++k) {
        const int32_t c = idx[i * n + k];
        const int32_t ip = (c >= 0 && c < N) ? iperm[c] : -1;
        const bool ok = ip >= 0;
        if (!ok) *bad = 1;
        const int32_t j = (int32_t)(row0 + (ok ? ip : p));
        const double wk = ok ? w[i * n + k] : 0.0;
        if (k == 0) {
            wd64[q] = wk;
        } else {
            const int64_t q32 = sl.off32 + slot_pos(k - 1, n - 1, r);
            idx32[q32] = j;
            w32[q32] = (float)wk;
            w64[q32] = wk;
        }
    }
    gperm[q] = (int32_t)(col0 + i);
}

// Halo of each slice for the FP32 path: the sorted distinct rows its 64 rows
// read (off-diagonal slots), and every slot entry rewritten as a position in
// that list.  One 256-thread block per slice: the <= 64 x 127 entries are
// sorted in LDS (bitonic), de-duplicated with a block scan, and each entry is
// located in the unique list by binary search.  Slices with more than
// OP_HALO_MAX distinct rows keep halo = -1 and are read directly.
constexpr int HB_CAP = 8192;  // >= 64 x 127 entries per slice

__global__ __launch_bounds__(256) void k_build_halo(int64_t nslices, OpSlice* __restrict__ slices,
                                                    const int32_t* __restrict__ idx32, uint16_t* __restrict__ lidx,
                                                    int32_t* __restrict__ halo) {
    __shared__ int32_t key[HB_CAP];
    __shared__ int32_t cnt[256];
    __shared__ int32_t uniq[OP_HALO_MAX];
    const int64_t s = blockIdx.x;
    if (s >= nslices) return;
    const OpSlice sl = slices[s];
    const int ns = sl.n - 1, rows = sl.rows, E = rows * ns, tid = threadIdx.x;
    for (int i = tid; i < HB_CAP; i += 256)
        key[i] = i < E ? idx32[sl.off32 + slot_pos(i % ns, ns, i / ns)] : 0x7fffffff;
    __syncthreads();
    for (int size = 2; size <= HB_CAP; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < HB_CAP / 2; i += 256) {
                const int lo = 2 * i - (i & (stride - 1));  // first of the pair (stride apart)
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const int a = key[lo], b = key[hi];
                if ((a > b) == up) {
                    key[lo] = b;
                    key[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    // distinct keys among the E sorted entries: thread t counts its 32 consecutive ones
    constexpr int PER = HB_CAP / 256;
    int c = 0;
    for (int q = 0; q < PER; ++q) {
        const int i = tid * PER + q;
        c += (i < E && (i == 0 || key[i] != key[i - 1])) ? 1 : 0;
    }
    cnt[tid] = c;
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int t = 0; t < 256; ++t) {
            const int v = cnt[t];
            cnt[t] = run;
            run += v;
        }
        slices[s].halo = run <= OP_HALO_MAX ? run : -1;
        key[HB_CAP - 1] = run <= OP_HALO_MAX ? run : -1;  // E < HB_CAP: the last slot is padding
    }
    __syncthreads();
    const int H = key[HB_CAP - 1];
    if (H < 0) return;
    int pos = cnt[tid];
    for (int q = 0; q < PER; ++q) {
        const int i = tid * PER + q;
        if (i < E && (i == 0 || key[i] != key[i - 1])) {
            uniq[pos] = key[i];
            halo[s * OP_HALO_MAX + pos] = key[i];
            ++pos;
        }
    }
    __syncthreads();
    for (int i = tid; i < E; i += 256) {
        const int64_t at = sl.off32 + slot_pos(i % ns, ns, i / ns);
        const int32_t j = idx32[at];
        int lo = 0, hi = H - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (uniq[mid] < j) lo = mid + 1;
            else hi = mid;
        }
        lidx[at] = (uint16_t)lo;
    }
}

// State lives species-interleaved in internal order: element (p, s) at p*S + s,
// so that one gather fetches every species of a neighbour.
// P internal rows, N caller rows; padding rows (perm -1) hold zero.
template <typename T>
__global__ void k_load_state(int64_t P, int64_t N, int S, const double* __restrict__ in,
                             const int32_t* __restrict__ perm, T* __restrict__ out) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int64_t i = perm[p];
    for (int s = 0; s < S; ++s) out[p * S + s] = i >= 0 ? (T)in[s * N + i] : (T)0;
}

template <typename T>
__global__ void k_store_state(int64_t P, int64_t N, int S, const T* __restrict__ in, const int32_t* __restrict__ perm,
                              double* __restrict__ out) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int64_t i = perm[p];
    if (i < 0) return;
    for (int s = 0; s < S; ++s) out[s * N + i] = (double)in[p * S + s];
}

struct ReactParams {
    double p[5];
};

template <typename T, int R>
__device__ __forceinline__ void reaction(const T (&y)[2], T (&r)[2], const ReactParams& rp) {
    if (R == RBFFD_REACT_SCHNAKENBERG) {
        const T a = (T)rp.p[0], b = (T)rp.p[1], g = (T)rp.p[2];
        const T u2v = y[0] * y[0] * y[1];
        r[0] = g * (a - y[0] + u2v);
        r[1] = g * (b - u2v);
    } else if (R == RBFFD_REACT_TURING) {
        const T al = (T)rp.p[0], be = (T)rp.p[1], ga = (T)rp.p[2], t1 = (T)rp.p[3], t2 = (T)rp.p[4];
        const T u = y[0], v = y[1];
        r[0] = al * u * ((T)1 - t1 * v * v) + v * ((T)1 - t2 * u);
        r[1] = be * v * ((T)1 + al * t1 / be * u * v) + u * (ga + t2 * v);
    } else {
        r[0] = (T)0;
        r[1] = (T)0;
    }
}

struct StageArgs {
    int64_t nslices;
    const OpSlice* slices;
    const uint16_t* lidx;   // halo positions of the slot entries
    const int32_t* halo;    // halo lists (OP_HALO_MAX per slice)
    const double* wd64;     // FP64 path: diagonal weight per internal row
    double D[2];
    double dt;
    ReactParams rp;
    int* nonfinite;         // set to 1 by the last stage when a state value is not finite
    // forcing f_s(t, x_p) = exp(lam t) F[p S + s] (FORCED kernels only): the
    // stage time is t0 + (*steps_done + step_in_launch + c_stage) dt, with
    // *steps_done advanced on the device after each launch sequence
    const void* F;
    double lam, t0, toff;   // toff = (step_in_launch + c_stage), set per launch
    const int64_t* steps_done;
};

// Blocks are dispatched round-robin over the 8 XCDs; remap them so that each
// XCD works on one contiguous range of rows (its L2 then holds the part of the
// gathered state those rows touch).
__device__ __forceinline__ int64_t xcd_block() {
    const int64_t nb = gridDim.x, b = blockIdx.x;
    const int64_t x = b & 7, q = nb >> 3, rem = nb & 7;
    return x * q + (x < rem ? x : rem) + (b >> 3);
}

template <typename T, int S>
struct Vec;
template <>
struct Vec<float, 1> { using type = float; };
template <>
struct Vec<float, 2> { using type = float2; };
template <>
struct Vec<double, 1> { using type = double; };
template <>
struct Vec<double, 2> { using type = double2; };

template <typename T, int S>
__device__ __forceinline__ void vload(const T* __restrict__ Y, int64_t j, T (&v)[2]) {
    if constexpr (S == 2) {
        const typename Vec<T, 2>::type t = reinterpret_cast<const typename Vec<T, 2>::type*>(Y)[j];
        v[0] = t.x;
        v[1] = t.y;
    } else {
        v[0] = Y[j];
        v[1] = (T)0;
    }
}
template <typename T, int S>
__device__ __forceinline__ void vstore(T* __restrict__ Y, int64_t j, const T (&v)[2]) {
    if constexpr (S == 2) {
        typename Vec<T, 2>::type t;
        t.x = v[0];
        t.y = v[1];
        reinterpret_cast<typename Vec<T, 2>::type*>(Y)[j] = t;
    } else {
        Y[j] = v[0];
    }
}

// Row of the calling thread: slice and lane.  Four slices per 256-thread block.
struct RowPos {
    int64_t p;      // internal row
    int64_t slice;  // -1: past the last slice (the whole wavefront)
    int64_t base;   // element offset of the slice's off-diagonal slots
    int lane;
    int ns;         // slots to read
    int halo;       // halo size, or -1 (direct gathers)
    bool live;
};

template <typename T>
__device__ __forceinline__ RowPos row_pos(const StageArgs& a) {
    RowPos rp;
    const int64_t slice = (int64_t)xcd_block() * (BLK / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    rp.lane = threadIdx.x & 63;
    rp.p = slice * 64 + rp.lane;
    rp.live = false;
    rp.base = 0;
    rp.ns = 0;
    rp.halo = -1;
    rp.slice = -1;
    if (slice >= a.nslices) return rp;
    const OpSlice sl = a.slices[slice];
    rp.slice = slice;
    rp.live = rp.lane < sl.rows;
    rp.base = sl.off32;
    rp.ns = sl.n - 1;
    rp.halo = sl.halo;
    return rp;
}

typedef int i4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

// four consecutive slots of one lane (streamed once: non-temporal)
__device__ __forceinline__ void load4(const int32_t* ix, const float* wx, int (&j)[4], float (&w)[4]) {
    const i4v jv = __builtin_nontemporal_load(reinterpret_cast<const i4v*>(ix));
    const f4v wv = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(wx));
    j[0] = jv.x; j[1] = jv.y; j[2] = jv.z; j[3] = jv.w;
    w[0] = wv.x; w[1] = wv.y; w[2] = wv.z; w[3] = wv.w;
}
__device__ __forceinline__ void load4(const int32_t* ix, const double* wx, int (&j)[4], double (&w)[4]) {
    const i4v jv = __builtin_nontemporal_load(reinterpret_cast<const i4v*>(ix));
    const d2v w0 = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(wx));
    const d2v w1 = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(wx) + 1);
    j[0] = jv.x; j[1] = jv.y; j[2] = jv.z; j[3] = jv.w;
    w[0] = w0.x; w[1] = w0.y; w[2] = w1.x; w[3] = w1.y;
}

template <typename T, int S>
__device__ __forceinline__ void accumulate(const T* __restrict__ Y, int j, T wk, const T (&yi)[2], T& s0, T& s1) {
    constexpr bool diff = sizeof(T) == 4;
    T y[2];
    vload<T, S>(Y, j, y);
    if (diff) {
        s0 = fma(wk, y[0] - yi[0], s0);
        if (S == 2) s1 = fma(wk, y[1] - yi[1], s1);
    } else {
        s0 = fma(wk, y[0], s0);
        if (S == 2) s1 = fma(wk, y[1], s1);
    }
}

// L applied to the stage input of row rp.p by direct gathers, in slot order.
// FP32: difference form over the n-1 off-diagonal slots; FP64: the diagonal
// term wd u_i, then the off-diagonal slots (plain form).
template <typename T, int S>
__device__ __forceinline__ void apply_row(const RowPos& rp, const int32_t* __restrict__ idx,
                                          const T* __restrict__ w, const T* __restrict__ Y, const T (&yi)[2],
                                          T wd, T (&acc)[2]) {
    const int ns = rp.ns;
    const int G = ns >> 2;
    const int32_t* ix = idx + rp.base + 4 * rp.lane;
    const T* wx = w + rp.base + 4 * rp.lane;
    T s0 = wd * yi[0], s1 = wd * yi[1];
    int g = 0;
    for (; g + 2 <= G; g += 2) {  // eight slots in flight
        int j[8];
        T wk[8];
        load4(ix + 256 * g, wx + 256 * g, *reinterpret_cast<int(*)[4]>(j), *reinterpret_cast<T(*)[4]>(wk));
        load4(ix + 256 * (g + 1), wx + 256 * (g + 1), *reinterpret_cast<int(*)[4]>(j + 4),
              *reinterpret_cast<T(*)[4]>(wk + 4));
#pragma unroll
        for (int t = 0; t < 8; ++t) accumulate<T, S>(Y, j[t], wk[t], yi, s0, s1);
    }
    if (g < G) {
        int j[4];
        T wk[4];
        load4(ix + 256 * g, wx + 256 * g, j, wk);
#pragma unroll
        for (int t = 0; t < 4; ++t) accumulate<T, S>(Y, j[t], wk[t], yi, s0, s1);
    }
    const int32_t* ir = idx + rp.base + 256 * G + rp.lane;
    const T* wr = w + rp.base + 256 * G + rp.lane;
    for (int t = 0; t < ns - 4 * G; ++t)
        accumulate<T, S>(Y, __builtin_nontemporal_load(ir + 64 * t), __builtin_nontemporal_load(wr + 64 * t), yi,
                         s0, s1);
    acc[0] = s0;
    acc[1] = s1;
}

typedef unsigned short u4v __attribute__((ext_vector_type(4)));

// Stage the slice's halo values (all 64 lanes of the wavefront take part).
template <typename T, int S>
__device__ __forceinline__ void load_halo(const RowPos& rp, const int32_t* __restrict__ halo,
                                          const T* __restrict__ Y, typename Vec<T, S>::type* ylds) {
    const int32_t* h = halo + rp.slice * OP_HALO_MAX;
    for (int t = rp.lane; t < rp.halo; t += 64) ylds[t] = reinterpret_cast<const typename Vec<T, S>::type*>(Y)[h[t]];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, int S>
__device__ __forceinline__ void halo_value(const typename Vec<T, S>::type* ylds, int l, T (&y)[2]) {
    if constexpr (S == 2) {
        const typename Vec<T, 2>::type v = ylds[l];
        y[0] = v.x;
        y[1] = v.y;
    } else {
        y[0] = ylds[l];
        y[1] = (T)0;
    }
}

// four consecutive weights of one lane
__device__ __forceinline__ void loadw4(const float* wx, float (&w)[4]) {
    const f4v wv = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(wx));
    w[0] = wv.x; w[1] = wv.y; w[2] = wv.z; w[3] = wv.w;
}
__device__ __forceinline__ void loadw4(const double* wx, double (&w)[4]) {
    const d2v w0 = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(wx));
    const d2v w1 = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(wx) + 1);
    w[0] = w0.x; w[1] = w0.y; w[2] = w1.x; w[3] = w1.y;
}

// The n-1 off-diagonal slots with neighbour values from the staged halo (same
// slot order as apply_row): FP32 difference form, FP64 plain form after the
// diagonal term.
template <typename T, int S>
__device__ __forceinline__ void apply_row_halo(const RowPos& rp, const uint16_t* __restrict__ lidx,
                                               const T* __restrict__ w, const typename Vec<T, S>::type* ylds,
                                               const T (&yi)[2], T wd, T (&acc)[2]) {
    constexpr bool diff = sizeof(T) == 4;
    const int ns = rp.ns;
    const int G = ns >> 2;
    const uint16_t* lx = lidx + rp.base + 4 * rp.lane;
    const T* wx = w + rp.base + 4 * rp.lane;
    T s0 = wd * yi[0], s1 = wd * yi[1];
    auto acc1 = [&](int l, T wk) {
        T y[2];
        halo_value<T, S>(ylds, l, y);
        if (diff) {
            s0 = fma(wk, y[0] - yi[0], s0);
            if (S == 2) s1 = fma(wk, y[1] - yi[1], s1);
        } else {
            s0 = fma(wk, y[0], s0);
            if (S == 2) s1 = fma(wk, y[1], s1);
        }
    };
    int g = 0;
    for (; g + 4 <= G; g += 4) {  // sixteen slots in flight
        u4v lv[4];
        T wv[4][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            lv[q] = __builtin_nontemporal_load(reinterpret_cast<const u4v*>(lx + 256 * (g + q)));
            loadw4(wx + 256 * (g + q), wv[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            acc1(lv[q].x, wv[q][0]);
            acc1(lv[q].y, wv[q][1]);
            acc1(lv[q].z, wv[q][2]);
            acc1(lv[q].w, wv[q][3]);
        }
    }
    for (; g < G; ++g) {
        const u4v lv = __builtin_nontemporal_load(reinterpret_cast<const u4v*>(lx + 256 * g));
        T wv[4];
        loadw4(wx + 256 * g, wv);
        acc1(lv.x, wv[0]);
        acc1(lv.y, wv[1]);
        acc1(lv.z, wv[2]);
        acc1(lv.w, wv[3]);
    }
    const uint16_t* lr = lidx + rp.base + 256 * G + rp.lane;
    const T* wr = w + rp.base + 256 * G + rp.lane;
    for (int t = 0; t < ns - 4 * G; ++t) acc1(__builtin_nontemporal_load(lr + 64 * t), __builtin_nontemporal_load(wr + 64 * t));
    acc[0] = s0;
    acc[1] = s1;
}

// L applied to the stage input of row rp.p: through the staged halo when the
// slice has one, otherwise by direct gathers.  Every lane of the wavefront
// must call this (the halo is loaded cooperatively).
template <typename T, int S>
__device__ __forceinline__ void laplacian_row(const StageArgs& a, const RowPos& rp, const int32_t* __restrict__ idx,
                                              const T* __restrict__ w, const T* __restrict__ Y, const T (&yi)[2],
                                              T (&lap)[2]) {
    __shared__ typename Vec<T, S>::type ylds[BLK / 64][OP_HALO_MAX];
    T wd = (T)0;
    if constexpr (sizeof(T) == 8) {
        if (rp.live) wd = __builtin_nontemporal_load(a.wd64 + rp.p);
    }
    if (rp.halo >= 0) {
        auto* yl = ylds[threadIdx.x >> 6];
        load_halo<T, S>(rp, a.halo, Y, yl);
        if (rp.live) apply_row_halo<T, S>(rp, a.lidx, w, yl, yi, wd, lap);
        return;
    }
    if (rp.live) apply_row<T, S>(rp, idx, w, Y, yi, wd, lap);
}

// RK4 stage `ST` (0..3).  Y: stage input; U: state at the start of the step;
// ACC: accumulator; YN: next stage input (stages 0-2) -- stage 3 updates U
// (FP32: YN is then the compensation term of the update).
template <typename T, int S, int R, int ST, bool FORCED>
__global__ __launch_bounds__(BLK) void k_rk4_stage(StageArgs a, const int32_t* __restrict__ idx,
                                                   const T* __restrict__ w, const T* __restrict__ Y,
                                                   T* __restrict__ U, T* __restrict__ ACC, T* __restrict__ YN) {
    const RowPos rp = row_pos<T>(a);
    if (rp.slice < 0) return;  // the whole wavefront
    const int64_t p = rp.p;
    T yi[2] = {0, 0};
    if (rp.live) vload<T, S>(Y, p, yi);
    T lap[2];
    laplacian_row<T, S>(a, rp, idx, w, Y, yi, lap);
    if (!rp.live) return;
    T r[2];
    reaction<T, R>(yi, r, a.rp);
    T k[2];
    k[0] = (T)a.D[0] * lap[0] + r[0];
    k[1] = (T)a.D[1] * lap[1] + r[1];
    if constexpr (FORCED) {
        const double t = a.t0 + ((double)*a.steps_done + a.toff) * a.dt;  // uniform
        const T ef = (T)exp(a.lam * t);
        T f[2];
        vload<T, S>(reinterpret_cast<const T*>(a.F), p, f);
        k[0] = fma(ef, f[0], k[0]);
        k[1] = fma(ef, f[1], k[1]);
    }
    const T dt = (T)a.dt;
    T u[2], c[2], o[2];
    if (ST == 0) {
        vload<T, S>(U, p, u);
        o[0] = u[0] + (T)0.5 * dt * k[0];
        o[1] = u[1] + (T)0.5 * dt * k[1];
        vstore<T, S>(ACC, p, k);
        vstore<T, S>(YN, p, o);
    } else if (ST == 1 || ST == 2) {
        vload<T, S>(U, p, u);
        vload<T, S>(ACC, p, c);
        const T h = ST == 1 ? (T)0.5 * dt : dt;
        o[0] = u[0] + h * k[0];
        o[1] = u[1] + h * k[1];
        c[0] = c[0] + (T)2 * k[0];
        c[1] = c[1] + (T)2 * k[1];
        vstore<T, S>(ACC, p, c);
        vstore<T, S>(YN, p, o);
    } else {
        vload<T, S>(U, p, u);
        vload<T, S>(ACC, p, c);
        if constexpr (sizeof(T) == 4) {
            // FP32 state: compensated (Kahan) update, the running rounding error
            // kept in YN; over 1e4 steps of increments ~1e-4 of the state the
            // plain update drifts by several 1e-5 against FP64
            T e[2];
            vload<T, S>(YN, p, e);
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const T d = dt / (T)6 * (c[q] + k[q]) - e[q];
                const T t = u[q] + d;
                e[q] = (t - u[q]) - d;
                o[q] = t;
            }
            vstore<T, S>(U, p, o);
            vstore<T, S>(YN, p, e);
        } else {
            o[0] = u[0] + dt / (T)6 * (c[0] + k[0]);
            o[1] = u[1] + dt / (T)6 * (c[1] + k[1]);
            vstore<T, S>(U, p, o);
        }
        if (!(isfinite(o[0]) && isfinite(o[1]))) *a.nonfinite = 1;  // every writer stores 1
    }
}

// Device-side step counter of the forced stages, advanced after each launch sequence.
__global__ void k_advance_steps(int64_t* steps_done, int64_t by) { *steps_done += by; }
__global__ void k_set_steps(int64_t* steps_done, int* nonfinite) {
    *steps_done = 0;
    *nonfinite = 0;
}

// one operator application (stage-free): out = L y (reaction-free, D = 1)
template <typename T>
__global__ __launch_bounds__(BLK) void k_apply(StageArgs a, const int32_t* __restrict__ idx, const T* __restrict__ w,
                                               const T* __restrict__ Y, T* __restrict__ out) {
    const RowPos rp = row_pos<T>(a);
    if (rp.slice < 0) return;  // the whole wavefront
    T yi[2] = {0, 0};
    if (rp.live) vload<T, 1>(Y, rp.p, yi);
    T lap[2];
    laplacian_row<T, 1>(a, rp, idx, w, Y, yi, lap);
    if (rp.live) out[rp.p] = lap[0];
}

// blocks of one stage launch: four slices each
inline dim3 stage_grid(int64_t nslices) { return dim3((unsigned)((nslices + BLK / 64 - 1) / (BLK / 64))); }

// One RK4 step, the i-th of its launch sequence; stage times t_n + c dt with
// c = 0, 1/2, 1/2, 1.
template <typename T, int S, int R, bool FORCED>
void enqueue_step(hipStream_t st, StageArgs a, int64_t i, const int32_t* idx, const T* w, T* U, T* ACC, T* Y1,
                  T* Y2, T* COMP) {
    const dim3 g = stage_grid(a.nslices), b(BLK);
    a.toff = (double)i;
    hipLaunchKernelGGL((k_rk4_stage<T, S, R, 0, FORCED>), g, b, 0, st, a, idx, w, U, U, ACC, Y1);
    a.toff = (double)i + 0.5;
    hipLaunchKernelGGL((k_rk4_stage<T, S, R, 1, FORCED>), g, b, 0, st, a, idx, w, Y1, U, ACC, Y2);
    hipLaunchKernelGGL((k_rk4_stage<T, S, R, 2, FORCED>), g, b, 0, st, a, idx, w, Y2, U, ACC, Y1);
    a.toff = (double)i + 1.0;
    hipLaunchKernelGGL((k_rk4_stage<T, S, R, 3, FORCED>), g, b, 0, st, a, idx, w, Y1, U, ACC, COMP);
}

template <typename T, bool FORCED>
void enqueue_steps_f(hipStream_t st, int S, int R, const StageArgs& a, const int32_t* idx, const T* w, T* U, T* ACC,
                     T* COMP, T* Y1, T* Y2, int64_t steps) {
    for (int64_t i = 0; i < steps; ++i) {
        if (S == 1) {
            enqueue_step<T, 1, RBFFD_REACT_NONE, FORCED>(st, a, i, idx, w, U, ACC, Y1, Y2, COMP);
        } else if (R == RBFFD_REACT_SCHNAKENBERG) {
            enqueue_step<T, 2, RBFFD_REACT_SCHNAKENBERG, FORCED>(st, a, i, idx, w, U, ACC, Y1, Y2, COMP);
        } else if (R == RBFFD_REACT_TURING) {
            enqueue_step<T, 2, RBFFD_REACT_TURING, FORCED>(st, a, i, idx, w, U, ACC, Y1, Y2, COMP);
        } else {
            enqueue_step<T, 2, RBFFD_REACT_NONE, FORCED>(st, a, i, idx, w, U, ACC, Y1, Y2, COMP);
        }
    }
    // forced stages read the step counter: advance it past this sequence
    if (FORCED) hipLaunchKernelGGL(k_advance_steps, dim3(1), dim3(1), 0, st, const_cast<int64_t*>(a.steps_done), steps);
}

template <typename T>
void enqueue_steps_t(hipStream_t st, int S, int R, const StageArgs& a, const int32_t* idx, const T* w, T* U, T* ACC,
                     T* COMP, T* Y1, T* Y2, int64_t steps) {
    if (a.F) enqueue_steps_f<T, true>(st, S, R, a, idx, w, U, ACC, COMP, Y1, Y2, steps);
    else enqueue_steps_f<T, false>(st, S, R, a, idx, w, U, ACC, COMP, Y1, Y2, steps);
}

int ensure_work(rbffd_op op) {
    // 4 buffers (U, ACC, Y1, Y2) x 2 species x FP64, and the forcing (2 species)
    size_t need = 5 * 2 * (size_t)op->P * sizeof(double);
    if (op->work_bytes >= need) return RBFFD_OK;
    if (op->work) {
        (void)hipStreamSynchronize(op->ctx->stream);
        (void)hipFree(op->work);
        op->work = nullptr;
    }
    if (hipMalloc(&op->work, need) != hipSuccess) {
        op->work = nullptr;
        return set_error(op->ctx, RBFFD_E_NOMEM, "cannot allocate %zu bytes of state", need);
    }
    op->work_bytes = need;
    return RBFFD_OK;
}

void reset_graph(rbffd_op op) {
    if (op->graph) {
        (void)hipGraphExecDestroy(op->graph);
        op->graph = nullptr;
    }
    op->graph_key_species = -1;
}

void reset_kgraph(rbffd_op op) {
    if (op->kgraph) {
        (void)hipGraphExecDestroy(op->kgraph);
        op->kgraph = nullptr;
    }
    op->kgraph_key = nullptr;
}

// Build the sliced operator of nsurf surfaces (validated by the callers).
int create_op(rbffd_ctx ctx, int nsurf, const rbffd_op_surface* surf, rbffd_op* out) {
    std::vector<OpSlice> sl;
    std::vector<int64_t> row0(nsurf), col0(nsurf);
    int64_t P = 0, N = 0, off32 = 0, maxN = 0;
    int32_t nmax = 0;
    for (int s = 0; s < nsurf; ++s) {
        row0[s] = P;
        col0[s] = N;
        const int64_t Ns = surf[s].N;
        const int n = surf[s].n;
        for (int64_t r = 0; r < Ns; r += 64) {
            OpSlice o;
            o.off32 = off32;
            o.n = n;
            o.rows = (int32_t)std::min<int64_t>(64, Ns - r);
            o.halo = -1;
            o.pad = 0;
            sl.push_back(o);
            off32 += 64 * (int64_t)(n - 1);
        }
        P += (Ns + 63) / 64 * 64;
        N += Ns;
        maxN = std::max(maxN, Ns);
        nmax = std::max(nmax, n);
    }
    if (P > 0x7fffffffLL) return set_error(ctx, RBFFD_E_ARG, "operator too large: %lld rows", (long long)P);
    rbffd_op op = new (std::nothrow) rbffd_op_s();
    if (!op) return set_error(ctx, RBFFD_E_NOMEM, "host allocation failed");
    op->ctx = ctx;
    op->N = N;
    op->P = P;
    op->n = nmax;
    op->nsurf = nsurf;
    op->nslices = (int64_t)sl.size();
    bool ok = hipMalloc(&op->slices, std::max<size_t>(1, sl.size()) * sizeof(OpSlice)) == hipSuccess &&
              hipMalloc(&op->wd64, std::max<int64_t>(1, P) * sizeof(double)) == hipSuccess &&
              hipMalloc(&op->w64, std::max<int64_t>(1, off32) * sizeof(double)) == hipSuccess &&
              hipMalloc(&op->idx32, std::max<int64_t>(1, off32) * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&op->w32, std::max<int64_t>(1, off32) * sizeof(float)) == hipSuccess &&
              hipMalloc(&op->lidx, std::max<int64_t>(1, off32) * sizeof(uint16_t)) == hipSuccess &&
              hipMalloc(&op->halo, std::max<size_t>(1, sl.size()) * OP_HALO_MAX * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&op->perm, std::max<int64_t>(1, P) * sizeof(int32_t)) == hipSuccess;
    ok = ok && hipMalloc(&op->counters, sizeof(int64_t) + sizeof(int)) == hipSuccess &&
         hipHostMalloc(reinterpret_cast<void**>(&op->nonfinite_host), sizeof(int), hipHostMallocDefault) == hipSuccess;
    int32_t* iperm = nullptr;
    int* bad = nullptr;
    ok = ok && hipMalloc(&iperm, std::max<int64_t>(1, maxN) * sizeof(int32_t)) == hipSuccess;
    ok = ok && hipMalloc(&bad, sizeof(int)) == hipSuccess;
    if (!ok) {
        rbffd_op_destroy(op);
        if (iperm) (void)hipFree(iperm);
        if (bad) (void)hipFree(bad);
        return set_error(ctx, RBFFD_E_NOMEM, "operator allocation failed");
    }
    hipStream_t st = ctx->stream;
    hipError_t e = hipMemcpyAsync(op->slices, sl.data(), sl.size() * sizeof(OpSlice), hipMemcpyHostToDevice, st);
    // padding rows: perm -1; their slots are never read (rows >= OpSlice::rows are skipped)
    if (e == hipSuccess) e = hipMemsetAsync(op->perm, 0xff, (size_t)P * sizeof(int32_t), st);
    if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(int), st);
    for (int s = 0; s < nsurf && e == hipSuccess; ++s) {
        const int64_t Ns = surf[s].N;
        const dim3 g((unsigned)((Ns + BLK - 1) / BLK)), b(BLK);
        e = hipMemsetAsync(iperm, 0xff, (size_t)Ns * sizeof(int32_t), st);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_inverse_perm, g, b, 0, st, Ns, surf[s].perm, iperm, bad);
        hipLaunchKernelGGL(k_build_sell, g, b, 0, st, Ns, surf[s].n, row0[s], col0[s], surf[s].idx, surf[s].w,
                           surf[s].perm, iperm, op->slices, op->wd64, op->w64, op->idx32, op->w32, op->perm, bad);
        e = hipGetLastError();
    }
    if (e == hipSuccess && !sl.empty()) {
        hipLaunchKernelGGL(k_build_halo, dim3((unsigned)sl.size()), dim3(256), 0, st, (int64_t)sl.size(), op->slices,
                           op->idx32, op->lidx, op->halo);
        e = hipGetLastError();
    }
    // the slice table comes from pageable host memory and iperm is reused per surface: wait here
    const hipError_t e2 = hipStreamSynchronize(st);
    if (e == hipSuccess) e = e2;
    int bad_h = 0;
    if (e == hipSuccess) e = hipMemcpy(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost);
    (void)hipFree(iperm);
    (void)hipFree(bad);
    if (e != hipSuccess) {
        rbffd_op_destroy(op);
        return set_error(ctx, RBFFD_E_HIP, "operator build failed: %s", hipGetErrorString(e));
    }
    if (bad_h) {
        rbffd_op_destroy(op);
        return set_error(ctx, RBFFD_E_ARG, "stencil or perm entry outside [0, N) (or perm not a permutation)");
    }
    *out = op;
    return RBFFD_OK;
}

int check_surface(rbffd_ctx ctx, int s, const rbffd_op_surface& d) {
    if (d.N <= 0 || d.N > 0x7fffffffLL) return set_error(ctx, RBFFD_E_ARG, "surface %d: N out of range", s);
    if (d.n < 2 || d.n > 128 || d.n > d.N)
        return set_error(ctx, RBFFD_E_ARG, "surface %d: stencil size n=%d invalid", s, d.n);
    if (!d.idx || !d.w) return set_error(ctx, RBFFD_E_ARG, "surface %d: null pointer", s);
    return RBFFD_OK;
}

}  // namespace

extern "C" int rbffd_op_create(rbffd_ctx ctx, int64_t N, int32_t n, const int32_t* idx, const double* w,
                               const int32_t* perm, rbffd_op* out) {
    if (!ctx || !out) return RBFFD_E_ARG;
    rbffd_op_surface d;
    d.N = N;
    d.n = n;
    d.reserved = 0;
    d.idx = idx;
    d.w = w;
    d.perm = perm;
    if (N <= 0 || N > 0x7fffffffLL) return set_error(ctx, RBFFD_E_ARG, "N out of range");
    if (n < 2 || n > 128 || n > N) return set_error(ctx, RBFFD_E_ARG, "stencil size n=%d invalid", n);
    if (!idx || !w) return set_error(ctx, RBFFD_E_ARG, "null pointer");
    return create_op(ctx, 1, &d, out);
}

extern "C" int rbffd_op_create_batched(rbffd_ctx ctx, int32_t nsurf, const rbffd_op_surface* surf, rbffd_op* out) {
    if (!ctx || !out) return RBFFD_E_ARG;
    if (nsurf < 1 || !surf) return set_error(ctx, RBFFD_E_ARG, "need at least one surface");
    for (int s = 0; s < nsurf; ++s) {
        int rc = check_surface(ctx, s, surf[s]);
        if (rc) return rc;
    }
    return create_op(ctx, nsurf, surf, out);
}

extern "C" int rbffd_op_destroy(rbffd_op op) {
    if (!op) return RBFFD_E_ARG;
    if (op->ctx) (void)hipStreamSynchronize(op->ctx->stream);
    reset_graph(op);
    reset_kgraph(op);
    if (op->slices) (void)hipFree(op->slices);
    if (op->wd64) (void)hipFree(op->wd64);
    if (op->w64) (void)hipFree(op->w64);
    if (op->idx32) (void)hipFree(op->idx32);
    if (op->w32) (void)hipFree(op->w32);
    if (op->lidx) (void)hipFree(op->lidx);
    if (op->halo) (void)hipFree(op->halo);
    if (op->perm) (void)hipFree(op->perm);
    if (op->work) (void)hipFree(op->work);
    if (op->impl) (void)hipFree(op->impl);
    if (op->counters) (void)hipFree(op->counters);
    if (op->nonfinite_host) (void)hipHostFree(op->nonfinite_host);
    delete op;
    return RBFFD_OK;
}

extern "C" int rbffd_op_stats(rbffd_op op, int64_t* nslices, int64_t* halo_slices, int64_t* halo_rows,
                              int64_t* halo_entries) {
    if (!op) return RBFFD_E_ARG;
    std::vector<OpSlice> sl((size_t)op->nslices);
    if (!sl.empty()) {
        HIP_TRY(op->ctx, hipStreamSynchronize(op->ctx->stream));
        HIP_TRY(op->ctx, hipMemcpy(sl.data(), op->slices, sl.size() * sizeof(OpSlice), hipMemcpyDeviceToHost));
    }
    int64_t hs = 0, hr = 0, he = 0;
    for (const OpSlice& o : sl)
        if (o.halo >= 0) {
            ++hs;
            hr += o.rows;
            he += o.halo;
        }
    if (nslices) *nslices = op->nslices;
    if (halo_slices) *halo_slices = hs;
    if (halo_rows) *halo_rows = hr;
    if (halo_entries) *halo_entries = he;
    return RBFFD_OK;
}

// ------------------------------------------------------------------------
// Allocation-free operator application.  The internal-order input and output
// vectors live in one fixed device array per GPU (RBFFD_NOALLOC_SCRATCH_BYTES),
// whose device address is looked up once per device when a context is
// created there.  The array's name is a host-side stand-in in host code: only
// the looked-up pointer is ever passed to kernels.
static __device__ __align__(256) unsigned char scratch[RBFFD_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

// Called by rbffd_create with `device` current.
int noalloc_scratch_setup(rbffd_ctx ctx, int device) {
    if (device < 0 || device >= MAX_DEVICES) return set_error(ctx, RBFFD_E_UNSUPPORTED, "device index %d", device);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return RBFFD_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return set_error(ctx, RBFFD_E_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
    return RBFFD_OK;
}

extern "C" int rbffd_apply_noalloc(rbffd_ctx ctx, rbffd_op op, int32_t prec, const double* u, double* Lu) {
    if (!ctx || !op || !u || !Lu) return set_error(ctx, RBFFD_E_ARG, "null argument");
    if (prec != RBFFD_F64 && prec != RBFFD_F32) return set_error(ctx, RBFFD_E_ARG, "prec must be F64 or F32");
    const int64_t N = op->N, P = op->P;
    const size_t need = 2 * (size_t)P * (prec == RBFFD_F64 ? sizeof(double) : sizeof(float));
    if (need > (size_t)RBFFD_NOALLOC_SCRATCH_BYTES)
        return set_error(ctx, RBFFD_E_UNSUPPORTED, "operator of %lld padded rows needs %zu bytes of scratch, above the "
                         "%d-byte array of the allocation-free call", (long long)P, need, RBFFD_NOALLOC_SCRATCH_BYTES);
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (ctx->device >= 0 && ctx->device < MAX_DEVICES) base = g_scratch_ptr[ctx->device];
    }
    if (!base) return set_error(ctx, RBFFD_E_HIP, "no scratch address for device %d", ctx->device);
    hipStream_t st = ctx->stream;
    const dim3 g((unsigned)((P + BLK - 1) / BLK)), b(BLK);
    StageArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nslices = op->nslices;
    a.slices = op->slices;
    a.lidx = op->lidx;
    a.halo = op->halo;
    a.wd64 = op->wd64;
    if (prec == RBFFD_F64) {
        double* Y = (double*)base;
        double* out = Y + P;
        hipLaunchKernelGGL(k_load_state<double>, g, b, 0, st, P, N, 1, u, op->perm, Y);
        hipLaunchKernelGGL(k_apply<double>, stage_grid(a.nslices), b, 0, st, a, op->idx32, op->w64, Y, out);
        hipLaunchKernelGGL(k_store_state<double>, g, b, 0, st, P, N, 1, out, op->perm, Lu);
    } else {
        float* Y = (float*)base;
        float* out = Y + P;
        hipLaunchKernelGGL(k_load_state<float>, g, b, 0, st, P, N, 1, u, op->perm, Y);
        hipLaunchKernelGGL(k_apply<float>, stage_grid(a.nslices), b, 0, st, a, op->idx32, op->w32, Y, out);
        hipLaunchKernelGGL(k_store_state<float>, g, b, 0, st, P, N, 1, out, op->perm, Lu);
    }
    HIP_TRY(ctx, hipGetLastError());
    return RBFFD_OK;
}

extern "C" int rbffd_apply(rbffd_ctx ctx, rbffd_op op, int32_t prec, const double* u, double* Lu) {
    if (!ctx || !op || !u || !Lu) return set_error(ctx, RBFFD_E_ARG, "null argument");
    if (prec != RBFFD_F64 && prec != RBFFD_F32) return set_error(ctx, RBFFD_E_ARG, "prec must be F64 or F32");
    op->ctx = ctx;
    int rc = ensure_work(op);
    if (rc) return rc;
    hipStream_t st = ctx->stream;
    const int64_t N = op->N, P = op->P;
    const dim3 g((unsigned)((P + BLK - 1) / BLK)), b(BLK);
    StageArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nslices = op->nslices;
    a.slices = op->slices;
    a.lidx = op->lidx;
    a.halo = op->halo;
    a.wd64 = op->wd64;
    if (prec == RBFFD_F64) {
        double* Y = (double*)op->work;
        double* out = Y + P;
        hipLaunchKernelGGL(k_load_state<double>, g, b, 0, st, P, N, 1, u, op->perm, Y);
        hipLaunchKernelGGL(k_apply<double>, stage_grid(a.nslices), b, 0, st, a, op->idx32, op->w64, Y, out);
        hipLaunchKernelGGL(k_store_state<double>, g, b, 0, st, P, N, 1, out, op->perm, Lu);
    } else {
        float* Y = (float*)op->work;
        float* out = Y + P;
        hipLaunchKernelGGL(k_load_state<float>, g, b, 0, st, P, N, 1, u, op->perm, Y);
        hipLaunchKernelGGL(k_apply<float>, stage_grid(a.nslices), b, 0, st, a, op->idx32, op->w32, Y, out);
        hipLaunchKernelGGL(k_store_state<float>, g, b, 0, st, P, N, 1, out, op->perm, Lu);
    }
    HIP_TRY(ctx, hipGetLastError());
    return RBFFD_OK;
}

namespace {

int step_impl(rbffd_ctx ctx, rbffd_op op, int32_t nspecies, double* state, int32_t prec, const double* D,
              int32_t reaction, const double* params, double dt, int64_t nsteps, int32_t graph_steps, double t0,
              const double* forcing, double lam) {
    if (!ctx || !op || !state || !D) return set_error(ctx, RBFFD_E_ARG, "null argument");
    if (nspecies != 1 && nspecies != 2) return set_error(ctx, RBFFD_E_ARG, "nspecies must be 1 or 2");
    if (prec != RBFFD_F64 && prec != RBFFD_F32) return set_error(ctx, RBFFD_E_ARG, "prec must be F64 or F32");
    if (reaction < 0 || reaction > 2) return set_error(ctx, RBFFD_E_ARG, "unknown reaction %d", reaction);
    if (reaction != RBFFD_REACT_NONE && nspecies != 2)
        return set_error(ctx, RBFFD_E_ARG, "reaction needs two species");
    if (reaction != RBFFD_REACT_NONE && !params) return set_error(ctx, RBFFD_E_ARG, "reaction params required");
    if (!(dt > 0.0)) return set_error(ctx, RBFFD_E_ARG, "dt must be > 0");
    if (nsteps < 0) return set_error(ctx, RBFFD_E_ARG, "nsteps must be >= 0");
    if (graph_steps < 0) return set_error(ctx, RBFFD_E_ARG, "graph_steps must be >= 0");
    if (forcing && !(std::isfinite(t0) && std::isfinite(lam)))
        return set_error(ctx, RBFFD_E_ARG, "t0 and lambda must be finite");
    op->ctx = ctx;
    int rc = ensure_work(op);
    if (rc) return rc;
    hipStream_t st = ctx->stream;
    const int64_t N = op->N, P = op->P;
    const dim3 g((unsigned)((P + BLK - 1) / BLK)), b(BLK);
    StageArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nslices = op->nslices;
    a.slices = op->slices;
    a.lidx = op->lidx;
    a.halo = op->halo;
    a.wd64 = op->wd64;
    a.D[0] = D[0];
    a.D[1] = nspecies == 2 ? D[1] : 0.0;
    a.dt = dt;
    const int np = reaction == RBFFD_REACT_SCHNAKENBERG ? 3 : (reaction == RBFFD_REACT_TURING ? 5 : 0);
    for (int i = 0; i < np; ++i) a.rp.p[i] = params[i];
    int64_t* steps_done = reinterpret_cast<int64_t*>(op->counters);
    int* nonfinite = reinterpret_cast<int*>(reinterpret_cast<char*>(op->counters) + sizeof(int64_t));
    a.nonfinite = nonfinite;
    a.steps_done = steps_done;
    const int G = graph_steps > 0 ? graph_steps : 50;
    const size_t esz = prec == RBFFD_F64 ? sizeof(double) : sizeof(float);
    char* base = (char*)op->work;
    void* U = base;
    void* ACC = base + 2 * P * esz;
    void* Y1 = base + 4 * P * esz;
    void* Y2 = base + 6 * P * esz;
    // FP32: compensation of the state update (inside the FP64-sized work area)
    void* COMP = prec == RBFFD_F64 ? nullptr : (void*)(base + 8 * P * esz);
    void* FI = base + 8 * P * sizeof(double);  // forcing in internal order, after the FP64 buffers
    if (forcing) {
        a.F = FI;
        a.lam = lam;
        a.t0 = t0;
    }
    const int32_t* idx = op->idx32;
    const void* w = prec == RBFFD_F64 ? (const void*)op->w64 : (const void*)op->w32;
    // counters are cleared by a kernel (no memset node near the captured graph)
    hipLaunchKernelGGL(k_set_steps, dim3(1), dim3(1), 0, st, steps_done, nonfinite);
    if (prec == RBFFD_F64) {
        hipLaunchKernelGGL(k_load_state<double>, g, b, 0, st, P, N, nspecies, state, op->perm, (double*)U);
        if (forcing) hipLaunchKernelGGL(k_load_state<double>, g, b, 0, st, P, N, nspecies, forcing, op->perm, (double*)FI);
    } else {
        hipLaunchKernelGGL(k_load_state<float>, g, b, 0, st, P, N, nspecies, state, op->perm, (float*)U);
        if (forcing) hipLaunchKernelGGL(k_load_state<float>, g, b, 0, st, P, N, nspecies, forcing, op->perm, (float*)FI);
        HIP_TRY(ctx, hipMemsetAsync(COMP, 0, 2 * (size_t)P * sizeof(float), st));  // outside any captured graph
    }
    HIP_TRY(ctx, hipGetLastError());

    auto enqueue = [&](hipStream_t s, int64_t steps) {
        if (prec == RBFFD_F64)
            enqueue_steps_t<double>(s, nspecies, reaction, a, idx, (const double*)w, (double*)U, (double*)ACC,
                                    nullptr, (double*)Y1, (double*)Y2, steps);
        else
            enqueue_steps_t<float>(s, nspecies, reaction, a, idx, (const float*)w, (float*)U, (float*)ACC,
                                   (float*)COMP, (float*)Y1, (float*)Y2, steps);
    };
    const int64_t reps = nsteps / G;
    const int64_t rest = nsteps % G;
    volatile int* nf_host = reinterpret_cast<volatile int*>(op->nonfinite_host);
    *nf_host = 0;
    bool stopped = false;
    if (reps > 0) {
        const int forced = forcing ? 1 : 0;
        bool same = op->graph && op->graph_key_species == nspecies && op->graph_key_prec == prec &&
                    op->graph_key_react == reaction && op->graph_key_steps == G && op->graph_key_dt == dt &&
                    op->graph_key_D[0] == a.D[0] && op->graph_key_D[1] == a.D[1] &&
                    std::memcmp(op->graph_key_params, a.rp.p, sizeof(a.rp.p)) == 0 &&
                    op->graph_key_forced == forced && (!forced || (op->graph_key_t0 == t0 && op->graph_key_lam == lam));
        if (!same) {
            reset_graph(op);
            hipGraph_t graph;
            HIP_TRY(ctx, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            enqueue(st, G);
            hipError_t ce = hipStreamEndCapture(st, &graph);
            if (ce != hipSuccess) return set_error(ctx, RBFFD_E_HIP, "graph capture failed: %s", hipGetErrorString(ce));
            hipError_t ie = hipGraphInstantiate(&op->graph, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) {
                op->graph = nullptr;
                return set_error(ctx, RBFFD_E_HIP, "graph instantiate failed: %s", hipGetErrorString(ie));
            }
            op->graph_key_species = nspecies;
            op->graph_key_prec = prec;
            op->graph_key_react = reaction;
            op->graph_key_steps = G;
            op->graph_key_dt = dt;
            op->graph_key_D[0] = a.D[0];
            op->graph_key_D[1] = a.D[1];
            std::memcpy(op->graph_key_params, a.rp.p, sizeof(a.rp.p));
            op->graph_key_forced = forced;
            op->graph_key_t0 = t0;
            op->graph_key_lam = lam;
        }
        for (int64_t r = 0; r < reps; ++r) {
            // the flag copied after an earlier replay has already landed: stop on a blow-up
            if (*nf_host) {
                stopped = true;
                break;
            }
            HIP_TRY(ctx, hipGraphLaunch(op->graph, st));
            HIP_TRY(ctx, hipMemcpyAsync(op->nonfinite_host, nonfinite, sizeof(int), hipMemcpyDeviceToHost, st));
        }
    }
    if (rest > 0 && !stopped) enqueue(st, rest);
    if (prec == RBFFD_F64)
        hipLaunchKernelGGL(k_store_state<double>, g, b, 0, st, P, N, nspecies, (const double*)U, op->perm, state);
    else
        hipLaunchKernelGGL(k_store_state<float>, g, b, 0, st, P, N, nspecies, (const float*)U, op->perm, state);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipMemcpyAsync(op->nonfinite_host, nonfinite, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    if (*nf_host)
        return set_error(ctx, RBFFD_E_NONFINITE,
                         "the state became non-finite (steps stopped early; state holds the last values)");
    return RBFFD_OK;
}

}  // namespace

extern "C" int rbffd_step(rbffd_ctx ctx, rbffd_op op, int32_t nspecies, double* state, int32_t prec, const double* D,
                          int32_t reaction, const double* params, double dt, int64_t nsteps, int32_t graph_steps) {
    return step_impl(ctx, op, nspecies, state, prec, D, reaction, params, dt, nsteps, graph_steps, 0.0, nullptr,
                     0.0);
}

extern "C" int rbffd_step_forced(rbffd_ctx ctx, rbffd_op op, int32_t nspecies, double* state, int32_t prec,
                                 const double* D, int32_t reaction, const double* params, double dt, int64_t nsteps,
                                 int32_t graph_steps, double t0, const double* forcing, double lambda) {
    if (!forcing) return set_error(ctx, RBFFD_E_ARG, "forcing is required");
    return step_impl(ctx, op, nspecies, state, prec, D, reaction, params, dt, nsteps, graph_steps, t0, forcing,
                     lambda);
}

// ------------------------------------------------------------------------
// Semi-implicit BDF time stepping (the paper's BDF4 of Sec. 6 for the forced
// diffusion problems and SBDF2 of Sec. 7 for the Turing system): each step
//   sum_{j=0}^{k} a_j u^{n+1-j} = dt (D L u^{n+1} + f(t_{n+1}) + sum_{j=1}^{k} b_j R(u^{n+1-j})),
// i.e. (I - gamma L) u_s^{n+1} = rhs_s / a_0 with gamma = dt D_s / a_0, solved
// per species by unpreconditioned BiCGSTAB, restarted from the true residual
// after a breakdown.  There is no diagonal (Jacobi) scaling on purpose: on
// irregular node sets some stencils give L a positive diagonal entry, so the
// diagonal of I - gamma L passes through zero as dt grows and dividing by it
// wrecks the iteration, while the unscaled system stays well conditioned
// (its eigenvalues have real part >= 1 whenever L's are in the left half
// plane, the stability property of Sec. 5).  Vectors are FP64 in internal
// order, one array per species; every scalar of the iteration stays on the
// device, the host reads the residual norm once per iteration to stop.
namespace {

constexpr int RED_BLOCKS = 512;

struct BdfCoef {
    double a[5], b[4];
};

// k-step BDF row a and extrapolation row b (see the oracle's table).
BdfCoef bdf_coef(int k) {
    BdfCoef c;
    std::memset(&c, 0, sizeof(c));
    if (k == 1) {
        c.a[0] = 1.0; c.a[1] = -1.0;
        c.b[0] = 1.0;
    } else if (k == 2) {
        c.a[0] = 1.5; c.a[1] = -2.0; c.a[2] = 0.5;
        c.b[0] = 2.0; c.b[1] = -1.0;
    } else if (k == 3) {
        c.a[0] = 11.0 / 6.0; c.a[1] = -3.0; c.a[2] = 1.5; c.a[3] = -1.0 / 3.0;
        c.b[0] = 3.0; c.b[1] = -3.0; c.b[2] = 1.0;
    } else {
        c.a[0] = 25.0 / 12.0; c.a[1] = -4.0; c.a[2] = 3.0; c.a[3] = -4.0 / 3.0; c.a[4] = 0.25;
        c.b[0] = 4.0; c.b[1] = -6.0; c.b[2] = 4.0; c.b[3] = -1.0;
    }
    return c;
}

// Scalars of one BiCGSTAB solve (device).
struct KrylovScalars {
    double rho, alpha, omega, beta;
    double bb, rr;        // ||b||^2, ||r||^2
    double rr0;           // ||rhat||^2 (the residual at the last start)
    double tol2;          // tol^2
    double gamma;         // the solve's I - gamma L (read by the operator kernel)
    int breakdown;        // rhat (nearly) orthogonal to r, or a zero step
    int done;             // 0 running, 1 converged, 2 restart wanted, 3 non-finite residual
    int iters;            // iterations done since the solve began (restarts not counted)
    int pad;
};

// Iterations launched between two reads of the scalars by the host; the
// kernels of iterations after convergence (or a breakdown) return at once.
constexpr int KRYLOV_BATCH = 8;

struct HistPtrs {
    const double* u[4];   // u^n, u^{n-1}, ... (one species)
    const double* r[4];   // R_s at those states (nullable entries when no reaction)
};

// b = (-sum_{j>=1} a_j u^{n+1-j} + dt sum_j b_j R^{n+1-j} + dt ef F) / a_0
// (0 on padding rows, whose reaction values are not zero in general)
__global__ void k_bdf_rhs(int64_t P, int k, BdfCoef c, HistPtrs h, const double* __restrict__ F, double ef,
                          double dt, const int32_t* __restrict__ perm, double* __restrict__ out) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    if (perm[p] < 0) {
        out[p] = 0.0;
        return;
    }
    double v = 0.0;
    for (int j = 1; j <= k; ++j) {
        v = fma(-c.a[j], h.u[j - 1][p], v);
        if (h.r[j - 1]) v = fma(dt * c.b[j - 1], h.r[j - 1][p], v);
    }
    if (F) v = fma(dt * ef, F[p], v);
    out[p] = v / c.a[0];
}

// R(u) for both species of one state (rows in internal order, per-species arrays).
template <int R>
__global__ void k_reaction2(int64_t P, const double* __restrict__ u, const double* __restrict__ v, ReactParams rp,
                            double* __restrict__ ru, double* __restrict__ rv) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    double y[2] = {u[p], v[p]}, r[2];
    reaction<double, R>(y, r, rp);
    ru[p] = r[0];
    rv[p] = r[1];
}

// out = x - gamma L x (live rows; padding rows keep their zero).  With ks
// (inside the iteration, also inside its graph) gamma comes from ks and the
// kernel is a no-op once the solve is done.
__global__ __launch_bounds__(BLK) void k_amul(StageArgs a, const int32_t* __restrict__ idx,
                                              const double* __restrict__ w, const double* __restrict__ X,
                                              double gamma, double* __restrict__ out,
                                              const KrylovScalars* __restrict__ ks) {
    if (ks) {
        if (ks->done) return;
        gamma = ks->gamma;
    }
    const RowPos rp = row_pos<double>(a);
    if (rp.slice < 0) return;
    double yi[2] = {0.0, 0.0};
    if (rp.live) yi[0] = X[rp.p];
    double lap[2];
    laplacian_row<double, 1>(a, rp, idx, w, X, yi, lap);
    if (rp.live) out[rp.p] = fma(-gamma, lap[0], yi[0]);
}

__device__ __forceinline__ double wave_sum_block(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block sums of up to two dot products over P rows; partials[blk * 2 + q].
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum_block(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    __syncthreads();
    return t;
}

template <int NQ>
__global__ __launch_bounds__(256) void k_dots(int64_t P, const double* __restrict__ a0, const double* __restrict__ b0,
                                              const double* __restrict__ a1, const double* __restrict__ b1,
                                              double* __restrict__ partials, const KrylovScalars* __restrict__ ks) {
    if (ks && ks->done) return;
    __shared__ double sh[4];
    double s0 = 0.0, s1 = 0.0;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        s0 = fma(a0[p], b0[p], s0);
        if (NQ == 2) s1 = fma(a1[p], b1[p], s1);
    }
    const double t0 = block_sum(s0, sh);
    double t1 = 0.0;
    if (NQ == 2) t1 = block_sum(s1, sh);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = t0;
        partials[2 * blockIdx.x + 1] = t1;
    }
}

// Sum the block partials in a fixed order (one wave): deterministic.
__device__ __forceinline__ void sum_partials(const double* __restrict__ partials, double& d0, double& d1) {
    double s0 = 0.0, s1 = 0.0;
    for (int i = threadIdx.x; i < RED_BLOCKS; i += 64) {
        s0 += partials[2 * i];
        s1 += partials[2 * i + 1];
    }
    d0 = wave_sum_block(s0);
    d1 = wave_sum_block(s1);
}

// Scalar steps of the iteration (one wave each); every mode but 0 is a no-op
// once the solve is done.
// MODE 0 (start; d0 = b.b, d1 = r.r, rhat = r): bb, rr = rr0 = rho = d1,
//         alpha = omega = 1, tol and gamma stored; iters = 0 on the first
//         start of a solve; done at once if r already meets tol
// MODE 2: alpha = rho / d0 (d0 = rhat.v)
// MODE 3: omega = d0 / d1 (t.s / t.t)
// MODE 4 (end of an iteration; d0 = r.r, d1 = rhat.r): rr = d0; converged,
//         non-finite, or else rho' = d1 and beta = (rho' / rho) (alpha / omega)
//         for the next iteration, unless |rho'| <= 1e-14 ||rhat|| ||r|| or
//         omega = 0 (breakdown: the host restarts from the true residual)
__device__ __forceinline__ int residual_state(const KrylovScalars* ks, double rr) {
    if (!(rr <= 1.79e308)) return 3;
    const double lim = ks->bb > 0.0 ? ks->tol2 * ks->bb : ks->tol2;
    return rr <= lim ? 1 : 0;
}

template <int MODE>
__global__ void k_krylov_scalar(const double* __restrict__ partials, KrylovScalars* __restrict__ ks, double tol,
                                int first, double gamma) {
    if (MODE != 0 && ks->done) return;
    double d0, d1;
    sum_partials(partials, d0, d1);
    if (threadIdx.x != 0) return;
    if (MODE == 0) {
        ks->bb = d0;
        ks->rr = ks->rr0 = ks->rho = d1;
        ks->alpha = ks->omega = 1.0;
        ks->beta = 0.0;
        ks->tol2 = tol * tol;
        ks->gamma = gamma;
        ks->breakdown = 0;
        if (first) ks->iters = 0;
        ks->done = residual_state(ks, d1);
    } else if (MODE == 2) {
        if (d0 == 0.0) ks->breakdown = 1;
        ks->alpha = ks->breakdown ? 0.0 : ks->rho / d0;
    } else if (MODE == 3) {
        ks->omega = d1 > 0.0 ? d0 / d1 : 0.0;
    } else {
        ks->iters += 1;
        ks->rr = d0;
        const int st = residual_state(ks, d0);
        if (st) {
            ks->done = st;
            return;
        }
        const double rho = d1;
        if (ks->breakdown || !(std::fabs(rho) > 1e-14 * std::sqrt(ks->rr0 * d0)) || ks->omega == 0.0) {
            ks->breakdown = 1;
            ks->done = 2;
            return;
        }
        ks->beta = (rho / ks->rho) * (ks->alpha / ks->omega);
        ks->rho = rho;
    }
}

// r = b - Ax; rhat = r; p = v = 0
__global__ void k_kry_init(int64_t P, const double* __restrict__ b, const double* __restrict__ ax,
                           double* __restrict__ r, double* __restrict__ rh, double* __restrict__ pv,
                           double* __restrict__ v) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    const double rv = b[p] - ax[p];
    r[p] = rv;
    rh[p] = rv;
    pv[p] = 0.0;
    v[p] = 0.0;
}

// p = r + beta (p - omega v)
__global__ void k_kry_p(int64_t P, const KrylovScalars* __restrict__ ks, const double* __restrict__ r,
                        double* __restrict__ pv, const double* __restrict__ v) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P || ks->done) return;
    const double beta = ks->beta, omega = ks->omega;
    pv[p] = fma(beta, fma(-omega, v[p], pv[p]), r[p]);
}

// s = r - alpha v
__global__ void k_kry_s(int64_t P, const KrylovScalars* __restrict__ ks, const double* __restrict__ r,
                        const double* __restrict__ v, double* __restrict__ s) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P || ks->done) return;
    s[p] = fma(-ks->alpha, v[p], r[p]);
}

// x += alpha p + omega s; r = s - omega t
__global__ void k_kry_xr(int64_t P, const KrylovScalars* __restrict__ ks, const double* __restrict__ pv,
                         const double* __restrict__ s, const double* __restrict__ t, double* __restrict__ x,
                         double* __restrict__ r) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P || ks->done) return;
    const double alpha = ks->alpha, omega = ks->omega;
    const double sv = s[p];
    x[p] = fma(omega, sv, fma(alpha, pv[p], x[p]));
    r[p] = fma(-omega, t[p], sv);
}

__global__ void k_copy(int64_t P, const double* __restrict__ src, double* __restrict__ dst) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p < P) dst[p] = src[p];
}

int ensure_impl(rbffd_op op, size_t bytes) {
    if (op->impl_bytes >= bytes) return RBFFD_OK;
    if (op->impl) {
        (void)hipStreamSynchronize(op->ctx->stream);
        reset_kgraph(op);
        (void)hipFree(op->impl);
        op->impl = nullptr;
        op->impl_bytes = 0;
    }
    if (hipMalloc(&op->impl, bytes) != hipSuccess) {
        op->impl = nullptr;
        return set_error(op->ctx, RBFFD_E_NOMEM, "cannot allocate %zu bytes for the implicit stepper", bytes);
    }
    op->impl_bytes = bytes;
    // every vector starts at zero (padding rows are never written again)
    HIP_TRY(op->ctx, hipMemsetAsync(op->impl, 0, bytes, op->ctx->stream));
    return RBFFD_OK;
}

}  // namespace

extern "C" int rbffd_step_imex(rbffd_ctx ctx, rbffd_op op, int32_t nspecies, double* state, const double* D,
                               int32_t reaction, const double* params, double dt, int64_t nsteps, int32_t order,
                               const double* history, double t0, const double* forcing, double lambda, double tol,
                               int32_t maxit, int64_t* iters_out, double* relres_out) {
    if (!ctx || !op || !state || !D) return set_error(ctx, RBFFD_E_ARG, "null argument");
    if (nspecies != 1 && nspecies != 2) return set_error(ctx, RBFFD_E_ARG, "nspecies must be 1 or 2");
    if (reaction < 0 || reaction > 2) return set_error(ctx, RBFFD_E_ARG, "unknown reaction %d", reaction);
    if (reaction != RBFFD_REACT_NONE && nspecies != 2) return set_error(ctx, RBFFD_E_ARG, "reaction needs two species");
    if (reaction != RBFFD_REACT_NONE && !params) return set_error(ctx, RBFFD_E_ARG, "reaction params required");
    if (!(dt > 0.0)) return set_error(ctx, RBFFD_E_ARG, "dt must be > 0");
    if (nsteps < 0) return set_error(ctx, RBFFD_E_ARG, "nsteps must be >= 0");
    if (order < 1 || order > 4) return set_error(ctx, RBFFD_E_ARG, "order must be 1..4");
    if (!(tol > 0.0) || maxit < 1) return set_error(ctx, RBFFD_E_ARG, "tol must be > 0 and maxit >= 1");
    if (forcing && !(std::isfinite(t0) && std::isfinite(lambda)))
        return set_error(ctx, RBFFD_E_ARG, "t0 and lambda must be finite");
    op->ctx = ctx;
    const int64_t N = op->N, P = op->P;
    const int S = nspecies;
    const bool react = reaction != RBFFD_REACT_NONE;
    // layout: U[s][order], R[s][order] (reaction), F[s], b, x, r, rh, p, v, s, t; partials; scalars
    const int nvec = S * order * (react ? 2 : 1) + S + 8;
    const size_t vbytes = (size_t)P * sizeof(double);
    const size_t bytes = nvec * vbytes + 2 * RED_BLOCKS * sizeof(double) + 256;
    int rc = ensure_impl(op, bytes);
    if (rc) return rc;
    hipStream_t st = ctx->stream;
    double* base = (double*)op->impl;
    auto vec = [&](int i) { return base + (size_t)i * P; };
    int vi = 0;
    double* U[2][4] = {};
    double* Rh[2][4] = {};
    for (int s = 0; s < S; ++s)
        for (int j = 0; j < order; ++j) U[s][j] = vec(vi++);
    if (react)
        for (int s = 0; s < S; ++s)
            for (int j = 0; j < order; ++j) Rh[s][j] = vec(vi++);
    double* Fi[2] = {};
    for (int s = 0; s < S; ++s) Fi[s] = vec(vi++);
    double* bvec = vec(vi++);
    double* x = vec(vi++);
    double* r = vec(vi++);
    double* rh = vec(vi++);
    double* pv = vec(vi++);
    double* v = vec(vi++);
    double* sv = vec(vi++);
    double* tv = vec(vi++);
    double* partials = vec(vi);
    KrylovScalars* ks = reinterpret_cast<KrylovScalars*>(partials + 2 * RED_BLOCKS);
    const dim3 g((unsigned)((P + BLK - 1) / BLK)), b(BLK);
    StageArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nslices = op->nslices;
    a.slices = op->slices;
    a.lidx = op->lidx;
    a.halo = op->halo;
    a.wd64 = op->wd64;
    ReactParams rp;
    std::memset(&rp, 0, sizeof(rp));
    const int np = reaction == RBFFD_REACT_SCHNAKENBERG ? 3 : (reaction == RBFFD_REACT_TURING ? 5 : 0);
    for (int i = 0; i < np; ++i) rp.p[i] = params[i];
    // history: state (and the caller's earlier states, if any) into internal order
    const int have0 = history ? order : 1;
    for (int s = 0; s < S; ++s) {
        hipLaunchKernelGGL(k_load_state<double>, g, b, 0, st, P, N, 1, state + (size_t)s * N, op->perm, U[s][0]);
        for (int j = 1; j < have0; ++j)
            hipLaunchKernelGGL(k_load_state<double>, g, b, 0, st, P, N, 1,
                               history + ((size_t)(j - 1) * S + s) * N, op->perm, U[s][j]);
        if (forcing)
            hipLaunchKernelGGL(k_load_state<double>, g, b, 0, st, P, N, 1, forcing + (size_t)s * N, op->perm, Fi[s]);
    }
    auto eval_reaction = [&](int j) {
        if (!react) return;
        if (reaction == RBFFD_REACT_SCHNAKENBERG)
            hipLaunchKernelGGL(k_reaction2<RBFFD_REACT_SCHNAKENBERG>, g, b, 0, st, P, U[0][j], U[1][j], rp, Rh[0][j],
                               Rh[1][j]);
        else
            hipLaunchKernelGGL(k_reaction2<RBFFD_REACT_TURING>, g, b, 0, st, P, U[0][j], U[1][j], rp, Rh[0][j], Rh[1][j]);
    };
    for (int j = 0; j < have0; ++j) eval_reaction(j);
    HIP_TRY(ctx, hipGetLastError());
    // ring of history slots: slot[j] = index into U/Rh of u^{n-j}
    int slot[4] = {0, 1, 2, 3};
    int have = have0;
    int64_t iters = 0;
    double worst = 0.0;
    int result = RBFFD_OK;
    const unsigned rg = RED_BLOCKS;
    for (int64_t n = 0; n < nsteps && result == RBFFD_OK; ++n) {
        const int k = std::min(order, have);
        const BdfCoef c = bdf_coef(k);
        const double t1 = t0 + (double)(n + 1) * dt;
        // the new state goes to the oldest slot (order == k) or the next free one
        const int newslot = have < order ? slot[have] : slot[order - 1];
        for (int s = 0; s < S; ++s) {
            HistPtrs h;
            std::memset(&h, 0, sizeof(h));
            for (int j = 0; j < k; ++j) {
                h.u[j] = U[s][slot[j]];
                h.r[j] = react ? Rh[s][slot[j]] : nullptr;
            }
            const double ef = forcing ? std::exp(lambda * t1) : 0.0;
            hipLaunchKernelGGL(k_bdf_rhs, g, b, 0, st, P, k, c, h, forcing ? (const double*)Fi[s] : nullptr, ef, dt,
                               op->perm, bvec);
            const double gamma = dt * D[s] / c.a[0];
            // (re)start from the true residual of x
            auto krylov_start = [&](int first) {
                hipLaunchKernelGGL(k_amul, stage_grid(a.nslices), b, 0, st, a, op->idx32, op->w64, x, gamma, tv,
                                   (const KrylovScalars*)nullptr);
                hipLaunchKernelGGL(k_kry_init, g, b, 0, st, P, bvec, tv, r, rh, pv, v);
                hipLaunchKernelGGL(k_dots<2>, dim3(rg), dim3(256), 0, st, P, bvec, bvec, r, r, partials,
                                   (const KrylovScalars*)nullptr);
                hipLaunchKernelGGL(k_krylov_scalar<0>, dim3(1), dim3(64), 0, st, partials, ks, tol, first, gamma);
            };
            // one iteration; every kernel takes its scalars (gamma too) from ks,
            // so the same launches serve every species, step and tolerance
            auto iteration = [&]() {
                hipLaunchKernelGGL(k_kry_p, g, b, 0, st, P, ks, r, pv, v);
                hipLaunchKernelGGL(k_amul, stage_grid(a.nslices), b, 0, st, a, op->idx32, op->w64, pv, 0.0, v, ks);
                hipLaunchKernelGGL(k_dots<1>, dim3(rg), dim3(256), 0, st, P, rh, v, nullptr, nullptr, partials, ks);
                hipLaunchKernelGGL(k_krylov_scalar<2>, dim3(1), dim3(64), 0, st, partials, ks, 0.0, 0, 0.0);
                hipLaunchKernelGGL(k_kry_s, g, b, 0, st, P, ks, r, v, sv);
                hipLaunchKernelGGL(k_amul, stage_grid(a.nslices), b, 0, st, a, op->idx32, op->w64, sv, 0.0, tv, ks);
                hipLaunchKernelGGL(k_dots<2>, dim3(rg), dim3(256), 0, st, P, tv, sv, tv, tv, partials, ks);
                hipLaunchKernelGGL(k_krylov_scalar<3>, dim3(1), dim3(64), 0, st, partials, ks, 0.0, 0, 0.0);
                hipLaunchKernelGGL(k_kry_xr, g, b, 0, st, P, ks, pv, sv, tv, x, r);
                hipLaunchKernelGGL(k_dots<2>, dim3(rg), dim3(256), 0, st, P, r, r, rh, r, partials, ks);
                hipLaunchKernelGGL(k_krylov_scalar<4>, dim3(1), dim3(64), 0, st, partials, ks, 0.0, 0, 0.0);
            };
            // KRYLOV_BATCH iterations from one HIP graph (88 launches), captured
            // once per operator and vector layout
            auto batch_graph = [&]() -> int {
                if (!op->kgraph || op->kgraph_key != (const void*)x) {
                    reset_kgraph(op);
                    hipGraph_t graph;
                    HIP_TRY(ctx, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                    for (int q = 0; q < KRYLOV_BATCH; ++q) iteration();
                    hipError_t ce = hipStreamEndCapture(st, &graph);
                    if (ce != hipSuccess)
                        return set_error(ctx, RBFFD_E_HIP, "graph capture failed: %s", hipGetErrorString(ce));
                    hipError_t ie = hipGraphInstantiate(&op->kgraph, graph, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(graph);
                    if (ie != hipSuccess) {
                        op->kgraph = nullptr;
                        return set_error(ctx, RBFFD_E_HIP, "graph instantiate failed: %s", hipGetErrorString(ie));
                    }
                    op->kgraph_key = x;
                }
                HIP_TRY(ctx, hipGraphLaunch(op->kgraph, st));
                return RBFFD_OK;
            };
            // initial guess: the current state
            hipLaunchKernelGGL(k_copy, g, b, 0, st, P, U[s][slot[0]], x);
            krylov_start(1);
            HIP_TRY(ctx, hipGetLastError());
            bool conv = false;
            double relres = 0.0;
            int restarts = 0;
            for (;;) {
                KrylovScalars hs;
                HIP_TRY(ctx, hipMemcpyAsync(&hs, ks, sizeof(hs), hipMemcpyDeviceToHost, st));
                HIP_TRY(ctx, hipStreamSynchronize(st));
                relres = hs.bb > 0.0 ? std::sqrt(hs.rr / hs.bb) : std::sqrt(hs.rr);
                if (hs.done == 3 || !std::isfinite(relres)) {
                    result = set_error(ctx, RBFFD_E_NONFINITE, "implicit solve: non-finite residual at step %lld",
                                       (long long)n);
                    break;
                }
                if (hs.done == 1) {
                    conv = true;
                    iters += hs.iters + restarts;
                    break;
                }
                const int used = hs.iters + restarts;
                if (used >= maxit) {
                    iters += used;
                    break;
                }
                if (hs.done == 2) {
                    ++restarts;
                    krylov_start(0);
                } else if (maxit - used >= KRYLOV_BATCH) {
                    const int rc = batch_graph();
                    if (rc) {
                        result = rc;
                        break;
                    }
                } else {
                    for (int q = 0; q < maxit - used; ++q) iteration();
                }
                HIP_TRY(ctx, hipGetLastError());
            }
            if (result != RBFFD_OK) break;
            worst = std::max(worst, relres);
            hipLaunchKernelGGL(k_copy, g, b, 0, st, P, x, U[s][newslot]);
            if (!conv) {
                result = set_error(ctx, RBFFD_E_NOCONV,
                                   "implicit solve did not reach tol %g in %d iterations (relative residual %g) at "
                                   "step %lld", tol, maxit, relres, (long long)n);
            }
        }
        if (result != RBFFD_OK) break;
        // rotate the history: the new state is u^n from here on, then the
        // previous ones (at most order - 1 of them), then the unused slots
        int ns[4] = {0, 0, 0, 0};
        int q = 0;
        ns[q++] = newslot;
        for (int j = 0; j < std::min(have, order - 1); ++j) ns[q++] = slot[j];
        for (int idx = 0; idx < order && q < order; ++idx) {
            bool used = false;
            for (int j = 0; j < q; ++j) used = used || ns[j] == idx;
            if (!used) ns[q++] = idx;
        }
        for (int j = 0; j < order; ++j) slot[j] = ns[j];
        have = std::min(order, have + 1);
        eval_reaction(slot[0]);
    }
    for (int s = 0; s < S; ++s)
        hipLaunchKernelGGL(k_store_state<double>, g, b, 0, st, P, N, 1, U[s][slot[0]], op->perm, state + (size_t)s * N);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipStreamSynchronize(st));
    if (iters_out) *iters_out = iters;
    if (relres_out) *relres_out = worst;
    return result;
}
