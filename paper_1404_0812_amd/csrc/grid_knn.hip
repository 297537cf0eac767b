// Stencil gather (Sec. 4: each node and its n-1 nearest neighbours by
// Euclidean distance in R^3).  The paper builds a k-d tree (Sec. 4.1); here a
// uniform grid hash does the job on the GPU:
//   1. bounding box (two-pass reduction),
//   2. cell size ~ the expected stencil radius, cells keyed by the Morton code
//      of their integer coordinates,
//   3. counting sort of nodes by cell key (stable within a cell by node index),
//      which also yields the spatial order used by the sparse operator,
//   4. one wavefront per query: expanding shells of cells, candidates in LDS,
//      bitonic sort by (squared distance, index), stop once the n-1-th best
//      distance is inside the searched box.
// Squared distances are ((dx*dx + dy*dy) + dz*dz) in FP64 with contraction
// disabled, so the order (and ties, broken by node index) is exact.
#include "common.h"

#include <algorithm>
#include <cmath>
#include <vector>

#pragma clang fp contract(off)

namespace {

#ifndef KNN_CELL_SCALE
#define KNN_CELL_SCALE 1.0  // cell edge relative to the expected stencil radius
#endif
// Candidate buffer per query (entries; a power of two for the bitonic sort).
// At least need + 64 = 191 for n <= 128, so that a chunk fits after a cut.
// 512 holds the ~430 candidates of the 27 cells at n = 50 without a cut and
// keeps the LDS per query at 6 KB: the search is latency-bound, and 1024
// entries (12 KB) let half as many queries run per CU (7.5 vs 4.9 ms at
// N = 1e6, n = 50; 17.5 vs 10.9 ms at n = 101); 256 cuts every n = 101 query
// at least once (14.4 ms).
constexpr int KNN_CAP = 512;
static_assert(KNN_CAP >= 127 + 64 && (KNN_CAP & (KNN_CAP - 1)) == 0, "candidate buffer");
constexpr int MAX_BITS = 9;    // Morton bits per axis (2^27 cells at most)

__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

struct Grid {
    double lo[3];
    double h;      // cell size
    double inv_h;
    int g[3];      // cells per axis
};

__device__ __forceinline__ int cell_coord(double x, double lo, double inv_h, int g) {
    int c = (int)floor((x - lo) * inv_h);
    return c < 0 ? 0 : (c >= g ? g - 1 : c);
}

__global__ void k_bbox_partial(int64_t N, const double* __restrict__ xyz, double* __restrict__ part) {
    __shared__ double s[6][256];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int d = 0; d < 3; ++d) {
            double v = xyz[3 * i + d];
            mn[d] = fmin(mn[d], v);
            mx[d] = fmax(mx[d], v);
        }
    }
    for (int d = 0; d < 3; ++d) {
        s[d][threadIdx.x] = mn[d];
        s[3 + d][threadIdx.x] = mx[d];
    }
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            for (int d = 0; d < 3; ++d) {
                s[d][threadIdx.x] = fmin(s[d][threadIdx.x], s[d][threadIdx.x + st]);
                s[3 + d][threadIdx.x] = fmax(s[3 + d][threadIdx.x], s[3 + d][threadIdx.x + st]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void k_bbox_final(int nblk, const double* __restrict__ part, double* __restrict__ out) {
    if (threadIdx.x < 6) {
        int d = threadIdx.x;
        double v = d < 3 ? INFINITY : -INFINITY;
        for (int b = 0; b < nblk; ++b) {
            double p = part[b * 6 + d];
            v = d < 3 ? fmin(v, p) : fmax(v, p);
        }
        out[d] = v;
    }
}

__global__ void k_cell_keys(int64_t N, const double* __restrict__ xyz, Grid G, uint32_t* __restrict__ key,
                            int32_t* __restrict__ count) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    int cx = cell_coord(xyz[3 * i + 0], G.lo[0], G.inv_h, G.g[0]);
    int cy = cell_coord(xyz[3 * i + 1], G.lo[1], G.inv_h, G.g[1]);
    int cz = cell_coord(xyz[3 * i + 2], G.lo[2], G.inv_h, G.g[2]);
    uint32_t k = morton3(cx, cy, cz);
    key[i] = k;
    atomicAdd(&count[k], 1);
}

// ---- exclusive scan of int32 counts (in place into `start`, K+1 entries) ----
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

__device__ int block_exclusive_scan(int v, int* sh, int* total) {
    int lane = threadIdx.x;
    sh[lane] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
        int t = lane >= off ? sh[lane - off] : 0;
        __syncthreads();
        sh[lane] += t;
        __syncthreads();
    }
    int incl = sh[lane];
    *total = sh[SCAN_BLOCK - 1];
    __syncthreads();
    return incl - v;
}

__global__ void k_scan_tiles(int64_t K, const int32_t* __restrict__ in, int32_t* __restrict__ out,
                             int32_t* __restrict__ tile_sums) {
    __shared__ int sh[SCAN_BLOCK];
    int64_t base = blockIdx.x * (int64_t)SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int s = 0;
    for (int t = 0; t < SCAN_ITEMS; ++t) {
        int64_t i = base + t;
        v[t] = i < K ? in[i] : 0;
        s += v[t];
    }
    int tot;
    int ex = block_exclusive_scan(s, sh, &tot);
    for (int t = 0; t < SCAN_ITEMS; ++t) {
        int64_t i = base + t;
        if (i < K) out[i] = ex;
        ex += v[t];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

// single block: exclusive scan of the tile sums (sequential chunks of 256)
__global__ void k_scan_sums(int ntiles, int32_t* __restrict__ sums, int32_t* __restrict__ grand) {
    __shared__ int sh[SCAN_BLOCK];
    int carry = 0;
    for (int b = 0; b < ntiles; b += SCAN_BLOCK) {
        int i = b + threadIdx.x;
        int v = i < ntiles ? sums[i] : 0;
        int tot;
        int ex = block_exclusive_scan(v, sh, &tot);
        if (i < ntiles) sums[i] = ex + carry;
        carry += tot;
    }
    if (threadIdx.x == 0) *grand = carry;
}

__global__ void k_scan_add(int64_t K, int32_t* __restrict__ out, const int32_t* __restrict__ sums) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < K) out[i] += sums[i / SCAN_TILE];
}

__global__ void k_scatter(int64_t N, const uint32_t* __restrict__ key, const int32_t* __restrict__ start,
                          int32_t* __restrict__ fill, int32_t* __restrict__ order) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    uint32_t k = key[i];
    int pos = start[k] + atomicAdd(&fill[k], 1);
    order[pos] = (int32_t)i;
}

// Sort each cell's nodes by index (insertion sort; cells hold a few dozen nodes).
// One thread per sorted position; the first position of each cell does the work.
__global__ void k_cell_sort(int64_t N, const uint32_t* __restrict__ key, const int32_t* __restrict__ start,
                            int32_t* __restrict__ order) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= N) return;
    uint32_t k = key[order[p]];
    // `order` is being permuted within cells only, so the key of any member of
    // the cell is k; the cell begins at start[k]
    if (start[k] != p) return;
    int e = start[k + 1];
    for (int a = (int)p + 1; a < e; ++a) {
        int v = order[a];
        int b = a - 1;
        while (b >= (int)p && order[b] > v) {
            order[b + 1] = order[b];
            --b;
        }
        order[b + 1] = v;
    }
}

__global__ void k_gather_sorted(int64_t N, const double* __restrict__ xyz, const int32_t* __restrict__ order,
                                double* __restrict__ xs, double* __restrict__ ys, double* __restrict__ zs) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= N) return;
    int i = order[p];
    xs[p] = xyz[3 * (int64_t)i + 0];
    ys[p] = xyz[3 * (int64_t)i + 1];
    zs[p] = xyz[3 * (int64_t)i + 2];
}

__device__ __forceinline__ bool key_less(double da, int ia, double db, int ib) {
    return da < db || (da == db && ia < ib);
}

// Bitonic sort of the first S (power of two) entries of the wave's buffer.
// Up to 128 entries: entries lane and lane + 64 in registers, exchanged across
// the lanes (no barrier between the stages); up to 64 only the first half.
// Entries S.. of the network are padding (+inf, INT_MAX) that sorts last, and
// only the first S are written back.
__device__ __forceinline__ void lane_exchange(double& v, int& x, int pos, int j, int k) {
    const double ov = __shfl_xor(v, j, 64);
    const int ox = __shfl_xor(x, j, 64);
    const bool keep_min = ((pos & j) == 0) == ((pos & k) == 0);
    const bool take = keep_min ? key_less(ov, ox, v, x) : key_less(v, x, ov, ox);
    if (take) {
        v = ov;
        x = ox;
    }
}
__device__ void wave_bitonic(double* d2, int* id, int S) {
    const int lane = threadIdx.x;
    if (S > 64 && S <= 128) {
        double v0 = d2[lane], v1 = lane + 64 < S ? d2[lane + 64] : INFINITY;
        int x0 = id[lane], x1 = lane + 64 < S ? id[lane + 64] : 0x7fffffff;
#pragma unroll
        for (int k = 2; k <= 128; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                if (j == 64) {  // the pair (lane, lane + 64) is in one lane
                    const bool asc = (lane & k) == 0;
                    const bool sw = asc ? key_less(v1, x1, v0, x0) : key_less(v0, x0, v1, x1);
                    if (sw) {
                        const double tv = v0;
                        const int tx = x0;
                        v0 = v1; x0 = x1;
                        v1 = tv; x1 = tx;
                    }
                } else {
                    lane_exchange(v0, x0, lane, j, k);
                    lane_exchange(v1, x1, lane + 64, j, k);
                }
            }
        }
        __syncthreads();  // every lane has read its entries
        d2[lane] = v0;
        id[lane] = x0;
        if (lane + 64 < S) {
            d2[lane + 64] = v1;
            id[lane + 64] = x1;
        }
        __syncthreads();
        return;
    }
    if (S <= 64) {
        double v = lane < S ? d2[lane] : INFINITY;
        int x = lane < S ? id[lane] : 0x7fffffff;
#pragma unroll
        for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                const double ov = __shfl_xor(v, j, 64);
                const int ox = __shfl_xor(x, j, 64);
                const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
                const bool take = keep_min ? key_less(ov, ox, v, x) : key_less(v, x, ov, ox);
                if (take) {
                    v = ov;
                    x = ox;
                }
            }
        }
        __syncthreads();  // every lane has read its entry
        if (lane < S) {
            d2[lane] = v;
            id[lane] = x;
        }
        __syncthreads();
        return;
    }
    for (int k = 2; k <= S; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < S; t += 64) {
                int u = t ^ j;
                if (u > t) {
                    double a = d2[t], b = d2[u];
                    int ia = id[t], ib = id[u];
                    bool up = (t & k) == 0;
                    bool sw = up ? key_less(b, ib, a, ia) : key_less(a, ia, b, ib);
                    if (sw) {
                        d2[t] = b;
                        d2[u] = a;
                        id[t] = ib;
                        id[u] = ia;
                    }
                }
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Drop candidates that cannot be among the `need` nearest before the sort.
// Entry t belongs to group (t / 64) % NG of lane t % 64; each of the 64 NG
// groups' minimum is a distance attained by a distinct candidate, so the
// need-th smallest of those minima (need <= 64 NG) bounds the need-th smallest
// distance from above.  Entries with a larger distance are discarded (ties
// with the bound are kept) and the rest compacted to the front.  Returns the
// new count.
template <int NG>
__device__ int prefilter(double* cd, int* cid, int cnt, int need) {
    const int lane = threadIdx.x;
    double lm[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) lm[g] = INFINITY;
    for (int b = 0; b < cnt; b += 64 * NG) {
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            const int t = b + 64 * g + lane;
            if (t < cnt) lm[g] = fmin(lm[g], cd[t]);
        }
    }
    double bound = INFINITY;
    if constexpr (NG == 1) {
        // the need-th smallest of the 64 minima: bitonic sort across the lanes
        double v = lm[0];
#pragma unroll
        for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                const double o = __shfl_xor(v, j, 64);
                const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
                v = keep_min ? fmin(v, o) : fmax(v, o);
            }
        }
        bound = __shfl(v, need - 1, 64);
    } else {
        static_assert(NG == 2, "64 or 128 groups");
        // 128 minima, lm[0] and lm[1] of every lane: the same sort, two per lane
        double v0 = lm[0], v1 = lm[1];
#pragma unroll
        for (int k = 2; k <= 128; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                if (j == 64) {  // the pair (lane, lane + 64) is in one lane
                    const bool asc = (lane & k) == 0;
                    const double lo = fmin(v0, v1), hi = fmax(v0, v1);
                    v0 = asc ? lo : hi;
                    v1 = asc ? hi : lo;
                } else {
                    const double o0 = __shfl_xor(v0, j, 64), o1 = __shfl_xor(v1, j, 64);
                    const bool m0 = ((lane & j) == 0) == ((lane & k) == 0);
                    const bool m1 = (((lane + 64) & j) == 0) == (((lane + 64) & k) == 0);
                    v0 = m0 ? fmin(v0, o0) : fmax(v0, o0);
                    v1 = m1 ? fmin(v1, o1) : fmax(v1, o1);
                }
            }
        }
        bound = need - 1 < 64 ? __shfl(v0, need - 1, 64) : __shfl(v1, need - 1 - 64, 64);
    }
    int kept = 0;
    for (int b = 0; b < cnt; b += 64) {
        const int t = b + lane;
        double d = INFINITY;
        int id = 0;
        bool keep = false;
        if (t < cnt) {
            d = cd[t];
            id = cid[t];
            keep = d <= bound;
        }
        const uint64_t m = __ballot(keep);
        __syncthreads();  // every lane has read its entry of this block
        if (keep) {
            const int pos = kept + __popcll(m & ((1ull << lane) - 1ull));  // pos <= t: earlier blocks are done
            cd[pos] = d;
            cid[pos] = id;
        }
        kept += __popcll(m);
        __syncthreads();
    }
    return kept;
}

// One 64-lane workgroup per query position p (spatial order).
__global__ __launch_bounds__(64) void k_knn(int64_t N, int n, Grid G, const double* __restrict__ xs,
                                             const double* __restrict__ ys, const double* __restrict__ zs,
                                             const int32_t* __restrict__ order, const int32_t* __restrict__ start,
                                             int32_t* __restrict__ idx_out) {
    __shared__ double cd[KNN_CAP];
    __shared__ int cid[KNN_CAP];
    const int lane = threadIdx.x;
    const int64_t p = blockIdx.x;
    if (p >= N) return;
    const double qx = xs[p], qy = ys[p], qz = zs[p];
    const int q = order[p];
    const int cx = cell_coord(qx, G.lo[0], G.inv_h, G.g[0]);
    const int cy = cell_coord(qy, G.lo[1], G.inv_h, G.g[1]);
    const int cz = cell_coord(qz, G.lo[2], G.inv_h, G.g[2]);
    const int need = n - 1;  // neighbours besides the centre
    int cnt = 0;
    double bound = INFINITY;  // current need-th best squared distance once known
    bool done = need == 0;
    // One chunk of up to 64 candidates (point index j in cell order, valid
    // when in range): squared distances, those within the bound appended to
    // the LDS list; on overflow the list is cut to its best `need` first.
    auto consider = [&](int j, bool valid) {
        double d2 = INFINITY;
        int oj = -1;
        bool ok = false;
        if (valid) {
            double ddx = xs[j] - qx, ddy = ys[j] - qy, ddz = zs[j] - qz;
            d2 = (ddx * ddx + ddy * ddy) + ddz * ddz;
            oj = order[j];
            ok = (oj != q) && (d2 <= bound);
        }
        uint64_t m = __ballot(ok);
        int add = __popcll(m);
        if (add == 0) return;
        if (cnt + add > KNN_CAP) {
            // keep only the best `need` candidates
            int S = next_pow2(cnt);
            for (int t = cnt + lane; t < S; t += 64) {
                cd[t] = INFINITY;
                cid[t] = 0x7fffffff;
            }
            __syncthreads();
            wave_bitonic(cd, cid, S);
            cnt = need;
            bound = cd[need - 1];
            ok = ok && (d2 <= bound);
            m = __ballot(ok);
            add = __popcll(m);
        }
        if (ok) {
            int pos = cnt + __popcll(m & ((1ull << lane) - 1ull));
            cd[pos] = d2;
            cid[pos] = oj;
        }
        cnt += add;
        __syncthreads();
    };
    // After the shells up to R: sort, bound, and stop once the searched box
    // provably holds the `need` nearest (or covers the whole grid).
    auto settle = [&](int R) {
        bool covers = (cx - R <= 0) && (cy - R <= 0) && (cz - R <= 0) && (cx + R >= G.g[0] - 1) &&
                      (cy + R >= G.g[1] - 1) && (cz + R >= G.g[2] - 1);
        if (cnt >= need) {
            if (need <= 64 && cnt > 128) cnt = prefilter<1>(cd, cid, cnt, need);
            else if (need <= 128 && cnt > 256) cnt = prefilter<2>(cd, cid, cnt, need);
            // a second pass over the survivors (groups of one or two) usually
            // leaves at most 64 (128) to sort
            if (need <= 64 && cnt > 64) cnt = prefilter<1>(cd, cid, cnt, need);
            else if (need <= 128 && cnt > 128) cnt = prefilter<2>(cd, cid, cnt, need);
            int S = next_pow2(cnt);
            for (int t = cnt + lane; t < S; t += 64) {
                cd[t] = INFINITY;
                cid[t] = 0x7fffffff;
            }
            __syncthreads();
            wave_bitonic(cd, cid, S);
            cnt = need;
            bound = cd[need - 1];
            double r_safe = INFINITY;
            const double q3[3] = {qx, qy, qz};
            const int c3[3] = {cx, cy, cz};
            for (int d = 0; d < 3; ++d) {
                if (c3[d] - R > 0) r_safe = fmin(r_safe, q3[d] - (G.lo[d] + (c3[d] - R) * G.h));
                if (c3[d] + R < G.g[d] - 1) r_safe = fmin(r_safe, (G.lo[d] + (c3[d] + R + 1) * G.h) - q3[d]);
            }
            if (covers || (r_safe > 0 && bound < r_safe * r_safe * (1.0 - 1e-12))) done = true;
        } else if (covers) {
            done = true;  // cannot happen when n <= N
        }
    };
    if (!done) {
        // R = 0 and 1 at once: the 27 cells of the 3 x 3 x 3 block, their point
        // ranges read by 27 lanes together and swept as one list (in place of
        // 27 sequential cell visits, each waiting on its range)
        int s0 = 0, c0 = 0;
        if (lane < 27) {
            const int ix = cx + lane % 3 - 1, iy = cy + (lane / 3) % 3 - 1, iz = cz + lane / 9 - 1;
            if (ix >= 0 && ix < G.g[0] && iy >= 0 && iy < G.g[1] && iz >= 0 && iz < G.g[2]) {
                const uint32_t k = morton3(ix, iy, iz);
                s0 = start[k];
                c0 = start[k + 1] - s0;
            }
        }
        // inclusive prefix sum of the counts over the wave
        int incl = c0;
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        const int total = __shfl(incl, 63, 64);
        __shared__ int cstart[27], cexcl[28];
        if (lane < 27) {
            cstart[lane] = s0;
            cexcl[lane] = incl - c0;
        }
        if (lane == 0) cexcl[27] = total;
        __syncthreads();
        for (int b = 0; b < total; b += 64) {
            const int t = b + lane;
            int j = 0;
            if (t < total) {
                int lo = 0, hi = 26;  // the cell whose exclusive prefix is the last <= t
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (cexcl[mid] <= t) lo = mid;
                    else hi = mid - 1;
                }
                j = cstart[lo] + (t - cexcl[lo]);
            }
            consider(j, t < total);
        }
        settle(1);
    }
    for (int R = 2; !done; ++R) {
        // the shell of cells at Chebyshev distance R from the query's cell
        for (int dx = -R; dx <= R; ++dx) {
            int ix = cx + dx;
            if (ix < 0 || ix >= G.g[0]) continue;
            for (int dy = -R; dy <= R; ++dy) {
                int iy = cy + dy;
                if (iy < 0 || iy >= G.g[1]) continue;
                bool edge_xy = (dx == -R || dx == R || dy == -R || dy == R);
                for (int dz = -R; dz <= R; dz += (edge_xy ? 1 : 2 * R)) {
                    int iz = cz + dz;
                    if (iz >= 0 && iz < G.g[2]) {
                        uint32_t k = morton3(ix, iy, iz);
                        int s = start[k], e = start[k + 1];
                        for (int b = s; b < e; b += 64) consider(b + lane, b + lane < e);
                    }
                }
            }
        }
        settle(R);
    }
    int32_t* row = idx_out + (int64_t)q * n;
    if (lane == 0) row[0] = q;
    for (int t = lane; t < need; t += 64) row[1 + t] = cid[t];
}

}  // namespace

int knn_internal(rbffd_ctx ctx, int64_t N, const double* xyz, int32_t n, int32_t* idx, int32_t* perm) {
    hipStream_t st = ctx->stream;
    const int nblk_bbox = 256;
    // bbox first (small scratch)
    int rc = ensure_scratch(ctx, nblk_bbox * 6 * sizeof(double) + 64);
    if (rc) return rc;
    double* part = (double*)ctx->scratch;
    double* bb = part + nblk_bbox * 6;
    hipLaunchKernelGGL(k_bbox_partial, dim3(nblk_bbox), dim3(256), 0, st, N, xyz, part);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, st, nblk_bbox, part, bb);
    double hb[6];
    HIP_TRY(ctx, hipMemcpyAsync(hb, bb, sizeof(hb), hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    for (int d = 0; d < 6; ++d)
        if (!std::isfinite(hb[d])) return set_error(ctx, RBFFD_E_ARG, "non-finite node coordinates");
    double ext[3] = {hb[3] - hb[0], hb[4] - hb[1], hb[5] - hb[2]};
    double emax = std::max(ext[0], std::max(ext[1], ext[2]));
    if (emax <= 0) emax = 1.0;
    // surface-area proxy: half the bounding-box surface; cell ~ expected stencil radius
    double area = ext[0] * ext[1] + ext[1] * ext[2] + ext[0] * ext[2];
    if (area <= 0) area = emax * emax;
    double h = KNN_CELL_SCALE * std::sqrt(std::max(n, 8) * area / (M_PI * (double)N));
    if (!(h > 0)) h = emax;
    h = std::max(h, emax / (double)(1 << MAX_BITS));
    Grid G;
    for (int d = 0; d < 3; ++d) {
        G.lo[d] = hb[d];
        G.g[d] = std::max(1, std::min(1 << MAX_BITS, (int)std::ceil(ext[d] / h)));
    }
    // the last cell must contain the maximum coordinate
    for (int d = 0; d < 3; ++d)
        while (G.g[d] < (1 << MAX_BITS) && G.lo[d] + G.g[d] * h <= hb[3 + d]) G.g[d]++;
    G.h = h;
    G.inv_h = 1.0 / h;
    int bits = 0;
    int gmax = std::max(G.g[0], std::max(G.g[1], G.g[2]));
    while ((1 << bits) < gmax) ++bits;
    const int64_t K = (int64_t)1 << (3 * bits);
    const int64_t ntiles = (K + 1 + SCAN_TILE - 1) / SCAN_TILE;
    // scratch layout
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    size_t o_key = take(N * sizeof(uint32_t));
    size_t o_cnt = take((K + 1) * sizeof(int32_t));
    size_t o_start = take((K + 1) * sizeof(int32_t));
    size_t o_fill = take((K + 1) * sizeof(int32_t));
    size_t o_sums = take((ntiles + 1) * sizeof(int32_t));
    size_t o_order = take(N * sizeof(int32_t));
    size_t o_xs = take(N * sizeof(double));
    size_t o_ys = take(N * sizeof(double));
    size_t o_zs = take(N * sizeof(double));
    rc = ensure_scratch(ctx, off);
    if (rc) return rc;
    char* base = (char*)ctx->scratch;
    uint32_t* key = (uint32_t*)(base + o_key);
    int32_t* cnt = (int32_t*)(base + o_cnt);
    int32_t* start = (int32_t*)(base + o_start);
    int32_t* fill = (int32_t*)(base + o_fill);
    int32_t* sums = (int32_t*)(base + o_sums);
    int32_t* order = perm ? perm : (int32_t*)(base + o_order);
    double* xs = (double*)(base + o_xs);
    double* ys = (double*)(base + o_ys);
    double* zs = (double*)(base + o_zs);

    HIP_TRY(ctx, hipMemsetAsync(cnt, 0, (K + 1) * sizeof(int32_t), st));
    HIP_TRY(ctx, hipMemsetAsync(fill, 0, (K + 1) * sizeof(int32_t), st));
    const int B = 256;
    int gN = (int)((N + B - 1) / B);
    hipLaunchKernelGGL(k_cell_keys, dim3(gN), dim3(B), 0, st, N, xyz, G, key, cnt);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(SCAN_BLOCK), 0, st, K + 1, cnt, start, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_BLOCK), 0, st, (int)ntiles, sums, sums + ntiles);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((K + 1 + B - 1) / B)), dim3(B), 0, st, K + 1, start, sums);
    hipLaunchKernelGGL(k_scatter, dim3(gN), dim3(B), 0, st, N, key, start, fill, order);
    hipLaunchKernelGGL(k_cell_sort, dim3(gN), dim3(B), 0, st, N, key, start, order);
    hipLaunchKernelGGL(k_gather_sorted, dim3(gN), dim3(B), 0, st, N, xyz, order, xs, ys, zs);
    if (idx) {
        hipLaunchKernelGGL(k_knn, dim3((unsigned)N), dim3(64), 0, st, N, n, G, xs, ys, zs, order, start, idx);
    }
    HIP_TRY(ctx, hipGetLastError());
    return RBFFD_OK;
}

extern "C" int rbffd_knn(rbffd_ctx ctx, int64_t N, const double* xyz, int32_t n, int32_t* idx, int32_t* perm) {
    if (!ctx) return RBFFD_E_ARG;
    if (N < 0 || N > 0x7fffffffLL) return set_error(ctx, RBFFD_E_ARG, "N out of range");
    if (N == 0) return RBFFD_OK;
    if (n < 1 || n > 128 || n > N) return set_error(ctx, RBFFD_E_ARG, "stencil size n=%d invalid for N=%lld", n, (long long)N);
    if (!xyz || (!idx && !perm)) return set_error(ctx, RBFFD_E_ARG, "null pointer");
    return knn_internal(ctx, N, xyz, n, idx, perm);
}
