// Learned shape parameter: a 128 -> 128 -> 128 -> 1 ReLU regressor of
// y = log(eps * rho) from the stencil's tangent-plane offsets, with BF16
// matrix-core (MFMA) forward and backward passes and FP32 Adam.
//
// The target is the per-stencil eps that the bisection of Sec. 5
// (eq. target_cond) finds; the network only proposes eps: the weights kernel
// checks kappa_2 at the proposal and falls back to bisection outside the band.
//
// Features (per stencil, centre x_1, unit normal nu, neighbours x_2..x_n):
// offsets d_j = x_j - x_1 in the canonical tangent frame tau_1 ~ Pi (x_2 - x_1)
// (the nearest neighbour), tau_2 = nu x tau_1, scaled by rho = max_j |d_j|:
// f[2(j-2)] = d_j . tau_1 / rho, f[2(j-2)+1] = d_j . tau_2 / rho, zero-padded
// to 128 entries, stored BF16.
//
// Parameters (FP32, this order): W1[128][128] (out, in), b1[128],
// W2[128][128], b2[128], w3[128], b3.  BF16 copies of W1, W2 and the
// transpose of W2 feed the MFMAs.
//
// Every GEMM below is a sum of 16 x 16 output tiles D[r][c] = sum_k A[r][k]
// B[c][k] with both operands K-contiguous; v_mfma_f32_16x16x32_bf16 takes, in
// lane l, A[l%16][8(l/16) .. +7] and B[l%16][8(l/16) .. +7] and returns
// D[4(l/16) + i][l%16], i = 0..3.
#include "common.h"

#include <cmath>

namespace {

constexpr int F = RBFFD_MLP_IN;       // 128
constexpr int H = RBFFD_MLP_HIDDEN;   // 128
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + H * F;
constexpr int OFF_W2 = OFF_B1 + H;
constexpr int OFF_B2 = OFF_W2 + H * H;
constexpr int OFF_W3 = OFF_B2 + H;
constexpr int OFF_B3 = OFF_W3 + H;
static_assert(OFF_B3 + 1 == RBFFD_MLP_PARAMS, "parameter layout");

constexpr int TB = 64;        // samples per workgroup tile
constexpr int WG = 256;       // 4 waves

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// float -> bf16, round to nearest even (NaN -> quiet NaN)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// One 16x16 output tile over K (multiple of 32): A rows at a (stride lda), B rows at b (stride ldb).
__device__ __forceinline__ void mma_tile(const uint16_t* a, int lda, const uint16_t* b, int ldb, int K,
                                         floatx4& acc) {
    const int l = threadIdx.x & 63;
    const int r = l & 15, kq = (l >> 4) * 8;
    for (int k0 = 0; k0 < K; k0 += 32) {
        const bf16x8 av = *reinterpret_cast<const bf16x8*>(a + (size_t)r * lda + k0 + kq);
        const bf16x8 bv = *reinterpret_cast<const bf16x8*>(b + (size_t)r * ldb + k0 + kq);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    }
}

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

struct Bf16Params {
    const uint16_t* W1;   // [H][F]
    const uint16_t* W2;   // [H][H]
    const uint16_t* W2T;  // [H][H] transposed
    const float* P;       // FP32 parameters (biases, w3, b3)
};

// Forward (and, when TRAIN, backward) over one tile of TB samples.
// TRAIN false: forward only, writes y.  TRAIN true: forward + backward,
// accumulates gradients into grad (FP32, atomics) and the summed squared
// error into loss.  Sample s of the tile is row base + s of x, or a hashed
// index when sampling.  The forward-only form keeps only the two row-major
// tiles in LDS (32 KB instead of 128 KB: five workgroups per CU instead of
// one); its arithmetic is the same, so y is the same bit for bit.
template <bool TRAIN>
__global__ __launch_bounds__(WG) void k_mlp(int64_t count, Bf16Params prm, const uint16_t* __restrict__ x,
                                            const float* __restrict__ target, float* __restrict__ y,
                                            float* __restrict__ grad, float* __restrict__ loss, float gscale,
                                            uint64_t seed, int64_t step) {
    __shared__ __attribute__((aligned(16))) uint16_t Xs[TB * F];   // [b][k]
    __shared__ __attribute__((aligned(16))) uint16_t H1s[TB * H];  // [b][i]
    // backward only
    __shared__ __attribute__((aligned(16))) uint16_t XT[TRAIN ? F * TB : 8];   // [k][b]
    __shared__ __attribute__((aligned(16))) uint16_t H1T[TRAIN ? H * TB : 8];  // [i][b]
    __shared__ __attribute__((aligned(16))) uint16_t H2s[TRAIN ? TB * H : 8];  // [b][o]
    __shared__ __attribute__((aligned(16))) uint16_t G2s[TRAIN ? TB * H : 8];  // dH2 [b][o]
    __shared__ __attribute__((aligned(16))) uint16_t G2T[TRAIN ? H * TB : 8];  // dH2 [o][b]
    __shared__ __attribute__((aligned(16))) uint16_t G1T[TRAIN ? H * TB : 8];  // dH1 [i][b]
    __shared__ float ys[TB], dys[TB];
    __shared__ int64_t rows[TB];
    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
    const int64_t base = (int64_t)blockIdx.x * TB;
    if (tid < TB) {
        int64_t rr = base + tid;
        if (seed != 0) rr = (int64_t)(mix64(seed ^ mix64((uint64_t)step * 0x9e3779b97f4a7c15ull + (uint64_t)rr)) %
                                      (uint64_t)count);
        rows[tid] = rr;
    }
    __syncthreads();
    // ---- load the input tile (zeros beyond count)
    for (int e = tid; e < TB * F / 8; e += WG) {
        const int b = e / (F / 8), k8 = (e % (F / 8)) * 8;
        const int64_t rr = rows[b];
        uint4 v = make_uint4(0, 0, 0, 0);
        if (rr < count) v = *reinterpret_cast<const uint4*>(x + rr * F + k8);
        *reinterpret_cast<uint4*>(Xs + b * F + k8) = v;
        if constexpr (TRAIN) {
            const uint16_t* hv = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
            for (int t = 0; t < 8; ++t) XT[(k8 + t) * TB + b] = hv[t];
        }
    }
    __syncthreads();
    const int r0 = wv * 16;              // this wave's 16 sample rows
    const int col = l & 15, rq = (l >> 4) * 4;
    // ---- layer 1: H1 = relu(X W1^T + b1)
    for (int ct = 0; ct < H / 16; ++ct) {
        floatx4 acc = {0, 0, 0, 0};
        mma_tile(Xs + r0 * F, F, prm.W1 + ct * 16 * F, F, F, acc);
        const int o = ct * 16 + col;
        const float bb = prm.P[OFF_B1 + o];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int b = r0 + rq + i;
            const uint16_t h = f2bf(fmaxf(acc[i] + bb, 0.0f));
            H1s[b * H + o] = h;
            if constexpr (TRAIN) H1T[o * TB + b] = h;
        }
    }
    __syncthreads();
    // ---- layer 2: H2 = relu(H1 W2^T + b2); layer 3: y = H2 . w3 + b3
    float part[4] = {0, 0, 0, 0};
    for (int ct = 0; ct < H / 16; ++ct) {
        floatx4 acc = {0, 0, 0, 0};
        mma_tile(H1s + r0 * H, H, prm.W2 + ct * 16 * H, H, H, acc);
        const int o = ct * 16 + col;
        const float bb = prm.P[OFF_B2 + o], w3 = prm.P[OFF_W3 + o];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int b = r0 + rq + i;
            const uint16_t h = f2bf(fmaxf(acc[i] + bb, 0.0f));
            if constexpr (TRAIN) H2s[b * H + o] = h;
            part[i] = fmaf(bf2f(h), w3, part[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int m = 1; m < 16; m <<= 1) part[i] += __shfl_xor(part[i], m, 64);
    }
    if (col == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) ys[r0 + rq + i] = part[i] + prm.P[OFF_B3];
    }
    __syncthreads();
    if constexpr (!TRAIN) {
        if (tid < TB && base + tid < count) y[base + tid] = ys[tid];
        return;
    }
    // ---- backward: L = gscale * sum_b (y_b - t_b)^2
    if (tid < TB) {
        const int64_t rr = rows[tid];
        float d = 0.0f;
        if (rr < count) {
            const float e = ys[tid] - target[rr];
            d = 2.0f * gscale * e;
            atomicAdd(loss, gscale * e * e);
        }
        dys[tid] = d;
    }
    __syncthreads();
    // dW3, db3 (one thread per output unit), dH2 = dy w3 [H2 > 0]
    if (tid < H) {
        float s = 0.0f;
        for (int b = 0; b < TB; ++b) s = fmaf(dys[b], bf2f(H2s[b * H + tid]), s);
        atomicAdd(grad + OFF_W3 + tid, s);
    }
    if (tid == H) {
        float s = 0.0f;
        for (int b = 0; b < TB; ++b) s += dys[b];
        atomicAdd(grad + OFF_B3, s);
    }
    for (int e = tid; e < TB * H; e += WG) {
        const int b = e / H, o = e % H;
        const float g = H2s[e] != 0 ? dys[b] * prm.P[OFF_W3 + o] : 0.0f;
        const uint16_t gh = f2bf(g);
        G2s[e] = gh;
        G2T[o * TB + b] = gh;
    }
    __syncthreads();
    // db2 = sum_b dH2
    if (tid < H) {
        float s = 0.0f;
        for (int b = 0; b < TB; ++b) s += bf2f(G2T[tid * TB + b]);
        atomicAdd(grad + OFF_B2 + tid, s);
    }
    // dW2[o][i] = sum_b dH2[b][o] H1[b][i]: wave w owns output tile rows 2w, 2w+1
    for (int rt = 2 * wv; rt < 2 * wv + 2; ++rt) {
        for (int ct = 0; ct < H / 16; ++ct) {
            floatx4 acc = {0, 0, 0, 0};
            mma_tile(G2T + rt * 16 * TB, TB, H1T + ct * 16 * TB, TB, TB, acc);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                atomicAdd(grad + OFF_W2 + (rt * 16 + rq + i) * H + ct * 16 + col, acc[i]);
        }
    }
    // dH1 = (dH2 W2) [H1 > 0]  (B operand: W2^T rows)
    for (int ct = 0; ct < H / 16; ++ct) {
        floatx4 acc = {0, 0, 0, 0};
        mma_tile(G2s + r0 * H, H, prm.W2T + ct * 16 * H, H, H, acc);
        const int i_ = ct * 16 + col;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int b = r0 + rq + i;
            const float g = H1s[b * H + i_] != 0 ? acc[i] : 0.0f;
            G1T[i_ * TB + b] = f2bf(g);
        }
    }
    __syncthreads();
    if (tid < H) {
        float s = 0.0f;
        for (int b = 0; b < TB; ++b) s += bf2f(G1T[tid * TB + b]);
        atomicAdd(grad + OFF_B1 + tid, s);
    }
    // dW1[i][k] = sum_b dH1[b][i] X[b][k]
    for (int rt = 2 * wv; rt < 2 * wv + 2; ++rt) {
        for (int ct = 0; ct < F / 16; ++ct) {
            floatx4 acc = {0, 0, 0, 0};
            mma_tile(G1T + rt * 16 * TB, TB, XT + ct * 16 * TB, TB, TB, acc);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                atomicAdd(grad + OFF_W1 + (rt * 16 + rq + i) * F + ct * 16 + col, acc[i]);
        }
    }
}

// BF16 copies of W1, W2 and W2^T from the FP32 parameters
__global__ void k_mlp_convert(const float* __restrict__ P, uint16_t* __restrict__ W1, uint16_t* __restrict__ W2,
                              uint16_t* __restrict__ W2T) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < H * F) W1[e] = f2bf(P[OFF_W1 + e]);
    if (e < H * H) {
        const uint16_t v = f2bf(P[OFF_W2 + e]);
        W2[e] = v;
        W2T[(e % H) * H + e / H] = v;
    }
}

// Adam on the FP32 parameters; clears the gradient; refreshes the BF16 copies.
__global__ void k_adam(float* __restrict__ P, float* __restrict__ M, float* __restrict__ V, float* __restrict__ G,
                       float lr, float b1, float b2, float eps, float c1, float c2, uint16_t* __restrict__ W1,
                       uint16_t* __restrict__ W2, uint16_t* __restrict__ W2T) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= RBFFD_MLP_PARAMS) return;
    const float g = G[e];
    const float m = b1 * M[e] + (1.0f - b1) * g;
    const float v = b2 * V[e] + (1.0f - b2) * g * g;
    M[e] = m;
    V[e] = v;
    const float p = P[e] - lr * (m * c1) / (sqrtf(v * c2) + eps);
    P[e] = p;
    G[e] = 0.0f;
    if (e < OFF_B1) W1[e - OFF_W1] = f2bf(p);
    if (e >= OFF_W2 && e < OFF_B2) {
        const int q = e - OFF_W2;
        const uint16_t h = f2bf(p);
        W2[q] = h;
        W2T[(q % H) * H + q / H] = h;
    }
}

// Features: one wavefront per FEAT_SPW consecutive stencils, lane j = stencil
// slot j (n <= 64; 2 (n - 1) <= 126 entries of the F = 128, the rest zero).  The loads of all of them are issued before any is used (stencils
// beyond N read stencil N - 1 and write nothing), so each wavefront has
// FEAT_SPW round trips to memory in flight instead of one.
constexpr int FEAT_SPW = 4;
__global__ __launch_bounds__(64) void k_features(int64_t N, int n, const double* __restrict__ xyz,
                                                 const double* __restrict__ nrm, const int32_t* __restrict__ idx,
                                                 uint16_t* __restrict__ feat, double* __restrict__ rho_out) {
    __shared__ double t1s[FEAT_SPW][3];
    const int l = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * FEAT_SPW;
    double dx[FEAT_SPW], dy[FEAT_SPW], dz[FEAT_SPW], nx[FEAT_SPW], ny[FEAT_SPW], nz[FEAT_SPW], rho[FEAT_SPW];
    // indices outside [0, N) read node 0 and make rho NaN (the proposal is then
    // unusable and the weights call flags the stencil)
#pragma unroll
    for (int u = 0; u < FEAT_SPW; ++u) {
        const int64_t s = s0 + u < N ? s0 + u : N - 1;
        int c = idx[s * n];
        bool bad = c < 0 || c >= N;
        if (bad) c = 0;
        int j = l < n ? idx[s * n + l] : c;
        if (j < 0 || j >= N) {
            bad = true;
            j = 0;
        }
        const double cx = xyz[3 * (int64_t)c], cy = xyz[3 * (int64_t)c + 1], cz = xyz[3 * (int64_t)c + 2];
        const double px = xyz[3 * (int64_t)j], py = xyz[3 * (int64_t)j + 1], pz = xyz[3 * (int64_t)j + 2];
        dx[u] = l < n ? px - cx : 0.0;
        dy[u] = l < n ? py - cy : 0.0;
        dz[u] = l < n ? pz - cz : 0.0;
        nx[u] = nrm[3 * (int64_t)c];
        ny[u] = nrm[3 * (int64_t)c + 1];
        nz[u] = nrm[3 * (int64_t)c + 2];
        double r2 = (dx[u] * dx[u] + dy[u] * dy[u]) + dz[u] * dz[u];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) r2 = fmax(r2, __shfl_xor(r2, o, 64));
        const bool any_bad = __ballot(bad) != 0;
        rho[u] = any_bad ? NAN : sqrt(r2);
        const double nn = sqrt(nx[u] * nx[u] + ny[u] * ny[u] + nz[u] * nz[u]);
        nx[u] /= nn; ny[u] /= nn; nz[u] /= nn;
        if (l == 1) {
            // tau_1: the nearest neighbour's offset projected on the tangent plane
            const double dn = dx[u] * nx[u] + dy[u] * ny[u] + dz[u] * nz[u];
            double tx = dx[u] - dn * nx[u], ty = dy[u] - dn * ny[u], tz = dz[u] - dn * nz[u];
            double tn = sqrt(tx * tx + ty * ty + tz * tz);
            if (!(tn > 1e-12 * rho[u])) {  // degenerate: any tangent direction
                const bool ax = fabs(nx[u]) < 0.9;
                tx = ax ? 0.0 : -nz[u]; ty = ax ? nz[u] : 0.0; tz = ax ? -ny[u] : nx[u];
                tn = sqrt(tx * tx + ty * ty + tz * tz);
            }
            t1s[u][0] = tx / tn; t1s[u][1] = ty / tn; t1s[u][2] = tz / tn;
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < FEAT_SPW; ++u) {
        const int64_t s = s0 + u;
        if (s >= N) break;
        const double ax = t1s[u][0], ay = t1s[u][1], az = t1s[u][2];
        const double bx = ny[u] * az - nz[u] * ay, by = nz[u] * ax - nx[u] * az, bz = nx[u] * ay - ny[u] * ax;
        uint16_t* f = feat + s * F;
        if (l >= 1 && l < n) {
            const float sv = (float)((dx[u] * ax + dy[u] * ay + dz[u] * az) / rho[u]);
            const float tv = (float)((dx[u] * bx + dy[u] * by + dz[u] * bz) / rho[u]);
            f[2 * (l - 1)] = f2bf(sv);
            f[2 * (l - 1) + 1] = f2bf(tv);
        }
        for (int k = 2 * (n - 1) + l; k < F; k += 64) f[k] = 0;
        if (l == 0 && rho_out) rho_out[s] = rho[u];
    }
}

__global__ void k_eps_from_y(int64_t N, const float* __restrict__ y, const double* __restrict__ rho,
                             double* __restrict__ eps) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s < N) eps[s] = exp((double)y[s]) / rho[s];
}

struct MlpScratch {
    uint16_t *W1, *W2, *W2T;
};

int mlp_scratch(rbffd_ctx ctx, size_t extra, MlpScratch& ms, char** extra_ptr) {
    const size_t wbytes = (size_t)(H * F + 2 * H * H) * sizeof(uint16_t);
    int rc = ensure_scratch(ctx, wbytes + extra + 512);
    if (rc) return rc;
    char* base = (char*)ctx->scratch;
    ms.W1 = (uint16_t*)base;
    ms.W2 = ms.W1 + H * F;
    ms.W2T = ms.W2 + H * H;
    if (extra_ptr) *extra_ptr = base + ((wbytes + 255) & ~(size_t)255);
    return RBFFD_OK;
}

void convert(hipStream_t st, const float* P, const MlpScratch& ms) {
    hipLaunchKernelGGL(k_mlp_convert, dim3((H * F + 255) / 256), dim3(256), 0, st, P, ms.W1, ms.W2, ms.W2T);
}

}  // namespace

extern "C" int rbffd_mlp_features(rbffd_ctx ctx, int64_t N, const double* xyz, const double* nrm,
                                  const int32_t* idx, int32_t n, uint16_t* feats, double* rho) {
    if (!ctx) return RBFFD_E_ARG;
    if (N < 0) return set_error(ctx, RBFFD_E_ARG, "N < 0");
    if (N == 0) return RBFFD_OK;
    if (n < 2 || n > 64) return set_error(ctx, RBFFD_E_ARG, "features need 2 <= n <= 64 (one lane per slot)");
    if (!xyz || !nrm || !idx || !feats) return set_error(ctx, RBFFD_E_ARG, "null pointer");
    hipLaunchKernelGGL(k_features, dim3((unsigned)((N + FEAT_SPW - 1) / FEAT_SPW)), dim3(64), 0, ctx->stream, N, n,
                       xyz, nrm, idx, feats, rho);
    HIP_TRY(ctx, hipGetLastError());
    return RBFFD_OK;
}

extern "C" int rbffd_mlp_forward(rbffd_ctx ctx, const float* params, int64_t B, const uint16_t* feats, float* y) {
    if (!ctx) return RBFFD_E_ARG;
    if (B < 0) return set_error(ctx, RBFFD_E_ARG, "B < 0");
    if (B == 0) return RBFFD_OK;
    if (!params || !feats || !y) return set_error(ctx, RBFFD_E_ARG, "null pointer");
    MlpScratch ms;
    int rc = mlp_scratch(ctx, 0, ms, nullptr);
    if (rc) return rc;
    convert(ctx->stream, params, ms);
    Bf16Params p{ms.W1, ms.W2, ms.W2T, params};
    hipLaunchKernelGGL(k_mlp<false>, dim3((unsigned)((B + TB - 1) / TB)), dim3(WG), 0, ctx->stream, B, p, feats,
                       nullptr, y, nullptr, nullptr, 0.0f, (uint64_t)0, (int64_t)0);
    HIP_TRY(ctx, hipGetLastError());
    return RBFFD_OK;
}

extern "C" int rbffd_mlp_grad(rbffd_ctx ctx, const float* params, int64_t B, const uint16_t* feats,
                              const float* target, float* grad, float* loss) {
    if (!ctx) return RBFFD_E_ARG;
    if (B <= 0) return set_error(ctx, RBFFD_E_ARG, "B must be > 0");
    if (!params || !feats || !target || !grad || !loss) return set_error(ctx, RBFFD_E_ARG, "null pointer");
    MlpScratch ms;
    int rc = mlp_scratch(ctx, 0, ms, nullptr);
    if (rc) return rc;
    convert(ctx->stream, params, ms);
    HIP_TRY(ctx, hipMemsetAsync(grad, 0, RBFFD_MLP_PARAMS * sizeof(float), ctx->stream));
    HIP_TRY(ctx, hipMemsetAsync(loss, 0, sizeof(float), ctx->stream));
    Bf16Params p{ms.W1, ms.W2, ms.W2T, params};
    hipLaunchKernelGGL(k_mlp<true>, dim3((unsigned)((B + TB - 1) / TB)), dim3(WG), 0, ctx->stream, B, p, feats,
                       target, nullptr, grad, loss, 1.0f / (float)B, (uint64_t)0, (int64_t)0);
    HIP_TRY(ctx, hipGetLastError());
    return RBFFD_OK;
}

extern "C" int rbffd_mlp_train(rbffd_ctx ctx, float* params, float* adam_m, float* adam_v, int64_t count,
                               const uint16_t* feats, const float* target, const rbffd_train_opts* o,
                               float* loss_per_step) {
    if (!ctx) return RBFFD_E_ARG;
    if (!o || !params || !adam_m || !adam_v || !feats || !target) return set_error(ctx, RBFFD_E_ARG, "null pointer");
    if (count <= 0 || o->batch <= 0 || o->batch % TB != 0 || o->steps < 0)
        return set_error(ctx, RBFFD_E_ARG, "count > 0, batch a positive multiple of %d, steps >= 0 required", TB);
    if (o->seed == 0) return set_error(ctx, RBFFD_E_ARG, "seed must be non-zero");
    MlpScratch ms;
    char* extra = nullptr;
    const size_t gbytes = (RBFFD_MLP_PARAMS + 64) * sizeof(float);
    int rc = mlp_scratch(ctx, gbytes + 256 * sizeof(float), ms, &extra);
    if (rc) return rc;
    float* grad = (float*)extra;
    float* loss_tmp = grad + RBFFD_MLP_PARAMS + 32;
    hipStream_t st = ctx->stream;
    HIP_TRY(ctx, hipMemsetAsync(grad, 0, RBFFD_MLP_PARAMS * sizeof(float), st));
    convert(st, params, ms);
    Bf16Params p{ms.W1, ms.W2, ms.W2T, params};
    const int nb = o->batch / TB;
    for (int64_t s = 0; s < o->steps; ++s) {
        float* lp = loss_per_step ? loss_per_step + s : loss_tmp;
        HIP_TRY(ctx, hipMemsetAsync(lp, 0, sizeof(float), st));
        hipLaunchKernelGGL(k_mlp<true>, dim3(nb), dim3(WG), 0, st, count, p, feats, target, nullptr, grad, lp,
                           1.0f / (float)o->batch, o->seed, o->step0 + s);
        const double t = (double)(o->step0 + s + 1);
        const float c1 = (float)(1.0 / (1.0 - pow(o->beta1, t)));
        const float c2 = (float)(1.0 / (1.0 - pow(o->beta2, t)));
        hipLaunchKernelGGL(k_adam, dim3((RBFFD_MLP_PARAMS + 255) / 256), dim3(256), 0, st, params, adam_m, adam_v,
                           grad, (float)o->lr, (float)o->beta1, (float)o->beta2, (float)o->adam_eps, c1, c2, ms.W1,
                           ms.W2, ms.W2T);
    }
    HIP_TRY(ctx, hipGetLastError());
    return RBFFD_OK;
}

extern "C" int rbffd_predict_eps(rbffd_ctx ctx, const float* params, int64_t N, const double* xyz,
                                 const double* nrm, const int32_t* idx, int32_t n, double* eps) {
    if (!ctx) return RBFFD_E_ARG;
    if (N < 0) return set_error(ctx, RBFFD_E_ARG, "N < 0");
    if (N == 0) return RBFFD_OK;
    if (!params || !xyz || !nrm || !idx || !eps) return set_error(ctx, RBFFD_E_ARG, "null pointer");
    if (n < 2 || n > 64) return set_error(ctx, RBFFD_E_ARG, "features need 2 <= n <= 64 (one lane per slot)");
    MlpScratch ms;
    char* extra = nullptr;
    const size_t fbytes = (size_t)N * F * sizeof(uint16_t);
    const size_t rbytes = (size_t)N * sizeof(double), ybytes = (size_t)N * sizeof(float);
    int rc = mlp_scratch(ctx, fbytes + rbytes + ybytes + 1024, ms, &extra);
    if (rc) return rc;
    uint16_t* feats = (uint16_t*)extra;
    double* rho = (double*)(extra + ((fbytes + 255) & ~(size_t)255));
    float* y = (float*)((char*)rho + ((rbytes + 255) & ~(size_t)255));
    hipStream_t st = ctx->stream;
    hipLaunchKernelGGL(k_features, dim3((unsigned)((N + FEAT_SPW - 1) / FEAT_SPW)), dim3(64), 0, st, N, n, xyz, nrm,
                       idx, feats, rho);
    convert(st, params, ms);
    Bf16Params p{ms.W1, ms.W2, ms.W2T, params};
    hipLaunchKernelGGL(k_mlp<false>, dim3((unsigned)((N + TB - 1) / TB)), dim3(WG), 0, st, N, p, feats, nullptr, y,
                       nullptr, nullptr, 0.0f, (uint64_t)0, (int64_t)0);
    hipLaunchKernelGGL(k_eps_from_y, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, N, y, rho, eps);
    HIP_TRY(ctx, hipGetLastError());
    return RBFFD_OK;
}
