// Batched weights over many surfaces: work list, persistent launches and the
// schedule autotuner with its JSON cache.
//
// Each surface is one weights job (Secs. 4 and 5 with that surface's N and n).
// Jobs fall into two buckets by the register tiling their local system needs
// (m = n + border <= 64: one wavefront per stencil; m <= 128: four).  A
// bucket's stencils are cut into work items of `stencils_per_item`
// consecutive stencils of one surface; a persistent grid of
// groups_per_cu x (compute units) workgroups takes items from an atomic
// counter.  Per-stencil work varies with n and with the number of bisection
// steps, so the counter balances the load; ordering the surfaces by
// decreasing n puts the costly stencils first and the cheap ones at the tail.
#include "batched.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace {

struct Bucket {
    std::vector<int> jobs;  // surface indices in this bucket
};

int bucket_of(int n, int degree) { return n + rbw::border_cols(degree) <= 64 ? 0 : 1; }

rbffd_batch_tuning default_tuning(int bucket) {
    rbffd_batch_tuning t;
    std::memset(&t, 0, sizeof(t));
    t.stencils_per_item = bucket == 0 ? 16 : 2;
    t.groups_per_cu = 2;
    t.order = 0;
    return t;
}

int check_tuning(rbffd_ctx ctx, const rbffd_batch_tuning& t) {
    if (t.stencils_per_item < 1 || t.stencils_per_item > 4096)
        return set_error(ctx, RBFFD_E_ARG, "stencils_per_item must be in [1, 4096]");
    if (t.groups_per_cu < 1 || t.groups_per_cu > 2) return set_error(ctx, RBFFD_E_ARG, "groups_per_cu must be 1 or 2");
    if (t.order < 0 || t.order > 1) return set_error(ctx, RBFFD_E_ARG, "order must be 0 or 1");
    return RBFFD_OK;
}

// Validated jobs of all surfaces; computes missing stencils (kNN).
int prepare_jobs(rbffd_ctx ctx, int nsurf, const rbffd_surface* surf, const rbffd_weight_opts* opts,
                 std::vector<rbw::Job>& jobs) {
    if (nsurf < 0) return set_error(ctx, RBFFD_E_ARG, "nsurf must be >= 0");
    if (nsurf > 0 && !surf) return set_error(ctx, RBFFD_E_ARG, "null surface array");
    if (!opts) return set_error(ctx, RBFFD_E_ARG, "null opts");
    jobs.assign(nsurf, rbw::Job{});
    for (int s = 0; s < nsurf; ++s) {
        const rbffd_surface& d = surf[s];
        rbffd_weight_opts o = *opts;
        o.n = d.n;
        rbw::Job& J = jobs[s];
        std::memset(&J, 0, sizeof(J));
        int rc = weights_check_opts(ctx, d.N, &o, J.o);
        if (rc) {
            char msg[512];
            std::snprintf(msg, sizeof(msg), "%s", ctx->err);
            return set_error(ctx, rc, "surface %d: %s", s, msg);
        }
        J.N = d.N;
        if (d.N == 0) continue;
        if (!d.xyz || !d.nrm || !d.w) return set_error(ctx, RBFFD_E_ARG, "surface %d: null pointer", s);
        if ((J.o.mode == RBFFD_EPS_GIVEN || J.o.mode == RBFFD_EPS_LEARNED) && !d.eps_in)
            return set_error(ctx, RBFFD_E_ARG, "surface %d: eps_in required for this eps_mode", s);
        if (!d.idx && !d.idx_out)
            return set_error(ctx, RBFFD_E_ARG, "surface %d: idx_out required when idx is NULL", s);
    }
    for (int s = 0; s < nsurf; ++s) {
        const rbffd_surface& d = surf[s];
        rbw::Job& J = jobs[s];
        if (d.N == 0) continue;
        const int32_t* idx = d.idx;
        if (!idx) {
            int rc = knn_internal(ctx, d.N, d.xyz, d.n, d.idx_out, nullptr);
            if (rc) return rc;
            idx = d.idx_out;
        } else if (d.idx_out && d.idx_out != d.idx) {
            HIP_TRY(ctx, hipMemcpyAsync(d.idx_out, d.idx, (size_t)d.N * d.n * sizeof(int32_t),
                                        hipMemcpyDeviceToDevice, ctx->stream));
        }
        J.xyz = d.xyz;
        J.nrm = d.nrm;
        J.idx = idx;
        J.eps_in = d.eps_in;
        J.w = d.w;
        J.eps = d.eps;
        J.kappa = d.kappa;
        J.status = d.status;
        J.nevals = d.nevals;
        J.kappa_only = 0;
    }
    return RBFFD_OK;
}

void split_buckets(const std::vector<rbw::Job>& jobs, Bucket (&b)[RBFFD_BUCKETS]) {
    for (int s = 0; s < (int)jobs.size(); ++s)
        if (jobs[s].N > 0) b[bucket_of(jobs[s].o.n, jobs[s].o.degree)].jobs.push_back(s);
}

// Work items of one bucket; `limit[s]` (nullable) caps the stencils taken from surface s.
void make_items(const std::vector<rbw::Job>& jobs, const Bucket& b, const rbffd_batch_tuning& t,
                const std::vector<int64_t>* limit, std::vector<WorkItem>& items) {
    std::vector<int> order = b.jobs;
    if (t.order == 0)
        std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return jobs[a].o.n > jobs[c].o.n; });
    for (int s : order) {
        const int64_t N = limit ? std::min<int64_t>((*limit)[s], jobs[s].N) : jobs[s].N;
        for (int64_t st = 0; st < N; st += t.stencils_per_item) {
            WorkItem w;
            w.job = s;
            w.count = (int32_t)std::min<int64_t>(t.stencils_per_item, N - st);
            w.start = st;
            items.push_back(w);
        }
    }
}

int ensure_batch(rbffd_ctx ctx, size_t bytes) {
    if (bytes <= ctx->batch_bytes) return RBFFD_OK;
    if (ctx->batch) {
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        HIP_TRY(ctx, hipFree(ctx->batch));
        ctx->batch = nullptr;
        ctx->batch_bytes = 0;
    }
    const size_t want = bytes + bytes / 2 + 4096;
    if (hipMalloc(&ctx->batch, want) != hipSuccess) {
        ctx->batch = nullptr;
        return set_error(ctx, RBFFD_E_NOMEM, "cannot allocate %zu bytes for the batch work list", want);
    }
    ctx->batch_bytes = want;
    return RBFFD_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int compute_units(rbffd_ctx ctx, int& cus) {
    HIP_TRY(ctx, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    if (cus < 1) cus = 1;
    return RBFFD_OK;
}

// Upload jobs and the items of both buckets, then launch each non-empty bucket.
// The host arrays are copied synchronously (the stream is drained first), so
// they need not outlive the call.
// Events t0/t1 (nullable) are recorded around the launches.
int run_batch(rbffd_ctx ctx, const std::vector<rbw::Job>& jobs, const std::vector<WorkItem> (&items)[RBFFD_BUCKETS],
              const rbffd_batch_tuning* tuning, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr) {
    int cus = 0;
    int rc = compute_units(ctx, cus);
    if (rc) return rc;
    const size_t jbytes = align256(jobs.size() * sizeof(rbw::Job));
    const size_t ibytes0 = align256(items[0].size() * sizeof(WorkItem));
    const size_t ibytes1 = align256(items[1].size() * sizeof(WorkItem));
    const size_t cbytes = 256;
    rc = ensure_batch(ctx, jbytes + ibytes0 + ibytes1 + cbytes);
    if (rc) return rc;
    char* base = (char*)ctx->batch;
    rbw::Job* djobs = (rbw::Job*)base;
    WorkItem* ditems[RBFFD_BUCKETS] = {(WorkItem*)(base + jbytes), (WorkItem*)(base + jbytes + ibytes0)};
    int* cursors = (int*)(base + jbytes + ibytes0 + ibytes1);
    // the previous batch may still be reading these buffers
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (!jobs.empty())
        HIP_TRY(ctx, hipMemcpy(djobs, jobs.data(), jobs.size() * sizeof(rbw::Job), hipMemcpyHostToDevice));
    for (int b = 0; b < RBFFD_BUCKETS; ++b)
        if (!items[b].empty())
            HIP_TRY(ctx, hipMemcpy(ditems[b], items[b].data(), items[b].size() * sizeof(WorkItem),
                                   hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemsetAsync(cursors, 0, cbytes, ctx->stream));
    const int kernel = jobs.empty() ? 0 : jobs[0].o.kernel;
    if (t0) HIP_TRY(ctx, hipEventRecord(t0, ctx->stream));
    // bucket 1 (the costlier stencils) first
    for (int b = RBFFD_BUCKETS - 1; b >= 0; --b) {
        if (items[b].empty()) continue;
        const int nitems = (int)items[b].size();
        const int grid = std::max(1, std::min(nitems, tuning[b].groups_per_cu * cus));
        rc = weights_launch_batched(ctx, kernel, b == 0 ? 1 : 2, djobs, ditems[b], nitems, cursors + 32 * b, grid);
        if (rc) return rc;
    }
    if (t1) HIP_TRY(ctx, hipEventRecord(t1, ctx->stream));
    return RBFFD_OK;
}

// ------------------------------------------------------------ tuning cache ----
std::mutex g_cache_mu;
std::map<std::string, rbffd_batch_tuning> g_cache;

std::string cache_key(rbffd_ctx ctx, const rbw::WOpts& o, int bucket) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch = arch.substr(0, colon);
    }
    char buf[160];
    std::snprintf(buf, sizeof(buf), "%s|kernel%d|degree%d|mode%d|bucket%d", arch.c_str(), o.kernel, o.degree, o.mode,
                  bucket);
    return buf;
}

bool parse_int(const char* obj, const char* field, int& v) {
    const char* f = std::strstr(obj, field);
    if (!f) return false;
    f = std::strchr(f + std::strlen(field), ':');
    return f && std::sscanf(f + 1, "%d", &v) == 1;
}

// The cache file holds one entry per line:  "key": {"stencils_per_item": 8, ...},
void read_cache_file(const char* path, std::map<std::string, rbffd_batch_tuning>& out) {
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[1024];
    while (std::fgets(line, sizeof(line), f)) {
        const char* q0 = std::strchr(line, '"');
        if (!q0) continue;
        const char* q1 = std::strchr(q0 + 1, '"');
        const char* brace = q1 ? std::strchr(q1, '{') : nullptr;
        if (!brace) continue;
        rbffd_batch_tuning t;
        std::memset(&t, 0, sizeof(t));
        if (!parse_int(brace, "\"stencils_per_item\"", t.stencils_per_item) ||
            !parse_int(brace, "\"groups_per_cu\"", t.groups_per_cu) || !parse_int(brace, "\"order\"", t.order))
            continue;
        const char* u = std::strstr(brace, "\"us_per_stencil\"");
        if (u && (u = std::strchr(u, ':'))) t.us_per_stencil = std::atof(u + 1);
        out[std::string(q0 + 1, q1)] = t;
    }
    std::fclose(f);
}

int write_cache_file(rbffd_ctx ctx, const char* path, const std::map<std::string, rbffd_batch_tuning>& entries) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return set_error(ctx, RBFFD_E_ARG, "cannot write autotune cache %s", path);
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto& kv : entries) {
        const rbffd_batch_tuning& t = kv.second;
        std::fprintf(f, "  \"%s\": {\"stencils_per_item\": %d, \"groups_per_cu\": %d, \"order\": %d, "
                        "\"us_per_stencil\": %.6g}%s\n",
                     kv.first.c_str(), t.stencils_per_item, t.groups_per_cu, t.order, t.us_per_stencil,
                     ++i < entries.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path) != 0)
        return set_error(ctx, RBFFD_E_ARG, "cannot write autotune cache %s", path);
    return RBFFD_OK;
}

// Time one bucket's launch over the sample for schedule t (milliseconds).
int time_candidate(rbffd_ctx ctx, const std::vector<rbw::Job>& jobs, const Bucket (&bk)[RBFFD_BUCKETS], int bucket,
                   const std::vector<int64_t>& limit, const rbffd_batch_tuning& t, float& ms) {
    std::vector<WorkItem> items[RBFFD_BUCKETS];
    make_items(jobs, bk[bucket], t, &limit, items[bucket]);
    const rbffd_batch_tuning tun[RBFFD_BUCKETS] = {t, t};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = RBFFD_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rc = set_error(ctx, RBFFD_E_HIP, "hipEventCreate failed");
    if (!rc) rc = run_batch(ctx, jobs, items, tun, e0, e1);
    if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = set_error(ctx, RBFFD_E_HIP, "hipEventSynchronize failed");
    if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = set_error(ctx, RBFFD_E_HIP, "hipEventElapsedTime failed");
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}

}  // namespace

extern "C" int rbffd_build_weights_batched(rbffd_ctx ctx, int32_t nsurf, const rbffd_surface* surf,
                                           const rbffd_weight_opts* opts, const rbffd_batch_tuning* tuning) {
    if (!ctx) return RBFFD_E_ARG;
    rbffd_batch_tuning tun[RBFFD_BUCKETS];
    for (int b = 0; b < RBFFD_BUCKETS; ++b) {
        tun[b] = tuning ? tuning[b] : default_tuning(b);
        int rc = check_tuning(ctx, tun[b]);
        if (rc) return rc;
    }
    std::vector<rbw::Job> jobs;
    int rc = prepare_jobs(ctx, nsurf, surf, opts, jobs);
    if (rc) return rc;
    Bucket bk[RBFFD_BUCKETS];
    split_buckets(jobs, bk);
    std::vector<WorkItem> items[RBFFD_BUCKETS];
    for (int b = 0; b < RBFFD_BUCKETS; ++b) make_items(jobs, bk[b], tun[b], nullptr, items[b]);
    if (items[0].empty() && items[1].empty()) return RBFFD_OK;
    return run_batch(ctx, jobs, items, tun);
}

extern "C" int rbffd_autotune_batched(rbffd_ctx ctx, int32_t nsurf, const rbffd_surface* surf,
                                      const rbffd_weight_opts* opts, const char* cache_path, int32_t retune,
                                      rbffd_batch_tuning* tuning) {
    if (!ctx) return RBFFD_E_ARG;
    if (!tuning) return set_error(ctx, RBFFD_E_ARG, "null tuning output");
    std::vector<rbw::Job> jobs;
    int rc = prepare_jobs(ctx, nsurf, surf, opts, jobs);
    if (rc) return rc;
    Bucket bk[RBFFD_BUCKETS];
    split_buckets(jobs, bk);
    std::lock_guard<std::mutex> lock(g_cache_mu);
    if (cache_path) read_cache_file(cache_path, g_cache);
    bool changed = false;
    for (int b = 0; b < RBFFD_BUCKETS; ++b) {
        tuning[b] = default_tuning(b);
        if (bk[b].jobs.empty()) continue;
        const std::string key = cache_key(ctx, jobs[bk[b].jobs[0]].o, b);
        auto it = g_cache.find(key);
        if (!retune && it != g_cache.end() && check_tuning(ctx, it->second) == RBFFD_OK) {
            tuning[b] = it->second;
            continue;
        }
        // sample: the first stencils of every surface, in proportion to its size
        int64_t total = 0;
        for (int s : bk[b].jobs) total += jobs[s].N;
        const int64_t want = b == 0 ? 32768 : 8192;
        const double frac = std::min(1.0, (double)want / (double)total);
        std::vector<int64_t> limit(jobs.size(), 0);
        int64_t sample = 0;
        for (int s : bk[b].jobs) {
            limit[s] = std::max<int64_t>(1, (int64_t)std::ceil(frac * (double)jobs[s].N));
            sample += std::min(limit[s], jobs[s].N);
        }
        std::vector<rbffd_batch_tuning> cands;
        const int spi0[] = {4, 8, 16, 32, 64};
        const int spi1[] = {1, 2, 4, 8};
        const int* spi = b == 0 ? spi0 : spi1;
        const int nspi = b == 0 ? 5 : 4;
        for (int i = 0; i < nspi; ++i)
            for (int g = 1; g <= 2; ++g)
                for (int ord = 0; ord <= 1; ++ord) {
                    rbffd_batch_tuning t = default_tuning(b);
                    t.stencils_per_item = spi[i];
                    t.groups_per_cu = g;
                    t.order = ord;
                    cands.push_back(t);
                }
        float warm = 0.0f;
        rc = time_candidate(ctx, jobs, bk, b, limit, cands[0], warm);  // loads code, warms caches
        if (rc) return rc;
        float best = INFINITY;
        for (const rbffd_batch_tuning& t : cands) {
            float ms = 0.0f;
            rc = time_candidate(ctx, jobs, bk, b, limit, t, ms);
            if (rc) return rc;
            if (ms < best) {
                best = ms;
                tuning[b] = t;
            }
        }
        tuning[b].us_per_stencil = 1e3 * (double)best / (double)sample;
        g_cache[key] = tuning[b];
        changed = true;
    }
    if (cache_path && changed) {
        rc = write_cache_file(ctx, cache_path, g_cache);
        if (rc) return rc;
    }
    return RBFFD_OK;
}
