// Context lifetime, errors and scratch.
#include "common.h"

#include <cstdlib>
#include <cstring>
#include <new>

int set_error(rbffd_ctx ctx, int code, const char* fmt, ...) {
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

int ensure_scratch(rbffd_ctx ctx, size_t bytes) {
    if (bytes <= ctx->scratch_bytes) return RBFFD_OK;
    if (ctx->scratch) {
        // work already enqueued may still read the old buffer
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        HIP_TRY(ctx, hipFree(ctx->scratch));
        ctx->scratch = nullptr;
        ctx->scratch_bytes = 0;
    }
    size_t want = bytes + bytes / 4 + (1u << 20);
    if (hipMalloc(&ctx->scratch, want) != hipSuccess) {
        ctx->scratch = nullptr;
        return set_error(ctx, RBFFD_E_NOMEM, "cannot allocate %zu bytes of scratch", want);
    }
    ctx->scratch_bytes = want;
    return RBFFD_OK;
}

extern "C" void rbffd_default_opts(rbffd_weight_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->n = 31;
    o->kernel = RBFFD_KERNEL_MQ;
    o->poly_degree = 2;
    o->eps_mode = RBFFD_EPS_FIXED;
    o->eps_fixed = 2.0;
    o->kappa_target = 1e12;
    o->eps_tol = 1e-4;
    o->bracket_lo = 0.05;
    o->bracket_hi = 20.0;
    o->band_lo = 1e11;
    o->band_hi = 1e13;
    o->rank_tol = 1e-10;
    o->band_stop = 0;
    o->max_expand = 8;
}

extern "C" int rbffd_create(rbffd_ctx* out, void* stream) {
    if (!out) return RBFFD_E_ARG;
    rbffd_ctx c = new (std::nothrow) rbffd_ctx_s();
    if (!c) return RBFFD_E_NOMEM;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return RBFFD_E_HIP;
    }
    if (noalloc_scratch_setup(c, c->device) != RBFFD_OK) {
        delete c;
        return RBFFD_E_HIP;
    }
    *out = c;
    return RBFFD_OK;
}

extern "C" int rbffd_destroy(rbffd_ctx ctx) {
    if (!ctx) return RBFFD_E_ARG;
    if (ctx->scratch) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(ctx->scratch);
    }
    if (ctx->batch) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(ctx->batch);
    }
    delete ctx;
    return RBFFD_OK;
}

extern "C" const char* rbffd_last_error(rbffd_ctx ctx) { return ctx ? ctx->err : "null context"; }
