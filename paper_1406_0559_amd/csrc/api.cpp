// C-ABI of the raylens library: argument validation, per-map parameter
// records, the context's scratch memory, batching work lists and statistics.
// The declarations and their contracts are in include/raylens.h.
#include "raylens.h"

#include <algorithm>
#include <cfloat>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "maps.h"

namespace {
thread_local std::string g_error;
}  // namespace

namespace rl {

rl_status set_error(rl_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return st;
}

void clear_error() { g_error.clear(); }

}  // namespace rl

namespace {

template <typename... A>
rl_status fail(rl_status st, const char* fmt, A... args) {
    return rl::set_error(st, fmt, args...);
}

rl_status hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? RL_E_NOMEM : RL_E_DEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

bool is_finite(double v) { return std::isfinite(v); }

// Folds the per-workgroup records of launch_count_stats / launch_prob_sum:
// out[0] and out[2] sum words 0 and 2, out[1] is the largest word 1.
void fold_records(const unsigned long long* rec, int nb, unsigned long long out[3]) {
    out[0] = out[1] = out[2] = 0;
    for (int i = 0; i < nb; ++i) {
        const unsigned long long* w = rec + (size_t)i * rl::kRecWords;
        out[0] += w[0];
        out[1] = w[1] > out[1] ? w[1] : out[1];
        out[2] += w[2];
    }
}

// ---------------------------------------------------------------------------
// validation (host only, before any HIP call)
// ---------------------------------------------------------------------------

rl_status check_grid(const rl_raygrid* g) {
    if (!g) return fail(RL_E_INVALID, "ray grid is NULL");
    if (g->n1 <= 0 || g->n2 <= 0) return fail(RL_E_INVALID, "ray grid needs n1, n2 > 0");
    // the ray count stays far inside int64 (ray, cell and escape counts); one
    // row of ray cells (>= 8 rays across) fits one launch of the shoot kernel
    if (g->n1 > (int64_t)1 << 26 || g->n2 > (int64_t)1 << 40 ||
        (double)g->n1 * (double)g->n2 > (double)((int64_t)1 << 50))
        return fail(RL_E_INVALID, "ray grid too large (at most 2^26 rays along x1, 2^40 along x2 "
                    "and 2^50 rays)");
    if (!is_finite(g->c1) || !is_finite(g->c2)) return fail(RL_E_INVALID, "ray grid centre not finite");
    if (!is_finite(g->half1) || !is_finite(g->half2) || !(g->half1 > 0.0) || !(g->half2 > 0.0))
        return fail(RL_E_INVALID, "ray grid half-widths must be finite and > 0");
    return RL_OK;
}

rl_status check_window(const rl_window* w) {
    if (!w) return fail(RL_E_INVALID, "window is NULL");
    if (w->p1 <= 0 || w->p2 <= 0) return fail(RL_E_INVALID, "window needs p1, p2 > 0");
    if (!is_finite(w->c1) || !is_finite(w->c2)) return fail(RL_E_INVALID, "window centre not finite");
    if (!is_finite(w->width1) || !is_finite(w->width2) || !(w->width1 > 0.0) || !(w->width2 > 0.0))
        return fail(RL_E_INVALID, "window widths must be finite and > 0");
    return RL_OK;
}

rl_status check_macro(const rl_macro* m) {
    if (!m) return fail(RL_E_INVALID, "macro model is NULL");
    if (!is_finite(m->kappa) || !is_finite(m->gamma) || !is_finite(m->s))
        return fail(RL_E_INVALID, "kappa, gamma and s must be finite");
    return RL_OK;
}

rl_status check_lenses(const rl_lenses* l) {
    if (!l) return fail(RL_E_INVALID, "lenses is NULL");
    if (l->n < 0) return fail(RL_E_INVALID, "lens count must be >= 0");
    if (l->n > ((int64_t)1 << 31)) return fail(RL_E_INVALID, "lens count too large");
    if (l->n > 0 && (!l->x1 || !l->x2)) return fail(RL_E_INVALID, "lens positions are NULL");
    return RL_OK;
}

rl_status check_precision(int32_t p) {
    if (p != RL_FP32_COMP && p != RL_FP64_PLAIN) return fail(RL_E_INVALID, "unknown precision");
    return RL_OK;
}

rl_status check_rows(const rl_raygrid* g, int64_t rb, int64_t re) {
    if (rb < 0 || re < rb || re > g->n2)
        return fail(RL_E_INVALID, "row range [%lld, %lld) outside [0, %lld]", (long long)rb,
                    (long long)re, (long long)g->n2);
    return RL_OK;
}


// ---------------------------------------------------------------------------
// parameter records
// ---------------------------------------------------------------------------

// Cell shape: 1024 rays, cx x cy with cx*d1 ~ cy*d2 (square on the sky), cx a
// power of two in [8, 128]. Depends only on the grid.
void cell_shape(double d1, double d2, int32_t* cx, int32_t* cy) {
    const int cands[5] = {8, 16, 32, 64, 128};
    int best = 32;
    double best_err = 1e300;
    for (int c : cands) {
        const double ext1 = c * d1, ext2 = (double)(rl::kCellRays / c) * d2;
        const double err = std::fabs(std::log(ext1 / ext2));
        if (err < best_err - 1e-12) { best_err = err; best = c; }
    }
    *cx = best;
    *cy = rl::kCellRays / best;
}

void build_params(const rl_macro* M, const rl_raygrid* G, const rl_window* W, int64_t rb,
                  int64_t re, rl::MapParams* P) {
    std::memset(P, 0, sizeof(*P));
    P->n1 = G->n1;
    P->n2 = G->n2;
    // ray (i, j) at base + (i + 1/2) d, d = 2 h / n (cell centres)
    P->base1 = G->c1 - G->half1;
    P->base2 = G->c2 - G->half2;
    P->d1 = (2.0 * G->half1) / (double)G->n1;
    P->d2 = (2.0 * G->half2) / (double)G->n2;
    P->d1f = (float)P->d1;
    P->d2f = (float)P->d2;
    cell_shape(P->d1, P->d2, &P->cx, &P->cy);
    P->cells_x = (G->n1 + P->cx - 1) / P->cx;
    P->row_begin = rb;
    P->row_end = re;
    if (re > rb) {
        P->cell_row0 = rb / P->cy;
        const int64_t last = (re - 1) / P->cy;
        P->n_cells = (last - P->cell_row0 + 1) * P->cells_x;
    } else {
        P->cell_row0 = 0;
        P->n_cells = 0;
    }
    // eq. 1 with kappa_s = s kappa (eq. 2): diag(1 - gamma, 1 + gamma) - kappa_s
    const double kappa_s = M->s * M->kappa;
    P->a1 = (1.0 - M->gamma) - kappa_s;
    P->a2 = (1.0 + M->gamma) - kappa_s;
    // half-open pixels from lo = centre - width / 2, u = (y - lo) * p / width
    P->p1 = W->p1;
    P->p2 = W->p2;
    P->lo1 = W->c1 - 0.5 * W->width1;
    P->lo2 = W->c2 - 0.5 * W->width2;
    P->inv1 = (double)W->p1 / W->width1;
    P->inv2 = (double)W->p2 / W->width2;
}


// RAII: make the context's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev) {
        err = hipGetDevice(&prev);
        if (err != hipSuccess) { ok = false; return; }
        if (prev != dev) {
            err = hipSetDevice(dev);
            if (err != hipSuccess) ok = false;
        }
    }
    ~DeviceGuard() {
        int cur = -1;
        if (ok && hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
    }
};

// Device scratch reused across calls in stream order: a new user waits (on the
// GPU) for the previous user's work before touching it.
struct Scratch {
    void* ptr = nullptr;
    size_t cap = 0;
    hipEvent_t last = nullptr;
    bool used = false;
    uint64_t gen = 0;    // bumped on every (re)allocation: contents from before are gone

    hipError_t acquire(size_t bytes, hipStream_t s) {
        hipError_t e;
        if (!last) {
            e = hipEventCreateWithFlags(&last, hipEventDisableTiming);
            if (e != hipSuccess) return e;
        }
        if (used) {
            e = hipStreamWaitEvent(s, last, 0);
            if (e != hipSuccess) return e;
        }
        if (cap < bytes) {
            if (ptr) {
                e = hipDeviceSynchronize();
                if (e != hipSuccess) return e;
                e = hipFree(ptr);
                if (e != hipSuccess) return e;
                ptr = nullptr;
                cap = 0;
            }
            size_t want = std::max<size_t>(bytes, 1 << 16);
            want = (want + 4095) & ~(size_t)4095;
            e = hipMalloc(&ptr, want);
            ++gen;
            if (e != hipSuccess) { ptr = nullptr; return e; }
            cap = want;
        }
        return hipSuccess;
    }
    hipError_t release(hipStream_t s) {
        used = true;
        return hipEventRecord(last, s);
    }
    void destroy() {
        if (ptr) (void)hipFree(ptr);
        if (last) (void)hipEventDestroy(last);
        ptr = nullptr;
        last = nullptr;
    }
};

}  // namespace

// Pinned read-back buffer: the reduction slots plus the escaped count.
constexpr size_t kReadBytes = rl::kRedBytes + 256;

struct rl_context {
    int device = 0;
    bool ready = false;
    int num_cus = 256;
    Scratch lens;        // FP32 lens copies
    Scratch batch;       // map records + work items + counter
    Scratch aux;         // MPD thresholds, codec tables, source samples
    Scratch fft;         // convolution planes
    // sides and scratch generation of the stage-twiddle tables the last
    // convolution left in the fft scratch (recomputed when either changes)
    int fft_tw_p1 = 0, fft_tw_p2 = 0;
    uint64_t fft_tw_gen = 0;
    void* host_stage = nullptr;  // pinned staging for batch records
    size_t host_cap = 0;
    // pinned, device-mapped buffer of kReadBytes: the reductions' records are
    // stored straight into it, and small copies back land in it
    void* host_read = nullptr;
    unsigned long long* host_read_dev = nullptr;   // its device address
    hipEvent_t stage_done = nullptr;
    bool stage_used = false;
    rl::KernelShape tuning[2][rl::kTuningClasses];
};

int rl::context_device(const rl_context* ctx) { return ctx->device; }

namespace {

rl_status ensure_ready(rl_context* ctx) {
    if (ctx->ready) return RL_OK;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) return fail(RL_E_DEVICE, "no HIP device available");
    if (ctx->device >= n) return fail(RL_E_DEVICE, "device %d not present (%d devices)", ctx->device, n);
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    ctx->num_cus = cus > 0 ? cus : 256;
    e = hipEventCreateWithFlags(&ctx->stage_done, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    e = hipHostMalloc(&ctx->host_read, kReadBytes, hipHostMallocMapped | hipHostMallocCoherent);
    if (e != hipSuccess) { ctx->host_read = nullptr; return hip_fail(e, "pinned read-back buffer"); }
    void* dev = nullptr;
    e = hipHostGetDevicePointer(&dev, ctx->host_read, 0);
    if (e != hipSuccess) {
        (void)hipHostFree(ctx->host_read);
        ctx->host_read = nullptr;
        return hip_fail(e, "device address of the read-back buffer");
    }
    ctx->host_read_dev = static_cast<unsigned long long*>(dev);
    ctx->ready = true;
    return RL_OK;
}

// Waits for a reduction launched into ctx->host_read_dev and folds its `nb`
// records (also returns the records, for words past them).
hipError_t fold_reduction(rl_context* ctx, int nb, hipStream_t s, unsigned long long out[3]) {
    const hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) fold_records(static_cast<const unsigned long long*>(ctx->host_read), nb, out);
    return e;
}

// Copies `bytes` of device results to host memory in stream order and waits
// for them: through the context's pinned buffer when they fit (a pageable
// destination costs an extra staged copy in the runtime), directly otherwise.
hipError_t read_back(rl_context* ctx, void* dst, const void* src, size_t bytes, hipStream_t s) {
    const bool pinned = ctx->host_read && bytes <= kReadBytes;
    hipError_t e = hipMemcpyAsync(pinned ? ctx->host_read : dst, src, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && pinned) std::memcpy(dst, ctx->host_read, bytes);
    return e;
}

// Prepares FP32 hi/lo lens copies in the context's lens scratch.
rl_status prepare_lenses_f32(rl_context* ctx, const rl_lenses* L, bool force_mass,
                             rl::MapParams* P, hipStream_t s) {
    const int64_t n = L->n;
    const bool masses = L->m != nullptr || force_mass;
    const size_t bytes = (size_t)std::max<int64_t>(n, 1) * (sizeof(float4) + sizeof(float));
    hipError_t e = ctx->lens.acquire(bytes, s);
    if (e != hipSuccess) return hip_fail(e, "lens scratch");
    float4* xy = static_cast<float4*>(ctx->lens.ptr);
    float* mf = reinterpret_cast<float*>(xy + std::max<int64_t>(n, 1));
    e = rl::launch_prep_lenses(L->x1, L->x2, L->m, n, xy, masses ? mf : nullptr, true, s);
    if (e != hipSuccess) return hip_fail(e, "prep_lenses launch");
    P->lens32 = xy;
    P->imass32 = masses ? mf : nullptr;
    P->n_lens = n;
    return RL_OK;
}

// Pinned host staging shared by the calls of one context: a caller writes the
// returned buffer, then stage_send copies it to device memory in stream order.
// The previous copy out of the buffer is waited for before it is reused.
rl_status stage_reserve(rl_context* ctx, size_t bytes, char** host) {
    hipError_t e;
    if (ctx->stage_used) {
        e = hipEventSynchronize(ctx->stage_done);
        if (e != hipSuccess) return hip_fail(e, "staging wait");
    }
    if (ctx->host_cap < bytes) {
        if (ctx->host_stage) (void)hipHostFree(ctx->host_stage);
        ctx->host_stage = nullptr;
        ctx->host_cap = 0;
        e = hipHostMalloc(&ctx->host_stage, bytes, hipHostMallocDefault);
        if (e != hipSuccess) { ctx->host_stage = nullptr; return hip_fail(e, "pinned staging"); }
        ctx->host_cap = bytes;
    }
    *host = static_cast<char*>(ctx->host_stage);
    return RL_OK;
}

rl_status stage_send(rl_context* ctx, void* dst, size_t bytes, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(dst, ctx->host_stage, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "staging copy");
    e = hipEventRecord(ctx->stage_done, s);
    if (e != hipSuccess) return hip_fail(e, "staging event");
    ctx->stage_used = true;
    return RL_OK;
}

rl_status check_counts(const int32_t* d_counts, const rl_window* win) {
    RL_TRY(check_window(win));
    if (!d_counts) return fail(RL_E_INVALID, "counts pointer is NULL");
    return RL_OK;
}

}  // namespace

extern "C" {

const char* rl_last_error(void) { return g_error.c_str(); }

#ifndef RL_KERNEL_ID
#define RL_KERNEL_ID "unversioned"
#endif

// The kernel id is a digest of the shoot kernel's sources, so tuning caches
// made by another build are not applied.
const char* rl_version(void) { return "raylens 0.2 (gfx950, kernels " RL_KERNEL_ID ")"; }

rl_status rl_create(int32_t hip_device, rl_context** out) {
    g_error.clear();
    if (!out) return fail(RL_E_INVALID, "out is NULL");
    if (hip_device < 0) return fail(RL_E_INVALID, "device index must be >= 0");
    rl_context* c = new (std::nothrow) rl_context();
    if (!c) return fail(RL_E_NOMEM, "context allocation failed");
    c->device = hip_device;
    // defaults measured on gfx950 (the autotuner refines them): 4 x 4 rays
    // per lane, 256-lens tiles, 4 waves, bounding-box sub-map
    for (int p = 0; p < 2; ++p)
        for (int k = 0; k < rl::kTuningClasses; ++k) c->tuning[p][k] = rl::KernelShape{4, 4, 256, 4, 1};
    *out = c;
    return RL_OK;
}

rl_status rl_destroy(rl_context* ctx) {
    g_error.clear();
    if (!ctx) return RL_OK;
    if (ctx->ready) {
        DeviceGuard dg(ctx->device);
        (void)hipDeviceSynchronize();
        ctx->lens.destroy();
        ctx->batch.destroy();
        ctx->aux.destroy();
        ctx->fft.destroy();
        if (ctx->host_stage) (void)hipHostFree(ctx->host_stage);
        if (ctx->host_read) (void)hipHostFree(ctx->host_read);
        if (ctx->stage_done) (void)hipEventDestroy(ctx->stage_done);
    }
    delete ctx;
    return RL_OK;
}

rl_status rl_n_avg(const rl_raygrid* grid, const rl_window* win, double* h_out) {
    g_error.clear();
    RL_TRY(check_grid(grid));
    RL_TRY(check_window(win));
    if (!h_out) return fail(RL_E_INVALID, "h_out is NULL");
    // eq. 4's N_avg: unlensed ray density times the pixel area
    const double ray_density = ((double)grid->n1 * (double)grid->n2) / (4.0 * grid->half1 * grid->half2);
    const double pixel_area = (win->width1 / (double)win->p1) * (win->width2 / (double)win->p2);
    *h_out = ray_density * pixel_area;
    return RL_OK;
}

rl_status rl_get_tuning(rl_context* ctx, int32_t precision, int32_t n_cls, rl_tuning* h_out) {
    g_error.clear();
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    RL_TRY(check_precision(precision));
    if (n_cls < 0 || n_cls >= rl::kTuningClasses)
        return fail(RL_E_INVALID, "tuning class must be in [0, %d)", rl::kTuningClasses);
    if (!h_out) return fail(RL_E_INVALID, "h_out is NULL");
    const rl::KernelShape& k = ctx->tuning[precision][n_cls];
    *h_out = rl_tuning{k.rays_x, k.rays_y, k.lens_tile, k.waves, k.submap};
    return RL_OK;
}

rl_status rl_set_tuning(rl_context* ctx, int32_t precision, int32_t n_cls, const rl_tuning* t) {
    g_error.clear();
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    RL_TRY(check_precision(precision));
    if (n_cls < 0 || n_cls >= rl::kTuningClasses)
        return fail(RL_E_INVALID, "tuning class must be in [0, %d)", rl::kTuningClasses);
    if (!t) return fail(RL_E_INVALID, "tuning is NULL");
    rl::KernelShape k{t->rays_x, t->rays_y, t->lens_tile, t->waves, t->submap};
    if (!rl::shape_supported((rl::Precision)precision, k))
        return fail(RL_E_INVALID, "unsupported kernel shape (%d x %d rays, tile %d, %d waves, submap %d)",
                    k.rays_x, k.rays_y, k.lens_tile, k.waves, k.submap);
    ctx->tuning[precision][n_cls] = k;
    return RL_OK;
}

rl_status rl_shoot(rl_context* ctx, const rl_lenses* lenses, const rl_macro* macro,
                   const rl_raygrid* grid, const rl_window* win, int32_t precision,
                   int64_t row_begin, int64_t row_end, int32_t* d_counts, int64_t* d_escaped,
                   hipStream_t stream) {
    g_error.clear();
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    RL_TRY(check_lenses(lenses));
    RL_TRY(check_macro(macro));
    RL_TRY(check_grid(grid));
    RL_TRY(check_window(win));
    RL_TRY(check_precision(precision));
    RL_TRY(check_rows(grid, row_begin, row_end));
    if (!d_counts || !d_escaped) return fail(RL_E_INVALID, "output pointers are NULL");
    if (row_end == row_begin) return RL_OK;

    rl::MapParams P;
    build_params(macro, grid, win, row_begin, row_end, &P);
    P.counts = d_counts;
    P.escaped = reinterpret_cast<unsigned long long*>(d_escaped);

    DeviceGuard dg(ctx->device);
    if (!dg.ok) return hip_fail(dg.err, "hipSetDevice");
    RL_TRY(ensure_ready(ctx));
    const rl::KernelShape& ks = ctx->tuning[precision][rl::tuning_class(lenses->n, lenses->m != nullptr)];
    hipError_t e;
    if (precision == RL_FP32_COMP) {
        RL_TRY(prepare_lenses_f32(ctx, lenses, false, &P, stream));
        e = rl::launch_shoot(P, rl::kFP32Comp, ks, false, ctx->num_cus, stream);
        hipError_t e2 = ctx->lens.release(stream);
        if (e == hipSuccess) e = e2;
    } else {
        P.lx1 = lenses->x1;
        P.lx2 = lenses->x2;
        P.lm = lenses->m;
        P.n_lens = lenses->n;
        e = rl::launch_shoot(P, rl::kFP64Plain, ks, false, ctx->num_cus, stream);
    }
    if (e != hipSuccess) return hip_fail(e, "shoot launch");
    return RL_OK;
}

rl_status rl_shoot_noalloc(rl_context* ctx, const rl_lenses* lenses, const rl_macro* macro,
                           const rl_raygrid* grid, const rl_window* win, int32_t precision,
                           int64_t row_begin, int64_t row_end, int32_t* d_counts,
                           int64_t* d_escaped, hipStream_t stream) {
    g_error.clear();
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    RL_TRY(check_lenses(lenses));
    RL_TRY(check_macro(macro));
    RL_TRY(check_grid(grid));
    RL_TRY(check_window(win));
    RL_TRY(check_precision(precision));
    RL_TRY(check_rows(grid, row_begin, row_end));
    if (!d_counts || !d_escaped) return fail(RL_E_INVALID, "output pointers are NULL");
    if (lenses->n > RL_NOALLOC_MAX_LENSES)
        return fail(RL_E_INVALID, "rl_shoot_noalloc takes at most %d lenses (%lld given); "
                    "use rl_shoot for larger fields", RL_NOALLOC_MAX_LENSES, (long long)lenses->n);
    if (row_end == row_begin) return RL_OK;

    rl::MapParams P;
    build_params(macro, grid, win, row_begin, row_end, &P);
    P.counts = d_counts;
    P.escaped = reinterpret_cast<unsigned long long*>(d_escaped);
    // no ensure_ready: that creates a HIP event on a context's first use
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return hip_fail(dg.err, "hipSetDevice");
    const rl::KernelShape& ks = ctx->tuning[precision][rl::tuning_class(lenses->n, lenses->m != nullptr)];
    const hipError_t e = rl::launch_shoot_noalloc(P, lenses->x1, lenses->x2, lenses->m, lenses->n,
                                                  (rl::Precision)precision, ks, ctx->device, stream);
    if (e != hipSuccess) return hip_fail(e, "shoot launch (no allocation)");
    return RL_OK;
}

rl_status rl_ray_positions(rl_context* ctx, const rl_lenses* lenses, const rl_macro* macro,
                           const rl_raygrid* grid, int32_t precision, int64_t row_begin,
                           int64_t row_end, double* d_y1, double* d_y2, hipStream_t stream) {
    g_error.clear();
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    RL_TRY(check_lenses(lenses));
    RL_TRY(check_macro(macro));
    RL_TRY(check_grid(grid));
    RL_TRY(check_precision(precision));
    RL_TRY(check_rows(grid, row_begin, row_end));
    if (!d_y1 || !d_y2) return fail(RL_E_INVALID, "output pointers are NULL");
    if (row_end == row_begin) return RL_OK;

    rl_window dummy{1, 1, 0.0, 0.0, 1.0, 1.0};
    rl::MapParams P;
    build_params(macro, grid, &dummy, row_begin, row_end, &P);
    P.out_y1 = d_y1;
    P.out_y2 = d_y2;

    DeviceGuard dg(ctx->device);
    if (!dg.ok) return hip_fail(dg.err, "hipSetDevice");
    RL_TRY(ensure_ready(ctx));
    rl::KernelShape ks = ctx->tuning[precision][rl::tuning_class(lenses->n, lenses->m != nullptr)];
    hipError_t e;
    if (precision == RL_FP32_COMP) {
        RL_TRY(prepare_lenses_f32(ctx, lenses, false, &P, stream));
        e = rl::launch_shoot(P, rl::kFP32Comp, ks, true, ctx->num_cus, stream);
        hipError_t e2 = ctx->lens.release(stream);
        if (e == hipSuccess) e = e2;
    } else {
        P.lx1 = lenses->x1;
        P.lx2 = lenses->x2;
        P.lm = lenses->m;
        P.n_lens = lenses->n;
        e = rl::launch_shoot(P, rl::kFP64Plain, ks, true, ctx->num_cus, stream);
    }
    if (e != hipSuccess) return hip_fail(e, "ray_positions launch");
    return RL_OK;
}

rl_status rl_bin_positions(rl_context* ctx, const double* d_y1, const double* d_y2, int64_t n,
                           const rl_window* win, int32_t* d_counts, int64_t* d_escaped,
                           hipStream_t stream) {
    g_error.clear();
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    if (n < 0) return fail(RL_E_INVALID, "n must be >= 0");
    RL_TRY(check_window(win));
    if (n > 0 && (!d_y1 || !d_y2)) return fail(RL_E_INVALID, "position pointers are NULL");
    if (!d_counts || !d_escaped) return fail(RL_E_INVALID, "output pointers are NULL");
    if (n == 0) return RL_OK;
    const double lo1 = win->c1 - 0.5 * win->width1;
    const double lo2 = win->c2 - 0.5 * win->width2;
    const double inv1 = (double)win->p1 / win->width1;
    const double inv2 = (double)win->p2 / win->width2;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return hip_fail(dg.err, "hipSetDevice");
    RL_TRY(ensure_ready(ctx));
    hipError_t e = rl::launch_bin_positions(d_y1, d_y2, n, win->p1, win->p2, lo1, lo2, inv1, inv2,
                                            d_counts, reinterpret_cast<unsigned long long*>(d_escaped),
                                            stream);
    if (e != hipSuccess) return hip_fail(e, "bin_positions launch");
    return RL_OK;
}

rl_status rl_normalise(rl_context* ctx, const int32_t* d_counts, const rl_window* win,
                       double n_avg, float* d_mu, hipStream_t stream) {
    g_error.clear();
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    RL_TRY(check_window(win));
    if (!is_finite(n_avg) || !(n_avg > 0.0)) return fail(RL_E_INVALID, "n_avg must be finite and > 0");
    if (!d_counts || !d_mu) return fail(RL_E_INVALID, "buffer pointers are NULL");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return hip_fail(dg.err, "hipSetDevice");
    RL_TRY(ensure_ready(ctx));
    hipError_t e = rl::launch_normalise(d_counts, (int64_t)win->p1 * win->p2, n_avg, d_mu, stream);
    if (e != hipSuccess) return hip_fail(e, "normalise launch");
    return RL_OK;
}

rl_status rl_stats_get(rl_context* ctx, const int32_t* d_counts, const int64_t* d_escaped,
                       const rl_macro* macro, const rl_raygrid* grid, const rl_window* win,
                       rl_stats* h_out, hipStream_t stream) {
    g_error.clear();
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    RL_TRY(check_macro(macro));
    RL_TRY(check_grid(grid));
    RL_TRY(check_window(win));
    if (!d_counts || !d_escaped || !h_out) return fail(RL_E_INVALID, "pointers are NULL");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return hip_fail(dg.err, "hipSetDevice");
    RL_TRY(ensure_ready(ctx));
    // the workgroups' records, then the escaped count in one more word, stored
    // in the pinned buffer
    const int64_t n = (int64_t)win->p1 * win->p2;
    hipError_t e = rl::launch_count_stats(d_counts, n, reinterpret_cast<const unsigned long long*>(d_escaped),
                                          ctx->host_read_dev, stream);
    unsigned long long host[4];
    if (e == hipSuccess) e = fold_reduction(ctx, rl::reduce_blocks(n), stream, host);
    if (e != hipSuccess) return hip_fail(e, "stats");
    host[3] = static_cast<const unsigned long long*>(ctx->host_read)[(size_t)rl::kRedBlocks * rl::kRecWords];
    double n_avg = 0.0;
    RL_TRY(rl_n_avg(grid, win, &n_avg));
    rl_stats st;
    st.shot = grid->n1 * grid->n2;
    st.binned = (int64_t)host[0];
    st.escaped = (int64_t)host[3];
    st.n_avg = n_avg;
    st.mean_count = (double)st.binned / ((double)win->p1 * (double)win->p2);
    st.mean_mu = st.mean_count / n_avg;
    const double k1 = 1.0 - macro->kappa;
    st.mu_th = 1.0 / (k1 * k1 - macro->gamma * macro->gamma);
    st.max_count = (int32_t)host[1];
    *h_out = st;
    if ((int64_t)host[1] >= INT32_MAX) return fail(RL_E_OVERFLOW, "a pixel count reached INT32_MAX");
    return RL_OK;
}

rl_status rl_shoot_batch(rl_context* ctx, const rl_map_desc* h_maps, int32_t n_maps,
                         int32_t precision, hipStream_t stream) {
    g_error.clear();
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    if (n_maps < 0) return fail(RL_E_INVALID, "n_maps must be >= 0");
    if (n_maps > 0 && !h_maps) return fail(RL_E_INVALID, "maps is NULL");
    RL_TRY(check_precision(precision));
    for (int32_t i = 0; i < n_maps; ++i) {
        const rl_map_desc& d = h_maps[i];
        rl_status st;
        if ((st = check_lenses(&d.lenses)) != RL_OK || (st = check_macro(&d.macro)) != RL_OK ||
            (st = check_grid(&d.grid)) != RL_OK || (st = check_window(&d.win)) != RL_OK ||
            (st = check_rows(&d.grid, d.row_begin, d.row_end)) != RL_OK) {
            std::string m = g_error;
            return fail(st, "map %d: %s", (int)i, m.c_str());
        }
        if (!d.d_counts || !d.d_escaped) return fail(RL_E_INVALID, "map %d: output pointers are NULL", (int)i);
    }
    if (n_maps == 0) return RL_OK;

    // per tuning class present: every map (or range of its cell rows) is a
    // segment of that class's launches, with the class's kernel shape (kernel
    // shapes change no result bit, so every map still equals the map shot
    // alone); segments in descending cost per workgroup, so the last
    // workgroups of a launch are the cheapest
    int64_t total_lens = 0;
    std::vector<int> cls((size_t)n_maps);
    for (int32_t i = 0; i < n_maps; ++i) {
        cls[i] = rl::tuning_class(h_maps[i].lenses.n, h_maps[i].lenses.m != nullptr);
        total_lens += h_maps[i].lenses.n;
    }
    std::vector<rl::MapParams> params((size_t)n_maps);
    for (int32_t i = 0; i < n_maps; ++i) {
        const rl_map_desc& d = h_maps[i];
        build_params(&d.macro, &d.grid, &d.win, d.row_begin, d.row_end, &params[i]);
        params[i].counts = d.d_counts;
        params[i].escaped = reinterpret_cast<unsigned long long*>(d.d_escaped);
        params[i].n_lens = d.lenses.n;
    }
    struct Launch {
        int cls;
        size_t seg0, nseg;
        int64_t blocks;
    };
    std::vector<int32_t> seg_map;     // map of each segment
    std::vector<int64_t> seg_row0, seg_cells, seg_first;
    std::vector<Launch> launches;
    for (int c = 0; c < rl::kTuningClasses; ++c) {
        std::vector<int32_t> order;
        for (int32_t i = 0; i < n_maps; ++i)
            if (cls[i] == c && params[i].n_cells > 0) order.push_back(i);
        if (order.empty()) continue;
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a, int32_t b) { return h_maps[a].lenses.n > h_maps[b].lenses.n; });
        const int64_t per = rl::batch_cells_per_block(ctx->tuning[precision][c]);
        Launch cur{c, seg_map.size(), 0, 0};
        for (int32_t i : order) {
            const rl::MapParams& P = params[i];
            const int64_t rows = P.n_cells / P.cells_x;
            const int64_t rows_per_seg = std::max<int64_t>(1, rl::kMaxLaunchBlocks * per / P.cells_x);
            for (int64_t r0 = 0; r0 < rows; r0 += rows_per_seg) {
                const int64_t nr = std::min(rows_per_seg, rows - r0);
                const int64_t span = ((nr * P.cells_x + per - 1) / per + 7) / 8 * 8;
                if (cur.blocks + span > rl::kMaxLaunchBlocks) {
                    launches.push_back(cur);
                    cur = Launch{c, seg_map.size(), 0, 0};
                }
                seg_map.push_back(i);
                seg_row0.push_back(P.cell_row0 + r0);
                seg_cells.push_back(nr * P.cells_x);
                seg_first.push_back(cur.blocks);
                cur.blocks += span;
                cur.nseg += 1;
            }
        }
        launches.push_back(cur);
    }
    if (launches.empty()) return RL_OK;

    DeviceGuard dg(ctx->device);
    if (!dg.ok) return hip_fail(dg.err, "hipSetDevice");
    RL_TRY(ensure_ready(ctx));
    hipError_t e;

    // FP32 lens copies for every map, one region per map; inverse masses for
    // the maps that have masses
    if (precision == RL_FP32_COMP) {
        const size_t bytes = (size_t)std::max<int64_t>(total_lens, 1) * (sizeof(float4) + sizeof(float));
        e = ctx->lens.acquire(bytes, stream);
        if (e != hipSuccess) return hip_fail(e, "lens scratch");
        float4* xy = static_cast<float4*>(ctx->lens.ptr);
        float* mf = reinterpret_cast<float*>(xy + std::max<int64_t>(total_lens, 1));
        int64_t off = 0;
        for (int32_t i = 0; i < n_maps; ++i) {
            const rl_lenses& L = h_maps[i].lenses;
            const bool mi = L.m != nullptr;
            e = rl::launch_prep_lenses(L.x1, L.x2, L.m, L.n, xy + off, mi ? mf + off : nullptr, true, stream);
            if (e != hipSuccess) return hip_fail(e, "prep_lenses launch");
            params[i].lens32 = xy + off;
            params[i].imass32 = mi ? mf + off : nullptr;
            off += L.n;
        }
    } else {
        for (int32_t i = 0; i < n_maps; ++i) {
            params[i].lx1 = h_maps[i].lenses.x1;
            params[i].lx2 = h_maps[i].lenses.x2;
            params[i].lm = h_maps[i].lenses.m;
        }
    }

    // records: [MapParams x n_segs][first block x n_segs], segments of one
    // launch contiguous
    const size_t nseg = seg_map.size();
    std::vector<rl::MapParams> segs(nseg);
    for (size_t k = 0; k < nseg; ++k) {
        segs[k] = params[(size_t)seg_map[k]];
        segs[k].cell_row0 = seg_row0[k];
        segs[k].n_cells = seg_cells[k];
    }
    const size_t pbytes = sizeof(rl::MapParams) * nseg;
    const size_t foff = (pbytes + 255) & ~(size_t)255;
    const size_t total = foff + sizeof(int64_t) * nseg;
    char* hs = nullptr;
    RL_TRY(stage_reserve(ctx, total, &hs));
    std::memcpy(hs, segs.data(), pbytes);
    std::memcpy(hs + foff, seg_first.data(), sizeof(int64_t) * nseg);
    e = ctx->batch.acquire(total, stream);
    if (e != hipSuccess) return hip_fail(e, "batch scratch");
    char* ds = static_cast<char*>(ctx->batch.ptr);
    RL_TRY(stage_send(ctx, ds, total, stream));

    const rl::MapParams* dsegs = reinterpret_cast<const rl::MapParams*>(ds);
    const int64_t* dfirst = reinterpret_cast<const int64_t*>(ds + foff);
    e = hipSuccess;
    for (size_t l = 0; l < launches.size() && e == hipSuccess; ++l) {
        const Launch& L = launches[l];
        e = rl::launch_shoot_batch(dsegs + L.seg0, dfirst + L.seg0, (int)L.nseg, L.blocks,
                                   (rl::Precision)precision, L.cls >= 3, ctx->tuning[precision][L.cls],
                                   stream);
    }
    hipError_t e2 = ctx->batch.release(stream);
    hipError_t e3 = precision == RL_FP32_COMP ? ctx->lens.release(stream) : hipSuccess;
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = e3;
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    return RL_OK;
}

rl_status rl_count_histogram(rl_context* ctx, const int32_t* d_counts, const rl_window* win,
                             int64_t n_values, int64_t* d_hist, hipStream_t stream) {
    g_error.clear();
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    RL_TRY(check_counts(d_counts, win));
    if (n_values < 1 || n_values > ((int64_t)1 << 31)) return fail(RL_E_INVALID, "n_values must be in [1, 2^31]");
    if (!d_hist) return fail(RL_E_INVALID, "histogram pointer is NULL");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return hip_fail(dg.err, "hipSetDevice");
    RL_TRY(ensure_ready(ctx));
    hipError_t e = rl::launch_count_hist(d_counts, (int64_t)win->p1 * win->p2, n_values,
                                         reinterpret_cast<unsigned long long*>(d_hist), stream);
    if (e != hipSuccess) return hip_fail(e, "count histogram launch");
    return RL_OK;
}

}  // extern "C"

namespace {

rl_status check_mpd_args(double mu_ref, double log_lo, double log_hi, int32_t nbins, const int64_t* d_bins) {
    if (!is_finite(mu_ref) || !(mu_ref > 0.0)) return fail(RL_E_INVALID, "mu_ref must be finite and > 0");
    if (!is_finite(log_lo) || !is_finite(log_hi) || !(log_hi > log_lo))
        return fail(RL_E_INVALID, "need finite log_lo < log_hi");
    if (nbins < 1 || nbins > rl::kMaxMpdBins) return fail(RL_E_INVALID, "nbins must be in [1, %d]", rl::kMaxMpdBins);
    if (!d_bins) return fail(RL_E_INVALID, "bins pointer is NULL");
    return RL_OK;
}

// Thresholds scale 10^(log_lo + k (log_hi - log_lo) / nbins), k = 0..nbins,
// in FP64 on the host; up to kMpdArgThr of them go with the launch, more
// through scratch. launch(args, thr) starts the binning kernel.
template <typename Launch>
rl_status mpd_with_thresholds(rl_context* ctx, double scale, double log_lo, double log_hi, int32_t nbins,
                              hipStream_t stream, Launch&& launch) {
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return hip_fail(dg.err, "hipSetDevice");
    RL_TRY(ensure_ready(ctx));
    const int nthr = nbins + 1;
    const double step = (log_hi - log_lo) / (double)nbins;
    auto threshold = [&](int k) { return scale * std::pow(10.0, log_lo + (double)k * step); };
    rl::MpdThresholds args{};
    hipError_t e;
    if (nthr <= rl::kMpdArgThr) {
        for (int k = 0; k < nthr; ++k) args.t[k] = threshold(k);
        e = launch(args, static_cast<const double*>(nullptr));
        if (e != hipSuccess) return hip_fail(e, "mpd launch");
        return RL_OK;
    }
    const size_t bytes = (size_t)nthr * sizeof(double);
    char* hs = nullptr;
    RL_TRY(stage_reserve(ctx, bytes, &hs));
    double* thr = reinterpret_cast<double*>(hs);
    for (int k = 0; k < nthr; ++k) thr[k] = threshold(k);
    e = ctx->aux.acquire(bytes, stream);
    if (e != hipSuccess) return hip_fail(e, "threshold scratch");
    RL_TRY(stage_send(ctx, ctx->aux.ptr, bytes, stream));
    e = launch(args, static_cast<const double*>(ctx->aux.ptr));
    hipError_t e2 = ctx->aux.release(stream);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return hip_fail(e, "mpd launch");
    return RL_OK;
}

}  // namespace

extern "C" {
rl_status rl_mpd(rl_context* ctx, const int32_t* d_counts, const rl_window* win, double n_avg,
                 double mu_ref, double log_lo, double log_hi, int32_t nbins, int64_t* d_bins,
                 hipStream_t stream) {
    g_error.clear();
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    RL_TRY(check_counts(d_counts, win));
    if (!is_finite(n_avg) || !(n_avg > 0.0)) return fail(RL_E_INVALID, "n_avg must be finite and > 0");
    RL_TRY(check_mpd_args(mu_ref, log_lo, log_hi, nbins, d_bins));
    // count thresholds: N >= n_avg mu_ref 10^edge
    const int64_t n = (int64_t)win->p1 * win->p2;
    return mpd_with_thresholds(ctx, n_avg * mu_ref, log_lo, log_hi, nbins, stream,
                               [&](const rl::MpdThresholds& a, const double* thr) {
                                   return rl::launch_mpd(d_counts, n, a, thr, nbins + 1,
                                                         reinterpret_cast<unsigned long long*>(d_bins), stream);
                               });
}

rl_status rl_mpd_values(rl_context* ctx, const double* d_mu, const rl_window* win, double mu_ref,
                        double log_lo, double log_hi, int32_t nbins, int64_t* d_bins, hipStream_t stream) {
    g_error.clear();
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    RL_TRY(check_window(win));
    if (!d_mu) return fail(RL_E_INVALID, "map pointer is NULL");
    RL_TRY(check_mpd_args(mu_ref, log_lo, log_hi, nbins, d_bins));
    // magnification thresholds: mu >= mu_ref 10^edge (the count rule with n_avg = 1)
    const int64_t n = (int64_t)win->p1 * win->p2;
    const float c0 = (float)(std::log10(mu_ref) + log_lo);
    const float inv_step = (float)((double)nbins / (log_hi - log_lo));
    return mpd_with_thresholds(ctx, 1.0 * mu_ref, log_lo, log_hi, nbins, stream,
                               [&](const rl::MpdThresholds& a, const double* thr) {
                                   return rl::launch_mpd_values(d_mu, n, a, thr, nbins + 1, c0, inv_step,
                                                                reinterpret_cast<unsigned long long*>(d_bins),
                                                                stream);
                               });
}

rl_status rl_probability_sums(rl_context* ctx, const int32_t* d_counts, const rl_window* win,
                              double n_avg, double mu_lim, int64_t* h_below, int64_t* h_above,
                              hipStream_t stream) {
    g_error.clear();
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    RL_TRY(check_counts(d_counts, win));
    if (!is_finite(n_avg) || !(n_avg > 0.0)) return fail(RL_E_INVALID, "n_avg must be finite and > 0");
    if (std::isnan(mu_lim)) return fail(RL_E_INVALID, "mu_lim is NaN");
    if (!h_below || !h_above) return fail(RL_E_INVALID, "output pointers are NULL");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return hip_fail(dg.err, "hipSetDevice");
    RL_TRY(ensure_ready(ctx));
    const int64_t n = (int64_t)win->p1 * win->p2;
    // N / N_avg in FP64 is non-decreasing in the integer N (IEEE division by a
    // positive number is monotone), so "N / N_avg < mu_lim" holds exactly for
    // N below the first int32 count where it fails: find that count by
    // bisection with the same division (2^31 if it never fails).
    int64_t lo = INT32_MIN, hi = (int64_t)INT32_MAX + 1;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if ((double)mid / n_avg < mu_lim) lo = mid + 1;
        else hi = mid;
    }
    hipError_t e = rl::launch_prob_sum(d_counts, n, lo, ctx->host_read_dev, stream);
    unsigned long long folded[3];
    if (e == hipSuccess) e = fold_reduction(ctx, rl::reduce_blocks(n), stream, folded);
    if (e != hipSuccess) return hip_fail(e, "probability sums");
    const unsigned long long below = folded[0];
    *h_below = (int64_t)below;
    *h_above = n - (int64_t)below;
    return RL_OK;
}

rl_status rl_mpd_moments(rl_context* ctx, const int64_t* d_bins, int32_t n_maps, int32_t n_bins,
                         int64_t n_pix, double* d_mean, double* d_std, hipStream_t stream) {
    g_error.clear();
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    if (!d_bins || !d_mean || !d_std) return fail(RL_E_INVALID, "pointers are NULL");
    if (n_maps < 1 || n_bins < 1 || n_pix < 1) return fail(RL_E_INVALID, "n_maps, n_bins, n_pix must be >= 1");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return hip_fail(dg.err, "hipSetDevice");
    RL_TRY(ensure_ready(ctx));
    hipError_t e = rl::launch_mpd_moments(reinterpret_cast<const unsigned long long*>(d_bins), n_maps,
                                          n_bins, (double)n_pix, d_mean, d_std, stream);
    if (e != hipSuccess) return hip_fail(e, "mpd moments launch");
    return RL_OK;
}

rl_status rl_codec_encode(rl_context* ctx, const int32_t* d_counts, const rl_window* win,
                          int32_t* d_values, int64_t values_capacity, uint32_t* d_packed,
                          int64_t packed_capacity, int64_t* h_n_distinct, int32_t* h_bits,
                          hipStream_t stream) {
    g_error.clear();
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    RL_TRY(check_counts(d_counts, win));
    if (!h_n_distinct || !h_bits) return fail(RL_E_INVALID, "output pointers are NULL");
    const bool size_only = !d_values || !d_packed;
    if (!size_only && (values_capacity < 1 || packed_capacity < 1))
        return fail(RL_E_INVALID, "capacities must be >= 1");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return hip_fail(dg.err, "hipSetDevice");
    RL_TRY(ensure_ready(ctx));
    const int64_t n_pix = (int64_t)win->p1 * win->p2;
    // 1. largest count and negatives
    hipError_t e = rl::launch_count_stats(d_counts, n_pix, nullptr, ctx->host_read_dev, stream);
    unsigned long long host[3];
    if (e == hipSuccess) e = fold_reduction(ctx, rl::reduce_blocks(n_pix), stream, host);
    if (e != hipSuccess) return hip_fail(e, "codec statistics");
    if (host[2]) return fail(RL_E_INVALID, "counts must be >= 0 (%llu negative)", host[2]);
    const int64_t n_values = (int64_t)host[1] + 1;
    // 2. histogram of values, distinct flags and their ranks
    const int64_t nb = rl::scan_blocks(n_values);
    const size_t hist_b = (size_t)n_values * 8, flag_b = (size_t)n_values * 4;
    const size_t off_flag = (hist_b + 255) & ~(size_t)255;
    const size_t off_rank = (off_flag + flag_b + 255) & ~(size_t)255;
    const size_t off_sums = (off_rank + flag_b + 255) & ~(size_t)255;
    const size_t off_total = (off_sums + (size_t)nb * 4 + 255) & ~(size_t)255;
    const size_t need = off_total + 256;
    e = ctx->aux.acquire(need, stream);
    if (e != hipSuccess) return hip_fail(e, "codec scratch");
    char* base = static_cast<char*>(ctx->aux.ptr);
    auto* hist = reinterpret_cast<unsigned long long*>(base);
    auto* flag = reinterpret_cast<int32_t*>(base + off_flag);
    auto* rank = reinterpret_cast<int32_t*>(base + off_rank);
    auto* sums = reinterpret_cast<int32_t*>(base + off_sums);
    auto* total = reinterpret_cast<int64_t*>(base + off_total);
    e = rl::launch_fill_u32(reinterpret_cast<unsigned int*>(hist), n_values * 2, 0u, stream);
    if (e == hipSuccess) e = rl::launch_count_hist(d_counts, n_pix, n_values, hist, stream);
    if (e == hipSuccess) e = rl::launch_distinct_ranks(hist, n_values, flag, rank, sums, total, stream);
    int64_t nd = 0;
    if (e == hipSuccess) e = read_back(ctx, &nd, total, sizeof(nd), stream);
    if (e != hipSuccess) { (void)ctx->aux.release(stream); return hip_fail(e, "codec ranks"); }
    int32_t bits = 1;
    while (bits < 32 && ((int64_t)1 << bits) < nd) ++bits;
    *h_n_distinct = nd;
    *h_bits = bits;
    const int64_t words = (n_pix * bits + 31) / 32;
    if (size_only) {
        e = ctx->aux.release(stream);
        return e == hipSuccess ? RL_OK : hip_fail(e, "codec scratch");
    }
    if (values_capacity < nd || packed_capacity < words) {
        (void)ctx->aux.release(stream);
        return fail(RL_E_INVALID, "need %lld value slots and %lld packed words", (long long)nd,
                    (long long)words);
    }
    // 3. index table and packed map
    e = rl::launch_codec_pack(d_counts, n_pix, flag, rank, n_values, bits, d_values, d_packed, stream);
    const hipError_t e2 = ctx->aux.release(stream);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return hip_fail(e, "codec pack");
    return RL_OK;
}

rl_status rl_codec_decode(rl_context* ctx, const uint32_t* d_packed, int32_t bits,
                          const int32_t* d_values, int64_t n_distinct, const rl_window* win,
                          int32_t* d_counts, hipStream_t stream) {
    g_error.clear();
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    RL_TRY(check_window(win));
    if (!d_packed || !d_values || !d_counts) return fail(RL_E_INVALID, "pointers are NULL");
    if (bits < 1 || bits > 32) return fail(RL_E_INVALID, "bits must be in [1, 32]");
    if (n_distinct < 1) return fail(RL_E_INVALID, "n_distinct must be >= 1");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return hip_fail(dg.err, "hipSetDevice");
    RL_TRY(ensure_ready(ctx));
    hipError_t e = rl::launch_codec_unpack(d_packed, (int64_t)win->p1 * win->p2, bits, d_values,
                                           n_distinct, d_counts, stream);
    if (e != hipSuccess) return hip_fail(e, "codec unpack");
    return RL_OK;
}

rl_status rl_source_kernel(rl_context* ctx, const rl_profile* profile, const rl_window* win,
                           double* d_kernel, hipStream_t stream) {
    g_error.clear();
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    RL_TRY(check_window(win));
    if (!profile || !d_kernel) return fail(RL_E_INVALID, "pointers are NULL");
    if (profile->shape < RL_PROFILE_UNIFORM || profile->shape > RL_PROFILE_POWER)
        return fail(RL_E_INVALID, "unknown profile shape");
    if (!is_finite(profile->radius) || !(profile->radius > 0.0) || !is_finite(profile->hole) ||
        profile->hole < 0.0)
        return fail(RL_E_INVALID, "radius must be finite and > 0, hole finite and >= 0");
    const double pix1 = win->width1 / (double)win->p1, pix2 = win->width2 / (double)win->p2;
    const double h1d = std::ceil(profile->radius / pix1), h2d = std::ceil(profile->radius / pix2);
    if (2.0 * h1d + 1.0 > (double)win->p1 || 2.0 * h2d + 1.0 > (double)win->p2)
        return fail(RL_E_INVALID, "source larger than the map");
    const int h1 = (int)h1d, h2 = (int)h2d;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return hip_fail(dg.err, "hipSetDevice");
    RL_TRY(ensure_ready(ctx));
    hipError_t e = ctx->aux.acquire(rl::source_scratch_bytes(h1, h2), stream);
    if (e != hipSuccess) return hip_fail(e, "source scratch");
    e = rl::launch_source_kernel(profile->shape, profile->radius, profile->hole, pix1, pix2, h1, h2,
                                 win->p1, win->p2, d_kernel, static_cast<double*>(ctx->aux.ptr), stream);
    hipError_t e2 = ctx->aux.release(stream);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return hip_fail(e, "source kernel launch");
    return RL_OK;
}

rl_status rl_source_kernel_table(rl_context* ctx, const float* h_x, int32_t nx, const float* h_y, int32_t ny,
                                 const float* h_b, const rl_window* win, double* d_kernel, hipStream_t stream) {
    g_error.clear();
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    RL_TRY(check_window(win));
    if (!h_x || !h_y || !h_b || !d_kernel) return fail(RL_E_INVALID, "pointers are NULL");
    if (nx < 1 || ny < 1 || nx > RL_MAX_TABLE_AXIS || ny > RL_MAX_TABLE_AXIS)
        return fail(RL_E_INVALID, "table axes must hold 1 .. RL_MAX_TABLE_AXIS samples");
    const double pix1 = win->width1 / (double)win->p1, pix2 = win->width2 / (double)win->p2;
    // The half-widths of the pixel box, in the same FP64 arithmetic as the bins
    // the kernels compute; a position too far out for an int is refused first.
    auto half = [](const float* v, int32_t n, double pix, int32_t p, int32_t* h) -> bool {
        double m = 0.0;
        for (int32_t k = 0; k < n; ++k) {
            if (!is_finite(v[k])) return false;
            const double c = std::floor((double)v[k] / pix + 0.5);
            m = std::max(m, std::fabs(c));
        }
        if (2.0 * m + 1.0 > (double)p) return false;
        *h = (int32_t)m;
        return true;
    };
    int32_t h1 = 0, h2 = 0;
    if (!half(h_x, nx, pix1, win->p1, &h1) || !half(h_y, ny, pix2, win->p2, &h2))
        return fail(RL_E_INVALID, "table positions must be finite and the source no larger than the map");
    // Branch-free over the (millions of) brightness values: NaN, negative and
    // infinite values all fail v >= 0 && v <= FLT_MAX.
    int bad = 0, any = 0;
    const int64_t nb = (int64_t)nx * ny;
    for (int64_t k = 0; k < nb; ++k) {
        const float v = h_b[k];
        bad |= !(v >= 0.0f && v <= FLT_MAX);
        any |= v > 0.0f;
    }
    if (bad) return fail(RL_E_INVALID, "table brightness must be finite and >= 0");
    if (!any) return fail(RL_E_INVALID, "empty source kernel: every brightness is 0");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return hip_fail(dg.err, "hipSetDevice");
    RL_TRY(ensure_ready(ctx));
    const size_t off = rl::table_data_offset(nx, ny, h1, h2);
    const size_t bytes = ((size_t)nx + ny + (size_t)nb) * sizeof(float);
    hipError_t e = ctx->aux.acquire(rl::table_scratch_bytes(nx, ny, h1, h2), stream);
    if (e != hipSuccess) return hip_fail(e, "table scratch");
    char* host = nullptr;
    rl_status st = stage_reserve(ctx, bytes, &host);
    if (st == RL_OK) {
        std::memcpy(host, h_x, (size_t)nx * sizeof(float));
        std::memcpy(host + (size_t)nx * sizeof(float), h_y, (size_t)ny * sizeof(float));
        std::memcpy(host + ((size_t)nx + ny) * sizeof(float), h_b, (size_t)nb * sizeof(float));
        st = stage_send(ctx, static_cast<char*>(ctx->aux.ptr) + off, bytes, stream);
    }
    if (st != RL_OK) {
        (void)ctx->aux.release(stream);
        return st;
    }
    e = rl::launch_table_kernel(nx, ny, pix1, pix2, h1, h2, win->p1, win->p2, d_kernel, ctx->aux.ptr, stream);
    hipError_t e2 = ctx->aux.release(stream);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return hip_fail(e, "table kernel launch");
    return RL_OK;
}

}  // extern "C"

namespace {

// One map against n kernels (n = 1 for rl_convolve); the arrays are host
// arrays of device pointers, validated by the caller.
rl_status convolve_many(rl_context* ctx, const int32_t* d_counts, const double* const* d_kernels,
                        int32_t n, const rl_window* win, double n_avg, double* const* d_outs,
                        hipStream_t stream) {
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return hip_fail(dg.err, "hipSetDevice");
    RL_TRY(ensure_ready(ctx));
    hipError_t e = ctx->fft.acquire(rl::convolve_scratch_bytes(win->p1, win->p2), stream);
    if (e != hipSuccess) return hip_fail(e, "convolution scratch");
    const bool tw_ready = ctx->fft_tw_gen == ctx->fft.gen && ctx->fft_tw_p1 == win->p1 &&
                          ctx->fft_tw_p2 == win->p2;
    e = rl::launch_convolve(d_counts, d_kernels, n, win->p1, win->p2, n_avg, d_outs, ctx->fft.ptr, tw_ready,
                            stream);
    hipError_t e2 = ctx->fft.release(stream);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) {
        ctx->fft_tw_p1 = 0;
        return hip_fail(e, "convolution launch");
    }
    ctx->fft_tw_gen = ctx->fft.gen;
    ctx->fft_tw_p1 = win->p1;
    ctx->fft_tw_p2 = win->p2;
    return RL_OK;
}

rl_status check_convolve(rl_context* ctx, const int32_t* d_counts, const rl_window* win, double n_avg) {
    if (!ctx) return fail(RL_E_INVALID, "context is NULL");
    RL_TRY(check_counts(d_counts, win));
    if (!is_finite(n_avg) || !(n_avg > 0.0)) return fail(RL_E_INVALID, "n_avg must be finite and > 0");
    if (!rl::fft_side_supported(win->p1) || !rl::fft_side_supported(win->p2))
        return fail(RL_E_INVALID, "map sides must be products of 2, 3 and 5 in [2, %d]", rl::kMaxFftSide);
    return RL_OK;
}

}  // namespace

extern "C" {
rl_status rl_convolve(rl_context* ctx, const int32_t* d_counts, const double* d_kernel,
                      const rl_window* win, double n_avg, double* d_out, hipStream_t stream) {
    g_error.clear();
    RL_TRY(check_convolve(ctx, d_counts, win, n_avg));
    if (!d_kernel || !d_out) return fail(RL_E_INVALID, "pointers are NULL");
    return convolve_many(ctx, d_counts, &d_kernel, 1, win, n_avg, &d_out, stream);
}

rl_status rl_convolve_batch(rl_context* ctx, const int32_t* d_counts, const double* const* h_kernels,
                            int32_t n_kernels, const rl_window* win, double n_avg, double* const* h_outs,
                            hipStream_t stream) {
    g_error.clear();
    RL_TRY(check_convolve(ctx, d_counts, win, n_avg));
    if (n_kernels < 1 || n_kernels > RL_MAX_CONVOLVE_BATCH)
        return fail(RL_E_INVALID, "n_kernels must be in [1, %d]", RL_MAX_CONVOLVE_BATCH);
    if (!h_kernels || !h_outs) return fail(RL_E_INVALID, "pointer arrays are NULL");
    // output q is written before kernel q + 1 is read: no output may be a
    // kernel's or the map's buffer, nor another output
    for (int32_t q = 0; q < n_kernels; ++q) {
        if (!h_kernels[q] || !h_outs[q]) return fail(RL_E_INVALID, "kernel or output %d is NULL", q);
        if (static_cast<const void*>(h_outs[q]) == static_cast<const void*>(d_counts))
            return fail(RL_E_INVALID, "output %d is the map's buffer", q);
        for (int32_t r = 0; r < q; ++r)
            if (h_outs[r] == h_outs[q]) return fail(RL_E_INVALID, "outputs %d and %d are the same buffer", r, q);
        for (int32_t r = 0; r < n_kernels; ++r)
            if (h_outs[q] == h_kernels[r]) return fail(RL_E_INVALID, "output %d is kernel %d's buffer", q, r);
    }
    return convolve_many(ctx, d_counts, h_kernels, n_kernels, win, n_avg, h_outs, stream);
}

}  // extern "C"
