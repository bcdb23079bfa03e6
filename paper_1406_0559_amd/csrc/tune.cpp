// Kernel-shape autotuner of the raylens library (rl_autotune).
//
// The tuner is a client of the library's own C-ABI: it shoots probe maps with
// rl_shoot / rl_shoot_batch under every candidate shape set with
// rl_set_tuning, times them with HIP events, checks that every shape gives
// the same counts (no shape may change a result bit), and keeps the fastest
// shape per precision and tuning class. The table is written to a JSON cache
// and applied from it on later calls, as long as the library build and the
// device architecture match.
//
// Probes: a GERLUMPH-like macro model (kappa = 0.41, gamma = 0.38, s = 0, a
// 1024^2-pixel window of 25 Einstein radii) with lenses uniform in a disc of
// radius sqrt(N / kappa_*), N = 400 / 2624 / 16000 for the three lens-count
// classes, unit masses or masses spread over [0.5, 1.5] for the mass classes,
// and enough rays to keep every SIMD busy for many rounds of waves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "internal.h"
#include "raylens.h"

namespace {

// ---------------------------------------------------------------------------
// a small JSON reader for the cache (objects, arrays, strings, numbers,
// true / false / null)
// ---------------------------------------------------------------------------

struct JValue {
    enum Kind { Null, Bool, Num, Str, Arr, Obj } kind = Null;
    bool b = false;
    double num = 0.0;
    std::string str;
    std::vector<JValue> arr;
    std::vector<std::pair<std::string, JValue>> obj;

    const JValue* get(const char* key) const {
        if (kind != Obj) return nullptr;
        for (const auto& kv : obj)
            if (kv.first == key) return &kv.second;
        return nullptr;
    }
};

struct JParser {
    const char* p;
    const char* end;
    bool ok = true;

    void ws() {
        while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
    }
    bool lit(const char* s) {
        const size_t n = std::strlen(s);
        if ((size_t)(end - p) < n || std::strncmp(p, s, n) != 0) return false;
        p += n;
        return true;
    }
    bool string(std::string* out) {
        if (p >= end || *p != '"') return false;
        ++p;
        out->clear();
        while (p < end && *p != '"') {
            char c = *p++;
            if (c == '\\') {
                if (p >= end) return false;
                const char e = *p++;
                switch (e) {
                    case 'n': c = '\n'; break;
                    case 't': c = '\t'; break;
                    case 'r': c = '\r'; break;
                    case 'b': c = '\b'; break;
                    case 'f': c = '\f'; break;
                    case 'u':  // keep the escape as text: the cache holds ASCII only
                        out->append("\\u");
                        continue;
                    default: c = e; break;
                }
            }
            out->push_back(c);
        }
        if (p >= end) return false;
        ++p;
        return true;
    }
    bool value(JValue* v, int depth) {
        if (depth > 32) return false;
        ws();
        if (p >= end) return false;
        if (*p == '{') {
            ++p;
            v->kind = JValue::Obj;
            ws();
            if (p < end && *p == '}') { ++p; return true; }
            for (;;) {
                ws();
                std::string k;
                if (!string(&k)) return false;
                ws();
                if (p >= end || *p != ':') return false;
                ++p;
                JValue child;
                if (!value(&child, depth + 1)) return false;
                v->obj.emplace_back(std::move(k), std::move(child));
                ws();
                if (p < end && *p == ',') { ++p; continue; }
                if (p < end && *p == '}') { ++p; return true; }
                return false;
            }
        }
        if (*p == '[') {
            ++p;
            v->kind = JValue::Arr;
            ws();
            if (p < end && *p == ']') { ++p; return true; }
            for (;;) {
                JValue child;
                if (!value(&child, depth + 1)) return false;
                v->arr.push_back(std::move(child));
                ws();
                if (p < end && *p == ',') { ++p; continue; }
                if (p < end && *p == ']') { ++p; return true; }
                return false;
            }
        }
        if (*p == '"') {
            v->kind = JValue::Str;
            return string(&v->str);
        }
        if (lit("true")) { v->kind = JValue::Bool; v->b = true; return true; }
        if (lit("false")) { v->kind = JValue::Bool; v->b = false; return true; }
        if (lit("null")) { v->kind = JValue::Null; return true; }
        char* q = nullptr;
        const std::string tok(p, (size_t)std::min<ptrdiff_t>(end - p, 64));
        v->num = std::strtod(tok.c_str(), &q);
        if (q == tok.c_str()) return false;
        p += q - tok.c_str();
        v->kind = JValue::Num;
        return true;
    }
};

bool parse_json(const std::string& text, JValue* out) {
    JParser jp{text.data(), text.data() + text.size()};
    if (!jp.value(out, 0)) return false;
    jp.ws();
    return jp.p == jp.end;
}

bool read_file(const char* path, std::string* out) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return false;
    char buf[4096];
    size_t n;
    out->clear();
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) out->append(buf, n);
    const bool err = std::ferror(f) != 0;
    std::fclose(f);
    return !err;
}

// ---------------------------------------------------------------------------
// tuning classes and candidate shapes
// ---------------------------------------------------------------------------

const char* prec_name(int p) { return p == RL_FP32_COMP ? "fp32c" : "fp64"; }

// Probe lens counts per class: near the geometric middle of 100..1000 for
// the small fields, the bench map's count for the middle class, 16000 for
// large fields.
constexpr int kClassLenses[3] = {300, 2624, 16000};

std::vector<rl_tuning> ray_shapes(int prec) {
    if (prec == RL_FP64_PLAIN) return {rl_tuning{4, 4, 256, 4, 1}};
    return {rl_tuning{4, 4, 256, 4, 1}, rl_tuning{2, 8, 256, 4, 1}, rl_tuning{8, 2, 256, 4, 1},
            rl_tuning{4, 8, 256, 4, 1}, rl_tuning{8, 4, 256, 4, 1}};
}

// ---------------------------------------------------------------------------
// probes
// ---------------------------------------------------------------------------

// splitmix64: a counter-based generator, deterministic across platforms
struct SplitMix {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

struct DeviceBuf {
    void* p = nullptr;
    ~DeviceBuf() { if (p) (void)hipFree(p); }
    hipError_t alloc(size_t n) { return hipMalloc(&p, n ? n : 1); }
};

// One probe map and its lens field in device memory.
struct Probe {
    rl_macro macro{0.41, 0.38, 0.0};
    rl_raygrid grid{};
    rl_window win{1024, 1024, 0.0, 0.0, 25.0, 25.0};
    rl_lenses lenses{};
    DeviceBuf x1, x2, m, counts, escaped;
    int64_t evals = 0;

    hipError_t make(int64_t n_lens, bool masses, int64_t rays, uint64_t seed) {
        // ray rectangle of the GERLUMPH-like workload: half-widths 65 x 14.2
        const double h1 = 65.0, h2 = 14.2;
        int64_t n2 = (int64_t)std::sqrt((double)rays * h2 / h1);
        n2 = std::max<int64_t>(n2, 16);
        const int64_t n1 = std::max<int64_t>(64, rays / n2);
        grid = rl_raygrid{n1, n2, 0.0, 0.0, h1, h2};
        evals = n1 * n2 * n_lens;
        const double R = std::sqrt((double)n_lens / (0.41 * (1.0 - macro.s)));
        std::vector<double> hx((size_t)n_lens), hy((size_t)n_lens), hm((size_t)n_lens);
        SplitMix g{seed};
        for (int64_t k = 0; k < n_lens; ++k) {
            const double r = R * std::sqrt(g.uniform()), t = 6.283185307179586 * g.uniform();
            hx[(size_t)k] = r * std::cos(t);
            hy[(size_t)k] = r * std::sin(t);
            hm[(size_t)k] = 0.5 + g.uniform();
        }
        const size_t nb = (size_t)n_lens * sizeof(double);
        hipError_t e;
        if ((e = x1.alloc(nb)) != hipSuccess || (e = x2.alloc(nb)) != hipSuccess) return e;
        if ((e = hipMemcpy(x1.p, hx.data(), nb, hipMemcpyHostToDevice)) != hipSuccess) return e;
        if ((e = hipMemcpy(x2.p, hy.data(), nb, hipMemcpyHostToDevice)) != hipSuccess) return e;
        if (masses) {
            if ((e = m.alloc(nb)) != hipSuccess) return e;
            if ((e = hipMemcpy(m.p, hm.data(), nb, hipMemcpyHostToDevice)) != hipSuccess) return e;
        }
        lenses = rl_lenses{static_cast<double*>(x1.p), static_cast<double*>(x2.p),
                           masses ? static_cast<double*>(m.p) : nullptr, n_lens};
        if ((e = counts.alloc((size_t)win.p1 * win.p2 * sizeof(int32_t))) != hipSuccess) return e;
        return escaped.alloc(sizeof(int64_t));
    }
    size_t map_bytes() const { return (size_t)win.p1 * win.p2 * sizeof(int32_t); }
};

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    hipError_t init() {
        hipError_t e = hipEventCreate(&a);
        return e == hipSuccess ? hipEventCreate(&b) : e;
    }
};

struct Result {
    double ms;
    rl_tuning t;
};

std::string shape_json(const rl_tuning& t) {
    char buf[200];
    std::snprintf(buf, sizeof buf,
                  "{\"lens_tile\": %d, \"rays_x\": %d, \"rays_y\": %d, "
                  "\"submap\": %d, \"waves\": %d}",
                  t.lens_tile, t.rays_x, t.rays_y, t.submap, t.waves);
    return buf;
}

bool same_shape(const rl_tuning& a, const rl_tuning& b) {
    return a.rays_x == b.rays_x && a.rays_y == b.rays_y && a.lens_tile == b.lens_tile &&
           a.waves == b.waves && a.submap == b.submap;
}

using Clock = std::chrono::steady_clock;

struct Tuner {
    rl_context* ctx;
    Clock::time_point deadline;
    int reps = 2;
    bool out_of_time = false;

    bool time_left() {
        if (Clock::now() >= deadline) out_of_time = true;
        return !out_of_time;
    }

    // Best-of-reps time of one rl_shoot of the probe (after one warm-up run),
    // and the counts it produced.
    rl_status time_shoot(Probe& pr, int prec, Timer& tm, double* ms, std::vector<int32_t>* counts) {
        *ms = 1e300;
        for (int r = 0; r <= reps; ++r) {
            hipError_t e = hipMemsetAsync(pr.counts.p, 0, pr.map_bytes(), nullptr);
            if (e == hipSuccess) e = hipMemsetAsync(pr.escaped.p, 0, sizeof(int64_t), nullptr);
            if (e == hipSuccess) e = hipEventRecord(tm.a, nullptr);
            if (e != hipSuccess) return rl::set_error(RL_E_DEVICE, hipGetErrorString(e));
            rl_status st = rl_shoot(ctx, &pr.lenses, &pr.macro, &pr.grid, &pr.win, prec,
                                    0, pr.grid.n2, static_cast<int32_t*>(pr.counts.p),
                                    static_cast<int64_t*>(pr.escaped.p), nullptr);
            if (st != RL_OK) return st;
            e = hipEventRecord(tm.b, nullptr);
            if (e == hipSuccess) e = hipEventSynchronize(tm.b);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, tm.a, tm.b);
            if (e != hipSuccess) return rl::set_error(RL_E_DEVICE, hipGetErrorString(e));
            if (r > 0) *ms = std::min(*ms, (double)t);
        }
        counts->resize((size_t)pr.win.p1 * pr.win.p2);
        hipError_t e = hipMemcpy(counts->data(), pr.counts.p, pr.map_bytes(), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return rl::set_error(RL_E_DEVICE, hipGetErrorString(e));
        return RL_OK;
    }

    // Tunes one (precision, class) entry; appends its JSON to `json`.
    rl_status tune_entry(int prec, int cls, std::string* json) {
        const int lc = cls % 3;
        const bool masses = cls >= 3;
        const int64_t n_lens = kClassLenses[lc];
        // >= 16 rounds of 256 CUs x 4 SIMDs x 3 waves of 1024-ray cells
        const int64_t min_rays = (int64_t)16 * 256 * 4 * 3 * 1024 / (prec == RL_FP64_PLAIN ? 4 : 1);
        const double target = prec == RL_FP64_PLAIN ? 5e10 : 2e11;
        const int64_t rays = std::max<int64_t>(min_rays, (int64_t)(target / (double)n_lens));
        Probe pr;
        hipError_t e = pr.make(n_lens, masses, rays, 0x5EED0000ull + (uint64_t)cls);
        if (e != hipSuccess) return rl::set_error(RL_E_NOMEM, "probe allocation failed");
        Timer tm;
        if ((e = tm.init()) != hipSuccess) return rl::set_error(RL_E_DEVICE, hipGetErrorString(e));

        std::vector<int32_t> ref, got;
        std::vector<Result> results;
        auto run = [&](rl_tuning t) -> rl_status {
            for (const Result& r : results)
                if (same_shape(r.t, t)) return RL_OK;
            // shapes the library does not support (e.g. a tile that is not a
            // whole number of compensation blocks) are skipped
            if (rl_set_tuning(ctx, prec, cls, &t) != RL_OK) return RL_OK;
            double ms;
            const rl_status st = time_shoot(pr, prec, tm, &ms, &got);
            if (st != RL_OK) return st;
            if (ref.empty()) {
                ref = got;
            } else if (got != ref) {
                return rl::set_error(RL_E_DEVICE,
                                     "kernel shape %dx%d tile %d waves %d submap %d changed the counts",
                                     t.rays_x, t.rays_y, t.lens_tile, t.waves, t.submap);
            }
            results.push_back(Result{ms, t});
            return RL_OK;
        };
        // stage 1: rays per lane at a middle tile; stage 2: every tile, wave
        // count and binning mode for the three best ray shapes
        for (const rl_tuning& t : ray_shapes(prec)) {
            if (!time_left() && !results.empty()) break;
            RL_TRY(run(t));
        }
        std::vector<Result> stage1 = results;
        std::sort(stage1.begin(), stage1.end(), [](const Result& a, const Result& b) { return a.ms < b.ms; });
        const size_t top = std::min<size_t>(3, stage1.size());
        for (size_t i = 0; i < top && time_left(); ++i)
            for (int tile : {256, 512, 1024, 2048})
                for (int waves : {1, 2, 4})
                    for (int sub : {1, 2}) {
                        if (!time_left()) break;
                        rl_tuning t = stage1[i].t;
                        t.lens_tile = tile;
                        t.waves = waves;
                        t.submap = sub;
                        RL_TRY(run(t));
                    }
        std::sort(results.begin(), results.end(), [](const Result& a, const Result& b) { return a.ms < b.ms; });
        rl_tuning best = results.front().t;

        RL_TRY(rl_set_tuning(ctx, prec, cls, &best));

        char head[512];
        std::snprintf(head, sizeof head,
                      "  \"%s/%d\": {\"shape\": %s, \"probe_lenses\": %lld, \"probe_masses\": %s, "
                      "\"probe_evals\": %lld, \"best_ms\": %.6g, \"worst_ms\": %.6g, "
                      "\"probe_evals_per_s\": %.6g, \"candidates\": %zu, \"top5\": [",
                      prec_name(prec), cls, shape_json(best).c_str(), (long long)n_lens,
                      masses ? "true" : "false", (long long)pr.evals, results.front().ms, results.back().ms,
                      (double)pr.evals / (results.front().ms * 1e-3), results.size());
        *json += head;
        for (size_t i = 0; i < std::min<size_t>(5, results.size()); ++i) {
            std::string s = shape_json(results[i].t);
            char ms[48];
            std::snprintf(ms, sizeof ms, ", \"ms\": %.6g}", results[i].ms);
            s.pop_back();
            *json += (i ? ", " : "") + s + ms;
        }
        *json += "]}";
        return RL_OK;
    }
};

std::string device_arch(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// Applies a cache file if it was written by this library build for this
// architecture. Returns true if it was applied.
bool apply_cache(rl_context* ctx, const char* path, const std::string& arch) {
    std::string text;
    JValue root;
    if (!path || !read_file(path, &text) || !parse_json(text, &root)) return false;
    const JValue* lib = root.get("library");
    const JValue* ar = root.get("arch");
    const JValue* ent = root.get("entries");
    if (!lib || lib->kind != JValue::Str || lib->str != rl_version()) return false;
    if (!ar || ar->kind != JValue::Str || ar->str != arch) return false;
    if (!ent || ent->kind != JValue::Obj) return false;
    // validate everything before applying anything
    std::vector<std::pair<std::pair<int, int>, rl_tuning>> todo;
    for (const auto& kv : ent->obj) {
        const std::string& key = kv.first;
        const size_t slash = key.find('/');
        if (slash == std::string::npos) return false;
        const std::string pn = key.substr(0, slash);
        const int prec = pn == "fp32c" ? RL_FP32_COMP : (pn == "fp64" ? RL_FP64_PLAIN : -1);
        const int cls = std::atoi(key.c_str() + slash + 1);
        const JValue* sh = kv.second.get("shape");
        if (prec < 0 || !sh) return false;
        int v[5];
        const char* names[5] = {"rays_x", "rays_y", "lens_tile", "waves", "submap"};
        for (int i = 0; i < 5; ++i) {
            const JValue* x = sh->get(names[i]);
            if (!x || x->kind != JValue::Num) return false;
            v[i] = (int)x->num;
        }
        todo.push_back({{prec, cls}, rl_tuning{v[0], v[1], v[2], v[3], v[4]}});
    }
    std::vector<rl_tuning> saved;
    for (const auto& t : todo) {
        rl_tuning cur;
        if (rl_get_tuning(ctx, t.first.first, t.first.second, &cur) != RL_OK) return false;
        if (rl_set_tuning(ctx, t.first.first, t.first.second, &t.second) != RL_OK) {
            // undo what was applied so far
            for (size_t i = 0; i < saved.size(); ++i)
                (void)rl_set_tuning(ctx, todo[i].first.first, todo[i].first.second, &saved[i]);
            return false;
        }
        saved.push_back(cur);
    }
    return true;
}

}  // namespace

extern "C" rl_status rl_autotune(rl_context* ctx, const char* cache_path, int32_t budget_ms) {
    rl::clear_error();
    if (!ctx) return rl::set_error(RL_E_INVALID, "context is NULL");
    if (budget_ms < 0) return rl::set_error(RL_E_INVALID, "budget_ms must be >= 0");
    const int device = rl::context_device(ctx);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev)
        return rl::set_error(RL_E_DEVICE, "no HIP device %d", device);
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess) return rl::set_error(RL_E_DEVICE, "hipSetDevice failed");
    struct Restore {
        int d;
        ~Restore() { (void)hipSetDevice(d); }
    } restore{prev};

    const std::string arch = device_arch(device);
    if (apply_cache(ctx, cache_path, arch)) return RL_OK;
    if (budget_ms == 0)
        return rl::set_error(RL_E_INVALID, "no tuning cache for this library build at %s",
                             cache_path ? cache_path : "(null)");

    Tuner tu{ctx, Clock::now() + std::chrono::milliseconds(budget_ms)};
    // RL_AUTOTUNE_LOG=1 prints one line per tuned class to stderr
    const char* env = std::getenv("RL_AUTOTUNE_LOG");
    const bool log = env && env[0] && env[0] != '0';
    std::string body;
    // FP32 first (the production path), unit then mass-weighted fields,
    // the middle lens-count class first
    const int order[6] = {1, 0, 2, 4, 3, 5};
    bool first = true;
    for (int prec : {(int)RL_FP32_COMP, (int)RL_FP64_PLAIN}) {
        for (int cls : order) {
            if (!tu.time_left()) break;
            std::string one;
            const auto t0 = Clock::now();
            rl_status st = tu.tune_entry(prec, cls, &one);
            if (st != RL_OK) return st;
            if (log) {
                rl_tuning t;
                (void)rl_get_tuning(ctx, prec, cls, &t);
                std::fprintf(stderr, "rl_autotune: %s class %d -> %dx%d tile %d waves %d submap %d (%.1f s)\n",
                             prec_name(prec), cls, t.rays_x, t.rays_y, t.lens_tile, t.waves, t.submap,
                             std::chrono::duration<double>(Clock::now() - t0).count());
                std::fflush(stderr);
            }
            body += (first ? "" : ",\n") + one;
            first = false;
        }
    }
    if (cache_path) {
        const std::string tmp = std::string(cache_path) + ".tmp";
        FILE* f = std::fopen(tmp.c_str(), "wb");
        if (!f) return rl::set_error(RL_E_INVALID, "cannot write %s", tmp.c_str());
        std::fprintf(f, "{\"arch\": \"%s\", \"library\": \"%s\", \"complete\": %s, \"budget_ms\": %d,\n"
                        "\"entries\": {\n%s\n}}\n",
                     arch.c_str(), rl_version(), tu.out_of_time ? "false" : "true", budget_ms, body.c_str());
        const bool bad = std::fclose(f) != 0;
        if (bad || std::rename(tmp.c_str(), cache_path) != 0)
            return rl::set_error(RL_E_INVALID, "cannot write %s", cache_path);
    }
    return RL_OK;
}
