// Self-tuning of kick launch shapes.  GENGA II picks its kernel parameters
// at start-up by timing them (Sect. 8); here candidate shapes are timed on
// the caller's own bodies, with a zero step factor so the state is not
// modified, and the fastest is kept, optionally in a plain-text cache file
// (one line per problem: key, shape, time; the last line of a key wins).
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "genga_internal.h"

namespace genga {
namespace {


struct Shape {
    int block = 0, ipt = 0, tile_cols = 0, grid = 0, slices = 0;
    int flags = 0;   // single system: GENGA_FLAG_DIRECTED or GENGA_FLAG_SYMMETRIC (0: library choice)
};

std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

int cus()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
        return 256;
    return v;
}

// Batch signature: S, total bodies and a histogram of log2 system sizes.
std::string batch_key(const genga_batch *bt, int precision)
{
    int hist[8] = {0};
    for (int64_t s = 0; s < bt->S; ++s) {
        const double ns = (double)(bt->offsets[s + 1] - bt->offsets[s]);
        int b = (int)std::floor(std::log2(ns) / 2.0);
        hist[std::min(std::max(b, 0), 7)] += 1;
    }
    char buf[256];
    snprintf(buf, sizeof buf, "batch:two-kicks:%s:p%d:S%lld:N%lld:h%d.%d.%d.%d.%d.%d.%d.%d",
             arch_name().c_str(), precision, (long long)bt->S, (long long)bt->offsets[bt->S],
             hist[0], hist[1], hist[2], hist[3], hist[4], hist[5], hist[6], hist[7]);
    return buf;
}

std::string single_key(int64_t n, int precision)
{
    int64_t bucket = 1;
    while (bucket < n) bucket <<= 1;
    char buf[128];
    snprintf(buf, sizeof buf, "single:%s:p%d:N%lld", arch_name().c_str(), precision,
             (long long)bucket);
    return buf;
}

bool cache_lookup(const char *path, const std::string &key, Shape &out, double &ms)
{
    if (!path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[512], k[384];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        Shape s;
        double t = 0.0;
        // (the kick-form flags are an optional eighth field)
        if (sscanf(line, "%383s %d %d %d %d %d %lf %d", k, &s.block, &s.ipt, &s.tile_cols, &s.grid,
                   &s.slices, &t, &s.flags) >= 7 &&
            key == k) {
            out = s;
            ms = t;
            found = true;
        }
    }
    fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &key, const Shape &s, double ms)
{
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d %d %d %.6f %d\n", key.c_str(), s.block, s.ipt, s.tile_cols, s.grid,
            s.slices, ms, s.flags);
    fclose(f);
}

void apply(const Shape &s, genga_params *p)
{
    p->block = s.block;
    p->ipt = s.ipt;
    p->tile_cols = s.tile_cols;
    p->grid = s.grid;
    p->slices = s.slices;
}

// Median over `reps` timed calls after one untimed call; < 0 on failure.
template <class F>
double time_ms(F &&call, hipStream_t s, int reps)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.0;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.0;
    }
    std::vector<float> t;
    bool ok = call() == GENGA_OK;
    for (int r = 0; ok && r < reps; ++r) {
        ok = hipEventRecord(e0, s) == hipSuccess && call() == GENGA_OK &&
             hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.0f;
        if (ok) ok = hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        t.push_back(ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!ok || t.empty()) return -1.0;
    std::sort(t.begin(), t.end());
    return (double)t[t.size() / 2];
}

// (binary64) the symmetric form with the plan's own slice width first, then
// with 1, 2 or 4 column slices per 512-row group (widths 512, 256, 128), and
// the one-sided tile shapes.
std::vector<Shape> batch_candidates(const genga_params *p)
{
    std::vector<Shape> v;
    if (p->precision == GENGA_FP64)
        for (int sl : {0, 1, 2, 4}) {
            Shape s;
            s.slices = sl;
            s.flags = GENGA_FLAG_SYMMETRIC;
            v.push_back(s);
        }
    const int cu = cus();
    for (int block : {64, KB})
        for (int ipt : {1, 2})
            for (int cols : {256, 512, 1024, 2048})
                for (int g : {0, cu * (32 * 64 / block)}) {
                    Shape s;
                    s.block = block;
                    s.ipt = ipt;
                    s.tile_cols = cols;
                    s.grid = g;
                    s.flags = GENGA_FLAG_DIRECTED;
                    v.push_back(s);
                }
    return v;
}

// One-sided form: rows per thread x column slices; symmetric form (binary64
// or mixed, every body massive): slice widths (slices d = 1, 2, 4, 8 of a
// 512-row group, or the library's width).
std::vector<Shape> single_candidates(const genga_params *p)
{
    std::vector<Shape> v;
    for (int ipt : {1, 2})
        for (int sl : {0, 8, 16, 32, 64}) {
            Shape s;
            s.ipt = ipt;
            s.slices = sl;
            s.flags = GENGA_FLAG_DIRECTED;
            v.push_back(s);
        }
    if (p->tp_mode == 0)
        for (int sl : {0, 1, 2, 4, 8}) {
            Shape s;
            s.slices = sl;
            s.flags = GENGA_FLAG_SYMMETRIC;
            v.push_back(s);
        }
    return v;
}

constexpr int FORM_FLAGS = GENGA_FLAG_DIRECTED | GENGA_FLAG_SYMMETRIC;

genga_params timing_params(const genga_params *p)
{
    genga_params q = *p;
    for (auto &e : q.prof_events) e = nullptr;
    return q;
}

}  // namespace
}  // namespace genga

using namespace genga;

extern "C" {

// The largest workspace any batched candidate needs.
static size_t batch_candidates_bytes(const genga_batch *bt, const genga_params *p)
{
    size_t most = 0;
    for (const Shape &s : batch_candidates(p)) {
        genga_params q = *p;
        apply(s, &q);
        q.flags = (p->flags & ~FORM_FLAGS) | s.flags;
        most = std::max(most, genga_batch_workspace_bytes(bt, &q));
    }
    return most;
}

// The batched tuner's encounter list, after the candidates' workspace: one
// int64 count, then TUNE_PAIRS_PER_BODY pairs per body (a list that
// overflows still counts its pairs and times the same work).
constexpr int64_t TUNE_PAIRS_PER_BODY = 16;

static size_t align_256(size_t v) { return (v + 255) & ~(size_t)255; }

static size_t tune_pair_bytes(const genga_batch *bt)
{
    const int64_t cap = TUNE_PAIRS_PER_BODY * std::max<int64_t>(bt->offsets[bt->S], 1);
    return 256 + 2 * align_256(sizeof(int32_t) * (size_t)cap);
}

size_t genga_autotune_batched_workspace_bytes(const genga_batch *bt, const genga_params *p)
{
    if (!p || !bt || !bt->offsets || bt->S < 1) return 0;
    const size_t most = batch_candidates_bytes(bt, p);
    return most ? align_256(most) + tune_pair_bytes(bt) : 0;
}

int genga_autotune_batched(const genga_bodies *b, const genga_batch *bt, genga_params *p,
                           void *ws, size_t ws_bytes, const char *cache_path, double *ms_out,
                           void *stream)
{
    if (!b || !bt || !p || !ws || !bt->offsets || bt->S < 1) return GENGA_E_INVAL;
    if (genga_batch_workspace_bytes(bt, p) == 0) return GENGA_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    const std::string key = batch_key(bt, p->precision);
    // a step's two kicks: one without the encounter list and one with it
    // (the list costs the symmetric form more the narrower its slices); the
    // list sits after the largest candidate's workspace when it fits, else
    // both timed kicks go without it
    const size_t lo = align_256(batch_candidates_bytes(bt, p));
    genga_pairs list{nullptr, nullptr, 0, nullptr};
    genga_pairs *plist = nullptr;
    if (lo > 0 && ws_bytes >= lo + tune_pair_bytes(bt)) {
        char *w = (char *)ws + lo;
        const int64_t cap = TUNE_PAIRS_PER_BODY * std::max<int64_t>(bt->offsets[bt->S], 1);
        list.count = (int64_t *)w;
        list.i = (int32_t *)(w + 256);
        list.j = (int32_t *)(w + 256 + align_256(sizeof(int32_t) * (size_t)cap));
        list.capacity = cap;
        plist = &list;
    }
    Shape best;
    double best_ms = -1.0;
    if (!cache_lookup(cache_path, key, best, best_ms)) {
        best_ms = -1.0;
        for (const Shape &c : batch_candidates(p)) {
            genga_params q = timing_params(p);
            apply(c, &q);
            q.flags = (p->flags & ~FORM_FLAGS) | c.flags;
            const size_t need = genga_batch_workspace_bytes(bt, &q);
            if (need == 0 || need > ws_bytes || (plist && need > lo)) continue;
            if (genga_batch_plan(bt, &q, ws, stream) != GENGA_OK) continue;
            const double ms = time_ms(
                [&] {
                    const int r = genga_kick_batched(b, bt, &q, 0.0, nullptr, nullptr, nullptr,
                                                     nullptr, ws, stream);
                    if (r != GENGA_OK) return r;
                    return genga_kick_batched(b, bt, &q, 0.0, nullptr, nullptr, nullptr, plist,
                                              ws, stream);
                },
                s, 5);
            // a later candidate has to be faster by more than the timing's
            // noise (1 %): the plan's own choice, timed first, wins ties
            if (ms >= 0.0 && (best_ms < 0.0 || ms < 0.99 * best_ms)) {
                best_ms = ms;
                best = c;
            }
        }
        if (best_ms < 0.0) return GENGA_E_UNSUPPORTED;
        cache_store(cache_path, key, best, best_ms);
    }
    apply(best, p);
    p->flags = (p->flags & ~FORM_FLAGS) | (best.flags & FORM_FLAGS);
    if (genga_batch_workspace_bytes(bt, p) > ws_bytes) return GENGA_E_INVAL;
    const int r = genga_batch_plan(bt, p, ws, stream);
    if (r != GENGA_OK) return r;
    if (ms_out) *ms_out = best_ms;
    return GENGA_OK;
}

size_t genga_autotune_workspace_bytes(int64_t n, const genga_params *p)
{
    if (!p || n < 1) return 0;
    size_t most = 0;
    for (const Shape &s : single_candidates(p)) {
        genga_params q = *p;
        apply(s, &q);
        q.flags = (p->flags & ~FORM_FLAGS) | s.flags;
        most = std::max(most, genga_workspace_bytes(n, &q));
    }
    return most;
}

int genga_autotune(const genga_bodies *b, genga_params *p, void *ws, size_t ws_bytes,
                   const char *cache_path, double *ms_out, void *stream)
{
    if (!b || !p || !ws || b->n < 1) return GENGA_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    const std::string key = single_key(b->n, p->precision);
    Shape best;
    double best_ms = -1.0;
    if (!cache_lookup(cache_path, key, best, best_ms)) {
        best_ms = -1.0;
        for (const Shape &c : single_candidates(p)) {
            genga_params q = timing_params(p);
            apply(c, &q);
            q.flags = (p->flags & ~FORM_FLAGS) | c.flags;
            q.block = p->block;
            q.tile_cols = p->tile_cols;
            q.grid = p->grid;
            if (genga_workspace_bytes(b->n, &q) > ws_bytes) continue;
            const double ms = time_ms(
                [&] {
                    return genga_kick(b, &q, 0.0, nullptr, nullptr, nullptr, nullptr, ws, stream);
                },
                s, 3);
            if (ms >= 0.0 && (best_ms < 0.0 || ms < best_ms)) {
                best_ms = ms;
                best = c;
            }
        }
        if (best_ms < 0.0) return GENGA_E_UNSUPPORTED;
        cache_store(cache_path, key, best, best_ms);
    }
    p->ipt = best.ipt;
    p->slices = best.slices;
    p->flags = (p->flags & ~FORM_FLAGS) | (best.flags & FORM_FLAGS);
    if (ms_out) *ms_out = best_ms;
    return GENGA_OK;
}

int genga_tune_levels(genga_bodies *b, genga_params *p, const int *levels, const int *substeps,
                      int ncand, int steps, void *ws, size_t ws_bytes, double *ms_out,
                      void *stream)
{
    if (!b || !p || !ws || !levels || !substeps || ncand < 1 || steps < 1) return GENGA_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return GENGA_E_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return GENGA_E_HIP;
    }
    int best = -1;
    double best_ms = -1.0;
    for (int c = 0; c < ncand; ++c) {
        genga_params q = timing_params(p);
        q.slevels = levels[c];
        q.substeps = substeps[c];
        q.flags |= GENGA_FLAG_NOSYNC;
        double ms = -1.0;
        const size_t need = genga_workspace_bytes(b->n, &q);
        // one untimed step (first use of this layout), then `steps` timed ones
        if (need > 0 && need <= ws_bytes && genga_step(b, &q, nullptr, ws, stream) == GENGA_OK) {
            bool ok = hipEventRecord(e0, s) == hipSuccess;
            for (int k = 0; ok && k < steps; ++k) ok = genga_step(b, &q, nullptr, ws, stream) == GENGA_OK;
            ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
            float t = 0.0f;
            if (ok && hipEventElapsedTime(&t, e0, e1) == hipSuccess &&
                genga_read_status(ws, stream) == GENGA_OK)
                ms = (double)t / steps;
        }
        if (ms_out) ms_out[c] = ms;
        if (ms >= 0.0 && (best < 0 || ms < best_ms)) {
            best = c;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best < 0) return GENGA_E_UNSUPPORTED;
    p->slevels = levels[best];
    p->substeps = substeps[best];
    return GENGA_OK;
}

}  // extern "C"
