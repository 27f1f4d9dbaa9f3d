// Autotuner for the hop traversal: times candidate 4D tiles and the XCD
// remap on the context's own lattice (A in FP64 / FP32, the block operator
// in the local-solve precision) with HIP events, keeps the fastest, and
// caches the choice per (dims, Ls, blocking) in a plain text file.
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "ctx.h"

namespace mspcg {

namespace {

struct Cand {
    int remap;
    int tile[4];
};

std::vector<Cand> candidates(const int L[4]) {
    std::vector<Cand> v;
    const int opts[][4] = {{0, 0, 0, 0}, {8, 4, 4, 4}, {L[0], 4, 4, 4}, {8, 8, 4, 4},
                           {4, 4, 4, 4}, {L[0], L[1], 2, 2}, {8, 8, 8, 8}};
    for (auto& o : opts) {
        Cand c;
        c.remap = 1;
        memcpy(c.tile, o, sizeof(c.tile));
        v.push_back(c);
    }
    Cand c0;
    c0.remap = 0;
    memset(c0.tile, 0, sizeof(c0.tile));
    v.push_back(c0);
    return v;
}

// average time of `reps` calls of f() on the stream, after one warm-up call
template <class F>
int time_ms(hipStream_t st, int reps, F f, float& ms) {
    hipEvent_t a, b;
    MSPCG_HIP(hipEventCreate(&a));
    MSPCG_HIP(hipEventCreate(&b));
    int e = f();
    if (e) return e;
    MSPCG_HIP(hipEventRecord(a, st));
    for (int i = 0; i < reps; ++i)
        if ((e = f())) return e;
    MSPCG_HIP(hipEventRecord(b, st));
    MSPCG_HIP(hipEventSynchronize(b));
    MSPCG_HIP(hipEventElapsedTime(&ms, a, b));
    ms /= reps;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return 0;
}

std::string cache_key(const mspcg_ctx* c, const mspcg_blocking* bk) {
    char k[256];
    snprintf(k, sizeof(k), "dims=%dx%dx%dx%d Ls=%d block=%dx%dx%dx%d pad=%d", c->L[0], c->L[1],
             c->L[2], c->L[3], c->Ls, bk ? bk->block[0] : 0, bk ? bk->block[1] : 0,
             bk ? bk->block[2] : 0, bk ? bk->block[3] : 0, bk ? bk->pad : 0);
    return k;
}

bool cache_lookup(const char* path, const std::string& key, mspcg_tuning& t) {
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof(line), f)) {
        const char* bar = strchr(line, '|');
        if (!bar || std::string(line, bar - line) != key) continue;
        mspcg_tuning r;
        if (sscanf(bar + 1, " remap=%d t64=%d,%d,%d,%d t32=%d,%d,%d,%d t16=%d,%d,%d,%d", &r.xcd_remap,
                   &r.tile[0][0], &r.tile[0][1], &r.tile[0][2], &r.tile[0][3], &r.tile[1][0],
                   &r.tile[1][1], &r.tile[1][2], &r.tile[1][3], &r.tile[2][0], &r.tile[2][1],
                   &r.tile[2][2], &r.tile[2][3]) == 13) {
            t = r;
            found = true;
        }
    }
    fclose(f);
    return found;
}

void cache_store(const char* path, const std::string& key, const mspcg_tuning& t) {
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s| remap=%d t64=%d,%d,%d,%d t32=%d,%d,%d,%d t16=%d,%d,%d,%d\n", key.c_str(),
            t.xcd_remap, t.tile[0][0], t.tile[0][1], t.tile[0][2], t.tile[0][3], t.tile[1][0],
            t.tile[1][1], t.tile[1][2], t.tile[1][3], t.tile[2][0], t.tile[2][1], t.tile[2][2],
            t.tile[2][3]);
    fclose(f);
}

}  // namespace

}  // namespace mspcg

using namespace mspcg;

extern "C" int mspcg_autotune(mspcg_ctx* c, const mspcg_blocking* bk, const char* cache_path,
                              hipStream_t st) {
    if (!c) return MSPCG_EINVAL;
    if (!c->gauge) return MSPCG_ENOGAUGE;
    MSPCG_HIP(hipSetDevice(c->device));
    const std::string key = cache_key(c, bk);
    mspcg_tuning t = c->tune;
    if (cache_path && cache_lookup(cache_path, key, t)) {
        c->tune = t;
        return MSPCG_OK;
    }
    const bool was_timing = c->timing;
    c->timing = false;
    const std::vector<Cand> cands = candidates(c->L);
    int e;
    // whole-lattice A in FP64 and FP32
    Field<F64> p64 = half_field<F64>(c, "d.cg_p", c->Nh);
    Field<F64> q64 = half_field<F64>(c, "d.cg_q", c->Nh);
    Field<F32> p32 = half_field<F32>(c, "s.cg_p", c->Nh);
    Field<F32> q32 = half_field<F32>(c, "s.cg_q", c->Nh);
    if (!p64.data || !q64.data || !p32.data || !q32.data) return MSPCG_ENOMEM;
    MSPCG_HIP(hipMemsetAsync(p64.data, 0, (size_t)12 * c->Nh * sizeof(double2), st));
    MSPCG_HIP(hipMemsetAsync(p32.data, 0, (size_t)12 * c->Nh * sizeof(float2), st));
    const int reps = 3;
    int best_remap = 1;
    for (int prec = MSPCG_FP64; prec <= MSPCG_FP32; ++prec) {
        float best = 1e30f;
        Cand bc = cands[0];
        for (const Cand& cd : cands) {
            c->tune.xcd_remap = cd.remap;
            memcpy(c->tune.tile[prec], cd.tile, sizeof(cd.tile));
            float ms = 0;
            if (prec == MSPCG_FP64)
                e = time_ms(st, reps, [&] { return op_A<F64>(c, q64, cfield(p64), nullptr, nullptr, st); }, ms);
            else
                e = time_ms(st, reps, [&] { return op_A<F32>(c, q32, cfield(p32), nullptr, nullptr, st); }, ms);
            if (e) return e;
            if (ms < best) {
                best = ms;
                bc = cd;
            }
        }
        memcpy(t.tile[prec], bc.tile, sizeof(bc.tile));
        if (prec == MSPCG_FP64) best_remap = bc.remap;
        c->tune = t;
    }
    t.xcd_remap = best_remap;
    // block operator of the local solves (FP16 storage)
    if (bk) {
        c->tune = t;
        if ((e = domains_setup(c, *bk, MSPCG_FP16, st))) return e;
        const Domains& D = c->dom;
        const long n = (long)D.ndom * D.interior.Vh * c->Ls;
        Field<F16> p = half_field<F16>(c, "dom16.p", n);
        Field<F16> w = half_field<F16>(c, "dom16.w", n);
        if (!p.data || !w.data) return MSPCG_ENOMEM;
        MSPCG_HIP(hipMemsetAsync(p.data, 0, (size_t)12 * n * sizeof(__half2), st));
        MSPCG_HIP(hipMemsetAsync(p.scale, 0, (size_t)n * sizeof(float), st));
        float best = 1e30f;
        Cand bc = cands[0];
        for (const Cand& cd : cands) {
            if (cd.remap != t.xcd_remap) continue;
            memcpy(c->tune.tile[MSPCG_FP16], cd.tile, sizeof(cd.tile));
            float ms = 0;
            if ((e = time_ms(st, reps, [&] { return block_A<F16>(c, w, cfield(p), nullptr, nullptr, st); }, ms)))
                return e;
            if (ms < best) {
                best = ms;
                bc = cd;
            }
        }
        memcpy(t.tile[MSPCG_FP16], bc.tile, sizeof(bc.tile));
    }
    c->tune = t;
    c->timing = was_timing;
    if (cache_path) cache_store(cache_path, key, t);
    return MSPCG_OK;
}
