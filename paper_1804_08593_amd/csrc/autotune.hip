// Autotuner for the hop traversal: times candidate 4D tiles and the XCD
// remap on the context's own lattice (A in FP64 / FP32, the block operator
// in the local-solve precision) with HIP events, keeps the fastest, and
// caches the choice per (dims, Ls, blocking) in a plain text file.
#include <math.h>
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
    const int opts[][4] = {{0, 0, 0, 0}, {8, 4, 4, 4},   {L[0], 4, 4, 4}, {8, 8, 4, 4},
                           {4, 4, 4, 4}, {L[0], L[1], 2, 2}, {8, 8, 8, 8},   {8, 8, 8, 4},
                           {8, 8, 4, 8}, {4, 8, 8, 8},   {12, 12, 12, 12}, {8, 8, 8, 16}};
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
    snprintf(k, sizeof(k), "dims=%dx%dx%dx%d Ls=%d block=%dx%dx%dx%d pad=%d%s", c->L[0], c->L[1],
             c->L[2], c->L[3], c->Ls, bk ? bk->block[0] : 0, bk ? bk->block[1] : 0,
             bk ? bk->block[2] : 0, bk ? bk->block[3] : 0, bk ? bk->pad : 0,
             bk && bk->form == MSPCG_FORM_SPLIT ? " split" : "");
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
            // the rule of mspcg_set_tuning: a line that breaks it is skipped
            bool ok = true;
            for (int p = 0; p < 3; ++p)
                for (int m = 0; m < 4; ++m) ok = ok && r.tile[p][m] >= 0 && !(r.tile[p][m] & 1);
            if (!ok) continue;
            r.xcd_remap = r.xcd_remap ? 1 : 0;
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
                              hipStream_t st) try {
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
MSPCG_ABI_CATCH

// ---------------------------------------------------------------------------
// Block-shape selection for MSPCG
// ---------------------------------------------------------------------------

namespace {

// deterministic pseudo-random fill in [-1, 1) (SplitMix64 of the index)
__global__ void fill_hash_kernel(double* p, long n, unsigned long long seed) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    p[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

std::vector<mspcg_blocking> block_candidates(const mspcg_ctx* c, int pad, int form) {
    std::vector<mspcg_blocking> v;
    auto ok = [&](int L, int b) { return b >= 2 && !(b & 1) && L % b == 0 && (L == b || L - b >= 2 * pad); };
    // every non-empty set of halved directions, then a quarter in every direction
    for (int mask = 1; mask < 16; ++mask) {
        mspcg_blocking b;
        b.pad = pad;
        b.form = form;
        bool good = true;
        for (int m = 0; m < 4; ++m) {
            b.block[m] = (mask >> m) & 1 ? c->L[m] / 2 : c->L[m];
            good = good && ok(c->L[m], b.block[m]);
        }
        if (good) v.push_back(b);
    }
    mspcg_blocking q;
    q.pad = pad;
    q.form = form;
    bool good = true;
    for (int m = 0; m < 4; ++m) {
        q.block[m] = c->L[m] >= 16 ? c->L[m] / 4 : c->L[m] / 2;
        good = good && ok(c->L[m], q.block[m]);
    }
    if (good) v.push_back(q);
    return v;
}

}  // namespace

extern "C" int mspcg_tune_blocking(mspcg_ctx* c, const mspcg_solve_params* base, int probe_iters,
                                   mspcg_blocking* chosen, hipStream_t st) try {
    if (!c || !base || probe_iters < 0) return MSPCG_EINVAL;
    if (probe_iters == 0 && !(base->tol > 0)) return MSPCG_EINVAL;
    // probe_iters == 0: every candidate is solved to base's tolerance and the
    // shortest time to solution decides
    const bool full = probe_iters == 0;
    if (!c->gauge) return MSPCG_ENOGAUGE;
    MSPCG_HIP(hipSetDevice(c->device));
    const int pad = base->blocking.pad > 0 || base->blocking.block[0] ? base->blocking.pad : 2;
    const int form = base->blocking.block[0] ? base->blocking.form : MSPCG_FORM_DOMAIN;
    std::vector<mspcg_blocking> cands = block_candidates(c, pad, form);
    if (cands.empty()) return MSPCG_EUNSUPPORTED;
    const size_t n = (size_t)c->V4 * c->Ls * 12;
    double2* b = (double2*)c->buf("tb.b", n * sizeof(double2));
    double2* x = (double2*)c->buf("tb.x", n * sizeof(double2));
    if (!b || !x) return MSPCG_ENOMEM;
    hipLaunchKernelGGL(fill_hash_kernel, dim3((unsigned)((2 * n + 255) / 256)), dim3(256), 0, st,
                       (double*)b, (long)(2 * n), 12345ull);
    if (hipGetLastError() != hipSuccess) return MSPCG_EHIP;
    mspcg_solve_params p = *base;
    p.solver = MSPCG_SOLVER_MSPCG;
    p.maxiter = full ? (base->maxiter > 0 ? base->maxiter : 20000) : probe_iters;
    p.tol = full ? base->tol : 1e-300;
    p.use_x0 = 0;
    p.timing = 0;
    p.rhs_normal = 0;
    double best = -1;
    mspcg_blocking bestb = cands[0];
    std::vector<double> hist(full ? 1 : probe_iters + 1);
    for (const mspcg_blocking& cb : cands) {
        p.blocking = cb;
        mspcg_solve_stats s;
        memset(&s, 0, sizeof(s));
        s.resid_history = hist.data();
        s.resid_history_cap = full ? 0 : probe_iters;
        // a first, short run builds the domain links outside the timed one
        mspcg_solve_params p1 = p;
        p1.maxiter = full ? 1 : p.maxiter;
        p1.tol = 1e-300;
        int e = solve_one(c, b, x, &p1, &s, st);
        if (e != MSPCG_OK && e != MSPCG_ENOCONV) return e;
        e = solve_one(c, b, x, &p, &s, st);
        if (e != MSPCG_OK && e != MSPCG_ENOCONV) return e;
        if (!(s.seconds > 0)) continue;
        double rate;
        if (full) {
            if (e != MSPCG_OK) continue;  // did not reach the tolerance
            rate = 1.0 / s.seconds;
        } else {
            if (s.resid_history_len < 1) continue;
            const double r = hist[s.resid_history_len - 1];
            if (!(r > 0)) continue;
            rate = -log(r) / s.seconds;  // e-folds of residual per second
        }
        if (rate > best) {
            best = rate;
            bestb = cb;
        }
    }
    c->blocking = bestb;
    c->has_blocking = true;
    if (chosen) *chosen = bestb;
    return MSPCG_OK;
}
MSPCG_ABI_CATCH
