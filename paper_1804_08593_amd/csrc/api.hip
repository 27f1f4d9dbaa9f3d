// C ABI entry points (context, gauge, operator application) and the
// whole-lattice operator compositions:
//   Mhat   = M5op - (1/4) D_h^eo X D_h^oe B,          X = B M5op^-1
//   Mhat^+ = M5op^+ - (1/4) B^+ Dd^eo X^+ Dd^oe        (Dd = dagger hop = g5 D_h g5)
//   A      = Mhat^+ Mhat,  <p, A p> = |Mhat p|^2 fused into the Mhat epilogue.
// Each composition is one 5D kernel plus hops whose 5D factors run as fused
// epilogues (fived.h), i.e. 5 launches per application of A.
#include <math.h>
#include <string.h>

#include <new>

#include "ctx.h"

using namespace mspcg;

namespace mspcg {

FiveDProg scaled(FiveDProg p, double s_up, double s_dn) {
    p.scale[0] *= s_up;
    p.scale[1] *= s_dn;
    return p;
}

static FiveDProg prog_scale(double s) {
    FiveDProg p;
    memset(&p, 0, sizeof(p));
    p.scale[0] = p.scale[1] = s;
    p.identity = 1;
    return p;
}

static void prog_push(FiveDProg& p, int kind, int dag, double a) {
    if (kind == STEP_BIDI && a == 0.0) return;
    p.kind[p.nsteps] = kind;
    p.dag[p.nsteps] = dag;
    p.a[p.nsteps] = a;
    p.nsteps++;
    p.identity = 0;
}

static Progs make_progs(const mspcg_action& a, double alpha, double q) {
    Progs r;
    const double cb = a.c / a.b;
    r.id = prog_scale(1.0);
    r.B = prog_scale(a.b);
    prog_push(r.B, STEP_BIDI, 0, cb);
    r.Bdag = prog_scale(a.b);
    prog_push(r.Bdag, STEP_BIDI, 1, cb);
    // X = B M5op^-1 = (b/alpha) (1 + (c/b) K) (1 - q K)^-1
    r.X = prog_scale(a.b / alpha);
    prog_push(r.X, STEP_INV, 0, q);
    prog_push(r.X, STEP_BIDI, 0, cb);
    // X^+ = (b/alpha) (1 - q K^+)^-1 (1 + (c/b) K^+)
    r.Xdag = prog_scale(a.b / alpha);
    prog_push(r.Xdag, STEP_BIDI, 1, cb);
    prog_push(r.Xdag, STEP_INV, 1, q);
    // M5op = alpha (1 - q K)
    r.M5 = prog_scale(alpha);
    prog_push(r.M5, STEP_BIDI, 0, -q);
    r.M5dag = prog_scale(alpha);
    prog_push(r.M5dag, STEP_BIDI, 1, -q);
    r.M5inv = prog_scale(1.0 / alpha);
    prog_push(r.M5inv, STEP_INV, 0, q);
    r.M5invdag = prog_scale(1.0 / alpha);
    prog_push(r.M5invdag, STEP_INV, 1, q);
    return r;
}

Timed::Timed(mspcg_ctx* c_, int kc_, double bytes_, hipStream_t st_)
    : c(c_), kc(kc_), bytes(bytes_), st(st_) {
    if (!c->timing) return;
    if (c->evused + 2 > c->evpool.size()) {
        for (int i = 0; i < 64; ++i) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            c->evpool.push_back(e);
        }
    }
    a = c->evpool[c->evused++];
    b = c->evpool[c->evused++];
    (void)hipEventRecord(a, st);
}

Timed::~Timed() {
    if (!a) return;
    (void)hipEventRecord(b, st);
    c->trecs.push_back({kc, a, b, bytes});
}

void timing_reset(mspcg_ctx* c) {
    c->trecs.clear();
    c->evused = 0;
}

void timing_collect(mspcg_ctx* c, mspcg_solve_stats* st) {
    if (!st) return;
    for (int k = 0; k < MSPCG_KC_COUNT; ++k) {
        st->kernel_ms[k] = 0;
        st->kernel_launches[k] = 0;
        st->kernel_bytes[k] = 0;
    }
    for (auto& r : c->trecs) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            st->kernel_ms[r.kc] += ms;
            st->kernel_launches[r.kc] += 1;
            st->kernel_bytes[r.kc] += r.bytes;
        }
    }
    timing_reset(c);
}

int ensure_partials(mspcg_ctx* c, size_t n) {
    if (n <= c->partials_len) return 0;
    if (c->partials) (void)hipFree(c->partials);
    c->partials = nullptr;
    c->partials_len = 0;
    if (hipMalloc(&c->partials, n * sizeof(double)) != hipSuccess) return MSPCG_ENOMEM;
    c->partials_len = n;
    return 0;
}

template <class S>
Field<S> half_field(mspcg_ctx* c, const std::string& name, long N) {
    Field<S> f;
    f.N = N;
    f.ls = c->Ls;
    f.data = (typename S::elem*)c->buf(name, (size_t)N * 12 * sizeof(typename S::elem));
    f.scale = S::has_scale ? (float*)c->buf(name + ".scale", (size_t)N * sizeof(float)) : nullptr;
    return f;
}
template Field<F64> half_field<F64>(mspcg_ctx*, const std::string&, long);
template Field<F32> half_field<F32>(mspcg_ctx*, const std::string&, long);
template Field<F16> half_field<F16>(mspcg_ctx*, const std::string&, long);

template <>
F64::elem* links_of<F64>(mspcg_ctx* c) { return c->L64; }
template <>
F32::elem* links_of<F32>(mspcg_ctx* c) { return c->L32; }
template <>
F16::elem* links_of<F16>(mspcg_ctx* c) { return c->L16; }

long hop_nparts(mspcg_ctx* c) { return hop_grid_x<F64>(c->Vh, c->Ls); }

void pick_tile(const int pref[4], const Box& b, int out[4]) {
    bool any = false;
    for (int m = 0; m < 4; ++m) any = any || pref[m] > 0;
    for (int m = 0; m < 4; ++m) {
        out[m] = 0;
        if (!any) continue;
        int t = pref[m] > 0 ? pref[m] : b.E[m];
        if (t > b.E[m]) t = b.E[m];
        t &= ~1;
        while (t > 2 && b.E[m] % t) t -= 2;
        out[m] = t < 2 ? 2 : t;
    }
}

template <>
int prec_index<F64>() { return MSPCG_FP64; }
template <>
int prec_index<F32>() { return MSPCG_FP32; }
template <>
int prec_index<F16>() { return MSPCG_FP16; }

template <class S>
static int kc_hop() {
    return std::is_same<S, F64>::value ? MSPCG_KC_HOP64
                                       : (std::is_same<S, F32>::value ? MSPCG_KC_HOP32
                                                                      : MSPCG_KC_HOPDOM);
}

template <class S>
static int op_hop_ex(mspcg_ctx* c, Field<S> out, CField<S> in, int out_par, bool dag,
                     const FiveDProg& ph, const CField<S>* aux, const FiveDProg& pa,
                     double* partials, const int* done, const CgUpdate<S>* cg, hipStream_t st) {
    HopArgs<S> a;
    memset(&a, 0, sizeof(a));
    a.in = in;
    a.out = out;
    if (aux) a.aux = *aux;
    a.links = links_of<S>(c);
    a.link_dom_stride = 0;
    a.g.out = a.g.in = a.g.aux = a.g.link = c->lat;
    a.g.out_par = out_par;
    a.g.periodic = 0xF;
    a.ph = ph;
    a.pa = pa;
    a.has_aux = aux != nullptr;
    a.mf = c->act.mf;
    a.partials = partials;
    a.done = done;
    a.xcd_remap = c->tune.xcd_remap;
    pick_tile(c->tune.tile[prec_index<S>()], c->lat, a.tile);
    // spinor passes: in, out, aux; a fused CG update reads r, x, p and writes
    // r, x (and out only if it is kept)
    int passes = 2 + (aux ? 1 : 0);
    if (cg) {
        a.cg_r = cg->r;
        a.cg_x = cg->x;
        a.cg_p = cg->p;
        a.cg_sc = cg->sc;
        a.cg_keep_out = cg->keep_out;
        passes += 5 - (cg->keep_out ? 0 : 1);
    }
    const double bytes = (double)c->Nh * S::bytes_spinor * passes + (double)c->Vh * 8 * S::bytes_link;
    Timed t(c, cg ? MSPCG_KC_HOPCG : kc_hop<S>(), bytes, st);
    return launch_hop<S>(a, c->Ls, 1, dag, st);
}

template <class S>
int op_hop(mspcg_ctx* c, Field<S> out, CField<S> in, int out_par, bool dag, const FiveDProg& ph,
           const CField<S>* aux, const FiveDProg& pa, double* partials, const int* done,
           hipStream_t st) {
    return op_hop_ex<S>(c, out, in, out_par, dag, ph, aux, pa, partials, done, nullptr, st);
}

template <class S>
int op_fived(mspcg_ctx* c, Field<S> out, CField<S> in, const FiveDProg& p, double* partials,
             const int* done, hipStream_t st) {
    FiveDArgs<S> a;
    memset(&a, 0, sizeof(a));
    a.in = in;
    a.out = out;
    a.Vh = c->Vh;
    a.p = p;
    a.mf = c->act.mf;
    a.partials = partials;
    a.done = done;
    Timed t(c, MSPCG_KC_FIVED, (double)c->Nh * S::bytes_spinor * 2, st);
    return launch_fived<S>(a, c->Ls, 1, st);
}

template <class S>
int op_mhat(mspcg_ctx* c, Field<S> y, CField<S> p, double* partials, const int* done,
            hipStream_t st) {
    const std::string pfx = std::is_same<S, F64>::value ? "d." : "s.";
    Field<S> t = half_field<S>(c, pfx + "mh_t", c->Nh);
    Field<S> u = half_field<S>(c, pfx + "mh_u", c->Nh);
    int e;
    if ((e = op_fived<S>(c, t, p, c->pr.B, nullptr, done, st))) return e;
    if ((e = op_hop<S>(c, u, cfield(t), 1, false, c->pr.X, nullptr, c->pr.id, nullptr, done, st)))
        return e;
    return op_hop<S>(c, y, cfield(u), 0, false, prog_scale(-0.25), &p, c->pr.M5, partials, done, st);
}

template <class S>
int op_mhatdag(mspcg_ctx* c, Field<S> q, CField<S> y, const int* done, hipStream_t st) {
    const std::string pfx = std::is_same<S, F64>::value ? "d." : "s.";
    Field<S> v = half_field<S>(c, pfx + "mh_v", c->Nh);
    int e;
    if ((e = op_hop<S>(c, v, y, 1, true, c->pr.Xdag, nullptr, c->pr.id, nullptr, done, st)))
        return e;
    return op_hop<S>(c, q, cfield(v), 0, true, scaled(c->pr.Bdag, -0.25, -0.25), &y, c->pr.M5dag,
                     nullptr, done, st);
}

// One CG step around q = A p with the vector updates fused into the operator
// kernels: p = src + beta p rides on the first 5D kernel (t = B p), alpha =
// (flexible ? zr : rr) / |Mhat p|^2 is formed after the Mhat half, and the last
// hop does r -= alpha q, x += alpha p with |r|^2 partials (q stored only when
// keep_q).  The caller follows with launch_cg_beta over hop_nparts partials.
template <class S>
int cg_step(mspcg_ctx* c, Field<S> x, Field<S> r, Field<S> p, Field<S> q, CField<S> src,
            bool keep_q, bool flexible, const int* done, hipStream_t st) {
    const std::string pfx = std::is_same<S, F64>::value ? "d." : "s.";
    Field<S> t = half_field<S>(c, pfx + "mh_t", c->Nh);
    Field<S> u = half_field<S>(c, pfx + "mh_u", c->Nh);
    Field<S> y = half_field<S>(c, pfx + "A_y", c->Nh);
    Field<S> v = half_field<S>(c, pfx + "mh_v", c->Nh);
    if (!t.data || !u.data || !y.data || !v.data) return MSPCG_ENOMEM;
    int e;
    {
        FiveDArgs<S> a;
        memset(&a, 0, sizeof(a));
        a.in = cfield(p);
        a.out = t;
        a.Vh = c->Vh;
        a.p = c->pr.B;
        a.mf = c->act.mf;
        a.done = done;
        a.xp_src = src;
        a.xp_in = p;
        a.xp_sc = c->sc;
        Timed tm(c, MSPCG_KC_FIVED, (double)c->Nh * S::bytes_spinor * 4, st);
        if (launch_fived<S>(a, c->Ls, 1, st)) return MSPCG_EHIP;
    }
    const CField<S> pc = cfield(p);
    if ((e = op_hop<S>(c, u, cfield(t), 1, false, c->pr.X, nullptr, c->pr.id, nullptr, done, st)))
        return e;
    if ((e = op_hop<S>(c, y, cfield(u), 0, false, prog_scale(-0.25), &pc, c->pr.M5, c->partials,
                       done, st)))
        return e;
    if (launch_cg_alpha(c->sc, c->partials, (int)hop_nparts(c), st, flexible ? 1 : 0))
        return MSPCG_EHIP;
    if ((e = op_hop<S>(c, v, cfield(y), 1, true, c->pr.Xdag, nullptr, c->pr.id, nullptr, done, st)))
        return e;
    CgUpdate<S> cg;
    cg.r = r;
    cg.x = x;
    cg.p = pc;
    cg.sc = c->sc;
    cg.keep_out = keep_q ? 1 : 0;
    const CField<S> yc = cfield(y);
    return op_hop_ex<S>(c, q, cfield(v), 0, true, scaled(c->pr.Bdag, -0.25, -0.25), &yc,
                        c->pr.M5dag, c->partials, done, &cg, st);
}
template int cg_step<F64>(mspcg_ctx*, Field<F64>, Field<F64>, Field<F64>, Field<F64>, CField<F64>,
                          bool, bool, const int*, hipStream_t);
template int cg_step<F32>(mspcg_ctx*, Field<F32>, Field<F32>, Field<F32>, Field<F32>, CField<F32>,
                          bool, bool, const int*, hipStream_t);

template <class S>
int op_A(mspcg_ctx* c, Field<S> q, CField<S> p, double* partials, const int* done,
         hipStream_t st) {
    const std::string pfx = std::is_same<S, F64>::value ? "d." : "s.";
    Field<S> y = half_field<S>(c, pfx + "A_y", c->Nh);
    int e;
    if ((e = op_mhat<S>(c, y, p, partials, done, st))) return e;
    return op_mhatdag<S>(c, q, cfield(y), done, st);
}

#define MSPCG_OPS(S)                                                                             \
    template int op_hop<S>(mspcg_ctx*, Field<S>, CField<S>, int, bool, const FiveDProg&,         \
                           const CField<S>*, const FiveDProg&, double*, const int*, hipStream_t); \
    template int op_fived<S>(mspcg_ctx*, Field<S>, CField<S>, const FiveDProg&, double*,         \
                             const int*, hipStream_t);                                           \
    template int op_mhat<S>(mspcg_ctx*, Field<S>, CField<S>, double*, const int*, hipStream_t);  \
    template int op_mhatdag<S>(mspcg_ctx*, Field<S>, CField<S>, const int*, hipStream_t);        \
    template int op_A<S>(mspcg_ctx*, Field<S>, CField<S>, double*, const int*, hipStream_t);
MSPCG_OPS(F64)
MSPCG_OPS(F32)

}  // namespace mspcg

void* mspcg_ctx::buf(const std::string& name, size_t bytes) {
    if (arena) {
        auto a = arena_slots.find(name);
        if (a != arena_slots.end()) return a->second.second >= bytes ? arena + a->second.first : nullptr;
        const size_t off = (arena_used + 255) & ~(size_t)255;
        if (off + bytes > arena_cap) return nullptr;
        arena_slots[name] = {off, bytes};
        arena_used = off + bytes;
        return arena + off;
    }
    auto it = bufs.find(name);
    if (it != bufs.end() && it->second.second >= bytes) return it->second.first;
    if (it != bufs.end()) {
        (void)hipFree(it->second.first);
        bufs.erase(it);
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    bufs[name] = {p, bytes};
    return p;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

static bool ls_supported(int Ls) {
    switch (Ls) {
#define MSPCG_CASE(L) \
    case L: return true;
        MSPCG_LS_LIST(MSPCG_CASE)
#undef MSPCG_CASE
        default: return false;
    }
}

extern "C" int mspcg_version(void) { return MSPCG_VERSION; }

extern "C" const char* mspcg_strerror(int code) {
    switch (code) {
        case MSPCG_OK: return "ok";
        case MSPCG_EINVAL: return "invalid argument";
        case MSPCG_ENOMEM: return "allocation failed";
        case MSPCG_EHIP: return "HIP runtime error";
        case MSPCG_ENOGAUGE: return "gauge field not loaded";
        case MSPCG_ENOCONV: return "solver did not converge within maxiter";
        case MSPCG_EBREAKDOWN: return "solver breakdown (non-positive curvature or non-finite value)";
        case MSPCG_EUNSUPPORTED: return "unsupported Ls or option";
        case MSPCG_ESCRATCH: return "lattice too large for the fixed scratch of the allocation-free entry point";
        case MSPCG_EINTERNAL: return "internal host-side failure";
        default: return "unknown error";
    }
}

extern "C" int mspcg_create(const mspcg_action* a, int device, mspcg_ctx** out) try {
    if (!a || !out) return MSPCG_EINVAL;
    *out = nullptr;
    for (int m = 0; m < 4; ++m)
        if (a->dims[m] < 2 || (a->dims[m] & 1)) return MSPCG_EINVAL;
    if (a->Ls < 2) return MSPCG_EINVAL;
    if (!ls_supported(a->Ls)) return MSPCG_EUNSUPPORTED;
    if (!isfinite(a->M5) || !isfinite(a->mf) || !isfinite(a->b) || !isfinite(a->c) || a->b == 0.0)
        return MSPCG_EINVAL;
    const double alpha = (4.0 - a->M5) * a->b + 1.0;
    const double beta = (4.0 - a->M5) * a->c - 1.0;
    if (alpha == 0.0) return MSPCG_EINVAL;
    const double q = -beta / alpha;
    if (fabs(1.0 + a->mf * pow(q, a->Ls)) < 1e-300) return MSPCG_EINVAL;
    const long V4 = (long)a->dims[0] * a->dims[1] * a->dims[2] * a->dims[3];
    if (V4 / 2 > (1L << 31) / a->Ls) return MSPCG_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return MSPCG_EHIP;
    if (hipSetDevice(device) != hipSuccess) return MSPCG_EHIP;
    if (int e = noalloc_init(device)) return e;
    mspcg_ctx* c = new (std::nothrow) mspcg_ctx();
    if (!c) return MSPCG_ENOMEM;
    c->act = *a;
    c->device = device;
    for (int m = 0; m < 4; ++m) c->L[m] = a->dims[m];
    c->Ls = a->Ls;
    c->V4 = V4;
    c->Vh = V4 / 2;
    c->Nh = c->Vh * a->Ls;
    c->alpha5 = alpha;
    c->beta5 = beta;
    c->q5 = q;
    c->pr = make_progs(*a, alpha, q);
    for (int m = 0; m < 4; ++m) {
        c->lat.E[m] = a->dims[m];
        c->lat.off[m] = 0;
    }
    c->lat.Vh = c->Vh;
    c->U = nullptr;
    c->L64 = nullptr;
    c->L32 = nullptr;
    c->L16 = nullptr;
    c->gauge = false;
    c->gauge_gen = 0;
    // the domain-wall construction needs a negative Wilson mass -M5 in
    // (-2, 0) for one light mode bound to the walls; other values are
    // accepted and flagged
    c->warnings = (a->M5 > 0.0 && a->M5 < 2.0) ? 0 : MSPCG_WARN_M5_RANGE;
    c->partials = nullptr;
    c->partials_len = 0;
    c->has_blocking = false;
    c->arena = nullptr;
    c->arena_cap = c->arena_used = 0;
    memset(&c->dom, 0, sizeof(c->dom));
    c->timing = false;
    c->evused = 0;
    // measured defaults: 4D tiles help the FP64/FP32 whole-lattice hop, the
    // lexicographic order is best for the FP16 block hops
    c->tune.xcd_remap = 1;
    const int t64[4] = {8, 4, 4, 4};
    for (int m = 0; m < 4; ++m) {
        c->tune.tile[MSPCG_FP64][m] = t64[m];
        c->tune.tile[MSPCG_FP32][m] = t64[m];
        c->tune.tile[MSPCG_FP16][m] = 0;
    }
    c->hist_cap = 0;
    c->hist = nullptr;
    if (hipMalloc(&c->sc, sizeof(DevScalars)) != hipSuccess ||
        hipHostMalloc(&c->sc_host, sizeof(DevScalars), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return MSPCG_ENOMEM;
    }
    *out = c;
    return MSPCG_OK;
}
MSPCG_ABI_CATCH

extern "C" void mspcg_destroy(mspcg_ctx* c) try {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : c->bufs) (void)hipFree(kv.second.first);
    if (c->U) (void)hipFree(c->U);
    if (c->L64) (void)hipFree(c->L64);
    if (c->L32) (void)hipFree(c->L32);
    if (c->L16) (void)hipFree(c->L16);
    if (c->partials) (void)hipFree(c->partials);
    if (c->hist) (void)hipFree(c->hist);
    if (c->dom.links) (void)hipFree(c->dom.links);
    if (c->dom.list_y) (void)hipFree(c->dom.list_y);
    if (c->dom.list_v) (void)hipFree(c->dom.list_v);
    (void)hipFree(c->sc);
    (void)hipHostFree(c->sc_host);
    for (auto e : c->evpool) (void)hipEventDestroy(e);
    delete c;
} catch (...) {
}

extern "C" int mspcg_load_gauge(mspcg_ctx* c, const void* U_dev, hipStream_t st) try {
    if (!c || !U_dev) return MSPCG_EINVAL;
    MSPCG_HIP(hipSetDevice(c->device));
    const size_t n = (size_t)4 * c->V4 * 9;
    const size_t nl = (size_t)2 * 8 * 9 * c->Vh;
    if (!c->U && hipMalloc(&c->U, n * sizeof(double2)) != hipSuccess) return MSPCG_ENOMEM;
    if (!c->L64 && hipMalloc(&c->L64, nl * sizeof(double2)) != hipSuccess) return MSPCG_ENOMEM;
    if (!c->L32 && hipMalloc(&c->L32, nl * sizeof(float2)) != hipSuccess) return MSPCG_ENOMEM;
    if (!c->L16 && hipMalloc(&c->L16, nl * sizeof(__half2)) != hipSuccess) return MSPCG_ENOMEM;
    MSPCG_HIP(hipMemcpyAsync(c->U, U_dev, n * sizeof(double2), hipMemcpyDeviceToDevice, st));
    const int one[4] = {1, 1, 1, 1};
    int e;
    if ((e = launch_pack_links<F64>(c->U, c->L64, c->L, c->L, one, c->lat, c->act.antiperiodic_t, st)))
        return MSPCG_EHIP;
    if ((e = launch_pack_links<F32>(c->U, c->L32, c->L, c->L, one, c->lat, c->act.antiperiodic_t, st)))
        return MSPCG_EHIP;
    if ((e = launch_pack_links<F16>(c->U, c->L16, c->L, c->L, one, c->lat, c->act.antiperiodic_t, st)))
        return MSPCG_EHIP;
    c->gauge = true;
    ++c->gauge_gen;
    c->dom.built = false;  // domain links depend on the gauge field
    return MSPCG_OK;
}
MSPCG_ABI_CATCH

extern "C" int mspcg_gauge_generation(mspcg_ctx* c, unsigned long long* gen) try {
    if (!c || !gen) return MSPCG_EINVAL;
    *gen = c->gauge_gen;
    return MSPCG_OK;
}
MSPCG_ABI_CATCH

extern "C" int mspcg_get_warnings(mspcg_ctx* c, int* warnings) try {
    if (!c || !warnings) return MSPCG_EINVAL;
    *warnings = c->warnings;
    return MSPCG_OK;
}
MSPCG_ABI_CATCH

template <class S>
static int apply_prec(mspcg_ctx* c, int op, const double2* in, double2* out, hipStream_t st) {
    const std::string pfx = std::is_same<S, F64>::value ? "d." : "s.";
    Field<S> ie = half_field<S>(c, pfx + "ap_ie", c->Nh);
    Field<S> io = half_field<S>(c, pfx + "ap_io", c->Nh);
    Field<S> oe = half_field<S>(c, pfx + "ap_oe", c->Nh);
    Field<S> oo = half_field<S>(c, pfx + "ap_oo", c->Nh);
    if (!ie.data || !io.data || !oe.data || !oo.data) return MSPCG_ENOMEM;
    const bool full = op == MSPCG_OP_D || op == MSPCG_OP_DDAG || op == MSPCG_OP_HOP ||
                      op == MSPCG_OP_HOPDAG || op == MSPCG_OP_M5INV || op == MSPCG_OP_PREPARE;
    int e = 0;
#define T_(x)                           \
    do {                                \
        if ((e = (x)) != 0) return e < 0 ? MSPCG_EHIP : e; \
    } while (0)
    T_(launch_pack_parity<S>(in, ie, c->L, c->Ls, 0, st));
    if (full) T_(launch_pack_parity<S>(in, io, c->L, c->Ls, 1, st));
    const Progs& P = c->pr;
    switch (op) {
        case MSPCG_OP_D: {
            // D = M5op - (1/2) D_h B
            Field<S> te = half_field<S>(c, pfx + "ap_te", c->Nh);
            Field<S> to = half_field<S>(c, pfx + "ap_to", c->Nh);
            T_(op_fived<S>(c, te, cfield(ie), P.B, nullptr, nullptr, st));
            T_(op_fived<S>(c, to, cfield(io), P.B, nullptr, nullptr, st));
            CField<S> ae = cfield(ie), ao = cfield(io);
            T_(op_hop<S>(c, oe, cfield(to), 0, false, prog_scale(-0.5), &ae, P.M5, nullptr, nullptr, st));
            T_(op_hop<S>(c, oo, cfield(te), 1, false, prog_scale(-0.5), &ao, P.M5, nullptr, nullptr, st));
            break;
        }
        case MSPCG_OP_DDAG: {
            // D^+ = M5op^+ - (1/2) B^+ Dd
            CField<S> ae = cfield(ie), ao = cfield(io);
            T_(op_hop<S>(c, oe, cfield(io), 0, true, scaled(P.Bdag, -0.5, -0.5), &ae, P.M5dag, nullptr, nullptr, st));
            T_(op_hop<S>(c, oo, cfield(ie), 1, true, scaled(P.Bdag, -0.5, -0.5), &ao, P.M5dag, nullptr, nullptr, st));
            break;
        }
        case MSPCG_OP_HOP:
        case MSPCG_OP_HOPDAG: {
            const bool dag = op == MSPCG_OP_HOPDAG;
            T_(op_hop<S>(c, oe, cfield(io), 0, dag, P.id, nullptr, P.id, nullptr, nullptr, st));
            T_(op_hop<S>(c, oo, cfield(ie), 1, dag, P.id, nullptr, P.id, nullptr, nullptr, st));
            break;
        }
        case MSPCG_OP_M5INV:
            T_(op_fived<S>(c, oe, cfield(ie), P.M5inv, nullptr, nullptr, st));
            T_(op_fived<S>(c, oo, cfield(io), P.M5inv, nullptr, nullptr, st));
            break;
        case MSPCG_OP_MHAT:
            T_(op_mhat<S>(c, oe, cfield(ie), nullptr, nullptr, st));
            break;
        case MSPCG_OP_MHATDAG:
            T_(op_mhatdag<S>(c, oe, cfield(ie), nullptr, st));
            break;
        case MSPCG_OP_A:
            T_(op_A<S>(c, oe, cfield(ie), nullptr, nullptr, st));
            break;
        case MSPCG_OP_PREPARE: {
            // b'_e = b_e + (1/2) D_h^eo X b_o ; bhat = Mhat^+ b'_e
            Field<S> w = half_field<S>(c, pfx + "ap_to", c->Nh);
            Field<S> bp = half_field<S>(c, pfx + "ap_te", c->Nh);
            CField<S> ae = cfield(ie);
            T_(op_fived<S>(c, w, cfield(io), P.X, nullptr, nullptr, st));
            T_(op_hop<S>(c, bp, cfield(w), 0, false, prog_scale(0.5), &ae, P.id, nullptr, nullptr, st));
            T_(op_mhatdag<S>(c, oe, cfield(bp), nullptr, st));
            break;
        }
        default:
            return MSPCG_EINVAL;
    }
    const bool full_out = op == MSPCG_OP_D || op == MSPCG_OP_DDAG || op == MSPCG_OP_HOP ||
                          op == MSPCG_OP_HOPDAG || op == MSPCG_OP_M5INV;
    T_(launch_unpack_parity<S>(cfield(oe), out, c->L, c->Ls, 0, full_out ? 0 : 1, st));
    if (full_out) T_(launch_unpack_parity<S>(cfield(oo), out, c->L, c->Ls, 1, 0, st));
#undef T_
    return MSPCG_OK;
}

extern "C" int mspcg_apply(mspcg_ctx* c, int op, int prec, const void* in_dev, void* out_dev,
                           hipStream_t st) try {
    if (!c || !in_dev || !out_dev || in_dev == out_dev) return MSPCG_EINVAL;
    if (!c->gauge) return MSPCG_ENOGAUGE;
    MSPCG_HIP(hipSetDevice(c->device));
    if (op == MSPCG_OP_KBLOCK) {
        if (!c->has_blocking) return MSPCG_EINVAL;
        int e = domains_setup(c, c->blocking, prec, st);
        if (e) return e;
        Field<F64> pe = half_field<F64>(c, "kb_p", c->Nh);
        Field<F64> qe = half_field<F64>(c, "kb_q", c->Nh);
        if ((e = launch_pack_parity<F64>((const double2*)in_dev, pe, c->L, c->Ls, 0, st)))
            return MSPCG_EHIP;
        switch (prec) {
            case MSPCG_FP64: e = kblock_apply<F64>(c, cfield(pe), qe, st); break;
            case MSPCG_FP32: e = kblock_apply<F32>(c, cfield(pe), qe, st); break;
            case MSPCG_FP16: e = kblock_apply<F16>(c, cfield(pe), qe, st); break;
            default: return MSPCG_EINVAL;
        }
        if (e) return e;
        if (launch_unpack_parity<F64>(cfield(qe), (double2*)out_dev, c->L, c->Ls, 0, 1, st))
            return MSPCG_EHIP;
        return MSPCG_OK;
    }
    return apply_op(c, op, prec, (const double2*)in_dev, (double2*)out_dev, st);
}
MSPCG_ABI_CATCH

int mspcg::apply_op(mspcg_ctx* c, int op, int prec, const double2* in, double2* out,
                    hipStream_t st) {
    if (op < 0 || op > MSPCG_OP_PREPARE) return MSPCG_EINVAL;
    if (prec == MSPCG_FP64) return apply_prec<F64>(c, op, in, out, st);
    if (prec == MSPCG_FP32) return apply_prec<F32>(c, op, in, out, st);
    return MSPCG_EINVAL;
}

extern "C" int mspcg_get_tuning(mspcg_ctx* c, mspcg_tuning* t) try {
    if (!c || !t) return MSPCG_EINVAL;
    *t = c->tune;
    return MSPCG_OK;
}
MSPCG_ABI_CATCH

extern "C" int mspcg_set_tuning(mspcg_ctx* c, const mspcg_tuning* t) try {
    if (!c || !t) return MSPCG_EINVAL;
    for (int p = 0; p < 3; ++p)
        for (int m = 0; m < 4; ++m)
            if (t->tile[p][m] < 0 || (t->tile[p][m] & 1)) return MSPCG_EINVAL;
    c->tune = *t;
    c->tune.xcd_remap = t->xcd_remap ? 1 : 0;
    return MSPCG_OK;
}
MSPCG_ABI_CATCH

extern "C" int mspcg_set_blocking(mspcg_ctx* c, const mspcg_blocking* b) try {
    if (!c || !b) return MSPCG_EINVAL;
    for (int m = 0; m < 4; ++m) {
        if (b->block[m] < 2 || (b->block[m] & 1) || c->L[m] % b->block[m]) return MSPCG_EINVAL;
    }
    if (b->pad < 0 || b->pad > 2) return MSPCG_EINVAL;
    if (b->form != MSPCG_FORM_DOMAIN && b->form != MSPCG_FORM_SPLIT) return MSPCG_EINVAL;
    if (b->form == MSPCG_FORM_SPLIT && b->pad < 1) return MSPCG_EINVAL;
    c->blocking = *b;
    c->has_blocking = true;
    return MSPCG_OK;
}
MSPCG_ABI_CATCH

extern "C" int mspcg_precond(mspcg_ctx* c, int inner_iters, int prec, const void* r_dev,
                             void* z_dev, hipStream_t st) try {
    if (!c || !r_dev || !z_dev || r_dev == z_dev || inner_iters < 0) return MSPCG_EINVAL;
    if (!c->gauge) return MSPCG_ENOGAUGE;
    if (!c->has_blocking) return MSPCG_EINVAL;
    MSPCG_HIP(hipSetDevice(c->device));
    int e = domains_setup(c, c->blocking, prec, st);
    if (e) return e;
    Field<F64> re = half_field<F64>(c, "pc_r", c->Nh);
    Field<F64> ze = half_field<F64>(c, "pc_z", c->Nh);
    if (launch_pack_parity<F64>((const double2*)r_dev, re, c->L, c->Ls, 0, st)) return MSPCG_EHIP;
    int done = 0;
    switch (prec) {
        case MSPCG_FP64: e = precond_apply<F64>(c, inner_iters, cfield(re), ze, st, &done); break;
        case MSPCG_FP32: e = precond_apply<F32>(c, inner_iters, cfield(re), ze, st, &done); break;
        case MSPCG_FP16: e = precond_apply<F16>(c, inner_iters, cfield(re), ze, st, &done); break;
        default: return MSPCG_EINVAL;
    }
    if (e) return e;
    if (launch_unpack_parity<F64>(cfield(ze), (double2*)z_dev, c->L, c->Ls, 0, 1, st))
        return MSPCG_EHIP;
    return MSPCG_OK;
}
MSPCG_ABI_CATCH

extern "C" int mspcg_solve(mspcg_ctx* c, const void* b_dev, void* x_dev,
                           const mspcg_solve_params* p, mspcg_solve_stats* stats,
                           hipStream_t st) try {
    if (!c || !b_dev || !x_dev || !p || b_dev == x_dev) return MSPCG_EINVAL;
    if (!c->gauge) return MSPCG_ENOGAUGE;
    MSPCG_HIP(hipSetDevice(c->device));
    return solve_one(c, b_dev, x_dev, p, stats, st);
}
MSPCG_ABI_CATCH

extern "C" int mspcg_pseudofermion_action(mspcg_ctx* c, const void* phi_dev, void* X_dev,
                                          void* dphi_dev, const mspcg_solve_params* p,
                                          double* S, mspcg_solve_stats* stats, hipStream_t st) try {
    if (!c || !phi_dev || !X_dev || !p || !S || phi_dev == X_dev || dphi_dev == phi_dev ||
        dphi_dev == X_dev)
        return MSPCG_EINVAL;
    if (!c->gauge) return MSPCG_ENOGAUGE;
    MSPCG_HIP(hipSetDevice(c->device));
    mspcg_solve_params q = *p;
    q.rhs_normal = 1;
    const int rc = solve_one(c, phi_dev, X_dev, &q, stats, st);
    if (rc != MSPCG_OK && rc != MSPCG_ENOCONV) return rc;
    // S = Re <phi, X> over the full-layout even fields (odd sites are zero
    // in X), fixed-order partial sums
    const long N = c->V4 * c->Ls;  // 5D entries of 12 complex values
    const long np = blas_grid_x(12 * N);
    int e = ensure_partials(c, (size_t)(2 * np + 16));
    if (e) return e;
    double* part = c->partials;
    if (launch_dot2((const double2*)phi_dev, (const double2*)X_dev, (const double2*)X_dev, N, part,
                    np, st))
        return MSPCG_EHIP;
    if (launch_reduce_sum(part, (int)np, part + 2 * np, st)) return MSPCG_EHIP;
    if (dphi_dev && launch_scale((double2*)dphi_dev, (const double2*)X_dev, 2.0, 12 * N, st))
        return MSPCG_EHIP;
    double v = 0;
    MSPCG_HIP(hipMemcpyAsync(&v, part + 2 * np, sizeof(double), hipMemcpyDeviceToHost, st));
    MSPCG_HIP(hipStreamSynchronize(st));
    *S = v;
    return rc;
}
MSPCG_ABI_CATCH

extern "C" int mspcg_solve_batch(mspcg_ctx* const* ctxs, int n, const void* const* b_dev,
                                 void* const* x_dev, const mspcg_solve_params* p,
                                 mspcg_solve_stats* stats, hipStream_t st) try {
    if (!ctxs || n < 0 || !b_dev || !x_dev || !p) return MSPCG_EINVAL;
    return solve_batch(ctxs, n, b_dev, x_dev, p, stats, st);
}
MSPCG_ABI_CATCH
