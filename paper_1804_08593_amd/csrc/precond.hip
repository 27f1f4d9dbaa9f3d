// The multisplitting preconditioner of Sec. 2.3 (eqs. (4)-(5), Fig. 3).
//
// K = (+)_s A_s with A_s = P_s A P_s: the diagonal block of A = Mhat^+ Mhat
// for block s, every entry coupling two different blocks set to zero.  A
// applied to a field supported on block s reaches at most two sites beyond
// the block (Mhat hops e -> o -> e), and only paths that return into the
// block survive the final projection, so
//     A_s p_s = P_s Mhat_D^+ Mhat_D p_s
// exactly, where Mhat_D is the Schur operator on the block padded by two
// sites (the "domain") with every hop leaving the domain dropped.  Each stage
// of Mhat_D^+ Mhat_D is evaluated only on the part of the domain that can
// still contribute (odd sites within one site of the block, even sites
// within two): the four hops run on boxes padded by 1, 2, 1 and 0, and the
// middle two only on the sites of their box within Manhattan distance 2 and
// 1 of the block (the first hop fills its whole box, so the sites the second
// reads beyond distance 1 hold exact zeros).
// A block that spans a whole lattice direction wraps periodically there.
// pad = 0 gives the cheaper Dirichlet-cut block operator Mhat_s^+ Mhat_s.
//
// K_l^-1 r: l CG iterations per block from a zero guess (eq. (4)), all blocks
// in one launch per step, with per-block scalars; storage precision S (FP16
// with per-(x,s) scales, FP32 or FP64), arithmetic in FP32 (FP64 for F64).
#include <string.h>

#include <vector>

#include "ctx.h"
#include "fived.h"

namespace mspcg {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void block_reduce_store(double v, double* dst) {
    __shared__ double red[kThreads / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) t += red[i];
        *dst = t;
    }
}

// per-domain scalars of the local CG
struct InnerScalars {
    double* gam;   // <rho, rho>
    double* a;     // step length
    double* beta;
    int* active;
};

// one workgroup per domain: fixed-order sum of that domain's partials
__device__ double domain_sum(const double* p, int n) {
    __shared__ double red2[kThreads];
    red2[threadIdx.x] = strided_sum(p, n);
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red2[threadIdx.x] += red2[threadIdx.x + o];
        __syncthreads();
    }
    const double r = red2[0];
    __syncthreads();
    return r;
}

__global__ void inner_start_scalars(InnerScalars s, const double* partials, int np,
                                    const int* done) {
    if (done && *done) return;
    const int d = blockIdx.x;
    const double g = domain_sum(partials + (long)d * np, np);
    if (threadIdx.x == 0) {
        s.gam[d] = g;
        s.active[d] = (g > 0.0 && isfinite(g)) ? 1 : 0;
    }
}

__global__ void inner_alpha(InnerScalars s, const double* partials, int np, const int* done) {
    if (done && *done) return;
    const int d = blockIdx.x;
    const double pw = domain_sum(partials + (long)d * np, np);
    if (threadIdx.x == 0) {
        int act = s.active[d] && pw > 0.0 && isfinite(pw);
        s.active[d] = act;
        s.a[d] = act ? s.gam[d] / pw : 0.0;
    }
}

__global__ void inner_beta(InnerScalars s, const double* partials, int np, const int* done) {
    if (done && *done) return;
    const int d = blockIdx.x;
    const double g2 = domain_sum(partials + (long)d * np, np);
    if (threadIdx.x == 0) {
        const int act = s.active[d];
        s.beta[d] = act ? g2 / s.gam[d] : 0.0;
        s.active[d] = act && g2 > 0.0 && isfinite(g2);
        s.gam[d] = g2;
    }
}

struct DomGeom {
    int L[4], blk[4], nb[4];
};

// rho = p = r on the block interior (global FP64 layout -> domain layout),
// per-domain |rho|^2 partials.
template <class S>
__global__ void inner_start_kernel(CField<F64> r, Field<S> rho, Field<S> p, DomGeom g, int Ls,
                                   long Vhb, double* partials, const int* done) {
    if (done && *done) return;
    const int spb = blockDim.x / Ls;
    const long cb = (long)blockIdx.x * spb + threadIdx.x / Ls;
    const int s = threadIdx.x % Ls;
    const int d = blockIdx.y;
    const bool active = (int)threadIdx.x < spb * Ls && cb < Vhb;
    double n2 = 0;
    if (active) {
        Box b;
        for (int m = 0; m < 4; ++m) {
            b.E[m] = g.blk[m];
            b.off[m] = 0;
        }
        b.Vh = Vhb;
        int c[4];
        box_coords(b, cb, 0, c);
        int rr = d, gc[4];
        for (int m = 0; m < 4; ++m) {
            gc[m] = (rr % g.nb[m]) * g.blk[m] + c[m];
            rr /= g.nb[m];
        }
        const long gcb = ((((long)gc[3] * g.L[2] + gc[2]) * g.L[1] + gc[1]) * g.L[0] + gc[0]) >> 1;
        cx<double> v[12];
        load_spinor_at<F64>(r, gcb * Ls, s, Ls, v);
        cx<typename S::real> w[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            w[k] = {(typename S::real)v[k].re, (typename S::real)v[k].im};
            n2 += (double)w[k].re * w[k].re + (double)w[k].im * w[k].im;
        }
        const long ib = ((long)d * Vhb + cb) * Ls;
        store_spinor_at<S>(rho, ib, s, Ls, w);
        store_spinor_at<S>(p, ib, s, Ls, w);
    }
    block_reduce_store(n2, partials + (long)d * gridDim.x + blockIdx.x);
}

int last_error() { return hipGetLastError() == hipSuccess ? 0 : MSPCG_EHIP; }

}  // namespace

static Box dom_box(const mspcg_ctx* c, const Domains& D, int padk) {
    Box b;
    long v = 1;
    for (int m = 0; m < 4; ++m) {
        if (D.nb[m] == 1) {
            b.E[m] = c->L[m];
            b.off[m] = 0;
        } else {
            b.E[m] = D.blk[m] + 2 * padk;
            b.off[m] = -padk;
        }
        v *= b.E[m];
    }
    b.Vh = v / 2;
    return b;
}

// Manhattan distance from the block of local site c of box b (directions the
// block spans wrap and count zero).
static int block_distance(const Domains& D, const Box& b, const int c[4]) {
    int dist = 0;
    for (int m = 0; m < 4; ++m) {
        if (D.nb[m] == 1) continue;
        const int x = c[m] + b.off[m];
        dist += x < 0 ? -x : (x >= D.blk[m] ? x - D.blk[m] + 1 : 0);
    }
    return dist;
}

// Host mirror of the kernels' checkerboard enumeration of a box.
static void host_box_coords(const Box& b, long cb, int par, int c[4]) {
    const int hx = b.E[0] >> 1;
    long r = cb / hx;
    const int xh = (int)(cb - r * hx);
    c[1] = (int)(r % b.E[1]);
    r /= b.E[1];
    c[2] = (int)(r % b.E[2]);
    c[3] = (int)(r / b.E[2]);
    const int so = b.off[0] + b.off[1] + b.off[2] + b.off[3];
    c[0] = 2 * xh + ((par + c[1] + c[2] + c[3] + so) & 1);
}

// Sites of parity `par` in box b within Manhattan distance `q` of the block
// (uploaded when `out` is given), and how many sites of the other parity
// in box `in` lie within q + 1 (what a hop onto those sites reads).
static int site_list(const Domains& D, const Box& b, int par, int q, const Box& in, int** out,
                     long* n, long* nread) {
    std::vector<int> v;
    int c[4];
    for (long cb = 0; cb < b.Vh; ++cb) {
        host_box_coords(b, cb, par, c);
        if (block_distance(D, b, c) <= q) v.push_back((int)cb);
    }
    long r = 0;
    for (long cb = 0; cb < in.Vh; ++cb) {
        host_box_coords(in, cb, par ^ 1, c);
        if (block_distance(D, in, c) <= q + 1) ++r;
    }
    *n = (long)v.size();
    *nread = r;
    if (hipMalloc(out, v.size() * sizeof(int)) != hipSuccess) return MSPCG_ENOMEM;
    if (hipMemcpy(*out, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
        return MSPCG_EHIP;
    return 0;
}

template <class S>
static size_t link_elems(const Domains& D) {
    return (size_t)D.ndom * 2 * 8 * 9 * D.pad2.Vh;
}

int domains_setup(mspcg_ctx* c, const mspcg_blocking& bk, int prec, hipStream_t st) {
    Domains& D = c->dom;
    bool same = D.built && D.prec == prec && D.pad == bk.pad && D.form == bk.form;
    for (int m = 0; m < 4; ++m) same = same && D.blk[m] == bk.block[m];
    if (same) return 0;
    D.built = false;  // until every field below describes the new blocking
    if (prec != MSPCG_FP16 && prec != MSPCG_FP32 && prec != MSPCG_FP64) return MSPCG_EINVAL;
    if (bk.pad < 0 || bk.pad > 2) return MSPCG_EINVAL;
    if (bk.form != MSPCG_FORM_DOMAIN && bk.form != MSPCG_FORM_SPLIT) return MSPCG_EINVAL;
    if (bk.form == MSPCG_FORM_SPLIT && bk.pad < 1) return MSPCG_EINVAL;
    int ndom = 1;
    for (int m = 0; m < 4; ++m) {
        const int b = bk.block[m];
        if (b < 2 || (b & 1) || c->L[m] % b) return MSPCG_EINVAL;
        D.blk[m] = b;
        D.nb[m] = c->L[m] / b;
        // the padded domain must not reach around the lattice onto the block
        if (D.nb[m] > 1 && c->L[m] - b < 2 * bk.pad) return MSPCG_EINVAL;
        ndom *= D.nb[m];
    }
    if (ndom > kMaxDomains) return MSPCG_EUNSUPPORTED;
    D.ndom = ndom;
    D.pad = bk.pad;
    D.form = bk.form;
    D.interior = dom_box(c, D, 0);
    D.pad1 = dom_box(c, D, bk.pad < 1 ? bk.pad : 1);
    D.pad2 = dom_box(c, D, bk.pad < 2 ? bk.pad : 2);
    D.Vh_int = D.interior.Vh;
    if (D.pad2.Vh >= (1L << 31)) return MSPCG_EUNSUPPORTED;  // 32-bit site indices
    // FP16 hops address a domain's sites with 32-bit offsets
    if (prec == MSPCG_FP16 &&
        (D.pad2.Vh >= (1L << 24) || D.pad2.Vh * c->Ls * (long)Chunk<F16>::K * 16 > 0xffffffffL))
        return MSPCG_EUNSUPPORTED;
    if (D.links) (void)hipFree(D.links);
    D.links = nullptr;
    size_t esz = prec == MSPCG_FP64 ? sizeof(double2) : (prec == MSPCG_FP32 ? sizeof(float2) : sizeof(__half2));
    const size_t n = (size_t)ndom * 2 * 8 * 9 * D.pad2.Vh;
    if (hipMalloc(&D.links, n * esz) != hipSuccess) return MSPCG_ENOMEM;
    int e = 0;
    if (prec == MSPCG_FP64)
        e = launch_pack_links<F64>(c->U, (double2*)D.links, c->L, D.blk, D.nb, D.pad2,
                                   c->act.antiperiodic_t, st);
    else if (prec == MSPCG_FP32)
        e = launch_pack_links<F32>(c->U, (float2*)D.links, c->L, D.blk, D.nb, D.pad2,
                                   c->act.antiperiodic_t, st);
    else
        e = launch_pack_links<F16>(c->U, (__half2*)D.links, c->L, D.blk, D.nb, D.pad2,
                                   c->act.antiperiodic_t, st);
    if (e) return MSPCG_EHIP;
    if (D.list_y) (void)hipFree(D.list_y);
    if (D.list_v) (void)hipFree(D.list_v);
    D.list_y = D.list_v = nullptr;
    D.n_y = D.n_v = D.rd_y = D.rd_v = 0;
    if (bk.pad > 0) {
        if ((e = site_list(D, D.pad2, 0, 2, D.pad1, &D.list_y, &D.n_y, &D.rd_y))) return e;
        if ((e = site_list(D, D.pad1, 1, 1, D.pad2, &D.list_v, &D.n_v, &D.rd_v))) return e;
    }
    D.prec = prec;
    D.built = true;
    return 0;
}

static int periodic_mask(const Domains& D) {
    int m = 0;
    for (int k = 0; k < 4; ++k)
        if (D.nb[k] == 1) m |= 1 << k;
    return m;
}

// Sites of box a inside box b (both parities).
static double box_overlap(const Box& a, const Box& b) {
    double v = 1;
    for (int m = 0; m < 4; ++m) {
        const int lo = a.off[m] > b.off[m] ? a.off[m] : b.off[m];
        const int hi = a.off[m] + a.E[m] < b.off[m] + b.E[m] ? a.off[m] + a.E[m] : b.off[m] + b.E[m];
        v *= hi > lo ? hi - lo : 0;
    }
    return v;
}

// Sites of the input box that a hop onto the output box reads: the output
// box itself and the one-site face slabs around it (no edges or corners).
static double hop_read_sites(const Box& in, const Box& out) {
    double n = box_overlap(in, out);
    for (int m = 0; m < 4; ++m)
        for (int side = 0; side < 2; ++side) {
            Box f = out;
            f.off[m] = side ? out.off[m] + out.E[m] : out.off[m] - 1;
            f.E[m] = 1;
            n += box_overlap(in, f);
        }
    return n;
}

// Arguments of one block-domain hop (every block in one launch) and its
// algorithmic bytes.
template <class S>
static HopArgs<S> dom_hop_args(mspcg_ctx* c, Field<S> out, const Box& bout, CField<S> in,
                               const Box& bin, int out_par, const FiveDProg& ph,
                               const CField<S>* aux, const Box& baux, const FiveDProg& pa,
                               double* partials, const int* done, const HopArgs<S>* cg,
                               const int* list, long nlist, long nread, double& bytes) {
    const Domains& D = c->dom;
    HopArgs<S> a;
    memset(&a, 0, sizeof(a));
    if (cg) {
        // fused local CG update (rho -= a w, z += a p) on the block interior
        a.cg_r = cg->cg_r;
        a.cg_x = cg->cg_x;
        a.cg_p = cg->cg_p;
        a.cg_alpha = cg->cg_alpha;
        a.cg_first = cg->cg_first;
        a.cg_keep_out = 0;
    }
    a.in = in;
    a.out = out;
    if (aux) a.aux = *aux;
    a.links = (const typename S::elem*)D.links;
    a.link_dom_stride = 2L * 8 * 9 * D.pad2.Vh;
    a.g.out = bout;
    a.g.in = bin;
    a.g.aux = aux ? baux : bout;
    a.g.link = D.pad2;
    a.g.out_par = out_par;
    a.g.periodic = periodic_mask(D);
    a.ph = ph;
    a.pa = pa;
    a.has_aux = aux != nullptr;
    a.mf = c->act.mf;
    a.partials = partials;
    a.done = done;
    a.xcd_remap = c->tune.xcd_remap;
    pick_tile(c->tune.tile[prec_index<S>()], bout, a.tile);
    a.site_list = list;
    a.n_list = nlist;
    // spinor entries per s moved (one parity): out, the input sites the hop
    // reads, aux at the output sites (aux boxes lie inside the listed region);
    // the fused update reads rho, p (z unless first) and writes rho, z in
    // place of out
    const double nout = list ? (double)nlist : (double)bout.Vh;
    double entries = nout + (list ? (double)nread : hop_read_sites(bin, bout) / 2) +
                     (aux ? box_overlap(baux, bout) / 2 : 0);
    if (cg) entries += nout * (cg->cg_x.data ? (cg->cg_first ? 3 : 4) : 1);
    bytes = (double)D.ndom * c->Ls * entries * S::bytes_spinor +
            (double)D.ndom * nout * 8 * S::bytes_link;
    return a;
}

template <class S>
static int dom_hop(mspcg_ctx* c, Field<S> out, const Box& bout, CField<S> in, const Box& bin,
                   int out_par, bool dag, const FiveDProg& ph, const CField<S>* aux,
                   const Box& baux, const FiveDProg& pa, double* partials, const int* done,
                   hipStream_t st, const HopArgs<S>* cg = nullptr, const int* list = nullptr,
                   long nlist = 0, long nread = 0) {
    double bytes;
    const HopArgs<S> a = dom_hop_args<S>(c, out, bout, in, bin, out_par, ph, aux, baux, pa,
                                         partials, done, cg, list, nlist, nread, bytes);
    Timed t(c, cg ? MSPCG_KC_HOPDOMCG : MSPCG_KC_HOPDOM, bytes, st);
    return launch_hop<S>(a, c->Ls, c->dom.ndom, dag, st);
}

template <class S>
static int dom_fived(mspcg_ctx* c, Field<S> out, CField<S> in, long Vh, const FiveDProg& p,
                     const int* done, hipStream_t st, const Field<S>* xp_in = nullptr,
                     CField<S> xp_src = {}, const double* xp_beta = nullptr,
                     const Field<S>* zd_z = nullptr, const double* zd_alpha = nullptr,
                     int zd_first = 0) {
    FiveDArgs<S> a;
    memset(&a, 0, sizeof(a));
    a.in = in;
    a.out = out;
    a.Vh = Vh;
    a.p = p;
    a.mf = c->act.mf;
    a.partials = nullptr;
    a.done = done;
    if (xp_in) {  // in = src + beta[domain] in, written back, before the program
        a.xp_in = *xp_in;
        a.xp_src = xp_src;
        a.xp_beta = xp_beta;
        if (zd_z) {  // z (+)= alpha[domain] in, with in before that update
            a.zd_z = *zd_z;
            a.zd_alpha = zd_alpha;
            a.zd_first = zd_first;
        }
    }
    const int entries = (xp_in ? 4 : 2) + (xp_in && zd_z ? (zd_first ? 1 : 2) : 0);
    Timed t(c, MSPCG_KC_FIVED, (double)c->dom.ndom * Vh * c->Ls * S::bytes_spinor * entries, st);
    return launch_fived<S>(a, c->Ls, c->dom.ndom, st);
}

// w = A_s p for every block: P_s Mhat_D^+ Mhat_D p (p supported on the block).
// partials (optional) receive per-domain |Mhat_D p|^2 = <p, A_s p>, laid out
// [ndom][hop_grid_x(n_y)] (pad2.Vh in place of n_y when pad = 0).
template <class S>
int block_A(mspcg_ctx* c, Field<S> w, CField<S> p, double* partials, const int* done,
            hipStream_t st) {
    const Domains& D = c->dom;
    const int Ls = c->Ls;
    const std::string pf = std::string("dom") + (std::is_same<S, F16>::value ? "16." : std::is_same<S, F32>::value ? "32." : "64.");
    Field<S> t = half_field<S>(c, pf + "t", (long)D.ndom * D.interior.Vh * Ls);
    Field<S> u = half_field<S>(c, pf + "u", (long)D.ndom * D.pad1.Vh * Ls);
    Field<S> y = half_field<S>(c, pf + "y", (long)D.ndom * D.pad2.Vh * Ls);
    Field<S> v = half_field<S>(c, pf + "v", (long)D.ndom * D.pad1.Vh * Ls);
    if (!t.data || !u.data || !y.data || !v.data) return MSPCG_ENOMEM;
    const Progs& P = c->pr;
    FiveDProg m14;
    memset(&m14, 0, sizeof(m14));
    m14.scale[0] = m14.scale[1] = -0.25;
    m14.identity = 1;
    int e;
    // t = B p (block)
    if ((e = dom_fived<S>(c, t, p, D.interior.Vh, P.B, done, st))) return e;
    // u = X D_h^oe t  (odd, pad 1)
    if ((e = dom_hop<S>(c, u, D.pad1, cfield(t), D.interior, 1, false, P.X, nullptr, D.interior,
                        P.id, nullptr, done, st)))
        return e;
    // y = M5op p - D_h^eo u / 4 = Mhat_D p  (even: widened block within
    // distance 2, or the block itself for the split form)
    if ((e = dom_hop<S>(c, y, D.ybox(), cfield(u), D.pad1, 0, false, m14, &p, D.interior, P.M5,
                        partials, done, st, nullptr, D.ylist(), D.yn(), D.yread())))
        return e;
    // v = X^+ Dd^oe y  (odd, pad 1, within distance 1)
    if ((e = dom_hop<S>(c, v, D.pad1, cfield(y), D.ybox(), 1, true, P.Xdag, nullptr, D.interior,
                        P.id, nullptr, done, st, nullptr, D.list_v, D.n_v, D.rd_v)))
        return e;
    // w = M5op^+ y - B^+ Dd^eo v / 4  (even, block)
    CField<S> yc = cfield(y);
    return dom_hop<S>(c, w, D.interior, cfield(v), D.pad1, 0, true, scaled(P.Bdag, -0.25, -0.25),
                      &yc, D.ybox(), P.M5dag, nullptr, done, st);
}

static InnerScalars inner_scalars(mspcg_ctx* c) {
    InnerScalars s;
    const int n = c->dom.ndom;
    s.gam = (double*)c->buf("in.gam", n * sizeof(double));
    s.a = (double*)c->buf("in.a", n * sizeof(double));
    s.beta = (double*)c->buf("in.beta", n * sizeof(double));
    s.active = (int*)c->buf("in.active", n * sizeof(int));
    return s;
}

// The local solves of one lattice: K_l^-1 r as l CG steps on every block
// (eq. (4)), split into the pieces that several lattices can interleave
// stage by stage.  One step:
//   B      t = B p; p = rho + beta p rides on it (step > 0), and the solution
//          update z += alpha p of the previous step (it reads the old p)
//   hop 0  u = X D_h^oe t                    (odd, block widened by 1)
//   hop 1  y = M5op p - D_h^eo u / 4 = Mhat_D p, |y|^2 = <p, A_s p> partials
//   alpha  per block: alpha = gamma / <p, A_s p>
//   hop 2  v = X^+ Dd^oe y                    (odd, within 1 of the block)
//   hop 3  A_s p = M5op^+ y - B^+ Dd^eo v / 4 on the block, fused with
//          rho -= alpha A_s p and its |rho|^2 partials (A_s p is not stored);
//          the last step also does z += alpha p there
//   beta   per block, for the next step
template <class S>
struct Local {
    mspcg_ctx* c = nullptr;
    Field<S> rho, p, zz, t, u, y, v;
    InnerScalars sc;
    long hop_np = 0, start_np = 0, upd_np = 0;
    FiveDProg m14;
};

template <class S>
static int local_init(mspcg_ctx* c, Local<S>& L) {
    const Domains& D = c->dom;
    const int Ls = c->Ls;
    const long nd = D.interior.Vh * Ls;  // (site, s) per domain
    const std::string pf = std::string("dom") + (std::is_same<S, F16>::value ? "16." : std::is_same<S, F32>::value ? "32." : "64.");
    L.c = c;
    L.rho = half_field<S>(c, pf + "rho", D.ndom * nd);
    L.p = half_field<S>(c, pf + "p", D.ndom * nd);
    L.zz = half_field<S>(c, pf + "z", D.ndom * nd);
    L.t = half_field<S>(c, pf + "t", (long)D.ndom * D.interior.Vh * Ls);
    L.u = half_field<S>(c, pf + "u", (long)D.ndom * D.pad1.Vh * Ls);
    L.y = half_field<S>(c, pf + "y", (long)D.ndom * D.pad2.Vh * Ls);
    L.v = half_field<S>(c, pf + "v", (long)D.ndom * D.pad1.Vh * Ls);
    if (!L.rho.data || !L.p.data || !L.zz.data || !L.t.data || !L.u.data || !L.y.data ||
        !L.v.data)
        return MSPCG_ENOMEM;
    L.sc = inner_scalars(c);
    if (!L.sc.gam || !L.sc.a || !L.sc.beta || !L.sc.active) return MSPCG_ENOMEM;
    L.hop_np = hop_grid_x<S>(D.yout(), Ls);
    const int spb = kThreads / Ls;
    L.start_np = (D.interior.Vh + spb - 1) / spb;
    // partials of the fused update: one per workgroup of the interior hop
    L.upd_np = hop_grid_x<S>(D.interior.Vh, Ls);
    const long vec_np = (nd + kThreads - 1) / kThreads;
    long need = L.hop_np > L.start_np ? L.hop_np : L.start_np;
    if (vec_np > need) need = vec_np;
    int e = ensure_partials(c, (size_t)(D.ndom * need + 64));
    if (e) return e;
    memset(&L.m14, 0, sizeof(L.m14));
    L.m14.scale[0] = L.m14.scale[1] = -0.25;
    L.m14.identity = 1;
    return 0;
}

// rho = p = r on every block, gamma = |rho|^2 per block
template <class S>
static int local_start(Local<S>& L, CField<F64> r, const int* done, hipStream_t st) {
    mspcg_ctx* c = L.c;
    const Domains& D = c->dom;
    const int Ls = c->Ls;
    const long nd = D.interior.Vh * Ls;
    DomGeom g;
    for (int m = 0; m < 4; ++m) {
        g.L[m] = c->L[m];
        g.blk[m] = D.blk[m];
        g.nb[m] = D.nb[m];
    }
    const int spb = kThreads / Ls;
    Timed t(c, MSPCG_KC_BLAS, (double)D.ndom * nd * (192.0 + 2 * S::bytes_spinor), st);
    hipLaunchKernelGGL(inner_start_kernel<S>, dim3((unsigned)L.start_np, D.ndom), dim3(spb * Ls), 0,
                       st, r, L.rho, L.p, g, Ls, D.interior.Vh, c->partials, done);
    if (last_error()) return MSPCG_EHIP;
    hipLaunchKernelGGL(inner_start_scalars, dim3(D.ndom), dim3(kThreads), 0, st, L.sc, c->partials,
                       (int)L.start_np, done);
    return last_error();
}

template <class S>
static int local_B(Local<S>& L, int it, const int* done, hipStream_t st) {
    mspcg_ctx* c = L.c;
    const Domains& D = c->dom;
    const CField<S> pc = cfield(L.p);
    if (it > 0)  // L.sc.a still holds the step length of step it - 1 here
        return dom_fived<S>(c, L.t, pc, D.interior.Vh, c->pr.B, done, st, &L.p, cfield(L.rho),
                            L.sc.beta, &L.zz, L.sc.a, it == 1 ? 1 : 0);
    return dom_fived<S>(c, L.t, pc, D.interior.Vh, c->pr.B, done, st);
}

// Arguments of hop k (0..3, see Local) of step it of l; dag: the dagger hop
template <class S>
static HopArgs<S> local_hop(Local<S>& L, int k, int it, int l, const int* done, double& bytes,
                            bool& dag) {
    mspcg_ctx* c = L.c;
    const Domains& D = c->dom;
    const Progs& P = c->pr;
    const CField<S> pc = cfield(L.p);
    const CField<S> yc = cfield(L.y);
    double* part = c->partials;
    dag = k >= 2;
    if (k == 0)
        return dom_hop_args<S>(c, L.u, D.pad1, cfield(L.t), D.interior, 1, P.X, nullptr,
                               D.interior, P.id, nullptr, done, nullptr, nullptr, 0, 0, bytes);
    if (k == 1)
        return dom_hop_args<S>(c, L.y, D.ybox(), cfield(L.u), D.pad1, 0, L.m14, &pc, D.interior,
                               P.M5, part, done, nullptr, D.ylist(), D.yn(), D.yread(), bytes);
    if (k == 2)
        return dom_hop_args<S>(c, L.v, D.pad1, yc, D.ybox(), 1, P.Xdag, nullptr, D.interior, P.id,
                               nullptr, done, nullptr, D.list_v, D.n_v, D.rd_v, bytes);
    HopArgs<S> cg;
    memset(&cg, 0, sizeof(cg));
    cg.cg_r = L.rho;
    if (it == l - 1) cg.cg_x = L.zz;  // earlier steps: deferred to the next B kernel
    cg.cg_p = pc;
    cg.cg_alpha = L.sc.a;
    cg.cg_first = it == 0 ? 1 : 0;
    Field<S> none;
    memset(&none, 0, sizeof(none));
    return dom_hop_args<S>(c, none, D.interior, cfield(L.v), D.pad1, 0,
                           scaled(P.Bdag, -0.25, -0.25), &yc, D.ybox(), P.M5dag, part, done, &cg,
                           nullptr, 0, 0, bytes);
}

template <class S>
static int local_alpha(Local<S>& L, const int* done, hipStream_t st) {
    hipLaunchKernelGGL(inner_alpha, dim3(L.c->dom.ndom), dim3(kThreads), 0, st, L.sc,
                       L.c->partials, (int)L.hop_np, done);
    return last_error();
}

template <class S>
static int local_beta(Local<S>& L, const int* done, hipStream_t st) {
    hipLaunchKernelGGL(inner_beta, dim3(L.c->dom.ndom), dim3(kThreads), 0, st, L.sc,
                       L.c->partials, (int)L.upd_np, done);
    return last_error();
}

// z written in FP64 from the domain copy (with the flexible-beta dots)
template <class S>
static int local_finish(Local<S>& L, int l, Field<F64> z, PrecondDots* dots, hipStream_t st) {
    mspcg_ctx* c = L.c;
    const Domains& D = c->dom;
    const int Ls = c->Ls;
    const long nd = D.interior.Vh * Ls;
    Timed t(c, MSPCG_KC_BLAS,
            (double)D.ndom * nd * (192.0 + S::bytes_spinor + (dots && l > 0 ? 2 * 192.0 : 0.0)), st);
    if (l == 0) return launch_zero(z.data, c->Nh, st) ? MSPCG_EHIP : 0;
    if (dots) {
        // z and the workgroup partials of Re<z, r>, Re<z, q> in one pass
        dots->np = launch_domain_to_global_dots<S>(cfield(L.zz), z, dots->r, dots->q, c->L, D.blk,
                                                   D.nb, Ls, c->partials, st);
        return dots->np < 0 ? MSPCG_EHIP : 0;
    }
    if (launch_domain_to_global<S, F64>(cfield(L.zz), z, c->L, D.blk, D.nb, Ls, 0, st))
        return MSPCG_EHIP;
    return 0;
}

// z_e = K_l^-1 r_e (FP64 whole-lattice even fields); `done` (device flag,
// may be null) skips the work once the outer solve has converged.
template <class S>
static int precond_core(mspcg_ctx* c, int l, CField<F64> r, Field<F64> z, const int* done,
                        hipStream_t st, PrecondDots* dots = nullptr) {
    Local<S> L;
    int e;
    if ((e = local_init<S>(c, L))) return e;
    if ((e = local_start<S>(L, r, done, st))) return e;
    for (int it = 0; it < l; ++it) {
        if ((e = local_B<S>(L, it, done, st))) return e;
        for (int k = 0; k < 4; ++k) {
            double bytes;
            bool dag;
            const HopArgs<S> a = local_hop<S>(L, k, it, l, done, bytes, dag);
            {
                Timed t(c, k == 3 ? MSPCG_KC_HOPDOMCG : MSPCG_KC_HOPDOM, bytes, st);
                if (launch_hop<S>(a, c->Ls, c->dom.ndom, dag, st)) return MSPCG_EHIP;
            }
            if (k == 1 && (e = local_alpha<S>(L, done, st))) return e;
        }
        if (it + 1 < l && (e = local_beta<S>(L, done, st))) return e;
    }
    return local_finish<S>(L, l, z, dots, st);
}

// Local solves of several lattices interleaved stage by stage; with `multi`
// every block-hop stage runs as one persistent launch per group of lattices
// that share Ls (MultiHop), otherwise one launch per lattice.
template <class S>
struct BatchPrecondImpl : BatchPrecond {
    std::vector<Local<S>> L;
    std::vector<const int*> done;
    // per group of lattices with one Ls: descriptors in device memory for
    // hops 0..2 (u, y, v), then hop 3 for (first step, last step) =
    // (0,0) (0,1) (1,0) (1,1); items < 0 marks a kind of step l does not have
    struct Group {
        int Ls = 0;
        std::vector<int> members;
        MultiHop<S>* dev = nullptr;
        long items[7] = {};
        bool dag[7] = {}, eph[7] = {}, epa[7] = {}, cgf[7] = {};
    };
    std::vector<Group> groups;
    ~BatchPrecondImpl() override {
        for (Group& g : groups)
            if (g.dev) (void)hipFree(g.dev);
    }
    static bool chain(const FiveDProg& P) {
        return !P.identity && !(P.nsteps == 1 && P.kind[0] == STEP_BIDI);
    }
    int build_group(Group& G, int l) {
        const int n = (int)G.members.size();
        std::vector<MultiHop<S>> h(7);
        for (int k = 0; k < 7; ++k) {
            memset(&h[k], 0, sizeof(MultiHop<S>));
            const int stage = k < 3 ? k : 3;
            int it = 0;
            if (k >= 3) {
                // a step with the wanted (first, last) flags, if l has one
                const bool want_first = ((k - 3) >> 1) & 1, want_last = (k - 3) & 1;
                it = want_first ? 0 : (want_last ? l - 1 : 1);
                if (it >= l || (it == 0) != want_first || (it == l - 1) != want_last) {
                    G.items[k] = -1;
                    continue;
                }
            }
            long first = 0;
            for (int j = 0; j < n; ++j) {
                const int i = G.members[j];
                double bytes;
                bool dg;
                const HopArgs<S> a = local_hop<S>(L[i], stage, it, l, done[i], bytes, dg);
                const long nout = a.site_list ? a.n_list : a.g.out.Vh;
                const bool e1 = chain(a.ph), e2 = a.has_aux && chain(a.pa);
                if (j == 0) {
                    G.dag[k] = dg;
                    G.eph[k] = e1;
                    G.epa[k] = e2;
                    G.cgf[k] = a.cg_r.data != nullptr;
                } else if (e1 != G.eph[k] || e2 != G.epa[k]) {
                    return MSPCG_EUNSUPPORTED;  // lattices need different kernel variants
                }
                h[k].a[j] = a;
                h[k].ls[j] = G.Ls;
                h[k].gx[j] = (int)hop_grid_x<S>(nout, G.Ls);
                h[k].first[j] = first;
                first += (long)L[i].c->dom.ndom * h[k].gx[j];
            }
            h[k].first[n] = first;
            h[k].n = n;
            G.items[k] = first;
        }
        if (hipMalloc(&G.dev, 7 * sizeof(MultiHop<S>)) != hipSuccess) return MSPCG_ENOMEM;
        if (hipMemcpy(G.dev, h.data(), 7 * sizeof(MultiHop<S>), hipMemcpyHostToDevice) != hipSuccess)
            return MSPCG_EHIP;
        return 0;
    }
    int build(int l) {
        for (size_t i = 0; i < L.size(); ++i) {
            const int Ls = L[i].c->Ls;
            if (!multi_hop_ls(Ls)) return MSPCG_EUNSUPPORTED;
            Group* g = nullptr;
            for (Group& x : groups)
                if (x.Ls == Ls && (int)x.members.size() < kMaxBatch) g = &x;
            if (!g) {
                groups.emplace_back();
                g = &groups.back();
                g->Ls = Ls;
            }
            g->members.push_back((int)i);
        }
        for (Group& g : groups) {
            const int e = build_group(g, l);
            if (e) return e;
        }
        return 0;
    }
    int hop(int k, int it, int l, hipStream_t st) {
        if (multi) {
            const int j = k < 3 ? k : 3 + 2 * (it == 0) + (it == l - 1);
            for (const Group& G : groups) {
                if (G.items[j] < 0) return MSPCG_EHIP;
                if (launch_multi_hop<S>(G.dev + j, G.items[j], G.Ls, G.dag[j], G.eph[j], G.epa[j],
                                        G.cgf[j], st))
                    return MSPCG_EHIP;
            }
            return 0;
        }
        for (size_t i = 0; i < L.size(); ++i) {
            double bytes;
            bool dg;
            const HopArgs<S> a = local_hop<S>(L[i], k, it, l, done[i], bytes, dg);
            if (launch_hop<S>(a, L[i].c->Ls, L[i].c->dom.ndom, dg, st)) return MSPCG_EHIP;
        }
        return 0;
    }
    int apply(int l, const CField<F64>* r, const Field<F64>* z, PrecondDots* dots,
              hipStream_t st) override {
        const size_t n = L.size();
        int e;
        for (size_t i = 0; i < n; ++i)
            if ((e = local_start<S>(L[i], r[i], done[i], st))) return e;
        for (int it = 0; it < l; ++it) {
            for (size_t i = 0; i < n; ++i)
                if ((e = local_B<S>(L[i], it, done[i], st))) return e;
            for (int k = 0; k < 4; ++k) {
                if ((e = hop(k, it, l, st))) return e;
                if (k == 1)
                    for (size_t i = 0; i < n; ++i)
                        if ((e = local_alpha<S>(L[i], done[i], st))) return e;
            }
            if (it + 1 < l)
                for (size_t i = 0; i < n; ++i)
                    if ((e = local_beta<S>(L[i], done[i], st))) return e;
        }
        for (size_t i = 0; i < n; ++i)
            if ((e = local_finish<S>(L[i], l, z[i], dots ? dots + i : nullptr, st))) return e;
        return 0;
    }
};

template <class S>
static int make_batch_impl(mspcg_ctx* const* cs, int n, int l, const int* const* done,
                           bool multi, std::unique_ptr<BatchPrecond>& out) {
    std::unique_ptr<BatchPrecondImpl<S>> b(new BatchPrecondImpl<S>());
    b->L.resize(n);
    b->done.assign(done, done + n);
    int e;
    for (int i = 0; i < n; ++i)
        if ((e = local_init<S>(cs[i], b->L[i]))) return e;
    if (multi && l > 0) {
        e = b->build(l);
        if (e && e != MSPCG_EUNSUPPORTED) return e;
        b->multi = e == 0;
    }
    out = std::move(b);
    return 0;
}

int make_batch_precond(mspcg_ctx* const* cs, int n, int prec, int l, const int* const* done,
                       bool multi, std::unique_ptr<BatchPrecond>& out) {
    switch (prec) {
        case MSPCG_FP16: return make_batch_impl<F16>(cs, n, l, done, multi, out);
        case MSPCG_FP32: return make_batch_impl<F32>(cs, n, l, done, multi, out);
        case MSPCG_FP64: return make_batch_impl<F64>(cs, n, l, done, multi, out);
        default: return MSPCG_EINVAL;
    }
}

size_t precond_partials_need(mspcg_ctx* c) {
    const Domains& D = c->dom;
    const int Ls = c->Ls;
    const long nd = D.interior.Vh * Ls;
    const long hop_np = hop_grid_x<F64>(D.yout(), Ls);
    const int spb = kThreads / Ls;
    const long start_np = (D.interior.Vh + spb - 1) / spb;
    const long vec_np = (nd + kThreads - 1) / kThreads;
    long need = hop_np > start_np ? hop_np : start_np;
    if (vec_np > need) need = vec_np;
    return (size_t)(D.ndom * need + 64);
}

template <class S>
int precond_apply(mspcg_ctx* c, int l, CField<F64> r, Field<F64> z, hipStream_t st, int*) {
    return precond_core<S>(c, l, r, z, nullptr, st);
}

template <class S>
int precond_apply_flag(mspcg_ctx* c, int l, CField<F64> r, Field<F64> z, const int* done,
                       hipStream_t st, PrecondDots* dots) {
    return precond_core<S>(c, l, r, z, done, st, dots);
}

template <class S>
int kblock_apply(mspcg_ctx* c, CField<F64> p_e, Field<F64> q_e, hipStream_t st) {
    const Domains& D = c->dom;
    const int Ls = c->Ls;
    const long nd = D.interior.Vh * Ls;
    const std::string pf = std::string("dom") + (std::is_same<S, F16>::value ? "16." : std::is_same<S, F32>::value ? "32." : "64.");
    Field<S> p = half_field<S>(c, pf + "p", D.ndom * nd);
    Field<S> w = half_field<S>(c, pf + "w", D.ndom * nd);
    if (!p.data || !w.data) return MSPCG_ENOMEM;
    if (launch_global_to_domain<F64, S>(p_e, p, c->L, D.blk, D.nb, Ls, 0, st)) return MSPCG_EHIP;
    int e = block_A<S>(c, w, cfield(p), nullptr, nullptr, st);
    if (e) return e;
    if (launch_domain_to_global<S, F64>(cfield(w), q_e, c->L, D.blk, D.nb, Ls, 0, st))
        return MSPCG_EHIP;
    return 0;
}

template int block_A<F64>(mspcg_ctx*, Field<F64>, CField<F64>, double*, const int*, hipStream_t);
template int block_A<F32>(mspcg_ctx*, Field<F32>, CField<F32>, double*, const int*, hipStream_t);
template int block_A<F16>(mspcg_ctx*, Field<F16>, CField<F16>, double*, const int*, hipStream_t);

#define MSPCG_PC(S)                                                                         \
    template int precond_apply<S>(mspcg_ctx*, int, CField<F64>, Field<F64>, hipStream_t,   \
                                  int*);                                                    \
    template int precond_apply_flag<S>(mspcg_ctx*, int, CField<F64>, Field<F64>,           \
                                       const int*, hipStream_t, PrecondDots*);              \
    template int kblock_apply<S>(mspcg_ctx*, CField<F64>, Field<F64>, hipStream_t);
MSPCG_PC(F64)
MSPCG_PC(F32)
MSPCG_PC(F16)

}  // namespace mspcg
