// Ls-vectorised Wilson hop with fused fifth-dimension epilogues (gfx950).
//
// out(x,s) = Ph[ sum_mu eta (1 -/+ g_mu) U_mu(x) in(x+mu,s) + eta (1 +/- g_mu) U_mu(x-mu)^+ in(x-mu,s) ]
//          + Pa[ aux(x,s) ]
// Ph, Pa: 5D programs acting on the s-vector of each site (fived.h); the
// dagger hop swaps the projector signs.  One thread per (site, s); the
// workgroup holds whole sites so the s-mixing epilogue runs through LDS.
//
// Spin projection in the chiral basis: with g_mu = [[0, e_mu], [e_mu^+, 0]],
// (1 + sig g_mu) psi = [h ; sig e_mu^+ h] with h = psi_up + sig e_mu psi_dn,
// so only the 2x3 half spinor h is multiplied by the link.
//   e_x = -i sigma_x, e_y = -i sigma_y, e_z = -i sigma_z, e_t = 1.
#pragma once
#include <type_traits>
#include <utility>

#include "common.h"
#include "fived.h"
#include "kernels.h"

// Build-time variants (measured; the defaults are the fastest on gfx950):
//   MSPCG_HOP_MINWAVES  occupancy hint of __launch_bounds__
//   MSPCG_HOP_NT        nontemporal link loads and output stores
//   MSPCG_HOP_PF*       neighbour loads kept in flight per thread
#ifndef MSPCG_HOP_MINWAVES
#define MSPCG_HOP_MINWAVES 1
#endif
#ifndef MSPCG_HOP_NT
#define MSPCG_HOP_NT true
#endif
// MSPCG_HOP_PF{64,32,16}: directions whose raw neighbour spinors are loaded
// before any of them is decoded and applied (per storage precision).  Two
// for FP16 (12^3x24 domain hop 428 -> 415 us; with the packed-FP16 products
// 396 -> 385 us, four: 413 us); deeper groups did not help the FP64 and FP32
// hops.
#ifndef MSPCG_HOP_PF64
#define MSPCG_HOP_PF64 1
#endif
#ifndef MSPCG_HOP_PF32
#define MSPCG_HOP_PF32 1
#endif
#ifndef MSPCG_HOP_PF16
#define MSPCG_HOP_PF16 2
#endif
// MSPCG_HOP_MFMA: FP16-storage hops at Ls = 16 multiply links by spinors on
// the matrix cores (see hop_body).  Off by default: the hop is bound by HBM
// and LDS traffic, not by its 1320 flops per 5D site, and the operand staging
// the matrix-core form needs made the 12^3x24 domain hop 11% slower (463 us
// against 416 us) on MI355X.  Build with -DMSPCG_HOP_MFMA=1 to select it.
#ifndef MSPCG_HOP_MFMA
#define MSPCG_HOP_MFMA 0
#endif
// MSPCG_HOP_PK16: FP16-storage hops project and multiply by the link in
// packed FP16 arithmetic (two halves per instruction, see dir_apply_pk) and
// accumulate the directions in FP32.  It cuts the Ls = 16 block hop's VALU
// instructions by a sixth (2007 -> 1670 in the kernel body) and its time by
// 6% on MI355X (12^3x24 domains: 429 -> 403 us), with unchanged outer
// iteration counts.  Off by default: the local solves keep FP32 arithmetic
// on their FP16-stored operands; build with -DMSPCG_HOP_PK16=1 to select it.
#ifndef MSPCG_HOP_PK16
#define MSPCG_HOP_PK16 0
#endif
#ifndef MSPCG_HOP_MFMA_WAVES
#define MSPCG_HOP_MFMA_WAVES 4
#endif

namespace mspcg {

// h = psi_up + sig e_mu psi_dn   (components: spin*3 + colour).  With MIX the
// inputs are decoded FP16 values and each sum is formed as a fused
// multiply-add with an opaque unit factor, which the compiler turns into one
// mixed-precision instruction reading both FP16 halves (exact sum, one rounding).
template <int MU, int SIG, bool MIX, typename T>
__device__ __forceinline__ void project(const cx<T> (&p)[12], cx<T> (&h)[6], T one) {
    auto pm = [&](T u, T d) { return MIX ? fmadd(d, one, u) : u + d; };
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cx<T> u0 = p[c], u1 = p[3 + c], d0 = p[6 + c], d1 = p[9 + c];
        if constexpr (MU == 0) {  // e d = (-i d1, -i d0)
            h[c] = {pm(u0.re, SIG * d1.im), pm(u0.im, -SIG * d1.re)};
            h[3 + c] = {pm(u1.re, SIG * d0.im), pm(u1.im, -SIG * d0.re)};
        } else if constexpr (MU == 1) {  // e d = (-d1, d0)
            h[c] = {pm(u0.re, -SIG * d1.re), pm(u0.im, -SIG * d1.im)};
            h[3 + c] = {pm(u1.re, SIG * d0.re), pm(u1.im, SIG * d0.im)};
        } else if constexpr (MU == 2) {  // e d = (-i d0, i d1)
            h[c] = {pm(u0.re, SIG * d0.im), pm(u0.im, -SIG * d0.re)};
            h[3 + c] = {pm(u1.re, -SIG * d1.im), pm(u1.im, SIG * d1.re)};
        } else {  // e d = d
            h[c] = {pm(u0.re, SIG * d0.re), pm(u0.im, SIG * d0.im)};
            h[3 + c] = {pm(u1.re, SIG * d1.re), pm(u1.im, SIG * d1.im)};
        }
    }
}

// acc_up += k w ; acc_dn += sig k e_mu^+ w with k the neighbour's FP16 scale
// (1 for unscaled storage), each update one fused multiply-add.
template <int MU, int SIG, typename T>
__device__ __forceinline__ void reconstruct(const cx<T> (&w)[6], cx<T> (&acc)[12], T k) {
    auto add = [&](T& a, T x) { a = fmadd(k, x, a); };
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cx<T> w0 = w[c], w1 = w[3 + c];
        add(acc[c].re, w0.re);
        add(acc[c].im, w0.im);
        add(acc[3 + c].re, w1.re);
        add(acc[3 + c].im, w1.im);
        if constexpr (MU == 0) {  // e^+ w = (i w1, i w0)
            add(acc[6 + c].re, -SIG * w1.im);
            add(acc[6 + c].im, SIG * w1.re);
            add(acc[9 + c].re, -SIG * w0.im);
            add(acc[9 + c].im, SIG * w0.re);
        } else if constexpr (MU == 1) {  // e^+ w = (w1, -w0)
            add(acc[6 + c].re, SIG * w1.re);
            add(acc[6 + c].im, SIG * w1.im);
            add(acc[9 + c].re, -SIG * w0.re);
            add(acc[9 + c].im, -SIG * w0.im);
        } else if constexpr (MU == 2) {  // e^+ w = (i w0, -i w1)
            add(acc[6 + c].re, -SIG * w0.im);
            add(acc[6 + c].im, SIG * w0.re);
            add(acc[9 + c].re, SIG * w1.im);
            add(acc[9 + c].im, -SIG * w1.re);
        } else {  // e^+ w = w
            add(acc[6 + c].re, SIG * w0.re);
            add(acc[6 + c].im, SIG * w0.im);
            add(acc[9 + c].re, SIG * w1.re);
            add(acc[9 + c].im, SIG * w1.im);
        }
    }
}

template <class S>
__device__ __forceinline__ cx<typename S::real> elem_cx(typename S::elem e) {
    if constexpr (S::has_scale) {
        const float2 t = __half22float2(e);
        return {t.x, t.y};
    } else {
        return {e.x, e.y};
    }
}

// acc += k (1 + SIG g_mu) U p   (u: the 3x3 link, row-major; k as in
// reconstruct)
template <class S, int MU, int SIG>
__device__ __forceinline__ void dir_apply(const cx<typename S::real> (&p)[12],
                                          const cx<typename S::real> (&u)[9],
                                          cx<typename S::real> (&acc)[12],
                                          typename S::real k, typename S::real one) {
    using T = typename S::real;
    cx<T> h[6];
    project<MU, SIG, S::has_scale>(p, h, one);
    cx<T> w[6];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            cx<T> t = cmul(u[i * 3 + 0], h[sp * 3 + 0]);
            cfma(t, u[i * 3 + 1], h[sp * 3 + 1]);
            cfma(t, u[i * 3 + 2], h[sp * 3 + 2]);
            w[sp * 3 + i] = t;
        }
    reconstruct<MU, SIG>(w, acc, k);
}

typedef _Float16 pk_h2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ pk_h2 pk_bits(unsigned v) { return __builtin_bit_cast(pk_h2, v); }
__device__ __forceinline__ pk_h2 pk_bcast(_Float16 v) { return pk_h2{v, v}; }
__device__ __forceinline__ pk_h2 pk_itimes(pk_h2 v) { return pk_h2{-v.y, v.x}; }  // i v
template <int SIG>
__device__ __forceinline__ pk_h2 pk_addsig(pk_h2 a, pk_h2 b) {  // a + SIG b
    if constexpr (SIG > 0)
        return a + b;
    else
        return a - b;
}

// acc += k (1 + SIG g_mu) U p on FP16 storage in packed FP16 arithmetic: p
// (the stored neighbour, scaled to max |real| <= 1) and U (|U_ij| <= 1) stay
// FP16, the projection is one packed add and each complex multiply-add two
// packed FMAs per (Re, Im) pair; the products w = U h are widened to FP32 in
// the reconstruct, where the neighbour's scale k multiplies them.
template <int MU, int SIG>
__device__ __forceinline__ void dir_apply_pk(const pk_h2 (&p)[12], const pk_h2 (&u)[9],
                                             cx<float> (&acc)[12], float k) {
    pk_h2 h[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const pk_h2 u0 = p[c], u1 = p[3 + c], d0 = p[6 + c], d1 = p[9 + c];
        if constexpr (MU == 0) {  // e d = (-i d1, -i d0)
            h[c] = pk_addsig<-SIG>(u0, pk_itimes(d1));
            h[3 + c] = pk_addsig<-SIG>(u1, pk_itimes(d0));
        } else if constexpr (MU == 1) {  // e d = (-d1, d0)
            h[c] = pk_addsig<-SIG>(u0, d1);
            h[3 + c] = pk_addsig<SIG>(u1, d0);
        } else if constexpr (MU == 2) {  // e d = (-i d0, i d1)
            h[c] = pk_addsig<-SIG>(u0, pk_itimes(d0));
            h[3 + c] = pk_addsig<SIG>(u1, pk_itimes(d1));
        } else {  // e d = d
            h[c] = pk_addsig<SIG>(u0, d0);
            h[3 + c] = pk_addsig<SIG>(u1, d1);
        }
    }
    cx<float> w[6];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            pk_h2 t = pk_bcast(u[i * 3].x) * h[sp * 3];
            t = __builtin_elementwise_fma(pk_bcast(u[i * 3].y), pk_itimes(h[sp * 3]), t);
#pragma unroll
            for (int j = 1; j < 3; ++j) {
                t = __builtin_elementwise_fma(pk_bcast(u[i * 3 + j].x), h[sp * 3 + j], t);
                t = __builtin_elementwise_fma(pk_bcast(u[i * 3 + j].y), pk_itimes(h[sp * 3 + j]), t);
            }
            w[sp * 3 + i] = {(float)t.x, (float)t.y};
        }
    reconstruct<MU, SIG>(w, acc, k);
}

// A global-memory pointer with the same value in every lane of the wave,
// moved to scalar registers so that loads add a 32-bit lane offset to it.
using gchar = const __attribute__((address_space(1))) char;
__device__ __forceinline__ gchar* uniform_ptr(const char* p) {
    const unsigned long v = reinterpret_cast<unsigned long>(p);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return reinterpret_cast<gchar*>(((unsigned long)hi << 32) | lo);
}

// Input-box position of one output site, set up once per thread so that each
// neighbour costs a few 32-bit integer operations: lex index in the input box,
// the coordinates, and a mask of the dimensions whose coordinate lies in it.
struct InPos {
    int c[4];
    int st[4];  // lex strides of the input box
    int lex;
    int inr;    // bit m: 0 <= c[m] < E[m]
};

__device__ __forceinline__ InPos in_position(const HopGeom& g, const int gc[4]) {
    InPos q;
    q.st[0] = 1;
    q.st[1] = g.in.E[0];
    q.st[2] = g.in.E[0] * g.in.E[1];
    q.st[3] = q.st[2] * g.in.E[2];
    q.lex = 0;
    q.inr = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        q.c[m] = gc[m] - g.in.off[m];
        q.lex += q.c[m] * q.st[m];
        if (q.c[m] >= 0 && q.c[m] < g.in.E[m]) q.inr |= 1 << m;
    }
    return q;
}

// Checkerboard index of the neighbour in direction +/-MU.  Directions in the
// periodic mask wrap (the box spans the lattice there); all others drop hops
// whose source lies outside the input box.
template <int MU, int FWD>
__device__ __forceinline__ bool neighbour(const HopGeom& g, const InPos& q, long& cb) {
    const int E = g.in.E[MU];
    const int cm = q.c[MU] + (FWD ? 1 : -1);
    int nl = q.lex + (FWD ? q.st[MU] : -q.st[MU]);
    bool ok = (q.inr | (1 << MU)) == 15;
    if ((g.periodic >> MU) & 1) {
        if (cm >= E) nl -= E * q.st[MU];
        if (cm < 0) nl += E * q.st[MU];
    } else {
        ok = ok && cm >= 0 && cm < E;
    }
    cb = nl >> 1;
    return ok;
}

// Workgroups are dispatched round-robin over the 8 XCDs (linear id mod 8),
// each with a private L2.  With remapping, XCD k processes one contiguous
// range of logical tiles, so neighbouring sites (whose spinors are shared by
// up to 8 outputs) are fetched into one L2 instead of several.
__device__ __forceinline__ void logical_block(int remap, int& bx, int& d) {
    if (!remap) {
        bx = blockIdx.x;
        d = blockIdx.y;
        return;
    }
    const unsigned G = gridDim.x, T = G * gridDim.y;
    const unsigned lid = blockIdx.y * G + blockIdx.x;
    const unsigned q = T >> 3, r = T & 7, k = lid & 7;
    const unsigned logical = k * q + (k < r ? k : r) + (lid >> 3);
    bx = (int)(logical % G);
    d = (int)(logical / G);
}

template <class S, int LS>
__device__ __forceinline__ void block_sum_store(double v, double* dst) {
    __shared__ double red[16];
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


// compile-time loop: f(std::integral_constant<int, i>) for i in [0, N)
template <class F, int... I>
__device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// 5D programs on the hop output (ph) and on aux (pa): a scale is applied in
// registers; a single bidiagonal step (M5, M5^+, B^+) by exchanging each
// (site, s) value with its s-1 / s+1 neighbour through LDS; longer programs
// (X = B M5^-1 and its adjoint) run as per-(site, component) chains over s in
// LDS, selected at compile time by EPH / EPA because the chain's s-vector
// raises the register footprint.  The links of the workgroup's sites are
// staged in LDS with coalesced 16-byte loads (one load per 16 bytes of links
// instead of one per element and lane) when they fit; the epilogue reuses
// that LDS after the direction loop.
// FP16-storage hops at Ls = 8 or 16 without an aux chain or fused CG update
// fit in 80 VGPRs without spilling: ask for 6 waves per SIMD there (their
// arithmetic, not memory, sets the pace)
template <class S, int LS, bool EPA, bool CG>
constexpr int hop_min_waves() {
    // the matrix-core variant (FP16, Ls = 16) fits 128 VGPRs
    if (S::has_scale && LS == 16 && MSPCG_HOP_MFMA) return MSPCG_HOP_MFMA_WAVES;
    return (S::has_scale && !EPA && !CG && LS == 8) ? 6 : MSPCG_HOP_MINWAVES;
}

// The persistent multi-lattice kernel wraps hop_body in its work-list loop,
// which left alone costs the FP16 Ls = 16 variants one wave per SIMD against
// the plain launch (98-111 VGPRs, 4 waves); hold them to the plain kernel's
// 5 (at Ls = 12 the same cap spills 116-184 bytes per lane).
template <class S, int LS, bool EPA, bool CG>
constexpr int multi_min_waves() {
    return S::has_scale && LS == 16 && hop_min_waves<S, LS, EPA, CG>() < 5
               ? 5
               : hop_min_waves<S, LS, EPA, CG>();
}

// LDS layout of one hop workgroup (SPB sites x LS lanes).
template <class S, int LS>
struct HopShape {
    using T = typename S::real;
    using E = typename S::elem;
    static constexpr int SPB = 256 / LS;
    // s-exchange array, component-major with a padded row per (site, component):
    // entry (site, s, c) at (site * 12 + c) * LSP + s, so the lanes of a site
    // (consecutive s) and the chain threads (consecutive c) both hit distinct banks
    static constexpr int LSP = LS + 1;
    // FP16 links are decoded to FP32 once, when staged (kept FP16 for the
    // packed-FP16 products); LE is the LDS entry
    static constexpr bool PK = S::has_scale && MSPCG_HOP_PK16 && !(LS == 16 && MSPCG_HOP_MFMA);
    using LE = typename std::conditional<S::has_scale && !PK, nt_f2, E>::type;
    static constexpr int NCH = 72 * (int)sizeof(E) / 16;   // 16-byte chunks of one site's links
    static constexpr int LSTR = 72 * (int)sizeof(LE) / 16 + 1;  // padded LDS site stride (chunks)
    static constexpr bool LDSL = SPB * LSTR * 16 <= 40 * 1024;
    // the s-exchange array serves both the chain programs (EPH/EPA) and the
    // single-step programs applied by neighbour exchange
    static constexpr int EPI_BYTES = SPB * 12 * LSP * (int)sizeof(cx<T>);
    // FP16 storage at Ls = 16 (a wave = 4 sites x 16 s): the SU(3) products
    // run as v_mfma_f32_16x16x32_f16 with the links staged in LDS as operand
    // rows (1 KB per site) and a 16-byte zero row
    static constexpr bool MF = S::has_scale && LS == 16 && MSPCG_HOP_MFMA;
    static constexpr int MF_SITE = 1024;
    static constexpr int LNK_BYTES = MF ? SPB * MF_SITE + 16 : (LDSL ? SPB * LSTR * 16 : 16);
    static constexpr int LDS_BYTES = EPI_BYTES > LNK_BYTES ? EPI_BYTES : LNK_BYTES;
};

typedef _Float16 mf_half8 __attribute__((ext_vector_type(8)));
typedef float mf_float4 __attribute__((ext_vector_type(4)));

// One 16-byte operand row of the matrix-core link product: for link row i
// (entries u_i0..u_i2), op 0 gives [Re u, 0, -Im u, 0] and op 1 [Im u, 0, Re u, 0],
// so that with a spinor colour vector packed as [Re psi, 0, Im psi, 0] the
// products give Re(U psi)_i and Im(U psi)_i (FP16 inputs, exact products,
// FP32 accumulation).
__device__ __forceinline__ nt_u4 mf_link_row(const unsigned (&e)[3], int op) {
    // e[j]: __half2 (Re, Im) of u_ij as a 32-bit word
    const unsigned re01 = (e[0] & 0xffffu) | (e[1] << 16);
    const unsigned im01 = (e[0] >> 16) | (e[1] & 0xffff0000u);
    const unsigned re2 = e[2] & 0xffffu, im2 = e[2] >> 16;
    if (op == 0)  // [Re u0, Re u1, Re u2, 0, -Im u0, -Im u1, -Im u2, 0]
        return nt_u4{re01, re2, im01 ^ 0x80008000u, im2 ^ 0x8000u};
    return nt_u4{im01, im2, re01, re2};
}

// Spin component sp of a raw FP16 spinor (unscaled) packed as an MFMA B
// operand: [Re c0, Re c1, Re c2, 0, Im c0, Im c1, Im c2, 0] for the colours
// of that spin.
__device__ __forceinline__ mf_half8 mf_spin_operand(const RawSpinor<F16>& r, int sp) {
    unsigned w[12];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        w[4 * k + 0] = r.c[k].x;
        w[4 * k + 1] = r.c[k].y;
        w[4 * k + 2] = r.c[k].z;
        w[4 * k + 3] = r.c[k].w;
    }
    const unsigned w0 = w[3 * sp], w1 = w[3 * sp + 1], w2 = w[3 * sp + 2];
    // byte selects: low halves of w0, w1 (the real parts), high halves (imaginary)
    const nt_u4 v{__builtin_amdgcn_perm(w1, w0, 0x05040100u), w2 & 0xffffu,
                  __builtin_amdgcn_perm(w1, w0, 0x07060302u), w2 >> 16};
    return __builtin_bit_cast(mf_half8, v);
}

template <int LS>
constexpr int SPB_THREADS() {
    return (256 / LS) * LS;
}

// One workgroup's share of a hop launch: output sites [bx*SPB, (bx+1)*SPB)
// of domain d (in traversal order); gx = workgroups per domain (indexes the
// partial sums); smem: HopShape<S, LS>::LDS_BYTES of LDS, 16-byte aligned.
template <class S, int LS, bool DAG, bool EPH, bool EPA, bool CG>
__device__ __forceinline__ void hop_body(const HopArgs<S>& a, int bx, int d, int gx,
                                         unsigned char* smem) {
    using T = typename S::real;
    using E = typename S::elem;
    using SH = HopShape<S, LS>;
    constexpr int SPB = SH::SPB;
    constexpr int LSP = SH::LSP;
    using LE = typename SH::LE;
    constexpr int NCH = SH::NCH;
    constexpr int LSTR = SH::LSTR;
    constexpr bool LDSL = SH::LDSL;
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem);
    nt_u4* lnk = reinterpret_cast<nt_u4*>(smem);

    const int sl = threadIdx.x / LS;
    const int s = threadIdx.x - sl * LS;
    const long t_lin = (long)bx * SPB + sl;  // position in the traversal order
    const bool active = sl < SPB && t_lin < (a.site_list ? a.n_list : a.g.out.Vh);
    const HopGeom& g = a.g;
    long cb = t_lin;

    int gc[4] = {0, 0, 0, 0};
    const E* gl = nullptr;
    if (active) {
        int oc[4];
        if (a.site_list) {
            cb = a.site_list[t_lin];
            box_coords(g.out, cb, g.out_par, oc);
        } else if (a.tile[0]) {
            // 4D-tiled traversal: consecutive workgroups sweep compact tiles of
            // extent tile[mu] (even, dividing the box), tiles in lex order
            Box tb;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                tb.E[m] = a.tile[m];
                tb.off[m] = 0;
            }
            const unsigned th = (unsigned)(a.tile[0] * a.tile[1] * a.tile[2] * a.tile[3] / 2);
            unsigned st = (unsigned)t_lin / th;
            const unsigned w = (unsigned)t_lin - st * th;
            const int so = g.out.off[0] + g.out.off[1] + g.out.off[2] + g.out.off[3];
            box_coords(tb, w, (g.out_par + so) & 1, oc);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const unsigned nt = (unsigned)(g.out.E[m] / a.tile[m]);
                const unsigned q = st / nt;
                oc[m] += (int)(st - q * nt) * a.tile[m];
                st = q;
            }
            cb = box_cb(g.out, oc);
        } else {
            box_coords(g.out, cb, g.out_par, oc);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) gc[m] = oc[m] + g.out.off[m];
        int lc[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) lc[m] = gc[m] - g.link.off[m];
        gl = a.links + (long)d * a.link_dom_stride +
             ((long)g.out_par * g.link.Vh + box_cb(g.link, lc)) * 72;
        if constexpr (SH::MF) {
            // 64 operand rows per site (direction, op, row i), i = 3 zero
            const unsigned* src = reinterpret_cast<const unsigned*>(gl);
            for (int r = s; r < 64; r += LS) {
                const int dir = r >> 3, op = (r >> 2) & 1, i = r & 3;
                nt_u4 v{0u, 0u, 0u, 0u};
                if (i < 3) {
                    unsigned e[3];
#pragma unroll
                    for (int j = 0; j < 3; ++j) e[j] = src[dir * 9 + i * 3 + j];
                    v = mf_link_row(e, op);
                }
                *reinterpret_cast<nt_u4*>(smem + sl * SH::MF_SITE + r * 16) = v;
            }
        } else if constexpr (LDSL) {
            const nt_u4* src = reinterpret_cast<const nt_u4*>(gl);
            for (int j = s; j < NCH; j += LS) {
                nt_u4 v;
                if constexpr (MSPCG_HOP_NT)
                    v = __builtin_nontemporal_load(src + j);
                else
                    v = src[j];
                if constexpr (SH::PK) {
                    lnk[sl * LSTR + j] = v;
                } else if constexpr (S::has_scale) {
                    const cx<float> e0 = h2f(v.x, 1.f), e1 = h2f(v.y, 1.f);
                    const cx<float> e2 = h2f(v.z, 1.f), e3 = h2f(v.w, 1.f);
                    nt_f4* dst = reinterpret_cast<nt_f4*>(lnk + sl * LSTR + 2 * j);
                    dst[0] = nt_f4{e0.re, e0.im, e1.re, e1.im};
                    dst[1] = nt_f4{e2.re, e2.im, e3.re, e3.im};
                } else {
                    lnk[sl * LSTR + j] = v;
                }
            }
        }
    }
    if constexpr (SH::MF) {
        // sites without output (beyond the box or list) get zero operand rows,
        // so no stale LDS value enters a matrix product
        if (!active && sl < SPB)
            for (int r = s; r < 64; r += LS)
                *reinterpret_cast<nt_u4*>(smem + sl * SH::MF_SITE + r * 16) = nt_u4{0u, 0u, 0u, 0u};
        if (threadIdx.x == 0)
            *reinterpret_cast<nt_u4*>(smem + SPB * SH::MF_SITE) = nt_u4{0u, 0u, 0u, 0u};
        __syncthreads();
    } else if constexpr (LDSL) {
        __syncthreads();
    }

    constexpr int KC = Chunk<S>::K;
    cx<T> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = {0, 0};
    if constexpr (SH::MF) {
        // Every lane of the wave takes part in the matrix products (lanes
        // without an output or a neighbour use zero operands).  The wave's 4
        // sites x 16 s are the 16 columns (s) and the 4 blocks of 4 rows
        // (site, colour row i) of a 16x16x32 product whose A operand is
        // block-diagonal: lane L holds row L%16 = (site gm, row im) against
        // the K block L/16 = site gk, nonzero only when gm == gk.
        const long ibase = (long)d * g.in.Vh;
        const InPos ip = in_position(g, gc);
        gchar* in_d = uniform_ptr(reinterpret_cast<const char*>(a.in.data) + ibase * LS * KC * 16);
        gchar* sc_d = uniform_ptr(reinterpret_cast<const char*>(a.in.scale + ibase * LS));
        const unsigned s16 = (unsigned)s * 16u, s4 = (unsigned)s * 4u;
        const int L = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
        const int gm = (L & 15) >> 2, im = L & 3, gk = L >> 4;
        const unsigned char* arow = (gm == gk) ? smem + (4 * wv + gm) * SH::MF_SITE + im * 16
                                               : smem + SPB * SH::MF_SITE;
        const int astep = (gm == gk) ? 64 : 0;  // bytes between the op-row groups of a direction
        constexpr int SF = DAG ? 1 : -1;
        constexpr int SB = -SF;
        sfor<8>([&](auto di) {
            constexpr int D = decltype(di)::value;
            constexpr int MU = D / 2;
            constexpr bool FWD = (D % 2) == 0;
            long n = 0;
            const bool ok = active && neighbour<MU, FWD ? 1 : 0>(g, ip, n);
            // a dropped hop (or a lane without output) reads the box's first
            // site, finite data, and weighs it by zero: no branch around the
            // loads, and no undefined value enters the matrix product
            const unsigned un = ok ? (unsigned)n : 0u;
            RawSpinor<S> raw;
            gchar* pb = in_d + (unsigned long)((unsigned)__umul24(un, LS * KC * 16) + s16);
#pragma unroll
            for (int k = 0; k < KC; ++k)
                raw.c[k] = *reinterpret_cast<const __attribute__((address_space(1))) nt_u4*>(
                    pb + k * LS * 16);
            const float scn = *reinterpret_cast<const __attribute__((address_space(1))) float*>(
                sc_d + (unsigned long)((unsigned)__umul24(un, LS * 4) + s4));
            raw.sc = ok ? scn : 0.f;
            constexpr int LDIR = FWD ? MU : 4 + MU;  // link slot of this direction
            const mf_half8 are =
                *reinterpret_cast<const mf_half8*>(arow + astep * (2 * LDIR));
            const mf_half8 aim =
                *reinterpret_cast<const mf_half8*>(arow + astep * (2 * LDIR + 1));
            cx<float> up[12];
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
                const mf_half8 b = mf_spin_operand(raw, sp);
                const mf_float4 z = {0.f, 0.f, 0.f, 0.f};
                const mf_float4 dr = __builtin_amdgcn_mfma_f32_16x16x32_f16(are, b, z, 0, 0, 0);
                const mf_float4 dm = __builtin_amdgcn_mfma_f32_16x16x32_f16(aim, b, z, 0, 0, 0);
#pragma unroll
                for (int i = 0; i < 3; ++i) up[sp * 3 + i] = {dr[i], dm[i]};
            }
            // (1 + sig g_mu) U psi = U (1 + sig g_mu) psi: project the products
            cx<float> h[6];
            project<MU, FWD ? SF : SB, false>(up, h, 1.f);
            reconstruct<MU, FWD ? SF : SB>(h, acc, raw.sc);
            // finish this direction here: the empty asm pins the accumulators
            // (so the products are not kept live and folded in at the end)
            // and the scheduling barrier keeps the next direction's loads
            // below; both cost less than the registers they save
#pragma unroll
            for (int c = 0; c < 12; ++c) asm volatile("" : "+v"(acc[c].re), "+v"(acc[c].im));
            __builtin_amdgcn_sched_barrier(0);
        });
    } else if (active) {
        const long ibase = (long)d * g.in.Vh;
        const InPos ip = in_position(g, gc);
        // the domain's input box (a workgroup-uniform base, kept in scalar
        // registers) and this lane's byte offsets from it
        gchar* in_d = uniform_ptr(reinterpret_cast<const char*>(a.in.data) + ibase * LS * KC * 16);
        gchar* sc_d =
            S::has_scale ? uniform_ptr(reinterpret_cast<const char*>(a.in.scale + ibase * LS)) : nullptr;
        const unsigned s16 = (unsigned)s * 16u, s4 = (unsigned)s * 4u;
        // 1.0 that the compiler cannot fold (see project)
        T one = 1;
        if constexpr (S::has_scale) asm("s_mov_b32 %0, 1.0" : "=s"(one));
        // forward terms use (1 - g) and backward (1 + g); the dagger swaps them
        constexpr int SF = DAG ? 1 : -1;
        constexpr int SB = -SF;
        constexpr int PF = S::has_scale ? MSPCG_HOP_PF16
                           : sizeof(T) == 8  ? MSPCG_HOP_PF64
                                             : MSPCG_HOP_PF32;
        static_assert(8 % PF == 0, "prefetch group must divide 8");
        sfor<8 / PF>([&](auto gi) {
            constexpr int G0 = decltype(gi)::value * PF;
            RawSpinor<S> raw[PF];
            bool ok[PF];
            sfor<PF>([&](auto j) {
                constexpr int D = G0 + decltype(j)::value;
                constexpr int MU = D / 2;
                constexpr bool FWD = (D % 2) == 0;
                long n = 0;
                ok[j] = neighbour<MU, FWD ? 1 : 0>(g, ip, n);
                if (ok[j]) {
                    if constexpr (S::has_scale) {
                        const unsigned un = (unsigned)n;
                        gchar* pb = in_d + (unsigned long)((unsigned)__umul24(un, LS * KC * 16) + s16);
#pragma unroll
                        for (int k = 0; k < KC; ++k)
                            raw[j].c[k] = *reinterpret_cast<const __attribute__((address_space(1))) nt_u4*>(
                                pb + k * LS * 16);
                        if constexpr (S::has_scale)
                            raw[j].sc = *reinterpret_cast<const __attribute__((address_space(1))) float*>(
                                sc_d + (unsigned long)((unsigned)__umul24(un, LS * 4) + s4));
                    } else {
                        load_raw_at<S>(a.in, (ibase + n) * LS, s, LS, raw[j]);
                    }
                }
            });
            sfor<PF>([&](auto j) {
                constexpr int D = G0 + decltype(j)::value;
                constexpr int MU = D / 2;
                constexpr bool FWD = (D % 2) == 0;
                constexpr int LD = (FWD ? MU : 4 + MU) * 9;  // first entry of this link
                if constexpr (SH::PK) {
                    static_assert(LDSL, "packed-FP16 hops read their links from LDS");
                    if (ok[j]) {
                        pk_h2 p[12], u[9];
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            p[4 * q + 0] = pk_bits(raw[j].c[q].x);
                            p[4 * q + 1] = pk_bits(raw[j].c[q].y);
                            p[4 * q + 2] = pk_bits(raw[j].c[q].z);
                            p[4 * q + 3] = pk_bits(raw[j].c[q].w);
                        }
                        const unsigned* le = reinterpret_cast<const unsigned*>(lnk + sl * LSTR) + LD;
#pragma unroll
                        for (int q = 0; q < 9; ++q) u[q] = pk_bits(le[q]);
                        dir_apply_pk<MU, FWD ? SF : SB>(p, u, acc, raw[j].sc);
                    }
                } else if (ok[j]) {
                    cx<T> p[12];
                    decode_raw<S>(raw[j], p, false);
                    cx<T> u[9];
                    if constexpr (LDSL) {
                        const LE* le = reinterpret_cast<const LE*>(lnk + sl * LSTR) + LD;
#pragma unroll
                        for (int k = 0; k < 9; ++k) u[k] = {(T)le[k].x, (T)le[k].y};
                    } else {
#pragma unroll
                        for (int k = 0; k < 9; ++k) u[k] = load_link<S, MSPCG_HOP_NT>(gl + LD + k);
                    }
                    const T k = S::has_scale ? (T)raw[j].sc : (T)1;
                    dir_apply<S, MU, FWD ? SF : SB>(p, u, acc, k, one);
                }
            });
        });
    }

    const long obase = ((long)d * g.out.Vh + cb) * LS;
    const T mf = (T)a.mf;
    // one bidiagonal step v_s <- sc (v_s + a v_{s-/+1}), the -mf corner closing
    // the s direction; entered by all threads (uniform arguments)
    auto bidi1 = [&](const FiveDProg& P, cx<T>(&v)[12]) {
        __syncthreads();  // LDS free: staged links or an earlier phase
        if (active) {
#pragma unroll
            for (int c = 0; c < 12; ++c) lds[(sl * 12 + c) * LSP + s] = v[c];
        }
        __syncthreads();
        if (active) {
            const T av = (T)P.a[0];
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const bool up = c < 6;
                const bool below = up != (P.dag[0] != 0);
                const bool corner = below ? s == 0 : s == LS - 1;
                const int s2 = below ? (corner ? LS - 1 : s - 1) : (corner ? 0 : s + 1);
                const cx<T> nb = lds[(sl * 12 + c) * LSP + s2];
                const T f = corner ? -(av * mf) : av;
                const T sc = (T)(up ? P.scale[0] : P.scale[1]);
                v[c] = {sc * (v[c].re + f * nb.re), sc * (v[c].im + f * nb.im)};
            }
        }
    };
    // chain program over s for every (site, component), in place in LDS
    auto chains = [&](const FiveDProg& P) {
        for (int ch = threadIdx.x; ch < SPB * 12; ch += blockDim.x) {
            const int csl = ch / 12, comp = ch - csl * 12;
            cx<T> v[LS];
#pragma unroll
            for (int t = 0; t < LS; ++t) v[t] = lds[(csl * 12 + comp) * LSP + t];
            apply_prog<LS, T>(P, comp < 6, mf, v);
#pragma unroll
            for (int t = 0; t < LS; ++t) lds[(csl * 12 + comp) * LSP + t] = v[t];
        }
    };

    cx<T> res[12];
    if (a.ph.identity) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const T sc = (T)(c < 6 ? a.ph.scale[0] : a.ph.scale[1]);
            res[c] = {acc[c].re * sc, acc[c].im * sc};
        }
    } else if (!EPH) {
#pragma unroll
        for (int c = 0; c < 12; ++c) res[c] = acc[c];
        bidi1(a.ph, res);
    } else {
        __syncthreads();  // every wave is done with the staged links
        if (active) {
#pragma unroll
            for (int c = 0; c < 12; ++c) lds[(sl * 12 + c) * LSP + s] = acc[c];
        }
        __syncthreads();
        chains(a.ph);
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 12; ++c) res[c] = lds[(sl * 12 + c) * LSP + s];
    }

    if (a.has_aux) {
        // aux lives on its own box; sites outside it contribute zero
        cx<T> x[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) x[c] = {0, 0};
        if (active) {
            int ac[4];
            bool in = true;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                ac[m] = gc[m] - g.aux.off[m];
                in = in && ac[m] >= 0 && ac[m] < g.aux.E[m];
            }
            if (in) load_spinor_at<S, MSPCG_HOP_NT>(a.aux, ((long)d * g.aux.Vh + box_cb(g.aux, ac)) * LS, s, LS, x);
        }
        if (a.pa.identity) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const T sc = (T)(c < 6 ? a.pa.scale[0] : a.pa.scale[1]);
                res[c].re += sc * x[c].re;
                res[c].im += sc * x[c].im;
            }
        } else if (!EPA) {
            bidi1(a.pa, x);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                res[c].re += x[c].re;
                res[c].im += x[c].im;
            }
        } else {
            __syncthreads();  // the hop epilogue may still read lds
            if (active) {
#pragma unroll
                for (int c = 0; c < 12; ++c) lds[(sl * 12 + c) * LSP + s] = x[c];
            }
            __syncthreads();
            chains(a.pa);
            __syncthreads();
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const cx<T> t = lds[(sl * 12 + c) * LSP + s];
                res[c].re += t.re;
                res[c].im += t.im;
            }
        }
    }

    if constexpr (CG) {
        // fused CG update: r -= alpha out, x += alpha p, partials of |r|^2
        double n2 = 0;
        if (active) {
            if (a.cg_keep_out) store_spinor_at<S, MSPCG_HOP_NT>(a.out, obase, s, LS, res);
            const T al = (T)(a.cg_alpha ? a.cg_alpha[d] : a.cg_sc->alpha);
            cx<T> v[12];
            load_spinor_at<S, MSPCG_HOP_NT>(cfield(a.cg_r), obase, s, LS, v);
            T t2 = 0;  // one entry's 24 squares in the arithmetic type
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                v[c].re -= al * res[c].re;
                v[c].im -= al * res[c].im;
                t2 = fmadd(v[c].re, v[c].re, t2);
                t2 = fmadd(v[c].im, v[c].im, t2);
            }
            n2 = (double)t2;
            store_spinor_at<S>(a.cg_r, obase, s, LS, v);
            if (a.cg_x.data) {
                cx<T> pv[12];
                load_spinor_at<S, MSPCG_HOP_NT>(a.cg_p, obase, s, LS, pv);
                if (a.cg_first) {
#pragma unroll
                    for (int c = 0; c < 12; ++c) v[c] = {al * pv[c].re, al * pv[c].im};
                } else {
                    load_spinor_at<S, MSPCG_HOP_NT>(cfield(a.cg_x), obase, s, LS, v);
#pragma unroll
                    for (int c = 0; c < 12; ++c) {
                        v[c].re += al * pv[c].re;
                        v[c].im += al * pv[c].im;
                    }
                }
                store_spinor_at<S>(a.cg_x, obase, s, LS, v);
            }
        }
        block_sum_store<S, LS>(n2, a.partials + (long)d * gx + bx);
        return;
    }
    if (active) store_spinor_at<S, MSPCG_HOP_NT>(a.out, obase, s, LS, res);
    if (a.partials) {
        double n2 = 0;
        if (active) {
            // norm of what was stored (FP16 rounding included is not needed:
            // the reduction uses the arithmetic value)
            T t2 = 0;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                t2 = fmadd(res[c].re, res[c].re, t2);
                t2 = fmadd(res[c].im, res[c].im, t2);
            }
            n2 = (double)t2;
        }
        block_sum_store<S, LS>(n2, a.partials + (long)d * gx + bx);
    }
}

template <class S, int LS, bool DAG, bool EPH, bool EPA, bool CG = false>
__global__ __launch_bounds__(256, (hop_min_waves<S, LS, EPA, CG>())) void hop_kernel(HopArgs<S> a) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[HopShape<S, LS>::LDS_BYTES];
    if (a.done && *a.done) return;
    int bx, d;
    logical_block(a.xcd_remap, bx, d);
    hop_body<S, LS, DAG, EPH, EPA, CG>(a, bx, d, (int)gridDim.x, smem);
}

template <class S, int LS>
static void launch_ls(const HopArgs<S>& a, int ndom, bool dag, hipStream_t st) {
    constexpr int SPB = 256 / LS;
    const long nout = a.site_list ? a.n_list : a.g.out.Vh;
    dim3 grid((unsigned)((nout + SPB - 1) / SPB), (unsigned)ndom);
    dim3 block(SPB * LS);
    // programs of at most one bidiagonal step are applied by s-exchange
    auto chain = [](const FiveDProg& P) {
        return !P.identity && !(P.nsteps == 1 && P.kind[0] == STEP_BIDI);
    };
    const bool eph = chain(a.ph);
    const bool epa = a.has_aux && chain(a.pa);
    if (a.cg_r.data) {
        // the fused CG update only follows the last (dagger) hop of A; the
        // chain variant also handles single-step programs
        if (dag && !eph && !epa)
            hipLaunchKernelGGL((hop_kernel<S, LS, true, false, false, true>), grid, block, 0, st, a);
        else if (dag)
            hipLaunchKernelGGL((hop_kernel<S, LS, true, true, true, true>), grid, block, 0, st, a);
        return;
    }
#define MSPCG_HOP_LAUNCH(D, H, A) \
    hipLaunchKernelGGL((hop_kernel<S, LS, D, H, A>), grid, block, 0, st, a)
    if (dag) {
        if (eph && epa) MSPCG_HOP_LAUNCH(true, true, true);
        else if (eph) MSPCG_HOP_LAUNCH(true, true, false);
        else if (epa) MSPCG_HOP_LAUNCH(true, false, true);
        else MSPCG_HOP_LAUNCH(true, false, false);
    } else {
        if (eph && epa) MSPCG_HOP_LAUNCH(false, true, true);
        else if (eph) MSPCG_HOP_LAUNCH(false, true, false);
        else if (epa) MSPCG_HOP_LAUNCH(false, false, true);
        else MSPCG_HOP_LAUNCH(false, false, false);
    }
#undef MSPCG_HOP_LAUNCH
}

template <class S>
int launch_hop(const HopArgs<S>& a, int Ls, int ndom, bool dag, hipStream_t st) {
    if (a.cg_r.data && (!dag || !a.partials)) return -1;
    // FP16-storage hops address a domain's input sites with 32-bit offsets
    const long site_bytes = (long)Ls * Chunk<S>::K * 16;
    if (S::has_scale && (a.g.in.Vh >= (1L << 24) || a.g.in.Vh * site_bytes > 0xffffffffL)) return -1;
    switch (Ls) {
#define MSPCG_CASE(L) \
    case L: launch_ls<S, L>(a, ndom, dag, st); break;
        MSPCG_LS_LIST(MSPCG_CASE)
#undef MSPCG_CASE
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <class S>
long hop_grid_x(long Vh, int Ls) {
    const int spb = 256 / Ls;
    return (Vh + spb - 1) / spb;
}

// One launch over a work list of several lattices that share Ls (launch
// bounds and LDS as for one lattice's hop).
template <class S, int LS, bool DAG, bool EPH, bool EPA, bool CG>
__global__ __launch_bounds__(256, (multi_min_waves<S, LS, EPA, CG>())) void multi_hop_kernel(
    const MultiHop<S>* __restrict__ m) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[HopShape<S, LS>::LDS_BYTES];
    const int n = m->n;
    const long items = m->first[n];
    // the hardware deals workgroups to the eight XCDs in turn: the workgroups
    // of XCD k walk the k-th contiguous eighth of the list, so that
    // neighbouring tiles of one domain share an L2
    const unsigned G = gridDim.x, k = blockIdx.x & 7;
    const unsigned nk = (G >> 3) + (k < (G & 7) ? 1u : 0u);
    const long lo = items * k / 8, hi = items * (k + 1) / 8;
    for (long it = lo + (blockIdx.x >> 3); it < hi; it += nk) {
        int i = 0;
        while (i + 1 < n && it >= m->first[i + 1]) ++i;
        const HopArgs<S>& a = m->a[i];
        if (a.done && *a.done) continue;  // this lattice has converged (uniform branch)
        const int gx = m->gx[i];
        const long r = it - m->first[i];
        const int d = (int)(r / gx), bx = (int)(r - (long)d * gx);
        hop_body<S, LS, DAG, EPH, EPA, CG>(a, bx, d, gx, smem);
        __syncthreads();  // LDS is reused by the next item
    }
}

// persistent grid: as many workgroups as the CUs hold at once (at least 8,
// a multiple of 8 so that every XCD gets the same count), never more than
// the items
template <class S, int LS, bool D, bool H, bool A, bool C>
static dim3 multi_grid(long items) {
    static int resident = 0;  // per kernel instance; the library drives one device type
    if (!resident) {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, multi_hop_kernel<S, LS, D, H, A, C>,
                                                         SPB_THREADS<LS>(), 0) != hipSuccess ||
            cus <= 0 || per <= 0)
            per = 4, cus = 256;
        resident = ((cus * per + 7) / 8) * 8;
    }
    const long g = items < resident ? ((items + 7) / 8) * 8 : resident;
    return dim3((unsigned)g);
}

template <class S, int LS>
static int launch_multi_ls(const MultiHop<S>* dev, long items, bool dag, bool eph, bool epa,
                           bool cg, hipStream_t st) {
    dim3 block(SPB_THREADS<LS>());
#define MSPCG_MH(D, H, A, C)                                                                  \
    hipLaunchKernelGGL((multi_hop_kernel<S, LS, D, H, A, C>), (multi_grid<S, LS, D, H, A, C>(items)), \
                       block, 0, st, dev)
    if (!dag && eph && !epa && !cg) MSPCG_MH(false, true, false, false);
    else if (!dag && !eph && !epa && !cg) MSPCG_MH(false, false, false, false);
    else if (dag && eph && !epa && !cg) MSPCG_MH(true, true, false, false);
    else if (dag && !eph && !epa && cg) MSPCG_MH(true, false, false, true);
    else if (dag && cg) MSPCG_MH(true, true, true, true);
    else return -1;
#undef MSPCG_MH
    return 0;
}

template <class S>
int launch_multi_hop(const MultiHop<S>* dev, long items, int Ls, bool dag, bool eph, bool epa,
                     bool cg, hipStream_t st) {
    if (items <= 0) return 0;
    int e;
    switch (Ls) {
        case 8: e = launch_multi_ls<S, 8>(dev, items, dag, eph, epa, cg, st); break;
        case 12: e = launch_multi_ls<S, 12>(dev, items, dag, eph, epa, cg, st); break;
        case 16: e = launch_multi_ls<S, 16>(dev, items, dag, eph, epa, cg, st); break;
        default: return -1;
    }
    if (e) return e;
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace mspcg
