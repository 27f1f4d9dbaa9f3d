// Shared device-side definitions of the MSPCG HIP library (gfx950).
//
// Internal data layout (all on device, chosen for coalesced wave64 access):
//   * A "box" is a 4D sub-lattice [0,E0)x[0,E1)x[0,E2)x[0,E3) placed at offset
//     `off` from the origin of its domain; the whole periodic lattice is the
//     special case of one domain whose boxes are the lattice itself.
//   * Sites of one parity in a box are numbered by cb = lex/2 with
//     lex = ((t*E2 + z)*E1 + y)*E0 + x (E0 even).
//   * Spinor fields are site-blocked: entry i = site*Ls + s (site = d*Vh + cb
//     for domain fields) keeps its 12 complex components in 16-byte chunks of
//     V = 16/sizeof(elem) components (V = 1, 2, 4 for FP64, FP32, FP16), and
//     chunk k of (site, s) is chunk number (site*K + k)*Ls + s of the array,
//     K = 12/V.  A thread owns one (site, s); consecutive lanes hold
//     consecutive s, so every chunk access of a wave is contiguous, and a
//     spinor costs K vector loads of 16 bytes per lane whatever the precision.
//   * FP16 fields store value/scale as __half2 per complex component plus one
//     FP32 scale per entry (the max |real| over its 24 reals), scale[i].
//   * Links are stored per output parity and link-box site as
//     [parity][Vh_linkbox][8][9]: dirs 0..3 hold U_mu(x), dirs 4..7 hold
//     U_mu(x-mu)^+ (already daggered), with the antiperiodic-time sign folded
//     in.  The 72 entries of a site are contiguous so a workgroup stages them
//     with a few coalesced 16-byte loads and all Ls lanes reuse them.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace mspcg {

constexpr int kMaxLs = 32;
constexpr int kMaxDomains = 4096;

template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// fused a*b + c in the arithmetic type (one rounding)
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
// a += b * c as a chain of four fused multiply-adds
template <typename T>
__device__ __forceinline__ void cfma(cx<T>& a, cx<T> b, cx<T> c) {
    a.re = fmadd(b.re, c.re, a.re);
    a.re = fmadd(-b.im, c.im, a.re);
    a.im = fmadd(b.re, c.im, a.im);
    a.im = fmadd(b.im, c.re, a.im);
}

// Storage policies.  `real` is the arithmetic type; `elem` the stored complex.
struct F64 {
    using real = double;
    using elem = double2;
    static constexpr bool has_scale = false;
    static constexpr int bytes_spinor = 192;  // 12 complex x 16 B
    static constexpr int bytes_link = 144;
};
struct F32 {
    using real = float;
    using elem = float2;
    static constexpr bool has_scale = false;
    static constexpr int bytes_spinor = 96;
    static constexpr int bytes_link = 72;
};
struct F16 {
    using real = float;
    using elem = __half2;
    static constexpr bool has_scale = true;
    static constexpr int bytes_spinor = 52;  // 12 x 4 B + 4 B scale
    static constexpr int bytes_link = 36;
};

// A field of N entries (site, s) with `ls` entries per site (+ scales for FP16).
template <class S>
struct Field {
    typename S::elem* data;
    float* scale;  // FP16 only
    long N;        // entries (site, s)
    int ls;        // entries per site (the Ls of the field)
};

template <class S>
struct CField {
    const typename S::elem* data;
    const float* scale;
    long N;
    int ls;
};

template <class S>
__host__ __device__ inline CField<S> cfield(Field<S> f) {
    return {f.data, f.scale, f.N, f.ls};
}

// 16-byte chunk types of the site-blocked layout
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef unsigned nt_u4 __attribute__((ext_vector_type(4)));

template <class S>
struct Chunk {
    static constexpr int V = 16 / (int)sizeof(typename S::elem);  // components per chunk
    static constexpr int K = 12 / V;                              // chunks per spinor
};

__device__ __forceinline__ cx<float> h2f(unsigned u, float sc) {
    __half2 h;
    __builtin_memcpy(&h, &u, 4);
    const float2 t = __half22float2(h);
    return {t.x * sc, t.y * sc};
}
__device__ __forceinline__ unsigned f2h(float re, float im) {
    const __half2 h = __floats2half2_rn(re, im);
    unsigned u;
    __builtin_memcpy(&u, &h, 4);
    return u;
}

// This thread's part of a fixed-order strided sum: p[t] + p[t + B] + ... for
// t = threadIdx.x, B = blockDim.x, added in that order.  Loads are issued in
// groups of eight before their adds so that they overlap instead of each
// waiting out a full memory latency; the order of the adds is unchanged.
__device__ __forceinline__ double strided_sum(const double* p, int n) {
    const int B = (int)blockDim.x;
    double v = 0;
    int i = (int)threadIdx.x;
    for (; i + 7 * B < n; i += 8 * B) {
        double t[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) t[k] = p[i + k * B];
#pragma unroll
        for (int k = 0; k < 8; ++k) v += t[k];
    }
    for (; i < n; i += B) v += p[i];
    return v;
}

// The undecoded 16-byte chunks of one entry (+ its FP16 scale): loading raw
// chunks first and decoding later lets a thread keep several neighbour
// spinors in flight in few registers.
template <class S>
struct RawSpinor {
    nt_u4 c[Chunk<S>::K];
    float sc;
};

// Entry (base + s) with base = site*ls.  Callers with a compile-time Ls pass
// it as `ls` so the index arithmetic folds.
// NT: the entry is read once (streamed), so its lines are not kept in cache.
template <class S, bool NT = false>
__device__ __forceinline__ void load_raw_at(CField<S> f, long base, int s, int ls, RawSpinor<S>& r) {
    const nt_u4* p = reinterpret_cast<const nt_u4*>(f.data) + base * Chunk<S>::K + s;
#pragma unroll
    for (int k = 0; k < Chunk<S>::K; ++k) {
        if constexpr (NT)
            r.c[k] = __builtin_nontemporal_load(p + (long)k * ls);
        else
            r.c[k] = p[(long)k * ls];
    }
    if constexpr (S::has_scale) {
        if constexpr (NT)
            r.sc = __builtin_nontemporal_load(f.scale + base + s);
        else
            r.sc = f.scale[base + s];
    }
}

template <class S>
__device__ __forceinline__ void decode_raw(const RawSpinor<S>& r, cx<typename S::real> (&v)[12],
                                           bool apply_scale = true) {
    if constexpr (S::has_scale) {
        const float sc = apply_scale ? r.sc : 1.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            v[4 * k + 0] = h2f(r.c[k].x, sc);
            v[4 * k + 1] = h2f(r.c[k].y, sc);
            v[4 * k + 2] = h2f(r.c[k].z, sc);
            v[4 * k + 3] = h2f(r.c[k].w, sc);
        }
    } else if constexpr (sizeof(typename S::real) == 8) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const nt_d2 t = __builtin_bit_cast(nt_d2, r.c[c]);
            v[c] = {t.x, t.y};
        }
    } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const nt_f4 t = __builtin_bit_cast(nt_f4, r.c[k]);
            v[2 * k] = {t.x, t.y};
            v[2 * k + 1] = {t.z, t.w};
        }
    }
}

template <class S, bool NT = false>
__device__ __forceinline__ void load_spinor_at(CField<S> f, long base, int s, int ls,
                                               cx<typename S::real> (&v)[12]) {
    RawSpinor<S> r;
    load_raw_at<S, NT>(f, base, s, ls, r);
    decode_raw<S>(r, v);
}

// entry i -> (base = site*ls, s); 32-bit division whenever the index fits
__device__ __forceinline__ int entry_lane(long i, int ls) {
    if (i <= 0xffffffffL) return (int)((unsigned)i % (unsigned)ls);
    return (int)(i % ls);
}

template <class S>
__device__ __forceinline__ void load_spinor(CField<S> f, long i, cx<typename S::real> (&v)[12]) {
    const int s = entry_lane(i, f.ls);
    load_spinor_at<S>(f, i - s, s, f.ls, v);
}

template <class V, bool NT>
__device__ __forceinline__ void put16(V* p, V v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Single-use streams (hop outputs, links) bypass L2 allocation with
// nontemporal accesses so that the L2 keeps the neighbour spinors, which are
// re-read by up to eight output sites.
template <class S, bool NT = false>
__device__ __forceinline__ void store_spinor_at(Field<S> f, long base, int s, int ls,
                                                const cx<typename S::real> (&v)[12]) {
    const long q = base * Chunk<S>::K + s;
    if constexpr (S::has_scale) {
        float m = 0.f;
#pragma unroll
        for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
        const float inv = m > 0.f ? 1.0f / m : 0.f;
        if (NT)
            __builtin_nontemporal_store(m, f.scale + base + s);
        else
            f.scale[base + s] = m;
        nt_u4* p = reinterpret_cast<nt_u4*>(f.data) + q;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            nt_u4 t;
            t.x = f2h(v[4 * k + 0].re * inv, v[4 * k + 0].im * inv);
            t.y = f2h(v[4 * k + 1].re * inv, v[4 * k + 1].im * inv);
            t.z = f2h(v[4 * k + 2].re * inv, v[4 * k + 2].im * inv);
            t.w = f2h(v[4 * k + 3].re * inv, v[4 * k + 3].im * inv);
            put16<nt_u4, NT>(p + (long)k * ls, t);
        }
    } else if constexpr (sizeof(typename S::real) == 8) {
        nt_d2* p = reinterpret_cast<nt_d2*>(f.data) + q;
#pragma unroll
        for (int c = 0; c < 12; ++c) put16<nt_d2, NT>(p + (long)c * ls, nt_d2{v[c].re, v[c].im});
    } else {
        nt_f4* p = reinterpret_cast<nt_f4*>(f.data) + q;
#pragma unroll
        for (int k = 0; k < 6; ++k)
            put16<nt_f4, NT>(p + (long)k * ls,
                             nt_f4{v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im});
    }
}

template <class S, bool NT = false>
__device__ __forceinline__ void store_spinor(Field<S> f, long i, const cx<typename S::real> (&v)[12]) {
    const int s = entry_lane(i, f.ls);
    store_spinor_at<S, NT>(f, i - s, s, f.ls, v);
}

template <class S, bool NT = false>
__device__ __forceinline__ cx<typename S::real> load_link(const typename S::elem* p) {
    if constexpr (S::has_scale) {
        if (NT) {
            const unsigned u = __builtin_nontemporal_load(reinterpret_cast<const unsigned*>(p));
            const float2 t = __half22float2(*reinterpret_cast<const __half2*>(&u));
            return {t.x, t.y};
        }
        const float2 t = __half22float2(*p);
        return {t.x, t.y};
    } else if constexpr (sizeof(typename S::real) == 8) {
        if (NT) {
            const nt_d2 t = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
            return {t.x, t.y};
        }
        const auto t = *p;
        return {t.x, t.y};
    } else {
        if (NT) {
            const nt_f2 t = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p));
            return {t.x, t.y};
        }
        const auto t = *p;
        return {t.x, t.y};
    }
}

// Geometry of one box (see the layout notes above).
struct Box {
    int E[4];
    int off[4];  // origin relative to the domain origin
    long Vh;     // sites per parity
};

// Local coordinates of checkerboard site cb of global parity `par` in box b.
// The domain origin has even global parity (domains start at multiples of
// even block extents), so the global parity of a local site is
// (x + y + z + t + sum(off)) mod 2.
// Box site counts stay below 2^31 (checked when contexts and domains are
// made), so the index arithmetic is 32-bit.
__device__ __forceinline__ void box_coords(const Box& b, long cb, int par, int c[4]) {
    const unsigned hx = (unsigned)b.E[0] >> 1, e1 = (unsigned)b.E[1], e2 = (unsigned)b.E[2];
    const unsigned u = (unsigned)cb;
    const unsigned r = u / hx;
    const int xh = (int)(u - r * hx);
    const unsigned r2 = r / e1;
    c[1] = (int)(r - r2 * e1);
    const unsigned r3 = r2 / e2;
    c[2] = (int)(r2 - r3 * e2);
    c[3] = (int)r3;
    const int so = b.off[0] + b.off[1] + b.off[2] + b.off[3];
    c[0] = 2 * xh + ((par + c[1] + c[2] + c[3] + so) & 1);
}

__device__ __forceinline__ long box_cb(const Box& b, const int c[4]) {
    const unsigned lex =
        (((unsigned)c[3] * b.E[2] + c[2]) * (unsigned)b.E[1] + c[1]) * (unsigned)b.E[0] + c[0];
    return (long)(lex >> 1);
}

// Dense per-chirality 5D operators are applied as short programs of
// elementary steps on the s-vector of one (site, component) (see fived.h).
enum StepKind : int { STEP_NONE = 0, STEP_BIDI = 1, STEP_INV = 2 };
struct FiveDProg {
    int nsteps;
    int kind[3];
    int dag[3];        // 0: K, 1: K^+
    double a[3];       // BIDI: 1 + a K ; INV: (1 - a K)^-1
    double scale[2];   // final scale for upper (spins 0,1) / lower (spins 2,3) chirality
    int identity;      // 1: program is scale only (no s mixing)
};

}  // namespace mspcg
