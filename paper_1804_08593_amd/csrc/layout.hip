// Layout conversion kernels: boundary (lexicographic complex128) fields to the
// internal parity / domain layouts, link packing, and precision conversion.
#include "common.h"
#include "kernels.h"

namespace mspcg {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void lex_coords(long lex, const int L[4], int c[4]) {
    c[0] = (int)(lex % L[0]);
    lex /= L[0];
    c[1] = (int)(lex % L[1]);
    lex /= L[1];
    c[2] = (int)(lex % L[2]);
    c[3] = (int)(lex / L[2]);
}

__device__ __forceinline__ long lex_of(const int c[4], const int L[4]) {
    return (((long)c[3] * L[2] + c[2]) * L[1] + c[1]) * L[0] + c[0];
}

struct Dims {
    int L[4];
};

// whole-lattice parity field: site cb of parity par -> lexicographic index
__device__ __forceinline__ long cb_to_lex(long cb, int par, const Dims& d) {
    Box b;
    for (int m = 0; m < 4; ++m) {
        b.E[m] = d.L[m];
        b.off[m] = 0;
    }
    b.Vh = 0;
    int c[4];
    box_coords(b, cb, par, c);
    return lex_of(c, d.L);
}

template <class S>
__global__ void pack_parity_kernel(const double2* full, Field<S> out, Dims d, int Ls, int par,
                                   long V4, long Vh) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Vh * Ls) return;
    const long cb = i / Ls;
    const int s = (int)(i - cb * Ls);
    const long lex = cb_to_lex(cb, par, d);
    const double2* src = full + ((long)s * V4 + lex) * 12;
    cx<typename S::real> v[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const double2 t = src[c];
        v[c] = {(typename S::real)t.x, (typename S::real)t.y};
    }
    store_spinor<S>(out, i, v);
}

template <class S>
__global__ void unpack_parity_kernel(CField<S> in, double2* full, Dims d, int Ls, int par,
                                     int zero_other, long V4, long Vh) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Vh * Ls) return;
    const long cb = i / Ls;
    const int s = (int)(i - cb * Ls);
    const long lex = cb_to_lex(cb, par, d);
    cx<typename S::real> v[12];
    load_spinor<S>(in, i, v);
    double2* dst = full + ((long)s * V4 + lex) * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) dst[c] = make_double2((double)v[c].re, (double)v[c].im);
    if (zero_other) {
        // the other-parity partner site in the same x pair is lex ^ 1
        const long lex2 = lex ^ 1;
        double2* d2 = full + ((long)s * V4 + lex2) * 12;
#pragma unroll
        for (int c = 0; c < 12; ++c) d2[c] = make_double2(0.0, 0.0);
    }
}

struct DomGrid {
    int L[4], blk[4], nb[4];
};

// domain d, interior site cb (parity par) -> global cb of the same site
__device__ __forceinline__ long dom_to_global_cb(const DomGrid& g, int d, long cb, int par) {
    Box b;
    for (int m = 0; m < 4; ++m) {
        b.E[m] = g.blk[m];
        b.off[m] = 0;
    }
    b.Vh = 0;
    int c[4];
    box_coords(b, cb, par, c);
    int dc[4];
    int r = d;
    for (int m = 0; m < 4; ++m) {
        dc[m] = r % g.nb[m];
        r /= g.nb[m];
    }
    int gcoord[4];
    for (int m = 0; m < 4; ++m) gcoord[m] = dc[m] * g.blk[m] + c[m];
    return lex_of(gcoord, g.L) >> 1;
}

template <class SG, class SD>
__global__ void global_to_domain_kernel(CField<SG> gl, Field<SD> dom, DomGrid g, int Ls, int par,
                                        long Vhb) {
    const long cb = (long)blockIdx.x * (blockDim.x / Ls) + threadIdx.x / Ls;
    const int s = threadIdx.x % Ls;
    const int d = blockIdx.y;
    if (threadIdx.x >= (blockDim.x / Ls) * Ls || cb >= Vhb) return;
    const long gcb = dom_to_global_cb(g, d, cb, par);
    cx<typename SG::real> v[12];
    load_spinor<SG>(gl, gcb * Ls + s, v);
    cx<typename SD::real> w[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) w[c] = {(typename SD::real)v[c].re, (typename SD::real)v[c].im};
    store_spinor<SD>(dom, ((long)d * Vhb + cb) * Ls + s, w);
}

template <class SD, class SG>
__global__ void domain_to_global_kernel(CField<SD> dom, Field<SG> gl, DomGrid g, int Ls, int par,
                                        long Vhb) {
    const long cb = (long)blockIdx.x * (blockDim.x / Ls) + threadIdx.x / Ls;
    const int s = threadIdx.x % Ls;
    const int d = blockIdx.y;
    if (threadIdx.x >= (blockDim.x / Ls) * Ls || cb >= Vhb) return;
    const long gcb = dom_to_global_cb(g, d, cb, par);
    cx<typename SD::real> v[12];
    load_spinor<SD>(dom, ((long)d * Vhb + cb) * Ls + s, v);
    cx<typename SG::real> w[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) w[c] = {(typename SG::real)v[c].re, (typename SG::real)v[c].im};
    store_spinor<SG>(gl, gcb * Ls + s, w);
}

// domain_to_global into an FP64 field z plus the workgroup partials of
// Re<z, r> and Re<z, q> (r, q: FP64 fields of the same layout as z), laid
// out [domain][workgroup] for each of the two sums, np entries apart.
template <class SD>
__global__ void domain_to_global_dots_kernel(CField<SD> dom, Field<F64> gl, CField<F64> r,
                                             CField<F64> q, DomGrid g, int Ls, long Vhb,
                                             double* partials, long np) {
    __shared__ double ra[kThreads], rb[kThreads];
    const long cb = (long)blockIdx.x * (blockDim.x / Ls) + threadIdx.x / Ls;
    const int s = threadIdx.x % Ls;
    const int d = blockIdx.y;
    double a = 0, b = 0;
    if (threadIdx.x < (blockDim.x / Ls) * Ls && cb < Vhb) {
        const long gcb = dom_to_global_cb(g, d, cb, 0);
        cx<typename SD::real> v[12];
        load_spinor<SD>(dom, ((long)d * Vhb + cb) * Ls + s, v);
        cx<double> w[12], rv[12], qv[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) w[c] = {(double)v[c].re, (double)v[c].im};
        store_spinor<F64>(gl, gcb * Ls + s, w);
        load_spinor<F64>(r, gcb * Ls + s, rv);
        load_spinor<F64>(q, gcb * Ls + s, qv);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            a += w[c].re * rv[c].re + w[c].im * rv[c].im;
            b += w[c].re * qv[c].re + w[c].im * qv[c].im;
        }
    }
    // fixed-order tree over the workgroup (blockDim.x need not be a power of 2)
    const int t = threadIdx.x;
    ra[t] = a;
    rb[t] = b;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (t < o && t + o < (int)blockDim.x) {
            ra[t] += ra[t + o];
            rb[t] += rb[t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        const long k = (long)d * gridDim.x + blockIdx.x;
        partials[k] = ra[0];
        partials[np + k] = rb[0];
    }
}

// One thread per (domain, parity, link-box site, direction).
template <class S>
__global__ void pack_links_kernel(const double2* U, typename S::elem* out, DomGrid g, Box lb,
                                  int antiperiodic_t, long V4) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int d = blockIdx.y;
    // consecutive threads take the 8 directions of one site (contiguous output)
    if (i >= 2 * 8 * lb.Vh) return;
    const long ps = i >> 3;
    const int dir = (int)(i & 7);
    const int par = (int)(ps / lb.Vh);
    const long cb = ps - par * lb.Vh;
    int c[4];
    box_coords(lb, cb, par, c);
    int dc[4];
    int r = d;
    for (int m = 0; m < 4; ++m) {
        dc[m] = r % g.nb[m];
        r /= g.nb[m];
    }
    int x[4];
    for (int m = 0; m < 4; ++m) {
        x[m] = dc[m] * g.blk[m] + c[m] + lb.off[m];
        x[m] = ((x[m] % g.L[m]) + g.L[m]) % g.L[m];
    }
    const int mu = dir & 3;
    const bool bwd = dir >= 4;
    double sign = 1.0;
    int y[4] = {x[0], x[1], x[2], x[3]};
    if (bwd) {
        y[mu] -= 1;
        if (y[mu] < 0) {
            y[mu] += g.L[mu];
            if (mu == 3 && antiperiodic_t) sign = -1.0;
        }
    } else if (mu == 3 && antiperiodic_t && x[3] == g.L[3] - 1) {
        sign = -1.0;
    }
    const double2* u = U + ((long)mu * V4 + lex_of(y, g.L)) * 9;
    const long obase = (long)d * (2 * 72 * lb.Vh) + ((long)par * lb.Vh + cb) * 72 + dir * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int row = k / 3, col = k % 3;
        double2 v;
        if (bwd) {  // (U^+)_{row,col} = conj(U_{col,row})
            const double2 t = u[col * 3 + row];
            v = make_double2(sign * t.x, -sign * t.y);
        } else {
            const double2 t = u[k];
            v = make_double2(sign * t.x, sign * t.y);
        }
        typename S::elem e;
        if constexpr (S::has_scale) {
            e = __floats2half2_rn((float)v.x, (float)v.y);
        } else {
            e.x = (typename S::real)v.x;
            e.y = (typename S::real)v.y;
        }
        out[obase + k] = e;
    }
}

template <class SI, class SO>
__global__ void convert_kernel(CField<SI> in, Field<SO> out, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    cx<typename SI::real> v[12];
    load_spinor<SI>(in, i, v);
    cx<typename SO::real> w[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) w[c] = {(typename SO::real)v[c].re, (typename SO::real)v[c].im};
    store_spinor<SO>(out, i, w);
}

inline unsigned nblocks(long n, int t) { return (unsigned)((n + t - 1) / t); }

int last_error() { return hipGetLastError() == hipSuccess ? 0 : -2; }

}  // namespace

template <class S>
int launch_pack_parity(const double2* full, Field<S> out, const int dims[4], int Ls, int par,
                       hipStream_t st) {
    Dims d{{dims[0], dims[1], dims[2], dims[3]}};
    const long V4 = (long)dims[0] * dims[1] * dims[2] * dims[3];
    const long Vh = V4 / 2;
    hipLaunchKernelGGL(pack_parity_kernel<S>, dim3(nblocks(Vh * Ls, kThreads)), dim3(kThreads), 0,
                       st, full, out, d, Ls, par, V4, Vh);
    return last_error();
}

template <class S>
int launch_unpack_parity(CField<S> in, double2* full, const int dims[4], int Ls, int par,
                         int zero_other, hipStream_t st) {
    Dims d{{dims[0], dims[1], dims[2], dims[3]}};
    const long V4 = (long)dims[0] * dims[1] * dims[2] * dims[3];
    const long Vh = V4 / 2;
    hipLaunchKernelGGL(unpack_parity_kernel<S>, dim3(nblocks(Vh * Ls, kThreads)), dim3(kThreads),
                       0, st, in, full, d, Ls, par, zero_other, V4, Vh);
    return last_error();
}

static DomGrid make_grid(const int dims[4], const int blk[4], const int nb[4]) {
    DomGrid g;
    for (int m = 0; m < 4; ++m) {
        g.L[m] = dims[m];
        g.blk[m] = blk[m];
        g.nb[m] = nb[m];
    }
    return g;
}

template <class SG, class SD>
int launch_global_to_domain(CField<SG> gl, Field<SD> dom, const int dims[4], const int blk[4],
                            const int nb[4], int Ls, int par, hipStream_t st) {
    const DomGrid g = make_grid(dims, blk, nb);
    const long Vhb = (long)blk[0] * blk[1] * blk[2] * blk[3] / 2;
    const int spb = kThreads / Ls;
    const int ndom = nb[0] * nb[1] * nb[2] * nb[3];
    hipLaunchKernelGGL((global_to_domain_kernel<SG, SD>), dim3(nblocks(Vhb, spb), ndom),
                       dim3(spb * Ls), 0, st, gl, dom, g, Ls, par, Vhb);
    return last_error();
}

template <class SD, class SG>
int launch_domain_to_global(CField<SD> dom, Field<SG> gl, const int dims[4], const int blk[4],
                            const int nb[4], int Ls, int par, hipStream_t st) {
    const DomGrid g = make_grid(dims, blk, nb);
    const long Vhb = (long)blk[0] * blk[1] * blk[2] * blk[3] / 2;
    const int spb = kThreads / Ls;
    const int ndom = nb[0] * nb[1] * nb[2] * nb[3];
    hipLaunchKernelGGL((domain_to_global_kernel<SD, SG>), dim3(nblocks(Vhb, spb), ndom),
                       dim3(spb * Ls), 0, st, dom, gl, g, Ls, par, Vhb);
    return last_error();
}

template <class SD>
long launch_domain_to_global_dots(CField<SD> dom, Field<F64> gl, CField<F64> r, CField<F64> q,
                                  const int dims[4], const int blk[4], const int nb[4], int Ls,
                                  double* partials, hipStream_t st) {
    const DomGrid g = make_grid(dims, blk, nb);
    const long Vhb = (long)blk[0] * blk[1] * blk[2] * blk[3] / 2;
    const int spb = kThreads / Ls;
    const int ndom = nb[0] * nb[1] * nb[2] * nb[3];
    const long gx = nblocks(Vhb, spb);
    const long np = gx * ndom;
    hipLaunchKernelGGL((domain_to_global_dots_kernel<SD>), dim3((unsigned)gx, ndom),
                       dim3(spb * Ls), 0, st, dom, gl, r, q, g, Ls, Vhb, partials, np);
    return last_error() ? -1 : np;
}

template <class S>
int launch_pack_links(const double2* U, typename S::elem* out, const int dims[4], const int blk[4],
                      const int nb[4], const Box& lb, int antiperiodic_t, hipStream_t st) {
    const DomGrid g = make_grid(dims, blk, nb);
    const long V4 = (long)dims[0] * dims[1] * dims[2] * dims[3];
    const int ndom = nb[0] * nb[1] * nb[2] * nb[3];
    hipLaunchKernelGGL(pack_links_kernel<S>, dim3(nblocks(2 * 8 * lb.Vh, kThreads), ndom),
                       dim3(kThreads), 0, st, U, out, g, lb, antiperiodic_t, V4);
    return last_error();
}

template <class SI, class SO>
int launch_convert(CField<SI> in, Field<SO> out, long n, hipStream_t st) {
    hipLaunchKernelGGL((convert_kernel<SI, SO>), dim3(nblocks(n, kThreads)), dim3(kThreads), 0, st,
                       in, out, n);
    return last_error();
}

#define MSPCG_INST1(S)                                                                             \
    template int launch_pack_parity<S>(const double2*, Field<S>, const int*, int, int,            \
                                       hipStream_t);                                               \
    template int launch_unpack_parity<S>(CField<S>, double2*, const int*, int, int, int,          \
                                         hipStream_t);                                             \
    template int launch_pack_links<S>(const double2*, typename S::elem*, const int*, const int*,  \
                                      const int*, const Box&, int, hipStream_t);
MSPCG_INST1(F64)
MSPCG_INST1(F32)
MSPCG_INST1(F16)
#define MSPCG_INST_DOTS(S)                                                                         \
    template long launch_domain_to_global_dots<S>(CField<S>, Field<F64>, CField<F64>, CField<F64>, \
                                                  const int*, const int*, const int*, int,         \
                                                  double*, hipStream_t);
MSPCG_INST_DOTS(F64)
MSPCG_INST_DOTS(F32)
MSPCG_INST_DOTS(F16)
#define MSPCG_INST2(A, B)                                                                          \
    template int launch_global_to_domain<A, B>(CField<A>, Field<B>, const int*, const int*,       \
                                               const int*, int, int, hipStream_t);                 \
    template int launch_domain_to_global<B, A>(CField<B>, Field<A>, const int*, const int*,       \
                                               const int*, int, int, hipStream_t);                 \
    template int launch_convert<A, B>(CField<A>, Field<B>, long, hipStream_t);                     \
    template int launch_convert<B, A>(CField<B>, Field<A>, long, hipStream_t);
MSPCG_INST2(F64, F16)
MSPCG_INST2(F64, F32)
MSPCG_INST2(F32, F16)
template int launch_global_to_domain<F64, F64>(CField<F64>, Field<F64>, const int*, const int*,
                                               const int*, int, int, hipStream_t);
template int launch_domain_to_global<F64, F64>(CField<F64>, Field<F64>, const int*, const int*,
                                               const int*, int, int, hipStream_t);
template int launch_global_to_domain<F32, F32>(CField<F32>, Field<F32>, const int*, const int*,
                                               const int*, int, int, hipStream_t);
template int launch_domain_to_global<F32, F32>(CField<F32>, Field<F32>, const int*, const int*,
                                               const int*, int, int, hipStream_t);

}  // namespace mspcg
