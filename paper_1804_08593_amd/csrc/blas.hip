// Fifth-dimension-only kernel (optionally with the fused search-direction
// update p = src + beta p), the CG scalar kernels, the remaining FP64 BLAS-1
// passes with fused reductions (residual set-up, flexible-PCG dots, reliable
// updates), and the fixed-order reductions that make every result bitwise
// reproducible (no float atomics).  The per-iteration CG vector updates ride
// on the operator kernels (cg_step, block_cg_step).
#include "common.h"
#include "fived.h"
#include "kernels.h"

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

template <class S, int LS>
__global__ __launch_bounds__(256) void fived_kernel(FiveDArgs<S> a) {
    using T = typename S::real;
    constexpr int SPB = 256 / LS;
    constexpr int SITE_STRIDE = LS * 12 + 1;
    __shared__ cx<T> lds[SPB * SITE_STRIDE];
    if (a.done && *a.done) return;
    const int d = blockIdx.y;
    const int sl = threadIdx.x / LS;
    const int s = threadIdx.x - sl * LS;
    const long cb = (long)blockIdx.x * SPB + sl;
    const bool active = sl < SPB && cb < a.Vh;
    const long ib = ((long)d * a.Vh + cb) * LS;
    cx<T> v[12];
    if (active) {
        load_spinor_at<S>(a.in, ib, s, LS, v);
        if (a.xp_src.data) {
            if (a.zd_z.data) {
                // deferred solution update z (+)= alpha p with the old p
                const T al = (T)a.zd_alpha[d];
                cx<T> zv[12];
                if (a.zd_first) {
#pragma unroll
                    for (int c = 0; c < 12; ++c) zv[c] = {al * v[c].re, al * v[c].im};
                } else {
                    load_spinor_at<S>(cfield(a.zd_z), ib, s, LS, zv);
#pragma unroll
                    for (int c = 0; c < 12; ++c) {
                        zv[c].re += al * v[c].re;
                        zv[c].im += al * v[c].im;
                    }
                }
                store_spinor_at<S>(a.zd_z, ib, s, LS, zv);
            }
            // search-direction update p = src + beta p, written back in place
            const T b = (T)(a.xp_beta ? a.xp_beta[d] : a.xp_sc->beta);
            cx<T> r[12];
            load_spinor_at<S>(a.xp_src, ib, s, LS, r);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                v[c].re = r[c].re + b * v[c].re;
                v[c].im = r[c].im + b * v[c].im;
            }
            store_spinor_at<S>(a.xp_in, ib, s, LS, v);
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) lds[sl * SITE_STRIDE + s * 12 + c] = v[c];
    }
    __syncthreads();
    for (int ch = threadIdx.x; ch < SPB * 12; ch += blockDim.x) {
        const int csl = ch / 12, comp = ch - csl * 12;
        cx<T> w[LS];
#pragma unroll
        for (int t = 0; t < LS; ++t) w[t] = lds[csl * SITE_STRIDE + t * 12 + comp];
        apply_prog<LS, T>(a.p, comp < 6, (T)a.mf, w);
#pragma unroll
        for (int t = 0; t < LS; ++t) lds[csl * SITE_STRIDE + t * 12 + comp] = w[t];
    }
    __syncthreads();
    double n2 = 0;
    if (active) {
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = lds[sl * SITE_STRIDE + s * 12 + c];
        store_spinor_at<S>(a.out, ib, s, LS, v);
        if (a.partials) {
#pragma unroll
            for (int c = 0; c < 12; ++c) n2 += (double)v[c].re * v[c].re + (double)v[c].im * v[c].im;
        }
    }
    if (a.partials) block_reduce_store(n2, a.partials + (long)d * gridDim.x + blockIdx.x);
}

template <class S, int LS>
void fived_launch_ls(const FiveDArgs<S>& a, int ndom, hipStream_t st) {
    constexpr int SPB = 256 / LS;
    hipLaunchKernelGGL((fived_kernel<S, LS>), dim3((unsigned)((a.Vh + SPB - 1) / SPB), ndom),
                       dim3(SPB * LS), 0, st, a);
}

// ---- reductions ----------------------------------------------------------

// One workgroup per output: fixed-order strided sums, then a fixed tree.
__global__ void reduce_rows_kernel(const double* partials, int nparts, double* out) {
    const double* p = partials + (long)blockIdx.x * nparts;
    const double v = strided_sum(p, nparts);
    block_reduce_store(v, out + blockIdx.x);
}

__device__ double block_sum_all(const double* p, int n) {
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

// alpha = rr / <p, A p> (CG) or <z, r> / <p, A p> (flexible PCG)
__global__ void cg_alpha_kernel(DevScalars* sc, const double* partials, int nparts, int flexible) {
    if (sc->done) return;
    const double pq = block_sum_all(partials, nparts);
    if (threadIdx.x == 0) {
        sc->pq = pq;
        if (!(pq > 0.0) || !isfinite(pq)) {
            sc->breakdown = 1;
            sc->done = 1;
            sc->alpha = 0.0;
        } else {
            sc->alpha = (flexible ? sc->zr : sc->rr) / pq;
        }
    }
}

// Flexible (Polak-Ribiere) beta from <z_new, r_new> and <z_new, q>:
// r_old = r_new + alpha q, so <z_new, r_new - r_old> = -alpha <z_new, q>.
__global__ void fpcg_beta_kernel(DevScalars* sc, const double* partials, int nparts, double* hist,
                                 int hist_cap) {
    if (sc->done) return;
    const double zr = block_sum_all(partials, nparts);
    const double zq = block_sum_all(partials + nparts, nparts);
    if (threadIdx.x == 0) {
        sc->beta = sc->zr != 0.0 ? -sc->alpha * zq / sc->zr : 0.0;
        // the flexible beta of the iteration just completed replaces the
        // residual ratio cg_beta_kernel recorded for it
        const int k = sc->iter - 1;
        if (hist && k >= 0 && k < hist_cap) hist[3 * k + 2] = sc->beta;
        sc->zr = zr;
        sc->zq = zq;
        if (!(zr > 0.0) || !isfinite(zr)) {
            sc->breakdown = 1;
            sc->done = 1;
        }
    }
}

__global__ void cg_beta_kernel(DevScalars* sc, const double* partials, int nparts, double* hist,
                               int hist_cap) {
    if (sc->done) return;
    const double rr = block_sum_all(partials, nparts);
    if (threadIdx.x == 0) {
        sc->beta = rr / sc->rr;
        sc->rr = rr;
        const int k = sc->iter;
        // per iteration: |r|^2 and the CG coefficients alpha, beta (their
        // Lanczos tridiagonal estimates the spectrum of A)
        if (hist && k < hist_cap) {
            hist[3 * k] = rr;
            hist[3 * k + 1] = sc->alpha;
            hist[3 * k + 2] = sc->beta;
        }
        sc->iter = k + 1;
        if (!isfinite(rr)) {
            sc->breakdown = 1;
            sc->done = 1;
        } else if (rr <= sc->tol2) {
            sc->done = 1;
        }
    }
}

__global__ void sub_norm_kernel(double2* r, const double2* b, const double2* ax, long n,
                                double* partials) {
    double acc = 0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        const double2 bv = b[i], av = ax[i];
        const double2 rv = make_double2(bv.x - av.x, bv.y - av.y);
        r[i] = rv;
        acc += rv.x * rv.x + rv.y * rv.y;
    }
    block_reduce_store(acc, partials + blockIdx.x);
}

__global__ void copy_norm_kernel(double2* dst, const double2* src, long n, double* partials) {
    double acc = 0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        const double2 v = src[i];
        if (dst) dst[i] = v;
        acc += v.x * v.x + v.y * v.y;
    }
    block_reduce_store(acc, partials + blockIdx.x);
}

// Re<z, r> and Re<z, q> partials: [0..nparts) and [nparts..2 nparts)
__global__ void dot2_kernel(const double2* z, const double2* r, const double2* q, long n,
                            double* partials, long nparts) {
    double a = 0, b = 0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        const double2 zv = z[i], rv = r[i], qv = q[i];
        a += zv.x * rv.x + zv.y * rv.y;
        b += zv.x * qv.x + zv.y * qv.y;
    }
    block_reduce_store(a, partials + blockIdx.x);
    __syncthreads();
    block_reduce_store(b, partials + nparts + blockIdx.x);
}

// x (FP64) += xs (FP32); xs = 0.  Both are site-blocked with 16-byte chunks,
// so FP64 element (site, c, s) at (site*12 + c)*Ls + s pairs with FP32
// element (site*6 + c/2)*2*Ls + 2*s + c%2.
__global__ void accum32_kernel(double2* x, float2* xs, long n, int Ls) {
    const long per_site = 12L * Ls;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        const long site = i / per_site;
        const int r = (int)(i - site * per_site);
        const int c = r / Ls, s = r - c * Ls;
        const long j = site * per_site + (long)(c >> 1) * 2 * Ls + 2 * s + (c & 1);
        const float2 v = xs[j];
        double2 xv = x[i];
        xv.x += (double)v.x;
        xv.y += (double)v.y;
        x[i] = xv;
        xs[j] = make_float2(0.f, 0.f);
    }
}

// y = 0 (a kernel, not a memset node, so it may sit in a captured graph)
__global__ void zero_kernel(double2* y, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        y[i] = make_double2(0.0, 0.0);
}

// x += z, skipped once the solve's `done` flag is set
__global__ void xpy_kernel(double2* x, const double2* z, long n, const int* done) {
    if (done && *done) return;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        const double2 a = x[i], b = z[i];
        x[i] = make_double2(a.x + b.x, a.y + b.y);
    }
}

__global__ void scale_kernel(double2* y, const double2* x, double a, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        const double2 v = x[i];
        y[i] = make_double2(a * v.x, a * v.y);
    }
}

int last_error() { return hipGetLastError() == hipSuccess ? 0 : -2; }

}  // namespace

int launch_xpy(double2* x, const double2* z, long N, const int* done, hipStream_t st) {
    hipLaunchKernelGGL(xpy_kernel, dim3((unsigned)blas_grid_x(12 * N)), dim3(kThreads), 0, st, x,
                       z, 12 * N, done);
    return last_error();
}

int launch_scale(double2* y, const double2* x, double a, long n, hipStream_t st) {
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)blas_grid_x(n)), dim3(kThreads), 0, st, y, x,
                       a, n);
    return last_error();
}

int launch_zero(double2* y, long N, hipStream_t st) {
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blas_grid_x(12 * N)), dim3(kThreads), 0, st, y,
                       12 * N);
    return last_error();
}

int launch_accum32(double2* x, float2* xs, long N, int Ls, hipStream_t st) {
    hipLaunchKernelGGL(accum32_kernel, dim3((unsigned)blas_grid_x(12 * N)), dim3(kThreads), 0, st,
                       x, xs, 12 * N, Ls);
    return last_error();
}

template <class S>
int launch_fived(const FiveDArgs<S>& a, int Ls, int ndom, hipStream_t st) {
    switch (Ls) {
#define MSPCG_CASE(L) \
    case L: fived_launch_ls<S, L>(a, ndom, st); break;
        MSPCG_LS_LIST(MSPCG_CASE)
#undef MSPCG_CASE
        default: return -1;
    }
    return last_error();
}
template int launch_fived<F64>(const FiveDArgs<F64>&, int, int, hipStream_t);
template int launch_fived<F32>(const FiveDArgs<F32>&, int, int, hipStream_t);
template int launch_fived<F16>(const FiveDArgs<F16>&, int, int, hipStream_t);

long fived_grid_x(long Vh, int Ls) {
    const int spb = 256 / Ls;
    return (Vh + spb - 1) / spb;
}

// Vector kernels use a fixed grid so partial counts are known in advance.
long blas_grid_x(long n) {
    long g = (n + kThreads - 1) / kThreads;
    return g < 2048 ? (g < 1 ? 1 : g) : 2048;
}

int launch_reduce_sum(const double* partials, int nparts, double* out, hipStream_t st) {
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(1), dim3(kThreads), 0, st, partials, nparts, out);
    return last_error();
}

int launch_reduce_domains(const double* partials, int ndom, int nparts, double* out,
                          hipStream_t st) {
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(ndom), dim3(kThreads), 0, st, partials, nparts,
                       out);
    return last_error();
}

int launch_cg_alpha(DevScalars* sc, const double* partials, int nparts, hipStream_t st,
                    int flexible) {
    hipLaunchKernelGGL(cg_alpha_kernel, dim3(1), dim3(kThreads), 0, st, sc, partials, nparts,
                       flexible);
    return last_error();
}

int launch_fpcg_beta(DevScalars* sc, const double* partials, int nparts, double* hist,
                     int hist_cap, hipStream_t st) {
    hipLaunchKernelGGL(fpcg_beta_kernel, dim3(1), dim3(kThreads), 0, st, sc, partials, nparts,
                       hist, hist_cap);
    return last_error();
}

int launch_cg_beta(DevScalars* sc, const double* partials, int nparts, double* hist,
                   int hist_cap, hipStream_t st) {
    hipLaunchKernelGGL(cg_beta_kernel, dim3(1), dim3(kThreads), 0, st, sc, partials, nparts, hist,
                       hist_cap);
    return last_error();
}

int launch_sub_norm(double2* r, const double2* b, const double2* ax, long N, double* partials,
                    long nparts, hipStream_t st) {
    hipLaunchKernelGGL(sub_norm_kernel, dim3((unsigned)nparts), dim3(kThreads), 0, st, r, b, ax,
                       12 * N, partials);
    return last_error();
}

int launch_copy_norm(double2* dst, const double2* src, long N, double* partials, long nparts,
                     hipStream_t st) {
    hipLaunchKernelGGL(copy_norm_kernel, dim3((unsigned)nparts), dim3(kThreads), 0, st, dst, src,
                       12 * N, partials);
    return last_error();
}

int launch_dot2(const double2* z, const double2* r, const double2* q, long N, double* partials,
                long nparts, hipStream_t st) {
    hipLaunchKernelGGL(dot2_kernel, dim3((unsigned)nparts), dim3(kThreads), 0, st, z, r, q, 12 * N,
                       partials, nparts);
    return last_error();
}

}  // namespace mspcg
