// HMC fermion force of S = phi^+ A^-1 phi, A = Mhat^+ Mhat (FP64).
//
// With X = A^-1 phi and Y = Mhat X, only the hopping term depends on the
// links, and dS = -Re[a^+ dD_h b] with the 5D fields
//   a = (Y on even sites,  W = M5op^-+ M_eo^+ Y = -(1/2) X^+ Dd^oe Y on odd),
//   b = (B X on even,      B M5op^-1 M_oe X = -(1/2) X D_h^oe B X on odd),
// (X = B M5op^-1 as a 5D operator, Dd = dagger hop).  For the link U_mu(x):
//   P = sum_{s,spin} [(1 - g_mu) b(x+mu)] a(x)^+ ,  Q = sum_{s,spin} b(x) [(1 + g_mu) a(x+mu)]^+
//   dS/deps = tr(T F) for U -> exp(i eps T) U, F = eta * TA[(G - G^+)/(2i)], G = U P - Q U^+
//   (TA: traceless part), and the gradient with respect to the unconstrained
//   complex link (dS = Re sum conj(g) dU) is g = -eta (P^+ + Q).
// eta (the antiperiodic-time sign) is already folded into the stored links.
// (1 -+ g_mu) = W W^+ with W = [1; -+e_mu^+] (chiral basis), so every spin
// sum above contracts two half spinors: P = sum_s h-(b(x+mu)) h-(a(x))^+ and
// Q = sum_s h+(b(x)) h+(a(x+mu))^+ with h_sig(psi) = psi_up + sig e_mu psi_dn
// (two spin rows of three colours each).
// A workgroup of one wave takes 64/Ls sites, one lane per (site, s).  For P,
// every lane keeps its a(x) in registers and, per direction, loads b(x+mu)
// and forms its slice's 3x3 partial; neighbouring slices are added across
// lanes, the pair sums go through LDS and are summed over s in a fixed order
// by one lane per (site, entry).  Q the same way with b(x) kept.  Then one
// lane per (site, direction, entry) writes that entry of F and of the
// gradient.  Spinor loads are 16-byte chunks of consecutive s, as in the hop,
// and each field is read once per direction that needs it.
#include <string.h>

#include "ctx.h"

namespace mspcg {

namespace {

// h = psi_up + SIG e_mu psi_dn (chiral basis, as project() in hop_impl.h): the two spin rows
// that (1 + SIG g_mu) keeps
template <int SIG>
__device__ __forceinline__ void proj_half(int mu, const cx<double> (&p)[12], cx<double> (&h)[6]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cx<double> u0 = p[c], u1 = p[3 + c], d0 = p[6 + c], d1 = p[9 + c];
        cx<double> h0, h1;
        if (mu == 0) {
            h0 = {u0.re + SIG * d1.im, u0.im - SIG * d1.re};
            h1 = {u1.re + SIG * d0.im, u1.im - SIG * d0.re};
        } else if (mu == 1) {
            h0 = {u0.re - SIG * d1.re, u0.im - SIG * d1.im};
            h1 = {u1.re + SIG * d0.re, u1.im + SIG * d0.im};
        } else if (mu == 2) {
            h0 = {u0.re + SIG * d0.im, u0.im - SIG * d0.re};
            h1 = {u1.re - SIG * d1.im, u1.im + SIG * d1.re};
        } else {
            h0 = {u0.re + SIG * d0.re, u0.im + SIG * d0.im};
            h1 = {u1.re + SIG * d1.re, u1.im + SIG * d1.im};
        }
        h[c] = h0;
        h[3 + c] = h1;
    }
}

// o_rq = sum_i x[i][r] conj(y[i][q]) over the two spin rows
__device__ __forceinline__ void outer_half(const cx<double> (&x)[6], const cx<double> (&y)[6],
                                           double (&o)[18]) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            double re = 0, im = 0;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const cx<double> u = x[3 * i + r], v = y[3 * i + q];
                re = fma(u.re, v.re, fma(u.im, v.im, re));
                im = fma(u.im, v.re, fma(-u.re, v.im, im));
            }
            o[2 * (3 * r + q)] = re;
            o[2 * (3 * r + q) + 1] = im;
        }
}

struct ForceArgs {
    CField<F64> a[2];  // by parity
    CField<F64> b[2];
    const double2* links;  // whole-lattice [par][Vh][8][9], forward dirs 0..3
    int L[4];
    int Ls;
    long Vh;
    int antiperiodic_t;
    double2* F;     // [4][lex][3][3] or null
    double2* grad;  // [4][lex][3][3] or null
};

constexpr int FPS = 19;  // LDS row of one lane's partial: 9 complex + 1 pad

// site index (both parities: par * Vh + cb) -> parity, cb and coordinates
__device__ __forceinline__ void site_at(const ForceArgs& a, long site, int& par, long& cb,
                                        int c[4]) {
    Box lat;
    for (int m = 0; m < 4; ++m) {
        lat.E[m] = a.L[m];
        lat.off[m] = 0;
    }
    lat.Vh = a.Vh;
    par = (int)(site / a.Vh);
    cb = site - par * a.Vh;
    box_coords(lat, cb, par, c);
}

__device__ __forceinline__ long forward_cb(const ForceArgs& a, const int c[4], int mu) {
    Box lat;
    for (int m = 0; m < 4; ++m) {
        lat.E[m] = a.L[m];
        lat.off[m] = 0;
    }
    lat.Vh = a.Vh;
    int n[4] = {c[0], c[1], c[2], c[3]};
    n[mu] = n[mu] + 1 == a.L[mu] ? 0 : n[mu] + 1;
    return box_cb(lat, n);
}

// value of the neighbouring lane (lane ^ 1): DPP quad_perm [1,0,3,2] on both
// halves of the double
__device__ __forceinline__ double swap_pair(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// workgroup -> range of sites: the hardware deals workgroups to the eight
// XCDs in turn, so workgroup b is given position (b mod 8) * G/8 + b/8 (with
// the remainder spread over the first XCDs); each XCD then walks one
// contiguous range of sites and finds most neighbours in its own L2
__device__ __forceinline__ long xcd_block() {
    const unsigned G = gridDim.x, lid = blockIdx.x;
    const unsigned q = G >> 3, r = G & 7, k = lid & 7;
    return (long)(k * q + (k < r ? k : r) + (lid >> 3));
}

// one lane per (site, entry (r, q)) of direction mu: F and the gradient
__device__ __forceinline__ void force_out(const ForceArgs& a, long st, int mu, int e,
                                          const double2* P, const double2* Q) {
    int p2, c2[4];
    long cb2;
    site_at(a, st, p2, cb2, c2);
    const long V4 = 2 * a.Vh;
    const long lex = (((long)c2[3] * a.L[2] + c2[2]) * a.L[1] + c2[1]) * a.L[0] + c2[0];
    const int r = e / 3, q = e - 3 * (e / 3);
    const double2* U = a.links + st * 72 + 9 * mu;  // eta U_mu(x)
    if (a.F) {
        // G = (eta U) P - Q (eta U)^+ at (r, q) and (q, r); F = TA[(G - G^+)/(2i)]
        cx<double> g[2];
#pragma unroll
        for (int z = 0; z < 2; ++z) {
            const int rr = z ? q : r, qq = z ? r : q;
            cx<double> acc = {0, 0};
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double2 u1 = U[3 * rr + j], p1 = P[3 * j + qq];
                const double2 q1 = Q[3 * rr + j], u2 = U[3 * qq + j];
                acc.re += u1.x * p1.x - u1.y * p1.y - (q1.x * u2.x + q1.y * u2.y);
                acc.im += u1.x * p1.y + u1.y * p1.x - (q1.y * u2.x - q1.x * u2.y);
            }
            g[z] = acc;
        }
        cx<double> f = {0.5 * (g[0].im + g[1].im), -0.5 * (g[0].re - g[1].re)};
        if (r == q) {
            // trace of (G - G^+)/(2i) = sum_d Im G_dd
            double tr = 0;
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const double2 u1 = U[3 * d + j], p1 = P[3 * j + d];
                    const double2 q1 = Q[3 * d + j];
                    tr += u1.x * p1.y + u1.y * p1.x - (q1.y * u1.x - q1.x * u1.y);
                }
            f.re -= tr / 3.0;
        }
        a.F[((long)mu * V4 + lex) * 9 + e] = make_double2(f.re, f.im);
    }
    if (a.grad) {
        // g = -eta (P^+ + Q), eta = -1 only for the time link that wraps
        const double eta = (mu == 3 && c2[3] == a.L[3] - 1 && a.antiperiodic_t) ? -1.0 : 1.0;
        const double2 pc = P[3 * q + r];  // (P^+)_{rq} = conj(P_qr)
        const double2 qv = Q[e];
        a.grad[((long)mu * V4 + lex) * 9 + e] =
            make_double2(-eta * (pc.x + qv.x), -eta * (-pc.y + qv.y));
    }
}

constexpr int FORCE_THREADS = 64;  // one wave per workgroup: its barriers cost no waiting

// 3 waves per SIMD (at most 168 VGPRs; the LDS of a workgroup allows 15)
template <int LS>
__global__ __launch_bounds__(FORCE_THREADS, 3) void force_kernel(ForceArgs a) {
    // sites per workgroup, one lane per (site, s); Ls is even, so lanes s and
    // s ^ 1 belong to the same site
    constexpr int SPB = FORCE_THREADS / LS;
    constexpr int R = LS / 2;  // partials per site after the pair sum
    __shared__ double part[SPB * R][FPS];
    __shared__ double2 sum[SPB][72];  // [P, Q][mu][3x3], summed over s
    const int t = threadIdx.x;
    const int sl = t / LS;
    const int s = t - sl * LS;
    const long site0 = xcd_block() * SPB;
    const long nsite = 2 * a.Vh;
    const bool act = sl < SPB && site0 + sl < nsite;
    int par = 0, c[4] = {0, 0, 0, 0};
    long cb = 0;
    if (act) site_at(a, site0 + sl, par, cb, c);
    // w = 0: P_mu = sum h-(b(x+mu)) h-(a(x))^+ ; w = 1: Q_mu = sum h+(b(x)) h+(a(x+mu))^+.
    // The site's own spinor (a(x), then b(x)) stays in registers for the four
    // directions; only the neighbour is loaded per direction.
#pragma unroll 1
    for (int w = 0; w < 2; ++w) {
        cx<double> own[12];
        if (act) load_spinor_at<F64>(w == 0 ? a.a[par] : a.b[par], cb * LS, s, LS, own);
#pragma unroll 1
        for (int mu = 0; mu < 4; ++mu) {
            if (act) {
                const long ncb = forward_cb(a, c, mu);
                cx<double> nb[12], hu[6], hv[6];
                load_spinor_at<F64>(w == 0 ? a.b[1 - par] : a.a[1 - par], ncb * LS, s, LS, nb);
                if (w == 0) {
                    proj_half<-1>(mu, nb, hu);
                    proj_half<-1>(mu, own, hv);
                } else {
                    proj_half<+1>(mu, own, hu);
                    proj_half<+1>(mu, nb, hv);
                }
                double o[18];
                outer_half(hu, hv, o);
#pragma unroll
                for (int k = 0; k < 18; ++k) o[k] += swap_pair(o[k]);  // slices s and s ^ 1
                if (!(s & 1))
#pragma unroll
                    for (int k = 0; k < 18; ++k) part[t >> 1][k] = o[k];
            }
            __syncthreads();
            for (int k = t; k < SPB * 9; k += FORCE_THREADS) {
                const int q = k / 9, e = k - 9 * q;
                double re = 0, im = 0;
                if (site0 + q < nsite)
                    for (int j = 0; j < R; ++j) {
                        re += part[q * R + j][2 * e];
                        im += part[q * R + j][2 * e + 1];
                    }
                sum[q][(4 * w + mu) * 9 + e] = make_double2(re, im);
            }
            __syncthreads();
        }
    }
    for (int k = t; k < SPB * 36; k += FORCE_THREADS) {
        const int q = k / 36, mu = (k - 36 * q) / 9, e = k - 36 * q - 9 * mu;
        if (site0 + q < nsite) force_out(a, site0 + q, mu, e, sum[q] + 9 * mu, sum[q] + 36 + 9 * mu);
    }
}

}  // namespace

}  // namespace mspcg

using namespace mspcg;

extern "C" int mspcg_force(mspcg_ctx* c, const void* X_dev, const void* Y_dev, void* F_dev,
                           void* G_dev, hipStream_t st) try {
    if (!c || !X_dev || !Y_dev || (!F_dev && !G_dev)) return MSPCG_EINVAL;
    if (!c->gauge) return MSPCG_ENOGAUGE;
    MSPCG_HIP(hipSetDevice(c->device));
    Field<F64> xe = half_field<F64>(c, "d.fo_x", c->Nh);
    Field<F64> ye = half_field<F64>(c, "d.fo_y", c->Nh);
    Field<F64> be = half_field<F64>(c, "d.fo_be", c->Nh);
    Field<F64> bo = half_field<F64>(c, "d.fo_bo", c->Nh);
    Field<F64> ao = half_field<F64>(c, "d.fo_ao", c->Nh);
    if (!xe.data || !ye.data || !be.data || !bo.data || !ao.data) return MSPCG_ENOMEM;
    if (launch_pack_parity<F64>((const double2*)X_dev, xe, c->L, c->Ls, 0, st)) return MSPCG_EHIP;
    if (launch_pack_parity<F64>((const double2*)Y_dev, ye, c->L, c->Ls, 0, st)) return MSPCG_EHIP;
    const Progs& P = c->pr;
    int e;
    // b = (B X, -(1/2) X D_h^oe B X) ; a = (Y, -(1/2) X^+ Dd^oe Y)
    if ((e = op_fived<F64>(c, be, cfield(xe), P.B, nullptr, nullptr, st))) return e;
    if ((e = op_hop<F64>(c, bo, cfield(be), 1, false, scaled(P.X, -0.5, -0.5), nullptr, P.id,
                         nullptr, nullptr, st)))
        return e;
    if ((e = op_hop<F64>(c, ao, cfield(ye), 1, true, scaled(P.Xdag, -0.5, -0.5), nullptr, P.id,
                         nullptr, nullptr, st)))
        return e;
    ForceArgs a;
    a.a[0] = cfield(ye);
    a.a[1] = cfield(ao);
    a.b[0] = cfield(be);
    a.b[1] = cfield(bo);
    a.links = c->L64;
    for (int m = 0; m < 4; ++m) a.L[m] = c->L[m];
    a.Ls = c->Ls;
    a.Vh = c->Vh;
    a.antiperiodic_t = c->act.antiperiodic_t;
    a.F = (double2*)F_dev;
    a.grad = (double2*)G_dev;
    const long nsites = 2 * c->Vh;
    switch (c->Ls) {
#define MSPCG_CASE(L)                                                                      \
    case L: {                                                                              \
        constexpr int spb = FORCE_THREADS / L;                                             \
        hipLaunchKernelGGL(force_kernel<L>, dim3((unsigned)((nsites + spb - 1) / spb)),     \
                           dim3(FORCE_THREADS), 0, st, a);                                 \
        break;                                                                             \
    }
        MSPCG_LS_LIST(MSPCG_CASE)
#undef MSPCG_CASE
        default: return MSPCG_EUNSUPPORTED;
    }
    if (hipGetLastError() != hipSuccess) return MSPCG_EHIP;
    MSPCG_HIP(hipStreamSynchronize(st));
    return MSPCG_OK;
}
MSPCG_ABI_CATCH
