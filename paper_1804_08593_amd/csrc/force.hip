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
// One thread per (link, direction); the s and spin sums run in the thread.
#include <string.h>

#include "ctx.h"

namespace mspcg {

namespace {

// h = psi_up + sig e_mu psi_dn ; lower = sig e_mu^+ h  (chiral basis, see hop.hip)
template <int SIG>
__device__ __forceinline__ void proj_full(int mu, const cx<double> (&p)[12], cx<double> (&o)[12]) {
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
        o[c] = h0;
        o[3 + c] = h1;
        cx<double> l0, l1;  // e^+ h
        if (mu == 0) {
            l0 = {-h1.im, h1.re};
            l1 = {-h0.im, h0.re};
        } else if (mu == 1) {
            l0 = h1;
            l1 = {-h0.re, -h0.im};
        } else if (mu == 2) {
            l0 = {-h0.im, h0.re};
            l1 = {h1.im, -h1.re};
        } else {
            l0 = h0;
            l1 = h1;
        }
        o[6 + c] = {SIG * l0.re, SIG * l0.im};
        o[9 + c] = {SIG * l1.re, SIG * l1.im};
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

__global__ void force_kernel(ForceArgs a) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 8 * a.Vh) return;
    const int mu = (int)(i % 4);
    const long site = i / 4;
    const int par = (int)(site / a.Vh);
    const long cb = site - par * a.Vh;
    Box lat;
    for (int m = 0; m < 4; ++m) {
        lat.E[m] = a.L[m];
        lat.off[m] = 0;
    }
    lat.Vh = a.Vh;
    int c[4];
    box_coords(lat, cb, par, c);
    int n[4] = {c[0], c[1], c[2], c[3]};
    n[mu] = (n[mu] + 1) % a.L[mu];
    const long ncb = box_cb(lat, n);
    const int npar = 1 - par;
    cx<double> P[9], Q[9];
    for (int k = 0; k < 9; ++k) P[k] = Q[k] = {0, 0};
    for (int s = 0; s < a.Ls; ++s) {
        cx<double> ax[12], bx[12], by[12], ay[12], pb[12], pa[12];
        load_spinor<F64>(a.a[par], cb * a.Ls + s, ax);
        load_spinor<F64>(a.b[par], cb * a.Ls + s, bx);
        load_spinor<F64>(a.b[npar], ncb * a.Ls + s, by);
        load_spinor<F64>(a.a[npar], ncb * a.Ls + s, ay);
        proj_full<-1>(mu, by, pb);  // (1 - g) b(x+mu)
        proj_full<+1>(mu, ay, pa);  // (1 + g) a(x+mu)
        for (int sp = 0; sp < 4; ++sp)
            for (int r = 0; r < 3; ++r)
                for (int q = 0; q < 3; ++q) {
                    // P_rq += pb_r conj(ax_q) ; Q_rq += bx_r conj(pa_q)
                    const cx<double> x1 = pb[sp * 3 + r], y1 = ax[sp * 3 + q];
                    P[r * 3 + q].re += x1.re * y1.re + x1.im * y1.im;
                    P[r * 3 + q].im += x1.im * y1.re - x1.re * y1.im;
                    const cx<double> x2 = bx[sp * 3 + r], y2 = pa[sp * 3 + q];
                    Q[r * 3 + q].re += x2.re * y2.re + x2.im * y2.im;
                    Q[r * 3 + q].im += x2.im * y2.re - x2.re * y2.im;
                }
    }
    // eta U_mu(x): forward link of this site (sign folded in)
    cx<double> U[9];
    for (int k = 0; k < 9; ++k) {
        const double2 t = a.links[(((long)par * a.Vh + cb) * 8 + mu) * 9 + k];
        U[k] = {t.x, t.y};
    }
    const long lex = (((long)c[3] * a.L[2] + c[2]) * a.L[1] + c[1]) * a.L[0] + c[0];
    const long V4 = 2 * a.Vh;
    if (a.F) {
        // G = (eta U) P - Q (eta U)^+ = eta (U P - Q U^+)
        cx<double> G[9];
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) {
                cx<double> g = {0, 0};
                for (int k = 0; k < 3; ++k) {
                    cfma(g, U[r * 3 + k], P[k * 3 + q]);
                    const cx<double> uc = {U[q * 3 + k].re, -U[q * 3 + k].im};  // (U^+)_{kq}
                    const cx<double> t = cmul(Q[r * 3 + k], uc);
                    g.re -= t.re;
                    g.im -= t.im;
                }
                G[r * 3 + q] = g;
            }
        cx<double> Fm[9];
        double tr = 0;
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) {
                // (G - G^+)/(2i) : (x - conj(y)) / (2i) with x = G_rq, y = G_qr
                const cx<double> x = G[r * 3 + q], y = G[q * 3 + r];
                const double dre = x.re - y.re, dim = x.im + y.im;
                Fm[r * 3 + q] = {0.5 * dim, -0.5 * dre};
                if (r == q) tr += Fm[r * 3 + q].re;
            }
        for (int r = 0; r < 3; ++r) Fm[r * 4].re -= tr / 3.0;
        double2* out = a.F + ((long)mu * V4 + lex) * 9;
        for (int k = 0; k < 9; ++k) out[k] = make_double2(Fm[k].re, Fm[k].im);
    }
    if (a.grad) {
        // g = -eta (P^+ + Q), eta = -1 only for the time link that wraps
        const double eta = (mu == 3 && c[3] == a.L[3] - 1 && a.antiperiodic_t) ? -1.0 : 1.0;
        double2* out = a.grad + ((long)mu * V4 + lex) * 9;
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) {
                const cx<double> pc = P[q * 3 + r];  // (P^+)_{rq} = conj(P_qr)
                out[r * 3 + q] = make_double2(-eta * (pc.re + Q[r * 3 + q].re),
                                              -eta * (-pc.im + Q[r * 3 + q].im));
            }
    }
}

}  // namespace

}  // namespace mspcg

using namespace mspcg;

extern "C" int mspcg_force(mspcg_ctx* c, const void* X_dev, const void* Y_dev, void* F_dev,
                           void* G_dev, hipStream_t st) {
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
    const long n = 8 * c->Vh;
    hipLaunchKernelGGL(force_kernel, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, a);
    if (hipGetLastError() != hipSuccess) return MSPCG_EHIP;
    MSPCG_HIP(hipStreamSynchronize(st));
    return MSPCG_OK;
}
