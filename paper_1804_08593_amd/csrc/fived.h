// Fifth-dimension (s-direction) operators applied to the s-vector of one
// (site, spin-colour component).
//
// Every 5D-local operator of the even-odd Moebius operator is a polynomial or
// rational function of the fifth-dimension hop K (and of K^+):
//   (K psi)_s   = P- psi_{s+1} + P+ psi_{s-1},   psi_{Ls} = -mf psi_0, psi_{-1} = -mf psi_{Ls-1}
//   (K^+ psi)_s = P- psi_{s-1} + P+ psi_{s+1}   (same -mf corners),
// P+ = spins 0,1 (upper chirality), P- = spins 2,3.  On one chirality K is a
// cyclic shift with a -mf corner, so
//   BIDI(a): (1 + a K) is bidiagonal with a corner, and
//   INV(q):  (1 - q K)^-1 is solved exactly in O(Ls) from K^Ls = -mf:
//            the far end is y_end = sum_k q^k x_{end-k} / (1 + mf q^Ls), then a
//            first-order recursion runs along s.
// This replaces the dense Ls x Ls product (48 Ls flop per (x,s)) by ~8 flop.
#pragma once
#include "common.h"

namespace mspcg {

// Apply program P to v[0..LS) of one component of chirality `up` (true: spins 0,1).
template <int LS, typename T>
__device__ __forceinline__ void apply_prog(const FiveDProg& P, bool up, T mf, cx<T> (&v)[LS]) {
    for (int k = 0; k < P.nsteps; ++k) {
        // K on the upper chirality and K^+ on the lower one take psi_{s-1}
        const bool from_below = (up != (P.dag[k] != 0));
        const T a = (T)P.a[k];
        if (P.kind[k] == STEP_BIDI) {
            if (from_below) {
                const cx<T> last = v[LS - 1];
#pragma unroll
                for (int s = LS - 1; s >= 1; --s) {
                    v[s].re += a * v[s - 1].re;
                    v[s].im += a * v[s - 1].im;
                }
                v[0].re -= a * mf * last.re;
                v[0].im -= a * mf * last.im;
            } else {
                const cx<T> first = v[0];
#pragma unroll
                for (int s = 0; s < LS - 1; ++s) {
                    v[s].re += a * v[s + 1].re;
                    v[s].im += a * v[s + 1].im;
                }
                v[LS - 1].re -= a * mf * first.re;
                v[LS - 1].im -= a * mf * first.im;
            }
        } else if (P.kind[k] == STEP_INV) {
            const T q = a;
            T qL = 1;
#pragma unroll
            for (int s = 0; s < LS; ++s) qL *= q;
            const T norm = T(1) / (T(1) + mf * qL);
            if (from_below) {
                // y_s - q y_{s-1} = x_s (s >= 1), y_0 + q mf y_{LS-1} = x_0
                cx<T> acc = v[0];
#pragma unroll
                for (int s = 1; s < LS; ++s) {
                    acc.re = q * acc.re + v[s].re;
                    acc.im = q * acc.im + v[s].im;
                }
                const cx<T> yend = {acc.re * norm, acc.im * norm};
                v[0].re -= q * mf * yend.re;
                v[0].im -= q * mf * yend.im;
#pragma unroll
                for (int s = 1; s < LS; ++s) {
                    v[s].re += q * v[s - 1].re;
                    v[s].im += q * v[s - 1].im;
                }
            } else {
                cx<T> acc = v[LS - 1];
#pragma unroll
                for (int s = LS - 2; s >= 0; --s) {
                    acc.re = q * acc.re + v[s].re;
                    acc.im = q * acc.im + v[s].im;
                }
                const cx<T> yend = {acc.re * norm, acc.im * norm};
                v[LS - 1].re -= q * mf * yend.re;
                v[LS - 1].im -= q * mf * yend.im;
#pragma unroll
                for (int s = LS - 2; s >= 0; --s) {
                    v[s].re += q * v[s + 1].re;
                    v[s].im += q * v[s + 1].im;
                }
            }
        }
    }
    const T sc = (T)(up ? P.scale[0] : P.scale[1]);
#pragma unroll
    for (int s = 0; s < LS; ++s) {
        v[s].re *= sc;
        v[s].im *= sc;
    }
}

}  // namespace mspcg
