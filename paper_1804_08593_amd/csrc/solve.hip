// Solvers on the even-odd normal equations A x_e = bhat, A = Mhat^+ Mhat
// (Sec. 2.2, eq. (3)), and the odd-site reconstruction.
//
//   CG        plain FP64 conjugate gradient (the baseline of Sec. 3)
//   MIXED_CG  FP32 iterations with FP64 solution accumulation and reliable
//             updates of the true FP64 residual
//   MSPCG     flexible FP64 outer PCG preconditioned by the block-diagonal
//             K = (+)_s A_s, applied as l local CG iterations from a zero
//             guess in lower precision (Sec. 2.3, eqs. (4)-(5))
//
// Scalars stay on the device (DevScalars); every kernel of an iteration
// returns immediately once the iterated residual has reached the tolerance,
// so the host polls only every `check_every` iterations.  The stop test is
// always re-done on the true residual bhat - A x in FP64.
#include <math.h>
#include <string.h>

#include <chrono>

#include "ctx.h"

namespace mspcg {

namespace {

struct HostPoll {
    DevScalars s;
};

int poll(mspcg_ctx* c, hipStream_t st, DevScalars& out) {
    MSPCG_HIP(hipMemcpyAsync(c->sc_host, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
    MSPCG_HIP(hipStreamSynchronize(st));
    out = *c->sc_host;
    return 0;
}

int push(mspcg_ctx* c, hipStream_t st, const DevScalars& in) {
    *c->sc_host = in;
    MSPCG_HIP(hipMemcpyAsync(c->sc, c->sc_host, sizeof(DevScalars), hipMemcpyHostToDevice, st));
    MSPCG_HIP(hipStreamSynchronize(st));
    return 0;
}

// |v|^2 of an FP64 half field, synchronously.
int norm2_sync(mspcg_ctx* c, const double2* v, double2* copy_to, hipStream_t st, double& out) {
    const long np = blas_grid_x(12 * c->Nh);
    int e = ensure_partials(c, 4 * np + 16);
    if (e) return e;
    double* res = c->partials + 4 * np;
    if (launch_copy_norm(copy_to, v, c->Nh, c->partials, np, st)) return MSPCG_EHIP;
    if (launch_reduce_sum(c->partials, (int)np, res, st)) return MSPCG_EHIP;
    MSPCG_HIP(hipMemcpyAsync(&c->sc_host->pq, res, sizeof(double), hipMemcpyDeviceToHost, st));
    MSPCG_HIP(hipStreamSynchronize(st));
    out = c->sc_host->pq;
    return 0;
}

// r = bhat - A x, returns |r|^2
int true_residual(mspcg_ctx* c, Field<F64> r, CField<F64> bhat, CField<F64> x, hipStream_t st,
                  double& rr) {
    Field<F64> ax = half_field<F64>(c, "d.tr_ax", c->Nh);
    if (!ax.data) return MSPCG_ENOMEM;
    int e = op_A<F64>(c, ax, x, nullptr, nullptr, st);
    if (e) return e;
    const long np = blas_grid_x(12 * c->Nh);
    if ((e = ensure_partials(c, 4 * np + 16))) return e;
    double* res = c->partials + 4 * np;
    if (launch_sub_norm(r.data, bhat.data, ax.data, c->Nh, c->partials, np, st)) return MSPCG_EHIP;
    if (launch_reduce_sum(c->partials, (int)np, res, st)) return MSPCG_EHIP;
    MSPCG_HIP(hipMemcpyAsync(&c->sc_host->pq, res, sizeof(double), hipMemcpyDeviceToHost, st));
    MSPCG_HIP(hipStreamSynchronize(st));
    rr = c->sc_host->pq;
    return 0;
}

int ensure_hist(mspcg_ctx* c, int cap) {
    if (cap <= c->hist_cap) return 0;
    if (c->hist) (void)hipFree(c->hist);
    c->hist = nullptr;
    c->hist_cap = 0;
    if (hipMalloc(&c->hist, (size_t)cap * sizeof(double)) != hipSuccess) return MSPCG_ENOMEM;
    c->hist_cap = cap;
    return 0;
}

// Plain FP64 CG on A x = bhat.  x holds the initial guess (or zero).
int cg_fp64(mspcg_ctx* c, CField<F64> bhat, Field<F64> x, bool x0, const mspcg_solve_params* p,
            double bb, mspcg_solve_stats* stats, hipStream_t st) {
    Field<F64> r = half_field<F64>(c, "d.cg_r", c->Nh);
    Field<F64> pp = half_field<F64>(c, "d.cg_p", c->Nh);
    Field<F64> q = half_field<F64>(c, "d.cg_q", c->Nh);
    if (!r.data || !pp.data || !q.data) return MSPCG_ENOMEM;
    const long nph = hop_nparts(c);
    const long npb = blas_grid_x(12 * c->Nh);
    int e;
    if ((e = ensure_partials(c, 4 * (nph > npb ? nph : npb) + 16))) return e;
    const int cap = p->maxiter + 1;
    if ((e = ensure_hist(c, cap))) return e;
    double rr;
    if (x0) {
        if ((e = true_residual(c, r, bhat, cfield(x), st, rr))) return e;
    } else {
        MSPCG_HIP(hipMemsetAsync(x.data, 0, (size_t)12 * c->Nh * sizeof(double2), st));
        if ((e = norm2_sync(c, bhat.data, r.data, st, rr))) return e;
    }
    MSPCG_HIP(hipMemcpyAsync(pp.data, r.data, (size_t)12 * c->Nh * sizeof(double2),
                             hipMemcpyDeviceToDevice, st));
    DevScalars s;
    memset(&s, 0, sizeof(s));
    s.rr = rr;
    s.bb = bb;
    s.tol2 = p->tol * p->tol * bb;
    s.done = rr <= s.tol2 ? 1 : 0;
    if ((e = push(c, st, s))) return e;
    int check = p->check_every > 0 ? p->check_every : 8;
    int restarts = 0;
    bool converged = false;
    double true_rr = rr;
    int iters = 0;
    while (true) {
        if (!s.done) {
            for (int k = 0; k < check && iters + k < p->maxiter; ++k) {
                if ((e = op_A<F64>(c, q, cfield(pp), c->partials, &c->sc->done, st))) return e;
                if (launch_cg_alpha(c->sc, c->partials, (int)nph, st)) return MSPCG_EHIP;
                if (launch_cg_update_xr(x.data, r.data, pp.data, q.data, c->Nh, c->sc, c->partials,
                                        npb, st))
                    return MSPCG_EHIP;
                if (launch_cg_beta(c->sc, c->partials, (int)npb, c->hist, cap, st)) return MSPCG_EHIP;
                if (launch_xpay(pp.data, r.data, c->Nh, c->sc, 0, st)) return MSPCG_EHIP;
            }
            if ((e = poll(c, st, s))) return e;
        }
        iters = s.iter;
        if (s.breakdown) {
            if (stats) stats->outer_iters = iters;
            return MSPCG_EBREAKDOWN;
        }
        if (s.done) {
            if ((e = true_residual(c, r, bhat, cfield(x), st, true_rr))) return e;
            if (true_rr <= s.tol2) {
                converged = true;
                break;
            }
            // continue from the true residual: the step that set `done` skipped
            // p = r + beta p, so redo it with beta = |r_true|^2 / |r_prev|^2
            restarts++;
            s.beta = s.beta * true_rr / s.rr;
            s.rr = true_rr;
            s.done = 0;
            if ((e = push(c, st, s))) return e;
            if (launch_xpay(pp.data, r.data, c->Nh, c->sc, 0, st)) return MSPCG_EHIP;
        }
        if (iters >= p->maxiter) {
            if ((e = true_residual(c, r, bhat, cfield(x), st, true_rr))) return e;
            break;
        }
    }
    if (stats) {
        stats->outer_iters = iters;
        stats->inner_iters_total = 0;
        stats->restarts = restarts;
        stats->converged = converged ? 1 : 0;
        stats->true_rel_resid = sqrt(true_rr / bb);
        if (stats->resid_history && stats->resid_history_cap > 0) {
            const int n = iters < stats->resid_history_cap ? iters : stats->resid_history_cap;
            std::vector<double> h(n > 0 ? n : 1);
            if (n > 0) {
                MSPCG_HIP(hipMemcpy(h.data(), c->hist, n * sizeof(double), hipMemcpyDeviceToHost));
                for (int i = 0; i < n; ++i) stats->resid_history[i] = sqrt(h[i] / bb);
            }
            stats->resid_history_len = n;
        }
    }
    return converged ? MSPCG_OK : MSPCG_ENOCONV;
}

void fill_stats(mspcg_ctx* c, mspcg_solve_stats* stats, int iters, int inner, int restarts,
                bool converged, double true_rr, double bb, const double* hist_dev) {
    if (!stats) return;
    stats->outer_iters = iters;
    stats->inner_iters_total = inner;
    stats->restarts = restarts;
    stats->converged = converged ? 1 : 0;
    stats->true_rel_resid = sqrt(true_rr / bb);
    stats->resid_history_len = 0;
    if (stats->resid_history && stats->resid_history_cap > 0 && hist_dev) {
        const int n = iters < stats->resid_history_cap ? iters : stats->resid_history_cap;
        if (n > 0) {
            std::vector<double> h(n);
            if (hipMemcpy(h.data(), hist_dev, n * sizeof(double), hipMemcpyDeviceToHost) ==
                hipSuccess) {
                for (int i = 0; i < n; ++i) stats->resid_history[i] = sqrt(h[i] / bb);
                stats->resid_history_len = n;
            }
        }
    }
}

// Flexible preconditioned CG (FP64) with z = K_l^-1 r in storage precision S.
template <class S>
int mspcg_fp64(mspcg_ctx* c, CField<F64> bhat, Field<F64> x, bool x0,
               const mspcg_solve_params* p, double bb, mspcg_solve_stats* stats, hipStream_t st) {
    Field<F64> r = half_field<F64>(c, "d.cg_r", c->Nh);
    Field<F64> pp = half_field<F64>(c, "d.cg_p", c->Nh);
    Field<F64> q = half_field<F64>(c, "d.cg_q", c->Nh);
    Field<F64> z = half_field<F64>(c, "d.cg_z", c->Nh);
    if (!r.data || !pp.data || !q.data || !z.data) return MSPCG_ENOMEM;
    int e;
    if ((e = domains_setup(c, p->blocking, p->inner_prec, st))) return e;
    const long nph = hop_nparts(c);
    const long npb = blas_grid_x(12 * c->Nh);
    size_t need = 4 * (size_t)(nph > npb ? nph : npb) + 16;
    const size_t pneed = precond_partials_need(c);
    if (pneed > need) need = pneed;
    if ((e = ensure_partials(c, need))) return e;
    const int cap = p->maxiter + 1;
    if ((e = ensure_hist(c, cap))) return e;
    const int l = p->inner_iters;
    double rr;
    if (x0) {
        if ((e = true_residual(c, r, bhat, cfield(x), st, rr))) return e;
    } else {
        MSPCG_HIP(hipMemsetAsync(x.data, 0, (size_t)12 * c->Nh * sizeof(double2), st));
        if ((e = norm2_sync(c, bhat.data, r.data, st, rr))) return e;
    }
    DevScalars s;
    memset(&s, 0, sizeof(s));
    s.rr = rr;
    s.bb = bb;
    s.tol2 = p->tol * p->tol * bb;
    s.done = rr <= s.tol2 ? 1 : 0;
    if ((e = push(c, st, s))) return e;
    // (re)start: z = K r ; p = z ; zr = <z, r>   (alpha = 0 makes beta = 0)
    auto restart = [&]() -> int {
        int e2;
        if ((e2 = precond_apply_flag<S>(c, l, cfield(r), z, &c->sc->done, st))) return e2;
        MSPCG_HIP(hipMemsetAsync(pp.data, 0, (size_t)12 * c->Nh * sizeof(double2), st));
        if (launch_dot2(z.data, r.data, r.data, c->Nh, c->partials, npb, st)) return MSPCG_EHIP;
        if (launch_fpcg_beta(c->sc, c->partials, (int)npb, st)) return MSPCG_EHIP;
        if (launch_xpay(pp.data, z.data, c->Nh, c->sc, 0, st)) return MSPCG_EHIP;
        return 0;
    };
    if (!s.done && (e = restart())) return e;
    const int check = p->check_every > 0 ? p->check_every : 4;
    int restarts = 0, iters = 0;
    bool converged = false;
    double true_rr = rr;
    while (true) {
        if (!s.done) {
            for (int k = 0; k < check && iters + k < p->maxiter; ++k) {
                if ((e = op_A<F64>(c, q, cfield(pp), c->partials, &c->sc->done, st))) return e;
                if (launch_cg_alpha(c->sc, c->partials, (int)nph, st, 1)) return MSPCG_EHIP;
                if (launch_cg_update_xr(x.data, r.data, pp.data, q.data, c->Nh, c->sc, c->partials,
                                        npb, st))
                    return MSPCG_EHIP;
                if (launch_cg_beta(c->sc, c->partials, (int)npb, c->hist, cap, st)) return MSPCG_EHIP;
                if ((e = precond_apply_flag<S>(c, l, cfield(r), z, &c->sc->done, st))) return e;
                if (launch_dot2(z.data, r.data, q.data, c->Nh, c->partials, npb, st)) return MSPCG_EHIP;
                if (launch_fpcg_beta(c->sc, c->partials, (int)npb, st)) return MSPCG_EHIP;
                if (launch_xpay(pp.data, z.data, c->Nh, c->sc, 0, st)) return MSPCG_EHIP;
            }
            if ((e = poll(c, st, s))) return e;
        }
        iters = s.iter;
        if (s.breakdown) {
            fill_stats(c, stats, iters, iters * l, restarts, false, s.rr, bb, c->hist);
            return MSPCG_EBREAKDOWN;
        }
        if (s.done) {
            if ((e = true_residual(c, r, bhat, cfield(x), st, true_rr))) return e;
            if (true_rr <= s.tol2) {
                converged = true;
                break;
            }
            restarts++;
            s.rr = true_rr;
            s.done = 0;
            s.alpha = 0.0;
            if ((e = push(c, st, s))) return e;
            if ((e = restart())) return e;
            if ((e = poll(c, st, s))) return e;
        }
        if (iters >= p->maxiter) {
            if ((e = true_residual(c, r, bhat, cfield(x), st, true_rr))) return e;
            break;
        }
    }
    fill_stats(c, stats, iters, (iters + 1 + restarts) * l, restarts, converged, true_rr, bb,
               c->hist);
    return converged ? MSPCG_OK : MSPCG_ENOCONV;
}

// Mixed-precision CG: FP32 iterations on A, FP64 solution, and a reliable
// update (FP64 true residual, FP32 iterate folded into x) whenever the
// iterated residual has dropped by delta since the last update.
int mixed_cg(mspcg_ctx* c, CField<F64> bhat, Field<F64> x, bool x0, const mspcg_solve_params* p,
             double bb, mspcg_solve_stats* stats, hipStream_t st) {
    Field<F64> r = half_field<F64>(c, "d.cg_r", c->Nh);
    Field<F32> rs = half_field<F32>(c, "s.cg_r", c->Nh);
    Field<F32> ps = half_field<F32>(c, "s.cg_p", c->Nh);
    Field<F32> qs = half_field<F32>(c, "s.cg_q", c->Nh);
    Field<F32> xs = half_field<F32>(c, "s.cg_x", c->Nh);
    if (!r.data || !rs.data || !ps.data || !qs.data || !xs.data) return MSPCG_ENOMEM;
    const long nph = hop_nparts(c);
    const long npb = blas_grid_x(12 * c->Nh);
    int e;
    if ((e = ensure_partials(c, 4 * (size_t)(nph > npb ? nph : npb) + 16))) return e;
    const int cap = p->maxiter + 1;
    if ((e = ensure_hist(c, cap))) return e;
    const double delta = p->delta > 0 ? p->delta : 0.1;
    double rr;
    if (x0) {
        if ((e = true_residual(c, r, bhat, cfield(x), st, rr))) return e;
    } else {
        MSPCG_HIP(hipMemsetAsync(x.data, 0, (size_t)12 * c->Nh * sizeof(double2), st));
        if ((e = norm2_sync(c, bhat.data, r.data, st, rr))) return e;
    }
    MSPCG_HIP(hipMemsetAsync(xs.data, 0, (size_t)12 * c->Nh * sizeof(float2), st));
    if (launch_convert<F64, F32>(cfield(r), rs, c->Nh, st)) return MSPCG_EHIP;
    MSPCG_HIP(hipMemcpyAsync(ps.data, rs.data, (size_t)12 * c->Nh * sizeof(float2),
                             hipMemcpyDeviceToDevice, st));
    DevScalars s;
    memset(&s, 0, sizeof(s));
    s.rr = rr;
    s.bb = bb;
    s.tol2 = p->tol * p->tol * bb;
    double rr_update = rr;  // |r|^2 at the last reliable update
    // the FP32 loop stops (done) at tol2 or when |r|^2 fell by delta^2
    auto set_target = [&](DevScalars& d) {
        const double t = delta * delta * rr_update;
        d.tol2 = t > p->tol * p->tol * bb ? t : p->tol * p->tol * bb;
    };
    set_target(s);
    s.done = rr <= p->tol * p->tol * bb ? 1 : 0;
    if ((e = push(c, st, s))) return e;
    const int check = p->check_every > 0 ? p->check_every : 8;
    int updates = 0, iters = 0;
    bool converged = false;
    double true_rr = rr;
    const double tol2 = p->tol * p->tol * bb;
    while (true) {
        if (!s.done) {
            for (int k = 0; k < check && iters + k < p->maxiter; ++k) {
                if ((e = op_A<F32>(c, qs, cfield(ps), c->partials, &c->sc->done, st))) return e;
                if (launch_cg_alpha(c->sc, c->partials, (int)nph, st, 0)) return MSPCG_EHIP;
                if (launch_cg_update_xr32(xs.data, rs.data, ps.data, qs.data, c->Nh, c->sc,
                                          c->partials, npb, st))
                    return MSPCG_EHIP;
                if (launch_cg_beta(c->sc, c->partials, (int)npb, c->hist, cap, st)) return MSPCG_EHIP;
                if (launch_xpay32(ps.data, rs.data, c->Nh, c->sc, st)) return MSPCG_EHIP;
            }
            if ((e = poll(c, st, s))) return e;
        }
        iters = s.iter;
        if (s.breakdown) {
            fill_stats(c, stats, iters, 0, updates, false, s.rr, bb, c->hist);
            return MSPCG_EBREAKDOWN;
        }
        if (s.done || iters >= p->maxiter) {
            // reliable update: x += xs ; r = bhat - A x in FP64 ; rs = r
            if (launch_accum32(x.data, xs.data, c->Nh, st)) return MSPCG_EHIP;
            if ((e = true_residual(c, r, bhat, cfield(x), st, true_rr))) return e;
            updates++;
            if (true_rr <= tol2) {
                converged = true;
                break;
            }
            if (iters >= p->maxiter) break;
            if (launch_convert<F64, F32>(cfield(r), rs, c->Nh, st)) return MSPCG_EHIP;
            rr_update = true_rr;
            // keep the search direction: p = r + beta p with beta = |r_true|^2 / |r_prev|^2
            s.beta = s.rr > 0 ? s.beta * true_rr / s.rr : 0.0;
            s.rr = true_rr;
            s.done = 0;
            set_target(s);
            if ((e = push(c, st, s))) return e;
            if (launch_xpay32(ps.data, rs.data, c->Nh, c->sc, st)) return MSPCG_EHIP;
        }
    }
    fill_stats(c, stats, iters, 0, updates, converged, true_rr, bb, c->hist);
    return converged ? MSPCG_OK : MSPCG_ENOCONV;
}

}  // namespace

int solve_one(mspcg_ctx* c, const void* b_dev, void* x_dev, const mspcg_solve_params* p,
              mspcg_solve_stats* stats, hipStream_t st) {
    if (p->maxiter < 0 || !(p->tol > 0)) return MSPCG_EINVAL;
    if (p->solver < MSPCG_SOLVER_CG || p->solver > MSPCG_SOLVER_MSPCG) return MSPCG_EINVAL;
    if (p->solver == MSPCG_SOLVER_MSPCG) {
        if (p->inner_iters < 0) return MSPCG_EINVAL;
        if (p->inner_prec < MSPCG_FP64 || p->inner_prec > MSPCG_FP16) return MSPCG_EINVAL;
        for (int m = 0; m < 4; ++m) {
            const int b = p->blocking.block[m];
            if (b < 2 || (b & 1) || c->L[m] % b) return MSPCG_EINVAL;
        }
        if (p->blocking.pad < 0 || p->blocking.pad > 2) return MSPCG_EINVAL;
    }
    c->timing = p->timing != 0;
    timing_reset(c);
    const Progs& P = c->pr;
    Field<F64> be = half_field<F64>(c, "d.sv_be", c->Nh);
    Field<F64> bo = half_field<F64>(c, "d.sv_bo", c->Nh);
    Field<F64> w = half_field<F64>(c, "d.sv_w", c->Nh);
    Field<F64> bp = half_field<F64>(c, "d.sv_bp", c->Nh);
    Field<F64> bhat = half_field<F64>(c, "d.sv_bhat", c->Nh);
    Field<F64> xe = half_field<F64>(c, "d.sv_xe", c->Nh);
    Field<F64> xo = half_field<F64>(c, "d.sv_xo", c->Nh);
    if (!be.data || !bo.data || !w.data || !bp.data || !bhat.data || !xe.data || !xo.data)
        return MSPCG_ENOMEM;
    hipEvent_t e0, e1;
    MSPCG_HIP(hipEventCreate(&e0));
    MSPCG_HIP(hipEventCreate(&e1));
    const auto wall0 = std::chrono::steady_clock::now();
    MSPCG_HIP(hipEventRecord(e0, st));
    int e;
    const double2* b = (const double2*)b_dev;
    if (launch_pack_parity<F64>(b, be, c->L, c->Ls, 0, st)) return MSPCG_EHIP;
    if (launch_pack_parity<F64>(b, bo, c->L, c->Ls, 1, st)) return MSPCG_EHIP;
    if (p->use_x0 && launch_pack_parity<F64>((const double2*)x_dev, xe, c->L, c->Ls, 0, st))
        return MSPCG_EHIP;
    CField<F64> ae = cfield(be);
    if (p->rhs_normal) {
        // the right-hand side of A x = bhat is given directly
        MSPCG_HIP(hipMemcpyAsync(bhat.data, be.data, (size_t)12 * c->Nh * sizeof(double2),
                                 hipMemcpyDeviceToDevice, st));
    } else {
        // b'_e = b_e + (1/2) D_h^eo X b_o ; bhat = Mhat^+ b'_e
        if ((e = op_fived<F64>(c, w, cfield(bo), P.X, nullptr, nullptr, st))) return e;
        if ((e = op_hop<F64>(c, bp, cfield(w), 0, false, scaled(P.id, 0.5, 0.5), &ae, P.id, nullptr,
                             nullptr, st)))
            return e;
        if ((e = op_mhatdag<F64>(c, bhat, cfield(bp), nullptr, st))) return e;
    }
    double bb;
    if ((e = norm2_sync(c, bhat.data, nullptr, st, bb))) return e;
    int rc;
    if (bb == 0.0) {
        MSPCG_HIP(hipMemsetAsync(xe.data, 0, (size_t)12 * c->Nh * sizeof(double2), st));
        if (stats) {
            stats->outer_iters = 0;
            stats->converged = 1;
            stats->true_rel_resid = 0.0;
            stats->resid_history_len = 0;
        }
        rc = MSPCG_OK;
    } else {
        if (p->solver == MSPCG_SOLVER_CG)
            rc = cg_fp64(c, cfield(bhat), xe, p->use_x0 != 0, p, bb, stats, st);
        else if (p->solver == MSPCG_SOLVER_MIXED_CG)
            rc = mixed_cg(c, cfield(bhat), xe, p->use_x0 != 0, p, bb, stats, st);
        else if (p->inner_prec == MSPCG_FP16)
            rc = mspcg_fp64<F16>(c, cfield(bhat), xe, p->use_x0 != 0, p, bb, stats, st);
        else if (p->inner_prec == MSPCG_FP32)
            rc = mspcg_fp64<F32>(c, cfield(bhat), xe, p->use_x0 != 0, p, bb, stats, st);
        else
            rc = mspcg_fp64<F64>(c, cfield(bhat), xe, p->use_x0 != 0, p, bb, stats, st);
        if (rc != MSPCG_OK && rc != MSPCG_ENOCONV) return rc;
    }
    double2* x = (double2*)x_dev;
    if (p->rhs_normal) {
        if (launch_unpack_parity<F64>(cfield(xe), x, c->L, c->Ls, 0, 1, st)) return MSPCG_EHIP;
    } else {
        // x_o = M5op^-1 (b_o + (1/2) D_h^oe B x_e)
        Field<F64> te = w;
        CField<F64> ao = cfield(bo);
        if ((e = op_fived<F64>(c, te, cfield(xe), P.B, nullptr, nullptr, st))) return e;
        if ((e = op_hop<F64>(c, xo, cfield(te), 1, false, scaled(P.M5inv, 0.5, 0.5), &ao, P.M5inv,
                             nullptr, nullptr, st)))
            return e;
        if (launch_unpack_parity<F64>(cfield(xe), x, c->L, c->Ls, 0, 0, st)) return MSPCG_EHIP;
        if (launch_unpack_parity<F64>(cfield(xo), x, c->L, c->Ls, 1, 0, st)) return MSPCG_EHIP;
    }
    MSPCG_HIP(hipEventRecord(e1, st));
    MSPCG_HIP(hipStreamSynchronize(st));
    const auto wall1 = std::chrono::steady_clock::now();
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (stats) {
        stats->seconds = std::chrono::duration<double>(wall1 - wall0).count();
        timing_collect(c, stats);
    } else {
        timing_reset(c);
    }
    c->timing = false;
    return rc;
}

}  // namespace mspcg
