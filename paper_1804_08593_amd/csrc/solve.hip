// Solvers on the even-odd normal equations A x_e = bhat, A = Mhat^+ Mhat
// (Sec. 2.2, eq. (3)), the right-hand-side preparation and the odd-site
// reconstruction.
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
// so the host polls only every `check_every` iterations, and an iteration can
// be captured once in a hipGraph and replayed (the batched solve).  The stop
// test is always re-done on the true residual bhat - A x in FP64.
//
// Each solver is an object with init (eager set-up), iterate (enqueue one
// outer iteration; no host interaction, no allocation, no memset) and
// after_poll (host-side convergence logic on the polled scalars).
#include <math.h>
#include <string.h>

#include <chrono>
#include <memory>

#include "ctx.h"

namespace mspcg {

namespace {

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

// |v|^2 of an FP64 half field (optionally copied to copy_to), synchronously.
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
    // three entries per iteration: |r|^2, alpha, beta
    if (hipMalloc(&c->hist, (size_t)cap * 3 * sizeof(double)) != hipSuccess) return MSPCG_ENOMEM;
    c->hist_cap = cap;
    return 0;
}

struct Solver {
    mspcg_ctx* c = nullptr;
    const mspcg_solve_params* p = nullptr;
    CField<F64> bhat;
    Field<F64> x;
    bool x0 = false;
    double bb = 0;
    DevScalars s;
    int iters = 0, restarts = 0, inner_total = 0;
    bool converged = false, finished = false, breakdown = false;
    double true_rr = 0;
    virtual ~Solver() {}
    virtual int init(hipStream_t st) = 0;
    virtual int iterate(hipStream_t st) = 0;
    virtual int after_poll(hipStream_t st) = 0;
    virtual int check_default() const = 0;
    // MSPCG solvers in a batch split one iteration around the local solves,
    // which the batch runs for every lattice together (BatchPrecond)
    virtual bool batch_mspcg() const { return false; }
    virtual int iterate_pre(hipStream_t) { return MSPCG_EUNSUPPORTED; }
    virtual int iterate_post(hipStream_t, long) { return MSPCG_EUNSUPPORTED; }
    virtual void batch_io(CField<F64>&, Field<F64>&, CField<F64>&) {}
    int rc() const {
        if (breakdown) return MSPCG_EBREAKDOWN;
        return converged ? MSPCG_OK : MSPCG_ENOCONV;
    }
    void fill(mspcg_solve_stats* st) const {
        if (!st) return;
        st->outer_iters = iters;
        st->inner_iters_total = inner_total;
        st->restarts = restarts;
        st->converged = converged ? 1 : 0;
        st->true_rel_resid = sqrt(true_rr / bb);
        st->resid_history_len = 0;
        st->cg_coef_len = 0;
        const bool want_h = st->resid_history && st->resid_history_cap > 0;
        const bool want_c = st->cg_coef && st->cg_coef_cap > 0 &&
                            (p->solver == MSPCG_SOLVER_CG || p->solver == MSPCG_SOLVER_MSPCG);
        const int cap_h = want_h ? st->resid_history_cap : 0;
        const int cap_c = want_c ? st->cg_coef_cap : 0;
        int n = cap_h > cap_c ? cap_h : cap_c;
        if (iters < n) n = iters;
        if (n > 0 && c->hist) {
            std::vector<double> h(3 * (size_t)n);
            if (hipMemcpy(h.data(), c->hist, h.size() * sizeof(double), hipMemcpyDeviceToHost) ==
                hipSuccess) {
                const int nh = n < cap_h ? n : cap_h;
                for (int i = 0; i < nh; ++i) st->resid_history[i] = sqrt(h[3 * i] / bb);
                st->resid_history_len = nh;
                const int nc = n < cap_c ? n : cap_c;
                for (int i = 0; i < nc; ++i) {
                    st->cg_coef[2 * i] = h[3 * i + 1];
                    st->cg_coef[2 * i + 1] = h[3 * i + 2];
                }
                st->cg_coef_len = nc;
            }
        }
    }
};

// Plain FP64 CG on A x = bhat.
struct CGSolver : Solver {
    Field<F64> r, pp, q;
    long nph = 0, npb = 0;
    int cap = 0;
    int check_default() const override { return 8; }
    int init(hipStream_t st) override {
        r = half_field<F64>(c, "d.cg_r", c->Nh);
        pp = half_field<F64>(c, "d.cg_p", c->Nh);
        q = half_field<F64>(c, "d.cg_q", c->Nh);
        if (!r.data || !pp.data || !q.data) return MSPCG_ENOMEM;
        nph = hop_nparts(c);
        npb = blas_grid_x(12 * c->Nh);
        int e;
        if ((e = ensure_partials(c, 4 * (nph > npb ? nph : npb) + 16))) return e;
        cap = p->maxiter + 1;
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
        memset(&s, 0, sizeof(s));
        s.rr = rr;
        s.bb = bb;
        s.tol2 = p->tol * p->tol * bb;
        s.done = rr <= s.tol2 ? 1 : 0;
        true_rr = rr;
        return push(c, st, s);
    }
    // p = r + beta p ; q = A p ; x += alpha p ; r -= alpha q ; beta  (all fused
    // into the operator kernels; beta = 0 on the first step makes p = r)
    int iterate(hipStream_t st) override {
        int e;
        if ((e = cg_step<F64>(c, x, r, pp, q, cfield(r), false, false, &c->sc->done, st))) return e;
        if (launch_cg_beta(c->sc, c->partials, (int)nph, c->hist, cap, st)) return MSPCG_EHIP;
        return 0;
    }
    int after_poll(hipStream_t st) override {
        int e;
        iters = s.iter;
        if (s.breakdown) {
            breakdown = finished = true;
            return 0;
        }
        if (s.done) {
            if ((e = true_residual(c, r, bhat, cfield(x), st, true_rr))) return e;
            if (true_rr <= s.tol2) {
                converged = finished = true;
                return 0;
            }
            // continue from the true residual: the next step forms p = r + beta p
            // with beta = |r_true|^2 / |r_prev|^2
            restarts++;
            s.beta = s.beta * true_rr / s.rr;
            s.rr = true_rr;
            s.done = 0;
            if ((e = push(c, st, s))) return e;
        }
        if (iters >= p->maxiter) {
            if ((e = true_residual(c, r, bhat, cfield(x), st, true_rr))) return e;
            finished = true;
        }
        return 0;
    }
};

// Flexible preconditioned CG (FP64) with z = K_l^-1 r in storage precision S.
template <class S>
struct MSPCGSolver : Solver {
    Field<F64> r, pp, q, z;
    long nph = 0, npb = 0;
    int cap = 0, l = 0;
    int check_default() const override { return 4; }
    // z = K r ; p = z ; zr = <z, r>   (alpha = 0 makes beta = 0)
    int restart(hipStream_t st) {
        int e;
        if ((e = precond_apply_flag<S>(c, l, cfield(r), z, &c->sc->done, st))) return e;
        MSPCG_HIP(hipMemsetAsync(pp.data, 0, (size_t)12 * c->Nh * sizeof(double2), st));
        if (launch_dot2(z.data, r.data, r.data, c->Nh, c->partials, npb, st)) return MSPCG_EHIP;
        if (launch_fpcg_beta(c->sc, c->partials, (int)npb, c->hist, cap, st)) return MSPCG_EHIP;
        return 0;
    }
    int init(hipStream_t st) override {
        r = half_field<F64>(c, "d.cg_r", c->Nh);
        pp = half_field<F64>(c, "d.cg_p", c->Nh);
        q = half_field<F64>(c, "d.cg_q", c->Nh);
        z = half_field<F64>(c, "d.cg_z", c->Nh);
        if (!r.data || !pp.data || !q.data || !z.data) return MSPCG_ENOMEM;
        int e;
        if ((e = domains_setup(c, p->blocking, p->inner_prec, st))) return e;
        nph = hop_nparts(c);
        npb = blas_grid_x(12 * c->Nh);
        size_t need = 4 * (size_t)(nph > npb ? nph : npb) + 16;
        const size_t pneed = precond_partials_need(c);
        if (pneed > need) need = pneed;
        if ((e = ensure_partials(c, need))) return e;
        cap = p->maxiter + 1;
        if ((e = ensure_hist(c, cap))) return e;
        l = p->inner_iters;
        double rr;
        if (x0) {
            if ((e = true_residual(c, r, bhat, cfield(x), st, rr))) return e;
        } else {
            MSPCG_HIP(hipMemsetAsync(x.data, 0, (size_t)12 * c->Nh * sizeof(double2), st));
            if ((e = norm2_sync(c, bhat.data, r.data, st, rr))) return e;
        }
        memset(&s, 0, sizeof(s));
        s.rr = rr;
        s.bb = bb;
        s.tol2 = p->tol * p->tol * bb;
        s.done = rr <= s.tol2 ? 1 : 0;
        true_rr = rr;
        if ((e = push(c, st, s))) return e;
        if (!s.done) {
            if ((e = restart(st))) return e;
            inner_total += l;
        }
        return 0;
    }
    // p = z + beta p ; q = A p ; x += alpha p ; r -= alpha q (fused, q kept) ;
    // z = K r ; flexible beta from <z, r> and <z, q>
    int iterate(hipStream_t st) override {
        int e;
        if ((e = iterate_pre(st))) return e;
        PrecondDots dots{cfield(r), cfield(q), 0};
        if ((e = precond_apply_flag<S>(c, l, cfield(r), z, &c->sc->done, st, &dots))) return e;
        return iterate_post(st, dots.np);
    }
    bool batch_mspcg() const override { return true; }
    int iterate_pre(hipStream_t st) override {
        int e;
        if ((e = cg_step<F64>(c, x, r, pp, q, cfield(z), true, true, &c->sc->done, st))) return e;
        if (launch_cg_beta(c->sc, c->partials, (int)nph, c->hist, cap, st)) return MSPCG_EHIP;
        return 0;
    }
    // np: partials of Re<z, r>, Re<z, q> left by the local solves (0: form them)
    int iterate_post(hipStream_t st, long np) override {
        if (np == 0) {
            if (launch_dot2(z.data, r.data, q.data, c->Nh, c->partials, npb, st)) return MSPCG_EHIP;
            np = npb;
        }
        if (launch_fpcg_beta(c->sc, c->partials, (int)np, c->hist, cap, st)) return MSPCG_EHIP;
        return 0;
    }
    void batch_io(CField<F64>& r_, Field<F64>& z_, CField<F64>& q_) override {
        r_ = cfield(r);
        z_ = z;
        q_ = cfield(q);
    }
    int after_poll(hipStream_t st) override {
        int e;
        // local solves run in every iteration except the one that set `done`
        const int new_iters = s.iter - iters;
        iters = s.iter;
        inner_total += l * (s.done ? (new_iters > 0 ? new_iters - 1 : 0) : new_iters);
        if (s.breakdown) {
            breakdown = finished = true;
            return 0;
        }
        if (s.done) {
            if ((e = true_residual(c, r, bhat, cfield(x), st, true_rr))) return e;
            if (true_rr <= s.tol2) {
                converged = finished = true;
                return 0;
            }
            restarts++;
            s.rr = true_rr;
            s.done = 0;
            s.alpha = 0.0;
            if ((e = push(c, st, s))) return e;
            if ((e = restart(st))) return e;
            inner_total += l;
        }
        if (iters >= p->maxiter) {
            if ((e = true_residual(c, r, bhat, cfield(x), st, true_rr))) return e;
            finished = true;
        }
        return 0;
    }
};

// Mixed-precision CG: FP32 iterations on A, FP64 solution, and a reliable
// update (FP64 true residual, FP32 iterate folded into x) whenever the
// iterated residual has dropped by delta since the last update.
struct MixedSolver : Solver {
    Field<F64> r;
    Field<F32> rs, ps, qs, xs;
    long nph = 0, npb = 0;
    int cap = 0;
    double delta = 0.1, rr_update = 0, tol2 = 0;
    int check_default() const override { return 8; }
    void set_target() {
        const double t = delta * delta * rr_update;
        s.tol2 = t > tol2 ? t : tol2;
    }
    int init(hipStream_t st) override {
        r = half_field<F64>(c, "d.cg_r", c->Nh);
        rs = half_field<F32>(c, "s.cg_r", c->Nh);
        ps = half_field<F32>(c, "s.cg_p", c->Nh);
        qs = half_field<F32>(c, "s.cg_q", c->Nh);
        xs = half_field<F32>(c, "s.cg_x", c->Nh);
        if (!r.data || !rs.data || !ps.data || !qs.data || !xs.data) return MSPCG_ENOMEM;
        nph = hop_nparts(c);
        npb = blas_grid_x(12 * c->Nh);
        int e;
        if ((e = ensure_partials(c, 4 * (size_t)(nph > npb ? nph : npb) + 16))) return e;
        cap = p->maxiter + 1;
        if ((e = ensure_hist(c, cap))) return e;
        delta = p->delta > 0 ? p->delta : 0.1;
        tol2 = p->tol * p->tol * bb;
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
        memset(&s, 0, sizeof(s));
        s.rr = rr;
        s.bb = bb;
        rr_update = rr;
        set_target();
        s.done = rr <= tol2 ? 1 : 0;
        true_rr = rr;
        return push(c, st, s);
    }
    // the FP32 CG step, fused as in plain CG
    int iterate(hipStream_t st) override {
        int e;
        if ((e = cg_step<F32>(c, xs, rs, ps, qs, cfield(rs), false, false, &c->sc->done, st)))
            return e;
        if (launch_cg_beta(c->sc, c->partials, (int)nph, c->hist, cap, st)) return MSPCG_EHIP;
        return 0;
    }
    int after_poll(hipStream_t st) override {
        int e;
        iters = s.iter;
        if (s.breakdown) {
            breakdown = finished = true;
            return 0;
        }
        if (s.done || iters >= p->maxiter) {
            // reliable update: x += xs ; r = bhat - A x in FP64 ; rs = r
            if (launch_accum32(x.data, xs.data, c->Nh, c->Ls, st)) return MSPCG_EHIP;
            if ((e = true_residual(c, r, bhat, cfield(x), st, true_rr))) return e;
            restarts++;
            if (true_rr <= tol2) {
                converged = finished = true;
                return 0;
            }
            if (iters >= p->maxiter) {
                finished = true;
                return 0;
            }
            if (launch_convert<F64, F32>(cfield(r), rs, c->Nh, st)) return MSPCG_EHIP;
            rr_update = true_rr;
            // keep the search direction: the next step forms p = r + beta p with
            // beta = |r_true|^2 / |r_prev|^2
            s.beta = s.rr > 0 ? s.beta * true_rr / s.rr : 0.0;
            s.rr = true_rr;
            s.done = 0;
            set_target();
            if ((e = push(c, st, s))) return e;
        }
        return 0;
    }
};

// The multisplitting iteration (Sec. 2.1, eq. (2)) as a solver of its own:
// every block solves its local system with the other blocks' current
// solution as Dirichlet data, which for the block-diagonal K is the sweep
//   x += K_l^-1 (bhat - A x),
// the local solves run on the correction from a zero guess (eq. (4) on the
// first sweep).  The residual is recomputed in FP64 after every sweep, so
// the iterated residual is the true one.
template <class S>
struct MultisplitSolver : Solver {
    Field<F64> r, z, q;
    long npb = 0;
    int cap = 0, l = 0;
    int check_default() const override { return 4; }
    int init(hipStream_t st) override {
        r = half_field<F64>(c, "d.cg_r", c->Nh);
        z = half_field<F64>(c, "d.cg_z", c->Nh);
        q = half_field<F64>(c, "d.cg_q", c->Nh);
        if (!r.data || !z.data || !q.data) return MSPCG_ENOMEM;
        int e;
        if ((e = domains_setup(c, p->blocking, p->inner_prec, st))) return e;
        npb = blas_grid_x(12 * c->Nh);
        size_t need = 4 * (size_t)npb + 16;
        const size_t pneed = precond_partials_need(c);
        if (pneed > need) need = pneed;
        if ((e = ensure_partials(c, need))) return e;
        cap = p->maxiter + 1;
        if ((e = ensure_hist(c, cap))) return e;
        l = p->inner_iters;
        double rr;
        if (x0) {
            if ((e = true_residual(c, r, bhat, cfield(x), st, rr))) return e;
        } else {
            MSPCG_HIP(hipMemsetAsync(x.data, 0, (size_t)12 * c->Nh * sizeof(double2), st));
            if ((e = norm2_sync(c, bhat.data, r.data, st, rr))) return e;
        }
        memset(&s, 0, sizeof(s));
        s.rr = rr;
        s.bb = bb;
        s.tol2 = p->tol * p->tol * bb;
        s.done = rr <= s.tol2 ? 1 : 0;
        true_rr = rr;
        return push(c, st, s);
    }
    // z = K_l^-1 r ; x += z ; r = bhat - A x with |r|^2
    int iterate(hipStream_t st) override {
        int e;
        const int* done = &c->sc->done;
        if ((e = precond_apply_flag<S>(c, l, cfield(r), z, done, st))) return e;
        if (launch_xpy(x.data, z.data, c->Nh, done, st)) return MSPCG_EHIP;
        if ((e = op_A<F64>(c, q, cfield(x), nullptr, done, st))) return e;
        if (launch_sub_norm(r.data, bhat.data, q.data, c->Nh, c->partials, npb, st))
            return MSPCG_EHIP;
        if (launch_cg_beta(c->sc, c->partials, (int)npb, c->hist, cap, st)) return MSPCG_EHIP;
        return 0;
    }
    int after_poll(hipStream_t) override {
        const int new_iters = s.iter - iters;
        iters = s.iter;
        inner_total += l * new_iters;
        true_rr = s.rr;
        if (s.breakdown) {
            breakdown = finished = true;
            return 0;
        }
        if (s.done) converged = finished = true;
        if (iters >= p->maxiter) finished = true;
        return 0;
    }
};

std::unique_ptr<Solver> make_solver(const mspcg_solve_params* p) {
    if (p->solver == MSPCG_SOLVER_MULTISPLIT) {
        if (p->inner_prec == MSPCG_FP16) return std::unique_ptr<Solver>(new MultisplitSolver<F16>());
        if (p->inner_prec == MSPCG_FP32) return std::unique_ptr<Solver>(new MultisplitSolver<F32>());
        return std::unique_ptr<Solver>(new MultisplitSolver<F64>());
    }
    if (p->solver == MSPCG_SOLVER_CG) return std::unique_ptr<Solver>(new CGSolver());
    if (p->solver == MSPCG_SOLVER_MIXED_CG) return std::unique_ptr<Solver>(new MixedSolver());
    if (p->inner_prec == MSPCG_FP16) return std::unique_ptr<Solver>(new MSPCGSolver<F16>());
    if (p->inner_prec == MSPCG_FP32) return std::unique_ptr<Solver>(new MSPCGSolver<F32>());
    return std::unique_ptr<Solver>(new MSPCGSolver<F64>());
}

// A solve whose params carry no blocking (block[0] == 0) uses the context's
// blocking (mspcg_set_blocking), so each system of a batch can have its own.
mspcg_solve_params effective(const mspcg_ctx* c, const mspcg_solve_params* p) {
    mspcg_solve_params q = *p;
    if ((q.solver == MSPCG_SOLVER_MSPCG || q.solver == MSPCG_SOLVER_MULTISPLIT) &&
        q.blocking.block[0] == 0 && c->has_blocking)
        q.blocking = c->blocking;
    return q;
}

int validate(const mspcg_ctx* c, const mspcg_solve_params* p) {
    if (p->maxiter < 0 || !(p->tol > 0)) return MSPCG_EINVAL;
    if (p->solver < MSPCG_SOLVER_CG || p->solver > MSPCG_SOLVER_MULTISPLIT) return MSPCG_EINVAL;
    if (p->solver == MSPCG_SOLVER_MSPCG || p->solver == MSPCG_SOLVER_MULTISPLIT) {
        if (p->inner_iters < 0) return MSPCG_EINVAL;
        if (p->inner_prec < MSPCG_FP64 || p->inner_prec > MSPCG_FP16) return MSPCG_EINVAL;
        if (p->blocking.pad < 0 || p->blocking.pad > 2) return MSPCG_EINVAL;
        if (p->blocking.form != MSPCG_FORM_DOMAIN && p->blocking.form != MSPCG_FORM_SPLIT)
            return MSPCG_EINVAL;
        if (p->blocking.form == MSPCG_FORM_SPLIT && p->blocking.pad < 1) return MSPCG_EINVAL;
        for (int m = 0; m < 4; ++m) {
            const int b = p->blocking.block[m];
            if (b < 2 || (b & 1) || c->L[m] % b) return MSPCG_EINVAL;
            if (c->L[m] / b > 1 && c->L[m] - b < 2 * p->blocking.pad) return MSPCG_EINVAL;
        }
    }
    return MSPCG_OK;
}

// Per-context fields of one solve: boundary b / x and the even-site system.
struct Problem {
    mspcg_ctx* c = nullptr;
    const double2* b = nullptr;
    double2* xout = nullptr;
    Field<F64> be, bo, w, bp, bhat, xe, xo;
    double bb = 0;
};

// pack b (and x0), bhat = Mhat^+ (b_e - M_eo M5op^-1 b_o) or b_e itself
int prepare(Problem& pb, const mspcg_solve_params* p, hipStream_t st) {
    mspcg_ctx* c = pb.c;
    const Progs& P = c->pr;
    pb.be = half_field<F64>(c, "d.sv_be", c->Nh);
    pb.bo = half_field<F64>(c, "d.sv_bo", c->Nh);
    pb.w = half_field<F64>(c, "d.sv_w", c->Nh);
    pb.bp = half_field<F64>(c, "d.sv_bp", c->Nh);
    pb.bhat = half_field<F64>(c, "d.sv_bhat", c->Nh);
    pb.xe = half_field<F64>(c, "d.sv_xe", c->Nh);
    pb.xo = half_field<F64>(c, "d.sv_xo", c->Nh);
    if (!pb.be.data || !pb.bo.data || !pb.w.data || !pb.bp.data || !pb.bhat.data || !pb.xe.data ||
        !pb.xo.data)
        return MSPCG_ENOMEM;
    if (launch_pack_parity<F64>(pb.b, pb.be, c->L, c->Ls, 0, st)) return MSPCG_EHIP;
    if (!p->rhs_normal && launch_pack_parity<F64>(pb.b, pb.bo, c->L, c->Ls, 1, st))
        return MSPCG_EHIP;
    if (p->use_x0 && launch_pack_parity<F64>(pb.xout, pb.xe, c->L, c->Ls, 0, st))
        return MSPCG_EHIP;
    int e;
    CField<F64> ae = cfield(pb.be);
    if (p->rhs_normal) {
        MSPCG_HIP(hipMemcpyAsync(pb.bhat.data, pb.be.data, (size_t)12 * c->Nh * sizeof(double2),
                                 hipMemcpyDeviceToDevice, st));
    } else {
        // b'_e = b_e + (1/2) D_h^eo X b_o ; bhat = Mhat^+ b'_e
        if ((e = op_fived<F64>(c, pb.w, cfield(pb.bo), P.X, nullptr, nullptr, st))) return e;
        if ((e = op_hop<F64>(c, pb.bp, cfield(pb.w), 0, false, scaled(P.id, 0.5, 0.5), &ae, P.id,
                             nullptr, nullptr, st)))
            return e;
        if ((e = op_mhatdag<F64>(c, pb.bhat, cfield(pb.bp), nullptr, st))) return e;
    }
    return norm2_sync(c, pb.bhat.data, nullptr, st, pb.bb);
}

// x_o = M5op^-1 (b_o + (1/2) D_h^oe B x_e) and unpack
int reconstruct(Problem& pb, const mspcg_solve_params* p, hipStream_t st) {
    mspcg_ctx* c = pb.c;
    const Progs& P = c->pr;
    int e;
    if (p->rhs_normal) {
        if (launch_unpack_parity<F64>(cfield(pb.xe), pb.xout, c->L, c->Ls, 0, 1, st))
            return MSPCG_EHIP;
        return 0;
    }
    CField<F64> ao = cfield(pb.bo);
    if ((e = op_fived<F64>(c, pb.w, cfield(pb.xe), P.B, nullptr, nullptr, st))) return e;
    if ((e = op_hop<F64>(c, pb.xo, cfield(pb.w), 1, false, scaled(P.M5inv, 0.5, 0.5), &ao,
                         P.M5inv, nullptr, nullptr, st)))
        return e;
    if (launch_unpack_parity<F64>(cfield(pb.xe), pb.xout, c->L, c->Ls, 0, 0, st)) return MSPCG_EHIP;
    if (launch_unpack_parity<F64>(cfield(pb.xo), pb.xout, c->L, c->Ls, 1, 0, st)) return MSPCG_EHIP;
    return 0;
}

void zero_stats(mspcg_solve_stats* st) {
    if (!st) return;
    st->outer_iters = st->inner_iters_total = st->restarts = 0;
    st->converged = 1;
    st->true_rel_resid = 0.0;
    st->resid_history_len = 0;
    st->cg_coef_len = 0;
}

void clear_timing(mspcg_solve_stats* st) {
    if (!st) return;
    for (int k = 0; k < MSPCG_KC_COUNT; ++k) {
        st->kernel_ms[k] = 0;
        st->kernel_launches[k] = 0;
        st->kernel_bytes[k] = 0;
    }
}

}  // namespace

int solve_one(mspcg_ctx* c, const void* b_dev, void* x_dev, const mspcg_solve_params* p_in,
              mspcg_solve_stats* stats, hipStream_t st) {
    int e;
    const mspcg_solve_params pe = effective(c, p_in);
    const mspcg_solve_params* p = &pe;
    if ((e = validate(c, p))) return e;
    c->timing = p->timing != 0;
    timing_reset(c);
    const auto wall0 = std::chrono::steady_clock::now();
    Problem pb;
    pb.c = c;
    pb.b = (const double2*)b_dev;
    pb.xout = (double2*)x_dev;
    if ((e = prepare(pb, p, st))) return e;
    int rc = MSPCG_OK;
    if (pb.bb == 0.0) {
        MSPCG_HIP(hipMemsetAsync(pb.xe.data, 0, (size_t)12 * c->Nh * sizeof(double2), st));
        zero_stats(stats);
    } else {
        std::unique_ptr<Solver> S = make_solver(p);
        S->c = c;
        S->p = p;
        S->bhat = cfield(pb.bhat);
        S->x = pb.xe;
        S->x0 = p->use_x0 != 0;
        S->bb = pb.bb;
        if ((e = S->init(st))) return e;
        const int check = p->check_every > 0 ? p->check_every : S->check_default();
        if (S->s.done && (e = S->after_poll(st))) return e;
        while (!S->finished) {
            if (!S->s.done) {
                for (int k = 0; k < check && S->iters + k < p->maxiter; ++k)
                    if ((e = S->iterate(st))) return e;
                if ((e = poll(c, st, S->s))) return e;
            }
            if ((e = S->after_poll(st))) return e;
        }
        S->fill(stats);
        rc = S->rc();
        if (rc == MSPCG_EBREAKDOWN) return rc;
    }
    if ((e = reconstruct(pb, p, st))) return e;
    MSPCG_HIP(hipStreamSynchronize(st));
    const auto wall1 = std::chrono::steady_clock::now();
    if (stats) {
        stats->seconds = std::chrono::duration<double>(wall1 - wall0).count();
        timing_collect(c, stats);
    } else {
        timing_reset(c);
    }
    c->timing = false;
    return rc;
}

// Batched solve: n independent systems (contexts of possibly different sizes
// and Ls) advance together.  One outer iteration of every system is captured
// once into a hipGraph on an internal stream and replayed; a converged
// system's kernels see its device `done` flag and return immediately (the
// per-lattice active mask), and the host polls every `check` replays.
int solve_batch(mspcg_ctx* const* cs, int n, const void* const* b, void* const* x,
                const mspcg_solve_params* p, mspcg_solve_stats* stats, hipStream_t ust) {
    int e;
    std::vector<mspcg_solve_params> ps(n > 0 ? n : 1);
    for (int i = 0; i < n; ++i) {
        if (!cs[i] || !b[i] || !x[i] || b[i] == x[i]) return MSPCG_EINVAL;
        if (!cs[i]->gauge) return MSPCG_ENOGAUGE;
        if (cs[i]->device != cs[0]->device) return MSPCG_EINVAL;
        for (int j = 0; j < i; ++j)
            if (cs[j] == cs[i]) return MSPCG_EINVAL;  // one system per context
        ps[i] = effective(cs[i], p);
        if ((e = validate(cs[i], &ps[i]))) return e;
    }
    if (p->solver == MSPCG_SOLVER_MIXED_CG || p->solver == MSPCG_SOLVER_MULTISPLIT)
        return MSPCG_EUNSUPPORTED;
    if (n == 0) return MSPCG_OK;
    MSPCG_HIP(hipSetDevice(cs[0]->device));
    hipStream_t st;
    MSPCG_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    hipEvent_t ev;
    MSPCG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    MSPCG_HIP(hipEventRecord(ev, ust));
    MSPCG_HIP(hipStreamWaitEvent(st, ev, 0));
    const auto wall0 = std::chrono::steady_clock::now();
    std::vector<Problem> pbs(n);
    std::vector<std::unique_ptr<Solver>> sv(n);
    int rc = MSPCG_OK;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::unique_ptr<BatchPrecond> bprec;
    bool batch_multi = false;
    auto body = [&]() -> int {
        for (int i = 0; i < n; ++i) {
            mspcg_ctx* c = cs[i];
            c->timing = false;
            timing_reset(c);
            pbs[i].c = c;
            pbs[i].b = (const double2*)b[i];
            pbs[i].xout = (double2*)x[i];
            if ((e = prepare(pbs[i], &ps[i], st))) return e;
            sv[i] = make_solver(&ps[i]);
            Solver& S = *sv[i];
            S.c = c;
            S.p = &ps[i];
            S.bhat = cfield(pbs[i].bhat);
            S.x = pbs[i].xe;
            S.x0 = p->use_x0 != 0;
            S.bb = pbs[i].bb;
            if (pbs[i].bb == 0.0) {
                MSPCG_HIP(hipMemsetAsync(pbs[i].xe.data, 0, (size_t)12 * c->Nh * sizeof(double2),
                                         st));
                S.finished = S.converged = true;
                continue;
            }
            if ((e = S.init(st))) return e;
            if (S.s.done && (e = S.after_poll(st))) return e;
        }
        // MSPCG: the local solves of all lattices run together, every block-hop
        // stage as one persistent multi-lattice launch (batch_kernels == 0)
        std::vector<int> act;  // systems with a nonzero right-hand side
        for (int i = 0; i < n; ++i)
            if (pbs[i].bb != 0.0) act.push_back(i);
        bool together = p->solver == MSPCG_SOLVER_MSPCG && !act.empty();
        for (int i : act) together = together && sv[i]->batch_mspcg();
        std::vector<CField<F64>> rr(act.size()), qq(act.size());
        std::vector<Field<F64>> zz(act.size());
        std::vector<PrecondDots> dots(act.size());
        if (together) {
            std::vector<mspcg_ctx*> ac;
            std::vector<const int*> dn;
            for (size_t j = 0; j < act.size(); ++j) {
                const int i = act[j];
                sv[i]->batch_io(rr[j], zz[j], qq[j]);
                ac.push_back(cs[i]);
                dn.push_back(&cs[i]->sc->done);
            }
            if ((e = make_batch_precond(ac.data(), (int)ac.size(), ps[act[0]].inner_prec,
                                        ps[act[0]].inner_iters, dn.data(),
                                        p->batch_kernels == 0, bprec)))
                return e;
            batch_multi = bprec->multi;
        }
        // One outer iteration of every system not yet finished.  Captured, a
        // finished system's kernels are left out of the graph altogether (its
        // device done flag also makes them return at once, which is what the
        // systems that finish between two captures rely on).
        auto iterate_all = [&](bool eager) -> int {
            if (!together) {
                for (int i = 0; i < n; ++i) {
                    Solver& S = *sv[i];
                    if (S.bb == 0.0 || S.finished || (eager && S.s.done)) continue;
                    if ((e = S.iterate(st))) return e;
                }
                return 0;
            }
            for (int i : act)
                if (!sv[i]->finished && (e = sv[i]->iterate_pre(st))) return e;
            for (size_t j = 0; j < act.size(); ++j) dots[j] = PrecondDots{rr[j], qq[j], 0};
            if ((e = bprec->apply(ps[act[0]].inner_iters, rr.data(), zz.data(), dots.data(), st)))
                return e;
            for (size_t j = 0; j < act.size(); ++j)
                if (!sv[act[j]]->finished && (e = sv[act[j]]->iterate_post(st, dots[j].np)))
                    return e;
            return 0;
        };
        // the set of unfinished systems the current graph was captured for
        std::vector<char> captured(n, 0);
        auto capture = [&]() -> int {
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            exec = nullptr;
            graph = nullptr;
            for (int i = 0; i < n; ++i) captured[i] = !sv[i]->finished;
            MSPCG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            if ((e = iterate_all(false))) {
                (void)hipStreamEndCapture(st, &graph);
                return e;
            }
            MSPCG_HIP(hipStreamEndCapture(st, &graph));
            MSPCG_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
            return 0;
        };
        // nothing to iterate (every right-hand side zero, or every warm start
        // already converged): no eager pass and no graph
        bool pending = false;
        for (int i = 0; i < n; ++i) pending = pending || !sv[i]->finished;
        const int check = p->check_every > 0 ? p->check_every : 4;
        int replays = 1;
        if (pending) {
            // one eager iteration creates every lazily allocated buffer before capture
            if ((e = iterate_all(true))) return e;
            MSPCG_HIP(hipStreamSynchronize(st));
            if ((e = capture())) return e;
        }
        while (pending) {
            bool all = true, changed = false;
            for (int i = 0; i < n; ++i) {
                Solver& S = *sv[i];
                if (S.finished) continue;
                if ((e = poll(S.c, st, S.s))) return e;
                if ((e = S.after_poll(st))) return e;
                all = all && S.finished;
            }
            if (all) break;
            if (replays >= p->maxiter) {
                for (int i = 0; i < n; ++i) sv[i]->finished = true;
                break;
            }
            for (int i = 0; i < n; ++i) changed = changed || (captured[i] && sv[i]->finished);
            if (changed && (e = capture())) return e;
            for (int k = 0; k < check && replays < p->maxiter; ++k, ++replays)
                MSPCG_HIP(hipGraphLaunch(exec, st));
        }
        for (int i = 0; i < n; ++i) {
            Solver& S = *sv[i];
            if (S.bb != 0.0) S.fill(stats ? stats + i : nullptr);
            else zero_stats(stats ? stats + i : nullptr);
            const int r = S.bb == 0.0 ? MSPCG_OK : S.rc();
            if (r == MSPCG_EBREAKDOWN) rc = r;
            else if (r == MSPCG_ENOCONV && rc == MSPCG_OK) rc = r;
            if ((e = reconstruct(pbs[i], &ps[i], st))) return e;
        }
        return 0;
    };
    e = body();
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (!e) {
        if (hipEventRecord(ev, st) != hipSuccess || hipStreamWaitEvent(ust, ev, 0) != hipSuccess)
            e = MSPCG_EHIP;
    }
    (void)hipStreamSynchronize(st);
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - wall0).count();
    for (int i = 0; i < n && stats; ++i) {
        stats[i].seconds = secs;
        stats[i].batch_persistent = batch_multi ? 1 : 0;
        clear_timing(stats + i);
    }
    (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(st);
    return e ? e : rc;
}

}  // namespace mspcg
