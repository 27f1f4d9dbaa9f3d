/*
 * mspcg.h -- C ABI of the MI355X (gfx950) library for the multisplitting-
 * preconditioned conjugate gradient (MSPCG) solve of the domain-wall /
 * Moebius Dirac equation.
 *
 * Paper: D. Guo, R. Mawhinney, J. Tu, "Solving DWF Dirac Equation Using
 * Multisplitting Preconditioned Conjugate Gradient", arXiv:1804.08593.
 *   Sec. 2.2, eq. (3): the non-Hermitian DWF system D x = b is solved through
 *     its normal equations; here the even-odd Schur complement Mhat of D is
 *     used and CG runs on A = Mhat^+ Mhat.
 *   Sec. 2.3, eqs. (4)-(5), Fig. 3: the preconditioner K = (+)_s A_s keeps the
 *     diagonal blocks of A (one block per node, all other entries zero); it is
 *     applied approximately by l local CG iterations from a zero guess, in
 *     lower precision, with no communication between blocks.
 *   Sec. 3: the figure of merit is the number of global (outer) iterations.
 *
 * Operator conventions (standard Shamir / Moebius domain-wall fermions; the
 * paper only says the operator is a Wilson operator with a large mass times a
 * fictitious fifth dimension, Sec. 2.2):
 *   D   = D_W (b + c K) + (1 - K),   D_W = (4 - M5) - D_h / 2,
 *   D_h psi(x) = sum_mu eta (1 - g_mu) U_mu(x) psi(x+mu) + eta (1 + g_mu) U_mu(x-mu)^+ psi(x-mu),
 *   (K psi)_s = P- psi_{s+1} + P+ psi_{s-1},  psi_{Ls} = -mf psi_0,  psi_{-1} = -mf psi_{Ls-1},
 *   chiral basis g_k = [[0, -i s_k], [i s_k, 0]], g_t = [[0, 1], [1, 0]],
 *   g5 = diag(1, 1, -1, -1), P+- = (1 +- g5)/2, eta = -1 on hops that cross
 *   the time boundary when antiperiodic_t is set.
 *   Even-odd: Mhat = M5op - D_h^eo (b + c K) M5op^-1 D_h^oe (b + c K) / 4 on the
 *   even sites (parity of x+y+z+t), M5op = ((4-M5) b + 1) + ((4-M5) c - 1) K.
 *
 * Boundary layouts (device memory, caller-owned, complex double interleaved):
 *   fermion  [Ls][Lt][Lz][Ly][Lx][4 spin][3 colour]
 *   gauge    [4 mu][Lt][Lz][Ly][Lx][3 row][3 col]   (mu = 0:x 1:y 2:z 3:t)
 *   force    same layout as gauge
 * "Even fields" use the fermion layout; only their even sites are read, and
 * the odd sites of an even-field output are set to zero.
 *
 * Ownership and synchronisation: the library never frees or retains a caller
 * pointer after a call returns.  The context owns its internal gauge copies,
 * work vectors and timing events; mspcg_destroy releases them.  All work is
 * enqueued on the given stream (0 = the null stream).  mspcg_apply and
 * mspcg_precond are asynchronous; mspcg_solve, mspcg_solve_batch and
 * mspcg_force return after the stream has completed because their statistics
 * are host-visible.  A context is not thread-safe: use one per (device,
 * stream).  Every call returns 0 on success or a negative MSPCG_E* code; no
 * exception crosses the ABI.  mspcg_strerror gives the text.
 */
#ifndef MSPCG_H
#define MSPCG_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSPCG_VERSION 1

enum {
    MSPCG_OK = 0,
    MSPCG_EINVAL = -1,    /* invalid argument (dims, Ls, parameters, null pointer) */
    MSPCG_ENOMEM = -2,    /* device (or host) allocation failed */
    MSPCG_EHIP = -3,      /* a HIP runtime call or kernel launch failed */
    MSPCG_ENOGAUGE = -4,  /* operator used before mspcg_load_gauge */
    MSPCG_ENOCONV = -5,   /* solve stopped at maxiter; x holds the last iterate */
    MSPCG_EBREAKDOWN = -6,/* non-positive curvature or non-finite value in a solve */
    MSPCG_EUNSUPPORTED = -7, /* Ls not compiled in, or an unsupported combination */
    MSPCG_ESCRATCH = -8,  /* lattice too large for the fixed scratch of mspcg_apply_noalloc */
    MSPCG_EINTERNAL = -9  /* unexpected host-side failure inside the library (no C++
                             exception ever leaves an entry point) */
};

typedef struct mspcg_ctx mspcg_ctx;

/* Action parameters.  dims = (Lx, Ly, Lz, Lt), every extent even; Ls >= 2 and
 * one of the compiled extents (2 4 6 8 10 12 16 20 24 32); Shamir is b=1, c=0. */
typedef struct {
    int dims[4];
    int Ls;
    double M5;
    double mf;
    double b;
    double c;
    int antiperiodic_t;
} mspcg_action;

/* Operators for mspcg_apply. */
enum {
    MSPCG_OP_D = 0,        /* full 5D operator D on a full field */
    MSPCG_OP_DDAG = 1,     /* D^+ */
    MSPCG_OP_HOP = 2,      /* Wilson hop D_h (both parities, every s slice) */
    MSPCG_OP_HOPDAG = 3,   /* D_h^+ */
    MSPCG_OP_MHAT = 4,     /* even-odd Schur complement Mhat on an even field */
    MSPCG_OP_MHATDAG = 5,  /* Mhat^+ */
    MSPCG_OP_A = 6,        /* A = Mhat^+ Mhat on an even field */
    MSPCG_OP_M5INV = 7,    /* M5op^-1 on a full field (5D-local) */
    MSPCG_OP_PREPARE = 8,  /* even field bhat = Mhat^+ (b_e - M_eo M5op^-1 b_o) from full b */
    MSPCG_OP_KBLOCK = 9    /* preconditioner K = (+)_s A_s on an even field (needs blocks) */
};

/* Arithmetic / storage precision of an operator application. */
enum {
    MSPCG_FP64 = 0,
    MSPCG_FP32 = 1,
    MSPCG_FP16 = 2  /* FP16 storage of spinors (per-(x,s) FP32 scale) and links, FP32 math */
};

/* Solvers. */
enum {
    MSPCG_SOLVER_CG = 0,       /* plain FP64 CG on A */
    MSPCG_SOLVER_MIXED_CG = 1, /* FP32 CG iterations, FP64 solution and reliable updates */
    MSPCG_SOLVER_MSPCG = 2,    /* FP64 flexible outer PCG, sloppy block preconditioner */
    MSPCG_SOLVER_MULTISPLIT = 3 /* the multisplitting iteration of Sec. 2.1, eq. (2), alone:
                                  x += K_l^-1 (bhat - A x), FP64 residual every sweep; it
                                  converges slowly or not at all (Sec. 2.2) */
};

/* Block decomposition of the preconditioner (Sec. 2.3, eq. (5), Fig. 3).
 * block[mu] divides dims[mu] and is even.  With form = MSPCG_FORM_DOMAIN each
 * block's operator is A_s = P_s Mhat_W^+ Mhat_W P_s, where W is the block
 * widened by `pad` sites on both sides of every direction that holds more
 * than one block, and Mhat_W is the even-odd Schur complement of the
 * principal submatrix of D on W (every hop into or out of W dropped):
 *   pad = 2: exactly the paper's A_s = P_s A P_s (the diagonal block of A,
 *            including every path that leaves the block and comes back);
 *   pad = 0: the Dirichlet-cut block Mhat_s^+ Mhat_s (no hop between blocks);
 *   pad = 1: only the paths that leave the block by one site come back.
 * With form = MSPCG_FORM_SPLIT (pad 1 or 2) the block is taken of Mhat before
 * the normal equations: A_s = (P_s Mhat P_s)^+ (P_s Mhat P_s).
 * In a cut direction dims[mu] - block[mu] >= 2 pad is required (the widened
 * block must not wrap onto itself).  With FP16 local solves one widened
 * block must hold fewer than 2^24 sites per parity and under 4 GB per FP16
 * field (MSPCG_EUNSUPPORTED otherwise). */
enum { MSPCG_FORM_DOMAIN = 0, MSPCG_FORM_SPLIT = 1 };
typedef struct {
    int block[4];
    int pad;
    int form;
} mspcg_blocking;

typedef struct {
    double tol;           /* stop when |bhat - A x| / |bhat| <= tol (true residual, FP64) */
    int maxiter;          /* outer iterations */
    int solver;           /* MSPCG_SOLVER_* */
    int use_x0;           /* 1: x holds the initial guess on entry (even part used) */
    mspcg_blocking blocking; /* MSPCG and MULTISPLIT; block[0] == 0: the context's
                                blocking (mspcg_set_blocking) is used */
    int inner_iters;      /* l: local CG iterations per outer iteration (MSPCG, MULTISPLIT) */
    int inner_prec;       /* MSPCG_FP16 / FP32 / FP64 for the local solves (MSPCG, MULTISPLIT) */
    int check_every;      /* host convergence poll interval in iterations (0: auto) */
    double delta;         /* reliable-update threshold of the mixed CG (0: 0.1) */
    int timing;           /* 1: record per-kernel-class times with HIP events */
    int rhs_normal;       /* 1: b is an even field solved directly as A x = b (x: even
                             field, odd sites zero); 0: solve D x = b */
    int batch_kernels;    /* mspcg_solve_batch with MSPCG: 0 = each block-hop stage of the
                             local solves runs as one persistent launch per Ls over a
                             (lattice, block, workgroup) work list that skips converged
                             lattices (when every lattice's Ls is 8, 12 or 16); 1 = one launch
                             per lattice and stage */
} mspcg_solve_params;

/* Launch tuning.  Hop kernels visit their output sites in 4D tiles so that
 * concurrently running workgroups share neighbour spinors in L2; tile[p] is
 * the preferred tile for precision p (MSPCG_FP64/FP32/FP16; all zero =
 * lexicographic order; each extent is reduced to the largest even divisor of
 * the box extent).  xcd_remap = 1 gives each of the 8 XCDs one contiguous
 * range of tiles. */
typedef struct {
    int xcd_remap;
    int tile[3][4];
} mspcg_tuning;

/* Kernel classes reported by the timing facility. */
enum {
    MSPCG_KC_HOP64 = 0,  /* FP64 whole-lattice hop (with fused 5D epilogues) */
    MSPCG_KC_HOP32 = 1,  /* FP32 whole-lattice hop */
    MSPCG_KC_HOPDOM = 2, /* block-domain hop of the local solves (inner precision) */
    MSPCG_KC_FIVED = 3,  /* 5D-only kernels */
    MSPCG_KC_BLAS = 4,   /* vector updates, reductions, conversions */
    MSPCG_KC_HOPCG = 5,  /* last hop of A with the CG vector update fused in (FP64/FP32) */
    MSPCG_KC_HOPDOMCG = 6, /* last block-domain hop of A_s with the local CG update fused in */
    MSPCG_KC_COUNT = 7
};

typedef struct {
    int outer_iters;       /* global iterations */
    int inner_iters_total; /* local iterations summed over outer iterations */
    int restarts;          /* true-residual replacements */
    int converged;
    double true_rel_resid; /* |bhat - A x| / |bhat| in FP64 at exit */
    double seconds;        /* wall time of the solve on the stream */
    double* resid_history; /* caller buffer (may be NULL): |r_k| / |bhat| per outer iteration */
    int resid_history_cap;
    int resid_history_len;
    double kernel_ms[MSPCG_KC_COUNT];     /* timing = 1: summed kernel time per class */
    long kernel_launches[MSPCG_KC_COUNT];
    double kernel_bytes[MSPCG_KC_COUNT];  /* algorithmic bytes of those launches */
    double* cg_coef;       /* caller buffer (may be NULL), plain CG and MSPCG: (alpha_k,
                              beta_k) per iteration k, 2 doubles each (MSPCG: the flexible
                              beta, 0 after a restart); the Lanczos tridiagonal they define
                              bounds the spectrum of A (plain CG) from inside, and estimates
                              that of K_l^-1 A (MSPCG; exact for an exact, fixed K) */
    int cg_coef_cap;       /* iterations the buffer holds */
    int cg_coef_len;
    int batch_persistent;  /* mspcg_solve_batch: 1 when the local solves' block hops ran as
                              persistent multi-lattice launches */
} mspcg_solve_stats;

/* Warning bits reported by mspcg_get_warnings. */
enum {
    MSPCG_WARN_M5_RANGE = 1 /* M5 outside (0, 2): no wall-bound light mode */
};

/* Create a context for one DWF operator D_dw (Sec. 2.2: a Wilson operator
 * with a large mass times a fictitious fifth dimension; the Moebius form of
 * Sec. 1.1's "(generalized) domain wall fermion") on HIP device `device`.
 * Validates the action: every extent even and >= 2, Ls compiled in, b != 0,
 * finite parameters, and the invertibility of M5op (1 + mf q^Ls != 0,
 * q = -beta/alpha); MSPCG_EINVAL otherwise.  M5 outside (0, 2) is accepted
 * and flagged (mspcg_get_warnings).  *ctx receives the new context, which
 * the caller releases with mspcg_destroy. */
int mspcg_create(const mspcg_action* action, int device, mspcg_ctx** ctx);
/* Wait for the context's device, then release every device buffer the
 * context owns (NULL: no-op). */
void mspcg_destroy(mspcg_ctx* ctx);
/* Static text for an MSPCG_* return code. */
const char* mspcg_strerror(int code);
/* MSPCG_VERSION of the header the library was built with. */
int mspcg_version(void);
/* *warnings = the MSPCG_WARN_* bits of the context's action. */
int mspcg_get_warnings(mspcg_ctx* ctx, int* warnings);

/* Load the gauge field U_mu(x) of the sub-lattice the context holds (Sec. 1.1:
 * gauge and pseudofermion fields are split into per-node sub-fields).  U_dev:
 * complex128 device pointer in the gauge layout, read during the call (the
 * caller keeps ownership); copied into the context's internal FP64/FP32/FP16
 * link layouts with the time-boundary sign folded in.  Every call increments
 * the context's gauge generation (mspcg_gauge_generation). */
int mspcg_load_gauge(mspcg_ctx* ctx, const void* U_dev, hipStream_t stream);
/* *gen = number of mspcg_load_gauge calls on this context so far. */
int mspcg_gauge_generation(mspcg_ctx* ctx, unsigned long long* gen);

/* out = op(in) in precision prec (FP64 or FP32; FP16 for MSPCG_OP_KBLOCK):
 * the operators of Sec. 2.2 (D_dw, its adjoint, the normal operator of
 * eq. (3) in even-odd Schur form) and the block preconditioner of Sec. 2.3
 * eq. (5).  in/out: complex128 device pointers in the fermion layout,
 * in != out, both caller-owned; asynchronous on `stream`.
 * MSPCG_OP_KBLOCK uses the blocking set by mspcg_set_blocking. */
int mspcg_apply(mspcg_ctx* ctx, int op, int prec, const void* in_dev, void* out_dev,
                hipStream_t stream);

/* Allocation-free variant of mspcg_apply, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, and
 * harnesses that forbid hipMalloc.  Same operators (MSPCG_OP_D ...
 * MSPCG_OP_PREPARE; MSPCG_OP_KBLOCK gives MSPCG_EUNSUPPORTED), precisions
 * (FP64, FP32), layouts, asynchrony and results as mspcg_apply; the
 * context's gauge field must already be loaded.  Its intermediate fields
 * live in one fixed scratch array per GPU of MSPCG_NOALLOC_SCRATCH_BYTES,
 * held by the library from load to process end, instead of context
 * buffers; no hipMalloc, hipFree or other allocating call is made.  An
 * application needs 8 one-parity fields, 8 * (V4/2) * Ls * 12 * 16 bytes in
 * FP64 (half in FP32), each rounded up to 256 bytes; a larger lattice is
 * rejected with MSPCG_ESCRATCH before any work is queued (FP64 reaches
 * V4 * Ls = 174762, e.g. 8^3x16 at Ls = 16).  Every call on one GPU shares
 * that GPU's scratch and leaves its contents behind: calls on one stream
 * are ordered, but calls that overlap in time on one GPU (several streams
 * or host threads without ordering) race and give undefined results. */
#define MSPCG_NOALLOC_SCRATCH_BYTES (128u << 20)
int mspcg_apply_noalloc(mspcg_ctx* ctx, int op, int prec, const void* in_dev, void* out_dev,
                        hipStream_t stream);

/* Blocking used by MSPCG_OP_KBLOCK and mspcg_precond. */
int mspcg_set_blocking(mspcg_ctx* ctx, const mspcg_blocking* blocking);

/* z = K_l^-1 r: l local CG iterations per block from a zero guess, in
 * precision prec (Sec. 2.3).  r, z: even fields (complex128). */
int mspcg_precond(mspcg_ctx* ctx, int inner_iters, int prec, const void* r_dev, void* z_dev,
                  hipStream_t stream);

/* Solve D_dw x = b through the normal equations (Sec. 2.2, eq. (3)) in
 * even-odd Schur form: CG (or mixed-precision CG) on A = Mhat^+ Mhat, or
 * the multisplitting-preconditioned CG of Sec. 2.3 (flexible outer PCG with
 * z = K_l^-1 r, eqs. (4)-(5)).  b, x: full fields, complex128 device
 * pointers, caller-owned, b != x (x is read as the initial guess when
 * params->use_x0).  The even part is solved and the odd part reconstructed.
 * Returns after the stream has completed.  On MSPCG_ENOCONV x holds the
 * last iterate and stats are filled.  stats may be NULL. */
int mspcg_solve(mspcg_ctx* ctx, const void* b_dev, void* x_dev, const mspcg_solve_params* params,
                mspcg_solve_stats* stats, hipStream_t stream);

/* Pseudofermion action of HMC ensemble generation (Sec. 1.1: the Dirac
 * inversion that dominates the cost): solves A X = phi (even fields, as
 * params->rhs_normal = 1) and returns S = phi^+ A^-1 phi = Re <phi, X> in
 * FP64 (fixed-order reduction).  dphi (may be NULL) receives 2 X, the
 * gradient of S with respect to phi in the convention dS = Re sum conj(dphi)
 * d(phi).  phi, X, dphi: distinct complex128 device pointers in the fermion
 * layout, caller-owned.  Returns after the stream has completed; S is
 * written also on MSPCG_ENOCONV. */
int mspcg_pseudofermion_action(mspcg_ctx* ctx, const void* phi_dev, void* X_dev, void* dphi_dev,
                               const mspcg_solve_params* params, double* S,
                               mspcg_solve_stats* stats, hipStream_t stream);

/* Solve n independent systems (one context each, possibly of different sizes)
 * with the same parameters: the paper's several nodes each solving their own
 * sub-problem (Sec. 2.1, Fig. 1), here several lattices sharing one GPU.  The
 * outer iterations of all still-active systems are interleaved on one
 * stream; arguments as for mspcg_solve, per system.  A system whose
 * right-hand side is zero gets x = 0 with zero iterations and takes no part
 * in the iterations of the others; n = 0 is a no-op.  stats: array of n (may
 * be NULL). */
int mspcg_solve_batch(mspcg_ctx* const* ctxs, int n, const void* const* b_dev, void* const* x_dev,
                      const mspcg_solve_params* params, mspcg_solve_stats* stats,
                      hipStream_t stream);

/* Read / replace the context's launch tuning (see mspcg_tuning).  Launch
 * tuning changes no result.  set: every tile extent must be even and >= 0
 * (MSPCG_EINVAL otherwise); at each launch a preference is clamped to the
 * largest even extent dividing the box it traverses. */
int mspcg_get_tuning(mspcg_ctx* ctx, mspcg_tuning* tuning);
int mspcg_set_tuning(mspcg_ctx* ctx, const mspcg_tuning* tuning);

/* Autotuner: times candidate traversal tiles and the XCD remap on this
 * context's lattice (A in FP64 and FP32; the block operator in FP16 when
 * blocking is not NULL) with HIP events and keeps the fastest.  Results are
 * cached per (dims, Ls, blocking) in the text file cache_path when it is not
 * NULL (read first, appended after tuning; a cached line whose tiles
 * mspcg_set_tuning would reject is skipped).  Needs the gauge field. */
int mspcg_autotune(mspcg_ctx* ctx, const mspcg_blocking* blocking, const char* cache_path,
                   hipStream_t stream);

/* Block-shape autotuner for MSPCG (the blocks play the role of the paper's
 * nodes, Sec. 3): for each candidate blocking (halving any non-empty set of
 * directions, or quartering long ones, where the padded domain still fits),
 * runs probe_iters outer iterations of MSPCG with
 * base's local-solve settings on a fixed synthetic right-hand side and keeps
 * the blocking with the fastest residual reduction per second; probe_iters = 0
 * instead solves every candidate to base's tolerance and keeps the shortest
 * time to solution (slower to tune, and the only reliable choice when a
 * blocking's advantage shows only late in the solve).  The choice becomes the
 * context's blocking and is returned in chosen (may be NULL).  probe_iters < 0:
 * MSPCG_EINVAL. */
int mspcg_tune_blocking(mspcg_ctx* ctx, const mspcg_solve_params* base, int probe_iters,
                        mspcg_blocking* chosen, hipStream_t stream);

/* HMC fermion force of S = phi^+ A^-1 phi (the solve inside ensemble
 * generation, Sec. 1.1).  X = A^-1 phi and Y = Mhat X are even fields.
 * F (gauge layout, may be NULL) receives per link the traceless Hermitian
 * matrix with dS/deps = tr(T F_mu(x)) for U_mu(x) -> exp(i eps T) U_mu(x);
 * G (gauge layout, may be NULL) receives the gradient with respect to the
 * unconstrained complex link, dS = Re sum_ij conj(G_ij) dU_ij.  At least one
 * of F and G must be given.  Returns after the stream has completed. */
int mspcg_force(mspcg_ctx* ctx, const void* X_dev, const void* Y_dev, void* F_dev, void* G_dev,
                hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* MSPCG_H */
