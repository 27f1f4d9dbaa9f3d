/*
 * Plain FP64 CPU oracle for the even-odd preconditioned domain-wall / Moebius
 * Dirac operator and its block-Dirichlet restriction.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it (through oracle/__init__.py).  It shares no code,
 * header, table or constant with the HIP path.
 *
 * Paper: Guo, Mawhinney, Tu, "Solving DWF Dirac Equation Using Multisplitting
 * Preconditioned Conjugate Gradient" (arXiv:1804.08593).  The paper states the
 * problem (normal equations of the DWF operator, Sec. 2.2 eq. (3); block
 * diagonal preconditioner, Sec. 2.3 eqs. (4)-(5)) but not the operator's
 * formula; the definitions used here are the standard public Shamir (1993) /
 * Moebius (Brower, Neff, Orginos) domain-wall ones.
 *
 * Everything is written in the most literal form: full-lattice fields in
 * lexicographic order, explicit 4x4 gamma matrices, complex arithmetic through
 * C99 <complex.h>, one OpenMP loop over output sites.  No spin projection, no
 * even-odd storage, no fusion.
 *
 * Layouts (all complex double, interleaved re/im):
 *   fermion  psi[s][site][spin 4][colour 3], s = 0..Ls-1
 *   gauge    U[mu][site][row 3][col 3],      mu = 0:x 1:y 2:z 3:t
 *   site     lex = ((t*Lz + z)*Ly + y)*Lx + x
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* Chiral basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] for
 * k = x, y, z and gamma_t = [[0, 1], [1, 0]] (2x2 blocks), so that
 * gamma_5 = gamma_x gamma_y gamma_z gamma_t = diag(1, 1, -1, -1). */
static cplx G[4][4][4];
static int G_ready = 0;

static void init_gamma(void) {
    if (G_ready) return;
    cplx sig[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(G, 0, sizeof(G));
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                G[k][i][2 + j] = -I * sig[k][i][j];
                G[k][2 + i][j] = I * sig[k][i][j];
            }
    for (int i = 0; i < 2; ++i) {
        G[3][i][2 + i] = 1;
        G[3][2 + i][i] = 1;
    }
    G_ready = 1;
}

/* Export the four gamma matrices (for the basis pins in the tests). */
void orc_gamma(double *out /* [4][4][4] complex */) {
    init_gamma();
    memcpy(out, G, sizeof(G));
}

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Scratch fields are kept between calls (one buffer per slot, grown on
 * demand): fresh multi-GB allocations would otherwise be page-faulted on every
 * operator application.  Each routine owns distinct slots, so nested calls
 * never share one.  Not thread-safe: the oracle is driven from one host thread. */
enum { WS_DWF = 0, WS_M5 = 3, WS_SCHUR = 6, WS_NORMAL = 9, WS_PREP = 10, WS_RECON = 12,
       WS_FORCE = 14, WS_NSLOT = 18 };
static cplx *ws_ptr[WS_NSLOT];
static long ws_len[WS_NSLOT];

static cplx *ws(int slot, long n) {
    if (ws_len[slot] < n) {
        free(ws_ptr[slot]);
        ws_ptr[slot] = malloc(n * sizeof(cplx));
        ws_len[slot] = ws_ptr[slot] ? n : 0;
    }
    return ws_ptr[slot];
}

void orc_release_workspace(void) {
    for (int i = 0; i < WS_NSLOT; ++i) {
        free(ws_ptr[i]);
        ws_ptr[i] = NULL;
        ws_len[i] = 0;
    }
}

static inline long lex_of(const int L[4], const int c[4]) {
    return ((long)(c[3] * L[2] + c[2]) * L[1] + c[1]) * L[0] + c[0];
}

static inline void coords_of(const int L[4], long lex, int c[4]) {
    c[0] = (int)(lex % L[0]); lex /= L[0];
    c[1] = (int)(lex % L[1]); lex /= L[1];
    c[2] = (int)(lex % L[2]); lex /= L[2];
    c[3] = (int)lex;
}

/* Wilson hopping term, applied slice by slice in s:
 *   (D_h psi)(x) = sum_mu  eta+ (1 - g_mu) U_mu(x)      psi(x+mu)
 *                        + eta- (1 + g_mu) U_mu(x-mu)^+ psi(x-mu)
 * eta = -1 exactly when the hop crosses the t boundary and antiperiodic_t is
 * set.  dagger != 0 gives D_h^+, which swaps the two projectors.
 * blk != NULL: block-Dirichlet restriction, a term is dropped iff its source
 * site lies in a different block (blocks of extent blk[mu], origins at
 * multiples of blk[mu]) than the output site.
 * only_sites != NULL: compute only those nsites output sites (all s) and
 * write them compactly as out[s][it][spin][colour]. */
/* One term of the hop: acc += eta (1 - pm g_mu)-style spin matrix times the
 * colour product of the link with the source spinor src[spin][colour]:
 *   forward  (dir 0): chi = U_mu(x) src,       acc += eta (1 + pm g_mu) chi
 *   backward (dir 1): chi = U_mu(x-mu)^+ src,  acc += eta (1 + pm g_mu) chi
 * with pm = -sgn forward and +sgn backward (sgn = -1 for the dagger), so the
 * forward term carries (1 - g_mu) and the backward one (1 + g_mu) for D_h. */
static void hop_term(long V4, const cplx *U, long x, long y, int mu, int dir, double eta,
                     double sgn, const cplx *src, cplx acc[4][3]) {
    cplx chi[4][3];
    if (dir == 0) {
        const cplx *u = U + ((long)mu * V4 + x) * 9;
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) {
                cplx t = 0;
                for (int b = 0; b < 3; ++b) t += u[a * 3 + b] * src[sp * 3 + b];
                chi[sp][a] = t;
            }
    } else {
        const cplx *u = U + ((long)mu * V4 + y) * 9;
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) {
                cplx t = 0;
                for (int b = 0; b < 3; ++b) t += conj(u[b * 3 + a]) * src[sp * 3 + b];
                chi[sp][a] = t;
            }
    }
    const double pm = (dir == 0) ? -sgn : sgn;
    for (int sp = 0; sp < 4; ++sp)
        for (int a = 0; a < 3; ++a) {
            cplx t = chi[sp][a];
            for (int sq = 0; sq < 4; ++sq) t += pm * G[mu][sp][sq] * chi[sq][a];
            acc[sp][a] += eta * t;
        }
}

/* Neighbour of site c in direction mu (dir 0: +mu, 1: -mu) with the
 * boundary sign eta; returns its lex index. */
static long neighbour(const int L[4], int antiperiodic_t, const int c[4], int mu, int dir,
                      int n[4], double *eta) {
    n[0] = c[0]; n[1] = c[1]; n[2] = c[2]; n[3] = c[3];
    *eta = 1.0;
    if (dir == 0) {
        n[mu] = c[mu] + 1;
        if (n[mu] == L[mu]) { n[mu] = 0; if (mu == 3 && antiperiodic_t) *eta = -1.0; }
    } else {
        n[mu] = c[mu] - 1;
        if (n[mu] < 0) { n[mu] = L[mu] - 1; if (mu == 3 && antiperiodic_t) *eta = -1.0; }
    }
    return lex_of(L, n);
}

static void hop_impl(const int L[4], int Ls, int antiperiodic_t, const int *blk,
                     const cplx *U, const cplx *in, cplx *out, int dagger,
                     const long *only_sites, long nsites) {
    init_gamma();
    const long V4 = (long)L[0] * L[1] * L[2] * L[3];
    const double sgn = dagger ? -1.0 : 1.0; /* forward term uses (1 - sgn g) */
    const long nloop = only_sites ? nsites : V4;
#pragma omp parallel for schedule(static)
    for (long it = 0; it < nloop; ++it) {
        const long x = only_sites ? only_sites[it] : it;
        int c[4];
        coords_of(L, x, c);
        for (int s = 0; s < Ls; ++s) {
            cplx acc[4][3];
            memset(acc, 0, sizeof(acc));
            for (int mu = 0; mu < 4; ++mu) {
                for (int dir = 0; dir < 2; ++dir) { /* 0: forward x+mu, 1: backward x-mu */
                    int n[4];
                    double eta;
                    const long y = neighbour(L, antiperiodic_t, c, mu, dir, n, &eta);
                    if (blk && (c[mu] / blk[mu]) != (n[mu] / blk[mu])) continue;
                    hop_term(V4, U, x, y, mu, dir, eta, sgn, in + ((long)s * V4 + y) * 12, acc);
                }
            }
            /* full mode: out[s][site]; site-list mode: compact out[s][it] */
            const long o = only_sites ? ((long)s * nsites + it) : ((long)s * V4 + x);
            memcpy(out + o * 12, acc, sizeof(acc));
        }
    }
}

void orc_hop(const int *L, int Ls, int antiperiodic_t, const int *blk, const double *U,
             const double *in, double *out, int dagger) {
    hop_impl(L, Ls, antiperiodic_t, blk, (const cplx *)U, (const cplx *)in, (cplx *)out, dagger,
             NULL, 0);
}

void orc_hop_sites(const int *L, int Ls, int antiperiodic_t, const int *blk, const double *U,
                   const double *in, double *out, int dagger, const long *sites, long nsites) {
    hop_impl(L, Ls, antiperiodic_t, blk, (const cplx *)U, (const cplx *)in, (cplx *)out, dagger,
             sites, nsites);
}

/* Fifth-dimension hopping:
 *   (K psi)_s   = P- psi_{s+1} + P+ psi_{s-1}
 *   (K^+ psi)_s = P- psi_{s-1} + P+ psi_{s+1}
 * with psi_{Ls} := -mf psi_0 and psi_{-1} := -mf psi_{Ls-1}.
 * P+ keeps spins 0,1 and P- keeps spins 2,3 (gamma_5 = diag(1,1,-1,-1)). */
static void ktilde(long V4, int Ls, double mf, const cplx *in, cplx *out, int dagger) {
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V4; ++x)
        for (int s = 0; s < Ls; ++s) {
            /* upper (P+) spins take s-1 for K, s+1 for K^+; lower (P-) the opposite */
            int s_up = dagger ? s + 1 : s - 1;
            int s_dn = dagger ? s - 1 : s + 1;
            double f_up = 1.0, f_dn = 1.0;
            if (s_up < 0) { s_up += Ls; f_up = -mf; }
            if (s_up >= Ls) { s_up -= Ls; f_up = -mf; }
            if (s_dn < 0) { s_dn += Ls; f_dn = -mf; }
            if (s_dn >= Ls) { s_dn -= Ls; f_dn = -mf; }
            cplx *o = out + ((long)s * V4 + x) * 12;
            const cplx *iu = in + ((long)s_up * V4 + x) * 12;
            const cplx *id = in + ((long)s_dn * V4 + x) * 12;
            for (int k = 0; k < 6; ++k) o[k] = f_up * iu[k];
            for (int k = 6; k < 12; ++k) o[k] = f_dn * id[k];
        }
}

void orc_ktilde(const int *L, int Ls, double mf, const double *in, double *out, int dagger) {
    const long V4 = (long)L[0] * L[1] * L[2] * L[3];
    ktilde(V4, Ls, mf, (const cplx *)in, (cplx *)out, dagger);
}

typedef struct {
    int L[4];
    int Ls;
    int antiperiodic_t;
    double M5, mf, b, c;
} orc_action;

/* Full 5D operator:
 *   D   = D_W B + (1 - K),      D_W = (4 - M5) - D_h / 2,  B = b + c K
 *   D^+ = B^+ D_W^+ + (1 - K^+), D_W^+ = (4 - M5) - D_h^+ / 2
 * blk != NULL uses the block-Dirichlet hop in D_W. */
void orc_dwf(const orc_action *a, const int *blk, const double *Ud, const double *ind,
             double *outd, int dagger) {
    const cplx *U = (const cplx *)Ud;
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    const long V4 = (long)a->L[0] * a->L[1] * a->L[2] * a->L[3];
    const long n = V4 * a->Ls * 12;
    cplx *t1 = ws(WS_DWF, n);
    cplx *t2 = ws(WS_DWF + 1, n);
    cplx *k = ws(WS_DWF + 2, n);
    const double m4 = 4.0 - a->M5;
    if (!dagger) {
        /* t1 = B in */
        ktilde(V4, a->Ls, a->mf, in, k, 0);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) t1[i] = a->b * in[i] + a->c * k[i];
        /* t2 = D_h t1 */
        hop_impl(a->L, a->Ls, a->antiperiodic_t, blk, U, t1, t2, 0, NULL, 0);
        /* out = (4-M5) t1 - t2/2 + in - K in */
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) out[i] = m4 * t1[i] - 0.5 * t2[i] + in[i] - k[i];
    } else {
        /* t1 = D_W^+ in */
        hop_impl(a->L, a->Ls, a->antiperiodic_t, blk, U, in, t2, 1, NULL, 0);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) t1[i] = m4 * in[i] - 0.5 * t2[i];
        /* out = b t1 + c K^+ t1 + in - K^+ in */
        ktilde(V4, a->Ls, a->mf, t1, t2, 1);
        ktilde(V4, a->Ls, a->mf, in, k, 1);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) out[i] = a->b * t1[i] + a->c * t2[i] + in[i] - k[i];
    }
}

/* (K psi)_s at one site y (the fifth-dimension hop of ktilde() above). */
static void ktilde_site(long V4, int Ls, double mf, const cplx *in, long y, int s, cplx out[12]) {
    int s_up = s - 1, s_dn = s + 1;
    double f_up = 1.0, f_dn = 1.0;
    if (s_up < 0) { s_up += Ls; f_up = -mf; }
    if (s_dn >= Ls) { s_dn -= Ls; f_dn = -mf; }
    const cplx *iu = in + ((long)s_up * V4 + y) * 12;
    const cplx *id = in + ((long)s_dn * V4 + y) * 12;
    for (int k = 0; k < 6; ++k) out[k] = f_up * iu[k];
    for (int k = 6; k < 12; ++k) out[k] = f_dn * id[k];
}

/* D psi at the listed output sites only (every s), written compactly as
 * out[s][it][spin][colour]; the same definition as orc_dwf,
 *   (D psi)(x,s) = (4 - M5) (B psi)(x,s) - (D_h B psi)(x,s) / 2 + psi(x,s) - (K psi)(x,s),
 * with B psi = b psi + c K psi formed only at x and its eight neighbours. */
void orc_dwf_sites(const orc_action *a, const double *Ud, const double *ind, double *outd,
                   const long *sites, long nsites) {
    init_gamma();
    const cplx *U = (const cplx *)Ud;
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    const int Ls = a->Ls;
    const long V4 = (long)a->L[0] * a->L[1] * a->L[2] * a->L[3];
    const double m4 = 4.0 - a->M5;
#pragma omp parallel for schedule(static)
    for (long it = 0; it < nsites; ++it) {
        const long x = sites[it];
        int c[4];
        coords_of(a->L, x, c);
        for (int s = 0; s < Ls; ++s) {
            cplx acc[4][3];
            memset(acc, 0, sizeof(acc));
            cplx kb[12], bsrc[12];
            for (int mu = 0; mu < 4; ++mu)
                for (int dir = 0; dir < 2; ++dir) {
                    int n[4];
                    double eta;
                    const long y = neighbour(a->L, a->antiperiodic_t, c, mu, dir, n, &eta);
                    ktilde_site(V4, Ls, a->mf, in, y, s, kb);
                    for (int k = 0; k < 12; ++k)
                        bsrc[k] = a->b * in[((long)s * V4 + y) * 12 + k] + a->c * kb[k];
                    hop_term(V4, U, x, y, mu, dir, eta, 1.0, bsrc, acc);
                }
            const cplx *ps = in + ((long)s * V4 + x) * 12;
            ktilde_site(V4, Ls, a->mf, in, x, s, kb);
            cplx *o = out + ((long)s * nsites + it) * 12;
            const cplx *h = &acc[0][0];
            for (int k = 0; k < 12; ++k) {
                const cplx bx = a->b * ps[k] + a->c * kb[k];
                o[k] = m4 * bx - 0.5 * h[k] + ps[k] - kb[k];
            }
        }
    }
}

/* The 5D-local parts of D = M5op - D_h B / 2 (second form):
 *   M5op = alpha + beta K, alpha = (4 - M5) b + 1, beta = (4 - M5) c - 1.
 * which: 0 M5op, 1 M5op^+, 2 B, 3 B^+, 4 M5op^-1, 5 M5op^-+.
 * The inverse is the closed form:
 *   M5op^-1 = (1/alpha) (1 + mf q^Ls)^-1 sum_{k=0}^{Ls-1} q^k K^k,  q = -beta/alpha,
 * evaluated by repeated application of K. */
void orc_m5(const orc_action *a, const double *ind, double *outd, int which) {
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    const long V4 = (long)a->L[0] * a->L[1] * a->L[2] * a->L[3];
    const long n = V4 * a->Ls * 12;
    const double alpha = (4.0 - a->M5) * a->b + 1.0;
    const double beta = (4.0 - a->M5) * a->c - 1.0;
    cplx *k = ws(WS_M5, n);
    if (which <= 3) {
        const int dag = which & 1;
        const double d0 = which <= 1 ? alpha : a->b;
        const double d1 = which <= 1 ? beta : a->c;
        ktilde(V4, a->Ls, a->mf, in, k, dag);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) out[i] = d0 * in[i] + d1 * k[i];
    } else {
        const int dag = which == 5;
        const double q = -beta / alpha;
        const double norm = 1.0 / (alpha * (1.0 + a->mf * pow(q, a->Ls)));
        cplx *cur = ws(WS_M5 + 1, n);
        memcpy(cur, in, n * sizeof(cplx));
        cplx *acc = ws(WS_M5 + 2, n);
        memcpy(acc, in, n * sizeof(cplx));
        double qk = 1.0;
        for (int kk = 1; kk < a->Ls; ++kk) {
            ktilde(V4, a->Ls, a->mf, cur, k, dag);
            memcpy(cur, k, n * sizeof(cplx));
            qk *= q;
#pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) acc[i] += qk * cur[i];
        }
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) out[i] = norm * acc[i];
    }
}

/* Keep only sites of the given parity (0 even, 1 odd); zero the rest. */
static void parity_mask(const int L[4], int Ls, cplx *f, int parity) {
    const long V4 = (long)L[0] * L[1] * L[2] * L[3];
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V4; ++x) {
        int c[4];
        coords_of(L, x, c);
        if (((c[0] + c[1] + c[2] + c[3]) & 1) != parity)
            for (int s = 0; s < Ls; ++s) memset(f + ((long)s * V4 + x) * 12, 0, 12 * sizeof(cplx));
    }
}

void orc_parity_mask(const int *L, int Ls, double *f, int parity) {
    parity_mask(L, Ls, (cplx *)f, parity);
}

/* Even-odd Schur complement on the even sites, from its
 * definition with the full operator and parity projectors P_e, P_o:
 *   Mhat   y = P_e D   y - P_e D   M5op^-1 P_o D   y
 *   Mhat^+ y = P_e D^+ y - P_e D^+ M5op^-+ P_o D^+ y
 * (M_ee = M_oo = M5op because D_h only couples opposite parities.)
 * in and out are full-lattice fields; only the even sites of in are read.
 * blk != NULL gives the block-Dirichlet Schur operator. */
void orc_schur(const orc_action *a, const int *blk, const double *U, const double *ind,
               double *outd, int dagger) {
    const long V4 = (long)a->L[0] * a->L[1] * a->L[2] * a->L[3];
    const long n = V4 * a->Ls * 12;
    cplx *y = ws(WS_SCHUR, n);
    cplx *t = ws(WS_SCHUR + 1, n);
    cplx *u = ws(WS_SCHUR + 2, n);
    memcpy(y, ind, n * sizeof(cplx));
    parity_mask(a->L, a->Ls, y, 0);
    orc_dwf(a, blk, U, (const double *)y, (double *)t, dagger); /* t = D y */
    memcpy(u, t, n * sizeof(cplx));
    parity_mask(a->L, a->Ls, u, 1);                              /* u = P_o D y */
    orc_m5(a, (const double *)u, (double *)y, dagger ? 5 : 4);   /* y = M5^-1 u (odd only) */
    orc_dwf(a, blk, U, (const double *)y, (double *)u, dagger);  /* u = D M5^-1 P_o D y */
    cplx *out = (cplx *)outd;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) out[i] = t[i] - u[i];
    parity_mask(a->L, a->Ls, out, 0);
}

/* Normal operator A = Mhat^+ Mhat on the even sites. */
void orc_normal(const orc_action *a, const int *blk, const double *U, const double *in,
                double *out) {
    const long n = (long)a->L[0] * a->L[1] * a->L[2] * a->L[3] * a->Ls * 12;
    double *t = (double *)ws(WS_NORMAL, n);
    orc_schur(a, blk, U, in, t, 0);
    orc_schur(a, blk, U, t, out, 1);
}

/* Right-hand side for the even-site system:
 *   b'_e = P_e b - P_e D M5op^-1 P_o b ,  bhat = Mhat^+ b'_e
 * Writes bprime (full lattice, even part) and bhat. */
void orc_prepare(const orc_action *a, const double *U, const double *bd, double *bprime,
                 double *bhat) {
    const long V4 = (long)a->L[0] * a->L[1] * a->L[2] * a->L[3];
    const long n = V4 * a->Ls * 12;
    cplx *bo = ws(WS_PREP, n);
    cplx *t = ws(WS_PREP + 1, n);
    memcpy(bo, bd, n * sizeof(cplx));
    parity_mask(a->L, a->Ls, bo, 1);
    orc_m5(a, (const double *)bo, (double *)t, 4);
    orc_dwf(a, NULL, U, (const double *)t, (double *)bo, 0);
    const cplx *b = (const cplx *)bd;
    cplx *bp = (cplx *)bprime;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) bp[i] = b[i] - bo[i];
    parity_mask(a->L, a->Ls, bp, 0);
    orc_schur(a, NULL, U, bprime, bhat, 1);
}

/* Odd-site reconstruction: x_o = M5op^-1 P_o (b - D x_e); x keeps x_e. */
void orc_reconstruct(const orc_action *a, const double *U, const double *bd, double *xd) {
    const long V4 = (long)a->L[0] * a->L[1] * a->L[2] * a->L[3];
    const long n = V4 * a->Ls * 12;
    cplx *x = (cplx *)xd;
    const cplx *b = (const cplx *)bd;
    cplx *t = ws(WS_RECON, n);
    cplx *u = ws(WS_RECON + 1, n);
    parity_mask(a->L, a->Ls, x, 0);
    orc_dwf(a, NULL, U, xd, (double *)t, 0);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) t[i] = b[i] - t[i];
    parity_mask(a->L, a->Ls, t, 1);
    orc_m5(a, (const double *)t, (double *)u, 4);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) x[i] += u[i];
}

/* Fermion force.  For S = phi^+ A^-1 phi, X = A^-1 phi,
 * Y = Mhat X, the derivative of S along U_mu(x) -> exp(i eps T) U_mu(x) with T
 * traceless Hermitian is tr(T F_mu(x)), where, with the 5D fields
 *   a = Y (even) + M5op^-+ P_o D^+ Y (odd)
 *   b = B X (even) + B M5op^-1 P_o D X (odd),
 *   P = sum_{s,spin} [(1 - g_mu) b(x+mu)] a(x)^+ ,
 *   Q = sum_{s,spin} b(x) [(1 + g_mu) a(x+mu)]^+ ,
 *   G = U_mu(x) P - Q U_mu(x)^+ ,
 *   F_mu(x) = eta * traceless part of (G - G^+)/(2i),
 * eta being the boundary sign of the link.  X and Y are full-lattice fields
 * whose odd sites are ignored.  F is [mu][site][3][3]. */
void orc_force(const orc_action *ac, const double *Ud, const double *Xd, const double *Yd,
               double *Fd) {
    init_gamma();
    const int *L = ac->L;
    const int Ls = ac->Ls;
    const long V4 = (long)L[0] * L[1] * L[2] * L[3];
    const long n = V4 * Ls * 12;
    const cplx *U = (const cplx *)Ud;
    cplx *a = ws(WS_FORCE, n);
    cplx *b = ws(WS_FORCE + 1, n);
    cplx *t = ws(WS_FORCE + 2, n);
    cplx *u = ws(WS_FORCE + 3, n);
    /* a */
    memcpy(t, Yd, n * sizeof(cplx));
    parity_mask(L, Ls, t, 0);
    memcpy(a, t, n * sizeof(cplx));
    orc_dwf(ac, NULL, Ud, (const double *)t, (double *)u, 1);
    parity_mask(L, Ls, u, 1);
    orc_m5(ac, (const double *)u, (double *)t, 5);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) a[i] += t[i];
    /* b */
    memcpy(t, Xd, n * sizeof(cplx));
    parity_mask(L, Ls, t, 0);
    orc_m5(ac, (const double *)t, (double *)b, 2);
    parity_mask(L, Ls, b, 0);
    orc_dwf(ac, NULL, Ud, (const double *)t, (double *)u, 0);
    parity_mask(L, Ls, u, 1);
    orc_m5(ac, (const double *)u, (double *)t, 4);
    orc_m5(ac, (const double *)t, (double *)u, 2);
    parity_mask(L, Ls, u, 1);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) b[i] += u[i];
    cplx *F = (cplx *)Fd;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V4; ++x) {
        int c[4];
        coords_of(L, x, c);
        for (int mu = 0; mu < 4; ++mu) {
            int nc[4] = {c[0], c[1], c[2], c[3]};
            double eta = 1.0;
            nc[mu] += 1;
            if (nc[mu] == L[mu]) { nc[mu] = 0; if (mu == 3 && ac->antiperiodic_t) eta = -1.0; }
            const long y = lex_of(L, nc);
            cplx P[3][3], Q[3][3];
            memset(P, 0, sizeof(P));
            memset(Q, 0, sizeof(Q));
            for (int s = 0; s < Ls; ++s) {
                const cplx *ax = a + ((long)s * V4 + x) * 12;
                const cplx *ay = a + ((long)s * V4 + y) * 12;
                const cplx *bx = b + ((long)s * V4 + x) * 12;
                const cplx *by = b + ((long)s * V4 + y) * 12;
                cplx pb[4][3], pa[4][3]; /* (1 - g) b(x+mu), (1 + g) a(x+mu) */
                for (int sp = 0; sp < 4; ++sp)
                    for (int cc = 0; cc < 3; ++cc) {
                        cplx tb = by[sp * 3 + cc], ta = ay[sp * 3 + cc];
                        for (int sq = 0; sq < 4; ++sq) {
                            tb -= G[mu][sp][sq] * by[sq * 3 + cc];
                            ta += G[mu][sp][sq] * ay[sq * 3 + cc];
                        }
                        pb[sp][cc] = tb;
                        pa[sp][cc] = ta;
                    }
                for (int sp = 0; sp < 4; ++sp)
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) {
                            P[i][j] += pb[sp][i] * conj(ax[sp * 3 + j]);
                            Q[i][j] += bx[sp * 3 + i] * conj(pa[sp][j]);
                        }
            }
            const cplx *Um = U + ((long)mu * V4 + x) * 9;
            cplx Gm[3][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    cplx t1 = 0, t2 = 0;
                    for (int k = 0; k < 3; ++k) {
                        t1 += Um[i * 3 + k] * P[k][j];
                        t2 += Q[i][k] * conj(Um[j * 3 + k]);
                    }
                    Gm[i][j] = t1 - t2;
                }
            cplx *Fo = F + ((long)mu * V4 + x) * 9;
            cplx tr = 0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    Fo[i * 3 + j] = eta * (Gm[i][j] - conj(Gm[j][i])) / (2.0 * I);
                    if (i == j) tr += Fo[i * 3 + j];
                }
            for (int i = 0; i < 3; ++i) Fo[i * 3 + i] -= tr / 3.0;
        }
    }
}
