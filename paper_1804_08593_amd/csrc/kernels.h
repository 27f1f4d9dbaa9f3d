// Kernel argument structures and host-side launchers of the MSPCG library.
#pragma once
#include "common.h"

// Fifth-dimension extents compiled into the kernels.
#define MSPCG_LS_LIST(X) X(2) X(4) X(6) X(8) X(10) X(12) X(16) X(20) X(24) X(32)

namespace mspcg {

// Geometry of one hop launch: every domain has an output box, an input box,
// an aux box and a link box (all relative to the domain origin).  The
// periodic (whole-lattice) case has one domain and four identical boxes.
struct HopGeom {
    Box out, in, aux, link;
    int out_par;   // global parity of the output sites
    int periodic;  // bit mu set: wrap at the input-box edges in direction mu (the
                   // box spans the lattice there); clear: drop hops leaving the box
};

struct DevScalars;

template <class S>
struct HopArgs {
    CField<S> in;
    Field<S> out;
    CField<S> aux;
    const typename S::elem* links;
    long link_dom_stride;  // elements between the link arrays of consecutive domains
    HopGeom g;
    FiveDProg ph;  // applied to the hop result
    FiveDProg pa;  // applied to aux
    int has_aux;
    double mf;
    double* partials;  // optional: per (domain, workgroup) sum |out|^2
    const int* done;   // optional: skip the launch when *done != 0
    int xcd_remap;     // map workgroups so each XCD walks a contiguous site range
    int tile[4];       // nonzero: traverse output sites in 4D tiles of this extent
    // optional CG update fused after the output is formed (the last hop of A,
    // whole lattice or block domains):
    //   r -= alpha out ; x += alpha p (x = alpha p when cg_first; no x update
    //   when cg_x.data is null) ; partials = |r|^2 ; out is stored only when
    //   cg_keep_out.
    //   alpha is cg_alpha[domain] when given, else cg_sc->alpha.
    Field<S> cg_r;
    Field<S> cg_x;
    CField<S> cg_p;
    const DevScalars* cg_sc;
    const double* cg_alpha;
    int cg_keep_out;
    int cg_first;
    // optional: the output sites to compute, as checkerboard indices of the
    // output box shared by every domain (n_list of them); the traversal tile
    // is ignored then
    const int* site_list;
    long n_list;
};

template <class S>
int launch_hop(const HopArgs<S>& a, int Ls, int ndom, bool dag, hipStream_t st);

// Several lattices' block-domain hops of one stage in one persistent launch.
// The work list is (lattice i, domain d, workgroup bx): lattice i owns items
// [first[i], first[i+1]), ndom_i * gx[i] of them; a workgroup walks the list
// with a stride of the grid size and skips the items of lattices whose
// `done` flag (a[i].done) is set.  The lattices of one launch share Ls (8, 12
// or 16, multi_hop_ls) and the kernel variant (dagger, chain programs, fused
// update).  The descriptor lives in device memory so a captured graph
// replays it.
constexpr int kMaxBatch = 8;
template <class S>
struct MultiHop {
    HopArgs<S> a[kMaxBatch];
    int ls[kMaxBatch];
    int gx[kMaxBatch];
    long first[kMaxBatch + 1];
    int n;
};
bool multi_hop_ls(int Ls);  // Ls handled by the multi-lattice kernel
template <class S>
int launch_multi_hop(const MultiHop<S>* dev, long items, int Ls, bool dag, bool eph, bool epa,
                     bool cg, hipStream_t st);
template <class S>
long hop_grid_x(long Vh, int Ls);  // workgroups per domain for Vh output sites

// out = P(in) on one box per domain (optionally |out|^2 partials).
template <class S>
struct FiveDArgs {
    CField<S> in;
    Field<S> out;
    long Vh;  // sites per domain
    FiveDProg p;
    double mf;
    double* partials;
    const int* done;
    // optional search-direction update before the program: in = src + beta in,
    // written back through xp_in (the same field as `in`); beta is
    // xp_beta[domain] when given, else xp_sc->beta
    CField<S> xp_src;
    Field<S> xp_in;
    const DevScalars* xp_sc;
    const double* xp_beta;
    // optional, with the update above: zd_z (+)= zd_alpha[domain] * (in before
    // the update); zd_z = that product when zd_first
    Field<S> zd_z;
    const double* zd_alpha;
    int zd_first;
};
template <class S>
int launch_fived(const FiveDArgs<S>& a, int Ls, int ndom, hipStream_t st);
long fived_grid_x(long Vh, int Ls);

// ---- layout conversion -------------------------------------------------
// boundary full field complex128 [Ls][Lt][Lz][Ly][Lx][4][3] <-> one parity of
// the internal whole-lattice layout.
template <class S>
int launch_pack_parity(const double2* full, Field<S> out, const int dims[4], int Ls, int par,
                       hipStream_t st);
template <class S>
int launch_unpack_parity(CField<S> in, double2* full, const int dims[4], int Ls, int par,
                         int zero_other, hipStream_t st);

// internal whole-lattice parity field <-> per-domain interior fields.  The
// domain grid is nb[4] blocks of extent blk[4]; domain d's origin is at
// blk * (d decomposed x-fastest).
template <class SG, class SD>
int launch_global_to_domain(CField<SG> g, Field<SD> dom, const int dims[4], const int blk[4],
                            const int nb[4], int Ls, int par, hipStream_t st);
template <class SD, class SG>
int launch_domain_to_global(CField<SD> dom, Field<SG> g, const int dims[4], const int blk[4],
                            const int nb[4], int Ls, int par, hipStream_t st);
// Even-parity domain_to_global into FP64 with the workgroup partials of
// Re<z, r> (partials[0, np)) and Re<z, q> (partials[np, 2 np)); returns np,
// or -1 on a launch error.
template <class SD>
long launch_domain_to_global_dots(CField<SD> dom, Field<F64> z, CField<F64> r, CField<F64> q,
                                  const int dims[4], const int blk[4], const int nb[4], int Ls,
                                  double* partials, hipStream_t st);

// Links for the link box of every domain (whole lattice: one domain, pad 0).
// U: boundary complex128 [4][Lt][Lz][Ly][Lx][3][3].
template <class S>
int launch_pack_links(const double2* U, typename S::elem* out, const int dims[4], const int blk[4],
                      const int nb[4], const Box& linkbox, int antiperiodic_t, hipStream_t st);

// ---- BLAS-1 and reductions ---------------------------------------------
// All vector kernels work on N = ndom*Vh*Ls elements per component; a 2D
// grid (x: chunks within a domain, y: domain) gives per-domain partial sums.
long blas_grid_x(long per_dom);

// Scalars of one solve, kept on the device.
struct DevScalars {
    double rr;       // current |r|^2 (iterated)
    double pq;       // <p, A p>
    double alpha;
    double beta;
    double zr;       // <z, r>   (flexible PCG)
    double zq;       // <z_new, q>
    double tol2;     // tol^2 |b|^2
    double bb;       // |b|^2
    int done;        // iterated residual reached tol2
    int iter;        // iterations done
    int breakdown;   // non-positive curvature or NaN
};

int launch_reduce_sum(const double* partials, int nparts, double* out, hipStream_t st);
// per-domain sums: partials [ndom][nparts] -> out[ndom]
int launch_reduce_domains(const double* partials, int ndom, int nparts, double* out,
                          hipStream_t st);

// CG scalar updates (single thread kernels)
int launch_cg_alpha(DevScalars* sc, const double* partials, int nparts, hipStream_t st,
                    int flexible = 0);
int launch_fpcg_beta(DevScalars* sc, const double* partials, int nparts, double* hist,
                     int hist_cap, hipStream_t st);
int launch_cg_beta(DevScalars* sc, const double* partials, int nparts, double* hist,
                   int hist_cap, hipStream_t st);

// FP64 whole-lattice vector kernels
int launch_sub_norm(double2* r, const double2* b, const double2* ax, long N, double* partials,
                    long nparts, hipStream_t st);
int launch_copy_norm(double2* dst, const double2* src, long N, double* partials, long nparts,
                     hipStream_t st);
int launch_dot2(const double2* z, const double2* r, const double2* q, long N, double* partials,
                long nparts, hipStream_t st);
int launch_zero(double2* y, long N, hipStream_t st);
// x += z on N whole-lattice entries (skipped when *done)
int launch_xpy(double2* x, const double2* z, long N, const int* done, hipStream_t st);
// y = a x on n complex values (any layout)
int launch_scale(double2* y, const double2* x, double a, long n, hipStream_t st);

// FP32 iterations of the mixed-precision CG
int launch_accum32(double2* x, float2* xs, long N, int Ls, hipStream_t st);

// Mixed-precision conversions (whole vectors)
template <class SI, class SO>
int launch_convert(CField<SI> in, Field<SO> out, long n_sites, hipStream_t st);

}  // namespace mspcg
