// Host-side context of the MSPCG library and the operator building blocks
// shared by apply, the solvers and the force.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <new>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mspcg.h"
#include "common.h"
#include "kernels.h"

// Closes an entry point written as a function-try-block, so that no C++
// exception leaves the C ABI: host allocation failures report MSPCG_ENOMEM,
// anything else MSPCG_EINTERNAL.
#define MSPCG_ABI_CATCH                                  \
    catch (const std::bad_alloc&) { return MSPCG_ENOMEM; } \
    catch (...) { return MSPCG_EINTERNAL; }

namespace mspcg {

#define MSPCG_HIP(call)                                  \
    do {                                                 \
        if ((call) != hipSuccess) return MSPCG_EHIP;     \
    } while (0)
#define MSPCG_TRY(call)              \
    do {                             \
        int _e = (call);             \
        if (_e != 0) return _e < -1 ? MSPCG_EHIP : MSPCG_EUNSUPPORTED; \
    } while (0)

// Per-kernel-class event timing (only when enabled).
struct TimingRec {
    int kc;
    hipEvent_t a, b;
    double bytes;
};

// The five-dimensional programs of the action.
struct Progs {
    FiveDProg id, B, Bdag, X, Xdag, M5, M5dag, M5inv, M5invdag;
};

FiveDProg scaled(FiveDProg p, double s_up, double s_dn);

// Padded block-domain geometry of the local solves.
struct Domains {
    int blk[4];
    int nb[4];
    int ndom;
    int pad;
    int form;      // MSPCG_FORM_DOMAIN / MSPCG_FORM_SPLIT
    Box interior;  // block, offset 0
    Box pad1;      // block padded by min(pad,1)
    Box pad2;      // block padded by min(pad,2) (also the link box)
    long Vh_int;
    bool built;
    int prec;      // precision of the links below
    void* links;   // [ndom][2][8][9][Vh(pad2)]
    // Output sites of the middle hops of the block operator that matter:
    // even sites of the pad2 box within Manhattan distance 2 of the block
    // (where Mhat_D p can be nonzero) and odd sites of the pad1 box within
    // distance 1 (the only ones the last hop reads).  Checkerboard indices
    // of the box, ascending, shared by all domains; null when pad = 0.
    // rd_*: sites of the hop's input box (one parity) that those outputs read.
    int* list_y;
    long n_y, rd_y;
    int* list_v;
    long n_v, rd_v;
    // box of the middle even field y = Mhat_D p: the widened block (within
    // distance 2 through list_y) for FORM_DOMAIN, the block itself for
    // FORM_SPLIT
    const Box& ybox() const { return form == MSPCG_FORM_SPLIT ? interior : pad2; }
    const int* ylist() const { return form == MSPCG_FORM_SPLIT ? nullptr : list_y; }
    long yn() const { return form == MSPCG_FORM_SPLIT ? 0 : n_y; }
    long yread() const { return form == MSPCG_FORM_SPLIT ? 0 : rd_y; }
    // output sites of the y hop (its partials count)
    long yout() const { return ylist() ? n_y : ybox().Vh; }
};

}  // namespace mspcg

struct mspcg_ctx {
    mspcg_action act;
    int device;
    int L[4];
    int Ls;
    long V4, Vh, Nh;  // sites, sites per parity, (site,s) per parity
    double alpha5, beta5, q5;
    mspcg::Progs pr;
    mspcg::Box lat;  // whole lattice box
    // gauge
    double2* U;      // boundary-layout copy
    double2* L64;
    float2* L32;
    __half2* L16;
    bool gauge;
    unsigned long long gauge_gen;  // incremented by every mspcg_load_gauge
    int warnings;                  // MSPCG_WARN_* bits found by mspcg_create
    // buffers
    std::map<std::string, std::pair<void*, size_t>> bufs;
    // allocation-free mode (mspcg_apply_noalloc): while `arena` is set, buf()
    // carves named fields out of it instead of allocating
    char* arena;
    size_t arena_cap, arena_used;
    std::map<std::string, std::pair<size_t, size_t>> arena_slots;
    double* partials;
    size_t partials_len;
    mspcg::DevScalars* sc;
    mspcg::DevScalars* sc_host;  // pinned mirror
    double* hist;
    int hist_cap;
    // blocking
    mspcg_blocking blocking;
    bool has_blocking;
    mspcg::Domains dom;
    // launch tuning (traversal tiles per precision, XCD remap)
    mspcg_tuning tune;
    // timing
    bool timing;
    std::vector<mspcg::TimingRec> trecs;
    std::vector<hipEvent_t> evpool;
    size_t evused;

    void* buf(const std::string& name, size_t bytes);
};

namespace mspcg {

// Timing scope: records events around the launches of one kernel class.
struct Timed {
    mspcg_ctx* c;
    int kc;
    double bytes;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(mspcg_ctx* c_, int kc_, double bytes_, hipStream_t st_);
    ~Timed();
};

void timing_reset(mspcg_ctx* c);
void timing_collect(mspcg_ctx* c, mspcg_solve_stats* st);

template <class S>
Field<S> half_field(mspcg_ctx* c, const std::string& name, long N);
template <class S>
typename S::elem* links_of(mspcg_ctx* c);

// Whole-lattice operator pieces on one-parity fields of precision S.
template <class S>
int op_hop(mspcg_ctx* c, Field<S> out, CField<S> in, int out_par, bool dag, const FiveDProg& ph,
           const CField<S>* aux, const FiveDProg& pa, double* partials, const int* done,
           hipStream_t st);
template <class S>
int op_fived(mspcg_ctx* c, Field<S> out, CField<S> in, const FiveDProg& p, double* partials,
             const int* done, hipStream_t st);
// y = Mhat p (even); optional |y|^2 partials
template <class S>
int op_mhat(mspcg_ctx* c, Field<S> y, CField<S> p, double* partials, const int* done,
            hipStream_t st);
template <class S>
int op_mhatdag(mspcg_ctx* c, Field<S> q, CField<S> y, const int* done, hipStream_t st);
// q = A p with <p, A p> = |Mhat p|^2 partials
template <class S>
int op_A(mspcg_ctx* c, Field<S> q, CField<S> p, double* partials, const int* done,
         hipStream_t st);
// fused CG update of a whole-lattice hop (see HopArgs)
template <class S>
struct CgUpdate {
    Field<S> r, x;
    CField<S> p;
    const DevScalars* sc;
    int keep_out;
};
template <class S>
int cg_step(mspcg_ctx* c, Field<S> x, Field<S> r, Field<S> p, Field<S> q, CField<S> src,
            bool keep_q, bool flexible, const int* done, hipStream_t st);
long hop_nparts(mspcg_ctx* c);
// traversal tile for a box: the largest even divisor of each extent that does
// not exceed the preferred tile (all zero: lexicographic order)
void pick_tile(const int pref[4], const Box& b, int out[4]);
template <class S>
int prec_index();

int ensure_partials(mspcg_ctx* c, size_t n);

// Domains of the block preconditioner
int domains_setup(mspcg_ctx* c, const mspcg_blocking& b, int prec, hipStream_t st);
size_t precond_partials_need(mspcg_ctx* c);
template <class S>
int precond_apply(mspcg_ctx* c, int inner_iters, CField<F64> r_e, Field<F64> z_e,
                  hipStream_t st, int* inner_done);
// Optional output of precond_apply_flag: with l > 0 the workgroup partials of
// Re<z, r> and Re<z, q> are left in ctx->partials ([0, np) and [np, 2 np));
// np stays 0 when they were not formed (l = 0).
struct PrecondDots {
    CField<F64> r, q;
    long np;
};
template <class S>
int precond_apply_flag(mspcg_ctx* c, int l, CField<F64> r, Field<F64> z, const int* done,
                       hipStream_t st, PrecondDots* dots = nullptr);
template <class S>
int kblock_apply(mspcg_ctx* c, CField<F64> p_e, Field<F64> q_e, hipStream_t st);
// The local solves of several lattices (mspcg_solve_batch) interleaved stage
// by stage; with `multi`, each block-hop stage of every lattice runs in one
// persistent multi-lattice launch (when every lattice's Ls allows it).
struct BatchPrecond {
    bool multi = false;
    virtual ~BatchPrecond() {}
    // z[i] = K_l^-1 r[i] on every lattice; dots[i] as in precond_apply_flag
    virtual int apply(int l, const CField<F64>* r, const Field<F64>* z, PrecondDots* dots,
                      hipStream_t st) = 0;
};
int make_batch_precond(mspcg_ctx* const* cs, int n, int prec, int l, const int* const* done,
                       bool multi, std::unique_ptr<BatchPrecond>& out);
// w = A_s p on every block (domain layout, precision S)
template <class S>
int block_A(mspcg_ctx* c, Field<S> w, CField<S> p, double* partials, const int* done,
            hipStream_t st);

// mspcg_apply's operators (every op but MSPCG_OP_KBLOCK) in FP64 or FP32
int apply_op(mspcg_ctx* c, int op, int prec, const double2* in, double2* out, hipStream_t st);
// the allocation-free scratch of the current device (set up by mspcg_create)
int noalloc_init(int device);

int solve_one(mspcg_ctx* c, const void* b_dev, void* x_dev, const mspcg_solve_params* p,
              mspcg_solve_stats* stats, hipStream_t st);
int solve_batch(mspcg_ctx* const* cs, int n, const void* const* b, void* const* x,
                const mspcg_solve_params* p, mspcg_solve_stats* stats, hipStream_t st);

}  // namespace mspcg
