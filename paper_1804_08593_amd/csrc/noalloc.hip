// Allocation-free operator application (mspcg_apply_noalloc).
//
// The intermediate one-parity fields of an operator application come from a
// fixed file-scope device array instead of context buffers, so the call
// makes no hipMalloc / hipFree.  Each GPU holds its own copy of the array at
// its own address; mspcg_create looks that address up once per device, with
// the device current, and host code only ever uses the looked-up pointer.
#include <mutex>

#include "ctx.h"

using namespace mspcg;

namespace {

__device__ __align__(256) unsigned char scratch[MSPCG_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
// an application of A needs 8 one-parity fields: in/out of both parities
// and the 4 intermediates of Mhat^+ Mhat
constexpr size_t kFields = 8;

std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices];
bool g_done[kMaxDevices];

unsigned char* scratch_of(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[device];
}

// Points the context's buffers at the scratch for one call; restores the
// normal allocating mode on exit.
struct ArenaScope {
    mspcg_ctx* c;
    ArenaScope(mspcg_ctx* c_, unsigned char* base, size_t cap) : c(c_) {
        c->arena = reinterpret_cast<char*>(base);
        c->arena_cap = cap;
        c->arena_used = 0;
        c->arena_slots.clear();
    }
    ~ArenaScope() {
        c->arena = nullptr;
        c->arena_cap = c->arena_used = 0;
        c->arena_slots.clear();
    }
};

}  // namespace

int mspcg::noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return MSPCG_OK;  // entry point reports it
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_done[device]) return MSPCG_OK;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MSPCG_EHIP;
    g_ptr[device] = static_cast<unsigned char*>(p);
    g_done[device] = true;
    return MSPCG_OK;
}

extern "C" int mspcg_apply_noalloc(mspcg_ctx* c, int op, int prec, const void* in_dev,
                                   void* out_dev, hipStream_t st) try {
    if (!c || !in_dev || !out_dev || in_dev == out_dev) return MSPCG_EINVAL;
    if (op == MSPCG_OP_KBLOCK) return MSPCG_EUNSUPPORTED;
    if (op < 0 || op > MSPCG_OP_PREPARE) return MSPCG_EINVAL;
    if (prec != MSPCG_FP64 && prec != MSPCG_FP32) return MSPCG_EINVAL;
    if (!c->gauge) return MSPCG_ENOGAUGE;
    unsigned char* base = scratch_of(c->device);
    if (!base) return MSPCG_EUNSUPPORTED;
    const size_t elem = prec == MSPCG_FP64 ? sizeof(double2) : sizeof(float2);
    const size_t field = ((size_t)c->Nh * 12 * elem + 255) & ~(size_t)255;
    if (kFields * field > (size_t)MSPCG_NOALLOC_SCRATCH_BYTES) return MSPCG_ESCRATCH;
    MSPCG_HIP(hipSetDevice(c->device));
    const bool timing = c->timing;
    c->timing = false;  // per-class timing would create events
    int e;
    {
        ArenaScope scope(c, base, MSPCG_NOALLOC_SCRATCH_BYTES);
        e = apply_op(c, op, prec, (const double2*)in_dev, (double2*)out_dev, st);
    }
    c->timing = timing;
    return e == MSPCG_ENOMEM ? MSPCG_ESCRATCH : e;
}
MSPCG_ABI_CATCH
