// Allocation-free diagnostics: ffpic_diagnostics with every piece of device
// scratch (per-block partial sums and maxima, result slots, the node charge
// map of the Gauss residual, the Poynting flux per radius) taken from one
// file-scope device array instead of hipMalloc.  For callers that may not
// allocate device memory (tight serving loops, harnesses that forbid it).
//
// The array exists once per GPU for the life of the process.  Every call on
// a GPU shares it and leaves its contents behind; what must start at zero
// (the node charge map) is cleared by the call itself.  Calls that overlap
// on one GPU (from several host threads) race on it; calls are serialised
// by the mutex below only for the set-up, not for the kernels.
#include <mutex>
#include <string>

#include "device_common.h"

namespace ffpic {
namespace {

// 32 MiB: partial sums, result slots and Poynting flux always fit; the rest
// holds the node charge map of the Gauss residual for grids of up to about
// 4.1 million nodes
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// device address of this GPU's scratch array (hipGetSymbolAddress once per
// device, with that device current); nullptr on failure
void *scratch_on(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace
}  // namespace ffpic

using namespace ffpic;

extern "C" int ffpic_diagnostics_noalloc(ffpic_ctx *c, uint32_t what, ffpic_diag *out,
                                         double *L) {
    if (!c) return FFPIC_EINVAL;
    if (!out) {
        c->last_error = "NULL output";
        return FFPIC_EINVAL;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != c->device) {
        (void)hipGetLastError();
        c->last_error = "ffpic_diagnostics_noalloc: the context's device is not the current device";
        return FFPIC_EINVAL;
    }
    // layout: partials | 16 result slots | L (nr + 1) | node charges (nn)
    const size_t o_out = align256((size_t)diag_partials() * 5 * sizeof(double));
    const size_t o_L = o_out + align256(16 * sizeof(double));
    const size_t o_qn = o_L + align256((size_t)(c->nr + 1) * sizeof(double));
    const size_t need = (what & FFPIC_DIAG_RESIDUALS) ? o_qn + c->nn * sizeof(double) : o_qn;
    if (need > kScratchBytes) {
        c->last_error = "ffpic_diagnostics_noalloc: the Gauss residual of a grid of " +
                        std::to_string(c->nn) + " nodes needs " + std::to_string(need) +
                        " bytes of scratch, more than the " + std::to_string(kScratchBytes) +
                        " it has (at most " +
                        std::to_string((kScratchBytes - o_qn) / sizeof(double)) + " nodes)";
        return FFPIC_EINVAL;
    }
    unsigned char *base = (unsigned char *)scratch_on(dev);
    if (!base) {
        c->last_error = "ffpic_diagnostics_noalloc: hipGetSymbolAddress of the scratch failed";
        return FFPIC_EHIP;
    }
    DiagBufs b;
    b.part = (double *)base;
    b.out = (double *)(base + o_out);
    b.L = (double *)(base + o_L);
    b.qn = (what & FFPIC_DIAG_RESIDUALS) ? (double *)(base + o_qn) : nullptr;
    return run_diagnostics_checked(c, what, out, L, b);
}
