// The even-odd Schur operator for callers that cannot allocate device memory (code under HIP
// graph capture, serving loops, harnesses that forbid hipMalloc): the odd-site intermediate
// t_o = A_oo^-1 D_oe in_e lives in a static device array of the library instead of context memory.
//
// The array is a module global, so every GPU the library runs on holds its own copy at its own
// address for the life of the process.  Host code never passes the array's name to a kernel
// (on the host it is a stand-in symbol, not a device address): the first call on a device, with
// that device current, resolves the device address once with hipGetSymbolAddress and keeps it
// per device.  The buffer needs no clearing between calls: the first launch of D-hat writes every
// real site of t_o before the second launch reads it, and padding sites are never read.  All
// calls on one GPU share the buffer, so calls that overlap in time on one GPU race.
#include <mutex>

#include "internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)DIRAC_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_dev_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (resolved once per device).
void *scratch_ptr() {
    int dev = -1;
    HIP_CHECK(hipGetDevice(&dev));
    dl::require(dev >= 0 && dev < kMaxDevices, "device index out of range for the static scratch table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_dev_ptr[dev]) {
        void *p = nullptr;
        HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        dl::require(p != nullptr, "hipGetSymbolAddress returned no address for the static scratch array",
                    DIRAC_EHIP);
        g_dev_ptr[dev] = p;
    }
    return g_dev_ptr[dev];
}

}  // namespace

namespace dl {

void schur_apply_noalloc(dirac_ctx *c, void *out_e, const void *in_e, int dagger, dirac_prec pr, hipStream_t s) {
    const size_t need = (size_t)24 * real_size(pr) * c->g.vhp;
    require(need <= kScratchBytes,
            std::string("the odd-site intermediate needs ") + std::to_string(need) + " bytes (" + prec_name(pr) +
                ", " + std::to_string(c->g.vhp) + " padded odd sites), more than the " +
                std::to_string(kScratchBytes) + "-byte static buffer of the no-allocation Schur apply");
    PrecFields &f = c->f[pr];
    require(f.links_ready && f.clover_ready && f.inv_ready[1],
            std::string("the ") + prec_name(pr) +
                " fields (links, clover field, odd-site inverse) have not been built; any apply in this "
                "precision builds them");
    schur_apply_into(c, out_e, in_e, scratch_ptr(), dagger, pr, s, 1, nullptr, true);
}

}  // namespace dl
