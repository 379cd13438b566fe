// The hop kernels of hop_kernels.h instantiated for __hip_bfloat16 storage.
#include "hop_kernels.h"

namespace dl {

void hop_prec_bf16(dirac_ctx *c, void *out, const void *in, const void *chi, int p, HopMode mode, double coef,
                   int dagger, hipStream_t s, int nrhs, const int *active, bool no_tune) {
    hop_t<__hip_bfloat16>(c, out, in, chi, p, mode, coef, dagger, DIRAC_BF16, s, nrhs, active, no_tune);
}

}  // namespace dl
