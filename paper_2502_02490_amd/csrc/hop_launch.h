// Entry points of the per-precision hop translation units (hop_f64.hip ... hop_bf16.hip):
// hop_t<S> of hop_kernels.h with S the storage type of the precision.
#pragma once

#include "internal.h"

namespace dl {

// hop_t<S> of hop_kernels.h for one storage precision, one translation unit each
void hop_prec_f64(dirac_ctx *c, void *out, const void *in, const void *chi, int p, HopMode mode, double coef,
                  int dagger, hipStream_t s, int nrhs, const int *active, bool no_tune);
void hop_prec_f32(dirac_ctx *c, void *out, const void *in, const void *chi, int p, HopMode mode, double coef,
                  int dagger, hipStream_t s, int nrhs, const int *active, bool no_tune);
void hop_prec_f16(dirac_ctx *c, void *out, const void *in, const void *chi, int p, HopMode mode, double coef,
                  int dagger, hipStream_t s, int nrhs, const int *active, bool no_tune);
void hop_prec_bf16(dirac_ctx *c, void *out, const void *in, const void *chi, int p, HopMode mode, double coef,
                   int dagger, hipStream_t s, int nrhs, const int *active, bool no_tune);

}  // namespace dl
