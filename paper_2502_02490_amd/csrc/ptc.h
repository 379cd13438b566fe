// Host-side state of a parallel-transport convolution network (ptc.hip).
#pragma once

#include "internal.h"

struct dirac_ptc {
    int nlayers = 0;
    int ch[9] = {0};           // channels: ch[0] (input) ... ch[nlayers] (output)
    size_t off[8] = {0};       // first complex weight of each layer
    size_t total = 0;          // complex weights in all layers
    dl::DevBuf w;              // FP32 master weights, complex [9][c_out][c_in][4][4] per layer
    dl::DevBuf wbf;            // BF16 working copy (re, im pairs)
    dl::DevBuf wt;             // BF16 adjoint weights of the input-gradient pass
    dl::DevBuf grad;           // dL/dW* accumulated (FP32 complex)
    dl::DevBuf m, v;           // Adam moments (FP32, per real parameter)
    dl::DevBuf acts, gbuf;     // activations of every layer, two gradient buffers
    dl::DevBuf part;           // weight-gradient partials per 64-site tile
    dl::DevBuf afw, afb;       // matrix-core A fragments: forward layers, adjoint (input-gradient) layers
    dl::DevBuf afz, zbuf;      // contract-first last layer: A fragments of z = W x, the 9 fields z_p
    size_t afw_off[8] = {0}, afb_off[8] = {0};  // first fragment (uint4) of each layer
    int step = 0;
    void grad_zero(hipStream_t s) { (void)hipMemsetAsync(grad.p, 0, total * 8, s); }
    // the last layer is summed contract-first (sum_p T_p (sum_c' W x_c')) when it has one output
    // channel and follows another layer, whose kernel then forms the contractions
    bool contract_last() const { return nlayers >= 2 && ch[nlayers] == 1; }
};

namespace dl {
size_t ptc_nweights(const dirac_ptc *n, int layer);
void ptc_alloc(dirac_ptc *n);
void ptc_refresh_bf16(dirac_ptc *n, hipStream_t s);
void ptc_ensure_acts(dirac_ctx *c, dirac_ptc *n);
float *ptc_act(dirac_ctx *c, dirac_ptc *n, int layer);
void ptc_forward_acts(dirac_ctx *c, dirac_ptc *n, hipStream_t s, bool keep_all = true, bool eo = false);
void ptc_backward_acts(dirac_ctx *c, dirac_ptc *n, const void *g_out, void *gin, hipStream_t s);
void ptc_adam(dirac_ptc *n, double lr, hipStream_t s);
}  // namespace dl
