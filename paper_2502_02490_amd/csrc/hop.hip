// Hopping term between parities, fused with the clover field, and the even-odd Schur and full
// operators built from it.  The kernels and their launch shapes are in hop_kernels.h, compiled
// once per storage precision (hop_f64.hip, hop_f32.hip, hop_f16.hip, hop_bf16.hip).
#include "hop_launch.h"
#include "internal.h"

namespace dl {

void hop_apply(dirac_ctx *c, void *out, const void *in, const void *chi, int p, HopMode mode, double coef, int dagger,
               dirac_prec pr, hipStream_t s, int nrhs, const int *active, bool no_alloc) {
    require(nrhs >= 1, "nrhs must be positive");
    require(p == 0 || p == 1, "parity must be 0 (even) or 1 (odd)");
    PrecFields &f = c->f[pr];
    if (no_alloc)
        require(f.links_ready && (mode == HOP_PLAIN || f.clover_ready),
                std::string("the ") + prec_name(pr) + " fields have not been built; any apply in this precision builds them");
    else
        ensure_prec(c, pr, s);
    require(mode != HOP_INV || f.inv_ready[p], "clover inverse of this parity not computed; call clover_invert");
    switch (pr) {
        case DIRAC_F64: hop_prec_f64(c, out, in, chi, p, mode, coef, dagger, s, nrhs, active, no_alloc); break;
        case DIRAC_F32: hop_prec_f32(c, out, in, chi, p, mode, coef, dagger, s, nrhs, active, no_alloc); break;
        case DIRAC_F16: hop_prec_f16(c, out, in, chi, p, mode, coef, dagger, s, nrhs, active, no_alloc); break;
        case DIRAC_BF16: hop_prec_bf16(c, out, in, chi, p, mode, coef, dagger, s, nrhs, active, no_alloc); break;
        default: throw Error(DIRAC_EINVAL, "unknown precision");
    }
}

// D-hat in_e = A_ee in_e - D_eo A_oo^-1 D_oe in_e, D_eo = -H_eo / 2:
//   t_o = A_oo^-1 (-1/2 H_oe in_e);   out_e = A_ee in_e + 1/2 H_eo t_o
void schur_apply(dirac_ctx *c, void *out_e, const void *in_e, int dagger, dirac_prec pr, hipStream_t s, int nrhs,
                 const int *active) {
    ensure_prec(c, pr, s);
    PrecFields &f = c->f[pr];
    require(f.inv_ready[1], "odd-site clover inverse not available (clover_invert failed or was not run)");
    f.tmp_half.alloc((size_t)nrhs * 24 * real_size(pr) * c->g.vhp);
    schur_apply_into(c, out_e, in_e, f.tmp_half.p, dagger, pr, s, nrhs, active, false);
}

// The two launches of D-hat with the odd intermediate t_o in `tmp` (nrhs odd half vectors of pr);
// no_alloc: build nothing and time nothing (the fields of pr must exist).
void schur_apply_into(dirac_ctx *c, void *out_e, const void *in_e, void *tmp, int dagger, dirac_prec pr,
                      hipStream_t s, int nrhs, const int *active, bool no_alloc) {
    require(c->f[pr].inv_ready[1], "odd-site clover inverse not available (clover_invert failed or was not run)");
    hop_apply(c, tmp, in_e, nullptr, 1, HOP_INV, -0.5, dagger, pr, s, nrhs, active, no_alloc);
    hop_apply(c, out_e, tmp, in_e, 0, HOP_CLOV, 0.5, dagger, pr, s, nrhs, active, no_alloc);
}

// D in: out_p = A_pp in_p - 1/2 H in_{1-p} for both parities (NATIVE full vectors).
void full_apply(dirac_ctx *c, void *out, const void *in, int dagger, dirac_prec pr, hipStream_t s) {
    const size_t hb = (size_t)24 * real_size(pr) * c->g.vhp;
    const char *ie = (const char *)in, *io = ie + hb;
    char *oe = (char *)out, *oo = oe + hb;
    hop_apply(c, oe, io, ie, 0, HOP_CLOV, -0.5, dagger, pr, s);
    hop_apply(c, oo, ie, io, 1, HOP_CLOV, -0.5, dagger, pr, s);
}

}  // namespace dl

