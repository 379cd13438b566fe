// Krylov solvers (placeholder until the BLAS kernels land).
#include "internal.h"

namespace dl {
void free_solver_work(dirac_ctx *) {}
}  // namespace dl

extern "C" dirac_status dirac_solve(dirac_ctx *, void *, const void *, dirac_layout, const dirac_solver_params *,
                                    dirac_solve_info *, void *) {
    return DIRAC_EUNSUPPORTED;
}
