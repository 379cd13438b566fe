/* A C program against include/dirac.h and libdirac.so alone (no Python): the free-field
 * operator on a point source, checked entry by entry against the hopping term written out by
 * hand, plus one refused call.  Built and run by tests/test_gpu_c_abi.py. */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "dirac.h"

#define L 4
#define V (L * L * L * L)

static int fail(const char *what) {
    fprintf(stderr, "FAIL: %s (%s)\n", what, dirac_last_error());
    return 1;
}

int main(void) {
    double complex *U = calloc((size_t)V * 4 * 9, sizeof(double complex));
    double complex *psi = calloc((size_t)V * 12, sizeof(double complex));
    double complex *out = calloc((size_t)V * 12, sizeof(double complex));
    double complex want[V][12];
    memset(want, 0, sizeof want);
    for (int s = 0; s < V * 4; ++s)
        for (int a = 0; a < 3; ++a) U[(size_t)s * 9 + a * 3 + a] = 1.0;
    void *dU, *dpsi, *dout;
    if (hipMalloc(&dU, (size_t)V * 4 * 9 * 16) || hipMalloc(&dpsi, (size_t)V * 192) || hipMalloc(&dout, (size_t)V * 192))
        return fail("hipMalloc");
    hipMemcpy(dU, U, (size_t)V * 4 * 9 * 16, hipMemcpyHostToDevice);
    /* unit links, no U(1) field, kappa = 1/8 (4 + m0 = 4), periodic in every direction: C = 0 */
    dirac_params p = {{L, L, L, L}, 0.125, 1.0, 1.0, 1, {0.0, 0.0, 0.0, 0.0}};
    dirac_ctx *ctx = NULL;
    if (dirac_create(&p, dU, NULL, NULL, &ctx) != DIRAC_OK) return fail("dirac_create");
    /* point source at x = 0, spin 0, colour 1 */
    psi[0 * 12 + 0 * 3 + 1] = 1.0;
    hipMemcpy(dpsi, psi, (size_t)V * 192, hipMemcpyHostToDevice);
    if (dirac_apply(ctx, dout, dpsi, DIRAC_F64, DIRAC_LAYOUT_LEX, 0, NULL) != DIRAC_OK) return fail("dirac_apply");
    hipDeviceSynchronize();
    hipMemcpy(out, dout, (size_t)V * 192, hipMemcpyDeviceToHost);
    /* D psi(y) = 4 psi(y) - 1/2 sum_mu [(1 - g_mu) psi(y + mu) + (1 + g_mu) psi(y - mu)]: the source
     * spinor e_0 (colour 1) appears at y = 0 (4 e_0), at y = -mu (-(1 - g_mu) e_0 / 2) and at
     * y = +mu (-(1 + g_mu) e_0 / 2).  Column 0 of the chiral gamma matrices has one entry:
     * g_0 e_0 = -e_2 (lower-left block -1), g_1 e_0 = i e_3 (i sigma_1), g_2 e_0 = -e_3
     * (i sigma_2 = [[0, 1], [-1, 0]]), g_3 e_0 = i e_2 (i sigma_3). */
    const int grow[4] = {2, 3, 3, 2};
    const double complex gval[4] = {-1.0, I, -1.0, I};
    want[0][0 * 3 + 1] = 4.0;
    const int stride[4] = {L * L * L, L * L, L, 1};
    for (int mu = 0; mu < 4; ++mu) {
        const int yp = stride[mu], ym = (L - 1) * stride[mu];  /* y = +mu and y = -mu (periodic) */
        want[ym][0 * 3 + 1] += -0.5;
        want[ym][grow[mu] * 3 + 1] += 0.5 * gval[mu];   /* -(1/2)(1 - g) e_0 */
        want[yp][0 * 3 + 1] += -0.5;
        want[yp][grow[mu] * 3 + 1] += -0.5 * gval[mu];  /* -(1/2)(1 + g) e_0 */
    }
    double maxerr = 0.0;
    for (int y = 0; y < V; ++y)
        for (int k = 0; k < 12; ++k) {
            const double e = cabs(out[(size_t)y * 12 + k] - want[y][k]);
            if (e > maxerr) maxerr = e;
        }
    printf("free-field point source: max |D psi - hand-written| = %.3e\n", maxerr);
    if (maxerr > 1e-15) return fail("free-field values");
    /* an aliased output is refused with DIRAC_EINVAL and a message */
    if (dirac_apply(ctx, dpsi, dpsi, DIRAC_F64, DIRAC_LAYOUT_LEX, 0, NULL) != DIRAC_EINVAL) return fail("aliasing");
    if (strlen(dirac_last_error()) == 0) return fail("empty error message");
    if (dirac_destroy(ctx) != DIRAC_OK) return fail("dirac_destroy");
    hipFree(dU);
    hipFree(dpsi);
    hipFree(dout);
    free(U);
    free(psi);
    free(out);
    printf("C ABI OK\n");
    return 0;
}
