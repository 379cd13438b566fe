// Host interface of the solver vector kernels (blas.hip).  Reductions write their results
// (FP64, already summed over the lattice and multiplied by `scale`) to device memory, so a
// solver iteration needs no host round trip except where it reads a norm to decide.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "internal.h"

namespace dl {

// A batch of nrhs systems sharing one lattice: vector r of an argument is r vectors after its
// base, basis vector j of system r is (j * nrhs + r) vectors after the base, and system r's
// device scalars are r * sstride doubles after a scalar pointer.  Systems with active[r] = 0
// are skipped.  The default is one system.
struct BatchSpec {
    int nrhs = 1;
    const int *active = nullptr;
    int sstride = 0;
};

constexpr int kSysScal = 8768;  // device scalar doubles per system: GCR(64) coefficients and 64 free slots

struct Blas {
    dirac_ctx *c = nullptr;
    DevBuf part, scal;

    void reserve(int64_t nsites_max, int kmax, int nrhs = 1);
    // out[j] = scale <Q_j, q>, j < k (complex, 2 doubles each)
    void mdot(dirac_prec pr, int nh, const void *Q, int k, const void *q, double *out_dev, double scale, hipStream_t s,
              const BatchSpec &bs = BatchSpec());
    // q -= sum_j coef_j Q_j; out = scale {|q|^2, <q, r>}
    void maxpy_dot(dirac_prec pr, int nh, const void *Q, int k, const double *coef_dev, void *q, const void *r,
                   double *out_dev, double scale, hipStream_t s, const BatchSpec &bs = BatchSpec());
    void gcr_scalars(const double *red, double *sc, double *gam, double *alp, int k, hipStream_t s,
                     const BatchSpec &bs = BatchSpec());
    // q /= gamma; r -= alpha q; pnext = r; out = scale |r|^2
    void gcr_update(dirac_prec pr, int nh, const double *sc, void *q, void *r, void *pnext, double *out_dev,
                    double scale, hipStream_t s, const BatchSpec &bs = BatchSpec());
    // x += xscale sum_j coef_j P_j, j < k (xscale_r = xscales[r * sstride] when given; system r sums
    // only j < kcount[r] when kcount is given)
    void axpy_multi(dirac_prec px, dirac_prec pp, int nh, void *x, const void *P, int k, const double *coef_dev,
                    double xscale, hipStream_t s, const BatchSpec &bs = BatchSpec(), const double *xscales = nullptr,
                    const int *kcount = nullptr);
    // out = alpha a + beta b; copy2 = out; out_dev = scale {|out|^2, nonfinite flag}
    void lincomb(dirac_prec po, dirac_prec pa, dirac_prec pb, int nh, void *out, void *copy2, double alpha,
                 const void *a, double beta, const void *b, double *out_dev, double scale, hipStream_t s,
                 const BatchSpec &bs = BatchSpec(), const double *alphas = nullptr);
    void cgls_xs(int nh, const double *rho, const double *wn, void *x, const void *p, void *sv, const void *w,
                 double *out_dev, hipStream_t s);
    void cgls_p(int nh, const double *rho_new, const double *rho_old, void *p, const void *r, hipStream_t s);
    void set(double *p, double v, hipStream_t s);
    void copy_scalar(const double *src, double *dst, hipStream_t s);
};

int blas_grid(int64_t nsites);

// Solver work space of a context (solver.hip)
struct SolverWork {
    Blas blas;
    DevBuf P, Q, r, e, b;   // Krylov vectors, inner solution / right-hand side (solve precision)
    DevBuf h64[4];          // FP64 half vectors: eta-hat, x_e, r, tmp
    DevBuf ctl;             // device-side iteration control of a GCR cycle (solver.hip)
    DevBuf f64[3];          // FP64 full vectors: b, x, r
    int m = 0;
    dirac_prec pr = DIRAC_F64;
    long syncs = 0;  // host waits on the device (value reads) since the current solve began
};

}  // namespace dl
