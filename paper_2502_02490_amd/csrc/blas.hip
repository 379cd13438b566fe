// Vector kernels of the Krylov solvers on NATIVE vectors (one thread per site, 24 reals).
// Every reduction accumulates in FP64 and is deterministic: each work-group reduces its sites
// in a fixed tree and writes one partial; a second kernel sums the partials in index order.
// No floating-point atomics anywhere.
//
// A "vector" here is nh consecutive half-lattice blocks (nh = 1 for an even-odd vector, 2 for
// a full-lattice vector): block h starts h * 24 vh reals after the base and holds 24 / W planes
// of vh sites.
#include "blas.h"

#include <algorithm>

namespace dl {
namespace {

constexpr int kRed = 256;  // work-group size of the reducing kernels

// (half h, base) of site t of an nh-half vector; halves are 24 / W planes of vhp sites apart
template <typename S>
DEV const typename St<S>::vec *blk_base(const typename St<S>::vec *p, int t, int vh, uint32_t &i) {
    const int h = t >= vh;
    i = (uint32_t)(t - h * vh);
    return p + (size_t)h * (24 / St<S>::W) * (size_t)padded_sites(vh);
}
template <typename S>
DEV typename St<S>::vec *blk_base(typename St<S>::vec *p, int t, int vh, uint32_t &i) {
    const int h = t >= vh;
    i = (uint32_t)(t - h * vh);
    return p + (size_t)h * (24 / St<S>::W) * (size_t)padded_sites(vh);
}

template <typename S>
DEV void ld(const typename St<S>::vec *p, int t, int vh, double *o) {
    uint32_t i;
    const typename St<S>::vec *b = blk_base<S>(p, t, vh, i);
    typename St<S>::acc r[24];
    load_field<S, 24>(b, i, r);
#pragma unroll
    for (int k = 0; k < 24; ++k) o[k] = (double)r[k];
}
template <typename S>
DEV void st(typename St<S>::vec *p, int t, int vh, const double *o) {
    uint32_t i;
    typename St<S>::vec *b = blk_base<S>(p, t, vh, i);
    typename St<S>::acc r[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) r[k] = (typename St<S>::acc)o[k];
    store_field<S, 24>(b, i, r);
}

// Sum of v over the work-group (fixed tree: wave shuffles, then the waves in order).
template <int N>
DEV void group_sum(double v[N], double *lds /* [N][kRed / 64] */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) lds[k * (kRed / 64) + wave] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < kRed / 64; ++w) s += lds[k * (kRed / 64) + w];
            v[k] = s;
        }
    }
}

// partials[blk][j] (complex) = sum over the group's sites of <Q_j, q>, j < k
template <typename S>
__global__ __launch_bounds__(kRed) void k_mdot(int n, int vh, const typename St<S>::vec *Q, size_t qstride, int k,
                                               const typename St<S>::vec *q, double2 *partials) {
    __shared__ double lds[2 * kRed / 64];
    const int t = blockIdx.x * kRed + threadIdx.x;
    double a[24];
    const bool on = t < n;
    if (on) ld<S>(q, t, vh, a);
    for (int j = 0; j < k; ++j) {
        double v[2] = {0.0, 0.0};
        if (on) {
            double b[24];
            ld<S>(Q + j * qstride, t, vh, b);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                v[0] = fma(b[2 * c], a[2 * c], v[0]);
                v[0] = fma(b[2 * c + 1], a[2 * c + 1], v[0]);
                v[1] = fma(b[2 * c], a[2 * c + 1], v[1]);
                v[1] = fma(-b[2 * c + 1], a[2 * c], v[1]);
            }
        }
        group_sum<2>(v, lds);
        if (threadIdx.x == 0) partials[(size_t)blockIdx.x * k + j] = make_double2(v[0], v[1]);
        __syncthreads();
    }
}

// out[j] = scale * sum_b partials[b][j] (b ascending), nc doubles per entry
__global__ __launch_bounds__(kRed) void k_reduce(int nblk, int nent, int nc, const double *partials, double scale,
                                                 double *out) {
    __shared__ double lds[4 * kRed / 64];
    const int j = blockIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += kRed)
        for (int c = 0; c < nc; ++c) v[c] += partials[((size_t)b * nent + j) * nc + c];
    group_sum<4>(v, lds);
    if (threadIdx.x == 0)
        for (int c = 0; c < nc; ++c) out[j * nc + c] = scale * v[c];
}

// q -= sum_j coef_j Q_j (coef complex double in device memory); partials: |q|^2, <q, r>
template <typename S>
__global__ __launch_bounds__(kRed) void k_maxpy_dot(int n, int vh, const typename St<S>::vec *Q, size_t qstride,
                                                    int k, const double2 *coef, typename St<S>::vec *q,
                                                    const typename St<S>::vec *r, double *partials) {
    __shared__ double lds[3 * kRed / 64];
    const int t = blockIdx.x * kRed + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    if (t < n) {
        double a[24], b[24];
        ld<S>(q, t, vh, a);
        for (int j = 0; j < k; ++j) {
            const double2 cj = coef[j];
            ld<S>(Q + j * qstride, t, vh, b);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                a[2 * c] -= cj.x * b[2 * c] - cj.y * b[2 * c + 1];
                a[2 * c + 1] -= cj.x * b[2 * c + 1] + cj.y * b[2 * c];
            }
        }
        st<S>(q, t, vh, a);
        ld<S>(q, t, vh, a);  // the stored (rounded) q is what the recurrence uses
        ld<S>(r, t, vh, b);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            v[0] += a[2 * c] * a[2 * c] + a[2 * c + 1] * a[2 * c + 1];
            v[1] += a[2 * c] * b[2 * c] + a[2 * c + 1] * b[2 * c + 1];
            v[2] += a[2 * c] * b[2 * c + 1] - a[2 * c + 1] * b[2 * c];
        }
    }
    group_sum<3>(v, lds);
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) partials[(size_t)blockIdx.x * 3 + c] = v[c];
}

// q_hat = q / gamma -> qout; r -= alpha q_hat; pnext = r (if given); partial |r|^2.
// sc = {1/gamma, alpha.re, alpha.im} in device memory.
template <typename S>
__global__ __launch_bounds__(kRed) void k_gcr_update(int n, int vh, const double *sc, typename St<S>::vec *q,
                                                     typename St<S>::vec *r, typename St<S>::vec *pnext,
                                                     double *partials) {
    __shared__ double lds[kRed / 64];
    const int t = blockIdx.x * kRed + threadIdx.x;
    double v[1] = {0.0};
    if (t < n) {
        const double ig = sc[0], ar = sc[1], ai = sc[2];
        double a[24], b[24];
        ld<S>(q, t, vh, a);
#pragma unroll
        for (int c = 0; c < 24; ++c) a[c] *= ig;
        st<S>(q, t, vh, a);
        ld<S>(q, t, vh, a);
        ld<S>(r, t, vh, b);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            b[2 * c] -= ar * a[2 * c] - ai * a[2 * c + 1];
            b[2 * c + 1] -= ar * a[2 * c + 1] + ai * a[2 * c];
        }
        st<S>(r, t, vh, b);
        if (pnext) st<S>(pnext, t, vh, b);
        ld<S>(r, t, vh, b);
#pragma unroll
        for (int c = 0; c < 24; ++c) v[0] += b[c] * b[c];
    }
    group_sum<1>(v, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = v[0];
}

// x += sum_j coef_j P_j (x and P may have different precisions)
template <typename SX, typename SP>
__global__ __launch_bounds__(kRed) void k_axpy_multi(int n, int vh, typename St<SX>::vec *x,
                                                     const typename St<SP>::vec *P, size_t pstride, int k,
                                                     const double2 *coef, double xscale) {
    const int t = blockIdx.x * kRed + threadIdx.x;
    if (t >= n) return;
    double a[24], b[24];
    ld<SX>(x, t, vh, a);
    for (int j = 0; j < k; ++j) {
        const double2 cj = coef[j];
        ld<SP>(P + j * pstride, t, vh, b);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            a[2 * c] += xscale * (cj.x * b[2 * c] - cj.y * b[2 * c + 1]);
            a[2 * c + 1] += xscale * (cj.x * b[2 * c + 1] + cj.y * b[2 * c]);
        }
    }
    st<SX>(x, t, vh, a);
}

// out = alpha a + beta b (converted to the output precision); optional copy2 = out; partial |out|^2
template <typename SO, typename SA, typename SB>
__global__ __launch_bounds__(kRed) void k_lincomb(int n, int vh, typename St<SO>::vec *out,
                                                  typename St<SO>::vec *copy2, double alpha,
                                                  const typename St<SA>::vec *a, double beta,
                                                  const typename St<SB>::vec *b, double *partials) {
    __shared__ double lds[2 * kRed / 64];
    const int t = blockIdx.x * kRed + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (t < n) {
        double x[24], y[24];
        ld<SA>(a, t, vh, x);
        if (b) {
            ld<SB>(b, t, vh, y);
#pragma unroll
            for (int c = 0; c < 24; ++c) x[c] = alpha * x[c] + beta * y[c];
        } else {
#pragma unroll
            for (int c = 0; c < 24; ++c) x[c] = alpha * x[c];
        }
        st<SO>(out, t, vh, x);
        if (copy2) st<SO>(copy2, t, vh, x);
        bool fin = true;
#pragma unroll
        for (int c = 0; c < 24; ++c) {
            v[0] += x[c] * x[c];
            fin = fin && isfinite(x[c]);
        }
        v[1] = fin ? 0.0 : 1.0;
    }
    if (partials) {
        group_sum<2>(v, lds);
        if (threadIdx.x == 0) {
            partials[(size_t)blockIdx.x * 2] = v[0];
            partials[(size_t)blockIdx.x * 2 + 1] = v[1];
        }
    }
}

// CG-style update for CGLS: x += alpha p; s -= alpha w (alpha = num / den from device scalars)
template <typename S>
__global__ __launch_bounds__(kRed) void k_cgls_xs(int n, int vh, const double *rho, const double *wn,
                                                  typename St<S>::vec *x, const typename St<S>::vec *p,
                                                  typename St<S>::vec *s, const typename St<S>::vec *w,
                                                  double *partials) {
    __shared__ double lds[kRed / 64];
    const int t = blockIdx.x * kRed + threadIdx.x;
    double v[1] = {0.0};
    if (t < n) {
        const double alpha = rho[0] / wn[0];
        double a[24], b[24];
        ld<S>(x, t, vh, a);
        ld<S>(p, t, vh, b);
#pragma unroll
        for (int c = 0; c < 24; ++c) a[c] += alpha * b[c];
        st<S>(x, t, vh, a);
        ld<S>(s, t, vh, a);
        ld<S>(w, t, vh, b);
#pragma unroll
        for (int c = 0; c < 24; ++c) {
            a[c] -= alpha * b[c];
            v[0] += a[c] * a[c];
        }
        st<S>(s, t, vh, a);
    }
    group_sum<1>(v, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = v[0];
}

// p = r + (rho_new / rho_old) p
template <typename S>
__global__ __launch_bounds__(kRed) void k_cgls_p(int n, int vh, const double *rho_new, const double *rho_old,
                                                 typename St<S>::vec *p, const typename St<S>::vec *r) {
    const int t = blockIdx.x * kRed + threadIdx.x;
    if (t >= n) return;
    const double beta = rho_new[0] / rho_old[0];
    double a[24], b[24];
    ld<S>(p, t, vh, a);
    ld<S>(r, t, vh, b);
#pragma unroll
    for (int c = 0; c < 24; ++c) a[c] = b[c] + beta * a[c];
    st<S>(p, t, vh, a);
}

// GCR scalars after k_maxpy_dot: red = {|q|^2, re <q,r>, im <q,r>}
// out: sc = {1/gamma, alpha}, gamma_k, alpha_k stored at slot k
__global__ void k_gcr_scalars(const double *red, double *sc, double *gam, double2 *alp, int k) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double n2 = red[0];
    const double g = sqrt(n2);
    const double ig = g > 0.0 ? 1.0 / g : 0.0;
    const double ar = red[1] * ig, ai = red[2] * ig;  // <q_hat, r>
    sc[0] = ig;
    sc[1] = ar;
    sc[2] = ai;
    gam[k] = g;
    alp[k] = make_double2(ar, ai);
}

__global__ void k_set(double *p, double v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = v;
}
__global__ void k_copy_scalar(const double *src, double *dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = src[0];
}

template <typename S> struct Tag {};

}  // namespace

// ------------------------------------------------------------------ host wrappers
int blas_grid(int64_t nsites) { return (int)((nsites + kRed - 1) / kRed); }

#define DISPATCH_PREC(pr, FN)                                                              \
    switch (pr) {                                                                          \
        case DIRAC_F64: FN(double); break;                                                 \
        case DIRAC_F32: FN(float); break;                                                  \
        case DIRAC_F16: FN(__half); break;                                                 \
        case DIRAC_BF16: FN(__hip_bfloat16); break;                                        \
        default: throw Error(DIRAC_EINVAL, "unknown precision");                           \
    }

void Blas::reserve(int64_t nsites_max, int kmax) {
    const size_t nb = (size_t)blas_grid(nsites_max);
    part.alloc(nb * (size_t)std::max(kmax, 4) * 2 * sizeof(double) + 64);
    scal.alloc(16384 * sizeof(double));
}

void Blas::mdot(dirac_prec pr, int nh, const void *Q, size_t qstride_bytes, int k, const void *q, double *out_dev,
                double scale, hipStream_t s) {
    const int vh = (int)c->vh, n = nh * vh, nb = blas_grid(n);
#define FN(S)                                                                                         \
    k_mdot<S><<<nb, kRed, 0, s>>>(n, vh, (const typename St<S>::vec *)Q,                              \
                                  qstride_bytes / sizeof(typename St<S>::vec), k,                    \
                                  (const typename St<S>::vec *)q, (double2 *)part.p);
    DISPATCH_PREC(pr, FN)
#undef FN
    k_reduce<<<k, kRed, 0, s>>>(nb, k, 2, (const double *)part.p, scale, out_dev);
    HIP_CHECK(hipGetLastError());
}

void Blas::maxpy_dot(dirac_prec pr, int nh, const void *Q, size_t qstride_bytes, int k, const double *coef_dev,
                     void *q, const void *r, double *out_dev, double scale, hipStream_t s) {
    const int vh = (int)c->vh, n = nh * vh, nb = blas_grid(n);
#define FN(S)                                                                                               \
    k_maxpy_dot<S><<<nb, kRed, 0, s>>>(n, vh, (const typename St<S>::vec *)Q,                               \
                                       qstride_bytes / sizeof(typename St<S>::vec), k,                      \
                                       (const double2 *)coef_dev, (typename St<S>::vec *)q,                 \
                                       (const typename St<S>::vec *)r, (double *)part.p);
    DISPATCH_PREC(pr, FN)
#undef FN
    k_reduce<<<1, kRed, 0, s>>>(nb, 1, 3, (const double *)part.p, scale, out_dev);
    HIP_CHECK(hipGetLastError());
}

void Blas::gcr_scalars(const double *red, double *sc, double *gam, double *alp, int k, hipStream_t s) {
    k_gcr_scalars<<<1, 1, 0, s>>>(red, sc, gam, (double2 *)alp, k);
    HIP_CHECK(hipGetLastError());
}

void Blas::gcr_update(dirac_prec pr, int nh, const double *sc, void *q, void *r, void *pnext, double *out_dev,
                      double scale, hipStream_t s) {
    const int vh = (int)c->vh, n = nh * vh, nb = blas_grid(n);
#define FN(S)                                                                                            \
    k_gcr_update<S><<<nb, kRed, 0, s>>>(n, vh, sc, (typename St<S>::vec *)q, (typename St<S>::vec *)r,    \
                                        (typename St<S>::vec *)pnext, (double *)part.p);
    DISPATCH_PREC(pr, FN)
#undef FN
    k_reduce<<<1, kRed, 0, s>>>(nb, 1, 1, (const double *)part.p, scale, out_dev);
    HIP_CHECK(hipGetLastError());
}

void Blas::axpy_multi(dirac_prec px, dirac_prec pp, int nh, void *x, const void *P, size_t pstride_bytes, int k,
                      const double *coef_dev, double xscale, hipStream_t s) {
    const int vh = (int)c->vh, n = nh * vh, nb = blas_grid(n);
#define FN2(SX, SP)                                                                                           \
    k_axpy_multi<SX, SP><<<nb, kRed, 0, s>>>(n, vh, (typename St<SX>::vec *)x, (const typename St<SP>::vec *)P, \
                                             pstride_bytes / sizeof(typename St<SP>::vec), k,                \
                                             (const double2 *)coef_dev, xscale);
#define FN(SP)                                                                                     \
    if (px == DIRAC_F64) { FN2(double, SP) } else if (px == DIRAC_F32) { FN2(float, SP) }          \
    else if (px == DIRAC_F16) { FN2(__half, SP) } else { FN2(__hip_bfloat16, SP) }
    DISPATCH_PREC(pp, FN)
#undef FN
#undef FN2
    HIP_CHECK(hipGetLastError());
}

// out = alpha a + beta b (b may be NULL), copy2 = out if given; returns |out|^2 * scale and a
// non-finite flag into out_dev[0..1] when out_dev is given.
void Blas::lincomb(dirac_prec po, dirac_prec pa, dirac_prec pb, int nh, void *out, void *copy2, double alpha,
                   const void *a, double beta, const void *b, double *out_dev, double scale, hipStream_t s) {
    const int vh = (int)c->vh, n = nh * vh, nb = blas_grid(n);
    double *pp = out_dev ? (double *)part.p : nullptr;
#define FN3(SO, SA, SB)                                                                                      \
    k_lincomb<SO, SA, SB><<<nb, kRed, 0, s>>>(n, vh, (typename St<SO>::vec *)out, (typename St<SO>::vec *)copy2, \
                                              alpha, (const typename St<SA>::vec *)a, beta,                  \
                                              (const typename St<SB>::vec *)b, pp);
    auto same = [&](dirac_prec x, dirac_prec y) { return x == y; };
    if (same(po, pa) && same(pa, pb)) {
#define FN(S) FN3(S, S, S)
        DISPATCH_PREC(po, FN)
#undef FN
    } else if (pa == DIRAC_F64 && pb == DIRAC_F64) {
#define FN(S) FN3(S, double, double)
        DISPATCH_PREC(po, FN)
#undef FN
    } else if (po == DIRAC_F64 && pb == DIRAC_F64) {
#define FN(S) FN3(double, S, double)
        DISPATCH_PREC(pa, FN)
#undef FN
    } else {
        throw Error(DIRAC_EUNSUPPORTED, "lincomb precision combination");
    }
#undef FN3
    if (out_dev) k_reduce<<<1, kRed, 0, s>>>(nb, 1, 2, (const double *)part.p, scale, out_dev);
    HIP_CHECK(hipGetLastError());
}

void Blas::cgls_xs(int nh, const double *rho, const double *wn, void *x, const void *p, void *sv, const void *w,
                   double *out_dev, hipStream_t s) {
    const int vh = (int)c->vh, n = nh * vh, nb = blas_grid(n);
    k_cgls_xs<double><<<nb, kRed, 0, s>>>(n, vh, rho, wn, (double2 *)x, (const double2 *)p, (double2 *)sv,
                                          (const double2 *)w, (double *)part.p);
    k_reduce<<<1, kRed, 0, s>>>(nb, 1, 1, (const double *)part.p, 1.0, out_dev);
    HIP_CHECK(hipGetLastError());
}

void Blas::cgls_p(int nh, const double *rho_new, const double *rho_old, void *p, const void *r, hipStream_t s) {
    const int vh = (int)c->vh, n = nh * vh, nb = blas_grid(n);
    k_cgls_p<double><<<nb, kRed, 0, s>>>(n, vh, rho_new, rho_old, (double2 *)p, (const double2 *)r);
    HIP_CHECK(hipGetLastError());
}

void Blas::set(double *p, double v, hipStream_t s) {
    k_set<<<1, 1, 0, s>>>(p, v);
    HIP_CHECK(hipGetLastError());
}
void Blas::copy_scalar(const double *src, double *dst, hipStream_t s) {
    k_copy_scalar<<<1, 1, 0, s>>>(src, dst);
    HIP_CHECK(hipGetLastError());
}

}  // namespace dl
