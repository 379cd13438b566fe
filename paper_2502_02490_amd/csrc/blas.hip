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
// The same load with a streaming hint: for the Krylov basis vectors, which a kernel reads once
// (so they do not push the vectors it writes and reads back out of L2).
template <typename S>
DEV void ld_basis(const typename St<S>::vec *p, int t, int vh, double *o) {
    uint32_t i;
    const typename St<S>::vec *b = blk_base<S>(p, t, vh, i);
    typename St<S>::acc r[24];
    load_planes_h<S, 24, true>(b, 24 / St<S>::W, 0, i, r);
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

// A batch of nrhs independent systems: vector r of an argument v is v + r * vs (vs = the
// vector length in 16-byte units), basis vector j of system r is Q + (j * nrhs + r) * vs;
// system r's device scalars start r * sstride doubles after a scalar pointer.  Work-group b
// works on system b / nb; systems whose `active` flag is 0 are skipped entirely.
struct Bat {
    int n, vh, nb, nrhs, sstride;
    const int *active;
};

template <typename S>
DEV size_t vstride(const Bat &b) {
    return (size_t)(b.n / b.vh) * (24 / St<S>::W) * (size_t)padded_sites(b.vh);
}
DEV bool sys_of(const Bat &b, int &r, int &t) {
    r = blockIdx.x / b.nb;
    t = (blockIdx.x - r * b.nb) * kRed + threadIdx.x;
    return !b.active || b.active[r];
}

// partials[sys][blk][j] (complex) = sum over the group's sites of <Q_j, q>, j < k
template <typename S>
__global__ __launch_bounds__(kRed) void k_mdot(Bat B, const typename St<S>::vec *Q, int k,
                                               const typename St<S>::vec *q, double2 *partials) {
    __shared__ double lds[2 * kRed / 64];
    int r, t;
    if (!sys_of(B, r, t)) return;
    const size_t vs = vstride<S>(B);
    q += r * vs;
    double a[24];
    const bool on = t < B.n;
    if (on) ld<S>(q, t, B.vh, a);
    for (int j = 0; j < k; ++j) {
        double v[2] = {0.0, 0.0};
        if (on) {
            double b[24];
            ld_basis<S>(Q + ((size_t)j * B.nrhs + r) * vs, t, B.vh, b);
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

// out_r[j] = scale * sum_b partials[r][b][j] (b ascending), nc doubles per entry; grid (nent, nrhs)
__global__ __launch_bounds__(kRed) void k_reduce(int nblk, int nent, int nc, const double *partials, double scale,
                                                 double *out, int sstride, const int *active) {
    __shared__ double lds[4 * kRed / 64];
    const int j = blockIdx.x, r = blockIdx.y;
    if (active && !active[r]) return;
    partials += (size_t)r * nblk * nent * nc;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += kRed)
        for (int c = 0; c < nc; ++c) v[c] += partials[((size_t)b * nent + j) * nc + c];
    group_sum<4>(v, lds);
    if (threadIdx.x == 0)
        for (int c = 0; c < nc; ++c) out[(size_t)r * sstride + j * nc + c] = scale * v[c];
}

// q -= sum_j coef_j Q_j (coef complex double in device memory); partials: |q|^2, <q, r>
template <typename S>
__global__ __launch_bounds__(kRed) void k_maxpy_dot(Bat B, const typename St<S>::vec *Q, int k, const double *coef,
                                                    typename St<S>::vec *q, const typename St<S>::vec *rv,
                                                    double *partials) {
    __shared__ double lds[3 * kRed / 64];
    int r, t;
    if (!sys_of(B, r, t)) return;
    const size_t vs = vstride<S>(B);
    q += r * vs;
    rv += r * vs;
    const double2 *cf = reinterpret_cast<const double2 *>(coef + (size_t)r * B.sstride);
    double v[3] = {0.0, 0.0, 0.0};
    if (t < B.n) {
        double a[24], b[24];
        ld<S>(q, t, B.vh, a);
        for (int j = 0; j < k; ++j) {
            const double2 cj = cf[j];
            ld_basis<S>(Q + ((size_t)j * B.nrhs + r) * vs, t, B.vh, b);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                a[2 * c] -= cj.x * b[2 * c] - cj.y * b[2 * c + 1];
                a[2 * c + 1] -= cj.x * b[2 * c + 1] + cj.y * b[2 * c];
            }
        }
        st<S>(q, t, B.vh, a);
        ld<S>(q, t, B.vh, a);  // the stored (rounded) q is what the recurrence uses
        ld<S>(rv, t, B.vh, b);
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

// q_hat = q / gamma -> q; r -= alpha q_hat; pnext = r (if given); partial |r|^2.
// sc = {1/gamma, alpha.re, alpha.im} in device memory.
template <typename S>
__global__ __launch_bounds__(kRed) void k_gcr_update(Bat B, const double *sc, typename St<S>::vec *q,
                                                     typename St<S>::vec *rv, typename St<S>::vec *pnext,
                                                     double *partials) {
    __shared__ double lds[kRed / 64];
    int r, t;
    if (!sys_of(B, r, t)) return;
    const size_t vs = vstride<S>(B);
    q += r * vs;
    rv += r * vs;
    if (pnext) pnext += r * vs;
    sc += (size_t)r * B.sstride;
    double v[1] = {0.0};
    if (t < B.n) {
        const double ig = sc[0], ar = sc[1], ai = sc[2];
        double a[24], b[24];
        ld<S>(q, t, B.vh, a);
#pragma unroll
        for (int c = 0; c < 24; ++c) a[c] *= ig;
        st<S>(q, t, B.vh, a);
        ld<S>(q, t, B.vh, a);
        ld<S>(rv, t, B.vh, b);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            b[2 * c] -= ar * a[2 * c] - ai * a[2 * c + 1];
            b[2 * c + 1] -= ar * a[2 * c + 1] + ai * a[2 * c];
        }
        st<S>(rv, t, B.vh, b);
        if (pnext) st<S>(pnext, t, B.vh, b);
        ld<S>(rv, t, B.vh, b);
#pragma unroll
        for (int c = 0; c < 24; ++c) v[0] += b[c] * b[c];
    }
    group_sum<1>(v, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = v[0];
}

// x += xscale_r sum_j coef_j P_j (x and P may have different precisions)
template <typename SX, typename SP>
__global__ __launch_bounds__(kRed) void k_axpy_multi(Bat B, typename St<SX>::vec *x, const typename St<SP>::vec *P,
                                                     int k, const double *coef, double xscale,
                                                     const double *xscales, const int *kcount) {
    int r, t;
    if (!sys_of(B, r, t) || t >= B.n) return;
    x += r * vstride<SX>(B);
    const size_t vp = vstride<SP>(B);
    const double2 *cf = reinterpret_cast<const double2 *>(coef + (size_t)r * B.sstride);
    const double xs = xscales ? xscales[(size_t)r * B.sstride] : xscale;
    // a system's own count of basis vectors: those past it were not written in this cycle
    const int kr = kcount ? min(k, kcount[r]) : k;
    double a[24], b[24];
    ld<SX>(x, t, B.vh, a);
    for (int j = 0; j < kr; ++j) {
        const double2 cj = cf[j];
        ld_basis<SP>(P + ((size_t)j * B.nrhs + r) * vp, t, B.vh, b);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            a[2 * c] += xs * (cj.x * b[2 * c] - cj.y * b[2 * c + 1]);
            a[2 * c + 1] += xs * (cj.x * b[2 * c + 1] + cj.y * b[2 * c]);
        }
    }
    st<SX>(x, t, B.vh, a);
}

// out = alpha_r a + beta b (converted to the output precision); optional copy2 = out; partial |out|^2
// and a non-finite flag.  alpha_r = alphas[r * sstride] when alphas is given.
template <typename SO, typename SA, typename SB>
__global__ __launch_bounds__(kRed) void k_lincomb(Bat B, typename St<SO>::vec *out, typename St<SO>::vec *copy2,
                                                  double alpha, const double *alphas, const typename St<SA>::vec *a,
                                                  double beta, const typename St<SB>::vec *b, double *partials) {
    __shared__ double lds[2 * kRed / 64];
    int r, t;
    if (!sys_of(B, r, t)) return;
    out += r * vstride<SO>(B);
    if (copy2) copy2 += r * vstride<SO>(B);
    a += r * vstride<SA>(B);
    if (b) b += r * vstride<SB>(B);
    const double al = alphas ? alphas[(size_t)r * B.sstride] : alpha;
    double v[2] = {0.0, 0.0};
    if (t < B.n) {
        double x[24], y[24];
        ld<SA>(a, t, B.vh, x);
        if (b) {
            ld<SB>(b, t, B.vh, y);
#pragma unroll
            for (int c = 0; c < 24; ++c) x[c] = al * x[c] + beta * y[c];
        } else {
#pragma unroll
            for (int c = 0; c < 24; ++c) x[c] = al * x[c];
        }
        st<SO>(out, t, B.vh, x);
        if (copy2) st<SO>(copy2, t, B.vh, x);
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

// GCR scalars after k_maxpy_dot, per system r (thread r): red = {|q|^2, re <q,r>, im <q,r>};
// out: sc = {1/gamma, alpha}, gamma_k and alpha_k stored at slot k
__global__ void k_gcr_scalars(int nrhs, int sstride, const int *active, const double *red, double *sc, double *gam,
                              double *alp, int k) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs || (active && !active[r])) return;
    const size_t o = (size_t)r * sstride;
    const double n2 = red[o];
    const double g = sqrt(n2);
    const double ig = g > 0.0 ? 1.0 / g : 0.0;
    const double ar = red[o + 1] * ig, ai = red[o + 2] * ig;  // <q_hat, r>
    sc[o] = ig;
    sc[o + 1] = ar;
    sc[o + 2] = ai;
    gam[o + k] = g;
    alp[o + 2 * k] = ar;
    alp[o + 2 * k + 1] = ai;
}

__global__ void k_set(double *p, double v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = v;
}
__global__ void k_copy_scalar(const double *src, double *dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = src[0];
}

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

void Blas::reserve(int64_t nsites_max, int kmax, int nrhs) {
    const size_t nb = (size_t)blas_grid(nsites_max);
    part.alloc(nb * (size_t)nrhs * (size_t)std::max(kmax, 4) * 2 * sizeof(double) + 64);
    scal.alloc((size_t)std::max(nrhs, 1) * kSysScal * sizeof(double));
}

namespace {
Bat make_bat(const dirac_ctx *c, int nh, const BatchSpec &bs) {
    Bat b;
    b.vh = (int)c->vh;
    b.n = nh * b.vh;
    b.nb = blas_grid(b.n);
    b.nrhs = bs.nrhs;
    b.sstride = bs.sstride;
    b.active = bs.active;
    return b;
}
}  // namespace

void Blas::mdot(dirac_prec pr, int nh, const void *Q, int k, const void *q, double *out_dev, double scale,
                hipStream_t s, const BatchSpec &bs) {
    const Bat b = make_bat(c, nh, bs);
#define FN(S)                                                                                        \
    k_mdot<S><<<b.nb * b.nrhs, kRed, 0, s>>>(b, (const typename St<S>::vec *)Q, k,                    \
                                             (const typename St<S>::vec *)q, (double2 *)part.p);
    DISPATCH_PREC(pr, FN)
#undef FN
    k_reduce<<<dim3(k, b.nrhs), kRed, 0, s>>>(b.nb, k, 2, (const double *)part.p, scale, out_dev, b.sstride,
                                              b.active);
    HIP_CHECK(hipGetLastError());
}

void Blas::maxpy_dot(dirac_prec pr, int nh, const void *Q, int k, const double *coef_dev, void *q, const void *r,
                     double *out_dev, double scale, hipStream_t s, const BatchSpec &bs) {
    const Bat b = make_bat(c, nh, bs);
#define FN(S)                                                                                            \
    k_maxpy_dot<S><<<b.nb * b.nrhs, kRed, 0, s>>>(b, (const typename St<S>::vec *)Q, k, coef_dev,         \
                                                  (typename St<S>::vec *)q, (const typename St<S>::vec *)r, \
                                                  (double *)part.p);
    DISPATCH_PREC(pr, FN)
#undef FN
    k_reduce<<<dim3(1, b.nrhs), kRed, 0, s>>>(b.nb, 1, 3, (const double *)part.p, scale, out_dev, b.sstride,
                                              b.active);
    HIP_CHECK(hipGetLastError());
}

void Blas::gcr_scalars(const double *red, double *sc, double *gam, double *alp, int k, hipStream_t s,
                       const BatchSpec &bs) {
    k_gcr_scalars<<<(bs.nrhs + 63) / 64, 64, 0, s>>>(bs.nrhs, bs.sstride, bs.active, red, sc, gam, alp, k);
    HIP_CHECK(hipGetLastError());
}

void Blas::gcr_update(dirac_prec pr, int nh, const double *sc, void *q, void *r, void *pnext, double *out_dev,
                      double scale, hipStream_t s, const BatchSpec &bs) {
    const Bat b = make_bat(c, nh, bs);
#define FN(S)                                                                                                   \
    k_gcr_update<S><<<b.nb * b.nrhs, kRed, 0, s>>>(b, sc, (typename St<S>::vec *)q, (typename St<S>::vec *)r,    \
                                                   (typename St<S>::vec *)pnext, (double *)part.p);
    DISPATCH_PREC(pr, FN)
#undef FN
    k_reduce<<<dim3(1, b.nrhs), kRed, 0, s>>>(b.nb, 1, 1, (const double *)part.p, scale, out_dev, b.sstride,
                                              b.active);
    HIP_CHECK(hipGetLastError());
}

void Blas::axpy_multi(dirac_prec px, dirac_prec pp, int nh, void *x, const void *P, int k, const double *coef_dev,
                      double xscale, hipStream_t s, const BatchSpec &bs, const double *xscales, const int *kcount) {
    const Bat b = make_bat(c, nh, bs);
#define FN2(SX, SP)                                                                                              \
    k_axpy_multi<SX, SP><<<b.nb * b.nrhs, kRed, 0, s>>>(b, (typename St<SX>::vec *)x,                             \
                                                        (const typename St<SP>::vec *)P, k, coef_dev, xscale,     \
                                                        xscales, kcount);
#define FN(SP)                                                                                     \
    if (px == DIRAC_F64) { FN2(double, SP) } else if (px == DIRAC_F32) { FN2(float, SP) }          \
    else if (px == DIRAC_F16) { FN2(__half, SP) } else { FN2(__hip_bfloat16, SP) }
    DISPATCH_PREC(pp, FN)
#undef FN
#undef FN2
    HIP_CHECK(hipGetLastError());
}

// out = alpha a + beta b (b may be NULL), copy2 = out if given; writes scale |out|^2 and a
// non-finite flag into out_dev[0..1] when out_dev is given.
void Blas::lincomb(dirac_prec po, dirac_prec pa, dirac_prec pb, int nh, void *out, void *copy2, double alpha,
                   const void *a, double beta, const void *b, double *out_dev, double scale, hipStream_t s,
                   const BatchSpec &bs, const double *alphas) {
    const Bat bt = make_bat(c, nh, bs);
    double *pp = out_dev ? (double *)part.p : nullptr;
#define FN3(SO, SA, SB)                                                                                           \
    k_lincomb<SO, SA, SB><<<bt.nb * bt.nrhs, kRed, 0, s>>>(bt, (typename St<SO>::vec *)out,                       \
                                                           (typename St<SO>::vec *)copy2, alpha, alphas,          \
                                                           (const typename St<SA>::vec *)a, beta,                 \
                                                           (const typename St<SB>::vec *)b, pp);
    if (po == pa && pa == pb) {
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
    if (out_dev)
        k_reduce<<<dim3(1, bt.nrhs), kRed, 0, s>>>(bt.nb, 1, 2, (const double *)part.p, scale, out_dev, bt.sstride,
                                                   bt.active);
    HIP_CHECK(hipGetLastError());
}

void Blas::cgls_xs(int nh, const double *rho, const double *wn, void *x, const void *p, void *sv, const void *w,
                   double *out_dev, hipStream_t s) {
    const int vh = (int)c->vh, n = nh * vh, nb = blas_grid(n);
    k_cgls_xs<double><<<nb, kRed, 0, s>>>(n, vh, rho, wn, (double2 *)x, (const double2 *)p, (double2 *)sv,
                                          (const double2 *)w, (double *)part.p);
    k_reduce<<<dim3(1, 1), kRed, 0, s>>>(nb, 1, 1, (const double *)part.p, 1.0, out_dev, 0, nullptr);
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
