// Field import and export: the user layouts of the boundary (LEX and EO site order,
// array-of-structs, paper Sec. 4.1) to and from the library's per-parity plane
// layout, link compression, and lower-precision copies of the operator fields.
#include <cstring>

#include "dirac_ops.h"
#include "internal.h"

namespace dl {
namespace {

// ------------------------------------------------------------------ links
// For site x of parity p (half index i) and direction mu:
//   dir 2 mu     : U_mu(x),        omega = qhat theta_mu(x) + phi_mu [x_mu = L_mu - 1]
//   dir 2 mu + 1 : U_mu(x - mu),   omega of that link (its x_mu is L_mu - 1 when x_mu = 0)
// Rows 0 and 1 of U are stored; row 2 is rebuilt as conj(row0 x row1) where used.
__global__ __launch_bounds__(kBlock) void k_import_links(Geom g, int p, const double *__restrict__ U,
                                                          const double *__restrict__ theta, int qhat,
                                                          double4 phase, double2 *__restrict__ planes,
                                                          double *__restrict__ omega,
                                                          unsigned long long *__restrict__ maxdev) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.vh) return;
    int x[4];
    site_coords(g, i, p, x);
    const double ph[4] = {phase.x, phase.y, phase.z, phase.w};
    const size_t vhp = (size_t)g.vhp;
    double dev = 0.0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
        for (int back = 0; back < 2; ++back) {
            int y[4] = {x[0], x[1], x[2], x[3]};
            if (back) {
                const bool cross = y[mu] == 0;
                y[mu] = wrap_dn(y[mu], g.L[mu]);
                y[1] = cstar_x1(g, mu, cross, y[1]);  // C*: the link behind x may sit in the mirror copy
            }
            const int lam = lex_index(g, y);
            const double *u = U + ((size_t)lam * 4 + mu) * 18;
            const int dir = 2 * mu + back;
            double2 *dst = site_ptr(planes + (size_t)dir * 6 * vhp, (uint32_t)i, 6);
#pragma unroll
            for (int k = 0; k < 6; ++k) dst[k * kSB] = make_double2(u[2 * k], u[2 * k + 1]);
            double w = (theta ? qhat * theta[(size_t)lam * 4 + mu] : 0.0) + (y[mu] == g.L[mu] - 1 ? ph[mu] : 0.0);
            omega[(size_t)dir * vhp + i] = w;
            if (!back) {
                // deviation from SU(3): max |U U^dag - 1| and |det U - 1|; the row-2 rebuild needs det U = 1
                cx<double> m[9];
#pragma unroll
                for (int k = 0; k < 9; ++k) m[k] = mk(u[2 * k], u[2 * k + 1]);
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        cx<double> s = mk(0.0, 0.0);
#pragma unroll
                        for (int k = 0; k < 3; ++k) s = s + m[3 * a + k] * conj(m[3 * b + k]);
                        if (a == b) s.r -= 1.0;
                        dev = fmax(dev, fabs(s.r) + fabs(s.i));
                    }
                cx<double> det = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
                                 m[2] * (m[3] * m[7] - m[4] * m[6]);
                dev = fmax(dev, fabs(det.r - 1.0) + fabs(det.i));
            }
        }
    }
    if (!(dev <= 1e300)) dev = 1e300;  // NaN input
    atomicMax(maxdev, (unsigned long long)__double_as_longlong(dev));
}

template <typename S>
__global__ __launch_bounds__(kBlock) void k_convert_links(int vh, int vhp, const double2 *__restrict__ src,
                                                           const double *__restrict__ om_src,
                                                           typename Lk<S>::vec *__restrict__ dst,
                                                           typename Lk<S>::om *__restrict__ om_dst) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= vh) return;
    constexpr int W = Lk<S>::W;
    const size_t n = (size_t)vhp;
    for (int dir = 0; dir < 8; ++dir) {
        double r[12];
        const double2 *s0 = site_ptr(src + (size_t)dir * 6 * n, (uint32_t)i, 6);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            double2 v = s0[k * kSB];
            r[2 * k] = v.x;
            r[2 * k + 1] = v.y;
        }
        typename Lk<S>::vec *d0 = site_ptr(dst + (size_t)dir * (12 / W) * n, (uint32_t)i, 12 / W);
#pragma unroll
        for (int k = 0; k < 12 / W; ++k) d0[k * kSB] = Lk<S>::pack(r + k * W);
        if constexpr (Lk<S>::phase_pair) {
            double si, co;
            sc(om_src[(size_t)dir * n + i], si, co);  // FP64, then rounded once to the 16-bit format
            om_dst[(size_t)dir * n + i] = Lk<S>::pack_phase((float)co, (float)si);
        } else {
            om_dst[(size_t)dir * n + i] = (typename Lk<S>::om)om_src[(size_t)dir * n + i];
        }
    }
}

// ------------------------------------------------------------------ clover (72 reals per site)
template <typename S>
__global__ __launch_bounds__(kBlock) void k_convert_clover(int vh, const double2 *__restrict__ src,
                                                            typename St<S>::vec *__restrict__ dst) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= vh) return;
    double r[72];
    load_field<double, 72>(src, i, r);
    typename St<S>::acc a[72];
#pragma unroll
    for (int k = 0; k < 72; ++k) a[k] = (typename St<S>::acc)r[k];
    store_field<S, 72>(dst, i, a);
}

// user index of the site (p, i): LEX -> Lambda, EO -> xhat, OPENQXD -> eq. (ipt) with the cache
// block (relative to the first site of the parity for half vectors)
DEV int64_t user_site(const Geom &g, int p, int i, int lay, int half) {
    if (lay == DIRAC_LAYOUT_LEX || lay == DIRAC_LAYOUT_OPENQXD) {
        int x[4];
        site_coords(g, i, p, x);
        if (lay == DIRAC_LAYOUT_LEX) return lex_index(g, x);
        const int64_t k = ipt_index(g, x);
        return half ? k - (int64_t)p * g.vh : k;
    }
    return half ? (int64_t)i : (int64_t)i + (int64_t)p * g.vh;
}

__global__ __launch_bounds__(kBlock) void k_clover_in(Geom g, int p, int lay, const double *__restrict__ user,
                                                       double2 *__restrict__ dst) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.vh) return;
    const double *u = user + user_site(g, p, i, lay, 0) * 72;
    double r[72];
#pragma unroll
    for (int k = 0; k < 72; ++k) r[k] = u[k];
    store_field<double, 72>(dst, i, r);
}

__global__ __launch_bounds__(kBlock) void k_clover_out(Geom g, int p, int lay, const double2 *__restrict__ src,
                                                        double *__restrict__ user) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.vh) return;
    double *u = user + user_site(g, p, i, lay, 0) * 72;
    double r[72];
    if (src) {
        load_field<double, 72>(src, i, r);
    } else {
#pragma unroll
        for (int k = 0; k < 72; ++k) r[k] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < 72; ++k) u[k] = r[k];
}

// ------------------------------------------------------------------ spinors (24 reals per site)
template <typename U, typename S>
__global__ __launch_bounds__(kBlock) void k_spinor_in(Geom g, int p, int lay, int half, const U *__restrict__ user,
                                                       typename St<S>::vec *__restrict__ dst) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.vh) return;
    const U *u = user + user_site(g, p, i, lay, half) * 24;
    typename St<S>::acc r[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) r[k] = (typename St<S>::acc)u[k];
    store_field<S, 24>(dst, i, r);
}

template <typename U, typename S>
__global__ __launch_bounds__(kBlock) void k_spinor_out(Geom g, int p, int lay, int half,
                                                        const typename St<S>::vec *__restrict__ src,
                                                        U *__restrict__ user) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.vh) return;
    U *u = user + user_site(g, p, i, lay, half) * 24;
    typename St<S>::acc r[24];
    load_field<S, 24>(src, i, r);
#pragma unroll
    for (int k = 0; k < 24; ++k) u[k] = (U)r[k];
}

template <typename S>
void convert_fields(dirac_ctx *c, dirac_prec pr, hipStream_t s) {
    PrecFields &lo = c->f[pr];
    PrecFields &hi = c->f[DIRAC_F64];
    const int vh = (int)c->vh;
    const size_t vhp = (size_t)c->g.vhp;
    if (!lo.links_ready) {
        for (int p = 0; p < 2; ++p) {
            lo.links[p].alloc((size_t)8 * 12 * sizeof(typename Lk<S>::vec) / Lk<S>::W * vhp);
            lo.omega[p].alloc((size_t)8 * sizeof(typename Lk<S>::om) * vhp);
            k_convert_links<S><<<grid_for(vh), kBlock, 0, s>>>(
                vh, (int)vhp, (const double2 *)hi.links[p].p, (const double *)hi.omega[p].p,
                (typename Lk<S>::vec *)lo.links[p].p, (typename Lk<S>::om *)lo.omega[p].p);
        }
        HIP_CHECK(hipGetLastError());
        lo.links_ready = true;
    }
    if (!lo.clover_ready) {
        for (int p = 0; p < 2; ++p) {
            lo.clov[p].alloc((size_t)72 * sizeof(S) * vhp);
            k_convert_clover<S><<<grid_for(vh), kBlock, 0, s>>>(vh, (const double2 *)hi.clov[p].p,
                                                                  (typename St<S>::vec *)lo.clov[p].p);
        }
        HIP_CHECK(hipGetLastError());
        lo.clover_ready = true;
    }
    for (int p = 0; p < 2; ++p) {
        if (hi.inv_ready[p] && !lo.inv_ready[p]) {
            lo.clinv[p].alloc((size_t)72 * sizeof(S) * vhp);
            k_convert_clover<S><<<grid_for(vh), kBlock, 0, s>>>(vh, (const double2 *)hi.clinv[p].p,
                                                                  (typename St<S>::vec *)lo.clinv[p].p);
            HIP_CHECK(hipGetLastError());
            lo.inv_ready[p] = true;
        }
    }
}

template <typename U, typename S>
void spinor_io(dirac_ctx *c, void *native, const void *user, bool in, int sites, dirac_layout lay, hipStream_t s) {
    const int vh = (int)c->vh;
    const size_t half_bytes = (size_t)24 * sizeof(S) * c->g.vhp;
    for (int p = 0; p < 2; ++p) {
        if (sites == 1 && p == 1) continue;
        if (sites == 2 && p == 0) continue;
        char *nat = (char *)native + (sites == 0 ? p * half_bytes : 0);
        const int half = sites != 0;
        if (in)
            k_spinor_in<U, S><<<grid_for(vh), kBlock, 0, s>>>(c->g, p, lay, half, (const U *)user,
                                                              (typename St<S>::vec *)nat);
        else
            k_spinor_out<U, S><<<grid_for(vh), kBlock, 0, s>>>(c->g, p, lay, half, (const typename St<S>::vec *)nat,
                                                               (U *)user);
    }
    HIP_CHECK(hipGetLastError());
}

template <typename S>
void spinor_io_user(dirac_ctx *c, void *native, const void *user, bool in, int sites, dirac_prec pr,
                    dirac_layout lay, hipStream_t s) {
    if (pr == DIRAC_F32)
        spinor_io<float, S>(c, native, user, in, sites, lay, s);
    else
        spinor_io<double, S>(c, native, user, in, sites, lay, s);
}

void spinor_dispatch(dirac_ctx *c, void *native, const void *user, bool in, int sites, dirac_prec pr,
                     dirac_layout lay, hipStream_t s) {
    require(lay == DIRAC_LAYOUT_LEX || lay == DIRAC_LAYOUT_EO || lay == DIRAC_LAYOUT_OPENQXD,
            "user layout must be LEX, EO or OPENQXD");
    require(sites >= 0 && sites <= 2, "sites must be 0 (full), 1 (even half) or 2 (odd half)");
    require(sites == 0 || lay != DIRAC_LAYOUT_LEX, "half vectors exist in the EO and OPENQXD layouts only");
    switch (pr) {
        case DIRAC_F64: spinor_io_user<double>(c, native, user, in, sites, pr, lay, s); break;
        case DIRAC_F32: spinor_io_user<float>(c, native, user, in, sites, pr, lay, s); break;
        case DIRAC_F16: spinor_io_user<__half>(c, native, user, in, sites, pr, lay, s); break;
        case DIRAC_BF16: spinor_io_user<__hip_bfloat16>(c, native, user, in, sites, pr, lay, s); break;
        default: throw Error(DIRAC_EINVAL, "unknown precision");
    }
}

// openQxD's gauge storage -> LEX: the thread of odd site (1, i) with ipt position V/2 + k reads the
// 8 links attached to it, slot 2 mu = U_mu(x) and slot 2 mu + 1 = U_mu(x - mu); every LEX link is
// written by exactly one thread (the forward link of an even site y ends at the odd site y + mu)
__global__ __launch_bounds__(kBlock) void k_openqxd_links(Geom g, const double *__restrict__ u_odd,
                                                           const double *__restrict__ a_odd,
                                                           double *__restrict__ U, double *__restrict__ th) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.vh) return;
    int x[4];
    site_coords(g, i, 1, x);
    const int64_t k = ipt_index(g, x) - g.vh;
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
#pragma unroll 1
        for (int back = 0; back < 2; ++back) {
            int y[4] = {x[0], x[1], x[2], x[3]};
            if (back) {
                const bool cross = y[mu] == 0;
                y[mu] = wrap_dn(y[mu], g.L[mu]);
                y[1] = cstar_x1(g, mu, cross, y[1]);  // C*: the link behind x may sit in the mirror copy
            }
            const int64_t lam = lex_index(g, y);
            const int64_t slot = k * 8 + 2 * mu + back;
            const double2 *src = reinterpret_cast<const double2 *>(u_odd) + slot * 9;
            double2 *dst = reinterpret_cast<double2 *>(U) + (lam * 4 + mu) * 9;
#pragma unroll
            for (int e = 0; e < 9; ++e) dst[e] = src[e];
            if (th) th[lam * 4 + mu] = a_odd[slot];
        }
    }
}

__global__ void k_zero16(size_t n, uint4 *__restrict__ p) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace

void zero_fill(void *p, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 16;
    k_zero16<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, (uint4 *)p);
    HIP_CHECK(hipGetLastError());
}

void openqxd_links_to_lex(const Geom &g, const double *u_odd, const double *a_odd, double *U, double *th,
                          hipStream_t s) {
    k_openqxd_links<<<grid_for(g.vh), kBlock, 0, s>>>(g, u_odd, a_odd, U, th);
    HIP_CHECK(hipGetLastError());
}

size_t link_plane_bytes(dirac_prec pr) { return pr == DIRAC_F64 ? 96 : pr == DIRAC_F32 ? 48 : 24; }

void import_links(dirac_ctx *c, hipStream_t s) {
    PrecFields &f = c->f[DIRAC_F64];
    c->flags.alloc(256);
    unsigned long long *maxdev = (unsigned long long *)c->flags.p;
    HIP_CHECK(hipMemsetAsync(maxdev, 0, sizeof(unsigned long long), s));
    const double4 ph = make_double4(c->p.bc_phase[0], c->p.bc_phase[1], c->p.bc_phase[2], c->p.bc_phase[3]);
    for (int p = 0; p < 2; ++p) {
        f.links[p].alloc((size_t)8 * 6 * sizeof(double2) * c->g.vhp);
        f.omega[p].alloc((size_t)8 * sizeof(double) * c->g.vhp);
        k_import_links<<<grid_for(c->vh), kBlock, 0, s>>>(c->g, p, (const double *)c->U_lex.p,
                                                          (const double *)c->theta_lex.p, c->p.qhat, ph,
                                                          (double2 *)f.links[p].p, (double *)f.omega[p].p, maxdev);
    }
    HIP_CHECK(hipGetLastError());
    unsigned long long h = 0;
    HIP_CHECK(hipMemcpyAsync(&h, maxdev, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    double dev;
    memcpy(&dev, &h, sizeof(dev));
    require(dev < 1e-10, "su3_links are not SU(3) matrices (max |U U^dag - 1| + |det U - 1| = " +
                             std::to_string(dev) + "); the two-row link compression needs det U = 1");
    f.links_ready = true;
}

void ensure_prec(dirac_ctx *c, dirac_prec pr, hipStream_t s) {
    switch (pr) {
        case DIRAC_F64: return;
        case DIRAC_F32: convert_fields<float>(c, pr, s); return;
        case DIRAC_F16: convert_fields<__half>(c, pr, s); return;
        case DIRAC_BF16: convert_fields<__hip_bfloat16>(c, pr, s); return;
        default: throw Error(DIRAC_EINVAL, "unknown precision");
    }
}

void spinor_import(dirac_ctx *c, void *native, const void *user, int sites, dirac_prec pr, dirac_layout lay,
                   hipStream_t s) {
    spinor_dispatch(c, native, user, true, sites, pr, lay, s);
}

void spinor_export(dirac_ctx *c, void *user, const void *native, int sites, dirac_prec pr, dirac_layout lay,
                   hipStream_t s) {
    spinor_dispatch(c, const_cast<void *>(native), user, false, sites, pr, lay, s);
}

void clover_import(dirac_ctx *c, const double *user, dirac_layout lay, hipStream_t s) {
    require(lay == DIRAC_LAYOUT_LEX || lay == DIRAC_LAYOUT_EO || lay == DIRAC_LAYOUT_OPENQXD,
            "clover layout must be LEX, EO or OPENQXD");
    PrecFields &f = c->f[DIRAC_F64];
    for (int p = 0; p < 2; ++p) {
        f.clov[p].alloc((size_t)72 * sizeof(double) * c->g.vhp);
        k_clover_in<<<grid_for(c->vh), kBlock, 0, s>>>(c->g, p, lay, user, (double2 *)f.clov[p].p);
    }
    HIP_CHECK(hipGetLastError());
    c->sap_ready = false;
    for (int q = 0; q < 4; ++q) {
        c->f[q].clover_ready = (q == DIRAC_F64);
        c->f[q].inv_ready[0] = c->f[q].inv_ready[1] = false;
    }
}

void clover_export(dirac_ctx *c, double *user, int inverse, dirac_layout lay, hipStream_t s) {
    require(lay == DIRAC_LAYOUT_LEX || lay == DIRAC_LAYOUT_EO || lay == DIRAC_LAYOUT_OPENQXD,
            "clover layout must be LEX, EO or OPENQXD");
    PrecFields &f = c->f[DIRAC_F64];
    for (int p = 0; p < 2; ++p) {
        const double2 *src = inverse ? (f.inv_ready[p] ? (const double2 *)f.clinv[p].p : nullptr)
                                     : (const double2 *)f.clov[p].p;
        k_clover_out<<<grid_for(c->vh), kBlock, 0, s>>>(c->g, p, lay, src, user);
    }
    HIP_CHECK(hipGetLastError());
}

}  // namespace dl
