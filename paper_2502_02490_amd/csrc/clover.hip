// Clover field on the device (paper Sec. 4.3 and the outlook's "generate the clover
// field on the GPU"): build A = (4 + m0) + C from the SU(3) and U(1) links in FP64,
// invert its 6x6 chirality blocks in FP64 registers, and apply A or A^-1.
#include "dirac_ops.h"
#include "internal.h"

namespace dl {
namespace {

struct M3 {
    C<double> m[9];
};

DEV M3 ld(const double *__restrict__ U, int lam, int mu) {
    const double2 *u = reinterpret_cast<const double2 *>(U + ((size_t)lam * 4 + mu) * 18);
    M3 r;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        double2 v = u[k];
        r.m[k] = mk(v.x, v.y);
    }
    return r;
}
DEV M3 mul(const M3 &a, const M3 &b) {  // a b
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            C<double> s = a.m[3 * i] * b.m[j];
            madd(s, a.m[3 * i + 1], b.m[3 + j]);
            madd(s, a.m[3 * i + 2], b.m[6 + j]);
            r.m[3 * i + j] = s;
        }
    return r;
}
DEV M3 mul_nd(const M3 &a, const M3 &b) {  // a b^dag
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            C<double> s = a.m[3 * i] * conj(b.m[3 * j]);
            madd(s, a.m[3 * i + 1], conj(b.m[3 * j + 1]));
            madd(s, a.m[3 * i + 2], conj(b.m[3 * j + 2]));
            r.m[3 * i + j] = s;
        }
    return r;
}
DEV M3 mul_dn(const M3 &a, const M3 &b) {  // a^dag b
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            C<double> s = conj_mul(a.m[i], b.m[j]);
            cmadd(s, a.m[3 + i], b.m[3 + j]);
            cmadd(s, a.m[6 + i], b.m[6 + j]);
            r.m[3 * i + j] = s;
        }
    return r;
}

// F'_{mu nu}(x) = c_sw (Q - Q^dag)/8 + c_qed qhat (q - q*)/8, Q / q the sum of the four
// plaquette leaves at x in the (mu, nu) plane from U / from exp(i theta).
DEV void plane_field(const Geom &g, const double *__restrict__ U, const double *__restrict__ th, const int x[4],
                     int mu, int nu, double csw, double cq, M3 &F) {
    int y[4];
    auto at = [&](int dm, int dn) {
        y[0] = x[0]; y[1] = x[1]; y[2] = x[2]; y[3] = x[3];
        // each step that crosses the boundary of a C* direction also moves x1 (the shifts commute)
        auto step = [&](int d, int k) {
            if (k == 0) return;
            const bool cross = k > 0 ? y[d] == g.L[d] - 1 : y[d] == 0;
            y[d] = k > 0 ? wrap_up(y[d], g.L[d]) : wrap_dn(y[d], g.L[d]);
            y[1] = cstar_x1(g, d, cross, y[1]);
        };
        step(mu, dm);
        step(nu, dn);
        return lex_index(g, y);
    };
    const int x0 = at(0, 0), xpm = at(1, 0), xpn = at(0, 1), xmm = at(-1, 0), xmn = at(0, -1);
    const int xmm_pn = at(-1, 1), xmm_mn = at(-1, -1), xpm_mn = at(1, -1);
    M3 q = mul_nd(mul(ld(U, x0, mu), ld(U, xpm, nu)), mul(ld(U, x0, nu), ld(U, xpn, mu)));
    M3 t = mul(mul_nd(ld(U, x0, nu), ld(U, xmm_pn, mu)), mul_dn(ld(U, xmm, nu), ld(U, xmm, mu)));
#pragma unroll
    for (int k = 0; k < 9; ++k) q.m[k] = q.m[k] + t.m[k];
    t = mul_dn(mul(ld(U, xmm_mn, nu), ld(U, xmm, mu)), mul(ld(U, xmm_mn, mu), ld(U, xmn, nu)));
#pragma unroll
    for (int k = 0; k < 9; ++k) q.m[k] = q.m[k] + t.m[k];
    t = mul(mul_dn(ld(U, xmn, nu), ld(U, xmn, mu)), mul_nd(ld(U, xpm_mn, nu), ld(U, x0, mu)));
#pragma unroll
    for (int k = 0; k < 9; ++k) q.m[k] = q.m[k] + t.m[k];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) F.m[3 * a + b] = (csw * 0.125) * (q.m[3 * a + b] - conj(q.m[3 * b + a]));
    if (th && cq != 0.0) {
        auto T = [&](int s, int d) { return th[(size_t)s * 4 + d]; };
        const double a1 = T(x0, mu) + T(xpm, nu) - T(xpn, mu) - T(x0, nu);
        const double a2 = T(x0, nu) - T(xmm_pn, mu) - T(xmm, nu) + T(xmm, mu);
        const double a3 = -T(xmm, mu) - T(xmm_mn, nu) + T(xmm_mn, mu) + T(xmn, nu);
        const double a4 = -T(xmn, nu) + T(xmn, mu) + T(xpm_mn, nu) - T(x0, mu);
        // (q - q*) / 8 = i Im(q) / 4
        const double im = cq * 0.25 * (sin(a1) + sin(a2) + sin(a3) + sin(a4));
#pragma unroll
        for (int a = 0; a < 3; ++a) F.m[4 * a].i += im;
    }
}

// One thread per site of parity p: A(x) packed as [72] reals, block + then block -.
// With sigma_0k = diag(s_k, -s_k), sigma_jk = -eps_jkl diag(s_l, s_l) (chiral basis) the
// term (i/4) sum sigma_{mu nu} F_{mu nu} is, per chirality block, [[G3, G1 - i G2], [G1 + i G2, -G3]]:
//   block +: G1 = (i/2)(F01 - F23), G2 = (i/2)(F02 + F13), G3 = (i/2)(F03 - F12)
//   block -: G1 = -(i/2)(F01 + F23), G2 = -(i/2)(F02 - F13), G3 = -(i/2)(F03 + F12)
__global__ __launch_bounds__(kBlock) void k_clover_build(Geom g, int p, const double *__restrict__ U,
                                                          const double *__restrict__ th, double csw, double cq,
                                                          double diag, double2 *__restrict__ out) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.vh) return;
    int x[4];
    site_coords(g, i, p, x);
    M3 F[6];
    plane_field(g, U, th, x, 0, 1, csw, cq, F[0]);
    plane_field(g, U, th, x, 0, 2, csw, cq, F[1]);
    plane_field(g, U, th, x, 0, 3, csw, cq, F[2]);
    plane_field(g, U, th, x, 1, 2, csw, cq, F[3]);
    plane_field(g, U, th, x, 1, 3, csw, cq, F[4]);
    plane_field(g, U, th, x, 2, 3, csw, cq, F[5]);
    double pk[72];
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        C<double> G1[9], G2[9], G3[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            // block +: (F01 - F23, F02 + F13, F03 - F12) * (i/2); block -: -(F01 + F23, F02 - F13, F03 + F12) * (i/2)
            C<double> f1 = blk == 0 ? F[0].m[k] - F[5].m[k] : -(F[0].m[k] + F[5].m[k]);
            C<double> f2 = blk == 0 ? F[1].m[k] + F[4].m[k] : -(F[1].m[k] - F[4].m[k]);
            C<double> f3 = blk == 0 ? F[2].m[k] - F[3].m[k] : -(F[2].m[k] + F[3].m[k]);
            G1[k] = 0.5 * times_i(f1);
            G2[k] = 0.5 * times_i(f2);
            G3[k] = 0.5 * times_i(f3);
        }
        auto B = [&](int r, int c) -> C<double> {
            const int s = r / 3, a = r % 3, t = c / 3, b = c % 3;
            const int k = 3 * a + b;
            C<double> v;
            if (s == 0 && t == 0) v = G3[k];
            else if (s == 0 && t == 1) v = G1[k] - times_i(G2[k]);
            else if (s == 1 && t == 0) v = G1[k] + times_i(G2[k]);
            else v = -G3[k];
            if (r == c) v.r += diag;
            return v;
        };
        double *o = pk + 36 * blk;
#pragma unroll
        for (int r = 0; r < 6; ++r) o[r] = B(r, r).r;
        int k = 6;
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int c = r + 1; c < 6; ++c) {
                C<double> v = B(r, c);
                o[k] = v.r;
                o[k + 1] = v.i;
                k += 2;
            }
    }
    store_field<double, 72>(out, (uint32_t)i, pk);
}

// Gauss-Jordan inversion of a 6x6 complex block with partial pivoting (pivot row chosen by
// max |re| + |im| as in LAPACK's zgetrf).  Returns false when a pivot modulus is below thr.
DEV bool invert6(C<double> a[6][6], C<double> v[6][6], double thr) {
    bool ok = true;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = 0; c < 6; ++c) v[r][c] = mk(r == c ? 1.0 : 0.0, 0.0);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        int piv = k;
        double best = fabs(a[k][k].r) + fabs(a[k][k].i);
#pragma unroll
        for (int r = k + 1; r < 6; ++r) {
            double m = fabs(a[r][k].r) + fabs(a[r][k].i);
            if (m > best) { best = m; piv = r; }
        }
#pragma unroll
        for (int r = k + 1; r < 6; ++r) {
            const bool sw = (piv == r);
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                C<double> t = a[k][c], u = a[r][c];
                a[k][c] = sw ? u : t;
                a[r][c] = sw ? t : u;
                t = v[k][c]; u = v[r][c];
                v[k][c] = sw ? u : t;
                v[r][c] = sw ? t : u;
            }
        }
        const C<double> pv = a[k][k];
        const double n2 = pv.r * pv.r + pv.i * pv.i;
        if (!(sqrt(n2) >= thr)) ok = false;
        const double inv = n2 > 0.0 ? 1.0 / n2 : 0.0;
        const C<double> rp = mk(pv.r * inv, -pv.i * inv);  // 1 / pivot
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            a[k][c] = a[k][c] * rp;
            v[k][c] = v[k][c] * rp;
        }
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            if (r == k) continue;
            const C<double> f = a[r][k];
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                a[r][c] = a[r][c] - f * a[k][c];
                v[r][c] = v[r][c] - f * v[k][c];
            }
        }
    }
    return ok;
}

__global__ __launch_bounds__(kBlock) void k_clover_invert(Geom g, int p, const double2 *__restrict__ A,
                                                           double2 *__restrict__ Ainv, int *__restrict__ first_bad) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.vh) return;
    bool ok = true;
    double out[72];
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        double pk[36];
        const double2 *Ai = site_ptr(A, (uint32_t)i, 36);
#pragma unroll
        for (int k = 0; k < 18; ++k) {
            double2 v = Ai[(18 * blk + k) * kSB];
            pk[2 * k] = v.x;
            pk[2 * k + 1] = v.y;
        }
        C<double> a[6][6], v[6][6];
        double amax = 0.0;
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            a[r][r] = mk(pk[r], 0.0);
            amax = fmax(amax, fabs(pk[r]));
        }
        int k = 6;
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int c = r + 1; c < 6; ++c) {
                a[r][c] = mk(pk[k], pk[k + 1]);
                a[c][r] = mk(pk[k], -pk[k + 1]);
                amax = fmax(amax, sqrt(pk[k] * pk[k] + pk[k + 1] * pk[k + 1]));
                k += 2;
            }
        ok = invert6(a, v, 1e-14 * amax) && ok;
        double *o = out + 36 * blk;
#pragma unroll
        for (int r = 0; r < 6; ++r) o[r] = v[r][r].r;
        k = 6;
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int c = r + 1; c < 6; ++c) {
                o[k] = v[r][c].r;
                o[k + 1] = v[r][c].i;
                k += 2;
            }
    }
    store_field<double, 72>(Ainv, (uint32_t)i, out);
    if (!ok) {
        int x[4];
        site_coords(g, i, p, x);
        atomicMin(first_bad, lex_index(g, x));
    }
}

template <typename S, int INV>
__global__ __launch_bounds__(kBlock) void k_clover_apply(int vh, size_t vs, const typename St<S>::vec *__restrict__ in,
                                                          const typename St<S>::vec *__restrict__ A,
                                                          typename St<S>::vec *__restrict__ out) {
    using T = typename St<S>::acc;
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= vh) return;
    in += blockIdx.y * vs;  // right-hand side blockIdx.y
    out += blockIdx.y * vs;
    T r[24], pk[72];
    load_field<S, 24>(in, (uint32_t)i, r);
    load_field<S, 72>(A, (uint32_t)i, pk);
    C<T> psi[12], y[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) psi[k] = mk(r[2 * k], r[2 * k + 1]);
    block_mul(pk, psi, y);
    block_mul(pk + 36, psi + 6, y + 6);
#pragma unroll
    for (int k = 0; k < 12; ++k) { r[2 * k] = y[k].r; r[2 * k + 1] = y[k].i; }
    store_field<S, 24>(out, (uint32_t)i, r);
}

template <typename S>
void clover_apply_t(dirac_ctx *c, void *out, const void *in, int parity, int inverse, dirac_prec pr, hipStream_t s,
                    int nrhs) {
    PrecFields &f = c->f[pr];
    const void *A = inverse ? f.clinv[parity].p : f.clov[parity].p;
    using V = typename St<S>::vec;
    const size_t vs = (size_t)(24 / St<S>::W) * c->g.vhp;
    const dim3 grid(grid_for(c->vh), nrhs);
    if (inverse)
        k_clover_apply<S, 1><<<grid, kBlock, 0, s>>>((int)c->vh, vs, (const V *)in, (const V *)A, (V *)out);
    else
        k_clover_apply<S, 0><<<grid, kBlock, 0, s>>>((int)c->vh, vs, (const V *)in, (const V *)A, (V *)out);
    HIP_CHECK(hipGetLastError());
}

}  // namespace

void clover_build(dirac_ctx *c, hipStream_t s) {
    PrecFields &f = c->f[DIRAC_F64];
    const double diag = 1.0 / (2.0 * c->p.kappa);
    for (int p = 0; p < 2; ++p) {
        f.clov[p].alloc((size_t)72 * sizeof(double) * c->g.vhp);
        k_clover_build<<<grid_for(c->vh), kBlock, 0, s>>>(c->g, p, (const double *)c->U_lex.p,
                                                          (const double *)c->theta_lex.p, c->p.csw,
                                                          c->p.csw_qed * c->p.qhat, diag, (double2 *)f.clov[p].p);
    }
    HIP_CHECK(hipGetLastError());
    c->sap_ready = false;
    for (int q = 0; q < 4; ++q) {
        c->f[q].clover_ready = (q == DIRAC_F64);
        c->f[q].inv_ready[0] = c->f[q].inv_ready[1] = false;
    }
}

int64_t clover_invert_parity(dirac_ctx *c, int p, hipStream_t s) {
    PrecFields &f = c->f[DIRAC_F64];
    require(f.clover_ready, "no clover field");
    f.clinv[p].alloc((size_t)72 * sizeof(double) * c->g.vhp);
    c->flags.alloc(256);
    int *bad = (int *)c->flags.p + 8;
    const int big = 0x7fffffff;
    HIP_CHECK(hipMemcpyAsync(bad, &big, sizeof(int), hipMemcpyHostToDevice, s));
    k_clover_invert<<<grid_for(c->vh), kBlock, 0, s>>>(c->g, p, (const double2 *)f.clov[p].p,
                                                       (double2 *)f.clinv[p].p, bad);
    HIP_CHECK(hipGetLastError());
    int h = big;
    HIP_CHECK(hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    for (int q = 0; q < 4; ++q) c->f[q].inv_ready[p] = false;
    f.inv_ready[p] = true;
    return h == big ? -1 : (int64_t)h;
}

void clover_apply(dirac_ctx *c, void *out, const void *in, int parity, int inverse, dirac_prec pr, hipStream_t s,
                  int nrhs) {
    require(parity == 0 || parity == 1, "parity must be 0 (even) or 1 (odd)");
    ensure_prec(c, pr, s);
    PrecFields &f = c->f[pr];
    require(!inverse || f.inv_ready[parity], "clover inverse of this parity not computed; call clover_invert");
    switch (pr) {
        case DIRAC_F64: clover_apply_t<double>(c, out, in, parity, inverse, pr, s, nrhs); break;
        case DIRAC_F32: clover_apply_t<float>(c, out, in, parity, inverse, pr, s, nrhs); break;
        case DIRAC_F16: clover_apply_t<__half>(c, out, in, parity, inverse, pr, s, nrhs); break;
        case DIRAC_BF16: clover_apply_t<__hip_bfloat16>(c, out, in, parity, inverse, pr, s, nrhs); break;
        default: throw Error(DIRAC_EINVAL, "unknown precision");
    }
}

}  // namespace dl
