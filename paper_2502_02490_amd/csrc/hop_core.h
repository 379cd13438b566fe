// Device pieces of the hopping term shared by the hop kernels (hop_kernels.h) and the Schwarz block
// solver (sap.hip): kernel arguments, spinor and link loads, the neighbour index and the
// projected accumulation of one direction.
#pragma once

#include "dirac_ops.h"
#include "internal.h"

namespace dl {
namespace {

template <typename S>
struct HopArgs {
    Geom g;
    int p;           // output parity
    int nb8;         // work-groups launched (a multiple of 8 with the XCD-contiguous order)
    int xcd;         // 1: XCD-contiguous work-group order
    int nrhs;        // right-hand sides: vector r of in / out / chi is r * vs vectors after the base
    size_t vs;       // 16-byte vectors per half-lattice spinor
    const int *active;  // per right-hand side, NULL = all
    const typename St<S>::vec *in;     // parity 1 - p, 24 reals per site
    const typename Lk<S>::vec *links;  // parity p, [8 dir][12 / W][vh]
    const typename Lk<S>::om *omega;   // parity p, [8 dir][vh]
    const typename St<S>::vec *clov;   // parity p, 72 reals: A (HOP_CLOV) or A^-1 (HOP_INV)
    const typename St<S>::vec *chi;    // parity p (HOP_CLOV)
    typename St<S>::vec *out;          // parity p
    typename St<S>::acc coef;
};

template <typename S>
DEV void load_spinor(const typename St<S>::vec *__restrict__ base, uint32_t s, C<typename St<S>::acc> psi[12]) {
    using T = typename St<S>::acc;
    T r[24];
    load_field<S, 24>(base, s, r);
#pragma unroll
    for (int k = 0; k < 12; ++k) psi[k] = mk(r[2 * k], r[2 * k + 1]);
}

template <typename S, bool NT>
DEV void load_link(const HopArgs<S> &a, int dir, uint32_t i, C<typename St<S>::acc> u[6], typename St<S>::acc &co,
                   typename St<S>::acc &si) {
    using T = typename St<S>::acc;
    using LV = typename Lk<S>::vec;
    using OM = typename Lk<S>::om;
    constexpr int W = Lk<S>::W;
    const size_t vhp = (size_t)a.g.vhp;
    const LV *b = site_ptr(a.links + (size_t)dir * (12 / W) * vhp, i, 12 / W);
    T r[12];
#pragma unroll
    for (int k = 0; k < 12 / W; ++k) Lk<S>::unpack(NT ? ld_stream(b + k * kSB) : b[k * kSB], r + k * W);
#pragma unroll
    for (int k = 0; k < 6; ++k) u[k] = mk(r[2 * k], r[2 * k + 1]);
    const OM *om = a.omega + (size_t)dir * vhp + i;
    const OM w = NT ? ld_stream(om) : *om;
    if constexpr (Lk<S>::phase_pair) Lk<S>::phase(w, co, si);
    else sc((T)w, si, co);
}

// Spin structure of gamma_mu = [[0, e_mu], [e_mu^dag, 0]]: e_mu is monomial, row k has its
// one entry c_k in column p_k, with p_1 = 1 - p_0.  Per mu: (p_0, c_0, c_1), c in {+-1, +-i}:
//   e_0 = -1: (0, -1, -1)   e_1 = -i sigma_1: (1, -i, -i)
//   e_2 = -i sigma_2: (1, -1, +1)   e_3 = -i sigma_3: (0, -i, +i)
// so (e l)_k = c_k l_{p_k} and (e^dag w)_{p_k} = conj(c_k) w_k.

// Index of the neighbour of site (x, row) in direction n = 2 mu + back, in the other parity.
template <typename S>
DEV uint32_t neighbour(const HopArgs<S> &a, const int x[4], int row, int n) {
    const int mu = n >> 1, back = n & 1;
    const int xm = mu == 0 ? x[0] : mu == 1 ? x[1] : mu == 2 ? x[2] : x[3];
    const int Lm = mu == 0 ? a.g.L[0] : mu == 1 ? a.g.L[1] : mu == 2 ? a.g.L[2] : a.g.L[3];
    const bool cross = back ? xm == 0 : xm + 1 == Lm;
    const int xn = back ? (xm == 0 ? Lm - 1 : xm - 1) : (xm + 1 == Lm ? 0 : xm + 1);
    const int rs = mu == 0 ? a.g.L[1] * a.g.L[2] : mu == 1 ? a.g.L[2] : 1;
    const int rw = row + (cstar_x1(a.g, mu, cross, x[1]) - x[1]) * a.g.L[2];  // C*: into the mirror copy
    return mu == 3 ? (uint32_t)(rw * a.g.h3 + (xn >> 1)) : (uint32_t)((rw + (xn - xm) * rs) * a.g.h3 + (x[3] >> 1));
}

// acc += the direction-n term for the neighbour spinor psi and the link (u, co, si): project to
// a half-spinor, multiply by the link (or its adjoint), reconstruct.
// z times a unit c = CR + i CI, c in {+-1, +-i}, as sign changes and swaps (exact).
template <int CR, int CI, typename T>
DEV C<T> unit_mul(C<T> z) {
    if constexpr (CR == 1) return z;
    else if constexpr (CR == -1) return mk(-z.r, -z.i);
    else if constexpr (CI == 1) return mk(-z.i, z.r);
    else return mk(z.i, -z.r);
}
// a + SG b with SG = +-1
template <int SG, typename T>
DEV C<T> add_signed(C<T> a, C<T> b) {
    if constexpr (SG > 0) return a + b;
    else return a - b;
}

// Direction N = 2 mu + back with its spin structure fixed at compile time: the projector sign
// (forward 1 + SF gamma, backward 1 - SF gamma; SF = -1 for D, +1 for D^dag), the spin swap and
// the units c_0, c_1 of e_mu become sign changes, swaps and additions.  r2: the link's third row,
// third_row(u), computed by the caller (once for several right-hand sides).
// project_dir_n: the half-spinor h of the neighbour spinor psi; apply_dir_n: the link product
// of h and the reconstruction into acc.  accumulate_dir_n is the two in sequence, so a
// half-spinor projected early and kept gives the same bits as the whole.
template <typename T, int DAG, int N>
DEV void project_dir_n(const C<T> psi[12], C<T> h[6]) {
    constexpr int mu = N >> 1, back = N & 1;
    constexpr int SG = (DAG ? 1 : -1) * (back ? -1 : 1);
    constexpr bool SW = (mu == 1 || mu == 2);
    constexpr int C0R = (mu == 0 || mu == 2) ? -1 : 0, C0I = (mu == 1 || mu == 3) ? -1 : 0;
    constexpr int C1R = mu == 0 ? -1 : mu == 2 ? 1 : 0, C1I = mu == 1 ? -1 : mu == 3 ? 1 : 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const C<T> e0 = unit_mul<C0R, C0I>(SW ? psi[9 + c] : psi[6 + c]);
        const C<T> e1 = unit_mul<C1R, C1I>(SW ? psi[6 + c] : psi[9 + c]);
        h[c] = add_signed<SG>(psi[c], e0);
        h[3 + c] = add_signed<SG>(psi[3 + c], e1);
    }
}

template <typename T, int DAG, int N>
DEV void apply_dir_n(const C<T> h[6], const C<T> u[6], const C<T> r2[3], T co, T si, C<T> acc[12]) {
    constexpr int mu = N >> 1, back = N & 1;
    constexpr int SG = (DAG ? 1 : -1) * (back ? -1 : 1);
    constexpr bool SW = (mu == 1 || mu == 2);
    constexpr int C0R = (mu == 0 || mu == 2) ? -1 : 0, C0I = (mu == 1 || mu == 3) ? -1 : 0;
    constexpr int C1R = mu == 0 ? -1 : mu == 2 ? 1 : 0, C1I = mu == 1 ? -1 : mu == 3 ? 1 : 0;
    C<T> w[6];
    if constexpr (back) link_adj_mul_r2(u, r2, co, si, h, w);
    else link_mul_r2(u, r2, co, si, h, w);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[c] = acc[c] + w[c];
        acc[3 + c] = acc[3 + c] + w[3 + c];
        const C<T> t0 = unit_mul<C0R, -C0I>(w[c]);      // conj(c_0) w_0 -> lower spin p_0
        const C<T> t1 = unit_mul<C1R, -C1I>(w[3 + c]);  // conj(c_1) w_1 -> lower spin p_1
        acc[6 + c] = add_signed<SG>(acc[6 + c], SW ? t1 : t0);
        acc[9 + c] = add_signed<SG>(acc[9 + c], SW ? t0 : t1);
    }
}

template <typename T, int DAG, int N>
DEV void accumulate_dir_n(const C<T> psi[12], const C<T> u[6], const C<T> r2[3], T co, T si, C<T> acc[12]) {
    C<T> h[6];
    project_dir_n<T, DAG, N>(psi, h);
    apply_dir_n<T, DAG, N>(h, u, r2, co, si, acc);
}

// acc += the direction-n term (n a run-time value, uniform over the wavefront): one of the eight
// specialised bodies above.
template <typename T, int DAG>
DEV void accumulate_dir_r2(int n, const C<T> psi[12], const C<T> u[6], const C<T> r2[3], T co, T si, C<T> acc[12]) {
    switch (n) {
        case 0: accumulate_dir_n<T, DAG, 0>(psi, u, r2, co, si, acc); break;
        case 1: accumulate_dir_n<T, DAG, 1>(psi, u, r2, co, si, acc); break;
        case 2: accumulate_dir_n<T, DAG, 2>(psi, u, r2, co, si, acc); break;
        case 3: accumulate_dir_n<T, DAG, 3>(psi, u, r2, co, si, acc); break;
        case 4: accumulate_dir_n<T, DAG, 4>(psi, u, r2, co, si, acc); break;
        case 5: accumulate_dir_n<T, DAG, 5>(psi, u, r2, co, si, acc); break;
        case 6: accumulate_dir_n<T, DAG, 6>(psi, u, r2, co, si, acc); break;
        default: accumulate_dir_n<T, DAG, 7>(psi, u, r2, co, si, acc); break;
    }
}

template <typename T, int DAG>
DEV void accumulate_dir(int n, const C<T> psi[12], const C<T> u[6], T co, T si, C<T> acc[12]) {
    C<T> r2[3];
    third_row(u, r2);
    accumulate_dir_r2<T, DAG>(n, psi, u, r2, co, si, acc);
}


}  // namespace
}  // namespace dl
