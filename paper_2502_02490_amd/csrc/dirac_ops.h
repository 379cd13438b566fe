// Device pieces of the Wilson-clover operator in the chiral basis:
// spin projection to half-spinors, SU(3) x U(1) link multiplication with the
// third row rebuilt from the first two, and the packed 6x6 Hermitian clover blocks.
//
// Basis: gamma_mu = [[0, e_mu], [e_mu^dag, 0]] with e_0 = -1, e_k = -i sigma_k, so
//   (1 + s gamma_mu) psi = (h, s e_mu^dag h),  h = u + s e_mu l,
// where u = spins (0, 1) and l = spins (2, 3) of psi (each 2 x 3 colours).  Only
// the half-spinor h (6 complex) is multiplied by the link.
#pragma once

#include "common.h"

template <typename T> using C = cx<T>;

// o = e_mu l, l = (l0, l1) two spins of three colours.
template <int MU, typename T>
DEV void e_mul(const C<T> l0, const C<T> l1, C<T> &o0, C<T> &o1) {
    if constexpr (MU == 0) { o0 = -l0; o1 = -l1; }                       // -1
    else if constexpr (MU == 1) { o0 = times_mi(l1); o1 = times_mi(l0); } // -i sigma_1
    else if constexpr (MU == 2) { o0 = -l1; o1 = l0; }                   // -i sigma_2 = [[0,-1],[1,0]]
    else { o0 = times_mi(l0); o1 = times_i(l1); }                        // -i sigma_3
}
// o = e_mu^dag w.
template <int MU, typename T>
DEV void edag_mul(const C<T> w0, const C<T> w1, C<T> &o0, C<T> &o1) {
    if constexpr (MU == 0) { o0 = -w0; o1 = -w1; }
    else if constexpr (MU == 1) { o0 = times_i(w1); o1 = times_i(w0); }  // i sigma_1
    else if constexpr (MU == 2) { o0 = w1; o1 = -w0; }                   // i sigma_2 = [[0,1],[-1,0]]
    else { o0 = times_i(w0); o1 = times_mi(w1); }                        // i sigma_3
}

// h = u + s e_mu l for a full spinor psi[spin * 3 + colour].
template <int MU, int S, typename T>
DEV void project(const C<T> *psi, C<T> h[6]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        C<T> e0, e1;
        e_mul<MU>(psi[6 + a], psi[9 + a], e0, e1);
        if constexpr (S > 0) { h[a] = psi[a] + e0; h[3 + a] = psi[3 + a] + e1; }
        else { h[a] = psi[a] - e0; h[3 + a] = psi[3 + a] - e1; }
    }
}

// acc += (w, s e_mu^dag w).
template <int MU, int S, typename T>
DEV void reconstruct_add(const C<T> w[6], C<T> *acc) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        C<T> e0, e1;
        edag_mul<MU>(w[a], w[3 + a], e0, e1);
        acc[a] = acc[a] + w[a];
        acc[3 + a] = acc[3 + a] + w[3 + a];
        if constexpr (S > 0) { acc[6 + a] = acc[6 + a] + e0; acc[9 + a] = acc[9 + a] + e1; }
        else { acc[6 + a] = acc[6 + a] - e0; acc[9 + a] = acc[9 + a] - e1; }
    }
}

// Third row of an SU(3) matrix from the first two: r2 = conj(r0 x r1).
template <typename T>
DEV void third_row(const C<T> u[6], C<T> r2[3]) {
    r2[0] = conj(u[1] * u[5] - u[2] * u[4]);
    r2[1] = conj(u[2] * u[3] - u[0] * u[5]);
    r2[2] = conj(u[0] * u[4] - u[1] * u[3]);
}

// w = e^{i om} U h (forward) for both spin rows of the half-spinor; r2 = third_row(u).
template <typename T>
DEV void link_mul_r2(const C<T> u[6], const C<T> r2[3], T co, T si, const C<T> h[6], C<T> w[6]) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const C<T> *hs = h + 3 * s;
        C<T> t0 = u[0] * hs[0], t1 = u[3] * hs[0], t2 = r2[0] * hs[0];
        madd(t0, u[1], hs[1]); madd(t1, u[4], hs[1]); madd(t2, r2[1], hs[1]);
        madd(t0, u[2], hs[2]); madd(t1, u[5], hs[2]); madd(t2, r2[2], hs[2]);
        const C<T> ph = mk(co, si);
        w[3 * s + 0] = ph * t0; w[3 * s + 1] = ph * t1; w[3 * s + 2] = ph * t2;
    }
}

template <typename T>
DEV void link_mul(const C<T> u[6], T co, T si, const C<T> h[6], C<T> w[6]) {
    C<T> r2[3];
    third_row(u, r2);
    link_mul_r2(u, r2, co, si, h, w);
}

// w = e^{-i om} U^dag h (backward); r2 = third_row(u).
template <typename T>
DEV void link_adj_mul_r2(const C<T> u[6], const C<T> r2[3], T co, T si, const C<T> h[6], C<T> w[6]) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const C<T> *hs = h + 3 * s;
        // (U^dag h)_a = sum_b conj(U_ba) h_b
        C<T> t0 = conj_mul(u[0], hs[0]), t1 = conj_mul(u[1], hs[0]), t2 = conj_mul(u[2], hs[0]);
        cmadd(t0, u[3], hs[1]); cmadd(t1, u[4], hs[1]); cmadd(t2, u[5], hs[1]);
        cmadd(t0, r2[0], hs[2]); cmadd(t1, r2[1], hs[2]); cmadd(t2, r2[2], hs[2]);
        const C<T> ph = mk(co, -si);
        w[3 * s + 0] = ph * t0; w[3 * s + 1] = ph * t1; w[3 * s + 2] = ph * t2;
    }
}

template <typename T>
DEV void link_adj_mul(const C<T> u[6], T co, T si, const C<T> h[6], C<T> w[6]) {
    C<T> r2[3];
    third_row(u, r2);
    link_adj_mul_r2(u, r2, co, si, h, w);
}

// out = B in for a packed Hermitian 6x6 block: pk[0..5] diagonal, then (re, im) of the
// 15 strictly-upper entries (r < c) in row-major order (paper Sec. 4.1.3).
template <typename T>
DEV void block_mul(const T *pk, const C<T> in[6], C<T> out[6]) {
#pragma unroll
    for (int r = 0; r < 6; ++r) out[r] = pk[r] * in[r];
    int k = 6;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = r + 1; c < 6; ++c) {
            const C<T> a = mk(pk[k], pk[k + 1]);
            k += 2;
            madd(out[r], a, in[c]);   // B_rc in_c
            cmadd(out[c], a, in[r]);  // B_cr = conj(B_rc)
        }
}

// sin and cos of a link angle omega (|omega| below a few times pi) in the accumulation
// precision, without the general-argument library routine (whose wide-range reduction needs
// per-lane scratch memory).  Cody-Waite reduction r = omega - k pi/2 with pi/2 split in two
// parts and fused multiply-adds, then the Taylor series of sin r and cos r on |r| <= pi/4
// (terms through r^17 in FP64, r^11 in FP32: truncation below 1e-19 and 1e-9 respectively),
// and the quadrant k mod 4 selects signs and the sin/cos swap.
template <typename T> struct PiHalf;
template <> struct PiHalf<double> {
    static constexpr double hi = 1.5707963267948966192313216916398, lo = 6.123233995736766035868820147292e-17;
    static constexpr int nterm = 9;
};
template <> struct PiHalf<float> {
    static constexpr float hi = 1.57079637050628662109375f, lo = -4.37113900018624283e-8f;
    static constexpr int nterm = 6;
};
template <typename T>
DEV void sc(T w, T &s, T &c) {
    const T k = rint(w * T(0.63661977236758134307553505349006));  // 2 / pi
    T r = fma(-k, PiHalf<T>::hi, w);
    r = fma(-k, PiHalf<T>::lo, r);
    const T r2 = r * r;
    // Horner on the Taylor coefficients: sin r = r sum (-r^2)^n / (2n+1)!, cos r = sum (-r^2)^n / (2n)!
    T ps = T(1), pc = T(1);
    constexpr int N = PiHalf<T>::nterm;
#pragma unroll
    for (int n = N - 1; n >= 1; --n) {
        ps = fma(-r2 * (T(1) / T((2 * n) * (2 * n + 1))), ps, T(1));
        pc = fma(-r2 * (T(1) / T((2 * n - 1) * (2 * n))), pc, T(1));
    }
    const T sr = r * ps, cr = pc;
    const int q = ((int)k) & 3;
    s = q == 0 ? sr : q == 1 ? cr : q == 2 ? -sr : -cr;
    c = q == 0 ? cr : q == 1 ? -sr : q == 2 ? -cr : sr;
}
