// Device-side building blocks shared by the HIP kernels: complex arithmetic,
// storage-precision traits for the 16-byte plane layout, and site geometry.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#define DEV __device__ __forceinline__
#define HD __host__ __device__ __forceinline__

// ------------------------------------------------------------------ complex
template <typename T>
struct cx {
    T r, i;
};
template <typename T> DEV cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T> DEV cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <typename T> DEV cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <typename T> DEV cx<T> operator-(cx<T> a) { return {-a.r, -a.i}; }
template <typename T> DEV cx<T> operator*(cx<T> a, cx<T> b) { return {fma(a.r, b.r, -a.i * b.i), fma(a.r, b.i, a.i * b.r)}; }
template <typename T> DEV cx<T> operator*(T s, cx<T> a) { return {s * a.r, s * a.i}; }
template <typename T> DEV cx<T> conj(cx<T> a) { return {a.r, -a.i}; }
template <typename T> DEV cx<T> times_i(cx<T> a) { return {-a.i, a.r}; }      // i a
template <typename T> DEV cx<T> times_mi(cx<T> a) { return {a.i, -a.r}; }     // -i a
template <typename T> DEV cx<T> conj_mul(cx<T> a, cx<T> b) { return {fma(a.r, b.r, a.i * b.i), fma(a.r, b.i, -a.i * b.r)}; }  // conj(a) b
template <typename T> DEV void madd(cx<T> &acc, cx<T> a, cx<T> b) {  // acc += a b
    acc.r = fma(a.r, b.r, acc.r); acc.r = fma(-a.i, b.i, acc.r);
    acc.i = fma(a.r, b.i, acc.i); acc.i = fma(a.i, b.r, acc.i);
}
template <typename T> DEV void cmadd(cx<T> &acc, cx<T> a, cx<T> b) {  // acc += conj(a) b
    acc.r = fma(a.r, b.r, acc.r); acc.r = fma(a.i, b.i, acc.r);
    acc.i = fma(a.r, b.i, acc.i); acc.i = fma(-a.i, b.r, acc.i);
}

// ------------------------------------------------------------------ storage precision
// A field of n reals per site is stored, per parity, as n / W planes of 16-byte
// vectors: plane k holds reals [k W, (k + 1) W) of every site, site-fastest.
// Accumulation is FP64 for FP64 storage and FP32 otherwise.
template <typename S> struct St;
template <> struct St<double> {
    using acc = double; using vec = double2; static constexpr int W = 2;
    static DEV void unpack(const vec &v, acc *o) { o[0] = v.x; o[1] = v.y; }
    static DEV vec pack(const acc *o) { return make_double2(o[0], o[1]); }
};
template <> struct St<float> {
    using acc = float; using vec = float4; static constexpr int W = 4;
    static DEV void unpack(const vec &v, acc *o) { o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w; }
    static DEV vec pack(const acc *o) { return make_float4(o[0], o[1], o[2], o[3]); }
};
template <> struct St<__half> {
    using acc = float; using vec = uint4; static constexpr int W = 8;
    static DEV void unpack(const vec &v, acc *o) {
        const __half2 *h = reinterpret_cast<const __half2 *>(&v);
#pragma unroll
        for (int k = 0; k < 4; ++k) { float2 f = __half22float2(h[k]); o[2 * k] = f.x; o[2 * k + 1] = f.y; }
    }
    // The values are rounded to FP32 first and then to FP16 (the C++ semantics).  The empty asm
    // keeps the compiler from merging the last multiply-add of a value with its FP16 conversion
    // into one mixed-precision instruction that rounds once: it does so in some kernels and not
    // in others, and two kernels computing the same sums would then disagree in the last bit.
    static DEV vec pack(const acc *o) {
        vec v;
        __half2 *h = reinterpret_cast<__half2 *>(&v);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float a = o[2 * k], b = o[2 * k + 1];
            asm volatile("" : "+v"(a), "+v"(b));
            h[k] = __floats2half2_rn(a, b);
        }
        return v;
    }
};
template <> struct St<__hip_bfloat16> {
    using acc = float; using vec = uint4; static constexpr int W = 8;
    static DEV void unpack(const vec &v, acc *o) {
        const uint32_t *w = reinterpret_cast<const uint32_t *>(&v);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            o[2 * k] = __uint_as_float(w[k] << 16);
            o[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
        }
    }
    static DEV uint32_t rne(float f) {  // round to nearest even (inputs are finite)
        uint32_t u = __float_as_uint(f);
        return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    }
    static DEV vec pack(const acc *o) {
        vec v;
        uint32_t *w = reinterpret_cast<uint32_t *>(&v);
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = rne(o[2 * k]) | (rne(o[2 * k + 1]) << 16);
        return v;
    }
};

// Site-blocked layout ("NATIVE"): the sites of one parity are grouped in blocks of kSB = 64
// (one wavefront); a field with np planes per site is stored as [block][plane][64 sites] of
// 16-byte vectors (8-byte for 16-bit links).  A wavefront's load of one plane is one contiguous
// 1 KB run, and all planes of a block sit next to each other, so the DRAM pages a wavefront
// touches are few and contiguous.  Plane k of a site is 64 vectors after plane k - 1, which the
// compiler folds into the load's immediate offset.  The site count is padded to a multiple of 64.
constexpr int kSB = 64;
HD int64_t padded_sites(int64_t vh) { return (vh + kSB - 1) & ~(int64_t)(kSB - 1); }

template <typename V>
DEV const V *site_ptr(const V *base, uint32_t s, int np) {
    return base + ((size_t)(s >> 6) * (size_t)np * kSB + (s & (kSB - 1)));
}
template <typename V>
DEV V *site_ptr(V *base, uint32_t s, int np) {
    return base + ((size_t)(s >> 6) * (size_t)np * kSB + (s & (kSB - 1)));
}

// Load / store N reals (a multiple of W) of site s, planes [p0, p0 + N / W) of a field with np planes.
template <typename S, int N>
DEV void load_planes(const typename St<S>::vec *__restrict__ base, int np, int p0, uint32_t s,
                     typename St<S>::acc *o) {
    constexpr int W = St<S>::W;
    const typename St<S>::vec *q = site_ptr(base, s, np) + p0 * kSB;
#pragma unroll
    for (int k = 0; k < N / W; ++k) St<S>::unpack(q[k * kSB], o + k * W);
}
template <typename S, int N>
DEV void store_planes(typename St<S>::vec *__restrict__ base, int np, int p0, uint32_t s,
                      const typename St<S>::acc *o) {
    constexpr int W = St<S>::W;
    typename St<S>::vec *q = site_ptr(base, s, np) + p0 * kSB;
#pragma unroll
    for (int k = 0; k < N / W; ++k) q[k * kSB] = St<S>::pack(o + k * W);
}
// whole-field shorthands: N reals per site in N / W planes
// Loads and stores with a non-temporal (streaming) hint, for data a kernel touches once, so that
// it does not displace data that other work-items of the kernel read again from the caches.
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
template <int B> struct RawOf;
template <> struct RawOf<16> { using type = u32x4_t; };
template <> struct RawOf<8> { using type = u32x2_t; };
template <typename V> DEV V ld_stream(const V *p) {
    using R = typename RawOf<sizeof(V)>::type;
    return __builtin_bit_cast(V, __builtin_nontemporal_load(reinterpret_cast<const R *>(p)));
}
DEV double ld_stream(const double *p) { return __builtin_nontemporal_load(p); }
DEV float ld_stream(const float *p) { return __builtin_nontemporal_load(p); }
DEV uint32_t ld_stream(const uint32_t *p) { return __builtin_nontemporal_load(p); }
template <typename V> DEV void st_stream(V *p, const V &v) {
    using R = typename RawOf<sizeof(V)>::type;
    __builtin_nontemporal_store(__builtin_bit_cast(R, v), reinterpret_cast<R *>(p));
}

template <typename S, int N, bool NT>
DEV void load_planes_h(const typename St<S>::vec *__restrict__ base, int np, int p0, uint32_t s,
                       typename St<S>::acc *o) {
    constexpr int W = St<S>::W;
    const typename St<S>::vec *q = site_ptr(base, s, np) + p0 * kSB;
#pragma unroll
    for (int k = 0; k < N / W; ++k) St<S>::unpack(NT ? ld_stream(q + k * kSB) : q[k * kSB], o + k * W);
}
template <typename S, int N, bool NT>
DEV void store_field_h(typename St<S>::vec *__restrict__ base, uint32_t s, const typename St<S>::acc *o) {
    constexpr int W = St<S>::W;
    typename St<S>::vec *q = site_ptr(base, s, N / W);
#pragma unroll
    for (int k = 0; k < N / W; ++k) {
        const typename St<S>::vec v = St<S>::pack(o + k * W);
        if constexpr (NT) st_stream(q + k * kSB, v);
        else q[k * kSB] = v;
    }
}

template <typename S, int N>
DEV void load_field(const typename St<S>::vec *__restrict__ base, uint32_t s, typename St<S>::acc *o) {
    load_planes<S, N>(base, N / St<S>::W, 0, s, o);
}
template <typename S, int N>
DEV void store_field(typename St<S>::vec *__restrict__ base, uint32_t s, const typename St<S>::acc *o) {
    store_planes<S, N>(base, N / St<S>::W, 0, s, o);
}

// ------------------------------------------------------------------ geometry
// Site of parity p with half index i: i = ((x0 L1 + x1) L2 + x2) (L3/2) + floor(x3/2),
// which is floor(Lambda / 2) (eq. (lexi) with x3 fastest).
struct Geom {
    int L[4];
    int h3;    // L3 / 2
    int vh;    // V / 2
    int vhp;   // V / 2 padded to a multiple of 64 (site blocks)
    int B[4];  // cache block of the OPENQXD user layout (B = L: the EO order)
    int cs;    // C* boundary conditions in directions 1 .. cs (0: none)
    int h1;    // L1 / 2: the shift of x1 on crossing the boundary of a C* direction mu >= 2
};

// Crossing the boundary of a C* direction mu >= 2 moves x1 into the mirror copy (C* boundary
// conditions on the lattice doubled in direction 1).
DEV int cstar_x1(const Geom &g, int mu, bool cross, int x1) {
    if (cross && mu >= 2 && mu <= g.cs) {
        x1 += g.h1;
        if (x1 >= 2 * g.h1) x1 -= 2 * g.h1;
    }
    return x1;
}

DEV void site_coords(const Geom &g, int i, int p, int x[4]) {
    int h = i % g.h3;
    int r = i / g.h3;
    x[2] = r % g.L[2];
    r /= g.L[2];
    x[1] = r % g.L[1];
    x[0] = r / g.L[1];
    x[3] = 2 * h + ((x[0] + x[1] + x[2] + p) & 1);
}
DEV int half_index(const Geom &g, const int x[4]) {
    return ((x[0] * g.L[1] + x[1]) * g.L[2] + x[2]) * g.h3 + (x[3] >> 1);
}
DEV int lex_index(const Geom &g, const int x[4]) {
    return ((x[0] * g.L[1] + x[1]) * g.L[2] + x[2]) * g.L[3] + x[3];
}
// eq. (ipt): openQxD's site index with cache block B, floor((V_B Lambda(n, N_B) + Lambda(b, B)) / 2)
// + P(x) V / 2 with b = x mod B, n = floor(x / B), N_B = L / B
DEV int64_t ipt_index(const Geom &g, const int x[4]) {
    int b[4], n[4], nb[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        b[m] = x[m] % g.B[m];
        n[m] = x[m] / g.B[m];
        nb[m] = g.L[m] / g.B[m];
    }
    const int64_t vb = (int64_t)g.B[0] * g.B[1] * g.B[2] * g.B[3];
    const int64_t lb = ((b[0] * g.B[1] + b[1]) * g.B[2] + b[2]) * g.B[3] + b[3];
    const int64_t ln = ((n[0] * nb[1] + n[1]) * nb[2] + n[2]) * nb[3] + n[3];
    const int par = (x[0] + x[1] + x[2] + x[3]) & 1;
    return (vb * ln + lb) / 2 + (int64_t)par * g.vh;
}
DEV void lex_coords(const Geom &g, int lam, int x[4]) {
    x[3] = lam % g.L[3];
    int r = lam / g.L[3];
    x[2] = r % g.L[2];
    r /= g.L[2];
    x[1] = r % g.L[1];
    x[0] = r / g.L[1];
}
DEV int wrap_up(int v, int L) { return v + 1 == L ? 0 : v + 1; }
DEV int wrap_dn(int v, int L) { return v == 0 ? L - 1 : v - 1; }

// Work-group order that gives each XCD a contiguous range of sites: dispatch sends
// work-group b to XCD b mod 8, so logical block (b mod 8) * (nb8 / 8) + b / 8 keeps
// neighbouring tiles (and their shared neighbour reads) in one XCD's L2.
DEV int xcd_block(int nb8) {
    int b = blockIdx.x;
    return (b & 7) * (nb8 >> 3) + (b >> 3);
}

// ------------------------------------------------------------------ link storage
// A link is 12 reals (rows 0 and 1 of the SU(3) matrix, row-major, (re, im)) in
// 12 / W planes of `vec`, plus one angle omega of type `om`.
template <typename S> struct Lk;
template <> struct Lk<double> {
    using vec = double2; using om = double; using acc = double; static constexpr int W = 2;
    static constexpr bool phase_pair = false;  // om is the angle omega itself
    static DEV void unpack(const vec &v, acc *o) { o[0] = v.x; o[1] = v.y; }
    static DEV vec pack(const double *o) { return make_double2(o[0], o[1]); }
};
template <> struct Lk<float> {
    using vec = float4; using om = float; using acc = float; static constexpr int W = 4;
    static constexpr bool phase_pair = false;
    static DEV void unpack(const vec &v, acc *o) { o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w; }
    static DEV vec pack(const double *o) { return make_float4((float)o[0], (float)o[1], (float)o[2], (float)o[3]); }
};
// 16-bit links store the phase as (cos omega, sin omega) in the same 16-bit format (low half cos,
// high half sin): 4 bytes, like an FP32 angle, and no sincos in the kernel.
template <> struct Lk<__half> {
    using vec = uint2; using om = uint32_t; using acc = float; static constexpr int W = 4;
    static constexpr bool phase_pair = true;
    static DEV void phase(om w, acc &co, acc &si) {
        const float2 f = __half22float2(*reinterpret_cast<const __half2 *>(&w));
        co = f.x;
        si = f.y;
    }
    static DEV om pack_phase(float co, float si) {
        const __half2 h = __floats2half2_rn(co, si);
        return *reinterpret_cast<const uint32_t *>(&h);
    }
    static DEV void unpack(const vec &v, acc *o) {
        const __half2 *h = reinterpret_cast<const __half2 *>(&v);
        float2 a = __half22float2(h[0]), b = __half22float2(h[1]);
        o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
    }
    static DEV vec pack(const double *o) {
        vec v;
        __half2 *h = reinterpret_cast<__half2 *>(&v);
        h[0] = __floats2half2_rn((float)o[0], (float)o[1]);
        h[1] = __floats2half2_rn((float)o[2], (float)o[3]);
        return v;
    }
};
template <> struct Lk<__hip_bfloat16> {
    using vec = uint2; using om = uint32_t; using acc = float; static constexpr int W = 4;
    static constexpr bool phase_pair = true;
    static DEV void phase(om w, acc &co, acc &si) {
        co = __uint_as_float(w << 16);
        si = __uint_as_float(w & 0xffff0000u);
    }
    static DEV om pack_phase(float co, float si) {
        return St<__hip_bfloat16>::rne(co) | (St<__hip_bfloat16>::rne(si) << 16);
    }
    static DEV void unpack(const vec &v, acc *o) {
        o[0] = __uint_as_float(v.x << 16); o[1] = __uint_as_float(v.x & 0xffff0000u);
        o[2] = __uint_as_float(v.y << 16); o[3] = __uint_as_float(v.y & 0xffff0000u);
    }
    static DEV vec pack(const double *o) {
        vec v;
        v.x = St<__hip_bfloat16>::rne((float)o[0]) | (St<__hip_bfloat16>::rne((float)o[1]) << 16);
        v.y = St<__hip_bfloat16>::rne((float)o[2]) | (St<__hip_bfloat16>::rne((float)o[3]) << 16);
        return v;
    }
};
