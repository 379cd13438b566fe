// Gauge-covariant parallel-transport convolution (PTC) network used as a learned
// preconditioner (a reading of the learned part; the paper has none):
//   y_c(x) = sum_{c'} sum_p W[p, c, c'] (T_p x_{c'})(x),   p in (0, +0, -0, +1, -1, +2, -2, +3, -3),
//   T_{+mu} psi(x) = V_mu(x) b+ psi(x + mu),  T_{-mu} psi(x) = V_mu(x - mu)^dag b- psi(x - mu),
// W a complex 4x4 spin matrix per (path, output, input) channel.  Activations are FP32 NATIVE
// full-lattice fields, one per channel; the working weights are BF16 (rounded from FP32 master
// weights); every product accumulates in FP32.
//   forward:   one thread per site, all output channels accumulated in registers;
//   backward:  input gradient = the same layer kernel with weights W'[q][c'][c] = W[adj q][c][c']^dag
//              (spin matrices commute with the transports, and T_p^dag = T_{adj p});
//              weight gradient dL/dW*[p,c,c'] = sum_{x, colour} g_c(x) (T_p x_{c'})(x)^dag, a
//              contraction over the sites done per 64-site tile in LDS, then reduced over tiles
//              in index order (deterministic);
//   Adam on (Re W, Im W) with FP32 state.
#include <cmath>
#include <vector>

#include "blas.h"
#include "dirac_ops.h"
#include "ptc.h"

namespace dl {
namespace {

constexpr int kPaths = 9;
constexpr int kTile = 64;  // sites per work-group of the weight-gradient kernel

struct PtcGeom {
    Geom g;
    const float4 *flinks[2];  // per parity: full FP32 links F = e^{i omega} U, [8 dir][5 planes] blocked
};

// The network's transports use the links with the U(1) and boundary phase folded in and the
// third row rebuilt, F_n(x) = e^{i omega_n(x)} U_n(x) as 9 complex numbers (row-major, 18 floats
// in 5 planes of float4, the last two floats unused), built once per context: the hop kernel's
// compressed form would cost a sincos and a cross product in every one of the 9 * c_in
// transports of a site.
constexpr int kFullPlanes = 5;

__global__ void k_full_links(Geom g, int p, const float4 *__restrict__ links, const float *__restrict__ omega,
                             float4 *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.vh) return;
    const size_t vhp = (size_t)g.vhp;
#pragma unroll 1
    for (int n = 0; n < 8; ++n) {
        const float4 *lb = site_ptr(links + (size_t)n * 3 * vhp, (uint32_t)i, 3);
        float u12[12];
#pragma unroll
        for (int k = 0; k < 3; ++k) Lk<float>::unpack(lb[k * kSB], u12 + 4 * k);
        C<float> u[6], r2[3];
#pragma unroll
        for (int k = 0; k < 6; ++k) u[k] = mk(u12[2 * k], u12[2 * k + 1]);
        third_row(u, r2);
        float si, co;
        sc(omega[(size_t)n * vhp + i], si, co);
        const C<float> ph = mk(co, si);
        float f[20];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const C<float> v = ph * u[k];
            f[2 * k] = v.r;
            f[2 * k + 1] = v.i;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const C<float> v = ph * r2[k];
            f[12 + 2 * k] = v.r;
            f[13 + 2 * k] = v.i;
        }
        f[18] = f[19] = 0.f;
        float4 *ob = site_ptr(out + (size_t)n * kFullPlanes * vhp, (uint32_t)i, kFullPlanes);
#pragma unroll
        for (int k = 0; k < kFullPlanes; ++k) ob[k * kSB] = make_float4(f[4 * k], f[4 * k + 1], f[4 * k + 2], f[4 * k + 3]);
    }
}

// Storage of an activation channel: a full NATIVE field (both parities), FP32 (six 16-byte
// planes of 4 reals per site) or BF16 (three planes of 8 reals).  The network's input and
// output and every gradient are FP32; its hidden activations are BF16, the precision in which
// the matrix cores read them anyway.
template <typename A> struct Act;
template <> struct Act<float> {
    using vec = float4;
    static constexpr int planes = 6;
};
template <> struct Act<__hip_bfloat16> {
    using vec = uint4;
    static constexpr int planes = 3;
};
using bf16s = __hip_bfloat16;
template <typename A> HD size_t chan_vecs(int vhp) { return (size_t)2 * Act<A>::planes * vhp; }  // per channel
template <typename A> HD size_t half_vecs(int vhp) { return (size_t)Act<A>::planes * vhp; }      // per parity

// Raw data of one transport: the (neighbour's) spinor and, for a hop, the full link.
template <typename A> struct TRaw {
    typename Act<A>::vec sp[Act<A>::planes];
    float4 lk[kFullPlanes];
};

// Load what T_path x_c needs at site (p, i) with coordinates x.  Every field of r is written on
// every path (the link is zero for the unshifted path), so the compiler keeps r in registers.
template <typename A>
DEV void transport_load(const PtcGeom &a, const typename Act<A>::vec *xc, int p, uint32_t i, const int x[4], int path,
                        TRaw<A> &r) {
    constexpr int NP = Act<A>::planes;
    const size_t hv = half_vecs<A>(a.g.vhp);
    const int n = path - 1;  // direction index 2 mu + back (path > 0)
    const int mu = n >> 1, back = n & 1;
    int y[4] = {x[0], x[1], x[2], x[3]};
    if (path > 0) {
        const int xm = mu == 0 ? x[0] : mu == 1 ? x[1] : mu == 2 ? x[2] : x[3];
        const int Lm = mu == 0 ? a.g.L[0] : mu == 1 ? a.g.L[1] : mu == 2 ? a.g.L[2] : a.g.L[3];
        const int xn = back ? (xm == 0 ? Lm - 1 : xm - 1) : (xm + 1 == Lm ? 0 : xm + 1);
        const bool cross = back ? xm == 0 : xm + 1 == Lm;
        if (mu == 0) y[0] = xn; else if (mu == 1) y[1] = xn; else if (mu == 2) y[2] = xn; else y[3] = xn;
        y[1] = cstar_x1(a.g, mu, cross, y[1]);  // C*: into the mirror copy
    }
    const uint32_t j = path > 0 ? (uint32_t)half_index(a.g, y) : i;
    const int q = path > 0 ? 1 - p : p;
    const typename Act<A>::vec *b = site_ptr(xc + q * hv, j, NP);
#pragma unroll
    for (int k = 0; k < NP; ++k) r.sp[k] = b[k * kSB];
    if (path > 0) {
        const float4 *lb = site_ptr(a.flinks[p] + (size_t)n * kFullPlanes * a.g.vhp, i, kFullPlanes);
#pragma unroll
        for (int k = 0; k < kFullPlanes; ++k) r.lk[k] = ld_stream(lb + k * kSB);  // read-once stream
    } else {
#pragma unroll
        for (int k = 0; k < kFullPlanes; ++k) r.lk[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

DEV void unpack4(const float4 *v, int nv, float *o) {
#pragma unroll
    for (int k = 0; k < nv; ++k) {
        o[4 * k] = v[k].x;
        o[4 * k + 1] = v[k].y;
        o[4 * k + 2] = v[k].z;
        o[4 * k + 3] = v[k].w;
    }
}
DEV void unpack_sp(const float4 *v, float *o) { unpack4(v, 6, o); }
DEV void unpack_sp(const uint4 *v, float *o) {
#pragma unroll
    for (int k = 0; k < 3; ++k) St<__hip_bfloat16>::unpack(v[k], o + 8 * k);
}

template <typename A>
DEV void transport_compute(const TRaw<A> &r, int path, C<float> t[12]) {
    float sp[24];
    unpack_sp(r.sp, sp);
    if (path == 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) t[k] = mk(sp[2 * k], sp[2 * k + 1]);
        return;
    }
    float lf[20];
    unpack4(r.lk, kFullPlanes, lf);
    C<float> f[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) f[k] = mk(lf[2 * k], lf[2 * k + 1]);
    const bool back = ((path - 1) & 1) != 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        C<float> ps[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) ps[b] = mk(sp[6 * s + 2 * b], sp[6 * s + 2 * b + 1]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            C<float> acc = mk(0.f, 0.f);
            if (back) {
#pragma unroll
                for (int b = 0; b < 3; ++b) cmadd(acc, f[3 * b + a], ps[b]);  // conj(F_ba) psi_b
            } else {
#pragma unroll
                for (int b = 0; b < 3; ++b) madd(acc, f[3 * a + b], ps[b]);
            }
            t[3 * s + a] = acc;
        }
    }
}

// t = T_path x_c at site (p, i)
template <typename A>
DEV void transport_site(const PtcGeom &a, const typename Act<A>::vec *xc, int p, uint32_t i, const int x[4],
                        int path, C<float> t[12]) {
    TRaw<A> r;
    transport_load<A>(a, xc, p, i, x, path, r);
    transport_compute<A>(r, path, t);
}

// Store 12 consecutive reals (reals 12 h .. 12 h + 11 of the 24, half h of the spinor) of site
// i of parity p of channel c.
DEV void store_half(float4 *base, int vhp, int c, int p, uint32_t i, int h, const float r[12]) {
    float4 *dst = site_ptr(base + c * chan_vecs<float>(vhp) + p * half_vecs<float>(vhp), i, 6) + 3 * h * kSB;
#pragma unroll
    for (int k = 0; k < 3; ++k) st_stream(dst + k * kSB, make_float4(r[4 * k], r[4 * k + 1], r[4 * k + 2], r[4 * k + 3]));
}
DEV void store_half(uint4 *base, int vhp, int c, int p, uint32_t i, int h, const float r[12]) {
    uint4 *site = site_ptr(base + c * chan_vecs<bf16s>(vhp) + p * half_vecs<bf16s>(vhp), i, 3);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int r0 = 12 * h + 4 * k;  // plane r0 / 8, half (r0 % 8) / 4 of it
        uint2 *dst = reinterpret_cast<uint2 *>(site + (r0 >> 3) * kSB) + ((r0 >> 2) & 1);
        const uint32_t lo = St<bf16s>::rne(r[4 * k]) | (St<bf16s>::rne(r[4 * k + 1]) << 16);
        const uint32_t hi = St<bf16s>::rne(r[4 * k + 2]) | (St<bf16s>::rne(r[4 * k + 3]) << 16);
        st_stream(dst, make_uint2(lo, hi));
    }
}

// ------------------------------------------------------------------ matrix-core layer
// The layer as a real GEMM on the 16x16x32 BF16 matrix cores (FP32 accumulation):
//   rows    m = 8 c + 2 sigma + ri_out          (output channel, spin, re/im)
//   columns n = (site, colour)                  (16 sites of a wavefront per tile, one colour per tile)
//   depth   k = 8 pair + 2 tau + ri_in,  pair = path * n_in + c' (path major: the four pairs of
//           a K step share one link, which the four lane groups load in one instruction; the
//           input-channel-major order was measured 1.5x slower, and channel groups outermost
//           with the paths into one neighbouring block consecutive fetched 5 % fewer bytes in
//           the same time)
// with the real embedding of the complex weights: (re, re) = (im, im) = Re W, (re, im) = -Im W,
// (im, re) = Im W.  A K step of 32 holds four (path, c') pairs; the lanes with k group g = lane / 16
// compute the transport T_path x_c' of pair 4 q + g at their site, and its 4 spins of colour a
// are exactly their 8 B-operand values for colour tile a, so each transport is computed once.
// The A operand (weights) is prepared once per weight update in the lane order of the
// instruction (row lane % 16, depth 8 (lane / 16) + j) and staged in LDS per work-group.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
typedef short s16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// A fragments of one layer: Af[(q * nm + t) * 64 + lane] = 8 BF16 values (uint4), q < nk, t < nm.
// W holds BF16 (re, im) pairs [9][nout][nin][4][4].
__global__ void k_ptc_afrag(int nin, int nout, int nk, int nm, const uint32_t *__restrict__ W,
                            uint4 *__restrict__ Af) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nk * nm * 64) return;
    const int lane = e & 63, t = (e >> 6) % nm, q = (e >> 6) / nm;
    const int m = 16 * t + (lane & 15), pair = 4 * q + (lane >> 4);
    const int c = m >> 3, sg = (m >> 1) & 3, rio = m & 1;
    uint32_t v[4] = {0u, 0u, 0u, 0u};
    if (c < nout && pair < kPaths * nin) {
        const int path = pair / nin, cp = pair % nin;
        const uint32_t *w = W + ((size_t)(path * nout + c) * nin + cp) * 16 + sg * 4;
#pragma unroll
        for (int tau = 0; tau < 4; ++tau) {
            const uint32_t re = w[tau] & 0xffffu, im = w[tau] >> 16;
            // (ri_out, ri_in = 0) and (ri_out, ri_in = 1)
            const uint32_t lo = rio ? im : re, hi = rio ? re : (im ^ 0x8000u);
            v[tau] = lo | (hi << 16);
        }
    }
    Af[e] = make_uint4(v[0], v[1], v[2], v[3]);
}

// A fragments of the contraction z = W x of a contract-first last layer (one output channel) on
// the 16x16x16 BF16 matrix cores: rows m = 8 p + 2 sigma + ri_out (path, spin, re/im; 5 tiles,
// the last half empty), depth k = 8 c' + 2 tau + ri_in (the previous layer's output rows, NM tiles
// of 16).  Az[(tz * nm + t) * 64 + lane] = 4 BF16 values (uint2): row 16 tz + lane % 16, depth
// 16 t + 4 (lane / 16) + j.  W holds BF16 (re, im) pairs [9][1][nin][4][4].
constexpr int kZTiles = 5;
__global__ void k_ptc_zfrag(int nin, int nm, const uint32_t *__restrict__ W, uint2 *__restrict__ Az) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kZTiles * nm * 64) return;
    const int lane = e & 63, t = (e >> 6) % nm, tz = (e >> 6) / nm;
    const int m = 16 * tz + (lane & 15);
    const int path = m >> 3, sg = (m >> 1) & 3, rio = m & 1;
    uint32_t h[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = 16 * t + 4 * (lane >> 4) + j;
        const int cp = k >> 3, tau = (k >> 1) & 3, rii = k & 1;
        if (path < kPaths && cp < nin) {
            const uint32_t w = W[((size_t)path * nin + cp) * 16 + sg * 4 + tau];
            const uint32_t re = w & 0xffffu, im = w >> 16;
            // (re, re) = (im, im) = Re W, (re, im) = -Im W, (im, re) = Im W
            h[j] = rio == rii ? re : (rio ? im : (im ^ 0x8000u));
        }
    }
    Az[e] = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
}

constexpr int kEoIn = 1, kEoOut = 2;  // even-odd deployment flags of the layer kernel

// One layer on the matrix cores.  Persistent: the grid's work-groups (4 wavefronts, 16 sites
// each) sweep the 64-site blocks of both parities; the A fragments are staged once per
// work-group.  NIN input channels, NM = ceil(8 NOUT / 16) row tiles.
// ZOUT: the next layer is a contract-first last layer; its contractions z_p = sum_c' W[p][c'] y_c'
// (p < 9) are formed from this layer's accumulators in registers -- the 16x16 accumulator tile t
// of a lane is, rounded to BF16, its B operand of depth step t on the 16x16x16 instruction -- and
// written to zout as 9 channels; y itself is written only when store_y is set.
template <int NIN, int NM, bool ZOUT, typename AI, typename AO>
__global__ __launch_bounds__(256, 2) void k_ptc_layer_mfma(PtcGeom a, int nout, const uint4 *__restrict__ Af,
                                                        const typename Act<AI>::vec *__restrict__ xin,
                                                        typename Act<AO>::vec *__restrict__ yout,
                                                        const uint2 *__restrict__ Az, float4 *__restrict__ zout,
                                                        int store_y, int eo) {
    constexpr int NPAIR = kPaths * NIN, NK = (NPAIR + 3) / 4;
    __shared__ uint4 af[NK * NM * 64];
    for (int e = threadIdx.x; e < NK * NM * 64; e += 256) af[e] = Af[e];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, sl = lane & 15;
    const int nbp = (a.g.vh + 63) / 64;
    const size_t chin = chan_vecs<AI>(a.g.vhp);
#pragma nounroll
    for (int blk = blockIdx.x; blk < 2 * nbp; blk += gridDim.x) {
        const int p = blk >= nbp;
        const int b = blk - p * nbp;
        const int i = b * 64 + wave * 16 + sl;
        const bool on = i < a.g.vh;
        // A lane past the end of the lattice computes the transports of the last site: the
        // matrix-core output column of a site depends on that site's B column alone, and its
        // results are not stored.  Depth slots past the last (path, c') pair load pair NPAIR - 1;
        // their A fragments are zero, and the loaded values are finite.
        const uint32_t ic = on ? (uint32_t)i : (uint32_t)(a.g.vh - 1);
        int x[4];
        site_coords(a.g, (int)ic, p, x);
        f32x4_t acc[NM][3];
#pragma unroll
        for (int t = 0; t < NM; ++t)
#pragma unroll
            for (int col = 0; col < 3; ++col) acc[t][col] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        auto pair_of = [&](int q) {
            const int pr = 4 * q + g;
            if constexpr (NPAIR % 4 != 0) return pr < NPAIR ? pr : NPAIR - 1;
            return pr;
        };
        auto load = [&](int q, TRaw<AI> &r) {
            const int pair = pair_of(q);
            transport_load<AI>(a, xin + (size_t)(pair % NIN) * chin, p, ic, x, pair / NIN, r);
        };
        auto step = [&](int q, const TRaw<AI> &r) {
            C<float> tr[12];
            transport_compute<AI>(r, pair_of(q) / NIN, tr);
            bf16x8_t b[3];
#pragma unroll
            for (int col = 0; col < 3; ++col) {
#pragma unroll
                for (int tau = 0; tau < 4; ++tau) {
                    b[col][2 * tau] = (__bf16)tr[3 * tau + col].r;  // round to nearest even
                    b[col][2 * tau + 1] = (__bf16)tr[3 * tau + col].i;
                }
            }
#pragma unroll
            for (int t = 0; t < NM; ++t) {
                const bf16x8_t A = __builtin_bit_cast(bf16x8_t, af[(q * NM + t) * 64 + lane]);
#pragma unroll
                for (int col = 0; col < 3; ++col)
                    acc[t][col] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, b[col], acc[t][col], 0, 0, 0);
            }
        };
        // software pipeline over three register sets in turn: the loads of K step q + 2 are
        // issued before the transport and the matrix-core work of step q
        // kEoIn: the input's odd half is zero, so at an even site every path but the unshifted
        // one transports zeros; its K steps after those of path 0 add exact zeros and are skipped
        const int nk = ((eo & kEoIn) && p == 0) ? (NIN + 3) / 4 : NK;
        TRaw<AI> ra, rb, rc;
        load(0, ra);
        if (1 < nk) load(1, rb);
#pragma nounroll
        for (int q = 0; q < nk; q += 3) {
            if (q + 2 < nk) load(q + 2, rc);
            step(q, ra);
            if (q + 1 < nk) {
                if (q + 3 < nk) load(q + 3, ra);
                step(q + 1, rb);
            }
            if (q + 2 < nk) {
                if (q + 4 < nk) load(q + 4, rb);
                step(q + 2, rc);
            }
        }
        // lane (g, site) holds rows m = 16 t + 4 g + r, r < 4: channel 2 t + g / 2, spins
        // 2 (g & 1) + r / 2, re/im r & 1 -- twelve consecutive reals (three planes) of one spinor
        auto store_tile = [&](const f32x4_t (&v)[3], auto *base, int c) {
            float r[12];
#pragma unroll
            for (int rr = 0; rr < 4; ++rr)
#pragma unroll
                for (int col = 0; col < 3; ++col) r[6 * (rr >> 1) + 2 * col + (rr & 1)] = v[col][rr];
            store_half(base, a.g.vhp, c, p, (uint32_t)i, g & 1, r);
        };
        if (!ZOUT || store_y) {
            if (on) {
#pragma unroll
                for (int t = 0; t < NM; ++t)
                    if (2 * t + (g >> 1) < nout) store_tile(acc[t], yout, 2 * t + (g >> 1));
            }
        }
        if constexpr (ZOUT) {
            // every lane takes part in the matrix-core steps; only the stores are masked.  One
            // output tile at a time keeps the extra accumulators at 12 registers.
            // kEoOut: only the even half of the network's output is wanted, which reads z_0 at even
            // sites and z_1 .. z_8 at odd ones
            const bool eo_out = (eo & kEoOut) != 0;
            const int ntz = eo_out && p == 0 ? 1 : kZTiles;
#pragma nounroll
            for (int tz = 0; tz < ntz; ++tz) {
                f32x4_t zacc[3];
#pragma unroll
                for (int col = 0; col < 3; ++col) zacc[col] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int t = 0; t < NM; ++t) {
                    const s16x4_t A = __builtin_bit_cast(s16x4_t, Az[(tz * NM + t) * 64 + lane]);
#pragma unroll
                    for (int col = 0; col < 3; ++col) {
                        bf16x4_t b;
#pragma unroll
                        for (int rr = 0; rr < 4; ++rr) b[rr] = (__bf16)acc[t][col][rr];
                        zacc[col] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, __builtin_bit_cast(s16x4_t, b),
                                                                              zacc[col], 0, 0, 0);
                    }
                }
                const int pz = 2 * tz + (g >> 1);
                const bool want = !eo_out || (p == 0 ? pz == 0 : pz > 0);
                if (on && pz < kPaths && want) store_tile(zacc, zout, pz);
            }
        }
    }
}

// y(x) = sum_p (T_p z_p)(x): the transports of a contract-first last layer (one output channel),
// one thread per site of either parity, the nine terms added in path order in FP32.
__global__ __launch_bounds__(256) void k_ptc_tsum(PtcGeom a, int nparity, const float4 *__restrict__ z,
                                                  float4 *__restrict__ y) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nparity * a.g.vh) return;
    const int p = s >= a.g.vh;
    const uint32_t i = (uint32_t)(s - p * a.g.vh);
    int x[4];
    site_coords(a.g, (int)i, p, x);
    const size_t chz = chan_vecs<float>(a.g.vhp);
    C<float> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = mk(0.f, 0.f);
#pragma nounroll
    for (int path = 0; path < kPaths; ++path) {
        C<float> t[12];
        transport_site<float>(a, z + (size_t)path * chz, p, i, x, path, t);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            acc[k].r += t[k].r;
            acc[k].i += t[k].i;
        }
    }
    float4 *dst = site_ptr(y + p * half_vecs<float>(a.g.vhp), i, 6);
#pragma unroll
    for (int k = 0; k < 6; ++k)
        st_stream(dst + k * kSB, make_float4(acc[2 * k].r, acc[2 * k].i, acc[2 * k + 1].r, acc[2 * k + 1].i));
}

// Partial weight gradients: part[wg][path][c][c'][s][t] (complex float), one slice per work-group.
// Persistent: work-group wg takes the 64-site tiles wg, wg + G, wg + 2G, ... (G = grid size) and
// sums their contributions into its slice in that order.  Per tile, four wavefronts: the gradient
// of the tile (all output channels) is staged in LDS once, as [site][colour][row] with the
// R = 4 NOUT rows (c, s) innermost; then each wavefront takes one (path, c') pair at a time and
// computes its transport at the 64 sites into its own LDS slot, as [site][colour][t].  The pair's
// 4 NOUT x 4 block of outputs is formed by the wavefront's 64 lanes as R rows x S = 64 / R site
// classes: lane (class k, row) sums g_row conj(t_t) for all four t over the sites k, k + S, ...
// (site, then colour, in index order; one read of g feeds four products and the transport reads
// are shared by the R lanes of a class), then the S class sums of a row are combined by a
// butterfly over the lanes, which gives every lane the same bits.  The running sums of a slice
// belong to one lane each: no atomics, deterministic.
template <int NOUT, typename AI>
__global__ __launch_bounds__(256) void k_ptc_wgrad(PtcGeom a, int nin, const typename Act<AI>::vec *__restrict__ xin,
                                                   const float4 *__restrict__ g, float2 *__restrict__ part) {
    constexpr int R = 4 * NOUT, S = kTile / R;
    static_assert(kTile % R == 0, "the rows of a pair must divide the tile");
    constexpr int GX = 3 * R + 1;  // complex per site in gs (one of padding: the staging writes of
                                   // the 64 sites then fall in distinct banks)
    constexpr int TX = 14;         // complex per site in ts (12 + 2: 16-byte rows, staggered banks)
    __shared__ float2 gs[kTile * GX];
    __shared__ float4 ts[4][kTile * TX / 2];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kTile - 1);
    const int row = lane % R, cls = lane / R;  // this lane's output row (c, s) and site class
    const int ntile = (2 * a.g.vh + kTile - 1) / kTile;
    const size_t chg = chan_vecs<float>(a.g.vhp), hg = half_vecs<float>(a.g.vhp), chin = chan_vecs<AI>(a.g.vhp);
    const int npair = kPaths * nin;
    float2 *slice = part + (size_t)blockIdx.x * npair * NOUT * 16;
    float4 *tw = ts[wave];
#pragma nounroll
    for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const bool first = tile == (int)blockIdx.x;
        const int s = tile * kTile + lane;
        const bool on = s < 2 * a.g.vh;
        const int p = on && s >= a.g.vh;
        const uint32_t i = on ? (uint32_t)(s - p * a.g.vh) : 0u;
        int x[4] = {0, 0, 0, 0};
        if (on) site_coords(a.g, (int)i, p, x);
        __syncthreads();  // the previous tile's reads of gs and ts are done
        for (int c = wave; c < NOUT; c += 4) {
            float r[24];
            if (on) load_field<float, 24>(g + c * chg + p * hg, i, r);
#pragma unroll
            for (int ss = 0; ss < 4; ++ss)
#pragma unroll
                for (int col = 0; col < 3; ++col)
                    gs[lane * GX + col * R + 4 * c + ss] =
                        on ? make_float2(r[2 * (3 * ss + col)], r[2 * (3 * ss + col) + 1]) : make_float2(0.f, 0.f);
        }
        // the gathers of a wavefront's next pair are issued before the reduction of the current one
        TRaw<AI> raw;
        if (on && wave < npair) transport_load<AI>(a, xin + (wave % nin) * chin, p, i, x, wave / nin, raw);
#pragma nounroll
        for (int base = 0; base < npair; base += 4) {
            const int pr = base + wave;
            const int path = pr / nin, cp = pr % nin;
            C<float> t[12];
            if (on && pr < npair) {
                transport_compute<AI>(raw, path, t);
            } else {
#pragma unroll
                for (int k = 0; k < 12; ++k) t[k] = mk(0.f, 0.f);
            }
            const int nx = pr + 4;
            if (on && nx < npair) transport_load<AI>(a, xin + (nx % nin) * chin, p, i, x, nx / nin, raw);
            __syncthreads();  // the previous pairs' reads of ts (and the staging of gs) are done
#pragma unroll
            for (int col = 0; col < 3; ++col)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    tw[lane * (TX / 2) + 2 * col + h] = make_float4(t[3 * (2 * h) + col].r, t[3 * (2 * h) + col].i,
                                                                    t[3 * (2 * h + 1) + col].r, t[3 * (2 * h + 1) + col].i);
            __syncthreads();
            if (pr < npair) {
                float ar[4] = {0.f, 0.f, 0.f, 0.f}, ai[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
                for (int j = 0; j < R; ++j) {
                    const int xs = j * S + cls;
#pragma unroll
                    for (int col = 0; col < 3; ++col) {
                        // g_row[col] conj(t_t[col]), t = 0..3
                        const float2 gv = gs[xs * GX + col * R + row];
                        const float4 t01 = tw[xs * (TX / 2) + 2 * col], t23 = tw[xs * (TX / 2) + 2 * col + 1];
                        const float tr[4] = {t01.x, t01.z, t23.x, t23.z}, ti[4] = {t01.y, t01.w, t23.y, t23.w};
#pragma unroll
                        for (int tt = 0; tt < 4; ++tt) {
                            ar[tt] = fmaf(gv.y, ti[tt], fmaf(gv.x, tr[tt], ar[tt]));
                            ai[tt] = fmaf(-gv.x, ti[tt], fmaf(gv.y, tr[tt], ai[tt]));
                        }
                    }
                }
#pragma unroll
                for (int o = R; o < kTile; o <<= 1)
#pragma unroll
                    for (int tt = 0; tt < 4; ++tt) {
                        ar[tt] += __shfl_xor(ar[tt], o, 64);
                        ai[tt] += __shfl_xor(ai[tt], o, 64);
                    }
                if (cls == 0) {
                    const int c = row >> 2, ss = row & 3;
                    float4 *dst = (float4 *)(slice + ((size_t)path * NOUT * nin + (size_t)c * nin + cp) * 16 + ss * 4);
                    if (first) {
                        dst[0] = make_float4(ar[0], ai[0], ar[1], ai[1]);
                        dst[1] = make_float4(ar[2], ai[2], ar[3], ai[3]);
                    } else {
                        const float4 o0 = dst[0], o1 = dst[1];
                        dst[0] = make_float4(o0.x + ar[0], o0.y + ai[0], o0.z + ar[1], o0.w + ai[1]);
                        dst[1] = make_float4(o1.x + ar[2], o1.y + ai[2], o1.z + ar[3], o1.w + ai[3]);
                    }
                }
            }
        }
    }
}

// out[k] += sum_b part[b][k] (b ascending), k < n complex entries.  A work-group of 256 threads
// takes 64 entries; wavefront w sums the partials b = w, w + 4, ... in FP64 and the four sums
// are added in the order w = 0..3 (deterministic).
constexpr int kRedK = 64;
__global__ __launch_bounds__(256) void k_ptc_reduce(int nblk, int n, const float2 *__restrict__ part,
                                                    float2 *__restrict__ out) {
    __shared__ double2 sum[4][kRedK];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int k = blockIdx.x * kRedK + l;
    double re = 0.0, im = 0.0;
    if (k < n) {
        for (int b = w; b < nblk; b += 4) {
            const float2 v = part[(size_t)b * n + k];
            re += v.x;
            im += v.y;
        }
    }
    sum[w][l] = make_double2(re, im);
    __syncthreads();
    if (w == 0 && k < n) {
        for (int j = 1; j < 4; ++j) {
            re += sum[j][l].x;
            im += sum[j][l].y;
        }
        out[k].x += (float)re;
        out[k].y += (float)im;
    }
}

// Adam on n real parameters (interleaved re, im); writes the BF16 working copy
// omb1 = 1 - b1 and omb2 = 1 - b2 come rounded once from their exact values: 1 - b2 formed in FP32
// from the rounded b2 = 0.999f would be 1.3e-5 off in relative terms.
__global__ void k_adam(int n, float *__restrict__ w, const float *__restrict__ grad_conj, float *__restrict__ m,
                       float *__restrict__ v, uint16_t *__restrict__ wbf, float lr, float b1, float omb1, float b2,
                       float omb2, float eps, float c1, float c2) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float g = 2.0f * grad_conj[k];  // dL/d(Re W) = 2 Re dL/dW*, dL/d(Im W) = 2 Im dL/dW*
    const float mk_ = b1 * m[k] + omb1 * g;
    const float vk = b2 * v[k] + omb2 * g * g;
    m[k] = mk_;
    v[k] = vk;
    const float nw = w[k] - lr * (mk_ / c1) / (sqrtf(vk / c2) + eps);
    w[k] = nw;
    wbf[k] = (uint16_t)St<__hip_bfloat16>::rne(nw);
}

__global__ void k_to_bf16(int n, const float *__restrict__ w, uint16_t *__restrict__ wbf) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) wbf[k] = (uint16_t)St<__hip_bfloat16>::rne(w[k]);
}

// W'[q][c'][c] = W[adj q][c][c']^dag (spin 4x4), on BF16 pairs (exact: a permutation and sign flips)
__global__ void k_adjoint_weights(int nout, int nin, const uint32_t *__restrict__ W, uint32_t *__restrict__ Wt) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int total = kPaths * nin * nout * 16;
    if (k >= total) return;
    const int st = k & 15, ss = st >> 2, tt = st & 3;
    int r = k >> 4;
    const int c = r % nout;  // Wt index [q][c'][c]: c fastest
    r /= nout;
    const int cp = r % nin;
    const int q = r / nin;
    const int adj[kPaths] = {0, 2, 1, 4, 3, 6, 5, 8, 7};
    const uint32_t w = W[((size_t)(adj[q] * nout + c) * nin + cp) * 16 + tt * 4 + ss];  // transpose
    Wt[k] = w ^ 0x80000000u;                                                              // conjugate
}

int compute_units() {
    static int n = 0;
    if (!n) {
        int dev = 0, v = 0;
        HIP_CHECK(hipGetDevice(&dev));
        HIP_CHECK(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev));
        n = v > 0 ? v : 256;
    }
    return n;
}
int row_tiles(int nout) { return (8 * nout + 15) / 16; }
int k_steps(int nin) { return (kPaths * nin + 3) / 4; }
size_t afrag_count(int nin, int nout) { return (size_t)k_steps(nin) * row_tiles(nout) * 64; }
size_t zfrag_count(int nin) { return (size_t)kZTiles * row_tiles(nin) * 64; }

void build_zfrags(int nin, const uint32_t *W, uint2 *Az, hipStream_t s) {
    const int n = (int)zfrag_count(nin);
    k_ptc_zfrag<<<(n + 255) / 256, 256, 0, s>>>(nin, row_tiles(nin), W, Az);
    HIP_CHECK(hipGetLastError());
}

void build_afrags(int nin, int nout, const uint32_t *W, uint4 *Af, hipStream_t s) {
    const int n = (int)afrag_count(nin, nout);
    k_ptc_afrag<<<(n + 255) / 256, 256, 0, s>>>(nin, nout, k_steps(nin), row_tiles(nout), W, Af);
    HIP_CHECK(hipGetLastError());
}

// Storage of a layer's input and output: FP32 -> FP32 (the input-gradient pass, and a network of
// one layer), FP32 -> BF16 (the first layer), BF16 -> BF16 (the hidden layers).
enum class Io { F32, In, Mid };
// The optional ZOUT arguments (Az, z, store_y) select the variant that also forms the
// contractions of a contract-first last layer.
struct ZArgs {
    const uint2 *Az = nullptr;
    void *z = nullptr;
    bool store_y = true;
    int eo = 0;  // kEoIn, kEoOut
};
template <int NIN, int NM, bool ZOUT, typename AI, typename AO>
void launch_io(int grid, const PtcGeom &a, int nout, const uint4 *Af, const void *x, void *y, const ZArgs &zo,
               hipStream_t s) {
    k_ptc_layer_mfma<NIN, NM, ZOUT, AI, AO><<<grid, 256, 0, s>>>(
        a, nout, Af, (const typename Act<AI>::vec *)x, (typename Act<AO>::vec *)y, zo.Az, (float4 *)zo.z,
        zo.store_y ? 1 : 0, zo.eo);
}
template <int NIN, int NM>
void launch_layer(const PtcGeom &a, int nout, const uint4 *Af, const void *x, void *y, const ZArgs &zo, Io io,
                  hipStream_t s) {
    const int nblk = 2 * (int)((a.g.vh + 63) / 64);
    const int grid = std::min(nblk, 2 * compute_units());
    if (zo.z) {
        if (io == Io::In) launch_io<NIN, NM, true, float, bf16s>(grid, a, nout, Af, x, y, zo, s);
        else if (io == Io::Mid) launch_io<NIN, NM, true, bf16s, bf16s>(grid, a, nout, Af, x, y, zo, s);
        else throw Error(DIRAC_EUNSUPPORTED, "contract-first epilogue needs a BF16 layer output");
    } else {
        if (io == Io::In) launch_io<NIN, NM, false, float, bf16s>(grid, a, nout, Af, x, y, zo, s);
        else if (io == Io::Mid) launch_io<NIN, NM, false, bf16s, bf16s>(grid, a, nout, Af, x, y, zo, s);
        else launch_io<NIN, NM, false, float, float>(grid, a, nout, Af, x, y, zo, s);
    }
}
template <int NIN>
void launch_layer_nm(const PtcGeom &a, int nout, const uint4 *Af, const void *x, void *y, const ZArgs &zo, Io io,
                     hipStream_t s) {
    switch (row_tiles(nout)) {
        case 1: launch_layer<NIN, 1>(a, nout, Af, x, y, zo, io, s); break;
        case 2: launch_layer<NIN, 2>(a, nout, Af, x, y, zo, io, s); break;
        default: launch_layer<NIN, 4>(a, nout, Af, x, y, zo, io, s); break;
    }
}
// y = layer(x) with the A fragments Af of a (nin -> nout) layer
void layer_dispatch(const PtcGeom &a, int nin, int nout, const void *x, const uint4 *Af, void *y, Io io, hipStream_t s,
                    const ZArgs &zo = ZArgs()) {
    switch (nin) {
        case 1: launch_layer_nm<1>(a, nout, Af, x, y, zo, io, s); break;
        case 2: launch_layer_nm<2>(a, nout, Af, x, y, zo, io, s); break;
        case 4: launch_layer_nm<4>(a, nout, Af, x, y, zo, io, s); break;
        case 8: launch_layer_nm<8>(a, nout, Af, x, y, zo, io, s); break;
        default: throw Error(DIRAC_EUNSUPPORTED, "PTC channel counts must be 1, 2, 4 or 8");
    }
    HIP_CHECK(hipGetLastError());
}
// work-groups of the weight-gradient kernel: as many per compute unit as its LDS tiles and
// registers let run at once (three for one or two output channels, two for four or eight), at
// most one per tile
int wgrad_grid(size_t vh, int nout) {
    const size_t ntile = (2 * vh + kTile - 1) / kTile;
    return (int)std::min(ntile, (size_t)(nout <= 2 ? 3 : 2) * compute_units());
}
template <int NOUT>
void launch_wgrad(const PtcGeom &a, int nin, const void *x, bool x_bf16, const void *g, void *part, hipStream_t s) {
    if (x_bf16)
        k_ptc_wgrad<NOUT, bf16s><<<wgrad_grid(a.g.vh, NOUT), 256, 0, s>>>(a, nin, (const uint4 *)x, (const float4 *)g,
                                                                    (float2 *)part);
    else
        k_ptc_wgrad<NOUT, float><<<wgrad_grid(a.g.vh, NOUT), 256, 0, s>>>(a, nin, (const float4 *)x, (const float4 *)g,
                                                                    (float2 *)part);
}
void wgrad_dispatch(const PtcGeom &a, int nin, int nout, const void *x, bool x_bf16, const void *g, void *part,
                    hipStream_t s) {
    switch (nout) {
        case 1: launch_wgrad<1>(a, nin, x, x_bf16, g, part, s); break;
        case 2: launch_wgrad<2>(a, nin, x, x_bf16, g, part, s); break;
        case 4: launch_wgrad<4>(a, nin, x, x_bf16, g, part, s); break;
        case 8: launch_wgrad<8>(a, nin, x, x_bf16, g, part, s); break;
        default: throw Error(DIRAC_EUNSUPPORTED, "PTC output channels must be 1, 2, 4 or 8");
    }
    HIP_CHECK(hipGetLastError());
}

PtcGeom geom_of(dirac_ctx *c, hipStream_t s) {
    ensure_prec(c, DIRAC_F32, s);
    if (!c->ptc_links_ready) {
        const size_t per = (size_t)8 * kFullPlanes * c->g.vhp * sizeof(float4);
        for (int p = 0; p < 2; ++p) {
            c->ptc_links[p].alloc(per);
            k_full_links<<<grid_for(c->vh), kBlock, 0, s>>>(c->g, p, (const float4 *)c->f[DIRAC_F32].links[p].p,
                                                            (const float *)c->f[DIRAC_F32].omega[p].p,
                                                            (float4 *)c->ptc_links[p].p);
            HIP_CHECK(hipGetLastError());
        }
        c->ptc_links_ready = true;
    }
    PtcGeom a;
    a.g = c->g;
    for (int p = 0; p < 2; ++p) a.flinks[p] = (const float4 *)c->ptc_links[p].p;
    return a;
}

}  // namespace

size_t ptc_nweights(const dirac_ptc *n, int l) { return (size_t)kPaths * n->ch[l] * n->ch[l + 1] * 16; }

void ptc_alloc(dirac_ptc *n) {
    size_t tot = 0;
    for (int l = 0; l < n->nlayers; ++l) {
        n->off[l] = tot;
        tot += ptc_nweights(n, l);
    }
    n->total = tot;  // complex entries
    size_t fw = 0, fb = 0;
    for (int l = 0; l < n->nlayers; ++l) {
        n->afw_off[l] = fw;
        n->afb_off[l] = fb;
        fw += afrag_count(n->ch[l], n->ch[l + 1]);
        fb += afrag_count(n->ch[l + 1], n->ch[l]);
    }
    n->afw.alloc(fw * sizeof(uint4));
    n->afb.alloc(fb * sizeof(uint4));
    if (n->contract_last()) n->afz.alloc(zfrag_count(n->ch[n->nlayers - 1]) * sizeof(uint2));
    n->w.alloc(tot * 8);
    n->wbf.alloc(tot * 4);
    n->wt.alloc(tot * 4);
    n->grad.alloc(tot * 8);
    n->m.alloc(tot * 8);
    n->v.alloc(tot * 8);
    HIP_CHECK(hipMemset(n->w.p, 0, tot * 8));
    HIP_CHECK(hipMemset(n->wbf.p, 0, tot * 4));
    HIP_CHECK(hipMemset(n->grad.p, 0, tot * 8));
    HIP_CHECK(hipMemset(n->m.p, 0, tot * 8));
    HIP_CHECK(hipMemset(n->v.p, 0, tot * 8));
    n->step = 0;
}

// forward A fragments of every layer from the BF16 working weights
static void refresh_afrags(dirac_ptc *n, hipStream_t s) {
    for (int l = 0; l < n->nlayers; ++l)
        build_afrags(n->ch[l], n->ch[l + 1], (const uint32_t *)n->wbf.p + n->off[l], (uint4 *)n->afw.p + n->afw_off[l],
                     s);
    if (n->contract_last()) {
        const int l = n->nlayers - 1;
        build_zfrags(n->ch[l], (const uint32_t *)n->wbf.p + n->off[l], (uint2 *)n->afz.p, s);
    }
}

void ptc_refresh_bf16(dirac_ptc *n, hipStream_t s) {
    const int nr = (int)(2 * n->total);
    k_to_bf16<<<(nr + 255) / 256, 256, 0, s>>>(nr, (const float *)n->w.p, (uint16_t *)n->wbf.p);
    HIP_CHECK(hipGetLastError());
    refresh_afrags(n, s);
}

// Activation l is stored in BF16 when it is a hidden layer's (0 < l < nlayers), else in FP32.
static bool act_bf16(const dirac_ptc *n, int l) { return l > 0 && l < n->nlayers; }
static size_t act_chan_bytes(const dirac_ctx *c, const dirac_ptc *n, int l) {
    return act_bf16(n, l) ? chan_vecs<bf16s>(c->g.vhp) * sizeof(uint4) : chan_vecs<float>(c->g.vhp) * sizeof(float4);
}

void ptc_ensure_acts(dirac_ctx *c, dirac_ptc *n) {
    const size_t chanb = chan_vecs<float>(c->g.vhp) * sizeof(float4);
    size_t need = 0;
    for (int l = 0; l <= n->nlayers; ++l) need += (size_t)n->ch[l] * act_chan_bytes(c, n, l);
    n->acts.alloc(need);
    int maxc = 0;
    for (int l = 0; l <= n->nlayers; ++l) maxc = std::max(maxc, n->ch[l]);
    n->gbuf.alloc(2 * (size_t)maxc * chanb);
    if (n->contract_last()) n->zbuf.alloc((size_t)kPaths * chanb);
    size_t maxpart = 0;  // complex entries of the weight-gradient slices of the largest layer
    for (int l = 0; l < n->nlayers; ++l)
        maxpart = std::max(maxpart, (size_t)wgrad_grid(c->vh, n->ch[l + 1]) * ptc_nweights(n, l));
    n->part.alloc(maxpart * 8);
}

float *ptc_act(dirac_ctx *c, dirac_ptc *n, int l) {
    size_t off = 0;
    for (int k = 0; k < l; ++k) off += (size_t)n->ch[k] * act_chan_bytes(c, n, k);
    return (float *)((char *)n->acts.p + off);
}

// forward: acts[0] must hold the input; leaves the output in acts[nlayers] and, with keep_all,
// every layer's output in acts[l + 1] (the backward pass needs them).  With eo the input's odd
// half must be zero, and only the even half of the output is formed (a network of one layer
// forms both).
void ptc_forward_acts(dirac_ctx *c, dirac_ptc *n, hipStream_t s, bool keep_all, bool eo) {
    PtcGeom a = geom_of(c, s);
    const int L = n->nlayers;
    const bool cf = n->contract_last();
    for (int l = 0; l < (cf ? L - 1 : L); ++l) {
        ZArgs zo;
        if (cf && l == L - 2) {
            zo.Az = (const uint2 *)n->afz.p;
            zo.z = n->zbuf.p;
            zo.store_y = keep_all;
            if (eo) zo.eo |= kEoOut;
        }
        if (eo && l == 0) zo.eo |= kEoIn;
        const Io io = act_bf16(n, l + 1) ? (act_bf16(n, l) ? Io::Mid : Io::In) : Io::F32;
        layer_dispatch(a, n->ch[l], n->ch[l + 1], ptc_act(c, n, l), (const uint4 *)n->afw.p + n->afw_off[l],
                       ptc_act(c, n, l + 1), io, s, zo);
    }
    if (cf) {
        const int npar = eo ? 1 : 2;
        k_ptc_tsum<<<(int)((npar * c->vh + 255) / 256), 256, 0, s>>>(a, npar, (const float4 *)n->zbuf.p,
                                                                     (float4 *)ptc_act(c, n, L));
        HIP_CHECK(hipGetLastError());
    }
}

// backward from g (dL/dy*, FP32 NATIVE full, 1 channel) at the output: accumulates dL/dW* into
// n->grad and, when gin is given, writes dL/dx* of the input.
void ptc_backward_acts(dirac_ctx *c, dirac_ptc *n, const void *g_out, void *gin, hipStream_t s) {
    PtcGeom a = geom_of(c, s);
    const size_t chanb = chan_vecs<float>(c->g.vhp) * sizeof(float4);
    int maxc = 0;
    for (int l = 0; l <= n->nlayers; ++l) maxc = std::max(maxc, n->ch[l]);
    char *gA = (char *)n->gbuf.p, *gB = gA + (size_t)maxc * chanb;
    HIP_CHECK(hipMemcpyAsync(gA, g_out, (size_t)n->ch[n->nlayers] * chanb, hipMemcpyDeviceToDevice, s));
    for (int l = n->nlayers - 1; l >= 0; --l) {
        const int nin = n->ch[l], nout = n->ch[l + 1];
        const int nw = (int)ptc_nweights(n, l);
        wgrad_dispatch(a, nin, nout, ptc_act(c, n, l), act_bf16(n, l), gA, n->part.p, s);
        k_ptc_reduce<<<(nw + kRedK - 1) / kRedK, 256, 0, s>>>(wgrad_grid(c->vh, nout), nw, (const float2 *)n->part.p,
                                                      (float2 *)n->grad.p + n->off[l]);
        HIP_CHECK(hipGetLastError());
        if (l == 0 && !gin) break;
        k_adjoint_weights<<<(nw + 255) / 256, 256, 0, s>>>(nout, nin, (const uint32_t *)n->wbf.p + n->off[l],
                                                           (uint32_t *)n->wt.p + n->off[l]);
        HIP_CHECK(hipGetLastError());
        uint4 *afb = (uint4 *)n->afb.p + n->afb_off[l];
        build_afrags(nout, nin, (const uint32_t *)n->wt.p + n->off[l], afb, s);
        void *dst = l == 0 ? gin : (void *)gB;
        layer_dispatch(a, nout, nin, gA, afb, dst, Io::F32, s);
        std::swap(gA, gB);
    }
}

void ptc_adam(dirac_ptc *n, double lr, hipStream_t s) {
    n->step += 1;
    // the decay rates and the bias corrections 1 - b^t in FP64, each rounded to FP32 once
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    const double c1 = 1.0 - std::pow(b1, (double)n->step), c2 = 1.0 - std::pow(b2, (double)n->step);
    const int nr = (int)(2 * n->total);
    k_adam<<<(nr + 255) / 256, 256, 0, s>>>(nr, (float *)n->w.p, (const float *)n->grad.p, (float *)n->m.p,
                                           (float *)n->v.p, (uint16_t *)n->wbf.p, (float)lr, (float)b1,
                                           (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), (float)eps, (float)c1,
                                           (float)c2);
    HIP_CHECK(hipGetLastError());
    refresh_afrags(n, s);
}

}  // namespace dl
