// Schwarz alternating procedure (SAP): the block preconditioner of openQxD's solver, on 4^4
// blocks coloured as a checkerboard of blocks.  One application psi = M r:
//   psi = 0, rho = r; ncy times, for colour 0 then colour 1: on every block of the colour,
//   delta = nmr minimal-residual steps on the block operator D_blk (hops that leave the block
//   dropped) for the residual on the block; psi += delta; rho = r - D psi.
// One work-group per block, one thread per site.  The residual of the block is staged in LDS
// (the neighbour reads of D_blk), and so are the block's links of in-block hops and, in
// registers, each site's clover block: they are read from memory once per block solve, not once
// per minimal-residual step.  The block reductions of the minimal-residual steps are
// shuffle trees and a fixed-order sum over the four wavefronts (deterministic).  The residual
// update after a colour's solves changes rho only on the faces of the other colour's blocks
// (D delta = -1/2 H delta there); it is done by the next step's work-groups on entry, from the
// corrections delta of the previous step, so a step is one launch.  FP32 throughout (the
// arithmetic of a preconditioner), on block-ordered copies of the F32 links and clover field.
#include "dirac_ops.h"
#include "hop_core.h"
#include "internal.h"

namespace dl {
namespace {

constexpr int kSapB = 4;                                  // block extent in every direction
constexpr int kSapSites = kSapB * kSapB * kSapB * kSapB;  // 256: one work-group
constexpr int kSapLinkPlanes = 4;  // a link in block order: 12 reals of rows 0, 1, then cos, sin of its phase
constexpr int kSapInner = kSapSites / kSapB * (kSapB - 1);  // 192 sites of a block with a neighbour inside it in +mu

// Block order: the fields of the Schwarz blocks are kept block by block (block k lexicographic in
// the block coordinates, site t = 64 b0 + 16 b1 + 4 b2 + b3 inside it), plane-major within a
// block, so that a work-group reads one contiguous chunk and every wavefront load is 1 KB of
// consecutive 16-byte vectors:  spinor [k][6][256], clover [k][18][256], links [k][8][4][256].
// (The sites of a 4^4 block lie in 2-site pieces of the x3-fastest NATIVE order: read from there,
// every wavefront load touches 32 cache lines for 32 bytes each.  The first cycle reads the
// residual from there all the same, which costs less than a separate reordering pass; the
// solution goes back through one, as scattered 32-byte writes of partial cache lines from the
// last cycle's steps cost more than the pass.)
struct SapArgs {
    Geom g;
    const float4 *links;  // block order
    const float4 *clov;   // block order
    float4 *rho, *psi, *dlt;  // block order, all blocks
    const float4 *rin;    // NATIVE input residual, read instead of rho when set (the first cycle)
    int nb[4];            // blocks per direction
    int colour, nmr, update;
    int first;            // the first cycle: psi is zero, so psi = delta
};

DEV int block_of(const SapArgs &a, const int n[4]) { return ((n[0] * a.nb[1] + n[1]) * a.nb[2] + n[2]) * a.nb[3] + n[3]; }
DEV size_t spinor_at(int k, int t) { return (size_t)k * 6 * kSapSites + t; }  // plane 0; plane j at + j * 256

// Block coordinates of the k-th block of colour c: blocks are lexicographic in (n0, n1, n2, n3),
// and every row of n3 (an even number of blocks) holds half of each colour.
DEV void sap_block(const SapArgs &a, int k, int n[4]) {
    const int half3 = a.nb[3] / 2;
    const int r = k / half3, m = k % half3;
    n[2] = r % a.nb[2];
    n[1] = (r / a.nb[2]) % a.nb[1];
    n[0] = r / (a.nb[2] * a.nb[1]);
    n[3] = 2 * m + ((a.colour + n[0] + n[1] + n[2]) & 1);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

DEV void load_sp(const float4 *base, C<float> r[12]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const float4 q = base[k * kSapSites];
        r[2 * k] = mk(q.x, q.y);
        r[2 * k + 1] = mk(q.z, q.w);
    }
}
DEV void store_sp(float4 *base, const C<float> r[12]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) base[k * kSapSites] = make_float4(r[2 * k].r, r[2 * k].i, r[2 * k + 1].r, r[2 * k + 1].i);
}
// link of direction d at site t of block k (block order)
DEV void load_blink(const SapArgs &a, int k, int d, int t, C<float> u[6], float &co, float &si) {
    const float4 *q = a.links + ((size_t)(k * 8 + d) * kSapLinkPlanes) * kSapSites + t;
    const float4 l0 = q[0], l1 = q[kSapSites], l2 = q[2 * kSapSites], l3 = q[3 * kSapSites];
    u[0] = mk(l0.x, l0.y); u[1] = mk(l0.z, l0.w);
    u[2] = mk(l1.x, l1.y); u[3] = mk(l1.z, l1.w);
    u[4] = mk(l2.x, l2.y); u[5] = mk(l2.z, l2.w);
    co = l3.x;
    si = l3.y;
}

// Forward link of direction mu at block site t (b_mu < 3, the links of the hops inside the block),
// in the LDS tile of the block: the 192 such sites of a direction, in site order.
DEV int inner_link(int mu, int t) {
    const int sh = 6 - 2 * mu;  // log2 of the site stride of direction mu
    return t - ((t >> (sh + 2)) << sh);
}

__global__ __launch_bounds__(kSapSites) void k_sap_step(SapArgs a) {
    __shared__ float4 rs[6][kSapSites];  // the block's residual, plane-major
    __shared__ float red[3][4];
    // the block's forward links of in-block hops (a backward hop from t takes the forward link of
    // t - stride): rows 0, 1 of the SU(3) matrix in three planes, (cos, sin) of the phase
    __shared__ float4 lq[4][3][kSapInner];
    __shared__ float2 lp[4][kSapInner];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int b[4] = {t >> 6, (t >> 4) & 3, (t >> 2) & 3, t & 3};
    int n[4];
    sap_block(a, blockIdx.x, n);
    const int k = block_of(a, n);

    // the site's position in the NATIVE full vectors (parity-major, 6 planes per site)
    int xs[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) xs[m] = kSapB * n[m] + b[m];
    const int par = (xs[0] + xs[1] + xs[2] + xs[3]) & 1;
    const int hi = half_index(a.g, xs);
    const size_t nat = (size_t)par * 6 * a.g.vhp + (size_t)(hi >> 6) * 6 * kSB + (hi & (kSB - 1));

    C<float> r[12];
    if (a.rin) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const float4 v = a.rin[nat + q * kSB];
            r[2 * q] = mk(v.x, v.y);
            r[2 * q + 1] = mk(v.z, v.w);
        }
    } else {
        load_sp(a.rho + spinor_at(k, t), r);
    }
    if (a.update) {
        // rho += 1/2 H delta over the faces of the block: the previous step's corrections live on
        // the neighbouring blocks (the other colour).  The 8 faces of 64 sites are taken face by
        // face, wavefront w the faces of directions w (first pass) and w + 4 (second pass), so no
        // lane idles; each face term, formed from zero, goes through LDS (the residual tile, free
        // until the minimal-residual steps) to its site, which adds its terms in direction order.
        float *fb = reinterpret_cast<float *>(&rs[0][0]);  // [4 directions][24 reals][64 face sites]
        C<float> acc[12];
#pragma unroll
        for (int q = 0; q < 12; ++q) acc[q] = mk(0.f, 0.f);
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            {
                // face site `lane` of direction d: b_mu on the face, the other coordinates from lane
                const int d = 4 * pass + wave, mu = d >> 1, back = d & 1;
                int bf[4], o = 0;
#pragma unroll
                for (int m = 3; m >= 0; --m) {
                    if (m == mu) {
                        bf[m] = back ? 0 : kSapB - 1;
                    } else {
                        bf[m] = (lane >> (2 * o)) & 3;
                        ++o;
                    }
                }
                const int tf = ((bf[0] * kSapB + bf[1]) * kSapB + bf[2]) * kSapB + bf[3];
                int y[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) y[m] = kSapB * n[m] + bf[m];
                // the neighbour across the face, with the lattice wrap and the C* mirror shift
                const int Lm = a.g.L[mu];
                const int ym = y[mu];
                const bool cross = back ? ym == 0 : ym == Lm - 1;
                const int yn = back ? (ym == 0 ? Lm - 1 : ym - 1) : (ym == Lm - 1 ? 0 : ym + 1);
                if (mu == 0) y[0] = yn; else if (mu == 1) y[1] = yn; else if (mu == 2) y[2] = yn; else y[3] = yn;
                y[1] = cstar_x1(a.g, mu, cross, y[1]);
                int nn[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) nn[m] = y[m] / kSapB;
                const int tn = ((y[0] % kSapB) * kSapB + (y[1] % kSapB)) * kSapB * kSapB + (y[2] % kSapB) * kSapB + (y[3] % kSapB);
                C<float> nb[12], u[6], v[12];
                float co, si;
                load_sp(a.dlt + spinor_at(block_of(a, nn), tn), nb);
                load_blink(a, k, d, tf, u, co, si);
#pragma unroll
                for (int q = 0; q < 12; ++q) v[q] = mk(0.f, 0.f);
                accumulate_dir<float, 0>(d, nb, u, co, si, v);
                float *dst = fb + (size_t)wave * 24 * 64 + lane;
#pragma unroll
                for (int q = 0; q < 12; ++q) {
                    dst[(2 * q) * 64] = v[q].r;
                    dst[(2 * q + 1) * 64] = v[q].i;
                }
            }
            __syncthreads();
            // this site's terms of the pass's four directions, in direction order
#pragma unroll
            for (int dd = 0; dd < 4; ++dd) {
                const int d = 4 * pass + dd, mu = d >> 1, back = d & 1;
                const int bm = mu == 0 ? b[0] : mu == 1 ? b[1] : mu == 2 ? b[2] : b[3];
                if (back ? bm != 0 : bm != kSapB - 1) continue;  // not on this face
                int f = 0, o = 0;
#pragma unroll
                for (int m = 3; m >= 0; --m) {
                    if (m == mu) continue;
                    f |= b[m] << (2 * o);
                    ++o;
                }
                const float *src = fb + (size_t)dd * 24 * 64 + f;
#pragma unroll
                for (int q = 0; q < 12; ++q) acc[q] = mk(acc[q].r + src[(2 * q) * 64], acc[q].i + src[(2 * q + 1) * 64]);
            }
            __syncthreads();  // the pass's terms are read before the next pass (or the residual tile) overwrites them
        }
#pragma unroll
        for (int q = 0; q < 12; ++q) r[q] = mk(fmaf(0.5f, acc[q].r, r[q].r), fmaf(0.5f, acc[q].i, r[q].i));
    }
    C<float> dl_[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) dl_[q] = mk(0.f, 0.f);
    // the block's inner links, read once for all minimal-residual steps (the first step's barrier
    // orders these writes before any read)
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        if (b[mu] == kSapB - 1) continue;
        const int ci = inner_link(mu, t);
        const float4 *q = a.links + ((size_t)(k * 8 + 2 * mu) * kSapLinkPlanes) * kSapSites + t;
        lq[mu][0][ci] = q[0];
        lq[mu][1][ci] = q[kSapSites];
        lq[mu][2][ci] = q[2 * kSapSites];
        const float4 ph = q[3 * kSapSites];
        lp[mu][ci] = make_float2(ph.x, ph.y);
    }
    // the site's clover block, read once for all minimal-residual steps
    float pk[72];
    {
        const float4 *cq = a.clov + (size_t)k * 18 * kSapSites + t;
#pragma unroll
        for (int q = 0; q < 18; ++q) {
            const float4 f = cq[q * kSapSites];
            pk[4 * q] = f.x;
            pk[4 * q + 1] = f.y;
            pk[4 * q + 2] = f.z;
            pk[4 * q + 3] = f.w;
        }
    }

#pragma nounroll
    for (int it = 0; it < a.nmr; ++it) {
        __syncthreads();  // the previous step's reads of rs are done
#pragma unroll
        for (int q = 0; q < 6; ++q) rs[q][t] = make_float4(r[2 * q].r, r[2 * q].i, r[2 * q + 1].r, r[2 * q + 1].i);
        __syncthreads();
        // v = D_blk r = A r - 1/2 sum over the neighbours inside the block
        C<float> v[12], hs[12];
#pragma unroll
        for (int q = 0; q < 12; ++q) hs[q] = mk(0.f, 0.f);
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            const int mu = d >> 1, back = d & 1;
            const int bm = mu == 0 ? b[0] : mu == 1 ? b[1] : mu == 2 ? b[2] : b[3];
            if (back ? bm == 0 : bm == kSapB - 1) continue;  // that neighbour is outside the block
            const int stride = mu == 0 ? 64 : mu == 1 ? 16 : mu == 2 ? 4 : 1;
            const int tn = back ? t - stride : t + stride;
            C<float> nb[12], u[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const float4 f = rs[q][tn];
                nb[2 * q] = mk(f.x, f.y);
                nb[2 * q + 1] = mk(f.z, f.w);
            }
            const int ci = inner_link(mu, back ? tn : t);
            const float4 l0 = lq[mu][0][ci], l1 = lq[mu][1][ci], l2 = lq[mu][2][ci];
            const float2 ph = lp[mu][ci];
            u[0] = mk(l0.x, l0.y); u[1] = mk(l0.z, l0.w);
            u[2] = mk(l1.x, l1.y); u[3] = mk(l1.z, l1.w);
            u[4] = mk(l2.x, l2.y); u[5] = mk(l2.z, l2.w);
            accumulate_dir<float, 0>(d, nb, u, ph.x, ph.y, hs);
        }
#pragma unroll
        for (int blk = 0; blk < 2; ++blk) block_mul(pk + 36 * blk, r + 6 * blk, v + 6 * blk);
#pragma unroll
        for (int q = 0; q < 12; ++q) v[q] = mk(fmaf(-0.5f, hs[q].r, v[q].r), fmaf(-0.5f, hs[q].i, v[q].i));
        // w = <v, r> / <v, v> over the block
        float vr = 0.f, vi = 0.f, vv = 0.f;
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            vr = fmaf(v[q].r, r[q].r, fmaf(v[q].i, r[q].i, vr));
            vi = fmaf(v[q].r, r[q].i, fmaf(-v[q].i, r[q].r, vi));
            vv = fmaf(v[q].r, v[q].r, fmaf(v[q].i, v[q].i, vv));
        }
        vr = wave_sum(vr);
        vi = wave_sum(vi);
        vv = wave_sum(vv);
        if (lane == 0) {
            red[0][wave] = vr;
            red[1][wave] = vi;
            red[2][wave] = vv;
        }
        __syncthreads();
        const float sr = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        const float si = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        const float sv = (red[2][0] + red[2][1]) + (red[2][2] + red[2][3]);
        const float inv = sv > 0.f ? 1.0f / sv : 0.f;
        const C<float> w = mk(sr * inv, si * inv);
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            madd(dl_[q], w, r[q]);
            const C<float> wv = w * v[q];
            r[q] = mk(r[q].r - wv.r, r[q].i - wv.i);
        }
        __syncthreads();  // red is read by every thread before the next step overwrites it
    }
    // psi += delta, rho = the block residual, delta kept for the next step's face update
    float4 *ps = a.psi + spinor_at(k, t);
    C<float> o[12];
    if (a.first) {
#pragma unroll
        for (int q = 0; q < 12; ++q) o[q] = dl_[q];
    } else {
        load_sp(ps, o);
#pragma unroll
        for (int q = 0; q < 12; ++q) o[q] = mk(o[q].r + dl_[q].r, o[q].i + dl_[q].i);
    }
    store_sp(ps, o);
    store_sp(a.rho + spinor_at(k, t), r);
    store_sp(a.dlt + spinor_at(k, t), dl_);
}

// Block order of the fields (once per field): site (p, i) -> block k, site t
DEV void block_pos(const Geom &g, const int nb[4], const int x[4], int &k, int &t) {
    int n[4], b[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        n[m] = x[m] / kSapB;
        b[m] = x[m] % kSapB;
    }
    k = ((n[0] * nb[1] + n[1]) * nb[2] + n[2]) * nb[3] + n[3];
    t = ((b[0] * kSapB + b[1]) * kSapB + b[2]) * kSapB + b[3];
}

__global__ void k_sap_fields(Geom g, int p, int4 nb4, const float4 *__restrict__ links, const float *__restrict__ omega,
                             const float4 *__restrict__ clov, float4 *__restrict__ blinks, float4 *__restrict__ bclov) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.vh) return;
    const int nb[4] = {nb4.x, nb4.y, nb4.z, nb4.w};
    int x[4], k, t;
    site_coords(g, i, p, x);
    block_pos(g, nb, x, k, t);
    const size_t vhp = (size_t)g.vhp;
#pragma unroll 1
    for (int d = 0; d < 8; ++d) {
        const float4 *src = site_ptr(links + (size_t)d * 3 * vhp, (uint32_t)i, 3);
        float4 *dst = blinks + ((size_t)(k * 8 + d) * kSapLinkPlanes) * kSapSites + t;
        dst[0] = src[0];
        dst[kSapSites] = src[kSB];
        dst[2 * kSapSites] = src[2 * kSB];
        float sn, cs;
        sc(omega[(size_t)d * vhp + i], sn, cs);
        dst[3 * kSapSites] = make_float4(cs, sn, 0.f, 0.f);
    }
    const float4 *cs = site_ptr(clov, (uint32_t)i, 18);
    float4 *cd = bclov + (size_t)k * 18 * kSapSites + t;
#pragma unroll
    for (int q = 0; q < 18; ++q) cd[q * kSapSites] = cs[q * kSB];
}

// Block order -> NATIVE F32 full vector, parity p (the solution at the end of an application)
__global__ void k_sap_unorder(Geom g, int p, int4 nb4, float4 *__restrict__ nat, const float4 *__restrict__ blk) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.vh) return;
    const int nb[4] = {nb4.x, nb4.y, nb4.z, nb4.w};
    int x[4], k, t;
    site_coords(g, i, p, x);
    block_pos(g, nb, x, k, t);
    float4 *q = site_ptr(nat + (size_t)p * 6 * g.vhp, (uint32_t)i, 6);
    const float4 *bq = blk + spinor_at(k, t);
#pragma unroll
    for (int j = 0; j < 6; ++j) q[j * kSB] = bq[j * kSapSites];
}

}  // namespace

bool sap_supported(const dirac_ctx *c) {
    for (int m = 0; m < 4; ++m)
        if (c->g.L[m] % (2 * kSapB) != 0) return false;
    // C*: crossing a shifted boundary moves x1 by L1/2, which must be an even number of blocks,
    // or two blocks of one colour would meet across that face
    if (c->g.cs >= 2 && c->g.h1 % (2 * kSapB) != 0) return false;
    return true;
}

// psi = M_SAP r on NATIVE F32 full vectors
void sap_apply(dirac_ctx *c, void *psi, const void *r, int ncy, int nmr, hipStream_t s) {
    require(sap_supported(c), "the Schwarz preconditioner needs every lattice extent to be a multiple of 8 "
                              "(an even number of 4^4 blocks per direction) and, with C* boundaries, dims[1] a "
                              "multiple of 16");
    require(ncy >= 1 && ncy <= 64 && nmr >= 1 && nmr <= 64, "SAP cycles and block steps must be 1..64");
    ensure_prec(c, DIRAC_F32, s);
    int nblk = 1;
    int nb[4];
    for (int m = 0; m < 4; ++m) {
        nb[m] = c->g.L[m] / kSapB;
        nblk *= nb[m];
    }
    const int4 nb4 = make_int4(nb[0], nb[1], nb[2], nb[3]);
    const int vh = (int)c->vh;
    if (!c->sap_ready) {
        c->sap_links.alloc((size_t)nblk * 8 * kSapLinkPlanes * kSapSites * sizeof(float4));
        c->sap_clov.alloc((size_t)nblk * 18 * kSapSites * sizeof(float4));
        for (int p = 0; p < 2; ++p)
            k_sap_fields<<<grid_for(vh), kBlock, 0, s>>>(c->g, p, nb4, (const float4 *)c->f[DIRAC_F32].links[p].p,
                                                         (const float *)c->f[DIRAC_F32].omega[p].p,
                                                         (const float4 *)c->f[DIRAC_F32].clov[p].p,
                                                         (float4 *)c->sap_links.p, (float4 *)c->sap_clov.p);
        HIP_CHECK(hipGetLastError());
        c->sap_ready = true;
    }
    const size_t vbytes = (size_t)nblk * 6 * kSapSites * sizeof(float4);
    c->sap_rho.alloc(3 * vbytes);  // rho, psi, delta in block order
    float4 *rho = (float4 *)c->sap_rho.p, *pb = rho + vbytes / sizeof(float4), *dlt = pb + vbytes / sizeof(float4);
    // the first cycle reads the residual from the NATIVE input (no reordering pass in), and psi
    // starts as the first cycle's corrections (no zero fill)
    SapArgs a{};
    a.g = c->g;
    a.links = (const float4 *)c->sap_links.p;
    a.clov = (const float4 *)c->sap_clov.p;
    a.rho = rho;
    a.psi = pb;
    a.dlt = dlt;
    for (int m = 0; m < 4; ++m) a.nb[m] = nb[m];
    a.nmr = nmr;
    for (int cy = 0; cy < ncy; ++cy)
        for (int col = 0; col < 2; ++col) {
            a.colour = col;
            a.update = !(cy == 0 && col == 0);
            a.first = cy == 0;
            a.rin = cy == 0 ? (const float4 *)r : nullptr;
            k_sap_step<<<nblk / 2, kSapSites, 0, s>>>(a);
            HIP_CHECK(hipGetLastError());
        }
    for (int p = 0; p < 2; ++p) k_sap_unorder<<<grid_for(vh), kBlock, 0, s>>>(c->g, p, nb4, (float4 *)psi, pb);
    HIP_CHECK(hipGetLastError());
}

}  // namespace dl
