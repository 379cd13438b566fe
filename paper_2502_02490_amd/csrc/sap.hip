// Schwarz alternating procedure (SAP): the block preconditioner of openQxD's solver, on 4^4
// blocks coloured as a checkerboard of blocks.  One application psi = M r:
//   psi = 0, rho = r; ncy times, for colour 0 then colour 1: on every block of the colour,
//   delta = nmr minimal-residual steps on the block operator D_blk (hops that leave the block
//   dropped) for the residual on the block; psi += delta; rho = r - D psi.
// One work-group per block, one thread per site.  The residual of the block is staged in LDS
// (the neighbour reads of D_blk); the block reductions of the minimal-residual steps are
// shuffle trees and a fixed-order sum over the four wavefronts (deterministic).  The residual
// update after a colour's solves changes rho only on the faces of the other colour's blocks
// (D delta = -1/2 H delta there); it is done by the next step's work-groups on entry, from the
// corrections delta of the previous step, so a step is one launch.  FP32 throughout (the
// arithmetic of a preconditioner), on the F32 copies of the links and the clover field.
#include "dirac_ops.h"
#include "hop_core.h"
#include "internal.h"

namespace dl {
namespace {

constexpr int kSapB = 4;                           // block extent in every direction
constexpr int kSapSites = kSapB * kSapB * kSapB * kSapB;  // 256: one work-group

struct SapArgs {
    Geom g;
    const float4 *links[2];  // F32 compressed links per parity, [8 dir][3 planes] blocked
    const float *omega[2];   // per parity, [8 dir][vhp]
    const float4 *clov[2];   // F32 clover field A per parity, 72 reals = 18 planes
    float4 *rho, *psi, *dlt;  // F32 NATIVE full vectors (even half, then odd half)
    int nb[4];               // blocks per direction
    int colour, nmr, update;
};

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

__global__ __launch_bounds__(kSapSites) void k_sap_step(SapArgs a) {
    __shared__ float4 rs[6][kSapSites];  // the block's residual, plane-major
    __shared__ float red[3][4];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int b[4] = {t >> 6, (t >> 4) & 3, (t >> 2) & 3, t & 3};
    int n[4];
    sap_block(a, blockIdx.x, n);
    int x[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) x[m] = kSapB * n[m] + b[m];
    const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
    const uint32_t i = (uint32_t)half_index(a.g, x);
    const size_t hv = (size_t)6 * a.g.vhp;
    HopArgs<float> h{};
    h.g = a.g;
    h.links = a.links[p];
    h.omega = a.omega[p];

    C<float> r[12];
    load_spinor<float>(a.rho + p * hv, i, r);
    if (a.update) {
        // rho += 1/2 H delta over the faces of the block: the previous step's corrections live on
        // the neighbouring blocks (the other colour)
        C<float> acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = mk(0.f, 0.f);
        h.in = a.dlt + (1 - p) * hv;
        const int row = (x[0] * a.g.L[1] + x[1]) * a.g.L[2] + x[2];
#pragma nounroll
        for (int d = 0; d < 8; ++d) {
            const int mu = d >> 1, back = d & 1;
            const int bm = mu == 0 ? b[0] : mu == 1 ? b[1] : mu == 2 ? b[2] : b[3];
            if (back ? bm != 0 : bm != kSapB - 1) continue;  // the neighbour is inside the block
            C<float> nb[12], u[6];
            float co, si;
            load_spinor<float>(h.in, neighbour(h, x, row, d), nb);
            load_link<float, false>(h, d, i, u, co, si);
            accumulate_dir<float, 0>(d, nb, u, co, si, acc);
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) r[k] = mk(fmaf(0.5f, acc[k].r, r[k].r), fmaf(0.5f, acc[k].i, r[k].i));
    }
    C<float> dl_[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) dl_[k] = mk(0.f, 0.f);

#pragma nounroll
    for (int it = 0; it < a.nmr; ++it) {
        __syncthreads();  // the previous step's reads of rs are done
#pragma unroll
        for (int k = 0; k < 6; ++k) rs[k][t] = make_float4(r[2 * k].r, r[2 * k].i, r[2 * k + 1].r, r[2 * k + 1].i);
        __syncthreads();
        // v = D_blk r = A r - 1/2 sum over the neighbours inside the block
        C<float> v[12], hs[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) hs[k] = mk(0.f, 0.f);
#pragma nounroll
        for (int d = 0; d < 8; ++d) {
            const int mu = d >> 1, back = d & 1;
            const int bm = mu == 0 ? b[0] : mu == 1 ? b[1] : mu == 2 ? b[2] : b[3];
            if (back ? bm == 0 : bm == kSapB - 1) continue;  // that neighbour is outside the block
            const int stride = mu == 0 ? 64 : mu == 1 ? 16 : mu == 2 ? 4 : 1;
            const int tn = back ? t - stride : t + stride;
            C<float> nb[12], u[6];
            float co, si;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const float4 q = rs[k][tn];
                nb[2 * k] = mk(q.x, q.y);
                nb[2 * k + 1] = mk(q.z, q.w);
            }
            load_link<float, false>(h, d, i, u, co, si);
            accumulate_dir<float, 0>(d, nb, u, co, si, hs);
        }
        {
            float pk[72];
            load_field<float, 72>(a.clov[p], i, pk);
#pragma unroll
            for (int blk = 0; blk < 2; ++blk) block_mul(pk + 36 * blk, r + 6 * blk, v + 6 * blk);
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = mk(fmaf(-0.5f, hs[k].r, v[k].r), fmaf(-0.5f, hs[k].i, v[k].i));
        // w = <v, r> / <v, v> over the block
        float vr = 0.f, vi = 0.f, vv = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            vr = fmaf(v[k].r, r[k].r, fmaf(v[k].i, r[k].i, vr));
            vi = fmaf(v[k].r, r[k].i, fmaf(-v[k].i, r[k].r, vi));
            vv = fmaf(v[k].r, v[k].r, fmaf(v[k].i, v[k].i, vv));
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
        for (int k = 0; k < 12; ++k) {
            madd(dl_[k], w, r[k]);
            const C<float> wv = w * v[k];
            r[k] = mk(r[k].r - wv.r, r[k].i - wv.i);
        }
        __syncthreads();  // red is read by every thread before the next step overwrites it
    }
    // psi += delta, rho = the block residual, delta kept for the next step's face update
    float4 *ps = site_ptr(a.psi + p * hv, i, 6);
    float4 *rh = site_ptr(a.rho + p * hv, i, 6);
    float4 *dd = site_ptr(a.dlt + p * hv, i, 6);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const float4 o = ps[k * kSB];
        ps[k * kSB] = make_float4(o.x + dl_[2 * k].r, o.y + dl_[2 * k].i, o.z + dl_[2 * k + 1].r, o.w + dl_[2 * k + 1].i);
        rh[k * kSB] = make_float4(r[2 * k].r, r[2 * k].i, r[2 * k + 1].r, r[2 * k + 1].i);
        dd[k * kSB] = make_float4(dl_[2 * k].r, dl_[2 * k].i, dl_[2 * k + 1].r, dl_[2 * k + 1].i);
    }
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
    const size_t bytes = (size_t)48 * c->g.vhp * sizeof(float);
    c->sap_rho.alloc(bytes);
    c->sap_dlt.alloc(bytes);
    HIP_CHECK(hipMemcpyAsync(c->sap_rho.p, r, bytes, hipMemcpyDeviceToDevice, s));
    zero_fill(psi, bytes, s);
    SapArgs a{};
    a.g = c->g;
    for (int p = 0; p < 2; ++p) {
        a.links[p] = (const float4 *)c->f[DIRAC_F32].links[p].p;
        a.omega[p] = (const float *)c->f[DIRAC_F32].omega[p].p;
        a.clov[p] = (const float4 *)c->f[DIRAC_F32].clov[p].p;
    }
    a.rho = (float4 *)c->sap_rho.p;
    a.psi = (float4 *)psi;
    a.dlt = (float4 *)c->sap_dlt.p;
    int nblk = 1;
    for (int m = 0; m < 4; ++m) {
        a.nb[m] = c->g.L[m] / kSapB;
        nblk *= a.nb[m];
    }
    a.nmr = nmr;
    for (int cy = 0; cy < ncy; ++cy)
        for (int col = 0; col < 2; ++col) {
            a.colour = col;
            a.update = !(cy == 0 && col == 0);
            k_sap_step<<<nblk / 2, kSapSites, 0, s>>>(a);
            HIP_CHECK(hipGetLastError());
        }
}

}  // namespace dl
