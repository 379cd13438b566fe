// Kernels and launch shapes of the hopping term between parities, fused with the clover field
// (one thread per output site), included by the per-precision translation units hop_f64.hip,
// hop_f32.hip, hop_f16.hip and hop_bf16.hip (so the four compile in parallel); hop.hip builds the
// even-odd Schur and full operators from them.
//
//   H psi(x) = sum_mu [ V_mu(x) b+ (1 - gamma_mu) psi(x + mu) + V_mu(x - mu)^dag b- (1 + gamma_mu) psi(x - mu) ]
//
// For each of the 8 neighbours the kernel loads the neighbour's spinor, projects it to a
// half-spinor, multiplies by the link (two stored rows, third rebuilt, phase exp(+-i omega)),
// and accumulates the reconstructed spinor.  The dagger, gamma_5 H gamma_5, flips the
// projector signs.  Epilogues: HOP_INV applies A_pp^-1 to the result, HOP_CLOV adds A_pp chi.
#pragma once

#include <algorithm>
#include <cstdio>
#include <type_traits>

#include "dirac_ops.h"
#include "hop_core.h"
#include "internal.h"

namespace dl {
namespace {

// One neighbour direction n = 2 mu + back of the hopping sum at site i (coordinates x, row =
// index of its (x0, x1, x2) row), accumulated into acc.  With `tile` the time-direction neighbour
// comes from LDS: slot `tslot` - 1 / + 1 of the tile holds the input block of the previous / next
// time slice at the same spatial block, and the neighbour sits at the same lane.
// What the right-hand-side blocked kernel stages in LDS for one 64-site block: per direction n
// and site, the link's two stored rows, its third row and its phase (cos, sin) in the
// accumulation precision ([n][20][64]: u[0..5], r2[0..2] as (re, im), then cos, sin), the
// neighbour's index ([n][64]), and the clover block in its HBM planes ([plane][64]).
template <typename S>
struct LdsBlock {
    const typename St<S>::acc *lk;
    const uint32_t *nb;
    const typename St<S>::vec *cl;
};

template <typename S, int DAG, bool NT>
DEV void hop_dir(const HopArgs<S> &a, const int x[4], int row, uint32_t i, int n, C<typename St<S>::acc> acc[12],
                 const typename St<S>::vec *tile, int tslot) {
    using T = typename St<S>::acc;
    const int mu = n >> 1, back = n & 1;
    C<T> psi[12], u[6];
    T co, si;
    if (tile && mu == 0) load_spinor<S>(tile + (size_t)(tslot + (back ? -1 : 1)) * (24 / St<S>::W) * kSB,
                                        i & (kSB - 1), psi);
    else load_spinor<S>(a.in, neighbour(a, x, row, n), psi);
    load_link<S, NT>(a, n, i, u, co, si);
    accumulate_dir<T, DAG>(n, psi, u, co, si, acc);
}

// The 8 neighbours run as iterations of a loop that is not unrolled, with the direction a
// uniform run-time value: straight-line code lets the compiler issue the loads of all eight
// neighbours up front, which needs more registers than a lane has (spills, one wave per SIMD).
// NPI = 1 keeps one neighbour's data live at a time; NPI = 2 takes the forward and backward
// neighbour of one mu per iteration, so each wave has twice the loads in flight; NPI = 4 takes
// two mu per iteration (four times the loads in flight, for the persistent shapes with one
// wavefront per SIMD, whose register file allows it).  The sums are accumulated in the same
// order either way.
template <typename S, int DAG, int NPI, bool NT>
DEV void hop_all(const HopArgs<S> &a, const int x[4], uint32_t i, C<typename St<S>::acc> acc[12],
                 const typename St<S>::vec *tile = nullptr, int tslot = 0) {
    const int row = (x[0] * a.g.L[1] + x[1]) * a.g.L[2] + x[2];
    if constexpr (NPI == 1) {
#pragma nounroll
        for (int n = 0; n < 8; ++n) hop_dir<S, DAG, NT>(a, x, row, i, n, acc, tile, tslot);
    } else if constexpr (NPI == 4) {
#pragma nounroll
        for (int mu = 0; mu < 4; mu += 2) {
            hop_dir<S, DAG, NT>(a, x, row, i, 2 * mu, acc, tile, tslot);
            hop_dir<S, DAG, NT>(a, x, row, i, 2 * mu + 1, acc, tile, tslot);
            hop_dir<S, DAG, NT>(a, x, row, i, 2 * mu + 2, acc, tile, tslot);
            hop_dir<S, DAG, NT>(a, x, row, i, 2 * mu + 3, acc, tile, tslot);
        }
    } else {
#pragma nounroll
        for (int mu = 0; mu < 4; ++mu) {
            hop_dir<S, DAG, NT>(a, x, row, i, 2 * mu, acc, tile, tslot);
            hop_dir<S, DAG, NT>(a, x, row, i, 2 * mu + 1, acc, tile, tslot);
        }
    }
}

// The scale, the clover epilogue / prologue and the store of output site i, from its hopping sum
// acc.  NT: the clover field, chi and the output, each touched once, carry a streaming hint.
// LDSF: the clover block comes from the LDS copy of the right-hand-side blocked kernel.
template <typename S, int MODE, bool NT, bool LDSF = false>
DEV void hop_finish(const HopArgs<S> &a, uint32_t i, const C<typename St<S>::acc> acc[12],
                    const LdsBlock<S> *lds = nullptr) {
    using T = typename St<S>::acc;
    C<T> y[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) y[k] = a.coef * acc[k];
    if constexpr (MODE != HOP_PLAIN) {
        // 72 packed reals per site: block + (spins 0, 1) then block - (spins 2, 3).  With 8 reals
        // per plane (16-bit storage) the two blocks share a plane, so all 72 are loaded at once;
        // otherwise one block at a time.
        constexpr int W = St<S>::W;
        constexpr bool split = (36 % W) == 0;
        T pk[split ? 36 : 72];
        C<T> t[6], chi[12];
        if constexpr (MODE == HOP_CLOV) {
            T cr[24];
            load_planes_h<S, 24, NT>(a.chi, 24 / W, 0, i, cr);
#pragma unroll
            for (int k = 0; k < 12; ++k) chi[k] = mk(cr[2 * k], cr[2 * k + 1]);
        }
#pragma unroll
        for (int blk = 0; blk < 2; ++blk) {
            const T *q = pk;
            if constexpr (split) {
                if constexpr (LDSF) {
#pragma unroll
                    for (int k = 0; k < 36 / W; ++k)
                        St<S>::unpack(lds->cl[(blk * (36 / W) + k) * kSB + (i & (kSB - 1))], pk + k * W);
                } else {
                    load_planes_h<S, 36, NT>(a.clov, 72 / W, blk * (36 / W), i, pk);
                }
            } else {
                if (blk == 0) {
                    if constexpr (LDSF) {
#pragma unroll
                        for (int k = 0; k < 72 / W; ++k) St<S>::unpack(lds->cl[k * kSB + (i & (kSB - 1))], pk + k * W);
                    } else {
                        load_planes_h<S, 72, NT>(a.clov, 72 / W, 0, i, pk);
                    }
                }
                q = pk + 36 * blk;
            }
            if constexpr (MODE == HOP_INV) {
                block_mul(q, y + 6 * blk, t);
#pragma unroll
                for (int k = 0; k < 6; ++k) y[6 * blk + k] = t[k];
            } else {
                block_mul(q, chi + 6 * blk, t);
#pragma unroll
                for (int k = 0; k < 6; ++k) y[6 * blk + k] = y[6 * blk + k] + t[k];
            }
        }
    }
    T r[24];
#pragma unroll
    for (int k = 0; k < 12; ++k) { r[2 * k] = y[k].r; r[2 * k + 1] = y[k].i; }
    store_field_h<S, 24, NT>(a.out, i, r);
}

// Everything of one output site after the work assignment: the 8 neighbours, then hop_finish.
// Every kernel below (the launch shapes) runs this same arithmetic per site, so all shapes give
// bitwise identical results; the tuner only picks the fastest.  NT: the links also carry the
// streaming hint.
template <typename S, int DAG, int MODE, int NPI = 1, bool NT = false>
DEV void hop_site(const HopArgs<S> &a, int ii, const typename St<S>::vec *tile, int tslot) {
    using T = typename St<S>::acc;
    const uint32_t i = (uint32_t)ii;
    int x[4];
    site_coords(a.g, ii, a.p, x);
    C<T> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = mk(T(0), T(0));
    hop_all<S, DAG, NPI, NT>(a, x, i, acc, tile, tslot);
    hop_finish<S, MODE, NT>(a, i, acc);
}

template <typename S, int DAG, int MODE, int BS>
__global__ __launch_bounds__(BS) void k_hop(HopArgs<S> a) {
    // logical work-group -> (site block, right-hand side), right-hand side fastest so that the
    // right-hand sides of a site block run close in time on one XCD and share its links in L2
    const int lb = a.xcd ? xcd_block(a.nb8) : (int)blockIdx.x;
    const int rhs = lb % a.nrhs, blk = lb / a.nrhs;
    if (a.active && !a.active[rhs]) return;
    const int ii = blk * BS + threadIdx.x;
    if (ii >= a.g.vh) return;
    if (rhs) {
        a.in += rhs * a.vs;
        a.out += rhs * a.vs;
        if (a.chi) a.chi += rhs * a.vs;
    }
    hop_site<S, DAG, MODE>(a, ii, nullptr, 0);
}

// Persistent variant: a grid of a few work-groups per compute unit sweeps the logical blocks
// in order (block lb + k * gridDim.x in step k).  Every compute unit works on the same narrow
// band of the lattice at a time, so the lattice window in flight on each XCD, and with it the
// data streamed through its L2 between two reads of one input spinor by different neighbours,
// is set by the grid rather than by the register-limited occupancy.
// With XCD the grid (a multiple of 8) is split by XCD instead: the work-groups of XCD k sweep
// the k-th contiguous eighth of the logical blocks.
template <typename S, int DAG, int MODE, int BS, int XCD, int NPI, bool NT>
__global__ __launch_bounds__(BS) void k_hop_p(HopArgs<S> a, int nlog) {
    const int region = XCD ? (nlog + 7) >> 3 : nlog;
    const int first = XCD ? (int)(blockIdx.x & 7) * region : 0;
    const int stride = XCD ? (int)(gridDim.x >> 3) : (int)gridDim.x;
#pragma nounroll
    for (int j = XCD ? (int)(blockIdx.x >> 3) : (int)blockIdx.x; j < region; j += stride) {
        const int lb = first + j;
        if (lb >= nlog) break;
        const int rhs = lb % a.nrhs, blk = lb / a.nrhs;
        if (a.active && !a.active[rhs]) continue;
        const int ii = blk * BS + threadIdx.x;
        if (ii >= a.g.vh) continue;
        HopArgs<S> b = a;
        if (rhs) {
            b.in += rhs * a.vs;
            b.out += rhs * a.vs;
            if (b.chi) b.chi += rhs * a.vs;
        }
        hop_site<S, DAG, MODE, NPI, NT>(b, ii, nullptr, 0);
    }
}

// Several right-hand sides per work-item: work-item (site, chunk) computes right-hand sides
// rhs0 .. rhs0 + NR - 1 of its site, reading each link and the clover block once for all of them
// (in registers) while every right-hand side's spinors are read exactly as in the one-RHS
// kernel; the per-right-hand-side sums run in the same order, so the results are bitwise those
// of the one-RHS kernel.  Right-hand sides at or beyond a.nrhs, or inactive, are skipped.
template <typename S, int DAG, int MODE, int NR, bool NT>
DEV void hop_site_mr(const HopArgs<S> &a, int ii, int rhs0) {
    using T = typename St<S>::acc;
    using V = typename St<S>::vec;
    constexpr int W = St<S>::W;
    const uint32_t i = (uint32_t)ii;
    int x[4];
    site_coords(a.g, ii, a.p, x);
    const int row = (x[0] * a.g.L[1] + x[1]) * a.g.L[2] + x[2];
    bool on[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) on[r] = rhs0 + r < a.nrhs && (!a.active || a.active[rhs0 + r]);
    C<T> acc[NR][12];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[r][k] = mk(T(0), T(0));
#pragma nounroll
    for (int n = 0; n < 8; ++n) {
        C<T> u[6];
        T co, si;
        load_link<S, NT>(a, n, i, u, co, si);
        const uint32_t j = neighbour(a, x, row, n);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (!on[r]) continue;
            C<T> psi[12];
            load_spinor<S>(a.in + (size_t)(rhs0 + r) * a.vs, j, psi);
            accumulate_dir<T, DAG>(n, psi, u, co, si, acc[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[r][k] = a.coef * acc[r][k];
    if constexpr (MODE != HOP_PLAIN) {
        // one chirality block (36 packed reals) of the clover field at a time where 36 reals are
        // whole planes (FP64, FP32); with 8 reals per plane (16-bit storage) all 72 at once
        constexpr bool split = (36 % W) == 0;
        auto apply_block = [&](const T *q, int blk, int r, const C<T> *chi) {
            C<T> t[6];
            if constexpr (MODE == HOP_INV) {
                block_mul(q, acc[r] + 6 * blk, t);
#pragma unroll
                for (int k = 0; k < 6; ++k) acc[r][6 * blk + k] = t[k];
            } else {
                block_mul(q, chi, t);
#pragma unroll
                for (int k = 0; k < 6; ++k) acc[r][6 * blk + k] = acc[r][6 * blk + k] + t[k];
            }
        };
        if constexpr (split) {
            T pk[36];
#pragma unroll
            for (int blk = 0; blk < 2; ++blk) {
                load_planes_h<S, 36, NT>(a.clov, 72 / W, blk * (36 / W), i, pk);
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    if (!on[r]) continue;
                    C<T> chi[6];
                    if constexpr (MODE == HOP_CLOV) {
                        T cr[12];
                        load_planes_h<S, 12, NT>(a.chi + (size_t)(rhs0 + r) * a.vs, 24 / W, blk * (12 / W), i, cr);
#pragma unroll
                        for (int k = 0; k < 6; ++k) chi[k] = mk(cr[2 * k], cr[2 * k + 1]);
                    }
                    apply_block(pk, blk, r, chi);
                }
            }
        } else {
            T pk[72];
            load_planes_h<S, 72, NT>(a.clov, 72 / W, 0, i, pk);
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (!on[r]) continue;
                C<T> chi[12];
                if constexpr (MODE == HOP_CLOV) {
                    T cr[24];
                    load_planes_h<S, 24, NT>(a.chi + (size_t)(rhs0 + r) * a.vs, 24 / W, 0, i, cr);
#pragma unroll
                    for (int k = 0; k < 12; ++k) chi[k] = mk(cr[2 * k], cr[2 * k + 1]);
                }
                apply_block(pk, 0, r, chi);
                apply_block(pk + 36, 1, r, chi + 6);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (!on[r]) continue;
        T o[24];
#pragma unroll
        for (int k = 0; k < 12; ++k) { o[2 * k] = acc[r][k].r; o[2 * k + 1] = acc[r][k].i; }
        store_field_h<S, 24, NT>((V *)(a.out + (size_t)(rhs0 + r) * a.vs), i, o);
    }
}

// Persistent sweep over (site block, chunk of NR right-hand sides), chunk fastest, so the chunks
// of one site block run back to back on one XCD and share its links and clover block in L2.
template <typename S, int DAG, int MODE, int BS, int NR, bool NT>
__global__ __launch_bounds__(BS) void k_hop_mr(HopArgs<S> a, int nlog) {
    const int nch = (a.nrhs + NR - 1) / NR;
#pragma nounroll
    for (int lb = blockIdx.x; lb < nlog; lb += gridDim.x) {
        const int ch = lb % nch, blk = lb / nch;
        const int ii = blk * BS + threadIdx.x;
        if (ii >= a.g.vh) continue;
        hop_site_mr<S, DAG, MODE, NR, NT>(a, ii, ch * NR);
    }
}

// Right-hand-side blocked kernel: a work-group of NW wavefronts takes one 64-site block and all
// right-hand sides.  First the work-group prepares, once for the block, everything of a site that
// does not depend on the right-hand side: per direction the link's stored rows with its third row
// rebuilt, the phase's cos and sin, and the neighbour's index (LdsBlock), and it copies the clover
// block.  Wavefront w then computes right-hand sides w, w + NW, ... of the block from LDS: per
// right-hand side only the neighbour spinors come from memory and only the projections, link
// products and reconstruction are computed.  So every link and clover entry is read from HBM once
// per site whatever the number of right-hand sides, and the third rows, phases and indices are
// computed once instead of once per right-hand side.  The rebuilt rows and phases are the values
// the one-RHS kernel computes with the same code, and each site's sums run in the same order, so
// the results equal the one-RHS kernel's bit for bit.  Work-group b takes block b (dispatch
// order: blocks 8 and 256 apart, the x1 and time neighbours at 32^3 x 64, run on the same XCD),
// or with X1S the blocks in the x1-split order of k_hop_px (XCD b % 8 walks the time slices of its
// eighth of the x1 range, so the x2 neighbours are on the same XCD too).
// PF: the loop over the 8 directions is unrolled by two with the next direction's spinor loads
// issued before the current direction's arithmetic.  The stores of the output and the loads of
// chi carry a streaming hint.
template <typename S, int DAG, int MODE, int NW, bool PF, bool X1S>
__global__ __launch_bounds__(64 * NW) void k_hop_rb(HopArgs<S> a) {
    using T = typename St<S>::acc;
    using V = typename St<S>::vec;
    constexpr int CP = 72 / St<S>::W;  // clover planes
    constexpr int NL = 20;             // reals per link in LDS: u[0..5], r2[0..2], cos, sin
    __shared__ T s_lk[8 * NL * kSB];
    __shared__ uint32_t s_nb[8 * kSB];
    __shared__ V s_cl[MODE != HOP_PLAIN ? CP * kSB : 1];
    int blk = (int)blockIdx.x;
    if constexpr (X1S) {
        const int bps = a.g.vh / (a.g.L[0] * 8 * kSB);  // blocks in an XCD's part of a time slice
        const int j = blk >> 3;
        blk = ((j / bps) * 8 + (blk & 7)) * bps + j % bps;
    }
    const int t = (int)threadIdx.x;
    for (int k = t; k < 8 * kSB; k += 64 * NW) {
        const int n = k / kSB, ln = k - n * kSB;
        const int ii = blk * kSB + ln;
        if (ii >= a.g.vh) continue;  // padding sites: never read below
        int x[4];
        site_coords(a.g, ii, a.p, x);
        const int row = (x[0] * a.g.L[1] + x[1]) * a.g.L[2] + x[2];
        s_nb[k] = neighbour(a, x, row, n);
        C<T> u[6], r2[3];
        T co, si;
        load_link<S, true>(a, n, (uint32_t)ii, u, co, si);
        third_row(u, r2);
        T *d = s_lk + (size_t)n * NL * kSB + ln;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            d[(2 * q) * kSB] = u[q].r;
            d[(2 * q + 1) * kSB] = u[q].i;
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            d[(12 + 2 * q) * kSB] = r2[q].r;
            d[(13 + 2 * q) * kSB] = r2[q].i;
        }
        d[18 * kSB] = co;
        d[19 * kSB] = si;
    }
    if constexpr (MODE != HOP_PLAIN) {
        for (int k = t; k < CP * kSB; k += 64 * NW) s_cl[k] = ld_stream(a.clov + (size_t)blk * CP * kSB + k);
    }
    __syncthreads();
    const LdsBlock<S> L{s_lk, s_nb, s_cl};
    const int w = t >> 6, lane = t & (kSB - 1), ii = blk * kSB + lane;
    if (ii >= a.g.vh) return;  // no barrier follows
    // direction n of the sum from the spinor psi already loaded
    auto dir = [&](int n, const C<T> psi[12], C<T> acc[12]) {
        C<T> u[6], r2[3];
        const T *q = L.lk + (size_t)n * NL * kSB + lane;
#pragma unroll
        for (int k = 0; k < 6; ++k) u[k] = mk(q[(2 * k) * kSB], q[(2 * k + 1) * kSB]);
#pragma unroll
        for (int k = 0; k < 3; ++k) r2[k] = mk(q[(12 + 2 * k) * kSB], q[(13 + 2 * k) * kSB]);
        accumulate_dir_r2<T, DAG>(n, psi, u, r2, q[18 * kSB], q[19 * kSB], acc);
    };
#pragma nounroll
    for (int r = w; r < a.nrhs; r += NW) {
        if (a.active && !a.active[r]) continue;
        HopArgs<S> b = a;
        b.in += r * a.vs;
        b.out += r * a.vs;
        if (b.chi) b.chi += r * a.vs;
        C<T> acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = mk(T(0), T(0));
        if constexpr (PF) {
            C<T> pa[12], pb[12];
            load_spinor<S>(b.in, L.nb[lane], pa);
#pragma nounroll
            for (int n = 0; n < 8; n += 2) {
                load_spinor<S>(b.in, L.nb[(n + 1) * kSB + lane], pb);
                dir(n, pa, acc);
                if (n + 2 < 8) load_spinor<S>(b.in, L.nb[(n + 2) * kSB + lane], pa);
                dir(n + 1, pb, acc);
            }
        } else {
#pragma nounroll
            for (int n = 0; n < 8; ++n) {
                C<T> psi[12];
                load_spinor<S>(b.in, L.nb[n * kSB + lane], psi);
                dir(n, psi, acc);
            }
        }
        hop_finish<S, MODE, true, true>(b, (uint32_t)ii, acc, &L);
    }
}

// Right-hand-side blocked column walk: a work-group of NW wavefronts owns one 64-site spatial
// block (the same half-index position in every time slice) for a chunk of tc consecutive time
// slices, with all right-hand sides (wavefront w takes right-hand sides w, w + NW, ..., at most R).
// Per slice it stages the block's links (third rows rebuilt, phases as cos and sin), neighbour
// indices and clover block in LDS as k_hop_rb does; the loads of the next slice's staging data are
// issued before the current slice's arithmetic and written to LDS after it.
// Time neighbours: the +t neighbour of output lane l in slice t is input lane l in slice t + 1,
// which is also the -t neighbour of output lane l in slice t + 2.  So when a wavefront loads it
// for the +t term it also forms its -t half-spinor (project_dir_n of direction 1) and keeps it in
// registers for two slices: after the first two slices of a chunk the -t neighbour is not loaded.
// Each site's terms are summed in the order of the one-RHS kernel, so the results are bitwise its.
// All waves of an XCD work on neighbouring columns at the same slice, so the spatial neighbours of
// slice t + 1 are read one slice after their +t loads.  Work-groups: spatial block fastest, then
// chunk; with X1S the spatial blocks of XCD k (work-group index = k mod 8) are the k-th eighth of
// a slice (its x1 range), so the x2 and x3 neighbours are on the same XCD.  Needs whole blocks per
// time slice; the host checks the fit.
template <typename T, int DAG, int N>
DEV void apply_lds(const T *lk, int lane, const C<T> h[6], C<T> acc[12]) {
    constexpr int NL = 20;
    const T *q = lk + (size_t)N * NL * kSB + lane;
    C<T> u[6], r2[3];
#pragma unroll
    for (int k = 0; k < 6; ++k) u[k] = mk(q[(2 * k) * kSB], q[(2 * k + 1) * kSB]);
#pragma unroll
    for (int k = 0; k < 3; ++k) r2[k] = mk(q[(12 + 2 * k) * kSB], q[(13 + 2 * k) * kSB]);
    apply_dir_n<T, DAG, N>(h, u, r2, q[18 * kSB], q[19 * kSB], acc);
}

template <typename T, int DAG, int N>
DEV void dir_lds(const T *lk, int lane, const C<T> psi[12], C<T> acc[12]) {
    C<T> h[6];
    project_dir_n<T, DAG, N>(psi, h);
    apply_lds<T, DAG, N>(lk, lane, h, acc);
}

// DB: the staging data is double-buffered in LDS, so a slice's data is written while the previous
// slice is still being computed from the other buffer (one barrier per slice instead of two).
template <typename S, int DAG, int MODE, int NW, int R, bool X1S, bool DB>
__global__ __launch_bounds__(64 * NW) void k_hop_rbc(HopArgs<S> a, int tc) {
    using T = typename St<S>::acc;
    using V = typename St<S>::vec;
    using LV = typename Lk<S>::vec;
    using OM = typename Lk<S>::om;
    constexpr int LW = Lk<S>::W;
    constexpr int CP = 72 / St<S>::W;  // clover planes
    constexpr int NL = 20;             // reals per link in LDS: u[0..5], r2[0..2], cos, sin
    constexpr int NTH = 64 * NW;
    constexpr int LI = (8 * kSB + NTH - 1) / NTH;                               // link items per thread
    constexpr int CI = MODE != HOP_PLAIN ? (CP * kSB + NTH - 1) / NTH : 1;     // clover vectors per thread
    constexpr int NB = DB ? 2 : 1;  // LDS buffers
    __shared__ T s_lk[NB][8 * NL * kSB];
    __shared__ uint32_t s_nb[NB][8 * kSB];
    __shared__ V s_cl[NB][MODE != HOP_PLAIN ? CP * kSB : 1];
    const int nsb = a.g.vh / (a.g.L[0] * kSB);  // spatial blocks per time slice
    int sb, ch;
    if constexpr (X1S) {
        const int per = nsb >> 3, j = (int)blockIdx.x >> 3;
        sb = ((int)blockIdx.x & 7) * per + j % per;
        ch = j / per;
    } else {
        sb = (int)blockIdx.x % nsb;
        ch = (int)blockIdx.x / nsb;
    }
    const int t0 = ch * tc;
    const int tid = (int)threadIdx.x, w = tid >> 6, lane = tid & (kSB - 1);
    const size_t vhp = (size_t)a.g.vhp;
    LV lraw[LI][12 / LW];
    OM oraw[LI];
    V craw[CI];
    // issue the loads of slice t's staging data (links, phases, clover block)
    auto fetch = [&](int t) {
        const int blk = t * nsb + sb;
#pragma unroll
        for (int k = 0; k < LI; ++k) {
            const int item = tid + k * NTH;
            if (item < 8 * kSB) {
                const int n = item / kSB;
                const uint32_t ii = (uint32_t)(blk * kSB + (item & (kSB - 1)));
                const LV *b = site_ptr(a.links + (size_t)n * (12 / LW) * vhp, ii, 12 / LW);
#pragma unroll
                for (int q = 0; q < 12 / LW; ++q) lraw[k][q] = ld_stream(b + q * kSB);
                oraw[k] = ld_stream(a.omega + (size_t)n * vhp + ii);
            }
        }
        if constexpr (MODE != HOP_PLAIN) {
#pragma unroll
            for (int k = 0; k < CI; ++k) {
                const int item = tid + k * NTH;
                if (item < CP * kSB) craw[k] = ld_stream(a.clov + (size_t)blk * CP * kSB + item);
            }
        }
    };
    // rebuild slice t's staging data and write it to LDS buffer bf
    auto commit = [&](int t, int bf) {
        const int blk = t * nsb + sb;
#pragma unroll
        for (int k = 0; k < LI; ++k) {
            const int item = tid + k * NTH;
            if (item < 8 * kSB) {
                const int n = item / kSB, ln = item & (kSB - 1);
                const int ii = blk * kSB + ln;
                int x[4];
                site_coords(a.g, ii, a.p, x);
                const int row = (x[0] * a.g.L[1] + x[1]) * a.g.L[2] + x[2];
                s_nb[bf][item] = neighbour(a, x, row, n);
                T r[12];
#pragma unroll
                for (int q = 0; q < 12 / LW; ++q) Lk<S>::unpack(lraw[k][q], r + q * LW);
                C<T> u[6], r2[3];
#pragma unroll
                for (int q = 0; q < 6; ++q) u[q] = mk(r[2 * q], r[2 * q + 1]);
                T co, si;
                if constexpr (Lk<S>::phase_pair) Lk<S>::phase(oraw[k], co, si);
                else sc((T)oraw[k], si, co);
                third_row(u, r2);
                T *d = s_lk[bf] + (size_t)n * NL * kSB + ln;
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    d[(2 * q) * kSB] = u[q].r;
                    d[(2 * q + 1) * kSB] = u[q].i;
                }
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    d[(12 + 2 * q) * kSB] = r2[q].r;
                    d[(13 + 2 * q) * kSB] = r2[q].i;
                }
                d[18 * kSB] = co;
                d[19 * kSB] = si;
            }
        }
        if constexpr (MODE != HOP_PLAIN) {
#pragma unroll
            for (int k = 0; k < CI; ++k) {
                const int item = tid + k * NTH;
                if (item < CP * kSB) s_cl[bf][item] = craw[k];
            }
        }
    };
    C<T> carry[R][2][6];  // [slot][k & 1]: -t half-spinor of the slice loaded as +t neighbour at step k
    // one time slice (step k of the chunk) with the carry slot SL = k & 1 fixed at compile time
    auto step = [&](int k, auto slot) {
        constexpr int SL = decltype(slot)::value;
        const int t = t0 + k;
        const int bf = DB ? SL : 0;  // buffer of slice t: k & 1 (= SL) with double buffering
        if constexpr (!DB) {
            __syncthreads();  // the previous slice's LDS data has been read
            commit(t, 0);
            __syncthreads();
            if (k + 1 < tc) fetch(t + 1);  // in flight during this slice's arithmetic
        }
        const LdsBlock<S> L{s_lk[bf], s_nb[bf], s_cl[bf]};
        const uint32_t ii = (uint32_t)((t * nsb + sb) * kSB + lane);
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = w + q * NW;
            if (r >= a.nrhs) break;
            if (a.active && !a.active[r]) continue;
            HopArgs<S> b = a;
            b.in += r * a.vs;
            b.out += r * a.vs;
            if (b.chi) b.chi += r * a.vs;
            C<T> acc[12];
#pragma unroll
            for (int j = 0; j < 12; ++j) acc[j] = mk(T(0), T(0));
            C<T> pa[12], pb[12];
            load_spinor<S>(b.in, L.nb[lane], pa);                                // +t neighbour
            if (k < 2) load_spinor<S>(b.in, L.nb[kSB + lane], pb);               // -t neighbour, not yet kept
            dir_lds<T, DAG, 0>(L.lk, lane, pa, acc);
            C<T> hb[6];
            project_dir_n<T, DAG, 1>(pa, hb);  // the -t half-spinor of output lane l two slices later
            load_spinor<S>(b.in, L.nb[2 * kSB + lane], pa);
            if (k < 2) {
                C<T> h1[6];
                project_dir_n<T, DAG, 1>(pb, h1);
                apply_lds<T, DAG, 1>(L.lk, lane, h1, acc);
            } else {
                apply_lds<T, DAG, 1>(L.lk, lane, carry[q][SL], acc);
            }
#pragma unroll
            for (int j = 0; j < 6; ++j) carry[q][SL][j] = hb[j];
            load_spinor<S>(b.in, L.nb[3 * kSB + lane], pb);
            dir_lds<T, DAG, 2>(L.lk, lane, pa, acc);
            load_spinor<S>(b.in, L.nb[4 * kSB + lane], pa);
            dir_lds<T, DAG, 3>(L.lk, lane, pb, acc);
            load_spinor<S>(b.in, L.nb[5 * kSB + lane], pb);
            dir_lds<T, DAG, 4>(L.lk, lane, pa, acc);
            load_spinor<S>(b.in, L.nb[6 * kSB + lane], pa);
            dir_lds<T, DAG, 5>(L.lk, lane, pb, acc);
            load_spinor<S>(b.in, L.nb[7 * kSB + lane], pb);
            dir_lds<T, DAG, 6>(L.lk, lane, pa, acc);
            dir_lds<T, DAG, 7>(L.lk, lane, pb, acc);
            hop_finish<S, MODE, true, true>(b, ii, acc, &L);
        }
        if constexpr (DB) {
            // the next slice into the other buffer (last read in the previous slice, before the
            // barrier that ended it), then the loads of the one after it
            if (k + 1 < tc) {
                commit(t + 1, SL ^ 1);
                if (k + 2 < tc) fetch(t + 2);
            }
            __syncthreads();
        }
    };
    fetch(t0);
    if constexpr (DB) {
        commit(t0, 0);
        if (tc > 1) fetch(t0 + 1);
        __syncthreads();
    }
#pragma nounroll
    for (int k = 0; k < tc; k += 2) {
        step(k, std::integral_constant<int, 0>());
        if (k + 1 < tc) step(k + 1, std::integral_constant<int, 1>());
    }
}

// Slab sweep: XCD k (work-groups b with b % 8 == k) owns the time slices [k L0 / 8, (k + 1) L0 / 8)
// and walks them with time faster than x1: the work-groups of one XCD in flight together cover a
// few (t, x1) planes of all its time slices, so the neighbours in every direction but across the
// slab's time boundaries are read by the same XCD within a short window and hit in its L2.
// Needs L0 % 8 == 0 and the sites of one parity in a (t, x1) plane a multiple of BS.
template <typename S, int DAG, int MODE, int BS, int NPI = 1, bool NT = false>
__global__ __launch_bounds__(BS) void k_hop_ps(HopArgs<S> a, int nper) {
    const int xcd = (int)(blockIdx.x & 7);
    const int T8 = a.g.L[0] >> 3;
    const int plane = a.g.vh / (a.g.L[0] * a.g.L[1]);
    const int cpp = plane / BS;
#pragma nounroll
    for (int j = (int)(blockIdx.x >> 3); j < nper; j += (int)(gridDim.x >> 3)) {
        const int rhs = j % a.nrhs;
        int r = j / a.nrhs;
        const int h = r % cpp;
        r /= cpp;
        const int t = xcd * T8 + r % T8, x1 = r / T8;
        if (a.active && !a.active[rhs]) continue;
        HopArgs<S> b = a;
        if (rhs) {
            b.in += rhs * a.vs;
            b.out += rhs * a.vs;
            if (b.chi) b.chi += rhs * a.vs;
        }
        hop_site<S, DAG, MODE, NPI, NT>(b, (t * a.g.L[1] + x1) * plane + h * BS + (int)threadIdx.x, nullptr, 0);
    }
}

// x1-split sweep: XCD k (work-groups b with b % 8 == k) owns the x1 range [k L1 / 8, (k + 1) L1 / 8)
// of every time slice, and its work-groups walk the time slices in order.  The sites of one
// parity in that part of a slice are contiguous in the half index, and the work-groups of one
// XCD in flight together cover a few consecutive slices of it: every neighbour but the x1
// neighbours across the XCD's range boundaries is read by the same XCD within a short window
// (a time slice earlier at most) and hits in its L2, while the once-touched streams carry the
// streaming hint.  Needs L1 % 8 == 0; the part of a slice is cut into chunks of BS sites, the last
// one partial when BS does not divide it.
template <typename S, int DAG, int MODE, int BS, int NPI, bool NT>
__global__ __launch_bounds__(BS) void k_hop_px(HopArgs<S> a, int nper) {
    const int xcd = (int)(blockIdx.x & 7);
    const int sub = a.g.vh / (a.g.L[0] * 8);  // sites of one parity in an XCD's part of a time slice
    const int cps = (sub + BS - 1) / BS;
#pragma nounroll
    for (int j = (int)(blockIdx.x >> 3); j < nper; j += (int)(gridDim.x >> 3)) {
        const int rhs = j % a.nrhs;
        const int r = j / a.nrhs;
        const int c = r % cps, t = r / cps;
        if (a.active && !a.active[rhs]) continue;
        if (c * BS + (int)threadIdx.x >= sub) continue;  // no barrier follows
        HopArgs<S> b = a;
        if (rhs) {
            b.in += rhs * a.vs;
            b.out += rhs * a.vs;
            if (b.chi) b.chi += rhs * a.vs;
        }
        hop_site<S, DAG, MODE, NPI, NT>(b, (t * 8 + xcd) * sub + c * BS + (int)threadIdx.x, nullptr, 0);
    }
}

// Time-tiled variant: a work-group of TT wavefronts takes one spatial block of 64 sites in TT
// consecutive time slices.  Each wavefront stages the input block of its slice in LDS, the
// first and last also the blocks of the slices just outside the tile (periodic in time), so
// both time-direction neighbours of every site are read from LDS and each input block is
// fetched once per tile instead of three times (its own slice and the slices above and
// below).  Needs (L1 L2 L3 / 2) % 64 == 0 and L0 % TT == 0.
template <typename S, int DAG, int MODE, int TT>
__global__ __launch_bounds__(64 * TT) void k_hop_t(HopArgs<S> a) {
    using V = typename St<S>::vec;
    constexpr int NP = 24 / St<S>::W;
    __shared__ V tile[(TT + 2) * NP * kSB];
    const int lb = a.xcd ? xcd_block(a.nb8) : (int)blockIdx.x;
    const int nsb = a.g.vh / (a.g.L[0] * kSB);  // site blocks per time slice
    const int rhs = lb % a.nrhs, wg = lb / a.nrhs;
    const int sb = wg % nsb, t0 = (wg / nsb) * TT;
    if (t0 >= a.g.L[0]) return;
    if (a.active && !a.active[rhs]) return;
    if (rhs) {
        a.in += rhs * a.vs;
        a.out += rhs * a.vs;
        if (a.chi) a.chi += rhs * a.vs;
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & (kSB - 1);
    auto stage = [&](int slot, int t) {
        const V *src = a.in + ((size_t)(t * nsb + sb) * NP) * kSB + lane;
        V *dst = tile + (size_t)slot * NP * kSB + lane;
#pragma unroll
        for (int k = 0; k < NP; ++k) dst[k * kSB] = src[k * kSB];
    };
    stage(w + 1, t0 + w);
    if (w == 0) stage(0, t0 == 0 ? a.g.L[0] - 1 : t0 - 1);
    if (w == TT - 1) stage(TT + 1, t0 + TT == a.g.L[0] ? 0 : t0 + TT);
    __syncthreads();
    const int ii = ((t0 + w) * nsb + sb) * kSB + lane;
    hop_site<S, DAG, MODE>(a, ii, tile, w + 1);
}

// Persistent form of the time-tiled kernel: the grid sweeps the tiles in order, spatial block
// fastest, so one band of TT time slices is in flight at a time.
template <typename S, int DAG, int MODE, int TT>
__global__ __launch_bounds__(64 * TT) void k_hop_tp(HopArgs<S> a, int nwg) {
    using V = typename St<S>::vec;
    constexpr int NP = 24 / St<S>::W;
    __shared__ V tile[(TT + 2) * NP * kSB];
    const int nsb = a.g.vh / (a.g.L[0] * kSB);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & (kSB - 1);
#pragma nounroll
    for (int lb = blockIdx.x; lb < nwg; lb += gridDim.x) {
        const int rhs = lb % a.nrhs, wg = lb / a.nrhs;
        if (a.active && !a.active[rhs]) continue;  // uniform over the work-group
        const int sb = wg % nsb, t0 = (wg / nsb) * TT;
        HopArgs<S> b = a;
        if (rhs) {
            b.in += rhs * a.vs;
            b.out += rhs * a.vs;
            if (b.chi) b.chi += rhs * a.vs;
        }
        auto stage = [&](int slot, int t) {
            const V *src = b.in + ((size_t)(t * nsb + sb) * NP) * kSB + lane;
            V *dst = tile + (size_t)slot * NP * kSB + lane;
#pragma unroll
            for (int k = 0; k < NP; ++k) dst[k * kSB] = src[k * kSB];
        };
        __syncthreads();  // the previous tile has been consumed
        stage(w + 1, t0 + w);
        if (w == 0) stage(0, t0 == 0 ? a.g.L[0] - 1 : t0 - 1);
        if (w == TT - 1) stage(TT + 1, t0 + TT == a.g.L[0] ? 0 : t0 + TT);
        __syncthreads();
        hop_site<S, DAG, MODE>(b, ((t0 + w) * nsb + sb) * kSB + lane, tile, w + 1);
    }
}

struct HopShape {
    int bs, xcd, tt, pers, slab, npi, nt, mr, rb, pf, x1s, cw, cr, db;
};
// Shape 0 is the default (used when tuning is off, and inside a graph capture before the key
// was tuned): the persistent sweep, one 256-wide work-group per compute unit, two neighbours per
// loop iteration, streaming hints.  tt > 0: the time-tiled kernel (bs = 64 tt); pers > 0: a
// persistent grid of pers work-groups per compute unit (xcd: each XCD sweeps its own eighth);
// slab: the XCD slab sweep; npi: neighbours per loop iteration; nt: streaming hints; mr: right-hand
// sides per work-item (the links and clover block read once for all of them); rb: the right-hand-
// side blocked kernel with rb wavefronts per work-group (link work and clover block in LDS), pf:
// its next-direction prefetch; x1s: the x1-split sweep (or block order); cw: the right-hand-side
// blocked column walk with cw wavefronts per work-group and at most cr right-hand sides each,
// pers work-groups per compute unit wanted (16-bit and FP32 storage only), db: its LDS staging
// double-buffered.
const HopShape kShapes[] = {
    {256, 0, 0, 1, 0, 2, 1, 1}, {256, 0, 0, 1, 0, 1, 1, 1}, {256, 0, 0, 2, 0, 1, 1, 1}, {256, 0, 0, 1, 0, 1, 0, 1},
    {256, 0, 0, 1, 0, 2, 0, 1}, {256, 1, 0, 0, 0, 1, 0, 1}, {256, 0, 0, 0, 0, 1, 0, 1}, {128, 1, 0, 0, 0, 1, 0, 1},
    {64, 1, 0, 0, 0, 1, 0, 1},  {256, 1, 4, 0, 0, 1, 0, 1}, {512, 1, 8, 0, 0, 1, 0, 1}, {512, 0, 0, 1, 0, 1, 0, 1},
    {256, 0, 0, 2, 0, 1, 0, 1}, {256, 1, 0, 1, 0, 1, 0, 1}, {256, 0, 4, 1, 0, 1, 0, 1}, {512, 0, 8, 1, 0, 1, 0, 1},
    {256, 0, 0, 1, 1, 1, 0, 1}, {256, 0, 0, 2, 1, 1, 0, 1}, {128, 0, 0, 2, 1, 1, 0, 1}, {256, 0, 0, 2, 0, 2, 0, 1},
    {256, 0, 0, 1, 0, 1, 1, 2}, {256, 0, 0, 1, 0, 1, 1, 4}, {256, 0, 0, 2, 0, 1, 1, 2},
    {256, 0, 0, 0, 0, 1, 1, 1, 4, 0}, {512, 0, 0, 0, 0, 1, 1, 1, 8, 0}, {256, 0, 0, 0, 0, 1, 1, 1, 4, 1},
    {512, 0, 0, 0, 0, 1, 1, 1, 8, 1}, {768, 0, 0, 0, 0, 1, 1, 1, 12, 1}, {256, 0, 0, 1, 0, 4, 1, 1, 0, 0},
    {256, 0, 0, 2, 0, 4, 1, 1, 0, 0}, {256, 0, 0, 1, 0, 2, 1, 1, 0, 0, 1}, {256, 0, 0, 2, 0, 2, 1, 1, 0, 0, 1},
    {128, 0, 0, 2, 0, 2, 1, 1, 0, 0, 1}, {256, 0, 0, 1, 0, 4, 1, 1, 0, 0, 1}, {256, 0, 0, 1, 1, 2, 1, 1, 0, 0, 0},
    {128, 0, 0, 2, 1, 2, 1, 1, 0, 0, 0}, {256, 0, 0, 2, 0, 4, 1, 1, 0, 0, 1}, {256, 0, 0, 4, 0, 2, 1, 1, 0, 0, 1},
    {256, 0, 0, 0, 0, 1, 1, 1, 4, 1, 1}, {512, 0, 0, 0, 0, 1, 1, 1, 8, 1, 1}, {256, 0, 0, 3, 0, 4, 1, 1, 0, 0, 1},
    {768, 0, 0, 1, 0, 1, 1, 1, 0, 0, 1, 12, 1}, {512, 0, 0, 1, 0, 1, 1, 1, 0, 0, 1, 8, 2},
    {256, 0, 0, 2, 0, 1, 1, 1, 0, 0, 1, 4, 3}, {384, 0, 0, 1, 0, 1, 1, 1, 0, 0, 1, 6, 2},
    {768, 0, 0, 1, 0, 1, 1, 1, 0, 0, 0, 12, 1}, {768, 0, 0, 1, 0, 1, 1, 1, 0, 0, 1, 12, 1, 1},
    {512, 0, 0, 1, 0, 1, 1, 1, 0, 0, 1, 8, 2, 1}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);
template <typename S> constexpr int num_shapes() { return kNumShapes; }

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
bool slab_ok(const Geom &g, int bs) {
    if (g.L[0] % 8) return false;
    const int plane = g.vh / (g.L[0] * g.L[1]);
    return plane % bs == 0;
}
// The x1-split order fits when L1 % 8 == 0; the right-hand-side blocked kernel takes whole site
// blocks, so its XCD's part of a time slice must be whole blocks.
bool x1split_ok(const Geom &g, bool whole_blocks) {
    if (g.L[1] % 8) return false;
    return !whole_blocks || (g.vh / (g.L[0] * 8)) % kSB == 0;
}
// The column walk needs whole 64-site blocks in each time slice.
bool column_ok(const Geom &g) { return (g.vh / g.L[0]) % kSB == 0; }
bool tiled_ok(const Geom &g, int tt) {
    const int ns = g.vh / g.L[0];
    return ns % kSB == 0 && g.L[0] % tt == 0;
}

template <typename S, int DAG, int MODE, int BS>
void launch_shape(HopArgs<S> a, int xcd, hipStream_t s) {
    const int nb = (a.g.vh + BS - 1) / BS * a.nrhs;
    a.xcd = xcd;
    a.nb8 = xcd ? (nb + 7) & ~7 : nb;
    k_hop<S, DAG, MODE, BS><<<a.nb8, BS, 0, s>>>(a);
}

template <typename S, int DAG, int MODE, int BS, int NPI = 1, bool NT = false>
void launch_persistent(HopArgs<S> a, int per_cu, int xcd, hipStream_t s) {
    const int nlog = (a.g.vh + BS - 1) / BS * a.nrhs;
    int grid = std::min(nlog, per_cu * compute_units());
    if (xcd) grid = std::max(8, grid & ~7);
    a.xcd = xcd;
    a.nb8 = grid;
    if (xcd) k_hop_p<S, DAG, MODE, BS, 1, NPI, NT><<<grid, BS, 0, s>>>(a, nlog);
    else k_hop_p<S, DAG, MODE, BS, 0, NPI, NT><<<grid, BS, 0, s>>>(a, nlog);
}

template <typename S, int DAG, int MODE, int BS, int NPI = 1, bool NT = false>
void launch_slab(HopArgs<S> a, int per_cu, hipStream_t s) {
    const int plane = a.g.vh / (a.g.L[0] * a.g.L[1]);
    const int nper = (a.g.L[0] / 8) * a.g.L[1] * (plane / BS) * a.nrhs;
    const int grid = 8 * std::max(1, std::min(nper, per_cu * compute_units() / 8));
    a.xcd = 0;
    a.nb8 = grid;
    k_hop_ps<S, DAG, MODE, BS, NPI, NT><<<grid, BS, 0, s>>>(a, nper);
}

template <typename S, int DAG, int MODE, int BS, int NPI>
void launch_x1split(HopArgs<S> a, int per_cu, hipStream_t s) {
    const int sub = a.g.vh / (a.g.L[0] * 8);
    const int nper = a.g.L[0] * ((sub + BS - 1) / BS) * a.nrhs;
    const int grid = 8 * std::max(1, std::min(nper, per_cu * compute_units() / 8));
    a.xcd = 0;
    a.nb8 = grid;
    k_hop_px<S, DAG, MODE, BS, NPI, true><<<grid, BS, 0, s>>>(a, nper);
}

template <typename S, int DAG, int MODE, int NR>
void launch_multi(HopArgs<S> a, int per_cu, hipStream_t s) {
    const int nch = (a.nrhs + NR - 1) / NR;
    const int nlog = (a.g.vh + 255) / 256 * nch;
    const int grid = std::min(nlog, per_cu * compute_units());
    a.xcd = 0;
    a.nb8 = grid;
    k_hop_mr<S, DAG, MODE, 256, NR, true><<<grid, 256, 0, s>>>(a, nlog);
}

template <typename S, int DAG, int MODE, int TT>
void launch_tiled_persistent(HopArgs<S> a, int per_cu, hipStream_t s) {
    const int nwg = (a.g.L[0] / TT) * (a.g.vh / (a.g.L[0] * kSB)) * a.nrhs;
    const int grid = std::min(nwg, per_cu * compute_units());
    a.xcd = 0;
    a.nb8 = grid;
    k_hop_tp<S, DAG, MODE, TT><<<grid, 64 * TT, 0, s>>>(a, nwg);
}

template <typename S, int DAG, int MODE, int TT>
void launch_tiled(HopArgs<S> a, hipStream_t s) {
    const int nb = (a.g.L[0] / TT) * (a.g.vh / (a.g.L[0] * kSB)) * a.nrhs;
    a.xcd = 1;
    a.nb8 = (nb + 7) & ~7;
    k_hop_t<S, DAG, MODE, TT><<<a.nb8, 64 * TT, 0, s>>>(a);
}

// Column walk: chunks of tc time slices, tc the largest divisor of L0 of at least 4 slices (or
// L0 itself) that still gives per_cu work-groups per compute unit where the lattice allows.
template <typename S, int DAG, int MODE, int NW, int R, bool DB = false>
void launch_rbc(HopArgs<S> a, int per_cu, bool x1s, hipStream_t s) {
    const int L0 = a.g.L[0];
    const int nsb = a.g.vh / (L0 * kSB);
    const int want = per_cu * compute_units();
    int nch = 1;
    while ((int64_t)nsb * nch < want) {
        int nx = nch + 1;
        while (nx <= L0 && L0 % nx) ++nx;
        if (nx > L0 || L0 / nx < 4) break;
        nch = nx;
    }
    const int tc = L0 / nch;
    const int grid = nsb * nch;
    a.xcd = 0;
    a.nb8 = grid;
    if (x1s && nsb % 8 == 0) k_hop_rbc<S, DAG, MODE, NW, R, true, DB><<<grid, 64 * NW, 0, s>>>(a, tc);
    else k_hop_rbc<S, DAG, MODE, NW, R, false, DB><<<grid, 64 * NW, 0, s>>>(a, tc);
}

template <typename S, int DAG, int MODE, int NW>
void launch_rb_nw(HopArgs<S> a, bool pf, bool x1s, hipStream_t s) {
    a.xcd = 0;
    a.nb8 = (a.g.vh + kSB - 1) / kSB;
    if (x1s) k_hop_rb<S, DAG, MODE, NW, true, true><<<a.nb8, 64 * NW, 0, s>>>(a);  // pf with x1s only
    else if (pf) k_hop_rb<S, DAG, MODE, NW, true, false><<<a.nb8, 64 * NW, 0, s>>>(a);
    else k_hop_rb<S, DAG, MODE, NW, false, false><<<a.nb8, 64 * NW, 0, s>>>(a);
}

template <typename S, int DAG, int MODE>
void launch_rb(const HopArgs<S> &a, int nw, bool pf, bool x1s, hipStream_t s) {
    // FP64 needs about 176 registers per lane: at most two wavefronts per SIMD, 8 per work-group
    if (nw == 4) launch_rb_nw<S, DAG, MODE, 4>(a, pf, x1s, s);
    else if (nw == 8 || std::is_same<S, double>::value) launch_rb_nw<S, DAG, MODE, 8>(a, pf, x1s, s);
    else if constexpr (!std::is_same<S, double>::value) launch_rb_nw<S, DAG, MODE, 12>(a, pf, false, s);
}

template <typename S, int DAG, int MODE>
void launch_hop(const HopArgs<S> &a, int shape, hipStream_t s) {
    HopShape h = kShapes[shape];
    if ((h.tt && !tiled_ok(a.g, h.tt)) || (h.slab && !slab_ok(a.g, h.bs)) ||
        (h.x1s && !h.cw && !x1split_ok(a.g, h.rb != 0)) ||
        (h.cw && (std::is_same<S, double>::value || !column_ok(a.g) || a.nrhs > h.cw * h.cr)))
        h = kShapes[0];  // does not fit
    if (h.cw) {
        if constexpr (!std::is_same<S, double>::value) {
            if (h.cw == 12 && h.db) launch_rbc<S, DAG, MODE, 12, 1, true>(a, h.pers, h.x1s != 0, s);
            else if (h.cw == 8 && h.db) launch_rbc<S, DAG, MODE, 8, 2, true>(a, h.pers, h.x1s != 0, s);
            else if (h.cw == 12) launch_rbc<S, DAG, MODE, 12, 1>(a, h.pers, h.x1s != 0, s);
            else if (h.cw == 8) launch_rbc<S, DAG, MODE, 8, 2>(a, h.pers, h.x1s != 0, s);
            else if (h.cw == 6) launch_rbc<S, DAG, MODE, 6, 2>(a, h.pers, h.x1s != 0, s);
            else launch_rbc<S, DAG, MODE, 4, 3>(a, h.pers, h.x1s != 0, s);
        }
    } else if (h.rb) {
        launch_rb<S, DAG, MODE>(a, h.rb, h.pf != 0, h.x1s != 0, s);
    } else if (h.mr > 1) {
        // two right-hand sides per work-item in FP64 (four would not fit the registers)
        if constexpr (std::is_same<S, double>::value) {
            launch_multi<S, DAG, MODE, 2>(a, h.pers, s);
        } else {
            if (h.mr == 2) launch_multi<S, DAG, MODE, 2>(a, h.pers, s);
            else launch_multi<S, DAG, MODE, 4>(a, h.pers, s);
        }
    } else if (h.tt) {
        if (h.pers) {
            if (h.tt == 4) launch_tiled_persistent<S, DAG, MODE, 4>(a, h.pers, s);
            else launch_tiled_persistent<S, DAG, MODE, 8>(a, h.pers, s);
        } else {
            if (h.tt == 4) launch_tiled<S, DAG, MODE, 4>(a, s);
            else launch_tiled<S, DAG, MODE, 8>(a, s);
        }
    } else if (h.x1s) {
        if (h.npi == 4) launch_x1split<S, DAG, MODE, 256, 4>(a, h.pers, s);
        else if (h.bs == 256) launch_x1split<S, DAG, MODE, 256, 2>(a, h.pers, s);
        else launch_x1split<S, DAG, MODE, 128, 2>(a, h.pers, s);
    } else if (h.slab) {
        if (h.nt && h.bs == 256) launch_slab<S, DAG, MODE, 256, 2, true>(a, h.pers, s);
        else if (h.nt) launch_slab<S, DAG, MODE, 128, 2, true>(a, h.pers, s);
        else if (h.bs == 256) launch_slab<S, DAG, MODE, 256>(a, h.pers, s);
        else launch_slab<S, DAG, MODE, 128>(a, h.pers, s);
    } else if (h.pers) {
        if (h.bs == 512) launch_persistent<S, DAG, MODE, 512>(a, h.pers, h.xcd, s);
        else if (h.nt && h.npi == 4) launch_persistent<S, DAG, MODE, 256, 4, true>(a, h.pers, 0, s);
        else if (h.nt && h.npi == 2) launch_persistent<S, DAG, MODE, 256, 2, true>(a, h.pers, 0, s);
        else if (h.nt) launch_persistent<S, DAG, MODE, 256, 1, true>(a, h.pers, 0, s);
        else if (h.npi == 2) launch_persistent<S, DAG, MODE, 256, 2>(a, h.pers, 0, s);
        else launch_persistent<S, DAG, MODE, 256>(a, h.pers, h.xcd, s);
    } else {
        if (h.bs == 256) launch_shape<S, DAG, MODE, 256>(a, h.xcd, s);
        else if (h.bs == 128) launch_shape<S, DAG, MODE, 128>(a, h.xcd, s);
        else launch_shape<S, DAG, MODE, 64>(a, h.xcd, s);
    }
}

template <typename S>
void hop_t(dirac_ctx *c, void *out, const void *in, const void *chi, int p, HopMode mode, double coef, int dagger,
           dirac_prec pr, hipStream_t s, int nrhs, const int *active, bool no_tune) {
    PrecFields &f = c->f[pr];
    HopArgs<S> a;
    a.g = c->g;
    a.p = p;
    a.nb8 = 0;
    a.nrhs = nrhs;
    a.vs = (size_t)(24 / St<S>::W) * c->g.vhp;
    a.active = active;
    a.in = (const typename St<S>::vec *)in;
    a.links = (const typename Lk<S>::vec *)f.links[p].p;
    a.omega = (const typename Lk<S>::om *)f.omega[p].p;
    a.clov = (const typename St<S>::vec *)(mode == HOP_INV ? f.clinv[p].p : mode == HOP_CLOV ? f.clov[p].p : nullptr);
    a.chi = (const typename St<S>::vec *)chi;
    a.out = (typename St<S>::vec *)out;
    a.coef = (typename St<S>::acc)coef;
    a.xcd = 1;
    auto launch = [&](int shape) {
        if (dagger) {
            if (mode == HOP_PLAIN) launch_hop<S, 1, HOP_PLAIN>(a, shape, s);
            else if (mode == HOP_INV) launch_hop<S, 1, HOP_INV>(a, shape, s);
            else launch_hop<S, 1, HOP_CLOV>(a, shape, s);
        } else {
            if (mode == HOP_PLAIN) launch_hop<S, 0, HOP_PLAIN>(a, shape, s);
            else if (mode == HOP_INV) launch_hop<S, 0, HOP_INV>(a, shape, s);
            else launch_hop<S, 0, HOP_CLOV>(a, shape, s);
        }
        HIP_CHECK(hipGetLastError());
    };
    char key[160];
    snprintf(key, sizeof key, "hop-v2|%s|dag%d|mode%d|%dx%dx%dx%d|nrhs%d", prec_name(pr), dagger, (int)mode,
             c->g.L[0], c->g.L[1], c->g.L[2], c->g.L[3], nrhs);
    if (no_tune) {
        // no timing runs (they create events): the shape tuned earlier for this key, else shape 0
        const int v = tuned_lookup(key);
        launch(v >= 0 && v < num_shapes<S>() ? v : 0);
    } else {
        launch(tuned_choice(key, num_shapes<S>(), launch, s));
    }
}

}  // namespace
}  // namespace dl
