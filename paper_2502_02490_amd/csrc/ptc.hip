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
    const float4 *links[2];  // FP32 links per parity: [8 dir][3 planes] blocked
    const float *omega[2];   // [8 dir][vhp]
    size_t chan;             // floats per channel (a full NATIVE FP32 vector)
};

DEV void bf2(uint32_t w, float &re, float &im) {
    re = __uint_as_float(w << 16);
    im = __uint_as_float(w & 0xffff0000u);
}

// t = T_path x_c (full spinor, 12 complex) at site (p, i) with coordinates x
DEV void transport_site(const PtcGeom &a, const float4 *xc, int p, uint32_t i, const int x[4], int path,
                        C<float> t[12]) {
    const size_t hv = (size_t)6 * a.g.vhp;  // float4 per half vector
    if (path == 0) {
        float r[24];
        load_field<float, 24>(xc + p * hv, i, r);
#pragma unroll
        for (int k = 0; k < 12; ++k) t[k] = mk(r[2 * k], r[2 * k + 1]);
        return;
    }
    const int n = path - 1;  // direction index 2 mu + back
    const int mu = n >> 1, back = n & 1;
    int y[4] = {x[0], x[1], x[2], x[3]};
    const int xm = mu == 0 ? x[0] : mu == 1 ? x[1] : mu == 2 ? x[2] : x[3];
    const int Lm = a.g.L[mu];
    const int xn = back ? (xm == 0 ? Lm - 1 : xm - 1) : (xm + 1 == Lm ? 0 : xm + 1);
    if (mu == 0) y[0] = xn; else if (mu == 1) y[1] = xn; else if (mu == 2) y[2] = xn; else y[3] = xn;
    const uint32_t j = (uint32_t)half_index(a.g, y);
    float r[24];
    load_field<float, 24>(xc + (1 - p) * hv, j, r);
    C<float> psi[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) psi[k] = mk(r[2 * k], r[2 * k + 1]);
    const float4 *lb = site_ptr(a.links[p] + (size_t)n * 3 * a.g.vhp, i, 3);
    float u12[12];
#pragma unroll
    for (int k = 0; k < 3; ++k) Lk<float>::unpack(lb[k * kSB], u12 + 4 * k);
    C<float> u[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) u[k] = mk(u12[2 * k], u12[2 * k + 1]);
    float si, co;
    sc(a.omega[p][(size_t)n * a.g.vhp + i], si, co);
    if (back) {
        link_adj_mul(u, co, si, psi, t);
        link_adj_mul(u, co, si, psi + 6, t + 6);
    } else {
        link_mul(u, co, si, psi, t);
        link_mul(u, co, si, psi + 6, t + 6);
    }
}

// y_c = sum_{c', p} W[p][c][c'] T_p x_{c'}; W BF16 complex pairs [9][nout][nin][4][4]
template <int NOUT>
__global__ __launch_bounds__(256) void k_ptc_layer(PtcGeom a, int nin, const float4 *__restrict__ xin,
                                                   const uint32_t *__restrict__ W, float4 *__restrict__ yout) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= 2 * a.g.vh) return;
    const int p = s >= a.g.vh;
    const uint32_t i = (uint32_t)(s - p * a.g.vh);
    int x[4];
    site_coords(a.g, (int)i, p, x);
    C<float> acc[NOUT][12];
#pragma unroll
    for (int c = 0; c < NOUT; ++c)
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[c][k] = mk(0.f, 0.f);
    const size_t chan4 = a.chan / 4;
#pragma nounroll
    for (int cp = 0; cp < nin; ++cp) {
#pragma nounroll
        for (int path = 0; path < kPaths; ++path) {
            C<float> t[12];
            transport_site(a, xin + cp * chan4, p, i, x, path, t);
#pragma unroll
            for (int c = 0; c < NOUT; ++c) {
                const uint32_t *w = W + ((size_t)(path * NOUT + c) * nin + cp) * 16;
#pragma unroll
                for (int ss = 0; ss < 4; ++ss)
#pragma unroll
                    for (int tt = 0; tt < 4; ++tt) {
                        float wr, wi;
                        bf2(w[ss * 4 + tt], wr, wi);
                        const C<float> wc = mk(wr, wi);
#pragma unroll
                        for (int col = 0; col < 3; ++col) madd(acc[c][3 * ss + col], wc, t[3 * tt + col]);
                    }
            }
        }
    }
    const size_t hv = (size_t)6 * a.g.vhp;
#pragma unroll
    for (int c = 0; c < NOUT; ++c) {
        float r[24];
#pragma unroll
        for (int k = 0; k < 12; ++k) { r[2 * k] = acc[c][k].r; r[2 * k + 1] = acc[c][k].i; }
        store_field<float, 24>(yout + c * chan4 + p * hv, i, r);
    }
}

// Partial weight gradient of one 64-site tile: part[tile][path][c][c'][s][t] (complex float)
template <int NOUT>
__global__ __launch_bounds__(kTile) void k_ptc_wgrad(PtcGeom a, int nin, const float4 *__restrict__ xin,
                                                     const float4 *__restrict__ g, float2 *__restrict__ part) {
    __shared__ C<float> gs[NOUT][kTile][12];
    __shared__ C<float> ts[kTile][12];
    const int s = blockIdx.x * kTile + threadIdx.x;
    const bool on = s < 2 * a.g.vh;
    const int p = on && s >= a.g.vh;
    const uint32_t i = on ? (uint32_t)(s - p * a.g.vh) : 0u;
    int x[4] = {0, 0, 0, 0};
    if (on) site_coords(a.g, (int)i, p, x);
    const size_t chan4 = a.chan / 4, hv = (size_t)6 * a.g.vhp;
#pragma unroll
    for (int c = 0; c < NOUT; ++c) {
        float r[24];
        if (on) load_field<float, 24>(g + c * chan4 + p * hv, i, r);
#pragma unroll
        for (int k = 0; k < 12; ++k) gs[c][threadIdx.x][k] = on ? mk(r[2 * k], r[2 * k + 1]) : mk(0.f, 0.f);
    }
    const int nout_st = NOUT * 16;  // outputs (c, s, t) of one (path, c') pair
#pragma nounroll
    for (int cp = 0; cp < nin; ++cp) {
#pragma nounroll
        for (int path = 0; path < kPaths; ++path) {
            C<float> t[12];
            if (on) transport_site(a, xin + cp * chan4, p, i, x, path, t);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 12; ++k) ts[threadIdx.x][k] = on ? t[k] : mk(0.f, 0.f);
            __syncthreads();
            for (int o = threadIdx.x; o < nout_st; o += kTile) {
                const int c = o >> 4, ss = (o >> 2) & 3, tt = o & 3;
                C<float> acc = mk(0.f, 0.f);
                for (int xs = 0; xs < kTile; ++xs)
#pragma unroll
                    for (int col = 0; col < 3; ++col) {
                        // g_c[s, col] conj(t[t, col])
                        const C<float> gv = gs[c][xs][3 * ss + col], tv = ts[xs][3 * tt + col];
                        acc.r += gv.r * tv.r + gv.i * tv.i;
                        acc.i += gv.i * tv.r - gv.r * tv.i;
                    }
                part[(((size_t)blockIdx.x * kPaths + path) * NOUT * nin + (size_t)c * nin + cp) * 16 + ss * 4 + tt] =
                    make_float2(acc.r, acc.i);
            }
        }
    }
}

// out[k] += sum_b part[b][k] (b ascending), k < n complex entries
__global__ void k_ptc_reduce(int nblk, int n, const float2 *__restrict__ part, float2 *__restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double re = 0.0, im = 0.0;
    for (int b = 0; b < nblk; ++b) {
        const float2 v = part[(size_t)b * n + k];
        re += v.x;
        im += v.y;
    }
    out[k].x += (float)re;
    out[k].y += (float)im;
}

// Adam on n real parameters (interleaved re, im); writes the BF16 working copy
__global__ void k_adam(int n, float *__restrict__ w, const float *__restrict__ grad_conj, float *__restrict__ m,
                       float *__restrict__ v, uint16_t *__restrict__ wbf, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float g = 2.0f * grad_conj[k];  // dL/d(Re W) = 2 Re dL/dW*, dL/d(Im W) = 2 Im dL/dW*
    const float mk_ = b1 * m[k] + (1.0f - b1) * g;
    const float vk = b2 * v[k] + (1.0f - b2) * g * g;
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

template <int NOUT>
void launch_layer(const PtcGeom &a, int nin, const void *x, const void *W, void *y, hipStream_t s) {
    k_ptc_layer<NOUT><<<(2 * a.g.vh + 255) / 256, 256, 0, s>>>(a, nin, (const float4 *)x, (const uint32_t *)W,
                                                             (float4 *)y);
}
void layer_dispatch(const PtcGeom &a, int nin, int nout, const void *x, const void *W, void *y, hipStream_t s) {
    switch (nout) {
        case 1: launch_layer<1>(a, nin, x, W, y, s); break;
        case 2: launch_layer<2>(a, nin, x, W, y, s); break;
        case 4: launch_layer<4>(a, nin, x, W, y, s); break;
        case 8: launch_layer<8>(a, nin, x, W, y, s); break;
        default: throw Error(DIRAC_EUNSUPPORTED, "PTC output channels must be 1, 2, 4 or 8");
    }
    HIP_CHECK(hipGetLastError());
}
template <int NOUT>
void launch_wgrad(const PtcGeom &a, int nin, const void *x, const void *g, void *part, hipStream_t s) {
    k_ptc_wgrad<NOUT><<<(2 * a.g.vh + kTile - 1) / kTile, kTile, 0, s>>>(a, nin, (const float4 *)x,
                                                                       (const float4 *)g, (float2 *)part);
}
void wgrad_dispatch(const PtcGeom &a, int nin, int nout, const void *x, const void *g, void *part, hipStream_t s) {
    switch (nout) {
        case 1: launch_wgrad<1>(a, nin, x, g, part, s); break;
        case 2: launch_wgrad<2>(a, nin, x, g, part, s); break;
        case 4: launch_wgrad<4>(a, nin, x, g, part, s); break;
        case 8: launch_wgrad<8>(a, nin, x, g, part, s); break;
        default: throw Error(DIRAC_EUNSUPPORTED, "PTC output channels must be 1, 2, 4 or 8");
    }
    HIP_CHECK(hipGetLastError());
}

PtcGeom geom_of(dirac_ctx *c, hipStream_t s) {
    ensure_prec(c, DIRAC_F32, s);
    PtcGeom a;
    a.g = c->g;
    for (int p = 0; p < 2; ++p) {
        a.links[p] = (const float4 *)c->f[DIRAC_F32].links[p].p;
        a.omega[p] = (const float *)c->f[DIRAC_F32].omega[p].p;
    }
    a.chan = (size_t)48 * c->g.vhp;
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

void ptc_refresh_bf16(dirac_ptc *n, hipStream_t s) {
    const int nr = (int)(2 * n->total);
    k_to_bf16<<<(nr + 255) / 256, 256, 0, s>>>(nr, (const float *)n->w.p, (uint16_t *)n->wbf.p);
    HIP_CHECK(hipGetLastError());
}

void ptc_ensure_acts(dirac_ctx *c, dirac_ptc *n) {
    const size_t chanb = (size_t)48 * c->g.vhp * sizeof(float);
    size_t need = 0;
    for (int l = 0; l <= n->nlayers; ++l) need += (size_t)n->ch[l] * chanb;
    n->acts.alloc(need);
    int maxc = 0;
    for (int l = 0; l <= n->nlayers; ++l) maxc = std::max(maxc, n->ch[l]);
    n->gbuf.alloc(2 * (size_t)maxc * chanb);
    const size_t ntile = (2 * (size_t)c->vh + kTile - 1) / kTile;
    size_t maxw = 0;
    for (int l = 0; l < n->nlayers; ++l) maxw = std::max(maxw, ptc_nweights(n, l));
    n->part.alloc(ntile * maxw * 8);
}

float *ptc_act(dirac_ctx *c, dirac_ptc *n, int l) {
    const size_t chan = (size_t)48 * c->g.vhp;
    size_t off = 0;
    for (int k = 0; k < l; ++k) off += (size_t)n->ch[k] * chan;
    return (float *)n->acts.p + off;
}

// forward: acts[0] must hold the input; leaves every layer's output in acts[l + 1]
void ptc_forward_acts(dirac_ctx *c, dirac_ptc *n, hipStream_t s) {
    PtcGeom a = geom_of(c, s);
    for (int l = 0; l < n->nlayers; ++l)
        layer_dispatch(a, n->ch[l], n->ch[l + 1], ptc_act(c, n, l), (const uint32_t *)n->wbf.p + n->off[l],
                       ptc_act(c, n, l + 1), s);
}

// backward from g (dL/dy*, FP32 NATIVE full, 1 channel) at the output: accumulates dL/dW* into
// n->grad and, when gin is given, writes dL/dx* of the input.
void ptc_backward_acts(dirac_ctx *c, dirac_ptc *n, const void *g_out, void *gin, hipStream_t s) {
    PtcGeom a = geom_of(c, s);
    const size_t chanb = (size_t)48 * c->g.vhp * sizeof(float);
    int maxc = 0;
    for (int l = 0; l <= n->nlayers; ++l) maxc = std::max(maxc, n->ch[l]);
    char *gA = (char *)n->gbuf.p, *gB = gA + (size_t)maxc * chanb;
    HIP_CHECK(hipMemcpyAsync(gA, g_out, (size_t)n->ch[n->nlayers] * chanb, hipMemcpyDeviceToDevice, s));
    const int ntile = (int)((2 * c->vh + kTile - 1) / kTile);
    for (int l = n->nlayers - 1; l >= 0; --l) {
        const int nin = n->ch[l], nout = n->ch[l + 1];
        const int nw = (int)ptc_nweights(n, l);
        wgrad_dispatch(a, nin, nout, ptc_act(c, n, l), gA, n->part.p, s);
        k_ptc_reduce<<<(nw + 255) / 256, 256, 0, s>>>(ntile, nw, (const float2 *)n->part.p,
                                                      (float2 *)n->grad.p + n->off[l]);
        HIP_CHECK(hipGetLastError());
        if (l == 0 && !gin) break;
        k_adjoint_weights<<<(nw + 255) / 256, 256, 0, s>>>(nout, nin, (const uint32_t *)n->wbf.p + n->off[l],
                                                           (uint32_t *)n->wt.p + n->off[l]);
        HIP_CHECK(hipGetLastError());
        void *dst = l == 0 ? gin : (void *)gB;
        layer_dispatch(a, nout, nin, gA, (const uint32_t *)n->wt.p + n->off[l], dst, s);
        std::swap(gA, gB);
    }
}

void ptc_adam(dirac_ptc *n, double lr, hipStream_t s) {
    n->step += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - std::pow(b1, (float)n->step), c2 = 1.0f - std::pow(b2, (float)n->step);
    const int nr = (int)(2 * n->total);
    k_adam<<<(nr + 255) / 256, 256, 0, s>>>(nr, (float *)n->w.p, (const float *)n->grad.p, (float *)n->m.p,
                                           (float *)n->v.p, (uint16_t *)n->wbf.p, (float)lr, b1, b2, eps, c1, c2);
    HIP_CHECK(hipGetLastError());
}

}  // namespace dl
