// Batched solves: many right-hand sides on each of many lattices of uneven size.
//
// Per lattice (one context) all nrhs systems advance together: every kernel of a GCR iteration
// covers all right-hand sides in one launch (the multi-RHS hop assigns consecutive work-groups
// on one XCD to the right-hand sides of one site block, so its links and clover are read from
// HBM once and served from L2 to the other right-hand sides), with per-system scalars and an
// active mask that freezes converged systems.  The launch sequence of iteration k of a cycle is
// captured once into a hipGraph and replayed; the host reads one strided array of residual norms
// per iteration.  Lattices run concurrently: one host thread and one stream per lattice.
// Method: FP64 even-odd GCR, or FP64 defect correction around a batched inner GCR in
// FP32 / FP16 / BF16 (the mixed scheme of solver.hip, per system).
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <thread>
#include <vector>

#include "blas.h"

namespace dl {

struct BWork {
    hipStream_t s = nullptr;
    DevBuf P, Q, r, e, b, act, act2;
    DevBuf h64[4];  // FP64 half vectors x nrhs: eta-hat, x_e, r, tmp
    DevBuf f64[3];  // FP64 full vectors x nrhs: b, x, r
    std::vector<hipGraphExec_t> graphs;
    std::vector<const void *> graph_key;  // (precision, m, nrhs and every buffer the graphs touch)
    ~BWork() {
        for (auto g : graphs)
            if (g) (void)hipGraphExecDestroy(g);
        if (s) (void)hipStreamDestroy(s);
        for (DevBuf *d : {&P, &Q, &r, &e, &b, &act, &act2}) d->release();
        for (auto &d : h64) d.release();
        for (auto &d : f64) d.release();
    }
};

namespace {

constexpr int S_RED = 0, S_SC = 8, S_MISC = 16, S_GAM = 64, S_ALP = 192, S_C = 320, S_BETA = 512;
constexpr int S_ALPHA = kSysScal - 64, S_XS = kSysScal - 62, S_ONE = kSysScal - 60;  // per-system free slots
constexpr int kMaxM = 64;

bool graphs_enabled() {
    const char *e = getenv("DIRAC_GRAPHS");
    return !e || atoi(e) != 0;
}

struct Lat {
    dirac_ctx *c;
    BWork *w;
    int nrhs;
    double *scal() { return (double *)c->work->blas.scal.p; }
    double *sp(int slot) { return scal() + slot; }
    BatchSpec spec(const int *act) const { return BatchSpec{nrhs, act, kSysScal}; }
};

// strided per-system scalars <-> host
void read_sys(Lat &L, int slot, std::vector<double> &h, hipStream_t s) {
    h.resize(L.nrhs);
    HIP_CHECK(hipMemcpy2DAsync(h.data(), sizeof(double), L.sp(slot), kSysScal * sizeof(double), sizeof(double),
                               L.nrhs, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
}
void write_sys(Lat &L, int slot, const std::vector<double> &h, hipStream_t s) {
    HIP_CHECK(hipMemcpy2DAsync(L.sp(slot), kSysScal * sizeof(double), h.data(), sizeof(double), sizeof(double),
                               L.nrhs, hipMemcpyHostToDevice, s));
    HIP_CHECK(hipStreamSynchronize(s));  // h may be a temporary
}
void upload_mask(const std::vector<int> &m, DevBuf &d, hipStream_t s) {
    HIP_CHECK(hipMemcpyAsync(d.p, m.data(), m.size() * sizeof(int), hipMemcpyHostToDevice, s));
    HIP_CHECK(hipStreamSynchronize(s));  // m may change right after
}

struct BOut {
    std::vector<int> iters, restarts;
    std::vector<char> converged;
    bool nonfinite = false;
};

// Batched GCR(m) on D-hat in precision pr for the systems with start[r] = 1: x_r solves
// D-hat x_r = b_r to |b_r - D-hat x_r| <= target[r] (normalised norms); x = 0 initially.
BOut gcr_batched(Lat &L, dirac_prec pr, void *x, const void *b, const std::vector<int> &start,
                 const std::vector<double> &target, int m, int max_iter, bool use_graph) {
    dirac_ctx *c = L.c;
    BWork &w = *L.w;
    Blas &B = c->work->blas;
    hipStream_t s = w.s;
    const int R = L.nrhs;
    const double scale = 1.0 / (24.0 * (double)c->vh);
    const size_t vb = (size_t)24 * real_size(pr) * c->g.vhp;  // bytes of one half vector
    const size_t kb = vb * R;                                   // bytes of one basis slot (all systems)
    char *P = (char *)w.P.p, *Q = (char *)w.Q.p;
    void *r = w.r.p;
    int *act = (int *)w.act.p, *cyc = (int *)w.act2.p;
    BOut out;
    out.iters.assign(R, 0);
    out.restarts.assign(R, 0);
    out.converged.assign(R, 0);
    std::vector<int> a(start), cy(R);
    upload_mask(a, w.act, s);
    B.lincomb(pr, pr, pr, 1, x, nullptr, 0.0, b, 0.0, nullptr, nullptr, 1.0, s, L.spec(act));
    B.lincomb(pr, pr, pr, 1, r, nullptr, 1.0, b, 0.0, nullptr, L.sp(S_RED + 4), scale, s, L.spec(act));
    std::vector<double> rn2, gam((size_t)R * kSysScal);
    read_sys(L, S_RED + 4, rn2, s);
    for (int q = 0; q < R; ++q) {
        if (!a[q]) continue;
        if (!std::isfinite(rn2[q])) { out.nonfinite = true; a[q] = 0; }
        else if (std::sqrt(rn2[q]) <= target[q]) { out.converged[q] = 1; a[q] = 0; }
    }
    // every buffer a captured iteration touches is allocated before capture; the graphs are
    // rebuilt whenever the precision, the cycle length, the batch or any of those buffers changes
    c->f[pr].tmp_half.alloc((size_t)R * 24 * real_size(pr) * c->g.vhp);
    const std::vector<const void *> key = {(const void *)(intptr_t)pr, (const void *)(intptr_t)m,
                                           (const void *)(intptr_t)R, w.P.p, w.Q.p, w.r.p, w.act.p,
                                           B.part.p, B.scal.p, c->f[pr].tmp_half.p};
    if (use_graph && key != w.graph_key) {
        for (auto g : w.graphs)
            if (g) HIP_CHECK(hipGraphExecDestroy(g));
        w.graphs.assign(m, nullptr);
        w.graph_key = key;
    }
    // the launch-shape tuner cannot time candidates inside a capture: one eager operator
    // application (on the residual, into basis slot 0, which iteration 0 overwrites) lets it
    // choose before the graphs are recorded
    if (use_graph && !w.graphs[0]) schur_apply(c, Q, r, 0, pr, s, R, act);
    auto iteration = [&](int k) {
        char *qk = Q + k * kb;
        schur_apply(c, qk, P + k * kb, 0, pr, s, R, act);
        double *bcol = L.sp(S_BETA + 2 * kMaxM * k);
        if (k > 0) B.mdot(pr, 1, Q, k, qk, bcol, scale, s, L.spec(act));
        B.maxpy_dot(pr, 1, Q, k, bcol, qk, r, L.sp(S_RED), scale, s, L.spec(act));
        B.gcr_scalars(L.sp(S_RED), L.sp(S_SC), L.sp(S_GAM), L.sp(S_ALP), k, s, L.spec(act));
        B.gcr_update(pr, 1, L.sp(S_SC), qk, r, P + (k + 1) * kb, L.sp(S_RED + 4), scale, s, L.spec(act));
    };
    auto any = [](const std::vector<int> &v) {
        for (int q : v)
            if (q) return true;
        return false;
    };
    int it = 0;
    while (any(a) && it < max_iter) {
        cy = a;
        upload_mask(cy, w.act2, s);
        upload_mask(a, w.act, s);
        B.lincomb(pr, pr, pr, 1, P, nullptr, 1.0, r, 0.0, nullptr, nullptr, 1.0, s, L.spec(act));
        std::vector<int> n(R, 0);
        int kmax = 0;
        for (int k = 0; k < m; ++k) {
            if (use_graph) {
                if (!w.graphs[k]) {
                    hipGraph_t g;
                    HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                    iteration(k);
                    HIP_CHECK(hipStreamEndCapture(s, &g));
                    HIP_CHECK(hipGraphInstantiate(&w.graphs[k], g, nullptr, nullptr, 0));
                    HIP_CHECK(hipGraphDestroy(g));
                }
                HIP_CHECK(hipGraphLaunch(w.graphs[k], s));
            } else {
                iteration(k);
            }
            read_sys(L, S_RED + 4, rn2, s);
            ++it;
            kmax = k + 1;
            bool changed = false;
            for (int q = 0; q < R; ++q) {
                if (!a[q]) continue;
                n[q] = k + 1;
                ++out.iters[q];
                if (!std::isfinite(rn2[q])) { out.nonfinite = true; a[q] = 0; changed = true; }
                else if (std::sqrt(rn2[q]) <= target[q]) { a[q] = 0; changed = true; }
            }
            if (!any(a) || it >= max_iter) break;
            if (changed) upload_mask(a, w.act, s);
        }
        // back-substitution per system over its own cycle length
        HIP_CHECK(hipMemcpyAsync(gam.data(), L.scal(), gam.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        for (int q = 0; q < R; ++q) {
            double *base = gam.data() + (size_t)q * kSysScal;
            std::vector<std::complex<double>> cc(kmax, 0.0);
            for (int j = n[q] - 1; j >= 0; --j) {
                std::complex<double> acc(base[S_ALP + 2 * j], base[S_ALP + 2 * j + 1]);
                for (int k = j + 1; k < n[q]; ++k)
                    acc -= std::complex<double>(base[S_BETA + 2 * kMaxM * k + 2 * j],
                                                base[S_BETA + 2 * kMaxM * k + 2 * j + 1]) * cc[k];
                cc[j] = acc / base[S_GAM + j];
            }
            for (int j = 0; j < kmax; ++j) {
                base[S_C + 2 * j] = cc[j].real();
                base[S_C + 2 * j + 1] = cc[j].imag();
            }
        }
        HIP_CHECK(hipMemcpy2DAsync(L.sp(S_C), kSysScal * sizeof(double), gam.data() + S_C, kSysScal * sizeof(double),
                                   2 * kmax * sizeof(double), R, hipMemcpyHostToDevice, s));
        B.axpy_multi(pr, pr, 1, x, P, kmax, L.sp(S_C), 1.0, s, L.spec(cyc));
        // true residuals of the systems that took part in the cycle
        schur_apply(c, Q, x, 0, pr, s, R, cyc);
        B.lincomb(pr, pr, pr, 1, r, nullptr, 1.0, b, -1.0, Q, L.sp(S_RED + 4), scale, s, L.spec(cyc));
        read_sys(L, S_RED + 4, rn2, s);
        for (int q = 0; q < R; ++q) {
            if (!cy[q]) continue;
            if (!std::isfinite(rn2[q])) { out.nonfinite = true; a[q] = 0; continue; }
            if (std::sqrt(rn2[q]) <= target[q]) { out.converged[q] = 1; a[q] = 0; }
            else { a[q] = 1; ++out.restarts[q]; }
        }
    }
    return out;
}

void ensure_bwork(dirac_ctx *c, int m, int nrhs, dirac_prec inner) {
    ensure_work(c, 1, DIRAC_F64, 1);
    c->work->blas.reserve(c->V, kMaxM, nrhs);
    if (!c->bwork) c->bwork = new BWork();
    BWork &w = *c->bwork;
    if (!w.s) HIP_CHECK(hipStreamCreateWithFlags(&w.s, hipStreamNonBlocking));
    const size_t hb = (size_t)nrhs * 24 * 8 * c->g.vhp;  // FP64 (the largest) sizing: fallback needs it
    w.P.alloc(hb * (m + 1));
    w.Q.alloc(hb * m);
    w.r.alloc(hb);
    w.e.alloc(hb);
    w.b.alloc(hb);
    w.act.alloc(nrhs * sizeof(int));
    w.act2.alloc(nrhs * sizeof(int));
    for (auto &d : w.h64) d.alloc(hb);
    for (auto &d : w.f64) d.alloc(2 * hb);
    (void)inner;
}

// One lattice: solve D x_r = b_r for nrhs NATIVE FP64 full vectors (in w.f64[0] -> w.f64[1]).
void solve_lattice(dirac_ctx *c, int nrhs, const dirac_solver_params *p, dirac_solve_info *info) {
    BWork &w = *c->bwork;
    Lat L{c, &w, nrhs};
    hipStream_t s = w.s;
    Blas &B = c->work->blas;
    const double scale = 1.0 / (24.0 * (double)c->vh);
    const size_t half64 = (size_t)24 * 8 * c->g.vhp;
    const size_t full64 = 2 * half64;
    char *bf = (char *)w.f64[0].p, *xf = (char *)w.f64[1].p, *rf = (char *)w.f64[2].p;
    void *eta = w.h64[0].p, *xe = w.h64[1].p, *r64 = w.h64[2].p, *t64 = w.h64[3].p;
    const bool graph = graphs_enabled();
    // split the full vectors into even / odd halves (per system) and back through the half buffers
    auto halves = [&](char *full, void *even, void *odd, bool to_halves) {
        for (int q = 0; q < nrhs; ++q) {
            char *f = full + q * full64;
            if (to_halves) {
                if (even) HIP_CHECK(hipMemcpyAsync((char *)even + q * half64, f, half64, hipMemcpyDeviceToDevice, s));
                if (odd) HIP_CHECK(hipMemcpyAsync((char *)odd + q * half64, f + half64, half64, hipMemcpyDeviceToDevice, s));
            } else {
                if (even) HIP_CHECK(hipMemcpyAsync(f, (char *)even + q * half64, half64, hipMemcpyDeviceToDevice, s));
                if (odd) HIP_CHECK(hipMemcpyAsync(f + half64, (char *)odd + q * half64, half64, hipMemcpyDeviceToDevice, s));
            }
        }
    };
    ensure_prec(c, DIRAC_F64, s);
    require(c->f[DIRAC_F64].inv_ready[1], "odd-site clover inverse not available");
    std::vector<int> all(nrhs, 1);
    upload_mask(all, w.act, s);
    // |b_r|
    B.mdot(DIRAC_F64, 2, bf, 1, bf, L.sp(S_MISC), scale, s, L.spec((int *)w.act.p));
    std::vector<double> bn;
    read_sys(L, S_MISC, bn, s);
    std::vector<double> target(nrhs);
    for (int q = 0; q < nrhs; ++q) {
        bn[q] = std::sqrt(bn[q]);
        require(std::isfinite(bn[q]), "right-hand side holds NaN or Inf", DIRAC_ENONFINITE);
        target[q] = p->tol * bn[q];
    }
    // eta-hat_e = b_e - D_eo A_oo^-1 b_o (all systems): even halves into eta, odd into r64
    halves(bf, eta, r64, true);
    clover_apply(c, t64, r64, 1, 1, DIRAC_F64, s, nrhs);
    hop_apply(c, r64, t64, nullptr, 0, HOP_PLAIN, -0.5, 0, DIRAC_F64, s, nrhs);
    B.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 1, eta, nullptr, 1.0, eta, -1.0, r64, nullptr, 1.0, s,
              L.spec((int *)w.act.p));
    std::vector<int> live(nrhs);
    for (int q = 0; q < nrhs; ++q) live[q] = bn[q] > 0.0;
    if (p->method == DIRAC_SOLVER_GCR) {
        BOut o = gcr_batched(L, DIRAC_F64, xe, eta, live, target, p->restart, p->max_iter, graph);
        for (int q = 0; q < nrhs; ++q) {
            info[q].iters = o.iters[q];
            info[q].restarts = o.restarts[q];
        }
    } else {
        // defect correction per system around the batched inner GCR
        dirac_prec cur = (dirac_prec)p->inner_prec;
        ensure_prec(c, cur, s);
        const double dtol = p->inner_tol > 0.0 ? p->inner_tol
                                               : (cur == DIRAC_F32 ? 1e-5 : cur == DIRAC_F16 ? 1e-3 : 1e-2);
        upload_mask(all, w.act, s);
        B.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 1, xe, nullptr, 0.0, eta, 0.0, nullptr, nullptr, 1.0, s,
                  L.spec((int *)w.act.p));
        B.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 1, r64, nullptr, 1.0, eta, 0.0, nullptr, L.sp(S_MISC + 2), scale,
                  s, L.spec((int *)w.act.p));
        std::vector<double> rn;
        read_sys(L, S_MISC + 2, rn, s);
        for (int q = 0; q < nrhs; ++q) rn[q] = std::sqrt(rn[q]);
        std::vector<int> outer(nrhs);
        int used = 0;
        std::vector<double> inv(nrhs), one(nrhs, 1.0), itarget(nrhs, dtol);
        bool fell_back = false;
        while (true) {
            for (int q = 0; q < nrhs; ++q) outer[q] = live[q] && rn[q] > target[q] && std::isfinite(rn[q]);
            bool anyo = false;
            for (int q : outer) anyo = anyo || q;
            if (!anyo || used >= p->max_iter) break;
            if (cur == DIRAC_F64) {
                fell_back = true;
                // plain FP64 batched GCR on the remaining systems from their current iterates:
                // solve the correction D-hat e = r64 and add it
                BOut o = gcr_batched(L, DIRAC_F64, w.e.p, r64, outer, target, p->restart, p->max_iter - used, graph);
                for (int q = 0; q < nrhs; ++q) {
                    info[q].iters += o.iters[q];
                    info[q].restarts += o.restarts[q];
                    if (outer[q]) info[q].fell_back = 1;
                }
                upload_mask(outer, w.act, s);
                write_sys(L, S_ONE, one, s);
                write_sys(L, S_ONE + 1, std::vector<double>(nrhs, 0.0), s);
                B.axpy_multi(DIRAC_F64, DIRAC_F64, 1, xe, w.e.p, 1, L.sp(S_ONE), 1.0, s, L.spec((int *)w.act.p));
                break;
            }
            for (int q = 0; q < nrhs; ++q) inv[q] = outer[q] ? 1.0 / rn[q] : 0.0;
            write_sys(L, S_ALPHA, inv, s);
            upload_mask(outer, w.act, s);
            B.lincomb(cur, DIRAC_F64, DIRAC_F64, 1, w.b.p, nullptr, 1.0, r64, 0.0, nullptr, nullptr, 1.0, s,
                      L.spec((int *)w.act.p), L.sp(S_ALPHA));
            BOut o = gcr_batched(L, cur, w.e.p, w.b.p, outer, itarget, p->restart, p->max_iter - used, graph);
            int mx = 0;
            for (int q = 0; q < nrhs; ++q) {
                info[q].iters += o.iters[q];
                info[q].restarts += o.restarts[q];
                if (outer[q]) ++info[q].outer;
                mx = std::max(mx, o.iters[q]);
            }
            used += mx;
            // x_e += rn_r e_r
            write_sys(L, S_XS, rn, s);
            write_sys(L, S_ONE, one, s);
            write_sys(L, S_ONE + 1, std::vector<double>(nrhs, 0.0), s);
            upload_mask(outer, w.act, s);
            B.axpy_multi(DIRAC_F64, cur, 1, xe, w.e.p, 1, L.sp(S_ONE), 1.0, s, L.spec((int *)w.act.p), L.sp(S_XS));
            schur_apply(c, t64, xe, 0, DIRAC_F64, s, nrhs, (int *)w.act.p);
            B.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 1, r64, nullptr, 1.0, eta, -1.0, t64, L.sp(S_MISC + 2), scale,
                      s, L.spec((int *)w.act.p));
            std::vector<double> rnew;
            read_sys(L, S_MISC + 2, rnew, s);
            bool stalled = o.nonfinite;
            for (int q = 0; q < nrhs; ++q) {
                if (!outer[q]) continue;
                rnew[q] = std::sqrt(rnew[q]);
                if (!(rnew[q] < 0.5 * rn[q])) stalled = true;
                rn[q] = rnew[q];
            }
            if (stalled) cur = cur == DIRAC_F32 ? DIRAC_F64 : DIRAC_F32;  // raise the inner precision
            if (cur != DIRAC_F64) ensure_prec(c, cur, s);
        }
        (void)fell_back;
    }
    // x_o = A_oo^-1 (b_o - D_oe x_e); assemble the full solutions
    halves(bf, nullptr, r64, true);  // r64 <- b_o
    hop_apply(c, t64, xe, nullptr, 1, HOP_PLAIN, -0.5, 0, DIRAC_F64, s, nrhs);
    upload_mask(all, w.act, s);
    B.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 1, r64, nullptr, 1.0, r64, -1.0, t64, nullptr, 1.0, s,
              L.spec((int *)w.act.p));
    clover_apply(c, t64, r64, 1, 1, DIRAC_F64, s, nrhs);
    halves(xf, xe, t64, false);
    // a-posteriori residuals
    for (int q = 0; q < nrhs; ++q) full_apply(c, rf + q * full64, xf + q * full64, 0, DIRAC_F64, s);
    B.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 2, rf, nullptr, 1.0, bf, -1.0, rf, L.sp(S_MISC + 4), scale, s,
              L.spec((int *)w.act.p));
    std::vector<double> tr;
    read_sys(L, S_MISC + 4, tr, s);
    for (int q = 0; q < nrhs; ++q) info[q].true_rel_res = bn[q] > 0.0 ? std::sqrt(tr[q]) / bn[q] : 0.0;
}

}  // namespace

void free_bwork(dirac_ctx *c) {
    if (c->bwork) {
        delete c->bwork;
        c->bwork = nullptr;
    }
}

// Solve all lattices concurrently (one host thread and one stream each).  x[l] / b[l] hold nrhs
// consecutive full-lattice FP64 vectors in `lay`.  Returns the first error met (all threads join).
dirac_status solve_batched(dirac_ctx *const *ctx, int nlat, void *const *x, const void *const *b, int nrhs,
                           dirac_layout lay, const dirac_solver_params *p, dirac_solve_info *info, hipStream_t user,
                           std::string &err) {
    std::vector<dirac_status> st(nlat, DIRAC_OK);
    std::vector<std::string> msg(nlat);
    // work is queued behind what the caller already put on its stream
    hipEvent_t ready;
    HIP_CHECK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    HIP_CHECK(hipEventRecord(ready, user));
    auto run = [&](int l) {
        const auto t0 = std::chrono::steady_clock::now();
        dirac_ctx *c = ctx[l];
        try {
            int dev = 0;
            HIP_CHECK(hipGetDevice(&dev));
            ensure_bwork(c, p->restart, nrhs, (dirac_prec)p->inner_prec);
            BWork &w = *c->bwork;
            HIP_CHECK(hipStreamWaitEvent(w.s, ready, 0));
            const size_t full64 = (size_t)48 * 8 * c->g.vhp;
            const size_t ub = (size_t)c->V * 24 * 8;
            for (int q = 0; q < nrhs; ++q) {
                char *dst = (char *)w.f64[0].p + q * full64;
                if (lay == DIRAC_LAYOUT_NATIVE)
                    HIP_CHECK(hipMemcpyAsync(dst, (const char *)b[l] + q * full64, full64, hipMemcpyDeviceToDevice, w.s));
                else
                    spinor_import(c, dst, (const char *)b[l] + q * ub, 0, DIRAC_F64, lay, w.s);
            }
            dirac_solve_info *inf = info + (size_t)l * nrhs;
            for (int q = 0; q < nrhs; ++q) inf[q] = dirac_solve_info{};
            solve_lattice(c, nrhs, p, inf);
            for (int q = 0; q < nrhs; ++q) {
                char *src = (char *)w.f64[1].p + q * full64;
                if (lay == DIRAC_LAYOUT_NATIVE)
                    HIP_CHECK(hipMemcpyAsync((char *)x[l] + q * full64, src, full64, hipMemcpyDeviceToDevice, w.s));
                else
                    spinor_export(c, (char *)x[l] + q * ub, src, 0, DIRAC_F64, lay, w.s);
            }
            HIP_CHECK(hipStreamSynchronize(w.s));
            const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            for (int q = 0; q < nrhs; ++q) {
                inf[q].seconds = sec;
                if (!std::isfinite(inf[q].true_rel_res)) st[l] = DIRAC_ENONFINITE;
                else if (!(inf[q].true_rel_res < p->tol) && st[l] == DIRAC_OK) st[l] = DIRAC_ENOCONV;
            }
            if (st[l] != DIRAC_OK) msg[l] = "lattice " + std::to_string(l) + ": a system did not reach the tolerance";
        } catch (const Error &e) {
            st[l] = e.status;
            msg[l] = "lattice " + std::to_string(l) + ": " + e.what();
        } catch (const std::exception &e) {
            st[l] = DIRAC_EHIP;
            msg[l] = "lattice " + std::to_string(l) + ": " + e.what();
        }
    };
    std::vector<std::thread> th;
    for (int l = 0; l < nlat; ++l) th.emplace_back(run, l);
    for (auto &t : th) t.join();
    (void)hipEventDestroy(ready);
    for (int l = 0; l < nlat; ++l)
        if (st[l] != DIRAC_OK) {
            err = msg[l];
            return st[l];
        }
    return DIRAC_OK;
}

}  // namespace dl
