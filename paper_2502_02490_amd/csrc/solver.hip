// Krylov solvers on the device (host-driven loops; all vector work in blas.hip kernels):
//   CGLS  - conjugate gradients on D^dag D for the full operator (least-squares CG, the
//           residual s = b - D x of the original system is tracked and re-checked);
//   GCR(m) on the even-odd Schur system, FP64 (Eisenstat, Elman and Schultz 1983), classical
//           Gram-Schmidt against the stored q_j, x updated by back-substitution at the end of
//           each cycle and the true residual recomputed at every restart;
//   MIXED - defect correction (iterative refinement): the FP64 residual of the Schur system is
//           scaled to unit RMS, rounded to FP32 / FP16 / BF16, solved there by GCR(m) to a
//           relative tolerance, and the correction added to the FP64 iterate; the residual is
//           recomputed with the FP64 operator after each step.  A step that reduces the residual
//           by less than 2x raises the inner precision (16-bit -> FP32 -> plain FP64 GCR).
// Inner products inside GCR are normalised by the vector length (mean instead of sum), so that
// unit-norm Krylov vectors have O(1) components in every storage precision.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <functional>
#include <vector>

#include "blas.h"
#include "ptc.h"

namespace dl {

namespace {

// device scalar slots (doubles) inside Blas::scal
constexpr int S_RED = 0, S_SC = 8, S_MISC = 16, S_GAM = 64, S_ALP = 192, S_C = 320, S_BETA = 512;
constexpr int kMaxRestart = 64;

struct GcrOut {
    int iters = 0, restarts = 0;
    bool converged = false, nonfinite = false, stagnated = false;
    double rnorm = 0.0;  // normalised norm of the last true residual
};

// p = M(r) for flexible GCR; vectors in the solve precision and shape
using Precond = std::function<void(void *p, const void *r)>;

double *sc_ptr(SolverWork &w, int slot) { return (double *)w.blas.scal.p + slot; }

// Device-side iteration control of one GCR cycle without a preconditioner: ctl[0] = 1 while the
// system is active, ctl[1] = iterations done in the cycle, ctl[2] = 1 after a non-finite residual.
// After each iteration k_gcr_poll compares the updated residual norm with the target and clears
// ctl[0]; every kernel of a later iteration of the cycle takes ctl as its active mask and does
// nothing, so the host only reads ctl every kPoll iterations and at the end of the cycle.
constexpr int kPoll = 4;

__global__ void k_gcr_ctl_start(int *ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl[0] = 1;
        ctl[1] = 0;
        ctl[2] = 0;
    }
}

__global__ void k_gcr_poll(const double *rn2p, double target, int *ctl) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || !ctl[0]) return;
    ++ctl[1];
    const double rn2 = *rn2p;
    if (!isfinite(rn2)) {
        ctl[2] = 1;
        ctl[0] = 0;
    } else if (sqrt(rn2) <= target) {
        ctl[0] = 0;
    }
}

double read_scalar(SolverWork &w, int slot, hipStream_t s) {
    double h = 0.0;
    HIP_CHECK(hipMemcpyAsync(&h, sc_ptr(w, slot), sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    ++w.syncs;
    return h;
}

}  // namespace

// Solver buffers; they only grow, so a later call with a wider precision or a longer
// restart reallocates (contents are not kept across calls).
void ensure_blas(dirac_ctx *c) {
    if (!c->work) {
        c->work = new SolverWork();
        c->work->blas.c = c;
    }
    c->work->blas.reserve(c->V, kMaxRestart);
}

void ensure_work(dirac_ctx *c, int m, dirac_prec inner, int nh) {
    if (!c->work) {
        c->work = new SolverWork();
        c->work->blas.c = c;
    }
    SolverWork &w = *c->work;
    w.blas.reserve(c->V, kMaxRestart);
    const size_t half64 = (size_t)24 * 8 * c->g.vhp;
    for (auto &b : w.h64) b.alloc(half64);
    for (auto &b : w.f64) b.alloc(2 * half64);
    const size_t hb = (size_t)nh * 24 * real_size(inner) * c->g.vhp;
    w.P.alloc(hb * (m + 1));
    w.Q.alloc(hb * m);
    w.r.alloc(hb);
    w.e.alloc(hb);
    w.b.alloc(hb);
    w.m = m;
    w.pr = inner;
    w.ctl.alloc(4 * sizeof(int));
}

namespace {

// GCR(m) in precision pr on D-hat (half vectors) or, when `full`, on D (full vectors): x solves
// A x = b to |b - A x| <= target (normalised norm); x holds the initial guess when x0.  With a
// preconditioner M the directions are p_k = M(r_k) (flexible GCR).  When min_red > 0 a cycle
// that reduces the residual by less than that factor ends the solve (stagnated).
GcrOut gcr(dirac_ctx *c, SolverWork &w, dirac_prec pr, void *x, const void *b, bool x0, double target, int m,
           int max_iter, hipStream_t s, bool full = false, const Precond *M = nullptr, double min_red = 0.0) {
    Blas &B = w.blas;
    const double scale = 1.0 / (24.0 * (double)c->vh);
    const int nh = full ? 2 : 1;
    const size_t hb = (size_t)nh * 24 * real_size(pr) * c->g.vhp;
    auto apply = [&](void *out, const void *in) {
        if (full) full_apply(c, out, in, 0, pr, s);
        else schur_apply(c, out, in, 0, pr, s);
    };
    char *P = (char *)w.P.p, *Q = (char *)w.Q.p;
    void *r = w.r.p;
    GcrOut out;
    if (x0) {
        apply(Q, x);
        B.lincomb(pr, pr, pr, nh, r, nullptr, 1.0, b, -1.0, Q, sc_ptr(w, S_RED + 4), scale, s);
    } else {
        B.lincomb(pr, pr, pr, nh, x, nullptr, 0.0, b, 0.0, nullptr, nullptr, 1.0, s);
        B.lincomb(pr, pr, pr, nh, r, nullptr, 1.0, b, 0.0, nullptr, sc_ptr(w, S_RED + 4), scale, s);
    }
    double rn2 = read_scalar(w, S_RED + 4, s);
    if (read_scalar(w, S_RED + 5, s) != 0.0 || !std::isfinite(rn2)) {
        out.nonfinite = true;
        return out;
    }
    out.rnorm = std::sqrt(rn2);
    if (out.rnorm <= target) {
        out.converged = true;
        return out;
    }
    std::vector<double> gam(m), alp(2 * m), beta(2 * m * m), cc(2 * m);
    while (out.iters < max_iter) {
        const double cycle_start = out.rnorm;
        if (M) (*M)(P, r);
        else B.lincomb(pr, pr, pr, nh, P, nullptr, 1.0, r, 0.0, nullptr, nullptr, 1.0, s);
        int n = 0;
        if (!M && !full) {
            // iterations decided on the device: the host queues up to kPoll iterations ahead
            int *ctl = (int *)w.ctl.p;
            const BatchSpec bs{1, ctl, 0};
            k_gcr_ctl_start<<<1, 64, 0, s>>>(ctl);
            const int kmax = std::min(m, max_iter - out.iters);
            int h[3] = {1, 0, 0};
            for (int k = 0; k < kmax; ++k) {
                char *qk = Q + k * hb;
                schur_apply(c, qk, P + k * hb, 0, pr, s, 1, ctl);
                double *bcol = sc_ptr(w, S_BETA + 2 * kMaxRestart * k);
                if (k > 0) B.mdot(pr, nh, Q, k, qk, bcol, scale, s, bs);
                B.maxpy_dot(pr, nh, Q, k, bcol, qk, r, sc_ptr(w, S_RED), scale, s, bs);
                B.gcr_scalars(sc_ptr(w, S_RED), sc_ptr(w, S_SC), sc_ptr(w, S_GAM), sc_ptr(w, S_ALP), k, s, bs);
                B.gcr_update(pr, nh, sc_ptr(w, S_SC), qk, r, P + (k + 1) * hb, sc_ptr(w, S_RED + 4), scale, s, bs);
                k_gcr_poll<<<1, 64, 0, s>>>(sc_ptr(w, S_RED + 4), target, ctl);
                HIP_CHECK(hipGetLastError());
                if ((k + 1) % kPoll == 0 || k + 1 == kmax) {
                    HIP_CHECK(hipMemcpyAsync(h, ctl, sizeof h, hipMemcpyDeviceToHost, s));
                    HIP_CHECK(hipStreamSynchronize(s));
                    ++w.syncs;
                    if (!h[0]) break;
                }
            }
            n = h[1];
            out.iters += n;
            if (h[2]) {
                out.nonfinite = true;
                return out;
            }
        } else {
            for (int k = 0; k < m; ++k) {
                char *qk = Q + k * hb;
                apply(qk, P + k * hb);
                double *bcol = sc_ptr(w, S_BETA + 2 * kMaxRestart * k);
                if (k > 0) B.mdot(pr, nh, Q, k, qk, bcol, scale, s);
                B.maxpy_dot(pr, nh, Q, k, bcol, qk, r, sc_ptr(w, S_RED), scale, s);
                B.gcr_scalars(sc_ptr(w, S_RED), sc_ptr(w, S_SC), sc_ptr(w, S_GAM), sc_ptr(w, S_ALP), k, s);
                // the next direction is r itself (copied by the update) or M(r)
                B.gcr_update(pr, nh, sc_ptr(w, S_SC), qk, r, M ? nullptr : P + (k + 1) * hb, sc_ptr(w, S_RED + 4),
                             scale, s);
                rn2 = read_scalar(w, S_RED + 4, s);
                ++out.iters;
                n = k + 1;
                if (!std::isfinite(rn2)) {
                    out.nonfinite = true;
                    return out;
                }
                if (std::sqrt(rn2) <= target || out.iters >= max_iter || k + 1 == m) break;
                if (M) (*M)(P + (k + 1) * hb, r);
            }
        }
        // back-substitution: alpha_j = c_j gamma_j + sum_{k > j} c_k beta_jk
        HIP_CHECK(hipMemcpyAsync(gam.data(), sc_ptr(w, S_GAM), n * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipMemcpyAsync(alp.data(), sc_ptr(w, S_ALP), 2 * n * sizeof(double), hipMemcpyDeviceToHost, s));
        for (int k = 1; k < n; ++k)
            HIP_CHECK(hipMemcpyAsync(beta.data() + 2 * m * k, sc_ptr(w, S_BETA + 2 * kMaxRestart * k),
                                     2 * k * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        ++w.syncs;
        for (int j = n - 1; j >= 0; --j) {
            std::complex<double> acc(alp[2 * j], alp[2 * j + 1]);
            for (int k = j + 1; k < n; ++k)
                acc -= std::complex<double>(beta[2 * m * k + 2 * j], beta[2 * m * k + 2 * j + 1]) *
                       std::complex<double>(cc[2 * k], cc[2 * k + 1]);
            acc /= gam[j];
            cc[2 * j] = acc.real();
            cc[2 * j + 1] = acc.imag();
        }
        HIP_CHECK(hipMemcpyAsync(sc_ptr(w, S_C), cc.data(), 2 * n * sizeof(double), hipMemcpyHostToDevice, s));
        B.axpy_multi(pr, pr, nh, x, P, n, sc_ptr(w, S_C), 1.0, s);
        // true residual of the updated iterate
        apply(Q, x);
        B.lincomb(pr, pr, pr, nh, r, nullptr, 1.0, b, -1.0, Q, sc_ptr(w, S_RED + 4), scale, s);
        rn2 = read_scalar(w, S_RED + 4, s);
        if (!std::isfinite(rn2) || read_scalar(w, S_RED + 5, s) != 0.0) {
            out.nonfinite = true;
            return out;
        }
        out.rnorm = std::sqrt(rn2);
        if (out.rnorm <= target) {
            out.converged = true;
            break;
        }
        if (min_red > 0.0 && !(out.rnorm * min_red <= cycle_start)) {
            out.stagnated = true;
            break;
        }
        if (out.iters < max_iter) ++out.restarts;
    }
    return out;
}

}  // namespace

void check_solver_params(const dirac_solver_params *p) {
    require(p != nullptr, "solver params are NULL");
    require(p->method >= DIRAC_SOLVER_CGLS && p->method <= DIRAC_SOLVER_FGCR_SAP, "unknown solver method");
    require(p->method != DIRAC_SOLVER_FGCR_SAP ||
                (p->sap_ncy >= 0 && p->sap_ncy <= 64 && p->sap_nmr >= 0 && p->sap_nmr <= 64),
            "sap_ncy and sap_nmr must be 0 (default) .. 64");
    require((p->method != DIRAC_SOLVER_FGCR_PTC && p->method != DIRAC_SOLVER_FGCR_PTC_EO) || p->ptc != nullptr,
            "FGCR_PTC needs a network (ptc)");
    require(std::isfinite(p->tol) && p->tol > 0.0 && p->tol < 1.0, "tol must be in (0, 1)");
    require(p->max_iter > 0, "max_iter must be positive");
    if (p->method != DIRAC_SOLVER_CGLS) require(p->restart >= 1 && p->restart <= kMaxRestart, "restart must be 1..64");
    if (p->method == DIRAC_SOLVER_MIXED_GCR)
        require(p->inner_prec == DIRAC_F32 || p->inner_prec == DIRAC_F16 || p->inner_prec == DIRAC_BF16,
                "inner_prec must be F32, F16 or BF16");
    else if (p->precision != DIRAC_F64)
        throw Error(DIRAC_EUNSUPPORTED, "CGLS and GCR run in F64; use MIXED_GCR for lower-precision inner solves");
}

namespace {

double default_inner_tol(dirac_prec pr) { return pr == DIRAC_F32 ? 1e-5 : pr == DIRAC_F16 ? 1e-3 : 1e-2; }

}  // namespace

void *solver_full64(dirac_ctx *c, int k) { return c->work->f64[k].p; }

void free_solver_work(dirac_ctx *c) {
    if (!c->work) return;
    SolverWork &w = *c->work;
    w.blas.part.release();
    w.blas.scal.release();
    w.P.release(); w.Q.release(); w.r.release(); w.e.release(); w.b.release();
    for (auto &b : w.h64) b.release();
    for (auto &b : w.f64) b.release();
    delete c->work;
    c->work = nullptr;
}

// Solve D x = b on NATIVE FP64 full vectors (b, x in w.f64[0], w.f64[1]): even-odd GCR,
// defect correction, or flexible GCR on the full D with a PTC preconditioner that falls back to
// even-odd GCR from its current iterate.
dirac_status solve_native(dirac_ctx *c, const dirac_solver_params *p, bool x0, dirac_solve_info *info,
                          hipStream_t s) {
    ensure_prec(c, DIRAC_F64, s);
    const dirac_prec inner = p->method == DIRAC_SOLVER_MIXED_GCR ? (dirac_prec)p->inner_prec : DIRAC_F64;
    if (inner != DIRAC_F64) ensure_prec(c, inner, s);
    SolverWork &w = *c->work;
    Blas &B = w.blas;
    const double scale = 1.0 / (24.0 * (double)c->vh);
    const size_t half64 = (size_t)24 * 8 * c->g.vhp;
    char *bf = (char *)w.f64[0].p, *xf = (char *)w.f64[1].p, *rf = (char *)w.f64[2].p;
    char *be = bf, *bo = bf + half64, *xe = xf, *xo = xf + half64;
    void *eta = w.h64[0].p, *r64 = w.h64[2].p, *t64 = w.h64[3].p;
    require(c->f[DIRAC_F64].inv_ready[1], "odd-site clover inverse not available (singular block?)");

    // |b|^2 (normalised by the half-vector length, like every norm below)
    B.mdot(DIRAC_F64, 2, bf, 1, bf, sc_ptr(w, S_MISC), scale, s);
    const double bn = std::sqrt(read_scalar(w, S_MISC, s));
    require(std::isfinite(bn), "right-hand side holds NaN or Inf", DIRAC_ENONFINITE);
    if (bn == 0.0) {
        B.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 2, xf, nullptr, 0.0, bf, 0.0, nullptr, nullptr, 1.0, s);
        info->true_rel_res = 0.0;
        return DIRAC_OK;
    }
    const double target = p->tol * bn;
    dirac_status st = DIRAC_OK;
    int iters = 0;
    bool done = false;

    if (p->method == DIRAC_SOLVER_FGCR_SAP) {
        require(sap_supported(c), "FGCR_SAP needs every lattice extent to be a multiple of 8");
        ensure_work(c, p->restart, DIRAC_F64, 2);
        const size_t b32 = (size_t)48 * c->g.vhp * sizeof(float);
        c->sap_in.alloc(b32);
        c->sap_out.alloc(b32);
        const int ncy = p->sap_ncy > 0 ? p->sap_ncy : 4, nmr = p->sap_nmr > 0 ? p->sap_nmr : 4;
        // p = M_SAP r: FP64 -> FP32 -> Schwarz cycles -> FP64
        const Precond M = [&](void *pv, const void *rv) {
            B.lincomb(DIRAC_F32, DIRAC_F64, DIRAC_F64, 2, c->sap_in.p, nullptr, 1.0, rv, 0.0, nullptr, nullptr, 1.0, s);
            sap_apply(c, c->sap_out.p, c->sap_in.p, ncy, nmr, s);
            B.lincomb(DIRAC_F64, DIRAC_F32, DIRAC_F64, 2, pv, nullptr, 1.0, c->sap_out.p, 0.0, nullptr, nullptr, 1.0, s);
        };
        GcrOut g = gcr(c, w, DIRAC_F64, xf, bf, x0, target, p->restart, p->max_iter, s, true, &M, 2.0);
        iters = g.iters;
        info->restarts = g.restarts;
        if (g.converged) {
            done = true;
        } else if (iters >= p->max_iter) {
            st = DIRAC_ENOCONV;
            done = true;
        } else {
            info->fell_back = 1;
            x0 = !g.nonfinite;
        }
    }

    if (p->method == DIRAC_SOLVER_FGCR_PTC) {
        dirac_ptc *net = const_cast<dirac_ptc *>(p->ptc);
        require(net->ch[0] == 1 && net->ch[net->nlayers] == 1, "the PTC network must map 1 channel to 1 channel");
        ptc_ensure_acts(c, net);
        ensure_work(c, p->restart, DIRAC_F64, 2);
        float *a_in = ptc_act(c, net, 0), *a_out = ptc_act(c, net, net->nlayers);
        // p = N(r): FP64 -> FP32 activations -> network -> FP64 (the network is linear: no scaling needed)
        const Precond M = [&](void *pv, const void *rv) {
            B.lincomb(DIRAC_F32, DIRAC_F64, DIRAC_F64, 2, a_in, nullptr, 1.0, rv, 0.0, nullptr, nullptr, 1.0, s);
            ptc_forward_acts(c, net, s, false);
            B.lincomb(DIRAC_F64, DIRAC_F32, DIRAC_F64, 2, pv, nullptr, 1.0, a_out, 0.0, nullptr, nullptr, 1.0, s);
        };
        GcrOut g = gcr(c, w, DIRAC_F64, xf, bf, x0, target, p->restart, p->max_iter, s, true, &M, 2.0);
        iters = g.iters;
        info->restarts = g.restarts;
        if (g.converged) {
            done = true;
        } else if (iters >= p->max_iter) {
            st = DIRAC_ENOCONV;
            done = true;
        } else {
            // a cycle gained less than 2x (or met a non-finite value): plain even-odd GCR from here
            info->fell_back = 1;
            x0 = !g.nonfinite;
        }
    }

    if (!done) {
        // eta-hat_e = b_e - D_eo A_oo^-1 b_o
        clover_apply(c, t64, bo, 1, 1, DIRAC_F64, s);
        hop_apply(c, r64, t64, nullptr, 0, HOP_PLAIN, -0.5, 0, DIRAC_F64, s);
        B.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 1, eta, nullptr, 1.0, be, -1.0, r64, nullptr, 1.0, s);
        bool plain = true;
        if (p->method == DIRAC_SOLVER_FGCR_PTC_EO) {
            dirac_ptc *net = const_cast<dirac_ptc *>(p->ptc);
            require(net->ch[0] == 1 && net->ch[net->nlayers] == 1, "the PTC network must map 1 channel to 1 channel");
            ptc_ensure_acts(c, net);
            ensure_work(c, p->restart, DIRAC_F64, 1);
            float *a_in = ptc_act(c, net, 0), *a_out = ptc_act(c, net, net->nlayers);
            const size_t half32 = (size_t)24 * c->g.vhp;  // floats in one parity of a NATIVE F32 vector
            // p_e = [N(r_e, 0)]_e
            const Precond M = [&](void *pv, const void *rv) {
                B.lincomb(DIRAC_F32, DIRAC_F64, DIRAC_F64, 1, a_in, nullptr, 1.0, rv, 0.0, nullptr, nullptr, 1.0, s);
                zero_fill(a_in + half32, half32 * sizeof(float), s);
                ptc_forward_acts(c, net, s, false, true);  // the even half of the output only
                B.lincomb(DIRAC_F64, DIRAC_F32, DIRAC_F64, 1, pv, nullptr, 1.0, a_out, 0.0, nullptr, nullptr, 1.0, s);
            };
            GcrOut g = gcr(c, w, DIRAC_F64, xe, eta, x0, target, p->restart, p->max_iter, s, false, &M, 2.0);
            iters = g.iters;
            info->restarts = g.restarts;
            if (g.converged) {
                plain = false;
            } else if (iters >= p->max_iter) {
                st = DIRAC_ENOCONV;
                plain = false;
            } else {
                info->fell_back = 1;
                x0 = !g.nonfinite;
            }
        }
        ensure_work(c, p->restart, inner, 1);
        if (!plain) {
            // solved by the flexible GCR above
        } else if (p->method == DIRAC_SOLVER_GCR || p->method == DIRAC_SOLVER_FGCR_PTC ||
                   p->method == DIRAC_SOLVER_FGCR_PTC_EO) {
            // the iterate lives directly in the even half of x
            GcrOut g = gcr(c, w, DIRAC_F64, xe, eta, x0, target, p->restart, p->max_iter - iters, s);
            iters += g.iters;
            info->restarts += g.restarts;
            if (g.nonfinite) st = DIRAC_ENONFINITE;
            else if (!g.converged) st = DIRAC_ENOCONV;
        } else {
            // defect correction around an inner GCR in precision `cur`
            dirac_prec cur = inner;
            double dtol = p->inner_tol > 0.0 ? p->inner_tol : default_inner_tol(cur);
            if (!x0)
                B.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 1, xe, nullptr, 0.0, eta, 0.0, nullptr, nullptr, 1.0, s);
            schur_apply(c, t64, xe, 0, DIRAC_F64, s);
            B.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 1, r64, nullptr, 1.0, eta, -1.0, t64, sc_ptr(w, S_MISC + 2),
                      scale, s);
            double rn = std::sqrt(read_scalar(w, S_MISC + 2, s));
            while (rn > target) {
                if (iters >= p->max_iter) { st = DIRAC_ENOCONV; break; }
                if (!std::isfinite(rn)) { st = DIRAC_ENONFINITE; break; }
                if (cur == DIRAC_F64) {  // fallback: plain FP64 GCR from the current iterate
                    info->fell_back = 1;
                    ensure_work(c, p->restart, DIRAC_F64, 1);
                    GcrOut g = gcr(c, w, DIRAC_F64, xe, eta, true, target, p->restart, p->max_iter - iters, s);
                    iters += g.iters;
                    info->restarts += g.restarts;
                    if (g.nonfinite) st = DIRAC_ENONFINITE;
                    else if (!g.converged) st = DIRAC_ENOCONV;
                    break;
                }
                ensure_prec(c, cur, s);
                ensure_work(c, p->restart, cur, 1);
                // r_lo = r64 / rn (unit normalised RMS), inner solve, x_e += rn e_lo
                B.lincomb(cur, DIRAC_F64, DIRAC_F64, 1, w.b.p, nullptr, 1.0 / rn, r64, 0.0, nullptr, nullptr, 1.0, s);
                GcrOut g = gcr(c, w, cur, w.e.p, w.b.p, false, dtol, p->restart, p->max_iter - iters, s);
                iters += g.iters;
                info->restarts += g.restarts;
                ++info->outer;
                if (!g.nonfinite) {
                    B.set(sc_ptr(w, S_C), 1.0, s);
                    B.set(sc_ptr(w, S_C + 1), 0.0, s);
                    B.axpy_multi(DIRAC_F64, cur, 1, xe, w.e.p, 1, sc_ptr(w, S_C), rn, s);
                }
                schur_apply(c, t64, xe, 0, DIRAC_F64, s);
                B.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 1, r64, nullptr, 1.0, eta, -1.0, t64,
                          sc_ptr(w, S_MISC + 2), scale, s);
                const double rn_new = std::sqrt(read_scalar(w, S_MISC + 2, s));
                if (g.nonfinite || !(rn_new < 0.5 * rn)) {
                    cur = cur == DIRAC_F32 ? DIRAC_F64 : DIRAC_F32;  // raise the inner precision
                    dtol = p->inner_tol > 0.0 && cur == DIRAC_F32 ? std::max(p->inner_tol, 1e-5)
                                                                   : default_inner_tol(cur);
                }
                rn = rn_new;
            }
        }
        // x_o = A_oo^-1 (b_o - D_oe x_e)
        hop_apply(c, t64, xe, nullptr, 1, HOP_PLAIN, -0.5, 0, DIRAC_F64, s);
        B.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 1, r64, nullptr, 1.0, bo, -1.0, t64, nullptr, 1.0, s);
        clover_apply(c, xo, r64, 1, 1, DIRAC_F64, s);
    }
    info->iters = iters;
    // a-posteriori check: |b - D x| / |b| in FP64
    full_apply(c, rf, xf, 0, DIRAC_F64, s);
    B.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 2, rf, nullptr, 1.0, bf, -1.0, rf, sc_ptr(w, S_MISC + 4), scale, s);
    info->true_rel_res = std::sqrt(read_scalar(w, S_MISC + 4, s)) / bn;
    if (st == DIRAC_OK && !(info->true_rel_res < p->tol)) st = DIRAC_ENOCONV;
    if (!std::isfinite(info->true_rel_res)) st = DIRAC_ENONFINITE;
    return st;
}

// CGLS on the full operator, FP64 NATIVE full vectors (b = w.f64[0], x = w.f64[1]).
dirac_status solve_cgls(dirac_ctx *c, const dirac_solver_params *p, bool x0, dirac_solve_info *info,
                        hipStream_t s) {
    SolverWork &w = *c->work;
    Blas &B = w.blas;
    const double scale = 1.0 / (24.0 * (double)c->vh);
    char *bf = (char *)w.f64[0].p, *xf = (char *)w.f64[1].p, *sv = (char *)w.f64[2].p;
    // CGLS needs three more full vectors: r, p, w (inside the inner-solver buffers, FP64)
    const size_t full64 = (size_t)48 * 8 * c->g.vhp;
    w.P.alloc(3 * full64);
    char *rv = (char *)w.P.p, *pv = rv + full64, *wv = pv + full64;
    double *rho = sc_ptr(w, S_MISC + 8), *rho_new = sc_ptr(w, S_MISC + 10), *wn = sc_ptr(w, S_MISC + 12);
    B.mdot(DIRAC_F64, 2, bf, 1, bf, sc_ptr(w, S_MISC), scale, s);
    const double bn = std::sqrt(read_scalar(w, S_MISC, s));
    require(std::isfinite(bn), "right-hand side holds NaN or Inf", DIRAC_ENONFINITE);
    if (!x0) B.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 2, xf, nullptr, 0.0, bf, 0.0, nullptr, nullptr, 1.0, s);
    const double target = p->tol * bn;
    dirac_status st = DIRAC_ENOCONV;
    int it = 0;
    while (it < p->max_iter) {
        // s = b - D x; r = D^dag s; p = r; rho = |r|^2
        full_apply(c, wv, xf, 0, DIRAC_F64, s);
        B.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 2, sv, nullptr, 1.0, bf, -1.0, wv, sc_ptr(w, S_MISC + 6), scale, s);
        double sn = std::sqrt(read_scalar(w, S_MISC + 6, s));
        if (!std::isfinite(sn)) { st = DIRAC_ENONFINITE; break; }
        if (sn <= target) { st = DIRAC_OK; break; }
        if (it > 0) ++info->restarts;
        full_apply(c, rv, sv, 1, DIRAC_F64, s);
        B.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 2, pv, nullptr, 1.0, rv, 0.0, nullptr, nullptr, 1.0, s);
        B.mdot(DIRAC_F64, 2, rv, 1, rv, rho, scale, s);
        while (it < p->max_iter) {
            full_apply(c, wv, pv, 0, DIRAC_F64, s);
            B.mdot(DIRAC_F64, 2, wv, 1, wv, wn, scale, s);
            B.cgls_xs(2, rho, wn, xf, pv, sv, wv, sc_ptr(w, S_MISC + 6), s);
            full_apply(c, rv, sv, 1, DIRAC_F64, s);
            B.mdot(DIRAC_F64, 2, rv, 1, rv, rho_new, scale, s);
            B.cgls_p(2, rho_new, rho, pv, rv, s);
            B.copy_scalar(rho_new, rho, s);
            ++it;
            sn = std::sqrt(read_scalar(w, S_MISC + 6, s));
            if (!std::isfinite(sn)) break;
            if (sn <= target) break;
        }
    }
    info->iters = it;
    // a-posteriori check
    full_apply(c, wv, xf, 0, DIRAC_F64, s);
    B.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 2, sv, nullptr, 1.0, bf, -1.0, wv, sc_ptr(w, S_MISC + 6), scale, s);
    info->true_rel_res = std::sqrt(read_scalar(w, S_MISC + 6, s)) / bn;
    if (st == DIRAC_OK && !(info->true_rel_res < p->tol)) st = DIRAC_ENOCONV;
    if (!std::isfinite(info->true_rel_res)) st = DIRAC_ENONFINITE;
    return st;
}

}  // namespace dl

