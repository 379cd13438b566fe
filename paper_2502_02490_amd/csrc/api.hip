// C ABI entry points (include/dirac.h): argument validation, context lifetime,
// staging between the user layouts and the NATIVE layout, status codes.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "blas.h"
#include "internal.h"
#include "ptc.h"

namespace {

thread_local std::string g_err;

dirac_status fail(dirac_status s, const std::string &m) {
    g_err = m;
    return s;
}

#define API_BEGIN \
    g_err.clear(); \
    try {
#define API_END                                                        \
    }                                                                  \
    catch (const dl::Error &e) {                                       \
        return fail(e.status, e.what());                               \
    }                                                                  \
    catch (const std::bad_alloc &) {                                   \
        return fail(DIRAC_ENOMEM, "host allocation failed");           \
    }                                                                  \
    catch (const std::exception &e) {                                  \
        return fail(DIRAC_EHIP, std::string("internal error: ") + e.what()); \
    }                                                                  \
    catch (...) {                                                      \
        return fail(DIRAC_EHIP, "internal error");                     \
    }                                                                  \
    return DIRAC_OK;

using dl::require;

// The pointer must be device memory with at least `bytes` bytes from `ptr` to the end
// of its allocation (a kernel reading past it would fault the GPU).
void check_dev(const void *ptr, size_t bytes, const char *name) {
    require(ptr != nullptr, std::string(name) + " is NULL");
    hipPointerAttribute_t at;
    hipError_t e = hipPointerGetAttributes(&at, ptr);
    if (e != hipSuccess) (void)hipGetLastError();
    require(e == hipSuccess && (at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged),
            std::string(name) + " is not device memory");
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return;  // range unknown (e.g. imported memory): the type check above still holds
    }
    const size_t off = (size_t)((const char *)ptr - (const char *)base);
    require(off <= size && size - off >= bytes,
            std::string(name) + " is smaller than the " + std::to_string(bytes) + " bytes this call reads or writes");
}

void check_no_alias(const void *a, size_t na, const void *b, size_t nb) {
    const char *x = (const char *)a, *y = (const char *)b;
    require(x + na <= y || y + nb <= x, "output buffer overlaps an input buffer");
}

void check_ctx(const dirac_ctx *c) { require(c != nullptr, "context is NULL"); }

void check_prec(int pr) { require(pr >= DIRAC_F64 && pr <= DIRAC_BF16, "unknown precision"); }

size_t user_bytes(const dirac_ctx *c, dirac_prec pr, int sites) {
    const size_t n = sites == 0 ? (size_t)c->V : (size_t)c->vh;
    return n * 24 * (pr == DIRAC_F32 ? 4 : 8);
}
size_t native_bytes(const dirac_ctx *c, dirac_prec pr, int sites) {
    const size_t n = (sites == 0 ? 2 : 1) * (size_t)c->g.vhp;
    return n * 24 * dl::real_size(pr);
}

// C* boundaries: directions 1 .. cstar; the mirror shift dims[1] / 2 must be even with cstar >= 2
// (it would otherwise join sites of equal parity)
void check_cstar(const dirac_params *prm) {
    require(prm->cstar >= 0 && prm->cstar <= 3, "cstar must be 0 .. 3");
    require(prm->cstar < 2 || prm->dims[1] % 4 == 0,
            "with C* boundaries in more than one direction dims[1] (the doubled extent) must be a multiple of 4");
}

// eq. (ipt) is one-to-one on each parity when the blocks tile the lattice and B3 is even: the
// two sites of each pair (2j, 2j + 1) of block order then differ in x3 alone
void check_cache_block(const int *dims, const int *block) {
    for (int m = 0; m < 4; ++m)
        require(block[m] >= 1 && dims[m] % block[m] == 0,
                "cache-block extent block[" + std::to_string(m) + "] = " + std::to_string(block[m]) +
                    " does not divide the lattice extent " + std::to_string(dims[m]));
    require(block[3] % 2 == 0, "the cache-block extent block[3] must be even");
}

void check_user_layout(dirac_prec pr, dirac_layout lay) {
    require(lay == DIRAC_LAYOUT_LEX || lay == DIRAC_LAYOUT_EO || lay == DIRAC_LAYOUT_NATIVE ||
                lay == DIRAC_LAYOUT_OPENQXD,
            "unknown layout");
    if (lay != DIRAC_LAYOUT_NATIVE && (pr == DIRAC_F16 || pr == DIRAC_BF16))
        throw dl::Error(DIRAC_EUNSUPPORTED, "F16 and BF16 fields exist in the NATIVE layout only");
}

}  // namespace

namespace dl {
// The status and message of a failed call, for entry points defined in other files.
dirac_status api_fail(dirac_status s, const std::string &m) { return fail(s, m); }
void api_clear_error() { g_err.clear(); }
void api_check_dev(const void *ptr, size_t bytes, const char *name) { check_dev(ptr, bytes, name); }
}  // namespace dl

extern "C" {

const char *dirac_last_error(void) { return g_err.c_str(); }

dirac_status dirac_create(const dirac_params *prm, const void *su3_links, const double *u1_angles, void *stream,
                          dirac_ctx **out) {
    dirac_ctx *c = nullptr;
    g_err.clear();
    try {
        require(prm != nullptr && out != nullptr, "params and out must not be NULL");
        *out = nullptr;
        int64_t V = 1;
        for (int m = 0; m < 4; ++m) {
            require(prm->dims[m] >= 2 && prm->dims[m] % 2 == 0,
                    "every lattice extent must be even and >= 2 (dims[" + std::to_string(m) + "] = " +
                        std::to_string(prm->dims[m]) + ")");
            V *= prm->dims[m];
        }
        require(V < (int64_t)1 << 30, "lattice too large for 32-bit site indices");
        require(std::isfinite(prm->kappa) && prm->kappa != 0.0, "kappa must be finite and non-zero");
        require(std::isfinite(prm->csw) && std::isfinite(prm->csw_qed), "c_sw and c_sw^QED must be finite");
        for (int m = 0; m < 4; ++m) require(std::isfinite(prm->bc_phase[m]), "boundary phases must be finite");
        check_cstar(prm);
        check_dev(su3_links, (size_t)V * 4 * 9 * 16, "su3_links");
        if (u1_angles) check_dev(u1_angles, (size_t)V * 4 * 8, "u1_angles");
        hipStream_t s = (hipStream_t)stream;
        c = new dirac_ctx();
        c->p = *prm;
        c->V = V;
        c->vh = V / 2;
        for (int m = 0; m < 4; ++m) c->g.L[m] = prm->dims[m];
        c->g.h3 = prm->dims[3] / 2;
        c->g.vh = (int)c->vh;
        c->g.vhp = (int)padded_sites(c->vh);
        for (int m = 0; m < 4; ++m) c->g.B[m] = prm->dims[m];
        c->g.cs = prm->cstar;
        c->g.h1 = prm->dims[1] / 2;
        c->U_lex.alloc((size_t)V * 4 * 9 * 16);
        HIP_CHECK(hipMemcpyAsync(c->U_lex.p, su3_links, (size_t)V * 4 * 9 * 16, hipMemcpyDeviceToDevice, s));
        if (u1_angles) {
            c->theta_lex.alloc((size_t)V * 4 * 8);
            HIP_CHECK(hipMemcpyAsync(c->theta_lex.p, u1_angles, (size_t)V * 4 * 8, hipMemcpyDeviceToDevice, s));
        }
        dl::import_links(c, s);
        dl::clover_build(c, s);
        const int64_t bad = dl::clover_invert_parity(c, 1, s);
        HIP_CHECK(hipStreamSynchronize(s));
        // the gauge input is no longer needed: links are compressed, the clover field is built
        c->U_lex.release();
        c->theta_lex.release();
        *out = c;
        if (bad >= 0) return fail(DIRAC_ESINGULAR, "singular odd-site clover block at Lambda = " + std::to_string(bad));
    } catch (const dl::Error &e) {
        if (c) { dirac_destroy(c); }
        return fail(e.status, e.what());
    } catch (const std::bad_alloc &) {
        if (c) dirac_destroy(c);
        return fail(DIRAC_ENOMEM, "host allocation failed");
    } catch (...) {
        if (c) dirac_destroy(c);
        return fail(DIRAC_EHIP, "internal error");
    }
    return DIRAC_OK;
}



dirac_status dirac_set_cache_block(dirac_ctx *c, const int *block) {
    API_BEGIN
    check_ctx(c);
    require(block != nullptr, "block is NULL");
    check_cache_block(c->p.dims, block);
    for (int m = 0; m < 4; ++m) c->g.B[m] = block[m];
    API_END
}

dirac_status dirac_create_openqxd(const dirac_params *prm, const int *block, const void *u_odd, const double *a_odd,
                                  void *stream, dirac_ctx **out) {
    dl::DevBuf U, th;
    g_err.clear();
    try {
        require(prm != nullptr && out != nullptr && block != nullptr, "params, block and out must not be NULL");
        *out = nullptr;
        int64_t V = 1;
        for (int m = 0; m < 4; ++m) {
            require(prm->dims[m] >= 2 && prm->dims[m] % 2 == 0, "every lattice extent must be even and >= 2");
            V *= prm->dims[m];
        }
        require(V < (int64_t)1 << 30, "lattice too large for 32-bit site indices");
        check_cache_block(prm->dims, block);
        check_cstar(prm);
        check_dev(u_odd, (size_t)V / 2 * 8 * 9 * 16, "u_odd");
        if (a_odd) check_dev(a_odd, (size_t)V / 2 * 8 * 8, "a_odd");
        hipStream_t s = (hipStream_t)stream;
        Geom g{};
        for (int m = 0; m < 4; ++m) {
            g.L[m] = prm->dims[m];
            g.B[m] = block[m];
        }
        g.h3 = prm->dims[3] / 2;
        g.cs = prm->cstar;
        g.h1 = prm->dims[1] / 2;
        g.vh = (int)(V / 2);
        g.vhp = (int)padded_sites(V / 2);
        U.alloc((size_t)V * 4 * 9 * 16);
        if (a_odd) th.alloc((size_t)V * 4 * 8);
        dl::openqxd_links_to_lex(g, (const double *)u_odd, a_odd, (double *)U.p, a_odd ? (double *)th.p : nullptr, s);
        HIP_CHECK(hipStreamSynchronize(s));
    } catch (const dl::Error &e) {
        return fail(e.status, e.what());
    } catch (const std::bad_alloc &) {
        return fail(DIRAC_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(DIRAC_EHIP, std::string("internal error: ") + e.what());
    }
    // the rest is dirac_create on the LEX copy, which is released on return
    const dirac_status st = dirac_create(prm, U.p, a_odd ? (const double *)th.p : nullptr, stream, out);
    if (*out) {
        for (int m = 0; m < 4; ++m) (*out)->g.B[m] = block[m];
    }
    return st;
}

dirac_status dirac_destroy(dirac_ctx *c) {
    API_BEGIN
    if (!c) return DIRAC_OK;
    (void)hipDeviceSynchronize();
    dl::free_bwork(c);
    dl::free_solver_work(c);
    c->U_lex.release();
    c->theta_lex.release();
    for (auto &f : c->f) {
        for (int p = 0; p < 2; ++p) {
            f.links[p].release(); f.omega[p].release(); f.clov[p].release(); f.clinv[p].release();
        }
        f.tmp_half.release(); f.user_in.release(); f.user_out.release();
    }
    for (auto &b : c->ptc_links) b.release();
    for (dl::DevBuf *b : {&c->sap_rho, &c->sap_in, &c->sap_out, &c->sap_links, &c->sap_clov}) b->release();
    c->flags.release();
    c->red.release();
    delete c;
    API_END
}

size_t dirac_native_bytes(const dirac_ctx *c, dirac_prec pr, int sites) {
    if (!c || pr < DIRAC_F64 || pr > DIRAC_BF16) return 0;
    return native_bytes(c, pr, sites);
}

dirac_status dirac_load_clover(dirac_ctx *c, const double *clover, dirac_layout lay, void *stream) {
    API_BEGIN
    check_ctx(c);
    check_dev(clover, (size_t)c->V * 72 * 8, "clover");
    dl::clover_import(c, clover, lay, (hipStream_t)stream);
    API_END
}

dirac_status dirac_get_clover(dirac_ctx *c, double *out, int inverse, dirac_layout lay, void *stream) {
    API_BEGIN
    check_ctx(c);
    check_dev(out, (size_t)c->V * 72 * 8, "out");
    dl::clover_export(c, out, inverse, lay, (hipStream_t)stream);
    API_END
}

dirac_status clover_invert(dirac_ctx *c, int mask, void *stream) {
    API_BEGIN
    check_ctx(c);
    require(mask >= 1 && mask <= 3, "parity_mask must be 1 (even), 2 (odd) or 3 (both)");
    std::string msg;
    for (int p = 0; p < 2; ++p) {
        if (!(mask & (1 << p))) continue;
        const int64_t bad = dl::clover_invert_parity(c, p, (hipStream_t)stream);
        if (bad >= 0 && msg.empty())
            msg = std::string("singular ") + (p ? "odd" : "even") + "-site clover block at Lambda = " +
                  std::to_string(bad);
    }
    if (!msg.empty()) return fail(DIRAC_ESINGULAR, msg);
    API_END
}

dirac_status dirac_import(dirac_ctx *c, void *native, const void *user, int sites, dirac_prec pr,
                          dirac_layout lay, void *stream) {
    API_BEGIN
    check_ctx(c);
    check_prec(pr);
    require(sites >= 0 && sites <= 2, "sites must be 0, 1 or 2");
    require(lay == DIRAC_LAYOUT_LEX || lay == DIRAC_LAYOUT_EO || lay == DIRAC_LAYOUT_OPENQXD,
            "user layout must be LEX, EO or OPENQXD");
    const size_t ub = sites == 0 ? (size_t)c->V * 24 * (pr == DIRAC_F32 ? 4 : 8) : (size_t)c->vh * 24 * (pr == DIRAC_F32 ? 4 : 8);
    check_dev(user, ub, "user");
    check_dev(native, native_bytes(c, pr, sites), "native");
    check_no_alias(native, native_bytes(c, pr, sites), user, ub);
    dl::spinor_import(c, native, user, sites, pr, lay, (hipStream_t)stream);
    API_END
}

dirac_status dirac_export(dirac_ctx *c, void *user, const void *native, int sites, dirac_prec pr,
                          dirac_layout lay, void *stream) {
    API_BEGIN
    check_ctx(c);
    check_prec(pr);
    require(sites >= 0 && sites <= 2, "sites must be 0, 1 or 2");
    require(lay == DIRAC_LAYOUT_LEX || lay == DIRAC_LAYOUT_EO || lay == DIRAC_LAYOUT_OPENQXD,
            "user layout must be LEX, EO or OPENQXD");
    const size_t ub = sites == 0 ? (size_t)c->V * 24 * (pr == DIRAC_F32 ? 4 : 8) : (size_t)c->vh * 24 * (pr == DIRAC_F32 ? 4 : 8);
    check_dev(user, ub, "user");
    check_dev(native, native_bytes(c, pr, sites), "native");
    check_no_alias(native, native_bytes(c, pr, sites), user, ub);
    dl::spinor_export(c, user, native, sites, pr, lay, (hipStream_t)stream);
    API_END
}

dirac_status dirac_apply(dirac_ctx *c, void *out, const void *in, dirac_prec pr, dirac_layout lay, int dagger,
                         void *stream) {
    API_BEGIN
    check_ctx(c);
    check_prec(pr);
    check_user_layout(pr, lay);
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = lay == DIRAC_LAYOUT_NATIVE ? native_bytes(c, pr, 0) : user_bytes(c, pr, 0);
    check_dev(in, nb, "in");
    check_dev(out, nb, "out");
    check_no_alias(out, nb, in, nb);
    if (lay == DIRAC_LAYOUT_NATIVE) {
        dl::full_apply(c, out, in, dagger != 0, pr, s);
    } else {
        dl::PrecFields &f = c->f[pr];
        f.user_in.alloc(native_bytes(c, pr, 0));
        f.user_out.alloc(native_bytes(c, pr, 0));
        dl::spinor_import(c, f.user_in.p, in, 0, pr, lay, s);
        dl::full_apply(c, f.user_out.p, f.user_in.p, dagger != 0, pr, s);
        dl::spinor_export(c, out, f.user_out.p, 0, pr, lay, s);
    }
    API_END
}

dirac_status dirac_apply_eo(dirac_ctx *c, void *out, const void *in, dirac_prec pr, dirac_layout lay, int dagger,
                            void *stream) {
    API_BEGIN
    check_ctx(c);
    check_prec(pr);
    check_user_layout(pr, lay);
    require(lay != DIRAC_LAYOUT_LEX, "an even half-vector is defined in the EO, OPENQXD or NATIVE layout, not LEX");
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = lay == DIRAC_LAYOUT_NATIVE ? native_bytes(c, pr, 1) : user_bytes(c, pr, 1);
    check_dev(in, nb, "in_e");
    check_dev(out, nb, "out_e");
    check_no_alias(out, nb, in, nb);
    if (lay == DIRAC_LAYOUT_NATIVE) {
        dl::schur_apply(c, out, in, dagger != 0, pr, s);
    } else {
        dl::PrecFields &f = c->f[pr];
        f.user_in.alloc(native_bytes(c, pr, 0));
        f.user_out.alloc(native_bytes(c, pr, 0));
        dl::spinor_import(c, f.user_in.p, in, 1, pr, lay, s);
        dl::schur_apply(c, f.user_out.p, f.user_in.p, dagger != 0, pr, s);
        dl::spinor_export(c, out, f.user_out.p, 1, pr, lay, s);
    }
    API_END
}

dirac_status dirac_apply_eo_multi(dirac_ctx *c, void *out, const void *in, int nrhs, dirac_prec pr, int dagger,
                                  void *stream) {
    API_BEGIN
    check_ctx(c);
    check_prec(pr);
    require(nrhs >= 1 && nrhs <= 4096, "nrhs must be 1..4096");
    const size_t nb = native_bytes(c, pr, 1) * (size_t)nrhs;
    check_dev(in, nb, "in");
    check_dev(out, nb, "out");
    check_no_alias(out, nb, in, nb);
    dl::schur_apply(c, out, in, dagger != 0, pr, (hipStream_t)stream, nrhs, nullptr);
    API_END
}

dirac_status dirac_apply_eo_noalloc(dirac_ctx *c, void *out, const void *in, dirac_prec pr, int dagger, void *stream) {
    API_BEGIN
    check_ctx(c);
    check_prec(pr);
    const size_t nb = native_bytes(c, pr, 1);
    check_dev(in, nb, "in_e");
    check_dev(out, nb, "out_e");
    check_no_alias(out, nb, in, nb);
    dl::schur_apply_noalloc(c, out, in, dagger != 0, pr, (hipStream_t)stream);
    API_END
}

dirac_status dirac_apply_hop(dirac_ctx *c, void *out, const void *in, int out_parity, dirac_prec pr, int dagger,
                             void *stream) {
    API_BEGIN
    check_ctx(c);
    check_prec(pr);
    const size_t nb = native_bytes(c, pr, 1);
    check_dev(in, nb, "in");
    check_dev(out, nb, "out");
    check_no_alias(out, nb, in, nb);
    dl::hop_apply(c, out, in, nullptr, out_parity, dl::HOP_PLAIN, -0.5, dagger != 0, pr, (hipStream_t)stream);
    API_END
}

dirac_status dirac_apply_clover(dirac_ctx *c, void *out, const void *in, int parity, int inverse, dirac_prec pr,
                                void *stream) {
    API_BEGIN
    check_ctx(c);
    check_prec(pr);
    const size_t nb = native_bytes(c, pr, 1);
    check_dev(in, nb, "in");
    check_dev(out, nb, "out");
    check_no_alias(out, nb, in, nb);
    dl::clover_apply(c, out, in, parity, inverse != 0, pr, (hipStream_t)stream);
    API_END
}

dirac_status dirac_solve(dirac_ctx *c, void *x, const void *b, dirac_layout lay, const dirac_solver_params *p,
                         dirac_solve_info *info, void *stream) {
    const auto t0 = std::chrono::steady_clock::now();
    API_BEGIN
    check_ctx(c);
    require(info != nullptr, "info is NULL");
    *info = dirac_solve_info{};
    dl::check_solver_params(p);
    require(lay == DIRAC_LAYOUT_LEX || lay == DIRAC_LAYOUT_EO || lay == DIRAC_LAYOUT_NATIVE ||
                lay == DIRAC_LAYOUT_OPENQXD,
            "unknown layout");
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = lay == DIRAC_LAYOUT_NATIVE ? native_bytes(c, DIRAC_F64, 0) : user_bytes(c, DIRAC_F64, 0);
    check_dev(b, nb, "b");
    check_dev(x, nb, "x");
    check_no_alias(x, nb, b, nb);
    const dirac_prec inner = p->method == DIRAC_SOLVER_MIXED_GCR ? (dirac_prec)p->inner_prec : DIRAC_F64;
    dl::ensure_work(c, p->method == DIRAC_SOLVER_CGLS ? 1 : p->restart, inner, 1);
    void *bn = dl::solver_full64(c, 0), *xn = dl::solver_full64(c, 1);
    c->work->syncs = 0;
    if (lay == DIRAC_LAYOUT_NATIVE) {
        HIP_CHECK(hipMemcpyAsync(bn, b, nb, hipMemcpyDeviceToDevice, s));
        if (p->x0_given) HIP_CHECK(hipMemcpyAsync(xn, x, nb, hipMemcpyDeviceToDevice, s));
    } else {
        dl::spinor_import(c, bn, b, 0, DIRAC_F64, lay, s);
        if (p->x0_given) dl::spinor_import(c, xn, x, 0, DIRAC_F64, lay, s);
    }
    const dirac_status st = p->method == DIRAC_SOLVER_CGLS ? dl::solve_cgls(c, p, p->x0_given != 0, info, s)
                                                            : dl::solve_native(c, p, p->x0_given != 0, info, s);
    if (lay == DIRAC_LAYOUT_NATIVE)
        HIP_CHECK(hipMemcpyAsync(x, xn, nb, hipMemcpyDeviceToDevice, s));
    else
        dl::spinor_export(c, x, xn, 0, DIRAC_F64, lay, s);
    HIP_CHECK(hipStreamSynchronize(s));
    info->host_syncs = (int)(c->work->syncs + 1);
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (st != DIRAC_OK) {
        char msg[160];
        snprintf(msg, sizeof msg, "solver stopped after %d iterations, true relative residual %.3e", info->iters,
                 info->true_rel_res);
        return fail(st, st == DIRAC_ENONFINITE ? std::string("non-finite value in the solve; ") + msg : msg);
    }
    API_END
}

dirac_status dirac_solve_batched(dirac_ctx *const *ctx, int nlat, void *const *x, const void *const *b, int nrhs,
                                 dirac_layout lay, const dirac_solver_params *p, dirac_solve_info *info,
                                 void *stream) {
    API_BEGIN
    require(ctx != nullptr && x != nullptr && b != nullptr && info != nullptr, "NULL argument");
    require(nlat >= 1 && nlat <= 64, "nlat must be 1..64");
    require(nrhs >= 1 && nrhs <= 64, "nrhs must be 1..64");
    dl::check_solver_params(p);
    require(p->method == DIRAC_SOLVER_GCR || p->method == DIRAC_SOLVER_MIXED_GCR,
            "batched solves run GCR or MIXED_GCR");
    require(lay == DIRAC_LAYOUT_LEX || lay == DIRAC_LAYOUT_EO || lay == DIRAC_LAYOUT_NATIVE ||
                lay == DIRAC_LAYOUT_OPENQXD,
            "unknown layout");
    for (int l = 0; l < nlat; ++l) {
        check_ctx(ctx[l]);
        for (int k = 0; k < l; ++k) require(ctx[k] != ctx[l], "each lattice needs its own context");
        const size_t nb = (size_t)nrhs *
                          (lay == DIRAC_LAYOUT_NATIVE ? native_bytes(ctx[l], DIRAC_F64, 0) : user_bytes(ctx[l], DIRAC_F64, 0));
        check_dev(b[l], nb, "b[l]");
        check_dev(x[l], nb, "x[l]");
        check_no_alias(x[l], nb, b[l], nb);
    }
    std::string err;
    const dirac_status st = dl::solve_batched(ctx, nlat, x, b, nrhs, lay, p, info, (hipStream_t)stream, err);
    if (st != DIRAC_OK) return fail(st, err);
    API_END
}

dirac_status dirac_sap(dirac_ctx *c, void *out, const void *in, int ncy, int nmr, void *stream) {
    API_BEGIN
    check_ctx(c);
    const size_t nb = native_bytes(c, DIRAC_F32, 0);
    check_dev(in, nb, "in");
    check_dev(out, nb, "out");
    check_no_alias(out, nb, in, nb);
    dl::sap_apply(c, out, in, ncy, nmr, (hipStream_t)stream);
    API_END
}

// ---------------------------------------------------------------- vector arithmetic
// Device scalars of these calls: free slots near the end of the context's scalar block.
static double *vec_slots(dirac_ctx *c) { return (double *)c->work->blas.scal.p + dl::kSysScal - 32; }

static void read_slots(double *host, const double *dev, int n, hipStream_t s) {
    HIP_CHECK(hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
}

dirac_status dirac_residual(dirac_ctx *c, void *r, const void *b, const void *x, dirac_prec pr, double *rel_res,
                            void *stream) {
    API_BEGIN
    check_ctx(c);
    require(pr == DIRAC_F64 || pr == DIRAC_F32, "the residual is formed in F64 or F32");
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = native_bytes(c, pr, 0);
    check_dev(r, nb, "r");
    check_dev(b, nb, "b");
    check_dev(x, nb, "x");
    check_no_alias(r, nb, b, nb);
    check_no_alias(r, nb, x, nb);
    dl::ensure_blas(c);
    dl::Blas &B = c->work->blas;
    double *sl = vec_slots(c);
    dl::full_apply(c, r, x, 0, pr, s);
    // r = b - D x in place (element-wise), with |r|^2 and the non-finite flag
    B.lincomb(pr, pr, pr, 2, r, nullptr, 1.0, b, -1.0, r, rel_res ? sl : nullptr, 1.0, s);
    if (rel_res) {
        B.mdot(pr, 2, b, 1, b, sl + 2, 1.0, s);
        double h[4];
        read_slots(h, sl, 4, s);
        require(h[1] == 0.0 && std::isfinite(h[0]) && std::isfinite(h[2]), "non-finite value in the residual",
                DIRAC_ENONFINITE);
        *rel_res = h[2] > 0.0 ? std::sqrt(h[0] / h[2]) : 0.0;
    }
    API_END
}

dirac_status dirac_lincomb(dirac_ctx *c, void *out, dirac_prec out_prec, double alpha, const void *a, double beta,
                           const void *b, dirac_prec in_prec, int sites, double *norm2, void *stream) {
    API_BEGIN
    check_ctx(c);
    check_prec(out_prec);
    check_prec(in_prec);
    require(sites == 0 || sites == 1, "sites must be 0 (full vectors) or 1 (one parity)");
    require(std::isfinite(alpha) && std::isfinite(beta), "coefficients must be finite");
    require(out_prec == in_prec || in_prec == DIRAC_F64,
            "inputs in the output precision, or F64 inputs converted to any output precision");
    hipStream_t s = (hipStream_t)stream;
    const size_t nbo = native_bytes(c, out_prec, sites), nbi = native_bytes(c, in_prec, sites);
    check_dev(a, nbi, "a");
    check_dev(out, nbo, "out");
    if (beta != 0.0) {
        check_dev(b, nbi, "b");
        check_no_alias(out, nbo, b, nbi);
    }
    check_no_alias(out, nbo, a, nbi);
    dl::ensure_blas(c);
    dl::Blas &B = c->work->blas;
    double *sl = vec_slots(c);
    B.lincomb(out_prec, in_prec, in_prec, sites == 0 ? 2 : 1, out, nullptr, alpha, a, beta, beta != 0.0 ? b : nullptr,
              norm2 ? sl : nullptr, 1.0, s);
    if (norm2) {
        double h[2];
        read_slots(h, sl, 2, s);
        require(h[1] == 0.0 && std::isfinite(h[0]), "non-finite value in the result", DIRAC_ENONFINITE);
        *norm2 = h[0];
    }
    API_END
}

dirac_status dirac_dot(dirac_ctx *c, const void *a, const void *b, dirac_prec pr, int sites, double *dot,
                       void *stream) {
    API_BEGIN
    check_ctx(c);
    check_prec(pr);
    require(dot != nullptr, "dot is NULL");
    require(sites == 0 || sites == 1, "sites must be 0 (full vectors) or 1 (one parity)");
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = native_bytes(c, pr, sites);
    check_dev(a, nb, "a");
    check_dev(b, nb, "b");
    dl::ensure_blas(c);
    double *sl = vec_slots(c);
    c->work->blas.mdot(pr, sites == 0 ? 2 : 1, a, 1, b, sl + 4, 1.0, s);
    read_slots(dot, sl + 4, 2, s);
    API_END
}

// ---------------------------------------------------------------- learned preconditioner
dirac_status ptc_create(const int *channels, int nlayers, dirac_ptc **out) {
    API_BEGIN
    require(channels != nullptr && out != nullptr, "channels and out must not be NULL");
    require(nlayers >= 1 && nlayers <= 8, "nlayers must be 1..8");
    require(channels[0] == 1 && channels[nlayers] == 1, "the network maps one channel to one channel");
    for (int l = 0; l <= nlayers; ++l)
        require(channels[l] == 1 || channels[l] == 2 || channels[l] == 4 || channels[l] == 8,
                "channel counts must be 1, 2, 4 or 8");
    dirac_ptc *n = new dirac_ptc();
    n->nlayers = nlayers;
    for (int l = 0; l <= nlayers; ++l) n->ch[l] = channels[l];
    try {
        dl::ptc_alloc(n);
    } catch (...) {
        delete n;
        throw;
    }
    *out = n;
    API_END
}

dirac_status ptc_destroy(dirac_ptc *n) {
    API_BEGIN
    if (!n) return DIRAC_OK;
    (void)hipDeviceSynchronize();
    for (dl::DevBuf *b : {&n->w, &n->wbf, &n->wt, &n->grad, &n->m, &n->v, &n->acts, &n->gbuf, &n->part, &n->afw, &n->afb, &n->afz, &n->zbuf})
        b->release();
    delete n;
    API_END
}

size_t ptc_num_weights(const dirac_ptc *n) { return n ? 2 * n->total : 0; }

dirac_status ptc_set_weights(dirac_ptc *n, const float *host_w, size_t cnt) {
    API_BEGIN
    require(n != nullptr && host_w != nullptr, "network and weights must not be NULL");
    require(cnt == 2 * n->total, "weight count must equal ptc_num_weights");
    HIP_CHECK(hipMemcpy(n->w.p, host_w, cnt * sizeof(float), hipMemcpyHostToDevice));
    HIP_CHECK(hipMemset(n->m.p, 0, cnt * sizeof(float)));
    HIP_CHECK(hipMemset(n->v.p, 0, cnt * sizeof(float)));
    n->step = 0;
    dl::ptc_refresh_bf16(n, nullptr);
    HIP_CHECK(hipDeviceSynchronize());
    API_END
}

dirac_status ptc_get_weights(const dirac_ptc *n, float *host_w, size_t cnt) {
    API_BEGIN
    require(n != nullptr && host_w != nullptr, "network and buffer must not be NULL");
    require(cnt == 2 * n->total, "weight count must equal ptc_num_weights");
    HIP_CHECK(hipDeviceSynchronize());
    HIP_CHECK(hipMemcpy(host_w, n->w.p, cnt * sizeof(float), hipMemcpyDeviceToHost));
    API_END
}

dirac_status ptc_get_grad(const dirac_ptc *n, float *host_g, size_t cnt) {
    API_BEGIN
    require(n != nullptr && host_g != nullptr, "network and buffer must not be NULL");
    require(cnt == 2 * n->total, "gradient count must equal ptc_num_weights");
    HIP_CHECK(hipDeviceSynchronize());
    HIP_CHECK(hipMemcpy(host_g, n->grad.p, cnt * sizeof(float), hipMemcpyDeviceToHost));
    API_END
}

dirac_status ptc_get_adam_state(const dirac_ptc *n, float *host_m, float *host_v, size_t cnt, int *step) {
    API_BEGIN
    require(n != nullptr && host_m != nullptr && host_v != nullptr && step != nullptr, "NULL argument");
    require(cnt == 2 * n->total, "moment count must equal ptc_num_weights");
    HIP_CHECK(hipDeviceSynchronize());
    HIP_CHECK(hipMemcpy(host_m, n->m.p, cnt * sizeof(float), hipMemcpyDeviceToHost));
    HIP_CHECK(hipMemcpy(host_v, n->v.p, cnt * sizeof(float), hipMemcpyDeviceToHost));
    *step = n->step;
    API_END
}

dirac_status ptc_set_adam_state(dirac_ptc *n, const float *host_m, const float *host_v, size_t cnt, int step) {
    API_BEGIN
    require(n != nullptr && host_m != nullptr && host_v != nullptr, "NULL argument");
    require(cnt == 2 * n->total, "moment count must equal ptc_num_weights");
    require(step >= 0, "step must not be negative");
    for (size_t i = 0; i < cnt; ++i)
        require(std::isfinite(host_m[i]) && std::isfinite(host_v[i]) && host_v[i] >= 0.0f,
                "moments must be finite, second moments non-negative");
    HIP_CHECK(hipDeviceSynchronize());
    HIP_CHECK(hipMemcpy(n->m.p, host_m, cnt * sizeof(float), hipMemcpyHostToDevice));
    HIP_CHECK(hipMemcpy(n->v.p, host_v, cnt * sizeof(float), hipMemcpyHostToDevice));
    n->step = step;
    API_END
}

dirac_status ptc_zero_grad(dirac_ptc *n, void *stream) {
    API_BEGIN
    require(n != nullptr, "network is NULL");
    n->grad_zero((hipStream_t)stream);
    API_END
}

dirac_status ptc_forward(dirac_ctx *c, dirac_ptc *n, void *out, const void *in, void *stream) {
    API_BEGIN
    check_ctx(c);
    require(n != nullptr, "network is NULL");
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = native_bytes(c, DIRAC_F32, 0);
    check_dev(in, nb, "in");
    check_dev(out, nb, "out");
    check_no_alias(out, nb, in, nb);
    dl::ptc_ensure_acts(c, n);
    HIP_CHECK(hipMemcpyAsync(dl::ptc_act(c, n, 0), in, nb, hipMemcpyDeviceToDevice, s));
    dl::ptc_forward_acts(c, n, s, false);
    HIP_CHECK(hipMemcpyAsync(out, dl::ptc_act(c, n, n->nlayers), nb, hipMemcpyDeviceToDevice, s));
    API_END
}

dirac_status ptc_forward_eo(dirac_ctx *c, dirac_ptc *n, void *out, const void *in, void *stream) {
    API_BEGIN
    check_ctx(c);
    require(n != nullptr, "network is NULL");
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = native_bytes(c, DIRAC_F32, 1);
    check_dev(in, nb, "in_e");
    check_dev(out, nb, "out_e");
    check_no_alias(out, nb, in, nb);
    dl::ptc_ensure_acts(c, n);
    char *a0 = (char *)dl::ptc_act(c, n, 0);
    HIP_CHECK(hipMemcpyAsync(a0, in, nb, hipMemcpyDeviceToDevice, s));
    dl::zero_fill(a0 + nb, nb, s);
    dl::ptc_forward_acts(c, n, s, false, true);
    HIP_CHECK(hipMemcpyAsync(out, dl::ptc_act(c, n, n->nlayers), nb, hipMemcpyDeviceToDevice, s));
    API_END
}

dirac_status ptc_backward(dirac_ctx *c, dirac_ptc *n, void *grad_in, const void *in, const void *grad_out,
                          void *stream) {
    API_BEGIN
    check_ctx(c);
    require(n != nullptr, "network is NULL");
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = native_bytes(c, DIRAC_F32, 0);
    check_dev(in, nb, "in");
    check_dev(grad_out, nb, "grad_out");
    if (grad_in) {
        check_dev(grad_in, nb, "grad_in");
        check_no_alias(grad_in, nb, in, nb);
        check_no_alias(grad_in, nb, grad_out, nb);
    }
    dl::ptc_ensure_acts(c, n);
    HIP_CHECK(hipMemcpyAsync(dl::ptc_act(c, n, 0), in, nb, hipMemcpyDeviceToDevice, s));
    dl::ptc_forward_acts(c, n, s);
    dl::ptc_backward_acts(c, n, grad_out, grad_in, s);
    API_END
}

dirac_status ptc_adam_step(dirac_ptc *n, double lr, void *stream) {
    API_BEGIN
    require(n != nullptr, "network is NULL");
    require(std::isfinite(lr) && lr > 0.0, "learning rate must be positive");
    dl::ptc_adam(n, lr, (hipStream_t)stream);
    API_END
}

dirac_status ptc_train_step(dirac_ctx *c, dirac_ptc *n, const void *const *r, const void *const *e, int nbatch,
                            double lr, double *loss, void *stream) {
    API_BEGIN
    check_ctx(c);
    require(n != nullptr && r != nullptr && e != nullptr && loss != nullptr, "NULL argument");
    require(nbatch >= 1, "nbatch must be positive");
    require(std::isfinite(lr) && lr > 0.0, "learning rate must be positive");
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = native_bytes(c, DIRAC_F32, 0);
    for (int i = 0; i < nbatch; ++i) {
        check_dev(r[i], nb, "r[i]");
        check_dev(e[i], nb, "e[i]");
    }
    dl::ptc_ensure_acts(c, n);
    dl::ensure_work(c, 1, DIRAC_F32, 2);
    n->grad_zero(s);
    dl::Blas &B = c->work->blas;
    double *sc = (double *)B.scal.p + dl::kSysScal - 16;  // free slots at the end of the scalar block
    const double scale = 1.0 / (24.0 * (double)c->vh);
    double total = 0.0;
    void *g = c->work->P.p;  // dL/dy* of the current pair (F32 full)
    for (int i = 0; i < nbatch; ++i) {
        HIP_CHECK(hipMemcpyAsync(dl::ptc_act(c, n, 0), r[i], nb, hipMemcpyDeviceToDevice, s));
        dl::ptc_forward_acts(c, n, s);
        const void *y = dl::ptc_act(c, n, n->nlayers);
        B.mdot(DIRAC_F32, 2, e[i], 1, e[i], sc, scale, s);
        double ne2 = 0.0;
        HIP_CHECK(hipMemcpyAsync(&ne2, sc, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        require(std::isfinite(ne2) && ne2 > 0.0, "target e is zero or not finite", DIRAC_ENONFINITE);
        // g = (y - e) / (|e|^2 nbatch), with |.|^2 in the normalised norm (the factor cancels in L)
        const double f = 1.0 / (ne2 / scale * nbatch);
        B.lincomb(DIRAC_F32, DIRAC_F32, DIRAC_F32, 2, g, nullptr, f, y, -f, e[i], sc + 2, 1.0, s);
        double gn = 0.0;
        HIP_CHECK(hipMemcpyAsync(&gn, sc + 2, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        total += gn / (f * f) / (ne2 / scale) / nbatch;  // |y - e|^2 / |e|^2 / nbatch
        dl::ptc_backward_acts(c, n, g, nullptr, s);
    }
    *loss = total;
    // the weights and Adam moments change only when the loss and every gradient entry are finite
    require(std::isfinite(total), "non-finite loss; weights and Adam state left unchanged", DIRAC_ENONFINITE);
    std::vector<float> hg(2 * n->total);
    HIP_CHECK(hipMemcpyAsync(hg.data(), n->grad.p, hg.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    for (float v : hg)
        require(std::isfinite(v), "non-finite weight gradient; weights and Adam state left unchanged",
                DIRAC_ENONFINITE);
    dl::ptc_adam(n, lr, s);
    HIP_CHECK(hipStreamSynchronize(s));
    API_END
}

dirac_status ptc_loss(dirac_ctx *c, dirac_ptc *n, const void *const *r, const void *const *e, int nbatch,
                      double *loss, void *stream) {
    API_BEGIN
    check_ctx(c);
    require(n != nullptr && r != nullptr && e != nullptr && loss != nullptr, "NULL argument");
    require(nbatch >= 1, "nbatch must be positive");
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = native_bytes(c, DIRAC_F32, 0);
    for (int i = 0; i < nbatch; ++i) {
        check_dev(r[i], nb, "r[i]");
        check_dev(e[i], nb, "e[i]");
    }
    dl::ptc_ensure_acts(c, n);
    dl::ensure_work(c, 1, DIRAC_F32, 2);
    dl::Blas &B = c->work->blas;
    double *sc = (double *)B.scal.p + dl::kSysScal - 16;
    void *d = c->work->P.p;  // N(r_i) - e_i
    double total = 0.0;
    for (int i = 0; i < nbatch; ++i) {
        HIP_CHECK(hipMemcpyAsync(dl::ptc_act(c, n, 0), r[i], nb, hipMemcpyDeviceToDevice, s));
        dl::ptc_forward_acts(c, n, s, false);
        B.mdot(DIRAC_F32, 2, e[i], 1, e[i], sc, 1.0, s);
        B.lincomb(DIRAC_F32, DIRAC_F32, DIRAC_F32, 2, d, nullptr, 1.0, dl::ptc_act(c, n, n->nlayers), -1.0, e[i],
                  sc + 2, 1.0, s);
        double h[4];
        HIP_CHECK(hipMemcpyAsync(h, sc, sizeof h, hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        require(std::isfinite(h[0]) && h[0] > 0.0, "target e is zero or not finite", DIRAC_ENONFINITE);
        total += h[2] / h[0] / nbatch;
    }
    *loss = total;
    require(std::isfinite(total), "non-finite loss", DIRAC_ENONFINITE);
    API_END
}

}  // extern "C"
