// Host-side definitions shared by the library's translation units: the context,
// device buffers, error handling and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <stdexcept>
#include <string>

#include "dirac.h"
#include "common.h"

namespace dl {

// Error carried from a failing step to the C ABI, where it becomes a status code.
struct Error : std::runtime_error {
    dirac_status status;
    Error(dirac_status s, const std::string &m) : std::runtime_error(m), status(s) {}
};

#define HIP_CHECK(expr)                                                                                 \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            throw ::dl::Error(e_ == hipErrorOutOfMemory ? DIRAC_ENOMEM : DIRAC_EHIP,                    \
                              std::string(#expr) + ": " + hipGetErrorString(e_));                       \
    } while (0)

inline void require(bool ok, const std::string &msg, dirac_status s = DIRAC_EINVAL) {
    if (!ok) throw Error(s, msg);
}

// Device allocation owned by the context (freed in dirac_destroy).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void alloc(size_t n) {
        if (p && bytes >= n) return;
        release();
        HIP_CHECK(hipMalloc(&p, n));
        bytes = n;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

inline size_t real_size(dirac_prec pr) { return pr == DIRAC_F64 ? 8 : pr == DIRAC_F32 ? 4 : 2; }

// Fields of one storage precision.  Links: per parity, 8 directions (2 mu = forward
// link V_mu(x), 2 mu + 1 = V_mu(x - mu) seen from x), 12 reals (rows 0, 1 of the SU(3)
// matrix) in planes of 16 bytes (8 for F16 / BF16) plus one angle omega per link
// (qhat theta plus the boundary phase where the link crosses the boundary), kept in
// FP64 for F64 and FP32 otherwise.  Clover: per parity 72 reals (2 x 36 packed).
struct PrecFields {
    bool links_ready = false, clover_ready = false;
    bool inv_ready[2] = {false, false};
    DevBuf links[2], omega[2], clov[2], clinv[2];
    DevBuf tmp_half;    // intermediate of the Schur operator (odd half)
    DevBuf user_in, user_out;  // NATIVE staging for user-layout calls (full vectors)
};

struct SolverWork;  // solver.hip
struct BWork;       // tune.hip: launch-shape tuner (see there)
const char *prec_name(dirac_prec pr);
int tuned_choice(const char *key, int nshapes, const std::function<void(int)> &launch, hipStream_t s);
int tuned_lookup(const char *key);  // -1 when the key has not been tuned

// batched.hip

}  // namespace dl

struct dirac_ctx {
    dirac_params p;
    Geom g;
    int64_t V, vh;
    dl::DevBuf U_lex, theta_lex;   // FP64 copies of the gauge input (clover rebuild, precision copies)
    dl::PrecFields f[4];           // indexed by dirac_prec
    dl::DevBuf ptc_links[2];       // full FP32 links with phases for the PTC network (built on first use)
    dl::DevBuf sap_rho;            // Schwarz preconditioner: residual, solution, corrections (block order)
    dl::DevBuf sap_in, sap_out;    // FGCR_SAP: the preconditioner's F32 input and output
    dl::DevBuf sap_links, sap_clov;  // Schwarz blocks: F32 links and clover field in block order
    bool sap_ready = false;        // sap_links / sap_clov match the current fields
    bool ptc_links_ready = false;
    dl::DevBuf flags;              // small device scratch: flags, maxima
    dl::DevBuf red;                // reduction partials
    dl::SolverWork *work = nullptr;
    dl::BWork *bwork = nullptr;
};

namespace dl {

constexpr int kBlock = 256;
inline int grid_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }
inline int grid_xcd(int64_t n) { return (grid_for(n) + 7) & ~7; }

size_t link_plane_bytes(dirac_prec pr);  // bytes of one 12-real link plane set, per site and direction

// fields.hip
void import_links(dirac_ctx *c, hipStream_t s);
// openQxD odd-point gauge storage (u_odd [V/2][8][3][3], a_odd [V/2][8] or NULL) to LEX [V][4] arrays
void openqxd_links_to_lex(const Geom &g, const double *u_odd, const double *a_odd, double *U, double *th,
                          hipStream_t s);
void ensure_prec(dirac_ctx *c, dirac_prec pr, hipStream_t s);
// zero `bytes` (a multiple of 16) with a kernel, so that a captured graph holds no memset node
void zero_fill(void *p, size_t bytes, hipStream_t s);
// Schwarz (SAP) preconditioner, psi = M r on NATIVE F32 full vectors (sap.hip)
bool sap_supported(const dirac_ctx *c);
void sap_apply(dirac_ctx *c, void *psi, const void *r, int ncy, int nmr, hipStream_t s);
void spinor_import(dirac_ctx *c, void *native, const void *user, int sites, dirac_prec pr, dirac_layout lay,
                   hipStream_t s);
void spinor_export(dirac_ctx *c, void *user, const void *native, int sites, dirac_prec pr, dirac_layout lay,
                   hipStream_t s);
void clover_import(dirac_ctx *c, const double *user, dirac_layout lay, hipStream_t s);
void clover_export(dirac_ctx *c, double *user, int inverse, dirac_layout lay, hipStream_t s);

// clover.hip
void clover_build(dirac_ctx *c, hipStream_t s);
int64_t clover_invert_parity(dirac_ctx *c, int parity, hipStream_t s);  // returns first singular Lambda or -1
void clover_apply(dirac_ctx *c, void *out, const void *in, int parity, int inverse, dirac_prec pr, hipStream_t s,
                  int nrhs = 1);

// hop.hip
enum HopMode { HOP_PLAIN = 0, HOP_INV = 1, HOP_CLOV = 2 };
// out_p = mode(coef * H in_{1-p}); HOP_INV applies A_pp^-1 after, HOP_CLOV adds A_pp chi_p.
// nrhs right-hand sides: vector r of out / in / chi is r half-lattice vectors after the base;
// right-hand sides whose active flag is 0 are skipped.
// no_alloc: neither build the fields of pr (they must exist) nor time launch shapes.
void hop_apply(dirac_ctx *c, void *out, const void *in, const void *chi, int out_parity, HopMode mode, double coef,
               int dagger, dirac_prec pr, hipStream_t s, int nrhs = 1, const int *active = nullptr,
               bool no_alloc = false);
void schur_apply(dirac_ctx *c, void *out_e, const void *in_e, int dagger, dirac_prec pr, hipStream_t s, int nrhs = 1,
                 const int *active = nullptr);
// D-hat with the odd intermediate in caller-provided device memory `tmp` (nrhs odd half vectors)
void schur_apply_into(dirac_ctx *c, void *out_e, const void *in_e, void *tmp, int dagger, dirac_prec pr,
                      hipStream_t s, int nrhs, const int *active, bool no_alloc);
void full_apply(dirac_ctx *c, void *out, const void *in, int dagger, dirac_prec pr, hipStream_t s);

// noalloc.hip: D-hat with the intermediate in the library's static device buffer (allocates nothing)
void schur_apply_noalloc(dirac_ctx *c, void *out_e, const void *in_e, int dagger, dirac_prec pr, hipStream_t s);

// solver.hip
void free_solver_work(dirac_ctx *c);
void ensure_work(dirac_ctx *c, int restart, dirac_prec inner, int nh);
void ensure_blas(dirac_ctx *c);  // the reduction buffers alone (no Krylov vectors)
void *solver_full64(dirac_ctx *c, int k);  // NATIVE FP64 full vectors: 0 = b, 1 = x, 2 = scratch
dirac_status solve_native(dirac_ctx *c, const dirac_solver_params *p, bool x0, dirac_solve_info *info,
                          hipStream_t s);
dirac_status solve_cgls(dirac_ctx *c, const dirac_solver_params *p, bool x0, dirac_solve_info *info, hipStream_t s);
void check_solver_params(const dirac_solver_params *p);

// tune.hip: launch-shape tuner (see there)
const char *prec_name(dirac_prec pr);
int tuned_choice(const char *key, int nshapes, const std::function<void(int)> &launch, hipStream_t s);
int tuned_lookup(const char *key);  // -1 when the key has not been tuned

// api.hip: status and thread-local message of a failed call, for entry points in other files
dirac_status api_fail(dirac_status s, const std::string &m);
void api_clear_error();
void api_check_dev(const void *ptr, size_t bytes, const char *name);  // device memory of at least `bytes`

// batched.hip
void free_bwork(dirac_ctx *c);
dirac_status solve_batched(dirac_ctx *const *ctx, int nlat, void *const *x, const void *const *b, int nrhs,
                           dirac_layout lay, const dirac_solver_params *p, dirac_solve_info *info, hipStream_t user,
                           std::string &err);

}  // namespace dl
