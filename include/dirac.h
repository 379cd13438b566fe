/*
 * dirac.h - C ABI of the MI355X (gfx950) library for the QCD+QED O(a)-improved
 * Wilson-Dirac operator and its even-odd preconditioned Krylov solves.
 *
 * Paper: R. Gruber et al., "O(a)-improved QCD+QED Wilson Dirac operator on GPUs",
 * arXiv:2502.02490 (LATTICE2024).
 *
 * ---------------------------------------------------------------------------
 * Operator (the paper names D_w in Sec. 2 but does not write it out; the
 * readings below are the library's definition and are fixed here):
 *
 *   D psi(x) = (4 + m0) psi(x) + C(x) psi(x)
 *              - 1/2 sum_mu [ V_mu(x) b+_mu(x) (1 - gamma_mu) psi(x + mu)
 *                           + V_mu(x - mu)^dag b-_mu(x) (1 + gamma_mu) psi(x - mu) ]
 *   m0 = 1/(2 kappa) - 4             (D itself, not 2 kappa D)
 *   V_mu(x) = exp(i qhat theta_mu(x)) U_mu(x)       (U(3) link, Sec. 4.3)
 *   b+_mu(x) = exp(i phi_mu) if x_mu = L_mu - 1, b-_mu(x) = exp(-i phi_mu) if x_mu = 0
 *   C(x) = c_sw (i/4) sum_{mu != nu} sigma_{mu nu} F_{mu nu}(x)
 *        + c_sw^QED qhat (i/4) sum_{mu != nu} sigma_{mu nu} F^U(1)_{mu nu}(x)   (Sec. 4.3)
 *   F = (Q - Q^dag)/8, Q = sum of the four plaquette leaves at x in the (mu, nu)
 *   plane, from U alone (SU(3) part) or from exp(i theta) alone (U(1) part);
 *   no traceless projection; boundary phases do not enter C.
 *   gamma matrices: chiral basis, gamma_0 = [[0,-1],[-1,0]],
 *   gamma_k = [[0,-i sigma_k],[i sigma_k,0]], gamma_5 = diag(1,1,-1,-1),
 *   sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu].  A = (4 + m0) + C is Hermitian and
 *   block-diagonal in chirality: an upper block (spins 0,1) and a lower block
 *   (spins 2,3), each 6x6 (Sec. 2).
 *
 * Even-odd (Schur) form: D = [[A_ee, D_eo], [D_oe, A_oo]] with D_eo = -H_eo / 2,
 *   D-hat = A_ee - D_eo A_oo^-1 D_oe  on the even sites,
 *   D-hat^dag = gamma_5 D-hat gamma_5.
 *
 * ---------------------------------------------------------------------------
 * Sites and layouts (Sec. 4.1.1).  Coordinates x = (x0, x1, x2, x3), x0 = time.
 * All four extents must be even (the checkerboard must survive the periodic wrap).
 *   Lambda(x) = L3 L2 L1 x0 + L3 L2 x1 + L3 x2 + x3                  eq. (lexi)
 *   parity P(x) = (x0 + x1 + x2 + x3) mod 2
 *   xhat(x) = floor(Lambda / 2) + P(x) V / 2      eq. (ipt) with one block (B = L)
 *
 * DIRAC_LAYOUT_LEX     spinor: [V][4 spin][3 colour] complex (re, im), colour
 *                      fastest (Sec. 2, Sec. 4.1.2), sites in Lambda order.
 * DIRAC_LAYOUT_EO      the same per-site layout, sites in xhat order (even
 *                      sites first).  A half (even-site) vector is the first
 *                      V/2 sites of an EO vector.
 * DIRAC_LAYOUT_NATIVE  the library's device layout.  Per parity, the V/2 sites (in
 *                      floor(Lambda / 2) order) are padded to Vp = a multiple of 64 and
 *                      grouped in blocks of 64: [Vp / 64][24 / W][64][W] reals with W = 2
 *                      for F64, 4 for F32, 8 for F16 and BF16 (16-byte vectors).  A full
 *                      vector is the even half then the odd half; dirac_native_bytes gives
 *                      the size.  Padding sites are never read or written.  Use this layout
 *                      when timing.
 * DIRAC_LAYOUT_OPENQXD the same per-site layout, sites in openQxD's order, eq. (ipt) with
 *                      the context's cache block B (Sec. 4.1.1):
 *                        xhat = floor((V_B Lambda(n, N_B) + Lambda(b, B)) / 2) + P(x) V / 2,
 *                      b = x mod B, n = floor(x / B), N_B = L / B, V_B = B0 B1 B2 B3;
 *                      dirac_set_cache_block sets B (default B = L, the EO order).  A half
 *                      (even-site) vector is the first V/2 sites.
 * User-layout (LEX/EO/OPENQXD) buffers are complex128 for DIRAC_F64 and complex64 for
 * DIRAC_F32; F16 and BF16 exist in the NATIVE layout only.
 *
 * Gauge input (Sec. 4.1.4): su3_links [V][mu = 0..3][a][b] complex128, row-major
 * 3x3 SU(3) matrices, four forward links per site, LEX order; u1_angles
 * [V][4] float64 (theta_mu(x)) or NULL for theta = 0.
 * Clover input/output (Sec. 4.1.3): [site][2][36] float64 per site, block + then
 * block -, each 6 diagonal reals followed by (re, im) of the 15 strictly-upper
 * entries in row-major order, block row index 3 * spin + colour.
 *
 * ---------------------------------------------------------------------------
 * Conventions of every call.
 *   All pointers to fields are device pointers; the caller owns them and keeps
 *   them alive until the work queued on `stream` has finished.  `stream` is a
 *   hipStream_t (NULL = the default stream).  Apply calls are asynchronous on
 *   `stream`; calls that return a value computed on the device (clover_invert,
 *   dirac_solve) synchronise `stream` before returning.
 *   No call aborts, throws or prints.  On failure it returns a status other than
 *   DIRAC_OK and dirac_last_error() returns a message (thread-local, valid until
 *   the next call on the same thread).  Output buffers must not alias inputs.
 *   A context is not thread-safe; distinct contexts are independent.
 */
#ifndef DIRAC_H
#define DIRAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dirac_ctx dirac_ctx;

typedef enum {
    DIRAC_OK = 0,
    DIRAC_EINVAL = 1,      /* bad argument: NULL pointer, odd extent, aliasing, bad enum */
    DIRAC_ENOMEM = 2,      /* device allocation failed */
    DIRAC_EHIP = 3,        /* a HIP runtime call failed */
    DIRAC_ESINGULAR = 4,   /* a 6x6 clover block is singular (first site in the message) */
    DIRAC_ENOCONV = 5,     /* solver stopped at max_iter; x holds the best iterate */
    DIRAC_ENONFINITE = 6,  /* NaN or Inf met in a reduction */
    DIRAC_EUNSUPPORTED = 7 /* precision / layout combination not offered */
} dirac_status;

typedef enum { DIRAC_F64 = 0, DIRAC_F32 = 1, DIRAC_F16 = 2, DIRAC_BF16 = 3 } dirac_prec;
typedef enum { DIRAC_LAYOUT_LEX = 0, DIRAC_LAYOUT_EO = 1, DIRAC_LAYOUT_NATIVE = 2, DIRAC_LAYOUT_OPENQXD = 3 } dirac_layout;

typedef struct {
    int dims[4];        /* L0 (time), L1, L2, L3; each even and >= 2 */
    double kappa;       /* hopping parameter: 4 + m0 = 1 / (2 kappa) */
    double csw;         /* SU(3) Sheikholeslami-Wohlert coefficient */
    double csw_qed;     /* U(1) SW coefficient c_sw^U(1) (Sec. 4.3) */
    int qhat;           /* integer charge multiplying theta in the link and the U(1) SW term */
    double bc_phase[4]; /* phi_mu in radians: {pi, 0, 0, 0} = antiperiodic time, periodic space */
    int cstar;          /* C* boundary conditions (Sec. 4.2) in directions 1 .. cstar, 0 = none:
                         * dims[1] is then the doubled extent (the physical lattice and its mirror
                         * copy), direction 1 is periodic with it, and crossing the boundary of a
                         * further C* direction mu >= 2 also moves x1 by dims[1] / 2; with cstar >= 2
                         * dims[1] must be a multiple of 4.  The caller supplies the links of the
                         * whole doubled lattice (for C* fields, the mirror copy holds the complex
                         * conjugate links and the negated U(1) angles). */
} dirac_params;

/* Create a context: copies the gauge field, compresses the links (two rows of
 * SU(3) plus one phase per link), builds the clover field on the device and
 * inverts its odd-site blocks.  Returns DIRAC_ESINGULAR if an odd-site block is
 * singular (the context is still created and must be destroyed).  Blocking. */
dirac_status dirac_create(const dirac_params *params, const void *su3_links, const double *u1_angles,
                          void *stream, dirac_ctx **out);
dirac_status dirac_destroy(dirac_ctx *ctx);

/* Create a context from openQxD's storage of the gauge field (Sec. 4.1.4, Fig. gauge): the 8
 * links attached to every odd point, the odd points in eq. (ipt) order with cache block
 * `block` (which also becomes the context's cache block), odd point V/2 + k at position k:
 *   u_odd [V/2][8][3][3] complex128, slot 2 mu = U_mu(x), slot 2 mu + 1 = U_mu(x - mu);
 *   a_odd [V/2][8] float64 U(1) angles theta in the same slots, or NULL for theta = 0.
 * Every link of the lattice is one of these exactly once.  Device pointers; otherwise as
 * dirac_create.  EINVAL when a block extent does not divide the lattice extent or B3 is odd. */
dirac_status dirac_create_openqxd(const dirac_params *params, const int block[4], const void *u_odd,
                                  const double *a_odd, void *stream, dirac_ctx **out);

/* Set the cache block B of the DIRAC_LAYOUT_OPENQXD user layout (default B = L).  Every B_mu
 * must divide L_mu and B3 must be even (then eq. (ipt) is one-to-one); EINVAL otherwise. */
dirac_status dirac_set_cache_block(dirac_ctx *ctx, const int block[4]);

/* Replace the clover field A = (4 + m0) + C by a user field (Sec. 4.1.3: the
 * application may compute the QCD+QED clover term itself and upload it).
 * `clover` is [V][2][36] float64 in LEX, EO or OPENQXD site order.  Inverses and
 * lower-precision copies are invalidated; call clover_invert next. */
dirac_status dirac_load_clover(dirac_ctx *ctx, const double *clover, dirac_layout layout, void *stream);

/* Copy the clover field (inverse = 0) or its inverse (inverse = 1) out, [V][2][36]
 * float64 in LEX, EO or OPENQXD order.  Sites whose inverse was not computed read 0. */
dirac_status dirac_get_clover(dirac_ctx *ctx, double *out, int inverse, dirac_layout layout, void *stream);

/* The clover field of Sec. 4.1.3 is the site-local coupling openQxD precomputes: two Hermitian
 * 6x6 chirality blocks per site (Sec. 2 places it beside the spinor and gauge fields, Sec. 4.3
 * adds its U(1) term).  This call inverts those blocks, which the even-odd form needs on the
 * odd sites (A_oo^-1 in D-hat).
 * Invert the 6x6 chirality blocks of A in FP64: parity_mask bit 0 = even sites,
 * bit 1 = odd sites.  A block is singular when a pivot of Gauss-Jordan
 * elimination with partial pivoting has modulus below 1e-14 * max|A_block|; the
 * call then returns DIRAC_ESINGULAR and names the first such site (Lambda).
 * Blocking. */
dirac_status clover_invert(dirac_ctx *ctx, int parity_mask, void *stream);

/* Size in bytes of a NATIVE vector: sites = 0 full lattice, 1 one parity. */
size_t dirac_native_bytes(const dirac_ctx *ctx, dirac_prec prec, int sites);

/* Layout conversion of a spinor field.  sites = 0: full vector (LEX, EO or OPENQXD
 * user layout); sites = 1: even half (EO or OPENQXD user layout); sites = 2: odd half
 * (EO or OPENQXD, the second V/2 sites of such a vector).  `user` is complex128
 * for F64 and F16/BF16 targets, complex64 for F32. */
dirac_status dirac_import(dirac_ctx *ctx, void *native, const void *user, int sites, dirac_prec prec,
                          dirac_layout user_layout, void *stream);
dirac_status dirac_export(dirac_ctx *ctx, void *user, const void *native, int sites, dirac_prec prec,
                          dirac_layout user_layout, void *stream);

/* The operator D_w of the linear system D_w psi = eta that the paper offloads (Sec. 2), in the
 * QCD+QED form of Sec. 4.3, on the field layouts of Sec. 4.1.
 * out = D in (dagger = 0) or D^dag in (dagger = 1), full lattice; in and out must not overlap. */
dirac_status dirac_apply(dirac_ctx *ctx, void *out, const void *in, dirac_prec prec, dirac_layout layout,
                         int dagger, void *stream);

/* out_e = D-hat in_e (dagger = 0) or D-hat^dag in_e, even half-vectors (EO, OPENQXD or NATIVE layout). */
dirac_status dirac_apply_eo(dirac_ctx *ctx, void *out_e, const void *in_e, dirac_prec prec, dirac_layout layout,
                            int dagger, void *stream);

/* D-hat on nrhs even half-vectors at once (the paper solves many right-hand sides on one gauge
 * field, Sec. 2): in and out hold nrhs NATIVE half vectors of `prec` back to back (vector r
 * starts r * dirac_native_bytes(ctx, prec, 1) bytes after the base), out must not overlap in.
 * Each kernel covers all right-hand sides in one launch, so every link and clover entry is
 * read from HBM once per site block and served to the others from L2.  Results equal nrhs
 * calls of dirac_apply_eo bit for bit.  Asynchronous on `stream`. */
dirac_status dirac_apply_eo_multi(dirac_ctx *ctx, void *out, const void *in, int nrhs, dirac_prec prec, int dagger,
                                  void *stream);

/* For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  out_e = D-hat in_e (dagger = 0) or D-hat^dag in_e on
 * NATIVE even half-vectors of `prec`, computed by the same kernels as dirac_apply_eo and bitwise
 * equal to it.  The odd-site intermediate A_oo^-1 D_oe in_e (24 reals per padded odd site) is kept
 * in a static device buffer of DIRAC_NOALLOC_SCRATCH_BYTES (64 MiB) that every GPU the library
 * runs on holds until the process ends, so this call allocates nothing and runs no launch-shape
 * timing (it takes the shape tuned earlier for the lattice, else the default shape).  Limits:
 * the intermediate must fit the buffer (at most 349,504 odd sites in F64, e.g. 24^3x48;
 * 699,008 in F32; 1,398,080 in F16 / BF16, e.g. 32^3x64), else DIRAC_EINVAL; the fields of
 * `prec` must exist (F64 always; the
 * others after any earlier apply or solve in that precision), else DIRAC_EINVAL.  Every call on
 * one GPU shares that GPU's buffer: calls that overlap in time on one GPU (other streams, other
 * threads) race.  Asynchronous on `stream`. */
#define DIRAC_NOALLOC_SCRATCH_BYTES (64u << 20)
dirac_status dirac_apply_eo_noalloc(dirac_ctx *ctx, void *out_e, const void *in_e, dirac_prec prec, int dagger,
                                    void *stream);

/* out_p = D_{p,1-p} in_{1-p} = -1/2 H in (the hopping term between parities), NATIVE
 * half-vectors; out_parity selects p.  dagger = 1 gives gamma_5 D_{p,1-p} gamma_5. */
dirac_status dirac_apply_hop(dirac_ctx *ctx, void *out, const void *in, int out_parity, dirac_prec prec,
                             int dagger, void *stream);

/* out_p = A_pp in_p (inverse = 0) or A_pp^-1 in_p (inverse = 1), NATIVE half-vectors. */
dirac_status dirac_apply_clover(dirac_ctx *ctx, void *out, const void *in, int parity, int inverse,
                                dirac_prec prec, void *stream);

/* ---------------------------------------------------------------- solvers */
typedef enum {
    DIRAC_SOLVER_CGLS = 0,      /* CG on D^dag D, full lattice, FP64 */
    DIRAC_SOLVER_GCR = 1,       /* even-odd GCR(restart), FP64 */
    DIRAC_SOLVER_MIXED_GCR = 2, /* FP64 defect correction around an inner_prec even-odd GCR */
    DIRAC_SOLVER_FGCR_PTC = 3,  /* flexible GCR on the full D with a PTC network as preconditioner */
    DIRAC_SOLVER_FGCR_PTC_EO = 4, /* flexible GCR on D-hat, preconditioner r_e -> even half of N(r_e, 0) */
    DIRAC_SOLVER_FGCR_SAP = 5   /* flexible GCR on the full D, Schwarz (SAP) preconditioner (dirac_sap) */
} dirac_solver;

typedef struct dirac_ptc dirac_ptc;  /* parallel-transport convolution network (see below) */

typedef struct {
    int method;          /* dirac_solver */
    int restart;         /* GCR cycle length (Krylov vectors kept), 1..64 */
    int max_iter;        /* operator applications allowed (inner ones for MIXED_GCR) */
    double tol;          /* stop when ||eta - D psi|| / ||eta|| < tol (FP64, recomputed) */
    int inner_prec;      /* MIXED_GCR: dirac_prec of the inner solve (F32, F16, BF16) */
    double inner_tol;    /* MIXED_GCR: relative reduction asked of each inner solve */
    int x0_given;        /* 1: x holds the initial guess */
    int precision;       /* GCR / CGLS: dirac_prec of the whole solve (F64 only) */
    const dirac_ptc *ptc; /* FGCR_PTC(_EO): the preconditioner network (trained weights) */
    int sap_ncy;         /* FGCR_SAP: Schwarz cycles per preconditioner application (0: 4) */
    int sap_nmr;         /* FGCR_SAP: minimal-residual steps per block solve (0: 4) */
} dirac_solver_params;

typedef struct {
    int iters;            /* operator applications (D-hat or D / D^dag) in the working precision */
    int restarts;         /* GCR cycles after the first (or CGLS residual recomputations) */
    int outer;            /* defect-correction steps (MIXED_GCR) */
    int fell_back;        /* 1 if MIXED_GCR finished in plain FP64 GCR */
    double true_rel_res;  /* ||eta - D psi|| / ||eta|| recomputed in FP64 at the end */
    double seconds;       /* wall time of the call */
    int host_syncs;       /* times the call waited on the device for a value (norms, counts) */
} dirac_solve_info;

/* The solve the paper offloads through invertQuda(h_x, h_b, param) (Sec. 4.1), stopped, as in
 * its runs, on the relative residual of the FP64 system (Sec. 5.1) and checked a posteriori as
 * Sec. 2 describes; here x and b are device pointers.
 * Solve D psi = eta.  x (solution) and b (right-hand side) are full-lattice FP64
 * vectors in `layout`.  GCR and MIXED_GCR run on the even-odd Schur system and
 * reconstruct the odd half; CGLS runs on the full D; FGCR_PTC runs flexible GCR
 * on the full D with p_k = N(r_k); FGCR_PTC_EO runs it on the Schur system with
 * p_k = [N(r_k, 0)]_e (the even half of the network applied to the even residual
 * extended by zero, an approximation of (D^-1)_ee = D-hat^-1) and reconstructs the
 * odd half.  Both fall back to even-odd GCR from the current iterate
 * (info.fell_back = 1) when a cycle reduces the residual by less than 2x or meets a
 * non-finite value.  Blocking.  Returns DIRAC_ENOCONV (x = last iterate) when
 * max_iter is reached first. */
dirac_status dirac_solve(dirac_ctx *ctx, void *x, const void *b, dirac_layout layout,
                         const dirac_solver_params *params, dirac_solve_info *info, void *stream);

/* Batched solves: nlat lattices (one context each; uneven sizes and parameters allowed),
 * nrhs right-hand sides per lattice.  x[l] and b[l] hold nrhs full-lattice FP64 vectors in
 * `layout`, one after another.  method GCR or MIXED_GCR.  All right-hand sides of a lattice
 * advance together: every kernel of an iteration covers all of them in one launch (the
 * multi-RHS hop reads each link once per site block and serves it to every right-hand side
 * from L2), converged systems are frozen by a device-side mask, and the launch sequence of
 * each iteration is captured once into a hipGraph and replayed.  The lattices run
 * concurrently, one host thread and one stream each, queued after the work already on
 * `stream`.  info has nlat * nrhs entries (lattice-major).  Blocking. */
dirac_status dirac_solve_batched(dirac_ctx *const *ctx, int nlat, void *const *x, const void *const *b, int nrhs,
                                 dirac_layout layout, const dirac_solver_params *params, dirac_solve_info *info,
                                 void *stream);

/* psi = M r, the Schwarz alternating procedure (SAP) of openQxD's solver (named in the
 * paper's outlook; the method is Luscher's multiplicative Schwarz preconditioner): the lattice
 * is tiled by 4^4 blocks coloured as a checkerboard of blocks; psi = 0, rho = r, and ncy times,
 * for colour 0 then colour 1, on every block of that colour nmr minimal-residual steps
 *   v = D_blk r_b, w = <v, r_b> / <v, v>, delta += w r_b, r_b -= w v   (from delta = 0, r_b = rho)
 * on the block operator D_blk (hops that leave the block dropped), psi += delta, rho = r - D psi.
 * in, out: NATIVE F32 full vectors; FP32 arithmetic on the F32 copies of the fields.  Every
 * lattice extent must be a multiple of 8, and with C* boundaries in two or more directions
 * dims[1] a multiple of 16 (the mirror shift an even number of blocks, so that blocks of one
 * colour never meet); EINVAL otherwise; ncy, nmr in 1..64.  Asynchronous. */
dirac_status dirac_sap(dirac_ctx *ctx, void *out, const void *in, int ncy, int nmr, void *stream);

/* ---------------------------------------------------------------- vector arithmetic
 * NATIVE vectors of the context's lattice: sites = 0 full vectors, 1 one parity.  Sums are
 * formed in FP64 whatever the storage precision.  Calls that return a number (rel_res, norm2,
 * dot not NULL) synchronise `stream`; the others are asynchronous. */

/* r = b - D x for full NATIVE vectors of `prec` (F64 or F32): the residual by which Sec. 2 checks
 * a solution a posteriori.  With rel_res != NULL, *rel_res = |r| / |b| (0 when b = 0);
 * DIRAC_ENONFINITE when r or b holds NaN or Inf.  r must not overlap b or x. */
dirac_status dirac_residual(dirac_ctx *ctx, void *r, const void *b, const void *x, dirac_prec prec, double *rel_res,
                            void *stream);

/* out = alpha a + beta b (element-wise; b is not read when beta = 0 and may then be NULL).  a and b
 * are in in_prec, out in out_prec: in_prec must equal out_prec, or be F64 (the values are then
 * rounded once to out_prec).  With norm2 != NULL, *norm2 = |out|^2 of the stored values;
 * DIRAC_ENONFINITE when out holds NaN or Inf.  out must not overlap a or b. */
dirac_status dirac_lincomb(dirac_ctx *ctx, void *out, dirac_prec out_prec, double alpha, const void *a, double beta,
                           const void *b, dirac_prec in_prec, int sites, double *norm2, void *stream);

/* dot[0] + i dot[1] = <a, b> = sum_i conj(a_i) b_i over NATIVE vectors of `prec`.  Blocking. */
dirac_status dirac_dot(dirac_ctx *ctx, const void *a, const void *b, dirac_prec prec, int sites, double *dot,
                       void *stream);

/* ---------------------------------------------------------------- learned preconditioner
 * A gauge-covariant parallel-transport convolution (PTC) network N (a reading of the
 * learned part; the paper has none):
 *   y_c(x) = sum_{c'} sum_p W[p][c][c'] (T_p x_{c'})(x),  p = 0, +0, -0, +1, -1, +2, -2, +3, -3,
 *   T_{+mu} psi(x) = V_mu(x) b+_mu(x) psi(x + mu),  T_{-mu} psi(x) = V_mu(x - mu)^dag b-_mu(x) psi(x - mu),
 * W[p][c][c'] a complex 4x4 spin matrix; no nonlinearity, no bias.  Weights of layer l
 * are [9][c_{l+1}][c_l][4][4] complex, stored as interleaved (re, im) float, layer after
 * layer.  FP32 master weights, BF16 working weights; each transported input is rounded to
 * BF16 for the matrix cores, products accumulate in FP32; hidden activations are stored in
 * BF16; a last layer (one output channel) is summed as sum_p T_p (sum_c' W x_c') with its
 * inputs rounded to BF16.  The network's input and output and all gradients are NATIVE F32
 * full-lattice vectors (one channel in and out).
 * Training: loss L = mean_i |N(r_i) - e_i|^2 / |e_i|^2, gradients dL/dW* (Wirtinger),
 * Adam (lr given, beta = 0.9, 0.999, eps = 1e-8) on (Re W, Im W). */
dirac_status ptc_create(const int *channels, int nlayers, dirac_ptc **out);  /* channels[0] = channels[nlayers] = 1 */
dirac_status ptc_destroy(dirac_ptc *net);
size_t ptc_num_weights(const dirac_ptc *net);                                /* floats (2 per complex weight) */
dirac_status ptc_set_weights(dirac_ptc *net, const float *host_w, size_t n); /* resets Adam state */
dirac_status ptc_get_weights(const dirac_ptc *net, float *host_w, size_t n);
dirac_status ptc_get_grad(const dirac_ptc *net, float *host_g, size_t n);   /* accumulated dL/dW* */
dirac_status ptc_zero_grad(dirac_ptc *net, void *stream);
/* out = N(in) */
dirac_status ptc_forward(dirac_ctx *ctx, dirac_ptc *net, void *out, const void *in, void *stream);
/* out_e = [N((in_e, 0))]_e: the network as a preconditioner of the even-odd Schur system.
 * in_e and out_e are NATIVE F32 even halves (native_bytes of one parity); bitwise equal to the
 * even half of ptc_forward on (in_e, 0), with the work that only reads the zero odd half or only
 * feeds the odd half of the output left out.  EINVAL on NULL, undersized or aliasing buffers. */
dirac_status ptc_forward_eo(dirac_ctx *ctx, dirac_ptc *net, void *out_e, const void *in_e, void *stream);
/* Given grad_out = dL/dN(in)*, accumulate dL/dW* into the network and, if grad_in is not
 * NULL, write dL/d(in)*.  Recomputes the forward activations of `in`. */
dirac_status ptc_backward(dirac_ctx *ctx, dirac_ptc *net, void *grad_in, const void *in, const void *grad_out,
                          void *stream);
dirac_status ptc_adam_step(dirac_ptc *net, double lr, void *stream);
/* Adam state (first and second moments, n floats each, same order as the weights, and the
 * step count) for checkpoint and resume.  ptc_set_adam_state after ptc_set_weights. */
dirac_status ptc_get_adam_state(const dirac_ptc *net, float *host_m, float *host_v, size_t n, int *step);
dirac_status ptc_set_adam_state(dirac_ptc *net, const float *host_m, const float *host_v, size_t n, int step);
/* One minibatch step: zero the gradient, accumulate over the nbatch pairs (r[i], e[i])
 * (NATIVE F32 full vectors), take one Adam step; *loss = L before the step.  When the loss or
 * an entry of the gradient is not finite the call returns DIRAC_ENONFINITE and leaves the
 * weights and the Adam state unchanged.  Blocking. */
dirac_status ptc_train_step(dirac_ctx *ctx, dirac_ptc *net, const void *const *r, const void *const *e, int nbatch,
                            double lr, double *loss, void *stream);
/* *loss = L over the nbatch pairs without any update (held-out evaluation).  Blocking. */
dirac_status ptc_loss(dirac_ctx *ctx, dirac_ptc *net, const void *const *r, const void *const *e, int nbatch,
                      double *loss, void *stream);

/* Message of the last failed call on this thread ("" if none). */
const char *dirac_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DIRAC_H */
