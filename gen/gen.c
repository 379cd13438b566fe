/*
 * Seeded synthetic inputs shared by the FP64 oracle and the HIP library.
 *
 * This file holds no arithmetic of the Dirac operator. It draws random
 * numbers and turns them into gauge links, U(1) angles, spinor fields and
 * gauge transformations, all in the lexicographic site order of eq. (lexi)
 * (time first, x3 fastest), so that every field is independent of the
 * memory layout and of the thread count.
 *
 * Random numbers: Philox4x32-10, the counter-based generator of
 * J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11. Key = (seed, stream), counter =
 * (site, direction or component block, word, 0).
 *
 * SU(3) links: U = exp(i eps H), H = sum_a h_a lambda_a / 2 with h_a ~ N(0,1)
 * and lambda_a the Gell-Mann matrices; the exponential is a Taylor series with
 * scaling and squaring, followed by a re-projection onto SU(3) (rows 0 and 1
 * orthonormalised, row 2 = conj(row0 x row1)) so that det U = 1 to rounding.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef double complex cplx;

enum { STREAM_SU3 = 1, STREAM_U1 = 2, STREAM_SPINOR = 16, STREAM_GT_SU3 = 3, STREAM_GT_U1 = 4 };

/* Philox4x32-10 (SC'11): ten rounds of the 4x32 S-box with Weyl key schedule. */
void gen_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static inline double u01(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

/* Four uniforms in (0,1) for (site, a, b) under (seed, stream). */
static void uniforms4(uint64_t seed, uint32_t stream, uint64_t site, uint32_t a, uint32_t b, double u[4])
{
    uint32_t key[2] = {(uint32_t)seed, stream};
    uint32_t ctr[4] = {(uint32_t)site, a, b, (uint32_t)(site >> 32)};
    uint32_t out[4];
    gen_philox4x32_10(ctr, key, out);
    for (int i = 0; i < 4; ++i) u[i] = u01(out[i]);
}

/* Four standard normals by the Box-Muller transform. */
static void normals4(uint64_t seed, uint32_t stream, uint64_t site, uint32_t a, uint32_t b, double z[4])
{
    double u[4];
    uniforms4(seed, stream, site, a, b, u);
    const double twopi = 6.283185307179586476925286766559;
    double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
    z[0] = r0 * cos(twopi * u[1]);
    z[1] = r0 * sin(twopi * u[1]);
    z[2] = r1 * cos(twopi * u[3]);
    z[3] = r1 * sin(twopi * u[3]);
}

static void mat3_mul(const cplx a[9], const cplx b[9], cplx c[9])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += a[3 * i + k] * b[3 * k + j];
            c[3 * i + j] = s;
        }
}

/* exp(X) for a 3x3 complex X: Taylor series after scaling by 2^-s, then s squarings. */
static void mat3_exp(const cplx X[9], cplx E[9])
{
    double nrm = 0;
    for (int i = 0; i < 9; ++i) nrm += creal(X[i] * conj(X[i]));
    nrm = sqrt(nrm);
    int s = 0;
    while (nrm > 0.125) { nrm *= 0.5; ++s; }
    double scale = ldexp(1.0, -s);
    cplx Y[9], term[9], tmp[9];
    for (int i = 0; i < 9; ++i) { Y[i] = X[i] * scale; E[i] = (i % 4 == 0) ? 1.0 : 0.0; term[i] = E[i]; }
    for (int k = 1; k <= 16; ++k) {
        mat3_mul(term, Y, tmp);
        for (int i = 0; i < 9; ++i) { term[i] = tmp[i] / (double)k; E[i] += term[i]; }
    }
    for (int q = 0; q < s; ++q) {
        mat3_mul(E, E, tmp);
        memcpy(E, tmp, sizeof(tmp));
    }
}

/* Project a near-unitary 3x3 matrix onto SU(3): Gram-Schmidt rows 0,1; row 2 = conj(r0 x r1). */
static void su3_project(cplx U[9])
{
    cplx *a = U, *b = U + 3, *c = U + 6;
    double na = 0;
    for (int i = 0; i < 3; ++i) na += creal(a[i] * conj(a[i]));
    na = 1.0 / sqrt(na);
    for (int i = 0; i < 3; ++i) a[i] *= na;
    cplx ab = 0;
    for (int i = 0; i < 3; ++i) ab += conj(a[i]) * b[i];
    for (int i = 0; i < 3; ++i) b[i] -= ab * a[i];
    double nb = 0;
    for (int i = 0; i < 3; ++i) nb += creal(b[i] * conj(b[i]));
    nb = 1.0 / sqrt(nb);
    for (int i = 0; i < 3; ++i) b[i] *= nb;
    c[0] = conj(a[1] * b[2] - a[2] * b[1]);
    c[1] = conj(a[2] * b[0] - a[0] * b[2]);
    c[2] = conj(a[0] * b[1] - a[1] * b[0]);
}

/* i*eps*H with H = sum_a h_a lambda_a / 2 (Gell-Mann basis), a traceless anti-Hermitian matrix. */
static void su3_algebra(const double h[8], double eps, cplx X[9])
{
    const double r3 = 1.0 / sqrt(3.0);
    cplx H[9];
    H[0] = 0.5 * (h[2] + r3 * h[7]);
    H[4] = 0.5 * (-h[2] + r3 * h[7]);
    H[8] = 0.5 * (-2.0 * r3 * h[7]);
    H[1] = 0.5 * (h[0] - I * h[1]);
    H[3] = 0.5 * (h[0] + I * h[1]);
    H[2] = 0.5 * (h[3] - I * h[4]);
    H[6] = 0.5 * (h[3] + I * h[4]);
    H[5] = 0.5 * (h[5] - I * h[6]);
    H[7] = 0.5 * (h[5] + I * h[6]);
    for (int i = 0; i < 9; ++i) X[i] = I * eps * H[i];
}

static void random_su3(uint64_t seed, uint32_t stream, uint64_t site, uint32_t mu, double eps, cplx U[9])
{
    double h[8];
    normals4(seed, stream, site, mu, 0, h);
    normals4(seed, stream, site, mu, 1, h + 4);
    cplx X[9];
    su3_algebra(h, eps, X);
    mat3_exp(X, U);
    su3_project(U);
}

/* SU(3) gauge field U[site][mu][a][b] (complex128, row-major), 4 forward links per site. */
void gen_su3_field(int64_t volume, double eps, uint64_t seed, double *out)
{
    cplx *U = (cplx *)out;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < volume; ++x)
        for (int mu = 0; mu < 4; ++mu) random_su3(seed, STREAM_SU3, (uint64_t)x, (uint32_t)mu, eps, U + (x * 4 + mu) * 9);
}

/* U(1) angles theta[site][mu] uniform in (-theta_max, theta_max). */
void gen_u1_field(int64_t volume, double theta_max, uint64_t seed, double *theta)
{
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < volume; ++x)
        for (int mu = 0; mu < 4; ++mu) {
            double u[4];
            uniforms4(seed, STREAM_U1, (uint64_t)x, (uint32_t)mu, 0, u);
            theta[x * 4 + mu] = theta_max * (2.0 * u[0] - 1.0);
        }
}

/* Gaussian spinor psi[site][spin][colour] (complex128): re, im ~ N(0,1). `index` selects one of many fields. */
void gen_spinor_field(int64_t volume, uint64_t seed, uint32_t index, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < volume; ++x)
        for (uint32_t blk = 0; blk < 6; ++blk) {
            double z[4];
            normals4(seed, STREAM_SPINOR + index, (uint64_t)x, blk, 0, z);
            for (int k = 0; k < 4; ++k) out[x * 24 + blk * 4 + k] = z[k];
        }
}

/* Random gauge transformation: Omega[site] in SU(3) (complex128 3x3) and lambda[site] in (-pi, pi). */
void gen_gauge_transform(int64_t volume, double eps, uint64_t seed, double *omega, double *lambda)
{
    cplx *W = (cplx *)omega;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < volume; ++x) {
        random_su3(seed, STREAM_GT_SU3, (uint64_t)x, 0, eps, W + x * 9);
        double u[4];
        uniforms4(seed, STREAM_GT_U1, (uint64_t)x, 0, 0, u);
        lambda[x] = 3.141592653589793238462643383 * (2.0 * u[0] - 1.0);
    }
}

/* Uniform draws in (0,1), n of them, for tests of the generator itself. */
void gen_uniforms(int64_t n, uint64_t seed, uint32_t stream, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (n + 3) / 4; ++i) {
        double u[4];
        uniforms4(seed, stream, (uint64_t)i, 0, 0, u);
        for (int k = 0; k < 4 && 4 * i + k < n; ++k) out[4 * i + k] = u[k];
    }
}
