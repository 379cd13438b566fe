/* Driver for an AddressSanitizer + UndefinedBehaviorSanitizer build of gen/gen.c (host code):
 * draws every kind of field on a small lattice and prints sums the test compares with the
 * library the other tests load. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void gen_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]);
void gen_su3_field(int64_t volume, double eps, uint64_t seed, double *out);
void gen_u1_field(int64_t volume, double theta_max, uint64_t seed, double *theta);
void gen_spinor_field(int64_t volume, uint64_t seed, uint32_t index, double *out);
void gen_gauge_transform(int64_t volume, double eps, uint64_t seed, double *omega, double *lambda);
void gen_uniforms(int64_t n, uint64_t seed, uint32_t stream, double *out);

static double sum(const double *a, int64_t n) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * (double)((i % 7) + 1);
    return s;
}

int main(void) {
    const int64_t V = 2 * 4 * 2 * 6;
    uint32_t c[4] = {1, 2, 3, 4}, k[2] = {5, 6}, o[4];
    gen_philox4x32_10(c, k, o);
    printf("philox %u %u %u %u\n", o[0], o[1], o[2], o[3]);
    double *u = malloc(sizeof(double) * V * 4 * 9 * 2), *t = malloc(sizeof(double) * V * 4);
    double *s = malloc(sizeof(double) * V * 24), *w = malloc(sizeof(double) * V * 18), *l = malloc(sizeof(double) * V);
    double *r = malloc(sizeof(double) * 1000);
    gen_su3_field(V, 0.5, 11, u);
    gen_u1_field(V, 0.3, 11, t);
    gen_spinor_field(V, 12, 3, s);
    gen_gauge_transform(V, 2.0, 13, w, l);
    gen_uniforms(1000, 14, 99, r);
    printf("su3 %.17g\nu1 %.17g\nspinor %.17g\nomega %.17g\nlambda %.17g\nuniform %.17g\n", sum(u, V * 72),
           sum(t, V * 4), sum(s, V * 24), sum(w, V * 18), sum(l, V), sum(r, 1000));
    free(u); free(t); free(s); free(w); free(l); free(r);
    return 0;
}
