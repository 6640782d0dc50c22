/*
 * Driver for the oracle built with AddressSanitizer and UndefinedBehaviorSanitizer:
 * every entry point of oracle/asf_oracle.c on small inputs, valid and invalid.
 * Exit status 0 when every call returned what it should; the sanitizers abort
 * the process on the first memory or undefined-behaviour error.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int asf_oracle_threads(int32_t requested);
int asf_oracle_direct(int64_t n, const double *x, const double *y, const double *d, const double *u,
                      double lambda, double z0, double p2x, double p2y, double x0, double y0, int32_t mx,
                      int32_t my, int32_t incident, int64_t n_eval, const int32_t *ix, const int32_t *iy,
                      double *out, int32_t threads);
int asf_oracle_adjoint(int64_t n, const double *x, const double *y, const double *d, double lambda,
                       double z0, double p2x, double p2y, double x0, double y0, int32_t mx, int32_t my,
                       int32_t incident, const double *g2, int64_t n_eval, const int64_t *jidx, double *out,
                       int32_t threads);
int asf_oracle_surface(int32_t model, int64_t n, const double *x, const double *y, const double *d,
                       const double *u, double lambda, double z0, double p2x, double p2y, double x0,
                       double y0, int32_t mx, int32_t my, int32_t incident, int64_t n_eval,
                       const int32_t *ix, const int32_t *iy, double *out, int32_t threads);
int asf_oracle_line(int32_t model, int64_t n, const double *x, const double *d, const double *u,
                    double lambda, double z0, double p2, double x0, int32_t m, int32_t incident,
                    int64_t n_eval, const int32_t *ix, double *out, int32_t threads);

static uint64_t state = 88172645463325252ull;
static double uniform(void) {   /* xorshift64, in [0, 1) */
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) * 0x1p-53;
}

static int all_finite(const double *v, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

#define CHECK(cond)                                                       \
    do {                                                                  \
        if (!(cond)) {                                                    \
            fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            return 1;                                                     \
        }                                                                 \
    } while (0)

int main(void) {
    enum { N = 37, MX = 12, MY = 9, NE = MX * MY };
    double *x = malloc(N * sizeof(double)), *y = malloc(N * sizeof(double)), *d = malloc(N * sizeof(double));
    double *u = malloc(2 * N * sizeof(double)), *g2 = malloc(2 * NE * sizeof(double));
    double *out = malloc(2 * NE * sizeof(double)), *g1 = malloc(2 * N * sizeof(double));
    int32_t *ix = malloc(NE * sizeof(int32_t)), *iy = malloc(NE * sizeof(int32_t));
    int64_t *jidx = malloc(N * sizeof(int64_t));
    for (int j = 0; j < N; ++j) {
        x[j] = (uniform() - 0.5) * 4e-4;
        y[j] = (uniform() - 0.5) * 3e-4;
        d[j] = uniform() * 40e-6;
        u[2 * j] = uniform() - 0.5;
        u[2 * j + 1] = uniform() - 0.5;
        jidx[j] = N - 1 - j;
    }
    for (int e = 0; e < NE; ++e) {
        ix[e] = e % MX;
        iy[e] = e / MX;
        g2[2 * e] = uniform() - 0.5;
        g2[2 * e + 1] = uniform() - 0.5;
    }
    CHECK(asf_oracle_threads(0) >= 1 && asf_oracle_threads(3) == 3);
    for (int inc = 0; inc < 2; ++inc) {
        CHECK(asf_oracle_direct(N, x, y, d, u, 532e-9, 0.1, 8e-6, 9e-6, 1e-5, -2e-5, MX, MY, inc, NE, ix, iy,
                                out, 2) == 0);
        CHECK(all_finite(out, 2 * NE));
        CHECK(asf_oracle_adjoint(N, x, y, d, 532e-9, 0.1, 8e-6, 9e-6, 1e-5, -2e-5, MX, MY, inc, g2, N, jidx,
                                 g1, 2) == 0);
        CHECK(all_finite(g1, 2 * N));
        for (int model = 2; model <= 5; model += 3) {
            CHECK(asf_oracle_surface(model, N, x, y, d, u, 532e-9, 0.1, 8e-6, 9e-6, 0.0, 0.0, MX, MY, inc, NE,
                                     ix, iy, out, 2) == 0);
            CHECK(all_finite(out, 2 * NE));
        }
        for (int model = 2; model <= 7; ++model) {
            if (model != 2 && model != 5 && model != 7) continue;
            CHECK(asf_oracle_line(model, N, x, d, u, 633e-9, 1.0, 10e-6, 3e-6, MX, inc, MX, ix, out, 2) == 0);
            CHECK(all_finite(out, 2 * MX));
        }
    }
    /* empty inputs and invalid arguments */
    CHECK(asf_oracle_direct(0, x, y, d, u, 532e-9, 0.1, 8e-6, 8e-6, 0.0, 0.0, MX, MY, 0, NE, ix, iy, out, 1) == 0);
    CHECK(out[0] == 0.0 && out[1] == 0.0);
    CHECK(asf_oracle_direct(-1, x, y, d, u, 532e-9, 0.1, 8e-6, 8e-6, 0.0, 0.0, MX, MY, 0, NE, ix, iy, out, 1) == -1);
    CHECK(asf_oracle_direct(N, x, y, d, u, -1.0, 0.1, 8e-6, 8e-6, 0.0, 0.0, MX, MY, 0, NE, ix, iy, out, 1) == -1);
    d[5] = 0.2;   /* r0 = z0 - d1 < 0 */
    CHECK(asf_oracle_direct(N, x, y, d, u, 532e-9, 0.1, 8e-6, 8e-6, 0.0, 0.0, MX, MY, 0, NE, ix, iy, out, 1) == -1);
    CHECK(asf_oracle_adjoint(N, x, y, d, 532e-9, 0.1, 8e-6, 8e-6, 0.0, 0.0, MX, MY, 0, g2, N, jidx, g1, 1) == -1);
    jidx[0] = N;  /* out of range */
    d[5] = 0.0;
    CHECK(asf_oracle_adjoint(N, x, y, d, 532e-9, 0.1, 8e-6, 8e-6, 0.0, 0.0, MX, MY, 0, g2, N, jidx, g1, 1) == -1);
    free(x); free(y); free(d); free(u); free(g2); free(out); free(g1); free(ix); free(iy); free(jidx);
    puts("oracle sanitizer driver: ok");
    return 0;
}
